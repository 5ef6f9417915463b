// Host-side operation count of the interior-face fluxes (RTLBFS and TLBFS) of
// the GPU library:
// the face function is instantiated with a number type that counts every
// addition, subtraction, multiplication and division.  Also checks on the
// host that the column form of the RTLBFS flux (the kernels' face_flux)
// agrees with the nodal form (face_flux_nodes) on random faces.  Test
// infrastructure.
#include <cmath>
#include <cstdio>
#include <random>

#include "rtlbfs_device.h"
#include "curv2d.h"

struct CountedReal {
    double v;
    static long adds, muls, divs;
    CountedReal(double x = 0) : v(x) {}
    friend CountedReal operator+(CountedReal a, CountedReal b) { ++adds; return CountedReal(a.v + b.v); }
    friend CountedReal operator-(CountedReal a, CountedReal b) { ++adds; return CountedReal(a.v - b.v); }
    friend CountedReal operator*(CountedReal a, CountedReal b) { ++muls; return CountedReal(a.v * b.v); }
    friend CountedReal operator/(CountedReal a, CountedReal b) { ++divs; return CountedReal(a.v / b.v); }
    CountedReal operator-() const { return CountedReal(-v); }
    CountedReal &operator+=(CountedReal b) { ++adds; v += b.v; return *this; }
    CountedReal &operator-=(CountedReal b) { ++adds; v -= b.v; return *this; }
    explicit operator double() const { return v; }
};
long CountedReal::adds = 0, CountedReal::muls = 0, CountedReal::divs = 0;

template <int D, bool DEV, bool TL, bool NODES = false>
void count(const char *name) {
    using R = CountedReal;
    rtlbfs::Side<R, D> L, Rt;
    for (int p = 0; p < D + 2; ++p) {
        L.v[p] = 1.0 + 0.1 * p;
        Rt.v[p] = 1.0 + 0.2 * p;
        for (int k = 0; k < D; ++k) {
            L.g[k][p] = 0.01;
            Rt.g[k][p] = 0.02;
        }
    }
    rtlbfs::Phys<R> ph;
    ph.nu = 0.1; ph.chi = 0.1; ph.dtl = 1.0; ph.tau_f = 0.8; ph.tau_g = 0.9; ph.bg = 1e-3;
    ph.h = 1.0; ph.inv2h = 0.5; ph.invh2 = 1.0; ph.inv4h2 = 0.25;
    R fdir[D];
    for (int k = 0; k < D; ++k) fdir[k] = k == 1 ? 1.0 : 0.0;
    R out[D + 2];
    R::adds = R::muls = R::divs = 0;
    if (TL) rtlbfs::face_flux_tlbfs<R, D, DEV>(L, Rt, R(0.5), R(0.5), fdir, ph, out);
    else if (NODES) rtlbfs::face_flux_nodes<R, D, DEV>(L, Rt, R(0.5), R(0.5), fdir, ph, out);
    else rtlbfs::face_flux<R, D, DEV>(L, Rt, R(0.5), R(0.5), fdir, ph, out);
    std::printf("%s %ld %ld %ld\n", name, R::adds, R::muls, R::divs);
}

// One interior face of a body-fitted mesh: both sides rotated into the face
// frame and shifted along t, the flux, and the rotation back.
template <bool DEV, bool TL>
void count_curv(const char *name) {
    using R = CountedReal;
    R P[4], Q[4], GP[4][2], GQ[4][2];
    for (int p = 0; p < 4; ++p) {
        P[p] = 0.1 * p;
        Q[p] = 0.2 * p;
        for (int a = 0; a < 2; ++a) {
            GP[p][a] = 0.01;
            GQ[p][a] = 0.02;
        }
    }
    rtlbfs::Phys<R> ph;
    ph.nu = 0.1; ph.chi = 0.1; ph.dtl = 1.0; ph.tau_f = 0.8; ph.tau_g = 0.9; ph.bg = 1e-3;
    ph.h = 1.0; ph.inv2h = 0.5; ph.invh2 = 1.0; ph.inv4h2 = 0.25; ph.Tref_s = 0.0;
    rtlbfs::Side<R, 2> A, B;
    R F[4];
    R::adds = R::muls = R::divs = 0;
    rtlbfs::side_in_frame(P, GP, R(0.6), R(0.8), R(0.1), A);
    rtlbfs::side_in_frame(Q, GQ, R(0.6), R(0.8), R(-0.1), B);
    rtlbfs::frame_flux<R, DEV, TL>(A, B, R(0.5), R(0.5), R(0.6), R(0.8), R(0.0), R(1.0), true, R(1.2), ph, F);
    std::printf("%s %ld %ld %ld\n", name, R::adds, R::muls, R::divs);
}

// Largest difference between the two forms over n random faces, relative to
// the largest flux component of each face.  Gradients up to `grad` per unit
// length, cell widths h in [0.3, 1.3], off-centre face distances.
template <int D, bool DEV>
double forms_agree(int n, unsigned seed, double grad) {
    std::mt19937_64 g(seed);
    std::uniform_real_distribution<double> U(-1.0, 1.0);
    double worst = 0.0;
    for (int it = 0; it < n; ++it) {
        rtlbfs::Side<double, D> L, Rt;
        for (int p = 0; p < D + 2; ++p) {
            const double base = p == 0 ? (DEV ? 0.01 : 1.0) : (p == D + 1 ? (DEV ? 0.05 : 1.0) : 0.05);
            L.v[p] = base + 0.02 * U(g);
            Rt.v[p] = base + 0.02 * U(g);
            for (int k = 0; k < D; ++k) {
                L.g[k][p] = grad * U(g);
                Rt.g[k][p] = grad * U(g);
            }
        }
        const double h = 0.3 + 0.5 * (U(g) + 1.0);
        rtlbfs::Phys<double> ph;
        ph.nu = 0.01; ph.chi = 0.014; ph.dtl = 0.5 * h; ph.tau_f = 0.7; ph.tau_g = 0.75; ph.bg = 1e-3 * (1.0 + U(g));
        ph.h = h; ph.inv2h = 1.0 / (2.0 * h); ph.invh2 = 1.0 / (h * h); ph.inv4h2 = 1.0 / (4.0 * h * h); ph.Tref_s = 0.0;
        double fdir[D];
        for (int k = 0; k < D; ++k) fdir[k] = U(g);
        const double dL = 0.5 * h * (1.0 + 0.3 * U(g)), dR = 0.5 * h * (1.0 + 0.3 * U(g));
        double a[D + 2], b[D + 2];
        rtlbfs::face_flux_nodes<double, D, DEV>(L, Rt, dL, dR, fdir, ph, a);
        rtlbfs::face_flux<double, D, DEV>(L, Rt, dL, dR, fdir, ph, b);
        double sc = 0.0;
        for (int p = 0; p < D + 2; ++p) sc = std::fmax(sc, std::fabs(a[p]));
        for (int p = 0; p < D + 2; ++p) worst = std::fmax(worst, std::fabs(a[p] - b[p]) / sc);
    }
    return worst;
}

int main() {
    count<2, false, false, true>("2d_plain");
    count<2, true, false, true>("2d_dev");
    count<3, false, false, true>("3d_plain");
    count<3, true, false, true>("3d_dev");
    count<2, false, false>("col_2d_plain");
    count<2, true, false>("col_2d_dev");
    count<3, false, false>("col_3d_plain");
    count<3, true, false>("col_3d_dev");
    count<2, false, true>("tlbfs_2d_plain");
    count<2, true, true>("tlbfs_2d_dev");
    count<3, false, true>("tlbfs_3d_plain");
    count<3, true, true>("tlbfs_3d_dev");
    count_curv<false, false>("curv_2d_plain");
    count_curv<true, false>("curv_2d_dev");
    count_curv<false, true>("curv_tlbfs_2d_plain");
    count_curv<true, true>("curv_tlbfs_2d_dev");
    std::printf("agree_2d_plain %.3e\n", forms_agree<2, false>(20000, 1, 0.01));
    std::printf("agree_2d_dev %.3e\n", forms_agree<2, true>(20000, 2, 0.01));
    std::printf("agree_3d_plain %.3e\n", forms_agree<3, false>(20000, 3, 0.01));
    std::printf("agree_3d_dev %.3e\n", forms_agree<3, true>(20000, 4, 0.01));
    std::printf("agree_steep_2d_dev %.3e\n", forms_agree<2, true>(20000, 5, 0.3));
    std::printf("agree_steep_3d_dev %.3e\n", forms_agree<3, true>(20000, 6, 0.3));
    return 0;
}
