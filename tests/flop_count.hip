// Host-side operation count of the interior-face fluxes (RTLBFS and TLBFS) of
// the GPU library:
// the face function is instantiated with a number type that counts every
// addition, subtraction, multiplication and division.  Test infrastructure.
#include <cstdio>

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

template <int D, bool DEV, bool TL>
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

int main() {
    count<2, false, false>("2d_plain");
    count<2, true, false>("2d_dev");
    count<3, false, false>("3d_plain");
    count<3, true, false>("3d_dev");
    count<2, false, true>("tlbfs_2d_plain");
    count<2, true, true>("tlbfs_2d_dev");
    count<3, false, true>("tlbfs_3d_plain");
    count<3, true, true>("tlbfs_3d_dev");
    count_curv<false, false>("curv_2d_plain");
    count_curv<true, false>("curv_2d_dev");
    count_curv<false, true>("curv_tlbfs_2d_plain");
    count_curv<true, true>("curv_tlbfs_2d_dev");
    return 0;
}
