// reduce.h -- FP64 diagnostics kernels: Eq. 65 finalisation, wall / volume
// Nusselt numbers (Eqs. 69, 75-76 form), volume integrals and the total-mass
// drift correction of the FP32 deviation storage.  Generic over 2D and 3D;
// each block writes partials, a single-block pass reduces them in a fixed
// order (deterministic for a given launch shape).
#pragma once

#include "rtlbfs_device.h"

namespace rtlbfs {

// Thread t of the block adds rows b0 + t, b0 + t + blockDim.x, ... (below
// b1) of K doubles into acc, in that order.  The loads of eight rows are
// issued before their additions, so a long range is not bound by one load
// latency per row; the order of the additions is the same as one row at a
// time.
template <int K>
__device__ inline void strided_row_sums(const double *__restrict__ parts, int64_t b0, int64_t b1,
                                        double (&acc)[K]) {
    constexpr int U = 8;
    const int64_t stride = blockDim.x;
    int64_t b = b0 + threadIdx.x;
    for (; b + (U - 1) * stride < b1; b += U * stride) {
        double v[U][K];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < K; ++k) v[u][k] = parts[(b + u * stride) * K + k];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < K; ++k) acc[k] += v[u][k];
    }
    for (; b < b1; b += stride)
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] += parts[b * K + k];
}

// Sum `nparts` rows of K doubles into out[0..K): one block, fixed order.
template <int K>
__global__ void __launch_bounds__(256) k_finalize_sum(const double *__restrict__ parts, int nparts,
                                                      double *__restrict__ out) {
    __shared__ double sred[K * 4];
    double acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0;
    strided_row_sums<K>(parts, 0, nparts, acc);
    block_sums<K>(acc, sred);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) out[k] = acc[k];
}

__device__ inline void cell_ijk(const Domain &d, int64_t c, int ijk[3]) {
    ijk[0] = (int)(c % d.n[0]);
    ijk[1] = (int)((c / d.n[0]) % d.n[1]);
    ijk[2] = d.dim == 3 ? (int)(c / ((int64_t)d.n[0] * d.n[1])) : 0;
}

template <typename R, bool DEV>
__device__ inline void load_prims(const Domain &d, const R *U, int64_t c, double &rho, double *u, double &Tdev) {
    const int64_t N = d.fstride;
    const double r = (double)U[c];
    rho = DEV ? 1.0 + r : r;
    for (int a = 0; a < d.dim; ++a) u[a] = (double)U[(1 + a) * N + c] / rho;
    const double e = (double)U[(d.dim + 1) * N + c];
    Tdev = DEV ? e / rho : e / rho - kT0;
}

// Nusselt partials per block: {hot_sum, hot_area, cold_sum, cold_area,
// vol_sum, vol} then maxima {hot_max, cold_max}.
constexpr int kNuParts = 8;

template <typename R, bool DEV>
__global__ void __launch_bounds__(256) k_nusselt(Domain d, const R *__restrict__ U, int haxis, int hot_hi,
                                                 double La, double dTw, double *__restrict__ parts) {
    __shared__ double sred[kNuParts * 4];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    double mx_hot = -1e300, mx_cold = -1e300;
    const int64_t stride_a = haxis == 0 ? 1 : haxis == 1 ? (int64_t)d.n[0] : (int64_t)d.n[0] * d.n[1];
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < d.cells;
         c += (int64_t)gridDim.x * blockDim.x) {
        int ijk[3];
        cell_ijk(d, c, ijk);
        double rho, u[3], Tp;
        load_prims<R, DEV>(d, U, c, rho, u, Tp);
        double area = 1.0, vol = 1.0;
        for (int a = 0; a < d.dim; ++a) {
            vol *= d.w[a][ijk[a]];
            if (a != haxis) area *= d.w[a][ijk[a]];
        }
        const int ia = ijk[haxis], na = d.n[haxis];
        const double wP = d.w[haxis][ia];
        // Eq. 55 gradient of T' along the heat axis with Eq. 56 face values.
        double flo, fhi;
        if (ia == 0) {
            flo = d.Tw[2 * haxis] - (DEV ? 0.0 : kT0);
        } else {
            double r2, u2[3], T2;
            load_prims<R, DEV>(d, U, c - stride_a, r2, u2, T2);
            const double wN = d.w[haxis][ia - 1];
            flo = (Tp * wN + T2 * wP) / (wP + wN);
        }
        if (ia == na - 1) {
            fhi = d.Tw[2 * haxis + 1] - (DEV ? 0.0 : kT0);
        } else {
            double r2, u2[3], T2;
            load_prims<R, DEV>(d, U, c + stride_a, r2, u2, T2);
            const double wN = d.w[haxis][ia + 1];
            fhi = (Tp * wN + T2 * wP) / (wP + wN);
        }
        const double dTda = (fhi - flo) / wP;
        // Eq. 69 integrand: u_a T with the absolute temperature (no density
        // factor) minus chi times the temperature gradient
        const double qa = u[haxis] * (Tp + kT0) - d.chi * dTda;
        acc[4] += (hot_hi ? -qa : qa) * vol;
        acc[5] += vol;
        for (int hi = 0; hi < 2; ++hi) {
            if (ia != (hi ? na - 1 : 0)) continue;
            const double Tw = d.Tw[2 * haxis + hi] - (DEV ? 0.0 : kT0);
            const bool is_hot = hi == hot_hi;
            const double nu = La / dTw * (is_hot ? (Tw - Tp) : (Tp - Tw)) / (0.5 * wP);
            if (is_hot) {
                acc[0] += nu * area;
                acc[1] += area;
                mx_hot = fmax(mx_hot, nu);
            } else {
                acc[2] += nu * area;
                acc[3] += area;
                mx_cold = fmax(mx_cold, nu);
            }
        }
    }
    double s[6] = {acc[0], acc[1], acc[2], acc[3], acc[4], acc[5]};
    block_sums<6>(s, sred);
    mx_hot = wave_max(mx_hot);
    mx_cold = wave_max(mx_cold);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (lane == 0) {
        sred[wave] = mx_hot;
        sred[4 + wave] = mx_cold;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double mh = -1e300, mc = -1e300;
        for (int w = 0; w < nw; ++w) {
            mh = fmax(mh, sred[w]);
            mc = fmax(mc, sred[4 + w]);
        }
        double *o = parts + (int64_t)blockIdx.x * kNuParts;
        for (int k = 0; k < 6; ++k) o[k] = s[k];
        o[6] = mh;
        o[7] = mc;
    }
}

template <int Unused = 0>
__global__ void __launch_bounds__(256) k_nusselt_finalize(const double *__restrict__ parts, int nparts,
                                                          double *__restrict__ out) {
    __shared__ double sred[6 * 4 + 8];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    double mh = -1e300, mc = -1e300;
    for (int b = threadIdx.x; b < nparts; b += blockDim.x) {
        for (int k = 0; k < 6; ++k) acc[k] += parts[(int64_t)b * kNuParts + k];
        mh = fmax(mh, parts[(int64_t)b * kNuParts + 6]);
        mc = fmax(mc, parts[(int64_t)b * kNuParts + 7]);
    }
    block_sums<6>(acc, sred);
    mh = wave_max(mh);
    mc = wave_max(mc);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (lane == 0) {
        sred[24 + wave] = mh;
        sred[28 + wave] = mc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 0; w < nw; ++w) {
            mh = fmax(mh, sred[24 + w]);
            mc = fmax(mc, sred[28 + w]);
        }
        for (int k = 0; k < 6; ++k) out[k] = acc[k];
        out[6] = mh;
        out[7] = mc;
    }
}

// Integrals per block: {sum (rho - 1) dV, sum rho (T - T0) dV, sum dV}.
constexpr int kIntParts = 3;

template <typename R, bool DEV>
__global__ void __launch_bounds__(256) k_integrals(Domain d, const R *__restrict__ U, double *__restrict__ parts) {
    __shared__ double sred[kIntParts * 4];
    double acc[kIntParts] = {0, 0, 0};
    const int64_t N = d.fstride;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < d.cells;
         c += (int64_t)gridDim.x * blockDim.x) {
        double vol = 1.0;
        if (d.vol) {
            vol = d.vol[c];
        } else {
            int ijk[3];
            cell_ijk(d, c, ijk);
            for (int a = 0; a < d.dim; ++a) vol *= d.w[a][ijk[a]];
        }
        const double r = (double)U[c];
        const double e = (double)U[(d.dim + 1) * N + c];
        const double rdev = DEV ? r : r - 1.0;
        const double theta = DEV ? e : e - kT0 * r;
        acc[0] += rdev * vol;
        acc[1] += theta * vol;
        acc[2] += vol;
    }
    block_sums<kIntParts>(acc, sred);
    if (threadIdx.x == 0)
        for (int k = 0; k < kIntParts; ++k) parts[(int64_t)blockIdx.x * kIntParts + k] = acc[k];
}

// Per-segment sums: out[m*K + k] = sum over rows [begin[m], begin[m+1]) of
// parts[row*K + k]; one block per segment, fixed order.
template <int K>
__global__ void __launch_bounds__(256) k_segment_sum(const double *__restrict__ parts, const int *__restrict__ begin,
                                                     double *__restrict__ out) {
    __shared__ double sred[K * 4];
    const int m = blockIdx.x;
    double acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0;
    strided_row_sums<K>(parts, begin[m], begin[m + 1], acc);
    block_sums<K>(acc, sred);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) out[(int64_t)m * K + k] = acc[k];
}

// Subtract the uniform density shift (sum r dV - M0)/V from r (FP32 path).
template <typename R>
__global__ void __launch_bounds__(256) k_mass_fix(R *__restrict__ r, int64_t N, const double *__restrict__ sums,
                                                  const double *__restrict__ m0) {
    const double shift = (sums[0] - m0[0]) / sums[2];
    const R s = (R)shift;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (int64_t)gridDim.x * blockDim.x)
        r[c] -= s;
}

}  // namespace rtlbfs
