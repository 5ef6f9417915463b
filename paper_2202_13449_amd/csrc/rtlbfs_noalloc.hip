// rtlbfs_noalloc.hip -- the Eq. 65 convergence ratios between two states that
// live in caller memory, with no handle and no allocation.
//
// The per-block partial sums go to `scratch`, a fixed file-scope device array
// (32 KiB per GPU).  Host code never passes the array's name to a kernel: its
// device address is looked up once per device with hipGetSymbolAddress and
// kept in `g_scratch`.  Every call on one GPU shares that GPU's array, so
// calls that overlap on one GPU (different streams, different host threads)
// race; calls on one stream are ordered and safe.  Each call overwrites every
// partial row it reads, so nothing has to be cleared between calls.
//
// The per-cell terms are formed exactly as the step kernels form them on a
// residual step: the old state's primitives in the storage precision (the
// reciprocal of the density times the conserved field), the new state's by
// FP64 division, the absolute temperature T0 + T' in deviation storage.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "../../include/rtlbfs.h"
#include "rtlbfs_device.h"

using namespace rtlbfs;

namespace {

constexpr int kResThreads = 256;
constexpr int kResRows = 1024;  // partial rows, one per block
constexpr int kResSums = 4;     // sum ||u|' - |u||, sum |u|', sum |T' - T|, sum T'  (primes: new state)
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kResRows * kResSums];

std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

template <typename R, bool DEV, int D>
__global__ void __launch_bounds__(kResThreads) k_residual_states(const R *__restrict__ Uo, const R *__restrict__ Un,
                                                                 int64_t cells, int64_t fs,
                                                                 double *__restrict__ part) {
    __shared__ double sred[kResSums * (kResThreads / 64)];
    double acc[kResSums] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t c = (int64_t)blockIdx.x * kResThreads + threadIdx.x; c < cells;
         c += (int64_t)gridDim.x * kResThreads) {
        // old state: primitives in the storage precision
        const R ro = Uo[c];
        const R inv_rho = recip<R>(DEV ? (R)1 + ro : ro);
        const double To = (double)(Uo[(D + 1) * fs + c] * inv_rho) + (DEV ? kT0 : 0.0);
        // new state: FP64 division
        const double rn = (double)Un[c];
        const double rhon = DEV ? 1.0 + rn : rn;
        const double Tn = (double)Un[(D + 1) * fs + c] / rhon + (DEV ? kT0 : 0.0);
        double an, ao;
        if constexpr (D == 2) {
            const double un = (double)Un[fs + c] / rhon, vn = (double)Un[2 * fs + c] / rhon;
            const double uo = (double)(Uo[fs + c] * inv_rho), vo = (double)(Uo[2 * fs + c] * inv_rho);
            an = sqrt(un * un + vn * vn);
            ao = sqrt(uo * uo + vo * vo);
        } else {
            an = 0.0;
            ao = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double un = (double)Un[(1 + a) * fs + c] / rhon, uo = (double)(Uo[(1 + a) * fs + c] * inv_rho);
                an += un * un;
                ao += uo * uo;
            }
            an = sqrt(an);
            ao = sqrt(ao);
        }
        acc[0] += fabs(an - ao);
        acc[1] += an;
        acc[2] += fabs(Tn - To);
        acc[3] += Tn;
    }
    block_sums<kResSums>(acc, sred);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < kResSums; ++k) part[(int64_t)blockIdx.x * kResSums + k] = acc[k];
}

// Sum the rows in a fixed order and form the two ratios of Eq. 65.
__global__ void __launch_bounds__(kResThreads) k_residual_states_ratio(const double *__restrict__ part, int rows,
                                                                       double *__restrict__ out) {
    __shared__ double sred[kResSums * (kResThreads / 64)];
    double acc[kResSums] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < rows; b += kResThreads)
#pragma unroll
        for (int k = 0; k < kResSums; ++k) acc[k] += part[(int64_t)b * kResSums + k];
    block_sums<kResSums>(acc, sred);
    if (threadIdx.x == 0) {
        out[0] = acc[1] > 0.0 ? acc[0] / acc[1] : 0.0;
        out[1] = acc[3] != 0.0 ? acc[2] / acc[3] : 0.0;
    }
}

template <typename R, bool DEV>
void launch(int dim, int rows, const void *old_state, const void *new_state, int64_t cells, int64_t fs,
            double *part, hipStream_t s) {
    if (dim == 2)
        k_residual_states<R, DEV, 2><<<rows, kResThreads, 0, s>>>((const R *)old_state, (const R *)new_state, cells,
                                                                  fs, part);
    else
        k_residual_states<R, DEV, 3><<<rows, kResThreads, 0, s>>>((const R *)old_state, (const R *)new_state, cells,
                                                                  fs, part);
}

}  // namespace

extern "C" int rtlbfs_residual_states(int dim, int precision, int64_t cells, int64_t fstride, const void *old_state,
                                      const void *new_state, double *dev_out, void *hip_stream) {
    if ((dim != 2 && dim != 3) || !old_state || !new_state || !dev_out) return RTLBFS_EINVAL;
    if (precision != RTLBFS_FP64_PLAIN && precision != RTLBFS_FP32_DEV && precision != RTLBFS_FP64_DEV)
        return RTLBFS_EINVAL;
    if (cells < 1 || cells > RTLBFS_RESIDUAL_STATES_MAX_CELLS || fstride < cells) return RTLBFS_EINVAL;
    if (fstride > ((int64_t)1 << 40)) return RTLBFS_EINVAL;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return RTLBFS_EDEVICE;
    void *part = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (!g_scratch[dev]) {
            void *p = nullptr;
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return RTLBFS_EDEVICE;
            g_scratch[dev] = p;
        }
        part = g_scratch[dev];
    }
    const int64_t want = (cells + kResThreads - 1) / kResThreads;
    const int rows = (int)(want < kResRows ? want : kResRows);
    hipStream_t s = (hipStream_t)hip_stream;
    if (precision == RTLBFS_FP64_PLAIN)
        launch<double, false>(dim, rows, old_state, new_state, cells, fstride, (double *)part, s);
    else if (precision == RTLBFS_FP64_DEV)
        launch<double, true>(dim, rows, old_state, new_state, cells, fstride, (double *)part, s);
    else
        launch<float, true>(dim, rows, old_state, new_state, cells, fstride, (double *)part, s);
    k_residual_states_ratio<<<1, kResThreads, 0, s>>>((const double *)part, rows, dev_out);
    return hipGetLastError() == hipSuccess ? RTLBFS_OK : RTLBFS_EDEVICE;
}
