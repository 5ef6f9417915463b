// rtlbfs_batch.hip -- many independent 2D domains advanced together.
//
// Every member keeps its own mesh, Eq. 63 parameters, Delta-t and ping-pong
// state; all members step in lock-step.  One step is ONE kernel launch over a
// flat work list of (member, tile) items (tiles of a member are contiguous, so
// the XCD-banded block order keeps most halos inside one XCD's L2), and every
// R-step chunk is replayed from a captured HIP graph.  Residuals are reduced
// per member with segment sums; the FP32 mass-drift correction is applied per
// member on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/rtlbfs.h"
#include "host_common.h"
#include "reduce.h"
#include "rtlbfs_device.h"
#include "step2d.h"

using namespace rtlbfs;
using namespace rtlbfs::host;

namespace {

constexpr int kBTX = 16, kBTY = 8;  // batch tile (the fastest of 32x8, 16x16, 64x4, 16x8, 8x8, 16x4 on the 256-cavity batch)
constexpr int kBRedBlocks = 512;

template <typename R, bool DEV, bool RES, bool TL>
__global__ void __launch_bounds__((tile2_threads<kBTX, kBTY>())) __attribute__((amdgpu_waves_per_eu(7, 8))) k_batch_step2d(const Domain *__restrict__ doms,
                                                                              const int2 *__restrict__ work, int cur,
                                                                              double *__restrict__ parts,
                                                                              uint32_t *__restrict__ ctr) {
    const int b = xcd_tile(blockIdx.x, gridDim.x);
    const int2 w = work[b];
    const Domain &d = doms[w.x];
    const int ntx = (d.n[0] + kBTX - 1) / kBTX;
    const int i0 = (w.y % ntx) * kBTX, j0 = (w.y / ntx) * kBTY;
    const uint32_t key = ctr[cur];  // step counter of the stochastic rounding
    tile_step_2d<R, DEV, kBTX, kBTY, RES, TL>(d, i0, j0, (const R *)d.U[cur], (R *)d.U[cur ^ 1],
                                          parts + (int64_t)b * kPartials, key);
    if (blockIdx.x == 0 && threadIdx.x == 0) ctr[cur ^ 1] = key + 1u;
}

// Per-tile integrals {sum r dV, sum theta dV, sum dV} of the deviation state.
template <typename R>
__global__ void __launch_bounds__(256) k_batch_tile_integrals(const Domain *__restrict__ doms,
                                                             const int2 *__restrict__ work, int cur,
                                                             double *__restrict__ parts) {
    __shared__ double sred[kIntParts * 4];
    const int2 w = work[blockIdx.x];
    const Domain &d = doms[w.x];
    const int ntx = (d.n[0] + kBTX - 1) / kBTX;
    const int i0 = (w.y % ntx) * kBTX, j0 = (w.y / ntx) * kBTY;
    const R *U = (const R *)d.U[cur];
    double acc[kIntParts] = {0, 0, 0};
    for (int q = threadIdx.x; q < kBTX * kBTY; q += blockDim.x) {
        const int gi = i0 + q % kBTX, gj = j0 + q / kBTX;
        if (gi >= d.n[0] || gj >= d.n[1]) continue;
        const int64_t c = (int64_t)gj * d.n[0] + gi;
        const double vol = d.w[0][gi] * d.w[1][gj];
        acc[0] += (double)U[c] * vol;
        acc[1] += (double)U[3 * d.fstride + c] * vol;
        acc[2] += vol;
    }
    block_sums<kIntParts>(acc, sred);
    if (threadIdx.x == 0)
        for (int k = 0; k < kIntParts; ++k) parts[(int64_t)blockIdx.x * kIntParts + k] = acc[k];
}

template <typename R>
__global__ void __launch_bounds__(256) k_batch_mass_fix(const Domain *__restrict__ doms,
                                                       const int2 *__restrict__ work, int cur,
                                                       const double *__restrict__ sums, const double *__restrict__ m0) {
    const int2 w = work[blockIdx.x];
    const Domain &d = doms[w.x];
    const int ntx = (d.n[0] + kBTX - 1) / kBTX;
    const int i0 = (w.y % ntx) * kBTX, j0 = (w.y / ntx) * kBTY;
    const R shift = (R)((sums[w.x * kIntParts] - m0[w.x]) / sums[w.x * kIntParts + 2]);
    R *r = (R *)d.U[cur];
    for (int q = threadIdx.x; q < kBTX * kBTY; q += blockDim.x) {
        const int gi = i0 + q % kBTX, gj = j0 + q / kBTX;
        if (gi >= d.n[0] || gj >= d.n[1]) continue;
        r[(int64_t)gj * d.n[0] + gi] -= shift;
    }
}

}  // namespace

struct rtlbfs_batch_handle {
    int count = 0;
    rtlbfs_opts opts;
    std::vector<Problem> prob;
    std::vector<Domain> dom;  // host copies with device pointers
    std::vector<int> begin;   // work-list range of each member
    int nwork = 0;
    hipStream_t stream = nullptr, cap_stream = nullptr;
    char *ws = nullptr;
    bool own_ws = false;
    size_t off_doms = 0, off_work = 0, off_begin = 0, off_parts = 0, off_red = 0, bytes = 0;
    int cur = 0;
    int64_t steps = 0, since_fix = 0;
    bool res_valid = false;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    double *host_buf = nullptr;  // pinned, count * 8 doubles + 16
    std::string err;

    Domain *doms_dev() { return (Domain *)(ws + off_doms); }
    int2 *work_dev() { return (int2 *)(ws + off_work); }
    int *begin_dev() { return (int *)(ws + off_begin); }
    double *parts() { return (double *)(ws + off_parts); }
    double *res_out() { return (double *)(ws + off_red); }                       // count * 8
    double *int_out() { return res_out() + (size_t)count * 8; }                  // count * 3
    double *m0() { return int_out() + (size_t)count * 3; }                        // count
    double *nu_out() { return m0() + count; }                                     // 8
    uint32_t *ctr() { return (uint32_t *)(nu_out() + 8); }                        // 2 step counters
};

namespace {

struct BatchLayout {
    size_t off_doms, off_work, off_begin, off_w, off_state, off_parts, off_red, bytes;
    std::vector<size_t> off_member_w, off_member_geo, off_member_state;
    int nwork;
};

int tiles_of(const rtlbfs_mesh &m) { return ((m.n[0] + kBTX - 1) / kBTX) * ((m.n[1] + kBTY - 1) / kBTY); }

// The batch step launch covers every member's tiles; a dispatch's grid holds
// at most 2^32 - 1 work-items (blocks x threads).
bool batch_launch_fits(int count, const rtlbfs_mesh *meshes) {
    int64_t items = 0;
    for (int m = 0; m < count; ++m) {
        if (meshes[m].n[0] > (1 << 20) || meshes[m].n[1] > (1 << 20)) return false;
        items += (int64_t)((meshes[m].n[0] + kBTX - 1) / kBTX) * ((meshes[m].n[1] + kBTY - 1) / kBTY) *
                 tile2_threads<kBTX, kBTY>();
        if (items > 0xFFFFFFFFll) return false;
    }
    return true;
}

BatchLayout batch_layout(int count, const rtlbfs_mesh *meshes, int precision) {
    BatchLayout l{};
    l.nwork = 0;
    for (int m = 0; m < count; ++m) l.nwork += tiles_of(meshes[m]);
    size_t off = 0;
    l.off_doms = off;
    off += align256(sizeof(Domain) * count);
    l.off_work = off;
    off += align256(sizeof(int2) * (size_t)l.nwork);
    l.off_begin = off;
    off += align256(sizeof(int) * (count + 1));
    l.off_w = off;
    for (int m = 0; m < count; ++m) {
        l.off_member_w.push_back(off);
        off += align256(sizeof(double) * (meshes[m].n[0] + meshes[m].n[1]));
        l.off_member_geo.push_back(off);
        rtlbfs_mesh mm = meshes[m];
        mm.dim = 2;
        off += geometry_bytes(mm, precision);
    }
    l.off_state = off;
    for (int m = 0; m < count; ++m) {
        l.off_member_state.push_back(off);
        const int64_t cells = (int64_t)meshes[m].n[0] * meshes[m].n[1];
        off += 2 * align256((size_t)4 * field_stride(cells) * elem_size(precision));
    }
    l.off_parts = off;
    off += align256(sizeof(double) * (size_t)std::max(l.nwork, kBRedBlocks) * 8);
    l.off_red = off;
    off += align256(sizeof(double) * ((size_t)count * 12 + 24));
    l.bytes = off;
    return l;
}

int bfail(rtlbfs_batch_t h, int code, const std::string &msg) {
    if (h) h->err = msg;
    return code;
}

#define BHIP_TRY(h, call)                                                                      \
    do {                                                                                       \
        hipError_t _e = (call);                                                                \
        if (_e != hipSuccess) return bfail((h), RTLBFS_EDEVICE, std::string(#call) + ": " +   \
                                                                    hipGetErrorString(_e));  \
    } while (0)

template <typename R, bool DEV, bool TL>
hipError_t batch_launch(rtlbfs_batch_t h, bool res, hipStream_t s) {
    if (res)
        k_batch_step2d<R, DEV, true, TL><<<h->nwork, tile2_threads<kBTX, kBTY>(), 0, s>>>(
            h->doms_dev(), h->work_dev(), h->cur, h->parts(), h->ctr());
    else
        k_batch_step2d<R, DEV, false, TL><<<h->nwork, tile2_threads<kBTX, kBTY>(), 0, s>>>(
            h->doms_dev(), h->work_dev(), h->cur, h->parts(), h->ctr());
    return hipGetLastError();
}

hipError_t batch_enqueue_step(rtlbfs_batch_t h, bool res, hipStream_t s) {
    hipError_t e;
    const bool tl = h->opts.method == RTLBFS_METHOD_TLBFS;
    switch (h->opts.precision) {
        case RTLBFS_FP64_PLAIN:
            e = tl ? batch_launch<double, false, true>(h, res, s) : batch_launch<double, false, false>(h, res, s);
            break;
        case RTLBFS_FP64_DEV:
            e = tl ? batch_launch<double, true, true>(h, res, s) : batch_launch<double, true, false>(h, res, s);
            break;
        default:
            e = tl ? batch_launch<float, true, true>(h, res, s) : batch_launch<float, true, false>(h, res, s);
            break;
    }
    if (e != hipSuccess) return e;
    h->cur ^= 1;
    if (res) {
        k_segment_sum<kPartials><<<h->count, 256, 0, s>>>(h->parts(), h->begin_dev(), h->res_out());
        e = hipGetLastError();
    }
    return e;
}

// Per-member integrals of the deviation state into int_out (count x 3).
hipError_t batch_integrals(rtlbfs_batch_t h, hipStream_t s) {
    if (h->opts.precision == RTLBFS_FP32_DEV)
        k_batch_tile_integrals<float><<<h->nwork, 256, 0, s>>>(h->doms_dev(), h->work_dev(), h->cur, h->parts());
    else
        k_batch_tile_integrals<double><<<h->nwork, 256, 0, s>>>(h->doms_dev(), h->work_dev(), h->cur, h->parts());
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_segment_sum<kIntParts><<<h->count, 256, 0, s>>>(h->parts(), h->begin_dev(), h->int_out());
    return hipGetLastError();
}

int batch_capture(rtlbfs_batch_t h, int par, int len) {
    const int saved = h->cur;
    h->cur = par;
    hipGraph_t g = nullptr;
    BHIP_TRY(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int k = 0; k < len && e == hipSuccess; ++k) e = batch_enqueue_step(h, k == len - 1, h->cap_stream);
    hipError_t e2 = hipStreamEndCapture(h->cap_stream, &g);
    h->cur = saved;
    if (e != hipSuccess) return bfail(h, RTLBFS_EDEVICE, std::string("capture: ") + hipGetErrorString(e));
    if (e2 != hipSuccess) return bfail(h, RTLBFS_EDEVICE, std::string("end capture: ") + hipGetErrorString(e2));
    hipError_t e3 = hipGraphInstantiate(&h->graph[par], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e3 != hipSuccess) return bfail(h, RTLBFS_EDEVICE, std::string("instantiate: ") + hipGetErrorString(e3));
    return RTLBFS_OK;
}

int check_member(rtlbfs_batch_t h, int m) {
    if (!h) return RTLBFS_EINVAL;
    if (m < 0 || m >= h->count) return bfail(h, RTLBFS_EINVAL, "member out of range");
    return RTLBFS_OK;
}

int read_member_field(rtlbfs_batch_t h, int m, int k, std::vector<double> &out) {
    const Domain &d = h->dom[m];
    const size_t es = elem_size(h->opts.precision);
    std::vector<char> buf((size_t)d.cells * es);
    BHIP_TRY(h, hipMemcpyAsync(buf.data(), (char *)d.U[h->cur] + (size_t)k * d.fstride * es, buf.size(),
                               hipMemcpyDeviceToHost, h->stream));
    BHIP_TRY(h, hipStreamSynchronize(h->stream));
    out.resize((size_t)d.cells);
    for (int64_t c = 0; c < d.cells; ++c)
        out[c] = es == 4 ? (double)((const float *)buf.data())[c] : ((const double *)buf.data())[c];
    return RTLBFS_OK;
}

}  // namespace

extern "C" {

size_t rtlbfs_batch_workspace_bytes(int count, const rtlbfs_mesh *meshes, const rtlbfs_opts *opts) {
    if (count <= 0 || !meshes) return 0;
    for (int m = 0; m < count; ++m)
        if (meshes[m].dim != 2 || meshes[m].n[0] < 4 || meshes[m].n[1] < 4) return 0;
    if (!batch_launch_fits(count, meshes)) return 0;
    rtlbfs_opts o;
    if (opts) o = *opts;
    else rtlbfs_opts_init(&o);
    return batch_layout(count, meshes, o.precision).bytes;
}

int rtlbfs_batch_create(int count, const rtlbfs_mesh *meshes, const double *Ra, const double *Pr, double Ma,
                        const rtlbfs_bc *bcs, const rtlbfs_opts *opts, void *hip_stream, void *workspace,
                        size_t ws_bytes, rtlbfs_batch_t *out) {
    if (!out) return RTLBFS_EINVAL;
    *out = nullptr;
    if (count <= 0 || !meshes || !bcs || (!Ra && !(opts && opts->phys_given)) || (!Pr && !(opts && opts->phys_given)))
        return RTLBFS_EINVAL;
    rtlbfs_opts o;
    if (opts) o = *opts;
    else rtlbfs_opts_init(&o);
    if (o.residual_every <= 0) o.residual_every = 100;
    if (o.mass_fix_every == 0) o.mass_fix_every = 1000;
    for (int m = 0; m < count; ++m)
        if (meshes[m].dim != 2) return RTLBFS_EUNSUPPORTED;  // batched members are 2D domains
    for (int m = 0; m < count; ++m)
        if (meshes[m].n[0] < 4 || meshes[m].n[1] < 4) return RTLBFS_EINVAL;
    if (!batch_launch_fits(count, meshes)) return RTLBFS_EINVAL;  // the step launch would exceed 2^32 - 1 work-items
    rtlbfs_batch_t h = new (std::nothrow) rtlbfs_batch_handle();
    if (!h) return RTLBFS_ENOMEM;
    h->count = count;
    h->opts = o;
    h->stream = (hipStream_t)hip_stream;
    h->prob.resize(count);
    for (int m = 0; m < count; ++m) {
        std::string why;
        int rc = setup_problem(&meshes[m], &bcs[m], o, Ra ? Ra[m] : 0.0, Pr ? Pr[m] : 0.0, Ma, h->prob[m], why);
        if (rc != RTLBFS_OK) {
            delete h;
            return rc;
        }
    }
    const BatchLayout L = batch_layout(count, meshes, o.precision);
    h->nwork = L.nwork;
    h->off_doms = L.off_doms;
    h->off_work = L.off_work;
    h->off_begin = L.off_begin;
    h->off_parts = L.off_parts;
    h->off_red = L.off_red;
    h->bytes = L.bytes;
    if (workspace) {
        if (ws_bytes < L.bytes) {
            delete h;
            return RTLBFS_ENOMEM;
        }
        h->ws = (char *)workspace;
    } else {
        if (hipMalloc((void **)&h->ws, L.bytes) != hipSuccess) {
            delete h;
            return RTLBFS_ENOMEM;
        }
        h->own_ws = true;
    }
    auto bail = [&](int rc) {
        rtlbfs_batch_destroy(h);
        return rc;
    };
    if (hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess ||
        hipHostMalloc((void **)&h->host_buf, sizeof(double) * ((size_t)count * 12 + 16), hipHostMallocDefault) !=
            hipSuccess)
        return bail(RTLBFS_EDEVICE);

    // Domains, work list, widths, initial states.
    const size_t es = elem_size(o.precision);
    std::vector<int2> work;
    h->begin.assign(count + 1, 0);
    h->dom.resize(count);
    std::vector<double> m0(count);
    for (int m = 0; m < count; ++m) {
        const Problem &P = h->prob[m];
        Domain &d = h->dom[m];
        fill_domain(P, o.precision, o.buoyancy_update_only ? 0 : 1, o.round_nearest, o.max_mach, d);
        double *wdev = (double *)(h->ws + L.off_member_w[m]);
        d.w[0] = wdev;
        d.w[1] = wdev + P.mesh.n[0];
        d.w[2] = nullptr;
        const size_t copy_bytes = align256((size_t)4 * d.fstride * es);
        d.U[0] = h->ws + L.off_member_state[m];
        d.U[1] = h->ws + L.off_member_state[m] + copy_bytes;
        std::vector<char> geo;
        size_t goff[3] = {0, 0, 0};
        pack_geometry(P, o.precision, geo, goff);
        d.geo[0] = h->ws + L.off_member_geo[m] + goff[0];
        d.geo[1] = h->ws + L.off_member_geo[m] + goff[1];
        d.geo[2] = nullptr;
        if (hipMemcpy(wdev, P.widths.data(), P.widths.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(h->ws + L.off_member_geo[m], geo.data(), geo.size(), hipMemcpyHostToDevice) != hipSuccess)
            return bail(RTLBFS_EDEVICE);
        h->begin[m] = (int)work.size();
        for (int t = 0; t < tiles_of(P.mesh); ++t) work.push_back(make_int2(m, t));
        // initial state: rho = 1, u = 0, T - T0 from the profile and noise
        std::vector<double> Tdev;
        initial_Tdev(P, o, Tdev);
        const bool dev = o.precision != RTLBFS_FP64_PLAIN;
        std::vector<char> buf((size_t)4 * d.fstride * es, 0);
        double mass = 0.0;
        for (int64_t c = 0; c < P.cells; ++c) {
            const double f[4] = {dev ? 0.0 : 1.0, 0.0, 0.0, dev ? Tdev[c] : kT0 + Tdev[c]};
            for (int k = 0; k < 4; ++k) {
                if (es == 4) ((float *)buf.data())[(size_t)k * d.fstride + c] = (float)f[k];
                else ((double *)buf.data())[(size_t)k * d.fstride + c] = f[k];
            }
        }
        (void)mass;
        if (hipMemcpy(d.U[0], buf.data(), buf.size(), hipMemcpyHostToDevice) != hipSuccess) return bail(RTLBFS_EDEVICE);
        m0[m] = 0.0;  // the initial density deviation is exactly zero
    }
    h->begin[count] = (int)work.size();
    if (hipMemcpy(h->doms_dev(), h->dom.data(), sizeof(Domain) * count, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->work_dev(), work.data(), sizeof(int2) * work.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->begin_dev(), h->begin.data(), sizeof(int) * (count + 1), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->m0(), m0.data(), sizeof(double) * count, hipMemcpyHostToDevice) != hipSuccess)
        return bail(RTLBFS_EDEVICE);
    const uint32_t zero2[2] = {0u, 0u};
    if (hipMemcpy(h->ctr(), zero2, sizeof(zero2), hipMemcpyHostToDevice) != hipSuccess) return bail(RTLBFS_EDEVICE);
    *out = h;
    return RTLBFS_OK;
}

int rtlbfs_batch_step(rtlbfs_batch_t h, int64_t n) {
    if (!h) return RTLBFS_EINVAL;
    if (n < 0) return bfail(h, RTLBFS_EINVAL, "negative step count");
    const int C = h->opts.residual_every;
    const bool graphs = h->opts.graph_steps >= 0;
    while (n > 0) {
        const int64_t chunk = std::min<int64_t>(n, C);
        if (graphs && chunk == C) {
            if (!h->graph[h->cur]) {
                int rc = batch_capture(h, h->cur, C);
                if (rc != RTLBFS_OK) return rc;
            }
            BHIP_TRY(h, hipGraphLaunch(h->graph[h->cur], h->stream));
            if (C & 1) h->cur ^= 1;
        } else {
            for (int64_t k = 0; k < chunk; ++k) BHIP_TRY(h, batch_enqueue_step(h, k == chunk - 1, h->stream));
        }
        n -= chunk;
        h->steps += chunk;
        h->since_fix += chunk;
        h->res_valid = true;
        if (h->opts.precision == RTLBFS_FP32_DEV && h->opts.mass_fix_every > 0 &&
            h->since_fix >= h->opts.mass_fix_every) {
            BHIP_TRY(h, batch_integrals(h, h->stream));
            k_batch_mass_fix<float><<<h->nwork, 256, 0, h->stream>>>(h->doms_dev(), h->work_dev(), h->cur,
                                                                     h->int_out(), h->m0());
            BHIP_TRY(h, hipGetLastError());
            h->since_fix = 0;
        }
    }
    return RTLBFS_OK;
}

int rtlbfs_batch_sync(rtlbfs_batch_t h) {
    if (!h) return RTLBFS_EINVAL;
    BHIP_TRY(h, hipMemcpyAsync(h->host_buf, h->res_out(), sizeof(double) * kPartials * h->count,
                               hipMemcpyDeviceToHost, h->stream));
    BHIP_TRY(h, hipStreamSynchronize(h->stream));
    if (h->res_valid)
        for (int m = 0; m < h->count; ++m)
            if (h->host_buf[m * kPartials + 4] != 0.0) return bfail(h, RTLBFS_EDIVERGED, "a member diverged");
    return RTLBFS_OK;
}

int rtlbfs_batch_diverged(rtlbfs_batch_t h, int *host_flags) {
    if (!h || !host_flags) return RTLBFS_EINVAL;
    if (!h->res_valid) return bfail(h, RTLBFS_ESTATE, "no residual step yet");
    BHIP_TRY(h, hipMemcpyAsync(h->host_buf, h->res_out(), sizeof(double) * kPartials * h->count,
                               hipMemcpyDeviceToHost, h->stream));
    BHIP_TRY(h, hipStreamSynchronize(h->stream));
    for (int m = 0; m < h->count; ++m) host_flags[m] = h->host_buf[m * kPartials + 4] != 0.0 ? 1 : 0;
    return RTLBFS_OK;
}

int rtlbfs_batch_residual(rtlbfs_batch_t h, int member, double *res_u, double *res_T) {
    int rc = check_member(h, member);
    if (rc != RTLBFS_OK) return rc;
    if (!res_u || !res_T) return RTLBFS_EINVAL;
    if (!h->res_valid) return bfail(h, RTLBFS_ESTATE, "no residual step yet");
    rc = rtlbfs_batch_sync(h);
    const double *r = h->host_buf + member * kPartials;
    *res_u = r[1] > 0.0 ? r[0] / r[1] : 0.0;
    *res_T = r[3] != 0.0 ? r[2] / r[3] : 0.0;
    return rc;
}

int rtlbfs_batch_nusselt(rtlbfs_batch_t h, int member, rtlbfs_nu *out) {
    int rc = check_member(h, member);
    if (rc != RTLBFS_OK) return rc;
    if (!out) return RTLBFS_EINVAL;
    const Problem &P = h->prob[member];
    const int ha = P.haxis;
    if (ha < 0) return bfail(h, RTLBFS_EINVAL, "no pair of isothermal walls");
    const double Tlo = P.bc.Tdev[2 * ha], Thi = P.bc.Tdev[2 * ha + 1];
    const double dTw = std::fabs(Thi - Tlo);
    if (dTw == 0.0) return bfail(h, RTLBFS_EINVAL, "isothermal walls at equal temperature");
    const int hot_hi = Thi > Tlo;
    const Domain &d = h->dom[member];
    switch (h->opts.precision) {
        case RTLBFS_FP64_PLAIN:
            k_nusselt<double, false><<<kBRedBlocks, 256, 0, h->stream>>>(d, (const double *)d.U[h->cur], ha, hot_hi,
                                                                         P.length[ha], dTw, h->parts());
            break;
        case RTLBFS_FP64_DEV:
            k_nusselt<double, true><<<kBRedBlocks, 256, 0, h->stream>>>(d, (const double *)d.U[h->cur], ha, hot_hi,
                                                                        P.length[ha], dTw, h->parts());
            break;
        default:
            k_nusselt<float, true><<<kBRedBlocks, 256, 0, h->stream>>>(d, (const float *)d.U[h->cur], ha, hot_hi,
                                                                       P.length[ha], dTw, h->parts());
            break;
    }
    BHIP_TRY(h, hipGetLastError());
    k_nusselt_finalize<0><<<1, 256, 0, h->stream>>>(h->parts(), kBRedBlocks, h->nu_out());
    BHIP_TRY(h, hipGetLastError());
    double *hb = h->host_buf + (size_t)h->count * 12;
    BHIP_TRY(h, hipMemcpyAsync(hb, h->nu_out(), 8 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    BHIP_TRY(h, hipStreamSynchronize(h->stream));
    out->hot_avg = hb[0] / hb[1];
    out->cold_avg = hb[2] / hb[3];
    out->volume = P.length[ha] / (d.chi * dTw) * hb[4] / hb[5];
    out->hot_max = hb[6];
    out->cold_max = hb[7];
    return RTLBFS_OK;
}

int rtlbfs_batch_get_field(rtlbfs_batch_t h, int member, int field, double *host_out, size_t count) {
    int rc = check_member(h, member);
    if (rc != RTLBFS_OK) return rc;
    if (!host_out || field < 0 || field > 3) return bfail(h, RTLBFS_EINVAL, "bad field or buffer");
    const Domain &d = h->dom[member];
    if (count < (size_t)d.cells) return bfail(h, RTLBFS_EINVAL, "count smaller than the member's cells");
    const bool dev = h->opts.precision != RTLBFS_FP64_PLAIN;
    std::vector<double> r, f;
    if ((rc = read_member_field(h, member, 0, r)) != RTLBFS_OK) return rc;
    if (field > 0 && (rc = read_member_field(h, member, field, f)) != RTLBFS_OK) return rc;
    for (int64_t c = 0; c < d.cells; ++c) {
        const double rho = dev ? 1.0 + r[c] : r[c];
        if (field == 0) host_out[c] = rho;
        else if (field <= 2) host_out[c] = f[c] / rho;
        else host_out[c] = f[c] / rho + (dev ? kT0 : 0.0);
    }
    return RTLBFS_OK;
}

int rtlbfs_batch_get_info(rtlbfs_batch_t h, int member, rtlbfs_info *out) {
    int rc = check_member(h, member);
    if (rc != RTLBFS_OK) return rc;
    if (!out) return RTLBFS_EINVAL;
    std::memset(out, 0, sizeof(*out));
    const Problem &P = h->prob[member];
    const Domain &d = h->dom[member];
    out->cells = P.cells;
    out->steps = h->steps;
    out->L = P.L;
    out->nu = d.nu;
    out->chi = d.chi;
    out->beta_g = d.bg;
    out->tau_f = d.tau_f;
    out->tau_g = d.tau_g;
    out->dtl = d.dtl;
    out->dt = d.dt;
    for (int a = 0; a < 3; ++a) out->length[a] = a < 2 ? P.length[a] : 1.0;
    out->precision = h->opts.precision;
    out->tile_x = kBTX;
    out->tile_y = kBTY;
    out->tile_z = 1;
    out->steps_per_launch = 1;
    return RTLBFS_OK;
}

int rtlbfs_batch_destroy(rtlbfs_batch_t h) {
    if (!h) return RTLBFS_OK;
    (void)hipStreamSynchronize(h->stream);
    for (int k = 0; k < 2; ++k)
        if (h->graph[k]) (void)hipGraphExecDestroy(h->graph[k]);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    if (h->host_buf) (void)hipHostFree(h->host_buf);
    if (h->own_ws && h->ws) (void)hipFree(h->ws);
    delete h;
    return RTLBFS_OK;
}

}  // extern "C"
