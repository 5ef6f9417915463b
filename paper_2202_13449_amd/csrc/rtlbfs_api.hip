// rtlbfs_api.hip -- host runtime behind include/rtlbfs.h: validation, mesh
// (Eq. 74), Eq. 63 parameters, seeded initial state, workspace layout,
// graph-captured step chunks, FP64 diagnostics and field access.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/rtlbfs.h"
#include "reduce.h"
#include "rtlbfs_device.h"
#include "step2d.h"
#include "step3d.h"
#include "step3d_march.h"
#include "host_common.h"
#include "curv2d.h"
#include "curv_host.h"
#include "curv3d.h"
#include "curv3_host.h"

using namespace rtlbfs;
using namespace rtlbfs::host;

// ----------------------------------------------------------------- kernels --

template <typename R, bool DEV, int TX, int TY, bool RES, bool TL, int NSUB>
__global__ void __launch_bounds__((tile2_threads<TX, TY, NSUB>())) __attribute__((amdgpu_waves_per_eu(7, 8))) k_step2d(Domain d, const R *__restrict__ Uin,
                                                                    R *__restrict__ Uout, double *__restrict__ parts,
                                                                    const uint32_t *__restrict__ ctr_in,
                                                                    uint32_t *__restrict__ ctr_out) {
    const uint32_t key = *ctr_in;  // step counter of the stochastic rounding
    const int ntx = (d.n[0] + TX - 1) / TX;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int i0 = (t % ntx) * TX, j0 = (t / ntx) * TY;
    tile_step_2d<R, DEV, TX, TY, RES, TL, NSUB>(d, i0, j0, Uin, Uout, parts + (int64_t)t * kPartials, key);
    if (blockIdx.x == 0 && threadIdx.x == 0) *ctr_out = key + (uint32_t)NSUB;
}

template <typename R, bool DEV, int TX, int TY, int TZ, bool RES, bool TL>
__global__ void __launch_bounds__((tile3_threads<TX, TY, TZ>())) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 5 : 3, 8))) k_step3d(Domain d, const R *__restrict__ Uin, R *__restrict__ Uout,
                                                double *__restrict__ parts, const uint32_t *__restrict__ ctr_in,
                                                uint32_t *__restrict__ ctr_out) {
    const uint32_t key = *ctr_in;
    // tiles x-fastest; each XCD takes a contiguous band of them (see xcd_tile)
    const int ntx = (d.n[0] + TX - 1) / TX, nty = (d.n[1] + TY - 1) / TY;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int bx = t % ntx, by = (t / ntx) % nty, bz = t / (ntx * nty);
    tile_step_3d<R, DEV, TX, TY, TZ, RES, TL>(d, bx * TX, by * TY, bz * TZ, Uin, Uout,
                                              parts + (int64_t)t * kPartials, key);
    if (blockIdx.x == 0 && threadIdx.x == 0) *ctr_out = key + 1u;
}

// Launch shapes of the body-fitted 2D step kernel (opts.tile = index + 1);
// the autotuner picks one per handle (the best shape depends on the mesh and
// the precision: 16 x 8 and 8 x 8 spread a 450 x 300 mesh over the CUs more
// evenly than 16 x 16).
struct TileC {
    int tx, ty;
};
constexpr TileC kTilesC[] = {{16, 16}, {16, 8}, {32, 8}, {8, 8}};
constexpr int kNumTilesC = sizeof(kTilesC) / sizeof(kTilesC[0]);

template <typename R, bool DEV, bool TL, int TX, int TY, bool RES>
__global__ void __launch_bounds__((curv_threads<TX, TY>())) k_curv_step(Domain d, CurvGeo g,
                                                                      const R *__restrict__ Uin,
                                                                      R *__restrict__ Uout,
                                                                      double *__restrict__ parts,
                                                                      const uint32_t *__restrict__ ctr_in,
                                                                      uint32_t *__restrict__ ctr_out) {
    const uint32_t key = *ctr_in;
    const int ntx = (d.n[0] + TX - 1) / TX;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    tile_step_curv<R, DEV, TL, TX, TY, RES>(d, g, (t % ntx) * TX, (t / ntx) * TY, Uin, Uout,
                                            parts + (int64_t)t * kPartials, key);
    if (blockIdx.x == 0 && threadIdx.x == 0) *ctr_out = key + 1u;
}

namespace {

// The column kernel: a TX x TY column marching through planes [z0, z0 + sz).
// FP32 targets five wavefronts per SIMD (three 16 x 8 blocks of seven per
// CU, about 47 KB of LDS each); FP64 needs twice the LDS and fits one block.
template <typename R, bool DEV, int TX, int TY, bool RES, bool TL>
__global__ void __launch_bounds__((col3_threads<TX, TY>())) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 4 : 2, 8))) k_step3d_col(Domain d, const R *__restrict__ Uin, R *__restrict__ Uout,
                                                double *__restrict__ parts, const uint32_t *__restrict__ ctr_in,
                                                uint32_t *__restrict__ ctr_out, int sz) {
    const uint32_t key = *ctr_in;
    // columns x-fastest, then segments; each XCD takes a contiguous band (see xcd_tile)
    const int ntx = (d.n[0] + TX - 1) / TX, nty = (d.n[1] + TY - 1) / TY;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int bx = t % ntx, by = (t / ntx) % nty, bs = t / (ntx * nty);
    const int z0 = bs * sz, z1 = min(z0 + sz, d.n[2]);
    column_step_3d<R, DEV, TX, TY, RES, TL>(d, bx * TX, by * TY, z0, z1, Uin, Uout, parts + (int64_t)t * kPartials, key);
    if (blockIdx.x == 0 && threadIdx.x == 0) *ctr_out = key + 1u;
}

// 2D launch shapes the autotuner chooses from (opts.tile = index + 1): tile
// size, time steps per launch, and the one-step shape of the same tile (used
// for an odd last step).
struct Tile2 {
    int tx, ty, nsub, single;
};
constexpr Tile2 kTiles2[] = {{32, 8, 1, 0},  {16, 16, 1, 1}, {64, 4, 1, 2}, {16, 8, 1, 3}, {8, 8, 1, 4},
                             {16, 16, 2, 1}, {32, 8, 2, 0},  {16, 8, 2, 3}, {8, 8, 2, 4}};
constexpr int kNumTiles2 = sizeof(kTiles2) / sizeof(kTiles2[0]);
// Threads per block of each 2D launch shape, in kTiles2 order (the shapes
// launch_step instantiates).
constexpr int kTiles2Threads[] = {tile2_threads<32, 8, 1>(),  tile2_threads<16, 16, 1>(), tile2_threads<64, 4, 1>(),
                                  tile2_threads<16, 8, 1>(),  tile2_threads<8, 8, 1>(),   tile2_threads<16, 16, 2>(),
                                  tile2_threads<32, 8, 2>(),  tile2_threads<16, 8, 2>(),  tile2_threads<8, 8, 2>()};
static_assert(sizeof(kTiles2Threads) / sizeof(kTiles2Threads[0]) == kNumTiles2, "one thread count per shape");
// 3D tile, one thread per face: 240 faces on four wavefronts.  In FP32 its
// ~30 KB of LDS and 96 VGPRs leave room for five blocks (20 wavefronts) per
// CU, where the 8 x 4 x 4 tile's eight wavefronts fit twice (16).
constexpr int kTX3 = 4, kTY3 = 4, kTZ3 = 4;
// 3D launch shapes (opts.tile = index + 1): the 4 x 4 x 4 tile kernel (the
// default), then columns of tx x ty cells marching through segments of sz
// planes.  The column kernels compute each face once per segment (3.2 faces
// per cell for 16 x 8 columns against 3.75 for the tiles) but fit fewer
// wavefronts per CU; on the 192^3 cube they are not faster in FP32, and
// their results differ from the tile kernel's in the last bit of a few
// cells (the two kernels contract multiply-adds differently), so they are
// taken only when asked for.
struct Tile3S {
    int col, tx, ty, sz;
};
constexpr Tile3S kTiles3[] = {{0, kTX3, kTY3, kTZ3}, {1, 16, 8, 32}, {1, 16, 8, 48},
                              {1, 16, 8, 64},        {1, 16, 8, 96}, {1, 8, 8, 48}};
constexpr int kNumTiles3 = sizeof(kTiles3) / sizeof(kTiles3[0]);
static_assert(kNumTiles3 <= kNumTiles2, "the autotuner's arrays hold every shape");

int blocks3(const rtlbfs_mesh &m, int tile) {
    const Tile3S t = kTiles3[tile];  // sz: the cube tile's depth, or the column's segment length
    return ((m.n[0] + t.tx - 1) / t.tx) * ((m.n[1] + t.ty - 1) / t.ty) * ((m.n[2] + t.sz - 1) / t.sz);
}

int threads3(int tile) {
    const Tile3S t = kTiles3[tile];
    if (!t.col) return tile3_threads<kTX3, kTY3, kTZ3>();
    return t.tx == 16 ? col3_threads<16, 8>() : col3_threads<8, 8>();
}

// A dispatch's grid holds at most 2^32 - 1 work-items (blocks x threads).
constexpr int64_t kMaxWorkItems = 0xFFFFFFFFll;

// Every step launch the autotuner may pick for this Cartesian mesh fits one
// dispatch (meshes within the per-axis limit of 2^20 cells).
bool step_launches_fit(const rtlbfs_mesh &m) {
    if (m.dim == 2) {
        for (int t = 0; t < kNumTiles2; ++t) {
            const int64_t b = (int64_t)((m.n[0] + kTiles2[t].tx - 1) / kTiles2[t].tx) *
                              ((m.n[1] + kTiles2[t].ty - 1) / kTiles2[t].ty);
            if (b * kTiles2Threads[t] > kMaxWorkItems) return false;
        }
        return true;
    }
    for (int t = 0; t < kNumTiles3; ++t)
        if ((int64_t)blocks3(m, t) * threads3(t) > kMaxWorkItems) return false;
    return true;
}
constexpr int kRedBlocks = 512;                // blocks of the diagnostics kernels

struct Layout {
    size_t off_U[2], off_w, off_geo, off_parts, off_red, bytes;
    int64_t cells;
    int nparts;
};


int step_blocks(const rtlbfs_mesh &m, int tile = 0) {
    if (m.dim == 2) {
        const Tile2 t = kTiles2[tile];
        return ((m.n[0] + t.tx - 1) / t.tx) * ((m.n[1] + t.ty - 1) / t.ty);
    }
    return blocks3(m, tile);
}


Layout make_layout(const rtlbfs_mesh &m, int precision) {
    Layout l{};
    l.cells = (int64_t)m.n[0] * m.n[1] * (m.dim == 3 ? m.n[2] : 1);
    const int nf = m.dim + 2;
    // Fields of one copy are `field_stride` elements apart (a multiple of 64
    // elements, so every field starts 256-byte aligned).
    const size_t copy_bytes = (size_t)nf * field_stride(l.cells) * elem_size(precision);
    size_t off = 0;
    l.off_U[0] = off;
    off += copy_bytes;
    l.off_U[1] = off;
    off += copy_bytes;
    l.off_w = off;
    off += align256(sizeof(double) * (m.n[0] + m.n[1] + (m.dim == 3 ? m.n[2] : 0)));
    l.off_geo = off;
    off += geometry_bytes(m, precision);
    l.nparts = kRedBlocks;
    for (int t = 0; t < (m.dim == 2 ? kNumTiles2 : kNumTiles3); ++t) l.nparts = std::max(l.nparts, step_blocks(m, t));
    l.off_parts = off;
    off += align256(sizeof(double) * (size_t)l.nparts * 8);
    l.off_red = off;  // residual sums (8), Nusselt (8), integrals (4), M0 (1), mass-fix sums (4)
    off += align256(sizeof(double) * 32);
    l.bytes = off;
    return l;
}

}  // namespace

struct rtlbfs_handle {
    rtlbfs_mesh mesh;
    rtlbfs_bc bc;
    rtlbfs_opts opts;
    Domain dom;
    Layout lay;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    char *ws = nullptr;
    bool own_ws = false;
    int cur = 0;  // which ping-pong copy holds the state
    int tile = 0; // index into kTiles2 (2D)
    float tune_ms[kNumTiles2] = {};  // autotuner timings per launch shape (ms per step)
    int64_t steps = 0;
    int64_t since_fix = 0;
    bool res_valid = false;
    double L = 0, length[3] = {1, 1, 1};
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    int graph_len = 0;
    double *host_buf = nullptr;  // pinned scratch for small reads
    std::string err;
    // body-fitted mesh (rtlbfs_curv_create)
    bool curv = false;
    CurvGeo cg{};
    const double *fi64 = nullptr, *fj64 = nullptr;  // FP64 face records (diagnostics)
    int64_t nfi = 0, nfj = 0;
    int ckind[6] = {0, 0, 0, 0, 0, 0};
    double cTw[6] = {0, 0, 0, 0, 0, 0};             // absolute wall temperatures
    std::vector<double> ccx, ccy, carea;            // host copy of the cell geometry
    // 3D body-fitted mesh (rtlbfs_curv3_create)
    bool curv3 = false;
    bool c3_layer = false;  // 3D body-fitted: the fused single-layer kernel (else three kernels)
    Curv3Geo c3{};
    const double *c3rec64[3] = {nullptr, nullptr, nullptr};  // FP64 face records (diagnostics)
    std::vector<double> c3cx, c3cy, c3cz, c3vol;

    void *U(int k) { return ws + lay.off_U[k]; }
    double *parts() { return (double *)(ws + lay.off_parts); }
    double *red() { return (double *)(ws + lay.off_red); }
    double *res_out() { return red(); }         // [0..5)
    double *nu_out() { return red() + 8; }      // [8..16)
    double *int_out() { return red() + 16; }    // [16..19)
    double *m0() { return red() + 20; }         // [20]
    double *fix_out() { return red() + 24; }    // [24..27)
    uint32_t *ctr() { return (uint32_t *)(red() + 28); }  // step counters of the two copies
};

namespace {

thread_local std::string g_create_err;  // detail of the last failed create on this thread

int fail(rtlbfs_t h, int code, const std::string &msg) {
    if (h) h->err = msg;
    g_create_err = msg;
    return code;
}

int hip_fail(rtlbfs_t h, hipError_t e, const char *what) {
    return fail(h, RTLBFS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(h, call)                                       \
    do {                                                       \
        hipError_t _e = (call);                                \
        if (_e != hipSuccess) return hip_fail((h), _e, #call); \
    } while (0)

template <typename R>
void to_storage(const std::vector<double> &src, std::vector<char> &dst) {
    dst.resize(src.size() * sizeof(R));
    R *p = (R *)dst.data();
    for (size_t i = 0; i < src.size(); ++i) p[i] = (R)src[i];
}

template <typename R>
void from_storage(const char *src, size_t n, double *dst) {
    const R *p = (const R *)src;
    for (size_t i = 0; i < n; ++i) dst[i] = (double)p[i];
}

// Upload the state given as primitives (rho, u axis-major, T' = T - T0).
int upload_prims(rtlbfs_t h, const double *rho, const double *u, const double *Tdev) {
    const int64_t N = h->lay.cells;
    const int D = h->mesh.dim, nf = D + 2;
    const bool dev = h->opts.precision != RTLBFS_FP64_PLAIN;
    std::vector<double> f((size_t)N);
    std::vector<char> buf;
    const size_t field_bytes = (size_t)h->dom.fstride * elem_size(h->opts.precision);
    for (int k = 0; k < nf; ++k) {
        for (int64_t c = 0; c < N; ++c) {
            if (k == 0) f[c] = dev ? rho[c] - 1.0 : rho[c];
            else if (k <= D) f[c] = rho[c] * u[(int64_t)(k - 1) * N + c];
            else f[c] = dev ? rho[c] * Tdev[c] : rho[c] * (kT0 + Tdev[c]);
        }
        if (h->opts.precision == RTLBFS_FP32_DEV) to_storage<float>(f, buf);
        else to_storage<double>(f, buf);
        HIP_TRY(h, hipMemcpyAsync((char *)h->U(h->cur) + k * field_bytes, buf.data(), buf.size(),
                                  hipMemcpyHostToDevice, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
    }
    h->res_valid = false;
    return RTLBFS_OK;
}

int read_stored(rtlbfs_t h, int k, std::vector<double> &out) {
    const int64_t N = h->lay.cells;
    const size_t es = elem_size(h->opts.precision);
    const size_t field_bytes = (size_t)h->dom.fstride * es;
    std::vector<char> buf((size_t)N * es);
    HIP_TRY(h, hipMemcpyAsync(buf.data(), (char *)h->U(h->cur) + k * field_bytes, buf.size(), hipMemcpyDeviceToHost,
                              h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    out.resize((size_t)N);
    if (es == 4) from_storage<float>(buf.data(), (size_t)N, out.data());
    else from_storage<double>(buf.data(), (size_t)N, out.data());
    return RTLBFS_OK;
}

template <typename R, bool DEV, int TX, int TY, bool TL, int NSUB>
hipError_t launch_step2d(const Domain &d, const R *Uin, R *Uout, double *parts, const uint32_t *ci, uint32_t *co,
                         bool res, hipStream_t s) {
    const int nb = ((d.n[0] + TX - 1) / TX) * ((d.n[1] + TY - 1) / TY);
    constexpr int nt = tile2_threads<TX, TY, NSUB>();
    if (res) k_step2d<R, DEV, TX, TY, true, TL, NSUB><<<nb, nt, 0, s>>>(d, Uin, Uout, parts, ci, co);
    else k_step2d<R, DEV, TX, TY, false, TL, NSUB><<<nb, nt, 0, s>>>(d, Uin, Uout, parts, ci, co);
    return hipGetLastError();
}

template <typename R, bool DEV, bool TL>
hipError_t launch_step(rtlbfs_t h, int tile, int src, bool res, hipStream_t s) {
    const Domain &d = h->dom;
    const R *Uin = (const R *)h->U(src);
    R *Uout = (R *)h->U(src ^ 1);
    const uint32_t *ci = h->ctr() + src;
    uint32_t *co = h->ctr() + (src ^ 1);
    if (d.dim == 2) {
        double *P = h->parts();
        switch (tile) {
            case 0: return launch_step2d<R, DEV, 32, 8, TL, 1>(d, Uin, Uout, P, ci, co, res, s);
            case 1: return launch_step2d<R, DEV, 16, 16, TL, 1>(d, Uin, Uout, P, ci, co, res, s);
            case 2: return launch_step2d<R, DEV, 64, 4, TL, 1>(d, Uin, Uout, P, ci, co, res, s);
            case 3: return launch_step2d<R, DEV, 16, 8, TL, 1>(d, Uin, Uout, P, ci, co, res, s);
            case 4: return launch_step2d<R, DEV, 8, 8, TL, 1>(d, Uin, Uout, P, ci, co, res, s);
            case 5: return launch_step2d<R, DEV, 16, 16, TL, 2>(d, Uin, Uout, P, ci, co, res, s);
            case 6: return launch_step2d<R, DEV, 32, 8, TL, 2>(d, Uin, Uout, P, ci, co, res, s);
            case 7: return launch_step2d<R, DEV, 16, 8, TL, 2>(d, Uin, Uout, P, ci, co, res, s);
            default: return launch_step2d<R, DEV, 8, 8, TL, 2>(d, Uin, Uout, P, ci, co, res, s);
        }
    }
    const int grid = blocks3(h->mesh, tile);
    const Tile3S t3 = kTiles3[tile];
    if (!t3.col) {
        constexpr int nt = tile3_threads<kTX3, kTY3, kTZ3>();
        if (res) k_step3d<R, DEV, kTX3, kTY3, kTZ3, true, TL><<<grid, nt, 0, s>>>(d, Uin, Uout, h->parts(), ci, co);
        else k_step3d<R, DEV, kTX3, kTY3, kTZ3, false, TL><<<grid, nt, 0, s>>>(d, Uin, Uout, h->parts(), ci, co);
    } else if (t3.tx == 16) {
        constexpr int nt = col3_threads<16, 8>();
        if (res) k_step3d_col<R, DEV, 16, 8, true, TL><<<grid, nt, 0, s>>>(d, Uin, Uout, h->parts(), ci, co, t3.sz);
        else k_step3d_col<R, DEV, 16, 8, false, TL><<<grid, nt, 0, s>>>(d, Uin, Uout, h->parts(), ci, co, t3.sz);
    } else {
        constexpr int nt = col3_threads<8, 8>();
        if (res) k_step3d_col<R, DEV, 8, 8, true, TL><<<grid, nt, 0, s>>>(d, Uin, Uout, h->parts(), ci, co, t3.sz);
        else k_step3d_col<R, DEV, 8, 8, false, TL><<<grid, nt, 0, s>>>(d, Uin, Uout, h->parts(), ci, co, t3.sz);
    }
    return hipGetLastError();
}

int curv_blocks(const rtlbfs_mesh &m, int tile) {
    const TileC t = kTilesC[tile];
    return ((m.n[0] + t.tx - 1) / t.tx) * ((m.n[1] + t.ty - 1) / t.ty);
}

// Threads per block of each body-fitted 2D launch shape, in kTilesC order.
constexpr int kTilesCThreads[] = {curv_threads<16, 16>(), curv_threads<16, 8>(), curv_threads<32, 8>(),
                                  curv_threads<8, 8>()};
static_assert(sizeof(kTilesCThreads) / sizeof(kTilesCThreads[0]) == kNumTilesC, "one thread count per shape");

// Every launch shape of the body-fitted 2D step fits one dispatch for an
// ni x nj mesh (each axis within 2^20 cells).
bool curv_launches_fit(int ni, int nj) {
    for (int t = 0; t < kNumTilesC; ++t) {
        const int64_t b = (int64_t)((ni + kTilesC[t].tx - 1) / kTilesC[t].tx) * ((nj + kTilesC[t].ty - 1) / kTilesC[t].ty);
        if (b * kTilesCThreads[t] > kMaxWorkItems) return false;
    }
    return true;
}

// The fused single-layer kernel applies: one periodic cell along j, walls
// along i and k.
bool c3_is_layer(const int n[3], const int kind[6]) {
    return n[1] == 1 && kind[2] == RTLBFS_PERIODIC && kind[0] != RTLBFS_PERIODIC && kind[4] != RTLBFS_PERIODIC;
}

int c3_layer_blocks(const int n[3]) {
    return ((n[0] + kC3LayerTX - 1) / kC3LayerTX) * ((n[2] + kC3LayerTZ - 1) / kC3LayerTZ);
}

// Blocks of one step launch of the handle (rows of residual partials).
int handle_blocks(const rtlbfs_t h, int tile) {
    if (h->curv3 && h->c3_layer) return c3_layer_blocks(h->mesh.n);
    if (h->curv3) return (int)((h->lay.cells + kC3Threads - 1) / kC3Threads);
    return h->curv ? curv_blocks(h->mesh, tile) : step_blocks(h->mesh, tile);
}

template <typename R, bool DEV, bool TL>
hipError_t launch_curv3(rtlbfs_t h, int src, bool res, hipStream_t s) {
    const R *Uin = (const R *)h->U(src);
    R *Uout = (R *)h->U(src ^ 1);
    if (h->c3_layer) {
        constexpr int TX = kC3LayerTX, TZ = kC3LayerTZ, lt = c3_layer_threads<TX, TZ>();
        const int lb = c3_layer_blocks(h->mesh.n);
        if (res) k_c3_layer<R, DEV, TL, true, TX, TZ><<<lb, lt, 0, s>>>(h->dom, h->c3, Uin, Uout, h->parts(), h->ctr() + src, h->ctr() + (src ^ 1));
        else k_c3_layer<R, DEV, TL, false, TX, TZ><<<lb, lt, 0, s>>>(h->dom, h->c3, Uin, Uout, h->parts(), h->ctr() + src, h->ctr() + (src ^ 1));
        return hipGetLastError();
    }
    constexpr int nt = kC3Threads;
    const int cb = (int)((h->lay.cells + nt - 1) / nt), fb = (int)((h->c3.nfaces + nt - 1) / nt);
    k_c3_grad<R, DEV><<<cb, nt, 0, s>>>(h->dom, h->c3, Uin);
    k_c3_flux<R, DEV, TL><<<fb, nt, 0, s>>>(h->dom, h->c3, Uin);
    if (res) k_c3_update<R, DEV, true><<<cb, nt, 0, s>>>(h->dom, h->c3, Uin, Uout, h->parts(), h->ctr() + src, h->ctr() + (src ^ 1));
    else k_c3_update<R, DEV, false><<<cb, nt, 0, s>>>(h->dom, h->c3, Uin, Uout, h->parts(), h->ctr() + src, h->ctr() + (src ^ 1));
    return hipGetLastError();
}

template <typename R, bool DEV, bool TL, int TX, int TY>
hipError_t launch_curv_shape(rtlbfs_t h, int src, bool res, hipStream_t s) {
    const R *Uin = (const R *)h->U(src);
    R *Uout = (R *)h->U(src ^ 1);
    const uint32_t *ci = h->ctr() + src;
    uint32_t *co = h->ctr() + (src ^ 1);
    const int nb = ((h->mesh.n[0] + TX - 1) / TX) * ((h->mesh.n[1] + TY - 1) / TY);
    constexpr int nt = curv_threads<TX, TY>();
    if (res) k_curv_step<R, DEV, TL, TX, TY, true><<<nb, nt, 0, s>>>(h->dom, h->cg, Uin, Uout, h->parts(), ci, co);
    else k_curv_step<R, DEV, TL, TX, TY, false><<<nb, nt, 0, s>>>(h->dom, h->cg, Uin, Uout, h->parts(), ci, co);
    return hipGetLastError();
}

template <typename R, bool DEV, bool TL>
hipError_t launch_curv(rtlbfs_t h, int tile, int src, bool res, hipStream_t s) {
    switch (tile) {
        case 0: return launch_curv_shape<R, DEV, TL, 16, 16>(h, src, res, s);
        case 1: return launch_curv_shape<R, DEV, TL, 16, 8>(h, src, res, s);
        case 2: return launch_curv_shape<R, DEV, TL, 32, 8>(h, src, res, s);
        default: return launch_curv_shape<R, DEV, TL, 8, 8>(h, src, res, s);
    }
}

// One step kernel from copy `src` into the other copy (no state change on the host side).
hipError_t launch_any(rtlbfs_t h, int tile, int src, bool res, hipStream_t s) {
    const bool tl = h->opts.method == RTLBFS_METHOD_TLBFS;
    if (h->curv3) {
        switch (h->opts.precision) {
            case RTLBFS_FP64_PLAIN:
                return tl ? launch_curv3<double, false, true>(h, src, res, s) : launch_curv3<double, false, false>(h, src, res, s);
            case RTLBFS_FP64_DEV:
                return tl ? launch_curv3<double, true, true>(h, src, res, s) : launch_curv3<double, true, false>(h, src, res, s);
            default:
                return tl ? launch_curv3<float, true, true>(h, src, res, s) : launch_curv3<float, true, false>(h, src, res, s);
        }
    }
    if (h->curv) {
        switch (h->opts.precision) {
            case RTLBFS_FP64_PLAIN:
                return tl ? launch_curv<double, false, true>(h, tile, src, res, s)
                          : launch_curv<double, false, false>(h, tile, src, res, s);
            case RTLBFS_FP64_DEV:
                return tl ? launch_curv<double, true, true>(h, tile, src, res, s)
                          : launch_curv<double, true, false>(h, tile, src, res, s);
            default:
                return tl ? launch_curv<float, true, true>(h, tile, src, res, s)
                          : launch_curv<float, true, false>(h, tile, src, res, s);
        }
    }
    switch (h->opts.precision) {
        case RTLBFS_FP64_PLAIN:
            return tl ? launch_step<double, false, true>(h, tile, src, res, s)
                      : launch_step<double, false, false>(h, tile, src, res, s);
        case RTLBFS_FP64_DEV:
            return tl ? launch_step<double, true, true>(h, tile, src, res, s)
                      : launch_step<double, true, false>(h, tile, src, res, s);
        default:
            return tl ? launch_step<float, true, true>(h, tile, src, res, s)
                      : launch_step<float, true, false>(h, tile, src, res, s);
    }
}

// Launches that advance n steps with the handle's launch shape: two-step
// launches while two or more steps remain, then the one-step shape of the
// same tile.  The Eq. 65 partials are taken on the last step when res.
int launches_for(const rtlbfs_t h, int64_t n) {
    const int ns = (h->mesh.dim == 2 && !h->curv) ? kTiles2[h->tile].nsub : 1;
    return (int)(n / ns + n % ns);
}

hipError_t enqueue_steps(rtlbfs_t h, int64_t n, bool res, hipStream_t s) {
    const int ns = (h->mesh.dim == 2 && !h->curv) ? kTiles2[h->tile].nsub : 1;
    while (n > 0) {
        const int tile = (h->mesh.dim == 2 && n < ns) ? kTiles2[h->tile].single : h->tile;
        const int64_t adv = n < ns ? 1 : ns;
        const bool last = n == adv;
        hipError_t e = launch_any(h, tile, h->cur, res && last, s);
        if (e != hipSuccess) return e;
        h->cur ^= 1;
        if (res && last) {
            k_finalize_sum<kPartials><<<1, 256, 0, s>>>(h->parts(), handle_blocks(h, tile), h->res_out());
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        n -= adv;
    }
    return hipSuccess;
}

hipError_t enqueue_integrals(rtlbfs_t h, double *out, hipStream_t s) {
    const Domain &d = h->dom;
    switch (h->opts.precision) {
        case RTLBFS_FP64_PLAIN:
            k_integrals<double, false><<<kRedBlocks, 256, 0, s>>>(d, (const double *)h->U(h->cur), h->parts());
            break;
        case RTLBFS_FP64_DEV:
            k_integrals<double, true><<<kRedBlocks, 256, 0, s>>>(d, (const double *)h->U(h->cur), h->parts());
            break;
        default:
            k_integrals<float, true><<<kRedBlocks, 256, 0, s>>>(d, (const float *)h->U(h->cur), h->parts());
            break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_finalize_sum<kIntParts><<<1, 256, 0, s>>>(h->parts(), kRedBlocks, out);
    return hipGetLastError();
}

hipError_t enqueue_mass_fix(rtlbfs_t h, hipStream_t s) {
    hipError_t e = enqueue_integrals(h, h->fix_out(), s);
    if (e != hipSuccess) return e;
    k_mass_fix<float><<<kRedBlocks, 256, 0, s>>>((float *)h->U(h->cur), h->lay.cells, h->fix_out(), h->m0());
    return hipGetLastError();
}

// Autotuner: time every 2D launch shape (tile size, steps per launch) on the
// live state and keep the fastest per step.  Each trial writes only the spare copy, so the state is unchanged.
// The launches of one tile are replayed from a captured graph (direct
// launches of a few-microsecond kernel would time the host's launch rate),
// and the tiles are timed in interleaved rounds, keeping each tile's best
// round, so that clock ramps and neighbours on the device bias no tile.
int autotune_tile(rtlbfs_t h) {
    if (h->curv3 || (h->mesh.dim == 3 && !h->curv)) return RTLBFS_OK;  // 3D: the tile kernel unless opts.tile
    constexpr int kLaunches = 32, kRounds = 4;
    const int nshapes = h->curv ? kNumTilesC : kNumTiles2;
    auto nsub = [&](int t) { return h->curv ? 1 : kTiles2[t].nsub; };
    hipGraphExec_t ge[kNumTiles2] = {};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = RTLBFS_OK;
    float best_ms[kNumTiles2];
    for (int t = 0; t < kNumTiles2; ++t) best_ms[t] = 1e30f;
    auto cleanup = [&]() {
        for (int t = 0; t < kNumTiles2; ++t)
            if (ge[t]) (void)hipGraphExecDestroy(ge[t]);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    for (int t = 0; t < nshapes && e == hipSuccess; ++t) {
        hipGraph_t g = nullptr;
        e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) break;
        hipError_t el = hipSuccess;
        for (int k = 0; k < kLaunches && el == hipSuccess; ++k) el = launch_any(h, t, h->cur, false, h->cap_stream);
        e = hipStreamEndCapture(h->cap_stream, &g);
        if (el != hipSuccess) e = el;
        if (e == hipSuccess) e = hipGraphInstantiate(&ge[t], g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
    }
    for (int t = 0; t < nshapes && e == hipSuccess; ++t) e = hipGraphLaunch(ge[t], h->stream);  // warm-up
    for (int r = 0; r < kRounds && e == hipSuccess; ++r) {
        for (int t = 0; t < nshapes && e == hipSuccess; ++t) {
            e = hipEventRecord(e0, h->stream);
            if (e == hipSuccess) e = hipGraphLaunch(ge[t], h->stream);
            if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess) best_ms[t] = std::min(best_ms[t], ms / (kLaunches * nsub(t)));
        }
    }
    if (e != hipSuccess) rc = hip_fail(h, e, "tile autotuning");
    cleanup();
    if (rc != RTLBFS_OK) return rc;
    int best_t = 0;
    for (int t = 0; t < nshapes; ++t) {
        h->tune_ms[t] = best_ms[t];
        if (best_ms[t] < best_ms[best_t]) best_t = t;
    }
    h->tile = best_t;
    return RTLBFS_OK;
}

// Capture `len` steps (the last with the residual) starting from copy `par`.
int capture_graph(rtlbfs_t h, int par, int len) {
    const int saved = h->cur;
    h->cur = par;
    hipGraph_t g = nullptr;
    HIP_TRY(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue_steps(h, len, true, h->cap_stream);
    hipError_t e2 = hipStreamEndCapture(h->cap_stream, &g);
    h->cur = saved;
    if (e != hipSuccess) return hip_fail(h, e, "step launch during capture");
    if (e2 != hipSuccess) return hip_fail(h, e2, "hipStreamEndCapture");
    hipError_t e3 = hipGraphInstantiate(&h->graph[par], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e3 != hipSuccess) return hip_fail(h, e3, "hipGraphInstantiate");
    return RTLBFS_OK;
}

}  // namespace

namespace {

// Workspace of a body-fitted mesh: two state copies, face records and 1/dV in
// the kernel precision, FP64 face records (a separate copy only for FP32) and
// FP64 areas, partials and the reduction slots.
struct CurvLayout {
    size_t off_U[2], off_fi, off_fj, off_ia, off_fi64, off_fj64, off_area, off_parts, off_red, bytes;
    int nparts;
};

CurvLayout make_curv_layout(int ni, int nj, int precision) {
    CurvLayout l{};
    const int64_t cells = (int64_t)ni * nj;
    const int64_t nfi = (int64_t)(ni + 1) * nj, nfj = (int64_t)ni * (nj + 1);
    const size_t es = elem_size(precision);
    const size_t copy_bytes = (size_t)4 * field_stride(cells) * es;
    size_t off = 0;
    l.off_U[0] = off;
    off += copy_bytes;
    l.off_U[1] = off;
    off += copy_bytes;
    l.off_fi = off;
    off += align256((size_t)kCurvFaceFields * nfi * es);
    l.off_fj = off;
    off += align256((size_t)kCurvFaceFields * nfj * es);
    l.off_ia = off;
    off += align256((size_t)cells * es);
    if (es == 4) {
        l.off_fi64 = off;
        off += align256((size_t)kCurvFaceFields * nfi * sizeof(double));
        l.off_fj64 = off;
        off += align256((size_t)kCurvFaceFields * nfj * sizeof(double));
    } else {
        l.off_fi64 = l.off_fi;
        l.off_fj64 = l.off_fj;
    }
    l.off_area = off;
    off += align256((size_t)cells * sizeof(double));
    rtlbfs_mesh m{};
    m.dim = 2;
    m.n[0] = ni;
    m.n[1] = nj;
    m.n[2] = 1;
    l.nparts = kRedBlocks;
    for (int t = 0; t < kNumTilesC; ++t) l.nparts = std::max(l.nparts, curv_blocks(m, t));
    l.off_parts = off;
    off += align256(sizeof(double) * (size_t)l.nparts * 8);
    l.off_red = off;
    off += align256(sizeof(double) * 32);
    l.bytes = off;
    return l;
}

// Workspace of a 3D body-fitted mesh: two state copies, face records of the
// three axes and 1/dV in the kernel precision (FP64 record copies only for
// FP32), FP64 volumes, the per-step scratch (primitives, gradients, face
// fluxes), partials and reduction slots.
struct Curv3Layout {
    size_t off_U[2], off_rec[3], off_rec64[3], off_iv, off_vol, off_prim, off_grad, off_flux, off_parts, off_red,
        bytes;
    int nparts;
    int64_t nf[3];
};

Curv3Layout make_curv3_layout(const int n[3], int precision) {
    Curv3Layout l{};
    const int64_t cells = (int64_t)n[0] * n[1] * n[2];
    const size_t es = elem_size(precision);
    size_t off = 0;
    for (int k = 0; k < 2; ++k) {
        l.off_U[k] = off;
        off += (size_t)5 * field_stride(cells) * es;
    }
    int64_t nfaces = 0;
    for (int a = 0; a < 3; ++a) {
        l.nf[a] = (int64_t)(n[0] + (a == 0)) * (n[1] + (a == 1)) * (n[2] + (a == 2));
        nfaces += l.nf[a];
        l.off_rec[a] = off;
        off += align256((size_t)kC3Fields * l.nf[a] * es);
    }
    for (int a = 0; a < 3; ++a) {
        if (es == 4) {
            l.off_rec64[a] = off;
            off += align256((size_t)kC3Fields * l.nf[a] * sizeof(double));
        } else {
            l.off_rec64[a] = l.off_rec[a];
        }
    }
    l.off_iv = off;
    off += align256((size_t)cells * es);
    l.off_vol = off;
    off += align256((size_t)cells * sizeof(double));
    l.off_prim = off;
    off += align256((size_t)5 * cells * es);
    l.off_grad = off;
    off += align256((size_t)15 * cells * es);
    l.off_flux = off;
    off += align256((size_t)5 * nfaces * es);
    // one row per update block of either path
    l.nparts = std::max<int>(kRedBlocks, std::max<int>((int)((cells + kC3Threads - 1) / kC3Threads), c3_layer_blocks(n)));
    l.off_parts = off;
    off += align256(sizeof(double) * (size_t)l.nparts * 8);
    l.off_red = off;
    off += align256(sizeof(double) * 32);
    l.bytes = off;
    return l;
}

template <typename R>
void put(char *dst, const std::vector<double> &src) {
    R *p = (R *)dst;
    for (size_t k = 0; k < src.size(); ++k) p[k] = (R)src[k];
}

}  // namespace

// ------------------------------------------------------------------- C ABI --

extern "C" {

const char *rtlbfs_strerror(int code) {
    switch (code) {
        case RTLBFS_OK: return "ok";
        case RTLBFS_EINVAL: return "invalid argument";
        case RTLBFS_ENOMEM: return "out of device memory or workspace too small";
        case RTLBFS_EDEVICE: return "HIP runtime error";
        case RTLBFS_EDIVERGED: return "solution diverged (NaN/Inf or local Mach above opts.max_mach)";
        case RTLBFS_EUNSUPPORTED: return "unsupported request";
        case RTLBFS_ESTATE: return "invalid call order";
        default: return "unknown status";
    }
}

const char *rtlbfs_last_error(rtlbfs_t h) { return h ? h->err.c_str() : g_create_err.c_str(); }

int rtlbfs_opts_init(rtlbfs_opts *o) {
    if (!o) return RTLBFS_EINVAL;
    std::memset(o, 0, sizeof(*o));
    o->precision = RTLBFS_FP64_PLAIN;
    o->residual_every = 100;
    o->mass_fix_every = 1000;
    o->graph_steps = 0;
    return RTLBFS_OK;
}

int rtlbfs_mesh_nodes(int n, double stretch, double *host_x, double *L) { return mesh_nodes(n, stretch, host_x, L); }

size_t rtlbfs_workspace_bytes(const rtlbfs_mesh *mesh, const rtlbfs_opts *opts) {
    if (!mesh || (mesh->dim != 2 && mesh->dim != 3)) return 0;
    for (int a = 0; a < mesh->dim; ++a)
        if (mesh->n[a] < 4 || mesh->n[a] > (1 << 20)) return 0;
    if (!step_launches_fit(*mesh)) return 0;
    rtlbfs_opts o;
    if (opts) o = *opts;
    else rtlbfs_opts_init(&o);
    return make_layout(*mesh, o.precision).bytes;
}

int rtlbfs_create(const rtlbfs_mesh *mesh, double Ra, double Pr, double Ma, const rtlbfs_bc *bc,
                  const rtlbfs_opts *opts, void *hip_stream, void *workspace, size_t ws_bytes, rtlbfs_t *out) {
    if (!out) return RTLBFS_EINVAL;
    *out = nullptr;
    rtlbfs_opts o;
    if (opts) o = *opts;
    else rtlbfs_opts_init(&o);
    std::string why;
    g_create_err.clear();
    Problem P;
    int rc = setup_problem(mesh, bc, o, Ra, Pr, Ma, P, why);
    if (rc != RTLBFS_OK) {
        g_create_err = why;
        return rc;
    }
    if (!step_launches_fit(P.mesh)) {
        g_create_err = "mesh too large: a step launch would exceed 2^32 - 1 work-items";
        return RTLBFS_EINVAL;
    }
    rtlbfs_t h = new (std::nothrow) rtlbfs_handle();
    if (!h) return RTLBFS_ENOMEM;
    h->mesh = P.mesh;
    h->bc = *bc;
    if (o.residual_every <= 0) o.residual_every = 100;
    if (o.mass_fix_every == 0) o.mass_fix_every = 1000;
    h->opts = o;
    h->opts.dtl = P.dtl;
    h->opts.dt = P.dt;
    h->opts.nu = P.nu;
    h->opts.chi = P.chi;
    h->opts.beta_g = P.bg;
    h->stream = (hipStream_t)hip_stream;
    h->lay = make_layout(h->mesh, o.precision);
    const int D = P.D;
    for (int a = 0; a < 3; ++a) h->length[a] = P.length[a];
    h->L = P.L;
    const std::vector<double> &widths = P.widths;
    Domain &d = h->dom;
    fill_domain(P, o.precision, o.buoyancy_update_only ? 0 : 1, o.round_nearest, o.max_mach, d);

    // Workspace.
    if (workspace) {
        if (ws_bytes < h->lay.bytes) {
            delete h;
            g_create_err = "workspace smaller than rtlbfs_workspace_bytes()";
            return RTLBFS_ENOMEM;
        }
        h->ws = (char *)workspace;
    } else {
        hipError_t e = hipMalloc((void **)&h->ws, h->lay.bytes);
        if (e != hipSuccess) {
            delete h;
            g_create_err = "hipMalloc of the workspace failed";
            return RTLBFS_ENOMEM;
        }
        h->own_ws = true;
    }
    for (int a = 0; a < D; ++a) d.w[a] = nullptr;
    {
        double *wdev = (double *)(h->ws + h->lay.off_w);
        size_t off = 0;
        for (int a = 0; a < D; ++a) {
            d.w[a] = wdev + off;
            off += h->mesh.n[a];
        }
        std::vector<char> geo;
        size_t goff[3] = {0, 0, 0};
        pack_geometry(P, o.precision, geo, goff);
        for (int a = 0; a < D; ++a) d.geo[a] = h->ws + h->lay.off_geo + goff[a];
        hipError_t e = hipMemcpy(wdev, widths.data(), widths.size() * sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(h->ws + h->lay.off_geo, geo.data(), geo.size(), hipMemcpyHostToDevice);
        const uint32_t zero2[2] = {0u, 0u};
        if (e == hipSuccess) e = hipMemcpy(h->ctr(), zero2, sizeof(zero2), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            int r2 = hip_fail(h, e, "upload geometry");
            rtlbfs_destroy(h);
            return r2;
        }
    }
    {
        hipError_t e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipHostMalloc((void **)&h->host_buf, 64 * sizeof(double), hipHostMallocDefault);
        if (e != hipSuccess) {
            int r2 = hip_fail(h, e, "capture stream / pinned buffer");
            rtlbfs_destroy(h);
            return r2;
        }
    }

    // Seeded initial state: rho = 1, u = 0, T - T0 from the profile and noise.
    const int64_t N = h->lay.cells;
    std::vector<double> rho((size_t)N, 1.0), u((size_t)N * D, 0.0), T;
    initial_Tdev(P, o, T);
    rc = upload_prims(h, rho.data(), u.data(), T.data());
    if (rc != RTLBFS_OK) {
        rtlbfs_destroy(h);
        return rc;
    }
    // Reference mass for the drift correction.
    {
        hipError_t e = enqueue_integrals(h, h->int_out(), h->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(h->m0(), h->int_out(), sizeof(double), hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) {
            int r2 = hip_fail(h, e, "initial integrals");
            rtlbfs_destroy(h);
            return r2;
        }
    }
    // Kernel tile: fixed by opts.tile (1-based), or chosen by the autotuner.
    if (o.tile > 0) {
        if (o.tile > (D == 2 ? kNumTiles2 : kNumTiles3)) {
            rtlbfs_destroy(h);
            g_create_err = "opts.tile out of range";
            return RTLBFS_EINVAL;
        }
        h->tile = o.tile - 1;
    } else if (D == 2) {
        rc = autotune_tile(h);
        if (rc != RTLBFS_OK) {
            rtlbfs_destroy(h);
            return rc;
        }
    }
    *out = h;
    return RTLBFS_OK;
}

int rtlbfs_step(rtlbfs_t h, int64_t n) {
    if (!h) return RTLBFS_EINVAL;
    if (n < 0) return fail(h, RTLBFS_EINVAL, "negative step count");
    const int C = h->opts.residual_every;
    const bool graphs = h->opts.graph_steps >= 0;
    while (n > 0) {
        const int64_t chunk = std::min<int64_t>(n, C);
        if (graphs && chunk == C) {
            if (!h->graph[h->cur]) {
                int rc = capture_graph(h, h->cur, C);
                if (rc != RTLBFS_OK) return rc;
            }
            HIP_TRY(h, hipGraphLaunch(h->graph[h->cur], h->stream));
            if (launches_for(h, C) & 1) h->cur ^= 1;
        } else {
            hipError_t e = enqueue_steps(h, chunk, true, h->stream);
            if (e != hipSuccess) return hip_fail(h, e, "step launch");
        }
        n -= chunk;
        h->steps += chunk;
        h->since_fix += chunk;
        h->res_valid = true;
        if (h->opts.precision == RTLBFS_FP32_DEV && h->opts.mass_fix_every > 0 &&
            h->since_fix >= h->opts.mass_fix_every) {
            hipError_t e = enqueue_mass_fix(h, h->stream);
            if (e != hipSuccess) return hip_fail(h, e, "mass fix");
            h->since_fix = 0;
        }
    }
    return RTLBFS_OK;
}

int rtlbfs_sync(rtlbfs_t h) {
    if (!h) return RTLBFS_EINVAL;
    HIP_TRY(h, hipMemcpyAsync(h->host_buf, h->res_out(), kPartials * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    if (h->res_valid && h->host_buf[4] != 0.0) return fail(h, RTLBFS_EDIVERGED, "NaN/Inf or local Mach above opts.max_mach detected");
    return RTLBFS_OK;
}

int rtlbfs_residual(rtlbfs_t h, double *res_u, double *res_T) {
    if (!h || !res_u || !res_T) return RTLBFS_EINVAL;
    if (!h->res_valid) return fail(h, RTLBFS_ESTATE, "no residual step yet");
    int rc = rtlbfs_sync(h);
    const double *r = h->host_buf;
    *res_u = r[1] > 0.0 ? r[0] / r[1] : 0.0;
    *res_T = r[3] != 0.0 ? r[2] / r[3] : 0.0;
    return rc;
}

int rtlbfs_nusselt(rtlbfs_t h, rtlbfs_nu *out) {
    if (!h || !out) return RTLBFS_EINVAL;
    if (h->curv || h->curv3) return fail(h, RTLBFS_EUNSUPPORTED, "body-fitted mesh: use rtlbfs_wall_heat");
    const int ha = heat_axis(h->mesh, h->bc);
    if (ha < 0) return fail(h, RTLBFS_EINVAL, "no pair of isothermal walls");
    const double Tlo = h->bc.Tdev[2 * ha], Thi = h->bc.Tdev[2 * ha + 1];
    const double dTw = std::fabs(Thi - Tlo);
    if (dTw == 0.0) return fail(h, RTLBFS_EINVAL, "isothermal walls at equal temperature");
    const int hot_hi = Thi > Tlo;
    const Domain &d = h->dom;
    double *parts = h->parts();
    switch (h->opts.precision) {
        case RTLBFS_FP64_PLAIN:
            k_nusselt<double, false><<<kRedBlocks, 256, 0, h->stream>>>(d, (const double *)h->U(h->cur), ha, hot_hi,
                                                                        h->length[ha], dTw, parts);
            break;
        case RTLBFS_FP64_DEV:
            k_nusselt<double, true><<<kRedBlocks, 256, 0, h->stream>>>(d, (const double *)h->U(h->cur), ha, hot_hi,
                                                                       h->length[ha], dTw, parts);
            break;
        default:
            k_nusselt<float, true><<<kRedBlocks, 256, 0, h->stream>>>(d, (const float *)h->U(h->cur), ha, hot_hi,
                                                                      h->length[ha], dTw, parts);
            break;
    }
    HIP_TRY(h, hipGetLastError());
    k_nusselt_finalize<0><<<1, 256, 0, h->stream>>>(parts, kRedBlocks, h->nu_out());
    HIP_TRY(h, hipGetLastError());
    HIP_TRY(h, hipMemcpyAsync(h->host_buf + 8, h->nu_out(), 8 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    const double *r = h->host_buf + 8;
    out->hot_avg = r[0] / r[1];
    out->cold_avg = r[2] / r[3];
    out->volume = h->length[ha] / (d.chi * dTw) * r[4] / r[5];
    out->hot_max = r[6];
    out->cold_max = r[7];
    return RTLBFS_OK;
}

int rtlbfs_integrals(rtlbfs_t h, double out[3]) {
    if (!h || !out) return RTLBFS_EINVAL;
    HIP_TRY(h, enqueue_integrals(h, h->int_out(), h->stream));
    HIP_TRY(h, hipMemcpyAsync(h->host_buf + 16, h->int_out(), 3 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    for (int k = 0; k < 3; ++k) out[k] = h->host_buf[16 + k];
    return RTLBFS_OK;
}

int rtlbfs_get_stored(rtlbfs_t h, int field, double *host_out, size_t count) {
    if (!h || !host_out) return RTLBFS_EINVAL;
    if (field < 0 || field > h->mesh.dim + 1) return fail(h, RTLBFS_EINVAL, "field out of range");
    if (count < (size_t)h->lay.cells) return fail(h, RTLBFS_EINVAL, "count smaller than the cell count");
    std::vector<double> f;
    int rc = read_stored(h, field, f);
    if (rc != RTLBFS_OK) return rc;
    std::memcpy(host_out, f.data(), f.size() * sizeof(double));
    return RTLBFS_OK;
}

int rtlbfs_get_field(rtlbfs_t h, int field, double *host_out, size_t count) {
    if (!h || !host_out) return RTLBFS_EINVAL;
    const int D = h->mesh.dim;
    if (field < 0 || field > D + 1) return fail(h, RTLBFS_EINVAL, "field out of range");
    if (count < (size_t)h->lay.cells) return fail(h, RTLBFS_EINVAL, "count smaller than the cell count");
    const bool dev = h->opts.precision != RTLBFS_FP64_PLAIN;
    std::vector<double> r, f;
    int rc = read_stored(h, 0, r);
    if (rc != RTLBFS_OK) return rc;
    if (field > 0 && (rc = read_stored(h, field, f)) != RTLBFS_OK) return rc;
    for (int64_t c = 0; c < h->lay.cells; ++c) {
        const double rho = dev ? 1.0 + r[c] : r[c];
        if (field == 0) host_out[c] = rho;
        else if (field <= D) host_out[c] = f[c] / rho;
        else host_out[c] = f[c] / rho + (dev ? kT0 : 0.0);
    }
    return RTLBFS_OK;
}

int rtlbfs_set_state(rtlbfs_t h, const double *rho, const double *u, const double *T, size_t cells) {
    if (!h || !rho || !u || !T) return RTLBFS_EINVAL;
    if (cells != (size_t)h->lay.cells) return fail(h, RTLBFS_EINVAL, "cell count mismatch");
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    std::vector<double> Tdev(cells);
    for (size_t c = 0; c < cells; ++c) Tdev[c] = T[c] - kT0;
    int rc = upload_prims(h, rho, u, Tdev.data());
    if (rc != RTLBFS_OK) return rc;
    HIP_TRY(h, enqueue_integrals(h, h->int_out(), h->stream));
    HIP_TRY(h, hipMemcpyAsync(h->m0(), h->int_out(), sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    h->since_fix = 0;
    return RTLBFS_OK;
}

int rtlbfs_get_checkpoint(rtlbfs_t h, rtlbfs_checkpoint *out) {
    if (!h || !out) return RTLBFS_EINVAL;
    double m0 = 0.0;
    HIP_TRY(h, hipMemcpyAsync(&m0, h->m0(), sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    out->steps = h->steps;
    out->since_fix = h->since_fix;
    out->mass0 = m0;
    return RTLBFS_OK;
}

int rtlbfs_restore(rtlbfs_t h, const double *host_stored, size_t count, const rtlbfs_checkpoint *ck) {
    if (!h || !host_stored || !ck) return RTLBFS_EINVAL;
    const int64_t N = h->lay.cells;
    const int nf = h->mesh.dim + 2;
    if (count < (size_t)nf * (size_t)N) return fail(h, RTLBFS_EINVAL, "count smaller than (dim + 2) * cells");
    if (ck->steps < 0 || ck->since_fix < 0) return fail(h, RTLBFS_EINVAL, "negative step count");
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    const size_t field_bytes = (size_t)h->dom.fstride * elem_size(h->opts.precision);
    std::vector<double> f((size_t)N);
    std::vector<char> buf;
    for (int k = 0; k < nf; ++k) {
        std::memcpy(f.data(), host_stored + (size_t)k * N, sizeof(double) * (size_t)N);
        if (h->opts.precision == RTLBFS_FP32_DEV) to_storage<float>(f, buf);
        else to_storage<double>(f, buf);
        HIP_TRY(h, hipMemcpyAsync((char *)h->U(h->cur) + k * field_bytes, buf.data(), buf.size(),
                                  hipMemcpyHostToDevice, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
    }
    // the step counter of the copy the next launch reads (the stochastic-rounding key)
    const uint32_t key = (uint32_t)(uint64_t)ck->steps;
    const double m0 = ck->mass0;
    HIP_TRY(h, hipMemcpyAsync(h->ctr() + h->cur, &key, sizeof(key), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipMemcpyAsync(h->m0(), &m0, sizeof(double), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    h->steps = ck->steps;
    h->since_fix = ck->since_fix;
    h->res_valid = false;
    return RTLBFS_OK;
}

int rtlbfs_get_info(rtlbfs_t h, rtlbfs_info *out) {
    if (!h || !out) return RTLBFS_EINVAL;
    std::memset(out, 0, sizeof(*out));
    out->cells = h->lay.cells;
    out->steps = h->steps;
    out->L = h->L;
    out->nu = h->dom.nu;
    out->chi = h->dom.chi;
    out->beta_g = h->dom.bg;
    out->tau_f = h->dom.tau_f;
    out->tau_g = h->dom.tau_g;
    out->dtl = h->dom.dtl;
    out->dt = h->dom.dt;
    for (int a = 0; a < 3; ++a) out->length[a] = a < h->mesh.dim ? h->length[a] : 1.0;
    out->precision = h->opts.precision;
    for (int t = 0; t < kNumTiles2; ++t) out->tune_ms[t] = h->tune_ms[t];
    if (h->curv3 && h->c3_layer) {
        out->tile_x = kC3LayerTX;  // fused kernel: one TX x 1 x TZ tile per block
        out->tile_y = 1;
        out->tile_z = kC3LayerTZ;
        out->steps_per_launch = 1;
    } else if (h->curv3) {
        out->tile_x = kC3Threads;  // one thread per cell or face, kC3Threads per block
        out->tile_y = 1;
        out->tile_z = 1;
        out->steps_per_launch = 1;
    } else if (h->curv) {
        out->tile_x = kTilesC[h->tile].tx;
        out->tile_y = kTilesC[h->tile].ty;
        out->tile_z = 1;
        out->steps_per_launch = 1;
    } else if (h->mesh.dim == 2) {
        out->tile_x = kTiles2[h->tile].tx;
        out->tile_y = kTiles2[h->tile].ty;
        out->steps_per_launch = kTiles2[h->tile].nsub;
        out->tile_z = 1;
    } else {
        out->tile_x = kTiles3[h->tile].tx;  // columns: tile_z is the segment length
        out->tile_y = kTiles3[h->tile].ty;
        out->tile_z = kTiles3[h->tile].sz;
        out->steps_per_launch = 1;
    }
    return RTLBFS_OK;
}

size_t rtlbfs_curv_workspace_bytes(const rtlbfs_curv_mesh *mesh, const rtlbfs_opts *opts) {
    if (!mesh || mesh->n[0] < 4 || mesh->n[1] < 4 || mesh->n[0] > (1 << 20) || mesh->n[1] > (1 << 20)) return 0;
    if (!curv_launches_fit(mesh->n[0], mesh->n[1])) return 0;
    rtlbfs_opts o;
    if (opts) o = *opts;
    else rtlbfs_opts_init(&o);
    return make_curv_layout(mesh->n[0], mesh->n[1], o.precision).bytes;
}

int rtlbfs_curv_create(const rtlbfs_curv_mesh *mesh, double nu, double chi, double beta_g, const rtlbfs_curv_bc *bc,
                       const rtlbfs_opts *opts, void *hip_stream, void *workspace, size_t ws_bytes, rtlbfs_t *out) {
    if (!out) return RTLBFS_EINVAL;
    *out = nullptr;
    g_create_err.clear();
    rtlbfs_opts o;
    if (opts) o = *opts;
    else rtlbfs_opts_init(&o);
    auto reject = [](const char *why) {
        g_create_err = why;
        return RTLBFS_EINVAL;
    };
    if (o.precision != RTLBFS_FP64_PLAIN && o.precision != RTLBFS_FP32_DEV && o.precision != RTLBFS_FP64_DEV)
        return reject("unknown precision");
    if (o.method != RTLBFS_METHOD_RTLBFS && o.method != RTLBFS_METHOD_TLBFS) return reject("unknown opts.method");
    if (o.tile < 0 || o.tile > kNumTilesC) return reject("opts.tile out of range for a body-fitted 2D mesh (0..4)");
    if (!(nu > 0.0) || !(chi > 0.0) || !(beta_g >= 0.0)) return reject("nu, chi > 0, beta_g >= 0");
    if (!(o.dtl >= 0.0) || !(o.dt >= 0.0)) return reject("dtl and dt must be >= 0");
    if (!(o.max_mach >= 0.0) || o.max_mach > 10.0) return reject("opts.max_mach out of range");
    CurvProblem cp;
    std::string why;
    int rc = curv_setup(mesh, bc, cp, why);
    if (rc != RTLBFS_OK) {
        g_create_err = why;
        return rc;
    }
    if (!curv_launches_fit(mesh->n[0], mesh->n[1])) {
        g_create_err = "mesh too large: a step launch would exceed 2^32 - 1 work-items";
        return RTLBFS_EINVAL;
    }
    Problem P;
    P.mesh.dim = 2;
    P.mesh.n[0] = cp.ni;
    P.mesh.n[1] = cp.nj;
    P.mesh.n[2] = 1;
    for (int s = 0; s < 6; ++s) {
        P.bc.kind[s] = s < 4 ? bc->kind[s] : RTLBFS_PERIODIC;
        P.bc.Tdev[s] = s < 4 ? bc->Tw[s] - kT0 : 0.0;
    }
    P.bc.gravity_axis = -1;  // buoyancy along bc->up, applied by the body-fitted kernel
    P.D = 2;
    P.cells = cp.cells;
    P.nu = nu;
    P.chi = chi;
    P.bg = beta_g;
    P.dtl = o.dtl > 0.0 ? o.dtl : 1.0;
    P.dt = o.dt > 0.0 ? o.dt : std::min(0.5, 0.15 / std::max(nu, chi));

    rtlbfs_t h = new (std::nothrow) rtlbfs_handle();
    if (!h) return RTLBFS_ENOMEM;
    h->curv = true;
    h->mesh = P.mesh;
    h->bc = P.bc;
    if (o.residual_every <= 0) o.residual_every = 100;
    if (o.mass_fix_every == 0) o.mass_fix_every = 1000;
    h->opts = o;
    h->opts.dtl = P.dtl;
    h->opts.dt = P.dt;
    h->opts.nu = nu;
    h->opts.chi = chi;
    h->opts.beta_g = beta_g;
    h->opts.phys_given = 1;
    h->stream = (hipStream_t)hip_stream;
    const CurvLayout cl = make_curv_layout(cp.ni, cp.nj, o.precision);
    h->lay = Layout{};
    h->lay.off_U[0] = cl.off_U[0];
    h->lay.off_U[1] = cl.off_U[1];
    h->lay.off_parts = cl.off_parts;
    h->lay.off_red = cl.off_red;
    h->lay.bytes = cl.bytes;
    h->lay.cells = cp.cells;
    h->lay.nparts = cl.nparts;
    h->L = 0.0;
    for (int s = 0; s < 4; ++s) {
        h->ckind[s] = bc->kind[s];
        h->cTw[s] = bc->Tw[s];
    }
    h->nfi = cp.nfi;
    h->nfj = cp.nfj;
    h->ccx = cp.cx;
    h->ccy = cp.cy;
    h->carea = cp.area;
    Domain &d = h->dom;
    fill_domain(P, o.precision, o.buoyancy_update_only ? 0 : 1, o.round_nearest, o.max_mach, d);
    const bool dev = o.precision != RTLBFS_FP64_PLAIN;
    d.phd.Tref_s = dev ? bc->T_ref - kT0 : bc->T_ref;
    d.phf.Tref_s = (float)d.phd.Tref_s;

    if (workspace) {
        if (ws_bytes < cl.bytes) {
            delete h;
            g_create_err = "workspace smaller than rtlbfs_curv_workspace_bytes()";
            return RTLBFS_ENOMEM;
        }
        h->ws = (char *)workspace;
    } else {
        hipError_t e = hipMalloc((void **)&h->ws, cl.bytes);
        if (e != hipSuccess) {
            delete h;
            g_create_err = "hipMalloc of the workspace failed";
            return RTLBFS_ENOMEM;
        }
        h->own_ws = true;
    }
    {
        std::vector<double> ia(cp.cells);
        for (int64_t c = 0; c < cp.cells; ++c) ia[c] = 1.0 / cp.area[c];
        std::vector<char> bfi, bfj, bia;
        const size_t es = elem_size(o.precision);
        bfi.resize(cp.fi.size() * es);
        bfj.resize(cp.fj.size() * es);
        bia.resize(ia.size() * es);
        if (es == 4) {
            put<float>(bfi.data(), cp.fi);
            put<float>(bfj.data(), cp.fj);
            put<float>(bia.data(), ia);
        } else {
            put<double>(bfi.data(), cp.fi);
            put<double>(bfj.data(), cp.fj);
            put<double>(bia.data(), ia);
        }
        hipError_t e = hipMemcpy(h->ws + cl.off_fi, bfi.data(), bfi.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(h->ws + cl.off_fj, bfj.data(), bfj.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(h->ws + cl.off_ia, bia.data(), bia.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess && es == 4)
            e = hipMemcpy(h->ws + cl.off_fi64, cp.fi.data(), cp.fi.size() * sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess && es == 4)
            e = hipMemcpy(h->ws + cl.off_fj64, cp.fj.data(), cp.fj.size() * sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(h->ws + cl.off_area, cp.area.data(), cp.area.size() * sizeof(double), hipMemcpyHostToDevice);
        const uint32_t zero2[2] = {0u, 0u};
        if (e == hipSuccess) e = hipMemcpy(h->ctr(), zero2, sizeof(zero2), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipHostMalloc((void **)&h->host_buf, 64 * sizeof(double), hipHostMallocDefault);
        if (e != hipSuccess) {
            int r2 = hip_fail(h, e, "upload geometry / capture stream");
            g_create_err = h->err;
            rtlbfs_destroy(h);
            return r2;
        }
    }
    d.vol = (const double *)(h->ws + cl.off_area);
    for (int a = 0; a < 3; ++a) {
        d.w[a] = nullptr;
        d.geo[a] = nullptr;
    }
    h->fi64 = (const double *)(h->ws + cl.off_fi64);
    h->fj64 = (const double *)(h->ws + cl.off_fj64);
    CurvGeo &g = h->cg;
    g.fi = h->ws + cl.off_fi;
    g.fj = h->ws + cl.off_fj;
    g.inv_area = h->ws + cl.off_ia;
    g.sfi = cp.nfi;
    g.sfj = cp.nfj;
    for (int a = 0; a < 2; ++a) {
        g.up[a] = bc->up[a];
        g.uinf[a] = bc->u_inf[a];
        g.upf[a] = (float)bc->up[a];
        g.uinff[a] = (float)bc->u_inf[a];
    }
    g.Tinf_s = dev ? bc->T_inf - kT0 : bc->T_inf;
    g.Tinff_s = (float)g.Tinf_s;

    // initial state: the far-field state, seeded noise on T
    const int64_t N = cp.cells;
    std::vector<double> rho((size_t)N, 1.0), u((size_t)N * 2), T((size_t)N);
    for (int64_t c = 0; c < N; ++c) {
        u[c] = bc->u_inf[0];
        u[N + c] = bc->u_inf[1];
        T[c] = bc->T_inf - kT0 + o.noise_amp * splitmix_uniform(o.seed, (uint64_t)c);
    }
    rc = upload_prims(h, rho.data(), u.data(), T.data());
    if (rc == RTLBFS_OK) {
        hipError_t e = enqueue_integrals(h, h->int_out(), h->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(h->m0(), h->int_out(), sizeof(double), hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) rc = hip_fail(h, e, "initial integrals");
    }
    if (rc == RTLBFS_OK) {
        if (o.tile > 0) h->tile = o.tile - 1;
        else rc = autotune_tile(h);
    }
    if (rc != RTLBFS_OK) {
        g_create_err = h->err;
        rtlbfs_destroy(h);
        return rc;
    }
    *out = h;
    return RTLBFS_OK;
}

int rtlbfs_wall_heat(rtlbfs_t h, int side, double out[2]) {
    if (!h || !out) return RTLBFS_EINVAL;
    if (h->curv3) {
        if (side < 0 || side > 5 || h->ckind[side] != RTLBFS_WALL_ISOTHERMAL)
            return fail(h, RTLBFS_EINVAL, "side is not an isothermal wall");
        double *dst = h->red() + 5;
        const int a = side / 2;
        switch (h->opts.precision) {
            case RTLBFS_FP64_PLAIN:
                k_c3_wall_heat<double, false><<<1, 256, 0, h->stream>>>(h->dom, h->c3rec64[a], h->c3.sf[a],
                                                                        (const double *)h->U(h->cur), side, h->cTw[side], dst);
                break;
            case RTLBFS_FP64_DEV:
                k_c3_wall_heat<double, true><<<1, 256, 0, h->stream>>>(h->dom, h->c3rec64[a], h->c3.sf[a],
                                                                       (const double *)h->U(h->cur), side, h->cTw[side], dst);
                break;
            default:
                k_c3_wall_heat<float, true><<<1, 256, 0, h->stream>>>(h->dom, h->c3rec64[a], h->c3.sf[a],
                                                                      (const float *)h->U(h->cur), side, h->cTw[side], dst);
                break;
        }
        HIP_TRY(h, hipGetLastError());
        HIP_TRY(h, hipMemcpyAsync(h->host_buf + 40, dst, 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        out[0] = h->host_buf[40];
        out[1] = h->host_buf[41];
        return RTLBFS_OK;
    }
    if (!h->curv) return fail(h, RTLBFS_EUNSUPPORTED, "rtlbfs_wall_heat needs a body-fitted mesh");
    if (side < 0 || side > 3 || h->ckind[side] != RTLBFS_WALL_ISOTHERMAL)
        return fail(h, RTLBFS_EINVAL, "side is not an isothermal wall");
    double *dst = h->red() + 5;
    switch (h->opts.precision) {
        case RTLBFS_FP64_PLAIN:
            k_curv_wall_heat<double, false><<<1, 256, 0, h->stream>>>(h->dom, h->fi64, h->fj64, h->nfi, h->nfj,
                                                                      (const double *)h->U(h->cur), side, h->cTw[side], dst);
            break;
        case RTLBFS_FP64_DEV:
            k_curv_wall_heat<double, true><<<1, 256, 0, h->stream>>>(h->dom, h->fi64, h->fj64, h->nfi, h->nfj,
                                                                     (const double *)h->U(h->cur), side, h->cTw[side], dst);
            break;
        default:
            k_curv_wall_heat<float, true><<<1, 256, 0, h->stream>>>(h->dom, h->fi64, h->fj64, h->nfi, h->nfj,
                                                                    (const float *)h->U(h->cur), side, h->cTw[side], dst);
            break;
    }
    HIP_TRY(h, hipGetLastError());
    HIP_TRY(h, hipMemcpyAsync(h->host_buf + 40, dst, 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    out[0] = h->host_buf[40];
    out[1] = h->host_buf[41];
    return RTLBFS_OK;
}

int rtlbfs_curv_cells(rtlbfs_t h, double *cx, double *cy, double *area, size_t count) {
    if (!h) return RTLBFS_EINVAL;
    if (!h->curv) return fail(h, RTLBFS_EUNSUPPORTED, "not a body-fitted mesh");
    if (count < h->ccx.size()) return fail(h, RTLBFS_EINVAL, "count smaller than the cell count");
    if (cx) std::memcpy(cx, h->ccx.data(), h->ccx.size() * sizeof(double));
    if (cy) std::memcpy(cy, h->ccy.data(), h->ccy.size() * sizeof(double));
    if (area) std::memcpy(area, h->carea.data(), h->carea.size() * sizeof(double));
    return RTLBFS_OK;
}

size_t rtlbfs_curv3_workspace_bytes(const rtlbfs_curv3_mesh *mesh, const rtlbfs_opts *opts) {
    if (!mesh) return 0;
    for (int a = 0; a < 3; ++a)
        if (mesh->n[a] < 1 || mesh->n[a] > (1 << 16)) return 0;
    if ((int64_t)mesh->n[0] * mesh->n[1] * mesh->n[2] > (int64_t)1 << 28) return 0;
    rtlbfs_opts o;
    if (opts) o = *opts;
    else rtlbfs_opts_init(&o);
    return make_curv3_layout(mesh->n, o.precision).bytes;
}

int rtlbfs_curv3_create(const rtlbfs_curv3_mesh *mesh, double nu, double chi, double beta_g, const rtlbfs_curv3_bc *bc,
                        const rtlbfs_opts *opts, void *hip_stream, void *workspace, size_t ws_bytes, rtlbfs_t *out) {
    if (!out) return RTLBFS_EINVAL;
    *out = nullptr;
    g_create_err.clear();
    rtlbfs_opts o;
    if (opts) o = *opts;
    else rtlbfs_opts_init(&o);
    auto reject = [](const char *why) {
        g_create_err = why;
        return RTLBFS_EINVAL;
    };
    if (o.precision != RTLBFS_FP64_PLAIN && o.precision != RTLBFS_FP32_DEV && o.precision != RTLBFS_FP64_DEV)
        return reject("unknown precision");
    if (o.method != RTLBFS_METHOD_RTLBFS && o.method != RTLBFS_METHOD_TLBFS) return reject("unknown opts.method");
    if (o.tile < 0 || o.tile > 2) return reject("opts.tile out of range for a 3D body-fitted mesh (0..2)");
    if (!(nu > 0.0) || !(chi > 0.0) || !(beta_g >= 0.0)) return reject("nu, chi > 0, beta_g >= 0");
    if (!(o.dtl >= 0.0) || !(o.dt >= 0.0)) return reject("dtl and dt must be >= 0");
    if (!(o.max_mach >= 0.0) || o.max_mach > 10.0) return reject("opts.max_mach out of range");
    Curv3Problem cp;
    std::string why;
    int rc = curv3_setup(mesh, bc, cp, why);
    if (rc != RTLBFS_OK) {
        g_create_err = why;
        return rc;
    }
    const bool layer = c3_is_layer(cp.n, bc->kind);
    if (o.tile == 2 && !layer) {
        g_create_err = "opts.tile 2 (fused kernel) needs a single periodic cell layer along j and walls along i and k";
        return RTLBFS_EINVAL;
    }
    Problem P;
    P.mesh.dim = 3;
    for (int a = 0; a < 3; ++a) P.mesh.n[a] = cp.n[a];
    for (int s = 0; s < 6; ++s) {
        P.bc.kind[s] = bc->kind[s];
        P.bc.Tdev[s] = bc->Tw[s] - kT0;
    }
    P.bc.gravity_axis = -1;  // buoyancy along bc->up, applied by the body-fitted kernels
    P.D = 3;
    P.cells = cp.cells;
    P.nu = nu;
    P.chi = chi;
    P.bg = beta_g;
    P.dtl = o.dtl > 0.0 ? o.dtl : 1.0;
    P.dt = o.dt > 0.0 ? o.dt : std::min(0.5, 0.15 / std::max(nu, chi));

    rtlbfs_t h = new (std::nothrow) rtlbfs_handle();
    if (!h) return RTLBFS_ENOMEM;
    h->curv3 = true;
    h->c3_layer = o.tile == 2 || (o.tile == 0 && layer);
    h->mesh = P.mesh;
    h->bc = P.bc;
    if (o.residual_every <= 0) o.residual_every = 100;
    if (o.mass_fix_every == 0) o.mass_fix_every = 1000;
    h->opts = o;
    h->opts.dtl = P.dtl;
    h->opts.dt = P.dt;
    h->opts.nu = nu;
    h->opts.chi = chi;
    h->opts.beta_g = beta_g;
    h->opts.phys_given = 1;
    h->stream = (hipStream_t)hip_stream;
    const Curv3Layout cl = make_curv3_layout(cp.n, o.precision);
    h->lay = Layout{};
    h->lay.off_U[0] = cl.off_U[0];
    h->lay.off_U[1] = cl.off_U[1];
    h->lay.off_parts = cl.off_parts;
    h->lay.off_red = cl.off_red;
    h->lay.bytes = cl.bytes;
    h->lay.cells = cp.cells;
    h->lay.nparts = cl.nparts;
    h->L = 0.0;
    for (int s = 0; s < 6; ++s) {
        h->ckind[s] = bc->kind[s];
        h->cTw[s] = bc->Tw[s];
    }
    h->c3cx = cp.cx;
    h->c3cy = cp.cy;
    h->c3cz = cp.cz;
    h->c3vol = cp.vol;
    Domain &d = h->dom;
    fill_domain(P, o.precision, o.buoyancy_update_only ? 0 : 1, o.round_nearest, o.max_mach, d);
    const bool dev = o.precision != RTLBFS_FP64_PLAIN;
    d.phd.Tref_s = dev ? bc->T_ref - kT0 : bc->T_ref;
    d.phf.Tref_s = (float)d.phd.Tref_s;
    if (workspace) {
        if (ws_bytes < cl.bytes) {
            delete h;
            g_create_err = "workspace smaller than rtlbfs_curv3_workspace_bytes()";
            return RTLBFS_ENOMEM;
        }
        h->ws = (char *)workspace;
    } else {
        hipError_t e = hipMalloc((void **)&h->ws, cl.bytes);
        if (e != hipSuccess) {
            delete h;
            g_create_err = "hipMalloc of the workspace failed";
            return RTLBFS_ENOMEM;
        }
        h->own_ws = true;
    }
    {
        const size_t es = elem_size(o.precision);
        std::vector<double> iv(cp.cells);
        for (int64_t c = 0; c < cp.cells; ++c) iv[c] = 1.0 / cp.vol[c];
        hipError_t e = hipSuccess;
        for (int a = 0; a < 3 && e == hipSuccess; ++a) {
            std::vector<char> b(cp.rec[a].size() * es);
            if (es == 4) put<float>(b.data(), cp.rec[a]);
            else put<double>(b.data(), cp.rec[a]);
            e = hipMemcpy(h->ws + cl.off_rec[a], b.data(), b.size(), hipMemcpyHostToDevice);
            if (e == hipSuccess && es == 4)
                e = hipMemcpy(h->ws + cl.off_rec64[a], cp.rec[a].data(), cp.rec[a].size() * sizeof(double),
                              hipMemcpyHostToDevice);
        }
        std::vector<char> biv(iv.size() * es);
        if (es == 4) put<float>(biv.data(), iv);
        else put<double>(biv.data(), iv);
        if (e == hipSuccess) e = hipMemcpy(h->ws + cl.off_iv, biv.data(), biv.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(h->ws + cl.off_vol, cp.vol.data(), cp.vol.size() * sizeof(double), hipMemcpyHostToDevice);
        const uint32_t zero2[2] = {0u, 0u};
        if (e == hipSuccess) e = hipMemcpy(h->ctr(), zero2, sizeof(zero2), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipHostMalloc((void **)&h->host_buf, 64 * sizeof(double), hipHostMallocDefault);
        if (e != hipSuccess) {
            int r2 = hip_fail(h, e, "upload geometry / capture stream");
            g_create_err = h->err;
            rtlbfs_destroy(h);
            return r2;
        }
    }
    d.vol = (const double *)(h->ws + cl.off_vol);
    for (int a = 0; a < 3; ++a) {
        d.w[a] = nullptr;
        d.geo[a] = nullptr;
    }
    Curv3Geo &g = h->c3;
    for (int a = 0; a < 3; ++a) {
        g.f[a] = h->ws + cl.off_rec[a];
        g.sf[a] = cl.nf[a];
        h->c3rec64[a] = (const double *)(h->ws + cl.off_rec64[a]);
        g.rc[a] = std::cos(bc->rot[a]);
        g.rs[a] = std::sin(bc->rot[a]);
        g.up[a] = bc->up[a];
        g.upf[a] = (float)bc->up[a];
    }
    g.nfaces = cl.nf[0] + cl.nf[1] + cl.nf[2];
    g.inv_vol = h->ws + cl.off_iv;
    g.prim = h->ws + cl.off_prim;
    g.grad = h->ws + cl.off_grad;
    g.flux = h->ws + cl.off_flux;

    const int64_t N = cp.cells;
    std::vector<double> rho((size_t)N, 1.0), u((size_t)N * 3, 0.0), T((size_t)N);
    for (int64_t c = 0; c < N; ++c) T[c] = bc->T_ref - kT0 + o.noise_amp * splitmix_uniform(o.seed, (uint64_t)c);
    rc = upload_prims(h, rho.data(), u.data(), T.data());
    if (rc == RTLBFS_OK) {
        hipError_t e = enqueue_integrals(h, h->int_out(), h->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(h->m0(), h->int_out(), sizeof(double), hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) rc = hip_fail(h, e, "initial integrals");
    }
    if (rc != RTLBFS_OK) {
        g_create_err = h->err;
        rtlbfs_destroy(h);
        return rc;
    }
    h->tile = 0;
    *out = h;
    return RTLBFS_OK;
}

int rtlbfs_curv3_cells(rtlbfs_t h, double *cx, double *cy, double *cz, double *vol, size_t count) {
    if (!h) return RTLBFS_EINVAL;
    if (!h->curv3) return fail(h, RTLBFS_EUNSUPPORTED, "not a 3D body-fitted mesh");
    if (count < h->c3cx.size()) return fail(h, RTLBFS_EINVAL, "count smaller than the cell count");
    const size_t b = h->c3cx.size() * sizeof(double);
    if (cx) std::memcpy(cx, h->c3cx.data(), b);
    if (cy) std::memcpy(cy, h->c3cy.data(), b);
    if (cz) std::memcpy(cz, h->c3cz.data(), b);
    if (vol) std::memcpy(vol, h->c3vol.data(), b);
    return RTLBFS_OK;
}

int rtlbfs_destroy(rtlbfs_t h) {
    if (!h) return RTLBFS_OK;
    if (h->stream || h->cap_stream) (void)hipStreamSynchronize(h->stream);
    for (int k = 0; k < 2; ++k)
        if (h->graph[k]) (void)hipGraphExecDestroy(h->graph[k]);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    if (h->host_buf) (void)hipHostFree(h->host_buf);
    if (h->own_ws && h->ws) (void)hipFree(h->ws);
    delete h;
    return RTLBFS_OK;
}

}  // extern "C"
