// lbm.hip -- host side of the C ABI declared in include/lbm.h.
//
// A domain holds one population array, updated in place by two alternating
// kernels (streaming step and local step), the list of 64-cell tiles that
// contain updated cells, and for tiles that touch a wall, inlet, box face or
// non-updated cell a 32-bit link mask per cell.  Interior tiles (every cell
// updated, every link a plain pull after periodic wrap) carry no mask and
// take the kernels' branch-free path.  Runs of steps are replayed from HIP
// graphs built node by node.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#define LBM_HOST_TU
#include "lbm_device.hpp"
#include "lbm_instances.hpp"
#include "../../include/lbm.h"

// the step and state-access kernels are compiled per storage format in
// lbm_kern.hip
namespace lbm {
LBM_INSTANCES(extern template, ST_FP32)
LBM_INSTANCES(extern template, ST_FP16S)
LBM_INSTANCES(extern template, ST_BF16S)
LBM_INSTANCES_WIDE(extern template, ST_FP32)
LBM_INSTANCES_WIDE(extern template, ST_FP16S)
LBM_INSTANCES_WIDE(extern template, ST_BF16S)
} // namespace lbm

using namespace lbm;

// Read-back buffer of lbm_get_moments_noalloc (see scratch_address).
constexpr uint64_t kScratchFloats = (uint64_t)16 << 20;
static __device__ __align__(256) float scratch[kScratchFloats];

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                                            \
    do {                                                                                                         \
        hipError_t e_ = (expr);                                                                                  \
        if (e_ != hipSuccess)                                                                                    \
            return fail(LBM_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));                          \
    } while (0)

size_t storage_bytes(int st) { return st == LBM_FP32 ? 4 : 2; }

FastDiv make_fastdiv(uint32_t d)
{
    FastDiv f{};
    uint32_t l = 0;
    while ((1ull << l) < d)
        ++l;
    f.m = (uint32_t)((((1ull << 32) * ((1ull << l) - d)) / d) + 1);
    f.s1 = l < 1 ? l : 1;
    f.s2 = l > 0 ? l - 1 : 0;
    f.d = d;
    return f;
}

bool updated(uint8_t fl) { return fl == LBM_FLUID || fl == LBM_OUTLET; }

// Link classification of one cell (host copy of the boundary rules):
// returns the wall mask (bit i: halfway bounce-back for population i,
// kMaskOutlet for an outlet cell, kMaskInlet if any link comes from an inlet
// cell, kMaskSkip if the cell is not updated) and the inlet mask; src[i]
// receives the inlet cell of each inlet link.
void classify_cell(const uint8_t *flags, int nx, int ny, int nz, unsigned per, uint64_t cell, uint32_t &wall,
                   uint32_t &inl, uint64_t *src = nullptr)
{
    wall = 0;
    inl = 0;
    const uint8_t self = flags[cell];
    if (!updated(self)) {
        wall = kMaskSkip;
        return;
    }
    if (self == LBM_OUTLET)
        wall |= kMaskOutlet;
    const int x = (int)(cell % nx), y = (int)((cell / nx) % ny), z = (int)(cell / ((uint64_t)nx * ny));
    for (int i = 0; i < Q; ++i) {
        int sx = x - cx(i), sy = y - cy(i), sz = z - cz(i);
        if (per & 1u)
            sx = (sx + nx) % nx;
        if (per & 2u)
            sy = (sy + ny) % ny;
        if (per & 4u)
            sz = (sz + nz) % nz;
        if (sx >= nx && !(per & 1u) && self == LBM_OUTLET)
            sx = nx - 1;
        if (sx < 0 || sx >= nx || sy < 0 || sy >= ny || sz < 0 || sz >= nz) {
            wall |= 1u << i;
            continue;
        }
        const uint64_t s = ((uint64_t)sz * ny + sy) * nx + sx;
        const uint8_t fs = flags[s];
        if (fs == LBM_SOLID) {
            wall |= 1u << i;
        } else if (fs == LBM_INLET) {
            wall |= (1u << i) | kMaskInlet;
            inl |= 1u << i;
            if (src)
                src[i] = s;
        }
    }
}

// Tile list of a domain.  wall: per cell of each wall tile the link mask;
// inlet: per cell of each wall tile the index of its inlet record (kNoRec
// if it has no inlet link); inlrec: per record the inlet link mask and 27
// inlet ordinals (the rank of the link's inlet cell among all inlet cells,
// kNoRec for other links); n_inl: tiles with an inlet-term block.
struct Tiles {
    std::vector<TileRec> recs;
    std::vector<uint32_t> wall, inlet, inlrec;
    uint64_t n_updated = 0;
    uint32_t n_inl = 0;
};

// Build the tile list in tile order.  Work is split over host threads by
// contiguous tile ranges and concatenated in order.  inlet_cells: the inlet
// cells in ascending order (their position is the inlet ordinal).
void build_tiles(const uint8_t *flags, int nx, int ny, int nz, unsigned per, const std::vector<uint64_t> &inlet_cells,
                 bool outlets, Tiles &out)
{
    const uint64_t ncells = (uint64_t)nx * ny * nz;
    const uint64_t ntiles = (ncells + 63) / 64;
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (ntiles < 4096)
        nth = 1;
    std::vector<Tiles> part(nth);
    auto work = [&](unsigned p) {
        const uint64_t t0 = ntiles * p / nth, t1 = ntiles * (p + 1) / nth;
        Tiles &T = part[p];
        uint32_t wl[64], il[64], rec[64];
        uint64_t src[Q];
        for (uint64_t t = t0; t < t1; ++t) {
            bool any = false, plain = true;
            TileRec r{0u, (uint32_t)t, -1, kNoRec, 0u, {0u, 0u}, 0u, 0u, 0u};
            for (int l = 0; l < 64; ++l) {
                const uint64_t c = t * 64 + l;
                rec[l] = kNoRec;
                if (c >= ncells) {
                    wl[l] = kMaskSkip;
                    il[l] = 0;
                } else {
                    classify_cell(flags, nx, ny, nz, per, c, wl[l], il[l], src);
                }
                if (il[l]) {
                    rec[l] = (uint32_t)(T.inlrec.size() / kRecWords);
                    T.inlrec.push_back(il[l]);
                    for (int i = 0; i < Q; ++i) {
                        uint32_t ord = kNoRec;
                        if (il[l] & (1u << i))
                            ord = (uint32_t)(std::lower_bound(inlet_cells.begin(), inlet_cells.end(), src[i]) -
                                             inlet_cells.begin());
                        T.inlrec.push_back(ord);
                    }
                }
                if (!(wl[l] & kMaskSkip)) {
                    any = true;
                    T.n_updated++;
                    r.act[l >> 5] |= 1u << (l & 31);
                    r.inlm |= il[l];
                    if (outlets && !(per & 1u) && (c % nx) == (uint64_t)nx - 1)
                        r.edge = 1u;
                }
                if (wl[l])
                    plain = false;
            }
            if (!any)
                continue;
            if (!plain) {
                r.wall = (int32_t)(T.wall.size() / 64);
                if (r.inlm)
                    r.inl = T.n_inl++;
                T.wall.insert(T.wall.end(), wl, wl + 64);
                T.inlet.insert(T.inlet.end(), rec, rec + 64);
            }
            T.recs.push_back(r);
        }
    };
    std::vector<std::thread> th;
    for (unsigned p = 1; p < nth; ++p)
        th.emplace_back(work, p);
    work(0);
    for (auto &t : th)
        t.join();
    for (unsigned p = 0; p < nth; ++p) {
        const int32_t off = (int32_t)(out.wall.size() / 64);
        const uint32_t roff = (uint32_t)(out.inlrec.size() / kRecWords);
        for (TileRec r : part[p].recs) {
            if (r.wall >= 0)
                r.wall += off;
            if (r.inl != kNoRec)
                r.inl += out.n_inl;
            r.ord = (uint32_t)out.recs.size();
            out.recs.push_back(r);
        }
        out.n_inl += part[p].n_inl;
        out.wall.insert(out.wall.end(), part[p].wall.begin(), part[p].wall.end());
        for (uint32_t r : part[p].inlet)
            out.inlet.push_back(r == kNoRec ? kNoRec : r + roff);
        out.inlrec.insert(out.inlrec.end(), part[p].inlrec.begin(), part[p].inlrec.end());
        out.n_updated += part[p].n_updated;
    }
}

// Step graphs: one per length 64, 32, ..., 2 steps (even lengths end in the
// phase they start in); a run of n steps replays the longest that fit.
constexpr int kGraphSizes = 6;
constexpr int graph_len(int j) { return 64 >> j; }

// Largest population array the buffer-instruction kernels address (their
// byte offsets are 32-bit); larger arrays take the 64-bit kernels.
constexpr uint64_t kNarrowBytes = (1ull << 32) - (1ull << 16);

// Bytes of a domain's population array: the tile blocks, then 2 x 9 side
// rows of ny * nz elements, rounded up to 256 bytes.
uint64_t array_bytes(uint64_t P, int ny, int nz, int storage)
{
    const uint64_t es = storage_bytes(storage);
    return (Q * P * es + 18ull * ny * nz * es + 255) / 256 * 256;
}

} // namespace

struct lbm_domain {
    int nx = 0, ny = 0, nz = 0, storage = 0;
    unsigned periodic = 0;
    uint64_t ncells = 0, P = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool own_buffers = true;
    int device = 0;
    char *buf = nullptr;  // the population array
    uint64_t bytes = 0;   // its size
    int phase = 0;        // phase of the stored state (k_stream_collide)
    bool outlets = false; // the domain has outlet cells
    int outlet_kind = LBM_OUTLET_ZERO_GRADIENT;
    double rho_out = 1.0; // outlet density of the constant-pressure outlet
    double *d_stats = nullptr;  // statistics sums, [15][64 ntiles]
    bool stats_on = false;
    uint64_t stats_samples = 0; // local steps accumulated
    uint8_t *d_flags = nullptr;
    TileRec *d_tiles = nullptr;
    uint32_t *d_wall = nullptr, *d_inlet = nullptr, *d_inlrec = nullptr;
    float *d_uin = nullptr;                // [3][n_inlet]
    float *d_iterm = nullptr;              // inlet terms, [27][64] per inlet tile
    float2 *d_bzc = nullptr;               // curved-wall coefficients, [27][64] per wall tile
    float *d_bzaux = nullptr;              // f*_k of the curved links, [27][64] per wall tile
    std::vector<uint32_t> h_wall, h_inlm;  // per wall-tile lane: link mask, inlet links
    uint32_t n_inl = 0;                    // inlet tiles
    std::vector<uint64_t> inlet_cells;     // inlet cells, ascending (index = inlet ordinal)
    uint32_t *d_status = nullptr;
    uint64_t ntiles = 0, nwall = 0, n_updated = 0;
    double omega = 1.0, omega_b = 1.0;
    double omega_o[4] = {1.0, 1.0, 1.0, 1.0}; // orders 3..6
    int feq_order = 6;                        // 6: the full equilibrium; 2..5: explicit truncated one
    bool high1() const { return omega_o[0] == 1.0 && omega_o[1] == 1.0 && omega_o[2] == 1.0 && omega_o[3] == 1.0; }
    bool curved() const { return d_bzc != nullptr; }
    bool explicit_feq() const { return feq_order < 6; }
    int variant() const
    {
        return (explicit_feq() ? kVarFeq : (high1() ? kVarH1 : 0)) | (curved() ? kVarCurved : 0) |
               (outlet_kind == LBM_OUTLET_PRESSURE ? kVarPressure : 0);
    }
    bool force_wide = false; // lbm_debug_wide_addressing
    uint32_t grid_blocks = 0; // lbm_debug_step_grid: blocks of a step launch (0: one wave per tile)
    // the step kernels address the array with 64-bit global instructions
    // (past the 4 GiB that buffer instructions reach)
    bool wide() const { return force_wide || bytes > kNarrowBytes; }
    bool unstable = false;
    hipGraphExec_t graph[kGraphSizes] = {};   // graph j runs graph_len(j) steps from phase 0
    hipGraph_t graph_def[kGraphSizes] = {};
    bool graph_dirty = true;
    std::vector<TileRec> h_tiles; // host copy of the tile list (batch tables are built from it)
    lbm_batch *batch = nullptr;    // resident in this batch
    uint64_t device_bytes = 0;
    uint64_t flags_hash = 0;       // FNV-1a 64 of the creation flags (state images name it)
};

namespace {

// Device memory of domains comes from the stream-ordered allocator: a free
// does not synchronise the device (a service frees domains while other
// domains keep running), and freed memory stays in the device's pool for
// the next domain.
std::mutex g_pool_mutex;
bool g_pool_ready[64];

void pool_setup(int device)
{
    std::lock_guard<std::mutex> lock(g_pool_mutex);
    if (device < 0 || device >= 64 || g_pool_ready[device])
        return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
        uint64_t keep = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    (void)hipGetLastError();
    g_pool_ready[device] = true;
}

hipError_t dalloc(hipStream_t s, void **p, size_t n)
{
    *p = nullptr;
    if (n == 0)
        return hipSuccess;
    hipError_t e = hipMallocAsync(p, n, s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
    }
    return e;
}

void dfree(hipStream_t s, void *p)
{
    if (p)
        (void)hipFreeAsync(p, s);
}

// Copies between host memory and the domain's memory, in the domain's
// stream order; they return once the copy is complete.
hipError_t copy_sync(hipStream_t s, void *dst, const void *src, size_t n, hipMemcpyKind kind)
{
    if (n == 0)
        return hipSuccess;
    hipError_t e = hipMemcpyAsync(dst, src, n, kind, s);
    if (e != hipSuccess)
        return e;
    return hipStreamSynchronize(s);
}

KDomain kdomain(const lbm_domain *d)
{
    KDomain k{};
    k.buf = d->buf;
    k.flags = d->d_flags;
    k.stats = d->stats_on ? d->d_stats : nullptr;
    k.sstride = (uint32_t)(d->ntiles * 64);
    k.wall = d->d_wall;
    k.iterm = d->d_iterm;
    k.bzc = d->d_bzc;
    k.bzaux = d->d_bzaux;
    k.rowtiles = d->nx % 64 == 0 ? (uint32_t)(d->nx / 64) : 0u;
    k.drow = make_fastdiv(k.rowtiles ? k.rowtiles : 1u);
    k.status = d->d_status;
    k.P = (uint32_t)d->P;
    k.tbytes = (uint32_t)(Q * 64 * storage_bytes(d->storage));
    k.side = d->P / 64 * k.tbytes;
    k.bufbytes = d->bytes <= kNarrowBytes ? (uint32_t)d->bytes : 0u; // read by the narrow kernels only
    k.nx = d->nx;
    k.ny = d->ny;
    k.nz = d->nz;
    k.ncells = (uint32_t)d->ncells;
    k.dnx = make_fastdiv(d->nx);
    k.dny = make_fastdiv(d->ny);
    k.periodic = d->periodic;
    k.omega = (float)d->omega;
    k.omega_b = (float)d->omega_b;
    for (int n = 0; n < 4; ++n)
        k.omega_o[n] = (float)d->omega_o[n];
    k.outlet = d->outlet_kind == LBM_OUTLET_PRESSURE ? 1u : 0u;
    k.high1 = d->high1() ? 1u : 0u;
    k.rho_out = (float)d->rho_out;
    k.feq_order = (uint32_t)d->feq_order;
    return k;
}

uint32_t grid8(uint64_t blocks) { return (uint32_t)((blocks + 7) / 8 * 8); }

// Grid of the single-domain kernels: one wave per tile (a wave's loads and
// collision do not overlap within the wave, and tiles per wave beyond one
// measured slower).
uint32_t step_grid(const lbm_domain *d)
{
    if (d->grid_blocks)
        return d->grid_blocks;
    return grid8((d->ntiles + kWavesPerBlock - 1) / kWavesPerBlock);
}

template <typename F> decltype(auto) dispatch_storage(int st, F &&f)
{
    if (st == LBM_FP32)
        return f(std::integral_constant<int, ST_FP32>{});
    else if (st == LBM_FP16S)
        return f(std::integral_constant<int, ST_FP16S>{});
    else
        return f(std::integral_constant<int, ST_BF16S>{});
}

int sync_status(lbm_domain *d)
{
    HIP_TRY(hipStreamSynchronize(d->stream));
    uint32_t st = 0;
    HIP_TRY(copy_sync(d->stream, &st, d->d_status, sizeof st, hipMemcpyDeviceToHost));
    if (st)
        d->unstable = true;
    return LBM_OK;
}

int check_domain(const lbm_domain *d)
{
    if (!d)
        return fail(LBM_ERR_ARG, "null domain");
    return LBM_OK;
}

void release_graph(lbm_domain *d)
{
    for (int j = 0; j < kGraphSizes; ++j) {
        if (d->graph[j])
            (void)hipGraphExecDestroy(d->graph[j]);
        if (d->graph_def[j])
            (void)hipGraphDestroy(d->graph_def[j]);
        d->graph[j] = nullptr;
        d->graph_def[j] = nullptr;
    }
    d->graph_dirty = true;
}

void free_domain(lbm_domain *d)
{
    release_graph(d);
    if (d->stream) {
        hipStream_t s = d->stream;
        if (d->own_buffers)
            dfree(s, d->buf);
        dfree(s, d->d_flags);
        dfree(s, d->d_tiles);
        dfree(s, d->d_wall);
        dfree(s, d->d_inlet);
        dfree(s, d->d_inlrec);
        dfree(s, d->d_uin);
        dfree(s, d->d_iterm);
        dfree(s, d->d_bzc);
        dfree(s, d->d_bzaux);
        dfree(s, d->d_stats);
        dfree(s, d->d_status);
        if (d->own_stream)
            (void)hipStreamDestroy(s);
    }
    delete d;
}

// Calls fn(std::integral_constant<int, ST>, std::integral_constant<int, V>)
// for a storage and a kernel variant known at run time.
// The explicit equilibrium always takes the general collision, so a variant
// with both bits set runs as the one without the reduced-collision bit.
template <class Fn> decltype(auto) with_kernel(int storage, int v, Fn &&fn)
{
    return dispatch_storage(storage, [&](auto st) {
        switch ((v & kVarFeq) ? (v & ~kVarH1) : v) {
        case 0:
            return fn(st, std::integral_constant<int, 0>{});
        case 1:
            return fn(st, std::integral_constant<int, 1>{});
        case 2:
            return fn(st, std::integral_constant<int, 2>{});
        case 3:
            return fn(st, std::integral_constant<int, 3>{});
        case 4:
            return fn(st, std::integral_constant<int, 4>{});
        case 5:
            return fn(st, std::integral_constant<int, 5>{});
        case 6:
            return fn(st, std::integral_constant<int, 6>{});
        case 7:
            return fn(st, std::integral_constant<int, 7>{});
        case 8:
            return fn(st, std::integral_constant<int, 8>{});
        case 10:
            return fn(st, std::integral_constant<int, 10>{});
        case 12:
            return fn(st, std::integral_constant<int, 12>{});
        default:
            return fn(st, std::integral_constant<int, 14>{});
        }
    });
}

// The step kernel of a phase: the streaming step (phase 0) with row-aligned
// or general addressing, or the local step; narrow or wide (Pops).
const void *step_kernel(int storage, int v, uint32_t phase, bool rows, bool wide)
{
    return with_kernel(storage, v, [&](auto st, auto vc) -> const void * {
        constexpr int ST = decltype(st)::value, V = decltype(vc)::value;
        if (wide) {
            if (phase == 1)
                return (const void *)k_local_collide<ST, V, true>;
            return rows ? (const void *)k_stream_collide<ST, V, true, true>
                        : (const void *)k_stream_collide<ST, V, false, true>;
        }
        if (phase == 1)
            return (const void *)k_local_collide<ST, V, false>;
        return rows ? (const void *)k_stream_collide<ST, V, true, false>
                    : (const void *)k_stream_collide<ST, V, false, false>;
    });
}

hipError_t launch_step(const lbm_domain *d, uint32_t phase)
{
    if (d->ntiles == 0)
        return hipSuccess;
    KDomain k = kdomain(d);
    const TileRec *tiles = d->d_tiles;
    uint32_t nt = (uint32_t)d->ntiles;
    void *args[] = {&k, &tiles, &nt};
    const hipError_t e = hipLaunchKernel(step_kernel(d->storage, d->variant(), phase, k.rowtiles != 0, d->wide()),
                                         dim3(step_grid(d)), dim3(kBlock), args, 0, d->stream);
    return e != hipSuccess ? e : hipGetLastError();
}

// Rebuild the inlet terms of the inlet tiles from the inlet velocity (all
// zero while none is set).
hipError_t build_inlet_terms(const lbm_domain *d)
{
    if (d->n_inl == 0)
        return hipSuccess;
    const uint32_t blocks = (uint32_t)((d->ntiles + 3) / 4);
    hipLaunchKernelGGL(k_inlet_terms, dim3(blocks), dim3(256), 0, d->stream, (const TileRec *)d->d_tiles,
                       (uint32_t)d->ntiles, (const uint32_t *)d->d_inlet, (const uint32_t *)d->d_inlrec,
                       (const float *)d->d_uin, (uint32_t)d->inlet_cells.size(), d->d_iterm);
    return hipGetLastError();
}

// First side rows of a phase-0 state (the outlet cells' clamped values).
hipError_t side_refresh(const lbm_domain *d)
{
    if (!d->outlets)
        return hipSuccess;
    const KDomain k = kdomain(d);
    const uint32_t blocks = (uint32_t)(((uint64_t)d->ny * d->nz + 255) / 256);
    dispatch_storage(d->storage, [&](auto st) {
        hipLaunchKernelGGL((k_side_refresh<decltype(st)::value>), dim3(blocks), dim3(256), 0, d->stream, k);
    });
    return hipGetLastError();
}

// Curved-wall values of a phase-0 state (k_curved_refresh).
hipError_t curved_refresh(const lbm_domain *d)
{
    if (!d->d_bzaux || !d->ntiles)
        return hipSuccess;
    const KDomain k = kdomain(d);
    const uint32_t blocks = (uint32_t)((d->ntiles + 3) / 4);
    dispatch_storage(d->storage, [&](auto st) {
        hipLaunchKernelGGL((k_curved_refresh<decltype(st)::value>), dim3(blocks), dim3(256), 0, d->stream, k,
                           (const TileRec *)d->d_tiles, (uint32_t)d->ntiles);
    });
    return hipGetLastError();
}

// Bring the stored state to phase 0, the form every state access uses.
hipError_t normalise(lbm_domain *d)
{
    if (d->phase == 0)
        return hipSuccess;
    if (d->ntiles) {
        const KDomain k = kdomain(d);
        const uint32_t blocks = (uint32_t)((d->ntiles + 3) / 4);
        dispatch_storage(d->storage, [&](auto st) {
            hipLaunchKernelGGL((k_normalise<decltype(st)::value>), dim3(blocks), dim3(256), 0, d->stream, k,
                               (const TileRec *)d->d_tiles, (uint32_t)d->ntiles);
        });
        if (hipError_t e = hipGetLastError())
            return e;
    }
    d->phase = 0;
    return hipSuccess;
}

// f^eq of the given fields (null: rho = 1, u = 0) in every cell, phase 0.
int init_eq(lbm_domain *d, const float *rho_dev, const float *u_dev)
{
    const KDomain k = kdomain(d);
    const uint32_t blocks = (uint32_t)((d->P + 255) / 256);
    dispatch_storage(d->storage, [&](auto st) {
        hipLaunchKernelGGL((k_init_eq<decltype(st)::value>), dim3(blocks), dim3(256), 0, d->stream, k, rho_dev, u_dev);
    });
    HIP_TRY(hipGetLastError());
    d->phase = 0;
    HIP_TRY(side_refresh(d));
    HIP_TRY(curved_refresh(d));
    HIP_TRY(hipMemsetAsync(d->d_status, 0, sizeof(uint32_t), d->stream));
    d->unstable = false;
    return LBM_OK;
}

// Cells rounded up to whole 64-cell tiles.
uint64_t plane_stride(uint64_t ncells) { return (ncells + 63) / 64 * 64; }

// Read-back buffer of lbm_get_moments_noalloc, for callers that cannot
// allocate: a fixed device array (64 MiB, 4 floats per cell) that each
// device holds from the library's load to the end of the process.  Host
// code uses it only through the device address hipGetSymbolAddress gives
// for the current device, resolved once per device.  Calls on one device
// share it, so they are serialised by a lock.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex[kMaxDevices];
std::mutex g_scratch_resolve;
float *g_scratch_ptr[kMaxDevices];

int scratch_address(int device, float **out)
{
    if (device < 0 || device >= kMaxDevices)
        return fail(LBM_ERR_DEVICE, "device %d out of range", device);
    std::lock_guard<std::mutex> lock(g_scratch_resolve);
    if (!g_scratch_ptr[device]) {
        int cur = 0;
        HIP_TRY(hipGetDevice(&cur));
        HIP_TRY(hipSetDevice(device));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        (void)hipSetDevice(cur);
        if (e != hipSuccess || !p)
            return fail(LBM_ERR_DEVICE, "read-back buffer address: %s", hipGetErrorString(e));
        g_scratch_ptr[device] = (float *)p;
    }
    *out = g_scratch_ptr[device];
    return LBM_OK;
}

int create(const uint8_t *flags, int nx, int ny, int nz, unsigned periodic, int storage, void *hip_stream, void *fa,
           lbm_domain **out)
{
    if (!out)
        return fail(LBM_ERR_ARG, "out is null");
    *out = nullptr;
    if (!flags)
        return fail(LBM_ERR_ARG, "flags is null");
    if (nx < 1 || ny < 1 || nz < 1 || nx > 65535 || ny > 65535 || nz > 65535)
        return fail(LBM_ERR_ARG, "bad grid %d x %d x %d", nx, ny, nz);
    if (storage < LBM_FP32 || storage > LBM_BF16S)
        return fail(LBM_ERR_ARG, "bad storage %d", storage);
    if (periodic > 7u)
        return fail(LBM_ERR_ARG, "bad periodic mask %u", periodic);
    const uint64_t ncells = (uint64_t)nx * ny * nz;
    const uint64_t P = plane_stride(ncells);
    const uint64_t bufbytes = array_bytes(P, ny, nz, storage);
    // cell indices are 32-bit
    if (P > (1ull << 32) - 64)
        return fail(LBM_ERR_ARG, "domain of %llu cells; the limit is 2^32 - 64 cells", (unsigned long long)ncells);
    std::vector<uint64_t> inlet_cells;
    bool outlets = false;
    uint64_t hash = 0xcbf29ce484222325ull;
    for (uint64_t c = 0; c < ncells; ++c) {
        const uint8_t f = flags[c];
        if (f > LBM_OUTLET)
            return fail(LBM_ERR_ARG, "bad flag %u at cell %llu", f, (unsigned long long)c);
        if (f == LBM_OUTLET && ((c % nx) != (uint64_t)nx - 1 || (periodic & 1u)))
            return fail(LBM_ERR_ARG, "outlet cell %llu not on the last x plane of a non-periodic x axis",
                        (unsigned long long)c);
        if (f == LBM_INLET)
            inlet_cells.push_back(c);
        outlets |= f == LBM_OUTLET;
        hash = (hash ^ f) * 0x100000001b3ull;
    }
    Tiles T;
    build_tiles(flags, nx, ny, nz, periodic, inlet_cells, outlets, T);

    lbm_domain *d = new lbm_domain();
    d->nx = nx;
    d->ny = ny;
    d->nz = nz;
    d->storage = storage;
    d->periodic = periodic;
    d->ncells = ncells;
    d->P = P;
    d->bytes = bufbytes;
    d->outlets = outlets;
    d->flags_hash = hash;
    d->ntiles = T.recs.size();
    d->nwall = T.wall.size() / 64;
    d->n_updated = T.n_updated;
    d->h_tiles = T.recs;
    d->h_wall = T.wall;
    d->h_inlm.assign(T.wall.size(), 0u);
    for (size_t l = 0; l < T.inlet.size(); ++l)
        if (T.inlet[l] != kNoRec)
            d->h_inlm[l] = T.inlrec[(size_t)T.inlet[l] * kRecWords];
    d->n_inl = T.n_inl;
    d->inlet_cells = std::move(inlet_cells);
    auto bail = [&](int code) {
        free_domain(d);
        return code;
    };
    if (hipGetDevice(&d->device) != hipSuccess)
        return bail(fail(LBM_ERR_DEVICE, "no HIP device"));
    if (hip_stream) {
        d->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&d->stream, hipStreamNonBlocking) != hipSuccess)
            return bail(fail(LBM_ERR_DEVICE, "hipStreamCreate failed"));
        d->own_stream = true;
    }
    pool_setup(d->device);
    auto dmalloc = [&](void **p, size_t n) -> bool {
        if (dalloc(d->stream, p, n) != hipSuccess)
            return false;
        d->device_bytes += n;
        return true;
    };
    if (fa) {
        d->own_buffers = false;
        d->buf = (char *)fa;
        if ((uintptr_t)fa & 255u)
            return bail(fail(LBM_ERR_ARG, "an adopted population array must be 256-byte aligned"));
        d->device_bytes += bufbytes;
    } else if (!dmalloc((void **)&d->buf, bufbytes)) {
        return bail(fail(LBM_ERR_OOM, "population array (%llu bytes)", (unsigned long long)bufbytes));
    }
    if (!dmalloc((void **)&d->d_flags, ncells) || !dmalloc((void **)&d->d_tiles, T.recs.size() * sizeof(TileRec)) ||
        !dmalloc((void **)&d->d_wall, T.wall.size() * 4) || !dmalloc((void **)&d->d_inlet, T.inlet.size() * 4) ||
        !dmalloc((void **)&d->d_inlrec, T.inlrec.size() * 4) || !dmalloc((void **)&d->d_status, sizeof(uint32_t)) ||
        !dmalloc((void **)&d->d_iterm, (size_t)T.n_inl * Q * 64 * sizeof(float)))
        return bail(fail(LBM_ERR_OOM, "domain tables"));
    auto up = [&](void *dst, const void *src, size_t n) {
        return copy_sync(d->stream, dst, src, n, hipMemcpyHostToDevice) == hipSuccess;
    };
    if (!up(d->d_flags, flags, ncells) || !up(d->d_tiles, T.recs.data(), T.recs.size() * sizeof(TileRec)) ||
        !up(d->d_wall, T.wall.data(), T.wall.size() * 4) || !up(d->d_inlet, T.inlet.data(), T.inlet.size() * 4) ||
        !up(d->d_inlrec, T.inlrec.data(), T.inlrec.size() * 4))
        return bail(fail(LBM_ERR_DEVICE, "upload of domain tables failed"));
    if (build_inlet_terms(d) != hipSuccess)
        return bail(fail(LBM_ERR_DEVICE, "inlet terms"));
    d->omega = d->omega_b = 1.0 / 0.6;
    // the side rows' elements that no outlet cell uses, and the padding
    // after them, are never written: zero, so that state images are
    // deterministic (the tile blocks are written by init_eq)
    const uint64_t tile_bytes = (uint64_t)Q * P * storage_bytes(storage);
    if (hipMemsetAsync(d->buf + tile_bytes, 0, bufbytes - tile_bytes, d->stream) != hipSuccess)
        return bail(fail(LBM_ERR_DEVICE, "side rows"));
    int rc = init_eq(d, nullptr, nullptr);
    if (rc == LBM_OK && hipStreamSynchronize(d->stream) != hipSuccess)
        rc = fail(LBM_ERR_DEVICE, "initialisation failed");
    if (rc != LBM_OK)
        return bail(rc);
    *out = d;
    return LBM_OK;
}

// Append a kernel node after `prev` (or as a root when prev is null).  The
// argument values are copied into the node.
hipError_t add_kernel_node(hipGraph_t g, hipGraphNode_t prev, const void *func, uint32_t grid, uint32_t block,
                           void **args, hipGraphNode_t *out)
{
    hipKernelNodeParams p{};
    p.func = const_cast<void *>(func);
    p.gridDim = dim3(grid);
    p.blockDim = dim3(block);
    p.sharedMemBytes = 0;
    p.kernelParams = args;
    p.extra = nullptr;
    return hipGraphAddKernelNode(out, g, prev ? &prev : nullptr, prev ? 1 : 0, &p);
}


// Build (not capture) the step graphs: graph j chains graph_len(j) step
// nodes starting in phase 0.  Built node by node so that work other threads
// issue meanwhile cannot interfere.
int build_graph(lbm_domain *d)
{
    release_graph(d);
    KDomain k = kdomain(d);
    const TileRec *tiles = d->d_tiles;
    uint32_t nt = (uint32_t)d->ntiles;
    for (int j = 0; j < kGraphSizes; ++j) {
        hipGraph_t g = nullptr;
        HIP_TRY(hipGraphCreate(&g, 0));
        hipGraphNode_t prev = nullptr;
        for (int s = 0; s < graph_len(j); ++s) {
            const void *fn = step_kernel(d->storage, d->variant(), (uint32_t)(s & 1), k.rowtiles != 0, d->wide());
            void *args[] = {&k, &tiles, &nt};
            hipGraphNode_t node = nullptr;
            hipError_t e = add_kernel_node(g, prev, fn, step_grid(d), kBlock, args, &node);
            if (e != hipSuccess) {
                (void)hipGraphDestroy(g);
                return fail(LBM_ERR_DEVICE, "graph node: %s", hipGetErrorString(e));
            }
            prev = node;
        }
        d->graph_def[j] = g;
        HIP_TRY(hipGraphInstantiate(&d->graph[j], g, nullptr, nullptr, 0));
    }
    d->graph_dirty = false;
    return LBM_OK;
}

} // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *lbm_last_error(void) { return g_err.c_str(); }

const char *lbm_version(void) { return "lbm-d3q27-chm gfx950 0.1"; }

uint64_t lbm_array_bytes(int nx, int ny, int nz, int storage)
{
    if (nx < 1 || ny < 1 || nz < 1 || nx > 65535 || ny > 65535 || nz > 65535 || storage < LBM_FP32 ||
        storage > LBM_BF16S)
        return 0;
    return array_bytes(plane_stride((uint64_t)nx * ny * nz), ny, nz, storage);
}

int lbm_create_domain(const uint8_t *flags, int nx, int ny, int nz, unsigned periodic, int storage,
                      void *hip_stream, lbm_domain **out)
{
    return create(flags, nx, ny, nz, periodic, storage, hip_stream, nullptr, out);
}

int lbm_create_domain_ext(const uint8_t *flags, int nx, int ny, int nz, unsigned periodic, int storage,
                          void *hip_stream, void *f, lbm_domain **out)
{
    if (!f)
        return fail(LBM_ERR_ARG, "adopted population array is null");
    return create(flags, nx, ny, nz, periodic, storage, hip_stream, f, out);
}

int lbm_set_rates(lbm_domain *d, double omega, double omega_bulk, double omega_high)
{
    if (int rc = check_domain(d))
        return rc;
    if (!(omega >= 0 && omega <= 2) || !(omega_bulk >= 0 && omega_bulk <= 2) ||
        !(omega_high >= 0 && omega_high <= 2))
        return fail(LBM_ERR_ARG, "rates must lie in [0, 2]");
    if (d->batch)
        return fail(LBM_ERR_STATE, "domain is resident in a batch");
    d->omega = omega;
    d->omega_b = omega_bulk;
    for (int n = 0; n < 4; ++n)
        d->omega_o[n] = omega_high;
    d->graph_dirty = true;
    return LBM_OK;
}

int lbm_set_order_rates(lbm_domain *d, double omega3, double omega4, double omega5, double omega6)
{
    if (int rc = check_domain(d))
        return rc;
    const double w[4] = {omega3, omega4, omega5, omega6};
    for (double v : w)
        if (!(v >= 0 && v <= 2))
            return fail(LBM_ERR_ARG, "rates must lie in [0, 2]");
    if (d->batch)
        return fail(LBM_ERR_STATE, "domain is resident in a batch");
    for (int n = 0; n < 4; ++n)
        d->omega_o[n] = w[n];
    d->graph_dirty = true;
    return LBM_OK;
}

int lbm_set_equilibrium_order(lbm_domain *d, int order)
{
    if (int rc = check_domain(d))
        return rc;
    if (order < 2 || order > 6)
        return fail(LBM_ERR_ARG, "equilibrium order %d outside 2..6", order);
    if (d->batch)
        return fail(LBM_ERR_STATE, "domain is resident in a batch");
    d->feq_order = order;
    d->graph_dirty = true;
    return LBM_OK;
}

int lbm_debug_wide_addressing(lbm_domain *d, int on)
{
    if (int rc = check_domain(d))
        return rc;
    if (on != 0 && on != 1)
        return fail(LBM_ERR_ARG, "on must be 0 or 1");
    if (d->batch)
        return fail(LBM_ERR_STATE, "domain is resident in a batch");
    d->force_wide = on == 1;
    d->graph_dirty = true;
    return LBM_OK;
}

int lbm_debug_step_grid(lbm_domain *d, int blocks)
{
    if (int rc = check_domain(d))
        return rc;
    if (blocks < 0 || blocks % 8 != 0 || blocks > (1 << 20))
        return fail(LBM_ERR_ARG, "blocks must be 0 or a positive multiple of 8 up to 2^20, got %d", blocks);
    if (d->batch)
        return fail(LBM_ERR_STATE, "domain is resident in a batch");
    d->grid_blocks = (uint32_t)blocks;
    d->graph_dirty = true;
    return LBM_OK;
}

int lbm_is_wide(const lbm_domain *d, int *wide)
{
    if (int rc = check_domain(d))
        return rc;
    if (!wide)
        return fail(LBM_ERR_ARG, "wide is null");
    *wide = d->wide() ? 1 : 0;
    return LBM_OK;
}

int lbm_set_outlet(lbm_domain *d, int kind, double rho_out)
{
    if (int rc = check_domain(d))
        return rc;
    if (kind != LBM_OUTLET_ZERO_GRADIENT && kind != LBM_OUTLET_PRESSURE)
        return fail(LBM_ERR_ARG, "unknown outlet kind %d", kind);
    if (!(rho_out > 0) || !std::isfinite(rho_out))
        return fail(LBM_ERR_ARG, "rho_out must be positive and finite");
    if (d->batch)
        return fail(LBM_ERR_STATE, "domain is resident in a batch");
    HIP_TRY(normalise(d));
    d->outlet_kind = kind;
    d->rho_out = rho_out;
    HIP_TRY(side_refresh(d));
    d->graph_dirty = true;
    return LBM_OK;
}

int lbm_set_wall_distances(lbm_domain *d, const float *q)
{
    if (int rc = check_domain(d))
        return rc;
    if (d->batch)
        return fail(LBM_ERR_STATE, "domain is resident in a batch");
    const size_t nco = (size_t)d->nwall * Q * 64;
    std::vector<float2> coef;
    std::vector<uint32_t> bz(d->h_tiles.size(), 0u);
    if (q) {
        coef.assign(nco, make_float2(1.f, 0.f));
        for (size_t t = 0; t < d->h_tiles.size(); ++t) {
            const TileRec &r = d->h_tiles[t];
            if (r.wall < 0)
                continue;
            for (uint32_t l = 0; l < 64; ++l) {
                if (!((r.act[l >> 5] >> (l & 31)) & 1u))
                    continue;
                const uint64_t c = (uint64_t)r.tile * 64 + l;
                const size_t wl = (size_t)r.wall * 64 + l;
                const uint32_t m = d->h_wall[wl], il = d->h_inlm[wl];
                for (int k = 0; k < Q; ++k) {
                    if (!((m >> k) & 1u) || ((il >> k) & 1u))
                        continue; // not a wall link
                    const double qq = q[(size_t)k * d->ncells + c];
                    if (!(qq > 0.0 && qq <= 1.0))
                        return fail(LBM_ERR_ARG, "wall fraction %g of link %d of cell %llu outside (0, 1]", qq, k,
                                    (unsigned long long)c);
                    double a, b;
                    if (qq == 0.5 || (qq < 0.5 && ((m >> (Q - 1 - k)) & 1u)))
                        continue; // halfway rule
                    if (qq < 0.5) {
                        a = 2.0 * qq;
                        b = 1.0 - 2.0 * qq;
                    } else {
                        a = 1.0 / (2.0 * qq);
                        b = -(1.0 - 1.0 / (2.0 * qq));
                    }
                    coef[((size_t)r.wall * Q + k) * 64 + l] = make_float2((float)a, (float)b);
                    bz[t] |= 1u << k;
                }
            }
        }
    }
    bool any = false;
    for (uint32_t b : bz)
        any |= b != 0;
    HIP_TRY(normalise(d));
    if (any && !d->d_bzc) {
        if (dalloc(d->stream, (void **)&d->d_bzc, nco * sizeof(float2)) != hipSuccess ||
            dalloc(d->stream, (void **)&d->d_bzaux, nco * sizeof(float)) != hipSuccess) {
            dfree(d->stream, d->d_bzc);
            d->d_bzc = nullptr;
            d->d_bzaux = nullptr;
            return fail(LBM_ERR_OOM, "curved-wall tables");
        }
        d->device_bytes += nco * (sizeof(float2) + sizeof(float));
    }
    if (!any && d->d_bzc) {
        dfree(d->stream, d->d_bzc);
        dfree(d->stream, d->d_bzaux);
        d->d_bzc = nullptr;
        d->d_bzaux = nullptr;
        d->device_bytes -= nco * (sizeof(float2) + sizeof(float));
    }
    for (size_t t = 0; t < bz.size(); ++t)
        d->h_tiles[t].bz = bz[t];
    if (!d->h_tiles.empty())
        HIP_TRY(copy_sync(d->stream, d->d_tiles, d->h_tiles.data(), d->h_tiles.size() * sizeof(TileRec),
                          hipMemcpyHostToDevice));
    if (any) {
        HIP_TRY(copy_sync(d->stream, d->d_bzc, coef.data(), nco * sizeof(float2), hipMemcpyHostToDevice));
        // kept values of lanes and links without a curved coefficient are
        // never written: zero, so that state images are deterministic
        HIP_TRY(hipMemsetAsync(d->d_bzaux, 0, nco * sizeof(float), d->stream));
        HIP_TRY(curved_refresh(d));
        HIP_TRY(hipStreamSynchronize(d->stream));
    }
    d->graph_dirty = true;
    return LBM_OK;
}

int lbm_set_params(lbm_domain *d, double tau, double omega_bulk, double omega_high)
{
    if (int rc = check_domain(d))
        return rc;
    if (!(tau > 0.5) || !std::isfinite(tau))
        return fail(LBM_ERR_ARG, "tau must be > 0.5");
    if (!(omega_bulk > 0 && omega_bulk < 2))
        return fail(LBM_ERR_ARG, "omega_bulk must lie in (0, 2)");
    if (!(omega_high > 0 && omega_high <= 2))
        return fail(LBM_ERR_ARG, "omega_high must lie in (0, 2]");
    return lbm_set_rates(d, 1.0 / tau, omega_bulk, omega_high);
}

int lbm_set_inlet_cells(lbm_domain *d, const float *u_inlet)
{
    if (int rc = check_domain(d))
        return rc;
    if (!u_inlet)
        return fail(LBM_ERR_ARG, "u_inlet is null");
    if (d->batch)
        return fail(LBM_ERR_STATE, "domain is resident in a batch");
    const size_t n = d->inlet_cells.size();
    if (n == 0)
        return LBM_OK;
    if (!d->d_uin) {
        if (dalloc(d->stream, (void **)&d->d_uin, 3 * n * sizeof(float)) != hipSuccess)
            return fail(LBM_ERR_OOM, "inlet velocity buffer");
        d->device_bytes += 3 * n * sizeof(float);
        d->graph_dirty = true;
    }
    // a phase-1 state carries the old terms in its bounce-back slots
    HIP_TRY(normalise(d));
    HIP_TRY(copy_sync(d->stream, d->d_uin, u_inlet, 3 * n * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(build_inlet_terms(d));
    HIP_TRY(hipStreamSynchronize(d->stream));
    return LBM_OK;
}

int lbm_set_inlet(lbm_domain *d, const float *u_in)
{
    if (int rc = check_domain(d))
        return rc;
    if (!u_in)
        return fail(LBM_ERR_ARG, "u_in is null");
    const size_t n = d->inlet_cells.size();
    std::vector<float> compact(3 * n);
    for (int a = 0; a < 3; ++a)
        for (size_t k = 0; k < n; ++k)
            compact[a * n + k] = u_in[a * d->ncells + d->inlet_cells[k]];
    return lbm_set_inlet_cells(d, compact.data());
}

int lbm_init_fields(lbm_domain *d, const float *rho, const float *u)
{
    if (int rc = check_domain(d))
        return rc;
    if (d->batch)
        return fail(LBM_ERR_STATE, "domain is resident in a batch");
    float *dr = nullptr, *du = nullptr;
    int rc = LBM_OK;
    if (rho && dalloc(d->stream, (void **)&dr, d->ncells * sizeof(float)) != hipSuccess)
        rc = fail(LBM_ERR_OOM, "staging buffer");
    if (rc == LBM_OK && u && dalloc(d->stream, (void **)&du, 3 * d->ncells * sizeof(float)) != hipSuccess)
        rc = fail(LBM_ERR_OOM, "staging buffer");
    if (rc == LBM_OK && rho &&
        copy_sync(d->stream, dr, rho, d->ncells * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        rc = fail(LBM_ERR_DEVICE, "upload of rho failed");
    if (rc == LBM_OK && u &&
        copy_sync(d->stream, du, u, 3 * d->ncells * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        rc = fail(LBM_ERR_DEVICE, "upload of u failed");
    if (rc == LBM_OK)
        rc = init_eq(d, dr, du);
    if (rc == LBM_OK && hipStreamSynchronize(d->stream) != hipSuccess)
        rc = fail(LBM_ERR_DEVICE, "initialisation failed");
    dfree(d->stream, dr);
    dfree(d->stream, du);
    return rc;
}

int lbm_step_async(lbm_domain *d, int n)
{
    if (int rc = check_domain(d))
        return rc;
    if (n < 0)
        return fail(LBM_ERR_ARG, "negative step count");
    if (d->batch)
        return fail(LBM_ERR_STATE, "domain is resident in a batch");
    if (d->unstable)
        return fail(LBM_ERR_UNSTABLE, "domain went unstable earlier; re-initialise it");
    if (d->ntiles == 0) // nothing is updated, the state stays as it is
        return LBM_OK;
    if (n >= 2 && d->graph_dirty)
        if (int rc = build_graph(d))
            return rc;
    int left = n;
    uint64_t local_steps = 0;
    if (left > 0 && d->phase == 1) {
        HIP_TRY(launch_step(d, 1));
        d->phase = 0;
        --left;
        ++local_steps;
    }
    for (int j = 0; j < kGraphSizes; ++j) {
        while (left >= graph_len(j)) {
            HIP_TRY(hipGraphLaunch(d->graph[j], d->stream));
            left -= graph_len(j);
            local_steps += (uint64_t)graph_len(j) / 2;
        }
    }
    while (left > 0) {
        HIP_TRY(launch_step(d, (uint32_t)d->phase));
        local_steps += (uint64_t)d->phase;
        d->phase ^= 1;
        --left;
    }
    if (d->stats_on)
        d->stats_samples += local_steps;
    return LBM_OK;
}

int lbm_step_wait(lbm_domain *d)
{
    if (int rc = check_domain(d))
        return rc;
    if (d->batch)
        return fail(LBM_ERR_STATE, "domain is resident in a batch");
    if (int rc = sync_status(d))
        return rc;
    if (d->unstable)
        return fail(LBM_ERR_UNSTABLE, "a step produced rho <= 0 or a non-finite value");
    return LBM_OK;
}

int lbm_step(lbm_domain *d, int n)
{
    if (int rc = lbm_step_async(d, n))
        return rc;
    if (d->ntiles == 0) // nothing is updated, the state stays as it is
        return LBM_OK;
    return lbm_step_wait(d);
}

int lbm_prepare_steps(lbm_domain *d)
{
    if (int rc = check_domain(d))
        return rc;
    if (d->batch)
        return fail(LBM_ERR_STATE, "domain is resident in a batch");
    if (d->ntiles && d->graph_dirty)
        return build_graph(d);
    return LBM_OK;
}

int lbm_get_moments_device(lbm_domain *d, float *rho_dev, float *u_dev)
{
    if (int rc = check_domain(d))
        return rc;
    if (!rho_dev || !u_dev)
        return fail(LBM_ERR_ARG, "null output");
    if (d->batch)
        return fail(LBM_ERR_STATE, "domain is resident in a batch");
    HIP_TRY(normalise(d));
    const KDomain k = kdomain(d);
    const uint32_t blocks = (uint32_t)((d->ncells + 255) / 256);
    dispatch_storage(d->storage, [&](auto st) {
        hipLaunchKernelGGL((k_moments<decltype(st)::value>), dim3(blocks), dim3(256), 0, d->stream, k, rho_dev,
                           u_dev);
    });
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(d->stream));
    return LBM_OK;
}

int lbm_get_moments_noalloc(lbm_domain *d, float *rho, float *u)
{
    if (int rc = check_domain(d))
        return rc;
    if (!rho || !u)
        return fail(LBM_ERR_ARG, "null output");
    if (d->batch)
        return fail(LBM_ERR_STATE, "domain is resident in a batch");
    if (d->ncells > kScratchFloats / 4)
        return fail(LBM_ERR_ARG, "domain of %llu cells exceeds the %llu cells of the static read-back buffer",
                    (unsigned long long)d->ncells, (unsigned long long)(kScratchFloats / 4));
    float *buf = nullptr;
    if (int rc = scratch_address(d->device, &buf))
        return rc;
    std::lock_guard<std::mutex> lock(g_scratch_mutex[d->device]);
    HIP_TRY(normalise(d));
    const KDomain k = kdomain(d);
    const uint32_t blocks = (uint32_t)((d->ncells + 255) / 256);
    dispatch_storage(d->storage, [&](auto st) {
        hipLaunchKernelGGL((k_moments<decltype(st)::value>), dim3(blocks), dim3(256), 0, d->stream, k, buf,
                           buf + d->ncells);
    });
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(rho, buf, d->ncells * sizeof(float), hipMemcpyDeviceToHost, d->stream));
    HIP_TRY(hipMemcpyAsync(u, buf + d->ncells, 3 * d->ncells * sizeof(float), hipMemcpyDeviceToHost, d->stream));
    HIP_TRY(hipStreamSynchronize(d->stream));
    return LBM_OK;
}

int lbm_get_moments(lbm_domain *d, float *rho, float *u)
{
    if (int rc = check_domain(d))
        return rc;
    if (!rho || !u)
        return fail(LBM_ERR_ARG, "null output");
    float *dr = nullptr;
    if (dalloc(d->stream, (void **)&dr, 4 * d->ncells * sizeof(float)) != hipSuccess)
        return fail(LBM_ERR_OOM, "staging buffer");
    int rc = lbm_get_moments_device(d, dr, dr + d->ncells);
    if (rc == LBM_OK &&
        (copy_sync(d->stream, rho, dr, d->ncells * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess ||
         copy_sync(d->stream, u, dr + d->ncells, 3 * d->ncells * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess))
        rc = fail(LBM_ERR_DEVICE, "download failed");
    dfree(d->stream, dr);
    return rc;
}

int lbm_get_populations(lbm_domain *d, float *f)
{
    if (int rc = check_domain(d))
        return rc;
    if (!f)
        return fail(LBM_ERR_ARG, "null output");
    if (d->batch)
        return fail(LBM_ERR_STATE, "domain is resident in a batch");
    HIP_TRY(normalise(d));
    float *df = nullptr;
    if (dalloc(d->stream, (void **)&df, (size_t)Q * d->ncells * sizeof(float)) != hipSuccess)
        return fail(LBM_ERR_OOM, "staging buffer");
    const KDomain k = kdomain(d);
    const uint32_t blocks = (uint32_t)((d->ncells + 255) / 256);
    dispatch_storage(d->storage, [&](auto st) {
        hipLaunchKernelGGL((k_export<decltype(st)::value>), dim3(blocks), dim3(256), 0, d->stream, k, df);
    });
    int rc = LBM_OK;
    if (hipGetLastError() != hipSuccess ||
        copy_sync(d->stream, f, df, (size_t)Q * d->ncells * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
        rc = fail(LBM_ERR_DEVICE, "population export failed");
    dfree(d->stream, df);
    return rc;
}

int lbm_set_populations(lbm_domain *d, const float *f)
{
    if (int rc = check_domain(d))
        return rc;
    if (!f)
        return fail(LBM_ERR_ARG, "null input");
    if (d->batch)
        return fail(LBM_ERR_STATE, "domain is resident in a batch");
    float *df = nullptr;
    if (dalloc(d->stream, (void **)&df, (size_t)Q * d->ncells * sizeof(float)) != hipSuccess)
        return fail(LBM_ERR_OOM, "staging buffer");
    int rc = LBM_OK;
    if (copy_sync(d->stream, df, f, (size_t)Q * d->ncells * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        rc = fail(LBM_ERR_DEVICE, "upload failed");
    if (rc == LBM_OK) {
        const KDomain k = kdomain(d);
        const uint32_t blocks = (uint32_t)((d->ncells + 255) / 256);
        dispatch_storage(d->storage, [&](auto st) {
            hipLaunchKernelGGL((k_import<decltype(st)::value>), dim3(blocks), dim3(256), 0, d->stream, k, df);
        });
        d->phase = 0;
        if (hipGetLastError() != hipSuccess || side_refresh(d) != hipSuccess || curved_refresh(d) != hipSuccess ||
            hipStreamSynchronize(d->stream) != hipSuccess)
            rc = fail(LBM_ERR_DEVICE, "population import failed");
    }
    dfree(d->stream, df);
    return rc;
}

namespace {

// State images (lbm_save_state): a header of eight uint64 words, then the
// population array, then the kept curved-wall values.
constexpr uint64_t kStateTag = 0x31544154534d424cull; // "LBMSTAT1", little-endian
constexpr size_t kStateHeader = 64;

uint64_t aux_bytes(const lbm_domain *d)
{
    return d->d_bzaux ? d->nwall * Q * 64 * sizeof(float) : 0;
}

void state_header(const lbm_domain *d, uint64_t (&h)[8])
{
    h[0] = kStateTag;
    h[1] = (uint64_t)d->nx | (uint64_t)d->ny << 16 | (uint64_t)d->nz << 32 | (uint64_t)d->periodic << 48 |
           (uint64_t)d->storage << 56;
    h[2] = d->bytes;
    h[3] = aux_bytes(d);
    h[4] = d->flags_hash;
    h[5] = (uint64_t)d->phase | (uint64_t)d->unstable << 1;
    h[6] = h[7] = 0;
}

} // namespace

int lbm_state_bytes(const lbm_domain *d, size_t *bytes)
{
    if (int rc = check_domain(d))
        return rc;
    if (!bytes)
        return fail(LBM_ERR_ARG, "null output");
    *bytes = kStateHeader + d->bytes + aux_bytes(d);
    return LBM_OK;
}

int lbm_save_state(lbm_domain *d, void *buf, size_t bytes)
{
    if (int rc = check_domain(d))
        return rc;
    if (!buf)
        return fail(LBM_ERR_ARG, "null buffer");
    if (d->batch)
        return fail(LBM_ERR_STATE, "domain is resident in a batch");
    const uint64_t aux = aux_bytes(d);
    if (bytes < kStateHeader + d->bytes + aux)
        return fail(LBM_ERR_ARG, "buffer of %zu bytes; the state takes %llu", bytes,
                    (unsigned long long)(kStateHeader + d->bytes + aux));
    uint64_t h[8];
    state_header(d, h);
    std::memcpy(buf, h, sizeof h);
    char *p = (char *)buf + kStateHeader;
    if (copy_sync(d->stream, p, d->buf, d->bytes, hipMemcpyDeviceToHost) != hipSuccess ||
        copy_sync(d->stream, p + d->bytes, d->d_bzaux, aux, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(LBM_ERR_DEVICE, "state download failed");
    return LBM_OK;
}

int lbm_load_state(lbm_domain *d, const void *buf, size_t bytes)
{
    if (int rc = check_domain(d))
        return rc;
    if (!buf)
        return fail(LBM_ERR_ARG, "null buffer");
    if (d->batch)
        return fail(LBM_ERR_STATE, "domain is resident in a batch");
    if (bytes < kStateHeader)
        return fail(LBM_ERR_ARG, "state image of %zu bytes is shorter than its header", bytes);
    uint64_t h[8], mine[8];
    std::memcpy(h, buf, sizeof h);
    state_header(d, mine);
    if (h[0] != kStateTag || h[6] != 0 || h[7] != 0 || h[5] > 3)
        return fail(LBM_ERR_ARG, "not a state image");
    if (h[1] != mine[1] || h[2] != mine[2])
        return fail(LBM_ERR_ARG, "state image of another grid, periodicity or storage");
    if (h[4] != mine[4])
        return fail(LBM_ERR_STATE, "state image of a domain with other flags");
    if (h[3] != mine[3])
        return fail(LBM_ERR_STATE, "state image %s curved walls and the domain %s", h[3] ? "has" : "has no",
                    mine[3] ? "has" : "has none");
    if (bytes != kStateHeader + h[2] + h[3])
        return fail(LBM_ERR_ARG, "state image of %zu bytes; its header gives %llu", bytes,
                    (unsigned long long)(kStateHeader + h[2] + h[3]));
    const char *p = (const char *)buf + kStateHeader;
    if (copy_sync(d->stream, d->buf, p, d->bytes, hipMemcpyHostToDevice) != hipSuccess ||
        copy_sync(d->stream, d->d_bzaux, p + d->bytes, h[3], hipMemcpyHostToDevice) != hipSuccess ||
        hipMemsetAsync(d->d_status, 0, sizeof(uint32_t), d->stream) != hipSuccess ||
        hipStreamSynchronize(d->stream) != hipSuccess)
        return fail(LBM_ERR_DEVICE, "state upload failed");
    d->phase = (int)(h[5] & 1u);
    d->unstable = (h[5] >> 1) != 0;
    return LBM_OK;
}

int lbm_stats_enable(lbm_domain *d, int on)
{
    if (int rc = check_domain(d))
        return rc;
    if (d->batch)
        return fail(LBM_ERR_STATE, "domain is resident in a batch");
    if (on) {
        const size_t bytes = (size_t)15 * d->ntiles * 64 * sizeof(double);
        if (!d->d_stats && bytes) {
            if (dalloc(d->stream, (void **)&d->d_stats, bytes) != hipSuccess)
                return fail(LBM_ERR_OOM, "statistics sums (%zu bytes)", bytes);
            d->device_bytes += bytes;
        }
        if (bytes)
            HIP_TRY(hipMemsetAsync(d->d_stats, 0, bytes, d->stream));
        HIP_TRY(hipStreamSynchronize(d->stream));
        d->stats_samples = 0;
    }
    d->stats_on = on != 0;
    d->graph_dirty = true;
    return LBM_OK;
}

int lbm_stats_get(lbm_domain *d, double *mean_u, double *mean_uu, double *mean_sigma, uint64_t *samples)
{
    if (int rc = check_domain(d))
        return rc;
    if (!mean_u || !mean_uu || !mean_sigma || !samples)
        return fail(LBM_ERR_ARG, "null output");
    if (d->batch)
        return fail(LBM_ERR_STATE, "domain is resident in a batch");
    *samples = d->stats_samples;
    const size_t n = d->ncells;
    double *dout = nullptr;
    if (dalloc(d->stream, (void **)&dout, 15 * n * sizeof(double)) != hipSuccess)
        return fail(LBM_ERR_OOM, "staging buffer");
    int rc = LBM_OK;
    if (hipMemsetAsync(dout, 0, 15 * n * sizeof(double), d->stream) != hipSuccess)
        rc = fail(LBM_ERR_DEVICE, "staging clear failed");
    if (rc == LBM_OK && d->d_stats && d->stats_samples && d->ntiles) {
        KDomain k = kdomain(d);
        k.stats = d->d_stats;
        const uint32_t blocks = (uint32_t)((d->ntiles + 3) / 4);
        hipLaunchKernelGGL(k_stats_export, dim3(blocks), dim3(256), 0, d->stream, k, (const TileRec *)d->d_tiles,
                           (uint32_t)d->ntiles, 1.0 / (double)d->stats_samples, dout);
        if (hipGetLastError() != hipSuccess)
            rc = fail(LBM_ERR_DEVICE, "statistics export failed");
    }
    if (rc == LBM_OK &&
        (copy_sync(d->stream, mean_u, dout, 3 * n * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess ||
         copy_sync(d->stream, mean_uu, dout + 3 * n, 6 * n * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess ||
         copy_sync(d->stream, mean_sigma, dout + 9 * n, 6 * n * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess))
        rc = fail(LBM_ERR_DEVICE, "statistics download failed");
    dfree(d->stream, dout);
    return rc;
}

int lbm_domain_get_info(const lbm_domain *d, lbm_domain_info *info)
{
    if (!d || !info)
        return fail(LBM_ERR_ARG, "null argument");
    info->nx = d->nx;
    info->ny = d->ny;
    info->nz = d->nz;
    info->storage = d->storage;
    info->periodic = d->periodic;
    info->ncells = d->ncells;
    info->plane_stride = d->P;
    info->n_updated = d->n_updated;
    info->n_tiles = d->ntiles;
    info->n_wall_tiles = d->nwall;
    info->n_inlet = d->inlet_cells.size();
    info->device_bytes = d->device_bytes;
    info->bytes_per_cell_update = 2ull * Q * storage_bytes(d->storage);

    return LBM_OK;
}

int lbm_destroy(lbm_domain *d)
{
    if (int rc = check_domain(d))
        return rc;
    if (d->batch)
        return fail(LBM_ERR_STATE, "domain is resident in a batch; release it first");
    (void)hipStreamSynchronize(d->stream);
    free_domain(d);
    return LBM_OK;
}

} // extern "C"

#include "lbm_batch.inc"
#include "lbm_selftest.inc"
