// lbm_device.hpp -- gfx950 kernels of the D3Q27 CHM-MRT lattice Boltzmann
// step (Huang, Noel, Berg, Hosseini, Sec. 2.1 and App. A).
//
// One lane updates one cell; one wave (64 lanes) updates one 64-cell tile of
// the linear cell index.  Each tile stores its 27 populations as 27
// contiguous 64-element rows, so the 27 stores of a wave are full-line
// writes and each load is one or two contiguous runs.  The whole moment
// transform runs in registers; the path is HBM-bound, so there is no LDS
// staging and no MFMA.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int Q = 27;
constexpr float kTheta0 = 1.0f / 3.0f; // stencil reference temperature
constexpr float kFp16Scale = 16384.0f; // 2^14: keeps f - w out of FP16 subnormals
constexpr float kFp16InvScale = 1.0f / 16384.0f;

enum : int { ST_FP32 = 0, ST_FP16S = 1, ST_BF16S = 2 };

// Launch shape and cache policy of the stream-collide kernels (tuned on
// MI355X; see the profiles).  Cache-policy bits of buffer instructions on
// gfx950: 1 sc0, 2 nt, 16 sc1.
#ifndef LBM_WAVES_PER_BLOCK
#define LBM_WAVES_PER_BLOCK 4
#endif
#ifndef LBM_LOAD_AUX
#define LBM_LOAD_AUX 0
#endif
#ifndef LBM_STORE_AUX
#define LBM_STORE_AUX 0
#endif
constexpr uint32_t kWavesPerBlock = LBM_WAVES_PER_BLOCK;
constexpr uint32_t kBlock = 64 * kWavesPerBlock;
enum : uint8_t { FL_FLUID = 0, FL_SOLID = 1, FL_INLET = 2, FL_OUTLET = 3 };

// wall-tile link mask of a cell: bits 0..26 halfway bounce-back for
// direction i, bit 30 the cell has moving-wall inlet links, bit 31 the cell
// is not updated.
constexpr uint32_t kMaskBB = (1u << Q) - 1;
constexpr uint32_t kMaskInlet = 1u << 30;
constexpr uint32_t kMaskSkip = 1u << 31;
// inlet record of a cell with moving-wall inlet links: word 0 the link mask,
// word 1 + i the ordinal of the inlet cell that link i comes from
constexpr uint32_t kRecWords = 28;
constexpr uint32_t kNoRec = 0xffffffffu;

// D3Q27 weights, product of the 1-D weights 2/3 (c = 0) and 1/6 (c = +-1)
// (App. A, Eqs. (A.1)-(A.2)); index i = (cx+1) + 3(cy+1) + 9(cz+1).
__host__ __device__ constexpr float weight(int i)
{
    return (((i % 3) == 1) ? 2.0f / 3.0f : 1.0f / 6.0f) * ((((i / 3) % 3) == 1) ? 2.0f / 3.0f : 1.0f / 6.0f) *
           (((i / 9) == 1) ? 2.0f / 3.0f : 1.0f / 6.0f);
}
__host__ __device__ constexpr int cx(int i) { return i % 3 - 1; }
__host__ __device__ constexpr int cy(int i) { return (i / 3) % 3 - 1; }
__host__ __device__ constexpr int cz(int i) { return i / 9 - 1; }

// Unsigned division by a run-time invariant divisor (round-up multiply
// method of Granlund and Montgomery): q = (t + ((n - t) >> s1)) >> s2 with
// t = umulhi(n, m).  Exact for every 32-bit n.
struct FastDiv {
    uint32_t m, s1, s2, d;
};

__host__ __device__ inline uint32_t fdiv(uint32_t n, FastDiv f)
{
#if defined(__HIP_DEVICE_COMPILE__)
    uint32_t t = __umulhi(n, f.m);
#else
    uint32_t t = (uint32_t)(((uint64_t)n * f.m) >> 32);
#endif
    return (t + ((n - t) >> f.s1)) >> f.s2;
}

// Everything a kernel needs to update one domain.
struct KDomain {
    char *buf[2];            // population buffers, 27 planes of P elements
    const uint32_t *wall;    // link masks of wall tiles, 64 per wall tile
    const float *iterm;      // inlet terms, [27][64] per inlet tile
    uint32_t *status;        // bit 0: a step went unstable
    uint32_t P;              // cells rounded up to whole tiles
    uint32_t tbytes;         // bytes of one tile block: 27 x 64 populations
    uint32_t bufbytes;       // bytes of one population buffer: (P / 64) tile blocks
    uint32_t nx, ny, nz, ncells;
    FastDiv dnx, dny;
    uint32_t periodic;
    float omega, omega_b, omega_h;
    // batched execution: the domain takes part in global steps
    // [step0, step0 + nsteps); its state at step0 is in buf[cur0].
    uint32_t step0, nsteps, cur0, pad;
};

// One entry of a tile list (32 bytes; a wave reads it with scalar loads).
// Everything the wave needs to issue its loads is here, so none of them
// waits for a per-cell table.
struct TileRec {
    uint32_t slot;   // domain slot in a packed launch (0 otherwise)
    uint32_t tile;   // cells [64 tile, 64 tile + 64)
    int32_t wall;    // wall-tile slot (per-cell link masks), -1 for an interior tile
    uint32_t bb;     // union of the cells' bounce-back links
    uint32_t inl;    // inlet-term block, kNoRec if no cell has an inlet link
    uint32_t inlm;   // union of the cells' inlet links
    uint32_t act[2]; // bit l of act[l / 32]: the cell of lane l is updated
};

// Tile-major population layout: the 27 populations of the 64 cells of a
// tile are one contiguous block, population i of the cell in lane l at
// byte tile * tbytes + (64 i + l) * es.  A wave writes one contiguous
// block, and reads each neighbouring row's three populations that share
// (cy, cz) as one contiguous run, which keeps HBM accesses long.
template <uint32_t ES> __device__ __forceinline__ uint32_t cell_bytes(uint32_t cell, uint32_t tbytes)
{
    return __umul24(cell >> 6, tbytes) + (cell & 63u) * ES;
}
template <uint32_t ES> constexpr uint32_t pop_bytes(int i) { return (uint32_t)i * 64u * ES; }

// Raw buffer resource over a population buffer (gfx9-family word 3).  Loads
// and stores go through buffer instructions: an SGPR resource, a 32-bit
// per-lane byte offset and a per-direction SGPR byte offset; a read past the
// buffer's size returns 0 instead of touching other memory.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const char *p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)p, (short)0, (int)bytes, 0x00020000);
}

template <int ST> struct Storage;
template <> struct Storage<ST_FP32> {
    using T = float;
    static constexpr uint32_t bytes = 4;
    __device__ static float load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, int)
    {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, LBM_LOAD_AUX));
    }
    __device__ static void store(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, float v, int)
    {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, LBM_STORE_AUX);
    }
    __device__ static float to_f(T v, int) { return v; }
    __device__ static T from_f(float v, int) { return v; }
    // stored bits, and their value for direction i
    __device__ static uint32_t raw(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
    {
        return __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, LBM_LOAD_AUX);
    }
    __device__ static float from_raw(uint32_t b, int) { return __uint_as_float(b); }
};
template <> struct Storage<ST_FP16S> {
    using T = _Float16;
    static constexpr uint32_t bytes = 2;
    __device__ static float load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, int i)
    {
        const uint16_t h = __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, LBM_LOAD_AUX);
        return to_f(__builtin_bit_cast(_Float16, h), i);
    }
    __device__ static void store(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, float v, int i)
    {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, from_f(v, i)), r, voff, soff, LBM_STORE_AUX);
    }
    __device__ static float to_f(T h, int i) { return __builtin_fmaf((float)h, kFp16InvScale, weight(i)); }
    // conversion to FP16 rounds to nearest even (v_cvt_f16_f32)
    __device__ static T from_f(float v, int i) { return (_Float16)((v - weight(i)) * kFp16Scale); }
    __device__ static uint32_t raw(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
    {
        return __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, LBM_LOAD_AUX);
    }
    __device__ static float from_raw(uint32_t b, int i) { return to_f(__builtin_bit_cast(_Float16, (uint16_t)b), i); }
};
template <> struct Storage<ST_BF16S> {
    using T = uint16_t;
    static constexpr uint32_t bytes = 2;
    __device__ static float load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, int i)
    {
        return to_f(__builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, LBM_LOAD_AUX), i);
    }
    __device__ static void store(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, float v, int i)
    {
        __builtin_amdgcn_raw_buffer_store_b16(from_f(v, i), r, voff, soff, LBM_STORE_AUX);
    }
    __device__ static float to_f(T h, int i) { return __uint_as_float((uint32_t)h << 16) + weight(i); }
    __device__ static uint32_t raw(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
    {
        return __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, LBM_LOAD_AUX);
    }
    __device__ static float from_raw(uint32_t b, int i) { return to_f((uint16_t)b, i); }
    // round to nearest even on the upper 16 bits (finite inputs)
    __device__ static T from_f(float v, int i)
    {
        uint32_t b = __float_as_uint(v - weight(i));
        b += 0x7fffu + ((b >> 16) & 1u);
        return (uint16_t)(b >> 16);
    }
};

// ---------------------------------------------------------------------------
// Collision: f <- T(u)^-1 M*, M = T(u) f (Sec. 2.1, Eqs. (6)-(8)).
//
// T(u) is the tensor product of three 1-D maps (one per axis) taking the
// populations at c = -1, 0, +1 to the central Hermite moments of orders
// 0, 1, 2 about u: {1, xi, xi^2 - theta0} at xi = c - u.  The forward
// transform is three sweeps of that 1-D map over 9 triples each, the inverse
// three sweeps of its closed-form inverse.  Slot k = a + 3 b + 9 c holds
// population (a-1, b-1, c-1) before the transform and moment x^a y^b z^c
// after it.  The equilibrium is implicit: with the full expansion the
// central moments of f^eq are (rho, 0, ..., 0) (App. A, Eqs. (A.5)-(A.6)),
// so relaxing towards it scales each non-conserved moment by (1 - rate).
// ---------------------------------------------------------------------------
template <bool HIGH1>
__device__ __forceinline__ float collide(float (&f)[Q], float omega, float omega_b, float omega_h, float &ux,
                                         float &uy, float &uz)
{
    // x sweep, raw: s0 = sum, s1 = first moment, s2 = second moment
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const float A = f[3 * t], B = f[3 * t + 1], C = f[3 * t + 2];
        f[3 * t] = A + B + C;
        f[3 * t + 1] = C - A;
        f[3 * t + 2] = C + A;
    }
    float rho = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        rho += f[3 * t];
        jx += f[3 * t + 1];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
        jy += f[3 * (3 * c + 2)] - f[3 * (3 * c + 0)];
#pragma unroll
    for (int b = 0; b < 3; ++b)
        jz += f[3 * (b + 6)] - f[3 * b];
    const float inv = __builtin_amdgcn_rcpf(rho);
    ux = jx * inv;
    uy = jy * inv;
    uz = jz * inv;
    // x sweep, shift to central moments about ux
    {
        const float k2 = ux * ux - kTheta0, tu = 2.f * ux;
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const float s0 = f[3 * t], s1 = f[3 * t + 1], s2 = f[3 * t + 2];
            f[3 * t + 1] = __builtin_fmaf(-ux, s0, s1);
            f[3 * t + 2] = __builtin_fmaf(k2, s0, __builtin_fmaf(-tu, s1, s2));
        }
    }
    // y and z sweeps
#define LBM_FWD_SWEEP(U, STRIDE, OUTER)                                                                          \
    {                                                                                                            \
        const float k2 = U * U - kTheta0, tu = 2.f * U;                                                          \
        _Pragma("unroll") for (int t = 0; t < 9; ++t)                                                            \
        {                                                                                                        \
            const int base = OUTER(t);                                                                           \
            const float A = f[base], B = f[base + STRIDE], C = f[base + 2 * STRIDE];                             \
            const float s0 = A + B + C, s1 = C - A, s2 = C + A;                                                  \
            f[base] = s0;                                                                                        \
            f[base + STRIDE] = __builtin_fmaf(-U, s0, s1);                                                       \
            f[base + 2 * STRIDE] = __builtin_fmaf(k2, s0, __builtin_fmaf(-tu, s1, s2));                          \
        }                                                                                                        \
    }
#define LBM_OUTER_Y(t) (((t) % 3) + 9 * ((t) / 3))
#define LBM_OUTER_Z(t) (t)
    LBM_FWD_SWEEP(uy, 3, LBM_OUTER_Y)
    LBM_FWD_SWEEP(uz, 9, LBM_OUTER_Z)

    // relaxation (Sec. 2.1 after Eq. (8); App. A after Eq. (A.6)):
    // order 0 and 1 conserved; second order: deviator and off-diagonal at
    // omega, trace at omega_b; order >= 3 at omega_h.
    const float ks = 1.f - omega, kb = 1.f - omega_b, kh = 1.f - omega_h;
    f[4] *= ks;
    f[10] *= ks;
    f[12] *= ks;
    {
        const float tr = (f[2] + f[6] + f[18]) * (1.0f / 3.0f);
        const float d = (kb - ks) * tr;
        f[2] = __builtin_fmaf(ks, f[2], d);
        f[6] = __builtin_fmaf(ks, f[6], d);
        f[18] = __builtin_fmaf(ks, f[18], d);
    }
    constexpr int high[17] = {5, 7, 8, 11, 13, 14, 15, 16, 17, 19, 20, 21, 22, 23, 24, 25, 26};
#pragma unroll
    for (int k = 0; k < 17; ++k)
        f[high[k]] = HIGH1 ? 0.f : f[high[k]] * kh;

    // inverse sweeps z, y, x: raw moments R0 = m0, R1 = m1 + u m0,
    // R2 = m2 + 2 u m1 + (u^2 + theta0) m0; then f(+1) = (R2 + R1)/2,
    // f(-1) = (R2 - R1)/2, f(0) = R0 - R2.
#define LBM_INV_SWEEP(U, STRIDE, OUTER)                                                                          \
    {                                                                                                            \
        const float k2 = U * U + kTheta0, tu = 2.f * U;                                                          \
        _Pragma("unroll") for (int t = 0; t < 9; ++t)                                                            \
        {                                                                                                        \
            const int base = OUTER(t);                                                                           \
            const float m0 = f[base], m1 = f[base + STRIDE], m2 = f[base + 2 * STRIDE];                          \
            const float R1 = __builtin_fmaf(U, m0, m1);                                                          \
            const float R2 = __builtin_fmaf(k2, m0, __builtin_fmaf(tu, m1, m2));                                 \
            f[base] = 0.5f * (R2 - R1);                                                                          \
            f[base + STRIDE] = m0 - R2;                                                                          \
            f[base + 2 * STRIDE] = 0.5f * (R2 + R1);                                                             \
        }                                                                                                        \
    }
#define LBM_OUTER_X(t) (3 * (t))
    LBM_INV_SWEEP(uz, 9, LBM_OUTER_Z)
    LBM_INV_SWEEP(uy, 3, LBM_OUTER_Y)
    LBM_INV_SWEEP(ux, 1, LBM_OUTER_X)
#undef LBM_FWD_SWEEP
#undef LBM_INV_SWEEP
#undef LBM_OUTER_X
#undef LBM_OUTER_Y
#undef LBM_OUTER_Z
    return rho;
}

// ---------------------------------------------------------------------------
// One wave updates one 64-cell tile: pull gather with boundary resolution,
// collision, store (Sec. 2.1, Eq. (6); boundary rules of Sec. 2.2).
// ---------------------------------------------------------------------------
template <int ST, bool HIGH1>
__device__ __forceinline__ void update_tile(const KDomain &d, const TileRec &rec, uint32_t src_idx, uint32_t lane)
{
    using S = Storage<ST>;
    constexpr uint32_t es = S::bytes;
    const auto rs = make_rsrc(d.buf[src_idx], d.bufbytes);
    const auto rd = make_rsrc(d.buf[src_idx ^ 1u], d.bufbytes);
    const uint32_t lin = rec.tile * 64u + lane;
    const bool active = ((lane < 32u ? rec.act[0] : rec.act[1]) >> (lane & 31u)) & 1u;

    // cell coordinates and the source coordinates per velocity component:
    // index 0 is the source of c = -1 (x + 1), 1 of c = 0, 2 of c = +1.
    // Periodic axes wrap; other axes clamp to the box (a clamped source is
    // either the zero-gradient outlet's or a bounce-back link's).
    const uint32_t q = fdiv(lin, d.dnx);
    const uint32_t x = lin - q * d.nx;
    const uint32_t z = fdiv(q, d.dny);
    const uint32_t y = q - z * d.ny;
    const bool px = d.periodic & 1u, py = d.periodic & 2u, pz = d.periodic & 4u;
    uint32_t sx[3], sy[3], sz[3];
    sx[1] = x;
    sx[0] = (x + 1 < d.nx) ? x + 1 : (px ? 0u : x);
    sx[2] = (x > 0) ? x - 1 : (px ? d.nx - 1 : 0u);
    sy[1] = y;
    sy[0] = (y + 1 < d.ny) ? y + 1 : (py ? 0u : y);
    sy[2] = (y > 0) ? y - 1 : (py ? d.ny - 1 : 0u);
    sz[1] = z;
    sz[0] = (z + 1 < d.nz) ? z + 1 : (pz ? 0u : z);
    sz[2] = (z > 0) ? z - 1 : (pz ? d.nz - 1 : 0u);
    // first cell of each source row (cy, cz)
    uint32_t row[9];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            row[b + 3 * c] = (sz[c] * d.ny + sy[b]) * d.nx;

    float f[Q];
    if (rec.wall < 0) {
        // interior tile: every cell is updated and every link is a pull
#pragma unroll
        for (int i = 0; i < Q; ++i)
            f[i] = S::load(rs, cell_bytes<es>(row[i / 3] + sx[i % 3], d.tbytes), pop_bytes<es>(i), i);
    } else {
        if (!active)
            return;
        // Bounce-back links take the cell's own opposite population (+ the
        // moving-wall term of an inlet link).  The tile entry says which
        // directions any cell of the tile bounces back; for those the wave
        // loads both candidates, for the others the own load is given an
        // offset past the end of the buffer, which returns 0 without a
        // memory access.  All loads are issued before the per-cell mask is
        // needed; it selects between stored bits (opposite directions share
        // their weight, so one conversion serves both candidates).
        const uint32_t m = d.wall[(uint32_t)rec.wall * 64u + lane];
        const uint32_t self = cell_bytes<es>(lin, d.tbytes);
        uint32_t p[Q], o[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i)
            p[i] = S::raw(rs, cell_bytes<es>(row[i / 3] + sx[i % 3], d.tbytes), pop_bytes<es>(i));
#pragma unroll
        for (int i = 0; i < Q; ++i)
            o[i] = S::raw(rs, ((rec.bb >> i) & 1u) ? self : d.bufbytes, pop_bytes<es>(Q - 1 - i));
#pragma unroll
        for (int i = 0; i < Q; ++i)
            f[i] = S::from_raw(((m >> i) & 1u) ? o[i] : p[i], i);
        if (rec.inlm) {
            // the term block holds 0 for links that are not inlet links
            constexpr uint32_t kTermBytes = Q * 64u * 4u;
            const auto rt = make_rsrc((const char *)(d.iterm + (size_t)rec.inl * (Q * 64u)), kTermBytes);
#pragma unroll
            for (int i = 0; i < Q; ++i)
                f[i] += __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
                    rt, ((rec.inlm >> i) & 1u) ? lane * 4u : kTermBytes, (uint32_t)i * 256u, 0));
        }
    }

    float ux, uy, uz;
    const float rho = collide<HIGH1>(f, d.omega, d.omega_b, d.omega_h, ux, uy, uz);
    if (!(rho > 0.f) || !(__builtin_fabsf(ux) + __builtin_fabsf(uy) + __builtin_fabsf(uz) < 1e30f))
        atomicOr(d.status, 1u);

    const uint32_t own = cell_bytes<es>(lin, d.tbytes);
#pragma unroll
    for (int i = 0; i < Q; ++i)
        S::store(rd, own, pop_bytes<es>(i), f[i], i);
}

// Inlet terms of the inlet tiles: for inlet link i of a cell, the moving-
// wall term 2 w_i (c_i . u_in) / theta0 with wall density 1 and u_in at the
// inlet cell the link comes from (Sec. 2.2); 0 for every other link and for
// every link when no inlet velocity is set.  One wave per tile entry.
__global__ __launch_bounds__(256) void k_inlet_terms(const TileRec *__restrict__ tiles, uint32_t ntiles,
                                                     const uint32_t *__restrict__ inlet,
                                                     const uint32_t *__restrict__ inlrec,
                                                     const float *__restrict__ uin, uint32_t n_inlet,
                                                     float *__restrict__ iterm)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t t = __builtin_amdgcn_readfirstlane(blockIdx.x * 4u + (threadIdx.x >> 6));
    if (t >= ntiles)
        return;
    const TileRec rec = tiles[t];
    if (rec.inl == kNoRec)
        return;
    const uint32_t r = inlet[(uint32_t)rec.wall * 64u + lane];
    const uint32_t *R = r == kNoRec ? nullptr : inlrec + (size_t)r * kRecWords;
    float *out = iterm + (size_t)rec.inl * (Q * 64u) + lane;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        float v = 0.f;
        if (R && uin && (R[0] & (1u << i))) {
            const uint32_t k = R[1 + i];
            const float cu = (float)cx(i) * uin[k] + (float)cy(i) * uin[n_inlet + k] +
                             (float)cz(i) * uin[2u * n_inlet + k];
            v = 6.0f * weight(i) * cu;
        }
        out[i * 64] = v;
    }
}

// Block index -> logical block: consecutive hardware blocks go round-robin
// to the 8 XCDs; give each XCD a contiguous range of tiles so that the cache
// lines shared by neighbouring tiles meet in the same L2.  G is a multiple
// of 8.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t G) { return (b & 7u) * (G >> 3) + (b >> 3); }

// Single-domain step.  Each wave takes whole tiles, walking the tile list
// with a stride of the grid's wave count (one pass when the grid covers
// every tile).
template <int ST, bool HIGH1>
__global__ __launch_bounds__(kBlock) void k_stream_collide(KDomain d, const TileRec *__restrict__ tiles,
                                                           uint32_t ntiles, uint32_t src_idx)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t nw = gridDim.x * kWavesPerBlock;
    const uint32_t w0 =
        __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + (threadIdx.x >> 6));
    for (uint32_t t = w0; t < ntiles; t += nw) {
        const TileRec rec = tiles[t];
        update_tile<ST, HIGH1>(d, rec, src_idx, lane);
    }
}

// Packed multi-domain step.  ctrl[0] = number of tile records, ctrl[1] =
// global step.  One wave per tile record (the host keeps the grid at least
// as large as the table); each tile belongs to one domain, whose descriptor
// says whether it takes part in this step.
template <int ST, bool HIGH1>
__global__ __launch_bounds__(kBlock) void k_stream_collide_batched(const KDomain *__restrict__ doms,
                                                                const TileRec *__restrict__ tiles,
                                                                const uint32_t *__restrict__ ctrl)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t ntiles = ctrl[0], g = ctrl[1];
    const uint32_t nw = gridDim.x * kWavesPerBlock;
    const uint32_t w0 =
        __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + (threadIdx.x >> 6));
    for (uint32_t t = w0; t < ntiles; t += nw) {
        const TileRec rec = tiles[t];
        const KDomain &dd = doms[rec.slot];
        const uint32_t k = g - dd.step0;
        if (k >= dd.nsteps)
            continue;
        const uint32_t s = (dd.cur0 + k) & 1u;
        update_tile<ST, HIGH1>(dd, rec, s, lane);
    }
}

__global__ void k_advance_step(uint32_t *ctrl)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        ctrl[1] = ctrl[1] + 1u;
}

// f = f^eq(rho, u) in product form: the sixth-order Hermite equilibrium of
// Eq. (4) factorises into rho prod_a phi(c_a, u_a), phi(0, u) = 2/3 - u^2,
// phi(+-1, u) = (1 +- 3u + 3u^2)/6 (App. A, Eqs. (A.2)-(A.4)).
template <int ST>
__global__ __launch_bounds__(256) void k_init_eq(KDomain d, const uint8_t *__restrict__ flags,
                                                 const float *__restrict__ rho, const float *__restrict__ u,
                                                 uint32_t dst_idx)
{
    using S = Storage<ST>;
    constexpr uint32_t es = S::bytes;
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.P)
        return;
    float r = 1.f, v[3] = {0.f, 0.f, 0.f};
    bool upd = false;
    if (c < d.ncells) {
        upd = flags[c] == FL_FLUID || flags[c] == FL_OUTLET;
        if (upd) {
            if (rho)
                r = rho[c];
            if (u) {
                v[0] = u[c];
                v[1] = u[d.ncells + c];
                v[2] = u[2u * d.ncells + c];
            }
        }
    }
    float phi[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float w = v[a], w2 = w * w;
        phi[a][0] = (1.f - 3.f * w + 3.f * w2) * (1.0f / 6.0f);
        phi[a][1] = 2.0f / 3.0f - w2;
        phi[a][2] = (1.f + 3.f * w + 3.f * w2) * (1.0f / 6.0f);
    }
    const uint32_t cb = cell_bytes<es>(c, d.tbytes);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const float fe = upd ? r * phi[0][i % 3] * phi[1][(i / 3) % 3] * phi[2][i / 9] : weight(i);
        *(typename S::T *)(d.buf[dst_idx] + cb + pop_bytes<es>(i)) = S::from_f(fe, i);
    }
}

template <int ST> __device__ __forceinline__ const typename Storage<ST>::T *pop_at(const char *buf, uint32_t cb, int i)
{
    return (const typename Storage<ST>::T *)(buf + cb + pop_bytes<Storage<ST>::bytes>(i));
}

// Density and velocity of the stored state at updated cells.
template <int ST>
__global__ __launch_bounds__(256) void k_moments(KDomain d, const uint8_t *__restrict__ flags, uint32_t cur,
                                                 float *__restrict__ rho, float *__restrict__ u)
{
    using S = Storage<ST>;
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.ncells)
        return;
    float r = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
    if (flags[c] == FL_FLUID || flags[c] == FL_OUTLET) {
        const uint32_t cb = cell_bytes<S::bytes>(c, d.tbytes);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const float fi = S::to_f(*pop_at<ST>(d.buf[cur], cb, i), i);
            r += fi;
            jx += (float)cx(i) * fi;
            jy += (float)cy(i) * fi;
            jz += (float)cz(i) * fi;
        }
        const float inv = 1.0f / r;
        jx *= inv;
        jy *= inv;
        jz *= inv;
    }
    rho[c] = r;
    u[c] = jx;
    u[d.ncells + c] = jy;
    u[2u * d.ncells + c] = jz;
}

// Stored populations <-> FP32 values of f_i, layout [i][cell] without padding.
template <int ST>
__global__ __launch_bounds__(256) void k_export(KDomain d, uint32_t cur, float *__restrict__ out)
{
    using S = Storage<ST>;
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.ncells)
        return;
    const uint32_t cb = cell_bytes<S::bytes>(c, d.tbytes);
#pragma unroll
    for (int i = 0; i < Q; ++i)
        out[(size_t)i * d.ncells + c] = S::to_f(*pop_at<ST>(d.buf[cur], cb, i), i);
}

template <int ST>
__global__ __launch_bounds__(256) void k_import(KDomain d, uint32_t cur, const float *__restrict__ in)
{
    using S = Storage<ST>;
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.ncells)
        return;
    const uint32_t cb = cell_bytes<S::bytes>(c, d.tbytes);
#pragma unroll
    for (int i = 0; i < Q; ++i)
        *(typename S::T *)(d.buf[cur] + cb + pop_bytes<S::bytes>(i)) = S::from_f(in[(size_t)i * d.ncells + c], i);
}

} // namespace lbm
