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

// Launch shape and cache policy of the stream-collide kernels (tuned by
// measurement on MI355X).  Cache-policy bits of buffer instructions on
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
#ifndef LBM_SETPRIO
#define LBM_SETPRIO 3
#endif
constexpr uint32_t kWavesPerBlock = LBM_WAVES_PER_BLOCK;

// Wave priority while a wave issues its loads (LBM_SETPRIO > 0), back to 0
// for the collision, so that waves starting a tile get their loads out
// ahead of the collisions of the waves already resident (about 1 % on the
// benchmark nozzle).
__device__ __forceinline__ void prio_loads()
{
    if constexpr (LBM_SETPRIO > 0)
        __builtin_amdgcn_s_setprio(LBM_SETPRIO);
}
__device__ __forceinline__ void prio_compute()
{
    if constexpr (LBM_SETPRIO > 0)
        __builtin_amdgcn_s_setprio(0);
}
constexpr uint32_t kBlock = 64 * kWavesPerBlock;
enum : uint8_t { FL_FLUID = 0, FL_SOLID = 1, FL_INLET = 2, FL_OUTLET = 3 };

// wall-tile link mask of a cell: bit i (0..26) halfway bounce-back for
// direction i, bit 29 the cell is an outlet cell, bit 30 the cell has
// moving-wall inlet links, bit 31 the cell is not updated.
constexpr uint32_t kMaskOutlet = 1u << 29;
constexpr uint32_t kMaskInlet = 1u << 30;
constexpr uint32_t kMaskSkip = 1u << 31;

// Step-kernel variants: bit 0 -- every rate of order >= 3 is 1 (the
// reduced collision); bit 1 -- curved walls (interpolated bounce-back);
// bit 2 -- constant-pressure outlet; bit 3 -- explicit equilibrium
// truncated below the full expansion (never with bit 0).  Domains without
// an option run kernels compiled without its code (fewer registers, more
// waves).
constexpr int kVarH1 = 1, kVarCurved = 2, kVarPressure = 4, kVarFeq = 8, kVariants = 16;
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
    char *buf;               // the population array: P / 64 tile blocks, then the outlet side rows
    const uint8_t *flags;    // cell flags
    const uint32_t *wall;    // link masks of wall tiles, 64 per wall tile
    const float *iterm;      // inlet terms, [27][64] per inlet tile
    uint32_t *status;        // bit 0: a step went unstable
    uint64_t side;           // byte offset of the side rows: 2 x 9 rows of ny * nz elements
    uint32_t P;              // cells rounded up to whole tiles
    uint32_t tbytes;         // bytes of one tile block: 27 x 64 populations
    uint32_t bufbytes;       // bytes of the whole array (below 4 GiB; see Pops)
    uint32_t nx, ny, nz, ncells;
    FastDiv dnx, dny;
    uint32_t periodic;
    float omega, omega_b;
    float omega_o[4];        // rates of the central moments of order 3, 4, 5, 6
    double *stats;           // statistics sums [15][sstride] (see local_finish), or null
    uint32_t sstride;        // 64 x number of tiles
    // batched execution: the domain takes part in global steps
    // [step0, step0 + nsteps), starting in phase ph0.
    uint32_t step0, nsteps, ph0, pad;
    uint32_t outlet;         // 0: zero-gradient outlet, 1: constant pressure rho_out / 3 (kernel variant kVarPressure)
    uint32_t high1;          // every rate of order >= 3 is one (see collide_lane)
    float rho_out;
    const float2 *bzc;       // curved-wall coefficients, [27][64] per wall tile (see curved_walls)
    float *bzaux;            // f*_k of the lanes' previous step, [27][64] per wall tile
    uint32_t rowtiles;       // nx / 64 when nx is a multiple of 64 (stream_tile_rows), else 0
    FastDiv drow;            // division by rowtiles
    uint32_t feq_order;      // 2..5: explicit equilibrium truncated at that order (variant kVarFeq); 6: full
};

// One entry of a tile list (40 bytes; a wave reads it with scalar loads).
// An interior tile needs nothing else; a wall tile adds one 32-bit link
// mask per lane (KDomain::wall).
struct TileRec {
    uint32_t slot;   // domain slot in a packed launch (0 otherwise)
    uint32_t tile;   // cells [64 tile, 64 tile + 64)
    int32_t wall;    // wall-tile slot (per-cell link masks), -1 for an interior tile
    uint32_t inl;    // inlet-term block, kNoRec if no cell has an inlet link
    uint32_t inlm;   // union of the cells' inlet links
    uint32_t act[2]; // bit l of act[l / 32]: the cell of lane l is updated
    uint32_t edge;   // 1: an updated cell of the tile lies on the outlet plane x = nx - 1
    uint32_t ord;    // position of the tile in its domain's tile list
    uint32_t bz;     // links with a curved-wall coefficient in some cell of the tile
};
static_assert(sizeof(TileRec) == 40, "tile record layout");

// Tile-major population layout: the 27 populations of the 64 cells of a
// tile are one contiguous block, population i of the cell in lane l at
// byte tile * tbytes + (64 i + l) * es.  A wave writes one contiguous
// block, and reads each neighbouring row's three populations that share
// (cy, cz) as one contiguous run, which keeps HBM accesses long.
template <uint32_t ES, class Off = uint32_t> __device__ __forceinline__ Off cell_bytes(uint32_t cell, uint32_t tbytes)
{
    if constexpr (sizeof(Off) == 4)
        return __umul24(cell >> 6, tbytes) + (cell & 63u) * ES;
    else
        return (uint64_t)(cell >> 6) * tbytes + (cell & 63u) * ES;
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
    __device__ static uint32_t to_raw(float v, int) { return __float_as_uint(v); }
    __device__ static void store_raw(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, uint32_t b)
    {
        __builtin_amdgcn_raw_buffer_store_b32(b, r, voff, soff, LBM_STORE_AUX);
    }
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
    __device__ static uint32_t to_raw(float v, int i) { return __builtin_bit_cast(uint16_t, from_f(v, i)); }
    __device__ static void store_raw(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, uint32_t b)
    {
        __builtin_amdgcn_raw_buffer_store_b16((uint16_t)b, r, voff, soff, LBM_STORE_AUX);
    }
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
    __device__ static uint32_t to_raw(float v, int i) { return from_f(v, i); }
    __device__ static void store_raw(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, uint32_t b)
    {
        __builtin_amdgcn_raw_buffer_store_b16((uint16_t)b, r, voff, soff, LBM_STORE_AUX);
    }
    // round to nearest even on the upper 16 bits (finite inputs)
    __device__ static T from_f(float v, int i)
    {
        uint32_t b = __float_as_uint(v - weight(i));
        b += 0x7fffu + ((b >> 16) & 1u);
        return (uint16_t)(b >> 16);
    }
};

// Access to a domain's population array at byte offset v + s, v per lane and
// s wave-uniform.  Arrays below 4 GiB take raw buffer instructions (v the
// lane offset, s the instruction's scalar offset).  Buffer addressing forms
// its offset sum in 32 bits, structured or raw, so it cannot reach past
// 4 GiB from the base: larger arrays (W64) take global instructions on
// 64-bit addresses buf + s + v, whose uniform part stays in scalar
// registers.  The kernels compile once for each.
template <int ST, bool W64> struct Pops;
template <int ST> struct Pops<ST, false> {
    using S = Storage<ST>;
    using Off = uint32_t;
    __amdgpu_buffer_rsrc_t r;
    __device__ explicit Pops(const KDomain &d) : r(make_rsrc(d.buf, d.bufbytes)) {}
    __device__ float load(Off v, Off s, int i) const { return S::load(r, v, s, i); }
    __device__ void store(Off v, Off s, float x, int i) const { S::store(r, v, s, x, i); }
    __device__ uint32_t raw(Off v, Off s) const { return S::raw(r, v, s); }
    __device__ void store_raw(Off v, Off s, uint32_t b) const { S::store_raw(r, v, s, b); }
};
template <int ST> struct Pops<ST, true> {
    using S = Storage<ST>;
    using Off = uint64_t;
    char *b;
    __device__ explicit Pops(const KDomain &d) : b(d.buf) {}
    __device__ uint32_t raw(Off v, Off s) const
    {
        if constexpr (S::bytes == 4)
            return *(const uint32_t *)(b + s + v);
        else
            return *(const uint16_t *)(b + s + v);
    }
    __device__ void store_raw(Off v, Off s, uint32_t x) const
    {
        if constexpr (S::bytes == 4)
            *(uint32_t *)(b + s + v) = x;
        else
            *(uint16_t *)(b + s + v) = (uint16_t)x;
    }
    __device__ float load(Off v, Off s, int i) const { return S::from_raw(raw(v, s), i); }
    __device__ void store(Off v, Off s, float x, int i) const { store_raw(v, s, S::to_raw(x, i)); }
};

// j / rho from inv = rcp(rho): the product j inv, corrected by one residual
// step (q + (j - rho q) inv), which rounds to within an ulp with no
// preferred sign.
__device__ __forceinline__ float quotient(float j, float rho, float inv)
{
    const float q = j * inv;
    return __builtin_fmaf(__builtin_fmaf(-rho, q, j), inv, q);
}

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
// Collision with omega_high = 1: every central moment of order >= 3 is set
// to zero, so the post-collision state depends only on rho, u and the six
// second-order central moments.  Those come straight from raw sums of f
// (M_ab = S_ab - rho u_a u_b - theta0 rho delta_ab, S_ab = sum c_a c_b f),
// without the full forward transform; the first-order central moments are
// zero by definition of u.  The inverse is the same three sweeps as below,
// over the ten moments that are left.
__device__ __forceinline__ float collide_h1(float (&f)[Q], float omega, float omega_b, float &ux, float &uy,
                                            float &uz, float (&m2)[6])
{
    // per (c_y, c_z) row t = b + 3c: s0 = sum over c_x, s1 = first, s2 = second moment in x
    float s0[9], s1[9], s2[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const float A = f[3 * t], B = f[3 * t + 1], C = f[3 * t + 2];
        s0[t] = A + B + C;
        s1[t] = C - A;
        s2[t] = C + A;
    }
    float rho = 0.f, jx = 0.f, sxx = 0.f;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        rho += s0[t];
        jx += s1[t];
        sxx += s2[t];
    }
    // rows with c_y = -1: t = 3c; c_y = +1: t = 2 + 3c; c_z = -1: t = b; c_z = +1: t = b + 6
    float jy = 0.f, syy = 0.f, sxy = 0.f, jz = 0.f, szz = 0.f, sxz = 0.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        jy += s0[2 + 3 * c] - s0[3 * c];
        syy += s0[2 + 3 * c] + s0[3 * c];
        sxy += s1[2 + 3 * c] - s1[3 * c];
    }
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        jz += s0[b + 6] - s0[b];
        szz += s0[b + 6] + s0[b];
        sxz += s1[b + 6] - s1[b];
    }
    const float syz = (s0[8] + s0[0]) - (s0[6] + s0[2]);
    // This form drops the first central moments (zero by definition of u),
    // so the momentum it hands on is rho u: u must be j / rho to within a
    // rounding of either sign.  j times a rounded 1 / rho errs to one side
    // for densities near 1 (about 1e-8 relative per step, which a long run
    // accumulates); one residual step per component removes that.
    const float inv = __builtin_amdgcn_rcpf(rho);
    ux = quotient(jx, rho, inv);
    uy = quotient(jy, rho, inv);
    uz = quotient(jz, rho, inv);
    // central second-order Hermite moments, relaxed: off-diagonal and
    // deviator at omega, trace at omega_b (Sec. 2.1 after Eq. (8))
    const float ks = 1.f - omega, kb = 1.f - omega_b;
    const float tr0 = kTheta0 * rho;
    float mxx = __builtin_fmaf(-jx, ux, sxx) - tr0;
    float myy = __builtin_fmaf(-jy, uy, syy) - tr0;
    float mzz = __builtin_fmaf(-jz, uz, szz) - tr0;
    m2[0] = mxx;
    m2[1] = myy;
    m2[2] = mzz;
    m2[3] = __builtin_fmaf(-jx, uy, sxy);
    m2[4] = __builtin_fmaf(-jx, uz, sxz);
    m2[5] = __builtin_fmaf(-jy, uz, syz);
    const float mxy = ks * m2[3];
    const float mxz = ks * m2[4];
    const float myz = ks * m2[5];
    {
        const float d = (kb - ks) * ((mxx + myy + mzz) * (1.0f / 3.0f));
        mxx = __builtin_fmaf(ks, mxx, d);
        myy = __builtin_fmaf(ks, myy, d);
        mzz = __builtin_fmaf(ks, mzz, d);
    }
#pragma unroll
    for (int k = 0; k < Q; ++k)
        f[k] = 0.f;
    f[0] = rho;
    f[2] = mxx;
    f[6] = myy;
    f[18] = mzz;
    f[4] = mxy;
    f[10] = mxz;
    f[12] = myz;
    return rho;
}

// Raw x sweep: per (c_y, c_z) row t = b + 3 c, slots 3t, 3t+1, 3t+2 take
// the zeroth, first and second raw moments in x of the row.
__device__ __forceinline__ void x_sweep_raw(float (&f)[Q])
{
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const float A = f[3 * t], B = f[3 * t + 1], C = f[3 * t + 2];
        f[3 * t] = A + B + C;
        f[3 * t + 1] = C - A;
        f[3 * t + 2] = C + A;
    }
}

// From the raw x sweep to the central Hermite moments about (ux, uy, uz):
// the x moments shifted to central ones, then the y and z sweeps.
__device__ __forceinline__ void central_sweeps(float (&f)[Q], float ux, float uy, float uz)
{
    {
        const float k2 = ux * ux - kTheta0, tu = 2.f * ux;
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const float s0 = f[3 * t], s1 = f[3 * t + 1], s2 = f[3 * t + 2];
            f[3 * t + 1] = __builtin_fmaf(-ux, s0, s1);
            f[3 * t + 2] = __builtin_fmaf(k2, s0, __builtin_fmaf(-tu, s1, s2));
        }
    }
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
#undef LBM_FWD_SWEEP
}

// Relaxation of the central moments (Sec. 2.1 after Eq. (8); App. A after
// Eq. (A.6)): order 0 and 1 kept; second order: deviator and off-diagonal
// scaled by 1 - omega, trace by 1 - omega_b; order n >= 3 (slot a + 3b + 9c
// has order a + b + c) by 1 - omega_o[n - 3].  m2 receives the six
// second-order moments before relaxation (xx, yy, zz, xy, xz, yz).
__device__ __forceinline__ void relax_moments(float (&f)[Q], float omega, float omega_b, const float (&omega_o)[4],
                                              float (&m2)[6])
{
    m2[0] = f[2];
    m2[1] = f[6];
    m2[2] = f[18];
    m2[3] = f[4];
    m2[4] = f[10];
    m2[5] = f[12];
    const float ks = 1.f - omega, kb = 1.f - omega_b;
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
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        const int n = k % 3 + (k / 3) % 3 + k / 9;
        if (n >= 3)
            f[k] *= 1.f - omega_o[n - 3];
    }
}

// Forward central-Hermite transform and relaxation for general rates of the
// orders 3..6: the raw x sweep gives rho and u, then the central sweeps
// and the relaxation.
__device__ __forceinline__ float moments_relax(float (&f)[Q], float omega, float omega_b, const float (&omega_o)[4],
                                               float &ux, float &uy, float &uz, float (&m2)[6])
{
    x_sweep_raw(f);
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
    central_sweeps(f, ux, uy, uz);
    relax_moments(f, omega, omega_b, omega_o, m2);
    return rho;
}

// Inverse sweeps z, y, x: raw moments R0 = m0, R1 = m1 + u m0,
// R2 = m2 + 2 u m1 + (u^2 + theta0) m0; then f(+1) = (R2 + R1)/2,
// f(-1) = (R2 - R1)/2, f(0) = R0 - R2.
__device__ __forceinline__ void inverse_sweeps(float (&f)[Q], float ux, float uy, float uz)
{
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
#undef LBM_INV_SWEEP
#undef LBM_OUTER_X
#undef LBM_OUTER_Y
#undef LBM_OUTER_Z
}

template <bool HIGH1>
__device__ __forceinline__ float collide(float (&f)[Q], float omega, float omega_b, const float (&omega_o)[4],
                                         float &ux, float &uy, float &uz, float (&m2)[6])
{
    const float rho = HIGH1 ? collide_h1(f, omega, omega_b, ux, uy, uz, m2)
                            : moments_relax(f, omega, omega_b, omega_o, ux, uy, uz, m2);
    inverse_sweeps(f, ux, uy, uz);
    return rho;
}

// The equilibrium of Eq. (4) truncated at order N (2 <= N <= 6), at every
// population.  With the per-axis Hermite terms (App. A, Eqs. (A.3)-(A.4))
// e_0 = 1, e_1(c, v) = c v / theta0, e_2(c, v) = (c^2 - theta0) v^2 /
// (2 theta0^2), the term of the expansion with n_a factors of axis a is
// rho w_i prod_a e_{n_a}(c_ia, u_a) (a tensor with axis a repeated n_a times
// appears n! / prod n_a! times in the sum over index tuples); the order of
// the term is n_x + n_y + n_z.  So f^eq_N is rho w_i times the sum of the
// coefficients of t^0 .. t^N of prod_a (1 + e_1 t + e_2 t^2).
__device__ __forceinline__ void feq_truncated(float rho, float ux, float uy, float uz, uint32_t N, float (&fe)[Q])
{
    // per axis and c = -1, 0, +1: (e_1, e_2)
    const float vx2 = ux * ux, vy2 = uy * uy, vz2 = uz * uz;
    const float e1x[3] = {-3.f * ux, 0.f, 3.f * ux}, e2x[3] = {3.f * vx2, -1.5f * vx2, 3.f * vx2};
    const float e1y[3] = {-3.f * uy, 0.f, 3.f * uy}, e2y[3] = {3.f * vy2, -1.5f * vy2, 3.f * vy2};
    const float e1z[3] = {-3.f * uz, 0.f, 3.f * uz}, e2z[3] = {3.f * vz2, -1.5f * vz2, 3.f * vz2};
    const float k3 = N >= 3u ? 1.f : 0.f, k4 = N >= 4u ? 1.f : 0.f, k5 = N >= 5u ? 1.f : 0.f,
                k6 = N >= 6u ? 1.f : 0.f;
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            // x times y: coefficients of t^1 .. t^4
            const float p1 = e1x[a] + e1y[b];
            const float p2 = e2x[a] + e1x[a] * e1y[b] + e2y[b];
            const float p3 = e2x[a] * e1y[b] + e1x[a] * e2y[b];
            const float p4 = e2x[a] * e2y[b];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float q1 = p1 + e1z[c];
                const float q2 = p2 + p1 * e1z[c] + e2z[c];
                const float q3 = p3 + p2 * e1z[c] + p1 * e2z[c];
                const float q4 = p4 + p3 * e1z[c] + p2 * e2z[c];
                const float q5 = p4 * e1z[c] + p3 * e2z[c];
                const float q6 = p4 * e2z[c];
                const float sum = 1.f + q1 + q2 + k3 * q3 + k4 * q4 + k5 * q5 + k6 * q6;
                const int i = a + 3 * b + 9 * c;
                fe[i] = rho * weight(i) * sum;
            }
        }
}

// Collision towards the explicit truncated equilibrium (Sec. 2.1, Eqs. (4)
// and (6) with the expansion summed to order N < 6): with g = f - f^eq_N,
// f* = f + T^-1 S T (f^eq_N - f) = f^eq_N + T^-1 (I - S) T g.  T g is the
// forward transform about the cell's velocity (its orders 0 and 1 vanish up
// to rounding; orders >= 3 no longer do, unlike with the full expansion);
// the relaxation and the inverse are those of the implicit form.
__device__ __forceinline__ float collide_feq(float (&f)[Q], float omega, float omega_b, const float (&omega_o)[4],
                                             uint32_t N, float &ux, float &uy, float &uz, float (&m2)[6])
{
    float s0[9], s1[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        s0[t] = f[3 * t] + f[3 * t + 1] + f[3 * t + 2];
        s1[t] = f[3 * t + 2] - f[3 * t];
    }
    float rho = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        rho += s0[t];
        jx += s1[t];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
        jy += s0[2 + 3 * c] - s0[3 * c];
#pragma unroll
    for (int b = 0; b < 3; ++b)
        jz += s0[b + 6] - s0[b];
    const float inv = __builtin_amdgcn_rcpf(rho);
    ux = jx * inv;
    uy = jy * inv;
    uz = jz * inv;
    // The opaque copies below fix the rounding of every value that meets
    // f^eq_N: without them the compiler may fuse a product into the
    // neighbouring add in one kernel and not in another (packed launches
    // inline this next to the other collisions), and a domain would no
    // longer end bit for bit where it ends alone.
    {
        float fe[Q];
        feq_truncated(rho, ux, uy, uz, N, fe);
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            asm volatile("" : "+v"(fe[k]));
            f[k] -= fe[k];
        }
    }
    x_sweep_raw(f);
    central_sweeps(f, ux, uy, uz);
    relax_moments(f, omega, omega_b, omega_o, m2);
    inverse_sweeps(f, ux, uy, uz);
    // f^eq_N again (recomputed rather than held through the transform; the
    // opaque copy keeps the compiler from reusing the first evaluation)
    float r2 = rho;
    asm volatile("" : "+v"(r2) : "v"(f[0]), "v"(f[26]));
    float fe[Q];
    feq_truncated(r2, ux, uy, uz, N, fe);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        asm volatile("" : "+v"(fe[k]), "+v"(f[k]));
        f[k] += fe[k];
    }
    return rho;
}

// Collision of a lane in kernel variant V.  In a packed launch a step runs
// one variant for every domain, the general collision as soon as one domain
// needs it (DYN); a domain whose higher-order rates are all one then still
// takes the reduced form, chosen per domain (the branch is wave-uniform), so
// that it ends bit for bit where it ends alone.
template <int V, bool DYN>
__device__ __forceinline__ float collide_lane(const KDomain &d, float (&f)[Q], float &ux, float &uy, float &uz,
                                              float (&m2)[6])
{
    if constexpr ((V & kVarFeq) != 0) {
        if constexpr (DYN) {
            // a packed domain with the full equilibrium takes its own path
            if (d.feq_order >= 6u) {
                if (d.high1)
                    return collide<true>(f, d.omega, d.omega_b, d.omega_o, ux, uy, uz, m2);
                return collide<false>(f, d.omega, d.omega_b, d.omega_o, ux, uy, uz, m2);
            }
        }
        return collide_feq(f, d.omega, d.omega_b, d.omega_o, d.feq_order, ux, uy, uz, m2);
    } else if constexpr ((V & kVarH1) != 0) {
        return collide<true>(f, d.omega, d.omega_b, d.omega_o, ux, uy, uz, m2);
    } else if constexpr (DYN) {
        if (d.high1)
            return collide<true>(f, d.omega, d.omega_b, d.omega_o, ux, uy, uz, m2);
        return collide<false>(f, d.omega, d.omega_b, d.omega_o, ux, uy, uz, m2);
    } else {
        return collide<false>(f, d.omega, d.omega_b, d.omega_o, ux, uy, uz, m2);
    }
}

// ---------------------------------------------------------------------------
// The step, in place on one population array (Sec. 2.1, Eq. (6); boundary
// rules of Sec. 2.2).  Steps alternate between two phases, so that each
// step reads and writes the same 27 slots per cell and no second array is
// needed; slot (x, k) is population k of cell x in the tile layout.
//
//  phase 0, streaming step.  On entry slot (x, k) holds f*_kbar(x), the
//   post-collision population kbar = 26 - k of x.  Link k of x reads slot
//   a_k(x) = (x - c_k, kbar), which holds f*_k(x - c_k) = f_k(x) after
//   streaming; a bounce-back link reads its own slot (x, k) = f*_kbar(x)
//   (+ the moving-wall term).  After the collision the lane writes
//   f*_kbar(x) (+ the term) to the same slot a_k(x): that is population
//   kbar of the downstream cell x - c_k after streaming, or, behind a wall,
//   population k of x itself.  On exit slot (x, k) holds f_k(x) of the
//   next step.
//  phase 1, local step.  The lane reads its own 27 slots (f_k), collides
//   and writes f*_k to slot (x, kbar).
//
// Every slot is read and written by one lane only.  Outlet cells take their
// clamped upstream values (zero-gradient, c_x = -1 links) from side rows
// that the local step fills for the cells of the last x plane; in the
// streaming step those cells also copy those values to the outlet cells
// they feed, and the outlet cells park their leaving c_x = +1 values in a
// second side row set, so that a phase-1 state can be turned back into the
// phase-0 form (k_normalise).
// ---------------------------------------------------------------------------

// Cell coordinates and source coordinates per velocity component: index 0
// is the source of c = -1 (x + 1), 1 of c = 0, 2 of c = +1.  Periodic axes
// wrap; other axes clamp to the box (a clamped source is the outlet's or
// belongs to a bounce-back link).  row[b + 3c]: first cell of the source
// row (cy = b - 1, cz = c - 1).
struct Coords {
    uint32_t x, y, z;
    uint32_t sx[3], sy[3], sz[3];
    uint32_t row[9];
};

__device__ __forceinline__ Coords coords(const KDomain &d, uint32_t lin)
{
    Coords C;
    const uint32_t q = fdiv(lin, d.dnx);
    C.x = lin - q * d.nx;
    C.z = fdiv(q, d.dny);
    C.y = q - C.z * d.ny;
    const bool px = d.periodic & 1u, py = d.periodic & 2u, pz = d.periodic & 4u;
    C.sx[1] = C.x;
    C.sx[0] = (C.x + 1 < d.nx) ? C.x + 1 : (px ? 0u : C.x);
    C.sx[2] = (C.x > 0) ? C.x - 1 : (px ? d.nx - 1 : 0u);
    C.sy[1] = C.y;
    C.sy[0] = (C.y + 1 < d.ny) ? C.y + 1 : (py ? 0u : C.y);
    C.sy[2] = (C.y > 0) ? C.y - 1 : (py ? d.ny - 1 : 0u);
    C.sz[1] = C.z;
    C.sz[0] = (C.z + 1 < d.nz) ? C.z + 1 : (pz ? 0u : C.z);
    C.sz[2] = (C.z > 0) ? C.z - 1 : (pz ? d.nz - 1 : 0u);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            C.row[b + 3 * c] = (C.sz[c] * d.ny + C.sy[b]) * d.nx;
    return C;
}

__device__ __forceinline__ bool lane_active(const TileRec &rec, uint32_t lane)
{
    return ((lane < 32u ? rec.act[0] : rec.act[1]) >> (lane & 31u)) & 1u;
}

// Byte offset of side row element (h, j, plane cell (y, z)): h = 0 holds
// f*_k of the last-plane cells for the nine c_x = -1 directions k = 3 j,
// h = 1 the leaving f*_k of the outlet cells for k = 3 j + 2.
template <uint32_t ES, class Off = uint32_t>
__device__ __forceinline__ Off side_bytes(const KDomain &d, uint32_t h, uint32_t j, uint32_t y, uint32_t z)
{
    return (Off)d.side + ((Off)(h * 9u + j) * (d.ny * d.nz) + z * d.ny + y) * ES;
}

// Plane coordinate y + dy wrapped or checked against the box; false if it
// leaves a non-periodic box.
__device__ __forceinline__ bool plane_step(uint32_t v, int dv, uint32_t n, bool per, uint32_t &out)
{
    int w = (int)v + dv;
    if (w < 0 || w >= (int)n) {
        if (!per)
            return false;
        w = w < 0 ? w + (int)n : w - (int)n;
    }
    out = (uint32_t)w;
    return true;
}

__device__ __forceinline__ void check_state(const KDomain &d, float rho, float ux, float uy, float uz)
{
    if (!(rho > 0.f) || !(__builtin_fabsf(ux) + __builtin_fabsf(uy) + __builtin_fabsf(uz) < 1e30f))
        atomicOr(d.status, 1u);
}

// Inlet term of link k of the lane (0 where link k is not an inlet link).
__device__ __forceinline__ float inlet_term(const KDomain &d, const TileRec &rec, uint32_t lane, int k)
{
    constexpr uint32_t kTermBytes = Q * 64u * 4u;
    const auto rt = make_rsrc((const char *)(d.iterm + (size_t)rec.inl * (Q * 64u)), kTermBytes);
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rt, ((rec.inlm >> k) & 1u) ? lane * 4u : kTermBytes,
                                                                (uint32_t)k * 256u, 0));
}

// Constant-pressure outlet by non-equilibrium extrapolation (Sec. 2.2): the
// ghost cell beyond the last plane has the velocity and non-equilibrium part
// of the last-plane cell s it faces and the density rho_out.  Its value of
// direction k = 3 j (c_x = -1) is f*_k(s) + (rho_out - rho_s) f^eq_k(1, u_s),
// f^eq being linear in rho; g[j] receives the second term, with f^eq(1, u)
// in product form, prod_a phi(c_a, u_a), phi(0, u) = 2/3 - u^2,
// phi(+-1, u) = (1 +- 3u + 3u^2)/6.  rho_s and u_s are the moments of s,
// which its collision keeps.
__device__ __forceinline__ void outlet_ghost_shift(const KDomain &d, float rho, float ux, float uy, float uz,
                                                   float (&g)[9])
{
    const float a = (d.rho_out - rho) * (1.f / 6.f) * (1.f - 3.f * ux + 3.f * ux * ux);
    const float py[3] = {(1.f / 6.f) * (1.f - 3.f * uy + 3.f * uy * uy), 2.f / 3.f - uy * uy,
                         (1.f / 6.f) * (1.f + 3.f * uy + 3.f * uy * uy)};
    const float pz[3] = {(1.f / 6.f) * (1.f - 3.f * uz + 3.f * uz * uz), 2.f / 3.f - uz * uz,
                         (1.f / 6.f) * (1.f + 3.f * uz + 3.f * uz * uz)};
#pragma unroll
    for (int j = 0; j < 9; ++j)
        g[j] = a * py[j % 3] * pz[j / 3];
}

// Curved walls (Sec. 2.2, interpolated bounce-back after Bouzidi et al.).
// For a wall link k of cell x, at fraction q of the link towards x - c_k,
// the linear interpolation gives f_k = 2q f*_kbar(x) + (1 - 2q) f*_kbar(x + c_k)
// for q < 1/2 and f_k = f*_kbar(x) / (2q) + (1 - 1/(2q)) f*_k(x) for
// q >= 1/2.  On entry f[k] holds the halfway value f*_kbar(x) and f[kbar]
// the value pulled for kbar, which is f*_kbar(x + c_k) (the host gives the
// halfway coefficients where kbar is no plain link).  f*_k(x) cannot be
// read from the slots: in the streaming step the lane of x + c_k owns
// that slot, so each step keeps it in bzaux.  The host stores per lane
// and link (a, b): f_k <- a f_k + b f_kbar for b > 0, a f_k - b aux_k
// otherwise; (1, 0) where the lane has no curved link k.
__device__ __forceinline__ void curved_walls(const KDomain &d, const TileRec &rec, uint32_t lane, float (&f)[Q])
{
    const size_t base = (size_t)(uint32_t)rec.wall * (Q * 64u) + lane;
    float nf[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        if ((rec.bz >> k) & 1u) {
            const float2 c = d.bzc[base + k * 64u];
            const float other = c.y > 0.f ? f[Q - 1 - k] : d.bzaux[base + k * 64u];
            nf[k] = c.x * f[k] + __builtin_fabsf(c.y) * other;
        }
    }
#pragma unroll
    for (int k = 0; k < Q; ++k)
        if ((rec.bz >> k) & 1u)
            f[k] = nf[k];
}

// Keeps f*_k of the lane's curved links for the next step.
__device__ __forceinline__ void curved_keep(const KDomain &d, const TileRec &rec, uint32_t lane, const float (&f)[Q])
{
    const size_t base = (size_t)(uint32_t)rec.wall * (Q * 64u) + lane;
#pragma unroll
    for (int k = 0; k < Q; ++k)
        if ((rec.bz >> k) & 1u)
            d.bzaux[base + k * 64u] = f[k];
}

// Byte offset of slot a_k of the lane whose coordinates are C: the plain
// neighbour slot, or for a c_x = -1 link of a cell on the outlet plane of
// an edge tile the side row named by h (0: the clamped upstream value to
// read, 1: where the leaving value of the opposite direction is parked).
// On that plane such a link is either the outlet's clamped link or a
// bounce-back link (a fluid cell there has no source beyond the box), and a
// bounce-back link uses the lane's own slot instead (selected by the mask).
template <uint32_t ES, class Off = uint32_t>
__device__ __forceinline__ Off slot_of(const KDomain &d, const Coords &C, int k, bool edge_lane, uint32_t h)
{
    if (edge_lane && k % 3 == 0) {
        const int j = k / 3;
        return h == 0u ? side_bytes<ES, Off>(d, 0u, (uint32_t)j, C.sy[j % 3], C.sz[j / 3])
                       : side_bytes<ES, Off>(d, 1u, (uint32_t)(8 - j), C.y, C.z);
    }
    return cell_bytes<ES, Off>(C.row[k / 3] + C.sx[k % 3], d.tbytes) + pop_bytes<ES>(Q - 1 - k);
}

// Phase 0 -> 1.  EDGE: the tile has cells on the outlet plane (tile entry
// `edge`); the other tiles compile without the outlet handling.
template <int ST, int V, bool EDGE, bool DYN = false, bool W64 = false>
__device__ __forceinline__ void stream_tile_t(const KDomain &d, const TileRec &rec, uint32_t lane)
{
    using S = Storage<ST>;
    using P = Pops<ST, W64>;
    using Off = typename P::Off;
    constexpr uint32_t es = S::bytes;
    const P r(d);
    const uint32_t lin = rec.tile * 64u + lane;
    const bool wall = rec.wall >= 0;
    if (wall && !lane_active(rec, lane))
        return;
    prio_loads();

    float f[Q];
    uint32_t m = 0;
    {
        const Coords C = coords(d, lin);
        if (!wall) {
#pragma unroll
            for (int k = 0; k < Q; ++k)
                f[k] = r.load(cell_bytes<es, Off>(C.row[k / 3] + C.sx[k % 3], d.tbytes), pop_bytes<es>(Q - 1 - k), k);
        } else {
            // The per-cell mask picks each link's slot: the own slot of a
            // bounce-back link, else a_k.  (Loading both candidates before
            // the mask arrives and selecting afterwards measured slower: it
            // issues twice the load instructions.)
            const Off self = cell_bytes<es, Off>(lin, d.tbytes);
            const bool edge_lane = EDGE && C.x == d.nx - 1u;
            m = d.wall[(uint32_t)rec.wall * 64u + lane];
#pragma unroll
            for (int k = 0; k < Q; ++k)
                f[k] = r.load(((m >> k) & 1u) ? self + pop_bytes<es>(k) : slot_of<es, Off>(d, C, k, edge_lane, 0u),
                              0u, k);
            if (rec.inlm) {
#pragma unroll
                for (int k = 0; k < Q; ++k)
                    f[k] += inlet_term(d, rec, lane, k);
            }
            if constexpr ((V & kVarCurved) != 0) {
                if (rec.bz)
                    curved_walls(d, rec, lane, f);
            }
        }
    }

    prio_compute();
    float ux, uy, uz, m2[6];
    const float rho = collide_lane<V, DYN>(d, f, ux, uy, uz, m2);
    check_state(d, rho, ux, uy, uz);
    if constexpr ((V & kVarCurved) != 0) {
        if (wall && rec.bz)
            curved_keep(d, rec, lane, f);
    }

    // The slot addresses are recomputed rather than kept through the
    // collision (an opaque copy of the index stops the compiler from
    // holding them in registers).
    uint32_t lin2 = lin;
    asm volatile("" : "+v"(lin2) : "v"(f[0]), "v"(f[13]), "v"(f[26]));
    const Coords C = coords(d, lin2);
    const bool edge_lane = EDGE && C.x == d.nx - 1u;
    if (edge_lane) {
        // last-plane cell: hand the clamped values to the outlet cells it
        // feeds, cell (nx - 1, y + c_y, z + c_z) for direction k = 3 j
        // (in a packed launch the pressure variant also runs domains with the
        // zero-gradient outlet: d.outlet decides)
        const bool pressure = (V & kVarPressure) != 0 && d.outlet;
        float g[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (pressure)
            outlet_ghost_shift(d, rho, ux, uy, uz, g);
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            const int k = 3 * j;
            uint32_t ty, tz;
            if (plane_step(C.y, cy(k), d.ny, d.periodic & 2u, ty) && plane_step(C.z, cz(k), d.nz, d.periodic & 4u, tz)) {
                const uint32_t t = (tz * d.ny + ty) * d.nx + d.nx - 1u;
                if (d.flags[t] == FL_OUTLET)
                    r.store(cell_bytes<es, Off>(t, d.tbytes), pop_bytes<es>(k), pressure ? f[k] + g[j] : f[k], k);
            }
        }
    }
    if (rec.inlm) {
        // bounce-back slots of inlet links carry the term into the next step
#pragma unroll
        for (int k = 0; k < Q; ++k)
            f[Q - 1 - k] += inlet_term(d, rec, lane, k);
    }
    // Each store address is formed just before its store (the opaque copy
    // of the row index, ordered after the previous store, keeps the
    // compiler from forming all 27 at once).
    if (!wall) {
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            uint32_t rowk = C.row[k / 3];
            asm volatile("" : "+v"(rowk)::"memory");
            r.store(cell_bytes<es, Off>(rowk + C.sx[k % 3], d.tbytes), pop_bytes<es>(Q - 1 - k), f[Q - 1 - k], k);
        }
    } else {
        const Off self = cell_bytes<es, Off>(lin2, d.tbytes);
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            Coords Ck = C;
            asm volatile("" : "+v"(Ck.row[k / 3])::"memory");
            r.store(((m >> k) & 1u) ? self + pop_bytes<es>(k) : slot_of<es, Off>(d, Ck, k, edge_lane, 1u), 0u,
                    f[Q - 1 - k], k);
        }
    }
}

// Row-aligned domains (nx a multiple of 64, KDomain::rowtiles = nx / 64):
// a tile lies in one row, so the first cell of each of the nine source rows
// (y - c_y, z - c_z) is the start of a tile, the same for every lane.  The
// byte offset of slot a_k then splits into that row's tile offset and the
// slot's offset, both wave-uniform (the buffer instruction's scalar offset),
// plus the lane's offset of cell x - c_x within its row, one of three
// per-lane values.  This drops the per-lane coordinate decode and address
// arithmetic of stream_tile_t.  On the outlet plane (EDGE) the only cell of
// a tile is its lane 63, and the side-row elements it uses and the outlet
// cells it feeds have wave-uniform addresses too.
template <class Off> struct RowAddr {
    uint32_t y, z, j; // the tile's row and its position in the row
    uint32_t xo[3];   // by c_x + 1: byte offset of cell (x - c_x) from the start of its row
    uint32_t sy[3], sz[3];
    Off row[9];       // by (c_y + 1) + 3 (c_z + 1): byte offset of the first tile of the source row
};

template <uint32_t ES, class Off = uint32_t>
__device__ __forceinline__ RowAddr<Off> row_addr(const KDomain &d, const TileRec &rec, uint32_t lane)
{
    RowAddr<Off> A;
    const uint32_t R = d.rowtiles, q = fdiv(rec.tile, d.drow);
    A.j = rec.tile - q * R;
    A.z = fdiv(q, d.dny);
    A.y = q - A.z * d.ny;
    const uint32_t x = A.j * 64u + lane, y = A.y, z = A.z;
    const bool px = d.periodic & 1u, py = d.periodic & 2u, pz = d.periodic & 4u;
    // a source outside a non-periodic box belongs to a bounce-back link (the
    // mask selects the own slot) or to the outlet (side rows); it is
    // clamped to stay in the array
    const uint32_t sx[3] = {x + 1u < d.nx ? x + 1u : (px ? 0u : x), x, x > 0u ? x - 1u : (px ? d.nx - 1u : 0u)};
    A.sy[0] = y + 1u < d.ny ? y + 1u : (py ? 0u : y);
    A.sy[1] = y;
    A.sy[2] = y > 0u ? y - 1u : (py ? d.ny - 1u : 0u);
    A.sz[0] = z + 1u < d.nz ? z + 1u : (pz ? 0u : z);
    A.sz[1] = z;
    A.sz[2] = z > 0u ? z - 1u : (pz ? d.nz - 1u : 0u);
#pragma unroll
    for (int a = 0; a < 3; ++a)
        A.xo[a] = (sx[a] >> 6) * d.tbytes + (sx[a] & 63u) * ES;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            A.row[b + 3 * c] = (Off)(A.sz[c] * d.ny + A.sy[b]) * (R * d.tbytes);
    return A;
}

// Phase 0 -> 1 for a tile of a row-aligned domain: stream_tile_t with the
// addressing above.  EDGE: the tile holds a cell of the outlet plane.
template <int ST, int V, bool EDGE, bool DYN = false, bool W64 = false>
__device__ __forceinline__ void stream_tile_rows(const KDomain &d, const TileRec &rec, uint32_t lane)
{
    using S = Storage<ST>;
    using P = Pops<ST, W64>;
    using Off = typename P::Off;
    constexpr uint32_t es = S::bytes;
    const P r(d);
    const bool wall = rec.wall >= 0;
    if (wall && !lane_active(rec, lane))
        return;
    prio_loads();
    const Off self = (Off)rec.tile * d.tbytes + lane * es;
    // the outlet-plane cell: lane 63 of the last tile of its row
    const bool edge_lane = EDGE && lane == 63u && rec.tile - fdiv(rec.tile, d.drow) * d.rowtiles == d.rowtiles - 1u;

    float f[Q];
    uint32_t m = 0;
    {
        const RowAddr<Off> A = row_addr<es, Off>(d, rec, lane);
        if (!wall) {
#pragma unroll
            for (int k = 0; k < Q; ++k)
                f[k] = r.load(A.xo[k % 3], A.row[k / 3] + pop_bytes<es>(Q - 1 - k), k);
        } else {
            m = d.wall[(uint32_t)rec.wall * 64u + lane];
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                Off off = A.xo[k % 3] + A.row[k / 3] + pop_bytes<es>(Q - 1 - k);
                if (EDGE && k % 3 == 0) // the clamped upstream value of an outlet cell
                    off = edge_lane ? side_bytes<es, Off>(d, 0u, (uint32_t)k / 3u, A.sy[(k / 3) % 3], A.sz[k / 9])
                                    : off;
                f[k] = r.load(((m >> k) & 1u) ? self + pop_bytes<es>(k) : off, 0u, k);
            }
            if (rec.inlm) {
#pragma unroll
                for (int k = 0; k < Q; ++k)
                    f[k] += inlet_term(d, rec, lane, k);
            }
            if constexpr ((V & kVarCurved) != 0) {
                if (rec.bz)
                    curved_walls(d, rec, lane, f);
            }
        }
    }

    prio_compute();
    float ux, uy, uz, m2[6];
    const float rho = collide_lane<V, DYN>(d, f, ux, uy, uz, m2);
    check_state(d, rho, ux, uy, uz);
    if constexpr ((V & kVarCurved) != 0) {
        if (wall && rec.bz)
            curved_keep(d, rec, lane, f);
    }
    // the lane offsets are recomputed after the collision (an opaque copy of
    // the lane index keeps the compiler from holding them through it)
    uint32_t lane2 = lane;
    asm volatile("" : "+v"(lane2) : "v"(f[0]), "v"(f[13]), "v"(f[26]));
    const RowAddr<Off> A = row_addr<es, Off>(d, rec, lane2);
    if constexpr (EDGE) {
        // the outlet-plane cell hands the clamped values to the outlet cells
        // it feeds, cell (nx - 1, y + c_y, z + c_z) for direction k = 3 j
        // (in a packed launch the pressure variant also runs domains with
        // the zero-gradient outlet: d.outlet decides)
        const bool pressure = (V & kVarPressure) != 0 && d.outlet;
        float g[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (pressure)
            outlet_ghost_shift(d, rho, ux, uy, uz, g);
#pragma unroll
        for (int jj = 0; jj < 9; ++jj) {
            const int k = 3 * jj;
            uint32_t ty, tz;
            if (plane_step(A.y, cy(k), d.ny, d.periodic & 2u, ty) && plane_step(A.z, cz(k), d.nz, d.periodic & 4u, tz)) {
                const uint32_t t = (tz * d.ny + ty) * d.nx + d.nx - 1u;
                if (d.flags[t] == FL_OUTLET && edge_lane)
                    r.store(cell_bytes<es, Off>(t, d.tbytes), pop_bytes<es>(k), pressure ? f[k] + g[jj] : f[k], k);
            }
        }
    }
    if (rec.inlm) {
        // bounce-back slots of inlet links carry the term into the next step
#pragma unroll
        for (int k = 0; k < Q; ++k)
            f[Q - 1 - k] += inlet_term(d, rec, lane, k);
    }
    const Off self2 = (Off)rec.tile * d.tbytes + lane2 * es;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        if (!wall) {
            r.store(A.xo[k % 3], A.row[k / 3] + pop_bytes<es>(Q - 1 - k), f[Q - 1 - k], k);
        } else {
            Off off = A.xo[k % 3] + A.row[k / 3] + pop_bytes<es>(Q - 1 - k);
            if (EDGE && k % 3 == 0) // an outlet cell parks its leaving value
                off = edge_lane ? side_bytes<es, Off>(d, 1u, 8u - (uint32_t)k / 3u, A.y, A.z) : off;
            r.store(((m >> k) & 1u) ? self2 + pop_bytes<es>(k) : off, 0u, f[Q - 1 - k], k);
        }
    }
}

// Phase 1 -> 0, in two halves so that a wave can issue the loads of its
// next tile before it collides the current one.  Lanes of cells that are
// not updated load nothing and store nothing.
template <int ST, bool W64 = false>
__device__ __forceinline__ void local_load(const KDomain &d, const TileRec &rec, uint32_t lane, float (&f)[Q])
{
    using P = Pops<ST, W64>;
    using Off = typename P::Off;
    constexpr uint32_t es = Storage<ST>::bytes;
    const P r(d);
    const Off self = cell_bytes<es, Off>(rec.tile * 64u + lane, d.tbytes);
    prio_loads();
    if (rec.wall < 0 || lane_active(rec, lane)) {
#pragma unroll
        for (int k = 0; k < Q; ++k)
            f[k] = r.load(self, pop_bytes<es>(k), k);
    } else {
#pragma unroll
        for (int k = 0; k < Q; ++k)
            f[k] = weight(k);
    }
}

// With statistics on (d.stats), the local step adds per cell, from the
// pre-collision state it collides: u (3 sums), u_a u_b (6: xx yy zz xy xz yz)
// and the viscous stress sigma_ab = 2 rho nu S_ab = -(1 - omega/2) M_ab from
// the central second-order Hermite moments M_ab (Sec. 2.2, Eqs. (15)-(19);
// App. A, Eqs. (A.7)-(A.8)); sums of component c at stats[c * sstride +
// 64 ord + lane].  The sums are FP64 and the products u_a u_b are formed
// exactly in FP64 from the FP32 velocities, so that averages over long
// windows keep their digits and the Reynolds stress <u_a u_b> - <u_a><u_b>
// does not cancel away.
template <int ST, int V, bool DYN = false, bool W64 = false>
__device__ __forceinline__ void local_finish(const KDomain &d, const TileRec &rec, uint32_t lane, float (&f)[Q])
{
    using P = Pops<ST, W64>;
    using Off = typename P::Off;
    constexpr uint32_t es = Storage<ST>::bytes;
    if (rec.wall >= 0 && !lane_active(rec, lane))
        return;
    const P r(d);
    const uint32_t lin = rec.tile * 64u + lane;
    const Off self = cell_bytes<es, Off>(lin, d.tbytes);
    if constexpr ((V & kVarCurved) != 0) {
        if (rec.wall >= 0 && rec.bz)
            curved_walls(d, rec, lane, f);
    }
    prio_compute();
    float ux, uy, uz, m2[6];
    const float rho = collide_lane<V, DYN>(d, f, ux, uy, uz, m2);
    check_state(d, rho, ux, uy, uz);
    if constexpr ((V & kVarCurved) != 0) {
        if (rec.wall >= 0 && rec.bz)
            curved_keep(d, rec, lane, f);
    }
#pragma unroll
    for (int k = 0; k < Q; ++k)
        r.store(self, pop_bytes<es>(Q - 1 - k), f[k], k);
    if (d.stats) {
        double *acc = d.stats + rec.ord * 64u + lane;
        const float ks = -(1.f - 0.5f * d.omega);
        const double vx = ux, vy = uy, vz = uz;
        const double v[15] = {vx, vy, vz, vx * vx, vy * vy, vz * vz, vx * vy, vx * vz, vy * vz,
                              ks * m2[0], ks * m2[1], ks * m2[2], ks * m2[3], ks * m2[4], ks * m2[5]};
#pragma unroll
        for (int c = 0; c < 15; ++c)
            acc[(size_t)c * d.sstride] += v[c];
    }
    if (rec.edge) {
        const uint32_t q = fdiv(lin, d.dnx);
        if (lin - q * d.nx == d.nx - 1u) {
            // last-plane cell: its c_x = -1 values for the outlet cells
            const uint32_t z = fdiv(q, d.dny), y = q - z * d.ny;
            const bool pressure = (V & kVarPressure) != 0 && d.outlet;
            float g[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            if (pressure)
                outlet_ghost_shift(d, rho, ux, uy, uz, g);
#pragma unroll
            for (int j = 0; j < 9; ++j)
                r.store(side_bytes<es, Off>(d, 0u, (uint32_t)j, y, z), 0u, pressure ? f[3 * j] + g[j] : f[3 * j],
                        3 * j);
        }
    }
}

template <int ST, int V, bool DYN = false, bool W64 = false>
__device__ __forceinline__ void local_tile(const KDomain &d, const TileRec &rec, uint32_t lane)
{
    float f[Q];
    local_load<ST, W64>(d, rec, lane, f);
    local_finish<ST, V, DYN, W64>(d, rec, lane, f);
}

#ifdef LBM_HOST_TU
// (The kernels that are not templates are defined in the library's host
// translation unit only; the templates are instantiated per storage in
// their own translation units.)

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

#endif // LBM_HOST_TU

// Block index -> logical block: consecutive hardware blocks go round-robin
// to the 8 XCDs; give each XCD a contiguous range of tiles so that the cache
// lines shared by neighbouring tiles meet in the same L2.  G is a multiple
// of 8.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t G) { return (b & 7u) * (G >> 3) + (b >> 3); }

// Single-domain steps, one kernel per phase (the local step needs far fewer
// registers than the streaming step).  Each wave takes whole tiles, walking
// the tile list with a stride of the grid's wave count (one pass when the
// grid covers every tile).
// Streaming step of a single domain; ROWS: the domain is row-aligned
// (stream_tile_rows), chosen per domain on the host, so that each kernel
// carries only one addressing scheme; W64: the array reaches past 4 GiB
// (Pops).
template <int ST, int V, bool ROWS, bool W64>
__global__ __launch_bounds__(kBlock) void k_stream_collide(KDomain d, const TileRec *__restrict__ tiles,
                                                           uint32_t ntiles)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t nw = gridDim.x * kWavesPerBlock;
    const uint32_t w0 =
        __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + (threadIdx.x >> 6));
    for (uint32_t t = w0; t < ntiles; t += nw) {
        const TileRec rec = tiles[t];
        if constexpr (ROWS) {
            if (rec.edge)
                stream_tile_rows<ST, V, true, false, W64>(d, rec, lane);
            else
                stream_tile_rows<ST, V, false, false, W64>(d, rec, lane);
        } else {
            if (rec.edge)
                stream_tile_t<ST, V, true, false, W64>(d, rec, lane);
            else
                stream_tile_t<ST, V, false, false, W64>(d, rec, lane);
        }
    }
}

template <int ST, int V, bool W64>
__global__ __launch_bounds__(kBlock) void k_local_collide(KDomain d, const TileRec *__restrict__ tiles,
                                                          uint32_t ntiles)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t nw = gridDim.x * kWavesPerBlock;
    const uint32_t w0 =
        __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + (threadIdx.x >> 6));
    for (uint32_t t = w0; t < ntiles; t += nw)
        local_tile<ST, V, false, W64>(d, tiles[t], lane);
}

// Packed multi-domain step over one range of a tile table (one group of
// domains of one parity class): the kernel runs global step
// g = ctrl[1] + soff (a graph of several steps gives each of its nodes its
// offset and advances ctrl[1] once at its end), and every domain of the
// range is in the phase PHASE at that step.  One wave per tile record; each
// tile belongs to one domain, whose descriptor says whether it takes part
// in this step.  The streaming kernel of the reduced collision without
// curved walls is bounded to six waves per SIMD: left alone the compiler
// takes 81 VGPRs (five waves) for FP16S, bounded 72, with no spills (packed
// steps 0.7 % faster); the curved-wall variants would spill under the same
// bound.
template <int V, uint32_t PHASE>
constexpr int kBatchedMinBlocks = ((V & kVarH1) != 0 && (V & kVarCurved) == 0 && PHASE == 0u) ? 6 : 1;

// ROWS (streaming phase only): every domain of the range is row-aligned
// (stream_tile_rows), or none is (stream_tile_t).  The host keeps the two
// kinds in separate groups, so that a kernel carries the code of one
// addressing scheme: with both in one kernel, ranges mixing the kinds ran
// 10-15 % slower than either kind alone.
template <int ST, int V, uint32_t PHASE, bool ROWS = false>
__global__ __launch_bounds__(kBlock, (kBatchedMinBlocks<V, PHASE>)) void k_collide_batched(
    const KDomain *__restrict__ doms, const TileRec *__restrict__ tiles, uint32_t ntiles,
    const uint32_t *__restrict__ ctrl, uint32_t soff)
{
    constexpr bool DYN = (V & kVarH1) == 0;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t g = ctrl[1] + soff;
    const uint32_t nw = gridDim.x * kWavesPerBlock;
    const uint32_t w0 =
        __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + (threadIdx.x >> 6));
    for (uint32_t t = w0; t < ntiles; t += nw) {
        const TileRec rec = tiles[t];
        const KDomain &dd = doms[rec.slot];
        const uint32_t k = g - dd.step0;
        if (k >= dd.nsteps || ((dd.ph0 + k) & 1u) != PHASE)
            continue;
        if constexpr (PHASE == 0u) {
            if constexpr (ROWS) {
                if (rec.edge)
                    stream_tile_rows<ST, V, true, DYN>(dd, rec, lane);
                else
                    stream_tile_rows<ST, V, false, DYN>(dd, rec, lane);
            } else {
                if (rec.edge)
                    stream_tile_t<ST, V, true, DYN>(dd, rec, lane);
                else
                    stream_tile_t<ST, V, false, DYN>(dd, rec, lane);
            }
        } else {
            local_tile<ST, V, DYN>(dd, rec, lane);
        }
    }
}

#ifdef LBM_HOST_TU
__global__ void k_advance_step(uint32_t *ctrl, uint32_t by)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        ctrl[1] = ctrl[1] + by;
}
#endif

// ---------------------------------------------------------------------------
// State access.  Outside a step the host keeps a domain in phase 0, where
// population i of cell x, f*_i(x), is slot (x, 26 - i).
// ---------------------------------------------------------------------------

// Phase 1 -> 0 without a collision: every slot pair (x, k) / a_k(x) of a
// link that is neither bounced back nor clamped swaps its two values; a
// bounce-back slot loses its inlet term; a clamped slot of an outlet cell
// hands the value it received (the ghost value of its source cell s) to
// the first side row of s, where the next streaming step reads it, and
// takes the leaving value parked in the second side row.  Every side-row
// entry a streaming step reads is rewritten that way, by the one outlet
// cell that reads it.
template <int ST>
__global__ __launch_bounds__(256) void k_normalise(KDomain d, const TileRec *__restrict__ tiles, uint32_t ntiles)
{
    using S = Storage<ST>;
    constexpr uint32_t es = S::bytes;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t t = __builtin_amdgcn_readfirstlane(blockIdx.x * 4u + (threadIdx.x >> 6));
    if (t >= ntiles)
        return;
    const TileRec rec = tiles[t];
    if (rec.wall >= 0 && !lane_active(rec, lane))
        return;
    const Pops<ST, true> r(d);
    const uint32_t lin = rec.tile * 64u + lane;
    const Coords C = coords(d, lin);
    const uint64_t self = cell_bytes<es, uint64_t>(lin, d.tbytes);
    const uint32_t m = rec.wall >= 0 ? d.wall[(uint32_t)rec.wall * 64u + lane] : 0u;
    const bool edge_lane = rec.edge && C.x == d.nx - 1u;
    for (int k = 0; k < Q; ++k) {
        if ((m >> k) & 1u) {
            if ((rec.inlm >> k) & 1u) {
                const float v = r.load(self, pop_bytes<es>(k), k) - inlet_term(d, rec, lane, k);
                r.store(self, pop_bytes<es>(k), v, k);
            }
        } else if (edge_lane && k % 3 == 0) {
            r.store_raw(slot_of<es, uint64_t>(d, C, k, true, 0u), 0u, r.raw(self + pop_bytes<es>(k), 0u));
            r.store_raw(self + pop_bytes<es>(k), 0u, r.raw(slot_of<es, uint64_t>(d, C, k, true, 1u), 0u));
        } else if (k > Q / 2) {
            const uint64_t ak =
                cell_bytes<es, uint64_t>(C.row[k / 3] + C.sx[k % 3], d.tbytes) + pop_bytes<es>(Q - 1 - k);
            const uint32_t u = r.raw(self + pop_bytes<es>(k), 0u), v = r.raw(ak, 0u);
            r.store_raw(self + pop_bytes<es>(k), 0u, v);
            r.store_raw(ak, 0u, u);
        }
    }
}

// First side rows from a phase-0 state (after an initialisation or an
// import): the ghost value of each updated last-plane cell for k = 3 j,
// f*_k from slot (x, 26 - 3 j), plus the pressure outlet's shift.  One lane
// per (y, z).
template <int ST>
__global__ __launch_bounds__(256) void k_side_refresh(KDomain d)
{
    using S = Storage<ST>;
    constexpr uint32_t es = S::bytes;
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= d.ny * d.nz)
        return;
    const uint32_t z = p / d.ny, y = p - z * d.ny;
    const uint32_t c = (z * d.ny + y) * d.nx + d.nx - 1u;
    if (d.flags[c] != FL_FLUID && d.flags[c] != FL_OUTLET)
        return;
    const Pops<ST, true> r(d);
    const uint64_t cb = cell_bytes<es, uint64_t>(c, d.tbytes);
    if (!d.outlet) {
        for (int j = 0; j < 9; ++j)
            r.store_raw(side_bytes<es, uint64_t>(d, 0u, (uint32_t)j, y, z), 0u,
                        r.raw(cb + pop_bytes<es>(Q - 1 - 3 * j), 0u));
        return;
    }
    float f[Q], rho = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        f[i] = r.load(cb, pop_bytes<es>(Q - 1 - i), i);
        rho += f[i];
        jx += (float)cx(i) * f[i];
        jy += (float)cy(i) * f[i];
        jz += (float)cz(i) * f[i];
    }
    float g[9];
    outlet_ghost_shift(d, rho, jx / rho, jy / rho, jz / rho, g);
#pragma unroll
    for (int j = 0; j < 9; ++j)
        r.store(side_bytes<es, uint64_t>(d, 0u, (uint32_t)j, y, z), 0u, f[3 * j] + g[j], 3 * j);
}

// bzaux from a phase-0 state (after an initialisation, an import or new
// wall fractions): f*_k of each curved link, slot (x, 26 - k).  One wave
// per tile entry.
template <int ST>
__global__ __launch_bounds__(256) void k_curved_refresh(KDomain d, const TileRec *__restrict__ tiles, uint32_t ntiles)
{
    using S = Storage<ST>;
    constexpr uint32_t es = S::bytes;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t t = __builtin_amdgcn_readfirstlane(blockIdx.x * 4u + (threadIdx.x >> 6));
    if (t >= ntiles)
        return;
    const TileRec rec = tiles[t];
    if (rec.wall < 0 || !rec.bz || !lane_active(rec, lane))
        return;
    const Pops<ST, true> r(d);
    const uint64_t self = cell_bytes<es, uint64_t>(rec.tile * 64u + lane, d.tbytes);
    float f[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k)
        f[k] = ((rec.bz >> k) & 1u) ? r.load(self, pop_bytes<es>(Q - 1 - k), k) : 0.f;
    curved_keep(d, rec, lane, f);
}

// f = f^eq(rho, u) in product form: the sixth-order Hermite equilibrium of
// Eq. (4) factorises into rho prod_a phi(c_a, u_a), phi(0, u) = 2/3 - u^2,
// phi(+-1, u) = (1 +- 3u + 3u^2)/6 (App. A, Eqs. (A.2)-(A.4)).  Written in
// the phase-0 form; cells that are not updated get the rest state.
template <int ST>
__global__ __launch_bounds__(256) void k_init_eq(KDomain d, const float *__restrict__ rho, const float *__restrict__ u)
{
    using S = Storage<ST>;
    constexpr uint32_t es = S::bytes;
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.P)
        return;
    float r = 1.f, v[3] = {0.f, 0.f, 0.f};
    bool upd = false;
    if (c < d.ncells) {
        upd = d.flags[c] == FL_FLUID || d.flags[c] == FL_OUTLET;
        if (upd) {
            if (rho)
                r = rho[c];
            if (u) {
                v[0] = u[c];
                v[1] = u[(size_t)d.ncells + c];
                v[2] = u[2 * (size_t)d.ncells + c];
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
    const Pops<ST, true> rr(d);
    const uint64_t cb = cell_bytes<es, uint64_t>(c, d.tbytes);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const float fe = upd ? r * phi[0][i % 3] * phi[1][(i / 3) % 3] * phi[2][i / 9] : weight(i);
        rr.store(cb, pop_bytes<es>(Q - 1 - i), fe, i);
    }
}

// Density and velocity of a phase-0 state at updated cells (0 elsewhere).
template <int ST>
__global__ __launch_bounds__(256) void k_moments(KDomain d, float *__restrict__ rho, float *__restrict__ u)
{
    using S = Storage<ST>;
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.ncells)
        return;
    float r = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
    if (d.flags[c] == FL_FLUID || d.flags[c] == FL_OUTLET) {
        const Pops<ST, true> rr(d);
        const uint64_t cb = cell_bytes<S::bytes, uint64_t>(c, d.tbytes);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const float fi = rr.load(cb, pop_bytes<S::bytes>(Q - 1 - i), i);
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
    u[(size_t)d.ncells + c] = jy;
    u[2 * (size_t)d.ncells + c] = jz;
}

#ifdef LBM_HOST_TU
// Means of the statistics sums (scale = 1 / samples) to [component][cell]
// arrays (3 for u, 6 for u_a u_b, 6 for sigma); cells that are not updated
// are left as they are (the host zeroes the outputs).  One wave per tile.
__global__ __launch_bounds__(256) void k_stats_export(KDomain d, const TileRec *__restrict__ tiles, uint32_t ntiles,
                                                      double scale, double *__restrict__ out)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t t = __builtin_amdgcn_readfirstlane(blockIdx.x * 4u + (threadIdx.x >> 6));
    if (t >= ntiles)
        return;
    const TileRec rec = tiles[t];
    if (!lane_active(rec, lane) && rec.wall >= 0)
        return;
    const uint32_t cell = rec.tile * 64u + lane;
    if (cell >= d.ncells)
        return;
    for (int c = 0; c < 15; ++c)
        out[(size_t)c * d.ncells + cell] = d.stats[(size_t)c * d.sstride + rec.ord * 64u + lane] * scale;
}

#endif // LBM_HOST_TU

// Phase-0 state <-> FP32 values of f_i, layout [i][cell] without padding.
template <int ST>
__global__ __launch_bounds__(256) void k_export(KDomain d, float *__restrict__ out)
{
    using S = Storage<ST>;
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.ncells)
        return;
    const Pops<ST, true> rr(d);
    const uint64_t cb = cell_bytes<S::bytes, uint64_t>(c, d.tbytes);
#pragma unroll
    for (int i = 0; i < Q; ++i)
        out[(size_t)i * d.ncells + c] = rr.load(cb, pop_bytes<S::bytes>(Q - 1 - i), i);
}

template <int ST>
__global__ __launch_bounds__(256) void k_import(KDomain d, const float *__restrict__ in)
{
    using S = Storage<ST>;
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.ncells)
        return;
    const Pops<ST, true> rr(d);
    const uint64_t cb = cell_bytes<S::bytes, uint64_t>(c, d.tbytes);
#pragma unroll
    for (int i = 0; i < Q; ++i)
        rr.store(cb, pop_bytes<S::bytes>(Q - 1 - i), in[(size_t)i * d.ncells + c], i);
}

} // namespace lbm
