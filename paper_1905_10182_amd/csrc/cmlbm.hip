// libcmlbm: MI355X (gfx950) D3Q27 central-moment lattice Boltzmann solver with
// Hermite-expanded external forcing (De Rosis, Huang & Coreixas, PRE 2019,
// Sec. II).  C ABI in include/cmlbm.h.
//
// Kernels
//   k_step       fused pull-stream gather + collision + store (the hot path);
//                with RED also the FP64 partial sums of the state it reads
//   k_red_waves  second level of those sums
//   k_init       inverse of the gather: writes a given pre-collision state
//   k_gather     rho/u or FP64 populations from the current state
//   k_reduce     per-block FP64 partial sums; k_reduce_final finishes them
//   k_linkmask   per-cell 27-bit bounce-back mask from walls and solid nodes
//   k_fill       plain fill (used instead of memset so work stays in kernels)
//
// Memory layout in HBM: every population is stored in rows of nxp elements
// (nx rounded up to 256 bytes), one value per cell, rows ordered
// [nbatch][nz][ny].  Population storage keeps the 27 population rows of one
// lattice row together (row blocks, [nbatch][nz][ny][27][nxp]); moment
// storage keeps planes ([9][nbatch][nz][ny][nxp], planes kPlanePad bytes
// apart beyond their rows).  Two such buffers alternate between steps.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "cmlbm.h"
#include "d3q27.hpp"

using namespace cmlbm;

namespace {

constexpr int kBlock = 256;   // threads per workgroup of every kernel
constexpr int kNPart = 10;    // partial-sum slots of k_reduce
// collision model bits of k_step (0: the method's closed-form collision)
constexpr int kModelGuo = 1;  // second-order forcing term
constexpr int kModelEq2 = 2;  // second-order equilibrium
constexpr int kModelBgk = 4;  // single relaxation time
constexpr int kMaxRedBlocks = 2048;  // reduce workgroups per batch member (half that for FP64 storage)
constexpr uint32_t kSolidBit = 1u << 27;
constexpr size_t kPlanePad = 4096;  // bytes between consecutive population planes (a multiple of 256)

// ---------------------------------------------------------------------------
// storage types

template <int ST>
struct storage;
// Every storage type also offers load_raw / pack_raw (/ pack_sr_raw): the
// stored number itself, which for FP16 is 256 h (kScale); the step kernel
// computes on that scale.
template <>
struct storage<CMLBM_FP64> {
    typedef double S;
    typedef double T;
    static constexpr T kScale = 1;
    static __device__ __forceinline__ T load(const S* p) { return *p; }
    static __device__ __forceinline__ S pack(T v) { return v; }
    static __device__ __forceinline__ T load_raw(const S* p) { return *p; }
    static __device__ __forceinline__ S pack_raw(T v) { return v; }
};
template <>
struct storage<CMLBM_FP32> {
    typedef float S;
    typedef float T;
    static constexpr T kScale = 1;
    static __device__ __forceinline__ T load(const S* p) { return *p; }
    static __device__ __forceinline__ S pack(T v) { return v; }
    static __device__ __forceinline__ T load_raw(const S* p) { return *p; }
    static __device__ __forceinline__ S pack_raw(T v) { return v; }
};
// 16-bit formats.  pack() rounds to nearest even.  pack_sr_raw() rounds
// stochastically with gfx950's conversion instructions (v_cvt_sr_f16_f32,
// v_cvt_sr_bf16_f32): the value goes to the 16-bit neighbour further from
// zero with probability equal to its fractional position between the two
// neighbours, the position being compared with the top bits of the 32-bit
// random operand -- the 13 (FP16) or 16 (BF16) discarded significand bits'
// worth (checked on the hardware: a value half-way between two neighbours
// rounds up exactly when bit 31 is set, and over random operands a value at
// 0.3 / 0.7 of the way rounds up with frequency 0.300 / 0.702).  An unbiased
// rounding.  pack2_sr_raw() converts two values into one packed pair, each
// with its own random operand.  FP16 values carry a factor 2^8 (h * 256 is
// stored) so that even the smallest shifted populations stay in FP16's
// normal range.
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf162_t __attribute__((ext_vector_type(2)));
template <>
struct storage<CMLBM_FP16> {
    typedef _Float16 S;
    typedef float T;
    static constexpr T kScale = 256;
    static __device__ __forceinline__ T load(const S* p) { return (float)*p * 0.00390625f; }
    static __device__ __forceinline__ S pack(T v) { return (_Float16)(v * 256.0f); }
    static __device__ __forceinline__ T load_raw(const S* p) { return (float)*p; }
    static __device__ __forceinline__ S pack_raw(T v) { return (_Float16)v; }
    static __device__ __forceinline__ S pack_sr_raw(T v, uint32_t rnd)
    {
        half2_t x = __builtin_amdgcn_cvt_sr_f16_f32(__builtin_bit_cast(half2_t, v), v, rnd, false);
        return x[0];
    }
    static __device__ __forceinline__ half2_t pack2_sr_raw(T a, T b, uint32_t ra, uint32_t rb)
    {
        half2_t x = __builtin_amdgcn_cvt_sr_f16_f32(__builtin_bit_cast(half2_t, a), a, ra, false);
        return __builtin_amdgcn_cvt_sr_f16_f32(x, b, rb, true);
    }
};
template <>
struct storage<CMLBM_BF16> {
    typedef __bf16 S;
    typedef float T;
    static constexpr T kScale = 1;
    static __device__ __forceinline__ T load(const S* p) { return (float)*p; }
    static __device__ __forceinline__ S pack(T v) { return (__bf16)v; }
    static __device__ __forceinline__ T load_raw(const S* p) { return load(p); }
    static __device__ __forceinline__ S pack_raw(T v) { return pack(v); }
    static __device__ __forceinline__ S pack_sr_raw(T v, uint32_t rnd)
    {
        bf162_t x = __builtin_amdgcn_cvt_sr_bf16_f32(__builtin_bit_cast(bf162_t, v), v, rnd, false);
        return x[0];
    }
    static __device__ __forceinline__ bf162_t pack2_sr_raw(T a, T b, uint32_t ra, uint32_t rb)
    {
        bf162_t x = __builtin_amdgcn_cvt_sr_bf16_f32(__builtin_bit_cast(bf162_t, a), a, ra, false);
        return __builtin_amdgcn_cvt_sr_bf16_f32(x, b, rb, true);
    }
};

// moment representation: nine FP32 planes (rho - rho0, u, (1 - omega) k4..k8)
template <>
struct storage<CMLBM_MOM32> {
    typedef float S;
    typedef float T;
};

// Counter-based random bits for stochastic rounding: one hashed 32-bit seed
// h per (lane, step) -- a 32-bit integer finaliser (xor-shift / multiply
// rounds) of the linear index of the lane's first cell and the step -- then 7
// words per cell, word k = h + k * 0x9E3779B9 (a Weyl sequence: one add per
// word; sr_words); population i of a cell takes word i / 4 rotated so that its
// byte i % 4 is on top (sr_operand).  Every operand is uniform, and operands
// of different cells or steps are independent.  Within a cell they are
// related: the conversion reads the top 13 or 16 bits, so two populations of
// one word share the low-order bits of their thresholds, and the same byte of
// consecutive words differs by a constant (plus a carry).  Each population's
// rounding stays unbiased; the words cost 13 adds per lane instead of an
// xorshift chain's 84 operations.
__device__ __forceinline__ uint32_t mix32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

template <int V>
__device__ __forceinline__ void sr_words(uint32_t lin0, uint32_t step, uint32_t rw[V][7])
{
    const uint32_t w = mix32(lin0 ^ mix32(step * 0x9E3779B9u + 0x632BE5ABu));
#pragma unroll
    for (int c = 0; c < V; ++c)
#pragma unroll
        for (int k = 0; k < 7; ++k) rw[c][k] = w + (uint32_t)(7 * c + k) * 0x9E3779B9u;
}

__device__ __forceinline__ uint32_t sr_operand(const uint32_t rw[7], int i)
{
    return __builtin_rotateright32(rw[i / 4], (uint32_t)(8 * (i % 4) + 8) & 31u);
}

size_t storage_bytes(int st) { return st == CMLBM_FP64 ? 8 : (st == CMLBM_FP32 || st == CMLBM_MOM32) ? 4 : 2; }
int planes_of(int st) { return st == CMLBM_MOM32 ? 9 : 27; }

// ---------------------------------------------------------------------------
// geometry passed to every kernel

struct Geom {
    int nx, ny, nz, nb;
    int nxp;           // padded row length (elements)
    int rows;          // ny * nz * nb
    int xblocks;       // workgroups along x per row group
    int bx, by;        // workgroup shape: bx threads along x (multiple of 64), by rows
    uint64_t pstride;  // elements from population i to i + 1 of one row
    uint64_t rstride;  // elements from one row of a population to the next row
    uint64_t ncell;    // nb * nz * ny * nx (unpadded)
};

struct Cell {
    int x, y, z, b;
    bool valid;
    uint32_t own;     // padded index within a plane (the link mask's index)
    uint64_t pown;    // index of the cell's population 0 (population i at + i * pstride)
    uint64_t lin;     // unpadded linear index
};

// Cell of this thread.  Each wave lies within one row (bx is a multiple of 64),
// so y, z, b are wave-uniform and live in scalar registers.
__device__ __forceinline__ Cell locate(const Geom& g)
{
    Cell c;
    const int blk = blockIdx.x;
    const int xb = blk % g.xblocks;
    const int rb = blk / g.xblocks;
    int row = rb * g.by + (int)threadIdx.y;
    row = __builtin_amdgcn_readfirstlane(row);
    c.x = xb * g.bx + (int)threadIdx.x;
    c.valid = row < g.rows && c.x < g.nx;
    const int y = row % g.ny;
    const int zb = row / g.ny;
    c.y = y;
    c.z = zb % g.nz;
    c.b = zb / g.nz;
    c.own = (uint32_t)row * (uint32_t)g.nxp + (uint32_t)c.x;
    c.pown = (uint64_t)row * g.rstride + (uint64_t)c.x;
    c.lin = (uint64_t)row * (uint64_t)g.nx + (uint64_t)c.x;
    return c;
}

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Source offsets (relative to population 0) of the pull gather for the 27
// directions: direction i reads cell x - c_i with periodic wrap.
struct Pull {
    uint64_t rowoff[3][3];  // [cy+1][cz+1] offset of the source row (wave-uniform)
    uint32_t xs[3];         // [cx+1] source x
};

__device__ __forceinline__ Pull make_pull(const Geom& g, const Cell& c)
{
    Pull p;
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int ys = wrap(c.y - (b - 1), g.ny);
            const int zs = wrap(c.z - (d - 1), g.nz);
            p.rowoff[b][d] = (uint64_t)((c.b * g.nz + zs) * g.ny + ys) * g.rstride;
        }
#pragma unroll
    for (int a = 0; a < 3; ++a) p.xs[a] = (uint32_t)wrap(c.x - (a - 1), g.nx);
    return p;
}

// A wave-uniform global pointer made opaque to the optimiser: it stays a
// scalar base of the "saddr + voffset" access form instead of being folded
// with the per-lane offset into a 64-bit vector address.
typedef __attribute__((address_space(1))) char gchar;
template <typename P>
__device__ __forceinline__ gchar* uniform_ptr(P* p)
{
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (gchar*)(((uint64_t)hi << 32) | lo);
}

// Raw buffer access for 4-byte vectors: a descriptor in four scalar registers
// (wave-uniform base, stride 0, size in bytes, the gfx9 raw-buffer format
// word) and a 32-bit per-lane byte offset, added to the base by the memory
// unit instead of by a 64-bit VALU add per access.  Offsets stay below the
// size (one padded row), so the range check never drops an access.
constexpr int kRawBufferWord3 = 0x00020000;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(gchar* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)bytes, kRawBufferWord3);
}
template <typename X>
__device__ __forceinline__ X ld_buf(gchar* base, uint32_t bytes, uint32_t byte_off)
{
    static_assert(sizeof(X) == 4, "4-byte buffer loads only");
    return __builtin_bit_cast(X, __builtin_amdgcn_raw_buffer_load_b32(row_rsrc(base, bytes), byte_off, 0, 0));
}
// aux bit 1: the non-temporal hint (nt) on gfx94x / gfx950
template <bool NT, typename X>
__device__ __forceinline__ void st_buf(gchar* base, uint32_t bytes, uint32_t byte_off, X v)
{
    static_assert(sizeof(X) == 4, "4-byte buffer stores only");
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), row_rsrc(base, bytes), byte_off, 0,
                                          NT ? 2 : 0);
}

// load of the X at byte_off from base
template <typename X>
__device__ __forceinline__ X ld_off(const void* base, uint32_t byte_off)
{
    return *(const X*)((const char*)base + byte_off);
}

// Gather the 27 shifted pre-collision populations of one cell.
template <int ST, bool MASK>
__device__ __forceinline__ void gather(const typename storage<ST>::S* __restrict__ src, const Geom& g,
                                       const Cell& c, uint32_t m, typename storage<ST>::T h[27])
{
    using SS = storage<ST>;
    const Pull p = make_pull(g, c);
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        const uint64_t off = p.rowoff[vel_y(i) + 1][vel_z(i) + 1] + p.xs[vel_x(i) + 1];
        if (MASK) {
            const bool bounce = (m >> i) & 1u;
            const uint64_t e = bounce ? (uint64_t)opposite(i) * g.pstride + c.pown : (uint64_t)i * g.pstride + off;
            h[i] = SS::load(src + e);
        } else {
            // wave-uniform source row plus a 32-bit per-lane byte offset (the
            // "saddr + voffset" load form; the row arithmetic stays scalar)
            const typename SS::S* row = src + (uint64_t)i * g.pstride + p.rowoff[vel_y(i) + 1][vel_z(i) + 1];
            typename SS::S e = ld_off<typename SS::S>(row, p.xs[vel_x(i) + 1] * (uint32_t)sizeof(typename SS::S));
            h[i] = SS::load(&e);
        }
    }
}

// ---------------------------------------------------------------------------
// the hot path: one time step

// ---------------------------------------------------------------------------
// cross-lane shifts for the vectorised row access of k_step

// lane l receives the value of lane l-1 (mod 64) / lane l+1 (mod 64)
__device__ __forceinline__ int dpp_from_prev(int v) { return __builtin_amdgcn_mov_dpp(v, 0x13C, 0xF, 0xF, false); }
__device__ __forceinline__ int dpp_from_next(int v) { return __builtin_amdgcn_mov_dpp(v, 0x134, 0xF, 0xF, false); }

template <typename S>
__device__ __forceinline__ S lane_shift(S v, bool from_prev)
{
    if constexpr (sizeof(S) == 4) {
        const int r = from_prev ? dpp_from_prev(__builtin_bit_cast(int, v)) : dpp_from_next(__builtin_bit_cast(int, v));
        return __builtin_bit_cast(S, r);
    } else if constexpr (sizeof(S) == 8) {
        const int2 w = __builtin_bit_cast(int2, v);
        int2 r;
        r.x = from_prev ? dpp_from_prev(w.x) : dpp_from_next(w.x);
        r.y = from_prev ? dpp_from_prev(w.y) : dpp_from_next(w.y);
        return __builtin_bit_cast(S, r);
    } else {
        const int w = (int)__builtin_bit_cast(unsigned short, v);
        const int r = from_prev ? dpp_from_prev(w) : dpp_from_next(w);
        return __builtin_bit_cast(S, (unsigned short)r);
    }
}

// ---------------------------------------------------------------------------
// the hot path: one fused time step
//
// Every cell pulls its 27 populations from x - c_i (eq. "streaming" read
// backwards), collides in central-moment space (collide() in d3q27.hpp) and
// stores its 27 post-collision populations at its own index with
// non-temporal stores (they are not read again in this step).
//
// Wave w owns segment (w mod segs) of row (w / segs): 64 lanes x V cells.
// With V > 1 a lane reads every plane as one aligned V-element vector; the
// 18 populations with c_x = +-1 need the row shifted by one cell, done in
// registers: the element crossing a lane boundary comes from the neighbouring
// lane by a DPP wave rotation (which also performs the periodic wrap when a
// row is exactly one wave), and the lanes at the ends of a segment otherwise
// reload that one element.
// All row-dependent address arithmetic is wave-uniform and lives in scalar
// registers; each access is a scalar base pointer plus a 32-bit per-lane byte
// offset (one of three x offsets for the loads, one for every store), which
// maps onto the global_load/store "saddr + voffset" form.  Needs per-plane
// byte offsets below 4 GiB.

template <bool NT, typename X>
__device__ __forceinline__ void st_off(gchar* base, uint32_t byte_off, X v)
{
    gchar* p = base + byte_off;
    typedef __attribute__((address_space(1))) X gX;
    if constexpr (NT) {
        if constexpr (sizeof(X) == 16) {
            typedef int i4 __attribute__((ext_vector_type(4)));
            typedef __attribute__((address_space(1))) i4 gi4;
            __builtin_nontemporal_store(__builtin_bit_cast(i4, v), (gi4*)p);
        } else if constexpr (sizeof(X) == 8) {
            __builtin_nontemporal_store(__builtin_bit_cast(unsigned long long, v),
                                        (__attribute__((address_space(1))) unsigned long long*)p);
        } else if constexpr (sizeof(X) == 4) {
            __builtin_nontemporal_store(__builtin_bit_cast(unsigned, v), (__attribute__((address_space(1))) unsigned*)p);
        } else {
            __builtin_nontemporal_store(__builtin_bit_cast(unsigned short, v),
                                        (__attribute__((address_space(1))) unsigned short*)p);
        }
    } else {
        *(gX*)p = v;
    }
}

// Threads per k_step workgroup: 1024 for FP32 storage, 512 for FP64 without a
// bounce-back mask, 256 otherwise (measured best for each; the grid is rows x
// segments of waves either way).
constexpr int step_block(int st, bool mask)
{
    return st == CMLBM_FP32 ? 1024 : (st == CMLBM_FP64 && !mask) ? 512 : 256;
}

// FP64 sum over the 64 lanes of a wave by a butterfly of lane exchanges: every
// lane ends with the same value (each level adds the same two operands), so
// the result does not depend on which lane writes it.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v = fmax(v, __shfl_xor(v, m));
    return v;
}

// One time step, one wave per 64 x V cell row segment.  With RED the step
// also forms, from the same gather, the FP64 partial sums of the state it
// reads (the quantities of k_reduce, from the per-cell values of the step's
// own arithmetic) and writes them for this wave to wpart[wave][kNPart]; every
// lane then stays live until that wave-wide sum, and lanes without a fluid
// cell only skip their contributions and stores.  (RED is a template flag of
// the kernel itself: a shared device function changed the register
// allocation of the RED = false kernels.)
template <int ST, int V, bool MASK, bool FIELD, bool NT, int MODEL, bool RED, bool SR>
__global__ __launch_bounds__(step_block(ST, MASK)) void k_step(const typename storage<ST>::S* __restrict__ src,
                                                  typename storage<ST>::S* __restrict__ dst, Geom g, int segs,
                                                  typename storage<ST>::T omega, typename storage<ST>::T rho0,
                                                  const typename storage<ST>::T* __restrict__ ftab,
                                                  const typename storage<ST>::T* __restrict__ field,
                                                  const uint32_t* __restrict__ mask, uint32_t step,
                                                  double* __restrict__ wpart)
{
    static_assert(V == 1 || !MASK, "bounce-back masks use one cell per lane");
    static_assert(MODEL == 0 || V == 1, "comparison models use one cell per lane");
    static_assert(!RED || MODEL == 0, "fused reductions are for the method's collision");
    using SS = storage<ST>;
    using S = typename SS::S;
    using T = typename SS::T;
    static_assert(!SR || sizeof(S) == 2, "stochastic rounding is for 16-bit storage");
    // FP16 stores 256 h: the step computes on that scale, with the force
    // density and rho0 scaled alike, so its loads and stores need no
    // rescaling.  The collision is homogeneous of degree one in (h, F, rho0)
    // at fixed u and a power-of-two scale is exact, so only the compiler's
    // different choice of fused multiply-adds separates this from computing on
    // h: about one stored value in 10^5 moves by one unit in the last place.
    constexpr T kS = SS::kScale;
    const T rho0s = rho0 * kS;
    typedef S vt __attribute__((ext_vector_type(V == 1 ? 2 : V)));
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (step_block(ST, MASK) / 64) + (threadIdx.x >> 6)));
    const int row = wave / segs;
    if (row >= g.rows) return;  // whole wave
    const int seg = wave - row * segs;
    const int y = row % g.ny;
    const int zb = row / g.ny;
    const int z = zb % g.nz;
    const int b = zb / g.nz;
    const int x0 = (seg * 64 + lane) * V;
    const bool active = x0 < g.nx;
    // wave-uniform row pointers: rowp[i] = plane i at the source row of direction i
    const S* srow[3][3];
#pragma unroll
    for (int bb = 0; bb < 3; ++bb)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int ys = wrap(y - (bb - 1), g.ny);
            const int zs = wrap(z - (d - 1), g.nz);
            srow[bb][d] = src + (uint64_t)((b * g.nz + zs) * g.ny + ys) * g.rstride;
        }
    const uint32_t own_row = (uint32_t)row * (uint32_t)g.nxp;  // the link mask's row
    const uint64_t pop_row = (uint64_t)row * g.rstride;       // population 0 of this row
    T h[V][27];
    bool live = active;  // this lane holds fluid cells (RED: a lane without one stays for the wave sum)
    if constexpr (V == 1) {
        const int xa = RED && !active ? 0 : x0;  // RED: in-bounds addresses for lanes past the row end
        const uint32_t bx[3] = {(uint32_t)wrap(xa + 1, g.nx) * (uint32_t)sizeof(S), (uint32_t)xa * (uint32_t)sizeof(S),
                                (uint32_t)wrap(xa - 1, g.nx) * (uint32_t)sizeof(S)};
        uint32_t m = 0;
        if (MASK) m = active ? mask[own_row + x0] : kSolidBit;
        if constexpr (RED)
            live = active && !(m & kSolidBit);
        else if (!active || (m & kSolidBit))
            return;
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            const S* plane_row = srow[vel_y(i) + 1][vel_z(i) + 1] + (uint64_t)i * g.pstride;
            S e;
            if (MASK && ((m >> i) & 1u))
                e = ld_off<S>(src + (uint64_t)opposite(i) * g.pstride + pop_row, bx[1]);
            else
                e = ld_off<S>(plane_row, bx[vel_x(i) + 1]);
            h[0][i] = SS::load_raw(&e);
        }
    } else {
        const bool whole = g.nx == 64 * V;
        const bool prev_in_reg = whole || lane > 0;
        const bool next_in_reg = whole || (lane < 63 && x0 + V < g.nx);
        const uint32_t bxm = (uint32_t)(x0 == 0 ? g.nx - 1 : x0 - 1) * (uint32_t)sizeof(S);
        const uint32_t bxp = (uint32_t)(x0 + V >= g.nx ? 0 : x0 + V) * (uint32_t)sizeof(S);
        // (Unconditional loads -- lanes past the row end reading the row's first
        // vector -- compile to one burst of 27 loads with fewer instructions, but
        // measured 2-5% slower at 512^3 than these predicated ones.)
        const uint32_t bx0 = (uint32_t)x0 * (uint32_t)sizeof(S);
        const uint32_t rowb = (uint32_t)g.nxp * (uint32_t)sizeof(S);
        vt v[27];
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            const S* plane_row = srow[vel_y(i) + 1][vel_z(i) + 1] + (uint64_t)i * g.pstride;
            v[i] = active ? ld_buf<vt>(uniform_ptr(plane_row), rowb, bx0) : vt(0);
        }
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            if (vel_x(i) == 0) continue;
            const bool from_prev = vel_x(i) == 1;
            S e = lane_shift<S>(from_prev ? v[i][V - 1] : v[i][0], from_prev);
            const bool in_reg = from_prev ? prev_in_reg : next_in_reg;
            if (!in_reg && active) {
                const S* plane_row = srow[vel_y(i) + 1][vel_z(i) + 1] + (uint64_t)i * g.pstride;
                e = ld_off<S>(plane_row, from_prev ? bxm : bxp);
            }
            // place the shifted row into h: cell c of c_x = +1 reads element c-1, of c_x = -1 element c+1
#pragma unroll
            for (int c = 0; c < V; ++c) {
                S src_e;
                if (from_prev)
                    src_e = c == 0 ? e : v[i][c - 1];
                else
                    src_e = c == V - 1 ? e : v[i][c + 1];
                h[c][i] = SS::load_raw(&src_e);
            }
        }
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            if (vel_x(i) != 0) continue;
#pragma unroll
            for (int c = 0; c < V; ++c) {
                S e = v[i][c];
                h[c][i] = SS::load_raw(&e);
            }
        }
        if constexpr (!RED)
            if (!active) return;
    }
    T Fx[V], Fy[V], Fz[V];
    if (FIELD) {
        const uint64_t lin = (uint64_t)row * (uint64_t)g.nx + (uint64_t)(RED && !live ? 0 : x0);
#pragma unroll
        for (int c = 0; c < V; ++c) {
            Fx[c] = field[lin + c];
            Fy[c] = field[g.ncell + lin + c];
            Fz[c] = field[2 * g.ncell + lin + c];
        }
    } else {
        const T* fr = ftab + 3 * (b * g.ny + y);
#pragma unroll
        for (int c = 0; c < V; ++c) {
            Fx[c] = fr[0];
            Fy[c] = fr[1];
            Fz[c] = fr[2];
        }
    }
    if constexpr (kS != T(1))
#pragma unroll
        for (int c = 0; c < V; ++c) {
            Fx[c] *= kS;
            Fy[c] *= kS;
            Fz[c] *= kS;
        }
    T mq[RED ? V : 1][4];  // RED: each cell's drho, ux, uy, uz
#pragma unroll
    for (int c = 0; c < V; ++c) {
        T rho, ux, uy, uz;
        if constexpr (RED) {
            // collide() with its density deviation kept for the mass sum
            T drho, k5[5], s5[5];
            pre_collision(h[c], Fx[c], Fy[c], Fz[c], rho0s, drho, ux, uy, uz, k5);
#pragma unroll
            for (int j = 0; j < 5; ++j) s5[j] = (T(1) - omega) * k5[j];
            reconstruct(drho, ux, uy, uz, Fx[c], Fy[c], Fz[c], s5, rho0s, h[c]);
            mq[c][0] = drho;
            mq[c][1] = ux;
            mq[c][2] = uy;
            mq[c][3] = uz;
        } else if constexpr (MODEL == 0) {
            collide<T>(h[c], Fx[c], Fy[c], Fz[c], omega, rho0s, rho, ux, uy, uz);
        } else {
            collide_model<T, (MODEL & kModelEq2) != 0, (MODEL & kModelGuo) != 0, (MODEL & kModelBgk) != 0>(
                h[c], Fx[c], Fy[c], Fz[c], omega, rho0s, rho, ux, uy, uz);
        }
    }
    if constexpr (RED) {
        // the stores below, as a lambda so that the sums can follow them (a
        // `return` inside leaves only the stores); the plain kernels keep the
        // stores inline: routed through the lambda they were allocated more
        // registers (FP16: 76 -> 81)
        auto store_all = [&]() {
            const uint32_t bst = (uint32_t)x0 * (uint32_t)sizeof(S);
            if constexpr (sizeof(S) == 2) {
                if constexpr (SR) {
                    uint32_t rw[V][7];
                    sr_words<V>((uint32_t)((uint64_t)row * (uint64_t)g.nx + (uint64_t)x0), step, rw);
#pragma unroll
                    for (int i = 0; i < 27; ++i) {
                        gchar* plane_row = uniform_ptr(dst + (uint64_t)i * g.pstride + pop_row);
                        if constexpr (V == 1)
                            st_off<NT>(plane_row, bst, SS::pack_sr_raw(h[0][i], sr_operand(rw[0], i)));
                        else
                            st_buf<NT>(plane_row, (uint32_t)g.nxp * (uint32_t)sizeof(S), bst,
                                       SS::pack2_sr_raw(h[0][i], h[1][i], sr_operand(rw[0], i), sr_operand(rw[1], i)));
                    }
                    return;
                }
            }
#pragma unroll
            for (int i = 0; i < 27; ++i) {
                gchar* plane_row = uniform_ptr(dst + (uint64_t)i * g.pstride + pop_row);
                if constexpr (V == 1) {
                    st_off<NT>(plane_row, bst, SS::pack_raw(h[0][i]));
                } else {
                    vt o;
#pragma unroll
                    for (int c = 0; c < V; ++c) o[c] = SS::pack_raw(h[c][i]);
                    if constexpr (sizeof(vt) == 4)
                        st_buf<NT>(plane_row, (uint32_t)g.nxp * (uint32_t)sizeof(S), bst, o);
                    else
                        st_off<NT>(plane_row, bst, o);
                }
            }
        };
        if (live) store_all();
        // FP64 sums of this lane's cells, then over the wave; after the stores,
        // so that the post-collision populations are not held across them
        double acc[kNPart];
#pragma unroll
        for (int k = 0; k < kNPart; ++k) acc[k] = 0.0;
#pragma unroll
        for (int c = 0; c < V; ++c) {
            if (!live || (V > 1 && x0 + c >= g.nx)) continue;
            const double dr = (double)mq[c][0] / (double)kS;  // the density deviation, unscaled
            const double r = (double)rho0 + dr;
            const double u[3] = {(double)mq[c][1], (double)mq[c][2], (double)mq[c][3]};
            const double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
            acc[7] += 1.0;
            if (!(isfinite(r) && isfinite(u2))) {
                acc[6] += 1.0;
                continue;
            }
            acc[0] += dr;
            acc[1] += r * u[0] - 0.5 * (double)Fx[c] / (double)kS;  // sum_i f_i c_i
            acc[2] += r * u[1] - 0.5 * (double)Fy[c] / (double)kS;
            acc[3] += r * u[2] - 0.5 * (double)Fz[c] / (double)kS;
            acc[4] += 0.5 * r * u2;
            acc[5] = fmax(acc[5], sqrt(u2));
            acc[9] += u2;
        }
#pragma unroll
        for (int k = 0; k < kNPart; ++k) acc[k] = k == 5 ? wave_max(acc[k]) : wave_sum(acc[k]);
        if (lane < kNPart) {
            double v = acc[0];
#pragma unroll
            for (int k = 1; k < kNPart; ++k) v = lane == k ? acc[k] : v;
            wpart[(uint64_t)wave * kNPart + lane] = v;
        }
        return;
    }
    const uint32_t bst = (uint32_t)x0 * (uint32_t)sizeof(S);
    if constexpr (sizeof(S) == 2) {
        if constexpr (SR) {
            uint32_t rw[V][7];
            sr_words<V>((uint32_t)((uint64_t)row * (uint64_t)g.nx + (uint64_t)x0), step, rw);
#pragma unroll
            for (int i = 0; i < 27; ++i) {
                gchar* plane_row = uniform_ptr(dst + (uint64_t)i * g.pstride + pop_row);
                if constexpr (V == 1)
                    st_off<NT>(plane_row, bst, SS::pack_sr_raw(h[0][i], sr_operand(rw[0], i)));
                else
                    st_buf<NT>(plane_row, (uint32_t)g.nxp * (uint32_t)sizeof(S), bst,
                               SS::pack2_sr_raw(h[0][i], h[1][i], sr_operand(rw[0], i), sr_operand(rw[1], i)));
            }
            return;
        }
    }
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        gchar* plane_row = uniform_ptr(dst + (uint64_t)i * g.pstride + pop_row);
        if constexpr (V == 1) {
            st_off<NT>(plane_row, bst, SS::pack_raw(h[0][i]));
        } else {
            vt o;
#pragma unroll
            for (int c = 0; c < V; ++c) o[c] = SS::pack_raw(h[c][i]);
            if constexpr (sizeof(vt) == 4)
                st_buf<NT>(plane_row, (uint32_t)g.nxp * (uint32_t)sizeof(S), bst, o);
            else
                st_off<NT>(plane_row, bst, o);
        }
    }
}

// ---------------------------------------------------------------------------
// initialisation: scatter a pre-collision state through the inverse gather

enum InitSrc { INIT_EQ_F64 = 0, INIT_EQ_F32 = 1, INIT_POPS_F64 = 2 };

// Complete 27-Hermite equilibrium (eq. "eq:truncation") in deviation form,
// e_i = f^eq_i - w_i rho0.  It factors over the axes as
// w_i rho prod_a (1 + c_a u_a / cs^2 + (c_a^2 - cs^2) u_a^2 / (2 cs^4)), evaluated
// as w_i [drho P_i + rho0 (P_i - 1)] to keep the deviation small.
template <typename T>
__device__ __forceinline__ void feq_dev(T drho, const T u[3], T rho0, T e[27])
{
    T am[3][3];  // am[axis][c+1] = P_axis(c) - 1
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const T uu = u[a];
        am[a][0] = T(-3) * uu + T(3) * uu * uu;
        am[a][1] = T(-1.5) * uu * uu;
        am[a][2] = T(3) * uu + T(3) * uu * uu;
    }
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        const T ax = am[0][vel_x(i) + 1], ay = am[1][vel_y(i) + 1], az = am[2][vel_z(i) + 1];
        const T pm1 = ax + ay + az + ax * ay + ax * az + ay * az + ax * ay * az;
        e[i] = (T)weight(i) * (drho * (T(1) + pm1) + rho0 * pm1);
    }
}

template <int ST, bool MASK, int SRC>
__global__ __launch_bounds__(kBlock) void k_init(typename storage<ST>::S* __restrict__ dst, Geom g, double rho0,
                                                 const void* __restrict__ rho_in, const void* __restrict__ u_in,
                                                 const double* __restrict__ pops, const uint32_t* __restrict__ mask)
{
    using SS = storage<ST>;
    using T = typename SS::T;
    const Cell c = locate(g);
    if (!c.valid) return;
    uint32_t m = 0;
    if (MASK) {
        m = mask[c.own];
        if (m & kSolidBit) return;
    }
    T e[27];
    if (SRC == INIT_POPS_F64) {
#pragma unroll
        for (int i = 0; i < 27; ++i) e[i] = (T)(pops[(uint64_t)i * g.ncell + c.lin] - weight(i) * rho0);
    } else {
        // complete 27-Hermite equilibrium
        T drho, u[3];
        if (SRC == INIT_EQ_F64) {
            const double* R = (const double*)rho_in;
            const double* U = (const double*)u_in;
            drho = R ? (T)(R[c.lin] - rho0) : T(0);
            for (int a = 0; a < 3; ++a) u[a] = U ? (T)U[a * g.ncell + c.lin] : T(0);
        } else {
            const float* R = (const float*)rho_in;
            const float* U = (const float*)u_in;
            drho = R ? (T)((double)R[c.lin] - rho0) : T(0);
            for (int a = 0; a < 3; ++a) u[a] = U ? (T)U[a * g.ncell + c.lin] : T(0);
        }
        feq_dev<T>(drho, u, (T)rho0, e);
    }
    const Pull p = make_pull(g, c);
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        const uint64_t off = p.rowoff[vel_y(i) + 1][vel_z(i) + 1] + p.xs[vel_x(i) + 1];
        const bool bounce = MASK && ((m >> i) & 1u);
        const uint64_t d = bounce ? (uint64_t)opposite(i) * g.pstride + c.pown : (uint64_t)i * g.pstride + off;
        dst[d] = SS::pack(e[i]);
    }
}

// ---------------------------------------------------------------------------
// moment-representation storage (CMLBM_MOM32)
//
// The state is the post-collision state of the current time t, kept as the
// nine numbers it is made of: m = (rho - rho0, u, s4..s8 = (1 - omega) k4..k8),
// FP32 planes [9][nb][nz][ny][nxp].  With the force density they determine the
// post-collision populations (reconstruct()), so a step moves 9 values per
// cell instead of 27 each way:
//   reconstruct f*(t) for a tile and a one-cell halo in LDS, pull
//   f(x, t + 1) = f*(x - c_i, t) from there, collide (pre_collision()) and
//   store m of t + 1.
// Workgroup: a 64 x 6 (x, y) tile marching up a chunk of kMomZC planes.  The
// 66 x 8 halo tile of a plane is reconstructed by 9 waves (waves 0-7 rows
// 0-7, columns 1-64; wave 8 the two edge columns of the 8 rows), one cell per
// lane.  LDS keeps populations by their c_z class: c_z = +1 of the two
// previous planes, c_z = 0 of the current plane, c_z = -1 of the next one, so
// every plane of the chunk (and the two halo planes) is reconstructed once.
// Waves 1-6 then collide the 64 x 6 interior cells of the current plane.

constexpr int kMomTX = 64, kMomHX = kMomTX + 2;
constexpr int kMomZC = 32;  // planes per workgroup

template <int HY>
__device__ __forceinline__ int mom_lds(int j, int hy, int hx) { return (j * HY + hy) * kMomHX + hx; }

template <bool FIELD>
__device__ __forceinline__ void mom_force(const Geom& g, uint64_t lin, int b, int y, const float* __restrict__ ftab,
                                          const float* __restrict__ field, float F[3])
{
    if (FIELD) {
        F[0] = field[lin];
        F[1] = field[g.ncell + lin];
        F[2] = field[2 * g.ncell + lin];
    } else {
        const float* fr = ftab + 3 * (b * g.ny + y);
        F[0] = fr[0];
        F[1] = fr[1];
        F[2] = fr[2];
    }
}

__device__ __forceinline__ void mom_store(float* __restrict__ dst, uint64_t pstride, uint64_t off, float drho,
                                          float ux, float uy, float uz, const float k[5], float om1)
{
    __builtin_nontemporal_store(drho, dst + off);
    __builtin_nontemporal_store(ux, dst + pstride + off);
    __builtin_nontemporal_store(uy, dst + 2 * pstride + off);
    __builtin_nontemporal_store(uz, dst + 3 * pstride + off);
#pragma unroll
    for (int j = 0; j < 5; ++j) __builtin_nontemporal_store(om1 * k[j], dst + (4 + j) * pstride + off);
}

// The same nine stores into one z plane of each moment: plane_k = dst + k *
// pstride (+ the plane's wave-uniform start), a 32-bit byte offset within it.
__device__ __forceinline__ void mom_store_plane(float* __restrict__ plane0, uint64_t pstride, uint32_t bytes,
                                                uint32_t byte_off, float drho, float ux, float uy, float uz,
                                                const float k[5], float om1)
{
    const float v[9] = {drho, ux, uy, uz, om1 * k[0], om1 * k[1], om1 * k[2], om1 * k[3], om1 * k[4]};
#pragma unroll
    for (int j = 0; j < 9; ++j) st_buf<true>((gchar*)(plane0 + j * pstride), bytes, byte_off, v[j]);
}

// TY interior rows per tile: TY + 2 halo rows reconstructed by waves 0..TY+1,
// the two edge columns of those rows by wave TY + 2.
template <bool FIELD, int TY>
__global__ __launch_bounds__((TY + 3) * 64) void k_step_mom(const float* __restrict__ src, float* __restrict__ dst,
                                                            Geom g, float omega, float rho0,
                                                            const float* __restrict__ ftab,
                                                            const float* __restrict__ field, int gens, int cpx)
{
    constexpr int HY = TY + 2;
    constexpr int SLOT = 9 * HY * kMomHX;  // floats: one c_z class of one halo plane
    __shared__ float sp[2][SLOT];          // c_z = +1 populations, by plane parity
    __shared__ float s0[SLOT];             // c_z = 0 populations of the current plane
    __shared__ float sm[SLOT];             // c_z = -1 populations of the next plane
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // Workgroups are dealt round-robin to the 8 XCDs; each XCD runs cpx of
    // them at a time (one per CU).
    const int ntx = (g.nx + kMomTX - 1) / kMomTX, nty = (g.ny + TY - 1) / TY;
    const int nzc = (g.nz + kMomZC - 1) / kMomZC;
    int tx, ty, b, zc;
    if (gens > 0) {
        // blocked schedule (cpx a multiple of ntx): a generation of an XCD is
        // cpx tiles covering the full x extent and cpx / ntx tile rows, all
        // starting together, so the halo rows and columns they share are read
        // from that XCD's L2; the XCD's next generation takes the same tiles
        // one z chunk up (the two planes around the chunk boundary are still
        // in L2).  Each XCD holds `gens` consecutive (member, y block, z chunk)
        // triples, z chunk fastest.
        const int xcd = (int)(blockIdx.x & 7u), k = (int)(blockIdx.x >> 3);
        const int by = cpx / ntx, nyb = (nty + by - 1) / by;
        const int pair = xcd * gens + k / cpx, slot = k % cpx;
        if (pair >= g.nb * nyb * nzc) return;
        zc = pair % nzc;
        b = pair / (nzc * nyb);
        tx = slot % ntx;
        ty = ((pair / nzc) % nyb) * by + slot / ntx;
        if (ty >= nty) return;
    } else {
        // tiles numbered x fastest, then y, then (member, z chunk); each XCD
        // takes a contiguous run, so neighbours share halo lines in one L2
        const unsigned total = gridDim.x;
        unsigned tile = blockIdx.x;
        if (total % 8 == 0) tile = (tile & 7u) * (total >> 3) + (tile >> 3);
        tx = (int)(tile % ntx);
        ty = (int)((tile / ntx) % nty);
        const int bzc = (int)(tile / (ntx * nty));
        b = bzc / nzc;
        zc = bzc % nzc;
    }
    const int x0 = tx * kMomTX;
    const int y0 = ty * TY;
    const int zs = zc * kMomZC;
    const int ze = zs + kMomZC < g.nz ? zs + kMomZC : g.nz;
    const int nxi = g.nx - x0 < kMomTX ? g.nx - x0 : kMomTX;
    const int nyi = g.ny - y0 < TY ? g.ny - y0 : TY;
    // reconstruction role: halo cell (hy, hx) of the 66 x HY tile; the right and
    // bottom halo follow the last interior column / row of a partial tile
    int hy, hx;
    bool rec;
    if (wave < HY) {
        hy = wave;
        hx = lane + 1;
        rec = lane < nxi && hy <= nyi + 1;
    } else {
        hy = lane >> 1;
        hx = (lane & 1) ? nxi + 1 : 0;
        rec = lane < 2 * HY && hy <= nyi + 1;
    }
    const int gx = wrap(x0 + hx - 1, g.nx), gy = wrap(y0 + hy - 1, g.ny);
    // collision role: interior cell (wave, lane + 1), waves 1..TY
    const bool inter = wave >= 1 && wave <= nyi && lane < nxi;
    const int iy = y0 + wave - 1, ix = x0 + lane;
    const float om1 = 1.f - omega;
    auto row_of = [&](int z, int y) -> uint64_t { return ((uint64_t)(b * g.nz + z) * g.ny + y) * g.nxp; };
    auto lin_of = [&](int z, int y, int x) -> uint64_t { return ((uint64_t)(b * g.nz + z) * g.ny + y) * g.nx + x; };
    // loads and stores address one z plane of a moment (wave-uniform start,
    // ny * nxp floats) with a loop-invariant 32-bit lane offset
    const uint32_t plane_bytes = (uint32_t)g.ny * (uint32_t)g.nxp * 4u;
    const uint32_t rec_off = ((uint32_t)gy * (uint32_t)g.nxp + (uint32_t)gx) * 4u;
    const uint32_t int_off = ((uint32_t)(inter ? iy : 0) * (uint32_t)g.nxp + (uint32_t)ix) * 4u;
    // the force field the same way, in its unpadded [3][cells] layout
    const uint32_t fplane_bytes = (uint32_t)g.ny * (uint32_t)g.nx * 4u;
    const uint32_t rec_foff = ((uint32_t)gy * (uint32_t)g.nx + (uint32_t)gx) * 4u;
    const uint32_t int_foff = ((uint32_t)(inter ? iy : 0) * (uint32_t)g.nx + (uint32_t)ix) * 4u;
    auto field_at = [&](int z, uint32_t off, float F[3]) {
        const float* p0 = field + lin_of(z, 0, 0);
#pragma unroll
        for (int a = 0; a < 3; ++a) F[a] = ld_buf<float>((gchar*)(p0 + a * g.ncell), fplane_bytes, off);
    };

    float mreg[9], freg[3] = {0.f, 0.f, 0.f};
    auto load_m = [&](int zu) {
        if (!rec) return;
        const int z = wrap(zu, g.nz);
        const float* plane0 = src + row_of(z, 0);
#pragma unroll
        for (int k = 0; k < 9; ++k) mreg[k] = ld_buf<float>((gchar*)(plane0 + k * g.pstride), plane_bytes, rec_off);
        if (FIELD) field_at(z, rec_foff, freg);
    };
    float h[27];
    auto recon = [&]() {
        float F[3];
        if (FIELD) {
            F[0] = freg[0];
            F[1] = freg[1];
            F[2] = freg[2];
        } else {
            mom_force<false>(g, 0, b, gy, ftab, field, F);
        }
        const float sh[5] = {mreg[4], mreg[5], mreg[6], mreg[7], mreg[8]};
        reconstruct<float>(mreg[0], mreg[1], mreg[2], mreg[3], F[0], F[1], F[2], sh, rho0, h);
    };
    auto put = [&](float* slot, int cz) {
#pragma unroll
        for (int i = 0; i < 27; ++i)
            if (vel_z(i) == cz) slot[mom_lds<HY>((vel_y(i) + 1) * 3 + vel_x(i) + 1, hy, hx)] = h[i];
    };

    // prologue: c_z = +1 populations of plane zs - 1, c_z = +1 and 0 of plane zs
    load_m(zs - 1);
    if (rec) {
        recon();
        put(sp[(zs - 1) & 1], 1);
    }
    load_m(zs);
    if (rec) {
        recon();
        put(sp[zs & 1], 1);
        put(s0, 0);
    }
    load_m(zs + 1);
    for (int z = zs; z < ze; ++z) {
        // plane z + 1 from the prefetched numbers; then prefetch plane z + 2
        if (rec) recon();
        if (z + 2 <= ze) load_m(z + 2);
        if (rec) put(sm, -1);
        __syncthreads();
        if (inter) {
            float f[27];
#pragma unroll
            for (int i = 0; i < 27; ++i) {
                const int cx = vel_x(i), cy = vel_y(i), cz = vel_z(i);
                const float* slot = cz > 0 ? sp[(z - 1) & 1] : (cz == 0 ? s0 : sm);
                f[i] = slot[mom_lds<HY>((cy + 1) * 3 + cx + 1, wave - cy, lane + 1 - cx)];
            }
            float F[3];
            if (FIELD)
                field_at(z, int_foff, F);
            else
                mom_force<false>(g, 0, b, iy, ftab, field, F);
            float drho, ux, uy, uz, k[5];
            pre_collision<float>(f, F[0], F[1], F[2], rho0, drho, ux, uy, uz, k);
            mom_store_plane(dst + row_of(z, 0), g.pstride, plane_bytes, int_off, drho, ux, uy, uz, k, om1);
        }
        __syncthreads();
        if (rec) {
            put(sp[(z + 1) & 1], 1);
            put(s0, 0);
        }
    }
}

// interior tile rows of the moment kernel: 12 when the lattice is tall enough
// (halo overhead 14/12 in y, one workgroup of 15 waves per CU), else 6
int mom_rows(const Geom& g) { return g.ny >= 24 ? 12 : 6; }

// First collision of a moment-representation state: f(x, 0) = f^eq(rho, u)
// at every cell, collided in place (cell-local), the nine numbers stored.
template <int SRC>
__global__ __launch_bounds__(kBlock) void k_init_mom(float* __restrict__ dst, Geom g, float omega, float rho0,
                                                     const void* __restrict__ rho_in, const void* __restrict__ u_in,
                                                     const float* __restrict__ ftab, const float* __restrict__ field)
{
    const Cell c = locate(g);
    if (!c.valid) return;
    float drho0, u[3];
    if (SRC == INIT_EQ_F64) {
        const double* R = (const double*)rho_in;
        const double* U = (const double*)u_in;
        drho0 = R ? (float)(R[c.lin] - rho0) : 0.f;
        for (int a = 0; a < 3; ++a) u[a] = U ? (float)U[a * g.ncell + c.lin] : 0.f;
    } else {
        const float* R = (const float*)rho_in;
        const float* U = (const float*)u_in;
        drho0 = R ? (float)((double)R[c.lin] - rho0) : 0.f;
        for (int a = 0; a < 3; ++a) u[a] = U ? U[a * g.ncell + c.lin] : 0.f;
    }
    float e[27];
    feq_dev<float>(drho0, u, rho0, e);
    float F[3];
    if (field)
        mom_force<true>(g, c.lin, c.b, c.y, ftab, field, F);
    else
        mom_force<false>(g, c.lin, c.b, c.y, ftab, field, F);
    float drho, ux, uy, uz, k[5];
    pre_collision<float>(e, F[0], F[1], F[2], rho0, drho, ux, uy, uz, k);
    mom_store(dst, g.pstride, c.pown, drho, ux, uy, uz, k, 1.f - omega);
}

// ---------------------------------------------------------------------------
// Shan-Chen pseudo-potential force (static-droplet test of Sec. III):
// F(x) = -G psi(x) sum_i w_i c_i psi(x + c_i), psi = 1 - exp(-rho), periodic.
// rho [N] and F [3][N] in the unpadded cell order of cmlbm_moments.

// Tiles of 64 x 4 cells march up a chunk of zc planes.  psi = 1 - exp(-rho) of
// each plane is computed once per tile and halo cell into a rolling window of
// four plane slots in LDS, and every cell sums its 26 neighbours from there,
// in the velocity order.  The density of the plane after next is loaded into
// registers while the current plane is summed, so the global-memory latency
// overlaps the arithmetic; with four slots one barrier per plane suffices
// (the slot a plane overwrites was last read two planes earlier, before the
// previous barrier).
constexpr int kPsiTX = 64, kPsiTY = 4;
constexpr int kPsiHX = kPsiTX + 2, kPsiHY = kPsiTY + 2, kPsiPlane = kPsiHX * kPsiHY;
static_assert(kPsiPlane <= 512 && kPsiTX * kPsiTY == 256, "each of the 256 threads owns at most two halo cells");

__device__ __forceinline__ int pmod(int v, int n) { return v < 0 ? v + n : (v < n ? v : v % n); }

template <typename T>
__global__ __launch_bounds__(256) void k_pseudopotential(Geom g, T G, int zc, const T* __restrict__ rho,
                                                         T* __restrict__ F)
{
    __shared__ T psi[4][kPsiPlane];
    const int ntx = (g.nx + kPsiTX - 1) / kPsiTX, nty = (g.ny + kPsiTY - 1) / kPsiTY;
    const int nzc = (g.nz + zc - 1) / zc;
    int r = (int)blockIdx.x;
    const int x0 = (r % ntx) * kPsiTX;
    r /= ntx;
    const int y0 = (r % nty) * kPsiTY;
    r /= nty;
    const int zs = (r % nzc) * zc, b = r / nzc;
    const int ze = zs + zc < g.nz ? zs + zc : g.nz;
    const int tid = (int)threadIdx.x, lx = tid & (kPsiTX - 1), ly = tid / kPsiTX;
    const uint64_t plane = (uint64_t)g.nx * g.ny;
    const T* rb = rho + (uint64_t)b * g.nz * plane;
    // this thread's halo cells k0 = tid and k1 = tid + 256 (if inside the
    // halo plane): their offsets within a plane are the same on every plane;
    // halo positions past a partial tile's end read some in-range cell and
    // are never used
    const int k1 = tid + 256;
    const bool has1 = k1 < kPsiPlane;
    auto halo_off = [&](int k) {
        const int hx = k % kPsiHX, hy = k / kPsiHX;
        return (uint64_t)pmod(y0 + hy - 1, g.ny) * g.nx + (uint64_t)pmod(x0 + hx - 1, g.nx);
    };
    const uint64_t o0 = halo_off(tid), o1 = has1 ? halo_off(k1) : 0;
    auto fetch = [&](int z, T& v0, T& v1) {  // density of halo plane z (-1 <= z <= nz + 1, periodic)
        const T* rp = rb + (uint64_t)pmod(z, g.nz) * plane;
        v0 = rp[o0];
        if (has1) v1 = rp[o1];
    };
    auto put = [&](int slot, T v0, T v1) {
        psi[slot][tid] = T(1) - exp(-v0);
        if (has1) psi[slot][k1] = T(1) - exp(-v1);
    };
    // plane z sits in slot (z - zs + 1) & 3; the first three planes are
    // loaded together
    T a0, a1 = T(0), b0, b1 = T(0), r0, r1 = T(0);
    fetch(zs - 1, a0, a1);
    fetch(zs, b0, b1);
    fetch(zs + 1, r0, r1);
    put(0, a0, a1);
    put(1, b0, b1);
    const int x = x0 + lx, y = y0 + ly;
    const bool live = x < g.nx && y < g.ny;
    for (int z = zs; z < ze; ++z) {
        const int q = z - zs;
        put((q + 2) & 3, r0, r1);  // plane z + 1, loaded during the previous plane
        if (z + 1 < ze) fetch(z + 2, r0, r1);
        __syncthreads();
        if (live) {
            T s[3] = {T(0), T(0), T(0)};
#pragma unroll
            for (int i = 1; i < 27; ++i) {
                const T p = psi[(q + 1 + vel_z(i)) & 3][(ly + 1 + vel_y(i)) * kPsiHX + lx + 1 + vel_x(i)];
                const T w = T(weight(i));
                s[0] += w * T(vel_x(i)) * p;
                s[1] += w * T(vel_y(i)) * p;
                s[2] += w * T(vel_z(i)) * p;
            }
            const T psi0 = psi[(q + 1) & 3][(ly + 1) * kPsiHX + lx + 1];
            const uint64_t lin = ((uint64_t)b * g.nz + z) * plane + (uint64_t)y * g.nx + x;
#pragma unroll
            for (int a = 0; a < 3; ++a) F[a * g.ncell + lin] = -G * psi0 * s[a];
        }
    }
}

// z chunk of the pseudo-potential tiles: the fewest generations of resident
// workgroups, each costing its chunk length plus the two halo planes; ties go
// to the longer chunk (fewer halo planes read)
template <typename T>
int psi_chunk(const Geom& g, int cus)
{
    int per_cu = 0;
    if (cus <= 0 ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_pseudopotential<T>, 256, 0) != hipSuccess ||
        per_cu <= 0)
        return 16;
    const uint64_t cap = (uint64_t)cus * (uint64_t)per_cu;
    const uint64_t cols = (uint64_t)((g.nx + kPsiTX - 1) / kPsiTX) * (uint64_t)((g.ny + kPsiTY - 1) / kPsiTY) * g.nb;
    const int top = g.nz < 64 ? g.nz : 64;
    int best = top;
    uint64_t best_cost = ~0ULL;
    for (int zc = top; zc >= 1; --zc) {
        const uint64_t blocks = cols * (uint64_t)((g.nz + zc - 1) / zc);
        const uint64_t cost = ((blocks + cap - 1) / cap) * (uint64_t)(zc + 2);
        if (cost < best_cost) {
            best_cost = cost;
            best = zc;
        }
    }
    return best;
}

// ---------------------------------------------------------------------------
// diagnostics: gather in FP64

template <int ST, bool MASK>
__device__ __forceinline__ bool gather_f64(const typename storage<ST>::S* __restrict__ src, const Geom& g,
                                           const Cell& c, const uint32_t* __restrict__ mask, double h[27])
{
    using SS = storage<ST>;
    uint32_t m = 0;
    if (MASK) {
        m = mask[c.own];
        if (m & kSolidBit) return false;
    }
    typename SS::T t[27];
    gather<ST, MASK>(src, g, c, m, t);
#pragma unroll
    for (int i = 0; i < 27; ++i) h[i] = (double)t[i];
    return true;
}

__device__ __forceinline__ void cell_force64(const Geom& g, const Cell& c, const double* ftab, const void* field,
                                             int field_f64, double F[3])
{
    if (field) {
        for (int a = 0; a < 3; ++a)
            F[a] = field_f64 ? ((const double*)field)[a * g.ncell + c.lin]
                             : (double)((const float*)field)[a * g.ncell + c.lin];
    } else {
        const double* fr = ftab + 3 * (c.b * g.ny + c.y);
        F[0] = fr[0];
        F[1] = fr[1];
        F[2] = fr[2];
    }
}

__device__ __forceinline__ void macro64(const double h[27], double rho0, const double F[3], double& rho, double u[3],
                                        double j[3], double& drho)
{
    double s = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        s += h[i];
        jx += vel_x(i) * h[i];
        jy += vel_y(i) * h[i];
        jz += vel_z(i) * h[i];
    }
    drho = s;
    rho = rho0 + s;
    j[0] = jx;
    j[1] = jy;
    j[2] = jz;
    u[0] = (jx + 0.5 * F[0]) / rho;
    u[1] = (jy + 0.5 * F[1]) / rho;
    u[2] = (jz + 0.5 * F[2]) / rho;
}

// rho/u (io FP64 or FP32) or FP64 populations of the current state
template <int ST, bool MASK>
__global__ __launch_bounds__(kBlock) void k_gather(const typename storage<ST>::S* __restrict__ src, Geom g,
                                                   double rho0, const double* __restrict__ ftab,
                                                   const void* __restrict__ field, int field_f64,
                                                   const uint32_t* __restrict__ mask, void* rho_out, void* u_out,
                                                   int out_f64, double* pops_out)
{
    const Cell c = locate(g);
    if (!c.valid) return;
    double rho = rho0, u[3] = {0, 0, 0};
    if constexpr (ST == CMLBM_MOM32) {
        // the stored numbers of the post-collision state are its density and velocity
        rho = rho0 + (double)src[c.pown];
        for (int a = 0; a < 3; ++a) u[a] = (double)src[(1 + a) * g.pstride + c.pown];
    } else {
        double h[27];
        const bool fluid = gather_f64<ST, MASK>(src, g, c, mask, h);
        if (pops_out) {
#pragma unroll
            for (int i = 0; i < 27; ++i) pops_out[(uint64_t)i * g.ncell + c.lin] = fluid ? h[i] + weight(i) * rho0 : 0.0;
        }
        if (!rho_out && !u_out) return;
        if (fluid && !u_out) {
            // the density alone: the force enters only the velocity, so
            // neither the force nor the divisions are needed (same sum order
            // as macro64, hence the same density bit for bit)
            double s = 0;
#pragma unroll
            for (int i = 0; i < 27; ++i) s += h[i];
            rho = rho0 + s;
        } else if (fluid) {
            double F[3], j[3], drho;
            cell_force64(g, c, ftab, field, field_f64, F);
            macro64(h, rho0, F, rho, u, j, drho);
        }
    }
    if (out_f64) {
        if (rho_out) ((double*)rho_out)[c.lin] = rho;
        if (u_out)
            for (int a = 0; a < 3; ++a) ((double*)u_out)[a * g.ncell + c.lin] = u[a];
    } else {
        if (rho_out) ((float*)rho_out)[c.lin] = (float)rho;
        if (u_out)
            for (int a = 0; a < 3; ++a) ((float*)u_out)[a * g.ncell + c.lin] = (float)u[a];
    }
}

// FP64 reductions.  Each batch member is split into `gpb` workgroups whose
// waves stride over its 64-cell row segments (wave-uniform row arithmetic, as
// in k_step); every workgroup writes kNPart partial values, summed in a fixed
// tree order, so results are reproducible bit for bit.
template <int ST, bool MASK>
__global__ __launch_bounds__(kBlock) void k_reduce(const typename storage<ST>::S* __restrict__ src, Geom g,
                                                   double rho0, const double* __restrict__ ftab,
                                                   const void* __restrict__ field, int field_f64,
                                                   const uint32_t* __restrict__ mask, int gpb, int residual,
                                                   int snapshot, double* __restrict__ snap, double* __restrict__ part)
{
    __shared__ double sh[kNPart][kBlock];
    const int b = blockIdx.x / gpb;
    const int gblk = blockIdx.x % gpb;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int segs = (g.nx + 63) >> 6;
    const int rows = g.nz * g.ny;  // rows of one batch member
    const int nseg = rows * segs;
    const int nwaves = gpb * (kBlock / 64);
    const int wave0 = __builtin_amdgcn_readfirstlane(gblk * (kBlock / 64) + (tid >> 6));
    double acc[kNPart];
    for (int k = 0; k < kNPart; ++k) acc[k] = 0.0;
    for (int sg = wave0; sg < nseg; sg += nwaves) {
        const int r = sg / segs;
        const int x = (sg - r * segs) * 64 + lane;
        if (x >= g.nx) continue;
        Cell c;
        c.x = x;
        c.y = r % g.ny;
        c.z = r / g.ny;
        c.b = b;
        const int row = b * rows + r;
        c.own = (uint32_t)row * (uint32_t)g.nxp + (uint32_t)x;
        c.pown = (uint64_t)row * g.rstride + (uint64_t)x;
        c.lin = (uint64_t)row * g.nx + x;
        c.valid = true;
        double F[3], rho, u[3], j[3], drho;
        if constexpr (ST == CMLBM_MOM32) {
            cell_force64(g, c, ftab, field, field_f64, F);
            drho = (double)src[c.pown];
            rho = rho0 + drho;
            for (int a = 0; a < 3; ++a) {
                u[a] = (double)src[(1 + a) * g.pstride + c.pown];
                j[a] = rho * u[a] - 0.5 * F[a];  // sum_i f_i c_i
            }
        } else {
            double h[27];
            if (!gather_f64<ST, MASK>(src, g, c, mask, h)) continue;
            cell_force64(g, c, ftab, field, field_f64, F);
            macro64(h, rho0, F, rho, u, j, drho);
        }
        const double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        const bool finite = isfinite(rho) && isfinite(u2);
        acc[7] += 1.0;
        if (!finite) {
            acc[6] += 1.0;
            continue;
        }
        acc[0] += drho;
        acc[1] += j[0];
        acc[2] += j[1];
        acc[3] += j[2];
        acc[4] += 0.5 * rho * u2;
        acc[5] = fmax(acc[5], sqrt(u2));
        acc[9] += u2;
        if (residual) {
            const double d0 = u[0] - snap[c.lin], d1 = u[1] - snap[g.ncell + c.lin], d2 = u[2] - snap[2 * g.ncell + c.lin];
            acc[8] += d0 * d0 + d1 * d1 + d2 * d2;
        }
        if (snapshot) {
            snap[c.lin] = u[0];
            snap[g.ncell + c.lin] = u[1];
            snap[2 * g.ncell + c.lin] = u[2];
        }
    }
    for (int k = 0; k < kNPart; ++k) sh[k][tid] = acc[k];
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (tid < s)
            for (int k = 0; k < kNPart; ++k)
                sh[k][tid] = (k == 5) ? fmax(sh[k][tid], sh[k][tid + s]) : sh[k][tid] + sh[k][tid + s];
        __syncthreads();
    }
    if (tid < kNPart) part[(uint64_t)blockIdx.x * kNPart + tid] = sh[tid][0];
}

// One workgroup per batch member: thread t sums the partials t, t + kBlock,
// ... in order, then the same fixed tree as k_reduce.
__global__ __launch_bounds__(kBlock) void k_reduce_final(const double* __restrict__ part, int gpb, double rho0,
                                                         double* __restrict__ out)
{
    __shared__ double sh[kNPart][kBlock];
    const int b = blockIdx.x;
    const int tid = threadIdx.x;
    double acc[kNPart];
    for (int k = 0; k < kNPart; ++k) acc[k] = 0.0;
    for (int i = tid; i < gpb; i += kBlock)
        for (int k = 0; k < kNPart; ++k) {
            const double v = part[((uint64_t)b * gpb + i) * kNPart + k];
            acc[k] = (k == 5) ? fmax(acc[k], v) : acc[k] + v;
        }
    for (int k = 0; k < kNPart; ++k) sh[k][tid] = acc[k];
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (tid < s)
            for (int k = 0; k < kNPart; ++k)
                sh[k][tid] = (k == 5) ? fmax(sh[k][tid], sh[k][tid + s]) : sh[k][tid] + sh[k][tid + s];
        __syncthreads();
    }
    if (tid >= kNPart) return;
    const int k = tid;
    const double s = sh[k][0];
    double* o = out + (uint64_t)b * CMLBM_NRED;
    switch (k) {
        case 0: o[CMLBM_RED_MASS] = s; break;  // completed on the host with rho0 * fluid
        case 1: o[CMLBM_RED_MOMX] = s; break;
        case 2: o[CMLBM_RED_MOMY] = s; break;
        case 3: o[CMLBM_RED_MOMZ] = s; break;
        case 4: o[CMLBM_RED_KE] = s; break;
        case 5: o[CMLBM_RED_UMAX] = s; break;
        case 6: o[CMLBM_RED_NONFINITE] = s; break;
        case 7: o[CMLBM_RED_FLUID] = s; break;
        case 8: o[CMLBM_RED_DU2] = s; break;
        case 9: o[CMLBM_RED_U2] = s; break;
    }
}

// Second level of the fused reductions: workgroup (b, k) sums, in a fixed
// order and tree, chunk k of the per-wave partials of batch member b (waves
// [b * wpm, (b + 1) * wpm)) into part[b][k], the layout k_reduce writes.
__global__ __launch_bounds__(kBlock) void k_red_waves(const double* __restrict__ wpart, int wpm, int nchunk,
                                                      double* __restrict__ part)
{
    __shared__ double sh[kNPart][kBlock];
    const int b = blockIdx.x / nchunk, k = blockIdx.x % nchunk, tid = threadIdx.x;
    const int per = (wpm + nchunk - 1) / nchunk;
    const int w0 = k * per, w1 = w0 + per < wpm ? w0 + per : wpm;
    double acc[kNPart];
    for (int q = 0; q < kNPart; ++q) acc[q] = 0.0;
    for (int w = w0 + tid; w < w1; w += kBlock)
        for (int q = 0; q < kNPart; ++q) {
            const double v = wpart[((uint64_t)b * wpm + w) * kNPart + q];
            acc[q] = q == 5 ? fmax(acc[q], v) : acc[q] + v;
        }
    for (int q = 0; q < kNPart; ++q) sh[q][tid] = acc[q];
    __syncthreads();
    for (int st = kBlock / 2; st > 0; st >>= 1) {
        if (tid < st)
            for (int q = 0; q < kNPart; ++q)
                sh[q][tid] = q == 5 ? fmax(sh[q][tid], sh[q][tid + st]) : sh[q][tid] + sh[q][tid + st];
        __syncthreads();
    }
    if (tid < kNPart) part[((uint64_t)b * nchunk + k) * kNPart + tid] = sh[tid][0];
}

// Per-cell link mask: bit i set if the node x - c_i lies beyond a wall or is
// solid (the population pulled along c_i then comes from the opposite
// direction at x itself), bit 27 set if x is solid.
__global__ __launch_bounds__(kBlock) void k_linkmask(Geom g, int wx, int wy, int wz,
                                                     const uint8_t* __restrict__ solid, uint32_t* __restrict__ mask)
{
    const Cell c = locate(g);
    if (!c.valid) return;
    const int dims[3] = {g.nx, g.ny, g.nz};
    const int walls[3] = {wx, wy, wz};
    uint32_t m = 0;
    if (solid && solid[c.lin]) m |= kSolidBit;
    for (int i = 0; i < 27; ++i) {
        int s[3] = {c.x - vel_x(i), c.y - vel_y(i), c.z - vel_z(i)};
        bool bounce = false;
        for (int a = 0; a < 3; ++a) {
            if (s[a] < 0 || s[a] >= dims[a]) {
                if (walls[a]) bounce = true;
                s[a] = wrap(s[a], dims[a]);
            }
        }
        if (!bounce && solid) {
            const uint64_t n = ((uint64_t)(c.b * g.nz + s[2]) * g.ny + s[1]) * g.nx + s[0];
            bounce = solid[n] != 0;
        }
        if (bounce) m |= 1u << i;
    }
    mask[c.own] = m;
}

// Plain copy with 16-byte non-temporal accesses, four loads in flight per
// thread before its stores (the device's practical read + write bandwidth; a
// measurement aid).  Of the variants measured (one or eight loads in flight,
// plain or non-temporal loads) this was the fastest.
typedef int v4i __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(kBlock) void k_copy16(const v4i* __restrict__ src, v4i* __restrict__ dst, uint64_t n)
{
    constexpr int U = 4;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock * U + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kBlock * U) {
        v4i v[U];
#pragma unroll
        for (int k = 0; k < U; ++k)
            if (i + k * kBlock < n) v[k] = __builtin_nontemporal_load(src + i + k * kBlock);
#pragma unroll
        for (int k = 0; k < U; ++k)
            if (i + k * kBlock < n) __builtin_nontemporal_store(v[k], dst + i + k * kBlock);
    }
}

// The FP32 step's memory traffic without its arithmetic (a measurement aid):
// one cell per lane in 1024-thread workgroups, each lane loads its cell of
// every plane, then stores them with non-temporal stores.
template <int NP>
__global__ __launch_bounds__(1024) void k_copy_planes(const float* __restrict__ src, float* __restrict__ dst,
                                                      uint64_t cells, uint64_t pstride)
{
    const uint64_t c = (uint64_t)blockIdx.x * 1024 + threadIdx.x;
    if (c >= cells) return;
    float v[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) v[p] = src[p * pstride + c];
#pragma unroll
    for (int p = 0; p < NP; ++p) __builtin_nontemporal_store(v[p], dst + p * pstride + c);
}

// The same for the row-block layout of the population step: population p of
// cell x in lattice row r at (r * 27 + p) * row_len + x.
__global__ __launch_bounds__(1024) void k_copy_row_blocks(const float* __restrict__ src, float* __restrict__ dst,
                                                          uint64_t cells, uint32_t row_len)
{
    const uint64_t c = (uint64_t)blockIdx.x * 1024 + threadIdx.x;
    if (c >= cells) return;
    const uint64_t base = c / row_len * 27 * row_len + c % row_len;
    float v[27];
#pragma unroll
    for (int p = 0; p < 27; ++p) v[p] = src[base + (uint64_t)p * row_len];
#pragma unroll
    for (int p = 0; p < 27; ++p) __builtin_nontemporal_store(v[p], dst + base + (uint64_t)p * row_len);
}

__global__ void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

}  // namespace

// ---------------------------------------------------------------------------
// host side

struct cmlbm_lattice {
    cmlbm_params p;
    Geom g;
    void* pop[2];
    int cur;  // buffer holding the state
    uint8_t* scratch;
    size_t off_ftab64, off_ftab32, off_mask, off_part, off_final, off_snap, off_wpart;
    int gpb;
    bool needs_mask, mask_ready, initialized, snap_valid;
    int force_mode;
    const void* field;
    int field_dtype;
    int64_t t;
    int cu_per_xcd;  // compute units per XCD of the lattice's device (the moment kernel's generation size)
    int cus;         // compute units of the lattice's device (0 if unknown)
    int psi_zc;      // z chunk of the pseudo-potential tiles (0 until the first launch)
    std::string err;
};

namespace {

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct Layout {
    Geom g;
    size_t pop_bytes, scratch_bytes;
    size_t off_ftab64, off_ftab32, off_mask, off_part, off_final, off_snap, off_wpart;
    int gpb;
    bool needs_mask;
};

// Cells per lane of k_step: two for 16-bit storage on rows of even length
// without a bounce-back mask, otherwise one.
int lanes_rule(int storage, int nx, bool needs_mask)
{
    if (needs_mask) return 1;
    if ((storage == CMLBM_FP16 || storage == CMLBM_BF16) && nx % 2 == 0) return 2;
    return 1;
}

int validate(const cmlbm_params* p)
{
    if (!p) return CMLBM_EINVAL;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1 || p->nbatch < 1) return CMLBM_EINVAL;
    if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return CMLBM_EINVAL;
    if (!(p->rho0 > 0.0) || !std::isfinite(p->rho0)) return CMLBM_EINVAL;
    if (p->storage < CMLBM_FP64 || p->storage > CMLBM_MOM32) return CMLBM_EINVAL;
    if (p->storage == CMLBM_MOM32 && (p->wall[0] || p->wall[1] || p->wall[2] ||
                                      (p->flags & ~(uint32_t)CMLBM_FLAG_RESIDUAL)))
        return CMLBM_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (p->wall[a] != CMLBM_PERIODIC && p->wall[a] != CMLBM_BOUNCEBACK) return CMLBM_EINVAL;
    if (p->flags & ~(CMLBM_FLAG_SOLID | CMLBM_FLAG_RESIDUAL | CMLBM_FLAG_STOCHASTIC | CMLBM_FLAG_FORCE_GUO |
                     CMLBM_FLAG_EQ_SECOND | CMLBM_FLAG_BGK | CMLBM_FLAG_FUSED_REDUCE))
        return CMLBM_EINVAL;
    const uint32_t model = p->flags & (CMLBM_FLAG_FORCE_GUO | CMLBM_FLAG_EQ_SECOND | CMLBM_FLAG_BGK);
    // fused reductions run in the kernel of the method's own collision on population storage
    if ((p->flags & CMLBM_FLAG_FUSED_REDUCE) && (model || p->storage == CMLBM_MOM32)) return CMLBM_EINVAL;
    if (model && p->storage != CMLBM_FP64 && p->storage != CMLBM_FP32) return CMLBM_EINVAL;
    if ((model & CMLBM_FLAG_BGK) && model != CMLBM_FLAG_BGK &&
        model != (CMLBM_FLAG_BGK | CMLBM_FLAG_FORCE_GUO | CMLBM_FLAG_EQ_SECOND))
        return CMLBM_EINVAL;
    // an axis of extent 1 with walls would bounce everything; periodic is required there
    const int dims[3] = {p->nx, p->ny, p->nz};
    for (int a = 0; a < 3; ++a)
        if (p->wall[a] == CMLBM_BOUNCEBACK && dims[a] < 2) return CMLBM_EINVAL;
    return CMLBM_OK;
}

// Population layout.  Planes: population i of every row together, planes
// kPlanePad bytes apart.  Row blocks: the 27 population rows of one lattice
// row stored together, rows one after another, so that a wave's 27 stores go
// to one contiguous block and its loads to nine.  Moment storage uses planes.
bool row_blocks(int storage) { return storage != CMLBM_MOM32; }

int make_layout(const cmlbm_params* p, Layout* L)
{
    int rc = validate(p);
    if (rc) return rc;
    const size_t sb = storage_bytes(p->storage);
    const size_t row_bytes = align256((size_t)p->nx * sb);
    Geom& g = L->g;
    g.nx = p->nx;
    g.ny = p->ny;
    g.nz = p->nz;
    g.nb = p->nbatch;
    g.nxp = (int)(row_bytes / sb);
    const uint64_t rows = (uint64_t)p->ny * p->nz * p->nbatch;
    if (rows > 0x7fffffffULL) return CMLBM_EINVAL;
    g.rows = (int)rows;
    // planes are kPlanePad bytes apart beyond their rows: at power-of-two plane sizes the 27
    // concurrent plane streams would otherwise map onto the same HBM channels
    const uint64_t plane = rows * (uint64_t)g.nxp + kPlanePad / sb;
    if (plane * sb >= (1ULL << 32)) return CMLBM_EINVAL;  // per-plane (and link-mask) offsets are 32-bit
    const bool blocks = row_blocks(p->storage);
    g.pstride = blocks ? (uint64_t)g.nxp : plane;
    g.rstride = blocks ? 27ull * g.nxp : (uint64_t)g.nxp;
    g.ncell = rows * (uint64_t)p->nx;
    const int nx64 = (p->nx + 63) / 64 * 64;
    g.bx = nx64 < kBlock ? nx64 : kBlock;
    g.by = kBlock / g.bx;
    g.xblocks = (p->nx + g.bx - 1) / g.bx;
    const uint64_t nblocks = (uint64_t)g.xblocks * ((rows + g.by - 1) / g.by);
    if (nblocks > 0x7fffffffULL) return CMLBM_EINVAL;
    if (p->storage == CMLBM_MOM32) {  // one-dimensional grid of moment tiles (6-row tiles: the most work-items)
        const uint64_t tiles = (uint64_t)((p->nx + 63) / 64) * ((p->ny + 5) / 6) * p->nbatch * ((p->nz + 31) / 32);
        if (tiles * 9 * 64 > 0xffffffffULL) return CMLBM_EINVAL;
    }

    L->pop_bytes = align256(blocks ? rows * g.rstride * sb : (uint64_t)planes_of(p->storage) * plane * sb);
    L->needs_mask = (p->flags & CMLBM_FLAG_SOLID) || p->wall[0] || p->wall[1] || p->wall[2];
    const uint64_t per = (uint64_t)p->nz * p->ny * p->nx;
    uint64_t gpb = (per + kBlock - 1) / kBlock;
    const uint64_t max_gpb = p->storage == CMLBM_FP64 ? kMaxRedBlocks / 2 : kMaxRedBlocks;
    if (gpb > max_gpb) gpb = max_gpb;
    L->gpb = (int)gpb;
    size_t off = 0;
    L->off_ftab64 = off;
    off = align256(off + (size_t)p->nbatch * p->ny * 3 * sizeof(double));
    L->off_ftab32 = off;
    off = align256(off + (size_t)p->nbatch * p->ny * 3 * sizeof(float));
    L->off_mask = off;
    if (L->needs_mask) off = align256(off + plane * sizeof(uint32_t));
    L->off_part = off;
    off = align256(off + (size_t)p->nbatch * gpb * kNPart * sizeof(double));
    L->off_final = off;
    off = align256(off + (size_t)p->nbatch * CMLBM_NRED * sizeof(double));
    L->off_snap = off;
    if (p->flags & CMLBM_FLAG_RESIDUAL) off = align256(off + 3 * g.ncell * sizeof(double));
    L->off_wpart = off;
    if (p->flags & CMLBM_FLAG_FUSED_REDUCE) {  // one partial row per k_step wave
        const int V = lanes_rule(p->storage, p->nx, L->needs_mask);
        const uint64_t segs = (uint64_t)(p->nx + 64 * V - 1) / (64 * V);
        if (segs * p->ny * p->nz > 0x7fffffffULL) return CMLBM_EINVAL;
        off = align256(off + rows * segs * kNPart * sizeof(double));
    }
    L->scratch_bytes = off;
    return CMLBM_OK;
}

int fail(cmlbm_lattice* lat, int code, const std::string& msg)
{
    if (lat) lat->err = msg;
    return code;
}

int hip_check(cmlbm_lattice* lat, hipError_t e, const char* what)
{
    if (e == hipSuccess) return CMLBM_OK;
    return fail(lat, CMLBM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

int launch_check(cmlbm_lattice* lat, const char* what) { return hip_check(lat, hipGetLastError(), what); }

dim3 grid_of(const Geom& g) { return dim3(g.xblocks * ((g.rows + g.by - 1) / g.by)); }
dim3 block_of(const Geom& g) { return dim3(g.bx, g.by); }

uint32_t* mask_ptr(cmlbm_lattice* lat) { return lat->needs_mask ? (uint32_t*)(lat->scratch + lat->off_mask) : nullptr; }

int build_mask(cmlbm_lattice* lat, const uint8_t* solid, hipStream_t s)
{
    const Geom& g = lat->g;
    uint32_t* m = mask_ptr(lat);
    k_fill_u32<<<1024, 256, 0, s>>>(m, (uint64_t)g.rows * g.nxp, kSolidBit);  // padding columns count as solid
    int rc = launch_check(lat, "link mask clear");
    if (rc) return rc;
    k_linkmask<<<grid_of(g), block_of(g), 0, s>>>(g, lat->p.wall[0], lat->p.wall[1], lat->p.wall[2], solid, m);
    rc = launch_check(lat, "link mask");
    if (rc) return rc;
    lat->mask_ready = true;
    return CMLBM_OK;
}

int ensure_mask(cmlbm_lattice* lat, hipStream_t s)
{
    if (!lat->needs_mask || lat->mask_ready) return CMLBM_OK;
    return build_mask(lat, nullptr, s);
}

// ---- kernel dispatch over (storage, mask, field)

// Cells per lane of k_step: 16-bit storage reads 2 cells (4 bytes) per lane
// where the row length allows, everything else one cell per lane.  (With the
// population planes spaced, 2 cells beat 4 by 2-5% at 512^3.)
int step_lanes(const cmlbm_lattice* lat) { return lanes_rule(lat->p.storage, lat->g.nx, lat->needs_mask); }

int lat_model(const cmlbm_lattice* lat)
{
    return ((lat->p.flags & CMLBM_FLAG_FORCE_GUO) ? kModelGuo : 0) | ((lat->p.flags & CMLBM_FLAG_EQ_SECOND) ? kModelEq2 : 0) |
           ((lat->p.flags & CMLBM_FLAG_BGK) ? kModelBgk : 0);
}

template <int ST, int V, bool MASK, bool FIELD, int MODEL = 0>
void launch_step_v(cmlbm_lattice* lat, hipStream_t s)
{
    using SS = storage<ST>;
    using T = typename SS::T;
    const Geom& g = lat->g;
    const int segs = (g.nx + 64 * V - 1) / (64 * V);
    const uint64_t waves = (uint64_t)g.rows * (uint64_t)segs;
    constexpr int wpb = step_block(ST, MASK) / 64;
    const dim3 grid((unsigned)((waves + wpb - 1) / wpb));
    const T* ftab = (const T*)(lat->scratch + (ST == CMLBM_FP64 ? lat->off_ftab64 : lat->off_ftab32));
    auto go = [&](auto sr) {
        k_step<ST, V, MASK, FIELD, true, MODEL, false, decltype(sr)::value><<<grid, dim3(step_block(ST, MASK)), 0, s>>>(
            (const typename SS::S*)lat->pop[lat->cur], (typename SS::S*)lat->pop[1 - lat->cur], g, segs,
            (T)(1.0 / lat->p.tau), (T)lat->p.rho0, ftab, (const T*)lat->field, mask_ptr(lat), (uint32_t)lat->t,
            nullptr);
    };
    if constexpr (sizeof(typename SS::S) == 2 && MODEL == 0) {
        if (lat->p.flags & CMLBM_FLAG_STOCHASTIC)
            go(std::true_type{});
        else
            go(std::false_type{});
    } else {
        go(std::false_type{});
    }
}

template <int ST, int MODEL>
void launch_step_model(cmlbm_lattice* lat, hipStream_t s)
{
    const bool F = lat->force_mode == CMLBM_FORCE_FIELD;
    if (lat->needs_mask) {
        if (F)
            launch_step_v<ST, 1, true, true, MODEL>(lat, s);
        else
            launch_step_v<ST, 1, true, false, MODEL>(lat, s);
    } else {
        if (F)
            launch_step_v<ST, 1, false, true, MODEL>(lat, s);
        else
            launch_step_v<ST, 1, false, false, MODEL>(lat, s);
    }
}

template <int ST>
int launch_step_st(cmlbm_lattice* lat, hipStream_t s)
{
    const bool F = lat->force_mode == CMLBM_FORCE_FIELD;
    const int V = step_lanes(lat);
    if constexpr (ST == CMLBM_FP64 || ST == CMLBM_FP32) {
        const int model = lat_model(lat);
        if (model) {
            if (model == kModelGuo)
                launch_step_model<ST, kModelGuo>(lat, s);
            else if (model == kModelEq2)
                launch_step_model<ST, kModelEq2>(lat, s);
            else if (model == (kModelGuo | kModelEq2))
                launch_step_model<ST, kModelGuo | kModelEq2>(lat, s);
            else if (model == kModelBgk)
                launch_step_model<ST, kModelBgk>(lat, s);
            else
                launch_step_model<ST, kModelBgk | kModelGuo | kModelEq2>(lat, s);
            return launch_check(lat, "step");
        }
    }
    if (lat->needs_mask) {
        if (F)
            launch_step_v<ST, 1, true, true>(lat, s);
        else
            launch_step_v<ST, 1, true, false>(lat, s);
    } else if constexpr (ST == CMLBM_FP16 || ST == CMLBM_BF16) {
        if (V == 2) {
            if (F)
                launch_step_v<ST, 2, false, true>(lat, s);
            else
                launch_step_v<ST, 2, false, false>(lat, s);
        } else {
            if (F)
                launch_step_v<ST, 1, false, true>(lat, s);
            else
                launch_step_v<ST, 1, false, false>(lat, s);
        }
    } else {
        if (F)
            launch_step_v<ST, 1, false, true>(lat, s);
        else
            launch_step_v<ST, 1, false, false>(lat, s);
    }
    return launch_check(lat, "step");
}

// One step with fused reductions: k_step with RED, then the two reduction levels
// into the final row of each batch member.
template <int ST, int V, bool MASK, bool FIELD>
void launch_step_red_v(cmlbm_lattice* lat, hipStream_t s)
{
    using SS = storage<ST>;
    using T = typename SS::T;
    const Geom& g = lat->g;
    const int segs = (g.nx + 64 * V - 1) / (64 * V);
    const uint64_t waves = (uint64_t)g.rows * (uint64_t)segs;
    constexpr int wpb = step_block(ST, MASK) / 64;
    const dim3 grid((unsigned)((waves + wpb - 1) / wpb));
    const T* ftab = (const T*)(lat->scratch + (ST == CMLBM_FP64 ? lat->off_ftab64 : lat->off_ftab32));
    auto go = [&](auto sr) {
        k_step<ST, V, MASK, FIELD, true, 0, true, decltype(sr)::value><<<grid, dim3(step_block(ST, MASK)), 0, s>>>(
            (const typename SS::S*)lat->pop[lat->cur], (typename SS::S*)lat->pop[1 - lat->cur], g, segs,
            (T)(1.0 / lat->p.tau), (T)lat->p.rho0, ftab, (const T*)lat->field, mask_ptr(lat), (uint32_t)lat->t,
            (double*)(lat->scratch + lat->off_wpart));
    };
    if constexpr (sizeof(typename SS::S) == 2) {
        if (lat->p.flags & CMLBM_FLAG_STOCHASTIC)
            go(std::true_type{});
        else
            go(std::false_type{});
    } else {
        go(std::false_type{});
    }
}

template <int ST>
int launch_step_red_st(cmlbm_lattice* lat, hipStream_t s)
{
    const bool F = lat->force_mode == CMLBM_FORCE_FIELD;
    const int V = step_lanes(lat);
    if (lat->needs_mask) {
        if (F)
            launch_step_red_v<ST, 1, true, true>(lat, s);
        else
            launch_step_red_v<ST, 1, true, false>(lat, s);
    } else if (V == 2) {
        if constexpr (ST == CMLBM_FP16 || ST == CMLBM_BF16) {
            if (F)
                launch_step_red_v<ST, 2, false, true>(lat, s);
            else
                launch_step_red_v<ST, 2, false, false>(lat, s);
        }
    } else {
        if (F)
            launch_step_red_v<ST, 1, false, true>(lat, s);
        else
            launch_step_red_v<ST, 1, false, false>(lat, s);
    }
    int rc = launch_check(lat, "step (fused reductions)");
    if (rc) return rc;
    const Geom& g = lat->g;
    const int segs = (g.nx + 64 * V - 1) / (64 * V);
    const int wpm = (g.rows / g.nb) * segs;  // waves per batch member
    int nchunk = (wpm + 1023) / 1024;
    if (nchunk > lat->gpb) nchunk = lat->gpb;
    k_red_waves<<<dim3(g.nb * nchunk), dim3(kBlock), 0, s>>>((const double*)(lat->scratch + lat->off_wpart), wpm,
                                                            nchunk, (double*)(lat->scratch + lat->off_part));
    rc = launch_check(lat, "reduce waves");
    if (rc) return rc;
    k_reduce_final<<<dim3(g.nb), dim3(kBlock), 0, s>>>((const double*)(lat->scratch + lat->off_part), nchunk,
                                                      lat->p.rho0, (double*)(lat->scratch + lat->off_final));
    return launch_check(lat, "reduce final");
}

int launch_step_red(cmlbm_lattice* lat, hipStream_t s)
{
    switch (lat->p.storage) {
        case CMLBM_FP64: return launch_step_red_st<CMLBM_FP64>(lat, s);
        case CMLBM_FP32: return launch_step_red_st<CMLBM_FP32>(lat, s);
        case CMLBM_FP16: return launch_step_red_st<CMLBM_FP16>(lat, s);
        default: return launch_step_red_st<CMLBM_BF16>(lat, s);
    }
}

template <int TY>
void launch_step_mom_t(cmlbm_lattice* lat, hipStream_t s)
{
    const Geom& g = lat->g;
    const int nzc = (g.nz + kMomZC - 1) / kMomZC;
    const int ntx = (g.nx + kMomTX - 1) / kMomTX, nty = (g.ny + TY - 1) / TY;
    dim3 grid((unsigned)(ntx * nty * g.nb * nzc));
    // the blocked schedule when an XCD's generation covers whole tile rows,
    // it takes no more rounds of one workgroup per CU than the plain order,
    // and each XCD runs at least 8 generations: it starts an XCD's workgroups
    // together instead of staggered, which measured 2% slower with 3
    // generations (256^3) and 1.2% faster with 22 (512^3, reads 1.17 -> 1.06x
    // the algorithmic bytes)
    const int cpx = lat->cu_per_xcd;
    int gens = 0;
    if (cpx > 0 && cpx % ntx == 0) {
        const int by = cpx / ntx;
        const long long pairs = (long long)g.nb * ((nty + by - 1) / by) * nzc;
        const long long round = 8LL * cpx, tiles = (long long)grid.x;
        if (pairs >= 64 && (pairs + 7) / 8 <= (tiles + round - 1) / round) {
            gens = (int)((pairs + 7) / 8);
            grid = dim3((unsigned)(round * gens));
        }
    }
    const float* ftab = (const float*)(lat->scratch + lat->off_ftab32);
    const float* src = (const float*)lat->pop[lat->cur];
    float* dst = (float*)lat->pop[1 - lat->cur];
    const float om = (float)(1.0 / lat->p.tau), r0 = (float)lat->p.rho0;
    const dim3 block((TY + 3) * 64);
    if (lat->force_mode == CMLBM_FORCE_FIELD)
        k_step_mom<true, TY><<<grid, block, 0, s>>>(src, dst, g, om, r0, ftab, (const float*)lat->field, gens, cpx);
    else
        k_step_mom<false, TY><<<grid, block, 0, s>>>(src, dst, g, om, r0, ftab, nullptr, gens, cpx);
}

int launch_step_mom(cmlbm_lattice* lat, hipStream_t s)
{
    if (mom_rows(lat->g) == 12)
        launch_step_mom_t<12>(lat, s);
    else
        launch_step_mom_t<6>(lat, s);
    return launch_check(lat, "step");
}

int launch_step(cmlbm_lattice* lat, hipStream_t s)
{
    switch (lat->p.storage) {
        case CMLBM_MOM32: return launch_step_mom(lat, s);
        case CMLBM_FP64: return launch_step_st<CMLBM_FP64>(lat, s);
        case CMLBM_FP32: return launch_step_st<CMLBM_FP32>(lat, s);
        case CMLBM_FP16: return launch_step_st<CMLBM_FP16>(lat, s);
        default: return launch_step_st<CMLBM_BF16>(lat, s);
    }
}

template <int ST, bool MASK>
void launch_init_m(cmlbm_lattice* lat, int src_kind, const void* rho, const void* u, const double* pops, hipStream_t s)
{
    using SS = storage<ST>;
    const Geom& g = lat->g;
    auto* dst = (typename SS::S*)lat->pop[lat->cur];
    const uint32_t* m = mask_ptr(lat);
    const double rho0 = lat->p.rho0;
    if (src_kind == INIT_EQ_F64)
        k_init<ST, MASK, INIT_EQ_F64><<<grid_of(g), block_of(g), 0, s>>>(dst, g, rho0, rho, u, pops, m);
    else if (src_kind == INIT_EQ_F32)
        k_init<ST, MASK, INIT_EQ_F32><<<grid_of(g), block_of(g), 0, s>>>(dst, g, rho0, rho, u, pops, m);
    else
        k_init<ST, MASK, INIT_POPS_F64><<<grid_of(g), block_of(g), 0, s>>>(dst, g, rho0, rho, u, pops, m);
}

template <int ST>
int launch_init_st(cmlbm_lattice* lat, int src_kind, const void* rho, const void* u, const double* pops,
                   hipStream_t s)
{
    if (lat->needs_mask)
        launch_init_m<ST, true>(lat, src_kind, rho, u, pops, s);
    else
        launch_init_m<ST, false>(lat, src_kind, rho, u, pops, s);
    return launch_check(lat, "init");
}

int launch_init_mom(cmlbm_lattice* lat, int src_kind, const void* rho, const void* u, hipStream_t s)
{
    const Geom& g = lat->g;
    const float* ftab = (const float*)(lat->scratch + lat->off_ftab32);
    const float* field = lat->force_mode == CMLBM_FORCE_FIELD ? (const float*)lat->field : nullptr;
    float* dst = (float*)lat->pop[lat->cur];
    const float om = (float)(1.0 / lat->p.tau), r0 = (float)lat->p.rho0;
    if (src_kind == INIT_EQ_F64)
        k_init_mom<INIT_EQ_F64><<<grid_of(g), block_of(g), 0, s>>>(dst, g, om, r0, rho, u, ftab, field);
    else
        k_init_mom<INIT_EQ_F32><<<grid_of(g), block_of(g), 0, s>>>(dst, g, om, r0, rho, u, ftab, field);
    return launch_check(lat, "init");
}

int launch_init(cmlbm_lattice* lat, int src_kind, const void* rho, const void* u, const double* pops, hipStream_t s)
{
    switch (lat->p.storage) {
        case CMLBM_MOM32: return launch_init_mom(lat, src_kind, rho, u, s);
        case CMLBM_FP64: return launch_init_st<CMLBM_FP64>(lat, src_kind, rho, u, pops, s);
        case CMLBM_FP32: return launch_init_st<CMLBM_FP32>(lat, src_kind, rho, u, pops, s);
        case CMLBM_FP16: return launch_init_st<CMLBM_FP16>(lat, src_kind, rho, u, pops, s);
        default: return launch_init_st<CMLBM_BF16>(lat, src_kind, rho, u, pops, s);
    }
}

const double* ftab64(cmlbm_lattice* lat) { return (const double*)(lat->scratch + lat->off_ftab64); }
const void* field64_or_null(cmlbm_lattice* lat)
{
    return lat->force_mode == CMLBM_FORCE_FIELD ? lat->field : nullptr;
}

template <int ST, bool MASK>
void launch_gather_m(cmlbm_lattice* lat, void* rho, void* u, int out_f64, double* pops, hipStream_t s)
{
    using SS = storage<ST>;
    const Geom& g = lat->g;
    k_gather<ST, MASK><<<grid_of(g), block_of(g), 0, s>>>(
        (const typename SS::S*)lat->pop[lat->cur], g, lat->p.rho0, ftab64(lat), field64_or_null(lat),
        lat->p.storage == CMLBM_FP64, mask_ptr(lat), rho, u, out_f64, pops);
}

template <int ST>
int launch_gather_st(cmlbm_lattice* lat, void* rho, void* u, int out_f64, double* pops, hipStream_t s)
{
    if (lat->needs_mask)
        launch_gather_m<ST, true>(lat, rho, u, out_f64, pops, s);
    else
        launch_gather_m<ST, false>(lat, rho, u, out_f64, pops, s);
    return launch_check(lat, "gather");
}

int launch_gather(cmlbm_lattice* lat, void* rho, void* u, int out_f64, double* pops, hipStream_t s)
{
    switch (lat->p.storage) {
        case CMLBM_MOM32: launch_gather_m<CMLBM_MOM32, false>(lat, rho, u, out_f64, pops, s); return launch_check(lat, "gather");
        case CMLBM_FP64: return launch_gather_st<CMLBM_FP64>(lat, rho, u, out_f64, pops, s);
        case CMLBM_FP32: return launch_gather_st<CMLBM_FP32>(lat, rho, u, out_f64, pops, s);
        case CMLBM_FP16: return launch_gather_st<CMLBM_FP16>(lat, rho, u, out_f64, pops, s);
        default: return launch_gather_st<CMLBM_BF16>(lat, rho, u, out_f64, pops, s);
    }
}

template <int ST, bool MASK>
void launch_reduce_m(cmlbm_lattice* lat, int residual, int snapshot, hipStream_t s)
{
    using SS = storage<ST>;
    const Geom& g = lat->g;
    double* snap = (lat->p.flags & CMLBM_FLAG_RESIDUAL) ? (double*)(lat->scratch + lat->off_snap) : nullptr;
    k_reduce<ST, MASK><<<dim3(g.nb * lat->gpb), dim3(kBlock), 0, s>>>(
        (const typename SS::S*)lat->pop[lat->cur], g, lat->p.rho0, ftab64(lat), field64_or_null(lat),
        lat->p.storage == CMLBM_FP64, mask_ptr(lat), lat->gpb, residual, snapshot, snap,
        (double*)(lat->scratch + lat->off_part));
}

template <int ST>
void launch_reduce_st(cmlbm_lattice* lat, int residual, int snapshot, hipStream_t s)
{
    if (lat->needs_mask)
        launch_reduce_m<ST, true>(lat, residual, snapshot, s);
    else
        launch_reduce_m<ST, false>(lat, residual, snapshot, s);
}

int launch_reduce(cmlbm_lattice* lat, int residual, int snapshot, hipStream_t s)
{
    switch (lat->p.storage) {
        case CMLBM_MOM32: launch_reduce_m<CMLBM_MOM32, false>(lat, residual, snapshot, s); break;
        case CMLBM_FP64: launch_reduce_st<CMLBM_FP64>(lat, residual, snapshot, s); break;
        case CMLBM_FP32: launch_reduce_st<CMLBM_FP32>(lat, residual, snapshot, s); break;
        case CMLBM_FP16: launch_reduce_st<CMLBM_FP16>(lat, residual, snapshot, s); break;
        default: launch_reduce_st<CMLBM_BF16>(lat, residual, snapshot, s); break;
    }
    int rc = launch_check(lat, "reduce");
    if (rc) return rc;
    k_reduce_final<<<dim3(lat->g.nb), dim3(kBlock), 0, s>>>((const double*)(lat->scratch + lat->off_part), lat->gpb,
                                                       lat->p.rho0, (double*)(lat->scratch + lat->off_final));
    return launch_check(lat, "reduce final");
}

bool aligned256(const void* p) { return ((uintptr_t)p & 255u) == 0; }

// Host completion of the FP64 reductions: the mass gets rho0 per finite fluid
// cell (the sums hold deviations), the residual its square root.
int finish_reduce(cmlbm_lattice* lat, bool residual, double* host_out)
{
    bool unstable = false;
    for (size_t b = 0; b < (size_t)lat->g.nb; ++b) {
        double* o = host_out + b * CMLBM_NRED;
        o[CMLBM_RED_MASS] += lat->p.rho0 * (o[CMLBM_RED_FLUID] - o[CMLBM_RED_NONFINITE]);
        o[CMLBM_RED_RESIDUAL] = residual && o[CMLBM_RED_U2] > 0 ? std::sqrt(o[CMLBM_RED_DU2] / o[CMLBM_RED_U2]) : 0.0;
        if (!residual) o[CMLBM_RED_DU2] = 0.0;
        if (o[CMLBM_RED_NONFINITE] > 0) unstable = true;
    }
    if (unstable) return fail(lat, CMLBM_EUNSTABLE, "non-finite density or velocity");
    return CMLBM_OK;
}

}  // namespace

extern "C" {

int cmlbm_required_bytes(const cmlbm_params* params, size_t* pop_buffer_bytes, size_t* scratch_bytes)
{
    Layout L;
    const int rc = make_layout(params, &L);
    if (rc) return rc;
    if (pop_buffer_bytes) *pop_buffer_bytes = L.pop_bytes;
    if (scratch_bytes) *scratch_bytes = L.scratch_bytes;
    return CMLBM_OK;
}

int cmlbm_create(const cmlbm_params* params, void* pop_a, size_t pop_a_bytes, void* pop_b, size_t pop_b_bytes,
                 void* scratch, size_t scratch_bytes, cmlbm_lattice** out)
{
    if (!out) return CMLBM_EINVAL;
    *out = nullptr;
    Layout L;
    int rc = make_layout(params, &L);
    if (rc) return rc;
    if (!pop_a || !pop_b || !scratch || pop_a == pop_b) return CMLBM_EINVAL;
    if (!aligned256(pop_a) || !aligned256(pop_b) || !aligned256(scratch)) return CMLBM_EINVAL;
    if (pop_a_bytes < L.pop_bytes || pop_b_bytes < L.pop_bytes || scratch_bytes < L.scratch_bytes)
        return CMLBM_ENOMEM;
    cmlbm_lattice* lat = new (std::nothrow) cmlbm_lattice();
    if (!lat) return CMLBM_ENOMEM;
    lat->p = *params;
    lat->g = L.g;
    lat->pop[0] = pop_a;
    lat->pop[1] = pop_b;
    lat->cur = 0;
    lat->scratch = (uint8_t*)scratch;
    lat->off_ftab64 = L.off_ftab64;
    lat->off_ftab32 = L.off_ftab32;
    lat->off_mask = L.off_mask;
    lat->off_part = L.off_part;
    lat->off_final = L.off_final;
    lat->off_snap = L.off_snap;
    lat->off_wpart = L.off_wpart;
    lat->gpb = L.gpb;
    lat->needs_mask = L.needs_mask;
    lat->mask_ready = false;
    lat->initialized = false;
    lat->snap_valid = false;
    lat->force_mode = -1;  // table not yet written
    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 0;
        lat->cu_per_xcd = cus % 8 == 0 ? cus / 8 : 0;
        lat->cus = cus;
    }
    lat->psi_zc = 0;  // chosen at the first pseudo-potential launch
    lat->field = nullptr;
    lat->field_dtype = CMLBM_FP64;
    lat->t = 0;
    *out = lat;
    return CMLBM_OK;
}

int cmlbm_set_solid(cmlbm_lattice* lat, const uint8_t* dev_solid, void* hip_stream)
{
    if (!lat) return CMLBM_EINVAL;
    if (!(lat->p.flags & CMLBM_FLAG_SOLID)) return fail(lat, CMLBM_ESTATE, "set_solid needs CMLBM_FLAG_SOLID");
    lat->initialized = false;
    lat->snap_valid = false;
    return build_mask(lat, dev_solid, (hipStream_t)hip_stream);
}

int cmlbm_set_force(cmlbm_lattice* lat, int mode, const double* host_values, const void* dev_field, int io_dtype,
                    void* hip_stream)
{
    if (!lat) return CMLBM_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    const Geom& g = lat->g;
    const size_t n = (size_t)g.nb * g.ny;
    std::vector<double> tab(3 * n, 0.0);
    switch (mode) {
        case CMLBM_FORCE_NONE: break;
        case CMLBM_FORCE_UNIFORM:
            if (!host_values) return fail(lat, CMLBM_EINVAL, "UNIFORM force needs host_values[3]");
            for (size_t r = 0; r < n; ++r)
                for (int a = 0; a < 3; ++a) tab[3 * r + a] = host_values[a];
            break;
        case CMLBM_FORCE_BATCH:
            if (!host_values) return fail(lat, CMLBM_EINVAL, "BATCH force needs host_values[nbatch][3]");
            for (int b = 0; b < g.nb; ++b)
                for (int y = 0; y < g.ny; ++y)
                    for (int a = 0; a < 3; ++a) tab[3 * ((size_t)b * g.ny + y) + a] = host_values[3 * b + a];
            break;
        case CMLBM_FORCE_PROFILE_Y:
            if (!host_values) return fail(lat, CMLBM_EINVAL, "PROFILE_Y force needs host_values[ny][3]");
            for (int b = 0; b < g.nb; ++b)
                for (int y = 0; y < g.ny; ++y)
                    for (int a = 0; a < 3; ++a) tab[3 * ((size_t)b * g.ny + y) + a] = host_values[3 * y + a];
            break;
        case CMLBM_FORCE_FIELD: {
            const int need = lat->p.storage == CMLBM_FP64 ? CMLBM_FP64 : CMLBM_FP32;
            if (!dev_field) return fail(lat, CMLBM_EINVAL, "FIELD force needs dev_field[3][N]");
            if (io_dtype != need)
                return fail(lat, CMLBM_EINVAL, "FIELD force dtype must be FP64 for FP64 storage, FP32 otherwise");
            if ((uintptr_t)dev_field & (need == CMLBM_FP64 ? 7u : 3u))
                return fail(lat, CMLBM_EINVAL, "FIELD force pointer misaligned");
            break;
        }
        default: return fail(lat, CMLBM_EINVAL, "unknown force mode");
    }
    for (double v : tab)
        if (!std::isfinite(v)) return fail(lat, CMLBM_EINVAL, "non-finite force");
    std::vector<float> tab32(tab.begin(), tab.end());
    int rc = hip_check(lat,
                       hipMemcpyAsync(lat->scratch + lat->off_ftab64, tab.data(), tab.size() * sizeof(double),
                                      hipMemcpyHostToDevice, s),
                       "force table copy");
    if (rc) return rc;
    rc = hip_check(lat,
                   hipMemcpyAsync(lat->scratch + lat->off_ftab32, tab32.data(), tab32.size() * sizeof(float),
                                  hipMemcpyHostToDevice, s),
                   "force table copy");
    if (rc) return rc;
    // the host vectors die on return: make sure the copies have consumed them
    rc = hip_check(lat, hipStreamSynchronize(s), "force table sync");
    if (rc) return rc;
    lat->force_mode = mode;
    lat->field = mode == CMLBM_FORCE_FIELD ? dev_field : nullptr;
    lat->field_dtype = io_dtype;
    return CMLBM_OK;
}

static int ensure_force(cmlbm_lattice* lat, hipStream_t s)
{
    if (lat->force_mode >= 0) return CMLBM_OK;
    return cmlbm_set_force(lat, CMLBM_FORCE_NONE, nullptr, nullptr, CMLBM_FP64, s);
}

int cmlbm_init(cmlbm_lattice* lat, const void* dev_rho, const void* dev_u, int io_dtype, void* hip_stream)
{
    if (!lat) return CMLBM_EINVAL;
    if (io_dtype != CMLBM_FP64 && io_dtype != CMLBM_FP32) return fail(lat, CMLBM_EINVAL, "io_dtype must be FP64/FP32");
    hipStream_t s = (hipStream_t)hip_stream;
    int rc = ensure_mask(lat, s);
    if (rc) return rc;
    rc = ensure_force(lat, s);
    if (rc) return rc;
    rc = launch_init(lat, io_dtype == CMLBM_FP64 ? INIT_EQ_F64 : INIT_EQ_F32, dev_rho, dev_u, nullptr, s);
    if (rc) return rc;
    lat->initialized = true;
    lat->snap_valid = false;
    lat->t = 0;
    return CMLBM_OK;
}

int cmlbm_load_populations(cmlbm_lattice* lat, const double* dev_in, void* hip_stream)
{
    if (!lat || !dev_in) return CMLBM_EINVAL;
    if (lat->p.storage == CMLBM_MOM32)
        return fail(lat, CMLBM_EINVAL, "moment storage keeps nine numbers per cell: populations cannot be loaded");
    hipStream_t s = (hipStream_t)hip_stream;
    int rc = ensure_mask(lat, s);
    if (rc) return rc;
    rc = ensure_force(lat, s);
    if (rc) return rc;
    rc = launch_init(lat, INIT_POPS_F64, nullptr, nullptr, dev_in, s);
    if (rc) return rc;
    lat->initialized = true;
    lat->snap_valid = false;
    return CMLBM_OK;
}

int cmlbm_step(cmlbm_lattice* lat, int32_t nsteps, void* hip_stream)
{
    if (!lat || nsteps < 0) return CMLBM_EINVAL;
    if (!lat->initialized) return fail(lat, CMLBM_ESTATE, "step before init");
    hipStream_t s = (hipStream_t)hip_stream;
    for (int32_t k = 0; k < nsteps; ++k) {
        int rc = launch_step(lat, s);
        if (rc) return rc;
        lat->cur = 1 - lat->cur;
        lat->t += 1;
    }
    return CMLBM_OK;
}

int cmlbm_moments(cmlbm_lattice* lat, void* dev_rho, void* dev_u, int io_dtype, void* hip_stream)
{
    if (!lat) return CMLBM_EINVAL;
    if (io_dtype != CMLBM_FP64 && io_dtype != CMLBM_FP32) return fail(lat, CMLBM_EINVAL, "io_dtype must be FP64/FP32");
    if (!lat->initialized) return fail(lat, CMLBM_ESTATE, "moments before init");
    if (!dev_rho && !dev_u) return CMLBM_OK;
    return launch_gather(lat, dev_rho, dev_u, io_dtype == CMLBM_FP64, nullptr, (hipStream_t)hip_stream);
}

int cmlbm_populations(cmlbm_lattice* lat, double* dev_out, void* hip_stream)
{
    if (!lat || !dev_out) return CMLBM_EINVAL;
    if (lat->p.storage == CMLBM_MOM32)
        return fail(lat, CMLBM_ESTATE, "moment storage keeps the post-collision state: no pre-collision populations");
    if (!lat->initialized) return fail(lat, CMLBM_ESTATE, "populations before init");
    return launch_gather(lat, nullptr, nullptr, 1, dev_out, (hipStream_t)hip_stream);
}

int cmlbm_pseudopotential_force(cmlbm_lattice* lat, double G, const void* dev_rho, int io_dtype, void* dev_field,
                                void* hip_stream)
{
    if (!lat || !dev_rho || !dev_field || !std::isfinite(G)) return CMLBM_EINVAL;
    if (lat->p.wall[0] || lat->p.wall[1] || lat->p.wall[2] || (lat->p.flags & CMLBM_FLAG_SOLID))
        return fail(lat, CMLBM_EINVAL, "the pseudo-potential force needs a periodic lattice without solids");
    const int need = lat->p.storage == CMLBM_FP64 ? CMLBM_FP64 : CMLBM_FP32;
    if (io_dtype != need)
        return fail(lat, CMLBM_EINVAL, "pseudo-potential dtype must be FP64 for FP64 storage, FP32 otherwise");
    const Geom& g = lat->g;
    hipStream_t s = (hipStream_t)hip_stream;
    if (!lat->psi_zc)
        lat->psi_zc = need == CMLBM_FP64 ? psi_chunk<double>(g, lat->cus) : psi_chunk<float>(g, lat->cus);
    const int zc = lat->psi_zc;
    const uint64_t tiles = (uint64_t)((g.nx + kPsiTX - 1) / kPsiTX) * ((g.ny + kPsiTY - 1) / kPsiTY) *
                           ((g.nz + zc - 1) / zc) * g.nb;
    if (tiles > 0x7fffffffULL) return fail(lat, CMLBM_EINVAL, "lattice too large for the pseudo-potential tiles");
    if (need == CMLBM_FP64)
        k_pseudopotential<double><<<(unsigned)tiles, 256, 0, s>>>(g, G, zc, (const double*)dev_rho,
                                                                 (double*)dev_field);
    else
        k_pseudopotential<float><<<(unsigned)tiles, 256, 0, s>>>(g, (float)G, zc, (const float*)dev_rho,
                                                                (float*)dev_field);
    return launch_check(lat, "pseudo-potential force");
}

int cmlbm_reduce(cmlbm_lattice* lat, uint32_t what, double* host_out, void* hip_stream)
{
    if (!lat || !host_out) return CMLBM_EINVAL;
    if (what & ~(CMLBM_REDUCE_RESIDUAL | CMLBM_REDUCE_SNAPSHOT)) return fail(lat, CMLBM_EINVAL, "unknown reduce bits");
    if (!lat->initialized) return fail(lat, CMLBM_ESTATE, "reduce before init");
    const bool residual = what & CMLBM_REDUCE_RESIDUAL, snapshot = what & CMLBM_REDUCE_SNAPSHOT;
    if ((residual || snapshot) && !(lat->p.flags & CMLBM_FLAG_RESIDUAL))
        return fail(lat, CMLBM_ESTATE, "residual/snapshot need CMLBM_FLAG_RESIDUAL");
    if (residual && !lat->snap_valid) return fail(lat, CMLBM_ESTATE, "residual before any snapshot");
    hipStream_t s = (hipStream_t)hip_stream;
    int rc = launch_reduce(lat, residual, snapshot, s);
    if (rc) return rc;
    const size_t nb = lat->g.nb;
    rc = hip_check(lat,
                   hipMemcpyAsync(host_out, lat->scratch + lat->off_final, nb * CMLBM_NRED * sizeof(double),
                                  hipMemcpyDeviceToHost, s),
                   "reduce copy");
    if (rc) return rc;
    rc = hip_check(lat, hipStreamSynchronize(s), "reduce sync");
    if (rc) return rc;
    if (snapshot) lat->snap_valid = true;
    return finish_reduce(lat, residual, host_out);
}

int cmlbm_step_reduce(cmlbm_lattice* lat, double* host_out, void* hip_stream)
{
    if (!lat || !host_out) return CMLBM_EINVAL;
    if (!(lat->p.flags & CMLBM_FLAG_FUSED_REDUCE))
        return fail(lat, CMLBM_ESTATE, "step_reduce needs CMLBM_FLAG_FUSED_REDUCE");
    if (!lat->initialized) return fail(lat, CMLBM_ESTATE, "step_reduce before init");
    hipStream_t s = (hipStream_t)hip_stream;
    int rc = launch_step_red(lat, s);
    if (rc) return rc;
    lat->cur = 1 - lat->cur;
    lat->t += 1;
    rc = hip_check(lat,
                   hipMemcpyAsync(host_out, lat->scratch + lat->off_final, lat->g.nb * CMLBM_NRED * sizeof(double),
                                  hipMemcpyDeviceToHost, s),
                   "step_reduce copy");
    if (rc) return rc;
    rc = hip_check(lat, hipStreamSynchronize(s), "step_reduce sync");
    if (rc) return rc;
    return finish_reduce(lat, false, host_out);
}

int cmlbm_save_state(cmlbm_lattice* lat, void* dev_blob, size_t blob_bytes, void* hip_stream)
{
    if (!lat || !dev_blob) return CMLBM_EINVAL;
    if (!lat->initialized) return fail(lat, CMLBM_ESTATE, "save_state before init");
    Layout L;
    make_layout(&lat->p, &L);
    if (blob_bytes < L.pop_bytes) return fail(lat, CMLBM_ENOMEM, "state blob too small");
    return hip_check(lat,
                     hipMemcpyAsync(dev_blob, lat->pop[lat->cur], L.pop_bytes, hipMemcpyDeviceToDevice,
                                    (hipStream_t)hip_stream),
                     "save_state copy");
}

int cmlbm_restore_state(cmlbm_lattice* lat, const void* dev_blob, size_t blob_bytes, void* hip_stream)
{
    if (!lat || !dev_blob) return CMLBM_EINVAL;
    Layout L;
    make_layout(&lat->p, &L);
    if (blob_bytes < L.pop_bytes) return fail(lat, CMLBM_ENOMEM, "state blob too small");
    hipStream_t s = (hipStream_t)hip_stream;
    int rc = ensure_mask(lat, s);
    if (rc) return rc;
    rc = ensure_force(lat, s);
    if (rc) return rc;
    rc = hip_check(lat, hipMemcpyAsync(lat->pop[lat->cur], dev_blob, L.pop_bytes, hipMemcpyDeviceToDevice, s),
                   "restore_state copy");
    if (rc) return rc;
    lat->initialized = true;
    lat->snap_valid = false;
    return CMLBM_OK;
}

int cmlbm_get_time(const cmlbm_lattice* lat, int64_t* t)
{
    if (!lat || !t) return CMLBM_EINVAL;
    *t = lat->t;
    return CMLBM_OK;
}

int cmlbm_set_time(cmlbm_lattice* lat, int64_t t)
{
    if (!lat || t < 0) return CMLBM_EINVAL;
    lat->t = t;
    return CMLBM_OK;
}

int cmlbm_destroy(cmlbm_lattice* lat)
{
    delete lat;
    return CMLBM_OK;
}

const char* cmlbm_last_error(const cmlbm_lattice* lat) { return lat ? lat->err.c_str() : ""; }

int cmlbm_device_copy(void* dev_dst, const void* dev_src, size_t bytes, void* hip_stream)
{
    if (!dev_dst || !dev_src || bytes == 0 || bytes % 16 || ((uintptr_t)dev_dst | (uintptr_t)dev_src) % 16)
        return CMLBM_EINVAL;
    const char *d = (const char*)dev_dst, *sp = (const char*)dev_src;
    if (d < sp + bytes && sp < d + bytes) return CMLBM_EINVAL;  // overlapping
    const uint64_t n = bytes / 16;
    uint64_t blocks = (bytes + (64ull << 20) - 1) / (64ull << 20) * 1024;
    const uint64_t need = (n + kBlock * 4 - 1) / (kBlock * 4);
    if (blocks > need) blocks = need;
    k_copy16<<<dim3((unsigned)blocks), dim3(kBlock), 0, (hipStream_t)hip_stream>>>((const v4i*)dev_src, (v4i*)dev_dst, n);
    return hipGetLastError() == hipSuccess ? CMLBM_OK : CMLBM_EHIP;
}

int cmlbm_plane_copy(void* dev_dst, const void* dev_src, int32_t planes, int64_t cells, int64_t plane_stride,
                     void* hip_stream)
{
    if (!dev_dst || !dev_src || (planes != 9 && planes != 27) || cells < 1 || plane_stride < cells ||
        ((uintptr_t)dev_dst | (uintptr_t)dev_src) % 4)
        return CMLBM_EINVAL;
    const uint64_t span = ((uint64_t)(planes - 1) * (uint64_t)plane_stride + (uint64_t)cells) * 4;
    const char *d = (const char*)dev_dst, *sp = (const char*)dev_src;
    if (d < sp + span && sp < d + span) return CMLBM_EINVAL;  // overlapping
    const uint64_t blocks = ((uint64_t)cells + 1023) / 1024;
    if (blocks > 0x7fffffffULL) return CMLBM_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    if (planes == 27)
        k_copy_planes<27><<<dim3((unsigned)blocks), dim3(1024), 0, s>>>((const float*)dev_src, (float*)dev_dst,
                                                                       (uint64_t)cells, (uint64_t)plane_stride);
    else
        k_copy_planes<9><<<dim3((unsigned)blocks), dim3(1024), 0, s>>>((const float*)dev_src, (float*)dev_dst,
                                                                      (uint64_t)cells, (uint64_t)plane_stride);
    return hipGetLastError() == hipSuccess ? CMLBM_OK : CMLBM_EHIP;
}

int cmlbm_row_block_copy(void* dev_dst, const void* dev_src, int64_t rows, int32_t row_len, void* hip_stream)
{
    if (!dev_dst || !dev_src || rows < 1 || row_len < 1 || ((uintptr_t)dev_dst | (uintptr_t)dev_src) % 4)
        return CMLBM_EINVAL;
    if ((uint64_t)rows >= (1ULL << 40) / (27ULL * 4ULL * (uint64_t)row_len)) return CMLBM_EINVAL;  // 2^40-byte spans
    const uint64_t cells = (uint64_t)rows * (uint64_t)row_len;
    const uint64_t span = cells * 27 * 4;
    const char *d = (const char*)dev_dst, *sp = (const char*)dev_src;
    if (d < sp + span && sp < d + span) return CMLBM_EINVAL;  // overlapping
    const uint64_t blocks = (cells + 1023) / 1024;
    if (blocks > 0x7fffffffULL) return CMLBM_EINVAL;
    k_copy_row_blocks<<<dim3((unsigned)blocks), dim3(1024), 0, (hipStream_t)hip_stream>>>(
        (const float*)dev_src, (float*)dev_dst, cells, (uint32_t)row_len);
    return hipGetLastError() == hipSuccess ? CMLBM_OK : CMLBM_EHIP;
}

const char* cmlbm_status_string(int status)
{
    switch (status) {
        case CMLBM_OK: return "CMLBM_OK";
        case CMLBM_EINVAL: return "CMLBM_EINVAL";
        case CMLBM_ENOMEM: return "CMLBM_ENOMEM";
        case CMLBM_EHIP: return "CMLBM_EHIP";
        case CMLBM_EUNSTABLE: return "CMLBM_EUNSTABLE";
        case CMLBM_ESTATE: return "CMLBM_ESTATE";
        default: return "CMLBM_UNKNOWN";
    }
}

}  // extern "C"
