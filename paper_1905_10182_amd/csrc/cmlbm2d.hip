// Two-dimensional D2Q9 central-moment lattice Boltzmann solver with Hermite
// forcing for gfx950 (MI355X): the model of App. B of De Rosis, Huang &
// Coreixas, PRE 2019.  C ABI: include/cmlbm2d.h.  The per-cell collision is in
// d2q9.hpp; this file holds the kernels and the host side.
//
// Data layout in HBM: every population in rows of nx values padded to 256
// bytes; FP32 and 16-bit storage keep the nine population rows of one lattice
// row together (row blocks, [ny][9][row]), FP64 keeps nine planes of ny rows
// kPlanePad bytes apart beyond their rows; values stored shifted (f_i - w_i rho0) in the storage type; two such
// buffers alternate (read one, write the other).  The stored array A_i(y)
// holds the population that the next pull gather moves to y + c_i, so
// f_i(x, t) = A_i(x - c_i): a step is gather (streaming), collision and a
// store at the cell's own index.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <string>

#include "cmlbm2d.h"
#include "d2q9.hpp"

using namespace cmlbm2d;

// Cells per lane of the step kernel for each storage type (overridable for
// tuning builds); a value above 1 is used only when it divides nx.
#ifndef CMLBM2D_LANES_FP64
#define CMLBM2D_LANES_FP64 1
#endif
#ifndef CMLBM2D_LANES_FP32
#define CMLBM2D_LANES_FP32 2
#endif
#ifndef CMLBM2D_LANES_16
#define CMLBM2D_LANES_16 4
#endif

namespace {

constexpr int kBlock = 256;         // threads per workgroup
constexpr size_t kPlanePad = 4096;  // bytes between consecutive FP64 population planes (a multiple of 256)

// ---------------------------------------------------------------------------
// storage types: S is stored, T is the arithmetic type

template <int ST>
struct storage2;
template <>
struct storage2<CMLBM2D_FP64> {
    typedef double S;
    typedef double T;
    static __device__ __forceinline__ T load(S v) { return v; }
    static __device__ __forceinline__ S pack(T v) { return v; }
};
template <>
struct storage2<CMLBM2D_FP32> {
    typedef float S;
    typedef float T;
    static __device__ __forceinline__ T load(S v) { return v; }
    static __device__ __forceinline__ S pack(T v) { return v; }
};
// FP16 carries a factor 2^8 so that the small shifted populations stay in
// its normal range.
template <>
struct storage2<CMLBM2D_FP16> {
    typedef _Float16 S;
    typedef float T;
    static __device__ __forceinline__ T load(S v) { return (float)v * 0.00390625f; }
    static __device__ __forceinline__ S pack(T v) { return (_Float16)(v * 256.0f); }
};
template <>
struct storage2<CMLBM2D_BF16> {
    typedef __bf16 S;
    typedef float T;
    static __device__ __forceinline__ T load(S v) { return (float)v; }
    static __device__ __forceinline__ S pack(T v) { return (__bf16)v; }
};

size_t storage_bytes(int st) { return st == CMLBM2D_FP64 ? 8 : st == CMLBM2D_FP32 ? 4 : 2; }

struct Geom2 {
    int nx, ny;
    int nxp;           // padded row length (elements)
    int V;             // cells per lane of the step kernel
    int segs;          // 64-lane segments per row in the step kernel
    int nblk;          // step workgroups
    uint64_t pstride;  // elements from population i to i + 1 of one row
    uint64_t rstride;  // elements from one row of a population to the next row
    uint64_t ncell;    // ny * nx
};

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// lane l receives the value of lane l - 1 (mod 64) / lane l + 1 (mod 64)
__device__ __forceinline__ int from_prev_lane(int v) { return __builtin_amdgcn_mov_dpp(v, 0x13C, 0xF, 0xF, false); }
__device__ __forceinline__ int from_next_lane(int v) { return __builtin_amdgcn_mov_dpp(v, 0x134, 0xF, 0xF, false); }

template <typename S>
__device__ __forceinline__ S shift_lane(S v, bool prev)
{
    if constexpr (sizeof(S) == 8) {
        const int2 w = __builtin_bit_cast(int2, v);
        int2 r;
        r.x = prev ? from_prev_lane(w.x) : from_next_lane(w.x);
        r.y = prev ? from_prev_lane(w.y) : from_next_lane(w.y);
        return __builtin_bit_cast(S, r);
    } else if constexpr (sizeof(S) == 4) {
        const int w = __builtin_bit_cast(int, v);
        return __builtin_bit_cast(S, prev ? from_prev_lane(w) : from_next_lane(w));
    } else {
        const int w = (int)__builtin_bit_cast(unsigned short, v);
        const int r = prev ? from_prev_lane(w) : from_next_lane(w);
        return __builtin_bit_cast(S, (unsigned short)r);
    }
}

template <typename X>
__device__ __forceinline__ X load_at(const void* base, uint32_t byte_off)
{
    return *(const X*)((const char*)base + byte_off);
}

// Non-temporal store: the post-collision populations are not read again in
// this step.
template <typename X>
__device__ __forceinline__ void store_nt(void* base, uint32_t byte_off, X v)
{
    X* p = (X*)((char*)base + byte_off);
    if constexpr (sizeof(X) == 16) {
        typedef int i4 __attribute__((ext_vector_type(4)));
        __builtin_nontemporal_store(__builtin_bit_cast(i4, v), (i4*)p);
    } else if constexpr (sizeof(X) == 8) {
        __builtin_nontemporal_store(__builtin_bit_cast(unsigned long long, v), (unsigned long long*)p);
    } else if constexpr (sizeof(X) == 4) {
        __builtin_nontemporal_store(__builtin_bit_cast(unsigned, v), (unsigned*)p);
    } else {
        __builtin_nontemporal_store(__builtin_bit_cast(unsigned short, v), (unsigned short*)p);
    }
}

// ---------------------------------------------------------------------------
// the hot path: one fused time step
//
// Wave w owns segment (w mod segs) of row (w / segs): 64 lanes x V cells.
// Every cell pulls its nine populations from x - c_i (periodic), collides
// (cmlbm2d::collide) and stores the nine post-collision values at its own
// index.  With V > 1 each lane reads every plane as one aligned V-element
// vector; the six planes with c_x = +-1 need the row shifted by one cell,
// done in registers: the element crossing a lane boundary comes from the
// neighbouring lane by a DPP wave rotation (which is also the periodic wrap
// when a row is exactly one wave), and the end lanes of a segment otherwise
// reload that element.  Row addressing is wave-uniform (scalar registers);
// each access is a scalar base plus a 32-bit per-lane byte offset.

template <int ST, int V, bool FIELD>
__global__ __launch_bounds__(kBlock) void k2_step(const typename storage2<ST>::S* __restrict__ src,
                                                   typename storage2<ST>::S* __restrict__ dst, Geom2 g,
                                                   typename storage2<ST>::T omega, typename storage2<ST>::T rho0,
                                                   typename storage2<ST>::T fx, typename storage2<ST>::T fy,
                                                   const typename storage2<ST>::T* __restrict__ field)
{
    using SS = storage2<ST>;
    using S = typename SS::S;
    using T = typename SS::T;
    typedef S vt __attribute__((ext_vector_type(V == 1 ? 2 : V)));
    const int blk = (int)blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(blk * (kBlock / 64) + (int)(threadIdx.x >> 6));
    const int row = wave / g.segs;
    if (row >= g.ny) return;  // whole wave
    const int seg = wave - row * g.segs;
    const int x0 = (seg * 64 + lane) * V;
    const bool active = x0 < g.nx;
    const S* srow[3];  // [c_y + 1]: source row y - c_y
#pragma unroll
    for (int b = 0; b < 3; ++b) srow[b] = src + (uint64_t)wrap(row - (b - 1), g.ny) * g.rstride;
    T h[V][9];
    if constexpr (V == 1) {
        if (!active) return;
        const uint32_t bx[3] = {(uint32_t)wrap(x0 + 1, g.nx) * (uint32_t)sizeof(S), (uint32_t)x0 * (uint32_t)sizeof(S),
                                (uint32_t)wrap(x0 - 1, g.nx) * (uint32_t)sizeof(S)};
#pragma unroll
        for (int i = 0; i < 9; ++i)
            h[0][i] = SS::load(load_at<S>(srow[vel_y(i) + 1] + (uint64_t)i * g.pstride, bx[vel_x(i) + 1]));
    } else {
        const bool whole = g.nx == 64 * V;
        const bool prev_in_reg = whole || lane > 0;
        const bool next_in_reg = whole || (lane < 63 && x0 + V < g.nx);
        const uint32_t bxm = (uint32_t)(x0 == 0 ? g.nx - 1 : x0 - 1) * (uint32_t)sizeof(S);
        const uint32_t bxp = (uint32_t)(x0 + V >= g.nx ? 0 : x0 + V) * (uint32_t)sizeof(S);
        const uint32_t bx0 = (uint32_t)x0 * (uint32_t)sizeof(S);
        vt v[9];
#pragma unroll
        for (int i = 0; i < 9; ++i)
            v[i] = active ? load_at<vt>(srow[vel_y(i) + 1] + (uint64_t)i * g.pstride, bx0) : vt(0);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            if (vel_x(i) == 0) {
#pragma unroll
                for (int c = 0; c < V; ++c) h[c][i] = SS::load(v[i][c]);
                continue;
            }
            // cell c of a c_x = +1 plane reads element c - 1, of a c_x = -1 plane element c + 1
            const bool prev = vel_x(i) == 1;
            S e = shift_lane<S>(prev ? v[i][V - 1] : v[i][0], prev);
            if (!(prev ? prev_in_reg : next_in_reg) && active)
                e = load_at<S>(srow[vel_y(i) + 1] + (uint64_t)i * g.pstride, prev ? bxm : bxp);
#pragma unroll
            for (int c = 0; c < V; ++c) {
                const S s = prev ? (c == 0 ? e : v[i][c - 1]) : (c == V - 1 ? e : v[i][c + 1]);
                h[c][i] = SS::load(s);
            }
        }
        if (!active) return;
    }
    T Fx[V], Fy[V];
#pragma unroll
    for (int c = 0; c < V; ++c) {
        if (FIELD) {
            const uint64_t lin = (uint64_t)row * (uint64_t)g.nx + (uint64_t)(x0 + c);
            Fx[c] = field[lin];
            Fy[c] = field[g.ncell + lin];
        } else {
            Fx[c] = fx;
            Fy[c] = fy;
        }
    }
#pragma unroll
    for (int c = 0; c < V; ++c) {
        T drho, ux, uy;
        collide<T>(h[c], Fx[c], Fy[c], omega, rho0, drho, ux, uy);
    }
    const uint32_t own = (uint32_t)x0 * (uint32_t)sizeof(S);
    const uint64_t orow = (uint64_t)row * g.rstride;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        S* plane_row = dst + (uint64_t)i * g.pstride + orow;
        if constexpr (V == 1) {
            store_nt<S>(plane_row, own, SS::pack(h[0][i]));
        } else {
            vt o;
#pragma unroll
            for (int c = 0; c < V; ++c) o[c] = SS::pack(h[c][i]);
            store_nt<vt>(plane_row, own, o);
        }
    }
}

// ---------------------------------------------------------------------------
// cell-parallel kernels (one thread per cell, 1D grid over the N cells)

enum InitSrc { INIT_EQ_F64 = 0, INIT_EQ_F32 = 1, INIT_POPS_F64 = 2 };

// Write a pre-collision state through the inverse of the pull gather:
// A_i(x - c_i) = h_i(x).  The complete equilibrium is the reconstruction with
// zero force and zero shear moments (all its central moments are those of
// the post-collision state of a force-free, fully relaxed cell).
template <int ST, int SRC>
__global__ __launch_bounds__(kBlock) void k2_init(typename storage2<ST>::S* __restrict__ dst, Geom2 g, double rho0,
                                                  const void* __restrict__ rho_in, const void* __restrict__ u_in,
                                                  const double* __restrict__ pops)
{
    using SS = storage2<ST>;
    using T = typename SS::T;
    const uint64_t n = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.ncell) return;
    const int x = (int)(n % (uint64_t)g.nx), y = (int)(n / (uint64_t)g.nx);
    T e[9];
    if constexpr (SRC == INIT_POPS_F64) {
#pragma unroll
        for (int i = 0; i < 9; ++i) e[i] = (T)(pops[(uint64_t)i * g.ncell + n] - weight(i) * rho0);
    } else {
        T drho = T(0), ux = T(0), uy = T(0);
        if constexpr (SRC == INIT_EQ_F64) {
            const double* R = (const double*)rho_in;
            const double* U = (const double*)u_in;
            if (R) drho = (T)(R[n] - rho0);
            if (U) {
                ux = (T)U[n];
                uy = (T)U[g.ncell + n];
            }
        } else {
            const float* R = (const float*)rho_in;
            const float* U = (const float*)u_in;
            if (R) drho = (T)((double)R[n] - rho0);
            if (U) {
                ux = (T)U[n];
                uy = (T)U[g.ncell + n];
            }
        }
        reconstruct<T>(drho, ux, uy, T(0), T(0), T(0), T(0), (T)rho0, e);
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const uint64_t d = (uint64_t)i * g.pstride + (uint64_t)wrap(y - vel_y(i), g.ny) * g.rstride +
                           (uint64_t)wrap(x - vel_x(i), g.nx);
        dst[d] = SS::pack(e[i]);
    }
}

// Gather the pre-collision state of every cell: rho and the half-force
// velocity (FP64 or FP32 out), and/or the unshifted FP64 populations.
template <int ST>
__global__ __launch_bounds__(kBlock) void k2_gather(const typename storage2<ST>::S* __restrict__ src, Geom2 g,
                                                    double rho0, double fx, double fy, const void* __restrict__ field,
                                                    void* __restrict__ rho_out, void* __restrict__ u_out, int out_f64,
                                                    double* __restrict__ pops)
{
    using SS = storage2<ST>;
    const uint64_t n = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.ncell) return;
    const int x = (int)(n % (uint64_t)g.nx), y = (int)(n / (uint64_t)g.nx);
    double h[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const uint64_t s = (uint64_t)i * g.pstride + (uint64_t)wrap(y - vel_y(i), g.ny) * g.rstride +
                           (uint64_t)wrap(x - vel_x(i), g.nx);
        h[i] = (double)SS::load(src[s]);
    }
    if (pops) {
#pragma unroll
        for (int i = 0; i < 9; ++i) pops[(uint64_t)i * g.ncell + n] = h[i] + weight(i) * rho0;
    }
    if (!rho_out && !u_out) return;
    double Fx = fx, Fy = fy;
    if (field) {
        if (ST == CMLBM2D_FP64) {
            Fx = ((const double*)field)[n];
            Fy = ((const double*)field)[g.ncell + n];
        } else {
            Fx = ((const float*)field)[n];
            Fy = ((const float*)field)[g.ncell + n];
        }
    }
    double drho = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        drho += h[i];
        jx += vel_x(i) * h[i];
        jy += vel_y(i) * h[i];
    }
    const double rho = rho0 + drho;
    const double ux = (jx + 0.5 * Fx) / rho, uy = (jy + 0.5 * Fy) / rho;
    if (out_f64) {
        if (rho_out) ((double*)rho_out)[n] = rho;
        if (u_out) {
            ((double*)u_out)[n] = ux;
            ((double*)u_out)[g.ncell + n] = uy;
        }
    } else {
        if (rho_out) ((float*)rho_out)[n] = (float)rho;
        if (u_out) {
            ((float*)u_out)[n] = (float)ux;
            ((float*)u_out)[g.ncell + n] = (float)uy;
        }
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// host side

struct cmlbm2d_lattice {
    cmlbm2d_params p;
    Geom2 g;
    void* pop[2];
    int cur;  // buffer holding the state
    int force_mode;
    double fu[2];  // UNIFORM force
    const void* field;
    bool initialized;
    int64_t t;
    std::string err;
};

namespace {

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

int lanes_for(int storage, int nx)
{
    int want = storage == CMLBM2D_FP64 ? CMLBM2D_LANES_FP64
                                        : storage == CMLBM2D_FP32 ? CMLBM2D_LANES_FP32 : CMLBM2D_LANES_16;
    const int vmax = 16 / (int)storage_bytes(storage);  // vectors of at most 16 bytes
    if (want > vmax) want = vmax;
    if (want > 4) want = 4;  // the step kernel is instantiated for 1, 2 and 4 cells per lane
    for (int v = want; v > 1; v /= 2)
        if (nx % v == 0) return v;
    return 1;
}

// Population layout: row blocks (the nine population rows of one lattice row
// stored together) for FP32 and 16-bit storage, planes (population i of every
// row together, 4 KiB apart) for FP64.  Measured at 8192^2 against planes: FP32
// +10%, FP16 +2.5%, FP64 -2.5% (against its spaced planes).
bool row_blocks2(int storage) { return storage != CMLBM2D_FP64; }

int make_geom(const cmlbm2d_params* p, Geom2* g, size_t* pop_bytes)
{
    if (!p) return CMLBM2D_EINVAL;
    if (p->nx < 1 || p->ny < 1) return CMLBM2D_EINVAL;
    if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return CMLBM2D_EINVAL;
    if (!(p->rho0 > 0.0) || !std::isfinite(p->rho0)) return CMLBM2D_EINVAL;
    if (p->storage < CMLBM2D_FP64 || p->storage > CMLBM2D_BF16) return CMLBM2D_EINVAL;
    if (p->flags != 0) return CMLBM2D_EINVAL;
    const size_t sb = storage_bytes(p->storage);
    g->nx = p->nx;
    g->ny = p->ny;
    g->nxp = (int)(align256((size_t)p->nx * sb) / sb);
    // FP64 planes kPlanePad bytes apart beyond their rows (at power-of-two plane sizes the
    // nine plane streams otherwise share HBM channels); measured on 8192^2 it raises FP64 by
    // 6% (dense planes lowered FP16/BF16 by 6% with it, before their row blocks)
    const size_t pad = p->storage == CMLBM2D_FP64 ? kPlanePad : 0;
    const uint64_t plane = (uint64_t)p->ny * (uint64_t)g->nxp + pad / sb;
    if (plane * sb >= (1ULL << 32)) return CMLBM2D_EINVAL;  // one population's byte offsets are 32-bit
    const bool blocks = row_blocks2(p->storage);
    g->pstride = blocks ? (uint64_t)g->nxp : plane;
    g->rstride = blocks ? 9ull * g->nxp : (uint64_t)g->nxp;
    g->ncell = (uint64_t)p->ny * (uint64_t)p->nx;
    g->V = lanes_for(p->storage, p->nx);
    g->segs = (p->nx + 64 * g->V - 1) / (64 * g->V);
    const uint64_t waves = (uint64_t)p->ny * (uint64_t)g->segs;
    const uint64_t nblk = (waves + kBlock / 64 - 1) / (kBlock / 64);
    if (nblk > 0x7fffffffULL || (g->ncell + kBlock - 1) / kBlock > 0x7fffffffULL) return CMLBM2D_EINVAL;
    g->nblk = (int)nblk;
    if (pop_bytes) *pop_bytes = align256(blocks ? (uint64_t)p->ny * g->rstride * sb : 9 * plane * sb);
    return CMLBM2D_OK;
}

int fail(cmlbm2d_lattice* lat, int code, const std::string& msg)
{
    if (lat) lat->err = msg;
    return code;
}

int launch_check(cmlbm2d_lattice* lat, const char* what)
{
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) return CMLBM2D_OK;
    return fail(lat, CMLBM2D_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

dim3 cell_grid(const Geom2& g) { return dim3((unsigned)((g.ncell + kBlock - 1) / kBlock)); }

template <int ST, int V>
void launch_step_v(cmlbm2d_lattice* lat, hipStream_t s)
{
    using SS = storage2<ST>;
    using T = typename SS::T;
    const Geom2& g = lat->g;
    const auto* src = (const typename SS::S*)lat->pop[lat->cur];
    auto* dst = (typename SS::S*)lat->pop[1 - lat->cur];
    const T om = (T)(1.0 / lat->p.tau), r0 = (T)lat->p.rho0;
    if (lat->force_mode == CMLBM2D_FORCE_FIELD)
        k2_step<ST, V, true><<<dim3(g.nblk), dim3(kBlock), 0, s>>>(src, dst, g, om, r0, T(0), T(0),
                                                                    (const T*)lat->field);
    else
        k2_step<ST, V, false><<<dim3(g.nblk), dim3(kBlock), 0, s>>>(src, dst, g, om, r0, (T)lat->fu[0],
                                                                     (T)lat->fu[1], nullptr);
}

template <int ST>
void launch_step_st(cmlbm2d_lattice* lat, hipStream_t s)
{
    // vectors of at most 16 bytes per lane
    if constexpr (sizeof(typename storage2<ST>::S) <= 4) {
        if (lat->g.V == 4) return launch_step_v<ST, 4>(lat, s);
    }
    if (lat->g.V == 2) return launch_step_v<ST, 2>(lat, s);
    launch_step_v<ST, 1>(lat, s);
}

void launch_step(cmlbm2d_lattice* lat, hipStream_t s)
{
    switch (lat->p.storage) {
        case CMLBM2D_FP64: launch_step_st<CMLBM2D_FP64>(lat, s); break;
        case CMLBM2D_FP32: launch_step_st<CMLBM2D_FP32>(lat, s); break;
        case CMLBM2D_FP16: launch_step_st<CMLBM2D_FP16>(lat, s); break;
        default: launch_step_st<CMLBM2D_BF16>(lat, s); break;
    }
}

template <int ST>
void launch_init_st(cmlbm2d_lattice* lat, int src_kind, const void* rho, const void* u, const double* pops,
                    hipStream_t s)
{
    using SS = storage2<ST>;
    auto* dst = (typename SS::S*)lat->pop[lat->cur];
    const Geom2& g = lat->g;
    if (src_kind == INIT_EQ_F64)
        k2_init<ST, INIT_EQ_F64><<<cell_grid(g), dim3(kBlock), 0, s>>>(dst, g, lat->p.rho0, rho, u, nullptr);
    else if (src_kind == INIT_EQ_F32)
        k2_init<ST, INIT_EQ_F32><<<cell_grid(g), dim3(kBlock), 0, s>>>(dst, g, lat->p.rho0, rho, u, nullptr);
    else
        k2_init<ST, INIT_POPS_F64><<<cell_grid(g), dim3(kBlock), 0, s>>>(dst, g, lat->p.rho0, nullptr, nullptr,
                                                                         pops);
}

void launch_init(cmlbm2d_lattice* lat, int src_kind, const void* rho, const void* u, const double* pops, hipStream_t s)
{
    switch (lat->p.storage) {
        case CMLBM2D_FP64: launch_init_st<CMLBM2D_FP64>(lat, src_kind, rho, u, pops, s); break;
        case CMLBM2D_FP32: launch_init_st<CMLBM2D_FP32>(lat, src_kind, rho, u, pops, s); break;
        case CMLBM2D_FP16: launch_init_st<CMLBM2D_FP16>(lat, src_kind, rho, u, pops, s); break;
        default: launch_init_st<CMLBM2D_BF16>(lat, src_kind, rho, u, pops, s); break;
    }
}

template <int ST>
void launch_gather_st(cmlbm2d_lattice* lat, void* rho, void* u, int out_f64, double* pops, hipStream_t s)
{
    using SS = storage2<ST>;
    const Geom2& g = lat->g;
    const void* field = lat->force_mode == CMLBM2D_FORCE_FIELD ? lat->field : nullptr;
    k2_gather<ST><<<cell_grid(g), dim3(kBlock), 0, s>>>((const typename SS::S*)lat->pop[lat->cur], g, lat->p.rho0,
                                                        lat->fu[0], lat->fu[1], field, rho, u, out_f64, pops);
}

void launch_gather(cmlbm2d_lattice* lat, void* rho, void* u, int out_f64, double* pops, hipStream_t s)
{
    switch (lat->p.storage) {
        case CMLBM2D_FP64: launch_gather_st<CMLBM2D_FP64>(lat, rho, u, out_f64, pops, s); break;
        case CMLBM2D_FP32: launch_gather_st<CMLBM2D_FP32>(lat, rho, u, out_f64, pops, s); break;
        case CMLBM2D_FP16: launch_gather_st<CMLBM2D_FP16>(lat, rho, u, out_f64, pops, s); break;
        default: launch_gather_st<CMLBM2D_BF16>(lat, rho, u, out_f64, pops, s); break;
    }
}

bool aligned256(const void* p) { return ((uintptr_t)p & 255u) == 0; }

}  // namespace

extern "C" {

int cmlbm2d_required_bytes(const cmlbm2d_params* params, size_t* pop_buffer_bytes)
{
    Geom2 g;
    size_t bytes = 0;
    const int rc = make_geom(params, &g, &bytes);
    if (rc) return rc;
    if (pop_buffer_bytes) *pop_buffer_bytes = bytes;
    return CMLBM2D_OK;
}

int cmlbm2d_create(const cmlbm2d_params* params, void* pop_a, size_t pop_a_bytes, void* pop_b, size_t pop_b_bytes,
                   cmlbm2d_lattice** out)
{
    if (!out) return CMLBM2D_EINVAL;
    *out = nullptr;
    Geom2 g;
    size_t bytes = 0;
    const int rc = make_geom(params, &g, &bytes);
    if (rc) return rc;
    if (!pop_a || !pop_b || pop_a == pop_b) return CMLBM2D_EINVAL;
    if (!aligned256(pop_a) || !aligned256(pop_b)) return CMLBM2D_EINVAL;
    if (pop_a_bytes < bytes || pop_b_bytes < bytes) return CMLBM2D_ENOMEM;
    cmlbm2d_lattice* lat = new (std::nothrow) cmlbm2d_lattice();
    if (!lat) return CMLBM2D_ENOMEM;
    lat->p = *params;
    lat->g = g;
    lat->pop[0] = pop_a;
    lat->pop[1] = pop_b;
    lat->cur = 0;
    lat->force_mode = CMLBM2D_FORCE_NONE;
    lat->fu[0] = lat->fu[1] = 0.0;
    lat->field = nullptr;
    lat->initialized = false;
    lat->t = 0;
    *out = lat;
    return CMLBM2D_OK;
}

int cmlbm2d_set_force(cmlbm2d_lattice* lat, int mode, const double* host_values, const void* dev_field, int io_dtype,
                      void* hip_stream)
{
    (void)hip_stream;
    if (!lat) return CMLBM2D_EINVAL;
    switch (mode) {
        case CMLBM2D_FORCE_NONE:
            lat->fu[0] = lat->fu[1] = 0.0;
            lat->field = nullptr;
            break;
        case CMLBM2D_FORCE_UNIFORM:
            if (!host_values) return fail(lat, CMLBM2D_EINVAL, "UNIFORM force needs host_values[2]");
            if (!std::isfinite(host_values[0]) || !std::isfinite(host_values[1]))
                return fail(lat, CMLBM2D_EINVAL, "non-finite force");
            lat->fu[0] = host_values[0];
            lat->fu[1] = host_values[1];
            lat->field = nullptr;
            break;
        case CMLBM2D_FORCE_FIELD: {
            const int need = lat->p.storage == CMLBM2D_FP64 ? CMLBM2D_FP64 : CMLBM2D_FP32;
            if (!dev_field) return fail(lat, CMLBM2D_EINVAL, "FIELD force needs dev_field[2][N]");
            if (io_dtype != need)
                return fail(lat, CMLBM2D_EINVAL, "FIELD force dtype must be FP64 for FP64 storage, FP32 otherwise");
            if ((uintptr_t)dev_field & (need == CMLBM2D_FP64 ? 7u : 3u))
                return fail(lat, CMLBM2D_EINVAL, "FIELD force pointer misaligned");
            lat->fu[0] = lat->fu[1] = 0.0;
            lat->field = dev_field;
            break;
        }
        default: return fail(lat, CMLBM2D_EINVAL, "unknown force mode");
    }
    lat->force_mode = mode;
    return CMLBM2D_OK;
}

int cmlbm2d_init(cmlbm2d_lattice* lat, const void* dev_rho, const void* dev_u, int io_dtype, void* hip_stream)
{
    if (!lat) return CMLBM2D_EINVAL;
    if (io_dtype != CMLBM2D_FP64 && io_dtype != CMLBM2D_FP32)
        return fail(lat, CMLBM2D_EINVAL, "io_dtype must be FP64 or FP32");
    launch_init(lat, io_dtype == CMLBM2D_FP64 ? INIT_EQ_F64 : INIT_EQ_F32, dev_rho, dev_u, nullptr,
                (hipStream_t)hip_stream);
    const int rc = launch_check(lat, "init");
    if (rc) return rc;
    lat->initialized = true;
    lat->t = 0;
    return CMLBM2D_OK;
}

int cmlbm2d_step(cmlbm2d_lattice* lat, int32_t nsteps, void* hip_stream)
{
    if (!lat) return CMLBM2D_EINVAL;
    if (nsteps < 0) return fail(lat, CMLBM2D_EINVAL, "nsteps must be >= 0");
    if (!lat->initialized) return fail(lat, CMLBM2D_ESTATE, "step before init");
    hipStream_t s = (hipStream_t)hip_stream;
    for (int32_t k = 0; k < nsteps; ++k) {
        launch_step(lat, s);
        const int rc = launch_check(lat, "step");
        if (rc) return rc;
        lat->cur = 1 - lat->cur;
        ++lat->t;
    }
    return CMLBM2D_OK;
}

int cmlbm2d_moments(cmlbm2d_lattice* lat, void* dev_rho, void* dev_u, int io_dtype, void* hip_stream)
{
    if (!lat) return CMLBM2D_EINVAL;
    if (io_dtype != CMLBM2D_FP64 && io_dtype != CMLBM2D_FP32)
        return fail(lat, CMLBM2D_EINVAL, "io_dtype must be FP64 or FP32");
    if (!lat->initialized) return fail(lat, CMLBM2D_ESTATE, "moments before init");
    if (!dev_rho && !dev_u) return CMLBM2D_OK;
    launch_gather(lat, dev_rho, dev_u, io_dtype == CMLBM2D_FP64, nullptr, (hipStream_t)hip_stream);
    return launch_check(lat, "moments");
}

int cmlbm2d_populations(cmlbm2d_lattice* lat, double* dev_out, void* hip_stream)
{
    if (!lat || !dev_out) return CMLBM2D_EINVAL;
    if (!lat->initialized) return fail(lat, CMLBM2D_ESTATE, "populations before init");
    launch_gather(lat, nullptr, nullptr, 1, dev_out, (hipStream_t)hip_stream);
    return launch_check(lat, "populations");
}

int cmlbm2d_load_populations(cmlbm2d_lattice* lat, const double* dev_in, void* hip_stream)
{
    if (!lat || !dev_in) return CMLBM2D_EINVAL;
    launch_init(lat, INIT_POPS_F64, nullptr, nullptr, dev_in, (hipStream_t)hip_stream);
    const int rc = launch_check(lat, "load populations");
    if (rc) return rc;
    lat->initialized = true;
    return CMLBM2D_OK;
}

int cmlbm2d_get_time(const cmlbm2d_lattice* lat, int64_t* t)
{
    if (!lat || !t) return CMLBM2D_EINVAL;
    *t = lat->t;
    return CMLBM2D_OK;
}

int cmlbm2d_destroy(cmlbm2d_lattice* lat)
{
    delete lat;
    return CMLBM2D_OK;
}

const char* cmlbm2d_last_error(const cmlbm2d_lattice* lat) { return lat ? lat->err.c_str() : ""; }

const char* cmlbm2d_status_string(int status)
{
    switch (status) {
        case CMLBM2D_OK: return "CMLBM2D_OK";
        case CMLBM2D_EINVAL: return "CMLBM2D_EINVAL";
        case CMLBM2D_ENOMEM: return "CMLBM2D_ENOMEM";
        case CMLBM2D_EHIP: return "CMLBM2D_EHIP";
        case CMLBM2D_ESTATE: return "CMLBM2D_ESTATE";
        default: return "CMLBM2D_UNKNOWN";
    }
}

}  // extern "C"
