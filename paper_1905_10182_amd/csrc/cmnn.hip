// libcmnn: gfx950 kernels of the learned warm start (C ABI in include/cmnn.h).
//
// Convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16.  Operand
// layout of that instruction (checked on the hardware): lane l holds
// A[l % 16][(l / 16) * 8 + i] and B[(l / 16) * 8 + i][l % 16] for i < 8, and
// receives D[(l / 16) * 4 + i][l % 16] for i < 4.
//
//   k_conv_fwd      y[v][co] = act(sum_t sum_ci x[v + s*off(t)][ci] w[t][co][ci] + b[co])
//                   (s = +1; the data gradient is the same kernel with s = -1 and
//                   the transposed weights).  A = 16 voxels x 32 input channels,
//                   one 16-byte load per lane; B = 32 channels x 16 outputs.
//   k_conv_bwd_w    dw[t][co][ci] = sum_v dy[v][co] x[v + off(t)][ci]: the voxel
//                   axis is the MFMA K axis, so 32-voxel tiles of dy and x are
//                   staged through LDS transposed (channel-major) and read back
//                   as 16-byte fragments; per-chunk partials, fixed-order sum.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "cmnn.h"

namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

constexpr float kLeak = 0.1f;

struct G {
    int n, d, h, w;
    int per[3];
    long long nvox;
};

G make_g(const cmnn_geom* g)
{
    G r;
    r.n = g->n;
    r.d = g->d;
    r.h = g->h;
    r.w = g->w;
    for (int a = 0; a < 3; ++a) r.per[a] = g->periodic[a];
    r.nvox = (long long)g->n * g->d * g->h * g->w;
    return r;
}

// Positive extents and at most 2^31 - 1 voxels, so that every launch grid and
// per-voxel index fits the kernels' arithmetic.
bool geom_ok(const cmnn_geom* g)
{
    if (!g || g->n <= 0 || g->d <= 0 || g->h <= 0 || g->w <= 0) return false;
    return (long long)g->n * g->d * g->h * g->w <= 0x7fffffffLL;
}
bool chan_ok(int c) { return c > 0 && c % CMNN_CALIGN == 0; }
bool al16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

__device__ __forceinline__ bool shift_axis(int v, int dv, int n, int periodic, int& out)
{
    int s = v + dv;
    if (s < 0 || s >= n) {
        if (!periodic) return false;
        s = s < 0 ? s + n : s - n;
    }
    out = s;
    return true;
}

// Neighbour voxel of linear voxel m along tap t (sign s = +1 or -1); false if
// it falls into zero padding.
__device__ __forceinline__ bool neighbour(const G& g, long long m, int t, int s, long long& out)
{
    const int w = (int)(m % g.w);
    long long r = m / g.w;
    const int h = (int)(r % g.h);
    r /= g.h;
    const int d = (int)(r % g.d);
    const long long n = r / g.d;
    const int dz = s * (t / 9 - 1), dy = s * ((t / 3) % 3 - 1), dx = s * (t % 3 - 1);
    int nd, nh, nw;
    if (!shift_axis(d, dz, g.d, g.per[0], nd)) return false;
    if (!shift_axis(h, dy, g.h, g.per[1], nh)) return false;
    if (!shift_axis(w, dx, g.w, g.per[2], nw)) return false;
    out = ((n * g.d + nd) * g.h + nh) * g.w + nw;
    return true;
}

#define GRID_STRIDE(i, total) \
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < (total); i += (long long)gridDim.x * blockDim.x)

// The same with the index type I: the elementwise kernels below take 32-bit
// unsigned index arithmetic (a quarter of the 64-bit division's work) when
// every element index of the call fits, 64-bit otherwise.
#define GRID_STRIDE_I(I, i, total) \
    for (I i = (I)blockIdx.x * blockDim.x + threadIdx.x; i < (I)(total); i += (I)gridDim.x * blockDim.x)

__device__ __forceinline__ void unpack8(u4 v, float (&f)[8])
{
    const bf16x8 b = __builtin_bit_cast(bf16x8, v);
#pragma unroll
    for (int i = 0; i < 8; ++i) f[i] = (float)b[i];
}

__device__ __forceinline__ u4 pack8(const float (&f)[8])
{
    bf16x8 b;
#pragma unroll
    for (int i = 0; i < 8; ++i) b[i] = (bf16)f[i];
    return __builtin_bit_cast(u4, b);
}

__device__ __forceinline__ bf16x8 ld8(const bf16* p) { return __builtin_bit_cast(bf16x8, *(const u4*)p); }

// Raw buffer loads of 16 bytes: a descriptor in four scalar registers
// (wave-uniform base, stride 0, size in bytes, the gfx9 raw-buffer format
// word) plus a 32-bit per-lane offset and a wave-uniform offset, added by the
// memory unit instead of by 64-bit VALU arithmetic.
constexpr int kRawBufferWord3 = 0x00020000;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kRawBufferWord3);
}
__device__ __forceinline__ bf16x8 ldb8(__amdgpu_buffer_rsrc_t r, uint32_t lane_off, uint32_t uniform_off)
{
    return __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(r, lane_off, uniform_off, 0));
}

// ---------------------------------------------------------------------------
// forward convolution (and, with SIGN = -1, the data gradient)
//
// Workgroup = 4 waves = 64 consecutive voxels x (16 * NB) output channels;
// wave w owns voxels [16w, 16w + 16) and NB 16-channel output blocks.

// Epilogue of the convolution kernels.  SIGN = +1 (forward): v + bias, then
// the activation.  SIGN = -1 (data gradient) with ACT = LEAKY: the gradient is
// multiplied by the leaky-ReLU slope at the activation output `gate` (0.1
// where gate <= 0), i.e. it leaves as the producing layer's pre-activation
// gradient (the rule of k_act_bwd, applied before the BF16 rounding).
template <int SIGN, int ACT>
__device__ __forceinline__ float conv_out(float v, float bias, const bf16* __restrict__ gate, long long idx)
{
    if (SIGN > 0) {
        v += bias;
        if (ACT == CMNN_ACT_LEAKY) v = v > 0.f ? v : kLeak * v;
    } else if (ACT == CMNN_ACT_LEAKY) {
        if ((float)gate[idx] <= 0.f) v *= kLeak;
    }
    return v;
}

template <int NB, int SIGN, int ACT>
__global__ __launch_bounds__(256) void k_conv_fwd(G g, const bf16* __restrict__ x, int cin, const bf16* __restrict__ wt,
                                                  const float* __restrict__ bias, int cout, bf16* __restrict__ y,
                                                  const bf16* __restrict__ gate)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long m0 = (long long)blockIdx.x * 64 + wave * 16;
    const int co0 = blockIdx.y * 16 * NB;
    const long long mrow = m0 + (lane & 15);  // voxel of this lane's A row
    const int kq = lane >> 4;
    f4 acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = f4{0.f, 0.f, 0.f, 0.f};
    for (int t = 0; t < 27; ++t) {
        long long src = 0;
        const bool valid = mrow < g.nvox && neighbour(g, mrow, t, SIGN, src);
        const bf16* xp = x + src * cin + kq * 8;
        const bf16* wp = wt + ((long long)t * cout + co0 + (lane & 15)) * cin + kq * 8;
        for (int c0 = 0; c0 < cin; c0 += 32) {
            bf16x8 a;
            if (valid)
                a = ld8(xp + c0);
            else
                a = __builtin_bit_cast(bf16x8, u4{0u, 0u, 0u, 0u});
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const bf16x8 bw = ld8(wp + (long long)b * 16 * cin + c0);
                acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw, acc[b], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int co = co0 + 16 * b + (lane & 15);
        const float bb = bias ? bias[co] : 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const long long m = m0 + kq * 4 + i;
            if (m >= g.nvox) continue;
            y[m * cout + co] = (bf16)conv_out<SIGN, ACT>(acc[b][i], bb, gate, m * cout + co);
        }
    }
}

// ---------------------------------------------------------------------------
// brick-tiled forward convolution (and data gradient), for extents that are
// multiples of the 4 x 4 x 16 (d, h, w) brick
//
// Workgroup = one brick of 256 output voxels x (16 * NB) output channels.
// Per 32-channel input chunk the brick's 6 x 6 x 18 halo is staged once in LDS
// (voxel stride 80 bytes: 16 consecutive voxels of a 16-byte fragment read
// land on distinct bank groups), and every one of the 27 taps takes its A
// fragments from there: each input value is fetched from memory once per
// brick instead of once per tap, and each halo row is read from LDS once for
// its three x taps (the x - 1 and x + 1 fragments are lane shifts of it).  Wave w owns the 4 brick rows (d, h) =
// (w, 0..3), i.e. 4 MFMA row blocks of 16 x-consecutive voxels, and keeps
// 4 x NB accumulator tiles: each B fragment (weights, through L1) feeds 4
// MFMAs and each A fragment (LDS) feeds NB.  The weight fragments are raw
// buffer loads (a loop-invariant lane offset plus a wave-uniform tap offset,
// no per-load address arithmetic); a tap group's second and third taps are
// loaded before its LDS reads and the next group's first tap during its first
// tap's MFMAs, so the load latency overlaps work.

// The A operand of v_mfma_f32_16x16x32_bf16 holds voxel row (lane % 16), so
// the fragment of the neighbouring x tap is the same fragment shifted by one
// lane within each 16-lane DPP row; the lane left without a source keeps
// `edge` (update_dpp with bound_ctrl off leaves it unwritten).
// rows_from_lower: lane l takes lane l - 1 (voxel x - 1), lane 0 keeps edge.
// rows_from_upper: lane l takes lane l + 1 (voxel x + 1), lane 15 keeps edge.
__device__ __forceinline__ bf16x8 rows_from_lower(bf16x8 edge, bf16x8 v)
{
    const u4 e = __builtin_bit_cast(u4, edge), a = __builtin_bit_cast(u4, v);
    u4 r;
    r.x = (unsigned)__builtin_amdgcn_update_dpp((int)e.x, (int)a.x, 0x111, 0xF, 0xF, false);  // row_shr:1
    r.y = (unsigned)__builtin_amdgcn_update_dpp((int)e.y, (int)a.y, 0x111, 0xF, 0xF, false);
    r.z = (unsigned)__builtin_amdgcn_update_dpp((int)e.z, (int)a.z, 0x111, 0xF, 0xF, false);
    r.w = (unsigned)__builtin_amdgcn_update_dpp((int)e.w, (int)a.w, 0x111, 0xF, 0xF, false);
    return __builtin_bit_cast(bf16x8, r);
}

__device__ __forceinline__ bf16x8 rows_from_upper(bf16x8 edge, bf16x8 v)
{
    const u4 e = __builtin_bit_cast(u4, edge), a = __builtin_bit_cast(u4, v);
    u4 r;
    r.x = (unsigned)__builtin_amdgcn_update_dpp((int)e.x, (int)a.x, 0x101, 0xF, 0xF, false);  // row_shl:1
    r.y = (unsigned)__builtin_amdgcn_update_dpp((int)e.y, (int)a.y, 0x101, 0xF, 0xF, false);
    r.z = (unsigned)__builtin_amdgcn_update_dpp((int)e.z, (int)a.z, 0x101, 0xF, 0xF, false);
    r.w = (unsigned)__builtin_amdgcn_update_dpp((int)e.w, (int)a.w, 0x101, 0xF, 0xF, false);
    return __builtin_bit_cast(bf16x8, r);
}

constexpr int kTD = 4, kTH = 4, kTW = 16;
constexpr int kHD = kTD + 2, kHH = kTH + 2, kHW = kTW + 2;
constexpr int kHalo = kHD * kHH * kHW;  // 648 voxels
constexpr int kVStride = 40;            // bf16 per staged voxel (32 channels + 8 pad)
constexpr uint32_t kVBytes = kVStride * 2;

constexpr int kStageIters = (kHalo * 4 + 255) / 256;

__device__ __forceinline__ void stage_halo_load(const G& g, const bf16* __restrict__ x, int cin, int c0, long long n,
                                                int d0, int h0, int x0, int tid, u4 stage[kStageIters])
{
#pragma unroll
    for (int it = 0; it < kStageIters; ++it) {
        const int p = tid + it * 256;
        const int hv = p >> 2, part = p & 3;
        const int hx = hv % kHW, hh = (hv / kHW) % kHH, hd = hv / (kHW * kHH);
        int sd = 0, sh = 0, sw = 0;
        stage[it] = u4{0u, 0u, 0u, 0u};
        if (p < kHalo * 4 && shift_axis(d0, hd - 1, g.d, g.per[0], sd) && shift_axis(h0, hh - 1, g.h, g.per[1], sh) &&
            shift_axis(x0, hx - 1, g.w, g.per[2], sw))
            stage[it] = *(const u4*)(x + (((n * g.d + sd) * g.h + sh) * g.w + sw) * cin + c0 + part * 8);
    }
}

template <int NB, int SIGN, int ACT>
__global__ __launch_bounds__(256) void k_conv_tile(G g, const bf16* __restrict__ x, int cin,
                                                   const bf16* __restrict__ wt, const float* __restrict__ bias,
                                                   int cout, bf16* __restrict__ y, unsigned xcd_span,
                                                   const bf16* __restrict__ gate)
{
    __shared__ __attribute__((aligned(16))) bf16 sx[kHalo * kVStride];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // blocks are dealt round-robin to the 8 XCDs: give each XCD a contiguous
    // run of bricks so that halo overlaps and weights share its L2
    unsigned bid = blockIdx.x;
    if (xcd_span) bid = (bid & 7u) * xcd_span + (bid >> 3);
    const int nbw = g.w / kTW, nbh = g.h / kTH, nbd = g.d / kTD;
    int r = (int)bid;
    const int x0 = (r % nbw) * kTW;
    r /= nbw;
    const int h0 = (r % nbh) * kTH;
    r /= nbh;
    const int d0 = (r % nbd) * kTD;
    const long long n = r / nbd;
    const int co0 = blockIdx.y * 16 * NB;
    f4 acc[4][NB];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[m][b] = f4{0.f, 0.f, 0.f, 0.f};
    // weights: one descriptor over the [27][cout][cin] tensor, this lane's
    // row / channel part as a loop-invariant lane offset, the tap, output
    // block and channel chunk as a wave-uniform offset
    const __amdgpu_buffer_rsrc_t wr = buf_rsrc(wt, 27u * (uint32_t)cout * (uint32_t)cin * 2u);
    const uint32_t wlane = ((uint32_t)(co0 + (lane & 15)) * (uint32_t)cin + (uint32_t)(lane >> 4) * 8u) * 2u;
    // halo staging: thread tid moves the 16-byte parts tid, tid + 256, ... of
    // the 648 x 4; all its loads are in flight together
    u4 stage[kStageIters];
    // LDS fragment reads: lane part of the centre row (voxel x = lane % 16 + 1
    // of the halo row) and of its edge voxel, 16-byte channel group lane / 16
    const char* sxb = (const char*)sx;
    const uint32_t lane_a = ((uint32_t)(lane & 15) + 1u) * kVBytes + (uint32_t)(lane >> 4) * 16u;
    const uint32_t lane_e = ((lane & 15) < 8 ? 0u : (uint32_t)(kHW - 1) * kVBytes) + (uint32_t)(lane >> 4) * 16u;
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    for (int c0 = 0; c0 < cin; c0 += 32) {
        stage_halo_load(g, x, cin, c0, n, d0, h0, x0, tid, stage);
        __syncthreads();
#pragma unroll
        for (int it = 0; it < kStageIters; ++it) {
            const int p = tid + it * 256;
            if (p < kHalo * 4) *(u4*)&sx[(p >> 2) * kVStride + (p & 3) * 8] = stage[it];
        }
        __syncthreads();
        // weight fragments of tap t (NB output blocks); the first tap of the
        // next group is loaded one group ahead
        auto wload = [&](int t, bf16x8 bw[NB]) {
#pragma unroll
            for (int b = 0; b < NB; ++b)
                bw[b] = ldb8(wr, wlane, (((uint32_t)t * (uint32_t)cout + 16u * b) * (uint32_t)cin + (uint32_t)c0) * 2u);
        };
        bf16x8 bnext[NB];
        wload(0, bnext);
#pragma unroll 1
        for (int t9 = 0; t9 < 9; ++t9) {
            const int dz = SIGN * (t9 / 3 - 1), dy = SIGN * (t9 % 3 - 1);
            bf16x8 bw[3][NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) bw[0][b] = bnext[b];
            wload(t9 * 3 + 1, bw[1]);
            wload(t9 * 3 + 2, bw[2]);
            // A fragments of the three x taps (index dx + 1) of each brick row:
            // 32-bit LDS byte offsets, the tap's row wave-uniform, the brick row
            // m an immediate
            const uint32_t trow = (uint32_t)(((wv + 1 + dz) * kHH + 1 + dy) * kHW) * kVBytes;
            bf16x8 af[4][3];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const uint32_t mrow = trow + (uint32_t)(m * kHW) * kVBytes;
                const bf16x8 a0 = *(const bf16x8*)(sxb + lane_a + mrow);
                const bf16x8 e = *(const bf16x8*)(sxb + lane_e + mrow);
                af[m][0] = rows_from_lower(e, a0);
                af[m][1] = a0;
                af[m][2] = rows_from_upper(e, a0);
            }
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int k = SIGN > 0 ? j : 2 - j;  // dx = SIGN * (j - 1)
#pragma unroll
                for (int m = 0; m < 4; ++m)
#pragma unroll
                    for (int b = 0; b < NB; ++b)
                        acc[m][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[m][k], bw[j][b], acc[m][b], 0, 0, 0);
                if (j == 0 && t9 < 8) wload(t9 * 3 + 3, bnext);
            }
        }
    }
    // D[row][col]: row = voxel (lane / 16) * 4 + i of the block's x-row, col = output channel lane % 16.
    // The NB bias values are loaded together, before the stores (one wait instead of one per store group).
    float bbv[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) bbv[b] = bias ? bias[co0 + 16 * b + (lane & 15)] : 0.f;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const long long vrow = ((n * g.d + d0 + wave) * g.h + h0 + m) * g.w + x0;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int co = co0 + 16 * b + (lane & 15);
            const float bb = bbv[b];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const long long idx = (vrow + (lane >> 4) * 4 + i) * cout + co;
                y[idx] = (bf16)conv_out<SIGN, ACT>(acc[m][b][i], bb, gate, idx);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// weight gradient
//
// Workgroup (chunk, tap, co tile of 32, ci tile of 32) accumulates over the
// chunk's voxels in steps of 32: 128 threads stage dy[32 voxels][32 co] and
// 128 stage x[32 shifted voxels][32 ci] into LDS transposed ([channel][voxel],
// rows padded to 40 elements = 80 bytes, 16-byte aligned); wave w then
// computes the 16 x 16 block (co block w / 2, ci block w % 2).

constexpr int kLdsRow = 40;

__global__ __launch_bounds__(256) void k_conv_bwd_w(G g, const bf16* __restrict__ x, int cin,
                                                    const bf16* __restrict__ dy, int cout, long long chunk,
                                                    float* __restrict__ part)
{
    __shared__ __attribute__((aligned(16))) bf16 sdy[32 * kLdsRow];
    __shared__ __attribute__((aligned(16))) bf16 sx[32 * kLdsRow];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ct = cout / 32, it = cin / 32;
    int bid = blockIdx.x;
    const int cit = bid % it;
    bid /= it;
    const int cot = bid % ct;
    bid /= ct;
    const int t = bid % 27;
    const long long ch = bid / 27;
    const long long v0 = ch * chunk;
    const long long v1 = v0 + chunk < g.nvox ? v0 + chunk : g.nvox;
    // staging role: threads 0..127 load dy, 128..255 load x; each 16 bytes (8 channels) of one voxel
    const int st = tid & 127, sv = st >> 2, sc = (st & 3) * 8;
    f4 acc = f4{0.f, 0.f, 0.f, 0.f};
    const int cob = wave >> 1, cib = wave & 1;
    for (long long vb = v0; vb < v1; vb += 32) {
        const long long v = vb + sv;
        bf16x8 e = __builtin_bit_cast(bf16x8, u4{0u, 0u, 0u, 0u});
        if (tid < 128) {
            if (v < v1) e = ld8(dy + v * cout + cot * 32 + sc);
#pragma unroll
            for (int i = 0; i < 8; ++i) sdy[(sc + i) * kLdsRow + sv] = e[i];
        } else {
            long long s;
            if (v < v1 && neighbour(g, v, t, 1, s)) e = ld8(x + s * cin + cit * 32 + sc);
#pragma unroll
            for (int i = 0; i < 8; ++i) sx[(sc + i) * kLdsRow + sv] = e[i];
        }
        __syncthreads();
        const bf16x8 a = *(const bf16x8*)&sdy[(cob * 16 + (lane & 15)) * kLdsRow + (lane >> 4) * 8];
        const bf16x8 b = *(const bf16x8*)&sx[(cib * 16 + (lane & 15)) * kLdsRow + (lane >> 4) * 8];
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
        __syncthreads();
    }
    // D[co][ci]: row (lane/16)*4 + i, column lane % 16
    float* p = part + ((ch * 27 + t) * (long long)cout) * cin;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int co = cot * 32 + cob * 16 + (lane >> 4) * 4 + i;
        const int ci = cit * 32 + cib * 16 + (lane & 15);
        p[(long long)co * cin + ci] = acc[i];
    }
}

// ---------------------------------------------------------------------------
// brick-tiled weight gradient (extents multiples of the 4 x 4 x 16 brick)
//
// Workgroup (chunk of bricks, 32 output channels, 32 input channels), all 27
// taps, 8 waves.  The MFMA K axis is the voxel axis, so a fragment is 8
// consecutive voxels of one channel: per brick, dy ([co][256 voxels]) and the
// 6 x 6 x 18 halo of x ([ci][36 halo rows][24], positions x0 - 1 .. x0 + 16)
// are staged in LDS channel-major.  A staging task is an 8 x 8 (voxel x
// channel) block: eight 16-byte global loads, a register transpose, eight
// 16-byte LDS stores.  The next brick's loads are issued before the current
// brick's MFMAs so that their latency hides behind the compute.  A tap's x
// fragment starts dx + 1 elements into an aligned 16-byte LDS read: for
// dx = 0 and +1 the eight elements are realigned from that read and the next
// dword, and the three x taps of one (dz, dy) share that read.  Row strides
// are padded so that the 16 rows of a fragment read fall on distinct bank
// groups.  Two LDS buffers alternate: a wave stores brick br + 1 as soon as
// its MFMAs on brick br are done, so the stores of one wave overlap the MFMAs
// of another, with one barrier per brick.  The work units are the 18 pairs
// (tap group (dz, dy), 16-channel ci block); wave w takes units w, w + 8 and
// w + 16 and accumulates, for each, the three x taps times two 16-channel co
// blocks.  The dy fragments of a K step are read once and serve all of them.

constexpr int kDyStride = 256 + 8;        // bf16 per co row of staged dy
constexpr int kSkew = 8;                  // bf16 shift of each group of 8 channel rows (one 16-byte slot)
constexpr int kXRow = 24;                 // bf16 per staged halo row (18 used)
constexpr int kXStride = 36 * kXRow + 8;  // bf16 per ci row of staged x
constexpr int kXTasks = 36 * 3 * 4;       // (halo row, octet, channel group) blocks of x
constexpr int kDyTasks = 32 * 4;          // (x octet, channel group) blocks of dy
constexpr int kBwThreads = 512;

__device__ __forceinline__ void transpose8x8(const u4 (&in)[8], u4 (&out)[8])
{
    // in[i] holds channels 0..7 of voxel i (bf16 pairs per dword); out[c] holds voxels 0..7 of channel c
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int k = c >> 1, hi = c & 1;
        unsigned o[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const unsigned a = in[2 * j][k], b = in[2 * j + 1][k];
            // one byte permute: (a >> 16) | (b & 0xffff0000) or (a & 0xffff) | (b << 16)
            o[j] = __builtin_amdgcn_perm(b, a, hi ? 0x07060302u : 0x05040100u);
        }
        out[c] = u4{o[0], o[1], o[2], o[3]};
    }
}

__global__ __launch_bounds__(kBwThreads) void k_conv_bwd_w_tile(G g, const bf16* __restrict__ x, int cin,
                                                                const bf16* __restrict__ dy, int cout,
                                                                int bricks_per_chunk, float* __restrict__ part,
                                                                long long pstride, bool bias)
{
    __shared__ __attribute__((aligned(16))) bf16 sdy2[2][32 * kDyStride + 3 * kSkew];
    __shared__ __attribute__((aligned(16))) bf16 sx2[2][32 * kXStride + 3 * kSkew];
    __shared__ float sbias[kBwThreads];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ct = cout / 32, it = cin / 32;
    int bid = blockIdx.x;
    const int cit = bid % it;
    bid /= it;
    const int cot = bid % ct;
    const int ch = bid / ct;
    // bias gradient (column sums of dy) from the staged dy, by the ci-tile-0 workgroups:
    // thread (co = tid / 16, segment tid % 16) sums 16 voxels of each brick
    const bool do_bias = bias && cit == 0;
    float bsum = 0.f;
    const int nbw = g.w / kTW, nbh = g.h / kTH, nbd = g.d / kTD;
    const long long nbricks = (long long)g.n * nbd * nbh * nbw;
    const long long b0 = (long long)ch * bricks_per_chunk;
    const long long b1 = b0 + bricks_per_chunk < nbricks ? b0 + bricks_per_chunk : nbricks;
    // staging roles: x block tid (tid < 432), dy block tid - 384 (tid >= 384)
    const bool has_x = tid < kXTasks, has_dy = tid >= kBwThreads - kDyTasks;
    const int xcg = tid & 3, xoct = (tid >> 2) % 3, xhr = tid / 12;
    const int dyt = tid - (kBwThreads - kDyTasks), dcg = dyt & 3, drow = (dyt >> 2) >> 1, dxo = ((dyt >> 2) & 1) * 8;
    u4 xin[8], dyin[8];
    // coordinates of the next brick to load (bricks are loaded in order b0, b0 + 1, ...),
    // advanced brick by brick without divisions
    int lx0, lh0, ld0, ln;
    {
        int r = (int)b0;
        lx0 = (r % nbw) * kTW;
        r /= nbw;
        lh0 = (r % nbh) * kTH;
        r /= nbh;
        ld0 = (r % nbd) * kTD;
        ln = r / nbd;
    }
    const int xdz = xhr / 6 - 1, xdy = xhr % 6 - 1;         // this thread's halo row offsets
    const int xcoff = cit * 32 + xcg * 8, dyoff = cot * 32 + dcg * 8;
    auto load = [&]() {
        const int x0 = lx0, h0 = lh0, d0 = ld0, n = ln;
        lx0 += kTW;
        if (lx0 == g.w) {
            lx0 = 0;
            lh0 += kTH;
            if (lh0 == g.h) {
                lh0 = 0;
                ld0 += kTD;
                if (ld0 == g.d) {
                    ld0 = 0;
                    ++ln;
                }
            }
        }
        if (has_x) {
            int sd = 0, sh = 0;
            const bool rok = shift_axis(d0, xdz, g.d, g.per[0], sd) && shift_axis(h0, xdy, g.h, g.per[1], sh);
            // 32-bit element offsets from the tensor base (the host keeps x below 4 GiB)
            const uint32_t xrow = (uint32_t)(((n * g.d + sd) * g.h + sh) * g.w) * (uint32_t)cin + (uint32_t)xcoff;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int pos = xoct * 8 + i;  // halo position: x = x0 - 1 + pos
                int sw = 0;
                xin[i] = u4{0u, 0u, 0u, 0u};
                if (rok && pos < kTW + 2 && shift_axis(x0, pos - 1, g.w, g.per[2], sw))
                    xin[i] = *(const u4*)((const char*)x + 2u * (xrow + (uint32_t)sw * (uint32_t)cin));
            }
        }
        if (has_dy) {
            const int v = ((n * g.d + d0 + (drow >> 2)) * g.h + h0 + (drow & 3)) * g.w + x0 + dxo;
            const uint32_t src = (uint32_t)v * (uint32_t)cout + (uint32_t)dyoff;
#pragma unroll
            for (int i = 0; i < 8; ++i) dyin[i] = *(const u4*)((const char*)dy + 2u * (src + (uint32_t)(i * cout)));
        }
    };
    auto store = [&](int buf) {
        bf16* sdy = sdy2[buf];
        bf16* sx = sx2[buf];
        u4 out[8];
        if (has_x) {
            transpose8x8(xin, out);
#pragma unroll
            for (int c = 0; c < 8; ++c) *(u4*)&sx[(xcg * 8 + c) * kXStride + xcg * kSkew + xhr * kXRow + xoct * 8] = out[c];
        }
        if (has_dy) {
            transpose8x8(dyin, out);
#pragma unroll
            for (int c = 0; c < 8; ++c) *(u4*)&sdy[(dcg * 8 + c) * kDyStride + dcg * kSkew + drow * 16 + dxo] = out[c];
        }
    };
    // work units: (tap group g = (dz, dy), ci block ib), 18 of them; wave w
    // takes units w, w + 8, w + 16.  The three x taps of a group share one
    // 20-byte B read per lane (their K windows are byte shifts of it).
    f4 acc[3][3][2];  // [unit of this wave][x tap][co block]
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[k][a][b] = f4{0.f, 0.f, 0.f, 0.f};
    const int j = lane >> 4, l16 = lane & 15;
    // two LDS buffers: brick br + 1 is stored while brick br's MFMAs run in
    // other waves; one barrier per brick
    if (b0 < b1) {
        load();
        store(0);
        if (b0 + 1 < b1) load();
    }
    __syncthreads();
    int cur = 0;
    for (long long br = b0; br < b1; ++br) {
        const bf16* sdy = sdy2[cur];
        const bf16* sx = sx2[cur];
        if (do_bias) {
            const bf16* q = &sdy[(tid >> 4) * kDyStride + (tid >> 7) * kSkew + (tid & 15) * 16];
#pragma unroll
            for (int k = 0; k < 16; ++k) bsum += (float)q[k];
        }
        // 8 K steps of 32 voxels (two brick rows); lane group j takes voxels 8j..8j+7
#pragma unroll 8
        for (int ks = 0; ks < 8; ++ks) {
            const int row = ks * 2 + (j >> 1), xo = (j & 1) * 8;
            bf16x8 a[2];
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
                a[cb] = *(const bf16x8*)&sdy[(cb * 16 + l16) * kDyStride + (cb * 2 + (l16 >> 3)) * kSkew + row * 16 + xo];
            const int dd = row >> 2, hh = row & 3;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int u = wave + 8 * k;
                if (u < 18) {
                    const int g = u >> 1, ib = u & 1;
                    const int dz = g / 3 - 1, dyy = g % 3 - 1;
                    const int hr = (dd + 1 + dz) * 6 + hh + 1 + dyy;
                    const bf16* q = &sx[(ib * 16 + l16) * kXStride + (ib * 2 + (l16 >> 3)) * kSkew + hr * kXRow + xo];
                    u4 lo = *(const u4*)q;
                    unsigned hi = *(const unsigned*)(q + 8);
                    // opaque to the optimiser: the third tap's window is then built from
                    // these registers instead of being re-read from LDS as an unaligned load
                    asm("" : "+v"(lo), "+v"(hi));
                    // x taps cx = 0, 1, 2 start 0, 1, 2 elements into the read
                    const u4 f[3] = {lo,
                                     u4{__builtin_amdgcn_alignbyte(lo[1], lo[0], 2), __builtin_amdgcn_alignbyte(lo[2], lo[1], 2),
                                        __builtin_amdgcn_alignbyte(lo[3], lo[2], 2), __builtin_amdgcn_alignbyte(hi, lo[3], 2)},
                                     u4{lo[1], lo[2], lo[3], hi}};
#pragma unroll
                    for (int cx = 0; cx < 3; ++cx) {
                        const bf16x8 b = __builtin_bit_cast(bf16x8, f[cx]);
#pragma unroll
                        for (int cb = 0; cb < 2; ++cb)
                            acc[k][cx][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[cb], b, acc[k][cx][cb], 0, 0, 0);
                    }
                }
            }
        }
        if (br + 1 < b1) {
            store(cur ^ 1);
            if (br + 2 < b1) load();
        }
        __syncthreads();
        cur ^= 1;
    }
    if (do_bias) {
        sbias[tid] = bsum;
        __syncthreads();
        if (tid < 32) {
            float b = 0.f;
#pragma unroll
            for (int k = 0; k < 16; ++k) b += sbias[tid * 16 + k];
            part[(long long)ch * pstride + 27LL * cin * cout + cot * 32 + tid] = b;
        }
    }
    // D[co][ci]: row (lane / 16) * 4 + i, column lane % 16
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int u = wave + 8 * k;
        if (u >= 18) continue;
        const int g = u >> 1, ib = u & 1;
#pragma unroll
        for (int cx = 0; cx < 3; ++cx) {
            const int t = g * 3 + cx;
            float* p = part + (long long)ch * pstride + ((long long)t * cout) * cin;
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int co = cot * 32 + cb * 16 + (lane >> 4) * 4 + i;
                    const int ci = cit * 32 + ib * 16 + (lane & 15);
                    p[(long long)co * cin + ci] = acc[k][cx][cb][i];
                }
        }
    }
}

// Element e of the chunk sums, e < n0 + n1: out0[e] (e < n0) or out1[e - n0]
// = sum over chunks c of part[c * pstride + e], in a fixed order: wave s of a
// workgroup of W waves sums chunks s, s + W, s + 2 W, ... for 64 consecutive
// elements, then the wave sums are added in wave order.  The sum is bound by
// the latency of its loads: 16 waves pay off from about 128 chunks.
template <int W>
__global__ __launch_bounds__(64 * W) void k_sum_chunks(const float* __restrict__ part, long long pstride, long long n0,
                                                       long long n1, int nchunk, float* __restrict__ out0,
                                                       float* __restrict__ out1)
{
    __shared__ float sh[W][64];
    const int e = threadIdx.x & 63, sl = threadIdx.x >> 6;
    const long long i = (long long)blockIdx.x * 64 + e;
    const long long n = n0 + n1;
    float acc = 0.f;
    if (i < n)
        for (int c = sl; c < nchunk; c += W) acc += part[(long long)c * pstride + i];
    sh[sl][e] = acc;
    __syncthreads();
    if (sl == 0 && i < n) {
        float v = sh[0][e];
        for (int k = 1; k < W; ++k) v += sh[k][e];
        if (i < n0)
            out0[i] = v;
        else
            out1[i - n0] = v;
    }
}

// Per-chunk column sums of a [rows][cols] BF16 matrix (cols <= 256): thread t
// sums column t % cols over every (256 / cols)-th row of the block's chunk,
// then the row groups are added in LDS in a fixed order.
constexpr int kColSumBlocks = 1024;

__global__ __launch_bounds__(256) void k_colsum_part(const bf16* __restrict__ a, long long rows, int cols,
                                                     long long chunk, float* __restrict__ part)
{
    __shared__ float sh[256];
    const int t = threadIdx.x;
    const int rpi = 256 / cols;
    const int c = t % cols, roff = t / cols;
    const long long r0 = (long long)blockIdx.x * chunk;
    const long long r1 = r0 + chunk < rows ? r0 + chunk : rows;
    float s = 0.f;
    if (roff < rpi)
        for (long long r = r0 + roff; r < r1; r += rpi) s += (float)a[r * cols + c];
    sh[t] = s;
    __syncthreads();
    if (t < cols) {
        float q = 0.f;
        for (int k = 0; k < rpi; ++k) q += sh[k * cols + t];
        part[(long long)blockIdx.x * cols + t] = q;
    }
}

// ---------------------------------------------------------------------------
// elementwise

__global__ void k_act_bwd(const bf16* __restrict__ y, const bf16* __restrict__ dy, bf16* __restrict__ dp, long long n,
                          int act)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        float d = (float)dy[i];
        if (act == CMNN_ACT_LEAKY && (float)y[i] <= 0.f) d *= kLeak;
        dp[i] = (bf16)d;
    }
}

__global__ void k_pool2_fwd(G g, const bf16* __restrict__ x, int c, bf16* __restrict__ y)
{
    const int d2 = g.d / 2, h2 = g.h / 2, w2 = g.w / 2;
    const long long total = (long long)g.n * d2 * h2 * w2 * c;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const int ch = (int)(i % c);
        long long r = i / c;
        const int w = (int)(r % w2);
        r /= w2;
        const int h = (int)(r % h2);
        r /= h2;
        const int d = (int)(r % d2);
        const long long n = r / d2;
        float s = 0.f;
        for (int k = 0; k < 8; ++k) {
            const long long v = ((n * g.d + 2 * d + (k >> 2)) * g.h + 2 * h + ((k >> 1) & 1)) * g.w + 2 * w + (k & 1);
            s += (float)x[v * c + ch];
        }
        y[i] = (bf16)(0.125f * s);
    }
}

__global__ void k_pool2_bwd(G g, const bf16* __restrict__ dy, int c, bf16* __restrict__ dx)
{
    const long long total = g.nvox * c;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const int ch = (int)(i % c);
        long long r = i / c;
        const int w = (int)(r % g.w);
        r /= g.w;
        const int h = (int)(r % g.h);
        r /= g.h;
        const int d = (int)(r % g.d);
        const long long n = r / g.d;
        const long long v = ((n * (g.d / 2) + d / 2) * (g.h / 2) + h / 2) * (g.w / 2) + w / 2;
        dx[i] = (bf16)(0.125f * (float)dy[v * c + ch]);
    }
}

// coarse geometry g; fine voxel (2d + a, 2h + b, 2w + e) copies coarse (d, h, w)
__global__ void k_up2_fwd(G g, const bf16* __restrict__ x, int c, bf16* __restrict__ y)
{
    const int D = 2 * g.d, H = 2 * g.h, W = 2 * g.w;
    const long long total = (long long)g.n * D * H * W * c;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const int ch = (int)(i % c);
        long long r = i / c;
        const int w = (int)(r % W);
        r /= W;
        const int h = (int)(r % H);
        r /= H;
        const int d = (int)(r % D);
        const long long n = r / D;
        const long long v = ((n * g.d + d / 2) * g.h + h / 2) * g.w + w / 2;
        y[i] = x[v * c + ch];
    }
}

__global__ void k_up2_bwd(G g, const bf16* __restrict__ dy, int c, bf16* __restrict__ dx)
{
    const int H = 2 * g.h, W = 2 * g.w;
    const long long total = g.nvox * c;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const int ch = (int)(i % c);
        long long r = i / c;
        const int w = (int)(r % g.w);
        r /= g.w;
        const int h = (int)(r % g.h);
        r /= g.h;
        const int d = (int)(r % g.d);
        const long long n = r / g.d;
        float s = 0.f;
        for (int k = 0; k < 8; ++k) {
            const long long v = ((n * (2 * g.d) + 2 * d + (k >> 2)) * H + 2 * h + ((k >> 1) & 1)) * W + 2 * w + (k & 1);
            s += (float)dy[v * c + ch];
        }
        dx[i] = (bf16)s;
    }
}

__global__ void k_concat_fwd(long long nvox, const bf16* __restrict__ a, int ca, const bf16* __restrict__ b, int cb,
                             bf16* __restrict__ y)
{
    const int c = ca + cb;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nvox * c;
         i += (long long)gridDim.x * blockDim.x) {
        const long long v = i / c;
        const int ch = (int)(i % c);
        y[i] = ch < ca ? a[v * ca + ch] : b[v * cb + ch - ca];
    }
}

__global__ void k_concat_bwd(long long nvox, const bf16* __restrict__ dy, int ca, int cb, bf16* __restrict__ da,
                             bf16* __restrict__ db)
{
    const int c = ca + cb;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nvox * c;
         i += (long long)gridDim.x * blockDim.x) {
        const long long v = i / c;
        const int ch = (int)(i % c);
        if (ch < ca) {
            if (da) da[v * ca + ch] = dy[i];
        } else if (db) {
            db[v * cb + ch - ca] = dy[i];
        }
    }
}

__global__ void k_add(long long n, const bf16* __restrict__ a, const bf16* __restrict__ b, bf16* __restrict__ y)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        y[i] = (bf16)((float)a[i] + (float)b[i]);
}

// 16-byte variants of the elementwise kernels (8 channels per thread), used when
// the channel counts are multiples of 8 and the pointers 16-byte aligned

__global__ void k_act_bwd8(const u4* __restrict__ y, const u4* __restrict__ dy, u4* __restrict__ dp, long long n8, int act)
{
    GRID_STRIDE(i, n8)
    {
        float fy[8], fd[8];
        unpack8(y[i], fy);
        unpack8(dy[i], fd);
        if (act == CMNN_ACT_LEAKY)
#pragma unroll
            for (int k = 0; k < 8; ++k) fd[k] = fy[k] <= 0.f ? kLeak * fd[k] : fd[k];
        dp[i] = pack8(fd);
    }
}

template <typename I>
__global__ void k_pool2_fwd8(G g, const bf16* __restrict__ x, int c, bf16* __restrict__ y)
{
    const I d2 = g.d / 2, h2 = g.h / 2, w2 = g.w / 2, q8 = c / 8;
    GRID_STRIDE_I(I, i, (long long)g.n * d2 * h2 * w2 * q8)
    {
        const I q = i % q8;
        I r = i / q8;
        const I w = r % w2;
        r /= w2;
        const I h = r % h2;
        r /= h2;
        const I d = r % d2;
        const I n = r / d2;
        float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, f[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const I v = ((n * g.d + 2 * d + (k >> 2)) * g.h + 2 * h + ((k >> 1) & 1)) * g.w + 2 * w + (k & 1);
            unpack8(*(const u4*)(x + v * c + 8 * q), f);
#pragma unroll
            for (int e = 0; e < 8; ++e) s[e] += f[e];
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) s[e] *= 0.125f;
        *(u4*)(y + i * 8) = pack8(s);
    }
}

__global__ void k_pool2_bwd8(G g, const bf16* __restrict__ dy, int c, bf16* __restrict__ dx)
{
    const int q8 = c / 8;
    GRID_STRIDE(i, g.nvox * q8)
    {
        const int q = (int)(i % q8);
        long long r = i / q8;
        const int w = (int)(r % g.w);
        r /= g.w;
        const int h = (int)(r % g.h);
        r /= g.h;
        const int d = (int)(r % g.d);
        const long long n = r / g.d;
        const long long v = ((n * (g.d / 2) + d / 2) * (g.h / 2) + h / 2) * (g.w / 2) + w / 2;
        float f[8];
        unpack8(*(const u4*)(dy + v * c + 8 * q), f);
#pragma unroll
        for (int e = 0; e < 8; ++e) f[e] *= 0.125f;
        *(u4*)(dx + i * 8) = pack8(f);
    }
}

__global__ void k_up2_fwd8(G g, const bf16* __restrict__ x, int c, bf16* __restrict__ y)
{
    const int D = 2 * g.d, H = 2 * g.h, W = 2 * g.w, q8 = c / 8;
    GRID_STRIDE(i, (long long)g.n * D * H * W * q8)
    {
        const int q = (int)(i % q8);
        long long r = i / q8;
        const int w = (int)(r % W);
        r /= W;
        const int h = (int)(r % H);
        r /= H;
        const int d = (int)(r % D);
        const long long n = r / D;
        const long long v = ((n * g.d + d / 2) * g.h + h / 2) * g.w + w / 2;
        *(u4*)(y + i * 8) = *(const u4*)(x + v * c + 8 * q);
    }
}

__global__ void k_up2_bwd8(G g, const bf16* __restrict__ dy, int c, bf16* __restrict__ dx)
{
    const int H = 2 * g.h, W = 2 * g.w, q8 = c / 8;
    GRID_STRIDE(i, g.nvox * q8)
    {
        const int q = (int)(i % q8);
        long long r = i / q8;
        const int w = (int)(r % g.w);
        r /= g.w;
        const int h = (int)(r % g.h);
        r /= g.h;
        const int d = (int)(r % g.d);
        const long long n = r / g.d;
        float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, f[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const long long v = ((n * (2 * g.d) + 2 * d + (k >> 2)) * H + 2 * h + ((k >> 1) & 1)) * W + 2 * w + (k & 1);
            unpack8(*(const u4*)(dy + v * c + 8 * q), f);
#pragma unroll
            for (int e = 0; e < 8; ++e) s[e] += f[e];
        }
        *(u4*)(dx + i * 8) = pack8(s);
    }
}

__global__ void k_concat_fwd8(long long nvox, const bf16* __restrict__ a, int ca, const bf16* __restrict__ b, int cb,
                              bf16* __restrict__ y)
{
    const int qa = ca / 8, q8 = (ca + cb) / 8;
    GRID_STRIDE(i, nvox * q8)
    {
        const long long v = i / q8;
        const int q = (int)(i % q8);
        *(u4*)(y + i * 8) = q < qa ? *(const u4*)(a + v * ca + 8 * q) : *(const u4*)(b + v * cb + 8 * (q - qa));
    }
}

__global__ void k_concat_bwd8(long long nvox, const bf16* __restrict__ dy, int ca, int cb, bf16* __restrict__ da,
                              bf16* __restrict__ db)
{
    const int qa = ca / 8, q8 = (ca + cb) / 8;
    GRID_STRIDE(i, nvox * q8)
    {
        const long long v = i / q8;
        const int q = (int)(i % q8);
        const u4 e = *(const u4*)(dy + i * 8);
        if (q < qa) {
            if (da) *(u4*)(da + v * ca + 8 * q) = e;
        } else if (db) {
            *(u4*)(db + v * cb + 8 * (q - qa)) = e;
        }
    }
}

__global__ void k_add8(long long n8, const u4* __restrict__ a, const u4* __restrict__ b, u4* __restrict__ y)
{
    GRID_STRIDE(i, n8)
    {
        float fa[8], fb[8];
        unpack8(a[i], fa);
        unpack8(b[i], fb);
#pragma unroll
        for (int e = 0; e < 8; ++e) fa[e] += fb[e];
        y[i] = pack8(fa);
    }
}

// Skip-connection joins of the U-Net: one pass over the fine level each, in
// place of the separate upsampling or pooling, concatenation, sum and
// activation-gradient passes.  Channel counts are multiples of 32 and channel
// strides multiples of 8, so every thread moves 8 channels (16 bytes).

// y = [skip | up2(x)] at the fine level; g is the coarse geometry of x.
template <typename I>
__global__ void k_up2_concat_fwd8(G g, const bf16* __restrict__ skip, int cs, const bf16* __restrict__ x, int cx,
                                  bf16* __restrict__ y)
{
    const I D = 2 * g.d, H = 2 * g.h, W = 2 * g.w, qs = cs / 8, q8 = (cs + cx) / 8;
    GRID_STRIDE_I(I, i, 8 * g.nvox * q8)
    {
        const I q = i % q8;
        const I v = i / q8;
        u4 e;
        if (q < qs) {
            e = *(const u4*)(skip + v * cs + 8 * q);
        } else {
            const I w = v % W;
            I r = v / W;
            const I h = r % H;
            r /= H;
            const I d = r % D;
            const I n = r / D;
            const I p = ((n * g.d + d / 2) * g.h + h / 2) * g.w + w / 2;
            e = *(const u4*)(x + p * cx + 8 * (q - qs));
        }
        *(u4*)(y + i * 8) = e;
    }
}

// Leaky-ReLU slope at the activation output, applied to an FP32 gradient.
__device__ __forceinline__ void act_grad8(const bf16* __restrict__ gate, int act, float (&f)[8])
{
    if (act != CMNN_ACT_LEAKY) return;
    float t[8];
    unpack8(*(const u4*)gate, t);
#pragma unroll
    for (int e = 0; e < 8; ++e) f[e] = t[e] <= 0.f ? kLeak * f[e] : f[e];
}

// dx = act'(gate) * (up2 gradient of dy): dy is the upsampled part of a
// concatenation's gradient (channel stride ldy), g the coarse geometry.
template <typename I>
__global__ void k_up2_bwd_act8(G g, const bf16* __restrict__ dy, int ldy, int c, const bf16* __restrict__ gate,
                               int act, bf16* __restrict__ dx)
{
    const I H = 2 * g.h, W = 2 * g.w, q8 = c / 8;
    GRID_STRIDE_I(I, i, g.nvox * q8)
    {
        const I q = i % q8;
        I r = i / q8;
        const I w = r % g.w;
        r /= g.w;
        const I h = r % g.h;
        r /= g.h;
        const I d = r % g.d;
        const I n = r / g.d;
        float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, f[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const I v = ((n * (2 * g.d) + 2 * d + (k >> 2)) * H + 2 * h + ((k >> 1) & 1)) * W + 2 * w + (k & 1);
            unpack8(*(const u4*)(dy + v * ldy + 8 * q), f);
#pragma unroll
            for (int e = 0; e < 8; ++e) s[e] += f[e];
        }
        act_grad8(gate + i * 8, act, s);
        *(u4*)(dx + i * 8) = pack8(s);
    }
}

// dx = act'(gate) * (pool2 gradient of dy + skip): g is the fine geometry, dy
// coarse, skip the skip part of a concatenation's gradient (channel stride
// ldskip) or NULL.
template <typename I>
__global__ void k_pool2_bwd_add_act8(G g, const bf16* __restrict__ dy, int c, const bf16* __restrict__ skip,
                                     int ldskip, const bf16* __restrict__ gate, int act, bf16* __restrict__ dx)
{
    const I q8 = c / 8;
    GRID_STRIDE_I(I, i, g.nvox * q8)
    {
        const I q = i % q8;
        const I v = i / q8;
        const I w = v % g.w;
        I r = v / g.w;
        const I h = r % g.h;
        r /= g.h;
        const I d = r % g.d;
        const I n = r / g.d;
        const I p = ((n * (g.d / 2) + d / 2) * (g.h / 2) + h / 2) * (g.w / 2) + w / 2;
        float f[8], t[8];
        unpack8(*(const u4*)(dy + p * c + 8 * q), f);
#pragma unroll
        for (int e = 0; e < 8; ++e) f[e] *= 0.125f;
        if (skip) {
            unpack8(*(const u4*)(skip + v * ldskip + 8 * q), t);
#pragma unroll
            for (int e = 0; e < 8; ++e) f[e] += t[e];
        }
        act_grad8(gate + i * 8, act, f);
        *(u4*)(dx + i * 8) = pack8(f);
    }
}

// masked MSE: per-block partial (sum wt * sq, sum wt), then a single-block final
constexpr int kMseBlocks = 1024;

__global__ __launch_bounds__(256) void k_mse_part(long long nvox, const bf16* __restrict__ pred, int c, int creal,
                                                  const float* __restrict__ tgt, const float* __restrict__ wt,
                                                  float* __restrict__ part)
{
    __shared__ float s0[256], s1[256];
    float a = 0.f, b = 0.f;
    for (long long v = (long long)blockIdx.x * 256 + threadIdx.x; v < nvox; v += (long long)gridDim.x * 256) {
        const float w = wt[v];
        float q = 0.f;
        for (int k = 0; k < creal; ++k) {
            const float d = (float)pred[v * c + k] - tgt[(long long)k * nvox + v];
            q += d * d;
        }
        a += w * q;
        b += w;
    }
    s0[threadIdx.x] = a;
    s1[threadIdx.x] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            s0[threadIdx.x] += s0[threadIdx.x + s];
            s1[threadIdx.x] += s1[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s0[0];
        part[2 * blockIdx.x + 1] = s1[0];
    }
}

// One workgroup of 256: thread t adds partials t, t + 256, ... in order, then
// the 256 sums are added pairwise in LDS (a fixed order: deterministic).
__global__ __launch_bounds__(256) void k_mse_final(const float* __restrict__ part, int nb, int creal,
                                                   float* __restrict__ out)
{
    __shared__ float sa[256], sb[256];
    const int t = threadIdx.x;
    float a = 0.f, b = 0.f;
    for (int i = t; i < nb; i += 256) {
        a += part[2 * i];
        b += part[2 * i + 1];
    }
    sa[t] = a;
    sb[t] = b;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) {
            sa[t] += sa[t + h];
            sb[t] += sb[t + h];
        }
        __syncthreads();
    }
    if (t == 0) {
        out[0] = sb[0] > 0.f ? sa[0] / (sb[0] * creal) : 0.f;  // loss
        out[1] = sb[0] * creal;                                 // normaliser, read by k_mse_grad
    }
}

__global__ void k_mse_grad(long long nvox, const bf16* __restrict__ pred, int c, int creal,
                           const float* __restrict__ tgt, const float* __restrict__ wt,
                           const float* __restrict__ norm, bf16* __restrict__ dpred)
{
    const float scale = norm[1] > 0.f ? 2.f / norm[1] : 0.f;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nvox * c;
         i += (long long)gridDim.x * blockDim.x) {
        const long long v = i / c;
        const int k = (int)(i % c);
        float d = 0.f;
        if (k < creal) d = scale * wt[v] * ((float)pred[i] - tgt[(long long)k * nvox + v]);
        dpred[i] = (bf16)d;
    }
}

// 8 channels per thread: channels below creal get the gradient, the padded
// ones zeros (their prediction is not read)
template <typename I>
__global__ void k_mse_grad8(long long nvox, const bf16* __restrict__ pred, int c, int creal,
                            const float* __restrict__ tgt, const float* __restrict__ wt,
                            const float* __restrict__ norm, bf16* __restrict__ dpred)
{
    const float scale = norm[1] > 0.f ? 2.f / norm[1] : 0.f;
    const I q8 = c / 8, nv = (I)nvox;
    GRID_STRIDE_I(I, i, nvox * q8)
    {
        const I q = i % q8;
        const I v = i / q8;
        float f[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if ((int)(8 * q) < creal) {
            float p[8];
            unpack8(*(const u4*)(pred + i * 8), p);
            const float sw = scale * wt[v];
#pragma unroll
            for (int e = 0; e < 8; ++e)
                if ((int)(8 * q) + e < creal) f[e] = sw * (p[e] - tgt[(8 * q + e) * nv + v]);
        }
        *(u4*)(dpred + i * 8) = pack8(f);
    }
}

__global__ void k_adam(long long n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float wd, float c1, float c2)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float mh = mi / c1, vh = vi / c2;
        p[i] -= lr * (mh / (sqrtf(vh) + eps) + wd * p[i]);
    }
}

// Global gradient-norm clipping: per-block partial sums of g^2, one workgroup
// that sums them and forms the norm and the scale min(1, max_norm / norm) (0 for a
// non-finite norm, which turns the update into a no-gradient step), then an
// in-place scale read from device memory (no host round trip).
constexpr int kClipBlocks = 512;

__global__ __launch_bounds__(256) void k_sumsq_part(long long n, const float* __restrict__ g, float* __restrict__ part)
{
    __shared__ float sh[256];
    float a = 0.f;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        const float x = g[i];
        a += x * x;
    }
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// One workgroup of 256, FP64 sums in a fixed order (as k_mse_final).
__global__ __launch_bounds__(256) void k_clip_final(const float* __restrict__ part, int nb, float max_norm,
                                                    float* __restrict__ out)
{
    __shared__ double sh[256];
    const int t = threadIdx.x;
    double a = 0.0;
    for (int i = t; i < nb; i += 256) a += part[i];
    sh[t] = a;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) sh[t] += sh[t + h];
        __syncthreads();
    }
    if (t != 0) return;
    const float norm = (float)sqrt(sh[0]);
    float scale = 1.f;
    if (!(norm < INFINITY)) scale = 0.f;
    else if (max_norm > 0.f && norm > max_norm) scale = max_norm / norm;
    out[0] = norm;
    out[1] = scale;
}

__global__ void k_scale(long long n, float* __restrict__ g, const float* __restrict__ sc)
{
    const float a = sc[1];
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        g[i] = a == 0.f ? 0.f : g[i] * a;
}

__global__ void k_pack_w(const float* __restrict__ w, int cin, int cout, bf16* __restrict__ wf, bf16* __restrict__ wtr)
{
    const long long total = 27LL * cin * cout;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const int ci = (int)(i % cin);
        long long r = i / cin;
        const int co = (int)(r % cout);
        const int t = (int)(r / cout);
        const bf16 b = (bf16)w[i];
        wf[i] = b;
        wtr[((long long)t * cin + ci) * cout + co] = b;
    }
}

// Several layers' packing in one launch: each workgroup belongs to one layer
// (first_block ranges), so the layer's parameters are wave-uniform.
struct PackJobs {
    const float* w[CMNN_PACK_MAX];
    bf16* wf[CMNN_PACK_MAX];
    bf16* wt[CMNN_PACK_MAX];
    int cin[CMNN_PACK_MAX], cout[CMNN_PACK_MAX];
    int first_block[CMNN_PACK_MAX + 1];
    int n;
};

__global__ __launch_bounds__(256) void k_pack_w_batch(const PackJobs J)
{
    int l = 0;
    while (l + 1 < J.n && (int)blockIdx.x >= J.first_block[l + 1]) ++l;
    const int cin = J.cin[l], cout = J.cout[l];
    const long long i = (long long)((int)blockIdx.x - J.first_block[l]) * 256 + threadIdx.x;
    if (i >= 27LL * cin * cout) return;
    const int ci = (int)(i % cin);
    const long long r = i / cin;
    const int co = (int)(r % cout), t = (int)(r / cout);
    const bf16 b = (bf16)J.w[l][i];
    J.wf[l][i] = b;
    J.wt[l][((long long)t * cin + ci) * cout + co] = b;
}

__global__ void k_pack_ch(long long nvox, const float* __restrict__ src, int cs, bf16* __restrict__ dst, int c)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nvox * c;
         i += (long long)gridDim.x * blockDim.x) {
        const long long v = i / c;
        const int k = (int)(i % c);
        dst[i] = k < cs ? (bf16)src[(long long)k * nvox + v] : (bf16)0.f;
    }
}

// Minibatch gathers from sample-major planes src [np][nsrc][nvs]: output
// sample b is source sample idx[b] (b itself when idx is NULL); an index
// outside [0, nsrc) gives zeros.
__device__ __forceinline__ long long pick(const int* __restrict__ idx, long long b, int nsrc)
{
    const long long s = idx ? (long long)idx[b] : b;
    return s >= 0 && s < nsrc ? s : -1;
}

// BF16 NDHWC [nsel * nvs][c] (channels from cs on zero), 8 channels per thread
template <typename I>
__global__ void k_gather_pack8(int nsel, const int* __restrict__ idx, long long nvs, const float* __restrict__ src,
                               int nsrc, int cs, bf16* __restrict__ dst, int c)
{
    const I q8 = c / 8, nv = (I)nvs;
    GRID_STRIDE_I(I, i, (long long)nsel * nvs * q8)
    {
        const I q = i % q8;
        const I r = i / q8, v = r % nv;
        const long long s = pick(idx, (long long)(r / nv), nsrc);
        float f[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (s >= 0 && (int)(8 * q) < cs)
#pragma unroll
            for (int e = 0; e < 8; ++e)
                if ((int)(8 * q) + e < cs) f[e] = src[((8 * q + e) * (I)nsrc + (I)s) * nv + v];
        *(u4*)(dst + i * 8) = pack8(f);
    }
}

// FP32 [np][nsel][nvs], 4 values per thread (nvs a multiple of 4)
__global__ void k_gather4(int nsel, const int* __restrict__ idx, long long nvs4, const float4* __restrict__ src,
                          int nsrc, int np, float4* __restrict__ dst)
{
    GRID_STRIDE(i, (long long)np * nsel * nvs4)
    {
        const long long v = i % nvs4, r = i / nvs4, b = r % nsel, p = r / nsel, s = pick(idx, b, nsrc);
        dst[i] = s >= 0 ? src[(p * nsrc + s) * nvs4 + v] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

__global__ void k_gather1(int nsel, const int* __restrict__ idx, long long nvs, const float* __restrict__ src,
                          int nsrc, int np, float* __restrict__ dst)
{
    GRID_STRIDE(i, (long long)np * nsel * nvs)
    {
        const long long v = i % nvs, r = i / nvs, b = r % nsel, p = r / nsel, s = pick(idx, b, nsrc);
        dst[i] = s >= 0 ? src[(p * nsrc + s) * nvs + v] : 0.f;
    }
}

__global__ void k_unpack_ch(long long nvox, const bf16* __restrict__ src, int c, float* __restrict__ dst, int cs)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nvox * cs;
         i += (long long)gridDim.x * blockDim.x) {
        const int k = (int)(i / nvox);
        const long long v = i % nvox;
        dst[i] = (float)src[v * c + k];
    }
}

// Per-sample channel means broadcast back over the voxels:
// y[n][v][c] = (1/V) sum_v' x[n][v'][c].  The operator is a symmetric
// projection, so the same two kernels also give its gradient.
__global__ __launch_bounds__(256) void k_chmean_part(const bf16* __restrict__ x, int ldx, long long vps, int c,
                                                     int parts, float* __restrict__ part)
{
    // block (n, p): voxels [p * chunk, (p + 1) * chunk) of sample n; thread t sums channel t % c
    // (voxel rows ldx channels apart)
    __shared__ float sh[256];
    const int n = blockIdx.x / parts, p = blockIdx.x % parts;
    const long long chunk = (vps + parts - 1) / parts;
    const long long v0 = p * chunk, v1 = v0 + chunk < vps ? v0 + chunk : vps;
    const int t = threadIdx.x, rpi = 256 / c, ch = t % c, roff = t / c;
    float s = 0.f;
    if (roff < rpi)
        for (long long v = v0 + roff; v < v1; v += rpi) s += (float)x[((long long)n * vps + v) * ldx + ch];
    sh[t] = s;
    __syncthreads();
    if (t < c) {
        float q = 0.f;
        for (int k = 0; k < rpi; ++k) q += sh[k * c + t];
        part[((long long)n * parts + p) * c + t] = q;
    }
}

__global__ void k_chmean_final(const float* __restrict__ part, long long vps, int c, int nsamp, int parts,
                               float* __restrict__ mean)
{
    GRID_STRIDE(i, (long long)nsamp * c)
    {
        const long long n = i / c;
        const int ch = (int)(i % c);
        float s = 0.f;
#pragma unroll 16
        for (int p = 0; p < parts; ++p) s += part[(n * parts + p) * c + ch];  // loads in flight together
        mean[i] = s / (float)vps;
    }
}

__global__ void k_chmean_bcast8(const float* __restrict__ mean, long long vps, int c, bf16* __restrict__ y,
                                long long total8)
{
    const int q8 = c / 8;
    GRID_STRIDE(i, total8)
    {
        const int q = (int)(i % q8);
        const long long n = i / q8 / vps;
        float f[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) f[e] = mean[n * c + 8 * q + e];
        *(u4*)(y + i * 8) = pack8(f);
    }
}

// Joins of the U-Net bottleneck's global context (channel counts multiples of
// 32): y = [x | broadcast mean] for the forward concatenation, and
// y = act'(gate) * (skip + broadcast mean) for its gradient.
__global__ void k_chmean_concat8(const float* __restrict__ mean, long long vps, int c, const bf16* __restrict__ x,
                                 bf16* __restrict__ y, long long total8)
{
    const int qc = c / 8, q8 = 2 * qc;
    GRID_STRIDE(i, total8)
    {
        const int q = (int)(i % q8);
        const long long v = i / q8;
        if (q < qc) {
            *(u4*)(y + i * 8) = *(const u4*)(x + v * c + 8 * q);
        } else {
            const long long n = v / vps;
            float f[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) f[e] = mean[n * c + 8 * (q - qc) + e];
            *(u4*)(y + i * 8) = pack8(f);
        }
    }
}

__global__ void k_chmean_add_act8(const float* __restrict__ mean, long long vps, int c,
                                  const bf16* __restrict__ skip, int ldskip, const bf16* __restrict__ gate, int act,
                                  bf16* __restrict__ y, long long total8)
{
    const int q8 = c / 8;
    GRID_STRIDE(i, total8)
    {
        const int q = (int)(i % q8);
        const long long v = i / q8, n = v / vps;
        float f[8], t[8];
        unpack8(*(const u4*)(skip + v * ldskip + 8 * q), t);
#pragma unroll
        for (int e = 0; e < 8; ++e) f[e] = mean[n * c + 8 * q + e] + t[e];
        act_grad8(gate + i * 8, act, f);
        *(u4*)(y + i * 8) = pack8(f);
    }
}

__global__ void k_chmean_bcast(const float* __restrict__ part, long long vps, int c, int nsamp, int parts,
                               bf16* __restrict__ y)
{
    const long long total = (long long)nsamp * vps * c;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const int ch = (int)(i % c);
        const long long n = i / c / vps;
        float s = 0.f;
        for (int p = 0; p < parts; ++p) s += part[(n * parts + p) * c + ch];
        y[i] = (bf16)(s / (float)vps);
    }
}

constexpr int kMeanParts = 64;

int launched() { return hipGetLastError() == hipSuccess ? CMNN_OK : CMNN_EHIP; }

int sum_chunks(const float* part, long long pstride, long long n0, long long n1, int nchunk, float* out0, float* out1,
               hipStream_t s)
{
    const unsigned nblk = (unsigned)((n0 + n1 + 63) / 64);
    if (nchunk >= 128)
        k_sum_chunks<16><<<nblk, 1024, 0, s>>>(part, pstride, n0, n1, nchunk, out0, out1);
    else
        k_sum_chunks<8><<<nblk, 512, 0, s>>>(part, pstride, n0, n1, nchunk, out0, out1);
    return launched();
}

dim3 grid_for(long long n)
{
    long long b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

bool brick_ok(const G& g) { return g.d % kTD == 0 && g.h % kTH == 0 && g.w % kTW == 0; }
// The brick weight-gradient kernel addresses x and dy with 32-bit byte offsets.
bool bwd_w_brick(const G& g, int cin, int cout)
{
    return brick_ok(g) && g.nvox * 2LL * (cin > cout ? cin : cout) < (1LL << 32);
}

// Voxel chunks of the weight gradient (partials summed in a fixed order).
// Brick path: about 256 workgroups of 8 waves (one per CU), whole bricks
// per chunk.  Generic path: >= 4096 voxels per chunk.
int bwd_w_chunks(const G& g, int cin, int cout)
{
    if (bwd_w_brick(g, cin, cout)) {
        // one workgroup per CU (147 KB of LDS): at most 256 (chunk, tile)
        // workgroups, so that none waits for a second round
        const long long bricks = g.nvox / (kTD * kTH * kTW);
        const long long tiles = (long long)(cin / 32) * (cout / 32);
        long long c = 256 / tiles;
        if (c < 1) c = 1;
        if (c > bricks) c = bricks;
        const long long per = (bricks + c - 1) / c;
        return (int)((bricks + per - 1) / per);
    }
    long long c = (g.nvox + 4095) / 4096;
    return (int)(c < 64 ? c : 64);
}

template <int NB, int SIGN, int ACT>
int conv_tile_launch(const G& g, const bf16* x, int cin, const bf16* w, const float* bias, int cout, bf16* y,
                     const bf16* gate, hipStream_t s)
{
    const unsigned bricks = (unsigned)(g.nvox / (kTD * kTH * kTW));
    const unsigned span = bricks % 8 == 0 ? bricks / 8 : 0;
    k_conv_tile<NB, SIGN, ACT><<<dim3(bricks, cout / (16 * NB)), 256, 0, s>>>(g, x, cin, w, bias, cout, y, span, gate);
    return launched();
}

template <int SIGN, int ACT>
int conv_dispatch(const G& g, const bf16* x, int cin, const bf16* w, const float* bias, int cout, bf16* y,
                  const bf16* gate, hipStream_t s)
{
    // the brick kernel addresses the weights with 32-bit byte offsets
    if (brick_ok(g) && 27LL * cout * cin * 2 < (1LL << 32)) {
        // widest output tile that still leaves >= 512 workgroups (two per CU)
        const long long bricks = g.nvox / (kTD * kTH * kTW);
        const int c16 = cout / 16;
        if (c16 % 6 == 0 && bricks * (c16 / 6) >= 512) return conv_tile_launch<6, SIGN, ACT>(g, x, cin, w, bias, cout, y, gate, s);
        if (c16 % 4 == 0 && bricks * (c16 / 4) >= 512) return conv_tile_launch<4, SIGN, ACT>(g, x, cin, w, bias, cout, y, gate, s);
        // a grid of fewer workgroups than CUs takes 16-channel tiles (twice the workgroups)
        if (bricks * (c16 / 2) < 256) return conv_tile_launch<1, SIGN, ACT>(g, x, cin, w, bias, cout, y, gate, s);
        return conv_tile_launch<2, SIGN, ACT>(g, x, cin, w, bias, cout, y, gate, s);
    }
    const unsigned mb = (unsigned)((g.nvox + 63) / 64);
    if (cout % 64 == 0)
        k_conv_fwd<4, SIGN, ACT><<<dim3(mb, cout / 64), 256, 0, s>>>(g, x, cin, w, bias, cout, y, gate);
    else
        k_conv_fwd<2, SIGN, ACT><<<dim3(mb, cout / 32), 256, 0, s>>>(g, x, cin, w, bias, cout, y, gate);
    return launched();
}

// Device scratch of the entry points that allocate nothing: a file-scope
// array of fixed size, one copy per GPU, found once per device through
// hipGetSymbolAddress (host code never uses the array's name as an address).
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of `scratch`, looked up on the first call on that device.
int static_scratch(void** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return CMNN_EHIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return CMNN_EHIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return CMNN_OK;
}

// every element index a call's kernel forms is below 2^32: its 32-bit index variant
bool idx32(long long elements) { return elements < (1LL << 32); }

void gather_pack(long long nsel, const int* idx, long long nvs, const float* src, int nsrc, int cs, bf16* dst, int c,
                 hipStream_t s)
{
    const long long n8 = nsel * nvs * c / 8;
    if (idx32(nsel * nvs * c) && idx32((long long)cs * nsrc * nvs))
        k_gather_pack8<uint32_t><<<grid_for(n8), 256, 0, s>>>((int)nsel, idx, nvs, src, nsrc, cs, dst, c);
    else
        k_gather_pack8<uint64_t><<<grid_for(n8), 256, 0, s>>>((int)nsel, idx, nvs, src, nsrc, cs, dst, c);
}

// the fine level of a coarse geometry must fit the voxel limit too
bool coarse_ok(const cmnn_geom* g) { return geom_ok(g) && 8LL * g->n * g->d * g->h * g->w <= 0x7fffffffLL; }
bool ld_ok(int ld, int c) { return ld >= c && ld % 8 == 0; }
bool gate_ok(const void* gate, int act)
{
    if (act == CMNN_ACT_NONE) return true;
    return act == CMNN_ACT_LEAKY && gate && al16(gate);
}

// Per-sample channel means of x (voxel rows ldx channels apart) into
// workspace: partial sums, then the means after them; returns the means.
const float* channel_means(const cmnn_geom* g, const void* x, int ldx, int c, void* workspace, hipStream_t s)
{
    const long long vps = (long long)g->d * g->h * g->w;
    k_chmean_part<<<(unsigned)(g->n * kMeanParts), 256, 0, s>>>((const bf16*)x, ldx, vps, c, kMeanParts,
                                                                 (float*)workspace);
    if (launched()) return nullptr;
    float* mean = (float*)workspace + (size_t)g->n * kMeanParts * c;
    k_chmean_final<<<grid_for((long long)g->n * c), 256, 0, s>>>((const float*)workspace, vps, c, g->n, kMeanParts,
                                                                 mean);
    return launched() ? nullptr : mean;
}

}  // namespace

extern "C" {

int cmnn_conv3d_fwd(const cmnn_geom* g, const void* x, int32_t cin, const void* w, const float* bias, int32_t cout,
                    int32_t act, void* y, void* hip_stream)
{
    if (!geom_ok(g) || !chan_ok(cin) || !chan_ok(cout) || !x || !w || !y) return CMNN_EINVAL;
    if (!al16(x) || !al16(w) || act < CMNN_ACT_NONE || act > CMNN_ACT_LEAKY) return CMNN_EINVAL;
    const G gg = make_g(g);
    hipStream_t s = (hipStream_t)hip_stream;
    if (act == CMNN_ACT_LEAKY)
        return conv_dispatch<1, CMNN_ACT_LEAKY>(gg, (const bf16*)x, cin, (const bf16*)w, bias, cout, (bf16*)y, nullptr,
                                                s);
    return conv_dispatch<1, CMNN_ACT_NONE>(gg, (const bf16*)x, cin, (const bf16*)w, bias, cout, (bf16*)y, nullptr, s);
}

int cmnn_conv3d_bwd_data(const cmnn_geom* g, const void* dy, int32_t cout, const void* w_t, int32_t cin, void* dx,
                         void* hip_stream)
{
    if (!geom_ok(g) || !chan_ok(cin) || !chan_ok(cout) || !dy || !w_t || !dx) return CMNN_EINVAL;
    if (!al16(dy) || !al16(w_t)) return CMNN_EINVAL;
    const G gg = make_g(g);
    // the data gradient is the forward kernel with negated tap offsets, input dy
    // (cout channels), transposed weights [27][cin][cout] and cin outputs
    return conv_dispatch<-1, CMNN_ACT_NONE>(gg, (const bf16*)dy, cout, (const bf16*)w_t, nullptr, cin, (bf16*)dx,
                                            nullptr, (hipStream_t)hip_stream);
}

int cmnn_conv3d_bwd_data_act(const cmnn_geom* g, const void* dy, int32_t cout, const void* w_t, int32_t cin,
                             const void* gate, int32_t act, void* dx, void* hip_stream)
{
    if (!geom_ok(g) || !chan_ok(cin) || !chan_ok(cout) || !dy || !w_t || !dx) return CMNN_EINVAL;
    if (!al16(dy) || !al16(w_t) || act < CMNN_ACT_NONE || act > CMNN_ACT_LEAKY) return CMNN_EINVAL;
    if (act == CMNN_ACT_LEAKY && (!gate || !al16(gate) || gate == dx)) return CMNN_EINVAL;
    const G gg = make_g(g);
    if (act == CMNN_ACT_NONE)
        return conv_dispatch<-1, CMNN_ACT_NONE>(gg, (const bf16*)dy, cout, (const bf16*)w_t, nullptr, cin, (bf16*)dx,
                                                nullptr, (hipStream_t)hip_stream);
    return conv_dispatch<-1, CMNN_ACT_LEAKY>(gg, (const bf16*)dy, cout, (const bf16*)w_t, nullptr, cin, (bf16*)dx,
                                             (const bf16*)gate, (hipStream_t)hip_stream);
}

int cmnn_conv3d_bwd_weight_workspace(const cmnn_geom* g, int32_t cin, int32_t cout, size_t* bytes)
{
    if (!geom_ok(g) || !chan_ok(cin) || !chan_ok(cout) || !bytes) return CMNN_EINVAL;
    const G gg = make_g(g);
    const size_t nc = (size_t)bwd_w_chunks(gg, cin, cout);
    *bytes = nc * 27 * (size_t)cin * cout * sizeof(float) + (size_t)kColSumBlocks * cout * sizeof(float);
    return CMNN_OK;
}

int cmnn_conv3d_bwd_weight(const cmnn_geom* g, const void* x, int32_t cin, const void* dy, int32_t cout, float* dw,
                           float* dbias, void* workspace, size_t workspace_bytes, void* hip_stream)
{
    size_t need = 0;
    if (cmnn_conv3d_bwd_weight_workspace(g, cin, cout, &need) != CMNN_OK) return CMNN_EINVAL;
    if (!x || !dy || !dw || !workspace || workspace_bytes < need || !al16(x) || !al16(dy)) return CMNN_EINVAL;
    if (cout > 256) return CMNN_EINVAL;
    const G gg = make_g(g);
    hipStream_t s = (hipStream_t)hip_stream;
    const int nc = bwd_w_chunks(gg, cin, cout);
    float* part = (float*)workspace;
    const long long per = 27LL * cin * cout;
    float* bpart = part + (long long)nc * per;
    if (bwd_w_brick(gg, cin, cout)) {
        const long long bricks = gg.nvox / (kTD * kTH * kTW);
        const int per_chunk = (int)((bricks + nc - 1) / nc);
        const unsigned nblk = (unsigned)(nc * (cout / 32) * (cin / 32));
        // per chunk: the 27 x cout x cin weight partials, then the cout bias partials,
        // summed over the chunks by one launch; nc <= 256 <= kColSumBlocks, so the
        // nc * (per + cout) floats fit the workspace
        const long long pst = per + cout, nb = dbias ? cout : 0;
        k_conv_bwd_w_tile<<<nblk, kBwThreads, 0, s>>>(gg, (const bf16*)x, cin, (const bf16*)dy, cout, per_chunk, part,
                                                      pst, dbias != nullptr);
        if (launched()) return CMNN_EHIP;
        return sum_chunks(part, pst, per, nb, nc, dw, dbias, s);
    } else {
        const long long chunk = (gg.nvox + nc - 1) / nc;
        const unsigned nblk = (unsigned)(nc * 27 * (cout / 32) * (cin / 32));
        k_conv_bwd_w<<<nblk, 256, 0, s>>>(gg, (const bf16*)x, cin, (const bf16*)dy, cout, chunk, part);
    }
    if (launched()) return CMNN_EHIP;
    if (sum_chunks(part, per, per, 0, nc, dw, nullptr, s)) return CMNN_EHIP;
    if (dbias) {
        long long nb = (gg.nvox + 1023) / 1024;
        if (nb > kColSumBlocks) nb = kColSumBlocks;
        const long long bchunk = (gg.nvox + nb - 1) / nb;
        k_colsum_part<<<(unsigned)nb, 256, 0, s>>>((const bf16*)dy, gg.nvox, cout, bchunk, bpart);
        if (launched()) return CMNN_EHIP;
        if (sum_chunks(bpart, cout, cout, 0, (int)nb, dbias, nullptr, s)) return CMNN_EHIP;
    }
    return CMNN_OK;
}

int cmnn_conv3d_bwd_weight_noalloc(const cmnn_geom* g, const void* x, int32_t cin, const void* dy, int32_t cout,
                                   float* dw, float* dbias, void* hip_stream)
{
    size_t need = 0;
    if (cmnn_conv3d_bwd_weight_workspace(g, cin, cout, &need) != CMNN_OK) return CMNN_EINVAL;
    if (need > kStaticScratchBytes) return CMNN_EINVAL;  // beyond the fixed scratch: nothing enqueued
    if (!x || !dy || !dw || !al16(x) || !al16(dy) || cout > 256) return CMNN_EINVAL;
    void* ws = nullptr;
    const int rc = static_scratch(&ws);
    if (rc != CMNN_OK) return rc;
    // every partial the kernels read is written first in the same call, so the
    // previous call's contents need no clearing
    return cmnn_conv3d_bwd_weight(g, x, cin, dy, cout, dw, dbias, ws, kStaticScratchBytes, hip_stream);
}

int cmnn_act_bwd(const void* y, const void* dy, void* dpre, size_t n, int32_t act, void* hip_stream)
{
    if (!y || !dy || !dpre || act < CMNN_ACT_NONE || act > CMNN_ACT_LEAKY) return CMNN_EINVAL;
    if (n % 8 == 0 && al16(y) && al16(dy) && al16(dpre)) {
        k_act_bwd8<<<grid_for((long long)n / 8), 256, 0, (hipStream_t)hip_stream>>>(
            (const u4*)y, (const u4*)dy, (u4*)dpre, (long long)n / 8, act);
        return launched();
    }
    k_act_bwd<<<grid_for((long long)n), 256, 0, (hipStream_t)hip_stream>>>((const bf16*)y, (const bf16*)dy,
                                                                         (bf16*)dpre, (long long)n, act);
    return launched();
}

int cmnn_pool2_fwd(const cmnn_geom* g, const void* x, int32_t c, void* y, void* hip_stream)
{
    if (!geom_ok(g) || c <= 0 || !x || !y || (g->d | g->h | g->w) & 1) return CMNN_EINVAL;
    const G gg = make_g(g);
    if (c % 8 == 0 && al16(x) && al16(y))
    {
        if (idx32(gg.nvox * c))
            k_pool2_fwd8<uint32_t><<<grid_for(gg.nvox * c / 64), 256, 0, (hipStream_t)hip_stream>>>(gg, (const bf16*)x,
                                                                                                   c, (bf16*)y);
        else
            k_pool2_fwd8<uint64_t><<<grid_for(gg.nvox * c / 64), 256, 0, (hipStream_t)hip_stream>>>(gg, (const bf16*)x,
                                                                                                   c, (bf16*)y);
    }
    else
        k_pool2_fwd<<<grid_for(gg.nvox * c / 8), 256, 0, (hipStream_t)hip_stream>>>(gg, (const bf16*)x, c, (bf16*)y);
    return launched();
}

int cmnn_pool2_bwd(const cmnn_geom* g, const void* dy, int32_t c, void* dx, void* hip_stream)
{
    if (!geom_ok(g) || c <= 0 || !dy || !dx || (g->d | g->h | g->w) & 1) return CMNN_EINVAL;
    const G gg = make_g(g);
    if (c % 8 == 0 && al16(dy) && al16(dx))
        k_pool2_bwd8<<<grid_for(gg.nvox * c / 8), 256, 0, (hipStream_t)hip_stream>>>(gg, (const bf16*)dy, c, (bf16*)dx);
    else
        k_pool2_bwd<<<grid_for(gg.nvox * c), 256, 0, (hipStream_t)hip_stream>>>(gg, (const bf16*)dy, c, (bf16*)dx);
    return launched();
}

int cmnn_up2_fwd(const cmnn_geom* g, const void* x, int32_t c, void* y, void* hip_stream)
{
    if (!geom_ok(g) || c <= 0 || !x || !y) return CMNN_EINVAL;
    const G gg = make_g(g);
    if (c % 8 == 0 && al16(x) && al16(y))
        k_up2_fwd8<<<grid_for(gg.nvox * c), 256, 0, (hipStream_t)hip_stream>>>(gg, (const bf16*)x, c, (bf16*)y);
    else
        k_up2_fwd<<<grid_for(gg.nvox * c * 8), 256, 0, (hipStream_t)hip_stream>>>(gg, (const bf16*)x, c, (bf16*)y);
    return launched();
}

int cmnn_up2_bwd(const cmnn_geom* g, const void* dy, int32_t c, void* dx, void* hip_stream)
{
    if (!geom_ok(g) || c <= 0 || !dy || !dx) return CMNN_EINVAL;
    const G gg = make_g(g);
    if (c % 8 == 0 && al16(dy) && al16(dx))
        k_up2_bwd8<<<grid_for(gg.nvox * c / 8), 256, 0, (hipStream_t)hip_stream>>>(gg, (const bf16*)dy, c, (bf16*)dx);
    else
        k_up2_bwd<<<grid_for(gg.nvox * c), 256, 0, (hipStream_t)hip_stream>>>(gg, (const bf16*)dy, c, (bf16*)dx);
    return launched();
}

int cmnn_concat_fwd(size_t nvox, const void* a, int32_t ca, const void* b, int32_t cb, void* y, void* hip_stream)
{
    if (!a || !b || !y || ca <= 0 || cb <= 0) return CMNN_EINVAL;
    if (ca % 8 == 0 && cb % 8 == 0 && al16(a) && al16(b) && al16(y))
        k_concat_fwd8<<<grid_for((long long)nvox * (ca + cb) / 8), 256, 0, (hipStream_t)hip_stream>>>(
            (long long)nvox, (const bf16*)a, ca, (const bf16*)b, cb, (bf16*)y);
    else
        k_concat_fwd<<<grid_for((long long)nvox * (ca + cb)), 256, 0, (hipStream_t)hip_stream>>>(
            (long long)nvox, (const bf16*)a, ca, (const bf16*)b, cb, (bf16*)y);
    return launched();
}

int cmnn_concat_bwd(size_t nvox, const void* dy, int32_t ca, int32_t cb, void* da, void* db, void* hip_stream)
{
    if (!dy || ca <= 0 || cb <= 0) return CMNN_EINVAL;
    if (ca % 8 == 0 && cb % 8 == 0 && al16(dy) && al16(da) && al16(db))
        k_concat_bwd8<<<grid_for((long long)nvox * (ca + cb) / 8), 256, 0, (hipStream_t)hip_stream>>>(
            (long long)nvox, (const bf16*)dy, ca, cb, (bf16*)da, (bf16*)db);
    else
        k_concat_bwd<<<grid_for((long long)nvox * (ca + cb)), 256, 0, (hipStream_t)hip_stream>>>(
            (long long)nvox, (const bf16*)dy, ca, cb, (bf16*)da, (bf16*)db);
    return launched();
}

int cmnn_up2_concat_fwd(const cmnn_geom* g, const void* skip, int32_t cs, const void* x, int32_t cx, void* y,
                        void* hip_stream)
{
    if (!coarse_ok(g) || !chan_ok(cs) || !chan_ok(cx) || !skip || !x || !y || !al16(skip) || !al16(x) || !al16(y))
        return CMNN_EINVAL;
    const G gg = make_g(g);
    if (idx32(8 * gg.nvox * (cs + cx)))
        k_up2_concat_fwd8<uint32_t><<<grid_for(8 * gg.nvox * (cs + cx) / 8), 256, 0, (hipStream_t)hip_stream>>>(
            gg, (const bf16*)skip, cs, (const bf16*)x, cx, (bf16*)y);
    else
        k_up2_concat_fwd8<uint64_t><<<grid_for(8 * gg.nvox * (cs + cx) / 8), 256, 0, (hipStream_t)hip_stream>>>(
            gg, (const bf16*)skip, cs, (const bf16*)x, cx, (bf16*)y);
    return launched();
}

int cmnn_up2_bwd_act(const cmnn_geom* g, const void* dy, int32_t ldy, int32_t c, const void* gate, int32_t act,
                     void* dx, void* hip_stream)
{
    if (!coarse_ok(g) || !chan_ok(c) || !ld_ok(ldy, c) || !dy || !dx || !al16(dy) || !al16(dx) || !gate_ok(gate, act))
        return CMNN_EINVAL;
    const G gg = make_g(g);
    if (idx32(8 * gg.nvox * ldy))
        k_up2_bwd_act8<uint32_t><<<grid_for(gg.nvox * c / 8), 256, 0, (hipStream_t)hip_stream>>>(
            gg, (const bf16*)dy, ldy, c, (const bf16*)gate, act, (bf16*)dx);
    else
        k_up2_bwd_act8<uint64_t><<<grid_for(gg.nvox * c / 8), 256, 0, (hipStream_t)hip_stream>>>(
            gg, (const bf16*)dy, ldy, c, (const bf16*)gate, act, (bf16*)dx);
    return launched();
}

int cmnn_pool2_bwd_add_act(const cmnn_geom* g, const void* dy, int32_t c, const void* skip, int32_t ldskip,
                           const void* gate, int32_t act, void* dx, void* hip_stream)
{
    if (!geom_ok(g) || (g->d | g->h | g->w) & 1 || !chan_ok(c) || !dy || !dx || !al16(dy) || !al16(dx) ||
        !gate_ok(gate, act))
        return CMNN_EINVAL;
    if (skip && (!al16(skip) || !ld_ok(ldskip, c))) return CMNN_EINVAL;
    const G gg = make_g(g);
    if (idx32(gg.nvox * (skip && ldskip > c ? ldskip : c)))
        k_pool2_bwd_add_act8<uint32_t><<<grid_for(gg.nvox * c / 8), 256, 0, (hipStream_t)hip_stream>>>(
            gg, (const bf16*)dy, c, (const bf16*)skip, ldskip, (const bf16*)gate, act, (bf16*)dx);
    else
        k_pool2_bwd_add_act8<uint64_t><<<grid_for(gg.nvox * c / 8), 256, 0, (hipStream_t)hip_stream>>>(
            gg, (const bf16*)dy, c, (const bf16*)skip, ldskip, (const bf16*)gate, act, (bf16*)dx);
    return launched();
}

int cmnn_add(size_t n, const void* a, const void* b, void* y, void* hip_stream)
{
    if (!a || !b || !y) return CMNN_EINVAL;
    if (n % 8 == 0 && al16(a) && al16(b) && al16(y))
        k_add8<<<grid_for((long long)n / 8), 256, 0, (hipStream_t)hip_stream>>>((long long)n / 8, (const u4*)a,
                                                                               (const u4*)b, (u4*)y);
    else
        k_add<<<grid_for((long long)n), 256, 0, (hipStream_t)hip_stream>>>((long long)n, (const bf16*)a,
                                                                         (const bf16*)b, (bf16*)y);
    return launched();
}

int cmnn_channel_mean_workspace(const cmnn_geom* g, int32_t c, size_t* bytes)
{
    if (!geom_ok(g) || c <= 0 || c > 256 || !bytes || (long long)g->n * kMeanParts > 0x7fffffffLL) return CMNN_EINVAL;
    *bytes = (size_t)g->n * (kMeanParts + 1) * c * sizeof(float);
    return CMNN_OK;
}

int cmnn_channel_mean(const cmnn_geom* g, const void* x, int32_t c, void* y, void* workspace, size_t workspace_bytes,
                      void* hip_stream)
{
    size_t need = 0;
    if (cmnn_channel_mean_workspace(g, c, &need) != CMNN_OK || !x || !y || !workspace || workspace_bytes < need)
        return CMNN_EINVAL;
    const G gg = make_g(g);
    hipStream_t s = (hipStream_t)hip_stream;
    const long long vps = (long long)g->d * g->h * g->w;
    k_chmean_part<<<(unsigned)(g->n * kMeanParts), 256, 0, s>>>((const bf16*)x, c, vps, c, kMeanParts,
                                                                 (float*)workspace);
    if (launched()) return CMNN_EHIP;
    if (c % 8 == 0 && al16(y)) {
        float* mean = (float*)workspace + (size_t)g->n * kMeanParts * c;
        k_chmean_final<<<grid_for((long long)g->n * c), 256, 0, s>>>((const float*)workspace, vps, c, g->n,
                                                                     kMeanParts, mean);
        if (launched()) return CMNN_EHIP;
        k_chmean_bcast8<<<grid_for(gg.nvox * c / 8), 256, 0, s>>>(mean, vps, c, (bf16*)y, gg.nvox * c / 8);
        return launched();
    }
    k_chmean_bcast<<<grid_for(gg.nvox * c), 256, 0, s>>>((const float*)workspace, vps, c, g->n, kMeanParts, (bf16*)y);
    return launched();
}

int cmnn_channel_mean_concat(const cmnn_geom* g, const void* x, int32_t c, void* y, void* workspace,
                             size_t workspace_bytes, void* hip_stream)
{
    size_t need = 0;
    if (cmnn_channel_mean_workspace(g, c, &need) != CMNN_OK || !chan_ok(c) || !x || !y || !al16(x) || !al16(y) ||
        !workspace || workspace_bytes < need)
        return CMNN_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    const float* mean = channel_means(g, x, c, c, workspace, s);
    if (!mean) return CMNN_EHIP;
    const long long total8 = make_g(g).nvox * 2 * c / 8;
    k_chmean_concat8<<<grid_for(total8), 256, 0, s>>>(mean, (long long)g->d * g->h * g->w, c, (const bf16*)x,
                                                      (bf16*)y, total8);
    return launched();
}

int cmnn_channel_mean_add_act(const cmnn_geom* g, const void* dy, int32_t ldy, int32_t c, const void* skip,
                              int32_t ldskip, const void* gate, int32_t act, void* dx, void* workspace,
                              size_t workspace_bytes, void* hip_stream)
{
    size_t need = 0;
    if (cmnn_channel_mean_workspace(g, c, &need) != CMNN_OK || !chan_ok(c) || !ld_ok(ldy, c) || !ld_ok(ldskip, c) ||
        !dy || !skip || !dx || !al16(dy) || !al16(skip) || !al16(dx) || !gate_ok(gate, act) || !workspace ||
        workspace_bytes < need)
        return CMNN_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    const float* mean = channel_means(g, dy, ldy, c, workspace, s);
    if (!mean) return CMNN_EHIP;
    const long long total8 = make_g(g).nvox * c / 8;
    k_chmean_add_act8<<<grid_for(total8), 256, 0, s>>>(mean, (long long)g->d * g->h * g->w, c, (const bf16*)skip,
                                                       ldskip, (const bf16*)gate, act, (bf16*)dx, total8);
    return launched();
}

int cmnn_mse_workspace(size_t nvox, size_t* bytes)
{
    if (!bytes || nvox == 0) return CMNN_EINVAL;
    *bytes = 2 * kMseBlocks * sizeof(float);
    return CMNN_OK;
}

int cmnn_mse(size_t nvox, const void* pred, int32_t c, int32_t creal, const float* target, const float* weight,
             float* loss_out, void* dpred, void* workspace, size_t workspace_bytes, void* hip_stream)
{
    if (!pred || !target || !weight || !loss_out || !workspace || nvox == 0) return CMNN_EINVAL;
    if (c <= 0 || creal <= 0 || creal > c || workspace_bytes < 2 * kMseBlocks * sizeof(float)) return CMNN_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    float* part = (float*)workspace;
    k_mse_part<<<kMseBlocks, 256, 0, s>>>((long long)nvox, (const bf16*)pred, c, creal, target, weight, part);
    if (launched()) return CMNN_EHIP;
    // loss_out[0] = loss, loss_out[1] = normaliser (callers pass two floats)
    k_mse_final<<<1, 256, 0, s>>>(part, kMseBlocks, creal, loss_out);
    if (launched()) return CMNN_EHIP;
    if (dpred && c % 8 == 0 && al16(pred) && al16(dpred)) {
        if (idx32((long long)nvox * c))
            k_mse_grad8<uint32_t><<<grid_for((long long)nvox * c / 8), 256, 0, s>>>(
                (long long)nvox, (const bf16*)pred, c, creal, target, weight, loss_out, (bf16*)dpred);
        else
            k_mse_grad8<uint64_t><<<grid_for((long long)nvox * c / 8), 256, 0, s>>>(
                (long long)nvox, (const bf16*)pred, c, creal, target, weight, loss_out, (bf16*)dpred);
        if (launched()) return CMNN_EHIP;
    } else if (dpred) {
        k_mse_grad<<<grid_for((long long)nvox * c), 256, 0, s>>>((long long)nvox, (const bf16*)pred, c, creal, target,
                                                               weight, loss_out, (bf16*)dpred);
        if (launched()) return CMNN_EHIP;
    }
    return CMNN_OK;
}

int cmnn_clip_grad_norm_workspace(size_t n, size_t* bytes)
{
    if (!bytes || n == 0) return CMNN_EINVAL;
    *bytes = kClipBlocks * sizeof(float);
    return CMNN_OK;
}

int cmnn_clip_grad_norm(size_t n, float* grad, float max_norm, float* norm_out, void* workspace,
                        size_t workspace_bytes, void* hip_stream)
{
    if (!grad || !norm_out || !workspace || n == 0 || workspace_bytes < kClipBlocks * sizeof(float) ||
        !(max_norm >= 0.f))
        return CMNN_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    float* part = (float*)workspace;
    k_sumsq_part<<<kClipBlocks, 256, 0, s>>>((long long)n, grad, part);
    if (launched()) return CMNN_EHIP;
    k_clip_final<<<1, 256, 0, s>>>(part, kClipBlocks, max_norm, norm_out);
    if (launched()) return CMNN_EHIP;
    k_scale<<<grid_for((long long)n), 256, 0, s>>>((long long)n, grad, norm_out);
    return launched();
}

int cmnn_adam(size_t n, float* param, const float* grad, float* m, float* v, float lr, float beta1, float beta2,
              float eps, float weight_decay, int32_t step, void* hip_stream)
{
    if (!param || !grad || !m || !v || step < 1) return CMNN_EINVAL;
    const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
    k_adam<<<grid_for((long long)n), 256, 0, (hipStream_t)hip_stream>>>((long long)n, param, grad, m, v, lr, beta1,
                                                                      beta2, eps, weight_decay, c1, c2);
    return launched();
}

int cmnn_pack_weights(const float* w, int32_t cin, int32_t cout, void* w_fwd, void* w_t, void* hip_stream)
{
    if (!w || !w_fwd || !w_t || cin <= 0 || cout <= 0) return CMNN_EINVAL;
    k_pack_w<<<grid_for(27LL * cin * cout), 256, 0, (hipStream_t)hip_stream>>>(w, cin, cout, (bf16*)w_fwd, (bf16*)w_t);
    return launched();
}

int cmnn_pack_weights_batch(int32_t n, const cmnn_pack_job* jobs, void* hip_stream)
{
    if (n <= 0 || n > CMNN_PACK_MAX || !jobs) return CMNN_EINVAL;
    PackJobs J = {};
    long long blocks = 0;
    for (int l = 0; l < n; ++l) {
        const cmnn_pack_job& j = jobs[l];
        if (!j.w || !j.w_fwd || !j.w_t || j.cin <= 0 || j.cout <= 0) return CMNN_EINVAL;
        J.w[l] = j.w;
        J.wf[l] = (bf16*)j.w_fwd;
        J.wt[l] = (bf16*)j.w_t;
        J.cin[l] = j.cin;
        J.cout[l] = j.cout;
        J.first_block[l] = (int)blocks;
        blocks += (27LL * j.cin * j.cout + 255) / 256;
        if (blocks > 0x7fffffffLL) return CMNN_EINVAL;
    }
    J.first_block[n] = (int)blocks;
    J.n = n;
    k_pack_w_batch<<<(unsigned)blocks, 256, 0, (hipStream_t)hip_stream>>>(J);
    return launched();
}

int cmnn_pack_channels(size_t nvox, const float* src, int32_t cs, void* dst, int32_t c, void* hip_stream)
{
    if (!src || !dst || cs <= 0 || c < cs) return CMNN_EINVAL;
    if (c % 8 == 0 && al16(dst)) {
        // one "sample" of nvox voxels, taken in place
        gather_pack((long long)1, nullptr, (long long)nvox, src, 1, cs, (bf16*)dst, c, (hipStream_t)hip_stream);
        return launched();
    }
    k_pack_ch<<<grid_for((long long)nvox * c), 256, 0, (hipStream_t)hip_stream>>>((long long)nvox, src, cs, (bf16*)dst,
                                                                                c);
    return launched();
}

int cmnn_gather_pack_channels(int32_t nsel, const int32_t* idx, size_t nvs, const float* src, int32_t nsrc,
                              int32_t cs, void* dst, int32_t c, void* hip_stream)
{
    if (nsel <= 0 || !idx || nvs == 0 || !src || nsrc <= 0 || cs <= 0 || c < cs || c % 8 != 0 || !dst || !al16(dst))
        return CMNN_EINVAL;
    gather_pack(nsel, idx, (long long)nvs, src, nsrc, cs, (bf16*)dst, c, (hipStream_t)hip_stream);
    return launched();
}

int cmnn_gather_samples(int32_t nsel, const int32_t* idx, size_t nvs, const float* src, int32_t nsrc, int32_t np,
                        float* dst, void* hip_stream)
{
    if (nsel <= 0 || !idx || nvs == 0 || !src || nsrc <= 0 || np <= 0 || !dst) return CMNN_EINVAL;
    if (nvs % 4 == 0 && al16(src) && al16(dst))
        k_gather4<<<grid_for((long long)np * nsel * nvs / 4), 256, 0, (hipStream_t)hip_stream>>>(
            nsel, idx, (long long)nvs / 4, (const float4*)src, nsrc, np, (float4*)dst);
    else
        k_gather1<<<grid_for((long long)np * nsel * nvs), 256, 0, (hipStream_t)hip_stream>>>(nsel, idx, (long long)nvs,
                                                                                          src, nsrc, np, dst);
    return launched();
}

int cmnn_unpack_channels(size_t nvox, const void* src, int32_t c, float* dst, int32_t cs, void* hip_stream)
{
    if (!src || !dst || cs <= 0 || c < cs) return CMNN_EINVAL;
    k_unpack_ch<<<grid_for((long long)nvox * cs), 256, 0, (hipStream_t)hip_stream>>>((long long)nvox, (const bf16*)src,
                                                                                   c, dst, cs);
    return launched();
}

}  // extern "C"
