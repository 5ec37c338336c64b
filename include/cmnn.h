/*
 * cmnn.h -- C ABI of the gfx950 kernels of the learned warm start: a small
 * 3D convolutional U-Net trained on the GPU to predict the steady velocity of
 * forced obstacle channels, whose prediction initialises the lattice
 * Boltzmann solver of cmlbm.h (an extension of the method of De Rosis, Huang
 * & Coreixas, PRE 2019; the paper itself has no learned component).
 *
 * Conventions
 * - Activations are BF16, layout NDHWC: [n][d][h][w][c], c fastest, with the
 *   channel count padded to a multiple of 32 (CMNN_CALIGN); padded channels
 *   hold zeros.  d, h, w are the lattice z, y, x axes.
 * - Convolutions are 3x3x3, stride 1, "same" size.  Per axis the padding is
 *   periodic (the lattice's periodic axes) or zero (the wall axis).  Tap
 *   t = (dz+1)*9 + (dy+1)*3 + (dx+1) reads the input at (d+dz, h+dy, w+dx):
 *   a cross-correlation, y[v][co] = sum_t sum_ci x[v + off(t)][ci] w[t][co][ci].
 * - Forward weights are BF16 [27][cout][cin] (cin fastest), bias FP32 [cout].
 *   The data gradient uses the transposed copy [27][cin][cout] written by
 *   cmnn_pack_weights.  Weight and bias gradients are FP32.
 * - Products run on BF16 MFMA (v_mfma_f32_16x16x32_bf16) with FP32
 *   accumulation; elementwise work is FP32 arithmetic on BF16 storage.
 * - Every function enqueues on hip_stream (NULL = null stream), returns 0 or
 *   a negative CMNN_E* code, checks its arguments on the host first and
 *   never allocates: buffers are caller-owned device memory, 16-byte aligned.
 * - A geometry needs positive extents and at most 2^31 - 1 voxels (EINVAL
 *   otherwise).
 */
#ifndef CMNN_H
#define CMNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CMNN_OK 0
#define CMNN_EINVAL (-1) /* bad argument; nothing enqueued */
#define CMNN_EHIP (-3)   /* HIP launch failure */

#define CMNN_CALIGN 32 /* channel padding of every activation tensor */

#define CMNN_ACT_NONE 0
#define CMNN_ACT_LEAKY 1 /* leaky ReLU, slope 0.1 for negative inputs */

typedef struct {
    int32_t n, d, h, w;   /* batch and spatial extent (z, y, x) */
    int32_t periodic[3];  /* d, h, w axes: 1 periodic padding, 0 zero padding */
} cmnn_geom;

/* y = act(conv3x3x3(x, w) + bias).  x [n][d][h][w][cin], y [..][cout]. */
int cmnn_conv3d_fwd(const cmnn_geom* g, const void* x, int32_t cin, const void* w, const float* bias,
                    int32_t cout, int32_t act, void* y, void* hip_stream);

/* dx = transposed convolution of dy (pre-activation gradient) with the
 * transposed weights w_t [27][cin][cout]; dx [..][cin], dy [..][cout]. */
int cmnn_conv3d_bwd_data(const cmnn_geom* g, const void* dy, int32_t cout, const void* w_t, int32_t cin, void* dx,
                         void* hip_stream);

/* The data gradient of cmnn_conv3d_bwd_data with the activation gradient of
 * the layer that produced this layer's input fused in: dx as above, then,
 * for act = CMNN_ACT_LEAKY, each element multiplied by 0.1 where the same
 * element of gate (that layer's activation output, [..][cin] BF16, i.e. this
 * layer's input) is <= 0 -- the rule of cmnn_act_bwd, applied to the FP32
 * accumulator before the one BF16 rounding.  dx is then that layer's
 * pre-activation gradient.  act = CMNN_ACT_NONE is cmnn_conv3d_bwd_data
 * (gate ignored).  EINVAL on a NULL or misaligned gate, or gate == dx. */
int cmnn_conv3d_bwd_data_act(const cmnn_geom* g, const void* dy, int32_t cout, const void* w_t, int32_t cin,
                             const void* gate, int32_t act, void* dx, void* hip_stream);

/* Workspace bytes needed by cmnn_conv3d_bwd_weight. */
int cmnn_conv3d_bwd_weight_workspace(const cmnn_geom* g, int32_t cin, int32_t cout, size_t* bytes);

/* dw[t][co][ci] = sum_v dy[v][co] x[v + off(t)][ci] and dbias[co] = sum_v dy[v][co]
 * (dbias may be NULL), FP32, overwritten; cout <= 256.  Deterministic:
 * per-chunk partials in the workspace are summed in a fixed order. */
int cmnn_conv3d_bwd_weight(const cmnn_geom* g, const void* x, int32_t cin, const void* dy, int32_t cout, float* dw,
                           float* dbias, void* workspace, size_t workspace_bytes, void* hip_stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving or training loops, harnesses that forbid allocation): the weight
 * gradient of cmnn_conv3d_bwd_weight, same arguments and results (bitwise:
 * the same kernels), without a workspace argument.  Its per-chunk partials
 * live in a fixed device array of the library, 64 MiB per GPU, held until the
 * process ends; it calls no allocator.  Geometries whose
 * cmnn_conv3d_bwd_weight_workspace exceeds 64 MiB are rejected with
 * CMNN_EINVAL before any device work (every brick geometry with cout <= 256 and
 * cin <= 256 fits).  Every call on one GPU within a process shares that GPU's
 * array: calls that overlap in time on one GPU (on different streams or from
 * different threads) race, and the caller must order them.  CMNN_EHIP if the
 * array's address cannot be obtained on the current device. */
int cmnn_conv3d_bwd_weight_noalloc(const cmnn_geom* g, const void* x, int32_t cin, const void* dy, int32_t cout,
                                   float* dw, float* dbias, void* hip_stream);

/* dpre = dy * act'(.) evaluated from the activation output y; n elements. */
int cmnn_act_bwd(const void* y, const void* dy, void* dpre, size_t n, int32_t act, void* hip_stream);

/* 2x2x2 average pooling; g is the fine geometry (d, h, w even). */
int cmnn_pool2_fwd(const cmnn_geom* g, const void* x, int32_t c, void* y, void* hip_stream);
int cmnn_pool2_bwd(const cmnn_geom* g, const void* dy, int32_t c, void* dx, void* hip_stream);

/* 2x nearest upsampling; g is the coarse geometry. */
int cmnn_up2_fwd(const cmnn_geom* g, const void* x, int32_t c, void* y, void* hip_stream);
int cmnn_up2_bwd(const cmnn_geom* g, const void* dy, int32_t c, void* dx, void* hip_stream);

/* Channel concatenation y = [a | b] over nvox voxels, and its split (da or
 * db may be NULL: that part is not written). */
int cmnn_concat_fwd(size_t nvox, const void* a, int32_t ca, const void* b, int32_t cb, void* y, void* hip_stream);
int cmnn_concat_bwd(size_t nvox, const void* dy, int32_t ca, int32_t cb, void* da, void* db, void* hip_stream);

/* Skip-connection joins of the U-Net, each one pass in place of the separate
 * upsampling or pooling, concatenation, sum and activation-gradient calls it
 * replaces.  Channel counts are multiples of 32; a channel stride ld (the
 * distance in elements between two voxels' rows, >= the channel count, a
 * multiple of 8) lets a part of a concatenation be read in place: pass the
 * pointer to its first channel.  Outputs must not overlap inputs.  act is
 * CMNN_ACT_NONE (gate ignored) or CMNN_ACT_LEAKY (gate: the activation output
 * of the layer whose gradient this is; the FP32 result is multiplied by 0.1
 * where gate <= 0 before the one BF16 rounding).  EINVAL on a NULL or
 * misaligned pointer, a bad channel count or stride, or more than 2^31 - 1
 * fine voxels. */

/* Decoder join, forward: y = [skip | up2(x)].  g is the coarse geometry of x
 * [..][cx]; skip [..][cs] and y [..][cs + cx] are at the fine level (2d, 2h,
 * 2w).  Bitwise cmnn_up2_fwd then cmnn_concat_fwd, without the upsampled
 * tensor in between. */
int cmnn_up2_concat_fwd(const cmnn_geom* g, const void* skip, int32_t cs, const void* x, int32_t cx, void* y,
                        void* hip_stream);

/* Decoder join, backward of its upsampled part: dx [..][c] (coarse) = the sum
 * over each coarse voxel's 8 fine children of dy, channel stride ldy (the
 * upsampled part of the concatenation's gradient), times act'(gate), gate
 * coarse [..][c].  g is the coarse geometry. */
int cmnn_up2_bwd_act(const cmnn_geom* g, const void* dy, int32_t ldy, int32_t c, const void* gate, int32_t act,
                     void* dx, void* hip_stream);

/* Encoder join, backward: dx [..][c] (fine) = act'(gate) * (dy / 8 + skip),
 * dy coarse [..][c] the gradient of the 2x2x2 average pool of this level's
 * output, skip (channel stride ldskip; NULL: no term) the skip part of the
 * decoder concatenation's gradient, gate fine [..][c].  g is the fine
 * geometry (d, h, w even). */
int cmnn_pool2_bwd_add_act(const cmnn_geom* g, const void* dy, int32_t c, const void* skip, int32_t ldskip,
                           const void* gate, int32_t act, void* dx, void* hip_stream);

/* Per-sample channel mean broadcast over the voxels (global context):
 * y[n][v][c] = (1/V) sum_v' x[n][v'][c], V = d*h*w, c <= 256.  The map is a
 * symmetric projection, so the same call on dy gives the gradient.
 * workspace: cmnn_channel_mean_workspace bytes; n <= 2^25. */
int cmnn_channel_mean_workspace(const cmnn_geom* g, int32_t c, size_t* bytes);
int cmnn_channel_mean(const cmnn_geom* g, const void* x, int32_t c, void* y, void* workspace, size_t workspace_bytes,
                      void* hip_stream);

/* Global-context join of the U-Net bottleneck, forward: y [..][2c] =
 * [x | the per-sample channel means of x broadcast over the voxels], bitwise
 * cmnn_channel_mean then cmnn_concat_fwd.  c a multiple of 32, <= 256;
 * workspace: cmnn_channel_mean_workspace(g, c) bytes. */
int cmnn_channel_mean_concat(const cmnn_geom* g, const void* x, int32_t c, void* y, void* workspace,
                             size_t workspace_bytes, void* hip_stream);

/* Its backward: dx [..][c] = act'(gate) * (skip + the broadcast per-sample
 * channel means of dy) -- the mean map is its own adjoint -- where dy and
 * skip are the two parts of the concatenation's gradient, read in place with
 * channel strides ldy and ldskip, and gate [..][c] is the activation output of
 * the layer that produced x (rules of the skip-connection joins above).
 * workspace: cmnn_channel_mean_workspace(g, c) bytes. */
int cmnn_channel_mean_add_act(const cmnn_geom* g, const void* dy, int32_t ldy, int32_t c, const void* skip,
                              int32_t ldskip, const void* gate, int32_t act, void* dx, void* workspace,
                              size_t workspace_bytes, void* hip_stream);

/* y = a + b elementwise (BF16), n elements. */
int cmnn_add(size_t n, const void* a, const void* b, void* y, void* hip_stream);

/* Masked mean-squared error over the first creal channels of pred
 * [nvox][c] against target [creal][nvox] (FP32), weight [nvox] (FP32, e.g.
 * 1 on fluid cells): loss = sum_v wt_v sum_k (p - t)^2 / (creal sum_v wt_v)
 * into loss_out[0] and the normaliser creal sum_v wt_v into loss_out[1]
 * (device FP32[2]), and, if dpred is not NULL, the gradient into dpred (BF16
 * [nvox][c], zero in padded channels).  workspace: cmnn_mse_workspace bytes. */
int cmnn_mse_workspace(size_t nvox, size_t* bytes);
int cmnn_mse(size_t nvox, const void* pred, int32_t c, int32_t creal, const float* target, const float* weight,
             float* loss_out, void* dpred, void* workspace, size_t workspace_bytes, void* hip_stream);

/* Global gradient-norm clipping, in place: norm = ||grad||_2 (FP64 sum of
 * FP32 partials), grad *= min(1, max_norm / norm); max_norm = 0 only
 * measures.  A non-finite norm zeroes grad.  norm_out (device, 2 floats)
 * receives {norm before clipping, scale applied}.  workspace:
 * cmnn_clip_grad_norm_workspace bytes. */
int cmnn_clip_grad_norm_workspace(size_t n, size_t* bytes);
int cmnn_clip_grad_norm(size_t n, float* grad, float max_norm, float* norm_out, void* workspace,
                        size_t workspace_bytes, void* hip_stream);

/* Adam with decoupled weight decay on FP32 master parameters (step >= 1). */
int cmnn_adam(size_t n, float* param, const float* grad, float* m, float* v, float lr, float beta1, float beta2,
              float eps, float weight_decay, int32_t step, void* hip_stream);

/* BF16 forward weights [27][cout][cin] and transposed [27][cin][cout] from
 * FP32 master weights [27][cout][cin]. */
int cmnn_pack_weights(const float* w, int32_t cin, int32_t cout, void* w_fwd, void* w_t, void* hip_stream);

/* cmnn_pack_weights for up to CMNN_PACK_MAX layers in one launch (bitwise the
 * same results).  jobs is a host array of n descriptors, read during the
 * call; EINVAL if any has a NULL pointer or a non-positive channel count. */
#define CMNN_PACK_MAX 32
typedef struct {
    const float* w; /* FP32 master weights [27][cout][cin] */
    void* w_fwd;    /* BF16 [27][cout][cin] */
    void* w_t;      /* BF16 [27][cin][cout] */
    int32_t cin, cout;
} cmnn_pack_job;
int cmnn_pack_weights_batch(int32_t n, const cmnn_pack_job* jobs, void* hip_stream);

/* FP32 planar [cs][nvox] -> BF16 NDHWC [nvox][c] (c >= cs, rest zero), and back. */
int cmnn_pack_channels(size_t nvox, const float* src, int32_t cs, void* dst, int32_t c, void* hip_stream);
int cmnn_unpack_channels(size_t nvox, const void* src, int32_t c, float* dst, int32_t cs, void* hip_stream);

/* Minibatch gathers from a data set held sample-major per plane, src FP32
 * [planes][nsrc][nvs] (nvs voxels per sample): output sample b is source
 * sample idx[b], idx a device int32 array of nsel entries.  An index outside
 * [0, nsrc) yields zeros (the call cannot report it).
 * cmnn_gather_samples: dst FP32 [np][nsel][nvs].
 * cmnn_gather_pack_channels: the gather of cs planes fused with
 * cmnn_pack_channels, dst BF16 NDHWC [nsel * nvs][c] (c >= cs, a multiple of
 * 8; channels from cs on zero). */
int cmnn_gather_samples(int32_t nsel, const int32_t* idx, size_t nvs, const float* src, int32_t nsrc, int32_t np,
                        float* dst, void* hip_stream);
int cmnn_gather_pack_channels(int32_t nsel, const int32_t* idx, size_t nvs, const float* src, int32_t nsrc,
                              int32_t cs, void* dst, int32_t c, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* CMNN_H */
