/*
 * cmlbm.h -- C ABI of the MI355X (gfx950) D3Q27 central-moment lattice
 * Boltzmann solver with Hermite-expanded external forcing.
 *
 * Method: De Rosis, Huang & Coreixas, "Three-dimensional central-moments-based
 * lattice Boltzmann method with external forcing", Phys. Rev. E (2019),
 * arXiv:1905.10182, Sec. II.  One time step is the five-step algorithm that
 * closes Sec. II: macroscopic variables with the half-force correction
 * (eq. "macroscopic"), the five pre-collision central moments
 * (eq. "pre_collision"), the nineteen non-zero post-collision central moments
 * (eq. "post_collision_central_moments_forcing"), reconstruction of the
 * post-collision populations (eq. "system"), and streaming (eq. "streaming").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns int: CMLBM_OK (0) or a negative CMLBM_E* code.
 *   No C++ exception crosses this boundary.  After an error the handle keeps
 *   a message readable with cmlbm_last_error().
 * - Cells: N = nbatch * nz * ny * nx.  Caller-visible per-cell arrays are
 *   x-fastest, [nbatch][nz][ny][nx]; vector fields are [3][N] (component
 *   slowest).  Population arrays are [27][N] in the velocity order of Sec. II.
 * - "dev" pointers are HIP device pointers, "host" pointers are host memory.
 * - Ownership: the two population buffers and the scratch buffer are
 *   allocated by the caller (sizes from cmlbm_required_bytes, 256-byte aligned)
 *   and borrowed for the life of the handle; the handle owns only host state.
 *   Output arrays are caller-owned.  A force field passed to cmlbm_set_force is
 *   borrowed until the next cmlbm_set_force or cmlbm_destroy.
 * - Streams: every device operation is enqueued on the hipStream_t passed as
 *   `hip_stream` (NULL = the null stream) and returns without waiting, except
 *   cmlbm_reduce, which waits for its own result.
 * - Not thread-safe per handle; distinct handles are independent.
 * - Storage: populations are stored shifted, s_i = f_i - w_i * rho0, in the
 *   storage type (FP16 stores 256 * s_i so small values stay normal); all
 *   arithmetic is FP32 for FP32/FP16/BF16 storage and FP64 for FP64 storage.
 *   16-bit conversions round to nearest even, or stochastically with
 *   CMLBM_FLAG_STOCHASTIC.
 * - Time: after cmlbm_init the state is the pre-collision f(x, 0); each step
 *   advances t by one.  Moments at time t use the force in effect.
 * - Walls: halfway bounce-back at rest on every axis flagged
 *   CMLBM_BOUNCEBACK and around solid nodes; a population that would leave
 *   through a wall or into a solid node returns to its node with the opposite
 *   velocity.  (The paper only names no-slip walls; this is the reading used.)
 */
#ifndef CMLBM_H
#define CMLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define CMLBM_OK 0
#define CMLBM_EINVAL (-1)    /* invalid argument; nothing was enqueued */
#define CMLBM_ENOMEM (-2)    /* a caller buffer is too small */
#define CMLBM_EHIP (-3)      /* a HIP runtime call or kernel launch failed */
#define CMLBM_EUNSTABLE (-4) /* cmlbm_reduce saw a non-finite rho or u */
#define CMLBM_ESTATE (-5)    /* call not valid in the handle's state */

/* population storage types */
#define CMLBM_FP64 0
#define CMLBM_FP32 1
#define CMLBM_FP16 2
#define CMLBM_BF16 3
/* Moment representation (FP32): instead of 27 populations a cell keeps the
 * nine numbers its post-collision state is made of -- rho - rho0, the
 * half-force-corrected u and the relaxed shear moments (1 - omega) k4..k8
 * (eq. "post_collision_central_moments_forcing") -- 36 bytes per cell per
 * buffer instead of 108.  The stored state is the post-collision state of
 * the current time t; a step rebuilds the neighbours' post-collision
 * populations in on-chip memory, streams and collides.  Restrictions:
 * periodic axes only, no solid mask, no stochastic rounding, no comparison
 * model; cmlbm_populations and cmlbm_load_populations are not available
 * (the pre-collision populations are not part of the state), and since the
 * first collision happens in cmlbm_init, set the force before cmlbm_init. */
#define CMLBM_MOM32 4

/* per-axis boundary kinds */
#define CMLBM_PERIODIC 0
#define CMLBM_BOUNCEBACK 1

/* force modes of cmlbm_set_force */
#define CMLBM_FORCE_NONE 0      /* F = 0 */
#define CMLBM_FORCE_UNIFORM 1   /* host_values[3]: one force density for every cell */
#define CMLBM_FORCE_BATCH 2     /* host_values[nbatch][3]: one force density per batch member */
#define CMLBM_FORCE_PROFILE_Y 3 /* host_values[ny][3]: force density depends on y only */
#define CMLBM_FORCE_FIELD 4     /* dev_field[3][N]: per-cell force density (borrowed) */

/* cmlbm_params.flags */
#define CMLBM_FLAG_SOLID 1u    /* reserve room for a solid-node mask (cmlbm_set_solid) */
#define CMLBM_FLAG_RESIDUAL 2u /* reserve room for the velocity snapshot of the residual */
#define CMLBM_FLAG_STOCHASTIC 4u /* 16-bit storage: stochastic (unbiased) instead of nearest-even rounding
                                    of the post-collision populations; bits from a counter-based hash
                                    of (cell, step), so runs are reproducible */
/* Comparison models of Sec. III (FP64 and FP32 storage only): the same
 * central-moment relaxation with a truncated equilibrium and/or forcing term.
 * Neither flag: the method itself (complete equilibrium and forcing, M1). */
#define CMLBM_FLAG_FORCE_GUO 8u  /* second-order (H1 + H2, Guo et al.) forcing term: M4 */
#define CMLBM_FLAG_EQ_SECOND 16u /* second-order equilibrium; with CMLBM_FLAG_FORCE_GUO: M5 */
#define CMLBM_FLAG_BGK 32u       /* stability control: every moment relaxes with omega (single relaxation
                                    time), with either both flags above (the classical BGK scheme with
                                    Guo forcing) or neither (the complete equilibrium and forcing) */
#define CMLBM_FLAG_FUSED_REDUCE 64u /* reserve room for cmlbm_step_reduce's per-wave partial sums (10 doubles
                                       per 64 x 1 or 64 x 2 cell row segment); population storage and the
                                       method's collision only (EINVAL with a comparison model or MOM32) */

/* cmlbm_reduce: `what` bits and the layout of one row of its output */
#define CMLBM_REDUCE_RESIDUAL 1u /* compare u with the last snapshot */
#define CMLBM_REDUCE_SNAPSHOT 2u /* store u as the new snapshot (after the comparison) */
#define CMLBM_RED_MASS 0         /* sum of rho over fluid cells */
#define CMLBM_RED_MOMX 1         /* sum over fluid cells of sum_i f_i c_i (no half-force term), x */
#define CMLBM_RED_MOMY 2
#define CMLBM_RED_MOMZ 3
#define CMLBM_RED_KE 4        /* sum of rho |u|^2 / 2, u half-force corrected */
#define CMLBM_RED_UMAX 5      /* max |u| */
#define CMLBM_RED_NONFINITE 6 /* number of fluid cells with a non-finite rho or u */
#define CMLBM_RED_FLUID 7     /* number of fluid cells */
#define CMLBM_RED_DU2 8       /* sum |u - u_snapshot|^2 (0 unless RESIDUAL) */
#define CMLBM_RED_U2 9        /* sum |u|^2 */
#define CMLBM_RED_RESIDUAL 10 /* sqrt(DU2 / U2) (0 unless RESIDUAL) */
#define CMLBM_NRED 11

typedef struct cmlbm_lattice cmlbm_lattice; /* opaque handle */

typedef struct {
    int32_t nx, ny, nz; /* lattice extent, each >= 1 (x is the fastest axis) */
    int32_t nbatch;     /* independent lattices advanced together, >= 1 */
    double tau;         /* relaxation time, > 1/2; omega = 1/tau, nu = (tau - 1/2)/3 (text after
                           eq. "macroscopic") */
    double rho0;        /* reference density of the storage shift and of rho = NULL in init, > 0 */
    int32_t storage;    /* CMLBM_FP64 | CMLBM_FP32 | CMLBM_FP16 | CMLBM_BF16 */
    int32_t wall[3];    /* x, y, z: CMLBM_PERIODIC or CMLBM_BOUNCEBACK */
    uint32_t flags;     /* CMLBM_FLAG_* */
} cmlbm_params;

/* Bytes the caller must provide for each of the two population buffers and for
 * the scratch buffer.  Pure host computation.  EINVAL on invalid params,
 * including one population over all cells (rows padded to 256 bytes, plus
 * 4 KiB) of 4 GiB or more: the link mask and the moment planes are addressed
 * with 32-bit offsets (FP32 up to ~1.07e9 cells, 16-bit up to ~2.1e9 cells).
 * Layout of a buffer: rows of nx values padded to 256 bytes, rows ordered
 * [nbatch][nz][ny]; population storage keeps the 27 population rows of one
 * lattice row together ([nbatch][nz][ny][27][row]), moment storage (nine
 * FP32 numbers per cell) keeps nine planes 4 KiB apart beyond their rows. */
int cmlbm_required_bytes(const cmlbm_params* params, size_t* pop_buffer_bytes, size_t* scratch_bytes);

/* Create a handle over caller-allocated device buffers (borrowed; each must be
 * 256-byte aligned and at least cmlbm_required_bytes large -- the sizes given
 * are checked).  Host-only: validates and records; enqueues nothing.  The
 * state is undefined until cmlbm_init or cmlbm_load_populations. */
int cmlbm_create(const cmlbm_params* params, void* pop_a, size_t pop_a_bytes, void* pop_b,
                 size_t pop_b_bytes, void* scratch, size_t scratch_bytes, cmlbm_lattice** out);

/* Mark solid nodes: dev_solid[N] (uint8, nonzero = solid) is read on the
 * stream and folded, together with the walls, into the handle's link mask.
 * Needs CMLBM_FLAG_SOLID.  NULL clears all solid nodes.  Call before
 * cmlbm_init / cmlbm_load_populations; changing geometry afterwards makes the
 * state undefined until the next init.  Solid nodes are not updated and
 * report rho = rho0, u = 0. */
int cmlbm_set_solid(cmlbm_lattice* lat, const uint8_t* dev_solid, void* hip_stream);

/* Set the external force density F (eq. "macroscopic", eq. "forcing" with F a
 * force density).  Table modes copy host_values on the stream; FIELD borrows
 * dev_field[3][N] of io_dtype, which must be CMLBM_FP64 for FP64 storage and
 * CMLBM_FP32 otherwise.  Takes effect for subsequent steps and moments. */
int cmlbm_set_force(cmlbm_lattice* lat, int mode, const double* host_values, const void* dev_field,
                    int io_dtype, void* hip_stream);

/* Initialise f(x, 0) = f^eq(rho(x), u(x)), the complete 27-Hermite
 * equilibrium of eq. "eq:truncation".  dev_rho[N] (NULL = rho0) and
 * dev_u[3][N] (NULL = 0) are of io_dtype CMLBM_FP64 or CMLBM_FP32.
 * Resets the step counter to 0. */
int cmlbm_init(cmlbm_lattice* lat, const void* dev_rho, const void* dev_u, int io_dtype, void* hip_stream);

/* Advance nsteps >= 0 time steps: each step is one fused launch doing the
 * pull-streaming gather (eq. "streaming"), collision in central-moment space
 * (eqs. "macroscopic", "pre_collision",
 * "post_collision_central_moments_forcing", "system") and the store. */
int cmlbm_step(cmlbm_lattice* lat, int32_t nsteps, void* hip_stream);

/* rho(x, t) into dev_rho[N] and u(x, t) = (sum f c + F/2)/rho into dev_u[3][N]
 * (either may be NULL), io_dtype CMLBM_FP64 or CMLBM_FP32.  With dev_u NULL
 * only the populations are read (the force enters the velocity alone); the
 * density is the same bit for bit as with dev_u given. */
int cmlbm_moments(cmlbm_lattice* lat, void* dev_rho, void* dev_u, int io_dtype, void* hip_stream);

/* Shan-Chen pseudo-potential interaction force of the static-droplet test
 * (Sec. III): field[a][n] = -G psi(x_n) sum_i w_i c_ia psi(x_n + c_i), with
 * psi = 1 - exp(-rho), from a density field in the cell order of
 * cmlbm_moments (dev_rho [N], dev_field [3][N], both FP64 for FP64 storage
 * and FP32 otherwise, device pointers).  Periodic lattices without solids
 * only.  To drive a step with it, register dev_field once with
 * cmlbm_set_force(CMLBM_FORCE_FIELD) and refresh it from cmlbm_moments before
 * every cmlbm_step.  The first call picks the kernel's z chunk for the
 * lattice's device (an occupancy query, no allocation); results do not
 * depend on it. */
int cmlbm_pseudopotential_force(cmlbm_lattice* lat, double G, const void* dev_rho, int io_dtype, void* dev_field,
                                void* hip_stream);

/* FP64 reductions over fluid cells, one row of CMLBM_NRED doubles per batch
 * member into host_out[nbatch][CMLBM_NRED] (layout CMLBM_RED_*).  The sums
 * use a fixed order, so results are bitwise reproducible.  RESIDUAL and
 * SNAPSHOT need CMLBM_FLAG_RESIDUAL; RESIDUAL without a prior snapshot is
 * ESTATE.  Waits for the stream.  Returns CMLBM_EUNSTABLE (output still
 * filled) if any fluid cell has a non-finite rho or u. */
int cmlbm_reduce(cmlbm_lattice* lat, uint32_t what, double* host_out, void* hip_stream);

/* One time step (cmlbm_step with nsteps = 1) whose kernel also forms the FP64
 * reductions of the state it reads, the state at the current step t (the
 * global sums that the per-step kinetic-energy and mass monitoring of the
 * method's validation needs), without a second pass over the populations.
 * Output as cmlbm_reduce without RESIDUAL (DU2 and RESIDUAL are 0).  The
 * per-cell density and velocity come from the step's own arithmetic (FP32 for
 * FP32 and 16-bit storage, FP64 for FP64) and are summed in FP64 in a fixed
 * order: bitwise reproducible, and within the FP32 rounding of the per-cell
 * values of cmlbm_reduce's sums.  The step runs in a separately compiled
 * kernel whose arithmetic may round differently in the last unit of the
 * stored format (measured: 99.97% or more of the populations bitwise equal to
 * cmlbm_step's, the rest one unit apart).  Needs CMLBM_FLAG_FUSED_REDUCE
 * (ESTATE otherwise).  The step is taken in every case; waits for the stream;
 * returns CMLBM_EUNSTABLE (output filled, step taken) if a fluid cell of the
 * state at t has a non-finite rho or u. */
int cmlbm_step_reduce(cmlbm_lattice* lat, double* host_out, void* hip_stream);

/* Export the pre-collision populations f_i(x, t) (unshifted, FP64) into
 * dev_out[27][N], paper order.  Solid cells are written as 0. */
int cmlbm_populations(cmlbm_lattice* lat, double* dev_out, void* hip_stream);

/* Import pre-collision populations dev_in[27][N] (FP64, unshifted, paper
 * order) as the state at the current step counter (checkpoint restore). */
int cmlbm_load_populations(cmlbm_lattice* lat, const double* dev_in, void* hip_stream);

/* Bitwise checkpoint: copy the state exactly as stored (shifted populations in
 * the storage type, internal padded layout; pop_buffer_bytes of
 * cmlbm_required_bytes) into dev_blob.  The blob is opaque and restores only
 * into a handle created with identical params.  Save the step counter with
 * cmlbm_get_time.  ENOMEM if blob_bytes is too small. */
int cmlbm_save_state(cmlbm_lattice* lat, void* dev_blob, size_t blob_bytes, void* hip_stream);
/* Restore a blob written by cmlbm_save_state as the current state (the step
 * counter is left unchanged; set it with cmlbm_set_time). */
int cmlbm_restore_state(cmlbm_lattice* lat, const void* dev_blob, size_t blob_bytes, void* hip_stream);

/* Step counter (number of steps since init). */
int cmlbm_get_time(const cmlbm_lattice* lat, int64_t* t);
/* Set the step counter (checkpoint restore). */
int cmlbm_set_time(cmlbm_lattice* lat, int64_t t);

/* Release the handle (the borrowed buffers are untouched).  NULL is OK. */
int cmlbm_destroy(cmlbm_lattice* lat);

/* Message of the last error on this handle ("" if none); never NULL. */
const char* cmlbm_last_error(const cmlbm_lattice* lat);
/* Static name of a status code. */
const char* cmlbm_status_string(int status);

/* Measurement aid, not part of the method: copy `bytes` (a multiple of 16)
 * from dev_src to dev_dst (16-byte aligned, not overlapping) with 16-byte
 * non-temporal loads and stores, four loads in flight per thread, a
 * grid-stride loop over at most 1024 workgroups per 64 MiB.  Its rate is the practical read + write bandwidth of the device,
 * the ceiling that the HBM-bound steps are compared with.  EINVAL on NULL,
 * misaligned or odd-sized arguments; nothing is enqueued then. */
int cmlbm_device_copy(void* dev_dst, const void* dev_src, size_t bytes, void* hip_stream);

/* Measurement aid, not part of the method: the FP32 step's memory traffic
 * without its arithmetic.  For every plane p < planes and cell c < cells,
 * dev_dst[p * plane_stride + c] = dev_src[p * plane_stride + c] (FP32
 * elements; both device pointers 4-byte aligned, the two spans not
 * overlapping), one cell per lane in 1024-thread workgroups: each lane loads
 * its cell of every plane, then stores them non-temporally -- the access
 * pattern of the FP32 population step (planes = 27) or of the moment
 * storage's nine numbers (planes = 9) with no collision.  Its rate is the
 * ceiling of that pattern.  EINVAL on NULL or misaligned pointers, planes
 * other than 9 or 27, cells < 1, plane_stride < cells, or overlapping spans;
 * nothing is enqueued then. */
int cmlbm_plane_copy(void* dev_dst, const void* dev_src, int32_t planes, int64_t cells, int64_t plane_stride,
                     void* hip_stream);

/* Measurement aid, not part of the method: the FP32 population step's memory
 * traffic in its row-block layout, without the arithmetic.  For every lattice
 * row r < rows, population p < 27 and cell x < row_len, the FP32 element at
 * (r * 27 + p) * row_len + x is copied from dev_src to dev_dst (both device
 * pointers 4-byte aligned, the two spans of rows * 27 * row_len elements not
 * overlapping), one cell per lane in 1024-thread workgroups: each lane loads
 * its 27 values, then stores them non-temporally.  EINVAL on NULL or
 * misaligned pointers, rows < 1, row_len < 1, spans of 2^40 bytes or more,
 * or overlapping spans; nothing is enqueued then. */
int cmlbm_row_block_copy(void* dev_dst, const void* dev_src, int64_t rows, int32_t row_len, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* CMLBM_H */
