/*
 * cmlbm2d.h -- C ABI of the MI355X (gfx950) D2Q9 central-moment lattice
 * Boltzmann solver with Hermite forcing: the two-dimensional model of App. B
 * of De Rosis, Huang & Coreixas, "Three-dimensional central-moments-based
 * lattice Boltzmann method with external forcing", Phys. Rev. E (2019),
 * arXiv:1905.10182.
 *
 * One time step: density and half-force-corrected velocity, the pre-collision
 * central moments k4 and k5 on the shifted basis T-bar of App. B, the nine
 * printed post-collision central moments (k0* = rho, k1,2* = F/2,
 * k3* = 2 rho cs^2, k4,5* = (1 - omega) k4,5, k6* = Fy cs^2/2,
 * k7* = Fx cs^2/2, k8* = rho cs^4), reconstruction of the post-collision
 * populations (eq. "system2") and streaming, fused into one kernel.
 *
 * Conventions
 * -----------
 * - Every function returns int: CMLBM2D_OK (0) or a negative CMLBM2D_E* code;
 *   no C++ exception crosses this boundary.  After an error the handle keeps a
 *   message readable with cmlbm2d_last_error().
 * - Cells: N = ny * nx, x fastest ([ny][nx]); vector fields are [2][N]
 *   (component slowest); population arrays are [9][N] in the velocity order of
 *   App. B.  Both axes are periodic.
 * - "dev" pointers are HIP device pointers, "host" pointers host memory.
 * - Ownership: the two population buffers are allocated by the caller (size
 *   from cmlbm2d_required_bytes, 256-byte aligned) and borrowed for the life of
 *   the handle; the handle owns only host state.  Output arrays are
 *   caller-owned.  A force field passed to cmlbm2d_set_force is borrowed until
 *   the next cmlbm2d_set_force or cmlbm2d_destroy.  No entry point allocates
 *   device memory.
 * - Streams: every device operation is enqueued on the hipStream_t passed as
 *   `hip_stream` (NULL = the null stream) and returns without waiting.
 * - Not thread-safe per handle; distinct handles are independent.
 * - Storage: populations are stored shifted, s_i = f_i - w_i rho0, in the
 *   storage type (FP16 stores 256 * s_i); arithmetic is FP64 for FP64 storage
 *   and FP32 otherwise; 16-bit conversions round to nearest even.
 * - Time: after cmlbm2d_init the state is the pre-collision f(x, 0); each step
 *   advances t by one.  Moments at time t use the force in effect.
 */
#ifndef CMLBM2D_H
#define CMLBM2D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CMLBM2D_OK 0
#define CMLBM2D_EINVAL (-1) /* invalid argument; nothing was enqueued */
#define CMLBM2D_ENOMEM (-2) /* a caller buffer is too small */
#define CMLBM2D_EHIP (-3)   /* a HIP runtime call or kernel launch failed */
#define CMLBM2D_ESTATE (-5) /* call not valid in the handle's state */

/* population storage types */
#define CMLBM2D_FP64 0
#define CMLBM2D_FP32 1
#define CMLBM2D_FP16 2
#define CMLBM2D_BF16 3

/* force modes of cmlbm2d_set_force */
#define CMLBM2D_FORCE_NONE 0    /* F = 0 */
#define CMLBM2D_FORCE_UNIFORM 1 /* host_values[2]: one force density for every cell */
#define CMLBM2D_FORCE_FIELD 2   /* dev_field[2][N]: per-cell force density (borrowed) */

typedef struct cmlbm2d_lattice cmlbm2d_lattice; /* opaque handle */

typedef struct {
    int32_t nx, ny;  /* lattice extent, each >= 1 (x is the fastest axis) */
    double tau;      /* relaxation time of k4, k5, > 1/2: omega = 1/tau, nu = (tau - 1/2)/3 */
    double rho0;     /* reference density of the storage shift and of rho = NULL in init, > 0 */
    int32_t storage; /* CMLBM2D_FP64 | CMLBM2D_FP32 | CMLBM2D_FP16 | CMLBM2D_BF16 */
    uint32_t flags;  /* reserved, must be 0 */
} cmlbm2d_params;

/* Bytes the caller must provide for each of the two population buffers.
 * Every population is stored in rows of nx values padded to 256 bytes; FP32
 * and 16-bit storage keep the nine population rows of one lattice row
 * together ([ny][9][row]), FP64 keeps nine planes of ny rows, 4 KiB apart
 * beyond that.  Pure host computation.
 * EINVAL on invalid params, including one population over all cells of
 * 4 GiB or more (32-bit byte offsets). */
int cmlbm2d_required_bytes(const cmlbm2d_params* params, size_t* pop_buffer_bytes);

/* Create a handle over two caller-allocated device buffers (borrowed, each
 * 256-byte aligned and at least cmlbm2d_required_bytes large; the sizes given
 * are checked, ENOMEM if too small).  Host-only.  The state is undefined until
 * cmlbm2d_init or cmlbm2d_load_populations. */
int cmlbm2d_create(const cmlbm2d_params* params, void* pop_a, size_t pop_a_bytes, void* pop_b, size_t pop_b_bytes,
                   cmlbm2d_lattice** out);

/* Set the force density F of App. B (F enters the velocity with weight 1/2 and
 * the post-collision moments k1, k2, k6, k7).  UNIFORM reads host_values[2]
 * (kept in the handle); FIELD borrows dev_field[2][N] of io_dtype, which must
 * be CMLBM2D_FP64 for FP64 storage and CMLBM2D_FP32 otherwise.  Takes effect
 * for subsequent steps and moments.  Host-only apart from the borrow. */
int cmlbm2d_set_force(cmlbm2d_lattice* lat, int mode, const double* host_values, const void* dev_field, int io_dtype,
                      void* hip_stream);

/* Initialise f(x, 0) = f^eq(rho(x), u(x)), the complete equilibrium of
 * eq. "eq:D2Q9".  dev_rho[N] (NULL = rho0) and dev_u[2][N] (NULL = 0) of
 * io_dtype CMLBM2D_FP64 or CMLBM2D_FP32.  Resets the step counter to 0. */
int cmlbm2d_init(cmlbm2d_lattice* lat, const void* dev_rho, const void* dev_u, int io_dtype, void* hip_stream);

/* Advance nsteps >= 0 time steps, one fused launch each: pull streaming,
 * central-moment collision with forcing, store. */
int cmlbm2d_step(cmlbm2d_lattice* lat, int32_t nsteps, void* hip_stream);

/* rho(x, t) into dev_rho[N] and u = (sum f c + F/2)/rho into dev_u[2][N]
 * (either may be NULL), io_dtype CMLBM2D_FP64 or CMLBM2D_FP32. */
int cmlbm2d_moments(cmlbm2d_lattice* lat, void* dev_rho, void* dev_u, int io_dtype, void* hip_stream);

/* Export the pre-collision populations f_i(x, t) (unshifted, FP64) into
 * dev_out[9][N], App. B order. */
int cmlbm2d_populations(cmlbm2d_lattice* lat, double* dev_out, void* hip_stream);

/* Import pre-collision populations dev_in[9][N] (FP64, unshifted, App. B
 * order) as the state at the current step counter. */
int cmlbm2d_load_populations(cmlbm2d_lattice* lat, const double* dev_in, void* hip_stream);

/* Step counter (number of steps since init). */
int cmlbm2d_get_time(const cmlbm2d_lattice* lat, int64_t* t);

/* Release the handle (the borrowed buffers are untouched).  NULL is OK. */
int cmlbm2d_destroy(cmlbm2d_lattice* lat);

/* Message of the last error on this handle ("" if none); never NULL. */
const char* cmlbm2d_last_error(const cmlbm2d_lattice* lat);
/* Static name of a status code. */
const char* cmlbm2d_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif /* CMLBM2D_H */
