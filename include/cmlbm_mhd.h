/*
 * cmlbm_mhd.h -- C ABI of the MI355X (gfx950) magnetic-field lattice of App. C
 * of De Rosis, Huang & Coreixas, "Three-dimensional central-moments-based
 * lattice Boltzmann method with external forcing", Phys. Rev. E (2019),
 * arXiv:1905.10182, and of the Lorentz force F = j x b that couples it to the
 * fluid solver of cmlbm.h (Sec. III: Hartmann flow, Orszag-Tang vortex).
 *
 * The magnetic field b is carried by vector-valued populations h_l (three
 * components each) on the D3Q7 velocity set (rest, +-x, +-y, +-z, weights
 * 1/4 and 1/8, cs^2 = 1/4), relaxed with one rate omega_m = 1/tau_m towards
 * h^eq_la = w_l [b_a + 4 xi_lb (u_b b_a - b_b u_a)] and streamed along xi_l;
 * b = sum_l h_l; the resistivity is eta = (tau_m - 1/2) / 4.
 *
 * The current j = curl b comes either from the populations -- the
 * pre-collision non-equilibrium electric tensor, j_c = -eps_cba
 * (Lambda - Lambda^eq)_ba / (tau_m cs^2) with Lambda_ba = sum_l xi_lb h_la,
 * Lambda^eq_ba = u_b b_a - b_b u_a (first-order Chapman-Enskog; it omits the
 * time derivative of Lambda^eq, a relative error of order |u|^2/cs^2 and
 * |b|^2/cs^2) -- or from second-order central differences of b.
 *
 * A coupled step (as the tests and studies drive it): read the fluid velocity
 * with cmlbm_moments, cmlbm_mhd_fields writes F = j x b into the fluid's
 * registered force field (cmlbm_set_force FIELD), read the fluid velocity
 * again, cmlbm_mhd_step with it, then cmlbm_step.
 *
 * Conventions
 * -----------
 * - Every function returns CMLBM_MHD_OK (0) or a negative CMLBM_MHD_E* code;
 *   after an error the handle keeps a message (cmlbm_mhd_last_error).
 * - Cells: N = nz * ny * nx, x fastest; vector fields are [3][N] (component
 *   slowest), the layout of cmlbm_moments and cmlbm_set_force FIELD for one
 *   batch member.  Population arrays are [7][3][N] (velocity, component, cell).
 *   Axes are periodic or carry walls (CMLBM_MHD_WALL).
 * - The two population buffers are caller-allocated (size from
 *   cmlbm_mhd_required_bytes, 256-byte aligned) and borrowed for the life of
 *   the handle; every other array is caller-owned.  No entry point allocates
 *   device memory.
 * - Field arrays (b, u, j, F) are FP64 for FP64 storage and FP32 for FP32
 *   storage, device pointers.
 * - Every device operation is enqueued on the hipStream_t `hip_stream`
 *   (NULL = the null stream) and returns without waiting.  Not thread-safe
 *   per handle.
 */
#ifndef CMLBM_MHD_H
#define CMLBM_MHD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CMLBM_MHD_OK 0
#define CMLBM_MHD_EINVAL (-1) /* invalid argument; nothing was enqueued */
#define CMLBM_MHD_ENOMEM (-2) /* a caller buffer is too small */
#define CMLBM_MHD_EHIP (-3)   /* a HIP runtime call or kernel launch failed */
#define CMLBM_MHD_ESTATE (-5) /* call not valid in the handle's state */

#define CMLBM_MHD_FP64 0
#define CMLBM_MHD_FP32 1

/* per-axis boundary kinds */
#define CMLBM_MHD_PERIODIC 0
#define CMLBM_MHD_WALL 1 /* walls halfway outside the first and last node, where b takes the value set by
                            cmlbm_mhd_set_wall_field (the Hartmann test); use the fluid's CMLBM_BOUNCEBACK
                            on the same axes */

/* current kinds of cmlbm_mhd_fields */
#define CMLBM_MHD_CURRENT_POPULATIONS 0 /* from the non-equilibrium electric tensor */
#define CMLBM_MHD_CURRENT_STENCIL 1     /* central differences of b (needs dev_b) */

typedef struct cmlbm_mhd_lattice cmlbm_mhd_lattice; /* opaque handle */

typedef struct {
    int32_t nx, ny, nz; /* lattice extent, each >= 1 (>= 2 on a wall axis) */
    double tau_m;       /* magnetic relaxation time, > 1/2: eta = (tau_m - 1/2) / 4 */
    int32_t storage;    /* CMLBM_MHD_FP64 | CMLBM_MHD_FP32 */
    int32_t wall[3];    /* x, y, z: CMLBM_MHD_PERIODIC or CMLBM_MHD_WALL */
    uint32_t flags;     /* reserved, must be 0 */
} cmlbm_mhd_params;

/* Bytes of each of the two population buffers (21 planes, rows padded to
 * 256 bytes).  Host-only.  EINVAL on invalid params, including a plane of
 * 4 GiB or more. */
int cmlbm_mhd_required_bytes(const cmlbm_mhd_params* params, size_t* pop_buffer_bytes);

/* Create a handle over two caller-allocated device buffers (borrowed; 256-byte
 * aligned, sizes checked: ENOMEM if too small).  Host-only. */
int cmlbm_mhd_create(const cmlbm_mhd_params* params, void* pop_a, size_t pop_a_bytes, void* pop_b,
                     size_t pop_b_bytes, cmlbm_mhd_lattice** out);

/* The field b_w (host_b_wall[3]) imposed at every wall: a population that
 * would stream into a wall returns as h_opp(x, t+1) = -h*_l(x, t) + 2 w_l b_w
 * (anti-bounce-back: the Dirichlet value sits at the half-way wall), and the
 * stencil current takes the ghost value 2 b_w - b beyond it.  The paper
 * assigns the missing wall population from b = sum h instead (App. C); this
 * halfway form matches the fluid's halfway bounce-back walls.  Host-only;
 * default 0.  Set it before cmlbm_mhd_init. */
int cmlbm_mhd_set_wall_field(cmlbm_mhd_lattice* lat, const double* host_b_wall);

/* A uniform force density host_f0[3] added to every Lorentz force that
 * cmlbm_mhd_fields writes (F = j x b + f0: the driving force of a channel such
 * as the Hartmann test).  Host-only; default 0. */
int cmlbm_mhd_set_body_force(cmlbm_mhd_lattice* lat, const double* host_f0);

/* h = h^eq(b, u) from dev_b[3][N] (required) and dev_u[3][N] (NULL = rest). */
int cmlbm_mhd_init(cmlbm_mhd_lattice* lat, const void* dev_b, const void* dev_u, void* hip_stream);

/* From the current populations: b into dev_b[3][N], j into dev_j[3][N] and
 * the Lorentz force density F = j x b (+ f0) into dev_F[3][N] (each may be NULL;
 * the STENCIL current needs dev_b, which it reads back).  dev_u[3][N] is the
 * fluid velocity for Lambda^eq (POPULATIONS current only; NULL = rest). */
int cmlbm_mhd_fields(cmlbm_mhd_lattice* lat, const void* dev_u, int current, void* dev_b, void* dev_j, void* dev_F,
                     void* hip_stream);

/* One step, one launch: collision towards h^eq(b, u) with the fluid velocity
 * dev_u[3][N] (NULL = rest), then streaming (pull form). */
int cmlbm_mhd_step(cmlbm_mhd_lattice* lat, const void* dev_u, void* hip_stream);

/* Export the pre-collision populations (FP64) into dev_out[7][3][N]. */
int cmlbm_mhd_populations(cmlbm_mhd_lattice* lat, double* dev_out, void* hip_stream);

/* Import pre-collision populations dev_in[7][3][N] (FP64). */
int cmlbm_mhd_load_populations(cmlbm_mhd_lattice* lat, const double* dev_in, void* hip_stream);

/* Steps since init. */
int cmlbm_mhd_get_time(const cmlbm_mhd_lattice* lat, int64_t* t);

/* Release the handle (NULL is OK). */
int cmlbm_mhd_destroy(cmlbm_mhd_lattice* lat);

/* Last error message ("" if none; never NULL) and the name of a status code. */
const char* cmlbm_mhd_last_error(const cmlbm_mhd_lattice* lat);
const char* cmlbm_mhd_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif /* CMLBM_MHD_H */
