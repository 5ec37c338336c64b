/*
 * Plain FP64 CPU oracle of the D3Q27 central-moment lattice Boltzmann method
 * with Hermite-expanded external forcing of De Rosis, Huang & Coreixas,
 * "Three-dimensional central-moments-based lattice Boltzmann method with
 * external forcing: a consistent, concise and universal formulation",
 * Phys. Rev. E (2019), arXiv:1905.10182.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent checker of the HIP
 * solver: only the tests, the smoke check and the cpu_baseline leg of the
 * benchmark may load it.  The GPU library never links, calls or includes it,
 * and the two share no code, tables or constants.
 *
 * Everything is unshifted FP64 (or 80-bit, see `real` below) (the textbook populations f_i, not f_i - w_i rho0).
 * Two collision routes are provided:
 *   - "literal" (orc_collide_literal): the matrix algebra of Sec. II as printed:
 *     build the central-moment basis T-bar (eq. "basis"), k = T^T f,
 *     k^eq = T^T f^eq with f^eq from the complete 27-Hermite equilibrium
 *     (eq. "eq:truncation"), R = T^T F with F from the complete Hermite
 *     forcing (eq. "forcing"), k* = (I - L) k + L k^eq + (I - L/2) R with the
 *     relaxation matrix L of eq. "eq:relaxationMatrix", then solve
 *     T^T f* = k* (eq. "system") by Gaussian elimination.
 *   - "closed" (orc_collide_closed): the five-step algorithm at the end of
 *     Sec. II: macroscopic variables (eq. "macroscopic"), the five pre-collision
 *     central moments (eq. "pre_collision"), the nineteen non-zero post-collision
 *     central moments (eq. "post_collision_central_moments_forcing"), and the
 *     reconstruction T^T f* = k* done with the fast central-moment transform the
 *     paper names at the end of its force-free discussion: the basis is mapped
 *     to monomial central moments, then three one-dimensional inverse transforms
 *     on the velocity set {-1, 0, +1} are applied along z, y and x.
 *
 * Readings of passages the paper leaves open (each is also listed in the
 * repository's design notes):
 *   R1  F is a force density everywhere.  Eq. "forcing" carries a rho prefactor,
 *       but its central moments are printed as R_1 = F_x (eq. "force_cms_sixth")
 *       and rho u = sum f c + F/2 (eq. "macroscopic"); these agree only if the
 *       forcing term is F . grad_u f^eq evaluated at rho = 1, i.e. eq. "forcing"
 *       with the rho prefactor dropped.  orc_forcing implements that reading.
 *   R2  The velocity u used in the shifted velocities, k^eq and R is the
 *       half-force-corrected velocity of eq. "macroscopic".
 *   R3  Walls are halfway bounce-back at rest: a population that would stream
 *       into a wall or a solid node returns to its node of origin with the
 *       opposite velocity.  The paper only names no-slip walls.
 *   R4  The initial state is f_i = f_i^eq(rho(x), u(x)) of eq. "eq:truncation".
 *
 * Lattice layout: population i of cell n lives at f[i*N + n], N = nb*nz*ny*nx,
 * n = ((b*nz + z)*ny + y)*nx + x; velocity order of Sec. II.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 27

/* Scalar type.  The default build is FP64; the extended build (-DORC_EXTENDED)
 * runs the same arithmetic in x87 80-bit long double and serves as the
 * reference where a bar is tighter than FP64 rounding of the unshifted form. */
#ifdef ORC_EXTENDED
typedef long double real;
#define RFABS fabsl
#else
typedef double real;
#define RFABS fabs
#endif

/* D3Q27 velocity components, in the order printed at the start of Sec. II. */
static const int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
static const int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, 1, -1, -1, 1, 1, -1, -1};
static const int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1};

/* Lattice weights listed after eq. "eq:truncation". */
static real weight(int i)
{
    if (i == 0) return (real)8 / 27;
    if (i <= 6) return (real)2 / 27;
    if (i <= 18) return (real)1 / 54;
    return (real)1 / 216;
}

static const real CS2 = (real)1 / 3; /* c_s^2, c_s = 1/sqrt(3) */

static int opposite(int i)
{
    for (int j = 0; j < Q; ++j)
        if (CX[j] == -CX[i] && CY[j] == -CY[i] && CZ[j] == -CZ[i]) return j;
    return -1;
}

void orc_lattice_constants(int* cx, int* cy, int* cz, real* w, int* opp)
{
    for (int i = 0; i < Q; ++i) {
        cx[i] = CX[i];
        cy[i] = CY[i];
        cz[i] = CZ[i];
        w[i] = weight(i);
        opp[i] = opposite(i);
    }
}

/* One-dimensional discrete Hermite polynomials of App. A: H^(0) = 1,
 * H^(1) = c, H^(2) = c^2 - c_s^2.  3D tensors are their products. */
static real herm1d(int order, real c)
{
    if (order == 0) return 1.0;
    if (order == 1) return c;
    return c * c - CS2;
}

typedef struct {
    /* H^(n) tensors of App. A for one lattice velocity, named by index string */
    real x, y, z;
    real xx, yy, zz, xy, xz, yz;
    real xxy, xxz, xyy, xzz, yzz, yyz, xyz;
    real xxyy, xxzz, yyzz, xyzz, xyyz, xxyz;
    real xxyzz, xxyyz, xyyzz;
    real xxyyzz;
} hermite_set;

static void hermite_tensors(int i, hermite_set* h)
{
    const real cx = CX[i], cy = CY[i], cz = CZ[i];
    const real Hx = herm1d(1, cx), Hy = herm1d(1, cy), Hz = herm1d(1, cz);
    const real Hxx = herm1d(2, cx), Hyy = herm1d(2, cy), Hzz = herm1d(2, cz);
    h->x = Hx;
    h->y = Hy;
    h->z = Hz;
    h->xx = Hxx;
    h->yy = Hyy;
    h->zz = Hzz;
    h->xy = Hx * Hy;
    h->xz = Hx * Hz;
    h->yz = Hy * Hz;
    h->xxy = Hxx * Hy;
    h->xxz = Hxx * Hz;
    h->yyz = Hyy * Hz;
    h->xyy = Hx * Hyy;
    h->xzz = Hx * Hzz;
    h->yzz = Hy * Hzz;
    h->xyz = Hx * Hy * Hz;
    h->xxyy = Hxx * Hyy;
    h->xxzz = Hxx * Hzz;
    h->yyzz = Hyy * Hzz;
    h->xxyz = Hxx * Hy * Hz;
    h->xyyz = Hx * Hyy * Hz;
    h->xyzz = Hx * Hy * Hzz;
    h->xxyyz = Hxx * Hyy * Hz;
    h->xxyzz = Hxx * Hy * Hzz;
    h->xyyzz = Hx * Hyy * Hzz;
    h->xxyyzz = Hxx * Hyy * Hzz;
}

/* 27-Hermite equilibrium, eq. "eq:truncation", term by term, keeping the
 * Hermite tensors up to the given order (2: the classical second-order
 * equilibrium the text mentions; 6: the complete expansion). */
void orc_feq_order(real rho, const real u[3], int order, real out[Q])
{
    const real ux = u[0], uy = u[1], uz = u[2];
    const real cs4 = CS2 * CS2, cs6 = cs4 * CS2, cs8 = cs4 * cs4, cs10 = cs8 * CS2, cs12 = cs6 * cs6;
    for (int i = 0; i < Q; ++i) {
        hermite_set H;
        hermite_tensors(i, &H);
        real s = 1.0;
        s += (CX[i] * ux + CY[i] * uy + CZ[i] * uz) / CS2;
        s += (H.xx * ux * ux + H.yy * uy * uy + H.zz * uz * uz +
              2.0 * (H.xy * ux * uy + H.xz * ux * uz + H.yz * uy * uz)) /
             (2.0 * cs4);
        if (order < 3) {
            out[i] = weight(i) * rho * s;
            continue;
        }
        s += (H.xxy * ux * ux * uy + H.xxz * ux * ux * uz + H.xyy * ux * uy * uy + H.xzz * ux * uz * uz +
              H.yzz * uy * uz * uz + H.yyz * uy * uy * uz + 2.0 * H.xyz * ux * uy * uz) /
             (2.0 * cs6);
        s += (H.xxyy * ux * ux * uy * uy + H.xxzz * ux * ux * uz * uz + H.yyzz * uy * uy * uz * uz +
              2.0 * (H.xyzz * ux * uy * uz * uz + H.xyyz * ux * uy * uy * uz + H.xxyz * ux * ux * uy * uz)) /
             (4.0 * cs8);
        s += (H.xxyzz * ux * ux * uy * uz * uz + H.xxyyz * ux * ux * uy * uy * uz +
              H.xyyzz * ux * uy * uy * uz * uz) /
             (4.0 * cs10);
        s += H.xxyyzz * ux * ux * uy * uy * uz * uz / (8.0 * cs12);
        out[i] = weight(i) * rho * s;
    }
}

/* Complete 27-Hermite equilibrium. */
void orc_feq(real rho, const real u[3], real out[Q]) { orc_feq_order(rho, u, 6, out); }

/* Hermite forcing term, eq. "forcing", term by term, under reading R1 (F is a
 * force density, so the rho prefactor of the printed formula is 1), keeping
 * the Hermite tensors up to the given order (2: H1 + H2, the Guo form the
 * text names; 6: the complete expansion). */
void orc_forcing_order(const real u[3], const real F[3], int order, real out[Q])
{
    const real ux = u[0], uy = u[1], uz = u[2];
    const real Fx = F[0], Fy = F[1], Fz = F[2];
    const real cs4 = CS2 * CS2, cs6 = cs4 * CS2, cs8 = cs4 * cs4, cs10 = cs8 * CS2, cs12 = cs6 * cs6;
    for (int i = 0; i < Q; ++i) {
        hermite_set H;
        hermite_tensors(i, &H);
        real s = (Fx * CX[i] + Fy * CY[i] + Fz * CZ[i]) / CS2;
        s += (H.xx * (2 * ux * Fx) + H.yy * (2 * uy * Fy) + H.zz * (2 * uz * Fz) +
              2 * H.xy * (ux * Fy + uy * Fx) + 2 * H.xz * (ux * Fz + uz * Fx) + 2 * H.yz * (uy * Fz + uz * Fy)) /
             (2 * cs4);
        if (order < 3) {
            out[i] = weight(i) * s;
            continue;
        }
        s += (H.xxy * (2 * ux * uy * Fx + ux * ux * Fy) + H.xxz * (2 * ux * uz * Fx + ux * ux * Fz) +
              H.xyy * (2 * ux * uy * Fy + uy * uy * Fx) + H.xzz * (2 * ux * uz * Fz + uz * uz * Fx) +
              H.yzz * (2 * uy * uz * Fz + uz * uz * Fy) + H.yyz * (2 * uy * uz * Fy + uy * uy * Fz) +
              2 * H.xyz * (ux * uy * Fz + ux * Fy * uz + Fx * uy * uz)) /
             (2 * cs6);
        s += (H.xxyy * (2 * ux * ux * uy * Fy + 2 * ux * uy * uy * Fx) +
              H.xxzz * (2 * ux * ux * uz * Fz + 2 * ux * uz * uz * Fx) +
              H.yyzz * (2 * uy * uy * uz * Fz + 2 * uy * uz * uz * Fy) +
              2 * H.xyzz * (2 * ux * uy * uz * Fz + ux * Fy * uz * uz + Fx * uy * uz * uz) +
              2 * H.xyyz * (2 * ux * uy * uz * Fy + ux * uy * uy * Fz + Fx * uy * uy * uz) +
              2 * H.xxyz * (2 * ux * uy * uz * Fx + uy * ux * ux * Fz + ux * ux * uz * Fy)) /
             (4 * cs8);
        s += (H.xxyyz * (2 * ux * uy * uy * uz * Fx + 2 * ux * ux * uy * uz * Fy + ux * ux * uy * uy * Fz) +
              H.xxyzz * (2 * ux * uy * uz * uz * Fx + ux * ux * uz * uz * Fy + 2 * ux * ux * uy * uz * Fz) +
              H.xyyzz * (uy * uy * uz * uz * Fx + 2 * ux * uy * uz * uz * Fy + 2 * ux * uy * uy * uz * Fz)) /
             (4 * cs10);
        s += H.xxyyzz * (2 * ux * uy * uy * uz * uz * Fx + 2 * ux * ux * uy * uz * uz * Fy +
                         2 * ux * ux * uy * uy * uz * Fz) /
             (8 * cs12);
        out[i] = weight(i) * s;
    }
}

/* Complete Hermite forcing term. */
void orc_forcing(const real u[3], const real F[3], real out[Q]) { orc_forcing_order(u, F, 6, out); }

/* The 27 basis polynomials of eq. "basis" evaluated at one shifted velocity. */
static void basis_polys(real X, real Y, real Z, real T[Q])
{
    const real X2 = X * X, Y2 = Y * Y, Z2 = Z * Z;
    T[0] = 1.0;
    T[1] = X;
    T[2] = Y;
    T[3] = Z;
    T[4] = X * Y;
    T[5] = X * Z;
    T[6] = Y * Z;
    T[7] = X2 - Y2;
    T[8] = X2 - Z2;
    T[9] = X2 + Y2 + Z2;
    T[10] = X * Y2 + X * Z2;
    T[11] = X2 * Y + Y * Z2;
    T[12] = X2 * Z + Y2 * Z;
    T[13] = X * Y2 - X * Z2;
    T[14] = X2 * Y - Y * Z2;
    T[15] = X2 * Z - Y2 * Z;
    T[16] = X * Y * Z;
    T[17] = X2 * Y2 + X2 * Z2 + Y2 * Z2;
    T[18] = X2 * Y2 + X2 * Z2 - Y2 * Z2;
    T[19] = X2 * Y2 - X2 * Z2;
    T[20] = X2 * Y * Z;
    T[21] = X * Y2 * Z;
    T[22] = X * Y * Z2;
    T[23] = X * Y2 * Z2;
    T[24] = X2 * Y * Z2;
    T[25] = X2 * Y2 * Z;
    T[26] = X2 * Y2 * Z2;
}

/* Transformation matrix T-bar: column j is the basis polynomial T_j evaluated at
 * the shifted velocities c-bar_i = c_i - u of eq. "central_directions".
 * Stored row-major: Tbar[i*27 + j] = T_j(c-bar_i). */
void orc_basis(const real u[3], real Tbar[Q * Q])
{
    for (int i = 0; i < Q; ++i) basis_polys(CX[i] - u[0], CY[i] - u[1], CZ[i] - u[2], &Tbar[i * Q]);
}

/* k = T^T f, i.e. k_j = sum_i T_j(c-bar_i) f_i. */
void orc_central_moments(const real u[3], const real f[Q], real k[Q])
{
    real T[Q * Q];
    orc_basis(u, T);
    for (int j = 0; j < Q; ++j) {
        real s = 0.0;
        for (int i = 0; i < Q; ++i) s += T[i * Q + j] * f[i];
        k[j] = s;
    }
}

/* Eq. "macroscopic": rho = sum f, rho u = sum f c + F/2. */
void orc_macroscopic(const real f[Q], const real F[3], real* rho, real u[3])
{
    real r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    for (int i = 0; i < Q; ++i) {
        r += f[i];
        jx += f[i] * CX[i];
        jy += f[i] * CY[i];
        jz += f[i] * CZ[i];
    }
    *rho = r;
    u[0] = (jx + 0.5 * F[0]) / r;
    u[1] = (jy + 0.5 * F[1]) / r;
    u[2] = (jz + 0.5 * F[2]) / r;
}

/* Solve A x = b for a dense n x n system by Gaussian elimination with partial
 * pivoting (A row-major, overwritten).  Returns 0 on success, -1 if singular. */
static int dense_solve(int n, real* A, real* b, real* x)
{
    for (int c = 0; c < n; ++c) {
        int piv = c;
        real best = RFABS(A[c * n + c]);
        for (int r = c + 1; r < n; ++r)
            if (RFABS(A[r * n + c]) > best) {
                best = RFABS(A[r * n + c]);
                piv = r;
            }
        if (best == 0.0) return -1;
        if (piv != c) {
            for (int k = 0; k < n; ++k) {
                real t = A[c * n + k];
                A[c * n + k] = A[piv * n + k];
                A[piv * n + k] = t;
            }
            real t = b[c];
            b[c] = b[piv];
            b[piv] = t;
        }
        for (int r = c + 1; r < n; ++r) {
            real m = A[r * n + c] / A[c * n + c];
            if (m == 0.0) continue;
            for (int k = c; k < n; ++k) A[r * n + k] -= m * A[c * n + k];
            b[r] -= m * b[c];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        real s = b[r];
        for (int k = r + 1; k < n; ++k) s -= A[r * n + k] * x[k];
        x[r] = s / A[r * n + r];
    }
    return 0;
}

/* Relaxation matrix of eq. "eq:relaxationMatrix": omega on k_4..k_8, 1 elsewhere. */
static real relax_rate(int j, real omega) { return (j >= 4 && j <= 8) ? omega : 1.0; }

/* Solve T^T f = k for f at velocity u (eq. "system"). */
int orc_reconstruct_literal(const real u[3], const real k[Q], real f[Q])
{
    real T[Q * Q], A[Q * Q], b[Q];
    orc_basis(u, T);
    for (int j = 0; j < Q; ++j)
        for (int i = 0; i < Q; ++i) A[j * Q + i] = T[i * Q + j]; /* A = T^T */
    memcpy(b, k, sizeof b);
    return dense_solve(Q, A, b, f);
}

/* Literal collision: every central-moment vector is formed by the matrix
 * products of Sec. II; k^eq and R come from eqs. "eq:truncation" and "forcing". */
/* Literal collision of a comparison model of Sec. III: the same central-moment
 * relaxation (eq. "eq:relaxationMatrix") with the equilibrium truncated at
 * eq_order and the forcing term at force_order (M1: 6, 6; M4: 6, 2; M5: 2, 2). */
int orc_collide_model_bgk(const real f[Q], const real F[3], real omega, int eq_order, int force_order, int bgk,
                          real fstar[Q]);

int orc_collide_model(const real f[Q], const real F[3], real omega, int eq_order, int force_order, real fstar[Q])
{
    return orc_collide_model_bgk(f, F, omega, eq_order, force_order, 0, fstar);
}

/* As orc_collide_model; bgk != 0 relaxes every central moment with omega
 * (Lambda = omega I, the single-relaxation-time control), which in population
 * space is f* = f - omega (f - f^eq) + (1 - omega / 2) F. */
int orc_collide_model_bgk(const real f[Q], const real F[3], real omega, int eq_order, int force_order, int bgk,
                          real fstar[Q])
{
    real rho, u[3];
    orc_macroscopic(f, F, &rho, u);
    real feq[Q], ff[Q], k[Q], keq[Q], R[Q], ks[Q];
    orc_feq_order(rho, u, eq_order, feq);
    orc_forcing_order(u, F, force_order, ff);
    orc_central_moments(u, f, k);
    orc_central_moments(u, feq, keq);
    orc_central_moments(u, ff, R);
    for (int j = 0; j < Q; ++j) {
        const real L = bgk ? omega : relax_rate(j, omega);
        ks[j] = (1.0 - L) * k[j] + L * keq[j] + (1.0 - 0.5 * L) * R[j];
    }
    return orc_reconstruct_literal(u, ks, fstar);
}

void orc_collide_closed(const real f[Q], const real F[3], real omega, real fstar[Q]);

int orc_collide_literal(const real f[Q], const real F[3], real omega, real fstar[Q])
{
    return orc_collide_model(f, F, omega, 6, 6, fstar);
}

/* Collision by variant code: 0 closed form (M1), 1 literal M1, 2 literal M4
 * (second-order forcing), 3 literal M5 (second-order equilibrium and
 * forcing), 4 literal with a second-order equilibrium and the complete
 * forcing, 5 BGK with the second-order equilibrium and forcing (the classical
 * single-relaxation-time scheme with Guo forcing), 6 BGK with the complete
 * ones.  Returns non-zero on a singular literal solve. */
static int collide_variant(const real f[Q], const real F[3], real omega, int variant, real fstar[Q])
{
    switch (variant) {
        case 0: orc_collide_closed(f, F, omega, fstar); return 0;
        case 1: return orc_collide_model(f, F, omega, 6, 6, fstar);
        case 2: return orc_collide_model(f, F, omega, 6, 2, fstar);
        case 3: return orc_collide_model(f, F, omega, 2, 2, fstar);
        case 4: return orc_collide_model(f, F, omega, 2, 6, fstar);
        case 5: return orc_collide_model_bgk(f, F, omega, 2, 2, 1, fstar);
        default: return orc_collide_model_bgk(f, F, omega, 6, 6, 1, fstar);
    }
}

/* Eq. "pre_collision": k_4..k_8 as direct sums with the shifted velocities. */
void orc_pre_collision(const real f[Q], const real u[3], real k48[5])
{
    real k4 = 0, k5 = 0, k6 = 0, k7 = 0, k8 = 0;
    for (int i = 0; i < Q; ++i) {
        const real X = CX[i] - u[0], Y = CY[i] - u[1], Z = CZ[i] - u[2];
        k4 += f[i] * X * Y;
        k5 += f[i] * X * Z;
        k6 += f[i] * Y * Z;
        k7 += f[i] * (X * X - Y * Y);
        k8 += f[i] * (X * X - Z * Z);
    }
    k48[0] = k4;
    k48[1] = k5;
    k48[2] = k6;
    k48[3] = k7;
    k48[4] = k8;
}

/* Eq. "post_collision_central_moments_forcing": the nineteen non-zero
 * post-collision central moments, all others zero. */
void orc_post_collision(real rho, const real k48[5], const real F[3], real omega, real ks[Q])
{
    const real cs4 = CS2 * CS2, cs6 = cs4 * CS2;
    for (int j = 0; j < Q; ++j) ks[j] = 0.0;
    ks[0] = rho;
    ks[1] = F[0] / 2;
    ks[2] = F[1] / 2;
    ks[3] = F[2] / 2;
    ks[4] = (1 - omega) * k48[0];
    ks[5] = (1 - omega) * k48[1];
    ks[6] = (1 - omega) * k48[2];
    ks[7] = (1 - omega) * k48[3];
    ks[8] = (1 - omega) * k48[4];
    ks[9] = 3 * rho * CS2;
    ks[10] = F[0] * CS2;
    ks[11] = F[1] * CS2;
    ks[12] = F[2] * CS2;
    ks[17] = rho * CS2;
    ks[18] = rho * cs4;
    ks[23] = F[0] * cs4 / 2;
    ks[24] = F[1] * cs4 / 2;
    ks[25] = F[2] * cs4 / 2;
    ks[26] = rho * cs6;
}

/* Inverse of the one-dimensional central-moment map on the velocities
 * {-1, 0, +1} shifted by u: given m0 = sum g, m1 = sum g (c-u),
 * m2 = sum g (c-u)^2, return g(-1), g(0), g(+1).  From m1 + u m0 = g+ - g- and
 * m2 + 2u m1 + u^2 m0 = g+ + g-. */
static void inverse_1d(real m0, real m1, real m2, real u, real g[3])
{
    const real odd = m1 + u * m0;                    /* g+ - g- */
    const real even = m2 + 2 * u * m1 + u * u * m0; /* g+ + g- */
    g[0] = 0.5 * (even - odd);
    g[1] = m0 - even;
    g[2] = 0.5 * (even + odd);
}

/* Fast reconstruction of f from the basis-ordered central moments k (the
 * inverse of k = T^T f).  Step 1 maps the basis of eq. "basis" to monomial
 * central moments K[p][q][r] = sum f (cx-ux)^p (cy-uy)^q (cz-uz)^r by
 * inverting its definitions; step 2 applies inverse_1d along z, y, x. */
void orc_reconstruct_fast(const real u[3], const real k[Q], real f[Q])
{
    real K[3][3][3];
    K[0][0][0] = k[0];
    K[1][0][0] = k[1];
    K[0][1][0] = k[2];
    K[0][0][1] = k[3];
    K[1][1][0] = k[4];
    K[1][0][1] = k[5];
    K[0][1][1] = k[6];
    /* k7 = K200 - K020, k8 = K200 - K002, k9 = K200 + K020 + K002 */
    K[2][0][0] = (k[7] + k[8] + k[9]) / 3;
    K[0][2][0] = (k[9] - 2 * k[7] + k[8]) / 3;
    K[0][0][2] = (k[9] + k[7] - 2 * k[8]) / 3;
    /* k10 = K120 + K102, k13 = K120 - K102, and cyclically */
    K[1][2][0] = (k[10] + k[13]) / 2;
    K[1][0][2] = (k[10] - k[13]) / 2;
    K[2][1][0] = (k[11] + k[14]) / 2;
    K[0][1][2] = (k[11] - k[14]) / 2;
    K[2][0][1] = (k[12] + k[15]) / 2;
    K[0][2][1] = (k[12] - k[15]) / 2;
    K[1][1][1] = k[16];
    /* k17 = K220 + K202 + K022, k18 = K220 + K202 - K022, k19 = K220 - K202 */
    K[0][2][2] = (k[17] - k[18]) / 2;
    K[2][2][0] = ((k[17] + k[18]) / 2 + k[19]) / 2;
    K[2][0][2] = ((k[17] + k[18]) / 2 - k[19]) / 2;
    K[2][1][1] = k[20];
    K[1][2][1] = k[21];
    K[1][1][2] = k[22];
    K[1][2][2] = k[23];
    K[2][1][2] = k[24];
    K[2][2][1] = k[25];
    K[2][2][2] = k[26];

    real A[3][3][3], B[3][3][3], C[3][3][3], g[3];
    for (int p = 0; p < 3; ++p) /* along z: A[p][q][cz] = sum_{fixed cz} f cbar_x^p cbar_y^q */
        for (int q = 0; q < 3; ++q) {
            inverse_1d(K[p][q][0], K[p][q][1], K[p][q][2], u[2], g);
            for (int c = 0; c < 3; ++c) A[p][q][c] = g[c];
        }
    for (int p = 0; p < 3; ++p) /* along y */
        for (int cz = 0; cz < 3; ++cz) {
            inverse_1d(A[p][0][cz], A[p][1][cz], A[p][2][cz], u[1], g);
            for (int c = 0; c < 3; ++c) B[p][c][cz] = g[c];
        }
    for (int cy = 0; cy < 3; ++cy) /* along x */
        for (int cz = 0; cz < 3; ++cz) {
            inverse_1d(B[0][cy][cz], B[1][cy][cz], B[2][cy][cz], u[0], g);
            for (int c = 0; c < 3; ++c) C[c][cy][cz] = g[c];
        }
    for (int i = 0; i < Q; ++i) f[i] = C[CX[i] + 1][CY[i] + 1][CZ[i] + 1];
}

/* Closed-form collision: the five steps listed at the end of Sec. II, minus the
 * streaming, which the lattice driver applies. */
void orc_collide_closed(const real f[Q], const real F[3], real omega, real fstar[Q])
{
    real rho, u[3], k48[5], ks[Q];
    orc_macroscopic(f, F, &rho, u);
    orc_pre_collision(f, u, k48);
    orc_post_collision(rho, k48, F, omega, ks);
    orc_reconstruct_fast(u, ks, fstar);
}

/* ------------------------------------------------------------------------ */
/* Lattice driver.                                                           */

typedef struct {
    int nx, ny, nz, nb;
    int wall[3];          /* per axis x,y,z: 0 periodic, 1 halfway bounce-back walls */
    const uint8_t* solid; /* [N], nonzero = solid node, or NULL */
    const real* force;  /* [3][N] force density, or NULL */
} grid_t;

static void make_grid(grid_t* g, int nx, int ny, int nz, int nb, const int* wall, const uint8_t* solid,
                      const real* force)
{
    g->nx = nx;
    g->ny = ny;
    g->nz = nz;
    g->nb = nb;
    for (int a = 0; a < 3; ++a) g->wall[a] = wall ? wall[a] : 0;
    g->solid = solid;
    g->force = force;
}

static long ncells(const grid_t* g) { return (long)g->nb * g->nz * g->ny * g->nx; }

static int is_solid(const grid_t* g, long n) { return g->solid && g->solid[n]; }

static void cell_force(const grid_t* g, long n, real F[3])
{
    const long N = ncells(g);
    for (int a = 0; a < 3; ++a) F[a] = g->force ? g->force[a * N + n] : 0.0;
}

/* Node reached from cell n along velocity i, or -1 if that is a wall or solid. */
static long neighbour(const grid_t* g, long n, int i)
{
    long x = n % g->nx, r = n / g->nx;
    long y = r % g->ny;
    r /= g->ny;
    long z = r % g->nz, b = r / g->nz;
    long c[3] = {x + CX[i], y + CY[i], z + CZ[i]};
    const long dim[3] = {g->nx, g->ny, g->nz};
    for (int a = 0; a < 3; ++a) {
        if (c[a] < 0 || c[a] >= dim[a]) {
            if (g->wall[a]) return -1;
            c[a] = (c[a] + dim[a]) % dim[a];
        }
    }
    long m = ((b * g->nz + c[2]) * g->ny + c[1]) * g->nx + c[0];
    if (is_solid(g, m)) return -1;
    return m;
}

void orc_lattice_init(int nx, int ny, int nz, int nb, const uint8_t* solid, const real* rho,
                      const real* u, real* f)
{
    grid_t g;
    make_grid(&g, nx, ny, nz, nb, NULL, solid, NULL);
    const long N = ncells(&g);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        real fe[Q];
        if (is_solid(&g, n)) {
            for (int i = 0; i < Q; ++i) fe[i] = 0.0;
        } else {
            const real uu[3] = {u[n], u[N + n], u[2 * N + n]};
            orc_feq(rho[n], uu, fe);
        }
        for (int i = 0; i < Q; ++i) f[i * N + n] = fe[i];
    }
}

/* Advance nsteps: collide every fluid cell (eq. "collision" in central-moment
 * form), then stream (eq. "streaming") with periodic wrap or halfway
 * bounce-back (reading R3).  variant: see collide_variant.
 * tmp is caller scratch of the same size as f.  Returns 0, or -1 if a literal
 * solve met a singular matrix. */
int orc_lattice_step(int nx, int ny, int nz, int nb, const int* wall, const uint8_t* solid,
                     const real* force, real omega, int variant, int nsteps, real* f, real* tmp)
{
    grid_t g;
    make_grid(&g, nx, ny, nz, nb, wall, solid, force);
    const long N = ncells(&g);
    int status = 0;
    for (int s = 0; s < nsteps; ++s) {
#pragma omp parallel for schedule(static)
        for (long n = 0; n < N; ++n) {
            if (is_solid(&g, n)) continue;
            real fc[Q], fs[Q], F[3];
            for (int i = 0; i < Q; ++i) fc[i] = f[i * N + n];
            cell_force(&g, n, F);
            if (collide_variant(fc, F, omega, variant, fs) != 0) {
#pragma omp atomic write
                status = -1;
            }
            for (int i = 0; i < Q; ++i) tmp[i * N + n] = fs[i];
        }
#pragma omp parallel for schedule(static)
        for (long n = 0; n < N; ++n) {
            if (is_solid(&g, n)) continue;
            for (int i = 0; i < Q; ++i) {
                const long m = neighbour(&g, n, i);
                if (m >= 0)
                    f[i * N + m] = tmp[i * N + n];
                else
                    f[opposite(i) * N + n] = tmp[i * N + n];
            }
        }
        if (status) return status;
    }
    return status;
}

/* Eq. "macroscopic" on every fluid cell; solid cells report rho = 0, u = 0. */
void orc_lattice_moments(int nx, int ny, int nz, int nb, const uint8_t* solid, const real* force,
                         const real* f, real* rho, real* u)
{
    grid_t g;
    make_grid(&g, nx, ny, nz, nb, NULL, solid, force);
    const long N = ncells(&g);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        if (is_solid(&g, n)) {
            rho[n] = 0.0;
            u[n] = u[N + n] = u[2 * N + n] = 0.0;
            continue;
        }
        real fc[Q], F[3], r, uu[3];
        for (int i = 0; i < Q; ++i) fc[i] = f[i * N + n];
        cell_force(&g, n, F);
        orc_macroscopic(fc, F, &r, uu);
        rho[n] = r;
        u[n] = uu[0];
        u[N + n] = uu[1];
        u[2 * N + n] = uu[2];
    }
}

/* Collide n independent cells (sampled checks): f, out are [27][n], F is
 * [3][n] or NULL.  variant: see collide_variant. */
int orc_collide_cells(long n, const real* f, const real* F, real omega, int variant, real* out)
{
    int status = 0;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < n; ++c) {
        real fc[Q], fs[Q], Fc[3];
        for (int i = 0; i < Q; ++i) fc[i] = f[i * n + c];
        for (int a = 0; a < 3; ++a) Fc[a] = F ? F[a * n + c] : 0.0;
        if (collide_variant(fc, Fc, omega, variant, fs) != 0) {
#pragma omp atomic write
            status = -1;
        }
        for (int i = 0; i < Q; ++i) out[i * n + c] = fs[i];
    }
    return status;
}

/* Shan-Chen pseudo-potential interaction force of the static-droplet test
 * (Sec. III): F(x) = -G psi(x) sum_i w_i c_i psi(x + c_i), psi = 1 - exp(-rho),
 * on a periodic lattice.  rho is [N], F is [3][N]. */
static real real_exp(real v)
{
#ifdef ORC_EXTENDED
    return expl(v);
#else
    return exp(v);
#endif
}

void orc_pseudopotential_force(int nx, int ny, int nz, int nb, real G, const real* rho, real* F)
{
    grid_t g;
    const int wall[3] = {0, 0, 0};
    make_grid(&g, nx, ny, nz, nb, wall, NULL, NULL);
    const long N = ncells(&g);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        real s[3] = {0, 0, 0};
        for (int i = 1; i < Q; ++i) {
            const long m = neighbour(&g, n, i);
            const real psi = 1.0 - real_exp(-rho[m]);
            s[0] += weight(i) * CX[i] * psi;
            s[1] += weight(i) * CY[i] * psi;
            s[2] += weight(i) * CZ[i] * psi;
        }
        const real psi0 = 1.0 - real_exp(-rho[n]);
        for (int a = 0; a < 3; ++a) F[a * N + n] = -G * psi0 * s[a];
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
