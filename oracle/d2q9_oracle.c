/*
 * Plain FP64 CPU oracle of the two-dimensional (D2Q9) central-moment lattice
 * Boltzmann method with Hermite forcing of App. B of De Rosis, Huang &
 * Coreixas, Phys. Rev. E (2019), arXiv:1905.10182.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent checker of the HIP
 * D2Q9 solver: only the tests, the smoke check and the cpu_baseline leg of
 * the benchmark may load it.  The GPU library never links, calls or includes
 * it, and the two share no code, tables or constants.
 *
 * Populations are unshifted FP64 (or 80-bit with -DORC_EXTENDED).  Two
 * collision routes, as for the three-dimensional oracle:
 *   - "literal" (orc2_collide_model): the matrix algebra of App. B: the
 *     shifted basis T-bar_0..T-bar_8, k = T^T f, k^eq = T^T f^eq with f^eq
 *     the Hermite expansion of eq. "eq:D2Q9", R = T^T F with F the Hermite
 *     forcing of App. B, k* = (I - L) k + L k^eq + (I - L/2) R with
 *     L = diag(1, 1, 1, 1, omega, omega, 1, 1, 1), then T^T f* = k* solved by
 *     Gaussian elimination.  Truncation orders give the comparison models.
 *   - "closed" (orc2_collide_closed): the printed post-collision central
 *     moments of App. B (k0* = rho, k1,2* = F/2, k3* = 2 rho cs^2,
 *     k4,5* = (1 - omega) k4,5, k6* = Fy cs^2 / 2, k7* = Fx cs^2 / 2,
 *     k8* = rho cs^4), mapped to monomial central moments and inverted by two
 *     one-dimensional transforms on {-1, 0, +1} (y, then x).
 *
 * Readings (each also listed in the repository's design notes):
 *   B1  The seventh basis vector is (cx - ux)(cy - uy)^2: its printed
 *       subscript is garbled, and this is the only cubic monomial left after
 *       T-bar_6 = (cx - ux)^2 (cy - uy) that makes the basis complete.
 *   B2  The Hermite forcing of App. B is the full-order expansion with the
 *       coefficients 1/cs^2, 1/(2 cs^4), 1/(6 cs^6), 1/(24 cs^8) of the fully
 *       symmetrised tensors [F], [Fu], [Fuu], [Fuuu] (the printed powers of
 *       c_s are garbled); F is a force density (no rho prefactor), u the
 *       half-force-corrected velocity, as in the three-dimensional model.
 *   B3  Periodic boundaries on both axes (the App. B model is only used on
 *       the periodic four-rolls mill here).
 *
 * Lattice layout: population i of cell n lives at f[i*N + n], N = ny*nx,
 * n = y*nx + x; velocity order of App. B.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define Q2 9

#ifdef ORC_EXTENDED
typedef long double real;
#define RFABS fabsl
#else
typedef double real;
#define RFABS fabs
#endif

/* D2Q9 velocities in the order printed at the start of App. B. */
static const int CX2[Q2] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
static const int CY2[Q2] = {0, 0, 0, 1, -1, 1, -1, -1, 1};

/* Weights listed after eq. "eq:D2Q9". */
static real weight2(int i)
{
    if (i == 0) return (real)4 / 9;
    if (i <= 4) return (real)1 / 9;
    return (real)1 / 36;
}

static const real CS2 = (real)1 / 3;

static int opposite2(int i)
{
    for (int j = 0; j < Q2; ++j)
        if (CX2[j] == -CX2[i] && CY2[j] == -CY2[i]) return j;
    return -1;
}

void orc2_lattice_constants(int* cx, int* cy, real* w, int* opp)
{
    for (int i = 0; i < Q2; ++i) {
        cx[i] = CX2[i];
        cy[i] = CY2[i];
        w[i] = weight2(i);
        opp[i] = opposite2(i);
    }
}

/* Hermite polynomials of App. A restricted to two dimensions, named by their
 * index string: H_x = cx, H_xx = cx^2 - cs^2, H_xy = cx cy, H_xxy = H_xx cy,
 * H_xyy = cx H_yy, H_xxyy = H_xx H_yy. */
typedef struct {
    real x, y, xx, yy, xy, xxy, xyy, xxyy;
} herm2;

static void hermite2(int i, herm2* h)
{
    const real cx = CX2[i], cy = CY2[i];
    h->x = cx;
    h->y = cy;
    h->xx = cx * cx - CS2;
    h->yy = cy * cy - CS2;
    h->xy = cx * cy;
    h->xxy = h->xx * cy;
    h->xyy = cx * h->yy;
    h->xxyy = h->xx * h->yy;
}

/* Equilibrium of eq. "eq:D2Q9", term by term.  order < 3 keeps H0..H2 (the
 * classical second-order equilibrium), otherwise every term through H4_xxyy. */
void orc2_feq_order(real rho, const real u[2], int order, real out[Q2])
{
    const real ux = u[0], uy = u[1];
    const real cs4 = CS2 * CS2, cs6 = cs4 * CS2, cs8 = cs4 * cs4;
    for (int i = 0; i < Q2; ++i) {
        herm2 H;
        hermite2(i, &H);
        real s = 1.0 + (H.x * ux + H.y * uy) / CS2;
        s += (H.xx * ux * ux + H.yy * uy * uy + 2.0 * H.xy * ux * uy) / (2.0 * cs4);
        if (order >= 3) {
            s += (H.xxy * ux * ux * uy + H.xyy * ux * uy * uy) / (2.0 * cs6);
            s += H.xxyy * ux * ux * uy * uy / (4.0 * cs8);
        }
        out[i] = weight2(i) * rho * s;
    }
}

/* Hermite forcing of App. B under reading B2:
 * w_i [H1.F/cs^2 + H2:[Fu]/(2 cs^4) + H3:[Fuu]/(6 cs^6) + H4:[Fuuu]/(24 cs^8)],
 * where a contraction with a symmetric tensor counts each distinct index
 * string with its multiplicity (xy twice; xxy, xyy three times; xxyy six
 * times), and only the Hermite tensors the D2Q9 set carries are kept.
 * order < 3 keeps H1 + H2 (the Guo et al. form the text names). */
void orc2_forcing_order(const real u[2], const real F[2], int order, real out[Q2])
{
    const real ux = u[0], uy = u[1], Fx = F[0], Fy = F[1];
    const real cs4 = CS2 * CS2, cs6 = cs4 * CS2, cs8 = cs4 * cs4;
    /* symmetrised tensors, one entry per index string */
    const real Fu_xx = 2 * Fx * ux, Fu_yy = 2 * Fy * uy, Fu_xy = Fx * uy + ux * Fy;
    const real Fuu_xxy = 2 * Fx * ux * uy + ux * ux * Fy;
    const real Fuu_xyy = Fx * uy * uy + 2 * ux * Fy * uy;
    const real Fuuu_xxyy = 2 * Fx * ux * uy * uy + 2 * ux * ux * Fy * uy;
    for (int i = 0; i < Q2; ++i) {
        herm2 H;
        hermite2(i, &H);
        real s = (H.x * Fx + H.y * Fy) / CS2;
        s += (H.xx * Fu_xx + H.yy * Fu_yy + 2 * H.xy * Fu_xy) / (2 * cs4);
        if (order >= 3) {
            s += 3 * (H.xxy * Fuu_xxy + H.xyy * Fuu_xyy) / (6 * cs6);
            s += 6 * H.xxyy * Fuuu_xxyy / (24 * cs8);
        }
        out[i] = weight2(i) * s;
    }
}

/* The nine basis vectors T-bar_0..T-bar_8 of App. B (reading B1 for the
 * seventh), evaluated at velocity i shifted by u: Tbar[i*9 + j]. */
void orc2_basis(const real u[2], real Tbar[Q2 * Q2])
{
    for (int i = 0; i < Q2; ++i) {
        const real X = CX2[i] - u[0], Y = CY2[i] - u[1];
        real* T = Tbar + i * Q2;
        T[0] = 1.0;
        T[1] = X;
        T[2] = Y;
        T[3] = X * X + Y * Y;
        T[4] = X * X - Y * Y;
        T[5] = X * Y;
        T[6] = X * X * Y;
        T[7] = X * Y * Y;
        T[8] = X * X * Y * Y;
    }
}

/* k = T^T f. */
void orc2_central_moments(const real u[2], const real f[Q2], real k[Q2])
{
    real T[Q2 * Q2];
    orc2_basis(u, T);
    for (int j = 0; j < Q2; ++j) {
        real s = 0.0;
        for (int i = 0; i < Q2; ++i) s += T[i * Q2 + j] * f[i];
        k[j] = s;
    }
}

/* Density and the half-force-corrected velocity (eq. "macroscopic" of the
 * three-dimensional model restricted to two dimensions). */
void orc2_macroscopic(const real f[Q2], const real F[2], real* rho, real u[2])
{
    real r = 0.0, jx = 0.0, jy = 0.0;
    for (int i = 0; i < Q2; ++i) {
        r += f[i];
        jx += CX2[i] * f[i];
        jy += CY2[i] * f[i];
    }
    *rho = r;
    u[0] = (jx + 0.5 * F[0]) / r;
    u[1] = (jy + 0.5 * F[1]) / r;
}

/* A x = b by Gaussian elimination with partial pivoting (A row-major, n x n,
 * overwritten).  Returns 0, or -1 if A is singular. */
static int solve2(int n, real* A, real* b, real* x)
{
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (RFABS(A[r * n + c]) > RFABS(A[piv * n + c])) piv = r;
        if (A[piv * n + c] == 0.0) return -1;
        if (piv != c) {
            for (int k = 0; k < n; ++k) {
                const real t = A[c * n + k];
                A[c * n + k] = A[piv * n + k];
                A[piv * n + k] = t;
            }
            const real t = b[c];
            b[c] = b[piv];
            b[piv] = t;
        }
        for (int r = c + 1; r < n; ++r) {
            const real m = A[r * n + c] / A[c * n + c];
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

/* Solve T^T f = k at velocity u (eq. "system2"). */
int orc2_reconstruct_literal(const real u[2], const real k[Q2], real f[Q2])
{
    real T[Q2 * Q2], A[Q2 * Q2], b[Q2];
    orc2_basis(u, T);
    for (int j = 0; j < Q2; ++j)
        for (int i = 0; i < Q2; ++i) A[j * Q2 + i] = T[i * Q2 + j];
    memcpy(b, k, sizeof b);
    return solve2(Q2, A, b, f);
}

/* Relaxation matrix of App. B: omega on k4 and k5, 1 elsewhere. */
static real relax2(int j, real omega) { return (j == 4 || j == 5) ? omega : 1.0; }

/* Literal collision with the equilibrium truncated at eq_order and the
 * forcing at force_order (4, 4: the method; 4, 2: Guo forcing; 2, 2: both
 * second order; 2, 4: second-order equilibrium, complete forcing). */
int orc2_collide_model(const real f[Q2], const real F[2], real omega, int eq_order, int force_order,
                       real fstar[Q2])
{
    real rho, u[2], feq[Q2], ff[Q2], k[Q2], keq[Q2], R[Q2], ks[Q2];
    orc2_macroscopic(f, F, &rho, u);
    orc2_feq_order(rho, u, eq_order, feq);
    orc2_forcing_order(u, F, force_order, ff);
    orc2_central_moments(u, f, k);
    orc2_central_moments(u, feq, keq);
    orc2_central_moments(u, ff, R);
    for (int j = 0; j < Q2; ++j) {
        const real L = relax2(j, omega);
        ks[j] = (1.0 - L) * k[j] + L * keq[j] + (1.0 - 0.5 * L) * R[j];
    }
    return orc2_reconstruct_literal(u, ks, fstar);
}

/* The printed post-collision central moments of App. B from the density,
 * the pre-collision k4, k5 and the force density. */
void orc2_post_collision(real rho, real k4, real k5, const real F[2], real omega, real ks[Q2])
{
    ks[0] = rho;
    ks[1] = 0.5 * F[0];
    ks[2] = 0.5 * F[1];
    ks[3] = 2.0 * rho * CS2;
    ks[4] = (1.0 - omega) * k4;
    ks[5] = (1.0 - omega) * k5;
    ks[6] = 0.5 * F[1] * CS2;
    ks[7] = 0.5 * F[0] * CS2;
    ks[8] = rho * CS2 * CS2;
}

/* (g-, g0, g+) on {-1, 0, +1} from the moments sum g (1, c - u, (c - u)^2):
 * the raw moments are m0, m1 + u m0, m2 + 2 u m1 + u^2 m0, and
 * g+- = (raw2 +- raw1) / 2, g0 = raw0 - raw2. */
static void inverse_1d_2(real m0, real m1, real m2, real u, real g[3])
{
    const real r1 = m1 + u * m0;
    const real r2 = m2 + 2.0 * u * m1 + u * u * m0;
    g[0] = 0.5 * (r2 - r1);
    g[1] = m0 - r2;
    g[2] = 0.5 * (r2 + r1);
}

/* Closed-form collision: direct sums for rho, u, k4, k5; the printed k*; the
 * basis mapped to monomial central moments K[p][q] = sum f (cx-ux)^p (cy-uy)^q
 * (K20 = (k3 + k4)/2, K02 = (k3 - k4)/2, K11 = k5, K21 = k6, K12 = k7,
 * K22 = k8), then the inverse transform along y and along x. */
void orc2_collide_closed(const real f[Q2], const real F[2], real omega, real fstar[Q2])
{
    real rho, u[2];
    orc2_macroscopic(f, F, &rho, u);
    real k4 = 0.0, k5 = 0.0;
    for (int i = 0; i < Q2; ++i) {
        const real X = CX2[i] - u[0], Y = CY2[i] - u[1];
        k4 += (X * X - Y * Y) * f[i];
        k5 += X * Y * f[i];
    }
    real ks[Q2];
    orc2_post_collision(rho, k4, k5, F, omega, ks);
    real K[3][3];
    K[0][0] = ks[0];
    K[1][0] = ks[1];
    K[0][1] = ks[2];
    K[2][0] = 0.5 * (ks[3] + ks[4]);
    K[0][2] = 0.5 * (ks[3] - ks[4]);
    K[1][1] = ks[5];
    K[2][1] = ks[6];
    K[1][2] = ks[7];
    K[2][2] = ks[8];
    /* along y: for each x-moment order p, the y-distribution G[p][cy+1] */
    real G[3][3];
    for (int p = 0; p < 3; ++p) inverse_1d_2(K[p][0], K[p][1], K[p][2], u[1], G[p]);
    for (int i = 0; i < Q2; ++i) fstar[i] = 0.0;
    for (int b = 0; b < 3; ++b) {
        real g[3];
        inverse_1d_2(G[0][b], G[1][b], G[2][b], u[0], g);
        for (int a = 0; a < 3; ++a)
            for (int i = 0; i < Q2; ++i)
                if (CX2[i] == a - 1 && CY2[i] == b - 1) fstar[i] = g[a];
    }
}

/* Variant code: 0 closed form, 1 literal method, 2 Guo forcing, 3 second-order
 * equilibrium and forcing, 4 second-order equilibrium with complete forcing. */
static int collide2_variant(const real f[Q2], const real F[2], real omega, int variant, real fstar[Q2])
{
    switch (variant) {
        case 0: orc2_collide_closed(f, F, omega, fstar); return 0;
        case 1: return orc2_collide_model(f, F, omega, 4, 4, fstar);
        case 2: return orc2_collide_model(f, F, omega, 4, 2, fstar);
        case 3: return orc2_collide_model(f, F, omega, 2, 2, fstar);
        default: return orc2_collide_model(f, F, omega, 2, 4, fstar);
    }
}

/* Collide n independent cells: f, out [9][n], F [2][n] or NULL. */
int orc2_collide_cells(long n, const real* f, const real* F, real omega, int variant, real* out)
{
    int status = 0;
    for (long c = 0; c < n; ++c) {
        real fc[Q2], fs[Q2], Fc[2];
        for (int i = 0; i < Q2; ++i) fc[i] = f[i * n + c];
        for (int a = 0; a < 2; ++a) Fc[a] = F ? F[a * n + c] : 0.0;
        if (collide2_variant(fc, Fc, omega, variant, fs) != 0) status = -1;
        for (int i = 0; i < Q2; ++i) out[i * n + c] = fs[i];
    }
    return status;
}

/* f(x, 0) = f^eq(rho(x), u(x)), complete equilibrium; u is [2][N]. */
void orc2_lattice_init(int nx, int ny, const real* rho, const real* u, real* f)
{
    const long N = (long)nx * ny;
    for (long n = 0; n < N; ++n) {
        const real uu[2] = {u[n], u[N + n]};
        real fe[Q2];
        orc2_feq_order(rho[n], uu, 4, fe);
        for (int i = 0; i < Q2; ++i) f[i * N + n] = fe[i];
    }
}

/* nsteps of collision (variant) then periodic streaming f_i(x + c_i) = f*_i(x).
 * force is [2][N] or NULL; tmp has the size of f.  Returns 0 or -1. */
int orc2_lattice_step(int nx, int ny, const real* force, real omega, int variant, int nsteps, real* f, real* tmp)
{
    const long N = (long)nx * ny;
    int status = 0;
    for (int s = 0; s < nsteps; ++s) {
        for (long n = 0; n < N; ++n) {
            real fc[Q2], fs[Q2], F[2];
            for (int i = 0; i < Q2; ++i) fc[i] = f[i * N + n];
            F[0] = force ? force[n] : 0.0;
            F[1] = force ? force[N + n] : 0.0;
            if (collide2_variant(fc, F, omega, variant, fs) != 0) status = -1;
            for (int i = 0; i < Q2; ++i) tmp[i * N + n] = fs[i];
        }
        for (long n = 0; n < N; ++n) {
            const long x = n % nx, y = n / nx;
            for (int i = 0; i < Q2; ++i) {
                const long xd = (x + CX2[i] + nx) % nx, yd = (y + CY2[i] + ny) % ny;
                f[i * N + yd * nx + xd] = tmp[i * N + n];
            }
        }
        if (status) return status;
    }
    return status;
}

/* rho and the half-force-corrected u ([2][N]) of every cell. */
void orc2_lattice_moments(int nx, int ny, const real* force, const real* f, real* rho, real* u)
{
    const long N = (long)nx * ny;
    for (long n = 0; n < N; ++n) {
        real fc[Q2], F[2], r, uu[2];
        for (int i = 0; i < Q2; ++i) fc[i] = f[i * N + n];
        F[0] = force ? force[n] : 0.0;
        F[1] = force ? force[N + n] : 0.0;
        orc2_macroscopic(fc, F, &r, uu);
        rho[n] = r;
        u[n] = uu[0];
        u[N + n] = uu[1];
    }
}
