/*
 * Plain FP64 CPU oracle of the magnetic-field lattice of App. C of De Rosis,
 * Huang & Coreixas, Phys. Rev. E (2019), arXiv:1905.10182, and of the Lorentz
 * force that couples it to the fluid (Sec. III, Hartmann and Orszag-Tang tests).
 *
 * TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the
 * cpu_baseline leg of the benchmark may load it.  The GPU library never
 * links, calls or includes it, and the two share no code, tables or constants.
 *
 * The magnetic field b is carried by vector-valued populations h_l (three
 * components each) on the D3Q7 velocity set, relaxed with one rate omega_m
 * (BGK) towards h^eq_la = w_l [b_a + (1/cs^2) xi_lb (u_b b_a - b_b u_a)],
 * cs^2 = 1/4, and streamed along xi_l; b = sum_l h_l; the resistivity is
 * eta = cs^2 (1/omega_m - 1/2).
 *
 * Readings (each also listed in the repository's design notes):
 *   C1  The current j = curl b "from the populations": the first-order
 *       Chapman-Enskog relation for the pre-collision non-equilibrium part of
 *       the electric tensor Lambda_ba = sum_l xi_lb h_la, Lambda^neq_ba =
 *       -tau_m cs^2 d_b b_a, gives j_c = -eps_cba Lambda^neq_ba / (tau_m cs^2)
 *       (tau_m = 1/omega_m).  It neglects the time derivative of the
 *       equilibrium tensor, an O(u^2/cs^2) relative term.  The central
 *       difference curl of b is the alternative ("stencil") current.
 *   C2  The Lorentz force F = j x b is a force density (b in units where the
 *       magnetic pressure is |b|^2/2).
 *   (C3, the order of the stages within a coupled step, is sequenced by the
 *   Python wrapper mhd.py.)
 *   C6  Periodic axes, or walls halfway between nodes on the axes flagged in
 *       `wall`: the magnetic field takes a given value b_w at the wall (the
 *       Hartmann test imposes it there).  A population that would stream into
 *       the wall comes back as h_opp(l)(x, t+1) = -h*_l(x, t) + 2 w_l b_w
 *       (anti-bounce-back, which places the Dirichlet value at the half-way
 *       point); the central-difference curl uses the ghost value 2 b_w - b(x)
 *       beyond a wall.
 *
 * Layout: h[(l*3 + a)*N + n], N = nz*ny*nx, n = (z*ny + y)*nx + x; vector
 * fields [3][N].
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#ifdef ORC_EXTENDED
typedef long double real;
#else
typedef double real;
#endif

#define QM 7

/* D3Q7 velocities in the order printed in App. C. */
static const int XI[QM][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};

/* Weights printed in App. C: 1/4 at rest, 1/8 on the six links. */
static real wm(int l) { return l == 0 ? (real)1 / 4 : (real)1 / 8; }

static const real CSM2 = (real)1 / 4; /* cs^2 of the D3Q7 set */

void orc_mhd_constants(int* xi, real* w)
{
    for (int l = 0; l < QM; ++l) {
        for (int a = 0; a < 3; ++a) xi[3 * l + a] = XI[l][a];
        w[l] = wm(l);
    }
}

/* Equilibrium of App. C: heq[l*3 + a] = w_l [b_a + 4 xi_lb (u_b b_a - b_b u_a)]. */
void orc_mhd_heq(const real b[3], const real u[3], real heq[QM * 3])
{
    for (int l = 0; l < QM; ++l)
        for (int a = 0; a < 3; ++a) {
            real s = 0.0;
            for (int c = 0; c < 3; ++c) s += XI[l][c] * (u[c] * b[a] - b[c] * u[a]);
            heq[3 * l + a] = wm(l) * (b[a] + s / CSM2);
        }
}

/* h = h^eq(b(x), u(x)) for every cell; u may be NULL (rest). */
void orc_mhd_init(int nx, int ny, int nz, const real* b, const real* u, real* h)
{
    const long N = (long)nx * ny * nz;
    for (long n = 0; n < N; ++n) {
        const real bb[3] = {b[n], b[N + n], b[2 * N + n]};
        real uu[3] = {0.0, 0.0, 0.0};
        if (u)
            for (int a = 0; a < 3; ++a) uu[a] = u[a * N + n];
        real e[QM * 3];
        orc_mhd_heq(bb, uu, e);
        for (int k = 0; k < QM * 3; ++k) h[k * N + n] = e[k];
    }
}

static void cell_b(const real* h, long N, long n, real b[3])
{
    for (int a = 0; a < 3; ++a) {
        real s = 0.0;
        for (int l = 0; l < QM; ++l) s += h[(3 * l + a) * N + n];
        b[a] = s;
    }
}

/* One step: collide every cell towards h^eq(b, u) with rate omega_m, then
 * stream, h_l(x + xi_l) = h*_l(x), periodic or through the wall rule of
 * reading C6 (wall[3] flags per axis, b_wall[3]; both may be NULL = periodic).
 * u is [3][N] or NULL. */
void orc_mhd_step_walls(int nx, int ny, int nz, const int* wall, const real* b_wall, const real* u, real omega_m,
                        real* h, real* tmp);

void orc_mhd_step(int nx, int ny, int nz, const real* u, real omega_m, real* h, real* tmp)
{
    orc_mhd_step_walls(nx, ny, nz, NULL, NULL, u, omega_m, h, tmp);
}

static int opp_m(int l) { return l == 0 ? 0 : (l % 2 ? l + 1 : l - 1); }

void orc_mhd_step_walls(int nx, int ny, int nz, const int* wall, const real* b_wall, const real* u, real omega_m,
                        real* h, real* tmp)
{
    const long N = (long)nx * ny * nz;
    for (long n = 0; n < N; ++n) {
        real b[3], uu[3] = {0.0, 0.0, 0.0}, e[QM * 3];
        cell_b(h, N, n, b);
        if (u)
            for (int a = 0; a < 3; ++a) uu[a] = u[a * N + n];
        orc_mhd_heq(b, uu, e);
        for (int k = 0; k < QM * 3; ++k) tmp[k * N + n] = h[k * N + n] + omega_m * (e[k] - h[k * N + n]);
    }
    const long dim[3] = {nx, ny, nz};
    for (long n = 0; n < N; ++n) {
        const long c[3] = {n % nx, (n / nx) % ny, n / ((long)nx * ny)};
        for (int l = 0; l < QM; ++l) {
            long d[3];
            int into_wall = 0;
            for (int a = 0; a < 3; ++a) {
                d[a] = c[a] + XI[l][a];
                if (d[a] < 0 || d[a] >= dim[a]) {
                    if (wall && wall[a]) into_wall = 1;
                    d[a] = (d[a] + dim[a]) % dim[a];
                }
            }
            if (into_wall) {
                const int o = opp_m(l);
                for (int a = 0; a < 3; ++a)
                    h[(3 * o + a) * N + n] = -tmp[(3 * l + a) * N + n] + 2.0 * wm(l) * (b_wall ? b_wall[a] : 0.0);
                continue;
            }
            const long m = (d[2] * ny + d[1]) * nx + d[0];
            for (int a = 0; a < 3; ++a) h[(3 * l + a) * N + m] = tmp[(3 * l + a) * N + n];
        }
    }
}

/* b = sum_l h_l and the population current of reading C1 (j may be NULL):
 * Lambda_ba = sum_l xi_lb h_la, Lambda^eq_ba = u_b b_a - b_b u_a,
 * j_c = -eps_cba (Lambda - Lambda^eq)_ba / (tau_m cs^2). */
void orc_mhd_fields(int nx, int ny, int nz, const real* u, real tau_m, const real* h, real* b, real* j)
{
    const long N = (long)nx * ny * nz;
    for (long n = 0; n < N; ++n) {
        real bb[3], uu[3] = {0.0, 0.0, 0.0};
        cell_b(h, N, n, bb);
        for (int a = 0; a < 3; ++a) b[a * N + n] = bb[a];
        if (!j) continue;
        if (u)
            for (int a = 0; a < 3; ++a) uu[a] = u[a * N + n];
        real L[3][3]; /* L[b][a] = Lambda_ba - Lambda^eq_ba */
        for (int p = 0; p < 3; ++p)
            for (int a = 0; a < 3; ++a) {
                real s = 0.0;
                for (int l = 0; l < QM; ++l) s += XI[l][p] * h[(3 * l + a) * N + n];
                L[p][a] = s - (uu[p] * bb[a] - bb[p] * uu[a]);
            }
        /* eps_cba L[b][a]: c = x: L[y][z] - L[z][y]; y: L[z][x] - L[x][z]; z: L[x][y] - L[y][x] */
        const real k = -1.0 / (tau_m * CSM2);
        j[n] = k * (L[1][2] - L[2][1]);
        j[N + n] = k * (L[2][0] - L[0][2]);
        j[2 * N + n] = k * (L[0][1] - L[1][0]);
    }
}

/* Central-difference curl of b ([3][N]) into j: periodic axes, or (wall[a]
 * set) the ghost value 2 b_wall - b(x) beyond a wall (reading C6).  wall and
 * b_wall may be NULL (periodic). */
void orc_curl_fd_walls(int nx, int ny, int nz, const int* wall, const real* b_wall, const real* b, real* j)
{
    const long N = (long)nx * ny * nz;
    const long dim[3] = {nx, ny, nz};
    const long stride[3] = {1, nx, (long)nx * ny};
    for (long n = 0; n < N; ++n) {
        const long c[3] = {n % nx, (n / nx) % ny, n / ((long)nx * ny)};
        real D[3][3]; /* D[a][comp] = d_a b_comp */
        for (int a = 0; a < 3; ++a) {
            for (int q = 0; q < 3; ++q) D[a][q] = 0.0;
            if (dim[a] < 2) continue; /* an axis of extent 1 has no derivative */
            for (int q = 0; q < 3; ++q) {
                real vp, vm;
                const real here = b[q * N + n];
                if (c[a] + 1 < dim[a])
                    vp = b[q * N + n + stride[a]];
                else
                    vp = (wall && wall[a]) ? 2.0 * (b_wall ? b_wall[q] : 0.0) - here : b[q * N + n - (dim[a] - 1) * stride[a]];
                if (c[a] > 0)
                    vm = b[q * N + n - stride[a]];
                else
                    vm = (wall && wall[a]) ? 2.0 * (b_wall ? b_wall[q] : 0.0) - here : b[q * N + n + (dim[a] - 1) * stride[a]];
                D[a][q] = 0.5 * (vp - vm);
            }
        }
        j[n] = D[1][2] - D[2][1];
        j[N + n] = D[2][0] - D[0][2];
        j[2 * N + n] = D[0][1] - D[1][0];
    }
}

void orc_curl_fd(int nx, int ny, int nz, const real* b, real* j) { orc_curl_fd_walls(nx, ny, nz, NULL, NULL, b, j); }

/* Lorentz force density F = j x b (reading C2). */
void orc_lorentz(long N, const real* j, const real* b, real* F)
{
    for (long n = 0; n < N; ++n) {
        const real jx = j[n], jy = j[N + n], jz = j[2 * N + n];
        const real bx = b[n], by = b[N + n], bz = b[2 * N + n];
        F[n] = jy * bz - jz * by;
        F[N + n] = jz * bx - jx * bz;
        F[2 * N + n] = jx * by - jy * bx;
    }
}
