// D3Q27 lattice constants and the per-cell collision of the central-moment
// lattice Boltzmann method with Hermite forcing (De Rosis, Huang & Coreixas,
// PRE 2019, Sec. II), written for gfx950 register-resident evaluation.
//
// The collision is done in "deviation form": populations are handled as
// h_i = f_i - w_i rho0 and every moment is carried minus its value for the
// rest state (rho0, populations w_i rho0), so FP32 arithmetic keeps its
// relative precision on the small quantities that carry the flow.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cmlbm {

// Velocity components in the order of Sec. II.
__host__ __device__ constexpr int vel_x(int i)
{
    constexpr int v[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
    return v[i];
}
__host__ __device__ constexpr int vel_y(int i)
{
    constexpr int v[27] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, 1, -1, -1, 1, 1, -1, -1};
    return v[i];
}
__host__ __device__ constexpr int vel_z(int i)
{
    constexpr int v[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1};
    return v[i];
}
// Index of the velocity (a, b, c), each in {-1, 0, 1}.
__host__ __device__ constexpr int vel_index(int a, int b, int c)
{
    for (int i = 0; i < 27; ++i)
        if (vel_x(i) == a && vel_y(i) == b && vel_z(i) == c) return i;
    return -1;
}
__host__ __device__ constexpr int opposite(int i) { return vel_index(-vel_x(i), -vel_y(i), -vel_z(i)); }

// 1 / x.  FP32: the hardware reciprocal (about one ulp) refined by one Newton
// step, e = 1 - x r, r + r e (within an ulp of the quotient; the density is
// near 1, far from FP32's range limits), in place of the correctly rounded
// division's scale / fix-up sequence.  FP64: the division.
template <typename T>
__device__ __forceinline__ T reciprocal(T x)
{
    return T(1) / x;
}
template <>
__device__ __forceinline__ float reciprocal<float>(float x)
{
    const float r = __builtin_amdgcn_rcpf(x);
    return __builtin_fmaf(__builtin_fmaf(-x, r, 1.0f), r, r);
}

// Lattice weight: the tensor product of the 1D weights (1/6, 2/3, 1/6),
// equal to 8/27, 2/27, 1/54, 1/216 for |c|^2 = 0, 1, 2, 3.
__host__ __device__ constexpr double weight(int i)
{
    return (vel_x(i) ? 1.0 / 6.0 : 2.0 / 3.0) * (vel_y(i) ? 1.0 / 6.0 : 2.0 / 3.0) *
           (vel_z(i) ? 1.0 / 6.0 : 2.0 / 3.0);
}

// Inverse of the 1D central-moment map on {-1, 0, +1} shifted by u:
// (m0, m1, m2) = sum g * (1, c - u, (c - u)^2)  ->  (g-, g0, g+).
template <typename T>
__device__ __forceinline__ void inv1d(T m0, T m1, T m2, T u, T& gm, T& g0, T& gp)
{
    const T odd = m1 + u * m0;                     // g+ - g-
    const T even = m2 + u * (T(2) * m1 + u * m0);  // g+ + g-
    gm = T(0.5) * (even - odd);
    g0 = m0 - even;
    gp = T(0.5) * (even + odd);
}

// inv1d with its first- and second-order inputs given at half scale
// (m1h = m1 / 2, m2h = m2 / 2) and hu = u / 2: with o = (g+ - g-) / 2 and
// e = (g+ + g-) / 2, o = m1h + hu m0, e = m2h + u (m1h + o), g-+ = e -+ o,
// g0 = m0 - 2 e.  Six operations instead of nine; the halving is folded into
// the construction of the moments (see reconstruct).
template <typename T>
__device__ __forceinline__ void inv1d_half(T m0, T m1h, T m2h, T u, T hu, T& gm, T& g0, T& gp)
{
    const T o = m1h + hu * m0;
    const T e = m2h + u * (m1h + o);
    gm = e - o;
    gp = e + o;
    g0 = m0 - T(2) * e;
}

// First half of the collision: density, half-force-corrected velocity
// (eq. "macroscopic") and the five pre-collision central moments k4..k8
// (eq. "pre_collision") of the pre-collision h_i = f_i - w_i rho0.
template <typename T>
__device__ __forceinline__ void pre_collision(const T h[27], T Fx, T Fy, T Fz, T rho0, T& drho, T& ux, T& uy, T& uz,
                                              T k[5])
{
    // Raw moments of h up to second order, by three 1D sums (x, then y, then z).
    T X[3][3][3];  // X[p][b][c] = sum_a h(a,b,c) a^p
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T hm = h[vel_index(-1, b - 1, c - 1)];
            const T h0 = h[vel_index(0, b - 1, c - 1)];
            const T hp = h[vel_index(1, b - 1, c - 1)];
            X[0][b][c] = hm + h0 + hp;
            X[1][b][c] = hp - hm;
            X[2][b][c] = hp + hm;
        }
    T Y[3][3][3];  // Y[p][q][c]
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Y[p][0][c] = X[p][0][c] + X[p][1][c] + X[p][2][c];
            Y[p][1][c] = X[p][2][c] - X[p][0][c];
            Y[p][2][c] = X[p][2][c] + X[p][0][c];
        }
    auto zsum = [&](int p, int q, int r) -> T {
        if (r == 0) return Y[p][q][0] + Y[p][q][1] + Y[p][q][2];
        if (r == 1) return Y[p][q][2] - Y[p][q][0];
        return Y[p][q][2] + Y[p][q][0];
    };
    drho = zsum(0, 0, 0);
    const T jx = zsum(1, 0, 0), jy = zsum(0, 1, 0), jz = zsum(0, 0, 1);
    const T Sxx = zsum(2, 0, 0), Syy = zsum(0, 2, 0), Szz = zsum(0, 0, 2);
    const T Sxy = zsum(1, 1, 0), Sxz = zsum(1, 0, 1), Syz = zsum(0, 1, 1);

    // Macroscopic variables with the half-force correction (eq. "macroscopic").
    const T rho = rho0 + drho;
    const T inv_rho = reciprocal(rho);
    ux = (jx + T(0.5) * Fx) * inv_rho;
    uy = (jy + T(0.5) * Fy) * inv_rho;
    uz = (jz + T(0.5) * Fz) * inv_rho;

    // The five pre-collision central moments k4..k8 from raw moments:
    // sum f (cx-ux)(cy-uy) = Pxy - rho ux uy + (ux Fy + uy Fx)/2, where the
    // rest state contributes nothing to Pxy or Pxx - Pyy.
    k[0] = Sxy - rho * ux * uy + T(0.5) * (ux * Fy + uy * Fx);
    k[1] = Sxz - rho * ux * uz + T(0.5) * (ux * Fz + uz * Fx);
    k[2] = Syz - rho * uy * uz + T(0.5) * (uy * Fz + uz * Fy);
    k[3] = (Sxx - Syy) - rho * (ux * ux - uy * uy) + (ux * Fx - uy * Fy);
    k[4] = (Sxx - Szz) - rho * (ux * ux - uz * uz) + (ux * Fx - uz * Fz);
}

// Second half: the post-collision populations h*_i = f*_i - w_i rho0 from
// the density deviation, the velocity, the force density and the relaxed
// shear moments s = (1 - omega) k4..k8, i.e. the nineteen non-zero
// post-collision central moments (eq. "post_collision_central_moments_forcing")
// and their inverse transform (eq. "system").
template <typename T>
__device__ __forceinline__ void reconstruct(T drho, T ux, T uy, T uz, T Fx, T Fy, T Fz, const T s[5], T rho0, T h[27])
{
    // Post-collision central moments on the monomials (cx-ux)^p (cy-uy)^q (cz-uz)^r,
    // minus the central moments of the rest state rho0 w_i, which factor as
    // rho0 M_p(ux) M_q(uy) M_r(uz) with M_0 = 1, M_1(u) = -u, M_2(u) = 1/3 + u^2.
    // D[p][q][r] is held at scale 2^-(number of non-zero p, q, r): each of the
    // three 1D passes below then receives its first- and second-order inputs
    // at half scale (inv1d_half), and by linearity the populations come out
    // unscaled.  The scale factors are powers of two, so they round nothing.
    const T third = T(1.0 / 3.0);
    const T ux2 = ux * ux, uy2 = uy * uy, uz2 = uz * uz;
    const T ax = third + ux2, ay = third + uy2, az = third + uz2;
    const T r1 = T(0.5) * rho0, r2 = T(0.25) * rho0, r3 = T(0.125) * rho0;
    T D[3][3][3];
    D[0][0][0] = drho;
    D[1][0][0] = T(0.25) * Fx + r1 * ux;
    D[0][1][0] = T(0.25) * Fy + r1 * uy;
    D[0][0][1] = T(0.25) * Fz + r1 * uz;
    D[1][1][0] = T(0.25) * s[0] - r2 * ux * uy;
    D[1][0][1] = T(0.25) * s[1] - r2 * ux * uz;
    D[0][1][1] = T(0.25) * s[2] - r2 * uy * uz;
    const T sixth = T(1.0 / 6.0);
    D[2][0][0] = (s[3] + s[4] + drho) * sixth - r1 * ux2;
    D[0][2][0] = (s[4] - T(2) * s[3] + drho) * sixth - r1 * uy2;
    D[0][0][2] = (s[3] - T(2) * s[4] + drho) * sixth - r1 * uz2;
    const T f24 = T(1.0 / 24.0);
    D[1][2][0] = f24 * Fx + r2 * ux * ay;
    D[1][0][2] = f24 * Fx + r2 * ux * az;
    D[2][1][0] = f24 * Fy + r2 * uy * ax;
    D[0][1][2] = f24 * Fy + r2 * uy * az;
    D[2][0][1] = f24 * Fz + r2 * uz * ax;
    D[0][2][1] = f24 * Fz + r2 * uz * ay;
    D[1][1][1] = r3 * ux * uy * uz;
    const T f36 = T(1.0 / 36.0);
    D[2][2][0] = f36 * drho - r2 * ((ux2 + uy2) * third + ux2 * uy2);
    D[2][0][2] = f36 * drho - r2 * ((ux2 + uz2) * third + ux2 * uz2);
    D[0][2][2] = f36 * drho - r2 * ((uy2 + uz2) * third + uy2 * uz2);
    D[2][1][1] = -r3 * ax * uy * uz;
    D[1][2][1] = -r3 * ay * ux * uz;
    D[1][1][2] = -r3 * az * ux * uy;
    const T f144 = T(1.0 / 144.0);
    D[1][2][2] = f144 * Fx + r3 * ux * ay * az;
    D[2][1][2] = f144 * Fy + r3 * uy * ax * az;
    D[2][2][1] = f144 * Fz + r3 * uz * ax * ay;
    D[2][2][2] = T(1.0 / 216.0) * drho -
                 r3 * ((ux2 + uy2 + uz2) * (T(1.0 / 9.0)) + (ux2 * uy2 + ux2 * uz2 + uy2 * uz2) * third + ux2 * uy2 * uz2);

    // Reconstruction (eq. "system") by the factorised inverse transform:
    // along z, then y, then x.
    const T hx = T(0.5) * ux, hy = T(0.5) * uy, hz = T(0.5) * uz;
    T A[3][3][3];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q)
            inv1d_half(D[p][q][0], D[p][q][1], D[p][q][2], uz, hz, A[p][q][0], A[p][q][1], A[p][q][2]);
    T B[3][3][3];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            inv1d_half(A[p][0][c], A[p][1][c], A[p][2][c], uy, hy, B[p][0][c], B[p][1][c], B[p][2][c]);
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            inv1d_half(B[0][b][c], B[1][b][c], B[2][b][c], ux, hx, h[vel_index(-1, b - 1, c - 1)],
                       h[vel_index(0, b - 1, c - 1)], h[vel_index(1, b - 1, c - 1)]);
}

// Collide one cell in place.
//   h[27]   in: pre-collision h_i = f_i - w_i rho0; out: post-collision h*_i
//   F       force density at the cell
//   omega   1/tau
//   rho0    reference density of the shift
// Outputs the density and the half-force-corrected velocity as well.
template <typename T>
__device__ __forceinline__ void collide(T h[27], T Fx, T Fy, T Fz, T omega, T rho0, T& rho_out, T& ux_out,
                                        T& uy_out, T& uz_out)
{
    T drho, ux, uy, uz, k[5];
    pre_collision(h, Fx, Fy, Fz, rho0, drho, ux, uy, uz, k);
    rho_out = rho0 + drho;
    ux_out = ux;
    uy_out = uy;
    uz_out = uz;
    const T om1 = T(1) - omega;
    T s[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) s[j] = om1 * k[j];
    reconstruct(drho, ux, uy, uz, Fx, Fy, Fz, s, rho0, h);
}

// Forward 1D central-moment map on {-1, 0, +1} shifted by u:
// (g-, g0, g+) -> (sum g, sum g (c - u), sum g (c - u)^2).
template <typename T>
__device__ __forceinline__ void fwd1d(T gm, T g0, T gp, T u, T& m0, T& m1, T& m2)
{
    m0 = gm + g0 + gp;
    const T odd = gp - gm, even = gp + gm;
    m1 = odd - u * m0;
    m2 = even - T(2) * u * odd + u * u * m0;
}

// Central monomial moments M[p][q][r] = sum_i g_i (cx-ux)^p (cy-uy)^q (cz-uz)^r,
// by three 1D maps (x, then y, then z).
template <typename T>
__device__ __forceinline__ void central_monomials(const T g[27], T ux, T uy, T uz, T M[3][3][3])
{
    T A[3][3][3];
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            fwd1d(g[vel_index(-1, b - 1, c - 1)], g[vel_index(0, b - 1, c - 1)], g[vel_index(1, b - 1, c - 1)], ux,
                  A[0][b][c], A[1][b][c], A[2][b][c]);
    T B[3][3][3];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int c = 0; c < 3; ++c) fwd1d(A[p][0][c], A[p][1][c], A[p][2][c], uy, B[p][0][c], B[p][1][c], B[p][2][c]);
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q) fwd1d(B[p][q][0], B[p][q][1], B[p][q][2], uz, M[p][q][0], M[p][q][1], M[p][q][2]);
}

// Collision of the comparison models of Sec. III: the same central-moment
// relaxation (omega on k4..k8, 1 on every other moment) with the equilibrium
// and the forcing term truncated in Hermite order.  EQ2: second-order
// equilibrium instead of the complete one; GUO: second-order (H1 + H2, Guo)
// forcing instead of the complete one.  (GUO: M4; EQ2 + GUO: M5.)  BGK:
// every moment relaxes with omega instead (the single-relaxation-time
// stability control), done directly on the populations.
//
// The truncated equilibrium and forcing have velocity-dependent central
// moments, so instead of a closed table this route builds both as
// populations (the equilibrium in deviation form, f^eq_i - w_i rho0), takes
// their central monomial moments, and relaxes:
//   rate-1 moments:  K* = K^eq + R / 2
//   k4..k8:          k* = (1 - omega) k + omega k^eq + (1 - omega / 2) R
// with k7 = K200 - K020, k8 = K200 - K002 and the trace K200 + K020 + K002
// relaxing at rate 1.  Everything is carried minus the rest state's central
// moments, as in collide().
template <typename T, bool EQ2, bool GUO, bool BGK>
__device__ __forceinline__ void collide_model(T h[27], T Fx, T Fy, T Fz, T omega, T rho0, T& rho_out, T& ux_out,
                                              T& uy_out, T& uz_out)
{
    // density, velocity and the pre-collision second-order central moments, as in collide()
    T X[3][3][3];
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T hm = h[vel_index(-1, b - 1, c - 1)];
            const T h0 = h[vel_index(0, b - 1, c - 1)];
            const T hp = h[vel_index(1, b - 1, c - 1)];
            X[0][b][c] = hm + h0 + hp;
            X[1][b][c] = hp - hm;
            X[2][b][c] = hp + hm;
        }
    T Y[3][3][3];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Y[p][0][c] = X[p][0][c] + X[p][1][c] + X[p][2][c];
            Y[p][1][c] = X[p][2][c] - X[p][0][c];
            Y[p][2][c] = X[p][2][c] + X[p][0][c];
        }
    auto zsum = [&](int p, int q, int r) -> T {
        if (r == 0) return Y[p][q][0] + Y[p][q][1] + Y[p][q][2];
        if (r == 1) return Y[p][q][2] - Y[p][q][0];
        return Y[p][q][2] + Y[p][q][0];
    };
    const T drho = zsum(0, 0, 0);
    const T jx = zsum(1, 0, 0), jy = zsum(0, 1, 0), jz = zsum(0, 0, 1);
    const T Sxx = zsum(2, 0, 0), Syy = zsum(0, 2, 0), Szz = zsum(0, 0, 2);
    const T Sxy = zsum(1, 1, 0), Sxz = zsum(1, 0, 1), Syz = zsum(0, 1, 1);
    const T rho = rho0 + drho;
    const T inv_rho = reciprocal(rho);
    const T ux = (jx + T(0.5) * Fx) * inv_rho;
    const T uy = (jy + T(0.5) * Fy) * inv_rho;
    const T uz = (jz + T(0.5) * Fz) * inv_rho;
    rho_out = rho;
    ux_out = ux;
    uy_out = uy;
    uz_out = uz;
    const T k4 = Sxy - rho * ux * uy + T(0.5) * (ux * Fy + uy * Fx);
    const T k5 = Sxz - rho * ux * uz + T(0.5) * (ux * Fz + uz * Fx);
    const T k6 = Syz - rho * uy * uz + T(0.5) * (uy * Fz + uz * Fy);
    const T k7 = (Sxx - Syy) - rho * (ux * ux - uy * uy) + (ux * Fx - uy * Fy);
    const T k8 = (Sxx - Szz) - rho * (ux * ux - uz * uz) + (ux * Fx - uz * Fz);

    // equilibrium (deviation form) and forcing populations of the model
    const T ux2 = ux * ux, uy2 = uy * uy, uz2 = uz * uz, usq = ux2 + uy2 + uz2;
    const T uF = ux * Fx + uy * Fy + uz * Fz;
    T e[27], g[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        constexpr T third = T(1.0 / 3.0);
        const int cx = vel_x(i), cy = vel_y(i), cz = vel_z(i);
        const T w = T(weight(i));
        // 1D factors of the complete equilibrium, phi(c, u) = 1 + 3 c u + (9/2)(c^2 - 1/3) u^2, minus 1
        const T ax = T(3 * cx) * ux + T(4.5) * (T(cx * cx) - third) * ux2;
        const T ay = T(3 * cy) * uy + T(4.5) * (T(cy * cy) - third) * uy2;
        const T az = T(3 * cz) * uz + T(4.5) * (T(cz * cz) - third) * uz2;
        const T cu = T(cx) * ux + T(cy) * uy + T(cz) * uz;
        T sm1;  // f^eq_i / (w_i rho) - 1
        if (EQ2)
            sm1 = T(3) * cu + T(4.5) * cu * cu - T(1.5) * usq;
        else
            sm1 = ax + ay + az + ax * ay + ax * az + ay * az + ax * ay * az;
        e[i] = w * (drho + rho * sm1);
        const T cF = T(cx) * Fx + T(cy) * Fy + T(cz) * Fz;
        if (GUO) {
            g[i] = w * (T(3) * (cF - uF) + T(9) * cu * cF);
        } else {
            // F . grad_u of the complete (product-form) equilibrium at rho = 1
            const T dx = T(3 * cx) + T(9) * (T(cx * cx) - third) * ux;
            const T dy = T(3 * cy) + T(9) * (T(cy * cy) - third) * uy;
            const T dz = T(3 * cz) + T(9) * (T(cz * cz) - third) * uz;
            g[i] = w * (Fx * dx * (T(1) + ay) * (T(1) + az) + Fy * (T(1) + ax) * dy * (T(1) + az) +
                        Fz * (T(1) + ax) * (T(1) + ay) * dz);
        }
    }
    if (BGK) {
        // every moment relaxes with omega: in population space h* = h - omega (h - e) + (1 - omega / 2) g
        const T hf = T(1) - T(0.5) * omega;
#pragma unroll
        for (int i = 0; i < 27; ++i) h[i] = h[i] - omega * (h[i] - e[i]) + hf * g[i];
        return;
    }
    T De[3][3][3], R[3][3][3];
    central_monomials(e, ux, uy, uz, De);
    central_monomials(g, ux, uy, uz, R);

    T D[3][3][3];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int r = 0; r < 3; ++r) D[p][q][r] = De[p][q][r] + T(0.5) * R[p][q][r];
    // second-order block; the rest state's central moments are rho0 (ux uy, ..., 1/3 + ux^2, ...)
    const T om1 = T(1) - omega, hf = T(1) - T(0.5) * omega, third = T(1.0 / 3.0);
    const T r110 = rho0 * ux * uy, r101 = rho0 * ux * uz, r011 = rho0 * uy * uz;
    D[1][1][0] = om1 * (k4 - r110) + omega * De[1][1][0] + hf * R[1][1][0];
    D[1][0][1] = om1 * (k5 - r101) + omega * De[1][0][1] + hf * R[1][0][1];
    D[0][1][1] = om1 * (k6 - r011) + omega * De[0][1][1] + hf * R[0][1][1];
    const T keq7 = De[2][0][0] - De[0][2][0] + rho0 * (ux2 - uy2);
    const T keq8 = De[2][0][0] - De[0][0][2] + rho0 * (ux2 - uz2);
    const T k7s = om1 * k7 + omega * keq7 + hf * (R[2][0][0] - R[0][2][0]);
    const T k8s = om1 * k8 + omega * keq8 + hf * (R[2][0][0] - R[0][0][2]);
    const T d9 = De[2][0][0] + De[0][2][0] + De[0][0][2] + T(0.5) * (R[2][0][0] + R[0][2][0] + R[0][0][2]);
    D[2][0][0] = (d9 + k7s + k8s) * third + rho0 * (uy2 + uz2 - T(2) * ux2) * third;
    D[0][2][0] = (d9 - T(2) * k7s + k8s) * third + rho0 * (ux2 + uz2 - T(2) * uy2) * third;
    D[0][0][2] = (d9 + k7s - T(2) * k8s) * third + rho0 * (ux2 + uy2 - T(2) * uz2) * third;

    T A[3][3][3];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q) inv1d(D[p][q][0], D[p][q][1], D[p][q][2], uz, A[p][q][0], A[p][q][1], A[p][q][2]);
    T B[3][3][3];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int c = 0; c < 3; ++c) inv1d(A[p][0][c], A[p][1][c], A[p][2][c], uy, B[p][0][c], B[p][1][c], B[p][2][c]);
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            inv1d(B[0][b][c], B[1][b][c], B[2][b][c], ux, h[vel_index(-1, b - 1, c - 1)], h[vel_index(0, b - 1, c - 1)],
                  h[vel_index(1, b - 1, c - 1)]);
}

}  // namespace cmlbm
