// D2Q9 lattice constants and the per-cell collision of the two-dimensional
// central-moment lattice Boltzmann model with Hermite forcing (De Rosis, Huang
// & Coreixas, PRE 2019, App. B), for register-resident evaluation on gfx950.
//
// Deviation form, as in the three-dimensional solver: populations are handled
// as h_i = f_i - w_i rho0 and every central moment is carried minus its value
// for the rest state, so FP32 keeps its relative precision on the small
// quantities that carry the flow.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "d3q27.hpp"  // inv1d: the 1D inverse central-moment map on {-1, 0, +1}

namespace cmlbm2d {

// Velocity components in the order of App. B.
__host__ __device__ constexpr int vel_x(int i)
{
    constexpr int v[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
    return v[i];
}
__host__ __device__ constexpr int vel_y(int i)
{
    constexpr int v[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
    return v[i];
}
// Index of the velocity (a, b), each in {-1, 0, 1}.
__host__ __device__ constexpr int vel_index(int a, int b)
{
    for (int i = 0; i < 9; ++i)
        if (vel_x(i) == a && vel_y(i) == b) return i;
    return -1;
}
// Lattice weight: the product of the 1D weights (1/6, 2/3, 1/6), i.e. 4/9,
// 1/9, 1/36 for |c|^2 = 0, 1, 2.
__host__ __device__ constexpr double weight(int i)
{
    return (vel_x(i) ? 1.0 / 6.0 : 2.0 / 3.0) * (vel_y(i) ? 1.0 / 6.0 : 2.0 / 3.0);
}

// Density deviation, half-force-corrected velocity and the two pre-collision
// central moments that relax with omega, k4 = sum f [(cx-ux)^2 - (cy-uy)^2]
// and k5 = sum f (cx-ux)(cy-uy), of the pre-collision h.
template <typename T>
__device__ __forceinline__ void pre_collision(const T h[9], T Fx, T Fy, T rho0, T& drho, T& ux, T& uy, T& k4, T& k5)
{
    T X[3][3];  // X[p][b] = sum over cx of h(cx, b - 1) cx^p
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const T hm = h[vel_index(-1, b - 1)];
        const T h0 = h[vel_index(0, b - 1)];
        const T hp = h[vel_index(1, b - 1)];
        X[0][b] = hm + h0 + hp;
        X[1][b] = hp - hm;
        X[2][b] = hp + hm;
    }
    drho = X[0][0] + X[0][1] + X[0][2];
    const T jx = X[1][0] + X[1][1] + X[1][2];
    const T jy = X[0][2] - X[0][0];
    const T Sxx = X[2][0] + X[2][1] + X[2][2];
    const T Syy = X[0][2] + X[0][0];
    const T Sxy = X[1][2] - X[1][0];
    const T rho = rho0 + drho;
    const T inv_rho = T(1) / rho;
    ux = (jx + T(0.5) * Fx) * inv_rho;
    uy = (jy + T(0.5) * Fy) * inv_rho;
    // central from raw moments; the rest state adds nothing to Sxx - Syy or Sxy
    k4 = (Sxx - Syy) - rho * (ux * ux - uy * uy) + (ux * Fx - uy * Fy);
    k5 = Sxy - rho * ux * uy + T(0.5) * (ux * Fy + uy * Fx);
}

// Post-collision h*_i = f*_i - w_i rho0 from the density deviation, the
// velocity, the force density and the relaxed moments s4 = (1 - omega) k4,
// s5 = (1 - omega) k5: the printed post-collision central moments of App. B
// (k0* = rho, k1,2* = F/2, k3* = 2 rho cs^2, k4,5* = s4,5, k6* = Fy cs^2/2,
// k7* = Fx cs^2/2, k8* = rho cs^4) on the monomials (cx-ux)^p (cy-uy)^q, minus
// the rest-state moments rho0 M_p(ux) M_q(uy) (M_0 = 1, M_1(u) = -u,
// M_2(u) = 1/3 + u^2), then the inverse transform along y and along x.
// As in the D3Q27 reconstruction, D[p][q] is held at scale 2^-(number of
// non-zero p, q) so that both 1D passes take their first- and second-order
// inputs at half scale (cmlbm::inv1d_half); the populations come out unscaled.
template <typename T>
__device__ __forceinline__ void reconstruct(T drho, T ux, T uy, T Fx, T Fy, T s4, T s5, T rho0, T h[9])
{
    const T third = T(1.0 / 3.0);
    const T ux2 = ux * ux, uy2 = uy * uy;
    const T r1 = T(0.5) * rho0, r2 = T(0.25) * rho0;
    T D[3][3];
    D[0][0] = drho;
    D[1][0] = T(0.25) * Fx + r1 * ux;
    D[0][1] = T(0.25) * Fy + r1 * uy;
    D[2][0] = drho * T(1.0 / 6.0) + T(0.25) * s4 - r1 * ux2;
    D[0][2] = drho * T(1.0 / 6.0) - T(0.25) * s4 - r1 * uy2;
    D[1][1] = T(0.25) * s5 - r2 * ux * uy;
    D[2][1] = Fy * T(1.0 / 24.0) + r2 * uy * (third + ux2);
    D[1][2] = Fx * T(1.0 / 24.0) + r2 * ux * (third + uy2);
    D[2][2] = drho * T(1.0 / 36.0) - r2 * ((ux2 + uy2) * third + ux2 * uy2);
    const T hx = T(0.5) * ux, hy = T(0.5) * uy;
    T G[3][3];  // G[p][cy + 1]: x-moment p of the populations with that cy (at scale 2^-[p > 0])
#pragma unroll
    for (int p = 0; p < 3; ++p) cmlbm::inv1d_half<T>(D[p][0], D[p][1], D[p][2], uy, hy, G[p][0], G[p][1], G[p][2]);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        T gm, g0, gp;
        cmlbm::inv1d_half<T>(G[0][b], G[1][b], G[2][b], ux, hx, gm, g0, gp);
        h[vel_index(-1, b - 1)] = gm;
        h[vel_index(0, b - 1)] = g0;
        h[vel_index(1, b - 1)] = gp;
    }
}

// One collision in place: h (pre-collision) -> h* (post-collision); returns
// the density deviation and velocity of the cell.
template <typename T>
__device__ __forceinline__ void collide(T h[9], T Fx, T Fy, T omega, T rho0, T& drho, T& ux, T& uy)
{
    T k4, k5;
    pre_collision<T>(h, Fx, Fy, rho0, drho, ux, uy, k4, k5);
    const T r = T(1) - omega;
    reconstruct<T>(drho, ux, uy, Fx, Fy, r * k4, r * k5, rho0, h);
}

}  // namespace cmlbm2d
