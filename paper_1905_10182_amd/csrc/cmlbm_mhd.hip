// Magnetic-field lattice of App. C (D3Q7 vector populations, BGK) and the
// Lorentz force that couples it to the fluid, for gfx950 (MI355X).
// De Rosis, Huang & Coreixas, PRE 2019.  C ABI: include/cmlbm_mhd.h.
//
// Data layout in HBM: 21 planes (velocity l, component a) of nz * ny rows,
// each row padded to 256 bytes, in the storage type; two buffers alternate.
// As in the fluid solver the stored array is in pull form: A_l(y) holds the
// population that the next gather moves to y + xi_l, so h_l(x, t) =
// A_l(x - xi_l) and a step stores its post-collision values at the cell's own
// index.  All kernels are one thread per cell over the unpadded cell index
// (x fastest, so a wave reads 64 consecutive cells of a row).
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <string>

#include "cmlbm_mhd.h"

namespace {

constexpr int kBlock = 256;

// D3Q7 velocities in the order of App. C: rest, +x, -x, +y, -y, +z, -z.
__host__ __device__ constexpr int xi(int l, int a)
{
    constexpr int v[7][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
    return v[l][a];
}
// Weights of App. C: 1/4 at rest, 1/8 on the links; cs^2 = 1/4.
__host__ __device__ constexpr double wm(int l) { return l == 0 ? 0.25 : 0.125; }

struct GeomM {
    int nx, ny, nz;
    int nxp;           // padded row length (elements)
    uint64_t pstride;  // elements from population k to k + 1 of one row
    uint64_t rstride;  // elements from one row of a population to the next row
    uint64_t ncell;    // nz * ny * nx
    int wall[3];       // per axis: 0 periodic, 1 walls halfway outside the first and last node
    double bw[3];      // field imposed at the walls
    double f0[3];      // uniform force density added to the Lorentz force
};

// opposite D3Q7 direction: rest, then the pairs (+x, -x), (+y, -y), (+z, -z)
__host__ __device__ constexpr int opp(int l) { return l == 0 ? 0 : ((l & 1) ? l + 1 : l - 1); }

// Does the link from (x, y, z) against xi_l leave the box through a wall?
__device__ __forceinline__ bool from_wall(const GeomM& g, int x, int y, int z, int l)
{
    const int s[3] = {x - xi(l, 0), y - xi(l, 1), z - xi(l, 2)};
    const int n[3] = {g.nx, g.ny, g.nz};
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (g.wall[a] && (s[a] < 0 || s[a] >= n[a])) return true;
    return false;
}

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

__device__ __forceinline__ void coords(const GeomM& g, uint64_t n, int& x, int& y, int& z)
{
    x = (int)(n % (uint64_t)g.nx);
    const uint64_t r = n / (uint64_t)g.nx;
    y = (int)(r % (uint64_t)g.ny);
    z = (int)(r / (uint64_t)g.ny);
}

__device__ __forceinline__ uint64_t plane_off(const GeomM& g, int x, int y, int z)
{
    return ((uint64_t)z * (uint64_t)g.ny + (uint64_t)y) * g.rstride + (uint64_t)x;
}

// Pull gather: h_l(x) = A_l(x - xi_l) across periodic axes.  A link coming
// in through a wall (the field is imposed there) is the anti-bounce-back of
// the population that left towards it: h_l(x) = -h*_opp(l)(x) + 2 w_l b_w,
// which puts the Dirichlet value at the half-way wall.
template <typename T>
__device__ __forceinline__ void gather(const T* __restrict__ A, const GeomM& g, int x, int y, int z, T h[7][3])
{
#pragma unroll
    for (int l = 0; l < 7; ++l) {
        if (l > 0 && from_wall(g, x, y, z, l)) {
            const uint64_t own = plane_off(g, x, y, z);
#pragma unroll
            for (int a = 0; a < 3; ++a)
                h[l][a] = -A[(uint64_t)(3 * opp(l) + a) * g.pstride + own] + T(2.0 * wm(l) * g.bw[a]);
            continue;
        }
        const uint64_t s = plane_off(g, wrap(x - xi(l, 0), g.nx), wrap(y - xi(l, 1), g.ny), wrap(z - xi(l, 2), g.nz));
#pragma unroll
        for (int a = 0; a < 3; ++a) h[l][a] = A[(uint64_t)(3 * l + a) * g.pstride + s];
    }
}

template <typename T>
__device__ __forceinline__ void field_b(const T h[7][3], T b[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        T s = T(0);
#pragma unroll
        for (int l = 0; l < 7; ++l) s += h[l][a];
        b[a] = s;
    }
}

// Equilibrium of App. C: e_la = w_l [b_a + (1/cs^2) xi_lc (u_c b_a - b_c u_a)].
template <typename T>
__device__ __forceinline__ void equilibrium(const T b[3], const T u[3], T e[7][3])
{
#pragma unroll
    for (int l = 0; l < 7; ++l)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            T s = T(0);
#pragma unroll
            for (int c = 0; c < 3; ++c)
                if (xi(l, c)) s += T(xi(l, c)) * (u[c] * b[a] - b[c] * u[a]);
            e[l][a] = T(wm(l)) * (b[a] + T(4) * s);
        }
}

template <typename T>
__device__ __forceinline__ void load_vec(const T* __restrict__ v, const GeomM& g, uint64_t n, T out[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) out[a] = v ? v[(uint64_t)a * g.ncell + n] : T(0);
}

template <typename T>
__device__ __forceinline__ void store_nt(T* p, T v)
{
    if constexpr (sizeof(T) == 8)
        __builtin_nontemporal_store(__builtin_bit_cast(unsigned long long, v), (unsigned long long*)p);
    else
        __builtin_nontemporal_store(__builtin_bit_cast(unsigned, v), (unsigned*)p);
}

// h = h^eq(b, u) or imported FP64 populations, written through the inverse
// of the pull gather: A_l(x - xi_l) = h_l(x), or for a link coming in through
// a wall A_opp(l)(x) = 2 w_l b_w - h_l(x).
template <typename T, bool POPS>
__global__ __launch_bounds__(kBlock) void k_mhd_init(T* __restrict__ dst, GeomM g, const T* __restrict__ b_in,
                                                     const T* __restrict__ u_in, const double* __restrict__ pops)
{
    const uint64_t n = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.ncell) return;
    int x, y, z;
    coords(g, n, x, y, z);
    T e[7][3];
    if constexpr (POPS) {
#pragma unroll
        for (int l = 0; l < 7; ++l)
#pragma unroll
            for (int a = 0; a < 3; ++a) e[l][a] = (T)pops[(uint64_t)(3 * l + a) * g.ncell + n];
    } else {
        T b[3], u[3];
        load_vec(b_in, g, n, b);
        load_vec(u_in, g, n, u);
        equilibrium(b, u, e);
    }
#pragma unroll
    for (int l = 0; l < 7; ++l) {
        if (l > 0 && from_wall(g, x, y, z, l)) {
            const uint64_t own = plane_off(g, x, y, z);
#pragma unroll
            for (int a = 0; a < 3; ++a)
                dst[(uint64_t)(3 * opp(l) + a) * g.pstride + own] = T(2.0 * wm(l) * g.bw[a]) - e[l][a];
            continue;
        }
        const uint64_t d = plane_off(g, wrap(x - xi(l, 0), g.nx), wrap(y - xi(l, 1), g.ny), wrap(z - xi(l, 2), g.nz));
#pragma unroll
        for (int a = 0; a < 3; ++a) dst[(uint64_t)(3 * l + a) * g.pstride + d] = e[l][a];
    }
}

// One step: gather, BGK collision towards h^eq(b, u), store at the own index.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_mhd_step(const T* __restrict__ src, T* __restrict__ dst, GeomM g,
                                                     T omega, const T* __restrict__ u_in)
{
    const uint64_t n = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.ncell) return;
    int x, y, z;
    coords(g, n, x, y, z);
    T h[7][3], b[3], u[3], e[7][3];
    gather(src, g, x, y, z, h);
    field_b(h, b);
    load_vec(u_in, g, n, u);
    equilibrium(b, u, e);
    const uint64_t own = plane_off(g, x, y, z);
#pragma unroll
    for (int l = 0; l < 7; ++l)
#pragma unroll
        for (int a = 0; a < 3; ++a)
            store_nt(dst + (uint64_t)(3 * l + a) * g.pstride + own, h[l][a] + omega * (e[l][a] - h[l][a]));
}

// F = j x b + f0
template <typename T>
__device__ __forceinline__ void lorentz(const GeomM& g, const T j[3], const T b[3], T F[3])
{
    F[0] = j[1] * b[2] - j[2] * b[1] + T(g.f0[0]);
    F[1] = j[2] * b[0] - j[0] * b[2] + T(g.f0[1]);
    F[2] = j[0] * b[1] - j[1] * b[0] + T(g.f0[2]);
}

template <typename T>
__device__ __forceinline__ void store_vec(T* __restrict__ v, const GeomM& g, uint64_t n, const T w[3])
{
    if (!v) return;
#pragma unroll
    for (int a = 0; a < 3; ++a) v[(uint64_t)a * g.ncell + n] = w[a];
}

// b = sum_l h_l and, with POP, the population current
// j_c = -eps_cba (Lambda - Lambda^eq)_ba / (tau_m cs^2) and F = j x b + f0.
template <typename T, bool POP>
__global__ __launch_bounds__(kBlock) void k_mhd_fields(const T* __restrict__ src, GeomM g, T tau_m,
                                                       const T* __restrict__ u_in, T* __restrict__ b_out,
                                                       T* __restrict__ j_out, T* __restrict__ F_out)
{
    const uint64_t n = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.ncell) return;
    int x, y, z;
    coords(g, n, x, y, z);
    T h[7][3], b[3];
    gather(src, g, x, y, z, h);
    field_b(h, b);
    store_vec(b_out, g, n, b);
    if constexpr (POP) {
        T u[3];
        load_vec(u_in, g, n, u);
        // L[p][a] = sum_l xi_lp h_la - (u_p b_a - b_p u_a); only the +-p links carry xi_lp
        T L[3][3];
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int a = 0; a < 3; ++a) L[p][a] = (h[1 + 2 * p][a] - h[2 + 2 * p][a]) - (u[p] * b[a] - b[p] * u[a]);
        const T k = T(-4) / tau_m;  // -1 / (tau_m cs^2)
        const T j[3] = {k * (L[1][2] - L[2][1]), k * (L[2][0] - L[0][2]), k * (L[0][1] - L[1][0])};
        store_vec(j_out, g, n, j);
        if (F_out) {
            T F[3];
            lorentz(g, j, b, F);
            store_vec(F_out, g, n, F);
        }
    }
}

// Central-difference curl of b ([3][N]; periodic axes, beyond a wall the
// ghost value 2 b_w - b(x); an axis of extent 1 has no derivative) and
// F = j x b.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_mhd_curl(GeomM g, const T* __restrict__ b, T* __restrict__ j_out,
                                                     T* __restrict__ F_out)
{
    const uint64_t n = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.ncell) return;
    int x, y, z;
    coords(g, n, x, y, z);
    const uint64_t row = (uint64_t)g.nx, sl = (uint64_t)g.nx * (uint64_t)g.ny;
    auto at = [&](int xx, int yy, int zz) { return (uint64_t)zz * sl + (uint64_t)yy * row + (uint64_t)xx; };
    const int c[3] = {x, y, z}, ext[3] = {g.nx, g.ny, g.nz};
    // derivative along axis a of component q
    auto d = [&](int a, int q) -> T {
        if (ext[a] < 2) return T(0);
        const T here = b[(uint64_t)q * g.ncell + n];
        T v[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            int p[3] = {x, y, z};
            p[a] = c[a] + (k == 0 ? 1 : -1);
            if (p[a] < 0 || p[a] >= ext[a]) {
                if (g.wall[a]) {
                    v[k] = T(2.0 * g.bw[q]) - here;
                    continue;
                }
                p[a] = wrap(p[a], ext[a]);
            }
            v[k] = b[(uint64_t)q * g.ncell + at(p[0], p[1], p[2])];
        }
        return T(0.5) * (v[0] - v[1]);
    };
    const T j[3] = {d(1, 2) - d(2, 1), d(2, 0) - d(0, 2), d(0, 1) - d(1, 0)};
    store_vec(j_out, g, n, j);
    if (F_out) {
        T bb[3], F[3];
        load_vec(b, g, n, bb);
        lorentz(g, j, bb, F);
        store_vec(F_out, g, n, F);
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_mhd_export(const T* __restrict__ src, GeomM g, double* __restrict__ out)
{
    const uint64_t n = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.ncell) return;
    int x, y, z;
    coords(g, n, x, y, z);
    T h[7][3];
    gather(src, g, x, y, z, h);
#pragma unroll
    for (int l = 0; l < 7; ++l)
#pragma unroll
        for (int a = 0; a < 3; ++a) out[(uint64_t)(3 * l + a) * g.ncell + n] = (double)h[l][a];
}

}  // namespace

struct cmlbm_mhd_lattice {
    cmlbm_mhd_params p;
    GeomM g;
    void* pop[2];
    int cur;
    bool initialized;
    int64_t t;
    std::string err;
};

namespace {

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Population layout: planes (population k of every row together).  Row blocks
// (the 21 population rows of one lattice row stored together), which speed up
// the D3Q27 and D2Q9 steps, measured slower here: 31.0-31.9 against
// 33.0-33.3 GLUPS at 256^3 (FP32, one box, two rounds).
bool row_blocks_mhd(int /*storage*/) { return false; }

int make_geom(const cmlbm_mhd_params* p, GeomM* g, size_t* bytes)
{
    if (!p) return CMLBM_MHD_EINVAL;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return CMLBM_MHD_EINVAL;
    if (!(p->tau_m > 0.5) || !std::isfinite(p->tau_m)) return CMLBM_MHD_EINVAL;
    if (p->storage != CMLBM_MHD_FP64 && p->storage != CMLBM_MHD_FP32) return CMLBM_MHD_EINVAL;
    if (p->flags != 0) return CMLBM_MHD_EINVAL;
    const int dims[3] = {p->nx, p->ny, p->nz};
    for (int a = 0; a < 3; ++a) {
        if (p->wall[a] != CMLBM_MHD_PERIODIC && p->wall[a] != CMLBM_MHD_WALL) return CMLBM_MHD_EINVAL;
        if (p->wall[a] == CMLBM_MHD_WALL && dims[a] < 2) return CMLBM_MHD_EINVAL;
        g->wall[a] = p->wall[a];
        g->bw[a] = 0.0;
        g->f0[a] = 0.0;
    }
    const size_t sb = p->storage == CMLBM_MHD_FP64 ? 8 : 4;
    g->nx = p->nx;
    g->ny = p->ny;
    g->nz = p->nz;
    g->nxp = (int)(align256((size_t)p->nx * sb) / sb);
    const uint64_t plane = (uint64_t)p->nz * (uint64_t)p->ny * (uint64_t)g->nxp;
    if (plane * sb >= (1ULL << 32)) return CMLBM_MHD_EINVAL;
    const bool blocks = row_blocks_mhd(p->storage);
    g->pstride = blocks ? (uint64_t)g->nxp : plane;
    g->rstride = blocks ? 21ull * g->nxp : (uint64_t)g->nxp;
    g->ncell = (uint64_t)p->nz * (uint64_t)p->ny * (uint64_t)p->nx;
    if ((g->ncell + kBlock - 1) / kBlock > 0x7fffffffULL) return CMLBM_MHD_EINVAL;
    if (bytes) *bytes = align256(21 * plane * sb);
    return CMLBM_MHD_OK;
}

int fail(cmlbm_mhd_lattice* lat, int code, const std::string& msg)
{
    if (lat) lat->err = msg;
    return code;
}

int launch_check(cmlbm_mhd_lattice* lat, const char* what)
{
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) return CMLBM_MHD_OK;
    return fail(lat, CMLBM_MHD_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

dim3 cells(const GeomM& g) { return dim3((unsigned)((g.ncell + kBlock - 1) / kBlock)); }

bool aligned256(const void* p) { return ((uintptr_t)p & 255u) == 0; }

template <typename T>
void init_t(cmlbm_mhd_lattice* lat, const void* b, const void* u, const double* pops, hipStream_t s)
{
    T* dst = (T*)lat->pop[lat->cur];
    if (pops)
        k_mhd_init<T, true><<<cells(lat->g), dim3(kBlock), 0, s>>>(dst, lat->g, nullptr, nullptr, pops);
    else
        k_mhd_init<T, false><<<cells(lat->g), dim3(kBlock), 0, s>>>(dst, lat->g, (const T*)b, (const T*)u, nullptr);
}

template <typename T>
void fields_t(cmlbm_mhd_lattice* lat, const void* u, int current, void* b, void* j, void* F, hipStream_t s)
{
    const T* src = (const T*)lat->pop[lat->cur];
    const T tm = (T)lat->p.tau_m;
    if (current == CMLBM_MHD_CURRENT_POPULATIONS) {
        k_mhd_fields<T, true><<<cells(lat->g), dim3(kBlock), 0, s>>>(src, lat->g, tm, (const T*)u, (T*)b, (T*)j,
                                                                     (T*)F);
    } else {
        k_mhd_fields<T, false><<<cells(lat->g), dim3(kBlock), 0, s>>>(src, lat->g, tm, nullptr, (T*)b, nullptr,
                                                                      nullptr);
        if (j || F) k_mhd_curl<T><<<cells(lat->g), dim3(kBlock), 0, s>>>(lat->g, (const T*)b, (T*)j, (T*)F);
    }
}

}  // namespace

extern "C" {

int cmlbm_mhd_required_bytes(const cmlbm_mhd_params* params, size_t* pop_buffer_bytes)
{
    GeomM g;
    size_t bytes = 0;
    const int rc = make_geom(params, &g, &bytes);
    if (rc) return rc;
    if (pop_buffer_bytes) *pop_buffer_bytes = bytes;
    return CMLBM_MHD_OK;
}

int cmlbm_mhd_create(const cmlbm_mhd_params* params, void* pop_a, size_t pop_a_bytes, void* pop_b,
                     size_t pop_b_bytes, cmlbm_mhd_lattice** out)
{
    if (!out) return CMLBM_MHD_EINVAL;
    *out = nullptr;
    GeomM g;
    size_t bytes = 0;
    const int rc = make_geom(params, &g, &bytes);
    if (rc) return rc;
    if (!pop_a || !pop_b || pop_a == pop_b || !aligned256(pop_a) || !aligned256(pop_b)) return CMLBM_MHD_EINVAL;
    if (pop_a_bytes < bytes || pop_b_bytes < bytes) return CMLBM_MHD_ENOMEM;
    cmlbm_mhd_lattice* lat = new (std::nothrow) cmlbm_mhd_lattice();
    if (!lat) return CMLBM_MHD_ENOMEM;
    lat->p = *params;
    lat->g = g;
    lat->pop[0] = pop_a;
    lat->pop[1] = pop_b;
    lat->cur = 0;
    lat->initialized = false;
    lat->t = 0;
    *out = lat;
    return CMLBM_MHD_OK;
}

int cmlbm_mhd_set_wall_field(cmlbm_mhd_lattice* lat, const double* host_b_wall)
{
    if (!lat || !host_b_wall) return CMLBM_MHD_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(host_b_wall[a])) return fail(lat, CMLBM_MHD_EINVAL, "non-finite wall field");
    for (int a = 0; a < 3; ++a) lat->g.bw[a] = host_b_wall[a];
    return CMLBM_MHD_OK;
}

int cmlbm_mhd_set_body_force(cmlbm_mhd_lattice* lat, const double* host_f0)
{
    if (!lat || !host_f0) return CMLBM_MHD_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(host_f0[a])) return fail(lat, CMLBM_MHD_EINVAL, "non-finite body force");
    for (int a = 0; a < 3; ++a) lat->g.f0[a] = host_f0[a];
    return CMLBM_MHD_OK;
}

int cmlbm_mhd_init(cmlbm_mhd_lattice* lat, const void* dev_b, const void* dev_u, void* hip_stream)
{
    if (!lat) return CMLBM_MHD_EINVAL;
    if (!dev_b) return fail(lat, CMLBM_MHD_EINVAL, "init needs dev_b[3][N]");
    hipStream_t s = (hipStream_t)hip_stream;
    if (lat->p.storage == CMLBM_MHD_FP64)
        init_t<double>(lat, dev_b, dev_u, nullptr, s);
    else
        init_t<float>(lat, dev_b, dev_u, nullptr, s);
    const int rc = launch_check(lat, "init");
    if (rc) return rc;
    lat->initialized = true;
    lat->t = 0;
    return CMLBM_MHD_OK;
}

int cmlbm_mhd_fields(cmlbm_mhd_lattice* lat, const void* dev_u, int current, void* dev_b, void* dev_j, void* dev_F,
                     void* hip_stream)
{
    if (!lat) return CMLBM_MHD_EINVAL;
    if (current != CMLBM_MHD_CURRENT_POPULATIONS && current != CMLBM_MHD_CURRENT_STENCIL)
        return fail(lat, CMLBM_MHD_EINVAL, "unknown current kind");
    if (current == CMLBM_MHD_CURRENT_STENCIL && !dev_b && (dev_j || dev_F))
        return fail(lat, CMLBM_MHD_EINVAL, "the stencil current needs dev_b");
    if (!lat->initialized) return fail(lat, CMLBM_MHD_ESTATE, "fields before init");
    hipStream_t s = (hipStream_t)hip_stream;
    if (lat->p.storage == CMLBM_MHD_FP64)
        fields_t<double>(lat, dev_u, current, dev_b, dev_j, dev_F, s);
    else
        fields_t<float>(lat, dev_u, current, dev_b, dev_j, dev_F, s);
    return launch_check(lat, "fields");
}

int cmlbm_mhd_step(cmlbm_mhd_lattice* lat, const void* dev_u, void* hip_stream)
{
    if (!lat) return CMLBM_MHD_EINVAL;
    if (!lat->initialized) return fail(lat, CMLBM_MHD_ESTATE, "step before init");
    hipStream_t s = (hipStream_t)hip_stream;
    const int nxt = 1 - lat->cur;
    if (lat->p.storage == CMLBM_MHD_FP64)
        k_mhd_step<double><<<cells(lat->g), dim3(kBlock), 0, s>>>((const double*)lat->pop[lat->cur],
                                                                  (double*)lat->pop[nxt], lat->g,
                                                                  1.0 / lat->p.tau_m, (const double*)dev_u);
    else
        k_mhd_step<float><<<cells(lat->g), dim3(kBlock), 0, s>>>((const float*)lat->pop[lat->cur],
                                                                 (float*)lat->pop[nxt], lat->g,
                                                                 (float)(1.0 / lat->p.tau_m), (const float*)dev_u);
    const int rc = launch_check(lat, "step");
    if (rc) return rc;
    lat->cur = nxt;
    ++lat->t;
    return CMLBM_MHD_OK;
}

int cmlbm_mhd_populations(cmlbm_mhd_lattice* lat, double* dev_out, void* hip_stream)
{
    if (!lat || !dev_out) return CMLBM_MHD_EINVAL;
    if (!lat->initialized) return fail(lat, CMLBM_MHD_ESTATE, "populations before init");
    hipStream_t s = (hipStream_t)hip_stream;
    if (lat->p.storage == CMLBM_MHD_FP64)
        k_mhd_export<double><<<cells(lat->g), dim3(kBlock), 0, s>>>((const double*)lat->pop[lat->cur], lat->g, dev_out);
    else
        k_mhd_export<float><<<cells(lat->g), dim3(kBlock), 0, s>>>((const float*)lat->pop[lat->cur], lat->g, dev_out);
    return launch_check(lat, "populations");
}

int cmlbm_mhd_load_populations(cmlbm_mhd_lattice* lat, const double* dev_in, void* hip_stream)
{
    if (!lat || !dev_in) return CMLBM_MHD_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    if (lat->p.storage == CMLBM_MHD_FP64)
        init_t<double>(lat, nullptr, nullptr, dev_in, s);
    else
        init_t<float>(lat, nullptr, nullptr, dev_in, s);
    const int rc = launch_check(lat, "load populations");
    if (rc) return rc;
    lat->initialized = true;
    return CMLBM_MHD_OK;
}

int cmlbm_mhd_get_time(const cmlbm_mhd_lattice* lat, int64_t* t)
{
    if (!lat || !t) return CMLBM_MHD_EINVAL;
    *t = lat->t;
    return CMLBM_MHD_OK;
}

int cmlbm_mhd_destroy(cmlbm_mhd_lattice* lat)
{
    delete lat;
    return CMLBM_MHD_OK;
}

const char* cmlbm_mhd_last_error(const cmlbm_mhd_lattice* lat) { return lat ? lat->err.c_str() : ""; }

const char* cmlbm_mhd_status_string(int status)
{
    switch (status) {
        case CMLBM_MHD_OK: return "CMLBM_MHD_OK";
        case CMLBM_MHD_EINVAL: return "CMLBM_MHD_EINVAL";
        case CMLBM_MHD_ENOMEM: return "CMLBM_MHD_ENOMEM";
        case CMLBM_MHD_EHIP: return "CMLBM_MHD_EHIP";
        case CMLBM_MHD_ESTATE: return "CMLBM_MHD_ESTATE";
        default: return "CMLBM_MHD_UNKNOWN";
    }
}

}  // extern "C"
