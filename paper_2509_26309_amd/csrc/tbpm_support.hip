// Support kernels of the TBPM library (gfx950): initial states, packing of
// given states, correlation sums and their fixed-order reductions, Chebyshev
// moment reductions, quasi-eigenstate accumulation, the LDOS gather, and the
// analysis and format conversion of an uploaded Hamiltonian.  The Chebyshev
// term kernels themselves are in tbpm_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "tbpm_device.h"

namespace tbpm {

// ---- random-phase initial states -----------------------------------------------------
// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): state += golden gamma, output
// is a 64-bit mixing of the state.  Vector r's key is output r+1 of the
// generator seeded with `seed`; element i draws output i+1 of the generator
// seeded with the key.

__device__ __forceinline__ uint64_t sm64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
constexpr uint64_t SM64_GAMMA = 0x9E3779B97F4A7C15ull;

// perm (nullable): original index of each stored row, so a reordered matrix
// receives the same state as the original one, reordered
template <typename T>
__global__ __launch_bounds__(WG) void init_random_kernel(T *psi0, T *p, int64_t n, int B, uint64_t seed, int64_t r0,
                                                         const int32_t *perm)
{
    using E = Elem<T>;
    const int64_t total = n * B;
    const double amp = 1.0 / sqrt((double)n);
    const double two_pi = 6.283185307179586476925286766559;
    for (int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x; e < total; e += (int64_t)gridDim.x * WG) {
        const int64_t i = perm ? (int64_t)perm[e / B] : e / B;
        const int64_t r = r0 + e % B;
        const uint64_t key = sm64_mix(seed + (uint64_t)(r + 1) * SM64_GAMMA);
        const uint64_t bits = sm64_mix(key + (uint64_t)(i + 1) * SM64_GAMMA);
        const double u = (double)(bits >> 11) * 0x1.0p-53;
        double sn, cs;
        sincos(two_pi * u, &sn, &cs);
        const T v = E::from_d(d2{amp * cs, amp * sn});
        psi0[e] = v;
        p[e] = v;
    }
}


hipError_t launch_init_random(int dtype, void *psi0, void *p, int64_t n, int B, uint64_t seed, int64_t r0,
                              const int32_t *perm, hipStream_t st)
{
    const int g = elem_grid(n * B);
    if (dtype == TBPM_C128)
        hipLaunchKernelGGL(init_random_kernel<d2>, dim3(g), dim3(WG), 0, st, (d2 *)psi0, (d2 *)p, n, B, seed, r0,
                           perm);
    else
        hipLaunchKernelGGL(init_random_kernel<f2>, dim3(g), dim3(WG), 0, st, (f2 *)psi0, (f2 *)p, n, B, seed, r0,
                           perm);
    return hipGetLastError();
}

// vector b = e_{rows[b]} (stored row order); psi0 and p may be the same buffer
template <typename T>
__global__ __launch_bounds__(WG) void init_sites_kernel(T *psi0, T *p, int64_t n, int B, SiteRows rows)
{
    const int64_t total = n * B;
    for (int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x; e < total; e += (int64_t)gridDim.x * WG) {
        const int64_t i = e / B;
        const int b = (int)(e % B);
        T v{};
        if (i == rows.r[b])
            v.x = 1;
        psi0[e] = v;
        p[e] = v;
    }
}

hipError_t launch_init_sites(int dtype, void *psi0, void *p, int64_t n, int B, const SiteRows &rows, hipStream_t st)
{
    if (B < 1 || B > 64 || n <= 0)
        return hipErrorInvalidValue;
    const int g = elem_grid(n * B);
    if (dtype == TBPM_C128)
        hipLaunchKernelGGL(init_sites_kernel<d2>, dim3(g), dim3(WG), 0, st, (d2 *)psi0, (d2 *)p, n, B, rows);
    else
        hipLaunchKernelGGL(init_sites_kernel<f2>, dim3(g), dim3(WG), 0, st, (f2 *)psi0, (f2 *)p, n, B, rows);
    return hipGetLastError();
}

// src: complex128 [B][n] (vector-major, original order) -> psi0, p: [n][B] in
// storage precision and stored row order
template <typename T>
__global__ __launch_bounds__(WG) void pack_kernel(const d2 *src, T *psi0, T *p, int64_t n, int B, const int32_t *perm)
{
    using E = Elem<T>;
    const int64_t total = n * B;
    for (int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x; e < total; e += (int64_t)gridDim.x * WG) {
        const int64_t i = perm ? (int64_t)perm[e / B] : e / B;
        const int64_t b = e % B;
        const T v = E::from_d(src[b * n + i]);
        psi0[e] = v;
        p[e] = v;
    }
}

hipError_t launch_pack_states(int dtype, const double *src, void *psi0, void *p, int64_t n, int B, const int32_t *perm,
                              hipStream_t st)
{
    const int g = elem_grid(n * B);
    if (dtype == TBPM_C128)
        hipLaunchKernelGGL(pack_kernel<d2>, dim3(g), dim3(WG), 0, st, (const d2 *)src, (d2 *)psi0, (d2 *)p, n, B,
                           perm);
    else
        hipLaunchKernelGGL(pack_kernel<f2>, dim3(g), dim3(WG), 0, st, (const d2 *)src, (f2 *)psi0, (f2 *)p, n, B,
                           perm);
    return hipGetLastError();
}

// vector b of a [n][B] block -> complex128 [n] in original row order
template <typename T>
__global__ __launch_bounds__(WG) void unpack_kernel(const T *src, d2 *dst, int64_t n, int B, int b,
                                                    const int32_t *perm)
{
    using E = Elem<T>;
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG)
        dst[perm ? (int64_t)perm[i] : i] = E::to_d(src[i * B + b]);
}

hipError_t launch_unpack_state(int dtype, const void *src, double *dst, int64_t n, int B, int b, const int32_t *perm,
                               hipStream_t st)
{
    const int g = elem_grid(n);
    if (dtype == TBPM_C128)
        hipLaunchKernelGGL(unpack_kernel<d2>, dim3(g), dim3(WG), 0, st, (const d2 *)src, (d2 *)dst, n, B, b, perm);
    else
        hipLaunchKernelGGL(unpack_kernel<f2>, dim3(g), dim3(WG), 0, st, (const f2 *)src, (d2 *)dst, n, B, b, perm);
    return hipGetLastError();
}

// ---- correlation sums -------------------------------------------------------------------

// partials[blk][b] = (sum conj(psi0) v, sum |v|^2) over the rows of workgroup blk
template <typename T>
__global__ __launch_bounds__(WG) void dot_partials_kernel(const T *psi0, const T *v, int64_t n, int B,
                                                          double *partials)
{
    using E = Elem<T>;
    __shared__ double red[WG][3];
    for (int b = 0; b < B; ++b) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG) {
            const d2 p = E::to_d(psi0[i * B + b]);
            const d2 o = E::to_d(v[i * B + b]);
            s0 += p.x * o.x + p.y * o.y;
            s1 += p.x * o.y - p.y * o.x;
            s2 += o.x * o.x + o.y * o.y;
        }
        red[threadIdx.x][0] = s0;
        red[threadIdx.x][1] = s1;
        red[threadIdx.x][2] = s2;
        __syncthreads();
        for (int h = WG / 2; h > 0; h >>= 1) {
            if (threadIdx.x < h) {
                red[threadIdx.x][0] += red[threadIdx.x + h][0];
                red[threadIdx.x][1] += red[threadIdx.x + h][1];
                red[threadIdx.x][2] += red[threadIdx.x + h][2];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            double *p = partials + ((int64_t)blockIdx.x * B + b) * 4;
            p[0] = red[0][0];
            p[1] = red[0][1];
            p[2] = red[0][2];
            p[3] = 0.0;
        }
        __syncthreads();
    }
}

hipError_t launch_dot_partials(int dtype, const void *psi0, const void *v, int64_t n, int B, double *partials,
                               int grid, hipStream_t st)
{
    if (dtype == TBPM_C128)
        hipLaunchKernelGGL(dot_partials_kernel<d2>, dim3(grid), dim3(WG), 0, st, (const d2 *)psi0, (const d2 *)v,
                           n, B, partials);
    else
        hipLaunchKernelGGL(dot_partials_kernel<f2>, dim3(grid), dim3(WG), 0, st, (const f2 *)psi0, (const f2 *)v,
                           n, B, partials);
    return hipGetLastError();
}

// corr[b] = sum over blocks of partials[blk][b][0..1], norms[b] likewise from [2];
// one workgroup of RWG lanes: lane t sums vector b = t mod B over the blocks
// t / B, t / B + RWG / B, ... (neighbouring lanes read neighbouring vectors of
// one block, so the partials stream once), then a fixed tree over the lanes
// of each vector: the order does not depend on timing, so results reproduce
// exactly.
constexpr int RWG = 1024;
// tol > 0: flag[0] = 1 when some |norm - 1| exceeds tol (or is not a number)
__device__ __forceinline__ void check_norm(double nrm, double tol, int32_t *flag)
{
    if (flag && tol > 0.0 && !(fabs(nrm - 1.0) <= tol))
        flag[0] = 1;
}

// the reduction itself, for rows corr[2 b], norms[b] of block width B (a power
// of two dividing RWG)
__device__ __forceinline__ void reduce_rows(const double *partials, int nblocks, int B, double *corr, double *norms,
                                            double tol, int32_t *flag)
{
    __shared__ double red[RWG][3];
    const int G = RWG / B;
    const int b = threadIdx.x % B, g = threadIdx.x / B;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int k = g; k < nblocks; k += G) {
        const double *p = partials + ((int64_t)k * B + b) * 4;
        s0 += p[0];
        s1 += p[1];
        s2 += p[2];
    }
    red[threadIdx.x][0] = s0;
    red[threadIdx.x][1] = s1;
    red[threadIdx.x][2] = s2;
    __syncthreads();
    for (int h = G / 2; h > 0; h >>= 1) {
        if (g < h) {
            red[threadIdx.x][0] += red[threadIdx.x + h * B][0];
            red[threadIdx.x][1] += red[threadIdx.x + h * B][1];
            red[threadIdx.x][2] += red[threadIdx.x + h * B][2];
        }
        __syncthreads();
    }
    if (g == 0) {
        corr[2 * b] = red[b][0];
        corr[2 * b + 1] = red[b][1];
        norms[b] = red[b][2];
        check_norm(red[b][2], tol, flag);
    }
}

__global__ __launch_bounds__(RWG) void reduce_kernel(const double *partials, int nblocks, int B, double *corr,
                                                     double *norms, double tol, int32_t *flag)
{
    reduce_rows(partials, nblocks, B, corr, norms, tol, flag);
}

hipError_t launch_reduce(const double *partials, int nblocks, int B, double *corr, double *norms, hipStream_t st,
                         double tol, int32_t *flag)
{
    if (B < 1 || B > 64 || (B & (B - 1)) != 0)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(RWG), 0, st, partials, nblocks, B, corr, norms, tol, flag);
    return hipGetLastError();
}

// the same fixed-order reduction; the row k comes from a device counter that
// the last step advances, so a captured step replays unchanged
__global__ __launch_bounds__(RWG) void reduce_step_kernel(const double *partials, int nblocks, int B, double *corr,
                                                          double *norms, int32_t *kstep, double tol, int32_t *flag)
{
    const int64_t k = kstep[0];
    reduce_rows(partials, nblocks, B, corr + k * B * 2, norms + k * B, tol, flag);
    __syncthreads();                                // every lane has read kstep
    if (threadIdx.x == 0)
        kstep[0] = (int32_t)(k + 1);
}

__global__ void set_counter_kernel(int32_t *counter, int32_t value)
{
    if (threadIdx.x == 0)
        counter[0] = value;
}

hipError_t launch_reduce_step(const double *partials, int nblocks, int B, double *corr, double *norms, int32_t *kstep,
                              hipStream_t st, double tol, int32_t *flag)
{
    if (B < 1 || B > 64 || (B & (B - 1)) != 0)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(reduce_step_kernel, dim3(1), dim3(RWG), 0, st, partials, nblocks, B, corr, norms, kstep, tol,
                       flag);
    return hipGetLastError();
}

hipError_t launch_set_counter(int32_t *counter, int32_t value, hipStream_t st)
{
    hipLaunchKernelGGL(set_counter_kernel, dim3(1), dim3(64), 0, st, counter, value);
    return hipGetLastError();
}

// ---- Chebyshev moments -------------------------------------------------------------------
// One workgroup per (launch j, vector b): lanes sum a fixed strided subset of
// the per-block partials, then a fixed tree, as in reduce_kernel.
constexpr int MWG = 256;
__global__ __launch_bounds__(MWG) void moment_reduce_kernel(const double *partials, int nblocks, int B,
                                                            int64_t stride, int m0, double *raw, int kmax)
{
    __shared__ double red[MWG][3];
    const int j = blockIdx.x;
    const int b = blockIdx.y;
    const double *base = partials + (int64_t)j * stride;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int k = threadIdx.x; k < nblocks; k += MWG) {
        const double *p = base + ((int64_t)k * B + b) * 4;
        s0 += p[0];
        s1 += p[1];
        s2 += p[2];
    }
    red[threadIdx.x][0] = s0;
    red[threadIdx.x][1] = s1;
    red[threadIdx.x][2] = s2;
    __syncthreads();
    for (int h = MWG / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            red[threadIdx.x][0] += red[threadIdx.x + h][0];
            red[threadIdx.x][1] += red[threadIdx.x + h][1];
            red[threadIdx.x][2] += red[threadIdx.x + h][2];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double *r = raw + ((int64_t)b * kmax + m0 + j) * 4;
        r[0] = red[0][0];
        r[1] = red[0][1];
        r[2] = red[0][2];
        r[3] = 0.0;
    }
}

hipError_t launch_moment_reduce(const double *partials, int nblocks, int B, int64_t stride, int count, int m0,
                                double *raw, int kmax, hipStream_t st)
{
    if (count <= 0 || B <= 0 || nblocks <= 0 || m0 < 0 || m0 + count > kmax)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(moment_reduce_kernel, dim3(count, B), dim3(MWG), 0, st, partials, nblocks, B, stride, m0,
                       raw, kmax);
    return hipGetLastError();
}

// Doubling (T_m T_n = (T_{m+n} + T_{|m-n|}) / 2 applied to <psi0|T_m T_n|psi0>):
// mu_2m = 2 <p_m|p_m> - mu_0 and mu_2m+1 = 2 <p_m|p_m+1> - mu_1, p_m = T_m(H/rho) psi0.
__global__ __launch_bounds__(WG) void moment_finish_kernel(const double *raw, int kmax, int B, int num, d2 *mu)
{
    const int64_t total = (int64_t)B * num;
    for (int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x; e < total; e += (int64_t)gridDim.x * WG) {
        const int b = (int)(e / num);
        const int q = (int)(e % num);
        const double *r = raw + (int64_t)b * kmax * 4;
        const double *rm = r + (int64_t)(q / 2) * 4;
        d2 v;
        if (q % 2 == 0)
            v = d2{2.0 * rm[2] - r[2], 0.0};
        else
            v = d2{2.0 * rm[0] - r[0], 2.0 * rm[1] - r[1]};
        mu[e] = v;
    }
}

hipError_t launch_moment_finish(const double *raw, int kmax, int B, int num, double *mu, hipStream_t st)
{
    if (num <= 0 || B <= 0 || (num + 1) / 2 > kmax)
        return hipErrorInvalidValue;
    const int g = elem_grid((int64_t)B * num);
    hipLaunchKernelGGL(moment_finish_kernel, dim3(g), dim3(WG), 0, st, raw, kmax, B, num, (d2 *)mu);
    return hipGetLastError();
}

// ---- operators in CSR (current, density) -------------------------------------------------

template <typename RP>
__device__ __forceinline__ void row_range(const void *rp, int64_t i, int64_t &b, int64_t &e)
{
    const RP *r = static_cast<const RP *>(rp);
    b = r[i];
    e = r[i + 1];
}

template <typename T, typename RP>
__global__ __launch_bounds__(WG) void op_apply_kernel(const void *rp, const int32_t *col, const T *val, int64_t n,
                                                      const T *x, T *y)
{
    using E = Elem<T>;
    using A = typename E::acc;
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG) {
        int64_t b, e;
        row_range<RP>(rp, i, b, e);
        A acc{0, 0};
        for (int64_t j = b; j < e; ++j)
            cmac(acc, (A)val[j], (A)x[col[j]]);
        y[i] = E::from_d(E::acc_to_d(acc));
    }
}

template <typename T, typename RP>
__global__ __launch_bounds__(WG) void op_dot_kernel(const void *rp, const int32_t *col, const T *val, int64_t n,
                                                    const T *u, const T *v, double *partials)
{
    using E = Elem<T>;
    using A = typename E::acc;
    __shared__ double red[WG][2];
    double sre = 0.0, sim = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG) {
        int64_t b, e;
        row_range<RP>(rp, i, b, e);
        A acc{0, 0};
        for (int64_t j = b; j < e; ++j)
            cmac(acc, (A)val[j], (A)v[col[j]]);
        const d2 av = E::acc_to_d(acc);
        const d2 ui = E::to_d(u[i]);
        sre += ui.x * av.x + ui.y * av.y;
        sim += ui.x * av.y - ui.y * av.x;
    }
    red[threadIdx.x][0] = sre;
    red[threadIdx.x][1] = sim;
    __syncthreads();
    for (int h = WG / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            red[threadIdx.x][0] += red[threadIdx.x + h][0];
            red[threadIdx.x][1] += red[threadIdx.x + h][1];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double *p = partials + (int64_t)blockIdx.x * 4;
        p[0] = red[0][0];
        p[1] = red[0][1];
        p[2] = 0.0;
        p[3] = 0.0;
    }
}

int op_dot_grid(int64_t n)
{
    int64_t g = (n + WG - 1) / WG;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, 1024));
}

hipError_t launch_op_apply(int dtype, const void *rp, int rp64, const int32_t *col, const void *val, int64_t n,
                           const void *x, void *y, hipStream_t st)
{
    if (n <= 0)
        return hipErrorInvalidValue;
    const int g = elem_grid(n);
    if (dtype == TBPM_C128) {
        if (rp64)
            hipLaunchKernelGGL((op_apply_kernel<d2, int64_t>), dim3(g), dim3(WG), 0, st, rp, col, (const d2 *)val, n,
                               (const d2 *)x, (d2 *)y);
        else
            hipLaunchKernelGGL((op_apply_kernel<d2, int32_t>), dim3(g), dim3(WG), 0, st, rp, col, (const d2 *)val, n,
                               (const d2 *)x, (d2 *)y);
    } else {
        if (rp64)
            hipLaunchKernelGGL((op_apply_kernel<f2, int64_t>), dim3(g), dim3(WG), 0, st, rp, col, (const f2 *)val, n,
                               (const f2 *)x, (f2 *)y);
        else
            hipLaunchKernelGGL((op_apply_kernel<f2, int32_t>), dim3(g), dim3(WG), 0, st, rp, col, (const f2 *)val, n,
                               (const f2 *)x, (f2 *)y);
    }
    return hipGetLastError();
}

hipError_t launch_op_dot(int dtype, const void *rp, int rp64, const int32_t *col, const void *val, int64_t n,
                         const void *u, const void *v, double *partials, hipStream_t st)
{
    if (n <= 0)
        return hipErrorInvalidValue;
    const int g = op_dot_grid(n);
    if (dtype == TBPM_C128) {
        if (rp64)
            hipLaunchKernelGGL((op_dot_kernel<d2, int64_t>), dim3(g), dim3(WG), 0, st, rp, col, (const d2 *)val, n,
                               (const d2 *)u, (const d2 *)v, partials);
        else
            hipLaunchKernelGGL((op_dot_kernel<d2, int32_t>), dim3(g), dim3(WG), 0, st, rp, col, (const d2 *)val, n,
                               (const d2 *)u, (const d2 *)v, partials);
    } else {
        if (rp64)
            hipLaunchKernelGGL((op_dot_kernel<f2, int64_t>), dim3(g), dim3(WG), 0, st, rp, col, (const f2 *)val, n,
                               (const f2 *)u, (const f2 *)v, partials);
        else
            hipLaunchKernelGGL((op_dot_kernel<f2, int32_t>), dim3(g), dim3(WG), 0, st, rp, col, (const f2 *)val, n,
                               (const f2 *)u, (const f2 *)v, partials);
    }
    return hipGetLastError();
}

// ---- quasi-eigenstates ------------------------------------------------------------------
// qe_j += f_j psi for a group of energies (f_j = w_k exp(i E_j t_k)); psi is
// read once per group, each qe_j read and written once (FP64 accumulators).
template <typename T>
__global__ __launch_bounds__(WG) void qe_accumulate_kernel(const T *psi, int64_t n, d2 *qe, int count, QeFactors f)
{
    using E = Elem<T>;
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG) {
        const d2 v = E::to_d(psi[i]);
        for (int j = 0; j < count; ++j) {
            d2 *q = qe + (int64_t)j * n + i;
            *q = *q + cmul(d2{f.re[j], f.im[j]}, v);
        }
    }
}

hipError_t launch_qe_accumulate(int dtype, const void *psi, int64_t n, double *qe, int count, const QeFactors &f,
                                hipStream_t st)
{
    if (count < 1 || count > QE_MAX || n <= 0)
        return hipErrorInvalidValue;
    const int g = elem_grid(n);
    if (dtype == TBPM_C128)
        hipLaunchKernelGGL(qe_accumulate_kernel<d2>, dim3(g), dim3(WG), 0, st, (const d2 *)psi, n, (d2 *)qe, count,
                           f);
    else
        hipLaunchKernelGGL(qe_accumulate_kernel<f2>, dim3(g), dim3(WG), 0, st, (const f2 *)psi, n, (d2 *)qe, count,
                           f);
    return hipGetLastError();
}

// site_corr[s * stride + k] += sum_b conj(psi0[i_s, b]) v[i_s, b]   (b in order)
template <typename T>
__global__ __launch_bounds__(WG) void ldos_gather_kernel(const T *psi0, const T *v, int64_t n, int B,
                                                         const int64_t *sites, int nsites, d2 *site_corr,
                                                         int stride, int k)
{
    using E = Elem<T>;
    const int s = blockIdx.x * WG + threadIdx.x;
    if (s >= nsites)
        return;
    const int64_t i = sites[s];
    if (i < 0 || i >= n)
        return;
    d2 acc{0.0, 0.0};
    for (int b = 0; b < B; ++b) {
        const d2 p = E::to_d(psi0[i * B + b]);
        const d2 o = E::to_d(v[i * B + b]);
        acc += d2{p.x * o.x + p.y * o.y, p.x * o.y - p.y * o.x};
    }
    site_corr[(int64_t)s * stride + k] += acc;
}

hipError_t launch_ldos_gather(int dtype, const void *psi0, const void *v, int64_t n, int B, const int64_t *sites,
                              int nsites, double *site_corr, int stride, int k, hipStream_t st)
{
    const int g = (nsites + WG - 1) / WG;
    if (g == 0)
        return hipSuccess;
    if (dtype == TBPM_C128)
        hipLaunchKernelGGL(ldos_gather_kernel<d2>, dim3(g), dim3(WG), 0, st, (const d2 *)psi0, (const d2 *)v, n, B,
                           sites, nsites, (d2 *)site_corr, stride, k);
    else
        hipLaunchKernelGGL(ldos_gather_kernel<f2>, dim3(g), dim3(WG), 0, st, (const f2 *)psi0, (const f2 *)v, n, B,
                           sites, nsites, (d2 *)site_corr, stride, k);
    return hipGetLastError();
}

// ---- Hamiltonian analysis and conversion ----------------------------------------------------
// res[0]: error flags (1 row_ptr, 2 column range, 4 column order, 8 not Hermitian)
// res[1]: longest row;  res[2]: bits of the Gershgorin bound max_i sum_j |H_ij|;
// res[3]: bits of max |H_ij|.  Non-negative doubles order like their bit patterns.

__global__ __launch_bounds__(WG) void csr_check_kernel(const int64_t *rp, const int32_t *col, const d2 *val,
                                                       int64_t n, int64_t nnz, unsigned long long *res)
{
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG) {
        const int64_t beg = rp[i], end = rp[i + 1];
        unsigned long long flags = 0;
        if (beg < 0 || end < beg || end > nnz || (i == 0 && beg != 0) || (i == n - 1 && end != nnz))
            flags |= 1;
        double rs = 0.0, mx = 0.0;
        if (!(flags & 1)) {
            int32_t prev = -1;
            for (int64_t j = beg; j < end; ++j) {
                const int32_t c = col[j];
                if (c < 0 || (int64_t)c >= n)
                    flags |= 2;
                if (c <= prev)
                    flags |= 4;
                prev = c;
                const d2 v = val[j];
                const double av = sqrt(v.x * v.x + v.y * v.y);
                rs += av;
                mx = av > mx ? av : mx;
            }
        }
        if (flags)
            atomicOr(&res[0], flags);
        atomicMax(&res[1], (unsigned long long)(end - beg > 0 ? end - beg : 0));
        atomicMax(&res[2], (unsigned long long)__double_as_longlong(rs));
        atomicMax(&res[3], (unsigned long long)__double_as_longlong(mx));
    }
}

hipError_t launch_csr_check(const int64_t *rp, const int32_t *col, const double *val, int64_t n, int64_t nnz,
                            unsigned long long *res, hipStream_t st)
{
    hipLaunchKernelGGL(csr_check_kernel, dim3(elem_grid(n)), dim3(WG), 0, st, rp, col, (const d2 *)val, n, nnz, res);
    return hipGetLastError();
}

// For every stored H_ij: find H_ji by binary search in row j (columns sorted)
// and flag |H_ij - conj(H_ji)| > tol.  Run only on a CSR that passed the check.
__global__ __launch_bounds__(WG) void hermitian_kernel(const int64_t *rp, const int32_t *col, const d2 *val,
                                                       int64_t n, double tol, unsigned long long *res)
{
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG) {
        bool bad = false;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int64_t j = col[k];
            int64_t lo = rp[j], hi = rp[j + 1];
            d2 hji{0.0, 0.0};
            while (lo < hi) {
                const int64_t mid = (lo + hi) / 2;
                const int32_t c = col[mid];
                if (c == i) {
                    hji = val[mid];
                    break;
                }
                if (c < i)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            const d2 hij = val[k];
            const double dr = hij.x - hji.x, di = hij.y + hji.y;
            if (sqrt(dr * dr + di * di) > tol)
                bad = true;
        }
        if (bad)
            atomicOr(&res[0], 8ull);
    }
}

hipError_t launch_hermitian_check(const int64_t *rp, const int32_t *col, const double *val, int64_t n, double tol,
                                  unsigned long long *res, hipStream_t st)
{
    hipLaunchKernelGGL(hermitian_kernel, dim3(elem_grid(n)), dim3(WG), 0, st, rp, col, (const d2 *)val, n, tol, res);
    return hipGetLastError();
}

template <typename T, typename RP>
__global__ __launch_bounds__(WG) void to_csr_kernel(const int64_t *rp, const int32_t *col, const d2 *val, int64_t n,
                                                    int64_t nnz, RP *rp_out, int32_t *col_out, T *val_out)
{
    using E = Elem<T>;
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i <= n; i += (int64_t)gridDim.x * WG)
        rp_out[i] = (RP)rp[i];
    for (int64_t j = (int64_t)blockIdx.x * WG + threadIdx.x; j < nnz; j += (int64_t)gridDim.x * WG) {
        col_out[j] = col[j];
        val_out[j] = E::from_d(val[j]);
    }
}

hipError_t launch_to_csr(int dtype, const int64_t *rp, const int32_t *col, const double *val, int64_t n, int64_t nnz,
                         void *rp_out, int rp64, int32_t *col_out, void *val_out, hipStream_t st)
{
    const int g = elem_grid(nnz > n ? nnz : n + 1);
    const d2 *v = (const d2 *)val;
    if (dtype == TBPM_C128) {
        if (rp64)
            hipLaunchKernelGGL((to_csr_kernel<d2, int64_t>), dim3(g), dim3(WG), 0, st, rp, col, v, n, nnz,
                               (int64_t *)rp_out, col_out, (d2 *)val_out);
        else
            hipLaunchKernelGGL((to_csr_kernel<d2, int32_t>), dim3(g), dim3(WG), 0, st, rp, col, v, n, nnz,
                               (int32_t *)rp_out, col_out, (d2 *)val_out);
    } else {
        if (rp64)
            hipLaunchKernelGGL((to_csr_kernel<f2, int64_t>), dim3(g), dim3(WG), 0, st, rp, col, v, n, nnz,
                               (int64_t *)rp_out, col_out, (f2 *)val_out);
        else
            hipLaunchKernelGGL((to_csr_kernel<f2, int32_t>), dim3(g), dim3(WG), 0, st, rp, col, v, n, nnz,
                               (int32_t *)rp_out, col_out, (f2 *)val_out);
    }
    return hipGetLastError();
}

// ELL slot s of row i at s*ld + i; rows shorter than w padded with (column i, 0)
template <typename T>
__global__ __launch_bounds__(WG) void to_ell_kernel(const int64_t *rp, const int32_t *col, const d2 *val, int64_t n,
                                                    int32_t w, int64_t ld, int32_t *col_out, T *val_out)
{
    using E = Elem<T>;
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < ld; i += (int64_t)gridDim.x * WG) {
        int64_t beg = 0, len = 0;
        if (i < n) {
            beg = rp[i];
            len = rp[i + 1] - beg;
        }
        const int32_t self = (int32_t)(i < n ? i : 0);
        for (int s = 0; s < w; ++s) {
            const int64_t o = (int64_t)s * ld + i;
            if (s < len) {
                col_out[o] = col[beg + s];
                val_out[o] = E::from_d(val[beg + s]);
            } else {
                col_out[o] = self;
                val_out[o] = E::from_d(d2{0.0, 0.0});
            }
        }
    }
}

hipError_t launch_to_ell(int dtype, const int64_t *rp, const int32_t *col, const double *val, int64_t n, int32_t w,
                         int64_t ld, int32_t *col_out, void *val_out, hipStream_t st)
{
    const int g = elem_grid(ld);
    if (dtype == TBPM_C128)
        hipLaunchKernelGGL(to_ell_kernel<d2>, dim3(g), dim3(WG), 0, st, rp, col, (const d2 *)val, n, w, ld, col_out,
                           (d2 *)val_out);
    else
        hipLaunchKernelGGL(to_ell_kernel<f2>, dim3(g), dim3(WG), 0, st, rp, col, (const d2 *)val, n, w, ld, col_out,
                           (f2 *)val_out);
    return hipGetLastError();
}

// copy of the ELL rows listed in halo_rows (slot-major, stride ldh)
template <typename T>
__global__ __launch_bounds__(WG) void halo_ell_kernel(const int32_t *col, const T *val, int64_t ld, int32_t w,
                                                      const int32_t *halo_rows, int64_t nhalo, int64_t ldh,
                                                      int32_t *hcol, T *hval)
{
    for (int64_t g = (int64_t)blockIdx.x * WG + threadIdx.x; g < nhalo; g += (int64_t)gridDim.x * WG) {
        const int64_t r = halo_rows[g];
        for (int s = 0; s < w; ++s) {
            hcol[(int64_t)s * ldh + g] = col[(int64_t)s * ld + r];
            hval[(int64_t)s * ldh + g] = val[(int64_t)s * ld + r];
        }
    }
}

hipError_t launch_halo_ell(int dtype, const int32_t *col, const void *val, int64_t ld, int32_t w,
                           const int32_t *halo_rows, int64_t nhalo, int64_t ldh, int32_t *hcol, void *hval,
                           hipStream_t st)
{
    if (nhalo == 0)
        return hipSuccess;
    const int g = elem_grid(nhalo);
    if (dtype == TBPM_C128)
        hipLaunchKernelGGL(halo_ell_kernel<d2>, dim3(g), dim3(WG), 0, st, col, (const d2 *)val, ld, w, halo_rows,
                           nhalo, ldh, hcol, (d2 *)hval);
    else
        hipLaunchKernelGGL(halo_ell_kernel<f2>, dim3(g), dim3(WG), 0, st, col, (const f2 *)val, ld, w, halo_rows,
                           nhalo, ldh, hcol, (f2 *)hval);
    return hipGetLastError();
}

// One-byte value indices of a stored ELL (see ValueTable): word q of row i
// (vidx[q * ld + i]) holds the indices of slots 4q .. 4q + 3 in its bytes,
// low byte first.  +0 (padding) is index 0; with `diag` (1, or 2 for real
// parts only), a nonzero entry in the row's own column is index 255 and its
// value goes to vdiag[i] (0 for rows without one); any other value is found
// by binary search in the sorted keys (two words a value).  A value not in
// the table sets *bad.
__device__ __forceinline__ void key_of(d2 v, uint64_t &re, uint64_t &im)
{
    re = (uint64_t)__double_as_longlong(v.x);
    im = (uint64_t)__double_as_longlong(v.y);
}
__device__ __forceinline__ void key_of(f2 v, uint64_t &re, uint64_t &im)
{
    re = (uint32_t)__float_as_uint(v.x);
    im = (uint32_t)__float_as_uint(v.y);
}

template <typename T>
__global__ __launch_bounds__(WG) void value_index_kernel(const int32_t *col, const T *val, int64_t n, int32_t w,
                                                         int64_t ld, const uint64_t *keys, int32_t nkeys,
                                                         int32_t diag, uint32_t *vidx, T *vdiag, int32_t *bad)
{
    using Re = decltype(T{}.x);
    Re *vre = reinterpret_cast<Re *>(vdiag);       // diag == 2: real parts only
    const int nw = (w + 3) / 4;
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG) {
        if (diag == 1)
            vdiag[i] = T{};
        else if (diag == 2)
            vre[i] = Re(0);
        for (int q = 0; q < nw; ++q) {
            uint32_t word = 0;
            for (int b = 0; b < 4 && 4 * q + b < w; ++b) {
                const int64_t at = (int64_t)(4 * q + b) * ld + i;
                const T v = val[at];
                uint64_t re, im;
                key_of(v, re, im);
                uint32_t idx = 0;
                if (re == 0 && im == 0) {
                    idx = 0;
                } else if (diag && col[at] == i) {
                    idx = 255;
                    if (diag == 1)
                        vdiag[i] = v;
                    else
                        vre[i] = v.x;
                } else {
                    int lo = 0, hi = nkeys - 1;        // first key >= (re, im)
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        const uint64_t kr = keys[2 * mid], ki = keys[2 * mid + 1];
                        if (kr < re || (kr == re && ki < im))
                            lo = mid + 1;
                        else
                            hi = mid;
                    }
                    if (keys[2 * lo] == re && keys[2 * lo + 1] == im)
                        idx = (uint32_t)lo;
                    else
                        *bad = 1;
                }
                word |= idx << (8 * b);
            }
            vidx[(int64_t)q * ld + i] = word;
        }
    }
}

hipError_t launch_value_index(int dtype, const int32_t *col, const void *val, int64_t n, int32_t w, int64_t ld,
                              const uint64_t *keys, int32_t nkeys, int32_t diag, uint32_t *vidx, void *vdiag,
                              int32_t *bad, hipStream_t st)
{
    if (n <= 0 || w <= 0 || nkeys <= 0 || nkeys > 255)
        return hipErrorInvalidValue;
    const int g = elem_grid(n);
    if (dtype == TBPM_C128)
        hipLaunchKernelGGL(value_index_kernel<d2>, dim3(g), dim3(WG), 0, st, col, (const d2 *)val, n, w, ld, keys,
                           nkeys, diag, vidx, (d2 *)vdiag, bad);
    else
        hipLaunchKernelGGL(value_index_kernel<f2>, dim3(g), dim3(WG), 0, st, col, (const f2 *)val, n, w, ld, keys,
                           nkeys, diag, vidx, (f2 *)vdiag, bad);
    return hipGetLastError();
}

// The value-index words of every patch's halo rows, contiguous in halo order
// (like halo_ell_kernel's copy of their columns and values).
__global__ __launch_bounds__(WG) void halo_vidx_kernel(const uint32_t *vidx, int64_t ld, int32_t nw,
                                                       const int32_t *halo_rows, int64_t nhalo, int64_t ldh,
                                                       uint32_t *hvidx)
{
    for (int64_t g = (int64_t)blockIdx.x * WG + threadIdx.x; g < nhalo; g += (int64_t)gridDim.x * WG) {
        const int64_t r = halo_rows[g];
        for (int q = 0; q < nw; ++q)
            hvidx[(int64_t)q * ldh + g] = vidx[(int64_t)q * ld + r];
    }
}

hipError_t launch_halo_vidx(const uint32_t *vidx, int64_t ld, int32_t nw, const int32_t *halo_rows, int64_t nhalo,
                            int64_t ldh, uint32_t *hvidx, hipStream_t st)
{
    if (nhalo == 0)
        return hipSuccess;
    hipLaunchKernelGGL(halo_vidx_kernel, dim3(elem_grid(nhalo)), dim3(WG), 0, st, vidx, ld, nw, halo_rows, nhalo,
                       ldh, hvidx);
    return hipGetLastError();
}

// Patch-local column indices of the patch-reordered ELL: for stored row i of
// patch q (rows patch_ptr[q] .. patch_ptr[q+1]-1, halo list halo_rows[halo_ptr[q]
// .. halo_ptr[q+1]-1], ascending), slot s holds col - patch_ptr[q] when the
// column is in the patch, else cnt + (its position in the halo list); the
// 16-bit indices of slots 4k .. 4k + 3 share one 64-bit word, lcol[k * ld + i]
// (bits 16 (s mod 4) up; slots past w hold 0), so a row's indices take one
// load per four slots.  A column found in neither (impossible for a plan built
// from this matrix) sets *bad and stores the row's own index.
__global__ __launch_bounds__(WG) void local_cols_kernel(const int32_t *col, int64_t ld, int32_t w, int64_t n,
                                                        const int32_t *patch_ptr, int64_t npatch,
                                                        const int32_t *halo_ptr, const int32_t *halo_rows,
                                                        uint64_t *lcol, int32_t *bad)
{
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG) {
        int64_t lo = 0, hi = npatch - 1;               // last q with patch_ptr[q] <= i
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (patch_ptr[mid] <= i)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int64_t base = patch_ptr[lo];
        const int cnt = patch_ptr[lo + 1] - (int)base;
        const int hb = halo_ptr[lo];
        const int hc = halo_ptr[lo + 1] - hb;
        uint64_t word = 0;
        for (int s = 0; s < w; ++s) {
            const int32_t c = col[(int64_t)s * ld + i];
            int l = (int)(c - base);
            if ((unsigned)l >= (unsigned)cnt) {
                int a = 0, b = hc;                      // first halo entry >= c
                while (a < b) {
                    const int mid = (a + b) >> 1;
                    if (halo_rows[hb + mid] < c)
                        a = mid + 1;
                    else
                        b = mid;
                }
                if (a < hc && halo_rows[hb + a] == c) {
                    l = cnt + a;
                } else {
                    l = (int)(i - base);
                    atomicOr(bad, 1);
                }
            }
            word |= (uint64_t)(uint16_t)l << (16 * (s % 4));
            if (s % 4 == 3 || s == w - 1) {
                lcol[(int64_t)(s / 4) * ld + i] = word;
                word = 0;
            }
        }
    }
}

hipError_t launch_local_cols(const int32_t *col, int64_t ld, int32_t w, int64_t n, const int32_t *patch_ptr,
                             int64_t npatch, const int32_t *halo_ptr, const int32_t *halo_rows, uint64_t *lcol,
                             int32_t *bad, hipStream_t st)
{
    if (n <= 0 || npatch <= 0)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(local_cols_kernel, dim3(elem_grid(n)), dim3(WG), 0, st, col, ld, w, n, patch_ptr, npatch,
                       halo_ptr, halo_rows, lcol, bad);
    return hipGetLastError();
}

// ELL of H' = P H P^T: stored row i is original row old_of_new[i], its
// columns renumbered with new_of_old; padding as in to_ell_kernel
template <typename T>
__global__ __launch_bounds__(WG) void to_ell_perm_kernel(const int64_t *rp, const int32_t *col, const d2 *val,
                                                         int64_t n, int32_t w, int64_t ld, const int32_t *old_of_new,
                                                         const int32_t *new_of_old, int32_t *col_out, T *val_out)
{
    using E = Elem<T>;
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < ld; i += (int64_t)gridDim.x * WG) {
        int64_t beg = 0, len = 0;
        if (i < n) {
            const int64_t o = old_of_new[i];
            beg = rp[o];
            len = rp[o + 1] - beg;
        }
        const int32_t self = (int32_t)(i < n ? i : 0);
        for (int s = 0; s < w; ++s) {
            const int64_t o = (int64_t)s * ld + i;
            if (s < len) {
                col_out[o] = new_of_old[col[beg + s]];
                val_out[o] = E::from_d(val[beg + s]);
            } else {
                col_out[o] = self;
                val_out[o] = E::from_d(d2{0.0, 0.0});
            }
        }
    }
}

hipError_t launch_to_ell_perm(int dtype, const int64_t *rp, const int32_t *col, const double *val, int64_t n,
                              int32_t w, int64_t ld, const int32_t *old_of_new, const int32_t *new_of_old,
                              int32_t *col_out, void *val_out, hipStream_t st)
{
    const int g = elem_grid(ld);
    if (dtype == TBPM_C128)
        hipLaunchKernelGGL(to_ell_perm_kernel<d2>, dim3(g), dim3(WG), 0, st, rp, col, (const d2 *)val, n, w, ld,
                           old_of_new, new_of_old, col_out, (d2 *)val_out);
    else
        hipLaunchKernelGGL(to_ell_perm_kernel<f2>, dim3(g), dim3(WG), 0, st, rp, col, (const d2 *)val, n, w, ld,
                           old_of_new, new_of_old, col_out, (f2 *)val_out);
    return hipGetLastError();
}

}  // namespace tbpm
