// HIP kernels of the TBPM propagation path for gfx950 (CDNA4, wave64).
//
// The hot kernel is one Chebyshev term (TBPLaS 2.0, "Migration to C++"): the
// sparse product with H fused with the three-term recurrence y <- 2(H/rho)x - y
// and the coefficient accumulation out <- out + c_m y.  The work is bound by
// HBM bandwidth (about 0.3 flop per byte), so the kernels use no matrix cores:
// they stream H once per term with non-temporal loads, gather x through L2,
// and touch each vector element once.
//
// Layouts
//   vectors: blocks of B complex vectors, element (row i, vector b) at i*B + b,
//            so the B values a row needs are contiguous;
//   CSR:     row pointer int32 (int64 when nnz >= 2^31), int32 columns;
//   ELL:     slot-major [w][ld]: slot s of row i at s*ld + i, padding slots
//            hold column i and value 0.
// Work split
//   a workgroup of 256 lanes owns tiles of 256/lr rows; lr lanes share a row
//   (B == 1: the row's entries are strided over the lr lanes and summed with
//   wave shuffles; B > 1: lr == B and each lane owns one vector of the row).
//   Tiles are dealt out so that each XCD (workgroup id mod 8) walks a
//   contiguous slab of rows: neighbouring rows share their gathered x entries
//   in that XCD's L2.
// Precision
//   double2 storage: FP64 throughout.  float2 storage: products and row sums
//   in FP32, the update (scale, recurrence, coefficient) in FP64 registers,
//   one rounding to FP32 on store, correlation sums in FP64.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "tbpm_internal.h"

namespace tbpm {

typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int WG = 256;      // lanes per workgroup
constexpr int NXCD = 8;      // XCDs per MI355X

// ---- element types -------------------------------------------------------------

template <typename T> struct Elem;
template <> struct Elem<d2> {
    using acc = d2;
    __device__ static d2 to_d(d2 v) { return v; }
    __device__ static d2 from_d(d2 v) { return v; }
    __device__ static d2 acc_to_d(d2 v) { return v; }
};
template <> struct Elem<f2> {
    using acc = f2;
    __device__ static d2 to_d(f2 v) { return d2{(double)v.x, (double)v.y}; }
    __device__ static f2 from_d(d2 v) { return f2{(float)v.x, (float)v.y}; }
    __device__ static d2 acc_to_d(f2 v) { return d2{(double)v.x, (double)v.y}; }
};

template <typename A>
__device__ __forceinline__ void cmac(A &acc, A a, A b)
{
    acc.x += a.x * b.x - a.y * b.y;
    acc.y += a.x * b.y + a.y * b.x;
}

__device__ __forceinline__ d2 cmul(d2 a, d2 b)
{
    return d2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

template <typename T>
__device__ __forceinline__ T ld_stream(const T *p)
{
    return __builtin_nontemporal_load(p);
}

// Tiles of XCD (blockIdx % 8) form one contiguous slab; block j of that XCD
// takes tiles lo + j, lo + j + nbx, ...
struct TileWalk {
    int64_t t, end, stride;
};
__device__ __forceinline__ TileWalk tile_walk(int64_t ntiles)
{
    const int64_t xcd = blockIdx.x % NXCD;
    const int64_t j = blockIdx.x / NXCD;
    const int64_t nbx = gridDim.x / NXCD;
    const int64_t lo = ntiles * xcd / NXCD;
    const int64_t hi = ntiles * (xcd + 1) / NXCD;
    return TileWalk{lo + j, hi, nbx};
}

// ---- the Chebyshev term kernel ---------------------------------------------------
//
// W > 0: ELL with a compile-time width, so every load of the row (its W column
// indices and values, and the vector operands of the update) is issued before
// the first dependent gather of x.  W == 0: runtime width (ELL) or CSR.
// Rows past n in the last tile load row n-1 (in bounds) and store nothing.

template <typename T>
__device__ __forceinline__ void st_stream(T v, T *p)
{
    __builtin_nontemporal_store(v, p);
}

template <typename T, int FMT, int B, int LR, int KIND, int W>
__global__ __launch_bounds__(WG) void term_kernel(TermArgs a)
{
    using E = Elem<T>;
    using A = typename E::acc;
    constexpr int ROWS = WG / LR;
    const int lr = threadIdx.x % LR;
    const int rloc = threadIdx.x / LR;
    const int64_t n = a.n;
    const int64_t ntiles = (n + ROWS - 1) / ROWS;
    const T *__restrict__ x = static_cast<const T *>(a.x);
    T *__restrict__ y = static_cast<T *>(a.y);
    T *__restrict__ out = static_cast<T *>(a.out);
    const T *__restrict__ val = static_cast<const T *>(a.val);
    const T *__restrict__ psi0 = static_cast<const T *>(a.psi0);
    const int32_t *__restrict__ col = a.col;
    const d2 ca = d2{a.ca_re, a.ca_im};
    const d2 cb = d2{a.cb_re, a.cb_im};
    const bool owner = (B > 1) || (lr == 0);

    double dre = 0.0, dim = 0.0, nrm = 0.0;

    TileWalk tw = tile_walk(ntiles);
    for (int64_t tile = tw.t; tile < tw.end; tile += tw.stride) {
        const int64_t row = tile * ROWS + rloc;
        const bool live = row < n;
        const int64_t rr = live ? row : n - 1;              // in-bounds row for loads
        const int64_t e = rr * B + (B > 1 ? lr : 0);

        // operands of the update, independent of the sparse product
        T xo{}, yo{}, oo{}, po{};
        if (owner) {
            if constexpr (KIND == K_FIRST || KIND == K_MOM0) {
                xo = x[e];
            } else if constexpr (KIND == K_MOM) {
                xo = x[e];
                yo = ld_stream(y + e);
            } else {
                yo = ld_stream(y + e);
                oo = ld_stream(out + e);
                if constexpr (KIND == K_LAST)
                    po = ld_stream(psi0 + e);
            }
        }

        A acc{0, 0};
        if constexpr (FMT == F_ELL && W > 0) {
            int32_t c[W];
            T v[W];
#pragma unroll
            for (int s = 0; s < W; ++s) {
                const int64_t idx = (int64_t)s * a.ld + rr;
                c[s] = ld_stream(col + idx);
                v[s] = ld_stream(val + idx);
            }
            T xv[W];
#pragma unroll
            for (int s = 0; s < W; ++s)
                xv[s] = x[(int64_t)c[s] * B + lr];
#pragma unroll
            for (int s = 0; s < W; ++s)
                cmac(acc, (A)v[s], (A)xv[s]);
        } else if constexpr (FMT == F_ELL) {
#pragma unroll 4
            for (int s = 0; s < a.w; ++s) {
                const int64_t idx = (int64_t)s * a.ld + rr;
                const int32_t c = ld_stream(col + idx);
                const T v = ld_stream(val + idx);
                cmac(acc, (A)v, (A)x[(int64_t)c * B + lr]);
            }
        } else {
            int64_t beg, end;
            if (a.rp64) {
                const int64_t *rp = static_cast<const int64_t *>(a.rp);
                beg = rp[rr];
                end = rp[rr + 1];
            } else {
                const int32_t *rp = static_cast<const int32_t *>(a.rp);
                beg = rp[rr];
                end = rp[rr + 1];
            }
            if constexpr (B == 1) {
                for (int64_t j = beg + lr; j < end; j += LR) {
                    const int32_t c = ld_stream(col + j);
                    const T v = ld_stream(val + j);
                    cmac(acc, (A)v, (A)x[c]);
                }
            } else {
                for (int64_t j = beg; j < end; ++j) {
                    const int32_t c = ld_stream(col + j);
                    const T v = ld_stream(val + j);
                    cmac(acc, (A)v, (A)x[(int64_t)c * B + lr]);
                }
            }
        }
        if constexpr (B == 1 && LR > 1) {
#pragma unroll
            for (int off = LR / 2; off > 0; off >>= 1) {
                acc.x += __shfl_xor(acc.x, off, LR);
                acc.y += __shfl_xor(acc.y, off, LR);
            }
        }
        if (live && owner) {
            const d2 s = E::acc_to_d(acc) * a.scale;
            if constexpr (KIND == K_MOM0 || KIND == K_MOM) {
                const T ys = E::from_d(KIND == K_MOM0 ? s : s - E::to_d(yo));
                st_stream(ys, y + e);
                const d2 xd = E::to_d(xo), yd = E::to_d(ys);
                dre += xd.x * yd.x + xd.y * yd.y;
                dim += xd.x * yd.y - xd.y * yd.x;
                nrm += xd.x * xd.x + xd.y * xd.y;
            } else if constexpr (KIND == K_FIRST) {
                st_stream(E::from_d(s), y + e);
                st_stream(E::from_d(cmul(ca, E::to_d(xo)) + cmul(cb, s)), out + e);
            } else {
                const d2 yn = s - E::to_d(yo);
                st_stream(E::from_d(yn), y + e);
                const T os = E::from_d(E::to_d(oo) + cmul(ca, yn));
                st_stream(os, out + e);
                if constexpr (KIND == K_LAST) {
                    const d2 p = E::to_d(po);
                    const d2 o = E::to_d(os);
                    dre += p.x * o.x + p.y * o.y;
                    dim += p.x * o.y - p.y * o.x;
                    nrm += o.x * o.x + o.y * o.y;
                }
            }
        }
    }

    if constexpr (KIND == K_LAST || KIND == K_MOM0 || KIND == K_MOM) {
        // lanes with equal (lane mod B) hold the same vector: fold them
        constexpr int STOP = (B > 1) ? B : 1;
#pragma unroll
        for (int off = 32; off >= STOP; off >>= 1) {
            dre += __shfl_xor(dre, off, 64);
            dim += __shfl_xor(dim, off, 64);
            nrm += __shfl_xor(nrm, off, 64);
        }
        __shared__ double red[WG / 64][B][3];
        const int lane = threadIdx.x % 64;
        const int wave = threadIdx.x / 64;
        if (lane < B) {
            red[wave][lane][0] = dre;
            red[wave][lane][1] = dim;
            red[wave][lane][2] = nrm;
        }
        __syncthreads();
        if (threadIdx.x < B) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
            for (int w = 0; w < WG / 64; ++w) {
                s0 += red[w][threadIdx.x][0];
                s1 += red[w][threadIdx.x][1];
                s2 += red[w][threadIdx.x][2];
            }
            double *p = a.partials + ((int64_t)blockIdx.x * B + threadIdx.x) * 4;
            p[0] = s0;
            p[1] = s1;
            p[2] = s2;
            p[3] = 0.0;
        }
    }
}

int rows_per_tile(const KernelShape &s) { return WG / s.lr; }

// Workgroups: one per tile up to 16 per CU (a few tiles each beyond that),
// rounded to a multiple of the 8 XCDs.
int term_grid(int64_t n, const KernelShape &s, int num_cu)
{
    const int64_t rows = WG / s.lr;
    const int64_t ntiles = (n + rows - 1) / rows;
    int64_t g = (ntiles + NXCD - 1) / NXCD * NXCD;
    const int64_t cap = (int64_t)num_cu * 16;
    if (g > cap)
        g = cap;
    if (g < NXCD)
        g = NXCD;
    return (int)g;
}

template <typename T, int FMT, int B, int LR, int W>
static hipError_t launch_kind(int kind, const TermArgs &a, int grid, hipStream_t st)
{
    switch (kind) {
    case K_FIRST:
        hipLaunchKernelGGL((term_kernel<T, FMT, B, LR, K_FIRST, W>), dim3(grid), dim3(WG), 0, st, a);
        break;
    case K_MID:
        hipLaunchKernelGGL((term_kernel<T, FMT, B, LR, K_MID, W>), dim3(grid), dim3(WG), 0, st, a);
        break;
    case K_MOM0:
        hipLaunchKernelGGL((term_kernel<T, FMT, B, LR, K_MOM0, W>), dim3(grid), dim3(WG), 0, st, a);
        break;
    case K_MOM:
        hipLaunchKernelGGL((term_kernel<T, FMT, B, LR, K_MOM, W>), dim3(grid), dim3(WG), 0, st, a);
        break;
    default:
        hipLaunchKernelGGL((term_kernel<T, FMT, B, LR, K_LAST, W>), dim3(grid), dim3(WG), 0, st, a);
        break;
    }
    return hipGetLastError();
}

// ELL: compile-time widths for the lattices' common row lengths
template <typename T, int B>
static hipError_t launch_ell(int kind, const TermArgs &a, int grid, hipStream_t st)
{
    switch (a.w) {
    case 3: return launch_kind<T, F_ELL, B, (B > 1 ? B : 1), 3>(kind, a, grid, st);
    case 4: return launch_kind<T, F_ELL, B, (B > 1 ? B : 1), 4>(kind, a, grid, st);
    case 5: return launch_kind<T, F_ELL, B, (B > 1 ? B : 1), 5>(kind, a, grid, st);
    case 8: return launch_kind<T, F_ELL, B, (B > 1 ? B : 1), 8>(kind, a, grid, st);
    case 12: return launch_kind<T, F_ELL, B, (B > 1 ? B : 1), 12>(kind, a, grid, st);
    default: return launch_kind<T, F_ELL, B, (B > 1 ? B : 1), 0>(kind, a, grid, st);
    }
}

// single vectors (both precisions) and complex128 blocks; complex64 blocks go
// to spmm2_kernel
template <typename T, int FMT>
static hipError_t launch_shape(int kind, const TermArgs &a, const KernelShape &s, hipStream_t st)
{
    if (s.B == 1) {
        if constexpr (FMT == F_ELL) {
            if (s.lr != 1)
                return hipErrorInvalidValue;
            return launch_ell<T, 1>(kind, a, s.grid, st);
        } else {
            switch (s.lr) {
            case 1: return launch_kind<T, FMT, 1, 1, 0>(kind, a, s.grid, st);
            case 2: return launch_kind<T, FMT, 1, 2, 0>(kind, a, s.grid, st);
            case 4: return launch_kind<T, FMT, 1, 4, 0>(kind, a, s.grid, st);
            case 8: return launch_kind<T, FMT, 1, 8, 0>(kind, a, s.grid, st);
            case 16: return launch_kind<T, FMT, 1, 16, 0>(kind, a, s.grid, st);
            default: return hipErrorInvalidValue;
            }
        }
    }
    if constexpr (!std::is_same<T, d2>::value) {
        return hipErrorInvalidValue;
    } else {
        if (s.lr != s.B)
            return hipErrorInvalidValue;
        if constexpr (FMT == F_ELL) {
            switch (s.B) {
            case 2: return launch_kind<T, FMT, 2, 2, 0>(kind, a, s.grid, st);
            case 4: return launch_kind<T, FMT, 4, 4, 0>(kind, a, s.grid, st);
            case 8: return launch_ell<T, 8>(kind, a, s.grid, st);
            case 16: return launch_ell<T, 16>(kind, a, s.grid, st);
            case 32: return launch_kind<T, FMT, 32, 32, 0>(kind, a, s.grid, st);
            case 64: return launch_kind<T, FMT, 64, 64, 0>(kind, a, s.grid, st);
            default: return hipErrorInvalidValue;
            }
        } else {
            switch (s.B) {
            case 2: return launch_kind<T, FMT, 2, 2, 0>(kind, a, s.grid, st);
            case 4: return launch_kind<T, FMT, 4, 4, 0>(kind, a, s.grid, st);
            case 8: return launch_kind<T, FMT, 8, 8, 0>(kind, a, s.grid, st);
            case 16: return launch_kind<T, FMT, 16, 16, 0>(kind, a, s.grid, st);
            case 32: return launch_kind<T, FMT, 32, 32, 0>(kind, a, s.grid, st);
            case 64: return launch_kind<T, FMT, 64, 64, 0>(kind, a, s.grid, st);
            default: return hipErrorInvalidValue;
            }
        }
    }
}

// ---- complex64 blocks: two vectors per lane ----------------------------------------------
//
// For complex64 blocks of B >= 2 vectors a lane owns two adjacent vectors of
// its row (one 16-byte access per row operand), B/2 lanes share a row and
// each loads the row's H entries (a broadcast within the group).  Same
// arithmetic as term_kernel's complex64 path.

__device__ __forceinline__ f2 lo2(f4 v) { return f2{v.x, v.y}; }
__device__ __forceinline__ f2 hi2(f4 v) { return f2{v.z, v.w}; }
__device__ __forceinline__ f4 join2(f2 a, f2 b) { return f4{a.x, a.y, b.x, b.y}; }
__device__ __forceinline__ d2 up(f2 v) { return d2{(double)v.x, (double)v.y}; }
__device__ __forceinline__ f2 down(d2 v) { return f2{(float)v.x, (float)v.y}; }

template <int FMT, int B, int KIND, int W>
__global__ __launch_bounds__(WG) void spmm2_kernel(TermArgs a)
{
    constexpr int LR = B / 2;
    constexpr int ROWS = WG / LR;
    const int lr = threadIdx.x % LR;
    const int rloc = threadIdx.x / LR;
    const int64_t n = a.n;
    const int64_t ntiles = (n + ROWS - 1) / ROWS;
    const f2 *__restrict__ x = static_cast<const f2 *>(a.x);
    f2 *__restrict__ y = static_cast<f2 *>(a.y);
    f2 *__restrict__ out = static_cast<f2 *>(a.out);
    const f2 *__restrict__ val = static_cast<const f2 *>(a.val);
    const f2 *__restrict__ psi0 = static_cast<const f2 *>(a.psi0);
    const int32_t *__restrict__ col = a.col;
    const d2 ca = d2{a.ca_re, a.ca_im};
    const d2 cb = d2{a.cb_re, a.cb_im};
    double dre[2] = {0.0, 0.0}, dim[2] = {0.0, 0.0}, nrm[2] = {0.0, 0.0};

    TileWalk tw = tile_walk(ntiles);
    for (int64_t tile = tw.t; tile < tw.end; tile += tw.stride) {
        const int64_t row = tile * ROWS + rloc;
        const bool live = row < n;
        const int64_t rr = live ? row : n - 1;
        const int64_t e = rr * B + 2 * lr;
        f4 xo{}, yo{}, oo{}, po{};
        if constexpr (KIND == K_FIRST || KIND == K_MOM0) {
            xo = *reinterpret_cast<const f4 *>(x + e);
        } else if constexpr (KIND == K_MOM) {
            xo = *reinterpret_cast<const f4 *>(x + e);
            yo = ld_stream(reinterpret_cast<const f4 *>(y + e));
        } else {
            yo = ld_stream(reinterpret_cast<const f4 *>(y + e));
            oo = ld_stream(reinterpret_cast<const f4 *>(out + e));
            if constexpr (KIND == K_LAST)
                po = ld_stream(reinterpret_cast<const f4 *>(psi0 + e));
        }
        f2 acc0{0, 0}, acc1{0, 0};
        if constexpr (FMT == F_ELL && W > 0) {
            int32_t c[W];
            f2 v[W];
#pragma unroll
            for (int s = 0; s < W; ++s) {
                const int64_t idx = (int64_t)s * a.ld + rr;
                c[s] = ld_stream(col + idx);
                v[s] = ld_stream(val + idx);
            }
            f4 xv[W];
#pragma unroll
            for (int s = 0; s < W; ++s)
                xv[s] = *reinterpret_cast<const f4 *>(x + (int64_t)c[s] * B + 2 * lr);
#pragma unroll
            for (int s = 0; s < W; ++s) {
                cmac(acc0, v[s], lo2(xv[s]));
                cmac(acc1, v[s], hi2(xv[s]));
            }
        } else if constexpr (FMT == F_ELL) {
            for (int s = 0; s < a.w; ++s) {
                const int64_t idx = (int64_t)s * a.ld + rr;
                const int32_t c = ld_stream(col + idx);
                const f2 v = ld_stream(val + idx);
                const f4 xv = *reinterpret_cast<const f4 *>(x + (int64_t)c * B + 2 * lr);
                cmac(acc0, v, lo2(xv));
                cmac(acc1, v, hi2(xv));
            }
        } else {
            int64_t beg, end;
            if (a.rp64) {
                const int64_t *rp = static_cast<const int64_t *>(a.rp);
                beg = rp[rr];
                end = rp[rr + 1];
            } else {
                const int32_t *rp = static_cast<const int32_t *>(a.rp);
                beg = rp[rr];
                end = rp[rr + 1];
            }
            for (int64_t j = beg; j < end; ++j) {
                const int32_t c = ld_stream(col + j);
                const f2 v = ld_stream(val + j);
                const f4 xv = *reinterpret_cast<const f4 *>(x + (int64_t)c * B + 2 * lr);
                cmac(acc0, v, lo2(xv));
                cmac(acc1, v, hi2(xv));
            }
        }
        if (live) {
            const d2 s0 = up(acc0) * a.scale, s1 = up(acc1) * a.scale;
            if constexpr (KIND == K_MOM0 || KIND == K_MOM) {
                const f2 ys0 = down(KIND == K_MOM0 ? s0 : s0 - up(lo2(yo)));
                const f2 ys1 = down(KIND == K_MOM0 ? s1 : s1 - up(hi2(yo)));
                st_stream(join2(ys0, ys1), reinterpret_cast<f4 *>(y + e));
                const f2 ys[2] = {ys0, ys1};
                const f2 xs[2] = {lo2(xo), hi2(xo)};
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const d2 xd = up(xs[q]), yd = up(ys[q]);
                    dre[q] += xd.x * yd.x + xd.y * yd.y;
                    dim[q] += xd.x * yd.y - xd.y * yd.x;
                    nrm[q] += xd.x * xd.x + xd.y * xd.y;
                }
            } else if constexpr (KIND == K_FIRST) {
                st_stream(join2(down(s0), down(s1)), reinterpret_cast<f4 *>(y + e));
                const d2 o0 = cmul(ca, up(lo2(xo))) + cmul(cb, s0);
                const d2 o1 = cmul(ca, up(hi2(xo))) + cmul(cb, s1);
                st_stream(join2(down(o0), down(o1)), reinterpret_cast<f4 *>(out + e));
            } else {
                const d2 y0 = s0 - up(lo2(yo)), y1 = s1 - up(hi2(yo));
                st_stream(join2(down(y0), down(y1)), reinterpret_cast<f4 *>(y + e));
                const f2 os0 = down(up(lo2(oo)) + cmul(ca, y0));
                const f2 os1 = down(up(hi2(oo)) + cmul(ca, y1));
                st_stream(join2(os0, os1), reinterpret_cast<f4 *>(out + e));
                if constexpr (KIND == K_LAST) {
                    const f2 os[2] = {os0, os1};
                    const f2 ps[2] = {lo2(po), hi2(po)};
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        const d2 p = up(ps[q]), o = up(os[q]);
                        dre[q] += p.x * o.x + p.y * o.y;
                        dim[q] += p.x * o.y - p.y * o.x;
                        nrm[q] += o.x * o.x + o.y * o.y;
                    }
                }
            }
        }
    }
    if constexpr (KIND == K_LAST || KIND == K_MOM0 || KIND == K_MOM) {
        // lanes with equal (lane mod LR) hold the same two vectors: fold them
#pragma unroll
        for (int off = 32; off >= LR; off >>= 1) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                dre[q] += __shfl_xor(dre[q], off, 64);
                dim[q] += __shfl_xor(dim[q], off, 64);
                nrm[q] += __shfl_xor(nrm[q], off, 64);
            }
        }
        __shared__ double red[WG / 64][B][3];
        const int lane = threadIdx.x % 64;
        const int wave = threadIdx.x / 64;
        if (lane < LR) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                red[wave][2 * lane + q][0] = dre[q];
                red[wave][2 * lane + q][1] = dim[q];
                red[wave][2 * lane + q][2] = nrm[q];
            }
        }
        __syncthreads();
        if (threadIdx.x < B) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
            for (int w = 0; w < WG / 64; ++w) {
                s0 += red[w][threadIdx.x][0];
                s1 += red[w][threadIdx.x][1];
                s2 += red[w][threadIdx.x][2];
            }
            double *p = a.partials + ((int64_t)blockIdx.x * B + threadIdx.x) * 4;
            p[0] = s0;
            p[1] = s1;
            p[2] = s2;
            p[3] = 0.0;
        }
    }
}

template <int FMT, int B, int W>
static hipError_t launch_spmm2_kind(int kind, const TermArgs &a, int grid, hipStream_t st)
{
    switch (kind) {
    case K_FIRST:
        hipLaunchKernelGGL((spmm2_kernel<FMT, B, K_FIRST, W>), dim3(grid), dim3(WG), 0, st, a);
        break;
    case K_MID:
        hipLaunchKernelGGL((spmm2_kernel<FMT, B, K_MID, W>), dim3(grid), dim3(WG), 0, st, a);
        break;
    case K_MOM0:
        hipLaunchKernelGGL((spmm2_kernel<FMT, B, K_MOM0, W>), dim3(grid), dim3(WG), 0, st, a);
        break;
    case K_MOM:
        hipLaunchKernelGGL((spmm2_kernel<FMT, B, K_MOM, W>), dim3(grid), dim3(WG), 0, st, a);
        break;
    default:
        hipLaunchKernelGGL((spmm2_kernel<FMT, B, K_LAST, W>), dim3(grid), dim3(WG), 0, st, a);
        break;
    }
    return hipGetLastError();
}

template <int B>
static hipError_t launch_spmm2_b(int kind, int fmt, const TermArgs &a, int grid, hipStream_t st)
{
    if (fmt == F_CSR)
        return launch_spmm2_kind<F_CSR, B, 0>(kind, a, grid, st);
    switch (a.w) {
    case 4: return launch_spmm2_kind<F_ELL, B, 4>(kind, a, grid, st);
    case 5: return launch_spmm2_kind<F_ELL, B, 5>(kind, a, grid, st);
    case 12: return launch_spmm2_kind<F_ELL, B, 12>(kind, a, grid, st);
    default: return launch_spmm2_kind<F_ELL, B, 0>(kind, a, grid, st);
    }
}

static hipError_t launch_spmm2(int kind, int fmt, const TermArgs &a, const KernelShape &s, hipStream_t st)
{
    if (s.lr * 2 != s.B)
        return hipErrorInvalidValue;
    switch (s.B) {
    case 2: return launch_spmm2_b<2>(kind, fmt, a, s.grid, st);
    case 4: return launch_spmm2_b<4>(kind, fmt, a, s.grid, st);
    case 8: return launch_spmm2_b<8>(kind, fmt, a, s.grid, st);
    case 16: return launch_spmm2_b<16>(kind, fmt, a, s.grid, st);
    case 32: return launch_spmm2_b<32>(kind, fmt, a, s.grid, st);
    case 64: return launch_spmm2_b<64>(kind, fmt, a, s.grid, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_term(int kind, int dtype, int fmt, const TermArgs &a, const KernelShape &s, hipStream_t st)
{
    if (s.grid % NXCD != 0 || s.grid <= 0 || a.n <= 0)
        return hipErrorInvalidValue;
    if (dtype == TBPM_C128)
        return fmt == F_CSR ? launch_shape<d2, F_CSR>(kind, a, s, st) : launch_shape<d2, F_ELL>(kind, a, s, st);
    if (s.B > 1 && s.lr * 2 == s.B)
        return launch_spmm2(kind, fmt, a, s, st);
    return fmt == F_CSR ? launch_shape<f2, F_CSR>(kind, a, s, st) : launch_shape<f2, F_ELL>(kind, a, s, st);
}

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

static int elem_grid(int64_t total)
{
    int64_t g = (total + WG - 1) / WG;
    if (g > 65536)
        g = 65536;
    if (g < 1)
        g = 1;
    return (int)g;
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
// one workgroup of RWG lanes, each summing a fixed strided subset, then a fixed
// tree: the order does not depend on timing, so results reproduce exactly.
constexpr int RWG = 1024;
__global__ __launch_bounds__(RWG) void reduce_kernel(const double *partials, int nblocks, int B, double *corr,
                                                     double *norms)
{
    __shared__ double red[RWG][3];
    for (int b = 0; b < B; ++b) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int k = threadIdx.x; k < nblocks; k += RWG) {
            const double *p = partials + ((int64_t)k * B + b) * 4;
            s0 += p[0];
            s1 += p[1];
            s2 += p[2];
        }
        red[threadIdx.x][0] = s0;
        red[threadIdx.x][1] = s1;
        red[threadIdx.x][2] = s2;
        __syncthreads();
        for (int h = RWG / 2; h > 0; h >>= 1) {
            if (threadIdx.x < h) {
                red[threadIdx.x][0] += red[threadIdx.x + h][0];
                red[threadIdx.x][1] += red[threadIdx.x + h][1];
                red[threadIdx.x][2] += red[threadIdx.x + h][2];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            corr[2 * b] = red[0][0];
            corr[2 * b + 1] = red[0][1];
            norms[b] = red[0][2];
        }
        __syncthreads();
    }
}

hipError_t launch_reduce(const double *partials, int nblocks, int B, double *corr, double *norms, hipStream_t st)
{
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(RWG), 0, st, partials, nblocks, B, corr, norms);
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

// ---- two Chebyshev terms per pass over H ------------------------------------------------
//
// Rows are renumbered into patches (compact regions of the sparsity graph,
// contiguous in the new order) with halos (rows outside a patch referenced by
// it).  One workgroup owns one patch:
//   phase A: y_m = scale H x_{m-1} - y_{m-2} for the patch rows (their H row
//            stays in registers) and for the halo rows, into LDS; patch rows
//            also to yout;
//   phase B: x_{m+1} = scale H y_m - x_{m-1} for the patch rows, gathering y_m
//            from LDS, then out += c_m y_m + c_{m+1} x_{m+1} (one update of
//            out for two terms).
// H is read once for two terms (plus the halo rows' H), out is touched once,
// and y_m is not read back from HBM.  Inputs (x_{m-1}, y_{m-2}) and outputs
// (y_m, x_{m+1}) are different buffers, since a halo row of one patch is a
// patch row of another.

template <typename T, int W, int NT, int R, int MODE>
__global__ __launch_bounds__(NT) void pair_kernel(PairArgs a)
{
    constexpr bool LAST = MODE == PAIR_LAST;
    constexpr bool MOM = MODE == PAIR_MOM;
    constexpr int NV = MOM ? 6 : 3;                 // partial sums per workgroup
    using E = Elem<T>;
    using A = typename E::acc;
    constexpr int S = NT * R;
    constexpr int HMAX = pair_halo_max(S);
    __shared__ T ylds[S + HMAX];
    __shared__ int32_t hidx[HMAX];
    __shared__ double red[NT / 64][NV];

    // one patch per workgroup; the patches of XCD (blockIdx % 8) are contiguous
    const int64_t per = (a.npatch + NXCD - 1) / NXCD;
    const int64_t patch = (int64_t)(blockIdx.x % NXCD) * per + blockIdx.x / NXCD;
    if (patch >= a.npatch)
        return;                                     // uniform over the workgroup
    const int64_t base = a.patch_ptr[patch];
    const int cnt = a.patch_ptr[patch + 1] - (int)base;
    const int hb = a.halo_ptr[patch];
    const int hc = min(a.halo_ptr[patch + 1] - hb, HMAX);
    const T *__restrict__ xin = static_cast<const T *>(a.xin);
    const T *__restrict__ yin = static_cast<const T *>(a.yin);
    T *__restrict__ yout = static_cast<T *>(a.yout);
    T *__restrict__ xout = static_cast<T *>(a.xout);
    T *__restrict__ out = static_cast<T *>(a.out);
    const T *__restrict__ val = static_cast<const T *>(a.val);
    const int32_t *__restrict__ col = a.col;
    const int64_t ld = a.ld;
    const double scale = a.scale;

    for (int h = threadIdx.x; h < hc; h += NT)
        hidx[h] = a.halo_rows[hb + h];

    // phase A, patch rows: lane t owns rows t, t + NT, ...
    int32_t c[R][W];
    T v[R][W];
    T yo[R], xo[R];
    d2 ym[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int li = threadIdx.x + r * NT;
        const int64_t row = base + (li < cnt ? li : cnt - 1);
#pragma unroll
        for (int s = 0; s < W; ++s) {
            c[r][s] = ld_stream(col + (int64_t)s * ld + row);
            v[r][s] = ld_stream(val + (int64_t)s * ld + row);
        }
        yo[r] = ld_stream(yin + row);
        xo[r] = xin[row];                           // x_{m-1} of the row, for phase B
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        T xv[W];
#pragma unroll
        for (int s = 0; s < W; ++s)
            xv[s] = xin[c[r][s]];
        A acc{0, 0};
#pragma unroll
        for (int s = 0; s < W; ++s)
            cmac(acc, (A)v[r][s], (A)xv[s]);
        ym[r] = E::acc_to_d(acc) * scale - E::to_d(yo[r]);
        if constexpr (MOM)
            ym[r] = E::to_d(E::from_d(ym[r]));      // the stored value enters the inner products
        const int li = threadIdx.x + r * NT;
        if (li < cnt) {
            const T ys = E::from_d(ym[r]);
            ylds[li] = ys;
            st_stream(ys, yout + base + li);
        }
    }
    __syncthreads();                                // hidx complete

    // phase A, halo rows (their H rows are stored contiguously per patch)
    const int32_t *__restrict__ hcol = a.hcol;
    const T *__restrict__ hval = static_cast<const T *>(a.hval);
    for (int h = threadIdx.x; h < hc; h += NT) {
        const int64_t rh = hidx[h];
        const int64_t g = (int64_t)hb + h;
        int32_t ch[W];
        T vh[W];
#pragma unroll
        for (int s = 0; s < W; ++s) {
            ch[s] = ld_stream(hcol + (int64_t)s * a.ldh + g);
            vh[s] = ld_stream(hval + (int64_t)s * a.ldh + g);
        }
        const T yh = yin[rh];
        T xv[W];
#pragma unroll
        for (int s = 0; s < W; ++s)
            xv[s] = xin[ch[s]];
        A acc{0, 0};
#pragma unroll
        for (int s = 0; s < W; ++s)
            cmac(acc, (A)vh[s], (A)xv[s]);
        ylds[cnt + h] = E::from_d(E::acc_to_d(acc) * scale - E::to_d(yh));
    }
    __syncthreads();                                // y_m of patch and halo in LDS

    // phase B
    const d2 c0 = d2{a.c0_re, a.c0_im};
    const d2 c1 = d2{a.c1_re, a.c1_im};
    // LAST: <psi0|out>, <out|out>.  MOM: with x = p_m (xin), y = p_m+1, z = p_m+2:
    // <x|y>, <x|x>, <y|z>, <y|y>
    double sum[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q)
        sum[q] = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int li = threadIdx.x + r * NT;
        if (li < cnt) {
            const int64_t row = base + li;
            A acc{0, 0};
#pragma unroll
            for (int s = 0; s < W; ++s) {
                int l = (int)(c[r][s] - base);
                if ((unsigned)l >= (unsigned)cnt) {     // halo: position in the sorted halo list
                    int lo = 0, hi = hc;
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (hidx[mid] < c[r][s])
                            lo = mid + 1;
                        else
                            hi = mid;
                    }
                    l = cnt + min(lo, hc - 1);
                }
                cmac(acc, (A)v[r][s], (A)ylds[l]);
            }
            const d2 xn = E::acc_to_d(acc) * scale - E::to_d(xo[r]);
            st_stream(E::from_d(xn), xout + row);
            if constexpr (MOM) {
                const d2 xd = E::to_d(xo[r]), yd = ym[r], zd = E::to_d(E::from_d(xn));
                sum[0] += xd.x * yd.x + xd.y * yd.y;
                sum[1] += xd.x * yd.y - xd.y * yd.x;
                sum[2] += xd.x * xd.x + xd.y * xd.y;
                sum[3] += yd.x * zd.x + yd.y * zd.y;
                sum[4] += yd.x * zd.y - yd.y * zd.x;
                sum[5] += yd.x * yd.x + yd.y * yd.y;
                continue;
            }
            const d2 on = (E::to_d(ld_stream(out + row)) + cmul(c0, ym[r])) + cmul(c1, xn);
            const T os = E::from_d(on);
            st_stream(os, out + row);
            if constexpr (LAST) {
                const d2 p = E::to_d(ld_stream(static_cast<const T *>(a.psi0) + row));
                const d2 o = E::to_d(os);
                sum[0] += p.x * o.x + p.y * o.y;
                sum[1] += p.x * o.y - p.y * o.x;
                sum[2] += o.x * o.x + o.y * o.y;
            }
        }
    }
    if constexpr (LAST || MOM) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
            for (int q = 0; q < NV; ++q)
                sum[q] += __shfl_xor(sum[q], off, 64);
        }
        const int wave = threadIdx.x / 64;
        if (threadIdx.x % 64 == 0) {
#pragma unroll
            for (int q = 0; q < NV; ++q)
                red[wave][q] = sum[q];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double t[NV];
#pragma unroll
            for (int q = 0; q < NV; ++q)
                t[q] = 0.0;
            for (int w = 0; w < NT / 64; ++w) {
#pragma unroll
                for (int q = 0; q < NV; ++q)
                    t[q] += red[w][q];
            }
            double *p = a.partials + patch * 4;
            p[0] = t[0];
            p[1] = t[1];
            p[2] = t[2];
            p[3] = 0.0;
            if constexpr (MOM) {
                double *p2 = a.partials2 + patch * 4;
                p2[0] = t[3];
                p2[1] = t[4];
                p2[2] = t[5];
                p2[3] = 0.0;
            }
        }
    }
}


bool pair_supported(int w, int patch_rows)
{
    return (w == 3 || w == 4 || w == 5 || w == 8 || w == 12) &&
           (patch_rows == PAIR_WG || patch_rows == 2 * PAIR_WG);
}

int pair_grid(int64_t npatch) { return (int)((npatch + NXCD - 1) / NXCD * NXCD); }

// 2048-row patches: 1024 lanes with 2 rows each; 1024-row patches: 512 lanes
// with 2 rows each (two workgroups per CU overlap each other's barriers)
template <typename T, int W, int R>
static hipError_t launch_pair_w(int mode, const PairArgs &a, hipStream_t st)
{
    const int g = pair_grid(a.npatch);
    constexpr int NT = R == 2 ? 1024 : 512;
    switch (mode) {
    case PAIR_LAST:
        hipLaunchKernelGGL((pair_kernel<T, W, NT, 2, PAIR_LAST>), dim3(g), dim3(NT), 0, st, a);
        break;
    case PAIR_MOM:
        hipLaunchKernelGGL((pair_kernel<T, W, NT, 2, PAIR_MOM>), dim3(g), dim3(NT), 0, st, a);
        break;
    default:
        hipLaunchKernelGGL((pair_kernel<T, W, NT, 2, PAIR_MID>), dim3(g), dim3(NT), 0, st, a);
        break;
    }
    return hipGetLastError();
}

template <typename T, int R>
static hipError_t launch_pair_r(int mode, const PairArgs &a, hipStream_t st)
{
    switch (a.w) {
    case 3: return launch_pair_w<T, 3, R>(mode, a, st);
    case 4: return launch_pair_w<T, 4, R>(mode, a, st);
    case 5: return launch_pair_w<T, 5, R>(mode, a, st);
    case 8: return launch_pair_w<T, 8, R>(mode, a, st);
    case 12: return launch_pair_w<T, 12, R>(mode, a, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pair(int mode, int dtype, const PairArgs &a, int patch_rows, hipStream_t st)
{
    if (!pair_supported(a.w, patch_rows) || a.npatch <= 0 || mode < PAIR_MID || mode > PAIR_MOM ||
        (mode == PAIR_MOM && !a.partials2))
        return hipErrorInvalidValue;
    const int R = patch_rows / PAIR_WG;
    if (dtype == TBPM_C128)
        return R == 1 ? launch_pair_r<d2, 1>(mode, a, st) : launch_pair_r<d2, 2>(mode, a, st);
    return R == 1 ? launch_pair_r<f2, 1>(mode, a, st) : launch_pair_r<f2, 2>(mode, a, st);
}


// ---- K = 3, 4 Chebyshev terms per pass -------------------------------------------------------
//
// Generalises pair_kernel: stage s (s = 0..K-1) forms p_{m+s} for the patch
// and halo layers 1..K-1-s (a row of layer l references only the patch and
// layers l-1..l+1, so every operand of stage s is in stage s-1's rows).  LDS
// holds p_{m+s} for s <= K-2, each buffer laid out as [patch rows | halo rows
// in layer order], so a row has the same position in every buffer that holds
// it.  Patch rows keep their H row in registers through all stages and
// accumulate out in FP64; only p_{m+K-2}, p_{m+K-1} and out go to HBM.

template <typename T, int W, int NT, int R, int K, bool LAST>
__global__ __launch_bounds__(NT) void multi_kernel(MultiArgs a)
{
    using E = Elem<T>;
    using A = typename E::acc;
    extern __shared__ __align__(16) unsigned char smem[];

    const int64_t per = (a.npatch + NXCD - 1) / NXCD;
    const int64_t patch = (int64_t)(blockIdx.x % NXCD) * per + blockIdx.x / NXCD;
    if (patch >= a.npatch)
        return;                                     // uniform over the workgroup
    const int64_t base = a.patch_ptr[patch];
    const int cnt = a.patch_ptr[patch + 1] - (int)base;
    const int hb = a.halo_ptr[patch];
    const int htot = a.halo_ptr[patch + 1] - hb;
    // hl[l]: halo rows in layers 1..l (prefix of the halo list)
    int hl[K];
    hl[0] = 0;
#pragma unroll
    for (int l = 1; l < K; ++l)
        hl[l] = hl[l - 1] + a.layer_cnt[patch * a.depth + (l - 1)];

    int32_t *skey = reinterpret_cast<int32_t *>(smem);
    int32_t *spos = skey + htot;
    T *buf[K - 1];
    {
        size_t off = ((size_t)htot * 8 + 15) & ~(size_t)15;
#pragma unroll
        for (int j = 0; j < K - 1; ++j) {
            buf[j] = reinterpret_cast<T *>(smem + off);
            off += (size_t)(cnt + hl[K - 1 - j]) * sizeof(T);
        }
    }
    for (int i = threadIdx.x; i < htot; i += NT) {
        skey[i] = a.key_rows[hb + i];
        spos[i] = a.key_pos[hb + i];
    }

    const T *__restrict__ xin = static_cast<const T *>(a.xin);
    const T *__restrict__ yin = static_cast<const T *>(a.yin);
    const T *__restrict__ val = static_cast<const T *>(a.val);
    const int32_t *__restrict__ col = a.col;
    const int32_t *__restrict__ hcol = a.hcol;
    const T *__restrict__ hval = static_cast<const T *>(a.hval);
    const int64_t ld = a.ld;
    const double scale = a.scale;

    // patch rows: H row, p_{m-2}, p_{m-1} and out of the row
    int32_t c[R][W];
    T v[R][W];
    T yo[R], xo[R];
    d2 oacc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int li = threadIdx.x + r * NT;
        const int64_t row = base + (li < cnt ? li : cnt - 1);
#pragma unroll
        for (int s = 0; s < W; ++s) {
            c[r][s] = ld_stream(col + (int64_t)s * ld + row);
            v[r][s] = ld_stream(val + (int64_t)s * ld + row);
        }
        yo[r] = ld_stream(yin + row);
        xo[r] = xin[row];
        oacc[r] = E::to_d(ld_stream(static_cast<const T *>(a.out) + row));
    }
    __syncthreads();                                // lookup keys in LDS

    // position of stored row cc in the LDS buffers
    auto lpos = [&](int32_t cc) -> int {
        int l = (int)(cc - base);
        if ((unsigned)l < (unsigned)cnt)
            return l;
        int lo = 0, hi = htot;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (skey[mid] < cc)
                lo = mid + 1;
            else
                hi = mid;
        }
        return cnt + spos[min(lo, htot - 1)];
    };

#pragma unroll
    for (int s = 0; s < K; ++s) {
        const d2 cs = d2{a.c_re[s], a.c_im[s]};
        // patch rows
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int li = threadIdx.x + r * NT;
            if (li < cnt) {
                A acc{0, 0};
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    const T src = (s == 0) ? xin[c[r][q]] : buf[s == 0 ? 0 : s - 1][lpos(c[r][q])];
                    cmac(acc, (A)v[r][q], (A)src);
                }
                const T yt = (s == 0) ? yo[r] : (s == 1) ? xo[r] : buf[s < 2 ? 0 : s - 2][li];
                const d2 p = E::acc_to_d(acc) * scale - E::to_d(yt);
                oacc[r] = oacc[r] + cmul(cs, p);
                const T ps = E::from_d(p);
                if (s <= K - 2)
                    buf[s <= K - 2 ? s : 0][li] = ps;
                if (s == K - 2)
                    st_stream(ps, static_cast<T *>(a.yout) + base + li);
                if (s == K - 1)
                    st_stream(ps, static_cast<T *>(a.xout) + base + li);
            }
        }
        // halo rows of layers 1..K-1-s
        if (s <= K - 2) {
            const int nh = hl[K - 1 - s];
            for (int h = threadIdx.x; h < nh; h += NT) {
                const int64_t g = (int64_t)hb + h;
                const int64_t rh = a.halo_rows[g];
                A acc{0, 0};
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    const int32_t cc = hcol[(int64_t)q * a.ldh + g];
                    const T vv = hval[(int64_t)q * a.ldh + g];
                    const T src = (s == 0) ? xin[cc] : buf[s == 0 ? 0 : s - 1][lpos(cc)];
                    cmac(acc, (A)vv, (A)src);
                }
                const T yt = (s == 0) ? yin[rh] : (s == 1) ? xin[rh] : buf[s < 2 ? 0 : s - 2][cnt + h];
                buf[s <= K - 2 ? s : 0][cnt + h] = E::from_d(E::acc_to_d(acc) * scale - E::to_d(yt));
            }
        }
        __syncthreads();
    }

    double dre = 0.0, dim = 0.0, nrm = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int li = threadIdx.x + r * NT;
        if (li < cnt) {
            const int64_t row = base + li;
            const T os = E::from_d(oacc[r]);
            st_stream(os, static_cast<T *>(a.out) + row);
            if constexpr (LAST) {
                const d2 p = E::to_d(ld_stream(static_cast<const T *>(a.psi0) + row));
                const d2 o = E::to_d(os);
                dre += p.x * o.x + p.y * o.y;
                dim += p.x * o.y - p.y * o.x;
                nrm += o.x * o.x + o.y * o.y;
            }
        }
    }
    if constexpr (LAST) {
        __shared__ double red[NT / 64][3];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            dre += __shfl_xor(dre, off, 64);
            dim += __shfl_xor(dim, off, 64);
            nrm += __shfl_xor(nrm, off, 64);
        }
        const int wave = threadIdx.x / 64;
        if (threadIdx.x % 64 == 0) {
            red[wave][0] = dre;
            red[wave][1] = dim;
            red[wave][2] = nrm;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
            for (int w = 0; w < NT / 64; ++w) {
                s0 += red[w][0];
                s1 += red[w][1];
                s2 += red[w][2];
            }
            double *p = a.partials + patch * 4;
            p[0] = s0;
            p[1] = s1;
            p[2] = s2;
            p[3] = 0.0;
        }
    }
}

template <typename T, int W, int K, bool LAST>
static hipError_t launch_multi_one(const MultiArgs &a, size_t lds, hipStream_t st)
{
    constexpr int NT = 512;                         // 1024-row patches, 2 rows per lane
    auto fn = multi_kernel<T, W, NT, 2, K, LAST>;
    static size_t granted = 0;                      // per instantiation
    if (lds > granted) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
        granted = lds;
    }
    hipLaunchKernelGGL(fn, dim3(pair_grid(a.npatch)), dim3(NT), lds, st, a);
    return hipGetLastError();
}

template <typename T, int K>
static hipError_t launch_multi_k(int last, const MultiArgs &a, size_t lds, hipStream_t st)
{
    switch (a.w) {
    case 3: return last ? launch_multi_one<T, 3, K, true>(a, lds, st) : launch_multi_one<T, 3, K, false>(a, lds, st);
    case 4: return last ? launch_multi_one<T, 4, K, true>(a, lds, st) : launch_multi_one<T, 4, K, false>(a, lds, st);
    case 5: return last ? launch_multi_one<T, 5, K, true>(a, lds, st) : launch_multi_one<T, 5, K, false>(a, lds, st);
    case 8: return last ? launch_multi_one<T, 8, K, true>(a, lds, st) : launch_multi_one<T, 8, K, false>(a, lds, st);
    case 12:
        return last ? launch_multi_one<T, 12, K, true>(a, lds, st) : launch_multi_one<T, 12, K, false>(a, lds, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_multi(int K, int last, int dtype, const MultiArgs &a, size_t lds_bytes, hipStream_t st)
{
    if (a.npatch <= 0 || (K != 3 && K != 4))
        return hipErrorInvalidValue;
    if (dtype == TBPM_C128)
        return K == 3 ? launch_multi_k<d2, 3>(last, a, lds_bytes, st) : launch_multi_k<d2, 4>(last, a, lds_bytes, st);
    return K == 3 ? launch_multi_k<f2, 3>(last, a, lds_bytes, st) : launch_multi_k<f2, 4>(last, a, lds_bytes, st);
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
