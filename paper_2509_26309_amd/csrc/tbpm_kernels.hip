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

#include <atomic>
#include <type_traits>

#include "tbpm_device.h"

namespace tbpm {

// ---- the Chebyshev term kernel ---------------------------------------------------
//
// W > 0: ELL with a compile-time width, so every load of the row (its W column
// indices and values, and the vector operands of the update) is issued before
// the first dependent gather of x.  W == 0: runtime width (ELL) or CSR.
// Rows past n in the last tile load row n-1 (in bounds) and store nothing.

template <typename T, int FMT, int B, int LR, int KIND, int W>
__global__ __launch_bounds__(WG) void term_kernel(TermArgs a)
{
    using E = Elem<T>;
    using A = typename E::acc;
    constexpr int ROWS = WG / LR;
    const int lr = threadIdx.x % LR;
    const int rloc = threadIdx.x / LR;
    const int64_t n = a.n;
    const bool listed = a.plist != nullptr;                 // only the listed patches' rows
    const int64_t ntiles = listed ? a.pcount * a.patch_tiles : (n + ROWS - 1) / ROWS;
    const T *__restrict__ x = static_cast<const T *>(a.x);
    T *__restrict__ y = static_cast<T *>(a.y);
    T *__restrict__ out = static_cast<T *>(a.out);
    const T *__restrict__ val = static_cast<const T *>(a.val);
    const T *__restrict__ psi0 = static_cast<const T *>(a.psi0);
    const int32_t *__restrict__ col = a.col;
    const d2 ca = d2{a.ca_re, a.ca_im};
    const d2 cb = d2{a.cb_re, a.cb_im};
    const bool owner = (B > 1) || (lr == 0);
    // Clenshaw (FIRST / MID / LAST kinds): no out; psi enters with c_a (c_b in FIRST)
    constexpr bool CLK = KIND == K_FIRST || KIND == K_MID || KIND == K_LAST;
    const bool cl = CLK && a.cl != 0;
    const bool use_y = !cl || a.no_y == 0;
    const T *__restrict__ psi = static_cast<const T *>(a.psi);

    double dre = 0.0, dim = 0.0, nrm = 0.0;

    TileWalk tw = tile_walk(ntiles);
    for (int64_t r0 = tw.t; r0 < tw.end; r0 += tw.stride)
    for (int64_t tile = r0, r1 = r0 + tw.run < tw.end ? r0 + tw.run : tw.end; tile < r1; ++tile) {
        int64_t row, end = n;
        if (listed) {
            const int64_t q = a.plist[tile / a.patch_tiles];
            end = a.patch_ptr[q + 1];
            row = a.patch_ptr[q] + (tile % a.patch_tiles) * ROWS + rloc;
        } else {
            row = tile * ROWS + rloc;
        }
        const bool live = row < end;
        const int64_t rr = live ? row : end - 1;            // in-bounds row for loads
        const int64_t e = rr * B + (B > 1 ? lr : 0);

        // operands of the update, independent of the sparse product
        T xo{}, yo{}, oo{}, po{}, qo{};
        if (owner) {
            if constexpr (KIND == K_FIRST || KIND == K_MOM0) {
                xo = x[e];
            } else if constexpr (KIND == K_MOM) {
                xo = x[e];
                yo = ld_stream(y + e);
            } else {
                if (use_y)
                    yo = ld_stream(y + e);
                if (cl)
                    qo = ld_stream(psi + e);
                else
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
                if (cl) {
                    st_stream(E::from_d(cmul(ca, s) + cmul(cb, E::to_d(xo))), y + e);
                } else {
                    st_stream(E::from_d(s), y + e);
                    st_stream(E::from_d(cmul(ca, E::to_d(xo)) + cmul(cb, s)), out + e);
                }
            } else if (cl) {
                const d2 yn = (use_y ? s - E::to_d(yo) : s) + cmul(ca, E::to_d(qo));
                const T ys = E::from_d(yn);
                st_stream(ys, y + e);
                if constexpr (KIND == K_LAST) {
                    const d2 p = E::to_d(po);
                    const d2 o = E::to_d(ys);
                    dre += p.x * o.x + p.y * o.y;
                    dim += p.x * o.y - p.y * o.x;
                    nrm += o.x * o.x + o.y * o.y;
                }
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

// The update of one row for a lane's two complex64 vectors (spmm2_kernel and
// patch_spmm_kernel): s0, s1 are the scaled products (FP64), xo/yo/oo/po/qo
// the row's x, y, out, psi0 and psi operands as loaded for KIND; yp, op the
// row's y and out (two vectors each); dots accumulate into dre/dim/nrm.
template <int KIND>
__device__ __forceinline__ void spmm2_update(d2 s0, d2 s1, f4 xo, f4 yo, f4 oo, f4 po, f4 qo, d2 ca, d2 cb, bool cl,
                                             bool use_y, f4 *yp, f4 *op, double (&dre)[2], double (&dim)[2],
                                             double (&nrm)[2])
{
    if constexpr (KIND == K_MOM0 || KIND == K_MOM) {
        const f2 ys0 = down(KIND == K_MOM0 ? s0 : s0 - up(lo2(yo)));
        const f2 ys1 = down(KIND == K_MOM0 ? s1 : s1 - up(hi2(yo)));
        st_stream(join2(ys0, ys1), yp);
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
        if (cl) {
            const d2 b0 = cmul(ca, s0) + cmul(cb, up(lo2(xo)));
            const d2 b1 = cmul(ca, s1) + cmul(cb, up(hi2(xo)));
            st_stream(join2(down(b0), down(b1)), yp);
        } else {
            st_stream(join2(down(s0), down(s1)), yp);
            const d2 o0 = cmul(ca, up(lo2(xo))) + cmul(cb, s0);
            const d2 o1 = cmul(ca, up(hi2(xo))) + cmul(cb, s1);
            st_stream(join2(down(o0), down(o1)), op);
        }
    } else if (cl) {
        const d2 y0 = (use_y ? s0 - up(lo2(yo)) : s0) + cmul(ca, up(lo2(qo)));
        const d2 y1 = (use_y ? s1 - up(hi2(yo)) : s1) + cmul(ca, up(hi2(qo)));
        const f2 ys0 = down(y0), ys1 = down(y1);
        st_stream(join2(ys0, ys1), yp);
        if constexpr (KIND == K_LAST) {
            const f2 os[2] = {ys0, ys1};
            const f2 ps[2] = {lo2(po), hi2(po)};
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const d2 p = up(ps[q]), o = up(os[q]);
                dre[q] += p.x * o.x + p.y * o.y;
                dim[q] += p.x * o.y - p.y * o.x;
                nrm[q] += o.x * o.x + o.y * o.y;
            }
        }
    } else {
        const d2 y0 = s0 - up(lo2(yo)), y1 = s1 - up(hi2(yo));
        st_stream(join2(down(y0), down(y1)), yp);
        const f2 os0 = down(up(lo2(oo)) + cmul(ca, y0));
        const f2 os1 = down(up(hi2(oo)) + cmul(ca, y1));
        st_stream(join2(os0, os1), op);
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

template <int FMT, int B, int KIND, int W>
__global__ __launch_bounds__(WG) void spmm2_kernel(TermArgs a)
{
    constexpr int LR = B / 2;
    constexpr int ROWS = WG / LR;
    const int lr = threadIdx.x % LR;
    const int rloc = threadIdx.x / LR;
    const int64_t n = a.n;
    const bool listed = a.plist != nullptr;
    const int64_t ntiles = listed ? a.pcount * a.patch_tiles : (n + ROWS - 1) / ROWS;
    const f2 *__restrict__ x = static_cast<const f2 *>(a.x);
    f2 *__restrict__ y = static_cast<f2 *>(a.y);
    f2 *__restrict__ out = static_cast<f2 *>(a.out);
    const f2 *__restrict__ val = static_cast<const f2 *>(a.val);
    const f2 *__restrict__ psi0 = static_cast<const f2 *>(a.psi0);
    const int32_t *__restrict__ col = a.col;
    const d2 ca = d2{a.ca_re, a.ca_im};
    const d2 cb = d2{a.cb_re, a.cb_im};
    constexpr bool CLK = KIND == K_FIRST || KIND == K_MID || KIND == K_LAST;
    const bool cl = CLK && a.cl != 0;                  // Clenshaw, as in term_kernel
    const bool use_y = !cl || a.no_y == 0;
    const f2 *__restrict__ psi = static_cast<const f2 *>(a.psi);
    double dre[2] = {0.0, 0.0}, dim[2] = {0.0, 0.0}, nrm[2] = {0.0, 0.0};

    TileWalk tw = tile_walk(ntiles);
    for (int64_t r0 = tw.t; r0 < tw.end; r0 += tw.stride)
    for (int64_t tile = r0, r1 = r0 + tw.run < tw.end ? r0 + tw.run : tw.end; tile < r1; ++tile) {
        int64_t row, end = n;
        if (listed) {
            const int64_t q = a.plist[tile / a.patch_tiles];
            end = a.patch_ptr[q + 1];
            row = a.patch_ptr[q] + (tile % a.patch_tiles) * ROWS + rloc;
        } else {
            row = tile * ROWS + rloc;
        }
        const bool live = row < end;
        const int64_t rr = live ? row : end - 1;
        const int64_t e = rr * B + 2 * lr;
        f4 xo{}, yo{}, oo{}, po{}, qo{};
        if constexpr (KIND == K_FIRST || KIND == K_MOM0) {
            xo = *reinterpret_cast<const f4 *>(x + e);
        } else if constexpr (KIND == K_MOM) {
            xo = *reinterpret_cast<const f4 *>(x + e);
            yo = ld_stream(reinterpret_cast<const f4 *>(y + e));
        } else {
            if (use_y)
                yo = ld_stream(reinterpret_cast<const f4 *>(y + e));
            if (cl)
                qo = ld_stream(reinterpret_cast<const f4 *>(psi + e));
            else
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
        if (live)
            spmm2_update<KIND>(up(acc0) * a.scale, up(acc1) * a.scale, xo, yo, oo, po, qo, ca, cb, cl, use_y,
                               reinterpret_cast<f4 *>(y + e), reinterpret_cast<f4 *>(out + e), dre, dim, nrm);
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

// ---- complex64 blocks on patch-reordered H: the patch's x staged in LDS ---------------
//
// One workgroup per (patch, run of TROWS rows of it), TROWS = 64 KiB / (B x 8
// bytes): the whole patch for blocks of 8 vectors, halves for 16.  Phase 1
// copies x of the run's rows (all B vectors, one contiguous span) into LDS
// with coalesced 16-byte loads; after a barrier, phase 2 forms the term for
// those rows exactly as spmm2_kernel does, taking x from LDS for columns
// inside the run and from global memory (L2) for the others.  So each x
// value is read from HBM once per term plus the halo, instead of once per
// line fill of every row that gathers it, which the L2 cannot hold across
// the many patches an XCD has in flight.  The runs of one patch are
// workgroups j and j + 8 (same XCD, dispatched together), so the second
// finds the first's rows in L2.  Partial sums (LAST, MOM0, MOM) are written
// per run: partials[patch * NSUB + run][b][4].

constexpr int PSPMM_WG = 512;            // lanes per workgroup
constexpr int PSPMM_ROWS = 1024;         // largest patch
constexpr int PSPMM_LDS = 65536;         // bytes of staged x per workgroup
constexpr int PSPMM_VPL = 2;             // vectors per lane (one 16-byte chunk of a row; 1, 4, 8 are slower)
typedef __attribute__((address_space(1))) const f4 gf4;   // f4 in global memory

// the per-row diagonal value of a value table (index 255): complex, or its
// real part alone with an imaginary part of +0; 0 without a per-row diagonal
// (NT: a non-temporal load)
template <typename T, bool NT = true>
__device__ __forceinline__ T diag_of(const T *vdiag, int32_t real, int64_t row)
{
    using Re = decltype(T{}.x);
    if (!vdiag)
        return T{};
    if (real) {
        const Re *re = reinterpret_cast<const Re *>(vdiag) + row;
        return T{NT ? ld_stream(re) : *re, Re(0)};
    }
    return NT ? ld_stream(vdiag + row) : vdiag[row];
}
constexpr int PSPMM_HMAX = pair_halo_max(PSPMM_ROWS);   // largest halo of a staged patch
constexpr int pspmm_rows(int B) { return PSPMM_LDS / (B * 8); }

// value of lane k of each quad of lanes (DPP quad_perm broadcast); k is a
// constant once the caller's loop is unrolled
__device__ __forceinline__ int quad_bcast(int v, int k)
{
    switch (k) {
    case 0: return __builtin_amdgcn_update_dpp(0, v, 0x00, 0xF, 0xF, false);
    case 1: return __builtin_amdgcn_update_dpp(0, v, 0x55, 0xF, 0xF, false);
    case 2: return __builtin_amdgcn_update_dpp(0, v, 0xAA, 0xF, 0xF, false);
    default: return __builtin_amdgcn_update_dpp(0, v, 0xFF, 0xF, 0xF, false);
    }
}
constexpr int pspmm_nsub(int B) { return (PSPMM_ROWS + pspmm_rows(B) - 1) / pspmm_rows(B); }

template <int B, int KIND, int W, bool DICT>
__global__ __launch_bounds__(PSPMM_WG) void patch_spmm_kernel(TermArgs a)
{
    constexpr int VPL = B < PSPMM_VPL ? B : PSPMM_VPL;
    constexpr int NC = VPL / 2;                // 16-byte chunks (two complex64) per lane
    constexpr int LR = B / VPL;                // lanes per row
    constexpr int RC = B / 2;                  // 16-byte chunks per row
    constexpr int ROWS = PSPMM_WG / LR;        // rows per pass
    constexpr int TROWS = pspmm_rows(B);       // rows staged per workgroup
    constexpr int NSUB = pspmm_nsub(B);
    constexpr bool DOTS = KIND == K_LAST || KIND == K_MOM0 || KIND == K_MOM;
    __shared__ f4 xs[TROWS * RC];              // x of the run's rows, [row][RC]
    __shared__ f2 vtab[DICT ? 256 : 1];        // value table (DICT: H entries are one-byte indices)
    __shared__ int32_t hrow[PSPMM_HMAX];       // the patch's halo rows (local columns >= the patch's rows)

    const int64_t per = (a.npatch + NXCD - 1) / NXCD;
    const int64_t u = blockIdx.x / NXCD;
    const int64_t patch = (int64_t)(blockIdx.x % NXCD) * per + u / NSUB;
    const int sub = (int)(u % NSUB);
    if (patch >= a.npatch)
        return;                                 // uniform over the workgroup
    const int64_t pbase = a.patch_ptr[patch];
    const int pcnt = a.patch_ptr[patch + 1] - (int)pbase;
    const int64_t base = pbase + (int64_t)sub * TROWS;
    const int cnt = max(0, min(TROWS, pcnt - sub * TROWS));
    const int lr = threadIdx.x % LR;
    const int rl = threadIdx.x / LR;
    const int c0 = lr * NC;                    // the lane's first chunk of a row
    const f4 *__restrict__ xg = static_cast<const f4 *>(a.x);
    const gf4 *__restrict__ xgl = (const gf4 *)xg;
    const f2 *__restrict__ val = static_cast<const f2 *>(a.val);
    const uint64_t *__restrict__ lcol = a.lcol;
    f4 *__restrict__ y = static_cast<f4 *>(a.y);
    f4 *__restrict__ out = static_cast<f4 *>(a.out);
    const f4 *__restrict__ psi0 = static_cast<const f4 *>(a.psi0);
    const f4 *__restrict__ psi = static_cast<const f4 *>(a.psi);
    const d2 ca = d2{a.ca_re, a.ca_im};
    const d2 cb = d2{a.cb_re, a.cb_im};
    constexpr bool CLK = KIND == K_FIRST || KIND == K_MID || KIND == K_LAST;
    const bool cl = CLK && a.cl != 0;
    const bool use_y = !cl || a.no_y == 0;

    // The four lanes of a quad share a row (LR is 4 or 8): lane k of the quad
    // loads the row's column word k (four 2-byte local columns) and its values
    // k, k + 4, ..., and the others take them by DPP broadcast, so H is loaded
    // LR / 4 times per row instead of LR times.  Each
    // pass loads the next pass's entries before its own gathers, into the other
    // of two register sets (the passes alternate between them).
    // With a value table (DICT) lane k < (W+3)/4 of the quad loads instead the
    // row's index word k (slot s in byte s % 4 of word s / 4), every lane the
    // row's diagonal value (index 255).
    static_assert(LR % 4 == 0, "the lanes of a quad share a row");
    constexpr int WQ = (W + 3) / 4;
    const int qk = threadIdx.x & 3;
    const f2 *__restrict__ vdiag = static_cast<const f2 *>(a.vdiag);
    struct HSet {
        uint64_t cw;
        f2 v[WQ];
        uint32_t w;
        f2 d;
    };
    auto load_h = [&](int r0, HSet &h) {
        const int64_t row = base + min(r0 + rl, cnt - 1);
        // lane k of the quad: the row's column word k (slots 4k .. 4k + 3)
        h.cw = qk < WQ ? ld_stream(lcol + (int64_t)qk * a.ld + row) : 0ull;
        if constexpr (!DICT) {
#pragma unroll
            for (int i = 0; i < WQ; ++i) {
                const int q = qk + 4 * i;
                h.v[i] = q < W ? ld_stream(val + (int64_t)q * a.ld + row) : f2{0.f, 0.f};
            }
        }
        if constexpr (DICT) {
            h.w = qk < WQ ? ld_stream(a.vidx + (int64_t)qk * a.ld + row) : 0u;
            h.d = diag_of(vdiag, a.vdiag_real, row);
        }
    };
    if constexpr (DICT) {
        for (int i = threadIdx.x; i < 256; i += PSPMM_WG)
            vtab[i] = static_cast<const f2 *>(a.vtab)[i];
    }
    // columns are patch-local (2 bytes a slot): l < pcnt is row pbase + l, else halo entry l - pcnt
    const int hb = a.halo_ptr[patch];
    const int hc = min(a.halo_ptr[patch + 1] - hb, PSPMM_HMAX);
    for (int i = threadIdx.x; i < hc; i += PSPMM_WG)
        hrow[i] = a.halo_rows[hb + i];
    HSet h0, h1;
    if (cnt > 0)
        load_h(0, h0);

    // phase 1: x of rows base .. base + cnt - 1, one contiguous span; every
    // load is issued before the first LDS write (lanes past the span reload
    // its last chunk and write nothing)
    if (cnt > 0) {
        constexpr int SPL = TROWS * RC / PSPMM_WG;
        static_assert(SPL * PSPMM_WG == TROWS * RC, "staged span is a whole number of loads per lane");
        const f4 *__restrict__ xsrc = xg + base * RC;
        const int span = cnt * RC;
        f4 stg[SPL];
#pragma unroll
        for (int k = 0; k < SPL; ++k)
            stg[k] = xsrc[min((int)threadIdx.x + k * PSPMM_WG, span - 1)];
#pragma unroll
        for (int k = 0; k < SPL; ++k) {
            const int i = threadIdx.x + k * PSPMM_WG;
            if (i < span)
                xs[i] = stg[k];
        }
    }
    __syncthreads();

    // phase 2: lane (rl, lr) owns chunks c0 .. c0 + NC - 1 of row base + r0 + rl
    double dre[NC][2] = {}, dim[NC][2] = {}, nrm[NC][2] = {};
    auto pass = [&](int r0, const HSet &hq, HSet &hn) {
        const int li = r0 + rl;
        const bool live = li < cnt;
        const int lic = live ? li : cnt - 1;
        const int64_t row = base + lic;
        const int64_t e = row * RC + c0;        // f4 index of the lane's first chunk
        __builtin_amdgcn_sched_barrier(0);      // keep the passes apart (register pressure)
        // loads without branches, so that the compiler counts them exactly and
        // waits for this pass's operands only (the last pass reloads its own H)
        load_h(r0 + ROWS, hn);
        f4 xo[NC] = {}, yo[NC] = {}, oo[NC] = {}, po[NC] = {}, qo[NC] = {};
        const f4 *__restrict__ src_o = cl ? psi : out;       // psi (Clenshaw) or out
        const f4 *__restrict__ src_y = use_y ? y : src_o;    // read but unused without y
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            if constexpr (KIND == K_FIRST || KIND == K_MOM0) {
                xo[j] = xs[lic * RC + c0 + j];
            } else if constexpr (KIND == K_MOM) {
                xo[j] = xs[lic * RC + c0 + j];
                yo[j] = ld_stream(y + e + j);
            } else {
                yo[j] = ld_stream(src_y + e + j);
                const f4 o = ld_stream(src_o + e + j);
                qo[j] = o;
                oo[j] = o;
                if constexpr (KIND == K_LAST)
                    po[j] = ld_stream(psi0 + e + j);
            }
        }
        f2 acc[NC][2] = {};
#pragma unroll
        for (int q = 0; q < W; ++q) {
            const uint32_t half = (q % 4) < 2 ? (uint32_t)hq.cw : (uint32_t)(hq.cw >> 32);
            const int cg = ((uint32_t)quad_bcast((int)half, q / 4) >> (16 * (q % 2))) & 0xFFFF;
            f2 vg;
            if constexpr (DICT) {
                const uint32_t k = ((uint32_t)quad_bcast((int)hq.w, q / 4) >> (8 * (q % 4))) & 255u;
                vg = k == 255u ? hq.d : vtab[k];
            } else {
                vg = f2{__int_as_float(quad_bcast(__float_as_int(hq.v[q / 4].x), q % 4)),
                        __int_as_float(quad_bcast(__float_as_int(hq.v[q / 4].y), q % 4))};
            }
            const int l = cg - sub * TROWS;         // row within the run, when in it
            const bool in = (unsigned)l < (unsigned)cnt;
#pragma unroll
            for (int j = 0; j < NC; ++j) {
                // LDS and global reads stay apart (a select of the two pointers
                // would make one flat load of every gather)
                const f4 xl = xs[(in ? l : 0) * RC + c0 + j];
                f4 xh = xl;
                if (!in) {
                    const int64_t g = cg < pcnt ? pbase + cg : (int64_t)hrow[cg - pcnt];
                    xh = xgl[g * RC + c0 + j];
                }
                const f4 xv = in ? xl : xh;
                cmac(acc[j][0], vg, lo2(xv));
                cmac(acc[j][1], vg, hi2(xv));
            }
        }
        if (live) {
#pragma unroll
            for (int j = 0; j < NC; ++j)
                spmm2_update<KIND>(up(acc[j][0]) * a.scale, up(acc[j][1]) * a.scale, xo[j], yo[j], oo[j], po[j], qo[j],
                                   ca, cb, cl, use_y, y + e + j, out + e + j, dre[j], dim[j], nrm[j]);
        }
    };
    for (int r0 = 0; r0 < cnt; r0 += 2 * ROWS) {
        pass(r0, h0, h1);
        if (r0 + ROWS < cnt)
            pass(r0 + ROWS, h1, h0);
    }
    if constexpr (DOTS) {
        // lanes with equal (lane mod LR) hold the same vectors: fold them
#pragma unroll
        for (int off = 32; off >= LR; off >>= 1) {
#pragma unroll
            for (int j = 0; j < NC; ++j)
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    dre[j][q] += __shfl_xor(dre[j][q], off, 64);
                    dim[j][q] += __shfl_xor(dim[j][q], off, 64);
                    nrm[j][q] += __shfl_xor(nrm[j][q], off, 64);
                }
        }
        __syncthreads();                         // xs is reused for the reduction
        double *red = reinterpret_cast<double *>(xs);    // [PSPMM_WG / 64][B][3]
        const int lane = threadIdx.x % 64;
        const int wave = threadIdx.x / 64;
        if (lane < LR) {
#pragma unroll
            for (int j = 0; j < NC; ++j)
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    double *r = red + ((size_t)wave * B + 2 * (c0 + j) + q) * 3;
                    r[0] = dre[j][q];
                    r[1] = dim[j][q];
                    r[2] = nrm[j][q];
                }
        }
        __syncthreads();
        if (threadIdx.x < B) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
            for (int w = 0; w < PSPMM_WG / 64; ++w) {
                const double *r = red + ((size_t)w * B + threadIdx.x) * 3;
                s0 += r[0];
                s1 += r[1];
                s2 += r[2];
            }
            double *p = a.partials + ((patch * NSUB + sub) * B + threadIdx.x) * 4;
            p[0] = s0;
            p[1] = s1;
            p[2] = s2;
            p[3] = 0.0;
        }
    }
}

template <int B, int W, bool DICT>
static hipError_t launch_patch_spmm_w(int kind, const TermArgs &a, hipStream_t st)
{
    const int64_t per = (a.npatch + NXCD - 1) / NXCD;
    const dim3 grid((unsigned)(per * pspmm_nsub(B) * NXCD));
    switch (kind) {
    case K_FIRST:
        hipLaunchKernelGGL((patch_spmm_kernel<B, K_FIRST, W, DICT>), grid, dim3(PSPMM_WG), 0, st, a);
        break;
    case K_MID:
        hipLaunchKernelGGL((patch_spmm_kernel<B, K_MID, W, DICT>), grid, dim3(PSPMM_WG), 0, st, a);
        break;
    case K_MOM0:
        hipLaunchKernelGGL((patch_spmm_kernel<B, K_MOM0, W, DICT>), grid, dim3(PSPMM_WG), 0, st, a);
        break;
    case K_MOM:
        hipLaunchKernelGGL((patch_spmm_kernel<B, K_MOM, W, DICT>), grid, dim3(PSPMM_WG), 0, st, a);
        break;
    default:
        hipLaunchKernelGGL((patch_spmm_kernel<B, K_LAST, W, DICT>), grid, dim3(PSPMM_WG), 0, st, a);
        break;
    }
    return hipGetLastError();
}

template <int B, bool DICT>
static hipError_t launch_patch_spmm_b(int kind, const TermArgs &a, hipStream_t st)
{
    switch (a.w) {
    case 3: return launch_patch_spmm_w<B, 3, DICT>(kind, a, st);
    case 4: return launch_patch_spmm_w<B, 4, DICT>(kind, a, st);
    case 5: return launch_patch_spmm_w<B, 5, DICT>(kind, a, st);
    case 8: return launch_patch_spmm_w<B, 8, DICT>(kind, a, st);
    case 12: return launch_patch_spmm_w<B, 12, DICT>(kind, a, st);
    default: return hipErrorInvalidValue;
    }
}

int staged_blocks(int B, int64_t npatch) { return (int)(npatch * pspmm_nsub(B)); }

bool staged_supported(int dtype, int B, int w, int patch_rows)
{
    return dtype == TBPM_C64 && (B == 8 || B == 16) && patch_rows <= PSPMM_ROWS &&
           (w == 3 || w == 4 || w == 5 || w == 8 || w == 12);
}

hipError_t launch_term(int kind, int dtype, int fmt, const TermArgs &a, const KernelShape &s, hipStream_t st)
{
    if (s.staged) {
        // partial sums per patch: s.grid is the patch count
        if (fmt != F_ELL || a.plist || !a.patch_ptr || !a.lcol || !a.halo_ptr || !a.halo_rows || a.npatch <= 0 ||
            s.grid != staged_blocks(s.B, a.npatch) || a.n <= 0 || !staged_supported(dtype, s.B, a.w, PSPMM_ROWS))
            return hipErrorInvalidValue;
        if (a.vidx && a.vtab)
            return s.B == 8 ? launch_patch_spmm_b<8, true>(kind, a, st) : launch_patch_spmm_b<16, true>(kind, a, st);
        return s.B == 8 ? launch_patch_spmm_b<8, false>(kind, a, st) : launch_patch_spmm_b<16, false>(kind, a, st);
    }
    if (s.grid % NXCD != 0 || s.grid <= 0 || a.n <= 0)
        return hipErrorInvalidValue;
    if (a.plist && (a.pcount <= 0 || !a.patch_ptr || a.patch_tiles * (int64_t)rows_per_tile(s) < 1))
        return hipErrorInvalidValue;
    if (dtype == TBPM_C128)
        return fmt == F_CSR ? launch_shape<d2, F_CSR>(kind, a, s, st) : launch_shape<d2, F_ELL>(kind, a, s, st);
    if (s.B > 1 && s.lr * 2 == s.B)
        return launch_spmm2(kind, fmt, a, s, st);
    return fmt == F_CSR ? launch_shape<f2, F_CSR>(kind, a, s, st) : launch_shape<f2, F_ELL>(kind, a, s, st);
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
//
// The Clenshaw modes run the same two phases on the backward recurrence
// b_m = c_m psi + scale H b_m+1 - b_m+2: phase A forms b_m (x = b_m+1,
// y = b_m+2) and phase B b_m-1, each adding its coefficient times psi, so the
// series needs no accumulator: per pair, reads of b_m+1, b_m+2 and psi and
// writes of b_m, b_m-1 instead of the forward pair's extra read and write of
// out.

template <typename T, int W, int NT, int R, int MODE, bool DICT>
__global__ __launch_bounds__(NT) void pair_kernel(PairArgs a)
{
    constexpr bool LAST = MODE == PAIR_LAST;
    constexpr bool MOM = MODE == PAIR_MOM;
    constexpr bool CLL = MODE == PAIR_CL_LAST;
    constexpr bool CLS = MODE == PAIR_CL_SINGLE;
    constexpr bool first = MODE == PAIR_CL_FIRST;        // xin = psi, no yin
    constexpr bool CL = MODE == PAIR_CL || CLL || CLS || first;   // Clenshaw: psi enters every phase, no out
    constexpr bool FST = MODE == PAIR_FIRST;             // terms 1 and 2 of a step: xin = psi, no yin, no out read
    constexpr bool CRS = MODE == PAIR_CROSS;             // the last term of a step and term 1 of the next
    constexpr bool DOTS = LAST || MOM || CLL || CRS;
    constexpr int NV = MOM ? 6 : 3;                 // partial sums per workgroup
    using E = Elem<T>;
    using A = typename E::acc;
    constexpr int S = NT * R;
    constexpr int HMAX = pair_halo_max(S);
    __shared__ T ylds[S + HMAX];
    __shared__ int32_t hidx[HMAX];
    __shared__ double red[NT / 64][NV];
    __shared__ T vtab[DICT ? 256 : 1];          // value table (DICT: H entries are one-byte indices)
    constexpr int NW = (W + 3) / 4;             // index words per row

    // one patch per workgroup; the patches of XCD (blockIdx % 8) are contiguous
    // (in the list order when only listed patches are processed)
    const int64_t np = a.plist ? a.pcount : a.npatch;
    const int64_t per = (np + NXCD - 1) / NXCD;
    const int64_t pidx = (int64_t)(blockIdx.x % NXCD) * per + blockIdx.x / NXCD;
    if (pidx >= np)
        return;                                     // uniform over the workgroup
    const int64_t patch = a.plist ? (int64_t)a.plist[pidx] : pidx;
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
    const uint64_t *__restrict__ lcol = a.lcol;
    const int64_t ld = a.ld;
    const double scale = a.scale;
    const T *__restrict__ psi = static_cast<const T *>(a.psi);
    const d2 ka = d2{a.ka_re, a.ka_im};
    const d2 c0 = d2{a.c0_re, a.c0_im};
    const d2 c1 = d2{a.c1_re, a.c1_im};
    const d2 c2 = d2{a.c2_re, a.c2_im};

    // the halo list maps local column indices >= cnt to rows
    for (int h = threadIdx.x; h < hc; h += NT)
        hidx[h] = a.halo_rows[hb + h];
    const T *__restrict__ vdiag = static_cast<const T *>(a.vdiag);
    if constexpr (DICT) {
        for (int i = threadIdx.x; i < 256; i += NT)
            vtab[i] = static_cast<const T *>(a.vtab)[i];
    }

    // phase A, patch rows: lane t owns rows t, t + NT, ...; H's columns are
    // patch-local (2 bytes a slot, four to a word): l < cnt is row base + l,
    // else halo entry l - cnt.
    // Values: v, or (DICT) index words vw (slot s in byte s % 4 of word s / 4)
    // into the table, index 255 taking the row's diagonal dg
    int c[R][W];
    T v[R][W];
    uint32_t vw[R][NW];
    T dg[R];
    T yo[R], xo[R], po[R], oo[R];
    d2 ym[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int li = threadIdx.x + r * NT;
        const int64_t row = base + (li < cnt ? li : cnt - 1);
        uint64_t cw[NW];
#pragma unroll
        for (int q = 0; q < NW; ++q)
            cw[q] = ld_stream(lcol + (int64_t)q * ld + row);
#pragma unroll
        for (int s = 0; s < W; ++s) {
            c[r][s] = (int)((cw[s / 4] >> (16 * (s % 4))) & 0xFFFFull);
            if constexpr (!DICT)
                v[r][s] = ld_stream(val + (int64_t)s * ld + row);
        }
        if constexpr (DICT) {
#pragma unroll
            for (int q = 0; q < NW; ++q)
                vw[r][q] = ld_stream(a.vidx + (int64_t)q * ld + row);
            dg[r] = diag_of(vdiag, a.vdiag_real, row);
        }
        yo[r] = (first || FST) ? T{} : ld_stream(yin + row);
        if constexpr (!CLS)
            xo[r] = xin[row];                       // x_{m-1} of the row, for phase B
        if constexpr (CRS)
            oo[r] = ld_stream(out + row);           // the step's accumulated series
        if constexpr (CL)
            po[r] = first ? xo[r] : ld_stream(psi + row);
    }
    __syncthreads();                                // hidx (and the value table) complete
    // the value of slot s of a patch row (after the barrier: the table is in LDS)
    auto hv = [&](int r, int s) -> T {
        if constexpr (DICT) {
            const uint32_t k = (vw[r][s / 4] >> (8 * (s % 4))) & 255u;
            return k == 255u ? dg[r] : vtab[k];
        } else {
            return v[r][s];
        }
    };
#pragma unroll
    for (int r = 0; r < R; ++r) {
        T xv[W];
#pragma unroll
        for (int s = 0; s < W; ++s) {
            const int l = c[r][s];
            xv[s] = xin[l < cnt ? base + l : (int64_t)hidx[l - cnt]];
        }
        A acc{0, 0};
#pragma unroll
        for (int s = 0; s < W; ++s)
            cmac(acc, (A)hv(r, s), (A)xv[s]);
        if constexpr (CL) {
            const d2 hx = E::acc_to_d(acc) * scale;
            ym[r] = (first ? cmul(ka, hx) : hx - E::to_d(yo[r])) + cmul(c0, E::to_d(po[r]));
        } else if constexpr (FST) {
            ym[r] = E::acc_to_d(acc) * scale;       // p_1 = (1/rho) H psi
        } else if constexpr (CRS) {
            // psi(t + dt) = out + c_{M-1} p_{M-1}, as stored (it starts the next step)
            ym[r] = E::to_d(E::from_d(E::to_d(oo[r]) + cmul(c0, E::acc_to_d(acc) * scale - E::to_d(yo[r]))));
        } else {
            ym[r] = E::acc_to_d(acc) * scale - E::to_d(yo[r]);
        }
        if constexpr (MOM)
            ym[r] = E::to_d(E::from_d(ym[r]));      // the stored value enters the inner products
        const int li = threadIdx.x + r * NT;
        if (li < cnt) {
            const T ys = E::from_d(ym[r]);
            if constexpr (!CLS)
                ylds[li] = ys;
            if constexpr (!CLL)                     // b_1 of a Clenshaw series stays on chip
                st_stream(ys, yout + base + li);
        }
    }
    if constexpr (CLS)
        return;                                     // one product: no halo, no second phase

    // phase A, halo rows (their H rows are stored contiguously per patch)
    const int32_t *__restrict__ hcol = a.hcol;
    const T *__restrict__ hval = static_cast<const T *>(a.hval);
    for (int h = threadIdx.x; h < hc; h += NT) {
        const int64_t rh = hidx[h];
        const int64_t g = (int64_t)hb + h;
        int32_t ch[W];
        T vh[W];
#pragma unroll
        for (int s = 0; s < W; ++s)
            ch[s] = ld_stream(hcol + (int64_t)s * a.ldh + g);
        if constexpr (DICT) {
            uint32_t hw[NW];
#pragma unroll
            for (int q = 0; q < NW; ++q)
                hw[q] = ld_stream(a.hvidx + (int64_t)q * a.ldh + g);
            const T dh = diag_of(vdiag, a.vdiag_real, rh);
#pragma unroll
            for (int s = 0; s < W; ++s) {
                const uint32_t k = (hw[s / 4] >> (8 * (s % 4))) & 255u;
                vh[s] = k == 255u ? dh : vtab[k];
            }
        } else {
#pragma unroll
            for (int s = 0; s < W; ++s)
                vh[s] = ld_stream(hval + (int64_t)s * a.ldh + g);
        }
        const T yh = (first || FST) ? T{} : yin[rh];
        T xv[W];
#pragma unroll
        for (int s = 0; s < W; ++s)
            xv[s] = xin[ch[s]];
        A acc{0, 0};
#pragma unroll
        for (int s = 0; s < W; ++s)
            cmac(acc, (A)vh[s], (A)xv[s]);
        if constexpr (CL) {
            const d2 hx = E::acc_to_d(acc) * scale;
            const d2 ph = E::to_d(first ? xin[rh] : psi[rh]);
            ylds[cnt + h] = E::from_d((first ? cmul(ka, hx) : hx - E::to_d(yh)) + cmul(c0, ph));
        } else if constexpr (FST) {
            ylds[cnt + h] = E::from_d(E::acc_to_d(acc) * scale);
        } else if constexpr (CRS) {
            ylds[cnt + h] = E::from_d(E::to_d(out[rh]) + cmul(c0, E::acc_to_d(acc) * scale - E::to_d(yh)));
        } else {
            ylds[cnt + h] = E::from_d(E::acc_to_d(acc) * scale - E::to_d(yh));
        }
    }
    __syncthreads();                                // y_m of patch and halo in LDS

    // phase B
    const double sb = (CL || FST || CRS) ? a.scale_b : scale;
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
            for (int s = 0; s < W; ++s)
                cmac(acc, (A)hv(r, s), (A)ylds[c[r][s]]);   // ylds: patch rows, then halo rows
            d2 xn;
            if constexpr (CL) {
                const d2 hy = E::acc_to_d(acc) * sb;
                const d2 xd = E::to_d(xo[r]);
                xn = (first ? hy - cmul(ka, xd) : hy - xd) + cmul(c1, E::to_d(po[r]));
            } else if constexpr (CRS) {
                xn = E::acc_to_d(acc) * sb;         // p_1 of the next step
            } else {
                xn = E::acc_to_d(acc) * sb - E::to_d(xo[r]);
            }
            const T xs = E::from_d(xn);
            st_stream(xs, xout + row);
            if constexpr (FST) {                    // out = c_0 psi + c_1 p_1 + c_2 p_2
                st_stream(E::from_d((cmul(c0, E::to_d(xo[r])) + cmul(c1, ym[r])) + cmul(c2, xn)), out + row);
                continue;
            }
            if constexpr (CRS) {                    // next step's out = c_0 psi + c_1 p_1; sums of psi
                st_stream(E::from_d(cmul(c1, ym[r]) + cmul(c2, xn)), static_cast<T *>(a.out2) + row);
                const d2 p = E::to_d(ld_stream(static_cast<const T *>(a.psi0) + row));
                const d2 o = ym[r];
                sum[0] += p.x * o.x + p.y * o.y;
                sum[1] += p.x * o.y - p.y * o.x;
                sum[2] += o.x * o.x + o.y * o.y;
                continue;
            }
            if constexpr (CL) {
                if constexpr (CLL) {                // O = psi(t + dt): <psi0|O>, <O|O>
                    const d2 p = E::to_d(ld_stream(static_cast<const T *>(a.psi0) + row));
                    const d2 o = E::to_d(xs);
                    sum[0] += p.x * o.x + p.y * o.y;
                    sum[1] += p.x * o.y - p.y * o.x;
                    sum[2] += o.x * o.x + o.y * o.y;
                }
                continue;
            }
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
    if constexpr (DOTS) {
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
template <typename T, int W, int R, bool DICT>
static hipError_t launch_pair_w(int mode, const PairArgs &a, hipStream_t st)
{
    const int g = pair_grid(a.plist ? a.pcount : a.npatch);
    constexpr int NT = R == 2 ? 1024 : 512;
    switch (mode) {
    case PAIR_LAST:
        hipLaunchKernelGGL((pair_kernel<T, W, NT, 2, PAIR_LAST, DICT>), dim3(g), dim3(NT), 0, st, a);
        break;
    case PAIR_MOM:
        hipLaunchKernelGGL((pair_kernel<T, W, NT, 2, PAIR_MOM, DICT>), dim3(g), dim3(NT), 0, st, a);
        break;
    case PAIR_CL:
        hipLaunchKernelGGL((pair_kernel<T, W, NT, 2, PAIR_CL, DICT>), dim3(g), dim3(NT), 0, st, a);
        break;
    case PAIR_CL_LAST:
        hipLaunchKernelGGL((pair_kernel<T, W, NT, 2, PAIR_CL_LAST, DICT>), dim3(g), dim3(NT), 0, st, a);
        break;
    case PAIR_CL_SINGLE:
        hipLaunchKernelGGL((pair_kernel<T, W, NT, 2, PAIR_CL_SINGLE, DICT>), dim3(g), dim3(NT), 0, st, a);
        break;
    case PAIR_CL_FIRST:
        hipLaunchKernelGGL((pair_kernel<T, W, NT, 2, PAIR_CL_FIRST, DICT>), dim3(g), dim3(NT), 0, st, a);
        break;
    case PAIR_FIRST:
        hipLaunchKernelGGL((pair_kernel<T, W, NT, 2, PAIR_FIRST, DICT>), dim3(g), dim3(NT), 0, st, a);
        break;
    case PAIR_CROSS:
        hipLaunchKernelGGL((pair_kernel<T, W, NT, 2, PAIR_CROSS, DICT>), dim3(g), dim3(NT), 0, st, a);
        break;
    default:
        hipLaunchKernelGGL((pair_kernel<T, W, NT, 2, PAIR_MID, DICT>), dim3(g), dim3(NT), 0, st, a);
        break;
    }
    return hipGetLastError();
}

template <typename T, int R, bool DICT>
static hipError_t launch_pair_r(int mode, const PairArgs &a, hipStream_t st)
{
    switch (a.w) {
    case 3: return launch_pair_w<T, 3, R, DICT>(mode, a, st);
    case 4: return launch_pair_w<T, 4, R, DICT>(mode, a, st);
    case 5: return launch_pair_w<T, 5, R, DICT>(mode, a, st);
    case 8: return launch_pair_w<T, 8, R, DICT>(mode, a, st);
    case 12: return launch_pair_w<T, 12, R, DICT>(mode, a, st);
    default: return hipErrorInvalidValue;
    }
}

// ---- complex64 blocks: two Chebyshev terms per pass over H --------------------------------
//
// The fused pair for blocks of B = 8 or 16 complex64 vectors on patch-reordered
// H (forward recurrence, MID and LAST).  One 1024-lane workgroup owns one
// patch and eight of the block's vectors (64 bytes of each row; for B = 16 the
// two halves of a patch are workgroups j and j + 8, on one XCD).  Four lanes
// share a row, each owning two vectors (one 16-byte chunk), so a wave reads
// whole 64-byte row segments; lane k of the four loads the row's column (and
// index) words k, k + 4, ... and the others take them by DPP.
//   phase A: x_{m-1} of the patch rows and of the halo rows is staged in LDS
//            (local row l: patch row l < cnt, else halo entry l - cnt);
//            y_m = scale H x_{m-1} - y_{m-2} for the halo rows (their H rows
//            carry global columns: those in the patch gather from LDS, the
//            others from L2) and for the patch rows (every gather from LDS),
//            into registers, the patch rows' also to yout;
//   phase B: after a barrier y_m replaces x_{m-1} in LDS; x_{m+1} = scale H
//            y_m - x_{m-1} gathers from LDS only, then out += c_m y_m +
//            c_{m+1} x_{m+1} (LAST: + per-vector partial sums <psi0|out>,
//            <out|out>, at partials[patch][b][4]).
// Per pair and row this moves H once (plus the halo rows' H) and six vector
// passes, against ten for two single terms.  LDS holds 1024 + 1280 rows of 64
// bytes (one workgroup per CU, 16 waves): the library takes this kernel only
// for patches of at most 1024 rows whose halos have at most 1280 rows
// (bpair_supported, launch_pair).  Eight vectors a workgroup rather than four:
// with four, each wave used a quarter (B = 16) or half (B = 8) of every line it
// touched and the L2-to-CU traffic set the pace (bilayer pair 3.96 against
// 3.20 ms).
// Arithmetic: products and row sums in FP32, the recurrence and coefficient
// updates in FP64, one rounding per stored value (as spmm2_update).

constexpr int BP_ROWS = 1024;              // largest patch
constexpr int BP_HMAX = 1280;              // largest halo
constexpr int BP_PASS = 256;               // rows per pass
constexpr int BP_NP = BP_ROWS / BP_PASS;   // passes over the patch rows
constexpr int BP_VG = 8;                   // vectors per workgroup (B = 16: two workgroups a patch)

// value of lane k (0 or 1) of each pair of lanes (DPP quad_perm [k, k, k+2, k+2]);
// k is a constant once the caller's loop is unrolled
__device__ __forceinline__ int pair_bcast(int v, int k)
{
    return k == 0 ? __builtin_amdgcn_update_dpp(0, v, 0xA0, 0xF, 0xF, false)
                  : __builtin_amdgcn_update_dpp(0, v, 0xF5, 0xF, 0xF, false);
}
// value of lane k of each group of LR (2 or 4) lanes
template <int LR>
__device__ __forceinline__ int group_bcast(int v, int k)
{
    if constexpr (LR == 2)
        return pair_bcast(v, k);
    else
        return quad_bcast(v, k);
}

// The two workgroups of a patch of a 16-vector block read and write disjoint
// halves of the same lines (and read the same H): ordinary loads and stores,
// so that the lines stay in L2 for the other instead of streaming past it
template <typename T>
__device__ __forceinline__ T ld_shared(const T *p)
{
    return *p;
}
template <typename T>
__device__ __forceinline__ void st_shared(T v, T *p)
{
    *p = v;
}

template <int W, bool DICT, int LR>
struct BpRow {                             // a lane's share of one patch row of H
    static constexpr int WQ = (W + 3) / 4;         // column (and index) words of a row
    static constexpr int WL = (WQ + LR - 1) / LR;  // words per lane
    static constexpr int VL = (W + LR - 1) / LR;   // values per lane (without a table)
    uint64_t cw[WL];                               // column words lr, lr + LR, ...
    uint32_t vw[DICT ? WL : 1];                    // index words lr, lr + LR, ...
    f2 v[DICT ? 1 : VL];                           // values of slots lr, lr + LR, ...
    f2 d;                                          // the row's diagonal (index 255)
};

template <int B, int W, int MODE, bool DICT>
__global__ __launch_bounds__(BP_PASS * BP_VG / 2) __attribute__((amdgpu_waves_per_eu(4))) void bpair_kernel(PairArgs a)
{
    constexpr bool LAST = MODE == PAIR_LAST;
    constexpr int LR = BP_VG / 2;          // lanes per row (two vectors each)
    constexpr int NT = BP_PASS * LR;       // lanes per workgroup
    constexpr int GR = B / BP_VG;          // vector groups per patch
    constexpr int RC = B / 2;              // 16-byte chunks per row
    constexpr int HP = (BP_HMAX + BP_PASS - 1) / BP_PASS;   // passes over the halo rows
    using H = BpRow<W, DICT, LR>;
    constexpr int WQ = H::WQ, WL = H::WL, VL = H::VL;
    // [local row][2]: rows 0 .. cnt-1 the patch, cnt .. cnt+hc-1 its halo; x_{m-1}, then y_m
    __shared__ f4 ys[(BP_ROWS + BP_HMAX) * LR];
    __shared__ f2 vtab[DICT ? 256 : 1];
    __shared__ double red[LAST ? NT / 64 : 1][BP_VG][3];

    const int64_t per = (a.npatch + NXCD - 1) / NXCD;
    const int64_t u = blockIdx.x / NXCD;
    const int64_t patch = (int64_t)(blockIdx.x % NXCD) * per + u / GR;
    const int g = (int)(u % GR);
    if (patch >= a.npatch)
        return;                                    // uniform over the workgroup
    const int64_t pbase = a.patch_ptr[patch];
    const int cnt = min(a.patch_ptr[patch + 1] - (int)pbase, BP_ROWS);
    const int hb = a.halo_ptr[patch];
    const int hc = min(a.halo_ptr[patch + 1] - hb, BP_HMAX);
    if (cnt <= 0)
        return;
    const int lr = threadIdx.x % LR;
    const int rl = threadIdx.x / LR;
    const int ch = LR * g + lr;                    // the lane's chunk of a row (vectors 2ch, 2ch + 1)
    const f4 *__restrict__ xin = static_cast<const f4 *>(a.xin);
    const f4 *__restrict__ yin = static_cast<const f4 *>(a.yin);
    f4 *__restrict__ yout = static_cast<f4 *>(a.yout);
    f4 *__restrict__ xout = static_cast<f4 *>(a.xout);
    f4 *__restrict__ out = static_cast<f4 *>(a.out);
    const f2 *__restrict__ val = static_cast<const f2 *>(a.val);
    const f2 *__restrict__ vdiag = static_cast<const f2 *>(a.vdiag);
    const int64_t ld = a.ld;
    const double scale = a.scale;
    const d2 c0 = d2{a.c0_re, a.c0_im};
    const d2 c1 = d2{a.c1_re, a.c1_im};

    auto load_row = [&](int p, H &h) {
        const int64_t row = pbase + min(p * BP_PASS + rl, cnt - 1);
        // loads without branches: a lane past the row's last word reloads it
#pragma unroll
        for (int k = 0; k < WL; ++k) {
            const int q = min(lr + LR * k, WQ - 1);
            h.cw[k] = ld_shared(a.lcol + (int64_t)q * ld + row);
            if constexpr (DICT)
                h.vw[k] = ld_shared(a.vidx + (int64_t)q * ld + row);
        }
        if constexpr (DICT) {
            h.d = diag_of<f2, false>(vdiag, a.vdiag_real, row);
        } else {
#pragma unroll
            for (int k = 0; k < VL; ++k)
                h.v[k] = ld_shared(val + (int64_t)min(lr + LR * k, W - 1) * ld + row);
        }
    };
    // slot s of a row: its local column (< cnt: patch row, else cnt + halo position) and value
    auto col_of = [&](const H &h, int s) -> int {
        const int q = s / 4;
        const uint32_t half = (s % 4) < 2 ? (uint32_t)h.cw[q / LR] : (uint32_t)(h.cw[q / LR] >> 32);
        return (int)(((uint32_t)group_bcast<LR>((int)half, q % LR) >> (16 * (s % 2))) & 0xFFFFu);
    };
    auto val_of = [&](const H &h, int s) -> f2 {
        if constexpr (DICT) {
            const int q = s / 4;
            const uint32_t k = ((uint32_t)group_bcast<LR>((int)h.vw[q / LR], q % LR) >> (8 * (s % 4))) & 255u;
            return k == 255u ? h.d : vtab[k];
        } else {
            return f2{__int_as_float(group_bcast<LR>(__float_as_int(h.v[s / LR].x), s % LR)),
                      __int_as_float(group_bcast<LR>(__float_as_int(h.v[s / LR].y), s % LR))};
        }
    };
    // a halo row of the lane (halo pass q): its H row (stored per patch with
    // global columns), y_{m-2} and diagonal
    struct HaloRow {
        int32_t c[W];
        uint32_t w[DICT ? WQ : 1];
        f2 v[DICT ? 1 : W];
        f2 d;
        f4 yo;
    };
    auto halo_load = [&](int q, int64_t rh, HaloRow &hr) {
        const int64_t gi = (int64_t)hb + min(q * BP_PASS + rl, hc - 1);
#pragma unroll
        for (int s = 0; s < W; ++s)
            hr.c[s] = ld_shared(a.hcol + (int64_t)s * a.ldh + gi);
        if constexpr (DICT) {
#pragma unroll
            for (int k = 0; k < WQ; ++k)
                hr.w[k] = ld_shared(a.hvidx + (int64_t)k * a.ldh + gi);
            hr.d = diag_of<f2, false>(vdiag, a.vdiag_real, rh);
        } else {
#pragma unroll
            for (int s = 0; s < W; ++s)
                hr.v[s] = ld_shared(static_cast<const f2 *>(a.hval) + (int64_t)s * a.ldh + gi);
        }
        hr.yo = ld_shared(yin + rh * RC + ch);
    };

    if constexpr (DICT) {
        for (int i = threadIdx.x; i < 256; i += NT)
            vtab[i] = static_cast<const f2 *>(a.vtab)[i];
    }
    // the lane's halo row of halo pass q (row q * BP_PASS + rl of the halo); a
    // patch without a halo uses its first row in its place (nothing is stored)
    auto halo_row = [&](int q) -> int64_t {
        return hc > 0 ? (int64_t)a.halo_rows[hb + min(q * BP_PASS + rl, hc - 1)] : pbase;
    };
    const int64_t rh0 = halo_row(0);
    // x_{m-1} of the patch rows and of the halo rows into LDS; y_{m-2} of the
    // lane's patch rows, and the first halo pass's H rows, into registers
    f4 yo[BP_NP];
    HaloRow h0;
    {
        f4 stg[BP_NP];
#pragma unroll
        for (int p = 0; p < BP_NP; ++p)
            stg[p] = xin[(pbase + min(p * BP_PASS + rl, cnt - 1)) * RC + ch];
#pragma unroll
        for (int p = 0; p < BP_NP; ++p)
            yo[p] = ld_shared(yin + (pbase + min(p * BP_PASS + rl, cnt - 1)) * RC + ch);
        // lanes past the halo load nothing for it (waves past it skip the halo pass)
        f4 hx0 = f4{0.f, 0.f, 0.f, 0.f};
        if (rl < hc) {
            hx0 = xin[rh0 * RC + ch];
            halo_load(0, rh0, h0);
        }
#pragma unroll
        for (int p = 0; p < BP_NP; ++p) {
            const int li = p * BP_PASS + rl;
            if (li < cnt)
                ys[li * LR + lr] = stg[p];
        }
        if (rl < hc)
            ys[(cnt + rl) * LR + lr] = hx0;
#pragma unroll
        for (int q = 1; q < HP; ++q) {
            if (q * BP_PASS >= hc)
                break;                             // uniform
            const int h = q * BP_PASS + rl;
            if (h < hc)
                ys[(cnt + h) * LR + lr] = xin[halo_row(q) * RC + ch];
        }
    }
    __syncthreads();                               // x of patch and halo rows staged, table complete

    // phase A, halo rows: y_m into registers (columns in the patch from LDS, others from L2)
    f4 yh[HP];
#pragma unroll
    for (int q = 0; q < HP; ++q) {
        yh[q] = f4{0.f, 0.f, 0.f, 0.f};
        if (q * BP_PASS >= hc)
            break;                                 // uniform
        __builtin_amdgcn_sched_barrier(0);
        if (q * BP_PASS + rl >= hc)
            continue;                              // past the halo (whole waves skip)
        if (q > 0)
            halo_load(q, halo_row(q), h0);         // later passes reuse the first pass's registers
        const HaloRow &hr = h0;
        f2 acc0 = {0.f, 0.f}, acc1 = {0.f, 0.f};
#pragma unroll
        for (int s = 0; s < W; ++s) {
            const int64_t l = (int64_t)hr.c[s] - pbase;
            f4 xv;
            if ((uint64_t)l < (uint64_t)cnt)
                xv = ys[(int)l * LR + lr];
            else
                xv = xin[(int64_t)hr.c[s] * RC + ch];
            f2 v;
            if constexpr (DICT) {
                const uint32_t k = (hr.w[s / 4] >> (8 * (s % 4))) & 255u;
                v = k == 255u ? hr.d : vtab[k];
            } else {
                v = hr.v[s];
            }
            cmac(acc0, v, lo2(xv));
            cmac(acc1, v, hi2(xv));
        }
        const d2 y0 = up(acc0) * scale - up(lo2(hr.yo));
        const d2 y1 = up(acc1) * scale - up(hi2(hr.yo));
        yh[q] = join2(down(y0), down(y1));
    }

    // phase A, patch rows: every gather from LDS
    f4 yk[BP_NP];
#pragma unroll
    for (int p = 0; p < BP_NP; ++p) {
        yk[p] = f4{0.f, 0.f, 0.f, 0.f};
        if (p * BP_PASS >= cnt)
            break;                                 // uniform
        __builtin_amdgcn_sched_barrier(0);         // keep the passes apart (register pressure)
        const int li = p * BP_PASS + rl;
        const int64_t e = (pbase + min(li, cnt - 1)) * RC + ch;
        H hq;                                      // (loaded again in phase B: registers)
        load_row(p, hq);
        f2 acc0 = {0.f, 0.f}, acc1 = {0.f, 0.f};
#pragma unroll
        for (int s = 0; s < W; ++s) {
            const f2 v = val_of(hq, s);
            const f4 xv = ys[col_of(hq, s) * LR + lr];
            cmac(acc0, v, lo2(xv));
            cmac(acc1, v, hi2(xv));
        }
        const d2 y0 = up(acc0) * scale - up(lo2(yo[p]));
        const d2 y1 = up(acc1) * scale - up(hi2(yo[p]));
        yk[p] = join2(down(y0), down(y1));
        if (li < cnt)
            st_shared(yk[p], yout + e);
    }
    // out of the lane's rows, for phase B (loaded while the barriers wait)
    f4 oo[BP_NP];
#pragma unroll
    for (int p = 0; p < BP_NP; ++p)
        oo[p] = ld_shared(out + (pbase + min(p * BP_PASS + rl, cnt - 1)) * RC + ch);
    __syncthreads();                               // every gather of the staged x done
    // y_m takes the place of x_{m-1}; the lane's own x_{m-1} stays for phase B
    f4 xk[BP_NP];
#pragma unroll
    for (int p = 0; p < BP_NP; ++p) {
        const int li = p * BP_PASS + rl;
        xk[p] = ys[min(li, cnt - 1) * LR + lr];
        if (li < cnt)
            ys[li * LR + lr] = yk[p];
    }
#pragma unroll
    for (int q = 0; q < HP; ++q) {
        const int h = q * BP_PASS + rl;
        if (h < hc)
            ys[(cnt + h) * LR + lr] = yh[q];
    }
    __syncthreads();                               // y_m of patch and halo rows in LDS

    // phase B: every gather from LDS
    double dre[2] = {0.0, 0.0}, dim[2] = {0.0, 0.0}, nrm[2] = {0.0, 0.0};
#pragma unroll
    for (int p = 0; p < BP_NP; ++p) {
        if (p * BP_PASS >= cnt)
            break;                                 // uniform
        __builtin_amdgcn_sched_barrier(0);         // keep the passes apart (register pressure)
        const int li = p * BP_PASS + rl;
        const int64_t e = (pbase + min(li, cnt - 1)) * RC + ch;
        H hq;
        load_row(p, hq);
        f2 acc0 = {0.f, 0.f}, acc1 = {0.f, 0.f};
#pragma unroll
        for (int s = 0; s < W; ++s) {
            const f2 v = val_of(hq, s);
            const f4 yv = ys[col_of(hq, s) * LR + lr];
            cmac(acc0, v, lo2(yv));
            cmac(acc1, v, hi2(yv));
        }
        const d2 xn0 = up(acc0) * a.scale_b - up(lo2(xk[p]));
        const d2 xn1 = up(acc1) * a.scale_b - up(hi2(xk[p]));
        const f2 os0 = down((up(lo2(oo[p])) + cmul(c0, up(lo2(yk[p])))) + cmul(c1, xn0));
        const f2 os1 = down((up(hi2(oo[p])) + cmul(c0, up(hi2(yk[p])))) + cmul(c1, xn1));
        if (li < cnt) {
            st_shared(join2(down(xn0), down(xn1)), xout + e);
            st_shared(join2(os0, os1), out + e);
            if constexpr (LAST) {
                const f4 pv = ld_shared(static_cast<const f4 *>(a.psi0) + e);
                const f2 ps[2] = {lo2(pv), hi2(pv)};
                const f2 os[2] = {os0, os1};
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const d2 pd = up(ps[q]), od = up(os[q]);
                    dre[q] += pd.x * od.x + pd.y * od.y;
                    dim[q] += pd.x * od.y - pd.y * od.x;
                    nrm[q] += od.x * od.x + od.y * od.y;
                }
            }
        }
    }
    if constexpr (LAST) {
        // lanes with equal lr hold the same vectors: fold them, then the waves in order
#pragma unroll
        for (int off = 32; off >= LR; off >>= 1) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                dre[q] += __shfl_xor(dre[q], off, 64);
                dim[q] += __shfl_xor(dim[q], off, 64);
                nrm[q] += __shfl_xor(nrm[q], off, 64);
            }
        }
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
        if (threadIdx.x < BP_VG) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
            for (int w = 0; w < NT / 64; ++w) {
                s0 += red[w][threadIdx.x][0];
                s1 += red[w][threadIdx.x][1];
                s2 += red[w][threadIdx.x][2];
            }
            double *pp = a.partials + (patch * B + BP_VG * g + threadIdx.x) * 4;
            pp[0] = s0;
            pp[1] = s1;
            pp[2] = s2;
            pp[3] = 0.0;
        }
    }
}

template <int B, int W, bool DICT>
static hipError_t launch_bpair_w(int mode, const PairArgs &a, hipStream_t st)
{
    const int64_t per = (a.npatch + NXCD - 1) / NXCD;
    const dim3 grid((unsigned)(per * (B / BP_VG) * NXCD));
    const dim3 block(BP_PASS * BP_VG / 2);
    if (mode == PAIR_LAST)
        hipLaunchKernelGGL((bpair_kernel<B, W, PAIR_LAST, DICT>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((bpair_kernel<B, W, PAIR_MID, DICT>), grid, block, 0, st, a);
    return hipGetLastError();
}

template <int B, bool DICT>
static hipError_t launch_bpair_b(int mode, const PairArgs &a, hipStream_t st)
{
    switch (a.w) {
    case 3: return launch_bpair_w<B, 3, DICT>(mode, a, st);
    case 4: return launch_bpair_w<B, 4, DICT>(mode, a, st);
    case 5: return launch_bpair_w<B, 5, DICT>(mode, a, st);
    case 8: return launch_bpair_w<B, 8, DICT>(mode, a, st);
    default: return hipErrorInvalidValue;
    }
}

bool bpair_supported(int dtype, int B, int w, int patch_rows, int max_halo)
{
    // rows of 12 slots spill registers (the staged single terms are faster there)
    return dtype == TBPM_C64 && (B == 8 || B == 16) && patch_rows <= BP_ROWS && max_halo <= BP_HMAX &&
           (w == 3 || w == 4 || w == 5 || w == 8);
}

static hipError_t launch_bpair(int mode, int dtype, const PairArgs &a, int patch_rows, hipStream_t st)
{
    if (!bpair_supported(dtype, a.B, a.w, patch_rows, a.max_halo) || (mode != PAIR_MID && mode != PAIR_LAST) ||
        a.plist || !a.hcol || (mode == PAIR_LAST && (!a.psi0 || !a.partials)))
        return hipErrorInvalidValue;
    const bool dict = a.vidx && a.hvidx && a.vtab;
    if (a.B == 8)
        return dict ? launch_bpair_b<8, true>(mode, a, st) : launch_bpair_b<8, false>(mode, a, st);
    return dict ? launch_bpair_b<16, true>(mode, a, st) : launch_bpair_b<16, false>(mode, a, st);
}

hipError_t launch_pair(int mode, int dtype, const PairArgs &a, int patch_rows, hipStream_t st)
{
    if (a.B > 1)
        return launch_bpair(mode, dtype, a, patch_rows, st);
    if (!pair_supported(a.w, patch_rows) || !a.lcol || a.npatch <= 0 || mode < PAIR_MID || mode > PAIR_CROSS ||
        (mode == PAIR_CROSS && (!a.out2 || !a.partials || !a.psi0)) ||
        (mode == PAIR_MOM && !a.partials2) || (a.plist && (a.pcount <= 0 || a.pcount > a.npatch)))
        return hipErrorInvalidValue;
    const bool cl = mode >= PAIR_CL && mode <= PAIR_CL_FIRST;
    if (cl && (!a.psi || (mode == PAIR_CL_LAST && (!a.psi0 || !a.partials))))
        return hipErrorInvalidValue;
    const int R = patch_rows / PAIR_WG;
    // the value table serves 1024-row patches; 2048-row patches read the values
    const bool dict = a.vidx && a.hvidx && a.vtab && R == 1;
    if (dtype == TBPM_C128) {
        if (R == 2)
            return launch_pair_r<d2, 2, false>(mode, a, st);
        return dict ? launch_pair_r<d2, 1, true>(mode, a, st) : launch_pair_r<d2, 1, false>(mode, a, st);
    }
    if (R == 2)
        return launch_pair_r<f2, 2, false>(mode, a, st);
    return dict ? launch_pair_r<f2, 1, true>(mode, a, st) : launch_pair_r<f2, 1, false>(mode, a, st);
}

}  // namespace tbpm
