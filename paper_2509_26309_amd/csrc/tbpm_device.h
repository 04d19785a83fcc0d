// Device helpers shared by the HIP sources of the library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

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

// Tiles of XCD (blockIdx % 8) form one contiguous slab that the XCD sweeps
// front to back.  Within it, block j of that XCD takes runs of `run`
// consecutive tiles: run j, run j + nbx, ...; run is the block's share of the
// slab, at most WALK_RUN (so every block has work).  A run keeps one
// workgroup's neighbour gathers close to the rows it has just loaded (on the
// 12-entry honeycomb SpMM, runs of 16 cut the time of a term by 4% against
// single tiles).  Loop: for (r = t; r < end; r += stride) tiles
// r .. min(r + run, end) - 1.
constexpr int64_t WALK_RUN = 16;
struct TileWalk {
    int64_t t, end, stride, run;
};
__device__ __forceinline__ TileWalk tile_walk(int64_t ntiles)
{
    const int64_t xcd = blockIdx.x % NXCD;
    const int64_t j = blockIdx.x / NXCD;
    const int64_t nbx = gridDim.x / NXCD;
    const int64_t lo = ntiles * xcd / NXCD;
    const int64_t hi = ntiles * (xcd + 1) / NXCD;
    int64_t run = (hi - lo) / nbx;
    run = run < 1 ? 1 : (run > WALK_RUN ? WALK_RUN : run);
    return TileWalk{lo + j * run, hi, nbx * run, run};
}

template <typename T>
__device__ __forceinline__ void st_stream(T v, T *p)
{
    __builtin_nontemporal_store(v, p);
}

// grid of a grid-stride elementwise kernel over `total` items
inline int elem_grid(int64_t total)
{
    int64_t g = (total + WG - 1) / WG;
    if (g > 65536)
        g = 65536;
    if (g < 1)
        g = 1;
    return (int)g;
}

}  // namespace tbpm
