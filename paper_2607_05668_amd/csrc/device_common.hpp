// Device helpers shared by the kernel translation units: storage
// conversions, the XCD-aware tile order, periodic neighbour indices, cell
// coordinates and block reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "impl.hpp"
#include "lattices.hpp"

// ----------------------------------------------------------- storage ----
template <class St> struct Store;
// ld/st convert between the stored type and the arithmetic type R; st_init
// rounds a double once to the stored type (round to nearest even).  A
// non-temporal store (NT) streams past the caches: it pays when the two
// population buffers do not fit the last-level (Infinity) cache, and costs
// when they do, since the next step would have read them from there.
template <bool NT, class T>
__device__ inline void st_pop(T *p, T v)
{
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

template <> struct Store<double> {
    using R = double;
    __device__ static double ld(const double *p) { return *p; }
    template <bool NT> __device__ static void st(double *p, double v) { st_pop<NT>(p, v); }
    __device__ static void st_init(double *p, double v) { *p = v; }
};
template <> struct Store<float> {
    using R = float;
    __device__ static float ld(const float *p) { return *p; }
    template <bool NT> __device__ static void st(float *p, float v) { st_pop<NT>(p, v); }
    __device__ static void st_init(float *p, double v) { *p = (float)v; }
};
template <> struct Store<_Float16> {
    using R = float;
    __device__ static float ld(const _Float16 *p) { return (float)*p; }
    template <bool NT> __device__ static void st(_Float16 *p, float v) { st_pop<NT>(p, (_Float16)v); }
    __device__ static void st_init(_Float16 *p, double v) { *p = (_Float16)v; }
};

// ------------------------------------------------------------ helpers ----
// Workgroup -> tile order.  Workgroups are dealt round-robin to the eight
// XCDs (bid % 8); renumbering gives each XCD a contiguous run of tiles, so
// the rows a stencil shares stay in that XCD's L2.
__device__ inline long long xcd_tile(unsigned bid, unsigned nb)
{
    if constexpr (!LBM_XCD_REMAP) return bid;
    const unsigned q = nb >> 3, r = nb & 7u;
    const unsigned x = bid & 7u, loc = bid >> 3;
    return (long long)x * q + (x < r ? x : r) + loc;
}

__device__ inline int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Linear indices of the periodic neighbours x + sign c_i, in the index type
// I (32-bit when the grid allows it).
template <class Lat, class I>
__device__ inline void neighbours(int x, int y, int z, int nx, int ny, int nz, int sign, I *idx)
{
#pragma unroll
    for (int i = 0; i < Lat::Q; ++i) {
        const int xs = wrapi(x + sign * Lat::cx[i], nx);
        const int ys = wrapi(y + sign * Lat::cy[i], ny);
        const int zs = Lat::D == 3 ? wrapi(z + sign * Lat::cz[i], nz) : 0;
        idx[i] = ((I)zs * (I)ny + (I)ys) * (I)nx + (I)xs;
    }
}

template <class I>
__device__ inline void cell_coords(I cell, int nx, int ny, int &x, int &y, int &z)
{
    const I row = cell / (I)nx;
    x = (int)(cell - row * (I)nx);
    z = (int)(row / (I)ny);
    y = (int)(row - (I)z * (I)ny);
}

// ------------------------------------------------------- addressing ----
// Population layout [nz][tiles][K][Q][kTile] (impl.hpp): the cells of a
// z-slab (P = nx ny, in-plane index yx = y nx + x) are cut into tiles of
// kTile, the slab padded to whole tiles.  Element offset inside a slab of
// population (k, i) of in-plane index yx:
template <int K, int Q, class I>
__device__ inline I tile_offset(I yx)
{
    return (yx / (I)kTile) * (I)(K * Q * kTile) + (yx % (I)kTile);
}
// and in the whole buffer, for cell c = z P + yx:
template <int K, int Q>
__device__ inline size_t pop_at(int k, int i, long long c, long long P)
{
    const long long z = c / P;
    const long long Pp = (P + kTile - 1) / kTile * kTile;
    return (size_t)z * K * Q * (size_t)Pp + (size_t)tile_offset<K, Q>(c - z * P) + (size_t)(k * Q + i) * kTile;
}

// A thread reaches population (k, i) of a cell through the wave-uniform
// base of its z-slab shifted by (k Q + i) kTile elements (kept in scalar
// registers) plus a per-lane byte offset inside the slab.  When a slab is
// below 4 GiB the offsets and the index arithmetic are 32-bit and every
// access takes the scalar-base + vector-offset form, with no 64-bit address
// arithmetic per load or store; larger slabs use 64-bit offsets.
template <bool O32> struct Index { using T = unsigned long long; };
template <> struct Index<true> { using T = unsigned; };

inline bool fits_o32(long long C, int Q, size_t elem) { return (unsigned long long)C * Q * elem <= 0xffffffffull; }

template <class T, class I>
__device__ inline T *byte_at(T *base, I off) { return (T *)((char *)base + off); }
template <class T, class I>
__device__ inline const T *byte_at(const T *base, I off) { return (const T *)((const char *)base + off); }

// wavefront-shuffle block reductions (kBlock threads)
template <class R>
__device__ inline R block_reduce_max(R v, R *sh)
{
    for (int o = 32; o > 0; o >>= 1) {
        const R w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    R r = sh[0];
    for (int j = 1; j < kBlock / 64; ++j) r = sh[j] > r ? sh[j] : r;
    __syncthreads();
    return r;
}

template <class R>
__device__ inline R block_reduce_sum(R v, R *sh)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    R r = sh[0];
    for (int j = 1; j < kBlock / 64; ++j) r += sh[j];
    __syncthreads();
    return r;
}

