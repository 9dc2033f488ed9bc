// Helpers shared by the window kernels (interpolation, spreading, gradient).
#pragma once

#include "launch.hpp"

namespace nfft {

namespace window {

template <typename T, int D> __device__ __forceinline__ void bin_coords(const Geom &g, int bin, int *bc)
{
    int r = bin;
#pragma unroll
    for (int t = D - 1; t >= 0; --t) {
        bc[t] = r % g.nb[t];
        r /= g.nb[t];
    }
}

// One complex entry of an LDS tile.  Single-precision entries are read with relaxed
// 64-bit atomic loads: as ordered memory operations they are not fused into ds_read2_b64
// pairs, which on gfx950 take about twice the LDS cycles of two ds_read_b64 for the
// scattered stencil rows of the window kernels.  No wait is attached to a relaxed load.
template <typename T> __device__ __forceinline__ Cplx<T> lds_entry(const Cplx<T> *p)
{
    if constexpr (sizeof(T) == 4) {
        const unsigned long long u = __hip_atomic_load(
            reinterpret_cast<unsigned long long *>(const_cast<Cplx<T> *>(p)), __ATOMIC_RELAXED,
            __HIP_MEMORY_SCOPE_WORKGROUP);
        return __builtin_bit_cast(Cplx<T>, u);
    } else {
        return *p;
    }
}

// Grid index of entry idx of the padded tile of bin bc (row-major P_0 x ... x P_{d-1}):
// origin b B - m per dimension, indices mod n (a mask when every n_t is a power of two, P2,
// else a remainder; a tile may wrap more than once when it is longer than the grid).
template <int D, bool P2> struct TileMap {
    int o[kMaxDim];
    __device__ __forceinline__ TileMap(const Geom &g, const int *bc)
    {
#pragma unroll
        for (int t = 0; t < D; ++t)
            o[t] = (bc[t] << g.lgB[t]) - g.m + g.n[t];  // + n keeps it non-negative
    }
    __device__ __forceinline__ int wrap(const Geom &g, int i, int t) const
    {
        return P2 ? (i & (g.n[t] - 1)) : i % g.n[t];
    }
    // the same index in 32 bits, for grids of fewer than 2^32 cells
    __device__ __forceinline__ uint32_t src32(const Geom &g, int idx) const
    {
        const int P12 = g.P[1] * g.P[2];
        const int i0 = idx / P12;
        const int rem = idx - i0 * P12;
        const int i1 = rem / g.P[2];
        const int i2 = rem - i1 * g.P[2];
        const uint32_t r0 = (uint32_t)wrap(g, o[0] + i0, 0);
        const uint32_t r1 = (uint32_t)wrap(g, o[1] + i1, 1);
        return (r0 * (uint32_t)g.n[1] + r1) * (uint32_t)g.n[2] + (uint32_t)wrap(g, o[2] + i2, 2);
    }
    __device__ __forceinline__ int64_t src(const Geom &g, int idx) const
    {
        if constexpr (D == 1) {
            return wrap(g, o[0] + idx, 0);
        } else if constexpr (D == 2) {
            const int i0 = idx / g.P[1];
            const int i1 = idx - i0 * g.P[1];
            const int64_t r0 = wrap(g, o[0] + i0, 0);
            return r0 * g.n[1] + wrap(g, o[1] + i1, 1);
        } else {
            const int P12 = g.P[1] * g.P[2];
            const int i0 = idx / P12;
            const int rem = idx - i0 * P12;
            const int i1 = rem / g.P[2];
            const int i2 = rem - i1 * g.P[2];
            const int64_t r0 = wrap(g, o[0] + i0, 0);
            const int64_t r1 = wrap(g, o[1] + i1, 1);
            return (r0 * g.n[1] + r1) * g.n[2] + wrap(g, o[2] + i2, 2);
        }
    }
};

// Stage the padded tile of bin `bc` into LDS (complex, row-major P_0 x ... x P_{d-1}).
// A thread takes tile entries idx = base + threadIdx.x + k kBlock, k < K: all K loads
// (entries past the tile read entry 0) are issued before the first LDS store, so their
// latencies overlap.  K = 12 for complex64 covers a 2-D tile of up to 3072 entries (m = 8
// and 32 x 32 bins: 49 x 49) in one round of loads.
template <typename T, int D, bool P2>
__device__ __forceinline__ void stage_tile_w(const Geom &g, const int *bc, const Cplx<T> *grid, Cplx<T> *tile)
{
    using C = Cplx<T>;
    constexpr int K = sizeof(T) == 4 ? 12 : 8;
    const TileMap<D, P2> map(g, bc);
    const int Ptot = g.Ptot;
    for (int base = 0; base < Ptot; base += K * kBlock) {
        C v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int idx = base + threadIdx.x + k * kBlock;
            v[k] = grid[map.src(g, idx < Ptot ? idx : 0)];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int idx = base + threadIdx.x + k * kBlock;
            if (idx < Ptot)
                tile[idx] = v[k];
        }
    }
}

// Planes z0 .. z0 + S - 1 (dimension 0) of the padded 3-D tile of bin `bc`, as the same
// loads and stores as stage_tile_w over S P_1 P_2 entries.
template <typename T, bool P2>
__device__ __forceinline__ void stage_slab_w(const Geom &g, const int *bc, int z0, int S, const Cplx<T> *grid,
                                             Cplx<T> *tile)
{
    using C = Cplx<T>;
    constexpr int K = sizeof(T) == 4 ? 12 : 8;
    TileMap<3, P2> map(g, bc);
    map.o[0] += z0;
    const int cnt = S * g.P[1] * g.P[2];
    for (int base = 0; base < cnt; base += K * kBlock) {
        C v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int idx = base + threadIdx.x + k * kBlock;
            v[k] = grid[map.src(g, idx < cnt ? idx : 0)];
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int idx = base + threadIdx.x + k * kBlock;
            if (idx < cnt)
                tile[idx] = v[k];
        }
    }
}

template <typename T>
__device__ __forceinline__ void stage_slab(const Geom &g, const int *bc, int z0, int S, const Cplx<T> *grid,
                                           Cplx<T> *tile)
{
    if (g.p2)
        stage_slab_w<T, true>(g, bc, z0, S, grid, tile);
    else
        stage_slab_w<T, false>(g, bc, z0, S, grid, tile);
}

template <typename T, int D>
__device__ __forceinline__ void stage_tile(const Geom &g, const int *bc, const Cplx<T> *grid, Cplx<T> *tile)
{
    if (g.p2)
        stage_tile_w<T, D, true>(g, bc, grid, tile);
    else
        stage_tile_w<T, D, false>(g, bc, grid, tile);
}

// Window factors of one dimension at all WM stencil points (zero beyond 2m+2).
template <typename T, int WM, bool AllW = true>
__device__ __forceinline__ void window_row(T delta, const Geom &g, int t, T *w)
{
#pragma unroll
    for (int s = 0; s < WM; ++s)
        w[s] = s < g.W ? win_point<T, AllW>(g, t, delta, s) : T(0);
}

template <typename T, int WM, bool AllW = true>
__device__ __forceinline__ void window_row_d(T delta, const Geom &g, const Nodes &nd, int t, T *w, T *dw)
{
#pragma unroll
    for (int s = 0; s < WM; ++s) {
        w[s] = s < g.W ? win_value<T, AllW>(g, nd, t, delta, s) : T(0);
        dw[s] = s < g.W ? win_value_d<T, AllW>(g, nd, t, delta, s) : T(0);
    }
}

}  // namespace window

}  // namespace nfft

// Dispatch over the compiled stencil widths and over (precision, dimension).
#define NFFT_WM_SWITCH(WMV, CALL)                                                                       \
    switch (WMV) {                                                                                     \
    case 6: CALL(6); break;                                                                            \
    case 10: CALL(10); break;                                                                          \
    case 14: CALL(14); break;                                                                          \
    case 18: CALL(18); break;                                                                          \
    case 22: CALL(22); break;                                                                          \
    case 26: CALL(26); break;                                                                          \
    default: return hipErrorInvalidValue;                                                              \
    }

#define NFFT_DT_SWITCH(FN, ...)                                                                        \
    switch (g.d * 2 + (dbl ? 1 : 0)) {                                                                 \
    case 2: return FN<float, 1>(__VA_ARGS__);                                                          \
    case 3: return FN<double, 1>(__VA_ARGS__);                                                         \
    case 4: return FN<float, 2>(__VA_ARGS__);                                                          \
    case 5: return FN<double, 2>(__VA_ARGS__);                                                         \
    case 6: return FN<float, 3>(__VA_ARGS__);                                                          \
    case 7: return FN<double, 3>(__VA_ARGS__);                                                         \
    default: return hipErrorInvalidValue;                                                              \
    }
