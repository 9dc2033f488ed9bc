// Device-side building blocks of the NFFT library for gfx950: complex helpers, the
// Kaiser-Bessel window in its normalised form, and the parameter blocks the host
// passes to the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nfft {

constexpr int kMaxDim = 3;
constexpr int kBlock = 256;  // threads per workgroup of the window and node kernels

// ------------------------------------------------------------------ complex helpers

template <typename T> struct CplxOf;
template <> struct CplxOf<float> { using type = float2; };
template <> struct CplxOf<double> { using type = double2; };
template <typename T> using Cplx = typename CplxOf<T>::type;
template <typename T> using Pair = Cplx<T>;  // two reals loaded together

template <typename C> __host__ __device__ __forceinline__ C cmul(C a, C b)
{
    return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename C> __host__ __device__ __forceinline__ C cmulc(C a, C b)
{
    return C{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename C> __host__ __device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __host__ __device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C, typename T> __host__ __device__ __forceinline__ C cscale(C a, T s)
{
    return C{a.x * s, a.y * s};
}

// ------------------------------------------------------------------ launch mapping

// The dispatcher hands consecutive workgroups to the 8 XCDs in turn, and each XCD has
// its own L2.  This bijection of [0, G) gives XCD x (blocks b with b mod 8 = x) one
// contiguous range of logical work items, so neighbouring items -- which share cache
// lines of the grid -- run behind the same L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_local_id(int b, int G)
{
    const int x = b % kXcds;
    const int q = G / kXcds, r = G % kXcds;
    const int start = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
    return start + b / kXcds;
}

// ------------------------------------------------------------------ window

// Stencil width bucket: kernels are compiled for WM = 6, 10, ..., 26 points per
// dimension; a plan with 2m+2 < WM pads its window with zeros up to WM.
__host__ __device__ constexpr int wm_bucket(int m)
{
    return m <= 2 ? 6 : m <= 4 ? 10 : m <= 6 ? 14 : m <= 8 ? 18 : m <= 10 ? 22 : 26;
}

// Normalised Kaiser-Bessel window, interior branch (|z| <= m):
//     e^{-bm} * sinh(b s) / (pi s),   s = sqrt(m^2 - z^2),
// evaluated as (e^{b(s-m)} - e^{-b(s+m)}) / (2 pi s) with s - m = -z^2/(s+m), so the
// exponent stays near zero where the window is large and FP32 does not amplify the
// rounding of z.  Near s = 0 the series e^{-bm} (b/pi)(1 + (bs)^2/6 + (bs)^4/120 + ...).
template <typename T> __device__ __forceinline__ T kb_interior(T z, T m, T b, T emb)
{
    const T inv_pi = T(0.318309886183790671537767526745028724);
    T z2 = z * z;
    T a = m * m - z2;
    a = a > T(0) ? a : T(0);
    T s = sqrt(a);
    T bs = b * s;
    if (bs < T(1e-2)) {
        T q = bs * bs;
        return emb * b * inv_pi * (T(1) + q * (T(1) / T(6) + q * (T(1) / T(120) + q * (T(1) / T(5040)))));
    }
    T e1 = exp(-b * z2 / (s + m));
    T e2 = exp(-b * (s + m));
    return (e1 - e2) * (T(0.5) * inv_pi) / s;
}

// Normalised window at the two end points of the stencil (|z| >= m), the analytic
// continuation e^{-bm} sin(b t)/(pi t), t = sqrt(z^2 - m^2).
template <typename T> __device__ __forceinline__ T kb_edge(T z, T m, T b, T emb)
{
    const T inv_pi = T(0.318309886183790671537767526745028724);
    T a = z * z - m * m;
    a = a > T(0) ? a : T(0);
    T t = sqrt(a);
    T bt = b * t;
    if (bt < T(1e-2)) {
        T q = bt * bt;
        return emb * b * inv_pi * (T(1) - q * (T(1) / T(6) - q * (T(1) / T(120))));
    }
    return emb * sin(bt) * inv_pi / t;
}

// Window value at stencil point s (0..W-1) of a node with offset delta in [0,1):
// z = delta - (s - m).  Points s = 0 and s = W-1 are the end points, the 2m points
// between them lie strictly inside |z| < m (or on |z| = m for delta = 0).
template <typename T> __device__ __forceinline__ T kb_point(T delta, int s, int W, T m, T b, T emb)
{
    T z = delta - T(s - (int)m);
    if (s == 0 || s == W - 1)
        return kb_edge(z, m, b, emb);
    return kb_interior(z, m, b, emb);
}

// d/dz of the normalised window, interior branch:
//     phi'(z) = -(z/pi) e^{-bm} (b s cosh(bs) - sinh(bs)) / s^3,
// with e^{-bm} cosh(bs) = (e1 + e2)/2 and e^{-bm} sinh(bs) = (e1 - e2)/2; for small bs the
// series b^3 sum_k 2k/(2k+1)! (bs)^{2k-2}.
template <typename T> __device__ __forceinline__ T kb_interior_d(T z, T m, T b, T emb)
{
    const T inv_pi = T(0.318309886183790671537767526745028724);
    T z2 = z * z;
    T a = m * m - z2;
    a = a > T(0) ? a : T(0);
    T s = sqrt(a);
    T bs = b * s;
    if (bs < T(0.1)) {
        T q = bs * bs;
        T ser = T(1) / T(3) +
                q * (T(1) / T(30) + q * (T(1) / T(840) + q * (T(1) / T(45360) + q * (T(1) / T(3991680)))));
        return -z * inv_pi * emb * b * b * b * ser;
    }
    T e1 = exp(-b * z2 / (s + m));
    T e2 = exp(-b * (s + m));
    T num = T(0.5) * (bs * (e1 + e2) - (e1 - e2));
    return -z * inv_pi * num / (s * s * s);
}

// d/dz at the end points: phi'(z) = (z/pi) e^{-bm} (b t cos(bt) - sin(bt)) / t^3.
template <typename T> __device__ __forceinline__ T kb_edge_d(T z, T m, T b, T emb)
{
    const T inv_pi = T(0.318309886183790671537767526745028724);
    T a = z * z - m * m;
    a = a > T(0) ? a : T(0);
    T t = sqrt(a);
    T bt = b * t;
    if (bt < T(0.1)) {
        T q = bt * bt;
        T ser = -T(1) / T(3) +
                q * (T(1) / T(30) - q * (T(1) / T(840) - q * (T(1) / T(45360) - q * (T(1) / T(3991680)))));
        return z * inv_pi * emb * b * b * b * ser;
    }
    const T sn = sin(bt), cs = cos(bt);
    return z * inv_pi * emb * (bt * cs - sn) / (t * t * t);
}

template <typename T> __device__ __forceinline__ T kb_point_d(T delta, int s, int W, T m, T b, T emb)
{
    T z = delta - T(s - (int)m);
    if (s == 0 || s == W - 1)
        return kb_edge_d(z, m, b, emb);
    return kb_interior_d(z, m, b, emb);
}

// Gaussian window (the other window with a closed-form Fourier pair that the NFFT library
// offers; standard pair of the NFFT literature), divided by its peak (pi b)^{-1/2}:
// exp(-z^2 / b) in the grid variable z; the peak is carried by the deconvolution table.
template <typename T> __device__ __forceinline__ T gauss_point(T delta, int s, T m, T b)
{
    const T z = delta - T(s - (int)m);
    return exp(-z * z / b);
}
template <typename T> __device__ __forceinline__ T gauss_point_d(T delta, int s, T m, T b)
{
    const T z = delta - T(s - (int)m);
    return T(-2) * z / b * exp(-z * z / b);
}

// ------------------------------------------------------------------ parameter blocks

// Geometry of a plan's window kernels.
struct Geom {
    int d;
    int m;
    int W;             // 2m+2
    int WM;            // compiled stencil width (>= W)
    int n[kMaxDim];    // grid lengths (1 for unused dimensions)
    int lgB[kMaxDim];  // log2 of the bin edge per dimension
    int nb[kMaxDim];   // bins per dimension
    int P[kMaxDim];    // padded tile edge B + WM - 1
    int Ptot;          // prod P
    int nbins;
    int window;           // 0 Kaiser-Bessel, 1 Gaussian
    int fold2;            // every grid index is covered by at most 2 tiles per dimension
    double b[kMaxDim];    // window shape per dimension
    double emb[kMaxDim];  // 1 / (factor the device window is divided by): e^{-b m} (Kaiser-Bessel),
                          // (pi b)^{1/2} (Gaussian)
};

// Window factor of dimension t at stencil point s of a node with offset delta, and its
// derivative with respect to the grid variable, for the plan's window.
template <typename T> __device__ __forceinline__ T win_point(const Geom &g, int t, T delta, int s)
{
    if (g.window == 1)
        return gauss_point<T>(delta, s, (T)g.m, (T)g.b[t]);
    return kb_point<T>(delta, s, g.W, (T)g.m, (T)g.b[t], (T)g.emb[t]);
}
template <typename T> __device__ __forceinline__ T win_point_d(const Geom &g, int t, T delta, int s)
{
    if (g.window == 1)
        return gauss_point_d<T>(delta, s, (T)g.m, (T)g.b[t]);
    return kb_point_d<T>(delta, s, g.W, (T)g.m, (T)g.b[t], (T)g.emb[t]);
}

// Sorted node data in the workspace (written by the node kernels).
struct Nodes {
    int32_t *u[kMaxDim];   // grid index floor(n x) mod n, sorted order
    void *delta[kMaxDim];  // n x - floor(n x) (float or double), sorted order
    int32_t *perm;         // sorted position -> caller index
    int32_t *key;          // bin of each node, caller order
    int32_t *rank;         // rank of each node inside its bin, caller order
    int32_t *bin_count;    // [nbins]
    int32_t *bin_start;    // [nbins+1]
    int32_t *bin_chunk;    // [nbins+1] first work item of each bin
    int32_t *chunk_bin;    // [max_chunks]
    int32_t *chunk_first;  // [max_chunks] first sorted node
    int32_t *chunk_len;    // [max_chunks]
    int32_t *counters;     // [0] = number of work items, [1] = non-finite node flag
    void *psi;             // window factors per sorted node: [M][d][W] (float or double)
    int32_t *spos;         // d = 2 spreading in registers, else null: per work item, its
                           // nodes in order of tile row as pairs ((offset << 10) | (row << 5)
                           // | column, caller index)
    const double *x;       // caller node array (only used while setting nodes)
    int64_t M;
    int chunk_cap;
    int max_chunks;
};

}  // namespace nfft
