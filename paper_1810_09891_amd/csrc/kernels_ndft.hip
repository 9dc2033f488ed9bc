// Direct sums on the device: f_j = sum_k fhat_k e^{-2 pi i k.x_j} (eq. (1.2)) and
// hhat_k = sum_j f_j e^{+2 pi i k.x_j} (eq. (1.3)).  O(M |I_N|) work, a reference path.
//
// The phase k.x is formed per dimension in FP64 with its exact rounding error (an FMA
// two-product), reduced to [-1/2, 1/2] and only then converted to the accumulation type
// for sincospi, so the exponential is accurate for any |k x|.
#include "launch.hpp"

namespace nfft {

namespace {

constexpr int kTile = 256;

// Fractional part of sum_t k_t x_t in [-1/2, 1/2], from exact products.
__device__ __forceinline__ double phase_frac(int d, const int *k, const double *x)
{
    double acc = 0.0;
    for (int t = 0; t < d; ++t) {
        double kk = (double)k[t];
        double p = kk * x[t];
        double e = fma(kk, x[t], -p);  // p + e == k x exactly
        double r = p - rint(p);        // exact
        acc += r + e;
    }
    return acc - rint(acc);
}

template <typename T> __device__ __forceinline__ void sc_pi(T a, T *s, T *c);
template <> __device__ __forceinline__ void sc_pi<float>(float a, float *s, float *c) { sincospif(a, s, c); }
template <> __device__ __forceinline__ void sc_pi<double>(double a, double *s, double *c) { sincospi(a, s, c); }

__device__ __forceinline__ void centred(int d, const int *N, int64_t idx, int *k)
{
    for (int t = d - 1; t >= 0; --t) {
        int64_t q = idx / N[t];
        k[t] = (int)(idx - q * N[t]) - N[t] / 2;
        idx = q;
    }
}

// One thread per node; coefficients staged through LDS in tiles.
template <typename T> __global__ __launch_bounds__(kTile) void k_ndft_trafo(NdftArgs a)
{
    using C = Cplx<T>;
    __shared__ C s_f[kTile];
    __shared__ int s_k[kTile][kMaxDim];
    const C *fhat = static_cast<const C *>(a.in);
    C *f = static_cast<C *>(a.out);
    int64_t j = (int64_t)blockIdx.x * kTile + threadIdx.x;
    double xj[kMaxDim] = {0.0, 0.0, 0.0};
    if (j < a.M)
        for (int t = 0; t < a.d; ++t)
            xj[t] = a.x[j * a.d + t];
    T ax = 0, ay = 0;
    for (int64_t k0 = 0; k0 < a.K; k0 += kTile) {
        int64_t idx = k0 + threadIdx.x;
        if (idx < a.K) {
            s_f[threadIdx.x] = fhat[idx];
            int kv[kMaxDim];
            centred(a.d, a.N, idx, kv);
            for (int t = 0; t < a.d; ++t)
                s_k[threadIdx.x][t] = kv[t];
        }
        __syncthreads();
        int cnt = (int)min((int64_t)kTile, a.K - k0);
        if (j < a.M) {
            for (int i = 0; i < cnt; ++i) {
                double ph = phase_frac(a.d, s_k[i], xj);
                T s, c;
                sc_pi<T>((T)(2.0 * ph), &s, &c);
                C v = s_f[i];  // v * (c - i s)
                ax += v.x * c + v.y * s;
                ay += v.y * c - v.x * s;
            }
        }
        __syncthreads();
    }
    if (j < a.M)
        f[j] = C{ax, ay};
}

// One thread per coefficient; nodes staged through LDS in tiles.
template <typename T> __global__ __launch_bounds__(kTile) void k_ndft_adjoint(NdftArgs a)
{
    using C = Cplx<T>;
    __shared__ C s_v[kTile];
    __shared__ double s_x[kTile][kMaxDim];
    const C *fin = static_cast<const C *>(a.in);
    C *h = static_cast<C *>(a.out);
    int64_t idx = (int64_t)blockIdx.x * kTile + threadIdx.x;
    int kv[kMaxDim] = {0, 0, 0};
    if (idx < a.K)
        centred(a.d, a.N, idx, kv);
    T ax = 0, ay = 0;
    for (int64_t j0 = 0; j0 < a.M; j0 += kTile) {
        int64_t j = j0 + threadIdx.x;
        if (j < a.M) {
            s_v[threadIdx.x] = fin[j];
            for (int t = 0; t < a.d; ++t)
                s_x[threadIdx.x][t] = a.x[j * a.d + t];
        }
        __syncthreads();
        int cnt = (int)min((int64_t)kTile, a.M - j0);
        if (idx < a.K) {
            for (int i = 0; i < cnt; ++i) {
                double ph = phase_frac(a.d, kv, s_x[i]);
                T s, c;
                sc_pi<T>((T)(2.0 * ph), &s, &c);
                C v = s_v[i];  // v * (c + i s)
                ax += v.x * c - v.y * s;
                ay += v.y * c + v.x * s;
            }
        }
        __syncthreads();
    }
    if (idx < a.K)
        h[idx] = C{ax, ay};
}

}  // namespace

hipError_t launch_ndft(const NdftArgs &a, bool dbl, bool adjoint, hipStream_t s)
{
    int64_t n = adjoint ? a.K : a.M;
    dim3 grid((unsigned)((n + kTile - 1) / kTile)), block(kTile);
    if (adjoint) {
        if (dbl)
            hipLaunchKernelGGL(k_ndft_adjoint<double>, grid, block, 0, s, a);
        else
            hipLaunchKernelGGL(k_ndft_adjoint<float>, grid, block, 0, s, a);
    } else {
        if (dbl)
            hipLaunchKernelGGL(k_ndft_trafo<double>, grid, block, 0, s, a);
        else
            hipLaunchKernelGGL(k_ndft_trafo<float>, grid, block, 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace nfft
