// NNFFT: nonequispaced nodes in both domains, the generalisation of the NFFT named in
// Sec. 1.  For frequencies v_k in [-N_t/2, N_t/2)^d and nodes x_j in [-1/2, 1/2)^d,
//     f_j = sum_k fhat_k e^{-2 pi i v_k . x_j},     hhat_k = sum_j f_j e^{+2 pi i v_k . x_j}.
//
// The frequencies are spread onto an equispaced frequency grid with the window of an
// inner plan A, which turns the sum into an NFFT (plan B) at scaled nodes.  Per
// dimension, with a grid of N2 points (a power of two), plan A's coefficient count N_A
// (even, sigma1 = N2 / N_A > 1) and the spacing h = 1 / sigma1:
//   u_k = N2 y_k with y_k = v_k / N_A   (plan A node; grid position sigma1 v_k),
//   z_j = h x_j = x_j N_A / N2          (plan B node, |z_j| <= 1 / (2 sigma1)).
// Poisson summation of the window psi_A = phi_A / lambda_A gives, for real z,
//   sum_l psi_A(u - l) e^{-2 pi i l z} = e^{-2 pi i u z} sum_r Phi_A(z + r) / lambda_A,
// and the r != 0 terms are the aliasing error of an NFFT with oversampling sigma1.  With
// u z = v_k x_j and w_A(z) = lambda_A / Phi_A(z) (the deconvolution factor of eq. (2.9)
// taken at a real argument):
//   f_j ~ w_A(z_j) sum_{l in I_N2} G_l e^{-2 pi i l z_j},   G_l = sum_k fhat_k psi_A(u_k - l),
// i.e. G = plan A's spreading step (Algorithm 2.2 step 1) of fhat at y, moved from the
// periodic grid order to the centred coefficient order, then f = w_A(z) (.) NFFT_B(G)
// (Algorithm 2.1 at nodes z).  N2 leaves m + 2 cells on each side of sigma1 [-N/2, N/2),
// so no stencil wraps around the grid and G holds the spread values at their true l.  The
// adjoint runs the transposed steps in reverse: NFFT_B^H(w_A(z) (.) f), centred to
// periodic order, then plan A's interpolation step (Algorithm 2.1 step 3) at y.
#include <cmath>
#include <new>

#include "plan_impl.hpp"

namespace nfft {

namespace {

constexpr int kNNBlock = 256;

inline int nn_blocks(int64_t items)
{
    int64_t b = (items + kNNBlock - 1) / kNNBlock;
    if (b < 1)
        b = 1;
    return (int)(b > 65535 ? 65535 : b);
}

struct NNScale {
    int d;
    double ya[kMaxDim];  // 1 / N_A per dimension: y = v / N_A
    double za[kMaxDim];  // N_A / N2 per dimension: z = x N_A / N2
};

// y[k][t] = v[k][t] / N_A[t] and z[j][t] = x[j][t] N_A[t] / N2[t]
__global__ __launch_bounds__(kNNBlock) void k_nn_nodes(NNScale sc, const double *__restrict__ v, double *__restrict__ y,
                                                       int64_t nv, const double *__restrict__ x,
                                                       double *__restrict__ z, int64_t nx)
{
    const int64_t stride = (int64_t)gridDim.x * kNNBlock;
    for (int64_t i = blockIdx.x * (int64_t)kNNBlock + threadIdx.x; i < nv + nx; i += stride) {
        if (i < nv) {
            const int t = (int)(i % sc.d);
            y[i] = v[i] * sc.ya[t];
        } else {
            const int64_t q = i - nv;
            const int t = (int)(q % sc.d);
            z[q] = x[q] * sc.za[t];
        }
    }
}

// Modified Bessel function I_0 by its power series sum_k ((x/2)^(2k)) / (k!)^2, all
// terms positive, summed until they no longer change the FP64 sum.
__device__ double bessel_i0(double x)
{
    const double q = 0.25 * x * x;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 500; ++k) {
        term *= q / ((double)k * (double)k);
        sum += term;
        if (term < sum * 1e-17)
            break;
    }
    return sum;
}

// Centred cardinal B-spline M_k(u) = N_k(u + k/2), de Boor's triangle in FP64 (k <= 24).
__device__ double centred_bspline_dev(int k, double u)
{
    const double x = u + 0.5 * k;
    if (!(x >= 0.0) || x >= (double)k)
        return 0.0;
    const double t = x - floor(x);
    const int j = (int)floor(x);
    double b[25];
    for (int i = 0; i <= k; ++i)
        b[i] = 0.0;
    b[0] = 1.0;
    for (int qd = 2; qd <= k; ++qd)
        for (int i = qd - 1; i >= 0; --i) {
            const double left = i > 0 ? b[i - 1] : 0.0;
            b[i] = ((t + i) * b[i] + (qd - t - i) * left) / (qd - 1);
        }
    return b[j];
}

// w(z) = lambda / Phi(z) of dimension t of a plan geometry at a real frequency z (cycles
// per grid cell): the deconvolution factor of eq. (2.9), whose table holds w(k / n).
__device__ double deconv_at(const Geom &g, int t, double z)
{
    const double pi = 3.14159265358979323846;
    const double b = g.b[t];
    switch (g.window) {
    case 1:  // Gaussian: lambda e^{b (pi z)^2}
        return exp(b * (pi * z) * (pi * z)) / g.emb[t];
    case 2: {  // B-spline: (sin(pi z) / (pi z))^(-2m)
        const double a = pi * z;
        const double s = a == 0.0 ? 1.0 : sin(a) / a;
        return 1.0 / pow(s, 2.0 * g.m);
    }
    case 3:  // sinc: 1 / ((pi / a) M_2m(pi z / a)), a = b
        return 1.0 / ((pi / b) * centred_bspline_dev(2 * g.m, pi * z / b));
    default: {  // Kaiser-Bessel: e^{b m} / I0(m sqrt(b^2 - (2 pi z)^2))
        const double w = 2.0 * pi * z;
        return 1.0 / (g.emb[t] * bessel_i0((double)g.m * sqrt(b * b - w * w)));
    }
    }
}

// fac[j] = prod_t w_A,t(z[j][t]) (NaN for a non-finite node)
__global__ __launch_bounds__(kNNBlock) void k_nn_factor(Geom ga, int d, const double *__restrict__ z,
                                                        double *__restrict__ fac, int64_t M)
{
    const int64_t stride = (int64_t)gridDim.x * kNNBlock;
    for (int64_t j = blockIdx.x * (int64_t)kNNBlock + threadIdx.x; j < M; j += stride) {
        double f = 1.0;
        for (int t = 0; t < d; ++t)
            f *= deconv_at(ga, t, z[j * d + t]);
        fac[j] = f;
    }
}

// out = in moved by N2_t / 2 cells in every dimension (periodic grid order <-> centred
// coefficient order; the move is its own inverse).  lg[t] = log2 N2_t.
template <typename T>
__global__ __launch_bounds__(kNNBlock) void k_nn_shift(int d, int3 lg, const Cplx<T> *__restrict__ in,
                                                       Cplx<T> *__restrict__ out, int64_t total)
{
    const int lgv[3] = {lg.x, lg.y, lg.z};
    const int64_t stride = (int64_t)gridDim.x * kNNBlock;
    for (int64_t i = blockIdx.x * (int64_t)kNNBlock + threadIdx.x; i < total; i += stride) {
        int64_t src = 0;
        int shift = 0;
        for (int t = d - 1; t >= 0; --t) {
            const int64_t n = (int64_t)1 << lgv[t];
            const int64_t it = (i >> shift) & (n - 1);
            src |= ((it + n / 2) & (n - 1)) << shift;
            shift += lgv[t];
        }
        out[i] = in[src];
    }
}

// out[j] = fac[j] in[j] (complex times FP64 factor rounded to T)
template <typename T>
__global__ __launch_bounds__(kNNBlock) void k_nn_scale(const double *__restrict__ fac, const Cplx<T> *__restrict__ in,
                                                       Cplx<T> *__restrict__ out, int64_t M)
{
    const int64_t stride = (int64_t)gridDim.x * kNNBlock;
    for (int64_t j = blockIdx.x * (int64_t)kNNBlock + threadIdx.x; j < M; j += stride) {
        const T f = (T)fac[j];
        const Cplx<T> a = in[j];
        out[j] = Cplx<T>{f * a.x, f * a.y};
    }
}

}  // namespace

}  // namespace nfft

using namespace nfft;

struct nnfft_plan_s {
    int d = 0, m = 0;
    bool dbl = false;
    uint32_t flags = 0;
    int64_t N[kMaxDim] = {1, 1, 1}, N2[kMaxDim] = {1, 1, 1}, NA[kMaxDim] = {1, 1, 1};
    int64_t K = 0, M = 0, ngrid = 1;
    double sigma1[kMaxDim] = {1, 1, 1};
    nfft_plan A = nullptr, B = nullptr;
    size_t wsA = 0, wsB = 0;
    size_t off_A = 0, off_B = 0, off_y = 0, off_z = 0, off_fac = 0, off_c = 0, off_tmp = 0, ws_bytes = 0;
    void *ws = nullptr;
    bool nodes_set = false;
};

namespace {

constexpr size_t kNNAlign = 256;
size_t nn_align(size_t x) { return (x + kNNAlign - 1) / kNNAlign * kNNAlign; }

int nn_hip(hipError_t e) { return e == hipSuccess ? NFFT_OK : NFFT_ERR_HIP; }

char *nn_at(const nnfft_plan_s *p, size_t off) { return static_cast<char *>(p->ws) + off; }

}  // namespace

int nnfft_plan_create(nnfft_plan *out, int d, const int64_t *N, int64_t K, int64_t M, double sigma, int m,
                      nfft_dtype dtype, uint32_t flags)
{
    if (!out || !N || d < 1 || d > kMaxDim || K < 1 || M < 1)
        return NFFT_ERR_ARG;
    if (dtype != NFFT_C64 && dtype != NFFT_C128)
        return NFFT_ERR_ARG;
    const uint32_t win = flags & (NFFT_WINDOW_GAUSSIAN | NFFT_WINDOW_BSPLINE | NFFT_WINDOW_SINC);
    if ((flags & ~(win | NFFT_SORT_NODES)) != 0)
        return NFFT_ERR_ARG;
    if (m == 0)
        m = 8;
    if (m < 1)
        return NFFT_ERR_ARG;
    const bool autos = sigma == 0.0;
    if (!autos && (!(sigma > 1.0) || !(sigma <= 16.0)))
        return NFFT_ERR_ARG;
    nnfft_plan_s *p = new (std::nothrow) nnfft_plan_s;
    if (!p)
        return NFFT_ERR_ARG;
    p->d = d;
    p->m = m;
    p->dbl = dtype == NFFT_C128;
    p->flags = flags;
    p->K = K;
    p->M = M;
    int64_t NB[kMaxDim], nA[kMaxDim];
    for (int t = 0; t < d; ++t) {
        if (N[t] < 2 || (N[t] & 1)) {
            delete p;
            return NFFT_ERR_ARG;
        }
        p->N[t] = N[t];
        // frequency grid: sigma N_t points plus m + 2 cells of margin on each side, rounded
        // up to a power of two; automatic: the power of two >= 2 N_t, doubled while the
        // margin would leave sigma1 below 1.5
        const int64_t need = autos ? 2 * N[t] : (int64_t)std::ceil(sigma * (double)N[t]) + 2 * m + 4;
        int64_t n2 = 2;
        while (n2 < need)
            n2 *= 2;
        // plan A's coefficient count: the smallest even N_A with
        // N2 N / N_A <= N2 - 2m - 4 (so sigma1 [-N/2, N/2) plus the stencil fits)
        auto coef_count = [&](int64_t g) -> int64_t {
            if (g <= 2 * m + 4)
                return g;  // no room: rejected below
            int64_t a = (int64_t)std::ceil((double)N[t] * (double)g / (double)(g - 2 * m - 4));
            while ((double)N[t] * (double)g > (double)a * (double)(g - 2 * m - 4))
                ++a;
            return a + (a & 1);
        };
        int64_t na = coef_count(n2);
        while (autos && (double)n2 < 1.5 * (double)na && n2 < (int64_t)1 << 30) {
            n2 *= 2;
            na = coef_count(n2);
        }
        if (na >= n2) {
            delete p;
            return NFFT_ERR_UNSUPPORTED;
        }
        p->N2[t] = n2;
        p->NA[t] = na;
        p->sigma1[t] = (double)n2 / (double)na;
        p->ngrid *= n2;
        NB[t] = n2;
        nA[t] = n2;
    }
    const uint32_t inner = win | (flags & NFFT_SORT_NODES);
    int st = nfft_plan_create(&p->A, d, p->NA, K, nA, m, dtype, inner);
    if (st == NFFT_OK)
        st = nfft_plan_create(&p->B, d, NB, M, nullptr, m, dtype, inner);
    if (st == NFFT_OK)
        st = nfft_workspace_bytes(p->A, &p->wsA);
    if (st == NFFT_OK)
        st = nfft_workspace_bytes(p->B, &p->wsB);
    if (st != NFFT_OK) {
        if (p->A)
            nfft_plan_destroy(p->A);
        if (p->B)
            nfft_plan_destroy(p->B);
        delete p;
        return st;
    }
    const size_t cs = p->dbl ? 16 : 8;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = nn_align(off + bytes);
        return o;
    };
    p->off_A = take(p->wsA);
    p->off_B = take(p->wsB);
    p->off_y = take(sizeof(double) * (size_t)K * d);
    p->off_z = take(sizeof(double) * (size_t)M * d);
    p->off_fac = take(sizeof(double) * (size_t)M);
    p->off_c = take(cs * (size_t)p->ngrid);
    p->off_tmp = take(cs * (size_t)M);
    p->ws_bytes = off;
    *out = p;
    return NFFT_OK;
}

int nnfft_plan_destroy(nnfft_plan p)
{
    if (!p)
        return NFFT_ERR_ARG;
    nfft_plan_destroy(p->A);
    nfft_plan_destroy(p->B);
    delete p;
    return NFFT_OK;
}

int nnfft_plan_get_info(nnfft_plan p, nnfft_plan_info *info)
{
    if (!p || !info)
        return NFFT_ERR_ARG;
    *info = nnfft_plan_info{};
    info->d = p->d;
    info->m = p->m;
    info->K = p->K;
    info->M = p->M;
    for (int t = 0; t < kMaxDim; ++t) {
        info->N[t] = p->N[t];
        info->N2[t] = p->N2[t];
        info->NA[t] = p->NA[t];
        info->sigma1[t] = p->sigma1[t];
    }
    info->workspace_bytes = p->ws_bytes;
    info->window = p->A->geom.window;
    return NFFT_OK;
}

int nnfft_workspace_bytes(nnfft_plan p, size_t *bytes)
{
    if (!p || !bytes)
        return NFFT_ERR_ARG;
    *bytes = p->ws_bytes;
    return NFFT_OK;
}

int nnfft_set_workspace(nnfft_plan p, void *ws, size_t bytes)
{
    if (!p)
        return NFFT_ERR_ARG;
    if (!ws || bytes < p->ws_bytes || (reinterpret_cast<uintptr_t>(ws) % kNNAlign) != 0)
        return NFFT_ERR_WORKSPACE;
    p->ws = ws;
    p->nodes_set = false;
    int st = nfft_set_workspace(p->A, nn_at(p, p->off_A), p->wsA);
    if (st == NFFT_OK)
        st = nfft_set_workspace(p->B, nn_at(p, p->off_B), p->wsB);
    return st;
}

int nnfft_set_nodes(nnfft_plan p, const double *x, const double *v, hipStream_t s)
{
    if (!p || !x || !v)
        return NFFT_ERR_ARG;
    if (!p->ws)
        return NFFT_ERR_WORKSPACE;
    p->nodes_set = false;
    NNScale sc{};
    sc.d = p->d;
    for (int t = 0; t < p->d; ++t) {
        sc.ya[t] = 1.0 / (double)p->NA[t];
        sc.za[t] = (double)p->NA[t] / (double)p->N2[t];
    }
    double *y = reinterpret_cast<double *>(nn_at(p, p->off_y));
    double *z = reinterpret_cast<double *>(nn_at(p, p->off_z));
    double *fac = reinterpret_cast<double *>(nn_at(p, p->off_fac));
    const int64_t nv = p->K * p->d, nx = p->M * p->d;
    hipLaunchKernelGGL(k_nn_nodes, dim3(nn_blocks(nv + nx)), dim3(kNNBlock), 0, s, sc, v, y, nv, x, z, nx);
    int st = nn_hip(hipGetLastError());
    if (st == NFFT_OK)
        st = nfft_set_nodes(p->A, y, s);
    if (st == NFFT_OK)
        st = nfft_set_nodes(p->B, z, s);
    if (st != NFFT_OK)
        return st;
    hipLaunchKernelGGL(k_nn_factor, dim3(nn_blocks(p->M)), dim3(kNNBlock), 0, s, p->A->geom, p->d, z, fac, p->M);
    st = nn_hip(hipGetLastError());
    if (st == NFFT_OK)
        p->nodes_set = true;
    return st;
}

namespace {

int nn_shift(const nnfft_plan_s *p, const void *in, void *out, hipStream_t s)
{
    int lg[3] = {0, 0, 0};
    for (int t = 0; t < p->d; ++t) {
        int l = 0;
        while (((int64_t)1 << l) < p->N2[t])
            ++l;
        lg[t] = l;
    }
    const int3 lgv = make_int3(lg[0], lg[1], lg[2]);
    if (p->dbl)
        hipLaunchKernelGGL(k_nn_shift<double>, dim3(nn_blocks(p->ngrid)), dim3(kNNBlock), 0, s, p->d, lgv,
                           static_cast<const double2 *>(in), static_cast<double2 *>(out), p->ngrid);
    else
        hipLaunchKernelGGL(k_nn_shift<float>, dim3(nn_blocks(p->ngrid)), dim3(kNNBlock), 0, s, p->d, lgv,
                           static_cast<const float2 *>(in), static_cast<float2 *>(out), p->ngrid);
    return nn_hip(hipGetLastError());
}

int nn_scale(const nnfft_plan_s *p, const void *in, void *out, hipStream_t s)
{
    const double *fac = reinterpret_cast<const double *>(nn_at(p, p->off_fac));
    if (p->dbl)
        hipLaunchKernelGGL(k_nn_scale<double>, dim3(nn_blocks(p->M)), dim3(kNNBlock), 0, s, fac,
                           static_cast<const double2 *>(in), static_cast<double2 *>(out), p->M);
    else
        hipLaunchKernelGGL(k_nn_scale<float>, dim3(nn_blocks(p->M)), dim3(kNNBlock), 0, s, fac,
                           static_cast<const float2 *>(in), static_cast<float2 *>(out), p->M);
    return nn_hip(hipGetLastError());
}

int nn_ready(const nnfft_plan_s *p)
{
    if (!p->ws)
        return NFFT_ERR_WORKSPACE;
    if (!p->nodes_set)
        return NFFT_ERR_STATE;
    return NFFT_OK;
}

}  // namespace

int nnfft_trafo(nnfft_plan p, const void *fhat, void *f, hipStream_t s)
{
    if (!p || !fhat || !f)
        return NFFT_ERR_ARG;
    int st = nn_ready(p);
    if (st != NFFT_OK)
        return st;
    // G on plan A's periodic grid (its workspace grid), then centred into c
    void *gA = static_cast<char *>(p->A->ws) + p->A->off_grid;
    void *c = nn_at(p, p->off_c);
    if ((st = nfft_step_spread(p->A, fhat, gA, s)) != NFFT_OK)
        return st;
    p->A->grid_valid = false;
    if ((st = nn_shift(p, gA, c, s)) != NFFT_OK)
        return st;
    if ((st = nfft_trafo(p->B, c, f, s)) != NFFT_OK)
        return st;
    return nn_scale(p, f, f, s);
}

int nnfft_adjoint(nnfft_plan p, const void *f, void *hhat, hipStream_t s)
{
    if (!p || !f || !hhat)
        return NFFT_ERR_ARG;
    int st = nn_ready(p);
    if (st != NFFT_OK)
        return st;
    void *tmp = nn_at(p, p->off_tmp);
    void *c = nn_at(p, p->off_c);
    void *gA = static_cast<char *>(p->A->ws) + p->A->off_grid;
    if ((st = nn_scale(p, f, tmp, s)) != NFFT_OK)
        return st;
    if ((st = nfft_adjoint(p->B, tmp, c, s)) != NFFT_OK)
        return st;
    if ((st = nn_shift(p, c, gA, s)) != NFFT_OK)
        return st;
    p->A->grid_valid = false;
    return nfft_step_interp(p->A, gA, hhat, s);
}
