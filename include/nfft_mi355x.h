/*
 * nfft_mi355x.h -- C ABI of the MI355X (gfx950) NFFT library.
 *
 * The library evaluates the multivariate trigonometric polynomial
 *     f_j = sum_{k in I_N} fhat_k exp(-2 pi i k . x_j),      j = 0..M-1
 * (arXiv:1810.09891, Sec. 1 eq. (1.2) and Sec. 2 eq. (2.1)) and its adjoint
 *     hhat_k = sum_j f_j exp(+2 pi i k . x_j),                k in I_N
 * (Sec. 1 eq. (1.3)), with I_N = {-N_t/2, ..., N_t/2-1}^d (Sec. 2 eq. (2.2)), by the
 * NFFT of Algorithm 2.1 (deconvolve, oversampled FFT, window interpolation) and the
 * adjoint NFFT of Algorithm 2.2 (window spreading, oversampled FFT, deconvolution),
 * with the Kaiser-Bessel window named in Sec. 4.  The direct sums are available too.
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 *  * Pointers marked [device] are HIP device memory owned by the caller; pointers
 *    marked [host] are host memory read before the call returns.  No transform, node
 *    or step entry point allocates or frees device memory: all scratch lives in a
 *    caller-provided workspace (nfft_workspace_bytes / nfft_set_workspace, and
 *    nfft_batch_workspace_bytes / nfft_batch_set_workspace for batches).  The
 *    exceptions are the tuning calls nfft_batch_autotune and nfft_plan_tune, which
 *    allocate and free their temporary stand-in inputs and candidate workspaces.
 *  * Results are bitwise reproducible from run to run for a given device, plan, workspace
 *    layout and input (see NFFT_DETERMINISTIC).
 *  * Every call that does device work enqueues it on the given stream and returns
 *    without waiting; results are ready when that stream reaches them.
 *  * Complex data are interleaved (re, im): float2 for NFFT_C64 plans, double2 for
 *    NFFT_C128 plans.  Node coordinates are always double.
 *  * Coefficient arrays fhat / hhat have shape N[0] x ... x N[d-1], row-major (last
 *    index fastest) and centred: position i_t holds frequency k_t = i_t - N_t/2.
 *  * Node arrays x have shape M x d, row-major; node values f have length M in the
 *    caller's node order.  Nodes may lie anywhere on the real line; the transform is
 *    1-periodic in every coordinate (the torus of Sec. 1).
 *  * Oversampled grids g have shape n[0] x ... x n[d-1], row-major; position l_t holds
 *    grid index l_t (frequency or spatial index taken modulo n_t).
 *  * Every function returns an nfft_status.  Argument and state errors are detected
 *    on the host before anything is enqueued; NFFT_ERR_HIP reports a failed launch.
 *    Device faults surface at the caller's next synchronisation.
 *  * A plan is used by one stream at a time; different plans may run concurrently
 *    on different streams.
 */
#ifndef NFFT_MI355X_H
#define NFFT_MI355X_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nfft_plan_s *nfft_plan;
typedef struct nfft_batch_s *nfft_batch;

/* Arithmetic type of a plan: complex64 (float data, FP32 window and accumulation,
 * FP64 node index and deconvolution table) or complex128 (FP64 throughout). */
typedef enum { NFFT_C64 = 1, NFFT_C128 = 2 } nfft_dtype;

typedef enum {
    NFFT_OK = 0,
    NFFT_ERR_ARG = -1,         /* invalid argument (size, pointer, parameter)        */
    NFFT_ERR_STATE = -2,       /* call out of order (no workspace, no nodes, ...)    */
    NFFT_ERR_WORKSPACE = -3,   /* workspace missing, too small or misaligned         */
    NFFT_ERR_HIP = -4,         /* a HIP call or kernel launch failed                 */
    NFFT_ERR_UNSUPPORTED = -5  /* valid by the paper, not implemented by this library */
} nfft_status;

/* Plan flags.
 *  NFFT_SORT_NODES: sort nodes into bins of grid cells before interpolation and
 *    spreading (the node sorting flag of Sec. 3.1, Table 3.2).  Always on; accepted
 *    for compatibility.
 *  NFFT_KEEP_GRID: keep the oversampled grid of the last nfft_trafo in the workspace
 *    (separate from the grid nfft_adjoint uses), as nfft_grad_x needs it.
 *  NFFT_WINDOW_GAUSSIAN: use the Gaussian window instead of the Kaiser-Bessel window of
 *    Sec. 4 (the library of Sec. 3 can be configured with either; the paper prints neither
 *    formula): phi(z) = (pi b)^{-1/2} exp(-z^2/b) in the grid variable z = n x - l,
 *    b = 2 sigma m / ((2 sigma - 1) pi), sigma = n/N, Fourier transform exp(-b (pi k/n)^2);
 *    same 2m+2-point stencil.  Less accurate than Kaiser-Bessel at equal m.
 *  NFFT_WINDOW_BSPLINE: the B-spline window (the third of the library's windows, standard
 *    pair of the NFFT literature): phi(z) = M_2m(z), the centred cardinal B-spline of order
 *    2m (support [-m, m]), Fourier transform (sin(pi k/n) / (pi k/n))^(2m).
 *  NFFT_WINDOW_SINC: the sinc window (the fourth): phi(z) = (sin(a z) / (a z))^(2m),
 *    a = pi (2 - 1/sigma) / (2m), Fourier transform (pi/a) M_2m(pi k / (n a)); truncated to
 *    the same 2m+2-point stencil.
 *  At most one window flag may be set (NFFT_ERR_ARG otherwise).
 *  NFFT_DETERMINISTIC: bitwise run-to-run reproducible results.  Always on; accepted so
 *    that callers can state the requirement.  Every floating-point sum of the library has
 *    a fixed order: no atomics touch floating-point data, the nodes of a bin are kept in
 *    caller-index order (so a bin's split into work items is fixed), and the partial
 *    results of the spreading step are folded in a fixed order.
 *  NFFT_PRE_LIN_PSI: the window factors that nfft_set_nodes precomputes, and the factors and
 *    derivatives of nfft_grad_x, come from lookup tables (Sec. 3.1, Table 3.2: PRE_LIN_PSI)
 *    instead of the closed form: per dimension and stencil point, 4097 samples in the offset
 *    delta in [0, 1] (evaluated in FP64 at set-up), linearly interpolated.  The
 *    interpolation adds a relative error of about 1e-8 to each factor (second differences
 *    of the window over steps of 1/4096); results are within 1e-7 of the exact transform for
 *    the windows and sizes tested, so complex128 plans with this flag do not meet 1e-12.
 *    The tables take 2 (2m+2) 4097 reals per dimension of the workspace. */
enum {
    NFFT_SORT_NODES = 1u << 0,
    NFFT_KEEP_GRID = 1u << 1,
    NFFT_WINDOW_GAUSSIAN = 1u << 2,
    NFFT_WINDOW_BSPLINE = 1u << 3,
    NFFT_WINDOW_SINC = 1u << 4,
    NFFT_DETERMINISTIC = 1u << 5,
    NFFT_PRE_LIN_PSI = 1u << 6
};

/* Read-only description of a plan (filled by nfft_plan_get_info). */
typedef struct {
    int d;                  /* dimension, 1..3                                   */
    int m;                  /* window size (stencil of 2m+2 points per dimension)  */
    int dtype;              /* nfft_dtype                                        */
    uint32_t flags;
    int64_t N[3];           /* bandwidths (unused entries 1)                     */
    int64_t n[3];           /* FFT lengths (unused entries 1)                    */
    int64_t M;              /* number of nodes                                   */
    int64_t bin[3];         /* bin edge, grid cells per dimension                */
    int64_t nbins;          /* number of bins                                    */
    int64_t chunk_cap;      /* maximum nodes per work item                       */
    int64_t max_chunks;     /* upper bound on work items for any node set        */
    size_t workspace_bytes; /* bytes nfft_set_workspace needs                    */
    size_t lds_bytes;       /* LDS bytes per workgroup of the window kernels       */
    double grid_scale;      /* prod_t lambda_t: factor carried by the grids of the
                               single-step entry points (see there); lambda_t =
                               e^{b_t m} (Kaiser-Bessel), (pi b_t)^{-1/2} (Gaussian) */
    int window;             /* 0 Kaiser-Bessel, 1 Gaussian, 2 B-spline, 3 sinc     */
    int own_tiles;          /* 3-D plans whose spreading runs by output tiles (each grid
                               cell written once by the workgroup that owns it): the
                               number of tiles; 0 when the plan uses padded work-item
                               tiles and a fold                                      */
    int64_t own_tile[3];    /* output tile edge per dimension (0 when own_tiles = 0) */
} nfft_plan_info;

/* ---------------------------------------------------------------- plans */

/* Create a plan for d-variate transforms with bandwidths N[0..d-1] (even, >= 2;
 * Sec. 3.1, Table 3.1), M >= 1 nodes, FFT lengths n[0..d-1] and window size m.
 *   N      [host] d entries.
 *   n      [host] d entries, or NULL for n_t = 2^(ceil(log2 N_t)+1) (Sec. 2 and Sec. 3.1).
 *          Each n_t must be even and > N_t (Sec. 3.1) and at most 4096, the longest FFT
 *          line one workgroup holds (else NFFT_ERR_UNSUPPORTED).  Any even length is
 *          accepted (the n-sweeps of Sec. 4.3.1 use 514, 614, 716, 820, 130, 154): lengths
 *          that are not powers of two run mixed-radix FFT passes whose odd prime factors
 *          are direct sums (cost L p per line for a factor p), so powers of two are fastest.
 *          Near n_t = N_t the deconvolution factors span many orders of magnitude and the
 *          rounding of any evaluation is amplified accordingly (Fig. 4.1(a), 4.2(a)).
 *   m      window size >= 1 with 2m+2 <= n_t (m << n_t, Sec. 2 eq. (2.10)); 0 selects the
 *          default m = 8 (Sec. 3.1).  Values up to 12 are supported when the window
 *          tile fits the LDS of one workgroup (else NFFT_ERR_UNSUPPORTED).  3-D plans whose
 *          smallest tile does not fit (complex128 m >= 9, complex64 m >= 11) are accepted
 *          when every n_t is a multiple of 16 with n_t >= 16 + 2m + 1 (spreading by output
 *          tiles): their interpolation and node gradient stage the tile in slabs of planes.
 *   dtype  NFFT_C64 or NFFT_C128.
 * Host only: no device work, no device memory.  *out receives the plan. */
int nfft_plan_create(nfft_plan *out, int d, const int64_t *N, int64_t M, const int64_t *n, int m,
                     nfft_dtype dtype, uint32_t flags);

/* Work decomposition of a plan's window steps (Sec. 3.1: the precomputation choices of
 * Table 3.2 and the measured tuning of Table 3.3 are the paper's counterparts).
 *   bin[t]     bin edge in grid cells per dimension: nodes are sorted into bins of
 *              bin[0] x ... x bin[d-1] cells and the window kernels stage one padded tile
 *              per bin.  Powers of two no longer than n_t; 0 in bin[0] selects the
 *              default rule (largest edges up to 512 / 32 x 32 / 8 x 8 x 8 whose tiles fit
 *              the LDS).  Entries past d are ignored.
 *   chunk_cap  maximum nodes per work item, a power of two in [32, 1024]; 0 selects the
 *              default (M / 512 rounded down to a power of two, within [128, 1024]). */
typedef struct {
    int32_t bin[3];
    int32_t chunk_cap;
} nfft_plan_params;

/* nfft_plan_create with a given work decomposition (params may be NULL: the defaults).
 * Errors as nfft_plan_create, plus NFFT_ERR_ARG for edges or caps outside the ranges above
 * and NFFT_ERR_UNSUPPORTED when the requested tiles do not fit the LDS.  Results do not
 * depend on params beyond rounding (every choice computes the same sums). Host only. */
int nfft_plan_create_params(nfft_plan *out, int d, const int64_t *N, int64_t M, const int64_t *n, int m,
                            nfft_dtype dtype, uint32_t flags, const nfft_plan_params *params);

/* Measured choice of the work decomposition for a plan shape and node set (the analogue of
 * FFTW's measured plans and wisdom that Sec. 3.1 uses for the FFT).  Candidates: chunk
 * caps 128 ... 1024 with the default bins, then bin edges halved or doubled per dimension
 * with the best cap; each is timed as nfft_set_nodes once and three nfft_trafo +
 * nfft_adjoint pairs on `stream`; a candidate replaces the best so far only when it is
 * more than 5% faster (short timings vary by a few percent), and shapes whose default
 * transform pair takes under 0.1 ms (launch latency) keep the defaults.
 *   x       [device] M x d FP64 nodes (as for nfft_set_nodes).
 *   cache   [host] path of a text file, or NULL: a shape already in the file (key: d, n,
 *           floor(log2 M), m, precision, window) is answered from it without timing, and a
 *           new result is appended.
 *   out     [host] receives the chosen parameters; best_ms (may be NULL) the measured time
 *           of one transform pair with them (0 when answered from the cache).
 * This call allocates and frees device memory (the candidate plans' workspaces and
 * stand-in data) and synchronises the stream; it is a set-up step, not a transform. */
int nfft_plan_tune(int d, const int64_t *N, int64_t M, const int64_t *n, int m, nfft_dtype dtype, uint32_t flags,
                   const double *x, const char *cache, hipStream_t stream, nfft_plan_params *out, double *best_ms);

/* Destroy a plan.  Host only; frees nothing the caller owns (not the workspace). */
int nfft_plan_destroy(nfft_plan p);

/* Fill *info (host struct). */
int nfft_plan_get_info(nfft_plan p, nfft_plan_info *info);

/* Bytes of device workspace the plan needs (host only). */
int nfft_workspace_bytes(nfft_plan p, size_t *bytes);

/* Attach a caller-owned device workspace of `bytes` bytes, 256-byte aligned.  The
 * plan keeps the pointer until the next nfft_set_workspace or nfft_plan_destroy;
 * the caller keeps the memory alive meanwhile.  Attaching a workspace forgets the
 * nodes (nfft_set_nodes must follow).  NFFT_ERR_WORKSPACE if too small or misaligned. */
int nfft_set_workspace(nfft_plan p, void *ws, size_t bytes);

/* Set the M nodes x [device, M x d doubles] and run the node precomputation (the
 * p.x = A step of Sec. 4.2): per node and dimension u = floor(n_t x) and
 * delta = n_t x - u in FP64 (stencil index set, Sec. 2 eq. (2.13)), then a counting
 * sort of the nodes into bins of grid cells.  The derived data and a copy of x (read
 * by the direct sums) live in the workspace; the caller's x is not referenced after
 * the enqueued work has run.  A node with a non-finite coordinate is placed at grid
 * index 0 with a NaN offset: the forward transform and the gradient are NaN at that node
 * only, while the adjoint (whose grid cells it touches pass through the FFT) is NaN
 * throughout.  nfft_nodes_finite reports whether this happened. */
int nfft_set_nodes(nfft_plan p, const double *x, hipStream_t stream);

/* Whether every coordinate passed to the last nfft_set_nodes was finite: *all_finite = 1
 * if so, 0 if any was NaN or infinite.  Waits for `stream` (the flag is written by the
 * node precomputation enqueued there).  NFFT_ERR_STATE before nfft_set_nodes. */
int nfft_nodes_finite(nfft_plan p, int *all_finite, hipStream_t stream);

/* ---------------------------------------------------------------- transforms */

/* NFFT, Algorithm 2.1: f [device, M] = A fhat for fhat [device, shape N].
 * NFFT_ERR_STATE before nfft_set_nodes. */
int nfft_trafo(nfft_plan p, const void *fhat, void *f, hipStream_t stream);

/* Adjoint NFFT, Algorithm 2.2: hhat [device, shape N] = A^H f for f [device, M]. */
int nfft_adjoint(nfft_plan p, const void *f, void *hhat, hipStream_t stream);

/* Fast summation (the kernel sums named in Sec. 1 as an application of the NFFT): for a
 * kernel given as a trigonometric polynomial with the sign of eq. (1.2),
 * K(z) = sum_{k in I_N} bhat_k e^{-2 pi i k.z},
 *     g_j = sum_l alpha_l K(y_j - x_l),   j < M_y,
 * computed as g = A_y (bhat (.) A_x^H alpha): the adjoint NFFT of alpha at the nodes x of
 * plan px (its last FFT pass multiplies by bhat), then the NFFT at the nodes y of plan py.
 *   px, py     plans with nodes set, equal d, N and dtype (px == py is allowed: y = x).
 *   bhat       [device, shape N] kernel coefficients, centred row-major.
 *   alpha      [device, M_x] coefficients; g [device, M_y] result.
 *   coef_work  [device, shape N] caller-owned scratch of |I_N| complex values.
 * Enqueued on `stream`; NFFT_ERR_STATE before both plans have nodes, NFFT_ERR_ARG on
 * mismatched plans or null pointers.  px's forward grid is overwritten unless it was
 * created with NFFT_KEEP_GRID. */
int nfft_fastsum(nfft_plan px, nfft_plan py, const void *bhat, const void *alpha, void *g, void *coef_work,
                 hipStream_t stream);

/* Direct sums eq. (1.2) / (1.3) on the device, O(M |I_N|) work: f = NDFT(fhat) and
 * hhat = NDFT^H(f).  Phases k.x are formed in FP64 and reduced before the
 * exponential; the sums accumulate in the plan's precision.  Need nfft_set_nodes
 * (they read the nodes' FP64 coordinates kept by it). */
int ndft_trafo(nfft_plan p, const void *fhat, void *f, hipStream_t stream);
int ndft_adjoint(nfft_plan p, const void *f, void *hhat, hipStream_t stream);

/* Gradient of the NFFT output with respect to the nodes, contracted with an upstream
 * vector v [device, M complex]:
 *     grad_x[j][t] = Re( conj(v_j) * d f_j / d x_{j,t} ),
 * where f = nfft_trafo(fhat) and the derivative is taken through the window of
 * Algorithm 2.1 step 3 (d/dx_t phi(n_t x_t - l_t) = n_t phi'(.)).  grad_x [device,
 * M x d] is float for NFFT_C64 plans and double for NFFT_C128 plans.  Needs
 * NFFT_KEEP_GRID and a preceding nfft_trafo on the same nodes (its grid is used);
 * else NFFT_ERR_STATE. */
int nfft_grad_x(nfft_plan p, const void *v, void *grad_x, hipStream_t stream);

/* ---------------------------------------------------------------- single steps */
/* The transforms above are compositions of these steps; they are exposed so each step
 * can be checked and timed on its own.  g is a caller grid [device, shape n].
 *
 * Grid scaling: the library evaluates the window divided by lambda_t in every dimension
 * (Kaiser-Bessel: lambda_t = e^{b_t m}, b_t = pi (2 - N_t/n_t), which keeps FP32 window
 * values accurate; Gaussian: lambda_t = (pi b_t)^{-1/2}, its peak) and carries lambda_t in
 * the deconvolution.  The grids these steps exchange are therefore the grids of
 * Algorithms 2.1 / 2.2 multiplied by S = prod_t lambda_t (forward, nfft_step_grid) or
 * divided by S (adjoint, nfft_step_spread), and
 * nfft_step_interp / nfft_step_coeffs expect grids scaled the same way.  S is reported
 * as nfft_plan_info.grid_scale.  Composed, the steps give exactly nfft_trafo and
 * nfft_adjoint. */

/* Steps 1-2 of Algorithm 2.1: g = S F D fhat (deconvolution with zero padding onto I_n,
 * eq. (2.9), then the d-variate FFT with sign -, unnormalised). */
int nfft_step_grid(nfft_plan p, const void *fhat, void *g, hipStream_t stream);

/* Step 3 of Algorithm 2.1: f_j = S^{-1} sum over the 2m+2 stencil points per dimension
 * of g_l * prod_t phi_t(n_t x_{j,t} - l_t) (eq. (2.12)-(2.13)). */
int nfft_step_interp(nfft_plan p, const void *g, void *f, hipStream_t stream);

/* Step 1 of Algorithm 2.2: g_l = S^{-1} sum_j f_j prod_t phi_t(n_t x_{j,t} - l_t) (the
 * transposed index set of Sec. 2).  Every cell of g is written. */
int nfft_step_spread(nfft_plan p, const void *f, void *g, hipStream_t stream);

/* Steps 2-3 of Algorithm 2.2: hhat = S D^H F^H g (FFT with sign +, unnormalised, only
 * frequencies in I_N kept, then the deconvolution). */
int nfft_step_coeffs(nfft_plan p, const void *g, void *hhat, hipStream_t stream);

/* ---------------------------------------------------------------- timing */

/* Kernel timing with HIP events recorded around every kernel the plan launches, on
 * the stream of the launching call.  Enable before the calls to be timed; read after
 * synchronising that stream.  names[i] / total_ms[i] / launches[i] are filled for up
 * to `cap` kernels (host arrays); *count receives the number of distinct kernels.
 * Reading resets the counters. */
int nfft_profile_enable(nfft_plan p, int on);
int nfft_profile_read(nfft_plan p, const char **names, double *total_ms, int64_t *launches, int cap,
                      int *count);

/* ---------------------------------------------------------------- batches */

/* A batch runs many independent plans, each with its own nodes (set through
 * nfft_set_nodes on its own workspace), with one launch per step kind instead of one per
 * plan and step.  Sec. 3 measures FFT plans once and keeps the result (FFTW's MEASURE
 * flag and wisdom); the batch autotuner does the same for its launch shapes.
 *
 * nfft_batch_create
 *   plans      [host] `count` >= 1 distinct plans, all NFFT_C64 or all NFFT_C128, each
 *              with its workspace attached; the workspaces must stay attached as they are
 *              (a later nfft_set_workspace on a member makes batch calls fail with
 *              NFFT_ERR_STATE).  The batch does not own the plans: destroy it first.
 *   tune_cache [host] path of a text file of tuned launch parameters, or NULL.  Read by
 *              nfft_batch_set_workspace, rewritten by nfft_batch_autotune.
 *   Plans are grouped by dimension, compiled stencil width and precision, and each group
 *   is cut into launch groups of at most 64 plans, largest M first.  Host-only call.
 * nfft_batch_workspace_bytes / nfft_batch_set_workspace attach the batch's own device
 *   memory (256-byte aligned; per-plan descriptor tables and work-queue counters), copy
 *   the descriptors to it and synchronise the device.
 * nfft_batch_trafo / nfft_batch_adjoint take host arrays of `count` device pointers, in
 *   the order of `plans`, shaped as for nfft_trafo / nfft_adjoint of each plan; every
 *   plan needs its nodes set.  Enqueued on `stream`; results equal the per-plan calls.
 *   A batch is used by one stream at a time.
 * nfft_batch_autotune times every candidate launch shape of each step kind on `stream`
 *   (with zero stand-in inputs in device memory it allocates and frees), keeps the
 *   fastest, synchronises `stream` and, with a cache file, rewrites the file.  Returns
 *   NFFT_ERR_ARG when the cache file cannot be written.
 * nfft_batch_get_params / nfft_batch_set_params read or set the NFFT_BATCH_NPARAMS launch
 *   parameters of launch group `group` (0 <= group < info.groups):
 *     [0] pack_fwd, [2] pack_adj   lines per FFT workgroup as a multiple (1, 2, 4, ...) of
 *                                  the plan's own packing (capped per plan);
 *     [1] k_fwd, [3] k_adj, [4] k_interp, [5] k_spread, [6] k_fold
 *                                  grid of k x (compute units) workgroups, 0 for one
 *                                  workgroup per work item;
 *     [7] reserved (0).
 *   plan_count (may be NULL) receives the number of plans of the launch group. */
#define NFFT_BATCH_NPARAMS 8

typedef struct {
    int count;              /* plans */
    int groups;             /* launch groups */
    int tuned;              /* 1 when every launch group has tuned (or cached) parameters */
    size_t workspace_bytes; /* device bytes of the batch */
} nfft_batch_info;

int nfft_batch_create(nfft_batch *out, int count, const nfft_plan *plans, const char *tune_cache);
int nfft_batch_get_info(nfft_batch b, nfft_batch_info *info);
int nfft_batch_workspace_bytes(nfft_batch b, size_t *bytes);
int nfft_batch_set_workspace(nfft_batch b, void *ws, size_t bytes);
int nfft_batch_autotune(nfft_batch b, hipStream_t stream);
int nfft_batch_get_params(nfft_batch b, int group, int *params, int *plan_count);
int nfft_batch_set_params(nfft_batch b, int group, const int *params);
int nfft_batch_trafo(nfft_batch b, const void *const *fhat, void *const *f, hipStream_t stream);

/* Allocation-free batched forward transform, for callers that cannot allocate device memory
 * (code under stream or graph capture, serving loops, harnesses that forbid allocation).
 * Same arguments, results and preconditions (every plan's nodes set, its workspace unchanged)
 * as nfft_batch_trafo, but the batch needs no workspace of its own: its per-plan descriptor
 * tables and work queues go to a 1 MiB device array held by the library (one per device, kept
 * until the process ends).  No call allocates or frees memory; each call copies the
 * descriptors into the array and clears the queues on `stream`.
 *   Returns NFFT_ERR_WORKSPACE when the batch's tables need more than 1 MiB (about 600
 *   plans), NFFT_ERR_STATE as nfft_batch_trafo, NFFT_ERR_HIP for a failed copy or launch.
 *   Calls that overlap on one device share the array and race: serialise them (one stream,
 *   or events).  The plans' own workspaces are used as by nfft_batch_trafo. */
int nfft_batch_trafo_noalloc(nfft_batch b, const void *const *fhat, void *const *f, hipStream_t stream);
int nfft_batch_adjoint(nfft_batch b, const void *const *f, void *const *hhat, hipStream_t stream);
int nfft_batch_destroy(nfft_batch b);

/* ---------------------------------------------------------------- NNFFT */

/* NNFFT, the transform with nonequispaced nodes in both domains that Sec. 1 names as a
 * generalisation of the NFFT: for K frequencies v_k with v_{k,t} in [-N_t/2, N_t/2) and M
 * nodes x_j in [-1/2, 1/2)^d,
 *     nnfft_trafo:    f_j    = sum_k fhat_k e^{-2 pi i v_k . x_j},   j < M,
 *     nnfft_adjoint:  hhat_k = sum_j f_j    e^{+2 pi i v_k . x_j},   k < K.
 * Computed with two inner plans sharing the window and m: plan A spreads the frequencies
 * onto an equispaced frequency grid of N2_t points (a power of two, see sigma; plan A has
 * N_A,t coefficients, the smallest even count with N_t N2_t / N_A,t <= N2_t - 2m - 4, i.e.
 * oversampling sigma1_t = N2_t / N_A,t with room for the stencils, and nodes v_k / N_A),
 * plan B is an NFFT with N2 coefficients at
 * the nodes z_j = x_j N_A / N2, and each output is multiplied by the deconvolution factor
 * of plan A's window taken at z_j (eq. (2.9) at a real frequency).  The adjoint runs the
 * transposed steps in reverse.  Accuracy is that of two NFFTs with oversampling about
 * sigma and window size m.
 *
 * nnfft_plan_create
 *   N      [host] d even bandwidths >= 2 of the frequency domain.
 *   K, M   numbers of frequencies and nodes, >= 1.
 *   sigma  frequency-grid oversampling in (1, 16]: N2_t is the smallest power of two
 *          >= ceil(sigma N_t) + 2m + 4.  0 selects it automatically: the smallest power
 *          of two >= 2 N_t, doubled while sigma1_t would be below 1.5.
 *   m      window size (0: 8), as for nfft_plan_create.
 *   flags  one of the window flags, and NFFT_SORT_NODES, or 0.
 *   NFFT_ERR_UNSUPPORTED when an inner plan is (N2_t > 2048, so that plan B's FFT length
 *   2 N2_t stays within 4096).  Host only.
 * nnfft_workspace_bytes / nnfft_set_workspace: one caller-owned device workspace
 *   (256-byte aligned) holding both inner plans' workspaces, the scaled nodes, the
 *   per-node factors and the frequency grid; attaching it forgets the nodes.
 * nnfft_set_nodes
 *   x      [device, M x d doubles] nodes; v [device, K x d doubles] frequencies.  Neither
 *          is referenced after the enqueued work has run.  Frequencies outside
 *          [-N_t/2, N_t/2) give wrong values (their spreading wraps around the frequency
 *          grid); a non-finite node or frequency gives NaN outputs as for nfft_set_nodes.
 * nnfft_trafo / nnfft_adjoint
 *   fhat [device, K], f [device, M]; complex of the plan's precision.  Enqueued on
 *   `stream`; NFFT_ERR_STATE before nnfft_set_nodes. */
typedef struct nnfft_plan_s *nnfft_plan;

typedef struct {
    int d, m;
    int64_t N[3];           /* frequency bandwidths                               */
    int64_t K, M;           /* frequencies, nodes                                 */
    int64_t N2[3];          /* frequency grid points = plan B's bandwidths         */
    int64_t NA[3];          /* plan A's coefficient counts                         */
    double sigma1[3];       /* N2 / NA: plan A's oversampling                      */
    size_t workspace_bytes; /* bytes nnfft_set_workspace needs                     */
    int window;             /* as nfft_plan_info.window                            */
} nnfft_plan_info;

int nnfft_plan_create(nnfft_plan *out, int d, const int64_t *N, int64_t K, int64_t M, double sigma, int m,
                      nfft_dtype dtype, uint32_t flags);
int nnfft_plan_destroy(nnfft_plan p);
int nnfft_plan_get_info(nnfft_plan p, nnfft_plan_info *info);
int nnfft_workspace_bytes(nnfft_plan p, size_t *bytes);
int nnfft_set_workspace(nnfft_plan p, void *ws, size_t bytes);
int nnfft_set_nodes(nnfft_plan p, const double *x, const double *v, hipStream_t stream);
int nnfft_trafo(nnfft_plan p, const void *fhat, void *f, hipStream_t stream);
int nnfft_adjoint(nnfft_plan p, const void *f, void *hhat, hipStream_t stream);

/* Human-readable name of a status code (static string). */
const char *nfft_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* NFFT_MI355X_H */
