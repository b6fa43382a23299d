/*
 * fastsum.h -- C ABI of the MI355X (gfx950) QMC-slicing fast kernel summation
 * library (libfastsum.so).
 *
 * Problem (Sec. 1, eq. kernel_sum): for sources x_n in R^d with real weights
 * w_n and targets y_m in R^d compute
 *
 *     s_m = sum_n w_n F(||x_n - y_m||),            m = 1..M,
 *
 * for a radial kernel F.  The library evaluates the slicing approximation
 * (Sec. 2.1, eq. kernel_sum_sliced)
 *
 *     s_m ~ (1/P) sum_p sum_n w_n f(|<xi_p, x_n - y_m>|)
 *
 * with caller-supplied unit directions xi_1..xi_P (QMC designs, Sec. 3) and
 * the 1-D basis function f of F (App. A).  Each 1-D sum is done by fast
 * Fourier summation (App. I, Steps 1-3): the projections are rescaled by
 * tau = min{T/R, 1/(2 g_max)}, the rescaled 1-D kernel is replaced by its
 * Fourier series truncated to |k| <= N_ft/2 (coefficients computed in FP64 on
 * the host), and the two non-uniform transforms of eq. (1d_sum_fourier) are
 * done by window spreading on an oversampled grid, an FFT, a coefficient
 * multiply, an inverse FFT and window interpolation.
 *
 * Conventions for every call:
 *  - Device pointers point to memory of the device that was current when the
 *    plan was created; float arrays are float32, row-major and contiguous.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Execution calls
 *    only enqueue work on it; they never allocate, free or synchronise.
 *  - Argument errors are reported synchronously by the return value and leave
 *    every output untouched.  No call aborts or throws across the ABI.
 *  - A plan is used by one stream at a time; distinct plans are independent.
 */
#ifndef FASTSUM_H
#define FASTSUM_H

#include <stdint.h>

#if defined(__GNUC__)
#define FASTSUM_API __attribute__((visibility("default")))
#else
#define FASTSUM_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FASTSUM_OK = 0,
    FASTSUM_EINVAL = 1,       /* invalid argument (null pointer, size, parameter) */
    FASTSUM_ENOMEM = 2,       /* device or host allocation failed               */
    FASTSUM_EDEVICE = 3,      /* a HIP runtime call failed                      */
    FASTSUM_ERANGE = 4,       /* a projected point lay outside the bound R       */
    FASTSUM_EUNSUPPORTED = 5, /* valid request this build does not implement     */
    FASTSUM_ESTATE = 6        /* call order violated (e.g. grad before exec)     */
} fastsum_status;

/* Kernels of Table 'tab:kernels' (App. A). */
typedef enum {
    FASTSUM_GAUSS = 0,   /* F(r) = exp(-r^2 / (2 scale^2))                       */
    FASTSUM_LAPLACE = 1, /* F(r) = exp(-r / scale)   (alpha = 1/scale)            */
    FASTSUM_ENERGY = 2,  /* F(r) = -r  (negative distance, Riesz r = 1)           */
    /* Matern of order nu, width beta = scale:                                  */
    /*   F(r) = 2^{1-nu}/Gamma(nu) z^nu K_nu(z),  z = sqrt(2 nu) r / beta,       */
    /* coefficients from the column-3 transform of Table 'tab:kernels'; App. I  */
    /* defaults T = 0.2, g_max = 5 beta (Sec. 4.1 uses nu = 3/2 and 7/2).       */
    FASTSUM_MATERN32 = 3,   /* nu = 3/2: F = (1 + z) e^{-z}                     */
    FASTSUM_MATERN52 = 4,   /* nu = 5/2: F = (1 + z + z^2/3) e^{-z}             */
    FASTSUM_MATERN72 = 5    /* nu = 7/2: F = (1 + z + 2z^2/5 + z^3/15) e^{-z}   */
} fastsum_kernel;

/* Arithmetic of the projection X . Xi (the only dense contraction). */
typedef enum {
    FASTSUM_PROJ_FP32 = 0, /* FP32 inputs, FP32 MFMA, FP32 accumulate            */
    FASTSUM_PROJ_BF16 = 1  /* inputs rounded to BF16 (nearest-even), BF16 MFMA,  */
                           /* FP32 accumulate; spread/FFT/gather stay FP32      */
} fastsum_precision;

/* fastsum_params.flags */
/* Results are bitwise reproducible without a flag: spreading adds integers
 * (fixed point per slice of 4096 sources) and every floating-point sum runs
 * in a fixed order.  Kernel sums are translation invariant, so a caller who
 * wants a tighter bound R (App. I Step 1) subtracts a common point from x
 * and y before the call and passes the centred bound. */
#define FASTSUM_FLAG_GRAD 1u /* keep what fastsum_grad needs (derivative grids) */
/* Write the projections tau <xi_p, x_n> to device memory (needed for
 * fastsum_debug_read of which = 0, 1).  Without it, plans with d <= 64,
 * FP32 projections and 16 * grid_nr <= 16384 compute the projections inside
 * the spreading and gathering kernels and never store them
 * (fastsum_plan_info.fused = 1); with FASTSUM_FLAG_GRAD they also form the
 * adjoint that way. */
#define FASTSUM_FLAG_MATERIALIZE 2u
/* Energy kernel only: compute every 1-D sum exactly by sorting instead of by
 * Fourier summation (the 1-D method the paper takes for the negative
 * distance kernel, Sec. 4.3).  Per direction the projected sources and targets
 * are sorted together (segmented radix sort) and, in sorted order, FP64
 * prefix sums W_< of w_n and S_< of w_n x~_n over the sources give
 * sum_n w_n |x~_n - y~| = y~ (2 W_< - W) - (2 S_< - S) at each target; each
 * direction's sum is stored in FP32 and their mean taken in FP64.  The only
 * approximation left is the slicing (eq. (3)); n_ft, window_w and
 * oversample are validated but unused.  Stores the projections.  With
 * FASTSUM_FLAG_GRAD, fastsum_grad_xyw is exact too: one scan of the rows the
 * exec sorted gives per direction the weight sums over strictly smaller and
 * strictly larger keys (entries of equal key form runs, handled as one),
 * i.e. the derivative sum_n w_n sign(y~ - x~_n) with sign(0) = 0 where
 * projections coincide, and the transposed sums for grad_w.  The plan
 * needs n_max, m_max <= 2^24 and P * L < 2^32 with
 * L = round_up(n_max, 64) + round_up(m_max, 64),
 * and about 4 P L (keys) + 4 P L (sorted keys) + 4 P L (positions) + 8 P L
 * (sort workspace) + 6 P ldm (per-direction sums and their target offsets)
 * + 384 ldm bytes of device memory, ldm = round_up(max(n_max, m_max), 64),
 * plus 20 P ldm with FASTSUM_FLAG_GRAD. */
#define FASTSUM_FLAG_SORTED 4u

/*
 * Plan parameters.  Zero in an optional field selects the default.
 *   d            dimension (1 <= d <= 4096)
 *   P            number of directions (1 <= P <= 65536)
 *   n_ft         number of Fourier modes N_ft, even, 16..1024; modes |k| <= N_ft/2
 *                are kept, with half weight at |k| = N_ft/2 (App. I Step 3)
 *   window_w     window width in grid cells: 4, 6 or 8; default 6 for Laplace,
 *                4 otherwise
 *   oversample   grid size n = oversample * n_ft, 2 (default) or 4; n <= 2048
 *   kernel       fastsum_kernel
 *   proj         fastsum_precision
 *   flags        FASTSUM_FLAG_*
 *   scale        sigma (Gauss) or 1/alpha (Laplace), > 0; ignored for ENERGY
 *   T            rescaling threshold (App. I Step 1); default 0.3 Gauss,
 *                0.1 Laplace, 0.45 energy; must satisfy 0 < T < 0.5
 *   gmax_factor  g_max = gmax_factor * scale (App. I Step 1); default 5
 *   R            bound R >= max_n ||x_n|| + max_m ||y_m|| (App. J,
 *                eq. radius_xy), > 0.  Every exec checks it on the device
 *                (fastsum_check reports a violation); fastsum_bound computes
 *                the right-hand side.
 */
typedef struct {
    int32_t d;
    int32_t P;
    int32_t n_ft;
    int32_t window_w;
    int32_t oversample;
    int32_t kernel;
    int32_t proj;
    uint32_t flags;
    double scale;
    double T;
    double gmax_factor;
    double R;
} fastsum_params;

/* Read-only facts about a plan (for tests and diagnostics). */
typedef struct {
    double tau;          /* rescaling factor (App. I Step 1)                  */
    double beta;         /* shape of the exponential-of-semicircle window     */
    int32_t n_grid;      /* oversampled grid size n                           */
    int32_t window_w;    /* window width W in grid cells                      */
    int32_t poly_degree; /* degree of the per-cell window polynomials         */
    int32_t n_ft;
    int64_t n_max, m_max;
    int32_t proj;
    uint32_t flags;
    int32_t grid_lo;     /* first grid cell that points inside the bound touch */
    int32_t grid_nr;     /* number of such cells (stored grids hold these)    */
    int32_t last_spread_chunks;  /* source chunks of the last exec's spread   */
    int32_t last_gather_groups;  /* direction groups of the last exec's gather */
    int32_t fused;       /* 1: projections are computed inside spread/gather  */
} fastsum_plan_info;

typedef struct fastsum_plan_s* fastsum_plan;

/*
 * Create a plan: FP64 host precompute of tau, the Fourier coefficients c_k
 * (App. I Step 2; App. J for the energy kernel), the window tables and the
 * coefficient multipliers; upload of tau*Xi; allocation of the workspace for
 * up to n_max sources and m_max targets.
 *   prm     parameters (copied)
 *   xi      HOST pointer, d x P row-major: column p (elements xi[i*P + p]) is
 *           direction xi_p; columns should have unit norm (not renormalised)
 *   n_max, m_max  capacity, >= 1
 *   stream  stream used for the uploads (the call returns after they finish)
 *   out     receives the plan; untouched on error
 * Errors: EINVAL (bad parameter or pointer), ENOMEM, EDEVICE.
 */
FASTSUM_API fastsum_status fastsum_plan_create(const fastsum_params* prm, const float* xi,
                                   int64_t n_max, int64_t m_max, void* stream,
                                   fastsum_plan* out);

/* Release every resource of a plan (synchronises the device).  NULL is a no-op. */
FASTSUM_API void fastsum_destroy(fastsum_plan plan);

/*
 * s_m ~ sum_n w_n F(||x_n - y_m||) by Fourier slicing.
 *   x  device, N x d;  w  device, N;  y  device, M x d, may equal x with
 *   M <= N: the targets are then the first M sources and their projections
 *   are computed once (FASTSUM_EINVAL for y == x with M > N);
 *   s  device, M (written).  1 <= N <= n_max, 1 <= M <= m_max.
 * Asynchronous on `stream`.  The projections (fused plans: the split
 * operand tiles of x and y) and the grids of the call are kept in the plan
 * for a following fastsum_grad.  If a projected point exceeds the bound
 * implied by R a device flag is set (see fastsum_check).
 */
FASTSUM_API fastsum_status fastsum_exec(fastsum_plan plan, const float* x, int64_t N,
                            const float* w, const float* y, int64_t M,
                            float* s, void* stream);

/*
 * Adjoint of the last fastsum_exec (which must have used a plan with
 * FASTSUM_FLAG_GRAD), for a cotangent v = grad_s (device, M):
 *   grad_y (device, M x d, or NULL): grad_y[m] = v_m * d s_m / d y_m, where
 *     d s_m/d y_m = (tau/P) sum_p xi_p t'_{m,p} and t'_{m,p} is the derivative
 *     of the rescaled 1-D Fourier sum at y~_{m,p} (spectral multiplier 2 pi i k).
 *   grad_w (device, N, or NULL): grad_w[n] = sum_m v_m d s_m / d w_n, the same
 *     sliced Fourier sum with sources and targets exchanged.
 * Fused plans interpolate t' at projections formed in the kernel and
 * back-project them on the matrix cores, with per-direction-range FP32
 * partial sums reduced in a second launch; stored plans write t' (P x M)
 * and back-project it.  The inputs of the last exec must still be valid.
 * Asynchronous.  Errors: ESTATE (no exec yet / plan without GRAD), EINVAL.
 */
FASTSUM_API fastsum_status fastsum_grad(fastsum_plan plan, const float* grad_s,
                            float* grad_y, float* grad_w, void* stream);

/*
 * As fastsum_grad, with the gradient in the sources as well:
 *   grad_x (device, N x d, or NULL): grad_x[n] = sum_m v_m d s_m / d x_n
 *     = w_n du/dx(x_n), u(x) = sum_m v_m K(x, y_m) the transposed sliced sum
 *     (sources y with weights v, targets x) whose derivative grids are
 *     interpolated at the sources and back-projected as for grad_y.
 * grad_w and grad_x share that transposed spreading and FFT.  Sorted plans
 * (FASTSUM_FLAG_SORTED) take the exact derivatives instead: t' is
 * -(c_d/tau) sum_n w_n sign(y~ - x~_n) from the rows the last exec sorted
 * (sign(0) = 0), the source side likewise with v, and grad_w the transposed
 * sorted sums; only the requested outputs are computed.  The weights w of
 * the last exec must still be valid.  Asynchronous.
 * Errors: ESTATE (no exec yet / plan without GRAD), EINVAL.
 */
FASTSUM_API fastsum_status fastsum_grad_xyw(fastsum_plan plan, const float* grad_s,
                                            float* grad_x, float* grad_y, float* grad_w,
                                            void* stream);

/*
 * Synchronise the plan's last stream and report device-side conditions:
 * returns ERANGE if an exec since the previous check violated the plan's
 * bound (results are then unreliable), OK otherwise; clears the flag.  Two
 * tests run in every exec, each with a slack of 1e-5 relative:
 *  - the bound of App. J, eq. radius_xy:
 *    (max_n |x_n| + max_m |y_m|) max_p |xi_p| <= R, from the row norms
 *    taken while the points are read; it keeps every difference
 *    tau <xi_p, x_n - y_m> inside the half period where the periodic
 *    rescaled kernel equals the true one;
 *  - per point: plans that store projections test every projection against
 *    tau*R, fused plans test |x| max_p|xi_p| <= R for every point; this keeps
 *    every window inside the stored grid cells.
 * Non-finite coordinates fail both.
 */
FASTSUM_API fastsum_status fastsum_check(fastsum_plan plan);

/*
 * The right-hand side of App. J, eq. radius_xy, on the device:
 *   *bound_out = max_n ||x_n|| + max_m ||y_m||
 * (Euclidean norms about the origin, FP32 sums of squares, returned as a
 * double), for x (device, N x d) and y (device, M x d; may equal x).  A
 * plan created with R >= *bound_out * (1 + 1e-5) passes the bound test of
 * fastsum_check for these points.  Allocates 8 bytes of device memory for
 * the call and synchronises `stream`.
 * Errors: EINVAL, ENOMEM, EDEVICE; ERANGE (with *bound_out = inf or NaN)
 * when a coordinate is not finite.
 */
FASTSUM_API fastsum_status fastsum_bound(const float* x, int64_t N, const float* y, int64_t M,
                                         int32_t d, void* stream, double* bound_out);

/* Copy plan facts into *info.  EINVAL on NULL. */
FASTSUM_API fastsum_status fastsum_get_info(fastsum_plan plan, fastsum_plan_info* info);

/*
 * Host-only (no device is touched): the FP64 quantities a plan would use.
 *   tau_out  receives tau (may be NULL)
 *   ck_out   receives c_0..c_K, K = n_ft/2 (K+1 doubles; may be NULL)
 *   phihat_out receives the window transform at k = 0..n/2 (n/2+1 doubles,
 *            n = oversample*n_ft; may be NULL)
 * Errors: EINVAL.
 */
FASTSUM_API fastsum_status fastsum_host_tables(const fastsum_params* prm, double* tau_out,
                                   double* ck_out, double* phihat_out);

/*
 * Diagnostics: synchronously copy an internal buffer of the last exec to host
 * memory.  which = 0: projections of x (P x N, row p = tau <xi_p, x_n>);
 * 1: projections of y (P x M); 2: convolved grids (P x grid_nr, cells
 * grid_lo .. grid_lo+grid_nr-1 of each direction's grid of n cells, which
 * holds the grid at position (j - n/2)/n).  count must equal the buffer's
 * element count.  Errors: EINVAL, ESTATE (no exec yet, or which = 0, 1 on a
 * fused plan, which stores no projections), EDEVICE.
 */
FASTSUM_API fastsum_status fastsum_debug_read(fastsum_plan plan, int32_t which,
                                  float* host_out, int64_t count);

/*
 * Launch shape of later execs (results do not depend on it beyond FP32
 * rounding of the per-chunk partial grids):
 *   chunk_len   sources per spreading workgroup, a multiple of 16 (plans
 *               that store projections round it up to a multiple of 4096),
 *               or 0 for the plan's rule; raised if N / chunk_len would
 *               exceed the workspace sized at plan time
 *   dir_range   directions per gathering workgroup of a fused plan, a
 *               multiple of 16, or 0 for the plan's rule
 * Errors: EINVAL (NULL plan, negative or misaligned values).
 */
FASTSUM_API fastsum_status fastsum_set_launch(fastsum_plan plan, int64_t chunk_len,
                                              int32_t dir_range);

/*
 * Batched form: many independent kernel-sum problems that share the kernel
 * type, P, the window and T, run by ONE launch per phase (projection or
 * operand split, chunk scaling, spreading, FFT convolution, gather,
 * reduction) whose workgroups walk a task list of tiles drawn from every
 * problem.  The six launches are captured into a HIP graph on a private
 * stream and the graph is replayed while pointers and sizes repeat.
 *
 * When every problem has d <= 64 (and FASTSUM_FLAG_MATERIALIZE is not
 * given) the batch runs the fused kernels of the single plans: points are
 * split into f16 operand tiles and the projections are computed inside the
 * spreading and gathering workgroups, one workgroup per task (16 directions
 * x a source chunk, or 1024 targets x a direction range), tasks ordered
 * largest first.  Otherwise the projections are stored (P x N per problem)
 * by an FP32 MFMA GEMM phase.
 *
 * Per problem at plan time: d_i, n_ft_i, scale_i, R_i, directions xi_i
 * (HOST, d_i x P row-major, as in fastsum_plan_create) and capacities.
 */
typedef struct {
    int32_t d;
    int32_t n_ft;
    double scale;
    double R;
    const float* xi;     /* host, d x P */
    int64_t n_max, m_max;
} fastsum_problem_desc;

/* Per problem at exec time: device pointers and sizes, 1 <= N <= n_max,
 * 1 <= M <= m_max; y may equal x (then N must equal M). */
typedef struct {
    const float* x;      /* N x d */
    const float* w;      /* N     */
    const float* y;      /* M x d */
    float* s;            /* M, written */
    int64_t N, M;
} fastsum_problem_io;

/* Launch-shape knobs (chosen by an autotuner); 0 selects the default. */
typedef struct {
    int32_t blocks_per_cu;  /* persistent workgroups per compute unit (default 4;  */
                            /* fused batches: scaling, FFT and reduction phases)   */
    int32_t spread_chunk;   /* sources per spread tile, multiple of 4096 (fused    */
                            /* default 16384)                                      */
    int32_t gather_group;   /* directions per gather tile, multiple of 8 (fused:   */
                            /* rounded up to 16, default all P)                    */
    int32_t use_graph;      /* 0/1: capture and replay a HIP graph (default); -1:  */
                            /* launch the phases directly on the caller's stream  */
} fastsum_batch_tuning;

typedef struct fastsum_batch_s* fastsum_batch;

/*
 * common supplies kernel, P, window_w, oversample, T and gmax_factor; proj
 * must be FASTSUM_PROJ_FP32 and flags 0 or FASTSUM_FLAG_MATERIALIZE (stored
 * projections; no adjoint in the batched form).
 * d, n_ft, scale and R of common are ignored.  tuning may be NULL.
 * Errors: EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED (BF16, GRAD or another flag).
 */
FASTSUM_API fastsum_status fastsum_batch_create(const fastsum_params* common,
                                                const fastsum_problem_desc* probs,
                                                int32_t n_problems,
                                                const fastsum_batch_tuning* tuning,
                                                void* stream, fastsum_batch* out);

/* Replace the launch-shape knobs (drops the captured graph). */
FASTSUM_API fastsum_status fastsum_batch_set_tuning(fastsum_batch batch,
                                                    const fastsum_batch_tuning* tuning);

/*
 * Run every problem: s_i ~ sum_n w_{i,n} F(||x_{i,n} - y_{i,m}||).  io has
 * n_problems entries in creation order.  When pointers or sizes differ from
 * the previous call the task lists are rebuilt, uploaded and the graph is
 * re-captured (this path synchronises `stream` once); otherwise the graph is
 * replayed on `stream` asynchronously.  Errors: EINVAL, EDEVICE.
 */
FASTSUM_API fastsum_status fastsum_batch_exec(fastsum_batch batch,
                                              const fastsum_problem_io* io,
                                              int32_t n_problems, void* stream);

/* As fastsum_check, for every problem of the batch. */
FASTSUM_API fastsum_status fastsum_batch_check(fastsum_batch batch);

FASTSUM_API void fastsum_batch_destroy(fastsum_batch batch);

/*
 * Distance QMC directions (App. H): iters projected Adam steps that raise
 * sum_{p,q} |xi_p - xi_q| + |xi_p + xi_q| (the symmetrised distance energy
 * of eq. distance-sym, lowered), each step on the tangent part of the
 * gradient followed by renormalising the rows; the step size falls
 * linearly from lr to lr/10 (Adam moments 0.9, 0.999).
 *   xi      device, P x d row-major (row p is direction p; the transpose of
 *           the d x P layout fastsum_plan_create takes): unit rows in, the
 *           design out (in place)
 *   d       1..64;  P >= 1;  iters >= 0;  lr > 0
 *   stream  the steps run on it; the call returns after they finish
 * Allocates its workspace for the call (8 P d bytes plus partial sums of
 * at most 260 P ceil(2048 / ceil(P/64)) bytes).  FP32 arithmetic; the
 * randomisation of App. E is fastsum_rotate_directions.
 * Errors: EINVAL, ENOMEM, EDEVICE.
 */
FASTSUM_API fastsum_status fastsum_distance_qmc(int32_t d, int32_t P, int32_t iters, double lr,
                                                float* xi, void* stream);

/*
 * Randomised directions (App. E): a QMC design rotated by an orthogonal
 * matrix Q drawn from the Haar measure keeps every direction uniformly
 * distributed on the sphere, so the sliced estimator stays unbiased.  Row p
 * of xi becomes Q xi_p / |Q xi_p|, (Q xi_p)_i = sum_j Q_ij (xi_p)_j (the
 * renormalisation only removes rounding when Q is orthogonal).
 *   q       device, d x d row-major FP32, caller-owned; the random draw is
 *           the caller's (passed in as an input)
 *   xi      device, P x d row-major (the layout of fastsum_distance_qmc),
 *           replaced in place
 *   d       1..64;  P >= 1
 *   stream  the kernel runs on it; the call returns after it finishes
 * FP32 products and sums.  A row that Q maps to zero becomes NaN.
 * Errors: EINVAL (arguments), EDEVICE.
 */
FASTSUM_API fastsum_status fastsum_rotate_directions(int32_t d, int32_t P, const float* q,
                                                     float* xi, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same
 * iteration as fastsum_distance_qmc, same arguments and the same result bit
 * for bit, with its workspace (Adam moments and partial gradient sums) in a
 * static device array of 5 Mi floats (20 MiB) that the library holds on
 * each GPU it runs on until the process ends.  It calls no allocator and
 * does not synchronise: the steps are only enqueued on `stream`.
 * Requires 2 P d + the partial sums (at most 65 P ceil(2048 / ceil(P/64))
 * floats) <= 5 Mi floats, which holds for every P <= 2048 at any d <= 64;
 * larger requests return EINVAL.  Calls on one GPU share the array, so
 * calls that overlap in time on one GPU (other streams, other threads)
 * race; serialise them.  Nothing needs clearing between calls.
 * Errors: EINVAL (arguments, or the workspace would exceed the array),
 * EDEVICE.
 */
FASTSUM_API fastsum_status fastsum_distance_qmc_noalloc(int32_t d, int32_t P, int32_t iters,
                                                        double lr, float* xi, void* stream);

/*
 * Momentum step of the MMD gradient flow (App. MMD flows), in place:
 *   v <- g + m v,   x <- x - step v,
 * for N particles of d coordinates (device, row-major float32; g the
 * gradient of the MMD functional at x, as fastsum_grad returns it).  z
 * (device, N x d, or NULL, or equal to x) receives a copy of the new x:
 * the particles' rows among the flow's sources.  *max_norm2 (device, one
 * float, caller-owned) is set to max_n ||x_n||^2 of the new particles, the
 * first term of the next step's bound (App. J, eq. radius_xy).  One pass,
 * FP32 (each update one fused multiply-add).  Asynchronous on `stream`.
 * Errors: EINVAL (arguments), EDEVICE.
 */
FASTSUM_API fastsum_status fastsum_flow_update(int64_t N, int32_t d, float momentum, float step,
                                               const float* g, float* v, float* x, float* z,
                                               float* max_norm2, void* stream);

/*
 * Host-only N_ft selection rule: the smallest candidate N_ft whose discarded
 * Fourier mass sum_{|k| > N_ft/2} |c_k| is at most tol * sum_k |c_k| (FP64,
 * c_k of prm's kernel, d, scale, T, R; tails summed to |k| = 4096).  Falls
 * back to the largest candidate.  Errors: EINVAL.
 */
FASTSUM_API fastsum_status fastsum_choose_nft(const fastsum_params* prm,
                                              const int32_t* candidates,
                                              int32_t n_candidates, double tol,
                                              int32_t* chosen);

/*
 * Per-phase timing.  While enabled, every exec/grad records a pair of HIP
 * events on its stream around each kernel launch of a phase.
 * fastsum_profile_read synchronises those events, adds their elapsed times
 * per phase into ms_total[FASTSUM_PHASE_COUNT] and counts launches into
 * launches[FASTSUM_PHASE_COUNT] (both may be NULL), then forgets them.
 * Errors: EINVAL, EDEVICE.
 */
typedef enum {
    FASTSUM_PHASE_PROJECT = 0,     /* x~ = tau X Xi (and y~)                */
    FASTSUM_PHASE_SPREAD = 1,      /* window spreading onto the grids       */
    FASTSUM_PHASE_FFTCONV = 2,     /* FFT, coefficient multiply, inverse FFT */
    FASTSUM_PHASE_GATHER = 3,      /* window interpolation + FP64 sum over P */
    FASTSUM_PHASE_REDUCE = 4,      /* final FP64 reduction of partial sums   */
    FASTSUM_PHASE_BACKPROJECT = 5, /* grad_y = (tau/P) sum_p xi_p t'_p       */
    FASTSUM_PHASE_SORT = 6,        /* sorted plans: sort + prefix-sum pass    */
    FASTSUM_PHASE_COUNT = 7
} fastsum_phase;

FASTSUM_API fastsum_status fastsum_profile(fastsum_plan plan, int32_t enable);
FASTSUM_API fastsum_status fastsum_profile_read(fastsum_plan plan, double* ms_total,
                                                int64_t* launches);

/* Static, human-readable name of a status code. */
FASTSUM_API const char* fastsum_status_string(fastsum_status status);

#ifdef __cplusplus
}
#endif

#endif /* FASTSUM_H */
