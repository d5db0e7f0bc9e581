/*
 * blnfft.h — C ABI of an MI355X (gfx950) library for the NFFT-like procedure for
 * bandlimited functions of Kircheis & Potts, "Nonequispaced fast Fourier transforms for
 * bandlimited functions" (Algorithm 4.2), with the classical NFFT (Algorithm 2.1) beside it.
 *
 * Problem (Section 4, opening paragraph and Algorithm 4.2, input/output): given samples
 * fhat(k), k in I_M = [-M/2, M/2)^d, of the Fourier transform (1.1) of a bandlimited
 * function f, compute f_j ~ f(x_j) at nonequispaced nodes x_j in [-1/2, 1/2)^d.
 *
 * Conventions used by every call
 * ------------------------------
 *  - Pointers named *_dev are device pointers (hipMalloc'd or equivalent, on the device the
 *    plan was created on).  The caller owns them; the library never frees them.
 *  - Precision: BL_F64 uses double / interleaved double2 complex.  BL_F32, BL_F32C and
 *    BL_F32D use float / interleaved float2 complex for every input and output.
 *  - fhat is an M^d complex array, row-major (last dimension fastest); array index i_t
 *    holds frequency k_t = i_t - M/2.
 *  - Nodes x are an N x d real array, row-major (x[j*d + t]), each coordinate in [-1/2, 1/2).
 *  - f and g are length-N complex arrays in the caller's node order.
 *  - Samples on the oversampled grid (theta) are an L^d complex array, row-major, index
 *    i_t holding grid point l_t = i_t - L/2 (the centred order of I_L).
 *  - `stream` is a hipStream_t passed as void*; NULL means the default stream.  Every
 *    compute call is asynchronous on the plan's stream unless stated otherwise.
 *  - Errors: every call returns a bl_status; nothing throws across the ABI.  On error
 *    bl_last_error() returns a thread-local message.  Invalid arguments are rejected
 *    before any allocation or launch.
 *  - A plan is used from one host thread and one stream at a time.
 */
#ifndef BLNFFT_H
#define BLNFFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BL_OK = 0,
    BL_EINVAL = 1,        /* invalid argument (size, pointer, parameter range)          */
    BL_EDOMAIN = 2,       /* a node is NaN/Inf or outside [-1/2, 1/2)^d                  */
    BL_ENOMEM = 3,        /* device or host allocation failed                           */
    BL_EDEVICE = 4,       /* a HIP runtime call failed                                   */
    BL_ESTATE = 5,        /* call out of order (e.g. forward before set_nodes)          */
    BL_EUNSUPPORTED = 6   /* valid but not implemented (e.g. m above the kernel range)  */
} bl_status;

typedef enum {
    BL_WIN_SINH = 0,      /* sinh-type window, eq. (3.4)                                */
    BL_WIN_CKB = 1        /* continuous Kaiser-Bessel window, Remark 3.1                */
} bl_window;

typedef enum {
    BL_SHANNON = 0,       /* Algorithm 4.2: psihat deconvolution, regularized-sinc sums  */
    BL_NFFT = 1           /* Algorithm 2.1 with M_sigma = L: phihat deconvolution,
                             periodic window sums over I_{L,m}(x_j), eq. (2.5)          */
} bl_method;

typedef enum {
    BL_F64 = 0,           /* everything in double                                       */
    BL_F32 = 1,           /* float data and arithmetic; twiddles and deconvolution
                             factors formed in FP64 and rounded to float; plain sums    */
    BL_F32C = 2,          /* float data, arithmetic and intermediates; FP64 kept only for
                             the FFT twiddles (and chirps) and the deconvolution factors,
                             whose products are formed in double and rounded once; short
                             sums with float weights and float inner sums, the outermost
                             sum compensated by error-free two-sums                     */
    BL_F32D = 3           /* float inputs, outputs and grid of samples; the FFT passes
                             compute in double with double intermediates (one rounding,
                             at the store of the grid); short sums as BL_F32C but with
                             the outermost sum accumulated in double (float products
                             are exact in double)                                       */
} bl_precision;

typedef struct bl_plan_s* bl_plan;
typedef struct bl_batch_s* bl_batch;

typedef struct {
    int64_t n_nodes;          /* N of the last bl_set_nodes                                */
    int64_t n_outside;        /* nodes outside the truncated domain [-1/2+m/L, 1/2-m/L)^d  */
    int64_t n_chunks;         /* work items of the short-sum kernels                       */
    int64_t tile[3];          /* grid cells per tile edge, per dimension                   */
    int64_t chunk_cap;        /* max nodes per work item                                   */
    int64_t workspace_bytes;  /* device memory owned by the plan                           */
    double beta;              /* window shape parameter in use                             */
    double weight_fit_err;    /* largest deviation of the fitted weight polynomials from
                                 the exact weights psi(x - l/L), relative to the largest
                                 weight (0 when FP64 plans evaluate them exactly)          */
    int64_t fft_lines[2][3];  /* lines per workgroup of the forward [0] and adjoint [1]
                                 transform pass over each axis (0: the built-in rule)      */
    int64_t fft_radix[2][3];  /* values per thread (radix, 4 or 16) of the same passes
                                 (0: the built-in rule; chirp-z passes use 16)             */
    int64_t tuned[2];         /* how the FFT lines [0] and the tile edge and chunk
                                 capacity [1] were chosen: 0 built-in rule or environment
                                 override, 1 timed by this plan, 2 from the tuning cache   */
} bl_stats;

/* Create a plan.  Algorithm 4.2 step 0a (psihat(k), k in I_M; eq. (4.9)) or Algorithm 2.1
 * step 0a (phihat(k)) is computed here on the host in double precision.
 *   d      : 1, 2 or 3.
 *   M      : bandwidth per dimension, even, >= 2 (I_M, Section 1).
 *   L      : oversampled grid per dimension, even, L >= M (Algorithm 4.2, L = M(1+lambda)),
 *            L <= 32768 for d = 1 and L <= 8192 for d = 2, 3 (BL_EUNSUPPORTED above).
 *            Any such L runs the short sums; bl_forward and bl_adjoint run every L of
 *            d = 1 and, for d >= 2, L with L + M - 1 within the in-LDS chirp-z transform
 *            or L a power of two (see bl_forward).
 *   m      : truncation, 1 <= m and 2m < L; this build's kernels take 2 <= m <= 8
 *            (BL_EUNSUPPORTED otherwise).
 *   win    : window: BL_WIN_SINH (eq. (3.4)) or BL_WIN_CKB (continuous Kaiser-Bessel,
 *            Remark 3.1).  The short sums evaluate either through fitted polynomials;
 *            with BL_WIN_CKB an FP64 plan needs its fit within 1e-13 (BL_EUNSUPPORTED
 *            otherwise), and FP64 bl_grad_x differentiates the fitted polynomials.
 *   beta   : window parameter; beta <= 0 picks the default: pi*m*(L-M)/L for BL_SHANNON,
 *            2*pi*m*(1 - M/(2L)) for BL_NFFT.  Float plans (BL_F32, BL_F32C) evaluate the
 *            weights by degree-11 polynomials and refuse (BL_EUNSUPPORTED) a beta at which
 *            their fit error exceeds 1e-7 (only far above the defaults, e.g. beta > ~25 at
 *            m = 2); bl_plan_stats reports the fit error.
 *   method : BL_SHANNON or BL_NFFT.
 *   prec   : BL_F64, BL_F32, BL_F32C or BL_F32D.
 *   stream : hipStream_t (as void*) for every later call.
 * Synchronous.  Allocates the plan's device workspace (grid of L^d complex samples,
 * FFT intermediates, tables).  On error *out is set to NULL and nothing is allocated. */
bl_status bl_plan_create(bl_plan* out, int d, int64_t M, int64_t L, int m, bl_window win,
                         double beta, bl_method method, bl_precision prec, void* stream);

/* Bind nodes (Algorithm 4.2 step 0b, realised as binning: nodes are sorted into grid tiles
 * so that the short sums of step 3 read a tile of samples from on-chip memory).
 *   N     : number of nodes, N >= 0.
 *   x_dev : N x d nodes, row-major, in the plan's real type; each coordinate must lie in
 *           [-1/2, 1/2).  The library copies them (sorted), so x_dev may be reused
 *           after this call returns.
 * Synchronizes with the plan's stream once.  Returns BL_EDOMAIN if any coordinate is NaN,
 * infinite or outside [-1/2, 1/2) (the plan then holds no nodes). */
bl_status bl_set_nodes(bl_plan plan, int64_t N, const void* x_dev);

/* Algorithm 4.2 step 0b in precomputed form: evaluate the d x 2m window weights
 * psi(x_jt - l_t / L) of every bound node once and keep them in plan workspace
 * (N * d * 2m values of the plan's real type), so that later bl_forward and bl_interpolate
 * calls read them instead of evaluating them (for repeated transforms with fixed nodes).
 *   enable : nonzero to compute and use them, 0 to free them and evaluate on the fly again.
 * BL_ESTATE without bound nodes, BL_EUNSUPPORTED for BL_NFFT plans.  The next
 * bl_set_nodes discards them.  Results equal the on-the-fly ones (same weight arithmetic).
 * Synchronous. */
bl_status bl_precompute_weights(bl_plan plan, int enable);

/* Forward transform, Algorithm 4.2 steps 1-3 (or Algorithm 2.1 steps 1-3):
 *   step 1: thetahat(k) = fhat(k) / psihat(k) on I_M, 0 on I_L \ I_M;
 *   step 2: theta_l = L^-d sum_{k in I_L} thetahat(k) e^{2 pi i k l / L}   (4.7);
 *   step 3: f_j = sum_{l in J_{L,m}(x_j)} theta_l psi(x_j - l/L)           (4.8),
 * with theta_l = 0 for l outside I_L (zero-extended sum; BL_NFFT wraps periodically).
 *   fhat_dev : M^d complex (input).   f_dev : N complex (output, overwritten).
 * Asynchronous.  Keeps theta for bl_grad_x / bl_get_theta.  Step 2 runs power-of-two
 * L <= 8192 as radix-4/16 passes and any other L as chirp-z (Bluestein) passes with a cyclic
 * convolution of power-of-two size P >= L + M - 1; BL_EUNSUPPORTED when d >= 2 and P exceeds
 * the in-LDS transform (8192 points for BL_F64 and BL_F32D, 16384 for BL_F32 and BL_F32C). */
bl_status bl_forward(bl_plan plan, const void* fhat_dev, void* f_dev);

/* Steps 1-2 alone (Algorithm 4.2 or 2.1): the samples theta_l, l in I_L, of (4.7) from
 * fhat_dev (M^d complex), kept in the plan for bl_get_theta and bl_grad_x.  Needs no bound
 * nodes.  The same L restrictions as bl_forward.  Asynchronous. */
bl_status bl_samples(bl_plan plan, const void* fhat_dev);

/* Regularized Shannon sampling formula (3.5) truncated to I_L: evaluate step 3 alone on
 * given samples theta_dev (L^d complex, centred order) at the bound nodes (BL_NFFT: the
 * periodic window sums of Algorithm 2.1 on those samples).  Any even L.
 *   f_dev : N complex (output).  Asynchronous. */
bl_status bl_interpolate(bl_plan plan, const void* theta_dev, void* f_dev);

/* Copy the samples theta_l, l in I_L, of the last bl_forward to theta_dev (L^d complex,
 * centred order).  BL_ESTATE before any forward.  Asynchronous. */
bl_status bl_get_theta(bl_plan plan, void* theta_dev);

/* Adjoint of the factorisation (4.11): fhat_out = D_psihat^H F^H Psi^T g  (BL_SHANNON), or
 * D^H F^H B^T g (BL_NFFT).  D is real; F^H uses e^{-2 pi i k l / L}.
 *   g_dev : N complex (input).   fhat_dev : M^d complex (output, overwritten).
 * Psi^T g is formed without atomic additions in device memory: each work chunk of nodes
 * writes its tile-plus-halo box, and the boxes are summed per grid point in a fixed order,
 * so for one node binding repeated calls give bitwise equal results (the LDS-atomic
 * spreading kernel, which only the BL_SPREAD_ATOMIC override or a tile edge set by BL_TILE
 * beyond the other kernels' boxes selects, sums within a work chunk in no fixed order).  The first call (and
 * a call after a binding with more work chunks) allocates the spreading grid and boxes.
 * Asynchronous.  The same L restrictions as bl_forward. */
bl_status bl_adjoint(bl_plan plan, const void* g_dev, void* fhat_dev);

/* bl_adjoint for callers that cannot allocate device memory (code under HIP stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same computation and
 * kernels, with the spreading grid and the work chunks' boxes held in a fixed device
 * scratch array of the library (64 MiB per GPU, held until the process ends) instead of
 * plan memory that bl_adjoint allocates on its first call.  Allocates nothing (the plan's
 * own FFT buffers, allocated by bl_plan_create, are used as by bl_adjoint).
 *   g_dev : N complex (input).   fhat_dev : M^d complex (output, overwritten).
 * BL_EUNSUPPORTED when the grid (L^d complex values of the plan's type) and the boxes (one
 * prod_t (tile_t + 2m - 1) complex values per work chunk, bl_plan_stats) exceed 64 MiB
 * (e.g. d = 3, L = 256).  All calls on one GPU share the one array and each leaves its
 * contents behind, so calls that overlap in time on one GPU (other streams or threads)
 * race; order them on one stream.  Asynchronous. */
bl_status bl_adjoint_noalloc(bl_plan plan, const void* g_dev, void* fhat_dev);

/* Gradient with respect to the nodes: gx[j*d + t] = Re( conj(g_j) * d f_j / d x_jt ),
 * f from the last bl_forward (BL_SHANNON only).  f_j is the short sum (4.8) over the
 * samples theta of step 2 (the factorisation (4.11) with Psi's entries psi(x_j - l/L)),
 * so d f_j / d x_jt = L sum_l theta_l psi'(L x_jt - l_t) prod_{s != t} psi(L x_js - l_s)
 * in grid units, with psi' of the regularized sinc (4.2).  With g = 2(f - y) this is the gradient
 * of sum_j |f_j - y_j|^2.   g_dev : N complex.  gx_dev : N x d real (output).
 * BL_ESTATE if no forward has run since the last bl_set_nodes.  FP64 plans with
 * BL_WIN_CKB take the weight derivatives from the fitted weight polynomials; their
 * relative deviation from the exact derivatives is checked at plan creation and
 * BL_EUNSUPPORTED is returned if it exceeds 5e-12.  Asynchronous. */
bl_status bl_grad_x(bl_plan plan, const void* g_dev, void* gx_dev);

/* Plan statistics: the bound node count and how many of the nodes lie outside the
 * truncated domain [-1/2 + m/L, 1/2 - m/L)^d of Algorithm 4.2 (Section 4, where the short
 * sums (4.8) reach grid points outside I_L), the work decomposition of step 3, the
 * workspace and the window's beta (3.4).  Synchronous with respect to host state only. */
bl_status bl_plan_stats(bl_plan plan, bl_stats* out);

/* Destroy a plan (synchronizes its stream, frees its workspace).  NULL is accepted. */
bl_status bl_plan_destroy(bl_plan plan);

/* Host-only: the window transform used for the deconvolution factors, by the library's
 * own quadrature.  out[i] = psihat(v[i]) for BL_SHANNON (Algorithm 4.2 step 0a, the
 * transform (3.1) of psi in (4.2)) or phihat(v[i]) for BL_NFFT (Algorithm 2.1 step 0a),
 * univariate.  beta <= 0 picks the default for (M, L, m, method).  Needs no GPU. */
bl_status bl_window_transform(bl_window win, bl_method method, int64_t M, int64_t L, int m,
                              double beta, int64_t n, const double* v, double* out);

/* Batched d = 1 transforms (Algorithm 4.2 with the sinh-type window of (3.4) and the
 * default shape parameter beta = pi m (L - M) / L) of `count` independent instances with
 * their own (M_i, L_i, m_i, N_i), executed as one graph launch: steps 1-2 of every
 * instance in one kernel (one workgroup per instance, any even L_i via the chirp-z form of
 * the length-L_i transform), step 3 of every instance in a second kernel.
 *   M, L, m, N : host arrays of length count; per instance M even >= 2, L even > M,
 *                2m < L, N >= 0 (else BL_EINVAL); 2 <= m <= 8 and L + M - 1 <= 32768
 *                (else BL_EUNSUPPORTED).
 *   prec       : BL_F32 or BL_F32C (float data; F32C accumulates the short sums in double);
 *                BL_F64 gives BL_EUNSUPPORTED.
 *   stream     : hipStream_t the calls are ordered on (NULL: default stream).
 * Packed device buffers (complex = interleaved float pairs): instance i's fhat occupies
 * complex elements [sum_{i'<i} M_i', +M_i) in the order k = -M_i/2 .. M_i/2 - 1, its nodes
 * and outputs [sum_{i'<i} N_i', +N_i).  The batch owns its device workspace; the caller
 * owns every buffer it passes.  Synchronous (builds the per-instance tables). */
bl_status bl_batch_create(bl_batch* out, int count, const int64_t* M, const int64_t* L,
                          const int* m, const int64_t* N, bl_precision prec, void* stream);
/* Bind the packed nodes (sum N_i floats in [-1/2, 1/2)); the pointer need not stay valid
 * afterwards.  The first call times the short sums for a few tile sizes and keeps the
 * fastest.  Synchronous; BL_EDOMAIN if a node is NaN/Inf or outside [-1/2, 1/2), after
 * which forward calls fail with BL_ESTATE until a binding succeeds. */
bl_status bl_batch_set_nodes(bl_batch batch, const void* x_dev);
/* Forward transform of every instance: packed fhat in, packed f out (both device).
 * Asynchronous on the batch's stream; the first call with a new (fhat, f) pointer pair
 * captures and instantiates the graph. */
bl_status bl_batch_forward(bl_batch batch, const void* fhat_dev, void* f_dev);
/* Synchronize the batch's stream and release everything the batch owns (NULL: no-op). */
bl_status bl_batch_destroy(bl_batch batch);

/* Status text (static storage) and the calling thread's last error message. */
const char* bl_status_string(bl_status s);
const char* bl_last_error(void);

/* Library version string (static storage). */
const char* bl_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BLNFFT_H */
