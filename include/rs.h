/*
 * rs.h -- C ABI of the range-separated (RS) canonical/Tucker potential library
 * for AMD Instinct MI355X (gfx950).
 *
 * The library assembles the N-particle potential sum
 *     P(x) = sum_nu z_nu p(|x - x_nu|),   x, x_nu in Omega = [-b, b]^3     (eq PotSum1)
 * on the uniform n x n x n grid of cell centres x_i = -b + (i + 1/2) h,
 * h = 2b/n, n even (section 2.2), in the RS-Tucker format
 *     A = beta x_1 V1 x_2 V2 x_3 V3 + sum_nu z_nu U_nu                     (Definition RS-Tucker_format)
 * where the Tucker part is the reduced-HOSVD (RHOSVD) compression of the
 * long-range canonical sum (eq Long-Range_Sum, Appendix eqs SVD_SideMatr,
 * alg1) and U_nu are short-range windows of the reference tensor
 * (Definitions ComCanF, CCT_Uniform).  It also evaluates P at points, the
 * interaction energy (Lemma InterEnergy, eq EnergyFree_Tensor) and the forces
 * F_j = -dE/dx_j (section 4.3).
 *
 * Conventions for every call
 *  - "device" pointers are HIP device memory on the context's device (for
 *    example torch CUDA tensors on ROCm); "host" pointers are ordinary memory.
 *  - The caller owns every pointer argument.  The library owns the opaque
 *    handles (rs_ctx, rs_factors, rs_tensor) and frees them only through the
 *    matching *_free / *_destroy call.
 *  - Work is enqueued on the HIP stream passed as `stream` (a hipStream_t;
 *    NULL = the null stream).  Calls return once their work is enqueued,
 *    except where a call says it synchronizes.
 *  - Stream lifetime: the library's device-buffer cache remembers the stream
 *    that last used each cached buffer and may later make another stream
 *    wait on it.  A stream handed to the library must therefore stay valid
 *    until the tensors made on it are freed and rs_stream_release(ctx,
 *    stream) has been called (or until rs_ctx_trim, or the end of the
 *    process).
 *  - Arguments are validated before anything is enqueued; on a non-OK
 *    status nothing has been written to caller memory.  rs_last_error()
 *    returns a thread-local message describing the last failure.  No C++
 *    exception crosses this boundary.
 *  - Results are deterministic: no floating-point atomics; every reduction
 *    runs in a fixed order that depends only on the request's own shape, so
 *    the same inputs give bitwise-identical outputs whatever else runs on
 *    the device.
 */
#ifndef RS_H
#define RS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RS_OK = 0,
  RS_E_INVALID = 1,      /* bad argument or input (see rs_last_error) */
  RS_E_NOMEM = 2,        /* device allocation failed */
  RS_E_DEVICE = 3,       /* a HIP call failed */
  RS_E_RANK_CAP = 4,     /* rank rule exceeded r_max: result produced at r_max (non-fatal) */
  RS_E_UNSUPPORTED = 5   /* valid request the library does not support */
} rs_status;

/* Generating kernel p(r) (section 2.2): Newton 1/r, Yukawa e^{-lambda r}/r,
 * or their sum.  All are Laplace-Gauss transforms p(z) = int a(t) e^{-t^2 z^2} dt
 * (eq laplace) with a(t) = 2/sqrt(pi) [ * e^{-lambda^2 / (4 t^2)} ]. */
typedef enum { RS_NEWTON = 0, RS_YUKAWA = 1, RS_NEWTON_PLUS_YUKAWA = 2 } rs_kernel;

/* Arithmetic of the assembly.
 *  RS_FP64: everything in FP64; the grid is FP64.
 *  RS_MIXED_FP16: the projection (U~ = V^T U), the core contraction, the
 *    second expansion contraction (T2 = X x_2 V2) and the last grid-expansion
 *    contraction (T2 x_3 V3) use split FP16 operands (value = hi + lo,
 *    power-of-two scaled, three MFMA products) with FP32 MFMA accumulation
 *    and FP64 sums across K chunks; the side matrices are formed directly as
 *    the projection's FP16 planes (FP64 only where an option needs them); the
 *    Gram, eigensolve, first expansion contraction, quadrature table, point
 *    evaluation and energy reduction stay FP64, and T2 is kept in FP64.  The
 *    grid is FP32.
 *  RS_MIXED_BF16: as RS_MIXED_FP16 with three-way split BF16 operands (six
 *    products).
 *  RS_FP32: assembled as RS_MIXED_FP16; point values, the energy's per-
 *    particle terms and the forces are evaluated from FP32 copies of the
 *    Tucker field in FP32 arithmetic (the energy and forces of sections 4.2-4.3 at
 *    single precision), with the energy's final reduction and every output
 *    in FP64. */
typedef enum { RS_FP64 = 0, RS_MIXED_FP16 = 1, RS_MIXED_BF16 = 2, RS_FP32 = 3 } rs_prec;

typedef struct rs_ctx rs_ctx;
typedef struct rs_factors rs_factors;
typedef struct rs_tensor rs_tensor;

/* Grid: Omega = [-b, b]^3, n points per axis, n even, n >= 8. */
typedef struct {
  double b;
  int64_t n;
} rs_grid;

/* Quadrature rule of eq laplace (section 2.2).
 *  RS_RULE_PAPER_LITERAL: t_k = k h_M, h_M = C0 log(M)/M (eq hM), weights
 *     folded onto k >= 0: a_0 = h_M a(0)/2, a_k = h_M a(t_k).  Accurate for
 *     1/r only on a narrow band of r (about [0.3, 2] at R = 20).
 *  RS_RULE_EXP_SINC: the exponential convergence of eq sinc_conv from the
 *     substitution t = e^s: M = R - 1 nodes t_k = e^{s_1 + (k-1) h} with
 *     weights a_k = (2/sqrt(pi)) h t_k a(t_k)/a_Newton, plus t_0 = 0 carrying
 *     the geometric sum of the nodes left of s_1; the step h and s_1 are
 *     chosen so that M nodes cover [r_lo, r_hi] with balanced
 *     discretisation and truncation errors (relative error against 1/r
 *     about 2e-4 at R = 20, 2e-5 at R = 32 for the default range). */
typedef enum { RS_RULE_PAPER_LITERAL = 0, RS_RULE_EXP_SINC = 1 } rs_rule;

/* Quadrature and range split (sections 2.2-2.3).
 *  R: number of terms, R = M + 1, by `rule` (rs_rule).
 *  R_l: long-range terms k = 0..R_l-1 (1 <= R_l <= R-1); -1 = choose by
 *     criterion (A) (eq Split_crit_max) for the support radius sigma = sigma_split.
 *  n_s: odd short-range window width in cells; -1 = the smallest odd n_s with
 *     (n_s/2) h >= sigma, sigma the radius beyond which every short term
 *     a_k e^{-t_k^2 sigma^2} <= delta_rel * S(0) (criterion (A) solved for sigma).
 *  C0 <= 0 selects the paper's C0 = 3. */
typedef struct {
  int32_t kernel;        /* rs_kernel */
  double lambda;         /* Yukawa screening, > 0 when used */
  int32_t R;
  int32_t R_l;
  int32_t n_s;
  double delta_rel;      /* criterion (A) threshold relative to S(0); <= 0 -> 1e-4 */
  double sigma_split;    /* only read when R_l == -1 */
  double C0;             /* literal rule only */
  int32_t rule;          /* rs_rule */
  double r_lo, r_hi;     /* exp-sinc rule: range of r it is fitted to; <= 0: h and 2 sqrt(3) b */
} rs_fdesc;

/* How the charge-weighted Gram matrices G_l = U_l diag(|xi|^{2/3}) U_l^T are formed.
 *  RS_GRAM_IDENTITY: by the Gaussian-product identity
 *     G[i, i'] = sum_k exp(-t_k^2 (x_i - x_i')^2 / 2) sum_nu w exp(-2 t_k^2 ((x_i + x_i')/2 - x_nu)^2),
 *     O(n N R_l + n^2 R_l) work (the columns are Gaussians of one width per k);
 *  RS_GRAM_GEMM: by the FP64 MFMA product U diag(w) U^T, 2 n^2 N R_l FLOP. */
typedef enum { RS_GRAM_IDENTITY = 0, RS_GRAM_GEMM = 1 } rs_gram_method;

/* Assembly options.
 *  eps_tucker: rank rule, keep singular values sigma_k > eps_tucker * sigma_1 of
 *     the charge-weighted side matrix U_l diag(|xi|^{1/3}) (Appendix, step (I)).
 *  r_max: rank cap per mode (<= n).  fixed_ranks[l] > 0 overrides the rule.
 *  oversample: extra subspace columns of the eigensolver beyond r_max (or
 *     beyond the largest fixed rank); default when <= 0: 16 for the rank rule,
 *     48 with fixed ranks.  The margin between the subspace size and the
 *     rank sets how well the basis resolves the directions at the threshold.
 *  power_iters: subspace iterations Q <- orth(G Q) after the range finder
 *     (default 0 when < 0).
 *  interp_order: even Lagrange order p of point evaluation (default 6 when <= 0).
 *  gram: rs_gram_method (default RS_GRAM_IDENTITY = 0).
 *  sketch: what the randomized range finder multiplies by the random matrix:
 *     0 (default) the Gram G_l itself (n x n, 2 n^2 p FLOP; its spectrum is
 *     the square of the side matrix's, so the directions at the threshold are
 *     resolved as by one subspace iteration), 1 the weighted side matrix
 *     U_l diag(|xi|^{1/3}) (n x N R_l, 2 n N R_l p FLOP).
 *  subspace_min: when > 0, the rank rule's subspace is searched: the
 *     eigensolver runs first with p = subspace_min and again with the full
 *     size (r_max + oversample) only when some mode's rank plus twice the
 *     oversampling exceeds p, so a system whose ranks are far below r_max
 *     does not pay for an r_max-sized eigenproblem (a system that grows pays
 *     for both passes and one more rank readback).  0 (default) or a value at
 *     or above the full size: no search.  Fixed ranks size the subspace
 *     directly.  The result depends only on the inputs and options, not on
 *     earlier calls.
 *  als_sweeps: sweeps of the ALS refinement that follows the RHOSVD bases
 *     (Appendix, steps (III)-(V), eq alg2; default 0): for l = 1, 2, 3 in
 *     turn, the partially projected image M_l = U_l diag(xi) (U~_m (.) U~_p)^T
 *     (n x r_m r_p, formed by the core's contraction in the core's
 *     precision) replaces the mode-l basis by its r_l dominant left singular
 *     vectors (eigenvectors of M_l M_l^T, FP64); the ranks stay those of the
 *     rank rule (or fixed).  Each sweep costs about 3 n / r_l times the
 *     core's contraction and does not decrease ||beta|| (the Tucker error
 *     does not grow). */
typedef struct {
  double eps_tucker;
  int32_t r_max;
  int32_t fixed_ranks[3];
  int32_t prec;          /* rs_prec */
  int32_t oversample;
  int32_t power_iters;
  int32_t interp_order;
  int32_t gram;          /* rs_gram_method */
  int32_t sketch;        /* 0: G_l, 1: U_l diag(|xi|^{1/3}) */
  int32_t subspace_min;  /* first subspace size of the rank rule's search */
  int32_t als_sweeps;    /* ALS refinement sweeps of the Tucker bases (0: none) */
} rs_aopts;

typedef struct {
  int64_t N, n;
  double b, h;
  int32_t R, R_l, n_s, prec, interp_order;
  int32_t ranks[3];          /* Tucker ranks r_1, r_2, r_3 */
  int32_t subspace[3];       /* eigensolver subspace size p per mode */
  double sigma_first[3];     /* sigma_1 of each mode */
  double sigma_last_kept[3]; /* sigma_r / sigma_1 */
  double sigma_next[3];      /* sigma_{r+1} / sigma_1 (0 if not resolved) */
  double S0, S_l0;           /* S(0) = sum a_k, S_l(0) = sum_{k<R_l} a_k */
  int64_t tucker_storage;    /* r1 r2 r3 + n (r1 + r2 + r3) (Lemma Property_RST_Tuck) */
  int64_t device_bytes;      /* device memory held by the tensor */
  int32_t rank_capped;       /* 1 if the rank rule hit r_max in some mode */
  /* Milliseconds per assembly stage, measured with HIP events on the
   * assembly stream when timing is enabled (rs_ctx_set_timing), else 0.
   * Stages: RS_STAGE_* below. */
  double stage_ms[12];
  /* With timing enabled: milliseconds of the eigensolver's phases
   * (RS_EIG_* below; all modes together). */
  double eig_phase_ms[4];
} rs_info;

enum {
  RS_STAGE_FACTORS = 0,   /* side matrices and weights */
  RS_STAGE_GRAM = 1,      /* n x n charge-weighted Gram GEMMs (only when the subspace is all of R^n) */
  RS_STAGE_EIGEN = 2,     /* dominant eigenvectors of the Gram matrices, rank rule (incl. rank readback) */
  RS_STAGE_BINS = 3,      /* short-range brick lists (first after the readback) */
  RS_STAGE_BASIS = 4,     /* V_l = Q W, canonical signs */
  RS_STAGE_PROJECT = 5,   /* U~_l = V_l^T U_l */
  RS_STAGE_CORE = 6,      /* Khatri-Rao core contraction */
  RS_STAGE_EXPAND1 = 7,   /* V1 beta_(1) */
  RS_STAGE_EXPAND2 = 8,   /* T2 = beta x_1 V1 x_2 V2 */
  RS_STAGE_GRID = 9,      /* grid = T2 x_3 V3 (one GEMM launch) */
  RS_STAGE_SHORT = 10,    /* short-range window gather into the grid */
  RS_STAGE_COUNT = 11,
  /* stage_ms[RS_STAGE_CORE_KERNEL]: the core's main contraction kernel alone,
   * without its operand preparation and split-K sum (timing mode 3 only) */
  RS_STAGE_CORE_KERNEL = 11
};

/* Phases of the eigen stage reported in rs_info.eig_phase_ms. */
enum {
  RS_EIG_SUBSPACE = 0,   /* sketch, Cholesky QR, Rayleigh-Ritz matrix B = Q^T G Q */
  RS_EIG_TRIDIAG = 1,    /* Householder tridiagonalisation of B */
  RS_EIG_VALUES = 2,     /* eigenvalues by bisection, eigenvectors by inverse iteration */
  RS_EIG_ORTH = 3,       /* Cholesky QR of the eigenvectors, back-transformation */
  RS_EIG_PHASES = 4
};

/* ---- context ---------------------------------------------------------- */

/* Bind the library to HIP device `device` (makes it current on this thread). */
rs_status rs_ctx_create(int device, rs_ctx** out);
/* Release the handle.  Tensors still alive keep the context (and its cached
   memory and pinned slots) until the last of them is freed with
   rs_tensor_free; a null handle is ignored. */
void rs_ctx_destroy(rs_ctx* ctx);
/* HIP-event timing of later assemblies made with this context, reported in
 * rs_info.stage_ms and eig_phase_ms: 0 off, 1 every stage and eigensolver
 * phase, 2 the grid stage only (two events around its one kernel, so that
 * the rest of the assembly runs without markers between launches), 3 the
 * core's main kernel only (stage_ms[RS_STAGE_CORE_KERNEL]).
 * Errors: RS_E_INVALID for another value. */
rs_status rs_ctx_set_timing(rs_ctx* ctx, int enable);
/* Synchronise `stream` and detach the library's cached buffers from it, so
 * that the caller may destroy it afterwards (see "Stream lifetime" above).
 * Tensors still alive that were made on `stream` keep using it when freed:
 * free them first.  Errors: RS_E_DEVICE if the synchronisation fails. */
rs_status rs_stream_release(rs_ctx* ctx, void* stream);
/* Device memory of the library's buffers comes from a per-device cache: a
 * released buffer is kept for reuse by later assemblies (immediately on the
 * stream it was released on, after an event wait on another stream) and is
 * returned to the driver only when an allocation would fail.  This call
 * synchronises the context's device and returns every cached block now.
 * Buffers still held by live tensors are not affected. */
rs_status rs_ctx_trim(rs_ctx* ctx);
/* Admission budget of the context, for callers that size several requests
 * against one device (a serving loop): rs_assemble refuses, with RS_E_NOMEM
 * and before it allocates anything, a request whose rs_footprint_bytes bound
 * (the factors' grid and quadrature, N, the larger of r_max and the fixed
 * ranks, the precision) exceeds `bytes`.  The bound is per request:
 * concurrent assemblies on one context are each checked alone.  0, the
 * default, sets no budget.  Errors: RS_E_INVALID for a null context. */
rs_status rs_ctx_set_hbm_budget(rs_ctx* ctx, size_t bytes);

/* ---- quadrature table and split (sections 2.2-2.3) --------------------- */

/* Build the FP64 quadrature table {t_k, a_k}, the long/short split R_l and
 * the window width n_s on the host, and copy the table to the device
 * (synchronous, a few hundred bytes).  Errors: RS_E_INVALID for R < 3,
 * R_l outside [1, R-1], n odd or < 8, even n_s, non-positive b, lambda <= 0
 * for a Yukawa kernel. */
rs_status rs_build_factors(rs_ctx* ctx, const rs_grid* grid, const rs_fdesc* fdesc,
                           rs_factors** out);
/* Host copies of the table (arrays of length R, or NULL) and the split. */
rs_status rs_factors_get(const rs_factors* f, double* t, double* a, int32_t* R,
                         int32_t* R_l, int32_t* n_s);
void rs_factors_free(rs_factors* f);

/* ---- assembly (sections 3.2-3.3, Appendix) ----------------------------- */

/* Assemble the RS-Tucker tensor of N particles.
 *  pos: device, N x 3 row-major FP64 coordinates, all inside [-b, b]^3.
 *  q:   device, N FP64 charges.
 *  grid_out: device, n^3 values in C order (i3 fastest) or NULL to skip the
 *     full-grid materialisation; FP64 for RS_FP64, FP32 for the mixed modes.
 *     It receives beta x_1 V1 x_2 V2 x_3 V3 + sum_nu z_nu U_nu at the cell centres.
 *  out: receives a new tensor handle (keeps its own copies of pos and q).
 * Steps: side matrices U_l[i, k*N+nu] = exp(-t_k^2 (x_i - x_{nu,l})^2) for
 * k < R_l; weighted Gram G_l = U_l diag(|xi|^{2/3}) U_l^T, xi = z_nu a_k
 * (opts->gram); dominant eigenvectors of G_l in FP64: a randomized range
 * finder (opts->sketch) orthonormalised by shifted Cholesky QR
 * (opts->power_iters more subspace iterations through G_l), the Rayleigh-Ritz
 * matrix Q^T G_l Q, Householder tridiagonalisation, bisection and inverse
 * iteration; rank rule; projection U~_l = V_l^T U_l; core
 * beta = sum_j xi_j u~1_j (x) u~2_j (x) u~3_j; short windows of width n_s
 * around each particle's cell.
 * Synchronizes `stream` once, after the eigensolve, to read the ranks back.
 * Errors: RS_E_INVALID (N < 1, non-finite input, a particle outside Omega,
 * bad options), RS_E_NOMEM, RS_E_DEVICE; RS_E_RANK_CAP is returned with a
 * valid tensor when some rank was capped. */
rs_status rs_assemble(rs_ctx* ctx, const rs_factors* f, int64_t N, const double* pos,
                      const double* q, const rs_aopts* opts, void* grid_out,
                      rs_tensor** out, void* stream);

/* The three charge-weighted Gram matrices G_l = U_l diag(|xi|^{2/3}) U_l^T of
 * the long-range side matrices (Appendix step (I) through the Gram), the
 * first step of the RHOSVD.  pos, q as in rs_assemble; method: rs_gram_method;
 * G: device, 3 x n x n FP64 (mode-major, symmetric).  Asynchronous.
 * Errors: RS_E_INVALID for an unknown method. */
rs_status rs_weighted_gram(rs_ctx* ctx, const rs_factors* f, int64_t N, const double* pos,
                           const double* q, int32_t method, double* G, void* stream);

/* ---- evaluation (Lemma Property_RST_Tuck, sections 4.2-4.3) ------------ */

/* Values of the RS tensor at M arbitrary points.
 *  pts: device, M x 3 row-major FP64 inside Omega;  vals: device, M FP64.
 *  part: 0 = long + short, 1 = long-range Tucker part, 2 = short-range part.
 * The long-range part is the order-p tensor Lagrange interpolant of the
 * Tucker factors on the cell-centred grid (exact at grid points); the short
 * part sums the short-range Gaussians of every particle whose window
 * contains the point's cell.  Asynchronous. */
rs_status rs_eval_points(const rs_tensor* T, int64_t M, const double* pts, double* vals,
                         int32_t part, void* stream);

/* Gradient of the RS tensor at M arbitrary points (section 4.3), or its
 * normal derivative: the long-range part is the derivative of the same
 * order-p interpolant rs_eval_points uses (the interpolated Tucker factor
 * rows differentiated, eq Gradients_Tens applied to the continuous
 * factors); the short-range part differentiates each windowed term
 * z_nu sum_{k>=R_l} a_k exp(-t_k^2 |y - x_nu|^2) analytically, for the
 * particles whose window holds the point's cell (as in rs_eval_points).
 * part: 0 long + short, 1 long only (what interface conditions on a surface
 * at least half a short-range support away from every particle need,
 * Proposition PBE_RSTensor), 2 short only.
 * pts: device, M x 3 row-major.  normals: device M x 3 (unit surface normals;
 * need not be unit, each output is the plain dot product) or NULL.
 * out: device FP64, M x 3 gradients when normals is NULL, else the M values
 * <grad P(y_i), normals_i>.  M = 0 is a no-op. */
rs_status rs_eval_gradient_points(const rs_tensor* T, int64_t M, const double* pts,
                                  const double* normals, double* out, int32_t part, void* stream);

/* Interaction energy E_N = 1/2 sum_j z_j (P_l(x_j) - z_j g_j) (eq EnergyFree_Tensor),
 * g_j the particle's own long-range term through the same interpolation
 * (= P_{R_l}(0) for a particle on a grid point).
 *  E: device, 1 FP64 (FP64 reduction in a fixed order).
 *  dEdq: device, N FP64 with dE/dz_j = P_l(x_j) - z_j g_j, or NULL. */
rs_status rs_energy(const rs_tensor* T, double* E, double* dEdq, void* stream);

/* Forces by the adjoint of the energy with the Tucker basis held fixed:
 * F: device, N x 3 FP64, F_j = -scale * dE/dx_j = -scale z_j grad[P_l - z_j g_j](x_j). */
rs_status rs_forces(const rs_tensor* T, double scale, double* F, void* stream);

/* Energy and forces from one evaluation pass at the particles: the results
 * of rs_energy(T, E, dEdq) and rs_forces(T, scale, F), bitwise, for the
 * price of one.  E, F as there; dEdq may be NULL. */
rs_status rs_energy_forces(const rs_tensor* T, double* E, double* dEdq, double scale, double* F,
                           void* stream);

/* rs_energy_forces for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same results, bitwise, with the
 * per-particle scratch (8 N doubles) carved from a static device array of
 * the library (8 MiB per GPU, held until the process ends) instead of the
 * library's allocator.  It calls no hipMalloc/hipFree.  Every call on one GPU
 * shares that array: calls that overlap on one GPU (other streams, other
 * threads) race and must be serialised by the caller.
 * Errors: RS_E_INVALID for N > 131072 (8 N doubles must fit the array), a
 * null E or F, or a non-finite scale. */
rs_status rs_energy_forces_noalloc(const rs_tensor* T, double* E, double* dEdq, double scale,
                                   double* F, void* stream);

/* Matrix-vector product with the RBF interpolation matrix of the kernel p
 * on the n^3 grid points in RS form (section 4.1, case (A)):
 *   y = A c,  A = sum_k a_k T_k (x) T_k (x) T_k,
 * T_k[i][j] = exp(-t_k^2 ((i - j) h)^2) the symmetric Toeplitz Gaussian of
 * quadrature node k, truncated for the short-range terms k >= R_l to the
 * window |i - j| <= (n_s - 1)/2 (the localised part of the split).  The
 * Kronecker factors are applied mode by mode as FP64 MFMA GEMMs, the sum
 * over k folded into the last one (6 R n^4 FLOP: dense Toeplitz products
 * suit the matrix cores for n up to a few hundred; the paper's 1D FFTs
 * would scale as R n^3 log n).
 * c, y: device, n^3 FP64 in C order (distinct buffers).  Takes R n^3 + n^3
 * doubles of device workspace. */
rs_status rs_rbf_matvec(rs_ctx* ctx, const rs_factors* f, const double* c, double* y,
                        void* stream);

/* Scalar product <A, B> = sum_i A(i) B(i) of two RS tensors over all n^3
 * cells of their common grid (section 3.4, item (d)), computed in the
 * format: the long-range parts through their Tucker factors
 * (M_l = V_l^A^T V_l^B and three small contractions of the cores), plus the
 * cells the short-range windows of either tensor touch (outside them each
 * tensor equals its long part), where A B - A_l B_l is summed brick by brick.
 * FP64 arithmetic (split-precision tensors keep FP64 factors and cores); the
 * sums run in a fixed order (deterministic).  The tensors may hold other
 * particles, charges, kernels and ranks.  out: device, 1 FP64.
 * Errors: RS_E_INVALID when n or b differ. */
rs_status rs_dot(const rs_tensor* A, const rs_tensor* B, double* out, void* stream);

/* The n^3 grid of the RS tensor (Definition RS-Tucker_format) from its
 * handle: T2 x_3 V3 plus the short-range windows, the same kernels and
 * arithmetic as the grid rs_assemble writes, so the result is bitwise that
 * grid (also for a tensor from rs_tensor_load).  grid_out: device, n^3 in C
 * order, FP64 for RS_FP64 tensors, FP32 otherwise.  Asynchronous. */
rs_status rs_tensor_grid(const rs_tensor* T, void* grid_out, void* stream);

/* The discrete gradient of the RS tensor along one axis on the whole grid
 * (eq Gradients_Tens in the Tucker form): grid_out receives the finite
 * difference along `axis` (0, 1, 2 = i1, i2, i3; central inside, one-sided
 * at the two ends of the axis, spacing h) of beta x_1 V1 x_2 V2 x_3 V3 +
 * sum_nu z_nu U_nu at every cell centre.  The long-range part is the Tucker
 * tensor with V_axis replaced by its column-wise difference D V_axis (the
 * other factors and the core unchanged); each windowed short-range term is
 * differenced in the same way along the axis (it then reaches one cell
 * beyond its window).  -grid_out approximates the axis component of the
 * field -grad P.  grid_out: device, n^3 in C order, FP64 for RS_FP64
 * tensors, FP32 otherwise.  Synchronizes `stream` once (the size of the
 * widened short-range lists).  Errors: RS_E_INVALID for another axis. */
rs_status rs_gradient_grid(const rs_tensor* T, int32_t axis, void* grid_out, void* stream);

/* ---- introspection, persistence --------------------------------------- */

/* Peak device memory rs_assemble needs for this request (with_grid != 0 adds
 * nothing: the grid belongs to the caller).  r_max bounds the ranks. */
size_t rs_footprint_bytes(const rs_grid* grid, const rs_fdesc* fdesc, int64_t N,
                          int32_t r_max, int32_t prec, int32_t with_grid);
rs_status rs_tensor_info(const rs_tensor* T, rs_info* info);

/* Copy the Tucker factors to caller device memory: V_l as n x r_l row-major
 * (any of V1, V2, V3 may be NULL) and beta as r1 x r2 x r3 C order (or NULL).
 * Synchronizes `stream`. */
rs_status rs_tensor_export(const rs_tensor* T, double* V1, double* V2, double* V3,
                           double* beta, void* stream);

/* Save the RS-Tucker parametrisation (table, split, ranks, V_l, beta,
 * particles, charges) to a versioned binary file; load rebuilds the tensor
 * on the context's device without recomputing the decomposition.  Both
 * synchronize. */
rs_status rs_tensor_save(const rs_tensor* T, const char* path);
rs_status rs_tensor_load(rs_ctx* ctx, const char* path, rs_tensor** out);
void rs_tensor_free(rs_tensor* T);

const char* rs_status_str(rs_status s);
const char* rs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RS_H */
