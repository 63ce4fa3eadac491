// Internal declarations of the RS library: handle structs, error plumbing and
// the host-side launchers of the HIP kernels.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <atomic>
#include <mutex>
#include <vector>

#include "../../include/rs.h"

namespace rs {

// ---- error plumbing ------------------------------------------------------
void set_error(const std::string& msg);
const char* last_error();

struct Error {
  rs_status status;
  std::string msg;
};

#define RS_HIP(expr)                                                               \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess)                                                          \
      throw ::rs::Error{_e == hipErrorOutOfMemory ? RS_E_NOMEM : RS_E_DEVICE,      \
                        std::string(#expr) + ": " + hipGetErrorString(_e)};        \
  } while (0)

#define RS_REQUIRE(cond, msg)                                                      \
  do {                                                                             \
    if (!(cond)) throw ::rs::Error{RS_E_INVALID, (msg)};                           \
  } while (0)

// ---- quadrature (host, FP64) ----------------------------------------------
struct Table {
  std::vector<double> t, a;   // R entries
  int R = 0, R_l = 0, n_s = 0;
  double S0 = 0, S_l0 = 0;
};
Table build_table(const rs_grid& g, const rs_fdesc& f);

// ---- device buffer that frees itself (stream-ordered) ---------------------
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipStream_t s = nullptr;
  DevBuf() = default;
  DevBuf(size_t nbytes, hipStream_t st);
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept { *this = std::move(o); }
  DevBuf& operator=(DevBuf&& o) noexcept;
  ~DevBuf();
  void reset();
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// Two events recorded on the launch stream immediately before and after the
// main kernel of a contraction (the core), or null for none.
struct KernelTimer {
  hipEvent_t begin = nullptr, end = nullptr;
};

}  // namespace rs

struct rs_ctx {
  int device = 0;
  int num_cu = 256;
  int timing = 0;
  int lds_limit = 65536;   // dynamic LDS bytes one workgroup may use
  size_t hbm_budget = 0;   // admission bound per assembly (0: none)
  double wall_khz = 100000.0;  // rate of the device wall clock
  // pinned host slots for the rank readback of concurrent assemblies
  // (hipHostMalloc'd on first use, freed with the context)
  std::mutex pin_mu;
  std::vector<void*> pin_free, pin_all;
  // references: the handle returned by rs_ctx_create plus one per live
  // tensor; the context is deleted when the last one is released, so a
  // tensor freed after rs_ctx_destroy still finds it
  std::atomic<int> refs{1};
  // a second stream of the context (default priority): the side matrices of
  // an assembly run there while the eigensolver, which they do not feed,
  // runs on the caller's stream
  hipStream_t aux = nullptr;
  ~rs_ctx();
};

namespace rs {
void ctx_release(rs_ctx* c);
// a counted reference to a context, released after the members declared
// after it (declare it first)
struct CtxRef {
  rs_ctx* p = nullptr;
  CtxRef() = default;
  CtxRef(const CtxRef&) = delete;
  CtxRef& operator=(const CtxRef&) = delete;
  void set(rs_ctx* c) {
    c->refs.fetch_add(1);
    p = c;
  }
  ~CtxRef() {
    if (p) ctx_release(p);
  }
};
}  // namespace rs

struct rs_factors {
  rs_grid grid;
  rs_fdesc fdesc;
  rs::Table table;
  double* t_dev = nullptr;  // R
  double* a_dev = nullptr;  // R
  int device = 0;
};

struct rs_tensor {
  rs::CtxRef ctx_ref;   // first: released after every buffer below
  rs_ctx* ctx = nullptr;
  int64_t N = 0, n = 0;
  double b = 0, h = 0;
  int R = 0, R_l = 0, n_s = 0, kernel = 0, prec = 0, interp = 6;
  double lambda = 0;
  rs::Table table;
  int r[3] = {0, 0, 0};
  int p[3] = {0, 0, 0};
  double sigma1[3] = {0, 0, 0}, sig_kept[3] = {0, 0, 0}, sig_next[3] = {0, 0, 0};
  int rank_capped = 0;
  hipStream_t stream = nullptr;  // stream the tensor's buffers were allocated on
  rs::DevBuf t_dev, a_dev;       // quadrature table
  rs::DevBuf pos, q;             // N x 3, N
  rs::DevBuf Q[3];               // n x r_l row-major
  rs::DevBuf beta;               // r1 x r2 x r3
  rs::DevBuf T2;                 // n x n x r3: beta x_1 V1 x_2 V2 (long-range, modes 1,2 expanded)
  rs::DevBuf T2f, V3f;           // FP32 copies of T2 and V3 (RS_FP32 tensors only)
  rs::DevBuf t2exp;              // 1 int: the split grid's scale exponent of T2 (split tensors)
  // short-range binning: bricks of 8^3 cells; pairs (brick, particle) sorted by particle
  int nb = 0;                    // bricks per axis
  int64_t n_pairs = 0;
  rs::DevBuf brick_start;        // nb^3 + 1
  rs::DevBuf brick_list;         // n_pairs particle indices
  rs::DevBuf brick_active;       // 1 + active_cap ints: count, then touched bricks
  int64_t active_cap = 0;
  // stage timing: events[k] recorded before stage k, events[RS_STAGE_COUNT] at the end
  std::vector<hipEvent_t> events;
  int timing_mode = 0;          // 1: every stage and eigen phase, 2: the grid stage only, 3: the core kernel only
  uint32_t recorded = 0;        // bit k: events[k] was recorded
  // eigensolver phases: eig_events[k] before phase k, eig_events[RS_EIG_PHASES] at the end
  std::vector<hipEvent_t> eig_events;
  // timing mode 3: around the core's main kernel launch
  rs::KernelTimer kevents;
  ~rs_tensor() {
    if (kevents.begin) (void)hipEventDestroy(kevents.begin);
    if (kevents.end) (void)hipEventDestroy(kevents.end);
    for (hipEvent_t e : events)
      if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : eig_events)
      if (e) (void)hipEventDestroy(e);
  }
};

namespace rs {

// ---- kernel launchers (k_*.hip) -------------------------------------------

// k_factor.hip
// flags[0] |= 1 for a non-finite position/charge, |= 2 for a position outside [-b,b]
void launch_validate(const double* pos, const double* q, int64_t N, double b, int* flags,
                     hipStream_t s);
// Side matrices U[l][i + j*n] = exp(-t_k^2 (x_i - x_{nu,l})^2), j = k*N + nu, k < R_l;
// xi[j] = q[nu] a_k, w[j] = |xi_j|^{2/3}.
// U (FP64, may be null) and/or planes16 (FP16 split planes of the
// projection, [mode][hi, lo][K][kp], scale 2^14; may be null); with on_side
// the side matrices go to side_s and the weights to s
void launch_side_matrices(const double* pos, const double* q, const double* t, const double* a,
                          int64_t N, int R_l, int64_t n, double b, double* U, double* xi,
                          double* w, double* sw, hipStream_t s, void* planes16 = nullptr,
                          int64_t kp = 0, hipStream_t side_s = nullptr, bool on_side = false);

// k_dot.hip : scalar product of two RS tensors (the touched-brick correction
// and fixed-order reductions; the long-long term is formed by the caller)
struct DotSide {
  const double *T2 = nullptr, *V3 = nullptr, *pos = nullptr, *q = nullptr, *t = nullptr,
               *a = nullptr;
  const int *start = nullptr, *list = nullptr;
  int r3 = 0, R = 0, R_l = 0, w = 0;
};
size_t dot_partials_bytes();
void launch_dot_partial(const double* x, const double* y, int64_t count, double* partial,
                        hipStream_t s);
// correction over the touched cells, one partial per brick column (nb^2 of them)
void launch_dot_cols(const DotSide& A, const DotSide& B, int nb, int64_t n, double b,
                     double* partials, hipStream_t s);
void launch_dot_final(const double* ll, const double* pc, int64_t ncols, double* out,
                      hipStream_t s);

// Toeplitz factors of the RS RBF matrix: T (R x n x n) and Acat (n x R n)
void launch_rbf_toeplitz(const double* t, const double* a, int R, int R_l, int64_t n, double h,
                         int w, double* T, double* Acat, hipStream_t s);
// DV = column-wise finite differences of V (n x r row-major) with spacing h:
// central inside, one-sided at the ends
void launch_fd_rows(const double* V, int64_t n, int r, double h, double* DV, hipStream_t s);

// k_gemm64.hip : FP64 MFMA GEMM, C[bt](m,n) = sum_k A[bt](m,k) B[bt](k,n) kscale[k]
struct Gemm64 {
  int64_t M = 0, N = 0, K = 0;
  int batch = 1;
  const double* A = nullptr; int64_t sam = 0, sak = 0, sab = 0;
  const double* B = nullptr; int64_t sbk = 0, sbn = 0, sbb = 0;
  double* C = nullptr; int64_t scm = 0, scn = 0, scb = 0;
  const double* kscale = nullptr;   // optional, length K (same for all batches)
  int upper_only = 0;               // square symmetric output: compute tiles on/above the diagonal, mirror
  int nontemporal = 0;              // streaming stores for a write-once output
  // optional column blocks: output column j goes to (j / ccb) sccb + (j % ccb) scn
  // (0: plain j scn), so that an (i, c) column pair can land in another layout
  int64_t ccb = 0, sccb = 0;
};
// Splits K so that at least ~2 waves of workgroups fill the chip; partial
// sums are reduced in a fixed order (deterministic).  `work` must hold
// gemm64_workspace_bytes(g, num_cu) bytes (may be null when that is 0).
size_t gemm64_workspace_bytes(const Gemm64& g, int num_cu);
void gemm64(const Gemm64& g, int num_cu, double* work, hipStream_t s);
// grid (n^2 x n, row-major) = T2 (n^2 x r3) V3^T (V3: n x r3), FP64, streamed
// through an LDS-resident V3 panel; returns false (nothing launched) when the
// panel of r3 does not fit the LDS, for the caller to use gemm64.
bool grid64_stream(const double* T2, const double* V3, int64_t n, int r3, double* grid, int num_cu,
                   int lds_limit, hipStream_t s);
// Range-finder sketch Y[bt] (M x N col-major) = A[bt] (M x K col-major) Omega_bt,
// Omega_bt[k, c] = scale[bt*scale_stride + k] * u(seed, bt, k, c), u uniform in [-1, 1)
// (scale null: 1).
size_t sketch64_workspace_bytes(int64_t M, int64_t K, int batch, int64_t N, int num_cu);
void sketch64(const double* A, int64_t M, int64_t K, int64_t sab, const double* scale,
              int64_t scale_stride, int batch, int64_t N, uint64_t seed, double* Y, int64_t scm,
              int64_t scn, int num_cu, double* work, hipStream_t s);

// k_gram.hip: G (3 x n x n) = U diag(w) U^T per mode by the Gaussian-product
// identity, from the particle coordinates, the nodes t and the weights w
size_t gauss_gram_workspace_bytes(int64_t N, int R_l, int64_t n, int num_cu);
void launch_gauss_gram(const double* pos, const double* t, const double* w, int64_t N, int R_l,
                       int64_t n, double b, double* G, double* work, int num_cu, hipStream_t s);

// k_eig.hip
void launch_identity(double* I, int64_t n, int modes, hipStream_t s);
void launch_symmetrize(double* B, int p, int modes, hipStream_t s);
void launch_perturb(double* Y, const double* G, int64_t n, int p, int modes, uint64_t seed,
                    hipStream_t s);
// Partial sums of |Y_mode|_F^2 (sketch_eta_bytes(modes) bytes), then
// Y += eta * uniform noise with eta = rel sqrt(|Y_mode|_F^2 / (n p)), the
// scale of the perturbation taken from the range-finder sketch
size_t sketch_eta_bytes(int modes);
void launch_sketch_eta(const double* Y, int64_t n, int p, int modes, double* part, hipStream_t s);
void launch_perturb_eta(double* Y, const double* part, int64_t n, int p, int modes, double rel,
                        uint64_t seed, hipStream_t s);
// Cholesky C = L L^T in place (lower, col-major), one workgroup per mode; the
// shifted variant adds 11 (nrows p + p (p+1)) u tr(C) to the diagonal first.
// fail |= fail_bit on a non-positive pivot.
void launch_chol(double* C, int p, int64_t nrows, int modes, int shifted, int lds_limit, int* fail,
                 int fail_bit, hipStream_t s);
// Y (n x p row-major per mode) <- Y L^{-T}
void launch_trsm_rows(double* Y, const double* L, int64_t n, int p, int modes, int lds_limit,
                      hipStream_t s);
// Dense symmetric eigensolver of B (p x p per mode), in steps so that the
// caller can orthonormalise the eigenvectors with its Cholesky QR:
//  tridiag: B = H T H^T (Householder vectors and d, e into ws);
//  values_vectors: eigenvalues of T (descending) onto the diagonal of B and
//    into ws; the rc leading eigenvectors of T by inverse iteration into Z
//    (p x rc row-major per mode, unit columns, not yet orthogonal);
//  backtransform: Z <- H Z.
// ws is scratch of eig_sym_workspace_bytes(p, rc, modes).
size_t eig_sym_workspace_bytes(int p, int rc, int modes);
void launch_eig_tridiag(double* B, double* ws, int p, int rc, int modes, int lds_limit,
                        hipStream_t s);
void launch_eig_values_vectors(double* B, double* ws, double* Z, int p, int rc, int modes,
                               int lds_limit, hipStream_t s);
void launch_eig_backtransform(double* Z, double* ws, int p, int rc, int modes, hipStream_t s);
// Sort eigenvalues descending, choose ranks; writes perm[mode][p], info doubles.
struct RankInfo {
  int r[3];
  int capped[3];
  double lam1[3], lam_kept[3], lam_next[3];
};
void launch_rank_select(const double* B, int p, int modes, double eps2, const int* fixed,
                        int r_max, int* perm, RankInfo* info_dev, hipStream_t s);
// Qout (n x r row-major) = Q0 (n x p col-major) * V[:, perm[0..r)], then
// canonical signs (largest-magnitude entry of each column positive).
void launch_gather_cols(const double* Z, int ldz, const int* perm, int p, int r, double* Wr,
                        hipStream_t s);
void launch_canonical_signs(double* Qrow, int64_t n, int r, hipStream_t s, double* W = nullptr,
                            int64_t m = 0);
// per-mode pointers and ranks, passed by value to the three-mode kernels
struct Mode3 {
  double* p[3];
  int r[3];
};
// gather_cols and canonical_signs for the three modes in one launch each:
// mode l reads Z + l zstride and perm + l p, writes Wr.p[l] (p x Wr.r[l]);
// signs are fixed on Q.p[l] (n x Q.r[l]) and carried to W.p[l] (m x r, or null)
void launch_gather_cols3(const double* Z, int ldz, int64_t zstride, const int* perm, int p,
                         const Mode3& Wr, hipStream_t s);
void launch_canonical_signs3(const Mode3& Q, int64_t n, const Mode3& W, int64_t m, hipStream_t s);

// k_gemm64.hip : C[b] = Z[b]^T diag(w) Z[b] for Z[b] K x p row-major at stride zstride, p <= 128
// (false otherwise: nothing launched); C exactly symmetric, p x p per batch.
size_t gram_stream_workspace_bytes(int p, int64_t K, int batch, int num_cu);
bool gram_stream(const double* Z, int64_t zstride, const double* w, int p, int64_t K, int batch,
                 double* C, int num_cu, double* work, hipStream_t s);
// beta(a, b*r3 + c) = sum_j U1t[j*r1+a] xi[j] U2t[j*r2+b] U3t[j*r3+c]
size_t core64_workspace_bytes(int r1, int r2, int r3, int64_t K, int num_cu);
void core64(const double* U1t, const double* U2t, const double* U3t, const double* xi,
            int r1, int r2, int r3, int64_t K, double* beta, int num_cu, double* work,
            hipStream_t s, const KernelTimer* kt = nullptr);

// fixed-order sum of `splits` partial arrays of `total` doubles
void core64_reduce(const double* part, int splits, int64_t total, double* out, hipStream_t s);

// k_mixed.hip: split-FP16 (prec RS_MIXED_FP16) or split-BF16 contractions
// U~^T (K x r, FP64) = U^T V in split precision: U n x K column-major, V n x r row-major
size_t proj_mixed_workspace_bytes(int64_t n, int64_t K, int r, bool a_given);
// a_planes: the FP16 planes of U written by the side-matrix kernel (scale
// 2^14), or null to split U here
void proj_mixed(int prec, const double* U, const void* a_planes, int64_t n, int64_t K,
                const double* V, int r, double* Ut, void* work, hipStream_t s);
// T2 (n x n x r3, FP64) = X x_2 V2 in split precision, X[b][i1][c] (r2 x n x r3)
size_t expand2_mixed_workspace_bytes(int64_t n, int r2, int r3);
// grid_work (the grid_mixed workspace, or null): also write the grid's A
// planes of T2 and their exponent there, for grid_mixed(..., planes_ready);
// grid_mixed with t2exp splits T2 under that exponent (the same planes)
// t2exp (device int): receives the exponent of the grid's T2 planes
void expand2_mixed(int prec, const double* X, const double* V2, int64_t n, int r2, int r3,
                   double* T2, void* work, void* grid_work, int* t2exp, hipStream_t s);
void grid_mixed_planes(void* work, int64_t n, int r3, void** planes, int** exps, int64_t* kp);
size_t core_mixed_workspace_bytes(int r1, int r2, int r3, int64_t K, int num_cu);
void core_mixed(int prec, const double* U1t, const double* U2t, const double* U3t, const double* xi,
                int r1, int r2, int r3, int64_t K, double* beta, int num_cu, double* work,
                hipStream_t s, const KernelTimer* kt = nullptr);
// FP32 grid[(i1 i2), i3] = sum_c T2[(i1 i2), c] V3[i3, c]; work holds
// grid_mixed_workspace_bytes(n, r3) bytes
size_t grid_mixed_workspace_bytes(int64_t n, int r3);
void grid_mixed(int prec, const double* T2, const double* V3, int64_t n, int r3, float* grid,
                void* work, int num_cu, hipStream_t s,
                bool planes_ready = false, const int* t2exp = nullptr);

// k_short.hip
struct ShortBins {
  int nb = 0;
  int64_t n_pairs = 0;
};
// Count (brick, particle) pairs; returns the total on the host (synchronizes).
void short_bin_count(const double* pos, int64_t N, int64_t n, double b, int n_s, int nb,
                     int* counts, hipStream_t s);
void short_bin_fill(const double* pos, int64_t N, int64_t n, double b, int n_s, int nb,
                    const int* start, int* cursor, int* list, hipStream_t s);
// Sorts every brick's list and writes the touched bricks to active[1..]
// (count in active[0]; at most active_cap entries, see short_active_capacity).
void short_bin_sort(const int* start, int* list, int nbricks, int* active, int64_t active_cap,
                    hipStream_t s);
// Upper bound on the number of bricks touched by the windows of N particles.
int64_t short_active_capacity(int64_t N, int n_s, int nb);
void exclusive_scan_int(const int* in, int* out, int count, hipStream_t s);
// the same with a caller-provided temporary of at least exclusive_scan_bytes(count)
size_t exclusive_scan_bytes(int count);
void exclusive_scan_int(const int* in, int* out, int count, void* tmp, size_t tmp_bytes,
                        hipStream_t s);
// grid (FP64 or FP32) += sum over particles of the short-range windows, or,
// with dax = 0, 1, 2, += its finite difference along that axis (central,
// one-sided at the grid ends; brick lists then built for windows of n_s + 2)
void short_gather(void* grid, int grid_fp32, const double* pos, const double* q,
                  const double* t, const double* a, int R, int R_l, int64_t n, double b,
                  int n_s, int nb, const int* start, const int* list, const int* active,
                  int64_t active_cap, int num_cu, hipStream_t s, int dax = -1);

// k_noalloc.hip: one file-scope device array per GPU for the entry points that
// allocate nothing (8 MiB: the per-particle evaluations of up to 131072
// particles); its address per device is looked up once, at context creation
constexpr int64_t kNoAllocScratchDoubles = (int64_t)1 << 20;
void noalloc_scratch_init(int device);   // with `device` current; idempotent
double* noalloc_scratch(int device);     // RS_E_DEVICE if not set up

// k_eval.hip
// vals[m] (part 0/1/2) and optionally grad (M x 3) and self terms at points
struct EvalOut {
  double* val = nullptr;       // long (+short) value per point
  double* grad = nullptr;      // M x 3 gradient of the long part, or null
  double* selfv = nullptr;     // self term g_j (when points are the particles), or null
  double* selfg = nullptr;     // M x 3 gradient of the self term, or null
};
// With FP32 copies of the field (RS_FP32 tensors) the long-range values,
// gradients and self terms are evaluated in FP32 arithmetic (outputs FP64).
void launch_eval_long(const rs_tensor* T, int64_t M, const double* pts, int with_self,
                      const EvalOut& out, hipStream_t s);
// out[i] = (float)in[i]
void launch_to_float(const double* in, int64_t count, float* out, hipStream_t s);
void launch_eval_short(const rs_tensor* T, int64_t M, const double* pts, double* vals,
                       int accumulate, hipStream_t s);
// M x 3 gradient of the short-range part at the points (analytic per term)
void launch_eval_short_grad(const rs_tensor* T, int64_t M, const double* pts, double* grad,
                            int accumulate, hipStream_t s);
// out[i] = <grad[i, :], normals[i, :]>
void launch_normal_dot(const double* grad, const double* normals, int64_t M, double* out,
                       hipStream_t s);
// E = 1/2 sum_j q_j (v_j - q_j g_j); dEdq_j = v_j - q_j g_j (optional)
void launch_energy_reduce(const double* q, const double* v, const double* g, int64_t N,
                          double* E, double* dEdq, hipStream_t s);
void launch_forces(const double* q, const double* gradv, const double* gradg, int64_t N,
                   double scale, double* F, hipStream_t s);

}  // namespace rs
