// The extern "C" entry points of the RS library: argument checks, device
// memory, and the order of the kernel launches of one RS-Tucker assembly.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>

#include "rs_internal.h"

namespace rs {

void ctx_release(rs_ctx* c) {
  if (c->refs.fetch_sub(1) == 1) delete c;
}

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
const char* last_error() { return g_err.c_str(); }

// ---- device memory: a stream-aware caching allocator ------------------------
// Device blocks are taken from the driver once and kept: a released block goes
// back to a host-side free list tagged with the stream it was released on.
// A request is served by the smallest cached block that fits (not much
// larger than asked); a block of the same stream is reusable at once (stream
// order puts every earlier use before the new one), a block of another stream
// after that stream's work so far (an event the requesting stream waits on).
// No driver call and no queue packet is spent on the steady-state path, so
// consecutive assemblies reuse their buffers without stalls.  Requests are
// rounded to 512 bytes (below 1 MiB) or 2 MiB; cached memory is returned only
// when the driver runs out (then every cached block of the device is freed
// after a device synchronisation) or by rs_ctx_trim().
namespace {
struct CachedBlock {
  void* p;
  hipStream_t s;
  bool idle;   // no work on it can be pending (its stream was synchronised and released)
};
struct DeviceCache {
  std::multimap<size_t, CachedBlock> free_blocks;  // by size
};
struct BlockInfo {
  int device;
  size_t bytes;
};
// heap-held and never destroyed: buffers may be released during process exit
std::mutex& g_cache_mu = *new std::mutex;
std::map<int, DeviceCache>& g_caches = *new std::map<int, DeviceCache>;
std::map<void*, BlockInfo>& g_blocks = *new std::map<void*, BlockInfo>;  // every block taken from the driver

size_t round_request(size_t n) {
  const size_t small = 512, large = (size_t)2 << 20;
  return n < ((size_t)1 << 20) ? (n + small - 1) / small * small : (n + large - 1) / large * large;
}

void release_cached(int device, DeviceCache& c) {  // caller holds the lock
  if (c.free_blocks.empty()) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(device);
  (void)hipDeviceSynchronize();
  for (auto& kv : c.free_blocks) {
    (void)hipFree(kv.second.p);
    g_blocks.erase(kv.second.p);
  }
  c.free_blocks.clear();
  (void)hipSetDevice(cur);
}
}  // namespace

static void* cache_alloc(size_t nbytes, hipStream_t st) {
  int dev = 0;
  RS_HIP(hipGetDevice(&dev));
  const size_t want = round_request(nbytes);
  const size_t limit = want + want / 4 + ((size_t)2 << 20);
  std::lock_guard<std::mutex> lock(g_cache_mu);
  DeviceCache& c = g_caches[dev];
  auto best = c.free_blocks.end();
  for (auto it = c.free_blocks.lower_bound(want); it != c.free_blocks.end() && it->first <= limit; ++it) {
    if (it->second.idle || it->second.s == st) { best = it; break; }
    if (best == c.free_blocks.end()) best = it;
  }
  if (best != c.free_blocks.end()) {
    CachedBlock b = best->second;
    c.free_blocks.erase(best);
    if (!b.idle && b.s != st) {
      hipEvent_t ev;
      RS_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      RS_HIP(hipEventRecord(ev, b.s));
      RS_HIP(hipStreamWaitEvent(st, ev, 0));
      RS_HIP(hipEventDestroy(ev));
    }
    return b.p;
  }
  void* p = nullptr;
  if (hipMalloc(&p, want) != hipSuccess) {
    (void)hipGetLastError();
    release_cached(dev, c);
    RS_HIP(hipMalloc(&p, want));
  }
  g_blocks[p] = BlockInfo{dev, want};
  return p;
}

static void cache_free(void* p, hipStream_t st) {
  std::lock_guard<std::mutex> lock(g_cache_mu);
  auto it = g_blocks.find(p);
  if (it == g_blocks.end()) return;  // not taken by cache_alloc (cannot happen)
  g_caches[it->second.device].free_blocks.emplace(it->second.bytes, CachedBlock{p, st, false});
}

// Detach the cached blocks of stream `st` from it (the caller has
// synchronised `st`), so that no later allocation records an event on it.
static void cache_forget_stream(hipStream_t st) {
  std::lock_guard<std::mutex> lock(g_cache_mu);
  for (auto& dc : g_caches)
    for (auto& kv : dc.second.free_blocks)
      if (kv.second.s == st) {
        kv.second.idle = true;
        kv.second.s = nullptr;
      }
}

static void cache_trim(int device) {
  std::lock_guard<std::mutex> lock(g_cache_mu);
  auto it = g_caches.find(device);
  if (it != g_caches.end()) release_cached(device, it->second);
}

DevBuf::DevBuf(size_t nbytes, hipStream_t st) : bytes(nbytes), s(st) {
  if (nbytes) p = cache_alloc(nbytes, st);
}
DevBuf& DevBuf::operator=(DevBuf&& o) noexcept {
  if (this != &o) {
    reset();
    p = o.p;
    bytes = o.bytes;
    s = o.s;
    o.p = nullptr;
    o.bytes = 0;
  }
  return *this;
}
DevBuf::~DevBuf() { reset(); }
void DevBuf::reset() {
  if (p) cache_free(p, s);
  p = nullptr;
  bytes = 0;
}

template <class F>
static rs_status guarded(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    set_error(e.msg);
    return e.status;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return RS_E_NOMEM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return RS_E_DEVICE;
  }
}

struct Plan {
  int64_t N, n, K;
  int R, R_l, n_s;
  int r_max, p, power_iters, interp, prec, gram, sketch;
  int os, p_first;   // oversampling; first subspace size of the rank rule's search
  int als;           // ALS refinement sweeps
  int fixed[3];
  double eps;
};

static Plan make_plan(const rs_factors* f, int64_t N, const rs_aopts* o) {
  Plan P;
  P.N = N;
  P.n = f->grid.n;
  P.R = f->table.R;
  P.R_l = f->table.R_l;
  P.n_s = f->table.n_s;
  P.K = N * P.R_l;
  rs_aopts d{};
  if (o) d = *o;
  RS_REQUIRE(N >= 1, "N must be >= 1");
  RS_REQUIRE(N <= (int64_t)1 << 26, "N too large");
  RS_REQUIRE(d.eps_tucker >= 0 && d.eps_tucker < 1 && std::isfinite(d.eps_tucker),
             "eps_tucker must be in [0, 1)");
  P.eps = d.eps_tucker;
  P.r_max = d.r_max > 0 ? d.r_max : (int)std::min<int64_t>(P.n, 256);
  RS_REQUIRE(P.r_max <= P.n, "r_max must not exceed n");
  int rcap = P.r_max;
  bool all_fixed = true;
  for (int l = 0; l < 3; ++l) {
    P.fixed[l] = d.fixed_ranks[l];
    RS_REQUIRE(P.fixed[l] >= 0 && P.fixed[l] <= P.n, "fixed rank outside [0, n]");
    if (P.fixed[l] == 0) all_fixed = false;
  }
  if (all_fixed) rcap = std::max(P.fixed[0], std::max(P.fixed[1], P.fixed[2]));
  else
    for (int l = 0; l < 3; ++l) rcap = std::max(rcap, P.fixed[l]);
  // the subspace oversampling sets how well the basis resolves the
  // directions at the rank threshold: with fixed ranks the subspace is sized
  // from them, so it gets a wider margin than the r_max budget of the rank rule
  const int os = d.oversample > 0 ? d.oversample : (all_fixed ? 48 : 16);
  int64_t p = std::min<int64_t>(P.n, (int64_t)rcap + os);
  if (p % 2) ++p;
  if (p > P.n) p = P.n;
  P.p = (int)p;
  P.os = os;
  RS_REQUIRE(P.p <= 512 || P.p == P.n, "r_max + oversample must not exceed 512 (eigensolver subspace)");
  // the rank rule's subspace search starts at subspace_min (even; 0, the
  // default, is the full size: no search); fixed ranks size the subspace
  // directly
  RS_REQUIRE(d.subspace_min >= 0, "subspace_min must be >= 0");
  int pf = d.subspace_min > 0 ? d.subspace_min : P.p;
  if (pf % 2) ++pf;
  P.p_first = all_fixed ? P.p : std::min(P.p, pf);
  RS_REQUIRE(d.als_sweeps >= 0 && d.als_sweeps <= 16, "als_sweeps must be in [0, 16]");
  P.als = d.als_sweeps;
  RS_REQUIRE(rcap <= 512, "r_max and fixed ranks must not exceed 512");
  P.power_iters = d.power_iters >= 0 ? d.power_iters : 0;
  RS_REQUIRE(P.power_iters <= 8, "power_iters must be <= 8");
  P.interp = d.interp_order > 0 ? d.interp_order : 6;
  RS_REQUIRE(P.interp % 2 == 0 && P.interp <= 8 && P.interp <= P.n, "interp_order must be even, <= 8");
  P.prec = d.prec;
  P.gram = d.gram;
  P.sketch = d.sketch;
  RS_REQUIRE(P.sketch == 0 || P.sketch == 1, "sketch must be 0 (Gram) or 1 (side matrix)");
  RS_REQUIRE(P.gram == RS_GRAM_IDENTITY || P.gram == RS_GRAM_GEMM, "unknown Gram method");
  RS_REQUIRE(P.prec == RS_FP64 || P.prec == RS_MIXED_FP16 || P.prec == RS_MIXED_BF16 ||
                 P.prec == RS_FP32,
             "unknown precision");
  RS_REQUIRE(P.R - P.R_l <= 64 && P.R_l <= 64, "at most 64 long and 64 short terms");
  return P;
}

static int bricks_per_axis(int64_t n) { return (int)((n + 7) / 8); }

// The contractions' arithmetic of an assembly precision: RS_FP32 assembles
// with the split-FP16 contractions (and evaluates its field in FP32).
static int contraction_prec(int prec) { return prec == RS_FP32 ? RS_MIXED_FP16 : prec; }

// FP32 copies of T2 and V3 for the FP32 evaluation of RS_FP32 tensors.
static void make_fp32_field(rs_tensor* T, hipStream_t s) {
  if (T->prec != RS_FP32) return;
  const int64_t nt2 = T->n * T->n * T->r[2], nv3 = T->n * T->r[2];
  T->T2f = DevBuf((size_t)nt2 * sizeof(float), s);
  T->V3f = DevBuf((size_t)nv3 * sizeof(float), s);
  launch_to_float(T->T2.as<double>(), nt2, T->T2f.as<float>(), s);
  launch_to_float(T->Q[2].as<double>(), nv3, T->V3f.as<float>(), s);
}

// Record the start of `stage` (and so the end of the previous one) when the
// tensor carries timing events.
static void mark(rs_tensor* T, int stage, hipStream_t s) {
  if (T->events.empty()) return;
  // grid-only timing records the grid kernel's start and end and the end of
  // the assembly; every other event would put a marker between two launches
  if (T->timing_mode == 2 && stage != RS_STAGE_GRID && stage != RS_STAGE_SHORT &&
      stage != RS_STAGE_COUNT)
    return;
  // core-kernel timing records the two events around that launch (inside the
  // core launchers) and the end of the assembly
  if (T->timing_mode == 3 && stage != RS_STAGE_COUNT) return;
  RS_HIP(hipEventRecord(T->events[stage], s));
  T->recorded |= 1u << stage;
}

// Gram matrices of the three modes into G (3 x n x n); U, xi, w computed into
// caller-provided buffers.
static Gemm64 gram_gemm(const Plan& P, const double* U, const double* w, double* G) {
  Gemm64 g;  // G = U diag(w) U^T per mode (upper tiles, mirrored)
  g.M = P.n;
  g.N = P.n;
  g.K = P.K;
  g.batch = 3;
  g.A = U; g.sam = 1; g.sak = P.n; g.sab = P.n * P.K;
  g.B = U; g.sbk = P.n; g.sbn = 1; g.sbb = P.n * P.K;
  g.C = G; g.scm = P.n; g.scn = 1; g.scb = P.n * P.n;
  g.kscale = w;
  g.upper_only = 1;
  return g;
}

static size_t gram_workspace_bytes(const Plan& P, int method, int ncu) {
  return method == RS_GRAM_GEMM ? gemm64_workspace_bytes(gram_gemm(P, nullptr, nullptr, nullptr), ncu)
                                : gauss_gram_workspace_bytes(P.N, P.R_l, P.n, ncu);
}

// Side matrices, weights and the three Gram matrices (method RS_GRAM_*).
// `work`: gram_workspace_bytes(P, method, ncu) bytes, or null to allocate here.
static void run_factors_and_gram(rs_ctx* ctx, const rs_factors* f, const Plan& P,
                                 const double* pos, const double* q, double* U, double* xi,
                                 double* w, double* sw, double* G, int method, hipStream_t s,
                                 rs_tensor* T = nullptr, double* work = nullptr,
                                 void* planes16 = nullptr, int64_t kp = 0,
                                 hipStream_t side_s = nullptr, bool on_side = false) {
  launch_side_matrices(pos, q, f->t_dev, f->a_dev, P.N, P.R_l, P.n, f->grid.b, U, xi, w, sw, s,
                       planes16, kp, side_s, on_side);
  if (T) mark(T, RS_STAGE_GRAM, s);
  DevBuf own;
  if (!work) {
    own = DevBuf(gram_workspace_bytes(P, method, ctx->num_cu), s);
    work = own.as<double>();
  }
  if (method == RS_GRAM_GEMM)
    gemm64(gram_gemm(P, U, w, G), ctx->num_cu, work, s);
  else
    launch_gauss_gram(pos, f->t_dev, w, P.N, P.R_l, P.n, f->grid.b, G, work, ctx->num_cu, s);
}

// Non-owning view of a piece of an arena, with DevBuf's accessors.
struct Span {
  void* p = nullptr;
  size_t bytes = 0;
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// The caller's stream waits for work put on the context's second stream:
// at join(), or when the assembly leaves early (declared after the arena
// that work writes, so that the wait is enqueued before the arena goes back
// to the allocator on the caller's stream).
struct SideJoin {
  hipEvent_t start = nullptr, done = nullptr;
  hipStream_t s = nullptr, aux = nullptr;
  void join() {
    if (start && !done && aux && hipEventCreateWithFlags(&done, hipEventDisableTiming) == hipSuccess)
      (void)hipEventRecord(done, aux);
    if (done) {
      (void)hipStreamWaitEvent(s, done, 0);
      (void)hipEventDestroy(done);
      done = nullptr;
    }
    if (start) {
      (void)hipEventDestroy(start);
      start = nullptr;
    }
  }
  ~SideJoin() { join(); }
};

// Scratch carved from one allocation: offsets are 256-byte aligned.
struct Carve {
  size_t total = 0;
  size_t add(size_t bytes) {
    const size_t off = total;
    total += (bytes + 255) & ~(size_t)255;
    return off;
  }
};

// The two-mode expansion T2[i1, i2, c] = sum_{a,b} V1[i1,a] V2[i2,b] beta[a,b,c]
// as two single GEMMs.  The first writes X[b][i1][c] = sum_a V1[i1,a] beta[a,b,c]
// (output column (b, c) of V1 beta_(1) sent to b n r3 + c); the second
// contracts b: T2 row i2, column (i1, c) = sum_b V2[i2,b] X[b][i1 r3 + c],
// sent to i1 n r3 + i2 r3 + c.
// (V1 may be another n x r1 factor, e.g. its finite difference)
static Gemm64 expand1_gemm(const rs_tensor* T, double* X, const double* V1 = nullptr) {
  const int64_t n = T->n;
  const int r1 = T->r[0], r2 = T->r[1], r3 = T->r[2];
  Gemm64 g;  // X[b][i1][c] = (V1 beta_(1))[i1, (b, c)]
  g.M = n; g.N = (int64_t)r2 * r3; g.K = r1;
  g.A = V1 ? V1 : T->Q[0].as<double>(); g.sam = r1; g.sak = 1;
  g.B = T->beta.as<double>(); g.sbk = (int64_t)r2 * r3; g.sbn = 1;
  g.C = X; g.scm = r3; g.scn = 1; g.ccb = r3; g.sccb = n * r3;
  return g;
}

// (V2 and the output may be another factor and buffer)
static Gemm64 expand2_gemm(const rs_tensor* T, const double* X, const double* V2 = nullptr,
                           double* T2out = nullptr) {
  const int64_t n = T->n;
  const int r2 = T->r[1], r3 = T->r[2];
  Gemm64 g;  // T2[i1][i2][c] = sum_b V2[i2, b] X[b][i1 r3 + c]
  g.M = n; g.N = n * r3; g.K = r2;
  g.A = V2 ? V2 : T->Q[1].as<double>(); g.sam = r2; g.sak = 1;
  g.B = X; g.sbk = n * r3; g.sbn = 1;
  g.C = T2out ? T2out : T->T2.as<double>(); g.scm = r3; g.scn = 1; g.ccb = r3; g.sccb = n * r3;
  return g;
}

static Gemm64 grid_gemm(const rs_tensor* T, void* grid, const double* T2 = nullptr,
                        const double* V3 = nullptr) {
  const int64_t n = T->n;
  const int r3 = T->r[2];
  Gemm64 g;  // grid[(i1,i2), i3] = sum_c T2[(i1,i2), c] V3[i3, c]
  g.M = n * n; g.N = n; g.K = r3;
  g.A = T2 ? T2 : T->T2.as<double>(); g.sam = r3; g.sak = 1;
  g.B = V3 ? V3 : T->Q[2].as<double>(); g.sbk = 1; g.sbn = r3;
  g.C = (double*)grid; g.scm = n; g.scn = 1;
  g.nontemporal = 1;
  return g;
}

// Scratch layout of build_expansion: X (n r2 r3), then the GEMM workspaces.
struct ExpansionScratch {
  size_t w1, wk1, wk2, wkg, total;
};

static ExpansionScratch expansion_scratch(const rs_tensor* T, bool with_grid) {
  const int ncu = T->ctx->num_cu;
  ExpansionScratch e{};
  Carve c;
  e.w1 = c.add((size_t)T->n * T->r[1] * T->r[2] * sizeof(double));
  e.wk1 = c.add(gemm64_workspace_bytes(expand1_gemm(T, nullptr), ncu));
  e.wk2 = c.add(T->prec == RS_FP64 ? gemm64_workspace_bytes(expand2_gemm(T, nullptr), ncu)
                                    : expand2_mixed_workspace_bytes(T->n, T->r[1], T->r[2]));
  e.wkg = c.add(!with_grid ? 0
                : T->prec == RS_FP64 ? gemm64_workspace_bytes(grid_gemm(T, nullptr), ncu)
                                     : grid_mixed_workspace_bytes(T->n, T->r[2]));
  e.total = c.total;
  return e;
}

// Expand T2 = beta x_1 V1 x_2 V2 and, when grid != null, the full grid
// (T2 x_3 V3) plus the short-range windows.  T2 must be allocated; scratch
// holds expansion_scratch(T, grid != null).total bytes.
static void build_expansion(rs_tensor* T, void* grid, char* scratch, hipStream_t s) {
  const int64_t n = T->n;
  const int r3 = T->r[2];
  const int ncu = T->ctx->num_cu;
  const ExpansionScratch e = expansion_scratch(T, grid != nullptr);
  double* X = (double*)(scratch + e.w1);
  mark(T, RS_STAGE_EXPAND1, s);
  gemm64(expand1_gemm(T, X), ncu, (double*)(scratch + e.wk1), s);
  mark(T, RS_STAGE_EXPAND2, s);
  if (T->prec == RS_FP64)
    gemm64(expand2_gemm(T, X), ncu, (double*)(scratch + e.wk2), s);
  else
    expand2_mixed(contraction_prec(T->prec), X, T->Q[1].as<double>(), n, T->r[1], r3,
                  T->T2.as<double>(), scratch + e.wk2, grid ? scratch + e.wkg : nullptr,
                  T->t2exp.as<int>(), s);
  if (grid && T->prec != RS_FP64) {
    mark(T, RS_STAGE_GRID, s);
    grid_mixed(contraction_prec(T->prec), T->T2.as<double>(), T->Q[2].as<double>(), n, r3, (float*)grid,
               scratch + e.wkg, ncu, s, true);
    mark(T, RS_STAGE_SHORT, s);
    short_gather(grid, 1, T->pos.as<double>(), T->q.as<double>(), T->t_dev.as<double>(),
                 T->a_dev.as<double>(), T->R, T->R_l, n, T->b, T->n_s, T->nb,
                 T->brick_start.as<int>(), T->brick_list.as<int>(), T->brick_active.as<int>(),
                 T->active_cap, ncu, s);
  } else if (grid) {
    mark(T, RS_STAGE_GRID, s);
    if (!grid64_stream(T->T2.as<double>(), T->Q[2].as<double>(), n, r3, (double*)grid, ncu,
                       T->ctx->lds_limit, s))
      gemm64(grid_gemm(T, grid), ncu, (double*)(scratch + e.wkg), s);
    mark(T, RS_STAGE_SHORT, s);
    short_gather(grid, 0, T->pos.as<double>(), T->q.as<double>(), T->t_dev.as<double>(),
                 T->a_dev.as<double>(), T->R, T->R_l, n, T->b, T->n_s, T->nb,
                 T->brick_start.as<int>(), T->brick_list.as<int>(), T->brick_active.as<int>(),
                 T->active_cap, ncu, s);
  }
  mark(T, RS_STAGE_COUNT, s);
}

// The r dominant eigenvectors of the symmetric n x n matrix G (row-major)
// into V (n x r row-major, canonical signs), by the same steps as the
// assembly's eigensolver for one matrix: the range finder Y = G Omega,
// shifted and plain Cholesky QR, Rayleigh-Ritz, the dense eigensolver,
// Cholesky QR of the eigenvectors, V = Q W.  Breakdowns set bits of *fail.
static void dominant_eigvecs(const rs_ctx* ctx, const double* G, int64_t n, int r, double* V,
                             int* fail, hipStream_t s) {
  const int ncu = ctx->num_cu, lds = ctx->lds_limit;
  int64_t pp = std::min<int64_t>(n, (int64_t)r + 48);
  if (pp % 2) ++pp;
  if (pp > n) pp = n;
  const int p = (int)pp;
  DevBuf Q0((size_t)n * p * sizeof(double), s), Bm((size_t)p * p * sizeof(double), s);
  if (p == n) {
    launch_identity(Q0.as<double>(), n, 1, s);
    RS_HIP(hipMemcpyAsync(Bm.p, G, (size_t)n * n * sizeof(double), hipMemcpyDeviceToDevice, s));
  } else {
    DevBuf Y((size_t)n * p * sizeof(double), s), Cq((size_t)p * p * sizeof(double), s);
    DevBuf eta(sketch_eta_bytes(1), s);
    Gemm64 yty;   // Cq = Q0^T Q0 (upper)
    yty.M = p; yty.N = p; yty.K = n; yty.upper_only = 1;
    yty.A = Q0.as<double>(); yty.sam = 1; yty.sak = p;
    yty.B = Q0.as<double>(); yty.sbk = p; yty.sbn = 1;
    yty.C = Cq.as<double>(); yty.scm = p; yty.scn = 1;
    Gemm64 gq;    // Y = G Q0
    gq.M = n; gq.N = p; gq.K = n;
    gq.A = G; gq.sam = n; gq.sak = 1;
    gq.B = Q0.as<double>(); gq.sbk = p; gq.sbn = 1;
    gq.C = Y.as<double>(); gq.scm = p; gq.scn = 1;
    Gemm64 qgq;   // B = Q0^T Y (upper)
    qgq.M = p; qgq.N = p; qgq.K = n; qgq.upper_only = 1;
    qgq.A = Q0.as<double>(); qgq.sam = 1; qgq.sak = p;
    qgq.B = Y.as<double>(); qgq.sbk = p; qgq.sbn = 1;
    qgq.C = Bm.as<double>(); qgq.scm = p; qgq.scn = 1;
    DevBuf work(std::max({sketch64_workspace_bytes(n, n, 1, p, ncu), gemm64_workspace_bytes(yty, ncu),
                          gemm64_workspace_bytes(gq, ncu), gemm64_workspace_bytes(qgq, ncu)}),
                s);
    sketch64(G, n, n, n * n, nullptr, 0, 1, p, 0x5eed1234ULL, Q0.as<double>(), p, 1, ncu,
             work.as<double>(), s);
    launch_sketch_eta(Q0.as<double>(), n, p, 1, eta.as<double>(), s);
    launch_perturb_eta(Q0.as<double>(), eta.as<double>(), n, p, 1, 1e-13, 0x9e3779b9ULL, s);
    for (int pass = 0; pass < 4; ++pass) {
      gemm64(yty, ncu, work.as<double>(), s);
      launch_chol(Cq.as<double>(), p, n, 1, pass < 2, lds, fail, 1, s);
      launch_trsm_rows(Q0.as<double>(), Cq.as<double>(), n, p, 1, lds, s);
    }
    gemm64(gq, ncu, work.as<double>(), s);
    gemm64(qgq, ncu, work.as<double>(), s);
  }
  DevBuf ews(eig_sym_workspace_bytes(p, r, 1), s), Z((size_t)p * r * sizeof(double), s);
  DevBuf Cz((size_t)r * r * sizeof(double), s), Wr((size_t)p * r * sizeof(double), s);
  DevBuf perm((size_t)p * sizeof(int), s), fixed(3 * sizeof(int), s), info(sizeof(RankInfo), s);
  launch_eig_tridiag(Bm.as<double>(), ews.as<double>(), p, r, 1, lds, s);
  launch_eig_values_vectors(Bm.as<double>(), ews.as<double>(), Z.as<double>(), p, r, 1, lds, s);
  Gemm64 gz;      // Cz = Z^T Z (upper)
  gz.M = r; gz.N = r; gz.K = p; gz.upper_only = 1;
  gz.A = Z.as<double>(); gz.sam = 1; gz.sak = r;
  gz.B = Z.as<double>(); gz.sbk = r; gz.sbn = 1;
  gz.C = Cz.as<double>(); gz.scm = r; gz.scn = 1;
  DevBuf wz(gemm64_workspace_bytes(gz, ncu), s);
  gemm64(gz, ncu, wz.as<double>(), s);
  launch_chol(Cz.as<double>(), r, p, 1, 0, lds, fail, 4, s);
  launch_trsm_rows(Z.as<double>(), Cz.as<double>(), p, r, 1, lds, s);
  launch_eig_backtransform(Z.as<double>(), ews.as<double>(), p, r, 1, s);
  const int fx[3] = {r, 0, 0};
  RS_HIP(hipMemcpyAsync(fixed.p, fx, sizeof(fx), hipMemcpyHostToDevice, s));
  launch_rank_select(Bm.as<double>(), p, 1, 0.0, fixed.as<int>(), r, perm.as<int>(),
                     info.as<RankInfo>(), s);
  Mode3 w{{Wr.as<double>(), nullptr, nullptr}, {r, 0, 0}};
  launch_gather_cols3(Z.as<double>(), r, (int64_t)p * r, perm.as<int>(), p, w, s);
  Gemm64 gb;      // V = Q0 W_r (n x r)
  gb.M = n; gb.N = r; gb.K = p;
  gb.A = Q0.as<double>(); gb.sam = p; gb.sak = 1;
  gb.B = Wr.as<double>(); gb.sbk = 1; gb.sbn = p;
  gb.C = V; gb.scm = r; gb.scn = 1;
  DevBuf wb(gemm64_workspace_bytes(gb, ncu), s);
  gemm64(gb, ncu, wb.as<double>(), s);
  Mode3 q{{V, nullptr, nullptr}, {r, 0, 0}};
  Mode3 none{{nullptr, nullptr, nullptr}, {r, 0, 0}};
  launch_canonical_signs3(q, n, none, p, s);
  RS_HIP(hipStreamSynchronize(s));   // the host-side constant above and the buffers' lifetimes
}

struct Readback {
  int flags;
  int chol_fail;
  RankInfo info;
  int total_pairs;
  int pad;
};

// Record the start of eigensolver phase `ph` when the tensor carries timing events.
static void mark_eig(rs_tensor* T, int ph, hipStream_t s) {
  if (!T->eig_events.empty()) RS_HIP(hipEventRecord(T->eig_events[ph], s));
}

}  // namespace rs

using namespace rs;

extern "C" {

const char* rs_status_str(rs_status s) {
  switch (s) {
    case RS_OK: return "RS_OK";
    case RS_E_INVALID: return "RS_E_INVALID";
    case RS_E_NOMEM: return "RS_E_NOMEM";
    case RS_E_DEVICE: return "RS_E_DEVICE";
    case RS_E_RANK_CAP: return "RS_E_RANK_CAP";
    case RS_E_UNSUPPORTED: return "RS_E_UNSUPPORTED";
  }
  return "unknown status";
}

const char* rs_last_error(void) { return rs::last_error(); }

rs_status rs_ctx_create(int device, rs_ctx** out) {
  return guarded([&]() -> rs_status {
    RS_REQUIRE(out != nullptr, "out is null");
    int count = 0;
    RS_HIP(hipGetDeviceCount(&count));
    RS_REQUIRE(device >= 0 && device < count, "no such HIP device");
    RS_HIP(hipSetDevice(device));
    auto c = std::make_unique<rs_ctx>();
    c->device = device;
    hipDeviceProp_t prop;
    RS_HIP(hipGetDeviceProperties(&prop, device));
    c->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    c->lds_limit = prop.sharedMemPerBlock > 0 ? (int)prop.sharedMemPerBlock : 65536;
    int wk = 0;
    if (hipDeviceGetAttribute(&wk, hipDeviceAttributeWallClockRate, device) == hipSuccess && wk > 0)
      c->wall_khz = (double)wk;
    noalloc_scratch_init(device);
    RS_HIP(hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking));
    *out = c.release();
    return RS_OK;
  });
}

rs_ctx::~rs_ctx() {
  if (aux) {
    (void)hipStreamSynchronize(aux);
    (void)hipStreamDestroy(aux);
  }
  for (void* p : pin_all) (void)hipHostFree(p);
}

void rs_ctx_destroy(rs_ctx* ctx) {
  if (ctx) rs::ctx_release(ctx);
}

rs_status rs_ctx_trim(rs_ctx* ctx) {
  return guarded([&]() -> rs_status {
    RS_REQUIRE(ctx != nullptr, "null context");
    cache_trim(ctx->device);
    return RS_OK;
  });
}

rs_status rs_stream_release(rs_ctx* ctx, void* stream) {
  return guarded([&]() -> rs_status {
    RS_REQUIRE(ctx != nullptr, "null context");
    RS_HIP(hipSetDevice(ctx->device));
    RS_HIP(hipStreamSynchronize((hipStream_t)stream));
    cache_forget_stream((hipStream_t)stream);
    return RS_OK;
  });
}

rs_status rs_ctx_set_timing(rs_ctx* ctx, int enable) {
  return guarded([&]() -> rs_status {
    RS_REQUIRE(ctx != nullptr, "null context");
    RS_REQUIRE(enable >= 0 && enable <= 3, "timing mode must be 0, 1, 2 or 3");
    ctx->timing = enable;
    return RS_OK;
  });
}

rs_status rs_ctx_set_hbm_budget(rs_ctx* ctx, size_t bytes) {
  return guarded([&]() -> rs_status {
    RS_REQUIRE(ctx != nullptr, "null context");
    ctx->hbm_budget = bytes;
    return RS_OK;
  });
}

rs_status rs_build_factors(rs_ctx* ctx, const rs_grid* grid, const rs_fdesc* fdesc,
                           rs_factors** out) {
  return guarded([&]() -> rs_status {
    RS_REQUIRE(ctx && grid && fdesc && out, "null argument");
    RS_HIP(hipSetDevice(ctx->device));
    auto f = std::make_unique<rs_factors>();
    f->grid = *grid;
    f->fdesc = *fdesc;
    f->table = build_table(*grid, *fdesc);
    f->device = ctx->device;
    const size_t bytes = f->table.R * sizeof(double);
    RS_HIP(hipMalloc(&f->t_dev, bytes));
    RS_HIP(hipMalloc(&f->a_dev, bytes));
    RS_HIP(hipMemcpy(f->t_dev, f->table.t.data(), bytes, hipMemcpyHostToDevice));
    RS_HIP(hipMemcpy(f->a_dev, f->table.a.data(), bytes, hipMemcpyHostToDevice));
    *out = f.release();
    return RS_OK;
  });
}

rs_status rs_factors_get(const rs_factors* f, double* t, double* a, int32_t* R, int32_t* R_l,
                         int32_t* n_s) {
  return guarded([&]() -> rs_status {
    RS_REQUIRE(f != nullptr, "null factors");
    if (t) std::memcpy(t, f->table.t.data(), f->table.R * sizeof(double));
    if (a) std::memcpy(a, f->table.a.data(), f->table.R * sizeof(double));
    if (R) *R = f->table.R;
    if (R_l) *R_l = f->table.R_l;
    if (n_s) *n_s = f->table.n_s;
    return RS_OK;
  });
}

void rs_factors_free(rs_factors* f) {
  if (!f) return;
  (void)hipFree(f->t_dev);
  (void)hipFree(f->a_dev);
  delete f;
}

rs_status rs_weighted_gram(rs_ctx* ctx, const rs_factors* f, int64_t N, const double* pos,
                           const double* q, int32_t method, double* G, void* stream) {
  return guarded([&]() -> rs_status {
    RS_REQUIRE(ctx && f && pos && q && G, "null argument");
    RS_REQUIRE(method == RS_GRAM_IDENTITY || method == RS_GRAM_GEMM, "unknown Gram method");
    RS_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    Plan P = make_plan(f, N, nullptr);
    DevBuf U((size_t)3 * P.n * P.K * sizeof(double), s);
    DevBuf xi((size_t)P.K * sizeof(double), s), w((size_t)P.K * sizeof(double), s);
    run_factors_and_gram(ctx, f, P, pos, q, U.as<double>(), xi.as<double>(), w.as<double>(),
                         nullptr, G, method, s);
    return RS_OK;
  });
}

rs_status rs_assemble(rs_ctx* ctx, const rs_factors* f, int64_t N, const double* pos,
                      const double* q, const rs_aopts* opts, void* grid_out, rs_tensor** out,
                      void* stream) {
  return guarded([&]() -> rs_status {
    RS_REQUIRE(ctx && f && pos && q && out, "null argument");
    RS_REQUIRE(f->device == ctx->device, "factors built for another device");
    RS_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const Plan P = make_plan(f, N, opts);
    if (ctx->hbm_budget) {   // admission, before anything is allocated
      const int rb = std::max({P.r_max, P.fixed[0], P.fixed[1], P.fixed[2]});
      const size_t need = rs_footprint_bytes(&f->grid, &f->fdesc, N, rb, P.prec, grid_out != nullptr);
      if (need > ctx->hbm_budget)
        throw Error{RS_E_NOMEM, "the request's footprint bound (" + std::to_string(need) +
                                    " bytes) exceeds the context's budget (" +
                                    std::to_string(ctx->hbm_budget) + " bytes)"};
    }
    const int64_t n = P.n, K = P.K;
    // eigensolver subspace: every buffer is sized for the plan's p; the rank
    // rule runs first at P.p_first and again at the plan's p only when a
    // mode's rank comes within twice the oversampling of the subspace
    const int p_max = P.p;
    int p = P.p_first;
    const int ncu = ctx->num_cu;

    auto T = std::make_unique<rs_tensor>();
    T->ctx = ctx;
    T->ctx_ref.set(ctx);
    T->N = N;
    T->n = n;
    T->b = f->grid.b;
    T->h = 2.0 * f->grid.b / (double)n;
    T->R = P.R;
    T->R_l = P.R_l;
    T->n_s = P.n_s;
    T->kernel = f->fdesc.kernel;
    T->lambda = f->fdesc.lambda;
    T->prec = P.prec;
    T->interp = P.interp;
    T->table = f->table;
    T->stream = s;
    for (int l = 0; l < 3; ++l) T->p[l] = p;
    if (ctx->timing) {
      T->timing_mode = ctx->timing;
      T->events.assign(RS_STAGE_COUNT + 1, nullptr);
      for (auto& e : T->events) RS_HIP(hipEventCreate(&e));
      if (ctx->timing == 1) {
        T->eig_events.assign(RS_EIG_PHASES + 1, nullptr);
        for (auto& e : T->eig_events) RS_HIP(hipEventCreate(&e));
      }
      if (ctx->timing == 3) {
        RS_HIP(hipEventCreate(&T->kevents.begin));
        RS_HIP(hipEventCreate(&T->kevents.end));
      }
    }

    T->pos = DevBuf((size_t)N * 3 * sizeof(double), s);
    T->q = DevBuf((size_t)N * sizeof(double), s);
    T->t_dev = DevBuf((size_t)P.R * sizeof(double), s);
    T->a_dev = DevBuf((size_t)P.R * sizeof(double), s);
    RS_HIP(hipMemcpyAsync(T->pos.p, pos, T->pos.bytes, hipMemcpyDeviceToDevice, s));
    RS_HIP(hipMemcpyAsync(T->q.p, q, T->q.bytes, hipMemcpyDeviceToDevice, s));
    RS_HIP(hipMemcpyAsync(T->t_dev.p, f->t_dev, T->t_dev.bytes, hipMemcpyDeviceToDevice, s));
    RS_HIP(hipMemcpyAsync(T->a_dev.p, f->a_dev, T->a_dev.bytes, hipMemcpyDeviceToDevice, s));
    const double* dpos = T->pos.as<double>();
    const double* dq = T->q.as<double>();

    // Every buffer of the stages before the rank readback is a piece of one
    // allocation (a stream-ordered allocation between two launches costs a
    // queue dependency each); the pieces live until the assembly returns.
    const int rcap_all = std::max({P.r_max, P.fixed[0], P.fixed[1], P.fixed[2]});
    const int rc_max = std::min<int>(p_max, rcap_all);
    int rc = std::min<int>(p, rcap_all);
    T->nb = bricks_per_axis(n);
    const int nbricks = T->nb * T->nb * T->nb;
    Gemm64 gq_shape, qgq_shape, yty_shape, zz_shape;
    auto set_shapes = [&](int pp, int rr) {
      gq_shape.M = n; gq_shape.N = pp; gq_shape.K = n; gq_shape.batch = 3;   // G Q0 (n x p)
      qgq_shape.M = pp; qgq_shape.N = pp; qgq_shape.K = n; qgq_shape.batch = 3;   // Q0^T (G Q0)
      qgq_shape.upper_only = 1;
      yty_shape.M = pp; yty_shape.N = pp; yty_shape.K = n; yty_shape.batch = 3;   // Y^T Y
      yty_shape.upper_only = 1;
      zz_shape.M = rr; zz_shape.N = rr; zz_shape.K = pp; zz_shape.batch = 3;   // Z^T Z
      zz_shape.upper_only = 1;
    };
    // workspace of the split-K products at either subspace size
    auto eig_ws = [&](int pp, int rr, bool sub_path, size_t* wke, size_t* wkz, size_t* ews) {
      set_shapes(pp, rr);
      *wke = sub_path ? std::max({sketch64_workspace_bytes(n, P.sketch ? K : n, 3, pp, ncu),
                                  gemm64_workspace_bytes(gq_shape, ncu),
                                  gemm64_workspace_bytes(qgq_shape, ncu),
                                  gemm64_workspace_bytes(yty_shape, ncu)})
                      : 0;
      *wkz = gemm64_workspace_bytes(zz_shape, ncu);
      *ews = eig_sym_workspace_bytes(pp, rr, 3);
    };
    size_t wke_a, wkz_a, ews_a, wke_b, wkz_b, ews_b;
    eig_ws(p_max, rc_max, p_max < n, &wke_a, &wkz_a, &ews_a);
    eig_ws(p, rc, p < n, &wke_b, &wkz_b, &ews_b);
    const size_t wke_bytes = std::max(wke_a, wke_b), wkz_bytes = std::max(wkz_a, wkz_b);
    const size_t ews_bytes = std::max(ews_a, ews_b);
    set_shapes(p, rc);
    const size_t d8 = sizeof(double);
    const size_t scan_bytes = exclusive_scan_bytes(nbricks + 1);
    Carve pre;
    const size_t o_rb = pre.add(sizeof(Readback));
    // The split-FP16 projection reads FP16 planes of U written with the side
    // matrices; U itself (FP64) is kept only where something else reads it
    // (FP64 or BF16 contractions, the GEMM Gram, the side-matrix sketch, ALS).
    const bool fused16 = contraction_prec(P.prec) == RS_MIXED_FP16;
    const bool need_u64 = !fused16 || P.gram == RS_GRAM_GEMM || P.sketch != 0 || P.als > 0;
    const int64_t kpn = (n + 31) / 32 * 32;
    const size_t o_U = pre.add(need_u64 ? (size_t)3 * n * K * d8 : 0), o_xi = pre.add((size_t)K * d8);
    const size_t o_P16 = pre.add(fused16 ? (size_t)3 * 2 * K * kpn * 2 : 0);
    const size_t o_w = pre.add((size_t)K * d8), o_sw = pre.add((size_t)K * d8);
    // the three n x n Gram matrices: by the Gaussian-product identity
    // (O(n K + n^2 R_l)) or by the MFMA GEMM U diag(w) U^T (2 n^2 K FLOP)
    const bool subspace = p < n;   // the first pass (the smaller subspace) runs the range finder
    const size_t o_G = pre.add((size_t)3 * n * n * d8);
    const size_t wgram_bytes = P.gram == RS_GRAM_GEMM
                                   ? gemm64_workspace_bytes(gram_gemm(P, nullptr, nullptr, nullptr), ncu)
                                   : gauss_gram_workspace_bytes(P.N, P.R_l, n, ncu);
    const size_t o_wgram = pre.add(wgram_bytes);
    const size_t o_Q0 = pre.add((size_t)3 * n * p_max * d8);
    const size_t o_Bm = pre.add((size_t)3 * p_max * p_max * d8);
    const size_t o_Y = pre.add(subspace ? (size_t)3 * n * p_max * d8 : 0);
    const size_t o_Cq = pre.add(subspace ? (size_t)3 * p_max * p_max * d8 : 0);
    const size_t o_eta = pre.add(sketch_eta_bytes(3));
    const size_t o_wke = pre.add(wke_bytes);
    const size_t o_ews = pre.add(ews_bytes);
    const size_t o_Z = pre.add((size_t)3 * p_max * rc_max * d8);
    const size_t o_Zsave = pre.add((size_t)3 * p_max * rc_max * d8);
    const size_t o_Cz = pre.add((size_t)3 * rc_max * rc_max * d8);
    const size_t o_wkz = pre.add(wkz_bytes);
    const size_t o_perm = pre.add((size_t)3 * p_max * sizeof(int)), o_fixed = pre.add(3 * sizeof(int));
    const size_t o_counts = pre.add((size_t)(nbricks + 1) * sizeof(int));
    const size_t o_scan = pre.add(scan_bytes);
    DevBuf pre_buf(pre.total, s);
    auto piece = [&](size_t off, size_t bytes) { return Span{pre_buf.as<char>() + off, bytes}; };

    Span rb = piece(o_rb, sizeof(Readback));
    RS_HIP(hipMemsetAsync(rb.p, 0, sizeof(Readback), s));
    Readback* rbd = rb.as<Readback>();
    launch_validate(dpos, dq, N, f->grid.b, &rbd->flags, s);

    // (a2, a3) side matrices and charge-weighted Gram matrices
    mark(T.get(), RS_STAGE_FACTORS, s);
    Span U = need_u64 ? piece(o_U, (size_t)3 * n * K * d8) : Span{};
    Span xi = piece(o_xi, (size_t)K * d8);
    Span P16 = fused16 ? piece(o_P16, (size_t)3 * 2 * K * kpn * 2) : Span{};
    Span w = piece(o_w, (size_t)K * d8), sw = piece(o_sw, (size_t)K * d8);
    Span G = piece(o_G, (size_t)3 * n * n * d8);
    // Nothing before the projection reads the side matrices on the identity
    // Gram route with the Gram sketch: they are formed on the context's
    // second stream, concurrently with the Gram and the eigensolver, and the
    // caller's stream waits for them before the projection (or, on an early
    // exit, before the arena that holds them is released).
    const bool side_overlap = ctx->aux && P.gram == RS_GRAM_IDENTITY && P.sketch == 0;
    SideJoin side_join;
    if (side_overlap) {
      side_join.s = s;
      side_join.aux = ctx->aux;
      RS_HIP(hipEventCreateWithFlags(&side_join.start, hipEventDisableTiming));
      RS_HIP(hipEventRecord(side_join.start, s));
      RS_HIP(hipStreamWaitEvent(ctx->aux, side_join.start, 0));
    }
    run_factors_and_gram(ctx, f, P, dpos, dq, U.as<double>(), xi.as<double>(), w.as<double>(),
                         sw.as<double>(), G.as<double>(), P.gram, s, T.get(),
                         (double*)(pre_buf.as<char>() + o_wgram), P16.p, kpn, ctx->aux, side_overlap);
    if (side_overlap) {
      RS_HIP(hipEventCreateWithFlags(&side_join.done, hipEventDisableTiming));
      RS_HIP(hipEventRecord(side_join.done, ctx->aux));
    }

    // short-range binning (counts and offsets; the total is read back with the ranks)
    Span counts = piece(o_counts, (size_t)(nbricks + 1) * sizeof(int));
    RS_HIP(hipMemsetAsync(counts.p, 0, counts.bytes, s));
    short_bin_count(dpos, N, n, f->grid.b, P.n_s, T->nb, counts.as<int>(), s);
    T->brick_start = DevBuf((size_t)(nbricks + 1) * sizeof(int), s);
    exclusive_scan_int(counts.as<int>(), T->brick_start.as<int>(), nbricks + 1,
                       pre_buf.as<char>() + o_scan, scan_bytes, s);
    RS_HIP(hipMemcpyAsync(&rbd->total_pairs, T->brick_start.as<int>() + nbricks, sizeof(int),
                          hipMemcpyDeviceToDevice, s));

    // (a4) dominant eigenvectors: Q0 (n x p per mode, row-major) spans the subspace
    mark(T.get(), RS_STAGE_EIGEN, s);
    Span Q0, Bm, ews, Z, Zsave, Cz, perm, fixed_dev;
    Readback host;
    for (;;) {   // the subspace search: at most two passes
    mark_eig(T.get(), 0, s);
    Q0 = piece(o_Q0, (size_t)3 * n * p * d8);
    Bm = piece(o_Bm, (size_t)3 * p * p * d8);
    if (p == n) {
      launch_identity(Q0.as<double>(), n, 3, s);
      RS_HIP(hipMemcpyAsync(Bm.p, G.p, G.bytes, hipMemcpyDeviceToDevice, s));
    } else {
      Span Y = piece(o_Y, (size_t)3 * n * p * d8), Cq = piece(o_Cq, (size_t)3 * p * p * d8);
      double* eta = (double*)(pre_buf.as<char>() + o_eta);
      auto gq_gemm = [&](const double* X, double* out) {  // out = G X (n x p, row-major)
        Gemm64 g = gq_shape;
        g.A = G.as<double>(); g.sam = n; g.sak = 1; g.sab = n * n;
        g.B = X; g.sbk = p; g.sbn = 1; g.sbb = n * p;
        g.C = out; g.scm = p; g.scn = 1; g.scb = n * p;
        return g;
      };
      auto qgq_gemm = [&](const double* X, const double* GX) {  // B = X^T (G X) (symmetric)
        Gemm64 g = qgq_shape;
        g.A = X; g.sam = 1; g.sak = p; g.sab = n * p;
        g.B = GX; g.sbk = p; g.sbn = 1; g.sbb = n * p;
        g.C = Bm.as<double>(); g.scm = p; g.scn = 1; g.scb = (int64_t)p * p;
        return g;
      };
      auto yty_gemm = [&](const double* Yp) {  // C = Y^T Y (symmetric)
        Gemm64 g = yty_shape;
        g.A = Yp; g.sam = 1; g.sak = p; g.sab = n * p;
        g.B = Yp; g.sbk = p; g.sbn = 1; g.sbb = n * p;
        g.C = Cq.as<double>(); g.scm = p; g.scn = 1; g.scb = (int64_t)p * p;
        return g;
      };
      Span wk_eig = piece(o_wke, wke_bytes);  // split-K workspace of every product here
      // Y = G X carries the squared spectrum (condition up to ~1e16 once the
      // perturbation below bounds it); Y = U diag(|xi|^{1/3}) Omega the
      // spectrum itself.  The perturbation must stay below the components
      // at the rank threshold (sigma^2 ~ 1e-12 sigma_1^2 for the Gram).
      // orthonormal basis of range(Y), in place: shifted Cholesky QR, twice
      // (each shifted pass maps cond(Y) to about sqrt(shift)/sigma_min(Y)),
      // then plain passes (two for the squared spectrum)
      auto orth = [&](double* Yp, bool squared) {
        const int passes = squared ? 4 : 3;
        for (int pass = 0; pass < passes; ++pass) {
          gemm64(yty_gemm(Yp), ncu, wk_eig.as<double>(), s);
          launch_chol(Cq.as<double>(), p, n, 3, pass < 2, ctx->lds_limit, &rbd->chol_fail, 1, s);
          launch_trsm_rows(Yp, Cq.as<double>(), n, p, 3, ctx->lds_limit, s);
        }
      };
      // a random perturbation of relative size `rel` (scaled from Y itself)
      // gives Y full column rank when the Gram has rank below p
      auto perturb = [&](double* Yp, uint64_t seed, bool squared) {
        launch_sketch_eta(Yp, n, p, 3, eta, s);
        launch_perturb_eta(Yp, eta, n, p, 3, squared ? 1e-13 : 1e-12, seed, s);
      };
      // range finder: Y = G Omega (n x n times n x p), or on the
      // charge-weighted side matrix itself, Y = U diag(|xi|^{1/3}) Omega
      // (n x K times K x p; the dynamic range of Y is that of the singular
      // values, not of their squares, but one pass resolves the directions
      // at the threshold less well and costs 2 n K p)
      if (P.sketch == 0)
        sketch64(G.as<double>(), n, n, n * n, nullptr, 0, 3, p, 0x5eed1234ULL, Q0.as<double>(), p,
                 1, ncu, wk_eig.as<double>(), s);
      else
        sketch64(U.as<double>(), n, K, n * K, sw.as<double>(), 0, 3, p, 0x5eed1234ULL,
                 Q0.as<double>(), p, 1, ncu, wk_eig.as<double>(), s);
      perturb(Q0.as<double>(), 0x9e3779b9ULL, P.sketch == 0);
      orth(Q0.as<double>(), P.sketch == 0);
      // subspace iterations Q0 <- orth(G Q0): n x n products through the Gram
      for (int it = 0; it < P.power_iters; ++it) {
        gemm64(gq_gemm(Q0.as<double>(), Y.as<double>()), ncu, wk_eig.as<double>(), s);
        perturb(Y.as<double>(), 0x9e3779b9ULL + it + 1, true);
        orth(Y.as<double>(), true);
        std::swap(Q0, Y);
      }
      // Rayleigh-Ritz matrix B = Q0^T G Q0
      gemm64(gq_gemm(Q0.as<double>(), Y.as<double>()), ncu, wk_eig.as<double>(), s);
      gemm64(qgq_gemm(Q0.as<double>(), Y.as<double>()), ncu, wk_eig.as<double>(), s);
    }
    // eigenvectors are formed only for the rc columns the rank rule can keep
    ews = piece(o_ews, eig_sym_workspace_bytes(p, rc, 3));
    Z = piece(o_Z, (size_t)3 * p * rc * d8);
    mark_eig(T.get(), 1, s);
    launch_eig_tridiag(Bm.as<double>(), ews.as<double>(), p, rc, 3, ctx->lds_limit, s);
    mark_eig(T.get(), 2, s);
    launch_eig_values_vectors(Bm.as<double>(), ews.as<double>(), Z.as<double>(), p, rc, 3,
                              ctx->lds_limit, s);
    mark_eig(T.get(), 3, s);
    // Cholesky QR of the eigenvectors in eigenvalue order.  Inverse
    // iteration leaves them nearly orthonormal, so two plain passes suffice;
    // a breakdown (near-parallel vectors, flag bit 4) is redone from the
    // saved vectors with a shifted pass first, after the readback.
    Zsave = piece(o_Zsave, (size_t)3 * p * rc * d8);
    RS_HIP(hipMemcpyAsync(Zsave.p, Z.p, Zsave.bytes, hipMemcpyDeviceToDevice, s));
    Cz = piece(o_Cz, (size_t)3 * rc * rc * d8);
    Gemm64 gz = zz_shape;  // C = Z^T Z (symmetric)
    gz.A = Z.as<double>(); gz.sam = 1; gz.sak = rc; gz.sab = (int64_t)p * rc;
    gz.B = Z.as<double>(); gz.sbk = rc; gz.sbn = 1; gz.sbb = (int64_t)p * rc;
    gz.C = Cz.as<double>(); gz.scm = rc; gz.scn = 1; gz.scb = (int64_t)rc * rc;
    Span wkz = piece(o_wkz, wkz_bytes);
    auto orth_z = [&](int passes, bool shifted_first, int fail_bit) {
      for (int pass = 0; pass < passes; ++pass) {
        gemm64(gz, ncu, wkz.as<double>(), s);
        launch_chol(Cz.as<double>(), rc, p, 3, shifted_first && pass == 0, ctx->lds_limit,
                    &rbd->chol_fail, fail_bit, s);
        launch_trsm_rows(Z.as<double>(), Cz.as<double>(), p, rc, 3, ctx->lds_limit, s);
      }
    };
    // one plain pass: the kept vectors are nearly orthonormal already (their
    // Gram is close to the identity), and Cholesky QR is causal, so the
    // leading columns come out orthonormal to rounding whatever the trailing
    // (unkept, clustered) ones do; a breakdown still flags the robust redo
    orth_z(1, false, 4);
    launch_eig_backtransform(Z.as<double>(), ews.as<double>(), p, rc, 3, s);
    mark_eig(T.get(), 4, s);
    perm = piece(o_perm, (size_t)3 * p * sizeof(int));
    fixed_dev = piece(o_fixed, 3 * sizeof(int));
    RS_HIP(hipMemcpyAsync(fixed_dev.p, P.fixed, 3 * sizeof(int), hipMemcpyHostToDevice, s));
    launch_rank_select(Bm.as<double>(), p, 3, P.eps * P.eps, fixed_dev.as<int>(), P.r_max,
                       perm.as<int>(), &rbd->info, s);

    // the readback lands in a pinned host slot of the context (a copy to
    // pageable memory would be staged through a driver buffer)
    {
      void* slot = nullptr;
      {
        std::lock_guard<std::mutex> lock(ctx->pin_mu);
        if (!ctx->pin_free.empty()) {
          slot = ctx->pin_free.back();
          ctx->pin_free.pop_back();
        }
      }
      if (!slot) {
        RS_HIP(hipHostMalloc(&slot, sizeof(Readback), hipHostMallocDefault));
        std::lock_guard<std::mutex> lock(ctx->pin_mu);
        ctx->pin_all.push_back(slot);
      }
      const hipError_t e1 = hipMemcpyAsync(slot, rbd, sizeof(Readback), hipMemcpyDeviceToHost, s);
      const hipError_t e2 = e1 == hipSuccess ? hipStreamSynchronize(s) : e1;
      if (e2 == hipSuccess) std::memcpy(&host, slot, sizeof(Readback));
      {
        std::lock_guard<std::mutex> lock(ctx->pin_mu);
        ctx->pin_free.push_back(slot);
      }
      RS_HIP(e2);
    }
    if (host.flags & 1) throw Error{RS_E_INVALID, "non-finite particle position or charge"};
    if (host.flags & 2) throw Error{RS_E_INVALID, "particle outside the box [-b, b]^3"};
    if (host.chol_fail & 1) throw Error{RS_E_DEVICE, "eigensolver: Cholesky breakdown in the subspace basis"};
    if (host.chol_fail & 4) {
      // rare path: redo the eigenvector orthonormalisation robustly
      RS_HIP(hipMemcpyAsync(Z.p, Zsave.p, Zsave.bytes, hipMemcpyDeviceToDevice, s));
      orth_z(3, true, 1);
      launch_eig_backtransform(Z.as<double>(), ews.as<double>(), p, rc, 3, s);
      int again = 0;
      RS_HIP(hipMemcpyAsync(&again, &rbd->chol_fail, sizeof(int), hipMemcpyDeviceToHost, s));
      RS_HIP(hipStreamSynchronize(s));
      if (again & 1) throw Error{RS_E_DEVICE, "eigensolver: Cholesky breakdown in the eigenvectors"};
    }
    // a rank within twice the oversampling of the subspace is not resolved
    // well enough: run the eigensolver again at the plan's full size
    bool grow = false;
    for (int l = 0; l < 3; ++l)
      if (host.info.r[l] + 2 * P.os > p) grow = true;
    if (!grow || p >= p_max) break;
    p = p_max;
    rc = rc_max;
    set_shapes(p, rc);
    RS_HIP(hipMemsetAsync(&rbd->chol_fail, 0, sizeof(int), s));
    }   // subspace search
    for (int l = 0; l < 3; ++l) T->p[l] = p;

    for (int l = 0; l < 3; ++l) {
      T->r[l] = host.info.r[l];
      T->rank_capped |= host.info.capped[l];
      const double l1 = host.info.lam1[l];
      T->sigma1[l] = std::sqrt(std::max(l1, 0.0));
      T->sig_kept[l] = l1 > 0 ? std::sqrt(std::max(host.info.lam_kept[l], 0.0) / l1) : 0.0;
      T->sig_next[l] = l1 > 0 ? std::sqrt(std::max(host.info.lam_next[l], 0.0) / l1) : 0.0;
    }

    // Everything below is sized by the ranks: allocate it all now (the
    // result's own buffers, then one scratch arena), so that the launches
    // that follow are not interleaved with allocator calls.
    const int r1 = T->r[0], r2 = T->r[1], r3 = T->r[2];
    for (int l = 0; l < 3; ++l) T->Q[l] = DevBuf((size_t)n * T->r[l] * sizeof(double), s);
    T->beta = DevBuf((size_t)r1 * r2 * r3 * sizeof(double), s);
    T->n_pairs = host.total_pairs;
    T->brick_list = DevBuf((size_t)std::max<int64_t>(T->n_pairs, 1) * sizeof(int), s);
    // (a6) short-range lists: fill and sort by particle index (first after the
    // readback: it keeps the device busy while the rank-sized launches are enqueued)
    mark(T.get(), RS_STAGE_BINS, s);
    RS_HIP(hipMemsetAsync(counts.p, 0, counts.bytes, s));
    short_bin_fill(dpos, N, n, f->grid.b, P.n_s, T->nb, T->brick_start.as<int>(), counts.as<int>(),
                   T->brick_list.as<int>(), s);
    T->active_cap = short_active_capacity(N, P.n_s, T->nb);
    T->brick_active = DevBuf((size_t)(T->active_cap + 1) * sizeof(int), s);
    short_bin_sort(T->brick_start.as<int>(), T->brick_list.as<int>(), nbricks,
                   T->brick_active.as<int>(), T->active_cap, s);

    T->T2 = DevBuf((size_t)n * n * r3 * sizeof(double), s);
    if (P.prec != RS_FP64) T->t2exp = DevBuf(sizeof(int), s);
    Gemm64 gb[3], gp[3];
    for (int l = 0; l < 3; ++l) {
      const int r = T->r[l];
      Gemm64& g = gb[l];  // V_l = Q0 W_r (n x r)
      g.M = n; g.N = r; g.K = p;
      g.A = Q0.as<double>() + (int64_t)l * n * p; g.sam = p; g.sak = 1;
      g.sbk = 1; g.sbn = p;
      g.C = T->Q[l].as<double>(); g.scm = r; g.scn = 1;
      Gemm64& h = gp[l];  // U~_l^T = U_l^T V_l (K x r row-major, i.e. U~[j*r + a]): the
      h.M = K; h.N = r; h.K = n;   // long dimension K is the GEMM's row dimension
      h.A = need_u64 ? U.as<double>() + (int64_t)l * n * K : nullptr; h.sam = n; h.sak = 1;
      h.B = T->Q[l].as<double>(); h.sbk = r; h.sbn = 1;
      h.scm = r; h.scn = 1;
    }
    Carve cv;
    size_t o_wr[3], o_wkb[3], o_ut[3], o_wkp[3];
    for (int l = 0; l < 3; ++l) {
      o_wr[l] = cv.add((size_t)p * T->r[l] * sizeof(double));
      o_wkb[l] = cv.add(gemm64_workspace_bytes(gb[l], ncu));
      o_ut[l] = cv.add((size_t)K * T->r[l] * sizeof(double));
      o_wkp[l] = P.prec == RS_FP64 ? cv.add(gemm64_workspace_bytes(gp[l], ncu)) : 0;
    }
    const size_t o_core = cv.add(P.prec == RS_FP64 ? core64_workspace_bytes(r1, r2, r3, K, ncu)
                                                   : core_mixed_workspace_bytes(r1, r2, r3, K, ncu));
    const size_t o_pmix =
        P.prec == RS_FP64 ? 0 : cv.add(proj_mixed_workspace_bytes(n, K, std::max(r1, std::max(r2, r3)), fused16));
    const size_t o_exp = cv.add(expansion_scratch(T.get(), grid_out != nullptr).total);
    DevBuf arena(cv.total, s);
    char* ab = arena.as<char>();
    auto at = [&](size_t off) { return (double*)(ab + off); };
    // U~_l^T = U_l^T V_l: FP64 GEMM, or split precision like the core
    auto project = [&](int l) {
      if (P.prec == RS_FP64)
        gemm64(gp[l], ncu, at(o_wkp[l]), s);
      else
        proj_mixed(contraction_prec(P.prec), need_u64 ? U.as<double>() + (int64_t)l * n * K : nullptr,
                   fused16 ? P16.as<char>() + (size_t)l * 2 * K * kpn * 2 : nullptr, n, K,
                   T->Q[l].as<double>(), T->r[l], gp[l].C, at(o_pmix), s);
    };

    // final bases V_l = Q0 W[:, perm[:r]] (n x r row-major), canonical signs
    mark(T.get(), RS_STAGE_BASIS, s);
    Mode3 wr3{{at(o_wr[0]), at(o_wr[1]), at(o_wr[2])}, {r1, r2, r3}};
    Mode3 q3{{T->Q[0].as<double>(), T->Q[1].as<double>(), T->Q[2].as<double>()}, {r1, r2, r3}};
    launch_gather_cols3(Z.as<double>(), rc, (int64_t)p * rc, perm.as<int>(), p, wr3, s);
    for (int l = 0; l < 3; ++l) {
      gb[l].B = at(o_wr[l]);
      gemm64(gb[l], ncu, at(o_wkb[l]), s);
    }
    // the sign of each kept column is fixed on V_l and carried to W_r,
    // which the projection below multiplies
    Mode3 none{{nullptr, nullptr, nullptr}, {r1, r2, r3}};
    launch_canonical_signs3(q3, n, none, p, s);

    // (a5) projection U~_l = V_l^T U_l and core
    side_join.join();
    mark(T.get(), RS_STAGE_PROJECT, s);
    for (int l = 0; l < 3; ++l) {
      gp[l].C = at(o_ut[l]);
      project(l);
    }
    // ALS refinement (Appendix, steps (III)-(IV)): for each mode in turn the
    // partially projected image M_l = U_l diag(xi) (U~_m (.) U~_p)^T (the
    // core's contraction with the side matrix itself as first factor: U_l,
    // column-major n x K, is the K x n row-major operand), its Gram M M^T,
    // the r_l dominant eigenvectors as the new basis, the new projection
    if (P.als > 0) {
      DevBuf dfail(sizeof(int), s);
      RS_HIP(hipMemsetAsync(dfail.p, 0, sizeof(int), s));
      for (int sweep = 0; sweep < P.als; ++sweep) {
        for (int l = 0; l < 3; ++l) {
          const int m = l == 0 ? 1 : 0, q = l == 2 ? 1 : 2;
          const int rm = T->r[m], rq = T->r[q];
          const int64_t W = (int64_t)rm * rq;
          DevBuf Mb((size_t)n * W * sizeof(double), s);
          const double* Ul = U.as<double>() + (int64_t)l * n * K;
          if (P.prec == RS_FP64) {
            DevBuf wc(core64_workspace_bytes((int)n, rm, rq, K, ncu), s);
            core64(Ul, at(o_ut[m]), at(o_ut[q]), xi.as<double>(), (int)n, rm, rq, K, Mb.as<double>(),
                   ncu, wc.as<double>(), s);
          } else {
            DevBuf wc(core_mixed_workspace_bytes((int)n, rm, rq, K, ncu), s);
            core_mixed(contraction_prec(P.prec), Ul, at(o_ut[m]), at(o_ut[q]), xi.as<double>(), (int)n,
                       rm, rq, K, Mb.as<double>(), ncu, wc.as<double>(), s);
          }
          DevBuf Gm((size_t)n * n * sizeof(double), s);
          Gemm64 gg;   // G = M M^T (upper, mirrored)
          gg.M = n; gg.N = n; gg.K = W; gg.upper_only = 1;
          gg.A = Mb.as<double>(); gg.sam = W; gg.sak = 1;
          gg.B = Mb.as<double>(); gg.sbk = 1; gg.sbn = W;
          gg.C = Gm.as<double>(); gg.scm = n; gg.scn = 1;
          DevBuf wg(gemm64_workspace_bytes(gg, ncu), s);
          gemm64(gg, ncu, wg.as<double>(), s);
          dominant_eigvecs(ctx, Gm.as<double>(), n, T->r[l], T->Q[l].as<double>(), dfail.as<int>(), s);
          project(l);
        }
      }
      int hf = 0;
      RS_HIP(hipMemcpyAsync(&hf, dfail.p, sizeof(int), hipMemcpyDeviceToHost, s));
      RS_HIP(hipStreamSynchronize(s));
      if (hf & 5) throw Error{RS_E_DEVICE, "ALS refinement: Cholesky breakdown in a basis"};
    }
    mark(T.get(), RS_STAGE_CORE, s);
    const KernelTimer* kt = T->kevents.begin ? &T->kevents : nullptr;
    if (P.prec == RS_FP64) {
      core64(at(o_ut[0]), at(o_ut[1]), at(o_ut[2]), xi.as<double>(), r1, r2, r3, K,
             T->beta.as<double>(), ncu, at(o_core), s, kt);
    } else {
      core_mixed(contraction_prec(P.prec), at(o_ut[0]), at(o_ut[1]), at(o_ut[2]), xi.as<double>(), r1, r2, r3, K,
                 T->beta.as<double>(), ncu, at(o_core), s, kt);
    }

    // (a7) T2 and the grid
    build_expansion(T.get(), grid_out, ab + o_exp, s);
    make_fp32_field(T.get(), s);

    *out = T.release();
    return (*out)->rank_capped ? RS_E_RANK_CAP : RS_OK;
  });
}

rs_status rs_eval_points(const rs_tensor* T, int64_t M, const double* pts, double* vals,
                         int32_t part, void* stream) {
  return guarded([&]() -> rs_status {
    RS_REQUIRE(T && pts && vals, "null argument");
    RS_REQUIRE(M >= 0, "M must be >= 0");
    RS_REQUIRE(part >= 0 && part <= 2, "part must be 0, 1 or 2");
    if (M == 0) return RS_OK;
    RS_HIP(hipSetDevice(T->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    if (part == 0 || part == 1) {
      EvalOut o;
      o.val = vals;
      launch_eval_long(T, M, pts, 0, o, s);
    }
    if (part == 0 || part == 2) launch_eval_short(T, M, pts, vals, part == 0 ? 1 : 0, s);
    return RS_OK;
  });
}

rs_status rs_eval_gradient_points(const rs_tensor* T, int64_t M, const double* pts,
                                  const double* normals, double* out, int32_t part, void* stream) {
  return guarded([&]() -> rs_status {
    RS_REQUIRE(T, "null tensor");
    RS_REQUIRE(M >= 0, "M must be >= 0");
    RS_REQUIRE(part >= 0 && part <= 2, "part must be 0, 1 or 2");
    if (M == 0) return RS_OK;
    RS_REQUIRE(pts && out, "null argument");
    RS_HIP(hipSetDevice(T->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    DevBuf gbuf;
    double* g = out;
    if (normals) {
      gbuf = DevBuf((size_t)M * 3 * sizeof(double), s);
      g = gbuf.as<double>();
    }
    if (part == 0 || part == 1) {
      DevBuf v((size_t)M * sizeof(double), s);
      EvalOut o;
      o.val = v.as<double>();
      o.grad = g;
      launch_eval_long(T, M, pts, 0, o, s);
    }
    if (part == 0 || part == 2) launch_eval_short_grad(T, M, pts, g, part == 0 ? 1 : 0, s);
    if (normals) launch_normal_dot(g, normals, M, out, s);
    return RS_OK;
  });
}

rs_status rs_energy(const rs_tensor* T, double* E, double* dEdq, void* stream) {
  return guarded([&]() -> rs_status {
    RS_REQUIRE(T && E, "null argument");
    RS_HIP(hipSetDevice(T->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    DevBuf v((size_t)T->N * sizeof(double), s), g((size_t)T->N * sizeof(double), s);
    EvalOut o;
    o.val = v.as<double>();
    o.selfv = g.as<double>();
    launch_eval_long(T, T->N, T->pos.as<double>(), 1, o, s);
    launch_energy_reduce(T->q.as<double>(), v.as<double>(), g.as<double>(), T->N, E, dEdq, s);
    return RS_OK;
  });
}

rs_status rs_forces(const rs_tensor* T, double scale, double* F, void* stream) {
  return guarded([&]() -> rs_status {
    RS_REQUIRE(T && F, "null argument");
    RS_REQUIRE(std::isfinite(scale), "scale must be finite");
    RS_HIP(hipSetDevice(T->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    DevBuf v((size_t)T->N * sizeof(double), s), gv((size_t)T->N * 3 * sizeof(double), s);
    DevBuf sv((size_t)T->N * sizeof(double), s), sg((size_t)T->N * 3 * sizeof(double), s);
    EvalOut o;
    o.val = v.as<double>();
    o.grad = gv.as<double>();
    o.selfv = sv.as<double>();
    o.selfg = sg.as<double>();
    launch_eval_long(T, T->N, T->pos.as<double>(), 1, o, s);
    launch_forces(T->q.as<double>(), gv.as<double>(), sg.as<double>(), T->N, scale, F, s);
    return RS_OK;
  });
}

rs_status rs_energy_forces(const rs_tensor* T, double* E, double* dEdq, double scale, double* F,
                           void* stream) {
  return guarded([&]() -> rs_status {
    RS_REQUIRE(T && E && F, "null argument");
    RS_REQUIRE(std::isfinite(scale), "scale must be finite");
    RS_HIP(hipSetDevice(T->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    DevBuf v((size_t)T->N * sizeof(double), s), gv((size_t)T->N * 3 * sizeof(double), s);
    DevBuf sv((size_t)T->N * sizeof(double), s), sg((size_t)T->N * 3 * sizeof(double), s);
    EvalOut o;
    o.val = v.as<double>();
    o.grad = gv.as<double>();
    o.selfv = sv.as<double>();
    o.selfg = sg.as<double>();
    launch_eval_long(T, T->N, T->pos.as<double>(), 1, o, s);
    launch_energy_reduce(T->q.as<double>(), v.as<double>(), sv.as<double>(), T->N, E, dEdq, s);
    launch_forces(T->q.as<double>(), gv.as<double>(), sg.as<double>(), T->N, scale, F, s);
    return RS_OK;
  });
}

rs_status rs_energy_forces_noalloc(const rs_tensor* T, double* E, double* dEdq, double scale,
                                   double* F, void* stream) {
  return guarded([&]() -> rs_status {
    RS_REQUIRE(T && E && F, "null argument");
    RS_REQUIRE(std::isfinite(scale), "scale must be finite");
    RS_REQUIRE(8 * T->N <= kNoAllocScratchDoubles,
               "rs_energy_forces_noalloc: N above " + std::to_string(kNoAllocScratchDoubles / 8) +
                   " (the size of the library's static scratch array)");
    RS_HIP(hipSetDevice(T->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    // the device array's address on this device (looked up at context
    // creation), carved like the buffers of rs_energy_forces; every value
    // is written before it is read, so nothing needs clearing
    double* sc = noalloc_scratch(T->ctx->device);
    const int64_t N = T->N;
    EvalOut o;
    o.val = sc;
    o.grad = sc + N;
    o.selfv = sc + 4 * N;
    o.selfg = sc + 5 * N;
    launch_eval_long(T, N, T->pos.as<double>(), 1, o, s);
    launch_energy_reduce(T->q.as<double>(), o.val, o.selfv, N, E, dEdq, s);
    launch_forces(T->q.as<double>(), o.grad, o.selfg, N, scale, F, s);
    return RS_OK;
  });
}

rs_status rs_rbf_matvec(rs_ctx* ctx, const rs_factors* f, const double* c, double* y,
                        void* stream) {
  return guarded([&]() -> rs_status {
    RS_REQUIRE(ctx && f && c && y, "null argument");
    RS_REQUIRE(f->device == ctx->device, "factors built for another device");
    RS_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = f->grid.n;
    const int R = f->table.R, R_l = f->table.R_l, ncu = ctx->num_cu;
    const double h = 2.0 * f->grid.b / (double)n;
    const int64_t n2 = n * n, n3 = n2 * n;
    DevBuf T((size_t)R * n2 * sizeof(double), s), Acat((size_t)R * n2 * sizeof(double), s);
    DevBuf Z1((size_t)n3 * sizeof(double), s), Z2((size_t)R * n3 * sizeof(double), s);
    launch_rbf_toeplitz(f->t_dev, f->a_dev, R, R_l, n, h, (f->table.n_s - 1) / 2, T.as<double>(),
                        Acat.as<double>(), s);
    // y = sum_k a_k (T_k (x) T_k (x) T_k) c: modes 3 and 2 per term (Z2_k kept
    // for every k), then mode 1 and the sum over k in one GEMM of depth R n
    Gemm64 g3, g2, g1;
    g3.M = n2; g3.N = n; g3.K = n;               // Z1 = c_(12) T_k
    g3.A = c; g3.sam = n; g3.sak = 1;
    g3.sbk = n; g3.sbn = 1;
    g3.C = Z1.as<double>(); g3.scm = n; g3.scn = 1;
    g2.M = n; g2.N = n; g2.K = n; g2.batch = n;   // Z2_k[i1] = T_k Z1[i1]
    g2.sam = n; g2.sak = 1; g2.sab = 0;
    g2.B = Z1.as<double>(); g2.sbk = n; g2.sbn = 1; g2.sbb = n2;
    g2.scm = n; g2.scn = 1; g2.scb = n2;
    g1.M = n; g1.N = n2; g1.K = (int64_t)R * n;   // y = [a_1 T_1 .. a_R T_R] [Z2_1; ..; Z2_R]
    g1.A = Acat.as<double>(); g1.sam = (int64_t)R * n; g1.sak = 1;
    g1.B = Z2.as<double>(); g1.sbk = n2; g1.sbn = 1;
    g1.C = y; g1.scm = n2; g1.scn = 1;
    DevBuf work(std::max({gemm64_workspace_bytes(g3, ncu), gemm64_workspace_bytes(g2, ncu),
                          gemm64_workspace_bytes(g1, ncu)}),
                s);
    for (int k = 0; k < R; ++k) {
      const double* Tk = T.as<double>() + (int64_t)k * n2;
      g3.B = Tk;
      gemm64(g3, ncu, work.as<double>(), s);
      g2.A = Tk;
      g2.C = Z2.as<double>() + (int64_t)k * n3;
      gemm64(g2, ncu, work.as<double>(), s);
    }
    gemm64(g1, ncu, work.as<double>(), s);
    return RS_OK;
  });
}

rs_status rs_dot(const rs_tensor* A, const rs_tensor* B, double* out, void* stream) {
  return guarded([&]() -> rs_status {
    RS_REQUIRE(A && B && out, "null argument");
    RS_REQUIRE(A->ctx->device == B->ctx->device, "tensors on different devices");
    RS_REQUIRE(A->n == B->n && A->b == B->b, "the tensors must live on the same grid (n and b)");
    RS_HIP(hipSetDevice(A->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = A->n;
    const int ncu = A->ctx->num_cu;
    const int ra[3] = {A->r[0], A->r[1], A->r[2]}, rb[3] = {B->r[0], B->r[1], B->r[2]};
    // <A_l, B_l> = sum beta_A[abc] beta_B[a'b'c'] M1[a,a'] M2[b,b'] M3[c,c'],
    // M_l = V_l^A^T V_l^B: X = beta_A x_1 M1^T x_2 M2^T x_3 M3^T, then X . beta_B
    Gemm64 gm[3], g1, g2, g3;
    DevBuf M[3];
    for (int l = 0; l < 3; ++l) {
      M[l] = DevBuf((size_t)ra[l] * rb[l] * sizeof(double), s);
      Gemm64& g = gm[l];   // M_l (ra x rb) = V_A^T V_B, contraction over the n grid points
      g.M = ra[l]; g.N = rb[l]; g.K = n;
      g.A = A->Q[l].as<double>(); g.sam = 1; g.sak = ra[l];
      g.B = B->Q[l].as<double>(); g.sbk = rb[l]; g.sbn = 1;
      g.C = M[l].as<double>(); g.scm = rb[l]; g.scn = 1;
    }
    DevBuf X1((size_t)rb[0] * ra[1] * ra[2] * sizeof(double), s);
    DevBuf X2((size_t)rb[0] * rb[1] * ra[2] * sizeof(double), s);
    DevBuf X3((size_t)rb[0] * rb[1] * rb[2] * sizeof(double), s);
    // X1[a', (b, c)] = sum_a M1[a, a'] beta_A[a, (b, c)]
    g1.M = rb[0]; g1.N = (int64_t)ra[1] * ra[2]; g1.K = ra[0];
    g1.A = M[0].as<double>(); g1.sam = 1; g1.sak = rb[0];
    g1.B = A->beta.as<double>(); g1.sbk = (int64_t)ra[1] * ra[2]; g1.sbn = 1;
    g1.C = X1.as<double>(); g1.scm = (int64_t)ra[1] * ra[2]; g1.scn = 1;
    // X2[a'][b', c] = sum_b M2[b, b'] X1[a'][b, c]   (batched over a')
    g2.M = rb[1]; g2.N = ra[2]; g2.K = ra[1]; g2.batch = rb[0];
    g2.A = M[1].as<double>(); g2.sam = 1; g2.sak = rb[1]; g2.sab = 0;
    g2.B = X1.as<double>(); g2.sbk = ra[2]; g2.sbn = 1; g2.sbb = (int64_t)ra[1] * ra[2];
    g2.C = X2.as<double>(); g2.scm = ra[2]; g2.scn = 1; g2.scb = (int64_t)rb[1] * ra[2];
    // X3[(a', b'), c'] = sum_c X2[(a', b'), c] M3[c, c']
    g3.M = (int64_t)rb[0] * rb[1]; g3.N = rb[2]; g3.K = ra[2];
    g3.A = X2.as<double>(); g3.sam = ra[2]; g3.sak = 1;
    g3.B = M[2].as<double>(); g3.sbk = rb[2]; g3.sbn = 1;
    g3.C = X3.as<double>(); g3.scm = rb[2]; g3.scn = 1;
    size_t wk = 0;
    for (int l = 0; l < 3; ++l) wk = std::max(wk, gemm64_workspace_bytes(gm[l], ncu));
    wk = std::max({wk, gemm64_workspace_bytes(g1, ncu), gemm64_workspace_bytes(g2, ncu),
                   gemm64_workspace_bytes(g3, ncu)});
    DevBuf work(wk, s);
    for (int l = 0; l < 3; ++l) gemm64(gm[l], ncu, work.as<double>(), s);
    gemm64(g1, ncu, work.as<double>(), s);
    gemm64(g2, ncu, work.as<double>(), s);
    gemm64(g3, ncu, work.as<double>(), s);
    DevBuf ll(dot_partials_bytes(), s);
    launch_dot_partial(X3.as<double>(), B->beta.as<double>(), (int64_t)rb[0] * rb[1] * rb[2],
                       ll.as<double>(), s);
    // the touched-brick correction: A's bricks, then B's bricks A does not touch
    auto side = [](const rs_tensor* T) {
      DotSide d;
      d.T2 = T->T2.as<double>(); d.V3 = T->Q[2].as<double>();
      d.pos = T->pos.as<double>(); d.q = T->q.as<double>();
      d.t = T->t_dev.as<double>(); d.a = T->a_dev.as<double>();
      d.start = T->brick_start.as<int>(); d.list = T->brick_list.as<int>();
      d.r3 = T->r[2]; d.R = T->R; d.R_l = T->R_l; d.w = (T->n_s - 1) / 2;
      return d;
    };
    const DotSide da = side(A), db = side(B);
    const int64_t ncols = (int64_t)A->nb * A->nb;
    DevBuf pc((size_t)ncols * sizeof(double), s);
    launch_dot_cols(da, db, A->nb, n, A->b, pc.as<double>(), s);
    launch_dot_final(ll.as<double>(), pc.as<double>(), ncols, out, s);
    return RS_OK;
  });
}

rs_status rs_tensor_grid(const rs_tensor* T, void* grid_out, void* stream) {
  return guarded([&]() -> rs_status {
    RS_REQUIRE(T && grid_out, "null argument");
    RS_HIP(hipSetDevice(T->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = T->n;
    const int r3 = T->r[2], ncu = T->ctx->num_cu;
    if (T->prec == RS_FP64) {
      if (!grid64_stream(T->T2.as<double>(), T->Q[2].as<double>(), n, r3, (double*)grid_out, ncu,
                         T->ctx->lds_limit, s)) {
        const Gemm64 gg = grid_gemm(T, grid_out);
        DevBuf wg(gemm64_workspace_bytes(gg, ncu), s);
        gemm64(gg, ncu, wg.as<double>(), s);
      }
    } else {
      // T2 split under the exponent the assembly's grid used: the same bits
      DevBuf wg(grid_mixed_workspace_bytes(n, r3), s);
      grid_mixed(contraction_prec(T->prec), T->T2.as<double>(), T->Q[2].as<double>(), n, r3,
                 (float*)grid_out, wg.p, ncu, s, false, T->t2exp.as<int>());
    }
    short_gather(grid_out, T->prec != RS_FP64, T->pos.as<double>(), T->q.as<double>(),
                 T->t_dev.as<double>(), T->a_dev.as<double>(), T->R, T->R_l, n, T->b, T->n_s, T->nb,
                 T->brick_start.as<int>(), T->brick_list.as<int>(), T->brick_active.as<int>(),
                 T->active_cap, ncu, s);
    return RS_OK;
  });
}

rs_status rs_gradient_grid(const rs_tensor* T, int32_t axis, void* grid_out, void* stream) {
  return guarded([&]() -> rs_status {
    RS_REQUIRE(T && grid_out, "null argument");
    RS_REQUIRE(axis >= 0 && axis <= 2, "axis must be 0, 1 or 2");
    RS_HIP(hipSetDevice(T->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = T->n;
    const int r3 = T->r[2], ra = T->r[axis];
    const int ncu = T->ctx->num_cu;
    // long range: the Tucker tensor with the axis factor replaced by its
    // finite difference (eq Gradients_Tens, the Tucker form of the sum)
    DevBuf dv((size_t)n * ra * sizeof(double), s);
    launch_fd_rows(T->Q[axis].as<double>(), n, ra, T->h, dv.as<double>(), s);
    DevBuf t2d;
    const double* T2src = T->T2.as<double>();
    const double* V3 = T->Q[2].as<double>();
    const bool f64 = T->prec == RS_FP64;
    DevBuf wg(f64 ? 0 : grid_mixed_workspace_bytes(n, r3), s);
    bool planes_ready = false;
    if (axis == 2) {
      V3 = dv.as<double>();
    } else {
      // the two expansions as in the assembly (the second in split precision
      // for split tensors, writing the grid's T2 planes as it goes)
      const double* V1 = axis == 0 ? dv.as<double>() : nullptr;
      const double* V2 = axis == 1 ? dv.as<double>() : nullptr;
      t2d = DevBuf((size_t)n * n * r3 * sizeof(double), s);
      DevBuf X((size_t)n * T->r[1] * r3 * sizeof(double), s);
      const Gemm64 g1 = expand1_gemm(T, X.as<double>(), V1);
      DevBuf w1(gemm64_workspace_bytes(g1, ncu), s);
      gemm64(g1, ncu, w1.as<double>(), s);
      if (f64) {
        const Gemm64 g2 = expand2_gemm(T, X.as<double>(), V2, t2d.as<double>());
        DevBuf w2(gemm64_workspace_bytes(g2, ncu), s);
        gemm64(g2, ncu, w2.as<double>(), s);
      } else {
        DevBuf w2(expand2_mixed_workspace_bytes(n, T->r[1], r3), s), e2(sizeof(int), s);
        expand2_mixed(contraction_prec(T->prec), X.as<double>(), V2 ? V2 : T->Q[1].as<double>(), n,
                      T->r[1], r3, t2d.as<double>(), w2.p, wg.p, e2.as<int>(), s);
        planes_ready = true;
      }
      T2src = t2d.as<double>();
    }
    if (f64) {
      if (!grid64_stream(T2src, V3, n, r3, (double*)grid_out, ncu, T->ctx->lds_limit, s)) {
        const Gemm64 gg = grid_gemm(T, grid_out, T2src, V3);
        DevBuf wgg(gemm64_workspace_bytes(gg, ncu), s);
        gemm64(gg, ncu, wgg.as<double>(), s);
      }
    } else {
      grid_mixed(contraction_prec(T->prec), T2src, V3, n, r3, (float*)grid_out, wg.p, ncu, s,
                 planes_ready, planes_ready ? nullptr : T->t2exp.as<int>());
    }
    // short range: brick lists for windows one cell wider on each side, then
    // the finite difference of every local term
    const int ns2 = T->n_s + 2, nbricks = T->nb * T->nb * T->nb;
    DevBuf counts((size_t)(nbricks + 1) * sizeof(int), s), start((size_t)(nbricks + 1) * sizeof(int), s);
    RS_HIP(hipMemsetAsync(counts.p, 0, counts.bytes, s));
    short_bin_count(T->pos.as<double>(), T->N, n, T->b, ns2, T->nb, counts.as<int>(), s);
    exclusive_scan_int(counts.as<int>(), start.as<int>(), nbricks + 1, s);
    int total = 0;
    RS_HIP(hipMemcpyAsync(&total, start.as<int>() + nbricks, sizeof(int), hipMemcpyDeviceToHost, s));
    RS_HIP(hipStreamSynchronize(s));
    DevBuf list((size_t)std::max(total, 1) * sizeof(int), s);
    RS_HIP(hipMemsetAsync(counts.p, 0, counts.bytes, s));
    short_bin_fill(T->pos.as<double>(), T->N, n, T->b, ns2, T->nb, start.as<int>(), counts.as<int>(),
                   list.as<int>(), s);
    const int64_t cap = short_active_capacity(T->N, ns2, T->nb);
    DevBuf active((size_t)(cap + 1) * sizeof(int), s);
    short_bin_sort(start.as<int>(), list.as<int>(), nbricks, active.as<int>(), cap, s);
    short_gather(grid_out, T->prec != RS_FP64, T->pos.as<double>(), T->q.as<double>(),
                 T->t_dev.as<double>(), T->a_dev.as<double>(), T->R, T->R_l, n, T->b, T->n_s, T->nb,
                 start.as<int>(), list.as<int>(), active.as<int>(), cap, ncu, s, axis);
    return RS_OK;
  });
}

size_t rs_footprint_bytes(const rs_grid* grid, const rs_fdesc* fdesc, int64_t N, int32_t r_max,
                          int32_t prec, int32_t with_grid) {
  (void)with_grid;
  if (!grid || !fdesc || N < 1) return 0;
  Table t;
  try {
    t = build_table(*grid, *fdesc);
  } catch (...) {
    return 0;
  }
  const int64_t n = grid->n, K = N * t.R_l;
  const int64_t r = r_max > 0 ? std::min<int64_t>(r_max, n) : std::min<int64_t>(n, 256);
  const int64_t p = std::min<int64_t>(n, r + 16);
  const size_t d = sizeof(double);
  const int ncu = 256;
  // Upper bound of what one assembly holds at once: its inputs, the factors
  // and the Gram stay live until the last launch is enqueued, together with
  // the subspace basis, the eigenvectors, the result's own buffers and the
  // scratch arena of the rank-sized stages.
  Gemm64 gram;
  gram.M = n; gram.N = n; gram.K = K; gram.batch = 3; gram.upper_only = 1;
  Gemm64 yty;
  yty.M = p; yty.N = p; yty.K = n; yty.batch = 3; yty.upper_only = 1;
  Gemm64 gx;
  gx.M = n; gx.N = p; gx.K = n; gx.batch = 3;
  Gemm64 zz;
  zz.M = r; zz.N = r; zz.K = p; zz.batch = 3; zz.upper_only = 1;
  size_t inputs = (size_t)N * 4 * d + 2 * (size_t)t.R * d;
  size_t factors = (size_t)(3 * n * K + 3 * K) * d +
                   (prec == RS_FP64 || prec == RS_MIXED_BF16 ? 0 : (size_t)12 * ((n + 31) / 32 * 32) * K);
  size_t gram_b = (size_t)3 * n * n * d + gemm64_workspace_bytes(gram, ncu);
  // the pieces of the pre-readback arena: subspace, eigenproblem, eigenvectors
  size_t eig = (size_t)(3 * n * p * 2 + 3 * p * p * 2) * d +
               std::max({sketch64_workspace_bytes(n, K, 3, p, ncu), gemm64_workspace_bytes(gx, ncu),
                         gemm64_workspace_bytes(yty, ncu)}) +
               eig_sym_workspace_bytes((int)p, (int)r, 3) + (size_t)(3 * p * r * 2 + 3 * r * r) * d +
               gemm64_workspace_bytes(zz, ncu) + 32 * 256;
  size_t result = (size_t)(3 * n * r + r * r * r + n * n * r) * d;
  size_t arena = (size_t)(3 * p * r + 3 * K * r + n * r * r) * d +
                 (prec == RS_FP64 ? core64_workspace_bytes((int)r, (int)r, (int)r, K, ncu)
                                  : core_mixed_workspace_bytes((int)r, (int)r, (int)r, K, ncu) +
                                        proj_mixed_workspace_bytes(n, K, (int)r, false)) +
                 (size_t)8 * n * n * d;  // split-K partials of the projections and expansions (bound)
  size_t bins = ((n / 8 + 1) * (n / 8 + 1) * (n / 8 + 1) * 3 + 64 * N + 1) * sizeof(int);
  return inputs + factors + gram_b + eig + result + arena + bins;
}

rs_status rs_tensor_info(const rs_tensor* T, rs_info* info) {
  return guarded([&]() -> rs_status {
    RS_REQUIRE(T && info, "null argument");
    rs_info I{};
    I.N = T->N;
    I.n = T->n;
    I.b = T->b;
    I.h = T->h;
    I.R = T->R;
    I.R_l = T->R_l;
    I.n_s = T->n_s;
    I.prec = T->prec;
    I.interp_order = T->interp;
    for (int l = 0; l < 3; ++l) {
      I.ranks[l] = T->r[l];
      I.subspace[l] = T->p[l];
      I.sigma_first[l] = T->sigma1[l];
      I.sigma_last_kept[l] = T->sig_kept[l];
      I.sigma_next[l] = T->sig_next[l];
    }
    I.S0 = T->table.S0;
    I.S_l0 = T->table.S_l0;
    I.tucker_storage = (int64_t)T->r[0] * T->r[1] * T->r[2] + T->n * (T->r[0] + T->r[1] + T->r[2]);
    size_t bytes = T->pos.bytes + T->q.bytes + T->t_dev.bytes + T->a_dev.bytes + T->beta.bytes +
                   T->T2.bytes + T->T2f.bytes + T->V3f.bytes + T->brick_start.bytes +
                   T->brick_list.bytes + T->brick_active.bytes;
    for (int l = 0; l < 3; ++l) bytes += T->Q[l].bytes;
    I.device_bytes = (int64_t)bytes;
    I.rank_capped = T->rank_capped;
    if (!T->eig_events.empty()) {
      RS_HIP(hipEventSynchronize(T->eig_events[RS_EIG_PHASES]));
      for (int k = 0; k < RS_EIG_PHASES; ++k) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, T->eig_events[k], T->eig_events[k + 1]) == hipSuccess)
          I.eig_phase_ms[k] = ms;
      }
    }
    if (!T->events.empty() && (T->recorded >> RS_STAGE_COUNT) & 1u) {
      RS_HIP(hipEventSynchronize(T->events[RS_STAGE_COUNT]));
      // a stage runs from its event to the next recorded one; a stage whose
      // event was not recorded (it did not run, or is not timed) reports 0
      for (int k = 0; k < RS_STAGE_COUNT; ++k) {
        I.stage_ms[k] = 0.0;
        if (!((T->recorded >> k) & 1u)) continue;
        int j = k + 1;
        while (!((T->recorded >> j) & 1u)) ++j;   // bit RS_STAGE_COUNT is set
        float ms = 0.f;
        RS_HIP(hipEventElapsedTime(&ms, T->events[k], T->events[j]));
        I.stage_ms[k] = ms;
      }
      if (T->kevents.begin) {
        float ms = 0.f;
        RS_HIP(hipEventElapsedTime(&ms, T->kevents.begin, T->kevents.end));
        I.stage_ms[RS_STAGE_CORE_KERNEL] = ms;
      }
    }
    *info = I;
    return RS_OK;
  });
}

rs_status rs_tensor_export(const rs_tensor* T, double* V1, double* V2, double* V3, double* beta,
                           void* stream) {
  return guarded([&]() -> rs_status {
    RS_REQUIRE(T, "null tensor");
    RS_HIP(hipSetDevice(T->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    double* Vs[3] = {V1, V2, V3};
    for (int l = 0; l < 3; ++l)
      if (Vs[l]) RS_HIP(hipMemcpyAsync(Vs[l], T->Q[l].p, T->Q[l].bytes, hipMemcpyDeviceToDevice, s));
    if (beta) RS_HIP(hipMemcpyAsync(beta, T->beta.p, T->beta.bytes, hipMemcpyDeviceToDevice, s));
    RS_HIP(hipStreamSynchronize(s));
    return RS_OK;
  });
}

static const char kMagic[8] = {'R', 'S', 'T', 'U', 'C', 'K', '0', '1'};

rs_status rs_tensor_save(const rs_tensor* T, const char* path) {
  return guarded([&]() -> rs_status {
    RS_REQUIRE(T && path, "null argument");
    RS_HIP(hipSetDevice(T->ctx->device));
    RS_HIP(hipStreamSynchronize(T->stream));
    std::ofstream os(path, std::ios::binary);
    RS_REQUIRE(os.good(), std::string("cannot open ") + path);
    auto put = [&](const void* p, size_t nb) { os.write((const char*)p, (std::streamsize)nb); };
    auto put_dev = [&](const DevBuf& b) {
      std::vector<char> h(b.bytes);
      if (b.bytes) RS_HIP(hipMemcpy(h.data(), b.p, b.bytes, hipMemcpyDeviceToHost));
      uint64_t nb = b.bytes;
      put(&nb, 8);
      put(h.data(), b.bytes);
    };
    put(kMagic, 8);
    int32_t ints[10] = {T->R, T->R_l, T->n_s, T->kernel, T->prec, T->interp,
                        T->r[0], T->r[1], T->r[2], 0};
    put(ints, sizeof(ints));
    int64_t sizes[2] = {T->N, T->n};
    put(sizes, sizeof(sizes));
    double dbl[2] = {T->b, T->lambda};
    put(dbl, sizeof(dbl));
    put(T->table.t.data(), T->R * sizeof(double));
    put(T->table.a.data(), T->R * sizeof(double));
    double sig[9];
    for (int l = 0; l < 3; ++l) {
      sig[l] = T->sigma1[l];
      sig[3 + l] = T->sig_kept[l];
      sig[6 + l] = T->sig_next[l];
    }
    put(sig, sizeof(sig));
    put_dev(T->pos);
    put_dev(T->q);
    for (int l = 0; l < 3; ++l) put_dev(T->Q[l]);
    put_dev(T->beta);
    RS_REQUIRE(os.good(), "write failed");
    return RS_OK;
  });
}

rs_status rs_tensor_load(rs_ctx* ctx, const char* path, rs_tensor** out) {
  return guarded([&]() -> rs_status {
    RS_REQUIRE(ctx && path && out, "null argument");
    RS_HIP(hipSetDevice(ctx->device));
    std::ifstream is(path, std::ios::binary);
    RS_REQUIRE(is.good(), std::string("cannot open ") + path);
    auto get = [&](void* p, size_t nb) {
      is.read((char*)p, (std::streamsize)nb);
      RS_REQUIRE(is.good(), "truncated tensor file");
    };
    char magic[8];
    get(magic, 8);
    RS_REQUIRE(std::memcmp(magic, kMagic, 8) == 0, "not an RS tensor file (bad magic/version)");
    auto T = std::make_unique<rs_tensor>();
    T->ctx = ctx;
    T->ctx_ref.set(ctx);
    hipStream_t s = nullptr;
    T->stream = s;
    int32_t ints[10];
    get(ints, sizeof(ints));
    T->R = ints[0]; T->R_l = ints[1]; T->n_s = ints[2]; T->kernel = ints[3]; T->prec = ints[4];
    T->interp = ints[5];
    for (int l = 0; l < 3; ++l) T->r[l] = ints[6 + l];
    int64_t sizes[2];
    get(sizes, sizeof(sizes));
    T->N = sizes[0];
    T->n = sizes[1];
    double dbl[2];
    get(dbl, sizeof(dbl));
    T->b = dbl[0];
    T->lambda = dbl[1];
    T->h = 2.0 * T->b / (double)T->n;
    RS_REQUIRE(T->R >= 3 && T->R <= 256 && T->N >= 1 && T->n >= 8, "corrupt tensor header");
    T->table.R = T->R;
    T->table.R_l = T->R_l;
    T->table.n_s = T->n_s;
    T->table.t.resize(T->R);
    T->table.a.resize(T->R);
    get(T->table.t.data(), T->R * sizeof(double));
    get(T->table.a.data(), T->R * sizeof(double));
    T->table.S0 = 0;
    T->table.S_l0 = 0;
    for (int k = 0; k < T->R; ++k) {
      T->table.S0 += T->table.a[k];
      if (k < T->R_l) T->table.S_l0 += T->table.a[k];
    }
    double sig[9];
    get(sig, sizeof(sig));
    for (int l = 0; l < 3; ++l) {
      T->sigma1[l] = sig[l];
      T->sig_kept[l] = sig[3 + l];
      T->sig_next[l] = sig[6 + l];
    }
    auto get_dev = [&](DevBuf& b, size_t expect) {
      uint64_t nb;
      get(&nb, 8);
      RS_REQUIRE(nb == expect, "corrupt tensor file (buffer size)");
      std::vector<char> h(nb);
      get(h.data(), nb);
      b = DevBuf(nb, s);
      RS_HIP(hipMemcpyAsync(b.p, h.data(), nb, hipMemcpyHostToDevice, s));
      RS_HIP(hipStreamSynchronize(s));
    };
    get_dev(T->pos, (size_t)T->N * 3 * sizeof(double));
    get_dev(T->q, (size_t)T->N * sizeof(double));
    for (int l = 0; l < 3; ++l) get_dev(T->Q[l], (size_t)T->n * T->r[l] * sizeof(double));
    get_dev(T->beta, (size_t)T->r[0] * T->r[1] * T->r[2] * sizeof(double));
    T->t_dev = DevBuf((size_t)T->R * sizeof(double), s);
    T->a_dev = DevBuf((size_t)T->R * sizeof(double), s);
    RS_HIP(hipMemcpyAsync(T->t_dev.p, T->table.t.data(), T->t_dev.bytes, hipMemcpyHostToDevice, s));
    RS_HIP(hipMemcpyAsync(T->a_dev.p, T->table.a.data(), T->a_dev.bytes, hipMemcpyHostToDevice, s));
    // rebuild the short-range lists and the expansion intermediate
    T->nb = bricks_per_axis(T->n);
    const int nbricks = T->nb * T->nb * T->nb;
    DevBuf counts((size_t)(nbricks + 1) * sizeof(int), s);
    RS_HIP(hipMemsetAsync(counts.p, 0, counts.bytes, s));
    short_bin_count(T->pos.as<double>(), T->N, T->n, T->b, T->n_s, T->nb, counts.as<int>(), s);
    T->brick_start = DevBuf((size_t)(nbricks + 1) * sizeof(int), s);
    exclusive_scan_int(counts.as<int>(), T->brick_start.as<int>(), nbricks + 1, s);
    int total = 0;
    RS_HIP(hipMemcpyAsync(&total, T->brick_start.as<int>() + nbricks, sizeof(int),
                          hipMemcpyDeviceToHost, s));
    RS_HIP(hipStreamSynchronize(s));
    T->n_pairs = total;
    T->brick_list = DevBuf((size_t)std::max(total, 1) * sizeof(int), s);
    RS_HIP(hipMemsetAsync(counts.p, 0, counts.bytes, s));
    short_bin_fill(T->pos.as<double>(), T->N, T->n, T->b, T->n_s, T->nb, T->brick_start.as<int>(),
                   counts.as<int>(), T->brick_list.as<int>(), s);
    T->active_cap = short_active_capacity(T->N, T->n_s, T->nb);
    T->brick_active = DevBuf((size_t)(T->active_cap + 1) * sizeof(int), s);
    short_bin_sort(T->brick_start.as<int>(), T->brick_list.as<int>(), nbricks,
                   T->brick_active.as<int>(), T->active_cap, s);
    T->T2 = DevBuf((size_t)T->n * T->n * T->r[2] * sizeof(double), s);
    if (T->prec != RS_FP64) T->t2exp = DevBuf(sizeof(int), s);
    DevBuf scratch(expansion_scratch(T.get(), false).total, s);
    build_expansion(T.get(), nullptr, scratch.as<char>(), s);
    make_fp32_field(T.get(), s);
    RS_HIP(hipStreamSynchronize(s));
    *out = T.release();
    return RS_OK;
  });
}

void rs_tensor_free(rs_tensor* T) {
  if (!T) return;
  (void)hipSetDevice(T->ctx->device);
  delete T;  // buffers are released in stream order on the assembly stream
}

}  // extern "C"
