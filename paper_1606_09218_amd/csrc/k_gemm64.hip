// FP64 GEMM on the CDNA matrix cores (v_mfma_f64_16x16x4f64).
//
//   C[bt](m, n) = sum_k A[bt](m, k) * B[bt](k, n) * kscale[k]
//
// with arbitrary element strides, so one kernel serves every dense
// contraction of the path: the charge-weighted Gram U diag(w) U^T, the
// eigensolver's products, the projection V^T U and the three mode products
// that expand the Tucker tensor onto the grid.
//
// Tiling: 64 x 64 output tile per 256-thread workgroup (4 wave64s in a 2 x 2
// arrangement, 32 x 32 per wave = 2 x 2 MFMA blocks of 16 x 16), K staged
// through LDS in steps of 16 with a register prefetch of the next step.
// Large K is split across workgroups; the partial tiles are summed by a
// second kernel in a fixed order, so the result is deterministic.
#include "rs_internal.h"

namespace rs {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 16, PAD = 2;
constexpr int LDA = BM + PAD, LDB = BN + PAD;

struct GemmDev {
  int64_t M, N, K;
  const double* A; int64_t sam, sak, sab;
  const double* B; int64_t sbk, sbn, sbb;
  double* C; int64_t scm, scn, scb;
  const double* kscale;
  double* part;        // split-K partials [bt][split][M][N] (or null)
  int splits;
  int64_t kchunk;      // K range per split (multiple of BK)
  int upper_only;
  int nontemporal;
  int tiles_m, tiles_n;
};

// Load the BK x 64 slab of A (as A^T: [k][m]) or B ([k][n]) into registers.
// Template flag: true when the 64-wide index (m or n) is the contiguous one.
template <bool WIDE_CONTIG>
__device__ __forceinline__ void load_slab(const double* __restrict__ P, int64_t s_wide,
                                          int64_t s_k, int64_t wide0, int64_t k0, int64_t W,
                                          int64_t K, const double* __restrict__ kscale,
                                          double (&reg)[4], int tid) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    int wl, kl;
    if (WIDE_CONTIG) {
      wl = tid & 63;
      kl = (tid >> 6) + 4 * r;
    } else {
      kl = tid & 15;
      wl = (tid >> 4) + 16 * r;
    }
    int64_t w = wide0 + wl, k = k0 + kl;
    double v = 0.0;
    if (w < W && k < K) {
      v = P[w * s_wide + k * s_k];
      if (kscale) v *= kscale[k];
    }
    reg[r] = v;
  }
}

template <bool WIDE_CONTIG>
__device__ __forceinline__ void store_slab(double* lds, int ld, const double (&reg)[4], int tid) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    int wl, kl;
    if (WIDE_CONTIG) {
      wl = tid & 63;
      kl = (tid >> 6) + 4 * r;
    } else {
      kl = tid & 15;
      wl = (tid >> 4) + 16 * r;
    }
    lds[kl * ld + wl] = reg[r];
  }
}

// Operand sources.  Each loads its share (4 values per thread) of a BK x 64
// slab into registers; `store` writes them to LDS as [k][wide].
template <bool WIDE_CONTIG>
struct StridedSrc {
  const double* P;
  int64_t s_wide, s_k, W;
  const double* kscale;
  __device__ __forceinline__ void load(int64_t wide0, int64_t k0, int64_t kend, double (&reg)[4],
                                       int tid) const {
    load_slab<WIDE_CONTIG>(P, s_wide, s_k, wide0, k0, W, kend, kscale, reg, tid);
  }
  __device__ __forceinline__ void store(double* lds, int ld, const double (&reg)[4], int tid) const {
    store_slab<WIDE_CONTIG>(lds, ld, reg, tid);
  }
};

// Khatri-Rao operand of the core contraction, generated on the fly:
// B[j, b*r3 + c] = xi_j * U2t[j*r2 + b] * U3t[j*r3 + c]  (never stored).
struct KhatriRaoSrc {
  const double* U2t;
  const double* U3t;
  const double* xi;
  int r2, r3;
  __device__ __forceinline__ void load(int64_t n0, int64_t k0, int64_t kend, double (&reg)[4],
                                       int tid) const {
    const int64_t bc = n0 + (tid & 63);
    const int64_t W = (int64_t)r2 * r3;
    const int b = (int)(bc / r3), c = (int)(bc - (bc / r3) * r3);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t k = k0 + (tid >> 6) + 4 * r;
      double v = 0.0;
      if (bc < W && k < kend) v = xi[k] * U2t[k * r2 + b] * U3t[k * r3 + c];
      reg[r] = v;
    }
  }
  __device__ __forceinline__ void store(double* lds, int ld, const double (&reg)[4], int tid) const {
    store_slab<true>(lds, ld, reg, tid);
  }
};

// Random test matrix of the range finder, generated on the fly:
// B[k, c] = scale[k] * u(seed, k, c), u uniform in [-1, 1) from a counter hash.
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ULL;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
  return x ^ (x >> 31);
}

struct HashSrc {
  const double* scale;
  uint64_t seed;
  int64_t W;
  __device__ __forceinline__ void load(int64_t n0, int64_t k0, int64_t kend, double (&reg)[4],
                                       int tid) const {
    const int64_t c = n0 + (tid & 63);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t k = k0 + (tid >> 6) + 4 * r;
      double v = 0.0;
      if (c < W && k < kend) {
        const uint64_t h = mix64(seed ^ mix64((uint64_t)k * 0x100000001B3ULL + (uint64_t)c));
        v = scale[k] * ((double)(h >> 11) * (2.0 / 9007199254740992.0) - 1.0);
      }
      reg[r] = v;
    }
  }
  __device__ __forceinline__ void store(double* lds, int ld, const double (&reg)[4], int tid) const {
    store_slab<true>(lds, ld, reg, tid);
  }
};

struct TileOut {
  int64_t M, N;
  double* C; int64_t scm, scn;
  double* part;   // split-K partial base for this (bt, split), row-major M x N, or null
  int nontemporal;
};

// One 64 x 64 output tile over k in [kbeg, kend).
template <class ASrc, class BSrc>
__device__ __forceinline__ void mfma64_tile(const ASrc& as_src, const BSrc& bs_src, int64_t m0,
                                            int64_t n0, int64_t kbeg, int64_t kend,
                                            const TileOut& o) {
  __shared__ double As[2][BK * LDA];
  __shared__ double Bs[2][BK * LDB];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  d4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  double ra[4], rb[4];
  int buf = 0;
  if (kbeg < kend) {
    as_src.load(m0, kbeg, kend, ra, tid);
    bs_src.load(n0, kbeg, kend, rb, tid);
    as_src.store(As[0], LDA, ra, tid);
    bs_src.store(Bs[0], LDB, rb, tid);
  }
  __syncthreads();

  for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) {
      as_src.load(m0, k0 + BK, kend, ra, tid);
      bs_src.load(n0, k0 + BK, kend, rb, tid);
    }
    const double* as = As[buf];
    const double* bs = Bs[buf];
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      double fa[2], fb[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) fa[i] = as[kr * LDA + wm * 32 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) fb[j] = bs[kr * LDB + wn * 32 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i], fb[j], acc[i][j], 0, 0, 0);
    }
    if (more) {
      as_src.store(As[buf ^ 1], LDA, ra, tid);
      bs_src.store(Bs[buf ^ 1], LDB, rb, tid);
    }
    __syncthreads();
    buf ^= 1;
  }

  // epilogue: for v_mfma_f64_16x16x4f64 lane holds D[lane/16 + 4 v][lane%16]
  // of each 16 x 16 block (register v = 0..3)
#pragma unroll
  for (int i = 0; i < 2; ++i) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t col = n0 + wn * 32 + j * 16 + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = m0 + wm * 32 + i * 16 + (lane >> 4) + 4 * v;
        if (row < o.M && col < o.N) {
          const double val = acc[i][j][v];
          if (o.part) {
            o.part[row * o.N + col] = val;
          } else {
            double* dst = o.C + row * o.scm + col * o.scn;
            if (o.nontemporal) __builtin_nontemporal_store(val, dst);
            else *dst = val;
          }
        }
      }
    }
  }
}

template <bool A_MC, bool B_NC>
__global__ __launch_bounds__(256) void gemm64_kernel(GemmDev g) {
  const int tile = blockIdx.x;
  const int tm = tile / g.tiles_n, tn = tile - tm * g.tiles_n;
  if (g.upper_only && tm > tn) return;
  const int bt = blockIdx.y;
  const int split = blockIdx.z;
  const int64_t kbeg = (int64_t)split * g.kchunk;
  int64_t kend = kbeg + g.kchunk;
  if (kend > g.K) kend = g.K;
  StridedSrc<A_MC> as{g.A + (int64_t)bt * g.sab, g.sam, g.sak, g.M, nullptr};
  StridedSrc<B_NC> bs{g.B + (int64_t)bt * g.sbb, g.sbn, g.sbk, g.N, g.kscale};
  TileOut o;
  o.M = g.M;
  o.N = g.N;
  o.C = g.C + (int64_t)bt * g.scb;
  o.scm = g.scm;
  o.scn = g.scn;
  o.part = g.part ? g.part + ((int64_t)bt * g.splits + split) * g.M * g.N : nullptr;
  o.nontemporal = g.nontemporal;
  mfma64_tile(as, bs, (int64_t)tm * BM, (int64_t)tn * BN, kbeg, kend, o);
}

// Y[bt] (M x N, col-major) = A[bt] (M x K, m-contiguous) * Omega_bt (K x N, hashed)
__global__ __launch_bounds__(256) void sketch64_kernel(GemmDev g, uint64_t seed) {
  const int tile = blockIdx.x;
  const int tm = tile / g.tiles_n, tn = tile - tm * g.tiles_n;
  const int bt = blockIdx.y;
  const int split = blockIdx.z;
  const int64_t kbeg = (int64_t)split * g.kchunk;
  int64_t kend = kbeg + g.kchunk;
  if (kend > g.K) kend = g.K;
  StridedSrc<true> as{g.A + (int64_t)bt * g.sab, 1, g.sak, g.M, nullptr};
  HashSrc bs{g.kscale + (int64_t)bt * g.sbb, seed + 0x51ED27ULL * (uint64_t)(bt + 1), g.N};
  TileOut o;
  o.M = g.M;
  o.N = g.N;
  o.C = g.C + (int64_t)bt * g.scb;
  o.scm = g.scm;
  o.scn = g.scn;
  o.part = g.part ? g.part + ((int64_t)bt * g.splits + split) * g.M * g.N : nullptr;
  o.nontemporal = 0;
  mfma64_tile(as, bs, (int64_t)tm * BM, (int64_t)tn * BN, kbeg, kend, o);
}

struct CoreDev {
  const double* U1t;
  KhatriRaoSrc kr;
  int r1;
  int64_t K;
  double* beta;
  double* part;
  int splits;
  int64_t kchunk;
  int tiles_n;
};

// beta_(1) (r1 x r2 r3) = U1t^T diag(xi) (U3t (.) U2t): the core of the
// RHOSVD, eq CP_form_RHOSVD, as one GEMM whose right operand is the
// Khatri-Rao product formed while staging it in LDS.
__global__ __launch_bounds__(256) void core64_kernel(CoreDev g) {
  const int tile = blockIdx.x;
  const int tm = tile / g.tiles_n, tn = tile - tm * g.tiles_n;
  const int split = blockIdx.z;
  const int64_t kbeg = (int64_t)split * g.kchunk;
  int64_t kend = kbeg + g.kchunk;
  if (kend > g.K) kend = g.K;
  const int64_t W = (int64_t)g.kr.r2 * g.kr.r3;
  StridedSrc<true> as{g.U1t, 1, g.r1, g.r1, nullptr};
  TileOut o;
  o.M = g.r1;
  o.N = W;
  o.C = g.beta;
  o.scm = W;
  o.scn = 1;
  o.part = g.part ? g.part + (int64_t)split * g.r1 * W : nullptr;
  o.nontemporal = 0;
  mfma64_tile(as, g.kr, (int64_t)tm * BM, (int64_t)tn * BN, kbeg, kend, o);
}

__global__ void core64_reduce_kernel(const double* __restrict__ part, int splits, int64_t total,
                                     double* __restrict__ beta) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int sp = 0; sp < splits; ++sp) s += part[(int64_t)sp * total + e];
    beta[e] = s;
  }
}

// Fixed-order sum of the split-K partials; for an upper-only symmetric
// product the lower triangle of tiles is read from its mirror.
__global__ void gemm64_reduce_kernel(GemmDev g) {
  const int bt = blockIdx.y;
  const int64_t total = g.M * g.N;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t row = e / g.N, col = e - row * g.N;
    int64_t sr = row, sc = col;
    if (g.upper_only && (row / BM) > (col / BN)) {
      sr = col;
      sc = row;
    }
    double s = 0.0;
    for (int sp = 0; sp < g.splits; ++sp)
      s += g.part[(((int64_t)bt * g.splits + sp) * g.M + sr) * g.N + sc];
    double* dst = g.C + (int64_t)bt * g.scb + row * g.scm + col * g.scn;
    *dst = s;
  }
}

static void plan(const Gemm64& g, int num_cu, int& splits, int64_t& kchunk, int& tm, int& tn) {
  tm = (int)((g.M + BM - 1) / BM);
  tn = (int)((g.N + BN - 1) / BN);
  int64_t tiles = (int64_t)tm * tn;
  if (g.upper_only) tiles = (int64_t)tm * (tm + 1) / 2;
  tiles *= g.batch;
  const int64_t target = 2LL * num_cu;
  splits = 1;
  if (tiles < target && g.K > 4 * BK) {
    int64_t want = (target + tiles - 1) / tiles;
    int64_t maxs = g.K / (4 * BK);  // at least 64 k per split
    splits = (int)std::max<int64_t>(1, std::min<int64_t>(want, std::min<int64_t>(maxs, 64)));
  }
  kchunk = (g.K + splits - 1) / splits;
  kchunk = (kchunk + BK - 1) / BK * BK;
  splits = (int)((g.K + kchunk - 1) / kchunk);
  if (splits < 1) splits = 1;
}

size_t gemm64_workspace_bytes(const Gemm64& g, int num_cu) {
  int splits, tm, tn;
  int64_t kchunk;
  plan(g, num_cu, splits, kchunk, tm, tn);
  if (splits == 1 && !g.upper_only) return 0;
  return (size_t)g.batch * splits * g.M * g.N * sizeof(double);
}

void gemm64(const Gemm64& g, int num_cu, double* work, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return;
  GemmDev d;
  d.M = g.M; d.N = g.N; d.K = g.K;
  d.A = g.A; d.sam = g.sam; d.sak = g.sak; d.sab = g.sab;
  d.B = g.B; d.sbk = g.sbk; d.sbn = g.sbn; d.sbb = g.sbb;
  d.C = g.C; d.scm = g.scm; d.scn = g.scn; d.scb = g.scb;
  d.kscale = g.kscale;
  d.upper_only = g.upper_only;
  d.nontemporal = g.nontemporal;
  plan(g, num_cu, d.splits, d.kchunk, d.tiles_m, d.tiles_n);
  const bool use_part = d.splits > 1 || g.upper_only;
  d.part = use_part ? work : nullptr;
  if (use_part && !work) throw Error{RS_E_DEVICE, "gemm64: missing split-K workspace"};
  if (g.K <= 0) {
    // empty contraction: zero output through the reduce path with no splits
    throw Error{RS_E_INVALID, "gemm64: K must be positive"};
  }
  const bool amc = (g.sam == 1), akc = (g.sak == 1);
  const bool bnc = (g.sbn == 1), bkc = (g.sbk == 1);
  if (!(amc || akc) || !(bnc || bkc)) throw Error{RS_E_DEVICE, "gemm64: unsupported operand strides"};
  dim3 grid((unsigned)(d.tiles_m * d.tiles_n), (unsigned)g.batch, (unsigned)d.splits);
  if (amc && bnc) hipLaunchKernelGGL((gemm64_kernel<true, true>), grid, dim3(256), 0, s, d);
  else if (amc && !bnc) hipLaunchKernelGGL((gemm64_kernel<true, false>), grid, dim3(256), 0, s, d);
  else if (!amc && bnc) hipLaunchKernelGGL((gemm64_kernel<false, true>), grid, dim3(256), 0, s, d);
  else hipLaunchKernelGGL((gemm64_kernel<false, false>), grid, dim3(256), 0, s, d);
  if (use_part) {
    int64_t total = g.M * g.N;
    int64_t blocks = std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(gemm64_reduce_kernel, dim3((unsigned)blocks, (unsigned)g.batch), dim3(256),
                       0, s, d);
  }
}

static void plan_core(int r1, int r2, int r3, int64_t K, int num_cu, int& splits,
                      int64_t& kchunk, int& tm, int& tn) {
  tm = (r1 + BM - 1) / BM;
  tn = (int)(((int64_t)r2 * r3 + BN - 1) / BN);
  int64_t tiles = (int64_t)tm * tn;
  const int64_t target = 2LL * num_cu;
  splits = 1;
  if (tiles < target && K > 16 * BK) {
    int64_t want = (target + tiles - 1) / tiles;
    splits = (int)std::min<int64_t>(want, std::min<int64_t>(K / (16 * BK), 64));
    if (splits < 1) splits = 1;
  }
  kchunk = (K + splits - 1) / splits;
  kchunk = (kchunk + BK - 1) / BK * BK;
  splits = (int)((K + kchunk - 1) / kchunk);
}

size_t core64_workspace_bytes(int r1, int r2, int r3, int64_t K, int num_cu) {
  int splits, tm, tn;
  int64_t kchunk;
  plan_core(r1, r2, r3, K, num_cu, splits, kchunk, tm, tn);
  return splits > 1 ? (size_t)splits * r1 * r2 * r3 * sizeof(double) : 0;
}

void core64(const double* U1t, const double* U2t, const double* U3t, const double* xi, int r1,
            int r2, int r3, int64_t K, double* beta, int num_cu, double* work, hipStream_t s) {
  CoreDev d;
  int tm;
  plan_core(r1, r2, r3, K, num_cu, d.splits, d.kchunk, tm, d.tiles_n);
  d.U1t = U1t;
  d.kr = KhatriRaoSrc{U2t, U3t, xi, r2, r3};
  d.r1 = r1;
  d.K = K;
  d.beta = beta;
  d.part = d.splits > 1 ? work : nullptr;
  if (d.splits > 1 && !work) throw Error{RS_E_DEVICE, "core64: missing workspace"};
  dim3 grid((unsigned)(tm * d.tiles_n), 1, (unsigned)d.splits);
  hipLaunchKernelGGL(core64_kernel, grid, dim3(256), 0, s, d);
  if (d.splits > 1) {
    int64_t total = (int64_t)r1 * r2 * r3;
    unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(core64_reduce_kernel, dim3(blocks), dim3(256), 0, s, (const double*)work,
                       d.splits, total, beta);
  }
}

void sketch64(const double* A, int64_t M, int64_t K, int64_t sab, const double* scale,
              int64_t scale_stride, int batch, int64_t N, uint64_t seed, double* Y, int64_t scm,
              int64_t scn, int num_cu, double* work, hipStream_t s) {
  Gemm64 g;
  g.M = M; g.N = N; g.K = K; g.batch = batch;
  g.A = A; g.sam = 1; g.sak = M; g.sab = sab;
  g.C = Y; g.scm = scm; g.scn = scn; g.scb = M * N;
  g.kscale = scale;
  g.sbb = scale_stride;
  GemmDev d;
  d.M = M; d.N = N; d.K = K;
  d.A = A; d.sam = 1; d.sak = M; d.sab = sab;
  d.B = nullptr; d.sbk = 0; d.sbn = 0; d.sbb = scale_stride;
  d.C = Y; d.scm = scm; d.scn = scn; d.scb = M * N;
  d.kscale = scale;
  d.upper_only = 0;
  d.nontemporal = 0;
  plan(g, num_cu, d.splits, d.kchunk, d.tiles_m, d.tiles_n);
  const bool use_part = d.splits > 1;
  d.part = use_part ? work : nullptr;
  if (use_part && !work) throw Error{RS_E_DEVICE, "sketch64: missing split-K workspace"};
  dim3 grid((unsigned)(d.tiles_m * d.tiles_n), (unsigned)batch, (unsigned)d.splits);
  hipLaunchKernelGGL(sketch64_kernel, grid, dim3(256), 0, s, d, seed);
  if (use_part) {
    int64_t total = M * N;
    int64_t blocks = std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(gemm64_reduce_kernel, dim3((unsigned)blocks, (unsigned)batch), dim3(256), 0,
                       s, d);
  }
}

size_t sketch64_workspace_bytes(int64_t M, int64_t K, int batch, int64_t N, int num_cu) {
  Gemm64 g;
  g.M = M; g.N = N; g.K = K; g.batch = batch;
  return gemm64_workspace_bytes(g, num_cu);
}

void core64_reduce(const double* part, int splits, int64_t total, double* out, hipStream_t s) {
  unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(core64_reduce_kernel, dim3(blocks), dim3(256), 0, s, part, splits, total, out);
}

}  // namespace rs
