// FP64 GEMM on the CDNA matrix cores (v_mfma_f64_16x16x4f64, or the four-block
// v_mfma_f64_4x4x4f64 form per configuration).
//
//   C[bt](m, n) = sum_k A[bt](m, k) * B[bt](k, n) * kscale[k]
//
// with arbitrary element strides, so one kernel family serves every dense
// contraction of the path: the charge-weighted Gram U diag(w) U^T, the
// eigensolver's products, the projection V^T U, the core contraction and
// the three mode products that expand the Tucker tensor onto the grid.
//
// Tiling (compile-time configurations): a workgroup of WM x WN wave64s owns
// a BM x BN output tile, each wave FM x FN blocks of 16 x 16 (one MFMA
// accumulator of 4 doubles per lane each).  K is staged through LDS in
// slabs of 16 (double-buffered, the next slab prefetched into registers
// while the current one feeds the MFMAs):
//   big   128 x 128 (4 x 2 waves of 32 x 64) for the grid expansion (M = n^2),
//   rank   96 x 64  (3 x 2 waves of 32 x 32) when M is a Tucker rank <= 96,
//   small  64 x 64  (2 x 2 waves of 32 x 32) for the rest.
// (Measured on gfx950 against 128 x 128 tiles of 64 x 64 per wave, k slabs
// of 32 and the 4x4x4 instruction form: these were the fastest per shape.)
// Large K is split across workgroups; the partial tiles are summed by a
// second kernel in a fixed order, so the result is deterministic.  When
// the M tiles divide among the 8 XCDs, consecutive workgroups of one XCD
// walk the N tiles of one M tile, so the A tile is re-read from that XCD's
// L2 rather than from HBM.
#include "rs_internal.h"
#include <algorithm>

namespace rs {

constexpr int PAD = 2;

// MF selects the matrix instruction: 16 for v_mfma_f64_16x16x4f64 (one
// 16 x 16 x 4 product), 4 for v_mfma_f64_4x4x4f64 (four 4 x 4 x 4 products).
template <int WM_, int WN_, int FM_, int FN_, int BK_, int MF_>
struct Cfg {
  static constexpr int WM = WM_, WN = WN_, FM = FM_, FN = FN_, BK = BK_, MF = MF_;
  static constexpr int BM = WM * FM * 16, BN = WN * FN * 16;
  static constexpr int NT = 64 * WM * WN;
  static constexpr int LDA = BM + PAD, LDB = BN + PAD;
  static constexpr int VA = (BM * BK + NT - 1) / NT, VB = (BN * BK + NT - 1) / NT;   // slab values per thread
};
using CfgBig = Cfg<4, 2, 2, 4, 16, 16>;   // 128 x 128, 8 waves of 32 x 64
using CfgRank = Cfg<3, 2, 2, 2, 16, 16>;  //  96 x 64,  6 waves of 32 x 32
using CfgSmall = Cfg<2, 2, 2, 2, 16, 16>; //  64 x 64,  4 waves of 32 x 32
constexpr int KALIGN = 32;                // split-K chunks are multiples of every slab depth

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
  int64_t ccb, sccb;  // column blocks of the output (ccb = 0: none)
  int tiles_m, tiles_n;
  int xcd_remap;       // tile order grouped by XCD (tiles_m % 8 == 0, one batch, no split)
  int bm, bn;          // tile shape (for the reduction's mirror test)
};

// Slab element e (0 <= e < WIDE * BK) of a thread's share: element index
// e = tid + NT r.  With the wide index contiguous in memory, consecutive
// threads take consecutive wide indices; with k contiguous, consecutive k.
template <bool WIDE_CONTIG, int WIDE, int BK>
__device__ __forceinline__ void slab_coord(int e, int& wl, int& kl) {
  if (WIDE_CONTIG) {
    wl = e % WIDE;
    kl = e / WIDE;
  } else {
    kl = e % BK;
    wl = e / BK;
  }
}

// Operand sources.  Each loads its share (V values per thread) of a
// BK x WIDE slab into registers; `store` writes them to LDS as [k][wide].
template <bool WIDE_CONTIG, int WIDE, int NT, int BK>
struct StridedSrc {
  static constexpr int V = (WIDE * BK + NT - 1) / NT;
  const double* P;
  int64_t s_wide, s_k, W;
  const double* kscale;
  __device__ __forceinline__ void load(int64_t wide0, int64_t k0, int64_t kend, double (&reg)[V],
                                       int tid) const {
#pragma unroll
    for (int r = 0; r < V; ++r) {
      const int e = tid + NT * r;
      int wl, kl;
      slab_coord<WIDE_CONTIG, WIDE, BK>(e, wl, kl);
      const int64_t w = wide0 + wl, k = k0 + kl;
      double v = 0.0;
      if (e < WIDE * BK && w < W && k < kend) {
        v = P[w * s_wide + k * s_k];
        if (kscale) v *= kscale[k];
      }
      reg[r] = v;
    }
  }
  __device__ __forceinline__ void store(double* lds, int ld, const double (&reg)[V], int tid) const {
#pragma unroll
    for (int r = 0; r < V; ++r) {
      const int e = tid + NT * r;
      int wl, kl;
      slab_coord<WIDE_CONTIG, WIDE, BK>(e, wl, kl);
      if (e < WIDE * BK) lds[kl * ld + wl] = reg[r];
    }
  }
};

// Khatri-Rao operand of the core contraction, generated on the fly:
// B[j, b*r3 + c] = xi_j * U2t[j*r2 + b] * U3t[j*r3 + c]  (never stored).
template <int WIDE, int NT, int BK>
struct KhatriRaoSrc {
  static constexpr int V = (WIDE * BK + NT - 1) / NT;
  const double* s2;   // xi_k U~2[k, b], [K][r2]
  const double* U3t;  // U~3[k, c], [K][r3]
  int r2, r3;
  // per-thread slab coordinates, fixed over k: set once by init()
  int kl_[V];
  int64_t o2_[V], o3_[V];
  bool ok_[V];
  __device__ __forceinline__ void init(int64_t n0, int tid) {
    const int W = r2 * r3;
#pragma unroll
    for (int r = 0; r < V; ++r) {
      const int e = tid + NT * r;
      int wl, kl;
      slab_coord<true, WIDE, BK>(e, wl, kl);
      const int bc = (int)n0 + wl;
      ok_[r] = e < WIDE * BK && bc < W;
      const int b = ok_[r] ? bc / r3 : 0, c = ok_[r] ? bc - b * r3 : 0;
      kl_[r] = kl;
      o2_[r] = (int64_t)kl * r2 + b;
      o3_[r] = (int64_t)kl * r3 + c;
    }
  }
  __device__ __forceinline__ void load(int64_t n0, int64_t k0, int64_t kend, double (&reg)[V],
                                       int tid) const {
    (void)n0;
    (void)tid;
    const double* p2 = s2 + k0 * r2;
    const double* p3 = U3t + k0 * r3;
#pragma unroll
    for (int r = 0; r < V; ++r) reg[r] = (ok_[r] && k0 + kl_[r] < kend) ? p2[o2_[r]] * p3[o3_[r]] : 0.0;
  }
  __device__ __forceinline__ void store(double* lds, int ld, const double (&reg)[V], int tid) const {
#pragma unroll
    for (int r = 0; r < V; ++r) {
      const int e = tid + NT * r;
      int wl, kl;
      slab_coord<true, WIDE, BK>(e, wl, kl);
      if (e < WIDE * BK) lds[kl * ld + wl] = reg[r];
    }
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

template <int WIDE, int NT, int BK>
struct HashSrc {
  static constexpr int V = (WIDE * BK + NT - 1) / NT;
  const double* scale;
  uint64_t seed;
  int64_t W;
  __device__ __forceinline__ void load(int64_t n0, int64_t k0, int64_t kend, double (&reg)[V],
                                       int tid) const {
#pragma unroll
    for (int r = 0; r < V; ++r) {
      const int e = tid + NT * r;
      int wl, kl;
      slab_coord<true, WIDE, BK>(e, wl, kl);
      const int64_t c = n0 + wl, k = k0 + kl;
      double v = 0.0;
      if (e < WIDE * BK && c < W && k < kend) {
        const uint64_t h = mix64(seed ^ mix64((uint64_t)k * 0x100000001B3ULL + (uint64_t)c));
        v = (scale ? scale[k] : 1.0) * ((double)(h >> 11) * (2.0 / 9007199254740992.0) - 1.0);
      }
      reg[r] = v;
    }
  }
  __device__ __forceinline__ void store(double* lds, int ld, const double (&reg)[V], int tid) const {
#pragma unroll
    for (int r = 0; r < V; ++r) {
      const int e = tid + NT * r;
      int wl, kl;
      slab_coord<true, WIDE, BK>(e, wl, kl);
      if (e < WIDE * BK) lds[kl * ld + wl] = reg[r];
    }
  }
};

struct TileOut {
  int64_t M, N;
  double* C; int64_t scm, scn;
  int64_t ccb = 0, sccb = 0;
  double* part;   // split-K partial base for this (bt, split), row-major M x N, or null
  int nontemporal;
};

// One BM x BN output tile over k in [kbeg, kend).
template <class CF, class ASrc, class BSrc>
__device__ __forceinline__ void mfma_tile(const ASrc& as_src, const BSrc& bs_src, int64_t m0,
                                          int64_t n0, int64_t kbeg, int64_t kend,
                                          const TileOut& o) {
  constexpr int FM = CF::FM, FN = CF::FN, LDA = CF::LDA, LDB = CF::LDB, BK = CF::BK;
  __shared__ double As[2][BK * LDA];
  __shared__ double Bs[2][BK * LDB];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / CF::WN, wn = wave - (wave / CF::WN) * CF::WN;

  // MF == 4: acc[i][j][t] is rows 4t..4t+3 of 16 x 16 block (i, j);
  // MF == 16: acc[i][j][v] is row v of each 4-row group of block (i, j)
  typedef double d4 __attribute__((ext_vector_type(4)));
  d4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  double ra[CF::VA], rb[CF::VB];
  int buf = 0;
  if (kbeg < kend) {
    as_src.load(m0, kbeg, kend, ra, tid);
    bs_src.load(n0, kbeg, kend, rb, tid);
    as_src.store(As[0], LDA, ra, tid);
    bs_src.store(Bs[0], LDB, rb, tid);
  }
  __syncthreads();

  // v_mfma_f64_16x16x4f64: lane holds A[lane % 16][lane / 16], B[lane / 16][lane % 16]
  // and D[lane / 16 + 4 v][lane % 16].
  // v_mfma_f64_4x4x4f64 runs 4 independent 4x4x4 products, one per lane
  // block blk = (lane >> 2) & 3: lane holds A[lane & 3][lane >> 4],
  // B[lane >> 4][lane & 3] and D[lane >> 4][lane & 3] of its block.  With
  // A rows 4t..4t+3 shared by the 4 blocks and B columns 4 blk..4 blk+3,
  // instruction t yields rows 4t..4t+3 of a 16 x 16 x 4 block product; the
  // B operand is then B[lane >> 4][lane & 15] for all t.
  for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) {
      as_src.load(m0, k0 + BK, kend, ra, tid);
      bs_src.load(n0, k0 + BK, kend, rb, tid);
    }
    const double* as = As[buf] + wm * (FM * 16) + (CF::MF == 4 ? (lane & 3) : (lane & 15));
    const double* bs = Bs[buf] + wn * (FN * 16) + (lane & 15);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      double fb[FN];
#pragma unroll
      for (int j = 0; j < FN; ++j) fb[j] = bs[kr * LDB + j * 16];
      if constexpr (CF::MF == 4) {
#pragma unroll
        for (int i = 0; i < FM; ++i) {
          double fa[4];
#pragma unroll
          for (int t = 0; t < 4; ++t) fa[t] = as[kr * LDA + i * 16 + 4 * t];
#pragma unroll
          for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int t = 0; t < 4; ++t)
              acc[i][j][t] = __builtin_amdgcn_mfma_f64_4x4x4f64(fa[t], fb[j], acc[i][j][t], 0, 0, 0);
        }
      } else {
        double fa[FM];
#pragma unroll
        for (int i = 0; i < FM; ++i) fa[i] = as[kr * LDA + i * 16];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i], fb[j], acc[i][j], 0, 0, 0);
      }
    }
    if (more) {
      as_src.store(As[buf ^ 1], LDA, ra, tid);
      bs_src.store(Bs[buf ^ 1], LDB, rb, tid);
    }
    __syncthreads();
    buf ^= 1;
  }

  // epilogue (both forms): acc[i][j][v] at lane l is C[16 i + l / 16 + 4 v][16 j + l % 16]
#pragma unroll
  for (int i = 0; i < FM; ++i) {
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int64_t col = n0 + wn * (FN * 16) + j * 16 + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = (lane >> 4) + 4 * v;
        const int64_t row = m0 + wm * (FM * 16) + i * 16 + r;
        if (row < o.M && col < o.N) {
          const double val = acc[i][j][v];
          if (o.part) {
            o.part[row * o.N + col] = val;
          } else {
            const int64_t coff = o.ccb ? (col / o.ccb) * o.sccb + (col % o.ccb) * o.scn : col * o.scn;
            double* dst = o.C + row * o.scm + coff;
            if (o.nontemporal) __builtin_nontemporal_store(val, dst);
            else *dst = val;
          }
        }
      }
    }
  }
}

__device__ __forceinline__ void tile_coords(const GemmDev& g, int& tm, int& tn) {
  const int t = blockIdx.x;
  if (g.xcd_remap) {
    // workgroup t runs on XCD t % 8; its i-th workgroup there takes the
    // N tiles of M tile (i / tiles_n) * 8 + t % 8 in order
    const int x = t & 7, i = t >> 3;
    tm = (i / g.tiles_n) * 8 + x;
    tn = i - (i / g.tiles_n) * g.tiles_n;
  } else {
    tm = t / g.tiles_n;
    tn = t - tm * g.tiles_n;
  }
}

template <class CF, bool A_MC, bool B_NC>
__global__ __launch_bounds__(CF::NT) void gemm_kernel(GemmDev g) {
  int tm, tn;
  tile_coords(g, tm, tn);
  if (g.upper_only && tm > tn) return;
  const int bt = blockIdx.y;
  const int split = blockIdx.z;
  const int64_t kbeg = (int64_t)split * g.kchunk;
  int64_t kend = kbeg + g.kchunk;
  if (kend > g.K) kend = g.K;
  StridedSrc<A_MC, CF::BM, CF::NT, CF::BK> as{g.A + (int64_t)bt * g.sab, g.sam, g.sak, g.M, nullptr};
  StridedSrc<B_NC, CF::BN, CF::NT, CF::BK> bs{g.B + (int64_t)bt * g.sbb, g.sbn, g.sbk, g.N, g.kscale};
  TileOut o;
  o.M = g.M;
  o.N = g.N;
  o.C = g.C + (int64_t)bt * g.scb;
  o.scm = g.scm;
  o.scn = g.scn;
  o.ccb = g.ccb;
  o.sccb = g.sccb;
  o.part = g.part ? g.part + ((int64_t)bt * g.splits + split) * g.M * g.N : nullptr;
  o.nontemporal = g.nontemporal;
  mfma_tile<CF>(as, bs, (int64_t)tm * CF::BM, (int64_t)tn * CF::BN, kbeg, kend, o);
}

// Y[bt] (M x N, col-major) = A[bt] (M x K, m-contiguous) * Omega_bt (K x N, hashed)
template <class CF>
__global__ __launch_bounds__(CF::NT) void sketch_kernel(GemmDev g, uint64_t seed) {
  int tm, tn;
  tile_coords(g, tm, tn);
  const int bt = blockIdx.y;
  const int split = blockIdx.z;
  const int64_t kbeg = (int64_t)split * g.kchunk;
  int64_t kend = kbeg + g.kchunk;
  if (kend > g.K) kend = g.K;
  StridedSrc<true, CF::BM, CF::NT, CF::BK> as{g.A + (int64_t)bt * g.sab, 1, g.sak, g.M, nullptr};
  HashSrc<CF::BN, CF::NT, CF::BK> bs{g.kscale + (int64_t)bt * g.sbb, seed + 0x51ED27ULL * (uint64_t)(bt + 1), g.N};
  TileOut o;
  o.M = g.M;
  o.N = g.N;
  o.C = g.C + (int64_t)bt * g.scb;
  o.scm = g.scm;
  o.scn = g.scn;
  o.part = g.part ? g.part + ((int64_t)bt * g.splits + split) * g.M * g.N : nullptr;
  o.nontemporal = 0;
  mfma_tile<CF>(as, bs, (int64_t)tm * CF::BM, (int64_t)tn * CF::BN, kbeg, kend, o);
}

struct CoreDev {
  const double* U1t;
  const double* s2;    // xi_k U~2[k, b], [K][r2]
  const double* U3t;
  int r1, r2, r3;
  int64_t K;
  double* beta;
  double* part;
  int splits;
  int64_t kchunk;
  int tiles_n;
};

// beta_(1) (r1 x r2 r3) = U1t^T diag(xi) (U3t (.) U2t): the core of the
// RHOSVD, eq CP_form_RHOSVD, as one GEMM whose right operand is the
// Khatri-Rao product formed while staging it in LDS (from xi U~2, scaled
// once beforehand, and U~3).
template <class CF>
__global__ __launch_bounds__(CF::NT) void core_kernel(CoreDev g) {
  const int tile = blockIdx.x;
  const int tm = tile / g.tiles_n, tn = tile - tm * g.tiles_n;
  const int split = blockIdx.z;
  const int64_t kbeg = (int64_t)split * g.kchunk;
  int64_t kend = kbeg + g.kchunk;
  if (kend > g.K) kend = g.K;
  const int64_t W = (int64_t)g.r2 * g.r3;
  StridedSrc<true, CF::BM, CF::NT, CF::BK> as{g.U1t, 1, g.r1, g.r1, nullptr};
  KhatriRaoSrc<CF::BN, CF::NT, CF::BK> bs{g.s2, g.U3t, g.r2, g.r3, {}, {}, {}, {}};
  bs.init((int64_t)tn * CF::BN, threadIdx.x);
  TileOut o;
  o.M = g.r1;
  o.N = W;
  o.C = g.beta;
  o.scm = W;
  o.scn = 1;
  o.part = g.part ? g.part + (int64_t)split * g.r1 * W : nullptr;
  o.nontemporal = 0;
  mfma_tile<CF>(as, bs, (int64_t)tm * CF::BM, (int64_t)tn * CF::BN, kbeg, kend, o);
}

// s2[k r2 + b] = xi_k U~2[k, b]
__global__ void scale_rows_kernel(const double* __restrict__ xi, const double* __restrict__ U2t,
                                  int64_t K, int r2, double* __restrict__ s2) {
  const int64_t total = K * r2;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x)
    s2[e] = xi[e / r2] * U2t[e];
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
    if (g.upper_only && (row / g.bm) > (col / g.bn)) {
      sr = col;
      sc = row;
    }
    double s = 0.0;
    for (int sp = 0; sp < g.splits; ++sp)
      s += g.part[(((int64_t)bt * g.splits + sp) * g.M + sr) * g.N + sc];
    const int64_t coff = g.ccb ? (col / g.ccb) * g.sccb + (col % g.ccb) * g.scn : col * g.scn;
    double* dst = g.C + (int64_t)bt * g.scb + row * g.scm + coff;
    *dst = s;
  }
}

// ---- grid expansion, streaming form ------------------------------------------
// C[m, col] = sum_k A[m, k] B[col, k]: A = T2 (M = n^2 rows of K = r3, k
// contiguous), B = V3 (n rows of K), C the grid (M x N, non-temporal
// stores).  Persistent workgroups of 16 waves: workgroup (panel, group) keeps
// the B rows of a panel of BN columns in LDS as [k][col] (zero-padded to kp,
// a multiple of 32) for its whole life, and each wave walks 16-row tiles of
// its group with the A values loaded straight from global memory into the
// MFMA operand.  Within each 32-k chunk, lane (r, q) = (lane % 16, lane / 16)
// holds A[r][32 c + 4 s + q] for s = 0..7, so that MFMA step s contracts
// k = 32 c + 4 s + q, q = 0..3, and each load instruction reads one
// contiguous 32-byte piece of each of the 16 rows.  The loop has no barrier; the
// next chunk's A values are loaded while the current one is multiplied.  The
// panels of one row group run on one XCD (workgroup w runs on XCD w % 8),
// so the T2 rows they share come from that XCD's L2.
template <int BN, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void grid64_stream_kernel(const double* __restrict__ A,
                                                            const double* __restrict__ B,
                                                            int64_t M, int N, int K, int kp,
                                                            int npanels, int groups,
                                                            double* __restrict__ C) {
  constexpr int FN = BN / 16, LDB = BN + 2;
  extern __shared__ double bsm[];   // [kp][LDB]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int w = blockIdx.x;
  const int xcd = w & 7, iw = w >> 3;
  const int panel = iw % npanels;
  const int g = (iw / npanels) * 8 + xcd;
  const int n0 = panel * BN;
  for (int e = threadIdx.x; e < kp * BN; e += 64 * WAVES) {
    const int col = e / kp, k = e - col * kp;
    bsm[k * LDB + col] = (n0 + col < N && k < K) ? B[(int64_t)(n0 + col) * K + k] : 0.0;
  }
  __syncthreads();
  if (g >= groups) return;   // uniform over the workgroup, after the only barrier
  const int64_t tiles = (M + 15) / 16;
  const int r = lane & 15, q = lane >> 4;
  const int nch = kp / 32;
  const double* bl = bsm + r;
  typedef double d4 __attribute__((ext_vector_type(4)));
  auto tile_of = [&](int64_t it) { return (it * groups + g) * WAVES + wave; };
  auto load = [&](int64_t tile, int c, double (&a)[8]) {
    const int64_t row = tile * 16 + r;
    const int k0 = 32 * c + q;
    const double* src = A + row * K + k0;
    const bool rok = tile < tiles && row < M;
#pragma unroll
    for (int s = 0; s < 8; ++s) a[s] = (rok && k0 + 4 * s < K) ? src[4 * s] : 0.0;
  };
  int64_t it = 0;
  int64_t tile = tile_of(0);
  if (tile >= tiles) return;
  double a[8];
  load(tile, 0, a);
  for (; tile < tiles; tile = tile_of(++it)) {
    d4 acc[FN];
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[j] = d4{0.0, 0.0, 0.0, 0.0};
    for (int c = 0; c < nch; ++c) {
      double an[8];
      if (c + 1 < nch) load(tile, c + 1, an);
      else load(tile_of(it + 1), 0, an);
      // steps whose four k are all >= K contribute nothing: skipped (uniform)
      const int smax = (K - 32 * c + 3) / 4;
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        if (s < smax) {
          const double* brow = bl + (32 * c + 4 * s + q) * LDB;
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], brow[j * 16], acc[j], 0, 0, 0);
        }
      }
#pragma unroll
      for (int s = 0; s < 8; ++s) a[s] = an[s];
    }
    // acc[j][v] is C[16 tile + q + 4 v][n0 + 16 j + r]
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int col = n0 + 16 * j + r;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = tile * 16 + q + 4 * v;
        if (row < M && col < N) __builtin_nontemporal_store(acc[j][v], C + row * N + col);
      }
    }
  }
}

constexpr int GRID_WAVES = 16;   // waves per workgroup, all sharing the panel

template <int BN>
static void launch_grid64_stream(const double* T2, const double* V3, int64_t M, int N, int K,
                                 int kp, double* C, int num_cu, hipStream_t s) {
  const int npanels = (N + BN - 1) / BN;
  const int64_t tiles = (M + 15) / 16;
  int gq = std::max(1, num_cu / (8 * npanels));
  while (gq > 1 && (int64_t)gq * 8 * GRID_WAVES > tiles) --gq;
  const int groups = gq * 8;
  const size_t lds = (size_t)kp * (BN + 2) * sizeof(double);
  auto fn = grid64_stream_kernel<BN, GRID_WAVES>;
  if (lds > 48 * 1024)
    RS_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(fn, dim3((unsigned)(8 * npanels * gq)), dim3(64 * GRID_WAVES), lds, s, T2, V3,
                     M, N, K, kp, npanels, groups, C);
}

bool grid64_stream(const double* T2, const double* V3, int64_t n, int r3, double* grid, int num_cu,
                   int lds_limit, hipStream_t s) {
  if (n <= 0 || r3 <= 0) return true;
  const int kp = (r3 + 31) / 32 * 32;
  // the panel opts in beyond the default 64 KB of dynamic LDS (gfx950 has 160 KB per CU)
  (void)lds_limit;
  const size_t budget = 150 * 1024;
  auto need = [&](int bn) { return (size_t)kp * (bn + 2) * sizeof(double); };
  const int64_t M = n * n;
  if (need(128) <= budget) launch_grid64_stream<128>(T2, V3, M, (int)n, r3, kp, grid, num_cu, s);
  else if (need(64) <= budget) launch_grid64_stream<64>(T2, V3, M, (int)n, r3, kp, grid, num_cu, s);
  else if (need(32) <= budget) launch_grid64_stream<32>(T2, V3, M, (int)n, r3, kp, grid, num_cu, s);
  else return false;   // rank too large for an LDS panel: the caller takes the tiled GEMM
  return true;
}

// ---- host: configuration choice and split-K plan -----------------------------
enum CfgId { CFG_SMALL = 0, CFG_RANK = 1, CFG_BIG = 2 };

static void cfg_shape(CfgId c, int& bm, int& bn) {
  if (c == CFG_BIG) { bm = CfgBig::BM; bn = CfgBig::BN; }
  else if (c == CFG_RANK) { bm = CfgRank::BM; bn = CfgRank::BN; }
  else { bm = CfgSmall::BM; bn = CfgSmall::BN; }
}

// Tucker-rank-sized M (65..96) takes the 96-row tile, a very tall product
// (the grid expansion) the big tile, everything else (and every upper-only
// product, whose tiles must be square) the small tile.  The big tile measured
// slower on the charge-weighted Gram (both operands transposed).
static CfgId choose(const Gemm64& g, int num_cu) {
  if (g.upper_only) return CFG_SMALL;
  if (g.M > 64 && g.M <= 96) return CFG_RANK;
  // the big tile only when it alone fills the chip (no split-K and its reduction)
  const int64_t big_tiles = ((g.M + CfgBig::BM - 1) / CfgBig::BM) * ((g.N + CfgBig::BN - 1) / CfgBig::BN) * g.batch;
  if (g.M >= 8192 && g.N >= 128 && big_tiles >= num_cu) return CFG_BIG;
  return CFG_SMALL;
}

struct Plan64 {
  CfgId cfg;
  int bm, bn, tm, tn, splits;
  int64_t kchunk;
};

static Plan64 plan_for(const Gemm64& g, CfgId cfg, int num_cu) {
  Plan64 P;
  P.cfg = cfg;
  cfg_shape(P.cfg, P.bm, P.bn);
  P.tm = (int)((g.M + P.bm - 1) / P.bm);
  P.tn = (int)((g.N + P.bn - 1) / P.bn);
  int64_t tiles = (int64_t)P.tm * P.tn;
  if (g.upper_only) tiles = (int64_t)P.tm * (P.tm + 1) / 2;
  tiles *= g.batch;
  const int64_t target = 2LL * num_cu;
  P.splits = 1;
  if (tiles < target && g.K > 2 * KALIGN) {
    int64_t want = (target + tiles - 1) / tiles;
    // at least 2 KALIGN k per split for the symmetric products and small
    // outputs; at least 128 for large outputs, whose reduction pass (a full
    // read and write of the output per split) outweighs the shorter k loop
    const bool small_out = g.M * g.N * g.batch <= ((int64_t)1 << 17);
    int64_t maxs = (g.upper_only || small_out) ? g.K / (2 * KALIGN) : g.K / 128;
    // a small symmetric output (p x p Rayleigh-Ritz or Cholesky QR Grams): at
    // most ~2^20 partial values, which the fixed-order reduction reads back
    const int64_t cap = g.upper_only
        ? std::max<int64_t>(4, ((int64_t)1 << 20) / std::max<int64_t>(1, g.M * g.N * g.batch))
        : (int64_t)64;
    P.splits = (int)std::max<int64_t>(1, std::min<int64_t>({want, maxs, cap, (int64_t)64}));
  }
  P.kchunk = (g.K + P.splits - 1) / P.splits;
  P.kchunk = (P.kchunk + KALIGN - 1) / KALIGN * KALIGN;
  P.splits = (int)((g.K + P.kchunk - 1) / P.kchunk);
  if (P.splits < 1) P.splits = 1;
  return P;
}

// A product whose N is a Tucker rank (65..96) and whose M is larger is
// computed transposed, C^T = B^T A^T, so that the rank sits on the 96-row side.
static Gemm64 canon(const Gemm64& g) {
  if (g.upper_only || g.ccb || !(g.N > 64 && g.N <= 96 && g.M > 96)) return g;
  Gemm64 t = g;
  t.M = g.N; t.N = g.M;
  t.A = g.B; t.sam = g.sbn; t.sak = g.sbk; t.sab = g.sbb;
  t.B = g.A; t.sbk = g.sak; t.sbn = g.sam; t.sbb = g.sab;
  t.scm = g.scn; t.scn = g.scm;
  return t;
}

size_t gemm64_workspace_bytes(const Gemm64& gin, int num_cu) {
  const Gemm64 g = canon(gin);
  const Plan64 P = plan_for(g, choose(g, num_cu), num_cu);
  if (P.splits == 1 && !g.upper_only) return 0;
  return (size_t)g.batch * P.splits * g.M * g.N * sizeof(double);
}

template <class CF>
static void launch_gemm_cfg(const GemmDev& d, dim3 grid, bool amc, bool bnc, hipStream_t s) {
  if (amc && bnc) hipLaunchKernelGGL((gemm_kernel<CF, true, true>), grid, dim3(CF::NT), 0, s, d);
  else if (amc && !bnc) hipLaunchKernelGGL((gemm_kernel<CF, true, false>), grid, dim3(CF::NT), 0, s, d);
  else if (!amc && bnc) hipLaunchKernelGGL((gemm_kernel<CF, false, true>), grid, dim3(CF::NT), 0, s, d);
  else hipLaunchKernelGGL((gemm_kernel<CF, false, false>), grid, dim3(CF::NT), 0, s, d);
}

void gemm64(const Gemm64& gin, int num_cu, double* work, hipStream_t s) {
  if (gin.M <= 0 || gin.N <= 0 || gin.batch <= 0) return;
  if (gin.K <= 0) throw Error{RS_E_INVALID, "gemm64: K must be positive"};
  const Gemm64 g = canon(gin);
  const Plan64 P = plan_for(g, choose(g, num_cu), num_cu);
  GemmDev d;
  d.M = g.M; d.N = g.N; d.K = g.K;
  d.A = g.A; d.sam = g.sam; d.sak = g.sak; d.sab = g.sab;
  d.B = g.B; d.sbk = g.sbk; d.sbn = g.sbn; d.sbb = g.sbb;
  d.C = g.C; d.scm = g.scm; d.scn = g.scn; d.scb = g.scb;
  d.kscale = g.kscale;
  d.upper_only = g.upper_only;
  d.nontemporal = g.nontemporal;
  d.ccb = g.ccb;
  d.sccb = g.sccb;
  d.splits = P.splits;
  d.kchunk = P.kchunk;
  d.tiles_m = P.tm;
  d.tiles_n = P.tn;
  d.bm = P.bm;
  d.bn = P.bn;
  d.xcd_remap = (g.batch == 1 && P.splits == 1 && !g.upper_only && P.tm % 8 == 0 && P.tn > 1) ? 1 : 0;
  const bool use_part = d.splits > 1 || g.upper_only;
  d.part = use_part ? work : nullptr;
  if (use_part && !work) throw Error{RS_E_DEVICE, "gemm64: missing split-K workspace"};
  const bool amc = (g.sam == 1), akc = (g.sak == 1);
  const bool bnc = (g.sbn == 1), bkc = (g.sbk == 1);
  if (!(amc || akc) || !(bnc || bkc)) throw Error{RS_E_DEVICE, "gemm64: unsupported operand strides"};
  dim3 grid((unsigned)(d.tiles_m * d.tiles_n), (unsigned)g.batch, (unsigned)d.splits);
  if (P.cfg == CFG_BIG) launch_gemm_cfg<CfgBig>(d, grid, amc, bnc, s);
  else if (P.cfg == CFG_RANK) launch_gemm_cfg<CfgRank>(d, grid, amc, bnc, s);
  else launch_gemm_cfg<CfgSmall>(d, grid, amc, bnc, s);
  if (use_part) {
    int64_t total = g.M * g.N;
    int64_t blocks = std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(gemm64_reduce_kernel, dim3((unsigned)blocks, (unsigned)g.batch), dim3(256),
                       0, s, d);
  }
}

// core: the rank tile when 64 < r1 <= 96 (a 96 x 128 tile measured slower), else the small tile
static void plan_core(int r1, int r2, int r3, int64_t K, int num_cu, bool& rank_tile, int& splits,
                      int64_t& kchunk, int& tm, int& tn) {
  rank_tile = r1 > 64 && r1 <= 96;
  const int bm = rank_tile ? CfgRank::BM : CfgSmall::BM;
  const int bn = rank_tile ? CfgRank::BN : CfgSmall::BN;
  tm = (r1 + bm - 1) / bm;
  tn = (int)(((int64_t)r2 * r3 + bn - 1) / bn);
  int64_t tiles = (int64_t)tm * tn;
  const int64_t target = 2LL * num_cu;
  splits = 1;
  if (tiles < target && K > 8 * KALIGN) {
    int64_t want = (target + tiles - 1) / tiles;
    splits = (int)std::min<int64_t>(want, std::min<int64_t>(K / (8 * KALIGN), 64));
    if (splits < 1) splits = 1;
  }
  kchunk = (K + splits - 1) / splits;
  kchunk = (kchunk + KALIGN - 1) / KALIGN * KALIGN;
  splits = (int)((K + kchunk - 1) / kchunk);
}

// ---- core, streaming form (r1 <= 128) -------------------------------------------
// beta_(1)[a, col] = sum_k U~1[k, a] s2[k, b] U~3[k, c], col = b r3 + c.  A
// workgroup of 8 waves owns 128 columns (16 per wave) and a k range; it
// stages 128-k chunks of U~1 (all r1 rows, [k][a]) in LDS, and each wave forms
// its Khatri-Rao fragment in registers: lane (r, q) holds B[k0 + 4s + q][col]
// = s2[k][b] U~3[k][c] for its column (the 16 lanes of a k read 16
// consecutive c), loaded four steps ahead.  Step s is RB MFMAs
// against the shared A chunk.
constexpr int CS_KC = 64, CS_NP = 4;

template <int RB>
__global__ __launch_bounds__(512) void core_stream_kernel(const double* __restrict__ U1t,
                                                          const double* __restrict__ s2,
                                                          const double* __restrict__ U3t, int r1,
                                                          int r2, int r3, int64_t K,
                                                          int64_t kchunk, double* __restrict__ out,
                                                          int64_t split_stride, int64_t sb1,
                                                          int64_t sbs, int64_t sb3) {
  constexpr int KC = CS_KC, NP = CS_NP, AR = 16 * RB;
  constexpr int LDA = AR + ((RB & 1) ? 0 : 16);   // row starts 32 banks apart per q
  constexpr int AV = (KC * AR + 511) / 512;
  typedef double d4 __attribute__((ext_vector_type(4)));
  extern __shared__ double As[];   // [KC][LDA]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r = lane & 15, q = lane >> 4;
  const int W = r2 * r3;
  const int col = blockIdx.x * 128 + wave * 16 + r;
  // batch blockIdx.y: its factors at the given strides, its splits after the
  // previous batch's
  U1t += (int64_t)blockIdx.y * sb1;
  s2 += (int64_t)blockIdx.y * sbs;
  U3t += (int64_t)blockIdx.y * sb3;
  const bool colok = col < W;
  const int b = colok ? col / r3 : 0, c = colok ? col - b * r3 : 0;
  const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
  const int64_t kend = kbeg + kchunk < K ? kbeg + kchunk : K;
  double ra[AV];
  auto loadA = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < AV; ++u) {
      const int e = tid + 512 * u;
      const int kk = e / AR, a = e - kk * AR;
      ra[u] = (e < KC * AR && k0 + kk < kend && a < r1) ? U1t[(k0 + kk) * r1 + a] : 0.0;
    }
  };
  auto storeA = [&]() {
#pragma unroll
    for (int u = 0; u < AV; ++u) {
      const int e = tid + 512 * u;
      const int kk = e / AR, a = e - kk * AR;
      if (e < KC * AR) As[kk * LDA + a] = ra[u];
    }
  };
  // raw Khatri-Rao factors of NP consecutive steps (k = k0 + 4 s + q)
  auto loadB = [&](int64_t k0, double (&x2)[NP], double (&x3)[NP]) {
#pragma unroll
    for (int s8 = 0; s8 < NP; ++s8) {
      const int64_t k = k0 + 4 * s8 + q;
      const bool ok = colok && k < kend;
      x2[s8] = ok ? s2[k * r2 + b] : 0.0;
      x3[s8] = ok ? U3t[k * r3 + c] : 0.0;
    }
  };
  d4 acc[RB];
#pragma unroll
  for (int i = 0; i < RB; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};
  if (kbeg < kend) {
    loadA(kbeg);
    storeA();
  }
  __syncthreads();
  double c2[NP], c3[NP];
  loadB(kbeg, c2, c3);
  for (int64_t k0 = kbeg; k0 < kend; k0 += KC) {
    const bool more = k0 + KC < kend;
    if (more) loadA(k0 + KC);
#pragma unroll 2
    for (int g = 0; g < KC / (4 * NP); ++g) {
      // the next NP steps are fetched NP steps ahead, across chunk ends
      double n2[NP], n3[NP];
      loadB(k0 + 4 * NP * (g + 1), n2, n3);
#pragma unroll
      for (int s8 = 0; s8 < NP; ++s8) {
        const double bv = c2[s8] * c3[s8];
        const double* arow = As + (4 * NP * g + 4 * s8 + q) * LDA + r;
#pragma unroll
        for (int i = 0; i < RB; ++i)
          acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(arow[16 * i], bv, acc[i], 0, 0, 0);
      }
#pragma unroll
      for (int s8 = 0; s8 < NP; ++s8) {
        c2[s8] = n2[s8];
        c3[s8] = n3[s8];
      }
    }
    __syncthreads();
    if (more) {
      storeA();
      __syncthreads();
    }
  }
  // acc[i][v] is beta_(1)[16 i + q + 4 v][col]
  double* o = out + ((int64_t)blockIdx.y * gridDim.z + blockIdx.z) * split_stride;
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int a = 16 * i + q + 4 * v;
      if (a < r1 && colok) o[(int64_t)a * W + col] = acc[i][v];
    }
}

static int core_stream_rb(int r1) { return r1 <= 32 ? 2 : r1 <= 64 ? 4 : r1 <= 96 ? 6 : 8; }

static void plan_core_stream(int r1, int r2, int r3, int64_t K, int num_cu, int& splits,
                             int64_t& kchunk) {
  const int64_t groups = ((int64_t)r2 * r3 + 127) / 128;
  // one 8-wave workgroup per CU: fill the chip once without a ragged second wave
  splits = (int)std::max<int64_t>(1, std::min<int64_t>(num_cu / groups, (K + CS_KC - 1) / CS_KC));
  splits = std::min(splits, 32);
  kchunk = (K + splits - 1) / splits;
  kchunk = (kchunk + CS_KC - 1) / CS_KC * CS_KC;
  splits = (int)((K + kchunk - 1) / kchunk);
}

// workspace: xi U~2 (K x r2), then the split-K partials
static size_t core64_s2_bytes(int r2, int64_t K) { return ((size_t)K * r2 * sizeof(double) + 255) & ~(size_t)255; }

size_t core64_workspace_bytes(int r1, int r2, int r3, int64_t K, int num_cu) {
  bool rt;
  int splits, tm, tn;
  int64_t kchunk;
  if (r1 <= 128) plan_core_stream(r1, r2, r3, K, num_cu, splits, kchunk);
  else plan_core(r1, r2, r3, K, num_cu, rt, splits, kchunk, tm, tn);
  return core64_s2_bytes(r2, K) + (splits > 1 ? (size_t)splits * r1 * r2 * r3 * sizeof(double) : 0);
}

void core64(const double* U1t, const double* U2t, const double* U3t, const double* xi, int r1,
            int r2, int r3, int64_t K, double* beta, int num_cu, double* work, hipStream_t s,
            const KernelTimer* kt) {
  CoreDev d;
  bool rank_tile;
  int tm;
  plan_core(r1, r2, r3, K, num_cu, rank_tile, d.splits, d.kchunk, tm, d.tiles_n);
  if (!work) throw Error{RS_E_DEVICE, "core64: missing workspace"};
  double* s2 = work;
  double* part = (double*)((char*)work + core64_s2_bytes(r2, K));
  {
    const int64_t total = K * r2;
    const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(scale_rows_kernel, dim3(blocks), dim3(256), 0, s, xi, U2t, K, r2, s2);
  }
  if (r1 <= 128) {
    int splits;
    int64_t kchunk;
    plan_core_stream(r1, r2, r3, K, num_cu, splits, kchunk);
    double* outp = splits > 1 ? part : beta;
    const int64_t W = (int64_t)r2 * r3;
    const dim3 grid((unsigned)((W + 127) / 128), 1, (unsigned)splits);
    const int rb = core_stream_rb(r1);
    auto launch = [&](auto fn, int RBv) {
      const size_t lds = (size_t)CS_KC * (16 * RBv + ((RBv & 1) ? 0 : 16)) * sizeof(double);
      if (lds > 48 * 1024)
        RS_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds));
      if (kt) RS_HIP(hipEventRecord(kt->begin, s));
      hipLaunchKernelGGL(fn, grid, dim3(512), lds, s, U1t, (const double*)s2, U3t, r1, r2, r3, K,
                         kchunk, outp, (int64_t)r1 * W, (int64_t)0, (int64_t)0, (int64_t)0);
      if (kt) RS_HIP(hipEventRecord(kt->end, s));
    };
    if (rb == 2) launch(core_stream_kernel<2>, 2);
    else if (rb == 4) launch(core_stream_kernel<4>, 4);
    else if (rb == 6) launch(core_stream_kernel<6>, 6);
    else launch(core_stream_kernel<8>, 8);
    if (splits > 1) {
      const int64_t total = (int64_t)r1 * W;
      unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 8192);
      hipLaunchKernelGGL(core64_reduce_kernel, dim3(blocks), dim3(256), 0, s, (const double*)part,
                         splits, total, beta);
    }
    return;
  }
  d.U1t = U1t;
  d.s2 = s2;
  d.U3t = U3t;
  d.r1 = r1;
  d.r2 = r2;
  d.r3 = r3;
  d.K = K;
  d.beta = beta;
  d.part = d.splits > 1 ? part : nullptr;
  dim3 grid((unsigned)(tm * d.tiles_n), 1, (unsigned)d.splits);
  if (kt) RS_HIP(hipEventRecord(kt->begin, s));
  if (rank_tile) hipLaunchKernelGGL(core_kernel<CfgRank>, grid, dim3(CfgRank::NT), 0, s, d);
  else hipLaunchKernelGGL(core_kernel<CfgSmall>, grid, dim3(CfgSmall::NT), 0, s, d);
  if (kt) RS_HIP(hipEventRecord(kt->end, s));
  if (d.splits > 1) {
    int64_t total = (int64_t)r1 * r2 * r3;
    unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(core64_reduce_kernel, dim3(blocks), dim3(256), 0, s, (const double*)part,
                       d.splits, total, beta);
  }
}

// ---- tall Gram, streaming form --------------------------------------------------
// C[b] = Z[b]^T diag(w) Z[b] (p x p, p <= 128) for Z[b] K x p row-major: the
// streaming core with r1 = r3 = p, r2 = 1 (its scaled factor is w itself),
// K split over the workgroups of all batches; the splits are summed in a
// fixed order for the upper triangle, which is written to both triangles
// (C exactly symmetric).
__global__ void gram_sym_reduce_kernel(const double* __restrict__ part, int splits, int p,
                                       int batch, double* __restrict__ C) {
  const int64_t pp = (int64_t)p * p, total = (int64_t)batch * pp;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / pp, rem = e - b * pp;
    const int i = (int)(rem / p), j = (int)(rem - (int64_t)i * p);
    if (j < i) continue;
    const double* src = part + b * splits * pp + rem;
    double v = 0.0;
    for (int z = 0; z < splits; ++z) v += src[z * pp];
    C[b * pp + (int64_t)i * p + j] = v;
    C[b * pp + (int64_t)j * p + i] = v;
  }
}

static void plan_gram_stream(int64_t K, int batch, int num_cu, int& splits, int64_t& kchunk) {
  splits = (int)std::max<int64_t>(1, std::min<int64_t>(num_cu / std::max(1, batch),
                                                        (K + CS_KC - 1) / CS_KC));
  kchunk = (K + splits - 1) / splits;
  kchunk = (kchunk + CS_KC - 1) / CS_KC * CS_KC;
  splits = (int)((K + kchunk - 1) / kchunk);
}

size_t gram_stream_workspace_bytes(int p, int64_t K, int batch, int num_cu) {
  if (p > 128 || p <= 0 || K <= 0) return 0;
  int splits;
  int64_t kchunk;
  plan_gram_stream(K, batch, num_cu, splits, kchunk);
  return (size_t)batch * splits * p * p * sizeof(double);
}

bool gram_stream(const double* Z, int64_t zstride, const double* w, int p, int64_t K, int batch,
                 double* C, int num_cu, double* work, hipStream_t s) {
  if (p > 128 || p <= 0 || K <= 0 || batch <= 0) return false;
  int splits;
  int64_t kchunk;
  plan_gram_stream(K, batch, num_cu, splits, kchunk);
  const dim3 grid((unsigned)((p + 127) / 128), (unsigned)batch, (unsigned)splits);
  auto launch = [&](auto fn, int RBv) {
    const size_t lds = (size_t)CS_KC * (16 * RBv + ((RBv & 1) ? 0 : 16)) * sizeof(double);
    if (lds > 48 * 1024)
      RS_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds));
    hipLaunchKernelGGL(fn, grid, dim3(512), lds, s, Z, w, Z, p, 1, p, K, kchunk, work,
                       (int64_t)p * p, zstride, (int64_t)0, zstride);
  };
  const int rb = core_stream_rb(p);
  if (rb == 2) launch(core_stream_kernel<2>, 2);
  else if (rb == 4) launch(core_stream_kernel<4>, 4);
  else if (rb == 6) launch(core_stream_kernel<6>, 6);
  else launch(core_stream_kernel<8>, 8);
  const int64_t total = (int64_t)batch * p * p;
  const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(gram_sym_reduce_kernel, dim3(blocks), dim3(256), 0, s, (const double*)work,
                     splits, p, batch, C);
  return true;
}


// the sketch takes the big tile when both M and the subspace size N fill it
static CfgId sketch_cfg(int64_t M, int64_t N) { return (M >= 256 && N >= 128) ? CFG_BIG : CFG_SMALL; }

void sketch64(const double* A, int64_t M, int64_t K, int64_t sab, const double* scale,
              int64_t scale_stride, int batch, int64_t N, uint64_t seed, double* Y, int64_t scm,
              int64_t scn, int num_cu, double* work, hipStream_t s) {
  Gemm64 g;
  g.M = M; g.N = N; g.K = K; g.batch = batch;
  GemmDev d;
  d.M = M; d.N = N; d.K = K;
  d.A = A; d.sam = 1; d.sak = M; d.sab = sab;
  d.B = nullptr; d.sbk = 0; d.sbn = 0; d.sbb = scale_stride;
  d.C = Y; d.scm = scm; d.scn = scn; d.scb = M * N;
  d.kscale = scale;
  d.upper_only = 0;
  d.nontemporal = 0;
  d.ccb = 0;
  d.sccb = 0;
  const Plan64 P = plan_for(g, sketch_cfg(M, N), num_cu);
  d.splits = P.splits;
  d.kchunk = P.kchunk;
  d.bm = P.bm;
  d.bn = P.bn;
  d.tiles_m = P.tm;
  d.tiles_n = P.tn;
  d.xcd_remap = 0;
  const bool use_part = d.splits > 1;
  d.part = use_part ? work : nullptr;
  if (use_part && !work) throw Error{RS_E_DEVICE, "sketch64: missing split-K workspace"};
  dim3 grid((unsigned)(d.tiles_m * d.tiles_n), (unsigned)batch, (unsigned)d.splits);
  if (P.cfg == CFG_BIG)
    hipLaunchKernelGGL(sketch_kernel<CfgBig>, grid, dim3(CfgBig::NT), 0, s, d, seed);
  else
    hipLaunchKernelGGL(sketch_kernel<CfgSmall>, grid, dim3(CfgSmall::NT), 0, s, d, seed);
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
  const Plan64 P = plan_for(g, sketch_cfg(M, N), num_cu);
  if (P.splits == 1) return 0;
  return (size_t)g.batch * P.splits * g.M * g.N * sizeof(double);
}

void core64_reduce(const double* part, int splits, int64_t total, double* out, hipStream_t s) {
  unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(core64_reduce_kernel, dim3(blocks), dim3(256), 0, s, part, splits, total, out);
}

}  // namespace rs
