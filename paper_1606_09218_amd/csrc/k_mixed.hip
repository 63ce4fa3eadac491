// Split-precision contractions for the mixed path (core and grid expansion).
//
// Each FP64 operand value x is represented by low-precision terms:
//  FP16: x 2^s = hi + lo 2^-11 (hi, lo FP16), with a power-of-two scale 2^s
//        from the operand's max |x| so that |x 2^s| < 2^14; three products
//        hi*hi, hi*lo, lo*hi.
//  BF16: x = hi + mid + lo (BF16 of the successive residuals, no scale); six
//        products down to the 2^-16 level (hh, hm, mh, hl, lh, mm).
// The products run on v_mfma_f32_16x16x32_{f16,bf16} with FP32 accumulation,
// one accumulator per magnitude level, folded into FP64 registers every
// KCHUNK values of k.
//
// The FP64 operands are split once into planes, [term][row][kp] with the
// contraction index k contiguous and padded with zeros to kp (a multiple of
// 32): an MFMA fragment (8 consecutive k of one row, 16 bytes) is one load.
// The grid expansion streams its A fragments straight from the planes; the
// core stages 32-k slabs of both operands in LDS.  The Khatri-Rao operand of
// the core, xi_j U~2[j,b] U~3[j,c], is never stored: each workgroup forms
// its slab in FP32 from xi U~2 and U~3 (transposed, FP32) and splits it once.
//
// v_mfma_f32_16x16x32_{f16,bf16}: lane l holds A[l % 16][8 (l / 16) + t] and
// B[8 (l / 16) + t][l % 16] (t = 0..7), and D[4 (l / 16) + v][l % 16].
#include "rs_internal.h"

namespace rs {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int KCHUNK = 256;   // FP32 accumulation span before folding into FP64

struct SplitF16 {
  static constexpr int TERMS = 2;
  static constexpr int LEVELS = 2;
  static constexpr bool SCALED = true;
  static constexpr bool PAIRED = false;
  typedef _Float16 T;
  typedef h8 V8;
  // FP64 -> FP16 through FP32 (hi need not be the nearest FP16 value: lo
  // takes the exact residual x - hi)
  __device__ static void split(double x, T* o) {
    const T hi = (T)(float)x;
    o[0] = hi;
    o[1] = (T)(float)((x - (double)hi) * 2048.0);
  }
  __device__ static void split32(float x, T* o) {
    const T hi = (T)x;
    o[0] = hi;
    o[1] = (T)((x - (float)hi) * 2048.0f);
  }
  __device__ static f4 mfma(V8 a, V8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
  // level 0: hi*hi; level 1: hi*lo + lo*hi (weight 2^-11).  Product p is
  // a[PA[p]] b[PB[p]] into level PL[p], in this order within a level.
  static constexpr int NPROD = 3;
  static constexpr int PA[NPROD] = {0, 0, 1}, PB[NPROD] = {0, 1, 0}, PL[NPROD] = {0, 1, 1};
  __device__ static double combine(const f4 (&acc)[LEVELS], int v) {
    return (double)acc[0][v] + (double)acc[1][v] * (1.0 / 2048.0);
  }
};

struct SplitBF16 {
  static constexpr int TERMS = 3;
  static constexpr int LEVELS = 3;
  static constexpr bool SCALED = false;
  static constexpr bool PAIRED = false;
  typedef __bf16 T;
  typedef b8 V8;
  __device__ static void split(double x, T* o) {
    const T hi = (T)(float)x;
    const double r1 = x - (double)(float)hi;
    const T mid = (T)(float)r1;
    const double r2 = r1 - (double)(float)mid;
    o[0] = hi;
    o[1] = mid;
    o[2] = (T)(float)r2;
  }
  __device__ static void split32(float x, T* o) {
    const T hi = (T)x;
    const float r1 = x - (float)hi;
    const T mid = (T)r1;
    o[0] = hi;
    o[1] = mid;
    o[2] = (T)(r1 - (float)mid);
  }
  __device__ static f4 mfma(V8 a, V8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  // level 0: hi*hi; level 1: hi*mid + mid*hi; level 2: hi*lo + lo*hi + mid*mid
  static constexpr int NPROD = 6;
  static constexpr int PA[NPROD] = {0, 0, 1, 0, 2, 1}, PB[NPROD] = {0, 1, 0, 2, 0, 1},
                       PL[NPROD] = {0, 1, 1, 2, 2, 2};
  __device__ static double combine(const f4 (&acc)[LEVELS], int v) {
    return (double)acc[0][v] + (double)acc[1][v] + (double)acc[2][v];
  }
};

typedef _Float16 h2 __attribute__((ext_vector_type(2)));

// The core's FP16 split: x 2^s = hi + lo with lo unscaled, and the three
// products hi*hi, hi*lo, lo*hi summed in one FP32 accumulator (the lo
// products are 2^-11 of the hi product, so they add no rounding beyond the
// accumulator's own).  For the Khatri-Rao operand hi is x rounded toward
// zero, two values per conversion; x - hi is exact in FP32 and lo is it
// rounded to nearest, so the representation error is unbiased.
struct CoreF16 {
  static constexpr int TERMS = 2;
  static constexpr int LEVELS = 1;
  static constexpr bool SCALED = true;
  static constexpr bool PAIRED = true;
  typedef _Float16 T;
  typedef h8 V8;
  __device__ static void split(double x, T* o) {
    const T hi = (T)(float)x;
    o[0] = hi;
    o[1] = (T)(float)(x - (double)hi);
  }
  __device__ static h2 pk(float a, float b) {
    return __builtin_bit_cast(h2, __builtin_amdgcn_cvt_pkrtz(a, b));
  }
  __device__ static void split8(const float (&x)[8], V8& hi, V8& lo) {
    h2 H[4], L[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      H[p] = pk(x[2 * p], x[2 * p + 1]);
      L[p] = h2{(_Float16)(x[2 * p] - (float)H[p][0]), (_Float16)(x[2 * p + 1] - (float)H[p][1])};
    }
    hi = __builtin_shufflevector(__builtin_shufflevector(H[0], H[1], 0, 1, 2, 3),
                                 __builtin_shufflevector(H[2], H[3], 0, 1, 2, 3), 0, 1, 2, 3, 4, 5,
                                 6, 7);
    lo = __builtin_shufflevector(__builtin_shufflevector(L[0], L[1], 0, 1, 2, 3),
                                 __builtin_shufflevector(L[2], L[3], 0, 1, 2, 3), 0, 1, 2, 3, 4, 5,
                                 6, 7);
  }
  __device__ static f4 mfma(V8 a, V8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
  static constexpr int NPROD = 3;
  static constexpr int PA[NPROD] = {0, 0, 1}, PB[NPROD] = {0, 1, 0}, PL[NPROD] = {0, 0, 0};
  __device__ static double combine(const f4 (&acc)[LEVELS], int v) { return (double)acc[0][v]; }
};

static inline int64_t pad32(int64_t k) { return (k + 31) / 32 * 32; }

// 2^s from the exponent table written by scale_exponents_kernel
__device__ __forceinline__ double pow2(int s) { return ldexp(1.0, s); }

// ---- split planes ---------------------------------------------------------------
// out[term][row][k] (k < kp, zero beyond cols) = term of x(row, k) 2^s,
// x(row, k) = src[row * s_row + k * s_col].  Thread (k, row): k = threadIdx.x
// + 256 blockIdx.x, rows strided by gridDim.y.
template <class SP>
__global__ __launch_bounds__(256) void split_planes_kernel(const double* __restrict__ src,
                                                           int64_t rows, int cols, int64_t s_row,
                                                           int64_t s_col, int kp, const int* exps,
                                                           int which,
                                                           typename SP::T* __restrict__ out) {
  const double scale = SP::SCALED && exps ? pow2(exps[which]) : 1.0;
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= kp) return;
  const int64_t plane = rows * kp;
  for (int64_t row = blockIdx.y; row < rows; row += gridDim.y) {
    const double x = k < cols ? src[row * s_row + k * s_col] * scale : 0.0;
    typename SP::T t[SP::TERMS];
    SP::split(x, t);
    const int64_t e = row * kp + k;
#pragma unroll
    for (int term = 0; term < SP::TERMS; ++term) out[term * plane + e] = t[term];
  }
}

// The core's operands from the projected factors in one pass: U~_l^T is
// K x r_l (row j holds the r_l values of term j), the core wants rows of K
// values per rank index.  A workgroup transposes a 64 j x 64 rank tile
// through LDS (reads and writes both along contiguous rows) and writes
//   op 0: the split planes of U~1^T, planes[term][a][j], scaled by 2^exps[0],
//   op 1: s2[b][j] = 2^exps[1] xi_j U~2[j, b] (FP32),
//   op 2: u3[c][j] = U~3[j, c] (FP32),
// zero for K <= j < kp.  The Khatri-Rao operand s2[b][j] u3[c][j] itself is
// formed on chip by the core kernel.
template <class SP>
__global__ __launch_bounds__(256) void core_operands_kernel(
    const double* __restrict__ U1t, const double* __restrict__ U2t, const double* __restrict__ U3t,
    const double* __restrict__ xi, int r1, int r2, int r3, int64_t K, int64_t kp, const int* exps,
    typename SP::T* __restrict__ planes, float* __restrict__ s2, float* __restrict__ u3) {
  __shared__ double tile[64][65];
  const int op = blockIdx.z;
  const int r = op == 0 ? r1 : (op == 1 ? r2 : r3);
  const double* src = op == 0 ? U1t : (op == 1 ? U2t : U3t);
  const int c0 = blockIdx.y * 64;
  if (c0 >= r) return;   // uniform over the workgroup
  const int64_t j0 = (int64_t)blockIdx.x * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll 4
  for (int i = 0; i < 16; ++i) {
    const int jl = ty + 4 * i;
    const int64_t j = j0 + jl;
    const int c = c0 + tx;
    double v = 0.0;
    if (j < K && c < r) {
      v = src[j * r + c];
      if (op == 1) v = xi[j] * v;
    }
    tile[jl][tx] = v;
  }
  __syncthreads();
  const double scale = SP::SCALED && exps && op < 2 ? pow2(exps[op]) : 1.0;
  const int64_t plane = (int64_t)r1 * kp;
  const int64_t j = j0 + tx;
#pragma unroll 4
  for (int i = 0; i < 16; ++i) {
    const int cl = ty + 4 * i;
    const int c = c0 + cl;
    if (c >= r || j >= kp) continue;
    const double x = tile[tx][cl];
    if (op == 0) {
      typename SP::T t[SP::TERMS];
      SP::split(x * scale, t);
#pragma unroll
      for (int term = 0; term < SP::TERMS; ++term) planes[term * plane + c * kp + j] = t[term];
    } else if (op == 1) {
      s2[c * kp + j] = (float)(x * scale);
    } else {
      u3[c * kp + j] = (float)x;
    }
  }
}

// out[term][c][j] = term of src[j * cols + c] 2^exps[which] (zero for
// rows <= j < kp): the split planes of a row-major matrix's transpose, a
// 64 x 64 tile per workgroup through LDS (coalesced reads and writes).
template <class SP>
__global__ __launch_bounds__(256) void transpose_split_kernel(const double* __restrict__ src,
                                                              int64_t rows, int64_t cols,
                                                              int64_t kp, const int* exps,
                                                              int which,
                                                              typename SP::T* __restrict__ out) {
  __shared__ double tile[64][65];
  const int64_t j0 = (int64_t)blockIdx.x * 64, c0 = (int64_t)blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll 4
  for (int i = 0; i < 16; ++i) {
    const int jl = ty + 4 * i;
    const int64_t j = j0 + jl, c = c0 + tx;
    tile[jl][tx] = j < rows && c < cols ? src[j * cols + c] : 0.0;
  }
  __syncthreads();
  const double scale = SP::SCALED && exps ? pow2(exps[which]) : 1.0;
  const int64_t plane = cols * kp;
  const int64_t j = j0 + tx;
#pragma unroll 4
  for (int i = 0; i < 16; ++i) {
    const int cl = ty + 4 * i;
    const int64_t c = c0 + cl;
    if (c >= cols || j >= kp) continue;
    typename SP::T t[SP::TERMS];
    SP::split(tile[tx][cl] * scale, t);
#pragma unroll
    for (int term = 0; term < SP::TERMS; ++term) out[term * plane + c * kp + j] = t[term];
  }
}

// ---- grid, streaming form -------------------------------------------------------
// B rows in LDS are padded by GRID_BPAD elements.  A 16-byte LDS read is served
// in passes of lanes {0-7, 16-23} (and the like) over 64 four-byte banks; the
// B fragment reads of such a pass take two adjacent 16-byte chunks of 8
// consecutive rows.  With kp a multiple of 32, a row stride of kp + 16 half
// words is an odd multiple of 8 banks modulo 64, so the 8 rows start on 8
// distinct multiples of 8 banks and the 16 reads hit 64 distinct banks (a pad
// of 8 gave a stride of 52 banks at kp = 352: rows 5, 6, 7 met the second
// chunks of rows 0, 1, 2, a two-way conflict in every pass).
constexpr int GRID_BPAD = 16;

// Persistent workgroups of 8 waves.  Workgroup (panel, group) keeps the B
// planes of a panel of BN columns in LDS and walks the row tiles (128 rows:
// 16 per wave) of its group; the A fragments of the next tile are loaded
// while the current one is multiplied.  Each wave stages its 16 x BN FP32
// tile in LDS and writes whole rows with 16-byte stores.  The panels of one
// row group run on one XCD (workgroup w runs on XCD w % 8), so the A rows
// they share are read from that XCD's L2.
template <class SP, int BN, bool FOLD>
__global__ __launch_bounds__(512) void grid_stream_kernel(const typename SP::T* __restrict__ Ap,
                                                          const typename SP::T* __restrict__ Bp,
                                                          int64_t M, int64_t N, int kp,
                                                          int npanels, int groups,
                                                          float* __restrict__ grid,
                                                          const int* exps) {
  typedef typename SP::T T;
  typedef typename SP::V8 V8;
  constexpr int FN = BN / 16;
  constexpr int SLD = BN + 4;   // staging row stride (floats)
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int ks = kp + GRID_BPAD;
  T* Bs = (T*)smem;                                          // [term][BN][ks]
  float* stage = (float*)(smem + (size_t)SP::TERMS * BN * ks * sizeof(T));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int w = blockIdx.x;
  const int xcd = w & 7, iw = w >> 3;
  const int panel = iw % npanels;
  const int g = (iw / npanels) * 8 + xcd;
  const int64_t n0 = (int64_t)panel * BN;
  // B panel to LDS (rows beyond N are zero)
  const int64_t planeB = N * kp;
  for (int e = threadIdx.x; e < SP::TERMS * BN * kp; e += 512) {
    const int term = e / (BN * kp), rem = e - term * (BN * kp);
    const int col = rem / kp, k = rem - col * kp;
    Bs[(term * BN + col) * ks + k] = n0 + col < N ? Bp[term * planeB + (n0 + col) * kp + k] : (T)0.0f;
  }
  __syncthreads();
  const int64_t tiles = (M + 127) / 128;
  if (g >= groups) return;   // uniform over the workgroup, after the only barrier
  const int64_t planeA = M * kp;
  const int kofs = 8 * (lane >> 4);
  const double out_scale = SP::SCALED && exps ? pow2(-exps[0] - exps[1]) : 1.0;
  float* st = stage + wave * 16 * SLD;
  auto arow_of = [&](int64_t tile) {
    const int64_t r = tile * 128 + wave * 16 + (lane & 15);
    return (r < M ? r : 0) * kp + kofs;
  };
  // A fragments two steps ahead in two register sets: a0 / a1 hold steps
  // kb, kb + 1 of the tile; a step past the tile's end is that step of the
  // next tile of this group (or a valid reload of this one after the last
  // tile), so the loads run ahead across tiles too
  const int nkb = kp / 32;
  int64_t tile = g;
  if (tile >= tiles) return;
  int64_t arow = arow_of(tile);
  auto loadA = [&](int64_t ar, int64_t ar_next, int step, V8 (&dst)[SP::TERMS]) {
    const int sn = step - nkb < nkb - 1 ? step - nkb : nkb - 1;
    const int64_t off = step < nkb ? ar + 32 * (int64_t)step : ar_next + 32 * (int64_t)sn;
#pragma unroll
    for (int term = 0; term < SP::TERMS; ++term) dst[term] = *(const V8*)(Ap + term * planeA + off);
  };
  V8 a0[SP::TERMS], a1[SP::TERMS];
  {
    const int64_t t1 = tile + groups;
    const int64_t ar_next = t1 < tiles ? arow_of(t1) : arow;
    loadA(arow, ar_next, 0, a0);
    loadA(arow, ar_next, 1, a1);
  }
  for (; tile < tiles; tile += groups) {
    const int64_t next = tile + groups;
    const int64_t arow_next = next < tiles ? arow_of(next) : arow;
    f4 acc[FN][SP::LEVELS];
    double acc64[FOLD ? FN : 1][4];
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int l = 0; l < SP::LEVELS; ++l) acc[j][l] = f4{0.f, 0.f, 0.f, 0.f};
    if (FOLD)
#pragma unroll
      for (int j = 0; j < (FOLD ? FN : 1); ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc64[j][v] = 0.0;
    int since = 0;
    auto step = [&](const V8 (&a)[SP::TERMS], int kb) {
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        V8 b[SP::TERMS];
#pragma unroll
        for (int term = 0; term < SP::TERMS; ++term)
          b[term] = *(const V8*)(Bs + (size_t)(term * BN + j * 16 + (lane & 15)) * ks + 32 * kb + kofs);
#pragma unroll
        for (int pi = 0; pi < SP::NPROD; ++pi)
          acc[j][SP::PL[pi]] = SP::mfma(a[SP::PA[pi]], b[SP::PB[pi]], acc[j][SP::PL[pi]]);
      }
      if (FOLD) {
        since += 32;
        if (since >= KCHUNK && kb + 1 < nkb) {
#pragma unroll
          for (int j = 0; j < (FOLD ? FN : 1); ++j) {
#pragma unroll
            for (int v = 0; v < 4; ++v) acc64[j][v] += SP::combine(acc[j], v);
#pragma unroll
            for (int l = 0; l < SP::LEVELS; ++l) acc[j][l] = f4{0.f, 0.f, 0.f, 0.f};
          }
          since = 0;
        }
      }
    };
    for (int kb = 0; kb < nkb; kb += 2) {
      V8 f0[SP::TERMS];
      loadA(arow, arow_next, kb + 2, f0);
      step(a0, kb);
#pragma unroll
      for (int term = 0; term < SP::TERMS; ++term) a0[term] = f0[term];
      if (kb + 1 < nkb) {
        V8 f1[SP::TERMS];
        loadA(arow, arow_next, kb + 3, f1);
        step(a1, kb + 1);
#pragma unroll
        for (int term = 0; term < SP::TERMS; ++term) a1[term] = f1[term];
      }
    }
    if (nkb & 1) {
      // odd step count: the next tile's step 0 landed in a1, its step 1 in a0
#pragma unroll
      for (int term = 0; term < SP::TERMS; ++term) {
        const V8 t = a0[term];
        a0[term] = a1[term];
        a1[term] = t;
      }
    }
    // stage the 16 x BN tile: lane holds D[4 (lane / 16) + v][16 j + lane % 16]
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double val = SP::combine(acc[j], v);
        if (FOLD) val += acc64[FOLD ? j : 0][v];
        st[(4 * (lane >> 4) + v) * SLD + j * 16 + (lane & 15)] = (float)(val * out_scale);
      }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // write rows: BN / 4 lanes per row
    constexpr int LPR = BN / 4;            // lanes per row (float4 each)
    constexpr int RPI = 64 / LPR;          // rows per instruction
    const int64_t row0 = tile * 128 + wave * 16;
#pragma unroll
    for (int r0 = 0; r0 < 16; r0 += RPI) {
      const int r = r0 + lane / LPR, cq = lane % LPR;
      const int64_t row = row0 + r, col = n0 + 4 * cq;
      if (row < M && col < N) {
        const f4 v4 = *(const f4*)(st + r * SLD + 4 * cq);
        float* dst = grid + row * N + col;
        if (col + 3 < N && ((row * N + col) & 3) == 0) {
          __builtin_nontemporal_store(v4, (f4*)dst);
        } else {
          const float vv[4] = {v4[0], v4[1], v4[2], v4[3]};
          for (int q = 0; q < 4 && col + q < N; ++q) __builtin_nontemporal_store(vv[q], dst + q);
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    arow = arow_next;
  }
}

// ---- core, LDS-tiled: beta_(1)[a, col] = sum_j A[a, j] B[j, col] ------------------
// col = b r3 + c, B[j, col] = s2[b][j] u3[c][j] formed in FP32 and split once
// per workgroup into LDS.  Workgroup tile 32 WGM rows x 32 FN columns, the
// columns being FN values of b times 32 values of c (so that a tile reads 32
// rows of u3 and FN of s2, and the workgroups resident together share
// them), 2 WGM waves of 32 x 16 FN (2 x FN MFMA blocks).  Per step of 32 k the next A
// fragments (from the split planes) and the raw s2/u3 values are loaded into
// registers while the MFMAs of the current step run, then written to LDS.
// LDS layout: rows of 32 elements (64 bytes, four 16-byte chunks), chunk c
// of row r stored at chunk c ^ sw(r), sw(r) = 2 ((r / 4) % 2).  A 16-byte
// LDS access is served in passes of lanes {0-7, 16-23} (and the like); the
// fragment reads of such a pass (8 consecutive rows, 2 chunks) then hit 16
// distinct four-bank groups of the 64 banks.  The loads keep 4 consecutive
// lanes on one row (64 contiguous bytes: one request per quad), and quad Q
// of a 16-row group takes row rho(Q), Q with bits 1 and 2 swapped, so that
// the 4 quads of a store pass write 4 rows of distinct r % 4 with one sw:
// also conflict-free.  FP32 accumulators are folded into FP64 every KCHUNK.
// FN column blocks per wave: 4 for the two-term FP16 split, 2 for the
// three-term BF16 split (whose accumulators take more registers).
// LDS row of loader quad Q (bits 1 and 2 of Q swapped within its 16-row
// group) and the chunk swizzle of row r
__device__ __forceinline__ int lds_row(int Q) {
  return (Q & ~6) | ((Q & 2) << 1) | ((Q & 4) >> 1);
}
__device__ __forceinline__ int lds_sw(int r) { return ((r >> 2) & 1) << 1; }

template <class SP, int WGM, int FN>
__global__ __launch_bounds__(128 * WGM) void core_tile_kernel(
    const typename SP::T* __restrict__ Ap, const float* __restrict__ s2,
    const float* __restrict__ u3, int r1, int r2, int r3, int64_t kp, int64_t kchunk,
    int row_tiles, int b_tiles, double* __restrict__ out, int64_t split_stride, const int* exps) {
  typedef typename SP::T T;
  typedef typename SP::V8 V8;
  constexpr int NT = 128 * WGM, BM = 32 * WGM, BN = 32 * FN, LDK = 32;
  constexpr int BB = FN;   // column tile: BB values of b x 32 values of c
  constexpr int A_ITEMS = BM * 4 * SP::TERMS, A_PER = (A_ITEMS + NT - 1) / NT;
  constexpr int B_ITEMS = BN * 4, B_PER = (B_ITEMS + NT - 1) / NT;
  __shared__ __attribute__((aligned(16))) T As[2][SP::TERMS][BM][LDK];
  __shared__ __attribute__((aligned(16))) T Bs[2][SP::TERMS][BN][LDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int W = r2 * r3;
  // workgroup order: row tile fastest, then b tile, then c group, so that the
  // workgroups resident at one time (spread over the XCDs in order) share
  // the 32 u3 rows of one c group and the A rows of every row tile in L2
  const int rt = blockIdx.x % row_tiles;
  const int bt = (blockIdx.x / row_tiles) % b_tiles, cg = blockIdx.x / row_tiles / b_tiles;
  const int a0 = rt * BM, b0 = bt * BB, c0 = cg * 32;
  const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
  const int64_t kend = kbeg + kchunk < kp ? kbeg + kchunk : kp;
  const int64_t planeA = (int64_t)r1 * kp;

  // loader coordinates (fixed over k); item i of a term: quad Q = i / 4 on
  // row (Q & ~15) | rho(Q & 15), 16-byte chunk i % 4.  Rows of A beyond r1
  // and columns beyond the b, c ranges load a valid row instead (the last
  // one): they only feed output rows and columns that are never written, so
  // the loads need no branches.  Items past the tile (when the threads
  // outnumber them) reload item 0 and are not stored.
  int64_t a_src[A_PER];
  int a_dst[A_PER];
#pragma unroll
  for (int u = 0; u < A_PER; ++u) {
    const int idx = tid + NT * u < A_ITEMS ? tid + NT * u : 0;
    const int term = idx / (BM * 4), rem = idx - term * (BM * 4);
    const int row = lds_row(rem >> 2), q = rem & 3;
    const int grow = a0 + row < r1 ? a0 + row : r1 - 1;
    a_src[u] = term * planeA + (int64_t)grow * kp + 8 * q;
    a_dst[u] = (term * BM + row) * LDK + 8 * (q ^ lds_sw(row));
  }
  int64_t s_src[B_PER], u_src[B_PER];
  int b_dst[B_PER];
#pragma unroll
  for (int u = 0; u < B_PER; ++u) {
    const int idx = tid + NT * u < B_ITEMS ? tid + NT * u : 0;
    const int n = lds_row(idx >> 2), q = idx & 3;
    const int b = b0 + n / 32 < r2 ? b0 + n / 32 : r2 - 1;
    const int c = c0 + n % 32 < r3 ? c0 + n % 32 : r3 - 1;
    s_src[u] = (int64_t)b * kp + 8 * q;
    u_src[u] = (int64_t)c * kp + 8 * q;
    b_dst[u] = n * LDK + 8 * (q ^ lds_sw(n));
  }
  // Pipeline: LDS buffer s % 2 holds step s.  While the MFMAs of step s
  // run, the workgroup forms step s + 1 (from registers) into the other
  // buffer and issues the loads of step s + 3; one barrier per step.  Two
  // register sets hold steps s + 1 and s + 2, so a load has two steps to
  // land.  The loop body has no branch (loads past the end re-read the last
  // step, and the last step's formation goes to a buffer nobody reads), so
  // the MFMAs and the formation share one scheduling region and interleave.
  struct Regs {
    V8 ra[A_PER];
    float4 rs[B_PER][2], ru[B_PER][2];
  };
  Regs R0, R1;
  const int64_t klast = kend - 32;
  auto load = [&](int64_t k0, Regs& R) {
    k0 = k0 < klast ? k0 : klast;
#pragma unroll
    for (int u = 0; u < A_PER; ++u) R.ra[u] = *(const V8*)(Ap + a_src[u] + k0);
#pragma unroll
    for (int u = 0; u < B_PER; ++u) {
      R.rs[u][0] = *(const float4*)(s2 + s_src[u] + k0);
      R.rs[u][1] = *(const float4*)(s2 + s_src[u] + k0 + 4);
      R.ru[u][0] = *(const float4*)(u3 + u_src[u] + k0);
      R.ru[u][1] = *(const float4*)(u3 + u_src[u] + k0 + 4);
    }
  };
  auto store = [&](const Regs& R, int buf) {
#pragma unroll
    for (int u = 0; u < A_PER; ++u)
      if (A_ITEMS % NT == 0 || tid + NT * u < A_ITEMS)
        *(V8*)(&As[buf][0][0][0] + a_dst[u]) = R.ra[u];
#pragma unroll
    for (int u = 0; u < B_PER; ++u) {
      // threads past the tile store nothing (no test where the items fill
      // every thread: the formation then stays in the MFMAs' basic block)
      if (B_ITEMS % NT != 0 && tid + NT * u >= B_ITEMS) break;
      const float x[8] = {R.rs[u][0].x * R.ru[u][0].x, R.rs[u][0].y * R.ru[u][0].y,
                          R.rs[u][0].z * R.ru[u][0].z, R.rs[u][0].w * R.ru[u][0].w,
                          R.rs[u][1].x * R.ru[u][1].x, R.rs[u][1].y * R.ru[u][1].y,
                          R.rs[u][1].z * R.ru[u][1].z, R.rs[u][1].w * R.ru[u][1].w};
      V8 bv[SP::TERMS];
      if constexpr (SP::PAIRED) {
        SP::split8(x, bv[0], bv[1]);
      } else {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          T parts[SP::TERMS];
          SP::split32(x[t], parts);
#pragma unroll
          for (int term = 0; term < SP::TERMS; ++term) bv[term][t] = parts[term];
        }
      }
#pragma unroll
      for (int term = 0; term < SP::TERMS; ++term)
        *(V8*)(&Bs[buf][term][0][0] + b_dst[u]) = bv[term];
    }
  };

  f4 acc[2][FN][SP::LEVELS];
  double acc64[2][FN][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
#pragma unroll
      for (int l = 0; l < SP::LEVELS; ++l) acc[i][j][l] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int v = 0; v < 4; ++v) acc64[i][j][v] = 0.0;
    }
  const int nsteps = kbeg < kend ? (int)((kend - kbeg) / 32) : 0;
  if (nsteps > 0) {
    load(kbeg, R0);
    load(kbeg + 32, R1);
    store(R0, 0);
    load(kbeg + 64, R0);
  }
  __syncthreads();
  const int frow = lane & 15, fc = lane >> 4;
  // step s: MFMAs on buffer s % 2; `R` holds step s + 1 (formed into the
  // other buffer) and then receives step s + 3
  auto step = [&](int st, Regs& R) {
    const int cur = st & 1;
    V8 af[2][SP::TERMS], bf[FN][SP::TERMS];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int r = wm * 32 + i * 16 + frow;
#pragma unroll
      for (int term = 0; term < SP::TERMS; ++term)
        af[i][term] = *(const V8*)(&As[cur][term][r][8 * (fc ^ lds_sw(r))]);
    }
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int r = wn * (16 * FN) + j * 16 + frow;
#pragma unroll
      for (int term = 0; term < SP::TERMS; ++term)
        bf[j][term] = *(const V8*)(&Bs[cur][term][r][8 * (fc ^ lds_sw(r))]);
    }
    // products in the outer loop: the MFMAs that accumulate into one level
    // of one block are 2 FN instructions apart
#pragma unroll
    for (int pi = 0; pi < SP::NPROD; ++pi)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j][SP::PL[pi]] =
              SP::mfma(af[i][SP::PA[pi]], bf[j][SP::PB[pi]], acc[i][j][SP::PL[pi]]);
    store(R, cur ^ 1);
    load(kbeg + 32 * (int64_t)(st + 3), R);
    // schedule: fragment reads first, then each MFMA followed by a share of
    // the formation's VALU work, LDS writes and global loads
    constexpr int NMF = SP::NPROD * 2 * FN;
    __builtin_amdgcn_sched_group_barrier(0x100, 2 * SP::TERMS + FN * SP::TERMS, 0);
#pragma unroll
    for (int m = 0; m < NMF; ++m) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);
      if (m % 4 == 3) __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);
      if (m % 4 == 1) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
    }
    if ((st + 1) % (KCHUNK / 32) == 0 || st + 1 == nsteps) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
#pragma unroll
          for (int v = 0; v < 4; ++v) acc64[i][j][v] += SP::combine(acc[i][j], v);
#pragma unroll
          for (int l = 0; l < SP::LEVELS; ++l) acc[i][j][l] = f4{0.f, 0.f, 0.f, 0.f};
        }
    }
    __syncthreads();
  };
  for (int st = 0; st < nsteps; st += 2) {
    step(st, R1);
    if (st + 1 < nsteps) step(st + 1, R0);
  }
  const double out_scale = SP::SCALED && exps ? pow2(-exps[0] - exps[1]) : 1.0;
  double* o = out + (int64_t)blockIdx.z * split_stride;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int n = wn * (16 * FN) + j * 16 + frow;
      const int b = b0 + n / 32, c = c0 + n % 32;
      const int col = b * r3 + c;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = a0 + wm * 32 + i * 16 + 4 * (lane >> 4) + v;
        if (a < r1 && b < r2 && c < r3) o[(int64_t)a * W + col] = acc64[i][j][v] * out_scale;
      }
    }
}

// ---- split GEMM, LDS-tiled: C[m, c] = sum_i A[m, i] B[c, i] ----------------------
// Both operands come as split planes [term][row][kp] (the projection: A the
// side matrix, one row per canonical term, i over the grid, B the basis
// transposed; the second expansion: A the basis V2, B the first expansion
// with the rank index b contiguous).  The same tiling, LDS layout,
// two-register-set pipeline and FP64 folds as the core kernel below, with B
// loaded like A instead of formed.  Output FP64 at
// (c / ccb) sccb + (c % ccb) + m ldc.  Workgroup order: column tile fastest
// (the workgroups that share a row tile of A run together) or, with
// row_fast, row tile fastest (they share a column tile of B).
template <class SP> struct GridSplitOf { typedef SplitF16 type; };
template <> struct GridSplitOf<SplitBF16> { typedef SplitBF16 type; };

template <class SP, int WGM, int FN>
__global__ __launch_bounds__(128 * WGM) void proj_tile_kernel(
    const typename SP::T* __restrict__ Ap, const typename SP::T* __restrict__ Bp, int64_t M,
    int64_t N, int64_t kp, int64_t col_tiles, int64_t row_tiles, int row_fast,
    double* __restrict__ out, int64_t ldc, int64_t ccb, int64_t sccb, const int* exps,
    typename GridSplitOf<SP>::type::T* __restrict__ pout, int64_t pkp, const int* pexp) {
  typedef typename SP::T T;
  typedef typename SP::V8 V8;
  constexpr int NT = 128 * WGM, BM = 32 * WGM, BN = 32 * FN, LDK = 32;
  constexpr int A_ITEMS = BM * 4 * SP::TERMS, A_PER = (A_ITEMS + NT - 1) / NT;
  constexpr int B_ITEMS = BN * 4 * SP::TERMS, B_PER = (B_ITEMS + NT - 1) / NT;
  __shared__ __attribute__((aligned(16))) T As[2][SP::TERMS][BM][LDK];
  __shared__ __attribute__((aligned(16))) T Bs[2][SP::TERMS][BN][LDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t x = blockIdx.x;
  const int64_t ct = row_fast ? x / row_tiles : x % col_tiles;
  const int64_t m0 = (row_fast ? x % row_tiles : x / col_tiles) * BM;
  const int64_t c0 = ct * BN;
  const int64_t planeA = M * kp, planeB = N * kp;
  int64_t a_src[A_PER];
  int a_dst[A_PER];
#pragma unroll
  for (int u = 0; u < A_PER; ++u) {
    const int idx = tid + NT * u < A_ITEMS ? tid + NT * u : 0;
    const int term = idx / (BM * 4), rem = idx - term * (BM * 4);
    const int row = lds_row(rem >> 2), q = rem & 3;
    const int64_t grow = m0 + row < M ? m0 + row : M - 1;
    a_src[u] = term * planeA + grow * kp + 8 * q;
    a_dst[u] = (term * BM + row) * LDK + 8 * (q ^ lds_sw(row));
  }
  int64_t b_src[B_PER];
  int b_dst[B_PER];
#pragma unroll
  for (int u = 0; u < B_PER; ++u) {
    const int idx = tid + NT * u < B_ITEMS ? tid + NT * u : 0;
    const int term = idx / (BN * 4), rem = idx - term * (BN * 4);
    const int row = lds_row(rem >> 2), q = rem & 3;
    const int64_t gcol = c0 + row < N ? c0 + row : N - 1;
    b_src[u] = term * planeB + gcol * kp + 8 * q;
    b_dst[u] = (term * BN + row) * LDK + 8 * (q ^ lds_sw(row));
  }
  struct Regs {
    V8 ra[A_PER], rb[B_PER];
  };
  Regs R0, R1;
  const int64_t klast = kp - 32;
  auto load = [&](int64_t k0, Regs& R) {
    k0 = k0 < klast ? k0 : klast;
#pragma unroll
    for (int u = 0; u < A_PER; ++u) R.ra[u] = *(const V8*)(Ap + a_src[u] + k0);
#pragma unroll
    for (int u = 0; u < B_PER; ++u) R.rb[u] = *(const V8*)(Bp + b_src[u] + k0);
  };
  auto store = [&](const Regs& R, int buf) {
#pragma unroll
    for (int u = 0; u < A_PER; ++u)
      if (A_ITEMS % NT == 0 || tid + NT * u < A_ITEMS)
        *(V8*)(&As[buf][0][0][0] + a_dst[u]) = R.ra[u];
#pragma unroll
    for (int u = 0; u < B_PER; ++u)
      if (B_ITEMS % NT == 0 || tid + NT * u < B_ITEMS)
        *(V8*)(&Bs[buf][0][0][0] + b_dst[u]) = R.rb[u];
  };
  f4 acc[2][FN][SP::LEVELS];
  double acc64[2][FN][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
#pragma unroll
      for (int l = 0; l < SP::LEVELS; ++l) acc[i][j][l] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int v = 0; v < 4; ++v) acc64[i][j][v] = 0.0;
    }
  const int nsteps = (int)(kp / 32);
  load(0, R0);
  load(32, R1);
  store(R0, 0);
  load(64, R0);
  __syncthreads();
  const int frow = lane & 15, fc = lane >> 4;
  auto step = [&](int st, Regs& R) {
    const int cur = st & 1;
    V8 af[2][SP::TERMS], bf[FN][SP::TERMS];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int r = wm * 32 + i * 16 + frow;
#pragma unroll
      for (int term = 0; term < SP::TERMS; ++term)
        af[i][term] = *(const V8*)(&As[cur][term][r][8 * (fc ^ lds_sw(r))]);
    }
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int r = wn * (16 * FN) + j * 16 + frow;
#pragma unroll
      for (int term = 0; term < SP::TERMS; ++term)
        bf[j][term] = *(const V8*)(&Bs[cur][term][r][8 * (fc ^ lds_sw(r))]);
    }
#pragma unroll
    for (int pi = 0; pi < SP::NPROD; ++pi)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j][SP::PL[pi]] =
              SP::mfma(af[i][SP::PA[pi]], bf[j][SP::PB[pi]], acc[i][j][SP::PL[pi]]);
    store(R, cur ^ 1);
    load(32 * (int64_t)(st + 3), R);
    if ((st + 1) % (KCHUNK / 32) == 0 || st + 1 == nsteps) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
#pragma unroll
          for (int v = 0; v < 4; ++v) acc64[i][j][v] += SP::combine(acc[i][j], v);
#pragma unroll
          for (int l = 0; l < SP::LEVELS; ++l) acc[i][j][l] = f4{0.f, 0.f, 0.f, 0.f};
        }
    }
    __syncthreads();
  };
  for (int st = 0; st < nsteps; st += 2) {
    step(st, R1);
    if (st + 1 < nsteps) step(st + 1, R0);
  }
  const double out_scale = SP::SCALED && exps ? pow2(-exps[0] - exps[1]) : 1.0;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int64_t c = c0 + wn * (16 * FN) + j * 16 + frow;
      const int64_t cb = c / ccb, cr = c - cb * ccb;
      const int64_t coff = cb * sccb + cr;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t m = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + v;
        if (m < M && c < N) out[coff + m * ldc] = acc64[i][j][v] * out_scale;
      }
    }
  if (!pout) return;
  // The grid's split planes of the output: element (m, c) goes to plane row
  // (c / ccb) M + m, column c % ccb.  The tile is staged in LDS (the B
  // buffers, free after the last step) and written along plane rows, 64
  // consecutive columns per store instruction.
  typedef typename GridSplitOf<SP>::type GP;
  typedef typename GP::T PT;
  const double pscale = GP::SCALED ? pow2(pexp[0]) : 1.0;
  const int64_t pplane = (N / ccb) * M * pkp;
  if constexpr (GP::TERMS * BM * BN > 2 * SP::TERMS * BN * LDK) {
    // (tiles whose staging would exceed the B buffers: element by element)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int64_t c = c0 + wn * (16 * FN) + j * 16 + frow;
        const int64_t cb = c / ccb, cr = c - cb * ccb;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t m = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + v;
          if (m >= M || c >= N) continue;
          PT t[GP::TERMS];
          GP::split(acc64[i][j][v] * out_scale * pscale, t);
#pragma unroll
          for (int term = 0; term < GP::TERMS; ++term) pout[term * pplane + (cb * M + m) * pkp + cr] = t[term];
        }
      }
    return;
  }
  PT* stg = (PT*)&Bs[0][0][0][0];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wm * 32 + i * 16 + 4 * (lane >> 4) + v;
        const int col = wn * (16 * FN) + j * 16 + frow;
        PT t[GP::TERMS];
        GP::split(acc64[i][j][v] * out_scale * pscale, t);
#pragma unroll
        for (int term = 0; term < GP::TERMS; ++term) stg[(term * BM + row) * BN + col] = t[term];
      }
  __syncthreads();
  int64_t pcb[BN / 64], pcr[BN / 64];
#pragma unroll
  for (int hh = 0; hh < BN / 64; ++hh) {
    const int64_t c = c0 + hh * 64 + lane;
    pcb[hh] = c / ccb;
    pcr[hh] = c - pcb[hh] * ccb;
  }
  for (int row = wave; row < BM; row += NT / 64) {
    const int64_t m = m0 + row;
    if (m >= M) break;
#pragma unroll
    for (int hh = 0; hh < BN / 64; ++hh) {
      const int64_t c = c0 + hh * 64 + lane;
      if (c >= N) continue;
      const int64_t pe = (pcb[hh] * M + m) * pkp + pcr[hh];
#pragma unroll
      for (int term = 0; term < GP::TERMS; ++term)
        pout[term * pplane + pe] = stg[(term * BM + row) * BN + hh * 64 + lane];
    }
  }
}

// ---- max |x| of FP64 arrays as ordered bit patterns (deterministic) ----------
// Wave maxima are combined in LDS; one integer atomic per workgroup (the
// maximum does not depend on the order).  Device-scope atomics on one address
// are serialised (about 12 ns each), so the launch holds few workgroups and
// each thread keeps ABS_UNROLL coalesced loads in flight per pass.
constexpr int ABS_UNROLL = 8;
constexpr int ABS_MAX_BLOCKS = 512;

__global__ __launch_bounds__(256) void absmax_kernel(const double* __restrict__ x, int64_t count,
                                                     unsigned long long* __restrict__ out) {
  __shared__ double wmax[4];
  double m = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; e + (ABS_UNROLL - 1) * stride < count; e += ABS_UNROLL * stride) {
    double v[ABS_UNROLL];
#pragma unroll
    for (int k = 0; k < ABS_UNROLL; ++k) v[k] = fabs(x[e + k * stride]);
#pragma unroll
    for (int k = 0; k < ABS_UNROLL; ++k)
      if (v[k] > m) m = v[k];
  }
  for (; e < count; e += stride) {
    const double v = fabs(x[e]);
    if (v > m) m = v;
  }
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double b = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
    if (b > 0.0) atomicMax(out, (unsigned long long)__double_as_longlong(b));
  }
}

// exps[i] = 14 - ceil(log2(prod of the listed maxima)) so that the scaled
// operand stays below 2^14 in FP16 (0 for BF16 or an all-zero operand).
__global__ void scale_exponents_kernel(const unsigned long long* mx, int nbops, int fp16, int* exps) {
  if (threadIdx.x != 0) return;
  // operand A: mx[0]; operand B: the product of mx[1 .. nbops]
  const double a = __longlong_as_double((long long)mx[0]);
  double b = 1.0;
  for (int i = 0; i < nbops; ++i) b *= __longlong_as_double((long long)mx[1 + i]);
  int ea = 0, eb = 0;
  if (fp16) {
    if (a > 0.0) ea = 14 - (int)ceil(log2(a));
    if (b > 0.0) eb = 14 - (int)ceil(log2(b));
  }
  exps[0] = ea;
  exps[1] = eb;
}

static void absmax(const double* x, int64_t count, unsigned long long* out, hipStream_t s) {
  unsigned blocks = (unsigned)std::min<int64_t>((count + 256 * ABS_UNROLL - 1) / (256 * ABS_UNROLL),
                                                 ABS_MAX_BLOCKS);
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(absmax_kernel, dim3(blocks), dim3(256), 0, s, x, count, out);
}

// mx: 4 u64, exps: 2 int (device)
static void scale_setup(const double* A, int64_t na, const double* const* B, const int64_t* nb,
                        int nbops, int fp16, unsigned long long* mx, int* exps, hipStream_t s) {
  RS_HIP(hipMemsetAsync(mx, 0, 4 * sizeof(unsigned long long), s));
  absmax(A, na, mx, s);
  for (int i = 0; i < nbops; ++i) absmax(B[i], nb[i], mx + 1 + i, s);
  hipLaunchKernelGGL(scale_exponents_kernel, dim3(1), dim3(64), 0, s, mx, nbops, fp16, exps);
}

static unsigned grid_blocks(int64_t total) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 8192));
}

template <class SP>
static void split_planes(const double* src, int64_t rows, int64_t cols, int64_t s_row,
                         int64_t s_col, int64_t kp, const int* exps, int which,
                         typename SP::T* out, hipStream_t s) {
  const unsigned gx = (unsigned)((kp + 255) / 256);
  const unsigned gy = (unsigned)std::max<int64_t>(1, std::min<int64_t>(rows, 8192));
  hipLaunchKernelGGL(split_planes_kernel<SP>, dim3(gx, gy), dim3(256), 0, s, src, rows, (int)cols,
                     s_row, s_col, (int)kp, exps, which, out);
}

// ---- core ------------------------------------------------------------------------
struct CoreMixedPlan {
  int64_t kp, kchunk;
  int splits, wgm, row_tiles, col_tiles, b_tiles;
  size_t o_mx, o_exps, o_planes, o_s2, o_u3, o_part, total;
};

// rows per workgroup tile 32 WGM, WGM in {4, 3, 2}: the least padding of r1
// (ties to the larger tile)
static int core_wgm(int r1) {
  int best = 4;
  int64_t best_pad = INT64_MAX;
  for (int w : {4, 3, 2}) {
    const int64_t pad = (int64_t)((r1 + 32 * w - 1) / (32 * w)) * 32 * w;
    if (pad < best_pad) {
      best_pad = pad;
      best = w;
    }
  }
  return best;
}

static CoreMixedPlan plan_core_mixed(int prec, int r1, int r2, int r3, int64_t K, int num_cu) {
  CoreMixedPlan P{};
  const int fn = prec == RS_MIXED_BF16 ? 2 : 4;
  P.kp = pad32(K);
  P.wgm = core_wgm(r1);
  P.row_tiles = (r1 + 32 * P.wgm - 1) / (32 * P.wgm);
  P.b_tiles = (r2 + fn - 1) / fn;   // column tiles: fn values of b x 32 of c
  P.col_tiles = P.b_tiles * ((r3 + 31) / 32);
  const int64_t wgs = (int64_t)P.row_tiles * P.col_tiles;
  P.splits = 1;
  if (wgs < 2LL * num_cu) {
    const int64_t want = (2LL * num_cu + wgs - 1) / wgs;
    P.splits = (int)std::max<int64_t>(1, std::min<int64_t>(want, std::min<int64_t>(P.kp / KCHUNK, 64)));
  }
  P.kchunk = (P.kp + P.splits - 1) / P.splits;
  P.kchunk = (P.kchunk + 31) / 32 * 32;
  P.splits = (int)((P.kp + P.kchunk - 1) / P.kchunk);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  };
  P.o_mx = take(4 * sizeof(unsigned long long));
  P.o_exps = take(2 * sizeof(int));
  P.o_planes = take((size_t)3 * r1 * P.kp * 2);     // up to 3 terms of 2 bytes
  P.o_s2 = take((size_t)r2 * P.kp * sizeof(float));
  P.o_u3 = take((size_t)r3 * P.kp * sizeof(float));
  P.o_part = take(P.splits > 1 ? (size_t)P.splits * r1 * r2 * r3 * sizeof(double) : 0);
  P.total = off;
  return P;
}

// enough for either split (their tiles, and so their split-K plans, differ)
size_t core_mixed_workspace_bytes(int r1, int r2, int r3, int64_t K, int num_cu) {
  return std::max(plan_core_mixed(RS_MIXED_FP16, r1, r2, r3, K, num_cu).total,
                  plan_core_mixed(RS_MIXED_BF16, r1, r2, r3, K, num_cu).total);
}

template <class SP>
static void core_mixed_t(int fp16, const double* U1t, const double* U2t, const double* U3t,
                         const double* xi, int r1, int r2, int r3, int64_t K, double* beta,
                         int num_cu, char* work, hipStream_t s, const KernelTimer* kt) {
  const CoreMixedPlan P =
      plan_core_mixed(fp16 ? RS_MIXED_FP16 : RS_MIXED_BF16, r1, r2, r3, K, num_cu);
  unsigned long long* mx = (unsigned long long*)(work + P.o_mx);
  int* exps = (int*)(work + P.o_exps);
  typename SP::T* planes = (typename SP::T*)(work + P.o_planes);
  float* s2 = (float*)(work + P.o_s2);
  float* u3 = (float*)(work + P.o_u3);
  double* part = P.splits > 1 ? (double*)(work + P.o_part) : nullptr;
  const double* Bops[3] = {xi, U2t, U3t};
  const int64_t nb[3] = {K, K * r2, K * r3};
  scale_setup(U1t, K * r1, Bops, nb, 3, fp16, mx, exps, s);
  // A = U~1^T: row a, column j at U1t[j r1 + a]; the Khatri-Rao factors s2, u3
  const int rmax = std::max(r1, std::max(r2, r3));
  hipLaunchKernelGGL(core_operands_kernel<SP>,
                     dim3((unsigned)((P.kp + 63) / 64), (unsigned)((rmax + 63) / 64), 3), dim3(256),
                     0, s, U1t, U2t, U3t, xi, r1, r2, r3, K, P.kp, exps, planes, s2, u3);
  const dim3 grid((unsigned)(P.row_tiles * P.col_tiles), 1, (unsigned)P.splits);
  double* out = part ? part : beta;
  const int64_t stride = (int64_t)r1 * r2 * r3;
  constexpr int FN = SP::TERMS == 2 ? 4 : 2;
  if (kt) RS_HIP(hipEventRecord(kt->begin, s));
  if (P.wgm == 4)
    hipLaunchKernelGGL((core_tile_kernel<SP, 4, FN>), grid, dim3(512), 0, s, planes, s2, u3, r1, r2,
                       r3, P.kp, P.kchunk, P.row_tiles, P.b_tiles, out, stride, exps);
  else if (P.wgm == 3)
    hipLaunchKernelGGL((core_tile_kernel<SP, 3, FN>), grid, dim3(384), 0, s, planes, s2, u3, r1, r2,
                       r3, P.kp, P.kchunk, P.row_tiles, P.b_tiles, out, stride, exps);
  else
    hipLaunchKernelGGL((core_tile_kernel<SP, 2, FN>), grid, dim3(256), 0, s, planes, s2, u3, r1, r2,
                       r3, P.kp, P.kchunk, P.row_tiles, P.b_tiles, out, stride, exps);
  if (kt) RS_HIP(hipEventRecord(kt->end, s));
  if (part) core64_reduce(part, P.splits, (int64_t)r1 * r2 * r3, beta, s);
}

void core_mixed(int prec, const double* U1t, const double* U2t, const double* U3t, const double* xi,
                int r1, int r2, int r3, int64_t K, double* beta, int num_cu, double* work,
                hipStream_t s, const KernelTimer* kt) {
  if (prec == RS_MIXED_FP16)
    core_mixed_t<CoreF16>(1, U1t, U2t, U3t, xi, r1, r2, r3, K, beta, num_cu, (char*)work, s, kt);
  else
    core_mixed_t<SplitBF16>(0, U1t, U2t, U3t, xi, r1, r2, r3, K, beta, num_cu, (char*)work, s, kt);
}

// ---- grid ------------------------------------------------------------------------
struct GridMixedPlan {
  int64_t kp;
  size_t o_mx, o_exps, o_a, o_b, total;
};

static GridMixedPlan plan_grid_mixed(int64_t n, int r3) {
  GridMixedPlan P{};
  P.kp = pad32(r3);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  };
  P.o_mx = take(4 * sizeof(unsigned long long));
  P.o_exps = take(2 * sizeof(int));
  P.o_a = take((size_t)3 * n * n * P.kp * 2);
  P.o_b = take((size_t)3 * n * P.kp * 2);
  P.total = off;
  return P;
}

size_t grid_mixed_workspace_bytes(int64_t n, int r3) { return plan_grid_mixed(n, r3).total; }

template <class SP, int BN, bool FOLD>
static void launch_grid_stream(const typename SP::T* ap, const typename SP::T* bp, int64_t M,
                               int64_t N, int64_t kp, float* grid, const int* exps, int num_cu,
                               hipStream_t s) {
  const int npanels = (int)((N + BN - 1) / BN);
  const int64_t tiles = (M + 127) / 128;
  // groups: a multiple of 8 (one XCD per group residue), one workgroup per CU
  // (the B panel and staging take most of the LDS)
  int gq = std::max(1, num_cu / (8 * npanels));
  while (gq > 1 && (int64_t)gq * 8 > tiles) --gq;
  const int groups = gq * 8;
  // padded B rows (kp + GRID_BPAD elements) and the per-wave staging tiles
  const size_t lds = (size_t)SP::TERMS * BN * (kp + GRID_BPAD) * sizeof(typename SP::T) +
                     (size_t)8 * 16 * (BN + 4) * sizeof(float);
  auto fn = grid_stream_kernel<SP, BN, FOLD>;
  if (lds > 48 * 1024)
    RS_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(fn, dim3((unsigned)(8 * npanels * gq)), dim3(512), lds, s, ap, bp, M, N,
                     (int)kp, npanels, groups, grid, exps);
}

// widest column panel whose B planes and staging fit the LDS budget
template <class SP>
static void grid_stream(const typename SP::T* ap, const typename SP::T* bp, int64_t M, int64_t N,
                        int64_t kp, float* grid, const int* exps, int num_cu, hipStream_t s) {
  const size_t budget = 150 * 1024;
  auto need = [&](int bn) {
    return (size_t)SP::TERMS * bn * (kp + GRID_BPAD) * 2 + (size_t)8 * 16 * (bn + 4) * 4;
  };
  const bool fold = kp > KCHUNK;
  if (need(128) <= budget && !fold) launch_grid_stream<SP, 128, false>(ap, bp, M, N, kp, grid, exps, num_cu, s);
  else if (need(64) <= budget) {
    if (fold) launch_grid_stream<SP, 64, true>(ap, bp, M, N, kp, grid, exps, num_cu, s);
    else launch_grid_stream<SP, 64, false>(ap, bp, M, N, kp, grid, exps, num_cu, s);
  } else if (need(32) <= budget) {
    launch_grid_stream<SP, 32, true>(ap, bp, M, N, kp, grid, exps, num_cu, s);
  } else {
    launch_grid_stream<SP, 16, true>(ap, bp, M, N, kp, grid, exps, num_cu, s);
  }
}

// exps[1] = 14 - ceil(log2(mx[1])) (0 for BF16 or a zero operand); exps[0]
// = *e0 when given, else kept
__global__ void b_exp_kernel(const unsigned long long* mx, int fp16, const int* e0, int* exps) {
  if (threadIdx.x != 0) return;
  const double b = __longlong_as_double((long long)mx[1]);
  exps[1] = fp16 && b > 0.0 ? 14 - (int)ceil(log2(b)) : 0;
  if (e0) exps[0] = e0[0];
}

template <class SP>
static void grid_mixed_t(int fp16, const double* T2, const double* V3, int64_t n, int r3,
                         float* grid, char* work, int num_cu, bool planes_ready, const int* t2exp,
                         hipStream_t s) {
  const GridMixedPlan P = plan_grid_mixed(n, r3);
  if (P.kp > 512) throw Error{RS_E_UNSUPPORTED, "mixed grid: Tucker rank above 512"};
  unsigned long long* mx = (unsigned long long*)(work + P.o_mx);
  int* exps = (int*)(work + P.o_exps);
  typename SP::T* ap = (typename SP::T*)(work + P.o_a);
  typename SP::T* bp = (typename SP::T*)(work + P.o_b);
  if (planes_ready || t2exp) {
    // T2's planes and exps[0] came with the second expansion, or T2 is
    // split here under the exponent that expansion chose
    RS_HIP(hipMemsetAsync(mx, 0, 4 * sizeof(unsigned long long), s));
    absmax(V3, n * r3, mx + 1, s);
    hipLaunchKernelGGL(b_exp_kernel, dim3(1), dim3(64), 0, s, mx, fp16, planes_ready ? nullptr : t2exp,
                       exps);
    if (!planes_ready) split_planes<SP>(T2, n * n, r3, r3, 1, P.kp, exps, 0, ap, s);
  } else {
    const double* Bops[1] = {V3};
    const int64_t nb[1] = {n * r3};
    scale_setup(T2, n * n * r3, Bops, nb, 1, fp16, mx, exps, s);
    split_planes<SP>(T2, n * n, r3, r3, 1, P.kp, exps, 0, ap, s);
  }
  split_planes<SP>(V3, n, r3, r3, 1, P.kp, exps, 1, bp, s);
  grid_stream<SP>(ap, bp, n * n, n, P.kp, grid, exps, num_cu, s);
}

// ---- projection ------------------------------------------------------------------
struct ProjMixedPlan {
  int64_t kp;
  size_t o_mx, o_exps, o_a, o_b, total;
};

static ProjMixedPlan plan_proj_mixed(int64_t n, int64_t K, int r, bool a_given) {
  ProjMixedPlan P{};
  P.kp = pad32(n);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  };
  P.o_mx = take(4 * sizeof(unsigned long long));
  P.o_exps = take(2 * sizeof(int));
  P.o_a = take(a_given ? 0 : (size_t)3 * K * P.kp * 2);   // up to 3 terms of 2 bytes
  P.o_b = take((size_t)3 * r * P.kp * 2);
  P.total = off;
  return P;
}

size_t proj_mixed_workspace_bytes(int64_t n, int64_t K, int r, bool a_given) {
  return plan_proj_mixed(n, K, r, a_given).total;
}

// mx[0] = 1.0 (the bound of a side-matrix entry) as an ordered bit pattern
__global__ void unit_max_kernel(unsigned long long* mx) {
  if (threadIdx.x == 0) mx[0] = (unsigned long long)__double_as_longlong(1.0);
}

template <class SP>
static void proj_mixed_t(int fp16, const double* U, const void* a_planes, int64_t n, int64_t K,
                         const double* V, int r, double* Ut, char* work, hipStream_t s) {
  const ProjMixedPlan P = plan_proj_mixed(n, K, r, a_planes != nullptr);
  unsigned long long* mx = (unsigned long long*)(work + P.o_mx);
  int* exps = (int*)(work + P.o_exps);
  typename SP::T* ap = (typename SP::T*)(work + P.o_a);
  typename SP::T* bp = (typename SP::T*)(work + P.o_b);
  const double* Bops[1] = {V};
  const int64_t nb[1] = {n * r};
  // A: row j = column j of U (n x K column-major); B: row a = column a of V (n x r row-major)
  if (a_planes) {
    // planes formed with the fixed scale 2^14 = 2^(14 - ceil(log2 1))
    RS_HIP(hipMemsetAsync(mx, 0, 4 * sizeof(unsigned long long), s));
    hipLaunchKernelGGL(unit_max_kernel, dim3(1), dim3(64), 0, s, mx);
    absmax(V, n * r, mx + 1, s);
    hipLaunchKernelGGL(scale_exponents_kernel, dim3(1), dim3(64), 0, s, mx, 1, fp16, exps);
    ap = (typename SP::T*)a_planes;
  } else {
    scale_setup(U, n * K, Bops, nb, 1, fp16, mx, exps, s);
    split_planes<SP>(U, K, n, n, 1, P.kp, exps, 0, ap, s);
  }
  split_planes<SP>(V, r, n, 1, r, P.kp, exps, 1, bp, s);
  constexpr int FN = SP::TERMS == 2 ? 4 : 2;
  constexpr int WGM = 4;
  const int64_t col_tiles = (r + 32 * FN - 1) / (32 * FN);
  const int64_t row_tiles = (K + 32 * WGM - 1) / (32 * WGM);
  hipLaunchKernelGGL((proj_tile_kernel<SP, WGM, FN>), dim3((unsigned)(row_tiles * col_tiles)),
                     dim3(128 * WGM), 0, s, ap, bp, K, (int64_t)r, P.kp, col_tiles, row_tiles, 0, Ut,
                     (int64_t)r, (int64_t)r, (int64_t)0, exps,
                     (typename GridSplitOf<SP>::type::T*)nullptr, (int64_t)0, (const int*)nullptr);
}

void proj_mixed(int prec, const double* U, const void* a_planes, int64_t n, int64_t K,
                const double* V, int r, double* Ut, void* work, hipStream_t s) {
  if (prec == RS_MIXED_BF16) {
    if (a_planes) throw Error{RS_E_INVALID, "split-BF16 projection from FP16 planes"};
    proj_mixed_t<SplitBF16>(0, U, nullptr, n, K, V, r, Ut, (char*)work, s);
  } else {
    proj_mixed_t<CoreF16>(1, U, a_planes, n, K, V, r, Ut, (char*)work, s);
  }
}

// ---- second expansion --------------------------------------------------------------
// T2[i1][i2][c] = sum_b V2[i2, b] X[b][i1][c] in split precision: A = V2
// (rows i2, b contiguous), B = X transposed to rows (i1, c) with b
// contiguous; the output's column (i1, c) goes to i1 n r3 + i2 r3 + c.
struct Expand2MixedPlan {
  int64_t kp;
  size_t o_mx, o_exps, o_a, o_b, total;
};

static Expand2MixedPlan plan_expand2_mixed(int64_t n, int r2, int r3) {
  Expand2MixedPlan P{};
  P.kp = pad32(r2);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  };
  P.o_mx = take(4 * sizeof(unsigned long long));
  P.o_exps = take(2 * sizeof(int));
  P.o_a = take((size_t)3 * n * P.kp * 2);
  P.o_b = take((size_t)3 * n * r3 * P.kp * 2);
  P.total = off;
  return P;
}

size_t expand2_mixed_workspace_bytes(int64_t n, int r2, int r3) {
  return plan_expand2_mixed(n, r2, r3).total;
}

// zero the padding columns r3 <= k < kp of the grid's A planes (rows n^2)
template <class GP>
__global__ void pad_planes_kernel(typename GP::T* __restrict__ planes, int64_t rows, int r3, int kp) {
  const int w = kp - r3;
  const int64_t total = rows * w;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = e / w;
    const int k = r3 + (int)(e - row * w);
#pragma unroll
    for (int term = 0; term < GP::TERMS; ++term) planes[(term * rows + row) * kp + k] = (typename GP::T)0.0f;
  }
}

// The grid's scale for T2 from a bound: |T2[i1, i2, c]| <= |V2[i2, :]|_2
// |X[:, i1, c]|_2 <= sqrt(r2) max|X| (the rows of the orthonormal V2 have
// norm at most 1), so gexps[0] = 14 - ceil(log2(sqrt(r2) max|X|)) keeps the
// scaled T2 below 2^14 (0 for the unscaled BF16 split).
__global__ void t2_bound_exp_kernel(const unsigned long long* mx_x, int r2, int fp16, int* t2exp,
                                    int* gexps) {
  if (threadIdx.x != 0) return;
  const double b = __longlong_as_double((long long)mx_x[0]) * sqrt((double)r2);
  const int e = fp16 && b > 0.0 ? 14 - (int)ceil(log2(b)) : 0;
  t2exp[0] = e;
  if (gexps) gexps[0] = e;
}

template <class SP>
static void expand2_mixed_t(int fp16, const double* X, const double* V2, int64_t n, int r2, int r3,
                            double* T2, char* work, char* gwork, int* t2exp, hipStream_t s) {
  const Expand2MixedPlan P = plan_expand2_mixed(n, r2, r3);
  unsigned long long* mx = (unsigned long long*)(work + P.o_mx);
  int* exps = (int*)(work + P.o_exps);
  typename SP::T* ap = (typename SP::T*)(work + P.o_a);
  typename SP::T* bp = (typename SP::T*)(work + P.o_b);
  const int64_t cols = n * r3;
  const double* Bops[1] = {X};
  const int64_t nb[1] = {(int64_t)r2 * cols};
  scale_setup(V2, n * r2, Bops, nb, 1, fp16, mx, exps, s);
  split_planes<SP>(V2, n, r2, r2, 1, P.kp, exps, 0, ap, s);
  hipLaunchKernelGGL(transpose_split_kernel<SP>,
                     dim3((unsigned)((P.kp + 63) / 64), (unsigned)((cols + 63) / 64)), dim3(256), 0,
                     s, X, (int64_t)r2, cols, P.kp, exps, 1, bp);
  // short contraction (r2): 64-row tiles, so that two workgroups share a
  // compute unit and one's loads and stores overlap the other's MFMAs
  constexpr int FN = SP::TERMS == 2 ? 4 : 2;
  constexpr int WGM = 2;
  const int64_t row_tiles = (n + 32 * WGM - 1) / (32 * WGM);
  const int64_t col_tiles = (cols + 32 * FN - 1) / (32 * FN);
  typedef typename GridSplitOf<SP>::type GP;
  typename GP::T* gp = nullptr;
  int* gexps = nullptr;
  int64_t gkp = 0;
  if (gwork) grid_mixed_planes(gwork, n, r3, (void**)&gp, &gexps, &gkp);
  hipLaunchKernelGGL(t2_bound_exp_kernel, dim3(1), dim3(64), 0, s, mx + 1, r2, fp16, t2exp, gexps);
  if (gwork) {
    // the grid's A planes of T2, written by the epilogue below
    if (gkp > r3)
      hipLaunchKernelGGL(pad_planes_kernel<GP>, dim3(grid_blocks(n * n * (gkp - r3))), dim3(256), 0, s,
                         gp, n * n, r3, (int)gkp);
  }
  hipLaunchKernelGGL((proj_tile_kernel<SP, WGM, FN>), dim3((unsigned)(row_tiles * col_tiles)),
                     dim3(128 * WGM), 0, s, ap, bp, n, cols, P.kp, col_tiles, row_tiles, 1, T2,
                     (int64_t)r3, (int64_t)r3, n * r3, exps, gp, gkp, (const int*)gexps);
}

void expand2_mixed(int prec, const double* X, const double* V2, int64_t n, int r2, int r3,
                   double* T2, void* work, void* grid_work, int* t2exp, hipStream_t s) {
  if (prec == RS_MIXED_BF16)
    expand2_mixed_t<SplitBF16>(0, X, V2, n, r2, r3, T2, (char*)work, (char*)grid_work, t2exp, s);
  else
    expand2_mixed_t<CoreF16>(1, X, V2, n, r2, r3, T2, (char*)work, (char*)grid_work, t2exp, s);
}

void grid_mixed(int prec, const double* T2, const double* V3, int64_t n, int r3, float* grid,
                void* work, int num_cu, hipStream_t s, bool planes_ready, const int* t2exp) {
  if (prec == RS_MIXED_FP16)
    grid_mixed_t<SplitF16>(1, T2, V3, n, r3, grid, (char*)work, num_cu, planes_ready, t2exp, s);
  else
    grid_mixed_t<SplitBF16>(0, T2, V3, n, r3, grid, (char*)work, num_cu, planes_ready, t2exp, s);
}

void grid_mixed_planes(void* work, int64_t n, int r3, void** planes, int** exps, int64_t* kp) {
  const GridMixedPlan P = plan_grid_mixed(n, r3);
  *planes = (char*)work + P.o_a;
  *exps = (int*)((char*)work + P.o_exps);
  *kp = P.kp;
}

}  // namespace rs
