// Split-precision contractions for the mixed path (core and grid expansion).
//
// Each FP64 operand value is split while it is staged into LDS:
//  FP16: x 2^s = hi + lo 2^-11 (hi, lo FP16), |x 2^s| <= 2^14 by a power-of-two
//        scale from the operand's max |x|; three products hi*hi, hi*lo, lo*hi.
//  BF16: x = hi + mid + lo (BF16 of the successive residuals); six products
//        down to the 2^-16 level (hh, hm, mh, hl, lh, mm).
// The products run on v_mfma_f32_16x16x32_{f16,bf16} with FP32 accumulation,
// one accumulator per magnitude level, folded into FP64 registers every
// KCHUNK values of k (FP64 sums across K chunks).  Output is FP64 (core, then
// split-K partials summed in a fixed order) or FP32 (the grid).
#include "rs_internal.h"

namespace rs {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int XBM = 64, XBN = 64, XBK = 32, XLDK = 40;  // LDS row of 32 halves, padded
constexpr int KCHUNK = 256;

struct SplitF16 {
  static constexpr int TERMS = 2;
  static constexpr int LEVELS = 2;
  typedef _Float16 T;
  typedef h8 V8;
  __device__ static void split(double x, T* o) {
    const T hi = (T)x;
    o[0] = hi;
    o[1] = (T)((x - (double)hi) * 2048.0);
  }
  __device__ static f4 mfma(V8 a, V8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
  // level 0: hi*hi; level 1: hi*lo + lo*hi (weight 2^-11)
  __device__ static void products(const V8 (&a)[TERMS], const V8 (&b)[TERMS], f4 (&acc)[LEVELS]) {
    acc[0] = mfma(a[0], b[0], acc[0]);
    acc[1] = mfma(a[0], b[1], acc[1]);
    acc[1] = mfma(a[1], b[0], acc[1]);
  }
  __device__ static double combine(const f4 (&acc)[LEVELS], int v) {
    return (double)acc[0][v] + (double)acc[1][v] * (1.0 / 2048.0);
  }
};

struct SplitBF16 {
  static constexpr int TERMS = 3;
  static constexpr int LEVELS = 3;
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
  __device__ static f4 mfma(V8 a, V8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  __device__ static void products(const V8 (&a)[TERMS], const V8 (&b)[TERMS], f4 (&acc)[LEVELS]) {
    acc[0] = mfma(a[0], b[0], acc[0]);
    acc[1] = mfma(a[0], b[1], acc[1]);
    acc[1] = mfma(a[1], b[0], acc[1]);
    acc[2] = mfma(a[0], b[2], acc[2]);
    acc[2] = mfma(a[2], b[0], acc[2]);
    acc[2] = mfma(a[1], b[1], acc[2]);
  }
  __device__ static double combine(const f4 (&acc)[LEVELS], int v) {
    return (double)acc[0][v] + (double)acc[1][v] + (double)acc[2][v];
  }
};

// ---- FP64 operand sources for a 64 (wide) x 32 (k) slab, 8 values per thread ----
// K-contiguous storage: element (w, k) at P[w * s_w + k].
struct KContigSrc {
  const double* P;
  int64_t s_w, W;
  static constexpr bool KVEC = true;   // the 8 values of a thread run along k
  __device__ __forceinline__ void load(int64_t w0, int64_t k0, int64_t kend, double (&v)[8], int tid,
                                       int& wl, int& kl) const {
    wl = tid >> 2;
    kl = (tid & 3) * 8;
    const int64_t w = w0 + wl;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int64_t k = k0 + kl + t;
      v[t] = (w < W && k < kend) ? P[w * s_w + k] : 0.0;
    }
  }
};

// Wide-contiguous storage: element (w, k) at P[k * s_k + w].
struct WContigSrc {
  const double* P;
  int64_t s_k, W;
  static constexpr bool KVEC = false;  // the 8 values of a thread run along w
  __device__ __forceinline__ void load(int64_t w0, int64_t k0, int64_t kend, double (&v)[8], int tid,
                                       int& wl, int& kl) const {
    kl = tid >> 3;
    wl = (tid & 7) * 8;
    const int64_t k = k0 + kl;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int64_t w = w0 + wl + t;
      v[t] = (w < W && k < kend) ? P[k * s_k + w] : 0.0;
    }
  }
};

// Khatri-Rao operand of the core: (w = b r3 + c, k = j) -> xi_j U2t[j r2 + b] U3t[j r3 + c]
struct KRSrc {
  const double* U2t;
  const double* U3t;
  const double* xi;
  int r2, r3;
  static constexpr bool KVEC = false;
  __device__ __forceinline__ void load(int64_t w0, int64_t k0, int64_t kend, double (&v)[8], int tid,
                                       int& wl, int& kl) const {
    kl = tid >> 3;
    wl = (tid & 7) * 8;
    const int64_t k = k0 + kl;
    const int64_t W = (int64_t)r2 * r3;
    int64_t bc = w0 + wl;
    int b = (int)(bc / r3), c = (int)(bc - (int64_t)(bc / r3) * r3);
    const bool kin = k < kend;
    const double xk = kin ? xi[k] : 0.0;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      v[t] = (kin && bc + t < W) ? xk * U2t[k * r2 + b] * U3t[k * r3 + c] : 0.0;
      if (++c == r3) {
        c = 0;
        ++b;
      }
    }
  }
};

template <class SP, class Src>
__device__ __forceinline__ void stage(const Src& src, typename SP::T* lds, int64_t w0, int64_t k0,
                                      int64_t kend, double scale, int tid) {
  double v[8];
  int wl, kl;
  src.load(w0, k0, kend, v, tid, wl, kl);
  typename SP::T parts[8][SP::TERMS];
#pragma unroll
  for (int t = 0; t < 8; ++t) SP::split(v[t] * scale, parts[t]);
  // lds layout: [term][w][k] with row stride XLDK halves
#pragma unroll
  for (int term = 0; term < SP::TERMS; ++term) {
    typename SP::T* base = lds + term * (XBM * XLDK);
    if (Src::KVEC) {
#pragma unroll
      for (int t = 0; t < 8; ++t) base[wl * XLDK + kl + t] = parts[t][term];
    } else {
#pragma unroll
      for (int t = 0; t < 8; ++t) base[(wl + t) * XLDK + kl] = parts[t][term];
    }
  }
}

struct MixedOut {
  int64_t M, N;
  double* C64;      // FP64 output (row-major with scm, scn) or split-K partial base
  float* C32;       // FP32 output (nontemporal), when C64 is null
  int64_t scm, scn;
};

template <class SP, class ASrc, class BSrc>
__device__ __forceinline__ void mixed_tile(const ASrc& as, const BSrc& bs, int64_t m0, int64_t n0,
                                           int64_t kbeg, int64_t kend, double sa, double sb,
                                           double out_scale, const MixedOut& o) {
  typedef typename SP::T T;
  typedef typename SP::V8 V8;
  __shared__ __attribute__((aligned(16))) T Al[SP::TERMS * XBM * XLDK];
  __shared__ __attribute__((aligned(16))) T Bl[SP::TERMS * XBN * XLDK];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  double acc64[2][2][4];
  f4 acc[2][2][SP::LEVELS];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
#pragma unroll
      for (int v = 0; v < 4; ++v) acc64[i][j][v] = 0.0;
#pragma unroll
      for (int l = 0; l < SP::LEVELS; ++l) acc[i][j][l] = f4{0.f, 0.f, 0.f, 0.f};
    }

  int since_fold = 0;
  for (int64_t k0 = kbeg; k0 < kend; k0 += XBK) {
    __syncthreads();
    stage<SP>(as, Al, m0, k0, kend, sa, tid);
    stage<SP>(bs, Bl, n0, k0, kend, sb, tid);
    __syncthreads();
    V8 a[2][SP::TERMS], b[2][SP::TERMS];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int term = 0; term < SP::TERMS; ++term) {
        a[i][term] = *(const V8*)(Al + term * XBM * XLDK + (wm * 32 + i * 16 + (lane & 15)) * XLDK +
                                   8 * (lane >> 4));
        b[i][term] = *(const V8*)(Bl + term * XBN * XLDK + (wn * 32 + i * 16 + (lane & 15)) * XLDK +
                                   8 * (lane >> 4));
      }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) SP::products(a[i], b[j], acc[i][j]);
    since_fold += XBK;
    if (since_fold >= KCHUNK || k0 + XBK >= kend) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
#pragma unroll
          for (int v = 0; v < 4; ++v) acc64[i][j][v] += SP::combine(acc[i][j], v);
#pragma unroll
          for (int l = 0; l < SP::LEVELS; ++l) acc[i][j][l] = f4{0.f, 0.f, 0.f, 0.f};
        }
      since_fold = 0;
    }
  }
  // epilogue: for the 16 x 16 f32 MFMAs lane holds D[4 (lane/16) + v][lane % 16]
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t col = n0 + wn * 32 + j * 16 + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + v;
        if (row < o.M && col < o.N) {
          const double val = acc64[i][j][v] * out_scale;
          if (o.C64) o.C64[row * o.scm + col * o.scn] = val;
          else __builtin_nontemporal_store((float)val, o.C32 + row * o.scm + col * o.scn);
        }
      }
    }
}

// 2^s from the exponent table written by the absmax kernels
__device__ __forceinline__ double pow2(int s) { return ldexp(1.0, s); }

template <class SP>
__global__ __launch_bounds__(256) void core_mixed_kernel(const double* U1t, KRSrc kr, int r1,
                                                         int64_t K, int64_t kchunk, int tiles_n,
                                                         double* beta, double* part,
                                                         const int* exps) {
  const int tile = blockIdx.x;
  const int tm = tile / tiles_n, tn = tile - tm * tiles_n;
  const int split = blockIdx.z;
  const int64_t kbeg = (int64_t)split * kchunk;
  int64_t kend = kbeg + kchunk;
  if (kend > K) kend = K;
  const int64_t W = (int64_t)kr.r2 * kr.r3;
  WContigSrc as{U1t, r1, r1};
  MixedOut o;
  o.M = r1;
  o.N = W;
  o.C64 = part ? part + (int64_t)split * r1 * W : beta;
  o.C32 = nullptr;
  o.scm = W;
  o.scn = 1;
  const int sa = exps ? exps[0] : 0, sb = exps ? exps[1] : 0;
  mixed_tile<SP>(as, kr, (int64_t)tm * XBM, (int64_t)tn * XBN, kbeg, kend, pow2(sa), pow2(sb),
                 pow2(-sa - sb), o);
}

// grid[(i1 i2), i3] (FP32) = sum_c T2[(i1 i2), c] V3[i3, c]
template <class SP>
__global__ __launch_bounds__(256) void grid_mixed_kernel(const double* T2, const double* V3,
                                                         int64_t n, int r3, int tiles_n,
                                                         float* grid, const int* exps) {
  const int64_t tile = blockIdx.x;
  const int64_t tm = tile / tiles_n, tn = tile - tm * tiles_n;
  KContigSrc as{T2, r3, n * n};
  KContigSrc bs{V3, r3, n};
  MixedOut o;
  o.M = n * n;
  o.N = n;
  o.C64 = nullptr;
  o.C32 = grid;
  o.scm = n;
  o.scn = 1;
  const int sa = exps ? exps[0] : 0, sb = exps ? exps[1] : 0;
  mixed_tile<SP>(as, bs, tm * XBM, tn * XBN, 0, r3, pow2(sa), pow2(sb), pow2(-sa - sb), o);
}

// ---- max |x| of FP64 arrays as ordered bit patterns (deterministic) ----------
__global__ void absmax_kernel(const double* __restrict__ x, int64_t count,
                              unsigned long long* __restrict__ out) {
  double m = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double v = fabs(x[e]);
    if (v > m) m = v;
  }
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0 && m > 0.0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
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
  unsigned blocks = (unsigned)std::min<int64_t>((count + 255) / 256, 2048);
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(absmax_kernel, dim3(blocks), dim3(256), 0, s, x, count, out);
}

static void scale_setup(const double* A, int64_t na, const double* const* B, const int64_t* nb,
                        int nbops, int fp16, unsigned long long* mx, int* exps, hipStream_t s) {
  RS_HIP(hipMemsetAsync(mx, 0, 4 * sizeof(unsigned long long), s));
  absmax(A, na, mx, s);
  for (int i = 0; i < nbops; ++i) absmax(B[i], nb[i], mx + 1 + i, s);
  hipLaunchKernelGGL(scale_exponents_kernel, dim3(1), dim3(64), 0, s, mx, nbops, fp16, exps);
}

size_t core_mixed_workspace_bytes(int r1, int r2, int r3, int64_t K, int num_cu) {
  const int tm = (r1 + XBM - 1) / XBM;
  const int64_t tn = ((int64_t)r2 * r3 + XBN - 1) / XBN;
  const int64_t tiles = tm * tn;
  int splits = 1;
  if (tiles < 2LL * num_cu && K > 4 * KCHUNK)
    splits = (int)std::min<int64_t>((2LL * num_cu + tiles - 1) / tiles,
                                    std::min<int64_t>(K / (2 * KCHUNK), 64));
  if (splits < 1) splits = 1;
  return (splits > 1 ? (size_t)splits * r1 * r2 * r3 * sizeof(double) : 0) + 64;
}

void core_mixed(int prec, const double* U1t, const double* U2t, const double* U3t, const double* xi,
                int r1, int r2, int r3, int64_t K, double* beta, int num_cu, double* work,
                hipStream_t s) {
  const int tm = (r1 + XBM - 1) / XBM;
  const int tn = (int)(((int64_t)r2 * r3 + XBN - 1) / XBN);
  const int64_t tiles = (int64_t)tm * tn;
  int splits = 1;
  if (tiles < 2LL * num_cu && K > 4 * KCHUNK)
    splits = (int)std::min<int64_t>((2LL * num_cu + tiles - 1) / tiles,
                                    std::min<int64_t>(K / (2 * KCHUNK), 64));
  if (splits < 1) splits = 1;
  int64_t kchunk = (K + splits - 1) / splits;
  kchunk = (kchunk + KCHUNK - 1) / KCHUNK * KCHUNK;
  splits = (int)((K + kchunk - 1) / kchunk);
  const size_t part_bytes = splits > 1 ? (size_t)splits * r1 * r2 * r3 * sizeof(double) : 0;
  double* part = splits > 1 ? work : nullptr;
  // scale exponents after the partial buffer (64 bytes reserved)
  unsigned long long* mx = (unsigned long long*)((char*)work + part_bytes);
  DevBuf ex(2 * sizeof(int), s);
  const double* Bops[3] = {xi, U2t, U3t};
  const int64_t nb[3] = {K, K * r2, K * r3};
  scale_setup(U1t, K * r1, Bops, nb, 3, prec == RS_MIXED_FP16, mx, ex.as<int>(), s);
  KRSrc kr{U2t, U3t, xi, r2, r3};
  dim3 grid((unsigned)tiles, 1, (unsigned)splits);
  if (prec == RS_MIXED_FP16)
    hipLaunchKernelGGL(core_mixed_kernel<SplitF16>, grid, dim3(256), 0, s, U1t, kr, r1, K, kchunk,
                       tn, beta, part, ex.as<int>());
  else
    hipLaunchKernelGGL(core_mixed_kernel<SplitBF16>, grid, dim3(256), 0, s, U1t, kr, r1, K, kchunk,
                       tn, beta, part, ex.as<int>());
  if (splits > 1) core64_reduce(part, splits, (int64_t)r1 * r2 * r3, beta, s);
}

void grid_mixed(int prec, const double* T2, const double* V3, int64_t n, int r3, float* grid,
                hipStream_t s) {
  DevBuf mxb(4 * sizeof(unsigned long long), s);
  DevBuf ex(2 * sizeof(int), s);
  const double* Bops[1] = {V3};
  const int64_t nb[1] = {n * r3};
  scale_setup(T2, n * n * r3, Bops, nb, 1, prec == RS_MIXED_FP16, mxb.as<unsigned long long>(),
              ex.as<int>(), s);
  const int tn = (int)((n + XBN - 1) / XBN);
  const int64_t tiles = ((n * n + XBM - 1) / XBM) * tn;
  if (prec == RS_MIXED_FP16)
    hipLaunchKernelGGL(grid_mixed_kernel<SplitF16>, dim3((unsigned)tiles), dim3(256), 0, s, T2, V3, n,
                       r3, tn, grid, ex.as<int>());
  else
    hipLaunchKernelGGL(grid_mixed_kernel<SplitBF16>, dim3((unsigned)tiles), dim3(256), 0, s, T2, V3,
                       n, r3, tn, grid, ex.as<int>());
}

}  // namespace rs
