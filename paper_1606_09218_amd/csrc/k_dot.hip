// Scalar product of two RS tensors on one grid (section 3.4, item (d)):
//   <A, B> = sum_i A(i) B(i) = <A_l, B_l> + sum_{i in W} (A(i) B(i) - A_l(i) B_l(i)),
// W = the cells some short-range window of A or of B touches: outside every
// window a tensor equals its long-range Tucker part.  <A_l, B_l> is formed
// from the Tucker factors by the host (small GEMMs); this file holds the
// correction over the touched bricks and the fixed-order reductions.
#include "rs_internal.h"

namespace rs {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double dot_readlane(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double dot_wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);   // same tree on every call
  return v;
}

// Wave-scope barrier for LDS data exchanged between the lanes of one wave
// (the waves of a workgroup run different trip counts here).
__device__ __forceinline__ void dot_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Short-range values of one tensor at the cells (bs0 + m, bs1 + c1, bs2 + c2),
// m = 0..7, of this lane (c1 = lane / 8, c2 = lane % 8): the windowed terms
// z_nu sum_{k >= R_l} a_k g g g of the particles listed for brick `br` (the
// same sum the grid's short gather adds).  Run by one wave; f: its LDS table
// [3][Rs][8] of 1D factors, ak / tk2: LDS [Rs] weights and squared exponents.
__device__ void dot_side_short(const DotSide& S, int br, int64_t n, double b, const int bs[3],
                               double* f, const double* ak, const double* tk2,
                               double (&out)[8]) {
  const int lane = threadIdx.x & 63;
  const int c1 = lane >> 3, c2 = lane & 7;
  const int Rs = S.R - S.R_l;
#pragma unroll
  for (int m = 0; m < 8; ++m) out[m] = 0.0;
  if (Rs <= 0) return;
  const double h = 2.0 * b / (double)n;
  const int s0 = S.start[br], s1 = S.start[br + 1];
  for (int e0 = s0; e0 < s1; e0 += 64) {
    const int cnt = s1 - e0 < 64 ? s1 - e0 : 64;
    const int mynu = lane < cnt ? S.list[e0 + lane] : S.list[e0];
    const double px = S.pos[3 * (int64_t)mynu], py = S.pos[3 * (int64_t)mynu + 1],
                 pz = S.pos[3 * (int64_t)mynu + 2], pq = S.q[mynu];
    for (int e = 0; e < cnt; ++e) {
      const double p[3] = {dot_readlane(px, e), dot_readlane(py, e), dot_readlane(pz, e)};
      const double z = dot_readlane(pq, e);
      int lo[3], hi[3];
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        int64_t jc = (int64_t)floor((p[l] + b) / h);
        jc = jc < 0 ? 0 : (jc > n - 1 ? n - 1 : jc);
        const int64_t glo = jc - S.w < 0 ? 0 : jc - S.w;
        const int64_t ghi = jc + S.w > n - 1 ? n - 1 : jc + S.w;
        lo[l] = (int)(glo - bs[l]);
        hi[l] = (int)(ghi - bs[l]);
      }
      dot_wave_sync();   // the previous particle's table has been read
      for (int idx = lane; idx < 24 * Rs; idx += 64) {
        const int l = idx / (8 * Rs);
        const int rem = idx - l * 8 * Rs;
        const int k = rem >> 3, m = rem & 7;
        const double d = (-b + ((double)(bs[l] + m) + 0.5) * h) - p[l];
        f[idx] = exp(-tk2[k] * (d * d));
      }
      dot_wave_sync();
      if (c1 >= lo[1] && c1 <= hi[1] && c2 >= lo[2] && c2 <= hi[2]) {
        double sm[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) sm[m] = 0.0;
        for (int k = 0; k < Rs; ++k) {
          const double g = ak[k] * f[(Rs + k) * 8 + c1] * f[(2 * Rs + k) * 8 + c2];
#pragma unroll
          for (int m = 0; m < 8; ++m) sm[m] += g * f[k * 8 + m];
        }
#pragma unroll
        for (int m = 0; m < 8; ++m)
          if (m >= lo[0] && m <= hi[0]) out[m] += z * sm[m];
      }
    }
  }
  dot_wave_sync();   // the table is free for the next brick
}

// ---- the touched-cell correction, one workgroup per brick column ---------------
// Workgroup (b0, b1) lists the bricks b2 of its column that a window of A or
// of B touches (in increasing b2) and takes them in groups of DG.  For a
// group, wave j forms the short-range values of A and B on brick j (LDS sv),
// then the four waves contract the long parts on the matrix cores:
//   L[rho][kappa] = sum_c T2[(i0 n + i1) r3 + c] V3[i2 r3 + c],
// rho = 8 (i0 - 8 b0) + (i1 - 8 b1) (64 rows), kappa = 8 j + (i2 - 8 b2_j)
// (32 columns), T2 and V3 chunks of DKC values staged through LDS (double
// buffered); wave w holds rows 16w..16w+15 as two 16 x 16 blocks of
// v_mfma_f64_16x16x4f64.  Each lane then adds L_A S_B + S_A L_B + S_A S_B
// over its 8 cells.  partials[column] is the column's sum, formed in a fixed
// order (the same tree on every call).
constexpr int DG = 4;           // bricks per group
constexpr int DKC = 16;         // k values per LDS chunk
constexpr int DLA = DKC + 1;    // padded LDS row of a chunk (doubles)

__device__ __forceinline__ void dot_long(const DotSide& S, int64_t n, int bs0, int bs1,
                                         const int* b2g, int gc, double* as, double* bsm,
                                         d4 (&acc)[2]) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int K = S.r3;
  acc[0] = d4{0.0, 0.0, 0.0, 0.0};
  acc[1] = d4{0.0, 0.0, 0.0, 0.0};
  // loader of thread tid: T2 row tid / 4 (4 values), V3 row tid / 8 (2 values)
  const int ra = tid >> 2, ka = (tid & 3) * 4;
  int64_t i0 = bs0 + (ra >> 3), i1 = bs1 + (ra & 7);
  i0 = i0 < n ? i0 : n - 1;
  i1 = i1 < n ? i1 : n - 1;
  const double* pa = S.T2 + (i0 * n + i1) * K;
  const int rb = tid >> 3, kb = (tid & 7) * 2;
  const int jb = (rb >> 3) < gc ? (rb >> 3) : gc - 1;
  int64_t i2 = 8 * (int64_t)b2g[jb] + (rb & 7);
  i2 = i2 < n ? i2 : n - 1;
  const double* pb = S.V3 + i2 * K;
  double va[4], vb[2];
  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = k0 + ka + e;
      const double v = pa[k < K ? k : K - 1];
      va[e] = k < K ? v : 0.0;
    }
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int k = k0 + kb + e;
      const double v = pb[k < K ? k : K - 1];
      vb[e] = k < K ? v : 0.0;
    }
  };
  auto store = [&](int buf) {
    double* a = as + buf * 64 * DLA + ra * DLA + ka;
#pragma unroll
    for (int e = 0; e < 4; ++e) a[e] = va[e];
    double* bq = bsm + buf * 32 * DLA + rb * DLA + kb;
#pragma unroll
    for (int e = 0; e < 2; ++e) bq[e] = vb[e];
  };
  const int nch = (K + DKC - 1) / DKC;
  load(0);
  store(0);
  __syncthreads();
  int buf = 0;
  for (int ch = 0; ch < nch; ++ch) {
    const bool more = ch + 1 < nch;
    if (more) load((ch + 1) * DKC);
    const double* a = as + buf * 64 * DLA + (16 * wave + (lane & 15)) * DLA;
    const double* b0 = bsm + buf * 32 * DLA + (lane & 15) * DLA;
    const double* b1 = b0 + 16 * DLA;
#pragma unroll
    for (int kk = 0; kk < DKC; kk += 4) {
      const int kr = kk + (lane >> 4);
      const double fa = a[kr];
      acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa, b0[kr], acc[0], 0, 0, 0);
      acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa, b1[kr], acc[1], 0, 0, 0);
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
}

__global__ __launch_bounds__(256) void dot_cols_kernel(DotSide A, DotSide B, int nb, int64_t n,
                                                       double b, int rs_max,
                                                       double* __restrict__ partials) {
  extern __shared__ double dlds[];
  double* sv = dlds;                        // [2][DG][512] short values of A and B
  double* as = sv + 2 * DG * 512;           // [2][64][DLA]
  double* bsm = as + 2 * 64 * DLA;          // [2][32][DLA]
  double* ftab = bsm + 2 * 32 * DLA;        // [4][24 rs_max]
  double* akA = ftab + 4 * 24 * rs_max;     // [rs_max] x 4: akA, tkA, akB, tkB
  double* tkA = akA + rs_max;
  double* akB = tkA + rs_max;
  double* tkB = akB + rs_max;
  double* wsum = tkB + rs_max;              // [4]
  int* wcnt = (int*)(wsum + 4);             // [4]
  int* blist = wcnt + 4;                    // [nb]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = blockIdx.x;
  const int b0 = col / nb, b1 = col - (col / nb) * nb;
  const int64_t cbase = ((int64_t)b0 * nb + b1) * nb;
  // the touched bricks of the column, in increasing b2
  int total = 0;
  for (int base = 0; base < nb; base += 256) {
    const int b2 = base + tid;
    bool touched = false;
    if (b2 < nb) {
      const int64_t br = cbase + b2;
      touched = A.start[br + 1] > A.start[br] || B.start[br + 1] > B.start[br];
    }
    const unsigned long long m = __ballot(touched);
    if (lane == 0) wcnt[wave] = __popcll(m);
    __syncthreads();
    int off = total;
    for (int w = 0; w < wave; ++w) off += wcnt[w];
    if (touched) blist[off + __popcll(m & ((1ull << lane) - 1ull))] = b2;
    total += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    __syncthreads();
  }
  if (total == 0) {
    if (tid == 0) partials[col] = 0.0;
    return;
  }
  const int RsA = A.R - A.R_l, RsB = B.R - B.R_l;
  for (int k = tid; k < RsA; k += 256) {
    akA[k] = A.a[A.R_l + k];
    tkA[k] = A.t[A.R_l + k] * A.t[A.R_l + k];
  }
  for (int k = tid; k < RsB; k += 256) {
    akB[k] = B.a[B.R_l + k];
    tkB[k] = B.t[B.R_l + k] * B.t[B.R_l + k];
  }
  __syncthreads();
  const int bs0 = 8 * b0, bs1 = 8 * b1;
  double* fw = ftab + wave * 24 * rs_max;
  double wacc = 0.0;
  for (int g0 = 0; g0 < total; g0 += DG) {
    const int gc = total - g0 < DG ? total - g0 : DG;
    const int* b2g = blist + g0;
    if (wave < gc) {
      const int br = (int)(cbase + b2g[wave]);
      const int bs[3] = {bs0, bs1, 8 * b2g[wave]};
      double o[8];
      dot_side_short(A, br, n, b, bs, fw, akA, tkA, o);
#pragma unroll
      for (int m = 0; m < 8; ++m) sv[wave * 512 + m * 64 + lane] = o[m];
      dot_side_short(B, br, n, b, bs, fw, akB, tkB, o);
#pragma unroll
      for (int m = 0; m < 8; ++m) sv[(DG + wave) * 512 + m * 64 + lane] = o[m];
    }
    d4 la[2], lb[2];
    dot_long(A, n, bs0, bs1, b2g, gc, as, bsm, la);   // its first barrier publishes sv
    dot_long(B, n, bs0, bs1, b2g, gc, as, bsm, lb);
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
      const int kap = 16 * blk + (lane & 15);
      const int j = kap >> 3, c2 = kap & 7;
      const bool colok = j < gc && 8 * (int64_t)b2g[j < gc ? j : 0] + c2 < n;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rho = 16 * wave + (lane >> 4) + 4 * v;
        const bool ok = colok && bs0 + (rho >> 3) < n && bs1 + (rho & 7) < n;
        if (ok) {
          const double sa = sv[j * 512 + rho * 8 + c2], sb = sv[(DG + j) * 512 + rho * 8 + c2];
          wacc += la[blk][v] * sb + sa * lb[blk][v] + sa * sb;
        }
      }
    }
    __syncthreads();   // sv is rewritten by the next group
  }
  wacc = dot_wave_sum(wacc);
  if (lane == 0) wsum[wave] = wacc;
  __syncthreads();
  if (tid == 0) partials[col] = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
}

// partial[blk] = sum over the fixed stride class of x[i] y[i]; one value per block
constexpr int DOT_THREADS = 256, DOT_BLOCKS = 1024;
__global__ __launch_bounds__(DOT_THREADS) void dot_partial_kernel(const double* __restrict__ x,
                                                                  const double* __restrict__ y,
                                                                  int64_t count,
                                                                  double* __restrict__ partial) {
  __shared__ double red[DOT_THREADS];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * DOT_THREADS + threadIdx.x; i < count;
       i += (int64_t)DOT_BLOCKS * DOT_THREADS)
    s += x[i] * y[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = DOT_THREADS / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// out = sum of the DOT_BLOCKS long-long partials + the ncols column partials
// of the correction (fixed order)
__global__ __launch_bounds__(1024) void dot_final_kernel(const double* __restrict__ ll,
                                                         const double* __restrict__ pc,
                                                         int64_t ncols, double* __restrict__ out) {
  __shared__ double red[1024];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < DOT_BLOCKS; i += 1024) s += ll[i];
  for (int64_t i = threadIdx.x; i < ncols; i += 1024) s += pc[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

size_t dot_partials_bytes() { return (size_t)DOT_BLOCKS * sizeof(double); }

void launch_dot_partial(const double* x, const double* y, int64_t count, double* partial,
                        hipStream_t s) {
  hipLaunchKernelGGL(dot_partial_kernel, dim3(DOT_BLOCKS), dim3(DOT_THREADS), 0, s, x, y, count,
                     partial);
}

void launch_dot_cols(const DotSide& A, const DotSide& B, int nb, int64_t n, double b,
                     double* partials, hipStream_t s) {
  const int rs_max = std::max(std::max(A.R - A.R_l, B.R - B.R_l), 1);
  if (rs_max > 64) throw Error{RS_E_UNSUPPORTED, "more than 64 short-range terms"};
  if (A.r3 < 1 || B.r3 < 1) throw Error{RS_E_INVALID, "scalar product: empty Tucker rank"};
  const size_t lds = sizeof(double) * ((size_t)2 * DG * 512 + 2 * 64 * DLA + 2 * 32 * DLA +
                                       (size_t)4 * 24 * rs_max + 4 * (size_t)rs_max + 4) +
                     sizeof(int) * (4 + (size_t)nb);
  if (lds > 160 * 1024) throw Error{RS_E_UNSUPPORTED, "scalar product: grid too large for one column"};
  if (lds > 64 * 1024)
    RS_HIP(hipFuncSetAttribute((const void*)dot_cols_kernel,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  const int64_t ncols = (int64_t)nb * nb;
  hipLaunchKernelGGL(dot_cols_kernel, dim3((unsigned)ncols), dim3(256), lds, s, A, B, nb, n, b,
                     rs_max, partials);
}

void launch_dot_final(const double* ll, const double* pc, int64_t ncols, double* out,
                      hipStream_t s) {
  hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(1024), 0, s, ll, pc, ncols, out);
}

}  // namespace rs
