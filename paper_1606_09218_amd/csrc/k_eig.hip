// FP64 dominant-eigenspace solver for the charge-weighted Gram matrices.
//
// The RHOSVD keeps the dominant left singular vectors of each side matrix
// (Appendix step (I), eq SVD_SideMatr).  They are the dominant eigenvectors
// of G_l = U_l diag(w) U_l^T.  With a rapidly decaying spectrum a subspace
// of p = r + oversample columns captures them:
//   Y = U_l diag(|xi|^{1/3}) Omega, Q = orth(Y), [Y = G Q, Q = orth(Y)]^q, B = Q^T G Q,
//   B = W Lambda W^T (tridiagonalisation, bisection, inverse iteration), V = Q W.
// The subspace comes from a sketch of the charge-weighted side matrix (the
// range finder of Halko, Martinsson and Tropp) orthonormalised by shifted
// Cholesky QR.  Everything is FP64.  Each small kernel runs one workgroup per
// mode.
#include <hip/hip_cooperative_groups.h>

#include "rs_internal.h"

namespace rs {

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ULL;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
  return x ^ (x >> 31);
}

// uniform in [-1, 1), from a counter
__device__ __forceinline__ double hash_uniform(uint64_t seed, uint64_t i, uint64_t j) {
  uint64_t h = splitmix64(seed ^ splitmix64(i * 0x100000001B3ULL + j));
  return (double)(h >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ void identity_kernel(double* I, int64_t n) {
  const int mode = blockIdx.y;
  const int64_t total = n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x)
    I[mode * total + e] = (e / n == e % n) ? 1.0 : 0.0;
}

void launch_identity(double* I, int64_t n, int modes, hipStream_t s) {
  int64_t total = n * n;
  unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(identity_kernel, dim3(blocks, modes), dim3(256), 0, s, I, n);
}

// ---- block reductions (fixed order: wave shuffle tree, then waves in order) --
constexpr int EIG_THREADS = 512;
constexpr int EIG_WAVES = EIG_THREADS / 64;

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < EIG_WAVES; ++w) s += red[w];
  return s;
}

// Cross-lane sums on the data-parallel-primitive (DPP) path: a row of 16
// lanes is reduced with quad_perm (xor 1, xor 2), row_half_mirror and
// row_mirror moves, rows are combined with readlane.  Every stage adds
// symmetric pairs, so all lanes end with bitwise-identical sums.
template <int CTRL>
__device__ __forceinline__ double dpp_mov_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// sum over the 16 lanes of each row (all lanes of the row receive it)
__device__ __forceinline__ double row_sum16(double v) {
  v += dpp_mov_f64<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_mov_f64<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_mov_f64<0x141>(v);   // row_half_mirror
  v += dpp_mov_f64<0x140>(v);   // row_mirror
  return v;
}

__device__ __forceinline__ double lane_f64(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// sum over the whole wave (uniform result)
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v = row_sum16(v);
  return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}

__global__ void symmetrize_kernel(double* B, int p) {
  double* Bm = B + (int64_t)blockIdx.y * p * p;
  int64_t total = (int64_t)p * p;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int i = (int)(e / p), j = (int)(e % p);
    if (i < j) {
      double v = 0.5 * (Bm[(int64_t)i * p + j] + Bm[(int64_t)j * p + i]);
      Bm[(int64_t)i * p + j] = v;
      Bm[(int64_t)j * p + i] = v;
    }
  }
}

void launch_symmetrize(double* B, int p, int modes, hipStream_t s) {
  int64_t total = (int64_t)p * p;
  unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 1024);
  hipLaunchKernelGGL(symmetrize_kernel, dim3(blocks, modes), dim3(256), 0, s, B, p);
}

// ---- sort eigenvalues, rank rule ------------------------------------------------
// perm[mode][0..p) lists eigen-indices by decreasing eigenvalue (ties by index).
// rank: #{lambda_i > eps^2 lambda_1} (sigma_i > eps sigma_1), capped at r_max;
// fixed[mode] > 0 overrides.
__global__ __launch_bounds__(EIG_THREADS) void rank_select_kernel(const double* __restrict__ Ball,
                                                                  int p, double eps2,
                                                                  const int* __restrict__ fixed,
                                                                  int r_max, int* __restrict__ perm,
                                                                  RankInfo* info) {
  const int mode = blockIdx.x;
  const double* B = Ball + (int64_t)mode * p * p;
  __shared__ double lam1_s;
  __shared__ int cnt_s;
  int* pm = perm + mode * p;
  if (threadIdx.x == 0) cnt_s = 0;
  __syncthreads();
  // the diagonal staged in LDS once; NaN (from invalid input, rejected by
  // the host afterwards) orders as -inf so that perm is always a
  // permutation of 0..p-1
  extern __shared__ double dg[];   // p
  for (int i = threadIdx.x; i < p; i += EIG_THREADS) {
    const double v = B[(int64_t)i * p + i];
    dg[i] = v != v ? -HUGE_VAL : v;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < p; i += EIG_THREADS) {
    const double li = dg[i];
    int rank = 0;
    for (int j = 0; j < p; ++j) {
      const double lj = dg[j];
      if (lj > li || (lj == li && j < i)) ++rank;
    }
    pm[rank] = i;
  }
  __syncthreads();
  if (threadIdx.x == 0) lam1_s = fmax(B[(int64_t)pm[0] * p + pm[0]], 0.0);
  __syncthreads();
  const double lam1 = lam1_s;
  int local = 0;
  for (int i = threadIdx.x; i < p; i += EIG_THREADS)
    if (B[(int64_t)i * p + i] > eps2 * lam1) ++local;
  atomicAdd(&cnt_s, local);  // integer count: order independent
  __syncthreads();
  if (threadIdx.x == 0) {
    int r = cnt_s;
    int capped = 0;
    if (fixed && fixed[mode] > 0) {
      r = fixed[mode];
    } else if (r > r_max) {
      r = r_max;
      capped = 1;
    }
    if (r < 1) r = 1;
    if (r > p) r = p;
    info->r[mode] = r;
    info->capped[mode] = capped;
    info->lam1[mode] = lam1;
    info->lam_kept[mode] = B[(int64_t)pm[r - 1] * p + pm[r - 1]];
    info->lam_next[mode] = r < p ? B[(int64_t)pm[r] * p + pm[r]] : 0.0;
  }
}

void launch_rank_select(const double* B, int p, int modes, double eps2, const int* fixed,
                        int r_max, int* perm, RankInfo* info_dev, hipStream_t s) {
  hipLaunchKernelGGL(rank_select_kernel, dim3(modes), dim3(EIG_THREADS), (size_t)p * sizeof(double),
                     s, B, p, eps2, fixed, r_max, perm, info_dev);
}

// Wr (p x r col-major) = Z[:, perm[0..r)] for row-major Z (p x ldz); an
// index outside Z's columns (possible only for non-finite eigenvalues,
// which the host rejects) yields a zero column.
__global__ void gather_cols_kernel(const double* __restrict__ Z, int ldz,
                                   const int* __restrict__ perm, int p, int r,
                                   double* __restrict__ Wr) {
  int64_t total = (int64_t)p * r;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int col = (int)(e / p), row = (int)(e % p);
    const int src = perm[col];
    Wr[e] = (src >= 0 && src < ldz) ? Z[(int64_t)row * ldz + src] : 0.0;
  }
}

void launch_gather_cols(const double* Z, int ldz, const int* perm, int p, int r, double* Wr,
                        hipStream_t s) {
  int64_t total = (int64_t)p * r;
  unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(gather_cols_kernel, dim3(blocks), dim3(256), 0, s, Z, ldz, perm, p, r, Wr);
}

// One wave per column of the row-major n x r matrix: find the entry of
// largest magnitude (first on ties) and flip the column if it is negative.
// Column c of Q (n x r, row-major) is negated when its entry of largest
// magnitude (lowest row on ties) is negative; the same columns of W (m x r,
// column-major, when given) are negated with it.
__global__ void canonical_signs_kernel(double* Q, int64_t n, int r, double* W, int64_t m) {
  const int col = blockIdx.x;
  const int lane = threadIdx.x;
  double best = -1.0;
  int64_t bi = 0;
  for (int64_t i = lane; i < n; i += 64) {
    double v = fabs(Q[i * r + col]);
    if (v > best) {
      best = v;
      bi = i;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    double ob = __shfl_xor(best, off);
    int64_t oi = __shfl_xor(bi, off);
    if (ob > best || (ob == best && oi < bi)) {
      best = ob;
      bi = oi;
    }
  }
  const bool flip = Q[bi * r + col] < 0.0;
  if (flip) {
    for (int64_t i = lane; i < n; i += 64) Q[i * r + col] = -Q[i * r + col];
    if (W)
      for (int64_t i = lane; i < m; i += 64) W[col * m + i] = -W[col * m + i];
  }
}

void launch_canonical_signs(double* Qrow, int64_t n, int r, hipStream_t s, double* W, int64_t m) {
  hipLaunchKernelGGL(canonical_signs_kernel, dim3(r), dim3(64), 0, s, Qrow, n, r, W, m);
}

// The three modes in one launch each (blockIdx.y = mode).
__global__ void gather_cols3_kernel(const double* __restrict__ Z, int ldz, int64_t zstride,
                                    const int* __restrict__ perm, int p, Mode3 w) {
  const int mode = blockIdx.y;
  const int r = w.r[mode];
  const double* Zm = Z + (int64_t)mode * zstride;
  const int* pm = perm + (int64_t)mode * p;
  double* Wr = w.p[mode];
  const int64_t total = (int64_t)p * r;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int col = (int)(e / p), row = (int)(e % p);
    const int src = pm[col];
    Wr[e] = (src >= 0 && src < ldz) ? Zm[(int64_t)row * ldz + src] : 0.0;
  }
}

void launch_gather_cols3(const double* Z, int ldz, int64_t zstride, const int* perm, int p,
                         const Mode3& Wr, hipStream_t s) {
  const int rmax = std::max({Wr.r[0], Wr.r[1], Wr.r[2]});
  const int64_t total = (int64_t)p * rmax;
  const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 4096));
  hipLaunchKernelGGL(gather_cols3_kernel, dim3(blocks, 3), dim3(256), 0, s, Z, ldz, zstride, perm, p,
                     Wr);
}

__global__ void canonical_signs3_kernel(Mode3 q, int64_t n, Mode3 w, int64_t m) {
  const int mode = blockIdx.y;
  const int r = q.r[mode];
  const int col = blockIdx.x;
  if (col >= r) return;   // uniform over the (one-wave) workgroup
  double* Q = q.p[mode];
  double* W = w.p[mode];
  const int lane = threadIdx.x;
  double best = -1.0;
  int64_t bi = 0;
  // unrolled: the strided loads of a lane are issued together
#pragma unroll 8
  for (int64_t i = lane; i < n; i += 64) {
    double v = fabs(Q[i * r + col]);
    if (v > best) {
      best = v;
      bi = i;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    double ob = __shfl_xor(best, off);
    int64_t oi = __shfl_xor(bi, off);
    if (ob > best || (ob == best && oi < bi)) {
      best = ob;
      bi = oi;
    }
  }
  const bool flip = Q[bi * r + col] < 0.0;
  if (flip) {
#pragma unroll 8
    for (int64_t i = lane; i < n; i += 64) Q[i * r + col] = -Q[i * r + col];
    if (W)
      for (int64_t i = lane; i < m; i += 64) W[col * m + i] = -W[col * m + i];
  }
}

void launch_canonical_signs3(const Mode3& Q, int64_t n, const Mode3& W, int64_t m, hipStream_t s) {
  const int rmax = std::max({Q.r[0], Q.r[1], Q.r[2]});
  hipLaunchKernelGGL(canonical_signs3_kernel, dim3((unsigned)std::max(rmax, 1), 3), dim3(64), 0, s, Q,
                     n, W, m);
}

// ---- shifted Cholesky QR ---------------------------------------------------------
// Y (n x p, col-major) <- Y R^{-1} with C = Y^T Y = R^T R.  A shifted pass
// adds s = 11 (n p + p (p + 1)) u tr(C) to the diagonal so that the
// factorisation exists for condition numbers up to ~1/u (shifted CholeskyQR,
// Fukaya, Kannan, Nakatsukasa, Yamamoto, Yanagisawa 2020); plain passes then
// restore orthogonality.
// The factor is kept as the lower L = R^T.  The p x p matrix is worked on in
// LDS when it fits, else in the global scratch it came in.
constexpr int CHOL_THREADS = 1024;
constexpr int CF_THREADS = 256;   // Cholesky factorisation workgroup (16 x 16 layout)

template <bool LDS>
__global__ __launch_bounds__(CF_THREADS) void chol_kernel(double* __restrict__ Call, int p,
                                                          int64_t nrows, int shifted,
                                                          int* __restrict__ fail, int fail_bit) {
  extern __shared__ double shc[];
  __shared__ double red[CF_THREADS / 64];
  __shared__ double piv_s;
  const int mode = blockIdx.x;
  double* Cg = Call + (int64_t)mode * p * p;
  double* C = LDS ? shc : Cg;
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int pp = p * p;
  if (LDS)
    for (int e = tid; e < pp; e += CF_THREADS) C[e] = Cg[e];
  __syncthreads();
  if (shifted) {
    double tr = 0.0;
    for (int i = tid; i < p; i += CF_THREADS) tr += C[i * p + i];
    tr = wave_sum(tr);
    if ((tid & 63) == 0) red[tid >> 6] = tr;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int w = 0; w < CF_THREADS / 64; ++w) t += red[w];
      piv_s = 11.0 * ((double)nrows * p + (double)p * (p + 1)) * 1.1102230246251565e-16 * t;
    }
    __syncthreads();
    const double sh = piv_s;
    for (int i = tid; i < p; i += CF_THREADS) C[i * p + i] += sh;
    __syncthreads();
  }
  // right-looking, lower triangle in place (column-major: C[row + col*p]);
  // step k: the trailing update uses the unscaled column k and the pivot d,
  // then column k is scaled by 1/sqrt(d)
  for (int k = 0; k < p; ++k) {
    double d = C[k * p + k];
    if (!(d > 0.0)) {
      if (tid == 0) atomicOr(fail, fail_bit);
      d = 1e-300;
    }
    const double invd = 1.0 / d;
    for (int j = k + 1 + ty; j < p; j += 16) {
      const double cj = C[k * p + j] * invd;
      for (int i = j + tx; i < p; i += 16) C[j * p + i] -= C[k * p + i] * cj;
    }
    __syncthreads();
    const double sq = sqrt(d), isq = 1.0 / sq;
    for (int i = k + 1 + tid; i < p; i += CF_THREADS) C[k * p + i] *= isq;
    if (tid == 0) C[k * p + k] = sq;
    __syncthreads();
  }
  if (LDS)
    for (int e = tid; e < pp; e += CF_THREADS) Cg[e] = C[e];
}

// Cholesky factorisation with the matrix in registers, for p <= 16 RT: a
// 16 x 16 thread grid, thread (tx, ty) holds C[i, j] for i = tx + 16 a,
// j = ty + 16 b.  Step k: the threads holding column k publish it in LDS
// (rows above k as zeros; double-buffered, one barrier per step), every
// thread applies the rank-1 update with l = c_k / c_kk to its entries on
// or below the diagonal, and wave 0 writes column k of L.  The steps are
// grouped by the column block KB = k / 16, a compile-time constant, so that
// finished blocks are skipped without branches and the owning registers
// are addressed statically.
template <int RT, int KB>
__device__ __forceinline__ void chol_reg_steps(double (&c)[RT][RT], double (&colk)[2][16 * RT],
                                               double* __restrict__ C, int p, int tx, int ty,
                                               int tid, bool& bad) {
  if constexpr (KB < RT) {
    for (int kk = 0; kk < 16; ++kk) {
      const int k = 16 * KB + kk;
      if (k >= p) return;
      double* cb = colk[k & 1];
      if (ty == kk) {
#pragma unroll
        for (int a = 0; a < RT; ++a) {
          const int i = tx + 16 * a;
          cb[i] = i >= k ? c[a][KB] : 0.0;
        }
      }
      __syncthreads();
      double dkk = cb[k];
      bad |= !(dkk > 0.0);
      dkk = dkk > 0.0 ? dkk : 1e-300;
      const double rd = 1.0 / dkk;
      if (tid < 64) {
        const double sq = sqrt(dkk), isq = 1.0 / sq;
        for (int i = k + tid; i < p; i += 64) C[(int64_t)k * p + i] = i == k ? sq : cb[i] * isq;
      }
      double li[RT], lj[RT];
#pragma unroll
      for (int a = KB; a < RT; ++a) li[a] = cb[tx + 16 * a] * rd;
#pragma unroll
      for (int b = KB; b < RT; ++b) lj[b] = cb[ty + 16 * b];
#pragma unroll
      for (int a = KB; a < RT; ++a)
#pragma unroll
        for (int b = KB; b <= a; ++b) c[a][b] = fma(-li[a], lj[b], c[a][b]);
    }
    chol_reg_steps<RT, KB + 1>(c, colk, C, p, tx, ty, tid, bad);
  }
}

// Blocked form of the register Cholesky: panels of 4 columns.  The 4
// columns k0..k0+3 (k0 a multiple of 4) are held by the threads ty = k0 % 16
// .. + 3, which form exactly one wave.  That wave publishes them in LDS,
// factors the 4 x 4 diagonal block (every lane redundantly), solves the
// panel rows (2 rows per lane), writes column k0..k0+3 of L to memory and
// the scaled panel to LDS; after one barrier every thread applies the rank-4
// update to its entries on or below the diagonal.
template <int RT, int KB>
__device__ __forceinline__ void chol4_steps(double (&c)[RT][RT], double (&colk)[2][4][16 * RT],
                                            double (&lpan)[2][4][16 * RT], double* __restrict__ C,
                                            int p, int tx, int ty, int tid, bool& bad) {
  if constexpr (KB < RT) {
#pragma unroll 1
    for (int s4 = 0; s4 < 4; ++s4) {
      const int k0 = 16 * KB + 4 * s4;
      if (k0 >= p) return;
      const int buf = s4 & 1;
      const int kk0 = 4 * s4;
      if ((tid >> 6) == s4) {
        // the owner wave: lane = tx + 16 (ty - kk0)
        const int cc = ty - kk0;
#pragma unroll
        for (int a = 0; a < RT; ++a) {
          const int i = tx + 16 * a;
          colk[buf][cc][i] = (i >= k0 && k0 + cc < p) ? c[a][KB] : 0.0;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        // 4 x 4 diagonal block (columns beyond p act as identity)
        double Ld[4][4], dinv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          double sdiag = k0 + q < p ? colk[buf][q][k0 + q] : 1.0;
#pragma unroll
          for (int m = 0; m < q; ++m) sdiag -= Ld[q][m] * Ld[q][m];
          if (k0 + q < p) bad |= !(sdiag > 0.0);
          sdiag = sdiag > 0.0 ? sdiag : 1e-300;
          const double sq = sqrt(sdiag);
          dinv[q] = 1.0 / sq;
          Ld[q][q] = sq;
#pragma unroll
          for (int r = q + 1; r < 4; ++r) {
            double x = (k0 + r < p && k0 + q < p) ? colk[buf][q][k0 + r] : 0.0;
#pragma unroll
            for (int m = 0; m < q; ++m) x -= Ld[r][m] * Ld[q][m];
            Ld[r][q] = x * dinv[q];
          }
        }
        // panel rows i = lane, lane + 64 (i >= k0 + 4), the diagonal block rows from Ld
        const int lane = tid & 63;
#pragma unroll
        for (int h = 0; h < 2 * RT / 8 + 1; ++h) {
          const int i = lane + 64 * h;
          if (i < 16 * RT) {
            double l[4];
            if (i >= k0 + 4) {
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                double x = colk[buf][q][i];
#pragma unroll
                for (int m = 0; m < q; ++m) x -= l[m] * Ld[q][m];
                l[q] = x * dinv[q];
              }
            } else {
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                l[q] = 0.0;
#pragma unroll
                for (int r = q; r < 4; ++r)
                  if (i == k0 + r) l[q] = Ld[r][q];
              }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              lpan[buf][q][i] = i >= k0 + 4 ? l[q] : 0.0;
              if (i >= k0 && i < p && k0 + q < p && i >= k0 + q) C[(int64_t)(k0 + q) * p + i] = l[q];
            }
          }
        }
      }
      __syncthreads();
      double li[RT][4], lj[RT][4];
#pragma unroll
      for (int a = KB; a < RT; ++a)
#pragma unroll
        for (int q = 0; q < 4; ++q) li[a][q] = lpan[buf][q][tx + 16 * a];
#pragma unroll
      for (int b = KB; b < RT; ++b)
#pragma unroll
        for (int q = 0; q < 4; ++q) lj[b][q] = lpan[buf][q][ty + 16 * b];
#pragma unroll
      for (int a = KB; a < RT; ++a)
#pragma unroll
        for (int b = KB; b <= a; ++b) {
          double v = c[a][b];
#pragma unroll
          for (int q = 0; q < 4; ++q) v = fma(-li[a][q], lj[b][q], v);
          c[a][b] = v;
        }
    }
    chol4_steps<RT, KB + 1>(c, colk, lpan, C, p, tx, ty, tid, bad);
  }
}

template <int RT>
__global__ __launch_bounds__(256) void chol4_reg_kernel(double* __restrict__ Call, int p,
                                                        int64_t nrows, int shifted,
                                                        int* __restrict__ fail, int fail_bit) {
  __shared__ double colk[2][4][16 * RT];
  __shared__ double lpan[2][4][16 * RT];
  __shared__ double red[4];
  const int mode = blockIdx.x;
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  double* C = Call + (int64_t)mode * p * p;
  double c[RT][RT];
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int b = 0; b < RT; ++b) {
      const int i = tx + 16 * a, j = ty + 16 * b;
      c[a][b] = (i < p && j < p && i >= j) ? C[(int64_t)j * p + i] : 0.0;
    }
  if (shifted) {
    double tr = 0.0;
    if (tx == ty)
#pragma unroll
      for (int a = 0; a < RT; ++a) tr += c[a][a];
    tr = wave_sum(tr);
    if ((tid & 63) == 0) red[tid >> 6] = tr;
    __syncthreads();
    const double t = (red[0] + red[1]) + (red[2] + red[3]);
    const double shift = 11.0 * ((double)nrows * p + (double)p * (p + 1)) * 1.1102230246251565e-16 * t;
    if (tx == ty)
#pragma unroll
      for (int a = 0; a < RT; ++a)
        if (tx + 16 * a < p) c[a][a] += shift;
  }
  __syncthreads();   // all reads of C precede the first write of L
  bool bad = false;
  chol4_steps<RT, 0>(c, colk, lpan, C, p, tx, ty, tid, bad);
  if (bad) atomicOr(fail, fail_bit);
}

template <int RT>
__global__ __launch_bounds__(256) void chol_reg_kernel(double* __restrict__ Call, int p,
                                                       int64_t nrows, int shifted,
                                                       int* __restrict__ fail, int fail_bit) {
  __shared__ double colk[2][16 * RT];
  __shared__ double red[4];
  const int mode = blockIdx.x;
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  double* C = Call + (int64_t)mode * p * p;
  double c[RT][RT];
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int b = 0; b < RT; ++b) {
      const int i = tx + 16 * a, j = ty + 16 * b;
      c[a][b] = (i < p && j < p && i >= j) ? C[(int64_t)j * p + i] : 0.0;
    }
  for (int x = tid; x < 2 * 16 * RT; x += 256) (&colk[0][0])[x] = 0.0;
  if (shifted) {
    double tr = 0.0;
    if (tx == ty)
#pragma unroll
      for (int a = 0; a < RT; ++a) tr += c[a][a];
    tr = wave_sum(tr);
    if ((tid & 63) == 0) red[tid >> 6] = tr;
    __syncthreads();
    const double t = (red[0] + red[1]) + (red[2] + red[3]);
    const double shift = 11.0 * ((double)nrows * p + (double)p * (p + 1)) * 1.1102230246251565e-16 * t;
    if (tx == ty)
#pragma unroll
      for (int a = 0; a < RT; ++a)
        if (tx + 16 * a < p) c[a][a] += shift;
  }
  __syncthreads();   // all reads of C and the zero fill precede the first step
  bool bad = false;
  chol_reg_steps<RT, 0>(c, colk, C, p, tx, ty, tid, bad);
  if (bad && tid == 0) atomicOr(fail, fail_bit);
}

// Y[i, :] <- Y[i, :] L^{-T} for row-major Y (n x p): one wave per row, the
// row held in registers (lane l keeps entries l, l + 64, ...), right-looking
// substitution: x_c = y_c / L_cc is read from its lane, then every lane
// subtracts x_c L[i, c] from its entries i > c.  L (lower, column-major) is
// staged in LDS packed by columns so that the lanes read consecutive words,
// with the reciprocal diagonal after it.
template <int RPL, bool LDS>
__global__ __launch_bounds__(1024) void trsm_rows_kernel(double* __restrict__ Yall,
                                                         const double* __restrict__ Lall,
                                                         int64_t n, int p) {
  extern __shared__ double sht[];
  const int mode = blockIdx.y;
  const double* L = Lall + (int64_t)mode * p * p;
  // LDS: column c holds L[c..p-1, c] at offset c p - c (c - 1) / 2; global:
  // column c of the column-major L starts at c p + c.  Either way Lc[i - c] = L[i, c].
  const int packed = p * (p + 1) / 2;
  if (LDS) {
    // loads in batches of SB per thread, issued together before their stores
    constexpr int SB = 16;
    for (int e0 = 0; e0 < p * p; e0 += SB * (int)blockDim.x) {
      double v[SB];
#pragma unroll
      for (int t = 0; t < SB; ++t) {
        const int e = e0 + t * (int)blockDim.x + (int)threadIdx.x;
        v[t] = e < p * p ? L[e] : 0.0;
      }
#pragma unroll
      for (int t = 0; t < SB; ++t) {
        const int e = e0 + t * (int)blockDim.x + (int)threadIdx.x;
        const int c = e / p, i = e - c * p;
        if (e < p * p && i >= c) sht[c * p - c * (c - 1) / 2 + (i - c)] = v[t];
      }
    }
    for (int c = threadIdx.x; c < p; c += blockDim.x) sht[packed + c] = 1.0 / L[(int64_t)c * p + c];
    __syncthreads();
  }
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= n) return;
  double* Y = Yall + (int64_t)mode * n * p + row * p;
  double y[RPL];
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    const int c = lane + 64 * u;
    y[u] = c < p ? Y[c] : 0.0;
  }
  // steps in groups of D: the L entries and reciprocal pivots of a group are
  // loaded before its dependent chain of substitutions
  constexpr int D = RPL <= 2 ? 8 : 4;
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    for (int cc0 = 0; cc0 < 64; cc0 += D) {
      const int c0 = 64 * u + cc0;
      if (c0 >= p) break;
      double lv[D][RPL], rdg[D];
#pragma unroll
      for (int t = 0; t < D; ++t) {
        const int c = c0 + t < p ? c0 + t : p - 1;
        const double* Lc = LDS ? sht + c * p - c * (c - 1) / 2 : L + (int64_t)c * p + c;
        rdg[t] = LDS ? sht[packed + c] : 1.0 / Lc[0];
#pragma unroll
        for (int u2 = u; u2 < RPL; ++u2) {
          const int i = 64 * u2 + lane;
          lv[t][u2] = (i > c && i < p) ? Lc[i - c] : 0.0;
        }
      }
#pragma unroll
      for (int t = 0; t < D; ++t) {
        const int cc = cc0 + t;
        if (c0 + t >= p) break;
        const double x = lane_f64(y[u], cc) * rdg[t];
        if (lane == cc) y[u] = x;
#pragma unroll
        for (int u2 = u; u2 < RPL; ++u2) y[u2] -= x * lv[t][u2];
      }
    }
  }
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    const int c = lane + 64 * u;
    if (c < p) Y[c] = y[u];
  }
}

// Blocked Cholesky for 128 < p <= 512: one workgroup of 1024 threads per
// mode, the matrix in global memory (it stays in L2), worked on in panels of
// CB = 16 rows of R.  A panel (rows K0..K0+15, columns K0..p-1) is loaded to
// LDS; one wave factors its 16 x 16 diagonal block, M11 = R11^T R11; every
// thread then solves R11^T R12[:, i] = M12[:, i] for its columns i (forward
// substitution, R11 read as broadcasts); the panel is written back as rows
// of R, and the trailing upper triangle then takes one rank-16 update
//   M[j][i] -= sum_k R[k][j] R[k][i],  K0 + 16 <= j <= i < p,
// so that every trailing entry is read and written once per panel instead
// of once per column.  The shift of a shifted pass is added to each diagonal
// entry when its panel is loaded.
constexpr int CB = 16;
constexpr int CHB_THREADS = 1024;

__global__ __launch_bounds__(CHB_THREADS) void chol_blk_kernel(double* __restrict__ Call, int p,
                                                               int64_t nrows, int shifted,
                                                               int* __restrict__ fail,
                                                               int fail_bit) {
  extern __shared__ double pan[];   // [CB][p + 1]
  __shared__ double red[CHB_THREADS / 64];
  __shared__ double sh_s;
  const int mode = blockIdx.x;
  double* C = Call + (int64_t)mode * p * p;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ldp = p + 1;
  double sh = 0.0;
  if (shifted) {
    double tr = 0.0;
    for (int i = tid; i < p; i += CHB_THREADS) tr += C[(int64_t)i * p + i];
    tr = wave_sum(tr);
    if (lane == 0) red[wave] = tr;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int w = 0; w < CHB_THREADS / 64; ++w) t += red[w];
      sh_s = 11.0 * ((double)nrows * p + (double)p * (p + 1)) * 1.1102230246251565e-16 * t;
    }
    __syncthreads();
    sh = sh_s;
  }
  for (int K0 = 0; K0 < p; K0 += CB) {
    const int nb = p - K0 < CB ? p - K0 : CB;
    const int w = p - K0;
    for (int e = tid; e < nb * w; e += CHB_THREADS) {
      const int r = e / w, c = e - r * w;
      double v = C[(int64_t)(K0 + r) * p + K0 + c];
      if (c == r) v += sh;
      pan[r * ldp + c] = v;
    }
    __syncthreads();
    // the diagonal block by wave 0: lane entries (r, c) = (e / 16, e % 16), e = lane + 64 t
    if (wave == 0) {
      for (int k = 0; k < nb; ++k) {
        double d = pan[k * ldp + k];
        if (!(d > 0.0)) {
          if (lane == 0) atomicOr(fail, fail_bit);
          d = 1e-300;
        }
        const double invd = 1.0 / d;
#pragma unroll
        for (int t = 0; t < CB * CB / 64; ++t) {
          const int e = lane + 64 * t, j = e / CB, i = e - (e / CB) * CB;
          if (j > k && i >= j && i < nb) pan[j * ldp + i] -= pan[k * ldp + i] * (pan[k * ldp + j] * invd);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const double sq = sqrt(d), isq = 1.0 / sq;
        if (lane > k && lane < nb) pan[k * ldp + lane] *= isq;
        if (lane == 0) pan[k * ldp + k] = sq;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
    __syncthreads();
    // the rest of the panel's rows: R12 = R11^{-T} M12, one column per thread
    for (int i = nb + tid; i < w; i += CHB_THREADS) {
      double x[CB];
#pragma unroll
      for (int k = 0; k < CB; ++k) {
        if (k < nb) {
          double v = pan[k * ldp + i];
#pragma unroll
          for (int l = 0; l < k; ++l) v -= pan[l * ldp + k] * x[l];
          x[k] = v / pan[k * ldp + k];
          pan[k * ldp + i] = x[k];
        }
      }
    }
    __syncthreads();
    for (int e = tid; e < nb * w; e += CHB_THREADS) {
      const int r = e / w, c = e - r * w;
      if (c >= r) C[(int64_t)(K0 + r) * p + K0 + c] = pan[r * ldp + c];
    }
    // trailing update, rows in groups of 4 (one wave per group), lanes over columns
    const int j0 = K0 + nb;
    const int ngroups = (p - j0 + 3) / 4;
    for (int g = wave; g < ngroups; g += CHB_THREADS / 64) {
      const int jb = j0 + 4 * g;
      for (int i = jb + lane; i < p; i += 64) {
        double acc[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = jb + r;
          acc[r] = (j < p && i >= j) ? C[(int64_t)j * p + i] : 0.0;
        }
        for (int k = 0; k < nb; ++k) {
          const double rki = pan[k * ldp + (i - K0)];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const double rkj = jb + r < p ? pan[k * ldp + (jb + r - K0)] : 0.0;
            acc[r] -= rkj * rki;
          }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = jb + r;
          if (j < p && i >= j) C[(int64_t)j * p + i] = acc[r];
        }
      }
    }
    __syncthreads();
  }
}

// Blocked Cholesky for 128 < p <= 512 on CG workgroups per mode (cooperative
// launch: all co-resident).  Workgroup g keeps rows i = g + CG t of M in LDS
// (the upper part, from column i) for the whole factorisation.  Per panel of
// CB rows: the owners publish their panel rows through the lower triangle of
// C (M[i][c], c >= i, at C[c][i]: nothing reads that part, and the panels
// use distinct columns of it), one grid barrier, then every workgroup loads
// the panel and factors it with the same arithmetic as chol_blk_kernel (the
// 16 x 16 diagonal block by one wave, forward substitution per column), and
// applies the rank-CB update to its own rows in LDS.  Workgroup 0 writes R:
// the strictly upper entries of each panel at once, the diagonal (whose slot
// carried the published M[i][i]) after a last barrier.
constexpr int CC_THREADS = 512;

__global__ __launch_bounds__(CC_THREADS) void chol_coop_kernel(double* __restrict__ Call, int p,
                                                               int64_t nrows, int shifted, int cg,
                                                               int* __restrict__ fail, int fail_bit) {
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  extern __shared__ double ccl[];
  __shared__ double red[CC_THREADS / 64];
  __shared__ double sh_s;
  const int mode = blockIdx.x / cg, g = blockIdx.x - (blockIdx.x / cg) * cg;
  double* C = Call + (int64_t)mode * p * p;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ldp = p + 1;
  const int nlm = (p + cg - 1) / cg;
  const int nloc = (p - g + cg - 1) / cg;   // own rows i = g + cg t, t < nloc
  double* rows = ccl;                        // [nlm][p], row t at rows + t p (columns >= i used)
  double* pan = rows + (size_t)nlm * p;      // [CB][ldp]
  double* rdiag = pan + (size_t)CB * ldp;    // [p] the diagonal of R (workgroup 0)
  double sh = 0.0;
  if (shifted) {
    double tr = 0.0;
    for (int i = tid; i < p; i += CC_THREADS) tr += C[(int64_t)i * p + i];
    tr = wave_sum(tr);
    if (lane == 0) red[wave] = tr;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int w = 0; w < CC_THREADS / 64; ++w) t += red[w];
      sh_s = 11.0 * ((double)nrows * p + (double)p * (p + 1)) * 1.1102230246251565e-16 * t;
    }
    __syncthreads();
    sh = sh_s;
  }
  // own rows, column j = i + tid (p <= CC_THREADS), RB rows per batch of
  // loads issued together before their LDS stores
  {
    constexpr int RB = 8;
    for (int t0 = 0; t0 < nloc; t0 += RB) {
      double v[RB];
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        const int t = t0 + u, i = g + cg * t, j = i + tid;
        v[u] = t < nloc && j < p ? C[(int64_t)i * p + j] : 0.0;
      }
      // the shift goes onto the diagonal after the batch (an add inside the
      // load's branch would make each load wait for its data)
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        const int t = t0 + u, i = g + cg * t, j = i + tid;
        if (t < nloc && j < p) {
          double x = v[u];
          if (j == i) x += sh;
          rows[(size_t)t * p + j] = x;
        }
      }
    }
  }
  grid.sync();   // every workgroup has read the diagonal (the shift) and its rows
  for (int K0 = 0; K0 < p; K0 += CB) {
    const int nb = p - K0 < CB ? p - K0 : CB;
    const int w = p - K0;
    // publish the owned panel rows: M[i][c] (c >= i) to C[c][i]
    for (int rr = 0; rr < nb; ++rr) {
      const int i = K0 + rr;
      if (i % cg != g) continue;   // uniform over the workgroup
      const double* ri = rows + (size_t)(i / cg) * p;
      for (int c = i + tid; c < p; c += CC_THREADS) C[(int64_t)c * p + i] = ri[c];
    }
    grid.sync();
    // the panel, pan[rr][cc] = M[K0 + rr][K0 + cc] for cc >= rr: loads in
    // batches of PB per thread, issued together before their LDS stores (one
    // memory latency per batch instead of one per element)
    {
      constexpr int PB = 8;
      const int tot = nb * w;
      for (int e0 = 0; e0 < tot; e0 += PB * CC_THREADS) {
        double v[PB];
#pragma unroll
        for (int u = 0; u < PB; ++u) {
          const int e = e0 + u * CC_THREADS + tid;
          const int cc = e / nb, rr = e - (e / nb) * nb;
          v[u] = e < tot && cc >= rr ? C[(int64_t)(K0 + cc) * p + K0 + rr] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < PB; ++u) {
          const int e = e0 + u * CC_THREADS + tid;
          const int cc = e / nb, rr = e - (e / nb) * nb;
          if (e < tot) pan[rr * ldp + cc] = v[u];
        }
      }
    }
    __syncthreads();
    // the diagonal block by wave 0 (as chol_blk_kernel)
    if (wave == 0) {
      for (int k = 0; k < nb; ++k) {
        double d = pan[k * ldp + k];
        if (!(d > 0.0)) {
          if (lane == 0 && g == 0) atomicOr(fail, fail_bit);
          d = 1e-300;
        }
        const double invd = 1.0 / d;
#pragma unroll
        for (int t = 0; t < CB * CB / 64; ++t) {
          const int e = lane + 64 * t, j = e / CB, i = e - (e / CB) * CB;
          if (j > k && i >= j && i < nb) pan[j * ldp + i] -= pan[k * ldp + i] * (pan[k * ldp + j] * invd);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const double sq = sqrt(d), isq = 1.0 / sq;
        if (lane > k && lane < nb) pan[k * ldp + lane] *= isq;
        if (lane == 0) pan[k * ldp + k] = sq;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
    __syncthreads();
    // the rest of the panel's rows: R12 = R11^{-T} M12, one column per thread
    for (int i = nb + tid; i < w; i += CC_THREADS) {
      double x[CB];
#pragma unroll
      for (int k = 0; k < CB; ++k) {
        if (k < nb) {
          double v = pan[k * ldp + i];
#pragma unroll
          for (int l = 0; l < k; ++l) v -= pan[l * ldp + k] * x[l];
          x[k] = v / pan[k * ldp + k];
          pan[k * ldp + i] = x[k];
        }
      }
    }
    __syncthreads();
    if (g == 0) {   // R's panel rows: strictly upper entries now, the diagonal at the end
      for (int e = tid; e < nb * w; e += CC_THREADS) {
        const int r = e / w, c = e - (e / w) * w;
        if (c > r) C[(int64_t)(K0 + r) * p + K0 + c] = pan[r * ldp + c];
        else if (c == r) rdiag[K0 + r] = pan[r * ldp + c];
      }
    }
    // rank-nb update of the own rows j >= K0 + nb: M[j][i] -= sum_k R[k][j] R[k][i], i >= j
    for (int t = wave; t < nloc; t += CC_THREADS / 64) {
      const int j = g + cg * t;
      if (j < K0 + nb) continue;   // uniform over the wave
      double* rj = rows + (size_t)t * p;
      for (int i = j + lane; i < p; i += 64) {
        double acc = rj[i];
        for (int k = 0; k < nb; ++k) acc -= pan[k * ldp + (j - K0)] * pan[k * ldp + (i - K0)];
        rj[i] = acc;
      }
    }
    __syncthreads();
  }
  grid.sync();   // every panel has been read: the diagonal slots are free
  if (g == 0)
    for (int i = tid; i < p; i += CC_THREADS) C[(int64_t)i * p + i] = rdiag[i];
}

static size_t chol_coop_lds(int p, int cg) {
  const int nlm = (p + cg - 1) / cg;
  return ((size_t)nlm * p + (size_t)CB * (p + 1) + (size_t)p) * sizeof(double);
}

// kernels that use more than the default dynamic LDS opt in to the device limit
static void allow_lds(const void* fn, size_t bytes) {
  if (bytes > 48 * 1024)
    RS_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

// the cooperative form, when the device can launch it and its LDS fits
static bool launch_chol_coop(double* C, int p, int64_t nrows, int modes, int shifted, int lds_limit,
                             int* fail, int fail_bit, hipStream_t s) {
  static int coop = -1;
  if (coop < 0) {
    int dev = 0, v = 0;
    coop = (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeCooperativeLaunch, dev) == hipSuccess && v)
               ? 1 : 0;
  }
  if (!coop || p > CC_THREADS) return false;
  int cg = 16;
  if (chol_coop_lds(p, cg) + 1024 > (size_t)lds_limit) cg = 32;
  const size_t lds = chol_coop_lds(p, cg);
  if (lds + 1024 > (size_t)lds_limit) return false;
  allow_lds((const void*)chol_coop_kernel, lds);
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, chol_coop_kernel, CC_THREADS, lds) !=
          hipSuccess || per_cu < 1)
    return false;
  void* args[] = {&C, &p, &nrows, &shifted, &cg, &fail, &fail_bit};
  RS_HIP(hipLaunchCooperativeKernel((const void*)chol_coop_kernel, dim3(modes * cg),
                                    dim3(CC_THREADS), args, lds, s));
  return true;
}

void launch_chol(double* C, int p, int64_t nrows, int modes, int shifted, int lds_limit, int* fail,
                 int fail_bit, hipStream_t s) {
  if (p <= 64) {
    hipLaunchKernelGGL(chol_reg_kernel<4>, dim3(modes), dim3(256), 0, s, C, p, nrows, shifted, fail,
                       fail_bit);
    return;
  }
  if (p <= 128) {
    hipLaunchKernelGGL(chol4_reg_kernel<8>, dim3(modes), dim3(256), 0, s, C, p, nrows, shifted, fail,
                       fail_bit);
    return;
  }
  const size_t bytes = (size_t)p * p * sizeof(double);
  const size_t pbytes = (size_t)CB * (p + 1) * sizeof(double);
  if (p <= 512 && launch_chol_coop(C, p, nrows, modes, shifted, lds_limit, fail, fail_bit, s)) return;
  if (p <= 512 && pbytes + 1024 <= (size_t)lds_limit) {
    allow_lds((const void*)chol_blk_kernel, pbytes);
    hipLaunchKernelGGL(chol_blk_kernel, dim3(modes), dim3(CHB_THREADS), pbytes, s, C, p, nrows,
                       shifted, fail, fail_bit);
  } else if (bytes + 1024 <= (size_t)lds_limit) {
    allow_lds((const void*)chol_kernel<true>, bytes);
    hipLaunchKernelGGL(chol_kernel<true>, dim3(modes), dim3(CF_THREADS), bytes, s, C, p, nrows,
                       shifted, fail, fail_bit);
  } else {
    hipLaunchKernelGGL(chol_kernel<false>, dim3(modes), dim3(CF_THREADS), 0, s, C, p, nrows,
                       shifted, fail, fail_bit);
  }
}

template <int RPL>
static void trsm_launch(double* Y, const double* L, int64_t n, int p, int modes, size_t bytes,
                        bool lds, hipStream_t s) {
  const int waves = 16;
  const dim3 grid((unsigned)((n + waves - 1) / waves), modes);
  if (lds) {
    allow_lds((const void*)trsm_rows_kernel<RPL, true>, bytes);
    hipLaunchKernelGGL((trsm_rows_kernel<RPL, true>), grid, dim3(64 * waves), bytes, s, Y, L, n, p);
  } else {
    hipLaunchKernelGGL((trsm_rows_kernel<RPL, false>), grid, dim3(64 * waves), 0, s, Y, L, n, p);
  }
}

void launch_trsm_rows(double* Y, const double* L, int64_t n, int p, int modes, int lds_limit,
                      hipStream_t s) {
  const size_t bytes = ((size_t)p * (p + 1) / 2 + (size_t)p) * sizeof(double);
  const bool lds = bytes + 1024 <= (size_t)lds_limit;
  if (p <= 64) trsm_launch<1>(Y, L, n, p, modes, bytes, lds, s);
  else if (p <= 128) trsm_launch<2>(Y, L, n, p, modes, bytes, lds, s);
  else if (p <= 256) trsm_launch<4>(Y, L, n, p, modes, bytes, lds, s);
  else if (p <= 512) trsm_launch<8>(Y, L, n, p, modes, bytes, lds, s);
  else throw Error{RS_E_UNSUPPORTED, "eigensolver subspace above 512"};
}

// Y[i, c] += eta * u(i, c) with eta = 1e-12 sqrt(tr(G) / (3 n)): a random
// perturbation far below the directions the rank rule keeps, which gives the
// sketch full column rank (the Gram can have rank below p, e.g. when
// R_l N < p) so that the Cholesky-based orthonormalisation cannot break down.
__global__ void perturb_kernel(double* __restrict__ Yall, const double* __restrict__ Gall,
                               int64_t n, int p, uint64_t seed) {
  const int mode = blockIdx.y;
  const double* G = Gall + (int64_t)mode * n * n;
  __shared__ double eta_s;
  if (threadIdx.x < 64) {
    double tr = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 64) tr += G[i * n + i];
    tr = wave_sum(tr);
    if (threadIdx.x == 0) eta_s = 1e-12 * sqrt(fmax(tr, 0.0) / (3.0 * (double)n));
  }
  __syncthreads();
  const double eta = eta_s > 0 ? eta_s : 1e-300;
  double* Y = Yall + (int64_t)mode * n * p;
  const int64_t total = n * p;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x)
    Y[e] += eta * hash_uniform(seed + mode, (uint64_t)(e % n), (uint64_t)(e / n));
}

// The same perturbation with the scale taken from the sketch itself:
// eta = rel sqrt(|Y|_F^2 / (n p)).  For the range-finder sketch
// Y = U diag(w^1/2) Omega with Omega uniform in [-1, 1), E |Y|_F^2 = p tr(G) / 3,
// so this is the scale above without forming G.  ETA_PARTS workgroups per
// mode write partial sums of |Y|_F^2; every workgroup of the perturbation
// adds them in the same order.
constexpr int ETA_PARTS = 32;
__global__ __launch_bounds__(256) void sketch_eta_kernel(const double* __restrict__ Yall,
                                                         int64_t n, int p,
                                                         double* __restrict__ part) {
  __shared__ double red[4];
  const int mode = blockIdx.y;
  const double* Y = Yall + (int64_t)mode * n * p;
  const int64_t total = n * p;
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += 256 * ETA_PARTS)
    acc += Y[e] * Y[e];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[mode * ETA_PARTS + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void perturb_eta_kernel(double* __restrict__ Yall, const double* __restrict__ part,
                                   int64_t n, int p, double rel, uint64_t seed) {
  const int mode = blockIdx.y;
  double t = 0.0;
  for (int b = 0; b < ETA_PARTS; ++b) t += part[mode * ETA_PARTS + b];
  const double eta0 = rel * sqrt(fmax(t, 0.0) / ((double)n * p));
  const double eta = eta0 > 0 ? eta0 : 1e-300;
  double* Y = Yall + (int64_t)mode * n * p;
  const int64_t total = n * p;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x)
    Y[e] += eta * hash_uniform(seed + mode, (uint64_t)(e % n), (uint64_t)(e / n));
}

size_t sketch_eta_bytes(int modes) { return (size_t)modes * ETA_PARTS * sizeof(double); }

void launch_sketch_eta(const double* Y, int64_t n, int p, int modes, double* part, hipStream_t s) {
  hipLaunchKernelGGL(sketch_eta_kernel, dim3(ETA_PARTS, modes), dim3(256), 0, s, Y, n, p, part);
}

void launch_perturb_eta(double* Y, const double* part, int64_t n, int p, int modes, double rel,
                        uint64_t seed, hipStream_t s) {
  const int64_t total = n * p;
  unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 2048);
  hipLaunchKernelGGL(perturb_eta_kernel, dim3(blocks, modes), dim3(256), 0, s, Y, part, n, p, rel,
                     seed);
}

void launch_perturb(double* Y, const double* G, int64_t n, int p, int modes, uint64_t seed,
                    hipStream_t s) {
  const int64_t total = n * p;
  unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 2048);
  hipLaunchKernelGGL(perturb_kernel, dim3(blocks, modes), dim3(256), 0, s, Y, G, n, p, seed);
}

// ---- dense symmetric eigensolver: tridiagonalisation, bisection, inverse iteration --
// B (p x p per mode) = W diag(lambda) W^T in four launches:
//  1. Householder tridiagonalisation Q^T B Q = T (Golub & Van Loan, Alg. 8.3.1),
//     one workgroup per mode; the Householder vectors are kept for step 4.
//  2. Eigenvalues of T by multisection on Sturm counts (Golub & Van Loan, Sec. 8.4.1),
//     one wave per eigenvalue: each lane counts at one of 64 interior points,
//     so the bracket shrinks 65-fold per round; eigenvalues come out sorted
//     descending and accurate to a few u ||T||.
//  3. Eigenvectors of T by inverse iteration (Golub & Van Loan, Sec. 8.2.2), one
//     thread per wanted eigenvector, three solves with T - lambda I from a
//     hashed start vector.
//  4. (by the caller) Cholesky QR of the vectors in eigenvalue order, which
//     also separates eigenvectors of near-equal eigenvalues; then
//  5. back-transformation W = H_0 H_1 ... H_{p-3} Z, one wave per column.
// Only the rc leading eigenvectors are formed (those the rank rule can keep).
constexpr int ES_THREADS = 256;

__device__ double es_block_sum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < ES_THREADS / 64; ++w) s += red[w];
  return s;
}

// Per-mode workspace (doubles): Householder vectors p x p (column k, rows
// k+2..p-1), betas p, d p, e p, lambda p, then the inverse-iteration scratch:
// multipliers p x rc and reciprocal pivots p x rc (row-major, thread j owns
// column j so that a wave touches consecutive words).  The vectors Z live in
// their own array, p x rc row-major per mode.
constexpr int TD_G = 16;   // workgroups per mode of the distributed tridiagonalisation

struct EigWs {
  double *hv, *beta, *d, *e, *lam, *lm, *ru, *sx;
  __host__ __device__ EigWs(double* base, int p, int rc, int mode) {
    const int64_t per = (int64_t)p * p + 4 * (int64_t)p + 2 * (int64_t)p * rc + 4 * (int64_t)p + 2 * TD_G;
    double* b = base + mode * per;
    hv = b;
    beta = hv + (int64_t)p * p;
    d = beta + p;
    e = d + p;
    lam = e + p;
    lm = lam + p;
    ru = lm + (int64_t)p * rc;
    sx = ru + (int64_t)p * rc;   // exchange buffers of the distributed tridiagonalisation
  }
};

size_t eig_sym_workspace_bytes(int p, int rc, int modes) {
  return (size_t)modes *
         ((size_t)p * p + 4 * (size_t)p + 2 * (size_t)p * rc + 4 * (size_t)p + 2 * TD_G) *
         sizeof(double);
}

// Householder tridiagonalisation with B in registers, for p <= 16 RT: thread
// (tx, ty) of a 16 x 16 grid holds B[i, j] for i = tx + 16 a, j = ty + 16 b,
// with tid = ty + 16 tx, so that the 16 lanes of a row share tx (the same
// rows of B) and differ in ty (the columns).  Step k:
//  1. the threads holding column k publish it in LDS (one barrier);
//  2. every wave forms the Householder vector from that column (norm by a
//     wave reduction, identical in all waves);
//  3. each lane multiplies its block by v; the sum over the 16 lanes of a
//     row gives (B22 v)_i in full for the wave's rows; it goes to LDS (one
//     barrier);
//  4. every wave forms kc = (beta/2) w^T v by a wave reduction and each
//     thread applies the rank-2 update B22 -= v w^T + w v^T to its entries.
// Steps are grouped by the column block KB = k / 16 (compile time): blocks
// of rows or columns below KB are finished and skipped.
struct TriLds {
  double col[2][128];
  double pw[2][128];
};

template <int RT, int KB>
__device__ __forceinline__ void tridiag_reg_steps(double (&c)[RT][RT], TriLds& L, EigWs& W, int p,
                                                  int tx, int ty) {
  if constexpr (KB < RT) {
    const int lane = threadIdx.x & 63;
    for (int kk = 0; kk < 16; ++kk) {
      const int k = 16 * KB + kk;
      if (k + 2 >= p) return;
      const int s = k & 1;
      // 1. publish column k (rows >= k), zeros above
      if (ty == kk) {
#pragma unroll
        for (int a = 0; a < RT; ++a) {
          const int i = tx + 16 * a;
          L.col[s][i] = (a >= KB && i >= k) ? c[a][KB] : 0.0;
        }
      }
      __syncthreads();
      // 2. Householder vector (every wave, uniform values)
      const double* col = L.col[s];
      double part = 0.0;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int i = lane + 64 * h;
        const double x = (i >= k + 2 && i < 16 * RT) ? col[i] : 0.0;
        part = fma(x, x, part);
      }
      const double sigma = wave_sum_dpp(part);
      const double x1 = col[k + 1];
      double beta = 0.0, v1 = 1.0, sub = x1;
      if (sigma > 0.0) {
        const double mu = sqrt(x1 * x1 + sigma);
        v1 = x1 <= 0.0 ? x1 - mu : -sigma / (x1 + mu);
        beta = 2.0 * v1 * v1 / (sigma + v1 * v1);
        sub = mu;
      }
      const double inv1 = 1.0 / v1;
      if (threadIdx.x < 64) {
        if (lane == 0) {
          W.d[k] = col[k];
          W.e[k] = sub;
          W.beta[k] = beta;
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int i = lane + 64 * h;
          if (i >= k + 2 && i < p) W.hv[(int64_t)k * p + i] = col[i] * inv1;
        }
      }
      if (beta == 0.0) continue;   // uniform: column already reduced
      double vi[RT], vj[RT];
#pragma unroll
      for (int a = KB; a < RT; ++a) {
        const int i = tx + 16 * a;
        vi[a] = i == k + 1 ? 1.0 : (i >= k + 2 ? col[i] * inv1 : 0.0);
      }
#pragma unroll
      for (int b = KB; b < RT; ++b) {
        const int j = ty + 16 * b;
        vj[b] = j == k + 1 ? 1.0 : (j >= k + 2 ? col[j] * inv1 : 0.0);
      }
      // 3. (B22 v) for the rows of this thread, summed over the row's lanes
#pragma unroll
      for (int a = KB; a < RT; ++a) {
        double acc = 0.0;
#pragma unroll
        for (int b = KB; b < RT; ++b) acc = fma(c[a][b], vj[b], acc);
        acc = row_sum16(acc);
        if (ty == 0) L.pw[s][tx + 16 * a] = beta * acc;
      }
      __syncthreads();
      // 4. w = pw - kc v with kc = (beta / 2) pw^T v, then the rank-2 update
      const double* pw = L.pw[s];
      double t = 0.0;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int i = lane + 64 * h;
        if (i > k && i < p) t = fma(pw[i], i == k + 1 ? 1.0 : col[i] * inv1, t);
      }
      const double kc = 0.5 * beta * wave_sum_dpp(t);
      double wi[RT], wj[RT];
#pragma unroll
      for (int a = KB; a < RT; ++a) {
        const int i = tx + 16 * a;
        wi[a] = (i > k && i < p) ? fma(-kc, vi[a], pw[i]) : 0.0;
      }
#pragma unroll
      for (int b = KB; b < RT; ++b) {
        const int j = ty + 16 * b;
        wj[b] = (j > k && j < p) ? fma(-kc, vj[b], pw[j]) : 0.0;
      }
#pragma unroll
      for (int a = KB; a < RT; ++a)
#pragma unroll
        for (int b = KB; b < RT; ++b) c[a][b] = fma(-vi[a], wj[b], fma(-wi[a], vj[b], c[a][b]));
    }
    tridiag_reg_steps<RT, KB + 1>(c, L, W, p, tx, ty);
  }
}

template <int RT>
__global__ __launch_bounds__(256) void tridiag_reg_kernel(const double* __restrict__ Ball,
                                                          double* __restrict__ ws, int p, int rc) {
  __shared__ TriLds L;
  const int mode = blockIdx.x;
  const int tid = threadIdx.x;
  const int ty = tid & 15, tx = tid >> 4;
  const double* Bg = Ball + (int64_t)mode * p * p;
  EigWs W(ws, p, rc, mode);
  double c[RT][RT];
  // consecutive lanes (ty) read consecutive words of a row of B
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int b = 0; b < RT; ++b) {
      const int i = tx + 16 * a, j = ty + 16 * b;
      c[a][b] = (i < p && j < p) ? Bg[(int64_t)i * p + j] : 0.0;
    }
  for (int x = tid; x < p; x += 256) {
    W.e[x] = 0.0;
    W.beta[x] = 0.0;
  }
  __syncthreads();   // the zero fill lands before the steps write d, e, beta
  tridiag_reg_steps<RT, 0>(c, L, W, p, tx, ty);
  // trailing 2 x 2 block
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int b = 0; b < RT; ++b) {
      const int i = tx + 16 * a, j = ty + 16 * b;
      if (p >= 2 && i == p - 2 && j == p - 2) W.d[p - 2] = c[a][b];
      if (p >= 2 && i == p - 1 && j == p - 2) W.e[p - 2] = c[a][b];
      if (i == p - 1 && j == p - 1) W.d[p - 1] = c[a][b];
    }
}

template <bool LDS>
__global__ __launch_bounds__(ES_THREADS) void tridiag_kernel(double* __restrict__ Ball,
                                                             double* __restrict__ ws, int p,
                                                             int rc) {
  extern __shared__ double sh[];
  __shared__ double red[ES_THREADS / 64];
  __shared__ double v1_s;
  const int mode = blockIdx.x;
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  double* Bg = Ball + (int64_t)mode * p * p;
  EigWs W(ws, p, rc, mode);
  const int ldb = LDS ? p + 1 : p;                              // padded against bank conflicts
  double* B = LDS ? sh : Bg;                                    // row-major B(i, j) = B[i ldb + j]
  double* pw = LDS ? sh + (int64_t)p * (p + 1) : sh;            // p doubles
  double* d = W.d;
  double* e = W.e;
  double* betas = W.beta;
  const int pp = p * p;
  if (LDS)
    for (int x = tid; x < pp; x += ES_THREADS) {
      const int i = x / p, j = x - i * p;
      B[i * ldb + j] = Bg[x];
    }
  for (int x = tid; x < p; x += ES_THREADS) {
    e[x] = 0.0;
    betas[x] = 0.0;
  }
  __syncthreads();

  for (int k = 0; k + 2 < p; ++k) {
    double part = 0.0;
    for (int i = k + 2 + tid; i < p; i += ES_THREADS) part += B[i * ldb + k] * B[i * ldb + k];
    const double sigma = es_block_sum(part, red);
    if (tid == 0) {
      const double x1 = B[(k + 1) * ldb + k];
      double beta = 0.0, v1 = 1.0, sub = x1;
      if (sigma > 0.0) {
        const double mu = sqrt(x1 * x1 + sigma);
        v1 = x1 <= 0.0 ? x1 - mu : -sigma / (x1 + mu);
        beta = 2.0 * v1 * v1 / (sigma + v1 * v1);
        sub = mu;
      }
      d[k] = B[k * ldb + k];
      e[k] = sub;
      betas[k] = beta;
      v1_s = v1;
    }
    __syncthreads();
    const double beta = betas[k];
    if (beta == 0.0) continue;  // uniform: column already reduced
    const double inv1 = 1.0 / v1_s;
    for (int i = k + 2 + tid; i < p; i += ES_THREADS) B[i * ldb + k] *= inv1;   // v_i, v_{k+1} = 1
    __syncthreads();
    // pw = beta B22 v, reading B22 by columns (B symmetric) so that the
    // threads of a wave touch consecutive words
    for (int i = k + 1 + tid; i < p; i += ES_THREADS) {
      double acc0 = B[(k + 1) * ldb + i], acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
      int j = k + 2;
      for (; j + 3 < p; j += 4) {
        acc0 += B[j * ldb + i] * B[j * ldb + k];
        acc1 += B[(j + 1) * ldb + i] * B[(j + 1) * ldb + k];
        acc2 += B[(j + 2) * ldb + i] * B[(j + 2) * ldb + k];
        acc3 += B[(j + 3) * ldb + i] * B[(j + 3) * ldb + k];
      }
      for (; j < p; ++j) acc0 += B[j * ldb + i] * B[j * ldb + k];
      pw[i] = beta * ((acc0 + acc1) + (acc2 + acc3));
    }
    __syncthreads();
    part = 0.0;
    for (int i = k + 1 + tid; i < p; i += ES_THREADS) part += pw[i] * (i == k + 1 ? 1.0 : B[i * ldb + k]);
    const double kc = 0.5 * beta * es_block_sum(part, red);
    for (int i = k + 1 + tid; i < p; i += ES_THREADS) pw[i] -= kc * (i == k + 1 ? 1.0 : B[i * ldb + k]);
    __syncthreads();
    // B22 -= v w^T + w v^T
    for (int i = k + 1 + ty; i < p; i += 16) {
      const double vi = i == k + 1 ? 1.0 : B[i * ldb + k];
      const double wi = pw[i];
      for (int j = k + 1 + tx; j < p; j += 16) {
        const double vj = j == k + 1 ? 1.0 : B[j * ldb + k];
        B[i * ldb + j] -= vi * pw[j] + wi * vj;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (p >= 2) {
      d[p - 2] = B[(p - 2) * ldb + (p - 2)];
      e[p - 2] = B[(p - 1) * ldb + (p - 2)];
    }
    d[p - 1] = B[(p - 1) * ldb + (p - 1)];
    e[p - 1] = 0.0;
  }
  for (int x = tid; x < pp; x += ES_THREADS) {
    const int i = x / p, k = x - i * p;
    if (i >= k + 2) W.hv[(int64_t)k * p + i] = B[i * ldb + k];
  }
}

// Householder tridiagonalisation for 128 < p <= 512: one workgroup of 1024
// threads per mode, B (row-major, kept full and symmetric) in global memory,
// where it stays in L2.  Step k takes the Householder vector from row k
// (equal to column k), the product B22 v with the 16 waves over slices of
// the rows of B22 and the lanes over its columns (coalesced; the slices are
// summed in LDS in wave order), and the rank-2 update one row per wave,
// lanes over the columns.  Same outputs as the other tridiagonalisations:
// d, e, beta and the vectors v (v_{k+1} = 1 implicit) in hv.
constexpr int TW_THREADS = 1024;
constexpr int TW_WAVES = TW_THREADS / 64;
constexpr int TW_MAXA = 8;   // columns per lane: p <= 64 TW_MAXA

__device__ double tw_block_sum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < TW_WAVES; ++w) s += red[w];
  return s;
}

__global__ __launch_bounds__(TW_THREADS) void tridiag_wide_kernel(double* __restrict__ Ball,
                                                                  double* __restrict__ ws, int p,
                                                                  int rc) {
  extern __shared__ double tsh[];
  double* part = tsh;                   // [TW_WAVES][p]
  double* vs = tsh + TW_WAVES * p;      // [p]
  double* pw = vs + p;                  // [p]
  __shared__ double red[TW_WAVES];
  __shared__ double v1_s, beta_s;
  const int mode = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* B = Ball + (int64_t)mode * p * p;
  EigWs W(ws, p, rc, mode);
  for (int x = tid; x < p; x += TW_THREADS) {
    W.e[x] = 0.0;
    W.beta[x] = 0.0;
  }
  __syncthreads();
  for (int k = 0; k + 2 < p; ++k) {
    const double* rowk = B + (int64_t)k * p;
    double prt = 0.0;
    for (int i = k + 2 + tid; i < p; i += TW_THREADS) prt += rowk[i] * rowk[i];
    const double sigma = tw_block_sum(prt, red);
    if (tid == 0) {
      const double x1 = rowk[k + 1];
      double beta = 0.0, v1 = 1.0, sub = x1;
      if (sigma > 0.0) {
        const double mu = sqrt(x1 * x1 + sigma);
        v1 = x1 <= 0.0 ? x1 - mu : -sigma / (x1 + mu);
        beta = 2.0 * v1 * v1 / (sigma + v1 * v1);
        sub = mu;
      }
      W.d[k] = rowk[k];
      W.e[k] = sub;
      W.beta[k] = beta;
      v1_s = v1;
      beta_s = beta;
    }
    __syncthreads();
    const double beta = beta_s;
    if (beta == 0.0) {  // uniform: column already reduced (its entries below k+1 are zero)
      for (int i = k + 2 + tid; i < p; i += TW_THREADS) W.hv[(int64_t)k * p + i] = rowk[i];
      continue;
    }
    const double inv1 = 1.0 / v1_s;
    for (int i = k + 1 + tid; i < p; i += TW_THREADS) {
      const double v = i == k + 1 ? 1.0 : rowk[i] * inv1;
      vs[i] = v;
      if (i >= k + 2) W.hv[(int64_t)k * p + i] = v;
    }
    __syncthreads();
    double acc[TW_MAXA];
#pragma unroll
    for (int a = 0; a < TW_MAXA; ++a) acc[a] = 0.0;
    for (int j = k + 1 + wave; j < p; j += TW_WAVES) {
      const double vj = vs[j];
      const double* rowj = B + (int64_t)j * p;
#pragma unroll
      for (int a = 0; a < TW_MAXA; ++a) {
        const int i = k + 1 + lane + 64 * a;
        if (i < p) acc[a] += rowj[i] * vj;
      }
    }
#pragma unroll
    for (int a = 0; a < TW_MAXA; ++a) {
      const int i = k + 1 + lane + 64 * a;
      if (i < p) part[wave * p + i] = acc[a];
    }
    __syncthreads();
    for (int i = k + 1 + tid; i < p; i += TW_THREADS) {
      double sacc = 0.0;
      for (int w = 0; w < TW_WAVES; ++w) sacc += part[w * p + i];
      pw[i] = beta * sacc;
    }
    __syncthreads();
    prt = 0.0;
    for (int i = k + 1 + tid; i < p; i += TW_THREADS) prt += pw[i] * vs[i];
    const double kc = 0.5 * beta * tw_block_sum(prt, red);
    for (int i = k + 1 + tid; i < p; i += TW_THREADS) pw[i] -= kc * vs[i];
    __syncthreads();
    for (int i = k + 1 + wave; i < p; i += TW_WAVES) {
      const double vi = vs[i], wi = pw[i];
      double* rowi = B + (int64_t)i * p;
      for (int j = k + 1 + lane; j < p; j += 64) rowi[j] -= vi * pw[j] + wi * vs[j];
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (p >= 2) {
      W.d[p - 2] = B[(int64_t)(p - 2) * p + (p - 2)];
      W.e[p - 2] = B[(int64_t)(p - 1) * p + (p - 2)];
    }
    W.d[p - 1] = B[(int64_t)(p - 1) * p + (p - 1)];
    W.e[p - 1] = 0.0;
  }
}

// Householder tridiagonalisation for 128 < p <= 512 on TD_G workgroups per
// mode (cooperative launch: all co-resident).  Workgroup g keeps rows
// i = g + TD_G t of B in LDS for the whole factorisation.  The rank-2 update
// of step k-1 is applied lazily, fused with the product B22 v of step k in one
// pass over the workgroup's rows; the owner of row k+1 publishes that row
// (through global memory), and after the grid barrier every workgroup
// derives the next Householder vector from it with identical arithmetic, so
// one grid barrier per step suffices.  Exchange buffers (per mode, parity
// k & 1): the products pw[2][p], the published rows row[2][p] and the
// per-workgroup partial sums of pw . v, part[2][TD_G].  Same outputs as the
// other tridiagonalisations.
constexpr int TD_THREADS = 512;
constexpr int TD_WAVES = TD_THREADS / 64;

__global__ __launch_bounds__(TD_THREADS) void tridiag_dist_kernel(const double* __restrict__ Ball,
                                                                  double* __restrict__ ws, int p,
                                                                  int rc) {
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  extern __shared__ double tds[];
  __shared__ double red[TD_WAVES];
  __shared__ double sh_beta, sh_v1;
  const int mode = blockIdx.x / TD_G, g = blockIdx.x - (blockIdx.x / TD_G) * TD_G;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nlm = (p + TD_G - 1) / TD_G;
  const int nloc = (p - g + TD_G - 1) / TD_G;   // rows i = g + TD_G t, t < nloc
  double* rows = tds;                           // [nlm][p]
  double* vold = rows + (size_t)nlm * p;        // pending vector v_{k-1}
  double* wold = vold + p;                      // pending w_{k-1}
  double* vnew = wold + p;                      // v_k
  double* rk = vnew + p;                        // current row k
  const double* B = Ball + (int64_t)mode * p * p;
  EigWs W(ws, p, rc, mode);
  double* pwb[2] = {W.sx, W.sx + p};
  double* rowb[2] = {W.sx + 2 * p, W.sx + 3 * p};
  double* partb[2] = {W.sx + 4 * p, W.sx + 4 * p + TD_G};
  {   // own rows, column tid (p <= TD_THREADS), RB rows per batch of loads
    constexpr int RB = 8;
    for (int t0 = 0; t0 < nloc; t0 += RB) {
      double v[RB];
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        const int t = t0 + u;
        v[u] = t < nloc && tid < p ? B[(int64_t)(g + TD_G * t) * p + tid] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        const int t = t0 + u;
        if (t < nloc && tid < p) rows[t * p + tid] = v[u];
      }
    }
  }
  for (int j = tid; j < p; j += TD_THREADS) {
    vold[j] = 0.0;
    wold[j] = 0.0;
    if (g == 0) {
      W.e[j] = 0.0;
      W.beta[j] = 0.0;
    }
  }
  __syncthreads();
  double beta_prev = 0.0;
  for (int k = 0; k + 2 < p; ++k) {
    const int par = k & 1, ppar = par ^ 1;
    // one column per thread (p <= TD_THREADS); row k as published is loaded
    // with the previous step's products and partial sums, in one memory latency
    const int jc = k + tid;
    const double* pub = k == 0 ? B : rowb[ppar];   // row k before the pending update
    const double pub_j = jc < p ? pub[jc] : 0.0;
    if (k > 0) {   // the pending w_{k-1} = pw_{k-1} - kc v_{k-1}
      double ps = 0.0;
      for (int b = 0; b < TD_G; ++b) ps += partb[ppar][b];
      const double kc = 0.5 * beta_prev * ps;
      if (jc < p) wold[jc] = pwb[ppar][jc] - kc * vold[jc];
    }
    __syncthreads();
    {
      const double vk = vold[k], wk = wold[k];
      if (jc < p) rk[jc] = pub_j - (vk * wold[jc] + wk * vold[jc]);
    }
    __syncthreads();
    double prt = 0.0;
    for (int j = k + 2 + tid; j < p; j += TD_THREADS) prt += rk[j] * rk[j];
    prt = wave_sum(prt);
    if (lane == 0) red[wave] = prt;
    __syncthreads();
    if (tid == 0) {
      double sigma = 0.0;
      for (int w = 0; w < TD_WAVES; ++w) sigma += red[w];
      const double x1 = rk[k + 1];
      double beta = 0.0, v1 = 1.0, sub = x1;
      if (sigma > 0.0) {
        const double mu = sqrt(x1 * x1 + sigma);
        v1 = x1 <= 0.0 ? x1 - mu : -sigma / (x1 + mu);
        beta = 2.0 * v1 * v1 / (sigma + v1 * v1);
        sub = mu;
      }
      sh_beta = beta;
      sh_v1 = v1;
      if (g == 0) {
        W.d[k] = rk[k];
        W.e[k] = sub;
        W.beta[k] = beta;
      }
    }
    __syncthreads();
    const double beta = sh_beta, inv1 = 1.0 / sh_v1;
    for (int j = k + 1 + tid; j < p; j += TD_THREADS) {
      const double v = j == k + 1 ? 1.0 : rk[j] * inv1;
      vnew[j] = v;
      if (g == 0 && j >= k + 2) W.hv[(int64_t)k * p + j] = v;
    }
    __syncthreads();
    // own rows i >= k+1: apply the pending update, then pw_i = beta (B v_k)_i
    double kpart = 0.0;
    for (int t = wave; t < nloc; t += TD_WAVES) {
      const int i = g + TD_G * t;
      if (i < k + 1) continue;   // uniform over the wave
      const double vi = vold[i], wi = wold[i];
      double* ri = rows + (size_t)t * p;
      double acc = 0.0;
      for (int j = k + 1 + lane; j < p; j += 64) {
        const double b = ri[j] - (vi * wold[j] + wi * vold[j]);
        ri[j] = b;
        acc += b * vnew[j];
      }
      acc = wave_sum(acc);
      const double pwi = beta * acc;
      if (lane == 0) pwb[par][i] = pwi;
      kpart += pwi * vnew[i];
      if (i == k + 1)
        for (int j = k + 1 + lane; j < p; j += 64) rowb[par][j] = ri[j];
    }
    if (lane == 0) red[wave] = kpart;
    __syncthreads();
    if (tid == 0) {
      double sp = 0.0;
      for (int w = 0; w < TD_WAVES; ++w) sp += red[w];
      partb[par][g] = sp;
    }
    for (int j = k + 1 + tid; j < p; j += TD_THREADS) vold[j] = vnew[j];
    beta_prev = beta;
    grid.sync();
  }
  // the last pending update (of step p-3) on rows p-2 and p-1
  if (p >= 3) {
    const int par = (p - 3) & 1;
    double ps = 0.0;
    for (int b = 0; b < TD_G; ++b) ps += partb[par][b];
    const double kc = 0.5 * beta_prev * ps;
    if (tid == 0) {
      double w2[2];
      for (int q = 0; q < 2; ++q) w2[q] = pwb[par][p - 2 + q] - kc * vold[p - 2 + q];
      for (int t = 0; t < nloc; ++t) {
        const int i = g + TD_G * t;
        if (i < p - 2) continue;
        const double vi = vold[i], wi = w2[i - (p - 2)];
        double* ri = rows + (size_t)t * p;
        for (int q = 0; q < 2; ++q) ri[p - 2 + q] -= vi * w2[q] + wi * vold[p - 2 + q];
        if (i == p - 2) {
          W.d[p - 2] = ri[p - 2];
          W.e[p - 2] = ri[p - 1];
        } else {
          W.d[p - 1] = ri[p - 1];
          W.e[p - 1] = 0.0;
        }
      }
    }
  }
}

// the distributed form when the device can launch it cooperatively
static bool launch_tridiag_dist(double* B, double* ws, int p, int rc, int modes, hipStream_t s) {
  static int coop = -1;
  if (coop < 0) {
    int dev = 0, v = 0;
    coop = (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeCooperativeLaunch, dev) == hipSuccess && v)
               ? 1 : 0;
  }
  if (!coop || p < 3 || p > TD_THREADS) return false;
  const int nlm = (p + TD_G - 1) / TD_G;
  const size_t lds = ((size_t)nlm * p + 4 * (size_t)p) * sizeof(double);
  if (lds > 150 * 1024) return false;
  allow_lds((const void*)tridiag_dist_kernel, lds);
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, tridiag_dist_kernel, TD_THREADS, lds) !=
          hipSuccess || per_cu < 1)
    return false;
  void* args[] = {&B, &ws, &p, &rc};
  RS_HIP(hipLaunchCooperativeKernel((const void*)tridiag_dist_kernel, dim3(modes * TD_G),
                                    dim3(TD_THREADS), args, lds, s));
  return true;
}

// 1/q for finite nonzero q: the hardware reciprocal estimate refined by two
// Newton steps t <- t + t (1 - q t) (each roughly doubles the correct bits).
__device__ __forceinline__ double recip(double q) {
  double t = __builtin_amdgcn_rcp(q);
  t = fma(t, fma(-q, t, 1.0), t);
  t = fma(t, fma(-q, t, 1.0), t);
  return t;
}

// Number of eigenvalues of T below x (Sturm count on the LDL^T pivots of
// T - x I), with tiny pivots replaced by -pivmin and huge ones clamped so
// that the reciprocal stays finite.
__device__ __forceinline__ int sturm_count(const double* d, const double* ee, int p, double x,
                                           double pivmin) {
  const double big = 1e300;
  double q = d[0] - x;
  if (fabs(q) <= pivmin) q = -pivmin;
  int c = q < 0.0;
#pragma unroll 8
  for (int i = 1; i < p; ++i) {
    q = fmin(fmax(q, -big), big);
    q = (d[i] - x) - ee[i - 1] * recip(q);
    if (fabs(q) <= pivmin) q = -pivmin;
    c += q < 0.0;
  }
  return c;
}

constexpr int BIS_WAVES = 4;

__global__ __launch_bounds__(64 * BIS_WAVES) void bisect_kernel(double* __restrict__ Ball,
                                                                double* __restrict__ ws, int p,
                                                                int rc) {
  extern __shared__ double shb[];
  const int mode = blockIdx.y;
  EigWs W(ws, p, rc, mode);
  double* d = shb;
  double* ee = shb + p;
  for (int i = threadIdx.x; i < p; i += blockDim.x) {
    d[i] = W.d[i];
    ee[i] = W.e[i] * W.e[i];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * BIS_WAVES + (threadIdx.x >> 6);   // j-th largest eigenvalue
  if (j >= p) return;
  // Gershgorin interval and pivot floor, reduced over the wave
  double gl = HUGE_VAL, gu = -HUGE_VAL, emax = 0.0;
  for (int i = lane; i < p; i += 64) {
    const double r = (i > 0 ? fabs(W.e[i - 1]) : 0.0) + (i + 1 < p ? fabs(W.e[i]) : 0.0);
    gl = fmin(gl, d[i] - r);
    gu = fmax(gu, d[i] + r);
    emax = fmax(emax, ee[i]);
  }
  for (int off = 32; off > 0; off >>= 1) {
    gl = fmin(gl, __shfl_xor(gl, off));
    gu = fmax(gu, __shfl_xor(gu, off));
    emax = fmax(emax, __shfl_xor(emax, off));
  }
  const double u = 1.1102230246251565e-16;
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax);
  const double tn = fmax(fabs(gl), fabs(gu));
  const double pad = 2.0 * u * tn * (double)p + 2.0 * pivmin;
  double lo = gl - pad, hi = gu + pad;
  const int m = p - 1 - j;   // ascending index: count(x) <= m below lambda_m, > m above
  const double tol = 4.0 * u * tn + 2.0 * pivmin;
  for (int round = 0; round < 24 && hi - lo > tol; ++round) {
    const double x = lo + (hi - lo) * ((double)(lane + 1) / 65.0);
    const int c = sturm_count(d, ee, p, x, pivmin);
    const uint64_t above = __ballot(c > m);
    if (above == 0) {
      lo = __shfl(x, 63);
    } else {
      const int f = __ffsll((unsigned long long)above) - 1;
      const double xf = __shfl(x, f);
      const double xb = __shfl(x, f > 0 ? f - 1 : 0);
      if (f > 0) lo = xb;
      hi = xf;
    }
  }
  if (lane == 0) {
    const double lam = 0.5 * (lo + hi);
    W.lam[j] = lam;
    Ball[(int64_t)mode * p * p + (int64_t)j * p + j] = lam;
  }
}

// Thread j < rc: z_j solves (T - lambda_j I)^3 z = hashed start vector, with
// the pivots of the LU factorisation (no pivoting) kept away from zero by
// u ||T||; each solve is rescaled by its largest entry; final unit norm.
// The recurrences run over chunks of IC rows whose loads are issued before
// the chunk's dependent chain, so each chunk waits on memory once.
constexpr int IC = 16;

__global__ __launch_bounds__(256) void invit_kernel(double* __restrict__ ws,
                                                    double* __restrict__ Zall, int p, int rc,
                                                    uint64_t seed) {
  const int mode = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= rc) return;
  EigWs W(ws, p, rc, mode);
  const double lam = W.lam[j];
  const double u = 1.1102230246251565e-16;
  const double tiny = u * fmax(fmax(fabs(W.lam[0]), fabs(W.lam[p - 1])), 1e-280);
  const double* __restrict__ dg = W.d;
  const double* __restrict__ eg = W.e;
  double* __restrict__ lm = W.lm + j;
  double* __restrict__ ru = W.ru + j;
  double* __restrict__ z = Zall + (int64_t)mode * p * rc + j;
  const int64_t ld = rc;
  // LU of T - lambda I: u_0 = d_0 - lambda, l_i = e_{i-1} / u_{i-1},
  // u_i = d_i - lambda - l_i e_{i-1}; the reciprocal pivots are stored
  double rprev = 0.0;
  for (int i0 = 0; i0 < p; i0 += IC) {
    double dd[IC], ee[IC], ll[IC], rr[IC];
#pragma unroll
    for (int c = 0; c < IC; ++c) {
      const int i = i0 + c;
      dd[c] = i < p ? dg[i] : 0.0;
      ee[c] = (i > 0 && i < p) ? eg[i - 1] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < IC; ++c) {
      const double l = ee[c] * rprev;
      double up = (dd[c] - lam) - l * ee[c];
      if (fabs(up) < tiny) up = up < 0.0 ? -tiny : tiny;
      rprev = 1.0 / up;
      ll[c] = l;
      rr[c] = rprev;
    }
#pragma unroll
    for (int c = 0; c < IC; ++c) {
      const int i = i0 + c;
      if (i < p) {
        lm[i * ld] = ll[c];
        ru[i * ld] = rr[c];
        z[i * ld] = hash_uniform(seed + mode, (uint64_t)j, (uint64_t)i);
      }
    }
  }
  double scale = 1.0;
  const int last = ((p - 1) / IC) * IC;   // start of the last chunk
  for (int it = 0; it < 3; ++it) {
    // forward: L y = scale z (l_0 = 0)
    double prev = 0.0;
    for (int i0 = 0; i0 < p; i0 += IC) {
      double zz[IC], ll[IC];
#pragma unroll
      for (int c = 0; c < IC; ++c) {
        const int i = i0 + c;
        zz[c] = i < p ? z[i * ld] : 0.0;
        ll[c] = i < p ? lm[i * ld] : 0.0;
      }
#pragma unroll
      for (int c = 0; c < IC; ++c) {
        prev = scale * zz[c] - ll[c] * prev;
        zz[c] = prev;
      }
#pragma unroll
      for (int c = 0; c < IC; ++c) {
        const int i = i0 + c;
        if (i < p) z[i * ld] = zz[c];
      }
    }
    // backward: U x = y, U = upper bidiagonal (u_i, e_i), e_{p-1} = 0
    double nxt = 0.0, mx = 0.0;
    for (int i0 = last; i0 >= 0; i0 -= IC) {
      double zz[IC], rr[IC], ee[IC];
#pragma unroll
      for (int c = 0; c < IC; ++c) {
        const int i = i0 + c;
        zz[c] = i < p ? z[i * ld] : 0.0;
        rr[c] = i < p ? ru[i * ld] : 0.0;
        ee[c] = i < p ? eg[i] : 0.0;
      }
#pragma unroll
      for (int c = IC - 1; c >= 0; --c) {
        if (i0 + c < p) {
          nxt = (zz[c] - ee[c] * nxt) * rr[c];
          zz[c] = nxt;
          mx = fmax(mx, fabs(nxt));
        }
      }
#pragma unroll
      for (int c = 0; c < IC; ++c) {
        const int i = i0 + c;
        if (i < p) z[i * ld] = zz[c];
      }
    }
    scale = mx > 0.0 ? 1.0 / mx : 1.0;
  }
  // unit norm; chunks of IC loads issued together, the sum in row order
  double nrm = 0.0;
  for (int i0 = 0; i0 < p; i0 += IC) {
    double zz[IC];
#pragma unroll
    for (int c = 0; c < IC; ++c) zz[c] = i0 + c < p ? z[(i0 + c) * ld] : 0.0;
#pragma unroll
    for (int c = 0; c < IC; ++c)
      if (i0 + c < p) {
        const double v = scale * zz[c];
        nrm += v * v;
      }
  }
  const double s = nrm > 0.0 ? scale / sqrt(nrm) : 0.0;
  for (int i0 = 0; i0 < p; i0 += IC) {
    double zz[IC];
#pragma unroll
    for (int c = 0; c < IC; ++c) zz[c] = i0 + c < p ? z[(i0 + c) * ld] : 0.0;
#pragma unroll
    for (int c = 0; c < IC; ++c)
      if (i0 + c < p) z[(i0 + c) * ld] = zz[c] * s;
  }
}

// The same inverse iteration with the per-vector arrays in LDS ([array][i][t],
// t the thread, so that a wavefront touches consecutive words) for TPB
// vectors per workgroup; d and e are shared.
template <int TPB>
__global__ __launch_bounds__(TPB) void invit_lds_kernel(double* __restrict__ ws,
                                                        double* __restrict__ Zall, int p, int rc,
                                                        uint64_t seed) {
  extern __shared__ double shi[];
  const int mode = blockIdx.y;
  const int t = threadIdx.x;
  EigWs W(ws, p, rc, mode);
  double* dS = shi;
  double* eS = shi + p;
  double* lm = shi + 2 * p + t;
  double* ru = lm + (int64_t)p * TPB;
  double* z = ru + (int64_t)p * TPB;
  for (int i = t; i < p; i += TPB) {
    dS[i] = W.d[i];
    eS[i] = W.e[i];
  }
  __syncthreads();
  const int j = blockIdx.x * TPB + t;
  if (j >= rc) return;
  const double lam = W.lam[j];
  const double u = 1.1102230246251565e-16;
  const double tiny = u * fmax(fmax(fabs(W.lam[0]), fabs(W.lam[p - 1])), 1e-280);
  double up = dS[0] - lam;
  if (fabs(up) < tiny) up = up < 0.0 ? -tiny : tiny;
  double rprev = recip(up);
  lm[0] = 0.0;
  ru[0] = rprev;
  // unrolled so that the LDS loads of a chunk precede its dependent chain
#pragma unroll 8
  for (int i = 1; i < p; ++i) {
    const double ei = eS[i - 1];
    const double l = ei * rprev;
    up = (dS[i] - lam) - l * ei;
    if (fabs(up) < tiny) up = up < 0.0 ? -tiny : tiny;
    rprev = recip(up);
    lm[i * TPB] = l;
    ru[i * TPB] = rprev;
  }
  for (int i = 0; i < p; ++i) z[i * TPB] = hash_uniform(seed + mode, (uint64_t)j, (uint64_t)i);
  double scale = 1.0;
  for (int it = 0; it < 3; ++it) {
    double prev = 0.0;
#pragma unroll 8
    for (int i = 0; i < p; ++i) {
      prev = scale * z[i * TPB] - lm[i * TPB] * prev;
      z[i * TPB] = prev;
    }
    double nxt = 0.0, mx = 0.0;
#pragma unroll 8
    for (int i = p - 1; i >= 0; --i) {
      nxt = (z[i * TPB] - eS[i] * nxt) * ru[i * TPB];
      z[i * TPB] = nxt;
      mx = fmax(mx, fabs(nxt));
    }
    scale = mx > 0.0 ? 1.0 / mx : 1.0;
  }
  double nrm = 0.0;
#pragma unroll 8
  for (int i = 0; i < p; ++i) {
    const double v = scale * z[i * TPB];
    nrm += v * v;
  }
  const double sc = nrm > 0.0 ? scale / sqrt(nrm) : 0.0;
  double* zg = Zall + (int64_t)mode * p * rc + j;
  for (int i = 0; i < p; ++i) zg[(int64_t)i * rc] = z[i * TPB] * sc;
}

// Z (p x rc row-major per mode) <- H_0 H_1 ... H_{p-3} Z, H_k = I - beta_k v_k v_k^T:
// one wave per column, the column in registers (lane l keeps rows l, l + 64, ...).
template <int UPL>
__global__ __launch_bounds__(256) void reflect_cols_kernel(double* __restrict__ Zall,
                                                           double* __restrict__ ws, int p,
                                                           int rc) {
  const int mode = blockIdx.y;
  const int col = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (col >= rc) return;
  EigWs W(ws, p, rc, mode);
  double* Z = Zall + (int64_t)mode * p * rc + col;
  double y[UPL];
#pragma unroll
  for (int u = 0; u < UPL; ++u) {
    const int i = lane + 64 * u;
    y[u] = i < p ? Z[(int64_t)i * rc] : 0.0;
  }
  // reflectors in blocks of D (k = kb, kb - 1, ...); the next block's vectors
  // are loaded while the current block is applied
  constexpr int D = UPL <= 4 ? 8 : UPL <= 8 ? 4 : 2;
  auto load_block = [&](int kb, double (&vb)[D][UPL], double (&bb)[D]) {
#pragma unroll
    for (int t = 0; t < D; ++t) {
      const int k = kb - t;
      bb[t] = k >= 0 ? W.beta[k] : 0.0;
      const double* v = W.hv + (int64_t)(k >= 0 ? k : 0) * p;
#pragma unroll
      for (int u = 0; u < UPL; ++u) {
        const int i = lane + 64 * u;
        vb[t][u] = k < 0 ? 0.0 : (i == k + 1 ? 1.0 : ((i >= k + 2 && i < p) ? v[i] : 0.0));
      }
    }
  };
  double cv[D][UPL], cb[D];
  load_block(p - 3, cv, cb);
  for (int kb = p - 3; kb >= 0; kb -= D) {
    double nv[D][UPL], nb[D];
    load_block(kb - D, nv, nb);
#pragma unroll
    for (int t = 0; t < D; ++t) {
      if (cb[t] == 0.0) continue;
      double part = 0.0;
#pragma unroll
      for (int u = 0; u < UPL; ++u) part = fma(cv[t][u], y[u], part);
      const double dot = cb[t] * wave_sum_dpp(part);
#pragma unroll
      for (int u = 0; u < UPL; ++u) y[u] = fma(-dot, cv[t][u], y[u]);
    }
#pragma unroll
    for (int t = 0; t < D; ++t) {
      cb[t] = nb[t];
#pragma unroll
      for (int u = 0; u < UPL; ++u) cv[t][u] = nv[t][u];
    }
  }
#pragma unroll
  for (int u = 0; u < UPL; ++u) {
    const int i = lane + 64 * u;
    if (i < p) Z[(int64_t)i * rc] = y[u];
  }
}

void launch_eig_tridiag(double* B, double* ws, int p, int rc, int modes, int lds_limit,
                        hipStream_t s) {
  if (p <= 64) {
    hipLaunchKernelGGL(tridiag_reg_kernel<4>, dim3(modes), dim3(256), 0, s, B, ws, p, rc);
    return;
  }
  if (p <= 128) {
    hipLaunchKernelGGL(tridiag_reg_kernel<8>, dim3(modes), dim3(256), 0, s, B, ws, p, rc);
    return;
  }
  const size_t tri_lds = ((size_t)p * (p + 1) + (size_t)p) * sizeof(double);
  const size_t wide_lds = (size_t)(TW_WAVES + 2) * p * sizeof(double);
  if (p <= 512 && launch_tridiag_dist(B, ws, p, rc, modes, s)) return;
  if (p <= 64 * TW_MAXA && wide_lds + 1024 <= (size_t)lds_limit) {
    allow_lds((const void*)tridiag_wide_kernel, wide_lds);
    hipLaunchKernelGGL(tridiag_wide_kernel, dim3(modes), dim3(TW_THREADS), wide_lds, s, B, ws, p,
                       rc);
  } else if (tri_lds + 1024 <= (size_t)lds_limit) {
    allow_lds((const void*)tridiag_kernel<true>, tri_lds);
    hipLaunchKernelGGL(tridiag_kernel<true>, dim3(modes), dim3(ES_THREADS), tri_lds, s, B, ws, p,
                       rc);
  } else {
    const size_t bytes = (size_t)p * sizeof(double);
    hipLaunchKernelGGL(tridiag_kernel<false>, dim3(modes), dim3(ES_THREADS), bytes, s, B, ws, p,
                       rc);
  }
}

void launch_eig_values_vectors(double* B, double* ws, double* Z, int p, int rc, int modes,
                               int lds_limit, hipStream_t s) {
  if (rc < 1 || rc > p) throw Error{RS_E_INVALID, "eigensolver: wanted vectors outside [1, p]"};
  hipLaunchKernelGGL(bisect_kernel, dim3((unsigned)((p + BIS_WAVES - 1) / BIS_WAVES), modes),
                     dim3(64 * BIS_WAVES), 2 * (size_t)p * sizeof(double), s, B, ws, p, rc);
  constexpr int TPB = 32;
  const size_t inv_lds = ((size_t)2 * p + (size_t)3 * p * TPB) * sizeof(double);
  if (inv_lds + 1024 <= (size_t)lds_limit) {
    allow_lds((const void*)invit_lds_kernel<TPB>, inv_lds);
    hipLaunchKernelGGL(invit_lds_kernel<TPB>, dim3((unsigned)((rc + TPB - 1) / TPB), modes),
                       dim3(TPB), inv_lds, s, ws, Z, p, rc, 0x1a2b3c4d5e6fULL);
  } else {
    hipLaunchKernelGGL(invit_kernel, dim3((unsigned)((rc + 255) / 256), modes), dim3(256), 0, s,
                       ws, Z, p, rc, 0x1a2b3c4d5e6fULL);
  }
}

void launch_eig_backtransform(double* Z, double* ws, int p, int rc, int modes, hipStream_t s) {
  const dim3 grid((unsigned)((rc + 3) / 4), modes);
  if (p <= 64) hipLaunchKernelGGL(reflect_cols_kernel<1>, grid, dim3(256), 0, s, Z, ws, p, rc);
  else if (p <= 128) hipLaunchKernelGGL(reflect_cols_kernel<2>, grid, dim3(256), 0, s, Z, ws, p, rc);
  else if (p <= 256) hipLaunchKernelGGL(reflect_cols_kernel<4>, grid, dim3(256), 0, s, Z, ws, p, rc);
  else if (p <= 512) hipLaunchKernelGGL(reflect_cols_kernel<8>, grid, dim3(256), 0, s, Z, ws, p, rc);
  else if (p <= 1024) hipLaunchKernelGGL(reflect_cols_kernel<16>, grid, dim3(256), 0, s, Z, ws, p, rc);
  else throw Error{RS_E_UNSUPPORTED, "eigensolver subspace above 1024"};
}

}  // namespace rs
