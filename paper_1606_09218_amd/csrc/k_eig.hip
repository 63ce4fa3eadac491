// FP64 dominant-eigenspace solver for the charge-weighted Gram matrices.
//
// The RHOSVD keeps the dominant left singular vectors of each side matrix
// (Appendix step (I), eq SVD_SideMatr).  They are the dominant eigenvectors
// of G_l = U_l diag(w) U_l^T.  With a rapidly decaying spectrum a subspace
// of p = r + oversample columns captures them:
//   Y = U_l diag(|xi|^{1/3}) Omega, Q = orth(Y), [Y = G Q, Q = orth(Y)]^q, B = Q^T G Q,
//   B = W Lambda W^T (tridiagonalisation + implicit QR), V = Q W (sorted, truncated).
// The subspace comes from a sketch of the charge-weighted side matrix (the
// range finder of Halko, Martinsson and Tropp) orthonormalised by shifted
// Cholesky QR.  Everything is FP64.  Each small kernel runs one workgroup per
// mode.
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
  // NaN (from invalid input, rejected by the host afterwards) orders as -inf
  // so that perm is always a permutation of 0..p-1
  for (int i = threadIdx.x; i < p; i += EIG_THREADS) {
    double li = B[(int64_t)i * p + i];
    if (li != li) li = -HUGE_VAL;
    int rank = 0;
    for (int j = 0; j < p; ++j) {
      double lj = B[(int64_t)j * p + j];
      if (lj != lj) lj = -HUGE_VAL;
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
  hipLaunchKernelGGL(rank_select_kernel, dim3(modes), dim3(EIG_THREADS), 0, s, B, p, eps2, fixed,
                     r_max, perm, info_dev);
}

// Wr (p x r col-major) = V[:, perm[0..r)]
__global__ void gather_cols_kernel(const double* __restrict__ V, const int* __restrict__ perm,
                                   int p, int r, double* __restrict__ Wr) {
  int64_t total = (int64_t)p * r;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    int col = (int)(e / p), row = (int)(e % p);
    Wr[e] = V[(int64_t)perm[col] * p + row];
  }
}

void launch_gather_cols(const double* V, const int* perm, int p, int r, double* Wr,
                        hipStream_t s) {
  int64_t total = (int64_t)p * r;
  unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(gather_cols_kernel, dim3(blocks), dim3(256), 0, s, V, perm, p, r, Wr);
}

// One wave per column of the row-major n x r matrix: find the entry of
// largest magnitude (first on ties) and flip the column if it is negative.
__global__ void canonical_signs_kernel(double* Q, int64_t n, int r) {
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
  if (flip)
    for (int64_t i = lane; i < n; i += 64) Q[i * r + col] = -Q[i * r + col];
}

void launch_canonical_signs(double* Qrow, int64_t n, int r, hipStream_t s) {
  hipLaunchKernelGGL(canonical_signs_kernel, dim3(r), dim3(64), 0, s, Qrow, n, r);
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
                                                          int* __restrict__ fail) {
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
      if (tid == 0) atomicOr(fail, 1);
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

// Y[i, :] <- Y[i, :] L^{-T} for row-major Y (n x p): one wave per row, the
// row held in registers (lane l keeps entries l, l + 64, ...), right-looking
// substitution: x_c = y_c / L_cc is broadcast from its lane, then every lane
// subtracts x_c L[i, c] from its entries i > c.  L (lower, column-major) is
// staged in LDS packed by columns so that the lanes read consecutive words.
template <int RPL, bool LDS>
__global__ __launch_bounds__(1024) void trsm_rows_kernel(double* __restrict__ Yall,
                                                         const double* __restrict__ Lall,
                                                         int64_t n, int p) {
  extern __shared__ double sht[];
  const int mode = blockIdx.y;
  const double* L = Lall + (int64_t)mode * p * p;
  // LDS: column c holds L[c..p-1, c] at offset c p - c (c - 1) / 2; global:
  // column c of the column-major L starts at c p + c.  Either way Lc[i - c] = L[i, c].
  if (LDS) {
    for (int e = threadIdx.x; e < p * p; e += blockDim.x) {
      const int c = e / p, i = e - c * p;
      if (i >= c) sht[c * p - c * (c - 1) / 2 + (i - c)] = L[e];
    }
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
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    for (int cc = 0; cc < 64; ++cc) {
      const int c = 64 * u + cc;
      if (c >= p) break;
      const double* Lc = LDS ? sht + c * p - c * (c - 1) / 2 : L + (int64_t)c * p + c;
      const double x = __shfl(y[u], cc) / Lc[0];
      if (lane == cc) y[u] = x;
      if (lane > cc) {
        const int i = 64 * u + lane;
        if (i < p) y[u] -= x * Lc[i - c];
      }
#pragma unroll
      for (int u2 = u + 1; u2 < RPL; ++u2) {
        const int i = 64 * u2 + lane;
        if (i < p) y[u2] -= x * Lc[i - c];
      }
    }
  }
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    const int c = lane + 64 * u;
    if (c < p) Y[c] = y[u];
  }
}

// kernels that use more than the default dynamic LDS opt in to the device limit
static void allow_lds(const void* fn, size_t bytes) {
  if (bytes > 48 * 1024)
    RS_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

void launch_chol(double* C, int p, int64_t nrows, int modes, int shifted, int lds_limit, int* fail,
                 hipStream_t s) {
  const size_t bytes = (size_t)p * p * sizeof(double);
  if (bytes + 1024 <= (size_t)lds_limit) {
    allow_lds((const void*)chol_kernel<true>, bytes);
    hipLaunchKernelGGL(chol_kernel<true>, dim3(modes), dim3(CF_THREADS), bytes, s, C, p, nrows,
                       shifted, fail);
  } else {
    hipLaunchKernelGGL(chol_kernel<false>, dim3(modes), dim3(CF_THREADS), 0, s, C, p, nrows,
                       shifted, fail);
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
  const size_t bytes = (size_t)p * (p + 1) / 2 * sizeof(double);
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

void launch_perturb(double* Y, const double* G, int64_t n, int p, int modes, uint64_t seed,
                    hipStream_t s) {
  const int64_t total = n * p;
  unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 2048);
  hipLaunchKernelGGL(perturb_kernel, dim3(blocks, modes), dim3(256), 0, s, Y, G, n, p, seed);
}

// ---- dense symmetric eigensolver: tridiagonalisation + implicit QR -------------
// One workgroup per mode computes B = V diag(lambda) V^T for the p x p
// Rayleigh-Ritz matrix:
//  1. Householder tridiagonalisation Q^T B Q = T (Golub & Van Loan, Alg. 8.3.1);
//     the Householder vectors are kept below the subdiagonal of B.
//  2. Implicit symmetric QR steps with the Wilkinson shift on T (GVL Alg. 8.3.2,
//     8.3.3), deflating negligible off-diagonal entries; thread 0 chases the
//     bulge of one QR step and records its Givens rotations, then every thread
//     applies them to its rows of Z (a sliding window along the row).
//  3. Back-transformation V = Q Z, one thread per column (columns independent).
// B and Z live in LDS when p x p FP64 fits (Z reuses B's space after the
// Householder vectors are copied out), else in global memory.
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

template <bool LDS>
__global__ __launch_bounds__(ES_THREADS) void eig_sym_kernel(double* __restrict__ Ball,
                                                             double* __restrict__ Vall,
                                                             double* __restrict__ HVall, int p,
                                                             int* __restrict__ fail,
                                                             double* __restrict__ profall) {
  extern __shared__ double sh[];
  __shared__ double red[ES_THREADS / 64];
  __shared__ double v1_s, kc_s;
  __shared__ int lo_s, hi_s, done_s;
  const int mode = blockIdx.x;
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  double* Bg = Ball + (int64_t)mode * p * p;
  double* Vg = Vall + (int64_t)mode * p * p;
  double* HV = HVall + (int64_t)mode * ((int64_t)p * p + p);   // p x p vectors + p betas
  const int ldb = LDS ? p + 1 : p;                              // padded against bank conflicts
  double* B = LDS ? sh : Bg;                                    // row-major B(i, j) = B[i ldb + j]
  double* vec = LDS ? sh + (int64_t)p * (p + 1) : sh;           // 6 p doubles after Z's padded extent
  double* d = vec;
  double* e = vec + p;
  double* pw = vec + 2 * p;
  double* cs = vec + 3 * p;
  double* sn = vec + 4 * p;
  double* betas = vec + 5 * p;
  const int pp = p * p;
  // wall-clock stamps (constant-rate counter) at the phase boundaries, when asked
  double* prof = profall ? profall + 4 * mode : nullptr;
  if (prof && tid == 0) prof[0] = (double)wall_clock64();
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

  // 1. tridiagonalisation
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
  }
  // Householder vectors out of the way (column k, rows k+2..p-1; kept in HV)
  for (int x = tid; x < pp; x += ES_THREADS) {
    const int i = x / p, k = x - i * p;
    if (i >= k + 2) HV[(int64_t)k * p + i] = B[i * ldb + k];
  }
  for (int x = tid; x < p; x += ES_THREADS) HV[(int64_t)pp + x] = betas[x];
  __syncthreads();

  if (prof && tid == 0) prof[1] = (double)wall_clock64();
  // 2. Z = I, row-major with padded stride
  const int ldz = LDS ? p + 1 : p;
  double* Z = LDS ? sh : Vg;
  for (int x = tid; x < p * ldz; x += ES_THREADS) {
    const int i = x / ldz, j = x - i * ldz;
    Z[x] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();

  // 3. implicit symmetric QR with Wilkinson shifts
  const double eps = 1.1102230246251565e-16;
  int hi = p - 1;
  int iters = 0;
  for (;;) {
    if (tid == 0) {
      int done = 0;
      while (hi > 0 && fabs(e[hi - 1]) <= eps * (fabs(d[hi - 1]) + fabs(d[hi]))) {
        e[hi - 1] = 0.0;
        --hi;
      }
      if (hi == 0 || iters > 30 * p) {
        if (hi > 0) atomicOr(fail, 2);
        done = 1;
      } else {
        int lo = hi - 1;
        while (lo > 0 && fabs(e[lo - 1]) > eps * (fabs(d[lo - 1]) + fabs(d[lo]))) --lo;
        if (lo > 0) e[lo - 1] = 0.0;
        // Wilkinson shift from the trailing 2 x 2 block
        const double bb = e[hi - 1];
        const double dd = 0.5 * (d[hi - 1] - d[hi]);
        const double den = dd + (dd >= 0.0 ? 1.0 : -1.0) * sqrt(dd * dd + bb * bb);
        const double mu = den != 0.0 ? d[hi] - bb * bb / den : d[hi];
        double x = d[lo] - mu, z = e[lo];
        // carried in registers: a = current d[k], bk = current e[k]; the
        // untouched d[k+1], e[k+1] are read one step ahead
        double a = d[lo], bk = e[lo];
        double dn = d[lo + 1], en = (lo + 1 < hi) ? e[lo + 1] : 0.0;
        for (int k = lo; k < hi; ++k) {
          const double ak1 = dn, ek1 = en;
          if (k + 2 <= hi) dn = d[k + 2];
          if (k + 2 < hi) en = e[k + 2];
          const double q2 = x * x + z * z;
          double c = 1.0, s = 0.0, r = 0.0;
          if (q2 > 0.0) {
            const double ri = rsqrt(q2);
            c = x * ri;
            s = z * ri;
            r = q2 * ri;
          }
          if (k > lo) e[k - 1] = r;
          const double cc = c * c, ss = s * s, cs2 = 2.0 * c * s * bk;
          d[k] = cc * a + cs2 + ss * ak1;
          const double dk1 = ss * a - cs2 + cc * ak1;
          const double ek = c * s * (ak1 - a) + (cc - ss) * bk;
          e[k] = ek;
          a = dk1;
          if (k + 1 < hi) {
            x = ek;
            z = s * ek1;
            bk = c * ek1;
          }
          cs[k] = c;
          sn[k] = s;
        }
        d[hi] = a;
        lo_s = lo;
        hi_s = hi;
        ++iters;
      }
      done_s = done;
    }
    __syncthreads();
    if (done_s) break;
    const int lo = lo_s, h = hi_s;
    for (int row = tid; row < p; row += ES_THREADS) {
      double* zr = Z + (int64_t)row * ldz;
      double zc = zr[lo];
      for (int k = lo; k < h; ++k) {
        const double zn = zr[k + 1];
        const double c = cs[k], s = sn[k];
        zr[k] = c * zc + s * zn;
        zc = -s * zc + c * zn;
      }
      zr[h] = zc;
    }
    __syncthreads();
  }

  if (prof && tid == 0) prof[2] = (double)wall_clock64();
  // 4. back-transformation Z <- H_0 H_1 ... H_{p-3} Z: v_k staged in LDS,
  //    one thread per column
  double* vk = pw;
  double* part_lo = cs;   // partial dots over the lower half of the rows (cs, sn are free now)
  double* part_hi = sn;   // partial dots over the upper half
  for (int k = p - 3; k >= 0; --k) {
    const double beta = HV[(int64_t)pp + k];   // uniform
    if (beta == 0.0) continue;
    for (int i = k + 1 + tid; i < p; i += ES_THREADS)
      vk[i] = i == k + 1 ? 1.0 : HV[(int64_t)k * p + i];
    __syncthreads();
    const int mid = (k + 1 + p) / 2;
    // thread t < 128 sums rows [k+1, mid), thread t + 128 rows [mid, p) of column t
    for (int col = tid & 127; col < p; col += 128) {
      const int i0 = tid < 128 ? k + 1 : mid, i1 = tid < 128 ? mid : p;
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int i = i0;
      for (; i + 3 < i1; i += 4) {
        s0 += vk[i] * Z[(int64_t)i * ldz + col];
        s1 += vk[i + 1] * Z[(int64_t)(i + 1) * ldz + col];
        s2 += vk[i + 2] * Z[(int64_t)(i + 2) * ldz + col];
        s3 += vk[i + 3] * Z[(int64_t)(i + 3) * ldz + col];
      }
      for (; i < i1; ++i) s0 += vk[i] * Z[(int64_t)i * ldz + col];
      if (tid >= 128) part_hi[col] = (s0 + s1) + (s2 + s3);
      else part_lo[col] = (s0 + s1) + (s2 + s3);
    }
    __syncthreads();
    for (int col = tid & 127; col < p; col += 128) {
      const double dot = beta * (part_lo[col] + part_hi[col]);
      const int i0 = tid < 128 ? k + 1 : mid, i1 = tid < 128 ? mid : p;
      for (int i = i0; i < i1; ++i) Z[(int64_t)i * ldz + col] -= dot * vk[i];
    }
    __syncthreads();
  }
  if (prof && tid == 0) prof[3] = (double)wall_clock64();
  // 5. eigenvalues on the diagonal of B, eigenvectors to V (column-major)
  for (int x = tid; x < p; x += ES_THREADS) Bg[(int64_t)x * p + x] = d[x];
  if (LDS) {
    for (int x = tid; x < pp; x += ES_THREADS) {
      const int c = x / p, r = x - c * p;
      Vg[x] = Z[(int64_t)r * ldz + c];
    }
  } else {
    // Z (row-major) is in Vg: transpose in place to column-major
    __syncthreads();
    for (int x = tid; x < pp; x += ES_THREADS) {
      const int r = x / p, c = x - r * p;
      if (c > r) {
        const double a = Vg[(int64_t)r * p + c], b2 = Vg[(int64_t)c * p + r];
        Vg[(int64_t)r * p + c] = b2;
        Vg[(int64_t)c * p + r] = a;
      }
    }
  }
}

void launch_eig_sym(double* B, double* V, double* HV, int p, int modes, int lds_limit, int* fail,
                    double* prof, hipStream_t s) {
  const size_t lds_bytes = ((size_t)p * (p + 1) + 6 * (size_t)p) * sizeof(double);
  if (lds_bytes + 1024 <= (size_t)lds_limit) {
    allow_lds((const void*)eig_sym_kernel<true>, lds_bytes);
    hipLaunchKernelGGL(eig_sym_kernel<true>, dim3(modes), dim3(ES_THREADS), lds_bytes, s, B, V, HV,
                       p, fail, prof);
  } else {
    const size_t bytes = 6 * (size_t)p * sizeof(double);
    allow_lds((const void*)eig_sym_kernel<false>, bytes);
    hipLaunchKernelGGL(eig_sym_kernel<false>, dim3(modes), dim3(ES_THREADS), bytes, s, B, V, HV, p,
                       fail, prof);
  }
}

}  // namespace rs
