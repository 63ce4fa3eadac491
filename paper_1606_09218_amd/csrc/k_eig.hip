// FP64 dominant-eigenspace solver for the charge-weighted Gram matrices.
//
// The RHOSVD keeps the dominant left singular vectors of each side matrix
// (Appendix step (I), eq SVD_SideMatr).  They are the dominant eigenvectors
// of G_l = U_l diag(w) U_l^T.  With a rapidly decaying spectrum a subspace
// of p = r + oversample columns captures them:
//   Y = G Omega, Q = orth(Y), [Y = G Q, Q = orth(Y)]^q, B = Q^T G Q,
//   B = W Lambda W^T (cyclic parallel Jacobi), V = Q W (sorted, truncated).
// Everything is FP64.  Each small kernel runs one workgroup per mode.
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

__global__ void omega_kernel(double* Om, int64_t n, int p, uint64_t seed) {
  const int mode = blockIdx.y;
  const int64_t total = n * p;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x)
    Om[mode * total + e] = hash_uniform(seed + mode, (uint64_t)(e % n), (uint64_t)(e / n));
}

void launch_fill_omega(double* Om, int64_t n, int p, int modes, uint64_t seed, hipStream_t s) {
  int64_t total = n * p;
  unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(omega_kernel, dim3(blocks, modes), dim3(256), 0, s, Om, n, p, seed);
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

// ---- classical Gram-Schmidt with reorthogonalisation ------------------------
// One workgroup per mode; the working column lives in LDS (n <= 2048).
__global__ __launch_bounds__(EIG_THREADS) void cgs2_kernel(const double* __restrict__ Yall,
                                                           double* __restrict__ Qall, int64_t n,
                                                           int p, uint64_t seed) {
  extern __shared__ double sh[];
  double* v = sh;            // n
  double* c = sh + n;        // p coefficients
  __shared__ double red[EIG_WAVES];
  const int mode = blockIdx.x;
  const double* Y = Yall + (int64_t)mode * n * p;
  double* Q = Qall + (int64_t)mode * n * p;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  for (int j = 0; j < p; ++j) {
    for (int64_t i = tid; i < n; i += EIG_THREADS) v[i] = Y[(int64_t)j * n + i];
    __syncthreads();
    double acc = 0.0;
    for (int64_t i = tid; i < n; i += EIG_THREADS) acc += v[i] * v[i];
    double nrm0 = sqrt(block_sum(acc, red));
    double nrm = nrm0;
    for (int attempt = 0; attempt < 2; ++attempt) {
      if (nrm0 == 0.0 || attempt == 1) {
        // zero column, or a column lost to cancellation: restart from a
        // deterministic pseudo-random vector
        for (int64_t i = tid; i < n; i += EIG_THREADS)
          v[i] = hash_uniform(seed + 7919 * (mode + 1), (uint64_t)i, (uint64_t)j + 1000003ULL);
        __syncthreads();
        acc = 0.0;
        for (int64_t i = tid; i < n; i += EIG_THREADS) acc += v[i] * v[i];
        nrm0 = sqrt(block_sum(acc, red));
        nrm = nrm0;
      }
      for (int pass = 0; pass < 3 && j > 0; ++pass) {
        // c = Q[:, :j]^T v : one wave per column, lanes over rows
        for (int k = wave; k < j; k += EIG_WAVES) {
          double d = 0.0;
          for (int64_t i = lane; i < n; i += 64) d += Q[(int64_t)k * n + i] * v[i];
          d = wave_sum(d);
          if (lane == 0) c[k] = d;
        }
        __syncthreads();
        for (int64_t i = tid; i < n; i += EIG_THREADS) {
          double s = 0.0;
          for (int k = 0; k < j; ++k) s += Q[(int64_t)k * n + i] * c[k];
          v[i] -= s;
        }
        __syncthreads();
        acc = 0.0;
        for (int64_t i = tid; i < n; i += EIG_THREADS) acc += v[i] * v[i];
        double nn = sqrt(block_sum(acc, red));
        bool done = pass >= 1 && nn > 0.5 * nrm;  // "twice is enough"
        nrm = nn;
        if (done) break;
      }
      if (nrm > 1e-300 && nrm > 1e-30 * nrm0) break;
    }
    const double inv = 1.0 / nrm;
    for (int64_t i = tid; i < n; i += EIG_THREADS) Q[(int64_t)j * n + i] = v[i] * inv;
    __syncthreads();
  }
}

void launch_cgs2(const double* Y, double* Q, int64_t n, int p, int modes, uint64_t seed,
                 hipStream_t s) {
  size_t shm = (size_t)(n + p) * sizeof(double);
  hipLaunchKernelGGL(cgs2_kernel, dim3(modes), dim3(EIG_THREADS), shm, s, Y, Q, n, p, seed);
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

// ---- cyclic parallel Jacobi ----------------------------------------------------
// Round-robin ordering: in round s (0..p-2) the pairs are (p-1, s) and
// ((s+m) mod (p-1), (s-m) mod (p-1)) for m = 1..p/2-1; every pair of indices
// meets once per sweep and the p/2 rotations of a round are disjoint, so the
// two-sided update acts on independent 2 x 2 blocks.  One workgroup per mode;
// B and V (p x p) stay in global memory (L2 resident).
__device__ __forceinline__ void round_pair(int p, int s, int m, int& i, int& j) {
  const int q = p - 1;
  if (m == 0) {
    i = s;
    j = q;
  } else {
    i = (s + m) % q;
    j = (s - m + q) % q;
  }
  if (i > j) {
    int t = i;
    i = j;
    j = t;
  }
}

__global__ __launch_bounds__(EIG_THREADS) void jacobi_kernel(double* __restrict__ Ball,
                                                             double* __restrict__ Vall, int p,
                                                             int max_sweeps) {
  extern __shared__ double sh[];
  const int P2 = p / 2;
  double* cs = sh;               // P2 cosines
  double* sn = sh + P2;          // P2 sines
  int* pi = (int*)(sh + 2 * P2); // P2 first indices
  int* pj = pi + P2;             // P2 second indices
  __shared__ double red[EIG_WAVES];
  const int mode = blockIdx.x;
  double* B = Ball + (int64_t)mode * p * p;
  double* V = Vall + (int64_t)mode * p * p;
  const int tid = threadIdx.x;

  for (int64_t e = tid; e < (int64_t)p * p; e += EIG_THREADS) V[e] = (e / p == e % p) ? 1.0 : 0.0;
  __syncthreads();

  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    // convergence test: off-diagonal mass against the diagonal
    double off = 0.0, dia = 0.0;
    for (int64_t e = tid; e < (int64_t)p * p; e += EIG_THREADS) {
      int r = (int)(e / p), c = (int)(e % p);
      double v = B[e];
      if (r == c) dia += v * v;
      else off += v * v;
    }
    off = block_sum(off, red);
    dia = block_sum(dia, red);
    if (off <= 1e-30 * dia || off == 0.0) break;

    for (int s = 0; s < p - 1; ++s) {
      for (int m = tid; m < P2; m += EIG_THREADS) {
        int i, j;
        round_pair(p, s, m, i, j);
        double app = B[(int64_t)i * p + i], aqq = B[(int64_t)j * p + j], apq = B[(int64_t)i * p + j];
        double c = 1.0, sv = 0.0;
        if (apq != 0.0 && fabs(apq) > 1e-300) {
          double tau = (aqq - app) / (2.0 * apq);
          double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          sv = t * c;
        }
        cs[m] = c;
        sn[m] = sv;
        pi[m] = i;
        pj[m] = j;
      }
      __syncthreads();
      // B <- J^T B J on independent 2 x 2 blocks (pair M rows, pair N columns)
      for (int64_t blk = tid; blk < (int64_t)P2 * P2; blk += EIG_THREADS) {
        const int M = (int)(blk / P2), Nn = (int)(blk % P2);
        const int r0 = pi[M], r1 = pj[M], c0 = pi[Nn], c1 = pj[Nn];
        const double cr = cs[M], sr = sn[M], cc = cs[Nn], sc = sn[Nn];
        double b00 = B[(int64_t)r0 * p + c0], b01 = B[(int64_t)r0 * p + c1];
        double b10 = B[(int64_t)r1 * p + c0], b11 = B[(int64_t)r1 * p + c1];
        // columns: [x0 x1] -> [c x0 - s x1, s x0 + c x1]
        double t00 = cc * b00 - sc * b01, t01 = sc * b00 + cc * b01;
        double t10 = cc * b10 - sc * b11, t11 = sc * b10 + cc * b11;
        // rows
        double u00 = cr * t00 - sr * t10, u10 = sr * t00 + cr * t10;
        double u01 = cr * t01 - sr * t11, u11 = sr * t01 + cr * t11;
        if (M == Nn) u01 = u10 = 0.0;  // the annihilated pair
        B[(int64_t)r0 * p + c0] = u00;
        B[(int64_t)r0 * p + c1] = u01;
        B[(int64_t)r1 * p + c0] = u10;
        B[(int64_t)r1 * p + c1] = u11;
      }
      // V <- V J (column pairs), V col-major: V[row + col*p]
      for (int64_t e = tid; e < (int64_t)p * P2; e += EIG_THREADS) {
        const int M = (int)(e / p), row = (int)(e % p);
        const int c0 = pi[M], c1 = pj[M];
        const double c = cs[M], sv = sn[M];
        double x0 = V[(int64_t)c0 * p + row], x1 = V[(int64_t)c1 * p + row];
        V[(int64_t)c0 * p + row] = c * x0 - sv * x1;
        V[(int64_t)c1 * p + row] = sv * x0 + c * x1;
      }
      __syncthreads();
    }
  }
}

void launch_jacobi(double* B, double* V, int p, int modes, int max_sweeps, hipStream_t s) {
  size_t shm = (size_t)(p / 2) * (2 * sizeof(double) + 2 * sizeof(int));
  hipLaunchKernelGGL(jacobi_kernel, dim3(modes), dim3(EIG_THREADS), shm, s, B, V, p, max_sweeps);
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

}  // namespace rs
