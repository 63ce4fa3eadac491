// Long-range factor columns (side matrices) of the N-particle canonical sum.
//
// The long-range part of the potential sum is the canonical tensor
//   P_l = sum_nu z_nu sum_{k<R_l} a_k g_k(. - x_nu),  g_k(x) = prod_l exp(-t_k^2 x_l^2)
// of rank R_l N (eq Long-Range_Sum), collocated at the cell centres.  Its side
// matrices hold one column per (k, nu): U_l[i, j] = exp(-t_k^2 (x_i - x_{nu,l})^2),
// j = k N + nu; the canonical weights are xi_j = z_nu a_k.
//
// Layout: U is three n x K column-major blocks (mode-major), each column
// contiguous, so that the Gram and projection GEMMs stream whole columns.
#include "rs_internal.h"

namespace rs {

__global__ void validate_kernel(const double* __restrict__ pos, const double* __restrict__ q,
                                int64_t N, double b, int* flags) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int f = 0;
  if (i < N) {
    for (int l = 0; l < 3; ++l) {
      double x = pos[3 * i + l];
      if (!isfinite(x)) f |= 1;
      else if (x < -b || x > b) f |= 2;
    }
    if (!isfinite(q[i])) f |= 1;
  }
  // wave-level OR, then one integer atomic per wave (order-independent)
  for (int off = 32; off > 0; off >>= 1) f |= __shfl_xor(f, off);
  if ((threadIdx.x & 63) == 0 && f) atomicOr(flags, f);
}

void launch_validate(const double* pos, const double* q, int64_t N, double b, int* flags,
                     hipStream_t s) {
  int threads = 256;
  int64_t blocks = (N + threads - 1) / threads;
  hipLaunchKernelGGL(validate_kernel, dim3((unsigned)blocks), dim3(threads), 0, s, pos, q, N, b,
                     flags);
}

// One thread per (i, j): consecutive threads walk down a column (i fastest),
// so the stores are fully coalesced.  grid.y = mode.
__global__ void side_matrix_kernel(const double* __restrict__ pos, const double* __restrict__ t,
                                   int64_t N, int R_l, int64_t n, double b, double* __restrict__ U) {
  // one column j = k N + nu per workgroup step (its index arithmetic done
  // once), the threads over the n grid points of the column (coalesced)
  const int l = blockIdx.y;
  const int64_t K = N * R_l;
  const double h = 2.0 * b / (double)n;
  double* Ul = U + (int64_t)l * n * K;
  for (int64_t j = blockIdx.x; j < K; j += gridDim.x) {
    const int64_t k = j / N;
    const int64_t nu = j - k * N;
    const double x = pos[3 * nu + l];
    const double tk = t[k];
    double* col = Ul + j * n;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
      const double xi = -b + ((double)i + 0.5) * h;
      const double d = xi - x;
      col[i] = exp(-(tk * tk) * (d * d));
    }
  }
}

__global__ void weights_kernel(const double* __restrict__ q, const double* __restrict__ a,
                               int64_t N, int R_l, double* __restrict__ xi, double* __restrict__ w,
                               double* __restrict__ sw) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N * R_l) return;
  int64_t k = j / N;
  int64_t nu = j - k * N;
  double v = q[nu] * a[k];
  xi[j] = v;
  w[j] = cbrt(v * v);  // |xi|^{2/3}
  if (sw) sw[j] = cbrt(fabs(v));  // |xi|^{1/3}
}

void launch_side_matrices(const double* pos, const double* q, const double* t, const double* a,
                          int64_t N, int R_l, int64_t n, double b, double* U, double* xi,
                          double* w, double* sw, hipStream_t s) {
  const int64_t K = N * R_l;
  const int threads = n >= 256 ? 256 : 64;
  const int64_t blocks = std::min<int64_t>(K, 65535LL * 16);
  if (blocks <= 0 || n <= 0) return;
  hipLaunchKernelGGL(side_matrix_kernel, dim3((unsigned)blocks, 3), dim3(threads), 0, s, pos, t,
                     N, R_l, n, b, U);
  hipLaunchKernelGGL(weights_kernel, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, s, q, a, N,
                     R_l, xi, w, sw);
}

// The Toeplitz factors of the RS form of the RBF matrix (section 4.1):
// T[k][i][j] = exp(-t_k^2 ((i - j) h)^2), for the short-range terms k >= R_l
// only within the window |i - j| <= w; Acat[i][k n + j] = a_k T[k][i][j].
__global__ void rbf_toeplitz_kernel(const double* __restrict__ t, const double* __restrict__ a,
                                    int R, int R_l, int64_t n, double h, int w,
                                    double* __restrict__ T, double* __restrict__ Acat) {
  const int64_t total = (int64_t)R * n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(e / (n * n));
    const int64_t ij = e - (int64_t)k * n * n, i = ij / n, j = ij - (ij / n) * n;
    const int64_t d = i - j;
    double v = 0.0;
    if (k < R_l || (d <= w && d >= -w)) {
      const double x = (double)d * h;
      v = exp(-t[k] * t[k] * (x * x));
    }
    T[e] = v;
    Acat[i * (int64_t)R * n + (int64_t)k * n + j] = a[k] * v;
  }
}

void launch_rbf_toeplitz(const double* t, const double* a, int R, int R_l, int64_t n, double h,
                         int w, double* T, double* Acat, hipStream_t s) {
  const int64_t total = (int64_t)R * n * n;
  const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(rbf_toeplitz_kernel, dim3(blocks), dim3(256), 0, s, t, a, R, R_l, n, h, w, T,
                     Acat);
}

// DV[i, c] = d/dx of column c of V (n x r row-major) on the cell-centred grid:
// central differences inside, one-sided at the two ends (eq Gradients_Tens).
__global__ void fd_rows_kernel(const double* __restrict__ V, int64_t n, int r, double h,
                               double* __restrict__ DV) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * r;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / r, c = e - (e / r) * r;
    double d;
    if (i == 0) d = (V[r + c] - V[c]) / h;
    else if (i == n - 1) d = (V[i * r + c] - V[(i - 1) * r + c]) / h;
    else d = (V[(i + 1) * r + c] - V[(i - 1) * r + c]) / (2.0 * h);
    DV[e] = d;
  }
}

void launch_fd_rows(const double* V, int64_t n, int r, double h, double* DV, hipStream_t s) {
  const int64_t total = n * r;
  if (total <= 0) return;
  const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(fd_rows_kernel, dim3(blocks), dim3(256), 0, s, V, n, r, h, DV);
}

}  // namespace rs
