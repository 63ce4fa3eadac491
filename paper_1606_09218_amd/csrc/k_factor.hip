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

// U (FP64, column j = k N + nu contiguous) and/or the FP16 split planes of
// the projection, planes[l][term][j][i] with i padded to kp (a multiple of
// 32) by zeros.  Every entry is at most 1, so the planes hold
// x 2^14 = hi + lo (x from plane_exp in FP32, hi = x 2^14 rounded to FP16,
// lo = the exact FP32 rest rounded to FP16) under the fixed scale 2^14.
// grid.y = mode.
typedef _Float16 sm_h8 __attribute__((ext_vector_type(8)));

// e^arg (arg <= 0) to about 2^-23 relative for the FP16 planes, with
// zero-mean rounding errors: arg log2 e = m + f (m integer, |f| <= 1/2, both
// in FP64), e^(f ln 2) by its Taylor series to degree 7 in FP32 (truncation
// below 6e-9 for |f ln 2| <= 0.35), scaled by 2^m.
__device__ __forceinline__ float plane_exp(double arg) {
  const double A = arg * 1.4426950408889634;
  const double m = rint(A);
  const float x = (float)(A - m) * 0.69314718f;
  float p = 1.0f / 5040.0f;
  p = fmaf(p, x, 1.0f / 720.0f);
  p = fmaf(p, x, 1.0f / 120.0f);
  p = fmaf(p, x, 1.0f / 24.0f);
  p = fmaf(p, x, 1.0f / 6.0f);
  p = fmaf(p, x, 0.5f);
  p = fmaf(p, x, 1.0f);
  p = fmaf(p, x, 1.0f);
  return m < -200.0 ? 0.0f : ldexpf(p, (int)m);
}

__global__ void side_matrix_kernel(const double* __restrict__ pos, const double* __restrict__ t,
                                   int64_t N, int R_l, int64_t n, double b, double* __restrict__ U,
                                   _Float16* __restrict__ planes, int64_t kp) {
  const int l = blockIdx.y;
  const int64_t K = N * R_l;
  const double h = 2.0 * b / (double)n;
  double* Ul = U ? U + (int64_t)l * n * K : nullptr;
  if (!planes) {
    // one column per workgroup step, the threads over its n grid points
    // (consecutive threads, consecutive addresses)
    for (int64_t j = blockIdx.x; j < K; j += gridDim.x) {
      const int64_t k = j / N;
      const int64_t nu = j - k * N;
      const double x = pos[3 * nu + l];
      const double tk = t[k];
      for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const double d = (-b + ((double)i + 0.5) * h) - x;
        Ul[j * n + i] = exp(-(tk * tk) * (d * d));
      }
    }
    return;
  }
  // eight consecutive grid points per thread (one 16-byte store per plane),
  // cpb columns per workgroup step when a column needs at most 256 threads
  _Float16* P0 = planes + (int64_t)l * 2 * K * kp;
  const int kq = (int)(kp / 8);
  const int cpb = kq <= (int)blockDim.x ? (int)blockDim.x / kq : 1;
  const int cs = kq <= (int)blockDim.x ? (int)threadIdx.x / kq : 0;
  const int i8s = kq <= (int)blockDim.x ? (int)threadIdx.x - cs * kq : (int)threadIdx.x;
  const int istep = kq <= (int)blockDim.x ? kq : (int)blockDim.x;
  if (cs >= cpb) return;
  for (int64_t j = (int64_t)blockIdx.x * cpb + cs; j < K; j += (int64_t)gridDim.x * cpb) {
    const int k = (int)j / (int)N;   // K < 2^31 (checked by the launcher)
    const int nu = (int)j - k * (int)N;
    const double x = pos[3 * (int64_t)nu + l];
    const double tk = t[k];
    for (int i8 = i8s; i8 < kq; i8 += istep) {
      const int64_t i0 = 8 * (int64_t)i8;
      sm_h8 hi, lo;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t i = i0 + u;
        const double d = (-b + ((double)i + 0.5) * h) - x;
        const double arg = -(tk * tk) * (d * d);
        if (Ul && i < n) Ul[j * n + i] = exp(arg);
        const float v = i < n ? plane_exp(arg) : 0.0f;
        const float y = v * 16384.0f;
        hi[u] = (_Float16)y;
        lo[u] = (_Float16)(y - (float)hi[u]);
      }
      *(sm_h8*)(P0 + j * kp + i0) = hi;
      *(sm_h8*)(P0 + (K + j) * kp + i0) = lo;
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
                          double* w, double* sw, hipStream_t s, void* planes16, int64_t kp,
                          hipStream_t side_s, bool on_side) {
  const int64_t K = N * R_l;
  const int threads = planes16 ? 256 : (n >= 256 ? 256 : 64);
  const int64_t cpb = planes16 && kp / 8 <= 256 ? 256 / (kp / 8) : 1;
  const int64_t blocks = planes16 ? std::min<int64_t>((K + cpb - 1) / cpb, 65535LL * 16)
                                  : std::min<int64_t>(K, 65535LL * 16);
  if (blocks <= 0 || n <= 0) return;
  if (planes16 && (kp % 32 != 0 || kp < n)) throw Error{RS_E_INVALID, "side-matrix planes: bad padding"};
  if (planes16 && K >= (1LL << 31)) throw Error{RS_E_UNSUPPORTED, "side matrices: more than 2^31 terms"};
  hipLaunchKernelGGL(side_matrix_kernel, dim3((unsigned)blocks, 3), dim3(threads), 0,
                     on_side ? side_s : s, pos, t, N, R_l, n, b, U, (_Float16*)planes16, kp);
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
