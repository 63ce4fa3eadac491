// Short-range part of the RS tensor: the cumulated canonical tensor
//   sum_nu z_nu U_nu,  U_nu(i) = sum_{k >= R_l} a_k prod_l exp(-t_k^2 (x_{i_l} - x_{nu,l})^2)
// restricted to the window of n_s cells around the particle's cell
// (Definitions ComCanF and CCT_Uniform; windows may overlap, the "soft"
// separation of section 3.3).
//
// The grid is split into bricks of 8^3 cells.  Binning lists, for every
// brick, the particles whose window touches it, sorted by particle index.
// The gather then runs one workgroup per touched brick: it forms the 1D
// factors of each listed particle over the brick's 8 coordinates in LDS and
// adds the windowed sum to the brick's cells with a read-modify-write.  Every
// cell is written by one thread and particles are visited in index order, so
// the result is deterministic without floating-point atomics.
#include <hipcub/hipcub.hpp>

#include "rs_internal.h"

namespace rs {

constexpr int BRICK = 8;

__device__ __forceinline__ void particle_window(const double* __restrict__ pos, int64_t nu,
                                                int64_t n, double b, int w, int lo[3], int hi[3]) {
  const double h = 2.0 * b / (double)n;
  for (int l = 0; l < 3; ++l) {
    double x = pos[3 * nu + l];
    int64_t j = (int64_t)floor((x + b) / h);
    if (j < 0) j = 0;
    if (j > n - 1) j = n - 1;
    int64_t a = j - w, c = j + w;
    lo[l] = (int)(a < 0 ? 0 : a);
    hi[l] = (int)(c > n - 1 ? n - 1 : c);
  }
}

__global__ void bin_count_kernel(const double* __restrict__ pos, int64_t N, int64_t n, double b,
                                 int w, int nb, int* __restrict__ counts) {
  int64_t nu = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (nu >= N) return;
  int lo[3], hi[3];
  particle_window(pos, nu, n, b, w, lo, hi);
  for (int b0 = lo[0] / BRICK; b0 <= hi[0] / BRICK; ++b0)
    for (int b1 = lo[1] / BRICK; b1 <= hi[1] / BRICK; ++b1)
      for (int b2 = lo[2] / BRICK; b2 <= hi[2] / BRICK; ++b2)
        atomicAdd(&counts[((int64_t)b0 * nb + b1) * nb + b2], 1);
}

void short_bin_count(const double* pos, int64_t N, int64_t n, double b, int n_s, int nb,
                     int* counts, hipStream_t s) {
  hipLaunchKernelGGL(bin_count_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, pos, N,
                     n, b, (n_s - 1) / 2, nb, counts);
}

__global__ void bin_fill_kernel(const double* __restrict__ pos, int64_t N, int64_t n, double b,
                                int w, int nb, const int* __restrict__ start,
                                int* __restrict__ cursor, int* __restrict__ list) {
  int64_t nu = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (nu >= N) return;
  int lo[3], hi[3];
  particle_window(pos, nu, n, b, w, lo, hi);
  for (int b0 = lo[0] / BRICK; b0 <= hi[0] / BRICK; ++b0)
    for (int b1 = lo[1] / BRICK; b1 <= hi[1] / BRICK; ++b1)
      for (int b2 = lo[2] / BRICK; b2 <= hi[2] / BRICK; ++b2) {
        int64_t br = ((int64_t)b0 * nb + b1) * nb + b2;
        int slot = atomicAdd(&cursor[br], 1);
        list[start[br] + slot] = (int)nu;
      }
}

void short_bin_fill(const double* pos, int64_t N, int64_t n, double b, int n_s, int nb,
                    const int* start, int* cursor, int* list, hipStream_t s) {
  hipLaunchKernelGGL(bin_fill_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, pos, N,
                     n, b, (n_s - 1) / 2, nb, start, cursor, list);
}

// insertion sort of each brick's (short) list, making the visiting order
// independent of the atomic fill order
__global__ void bin_sort_kernel(const int* __restrict__ start, int* __restrict__ list,
                                int nbricks) {
  int br = blockIdx.x * blockDim.x + threadIdx.x;
  if (br >= nbricks) return;
  int s0 = start[br], s1 = start[br + 1];
  for (int i = s0 + 1; i < s1; ++i) {
    int v = list[i];
    int j = i - 1;
    while (j >= s0 && list[j] > v) {
      list[j + 1] = list[j];
      --j;
    }
    list[j + 1] = v;
  }
}

void short_bin_sort(const int* start, int* list, int nbricks, hipStream_t s) {
  hipLaunchKernelGGL(bin_sort_kernel, dim3((unsigned)((nbricks + 255) / 256)), dim3(256), 0, s,
                     start, list, nbricks);
}

void exclusive_scan_int(const int* in, int* out, int count, hipStream_t s) {
  size_t tmp_bytes = 0;
  if (hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, in, out, count, s) != hipSuccess)
    throw Error{RS_E_DEVICE, "hipcub scan sizing failed"};
  DevBuf tmp(tmp_bytes > 0 ? tmp_bytes : 16, s);
  RS_HIP(hipcub::DeviceScan::ExclusiveSum(tmp.p, tmp_bytes, in, out, count, s));
}

constexpr int GATHER_THREADS = 256;
constexpr int MAX_RS = 64;  // short-range terms handled per particle

// One workgroup per brick (grid.x enumerates all bricks; empty ones exit).
template <typename GT>
__global__ __launch_bounds__(GATHER_THREADS) void short_gather_kernel(
    GT* __restrict__ grid, const double* __restrict__ pos, const double* __restrict__ q,
    const double* __restrict__ t, const double* __restrict__ a, int R, int R_l, int64_t n,
    double b, int w, int nb, const int* __restrict__ start, const int* __restrict__ list) {
  const int64_t br = blockIdx.x;
  const int s0 = start[br], s1 = start[br + 1];
  if (s0 == s1) return;
  __shared__ double f[3][MAX_RS][BRICK];
  __shared__ double ak[MAX_RS];
  __shared__ int win[6];
  const int Rs = R - R_l;
  const int b0 = (int)(br / ((int64_t)nb * nb)), b1 = (int)((br / nb) % nb), b2 = (int)(br % nb);
  const int base[3] = {b0 * BRICK, b1 * BRICK, b2 * BRICK};
  const double h = 2.0 * b / (double)n;
  const int tid = threadIdx.x;
  if (tid < Rs) ak[tid] = a[R_l + tid];

  // two cells per thread: (c0, c1, c2) and (c0 + 4, c1, c2)
  const int c2 = tid & 7, c1 = (tid >> 3) & 7, c0 = tid >> 6;  // c0 in 0..3
  double acc[2] = {0.0, 0.0};

  for (int e = s0; e < s1; ++e) {
    const int nu = list[e];
    __syncthreads();  // previous particle's factors are no longer read
    if (tid == 0) {
      int lo[3], hi[3];
      particle_window(pos, nu, n, b, w, lo, hi);
      for (int l = 0; l < 3; ++l) {
        win[2 * l] = lo[l] - base[l];
        win[2 * l + 1] = hi[l] - base[l];
      }
    }
    for (int idx = tid; idx < 3 * Rs * BRICK; idx += GATHER_THREADS) {
      const int l = idx / (Rs * BRICK);
      const int rem = idx - l * Rs * BRICK;
      const int k = rem / BRICK, m = rem - k * BRICK;
      const double x = -b + ((double)(base[l] + m) + 0.5) * h;
      const double d = x - pos[3 * nu + l];
      const double tk = t[R_l + k];
      f[l][k][m] = exp(-(tk * tk) * (d * d));
    }
    __syncthreads();
    const double z = q[nu];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int m0 = c0 + 4 * u;
      if (m0 >= win[0] && m0 <= win[1] && c1 >= win[2] && c1 <= win[3] && c2 >= win[4] &&
          c2 <= win[5]) {
        double s = 0.0;
        for (int k = 0; k < Rs; ++k) s += ak[k] * f[0][k][m0] * f[1][k][c1] * f[2][k][c2];
        acc[u] += z * s;
      }
    }
  }
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int64_t i0 = base[0] + c0 + 4 * u, i1 = base[1] + c1, i2 = base[2] + c2;
    if (i0 < n && i1 < n && i2 < n && acc[u] != 0.0) {
      GT* dst = grid + (i0 * n + i1) * n + i2;
      *dst = (GT)((double)(*dst) + acc[u]);
    }
  }
}

void short_gather(void* grid, int grid_fp32, const double* pos, const double* q, const double* t,
                  const double* a, int R, int R_l, int64_t n, double b, int n_s, int nb,
                  const int* start, const int* list, hipStream_t s) {
  if (R - R_l > MAX_RS) throw Error{RS_E_UNSUPPORTED, "more than 64 short-range terms"};
  const int64_t nbricks = (int64_t)nb * nb * nb;
  const int w = (n_s - 1) / 2;
  if (grid_fp32)
    hipLaunchKernelGGL(short_gather_kernel<float>, dim3((unsigned)nbricks), dim3(GATHER_THREADS), 0,
                       s, (float*)grid, pos, q, t, a, R, R_l, n, b, w, nb, start, list);
  else
    hipLaunchKernelGGL(short_gather_kernel<double>, dim3((unsigned)nbricks), dim3(GATHER_THREADS), 0,
                       s, (double*)grid, pos, q, t, a, R, R_l, n, b, w, nb, start, list);
}

}  // namespace rs
