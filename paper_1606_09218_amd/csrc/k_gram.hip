// Charge-weighted Gram matrices of the long-range side matrices without the
// n x n x K product.
//
// The columns of a side matrix are collocated Gaussians, u_j(x) =
// exp(-t_k^2 (x - X_nu)^2) (eq Long-Range_Sum), and the product of two
// Gaussians of one width is again a Gaussian:
//   exp(-t^2 (x - X)^2) exp(-t^2 (x' - X)^2)
//     = exp(-t^2 (x - x')^2 / 2) exp(-2 t^2 ((x + x')/2 - X)^2).
// So the Gram G = U diag(w) U^T of one mode is
//   G[i, i'] = sum_k exp(-t_k^2 ((i - i') h)^2 / 2) S_k[i + i'],
//   S_k[m]   = sum_nu w_{k N + nu} exp(-2 t_k^2 (y_m - X_nu)^2),
// with y_m = -b + (m + 1) h / 2 the midpoint of the cell centres x_i, x_i'
// (i + i' = m, m = 0 .. 2n - 2).  That is O(n N R_l) exponentials for the
// midpoint sums and O(n^2 R_l) for G, instead of 2 n^2 N R_l FLOP: the
// subspace step of the reduced HOSVD becomes linear in the number of terms
// (the paper reduces the side-matrix SVDs by a multigrid scheme to the same
// end; see its remark on the cost of the canonical-to-Tucker step).
//
// Every term is positive (w >= 0), so each entry is a sum without
// cancellation, and the sums over particles and over the particle chunks
// run in a fixed order (deterministic).
#include "rs_internal.h"

namespace rs {

namespace {
constexpr int GG_THREADS = 256;   // midpoints per workgroup
constexpr int GG_STAGE = 512;     // particles staged in LDS per round
}  // namespace

// part[c][l][k][m] = sum over particle chunk c of w_{kN+nu} exp(-2 t_k^2 (y_m - X_nu,l)^2).
// Grid: x = midpoint blocks, y = k + R_l l, z = particle chunk.
__global__ __launch_bounds__(GG_THREADS) void gram_midpoint_kernel(
    const double* __restrict__ pos, const double* __restrict__ t, const double* __restrict__ w,
    int64_t N, int R_l, int64_t n, double b, int64_t chunk, double* __restrict__ part) {
  __shared__ double xs[GG_STAGE], ws[GG_STAGE];
  const int l = blockIdx.y / R_l, k = blockIdx.y - (blockIdx.y / R_l) * R_l;
  const int64_t nm = 2 * n - 1;
  const int64_t m = (int64_t)blockIdx.x * GG_THREADS + threadIdx.x;
  const double h = 2.0 * b / (double)n;
  const double y = -b + (double)(m + 1) * 0.5 * h;
  const double c2 = 2.0 * t[k] * t[k];
  const int64_t nu0 = (int64_t)blockIdx.z * chunk;
  const int64_t nu1 = nu0 + chunk < N ? nu0 + chunk : N;
  const double* wk = w + (int64_t)k * N;
  double acc = 0.0;
  for (int64_t s0 = nu0; s0 < nu1; s0 += GG_STAGE) {
    const int cnt = (int)(nu1 - s0 < GG_STAGE ? nu1 - s0 : GG_STAGE);
    __syncthreads();
    for (int e = threadIdx.x; e < cnt; e += GG_THREADS) {
      xs[e] = pos[3 * (s0 + e) + l];
      ws[e] = wk[s0 + e];
    }
    __syncthreads();
    for (int e = 0; e < cnt; ++e) {
      const double d = y - xs[e];
      acc += ws[e] * exp(-c2 * (d * d));
    }
  }
  if (m < nm) part[(((int64_t)blockIdx.z * 3 + l) * R_l + k) * nm + m] = acc;
}

// G[l][i][i'] = sum_k exp(-t_k^2 ((i - i') h)^2 / 2) sum_c part[c][l][k][i + i'],
// one thread per entry; grid.y = mode.
__global__ __launch_bounds__(256) void gram_assemble_kernel(const double* __restrict__ part,
                                                            const double* __restrict__ t,
                                                            int R_l, int64_t n, double b,
                                                            int chunks, double* __restrict__ G) {
  const int l = blockIdx.y;
  const int64_t nm = 2 * n - 1;
  const double h = 2.0 * b / (double)n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / n, ip = e - (e / n) * n;
    const int64_t m = i + ip;
    const double d = (double)(i - ip) * h;
    double g = 0.0;
    for (int k = 0; k < R_l; ++k) {
      double sk = 0.0;
      for (int c = 0; c < chunks; ++c) sk += part[(((int64_t)c * 3 + l) * R_l + k) * nm + m];
      g += exp(-0.5 * t[k] * t[k] * (d * d)) * sk;
    }
    G[(int64_t)l * n * n + e] = g;
  }
}

// particle chunks: enough workgroups for about four per CU
static int gram_chunks(int64_t N, int R_l, int64_t n, int num_cu) {
  const int64_t base = (2 * n - 1 + GG_THREADS - 1) / GG_THREADS * 3 * R_l;
  int64_t c = (4LL * num_cu + base - 1) / base;
  c = std::max<int64_t>(1, std::min<int64_t>(c, (N + 255) / 256));
  return (int)std::min<int64_t>(c, 64);
}

size_t gauss_gram_workspace_bytes(int64_t N, int R_l, int64_t n, int num_cu) {
  return (size_t)gram_chunks(N, R_l, n, num_cu) * 3 * R_l * (2 * n - 1) * sizeof(double);
}

void launch_gauss_gram(const double* pos, const double* t, const double* w, int64_t N, int R_l,
                       int64_t n, double b, double* G, double* work, int num_cu, hipStream_t s) {
  const int chunks = gram_chunks(N, R_l, n, num_cu);
  const int64_t chunk = (N + chunks - 1) / chunks;
  const int64_t nm = 2 * n - 1;
  const dim3 g1((unsigned)((nm + GG_THREADS - 1) / GG_THREADS), (unsigned)(3 * R_l), (unsigned)chunks);
  hipLaunchKernelGGL(gram_midpoint_kernel, g1, dim3(GG_THREADS), 0, s, pos, t, w, N, R_l, n, b,
                     chunk, work);
  const unsigned blocks = (unsigned)std::min<int64_t>((n * n + 255) / 256, 4096);
  hipLaunchKernelGGL(gram_assemble_kernel, dim3(blocks, 3), dim3(256), 0, s, (const double*)work,
                     t, R_l, n, b, chunks, G);
}

}  // namespace rs
