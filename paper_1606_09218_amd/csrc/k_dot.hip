// Scalar product of two RS tensors on one grid (section 3.4, item (d)):
//   <A, B> = sum_i A(i) B(i) = <A_l, B_l> + sum_{i in W} (A(i) B(i) - A_l(i) B_l(i)),
// W = the cells some short-range window of A or of B touches: outside every
// window a tensor equals its long-range Tucker part.  <A_l, B_l> is formed
// from the Tucker factors by the host (small GEMMs); this file holds the
// correction over the touched bricks and the fixed-order reductions.
#include "rs_internal.h"

namespace rs {

__device__ __forceinline__ double dot_readlane(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double dot_wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);   // same tree on every call
  return v;
}

// Short-range values of one tensor at the cells (base0 + m, i1, i2), m = 0..7,
// of this lane: the windowed terms z_nu sum_{k >= R_l} a_k g g g of the
// particles listed for brick `br` (the same sum the grid's short gather adds).
// f: LDS [3][Rs][8] factors, ak / tk2: LDS [Rs] (one wave per workgroup, so
// __syncthreads is a wave barrier).
__device__ void dot_side_short(const DotSide& S, int br, int64_t n, double b, const int bs[3],
                               int c1, int c2, double* f, double* ak, double* tk2,
                               double (&out)[8]) {
  const int lane = threadIdx.x;
  const int Rs = S.R - S.R_l;
#pragma unroll
  for (int m = 0; m < 8; ++m) out[m] = 0.0;
  if (Rs <= 0) return;
  __syncthreads();   // the previous side's factors are no longer read
  for (int k = lane; k < Rs; k += 64) {
    ak[k] = S.a[S.R_l + k];
    tk2[k] = S.t[S.R_l + k] * S.t[S.R_l + k];
  }
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
      __syncthreads();
      for (int idx = lane; idx < 24 * Rs; idx += 64) {
        const int l = idx / (8 * Rs);
        const int rem = idx - l * 8 * Rs;
        const int k = rem >> 3, m = rem & 7;
        const double d = (-b + ((double)(bs[l] + m) + 0.5) * h) - p[l];
        f[idx] = exp(-tk2[k] * (d * d));
      }
      __syncthreads();
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
}

// long-range Tucker values of one tensor at the lane's 8 cells:
// sum_c T2[(i0 n + i1) r3 + c] V3[i2 r3 + c]
__device__ void dot_side_long(const DotSide& S, int64_t n, int64_t i0b, int64_t i1, int64_t i2,
                              double (&out)[8]) {
  const double* v = S.V3 + i2 * S.r3;
  const double* t[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const int64_t i0 = i0b + m < n ? i0b + m : n - 1;
    t[m] = S.T2 + (i0 * n + i1) * S.r3;
    out[m] = 0.0;
  }
  for (int c = 0; c < S.r3; ++c) {
    const double vc = v[c];
#pragma unroll
    for (int m = 0; m < 8; ++m) out[m] += t[m][c] * vc;
  }
}

// One wave per brick of `active` (count in active[0]); bricks that `skip`
// (a start array) lists as touched are left out (they were counted in the
// other tensor's pass).  partials[ia] = the brick's sum of A B - A_l B_l.
__global__ __launch_bounds__(64) void dot_bricks_kernel(DotSide A, DotSide B, const int* active,
                                                        int64_t cap, const int* skip, int nb,
                                                        int64_t n, double b, int rs_max,
                                                        double* __restrict__ partials) {
  extern __shared__ double dlds[];
  double* f = dlds;                  // [3][rs_max][8]
  double* ak = dlds + 24 * rs_max;   // [rs_max]
  double* tk2 = ak + rs_max;         // [rs_max]
  const int lane = threadIdx.x;
  const int c1 = lane >> 3, c2 = lane & 7;
  const int64_t count = active[0] < cap ? active[0] : cap;
  for (int64_t ia = blockIdx.x; ia < count; ia += gridDim.x) {
    const int br = active[1 + ia];
    double sum = 0.0;
    if (!skip || skip[br + 1] == skip[br]) {
      const int b0 = br / (nb * nb), b1 = (br / nb) % nb, b2 = br % nb;
      const int bs[3] = {b0 * 8, b1 * 8, b2 * 8};
      const int64_t i1 = bs[1] + c1, i2 = bs[2] + c2;
      const bool col_ok = i1 < n && i2 < n;
      double la[8], lb[8], sa[8], sb[8];
      dot_side_long(A, n, bs[0], col_ok ? i1 : 0, col_ok ? i2 : 0, la);
      dot_side_long(B, n, bs[0], col_ok ? i1 : 0, col_ok ? i2 : 0, lb);
      dot_side_short(A, br, n, b, bs, c1, c2, f, ak, tk2, sa);
      dot_side_short(B, br, n, b, bs, c1, c2, f, ak, tk2, sb);
#pragma unroll
      for (int m = 0; m < 8; ++m)
        if (col_ok && bs[0] + m < n) sum += la[m] * sb[m] + sa[m] * lb[m] + sa[m] * sb[m];
    }
    sum = dot_wave_sum(sum);
    if (lane == 0) partials[ia] = sum;
  }
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

// out = sum of the DOT_BLOCKS long-long partials + the first active_a[0]
// brick partials of pass A + the first active_b[0] of pass B (fixed order)
__global__ __launch_bounds__(1024) void dot_final_kernel(const double* __restrict__ ll,
                                                         const double* __restrict__ pa,
                                                         const int* active_a, int64_t cap_a,
                                                         const double* __restrict__ pb,
                                                         const int* active_b, int64_t cap_b,
                                                         double* __restrict__ out) {
  __shared__ double red[1024];
  const int64_t na = active_a[0] < cap_a ? active_a[0] : cap_a;
  const int64_t nbk = active_b[0] < cap_b ? active_b[0] : cap_b;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < DOT_BLOCKS; i += 1024) s += ll[i];
  for (int64_t i = threadIdx.x; i < na; i += 1024) s += pa[i];
  for (int64_t i = threadIdx.x; i < nbk; i += 1024) s += pb[i];
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

void launch_dot_bricks(const DotSide& A, const DotSide& B, const int* active, int64_t cap,
                       const int* skip, int nb, int64_t n, double b, int num_cu, double* partials,
                       hipStream_t s) {
  const int rs_max = std::max(std::max(A.R - A.R_l, B.R - B.R_l), 1);
  if (rs_max > 64) throw Error{RS_E_UNSUPPORTED, "more than 64 short-range terms"};
  const int64_t wgs = std::max<int64_t>(1, std::min<int64_t>(cap, (int64_t)num_cu * 16));
  const size_t lds = (size_t)26 * rs_max * sizeof(double);
  hipLaunchKernelGGL(dot_bricks_kernel, dim3((unsigned)wgs), dim3(64), lds, s, A, B, active, cap,
                     skip, nb, n, b, rs_max, partials);
}

void launch_dot_final(const double* ll, const double* pa, const int* active_a, int64_t cap_a,
                      const double* pb, const int* active_b, int64_t cap_b, double* out,
                      hipStream_t s) {
  hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(1024), 0, s, ll, pa, active_a, cap_a, pb,
                     active_b, cap_b, out);
}

}  // namespace rs
