// Short-range part of the RS tensor: the cumulated canonical tensor
//   sum_nu z_nu U_nu,  U_nu(i) = sum_{k >= R_l} a_k prod_l exp(-t_k^2 (x_{i_l} - x_{nu,l})^2)
// restricted to the window of n_s cells around the particle's cell
// (Definitions ComCanF and CCT_Uniform; windows may overlap, the "soft"
// separation of section 3.3).
//
// The grid is split into bricks of 8^3 cells.  Binning lists, for every
// brick, the particles whose window touches it, sorted by particle index.
// The gather then visits every touched brick with one wave: it forms the 1D
// factors of each listed particle over the brick's 8 coordinates in LDS and
// adds the windowed sum to the brick's cells with a read-modify-write.  Every
// cell is written by one lane and particles are visited in index order, so
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

// bricks per axis that a window of n_s cells can meet
__host__ __device__ inline int window_bricks(int n_s) { return (n_s + 6) / BRICK + 1; }

// one thread per (particle, brick of its window): the brick at offset
// (d0, d1, d2) from the window's first brick, if the window reaches it
__device__ __forceinline__ bool pair_brick(const double* __restrict__ pos, int64_t t, int64_t N,
                                           int64_t n, double b, int w, int per, int nb,
                                           int64_t& nu, int64_t& br) {
  const int64_t ppp = (int64_t)per * per * per;
  if (t >= N * ppp) return false;
  nu = t / ppp;
  const int sl = (int)(t - nu * ppp);
  const int d0 = sl / (per * per), d1 = (sl / per) % per, d2 = sl % per;
  int lo[3], hi[3];
  particle_window(pos, nu, n, b, w, lo, hi);
  const int b0 = lo[0] / BRICK + d0, b1 = lo[1] / BRICK + d1, b2 = lo[2] / BRICK + d2;
  if (b0 > hi[0] / BRICK || b1 > hi[1] / BRICK || b2 > hi[2] / BRICK) return false;
  br = ((int64_t)b0 * nb + b1) * nb + b2;
  return true;
}

__global__ void bin_count_kernel(const double* __restrict__ pos, int64_t N, int64_t n, double b,
                                 int w, int per, int nb, int* __restrict__ counts) {
  int64_t nu, br;
  if (pair_brick(pos, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, N, n, b, w, per, nb, nu, br))
    atomicAdd(&counts[br], 1);
}

void short_bin_count(const double* pos, int64_t N, int64_t n, double b, int n_s, int nb,
                     int* counts, hipStream_t s) {
  const int per = window_bricks(n_s);
  const int64_t pairs = N * per * per * per;
  if (pairs <= 0) return;
  hipLaunchKernelGGL(bin_count_kernel, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, s, pos,
                     N, n, b, (n_s - 1) / 2, per, nb, counts);
}

__global__ void bin_fill_kernel(const double* __restrict__ pos, int64_t N, int64_t n, double b,
                                int w, int per, int nb, const int* __restrict__ start,
                                int* __restrict__ cursor, int* __restrict__ list) {
  int64_t nu, br;
  if (pair_brick(pos, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, N, n, b, w, per, nb, nu, br)) {
    const int slot = atomicAdd(&cursor[br], 1);
    list[start[br] + slot] = (int)nu;
  }
}

void short_bin_fill(const double* pos, int64_t N, int64_t n, double b, int n_s, int nb,
                    const int* start, int* cursor, int* list, hipStream_t s) {
  const int per = window_bricks(n_s);
  const int64_t pairs = N * per * per * per;
  if (pairs <= 0) return;
  hipLaunchKernelGGL(bin_fill_kernel, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, s, pos,
                     N, n, b, (n_s - 1) / 2, per, nb, start, cursor, list);
}

// insertion sort of each brick's (short) list, making the visiting order
// independent of the atomic fill order; touched bricks are appended to
// active[1..] (active[0] counts them, zero on entry).  The order of that
// list is arbitrary and does not affect the result: every brick is still
// gathered by one workgroup from its sorted list.
__global__ void bin_sort_kernel(const int* __restrict__ start, int* __restrict__ list,
                                int nbricks, int* __restrict__ active, int64_t active_cap) {
  const int br = blockIdx.x * blockDim.x + threadIdx.x;
  const int s0 = br < nbricks ? start[br] : 0, s1 = br < nbricks ? start[br + 1] : 0;
  // slots in the active list: one atomic per wave for its touched bricks
  const unsigned long long m = __ballot(s1 > s0);
  const int lane = threadIdx.x & 63;
  int base = 0;
  if (lane == 0 && m) base = atomicAdd(&active[0], __popcll(m));
  base = __shfl(base, 0);
  if (s1 > s0) {
    const int slot = base + __popcll(m & ((1ULL << lane) - 1ULL));
    if (slot < active_cap) active[1 + slot] = br;  // the capacity bounds every window
  }
  if (br >= nbricks) return;
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

int64_t short_active_capacity(int64_t N, int n_s, int nb) {
  // a window of n_s cells meets at most (n_s + 6) / 8 + 1 bricks per axis
  const int64_t per = window_bricks(n_s);
  const int64_t nbricks = (int64_t)nb * nb * nb;
  return std::min<int64_t>(nbricks, std::max<int64_t>(N, 0) * per * per * per);
}

void short_bin_sort(const int* start, int* list, int nbricks, int* active, int64_t active_cap,
                    hipStream_t s) {
  RS_HIP(hipMemsetAsync(active, 0, sizeof(int), s));
  hipLaunchKernelGGL(bin_sort_kernel, dim3((unsigned)((nbricks + 255) / 256)), dim3(256), 0, s,
                     start, list, nbricks, active, active_cap);
}

size_t exclusive_scan_bytes(int count) {
  size_t tmp_bytes = 0;
  if (hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, (const int*)nullptr, (int*)nullptr,
                                       count) != hipSuccess)
    throw Error{RS_E_DEVICE, "hipcub scan sizing failed"};
  return tmp_bytes > 0 ? tmp_bytes : 16;
}

void exclusive_scan_int(const int* in, int* out, int count, void* tmp, size_t tmp_bytes,
                        hipStream_t s) {
  size_t need = exclusive_scan_bytes(count);
  if (tmp_bytes < need) throw Error{RS_E_DEVICE, "scan workspace too small"};
  RS_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, need, in, out, count, s));
}

void exclusive_scan_int(const int* in, int* out, int count, hipStream_t s) {
  const size_t tmp_bytes = exclusive_scan_bytes(count);
  DevBuf tmp(tmp_bytes, s);
  exclusive_scan_int(in, out, count, tmp.p, tmp_bytes, s);
}

constexpr int MAX_RS = 64;  // short-range terms handled per particle

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// One wave per touched brick.  Lane (c1, c2) = (lane / 8, lane % 8) owns the
// eight cells (base0 + m, base1 + c1, base2 + c2), m = 0..7.  Per wave: the
// brick ids of its next bricks, the listed particles and their positions and
// charges are loaded one per lane and broadcast with readlane, and the cells
// to be updated are read before the particle loop, so the dependent global
// loads of a brick overlap.  The 1D factors exp(-t_k^2 (x - x_nu)^2) of one
// particle over the brick's 8 coordinates per axis live in LDS
// f[3][Rs][8] (each thread fills a few), then every lane sums its cells.
// The workgroup is one wave, so its barriers are cheap and many bricks stay
// in flight per compute unit; every wave leaves once active[0] bricks are
// done.
// DAX = -1: grid += the windowed short-range sum.  DAX = 0, 1 or 2: grid +=
// its finite difference along axis DAX (central, one-sided at the grid ends;
// the discrete gradient of eq Gradients_Tens applied to each local term):
// every local term is separable, a_k z prod_l g_kl(i_l) chi_l(i_l) with chi_l
// the window's indicator, so only the axis-DAX factor changes, to the
// difference of g chi, which reaches one cell beyond the window (the brick
// lists must be built for windows of n_s + 2).
// The factors, their products and the sums are formed in the grid's own
// type (FP32 for an FP32 grid, exponentials from FP64 arguments), the
// positions and the exponents' arguments in FP64.
template <class GT, int DAX>
__global__ __launch_bounds__(64) void short_gather_kernel(
    GT* __restrict__ grid, const double* __restrict__ pos, const double* __restrict__ q,
    const double* __restrict__ t, const double* __restrict__ a, int R, int R_l, int64_t n,
    double b, int w, int nb, const int* __restrict__ start, const int* __restrict__ list,
    const int* __restrict__ active, int64_t active_cap) {
  extern __shared__ double sg_lds[];
  const int Rs = R - R_l;
  GT* f = (GT*)sg_lds;              // [3][Rs][8] (in the space of 24 Rs doubles)
  double* ak = sg_lds + 24 * Rs;    // [Rs]
  double* tk2 = ak + Rs;            // [Rs]
  const int lane = threadIdx.x;
  for (int k = lane; k < Rs; k += 64) {
    ak[k] = a[R_l + k];
    tk2[k] = t[R_l + k] * t[R_l + k];
  }
  const double h = 2.0 * b / (double)n;
  const int c1 = lane >> 3, c2 = lane & 7;
  const int n_active = (int)(active[0] < active_cap ? active[0] : active_cap);
  const int G = gridDim.x;
  for (int ia0 = blockIdx.x; ia0 < n_active; ia0 += 64 * G) {
    // lane j holds brick ia0 + j * G of this wave's share
    const int64_t mine = (int64_t)ia0 + (int64_t)lane * G;
    const int mybr = mine < n_active ? active[1 + mine] : 0;
    const int nbk = (int)std::min<int64_t>(64, ((int64_t)n_active - ia0 + G - 1) / G);
    for (int j = 0; j < nbk; ++j) {
      const int br = __builtin_amdgcn_readlane(mybr, j);
      const int b0 = br / (nb * nb), b1 = (br / nb) % nb, b2 = br % nb;
      const int base0 = b0 * 8, base1 = b1 * 8, base2 = b2 * 8;
      const int64_t i1 = base1 + c1, i2 = base2 + c2;
      const bool col_ok = i1 < n && i2 < n;
      GT old[8];
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const int64_t i0 = base0 + m;
        old[m] = (col_ok && i0 < n) ? grid[(i0 * n + i1) * n + i2] : (GT)0;
      }
      GT acc[8];
#pragma unroll
      for (int m = 0; m < 8; ++m) acc[m] = (GT)0;
      const int s0 = start[br], s1 = start[br + 1];
      for (int e0 = s0; e0 < s1; e0 += 64) {
        const int cnt = std::min(64, s1 - e0);
        const int mynu = lane < cnt ? list[e0 + lane] : list[e0];
        const double px = pos[3 * (int64_t)mynu], py = pos[3 * (int64_t)mynu + 1],
                     pz = pos[3 * (int64_t)mynu + 2], pq = q[mynu];
        for (int e = 0; e < cnt; ++e) {
          const double p[3] = {readlane_f64(px, e), readlane_f64(py, e), readlane_f64(pz, e)};
          const double z = readlane_f64(pq, e);
          int lo[3], hi[3];
          int64_t glo[3], ghi[3];
          const int bs[3] = {base0, base1, base2};
#pragma unroll
          for (int l = 0; l < 3; ++l) {
            int64_t jc = (int64_t)floor((p[l] + b) / h);
            jc = jc < 0 ? 0 : (jc > n - 1 ? n - 1 : jc);
            glo[l] = jc - w < 0 ? 0 : jc - w;
            ghi[l] = jc + w > n - 1 ? n - 1 : jc + w;
            lo[l] = (int)(glo[l] - bs[l]);
            hi[l] = (int)(ghi[l] - bs[l]);
          }
          if (DAX >= 0) {   // the masked difference vanishes outside itself
            lo[DAX] = -BRICK;
            hi[DAX] = 2 * BRICK;
          }
          __syncthreads();  // the previous particle's factors are no longer read
          for (int idx = lane; idx < 24 * Rs; idx += 64) {
            const int l = idx / (8 * Rs);
            const int rem = idx - l * 8 * Rs;
            const int k = rem >> 3, m = rem & 7;
            const int64_t gi = bs[l] + m;
            if (l != DAX) {
              const double d = (-b + ((double)gi + 0.5) * h) - p[l];
              if constexpr (sizeof(GT) == 4) f[idx] = expf((float)(-tk2[k] * (d * d)));
              else f[idx] = exp(-tk2[k] * (d * d));
            } else {
              // g chi at global index j (0 outside the window and the grid)
              auto gchi = [&](int64_t j) {
                if (j < glo[l] || j > ghi[l]) return 0.0;
                const double d = (-b + ((double)j + 0.5) * h) - p[l];
                return exp(-tk2[k] * (d * d));
              };
              double v = 0.0;
              if (gi < n) {
                if (gi == 0) v = (gchi(1) - gchi(0)) / h;
                else if (gi == n - 1) v = (gchi(n - 1) - gchi(n - 2)) / h;
                else v = (gchi(gi + 1) - gchi(gi - 1)) / (2.0 * h);
              }
              f[idx] = (GT)v;
            }
          }
          __syncthreads();
          if (c1 >= lo[1] && c1 <= hi[1] && c2 >= lo[2] && c2 <= hi[2]) {
            GT s[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) s[m] = (GT)0;
            for (int k = 0; k < Rs; ++k) {
              const GT g = (GT)ak[k] * f[(Rs + k) * 8 + c1] * f[(2 * Rs + k) * 8 + c2];
#pragma unroll
              for (int m = 0; m < 8; ++m) s[m] += g * f[k * 8 + m];
            }
#pragma unroll
            for (int m = 0; m < 8; ++m)
              if (m >= lo[0] && m <= hi[0]) acc[m] += (GT)z * s[m];
          }
        }
      }
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const int64_t i0 = base0 + m;
        if (col_ok && i0 < n && acc[m] != (GT)0)
          grid[(i0 * n + i1) * n + i2] = old[m] + acc[m];
      }
    }
  }
}

template <class GT, int DAX>
static void short_gather_t(GT* grid, const double* pos, const double* q, const double* t,
                           const double* a, int R, int R_l, int64_t n, double b, int w, int nb,
                           const int* start, const int* list, const int* active, int64_t active_cap,
                           int64_t wgs, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL((short_gather_kernel<GT, DAX>), dim3((unsigned)wgs), dim3(64), lds, s, grid,
                     pos, q, t, a, R, R_l, n, b, w, nb, start, list, active, active_cap);
}

template <class GT>
static void short_gather_axis(int dax, GT* grid, const double* pos, const double* q,
                              const double* t, const double* a, int R, int R_l, int64_t n, double b,
                              int w, int nb, const int* start, const int* list, const int* active,
                              int64_t active_cap, int64_t wgs, size_t lds, hipStream_t s) {
  switch (dax) {
    case -1: short_gather_t<GT, -1>(grid, pos, q, t, a, R, R_l, n, b, w, nb, start, list, active, active_cap, wgs, lds, s); break;
    case 0: short_gather_t<GT, 0>(grid, pos, q, t, a, R, R_l, n, b, w, nb, start, list, active, active_cap, wgs, lds, s); break;
    case 1: short_gather_t<GT, 1>(grid, pos, q, t, a, R, R_l, n, b, w, nb, start, list, active, active_cap, wgs, lds, s); break;
    case 2: short_gather_t<GT, 2>(grid, pos, q, t, a, R, R_l, n, b, w, nb, start, list, active, active_cap, wgs, lds, s); break;
    default: throw Error{RS_E_INVALID, "axis must be 0, 1 or 2"};
  }
}

void short_gather(void* grid, int grid_fp32, const double* pos, const double* q, const double* t,
                  const double* a, int R, int R_l, int64_t n, double b, int n_s, int nb,
                  const int* start, const int* list, const int* active, int64_t active_cap,
                  int num_cu, hipStream_t s, int dax) {
  if (R - R_l > MAX_RS) throw Error{RS_E_UNSUPPORTED, "more than 64 short-range terms"};
  if (R - R_l <= 0) return;  // no short-range terms: nothing to add
  const int w = (n_s - 1) / 2;
  // 16 resident one-wave workgroups per compute unit, never more than there are bricks
  const int64_t wgs = std::max<int64_t>(1, std::min<int64_t>(active_cap, (int64_t)num_cu * 16));
  const size_t lds = (size_t)26 * (R - R_l) * sizeof(double);
  if (grid_fp32)
    short_gather_axis<float>(dax, (float*)grid, pos, q, t, a, R, R_l, n, b, w, nb, start, list,
                             active, active_cap, wgs, lds, s);
  else
    short_gather_axis<double>(dax, (double*)grid, pos, q, t, a, R, R_l, n, b, w, nb, start, list,
                              active, active_cap, wgs, lds, s);
}

}  // namespace rs
