// Point evaluation of the RS-Tucker tensor, interaction energy and forces.
//
// Long-range part at a point y: order-p tensor Lagrange interpolation of the
// Tucker field on the cell-centred grid.  With T2 = beta x_1 V1 x_2 V2
// (n x n x r3, kept by the tensor) and q3(y) = sum_m L_m(y_3) V3[s3 + m, :],
//   P_l(y) = sum_{m1, m2} L_{m1}(y_1) L_{m2}(y_2) < T2[s1+m1, s2+m2, :], q3(y) >,
// which equals beta x_1 q1(y) x_2 q2(y) x_3 q3(y) (Lemma Property_RST_Tuck at
// grid points, interpolated between them) at p^2 r3 instead of r^3 work.
// The gradient uses the derivative weights in one mode at a time.
//
// Energy (Lemma InterEnergy, eq EnergyFree_Tensor):
//   E = 1/2 sum_j z_j (P_l(x_j) - z_j g_j),
// g_j = particle j's own long-range reference term through the same
// interpolation operator (P_{R_l}(0) exactly when x_j is a grid point).
// Forces: F_j = -z_j grad[P_l - z_j g_j](x_j) (section 4.3, basis held fixed).
#include "rs_internal.h"

namespace rs {

constexpr int PMAX = 8;        // largest interpolation order

struct EvalDev {
  const double* T2;    // n x n x r3
  const double* V3;    // n x r3 row-major
  const float* T2f;    // FP32 copies (FP32 evaluation), or null
  const float* V3f;
  const double* t;     // R
  const double* a;     // R
  int64_t n;
  double b;
  int r3, R_l, p;
};

// Lagrange weights L_i and derivatives dL_i of the P-point stencil around y
// (cell-centred nodes s..s+P-1, clamped to the grid).
template <int P>
__device__ __forceinline__ void stencil(double y, double b, int64_t n, int& start, double* L,
                                        double* dL) {
  const double h = 2.0 * b / (double)n;
  const double u = (y + b) / h - 0.5;
  int m = (int)floor(u);
  int s = m - P / 2 + 1;
  if (s < 0) s = 0;
  if (s > (int)n - P) s = (int)n - P;
  start = s;
#pragma unroll
  for (int i = 0; i < P; ++i) {
    double num = 1.0, den = 1.0;
#pragma unroll
    for (int j = 0; j < P; ++j)
      if (j != i) {
        num *= (u - (double)(s + j));
        den *= (double)(i - j);
      }
    L[i] = num / den;
    double d = 0.0;
#pragma unroll
    for (int mm = 0; mm < P; ++mm) {
      if (mm == i) continue;
      double prod = 1.0;
#pragma unroll
      for (int j = 0; j < P; ++j)
        if (j != i && j != mm) prod *= (u - (double)(s + j));
      d += prod;
    }
    dL[i] = d / den / h;
  }
}

template <class VT>
__device__ __forceinline__ VT wsum(VT v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

template <class VT> __device__ __forceinline__ const VT* field_t2(const EvalDev& e);
template <> __device__ __forceinline__ const double* field_t2<double>(const EvalDev& e) { return e.T2; }
template <> __device__ __forceinline__ const float* field_t2<float>(const EvalDev& e) { return e.T2f; }
template <class VT> __device__ __forceinline__ const VT* field_v3(const EvalDev& e);
template <> __device__ __forceinline__ const double* field_v3<double>(const EvalDev& e) { return e.V3; }
template <> __device__ __forceinline__ const float* field_v3<float>(const EvalDev& e) { return e.V3f; }

// One wave per point; lanes over the rank index c (NC values each).  The
// stencil order P and NC are compile-time constants, so the P^2 rows of T2
// are addressed statically and their loads are all issued up front.  VT is
// the arithmetic of the field contraction and of the self terms (double, or
// float for the FP32 evaluation); the stencil weights are formed in FP64.
template <int P, int NC, class VT>
__global__ __launch_bounds__(256) void eval_long_kernel(EvalDev e, int64_t M,
                                                        const double* __restrict__ pts,
                                                        int with_self, double* __restrict__ val,
                                                        double* __restrict__ grad,
                                                        double* __restrict__ selfv,
                                                        double* __restrict__ selfg) {
  const int lane = threadIdx.x & 63;
  const int64_t pt = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (pt >= M) return;
  double y[3];
  int s[3];
  VT L[3][P], dL[3][P];
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    double Ld[P], dLd[P];
    y[l] = pts[3 * pt + l];
    stencil<P>(y[l], e.b, e.n, s[l], Ld, dLd);
#pragma unroll
    for (int m = 0; m < P; ++m) {
      L[l][m] = (VT)Ld[m];
      dL[l][m] = (VT)dLd[m];
    }
  }
  const int r3 = e.r3;
  const VT* V3 = field_v3<VT>(e);
  const VT* T2 = field_t2<VT>(e);
  VT q3[NC], dq3[NC];
#pragma unroll
  for (int u = 0; u < NC; ++u) {
    const int c = lane + 64 * u;
    VT qa = 0, qd = 0;
    if (c < r3) {
#pragma unroll
      for (int m = 0; m < P; ++m) {
        const VT v = V3[(int64_t)(s[2] + m) * r3 + c];
        qa += L[2][m] * v;
        qd += dL[2][m] * v;
      }
    }
    q3[u] = qa;
    dq3[u] = qd;
  }
  VT v = 0, g1 = 0, g2 = 0, g3 = 0;
#pragma unroll
  for (int m1 = 0; m1 < P; ++m1) {
#pragma unroll
    for (int m2 = 0; m2 < P; ++m2) {
      const VT* row = T2 + ((int64_t)(s[0] + m1) * e.n + (s[1] + m2)) * r3;
      VT d = 0, dd = 0;
#pragma unroll
      for (int u = 0; u < NC; ++u) {
        const int c = lane + 64 * u;
        const VT tv = c < r3 ? row[c] : (VT)0;
        d += tv * q3[u];
        dd += tv * dq3[u];
      }
      const VT w12 = L[0][m1] * L[1][m2];
      v += w12 * d;
      g1 += dL[0][m1] * L[1][m2] * d;
      g2 += L[0][m1] * dL[1][m2] * d;
      g3 += w12 * dd;
    }
  }
  v = wsum(v);
  if (grad) {
    g1 = wsum(g1);
    g2 = wsum(g2);
    g3 = wsum(g3);
  }
  VT sv = 0, sg[3] = {0, 0, 0};
  if (with_self) {
    // lanes over the long-range terms k < R_l (R_l <= 64)
    const double h = 2.0 * e.b / (double)e.n;
    VT phi[3] = {0, 0, 0}, dphi[3] = {0, 0, 0};
    if (lane < e.R_l) {
      const VT tk = (VT)e.t[lane];
#pragma unroll
      for (int l = 0; l < 3; ++l) {
#pragma unroll
        for (int m = 0; m < P; ++m) {
          const VT d = (VT)((-e.b + ((double)(s[l] + m) + 0.5) * h) - y[l]);
          const VT g = exp(-(tk * tk) * (d * d));
          phi[l] += L[l][m] * g;
          dphi[l] += dL[l][m] * g;
        }
      }
      const VT ak = (VT)e.a[lane];
      sv = ak * phi[0] * phi[1] * phi[2];
      sg[0] = ak * dphi[0] * phi[1] * phi[2];
      sg[1] = ak * phi[0] * dphi[1] * phi[2];
      sg[2] = ak * phi[0] * phi[1] * dphi[2];
    }
    sv = wsum(sv);
    for (int l = 0; l < 3; ++l) sg[l] = wsum(sg[l]);
  }
  if (lane == 0) {
    val[pt] = v;
    if (grad) {
      grad[3 * pt + 0] = g1;
      grad[3 * pt + 1] = g2;
      grad[3 * pt + 2] = g3;
    }
    if (with_self && selfv) selfv[pt] = sv;
    if (with_self && selfg)
      for (int l = 0; l < 3; ++l) selfg[3 * pt + l] = sg[l];
  }
}

template <int P>
static void launch_eval_p(const EvalDev& e, int64_t M, const double* pts, int with_self,
                          const EvalOut& out, hipStream_t s) {
  const int waves = 4;
  const dim3 grid((unsigned)((M + waves - 1) / waves)), block(64 * waves);
  const int nc = (e.r3 + 63) / 64;
#define RS_EVAL(NC, VT)                                                                           \
  hipLaunchKernelGGL((eval_long_kernel<P, NC, VT>), grid, block, 0, s, e, M, pts, with_self,      \
                     out.val, out.grad, out.selfv, out.selfg)
  if (e.T2f) {
    if (nc <= 1) RS_EVAL(1, float);
    else if (nc <= 2) RS_EVAL(2, float);
    else if (nc <= 4) RS_EVAL(4, float);
    else if (nc <= 8) RS_EVAL(8, float);
    else RS_EVAL(16, float);
  } else {
    if (nc <= 1) RS_EVAL(1, double);
    else if (nc <= 2) RS_EVAL(2, double);
    else if (nc <= 4) RS_EVAL(4, double);
    else if (nc <= 8) RS_EVAL(8, double);
    else RS_EVAL(16, double);
  }
#undef RS_EVAL
}

void launch_eval_long(const rs_tensor* T, int64_t M, const double* pts, int with_self,
                      const EvalOut& out, hipStream_t s) {
  if (T->r[2] > 1024) throw Error{RS_E_UNSUPPORTED, "rank r3 above 1024"};
  if (T->interp > PMAX || T->interp < 2 || T->interp % 2)
    throw Error{RS_E_UNSUPPORTED, "interpolation order must be 2, 4, 6 or 8"};
  if (with_self && T->R_l > 64) throw Error{RS_E_UNSUPPORTED, "more than 64 long-range terms"};
  if (M <= 0) return;
  EvalDev e;
  e.T2 = T->T2.as<double>();
  e.V3 = T->Q[2].as<double>();
  e.T2f = T->T2f.as<float>();
  e.V3f = T->V3f.as<float>();
  e.t = T->t_dev.as<double>();
  e.a = T->a_dev.as<double>();
  e.n = T->n;
  e.b = T->b;
  e.r3 = T->r[2];
  e.R_l = T->R_l;
  e.p = T->interp;
  switch (T->interp) {
    case 2: launch_eval_p<2>(e, M, pts, with_self, out, s); break;
    case 4: launch_eval_p<4>(e, M, pts, with_self, out, s); break;
    case 6: launch_eval_p<6>(e, M, pts, with_self, out, s); break;
    default: launch_eval_p<8>(e, M, pts, with_self, out, s); break;
  }
}

// Short-range part at arbitrary points: particles whose window contains the
// point's cell, in index order (from the brick lists), Gaussians at the point.
// GRAD: the gradient in y of the same terms instead (M x 3 output), each term
// a_k exp(-t_k^2 |y - x|^2) differentiated analytically.
template <bool GRAD>
__global__ void eval_short_kernel(int64_t M, const double* __restrict__ pts,
                                  const double* __restrict__ pos, const double* __restrict__ q,
                                  const double* __restrict__ t, const double* __restrict__ a,
                                  int R, int R_l, int64_t n, double b, int w, int nb,
                                  const int* __restrict__ start, const int* __restrict__ list,
                                  double* __restrict__ vals, int accumulate) {
  int64_t pt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pt >= M) return;
  const double h = 2.0 * b / (double)n;
  double y[3];
  int64_t cell[3];
  for (int l = 0; l < 3; ++l) {
    y[l] = pts[3 * pt + l];
    int64_t j = (int64_t)floor((y[l] + b) / h);
    cell[l] = j < 0 ? 0 : (j > n - 1 ? n - 1 : j);
  }
  const int64_t br = ((cell[0] / 8) * nb + cell[1] / 8) * nb + cell[2] / 8;
  double acc = 0.0, gacc[3] = {0.0, 0.0, 0.0};
  for (int e = start[br]; e < start[br + 1]; ++e) {
    const int nu = list[e];
    bool inside = true;
    double r2 = 0.0, d[3];
    for (int l = 0; l < 3; ++l) {
      const double x = pos[3 * nu + l];
      int64_t j = (int64_t)floor((x + b) / h);
      j = j < 0 ? 0 : (j > n - 1 ? n - 1 : j);
      if (cell[l] < j - w || cell[l] > j + w) inside = false;
      d[l] = y[l] - x;
      r2 += d[l] * d[l];
    }
    if (!inside) continue;
    if (GRAD) {
      double ds = 0.0;   // d/d(r^2) of the term sum
      for (int k = R_l; k < R; ++k) ds -= t[k] * t[k] * a[k] * exp(-t[k] * t[k] * r2);
      for (int l = 0; l < 3; ++l) gacc[l] += q[nu] * 2.0 * ds * d[l];
    } else {
      double sum = 0.0;
      for (int k = R_l; k < R; ++k) sum += a[k] * exp(-t[k] * t[k] * r2);
      acc += q[nu] * sum;
    }
  }
  if (GRAD) {
    for (int l = 0; l < 3; ++l)
      vals[3 * pt + l] = accumulate ? vals[3 * pt + l] + gacc[l] : gacc[l];
  } else {
    vals[pt] = accumulate ? vals[pt] + acc : acc;
  }
}

static void launch_short(bool grad, const rs_tensor* T, int64_t M, const double* pts, double* out,
                         int accumulate, hipStream_t s) {
  const dim3 grid((unsigned)((M + 127) / 128)), block(128);
#define RS_SHORT(G)                                                                               \
  hipLaunchKernelGGL(eval_short_kernel<G>, grid, block, 0, s, M, pts, T->pos.as<double>(),        \
                     T->q.as<double>(), T->t_dev.as<double>(), T->a_dev.as<double>(), T->R,        \
                     T->R_l, T->n, T->b, (T->n_s - 1) / 2, T->nb, T->brick_start.as<int>(),      \
                     T->brick_list.as<int>(), out, accumulate)
  if (grad) RS_SHORT(true);
  else RS_SHORT(false);
#undef RS_SHORT
}

void launch_eval_short(const rs_tensor* T, int64_t M, const double* pts, double* vals,
                       int accumulate, hipStream_t s) {
  launch_short(false, T, M, pts, vals, accumulate, s);
}

void launch_eval_short_grad(const rs_tensor* T, int64_t M, const double* pts, double* grad,
                            int accumulate, hipStream_t s) {
  launch_short(true, T, M, pts, grad, accumulate, s);
}

__global__ void normal_dot_kernel(const double* __restrict__ g, const double* __restrict__ nrm,
                                  int64_t M, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < M) out[i] = g[3 * i] * nrm[3 * i] + g[3 * i + 1] * nrm[3 * i + 1] + g[3 * i + 2] * nrm[3 * i + 2];
}

void launch_normal_dot(const double* grad, const double* normals, int64_t M, double* out,
                       hipStream_t s) {
  hipLaunchKernelGGL(normal_dot_kernel, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, grad,
                     normals, M, out);
}

// Single workgroup, fixed-order FP64 reduction.
constexpr int RED_THREADS = 1024;
__global__ __launch_bounds__(RED_THREADS) void energy_kernel(const double* __restrict__ q,
                                                             const double* __restrict__ v,
                                                             const double* __restrict__ g,
                                                             int64_t N, double* __restrict__ E,
                                                             double* __restrict__ dEdq) {
  __shared__ double red[RED_THREADS / 64];
  double acc = 0.0;
  for (int64_t j = threadIdx.x; j < N; j += RED_THREADS) {
    const double d = v[j] - q[j] * g[j];
    if (dEdq) dEdq[j] = d;
    acc += q[j] * d;
  }
  acc = wsum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < RED_THREADS / 64; ++w) s += red[w];
    *E = 0.5 * s;
  }
}

void launch_energy_reduce(const double* q, const double* v, const double* g, int64_t N, double* E,
                          double* dEdq, hipStream_t s) {
  hipLaunchKernelGGL(energy_kernel, dim3(1), dim3(RED_THREADS), 0, s, q, v, g, N, E, dEdq);
}

__global__ void forces_kernel(const double* __restrict__ q, const double* __restrict__ gv,
                              const double* __restrict__ gg, int64_t N, double scale,
                              double* __restrict__ F) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 3 * N) return;
  const int64_t j = e / 3;
  F[e] = -scale * q[j] * (gv[e] - q[j] * gg[e]);
}

__global__ void to_float_kernel(const double* __restrict__ in, int64_t count, float* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}

void launch_to_float(const double* in, int64_t count, float* out, hipStream_t s) {
  if (count <= 0) return;
  const unsigned blocks = (unsigned)std::min<int64_t>((count + 255) / 256, 8192);
  hipLaunchKernelGGL(to_float_kernel, dim3(blocks), dim3(256), 0, s, in, count, out);
}

void launch_forces(const double* q, const double* gradv, const double* gradg, int64_t N,
                   double scale, double* F, hipStream_t s) {
  hipLaunchKernelGGL(forces_kernel, dim3((unsigned)((3 * N + 255) / 256)), dim3(256), 0, s, q,
                     gradv, gradg, N, scale, F);
}

}  // namespace rs
