// Vector kernels of the Krylov solvers (paper Sec. 1: flexible GMRES outer
// solver; GMRES on the coarsest level).  Every reduction is deterministic:
// per-workgroup partial sums in FP64 written to a fixed slot, then summed in a
// fixed order by a second kernel.  All Krylov scalars (Hessenberg matrix,
// Givens rotations, least-squares right-hand side) live in device memory; the
// host reads back one residual estimate per iteration at most.
#include "kernels.hpp"

namespace ddamg {

constexpr int KCHUNK = 8;

// partial[i*nwg + blk] = sum over this workgroup's elements of conj(V_i) w
template <class R>
__global__ void __launch_bounds__(256) k_multidot(const cx<R>* __restrict__ V, long ldv, int k,
                                                  const cx<R>* __restrict__ w, long N,
                                                  cx<double>* __restrict__ partial) {
  __shared__ double red[KCHUNK][4][2];
  int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  long stride = (long)gridDim.x * blockDim.x;
  for (int i0 = 0; i0 < k; i0 += KCHUNK) {
    double acc[KCHUNK][2];
#pragma unroll
    for (int ii = 0; ii < KCHUNK; ++ii) acc[ii][0] = acc[ii][1] = 0.0;
    for (long e = (long)blockIdx.x * blockDim.x + t; e < N; e += stride) {
      cx<R> wv_ = w[e];
#pragma unroll
      for (int ii = 0; ii < KCHUNK; ++ii) {
        if (i0 + ii < k) {
          cx<R> v = V[(long)(i0 + ii) * ldv + e];
          acc[ii][0] += (double)v.re * wv_.re + (double)v.im * wv_.im;
          acc[ii][1] += (double)v.re * wv_.im - (double)v.im * wv_.re;
        }
      }
    }
#pragma unroll
    for (int ii = 0; ii < KCHUNK; ++ii)
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        double v = wave_sum_n(acc[ii][p], 64);
        if (lane == 0) red[ii][wv][p] = v;
      }
    __syncthreads();
    if (t < KCHUNK && i0 + t < k) {
      double re = red[t][0][0] + red[t][1][0] + red[t][2][0] + red[t][3][0];
      double im = red[t][0][1] + red[t][1][1] + red[t][2][1] + red[t][3][1];
      partial[(long)(i0 + t) * gridDim.x + blockIdx.x] = mk(re, im);
    }
    __syncthreads();
  }
}

template <class R>
void launch_multidot(const cx<R>* V, long ldv, int k, const cx<R>* w, long N, cx<double>* partial, int nwg,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_multidot<R>, dim3(nwg), dim3(256), 0, st, V, ldv, k, w, N, partial);
}

// mode 0: out[i] = sum;  1: out[i] += sum;  2: out[i] = sqrt(re(sum))
__global__ void __launch_bounds__(256) k_reduce(const cx<double>* __restrict__ partial, int nwg,
                                                cx<double>* __restrict__ out, int mode) {
  __shared__ double red[4][2];
  int i = blockIdx.x, t = threadIdx.x, lane = t & 63, wv = t >> 6;
  double re = 0, im = 0;
  for (int e = t; e < nwg; e += 256) {
    cx<double> v = partial[(long)i * nwg + e];
    re += v.re;
    im += v.im;
  }
  re = wave_sum_n(re, 64);
  im = wave_sum_n(im, 64);
  if (lane == 0) {
    red[wv][0] = re;
    red[wv][1] = im;
  }
  __syncthreads();
  if (t == 0) {
    double r = red[0][0] + red[1][0] + red[2][0] + red[3][0];
    double m = red[0][1] + red[1][1] + red[2][1] + red[3][1];
    if (mode == 0) out[i] = mk(r, m);
    else if (mode == 1) out[i] = out[i] + mk(r, m);
    else out[i] = mk(sqrt(r > 0 ? r : 0.0), 0.0);
  }
}
void launch_reduce(const cx<double>* partial, int k, int nwg, cx<double>* out, int mode, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce, dim3(k), dim3(256), 0, st, partial, nwg, out, mode);
}

// w += sign * sum_i coef_i V_i
template <class R>
__global__ void __launch_bounds__(256) k_multi_axpy(const cx<R>* __restrict__ V, long ldv, int k,
                                                    const cx<double>* __restrict__ coef, double sign,
                                                    cx<R>* __restrict__ w, long N) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  cx<double> acc = mk(0.0, 0.0);
  for (int i = 0; i < k; ++i) {
    cx<R> v = V[(long)i * ldv + e];
    cmac(acc, coef[i], mk<double>(v.re, v.im));
  }
  cx<R> x = w[e];
  w[e] = mk<R>((R)(x.re + sign * acc.re), (R)(x.im + sign * acc.im));
}
template <class R>
void launch_multi_axpy(const cx<R>* V, long ldv, int k, const cx<double>* coef, double sign, cx<R>* w, long N,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_multi_axpy<R>, dim3((N + 255) / 256), dim3(256), 0, st, V, ldv, k, coef, sign, w, N);
}

// out = in / s  (s real, stored as the real part)
template <class R>
__global__ void k_scale_by_inv(const cx<R>* __restrict__ in, const cx<double>* __restrict__ s, cx<R>* __restrict__ out,
                               long N) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  double d = s[0].re;
  double f = d > 0 ? 1.0 / d : 0.0;
  cx<R> v = in[e];
  out[e] = mk<R>((R)(f * v.re), (R)(f * v.im));
}
template <class R>
void launch_scale_by_inv(const cx<R>* in, const cx<double>* s, cx<R>* out, long N, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_by_inv<R>, dim3((N + 255) / 256), dim3(256), 0, st, in, s, out, N);
}

template <class RA, class RB>
__global__ void k_copy_cvt(const cx<RA>* __restrict__ in, cx<RB>* __restrict__ out, long N) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  cx<RA> v = in[e];
  out[e] = mk<RB>((RB)v.re, (RB)v.im);
}
template <class RA, class RB>
void launch_copy_cvt(const cx<RA>* in, cx<RB>* out, long N, hipStream_t st) {
  hipLaunchKernelGGL((k_copy_cvt<RA, RB>), dim3((N + 255) / 256), dim3(256), 0, st, in, out, N);
}

template <class R>
__global__ void k_axpby(long N, double a, const cx<R>* __restrict__ x, double b, cx<R>* __restrict__ y) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  cx<R> xv = x[e], yv = y[e];
  y[e] = mk<R>((R)(a * xv.re + b * yv.re), (R)(a * xv.im + b * yv.im));
}
template <class R>
void launch_axpby(long N, double a, const cx<R>* x, double b, cx<R>* y, hipStream_t st) {
  hipLaunchKernelGGL(k_axpby<R>, dim3((N + 255) / 256), dim3(256), 0, st, N, a, x, b, y);
}

template <class R>
__global__ void k_sub(long N, const cx<R>* __restrict__ a, const cx<R>* __restrict__ b, cx<R>* __restrict__ out) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  out[e] = a[e] - b[e];
}
template <class R>
void launch_sub(long N, const cx<R>* a, const cx<R>* b, cx<R>* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sub<R>, dim3((N + 255) / 256), dim3(256), 0, st, N, a, b, out);
}

template <class R>
__global__ void k_zero(long N, cx<R>* __restrict__ x) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < N) x[e] = mk<R>(0, 0);
}
template <class R>
void launch_zero(long N, cx<R>* x, hipStream_t st) {
  if (N > 0) hipLaunchKernelGGL(k_zero<R>, dim3((N + 255) / 256), dim3(256), 0, st, N, x);
}

// Givens step j on the Hessenberg column j (column-major, leading dimension
// ldh): apply the previous rotations, form rotation j (real cosine), update g,
// write |g_{j+1}| to resid.
__global__ void k_givens(cx<double>* H, int ldh, double* cs, cx<double>* sn, cx<double>* g, int j, double* resid) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  cx<double>* h = H + (long)j * ldh;
  for (int i = 0; i < j; ++i) {
    cx<double> a = h[i], b = h[i + 1];
    h[i] = cs[i] * a + sn[i] * b;
    h[i + 1] = cs[i] * b - conj(sn[i]) * a;
  }
  cx<double> a = h[j], b = h[j + 1];
  double den = sqrt(norm2(a) + norm2(b));
  double c;
  cx<double> s;
  if (den == 0.0) {
    c = 1.0;
    s = mk(0.0, 0.0);
  } else if (norm2(a) == 0.0) {
    c = 0.0;
    s = mk(1.0, 0.0);
  } else {
    double aa = sqrt(norm2(a));
    c = aa / den;
    s = (1.0 / (aa * den)) * (a * conj(b));
  }
  cs[j] = c;
  sn[j] = s;
  h[j] = c * a + s * b;
  h[j + 1] = mk(0.0, 0.0);
  cx<double> gj = g[j];
  g[j + 1] = -(conj(s) * gj);
  g[j] = c * gj;
  resid[0] = sqrt(norm2(g[j + 1]));
}
void launch_givens(cx<double>* H, int ldh, double* cs, cx<double>* sn, cx<double>* g, int j, double* resid,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_givens, dim3(1), dim3(64), 0, st, H, ldh, cs, sn, g, j, resid);
}

// back substitution of the j x j upper-triangular least-squares system
__global__ void k_trisolve(const cx<double>* H, int ldh, const cx<double>* g, cx<double>* y, int j) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = j - 1; i >= 0; --i) {
    cx<double> s = g[i];
    for (int k = i + 1; k < j; ++k) s = s - H[(long)k * ldh + i] * y[k];
    cx<double> d = H[(long)i * ldh + i];
    double dn = norm2(d);
    y[i] = dn > 0 ? (1.0 / dn) * (s * conj(d)) : mk(0.0, 0.0);
  }
}
void launch_trisolve(const cx<double>* H, int ldh, const cx<double>* g, cx<double>* y, int j, hipStream_t st) {
  hipLaunchKernelGGL(k_trisolve, dim3(1), dim3(64), 0, st, H, ldh, g, y, j);
}

__global__ void k_set_scalar(cx<double>* dst, const cx<double>* src) {
  if (threadIdx.x == 0 && blockIdx.x == 0) dst[0] = src[0];
}
void launch_set_scalar(cx<double>* dst, const cx<double>* src, hipStream_t st) {
  hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(64), 0, st, dst, src);
}

#define INST_B(R)                                                                                                \
  template void launch_multidot<R>(const cx<R>*, long, int, const cx<R>*, long, cx<double>*, int, hipStream_t); \
  template void launch_multi_axpy<R>(const cx<R>*, long, int, const cx<double>*, double, cx<R>*, long,          \
                                     hipStream_t);                                                              \
  template void launch_scale_by_inv<R>(const cx<R>*, const cx<double>*, cx<R>*, long, hipStream_t);             \
  template void launch_axpby<R>(long, double, const cx<R>*, double, cx<R>*, hipStream_t);                       \
  template void launch_sub<R>(long, const cx<R>*, const cx<R>*, cx<R>*, hipStream_t);                           \
  template void launch_zero<R>(long, cx<R>*, hipStream_t);
INST_B(double)
INST_B(float)
template void launch_copy_cvt<double, float>(const cx<double>*, cx<float>*, long, hipStream_t);
template void launch_copy_cvt<float, double>(const cx<float>*, cx<double>*, long, hipStream_t);
template void launch_copy_cvt<double, double>(const cx<double>*, cx<double>*, long, hipStream_t);
template void launch_copy_cvt<float, float>(const cx<float>*, cx<float>*, long, hipStream_t);



// ---------------------------------------------------------------------------
// Column-batched forms: K independent Krylov processes advance in lock step.
// Column r = blockIdx.y; every vector argument carries a column stride (cs*),
// every scalar array a per-column stride; columns with act[r] == 0 are skipped.
namespace {
__device__ __forceinline__ bool col_off(const int* act) { return act && !act[blockIdx.y]; }
}  // namespace

template <class R>
__global__ void __launch_bounds__(256) k_multidot_b(const cx<R>* __restrict__ V, long ldv, long csV, int k,
                                                    const cx<R>* __restrict__ w, long csw, long N,
                                                    cx<double>* __restrict__ partial, long pcs, const int* act) {
  if (col_off(act)) return;
  const long r = blockIdx.y;
  V += r * csV;
  w += r * csw;
  partial += r * pcs;
  __shared__ double red[KCHUNK][4][2];
  int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  long stride = (long)gridDim.x * blockDim.x;
  for (int i0 = 0; i0 < k; i0 += KCHUNK) {
    double acc[KCHUNK][2];
#pragma unroll
    for (int ii = 0; ii < KCHUNK; ++ii) acc[ii][0] = acc[ii][1] = 0.0;
    for (long e = (long)blockIdx.x * blockDim.x + t; e < N; e += stride) {
      cx<R> wv_ = w[e];
#pragma unroll
      for (int ii = 0; ii < KCHUNK; ++ii) {
        if (i0 + ii < k) {
          cx<R> v = V[(long)(i0 + ii) * ldv + e];
          acc[ii][0] += (double)v.re * wv_.re + (double)v.im * wv_.im;
          acc[ii][1] += (double)v.re * wv_.im - (double)v.im * wv_.re;
        }
      }
    }
#pragma unroll
    for (int ii = 0; ii < KCHUNK; ++ii)
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        double v = wave_sum_n(acc[ii][p], 64);
        if (lane == 0) red[ii][wv][p] = v;
      }
    __syncthreads();
    if (t < KCHUNK && i0 + t < k) {
      double re = red[t][0][0] + red[t][1][0] + red[t][2][0] + red[t][3][0];
      double im = red[t][0][1] + red[t][1][1] + red[t][2][1] + red[t][3][1];
      partial[(long)(i0 + t) * gridDim.x + blockIdx.x] = mk(re, im);
    }
    __syncthreads();
  }
}
template <class R>
void launch_multidot_b(const cx<R>* V, long ldv, long csV, int k, const cx<R>* w, long csw, long N, cx<double>* partial,
                       long pcs, int nwg, int K, const int* act, hipStream_t st) {
  hipLaunchKernelGGL(k_multidot_b<R>, dim3(nwg, K), dim3(256), 0, st, V, ldv, csV, k, w, csw, N, partial, pcs, act);
}

__global__ void __launch_bounds__(256) k_reduce_b(const cx<double>* __restrict__ partial, long pcs, int nwg,
                                                  cx<double>* __restrict__ out, long ocs, int mode, const int* act) {
  if (col_off(act)) return;
  partial += blockIdx.y * pcs;
  out += blockIdx.y * ocs;
  __shared__ double red[4][2];
  int i = blockIdx.x, t = threadIdx.x, lane = t & 63, wv = t >> 6;
  double re = 0, im = 0;
  for (int e = t; e < nwg; e += 256) {
    cx<double> v = partial[(long)i * nwg + e];
    re += v.re;
    im += v.im;
  }
  re = wave_sum_n(re, 64);
  im = wave_sum_n(im, 64);
  if (lane == 0) {
    red[wv][0] = re;
    red[wv][1] = im;
  }
  __syncthreads();
  if (t == 0) {
    double r = red[0][0] + red[1][0] + red[2][0] + red[3][0];
    double m = red[0][1] + red[1][1] + red[2][1] + red[3][1];
    if (mode == 0) out[i] = mk(r, m);
    else if (mode == 1) out[i] = out[i] + mk(r, m);
    else out[i] = mk(sqrt(r > 0 ? r : 0.0), 0.0);
  }
}
void launch_reduce_b(const cx<double>* partial, long pcs, int k, int nwg, cx<double>* out, long ocs, int mode, int K,
                     const int* act, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_b, dim3(k, K), dim3(256), 0, st, partial, pcs, nwg, out, ocs, mode, act);
}

// w_r += sign * sum_{i<k_r} coef_r[i] V_r[i]   (k_r = kcol ? kcol[r] : k)
template <class R, class RW = R>
__global__ void __launch_bounds__(256) k_multi_axpy_b(const cx<R>* __restrict__ V, long ldv, long csV, int k,
                                                      const int* kcol, const cx<double>* __restrict__ coef, long ccs,
                                                      double sign, cx<RW>* __restrict__ w, long csw, long N,
                                                      const int* act) {
  if (col_off(act)) return;
  const long r = blockIdx.y;
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  const int kk = kcol ? kcol[r] : k;
  V += r * csV;
  coef += r * ccs;
  w += r * csw;
  cx<double> acc = mk(0.0, 0.0);
  for (int i = 0; i < kk; ++i) {
    cx<R> v = V[(long)i * ldv + e];
    cmac(acc, coef[i], mk<double>(v.re, v.im));
  }
  cx<RW> x = w[e];
  w[e] = mk<RW>((RW)(x.re + sign * acc.re), (RW)(x.im + sign * acc.im));
}
template <class R>
void launch_multi_axpy_b(const cx<R>* V, long ldv, long csV, int k, const int* kcol, const cx<double>* coef, long ccs,
                         double sign, cx<R>* w, long csw, long N, int K, const int* act, hipStream_t st) {
  hipLaunchKernelGGL(k_multi_axpy_b<R>, dim3((N + 255) / 256, K), dim3(256), 0, st, V, ldv, csV, k, kcol, coef, ccs,
                     sign, w, csw, N, act);
}
// w (FP64) += sign * sum_i coef_i V_i with an FP32 basis V (the outer solve's
// preconditioned directions in the mixed form)
void launch_multi_axpy_b_mixed(const cx<float>* V, long ldv, long csV, int k, const int* kcol, const cx<double>* coef,
                               long ccs, double sign, cx<double>* w, long csw, long N, int K, const int* act,
                               hipStream_t st) {
  hipLaunchKernelGGL((k_multi_axpy_b<float, double>), dim3((N + 255) / 256, K), dim3(256), 0, st, V, ldv, csV, k,
                     kcol, coef, ccs, sign, w, csw, N, act);
}

// out_r = in_r / s_r (real part);  an inactive column is zeroed when zero_off
template <class R>
__global__ void k_scale_by_inv_b(const cx<R>* __restrict__ in, long csi, const cx<double>* __restrict__ s, long scs,
                                 cx<R>* __restrict__ out, long cso, long N, const int* act, int zero_off) {
  const long r = blockIdx.y;
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  if (act && !act[r]) {
    if (zero_off) out[r * cso + e] = mk<R>(0, 0);
    return;
  }
  double d = s[r * scs].re;
  double f = d > 0 ? 1.0 / d : 0.0;
  cx<R> v = in[r * csi + e];
  out[r * cso + e] = mk<R>((R)(f * v.re), (R)(f * v.im));
}
template <class R>
void launch_scale_by_inv_b(const cx<R>* in, long csi, const cx<double>* s, long scs, cx<R>* out, long cso, long N,
                           int K, const int* act, int zero_off, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_by_inv_b<R>, dim3((N + 255) / 256, K), dim3(256), 0, st, in, csi, s, scs, out, cso, N, act,
                     zero_off);
}

template <class RA, class RB>
__global__ void k_copy_cvt_b(const cx<RA>* __restrict__ in, long csi, cx<RB>* __restrict__ out, long cso, long N) {
  const long r = blockIdx.y;
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  cx<RA> v = in[r * csi + e];
  out[r * cso + e] = mk<RB>((RB)v.re, (RB)v.im);
}
template <class RA, class RB>
void launch_copy_cvt_b(const cx<RA>* in, long csi, cx<RB>* out, long cso, long N, int K, hipStream_t st) {
  hipLaunchKernelGGL((k_copy_cvt_b<RA, RB>), dim3((N + 255) / 256, K), dim3(256), 0, st, in, csi, out, cso, N);
}

// out_r = a_r - b_r
template <class R>
__global__ void k_sub_b(long N, const cx<R>* __restrict__ a, long csa, const cx<R>* __restrict__ b, long csb,
                        cx<R>* __restrict__ out, long cso) {
  const long r = blockIdx.y;
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  out[r * cso + e] = a[r * csa + e] - b[r * csb + e];
}
template <class R>
void launch_sub_b(long N, const cx<R>* a, long csa, const cx<R>* b, long csb, cx<R>* out, long cso, int K,
                  hipStream_t st) {
  if (N > 0) hipLaunchKernelGGL(k_sub_b<R>, dim3((N + 255) / 256, K), dim3(256), 0, st, N, a, csa, b, csb, out, cso);
}

template <class R>
__global__ void k_zero_b(long N, cx<R>* __restrict__ x, long cs) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < N) x[blockIdx.y * cs + e] = mk<R>(0, 0);
}
template <class R>
void launch_zero_b(long N, cx<R>* x, long cs, int K, hipStream_t st) {
  if (N > 0) hipLaunchKernelGGL(k_zero_b<R>, dim3((N + 255) / 256, K), dim3(256), 0, st, N, x, cs);
}

// Givens step j of one column: apply the previous rotations to Hessenberg
// column j (h = H + j*ldh), form rotation j, update g and the residual estimate.
__device__ void givens_col(cx<double>* h, double* c_, cx<double>* s_, cx<double>* g_, int j, double* resid) {
  for (int i = 0; i < j; ++i) {
    cx<double> a = h[i], b = h[i + 1];
    h[i] = c_[i] * a + s_[i] * b;
    h[i + 1] = c_[i] * b - conj(s_[i]) * a;
  }
  cx<double> a = h[j], b = h[j + 1];
  double den = sqrt(norm2(a) + norm2(b));
  double c;
  cx<double> s;
  if (den == 0.0) {
    c = 1.0;
    s = mk(0.0, 0.0);
  } else if (norm2(a) == 0.0) {
    c = 0.0;
    s = mk(1.0, 0.0);
  } else {
    double aa = sqrt(norm2(a));
    c = aa / den;
    s = (1.0 / (aa * den)) * (a * conj(b));
  }
  c_[j] = c;
  s_[j] = s;
  h[j] = c * a + s * b;
  h[j + 1] = mk(0.0, 0.0);
  cx<double> gj = g_[j];
  g_[j + 1] = -(conj(s) * gj);
  g_[j] = c * gj;
  *resid = sqrt(norm2(g_[j + 1]));
}

// Givens step j of every active column: thread r handles column r.  Scalar
// arrays per column: H (ldh*m, column-major, leading dimension ldh), cs, sn (m),
// g (ldh), resid (1).
__global__ void k_givens_b(cx<double>* H, int ldh, int m, double* cs, cx<double>* sn, cx<double>* g, int j,
                           double* resid, int K, const int* act) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= K || (act && !act[r])) return;
  givens_col(H + (long)r * ldh * m + (long)j * ldh, cs + (long)r * m, sn + (long)r * m, g + (long)r * ldh, j,
             resid + r);
}
void launch_givens_b(cx<double>* H, int ldh, int m, double* cs, cx<double>* sn, cx<double>* g, int j, double* resid,
                     int K, const int* act, hipStream_t st) {
  hipLaunchKernelGGL(k_givens_b, dim3(1), dim3(64), 0, st, H, ldh, m, cs, sn, g, j, resid, K, act);
}

// back substitution of column r's jd[r] x jd[r] system; y_r[i] = 0 for i >= jd[r]
__global__ void k_trisolve_b(const cx<double>* H, int ldh, int m, const cx<double>* g, cx<double>* y,
                             const int* jd, int K) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= K) return;
  const cx<double>* Hr = H + (long)r * ldh * m;
  const cx<double>* gr = g + (long)r * ldh;
  cx<double>* yr = y + (long)r * ldh;
  const int j = jd[r];
  for (int i = m; i >= j; --i) yr[i] = mk(0.0, 0.0);
  for (int i = j - 1; i >= 0; --i) {
    cx<double> s = gr[i];
    for (int k = i + 1; k < j; ++k) s = s - Hr[(long)k * ldh + i] * yr[k];
    cx<double> d = Hr[(long)i * ldh + i];
    double dn = norm2(d);
    yr[i] = dn > 0 ? (1.0 / dn) * (s * conj(d)) : mk(0.0, 0.0);
  }
}
// the same for m <= 32: one workgroup per column, the triangle staged in LDS
// with all loads in flight, then column-oriented substitution (after y_k,
// every row t < k takes s_t -= H[t][k] y_k in parallel)
__global__ void __launch_bounds__(64) k_trisolve_lds_b(const cx<double>* __restrict__ H, int ldh, int m,
                                                       const cx<double>* __restrict__ g, cx<double>* __restrict__ y,
                                                       const int* __restrict__ jd) {
  __shared__ cx<double> Hs[32][33];  // Hs[k][i] = H[i][k] (column k of the triangle)
  __shared__ cx<double> sv[32], yv[32];
  const int r = blockIdx.x, t = threadIdx.x;
  const cx<double>* Hr = H + (long)r * ldh * m;
  const cx<double>* gr = g + (long)r * ldh;
  cx<double>* yr = y + (long)r * ldh;
  const int j = jd[r];
  for (int q = t; q < j * 32; q += 64) {
    const int k = q >> 5, i = q & 31;
    if (i <= k) Hs[k][i] = Hr[(long)k * ldh + i];
  }
  if (t < j) sv[t] = gr[t];
  __syncthreads();
  for (int k = j - 1; k >= 0; --k) {
    if (t == 0) {
      const cx<double> d = Hs[k][k];
      const double dn = norm2(d);
      yv[k] = dn > 0 ? (1.0 / dn) * (sv[k] * conj(d)) : mk(0.0, 0.0);
    }
    __syncthreads();
    if (t < k) sv[t] = sv[t] - Hs[k][t] * yv[k];
    __syncthreads();
  }
  for (int i = t; i <= m; i += 64) yr[i] = i < j ? yv[i] : mk(0.0, 0.0);
}
void launch_trisolve_b(const cx<double>* H, int ldh, int m, const cx<double>* g, cx<double>* y, const int* jd, int K,
                       hipStream_t st) {
  if (m <= 32)
    hipLaunchKernelGGL(k_trisolve_lds_b, dim3(K), dim3(64), 0, st, H, ldh, m, g, y, jd);
  else
    hipLaunchKernelGGL(k_trisolve_b, dim3(1), dim3(64), 0, st, H, ldh, m, g, y, jd, K);
}

// g_r = 0 except g_r[0] = s_r  (start of a cycle)
__global__ void k_init_g_b(cx<double>* g, int ldh, const cx<double>* s, long scs, int K, const int* act) {
  const int r = blockIdx.x;
  if (r >= K || (act && !act[r])) return;
  for (int i = threadIdx.x; i < ldh; i += blockDim.x) g[(long)r * ldh + i] = i == 0 ? s[r * scs] : mk(0.0, 0.0);
}
void launch_init_g_b(cx<double>* g, int ldh, const cx<double>* s, long scs, int K, const int* act, hipStream_t st) {
  hipLaunchKernelGGL(k_init_g_b, dim3(K), dim3(64), 0, st, g, ldh, s, scs, K, act);
}


// ---------------------------------------------------------------------------
// Classical Gram-Schmidt, norm and Givens step of K lock-step Arnoldi
// processes: two Gram-Schmidt passes (four launches) or one (three launches),
// as cgs_two_pass decides from the vector type and the cycle length.
// Grid (nwg, K), column r = blockIdx.y; inactive
// columns return at once (the last launch zeroes their next basis vector).
// Every workgroup stores per-workgroup partial sums; the next launch begins by
// reducing them in every workgroup (fixed order, so results are deterministic
// and no workgroup waits for another).  Partials alternate between two
// buffers, pa and pb, each [K][ldh][nwg] complex.  Basis V_0..V_{k-1} at
// stride ldv, k <= KM <= 32.
namespace {
// smallest power of two >= km (the transposing wavefront sum needs one)
constexpr int cgs_pow2(int km) { return km <= 2 ? 2 : km <= 4 ? 4 : km <= 8 ? 8 : km <= 16 ? 16 : 32; }
// this workgroup's sums of acc[0..nval) -> partd[(v/2) * nwg + wg] (as doubles;
// NW wavefronts, the wavefront totals added in FP64 in wavefront order)
template <int KM, int NW, class A>
__device__ __forceinline__ void store_partials(A (&acc)[2 * KM], int nval, double* partd) {
  __shared__ double red[NW][2 * KM];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const A v = wave_transpose_sum<2 * KM>(acc, lane);
  if (lane < 2 * KM) red[wv][lane] = (double)v;
  __syncthreads();
  if (t < nval) {
    double sv = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) sv += red[q][t];
    partd[2 * ((long)(t >> 1) * gridDim.x + blockIdx.x) + (t & 1)] = sv;
  }
}

// totals of values v < nval over the nwg partials of the previous launch ->
// out[v], out[v] = 0 for nval <= v < nout (<= 64).  tpv lanes of one wavefront
// per value (the largest power of two with tpv * nval <= blockDim, at most 64)
// sum strided partials with four independent sums, then combine by xor
// shuffles: a fixed order.  Ends with a barrier.
__device__ __forceinline__ void reduce_partials(const double* partd, int nval, int nout, int nwg, double* out) {
  int tpv = 64;
  while (tpv > 1 && tpv * nval > (int)blockDim.x) tpv >>= 1;
  const int t = threadIdx.x, v = t / tpv, q = t - v * tpv;
  double x = 0.0;
  if (v < nval) {
    const double* p = partd + 2L * (v >> 1) * nwg + (v & 1);
    double x1 = 0.0, x2 = 0.0, x3 = 0.0;
    int w = q;
    for (; w + 3 * tpv < nwg; w += 4 * tpv) {
      x += p[2L * w];
      x1 += p[2L * (w + tpv)];
      x2 += p[2L * (w + 2 * tpv)];
      x3 += p[2L * (w + 3 * tpv)];
    }
    for (; w < nwg; w += tpv) x += p[2L * w];
    x = (x + x1) + (x2 + x3);
  }
  for (int o = 1; o < tpv; o <<= 1) x += __shfl_xor(x, o, 64);
  if (v < nval && q == 0) out[v] = x;
  for (int z = nval + t; z < nout; z += blockDim.x) out[z] = 0.0;
  __syncthreads();
}
}  // namespace

// Per-thread sums and the updates w -= sum_i c_i V_i are in R (FP32 for FP32
// vectors; the coefficients are rounded to R), every sum across threads in FP64
// from the wavefront totals on.
// pa_r: partials of V_{r,i}^H w_r  (i < k)
template <class R, int KM, int BS>
__global__ void __launch_bounds__(BS) k_cgs_dot(const cx<R>* __restrict__ V, long ldv, long csV, int k,
                                                const cx<R>* __restrict__ w, long csw, long N, double* pa,
                                                long pcs, const int* act) {
  const int r = blockIdx.y;
  if (act && !act[r]) return;
  V += r * csV;
  w += r * csw;
  // sums for KM vectors, padded to a power of two for the wavefront reduction
  constexpr int KP = cgs_pow2(KM);
  R acc[2 * KP];
#pragma unroll
  for (int q = 0; q < 2 * KP; ++q) acc[q] = R(0);
  const long stride = (long)gridDim.x * BS;
  for (long e = (long)blockIdx.x * BS + threadIdx.x; e < N; e += stride) {
    const cx<R> x = w[e];
#pragma unroll
    for (int i = 0; i < KM; ++i) {  // every load issued (index clamped); sums past k unused
      const cx<R> v = V[(long)min(i, k - 1) * ldv + e];
      acc[2 * i] += v.re * x.re + v.im * x.im;
      acc[2 * i + 1] += v.re * x.im - v.im * x.re;
    }
  }
  store_partials<KP, BS / 64>(acc, 2 * k, pa + 2 * r * pcs);
}

// h_r = sum of pa_r (workgroup 0 stores it in hcol_r);  w_r -= sum_i h_r[i] V_{r,i};
// pb_r: partials of V_{r,i}^H w_r
template <class R, int KM, int BS>
__global__ void __launch_bounds__(BS) k_cgs_axpy_dot(const cx<R>* __restrict__ V, long ldv, long csV, int k,
                                                     cx<R>* w, long csw, long N, const double* pa, double* pb,
                                                     long pcs, cx<double>* hcol, long hcs, const int* act) {
  const int r = blockIdx.y;
  if (act && !act[r]) return;
  V += r * csV;
  w += r * csw;
  __shared__ double cf[2 * KM];
  __shared__ cx<R> cfr[KM];
  reduce_partials(pa + 2 * r * pcs, 2 * k, 2 * KM, gridDim.x, cf);
  if (blockIdx.x == 0 && threadIdx.x < 2 * k) reinterpret_cast<double*>(hcol + r * hcs)[threadIdx.x] = cf[threadIdx.x];
  if (threadIdx.x < KM) cfr[threadIdx.x] = mk<R>((R)cf[2 * threadIdx.x], (R)cf[2 * threadIdx.x + 1]);
  __syncthreads();
  // sums for KM vectors, padded to a power of two for the wavefront reduction
  constexpr int KP = cgs_pow2(KM);
  R acc[2 * KP];
#pragma unroll
  for (int q = 0; q < 2 * KP; ++q) acc[q] = R(0);
  const long stride = (long)gridDim.x * BS;
  for (long e = (long)blockIdx.x * BS + threadIdx.x; e < N; e += stride) {
    const cx<R> x0 = w[e];
    cx<R> s = mk<R>(0, 0);
#pragma unroll
    for (int i = 0; i < KM; ++i) {  // coefficients past k are zero
      const cx<R> v = V[(long)min(i, k - 1) * ldv + e];
      cmac(s, cfr[i], v);
    }
    const cx<R> x = mk<R>(x0.re - s.re, x0.im - s.im);
    w[e] = x;
    // reload the basis entries (cache hits) rather than hold KM of them in registers
    asm volatile("" ::: "memory");
#pragma unroll
    for (int i = 0; i < KM; ++i) {
      const cx<R> v = V[(long)min(i, k - 1) * ldv + e];
      acc[2 * i] += v.re * x.re + v.im * x.im;
      acc[2 * i + 1] += v.re * x.im - v.im * x.re;
    }
  }
  store_partials<KP, BS / 64>(acc, 2 * k, pb + 2 * r * pcs);
}

// c_r = sum of pb_r (workgroup 0: hcol_r += c_r, or hcol_r = c_r when this is
// the only pass);  w_r -= sum_i c_r[i] V_{r,i};  pa_r: partials of ||w_r||^2
template <class R, int KM, int BS, bool FIRST = false>
__global__ void __launch_bounds__(BS) k_cgs_axpy_norm(const cx<R>* __restrict__ V, long ldv, long csV, int k,
                                                      cx<R>* w, long csw, long N, const double* pb, double* pa,
                                                      long pcs, cx<double>* hcol, long hcs, const int* act) {
  const int r = blockIdx.y;
  if (act && !act[r]) return;
  V += r * csV;
  w += r * csw;
  __shared__ double cf[2 * KM];
  __shared__ cx<R> cfr[KM];
  reduce_partials(pb + 2 * r * pcs, 2 * k, 2 * KM, gridDim.x, cf);
  if (blockIdx.x == 0 && threadIdx.x < 2 * k) {
    double& hv = reinterpret_cast<double*>(hcol + r * hcs)[threadIdx.x];
    hv = FIRST ? cf[threadIdx.x] : hv + cf[threadIdx.x];
  }
  if (threadIdx.x < KM) cfr[threadIdx.x] = mk<R>((R)cf[2 * threadIdx.x], (R)cf[2 * threadIdx.x + 1]);
  __syncthreads();
  R acc[2] = {R(0), R(0)};
  const long stride = (long)gridDim.x * BS;
  for (long e = (long)blockIdx.x * BS + threadIdx.x; e < N; e += stride) {
    const cx<R> x0 = w[e];
    cx<R> s = mk<R>(0, 0);
#pragma unroll
    for (int i = 0; i < KM; ++i) {  // coefficients past k are zero
      const cx<R> v = V[(long)min(i, k - 1) * ldv + e];
      cmac(s, cfr[i], v);
    }
    const cx<R> x = mk<R>(x0.re - s.re, x0.im - s.im);
    w[e] = x;
    acc[0] += x.re * x.re + x.im * x.im;
  }
  store_partials<1, BS / 64>(acc, 1, pa + 2 * r * pcs);
}

// ||w_r|| from pa_r; workgroup 0 stores it as H_r[j+1][j] and takes Givens
// step j (column j, rotations and g staged in LDS); every workgroup scales its
// part of w_r by 1/||w_r|| (w_r zeroed for an inactive column).  With
// resid_host (pinned host memory) the residual estimate is also stored there.
template <class R, int BS>
__global__ void __launch_bounds__(BS) k_cgs_scale_givens(cx<R>* w, long csw, long N, const double* pa, long pcs,
                                                          cx<double>* H, int ldh, int m, double* cs, cx<double>* sn,
                                                          cx<double>* g, int j, double* resid, double* resid_host,
                                                          const int* act) {
  const int r = blockIdx.y;
  const long stride = (long)gridDim.x * BS;
  w += r * csw;
  if (act && !act[r]) {
    for (long e = (long)blockIdx.x * BS + threadIdx.x; e < N; e += stride) w[e] = mk<R>(0, 0);
    return;
  }
  __shared__ double nn[1];
  reduce_partials(pa + 2 * r * pcs, 1, 1, gridDim.x, nn);
  const double nv = sqrt(nn[0] > 0 ? nn[0] : 0.0);
  if (blockIdx.x == 0) {
    __shared__ cx<double> hl[64], sl[64], gl[64];
    __shared__ double cl[64];
    cx<double>* h = H + (long)r * ldh * m + (long)j * ldh;
    const int t = threadIdx.x;
    if (t <= j) {
      hl[t] = h[t];
      if (t < j) {
        cl[t] = cs[(long)r * m + t];
        sl[t] = sn[(long)r * m + t];
      }
    }
    if (t == 0) {
      hl[j + 1] = mk(nv, 0.0);
      gl[j] = g[(long)r * ldh + j];
    }
    __syncthreads();
    if (t == 0) {
      givens_col(hl, cl, sl, gl, j, resid + r);
      if (resid_host) resid_host[r] = resid[r];
      // rotation j and the new g entries are the only state kept besides H
      cs[(long)r * m + j] = cl[j];
      sn[(long)r * m + j] = sl[j];
      g[(long)r * ldh + j] = gl[j];
      g[(long)r * ldh + j + 1] = gl[j + 1];
    }
    __syncthreads();
    if (t <= j + 1) h[t] = hl[t];
  }
  const double f = nv > 0 ? 1.0 / nv : 0.0;
  for (long e = (long)blockIdx.x * BS + threadIdx.x; e < N; e += stride) {
    const cx<R> x = w[e];
    w[e] = mk<R>((R)(f * x.re), (R)(f * x.im));
  }
}

template <class R, int BS>
static void cgs_step_bs(const cx<R>* V, long ldv, long csV, int k, cx<R>* w, long csw, long N, double* a, double* b,
                        long pcs, int nwg, cx<double>* hcol, long hcs, cx<double>* H, int ldh, int m, double* cs,
                        cx<double>* sn, cx<double>* g, int j, double* resid, double* resid_host, int K, const int* act,
                        hipStream_t st) {
  const dim3 grid(nwg, K), blk(BS);
  const bool two_pass = cgs_two_pass<R>(m);
  // the axpy kernels of 16 or more vectors hold twice the registers: half the
  // threads per workgroup (same workgroup count, so the partials match)
#define CGS_LAUNCH(KM)                                                                                                 \
  {                                                                                                                    \
    constexpr int BA = (BS == 1024 && KM >= 16) ? 512 : BS;                                                            \
    hipLaunchKernelGGL((k_cgs_dot<R, KM, BS>), grid, blk, 0, st, V, ldv, csV, k, (const cx<R>*)w, csw, N, a, pcs,     \
                       act);                                                                                           \
    if (two_pass) {                                                                                                    \
      hipLaunchKernelGGL((k_cgs_axpy_dot<R, KM, BA>), grid, dim3(BA), 0, st, V, ldv, csV, k, w, csw, N,               \
                         (const double*)a, b, pcs, hcol, hcs, act);                                                    \
      hipLaunchKernelGGL((k_cgs_axpy_norm<R, KM, BA>), grid, dim3(BA), 0, st, V, ldv, csV, k, w, csw, N,              \
                         (const double*)b, a, pcs, hcol, hcs, act);                                                    \
    } else {                                                                                                           \
      hipLaunchKernelGGL((k_cgs_axpy_norm<R, KM, BA, true>), grid, dim3(BA), 0, st, V, ldv, csV, k, w, csw, N,        \
                         (const double*)a, b, pcs, hcol, hcs, act);                                                    \
    }                                                                                                                  \
  }
  // buckets of basis sizes: at most three clamped loads past k per element
  if (k <= 2) {
    CGS_LAUNCH(2)
  } else if (k <= 4) {
    CGS_LAUNCH(4)
  } else if (k <= 6) {
    CGS_LAUNCH(6)
  } else if (k <= 8) {
    CGS_LAUNCH(8)
  } else if (k <= 12) {
    CGS_LAUNCH(12)
  } else if (k <= 16) {
    CGS_LAUNCH(16)
  } else if (k <= 20) {
    CGS_LAUNCH(20)
  } else if (k <= 24) {
    CGS_LAUNCH(24)
  } else if (k <= 28) {
    CGS_LAUNCH(28)
  } else {
    CGS_LAUNCH(32)
  }
#undef CGS_LAUNCH
  hipLaunchKernelGGL((k_cgs_scale_givens<R, BS>), grid, blk, 0, st, w, csw, N, (const double*)(two_pass ? a : b), pcs,
                     H, ldh, m, cs, sn, g, j, resid, resid_host, act);
}

// FP32 vectors: 512-thread workgroups with FP32 per-thread sums (at most 128
// registers; with up to 256 workgroups a coarsest column of 82,944 entries
// spreads over all 256 CUs); FP64 vectors: 256-thread workgroups
template <class R>
int cgs_block_size() {
  return sizeof(R) == 4 ? 512 : 256;
}
template <class R>
void launch_cgs_step(const cx<R>* V, long ldv, long csV, int k, cx<R>* w, long csw, long N, cx<double>* pa,
                     cx<double>* pb, long pcs, int nwg, cx<double>* hcol, long hcs, cx<double>* H, int ldh, int m,
                     double* cs, cx<double>* sn, cx<double>* g, int j, double* resid, double* resid_host, int K,
                     const int* act, hipStream_t st) {
  double* a = reinterpret_cast<double*>(pa);
  double* b = reinterpret_cast<double*>(pb);
  if constexpr (sizeof(R) == 4)
    cgs_step_bs<R, 512>(V, ldv, csV, k, w, csw, N, a, b, pcs, nwg, hcol, hcs, H, ldh, m, cs, sn, g, j, resid, resid_host, K, act, st);
  else
    cgs_step_bs<R, 256>(V, ldv, csV, k, w, csw, N, a, b, pcs, nwg, hcol, hcs, H, ldh, m, cs, sn, g, j, resid, resid_host, K, act, st);
}
#define INST_CGS(R)                                                                                             \
  template int cgs_block_size<R>();                                                                               \
  template void launch_cgs_step<R>(const cx<R>*, long, long, int, cx<R>*, long, long, cx<double>*, cx<double>*,   \
                                   long, int, cx<double>*, long, cx<double>*, int, int, double*, cx<double>*,     \
                                   cx<double>*, int, double*, double*, int, const int*, hipStream_t);
INST_CGS(double)
INST_CGS(float)

#define INST_BB(R)                                                                                                  \
  template void launch_multidot_b<R>(const cx<R>*, long, long, int, const cx<R>*, long, long, cx<double>*, long,   \
                                     int, int, const int*, hipStream_t);                                            \
  template void launch_multi_axpy_b<R>(const cx<R>*, long, long, int, const int*, const cx<double>*, long, double,  \
                                       cx<R>*, long, long, int, const int*, hipStream_t);                           \
  template void launch_scale_by_inv_b<R>(const cx<R>*, long, const cx<double>*, long, cx<R>*, long, long, int,      \
                                         const int*, int, hipStream_t);                                             \
  template void launch_sub_b<R>(long, const cx<R>*, long, const cx<R>*, long, cx<R>*, long, int, hipStream_t);     \
  template void launch_zero_b<R>(long, cx<R>*, long, int, hipStream_t);
INST_BB(double)
INST_BB(float)
template void launch_copy_cvt_b<double, float>(const cx<double>*, long, cx<float>*, long, long, int, hipStream_t);
template void launch_copy_cvt_b<float, double>(const cx<float>*, long, cx<double>*, long, long, int, hipStream_t);
template void launch_copy_cvt_b<double, double>(const cx<double>*, long, cx<double>*, long, long, int, hipStream_t);
template void launch_copy_cvt_b<float, float>(const cx<float>*, long, cx<float>*, long, long, int, hipStream_t);

}  // namespace ddamg
