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

}  // namespace ddamg
