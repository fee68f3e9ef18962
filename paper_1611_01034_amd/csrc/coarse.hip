// Coarse-level kernels: the coarse operator stencil
//   (D_c y)(c) = S(c) y(c) + i tw Gamma5 y(c)
//               + sum_mu [ F_mu(c) y(c+mu) + Gamma5 F_mu(c-mu)^dag Gamma5 y(c-mu) ]
// (paper Sec. 1: D_c = P^dag D_W P, D_c^dag = Gamma5,c D_c Gamma5,c and
// D_c(mu) = D_c + i mu Gamma5,c), its SAP smoother, restriction / prolongation
// to the next level, block orthonormalisation, Galerkin assembly of the next
// coarse operator, and the odd-even reduced system of the coarsest level
// (Sec. 3: odd-even on the coarsest level).
//
// Storage: vectors [site][n] (n = 2 Nv of the level above, Gamma5,c =
// diag(-1 x n/2, +1 x n/2)); operator [site][5][n][n], block 0 = S without the
// twist, block 1+mu = F_mu, each block column-major (element (k,l) at l*n+k).
// Sites are numbered even parity first, so the even half of a vector is a
// prefix.  One wavefront handles one site; lane k computes row k (n <= 64).
#include "kernels.hpp"

namespace ddamg {

__device__ __forceinline__ double g5(int k, int n) { return k < (n >> 1) ? -1.0 : 1.0; }

template <class R, class S>
__device__ __forceinline__ cx<R> Dld(const typename store_traits<S>::elem* D, long idx) {
  return ld<R, S>(D, idx);
}

// stage y at the site (slot 0) and its 8 neighbours (slots 1..8) in LDS
template <class R>
__device__ __forceinline__ void stage9(cx<R> (*ys)[64], const CGeom& cg, int site, bool valid, const cx<R>* in,
                                       int lane) {
  if (valid && lane < cg.n) {
    ys[0][lane] = in[(long)site * cg.n + lane];
#pragma unroll
    for (int j = 0; j < 8; ++j) ys[1 + j][lane] = in[(long)cg.nbr[site * 8 + j] * cg.n + lane];
  }
}

template <class R, class S>
__device__ __forceinline__ cx<R> self_row(const CGeom& cg, const typename store_traits<S>::elem* D, int site, int k,
                                          R tw, const cx<R>* y) {
  const int n = cg.n;
  long base = (long)site * 5 * n * n;
  cx<R> acc = mk<R>(0, 0);
  for (int l = 0; l < n; ++l) cmac(acc, Dld<R, S>(D, base + (long)l * n + k), y[l]);
  acc += (R)(tw * g5(k, n)) * times_i(y[k]);
  return acc;
}

template <class R, class S>
__device__ __forceinline__ cx<R> hop_row(const CGeom& cg, const typename store_traits<S>::elem* D, int site, int k,
                                         cx<R> (*ys)[64]) {
  const int n = cg.n;
  const long nn = (long)n * n;
  cx<R> acc = mk<R>(0, 0);
#pragma unroll 1
  for (int mu = 0; mu < 4; ++mu) {
    long bf = ((long)site * 5 + 1 + mu) * nn;
    const cx<R>* yf = ys[1 + mu];
    for (int l = 0; l < n; ++l) cmac(acc, Dld<R, S>(D, bf + (long)l * n + k), yf[l]);
    int cb = cg.nbr[site * 8 + 4 + mu];
    long bb = ((long)cb * 5 + 1 + mu) * nn + (long)k * n;
    const cx<R>* yb = ys[5 + mu];
    cx<R> t = mk<R>(0, 0);
    const int h = n >> 1;
    for (int l = 0; l < h; ++l) cjmac(t, Dld<R, S>(D, bb + l), yb[l]);
    cx<R> t2 = mk<R>(0, 0);
    for (int l = h; l < n; ++l) cjmac(t2, Dld<R, S>(D, bb + l), yb[l]);
    // g_k * (g_l sums): lower half g_l = -1, upper half +1
    cx<R> tb = t2 - t;
    if (k < h) acc -= tb;
    else acc += tb;
  }
  return acc;
}

// out = D y   (or out = b - D y when b != nullptr)
template <class R, class S>
__global__ void __launch_bounds__(256) k_coarse_apply(CGeom cg, const typename store_traits<S>::elem* __restrict__ D,
                                                      R tw, const cx<R>* __restrict__ in, const cx<R>* __restrict__ b,
                                                      cx<R>* __restrict__ out) {
  __shared__ cx<R> ys[4][9][64];
  int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int site = blockIdx.x * 4 + wv;
  bool valid = site < cg.nsites;
  stage9(ys[wv], cg, site, valid, in, lane);
  __syncthreads();
  if (valid && lane < cg.n) {
    cx<R> acc = self_row<R, S>(cg, D, site, lane, tw, ys[wv][0]) + hop_row<R, S>(cg, D, site, lane, ys[wv]);
    long o = (long)site * cg.n + lane;
    out[o] = b ? b[o] - acc : acc;
  }
}

template <class R, class S>
void launch_coarse_apply(const CGeom& cg, const void* D, double tw, const cx<R>* in, cx<R>* out, hipStream_t st) {
  hipLaunchKernelGGL((k_coarse_apply<R, S>), dim3((cg.nsites + 3) / 4), dim3(256), 0, st, cg,
                     (const typename store_traits<S>::elem*)D, (R)tw, in, (const cx<R>*)nullptr, out);
}
template <class R, class S>
void launch_coarse_residual(const CGeom& cg, const void* D, double tw, const cx<R>* b, const cx<R>* x, cx<R>* r,
                            hipStream_t st) {
  hipLaunchKernelGGL((k_coarse_apply<R, S>), dim3((cg.nsites + 3) / 4), dim3(256), 0, st, cg,
                     (const typename store_traits<S>::elem*)D, (R)tw, x, b, r);
}

// ---------------------------------------------------------------------------
// coarse SAP: one workgroup per block of the colour, one wavefront per block
// site; n_mr MR steps on the Dirichlet block operator D_B.
template <class R, class S>
__global__ void __launch_bounds__(1024) k_coarse_sap(CGeom cg, const typename store_traits<S>::elem* __restrict__ D,
                                                     R tw, int bsz, const int* __restrict__ blk_sites,
                                                     const int* __restrict__ blk_nbr, const cx<R>* __restrict__ r,
                                                     cx<R>* __restrict__ x, int n_mr, int K, long ld) {
  extern __shared__ char smem_raw[];
  cx<R>* rho = reinterpret_cast<cx<R>*>(smem_raw);  // [bsz][64]
  __shared__ double red[3][16];
  const int n = cg.n;
  const long nn = (long)n * n;
  // K fields interleaved: consecutive workgroups take one block for different fields
  const int blk = blockIdx.x / K, rr = blockIdx.x - blk * K;
  r += (long)rr * ld;
  x += (long)rr * ld;
  int j = threadIdx.x >> 6, k = threadIdx.x & 63;
  int site = blk_sites[blk * bsz + j];
  const int* lnb = blk_nbr + ((long)blk * bsz + j) * 8;
  bool act = k < n;
  rho[j * 64 + k] = act ? r[(long)site * n + k] : mk<R>(0, 0);
  cx<R> eps = mk<R>(0, 0);
  const int h = n >> 1;
  for (int it = 0; it < n_mr; ++it) {
    __syncthreads();
    cx<R> q = mk<R>(0, 0);
    if (act) {
      q = self_row<R, S>(cg, D, site, k, tw, rho + j * 64);
      for (int mu = 0; mu < 4; ++mu) {
        int jf = lnb[mu];
        if (jf >= 0) {
          long bf = ((long)site * 5 + 1 + mu) * nn;
          const cx<R>* yf = rho + jf * 64;
          for (int l = 0; l < n; ++l) cmac(q, Dld<R, S>(D, bf + (long)l * n + k), yf[l]);
        }
        int jb = lnb[4 + mu];
        if (jb >= 0) {
          int cb = blk_sites[blk * bsz + jb];
          long bb = ((long)cb * 5 + 1 + mu) * nn + (long)k * n;
          const cx<R>* yb = rho + jb * 64;
          cx<R> t = mk<R>(0, 0), t2 = mk<R>(0, 0);
          for (int l = 0; l < h; ++l) cjmac(t, Dld<R, S>(D, bb + l), yb[l]);
          for (int l = h; l < n; ++l) cjmac(t2, Dld<R, S>(D, bb + l), yb[l]);
          cx<R> tb = t2 - t;
          if (k < h) q -= tb;
          else q += tb;
        }
      }
    }
    cx<R> rk = rho[j * 64 + k];
    double qr_re = (double)q.re * rk.re + (double)q.im * rk.im;
    double qr_im = (double)q.re * rk.im - (double)q.im * rk.re;
    double qq = (double)q.re * q.re + (double)q.im * q.im;
    qr_re = wave_sum_n(qr_re, 64);
    qr_im = wave_sum_n(qr_im, 64);
    qq = wave_sum_n(qq, 64);
    if (k == 0) {
      red[0][j] = qr_re;
      red[1][j] = qr_im;
      red[2][j] = qq;
    }
    __syncthreads();
    double sr = 0, si = 0, sq = 0;
    for (int v = 0; v < bsz; ++v) {
      sr += red[0][v];
      si += red[1][v];
      sq += red[2][v];
    }
    cx<R> alpha = mk<R>(0, 0);
    if (sq > 0) alpha = mk<R>((R)(sr / sq), (R)(si / sq));
    eps += alpha * rk;
    rho[j * 64 + k] = rk - alpha * q;
  }
  if (act) {
    long o = (long)site * n + k;
    x[o] = x[o] + eps;
  }
}

template <class R, class S>
void launch_coarse_sap(const CGeom& cg, const void* D, double tw, int nblk_colour, int bsz, const int* blk_sites,
                       const int* blk_nbr, const cx<R>* r, cx<R>* x, int n_mr, hipStream_t st) {
  launch_coarse_sap_multi<R, S>(cg, D, tw, nblk_colour, bsz, blk_sites, blk_nbr, r, x, n_mr, 1, 0, st);
}
template <class R, class S>
void launch_coarse_sap_multi(const CGeom& cg, const void* D, double tw, int nblk_colour, int bsz, const int* blk_sites,
                             const int* blk_nbr, const cx<R>* r, cx<R>* x, int n_mr, int K, long ld, hipStream_t st) {
  size_t sm = (size_t)bsz * 64 * sizeof(cx<R>);
  hipLaunchKernelGGL((k_coarse_sap<R, S>), dim3(nblk_colour * K), dim3(64 * bsz), sm, st, cg,
                     (const typename store_traits<S>::elem*)D, (R)tw, bsz, blk_sites, blk_nbr, r, x, n_mr, K, ld);
}

// ---------------------------------------------------------------------------
// restriction to the next level: r_c[A][s*Nv+i] = sum_{j in A, k in half s}
// conj(Q_i[site_j][k]) r[site_j][k].  One workgroup (256) per aggregate;
// wavefront w takes the vectors 8w..8w+7 (then +32, ...) over all entries of
// the aggregate (lanes on consecutive entries) and sums its 32 values
// (8 vectors x 2 halves x re/im) with one transposing wavefront sum: no LDS,
// no barriers, the four wavefronts independent.
template <class R>
__global__ void __launch_bounds__(256) k_restrict_coarse(int n, int Nv, int asz, const int* __restrict__ agg_sites,
                                                         const cx<R>* __restrict__ Q, long qstride,
                                                         const cx<R>* __restrict__ r, cx<R>* __restrict__ rc) {
  const int A = blockIdx.x, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int tot = asz * n, hn = n >> 1;
  for (int i0 = 8 * w; i0 < Nv; i0 += 32) {
    double acc[32];  // [4 ii + 2 h + p]
#pragma unroll
    for (int q = 0; q < 32; ++q) acc[q] = 0.0;
#pragma unroll 2
    for (int e = lane; e < tot; e += 64) {
      const int j = e / n, k = e - j * n;
      const long idx = (long)agg_sites[A * asz + j] * n + k;
      const cx<R> rv = r[idx];
      const bool up = k >= hn;
#pragma unroll
      for (int ii = 0; ii < 8; ++ii) {
        const int iv = i0 + ii < Nv ? i0 + ii : Nv - 1;  // clamped: every load in flight
        const cx<R> qv = Q[(long)iv * qstride + idx];
        const double re = (double)qv.re * rv.re + (double)qv.im * rv.im;
        const double im = (double)qv.re * rv.im - (double)qv.im * rv.re;
        acc[4 * ii + 0] += up ? 0.0 : re;
        acc[4 * ii + 1] += up ? 0.0 : im;
        acc[4 * ii + 2] += up ? re : 0.0;
        acc[4 * ii + 3] += up ? im : 0.0;
      }
    }
    const double v = wave_transpose_sum<32>(acc, lane);  // lane l: total of value l % 32
    if (lane < 32) {
      const int ii = lane >> 2, hh = (lane >> 1) & 1, p = lane & 1;
      if (i0 + ii < Nv) reinterpret_cast<R*>(rc + (long)A * 2 * Nv + hh * Nv + i0 + ii)[p] = (R)v;
    }
  }
}
template <class R>
void launch_restrict_coarse(int n, int Nv, int nagg, int asz, const int* agg_sites, const cx<R>* Q, long qstride,
                            const cx<R>* r, cx<R>* rc, hipStream_t st) {
  hipLaunchKernelGGL(k_restrict_coarse<R>, dim3(nagg), dim3(256), 0, st, n, Nv, asz, agg_sites, Q, qstride, r, rc);
}

// K columns (stride rld in, cld out): one workgroup per (aggregate, column),
// the K columns of an aggregate in consecutive workgroups of one XCD, so its
// part of Q comes from HBM once and from L2 for the other columns
template <class R>
__global__ void __launch_bounds__(256) k_restrict_coarse_m(int n, int Nv, int asz, const int* __restrict__ agg_sites,
                                                           const cx<R>* __restrict__ Q, long qstride,
                                                           const cx<R>* __restrict__ r, long rld,
                                                           cx<R>* __restrict__ rc, long cld, int K) {
  const int wq = xcd_remap(blockIdx.x, gridDim.x), A = wq / K, col = wq - A * K;
  r += (long)col * rld;
  rc += (long)col * cld;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int tot = asz * n, hn = n >> 1;
  for (int i0 = 8 * w; i0 < Nv; i0 += 32) {
    double acc[32];  // [4 ii + 2 h + p]
#pragma unroll
    for (int q = 0; q < 32; ++q) acc[q] = 0.0;
#pragma unroll 2
    for (int e = lane; e < tot; e += 64) {
      const int j = e / n, k = e - j * n;
      const long idx = (long)agg_sites[A * asz + j] * n + k;
      const cx<R> rv = r[idx];
      const bool up = k >= hn;
#pragma unroll
      for (int ii = 0; ii < 8; ++ii) {
        const int iv = i0 + ii < Nv ? i0 + ii : Nv - 1;  // clamped: every load in flight
        const cx<R> qv = Q[(long)iv * qstride + idx];
        const double re = (double)qv.re * rv.re + (double)qv.im * rv.im;
        const double im = (double)qv.re * rv.im - (double)qv.im * rv.re;
        acc[4 * ii + 0] += up ? 0.0 : re;
        acc[4 * ii + 1] += up ? 0.0 : im;
        acc[4 * ii + 2] += up ? re : 0.0;
        acc[4 * ii + 3] += up ? im : 0.0;
      }
    }
    const double v = wave_transpose_sum<32>(acc, lane);  // lane l: total of value l % 32
    if (lane < 32) {
      const int ii = lane >> 2, hh = (lane >> 1) & 1, p = lane & 1;
      if (i0 + ii < Nv) reinterpret_cast<R*>(rc + (long)A * 2 * Nv + hh * Nv + i0 + ii)[p] = (R)v;
    }
  }
}
template <class R>
void launch_restrict_coarse_m(int n, int Nv, int nagg, int asz, const int* agg_sites, const cx<R>* Q, long qstride,
                              const cx<R>* r, long rld, cx<R>* rc, long cld, int K, hipStream_t st) {
  hipLaunchKernelGGL(k_restrict_coarse_m<R>, dim3(nagg * K), dim3(256), 0, st, n, Nv, asz, agg_sites, Q, qstride, r,
                     rld, rc, cld, K);
}

// K columns: one thread per entry for all columns, in groups of KC whose
// accumulators stay in registers (Q read once per group)
template <class R, int KC>
__global__ void k_prolong_coarse_m(int n, int Nv, int nsites, const int* __restrict__ site_agg,
                                   const cx<R>* __restrict__ Q, long qstride, const cx<R>* __restrict__ ec, long cld,
                                   cx<R>* __restrict__ x, long xld, int K, int accumulate) {
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)nsites * n) return;
  const int site = (int)(gid / n), k = (int)(gid - (long)site * n);
  const int h = k >= (n >> 1) ? 1 : 0;
  const cx<R>* e = ec + (long)site_agg[site] * 2 * Nv + h * Nv;
  for (int k0 = 0; k0 < K; k0 += KC) {
    cx<R> acc[KC];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk)
      acc[kk] = accumulate && k0 + kk < K ? x[(long)(k0 + kk) * xld + gid] : mk<R>(0, 0);
    for (int i = 0; i < Nv; ++i) {
      const cx<R> q = Q[(long)i * qstride + gid];
#pragma unroll
      for (int kk = 0; kk < KC; ++kk)
        if (k0 + kk < K) cmac(acc[kk], q, e[(long)(k0 + kk) * cld + i]);
    }
#pragma unroll
    for (int kk = 0; kk < KC; ++kk)
      if (k0 + kk < K) x[(long)(k0 + kk) * xld + gid] = acc[kk];
  }
}
template <class R>
void launch_prolong_coarse_m(int n, int Nv, int nsites, const int* site_agg, const cx<R>* Q, long qstride,
                             const cx<R>* ec, long cld, cx<R>* x, long xld, int K, int accumulate, hipStream_t st) {
  const long tot = (long)nsites * n;
  const dim3 grid((unsigned)((tot + 255) / 256)), blk(256);
  if (K <= 4)
    hipLaunchKernelGGL((k_prolong_coarse_m<R, 4>), grid, blk, 0, st, n, Nv, nsites, site_agg, Q, qstride, ec, cld, x,
                       xld, K, accumulate);
  else
    hipLaunchKernelGGL((k_prolong_coarse_m<R, 8>), grid, blk, 0, st, n, Nv, nsites, site_agg, Q, qstride, ec, cld, x,
                       xld, K, accumulate);
}

template <class R>
__global__ void k_prolong_coarse(int n, int Nv, int nsites, const int* __restrict__ site_agg,
                                 const cx<R>* __restrict__ Q, long qstride, const cx<R>* __restrict__ ec,
                                 cx<R>* __restrict__ x, int accumulate) {
  long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)nsites * n) return;
  int site = (int)(gid / n), k = (int)(gid - (long)site * n);
  int h = k >= (n >> 1) ? 1 : 0;
  const cx<R>* e = ec + (long)site_agg[site] * 2 * Nv + h * Nv;
  cx<R> acc = accumulate ? x[gid] : mk<R>(0, 0);
  for (int i = 0; i < Nv; ++i) cmac(acc, Q[(long)i * qstride + gid], e[i]);
  x[gid] = acc;
}
template <class R>
void launch_prolong_coarse(int n, int Nv, int nsites, const int* site_agg, const cx<R>* Q, long qstride,
                           const cx<R>* ec, cx<R>* x, int accumulate, hipStream_t st) {
  long tot = (long)nsites * n;
  hipLaunchKernelGGL(k_prolong_coarse<R>, dim3((tot + 255) / 256), dim3(256), 0, st, n, Nv, nsites, site_agg, Q,
                     qstride, ec, x, accumulate);
}

// ---------------------------------------------------------------------------
// block orthonormalisation on a coarse level (CGS2, FP64), one workgroup per
// (aggregate, half), one thread per row (site j, component c of the half)
template <class RI, class RO>
__global__ void __launch_bounds__(1024) k_qr_coarse(int n, int Nv, int asz, const int* __restrict__ agg_sites,
                                                    const cx<RI>* __restrict__ V, long vstride,
                                                    RO* __restrict__ Qraw, long qstride, int* __restrict__ fail) {
  cx<RO>* Qout = reinterpret_cast<cx<RO>*>(Qraw);
  __shared__ double red[32][16][2];
  __shared__ double dsh[32][2];
  int A = blockIdx.x >> 1, h = blockIdx.x & 1;
  int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int hn = n >> 1, rows = asz * hn;
  const int nw = (rows + 63) >> 6;
  const int nact = min(64, rows - wv * 64);
  bool act = t < rows;
  long idx = 0;
  if (act) {
    int j = t / hn, c = t - j * hn;
    idx = (long)agg_sites[A * asz + j] * n + h * hn + c;
  }
  auto reduce = [&](double a, double b, int slot) {
    a = wave_sum_n(a, nact);
    b = wave_sum_n(b, nact);
    if (lane == 0) {
      red[slot][wv][0] = a;
      red[slot][wv][1] = b;
    }
  };
  for (int i = 0; i < Nv; ++i) {
    cx<double> v = mk(0.0, 0.0);
    if (act) {
      cx<RI> vi = V[(long)i * vstride + idx];
      v = mk<double>(vi.re, vi.im);
    }
    reduce(norm2(v), 0.0, 0);
    __syncthreads();
    double nrm0 = 0;
    for (int w = 0; w < nw; ++w) nrm0 += red[0][w][0];
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
      for (int jj = 0; jj < i; ++jj) {
        double ar = 0, ai = 0;
        if (act) {
          cx<RO> q = Qout[(long)jj * qstride + idx];
          ar = (double)q.re * v.re + (double)q.im * v.im;
          ai = (double)q.re * v.im - (double)q.im * v.re;
        }
        reduce(ar, ai, jj);
      }
      __syncthreads();
      if (t < i) {
        double re = 0, im = 0;
        for (int w = 0; w < nw; ++w) {
          re += red[t][w][0];
          im += red[t][w][1];
        }
        dsh[t][0] = re;
        dsh[t][1] = im;
      }
      __syncthreads();
      if (act)
        for (int jj = 0; jj < i; ++jj) {
          cx<RO> q = Qout[(long)jj * qstride + idx];
          v = v - mk(dsh[jj][0], dsh[jj][1]) * mk<double>(q.re, q.im);
        }
      __syncthreads();
    }
    reduce(norm2(v), 0.0, 0);
    __syncthreads();
    double nrm = 0;
    for (int w = 0; w < nw; ++w) nrm += red[0][w][0];
    __syncthreads();
    if (!(nrm > 1e-24 * nrm0) && t == 0) atomicOr(fail, 1);
    double inv = nrm > 0 ? 1.0 / sqrt(nrm) : 0.0;
    if (act) Qout[(long)i * qstride + idx] = mk<RO>((RO)(inv * v.re), (RO)(inv * v.im));
  }
}
template <class RI, class RO>
void launch_qr_coarse(int n, int Nv, int nagg, int asz, const int* agg_sites, const cx<RI>* V, long vstride,
                      cx<RO>* Q, long qstride, int* fail, hipStream_t st) {
  int rows = asz * (n / 2);
  int threads = ((rows + 63) / 64) * 64;
  hipLaunchKernelGGL((k_qr_coarse<RI, RO>), dim3(2 * nagg), dim3(threads), 0, st, n, Nv, asz, agg_sites, V, vstride,
                     (RO*)Q, qstride, fail);
}

// ---------------------------------------------------------------------------
// Galerkin assembly of the next coarse operator from a coarse level, FP64.
// One workgroup per (aggregate A, kind): kind 0 = self (site blocks + links
// inside A), kind 1+mu = forward block (links across the upper mu face).
// q = Q(c) staged per site, Q(y) staged per piece; W = (operator block) * Q(y)
// per half of the output columns, one thread per (component k, group of 8
// vectors): each operator entry is loaded once (all loads in flight) and used
// for the 8 vectors from LDS.
template <class RQ>
__global__ void __launch_bounds__(256) k_assemble_coarse(CGeom cg, int Nv, int a0, int a1, int a2, int a3,
                                                         const int* __restrict__ agg_sites,
                                                         const cx<double>* __restrict__ D,
                                                         const cx<RQ>* __restrict__ Q, long qstride,
                                                         cx<double>* __restrict__ Dn, cx<double>* __restrict__ Xs) {
  const int n = cg.n, hn = n >> 1, np = 2 * Nv;
  const long nn = (long)n * n;
  const int asz = a0 * a1 * a2 * a3;
  const int ab[4] = {a0, a1, a2, a3};
  extern __shared__ char smem_raw[];
  // q rows padded to n + 1 entries: the output sums read 32 rows at one k
  cx<double>* q = reinterpret_cast<cx<double>*>(smem_raw);  // q[i][k] = Q_i(c)[k] at i (n + 1) + k
  cx<double>* W = q + Nv * (n + 1);                           // W[i][k] for output columns of one half
  cx<double>* qy = W + Nv * n;                                // qy[i][k] = Q_i(y)[k]
  // workgroup = (aggregate, kind, half hc of the output columns)
  const int A = blockIdx.x / 10, kind = (blockIdx.x % 10) >> 1, hc = blockIdx.x & 1;
  int t = threadIdx.x;
  const int nent = np * np, nh = Nv * np;  // entries per column half: e = hc nh + t + 256 m
  cx<double> accS[8], accX[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) accS[m] = accX[m] = mk(0.0, 0.0);
  for (int j = 0; j < asz; ++j) {
    int l[4];
    {
      int r = j;
      l[3] = r % a3;
      r /= a3;
      l[2] = r % a2;
      r /= a2;
      l[1] = r % a1;
      l[0] = r / a1;
    }
    if (kind > 0 && l[kind - 1] != ab[kind - 1] - 1) continue;
    int c = agg_sites[A * asz + j];
    __syncthreads();
    for (int e = t; e < Nv * n; e += 256) {
      int i = e / n, k = e - i * n;
      cx<RQ> v = Q[(long)i * qstride + (long)c * n + k];
      q[i * (n + 1) + k] = mk<double>(v.re, v.im);
    }
    // pieces: piece -1 = site block, piece mu = forward link in direction mu
    for (int piece = -1; piece < 4; ++piece) {
      int y;
      long blk;
      if (piece < 0) {
        if (kind != 0) continue;
        y = c;
        blk = (long)c * 5 * nn;
      } else {
        bool take = (kind == 0) ? (l[piece] + 1 < ab[piece]) : (piece == kind - 1);
        if (!take) continue;
        y = cg.nbr[c * 8 + piece];
        blk = ((long)c * 5 + 1 + piece) * nn;
      }
      bool toX = (kind == 0 && piece >= 0);
      __syncthreads();
      for (int e = t; e < Nv * n; e += 256) {
        int i = e / n, k = e - i * n;
        cx<RQ> v = Q[(long)i * qstride + (long)y * n + k];
        qy[e] = mk<double>(v.re, v.im);
      }
      {
        __syncthreads();
        // W[i][k] = sum_{k2 in half hc} B[k][k2] Q_i(y)[k2]
        const int ng = (Nv + 7) / 8;
        for (int task = t; task < n * ng; task += 256) {
          const int k = task % n, i0 = 8 * (task / n);
          cx<double> acc[8];
#pragma unroll
          for (int ii = 0; ii < 8; ++ii) acc[ii] = mk(0.0, 0.0);
#pragma unroll 4
          for (int k2 = hc * hn; k2 < (hc + 1) * hn; ++k2) {
            const cx<double> d = D[blk + (long)k2 * n + k];
#pragma unroll
            for (int ii = 0; ii < 8; ++ii)
              if (i0 + ii < Nv) cmac(acc[ii], d, qy[(i0 + ii) * n + k2]);
          }
#pragma unroll
          for (int ii = 0; ii < 8; ++ii)
            if (i0 + ii < Nv) W[(i0 + ii) * n + k] = acc[ii];
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          const int eh = t + 256 * m;
          if (eh < nh) {
            const int ic = eh / np, row = eh - ic * np;
            const int hr = row >= Nv ? 1 : 0, ir = row - hr * Nv;
            cx<double> acc = mk(0.0, 0.0);
            for (int k = hr * hn; k < (hr + 1) * hn; ++k) cjmac(acc, q[ir * (n + 1) + k], W[ic * n + k]);
            if (toX) accX[m] += acc;
            else accS[m] += acc;
          }
        }
      }
    }
  }
  cx<double>* out = Dn + ((long)A * 5 + kind) * nent;
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const int eh = t + 256 * m;
    if (eh < nh) {
      const int e = hc * nh + eh;
      out[e] = accS[m] + accX[m];
      if (kind == 0) Xs[(long)A * nent + e] = accX[m];
    }
  }
}
template <class RQ>
void launch_assemble_coarse(const CGeom& cg, int Nv, int nagg, const int ab[4], const int* agg_sites,
                            const cx<double>* D, const cx<RQ>* Q, long qstride, cx<double>* Dn, cx<double>* Xs,
                            hipStream_t st) {
  size_t sm = (3 * (size_t)Nv * cg.n + Nv) * sizeof(cx<double>);
  if (Nv > 32) throw Error(INVALID_ARG, "coarse assembly supports Nv <= 32");
  hipLaunchKernelGGL(k_assemble_coarse<RQ>, dim3(10 * nagg), dim3(256), sm, st, cg, Nv, ab[0], ab[1], ab[2], ab[3],
                     agg_sites, D, Q, qstride, Dn, Xs);
}

// S += Gamma5 X^dag Gamma5 (self blocks, column-major), and S += X first when
// the assembly wrote the internal forward links to X only (add_x)
__global__ void k_self_fixup(int n, int nsites, cx<double>* __restrict__ D, const cx<double>* __restrict__ Xs,
                             int add_x) {
  long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long nn = (long)n * n;
  if (gid >= (long)nsites * nn) return;
  int site = (int)(gid / nn);
  int e = (int)(gid - (long)site * nn);
  int col = e / n, row = e - col * n;
  cx<double> xv = Xs[(long)site * nn + (long)row * n + col];  // X(col,row)
  double s = g5(row, n) * g5(col, n);
  cx<double> d = D[(long)site * 5 * nn + e] + s * conj(xv);
  if (add_x) d += Xs[(long)site * nn + e];
  D[(long)site * 5 * nn + e] = d;
}
void launch_self_fixup(int n, int nsites, cx<double>* D, const cx<double>* Xs, int add_x, hipStream_t st) {
  long tot = (long)nsites * n * n;
  hipLaunchKernelGGL(k_self_fixup, dim3((tot + 255) / 256), dim3(256), 0, st, n, nsites, D, Xs, add_x);
}

// ---------------------------------------------------------------------------
// (S(c) + i tw Gamma5)^{-1} on the odd sites of the coarsest level: Gauss-Jordan
// with partial pivoting in FP64, one workgroup (64 threads) per odd site,
// working matrices in global scratch [nodd][2][n][n] (row-major A | inverse).
template <class R>
__global__ void __launch_bounds__(64) k_coarse_odd_inverse(CGeom cg, const cx<double>* __restrict__ D, double tw,
                                                           cx<double>* __restrict__ scr, cx<R>* __restrict__ Minv) {
  const int n = cg.n;
  const long nn = (long)n * n;
  int io = blockIdx.x;
  int site = cg.neven + io;
  int t = threadIdx.x;
  cx<double>* A = scr + (long)io * 2 * nn;
  cx<double>* Bm = A + nn;
  __shared__ cx<double> fcol[64];
  __shared__ int piv;
  if (t < n) {
    for (int r = 0; r < n; ++r) {
      cx<double> v = D[(long)site * 5 * nn + (long)t * n + r];  // element (r, t)
      if (r == t) v += mk(0.0, tw * g5(r, n));
      A[(long)r * n + t] = v;
      Bm[(long)r * n + t] = mk(r == t ? 1.0 : 0.0, 0.0);
    }
  }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    // pivot search over rows k..n-1 (thread t plays row t)
    double val = -1.0;
    int idx = k;
    if (t >= k && t < n) {
      val = norm2(A[(long)t * n + k]);
      idx = t;
    }
    for (int off = 32; off > 0; off >>= 1) {
      double ov = __shfl_xor(val, off, 64);
      int oi = __shfl_xor(idx, off, 64);
      if (ov > val || (ov == val && oi < idx)) {
        val = ov;
        idx = oi;
      }
    }
    if (t == 0) piv = idx;
    __syncthreads();
    int p = piv;
    if (t < n && p != k) {
      cx<double> a = A[(long)k * n + t], b = A[(long)p * n + t];
      A[(long)k * n + t] = b;
      A[(long)p * n + t] = a;
      a = Bm[(long)k * n + t];
      b = Bm[(long)p * n + t];
      Bm[(long)k * n + t] = b;
      Bm[(long)p * n + t] = a;
    }
    __syncthreads();
    cx<double> pv = A[(long)k * n + k];
    double d = norm2(pv);
    cx<double> inv = mk(pv.re / d, -pv.im / d);
    __syncthreads();
    if (t < n) {
      A[(long)k * n + t] = A[(long)k * n + t] * inv;
      Bm[(long)k * n + t] = Bm[(long)k * n + t] * inv;
      fcol[t] = A[(long)t * n + k];
    }
    __syncthreads();
    if (t < n) {
      cx<double> ak = A[(long)k * n + t], bk = Bm[(long)k * n + t];
      for (int r = 0; r < n; ++r) {
        if (r == k) continue;
        cx<double> f = fcol[r];
        A[(long)r * n + t] -= f * ak;
        Bm[(long)r * n + t] -= f * bk;
      }
    }
    __syncthreads();
  }
  if (t < n)
    for (int r = 0; r < n; ++r) {
      cx<double> v = Bm[(long)r * n + t];
      Minv[(long)io * nn + (long)t * n + r] = mk<R>((R)v.re, (R)v.im);  // column-major
    }
}
template <class R>
void launch_coarse_odd_inverse(const CGeom& cg, const cx<double>* D, double tw, cx<double>* scratch, cx<R>* Minv,
                               hipStream_t st) {
  int nodd = cg.nsites - cg.neven;
  hipLaunchKernelGGL(k_coarse_odd_inverse<R>, dim3(nodd), dim3(64), 0, st, cg, D, tw, scratch, Minv);
}

// ---------------------------------------------------------------------------
// odd sites: out = M (base - hop(in)) if base, else out = M hop(in)
template <class R, class S>
__global__ void __launch_bounds__(256) k_coarse_hop_inv_odd(CGeom cg,
                                                            const typename store_traits<S>::elem* __restrict__ D,
                                                            const cx<R>* __restrict__ Minv,
                                                            const cx<R>* __restrict__ in,
                                                            const cx<R>* __restrict__ base, cx<R>* __restrict__ out) {
  __shared__ cx<R> ys[4][9][64];
  __shared__ cx<R> us[4][64];
  int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int io = blockIdx.x * 4 + wv;
  int site = cg.neven + io;
  bool valid = site < cg.nsites;
  stage9(ys[wv], cg, site, valid, in, lane);
  __syncthreads();
  const int n = cg.n;
  if (valid && lane < n) {
    cx<R> u = hop_row<R, S>(cg, D, site, lane, ys[wv]);
    if (base) u = base[(long)site * n + lane] - u;
    us[wv][lane] = u;
  }
  __syncthreads();
  if (valid && lane < n) {
    const cx<R>* M = Minv + (long)io * n * n;
    cx<R> acc = mk<R>(0, 0);
    for (int l = 0; l < n; ++l) cmac(acc, M[(long)l * n + lane], us[wv][l]);
    out[(long)site * n + lane] = acc;
  }
}
template <class R, class S>
void launch_coarse_hop_inv_odd(const CGeom& cg, const void* D, const cx<R>* Minv, const cx<R>* in, cx<R>* out,
                               int subtract_from, hipStream_t st) {
  (void)subtract_from;
  int nodd = cg.nsites - cg.neven;
  hipLaunchKernelGGL((k_coarse_hop_inv_odd<R, S>), dim3((nodd + 3) / 4), dim3(256), 0, st, cg,
                     (const typename store_traits<S>::elem*)D, Minv, in, (const cx<R>*)nullptr, out);
}
template <class R, class S>
void launch_coarse_hop_inv_odd_base(const CGeom& cg, const void* D, const cx<R>* Minv, const cx<R>* in,
                                    const cx<R>* base, cx<R>* out, hipStream_t st) {
  int nodd = cg.nsites - cg.neven;
  hipLaunchKernelGGL((k_coarse_hop_inv_odd<R, S>), dim3((nodd + 3) / 4), dim3(256), 0, st, cg,
                     (const typename store_traits<S>::elem*)D, Minv, in, base, out);
}

// even sites: mode 0: out = (S + i tw G5) v - hop(t);  mode 1: out = v - hop(t)
template <class R, class S>
__global__ void __launch_bounds__(256) k_coarse_schur_even(CGeom cg,
                                                           const typename store_traits<S>::elem* __restrict__ D, R tw,
                                                           const cx<R>* __restrict__ v, const cx<R>* __restrict__ tv,
                                                           cx<R>* __restrict__ out, int mode) {
  __shared__ cx<R> ys[4][9][64];
  __shared__ cx<R> vs[4][64];
  int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int site = blockIdx.x * 4 + wv;
  bool valid = site < cg.neven;
  stage9(ys[wv], cg, site, valid, tv, lane);
  const int n = cg.n;
  if (valid && lane < n) vs[wv][lane] = v[(long)site * n + lane];
  __syncthreads();
  if (valid && lane < n) {
    cx<R> acc = mode == 0 ? self_row<R, S>(cg, D, site, lane, tw, vs[wv]) : vs[wv][lane];
    acc -= hop_row<R, S>(cg, D, site, lane, ys[wv]);
    out[(long)site * n + lane] = acc;
  }
}
template <class R, class S>
void launch_coarse_schur_even(const CGeom& cg, const void* D, double tw, const cx<R>* v, const cx<R>* t, cx<R>* out,
                              int mode, hipStream_t st) {
  hipLaunchKernelGGL((k_coarse_schur_even<R, S>), dim3((cg.neven + 3) / 4), dim3(256), 0, st, cg,
                     (const typename store_traits<S>::elem*)D, (R)tw, v, t, out, mode);
}

// ---------------------------------------------------------------------------
#define INST_RS(R, S)                                                                                              \
  template void launch_coarse_apply<R, S>(const CGeom&, const void*, double, const cx<R>*, cx<R>*, hipStream_t);  \
  template void launch_coarse_residual<R, S>(const CGeom&, const void*, double, const cx<R>*, const cx<R>*,       \
                                             cx<R>*, hipStream_t);                                                \
  template void launch_coarse_sap<R, S>(const CGeom&, const void*, double, int, int, const int*, const int*,      \
                                        const cx<R>*, cx<R>*, int, hipStream_t);                                  \
  template void launch_coarse_sap_multi<R, S>(const CGeom&, const void*, double, int, int, const int*,            \
                                              const int*, const cx<R>*, cx<R>*, int, int, long, hipStream_t);     \
  template void launch_coarse_hop_inv_odd<R, S>(const CGeom&, const void*, const cx<R>*, const cx<R>*, cx<R>*,    \
                                                int, hipStream_t);                                                \
  template void launch_coarse_hop_inv_odd_base<R, S>(const CGeom&, const void*, const cx<R>*, const cx<R>*,       \
                                                     const cx<R>*, cx<R>*, hipStream_t);                          \
  template void launch_coarse_schur_even<R, S>(const CGeom&, const void*, double, const cx<R>*, const cx<R>*,     \
                                               cx<R>*, int, hipStream_t);
INST_RS(double, double)
INST_RS(float, float)
INST_RS(float, f16)
INST_RS(float, bf16)

#define INST_R(R)                                                                                                   \
  template void launch_restrict_coarse<R>(int, int, int, int, const int*, const cx<R>*, long, const cx<R>*,        \
                                          cx<R>*, hipStream_t);                                                    \
  template void launch_prolong_coarse<R>(int, int, int, const int*, const cx<R>*, long, const cx<R>*, cx<R>*, int, \
                                         hipStream_t);                                                             \
  template void launch_restrict_coarse_m<R>(int, int, int, int, const int*, const cx<R>*, long, const cx<R>*, long, \
                                            cx<R>*, long, int, hipStream_t);                                       \
  template void launch_prolong_coarse_m<R>(int, int, int, const int*, const cx<R>*, long, const cx<R>*, long, cx<R>*, \
                                           long, int, int, hipStream_t);                                           \
  template void launch_qr_coarse<R, R>(int, int, int, int, const int*, const cx<R>*, long, cx<R>*, long, int*,   \
                                       hipStream_t);                                                               \
  template void launch_assemble_coarse<R>(const CGeom&, int, int, const int*, const int*, const cx<double>*,       \
                                          const cx<R>*, long, cx<double>*, cx<double>*, hipStream_t);              \
  template void launch_coarse_odd_inverse<R>(const CGeom&, const cx<double>*, double, cx<double>*, cx<R>*,         \
                                             hipStream_t);
INST_R(double)
INST_R(float)

}  // namespace ddamg
