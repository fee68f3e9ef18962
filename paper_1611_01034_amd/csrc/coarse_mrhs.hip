// Coarse operator on several right-hand sides at once, on the matrix cores.
//
// For K right-hand sides (K <= 16) stored one after the other (stride ldv
// complex), every coarse site needs
//   Y_r(c) = S(c) X_r(c) + sum_mu F_mu(c) X_r(c+mu)
//          + sum_mu Gamma5 F_mu(c-mu)^dag Gamma5 X_r(c-mu) + i tw Gamma5 X_r(c)
// (Sec. 1: D_c = P^dag D_W P, Gamma5,c-hermiticity, twist i mu Gamma5,c).
// Each of the 9 blocks times the K inputs is one real matrix product on the
// matrix cores: with A the n x n complex block and X the n x K inputs,
//   rows    i       : output component i,
//   columns (r, c)  : c = 0 real part, c = 1 imaginary part of right-hand side r,
//   inner   (l, c') : real / imaginary part of input component l,
//   A_real[i][(l,0)] = Re A_il,  A_real[i][(l,1)] = Im A_il,
//   B[(l,0)][(r,0)] = Re x_lr,  B[(l,1)][(r,0)] = -Im x_lr,
//   B[(l,0)][(r,1)] = Im x_lr,  B[(l,1)][(r,1)] =  Re x_lr,
// so that (A_real B)[i][(r,0)] = Re (A x_r)_i and [i][(r,1)] = Im (A x_r)_i.
// The interleaved (re, im) storage of the blocks is A_real row by row, so the
// stored 16-bit entries feed the matrix cores unconverted.  Inputs are rounded
// to the storage format for the product; accumulation is FP32; the twist is
// added in FP32 from the unrounded input.
//
// v_mfma_f32_16x16x32_{f16,bf16} (wave64) fragments: lane L holds A[L%16][8(L/16) + e]
// and B[8(L/16) + e][L%16] for e < 8; the result D[4(L/16) + e][L%16] for e < 4.
//
// One workgroup per coarse site with n/16 wavefronts, wavefront t computing
// output rows 16t..16t+15 (n = 2 N_v a multiple of 16, n <= 64): short
// dependency chains and n/16 times the wavefronts of a one-per-site mapping,
// which is what keeps these small, latency-bound grids busy.
#include "kernels.hpp"

namespace ddamg {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef __bf16 v8b __attribute__((ext_vector_type(8)));

template <class S> struct mm16;
template <> struct mm16<f16> {
  using frag = v8h;
  using e16 = f16;
  static __device__ __forceinline__ v4f mma(frag a, frag b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};
template <> struct mm16<bf16> {
  using frag = v8b;
  using e16 = bf16;
  static __device__ __forceinline__ v4f mma(frag a, frag b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

// B fragment of input x (n components, right-hand side stride ldv) for the
// lane's column j = 16u + L%16 and complex inputs lc..lc+3; sgn scales x.
template <class S>
__device__ __forceinline__ typename mm16<S>::frag b_frag(const cx<float>* x, long ldv, int K, int j, int lc, float sgn) {
  using E = typename mm16<S>::e16;
  typename mm16<S>::frag f;
  const int r = j >> 1, c = j & 1;
  if (r < K) {
    const float4* p = reinterpret_cast<const float4*>(x + (long)r * ldv + lc);
    float4 a = p[0], b = p[1];
    float v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      float re = sgn * v[2 * q], im = sgn * v[2 * q + 1];
      f[2 * q] = (E)(c == 0 ? re : im);
      f[2 * q + 1] = (E)(c == 0 ? -im : re);
    }
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q) f[q] = (E)0.0f;
  }
  return f;
}

// A fragment of a block stored column-major (entry (i,l) at l*n + i): row i,
// complex columns lc..lc+3
template <class S>
__device__ __forceinline__ typename mm16<S>::frag a_frag_col(const typename store_traits<S>::elem* blk, int n, int i,
                                                            int lc) {
  typename mm16<S>::frag f;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    auto e = blk[(long)(lc + q) * n + i];
    f[2 * q] = e.re;
    f[2 * q + 1] = e.im;
  }
  return f;
}

// A fragment of g_i conj(F[l][i]) (F column-major: (l,i) at i*n + l), i.e. the
// backward block Gamma5 F^dag Gamma5 without the g_l factor (applied to x)
template <class S>
__device__ __forceinline__ typename mm16<S>::frag a_frag_bwd(const typename store_traits<S>::elem* blk, int n, int i,
                                                            int lc, bool neg_row) {
  using E = typename mm16<S>::e16;
  typename mm16<S>::frag f;
  const typename store_traits<S>::elem* p = blk + (long)i * n + lc;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    auto e = p[q];
    E re = e.re, im = e.im;
    f[2 * q] = neg_row ? (E)(-(float)re) : re;
    f[2 * q + 1] = neg_row ? im : (E)(-(float)im);
  }
  return f;
}

// acc[u] += sum over the selected blocks, output rows 16t..16t+15, columns 16u..
//   self: S(site) xs(site);  hops: hs * (forward + backward hops of xh)
// RT = n / 16 k-steps per block.  For one column tile every fragment of a block
// is loaded before its products and two blocks are in flight, so a wavefront
// waits on about one memory latency per two blocks.
template <class S, int NT, int RT>
__device__ __forceinline__ void stencil_mfma(const CGeom& cg, const typename store_traits<S>::elem* D, int site,
                                             int t, const cx<float>* xs, const cx<float>* xh, float hs, int K,
                                             long ldv, int lane, v4f acc[NT]) {
  constexpr int n = 16 * RT, h = n / 2;
  constexpr long nn = (long)n * n;
  const int row = lane & 15, grp = lane >> 4;
  const int i = 16 * t + row;
#pragma unroll(NT == 1 ? 2 : 1)
  for (int b = xs ? 0 : 1; b < (xh ? 9 : 1); ++b) {
    const typename store_traits<S>::elem* blk;
    const cx<float>* x;
    float sgn = 1.0f;
    const bool bwd = b >= 5;
    if (b == 0) {
      blk = D + (long)site * 5 * nn;
      x = xs + (long)site * n;
    } else if (!bwd) {
      const int mu = b - 1;
      blk = D + ((long)site * 5 + 1 + mu) * nn;
      x = xh + (long)cg.nbr[site * 8 + mu] * n;
      sgn = hs;
    } else {
      const int mu = b - 5;
      const int cb = cg.nbr[site * 8 + 4 + mu];
      blk = D + ((long)cb * 5 + 1 + mu) * nn;
      x = xh + (long)cb * n;
      sgn = hs;
    }
    if constexpr (NT == 1) {
      typename mm16<S>::frag af[RT], bf[RT];
#pragma unroll
      for (int s = 0; s < RT; ++s) {
        const int lc = 16 * s + 4 * grp;
        // g_l of the backward block goes on the input (lc..lc+3 lie in one half)
        const float gs = bwd ? (lc < h ? -sgn : sgn) : sgn;
        bf[s] = b_frag<S>(x, ldv, K, row, lc, gs);
        af[s] = bwd ? a_frag_bwd<S>(blk, n, i, lc, i < h) : a_frag_col<S>(blk, n, i, lc);
      }
#pragma unroll
      for (int s = 0; s < RT; ++s) acc[0] = mm16<S>::mma(af[s], bf[s], acc[0]);
    } else {
      // two column tiles: one k-step at a time keeps the registers (and the
      // occupancy) of the wider products
#pragma unroll 1
      for (int s = 0; s < RT; ++s) {
        const int lc = 16 * s + 4 * grp;
        const float gs = bwd ? (lc < h ? -sgn : sgn) : sgn;
        typename mm16<S>::frag bf[NT];
#pragma unroll
        for (int u = 0; u < NT; ++u) bf[u] = b_frag<S>(x, ldv, K, 16 * u + row, lc, gs);
        const typename mm16<S>::frag af = bwd ? a_frag_bwd<S>(blk, n, i, lc, i < h) : a_frag_col<S>(blk, n, i, lc);
#pragma unroll
        for (int u = 0; u < NT; ++u) acc[u] = mm16<S>::mma(af, bf[u], acc[u]);
      }
    }
  }
}

template <int NT>
__device__ __forceinline__ void zero_acc(v4f acc[NT]) {
#pragma unroll
  for (int u = 0; u < NT; ++u) acc[u] = v4f{0.f, 0.f, 0.f, 0.f};
}

// Write the result of the site: y = acc (+ i tw Gamma5 xt) or y = base - (...)
// (xt: input of the twist term, or null).
template <int NT>
__device__ __forceinline__ void store_mfma(const CGeom& cg, int site, int t, v4f acc[NT], float tw,
                                           const cx<float>* xt, const cx<float>* base, float base_sign, int K,
                                           long ldv, int lane, cx<float>* y) {
  const int n = cg.n, h = n >> 1;
  const int col = lane & 15, grp = lane >> 4;
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    const int j = 16 * u + col, r = j >> 1, c = j & 1;
    if (r >= K) continue;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = 16 * t + 4 * grp + e;
      const long o = (long)r * ldv + (long)site * n + i;
      float v = acc[u][e];
      if (xt) {
        cx<float> xv = xt[o];
        float g = i < h ? -tw : tw;
        v += c == 0 ? -g * xv.im : g * xv.re;
      }
      if (base) {
        const float* bp = reinterpret_cast<const float*>(base + o);
        v = bp[c] + base_sign * v;
      }
      reinterpret_cast<float*>(y + o)[c] = v;
    }
  }
}

// y_r = D x_r (b == null) or y_r = b_r - D x_r, on every site or on the sites
// of a list.  On every site, each XCD takes a contiguous range of sites in
// lexicographic order (both parities interleaved), so the forward block a
// site reads for its own hop is still in that XCD's L2 when its X and Y
// neighbours read it for their backward hops (level 1 of 48^3x96 at six
// columns: 0.93 -> 0.81 ms per application).
template <class S, int NT, int RT>
__global__ void __launch_bounds__(256) k_coarse_apply_mrhs(CGeom cg, const typename store_traits<S>::elem* __restrict__ D,
                                                           float tw, int K, long ldv, const cx<float>* __restrict__ x,
                                                           const cx<float>* __restrict__ b, cx<float>* __restrict__ y,
                                                           const int* __restrict__ sites) {
  const int lane = threadIdx.x & 63, t = threadIdx.x >> 6;
  const int site = sites ? sites[blockIdx.x] : cg.lexord[xcd_remap(blockIdx.x, gridDim.x)];
  v4f acc[NT];
  zero_acc<NT>(acc);
  stencil_mfma<S, NT, RT>(cg, D, site, t, x, x, 1.0f, K, ldv, lane, acc);
  store_mfma<NT>(cg, site, t, acc, tw, x, b, -1.0f, K, ldv, lane, y);
}

// even sites of the odd-even reduced system: mode 0: y = (S + i tw G5) v - H t;
// mode 1: y = v - H t   (H: the hops, t lives on the odd sites)
template <class S, int NT, int RT>
__global__ void __launch_bounds__(256) k_coarse_schur_even_mrhs(CGeom cg,
                                                                const typename store_traits<S>::elem* __restrict__ D,
                                                                float tw, int K, long ldv,
                                                                const cx<float>* __restrict__ v,
                                                                const cx<float>* __restrict__ t,
                                                                cx<float>* __restrict__ y, int mode) {
  const int lane = threadIdx.x & 63, rt = threadIdx.x >> 6;
  const int site = blockIdx.x;
  v4f acc[NT];
  zero_acc<NT>(acc);
  stencil_mfma<S, NT, RT>(cg, D, site, rt, mode == 0 ? v : nullptr, t, -1.0f, K, ldv, lane, acc);
  if (mode == 0) store_mfma<NT>(cg, site, rt, acc, tw, v, nullptr, 1.0f, K, ldv, lane, y);
  else store_mfma<NT>(cg, site, rt, acc, 0.0f, nullptr, v, 1.0f, K, ldv, lane, y);
}

// odd sites: y = Minv H x, or y = Minv (base - H x) with base.  Minv:
// [odd site][n][n] FP32 column-major.  The hop result goes through LDS
// ([n][K] complex) to the FP32 products with Minv, which all threads of the
// workgroup share: thread -> row i = tid % n and a quarter g = tid / n of the
// inner index (16 terms, all loads in flight), the four partial sums added in
// LDS ([4][n][K]) in fixed order.  For K > 8 a thread takes row i and every
// fourth column instead, with all n inner terms, and the partial sums go
// away.  The LDS is sized by K at launch: at K = 2 the kernel holds 6
// wavefronts per SIMD instead of 4 (13 % faster odd-even operator at 48^3x96).
template <class S, int NT, int RT>
__global__ void __launch_bounds__(256) k_coarse_hop_inv_odd_mrhs(CGeom cg,
                                                                 const typename store_traits<S>::elem* __restrict__ D,
                                                                 const cx<float>* __restrict__ Minv, int K, long ldv,
                                                                 const cx<float>* __restrict__ x,
                                                                 const cx<float>* __restrict__ base,
                                                                 cx<float>* __restrict__ y) {
  constexpr int n = 16 * RT, LQ = n / 4;
  extern __shared__ char smem_raw[];
  cx<float>* us = reinterpret_cast<cx<float>*>(smem_raw);  // [n][K]
  cx<float>* ps = us + n * K;                               // [4][n][K]
  const int lane = threadIdx.x & 63, rt = threadIdx.x >> 6;
  const int io = blockIdx.x;
  const int site = cg.neven + io;
  const int i = threadIdx.x % n, gq = threadIdx.x / n;  // gq < 4 (blockDim = 4 n)
  cx<float> m[LQ];
  {
    v4f acc[NT];
    zero_acc<NT>(acc);
    stencil_mfma<S, NT, RT>(cg, D, site, rt, nullptr, x, 1.0f, K, ldv, lane, acc);
    const int col = lane & 15, grp = lane >> 4;
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      const int j = 16 * u + col, r = j >> 1, c = j & 1;
      if (r >= K) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = 16 * rt + 4 * grp + e;
        float v = acc[u][e];
        if (base) v = reinterpret_cast<const float*>(base + (long)r * ldv + (long)site * n + i)[c] - v;
        reinterpret_cast<float*>(&us[i * K + r])[c] = v;
      }
    }
  }
  __syncthreads();
  if constexpr (NT == 2) {
    // K > 8: thread (row i, column group gq) sums all n inner terms for the
    // columns gq, gq + 4, ... (no partial sums in LDS; the four column groups
    // read the same inverse entries, which the L1 shares)
    const cx<float>* M = Minv + (long)io * n * n;
    cx<float> o[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) o[q] = mk<float>(0, 0);
#pragma unroll 1
    for (int l0 = 0; l0 < n; l0 += 16) {
      cx<float> mm[16];
#pragma unroll
      for (int l = 0; l < 16; ++l) mm[l] = M[(long)(l0 + l) * n + i];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = gq + 4 * q;
        if (r < K) {
#pragma unroll
          for (int l = 0; l < 16; ++l) cmac(o[q], mm[l], us[(l0 + l) * K + r]);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = gq + 4 * q;
      if (r < K) y[(long)r * ldv + (long)site * n + i] = o[q];
    }
    return;
  }
  {
    const cx<float>* M = Minv + (long)io * n * n;
#pragma unroll
    for (int l = 0; l < LQ; ++l) m[l] = M[(long)(gq * LQ + l) * n + i];
  }
  for (int r = 0; r < K; ++r) {
    cx<float> o = mk<float>(0, 0);
#pragma unroll
    for (int l = 0; l < LQ; ++l) cmac(o, m[l], us[(gq * LQ + l) * K + r]);
    ps[(gq * n + i) * K + r] = o;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n * K; e += blockDim.x) {
    const int ii = e % n, r = e / n;
    const cx<float> o = (ps[(0 * n + ii) * K + r] + ps[(1 * n + ii) * K + r]) +
                        (ps[(2 * n + ii) * K + r] + ps[(3 * n + ii) * K + r]);
    y[(long)r * ldv + (long)site * n + ii] = o;
  }
}

// SAP on the blocks of one colour of an intermediate level for K fields in
// one workgroup per block: n_mr MR steps on the block operator D_B (hops
// leaving the block dropped).  Wavefront j takes block site j and computes
// q = D_B rho for its n rows and all K fields on the matrix cores (the
// operator is read once per step for all fields); rho of the block lives in
// LDS as [site][field][n] complex FP32 and is rounded to the storage format for
// the products, as in the K-column stencil.  Per field the MR coefficient
// <q, rho> / <q, q> is summed over the block in fixed order (FP32 per lane,
// FP64 over the sites).  x += the accumulated correction at the end.
template <class S, int NT, int RT>
__global__ void __launch_bounds__(1024) k_coarse_sap_mrhs(CGeom cg,
                                                          const typename store_traits<S>::elem* __restrict__ D,
                                                          float tw, int bsz, const int* __restrict__ blk_sites,
                                                          const int* __restrict__ blk_nbr,
                                                          const cx<float>* __restrict__ r, cx<float>* __restrict__ x,
                                                          int n_mr, int K, long ld) {
  constexpr int n = 16 * RT, h = n / 2;
  constexpr long nn = (long)n * n;
  extern __shared__ char smem_raw[];
  cx<float>* rho = reinterpret_cast<cx<float>*>(smem_raw);  // [bsz][K][n]
  __shared__ float red[16][16][3];                          // [site][field][<q,rho> re, im, <q,q>]
  __shared__ cx<float> alpha[16];
  const int blk = blockIdx.x;
  const int j = threadIdx.x >> 6, lane = threadIdx.x & 63, row = lane & 15, grp = lane >> 4;
  const int site = blk_sites[blk * bsz + j];
  const int* lnb = blk_nbr + ((long)blk * bsz + j) * 8;
  for (int e = lane; e < K * n; e += 64) {
    const int rr = e / n, l = e - rr * n;
    rho[((long)j * K + rr) * n + l] = r[(long)rr * ld + (long)site * n + l];
  }
  float eps[RT][NT][4], qm[RT][NT][4], qp[RT][NT][4];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int u = 0; u < NT; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) eps[t][u][e] = 0.f;
  for (int it = 0; it < n_mr; ++it) {
    __syncthreads();  // rho of every site complete
    v4f acc[RT][NT];
#pragma unroll
    for (int t = 0; t < RT; ++t) zero_acc<NT>(acc[t]);
#pragma unroll 1
    for (int b = 0; b < 9; ++b) {
      const typename store_traits<S>::elem* bp;
      int jn;
      const bool bwd = b >= 5;
      if (b == 0) {
        jn = j;
        bp = D + (long)site * 5 * nn;
      } else if (!bwd) {
        jn = lnb[b - 1];
        if (jn < 0) continue;
        bp = D + ((long)site * 5 + b) * nn;
      } else {
        jn = lnb[b - 1];
        if (jn < 0) continue;
        bp = D + ((long)blk_sites[blk * bsz + jn] * 5 + b - 4) * nn;
      }
      const cx<float>* xr = rho + (long)jn * K * n;
#pragma unroll
      for (int s = 0; s < RT; ++s) {
        const int lc = 16 * s + 4 * grp;
        const float gs = bwd ? (lc < h ? -1.0f : 1.0f) : 1.0f;
        typename mm16<S>::frag bf[NT], af[RT];
#pragma unroll
        for (int u = 0; u < NT; ++u) bf[u] = b_frag<S>(xr, n, K, 16 * u + row, lc, gs);
#pragma unroll
        for (int t = 0; t < RT; ++t) {
          const int i = 16 * t + row;
          af[t] = bwd ? a_frag_bwd<S>(bp, n, i, lc, i < h) : a_frag_col<S>(bp, n, i, lc);
        }
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
          for (int u = 0; u < NT; ++u) acc[t][u] = mm16<S>::mma(af[t], bf[u], acc[t][u]);
      }
    }
    // twist, then the complex q of every entry (own part and the partner lane's)
    float pr[NT][3];
#pragma unroll
    for (int u = 0; u < NT; ++u) pr[u][0] = pr[u][1] = pr[u][2] = 0.f;
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int u = 0; u < NT; ++u) {
        const int jc = 16 * u + row, rr = jc >> 1, c = jc & 1;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int i = 16 * t + 4 * grp + e;
          float v = acc[t][u][e];
          cx<float> rv = mk<float>(0.f, 0.f);
          if (rr < K) {
            rv = rho[((long)j * K + rr) * n + i];
            const float g = i < h ? -tw : tw;
            v += c == 0 ? -g * rv.im : g * rv.re;
          }
          const float o = __shfl_xor(v, 1, 64);
          qm[t][u][e] = v;
          qp[t][u][e] = o;
          const float qre = c == 0 ? v : o, qim = c == 0 ? o : v;
          if (c == 0 && rr < K) {
            pr[u][0] += qre * rv.re + qim * rv.im;
            pr[u][1] += qre * rv.im - qim * rv.re;
            pr[u][2] += qre * qre + qim * qim;
          }
        }
      }
#pragma unroll
    for (int u = 0; u < NT; ++u)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        float v = pr[u][k];
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        const int rr = (16 * u + row) >> 1;
        if (grp == 0 && (row & 1) == 0 && rr < K) red[j][rr][k] = v;
      }
    __syncthreads();
    if (threadIdx.x < K) {
      double sr = 0, si = 0, sq = 0;
      for (int q = 0; q < bsz; ++q) {
        sr += red[q][threadIdx.x][0];
        si += red[q][threadIdx.x][1];
        sq += red[q][threadIdx.x][2];
      }
      alpha[threadIdx.x] = sq > 0 ? mk<float>((float)(sr / sq), (float)(si / sq)) : mk<float>(0.f, 0.f);
    }
    __syncthreads();
    // eps += alpha rho;  rho -= alpha q   (own component c of each entry)
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int u = 0; u < NT; ++u) {
        const int jc = 16 * u + row, rr = jc >> 1, c = jc & 1;
        const cx<float> a = alpha[rr < K ? rr : 0];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int i = 16 * t + 4 * grp + e;
          // each lane reads and writes only its own component c of rho; the
          // other one comes from the partner lane
          float* rp = reinterpret_cast<float*>(&rho[((long)j * K + (rr < K ? rr : 0)) * n + i]);
          const float ro = rr < K ? rp[c] : 0.f;
          const float rq = __shfl_xor(ro, 1, 64);
          const float qo = qm[t][u][e], qq = qp[t][u][e];
          // (a z)_c: c = 0 -> a.re z.re - a.im z.im;  c = 1 -> a.re z.im + a.im z.re
          const float sgn = c == 0 ? -1.f : 1.f;
          if (rr < K) {
            eps[t][u][e] += a.re * ro + sgn * a.im * rq;
            rp[c] = ro - (a.re * qo + sgn * a.im * qq);
          }
        }
      }
  }
  // x += eps
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      const int jc = 16 * u + row, rr = jc >> 1, c = jc & 1;
      if (rr >= K) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = 16 * t + 4 * grp + e;
        reinterpret_cast<float*>(x + (long)rr * ld + (long)site * n + i)[c] += eps[t][u][e];
      }
    }
}

static inline int nt_of(int K) { return K <= 8 ? 1 : 2; }

// instantiate KERNEL<S, NT, RT> for NT = nt_of(K), RT = n / 16
#define MRHS_DISPATCH(KERNEL, ...)                                                   \
  do {                                                                               \
    const int nt = nt_of(K), rt = cg.n / 16;                                         \
    if (cg.n % 16 || rt < 1 || rt > 4) throw Error(INVALID_ARG, "coarse n must be 16, 32, 48 or 64"); \
    if (nt == 1) {                                                                   \
      switch (rt) {                                                                  \
        case 1: hipLaunchKernelGGL((KERNEL<S, 1, 1>), __VA_ARGS__); break;           \
        case 2: hipLaunchKernelGGL((KERNEL<S, 1, 2>), __VA_ARGS__); break;           \
        case 3: hipLaunchKernelGGL((KERNEL<S, 1, 3>), __VA_ARGS__); break;           \
        default: hipLaunchKernelGGL((KERNEL<S, 1, 4>), __VA_ARGS__); break;          \
      }                                                                              \
    } else {                                                                         \
      switch (rt) {                                                                  \
        case 1: hipLaunchKernelGGL((KERNEL<S, 2, 1>), __VA_ARGS__); break;           \
        case 2: hipLaunchKernelGGL((KERNEL<S, 2, 2>), __VA_ARGS__); break;           \
        case 3: hipLaunchKernelGGL((KERNEL<S, 2, 3>), __VA_ARGS__); break;           \
        default: hipLaunchKernelGGL((KERNEL<S, 2, 4>), __VA_ARGS__); break;          \
      }                                                                              \
    }                                                                                \
  } while (0)

template <class S>
void launch_coarse_apply_mrhs(const CGeom& cg, const void* D, double tw, int K, long ldv, const cx<float>* x,
                              const cx<float>* b, cx<float>* y, hipStream_t st, const int* sites, int nlist) {
  dim3 grid(sites ? nlist : cg.nsites), blk(4 * cg.n);
  if (grid.x == 0) return;
  auto Dp = (const typename store_traits<S>::elem*)D;
  MRHS_DISPATCH(k_coarse_apply_mrhs, grid, blk, 0, st, cg, Dp, (float)tw, K, ldv, x, b, y, sites);
}

template <class S>
void launch_coarse_schur_even_mrhs(const CGeom& cg, const void* D, double tw, int K, long ldv, const cx<float>* v,
                                   const cx<float>* t, cx<float>* y, int mode, hipStream_t st) {
  dim3 grid(cg.neven), blk(4 * cg.n);
  auto Dp = (const typename store_traits<S>::elem*)D;
  MRHS_DISPATCH(k_coarse_schur_even_mrhs, grid, blk, 0, st, cg, Dp, (float)tw, K, ldv, v, t, y, mode);
}

template <class S>
void launch_coarse_hop_inv_odd_mrhs(const CGeom& cg, const void* D, const cx<float>* Minv, int K, long ldv,
                                    const cx<float>* x, const cx<float>* base, cx<float>* y, hipStream_t st) {
  int nodd = cg.nsites - cg.neven;
  if (K < 1 || K > 16) throw Error(INVALID_ARG, "K-column coarse operator: 1 <= K <= 16");
  dim3 grid(nodd), blk(4 * cg.n);
  // hop result [n][K], and for K <= 8 the four partial sums [4][n][K]
  const size_t sm = (size_t)(nt_of(K) == 2 ? 1 : 5) * cg.n * K * sizeof(cx<float>);
  auto Dp = (const typename store_traits<S>::elem*)D;
  MRHS_DISPATCH(k_coarse_hop_inv_odd_mrhs, grid, blk, sm, st, cg, Dp, Minv, K, ldv, x, base, y);
}

template <class S>
void launch_coarse_sap_mrhs(const CGeom& cg, const void* D, double tw, int nblk_colour, int bsz, const int* blk_sites,
                            const int* blk_nbr, const cx<float>* r, cx<float>* x, int n_mr, int K, long ld,
                            hipStream_t st) {
  if (bsz < 1 || bsz > 16 || K < 1 || K > 16) throw Error(INVALID_ARG, "K-field coarse SAP: bad block or field count");
  const size_t sm = (size_t)bsz * K * cg.n * sizeof(cx<float>);
  dim3 grid(nblk_colour), blk(64 * bsz);
  auto Dp = (const typename store_traits<S>::elem*)D;
  MRHS_DISPATCH(k_coarse_sap_mrhs, grid, blk, sm, st, cg, Dp, (float)tw, bsz, blk_sites, blk_nbr, r, x, n_mr, K, ld);
}

#define INST_MRHS(S)                                                                                              \
  template void launch_coarse_apply_mrhs<S>(const CGeom&, const void*, double, int, long, const cx<float>*,      \
                                            const cx<float>*, cx<float>*, hipStream_t, const int*, int);         \
  template void launch_coarse_schur_even_mrhs<S>(const CGeom&, const void*, double, int, long, const cx<float>*, \
                                                 const cx<float>*, cx<float>*, int, hipStream_t);                \
  template void launch_coarse_hop_inv_odd_mrhs<S>(const CGeom&, const void*, const cx<float>*, int, long,        \
                                                  const cx<float>*, const cx<float>*, cx<float>*, hipStream_t);  \
  template void launch_coarse_sap_mrhs<S>(const CGeom&, const void*, double, int, int, const int*, const int*,  \
                                          const cx<float>*, cx<float>*, int, int, long, hipStream_t);
INST_MRHS(f16)
INST_MRHS(bf16)

}  // namespace ddamg
