// Fine-lattice kernels: layout transforms, clover term, the twisted-mass
// Wilson-clover operator D(mu) = D_W + i mu Gamma5 (paper Sec. 1), the SAP
// smoother with odd-even block MR (Sec. 1 smoother, Sec. 3 odd-even in the
// smoother), Gamma5-compatible restriction / prolongation and block
// orthonormalisation (Sec. 1 aggregation), and the Galerkin assembly of the
// first coarse operator D_c = P^dag D_W P (Sec. 1, Eq. 1 context).
//
// Operator conventions (the paper fixes gamma5 = diag(-1,-1,1,1) and TZYX
// order only):
//   (D psi)(x) = T(x) psi(x) - 1/2 sum_mu [(1-g_mu) U_mu(x) psi(x+mu)
//                                        + (1+g_mu) U_mu(x-mu)^dag psi(x-mu)]
//   T(x) = (m0+4) + A(x) + i tw gamma5,   A = (i c_sw/4) sum sigma_{mu nu} F_{mu nu}
// Chiral gamma basis: g_k = [[0,-i s_k],[i s_k,0]] (k = X,Y,Z), g_T = [[0,-1],[-1,0]].
// With g_mu = [[0,B],[B^dag,0]] the projector (1 -+ g_mu) has rank 2: only the
// half spinor h = psi_up -+ B psi_dn is transported by U, the lower half is
// rebuilt from it.  Per direction and sign the reconstruction is a pair of
// phases in {1, i, -1, -i} and a spin permutation (tables below).
#include "finedev.hpp"


namespace ddamg {



// ---------------------------------------------------------------------------
// workgroup reduction helpers (deterministic: fixed shuffle and wave order)

// ---------------------------------------------------------------------------
// SAP: one colour sweep.  One workgroup per block of the colour, one thread per
// slot (even slots first).  r = b - D x on the block, then n_mr MR steps
// on the block-local even-site Schur complement S = T_ee - D_eo T_oo^{-1} D_oe
// (hops leaving the block dropped), odd reconstruction, x += e.

// In-block neighbours of a slot, packed: for direction mu the forward and the
// backward neighbour's index within the other parity's half of the block
// (bytes 2(mu&1) and 2(mu&1)+1 of word mu>>1), or `half` where the hop
// leaves the block.  Computed once per thread; the block solve reads its
// neighbours from LDS halves whose index `half` holds a zero spinor, so a
// dropped hop costs neither an index computation nor a mask.
struct BlockNbr {
  unsigned w[2];
};
__device__ __forceinline__ BlockNbr block_nbrs(const Geom& g, const SiteNbr& me) {
  BlockNbr nb{{0u, 0u}};
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    int l[4] = {me.l[0], me.l[1], me.l[2], me.l[3]};
    const int l0 = l[mu];
    int f = g.half, b = g.half;
    if (l0 + 1 < g.b[mu]) {
      l[mu] = l0 + 1;
      const int sn = local_slot(g, l);
      f = sn >= g.half ? sn - g.half : sn;
    }
    if (l0 > 0) {
      l[mu] = l0 - 1;
      const int sn = local_slot(g, l);
      b = sn >= g.half ? sn - g.half : sn;
    }
    nb.w[mu >> 1] |= (unsigned)(f | (b << 8)) << (16 * (mu & 1));
  }
  return nb;
}

// out += (or -= with SUB) the in-block hops of slot s, the neighbours' spinors
// read from lds (12 x hs, component-major, the other parity's half of the
// block; entry `half` of every component is zero).  noff: slot offset of the
// neighbours' parity (their links are read for the backward hops).  Both links
// of a direction are loaded before its arithmetic (one memory latency per
// direction); a dropped backward hop reads a link of the block, multiplied by
// the zero spinor.
template <class R, class S, bool SUB = false>
__device__ __forceinline__ void hop_block_lds(const typename store_traits<S>::elem* U, const Geom& g, int B, int s,
                                              BlockNbr nb, int noff, const cx<R>* lds, int hs, cx<R> out[12]) {
  using E = typename store_traits<S>::elem;
  // opaque per call: nothing derived from the neighbour words or the slot is
  // kept live across the MR steps
  __asm__ volatile("" : "+v"(nb.w[0]), "+v"(nb.w[1]), "+v"(s));
  const long blk = (long)B * (g.bs / TILE) * 36 * TILE;
  const long base_s = blk + (long)(s / TILE) * 36 * TILE + (s % TILE);
#pragma unroll 1
  for (int mu = 0; mu < 4; ++mu) {
    const unsigned wd = (mu < 2 ? nb.w[0] : nb.w[1]) >> (16 * (mu & 1));
    const int sf = wd & 255, sb = (wd >> 8) & 255;
    const int lb = min(sb, g.half - 1) + noff;
    const long bf = base_s + (long)mu * 9 * TILE;
    const long bb = blk + (long)(lb / TILE) * 36 * TILE + (lb % TILE) + (long)mu * 9 * TILE;
    E cf[9], cb[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      cf[k] = U[bf + (long)k * TILE];
      cb[k] = U[bb + (long)k * TILE];
    }
    cx<R> psi[12], u[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) u[k] = mk<R>((R)cf[k].re, (R)cf[k].im);
#pragma unroll
    for (int c = 0; c < 12; ++c) psi[c] = SUB ? -lds[c * hs + sf] : lds[c * hs + sf];
    hop_accum<0>(mu, psi, u, out);
#pragma unroll
    for (int k = 0; k < 9; ++k) u[k] = mk<R>((R)cb[k].re, (R)cb[k].im);
#pragma unroll
    for (int c = 0; c < 12; ++c) psi[c] = SUB ? -lds[c * hs + sb] : lds[c * hs + sb];
    hop_accum<1>(mu, psi, u, out);
  }
}

// SAP colour sweep.  One workgroup per block of the colour (and field), one
// thread per pair of slots: thread i owns even slot i and odd slot half + i,
// so both wavefronts of a block have work in the even-site and in the
// odd-site half of every MR step.
//   r = b - D x on the block;  t_o = T_oo^{-1} r_o,  x_o += t_o;
//   rho = r_e - D_eo t_o;  n_mr MR steps on S = T_ee - D_eo T_oo^{-1} D_oe
//   (block-local hops only) accumulate e_e;  x_e += e_e,
//   x_o -= T_oo^{-1} D_oe e_e  (together: x_o += T_oo^{-1} (r_o - D_oe e_e)).
// x of a block is read and written by its own workgroup only: the residual
// reads the other colour's blocks, which this sweep leaves unchanged.
template <class R, class S>
__global__ void __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 8 ? 1 : 2, 8)))
k_sap(Geom g, int colour, const typename store_traits<S>::elem* __restrict__ U, const R* __restrict__ H,
      const R* __restrict__ Minv, TwistR<R> tw, const cx<R>* __restrict__ b, cx<R>* __restrict__ x, int n_mr, int K,
      long ld) {
  extern __shared__ char smem_raw[];
  // the residual stages x of the block parity-split (24 x half); the block
  // solve then keeps one field per parity as 12 x hs (hs = half + 1: entry
  // half of each component is the zero spinor of dropped hops)
  const int hs = g.half + 1;
  cx<R>* ev = reinterpret_cast<cx<R>*>(smem_raw);  // 12 x hs, even slots
  cx<R>* od = ev + 12 * hs;                         // 12 x hs, odd slots
  __shared__ double red[2][3][2];                    // per-wavefront sums, by MR step parity
  int B;
  {
    // K right-hand sides interleaved: consecutive workgroups (same XCD) take
    // the same lattice block for different fields, so its links, clover and
    // odd-site inverses are shared through L2
    const int w = xcd_remap(blockIdx.x, gridDim.x);
    const int pair = w / K, rr = w - pair * K;
    b += (long)rr * ld;
    x += (long)rr * ld;
    int B0 = 2 * pair;
    int bc[4];
    block_coords(g, B0, bc);
    int par = (bc[0] + bc[1] + bc[2] + bc[3]) & 1;
    B = B0 + ((par ^ colour) & 1);
  }
  const int i = threadIdx.x;
  const int se = i, so = g.half + i;
  const int lane = i & 63, wv = i >> 6, nw = (g.half + 63) >> 6;
  SiteNbr me_e, me_o;
  me_of(g, B, se, me_e);
  me_of(g, B, so, me_o);
  cx<R> rho[12], ee[12], tmp[12];
  {
    // r = b - D x with x of this block staged in ev/od
    cx<R> psi[12], ro[12];
    load_spinor(x, g, B, se, psi);
#pragma unroll
    for (int c = 0; c < 12; ++c) *lds_site(ev, g, se, c) = psi[c];
    site_term(H, g, B, se, tw, psi, rho);
    __asm__ volatile("" ::: "memory");
    load_spinor(x, g, B, so, psi);
#pragma unroll
    for (int c = 0; c < 12; ++c) *lds_site(ev, g, so, c) = psi[c];
    site_term(H, g, B, so, tw, psi, ro);
    __syncthreads();
    hop_staged<R, S>(U, x, ev, g, B, se, me_e, rho);
    __asm__ volatile("" ::: "memory");
    hop_staged<R, S>(U, x, ev, g, B, so, me_o, ro);
    load_spinor(b, g, B, se, psi);
#pragma unroll
    for (int c = 0; c < 12; ++c) rho[c] = psi[c] - rho[c];
    load_spinor(b, g, B, so, psi);
#pragma unroll
    for (int c = 0; c < 12; ++c) ro[c] = psi[c] - ro[c];
    __syncthreads();
    __asm__ volatile("" ::: "memory");
    site_inv(H, Minv, g, B, so, tw, ro, tmp);
    load_spinor(x, g, B, so, psi);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      od[c * hs + i] = tmp[c];
      psi[c] += tmp[c];
    }
    store_spinor(x, g, B, so, psi);
    for (int e = i; e < 24; e += g.half) (e < 12 ? ev : od)[(e % 12) * hs + g.half] = mk<R>(0, 0);
  }
  const BlockNbr nb_e = block_nbrs(g, me_e), nb_o = block_nbrs(g, me_o);
  __syncthreads();
  hop_block_lds<R, S, true>(U, g, B, se, nb_e, g.half, od, hs, rho);  // rho = r_e - D_eo t_o
#pragma unroll
  for (int c = 0; c < 12; ++c) ee[c] = mk<R>(0, 0);
  const int nact = min(64, g.half - wv * 64);
  for (int k = 0; k < n_mr; ++k) {
    // the block operator is re-read in every step: keeping the loop-invariant
    // links, clover and inverses in registers would exceed the register file
    __asm__ volatile("" ::: "memory");
#pragma unroll
    for (int c = 0; c < 12; ++c) ev[c * hs + i] = rho[c];
    __syncthreads();
    {  // w = T_oo^{-1} D_oe rho
      cx<R> u[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) u[c] = mk<R>(0, 0);
      hop_block_lds<R, S>(U, g, B, so, nb_o, 0, ev, hs, u);
      site_inv(H, Minv, g, B, so, tw, u, tmp);
#pragma unroll
      for (int c = 0; c < 12; ++c) od[c * hs + i] = tmp[c];
    }
    __syncthreads();
    __asm__ volatile("" ::: "memory");
    // q = T_ee rho - D_eo w
    site_term(H, g, B, se, tw, rho, tmp);
    hop_block_lds<R, S, true>(U, g, B, se, nb_e, g.half, od, hs, tmp);
    double qr_re = 0, qr_im = 0, qq = 0;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      qr_re += (double)tmp[c].re * rho[c].re + (double)tmp[c].im * rho[c].im;
      qr_im += (double)tmp[c].re * rho[c].im - (double)tmp[c].im * rho[c].re;
      qq += (double)tmp[c].re * tmp[c].re + (double)tmp[c].im * tmp[c].im;
    }
    qr_re = wave_sum_n(qr_re, nact);
    qr_im = wave_sum_n(qr_im, nact);
    qq = wave_sum_n(qq, nact);
    if (lane == 0) {
      red[k & 1][0][wv] = qr_re;
      red[k & 1][1][wv] = qr_im;
      red[k & 1][2][wv] = qq;
    }
    __syncthreads();
    double sr = 0, si = 0, sq = 0;
    for (int v = 0; v < nw; ++v) {
      sr += red[k & 1][0][v];
      si += red[k & 1][1][v];
      sq += red[k & 1][2][v];
    }
    cx<R> alpha = mk<R>(0, 0);
    if (sq > 0) alpha = mk<R>((R)(sr / sq), (R)(si / sq));
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      ee[c] += alpha * rho[c];
      rho[c] -= alpha * tmp[c];
    }
  }
#pragma unroll
  for (int c = 0; c < 12; ++c) ev[c * hs + i] = ee[c];
  __syncthreads();
  {  // x_o -= T_oo^{-1} D_oe e_e
    cx<R> u[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) u[c] = mk<R>(0, 0);
    hop_block_lds<R, S>(U, g, B, so, nb_o, 0, ev, hs, u);
    site_inv(H, Minv, g, B, so, tw, u, tmp);
    load_spinor(x, g, B, so, u);
#pragma unroll
    for (int c = 0; c < 12; ++c) u[c] -= tmp[c];
    store_spinor(x, g, B, so, u);
  }
  load_spinor(x, g, B, se, tmp);
#pragma unroll
  for (int c = 0; c < 12; ++c) tmp[c] += ee[c];
  store_spinor(x, g, B, se, tmp);
}

template <class R, class S>
void launch_sap(const Geom& g, int colour, const void* U, const R* H, const R* Minv, Twist tw, const cx<R>* b,
                cx<R>* x, int n_mr, hipStream_t st) {
  launch_sap_multi<R, S>(g, colour, U, H, Minv, tw, b, x, n_mr, 1, 0, st);
}
template <class R, class S>
void launch_sap_multi(const Geom& g, int colour, const void* U, const R* H, const R* Minv, Twist tw, const cx<R>* b,
                      cx<R>* x, int n_mr, int K, long ld, hipStream_t st) {
  size_t sm = 2 * 12 * (size_t)(g.half + 1) * sizeof(cx<R>);
  hipLaunchKernelGGL((k_sap<R, S>), dim3((g.nblocks / 2) * K), dim3(g.half), sm, st, g, colour,
                     (const typename store_traits<S>::elem*)U, H, Minv, TwistR<R>(tw), b, x, n_mr, K, ld);
}
template void launch_sap_multi<double, double>(const Geom&, int, const void*, const double*, const double*, Twist,
                                               const cx<double>*, cx<double>*, int, int, long, hipStream_t);
template void launch_sap_multi<float, float>(const Geom&, int, const void*, const float*, const float*, Twist,
                                             const cx<float>*, cx<float>*, int, int, long, hipStream_t);
template void launch_sap_multi<float, f16>(const Geom&, int, const void*, const float*, const float*, Twist,
                                           const cx<float>*, cx<float>*, int, int, long, hipStream_t);
template void launch_sap_multi<float, bf16>(const Geom&, int, const void*, const float*, const float*, Twist,
                                            const cx<float>*, cx<float>*, int, int, long, hipStream_t);
template void launch_sap<double, double>(const Geom&, int, const void*, const double*, const double*, Twist,
                                         const cx<double>*, cx<double>*, int, hipStream_t);
template void launch_sap<float, float>(const Geom&, int, const void*, const float*, const float*, Twist,
                                       const cx<float>*, cx<float>*, int, hipStream_t);
template void launch_sap<float, f16>(const Geom&, int, const void*, const float*, const float*, Twist,
                                        const cx<float>*, cx<float>*, int, hipStream_t);
template void launch_sap<float, bf16>(const Geom&, int, const void*, const float*, const float*, Twist,
                                                const cx<float>*, cx<float>*, int, hipStream_t);

// ---------------------------------------------------------------------------
// host TZYX lexicographic <-> block layout
template <class R>
__global__ void k_spinor_from_lex(Geom g, const cx<double>* __restrict__ lex, cx<R>* __restrict__ out, int ncomp) {
  long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= g.V) return;
  int B = (int)(gid / g.bs), s = (int)(gid - (long)B * g.bs);
  int x[4];
  site_coords(g, B, s, x);
  long li = lex_index(g, x);
  for (int c = 0; c < ncomp; ++c) {
    cx<double> v = lex[li * ncomp + c];
    out[fidx(g, B, s, ncomp) + (long)c * TILE] = mk<R>((R)v.re, (R)v.im);
  }
}

template <class R>
__global__ void k_spinor_to_lex(Geom g, const cx<R>* __restrict__ in, cx<double>* __restrict__ lex, int ncomp) {
  long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= g.V) return;
  int B = (int)(gid / g.bs), s = (int)(gid - (long)B * g.bs);
  int x[4];
  site_coords(g, B, s, x);
  long li = lex_index(g, x);
  for (int c = 0; c < ncomp; ++c) {
    cx<R> v = in[fidx(g, B, s, ncomp) + (long)c * TILE];
    lex[li * ncomp + c] = mk<double>(v.re, v.im);
  }
}

template <class R>
void launch_from_lex(const Geom& g, const cx<double>* lex, cx<R>* out, int ncomp, hipStream_t st) {
  hipLaunchKernelGGL(k_spinor_from_lex<R>, dim3((g.V + 255) / 256), dim3(256), 0, st, g, lex, out, ncomp);
}
template <class R>
void launch_to_lex(const Geom& g, const cx<R>* in, cx<double>* lex, int ncomp, hipStream_t st) {
  hipLaunchKernelGGL(k_spinor_to_lex<R>, dim3((g.V + 255) / 256), dim3(256), 0, st, g, in, lex, ncomp);
}
template void launch_from_lex<double>(const Geom&, const cx<double>*, cx<double>*, int, hipStream_t);
template void launch_from_lex<float>(const Geom&, const cx<double>*, cx<float>*, int, hipStream_t);
template void launch_to_lex<double>(const Geom&, const cx<double>*, cx<double>*, int, hipStream_t);
template void launch_to_lex<float>(const Geom&, const cx<float>*, cx<double>*, int, hipStream_t);

// ---------------------------------------------------------------------------
// clover term from the links: per site the six F_{mu nu} (mu<nu) from the four
// same-orientation plaquette leaves, then the two chirality blocks
// A_chi = (i c_sw / 2) sum_{mu<nu} sigma^chi_{mu nu} (x) F_{mu nu}; stored as
// H = (m0+4) + A, packed Hermitian.
struct Mat3 {
  cx<double> m[9];
};
__device__ __forceinline__ Mat3 mul(const Mat3& a, const Mat3& b) {
  Mat3 r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      cx<double> acc = mk(0.0, 0.0);
      for (int k = 0; k < 3; ++k) cmac(acc, a.m[3 * i + k], b.m[3 * k + j]);
      r.m[3 * i + j] = acc;
    }
  return r;
}
__device__ __forceinline__ Mat3 dagm(const Mat3& a) {
  Mat3 r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) r.m[3 * i + j] = conj(a.m[3 * j + i]);
  return r;
}

__device__ __forceinline__ Mat3 link_at(const cx<double>* U, const Geom& g, const int x0[4], int d0, int s0, int d1,
                                        int s1, int mu) {
  int x[4] = {x0[0], x0[1], x0[2], x0[3]};
  if (s0) x[d0] = (x[d0] + s0 + g.L[d0]) % g.L[d0];
  if (s1) x[d1] = (x[d1] + s1 + g.L[d1]) % g.L[d1];
  int B, s;
  coords_site(g, x, B, s);
  Mat3 r;
  long base = fidx(g, B, s, 36) + (long)mu * 9 * TILE;
  for (int k = 0; k < 9; ++k) r.m[k] = U[base + (long)k * TILE];
  return r;
}

// sigma^chi_{mu nu} for mu<nu, pair index p (01,02,03,12,13,23), 2x2 per chirality
__constant__ double c_sigma[6][2][4][2];

__global__ void k_clover(Geom g, const cx<double>* __restrict__ U, double csw, double diag, double* __restrict__ H) {
  long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= g.V) return;
  int B = (int)(gid / g.bs), s = (int)(gid - (long)B * g.bs);
  int x[4];
  site_coords(g, B, s, x);
  cx<double> A[2][6][6];
  for (int c = 0; c < 2; ++c)
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) A[c][i][j] = mk(0.0, 0.0);
  int p = 0;
  for (int mu = 0; mu < 4; ++mu)
    for (int nu = mu + 1; nu < 4; ++nu, ++p) {
      Mat3 Umx = link_at(U, g, x, mu, 0, nu, 0, mu), Unx = link_at(U, g, x, mu, 0, nu, 0, nu);
      // leaf 1: U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
      Mat3 Q = mul(mul(Umx, link_at(U, g, x, mu, 1, nu, 0, nu)),
                   mul(dagm(link_at(U, g, x, mu, 0, nu, 1, mu)), dagm(Unx)));
      // leaf 2: U_nu(x) U_mu(x-mu+nu)^dag U_nu(x-mu)^dag U_mu(x-mu)
      Mat3 L2 = mul(mul(Unx, dagm(link_at(U, g, x, mu, -1, nu, 1, mu))),
                    mul(dagm(link_at(U, g, x, mu, -1, nu, 0, nu)), link_at(U, g, x, mu, -1, nu, 0, mu)));
      // leaf 3: U_mu(x-mu)^dag U_nu(x-mu-nu)^dag U_mu(x-mu-nu) U_nu(x-nu)
      Mat3 L3 = mul(mul(dagm(link_at(U, g, x, mu, -1, nu, 0, mu)), dagm(link_at(U, g, x, mu, -1, nu, -1, nu))),
                    mul(link_at(U, g, x, mu, -1, nu, -1, mu), link_at(U, g, x, mu, 0, nu, -1, nu)));
      // leaf 4: U_nu(x-nu)^dag U_mu(x-nu) U_nu(x+mu-nu) U_mu(x)^dag
      Mat3 L4 = mul(mul(dagm(link_at(U, g, x, mu, 0, nu, -1, nu)), link_at(U, g, x, mu, 0, nu, -1, mu)),
                    mul(link_at(U, g, x, mu, 1, nu, -1, nu), dagm(Umx)));
      for (int k = 0; k < 9; ++k) Q.m[k] = Q.m[k] + L2.m[k] + L3.m[k] + L4.m[k];
      // F = (Q - Q^dag)/8;  contribution (i c_sw/2) sigma (x) F
      cx<double> F[9];
      for (int a = 0; a < 3; ++a)
        for (int bb = 0; bb < 3; ++bb) F[3 * a + bb] = 0.125 * (Q.m[3 * a + bb] - conj(Q.m[3 * bb + a]));
      for (int c = 0; c < 2; ++c)
        for (int s1 = 0; s1 < 2; ++s1)
          for (int s2 = 0; s2 < 2; ++s2) {
            cx<double> sg = mk(c_sigma[p][c][2 * s1 + s2][0], c_sigma[p][c][2 * s1 + s2][1]);
            cx<double> f = (0.5 * csw) * times_i(sg);
            for (int a = 0; a < 3; ++a)
              for (int bb = 0; bb < 3; ++bb) A[c][3 * s1 + a][3 * s2 + bb] += f * F[3 * a + bb];
          }
    }
  double* hp = H + fidx(g, B, s, 72);
  for (int c = 0; c < 2; ++c) {
    double* h = hp + 36L * c * TILE;
    for (int i = 0; i < 6; ++i) h[(long)i * TILE] = diag + A[c][i][i].re;
    for (int i = 0; i < 6; ++i)
      for (int j = i + 1; j < 6; ++j) {
        int k = 6 + 2 * herm_idx(i, j);
        cx<double> v = 0.5 * (A[c][i][j] + conj(A[c][j][i]));
        h[(long)k * TILE] = v.re;
        h[(long)(k + 1) * TILE] = v.im;
      }
  }
}

void set_sigma_table(const double* tab /* [6][2][4][2] */) {
  HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(c_sigma), tab, sizeof(double) * 6 * 2 * 4 * 2));
}

void launch_clover(const Geom& g, const cx<double>* U, double csw, double diag, double* H, hipStream_t st) {
  hipLaunchKernelGGL(k_clover, dim3((g.V + 127) / 128), dim3(128), 0, st, g, U, csw, diag, H);
}

// user-supplied clover term [V][2][6][6] (lexicographic) -> packed H = diag + A
__global__ void k_clover_from_lex(Geom g, const cx<double>* __restrict__ lex, double diag, double* __restrict__ H) {
  long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= g.V) return;
  int B = (int)(gid / g.bs), s = (int)(gid - (long)B * g.bs);
  int x[4];
  site_coords(g, B, s, x);
  long li = lex_index(g, x);
  double* hp = H + fidx(g, B, s, 72);
  for (int c = 0; c < 2; ++c) {
    const cx<double>* a = lex + (li * 2 + c) * 36;
    double* h = hp + 36L * c * TILE;
    for (int i = 0; i < 6; ++i) h[(long)i * TILE] = diag + a[6 * i + i].re;
    for (int i = 0; i < 6; ++i)
      for (int j = i + 1; j < 6; ++j) {
        int k = 6 + 2 * herm_idx(i, j);
        cx<double> v = 0.5 * (a[6 * i + j] + conj(a[6 * j + i]));
        h[(long)k * TILE] = v.re;
        h[(long)(k + 1) * TILE] = v.im;
      }
  }
}
void launch_clover_from_lex(const Geom& g, const cx<double>* lex, double diag, double* H, hipStream_t st) {
  hipLaunchKernelGGL(k_clover_from_lex, dim3((g.V + 127) / 128), dim3(128), 0, st, g, lex, diag, H);
}

// packed H (without m0+4) back to [V][2][6][6] lexicographic
__global__ void k_clover_to_lex(Geom g, const double* __restrict__ H, double diag, cx<double>* __restrict__ lex) {
  long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= g.V) return;
  int B = (int)(gid / g.bs), s = (int)(gid - (long)B * g.bs);
  int x[4];
  site_coords(g, B, s, x);
  long li = lex_index(g, x);
  const double* hp = H + fidx(g, B, s, 72);
  for (int c = 0; c < 2; ++c) {
    cx<double>* a = lex + (li * 2 + c) * 36;
    const double* h = hp + 36L * c * TILE;
    for (int i = 0; i < 6; ++i) a[6 * i + i] = mk(h[(long)i * TILE] - diag, 0.0);
    for (int i = 0; i < 6; ++i)
      for (int j = i + 1; j < 6; ++j) {
        int k = 6 + 2 * herm_idx(i, j);
        cx<double> v = mk(h[(long)k * TILE], h[(long)(k + 1) * TILE]);
        a[6 * i + j] = v;
        a[6 * j + i] = conj(v);
      }
  }
}
void launch_clover_to_lex(const Geom& g, const double* H, double diag, cx<double>* lex, hipStream_t st) {
  hipLaunchKernelGGL(k_clover_to_lex, dim3((g.V + 127) / 128), dim3(128), 0, st, g, H, diag, lex);
}

// links [V][4][3][3] lexicographic -> block layout FP64
__global__ void k_links_from_lex(Geom g, const cx<double>* __restrict__ lex, cx<double>* __restrict__ U,
                                 LinkPhases ph) {
  long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= g.V) return;
  int B = (int)(gid / g.bs), s = (int)(gid - (long)B * g.bs);
  int x[4];
  site_coords(g, B, s, x);
  long li = lex_index(g, x);
  for (int mu = 0; mu < 4; ++mu) {
    const bool edge = x[mu] == g.L[mu] - 1;
    const cx<double> f = edge ? mk(ph.re[mu], ph.im[mu]) : mk(1.0, 0.0);
    for (int k = 0; k < 9; ++k) {
      const cx<double> v = lex[(li * 4 + mu) * 9 + k];
      U[fidx(g, B, s, 36) + (long)(mu * 9 + k) * TILE] = edge ? f * v : v;
    }
  }
}
void launch_links_from_lex(const Geom& g, const cx<double>* lex, cx<double>* U, const LinkPhases& ph,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_links_from_lex, dim3((g.V + 255) / 256), dim3(256), 0, st, g, lex, U, ph);
}

// twisted boundary conditions psi(x + L_mu e_mu) = e^{i theta_mu} psi(x) as a
// phase on the links that cross the boundary (forward hop from x_mu = L_mu - 1
// and, through U^dag, the backward hop from x_mu = 0)
__global__ void k_link_phase(Geom g, cx<double>* __restrict__ U, LinkPhases ph) {
  long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= g.V) return;
  int B = (int)(gid / g.bs), s = (int)(gid - (long)B * g.bs);
  int x[4];
  site_coords(g, B, s, x);
  for (int mu = 0; mu < 4; ++mu) {
    if (x[mu] != g.L[mu] - 1) continue;
    const cx<double> f = mk(ph.re[mu], ph.im[mu]);
    for (int k = 0; k < 9; ++k) {
      cx<double>& v = U[fidx(g, B, s, 36) + (long)(mu * 9 + k) * TILE];
      v = f * v;
    }
  }
}
void launch_link_phase(const Geom& g, cx<double>* U, const LinkPhases& ph, hipStream_t st) {
  hipLaunchKernelGGL(k_link_phase, dim3((g.V + 255) / 256), dim3(256), 0, st, g, U, ph);
}

// out += i rho Gamma5 in on the odd sites: the twist of the odd sites raised
// by rho over that of the even sites (FP64 fine fields)
__global__ void k_odd_twist_add(Geom g, const cx<double>* __restrict__ in, cx<double>* __restrict__ out, double rho) {
  long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)g.nblocks * g.half) return;
  int B = (int)(gid / g.half), s = g.half + (int)(gid - (long)B * g.half);
  const long o = fidx(g, B, s, 12);
  for (int c = 0; c < 12; ++c) {
    const double t = c < 6 ? -rho : rho;  // Gamma5 = diag(-1, -1, 1, 1) in spin
    const cx<double> v = in[o + (long)c * TILE];
    cx<double> w = out[o + (long)c * TILE];
    w.re -= t * v.im;
    w.im += t * v.re;
    out[o + (long)c * TILE] = w;
  }
}
void launch_odd_twist_add(const Geom& g, const cx<double>* in, cx<double>* out, double rho, hipStream_t st) {
  const long n = (long)g.nblocks * g.half;
  hipLaunchKernelGGL(k_odd_twist_add, dim3((n + 255) / 256), dim3(256), 0, st, g, in, out, rho);
}

// x = 0 on the even sites (FP64 fine field)
__global__ void k_zero_even(Geom g, cx<double>* __restrict__ x) {
  long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)g.nblocks * g.half) return;
  int B = (int)(gid / g.half), s = (int)(gid - (long)B * g.half);
  const long o = fidx(g, B, s, 12);
  for (int c = 0; c < 12; ++c) x[o + (long)c * TILE] = mk(0.0, 0.0);
}
void launch_zero_even(const Geom& g, cx<double>* x, hipStream_t st) {
  const long n = (long)g.nblocks * g.half;
  hipLaunchKernelGGL(k_zero_even, dim3((n + 255) / 256), dim3(256), 0, st, g, x);
}

// ---------------------------------------------------------------------------
// odd-site inverse factor M_chi = (H_chi^2 + tw^2)^{-1} (Hermitian positive
// definite), by Cholesky; stored packed like H.
__global__ void k_odd_inverse(Geom g, const double* __restrict__ H, double tw, double* __restrict__ M) {
  long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long nodd = (long)g.nblocks * g.half;
  if (gid >= nodd) return;
  int B = (int)(gid / g.half), io = (int)(gid - (long)B * g.half);
  int s = g.half + io;
  const double* hp = H + fidx(g, B, s, 72);
  for (int c = 0; c < 2; ++c) {
    cx<double> h[6][6], G[6][6], L[6][6], Inv[6][6];
    const double* hc = hp + 36L * c * TILE;
    for (int i = 0; i < 6; ++i) h[i][i] = mk(hc[(long)i * TILE], 0.0);
    for (int i = 0; i < 6; ++i)
      for (int j = i + 1; j < 6; ++j) {
        int k = 6 + 2 * herm_idx(i, j);
        h[i][j] = mk(hc[(long)k * TILE], hc[(long)(k + 1) * TILE]);
        h[j][i] = conj(h[i][j]);
      }
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) {
        cx<double> acc = mk(i == j ? tw * tw : 0.0, 0.0);
        for (int k = 0; k < 6; ++k) cmac(acc, h[i][k], h[k][j]);
        G[i][j] = acc;
      }
    // Cholesky G = L L^dag
    for (int j = 0; j < 6; ++j) {
      double d = G[j][j].re;
      for (int k = 0; k < j; ++k) d -= norm2(L[j][k]);
      d = sqrt(d);
      L[j][j] = mk(d, 0.0);
      for (int i = j + 1; i < 6; ++i) {
        cx<double> acc = G[i][j];
        for (int k = 0; k < j; ++k) acc = acc - L[i][k] * conj(L[j][k]);
        L[i][j] = (1.0 / d) * acc;
      }
      for (int i = 0; i < j; ++i) L[i][j] = mk(0.0, 0.0);
    }
    // inverse: solve L L^dag X = I column by column
    for (int col = 0; col < 6; ++col) {
      cx<double> y[6];
      for (int i = 0; i < 6; ++i) {
        cx<double> acc = mk(i == col ? 1.0 : 0.0, 0.0);
        for (int k = 0; k < i; ++k) acc = acc - L[i][k] * y[k];
        y[i] = (1.0 / L[i][i].re) * acc;
      }
      for (int i = 5; i >= 0; --i) {
        cx<double> acc = y[i];
        for (int k = i + 1; k < 6; ++k) acc = acc - conj(L[k][i]) * Inv[k][col];
        Inv[i][col] = (1.0 / L[i][i].re) * acc;
      }
    }
    double* mp = M + oidx(g, B, io, 72) + 36L * c * TILE;
    for (int i = 0; i < 6; ++i) mp[(long)i * TILE] = Inv[i][i].re;
    for (int i = 0; i < 6; ++i)
      for (int j = i + 1; j < 6; ++j) {
        int k = 6 + 2 * herm_idx(i, j);
        cx<double> v = 0.5 * (Inv[i][j] + conj(Inv[j][i]));
        mp[(long)k * TILE] = v.re;
        mp[(long)(k + 1) * TILE] = v.im;
      }
  }
}
void launch_odd_inverse(const Geom& g, const double* H, double tw, double* M, hipStream_t st) {
  long n = (long)g.nblocks * g.half;
  hipLaunchKernelGGL(k_odd_inverse, dim3((n + 127) / 128), dim3(128), 0, st, g, H, tw, M);
}

// ---------------------------------------------------------------------------
// restriction P^dag on the fine level: one workgroup per block (= aggregate),
// one thread per slot; output r_c[site][s*Nv + i].
template <class R>
__global__ void __launch_bounds__(256) k_restrict_fine(Geom g, int Nv, const cx<R>* __restrict__ Q, long vstride,
                                                       const cx<R>* __restrict__ r, const int* __restrict__ f2c,
                                                       cx<R>* __restrict__ rc) {
  __shared__ double red[16][4][2];
  int B = blockIdx.x, s = threadIdx.x;
  int lane = s & 63, wv = s >> 6, nw = (g.bs + 63) >> 6;
  cx<R> rv[12];
  load_spinor(r, g, B, s, rv);
  int site = f2c[B];
  for (int i0 = 0; i0 < Nv; i0 += 8) {
    int ni = min(8, Nv - i0);
    double acc[8][2][2];
    for (int ii = 0; ii < 8; ++ii) {
      acc[ii][0][0] = acc[ii][0][1] = acc[ii][1][0] = acc[ii][1][1] = 0.0;
      if (ii < ni) {
        const cx<R>* q = Q + (long)(i0 + ii) * vstride;
        long base = fidx(g, B, s, 12);
        for (int c = 0; c < 12; ++c) {
          cx<R> qv = q[base + (long)c * TILE];
          int h = c / 6;
          acc[ii][h][0] += (double)qv.re * rv[c].re + (double)qv.im * rv[c].im;
          acc[ii][h][1] += (double)qv.re * rv[c].im - (double)qv.im * rv[c].re;
        }
      }
    }
    for (int ii = 0; ii < 8; ++ii)
      for (int h = 0; h < 2; ++h)
        for (int p = 0; p < 2; ++p) {
          double v = wave_sum_n(acc[ii][h][p], min(64, g.bs - wv * 64));
          if (lane == 0) red[2 * ii + h][wv][p] = v;
        }
    __syncthreads();
    if (s < 2 * ni) {
      int ii = s >> 1, h = s & 1;
      double re = 0, im = 0;
      for (int v = 0; v < nw; ++v) {
        re += red[s][v][0];
        im += red[s][v][1];
      }
      rc[(long)site * 2 * Nv + h * Nv + i0 + ii] = mk<R>((R)re, (R)im);
    }
    __syncthreads();
  }
}

template <class R>
void launch_restrict_fine(const Geom& g, int Nv, const cx<R>* Q, long vstride, const cx<R>* r, const int* f2c,
                          cx<R>* rc, hipStream_t st) {
  hipLaunchKernelGGL(k_restrict_fine<R>, dim3(g.nblocks), dim3(g.bs), 0, st, g, Nv, Q, vstride, r, f2c, rc);
}
template void launch_restrict_fine<double>(const Geom&, int, const cx<double>*, long, const cx<double>*,
                                           const int*, cx<double>*, hipStream_t);
template void launch_restrict_fine<float>(const Geom&, int, const cx<float>*, long, const cx<float>*, const int*,
                                          cx<float>*, hipStream_t);

// prolongation P: x (+)= sum_i Q_i e_c(s(comp)*Nv + i)
template <class R>
__global__ void __launch_bounds__(256) k_prolong_fine(Geom g, int Nv, const cx<R>* __restrict__ Q, long vstride,
                                                      const cx<R>* __restrict__ ec, const int* __restrict__ f2c,
                                                      cx<R>* __restrict__ x, int accumulate) {
  long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= g.V) return;
  int B = (int)(gid / g.bs), s = (int)(gid - (long)B * g.bs);
  const cx<R>* e = ec + (long)f2c[B] * 2 * Nv;
  cx<R> acc[12];
  if (accumulate) load_spinor(x, g, B, s, acc);
  else
    for (int c = 0; c < 12; ++c) acc[c] = mk<R>(0, 0);
  long base = fidx(g, B, s, 12);
  for (int i = 0; i < Nv; ++i) {
    cx<R> e0 = e[i], e1 = e[Nv + i];
    const cx<R>* q = Q + (long)i * vstride + base;
#pragma unroll
    for (int c = 0; c < 6; ++c) cmac(acc[c], q[(long)c * TILE], e0);
#pragma unroll
    for (int c = 6; c < 12; ++c) cmac(acc[c], q[(long)c * TILE], e1);
  }
  store_spinor(x, g, B, s, acc);
}
template <class R>
void launch_prolong_fine(const Geom& g, int Nv, const cx<R>* Q, long vstride, const cx<R>* ec, const int* f2c,
                         cx<R>* x, int accumulate, hipStream_t st) {
  hipLaunchKernelGGL(k_prolong_fine<R>, dim3((g.V + 255) / 256), dim3(256), 0, st, g, Nv, Q, vstride, ec, f2c, x,
                     accumulate);
}
template void launch_prolong_fine<double>(const Geom&, int, const cx<double>*, long, const cx<double>*, const int*,
                                          cx<double>*, int, hipStream_t);
template void launch_prolong_fine<float>(const Geom&, int, const cx<float>*, long, const cx<float>*, const int*,
                                         cx<float>*, int, hipStream_t);

// K-column restriction: one thread per slot (threads past the block's slots
// contribute zero), columns in groups of KC whose inputs stay in registers, test
// vectors in groups of II, so Q is read once per group of columns.  The 4 II KC
// values (vector, column, half, re/im) of a group, padded to a power of two,
// are summed over the wavefront by a transposing butterfly and over the
// wavefronts in LDS in fixed order.
template <int N>
constexpr int pow2_ceil() {
  int p = 1;
  while (p < N) p *= 2;
  return p;
}
template <class R, int KC, int II>
__global__ void __launch_bounds__(256) k_restrict_fine_m(Geom g, int Nv, const cx<R>* __restrict__ Q, long vstride,
                                                         const cx<R>* __restrict__ r, long rld, int K,
                                                         const int* __restrict__ f2c, cx<R>* __restrict__ rc,
                                                         long cld) {
  constexpr int NV0 = 4 * II * KC, NVAL = pow2_ceil<NV0>();
  __shared__ R red[4][NVAL];
  const int B = blockIdx.x, s = threadIdx.x, lane = s & 63, wv = s >> 6, nw = blockDim.x >> 6;
  const bool live = s < g.bs;
  const long site = f2c[B];
  const long base = live ? fidx(g, B, s, 12) : 0;
  for (int k0 = 0; k0 < K; k0 += KC) {
    cx<R> rv[KC][12];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk)
#pragma unroll
      for (int c = 0; c < 12; ++c)
        rv[kk][c] = live && k0 + kk < K ? r[(long)(k0 + kk) * rld + base + (long)c * TILE] : mk<R>(0, 0);
    for (int i0 = 0; i0 < Nv; i0 += II) {
      R acc[NVAL];
#pragma unroll
      for (int v = 0; v < NVAL; ++v) acc[v] = R(0);
#pragma unroll
      for (int ii = 0; ii < II; ++ii) {
        const int i = i0 + ii;
        if (i < Nv && live) {
          cx<R> q[12];
#pragma unroll
          for (int c = 0; c < 12; ++c) q[c] = Q[(long)i * vstride + base + (long)c * TILE];
#pragma unroll
          for (int kk = 0; kk < KC; ++kk)
#pragma unroll
            for (int c = 0; c < 12; ++c) {
              const int v = ((ii * KC + kk) * 2 + c / 6) * 2;
              acc[v] += q[c].re * rv[kk][c].re + q[c].im * rv[kk][c].im;
              acc[v + 1] += q[c].re * rv[kk][c].im - q[c].im * rv[kk][c].re;
            }
        }
      }
      const R tot = wave_transpose_sum<NVAL>(acc, lane);
      if (lane < NVAL) red[wv][lane] = tot;
      __syncthreads();
      if (s < NV0) {
        R sum = R(0);
        for (int w = 0; w < nw; ++w) sum += red[w][s];
        const int p = s & 1, h = (s >> 1) & 1, kk = (s >> 2) % KC, ii = (s >> 2) / KC;
        const int i = i0 + ii, k = k0 + kk;
        if (i < Nv && k < K) reinterpret_cast<R*>(rc + (long)k * cld + site * 2 * Nv + h * Nv + i)[p] = sum;
      }
      __syncthreads();
    }
  }
}
template <class R>
void launch_restrict_fine_m(const Geom& g, int Nv, const cx<R>* Q, long vstride, const cx<R>* r, long rld, int K,
                            const int* f2c, cx<R>* rc, long cld, hipStream_t st) {
  const dim3 grid(g.nblocks), blk(((g.bs + 63) / 64) * 64);
  if (K == 1)
    hipLaunchKernelGGL((k_restrict_fine_m<R, 1, 4>), grid, blk, 0, st, g, Nv, Q, vstride, r, rld, K, f2c, rc, cld);
  else if (K == 2 || sizeof(R) == 8)
    hipLaunchKernelGGL((k_restrict_fine_m<R, 2, 4>), grid, blk, 0, st, g, Nv, Q, vstride, r, rld, K, f2c, rc, cld);
  else if (K == 5 || K == 6)
    hipLaunchKernelGGL((k_restrict_fine_m<R, 6, 1>), grid, blk, 0, st, g, Nv, Q, vstride, r, rld, K, f2c, rc, cld);
  else
    hipLaunchKernelGGL((k_restrict_fine_m<R, 4, 4>), grid, blk, 0, st, g, Nv, Q, vstride, r, rld, K, f2c, rc, cld);
}
template void launch_restrict_fine_m<double>(const Geom&, int, const cx<double>*, long, const cx<double>*, long, int,
                                             const int*, cx<double>*, long, hipStream_t);
template void launch_restrict_fine_m<float>(const Geom&, int, const cx<float>*, long, const cx<float>*, long, int,
                                            const int*, cx<float>*, long, hipStream_t);

// K-column prolongation: x_k (+)= sum_i Q_i e_k, one thread per site, columns in
// groups of KC accumulated in registers (Q read once per group)
template <class R, int KC>
__global__ void __launch_bounds__(256) k_prolong_fine_m(Geom g, int Nv, const cx<R>* __restrict__ Q, long vstride,
                                                        const cx<R>* __restrict__ ec, long cld, int K,
                                                        const int* __restrict__ f2c, cx<R>* __restrict__ x, long xld,
                                                        int accumulate) {
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= g.V) return;
  const int B = (int)(gid / g.bs), s = (int)(gid - (long)B * g.bs);
  const cx<R>* e = ec + (long)f2c[B] * 2 * Nv;
  const long base = fidx(g, B, s, 12);
  for (int k0 = 0; k0 < K; k0 += KC) {
    cx<R> acc[KC][12];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk)
#pragma unroll
      for (int c = 0; c < 12; ++c)
        acc[kk][c] = accumulate && k0 + kk < K ? x[(long)(k0 + kk) * xld + base + (long)c * TILE] : mk<R>(0, 0);
    for (int i = 0; i < Nv; ++i) {
      cx<R> q[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) q[c] = Q[(long)i * vstride + base + (long)c * TILE];
#pragma unroll
      for (int kk = 0; kk < KC; ++kk) {
        if (k0 + kk >= K) continue;
        const cx<R> e0 = e[(long)(k0 + kk) * cld + i], e1 = e[(long)(k0 + kk) * cld + Nv + i];
#pragma unroll
        for (int c = 0; c < 6; ++c) cmac(acc[kk][c], q[c], e0);
#pragma unroll
        for (int c = 6; c < 12; ++c) cmac(acc[kk][c], q[c], e1);
      }
    }
#pragma unroll
    for (int kk = 0; kk < KC; ++kk)
      if (k0 + kk < K)
#pragma unroll
        for (int c = 0; c < 12; ++c) x[(long)(k0 + kk) * xld + base + (long)c * TILE] = acc[kk][c];
  }
}
template <class R>
void launch_prolong_fine_m(const Geom& g, int Nv, const cx<R>* Q, long vstride, const cx<R>* ec, long cld, int K,
                           const int* f2c, cx<R>* x, long xld, int accumulate, hipStream_t st) {
  const dim3 grid((unsigned)((g.V + 255) / 256)), blk(256);
  if (K == 1)
    hipLaunchKernelGGL((k_prolong_fine_m<R, 1>), grid, blk, 0, st, g, Nv, Q, vstride, ec, cld, K, f2c, x, xld, accumulate);
  else if (K == 2 || sizeof(R) == 8)
    hipLaunchKernelGGL((k_prolong_fine_m<R, 2>), grid, blk, 0, st, g, Nv, Q, vstride, ec, cld, K, f2c, x, xld, accumulate);
  else if (K == 5 || K == 6)
    hipLaunchKernelGGL((k_prolong_fine_m<R, 6>), grid, blk, 0, st, g, Nv, Q, vstride, ec, cld, K, f2c, x, xld, accumulate);
  else
    hipLaunchKernelGGL((k_prolong_fine_m<R, 4>), grid, blk, 0, st, g, Nv, Q, vstride, ec, cld, K, f2c, x, xld, accumulate);
}
template void launch_prolong_fine_m<double>(const Geom&, int, const cx<double>*, long, const cx<double>*, long, int,
                                            const int*, cx<double>*, long, int, hipStream_t);
template void launch_prolong_fine_m<float>(const Geom&, int, const cx<float>*, long, const cx<float>*, long, int,
                                           const int*, cx<float>*, long, int, hipStream_t);

// ---------------------------------------------------------------------------
// Galerkin assembly of the first coarse operator on the matrix cores.  One
// workgroup (4 wavefronts) per (block, kind), each kind a sum over a list of
// sites x of rank-6 products
//   C[(i,a),(j,b)] += sum_{c in half a} conj(Q_i(x)_c) Y_(j,b)(x)_c,
// with Y_(j,b) a right factor applied to the chirality-b half of Q_j:
//   kind 0 (self block S, every site):  Y = H(x) P_b Q_j(x)
//   kind 1 (internal links X, every site):
//       Y = sum_{mu: x+mu in block} -1/2 (1-g_mu) U_mu(x) P_b Q_j(x+mu)
//   kind 2+mu (forward block mu, sites on the upper mu face):
//       Y = -1/2 (1-g_mu) U_mu(x) P_b Q_j(x+mu)
// S goes to the self block, X to Xs for the fix-up S += X + Gamma5 X^dag Gamma5
// (k_self_fixup), the face kinds to the forward blocks; output blocks are
// column-major (element (k,l) at l*n + k).
// The complex products run as real ones on 16x16x4 MFMA (FP64 for an FP64 Q,
// FP32 for an FP32 Q): rows (i,a) are padded to 32 per half, wavefront w owning
// half a = w/2 and rows 16(w%2)..+15; the contraction index is (x, c in half a,
// re/im); columns (j,b) go in groups of 16 with a real and an imaginary tile
// (conj(q) y = (q.re y.re + q.im y.im) + i (q.re y.im - q.im y.re)).  CS sites
// at a time are staged in LDS: Q(x) with H(x) or U(x), then Y, built in the
// product's precision by one thread per (site, column).
namespace {
typedef double v4d_a __attribute__((ext_vector_type(4)));
typedef float v4f_a __attribute__((ext_vector_type(4)));
// lane L supplies A[L%16][L/16] and B[L/16][L%16]; element e of the
// accumulator holds D[row(L, e)][L%16], with row = L/16 + 4e for FP64 and
// 4(L/16) + e for FP32 (measured on gfx950)
template <class T> struct mfma_k4;
template <> struct mfma_k4<double> {
  typedef v4d_a acc;
  static __device__ __forceinline__ acc step(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int e) { return (lane >> 4) + 4 * e; }
};
template <> struct mfma_k4<float> {
  typedef v4f_a acc;
  static __device__ __forceinline__ acc step(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int e) { return 4 * (lane >> 4) + e; }
};

// slot of face site f of the upper mu face (the other coordinates in TZYX order)
__device__ __forceinline__ int face_slot(const Geom& g, int mu, int f) {
  int l[4];
  for (int d = 3; d >= 0; --d) {
    if (d == mu) {
      l[d] = g.b[d] - 1;
    } else {
      l[d] = f % g.b[d];
      f /= g.b[d];
    }
  }
  return local_slot(g, l);
}

// y += -1/2 (1-g_MU) U psi, psi = the chirality-HB half p6 of a spinor (other
// half zero), U = up[0..8]; arithmetic in T
template <int MU, int HB, class RQ, class T>
__device__ __forceinline__ void half_hop(const cx<RQ> p6[6], const cx<T>* up, cx<T> y[12]) {
  cx<T> psi[12], u[9];
#pragma unroll
  for (int c = 0; c < 12; ++c) psi[c] = mk<T>(0, 0);
#pragma unroll
  for (int c = 0; c < 6; ++c) psi[6 * HB + c] = mk<T>((T)p6[c].re, (T)p6[c].im);
#pragma unroll
  for (int k = 0; k < 9; ++k) u[k] = up[k];
  hop_accum_t<0, MU>(psi, u, y);
}
template <int MU, class RQ, class T>
__device__ __forceinline__ void half_hop(int hb, const cx<RQ> p6[6], const cx<T>* up, cx<T> y[12]) {
  if (hb) half_hop<MU, 1>(p6, up, y);
  else half_hop<MU, 0>(p6, up, y);
}
}  // namespace

template <class RQ, class T, int CS, int NG>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 2 : 4, 8)))
k_assemble_fine(Geom g, int Nv, const cx<double>* __restrict__ U, const double* __restrict__ H, double dtw,
                const cx<RQ>* __restrict__ Q, long qstride, const int* __restrict__ f2c, cx<double>* __restrict__ Dc,
                cx<double>* __restrict__ Xs) {
  using MF = mfma_k4<T>;
  using acc_t = typename MF::acc;
  constexpr int NC = 16 * NG;         // padded complex columns
  __shared__ cx<T> qs[CS][12][32];    // Q_i(x)_c, rows i padded to 32
  __shared__ cx<T> ys[CS][12][NC];    // Y_col(x)_c
  __shared__ cx<T> us[CS][4][9];      // U_mu(x) (link kinds)
  __shared__ T hs[CS][72];            // H(x) (site kind)
  const int wg = xcd_remap(blockIdx.x, gridDim.x);
  const int B = wg / 6, kind = wg - 6 * (wg / 6);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int n = 2 * Nv;
  const int nsites = kind < 2 ? g.bs : g.bs / g.b[kind - 2];
  int bc[4];
  block_coords(g, B, bc);
  acc_t acc[NG][2];
#pragma unroll
  for (int q = 0; q < NG; ++q) acc[q][0] = acc[q][1] = acc_t{0, 0, 0, 0};

  for (int x0 = 0; x0 < nsites; x0 += CS) {
    // stage Q(x), and H(x) or U(x), of the CS sites (zero past the list and past Nv)
    for (int e = t; e < CS * 12 * 32; e += 256) {
      const int xs = e / 384, r = e - xs * 384, c = r >> 5, i = r & 31;
      cx<T> v = mk<T>(0, 0);
      if (x0 + xs < nsites && i < Nv) {
        const int sx = kind < 2 ? x0 + xs : face_slot(g, kind - 2, x0 + xs);
        const cx<RQ> q = Q[(long)i * qstride + fidx(g, B, sx, 12) + (long)c * TILE];
        v = mk<T>((T)q.re, (T)q.im);
      }
      qs[xs][c][i] = v;
    }
    if (kind == 0) {
      for (int e = t; e < CS * 72; e += 256) {
        const int xs = e / 72, k = e - xs * 72;
        hs[xs][k] = x0 + xs < nsites ? (T)H[fidx(g, B, x0 + xs, 72) + (long)k * TILE] : T(0);
      }
    } else {
      for (int e = t; e < CS * 36; e += 256) {
        const int xs = e / 36, k = e - xs * 36;
        cx<T> v = mk<T>(0, 0);
        if (x0 + xs < nsites) {
          const int sx = kind < 2 ? x0 + xs : face_slot(g, kind - 2, x0 + xs);
          const cx<double> ud = U[fidx(g, B, sx, 36) + (long)k * TILE];
          v = mk<T>((T)ud.re, (T)ud.im);
        }
        us[xs][k / 9][k % 9] = v;
      }
    }
    __syncthreads();
    // right factors: one thread per (site, column)
    for (int it = t; it < CS * NC; it += 256) {
      const int xs = it / NC, col = it - xs * NC;
      cx<T> y[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) y[c] = mk<T>(0, 0);
      if (x0 + xs < nsites && col < n) {
        const int hb = col >= Nv ? 1 : 0, j = col - hb * Nv;
        if (kind == 0) {
          cx<T> psi[6], hy[6];
#pragma unroll
          for (int c = 0; c < 6; ++c) psi[c] = qs[xs][6 * hb + c][j];
          herm_mv(&hs[xs][36 * hb], 1, psi, hy);
          if (dtw != 0) {
            // the parity rest of the twist, i d(x) Gamma5 with d = -+ dtw on
            // even / odd sites (Gamma5 = -1 on chirality 0, +1 on chirality 1)
            const T d = (T)((x0 + xs >= g.half) == (hb == 1) ? dtw : -dtw);
#pragma unroll
            for (int c = 0; c < 6; ++c) hy[c] += mk<T>(-d * psi[c].im, d * psi[c].re);
          }
#pragma unroll
          for (int c = 0; c < 6; ++c) {
            y[c] = hb == 0 ? hy[c] : mk<T>(0, 0);
            y[6 + c] = hb == 0 ? mk<T>(0, 0) : hy[c];
          }
        } else {
          const int sx = kind < 2 ? x0 + xs : face_slot(g, kind - 2, x0 + xs);
          SiteNbr me;
          for (int d = 0; d < 4; ++d) me.bc[d] = bc[d];
          slot_local(g, sx, me.l);
          // every direction loads (from x itself when its link is not taken), so
          // that all gathers are in flight together
          bool take[4];
          long off[4];
#pragma unroll
          for (int mu = 0; mu < 4; ++mu) {
            take[mu] = mu < g.ndir && (kind == 1 ? me.l[mu] + 1 < g.b[mu] : mu == kind - 2);
            int By = B, sy = sx;
            if (take[mu]) nbr_of(g, me, mu, +1, By, sy);
            off[mu] = (long)j * qstride + fidx(g, By, sy, 12) + (long)(6 * hb) * TILE;
          }
          cx<RQ> pv[4][6];
#pragma unroll
          for (int mu = 0; mu < 4; ++mu)
#pragma unroll
            for (int c = 0; c < 6; ++c) pv[mu][c] = Q[off[mu] + (long)c * TILE];
          if (take[0]) half_hop<0>(hb, pv[0], us[xs][0], y);
          if (take[1]) half_hop<1>(hb, pv[1], us[xs][1], y);
          if (take[2]) half_hop<2>(hb, pv[2], us[xs][2], y);
          if (take[3]) half_hop<3>(hb, pv[3], us[xs][3], y);
        }
      }
#pragma unroll
      for (int c = 0; c < 12; ++c) ys[xs][c][col] = y[c];
    }
    __syncthreads();
    {
      const int a = w >> 1, i0 = 16 * (w & 1), r16 = lane & 15, kq = lane >> 4;
#pragma unroll
      for (int xs = 0; xs < CS; ++xs)
#pragma unroll
        for (int s = 0; s < 3; ++s) {
          const int kl = 4 * s + kq, c = 6 * a + (kl >> 1), p = kl & 1;
          const cx<T> qv = qs[xs][c][i0 + r16];
          const T av = p ? qv.im : qv.re;
#pragma unroll
          for (int q = 0; q < NG; ++q) {
            const cx<T> yv = ys[xs][c][16 * q + r16];
            const T bre = p ? yv.im : yv.re;
            const T bim = p ? -yv.re : yv.im;
            acc[q][0] = MF::step(av, bre, acc[q][0]);
            acc[q][1] = MF::step(av, bim, acc[q][1]);
          }
        }
    }
    __syncthreads();
  }
  const long site = f2c[B];
  const long nn = (long)n * n;
  cx<double>* out = kind == 1 ? Xs + site * nn : Dc + (site * 5 + (kind == 0 ? 0 : kind - 1)) * nn;
  const int a = w >> 1, i0 = 16 * (w & 1);
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    const int col = 16 * q + (lane & 15);
    if (col >= n) continue;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = i0 + MF::row(lane, e);
      if (i < Nv) out[(long)col * n + a * Nv + i] = mk<double>(acc[q][0][e], acc[q][1][e]);
    }
  }
}
template <class RQ>
void launch_assemble_fine(const Geom& g, int Nv, const cx<double>* U, const double* H, double dtw, const cx<RQ>* Q,
                          long qstride, const int* f2c, cx<double>* Dc, cx<double>* Xs, hipStream_t st) {
  if (Nv < 1 || Nv > 32) throw Error(INVALID_ARG, "assembly: nvec must be in [1, 32]");
  // The Galerkin products are formed and summed in FP64 on the FP64 matrix
  // cores for both storage formats of the test vectors (FP32 vectors are
  // widened as they are staged).  Sites per stage: LDS of two workgroups per CU.
  using T = double;
  constexpr int CS = 4, CS4 = 3;
  const dim3 grid(6 * g.nblocks), blk(256);
  switch ((2 * Nv + 15) / 16) {
    case 1: hipLaunchKernelGGL((k_assemble_fine<RQ, T, CS, 1>), grid, blk, 0, st, g, Nv, U, H, dtw, Q, qstride, f2c, Dc, Xs); break;
    case 2: hipLaunchKernelGGL((k_assemble_fine<RQ, T, CS, 2>), grid, blk, 0, st, g, Nv, U, H, dtw, Q, qstride, f2c, Dc, Xs); break;
    case 3: hipLaunchKernelGGL((k_assemble_fine<RQ, T, CS, 3>), grid, blk, 0, st, g, Nv, U, H, dtw, Q, qstride, f2c, Dc, Xs); break;
    default: hipLaunchKernelGGL((k_assemble_fine<RQ, T, CS4, 4>), grid, blk, 0, st, g, Nv, U, H, dtw, Q, qstride, f2c, Dc, Xs); break;
  }
}
template void launch_assemble_fine<double>(const Geom&, int, const cx<double>*, const double*, double, const cx<double>*,
                                           long, const int*, cx<double>*, cx<double>*, hipStream_t);
template void launch_assemble_fine<float>(const Geom&, int, const cx<double>*, const double*, double, const cx<float>*,
                                          long, const int*, cx<double>*, cx<double>*, hipStream_t);

// ---------------------------------------------------------------------------
// precision copies of operator data
template <class S>
__global__ void k_cvt_cx(long n, const cx<double>* __restrict__ in, typename store_traits<S>::elem* __restrict__ out) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = st_cvt<S, double>(in[i]);
}
template <class S>
void launch_cvt_cx(long n, const cx<double>* in, void* out, hipStream_t st) {
  hipLaunchKernelGGL(k_cvt_cx<S>, dim3((n + 255) / 256), dim3(256), 0, st, n, in,
                     (typename store_traits<S>::elem*)out);
}
template void launch_cvt_cx<double>(long, const cx<double>*, void*, hipStream_t);
template void launch_cvt_cx<float>(long, const cx<double>*, void*, hipStream_t);
template void launch_cvt_cx<f16>(long, const cx<double>*, void*, hipStream_t);
template void launch_cvt_cx<bf16>(long, const cx<double>*, void*, hipStream_t);

__global__ void k_cvt_real(long n, const double* __restrict__ in, float* __restrict__ out) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}
void launch_cvt_real(long n, const double* in, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_cvt_real, dim3((n + 255) / 256), dim3(256), 0, st, n, in, out);
}

// ---------------------------------------------------------------------------
// Block orthonormalisation per aggregate half (Sec. 1 aggregation): the
// aggregate's rows of v_1..v_Nv are replaced by Q with V = Q R, R upper
// triangular with a real positive diagonal; that factor is unique, so it is the
// one Gram-Schmidt in the order v_1..v_Nv produces.  It is computed as a
// Cholesky QR in FP64: G = V^H V on the matrix cores, G = R^H R in LDS, then
// Q = V R^{-1} on the matrix cores.  The loss of orthogonality of one pass
// grows like eps64 cond(V)^2: an FP64 output always takes a second pass on Q,
// an FP32 output when the aggregate's smallest pivot ratio R_kk^2 / |v_k|^2 is
// below 1e-6.  A pivot ratio at or below 1e-14 (|R_kk| <= 1e-7 |v_k|, where
// the FP64 Gram matrix no longer resolves the column: linearly dependent test
// vectors) sets *fail.
//
// One workgroup (4 wavefronts) per (block, half); rows r of the aggregate are
// (tile of 8 slots, component of the half, slot in the tile), so 8 consecutive
// rows are contiguous in the block layout.  Nv <= 32 (two 16-wide tiles).
namespace {
constexpr int QR_NT = 256;

__device__ __forceinline__ long qr_row_addr(const Geom& g, int B, int h, int r) {
  const int tau = r / 48, rem = r - 48 * tau, c = rem >> 3, sig = rem & 7;
  return ((long)B * (g.bs / TILE) + tau) * 12 * TILE + (long)(6 * h + c) * TILE + sig;
}

template <class T>
__device__ __forceinline__ cx<double> qr_ld(const cx<T>* p, long stride, int j, int Nv, long a) {
  if (j >= Nv) return mk<double>(0, 0);
  cx<T> v = p[(long)j * stride + a];
  return mk<double>((double)v.re, (double)v.im);
}

// one Cholesky QR pass: src (rows of this aggregate) -> dst; Gr/Gi/Xr/Xi/d0 in LDS
template <class TS, class TD>
__device__ __forceinline__ void cholqr_pass(const Geom& g, int B, int h, int Nv, const cx<TS>* src, long sstride, cx<TD>* dst,
                            long dstride, double (*Gr)[33], double (*Gi)[33], double (*Xr)[33], double (*Xi)[33],
                            double* d0, int* fail, double* ratio) {
  using MF = mfma_k4<double>;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int rows = 6 * g.bs;
  const int NT = Nv > 16 ? 2 : 1;
  const int j0 = lane & 15, kq = lane >> 4, p = kq & 1;
  // ---- G = V^H V: wavefront w sums the complex row pairs ks = w, w+4, ...
  MF::acc a00r = {0, 0, 0, 0}, a00i = {0, 0, 0, 0}, a01r = {0, 0, 0, 0}, a01i = {0, 0, 0, 0}, a11r = {0, 0, 0, 0},
          a11i = {0, 0, 0, 0};
#pragma unroll 4
  for (int ks = w; ks < rows / 2; ks += 4) {
    const long a = qr_row_addr(g, B, h, 2 * ks + (kq >> 1));
    const cx<double> v0 = qr_ld(src, sstride, j0, Nv, a);
    const double x0 = p ? v0.im : v0.re, y0 = p ? -v0.re : v0.im;
    a00r = MF::step(x0, x0, a00r);
    a00i = MF::step(x0, y0, a00i);
    if (NT == 2) {
      const cx<double> v1 = qr_ld(src, sstride, 16 + j0, Nv, a);
      const double x1 = p ? v1.im : v1.re, y1 = p ? -v1.re : v1.im;
      a01r = MF::step(x0, x1, a01r);
      a01i = MF::step(x0, y1, a01i);
      a11r = MF::step(x1, x1, a11r);
      a11i = MF::step(x1, y1, a11i);
    }
  }
  // deterministic sum over the 4 wavefronts, in wavefront order
  for (int v = 0; v < 4; ++v) {
    if (w == v) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = MF::row(lane, e), c = j0;
        Gr[r][c] = (v ? Gr[r][c] : 0.0) + a00r[e];
        Gi[r][c] = (v ? Gi[r][c] : 0.0) + a00i[e];
        if (NT == 2) {
          Gr[r][16 + c] = (v ? Gr[r][16 + c] : 0.0) + a01r[e];
          Gi[r][16 + c] = (v ? Gi[r][16 + c] : 0.0) + a01i[e];
          Gr[16 + r][16 + c] = (v ? Gr[16 + r][16 + c] : 0.0) + a11r[e];
          Gi[16 + r][16 + c] = (v ? Gi[16 + r][16 + c] : 0.0) + a11i[e];
        }
      }
    }
    __syncthreads();
  }
  if (t < Nv) d0[t] = Gr[t][t];
  __syncthreads();
  // ---- G = R^H R in place on the upper triangle (R[k][k] real)
  double rmin = 1.0;  // smallest pivot ratio (thread 0)
  for (int k = 0; k < Nv; ++k) {
    const double dk = Gr[k][k];
    const double rkk = dk > 0 ? sqrt(dk) : 0.0, rinv = rkk > 0 ? 1.0 / rkk : 0.0;
    __syncthreads();
    if (t == 0) {
      const double rk = d0[k] > 0 ? dk / d0[k] : 0.0;
      rmin = rk < rmin ? rk : rmin;
      if (fail && !(rk > 1e-14)) atomicOr(fail, 1);
      Gr[k][k] = rkk;
      Gi[k][k] = 0.0;
    } else if (t > k && t < Nv) {
      Gr[k][t] *= rinv;
      Gi[k][t] *= rinv;
    }
    __syncthreads();
    for (int q = t; q < 32 * 32; q += QR_NT) {
      const int j = q >> 5, l = q & 31;
      if (j > k && l >= j && l < Nv) {
        // G[j][l] -= conj(R[k][j]) R[k][l]
        const double ar = Gr[k][j], ai = Gi[k][j], br = Gr[k][l], bi = Gi[k][l];
        Gr[j][l] -= ar * br + ai * bi;
        Gi[j][l] -= ar * bi - ai * br;
      }
    }
    __syncthreads();
  }
  if (t == 0) *ratio = rmin;
  // ---- X = R^{-1} (upper), one thread per column; zero elsewhere (padding)
  for (int q = t; q < 32 * 32; q += QR_NT) {
    Xr[q >> 5][q & 31] = 0.0;
    Xi[q >> 5][q & 31] = 0.0;
  }
  __syncthreads();
  if (t < Nv) {
    const int i = t;
    Xr[i][i] = Gr[i][i] > 0 ? 1.0 / Gr[i][i] : 0.0;
    for (int j = i - 1; j >= 0; --j) {
      double sr = 0, si = 0;
      for (int m = j + 1; m <= i; ++m) {
        const double ar = Gr[j][m], ai = Gi[j][m], xr = Xr[m][i], xi = Xi[m][i];
        sr += ar * xr - ai * xi;
        si += ar * xi + ai * xr;
      }
      const double ri = Gr[j][j] > 0 ? 1.0 / Gr[j][j] : 0.0;
      Xr[j][i] = -sr * ri;
      Xi[j][i] = -si * ri;
    }
  }
  __syncthreads();
  // ---- Q = V X: wavefront w takes row tiles w, w+4, ...; contraction over (j, re/im)
  const int nks = (Nv + 1) / 2;
  for (int rt = w; rt < rows / 16; rt += 4) {
    const long a = qr_row_addr(g, B, h, 16 * rt + j0);
    MF::acc q0r = {0, 0, 0, 0}, q0i = {0, 0, 0, 0}, q1r = {0, 0, 0, 0}, q1i = {0, 0, 0, 0};
    for (int ks = 0; ks < nks; ++ks) {
      const int j = 2 * ks + (kq >> 1);
      const cx<double> v = qr_ld(src, sstride, j, Nv, a);
      const double av = p ? v.im : v.re;
      const int jj = j < 32 ? j : 31;
      double xr = Xr[jj][j0], xi = Xi[jj][j0];
      q0r = MF::step(av, p ? -xi : xr, q0r);
      q0i = MF::step(av, p ? xr : xi, q0i);
      if (NT == 2) {
        xr = Xr[jj][16 + j0];
        xi = Xi[jj][16 + j0];
        q1r = MF::step(av, p ? -xi : xr, q1r);
        q1i = MF::step(av, p ? xr : xi, q1i);
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const long ar = qr_row_addr(g, B, h, 16 * rt + MF::row(lane, e));
      if (j0 < Nv) dst[(long)j0 * dstride + ar] = mk<TD>((TD)q0r[e], (TD)q0i[e]);
      if (NT == 2 && 16 + j0 < Nv) dst[(long)(16 + j0) * dstride + ar] = mk<TD>((TD)q1r[e], (TD)q1i[e]);
    }
  }
  __syncthreads();
}
}  // namespace

template <class RI, class RO>
__global__ void __launch_bounds__(QR_NT) __attribute__((amdgpu_waves_per_eu(3, 8))) k_qr_fine(Geom g, int Nv, const cx<RI>* V, long vstride, RO* Qout_raw,
                                                   long qstride, int* __restrict__ fail) {
  __shared__ double Gr[32][33], Gi[32][33], Xr[32][33], Xi[32][33], d0[32], ratio;
  cx<RO>* Q = reinterpret_cast<cx<RO>*>(Qout_raw);
  const int B = blockIdx.x >> 1, h = blockIdx.x & 1;
  static_assert(std::is_same<RI, RO>::value, "both passes share one body");
  // pass 0 on V; pass 1 on Q for an FP64 output or an ill-conditioned aggregate
  // (ratio is an LDS value after a barrier: uniform over the workgroup)
#pragma unroll 1
  for (int pass = 0; pass < 2; ++pass) {
    cholqr_pass<RI, RO>(g, B, h, Nv, pass == 0 ? V : reinterpret_cast<const cx<RI>*>(Q),
                        pass == 0 ? vstride : qstride, Q, qstride, Gr, Gi, Xr, Xi, d0, pass == 0 ? fail : nullptr,
                        &ratio);
    if (!(sizeof(RO) == 8 || ratio < 1e-6)) break;
  }
}
template <class RI, class RO>
void launch_qr_fine(const Geom& g, int Nv, const cx<RI>* V, long vstride, cx<RO>* Q, long qstride, int* fail,
                    hipStream_t st) {
  if (Nv < 1 || Nv > 32 || g.bs % TILE) throw Error(INVALID_ARG, "block orthonormalisation needs 1 <= Nv <= 32");
  hipLaunchKernelGGL((k_qr_fine<RI, RO>), dim3(2 * g.nblocks), dim3(QR_NT), 0, st, g, Nv, V, vstride, (RO*)Q, qstride,
                     fail);
}
template void launch_qr_fine<double, double>(const Geom&, int, const cx<double>*, long, cx<double>*, long, int*,
                                             hipStream_t);
template void launch_qr_fine<float, float>(const Geom&, int, const cx<float>*, long, cx<float>*, long, int*,
                                           hipStream_t);

}  // namespace ddamg
