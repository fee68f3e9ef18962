// Device helpers of the fine lattice shared by the operator, smoother,
// transfer and network kernels: spin projection of the Wilson hops, site
// loads and stores in the tiled block layout, packed Hermitian 6x6 blocks,
// neighbour lookup.
#pragma once
#include "kernels.hpp"

namespace ddamg {

// phase codes: 0:+1 1:+i 2:-1 3:-i
template <int K, class R>
__device__ __forceinline__ cx<R> ph(cx<R> a) {
  if constexpr (K == 0) return a;
  else if constexpr (K == 1) return times_i(a);
  else if constexpr (K == 2) return -a;
  else return times_mi(a);
}

// Spin-projection tables for -1/2 (1 -+ g_mu): h0 = psi0 + a0 psi_p0,
// h1 = psi1 + a1 psi_p1;  out0 -= h0'/2, out1 -= h1'/2, out2 += c2/2 * h_q2',
// out3 += c3/2 * h_q3'  (h' = U h forward, U^dag h backward).
struct ProjT {
  int a0, p0, a1, p1, c2, q2, c3, q3;
};
__host__ __device__ constexpr ProjT proj_tab(int bwd, int mu) {
  constexpr ProjT t[2][4] = {
      {{0, 2, 0, 3, 2, 0, 2, 1}, {1, 2, 3, 3, 1, 0, 3, 1}, {0, 3, 2, 2, 0, 1, 2, 0}, {1, 3, 1, 2, 1, 1, 1, 0}},
      {{2, 2, 2, 3, 0, 0, 0, 1}, {3, 2, 1, 3, 3, 0, 1, 1}, {2, 3, 0, 2, 2, 1, 0, 0}, {3, 3, 3, 2, 3, 1, 3, 0}}};
  return t[bwd][mu];
}

// accumulate -1/2 (1 -+ g_mu) W psi into out (W = U forward, U^dag backward)
template <int BWD, int MU, class R>
__device__ __forceinline__ void hop_accum_t(const cx<R> psi[12], const cx<R> u[9], cx<R> out[12]) {
  constexpr ProjT t = proj_tab(BWD, MU);
  cx<R> h[2][3], w[2][3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    h[0][c] = psi[c] + ph<t.a0>(psi[3 * t.p0 + c]);
    h[1][c] = psi[3 + c] + ph<t.a1>(psi[3 * t.p1 + c]);
  }
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<R> acc = mk<R>(0, 0);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        if constexpr (BWD) cjmac(acc, u[3 * b + a], h[s][b]);
        else cmac(acc, u[3 * a + b], h[s][b]);
      }
      w[s][a] = acc;
    }
  const R hf = R(0.5);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    out[a] -= hf * w[0][a];
    out[3 + a] -= hf * w[1][a];
    out[6 + a] += hf * ph<t.c2>(w[t.q2][a]);
    out[9 + a] += hf * ph<t.c3>(w[t.q3][a]);
  }
}

template <int BWD, class R>
__device__ __forceinline__ void hop_accum(int mu, const cx<R> psi[12], const cx<R> u[9], cx<R> out[12]) {
  switch (mu) {
    case 0: hop_accum_t<BWD, 0>(psi, u, out); break;
    case 1: hop_accum_t<BWD, 1>(psi, u, out); break;
    case 2: hop_accum_t<BWD, 2>(psi, u, out); break;
    default: hop_accum_t<BWD, 3>(psi, u, out); break;
  }
}

template <class R, class S>
__device__ __forceinline__ void load_link(const typename store_traits<S>::elem* U, const Geom& g, int B, int s, int mu,
                                          cx<R> u[9]) {
  long base = fidx(g, B, s, 36) + (long)mu * 9 * TILE;
#pragma unroll
  for (int k = 0; k < 9; ++k) u[k] = ld<R, S>(U, base + (long)k * TILE);
}

template <class R>
__device__ __forceinline__ void load_spinor(const cx<R>* f, const Geom& g, int B, int s, cx<R> p[12]) {
  long base = fidx(g, B, s, 12);
#pragma unroll
  for (int c = 0; c < 12; ++c) p[c] = f[base + (long)c * TILE];
}

template <class R>
__device__ __forceinline__ void store_spinor(cx<R>* f, const Geom& g, int B, int s, const cx<R> p[12]) {
  long base = fidx(g, B, s, 12);
#pragma unroll
  for (int c = 0; c < 12; ++c) f[base + (long)c * TILE] = p[c];
}

// packed Hermitian 6x6: 6 real diagonal entries, then the 15 upper entries
// (i<j, row-major) as (re,im) pairs
__host__ __device__ __forceinline__ int herm_idx(int i, int j) { return 5 * i - (i * (i - 1)) / 2 + (j - i - 1); }

template <class R>
__device__ __forceinline__ void herm_mv(const R* hp, long stride, const cx<R> x[6], cx<R> y[6]) {
  // streams the packed entries once: y_i += H_ij x_j and y_j += conj(H_ij) x_i
#pragma unroll
  for (int i = 0; i < 6; ++i) y[i] = hp[(long)i * stride] * x[i];
  int k = 6;
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = i + 1; j < 6; ++j) {
      cx<R> h = mk<R>(hp[(long)k * stride], hp[(long)(k + 1) * stride]);
      k += 2;
      cmac(y[i], h, x[j]);
      cjmac(y[j], h, x[i]);
    }
}

// T psi at (B,s): (m0+4+A) psi + i tw gamma5 psi, tw the twist of the slot's parity
template <class R>
__device__ __forceinline__ void site_term(const R* H, const Geom& g, int B, int s, TwistR<R> twp,
                                          const cx<R> psi[12], cx<R> out[12]) {
  const R tw = s < g.half ? twp.e : twp.o;
  const R* hp = H + fidx(g, B, s, 72);
  herm_mv(hp, TILE, psi, out);
  herm_mv(hp + 36L * TILE, TILE, psi + 6, out + 6);
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    out[c] += tw * times_mi(psi[c]);
    out[6 + c] += tw * times_i(psi[6 + c]);
  }
}

// T^{-1} psi on an odd slot: per chirality (H -+ i tw) M psi with M = (H^2+tw^2)^{-1}
// (H is Hermitian, so (H + i a)^{-1} = (H - i a)(H^2 + a^2)^{-1}); chirality 0 has
// the twist -i tw, chirality 1 +i tw.
template <class R>
__device__ __forceinline__ void site_inv(const R* H, const R* Minv, const Geom& g, int B, int s, TwistR<R> twp,
                                         const cx<R> psi[12], cx<R> out[12]) {
  const R tw = twp.o;
  const R* hp = H + fidx(g, B, s, 72);
  const R* mp = Minv + oidx(g, B, s - g.half, 72);
  cx<R> t[12];
  herm_mv(mp, TILE, psi, t);
  herm_mv(mp + 36L * TILE, TILE, psi + 6, t + 6);
  herm_mv(hp, TILE, t, out);
  herm_mv(hp + 36L * TILE, TILE, t + 6, out + 6);
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    out[c] += tw * times_i(t[c]);
    out[6 + c] += tw * times_mi(t[6 + c]);
  }
}

struct SiteNbr {
  int bc[4], l[4];
};

__device__ __forceinline__ void nbr_of(const Geom& g, const SiteNbr& sn, int mu, int dir, int& Bn, int& snb) {
  int bc[4] = {sn.bc[0], sn.bc[1], sn.bc[2], sn.bc[3]};
  int l[4] = {sn.l[0], sn.l[1], sn.l[2], sn.l[3]};
  l[mu] += dir;
  if (l[mu] == g.b[mu]) {
    l[mu] = 0;
    bc[mu] = (bc[mu] + 1 == g.nb[mu]) ? 0 : bc[mu] + 1;
  } else if (l[mu] < 0) {
    l[mu] = g.b[mu] - 1;
    bc[mu] = (bc[mu] == 0) ? g.nb[mu] - 1 : bc[mu] - 1;
  }
  Bn = block_index(g, bc);
  snb = local_slot(g, l);
}

// Spinors of one block staged in LDS, parity-split: component c of slot s sits
// at lds[(p * 12 + c) * half + (s - p * half)], p = parity of s.
template <class R>
__device__ __forceinline__ cx<R>* lds_site(cx<R>* lds, const Geom& g, int s, int c) {
  int p = s >= g.half ? 1 : 0;
  return lds + (long)(p * 12 + c) * g.half + (s - p * g.half);
}

template <class R>
__device__ __forceinline__ void load_nbr_staged(const cx<R>* in, const cx<R>* lds, const Geom& g, int B, int Bn, int sn,
                                                cx<R> p[12]) {
  if (Bn == B) {
    int par = sn >= g.half ? 1 : 0;
    const cx<R>* q = lds + (long)par * 12 * g.half + (sn - par * g.half);
#pragma unroll
    for (int c = 0; c < 12; ++c) p[c] = q[(long)c * g.half];
  } else {
    load_spinor(in, g, Bn, sn, p);
  }
}

// hopping part of D at (B,s) with the neighbours inside block B read from the
// block's staged copy in LDS and the others from global memory
template <int MU, class R, class S>
__device__ __forceinline__ void hop_staged_dir(const typename store_traits<S>::elem* U, const cx<R>* in,
                                               const cx<R>* lds, const Geom& g, int B, int s, const SiteNbr& me,
                                               cx<R> out[12]) {
  cx<R> psi[12], u[9];
  int Bn, sn;
  nbr_of(g, me, MU, +1, Bn, sn);
  load_nbr_staged(in, lds, g, B, Bn, sn, psi);
  load_link<R, S>(U, g, B, s, MU, u);
  hop_accum_t<0, MU>(psi, u, out);
  nbr_of(g, me, MU, -1, Bn, sn);
  load_nbr_staged(in, lds, g, B, Bn, sn, psi);
  load_link<R, S>(U, g, Bn, sn, MU, u);
  hop_accum_t<1, MU>(psi, u, out);
}

template <class R, class S>
__device__ __forceinline__ void hop_staged(const typename store_traits<S>::elem* U, const cx<R>* in, const cx<R>* lds,
                                           const Geom& g, int B, int s, const SiteNbr& me, cx<R> out[12]) {
#pragma unroll 1
  for (int mu = 0; mu < g.ndir; ++mu) {
    switch (mu) {
      case 0: hop_staged_dir<0, R, S>(U, in, lds, g, B, s, me, out); break;
      case 1: hop_staged_dir<1, R, S>(U, in, lds, g, B, s, me, out); break;
      case 2: hop_staged_dir<2, R, S>(U, in, lds, g, B, s, me, out); break;
      default: hop_staged_dir<3, R, S>(U, in, lds, g, B, s, me, out); break;
    }
  }
}

__device__ __forceinline__ void me_of(const Geom& g, int B, int s, SiteNbr& me) {
  block_coords(g, B, me.bc);
  slot_local(g, s, me.l);
}

}  // namespace ddamg
