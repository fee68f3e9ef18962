// Gauge-covariant parallel-transport network that proposes the initial test
// vectors of the adaptive setup (the paper's setup starts from random vectors,
// Sec. 1; the plain setup stays the fallback).  FP32 VALU kernels:
//
//   layer  z_c(x) = sum_{d=0..8} sum_{c'} W_{d,c,c'} (T_d x_{c'})(x)
//          T_0 = 1, T_{+mu} x(x) = U_mu(x) x(x+mu), T_{-mu} x(x) = U_mu(x-mu)^dag x(x-mu)
//          W_{d,c,c'}: 4x4 complex spin matrix (gauge covariant, no bias)
//   gate   y_c(x) = z_c(x) sigmoid(a_c |z_c(x)|^2 + b_c)   (all layers but the last)
//   loss   L = sum_{aggregate halves} |(I - Pi_Y) Q*|_F^2 / sum |Q*|_F^2
//
// Offsets d: 0 identity, 1..4 forward T,Z,Y,X, 5..8 backward.  The adjoint
// of T_{+mu} is T_{-mu} and vice versa, and W acts on spin while T acts on
// colour and position, so the input gradient sum_d T_d^dag W_d^dag G_z has the
// same structure as the forward layer: the same kernel runs it with swapped
// offsets and conjugate-transposed weights.
//
// Fields: C channels, each a fine field in the tiled block layout (FP32),
// channel c at offset c * V * 12.  Weights W[l]: [9][C][C][4][4] complex.
#include "finedev.hpp"

namespace ddamg {

// T_d x at (B,s), colour transport only (all four spins)
__device__ __forceinline__ void transport_site(const Geom& g, const cx<float>* U, const cx<float>* x, int d, int B,
                                               int s, cx<float> out[12]) {
  if (d == 0) {
    load_spinor(x, g, B, s, out);
    return;
  }
  SiteNbr me;
  me_of(g, B, s, me);
  const int mu = (d - 1) & 3;
  const bool fwd = d <= 4;
  int Bn, sn;
  nbr_of(g, me, mu, fwd ? 1 : -1, Bn, sn);
  cx<float> psi[12], u[9];
  load_spinor(x, g, Bn, sn, psi);
  if (fwd) load_link<float, float>(U, g, B, s, mu, u);
  else load_link<float, float>(U, g, Bn, sn, mu, u);
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx<float> acc = mk<float>(0, 0);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        if (fwd) cmac(acc, u[3 * a + b], psi[3 * sp + b]);
        else cjmac(acc, u[3 * b + a], psi[3 * sp + b]);
      }
      out[3 * sp + a] = acc;
    }
}

// ---------------------------------------------------------------------------
// mixing layer: 64 sites per workgroup, wave w computes output channels
// [w*CW, (w+1)*CW) (C = 4*CW); transported inputs staged in LDS 8 channels
// at a time; the weights are wave-uniform (scalar loads).
template <int CW, bool ADJ>
__global__ void __launch_bounds__(256) k_net_mix(Geom g, const cx<float>* __restrict__ U,
                                                 const cx<float>* __restrict__ in, const cx<float>* __restrict__ W,
                                                 cx<float>* __restrict__ out) {
  constexpr int C = 4 * CW;
  __shared__ cx<float> txs[8][12][64];
  const int t = threadIdx.x, lane = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  const long fl = g.V * 12;
  const long gsite = (long)blockIdx.x * 64 + lane;
  const int B = (int)(gsite / g.bs), s = (int)(gsite - (long)B * g.bs);
  cx<float> acc[CW][4][3];
#pragma unroll
  for (int cc = 0; cc < CW; ++cc)
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int k = 0; k < 3; ++k) acc[cc][sp][k] = mk<float>(0, 0);
#pragma unroll 1
  for (int d = 0; d < 9; ++d) {
    // the adjoint swaps forward and backward offsets
    const int dt = ADJ ? (d == 0 ? 0 : (d <= 4 ? d + 4 : d - 4)) : d;
#pragma unroll 1
    for (int k0 = 0; k0 < C; k0 += 8) {
      const int nch = min(8, C - k0);
      __syncthreads();
      for (int p = t; p < 64 * 8; p += 256) {
        int i = p & 63, ch = p >> 6;
        if (ch < nch) {
          long gs = (long)blockIdx.x * 64 + i;
          int Bi = (int)(gs / g.bs), si = (int)(gs - (long)Bi * g.bs);
          cx<float> v[12];
          transport_site(g, U, in + (long)(k0 + ch) * fl, dt, Bi, si, v);
#pragma unroll
          for (int c = 0; c < 12; ++c) txs[ch][c][i] = v[c];
        }
      }
      __syncthreads();
      for (int ch = 0; ch < nch; ++ch) {
        const int ci = k0 + ch;
#pragma unroll
        for (int sq = 0; sq < 4; ++sq) {
          cx<float> v[3];
#pragma unroll
          for (int k = 0; k < 3; ++k) v[k] = txs[ch][3 * sq + k][lane];
#pragma unroll
          for (int cc = 0; cc < CW; ++cc) {
            const int co = w * CW + cc;
#pragma unroll
            for (int sp = 0; sp < 4; ++sp) {
              cx<float> wv;
              if (ADJ) wv = conj(W[((long)(d * C + ci) * C + co) * 16 + sq * 4 + sp]);
              else wv = W[((long)(d * C + co) * C + ci) * 16 + sp * 4 + sq];
#pragma unroll
              for (int k = 0; k < 3; ++k) cmac(acc[cc][sp][k], wv, v[k]);
            }
          }
        }
      }
    }
  }
  const long base = fidx(g, B, s, 12);
#pragma unroll
  for (int cc = 0; cc < CW; ++cc) {
    cx<float>* o = out + (long)(w * CW + cc) * fl + base;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int k = 0; k < 3; ++k) o[(long)(3 * sp + k) * TILE] = acc[cc][sp][k];
  }
}

// ---------------------------------------------------------------------------
// The mixing layer on the matrix cores (inference).  Per site and colour k the
// layer is z[(c,s)] = sum_{(d,c',t)} W[d][c][c'][s][t] (T_d x_{c'})[t][k]: a
// complex matrix of 4C rows (c,s) and 9*4C columns (d,c',t) times one column
// per (site, colour).  It runs as a real product with the embedding
//   A[i][(l,0)] = Re W_il, A[i][(l,1)] = Im W_il,
//   B[(l,0)][(col,0)] = Re v, B[(l,1)][(col,0)] = -Im v, B[(l,0)][(col,1)] = Im v,
//   B[(l,1)][(col,1)] = Re v.
// FP32 accuracy on the BF16 matrix cores: every FP32 operand x is split into
// three BF16 parts x = x0 + x1 + x2 (x0 = bf16(x), x1 = bf16(x - x0),
// x2 = bf16(x - x0 - x1), 24 significant bits together), and a*b is summed as
// the six products a_i b_j with i + j <= 2; the dropped terms are below
// 2^-24 |a b|, the products are exact in FP32 and the sums are FP32 (the
// same rounding level as the FP32 VALU kernel, in another order).  That is
// six v_mfma_f32_16x16x32_bf16 per 32 inner terms against eight
// v_mfma_f32_16x16x4f32 for the same terms in FP32, at 16 times the rate.
// Fragments (wave64): lane L holds A[L%16][8(L/16) + e] and B[8(L/16) + e][L%16]
// (e < 8); the result D[4(L/16) + e][L%16] (e < 4).
// A workgroup takes 64 sites, wavefront w sites 16w..16w+15 (96 real columns:
// 6 tiles, each one colour and 8 consecutive sites); the transported inputs of
// 8 channels of one offset are staged in LDS per chunk as in the VALU kernel.  The weights are split and packed once
// per layer in fragment order (k_net_pack): one 16 B load per A fragment part.
typedef float v4f_n __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf_n __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void split3(float x, __bf16& x0, __bf16& x1, __bf16& x2) {
  x0 = (__bf16)x;
  const float r = x - (float)x0;
  x1 = (__bf16)r;
  x2 = (__bf16)(r - (float)x1);
}

// packed[(((chunk * 2 + ks) * RT + t) * 3 + part) * 64 + lane][e] (BF16),
// chunk = d * (C/8) + k0/8; entry = part `part` of A[16t + lane%16][32 ks + 8 (lane/16) + e]
__global__ void k_net_pack(int C, const cx<float>* __restrict__ W, __bf16* __restrict__ P) {
  const int RT = C / 4, nch = C / 8;
  const long total = 9L * nch * 2 * RT * 3 * 64 * 8;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int e8 = (int)(e & 7);
    const int lane = (int)((e >> 3) & 63);
    long r = e >> 9;
    const int part = (int)(r % 3);
    r /= 3;
    const int t = (int)(r % RT);
    r /= RT;
    const int ks = (int)(r & 1);
    const int chunk = (int)(r >> 1);
    const int d = chunk / nch, k0 = (chunk % nch) * 8;
    const int i = 16 * t + (lane & 15);               // row (c, s)
    const int q = 32 * ks + 8 * (lane >> 4) + e8;      // real inner index in the chunk
    const int l = q >> 1, cp = q & 1;                  // complex inner (c', t), part
    const int ci = k0 + (l >> 2), tt = l & 3;
    const int co = i >> 2, sp = i & 3;
    const cx<float> w = W[((long)(d * C + co) * C + ci) * 16 + sp * 4 + tt];
    __bf16 x[3];
    split3(cp == 0 ? w.re : w.im, x[0], x[1], x[2]);
    P[e] = x[part];
  }
}
void launch_net_pack(int C, const cx<float>* W, __bf16* P, hipStream_t st) {
  hipLaunchKernelGGL(k_net_pack, dim3(256), dim3(256), 0, st, C, W, P);
}

template <int RT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8)))
k_net_mix_mfma(Geom g, const cx<float>* __restrict__ U, const cx<float>* __restrict__ in,
               const v8bf_n* __restrict__ P, cx<float>* __restrict__ out) {
  constexpr int C = 4 * RT, NCH = C / 8;
  // transported inputs [channel][component][site]; the channel stride is padded
  // by 8 entries so that the four channel groups of a wavefront read disjoint banks
  constexpr int TXC = 12 * 64 + 8;
  __shared__ cx<float> txs[8 * TXC];
  const int t = threadIdx.x, lane = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  const long fl = g.V * 12;
  v4f_n acc[RT][6];
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int u = 0; u < 6; ++u) acc[a][u] = v4f_n{0.f, 0.f, 0.f, 0.f};
  // this lane's B column in tile u: colour k = u/2, site 8 (u%2) + (lane%16)/2 of
  // the wave's 16, part c = lane%2 (8 consecutive sites per tile and colour)
  const int kk = lane >> 4;
#pragma unroll 1
  for (int chunk = 0; chunk < 9 * NCH; ++chunk) {
    const int d = chunk / NCH, k0 = (chunk % NCH) * 8;
    __syncthreads();
#pragma unroll 1
    for (int p = t; p < 64 * 8; p += 256) {
      int i = p & 63, ch = p >> 6;
      long gs = (long)blockIdx.x * 64 + i;
      int Bi = (int)(gs / g.bs), si = (int)(gs - (long)Bi * g.bs);
      cx<float> v[12];
      transport_site(g, U, in + (long)(k0 + ch) * fl, d, Bi, si, v);
#pragma unroll
      for (int c = 0; c < 12; ++c) txs[ch * TXC + c * 64 + i] = v[c];
    }
    __syncthreads();
#pragma unroll 1
    for (int ks = 0; ks < 2; ++ks) {
      // B fragments: lane's inner terms 32 ks + 8 kk + e = (channel 4 ks + kk,
      // spin e/2, part e%2)
      const int ch = 4 * ks + kk;
      const v8bf_n* Pc = P + (long)(chunk * 2 + ks) * RT * 3 * 64 + lane;
      // three column tiles per pass; within a pass the A parts of row tile a+1
      // are loaded while tile a multiplies, and the compiler barrier keeps the
      // loads of later tiles from being hoisted (registers: 144 accumulators)
#pragma unroll
      for (int uh = 0; uh < 2; ++uh) {
        v8bf_n b0[3], b1[3], b2[3];
#pragma unroll
        for (int uu = 0; uu < 3; ++uu) {
          const int u = 3 * uh + uu;
          const int c = lane & 1, k = u >> 1, site = 8 * (u & 1) + ((lane & 15) >> 1);
#pragma unroll
          for (int tt = 0; tt < 4; ++tt) {
            const cx<float> v = txs[ch * TXC + (3 * tt + k) * 64 + 16 * w + site];
            __bf16 h, m, lo;
            split3(c == 0 ? v.re : v.im, h, m, lo);
            b0[uu][2 * tt] = h;
            b1[uu][2 * tt] = m;
            b2[uu][2 * tt] = lo;
            split3(c == 0 ? -v.im : v.re, h, m, lo);
            b0[uu][2 * tt + 1] = h;
            b1[uu][2 * tt + 1] = m;
            b2[uu][2 * tt + 1] = lo;
          }
        }
        v8bf_n a0 = Pc[0], a1 = Pc[64], a2 = Pc[128];
#pragma unroll
        for (int a = 0; a < RT; ++a) {
          v8bf_n n0 = a0, n1 = a1, n2 = a2;
          if (a + 1 < RT) {
            n0 = Pc[((a + 1) * 3 + 0) * 64];
            n1 = Pc[((a + 1) * 3 + 1) * 64];
            n2 = Pc[((a + 1) * 3 + 2) * 64];
          }
          v4f_n* ac = acc[a] + 3 * uh;
          // smallest terms first; the column tiles interleave the dependent products
#pragma unroll
          for (int uu = 0; uu < 3; ++uu) ac[uu] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, b0[uu], ac[uu], 0, 0, 0);
#pragma unroll
          for (int uu = 0; uu < 3; ++uu) ac[uu] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1[uu], ac[uu], 0, 0, 0);
#pragma unroll
          for (int uu = 0; uu < 3; ++uu) ac[uu] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b2[uu], ac[uu], 0, 0, 0);
#pragma unroll
          for (int uu = 0; uu < 3; ++uu) ac[uu] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0[uu], ac[uu], 0, 0, 0);
#pragma unroll
          for (int uu = 0; uu < 3; ++uu) ac[uu] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1[uu], ac[uu], 0, 0, 0);
#pragma unroll
          for (int uu = 0; uu < 3; ++uu) ac[uu] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0[uu], ac[uu], 0, 0, 0);
          asm volatile("" ::: "memory");
          a0 = n0;
          a1 = n1;
          a2 = n2;
        }
      }
    }
  }
  // rows 16a + 4 kk + e = (c, s) = (i/4, i%4); column -> (site, colour, part) as above
#pragma unroll
  for (int u = 0; u < 6; ++u) {
    const int c = lane & 1, k = u >> 1, site = 8 * (u & 1) + ((lane & 15) >> 1);
    const long gs = (long)blockIdx.x * 64 + 16 * w + site;
    const int Bs = (int)(gs / g.bs), ss = (int)(gs - (long)Bs * g.bs);
    const long base = fidx(g, Bs, ss, 12);
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = 16 * a + 4 * kk + e;
        const int co = i >> 2, sp = i & 3;
        reinterpret_cast<float*>(out + (long)co * fl + base + (long)(3 * sp + k) * TILE)[c] = acc[a][u][e];
      }
  }
}

void launch_net_mix_mfma(const Geom& g, int C, const cx<float>* U, const cx<float>* in, const __bf16* P,
                         cx<float>* out, hipStream_t st) {
  dim3 grid((unsigned)(g.V / 64));
  const v8bf_n* Pv = reinterpret_cast<const v8bf_n*>(P);
  switch (C) {
    case 8: hipLaunchKernelGGL((k_net_mix_mfma<2>), grid, dim3(256), 0, st, g, U, in, Pv, out); break;
    case 16: hipLaunchKernelGGL((k_net_mix_mfma<4>), grid, dim3(256), 0, st, g, U, in, Pv, out); break;
    case 24: hipLaunchKernelGGL((k_net_mix_mfma<6>), grid, dim3(256), 0, st, g, U, in, Pv, out); break;
    default: throw Error(INVALID_ARG, "matrix-core network layer needs 8, 16 or 24 channels");
  }
}

// ---------------------------------------------------------------------------
// gate: y = z * sigmoid(a |z|^2 + b); keeps the sigmoid for the backward pass
__global__ void k_net_gate(Geom g, int C, const cx<float>* __restrict__ z, const float* __restrict__ a,
                           const float* __restrict__ b, cx<float>* __restrict__ y, float* __restrict__ sv) {
  long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  int c = blockIdx.y;
  if (gid >= g.V) return;
  int B = (int)(gid / g.bs), s = (int)(gid - (long)B * g.bs);
  const long fl = g.V * 12;
  const long base = (long)c * fl + fidx(g, B, s, 12);
  cx<float> v[12];
  float n = 0.f;
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    v[k] = z[base + (long)k * TILE];
    n += norm2(v[k]);
  }
  float u = a[c] * n + b[c];
  float sg = 1.f / (1.f + expf(-u));
#pragma unroll
  for (int k = 0; k < 12; ++k) y[base + (long)k * TILE] = sg * v[k];
  sv[(long)c * g.V + gid] = sg;
}

// the gate in place, inference only (no record of the sigmoid for a backward pass)
__global__ void k_net_gate_inplace(Geom g, const float* a, const float* b, cx<float>* z) {
  long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  int c = blockIdx.y;
  if (gid >= g.V) return;
  int B = (int)(gid / g.bs), s = (int)(gid - (long)B * g.bs);
  const long base = (long)c * g.V * 12 + fidx(g, B, s, 12);
  cx<float> v[12];
  float n = 0.f;
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    v[k] = z[base + (long)k * TILE];
    n += norm2(v[k]);
  }
  float sg = 1.f / (1.f + expf(-(a[c] * n + b[c])));
#pragma unroll
  for (int k = 0; k < 12; ++k) z[base + (long)k * TILE] = sg * v[k];
}
void launch_net_gate_inplace(const Geom& g, int C, const float* a, const float* b, cx<float>* z, hipStream_t st) {
  hipLaunchKernelGGL(k_net_gate_inplace, dim3((unsigned)((g.V + 255) / 256), C), dim3(256), 0, st, g, a, b, z);
}

// gate backward: G_z = s G_y + 2 t a s(1-s) z, t = Re <z, G_y>; per-workgroup
// partial sums of t s(1-s) |z|^2 (-> G_a) and t s(1-s) (-> G_b), FP64
__global__ void __launch_bounds__(256) k_net_gate_bwd(Geom g, int C, const cx<float>* __restrict__ Gy,
                                                      const cx<float>* __restrict__ z, const float* __restrict__ sv,
                                                      const float* __restrict__ a, cx<float>* __restrict__ Gz,
                                                      double* __restrict__ partial) {
  __shared__ double red[4][2];
  long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  int c = blockIdx.y;
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double pa = 0, pb = 0;
  if (gid < g.V) {
    int B = (int)(gid / g.bs), s = (int)(gid - (long)B * g.bs);
    const long fl = g.V * 12;
    const long base = (long)c * fl + fidx(g, B, s, 12);
    cx<float> zv[12], gv[12];
    float n = 0.f, tt = 0.f;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      zv[k] = z[base + (long)k * TILE];
      gv[k] = Gy[base + (long)k * TILE];
      n += norm2(zv[k]);
      tt += gv[k].re * zv[k].re + gv[k].im * zv[k].im;
    }
    float sg = sv[(long)c * g.V + gid];
    float sp = sg * (1.f - sg);
    float f = 2.f * tt * a[c] * sp;
#pragma unroll
    for (int k = 0; k < 12; ++k) Gz[base + (long)k * TILE] = sg * gv[k] + f * zv[k];
    pa = (double)tt * sp * n;
    pb = (double)tt * sp;
  }
  pa = wave_sum_n(pa, 64);
  pb = wave_sum_n(pb, 64);
  if (lane == 0) {
    red[wv][0] = pa;
    red[wv][1] = pb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    partial[((long)c * gridDim.x + blockIdx.x) * 2 + 0] = red[0][0] + red[1][0] + red[2][0] + red[3][0];
    partial[((long)c * gridDim.x + blockIdx.x) * 2 + 1] = red[0][1] + red[1][1] + red[2][1] + red[3][1];
  }
}

// sums of the gate partials: out[c] = sum over workgroups (stride 2, component comp)
__global__ void k_net_sum_partials(const double* __restrict__ partial, int nwg, int C, float* __restrict__ Ga,
                                   float* __restrict__ Gb) {
  int c = threadIdx.x;
  if (c >= C) return;
  double sa = 0, sb = 0;
  for (int i = 0; i < nwg; ++i) {
    sa += partial[((long)c * nwg + i) * 2 + 0];
    sb += partial[((long)c * nwg + i) * 2 + 1];
  }
  Ga[c] = (float)sa;
  Gb[c] = (float)sb;
}

// ---------------------------------------------------------------------------
// weight gradient of one offset d (blockIdx.y): G_W[d][c][c'][s][s'] =
// sum_{x, colour} G_z[c][s](x) conj((T_d x_{c'})[s'](x)); per-workgroup
// partials over a strided set of 8-site tiles.  Thread (s,s') = t & 15 owns the
// CW x CW channel block ((t>>4)>>2, (t>>4)&3).
template <int CW>
__global__ void __launch_bounds__(256) k_net_wgrad(Geom g, const cx<float>* __restrict__ U,
                                                   const cx<float>* __restrict__ x, const cx<float>* __restrict__ Gz,
                                                   cx<float>* __restrict__ partial) {
  constexpr int C = 4 * CW;
  constexpr int TS = 8;
  __shared__ cx<float> tx[C][12][TS];
  __shared__ cx<float> gz[C][12][TS];
  const int d = blockIdx.y;
  const int t = threadIdx.x;
  const int ss = t & 15, sp = ss >> 2, sq = ss & 3;
  const int cb = (t >> 4) >> 2, qb = (t >> 4) & 3;
  const long fl = g.V * 12;
  const long ntiles = g.V / TS;
  cx<float> acc[CW][CW];
#pragma unroll
  for (int i = 0; i < CW; ++i)
#pragma unroll
    for (int j = 0; j < CW; ++j) acc[i][j] = mk<float>(0, 0);
  for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    __syncthreads();
    for (int p = t; p < TS * C; p += 256) {
      int i = p % TS, ch = p / TS;
      long gs = tile * TS + i;
      int Bi = (int)(gs / g.bs), si = (int)(gs - (long)Bi * g.bs);
      cx<float> v[12];
      transport_site(g, U, x + (long)ch * fl, d, Bi, si, v);
#pragma unroll
      for (int k = 0; k < 12; ++k) tx[ch][k][i] = v[k];
      const long base = (long)ch * fl + fidx(g, Bi, si, 12);
#pragma unroll
      for (int k = 0; k < 12; ++k) gz[ch][k][i] = Gz[base + (long)k * TILE];
    }
    __syncthreads();
#pragma unroll 1
    for (int i = 0; i < TS; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        cx<float> gv[CW], tv[CW];
#pragma unroll
        for (int j = 0; j < CW; ++j) {
          gv[j] = gz[cb * CW + j][3 * sp + k][i];
          tv[j] = tx[qb * CW + j][3 * sq + k][i];
        }
#pragma unroll
        for (int a = 0; a < CW; ++a)
#pragma unroll
          for (int b = 0; b < CW; ++b) cjmac(acc[a][b], tv[b], gv[a]);
      }
  }
  cx<float>* out = partial + ((long)blockIdx.x * 9 + d) * C * C * 16;
#pragma unroll
  for (int a = 0; a < CW; ++a)
#pragma unroll
    for (int b = 0; b < CW; ++b) out[((long)(cb * CW + a) * C + (qb * CW + b)) * 16 + sp * 4 + sq] = acc[a][b];
}

// sum of the weight-gradient partials (FP64 accumulation), one thread per entry
__global__ void k_net_wgrad_reduce(const cx<float>* __restrict__ partial, int nwg, long nent, float scale,
                                   cx<float>* __restrict__ GW) {
  long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nent) return;
  double re = 0, im = 0;
  for (int i = 0; i < nwg; ++i) {
    cx<float> v = partial[(long)i * nent + e];
    re += v.re;
    im += v.im;
  }
  GW[e] = mk<float>((float)(scale * re), (float)(scale * im));
}

// ---------------------------------------------------------------------------
// subspace loss and its gradient on one aggregate half (block B, half h), FP64
// small-matrix algebra: G = Y^dag Y, Cm = Y^dag Q, M = G^{-1} Cm,
// L_A = |Q|^2 - tr(Cm^dag M), G_Y = -2 (Q - Y M) M^dag / norm.
// Rows are (slot, component of the half).  scr: [nagg][3][C][C] FP64 scratch.
__global__ void __launch_bounds__(256) k_net_loss(Geom g, int C, const cx<float>* __restrict__ Y,
                                                  const cx<float>* __restrict__ Q, double inv_norm,
                                                  cx<double>* __restrict__ scr, cx<float>* __restrict__ GY,
                                                  double* __restrict__ lpart) {
  __shared__ cx<float> ys[64][32];
  __shared__ cx<float> qs[64][32];
  __shared__ double lred[4];
  const int A = blockIdx.x, B = A >> 1, h = A & 1;
  const int t = threadIdx.x;
  const long fl = g.V * 12;
  const int rows = g.bs * 6;
  const int CC = C * C;
  cx<double>* Gm = scr + (long)A * 3 * CC;
  cx<double>* Cm = Gm + CC;
  cx<double>* Mm = Cm + CC;
  // accumulate G and Cm: thread owns entries e = t, t+256, ... of the 2*CC list
  cx<double> accv[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) accv[m] = mk(0.0, 0.0);
  double qn = 0.0;
  for (int r0 = 0; r0 < rows; r0 += 64) {
    __syncthreads();
    for (int p = t; p < 64 * C; p += 256) {
      int rr = p % 64, c = p / 64;
      int r = r0 + rr;
      cx<float> yv = mk<float>(0, 0), qv = mk<float>(0, 0);
      if (r < rows) {
        int slot = r / 6, comp = 6 * h + (r % 6);
        long idx = (long)c * fl + fidx(g, B, slot, 12) + (long)comp * TILE;
        yv = Y[idx];
        qv = Q[idx];
      }
      ys[rr][c] = yv;
      qs[rr][c] = qv;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      int e = t + 256 * m;
      if (e < 2 * CC) {
        bool isG = e < CC;
        int ee = isG ? e : e - CC;
        int i = ee / C, j = ee % C;
        cx<double> a = accv[m];
        for (int rr = 0; rr < 64; ++rr) {
          cx<float> yi = ys[rr][i];
          cx<float> v = isG ? ys[rr][j] : qs[rr][j];
          cjmac(a, mk<double>(yi.re, yi.im), mk<double>(v.re, v.im));
        }
        accv[m] = a;
      }
    }
    if (t < 64) {
      for (int c = 0; c < C; ++c) qn += norm2(qs[t][c]);
    }
  }
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    int e = t + 256 * m;
    if (e < 2 * CC) {
      if (e < CC) Gm[e] = accv[m];
      else Cm[e - CC] = accv[m];
    }
  }
  qn = wave_sum_n(qn, 64);
  __syncthreads();
  // M = G^{-1} Cm by Gauss-Jordan on [G | Cm] (one thread; C <= 32)
  if (t == 0) {
    for (int e = 0; e < CC; ++e) Mm[e] = Cm[e];
    for (int k = 0; k < C; ++k) {
      int piv = k;
      double best = norm2(Gm[k * C + k]);
      for (int r = k + 1; r < C; ++r)
        if (norm2(Gm[r * C + k]) > best) {
          best = norm2(Gm[r * C + k]);
          piv = r;
        }
      if (piv != k)
        for (int j = 0; j < C; ++j) {
          cx<double> tmp = Gm[k * C + j];
          Gm[k * C + j] = Gm[piv * C + j];
          Gm[piv * C + j] = tmp;
          tmp = Mm[k * C + j];
          Mm[k * C + j] = Mm[piv * C + j];
          Mm[piv * C + j] = tmp;
        }
      cx<double> pv = Gm[k * C + k];
      double dn = norm2(pv);
      cx<double> inv = dn > 0 ? mk(pv.re / dn, -pv.im / dn) : mk(0.0, 0.0);
      for (int j = 0; j < C; ++j) {
        Gm[k * C + j] = Gm[k * C + j] * inv;
        Mm[k * C + j] = Mm[k * C + j] * inv;
      }
      for (int r = 0; r < C; ++r) {
        if (r == k) continue;
        cx<double> f = Gm[r * C + k];
        for (int j = 0; j < C; ++j) {
          Gm[r * C + j] -= f * Gm[k * C + j];
          Mm[r * C + j] -= f * Mm[k * C + j];
        }
      }
    }
    // L_A = |Q|^2 - tr(Cm^dag M)
    double tr = 0;
    for (int i = 0; i < C; ++i)
      for (int j = 0; j < C; ++j) {
        cx<double> cv = Cm[i * C + j], mv = Mm[i * C + j];
        tr += cv.re * mv.re + cv.im * mv.im;
      }
    lred[0] = tr;
  }
  __syncthreads();
  if (t == 0) lpart[A] = (qn - lred[0]) * inv_norm;
  // gradient rows: G_Y[r] = -2 inv_norm (Q[r] - Y[r] M) M^dag
  for (int r = t; r < rows; r += 256) {
    int slot = r / 6, comp = 6 * h + (r % 6);
    long off = fidx(g, B, slot, 12) + (long)comp * TILE;
    cx<double> yr[32], rr[32];
    for (int c = 0; c < C; ++c) {
      cx<float> v = Y[(long)c * fl + off];
      yr[c] = mk<double>(v.re, v.im);
    }
    for (int j = 0; j < C; ++j) {
      cx<float> qv = Q[(long)j * fl + off];
      cx<double> a = mk<double>(qv.re, qv.im);
      for (int i = 0; i < C; ++i) a -= yr[i] * Mm[i * C + j];
      rr[j] = a;
    }
    for (int i = 0; i < C; ++i) {
      cx<double> a = mk(0.0, 0.0);
      for (int j = 0; j < C; ++j) cmac(a, rr[j], conj(Mm[i * C + j]));
      GY[(long)i * fl + off] = mk<float>((float)(-2.0 * inv_norm * a.re), (float)(-2.0 * inv_norm * a.im));
    }
  }
}

// Adam on a real view of all parameters: p -= lr mhat / (sqrt(vhat) + eps)
__global__ void k_adam(long n, float* __restrict__ p, const float* __restrict__ gr, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float gi = gr[i];
  float mi = b1 * m[i] + (1.f - b1) * gi;
  float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------------------
template <int CW>
static void mix_dispatch(const Geom& g, const cx<float>* U, const cx<float>* in, const cx<float>* W, cx<float>* out,
                         bool adj, hipStream_t st) {
  dim3 grid((unsigned)(g.V / 64));
  if (adj) hipLaunchKernelGGL((k_net_mix<CW, true>), grid, dim3(256), 0, st, g, U, in, W, out);
  else hipLaunchKernelGGL((k_net_mix<CW, false>), grid, dim3(256), 0, st, g, U, in, W, out);
}

void launch_net_mix(const Geom& g, int C, const cx<float>* U, const cx<float>* in, const cx<float>* W, cx<float>* out,
                    bool adj, hipStream_t st) {
  switch (C) {
    case 4: mix_dispatch<1>(g, U, in, W, out, adj, st); break;
    case 8: mix_dispatch<2>(g, U, in, W, out, adj, st); break;
    case 12: mix_dispatch<3>(g, U, in, W, out, adj, st); break;
    case 16: mix_dispatch<4>(g, U, in, W, out, adj, st); break;
    case 24: mix_dispatch<6>(g, U, in, W, out, adj, st); break;
    default: throw Error(INVALID_ARG, "network channels must be 4, 8, 12, 16 or 24");
  }
}

void launch_net_gate(const Geom& g, int C, const cx<float>* z, const float* a, const float* b, cx<float>* y, float* sv,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_net_gate, dim3((unsigned)((g.V + 255) / 256), C), dim3(256), 0, st, g, C, z, a, b, y, sv);
}

void launch_net_gate_bwd(const Geom& g, int C, const cx<float>* Gy, const cx<float>* z, const float* sv,
                         const float* a, cx<float>* Gz, double* partial, float* Ga, float* Gb, hipStream_t st) {
  int nwg = (int)((g.V + 255) / 256);
  hipLaunchKernelGGL(k_net_gate_bwd, dim3(nwg, C), dim3(256), 0, st, g, C, Gy, z, sv, a, Gz, partial);
  hipLaunchKernelGGL(k_net_sum_partials, dim3(1), dim3(64), 0, st, partial, nwg, C, Ga, Gb);
}

template <int CW>
static void wgrad_dispatch(const Geom& g, const cx<float>* U, const cx<float>* x, const cx<float>* Gz,
                           cx<float>* partial, int nwg, hipStream_t st) {
  hipLaunchKernelGGL((k_net_wgrad<CW>), dim3(nwg, 9), dim3(256), 0, st, g, U, x, Gz, partial);
}

void launch_net_wgrad(const Geom& g, int C, const cx<float>* U, const cx<float>* x, const cx<float>* Gz,
                      cx<float>* partial, int nwg, cx<float>* GW, hipStream_t st) {
  switch (C) {
    case 4: wgrad_dispatch<1>(g, U, x, Gz, partial, nwg, st); break;
    case 8: wgrad_dispatch<2>(g, U, x, Gz, partial, nwg, st); break;
    case 12: wgrad_dispatch<3>(g, U, x, Gz, partial, nwg, st); break;
    case 16: wgrad_dispatch<4>(g, U, x, Gz, partial, nwg, st); break;
    case 24: wgrad_dispatch<6>(g, U, x, Gz, partial, nwg, st); break;
    default: throw Error(INVALID_ARG, "network channels must be 4, 8, 12, 16 or 24");
  }
  long nent = 9L * C * C * 16;
  hipLaunchKernelGGL(k_net_wgrad_reduce, dim3((unsigned)((nent + 255) / 256)), dim3(256), 0, st, partial, nwg, nent,
                     1.0f, GW);
}

void launch_net_loss(const Geom& g, int C, const cx<float>* Y, const cx<float>* Q, double inv_norm, cx<double>* scr,
                     cx<float>* GY, double* lpart, hipStream_t st) {
  hipLaunchKernelGGL(k_net_loss, dim3(2 * g.nblocks), dim3(256), 0, st, g, C, Y, Q, inv_norm, scr, GY, lpart);
}

void launch_adam(long n, float* p, const float* gr, float* m, float* v, float lr, float b1, float b2, float eps,
                 float c1, float c2, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, p, gr, m, v, lr, b1, b2, eps, c1,
                     c2);
}

}  // namespace ddamg
