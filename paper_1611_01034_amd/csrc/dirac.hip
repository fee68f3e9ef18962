// The fine operator D(+-mu) = D_W +- i Gamma5 mu (Sec. 1) on the whole
// lattice: Wilson hops with spin projection, the clover site term and the
// twist, in FP64 or FP32 arithmetic with FP64/FP32/FP16/BF16 link storage.
#include "finedev.hpp"

namespace ddamg {

// ---------------------------------------------------------------------------
// D(tw) psi, full lattice (tw: the twist of each parity), for K fields at a
// stride of ld complex.  One workgroup per (lattice block, field), one
// work-item per site; the block's input spinors are staged in LDS, so only
// hops that leave the block read neighbours from global memory.  The K
// fields of a block run in consecutive workgroups of one XCD, so the block's
// links and clover come from HBM once for all of them and from L2 for the
// rest.  With gm > 0 each XCD takes groups of gm consecutive blocks (two rows
// of blocks along X) while the XCDs sweep neighbouring groups together
// (group_remap); else each XCD sweeps one contiguous range of blocks
// (xcd_remap).
template <class R, class S>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 8 ? 2 : 3, 8)))
k_dirac(Geom g, int gm, const typename store_traits<S>::elem* __restrict__ U, const R* __restrict__ H, TwistR<R> tw,
        int K, long ld, const cx<R>* __restrict__ in, cx<R>* __restrict__ out) {
  extern __shared__ char smem_raw[];
  cx<R>* lds = reinterpret_cast<cx<R>*>(smem_raw);  // 12 x bs, parity-split
  const int w = gm > 0 ? group_remap(blockIdx.x, gm * K) : xcd_remap(blockIdx.x, gridDim.x), s = threadIdx.x;
  const int B = w / K, col = w - B * K;
  in += (long)col * ld;
  out += (long)col * ld;
  SiteNbr me;
  me_of(g, B, s, me);
  cx<R> psi[12], acc[12];
  load_spinor(in, g, B, s, psi);
#pragma unroll
  for (int c = 0; c < 12; ++c) *lds_site(lds, g, s, c) = psi[c];
  site_term(H, g, B, s, tw, psi, acc);
  __syncthreads();
  hop_staged<R, S>(U, in, lds, g, B, s, me, acc);
  // streaming stores: the result is not read again by this sweep, so it does
  // not need to take L2 from the halo lines of the blocks still running
  const long base = fidx(g, B, s, 12);
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    __builtin_nontemporal_store(acc[c].re, &out[base + (long)c * TILE].re);
    __builtin_nontemporal_store(acc[c].im, &out[base + (long)c * TILE].im);
  }
}

template <class R, class S>
void launch_dirac_multi(const Geom& g, const void* U, const R* H, Twist tw, int K, long ld, const cx<R>* in,
                        cx<R>* out, hipStream_t st) {
  size_t sm = 12 * (size_t)g.bs * sizeof(cx<R>);
  const int gm = g.nblocks % (16 * g.nb[3]) == 0 ? 2 * g.nb[3] : 0;
  hipLaunchKernelGGL((k_dirac<R, S>), dim3(g.nblocks * K), dim3(g.bs), sm, st, g, gm,
                     (const typename store_traits<S>::elem*)U, H, TwistR<R>(tw), K, ld, in, out);
}
template <class R, class S>
void launch_dirac(const Geom& g, const void* U, const R* H, Twist tw, const cx<R>* in, cx<R>* out, hipStream_t st) {
  launch_dirac_multi<R, S>(g, U, H, tw, 1, 0, in, out, st);
}
#define DIRAC_INST(R, S)                                                                                     \
  template void launch_dirac<R, S>(const Geom&, const void*, const R*, Twist, const cx<R>*, cx<R>*, hipStream_t); \
  template void launch_dirac_multi<R, S>(const Geom&, const void*, const R*, Twist, int, long, const cx<R>*, cx<R>*, \
                                         hipStream_t);
DIRAC_INST(double, double)
DIRAC_INST(float, float)
DIRAC_INST(float, f16)
DIRAC_INST(float, bf16)
#undef DIRAC_INST

}  // namespace ddamg
