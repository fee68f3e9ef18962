// Launch wrappers of every kernel of the library (host-callable).
#pragma once
#include "common.hpp"

namespace ddamg {

// ---- device helpers shared by the kernel files -------------------------------
#ifdef __HIPCC__
// Sum over the active lanes 0..nact-1 of a wavefront; the full sum ends up in
// lane 0 (xor butterfly that skips partners beyond the active range).
template <class T>
__device__ __forceinline__ T wave_sum_n(T v, int nact) {
  int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    T o = __shfl_xor(v, off, 64);
    if ((lane ^ off) < nact) v += o;
  }
  return v;
}

// Sum over the wavefront of v[0..NV) (NV a power of two <= 64): lane l ends
// with the total of v[l % NV] (transposing butterfly: plain xor steps across
// groups of NV lanes, then steps that each halve the values kept per lane).
template <int NV, class T>
__device__ __forceinline__ T wave_transpose_sum(T (&v)[NV], int lane) {
#pragma unroll
  for (int o = 32; o >= NV; o >>= 1)
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] += __shfl_xor(v[q], o, 64);
#pragma unroll
  for (int S = NV; S > 1; S >>= 1) {
    const int o = S >> 1;
    const bool up = (lane & o) != 0;
#pragma unroll
    for (int q = 0; q < S / 2; ++q) {
      const T lo = v[q], hi = v[q + S / 2];
      v[q] = (up ? hi : lo) + __shfl_xor(up ? lo : hi, o, 64);
    }
  }
  return v[0];
}
#endif

// coarse-level geometry as seen by the kernels
struct CGeom {
  int n;           // complex components per site (2 Nv of the level above)
  int nsites;      // sites
  int neven;       // even sites (stored first)
  const int* nbr;  // [nsites][8]: +T +Z +Y +X -T -Z -Y -X
  const int* lexord = nullptr;  // [nsites]: ordered index of the site at each lexicographic position
};

// ---------------------------------------------------------------- fine level
template <class R, class S>
void launch_dirac(const Geom& g, const void* U, const R* H, Twist tw, const cx<R>* in, cx<R>* out, hipStream_t st);
// K fields at a stride of ld complex in one launch (links and clover read once)
template <class R, class S>
void launch_dirac_multi(const Geom& g, const void* U, const R* H, Twist tw, int K, long ld, const cx<R>* in,
                        cx<R>* out, hipStream_t st);
template <class R, class S>
void launch_sap(const Geom& g, int colour, const void* U, const R* H, const R* Minv, Twist tw, const cx<R>* b,
                cx<R>* x, int n_mr, hipStream_t st);
template <class R, class S>
void launch_sap_multi(const Geom& g, int colour, const void* U, const R* H, const R* Minv, Twist tw, const cx<R>* b,
                      cx<R>* x, int n_mr, int K, long ld, hipStream_t st);
template <class R>
void launch_from_lex(const Geom& g, const cx<double>* lex, cx<R>* out, int ncomp, hipStream_t st);
template <class R>
void launch_to_lex(const Geom& g, const cx<R>* in, cx<double>* lex, int ncomp, hipStream_t st);
void set_sigma_table(const double* tab);
void launch_clover(const Geom& g, const cx<double>* U, double csw, double diag, double* H, hipStream_t st);
void launch_clover_from_lex(const Geom& g, const cx<double>* lex, double diag, double* H, hipStream_t st);
void launch_clover_to_lex(const Geom& g, const double* H, double diag, cx<double>* lex, hipStream_t st);
// boundary phases e^{i theta_mu} of twisted boundary conditions: the link
// U_mu(x) with x_mu = L_mu - 1 carries the phase (periodic: 1)
struct LinkPhases {
  double re[4], im[4];
};
void launch_links_from_lex(const Geom& g, const cx<double>* lex, cx<double>* U, const LinkPhases& ph,
                           hipStream_t st);
// out += i rho Gamma5 in on the odd sites; x = 0 on the even sites (FP64)
void launch_odd_twist_add(const Geom& g, const cx<double>* in, cx<double>* out, double rho, hipStream_t st);
void launch_zero_even(const Geom& g, cx<double>* x, hipStream_t st);
// multiply the boundary links of U (block layout) by ph in place
void launch_link_phase(const Geom& g, cx<double>* U, const LinkPhases& ph, hipStream_t st);
void launch_odd_inverse(const Geom& g, const double* H, double tw, double* M, hipStream_t st);
// K-column forms (column k at in + k*ld_in, out + k*ld_out): Q is read once
// per group of columns
template <class R>
void launch_restrict_fine_m(const Geom& g, int Nv, const cx<R>* Q, long vstride, const cx<R>* r, long rld, int K,
                            const int* f2c, cx<R>* rc, long cld, hipStream_t st);
template <class R>
void launch_prolong_fine_m(const Geom& g, int Nv, const cx<R>* Q, long vstride, const cx<R>* ec, long cld, int K,
                           const int* f2c, cx<R>* x, long xld, int accumulate, hipStream_t st);
template <class R>
void launch_restrict_fine(const Geom& g, int Nv, const cx<R>* Q, long vstride, const cx<R>* r, const int* f2c,
                          cx<R>* rc, hipStream_t st);
template <class R>
void launch_prolong_fine(const Geom& g, int Nv, const cx<R>* Q, long vstride, const cx<R>* ec, const int* f2c,
                         cx<R>* x, int accumulate, hipStream_t st);
template <class RI, class RO>
void launch_qr_fine(const Geom& g, int Nv, const cx<RI>* V, long vstride, cx<RO>* Q, long qstride, int* fail,
                    hipStream_t st);
template <class RQ>
// dtw: half the difference of the odd- and even-site twists, whose parity
// rest i (-+dtw) Gamma5 enters the coarse site blocks (0: one twist)
void launch_assemble_fine(const Geom& g, int Nv, const cx<double>* U, const double* H, double dtw, const cx<RQ>* Q,
                          long qstride, const int* f2c, cx<double>* Dc, cx<double>* Xs, hipStream_t st);
template <class S>
void launch_cvt_cx(long n, const cx<double>* in, void* out, hipStream_t st);
void launch_cvt_real(long n, const double* in, float* out, hipStream_t st);

// -------------------------------------------------------------- coarse levels
// D_c blocks: [site][5][n][n] column-major (self without twist, forward T,Z,Y,X)
template <class R, class S>
void launch_coarse_apply(const CGeom& cg, const void* D, double tw, const cx<R>* in, cx<R>* out, hipStream_t st);
// r = b - D x
template <class R, class S>
void launch_coarse_residual(const CGeom& cg, const void* D, double tw, const cx<R>* b, const cx<R>* x, cx<R>* r,
                            hipStream_t st);
// SAP colour sweep with block MR (no odd-even): x += e on blocks of the colour
template <class R, class S>
void launch_coarse_sap(const CGeom& cg, const void* D, double tw, int nblk_colour, int bsz, const int* blk_sites,
                       const int* blk_nbr, const cx<R>* r, cx<R>* x, int n_mr, hipStream_t st);
template <class R, class S>
void launch_coarse_sap_multi(const CGeom& cg, const void* D, double tw, int nblk_colour, int bsz, const int* blk_sites,
                             const int* blk_nbr, const cx<R>* r, cx<R>* x, int n_mr, int K, long ld, hipStream_t st);
// restriction / prolongation between coarse levels
template <class R>
void launch_restrict_coarse(int n, int Nv, int nagg, int asz, const int* agg_sites, const cx<R>* Q, long qstride,
                            const cx<R>* r, cx<R>* rc, hipStream_t st);
template <class R>
void launch_prolong_coarse(int n, int Nv, int nsites, const int* site_agg, const cx<R>* Q, long qstride,
                           const cx<R>* ec, cx<R>* x, int accumulate, hipStream_t st);
// K columns at strides rld / cld (restriction) and cld / xld (prolongation)
template <class R>
void launch_restrict_coarse_m(int n, int Nv, int nagg, int asz, const int* agg_sites, const cx<R>* Q, long qstride,
                              const cx<R>* r, long rld, cx<R>* rc, long cld, int K, hipStream_t st);
template <class R>
void launch_prolong_coarse_m(int n, int Nv, int nsites, const int* site_agg, const cx<R>* Q, long qstride,
                             const cx<R>* ec, long cld, cx<R>* x, long xld, int K, int accumulate, hipStream_t st);
template <class RI, class RO>
void launch_qr_coarse(int n, int Nv, int nagg, int asz, const int* agg_sites, const cx<RI>* V, long vstride,
                      cx<RO>* Q, long qstride, int* fail, hipStream_t st);
template <class RQ>
void launch_assemble_coarse(const CGeom& cg, int Nv, int nagg, const int ab[4], const int* agg_sites,
                            const cx<double>* D, const cx<RQ>* Q, long qstride, cx<double>* Dn, cx<double>* Xs,
                            hipStream_t st);
void launch_self_fixup(int n, int nsites, cx<double>* D, const cx<double>* Xs, int add_x, hipStream_t st);
// inverse of the site blocks (S + i tw Gamma5) on odd sites of the coarsest level
template <class R>
void launch_coarse_odd_inverse(const CGeom& cg, const cx<double>* D, double tw, cx<double>* scratch, cx<R>* Minv,
                               hipStream_t st);
// odd-even Schur pieces on the coarsest level
template <class R, class S>
void launch_coarse_hop_inv_odd(const CGeom& cg, const void* D, const cx<R>* Minv, const cx<R>* in, cx<R>* out,
                               int unused, hipStream_t st);
template <class R, class S>
void launch_coarse_hop_inv_odd_base(const CGeom& cg, const void* D, const cx<R>* Minv, const cx<R>* in,
                                    const cx<R>* base, cx<R>* out, hipStream_t st);
template <class R, class S>
void launch_coarse_schur_even(const CGeom& cg, const void* D, double tw, const cx<R>* v, const cx<R>* t, cx<R>* out,
                              int mode, hipStream_t st);

// ------------------------------------------------------------- learned setup
void launch_net_mix(const Geom& g, int C, const cx<float>* U, const cx<float>* in, const cx<float>* W, cx<float>* out,
                    bool adj, hipStream_t st);
void launch_net_gate(const Geom& g, int C, const cx<float>* z, const float* a, const float* b, cx<float>* y, float* sv,
                     hipStream_t st);
// the forward mixing layer on the matrix cores (inference; C = 8, 16, 24): the
// layer's weights split into three BF16 parts and packed once by
// launch_net_pack (net_packed_bytes(C) bytes per layer)
inline long net_packed_bytes(int C) { return 9L * C * C * 192; }
void launch_net_pack(int C, const cx<float>* W, bf16* P, hipStream_t st);
void launch_net_mix_mfma(const Geom& g, int C, const cx<float>* U, const cx<float>* in, const bf16* P,
                         cx<float>* out, hipStream_t st);
void launch_net_gate_inplace(const Geom& g, int C, const float* a, const float* b, cx<float>* z, hipStream_t st);
void launch_net_gate_bwd(const Geom& g, int C, const cx<float>* Gy, const cx<float>* z, const float* sv,
                         const float* a, cx<float>* Gz, double* partial, float* Ga, float* Gb, hipStream_t st);
void launch_net_wgrad(const Geom& g, int C, const cx<float>* U, const cx<float>* x, const cx<float>* Gz,
                      cx<float>* partial, int nwg, cx<float>* GW, hipStream_t st);
void launch_net_loss(const Geom& g, int C, const cx<float>* Y, const cx<float>* Q, double inv_norm, cx<double>* scr,
                     cx<float>* GY, double* lpart, hipStream_t st);
void launch_adam(long n, float* p, const float* gr, float* m, float* v, float lr, float b1, float b2, float eps,
                 float c1, float c2, hipStream_t st);

// ---------------------------------------------------------------------- BLAS
// partial sums of <V_i, w> (i < k) into partial[i][nwg]; then reduced into out
template <class R>
void launch_multidot(const cx<R>* V, long ldv, int k, const cx<R>* w, long N, cx<double>* partial, int nwg,
                     hipStream_t st);
void launch_reduce(const cx<double>* partial, int k, int nwg, cx<double>* out, int mode, hipStream_t st);
template <class R>
void launch_multi_axpy(const cx<R>* V, long ldv, int k, const cx<double>* coef, double sign, cx<R>* w, long N,
                       hipStream_t st);
template <class R>
void launch_scale_by_inv(const cx<R>* in, const cx<double>* s, cx<R>* out, long N, hipStream_t st);
template <class RA, class RB>
void launch_copy_cvt(const cx<RA>* in, cx<RB>* out, long N, hipStream_t st);
template <class R>
void launch_axpby(long N, double a, const cx<R>* x, double b, cx<R>* y, hipStream_t st);  // y = a x + b y
template <class R>
void launch_sub(long N, const cx<R>* a, const cx<R>* b, cx<R>* out, hipStream_t st);     // out = a - b
template <class R>
void launch_zero(long N, cx<R>* x, hipStream_t st);
void launch_givens(cx<double>* H, int ldh, double* cs, cx<double>* sn, cx<double>* g, int j, double* resid,
                   hipStream_t st);
void launch_trisolve(const cx<double>* H, int ldh, const cx<double>* g, cx<double>* y, int j, hipStream_t st);
void launch_set_scalar(cx<double>* dst, const cx<double>* src_norm2_sqrt, hipStream_t st);

// column-batched Krylov kernels (K columns, column r = blockIdx.y; act: per-column
// mask or null; cs*: column strides of vectors and scalar arrays)
template <class R>
void launch_multidot_b(const cx<R>* V, long ldv, long csV, int k, const cx<R>* w, long csw, long N, cx<double>* partial,
                       long pcs, int nwg, int K, const int* act, hipStream_t st);
void launch_reduce_b(const cx<double>* partial, long pcs, int k, int nwg, cx<double>* out, long ocs, int mode, int K,
                     const int* act, hipStream_t st);
template <class R>
void launch_multi_axpy_b(const cx<R>* V, long ldv, long csV, int k, const int* kcol, const cx<double>* coef, long ccs,
                         double sign, cx<R>* w, long csw, long N, int K, const int* act, hipStream_t st);
void launch_multi_axpy_b_mixed(const cx<float>* V, long ldv, long csV, int k, const int* kcol, const cx<double>* coef,
                               long ccs, double sign, cx<double>* w, long csw, long N, int K, const int* act,
                               hipStream_t st);
template <class R>
void launch_scale_by_inv_b(const cx<R>* in, long csi, const cx<double>* s, long scs, cx<R>* out, long cso, long N,
                           int K, const int* act, int zero_off, hipStream_t st);
template <class RA, class RB>
void launch_copy_cvt_b(const cx<RA>* in, long csi, cx<RB>* out, long cso, long N, int K, hipStream_t st);
template <class R>
void launch_sub_b(long N, const cx<R>* a, long csa, const cx<R>* b, long csb, cx<R>* out, long cso, int K,
                  hipStream_t st);
template <class R>
void launch_zero_b(long N, cx<R>* x, long cs, int K, hipStream_t st);
// Arnoldi step of K lock-step processes: classical Gram-Schmidt against
// V_0..V_{k-1} (k <= 32; two passes for FP64 vectors, one for FP32), norm,
// scaling of w and Givens step j, in four (three) launches;
// pa, pb: two partial buffers of pcs >= ldh * nwg complex per column; nwg
// workgroups of cgs_block_size<R>() threads per column; resid_host (pinned host
// memory, may be null) receives a copy of the K residual estimates
template <class R>
int cgs_block_size();
// Gram-Schmidt passes of the Arnoldi step of a cycle of m steps: two for
// FP64 vectors in cycles longer than 8 steps, one otherwise.  One classical
// pass loses orthogonality in proportion to the squared condition number of
// the basis it orthogonalises against, which a short cycle keeps small; FP32
// inner solves stop at loose tolerances, far above what one pass keeps.
template <class R>
inline bool cgs_two_pass(int m) {
  return sizeof(R) == 8 && m > 8;
}
template <class R>
void launch_cgs_step(const cx<R>* V, long ldv, long csV, int k, cx<R>* w, long csw, long N, cx<double>* pa,
                     cx<double>* pb, long pcs, int nwg, cx<double>* hcol, long hcs, cx<double>* H, int ldh, int m,
                     double* cs, cx<double>* sn, cx<double>* g, int j, double* resid, double* resid_host, int K,
                     const int* act, hipStream_t st);
void launch_givens_b(cx<double>* H, int ldh, int m, double* cs, cx<double>* sn, cx<double>* g, int j, double* resid,
                     int K, const int* act, hipStream_t st);
void launch_trisolve_b(const cx<double>* H, int ldh, int m, const cx<double>* g, cx<double>* y, const int* jd, int K,
                       hipStream_t st);
void launch_init_g_b(cx<double>* g, int ldh, const cx<double>* s, long scs, int K, const int* act, hipStream_t st);

// coarse operator on K <= 16 right-hand sides at once (matrix cores; 16-bit
// operator storage S; n = 2 N_v a multiple of 16).  Vectors FP32, right-hand
// side r at offset r * ldv.
template <class S>
void launch_coarse_apply_mrhs(const CGeom& cg, const void* D, double tw, int K, long ldv, const cx<float>* x,
                              const cx<float>* b, cx<float>* y, hipStream_t st, const int* sites = nullptr,
                              int nlist = 0);
template <class S>
void launch_coarse_schur_even_mrhs(const CGeom& cg, const void* D, double tw, int K, long ldv, const cx<float>* v,
                                   const cx<float>* t, cx<float>* y, int mode, hipStream_t st);
// SAP colour sweep of an intermediate level for K fields (K <= 16), one
// workgroup per block (bsz <= 16 sites), matrix cores
template <class S>
void launch_coarse_sap_mrhs(const CGeom& cg, const void* D, double tw, int nblk_colour, int bsz, const int* blk_sites,
                            const int* blk_nbr, const cx<float>* r, cx<float>* x, int n_mr, int K, long ld,
                            hipStream_t st);
template <class S>
void launch_coarse_hop_inv_odd_mrhs(const CGeom& cg, const void* D, const cx<float>* Minv, int K, long ldv,
                                    const cx<float>* x, const cx<float>* base, cx<float>* y, hipStream_t st);

}  // namespace ddamg
