// Host orchestration of the DD-alpha-AMG solver (paper Sec. 1, Eq. 1):
// flexible GMRES on the fine level, preconditioned by the multigrid cycle
//   x = k SAP iterations after  x = P D_c^{-1} P^dag (v - D x_j)  after j SAP
// iterations; coarse solves by FGMRES preconditioned with the next level's
// cycle, and odd-even GMRES on the coarsest level (Sec. 3).  The adaptive
// setup builds the test vectors that span P (Sec. 1; setup iterations as in
// Listing 1).  All arithmetic runs in the kernels; this file only sequences
// launches and moves at most one scalar per Krylov iteration to the host.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "solver.hpp"

namespace ddamg {

// ---------------------------------------------------------------------------
// small helper kernels: permutations between lexicographic and ordered coarse
// site numbering, odd-site inverse application
template <class RA, class RB>
__global__ void k_permute(int n, int nsites, const int* __restrict__ map, const cx<RA>* __restrict__ in,
                          cx<RB>* __restrict__ out, int scatter) {
  long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)nsites * n) return;
  int s = (int)(gid / n), k = (int)(gid - (long)s * n);
  long src, dst;
  if (scatter) {  // out[map[s]] = in[s]
    src = gid;
    dst = (long)map[s] * n + k;
  } else {        // out[s] = in[map[s]]
    src = (long)map[s] * n + k;
    dst = gid;
  }
  cx<RA> v = in[src];
  out[dst] = mk<RB>((RB)v.re, (RB)v.im);
}
template <class RA, class RB>
static void permute(int n, int nsites, const int* map, const cx<RA>* in, cx<RB>* out, int scatter, hipStream_t st) {
  long tot = (long)nsites * n;
  hipLaunchKernelGGL((k_permute<RA, RB>), dim3((tot + 255) / 256), dim3(256), 0, st, n, nsites, map, in, out,
                     scatter);
}

template <class R>
__global__ void __launch_bounds__(256) k_minv_odd(CGeom cg, const cx<R>* __restrict__ Minv, const cx<R>* __restrict__ in,
                                                  cx<R>* __restrict__ out) {
  __shared__ cx<R> us[4][64];
  int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int io = blockIdx.x * 4 + wv;
  int site = cg.neven + io;
  bool valid = site < cg.nsites;
  const int n = cg.n;
  if (valid && lane < n) us[wv][lane] = in[(long)site * n + lane];
  __syncthreads();
  if (valid && lane < n) {
    const cx<R>* M = Minv + (long)io * n * n;
    cx<R> acc = mk<R>(0, 0);
    for (int l = 0; l < n; ++l) cmac(acc, M[(long)l * n + lane], us[wv][l]);
    out[(long)site * n + lane] = acc;
  }
}

__global__ void k_all_finite(long n, const double* __restrict__ a, int* __restrict__ flag) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !isfinite(a[i])) atomicOr(flag, 1);
}

// ---------------------------------------------------------------------------
MemPool*& current_pool() {
  static thread_local MemPool* p = nullptr;
  return p;
}

namespace {
constexpr size_t kGranule = 256;
constexpr size_t kMinSlab = size_t(64) << 20;  // small buffers share 64 MiB slabs
constexpr size_t kSlabRound = size_t(2) << 20;
}  // namespace

void* MemPool::get(size_t b, bool transient) {
  b = (b + kGranule - 1) / kGranule * kGranule;
  // best fit over the free ranges of every slab of the same kind
  Slab* best = nullptr;
  size_t best_off = 0, best_len = ~size_t(0);
  for (auto& s : slabs)
    if (s.transient == transient)
      for (auto& fr : s.free)
      if (fr.second >= b && fr.second < best_len) {
        best = &s;
        best_off = fr.first;
        best_len = fr.second;
      }
  if (best) {
    if (dirty) {
      HIP_CHECK(hipStreamSynchronize(st));
      dirty = false;
    }
    best->free.erase(best_off);
    if (best_len > b) best->free[best_off + b] = best_len - b;
    best->used += b;
    return best->base + best_off;
  }
  size_t sb = std::max(b, kMinSlab);
  sb = (sb + kSlabRound - 1) / kSlabRound * kSlabRound;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, sb);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
    (void)hipGetLastError();
    trim();
    e = hipMalloc(&p, sb);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
      (void)hipGetLastError();
      throw Error(OUT_OF_MEMORY, "device allocation of " + std::to_string(b) + " bytes failed (" +
                                     std::to_string(reserved()) + " bytes held by the context)");
    }
  }
  HIP_CHECK(e);
  Slab s;
  s.base = (char*)p;
  s.bytes = sb;
  s.used = b;
  s.transient = transient;
  if (sb > b) s.free[b] = sb - b;
  slabs.push_back(std::move(s));
  return p;
}

void MemPool::put(void* p, size_t b) {
  b = (b + kGranule - 1) / kGranule * kGranule;
  char* c = (char*)p;
  for (auto& s : slabs) {
    if (c < s.base || c >= s.base + s.bytes) continue;
    size_t off = (size_t)(c - s.base), len = b;
    auto next = s.free.find(off + len);
    if (next != s.free.end()) {
      len += next->second;
      s.free.erase(next);
    }
    auto it = s.free.lower_bound(off);
    if (it != s.free.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == off) {
        off = prev->first;
        len += prev->second;
        s.free.erase(prev);
      }
    }
    s.free[off] = len;
    s.used -= b;
    dirty = true;
    return;
  }
}

void MemPool::trim() {
  (void)hipStreamSynchronize(st);
  std::vector<Slab> keep;
  for (auto& s : slabs) {
    if (s.used == 0) (void)hipFree(s.base);
    else keep.push_back(std::move(s));
  }
  slabs.swap(keep);
  dirty = false;
}

size_t MemPool::reserved() const {
  size_t t = 0;
  for (auto& s : slabs) t += s.bytes;
  return t;
}

MemPool::~MemPool() {
  if (!slabs.empty()) (void)hipStreamSynchronize(st);
  for (auto& s : slabs) (void)hipFree(s.base);
}

// ---------------------------------------------------------------------------
hipEvent_t KernelTimer::get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HIP_CHECK(hipEventCreate(&e));
  return e;
}
void KernelTimer::begin(int kind, hipEvent_t* a) {
  (void)kind;
  *a = nullptr;
  if (!on) return;
  *a = get();
  HIP_CHECK(hipEventRecord(*a, st));
}
void KernelTimer::end(int kind, hipEvent_t a, double nbytes, double nflops) {
  if (!on || !a) return;
  bytes[kind] += nbytes;
  flops[kind] += nflops;
  hipEvent_t b = get();
  HIP_CHECK(hipEventRecord(b, st));
  recs.push_back({kind, a, b});
  if (recs.size() > 4096) flush();
}
void KernelTimer::flush() {
  if (recs.empty()) return;
  HIP_CHECK(hipStreamSynchronize(st));
  for (auto& r : recs) {
    float t = 0;
    HIP_CHECK(hipEventElapsedTime(&t, r.a, r.b));
    count[r.kind] += 1;
    ms[r.kind] += t;
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  recs.clear();
}
void KernelTimer::reset() {
  for (int i = 0; i < NKIND; ++i) {
    count[i] = 0;
    ms[i] = 0;
    bytes[i] = 0;
    flops[i] = 0;
  }
}
KernelTimer::~KernelTimer() {
  for (auto& r : recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : pool) (void)hipEventDestroy(e);
}

struct TimeScope {
  KernelTimer& t;
  int kind;
  hipEvent_t a;
  double b, f;
  TimeScope(KernelTimer& t_, int k, double bytes = 0, double flops = 0) : t(t_), kind(k), b(bytes), f(flops) {
    t.begin(k, &a);
  }
  ~TimeScope() { t.end(kind, a, b, f); }
};

// Real flops of one fine SAP colour sweep of K fields (a complex multiply-add
// counts 8, a real-times-complex product 2, an addition 1).  A packed
// Hermitian 6x6 product is 252 (6 diagonal, 15 off-diagonal entries used
// twice), the twist 4 per component, one hop 204 (spin projection 12, two
// 3x3 link products 144, reconstruction 48).  Per site of the swept colour:
// the residual b - D x (site term 552, eight hops 1632, subtraction 24), and
// on half of the sites each: T_oo^-1 r_o with x_o += t_o (1056 + 24), the
// first rho (hops), per MR step w = T_oo^-1 D_oe rho and q = T_ee rho - D_eo w
// with the dots and updates (5208 per pair), and the closing correction (hops,
// T_oo^-1, two updates: 2736 per pair).
static double sap_sweep_flops(const Geom& g, int K, int n_mr) {
  const double per_site = 4932.0 + 2604.0 * n_mr;
  return 0.5 * (double)g.V * K * per_site;
}

// Algorithmic bytes of one fine SAP colour sweep of K fields (each datum
// moved once): per site of the swept colour the links (36 entries of the
// storage format), the clover term (72 reals) and, on odd sites, the inverse
// factors (72 reals, 36 per site on average) once for all fields; per field
// b, x read and written, and x of the other colour read once for the residual.
template <class R, class S>
static double sap_sweep_bytes(const Geom& g, int K) {
  const double shared = 36.0 * sizeof(typename store_traits<S>::elem) + 108.0 * sizeof(R);
  const double field = 4.0 * 12 * sizeof(cx<R>);
  return 0.5 * (double)g.V * (shared + K * field);
}

// ---------------------------------------------------------------------------
template <class R>
void KrylovWS<R>::init(int m_, long ld_, long N, bool flex) {
  m = m_;
  ld = ld_;
  flexible = flex;
  V.ensure(sizeof(cx<R>) * (size_t)(m + 1) * ld);
  if (flex) Z.ensure(sizeof(cx<R>) * (size_t)m * ld);
  tmp.ensure(sizeof(cx<R>) * (size_t)ld);
  H.ensure(sizeof(cx<double>) * (size_t)(m + 1) * m);
  cs.ensure(sizeof(double) * m);
  sn.ensure(sizeof(cx<double>) * m);
  g.ensure(sizeof(cx<double>) * (m + 1));
  y.ensure(sizeof(cx<double>) * (m + 1));
  nwg = (int)std::min<long>(1024, std::max<long>(1, (N + 255) / 256));
  part.ensure(sizeof(cx<double>) * (size_t)nwg * (m + 1));
  scal.ensure(sizeof(cx<double>) * 4);
  resid.ensure(sizeof(double));
  if (!h_resid) HIP_CHECK(hipHostMalloc((void**)&h_resid, sizeof(double) * 4, hipHostMallocDefault));
  for (auto& e : ready)
    if (!e) HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
}
template <class R>
KrylovWS<R>::~KrylovWS() {
  if (h_resid) (void)hipHostFree(h_resid);
  for (auto e : ready)
    if (e) (void)hipEventDestroy(e);
}
template struct KrylovWS<double>;
template struct KrylovWS<float>;

template <class R>
KrylovResult fgmres(Ctx& c, KrylovWS<R>& ws, long N, const std::function<void(const cx<R>*, cx<R>*)>& A,
                    const std::function<void(const cx<R>*, cx<R>*)>* M, const cx<R>* b, cx<R>* x, double tol,
                    int max_iter, bool fixed, bool x_is_zero) {
  hipStream_t st = c.st;
  const int m = ws.m;
  const long ld = ws.ld;
  int nwg = (int)std::min<long>(ws.nwg, std::max<long>(1, (N + 255) / 256));
  cx<R>* V = ws.V.template as<cx<R>>();
  cx<R>* Z = M ? ws.Z.template as<cx<R>>() : V;
  cx<R>* r = ws.tmp.template as<cx<R>>();
  cx<double>* H = ws.H.template as<cx<double>>();
  cx<double>* scal = ws.scal.template as<cx<double>>();
  cx<double>* part = ws.part.template as<cx<double>>();
  auto norm_to = [&](const cx<R>* v, cx<double>* dst) {
    launch_multidot<R>(v, 0, 1, v, N, part, nwg, st);
    launch_reduce(part, 1, nwg, dst, 2, st);
  };
  auto read = [&](const void* dptr) -> double {
    HIP_CHECK(hipMemcpyAsync(ws.h_resid, dptr, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
    return ws.h_resid[0];
  };
  KrylovResult res;
  norm_to(b, scal);
  double bnorm = read(scal);
  if (bnorm == 0.0) {
    launch_zero<R>(N, x, st);
    res.converged = true;
    return res;
  }
  if (x_is_zero) {
    launch_zero<R>(N, x, st);
    launch_copy_cvt<R, R>(b, r, N, st);
  } else {
    A(x, r);
    launch_sub<R>(N, b, r, r, st);
  }
  norm_to(r, scal + 1);
  double beta = read(scal + 1);
  int it = 0;
  while (true) {
    if (!fixed && beta <= tol * bnorm) break;
    if (it >= max_iter) break;
    int mm = fixed ? std::min(m, max_iter - it) : m;
    launch_scale_by_inv<R>(r, scal + 1, V, N, st);
    launch_zero<double>(m + 1, ws.g.template as<cx<double>>(), st);
    launch_set_scalar(ws.g.template as<cx<double>>(), scal + 1, st);
    int jd = 0;
    // Without a preconditioner an iteration is cheap, so the convergence test
    // of iteration j is taken while iteration j+1 is already queued (no idle
    // gap on the device).  If iteration j met the tolerance, the queued
    // iteration j+1 is discarded: it changes only Hessenberg column j+1 and
    // g[j+1], g[j+2], so the update from columns 0..j is unaffected.
    const bool lookahead = !fixed && M == nullptr;
    bool pending = false;  // an estimate of iteration jd-1 is in flight
    for (int j = 0; j < mm; ++j) {
      cx<R>* Vj = V + (long)j * ld;
      cx<R>* Vn = V + (long)(j + 1) * ld;
      cx<R>* z = Vj;
      if (M) {
        z = Z + (long)j * ld;
        (*M)(Vj, z);
      }
      A(z, Vn);
      cx<double>* hcol = H + (long)j * (m + 1);
      launch_multidot<R>(V, ld, j + 1, Vn, N, part, nwg, st);
      launch_reduce(part, j + 1, nwg, hcol, 0, st);
      launch_multi_axpy<R>(V, ld, j + 1, hcol, -1.0, Vn, N, st);
      if (cgs_two_pass<R>(m)) {  // second classical Gram-Schmidt pass
        launch_multidot<R>(V, ld, j + 1, Vn, N, part, nwg, st);
        launch_reduce(part, j + 1, nwg, ws.y.template as<cx<double>>(), 0, st);
        launch_reduce(part, j + 1, nwg, hcol, 1, st);
        launch_multi_axpy<R>(V, ld, j + 1, ws.y.template as<cx<double>>(), -1.0, Vn, N, st);
      }
      norm_to(Vn, hcol + j + 1);
      launch_scale_by_inv<R>(Vn, hcol + j + 1, Vn, N, st);
      launch_givens(H, m + 1, ws.cs.template as<double>(), ws.sn.template as<cx<double>>(), ws.g.template as<cx<double>>(), j,
                    ws.resid.template as<double>(), st);
      ++it;
      jd = j + 1;
      if (lookahead) {
        const int k = j & 1;
        HIP_CHECK(hipMemcpyAsync(ws.h_resid + 2 + k, ws.resid.p, sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_CHECK(hipEventRecord(ws.ready[k], st));
        if (pending) {
          HIP_CHECK(hipEventSynchronize(ws.ready[k ^ 1]));
          if (ws.h_resid[2 + (k ^ 1)] <= tol * bnorm) {  // iteration j-1 converged: drop iteration j
            --it;
            jd = j;
            pending = false;
            break;
          }
        }
        pending = true;
      } else if (!fixed) {
        double est = read(ws.resid.p);
        if (est <= tol * bnorm) break;
      }
      if (it >= max_iter) break;
    }
    if (pending) {  // test the last queued estimate before the restart
      HIP_CHECK(hipEventSynchronize(ws.ready[(jd - 1) & 1]));
      pending = false;
    }
    launch_trisolve(H, m + 1, ws.g.template as<cx<double>>(), ws.y.template as<cx<double>>(), jd, st);
    launch_multi_axpy<R>(Z, ld, jd, ws.y.template as<cx<double>>(), 1.0, x, N, st);
    A(x, r);
    launch_sub<R>(N, b, r, r, st);
    norm_to(r, scal + 1);
    beta = read(scal + 1);
    if (fixed && it >= max_iter) break;
    if (beta == 0.0) break;
  }
  res.iters = it;
  res.resid = beta / bnorm;
  res.converged = beta <= tol * bnorm;
  return res;
}
// ---------------------------------------------------------------------------
// K (F)GMRES processes in lock step: one launch per step serves every column
// (the batched operator reads its matrix once for all columns).  Each column
// keeps its own Hessenberg matrix, rotations and stopping test; a column that
// meets its tolerance drops out of the reductions and its next basis vector is
// zeroed, so nested solves see a zero right-hand side for it.  The iterates are
// those of K separate solves in exact arithmetic.
// workgroups per column of the fused Arnoldi step: about one element per
// thread of an FP32 vector (at most 128 workgroups, so every workgroup's
// prologue sums few partials), four per thread of an FP64 one (at most 1024)
template <class R>
static int cgs_nwg(long N) {
  const long per = sizeof(R) == 4 ? cgs_block_size<R>() : 4L * cgs_block_size<R>();
  const long cap = sizeof(R) == 4 ? 256 : 1024;
  return (int)std::min<long>(cap, std::max<long>(1, (N + per - 1) / per));
}

template <class R>
void KrylovWSm<R>::init(int m_, int K_, long ld_, long N, bool flex, bool z_fp32, bool transient) {
  m = m_;
  K = K_;
  ld = ld_;
  flexible = flex;
  zf32 = z_fp32;
  V.ensure(sizeof(cx<R>) * (size_t)(m + 1) * K * ld, transient);
  if (flex) Z.ensure((z_fp32 ? sizeof(cx<float>) : sizeof(cx<R>)) * (size_t)m * K * ld, transient);
  r.ensure(sizeof(cx<R>) * (size_t)K * ld, transient);
  H.ensure(sizeof(cx<double>) * (size_t)(m + 1) * m * K);
  cs.ensure(sizeof(double) * m * K);
  sn.ensure(sizeof(cx<double>) * m * K);
  g.ensure(sizeof(cx<double>) * (m + 1) * K);
  y.ensure(sizeof(cx<double>) * (m + 1) * K);
  nwg = (int)std::min<long>(256, std::max<long>(1, (N + 255) / 256));
  nwgf = cgs_nwg<R>(N);
  part.ensure(sizeof(cx<double>) * (size_t)std::max(nwg, nwgf) * (m + 1) * K * 2);  // two halves for the fused step
  scal.ensure(sizeof(cx<double>) * 4 * K);
  resid.ensure(sizeof(double) * K);
  act.ensure(sizeof(int) * K);
  jd.ensure(sizeof(int) * K);
  if (!h_resid) {
    // coherent: the Arnoldi kernels store residual estimates here directly
    HIP_CHECK(hipHostMalloc((void**)&h_resid, sizeof(double) * 96, hipHostMallocCoherent));
    HIP_CHECK(hipHostMalloc((void**)&h_scal, sizeof(cx<double>) * 4 * 64, hipHostMallocDefault));
    HIP_CHECK(hipHostMalloc((void**)&h_act, sizeof(int) * 64, hipHostMallocDefault));
    HIP_CHECK(hipHostMalloc((void**)&h_jd, sizeof(int) * 64, hipHostMallocDefault));
    HIP_CHECK(hipHostMalloc((void**)&h_act_ring, sizeof(int) * 64, hipHostMallocDefault));
  }
  for (auto& e : ready)
    if (!e) HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
}
template <class R>
KrylovWSm<R>::~KrylovWSm() {
  for (auto e : ready)
    if (e) (void)hipEventDestroy(e);
  if (h_resid) (void)hipHostFree(h_resid);
  if (h_scal) (void)hipHostFree(h_scal);
  if (h_act) (void)hipHostFree(h_act);
  if (h_jd) (void)hipHostFree(h_jd);
  if (h_act_ring) (void)hipHostFree(h_act_ring);
}
template struct KrylovWSm<double>;
template struct KrylovWSm<float>;

template <class R>
KrylovResultM fgmres_multi(Ctx& c, KrylovWSm<R>& ws, int K, long N, const OpM<R>& A, const OpM<R>* M, const cx<R>* b,
                           cx<R>* x, double tol, int max_iter, bool fixed, bool x_is_zero, const OpMf* Mf) {
  if (K < 1 || K > ws.K || K > 16) throw Error(INVALID_ARG, "lock-step solve: bad column count");
  if (Mf && (!std::is_same<R, double>::value || !ws.zf32 || M))
    throw Error(INVALID_ARG, "FP32 directions need an FP64 solve with an FP32 workspace");
  hipStream_t st = c.st;
  const int m = ws.m, ldh = m + 1;
  const long ld = ws.ld, hcs = (long)ldh * m;
  const int nwg = (int)std::min<long>(ws.nwg, std::max<long>(1, (N + 255) / 256));
  // fused Arnoldi launches: for FP32 vectors about 512 workgroups over all K
  // columns (two per CU) fill the device; more only add per-workgroup
  // partial sums to reduce
  int nwgf = std::min(ws.nwgf, cgs_nwg<R>(N));
  if (sizeof(R) == 4) nwgf = std::min(nwgf, std::max(32, (512 + K - 1) / K));
  const long pcs = (long)std::max(ws.nwg, ws.nwgf) * ldh;
  cx<R>* V = ws.V.template as<cx<R>>();
  cx<R>* Z = M ? ws.Z.template as<cx<R>>() : V;
  cx<float>* Zf = Mf ? ws.Z.template as<cx<float>>() : nullptr;
  cx<R>* r = ws.r.template as<cx<R>>();
  cx<double>* H = ws.H.template as<cx<double>>();
  cx<double>* scal = ws.scal.template as<cx<double>>();
  cx<double>* part = ws.part.template as<cx<double>>();
  cx<double>* g = ws.g.template as<cx<double>>();
  cx<double>* y = ws.y.template as<cx<double>>();
  int* act = ws.act.template as<int>();
  int* jd = ws.jd.template as<int>();
  // ||v_r|| of every column into scal[r*4 + slot]
  auto norms = [&](const cx<R>* v, int slot, const int* a) {
    launch_multidot_b<R>(v, 0, ld, 1, v, ld, N, part, pcs, nwg, K, a, st);
    launch_reduce_b(part, pcs, 1, nwg, scal + slot, 4, 2, K, a, st);
  };
  auto read_scal = [&]() {
    HIP_CHECK(hipMemcpyAsync(ws.h_scal, scal, sizeof(cx<double>) * 4 * K, hipMemcpyDeviceToHost, st));
    HIP_CHECK(hipStreamSynchronize(st));
  };
  // Each push copies from its own staging slot: with the look-ahead a slot is
  // reused only after the host has waited on an event recorded after its copy
  // (one is waited on per step, and a push happens at most once per step).
  auto push_act = [&]() {
    int* slot = ws.h_act_ring + 16 * ws.act_slot;
    ws.act_slot = (ws.act_slot + 1) & 3;
    for (int k = 0; k < K; ++k) slot[k] = ws.h_act[k];
    HIP_CHECK(hipMemcpyAsync(act, slot, sizeof(int) * K, hipMemcpyHostToDevice, st));
  };
  KrylovResultM res;
  res.iters.assign(K, 0);
  res.resid.assign(K, 0.0);
  res.converged.assign(K, 0);
  norms(b, 0, nullptr);
  if (x_is_zero) {
    launch_zero_b<R>(N, x, ld, K, st);
    launch_copy_cvt_b<R, R>(b, ld, r, ld, N, K, st);
  } else {
    A(x, r, K);
    launch_sub_b<R>(N, b, ld, r, ld, r, ld, K, st);
  }
  norms(r, 1, nullptr);
  read_scal();
  std::vector<double> bn(K), beta(K);
  for (int k = 0; k < K; ++k) {
    bn[k] = ws.h_scal[4 * k].re;
    beta[k] = ws.h_scal[4 * k + 1].re;
  }
  auto update_active = [&]() {
    int n_act = 0;
    for (int k = 0; k < K; ++k) {
      bool done = bn[k] == 0.0 || (!fixed && beta[k] <= tol * bn[k]) || beta[k] == 0.0;
      ws.h_act[k] = done ? 0 : 1;
      n_act += ws.h_act[k];
    }
    return n_act;
  };
  int steps = 0;
  while (update_active() > 0 && steps < max_iter) {
    push_act();
    const int mm = fixed ? std::min(m, max_iter - steps) : m;
    // V_0 = r / beta (inactive columns zeroed), g = beta e_0
    launch_scale_by_inv_b<R>(r, ld, scal + 1, 4, V, ld, N, K, act, 1, st);
    launch_init_g_b(g, ldh, scal + 1, 4, K, act, st);
    for (int k = 0; k < K; ++k) ws.h_jd[k] = 0;
    // Without a preconditioner the test of step s is taken while steps s+1 and
    // s+2 are already queued (the device never waits for the host); a column
    // that met its tolerance at step s then drops the later steps it ran, which
    // changed only its Hessenberg columns after s and g entries after s+1.
    const bool lookahead = !fixed && M == nullptr && Mf == nullptr;
    constexpr int LAG = 2, NSLOT = LAG + 1;
    int tested = 0;                // steps 0..tested-1 of this cycle are tested
    int last = -1;                 // last step queued in this cycle
    int act_at[NSLOT][16];         // columns active in the step of each slot
    for (int j = 0; j < mm; ++j) {
      cx<R>* Vj = V + (long)j * K * ld;
      cx<R>* Vn = V + (long)(j + 1) * K * ld;
      cx<R>* z = Vj;
      if (M) {
        z = Z + (long)j * K * ld;
        (*M)(Vj, z, K);
      } else if (Mf) {
        if constexpr (std::is_same<R, double>::value) {
          // r is free until the restart: it holds the widened direction
          cx<float>* zf = Zf + (long)j * K * ld;
          (*Mf)(Vj, zf, K);
          launch_copy_cvt_b<float, R>(zf, ld, r, ld, N, K, st);
          z = r;
        }
      }
      A(z, Vn, K);
      cx<double>* hcol = H + (long)j * ldh;
      if (j + 1 <= 32) {
        // classical Gram-Schmidt (one or two passes, cgs_two_pass), norm,
        // scaling and Givens step
        // the look-ahead estimate goes straight to its pinned slot (no copy launch)
        launch_cgs_step<R>(V, (long)K * ld, ld, j + 1, Vn, ld, N, part, part + (long)K * pcs, pcs, nwgf, hcol, hcs, H,
                           ldh, m, ws.cs.template as<double>(), ws.sn.template as<cx<double>>(), g, j,
                           ws.resid.template as<double>(), lookahead ? ws.h_resid + 32 * (j % NSLOT) : nullptr, K,
                           act, st);
      } else {
        launch_multidot_b<R>(V, (long)K * ld, ld, j + 1, Vn, ld, N, part, pcs, nwg, K, act, st);
        launch_reduce_b(part, pcs, j + 1, nwg, hcol, hcs, 0, K, act, st);
        launch_multi_axpy_b<R>(V, (long)K * ld, ld, j + 1, nullptr, hcol, hcs, -1.0, Vn, ld, N, K, act, st);
        if (cgs_two_pass<R>(m)) {
          launch_multidot_b<R>(V, (long)K * ld, ld, j + 1, Vn, ld, N, part, pcs, nwg, K, act, st);
          launch_reduce_b(part, pcs, j + 1, nwg, y, ldh, 0, K, act, st);
          launch_reduce_b(part, pcs, j + 1, nwg, hcol, hcs, 1, K, act, st);
          launch_multi_axpy_b<R>(V, (long)K * ld, ld, j + 1, nullptr, y, ldh, -1.0, Vn, ld, N, K, act, st);
        }
        launch_multidot_b<R>(Vn, 0, ld, 1, Vn, ld, N, part, pcs, nwg, K, act, st);
        launch_reduce_b(part, pcs, 1, nwg, hcol + j + 1, hcs, 2, K, act, st);
        launch_scale_by_inv_b<R>(Vn, ld, hcol + j + 1, hcs, Vn, ld, N, K, act, 1, st);
        launch_givens_b(H, ldh, m, ws.cs.template as<double>(), ws.sn.template as<cx<double>>(), g, j,
                        ws.resid.template as<double>(), K, act, st);
      }
      ++steps;
      int still = 0;
      for (int k = 0; k < K; ++k)
        if (ws.h_act[k]) {
          ws.h_jd[k] = j + 1;
          ++res.iters[k];
        }
      if (lookahead) {
        const int slot = j % NSLOT;
        if (j + 1 > 32)
          HIP_CHECK(hipMemcpyAsync(ws.h_resid + 32 * slot, ws.resid.p, sizeof(double) * K, hipMemcpyDeviceToHost, st));
        HIP_CHECK(hipEventRecord(ws.ready[slot], st));
        for (int k = 0; k < K; ++k) act_at[slot][k] = ws.h_act[k];
        last = j;
        bool stop = false;
        while (tested <= j - LAG) {
          const int s = tested++, ps = s % NSLOT;
          HIP_CHECK(hipEventSynchronize(ws.ready[ps]));
          bool changed = false;
          for (int k = 0; k < K; ++k)
            if (act_at[ps][k] && ws.h_act[k] && ws.h_resid[32 * ps + k] <= tol * bn[k]) {
              ws.h_act[k] = 0;
              changed = true;
              for (int t = s + 1; t <= j; ++t)  // the steps it ran after s are dropped
                if (act_at[t % NSLOT][k]) --res.iters[k];
              ws.h_jd[k] = s + 1;
            }
          still = 0;
          for (int k = 0; k < K; ++k) still += ws.h_act[k];
          if (changed) push_act();
          if (still == 0) {
            stop = true;
            break;
          }
        }
        if (stop) break;
      } else if (!fixed) {
        HIP_CHECK(hipMemcpyAsync(ws.h_resid, ws.resid.p, sizeof(double) * K, hipMemcpyDeviceToHost, st));
        HIP_CHECK(hipStreamSynchronize(st));
        bool changed = false;
        for (int k = 0; k < K; ++k)
          if (ws.h_act[k] && ws.h_resid[k] <= tol * bn[k]) {
            ws.h_act[k] = 0;
            changed = true;
          }
        for (int k = 0; k < K; ++k) still += ws.h_act[k];
        if (changed) push_act();
        if (still == 0) break;
      }
      if (steps >= max_iter) break;
    }
    // the estimate slots of untested steps are reused by the next cycle
    for (int s = tested; s <= last; ++s) HIP_CHECK(hipEventSynchronize(ws.ready[s % NSLOT]));
    HIP_CHECK(hipMemcpyAsync(jd, ws.h_jd, sizeof(int) * K, hipMemcpyHostToDevice, st));
    launch_trisolve_b(H, ldh, m, g, y, jd, K, st);
    if constexpr (std::is_same<R, double>::value) {
      if (Mf)
        launch_multi_axpy_b_mixed(Zf, (long)K * ld, ld, m, jd, y, ldh, 1.0, x, ld, N, K, nullptr, st);
      else
        launch_multi_axpy_b<R>(Z, (long)K * ld, ld, m, jd, y, ldh, 1.0, x, ld, N, K, nullptr, st);
    } else {
      launch_multi_axpy_b<R>(Z, (long)K * ld, ld, m, jd, y, ldh, 1.0, x, ld, N, K, nullptr, st);
    }
    A(x, r, K);
    launch_sub_b<R>(N, b, ld, r, ld, r, ld, K, st);
    norms(r, 1, nullptr);
    read_scal();
    for (int k = 0; k < K; ++k) beta[k] = ws.h_scal[4 * k + 1].re;
    if (fixed && steps >= max_iter) break;
  }
  res.steps = steps;
  for (int k = 0; k < K; ++k) {
    res.resid[k] = bn[k] > 0 ? beta[k] / bn[k] : 0.0;
    res.converged[k] = bn[k] == 0.0 || beta[k] <= tol * bn[k];
  }
  return res;
}
template KrylovResultM fgmres_multi<double>(Ctx&, KrylovWSm<double>&, int, long, const OpM<double>&,
                                            const OpM<double>*, const cx<double>*, cx<double>*, double, int, bool,
                                            bool, const OpMf*);
template KrylovResultM fgmres_multi<float>(Ctx&, KrylovWSm<float>&, int, long, const OpM<float>&, const OpM<float>*,
                                           const cx<float>*, cx<float>*, double, int, bool, bool, const OpMf*);

template KrylovResult fgmres<double>(Ctx&, KrylovWS<double>&, long,
                                     const std::function<void(const cx<double>*, cx<double>*)>&,
                                     const std::function<void(const cx<double>*, cx<double>*)>*, const cx<double>*,
                                     cx<double>*, double, int, bool, bool);
template KrylovResult fgmres<float>(Ctx&, KrylovWS<float>&, long,
                                    const std::function<void(const cx<float>*, cx<float>*)>&,
                                    const std::function<void(const cx<float>*, cx<float>*)>*, const cx<float>*,
                                    cx<float>*, double, int, bool, bool);

// ---------------------------------------------------------------------------
void Ctx::ensure_32() {
  if (have_32) return;
  U32.ensure(sizeof(cx<float>) * (size_t)g.V * 36);
  H32.ensure(sizeof(float) * (size_t)g.V * 72);
  M32.ensure(sizeof(float) * (size_t)g.V * 36);
  launch_cvt_cx<float>((long)g.V * 36, U64.as<cx<double>>(), U32.p, st);
  launch_cvt_real((long)g.V * 72, H64.as<double>(), H32.as<float>(), st);
  launch_cvt_real((long)g.V * 36, M64.as<double>(), M32.as<float>(), st);
  have_32 = true;
}
void Ctx::ensure_16(int kind) {
  ensure_32();
  if (u16_kind == kind) return;
  U16.ensure(4 * (size_t)g.V * 36);
  if (kind == DDAMG_FP16) launch_cvt_cx<f16>((long)g.V * 36, U64.as<cx<double>>(), U16.p, st);
  else launch_cvt_cx<bf16>((long)g.V * 36, U64.as<cx<double>>(), U16.p, st);
  u16_kind = kind;
}
void Ctx::rebuild_odd_inverse() {
  launch_odd_inverse(g, H64.as<double>(), mu_odd, M64.as<double>(), st);
  if (have_32) launch_cvt_real((long)g.V * 36, M64.as<double>(), M32.as<float>(), st);
}
void Ctx::dirac64(const cx<double>* in, cx<double>* out, Twist tw) { dirac64_multi(in, out, 1, 0, tw); }
void Ctx::dirac64_multi(const cx<double>* in, cx<double>* out, int K, long ld, Twist tw) {
  // per site links and clover once (1152 bytes), spinor in and out per field
  // (384 bytes)
  TimeScope ts(timer, 0, (1152.0 + 384.0 * K) * (double)g.V);
  launch_dirac_multi<double, double>(g, U64.p, H64.as<double>(), tw, K, ld, in, out, st);
}
void Ctx::upload_fine(const void* src, int on_device, cx<double>* dst64) {
  const cx<double>* s = (const cx<double>*)src;
  if (!on_device) {
    lex.ensure(sizeof(cx<double>) * fine_len());
    HIP_CHECK(hipMemcpyAsync(lex.p, src, sizeof(cx<double>) * fine_len(), hipMemcpyHostToDevice, st));
    s = lex.as<cx<double>>();
  }
  launch_from_lex<double>(g, s, dst64, 12, st);
}
void Ctx::download_fine(const cx<double>* src64, void* dst, int on_device) {
  if (on_device) {
    launch_to_lex<double>(g, src64, (cx<double>*)dst, 12, st);
    return;
  }
  lex.ensure(sizeof(cx<double>) * fine_len());
  launch_to_lex<double>(g, src64, lex.as<cx<double>>(), 12, st);
  HIP_CHECK(hipMemcpyAsync(dst, lex.p, sizeof(cx<double>) * fine_len(), hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
}

// ---------------------------------------------------------------------------
static void lex_coords(const int L[4], int s, int x[4]) {
  x[3] = s % L[3];
  s /= L[3];
  x[2] = s % L[2];
  s /= L[2];
  x[1] = s % L[1];
  x[0] = s / L[1];
}
static int lex_of(const int L[4], const int x[4]) { return ((x[0] * L[1] + x[1]) * L[2] + x[2]) * L[3] + x[3]; }

static void build_order(CoarseGeo& G) {
  G.nsites = G.L[0] * G.L[1] * G.L[2] * G.L[3];
  G.order.assign(G.nsites, 0);
  G.lexof.assign(G.nsites, 0);
  int k = 0;
  for (int par = 0; par < 2; ++par)
    for (int s = 0; s < G.nsites; ++s) {
      int x[4];
      lex_coords(G.L, s, x);
      if (((x[0] + x[1] + x[2] + x[3]) & 1) == par) {
        G.order[s] = k;
        G.lexof[k] = s;
        ++k;
      }
    }
  G.neven = 0;
  for (int s = 0; s < G.nsites; ++s) {
    int x[4];
    lex_coords(G.L, s, x);
    if (((x[0] + x[1] + x[2] + x[3]) & 1) == 0) ++G.neven;
  }
  std::vector<int> nb((size_t)G.nsites * 8);
  for (int o = 0; o < G.nsites; ++o) {
    int x[4];
    lex_coords(G.L, G.lexof[o], x);
    for (int mu = 0; mu < 4; ++mu)
      for (int d = 0; d < 2; ++d) {
        int y[4] = {x[0], x[1], x[2], x[3]};
        y[mu] = (y[mu] + (d == 0 ? 1 : -1) + G.L[mu]) % G.L[mu];
        nb[(size_t)o * 8 + d * 4 + mu] = G.order[lex_of(G.L, y)];
      }
  }
  G.nbr.alloc(sizeof(int) * nb.size());
  HIP_CHECK(hipMemcpy(G.nbr.p, nb.data(), sizeof(int) * nb.size(), hipMemcpyHostToDevice));
  G.d_order.alloc(sizeof(int) * G.nsites);
  HIP_CHECK(hipMemcpy(G.d_order.p, G.order.data(), sizeof(int) * G.nsites, hipMemcpyHostToDevice));
}

// aggregation tables of level G towards the next level Gn (blocks ab)
static void build_agg(CoarseGeo& G, const CoarseGeo& Gn, const int ab[4]) {
  for (int d = 0; d < 4; ++d) G.ab[d] = ab[d];
  G.asz = ab[0] * ab[1] * ab[2] * ab[3];
  G.nagg = Gn.nsites;
  std::vector<int> as((size_t)G.nagg * G.asz), sa(G.nsites);
  for (int A = 0; A < G.nagg; ++A) {
    int X[4];
    lex_coords(Gn.L, Gn.lexof[A], X);
    for (int j = 0; j < G.asz; ++j) {
      int l[4];
      lex_coords(ab, j, l);
      int x[4];
      for (int d = 0; d < 4; ++d) x[d] = X[d] * ab[d] + l[d];
      int o = G.order[lex_of(G.L, x)];
      as[(size_t)A * G.asz + j] = o;
      sa[o] = A;
    }
  }
  G.agg_sites.alloc(sizeof(int) * as.size());
  HIP_CHECK(hipMemcpy(G.agg_sites.p, as.data(), sizeof(int) * as.size(), hipMemcpyHostToDevice));
  G.site_agg.alloc(sizeof(int) * sa.size());
  HIP_CHECK(hipMemcpy(G.site_agg.p, sa.data(), sizeof(int) * sa.size(), hipMemcpyHostToDevice));
}

static void build_sap_blocks(CoarseGeo& G, const int sb[4]) {
  int nb[4];
  for (int d = 0; d < 4; ++d) {
    G.sb[d] = sb[d];
    if (sb[d] <= 0 || G.L[d] % sb[d]) throw Error(INVALID_ARG, "coarse SAP block does not divide the coarse lattice");
    nb[d] = G.L[d] / sb[d];
    if (nb[d] % 2) throw Error(INVALID_ARG, "coarse SAP needs an even number of blocks per direction");
  }
  G.ssz = sb[0] * sb[1] * sb[2] * sb[3];
  if (G.ssz > 16) throw Error(INVALID_ARG, "coarse SAP blocks are limited to 16 sites");
  G.nsblk = nb[0] * nb[1] * nb[2] * nb[3];
  std::vector<int> sites, nbr;
  for (int col = 0; col < 2; ++col) {
    G.nsblk_col[col] = 0;
    for (int Bl = 0; Bl < G.nsblk; ++Bl) {
      int Bc[4];
      lex_coords(nb, Bl, Bc);
      if (((Bc[0] + Bc[1] + Bc[2] + Bc[3]) & 1) != col) continue;
      G.nsblk_col[col]++;
      for (int j = 0; j < G.ssz; ++j) {
        int l[4];
        lex_coords(sb, j, l);
        int x[4];
        for (int d = 0; d < 4; ++d) x[d] = Bc[d] * sb[d] + l[d];
        sites.push_back(G.order[lex_of(G.L, x)]);
        for (int dir = 0; dir < 2; ++dir)
          for (int mu = 0; mu < 4; ++mu) {
            int m2[4] = {l[0], l[1], l[2], l[3]};
            m2[mu] += dir == 0 ? 1 : -1;
            nbr.push_back((m2[mu] >= 0 && m2[mu] < sb[mu]) ? lex_of(sb, m2) : -1);
          }
      }
    }
  }
  G.sap_sites.alloc(sizeof(int) * sites.size());
  HIP_CHECK(hipMemcpy(G.sap_sites.p, sites.data(), sizeof(int) * sites.size(), hipMemcpyHostToDevice));
  G.sap_nbr.alloc(sizeof(int) * nbr.size());
  HIP_CHECK(hipMemcpy(G.sap_nbr.p, nbr.data(), sizeof(int) * nbr.size(), hipMemcpyHostToDevice));
}

// ---------------------------------------------------------------------------
template <class R, class S>
struct MG : MGBase {
  Ctx& c;
  ddamg_params p;
  int L;
  std::vector<std::unique_ptr<CoarseGeo>> geos;  // index = level (0 unused)
  DevBuf f2c;
  const void* U = nullptr;
  const R* Hf = nullptr;
  const R* Mf = nullptr;
  int Nv[3] = {0, 0, 0};
  DevBuf Vraw[3], Q[3];
  DevBuf D64[4], DS[4], Minvc, Xs, invscr;
  size_t xs_bytes = 0;  // assembly scratch (transient: taken per assembly, released after the setup)
  double tw[4] = {0, 0, 0, 0};  // twist of each coarse level (tw[0]: the fine mean)
  Twist tw0;                      // the fine level's twists
  double dtw_asm = 0;             // parity rest of the fine twist in the coarse site blocks
  DevBuf fx, fb, fr;              // fine R vectors
  DevBuf rc[4], ec[4], wk[4][4];  // coarse vectors per level
  KrylovWS<R> kws[4];
  std::function<void(const cx<R>*, cx<R>*)> Aop[4], Mop[4];
  // lock-step (K-column) forms: buffers sized for Km columns
  int Km = 0;
  DevBuf rcm[4], ecm[4], wkm[4][2], fxm;
  KrylovWSm<R> kwsm[4];
  OpM<R> AopM[4], MopM[4];

  MG(Ctx& c_, const ddamg_params& p_) : c(c_), p(p_), L(p_.levels) {
    const Geom& g = c.g;
    for (int l = 0; l < L - 1; ++l) Nv[l] = p.nvec[l];
    if (L < 2 || L > 3) throw Error(INVALID_ARG, "levels must be 2 or 3");
    for (int d = 0; d < 4; ++d)
      if (p.block[0][d] != g.b[d]) throw Error(INVALID_ARG, "block[0] must equal the block given to ddamg_create");
    if (Nv[0] < 1 || 2 * Nv[0] > 64 || Nv[0] > g.bs * 6)
      throw Error(INVALID_ARG, "nvec[0] must satisfy 1 <= nvec <= 32 and nvec <= 6 * block sites");
    geos.resize(L);
    // level 1
    geos[1].reset(new CoarseGeo());
    for (int d = 0; d < 4; ++d) geos[1]->L[d] = g.nb[d];
    geos[1]->n = 2 * Nv[0];
    build_order(*geos[1]);
    for (int l = 2; l < L; ++l) {
      CoarseGeo& Gp = *geos[l - 1];
      geos[l].reset(new CoarseGeo());
      for (int d = 0; d < 4; ++d) {
        int b = p.block[l - 1][d];
        if (b <= 0 || Gp.L[d] % b) throw Error(INVALID_ARG, "block does not divide the coarse lattice");
        geos[l]->L[d] = Gp.L[d] / b;
      }
      if (Nv[l - 1] < 1 || 2 * Nv[l - 1] > 64) throw Error(INVALID_ARG, "nvec must satisfy 1 <= nvec <= 32");
      int asz = p.block[l - 1][0] * p.block[l - 1][1] * p.block[l - 1][2] * p.block[l - 1][3];
      if (Nv[l - 1] > asz * Gp.n / 2) throw Error(INVALID_ARG, "nvec exceeds the rows of an aggregate half");
      if (asz * Gp.n / 2 > 1024) throw Error(INVALID_ARG, "coarse aggregate too large");
      geos[l]->n = 2 * Nv[l - 1];
      build_order(*geos[l]);
      build_agg(Gp, *geos[l], p.block[l - 1]);
      build_sap_blocks(Gp, p.coarse_sap_block);
    }
    for (int d = 0; d < 4; ++d)
      if (geos[L - 1]->L[d] % 2) throw Error(INVALID_ARG, "the coarsest lattice needs even extents (odd-even)");
    // fine block -> level-1 ordered index
    {
      std::vector<int> m(g.nblocks);
      for (int B = 0; B < g.nblocks; ++B) m[B] = geos[1]->order[B];
      f2c.alloc(sizeof(int) * g.nblocks);
      HIP_CHECK(hipMemcpy(f2c.p, m.data(), sizeof(int) * g.nblocks, hipMemcpyHostToDevice));
    }
    // operator data of the fine level in this precision
    if constexpr (std::is_same<R, double>::value) {
      U = c.U64.p;
      Hf = c.H64.as<double>();
      Mf = c.M64.as<double>();
    } else {
      if constexpr (std::is_same<S, float>::value) {
        c.ensure_32();
        U = c.U32.p;
      } else {
        c.ensure_16(std::is_same<S, f16>::value ? DDAMG_FP16 : DDAMG_BF16);
        U = c.U16.p;
      }
      Hf = c.H32.template as<float>();
      Mf = c.M32.template as<float>();
    }
    set_twists(c.twist());
    // allocations
    long fl = c.fine_len();
    fx.alloc(sizeof(cx<R>) * fl);
    fb.alloc(sizeof(cx<R>) * fl);
    fr.alloc(sizeof(cx<R>) * fl);
    // the raw test vectors live through the setup only, unless kept for an update
    const bool vt = !p.keep_test_vectors;
    Vraw[0].alloc(sizeof(cx<R>) * fl * Nv[0], vt);
    Q[0].alloc(sizeof(cx<R>) * fl * Nv[0]);
    size_t maxnn = 0;
    for (int l = 1; l < L; ++l) {
      CoarseGeo& G = *geos[l];
      long len = (long)G.nsites * G.n;
      size_t nn = (size_t)G.n * G.n;
      maxnn = std::max(maxnn, nn * G.nsites);
      D64[l].alloc(sizeof(cx<double>) * nn * 5 * G.nsites);
      if (!std::is_same<S, double>::value) DS[l].alloc(sizeof(typename store_traits<S>::elem) * nn * 5 * G.nsites);
      rc[l].alloc(sizeof(cx<R>) * len);
      ec[l].alloc(sizeof(cx<R>) * len);
      for (int k = 0; k < 4; ++k) wk[l][k].alloc(sizeof(cx<R>) * len);
      if (l < L - 1) {
        Vraw[l].alloc(sizeof(cx<R>) * len * Nv[l]);
        Q[l].alloc(sizeof(cx<R>) * len * Nv[l]);
        kws[l].init(p.inter_restart, len, len, true);
      } else {
        kws[l].init(p.coarse_restart, len, (long)G.neven * G.n, false);
        Minvc.alloc(sizeof(cx<R>) * nn * (G.nsites - G.neven));
        invscr.alloc(sizeof(cx<double>) * nn * 2 * (G.nsites - G.neven));
      }
    }
    xs_bytes = sizeof(cx<double>) * maxnn;
    for (int l = 1; l < L; ++l) {
      CoarseGeo& G = *geos[l];
      CGeom cg = G.cg();
      const void* Dp = Dst(l);
      if (l == L - 1) {
        cx<R>* t = wk[l][0].template as<cx<R>>();
        Aop[l] = [this, cg, l, t](const cx<R>* in, cx<R>* out) {
          TimeScope ts(c.timer, 5);
          launch_coarse_hop_inv_odd<R, S>(cg, Dst(l), Minvc.template as<cx<R>>(), in, t, 0, c.st);
          launch_coarse_schur_even<R, S>(cg, Dst(l), tw[l], in, t, out, 0, c.st);
        };
      } else {
        Aop[l] = [this, cg, l](const cx<R>* in, cx<R>* out) {
          TimeScope ts(c.timer, 2);
          launch_coarse_apply<R, S>(cg, Dst(l), tw[l], in, out, c.st);
        };
        Mop[l] = [this, l](const cx<R>* in, cx<R>* out) { vcycle(l, in, out); };
      }
      (void)Dp;
    }
  }

  const void* Dst(int l) const {
    if constexpr (std::is_same<S, double>::value) return D64[l].p;
    else return DS[l].p;
  }

  // coarse levels carry the mean of the two fine twists (delta times it on the
  // coarsest); the parity rest enters their site blocks through the assembly
  void set_twists(const Twist& t) {
    tw0 = t;
    const double mu = t.mean();
    tw[0] = mu;
    for (int l = 1; l < L; ++l) tw[l] = (l == L - 1) ? p.coarse_mu_factor * mu : mu;
  }

  int nlev() const override { return L; }
  const CoarseGeo& geo(int l) const override { return *geos[l]; }

  // ---- level operations ----------------------------------------------------
  void fine_dirac(const cx<R>* in, cx<R>* out) {
    TimeScope ts(c.timer, 4);
    launch_dirac<R, S>(c.g, U, Hf, tw0, in, out, c.st);
  }
  void fine_sap(const cx<R>* b, cx<R>* x, int iters, int nmr) {
    for (int it = 0; it < iters; ++it)
      for (int col = 0; col < 2; ++col) {
        TimeScope ts(c.timer, 1, sap_sweep_bytes<R, S>(c.g, 1), sap_sweep_flops(c.g, 1, nmr));
        launch_sap<R, S>(c.g, col, U, Hf, Mf, tw0, b, x, nmr, c.st);
      }
  }
  // SAP on K fine fields (stride = fine length), one launch per colour
  void fine_sap_m(const cx<R>* b, cx<R>* x, int K, int iters, int nmr) {
    for (int it = 0; it < iters; ++it)
      for (int col = 0; col < 2; ++col) {
        TimeScope ts(c.timer, 1, sap_sweep_bytes<R, S>(c.g, K), sap_sweep_flops(c.g, K, nmr));
        launch_sap_multi<R, S>(c.g, col, U, Hf, Mf, tw0, b, x, nmr, K, c.fine_len(), c.st);
      }
  }
  // SAP on K fields of an intermediate level: residuals of all fields in one
  // launch, then one launch per colour for all fields
  void coarse_sap_m(int l, const cx<R>* b, cx<R>* x, int K, int iters) {
    CoarseGeo& G = *geos[l];
    CGeom cg = G.cg();
    const long len = level_len(l);
    cx<R>* r = wkm[l][1].template as<cx<R>>();
    for (int it = 0; it < iters; ++it)
      for (int col = 0; col < 2; ++col) {
        {
          TimeScope ts(c.timer, 2);
          bool done = false;
          if constexpr (kMfma) {
            if (mfma_level(l)) {
              // the residual is read on the sites of this colour's blocks only
              const int off = col == 0 ? 0 : G.nsblk_col[0];
              launch_coarse_apply_mrhs<S>(cg, Dst(l), tw[l], K, len, x, b, r, c.st,
                                          G.sap_sites.template as<int>() + off * G.ssz, G.nsblk_col[col] * G.ssz);
              done = true;
            }
          }
          if (!done)
            for (int k = 0; k < K; ++k)
              launch_coarse_residual<R, S>(cg, Dst(l), tw[l], b + k * len, x + k * len, r + k * len, c.st);
        }
        int off = col == 0 ? 0 : G.nsblk_col[0];
        if constexpr (kMfma) {
          if (mfma_level(l) && G.ssz <= 16) {
            launch_coarse_sap_mrhs<S>(cg, Dst(l), tw[l], G.nsblk_col[col], G.ssz,
                                      G.sap_sites.template as<int>() + off * G.ssz,
                                      G.sap_nbr.template as<int>() + (long)off * G.ssz * 8, r, x, p.coarse_mr_steps, K,
                                      len, c.st);
            continue;
          }
        }
        launch_coarse_sap_multi<R, S>(cg, Dst(l), tw[l], G.nsblk_col[col], G.ssz,
                                      G.sap_sites.template as<int>() + off * G.ssz,
                                      G.sap_nbr.template as<int>() + (long)off * G.ssz * 8, r, x, p.coarse_mr_steps, K,
                                      len, c.st);
      }
  }
  void coarse_sap(int l, const cx<R>* b, cx<R>* x, int iters) {
    CoarseGeo& G = *geos[l];
    CGeom cg = G.cg();
    cx<R>* r = wk[l][1].template as<cx<R>>();
    for (int it = 0; it < iters; ++it)
      for (int col = 0; col < 2; ++col) {
        {
          TimeScope ts(c.timer, 2);
          launch_coarse_residual<R, S>(cg, Dst(l), tw[l], b, x, r, c.st);
        }
        int off = col == 0 ? 0 : G.nsblk_col[0];
        launch_coarse_sap<R, S>(cg, Dst(l), tw[l], G.nsblk_col[col], G.ssz, G.sap_sites.template as<int>() + off * G.ssz,
                                G.sap_nbr.template as<int>() + (long)off * G.ssz * 8, r, x, p.coarse_mr_steps, c.st);
      }
  }
  void restrict_(int l, const cx<R>* in, cx<R>* out) {
    TimeScope ts(c.timer, 3);
    if (l == 0) {
      launch_restrict_fine<R>(c.g, Nv[0], Q[0].template as<cx<R>>(), c.fine_len(), in, f2c.template as<int>(), out,
                              c.st);
    } else {
      CoarseGeo& G = *geos[l];
      launch_restrict_coarse<R>(G.n, Nv[l], G.nagg, G.asz, G.agg_sites.template as<int>(), Q[l].template as<cx<R>>(),
                                (long)G.nsites * G.n, in, out, c.st);
    }
  }
  // K columns between coarse levels l >= 1 and l + 1 (strides ld, ldc)
  void restrict_m(int l, const cx<R>* in, long ld, cx<R>* out, long ldc, int K) {
    TimeScope ts(c.timer, 3);
    CoarseGeo& G = *geos[l];
    launch_restrict_coarse_m<R>(G.n, Nv[l], G.nagg, G.asz, G.agg_sites.template as<int>(), Q[l].template as<cx<R>>(),
                                (long)G.nsites * G.n, in, ld, out, ldc, K, c.st);
  }
  void prolong_m(int l, const cx<R>* in, long ldc, cx<R>* out, long ld, int K) {
    TimeScope ts(c.timer, 3);
    CoarseGeo& G = *geos[l];
    launch_prolong_coarse_m<R>(G.n, Nv[l], G.nsites, G.site_agg.template as<int>(), Q[l].template as<cx<R>>(),
                               (long)G.nsites * G.n, in, ldc, out, ld, K, 0, c.st);
  }
  void prolong_(int l, const cx<R>* in, cx<R>* out, int acc) {
    TimeScope ts(c.timer, 3);
    if (l == 0) {
      launch_prolong_fine<R>(c.g, Nv[0], Q[0].template as<cx<R>>(), c.fine_len(), in, f2c.template as<int>(), out, acc,
                             c.st);
    } else {
      CoarseGeo& G = *geos[l];
      launch_prolong_coarse<R>(G.n, Nv[l], G.nsites, G.site_agg.template as<int>(), Q[l].template as<cx<R>>(),
                               (long)G.nsites * G.n, in, out, acc, c.st);
    }
  }

  void coarse_solve(int l, const cx<R>* b, cx<R>* x) {
    CoarseGeo& G = *geos[l];
    CGeom cg = G.cg();
    KrylovResult kr;
    if (l == L - 1) {
      cx<R>* t = wk[l][2].template as<cx<R>>();
      cx<R>* rhs = wk[l][3].template as<cx<R>>();
      // t_o = D_oo^{-1} b_o ;  rhs_e = b_e - D_eo t_o
      hipLaunchKernelGGL(k_minv_odd<R>, dim3((G.nsites - G.neven + 3) / 4), dim3(256), 0, c.st, cg,
                         Minvc.template as<cx<R>>(), b, t);
      launch_coarse_schur_even<R, S>(cg, Dst(l), tw[l], b, t, rhs, 1, c.st);
      kr = fgmres<R>(c, kws[l], (long)G.neven * G.n, Aop[l], nullptr, rhs, x, p.coarse_tol, p.coarse_max_iter,
                     p.fixed_iters != 0, true);
      // x_o = D_oo^{-1} (b_o - D_oe x_e)
      launch_coarse_hop_inv_odd_base<R, S>(cg, Dst(l), Minvc.template as<cx<R>>(), x, b, x, c.st);
    } else {
      kr = fgmres<R>(c, kws[l], (long)G.nsites * G.n, Aop[l], &Mop[l], b, x, p.inter_tol, p.inter_max_iter,
                     p.fixed_iters != 0, true);
    }
    coarse_iters[l] += kr.iters;
  }

  // x = cycle(v) on level l, x0 = 0
  void vcycle(int l, const cx<R>* v, cx<R>* x) {
    if (l == 0) {
      ++vcycles;
      const cx<R>* rin = v;
      if (p.sap_pre > 0) {
        launch_zero<R>(c.fine_len(), x, c.st);
        fine_sap(v, x, p.sap_pre, p.mr_steps);
        fine_dirac(x, fr.template as<cx<R>>());
        launch_sub<R>(c.fine_len(), v, fr.template as<cx<R>>(), fr.template as<cx<R>>(), c.st);
        rin = fr.template as<cx<R>>();
      }
      restrict_(0, rin, rc[1].template as<cx<R>>());
      coarse_solve(1, rc[1].template as<cx<R>>(), ec[1].template as<cx<R>>());
      prolong_(0, ec[1].template as<cx<R>>(), x, p.sap_pre > 0);
      fine_sap(v, x, p.sap_post, p.mr_steps);
    } else {
      restrict_(l, v, rc[l + 1].template as<cx<R>>());
      coarse_solve(l + 1, rc[l + 1].template as<cx<R>>(), ec[l + 1].template as<cx<R>>());
      prolong_(l, ec[l + 1].template as<cx<R>>(), x, 0);
      coarse_sap(l, v, x, p.coarse_sap_post);
    }
  }

  // ---- lock-step forms on K columns (column k of a level-l K-vector at k * len(l))
  static constexpr bool kMfma = std::is_same<S, f16>::value || std::is_same<S, bf16>::value;
  bool mfma_level(int l) const { return kMfma && geos[l]->n % 16 == 0 && geos[l]->n <= 64; }

  void ensure_multi(int K) {
    if (K <= Km) return;
    for (int l = 1; l < L; ++l) {
      CoarseGeo& G = *geos[l];
      long len = (long)G.nsites * G.n;
      rcm[l].ensure(sizeof(cx<R>) * len * K);
      ecm[l].ensure(sizeof(cx<R>) * len * K);
      for (int k = 0; k < 2; ++k) wkm[l][k].ensure(sizeof(cx<R>) * len * K);
      // the lock-step Krylov bases are transient: the setup's batch width and
      // the solve's group width differ (released at the end of the setup)
      if (l < L - 1) kwsm[l].init(p.inter_restart, K, len, len, true, false, true);
      else kwsm[l].init(p.coarse_restart, K, len, (long)G.neven * G.n, false, false, true);
      CGeom cg = G.cg();
      if (l == L - 1) {
        cx<R>* t = wkm[l][0].template as<cx<R>>();
        AopM[l] = [this, cg, l, t, len](const cx<R>* in, cx<R>* out, int K_) {
          TimeScope ts(c.timer, 5);
          if constexpr (kMfma) {
            if (mfma_level(l)) {
              launch_coarse_hop_inv_odd_mrhs<S>(cg, Dst(l), Minvc.template as<cx<R>>(), K_, len, in, nullptr, t,
                                                c.st);
              launch_coarse_schur_even_mrhs<S>(cg, Dst(l), tw[l], K_, len, in, t, out, 0, c.st);
              return;
            }
          }
          for (int k = 0; k < K_; ++k) {
            launch_coarse_hop_inv_odd<R, S>(cg, Dst(l), Minvc.template as<cx<R>>(), in + k * len, t + k * len, 0,
                                            c.st);
            launch_coarse_schur_even<R, S>(cg, Dst(l), tw[l], in + k * len, t + k * len, out + k * len, 0, c.st);
          }
        };
      } else {
        AopM[l] = [this, cg, l, len](const cx<R>* in, cx<R>* out, int K_) {
          TimeScope ts(c.timer, 2);
          if constexpr (kMfma) {
            if (mfma_level(l)) {
              launch_coarse_apply_mrhs<S>(cg, Dst(l), tw[l], K_, len, in, nullptr, out, c.st);
              return;
            }
          }
          for (int k = 0; k < K_; ++k) launch_coarse_apply<R, S>(cg, Dst(l), tw[l], in + k * len, out + k * len, c.st);
        };
        MopM[l] = [this, l](const cx<R>* in, cx<R>* out, int K_) { vcycle_m(l, in, out, K_); };
      }
    }
    Km = K;
  }

  void coarse_solve_m(int l, const cx<R>* b, cx<R>* x, int K) {
    CoarseGeo& G = *geos[l];
    CGeom cg = G.cg();
    const long len = (long)G.nsites * G.n;
    KrylovResultM kr;
    if (l == L - 1) {
      cx<R>* t = wkm[l][0].template as<cx<R>>();
      cx<R>* rhs = wkm[l][1].template as<cx<R>>();
      for (int k = 0; k < K; ++k)
        hipLaunchKernelGGL(k_minv_odd<R>, dim3((G.nsites - G.neven + 3) / 4), dim3(256), 0, c.st, cg,
                           Minvc.template as<cx<R>>(), b + k * len, t + k * len);
      bool done = false;
      if constexpr (kMfma) {
        if (mfma_level(l)) {
          launch_coarse_schur_even_mrhs<S>(cg, Dst(l), tw[l], K, len, b, t, rhs, 1, c.st);
          done = true;
        }
      }
      if (!done)
        for (int k = 0; k < K; ++k)
          launch_coarse_schur_even<R, S>(cg, Dst(l), tw[l], b + k * len, t + k * len, rhs + k * len, 1, c.st);
      kr = fgmres_multi<R>(c, kwsm[l], K, (long)G.neven * G.n, AopM[l], nullptr, rhs, x, p.coarse_tol,
                           p.coarse_max_iter, p.fixed_iters != 0, true);
      done = false;
      if constexpr (kMfma) {
        if (mfma_level(l)) {
          launch_coarse_hop_inv_odd_mrhs<S>(cg, Dst(l), Minvc.template as<cx<R>>(), K, len, x, b, x, c.st);
          done = true;
        }
      }
      if (!done)
        for (int k = 0; k < K; ++k)
          launch_coarse_hop_inv_odd_base<R, S>(cg, Dst(l), Minvc.template as<cx<R>>(), x + k * len, b + k * len,
                                               x + k * len, c.st);
    } else {
      kr = fgmres_multi<R>(c, kwsm[l], K, len, AopM[l], &MopM[l], b, x, p.inter_tol, p.inter_max_iter,
                           p.fixed_iters != 0, true);
    }
    for (int k = 0; k < K; ++k) coarse_iters[l] += kr.iters[k];
  }

  // x = cycle(v) on level l for K columns, x0 = 0
  void vcycle_m(int l, const cx<R>* v, cx<R>* x, int K) {
    const long len = level_len(l), lenc = level_len(l + 1);
    cx<R>* rc_ = rcm[l + 1].template as<cx<R>>();
    cx<R>* ec_ = ecm[l + 1].template as<cx<R>>();
    if (l == 0) {
      vcycles += K;
      if (p.sap_pre > 0) {
        launch_zero<R>(len * K, x, c.st);
        fine_sap_m(v, x, K, p.sap_pre, p.mr_steps);
      }
      if (p.sap_pre > 0) {
        for (int k = 0; k < K; ++k) {
          fine_dirac(x + k * len, fr.template as<cx<R>>());
          launch_sub<R>(len, v + k * len, fr.template as<cx<R>>(), fr.template as<cx<R>>(), c.st);
          restrict_(0, fr.template as<cx<R>>(), rc_ + k * lenc);
        }
      } else {
        TimeScope ts(c.timer, 3);
        launch_restrict_fine_m<R>(c.g, Nv[0], Q[0].template as<cx<R>>(), len, v, len, K, f2c.template as<int>(), rc_,
                                  lenc, c.st);
      }
      coarse_solve_m(1, rc_, ec_, K);
      {
        TimeScope ts(c.timer, 3);
        launch_prolong_fine_m<R>(c.g, Nv[0], Q[0].template as<cx<R>>(), len, ec_, lenc, K, f2c.template as<int>(), x,
                                 len, p.sap_pre > 0, c.st);
      }
      fine_sap_m(v, x, K, p.sap_post, p.mr_steps);
    } else {
      restrict_m(l, v, len, rc_, lenc, K);
      coarse_solve_m(l + 1, rc_, ec_, K);
      prolong_m(l, ec_, lenc, x, len, K);
      coarse_sap_m(l, v, x, K, p.coarse_sap_post);
    }
  }

  void load_fine_init(const cx<float>* v) override {
    const long len = c.fine_len();
    for (int i = 0; i < Nv[0]; ++i) load_fine_vec(i, v + (long)i * len);
    c.sync();
  }
  void load_fine_vec(int i, const cx<float>* v) override {
    const long len = c.fine_len();
    launch_copy_cvt<float, R>(v, Vraw[0].template as<cx<R>>() + (long)i * len, len, c.st);
    loaded[0] = true;
  }
  void adopt_vectors(MGBase& prev_) override {
    auto* prev = dynamic_cast<MG<R, S>*>(&prev_);
    if (!prev || prev->L != L) throw Error(INVALID_ARG, "the previous hierarchy has another precision or depth");
    for (int l = 0; l < L - 1; ++l)
      if (prev->Nv[l] != Nv[l] || prev->Q[l].bytes != Vraw[l].bytes || !prev->Q[l].p)
        throw Error(INVALID_ARG, "the previous hierarchy has other test vector counts or aggregates");
    for (int l = 0; l < L - 1; ++l) {
      Vraw[l].swap(prev->Vraw[l].p ? prev->Vraw[l] : prev->Q[l]);
      loaded[l] = true;
    }
  }
  DevBuf fbm;
  void precond_multi(const cx<double>* v, cx<double>* z, int K) override {
    ensure_multi(K);
    const long n = c.fine_len();
    if constexpr (std::is_same<R, double>::value) {
      vcycle_m(0, v, z, K);
    } else {
      fbm.ensure(sizeof(cx<R>) * n * K, true);
      fxm.ensure(sizeof(cx<R>) * n * K, true);
      launch_copy_cvt_b<double, R>(v, n, fbm.template as<cx<R>>(), n, n, K, c.st);
      vcycle_m(0, fbm.template as<cx<R>>(), fxm.template as<cx<R>>(), K);
      launch_copy_cvt_b<R, double>(fxm.template as<cx<R>>(), n, z, n, n, K, c.st);
    }
  }
  void precond_multi_f32(const cx<double>* v, cx<float>* z, int K) override {
    if constexpr (std::is_same<R, double>::value) {
      throw Error(INVALID_ARG, "FP32 directions need a reduced-precision hierarchy");
    } else {
      ensure_multi(K);
      const long n = c.fine_len();
      fbm.ensure(sizeof(cx<R>) * n * K, true);
      launch_copy_cvt_b<double, R>(v, n, fbm.template as<cx<R>>(), n, n, K, c.st);
      vcycle_m(0, fbm.template as<cx<R>>(), z, K);
    }
  }
  void precond(const cx<double>* v, cx<double>* z) override {
    if constexpr (std::is_same<R, double>::value) {
      vcycle(0, v, z);
    } else {
      long n = c.fine_len();
      launch_copy_cvt<double, R>(v, fb.template as<cx<R>>(), n, c.st);
      vcycle(0, fb.template as<cx<R>>(), fx.template as<cx<R>>());
      launch_copy_cvt<R, double>(fx.template as<cx<R>>(), z, n, c.st);
    }
  }

  void set_twist(const Twist& t) override {
    set_twists(t);
    if (t.half_diff() != dtw_asm) {
      // the parity rest lives in the coarse site blocks: Galerkin again from
      // the same P (this also rebuilds the coarsest odd-site inverses)
      for (int l = 0; l < L - 1; ++l) assemble_next(l);
      Xs.release();
      return;
    }
    CoarseGeo& G = *geos[L - 1];
    launch_coarse_odd_inverse<R>(G.cg(), D64[L - 1].template as<cx<double>>(), tw[L - 1],
                                 invscr.template as<cx<double>>(), Minvc.template as<cx<R>>(), c.st);
  }

  // ---- setup ---------------------------------------------------------------
  long level_len(int l) const { return l == 0 ? c.fine_len() : (long)geos[l]->nsites * geos[l]->n; }

  void upload_level(int l, const void* src, int on_device, cx<double>* dst) {
    if (l == 0) {
      c.upload_fine(src, on_device, dst);
      return;
    }
    CoarseGeo& G = *geos[l];
    long len = level_len(l);
    const cx<double>* s = (const cx<double>*)src;
    if (!on_device) {
      c.lex.ensure(sizeof(cx<double>) * std::max(len, c.fine_len()));
      HIP_CHECK(hipMemcpyAsync(c.lex.p, src, sizeof(cx<double>) * len, hipMemcpyHostToDevice, c.st));
      s = c.lex.template as<cx<double>>();
    }
    permute<double, double>(G.n, G.nsites, G.d_order.template as<int>(), s, dst, 1, c.st);
  }
  void download_level(int l, const cx<double>* src, cx<double>* host) {
    if (l == 0) {
      c.download_fine(src, host, 0);
      return;
    }
    CoarseGeo& G = *geos[l];
    long len = level_len(l);
    c.lex.ensure(sizeof(cx<double>) * std::max(len, c.fine_len()));
    permute<double, double>(G.n, G.nsites, G.d_order.template as<int>(), src, c.lex.template as<cx<double>>(), 0,
                            c.st);
    HIP_CHECK(hipMemcpyAsync(host, c.lex.p, sizeof(cx<double>) * len, hipMemcpyDeviceToHost, c.st));
    HIP_CHECK(hipStreamSynchronize(c.st));
  }

  void check_flag(const char* what) {
    int h = 0;
    HIP_CHECK(hipMemcpyAsync(&h, c.iflag.p, sizeof(int), hipMemcpyDeviceToHost, c.st));
    HIP_CHECK(hipStreamSynchronize(c.st));
    if (h) throw Error(NUMERICAL, what);
  }

  void build_next(int l) {
    HIP_CHECK(hipMemsetAsync(c.iflag.p, 0, sizeof(int), c.st));
    long len = level_len(l);
    CoarseGeo& Gn = *geos[l + 1];
    if (l == 0) {
      launch_qr_fine<R, R>(c.g, Nv[0], Vraw[0].template as<cx<R>>(), len, Q[0].template as<cx<R>>(), len,
                           c.iflag.template as<int>(), c.st);
    } else {
      CoarseGeo& G = *geos[l];
      launch_qr_coarse<R, R>(G.n, Nv[l], G.nagg, G.asz, G.agg_sites.template as<int>(), Vraw[l].template as<cx<R>>(),
                             len, Q[l].template as<cx<R>>(), len, c.iflag.template as<int>(), c.st);
    }
    check_flag("rank-deficient aggregate in the block orthonormalisation");
    assemble_next(l);
  }

  void assemble_next(int l) {
    Xs.ensure(xs_bytes, true);
    long len = level_len(l);
    CoarseGeo& Gn = *geos[l + 1];
    if (l == 0) {
      dtw_asm = tw0.half_diff();
      launch_assemble_fine<R>(c.g, Nv[0], c.U64.template as<cx<double>>(), c.H64.template as<double>(), dtw_asm,
                              Q[0].template as<cx<R>>(), len, f2c.template as<int>(), D64[1].template as<cx<double>>(),
                              Xs.template as<cx<double>>(), c.st);
    } else {
      CoarseGeo& G = *geos[l];
      launch_assemble_coarse<R>(G.cg(), Nv[l], G.nagg, G.ab, G.agg_sites.template as<int>(),
                                D64[l].template as<cx<double>>(), Q[l].template as<cx<R>>(), len,
                                D64[l + 1].template as<cx<double>>(), Xs.template as<cx<double>>(), c.st);
    }
    launch_self_fixup(Gn.n, Gn.nsites, D64[l + 1].template as<cx<double>>(), Xs.template as<cx<double>>(),
                      l == 0 ? 1 : 0, c.st);
    if constexpr (!std::is_same<S, double>::value)
      launch_cvt_cx<S>((long)Gn.n * Gn.n * 5 * Gn.nsites, D64[l + 1].template as<cx<double>>(), DS[l + 1].p, c.st);
    if (l + 1 == L - 1)
      launch_coarse_odd_inverse<R>(Gn.cg(), D64[l + 1].template as<cx<double>>(), tw[l + 1],
                                   invscr.template as<cx<double>>(), Minvc.template as<cx<R>>(), c.st);
  }

  // the level-l work vectors used as input/output of setup cycles
  cx<R>* setup_in(int l) { return l == 0 ? fb.template as<cx<R>>() : wk[l][2].template as<cx<R>>(); }
  cx<R>* setup_out(int l) { return l == 0 ? fx.template as<cx<R>>() : wk[l][3].template as<cx<R>>(); }
  cx<R>* setup_zero(int l) { return l == 0 ? fr.template as<cx<R>>() : wk[l][0].template as<cx<R>>(); }

  void smooth_level(int l, const cx<R>* b, cx<R>* x, int iters) {
    if (l == 0) fine_sap(b, x, iters, p.mr_steps);
    else coarse_sap(l, b, x, iters);
  }

  DevBuf npart;  // partial sums + scalar for normalisation
  void normalise(cx<R>* v, long len) {
    const int nwg = 1024;
    npart.ensure(sizeof(cx<double>) * (nwg + 1));
    cx<double>* part = npart.template as<cx<double>>();
    cx<double>* sc = part + nwg;
    int nw = (int)std::min<long>(nwg, (len + 255) / 256);
    launch_multidot<R>(v, 0, 1, v, len, part, nw, c.st);
    launch_reduce(part, 1, nw, sc, 2, c.st);
    launch_scale_by_inv<R>(v, sc, v, len, c.st);
  }

  void iterate(int l) {
    long len = level_len(l);
    if (p.batch > 1) {
      // chunks of up to p.batch test vectors through one lock-step V-cycle
      const int K = std::min(p.batch, Nv[l]);
      ensure_multi(K);
      cx<R>* out;
      if (l == 0) {
        fxm.ensure(sizeof(cx<R>) * len * K, true);
        out = fxm.template as<cx<R>>();
      } else {
        out = ecm[l].template as<cx<R>>();
      }
      for (int i0 = 0; i0 < Nv[l]; i0 += K) {
        const int k = std::min(K, Nv[l] - i0);
        cx<R>* v0 = Vraw[l].template as<cx<R>>() + (long)i0 * len;
        // level >= 1: the cycle's input must not alias its work vectors; Vraw does not
        vcycle_m(l, v0, out, k);
        for (int q = 0; q < k; ++q) {
          launch_copy_cvt<R, R>(out + (long)q * len, v0 + (long)q * len, len, c.st);
          normalise(v0 + (long)q * len, len);
        }
      }
      build_next(l);
      return;
    }
    for (int i = 0; i < Nv[l]; ++i) {
      cx<R>* vi = Vraw[l].template as<cx<R>>() + (long)i * len;
      launch_copy_cvt<R, R>(vi, setup_in(l), len, c.st);
      vcycle(l, setup_in(l), setup_out(l));
      launch_copy_cvt<R, R>(setup_out(l), vi, len, c.st);
      normalise(vi, len);
    }
    build_next(l);
  }

  // init vectors (FP64, lexicographic) -> level layout in precision R
  void upload_vec(int l, const void* src, int on_device, cx<R>* dst) {
    long len = level_len(l);
    if (l == 0) {
      c.f64c.ensure(sizeof(cx<double>) * len);
      c.upload_fine(src, on_device, c.f64c.template as<cx<double>>());
      launch_copy_cvt<double, R>(c.f64c.template as<cx<double>>(), dst, len, c.st);
      return;
    }
    CoarseGeo& G = *geos[l];
    const cx<double>* s = (const cx<double>*)src;
    if (!on_device) {
      c.lex.ensure(sizeof(cx<double>) * std::max(len, c.fine_len()));
      HIP_CHECK(hipMemcpyAsync(c.lex.p, src, sizeof(cx<double>) * len, hipMemcpyHostToDevice, c.st));
      s = c.lex.template as<cx<double>>();
    }
    permute<double, R>(G.n, G.nsites, G.d_order.template as<int>(), s, dst, 1, c.st);
  }

  // SAP smoothing of K fields of level l (zero right-hand sides b)
  void smooth_level_m(int l, const cx<R>* b, cx<R>* x, int K, int iters) {
    if (l == 0) fine_sap_m(b, x, K, iters, p.mr_steps);
    else coarse_sap_m(l, b, x, K, iters);
  }

  void build(const void* const* vecs, int on_device, bool run_setup) override {
    for (int l = 0; l < L - 1; ++l) {
      long len = level_len(l);
      const bool smooth = run_setup && p.init_sap_iters > 0;
      const bool batched = smooth && p.batch > 1;
      for (int i = 0; i < Nv[l]; ++i) {
        cx<R>* vi = Vraw[l].template as<cx<R>>() + (long)i * len;
        if (loaded[l]) {
          // already in place (load_fine_init, adopt_vectors)
        } else {
          const char* src = (const char*)vecs[l] + sizeof(cx<double>) * (size_t)len * i;
          upload_vec(l, src, on_device, vi);
        }
        if (smooth && !batched) {
          launch_zero<R>(len, setup_zero(l), c.st);
          smooth_level(l, setup_zero(l), vi, p.init_sap_iters);
        }
      }
      if (batched) {
        // the initial smoothing of chunks of p.batch test vectors in one
        // K-field SAP (every field takes the arithmetic of a one-field sweep)
        const int K = std::min(p.batch, Nv[l]);
        ensure_multi(K);
        cx<R>* zb;
        if (l == 0) {
          fxm.ensure(sizeof(cx<R>) * len * K, true);
          zb = fxm.template as<cx<R>>();
        } else {
          zb = ecm[l].template as<cx<R>>();
        }
        launch_zero<R>(len * K, zb, c.st);
        for (int i0 = 0; i0 < Nv[l]; i0 += K)
          smooth_level_m(l, zb, Vraw[l].template as<cx<R>>() + (long)i0 * len, std::min(K, Nv[l] - i0),
                         p.init_sap_iters);
      }
      build_next(l);
      c.progress(0, l, 0);
    }
    if (run_setup) {
      for (int it = 0; it < p.setup_iters; ++it) {
        iterate(0);
        if (L == 3) {
          assemble_next(1);
          for (int t = 0; t < p.coarse_setup_iters; ++t) {
            iterate(1);
            c.progress(1, 1, t);
          }
        }
        c.progress(1, 0, it);
      }
    }
    c.sync();
    // the raw test vectors and the setup's fine K-column buffer are not needed
    // by the solver: give the memory back (the largest items of the setup),
    // unless the vectors are kept for a later setup update
    if (!p.keep_test_vectors)
      for (int l = 0; l < L - 1; ++l) Vraw[l].release();
    fxm.release();
    Xs.release();
    // the K-column bases sized for the setup's batch: the solve re-creates
    // them at its own width (the K-column work fields keep their size)
    for (int l = 1; l < L; ++l) {
      kwsm[l].V.release();
      kwsm[l].Z.release();
      kwsm[l].r.release();
    }
    Km = 0;
  }

  // ---- parity helpers (host FP64 in/out) --------------------------------------
  void get_interp(int l, cx<double>* host) override {
    long len = level_len(l);
    DevBuf t;
    t.alloc(sizeof(cx<double>) * len);
    for (int i = 0; i < Nv[l]; ++i) {
      launch_copy_cvt<R, double>(Q[l].template as<cx<R>>() + (long)i * len, t.as<cx<double>>(), len, c.st);
      download_level(l, t.as<cx<double>>(), host + (long)i * len);
    }
  }
  void restrict_host(int l, const cx<double>* in, cx<double>* out) override {
    long len = level_len(l), lenc = level_len(l + 1);
    DevBuf a, b;
    a.alloc(sizeof(cx<double>) * len);
    b.alloc(sizeof(cx<double>) * lenc);
    upload_level(l, in, 0, a.as<cx<double>>());
    cx<R>* ar = setup_in(l);
    launch_copy_cvt<double, R>(a.as<cx<double>>(), ar, len, c.st);
    restrict_(l, ar, rc[l + 1].template as<cx<R>>());
    launch_copy_cvt<R, double>(rc[l + 1].template as<cx<R>>(), b.as<cx<double>>(), lenc, c.st);
    download_level(l + 1, b.as<cx<double>>(), out);
  }
  void prolong_host(int l, const cx<double>* in, cx<double>* out) override {
    long len = level_len(l), lenc = level_len(l + 1);
    DevBuf a, b;
    a.alloc(sizeof(cx<double>) * lenc);
    b.alloc(sizeof(cx<double>) * len);
    upload_level(l + 1, in, 0, a.as<cx<double>>());
    launch_copy_cvt<double, R>(a.as<cx<double>>(), ec[l + 1].template as<cx<R>>(), lenc, c.st);
    prolong_(l, ec[l + 1].template as<cx<R>>(), setup_out(l), 0);
    launch_copy_cvt<R, double>(setup_out(l), b.as<cx<double>>(), len, c.st);
    download_level(l, b.as<cx<double>>(), out);
  }
  // restriction (dir 0) or prolongation (dir 1) of K columns between levels l
  // and l + 1 with the K-column kernels of the lock-step cycle
  void transfer_multi_host(int l, int dir, int K, const cx<double>* in, cx<double>* out) override {
    const long len = level_len(l), lenc = level_len(l + 1);
    const long lin = dir == 0 ? len : lenc, lout = dir == 0 ? lenc : len;
    DevBuf a, b, ar, br;
    a.alloc(sizeof(cx<double>) * lin * K, true);
    b.alloc(sizeof(cx<double>) * lout * K, true);
    ar.alloc(sizeof(cx<R>) * lin * K, true);
    br.alloc(sizeof(cx<R>) * lout * K, true);
    for (int k = 0; k < K; ++k) upload_level(l + dir, in + k * lin, 0, a.as<cx<double>>() + k * lin);
    launch_copy_cvt<double, R>(a.as<cx<double>>(), ar.as<cx<R>>(), lin * K, c.st);
    if (l == 0 && dir == 0)
      launch_restrict_fine_m<R>(c.g, Nv[0], Q[0].template as<cx<R>>(), len, ar.as<cx<R>>(), len, K,
                                f2c.template as<int>(), br.as<cx<R>>(), lenc, c.st);
    else if (l == 0)
      launch_prolong_fine_m<R>(c.g, Nv[0], Q[0].template as<cx<R>>(), len, ar.as<cx<R>>(), lenc, K,
                               f2c.template as<int>(), br.as<cx<R>>(), len, 0, c.st);
    else if (dir == 0)
      restrict_m(l, ar.as<cx<R>>(), len, br.as<cx<R>>(), lenc, K);
    else
      prolong_m(l, ar.as<cx<R>>(), lenc, br.as<cx<R>>(), len, K);
    launch_copy_cvt<R, double>(br.as<cx<R>>(), b.as<cx<double>>(), lout * K, c.st);
    for (int k = 0; k < K; ++k) download_level(l + 1 - dir, b.as<cx<double>>() + k * lout, out + k * lout);
  }
  void get_coarse_op(int l, cx<double>* S_, cx<double>* F_) override {
    CoarseGeo& G = *geos[l];
    size_t nn = (size_t)G.n * G.n;
    std::vector<cx<double>> h(nn * 5 * G.nsites);
    HIP_CHECK(hipMemcpyAsync(h.data(), D64[l].p, sizeof(cx<double>) * h.size(), hipMemcpyDeviceToHost, c.st));
    HIP_CHECK(hipStreamSynchronize(c.st));
    for (int s = 0; s < G.nsites; ++s) {
      int o = G.order[s];
      for (int blk = 0; blk < 5; ++blk) {
        const cx<double>* src = h.data() + ((size_t)o * 5 + blk) * nn;
        cx<double>* dst = blk == 0 ? S_ + (size_t)s * nn : F_ + ((size_t)(blk - 1) * G.nsites + s) * nn;
        for (int r = 0; r < G.n; ++r)
          for (int k = 0; k < G.n; ++k) dst[(size_t)r * G.n + k] = src[(size_t)k * G.n + r];
      }
    }
  }
  void apply_coarse_host(int l, const cx<double>* in, cx<double>* out) override {
    CoarseGeo& G = *geos[l];
    long len = level_len(l);
    DevBuf a;
    a.alloc(sizeof(cx<double>) * len);
    upload_level(l, in, 0, a.as<cx<double>>());
    cx<R>* x = wk[l][2].template as<cx<R>>();
    cx<R>* y = wk[l][3].template as<cx<R>>();
    launch_copy_cvt<double, R>(a.as<cx<double>>(), x, len, c.st);
    launch_coarse_apply<R, S>(G.cg(), Dst(l), tw[l], x, y, c.st);
    launch_copy_cvt<R, double>(y, a.as<cx<double>>(), len, c.st);
    download_level(l, a.as<cx<double>>(), out);
  }
  void coarse_sap_host(int l, const cx<double>* b, cx<double>* x, int iters) override {
    long len = level_len(l);
    DevBuf a;
    a.alloc(sizeof(cx<double>) * len);
    upload_level(l, b, 0, a.as<cx<double>>());
    cx<R>* bb = wk[l][2].template as<cx<R>>();
    cx<R>* xx = wk[l][3].template as<cx<R>>();
    launch_copy_cvt<double, R>(a.as<cx<double>>(), bb, len, c.st);
    upload_level(l, x, 0, a.as<cx<double>>());
    launch_copy_cvt<double, R>(a.as<cx<double>>(), xx, len, c.st);
    coarse_sap(l, bb, xx, iters);
    launch_copy_cvt<R, double>(xx, a.as<cx<double>>(), len, c.st);
    download_level(l, a.as<cx<double>>(), x);
  }
  void apply_coarse_m(int l, const cx<R>* in, cx<R>* out, int K) {
    CoarseGeo& G = *geos[l];
    const long len = level_len(l);
    if constexpr (kMfma) {
      if (mfma_level(l)) {
        launch_coarse_apply_mrhs<S>(G.cg(), Dst(l), tw[l], K, len, in, nullptr, out, c.st);
        return;
      }
    }
    for (int k = 0; k < K; ++k) launch_coarse_apply<R, S>(G.cg(), Dst(l), tw[l], in + k * len, out + k * len, c.st);
  }
  void apply_coarse_multi_host(int l, int K, const cx<double>* in, cx<double>* out) override {
    ensure_multi(K);
    const long len = level_len(l);
    DevBuf a;
    a.alloc(sizeof(cx<double>) * len);
    cx<R>* x = rcm[l].template as<cx<R>>();
    cx<R>* y = ecm[l].template as<cx<R>>();
    for (int k = 0; k < K; ++k) {
      upload_level(l, in + k * len, 0, a.as<cx<double>>());
      launch_copy_cvt<double, R>(a.as<cx<double>>(), x + k * len, len, c.st);
    }
    apply_coarse_m(l, x, y, K);
    for (int k = 0; k < K; ++k) {
      launch_copy_cvt<R, double>(y + k * len, a.as<cx<double>>(), len, c.st);
      download_level(l, a.as<cx<double>>(), out + k * len);
    }
  }
  void coarse_solve_multi_host(int l, int K, const cx<double>* b, cx<double>* x) override {
    ensure_multi(K);
    const long len = level_len(l);
    DevBuf a;
    a.alloc(sizeof(cx<double>) * len);
    cx<R>* bb = rcm[l].template as<cx<R>>();
    cx<R>* xx = ecm[l].template as<cx<R>>();
    for (int k = 0; k < K; ++k) {
      upload_level(l, b + k * len, 0, a.as<cx<double>>());
      launch_copy_cvt<double, R>(a.as<cx<double>>(), bb + k * len, len, c.st);
    }
    coarse_solve_m(l, bb, xx, K);
    for (int k = 0; k < K; ++k) {
      launch_copy_cvt<R, double>(xx + k * len, a.as<cx<double>>(), len, c.st);
      download_level(l, a.as<cx<double>>(), x + k * len);
    }
  }
  void schur_multi_host(int l, int K, const cx<double>* in, cx<double>* out) override {
    if (l != L - 1) throw Error(INVALID_ARG, "the odd-even reduced operator is formed on the coarsest level only");
    ensure_multi(K);
    const long len = level_len(l);
    DevBuf a;
    a.alloc(sizeof(cx<double>) * len);
    cx<R>* x = rcm[l].template as<cx<R>>();
    cx<R>* y = ecm[l].template as<cx<R>>();
    for (int k = 0; k < K; ++k) {
      upload_level(l, in + k * len, 0, a.as<cx<double>>());
      launch_copy_cvt<double, R>(a.as<cx<double>>(), x + k * len, len, c.st);
    }
    launch_zero<R>(len * K, y, c.st);
    AopM[l](x, y, K);
    for (int k = 0; k < K; ++k) {
      launch_copy_cvt<R, double>(y + k * len, a.as<cx<double>>(), len, c.st);
      download_level(l, a.as<cx<double>>(), out + k * len);
    }
  }
  void coarse_sap_multi_host(int l, int K, const cx<double>* b, cx<double>* x, int iters) override {
    ensure_multi(K);
    const long len = level_len(l);
    DevBuf a;
    a.alloc(sizeof(cx<double>) * len);
    cx<R>* bb = rcm[l].template as<cx<R>>();
    cx<R>* xx = ecm[l].template as<cx<R>>();
    for (int k = 0; k < K; ++k) {
      upload_level(l, b + k * len, 0, a.as<cx<double>>());
      launch_copy_cvt<double, R>(a.as<cx<double>>(), bb + k * len, len, c.st);
      upload_level(l, x + k * len, 0, a.as<cx<double>>());
      launch_copy_cvt<double, R>(a.as<cx<double>>(), xx + k * len, len, c.st);
    }
    coarse_sap_m(l, bb, xx, K, iters);
    for (int k = 0; k < K; ++k) {
      launch_copy_cvt<R, double>(xx + k * len, a.as<cx<double>>(), len, c.st);
      download_level(l, a.as<cx<double>>(), x + k * len);
    }
  }
  void bench_coarse_multi(int l, int K, int napply, int which) override {
    ensure_multi(K);
    const long len = level_len(l);
    cx<R>* x = rcm[l].template as<cx<R>>();
    cx<R>* y = ecm[l].template as<cx<R>>();
    // any finite input serves for timing: fill with a constant
    launch_zero<R>(len * K, y, c.st);
    launch_axpby<R>(len * K, 0.0, y, 0.0, x, c.st);
    for (int i = 0; i < napply; ++i) {
      if (which == 1 && l == L - 1) AopM[l](x, y, K);
      else apply_coarse_m(l, x, y, K);
    }
  }
  void coarse_solve_host(int l, const cx<double>* b, cx<double>* x) override {
    long len = level_len(l);
    DevBuf a;
    a.alloc(sizeof(cx<double>) * len);
    upload_level(l, b, 0, a.as<cx<double>>());
    launch_copy_cvt<double, R>(a.as<cx<double>>(), rc[l].template as<cx<R>>(), len, c.st);
    coarse_solve(l, rc[l].template as<cx<R>>(), ec[l].template as<cx<R>>());
    launch_copy_cvt<R, double>(ec[l].template as<cx<R>>(), a.as<cx<double>>(), len, c.st);
    download_level(l, a.as<cx<double>>(), x);
  }
};

std::unique_ptr<MGBase> make_mg(Ctx& c) {
  switch (c.p.precision) {
    case DDAMG_FP64: return std::unique_ptr<MGBase>(new MG<double, double>(c, c.p));
    case DDAMG_FP32: return std::unique_ptr<MGBase>(new MG<float, float>(c, c.p));
    case DDAMG_FP16: return std::unique_ptr<MGBase>(new MG<float, f16>(c, c.p));
    case DDAMG_BF16: return std::unique_ptr<MGBase>(new MG<float, bf16>(c, c.p));
    default: throw Error(INVALID_ARG, "unknown precision");
  }
}

// exported for the API file
void check_finite(Ctx& c, const double* dev, long n) {
  HIP_CHECK(hipMemsetAsync(c.iflag.p, 0, sizeof(int), c.st));
  hipLaunchKernelGGL(k_all_finite, dim3((n + 255) / 256), dim3(256), 0, c.st, n, dev, c.iflag.as<int>());
  int h = 0;
  HIP_CHECK(hipMemcpyAsync(&h, c.iflag.p, sizeof(int), hipMemcpyDeviceToHost, c.st));
  HIP_CHECK(hipStreamSynchronize(c.st));
  if (h) throw Error(NUMERICAL, "input contains NaN or Inf");
}

}  // namespace ddamg
