// Host-side orchestration: device buffers, the multigrid hierarchy, Krylov
// solvers and the context behind the C interface.
#pragma once
#include <chrono>
#include <functional>
#include <map>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "kernels.hpp"
#include "ddamg.h"

namespace ddamg {

// Device memory of one context.  Slabs obtained with hipMalloc stay with the
// context until it is destroyed: on this device a hipMalloc of memory that
// the process freed earlier costs up to a second per few GB (a 7.6 GB block:
// 1.26 s), while a first-time allocation costs microseconds, so a setup or
// solve that gives its buffers back and takes them again would pay that on
// every call.  Buffers take best-fit ranges out of the slabs (256-byte
// granules); released ranges merge with free neighbours.  Every kernel of a
// context runs on its one stream, so a range released and handed out again is
// reused in stream order; the first reuse after any release synchronises that
// stream once, which covers synchronous host copies into a reused range
// (hipFree synchronised the device for the same reason).  When hipMalloc
// fails, slabs with nothing in use are freed and the allocation retried.
// Buffers that live only through one phase of a call (the network's
// activations, the setup's raw test vectors and work fields, the outer
// solve's Krylov basis) are "transient" and take ranges of transient slabs
// only; every other buffer takes ranges of persistent slabs.  The phases then
// reuse one another's ranges in turn, and a long-lived buffer never pins a
// slab that a later phase needs whole.
struct MemPool {
  struct Slab {
    char* base = nullptr;
    size_t bytes = 0, used = 0;
    bool transient = false;
    std::map<size_t, size_t> free;  // offset -> length of the free ranges
  };
  std::vector<Slab> slabs;
  hipStream_t st = nullptr;         // the owning context's stream
  bool dirty = false;               // a range was released since the last synchronisation
  void* get(size_t b, bool transient = false);
  void put(void* p, size_t b);
  void trim();                      // hipFree every slab with nothing in use
  size_t reserved() const;
  MemPool() = default;
  MemPool(const MemPool&) = delete;
  MemPool& operator=(const MemPool&) = delete;
  ~MemPool();
};

// the pool of the context whose entry point is running on this thread (set by
// the C interface for the duration of a call); without one, DevBuf uses
// hipMalloc/hipFree directly
MemPool*& current_pool();

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  MemPool* pool = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  void alloc(size_t b, bool transient = false) {
    release();
    if (!b) return;
    MemPool* mp = current_pool();
    if (mp) {
      p = mp->get(b, transient);
      pool = mp;
    } else {
      hipError_t e = hipMalloc(&p, b);
      if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
        (void)hipGetLastError();
        p = nullptr;
        throw Error(OUT_OF_MEMORY, "device allocation of " + std::to_string(b) + " bytes failed");
      }
      HIP_CHECK(e);
    }
    bytes = b;
  }
  void ensure(size_t b, bool transient = false) {
    if (bytes < b) alloc(b, transient);
  }
  void release() {
    if (p) {
      if (pool) pool->put(p, bytes);
      else (void)hipFree(p);
    }
    p = nullptr;
    bytes = 0;
    pool = nullptr;
  }
  ~DevBuf() { release(); }
  void swap(DevBuf& o) {
    std::swap(p, o.p);
    std::swap(bytes, o.bytes);
    std::swap(pool, o.pool);
  }
  template <class T> T* as() const { return reinterpret_cast<T*>(p); }
};

// per-kernel timing with event pairs recorded on the stream
struct KernelTimer {
  bool on = false;
  hipStream_t st = nullptr;
  struct Rec {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  static constexpr int NKIND = 6;
  long count[NKIND] = {0, 0, 0, 0, 0, 0};
  double ms[NKIND] = {0, 0, 0, 0, 0, 0};
  double bytes[NKIND] = {0, 0, 0, 0, 0, 0};  // algorithmic bytes of the timed launches (kinds 0, 1)
  double flops[NKIND] = {0, 0, 0, 0, 0, 0};  // algorithmic flops of the timed launches (kind 1)
  hipEvent_t get();
  void begin(int kind, hipEvent_t* a);
  void end(int kind, hipEvent_t a, double b = 0, double f = 0);
  void flush();
  void reset();
  ~KernelTimer();
};

struct Ctx;

// Krylov workspace: basis vectors in precision R, all scalars FP64 on device
template <class R>
struct KrylovWS {
  int m = 0;
  long ld = 0;  // allocated length of one vector
  bool flexible = false;
  DevBuf V, Z, tmp, H, cs, sn, g, y, part, scal, resid;
  double* h_resid = nullptr;  // pinned host mirror: [0] blocking reads, [2 + k] look-ahead slot k
  hipEvent_t ready[2] = {nullptr, nullptr};  // look-ahead: residual estimate k has reached h_resid[2 + k]
  int nwg = 0;
  void init(int m_, long ld_, long N, bool flex);
  ~KrylovWS();
};

// Workspace of K Krylov processes in lock step.  Every K-column vector is K
// vectors of stride ld (column r at offset r * ld); the basis is
// [m+1][K][ld] (V) and [m][K][ld] (Z); scalars per column.
template <class R>
struct KrylovWSm {
  int m = 0, K = 0;
  long ld = 0;
  bool flexible = false;
  DevBuf V, Z, r, H, cs, sn, g, y, part, scal, resid, act, jd;
  double* h_resid = nullptr;   // pinned: K residual estimates (three slots of 32 for the look-ahead)
  hipEvent_t ready[3] = {nullptr, nullptr, nullptr};
  int nwgf = 0;                  // workgroups per column of the fused Arnoldi step
  cx<double>* h_scal = nullptr;  // pinned: K x 4 scalars
  int* h_act = nullptr;        // pinned: K flags (host copy)
  int* h_act_ring = nullptr;   // pinned: 4 x 16 staging slots for the asynchronous pushes of h_act
  int act_slot = 0;
  int* h_jd = nullptr;         // pinned: K counts
  int nwg = 0;
  bool zf32 = false;            // Z holds FP32 directions (mixed outer solve)
  // transient: the basis (V, Z, r) comes from the pool's transient slabs
  void init(int m_, int K_, long ld_, long N, bool flex, bool z_fp32 = false, bool transient = false);
  ~KrylovWSm();
};

struct KrylovResultM {
  std::vector<int> iters;      // per column
  std::vector<double> resid;   // relative true residual at exit
  std::vector<char> converged;
  int steps = 0;               // lock-step iterations
};

// operator / preconditioner on K columns of stride ld
template <class R>
using OpM = std::function<void(const cx<R>*, cx<R>*, int)>;

// preconditioner that writes FP32 directions (the mixed form of the outer solve)
using OpMf = std::function<void(const cx<double>*, cx<float>*, int)>;

// Flexible GMRES(m) on K columns in lock step.  With Mf (R = double only) the
// preconditioned directions are stored in FP32 (ws initialised with z_fp32):
// each is widened to FP64 before the operator, and the iterate is updated in
// FP64; the basis V, every inner product and the residual stay in FP64.
template <class R>
KrylovResultM fgmres_multi(Ctx& c, KrylovWSm<R>& ws, int K, long N, const OpM<R>& A, const OpM<R>* M, const cx<R>* b,
                           cx<R>* x, double tol, int max_iter, bool fixed, bool x_is_zero, const OpMf* Mf = nullptr);

using OpR64 = std::function<void(const cx<double>*, cx<double>*)>;
using OpR32 = std::function<void(const cx<float>*, cx<float>*)>;

struct KrylovResult {
  int iters = 0;
  double resid = 0;  // relative (true residual at exit)
  bool converged = false;
};

// (F)GMRES(m): A, M act on vectors of length N (ld-strided basis); b, x may be
// longer than N (only the first N entries take part).
template <class R>
KrylovResult fgmres(Ctx& c, KrylovWS<R>& ws, long N, const std::function<void(const cx<R>*, cx<R>*)>& A,
                    const std::function<void(const cx<R>*, cx<R>*)>* M, const cx<R>* b, cx<R>* x, double tol,
                    int max_iter, bool fixed, bool x_is_zero);

struct CoarseGeo {
  int L[4];
  int n = 0;
  int nsites = 0, neven = 0;
  std::vector<int> order;  // lex -> ordered index
  std::vector<int> lexof;  // ordered -> lex
  DevBuf nbr;              // [nsites][8]
  DevBuf d_order;          // lex -> ordered (device)
  // aggregation to the next level
  int ab[4] = {0, 0, 0, 0};
  int nagg = 0, asz = 0;
  DevBuf agg_sites;  // [nagg][asz] ordered indices of this level, aggregate = next level ordered index
  DevBuf site_agg;   // [nsites] -> next-level ordered index
  // SAP blocks (intermediate levels)
  int sb[4] = {0, 0, 0, 0};
  int nsblk = 0, ssz = 0, nsblk_col[2] = {0, 0};
  DevBuf sap_sites;  // [nsblk][ssz], colour-0 blocks first
  DevBuf sap_nbr;    // [nsblk][ssz][8]
  CGeom cg() const { return CGeom{n, nsites, neven, nbr.as<int>(), d_order.as<int>()}; }
};

struct MGBase {
  virtual ~MGBase() = default;
  virtual void build(const void* const* vecs, int on_device, bool run_setup) = 0;
  virtual void precond(const cx<double>* v, cx<double>* z) = 0;  // fine block layout FP64
  // the same on K fine FP64 fields (stride = fine length), in lock step
  virtual void precond_multi(const cx<double>* v, cx<double>* z, int K) = 0;
  // the same with FP32 output (reduced-precision hierarchies only)
  virtual void precond_multi_f32(const cx<double>* v, cx<float>* z, int K) = 0;
  // new twists on every level from the same P: the coarse operators are
  // assembled again when the parity rest of the fine twist changes
  virtual void set_twist(const Twist& t) = 0;
  virtual int nlev() const = 0;
  virtual const CoarseGeo& geo(int l) const = 0;  // l >= 1
  virtual void get_interp(int l, cx<double>* host) = 0;
  virtual void restrict_host(int l, const cx<double>* in, cx<double>* out) = 0;
  virtual void prolong_host(int l, const cx<double>* in, cx<double>* out) = 0;
  virtual void transfer_multi_host(int l, int dir, int K, const cx<double>* in, cx<double>* out) = 0;
  virtual void get_coarse_op(int l, cx<double>* S, cx<double>* F) = 0;
  virtual void apply_coarse_host(int l, const cx<double>* in, cx<double>* out) = 0;
  virtual void coarse_sap_host(int l, const cx<double>* b, cx<double>* x, int iters) = 0;
  virtual void coarse_solve_host(int l, const cx<double>* b, cx<double>* x) = 0;
  // K columns of a level-l field, host FP64 [K][len] in the level layout
  virtual void apply_coarse_multi_host(int l, int K, const cx<double>* in, cx<double>* out) = 0;
  virtual void coarse_solve_multi_host(int l, int K, const cx<double>* b, cx<double>* x) = 0;
  // K columns of the coarsest level's odd-even reduced operator (even-site
  // parts of in; out zero on odd sites), and K-field SAP on an intermediate level
  virtual void schur_multi_host(int l, int K, const cx<double>* in, cx<double>* out) = 0;
  virtual void coarse_sap_multi_host(int l, int K, const cx<double>* b, cx<double>* x, int iters) = 0;
  // napply launches of the K-column coarse operator of level l on device-resident
  // work vectors (which = 0: full stencil, 1: odd-even reduced operator, coarsest level)
  virtual void bench_coarse_multi(int l, int K, int napply, int which) = 0;
  long coarse_iters[4] = {0, 0, 0, 0};
  long vcycles = 0;
  // level-0 initial vectors from the device (block layout, FP32, stride = fine
  // length), copied into the hierarchy; build() then skips vecs[0]
  virtual void load_fine_init(const cx<float>* v) = 0;
  // one of them (index i, block layout, FP32); build() then skips vecs[0]
  virtual void load_fine_vec(int i, const cx<float>* v) = 0;
  // the test vectors of a previous hierarchy of the same precision, levels
  // and N_v (the kept raw vectors, else its interpolation bases Q_l) become
  // this one's (moved, not copied); build() then skips vecs for those levels
  virtual void adopt_vectors(MGBase& prev) = 0;
  bool loaded[3] = {false, false, false};  // test vectors of level l already in place
};

// learned-setup network: parameters (real view, FP32), Adam moments, activations
struct NetState {
  int L = 0, C = 0;
  long nWc = 0;       // complex weights per layer: 9*C*C*16
  long nreal = 0;     // real parameters in total
  DevBuf params, grads, m, v;
  DevBuf act, zb, sb, g1, g2, wpart, gpart, lscr, lpart, host_stage;
  DevBuf packed;      // weights in matrix-core fragment order (inference)
  long V = 0;         // lattice the buffers are sized for
  long step = 0;
  cx<float>* W(int l) const { return params.as<cx<float>>() + (long)l * nWc; }
  float* ab(int l) const { return params.as<float>() + 2 * (long)L * nWc + 2L * l * C; }
  cx<float>* GW(int l) const { return grads.as<cx<float>>() + (long)l * nWc; }
  float* Gab(int l) const { return grads.as<float>() + 2 * (long)L * nWc + 2L * l * C; }
};

struct Ctx {
  MemPool pool;  // first member: destroyed after every buffer that returns to it
  hipStream_t st = nullptr;
  int dev = 0;                 // HIP device current at ddamg_create
  Geom g{};
  double kappa = 0, csw = 0, mu = 0, m0 = 0;
  double mu_odd = 0;           // twist of the odd sites (equal to mu unless set apart)
  double theta[4] = {0, 0, 0, 0};  // twisted boundary conditions (0: periodic)
  bool have_gauge = false, have_setup = false;
  DevBuf U64, H64, M64;        // fine operator, FP64
  DevBuf U32, H32, M32;        // FP32 copies
  DevBuf U16;                  // 16-bit link copy
  int u16_kind = -1;           // DDAMG_FP16 or DDAMG_BF16
  bool have_32 = false;
  DevBuf lex;                  // host-layout FP64 staging (one fine field)
  DevBuf f64a, f64b, f64c;     // fine FP64 block-layout vectors
  DevBuf f32a, f32b;           // fine FP32 block-layout vectors
  DevBuf iflag;                // int error flag
  ddamg_params p{};
  std::unique_ptr<MGBase> mg;
  KrylovWS<double> outer;
  KrylovWSm<double> outer_m;   // lock-step outer solves (basis released to the pool between solves)
  NetState net;
  KernelTimer timer;
  std::string err;
  ddamg_progress_fn progress_fn = nullptr;  // setup notifications (ddamg_set_progress)
  void* progress_user = nullptr;

  long fine_len() const { return g.V * 12; }
  void ensure_32();
  void ensure_16(int kind);
  void rebuild_odd_inverse();
  void sync() { HIP_CHECK(hipStreamSynchronize(st)); }
  // the fine operator's twists, both negated for sign < 0 (D(-mu))
  Twist twist(int sign = 1) const { return sign < 0 ? Twist(-mu, -mu_odd) : Twist(mu, mu_odd); }
  // setup stage finished: wait for the stream, then tell the caller
  void progress(int stage, int level, int index) {
    if (!progress_fn) return;
    sync();
    progress_fn(progress_user, stage, level, index);
  }
  // fine FP64 operator D(tw) in block layout
  void dirac64(const cx<double>* in, cx<double>* out, Twist tw);
  // K fields at a stride of ld complex in one launch
  void dirac64_multi(const cx<double>* in, cx<double>* out, int K, long ld, Twist tw);
  // host/device lex FP64 field -> block layout
  void upload_fine(const void* src, int on_device, cx<double>* dst64);
  void download_fine(const cx<double>* src64, void* dst, int on_device);
};

std::unique_ptr<MGBase> make_mg(Ctx& c);

// records the device address of ddamg_apply_dirac_noalloc's scratch array on
// device dev (the current device), once per device
void noalloc_scratch_init(int dev);

}  // namespace ddamg
