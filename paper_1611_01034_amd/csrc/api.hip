// extern "C" boundary of the library (declared in include/ddamg.h).  Every
// entry point catches all exceptions and turns them into status codes.
#include <cmath>
#include <complex>
#include <cstring>

#include "solver.hpp"

struct ddamg_ctx {
  ddamg::Ctx c;
};

namespace ddamg {
void check_finite(Ctx& c, const double* dev, long n);
}

using namespace ddamg;

namespace {

// sigma^chi_{mu nu} chirality blocks in the chiral basis, mu<nu over directions
// 0:T 1:Z 2:Y 3:X, computed from g_mu = [[0,B_mu],[B_mu^dag,0]]:
// sigma = (i/2)[g_mu, g_nu]; block chi=0 (spins 0,1): (i/2)(B_mu B_nu^dag - B_nu B_mu^dag),
// block chi=1 (spins 2,3): (i/2)(B_mu^dag B_nu - B_nu^dag B_mu).
void sigma_table(double* tab) {
  using C = std::complex<double>;
  const C I(0, 1);
  // B_mu for T, Z, Y, X: B_T = -1, B_k = -i s_k
  C B[4][2][2];
  C s1[2][2] = {{0, 1}, {1, 0}}, s2[2][2] = {{0, -I}, {I, 0}}, s3[2][2] = {{1, 0}, {0, -1}};
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      B[0][a][b] = a == b ? C(-1) : C(0);
      B[1][a][b] = -I * s3[a][b];
      B[2][a][b] = -I * s2[a][b];
      B[3][a][b] = -I * s1[a][b];
    }
  auto mul = [](const C x[2][2], const C y[2][2], bool dx, bool dy, C out[2][2]) {
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) {
        C acc = 0;
        for (int k = 0; k < 2; ++k) {
          C xv = dx ? std::conj(x[k][i]) : x[i][k];
          C yv = dy ? std::conj(y[j][k]) : y[k][j];
          acc += xv * yv;
        }
        out[i][j] = acc;
      }
  };
  int p = 0;
  for (int mu = 0; mu < 4; ++mu)
    for (int nu = mu + 1; nu < 4; ++nu, ++p) {
      C a[2][2], b[2][2];
      // chirality 0
      mul(B[mu], B[nu], false, true, a);
      mul(B[nu], B[mu], false, true, b);
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
          C v = 0.5 * I * (a[i][j] - b[i][j]);
          tab[((p * 2 + 0) * 4 + 2 * i + j) * 2 + 0] = v.real();
          tab[((p * 2 + 0) * 4 + 2 * i + j) * 2 + 1] = v.imag();
        }
      // chirality 1
      mul(B[mu], B[nu], true, false, a);
      mul(B[nu], B[mu], true, false, b);
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
          C v = 0.5 * I * (a[i][j] - b[i][j]);
          tab[((p * 2 + 1) * 4 + 2 * i + j) * 2 + 0] = v.real();
          tab[((p * 2 + 1) * 4 + 2 * i + j) * 2 + 1] = v.imag();
        }
    }
}

// every buffer a call allocates comes from the context's pool
struct PoolScope {
  MemPool* prev;
  explicit PoolScope(ddamg_ctx* ctx) : prev(current_pool()) { current_pool() = ctx ? &ctx->c.pool : nullptr; }
  ~PoolScope() { current_pool() = prev; }
};

template <class F>
int guard(ddamg_ctx* ctx, F&& f) {
  PoolScope scope(ctx);
  try {
    if (ctx) ctx->c.err.clear();
    return f();
  } catch (const Error& e) {
    if (ctx) ctx->c.err = e.what();
    return e.status;
  } catch (const HipError& e) {
    if (ctx) ctx->c.err = e.what();
    return e.code == hipErrorOutOfMemory ? DDAMG_OUT_OF_MEMORY : DDAMG_HIP_ERROR;
  } catch (const std::bad_alloc&) {
    if (ctx) ctx->c.err = "host allocation failed";
    return DDAMG_OUT_OF_MEMORY;
  } catch (const std::exception& e) {
    if (ctx) ctx->c.err = e.what();
    return DDAMG_HIP_ERROR;
  }
}

void need_gauge(Ctx& c) {
  if (!c.have_gauge) throw Error(BAD_STATE, "no gauge field set");
}
void need_setup(Ctx& c) {
  need_gauge(c);
  if (!c.have_setup || !c.mg) throw Error(BAD_STATE, "no multigrid setup");
}

void check_params(const ddamg_params* p) {
  if (!p) throw Error(INVALID_ARG, "params is NULL");
  if (p->levels < 2 || p->levels > 3) throw Error(INVALID_ARG, "levels must be 2 or 3");
  if (p->sap_pre < 0 || p->sap_post < 0 || p->mr_steps < 0 || p->coarse_sap_post < 0 || p->coarse_mr_steps < 0 ||
      p->init_sap_iters < 0 || p->setup_iters < 0 || p->coarse_setup_iters < 0)
    throw Error(INVALID_ARG, "negative iteration count");
  if (p->restart < 1 || p->inter_restart < 1 || p->coarse_restart < 1 || p->max_iter < 1 || p->inter_max_iter < 1 ||
      p->coarse_max_iter < 1)
    throw Error(INVALID_ARG, "restart lengths and iteration limits must be >= 1");
  if (!(p->coarse_mu_factor >= 1.0) || !std::isfinite(p->coarse_mu_factor))
    throw Error(INVALID_ARG, "coarse_mu_factor (delta) must be >= 1");
  if (!(p->inter_tol > 0) || !(p->coarse_tol > 0)) throw Error(INVALID_ARG, "inner tolerances must be > 0");
  if (p->precision < 0 || p->precision > 3) throw Error(INVALID_ARG, "unknown precision");
  if (p->batch < 1 || p->batch > 16) throw Error(INVALID_ARG, "batch must be in [1, 16]");
  if (p->rhs_batch < 1 || p->rhs_batch > 16) throw Error(INVALID_ARG, "rhs_batch must be in [1, 16]");
}

// links (lexicographic FP64, host or device) -> block layout, clover term and
// the fine odd-site inverses; throws before any change for a non-finite field
void load_links(Ctx& c, const void* links, int on_device) {
  if (!links) throw Error(INVALID_ARG, "links is NULL");
  size_t bytes = sizeof(cx<double>) * (size_t)c.g.V * 36;
  const cx<double>* src = (const cx<double>*)links;
  DevBuf stage;
  if (!on_device) {
    stage.alloc(bytes);
    HIP_CHECK(hipMemcpyAsync(stage.p, links, bytes, hipMemcpyHostToDevice, c.st));
    src = stage.as<cx<double>>();
  }
  check_finite(c, (const double*)src, (long)c.g.V * 72);
  LinkPhases ph;
  for (int d = 0; d < 4; ++d) {
    ph.re[d] = std::cos(c.theta[d]);
    ph.im[d] = std::sin(c.theta[d]);
  }
  launch_links_from_lex(c.g, src, c.U64.as<cx<double>>(), ph, c.st);
  launch_clover(c.g, c.U64.as<cx<double>>(), c.csw, c.m0 + 4.0, c.H64.as<double>(), c.st);
  c.have_32 = false;
  c.u16_kind = -1;
  c.rebuild_odd_inverse();
  c.sync();
  c.have_gauge = true;
}

}  // namespace

extern "C" {

void ddamg_default_params(ddamg_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->levels = 2;
  for (int d = 0; d < 4; ++d) {
    p->block[0][d] = 4;
    p->block[1][d] = 2;
    p->block[2][d] = 2;
    p->coarse_sap_block[d] = 2;
  }
  p->nvec[0] = 24;
  p->nvec[1] = 32;
  p->nvec[2] = 32;
  p->sap_pre = 0;
  p->sap_post = 3;
  p->mr_steps = 4;
  p->coarse_sap_post = 2;
  p->coarse_mr_steps = 3;
  p->init_sap_iters = 3;
  p->setup_iters = 3;
  p->coarse_setup_iters = 3;
  p->coarse_mu_factor = 1.0;
  p->restart = 10;
  p->max_iter = 1000;
  p->inter_restart = 10;
  p->inter_max_iter = 10;
  p->inter_tol = 0.1;
  p->coarse_restart = 30;
  p->coarse_max_iter = 300;
  p->coarse_tol = 0.1;
  p->precision = DDAMG_FP64;
  p->fixed_iters = 0;
  p->batch = 16;
  p->rhs_batch = 1;
}

int ddamg_create(const int dims[4], const int block[4], double kappa, double csw, double mu, void* stream,
                 ddamg_ctx** out) {
  if (!out) return DDAMG_INVALID_ARG;
  *out = nullptr;
  if (!dims || !block) return DDAMG_INVALID_ARG;
  for (int d = 0; d < 4; ++d) {
    if (dims[d] <= 0 || block[d] <= 0 || block[d] % 2 || dims[d] % block[d]) return DDAMG_INVALID_ARG;
    if ((dims[d] / block[d]) % 2) return DDAMG_INVALID_ARG;
  }
  int bs = block[0] * block[1] * block[2] * block[3];
  if (bs > 256) return DDAMG_INVALID_ARG;
  if (!(kappa > 0) || !std::isfinite(kappa) || !std::isfinite(csw) || !std::isfinite(mu)) return DDAMG_INVALID_ARG;
  ddamg_ctx* ctx = new (std::nothrow) ddamg_ctx();
  if (!ctx) return DDAMG_OUT_OF_MEMORY;
  int st = guard(ctx, [&]() {
    Ctx& c = ctx->c;
    c.st = (hipStream_t)stream;
    HIP_CHECK(hipGetDevice(&c.dev));
    noalloc_scratch_init(c.dev);
    c.pool.st = c.st;
    c.timer.st = c.st;
    Geom& g = c.g;
    g.V = 1;
    for (int d = 0; d < 4; ++d) {
      g.L[d] = dims[d];
      g.b[d] = block[d];
      g.nb[d] = dims[d] / block[d];
      g.V *= dims[d];
    }
    g.bs = bs;
    g.half = bs / 2;
    g.ndir = 4;
    g.nblocks = g.nb[0] * g.nb[1] * g.nb[2] * g.nb[3];
    c.kappa = kappa;
    c.csw = csw;
    c.mu = mu;
    c.mu_odd = mu;
    c.m0 = 1.0 / (2.0 * kappa) - 4.0;
    double tab[6 * 2 * 4 * 2];
    sigma_table(tab);
    set_sigma_table(tab);
    c.U64.alloc(sizeof(cx<double>) * (size_t)g.V * 36);
    c.H64.alloc(sizeof(double) * (size_t)g.V * 72);
    c.M64.alloc(sizeof(double) * (size_t)g.V * 36);
    c.f64a.alloc(sizeof(cx<double>) * c.fine_len());
    c.f64b.alloc(sizeof(cx<double>) * c.fine_len());
    c.iflag.alloc(sizeof(int) * 4);
    return DDAMG_OK;
  });
  if (st != DDAMG_OK) {
    delete ctx;
    return st;
  }
  *out = ctx;
  return DDAMG_OK;
}

void ddamg_destroy(ddamg_ctx* ctx) {
  if (!ctx) return;
  try {
    (void)hipStreamSynchronize(ctx->c.st);
  } catch (...) {
  }
  delete ctx;
}

const char* ddamg_last_error(const ddamg_ctx* ctx) { return ctx ? ctx->c.err.c_str() : "null context"; }

int ddamg_set_gauge(ddamg_ctx* ctx, const void* links, int on_device) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    load_links(c, links, on_device);
    c.have_setup = false;
    c.mg.reset();
    return DDAMG_OK;
  });
}

int ddamg_set_boundary_phases(ddamg_ctx* ctx, const double theta[4]) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    if (!theta) throw Error(INVALID_ARG, "theta is NULL");
    for (int d = 0; d < 4; ++d)
      if (!std::isfinite(theta[d])) throw Error(INVALID_ARG, "theta must be finite");
    if (c.have_gauge) {
      // the links in place carry the old phases: multiply by the difference
      LinkPhases ph;
      for (int d = 0; d < 4; ++d) {
        ph.re[d] = std::cos(theta[d] - c.theta[d]);
        ph.im[d] = std::sin(theta[d] - c.theta[d]);
      }
      launch_link_phase(c.g, c.U64.as<cx<double>>(), ph, c.st);
      c.have_32 = false;
      c.u16_kind = -1;
      c.sync();
      c.have_setup = false;
      c.mg.reset();
    }
    for (int d = 0; d < 4; ++d) c.theta[d] = theta[d];
    return DDAMG_OK;
  });
}

int ddamg_update_gauge(ddamg_ctx* ctx, const void* links, int on_device, const ddamg_params* p) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    need_setup(c);
    check_params(p);
    if (p->levels != c.p.levels || p->precision != c.p.precision)
      throw Error(INVALID_ARG, "levels and precision must equal those of the current setup");
    // on three levels the kept level-1 test vectors are coefficients in the
    // fine basis P_0: a fine iteration changes P_0, and only level-1
    // iterations adapt those vectors to it again
    if (p->levels == 3 && p->setup_iters > 0 && p->coarse_setup_iters == 0)
      throw Error(INVALID_ARG, "a three-level update with fine iterations needs coarse_setup_iters > 0");
    for (int l = 0; l < p->levels - 1; ++l) {
      if (p->nvec[l] != c.p.nvec[l]) throw Error(INVALID_ARG, "nvec must equal that of the current setup");
      for (int d = 0; d < 4; ++d)
        if (p->block[l][d] != c.p.block[l][d])
          throw Error(INVALID_ARG, "aggregation blocks must equal those of the current setup");
    }
    // a field with NaN or Inf is rejected here with the old state intact
    load_links(c, links, on_device);
    std::unique_ptr<MGBase> prev = std::move(c.mg);
    c.have_setup = false;
    c.p = *p;
    c.mg = make_mg(c);
    c.mg->adopt_vectors(*prev);
    prev.reset();
    const void* none[3] = {nullptr, nullptr, nullptr};
    c.mg->build(none, 1, true);
    c.have_setup = true;
    return DDAMG_OK;
  });
}

int ddamg_set_clover(ddamg_ctx* ctx, const void* clover, int on_device) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    need_gauge(c);
    if (!clover) {
      launch_clover(c.g, c.U64.as<cx<double>>(), c.csw, c.m0 + 4.0, c.H64.as<double>(), c.st);
    } else {
      size_t bytes = sizeof(cx<double>) * (size_t)c.g.V * 72;
      const cx<double>* src = (const cx<double>*)clover;
      DevBuf stage;
      if (!on_device) {
        stage.alloc(bytes);
        HIP_CHECK(hipMemcpyAsync(stage.p, clover, bytes, hipMemcpyHostToDevice, c.st));
        src = stage.as<cx<double>>();
      }
      check_finite(c, (const double*)src, (long)c.g.V * 144);
      launch_clover_from_lex(c.g, src, c.m0 + 4.0, c.H64.as<double>(), c.st);
    }
    c.have_32 = false;
    c.u16_kind = -1;
    c.rebuild_odd_inverse();
    c.sync();
    c.have_setup = false;
    c.mg.reset();
    return DDAMG_OK;
  });
}

int ddamg_get_clover(ddamg_ctx* ctx, void* clover) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    need_gauge(c);
    if (!clover) throw Error(INVALID_ARG, "clover is NULL");
    size_t bytes = sizeof(cx<double>) * (size_t)c.g.V * 72;
    DevBuf stage;
    stage.alloc(bytes);
    launch_clover_to_lex(c.g, c.H64.as<double>(), c.m0 + 4.0, stage.as<cx<double>>(), c.st);
    HIP_CHECK(hipMemcpyAsync(clover, stage.p, bytes, hipMemcpyDeviceToHost, c.st));
    c.sync();
    return DDAMG_OK;
  });
}

int ddamg_set_mu(ddamg_ctx* ctx, double mu) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    if (!std::isfinite(mu)) throw Error(INVALID_ARG, "mu must be finite");
    c.mu = mu;
    c.mu_odd = mu;
    if (c.have_gauge) c.rebuild_odd_inverse();
    if (c.mg) c.mg->set_twist(c.twist());
    c.sync();
    return DDAMG_OK;
  });
}

int ddamg_set_mu_eo(ddamg_ctx* ctx, double mu_even, double mu_odd) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    if (!std::isfinite(mu_even) || !std::isfinite(mu_odd)) throw Error(INVALID_ARG, "twists must be finite");
    c.mu = mu_even;
    c.mu_odd = mu_odd;
    if (c.have_gauge) c.rebuild_odd_inverse();
    if (c.mg) c.mg->set_twist(c.twist());
    c.sync();
    return DDAMG_OK;
  });
}

static int do_build(ddamg_ctx* ctx, const ddamg_params* p, const void* const* vecs, int on_device, bool run_setup) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    need_gauge(c);
    check_params(p);
    if (!vecs) throw Error(INVALID_ARG, "init vectors are NULL");
    for (int l = 0; l < p->levels - 1; ++l)
      if (!vecs[l]) throw Error(INVALID_ARG, "init vectors are NULL");
    c.have_setup = false;
    c.mg.reset();
    c.p = *p;
    c.mg = make_mg(c);
    c.mg->build(vecs, on_device, run_setup);
    c.have_setup = true;
    return DDAMG_OK;
  });
}

int ddamg_setup(ddamg_ctx* ctx, const ddamg_params* p, const void* const* init_vectors, int on_device) {
  return do_build(ctx, p, init_vectors, on_device, true);
}
int ddamg_setup_prec(ddamg_ctx* ctx, const ddamg_params* p, const void* const* init_vectors, int fine_precision,
                     int on_device) {
  if (fine_precision == DDAMG_FP64) return do_build(ctx, p, init_vectors, on_device, true);
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    need_gauge(c);
    check_params(p);
    if (fine_precision != DDAMG_FP32)
      throw Error(INVALID_ARG, "fine initial vectors must be complex128 (DDAMG_FP64) or complex64 (DDAMG_FP32)");
    if (!init_vectors || !init_vectors[0] || (p->levels == 3 && !init_vectors[1]))
      throw Error(INVALID_ARG, "init vectors are NULL");
    const long fl = c.fine_len();
    c.have_setup = false;
    c.mg.reset();
    c.p = *p;
    c.mg = make_mg(c);
    c.lex.ensure(sizeof(cx<double>) * fl);
    c.f64b.ensure(sizeof(cx<double>) * fl);
    c.f32a.ensure(sizeof(cx<float>) * fl);
    for (int i = 0; i < p->nvec[0]; ++i) {
      // complex64 lexicographic -> FP64 lexicographic staging -> FP32 block layout
      const cx<float>* src = (const cx<float>*)init_vectors[0] + (long)i * fl;
      if (!on_device) {
        HIP_CHECK(hipMemcpyAsync(c.f64b.p, src, sizeof(cx<float>) * fl, hipMemcpyHostToDevice, c.st));
        src = c.f64b.as<cx<float>>();
      }
      launch_copy_cvt<float, double>(src, c.lex.as<cx<double>>(), fl, c.st);
      launch_from_lex<float>(c.g, c.lex.as<cx<double>>(), c.f32a.as<cx<float>>(), 12, c.st);
      c.mg->load_fine_vec(i, c.f32a.as<cx<float>>());
    }
    const void* vecs[3] = {nullptr, init_vectors[1], nullptr};
    c.mg->build(vecs, on_device, true);
    c.have_setup = true;
    return DDAMG_OK;
  });
}

int ddamg_set_test_vectors(ddamg_ctx* ctx, const ddamg_params* p, const void* const* vectors, int on_device) {
  return do_build(ctx, p, vectors, on_device, false);
}

int ddamg_solve(ddamg_ctx* ctx, const void* b, void* x, int nrhs, double tol, ddamg_stats* stats, int on_device) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    need_setup(c);
    if (!b || !x || nrhs <= 0) throw Error(INVALID_ARG, "bad right-hand side arguments");
    if (!(tol > 0) || !std::isfinite(tol)) throw Error(INVALID_ARG, "tol must be > 0");
    auto t0 = std::chrono::steady_clock::now();
    long N = c.fine_len();
    c.f64c.ensure(sizeof(cx<double>) * N);
    std::function<void(const cx<double>*, cx<double>*)> A = [&c](const cx<double>* in, cx<double>* out) {
      c.dirac64(in, out, c.twist());
    };
    std::function<void(const cx<double>*, cx<double>*)> M = [&c](const cx<double>* in, cx<double>* out) {
      c.mg->precond(in, out);
    };
    for (int l = 0; l < 4; ++l) c.mg->coarse_iters[l] = 0;
    c.mg->vcycles = 0;
    int total_it = 0, it_min = 1 << 30, it_max = 0;
    double worst_all = 0;
    bool all_conv = true;
    KrylovResult kr;
    const int Kb = std::min(nrhs, c.p.rhs_batch);
    if (Kb > 1) {
      // right-hand sides in groups of Kb through one lock-step outer FGMRES
      // (the one-column workspace is not allocated on this path)
      // reduced-precision hierarchies: the preconditioned directions (the
      // cycle's FP32 output) are kept in FP32, halving that half of the basis
      const bool zf = c.p.precision != DDAMG_FP64;
      KrylovWSm<double>& ws = c.outer_m;
      ws.init(c.p.restart, Kb, N, N, true, zf, true);
      DevBuf bK, xK;
      bK.alloc(sizeof(cx<double>) * N * Kb, true);
      xK.alloc(sizeof(cx<double>) * N * Kb, true);
      OpM<double> AK = [&c, N](const cx<double>* in, cx<double>* out, int K) {
        c.dirac64_multi(in, out, K, N, c.twist());
      };
      OpM<double> MK = [&c](const cx<double>* in, cx<double>* out, int K) { c.mg->precond_multi(in, out, K); };
      OpMf MKf = [&c](const cx<double>* in, cx<float>* out, int K) { c.mg->precond_multi_f32(in, out, K); };
      double worst = 0;
      for (int r0 = 0; r0 < nrhs; r0 += Kb) {
        const int k = std::min(Kb, nrhs - r0);
        for (int q = 0; q < k; ++q) {
          const char* bs = (const char*)b + sizeof(cx<double>) * (size_t)N * (r0 + q);
          c.upload_fine(bs, on_device, bK.as<cx<double>>() + (long)q * N);
          check_finite(c, (const double*)(bK.as<cx<double>>() + (long)q * N), 2 * N);
        }
        KrylovResultM km = fgmres_multi<double>(c, ws, k, N, AK, zf ? nullptr : &MK, bK.as<cx<double>>(),
                                                xK.as<cx<double>>(), tol, c.p.max_iter, false, true, zf ? &MKf : nullptr);
        for (int q = 0; q < k; ++q) {
          char* xs = (char*)x + sizeof(cx<double>) * (size_t)N * (r0 + q);
          c.download_fine(xK.as<cx<double>>() + (long)q * N, xs, on_device);
          total_it += km.iters[q];
          it_min = std::min(it_min, km.iters[q]);
          it_max = std::max(it_max, km.iters[q]);
          all_conv = all_conv && km.converged[q];
          worst = std::max(worst, km.resid[q]);
        }
      }
      worst_all = std::max(worst_all, worst);
    }
    if (Kb <= 1) c.outer.init(c.p.restart, N, N, true);
    for (int r = Kb > 1 ? nrhs : 0; r < nrhs; ++r) {
      const char* bs = (const char*)b + sizeof(cx<double>) * (size_t)N * r;
      char* xs = (char*)x + sizeof(cx<double>) * (size_t)N * r;
      c.upload_fine(bs, on_device, c.f64a.as<cx<double>>());
      check_finite(c, (const double*)c.f64a.p, 2 * N);
      kr = fgmres<double>(c, c.outer, N, A, &M, c.f64a.as<cx<double>>(), c.f64b.as<cx<double>>(), tol, c.p.max_iter,
                          false, true);
      total_it += kr.iters;
      it_min = std::min(it_min, kr.iters);
      it_max = std::max(it_max, kr.iters);
      worst_all = std::max(worst_all, kr.resid);
      all_conv = all_conv && kr.converged;
      c.download_fine(c.f64b.as<cx<double>>(), xs, on_device);
    }
    c.sync();
    // the outer Krylov basis is the largest allocation: its ranges go back to
    // the context's pool between solves, for the setup's buffers to reuse
    c.outer.V.release();
    c.outer.Z.release();
    c.outer.tmp.release();
    c.outer_m.V.release();
    c.outer_m.Z.release();
    c.outer_m.r.release();
    if (stats) {
      stats->iters = total_it;
      stats->converged = all_conv ? 1 : 0;
      stats->resid = worst_all;
      for (int l = 0; l < 4; ++l) stats->coarse_iters[l] = c.mg->coarse_iters[l];
      stats->vcycles = c.mg->vcycles;
      stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      stats->nrhs = nrhs;
      stats->iters_min = it_min;
      stats->iters_max = it_max;
    }
    if (!all_conv) {
      c.err = "FGMRES reached max_iter before the tolerance";
      return DDAMG_NOT_CONVERGED;
    }
    return DDAMG_OK;
  });
}

int ddamg_solve_odd_shifted(ddamg_ctx* ctx, const void* b, void* x, double rho, double tol, ddamg_stats* stats,
                            int on_device) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    need_setup(c);
    if (!b || !x) throw Error(INVALID_ARG, "bad right-hand side arguments");
    if (!(tol > 0) || !std::isfinite(tol)) throw Error(INVALID_ARG, "tol must be > 0");
    if (!std::isfinite(rho)) throw Error(INVALID_ARG, "rho must be finite");
    if (c.mu_odd != c.mu)
      throw Error(INVALID_ARG, "the odd-shifted solve starts from one twist on both parities (ddamg_set_mu)");
    auto t0 = std::chrono::steady_clock::now();
    const long N = c.fine_len();
    c.f64c.ensure(sizeof(cx<double>) * N);
    // D(mu) with the odd-site twist raised by rho, preconditioned by the
    // cycle of the setup with the mean twist mu + rho/2 on every site of every
    // level (restored on return)
    const double mu0 = c.mu;
    std::function<void(const cx<double>*, cx<double>*)> A = [&c, mu0, rho](const cx<double>* in, cx<double>* out) {
      c.dirac64(in, out, Twist(mu0));
      launch_odd_twist_add(c.g, in, out, rho, c.st);
    };
    struct TwistScope {
      Ctx& c;
      double mu0;
      bool on;
      void restore() {
        on = false;
        c.mu = c.mu_odd = mu0;
        c.rebuild_odd_inverse();
        c.mg->set_twist(c.twist());
        c.sync();
      }
      // on an error path the solve's own error is the one reported
      ~TwistScope() {
        if (!on) return;
        try {
          restore();
        } catch (...) {
        }
      }
    } scope{c, mu0, rho != 0.0};
    if (rho != 0.0) {
      c.mu = c.mu_odd = mu0 + 0.5 * rho;
      c.rebuild_odd_inverse();
      c.mg->set_twist(c.twist());
    }
    std::function<void(const cx<double>*, cx<double>*)> M = [&c](const cx<double>* in, cx<double>* out) {
      c.mg->precond(in, out);
    };
    for (int l = 0; l < 4; ++l) c.mg->coarse_iters[l] = 0;
    c.mg->vcycles = 0;
    c.outer.init(c.p.restart, N, N, true);
    c.upload_fine(b, on_device, c.f64a.as<cx<double>>());
    check_finite(c, (const double*)c.f64a.p, 2 * N);
    launch_zero_even(c.g, c.f64a.as<cx<double>>(), c.st);
    KrylovResult kr = fgmres<double>(c, c.outer, N, A, &M, c.f64a.as<cx<double>>(), c.f64b.as<cx<double>>(), tol,
                                     c.p.max_iter, false, true);
    c.download_fine(c.f64b.as<cx<double>>(), x, on_device);
    if (scope.on) scope.restore();
    c.sync();
    c.outer.V.release();
    c.outer.Z.release();
    c.outer.tmp.release();
    if (stats) {
      stats->iters = kr.iters;
      stats->converged = kr.converged ? 1 : 0;
      stats->resid = kr.resid;
      for (int l = 0; l < 4; ++l) stats->coarse_iters[l] = c.mg->coarse_iters[l];
      stats->vcycles = c.mg->vcycles;
      stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      stats->nrhs = 1;
      stats->iters_min = kr.iters;
      stats->iters_max = kr.iters;
    }
    if (!kr.converged) {
      c.err = "FGMRES reached max_iter before the tolerance";
      return DDAMG_NOT_CONVERGED;
    }
    return DDAMG_OK;
  });
}

int ddamg_apply_dirac(ddamg_ctx* ctx, const void* in, void* out, int sign, int precision, int on_device) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    need_gauge(c);
    if (!in || !out) throw Error(INVALID_ARG, "NULL field");
    const Twist tw = c.twist(sign);
    long N = c.fine_len();
    c.upload_fine(in, on_device, c.f64a.as<cx<double>>());
    if (precision == DDAMG_FP64) {
      c.dirac64(c.f64a.as<cx<double>>(), c.f64b.as<cx<double>>(), tw);
    } else {
      c.ensure_32();
      c.f32a.ensure(sizeof(cx<float>) * N);
      c.f32b.ensure(sizeof(cx<float>) * N);
      launch_copy_cvt<double, float>(c.f64a.as<cx<double>>(), c.f32a.as<cx<float>>(), N, c.st);
      if (precision == DDAMG_FP32)
        launch_dirac<float, float>(c.g, c.U32.p, c.H32.as<float>(), tw, c.f32a.as<cx<float>>(),
                                   c.f32b.as<cx<float>>(), c.st);
      else if (precision == DDAMG_FP16 || precision == DDAMG_BF16) {
        c.ensure_16(precision);
        if (precision == DDAMG_FP16)
          launch_dirac<float, f16>(c.g, c.U16.p, c.H32.as<float>(), tw, c.f32a.as<cx<float>>(),
                                   c.f32b.as<cx<float>>(), c.st);
        else
          launch_dirac<float, bf16>(c.g, c.U16.p, c.H32.as<float>(), tw, c.f32a.as<cx<float>>(),
                                    c.f32b.as<cx<float>>(), c.st);
      } else
        throw Error(INVALID_ARG, "unknown precision");
      launch_copy_cvt<float, double>(c.f32b.as<cx<float>>(), c.f64b.as<cx<double>>(), N, c.st);
    }
    c.download_fine(c.f64b.as<cx<double>>(), out, on_device);
    c.sync();
    return DDAMG_OK;
  });
}

int ddamg_apply_dirac_multi(ddamg_ctx* ctx, int nfields, const void* in, void* out, int sign, int precision,
                            int on_device) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    need_gauge(c);
    if (!in || !out) throw Error(INVALID_ARG, "NULL field");
    if (nfields < 1 || nfields > 16) throw Error(INVALID_ARG, "nfields must be in [1, 16]");
    if (precision < DDAMG_FP64 || precision > DDAMG_BF16) throw Error(INVALID_ARG, "unknown precision");
    const Twist tw = c.twist(sign);
    const long N = c.fine_len();
    const size_t fb = sizeof(cx<double>) * (size_t)N;
    DevBuf a64, b64;
    a64.alloc(fb * nfields, true);
    b64.alloc(fb * nfields, true);
    for (int k = 0; k < nfields; ++k)
      c.upload_fine((const char*)in + fb * k, on_device, a64.as<cx<double>>() + (long)k * N);
    if (precision == DDAMG_FP64) {
      c.dirac64_multi(a64.as<cx<double>>(), b64.as<cx<double>>(), nfields, N, tw);
    } else {
      c.ensure_32();
      DevBuf a32, b32;
      a32.alloc(sizeof(cx<float>) * (size_t)N * nfields, true);
      b32.alloc(sizeof(cx<float>) * (size_t)N * nfields, true);
      launch_copy_cvt<double, float>(a64.as<cx<double>>(), a32.as<cx<float>>(), N * nfields, c.st);
      if (precision == DDAMG_FP32) {
        launch_dirac_multi<float, float>(c.g, c.U32.p, c.H32.as<float>(), tw, nfields, N, a32.as<cx<float>>(),
                                         b32.as<cx<float>>(), c.st);
      } else {
        c.ensure_16(precision);
        if (precision == DDAMG_FP16)
          launch_dirac_multi<float, f16>(c.g, c.U16.p, c.H32.as<float>(), tw, nfields, N, a32.as<cx<float>>(),
                                         b32.as<cx<float>>(), c.st);
        else
          launch_dirac_multi<float, bf16>(c.g, c.U16.p, c.H32.as<float>(), tw, nfields, N, a32.as<cx<float>>(),
                                          b32.as<cx<float>>(), c.st);
      }
      launch_copy_cvt<float, double>(b32.as<cx<float>>(), b64.as<cx<double>>(), N * nfields, c.st);
    }
    for (int k = 0; k < nfields; ++k)
      c.download_fine(b64.as<cx<double>>() + (long)k * N, (char*)out + fb * k, on_device);
    c.sync();
    return DDAMG_OK;
  });
}

int ddamg_sap_multi(ddamg_ctx* ctx, int nfields, const void* b, void* x, int iters, int mr_steps, int precision,
                    int on_device) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    need_gauge(c);
    if (!b || !x || iters < 0 || mr_steps < 0) throw Error(INVALID_ARG, "bad SAP arguments");
    if (nfields < 1 || nfields > 16) throw Error(INVALID_ARG, "nfields must be in [1, 16]");
    if (precision < DDAMG_FP64 || precision > DDAMG_BF16) throw Error(INVALID_ARG, "unknown precision");
    const long N = c.fine_len();
    const int K = nfields;
    const size_t fb = sizeof(cx<double>) * (size_t)N;
    // K fields in block layout, stride N: FP64 staging, then the working precision
    DevBuf b64, x64;
    b64.alloc(fb * K);
    x64.alloc(fb * K);
    for (int k = 0; k < K; ++k) {
      c.upload_fine((const char*)b + fb * k, on_device, b64.as<cx<double>>() + (long)k * N);
      c.upload_fine((const char*)x + fb * k, on_device, x64.as<cx<double>>() + (long)k * N);
    }
    if (precision == DDAMG_FP64) {
      for (int it = 0; it < iters; ++it)
        for (int col = 0; col < 2; ++col)
          launch_sap_multi<double, double>(c.g, col, c.U64.p, c.H64.as<double>(), c.M64.as<double>(), c.twist(),
                                           b64.as<cx<double>>(), x64.as<cx<double>>(), mr_steps, K, N, c.st);
    } else {
      c.ensure_32();
      const void* U = c.U32.p;
      if (precision != DDAMG_FP32) {
        c.ensure_16(precision);
        U = c.U16.p;
      }
      DevBuf b32, x32;
      b32.alloc(sizeof(cx<float>) * (size_t)N * K);
      x32.alloc(sizeof(cx<float>) * (size_t)N * K);
      launch_copy_cvt<double, float>(b64.as<cx<double>>(), b32.as<cx<float>>(), N * K, c.st);
      launch_copy_cvt<double, float>(x64.as<cx<double>>(), x32.as<cx<float>>(), N * K, c.st);
      for (int it = 0; it < iters; ++it)
        for (int col = 0; col < 2; ++col) {
          if (precision == DDAMG_FP32)
            launch_sap_multi<float, float>(c.g, col, U, c.H32.as<float>(), c.M32.as<float>(), c.twist(),
                                           b32.as<cx<float>>(), x32.as<cx<float>>(), mr_steps, K, N, c.st);
          else if (precision == DDAMG_FP16)
            launch_sap_multi<float, f16>(c.g, col, U, c.H32.as<float>(), c.M32.as<float>(), c.twist(),
                                         b32.as<cx<float>>(), x32.as<cx<float>>(), mr_steps, K, N, c.st);
          else
            launch_sap_multi<float, bf16>(c.g, col, U, c.H32.as<float>(), c.M32.as<float>(), c.twist(),
                                          b32.as<cx<float>>(), x32.as<cx<float>>(), mr_steps, K, N, c.st);
        }
      launch_copy_cvt<float, double>(x32.as<cx<float>>(), x64.as<cx<double>>(), N * K, c.st);
    }
    for (int k = 0; k < K; ++k) c.download_fine(x64.as<cx<double>>() + (long)k * N, (char*)x + fb * k, on_device);
    c.sync();
    return DDAMG_OK;
  });
}

int ddamg_sap(ddamg_ctx* ctx, const void* b, void* x, int iters, int mr_steps, int precision, int on_device) {
  return ddamg_sap_multi(ctx, 1, b, x, iters, mr_steps, precision, on_device);
}

int ddamg_level_info(ddamg_ctx* ctx, int level, int dims[4], int* ncomp) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    if (level == 0) {
      for (int d = 0; d < 4; ++d) dims[d] = c.g.L[d];
      *ncomp = 12;
      return DDAMG_OK;
    }
    need_setup(c);
    if (level < 0 || level >= c.mg->nlev()) throw Error(INVALID_ARG, "bad level");
    const CoarseGeo& G = c.mg->geo(level);
    for (int d = 0; d < 4; ++d) dims[d] = G.L[d];
    *ncomp = G.n;
    return DDAMG_OK;
  });
}

#define LEVEL_CHECK(lo, hi_off)                                                               \
  need_setup(c);                                                                              \
  if (level < (lo) || level >= c.mg->nlev() - (hi_off)) throw Error(INVALID_ARG, "bad level");

int ddamg_get_interpolation(ddamg_ctx* ctx, int level, void* Q) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    LEVEL_CHECK(0, 1);
    c.mg->get_interp(level, (cx<double>*)Q);
    return DDAMG_OK;
  });
}
int ddamg_restrict(ddamg_ctx* ctx, int level, const void* in, void* out) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    LEVEL_CHECK(0, 1);
    c.mg->restrict_host(level, (const cx<double>*)in, (cx<double>*)out);
    return DDAMG_OK;
  });
}
int ddamg_prolong(ddamg_ctx* ctx, int level, const void* in, void* out) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    LEVEL_CHECK(0, 1);
    c.mg->prolong_host(level, (const cx<double>*)in, (cx<double>*)out);
    return DDAMG_OK;
  });
}
int ddamg_restrict_multi(ddamg_ctx* ctx, int level, int nrhs, const void* in, void* out) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    LEVEL_CHECK(0, 1);
    if (!in || !out || nrhs < 1 || nrhs > 16) throw Error(INVALID_ARG, "bad K-column restriction arguments");
    c.mg->transfer_multi_host(level, 0, nrhs, (const cx<double>*)in, (cx<double>*)out);
    return DDAMG_OK;
  });
}
int ddamg_prolong_multi(ddamg_ctx* ctx, int level, int nrhs, const void* in, void* out) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    LEVEL_CHECK(0, 1);
    if (!in || !out || nrhs < 1 || nrhs > 16) throw Error(INVALID_ARG, "bad K-column prolongation arguments");
    c.mg->transfer_multi_host(level, 1, nrhs, (const cx<double>*)in, (cx<double>*)out);
    return DDAMG_OK;
  });
}
int ddamg_get_coarse_op(ddamg_ctx* ctx, int level, void* S, void* F) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    LEVEL_CHECK(1, 0);
    c.mg->get_coarse_op(level, (cx<double>*)S, (cx<double>*)F);
    return DDAMG_OK;
  });
}
int ddamg_apply_coarse(ddamg_ctx* ctx, int level, const void* in, void* out) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    LEVEL_CHECK(1, 0);
    c.mg->apply_coarse_host(level, (const cx<double>*)in, (cx<double>*)out);
    return DDAMG_OK;
  });
}
int ddamg_coarse_sap(ddamg_ctx* ctx, int level, const void* b, void* x, int iters) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    LEVEL_CHECK(1, 1);
    c.mg->coarse_sap_host(level, (const cx<double>*)b, (cx<double>*)x, iters);
    return DDAMG_OK;
  });
}
int ddamg_coarse_solve(ddamg_ctx* ctx, int level, const void* b, void* x) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    LEVEL_CHECK(1, 0);
    c.mg->coarse_solve_host(level, (const cx<double>*)b, (cx<double>*)x);
    return DDAMG_OK;
  });
}
int ddamg_apply_coarse_multi(ddamg_ctx* ctx, int level, int nrhs, const void* in, void* out) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    LEVEL_CHECK(1, 0);
    if (nrhs < 1 || nrhs > 16 || !in || !out) throw Error(INVALID_ARG, "nrhs must be in [1, 16]");
    c.mg->apply_coarse_multi_host(level, nrhs, (const cx<double>*)in, (cx<double>*)out);
    return DDAMG_OK;
  });
}
int ddamg_coarse_solve_multi(ddamg_ctx* ctx, int level, int nrhs, const void* b, void* x) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    LEVEL_CHECK(1, 0);
    if (nrhs < 1 || nrhs > 16 || !b || !x) throw Error(INVALID_ARG, "nrhs must be in [1, 16]");
    c.mg->coarse_solve_multi_host(level, nrhs, (const cx<double>*)b, (cx<double>*)x);
    return DDAMG_OK;
  });
}
int ddamg_apply_coarse_schur_multi(ddamg_ctx* ctx, int level, int nrhs, const void* in, void* out) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    LEVEL_CHECK(1, 0);
    if (level != c.mg->nlev() - 1) throw Error(INVALID_ARG, "level must be the coarsest");
    if (nrhs < 1 || nrhs > 16 || !in || !out) throw Error(INVALID_ARG, "nrhs must be in [1, 16]");
    c.mg->schur_multi_host(level, nrhs, (const cx<double>*)in, (cx<double>*)out);
    return DDAMG_OK;
  });
}
int ddamg_coarse_sap_multi(ddamg_ctx* ctx, int level, int nrhs, const void* b, void* x, int iters) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    LEVEL_CHECK(1, 1);
    if (nrhs < 1 || nrhs > 16 || !b || !x || iters < 0) throw Error(INVALID_ARG, "nrhs must be in [1, 16]");
    c.mg->coarse_sap_multi_host(level, nrhs, (const cx<double>*)b, (cx<double>*)x, iters);
    return DDAMG_OK;
  });
}
int ddamg_bench_coarse(ddamg_ctx* ctx, int level, int nrhs, int napply, int which) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    LEVEL_CHECK(1, 0);
    if (nrhs < 1 || nrhs > 16 || napply < 0 || which < 0 || which > 1) throw Error(INVALID_ARG, "bad arguments");
    c.mg->bench_coarse_multi(level, nrhs, napply, which);
    return DDAMG_OK;
  });
}
int ddamg_vcycle(ddamg_ctx* ctx, const void* in, void* out) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    need_setup(c);
    c.upload_fine(in, 0, c.f64a.as<cx<double>>());
    c.mg->precond(c.f64a.as<cx<double>>(), c.f64b.as<cx<double>>());
    c.download_fine(c.f64b.as<cx<double>>(), out, 0);
    return DDAMG_OK;
  });
}

int ddamg_bench_dirac(ddamg_ctx* ctx, int precision, int napply) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    need_gauge(c);
    long N = c.fine_len();
    if (precision == DDAMG_FP64) {
      for (int i = 0; i < napply; ++i) {
        const cx<double>* in = (i & 1) ? c.f64b.as<cx<double>>() : c.f64a.as<cx<double>>();
        cx<double>* out = (i & 1) ? c.f64a.as<cx<double>>() : c.f64b.as<cx<double>>();
        c.dirac64(in, out, c.twist());
      }
      return DDAMG_OK;
    }
    c.ensure_32();
    c.f32a.ensure(sizeof(cx<float>) * N);
    c.f32b.ensure(sizeof(cx<float>) * N);
    const void* U = c.U32.p;
    if (precision == DDAMG_FP16 || precision == DDAMG_BF16) {
      c.ensure_16(precision);
      U = c.U16.p;
    }
    for (int i = 0; i < napply; ++i) {
      const cx<float>* in = (i & 1) ? c.f32b.as<cx<float>>() : c.f32a.as<cx<float>>();
      cx<float>* out = (i & 1) ? c.f32a.as<cx<float>>() : c.f32b.as<cx<float>>();
      hipEvent_t a;
      c.timer.begin(4, &a);
      if (precision == DDAMG_FP32) launch_dirac<float, float>(c.g, U, c.H32.as<float>(), c.twist(), in, out, c.st);
      else if (precision == DDAMG_FP16) launch_dirac<float, f16>(c.g, U, c.H32.as<float>(), c.twist(), in, out, c.st);
      else launch_dirac<float, bf16>(c.g, U, c.H32.as<float>(), c.twist(), in, out, c.st);
      c.timer.end(4, a);
    }
    return DDAMG_OK;
  });
}

int ddamg_timing(ddamg_ctx* ctx, int enable) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    if (enable) {
      c.timer.flush();
      c.timer.reset();
      c.timer.on = true;
    } else {
      c.timer.flush();
      c.timer.on = false;
    }
    return DDAMG_OK;
  });
}

int ddamg_timing_query(ddamg_ctx* ctx, int kind, long* count, double* ms) {
  if (!ctx || kind < 0 || kind >= KernelTimer::NKIND) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    c.timer.flush();
    if (count) *count = c.timer.count[kind];
    if (ms) *ms = c.timer.ms[kind];
    return DDAMG_OK;
  });
}

int ddamg_error_reduction(ddamg_ctx* ctx, const void* e0, int on_device, int n, double* rho) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    need_setup(c);
    if (!e0 || !rho || n < 1) throw Error(INVALID_ARG, "bad error-reduction arguments");
    const long N = c.fine_len();
    DevBuf e, t, z, part;
    e.alloc(sizeof(cx<double>) * N);
    t.alloc(sizeof(cx<double>) * N);
    z.alloc(sizeof(cx<double>) * N);
    const int nwg = (int)std::min<long>(1024, (N + 255) / 256);
    part.alloc(sizeof(cx<double>) * (nwg + 1));
    cx<double>* ep = e.as<cx<double>>();
    cx<double>* nrm = part.as<cx<double>>() + nwg;
    auto norm = [&]() {
      launch_multidot<double>(ep, 0, 1, ep, N, part.as<cx<double>>(), nwg, c.st);
      launch_reduce(part.as<cx<double>>(), 1, nwg, nrm, 2, c.st);
      cx<double> h;
      HIP_CHECK(hipMemcpyAsync(&h, nrm, sizeof(h), hipMemcpyDeviceToHost, c.st));
      c.sync();
      return h.re;
    };
    c.upload_fine(e0, on_device, ep);
    check_finite(c, (const double*)ep, 2 * N);
    const double n0 = norm();
    if (!(n0 > 0)) throw Error(INVALID_ARG, "the probe vector is zero");
    for (int i = 0; i < n; ++i) {  // e <- (I - M D) e
      c.dirac64(ep, t.as<cx<double>>(), c.twist());
      c.mg->precond(t.as<cx<double>>(), z.as<cx<double>>());
      launch_sub<double>(N, ep, z.as<cx<double>>(), ep, c.st);
    }
    *rho = std::pow(norm() / n0, 1.0 / n);
    return DDAMG_OK;
  });
}

int ddamg_set_progress(ddamg_ctx* ctx, ddamg_progress_fn fn, void* user) {
  if (!ctx) return DDAMG_INVALID_ARG;
  ctx->c.progress_fn = fn;
  ctx->c.progress_user = fn ? user : nullptr;
  return DDAMG_OK;
}

int ddamg_release_memory(ddamg_ctx* ctx, double* held) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    c.pool.trim();
    if (held) *held = (double)c.pool.reserved();
    return DDAMG_OK;
  });
}

int ddamg_timing_bytes(ddamg_ctx* ctx, int kind, double* bytes) {
  if (!ctx || kind < 0 || kind >= KernelTimer::NKIND || !bytes) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    *bytes = ctx->c.timer.bytes[kind];
    return DDAMG_OK;
  });
}
int ddamg_timing_flops(ddamg_ctx* ctx, int kind, double* flops) {
  if (!ctx || kind < 0 || kind >= KernelTimer::NKIND || !flops) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    *flops = ctx->c.timer.flops[kind];
    return DDAMG_OK;
  });
}

}  // extern "C"

// ===========================================================================
// learned setup: gauge-covariant network (forward, loss, backward, Adam)
namespace {

void net_need(Ctx& c) {
  need_gauge(c);
  if (c.net.L == 0) throw Error(BAD_STATE, "no network created");
}

void net_buffers(Ctx& c) {
  NetState& n = c.net;
  if (n.V == c.g.V) return;
  long f = (long)n.C * c.fine_len();  // complex entries of one C-channel field
  n.act.alloc(sizeof(cx<float>) * f * (n.L + 1));
  n.zb.alloc(sizeof(cx<float>) * f * n.L);
  n.sb.alloc(sizeof(float) * (long)n.C * c.g.V * std::max(1, n.L - 1));
  n.g1.alloc(sizeof(cx<float>) * f);
  n.g2.alloc(sizeof(cx<float>) * f);
  n.gpart.alloc(sizeof(double) * 2 * (long)n.C * ((c.g.V + 255) / 256));
  n.wpart.alloc(sizeof(cx<float>) * 256L * n.nWc);
  n.lscr.alloc(sizeof(cx<double>) * 2L * c.g.nblocks * 3 * n.C * n.C);
  n.lpart.alloc(sizeof(double) * 2L * c.g.nblocks);
  n.V = c.g.V;
}

// C fields in the host layout (FP64, contiguous) -> C-channel block-layout FP32 field
void net_upload(Ctx& c, const void* src, int on_device, cx<float>* dst) {
  long fl = c.fine_len();
  for (int ch = 0; ch < c.net.C; ++ch) {
    const char* s = (const char*)src + sizeof(cx<double>) * (size_t)fl * ch;
    c.upload_fine(s, on_device, c.f64a.as<cx<double>>());
    launch_copy_cvt<double, float>(c.f64a.as<cx<double>>(), dst + (long)ch * fl, fl, c.st);
  }
}

void net_forward(Ctx& c) {
  NetState& n = c.net;
  long f = (long)n.C * c.fine_len();
  cx<float>* act = n.act.as<cx<float>>();
  cx<float>* zb = n.zb.as<cx<float>>();
  for (int l = 0; l < n.L; ++l) {
    launch_net_mix(c.g, n.C, c.U32.as<cx<float>>(), act + (long)l * f, n.W(l), zb + (long)l * f, false, c.st);
    if (l < n.L - 1)
      launch_net_gate(c.g, n.C, zb + (long)l * f, n.ab(l), n.ab(l) + n.C, act + (long)(l + 1) * f,
                      n.sb.as<float>() + (long)l * n.C * c.g.V, c.st);
  }
}

// forward pass with two C-channel buffers (inference: no activations kept);
// `in` holds the input and is overwritten; returns the buffer with the output
cx<float>* net_infer(Ctx& c, cx<float>* in, cx<float>* tmp) {
  NetState& n = c.net;
  // matrix cores when the channel count and the lattice allow (FP32 accuracy
  // from split BF16 products)
  const bool mf = n.C % 8 == 0 && n.C <= 24 && c.g.V % 64 == 0;
  const long per = net_packed_bytes(n.C) / (long)sizeof(bf16);
  if (mf) {
    n.packed.ensure(sizeof(bf16) * per * n.L);
    for (int l = 0; l < n.L; ++l) launch_net_pack(n.C, n.W(l), n.packed.as<bf16>() + l * per, c.st);
  }
  for (int l = 0; l < n.L; ++l) {
    if (mf)
      launch_net_mix_mfma(c.g, n.C, c.U32.as<cx<float>>(), in, n.packed.as<bf16>() + l * per, tmp, c.st);
    else
      launch_net_mix(c.g, n.C, c.U32.as<cx<float>>(), in, n.W(l), tmp, false, c.st);
    if (l < n.L - 1) launch_net_gate_inplace(c.g, n.C, n.ab(l), n.ab(l) + n.C, tmp, c.st);
    std::swap(in, tmp);
  }
  return in;
}

// loss of the last layer's output against targets (in g2); gradient into g1
double net_loss(Ctx& c) {
  NetState& n = c.net;
  long f = (long)n.C * c.fine_len();
  double inv_norm = 1.0 / ((double)n.C * 2.0 * c.g.nblocks);
  launch_net_loss(c.g, n.C, n.zb.as<cx<float>>() + (long)(n.L - 1) * f, n.g2.as<cx<float>>(), inv_norm,
                  n.lscr.as<cx<double>>(), n.g1.as<cx<float>>(), n.lpart.as<double>(), c.st);
  std::vector<double> lp(2L * c.g.nblocks);
  HIP_CHECK(hipMemcpyAsync(lp.data(), n.lpart.p, sizeof(double) * lp.size(), hipMemcpyDeviceToHost, c.st));
  c.sync();
  double L = 0;
  for (double v : lp) L += v;
  return L;
}

void net_backward(Ctx& c) {
  NetState& n = c.net;
  long f = (long)n.C * c.fine_len();
  cx<float>* act = n.act.as<cx<float>>();
  cx<float>* zb = n.zb.as<cx<float>>();
  cx<float>* G = n.g1.as<cx<float>>();   // gradient w.r.t. this layer's output
  cx<float>* Gz = n.g2.as<cx<float>>();
  int nwgw = (int)std::min<long>(256, std::max<long>(1, c.g.V / 8 / 4));
  for (int l = n.L - 1; l >= 0; --l) {
    cx<float>* gz = G;
    if (l < n.L - 1) {
      launch_net_gate_bwd(c.g, n.C, G, zb + (long)l * f, n.sb.as<float>() + (long)l * n.C * c.g.V, n.ab(l), Gz,
                          n.gpart.as<double>(), n.Gab(l), n.Gab(l) + n.C, c.st);
      gz = Gz;
    }
    launch_net_wgrad(c.g, n.C, c.U32.as<cx<float>>(), act + (long)l * f, gz, n.wpart.as<cx<float>>(), nwgw, n.GW(l),
                     c.st);
    if (l > 0) {
      cx<float>* dst = (gz == G) ? Gz : G;
      launch_net_mix(c.g, n.C, c.U32.as<cx<float>>(), gz, n.W(l), dst, true, c.st);
      G = dst;
      Gz = (dst == n.g1.as<cx<float>>()) ? n.g2.as<cx<float>>() : n.g1.as<cx<float>>();
    }
  }
}

void net_params_to_host(const NetState& n, const DevBuf& buf, double* out, hipStream_t st) {
  std::vector<float> h(n.nreal);
  HIP_CHECK(hipMemcpyAsync(h.data(), buf.p, sizeof(float) * n.nreal, hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  for (long i = 0; i < n.nreal; ++i) out[i] = h[i];
}

}  // namespace

extern "C" {

int ddamg_setup_learned(ddamg_ctx* ctx, const ddamg_params* p, const void* noise, int noise_precision,
                        int on_device, const void* coarse_init) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    need_gauge(c);
    check_params(p);
    if (c.net.L == 0) throw Error(BAD_STATE, "no network: call ddamg_net_create and ddamg_net_set_params");
    if (p->nvec[0] != c.net.C) throw Error(INVALID_ARG, "nvec[0] must equal the network's channel count");
    if (!noise || (p->levels == 3 && !coarse_init)) throw Error(INVALID_ARG, "NULL input");
    if (noise_precision != DDAMG_FP64 && noise_precision != DDAMG_FP32)
      throw Error(INVALID_ARG, "noise must be complex128 (DDAMG_FP64) or complex64 (DDAMG_FP32)");
    c.ensure_32();
    const long fl = c.fine_len(), f = (long)c.net.C * fl;
    DevBuf A, B;
    A.alloc(sizeof(cx<float>) * f, true);
    B.alloc(sizeof(cx<float>) * f, true);
    c.lex.ensure(sizeof(cx<double>) * fl);
    for (int ch = 0; ch < c.net.C; ++ch) {
      cx<float>* dst = A.as<cx<float>>() + (long)ch * fl;
      if (noise_precision == DDAMG_FP64) {
        c.upload_fine((const char*)noise + sizeof(cx<double>) * (size_t)fl * ch, on_device, c.f64a.as<cx<double>>());
        launch_copy_cvt<double, float>(c.f64a.as<cx<double>>(), dst, fl, c.st);
      } else {
        // complex64 lexicographic -> FP64 lexicographic staging -> block layout FP32
        const cx<float>* src = (const cx<float>*)noise + (long)ch * fl;
        if (!on_device) {
          HIP_CHECK(hipMemcpyAsync(c.f64b.p, src, sizeof(cx<float>) * fl, hipMemcpyHostToDevice, c.st));
          src = c.f64b.as<cx<float>>();
        }
        launch_copy_cvt<float, double>(src, c.lex.as<cx<double>>(), fl, c.st);
        launch_from_lex<float>(c.g, c.lex.as<cx<double>>(), dst, 12, c.st);
      }
    }
    cx<float>* out = net_infer(c, A.as<cx<float>>(), B.as<cx<float>>());
    c.have_setup = false;
    c.mg.reset();
    c.p = *p;
    c.mg = make_mg(c);
    c.mg->load_fine_init(out);
    A.release();
    B.release();
    const void* vecs[3] = {nullptr, coarse_init, nullptr};
    c.mg->build(vecs, on_device, true);
    c.have_setup = true;
    return DDAMG_OK;
  });
}



int ddamg_net_create(ddamg_ctx* ctx, int nlayers, int nchan) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    if (nlayers < 1 || nlayers > 16) throw Error(INVALID_ARG, "nlayers must be in 1..16");
    if (!(nchan == 4 || nchan == 8 || nchan == 12 || nchan == 16 || nchan == 24))
      throw Error(INVALID_ARG, "nchan must be 4, 8, 12, 16 or 24");
    if (c.g.V % 64) throw Error(INVALID_ARG, "the network needs a lattice volume divisible by 64");
    NetState& n = c.net;
    n.L = nlayers;
    n.C = nchan;
    n.nWc = 9L * nchan * nchan * 16;
    n.nreal = 2L * nlayers * n.nWc + 2L * (nlayers - 1) * nchan;
    n.params.alloc(sizeof(float) * n.nreal);
    n.grads.alloc(sizeof(float) * n.nreal);
    n.m.alloc(sizeof(float) * n.nreal);
    n.v.alloc(sizeof(float) * n.nreal);
    HIP_CHECK(hipMemsetAsync(n.params.p, 0, sizeof(float) * n.nreal, c.st));
    HIP_CHECK(hipMemsetAsync(n.grads.p, 0, sizeof(float) * n.nreal, c.st));
    HIP_CHECK(hipMemsetAsync(n.m.p, 0, sizeof(float) * n.nreal, c.st));
    HIP_CHECK(hipMemsetAsync(n.v.p, 0, sizeof(float) * n.nreal, c.st));
    n.V = 0;
    n.step = 0;
    c.sync();
    return DDAMG_OK;
  });
}

long ddamg_net_num_params(ddamg_ctx* ctx) { return ctx ? ctx->c.net.nreal : -1; }

int ddamg_net_set_params(ddamg_ctx* ctx, const double* params, long n) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    if (c.net.L == 0) throw Error(BAD_STATE, "no network created");
    if (!params || n != c.net.nreal) throw Error(INVALID_ARG, "parameter count mismatch");
    std::vector<float> h(n);
    for (long i = 0; i < n; ++i) {
      if (!std::isfinite(params[i])) throw Error(NUMERICAL, "non-finite network parameter");
      h[i] = (float)params[i];
    }
    HIP_CHECK(hipMemcpyAsync(c.net.params.p, h.data(), sizeof(float) * n, hipMemcpyHostToDevice, c.st));
    HIP_CHECK(hipMemsetAsync(c.net.m.p, 0, sizeof(float) * n, c.st));
    HIP_CHECK(hipMemsetAsync(c.net.v.p, 0, sizeof(float) * n, c.st));
    c.net.step = 0;
    c.sync();
    return DDAMG_OK;
  });
}

int ddamg_net_get_params(ddamg_ctx* ctx, double* params, long n) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    if (c.net.L == 0) throw Error(BAD_STATE, "no network created");
    if (!params || n != c.net.nreal) throw Error(INVALID_ARG, "parameter count mismatch");
    net_params_to_host(c.net, c.net.params, params, c.st);
    return DDAMG_OK;
  });
}

int ddamg_net_forward(ddamg_ctx* ctx, const void* noise, void* out, int on_device) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    net_need(c);
    if (!noise || !out) throw Error(INVALID_ARG, "NULL field");
    c.ensure_32();
    net_buffers(c);
    NetState& n = c.net;
    long fl = c.fine_len();
    net_upload(c, noise, on_device, n.act.as<cx<float>>());
    const cx<float>* y = net_infer(c, n.act.as<cx<float>>(), n.zb.as<cx<float>>());
    for (int ch = 0; ch < n.C; ++ch) {
      launch_copy_cvt<float, double>(y + (long)ch * fl, c.f64b.as<cx<double>>(), fl, c.st);
      char* dst = (char*)out + sizeof(cx<double>) * (size_t)fl * ch;
      c.download_fine(c.f64b.as<cx<double>>(), dst, on_device);
    }
    c.sync();
    return DDAMG_OK;
  });
}

// forward + loss + backward; grads (optional, host FP64, parameter layout)
int ddamg_net_loss_grad(ddamg_ctx* ctx, const void* noise, const void* target, int on_device, double* loss,
                        double* grads) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    net_need(c);
    if (!noise || !target) throw Error(INVALID_ARG, "NULL field");
    c.ensure_32();
    net_buffers(c);
    NetState& n = c.net;
    net_upload(c, noise, on_device, n.act.as<cx<float>>());
    net_upload(c, target, on_device, n.g2.as<cx<float>>());
    net_forward(c);
    double L = net_loss(c);
    net_backward(c);
    if (loss) *loss = L;
    if (grads) net_params_to_host(n, n.grads, grads, c.st);
    c.sync();
    return DDAMG_OK;
  });
}

int ddamg_net_train_step(ddamg_ctx* ctx, const void* noise, const void* target, int on_device, double lr,
                         double* loss) {
  if (!ctx) return DDAMG_INVALID_ARG;
  return guard(ctx, [&]() {
    Ctx& c = ctx->c;
    net_need(c);
    if (!noise || !target) throw Error(INVALID_ARG, "NULL field");
    if (!(lr > 0) || !std::isfinite(lr)) throw Error(INVALID_ARG, "lr must be > 0");
    c.ensure_32();
    net_buffers(c);
    NetState& n = c.net;
    net_upload(c, noise, on_device, n.act.as<cx<float>>());
    net_upload(c, target, on_device, n.g2.as<cx<float>>());
    net_forward(c);
    double L = net_loss(c);
    net_backward(c);
    n.step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    float c1 = 1.f - std::pow(b1, (float)n.step), c2 = 1.f - std::pow(b2, (float)n.step);
    launch_adam(n.nreal, n.params.as<float>(), n.grads.as<float>(), n.m.as<float>(), n.v.as<float>(), (float)lr, b1,
                b2, 1e-8f, c1, c2, c.st);
    c.sync();
    if (loss) *loss = L;
    return DDAMG_OK;
  });
}

}  // extern "C"
