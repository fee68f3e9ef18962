/*
 * ddamg.h -- C interface of the MI355X (gfx950) DD-alpha-AMG library for
 * twisted-mass Wilson-clover fermions.
 *
 * The method follows Bacchio, Alexandrou, Finkenrath, Frommer, Kahl,
 * Rottmann, "DDalphaAMG for Twisted Mass Fermions" (PoS LATTICE2016):
 *   - Sec. 1: flexible GMRES preconditioned at every step by the multigrid
 *     cycle of Eq. (1), SAP smoother, Gamma5-compatible aggregation P,
 *     coarse operator D_c = P^dag D_W P, twisted-mass operator
 *     D(+-mu) = D_W +- i Gamma5 mu with D_c(mu) = D_c + i mu Gamma5,c and the
 *     raised coarsest twist mu_coarse = delta * mu;
 *   - Sec. 2: gamma5 = diag(-1,-1,1,1), lexicographic site order TZYX,
 *     three levels with 4^4 and 2^4 aggregates, a minimal init interface plus
 *     defaulted parameters;
 *   - Sec. 3: Listing 1 parameter names (MGBlock*, MGSetupIter,
 *     MGCoarseSetupIter, MGNumberOfVectors, MGNumberOfLevels,
 *     MGCoarseMuFactor); odd-even preconditioning only in the smoother and on
 *     the coarsest level; one setup serves D(+mu) and D(-mu).
 *
 * Conventions of every host array (complex numbers are interleaved double
 * pairs, i.e. C99 double complex / numpy complex128):
 *   lattice extents dims = {T, Z, Y, X}; site index ((t*Z + z)*Y + y)*X + x;
 *   links   [V][4][3][3]  direction 0:T 1:Z 2:Y 3:X, row-major 3x3 SU(3);
 *   spinor  [V][4][3]     spin, colour;
 *   clover  [V][2][6][6]  the two chirality blocks of the clover term A(x)
 *                         (block 0: spins 0,1; 6-index = 3*(spin%2)+colour),
 *                         without the mass term m0 + 4;
 *   coarse vectors on level l >= 1: [Vl][n] with n = 2*nvec[l-1], sites in
 *     lexicographic order of the level-l lattice (dims / product of blocks),
 *     components [0, n/2) with Gamma5,c = -1, [n/2, n) with Gamma5,c = +1.
 * The gamma basis is the chiral one: g_k = [[0,-i s_k],[i s_k,0]] for k = X,Y,Z,
 * g_T = [[0,-1],[-1,0]]; D_W is the textbook Wilson + Sheikholeslami-Wohlert
 * operator in mass normalisation, m0 = 1/(2 kappa) - 4.
 *
 * Ownership: the caller owns every buffer it passes; the library copies what
 * it needs into its own device memory and never keeps a caller pointer after
 * a call returns.  `on_device` = 1 means the pointer is device memory of the
 * current HIP device (e.g. a torch tensor's data_ptr()), used on the
 * context's stream; 0 means host memory.
 *
 * Errors: every int-returning function returns a status (DDAMG_OK = 0).
 * Nothing is thrown across the interface and nothing exits the process;
 * ddamg_last_error() gives the message of the last failing call.
 * One context must not be used by two threads at once.
 */
#ifndef DDAMG_H
#define DDAMG_H

#ifdef __cplusplus
extern "C" {
#endif

#define DDAMG_OK 0
#define DDAMG_NOT_CONVERGED 1
#define DDAMG_INVALID_ARG (-1)
#define DDAMG_BAD_STATE (-2)
#define DDAMG_HIP_ERROR (-3)
#define DDAMG_OUT_OF_MEMORY (-4)
#define DDAMG_NUMERICAL (-5)

/* preconditioner precision (the outer FGMRES is always FP64) */
#define DDAMG_FP64 0
#define DDAMG_FP32 1
#define DDAMG_FP16 2 /* fine links and coarse operators stored in FP16, FP32 arithmetic */
#define DDAMG_BF16 3 /* same with BF16 storage */

typedef struct ddamg_ctx ddamg_ctx;

/* Solver parameters.  Names follow Listing 1 (Sec. 3) where the paper gives
 * one; everything else is a reading of the paper's silence, with the default
 * set by ddamg_default_params(). */
typedef struct ddamg_params {
  int levels;                  /* MGNumberOfLevels: 2 or 3 */
  int block[3][4];             /* MGBlockT/Z/Y/X per level transition; block[0] must equal the
                                  block given to ddamg_create (fine SAP block = first aggregate) */
  int nvec[3];                 /* MGNumberOfVectors per level transition */
  int coarse_sap_block[4];     /* SAP blocks on intermediate coarse levels (coarse sites) */
  int sap_pre, sap_post;       /* j, k of Eq. (1) on the fine level (default 0, 3) */
  int mr_steps;                /* MR steps per fine SAP block solve (default 4) */
  int coarse_sap_post;         /* SAP iterations on intermediate levels (default 2) */
  int coarse_mr_steps;         /* MR steps per coarse SAP block solve (default 3) */
  int init_sap_iters;          /* smoothing of the random test vectors (default 3) */
  int setup_iters;             /* MGSetupIter (default 3) */
  int coarse_setup_iters;      /* MGCoarseSetupIter (default 3) */
  double coarse_mu_factor;     /* MGCoarseMuFactor, delta (default 1) */
  int restart, max_iter;       /* outer FGMRES(m) (default 10, 1000) */
  int inter_restart, inter_max_iter; /* intermediate-level FGMRES (default 10, 10) */
  double inter_tol;            /* (default 0.1) */
  int coarse_restart, coarse_max_iter; /* coarsest odd-even GMRES (default 30, 300) */
  double coarse_tol;           /* (default 0.1) */
  int precision;               /* DDAMG_FP64 / FP32 / FP16 / BF16 */
  int fixed_iters;             /* 1: inner solves run exactly their max iteration counts */
  int batch;                   /* test vectors the setup advances together through one lock-step
                                  V-cycle (1 = one at a time; default 16, at most 16).  With
                                  FP16/BF16 storage the coarse operators of a batch run on the
                                  matrix cores. */
  int rhs_batch;               /* right-hand sides ddamg_solve advances together: one lock-step
                                  outer FGMRES whose V-cycles and coarse solves serve all of them
                                  (default 1, at most 16).  Each holds its own FP64 Krylov basis of
                                  2 * restart + 1 fine fields. */
  int keep_test_vectors;       /* 1: the setup keeps its test vectors (nvec[l] fields per level
                                  transition) for ddamg_update_gauge; 0: they are freed when the
                                  setup ends (default) */
} ddamg_params;

typedef struct ddamg_stats {
  int iters;             /* outer FGMRES iterations, summed over the right-hand sides */
  int converged;         /* 1 if the true relative residual <= tol (every right-hand side) */
  double resid;          /* true relative residual |b - D x| / |b| in FP64, largest over the
                            right-hand sides */
  long coarse_iters[4];  /* Krylov iterations per level (index = level), summed over right-hand sides */
  long vcycles;          /* fine-level V-cycles */
  double seconds;        /* wall time of the call */
  int nrhs;              /* right-hand sides solved */
  int iters_min;         /* fewest outer iterations of one right-hand side */
  int iters_max;         /* most outer iterations of one right-hand side */
} ddamg_stats;

/* Fill p with the defaults documented above (2 levels, 4^4 then 2^4 blocks,
 * nvec 24 then 32). */
void ddamg_default_params(ddamg_params* p);

/* Create a context.  dims {T,Z,Y,X}: even extents; block {bT,bZ,bY,bX}: even
 * block extents dividing dims with an even number of blocks per direction
 * (SAP domains, red/black coloured; Sec. 1 SAP).  mu: twisted mass in mass
 * normalisation (Sec. 1, D(mu) = D_W + i Gamma5 mu).  stream: hipStream_t on
 * which every kernel runs (NULL: the null stream).  Returns INVALID_ARG on bad
 * shapes, HIP_ERROR if no device is usable. */
int ddamg_create(const int dims[4], const int block[4], double kappa, double csw, double mu, void* stream,
                 ddamg_ctx** out);
void ddamg_destroy(ddamg_ctx* ctx);
const char* ddamg_last_error(const ddamg_ctx* ctx);

/* Gauge field U_mu(x) (links layout above).  Builds the clover term from the
 * links with the csw of ddamg_create (Sec. 1: Wilson clover operator).
 * Returns NUMERICAL if a link is not finite. */
int ddamg_set_gauge(ddamg_ctx* ctx, const void* links, int on_device);
/* Twisted boundary conditions (Sec. 2, the features the library adds):
 * psi(x + L_mu e_mu) = e^{i theta_mu} psi(x) in direction mu = 0:T 1:Z 2:Y
 * 3:X; theta = {pi, 0, 0, 0} is antiperiodic in time, all zero (the default)
 * periodic.  The library carries the phase on the links that cross the
 * boundary (U_mu(x) with x_mu = L_mu - 1), so every level and kernel sees the
 * same operator; the clover term does not change.  theta: 4 doubles, host,
 * read during the call.  Applies to the field in place (any setup is dropped)
 * and to every field uploaded later.  INVALID_ARG for NULL or non-finite
 * theta. */
int ddamg_set_boundary_phases(ddamg_ctx* ctx, const double theta[4]);
/* Replace the clover term by a caller-supplied one (clover layout above);
 * clover = NULL rebuilds it from the links.  Invalidates any setup. */
int ddamg_set_clover(ddamg_ctx* ctx, const void* clover, int on_device);
/* Copy the clover term the library uses into clover (host, layout above). */
int ddamg_get_clover(ddamg_ctx* ctx, void* clover);
/* Change mu for every later solve, keeping the setup (Sec. 1: the same setup
 * serves D(+mu) and D(-mu)); coarse twists are rescaled (delta on the
 * coarsest level).  Sets the same twist on both parities. */
int ddamg_set_mu(ddamg_ctx* ctx, double mu);
/* Different twisted masses on even and odd sites (Sec. 2 lists this among the
 * library's features; the Hasenbusch terms of Sec. 3.1 need it):
 * D = D_W + i mu(x) Gamma5 with mu(x) = mu_even on even and mu_odd on odd
 * sites (parity of the global coordinate sum), for ddamg_apply_dirac, the
 * SAP entry points and every later setup and solve.  A current setup keeps
 * its P on every level; its coarse operators become the Galerkin products of
 * the new operator: each level's i mu_c Gamma5,c term carries the mean
 * (mu_even + mu_odd)/2 (delta times it on the coarsest level), and the rest,
 * i (mu(x) - mean) Gamma5 summed over each aggregate, enters the coarse site
 * blocks.  When that rest changes, the coarse operators are assembled again
 * from the kept P (about the cost of one Galerkin assembly); otherwise only
 * the twists change.  ddamg_set_mu(mu) is ddamg_set_mu_eo(mu, mu).
 * INVALID_ARG for non-finite twists. */
int ddamg_set_mu_eo(ddamg_ctx* ctx, double mu_even, double mu_odd);

/* Adaptive setup (Sec. 1; setup_iters / coarse_setup_iters of Listing 1).
 * init_vectors[l] (l < levels-1) holds the random starting test vectors of
 * the interpolation from level l to l+1: nvec[l] fields, fine level in the
 * spinor layout, coarse levels in the coarse-vector layout.  The library
 * draws no random numbers itself.  Returns INVALID_ARG for shapes that do
 * not aggregate, NUMERICAL for a rank-deficient aggregate. */
int ddamg_setup(ddamg_ctx* ctx, const ddamg_params* p, const void* const* init_vectors, int on_device);
/* Progress of a long setup (a host-side notification; the method is
 * unchanged).  With fn set, ddamg_setup, ddamg_setup_learned and
 * ddamg_update_gauge call fn(user, stage, level, index) on the calling thread
 * once the context stream has finished that stage: stage 0 when the initial
 * phase of level `level` (its test vectors smoothed, level+1 built) is done,
 * stage 1 when iteration `index` (from 0) of the iterated setup phase on
 * level `level` is done.  Each notification waits for the stream once;
 * fn = NULL (the default) turns it off.  fn must not call the library with
 * the same context.  INVALID_ARG for a NULL context. */
typedef void (*ddamg_progress_fn)(void* user, int stage, int level, int index);
int ddamg_set_progress(ddamg_ctx* ctx, ddamg_progress_fn fn, void* user);
/* ddamg_setup with the fine level's initial vectors in a chosen precision:
 * fine_precision DDAMG_FP64 (complex128, exactly ddamg_setup) or DDAMG_FP32
 * (init_vectors[0] holds nvec[0] complex64 fields in the spinor layout, which
 * halves what the caller keeps resident for them; the setup converts each to
 * its own storage as it reads it).  Coarse-level vectors stay complex128.
 * Errors as for ddamg_setup; INVALID_ARG for another precision. */
int ddamg_setup_prec(ddamg_ctx* ctx, const ddamg_params* p, const void* const* init_vectors, int fine_precision,
                     int on_device);
/* Build the hierarchy directly from given test vectors (no smoothing, no
 * setup iteration): P from their block orthonormalisation, D_c by Galerkin
 * assembly.  Same shapes as ddamg_setup. */
int ddamg_set_test_vectors(ddamg_ctx* ctx, const ddamg_params* p, const void* const* vectors, int on_device);
/* Adaptive setup started from the learned network's vectors instead of random
 * ones (the network of ddamg_net_create / ddamg_net_set_params, C channels;
 * p->nvec[0] must equal C).  noise: the network input, C fields of the fine
 * lattice, lexicographic TZYX [C][V][4][3], complex128 (noise_precision =
 * DDAMG_FP64) or complex64 (DDAMG_FP32), caller-owned, host or device
 * (on_device).  The network runs in FP32 with two C-channel buffers that are
 * freed on return; its output takes the place of init_vectors[0] of
 * ddamg_setup, after which the setup proceeds exactly as there (p->init_sap_iters
 * smoothing, p->setup_iters refinement iterations).  coarse_init: level-1
 * initial vectors for three levels (as init_vectors[1] of ddamg_setup), else
 * ignored. */
int ddamg_setup_learned(ddamg_ctx* ctx, const ddamg_params* p, const void* noise, int noise_precision,
                        int on_device, const void* coarse_init);
/* Error-reduction factor of the current preconditioner (Eq. (1)):
 * rho = (|(I - M D)^n e0| / |e0|)^(1/n), e0 a fine spinor field (host or
 * device, caller-owned, nonzero), n >= 1 applications, all in FP64 on the
 * device (M is the setup's cycle in its stored precision).  This is the probe
 * that decides whether a learned start is kept or the plain setup runs
 * instead.  BAD_STATE without a setup. */
int ddamg_error_reduction(ddamg_ctx* ctx, const void* e0, int on_device, int n, double* rho);
/* Setup update for a changed gauge field (the HMC use of Sec. 3.1: during a
 * trajectory the setup is refreshed by one fine-level and three
 * first-coarse-level iterations instead of being rebuilt).  links: the
 * new field, as for ddamg_set_gauge.  The test vectors of the current
 * setup (kept when it ran with keep_test_vectors = 1; else the columns of its
 * interpolation bases P_l, which span the same space on every aggregate but
 * are not smooth across aggregates) become those of the new one: the library
 * moves them (no copy), then runs ddamg_setup's steps on them with p
 * (p->init_sap_iters smoothing sweeps, usually 0; p->setup_iters fine and
 * p->coarse_setup_iters level-1 iterations, 1 and 3 in the paper's use).
 * With both iteration counts 0 the new D_c is the Galerkin operator of the old
 * P on the new field.  On three levels p->setup_iters > 0 requires
 * p->coarse_setup_iters > 0 (INVALID_ARG otherwise, the current setup kept):
 * the level-1 test vectors are coefficients in the fine basis, which a fine
 * iteration changes.  p must keep the levels, precision, nvec and aggregation
 * blocks of the current setup (INVALID_ARG otherwise).  The old and the new
 * hierarchy are both held while the new one is allocated.  BAD_STATE without a
 * setup; a field with NaN or Inf returns NUMERICAL with the old field and
 * setup intact; any later error leaves the new field and no setup. */
int ddamg_update_gauge(ddamg_ctx* ctx, const void* links, int on_device, const ddamg_params* p);

/* Solve D(mu) x_r = b_r for nrhs right-hand sides (spinor layout, nrhs
 * contiguous fields) with FGMRES preconditioned by Eq. (1), stopping at a
 * true relative residual <= tol computed in FP64.  Returns NOT_CONVERGED
 * (x holds the last iterate) when max_iter is hit; BAD_STATE before setup.
 * st (may be NULL) receives the statistics of the call: iteration counts
 * summed over the right-hand sides, and the fewest and most outer iterations
 * of one right-hand side. */
int ddamg_solve(ddamg_ctx* ctx, const void* b, void* x, int nrhs, double tol, ddamg_stats* st, int on_device);

/* ---- single operators, for parity checks (host or device FP64 arrays) ---- */
/* Hasenbusch-shifted odd-even reduced system (Sec. 3.1): with the odd-site
 * reduced operator Dhat(mu) = D_oo - D_oe D_ee^-1 D_eo and Gamma5hat = Gamma5
 * on the odd sites, solves (Dhat(mu) + i rho Gamma5hat) x_o = b_o as the
 * full-lattice system D(mu; rho) x = (0, b_o), where D(mu; rho) is D(mu) with
 * the odd-site twist raised to mu + rho (the full operator is what the
 * multigrid cycle inverts, as the paper does for odd-even systems).  The
 * outer FGMRES runs on D(mu; rho) in FP64 and is preconditioned by the cycle
 * of the current setup run with the mean twist mu + rho/2 on every site and
 * level (the setup's twist is restored on return).  b: one fine spinor
 * field; its even sites are ignored.  x receives the full solution: its odd
 * sites are x_o, its even sites -D_ee^-1 D_eo x_o.  The second operator of the
 * pair, Gamma5hat Dhat(-mu) Gamma5hat - i rho Gamma5hat, is this solve after
 * ddamg_set_mu(-mu) with -rho and Gamma5 b, followed by Gamma5 on x.  Stops
 * at a true relative residual <= tol of the full system; NOT_CONVERGED, the
 * other errors and st as for ddamg_solve.  INVALID_ARG when the two parities
 * carry different twists (ddamg_set_mu_eo): the same system with a hierarchy
 * built for it is ddamg_set_mu_eo(mu, mu + rho) followed by ddamg_solve on
 * (0, b_o). */
int ddamg_solve_odd_shifted(ddamg_ctx* ctx, const void* b, void* x, double rho, double tol, ddamg_stats* st,
                            int on_device);
/* out = D(sign*mu) in, full lattice (Sec. 1); precision FP64 or FP32 (and
 * FP16/BF16 links with FP32 arithmetic). */
int ddamg_apply_dirac(ddamg_ctx* ctx, const void* in, void* out, int sign, int precision, int on_device);
/* out_k = D(sign*mu) in_k for nfields (1..16) fields in one launch (Sec. 1):
 * in and out hold the fields one after the other (spinor layout above, each
 * field V*12 complex128); the kernel reads the links and the clover term once
 * for all fields, as the lock-step outer solve does.  Same arithmetic per
 * field as ddamg_apply_dirac (bit-identical results); the library stages the
 * fields in device memory of its own for the call.  INVALID_ARG for NULL
 * fields, nfields out of range or an unknown precision; BAD_STATE without a
 * gauge field. */
int ddamg_apply_dirac_multi(ddamg_ctx* ctx, int nfields, const void* in, void* out, int sign, int precision,
                            int on_device);
/* out = D(sign*mu) in in FP64, allocating nothing: for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc).  Same operator and kernels as
 * ddamg_apply_dirac with precision DDAMG_FP64; in and out are device arrays
 * (spinor layout above, complex128, caller-owned, may not alias).  The two
 * block-layout fields it needs live in a scratch array of the library that
 * every device it runs on holds for the life of the process (48 MiB: two
 * fields of at most 131072 sites); lattices with more sites return
 * INVALID_ARG.  The call only enqueues its kernels on the context's stream and
 * returns: out is ready when that stream reaches them.  Every call on one
 * device shares the one scratch array, so calls that can overlap on one GPU
 * (contexts on different streams) race; the array needs no clearing, since
 * each call writes every entry it reads.  sign must be +1 or -1; BAD_STATE
 * without a gauge field. */
int ddamg_apply_dirac_noalloc(ddamg_ctx* ctx, const void* in, void* out, int sign);
/* iters SAP iterations on D x = b starting from x (updated in place): the
 * smoother M of Eq. (1) (Sec. 1), red then black 4^4 blocks, each block solved
 * by mr_steps MR steps on its even-site Schur complement (odd-even in the
 * smoother, Sec. 3).  precision: DDAMG_FP64 or DDAMG_FP32 arithmetic, or
 * DDAMG_FP16 / DDAMG_BF16 link storage with FP32 arithmetic (the links
 * rounded to nearest even once, the clover term and odd-site inverses in
 * FP32).  b, x: spinor layout, host or device. */
int ddamg_sap(ddamg_ctx* ctx, const void* b, void* x, int iters, int mr_steps, int precision, int on_device);
/* The same on nfields (1..16) independent systems D x_k = b_k at once, each
 * colour sweep one launch for all fields (the form the setup and the
 * preconditioner of several right-hand sides use); every field takes the
 * arithmetic of a one-field sweep.  b, x: nfields contiguous spinor fields. */
int ddamg_sap_multi(ddamg_ctx* ctx, int nfields, const void* b, void* x, int iters, int mr_steps, int precision,
                    int on_device);
/* level l >= 0: lattice dims of level l and components per site. */
int ddamg_level_info(ddamg_ctx* ctx, int level, int dims[4], int* ncomp);
/* orthonormalised test vectors spanning P from level l to l+1, level-l layout */
int ddamg_get_interpolation(ddamg_ctx* ctx, int level, void* Q);
/* r_c = P^dag r from level l to l+1; x = P e_c from level l+1 to l. */
int ddamg_restrict(ddamg_ctx* ctx, int level, const void* in, void* out);
int ddamg_prolong(ddamg_ctx* ctx, int level, const void* in, void* out);
/* The same two transfers between levels l and l+1 for nrhs (1..16) columns
 * stored one after the other (host arrays, complex128), through the K-column
 * kernels of the lock-step cycle, which read P once per group of columns
 * (Sec. 1, aggregation-based interpolation).  BAD_STATE without a setup;
 * INVALID_ARG for a bad level, NULL arrays or nrhs out of range. */
int ddamg_restrict_multi(ddamg_ctx* ctx, int level, int nrhs, const void* in, void* out);
int ddamg_prolong_multi(ddamg_ctx* ctx, int level, int nrhs, const void* in, void* out);
/* coarse operator of level l >= 1 as blocks: S [Vl][n][n] (self, without
 * twist) and F [4][Vl][n][n] (forward T,Z,Y,X), row-major, FP64, host. */
int ddamg_get_coarse_op(ddamg_ctx* ctx, int level, void* S, void* F);
/* out = D_c(mu_l) in on level l >= 1 (stored precision). */
int ddamg_apply_coarse(ddamg_ctx* ctx, int level, const void* in, void* out);
/* coarse SAP iterations on level l (intermediate levels). */
int ddamg_coarse_sap(ddamg_ctx* ctx, int level, const void* b, void* x, int iters);
/* coarse solve of level l: odd-even GMRES on the coarsest level, FGMRES with
 * the next level's cycle otherwise (parameters of the last setup). */
int ddamg_coarse_solve(ddamg_ctx* ctx, int level, const void* b, void* x);
/* out = V-cycle (Eq. 1) applied to in on the fine level, x0 = 0. */
int ddamg_vcycle(ddamg_ctx* ctx, const void* in, void* out);
/* The coarse operator of level l >= 1 (Sec. 1, D_c = P^dag D P with the
 * Gamma5,c-hermitian backward couplings and the twist of the level) on nrhs
 * fields at once, 1 <= nrhs <= 16.  in, out: host complex128 [nrhs][len_l],
 * caller-owned, same layout as ddamg_apply_coarse.  With FP16/BF16 storage
 * and 2 N_v a multiple of 16 the products run on the matrix cores with the
 * inputs rounded to the storage format (FP32 accumulation, twist in FP32);
 * otherwise the single-field kernel runs once per field. */
int ddamg_apply_coarse_multi(ddamg_ctx* ctx, int level, int nrhs, const void* in, void* out);
/* The odd-even reduced operator of the coarsest level (Sec. 3: odd-even
 * preconditioning on the coarsest level), S = D_ee - D_eo D_oo^-1 D_oe with the
 * coarsest twist delta*mu in D_ee and D_oo, on nrhs (1..16) fields at once in
 * the form the coarsest GMRES uses (matrix cores for FP16/BF16 storage and
 * 2 N_v a multiple of 16, the inputs of every product rounded to the storage
 * format, FP32 accumulation).  in, out: host complex128 [nrhs][len_l], layout
 * of ddamg_apply_coarse; the odd-site entries of in are not read, those of out
 * are zero.  level must be the coarsest. */
int ddamg_apply_coarse_schur_multi(ddamg_ctx* ctx, int level, int nrhs, const void* in, void* out);
/* iters SAP iterations of an intermediate coarse level (the coarse-level
 * smoother of the cycle; SAP blocks coarse_sap_block, coarse_mr_steps MR steps
 * on each block operator) on nrhs (1..16) systems D_c x_k = b_k at once, with
 * the block operator read once per MR step for all of them (matrix cores for
 * FP16/BF16 storage).  b, x: host complex128 [nrhs][len_l], x updated in
 * place. */
int ddamg_coarse_sap_multi(ddamg_ctx* ctx, int level, int nrhs, const void* b, void* x, int iters);
/* Coarse solves of nrhs right-hand sides in lock step (one operator launch
 * per step for all of them; each keeps its own Krylov space and stopping
 * test).  Same solver and layout as ddamg_coarse_solve; 1 <= nrhs <= 16. */
int ddamg_coarse_solve_multi(ddamg_ctx* ctx, int level, int nrhs, const void* b, void* x);

/* Device memory of a context: the library keeps the device memory it has
 * taken (slabs of its own pool) for the context's later calls, because
 * re-allocating freed device memory is slow on this device.  This call gives
 * back every slab with nothing in use (the workspaces of finished setups and
 * solves), keeping the operator, the hierarchy and every live buffer; held
 * (may be NULL) receives the bytes the context still holds.  Later calls take
 * memory again as they need it. */
int ddamg_release_memory(ddamg_ctx* ctx, double* held);

/* ---- measurement ---- */
/* Run napply applications of D(mu) on device-resident fields in the
 * library's own layout (inputs already in HBM), on the context stream;
 * returns immediately after enqueueing. */
int ddamg_bench_dirac(ddamg_ctx* ctx, int precision, int napply);
/* napply applications of the level-l coarse operator to nrhs device-resident
 * fields at once (which = 0: full stencil; 1: odd-even reduced operator of the
 * coarsest level), precision of the last setup; enqueued on the context stream. */
int ddamg_bench_coarse(ddamg_ctx* ctx, int level, int nrhs, int napply, int which);
/* Per-kernel timing with HIP events on the context stream.  kind: 0 = FP64
 * D(mu) (outer operator), 1 = fine SAP colour sweep, 2 = coarse operator
 * apply (intermediate levels, residuals included), 3 = restriction and
 * prolongation, 4 = reduced-precision fine D(mu), 5 = coarsest odd-even Schur
 * apply.  enable = 1 resets and starts recording, 0 stops; query returns the
 * launch count and total milliseconds so far (synchronises the stream). */
int ddamg_timing(ddamg_ctx* ctx, int enable);
int ddamg_timing_query(ddamg_ctx* ctx, int kind, long* count, double* ms);
/* Algorithmic bytes of the launches timed so far of a kind, each datum moved
 * once per launch: kind 0, 1536 bytes per site (spinor in and out, links,
 * clover in FP64); kind 1, per site of the swept colour the links (36
 * entries of the storage format), the clover term and the odd-site inverse
 * factors (108 reals on average) once, and per field b, x in, x out and the
 * other colour's x (48 complex); other kinds report 0.  bytes / (ms 1e-3) is
 * the achieved rate. */
int ddamg_timing_bytes(ddamg_ctx* ctx, int kind, double* bytes);
/* Real floating-point operations of the launches timed so far of a kind (a
 * complex multiply-add counts 8): kind 1, per site of the swept colour and
 * field 4932 + 2604 n_MR (the residual, the odd-site solves, the first rho,
 * n_MR MR steps on the even-site Schur complement and the odd-site
 * correction; 15348 at n_MR = 4); other kinds report 0. */
int ddamg_timing_flops(ddamg_ctx* ctx, int kind, double* flops);

/* ---- learned setup (not a method of the paper: it replaces the random start
 * of the adaptive setup; the plain setup stays the fallback) ----
 * Network: nlayers gauge-covariant parallel-transport layers with nchan
 * complex channels (4, 8, 12, 16 or 24); layer l computes
 *   z_c(x) = sum_{d=0..8} sum_{c'} W_l[d][c][c'] (T_d x_{c'})(x)
 * with T_0 = 1, T_{1+mu} x(x) = U_mu(x) x(x+mu), T_{5+mu} x(x) = U_mu(x-mu)^dag x(x-mu)
 * (mu = T,Z,Y,X) and W a 4x4 spin matrix; all layers but the last are gated,
 * y_c = z_c sigmoid(a_c |z_c|^2 + b_c).  Arithmetic in FP32.
 * Parameters (FP64 host vector): W_0 .. W_{L-1}, each [9][C][C][4][4] complex
 * with real/imag interleaved, then a_0, b_0, a_1, b_1, ... ([C] each).
 * Fields: nchan spinor fields (spinor layout above, contiguous). */
int ddamg_net_create(ddamg_ctx* ctx, int nlayers, int nchan);
long ddamg_net_num_params(ddamg_ctx* ctx);
int ddamg_net_set_params(ddamg_ctx* ctx, const double* params, long n);
int ddamg_net_get_params(ddamg_ctx* ctx, double* params, long n);
/* out = network(noise) on the context's gauge field */
int ddamg_net_forward(ddamg_ctx* ctx, const void* noise, void* out, int on_device);
/* subspace loss of network(noise) against orthonormal targets (the block
 * orthonormalised test vectors of a plain setup):
 *   L = sum_{aggregate halves} |(I - Pi_Y) Q|_F^2 / sum |Q|_F^2,
 * and its gradient dL/dRe + i dL/dIm per parameter (grads may be NULL). */
int ddamg_net_loss_grad(ddamg_ctx* ctx, const void* noise, const void* target, int on_device, double* loss,
                        double* grads);
/* one Adam step (beta 0.9/0.999, eps 1e-8) on that loss; returns the loss
 * before the update. */
int ddamg_net_train_step(ddamg_ctx* ctx, const void* noise, const void* target, int on_device, double lr,
                         double* loss);

#ifdef __cplusplus
}
#endif
#endif /* DDAMG_H */
