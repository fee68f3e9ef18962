"""Multigrid hierarchy, V-cycle (Eq. 1), adaptive setup and the outer solve.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper, Sec. 1, Eq. (1): every step of the flexible outer Krylov solver applies
the preconditioner whose error propagation is
    (I - M D)^k (I - P D_c^{-1} P^dag D) (I - M D)^j,
M the SAP smoother, j / k pre- / post-smoothing iterations.  The test vectors
that span P come from an adaptive setup phase (Sec. 1; 3 or 5 setup
iterations, Fig. 1 caption and Listing 1); Sec. 2: three levels with 4^4 then
2^4 aggregates is the standard hierarchy; Sec. 1: the coarsest level carries
the raised twist delta * mu.

Readings taken where the paper is silent (all tunable, all recorded):
  * V-cycle at level l applied to v (initial guess 0):
        x = j SAP iterations on D x = v
        x += P (coarse solve of D_c e = P^dag (v - D x))
        x = k further SAP iterations on D x = v
    coarse solve = odd-even GMRES(m_c) on the coarsest level (relative
    tolerance coarse_tol, at most coarse_max_iter iterations), otherwise
    FGMRES(inter_restart) preconditioned by the next level's V-cycle
    (tolerance inter_tol, at most inter_max_iter iterations);
  * fine smoother: SAP with odd-even MR block solves; coarse smoother: SAP
    with plain MR block solves (coarse_sap_block blocks);
  * adaptive setup:
      initial phase: v_i = given random vectors, each smoothed by n_init SAP
      iterations on D v = 0; orthonormalise -> P; assemble D_c; recurse;
      iterated phase (setup_iters times): v_i <- V-cycle(v_i) for every i,
      normalised; rebuild P and D_c; on a 3-level hierarchy then
      D_c,2 = P_2^dag D_c,1 P_2 with the current P_2, followed by
      coarse_setup_iters level-1 iterations (w_j <- V-cycle_1(w_j), rebuild).
  * the setup uses +mu; D(-mu) reuses it with every twist negated (Sec. 1).
  * different twists on even and odd sites (Sec. 2, needed by the Hasenbusch
    terms of Sec. 3.1): the fine level applies each site's own twist; the
    coarse operators are the Galerkin products of the full operator, with the
    mean of the two twists as their i mu_c Gamma5,c term (delta times the
    mean on the coarsest level) and the rest, i (mu(x) - mean) Gamma5 summed
    over each aggregate, in their site blocks.  The paper defines delta for a
    single twist only; reading: delta raises the mean, the parity rest enters
    unscaled.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

from . import aggregation as agg
from . import coarse, krylov, sap
from .stencil import FineLevel, Stencil, wilson_stencil


@dataclass
class Params:
    levels: int = 2
    blocks: list = field(default_factory=lambda: [(4, 4, 4, 4), (2, 2, 2, 2)])
    nvec: list = field(default_factory=lambda: [24, 32])
    sap_block: tuple = None          # fine SAP block (defaults to blocks[0])
    coarse_sap_block: tuple = (2, 2, 2, 2)
    sap_pre: int = 0
    sap_post: int = 3
    mr_steps: int = 4
    coarse_sap_post: int = 2
    coarse_mr_steps: int = 3
    delta: float = 1.0
    init_sap_iters: int = 3
    setup_iters: int = 3
    coarse_setup_iters: int = 3
    restart: int = 10
    inter_restart: int = 10
    inter_tol: float = 1e-1
    inter_max_iter: int = 10
    coarse_restart: int = 30
    coarse_tol: float = 1e-1
    coarse_max_iter: int = 300
    fixed: bool = False              # fixed iteration counts inside the preconditioner

    def sap_blk(self):
        return tuple(self.sap_block) if self.sap_block is not None else tuple(self.blocks[0])


class Level:
    def __init__(self, op, n):
        self.op = op          # FineLevel or Stencil (apply/site/site_inv/hop)
        self.n = n
        self.Q = None         # orthonormalised test vectors (interpolation to l+1)
        self.V = None         # raw test vectors
        self.bsize = None


class Hierarchy:
    def __init__(self, fine_op, params: Params):
        self.p = params
        self.fine_op = fine_op
        self.levels = [Level(FineLevel(fine_op), 12)]
        self.stats = dict(coarse_iters=[0] * params.levels, vcycles=0)

    @property
    def nlev(self):
        return len(self.levels)

    def mu_level(self, l, mu):
        """Twist on level l >= 1: delta*mu on the coarsest, mu elsewhere."""
        return self.p.delta * mu if l == self.p.levels - 1 else mu

    # ------------------------------------------------------------------
    def smooth(self, l, b, x, iters):
        if iters <= 0:
            return x
        L = self.levels[l]
        if l == 0:
            return sap.sap(L.op, b, x, self.p.sap_blk(), self.p.mr_steps, iters, schur=True)
        return sap.sap(L.op, b, x, self.p.coarse_sap_block, self.p.coarse_mr_steps, iters, schur=False)

    def coarse_solve(self, l, rc):
        """Approximate solve on level l (>= 1)."""
        p = self.p
        st = self.levels[l].op
        if l == self.nlev - 1:
            oe = coarse.OddEven(st)
            rhs = oe.rhs(rc)
            xe, info = krylov.gmres(oe.schur, rhs, tol=p.coarse_tol, restart=p.coarse_restart,
                                    max_iter=p.coarse_max_iter, fixed=p.fixed)
            self.stats["coarse_iters"][l] += info["iters"]
            return oe.reconstruct(xe, rc)
        x, info = krylov.fgmres(st.apply, rc, M=lambda v: self.vcycle(l, v), tol=p.inter_tol,
                                restart=p.inter_restart, max_iter=p.inter_max_iter, fixed=p.fixed)
        self.stats["coarse_iters"][l] += info["iters"]
        return x

    def vcycle(self, l, v):
        """The preconditioner of Eq. (1) on level l applied to v (x0 = 0)."""
        L = self.levels[l]
        pre = self.p.sap_pre if l == 0 else 0
        post = self.p.sap_post if l == 0 else self.p.coarse_sap_post
        if l == 0:
            self.stats["vcycles"] += 1
        x = np.zeros_like(v)
        x = self.smooth(l, v, x, pre)
        r = v - L.op.apply(x) if pre > 0 else v
        rc = agg.restrict(L.Q, r, L.bsize)
        ec = self.coarse_solve(l + 1, rc)
        x = x + agg.prolong(L.Q, ec, L.bsize)
        x = self.smooth(l, v, x, post)
        return x

    # ------------------------------------------------------------------
    def _build_next(self, l, mu):
        """(Re)build P_l from the raw vectors of level l and D_c on level l+1."""
        L = self.levels[l]
        L.Q = agg.orthonormalise(L.V, L.bsize)
        st = wilson_stencil(self.fine_op) if l == 0 else L.op
        Dc = coarse.assemble(st, L.Q, L.bsize, self.mu_level(l + 1, mu))
        if len(self.levels) > l + 1:
            self.levels[l + 1].op = Dc
        else:
            self.levels.append(Level(Dc, Dc.n))

    def _rebuild_from_Q(self, l, mu):
        """D_c on level l+1 from the current (unchanged) P_l."""
        L = self.levels[l]
        Dc = coarse.assemble(L.op, L.Q, L.bsize, self.mu_level(l + 1, mu))
        self.levels[l + 1].op = Dc

    def setup(self, init_vectors):
        """Adaptive setup.  init_vectors[l] = random starting vectors for the
        interpolation from level l to l+1 ([Nv_l, level-l field shape])."""
        p = self.p
        mu = self.fine_op.mean_twist()  # coarse levels carry the mean twist
        zero = None
        # initial phase, level by level
        for l in range(p.levels - 1):
            L = self.levels[l]
            L.bsize = tuple(p.blocks[l])
            V = np.array(init_vectors[l], dtype=np.complex128, copy=True)
            zero = np.zeros_like(V[0])
            sblk = p.sap_blk() if l == 0 else p.coarse_sap_block
            nmr = p.mr_steps if l == 0 else p.coarse_mr_steps
            for i in range(V.shape[0]):
                V[i] = sap.sap(L.op, zero, V[i], sblk, nmr, p.init_sap_iters, schur=(l == 0))
            L.V = V
            self._build_next(l, mu)
        # iterated phase
        for _ in range(p.setup_iters):
            self._iterate_level(0, mu)
            if p.levels == 3:
                self._rebuild_from_Q(1, mu)
                for _ in range(p.coarse_setup_iters):
                    self._iterate_level(1, mu)
        return self

    def _iterate_level(self, l, mu):
        L = self.levels[l]
        for i in range(L.V.shape[0]):
            w = self.vcycle(l, L.V[i])
            L.V[i] = w / np.sqrt(np.vdot(w, w).real)
        self._build_next(l, mu)

    def set_test_vectors(self, vecs, mu=None):
        """Build the hierarchy directly from given test vectors (no setup
        iterations): vecs[l] are the raw vectors of level l."""
        p = self.p
        mu = self.fine_op.mean_twist() if mu is None else mu
        for l in range(p.levels - 1):
            L = self.levels[l]
            L.bsize = tuple(p.blocks[l])
            L.V = np.array(vecs[l], dtype=np.complex128, copy=True)
            self._build_next(l, mu)
        return self

    def with_mu(self, mu):
        """Same P on every level, every twist recomputed from mu (Sec. 1:
        one setup serves D(+mu) and D(-mu))."""
        from .dirac import WilsonClover  # noqa: F401
        h = Hierarchy.__new__(Hierarchy)
        h.p = self.p
        fo = self.fine_op
        if getattr(fo, "mu_odd", None) is not None:
            raise NotImplementedError("different twists on the two parities: build a hierarchy per operator")
        new_fine = object.__new__(type(fo))
        new_fine.__dict__.update(fo.__dict__)
        new_fine.mu = mu
        h.fine_op = new_fine
        h.levels = []
        for l, L in enumerate(self.levels):
            if l == 0:
                NL = Level(FineLevel(new_fine), 12)
            else:
                NL = Level(L.op.with_mu(self.mu_level(l, mu)), L.n)
            NL.Q, NL.V, NL.bsize = L.Q, L.V, L.bsize
            h.levels.append(NL)
        h.stats = dict(coarse_iters=[0] * self.p.levels, vcycles=0)
        return h

    # ------------------------------------------------------------------
    def solve(self, b, tol=1e-10, max_iter=500):
        """Outer FGMRES(restart) on D(mu) x = b preconditioned by the V-cycle."""
        L0 = self.levels[0]
        return krylov.fgmres(L0.op.apply, b, M=lambda v: self.vcycle(0, v), tol=tol,
                             restart=self.p.restart, max_iter=max_iter)
