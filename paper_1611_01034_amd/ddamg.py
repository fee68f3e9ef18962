"""ctypes binding of libddamg.so (declared in include/ddamg.h).

Argument marshalling only: every numerical step runs in the library's HIP
kernels.  Arrays may be numpy complex128 arrays (host) or torch complex128
CUDA tensors (device, used on the context stream).  There is no CPU fallback:
if the shared library is missing this module raises at import.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libddamg.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "ddamg.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
# torch ships its own HIP runtime; load it first so that the library binds to
# the same runtime (one HIP context per process, shared streams and pointers)
try:
    import torch  # noqa: F401
except ImportError:  # pragma: no cover
    pass
_lib = ctypes.CDLL(LIB_PATH)

OK, NOT_CONVERGED, INVALID_ARG, BAD_STATE, HIP_ERROR, OUT_OF_MEMORY, NUMERICAL = 0, 1, -1, -2, -3, -4, -5
FP64, FP32, FP16, BF16 = 0, 1, 2, 3
PRECISIONS = {"fp64": FP64, "fp32": FP32, "fp16": FP16, "bf16": BF16}


class Params(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int),
        ("block", (ctypes.c_int * 4) * 3),
        ("nvec", ctypes.c_int * 3),
        ("coarse_sap_block", ctypes.c_int * 4),
        ("sap_pre", ctypes.c_int),
        ("sap_post", ctypes.c_int),
        ("mr_steps", ctypes.c_int),
        ("coarse_sap_post", ctypes.c_int),
        ("coarse_mr_steps", ctypes.c_int),
        ("init_sap_iters", ctypes.c_int),
        ("setup_iters", ctypes.c_int),
        ("coarse_setup_iters", ctypes.c_int),
        ("coarse_mu_factor", ctypes.c_double),
        ("restart", ctypes.c_int),
        ("max_iter", ctypes.c_int),
        ("inter_restart", ctypes.c_int),
        ("inter_max_iter", ctypes.c_int),
        ("inter_tol", ctypes.c_double),
        ("coarse_restart", ctypes.c_int),
        ("coarse_max_iter", ctypes.c_int),
        ("coarse_tol", ctypes.c_double),
        ("precision", ctypes.c_int),
        ("fixed_iters", ctypes.c_int),
        ("batch", ctypes.c_int),
        ("rhs_batch", ctypes.c_int),
        ("keep_test_vectors", ctypes.c_int),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int),
        ("converged", ctypes.c_int),
        ("resid", ctypes.c_double),
        ("coarse_iters", ctypes.c_long * 4),
        ("vcycles", ctypes.c_long),
        ("seconds", ctypes.c_double),
        ("nrhs", ctypes.c_int),
        ("iters_min", ctypes.c_int),
        ("iters_max", ctypes.c_int),
    ]

    def as_dict(self):
        return dict(iters=self.iters, converged=bool(self.converged), resid=self.resid,
                    coarse_iters=list(self.coarse_iters), vcycles=self.vcycles, seconds=self.seconds,
                    nrhs=self.nrhs, iters_min=self.iters_min, iters_max=self.iters_max)


_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double
_PROGRESS_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int)
_SIGS = {
    "ddamg_default_params": (None, [ctypes.POINTER(Params)]),
    "ddamg_create": (_i, [ctypes.POINTER(_i), ctypes.POINTER(_i), _d, _d, _d, _vp, ctypes.POINTER(_vp)]),
    "ddamg_destroy": (None, [_vp]),
    "ddamg_last_error": (ctypes.c_char_p, [_vp]),
    "ddamg_set_gauge": (_i, [_vp, _vp, _i]),
    "ddamg_update_gauge": (_i, [_vp, _vp, _i, ctypes.POINTER(Params)]),
    "ddamg_set_boundary_phases": (_i, [_vp, ctypes.POINTER(_d)]),
    "ddamg_set_clover": (_i, [_vp, _vp, _i]),
    "ddamg_get_clover": (_i, [_vp, _vp]),
    "ddamg_set_mu": (_i, [_vp, _d]),
    "ddamg_set_mu_eo": (_i, [_vp, _d, _d]),
    "ddamg_setup": (_i, [_vp, ctypes.POINTER(Params), ctypes.POINTER(_vp), _i]),
    "ddamg_set_test_vectors": (_i, [_vp, ctypes.POINTER(Params), ctypes.POINTER(_vp), _i]),
    "ddamg_setup_prec": (_i, [_vp, ctypes.POINTER(Params), ctypes.POINTER(_vp), _i, _i]),
    "ddamg_solve": (_i, [_vp, _vp, _vp, _i, _d, ctypes.POINTER(Stats), _i]),
    "ddamg_solve_odd_shifted": (_i, [_vp, _vp, _vp, _d, _d, ctypes.POINTER(Stats), _i]),
    "ddamg_apply_dirac": (_i, [_vp, _vp, _vp, _i, _i, _i]),
    "ddamg_apply_dirac_multi": (_i, [_vp, _i, _vp, _vp, _i, _i, _i]),
    "ddamg_apply_dirac_noalloc": (_i, [_vp, _vp, _vp, _i]),
    "ddamg_sap": (_i, [_vp, _vp, _vp, _i, _i, _i, _i]),
    "ddamg_sap_multi": (_i, [_vp, _i, _vp, _vp, _i, _i, _i, _i]),
    "ddamg_apply_coarse_schur_multi": (_i, [_vp, _i, _i, _vp, _vp]),
    "ddamg_coarse_sap_multi": (_i, [_vp, _i, _i, _vp, _vp, _i]),
    "ddamg_level_info": (_i, [_vp, _i, ctypes.POINTER(_i), ctypes.POINTER(_i)]),
    "ddamg_get_interpolation": (_i, [_vp, _i, _vp]),
    "ddamg_restrict": (_i, [_vp, _i, _vp, _vp]),
    "ddamg_prolong": (_i, [_vp, _i, _vp, _vp]),
    "ddamg_restrict_multi": (_i, [_vp, _i, _i, _vp, _vp]),
    "ddamg_prolong_multi": (_i, [_vp, _i, _i, _vp, _vp]),
    "ddamg_get_coarse_op": (_i, [_vp, _i, _vp, _vp]),
    "ddamg_apply_coarse": (_i, [_vp, _i, _vp, _vp]),
    "ddamg_coarse_sap": (_i, [_vp, _i, _vp, _vp, _i]),
    "ddamg_coarse_solve": (_i, [_vp, _i, _vp, _vp]),
    "ddamg_vcycle": (_i, [_vp, _vp, _vp]),
    "ddamg_setup_learned": (_i, [_vp, ctypes.POINTER(Params), _vp, _i, _i, _vp]),
    "ddamg_apply_coarse_multi": (_i, [_vp, _i, _i, _vp, _vp]),
    "ddamg_coarse_solve_multi": (_i, [_vp, _i, _i, _vp, _vp]),
    "ddamg_bench_coarse": (_i, [_vp, _i, _i, _i, _i]),
    "ddamg_bench_dirac": (_i, [_vp, _i, _i]),
    "ddamg_timing": (_i, [_vp, _i]),
    "ddamg_timing_query": (_i, [_vp, _i, ctypes.POINTER(ctypes.c_long), ctypes.POINTER(_d)]),
    "ddamg_timing_bytes": (_i, [_vp, _i, ctypes.POINTER(_d)]),
    "ddamg_release_memory": (_i, [_vp, ctypes.POINTER(_d)]),
    "ddamg_set_progress": (_i, [_vp, _vp, _vp]),
    "ddamg_timing_flops": (_i, [_vp, _i, ctypes.POINTER(_d)]),
    "ddamg_error_reduction": (_i, [_vp, _vp, _i, _i, ctypes.POINTER(_d)]),
    "ddamg_net_create": (_i, [_vp, _i, _i]),
    "ddamg_net_num_params": (ctypes.c_long, [_vp]),
    "ddamg_net_set_params": (_i, [_vp, ctypes.POINTER(_d), ctypes.c_long]),
    "ddamg_net_get_params": (_i, [_vp, ctypes.POINTER(_d), ctypes.c_long]),
    "ddamg_net_forward": (_i, [_vp, _vp, _vp, _i]),
    "ddamg_net_loss_grad": (_i, [_vp, _vp, _vp, _i, ctypes.POINTER(_d), ctypes.POINTER(_d)]),
    "ddamg_net_train_step": (_i, [_vp, _vp, _vp, _i, _d, ctypes.POINTER(_d)]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def pack_net(W, a, b):
    """Flat FP64 parameter vector of the network: every layer's W [9,C,C,4,4]
    complex (real/imag interleaved), then (a_l, b_l) of the gated layers."""
    parts = [np.asarray(w, dtype=np.complex128).reshape(-1).view(np.float64) for w in W]
    for al, bl in zip(a, b):
        parts += [np.asarray(al, dtype=np.float64), np.asarray(bl, dtype=np.float64)]
    return np.ascontiguousarray(np.concatenate(parts))


def unpack_net(v, C, L):
    nW = 9 * C * C * 16
    W = [v[2 * l * nW: 2 * (l + 1) * nW].view(np.complex128).reshape(9, C, C, 4, 4) for l in range(L)]
    off = 2 * L * nW
    a, b = [], []
    for l in range(L - 1):
        a.append(v[off: off + C])
        b.append(v[off + C: off + 2 * C])
        off += 2 * C
    return W, a, b


def exported_symbols():
    return sorted(_SIGS)


class DDAMGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"status {status}: {msg}")
        self.status = status


def default_params(**kw) -> Params:
    p = Params()
    _lib.ddamg_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if k == "block":
            for l, b in enumerate(v):
                for d in range(4):
                    p.block[l][d] = int(b[d])
        elif k in ("nvec", "coarse_sap_block"):
            arr = getattr(p, k)
            for i, x in enumerate(v):
                arr[i] = int(x)
        elif k == "precision":
            setattr(p, k, PRECISIONS[v] if isinstance(v, str) else int(v))
        else:
            setattr(p, k, v)
    return p


def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _ptr(a):
    """(pointer, on_device) of a numpy array or a torch tensor."""
    if _is_torch(a):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return ctypes.c_void_p(a.data_ptr()), int(a.is_cuda)
    if not (isinstance(a, np.ndarray) and a.flags["C_CONTIGUOUS"]):
        raise ValueError("array must be C-contiguous")
    return ctypes.c_void_p(a.ctypes.data), 0


def _c128(a):
    if _is_torch(a):
        import torch
        if a.dtype != torch.complex128:
            raise TypeError("tensor must be complex128")
        return a.contiguous()
    return np.ascontiguousarray(a, dtype=np.complex128)


class DDAMG:
    """One lattice, one gauge field, one multigrid hierarchy.

    dims = (T, Z, Y, X); block = fine SAP block and first aggregate.
    stream: a hipStream_t as int (torch.cuda.current_stream().cuda_stream),
    or None for the null stream."""

    def __init__(self, dims, block, kappa, csw, mu, stream=None):
        self.dims = tuple(int(d) for d in dims)
        self.block = tuple(int(b) for b in block)
        self.V = int(np.prod(self.dims))
        d = (ctypes.c_int * 4)(*self.dims)
        b = (ctypes.c_int * 4)(*self.block)
        h = ctypes.c_void_p()
        st = _lib.ddamg_create(d, b, float(kappa), float(csw), float(mu),
                               ctypes.c_void_p(stream) if stream else None, ctypes.byref(h))
        if st != OK:
            raise DDAMGError(st, "ddamg_create failed")
        self._h = h
        self.params = None

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.ddamg_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, st, allow=(OK,)):
        if st not in allow:
            raise DDAMGError(st, _lib.ddamg_last_error(self._h).decode())
        return st

    # ---- setup ------------------------------------------------------------
    def set_gauge(self, U):
        U = _c128(U)
        p, dev = _ptr(U)
        self._check(_lib.ddamg_set_gauge(self._h, p, dev))
        self._keep = U

    def set_boundary_phases(self, theta):
        """Twisted boundary conditions psi(x + L_mu) = exp(i theta_mu) psi(x)."""
        th = (_d * 4)(*[float(t) for t in theta])
        self._check(_lib.ddamg_set_boundary_phases(self._h, th))

    def update_gauge(self, U, params: Params):
        """New gauge field, keeping the hierarchy's interpolation as the test
        vectors of a refreshed setup (ddamg_update_gauge)."""
        U = _c128(U)
        p, dev = _ptr(U)
        self._check(_lib.ddamg_update_gauge(self._h, p, dev, ctypes.byref(params)))
        self._keep = U
        self.params = params

    def set_clover(self, A=None):
        if A is None:
            self._check(_lib.ddamg_set_clover(self._h, None, 0))
            return
        A = _c128(A)
        p, dev = _ptr(A)
        self._check(_lib.ddamg_set_clover(self._h, p, dev))

    def get_clover(self):
        out = np.empty(self.dims + (2, 6, 6), dtype=np.complex128)
        self._check(_lib.ddamg_get_clover(self._h, _ptr(out)[0]))
        return out

    def set_mu(self, mu):
        self._check(_lib.ddamg_set_mu(self._h, float(mu)))

    def set_mu_eo(self, mu_even, mu_odd):
        """Twisted mass mu_even on the even and mu_odd on the odd sites."""
        self._check(_lib.ddamg_set_mu_eo(self._h, float(mu_even), float(mu_odd)))

    def _vec_ptrs(self, vecs):
        arrs = [_c128(v) for v in vecs]
        ptrs = (ctypes.c_void_p * 3)()
        dev = 0
        for i, a in enumerate(arrs):
            p, dev = _ptr(a)
            ptrs[i] = p
        return arrs, ptrs, dev

    def setup(self, params: Params, init_vectors):
        """Adaptive setup from random initial vectors per level; the fine
        level's may be complex64 (numpy or torch), which is passed as it is."""
        v0 = init_vectors[0]
        c64 = (v0.dtype == np.complex64) if not _is_torch(v0) else (str(v0.dtype) == "torch.complex64")
        if not c64:
            arrs, ptrs, dev = self._vec_ptrs(init_vectors)
            self._check(_lib.ddamg_setup(self._h, ctypes.byref(params), ptrs, dev))
            self.params = params
            return
        v0 = v0.contiguous() if _is_torch(v0) else np.ascontiguousarray(v0)
        rest = [_c128(v) for v in init_vectors[1:]]
        ptrs = (ctypes.c_void_p * 3)()
        ptrs[0], dev = _ptr(v0)
        for i, a in enumerate(rest):
            ptrs[i + 1], dev_i = _ptr(a)
            if dev_i != dev:
                raise ValueError("initial vectors must all be on the host or all on the device")
        self._check(_lib.ddamg_setup_prec(self._h, ctypes.byref(params), ptrs, FP32, dev))
        self.params = params

    def setup_learned(self, params: Params, noise, coarse_init=None):
        """Adaptive setup from the network's output on `noise` (C fields,
        complex64 or complex128, numpy or torch); the network must be set."""
        if _is_torch(noise):
            import torch
            if noise.dtype not in (torch.complex64, torch.complex128):
                raise TypeError("noise must be complex64 or complex128")
            prec = FP32 if noise.dtype == torch.complex64 else FP64
            noise = noise.contiguous()
        else:
            noise = np.asarray(noise)
            prec = FP32 if noise.dtype == np.complex64 else FP64
            noise = np.ascontiguousarray(noise, dtype=np.complex64 if prec == FP32 else np.complex128)
        pn, dev = _ptr(noise)
        pc = ctypes.c_void_p(None)
        keep = None
        if coarse_init is not None:
            keep = _c128(coarse_init)
            pc, dev_c = _ptr(keep)
            if dev_c != dev:
                raise ValueError("noise and coarse_init must both be on the host or both on the device")
        self._check(_lib.ddamg_setup_learned(self._h, ctypes.byref(params), pn, prec, dev, pc))
        self.params = params

    def set_test_vectors(self, params: Params, vectors):
        arrs, ptrs, dev = self._vec_ptrs(vectors)
        self._check(_lib.ddamg_set_test_vectors(self._h, ctypes.byref(params), ptrs, dev))
        self.params = params

    # ---- solve ------------------------------------------------------------
    def solve(self, b, tol=1e-10, x=None, allow_not_converged=False):
        b = _c128(b)
        nrhs = 1 if b.ndim == 6 else b.shape[0]
        if x is None:
            if _is_torch(b):
                import torch
                x = torch.empty_like(b)
            else:
                x = np.empty_like(b)
        pb, dev = _ptr(b)
        px, _ = _ptr(x)
        st = Stats()
        allow = (OK, NOT_CONVERGED) if allow_not_converged else (OK,)
        self._check(_lib.ddamg_solve(self._h, pb, px, nrhs, float(tol), ctypes.byref(st), dev), allow)
        return x, st.as_dict()

    def solve_odd_shifted(self, b, rho, tol=1e-10, x=None, allow_not_converged=False):
        """Full solution of D(mu; rho) x = (0, b_odd) (ddamg_solve_odd_shifted):
        its odd sites solve (Dhat(mu) + i rho Gamma5hat) x_o = b_o."""
        b = _c128(b)
        if x is None:
            if _is_torch(b):
                import torch
                x = torch.empty_like(b)
            else:
                x = np.empty_like(b)
        pb, dev = _ptr(b)
        px, _ = _ptr(x)
        st = Stats()
        allow = (OK, NOT_CONVERGED) if allow_not_converged else (OK,)
        self._check(_lib.ddamg_solve_odd_shifted(self._h, pb, px, float(rho), float(tol), ctypes.byref(st), dev),
                    allow)
        return x, st.as_dict()

    # ---- single operators ---------------------------------------------------
    def apply_dirac(self, psi, sign=+1, precision="fp64"):
        psi = _c128(psi)
        out = np.empty_like(psi) if not _is_torch(psi) else psi.new_empty(psi.shape)
        pi, dev = _ptr(psi)
        self._check(_lib.ddamg_apply_dirac(self._h, pi, _ptr(out)[0], int(sign), PRECISIONS[precision], dev))
        return out

    def apply_dirac_multi(self, psis, sign=+1, precision="fp64"):
        """D(sign*mu) on K fields [K, T, Z, Y, X, 4, 3] (host array or
        complex128 CUDA tensor) in one launch."""
        psis = _c128(psis)
        out = np.empty_like(psis) if not _is_torch(psis) else psis.new_empty(psis.shape)
        pi, dev = _ptr(psis)
        self._check(_lib.ddamg_apply_dirac_multi(self._h, int(psis.shape[0]), pi, _ptr(out)[0], int(sign),
                                                 PRECISIONS[precision], dev))
        return out

    def apply_dirac_noalloc(self, psi, out, sign=+1):
        """D(sign*mu) psi into out, both complex128 CUDA tensors of the
        spinor shape, without any allocation by the library; enqueued on the
        context stream (synchronise before reading out)."""
        if not (_is_torch(psi) and _is_torch(out)) or not (psi.is_cuda and out.is_cuda):
            raise TypeError("apply_dirac_noalloc takes CUDA tensors")
        if psi.dtype != out.dtype or str(psi.dtype) != "torch.complex128" or psi.shape != out.shape:
            raise TypeError("psi and out must be complex128 tensors of one shape")
        if not (psi.is_contiguous() and out.is_contiguous()):
            raise ValueError("psi and out must be contiguous")
        self._check(_lib.ddamg_apply_dirac_noalloc(self._h, psi.data_ptr(), out.data_ptr(), int(sign)))
        return out

    def sap(self, b, x0, iters, mr_steps=4, precision="fp64"):
        b = _c128(b)
        x = np.array(x0, dtype=np.complex128, copy=True)
        self._check(_lib.ddamg_sap(self._h, _ptr(b)[0], _ptr(x)[0], int(iters), int(mr_steps),
                                   PRECISIONS[precision], 0))
        return x

    def sap_multi(self, bs, xs0, iters, mr_steps=4, precision="fp64"):
        """bs, xs0: [K, T, Z, Y, X, 4, 3] (host); K fields through one launch per colour."""
        bs = _c128(bs)
        xs = np.array(xs0, dtype=np.complex128, copy=True)
        self._check(_lib.ddamg_sap_multi(self._h, int(bs.shape[0]), _ptr(bs)[0], _ptr(xs)[0], int(iters),
                                         int(mr_steps), PRECISIONS[precision], 0))
        return xs

    def level_info(self, level):
        d = (ctypes.c_int * 4)()
        n = ctypes.c_int()
        self._check(_lib.ddamg_level_info(self._h, int(level), d, ctypes.byref(n)))
        return tuple(d), n.value

    def _level_shape(self, level):
        d, n = self.level_info(level)
        return tuple(d) + ((4, 3) if level == 0 else (n,))

    def get_interpolation(self, level):
        nv = self.params.nvec[level]
        out = np.empty((nv,) + self._level_shape(level), dtype=np.complex128)
        self._check(_lib.ddamg_get_interpolation(self._h, int(level), _ptr(out)[0]))
        return out

    def restrict(self, level, r):
        r = _c128(r)
        out = np.empty(self._level_shape(level + 1), dtype=np.complex128)
        self._check(_lib.ddamg_restrict(self._h, int(level), _ptr(r)[0], _ptr(out)[0]))
        return out

    def prolong(self, level, e):
        e = _c128(e)
        out = np.empty(self._level_shape(level), dtype=np.complex128)
        self._check(_lib.ddamg_prolong(self._h, int(level), _ptr(e)[0], _ptr(out)[0]))
        return out

    def restrict_multi(self, level, rs):
        """P^dag of K level-`level` fields [K, ...] through the K-column kernel."""
        rs = _c128(rs)
        out = np.empty((rs.shape[0],) + self._level_shape(level + 1), dtype=np.complex128)
        self._check(_lib.ddamg_restrict_multi(self._h, int(level), int(rs.shape[0]), _ptr(rs)[0], _ptr(out)[0]))
        return out

    def prolong_multi(self, level, es):
        """P of K level-(level+1) fields [K, ...] through the K-column kernel."""
        es = _c128(es)
        out = np.empty((es.shape[0],) + self._level_shape(level), dtype=np.complex128)
        self._check(_lib.ddamg_prolong_multi(self._h, int(level), int(es.shape[0]), _ptr(es)[0], _ptr(out)[0]))
        return out

    def get_coarse_op(self, level):
        d, n = self.level_info(level)
        S = np.empty(tuple(d) + (n, n), dtype=np.complex128)
        F = np.empty((4,) + tuple(d) + (n, n), dtype=np.complex128)
        self._check(_lib.ddamg_get_coarse_op(self._h, int(level), _ptr(S)[0], _ptr(F)[0]))
        return S, F

    def apply_coarse(self, level, y):
        y = _c128(y)
        out = np.empty_like(y)
        self._check(_lib.ddamg_apply_coarse(self._h, int(level), _ptr(y)[0], _ptr(out)[0]))
        return out

    def coarse_sap(self, level, b, x0, iters):
        b = _c128(b)
        x = np.array(x0, dtype=np.complex128, copy=True)
        self._check(_lib.ddamg_coarse_sap(self._h, int(level), _ptr(b)[0], _ptr(x)[0], int(iters)))
        return x

    def coarse_solve(self, level, b):
        b = _c128(b)
        x = np.empty_like(b)
        self._check(_lib.ddamg_coarse_solve(self._h, int(level), _ptr(b)[0], _ptr(x)[0]))
        return x

    def apply_coarse_multi(self, level, ys):
        """ys: [nrhs, ...] fields of level `level` (same layout as apply_coarse)."""
        ys = _c128(ys)
        out = np.empty_like(ys)
        self._check(_lib.ddamg_apply_coarse_multi(self._h, int(level), int(ys.shape[0]), _ptr(ys)[0], _ptr(out)[0]))
        return out

    def coarse_solve_multi(self, level, bs):
        bs = _c128(bs)
        x = np.empty_like(bs)
        self._check(_lib.ddamg_coarse_solve_multi(self._h, int(level), int(bs.shape[0]), _ptr(bs)[0], _ptr(x)[0]))
        return x

    def apply_coarse_schur_multi(self, level, ys):
        """Odd-even reduced operator of the coarsest level on [nrhs, ...] fields
        (odd-site entries of the input ignored, zero in the output)."""
        ys = _c128(ys)
        out = np.empty_like(ys)
        self._check(_lib.ddamg_apply_coarse_schur_multi(self._h, int(level), int(ys.shape[0]), _ptr(ys)[0],
                                                        _ptr(out)[0]))
        return out

    def coarse_sap_multi(self, level, bs, xs0, iters):
        bs = _c128(bs)
        xs = np.array(xs0, dtype=np.complex128, copy=True)
        self._check(_lib.ddamg_coarse_sap_multi(self._h, int(level), int(bs.shape[0]), _ptr(bs)[0], _ptr(xs)[0],
                                                int(iters)))
        return xs

    def bench_coarse(self, level, nrhs, napply, which=0):
        self._check(_lib.ddamg_bench_coarse(self._h, int(level), int(nrhs), int(napply), int(which)))

    def vcycle(self, v):
        v = _c128(v)
        out = np.empty_like(v)
        self._check(_lib.ddamg_vcycle(self._h, _ptr(v)[0], _ptr(out)[0]))
        return out

    # ---- learned setup ---------------------------------------------------------
    def net_create(self, nlayers, nchan):
        self._check(_lib.ddamg_net_create(self._h, int(nlayers), int(nchan)))
        self.net_shape = (int(nlayers), int(nchan))

    def net_set_params(self, vec):
        vec = np.ascontiguousarray(vec, dtype=np.float64)
        self._check(_lib.ddamg_net_set_params(self._h, vec.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                              vec.size))

    def net_get_params(self):
        n = _lib.ddamg_net_num_params(self._h)
        out = np.empty(n, dtype=np.float64)
        self._check(_lib.ddamg_net_get_params(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n))
        return out

    def net_forward(self, noise):
        noise = _c128(noise)
        out = np.empty_like(noise) if not _is_torch(noise) else noise.new_empty(noise.shape)
        pn, dev = _ptr(noise)
        self._check(_lib.ddamg_net_forward(self._h, pn, _ptr(out)[0], dev))
        return out

    def net_loss_grad(self, noise, target, want_grad=True):
        noise, target = _c128(noise), _c128(target)
        pn, dev = _ptr(noise)
        loss = ctypes.c_double()
        g = None
        gp = None
        if want_grad:
            g = np.empty(_lib.ddamg_net_num_params(self._h), dtype=np.float64)
            gp = g.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self._check(_lib.ddamg_net_loss_grad(self._h, pn, _ptr(target)[0], dev, ctypes.byref(loss), gp))
        return loss.value, g

    def net_train_step(self, noise, target, lr):
        noise, target = _c128(noise), _c128(target)
        pn, dev = _ptr(noise)
        loss = ctypes.c_double()
        self._check(_lib.ddamg_net_train_step(self._h, pn, _ptr(target)[0], dev, float(lr), ctypes.byref(loss)))
        return loss.value

    # ---- measurement ---------------------------------------------------------
    def bench_dirac(self, napply, precision="fp64"):
        self._check(_lib.ddamg_bench_dirac(self._h, PRECISIONS[precision], int(napply)))

    def set_progress(self, fn):
        """fn(stage, level, index) after every finished setup stage (stage 0:
        initial phase of a level, 1: one iteration of the iterated phase), or
        None to stop the notifications."""
        if fn is None:
            self._progress = None
            self._check(_lib.ddamg_set_progress(self._h, None, None))
            return
        cb = _PROGRESS_FN(lambda user, stage, level, index: fn(stage, level, index))
        self._progress = cb  # the library holds the pointer: keep the thunk alive
        self._check(_lib.ddamg_set_progress(self._h, ctypes.cast(cb, _vp), None))

    def timing(self, enable):
        self._check(_lib.ddamg_timing(self._h, int(bool(enable))))

    def timing_query(self, kind):
        c = ctypes.c_long()
        ms = ctypes.c_double()
        self._check(_lib.ddamg_timing_query(self._h, int(kind), ctypes.byref(c), ctypes.byref(ms)))
        return c.value, ms.value

    def error_reduction(self, e0, n=3):
        """rho = (|(I - M D)^n e0| / |e0|)^(1/n) of the current preconditioner."""
        e0 = _c128(e0)
        pe, dev = _ptr(e0)
        r = ctypes.c_double()
        self._check(_lib.ddamg_error_reduction(self._h, pe, dev, int(n), ctypes.byref(r)))
        return r.value

    def release_memory(self):
        """Give back the device memory of finished workspaces; returns the bytes still held."""
        h = ctypes.c_double()
        self._check(_lib.ddamg_release_memory(self._h, ctypes.byref(h)))
        return h.value

    def timing_bytes(self, kind):
        b = ctypes.c_double()
        self._check(_lib.ddamg_timing_bytes(self._h, int(kind), ctypes.byref(b)))
        return b.value

    def timing_flops(self, kind):
        f = ctypes.c_double()
        self._check(_lib.ddamg_timing_flops(self._h, int(kind), ctypes.byref(f)))
        return f.value
