"""ctypes binding of librb (include/rb.h).  Argument marshalling only: every step of
the solvers runs in the library's HIP kernels.  PyTorch provides device memory
(float64 CUDA/HIP tensors) and the stream.

The library must be built (``python -m paper_1804_06363_amd.build`` or
``__graft_entry__.build()``); importing this module without it raises at once.
RB_LIBRARY_PATH overrides the library file (e.g. a build with other tile constants).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("RB_LIBRARY_PATH") or os.path.join(_HERE, "librb.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"librb.so is not built ({LIB_PATH}); run __graft_entry__.build()")
_lib = C.CDLL(LIB_PATH)

# ---- enums -------------------------------------------------------------------------
RB_OK, RB_EINVAL, RB_ENOMEM, RB_EDEVICE, RB_ENOTSPD, RB_ENOCONV, RB_EBREAKDOWN, \
    RB_EDEGENERATE, RB_EUNSUPPORTED, RB_EIO = range(10)
STATUS_NAMES = {RB_OK: "ok", RB_EINVAL: "einval", RB_ENOMEM: "enomem", RB_EDEVICE: "edevice",
                RB_ENOTSPD: "enotspd", RB_ENOCONV: "enoconv", RB_EBREAKDOWN: "ebreakdown",
                RB_EDEGENERATE: "edegenerate", RB_EUNSUPPORTED: "eunsupported", RB_EIO: "eio"}
PREC = {"fp64": 0, "fp32": 1, "bf16": 2}
SOLVER = {"rbcg": 0, "rbi": 1, "cg": 2}
INDICATOR = {"residual": 0, "l1": 1}
SMOOTHER = {"rbgs": 0, "rbgs_sym": 1, "jacobi": 2, "none": 3}


class RBError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


# ---- structs -----------------------------------------------------------------------
class StencilDesc(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("blocks", C.c_int * 3)]


class SolveOpts(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("solver", C.c_int), ("precond_prec", C.c_int),
                ("smoother", C.c_int), ("rtol", C.c_double), ("maxit", C.c_int),
                ("beta_flexible", C.c_int), ("use_graph", C.c_int), ("fixed_iters", C.c_int),
                ("check_every", C.c_int), ("autotune", C.c_int), ("stencil_kind", C.c_int),
                ("adapt_gamma", C.c_double), ("floor_factor", C.c_double),
                ("smooth_sweeps", C.c_int), ("residual_copy", C.c_int),
                ("prolong_kind", C.c_int), ("paired_x_update", C.c_int)]


class QueryStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("rel_res_true", C.c_double),
                ("rel_res_recursive", C.c_double), ("status", C.c_int), ("n_used", C.c_int),
                ("at_floor", C.c_int)]


class Query(C.Structure):
    _fields_ = [("problem", C.c_int), ("n_use", C.c_int), ("theta", C.POINTER(C.c_double)),
                ("phi", C.POINTER(C.c_double)), ("x", C.c_void_p), ("rtol", C.c_double)]


class GreedyOpts(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("n_max", C.c_int), ("seed_index", C.c_int64),
                ("indicator", C.c_int), ("snapshot_rtol", C.c_double),
                ("snapshot_maxit", C.c_int), ("snapshot_flexible", C.c_int),
                ("use_surrogate", C.c_int), ("topk", C.c_int), ("explore", C.c_int),
                ("full_sweep_every", C.c_int), ("warmup_full_sweeps", C.c_int),
                ("train_steps", C.c_int), ("lr", C.c_double), ("mu_lo", C.c_double),
                ("mu_hi", C.c_double), ("seed", C.c_uint64), ("snapshot_prec", C.c_int),
                ("surrogate_prec", C.c_int), ("snapshot_sweeps", C.c_int)]


class SurrogateIO(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("step", C.c_int), ("counter", C.c_uint64),
                ("full_sweep", C.c_int), ("fallback", C.c_int), ("n_topk", C.c_int),
                ("n_explore", C.c_int), ("pick", C.c_int64), ("value", C.c_double),
                ("true_evals", C.c_int64), ("loss", C.c_float)]


class GreedyReport(C.Structure):
    _fields_ = [("n_built", C.c_int), ("picks", C.POINTER(C.c_int64)),
                ("max_indicator", C.POINTER(C.c_double)), ("snapshot_iters", C.POINTER(C.c_int)),
                ("true_evals", C.c_int64), ("full_sweeps", C.c_int), ("seconds", C.c_double),
                ("mlp_loss", C.c_double), ("surrogate_fallbacks", C.c_int)]


_P = C.c_void_p
_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int)


def _sig(name, args, res=C.c_int):
    f = getattr(_lib, name)
    f.argtypes = args
    f.restype = res
    return f


rb_last_error = _sig("rb_last_error", [], C.c_char_p)
rb_version = _sig("rb_version", [], C.c_char_p)
_sig("rb_ctx_create", [C.c_int, _P, C.POINTER(_P)])
_sig("rb_ctx_destroy", [_P])
_sig("rb_profile_enable", [_P, C.c_int])
_sig("rb_profile_reset", [_P])
_sig("rb_profile_get", [_P, C.c_int, C.c_char_p, C.c_size_t, _D, C.POINTER(C.c_int64)])
_sig("rb_problem_create_stencil", [_P, C.POINTER(StencilDesc), C.POINTER(_P)])
_sig("rb_problem_set_rhs", [_P, C.c_int, _D])
_sig("rb_problem_create_csr", [_P, C.c_int64, C.c_int, C.POINTER(C.c_int64),
                               C.POINTER(C.c_int32), _D, C.POINTER(_P)])
_sig("rb_problem_colors", [_P, C.POINTER(C.c_int32), _I])
_sig("rb_problem_info", [_P, C.POINTER(C.c_int64), _I, _I])
_sig("rb_problem_destroy", [_P])
_sig("rb_basis_from_host", [_P, _P, C.c_int, _D, C.POINTER(_P)])
_sig("rb_basis_info", [_P, _I, _D, _D, _D])
_sig("rb_basis_save", [_P, C.c_char_p])
_sig("rb_basis_load", [_P, _P, C.c_char_p, C.POINTER(_P)])
_sig("rb_basis_destroy", [_P])
_sig("rb_solve_opts_default", [C.POINTER(SolveOpts)], None)
_sig("rb_solve_batch", [_P, _P, _P, C.POINTER(SolveOpts), C.c_int, _D, _D, _I, _P,
                        C.POINTER(QueryStats)])
_sig("rb_solve_multi", [_P, C.c_int, C.POINTER(_P), C.POINTER(_P), C.POINTER(SolveOpts),
                        C.c_int, C.POINTER(Query), C.POINTER(QueryStats)])
_sig("rb_apply_batch", [_P, _P, C.c_int, _D, _P, _P])
_sig("rb_precond_batch", [_P, _P, _P, C.POINTER(SolveOpts), C.c_int, _D, _I, _P, _P])
_sig("rb_project_batch", [_P, _P, _P, C.c_int, C.c_int, _P, _D])
_sig("rb_reduced_factor_batch", [_P, _P, C.c_int, _D, _D, _I])
_sig("rb_reduced_factor_batch_noalloc", [_P, _P, C.c_int, _D, _D, _I])
_F = C.POINTER(C.c_float)
_sig("rb_mlp_forward", [_P, C.c_int, C.c_int, C.c_int, _F, C.c_int, _F, _F])
_sig("rb_mlp_loss_grad", [_P, C.c_int, C.c_int, C.c_int, _F, C.c_int, _F, _F, _F, _F])
_sig("rb_mlp_train", [_P, C.c_int, C.c_int, C.c_int, _F, C.c_int, _F, _F, C.c_int, C.c_double, _F])
_sig("rb_topk", [_P, C.c_int, C.c_int, _F, _I, _I, _I])
_I32 = C.POINTER(C.c_int32)
_sig("rb_surrogate_step", [_P, _P, _P, C.POINTER(GreedyOpts), C.c_int64, C.c_int, _D, _D, _I32,
                           _F, C.c_int, _I32, _F, _I32, _I32, _I32, C.POINTER(SurrogateIO)])
_sig("rb_greedy_opts_default", [C.POINTER(GreedyOpts)], None)
_sig("rb_offline_build", [_P, _P, C.POINTER(GreedyOpts), C.c_int64, C.c_int, _D, _D, _D,
                          C.POINTER(_P), C.POINTER(GreedyReport)])
_sig("rb_basis_from_parameters", [_P, _P, C.POINTER(GreedyOpts), C.c_int, _D, _D,
                                  C.POINTER(_P), C.POINTER(GreedyReport)])

EXPORTED = [
    "rb_ctx_create", "rb_ctx_destroy", "rb_last_error", "rb_version",
    "rb_profile_enable", "rb_profile_reset", "rb_profile_get",
    "rb_problem_create_stencil", "rb_problem_create_csr", "rb_problem_colors",
    "rb_problem_set_rhs", "rb_problem_info", "rb_problem_destroy",
    "rb_basis_from_host", "rb_basis_info", "rb_basis_save", "rb_basis_load", "rb_basis_destroy",
    "rb_solve_opts_default", "rb_solve_batch", "rb_solve_multi",
    "rb_apply_batch",
    "rb_precond_batch", "rb_project_batch", "rb_reduced_factor_batch",
    "rb_reduced_factor_batch_noalloc",
    "rb_greedy_opts_default", "rb_offline_build", "rb_basis_from_parameters",
    "rb_mlp_forward", "rb_mlp_loss_grad", "rb_mlp_train", "rb_topk", "rb_surrogate_step",
]


def _check(status):
    if status != RB_OK:
        raise RBError(status, rb_last_error().decode())


def _dptr(a):
    return a.ctypes.data_as(_D) if a is not None else None


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _tensor_ptr(t):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.is_contiguous()):
        raise TypeError("expected a contiguous float64 GPU tensor")
    return C.c_void_p(t.data_ptr())


# ---- objects -----------------------------------------------------------------------
class Context:
    """A device and a HIP stream.  stream=None: the library creates its own stream."""

    def __init__(self, device: int = 0, stream=None):
        h = _P()
        sp = None
        if stream is not None:
            sp = C.c_void_p(int(stream))
        _check(_lib.rb_ctx_create(device, sp, C.byref(h)))
        self.h = h
        self.device = device

    def profile(self, on=True):
        _check(_lib.rb_profile_enable(self.h, int(on)))

    def profile_reset(self):
        _check(_lib.rb_profile_reset(self.h))

    def profile_totals(self):
        """{kernel name: (total ms, launches)} accumulated while profiling was on."""
        out = {}
        i = 0
        buf = C.create_string_buffer(64)
        ms = C.c_double()
        n = C.c_int64()
        while _lib.rb_profile_get(self.h, i, buf, 64, C.byref(ms), C.byref(n)) == RB_OK:
            out[buf.value.decode()] = (ms.value, n.value)
            i += 1
        return out

    def close(self):
        if self.h:
            _lib.rb_ctx_destroy(self.h)
            self.h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Problem:
    def __init__(self, ctx: Context, dims=None, blocks=None, _handle=None):
        if _handle is None:
            d = StencilDesc()
            d.dim = len(dims)
            for a in range(3):
                d.n[a] = dims[a] if a < len(dims) else 1
                d.blocks[a] = blocks[a] if a < len(blocks) else 1
            h = _P()
            _check(_lib.rb_problem_create_stencil(ctx.h, C.byref(d), C.byref(h)))
            self.dims, self.blocks = tuple(dims), tuple(blocks)
        else:
            h = _handle
            self.dims, self.blocks = None, None
        self.h, self.ctx = h, ctx
        N = C.c_int64()
        Q = C.c_int()
        R = C.c_int()
        _check(_lib.rb_problem_info(h, C.byref(N), C.byref(Q), C.byref(R)))
        self.N, self.Q, self.R = N.value, Q.value, R.value

    @classmethod
    def from_csr(cls, ctx: Context, rowptr, col, vals):
        """General sparse affine problem: terms vals [Q][nnz] on the pattern (rowptr, col)."""
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        vals = _f64(np.atleast_2d(vals))
        N = len(rowptr) - 1
        h = _P()
        _check(_lib.rb_problem_create_csr(ctx.h, N, vals.shape[0],
                                          rowptr.ctypes.data_as(C.POINTER(C.c_int64)),
                                          col.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(vals),
                                          C.byref(h)))
        return cls(ctx, _handle=h)

    def colors(self):
        """Colour class of every unknown (natural order) of the Gauss-Seidel smoother."""
        out = np.zeros(self.N, dtype=np.int32)
        nc = C.c_int()
        _check(_lib.rb_problem_colors(self.h, out.ctypes.data_as(C.POINTER(C.c_int32)),
                                      C.byref(nc)))
        return out, nc.value

    def set_rhs(self, f):
        f = _f64(np.atleast_2d(f))
        _check(_lib.rb_problem_set_rhs(self.h, f.shape[0], _dptr(f)))
        self.R = f.shape[0]

    def __del__(self):
        try:
            if self.h:
                _lib.rb_problem_destroy(self.h)
        except Exception:
            pass


class Basis:
    def __init__(self, ctx: Context, prob: Problem, handle):
        self.ctx, self.prob, self.h = ctx, prob, handle
        n = C.c_int()
        _check(_lib.rb_basis_info(handle, C.byref(n), None, None, None))
        self.n = n.value

    @classmethod
    def from_host(cls, ctx, prob, W):
        """W: [n][N] (rows are basis vectors), natural ordering."""
        W = _f64(np.atleast_2d(W))
        h = _P()
        _check(_lib.rb_basis_from_host(ctx.h, prob.h, W.shape[0] if W.size else 0, _dptr(W),
                                       C.byref(h)))
        return cls(ctx, prob, h)

    @classmethod
    def load(cls, ctx, prob, path):
        h = _P()
        _check(_lib.rb_basis_load(ctx.h, prob.h, path.encode(), C.byref(h)))
        return cls(ctx, prob, h)

    def save(self, path):
        _check(_lib.rb_basis_save(self.h, path.encode()))

    def info(self):
        """(W [n][N], AN [Q][n][n], fN [R][n]) copied to the host."""
        n, N, Q, R = self.n, self.prob.N, self.prob.Q, self.prob.R
        W = np.empty((n, N))
        AN = np.empty((Q, n, n))
        fN = np.empty((R, n))
        _check(_lib.rb_basis_info(self.h, None, _dptr(W), _dptr(AN), _dptr(fN)))
        return W, AN, fN

    def __del__(self):
        try:
            if self.h:
                _lib.rb_basis_destroy(self.h)
        except Exception:
            pass


STENCIL_KIND = {"auto": 0, "chunked": 1, "zmarch": 2, "fused": 3, "zmarch4": 4}
PROLONG_KIND = {"auto": 0, "mfma": 1, "vector": 2}


def solve_opts(solver="rbcg", prec="fp64", smoother="rbgs", rtol=1e-10, maxit=2000,
               flexible=False, graph=False, fixed_iters=0, check_every=0, autotune=False,
               stencil="auto", adapt_gamma=0.0, sweeps=1, floor_factor=0.0, residual_copy=True,
               prolong="auto", paired_x=True):
    o = SolveOpts()
    _lib.rb_solve_opts_default(C.byref(o))
    o.solver = SOLVER[solver]
    o.precond_prec = PREC[prec]
    o.smoother = SMOOTHER[smoother]
    o.rtol = rtol
    o.maxit = maxit
    o.beta_flexible = int(flexible)
    o.use_graph = int(graph)
    o.fixed_iters = fixed_iters
    o.check_every = check_every
    o.autotune = int(autotune)
    o.stencil_kind = STENCIL_KIND[stencil]
    o.adapt_gamma = adapt_gamma
    o.smooth_sweeps = sweeps
    o.floor_factor = floor_factor
    o.residual_copy = int(residual_copy)
    o.prolong_kind = PROLONG_KIND[prolong]
    o.paired_x_update = int(paired_x)
    return o


@dataclass
class Stats:
    iters: np.ndarray
    rel_res_true: np.ndarray
    rel_res_recursive: np.ndarray
    status: np.ndarray
    n_used: np.ndarray
    at_floor: np.ndarray


def _stats(arr, B):
    return Stats(np.array([arr[i].iters for i in range(B)]),
                 np.array([arr[i].rel_res_true for i in range(B)]),
                 np.array([arr[i].rel_res_recursive for i in range(B)]),
                 np.array([arr[i].status for i in range(B)]),
                 np.array([arr[i].n_used for i in range(B)]),
                 np.array([arr[i].at_floor for i in range(B)]))


def solve_batch(ctx, prob, basis, theta, x=None, phi=None, n_use=None, **kw):
    """Solve B queries; x is a [B][N] float64 GPU tensor (allocated if None)."""
    import torch
    theta = _f64(np.atleast_2d(theta))
    B = theta.shape[0]
    if x is None:
        x = torch.empty((B, prob.N), dtype=torch.float64, device=f"cuda:{ctx.device}")
    phi = _f64(phi)
    nu = None if n_use is None else np.ascontiguousarray(n_use, dtype=np.int32)
    opts = kw.pop("opts", None) or solve_opts(**kw)
    st = (QueryStats * B)()
    _check(_lib.rb_solve_batch(ctx.h, prob.h, basis.h if basis is not None else None,
                               C.byref(opts), B, _dptr(theta), _dptr(phi),
                               nu.ctypes.data_as(_I) if nu is not None else None,
                               _tensor_ptr(x), st))
    return x, _stats(st, B)


def solve_multi(ctx, probs, bases, queries, **kw):
    """queries: list of (problem index, n_use, theta, phi or None, x tensor[, rtol])."""
    opts = kw.pop("opts", None) or solve_opts(**kw)
    B = len(queries)
    qs = (Query * B)()
    keep = []
    for i, q in enumerate(queries):
        pi, nu, th, ph, x = q[:5]
        qs[i].rtol = q[5] if len(q) > 5 else 0.0
        th = _f64(th)
        ph = _f64(ph)
        keep += [th, ph]
        qs[i].problem = pi
        qs[i].n_use = nu
        qs[i].theta = _dptr(th)
        qs[i].phi = _dptr(ph) if ph is not None else None
        qs[i].x = _tensor_ptr(x)
    ph_arr = (_P * len(probs))(*[p.h for p in probs])
    bs_arr = (_P * len(bases))(*[b.h if b is not None else None for b in bases])
    st = (QueryStats * B)()
    _check(_lib.rb_solve_multi(ctx.h, len(probs), ph_arr, bs_arr, C.byref(opts), B, qs, st))
    return _stats(st, B)


def apply_batch(ctx, prob, theta, u):
    import torch
    theta = _f64(np.atleast_2d(theta))
    y = torch.empty_like(u)
    _check(_lib.rb_apply_batch(ctx.h, prob.h, theta.shape[0], _dptr(theta), _tensor_ptr(u),
                               _tensor_ptr(y)))
    return y


def precond_batch(ctx, prob, basis, theta, r, n_use=None, **kw):
    import torch
    theta = _f64(np.atleast_2d(theta))
    opts = kw.pop("opts", None) or solve_opts(**kw)
    y = torch.empty_like(r)
    nu = None if n_use is None else np.ascontiguousarray(n_use, dtype=np.int32)
    _check(_lib.rb_precond_batch(ctx.h, prob.h, basis.h if basis is not None else None,
                                 C.byref(opts), theta.shape[0], _dptr(theta),
                                 nu.ctypes.data_as(_I) if nu is not None else None,
                                 _tensor_ptr(r), _tensor_ptr(y)))
    return y


def project_batch(ctx, prob, basis, r, prec="fp64"):
    B = r.shape[0]
    t = np.empty((B, basis.n))
    _check(_lib.rb_project_batch(ctx.h, prob.h, basis.h, PREC[prec], B, _tensor_ptr(r), _dptr(t)))
    return t


def reduced_factor_batch(ctx, basis, theta):
    theta = _f64(np.atleast_2d(theta))
    B, n = theta.shape[0], basis.n
    L = np.empty((B, n, n))
    st = np.empty(B, dtype=np.int32)
    _check(_lib.rb_reduced_factor_batch(ctx.h, basis.h, B, _dptr(theta), _dptr(L),
                                        st.ctypes.data_as(_I)))
    return L, st


def reduced_factor_batch_noalloc(ctx, basis, theta):
    """reduced_factor_batch through the entry point that allocates no device memory."""
    theta = _f64(np.atleast_2d(theta))
    B, n = theta.shape[0], basis.n
    L = np.empty((B, n, n))
    st = np.empty(B, dtype=np.int32)
    _check(_lib.rb_reduced_factor_batch_noalloc(ctx.h, basis.h, B, _dptr(theta), _dptr(L),
                                                st.ctypes.data_as(_I)))
    return L, st


def greedy_opts(**kw):
    o = GreedyOpts()
    _lib.rb_greedy_opts_default(C.byref(o))
    for k, v in kw.items():
        if k == "indicator":
            v = INDICATOR[v]
        elif k in ("snapshot_prec", "surrogate_prec"):
            v = PREC[v]
        setattr(o, k, v)
    return o


def offline_build(ctx, prob, theta, mu=None, phi=None, **kw):
    theta = _f64(np.atleast_2d(theta))
    M = theta.shape[0]
    mu = _f64(mu)
    P = mu.shape[1] if mu is not None else 0
    opts = greedy_opts(**kw)
    nmax = opts.n_max
    picks = np.zeros(nmax, dtype=np.int64)
    maxind = np.zeros(nmax)
    sit = np.zeros(nmax, dtype=np.int32)
    rep = GreedyReport()
    rep.picks = picks.ctypes.data_as(C.POINTER(C.c_int64))
    rep.max_indicator = _dptr(maxind)
    rep.snapshot_iters = sit.ctypes.data_as(_I)
    h = _P()
    _check(_lib.rb_offline_build(ctx.h, prob.h, C.byref(opts), M, P, _dptr(mu), _dptr(theta),
                                 _dptr(_f64(phi)), C.byref(h), C.byref(rep)))
    nb = rep.n_built
    report = {"n_built": nb, "picks": picks[:nb].tolist(), "max_indicator": maxind[:nb].tolist(),
              "snapshot_iters": sit[:nb].tolist(), "true_evals": rep.true_evals,
              "full_sweeps": rep.full_sweeps, "seconds": rep.seconds, "mlp_loss": rep.mlp_loss,
              "surrogate_fallbacks": rep.surrogate_fallbacks}
    return Basis(ctx, prob, h), report


def basis_from_parameters(ctx, prob, theta, phi=None, **kw):
    """Snapshot solves and basis updates of Alg. 4 for the given parameters (multi-fidelity build, Sec. 4.2)."""
    theta = _f64(np.atleast_2d(theta))
    K = theta.shape[0]
    opts = greedy_opts(**kw)
    picks = np.zeros(K, dtype=np.int64)
    sit = np.zeros(K, dtype=np.int32)
    rep = GreedyReport()
    rep.picks = picks.ctypes.data_as(C.POINTER(C.c_int64))
    rep.snapshot_iters = sit.ctypes.data_as(_I)
    h = _P()
    _check(_lib.rb_basis_from_parameters(ctx.h, prob.h, C.byref(opts), K, _dptr(theta),
                                         _dptr(_f64(phi)), C.byref(h), C.byref(rep)))
    nb = rep.n_built
    report = {"n_built": nb, "picks": picks[:nb].tolist(), "snapshot_iters": sit[:nb].tolist(),
              "seconds": rep.seconds}
    return Basis(ctx, prob, h), report


# ---- MLP surrogate diagnostics ------------------------------------------------------------
def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _fptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def mlp_forward(ctx, P, H, params, X, prec="bf16"):
    params, X = _f32(params), _f32(X)
    out = np.empty(X.shape[0], dtype=np.float32)
    _check(_lib.rb_mlp_forward(ctx.h, P, H, PREC[prec], _fptr(params), X.shape[0], _fptr(X),
                               _fptr(out)))
    return out


def mlp_loss_grad(ctx, P, H, params, X, y, prec="bf16"):
    params, X, y = _f32(params), _f32(X), _f32(y)
    g = np.empty_like(params)
    loss = np.zeros(1, dtype=np.float32)
    _check(_lib.rb_mlp_loss_grad(ctx.h, P, H, PREC[prec], _fptr(params), X.shape[0], _fptr(X),
                                 _fptr(y), _fptr(loss), _fptr(g)))
    return float(loss[0]), g


def mlp_train(ctx, P, H, params, X, y, steps, lr, prec="bf16"):
    params, X, y = _f32(params).copy(), _f32(X), _f32(y)
    loss = np.zeros(1, dtype=np.float32)
    _check(_lib.rb_mlp_train(ctx.h, P, H, PREC[prec], _fptr(params), X.shape[0], _fptr(X),
                             _fptr(y), steps, lr, _fptr(loss)))
    return params, float(loss[0])


def topk(ctx, v, K, excluded=None):
    v = _f32(v)
    M = v.shape[0]
    ex = None if excluded is None else np.ascontiguousarray(excluded, dtype=np.int32)
    out = np.empty(max(K, 1), dtype=np.int32)
    cnt = C.c_int()
    _check(_lib.rb_topk(ctx.h, M, K, _fptr(v), ex.ctypes.data_as(_I) if ex is not None else None,
                        out.ctypes.data_as(_I), C.byref(cnt)))
    return out[:cnt.value]


def surrogate_step(ctx, prob, basis, theta, mu, excluded, params, step, counter,
                   buffer=(), **kw):
    """One surrogate-ranked greedy step (rb_surrogate_step).  buffer: iterable of
    (candidate, target, step).  Returns a dict with the pick, its value, the top-K and
    exploration lists, the flags, the weights after training and the new counter."""
    theta = _f64(np.atleast_2d(theta))
    mu = _f64(np.atleast_2d(mu))
    M, P = mu.shape
    opts = greedy_opts(**kw)
    ex = np.ascontiguousarray(excluded, dtype=np.int32)
    par = _f32(params).copy()
    buf = list(buffer)
    bi = np.ascontiguousarray([b[0] for b in buf], dtype=np.int32)
    bt = _f32([b[1] for b in buf])
    bs = np.ascontiguousarray([b[2] for b in buf], dtype=np.int32)
    tk = np.zeros(max(opts.topk, 1), dtype=np.int32)
    xp = np.zeros(max(opts.explore, 1), dtype=np.int32)
    io = SurrogateIO()
    io.struct_size = C.sizeof(SurrogateIO)
    io.step = step
    io.counter = counter
    i32 = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))  # noqa: E731
    _check(_lib.rb_surrogate_step(ctx.h, prob.h, basis.h, C.byref(opts), M, P, _dptr(mu),
                                  _dptr(theta), i32(ex), _fptr(par), len(buf), i32(bi),
                                  _fptr(bt), i32(bs), i32(tk), i32(xp), C.byref(io)))
    return {"pick": io.pick, "value": io.value, "topk": tk[:io.n_topk].tolist(),
            "explore": xp[:io.n_explore].tolist(), "full_sweep": bool(io.full_sweep),
            "fallback": bool(io.fallback), "params": par, "counter": io.counter,
            "true_evals": io.true_evals, "loss": io.loss}
