"""Thin ctypes binding of libinla_bta.so (argument marshalling only).

Every computation runs in the HIP library; PyTorch supplies device memory and
the current stream.  There is no CPU fallback: if the library or a GPU is
missing, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np
import torch

from ._build import LIB, ROOT, source_hash

INLA_OK = 0
STATUS = {0: "ok", -1: "invalid argument", -2: "not positive definite", -3: "over HBM budget",
          -4: "HIP error", -5: "out of memory", -6: "library not usable"}


class InlaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Bta(C.Structure):
    _fields_ = [("b", C.c_int32), ("nt", C.c_int32), ("a", C.c_int32),
                ("D", C.c_void_p), ("S", C.c_void_p), ("R", C.c_void_p), ("T", C.c_void_p)]


class ModelDesc(C.Structure):
    _fields_ = [("N", C.c_int32), ("nt", C.c_int32), ("nb", C.c_int32), ("h", C.c_double),
                ("beta_prior_prec", C.c_double), ("m", C.c_int64),
                ("A_rowptr", C.c_void_p), ("A_col", C.c_void_p), ("A_val", C.c_void_p),
                ("y", C.c_void_p), ("theta_prior_mean", C.c_void_p),
                ("theta_prior_prec", C.c_void_p)]


class Opts(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_double), ("recompute", C.c_int32),
                ("keep_sigma", C.c_int32), ("tile", C.c_int32), ("reserved", C.c_int32),
                ("autotune_cache", C.c_char_p), ("sigma_out", C.POINTER(Bta))]


class BfgsOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("n_points", C.c_int32), ("gamma", C.c_double),
                ("gtol", C.c_double), ("ftol", C.c_double), ("eval_opts", C.POINTER(Opts)),
                ("max_step", C.c_double)]


class BfgsResult(C.Structure):
    _fields_ = [("theta", C.c_double * 4), ("f", C.c_double), ("grad", C.c_double * 4),
                ("iterations", C.c_int32), ("f_evals", C.c_int32), ("grad_evals", C.c_int32),
                ("reason", C.c_int32)]


class IntegrateOpts(C.Structure):
    _fields_ = [("h", C.c_double), ("dz", C.c_double), ("dpi", C.c_double),
                ("max_steps", C.c_int32), ("max_box", C.c_int32), ("eval_opts", C.POINTER(Opts))]


class IntegrateResult(C.Structure):
    _fields_ = [("f_mode", C.c_double), ("grad_mode", C.c_double * 4),
                ("hessian", C.c_double * 16), ("eigval", C.c_double * 4),
                ("eigvec", C.c_double * 16), ("theta_mean", C.c_double * 4),
                ("theta_cov", C.c_double * 16), ("log_evidence", C.c_double),
                ("lo", C.c_int32 * 4), ("hi", C.c_int32 * 4), ("n_box", C.c_int32),
                ("n_points", C.c_int32), ("f_evals", C.c_int32), ("grad_evals", C.c_int32)]


class NewtonOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("warm", C.c_int32), ("tol", C.c_double)]


class NewtonResult(C.Structure):
    _fields_ = [("f", C.c_double), ("grad", C.c_double * 4), ("logdet_p", C.c_double),
                ("logdet_c", C.c_double), ("log_lik", C.c_double), ("quad", C.c_double),
                ("iterations", C.c_int32), ("halvings", C.c_int32), ("status", C.c_int32),
                ("pad_", C.c_int32)]


_LIB = None

_SIGS = {
    "inla_model_create": (C.c_int, [C.POINTER(ModelDesc), C.c_void_p, C.POINTER(C.c_void_p)]),
    "inla_model_destroy": (None, [C.c_void_p]),
    "inla_model_shape": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                   C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                   C.POINTER(C.c_int64)]),
    "inla_assemble": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(Bta), C.c_void_p,
                                C.c_void_p]),
    "inla_factor_logdet": (C.c_int, [C.POINTER(Bta), C.c_void_p, C.c_void_p, C.c_void_p]),
    "inla_factor_logdet_noalloc": (C.c_int, [C.POINTER(Bta), C.c_void_p, C.c_void_p,
                                             C.c_void_p]),
    "inla_solve": (C.c_int, [C.POINTER(Bta), C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "inla_selinv": (C.c_int, [C.POINTER(Bta), C.POINTER(Bta), C.c_void_p, C.c_void_p]),
    "inla_eval_f": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.c_void_p, C.c_void_p,
                              C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(Opts), C.c_void_p]),
    "inla_eval_f_grad": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.POINTER(Opts), C.c_void_p]),
    "inla_eval_f_keep": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.POINTER(Opts), C.c_void_p,
                                   C.POINTER(C.c_void_p)]),
    "inla_eval_grad_kept": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p]),
    "inla_eval_state_kept": (C.c_int32, [C.c_void_p]),
    "inla_eval_state_destroy": (None, [C.c_void_p]),
    "inla_robust_quadratic_fit": (C.c_int, [C.POINTER(C.c_double), C.POINTER(C.c_double),
                                            C.c_int32, C.POINTER(C.c_double),
                                            C.POINTER(C.c_double)]),
    "inla_bfgs_minimize": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(BfgsOpts),
                                     C.POINTER(BfgsResult), C.POINTER(C.c_double), C.c_void_p]),
    "inla_integrate": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(IntegrateOpts),
                                 C.POINTER(IntegrateResult), C.POINTER(C.c_double), C.c_int32,
                                 C.c_void_p, C.c_void_p, C.c_void_p]),
    "inla_eval_f_grad_poisson": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(NewtonOpts),
                                           C.POINTER(NewtonResult), C.c_void_p, C.c_void_p,
                                           C.c_void_p]),
    "inla_release_workspace": (None, []),
    "inla_profile_begin": (C.c_int, []),
    "inla_profile_end": (C.c_int, [C.POINTER(C.c_double), C.c_int32]),
    "inla_profile_slots": (C.c_int32, []),
    "inla_status_string": (C.c_char_p, [C.c_int]),
    "inla_last_error": (C.c_char_p, []),
    "inla_build_id": (C.c_char_p, []),
}


def header_functions() -> list[str]:
    """Names of the functions declared in include/inla_bta.h."""
    with open(os.path.join(ROOT, "include", "inla_bta.h")) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(inla_[a-z_]+)\s*\(", text)))


def lib(path: str = LIB):
    """Load the HIP library (raises if it has not been built, or if it was
    built from other sources than the ones beside this package)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(path)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        built, want = L.inla_build_id().decode(), source_hash()
        if built != want:
            raise RuntimeError(f"{path} was built from other sources (build id {built}, sources "
                               f"{want}): rebuild it with __graft_entry__.build()")
        _LIB = L
    return _LIB


def build_id() -> str:
    """The source hash the loaded library was built from."""
    return lib().inla_build_id().decode()


def _check(code: int):
    if code != INLA_OK:
        raise InlaError(code, lib().inla_last_error().decode())


def _stream():
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU: the INLA library runs on the HIP device only")
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _dev_f64(x, device="cuda"):
    return torch.as_tensor(np.asarray(x, dtype=np.float64)).to(device).contiguous()


# ---------------------------------------------------------------------------
# BTA storage
# ---------------------------------------------------------------------------

class BtaTensors:
    """Device storage of one BTA matrix (see inla_bta in include/inla_bta.h)."""

    def __init__(self, b: int, nt: int, a: int, device="cuda", D=None, S=None, R=None, T=None):
        self.b, self.nt, self.a = b, nt, a
        z = lambda *s: torch.empty(*s, dtype=torch.float64, device=device)  # noqa: E731
        self.D = D if D is not None else z(nt, b, b)
        self.S = S if S is not None else (z(nt - 1, b, b) if nt > 1 else None)
        self.R = R if R is not None else (z(nt, b, a) if a > 0 else None)
        self.T = T if T is not None else (z(a, a) if a > 0 else None)

    # Blocks are column-major: element (i, j) of block t of D lives at D[t].view(-1)[i + j*b];
    # with torch's row-major view that is D[t][j, i].  The helpers return the logical blocks.
    def block(self, kind: str, t: int = 0):
        X = getattr(self, kind)
        if kind == "T":
            return X.t()
        return X[t].t()

    def struct(self) -> Bta:
        return Bta(self.b, self.nt, self.a, self.D.data_ptr(),
                   self.S.data_ptr() if self.S is not None else 0,
                   self.R.data_ptr() if self.R is not None else 0,
                   self.T.data_ptr() if self.T is not None else 0)

    @staticmethod
    def from_blocks(D, S, R, T, device="cuda"):
        """From logical numpy blocks D[nt,b,b], S[nt-1,b,b], R[nt,a,b], T[a,a]."""
        nt, b, _ = D.shape
        a = T.shape[0] if T is not None else 0
        cm = lambda X: torch.as_tensor(np.ascontiguousarray(np.swapaxes(X, -1, -2))).to(device)  # noqa: E731
        return BtaTensors(b, nt, a, device,
                          D=cm(D), S=cm(S) if nt > 1 else None,
                          R=cm(R) if a > 0 else None,
                          T=torch.as_tensor(np.ascontiguousarray(T.T)).to(device) if a > 0 else None)

    def to_blocks(self):
        """Logical numpy blocks (D, S, R, T)."""
        cm = lambda X: np.swapaxes(X.detach().cpu().numpy(), -1, -2).copy()  # noqa: E731
        D = cm(self.D)
        S = cm(self.S) if self.S is not None else np.zeros((0, self.b, self.b))
        R = cm(self.R) if self.R is not None else np.zeros((self.nt, 0, self.b))
        T = self.T.detach().cpu().numpy().T.copy() if self.T is not None else np.zeros((0, 0))
        return D, S, R, T


# ---------------------------------------------------------------------------
# model
# ---------------------------------------------------------------------------

class Model:
    """A model living on the GPU (inla_model_create)."""

    def __init__(self, N, nt, nb, h, A_rowptr, A_col, A_val, y, theta_prior_mean=None,
                 theta_prior_prec=None, beta_prior_prec=1e-3):
        L = lib()
        self._keep = [np.ascontiguousarray(A_rowptr, dtype=np.int64),
                      np.ascontiguousarray(A_col, dtype=np.int32),
                      np.ascontiguousarray(A_val, dtype=np.float64),
                      np.ascontiguousarray(y, dtype=np.float64),
                      np.ascontiguousarray(theta_prior_mean if theta_prior_mean is not None
                                           else np.zeros(4), dtype=np.float64),
                      np.ascontiguousarray(theta_prior_prec if theta_prior_prec is not None
                                           else np.full(4, 0.01), dtype=np.float64)]
        rp, col, val, yy, pm, pp = self._keep
        desc = ModelDesc(N, nt, nb, h, beta_prior_prec, yy.size,
                         rp.ctypes.data, col.ctypes.data, val.ctypes.data, yy.ctypes.data,
                         pm.ctypes.data, pp.ctypes.data)
        handle = C.c_void_p()
        _check(L.inla_model_create(C.byref(desc), _stream(), C.byref(handle)))
        self.handle = handle
        b, t_, a, n, m = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int64(), C.c_int64()
        _check(L.inla_model_shape(handle, b, t_, a, n, m))
        self.b, self.nt, self.a, self.n, self.m = b.value, t_.value, a.value, n.value, m.value
        self._keep = None

    @staticmethod
    def from_data(md) -> "Model":
        """From an inla_synth.ModelData."""
        return Model(md.N, md.nt, md.nb, md.h, md.A_rowptr, md.A_col, md.A_val, md.y,
                     md.theta_prior_mean, md.theta_prior_prec, md.beta_prior_prec)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _LIB is not None:
            _LIB.inla_model_destroy(h)
            self.handle = None


# ---------------------------------------------------------------------------
# the six operations
# ---------------------------------------------------------------------------

def assemble(model: Model, theta, which: int):
    """Q_prior (which=0) or Q_c (which=1) as BtaTensors; with which=1 also b = tau_y A^T y."""
    th = theta if torch.is_tensor(theta) else _dev_f64(theta)
    Q = BtaTensors(model.b, model.nt, model.a)
    rhs = torch.empty(model.n, dtype=torch.float64, device="cuda") if which == 1 else None
    st = Q.struct()
    _check(lib().inla_assemble(model.handle, _ptr(th), which, C.byref(st), _ptr(rhs), _stream()))
    return (Q, rhs) if which == 1 else Q


def factor_logdet(Q: BtaTensors):
    """In-place factorization; returns (logdet tensor[1], info tensor[1])."""
    ld = torch.empty(1, dtype=torch.float64, device="cuda")
    info = torch.empty(1, dtype=torch.int32, device="cuda")
    st = Q.struct()
    _check(lib().inla_factor_logdet(C.byref(st), _ptr(ld), _ptr(info), _stream()))
    return ld, info


def factor_logdet_noalloc(Q: BtaTensors, logdet=None, info=None):
    """inla_factor_logdet_noalloc: the same factorization with the library's
    fixed per-GPU workspace; logdet / info may be caller tensors (1 element)."""
    ld = logdet if logdet is not None else torch.empty(1, dtype=torch.float64, device="cuda")
    inf = info if info is not None else torch.empty(1, dtype=torch.int32, device="cuda")
    st = Q.struct()
    _check(lib().inla_factor_logdet_noalloc(C.byref(st), _ptr(ld), _ptr(inf), _stream()))
    return ld, inf


def solve(L: BtaTensors, rhs):
    """x = Q^{-1} rhs from the factor (rhs: n or n x nrhs, column-major per column)."""
    r = rhs.contiguous()
    nrhs = 1 if r.dim() == 1 else r.shape[0]
    x = torch.empty_like(r)
    st = L.struct()
    _check(lib().inla_solve(C.byref(st), _ptr(r), _ptr(x), nrhs, _stream()))
    return x


def selinv(L: BtaTensors, keep_sigma: bool = False):
    """Selected inverse: (BtaTensors of Sigma or None, diag tensor[n])."""
    n = L.b * L.nt + L.a
    diag = torch.empty(n, dtype=torch.float64, device="cuda")
    st = L.struct()
    sig = BtaTensors(L.b, L.nt, L.a) if keep_sigma else None
    sst = sig.struct() if sig is not None else None
    _check(lib().inla_selinv(C.byref(st), C.byref(sst) if sst is not None else None, _ptr(diag),
                             _stream()))
    return sig, diag


def _models_array(models):
    arr = (C.c_void_p * len(models))(*[m.handle.value for m in models])
    return arr


def _opts(budget=0.0, recompute=0, tile=0, autotune_cache=None, sigma=None):
    """inla_opts: HBM budget in bytes (0 = free memory minus a reserve);
    recompute 0 auto / 1 always / 2 never share one matrix's storage between
    Q_prior and Q_c; tile 0 (built-in rule or autotuner), 64 or 128;
    autotune_cache: JSON file the autotuner reads and extends (None: off);
    sigma: list of BtaTensors, one per item, receiving Sigma of Q_c (keep_sigma)."""
    path = None if autotune_cache is None else os.fsencode(os.fspath(autotune_cache))
    o = Opts(float(budget), int(recompute), 0, int(tile), 0, path, None)
    if sigma is not None:
        arr = (Bta * len(sigma))(*[x.struct() for x in sigma])
        o.keep_sigma = 1
        o.sigma_out = C.cast(arr, C.POINTER(Bta))
        o._keep = arr   # keeps the descriptor array alive with the options
    return o


def eval_f(models, thetas, want_mu=False, want_var=False, budget=0.0, recompute=0, tile=0,
           autotune_cache=None):
    """Batched f(theta).  Returns dict(f, status, [mu], [var]) of device tensors."""
    if isinstance(models, Model):
        models = [models]
    th = thetas if torch.is_tensor(thetas) else _dev_f64(np.atleast_2d(thetas))
    k = th.shape[0]
    if len(models) == 1 and k > 1:
        models = models * k
    ntot = sum(m.n for m in models)
    f = torch.empty(k, dtype=torch.float64, device="cuda")
    status = torch.empty(k, dtype=torch.int32, device="cuda")
    mu = torch.empty(ntot, dtype=torch.float64, device="cuda") if want_mu else None
    var = torch.empty(ntot, dtype=torch.float64, device="cuda") if want_var else None
    o = _opts(budget, recompute, tile, autotune_cache)
    _check(lib().inla_eval_f(_models_array(models), k, _ptr(th), _ptr(f), _ptr(mu), _ptr(var),
                             _ptr(status), C.byref(o), _stream()))
    out = dict(f=f, status=status)
    if want_mu:
        out["mu"] = mu
    if want_var:
        out["var"] = var
    return out


def eval_f_grad(models, thetas, want_mu=False, want_var=False, budget=0.0, recompute=0, tile=0,
                autotune_cache=None, sigma=None):
    """Batched f(theta) and its exact gradient.  Returns dict(f, grad, status, [mu], [var]).
    sigma: optional list of BtaTensors (one per item, the item's model shape)
    that receive the selected inverse of Q_c (keep_sigma)."""
    if isinstance(models, Model):
        models = [models]
    th = thetas if torch.is_tensor(thetas) else _dev_f64(np.atleast_2d(thetas))
    th = th.contiguous()
    k = th.shape[0]
    if len(models) == 1 and k > 1:
        models = models * k
    ntot = sum(m.n for m in models)
    f = torch.empty(k, dtype=torch.float64, device="cuda")
    g = torch.empty(k, 4, dtype=torch.float64, device="cuda")
    status = torch.empty(k, dtype=torch.int32, device="cuda")
    mu = torch.empty(ntot, dtype=torch.float64, device="cuda") if want_mu else None
    var = torch.empty(ntot, dtype=torch.float64, device="cuda") if want_var else None
    o = _opts(budget, recompute, tile, autotune_cache, sigma)
    _check(lib().inla_eval_f_grad(_models_array(models), k, _ptr(th), _ptr(f), _ptr(g), _ptr(mu),
                                  _ptr(var), _ptr(status), C.byref(o), _stream()))
    out = dict(f=f, grad=g, status=status)
    if want_mu:
        out["mu"] = mu
    if want_var:
        out["var"] = var
    return out


class EvalState:
    """f now, the gradient later (inla_eval_f_keep / inla_eval_grad_kept):
    the forward evaluation keeps the factors of the batch when they fit the
    HBM budget, and grad() runs only the selected inversions from them (or the
    whole evaluation again when they were not kept)."""

    def __init__(self, models, thetas, want_mu=False, budget=0.0, recompute=0, tile=0,
                 autotune_cache=None):
        if isinstance(models, Model):
            models = [models]
        th = thetas if torch.is_tensor(thetas) else _dev_f64(np.atleast_2d(thetas))
        th = th.contiguous()
        k = th.shape[0]
        if len(models) == 1 and k > 1:
            models = models * k
        self.models = list(models)   # the models must outlive the state
        self.k = k
        self.ntot = sum(m.n for m in models)
        self.f = torch.empty(k, dtype=torch.float64, device="cuda")
        self.status = torch.empty(k, dtype=torch.int32, device="cuda")
        self.mu = torch.empty(self.ntot, dtype=torch.float64, device="cuda") if want_mu else None
        o = _opts(budget, recompute, tile, autotune_cache)
        h = C.c_void_p()
        _check(lib().inla_eval_f_keep(_models_array(models), k, _ptr(th), _ptr(self.f),
                                      _ptr(self.mu), _ptr(self.status), C.byref(o), _stream(),
                                      C.byref(h)))
        self.handle = h

    @property
    def kept(self) -> bool:
        return bool(lib().inla_eval_state_kept(self.handle))

    def grad(self, want_var=False):
        """dict(f, grad, status, [var]) of the batch."""
        f = torch.empty(self.k, dtype=torch.float64, device="cuda")
        g = torch.empty(self.k, 4, dtype=torch.float64, device="cuda")
        st = torch.empty(self.k, dtype=torch.int32, device="cuda")
        var = torch.empty(self.ntot, dtype=torch.float64, device="cuda") if want_var else None
        _check(lib().inla_eval_grad_kept(self.handle, _ptr(f), _ptr(g), _ptr(var), _ptr(st),
                                         _stream()))
        out = dict(f=f, grad=g, status=st)
        if want_var:
            out["var"] = var
        return out

    def close(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _LIB is not None:
            _LIB.inla_eval_state_destroy(h)
        self.handle = None

    def __del__(self):
        self.close()


class InlaObjective(torch.autograd.Function):
    """f(theta) with the exact gradient from the selected-inversion adjoint.

    theta: (k, 4) float64 CUDA tensor; returns f (k,).  When theta requires a
    gradient the forward pass runs inla_eval_f_grad once and keeps grad f for
    the backward pass (opts defer_grad=False, the default), or runs f only and
    keeps the factors, and the backward pass recomputes the selected inverse
    from them (defer_grad=True: inla_eval_f_keep / inla_eval_grad_kept; the
    same gradient bit for bit).  Without a gradient it runs inla_eval_f.
    """

    @staticmethod
    def forward(ctx, theta, models, opts):
        th = theta.detach().contiguous()
        opts = dict(opts)
        defer = opts.pop("defer_grad", False)
        ctx.state = None
        if ctx.needs_input_grad[0]:
            if defer:
                ctx.state = EvalState(models, th, **opts)
                return ctx.state.f
            out = eval_f_grad(models, th, **opts)
            ctx.save_for_backward(out["grad"])
        else:
            out = eval_f(models, th, **opts)
        return out["f"]

    @staticmethod
    def backward(ctx, gout):
        if ctx.state is not None:
            g = ctx.state.grad()["grad"]
            ctx.state.close()
            ctx.state = None
        else:
            (g,) = ctx.saved_tensors
        return gout[:, None] * g, None, None


def objective(theta, models, **opts):
    """f(theta) as a differentiable function of theta (k x 4); opts as eval_f,
    plus defer_grad (see InlaObjective)."""
    return InlaObjective.apply(theta, models, opts)


BFGS_REASONS = {0: "gradient below gtol", 1: "decrease of f below ftol", 2: "max_iter reached",
                3: "no point of the search interval lowered f"}


def minimize(model: Model, theta0, max_iter=300, n_points=6, gamma=1.0, gtol=1e-6, ftol=1e-13,
             max_step=2.0, **eval_opts):
    """BFGS with the parallel line search (inla_bfgs_minimize) from theta0 (4 values).
    Returns dict(theta, f, grad, iterations, f_evals, grad_evals, reason, history)
    with history one row (f, max |grad|, alpha, theta[4], f evaluations) per iteration."""
    th0 = (C.c_double * 4)(*[float(v) for v in np.asarray(theta0, dtype=np.float64)])
    eo = _opts(**eval_opts) if eval_opts else None
    o = BfgsOpts(int(max_iter), int(n_points), float(gamma), float(gtol), float(ftol),
                 C.pointer(eo) if eo is not None else None, float(max_step))
    res = BfgsResult()
    hist = (C.c_double * ((max_iter + 1) * 8))()
    _check(lib().inla_bfgs_minimize(model.handle, th0, C.byref(o), C.byref(res), hist, _stream()))
    h = np.array(hist[:(res.iterations + 1) * 8]).reshape(-1, 8)
    return dict(theta=np.array(res.theta[:]), f=res.f, grad=np.array(res.grad[:]),
                iterations=res.iterations, f_evals=res.f_evals, grad_evals=res.grad_evals,
                reason=res.reason, history=h)


def integrate(model: Model, theta_mode, h=1e-3, dz=1.0, dpi=2.5, max_steps=6, max_box=20000,
              latent=True, points_cap=4096, **eval_opts):
    """The integration step at the mode (inla_integrate): the FD Hessian of the
    adjoint gradient, the standardised grid, the quadrature over theta and, if
    latent, the mixture mean and variance of the latent field (device tensors).
    Returns a dict of the result fields, 'points' (K x 10: s[4], theta[4], f, w)
    and 'x_mean' / 'x_var'."""
    th = (C.c_double * 4)(*[float(v) for v in np.asarray(theta_mode, dtype=np.float64)])
    eo = _opts(**eval_opts) if eval_opts else None
    o = IntegrateOpts(float(h), float(dz), float(dpi), int(max_steps), int(max_box),
                      C.pointer(eo) if eo is not None else None)
    res = IntegrateResult()
    pts = (C.c_double * (10 * points_cap))()
    xm = xv = None
    if latent:
        n = model.n
        xm = torch.empty(n, dtype=torch.float64, device="cuda")
        xv = torch.empty(n, dtype=torch.float64, device="cuda")
    _check(lib().inla_integrate(model.handle, th, C.byref(o), C.byref(res), pts, points_cap,
                                _ptr(xm), _ptr(xv), _stream()))
    K = res.n_points
    out = dict(f_mode=res.f_mode, grad_mode=np.array(res.grad_mode[:]),
               hessian=np.array(res.hessian[:]).reshape(4, 4), eigval=np.array(res.eigval[:]),
               eigvec=np.array(res.eigvec[:]).reshape(4, 4),
               theta_mean=np.array(res.theta_mean[:]),
               theta_cov=np.array(res.theta_cov[:]).reshape(4, 4),
               log_evidence=res.log_evidence, lo=np.array(res.lo[:]), hi=np.array(res.hi[:]),
               n_box=res.n_box, n_points=K, f_evals=res.f_evals, grad_evals=res.grad_evals,
               points=np.array(pts[:10 * min(K, points_cap)]).reshape(-1, 10))
    if latent:
        out["x_mean"], out["x_var"] = xm, xv
    return out


def eval_f_grad_poisson(model: Model, theta, max_iter=100, tol=1e-12, x0=None, want_var=False):
    """f(theta) and its exact gradient with a Poisson likelihood on the model's
    count responses (inla_eval_f_grad_poisson).  x0: optional device tensor
    (n) to start Newton's method from.  Returns dict(f, grad, logdet_p,
    logdet_c, log_lik, quad, iterations, halvings, status, x, [var])."""
    th = (C.c_double * 4)(*[float(v) for v in np.asarray(theta, dtype=np.float64)])
    x = torch.zeros(model.n, dtype=torch.float64, device="cuda")
    if x0 is not None:
        x.copy_(x0)
    var = torch.empty(model.n, dtype=torch.float64, device="cuda") if want_var else None
    o = NewtonOpts(int(max_iter), 1 if x0 is not None else 0, float(tol))
    res = NewtonResult()
    _check(lib().inla_eval_f_grad_poisson(model.handle, th, C.byref(o), C.byref(res), _ptr(x),
                                          _ptr(var), _stream()))
    out = dict(f=res.f, grad=np.array(res.grad[:]), logdet_p=res.logdet_p, logdet_c=res.logdet_c,
               log_lik=res.log_lik, quad=res.quad, iterations=res.iterations,
               halvings=res.halvings, status=res.status, x=x)
    if want_var:
        out["var"] = var
    return out


def release_workspace():
    lib().inla_release_workspace()


def profile_begin():
    _check(lib().inla_profile_begin())


PROFILE_SLOTS = ["diag0", "step", "diagc", "stepf", "offdiag_x", "offdiag", "schur_x", "schur", "arrow",
                 "si_init", "si_vu_x", "si_vu", "si_sr_x", "si_sr", "si_sd_x", "si_vu_b", "si_u_b",
                 "si_g_b", "solve", "trace", "assemble", "misc", "calls"]
PRODUCT_X = ("offdiag_x", "schur_x", "si_vu_x", "si_sr_x", "si_sd_x", "si_vu_b",
             "si_g_b")   # b x b products
FAT_PHASES = ("diag0", "diagc", "stepf", "arrow")   # run by the Cholesky-capable tile kernel


KERNEL_KINDS = ["tile_phase_kernel<false>", "tile_phase_kernel<true>", "tile_product_kernel", "other"]


def profile_end():
    """Per phase slot and per kernel: dict(launches, ms, flops)."""
    n = lib().inla_profile_slots()
    out = (C.c_double * (3 * n))()
    _check(lib().inla_profile_end(out, n))
    rows = [dict(launches=out[3 * k], ms=out[3 * k + 1], flops=out[3 * k + 2]) for k in range(n)]
    nph = len(PROFILE_SLOTS) - 1
    slots = {PROFILE_SLOTS[k]: rows[k] for k in range(nph)}
    calls = rows[nph]
    kernels = {KERNEL_KINDS[k]: rows[nph + 1 + k] for k in range(len(KERNEL_KINDS))}
    return {"slots": slots, "kernels": kernels, "calls": int(calls["launches"]),
            "bad": int(calls["ms"])}
