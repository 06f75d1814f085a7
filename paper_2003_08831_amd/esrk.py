"""Thin ctypes binding of libesrk.so (C-ABI in include/esrk.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Device arrays are torch tensors on the HIP device (float64, C
contiguous) or raw device addresses (int).  Loading fails loudly if the
library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libesrk.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "esrk.h")

FP64, FP32_FLUX = 0, 1
MLP_TRAINED, MLP_MODEL, MLP_IN = 1281, 1298, 5
SSPRK33, RK44, BSRK43, BSRK85 = 0, 1, 2, 3
RELAX_LOCAL, RELAX_GLOBAL, RELAX_NONE = 0, 1, 2
ROOT_ILLINOIS, ROOT_BRENT, ROOT_BISECTION, ROOT_ALEFELD = 0, 1, 2, 3
BC_DIRICHLET, BC_OUTFLOW = 0, 1

STATUS = {0: "OK", 1: "EINVAL", 2: "EHIP", 3: "ENOMEM", 4: "ENOROOT", 5: "ENONPHYS",
          6: "ENAN", 7: "ENOTSUP"}


class EsrkError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = code
        super().__init__(f"{where}: {STATUS.get(code, code)}")


class Config(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("deg", C.c_int), ("nel", C.c_int * 3),
        ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("gas_gamma", C.c_double), ("gas_r", C.c_double), ("mu", C.c_double),
        ("prandtl", C.c_double), ("lambda_scale", C.c_double),
        ("precision", C.c_int), ("tableau", C.c_int), ("cfl", C.c_double),
        ("root_tol", C.c_double), ("root_maxit", C.c_int), ("gamma_max", C.c_double),
    ]


_lib = None


def declared_symbols():
    """Function names declared in include/esrk.h."""
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(esrk_[a-z_]+)\s*\(", text)))


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library missing: {LIB_PATH} (run __graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    vp, dp, st = C.c_void_p, C.c_double, C.c_int
    L.esrk_create.argtypes = [C.POINTER(Config), C.POINTER(vp)]
    L.esrk_create.restype = st
    L.esrk_destroy.argtypes = [vp]
    L.esrk_destroy.restype = None
    L.esrk_num_nodes.argtypes = [vp]
    L.esrk_num_nodes.restype = C.c_size_t
    L.esrk_num_elems.argtypes = [vp]
    L.esrk_num_elems.restype = C.c_size_t
    L.esrk_num_vars.argtypes = [vp]
    L.esrk_num_vars.restype = C.c_int
    L.esrk_rhs_euler.argtypes = [vp, vp, vp, vp, vp]
    L.esrk_rhs_euler.restype = st
    L.esrk_rhs_ns.argtypes = [vp, vp, vp, vp, vp, vp]
    L.esrk_rhs_ns.restype = st
    L.esrk_rk_stage.argtypes = [vp, C.c_int, dp, vp, vp, vp, vp, vp, vp]
    L.esrk_rk_stage.restype = st
    L.esrk_local_relaxation_solve.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.esrk_local_relaxation_solve.restype = st
    L.esrk_step.argtypes = [vp, vp, vp, dp, vp, vp, vp]
    L.esrk_step.restype = st
    L.esrk_run_graph.argtypes = [vp, vp, vp, C.c_int, vp, vp]
    L.esrk_run_graph.restype = st
    L.esrk_global_relaxation_solve.argtypes = [vp, vp, vp, vp, vp, C.POINTER(C.c_int), vp]
    L.esrk_global_relaxation_solve.restype = st
    L.esrk_set_relaxation_mode.argtypes = [vp, C.c_int]
    L.esrk_set_relaxation_mode.restype = st
    L.esrk_stage_phi0.argtypes = [vp, vp, vp]
    L.esrk_stage_phi0.restype = st
    L.esrk_local_relaxation_solve_phi0.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.esrk_local_relaxation_solve_phi0.restype = st
    L.esrk_set_dirichlet.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.esrk_set_dirichlet.restype = st
    L.esrk_set_boundaries.argtypes = [vp, C.c_int, C.POINTER(C.c_double), C.c_int,
                                      C.POINTER(C.c_double)]
    L.esrk_set_boundaries.restype = st
    L.esrk_set_root_method.argtypes = [vp, C.c_int]
    L.esrk_set_root_method.restype = st
    L.esrk_set_adaptive.argtypes = [vp, dp, dp]
    L.esrk_set_adaptive.restype = st
    L.esrk_error_estimate.argtypes = [vp, vp, vp, vp]
    L.esrk_error_estimate.restype = st
    L.esrk_sync_status.argtypes = [vp, C.POINTER(C.c_int64)]
    L.esrk_sync_status.restype = st
    L.esrk_status_str.argtypes = [st]
    L.esrk_status_str.restype = C.c_char_p
    L.esrk_batch_create.argtypes = [C.POINTER(Config), C.c_int, C.POINTER(vp)]
    L.esrk_batch_create.restype = st
    L.esrk_batch_destroy.argtypes = [vp]
    L.esrk_batch_destroy.restype = None
    L.esrk_batch_num_sims.argtypes = [vp]
    L.esrk_batch_num_sims.restype = C.c_int
    for n in ("esrk_batch_state_len", "esrk_batch_num_elems"):
        getattr(L, n).argtypes = [vp]
        getattr(L, n).restype = C.c_size_t
    for n in ("esrk_batch_offset", "esrk_batch_elem_offset"):
        getattr(L, n).argtypes = [vp, C.c_int]
        getattr(L, n).restype = C.c_size_t
    L.esrk_batch_tile.argtypes = [vp]
    L.esrk_batch_tile.restype = C.c_int
    L.esrk_batch_step.argtypes = [vp, vp, vp, vp, vp]
    L.esrk_batch_step.restype = st
    L.esrk_batch_autotune.argtypes = [vp, vp, C.c_int, C.POINTER(C.c_int), vp]
    L.esrk_batch_autotune.restype = st
    L.esrk_batch_run_graph.argtypes = [vp, vp, vp, vp, C.c_int, vp]
    L.esrk_batch_run_graph.restype = st
    L.esrk_batch_sync_status.argtypes = [vp, C.POINTER(C.c_int64)]
    L.esrk_batch_sync_status.restype = st
    L.esrk_local_relaxation_solve_ml.argtypes = [vp, vp, vp, vp, dp, vp, vp, vp, vp, vp, vp,
                                                 vp]
    L.esrk_local_relaxation_solve_ml.restype = st
    L.esrk_set_step_model.argtypes = [vp, vp, vp]
    L.esrk_set_step_model.restype = st
    L.esrk_mlp_forward.argtypes = [vp, vp, C.c_int, vp, vp]
    L.esrk_mlp_forward.restype = st
    L.esrk_mlp_grad.argtypes = [vp, vp, vp, C.c_int, vp, vp, vp, vp]
    L.esrk_mlp_grad.restype = st
    L.esrk_mlp_grad_work_size.argtypes = [C.c_int]
    L.esrk_mlp_grad_work_size.restype = C.c_size_t
    L.esrk_mlp_adam.argtypes = [vp, vp, vp, vp, C.c_int, C.c_float, vp]
    L.esrk_mlp_adam.restype = st
    L.esrk_mlp_prepare.argtypes = [vp, vp, vp, C.c_int, C.c_int, vp, vp, vp]
    L.esrk_mlp_prepare.restype = st
    _lib = L
    return L


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check(rc, where):
    if rc != 0:
        raise EsrkError(rc, where)


def make_config(dim, deg, nel, lo, hi, gas_gamma=1.4, gas_r=1.0, mu=0.0, prandtl=0.72,
                lambda_scale=1.0, precision=FP64, tableau=SSPRK33, cfl=0.5,
                root_tol=1e-12, root_maxit=60, gamma_max=4.0) -> Config:
    c = Config()
    c.dim, c.deg = dim, deg
    nel = list(nel) + [1] * (3 - len(nel))
    lo = list(lo) + [0.0] * (3 - len(lo))
    hi = list(hi) + [1.0] * (3 - len(hi))
    for q in range(3):
        c.nel[q], c.lo[q], c.hi[q] = int(nel[q]), float(lo[q]), float(hi[q])
    c.gas_gamma, c.gas_r, c.mu, c.prandtl = gas_gamma, gas_r, mu, prandtl
    c.lambda_scale, c.precision, c.tableau, c.cfl = lambda_scale, precision, tableau, cfl
    c.root_tol, c.root_maxit, c.gamma_max = root_tol, root_maxit, gamma_max
    return c


class Context:
    """Owns one esrk_ctx.  Methods mirror the C entry points one to one."""

    def __init__(self, cfg: Config):
        L = load()
        h = C.c_void_p()
        _check(L.esrk_create(C.byref(cfg), C.byref(h)), "esrk_create")
        self._h = h
        self.cfg = cfg
        self.N = int(L.esrk_num_nodes(h))
        self.ne = int(L.esrk_num_elems(h))
        self.nv = int(L.esrk_num_vars(h))

    def close(self):
        if getattr(self, "_h", None):
            load().esrk_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def rhs_euler(self, u, dudt, eta_rate=None, stream=None):
        _check(load().esrk_rhs_euler(self._h, _ptr(u), _ptr(dudt), _ptr(eta_rate),
                                     _stream(stream)), "esrk_rhs_euler")

    def rhs_ns(self, u, dudt, eta_rate=None, visc_diss=None, stream=None):
        _check(load().esrk_rhs_ns(self._h, _ptr(u), _ptr(dudt), _ptr(eta_rate),
                                  _ptr(visc_diss), _stream(stream)), "esrk_rhs_ns")

    def rk_stage(self, stage, dt, u_old, y_in, y_out, du, deta, stream=None):
        _check(load().esrk_rk_stage(self._h, int(stage), float(dt), _ptr(u_old), _ptr(y_in),
                                    _ptr(y_out), _ptr(du), _ptr(deta), _stream(stream)),
               "esrk_rk_stage")

    def local_relaxation_solve(self, u_old, du, deta, gamma_k, gamma, gamma_guess=None,
                               iters=None, stream=None):
        _check(load().esrk_local_relaxation_solve(
            self._h, _ptr(u_old), _ptr(du), _ptr(deta), _ptr(gamma_guess), _ptr(gamma_k),
            _ptr(gamma), _ptr(iters), _stream(stream)), "esrk_local_relaxation_solve")

    def local_relaxation_solve_ml(self, u_old, du, deta, dt, gamma_k, gamma, visc_rate=None,
                                  model=None, feats=None, iters=None, stream=None):
        _check(load().esrk_local_relaxation_solve_ml(
            self._h, _ptr(u_old), _ptr(du), _ptr(deta), float(dt), _ptr(visc_rate),
            _ptr(model), _ptr(feats), _ptr(gamma_k), _ptr(gamma), _ptr(iters),
            _stream(stream)), "esrk_local_relaxation_solve_ml")

    def global_relaxation_solve(self, u_old, du, deta, gamma, stream=None):
        """Blocks until *gamma is written; returns the number of device passes."""
        passes = C.c_int(0)
        _check(load().esrk_global_relaxation_solve(
            self._h, _ptr(u_old), _ptr(du), _ptr(deta), _ptr(gamma), C.byref(passes),
            _stream(stream)), "esrk_global_relaxation_solve")
        return passes.value

    def set_relaxation_mode(self, mode):
        _check(load().esrk_set_relaxation_mode(self._h, int(mode)), "esrk_set_relaxation_mode")

    def stage_phi0(self, phi0, stream=None):
        _check(load().esrk_stage_phi0(self._h, _ptr(phi0), _stream(stream)), "esrk_stage_phi0")

    def local_relaxation_solve_phi0(self, u_old, du, deta, phi0, gamma_k, gamma, iters=None,
                                    stream=None):
        _check(load().esrk_local_relaxation_solve_phi0(
            self._h, _ptr(u_old), _ptr(du), _ptr(deta), _ptr(phi0), _ptr(gamma_k), _ptr(gamma),
            _ptr(iters), _stream(stream)), "esrk_local_relaxation_solve_phi0")

    def set_dirichlet(self, u_left=None, u_right=None):
        """Exterior conserved states (3 values each, host) of a 1-D context;
        None for both: periodic."""
        def arr(x):
            if x is None:
                return None
            return (C.c_double * 3)(*[float(v) for v in x])
        _check(load().esrk_set_dirichlet(self._h, arr(u_left), arr(u_right)), "esrk_set_dirichlet")

    def set_boundaries(self, kind_left, u_left, kind_right, u_right):
        """Boundary kind (BC_DIRICHLET, BC_OUTFLOW) and Dirichlet state (3
        conserved values, host; None for an outflow end) of each end of a
        1-D context."""
        def arr(x):
            if x is None:
                return None
            return (C.c_double * 3)(*[float(v) for v in x])
        _check(load().esrk_set_boundaries(self._h, int(kind_left), arr(u_left), int(kind_right),
                                          arr(u_right)), "esrk_set_boundaries")

    def set_root_method(self, method):
        _check(load().esrk_set_root_method(self._h, int(method)), "esrk_set_root_method")

    def set_adaptive(self, atol, rtol):
        _check(load().esrk_set_adaptive(self._h, float(atol), float(rtol)), "esrk_set_adaptive")

    def error_estimate(self, err=None, norm=None, stream=None):
        _check(load().esrk_error_estimate(self._h, _ptr(err), _ptr(norm), _stream(stream)),
               "esrk_error_estimate")

    def set_step_model(self, model=None, feats_out=None):
        # the context keeps the raw pointers: hold the tensors while they are set
        self._step_model_refs = (model, feats_out)
        _check(load().esrk_set_step_model(self._h, _ptr(model), _ptr(feats_out)),
               "esrk_set_step_model")

    def step(self, u, t, dt=0.0, gamma_k=None, stats=None, stream=None):
        if stats is not None and not isinstance(stats, int) and stats.numel() < 8:
            raise ValueError("stats needs 8 float64 entries")
        _check(load().esrk_step(self._h, _ptr(u), _ptr(t), float(dt), _ptr(gamma_k),
                                _ptr(stats), _stream(stream)), "esrk_step")

    def run_graph(self, u, t, nsteps, stats=None, stream=None):
        if stats is not None and not isinstance(stats, int) and stats.numel() < 8:
            raise ValueError("stats needs 8 float64 entries")
        _check(load().esrk_run_graph(self._h, _ptr(u), _ptr(t), int(nsteps), _ptr(stats),
                                     _stream(stream)), "esrk_run_graph")

    def sync_status(self):
        bad = C.c_int64(-1)
        rc = load().esrk_sync_status(self._h, C.byref(bad))
        return rc, bad.value


class Batch:
    """Owns one esrk_batch (many 2-D simulations advanced together)."""

    def __init__(self, cfgs):
        L = load()
        arr = (Config * len(cfgs))(*cfgs)
        h = C.c_void_p()
        _check(L.esrk_batch_create(arr, len(cfgs), C.byref(h)), "esrk_batch_create")
        self._h = h
        self.nsims = int(L.esrk_batch_num_sims(h))
        self.len = int(L.esrk_batch_state_len(h))
        self.nelems = int(L.esrk_batch_num_elems(h))
        self.offsets = [int(L.esrk_batch_offset(h, s)) for s in range(self.nsims)]
        self.elem_offsets = [int(L.esrk_batch_elem_offset(h, s)) for s in range(self.nsims)]

    @property
    def tile(self):
        return int(load().esrk_batch_tile(self._h))

    def close(self):
        if getattr(self, "_h", None):
            load().esrk_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, u, t, gamma=None, stream=None):
        _check(load().esrk_batch_step(self._h, _ptr(u), _ptr(t), _ptr(gamma), _stream(stream)),
               "esrk_batch_step")

    def autotune(self, u, reps=10, stream=None):
        tile = C.c_int(0)
        _check(load().esrk_batch_autotune(self._h, _ptr(u), int(reps), C.byref(tile),
                                          _stream(stream)), "esrk_batch_autotune")
        return tile.value

    def run_graph(self, u, t, nsteps, gamma=None, stream=None):
        _check(load().esrk_batch_run_graph(self._h, _ptr(u), _ptr(t), _ptr(gamma), int(nsteps),
                                           _stream(stream)), "esrk_batch_run_graph")

    def sync_status(self):
        bad = C.c_int64(-1)
        rc = load().esrk_batch_sync_status(self._h, C.byref(bad))
        return rc, bad.value


def mlp_forward(model, x_norm, y, stream=None):
    B = 0 if x_norm is None else x_norm.numel() // MLP_IN
    _check(load().esrk_mlp_forward(_ptr(model), _ptr(x_norm), B, _ptr(y), _stream(stream)),
           "esrk_mlp_forward")


def mlp_grad_work_size(B):
    return int(load().esrk_mlp_grad_work_size(int(B)))


def mlp_grad(model, x_norm, t_norm, grad, loss=None, work=None, stream=None):
    """work: device float buffer of mlp_grad_work_size(B) entries (allocated
    here with torch when not given)."""
    B = t_norm.numel()
    if work is None:
        import torch
        work = torch.empty(mlp_grad_work_size(B), dtype=torch.float32, device=model.device)
    elif not isinstance(work, int) and work.numel() < mlp_grad_work_size(B):
        raise ValueError("work buffer too small")
    _check(load().esrk_mlp_grad(_ptr(model), _ptr(x_norm), _ptr(t_norm), B, _ptr(grad),
                                _ptr(loss), _ptr(work), _stream(stream)), "esrk_mlp_grad")


def mlp_adam(model, grad, m, v, step, lr, stream=None):
    _check(load().esrk_mlp_adam(_ptr(model), _ptr(grad), _ptr(m), _ptr(v), int(step),
                                float(lr), _stream(stream)), "esrk_mlp_adam")


def mlp_prepare(model, raw, x_norm, gamma=None, t_norm=None, fit=False, stream=None):
    B = raw.numel() // MLP_IN
    _check(load().esrk_mlp_prepare(_ptr(model), _ptr(raw), _ptr(gamma), B, int(bool(fit)),
                                   _ptr(x_norm), _ptr(t_norm), _stream(stream)),
           "esrk_mlp_prepare")
