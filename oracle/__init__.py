"""ctypes front end of the CPU oracle (oracle/liboracle.so).

TEST INFRASTRUCTURE ONLY.  The oracle is the plain FP64 reference the HIP
path is checked against.  Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import it; the product package never does.

Arrays are numpy float64 in the layout u[v, element, node] flattened, see
``esrk_oracle.h``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "liboracle.so")

SSPRK33 = 0
RK44 = 1
BSRK43 = 2
BSRK85 = 3

ENOROOT = -4
ENONPHYS = -5


class Mesh(C.Structure):
    _fields_ = [
        ("dim", C.c_int),
        ("deg", C.c_int),
        ("nel", C.c_int * 3),
        ("lo", C.c_double * 3),
        ("hi", C.c_double * 3),
        ("gas_gamma", C.c_double),
        ("gas_r", C.c_double),
        ("mu", C.c_double),
        ("prandtl", C.c_double),
        ("lambda_scale", C.c_double),
        ("volume_flux", C.c_int),
        ("bc", C.c_int),
        ("ubc", C.c_double * 10),
        ("bckind", C.c_int * 2),
    ]


class RelaxOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("gamma_max", C.c_double), ("maxit", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from oracle import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        dp = C.POINTER(C.c_double)
        mp = C.POINTER(Mesh)
        L.orc_lgl.argtypes = [C.c_int, dp, dp]
        L.orc_dmat.argtypes = [C.c_int, dp]
        L.orc_logmean.argtypes = [C.c_double, C.c_double]
        L.orc_logmean.restype = C.c_double
        L.orc_entropy.argtypes = [C.c_int, C.c_double, dp]
        L.orc_entropy.restype = C.c_double
        L.orc_entropy_vars.argtypes = [C.c_int, C.c_double, dp, dp]
        L.orc_phys_flux.argtypes = [C.c_int, C.c_double, C.c_int, dp, dp]
        L.orc_ec_flux.argtypes = [C.c_int, C.c_double, C.c_int, dp, dp, dp]
        L.orc_wave_speed.argtypes = [C.c_int, C.c_double, dp]
        L.orc_wave_speed.restype = C.c_double
        L.orc_num_elems.argtypes = [mp]
        L.orc_num_elems.restype = C.c_long
        L.orc_num_nodes.argtypes = [mp]
        L.orc_num_nodes.restype = C.c_long
        L.orc_rhs.argtypes = [mp, dp, dp, dp, dp]
        L.orc_volume_term.argtypes = [mp, dp, dp]
        L.orc_interface_dissipation.argtypes = [mp, dp]
        L.orc_interface_dissipation.restype = C.c_double
        L.orc_br1_gradient.argtypes = [mp, dp, dp]
        L.orc_elem_entropy.argtypes = [mp, dp, dp]
        L.orc_cfl_dt.argtypes = [mp, dp, C.c_double]
        L.orc_cfl_dt.restype = C.c_double
        L.orc_tableau_stages.argtypes = [C.c_int]
        L.orc_rk_step.argtypes = [mp, C.c_int, dp, C.c_double, dp, dp, dp, dp, dp]
        L.orc_local_relaxation_solve.argtypes = [
            mp, C.POINTER(RelaxOpts), dp, dp, dp, dp, dp, dp, dp, dp,
            C.POINTER(C.c_int), C.POINTER(C.c_long)]
        L.orc_relax_r.argtypes = [mp, C.c_long, dp, dp, C.c_double, C.c_double,
                                  C.POINTER(C.c_int)]
        L.orc_relax_r.restype = C.c_longdouble
        L.orc_step.argtypes = [mp, C.c_int, C.POINTER(RelaxOpts), C.c_double, C.c_double,
                               dp, dp, dp, dp, dp, C.POINTER(C.c_long)]
        L.orc_global_relaxation_solve.argtypes = [mp, C.POINTER(RelaxOpts), dp, dp, dp, dp, dp,
                                                  dp, dp, C.POINTER(C.c_int)]
        L.orc_global_relax_r.argtypes = [mp, dp, dp, dp, C.c_double, C.POINTER(C.c_int)]
        L.orc_global_relax_r.restype = C.c_longdouble
        L.orc_mlp_forward.argtypes = [dp, dp, C.c_int, dp]
        L.orc_mlp_grad.argtypes = [dp, dp, dp, C.c_int, dp, dp]
        L.orc_mlp_adam.argtypes = [dp, dp, dp, dp, C.c_int, C.c_double]
        L.orc_mlp_prepare.argtypes = [dp, dp, dp, C.c_int, C.c_int, dp, dp]
        L.orc_elem_max_speed.argtypes = [mp, dp, dp]
        ip = C.POINTER(C.c_int)
        L.orc_tableau.argtypes = [C.c_int, dp, dp, dp, dp, ip, ip, ip]
        L.orc_rk_step_a.argtypes = [mp, C.c_int, dp, C.c_double, dp, dp, dp]
        L.orc_local_relaxation_solve_a.argtypes = [
            mp, C.POINTER(RelaxOpts), dp, dp, dp, dp, dp, dp, dp, dp, dp, ip,
            C.POINTER(C.c_long)]
        L.orc_global_relaxation_solve_a.argtypes = [mp, C.POINTER(RelaxOpts), dp, dp, dp, dp,
                                                    dp, dp, dp, dp, ip]
        L.orc_rk_step_err.argtypes = [mp, C.c_int, dp, C.c_double, dp, dp, dp]
        L.orc_error_norm.argtypes = [mp, dp, dp, dp, C.c_double, C.c_double]
        L.orc_error_norm.restype = C.c_double
        L.orc_adapt_factor.argtypes = [C.c_double, C.c_int, C.c_int]
        L.orc_adapt_factor.restype = C.c_double
        L.orc_adaptive_step.argtypes = [mp, C.c_int, C.POINTER(RelaxOpts), C.c_int,
                                        C.c_double, C.c_double, C.c_double, C.c_double, dp,
                                        dp, dp, dp, ip, dp, dp]
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def mesh(dim, deg, nel, lo, hi, gas_gamma=1.4, gas_r=1.0, mu=0.0, prandtl=0.72,
         lambda_scale=1.0, volume_flux=0, dirichlet=None, outflow=(False, False)) -> Mesh:
    """dirichlet = (u_left, u_right) conserved exterior states (1-D): Dirichlet
    boundaries at both ends instead of periodic ones.  outflow = (left, right):
    an end marked True takes its interior trace as the exterior state (its
    entry of dirichlet is then unused and may be None; outflow alone makes
    the mesh non-periodic)."""
    m = Mesh()
    m.dim, m.deg = dim, deg
    nel = list(nel) + [1] * (3 - len(nel))
    lo = list(lo) + [0.0] * (3 - len(lo))
    hi = list(hi) + [1.0] * (3 - len(hi))
    for q in range(3):
        m.nel[q], m.lo[q], m.hi[q] = nel[q], lo[q], hi[q]
    m.gas_gamma, m.gas_r, m.mu, m.prandtl = gas_gamma, gas_r, mu, prandtl
    m.lambda_scale, m.volume_flux = lambda_scale, volume_flux
    m.bc = 0
    if dirichlet is not None or any(outflow):
        m.bc = 1
        for s in range(2):
            m.bckind[s] = 1 if outflow[s] else 0
            if outflow[s]:
                continue
            st = list(dirichlet[s]) + [0.0] * (5 - len(dirichlet[s]))
            for v in range(5):
                m.ubc[5 * s + v] = float(st[v])
    return m


def relax_opts(tol=1e-15, gamma_max=4.0, maxit=200) -> RelaxOpts:
    o = RelaxOpts()
    o.tol, o.gamma_max, o.maxit = tol, gamma_max, maxit
    return o


def sizes(m: Mesh):
    return int(lib().orc_num_elems(C.byref(m))), int(lib().orc_num_nodes(C.byref(m)))


def lgl(deg):
    x = np.zeros(deg + 1)
    w = np.zeros(deg + 1)
    assert lib().orc_lgl(deg, _p(x), _p(w)) == 0
    return x, w


def dmat(deg):
    D = np.zeros((deg + 1) * (deg + 1))
    assert lib().orc_dmat(deg, _p(D)) == 0
    return D.reshape(deg + 1, deg + 1)


def logmean(a, b):
    return lib().orc_logmean(float(a), float(b))


def entropy(dim, gg, u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    return lib().orc_entropy(dim, gg, _p(u))


def entropy_vars(dim, gg, u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    w = np.zeros(dim + 2)
    lib().orc_entropy_vars(dim, gg, _p(u), _p(w))
    return w


def phys_flux(dim, gg, m, u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    f = np.zeros(dim + 2)
    lib().orc_phys_flux(dim, gg, m, _p(u), _p(f))
    return f


def ec_flux(dim, gg, m, uL, uR):
    uL = np.ascontiguousarray(uL, dtype=np.float64)
    uR = np.ascontiguousarray(uR, dtype=np.float64)
    f = np.zeros(dim + 2)
    lib().orc_ec_flux(dim, gg, m, _p(uL), _p(uR), _p(f))
    return f


def wave_speed(dim, gg, u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    return lib().orc_wave_speed(dim, gg, _p(u))


def rhs(m: Mesh, u, want_visc=False):
    ne, N = sizes(m)
    u = np.ascontiguousarray(u, dtype=np.float64)
    dudt = np.zeros_like(u)
    er = np.zeros(ne)
    vd = np.zeros(ne)
    rc = lib().orc_rhs(C.byref(m), _p(u), _p(dudt), _p(er), _p(vd))
    if rc != 0:
        raise RuntimeError(f"orc_rhs failed: {rc}")
    if want_visc:
        return dudt, er, vd
    return dudt, er


def volume_term(m: Mesh, u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    V = np.zeros_like(u)
    assert lib().orc_volume_term(C.byref(m), _p(u), _p(V)) == 0
    return V


def interface_dissipation(m: Mesh, u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    return lib().orc_interface_dissipation(C.byref(m), _p(u))


def br1_gradient(m: Mesh, u):
    ne, N = sizes(m)
    u = np.ascontiguousarray(u, dtype=np.float64)
    th = np.zeros(m.dim * (m.dim + 2) * N)
    assert lib().orc_br1_gradient(C.byref(m), _p(u), _p(th)) == 0
    return th


def elem_entropy(m: Mesh, u):
    ne, N = sizes(m)
    u = np.ascontiguousarray(u, dtype=np.float64)
    eta = np.zeros(ne)
    assert lib().orc_elem_entropy(C.byref(m), _p(u), _p(eta)) == 0
    return eta


def cfl_dt(m: Mesh, u, cfl):
    u = np.ascontiguousarray(u, dtype=np.float64)
    return lib().orc_cfl_dt(C.byref(m), _p(u), cfl)


def tableau_stages(tab):
    return int(lib().orc_tableau_stages(tab))


def rk_step(m: Mesh, tab, u_old, dt, want_stages=False):
    ne, N = sizes(m)
    s = tableau_stages(tab)
    u_old = np.ascontiguousarray(u_old, dtype=np.float64)
    du = np.zeros_like(u_old)
    deta = np.zeros(ne)
    ys = np.zeros((s,) + u_old.shape) if want_stages else None
    ks = np.zeros((s,) + u_old.shape) if want_stages else None
    es = np.zeros((s, ne)) if want_stages else None
    rc = lib().orc_rk_step(C.byref(m), tab, _p(u_old), float(dt), _p(du), _p(deta),
                           _p(ys), _p(ks), _p(es))
    if rc != 0:
        raise RuntimeError(f"orc_rk_step failed: {rc}")
    if want_stages:
        return du, deta, ys, ks, es
    return du, deta


def tableau(tab):
    """dict(A (s x s), b, bhat, c, s, p, q) of a Runge-Kutta method."""
    A = np.zeros(64)
    b, bh, c = np.zeros(8), np.zeros(8), np.zeros(8)
    s, p, q = C.c_int(), C.c_int(), C.c_int()
    assert lib().orc_tableau(tab, _p(A), _p(b), _p(bh), _p(c), C.byref(s), C.byref(p),
                             C.byref(q)) == 0
    n = s.value
    return dict(A=A.reshape(8, 8)[:n, :n].copy(), b=b[:n].copy(), bhat=bh[:n].copy(),
                c=c[:n].copy(), s=n, p=p.value, q=q.value)


def rk_step_a(m: Mesh, tab, u_old, dt):
    """(du, deta, a) with a_k = phi_k(0) from the stage-wise identity."""
    ne, N = sizes(m)
    u_old = np.ascontiguousarray(u_old, dtype=np.float64)
    du, deta, a = np.zeros_like(u_old), np.zeros(ne), np.zeros(ne)
    rc = lib().orc_rk_step_a(C.byref(m), tab, _p(u_old), float(dt), _p(du), _p(deta), _p(a))
    if rc != 0:
        raise RuntimeError(f"orc_rk_step_a failed: {rc}")
    return du, deta, a


def rk_step_err(m: Mesh, tab, u_old, dt):
    """(du, deta, err) with err = dt sum_i (b_i - bhat_i) k_i."""
    ne, N = sizes(m)
    u_old = np.ascontiguousarray(u_old, dtype=np.float64)
    du, err, deta = np.zeros_like(u_old), np.zeros_like(u_old), np.zeros(ne)
    rc = lib().orc_rk_step_err(C.byref(m), tab, _p(u_old), float(dt), _p(du), _p(deta),
                               _p(err))
    if rc != 0:
        raise RuntimeError(f"orc_rk_step_err failed: {rc}")
    return du, deta, err


def error_norm(m: Mesh, u_old, du, err, atol, rtol):
    return float(lib().orc_error_norm(C.byref(m), _p(np.ascontiguousarray(u_old)),
                                      _p(np.ascontiguousarray(du)),
                                      _p(np.ascontiguousarray(err)), atol, rtol))


def adapt_factor(err, q, accepted):
    return float(lib().orc_adapt_factor(float(err), int(q), int(bool(accepted))))


RELAX_LOCAL, RELAX_GLOBAL, RELAX_NONE = 0, 1, 2


def adaptive_step(m: Mesh, tab, u, t, dt=0.0, mode=RELAX_LOCAL, atol=1e-4, rtol=1e-4,
                  cfl=0.5, opts: RelaxOpts | None = None):
    """One error-controlled attempt, in place on u (numpy) if accepted.
    Returns dict(t, gamma, err, accepted, dt_next, dt, rc)."""
    opts = opts or relax_opts()
    assert u.dtype == np.float64 and u.flags["C_CONTIGUOUS"]
    tt, gam, en, dtn, dtu = (C.c_double(t), C.c_double(1.0), C.c_double(0.0),
                             C.c_double(0.0), C.c_double(0.0))
    acc = C.c_int(0)
    rc = lib().orc_adaptive_step(C.byref(m), tab, C.byref(opts), int(mode), float(atol),
                                 float(rtol), float(cfl), float(dt), _p(u), C.byref(tt),
                                 C.byref(gam), C.byref(en), C.byref(acc), C.byref(dtn),
                                 C.byref(dtu))
    return dict(t=tt.value, gamma=gam.value, err=en.value, accepted=bool(acc.value),
                dt_next=dtn.value, dt=dtu.value, rc=rc)


def local_relaxation_solve(m: Mesh, u_old, du, deta, opts: RelaxOpts | None = None, a=None):
    """Returns dict(gamma, gamma_k, phi0, curv, noise, iters, rc, bad_elem);
    a (optional, [ne]) supplies phi_k(0)."""
    ne, N = sizes(m)
    opts = opts or relax_opts()
    u_old = np.ascontiguousarray(u_old, dtype=np.float64)
    du = np.ascontiguousarray(du, dtype=np.float64)
    deta = np.ascontiguousarray(deta, dtype=np.float64)
    gk = np.zeros(ne)
    phi0 = np.zeros(ne)
    curv = np.zeros(ne)
    noise = np.zeros(ne)
    iters = np.zeros(ne, dtype=np.int32)
    gam = C.c_double(0.0)
    bad = C.c_long(-1)
    a = None if a is None else np.ascontiguousarray(a, dtype=np.float64)
    rc = lib().orc_local_relaxation_solve_a(
        C.byref(m), C.byref(opts), _p(u_old), _p(du), _p(deta), _p(a), _p(gk), C.byref(gam),
        _p(phi0), _p(curv), _p(noise), iters.ctypes.data_as(C.POINTER(C.c_int)),
        C.byref(bad))
    return dict(gamma=gam.value, gamma_k=gk, phi0=phi0, curv=curv, noise=noise,
                iters=iters, rc=rc, bad_elem=bad.value)


def relax_r(m: Mesh, k, u_old, du, deta_k, gamma):
    ok = C.c_int(1)
    u_old = np.ascontiguousarray(u_old, dtype=np.float64)
    du = np.ascontiguousarray(du, dtype=np.float64)
    r = lib().orc_relax_r(C.byref(m), k, _p(u_old), _p(du), float(deta_k), float(gamma),
                          C.byref(ok))
    return float(r), bool(ok.value)


def step(m: Mesh, tab, u, t, cfl=0.5, dt=0.0, opts: RelaxOpts | None = None):
    """In-place on u (numpy).  Returns dict(t, gamma, gamma_k, dt, rc, bad_elem)."""
    ne, N = sizes(m)
    opts = opts or relax_opts()
    assert u.dtype == np.float64 and u.flags["C_CONTIGUOUS"]
    tt = C.c_double(t)
    gam = C.c_double(0.0)
    dtu = C.c_double(0.0)
    gk = np.zeros(ne)
    bad = C.c_long(-1)
    rc = lib().orc_step(C.byref(m), tab, C.byref(opts), float(cfl), float(dt), _p(u),
                        C.byref(tt), C.byref(gam), _p(gk), C.byref(dtu), C.byref(bad))
    return dict(t=tt.value, gamma=gam.value, gamma_k=gk, dt=dtu.value, rc=rc,
                bad_elem=bad.value)


MLP_PARAMS = 1281


def mlp_forward(params, X):
    params = np.ascontiguousarray(params, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, 5)
    Y = np.zeros(X.shape[0])
    assert lib().orc_mlp_forward(_p(params), _p(X), X.shape[0], _p(Y)) == 0
    return Y


def mlp_grad(params, X, T):
    params = np.ascontiguousarray(params, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, 5)
    T = np.ascontiguousarray(T, dtype=np.float64)
    g = np.zeros(MLP_PARAMS)
    loss = C.c_double(0.0)
    assert lib().orc_mlp_grad(_p(params), _p(X), _p(T), X.shape[0], _p(g), C.byref(loss)) == 0
    return g, loss.value


MLP_MODEL = 1298


def mlp_adam(params, grad, m, v, step, lr):
    """In place on params, m, v (float64 arrays)."""
    for a in (params, grad, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    assert lib().orc_mlp_adam(_p(params), _p(grad), _p(m), _p(v), int(step), float(lr)) == 0


def mlp_prepare(model, raw, gamma=None, fit=False):
    """Returns (model', x_norm, t_norm or None); model' is a fitted copy."""
    model = np.array(model, dtype=np.float64)
    raw = np.ascontiguousarray(raw, dtype=np.float64).reshape(-1, 5)
    B = raw.shape[0]
    xn = np.zeros((B, 5))
    tn = None
    if gamma is not None:
        gamma = np.ascontiguousarray(gamma, dtype=np.float64)
        tn = np.zeros(B)
    assert lib().orc_mlp_prepare(_p(model), _p(raw), _p(gamma), B, int(bool(fit)), _p(xn),
                                 _p(tn)) == 0
    return model, xn, tn


def elem_max_speed(m: Mesh, u):
    ne = lib().orc_num_elems(C.byref(m))
    s = np.zeros(ne)
    assert lib().orc_elem_max_speed(C.byref(m), _p(np.ascontiguousarray(u)), _p(s)) == 0
    return s


def global_relaxation_solve(m: Mesh, u_old, du, deta, opts: RelaxOpts | None = None, a=None):
    """One global gamma (entropy equality); returns dict(gamma, phi0, curv, noise, iters, rc)."""
    opts = opts or relax_opts()
    u_old = np.ascontiguousarray(u_old, dtype=np.float64)
    du = np.ascontiguousarray(du, dtype=np.float64)
    deta = np.ascontiguousarray(deta, dtype=np.float64)
    g, p0, cu, no = C.c_double(), C.c_double(), C.c_double(), C.c_double()
    it = C.c_int(0)
    a = None if a is None else np.ascontiguousarray(a, dtype=np.float64)
    rc = lib().orc_global_relaxation_solve_a(C.byref(m), C.byref(opts), _p(u_old), _p(du),
                                             _p(deta), _p(a), C.byref(g), C.byref(p0),
                                             C.byref(cu), C.byref(no), C.byref(it))
    return dict(gamma=g.value, phi0=p0.value, curv=cu.value, noise=no.value, iters=it.value,
                rc=rc)


def global_relax_r(m: Mesh, u_old, du, deta, gamma):
    ok = C.c_int(1)
    r = lib().orc_global_relax_r(C.byref(m), _p(np.ascontiguousarray(u_old)),
                                 _p(np.ascontiguousarray(du)), _p(np.ascontiguousarray(deta)),
                                 float(gamma), C.byref(ok))
    return float(r), bool(ok.value)
