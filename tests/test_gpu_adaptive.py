"""GPU embedded pairs and error-controlled steps against the oracle:
BSRK(4,3) and BSRK(8,5) stage chains (stage states, increments, entropy
estimates and error estimates), whole steps without error control (the
zero-weight last stage skipped on the device), and sequences of
error-controlled attempts in the three relaxation modes (accept decisions,
error norms, step sizes and states)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_2003_08831_amd import esrk  # noqa: E402
from paper_2003_08831_amd import inputs as I  # noqa: E402
from tests.gpu_helpers import ctx_for, dev, host, rhs_close, term_scale, zeros  # noqa: E402
from tests.oracle_helpers import orc_mesh  # noqa: E402
from tests.test_gpu_parity import CASES, make_state  # noqa: E402

pytestmark = pytest.mark.gpu

PAIRS = [(esrk.BSRK43, O.BSRK43), (esrk.BSRK85, O.BSRK85)]
PAIR_IDS = ["bsrk43", "bsrk85"]


@pytest.mark.parametrize("tab,otab", PAIRS, ids=PAIR_IDS)
@pytest.mark.parametrize("name,ms,kind", [CASES[0], CASES[2], CASES[4], CASES[8]],
                         ids=["d1p3", "d2p3_vortex", "d2p4", "d3p3_rand"])
def test_pair_stage_chain_parity(tab, otab, name, ms, kind):
    u = make_state(ms, kind, seed=2)
    m = orc_mesh(O, ms)
    dt = 0.5 * O.cfl_dt(m, u, 0.5)
    du_ref, deta_ref, ys, ks, es = O.rk_step(m, otab, u, dt, want_stages=True)
    _, _, err_ref = O.rk_step_err(m, otab, u, dt)
    T = O.tableau(otab)
    S = term_scale(O, ms, u)
    ctx = ctx_for(ms, tableau=tab)
    ctx.set_adaptive(1e-5, 1e-5)
    ud = dev(u)
    bufs = [zeros(u.size), zeros(u.size)]
    du, deta = zeros(u.size), zeros(ctx.ne)
    yin = ud
    s = T["s"]
    for i in range(s):
        yout = bufs[i % 2] if i < s - 1 else None
        ctx.rk_stage(i, dt, ud, yin, yout, du, deta)
        if yout is not None:
            # y_{i+1} = u + dt sum_j a_{i+1,j} k_j: the k errors enter scaled by
            # dt sum_j |a_{i+1,j}|
            w = np.abs(T["A"][i + 1]).sum()
            assert rhs_close(host(yout), ys[i + 1], ms, dt * w * S) <= 1.0, i
        yin = yout
    assert rhs_close(host(du), du_ref, ms, dt * S, rel=1e-11) <= 1.0
    assert np.abs(host(deta) - deta_ref).max() <= 1e-11 * np.abs(deta_ref).max()
    err, norm = zeros(u.size), zeros(1)
    ctx.error_estimate(err, norm)
    we = np.abs(T["b"] - T["bhat"]).sum()
    assert rhs_close(host(err), err_ref, ms, dt * we * S, rel=1e-10) <= 1.0
    n_ref = O.error_norm(m, u, du_ref, err_ref, 1e-5, 1e-5)
    # the estimate is a cancelling sum: its absolute error bound (the one
    # checked above) over the smallest weight atol bounds the norm's error
    e3 = err_ref.reshape(ms.nv, -1)
    eabs = max(1e-10 * np.abs(e3[v]).max() + 1e-14 * dt * we * S[v] for v in range(ms.nv))
    assert abs(host(norm)[0] - n_ref) <= 1e-8 * n_ref + eabs / 1e-5
    assert ctx.sync_status()[0] == 0


@pytest.mark.parametrize("tab,otab", PAIRS, ids=PAIR_IDS)
@pytest.mark.parametrize("name,ms,kind", [CASES[2], CASES[7]], ids=["d2p3_vortex", "d3p3_tgv"])
def test_pair_step_parity_without_error_control(tab, otab, name, ms, kind):
    """Locally relaxed steps; the device skips the zero-weight last stage, the
    oracle evaluates it (its weight is exactly zero, so nothing changes)."""
    u = make_state(ms, kind, seed=4)
    m = orc_mesh(O, ms)
    ctx = ctx_for(ms, tableau=tab, cfl=0.5)
    stats = zeros(8)
    t_ref = 0.0
    for step in range(3):
        ud, t = dev(u), dev(np.array([t_ref]))
        dt = O.cfl_dt(m, u, 0.5)
        du, deta = O.rk_step(m, otab, u, dt)
        ref = O.local_relaxation_solve(m, u, du, deta)
        assert ref["rc"] == 0
        fin = np.isfinite(ref["gamma_k"])
        k = np.argmin(np.where(fin, ref["gamma_k"], np.inf))
        g = ref["gamma"]
        gtol = 2e-12 * max(1.0, g) + (ref["noise"][k] / ref["curv"][k] if fin.any() else 0.0)
        ctx.step(ud, t, 0.0, None, stats)
        st = host(stats)
        assert abs(st[1] - dt) <= 1e-14 * dt
        assert abs(st[0] - g) <= gtol
        assert st[6] == 0.0 and st[7] == 1.0
        got = host(ud).reshape(ms.nv, -1)
        u_next = u + g * du
        for v in range(ms.nv):
            r = u_next.reshape(ms.nv, -1)[v]
            tolv = 1e-12 * np.abs(r).max() + gtol * np.abs(du.reshape(ms.nv, -1)[v]).max()
            assert np.abs(got[v] - r).max() <= tolv, (step, v)
        u, t_ref = u_next, t_ref + g * dt
    assert ctx.sync_status()[0] == 0


def _mode_gamma_tol(m, u, du, deta, mode):
    if mode == O.RELAX_NONE:
        return 0.0
    if mode == O.RELAX_GLOBAL:
        ref = O.global_relaxation_solve(m, u, du, deta)
        return 2e-12 * max(1.0, ref["gamma"]) + (ref["noise"] / ref["curv"]
                                                  if ref["curv"] > 0 else 0.0)
    ref = O.local_relaxation_solve(m, u, du, deta)
    fin = np.isfinite(ref["gamma_k"])
    if not fin.any():
        return 0.0
    k = np.argmin(np.where(fin, ref["gamma_k"], np.inf))
    return 2e-12 * max(1.0, ref["gamma"]) + ref["noise"][k] / ref["curv"][k]


@pytest.mark.parametrize("tab,otab", PAIRS, ids=PAIR_IDS)
@pytest.mark.parametrize("mode", [esrk.RELAX_LOCAL, esrk.RELAX_GLOBAL, esrk.RELAX_NONE],
                         ids=["local", "global", "none"])
def test_error_controlled_attempts_parity(tab, otab, mode):
    """Ten error-controlled attempts on the 2-D vortex (8x8, p=3) with the
    device's own step sizes (the CFL rule first, then its proposals): the
    oracle repeats each attempt from the same state with the device's step and
    must agree on the accept decision, error norm, relaxation parameter, state
    and time; the device's next step must equal the oracle's proposal.  The
    first attempt (CFL number 1, tolerance 1e-6) is rejected."""
    ms = I.vortex_mesh(8, 3)
    m = orc_mesh(O, ms)
    u = I.vortex_state(ms)
    tol, cfl = 1e-6, 1.0
    T = O.tableau(otab)
    we = np.abs(T["b"] - T["bhat"]).sum()
    S = term_scale(O, ms, u)
    ctx = ctx_for(ms, tableau=tab, cfl=cfl)
    ctx.set_relaxation_mode(mode)
    ctx.set_adaptive(tol, tol)
    stats = zeros(8)
    ud, t = dev(u), zeros(1)
    t_ref, prev = 0.0, None
    n_rej = 0
    for attempt in range(10):
        u_before = u.copy()
        ctx.step(ud, t, 0.0, None, stats)
        st = host(stats)
        dt = st[1]
        if prev is None:
            assert abs(dt - O.cfl_dt(m, u, cfl)) <= 1e-14 * dt
        else:
            # err agrees to ~1e-10 relative, the proposal through err^(-1/(q+1))
            assert abs(dt - prev["dt_next"]) <= 1e-9 * dt, attempt
        r = O.adaptive_step(m, otab, u, t_ref, dt=dt, mode=mode, atol=tol, rtol=tol, cfl=cfl)
        assert r["rc"] == 0
        if abs(r["err"] - 1.0) > 1e-5:
            assert bool(st[7]) == r["accepted"], attempt
        du, deta, e_ref = O.rk_step_err(m, otab, u_before, dt)
        e3 = e_ref.reshape(ms.nv, -1)
        eabs = max(1e-10 * np.abs(e3[v]).max() + 1e-14 * dt * we * S[v] for v in range(ms.nv))
        assert abs(st[6] - r["err"]) <= 1e-8 * r["err"] + eabs / tol, (attempt, st[6], r["err"])
        gtol = _mode_gamma_tol(m, u_before, du, deta, mode) if r["accepted"] else 0.0
        if r["accepted"]:
            assert abs(st[0] - r["gamma"]) <= gtol, attempt
        else:
            n_rej += 1
            assert st[0] == 1.0
        got = host(ud).reshape(ms.nv, -1)
        ref = u.reshape(ms.nv, -1)
        for v in range(ms.nv):
            tolv = 1e-12 * np.abs(ref[v]).max() + gtol * np.abs(du.reshape(ms.nv, -1)[v]).max()
            assert np.abs(got[v] - ref[v]).max() <= tolv, (attempt, v)
        assert abs(host(t)[0] - r["t"]) <= 1e-13 * r["t"] + gtol * dt
        # both continue from the oracle's state
        t_ref, prev = r["t"], r
        ud.copy_(dev(u))
        t.fill_(t_ref)
    print(f"[adaptive {PAIR_IDS[tab - 2]} mode {mode}] rejections {n_rej}")
    assert n_rej >= 1
    assert ctx.sync_status()[0] == 0


@pytest.mark.parametrize("tab,otab", [(esrk.RK44, O.RK44), (esrk.BSRK85, O.BSRK85)],
                         ids=["rk44", "bsrk85"])
@pytest.mark.parametrize("name,ms,kind", [CASES[2], CASES[7], CASES[9]],
                         ids=["d2p3_vortex", "d3p3_tgv", "d3p4"])
def test_step_roots_from_stagewise_phi0(tab, otab, name, ms, kind):
    """The step solves with phi_k(0) accumulated by the stages: every
    element's root against the oracle's roots from its own stage-wise phi_k(0),
    to a bound a thousand times tighter than the difference form allows
    (the oracle's extended-precision level, 2^-11 of the FP64 one, plus the
    root tolerance)."""
    u = make_state(ms, kind, seed=5)
    m = orc_mesh(O, ms)
    ctx = ctx_for(ms, tableau=tab, cfl=0.5)
    dt = O.cfl_dt(m, u, 0.5)
    du, deta, a = O.rk_step_a(m, otab, u, dt)
    ref = O.local_relaxation_solve(m, u, du, deta, a=a)
    assert ref["rc"] == 0
    gk, stats = zeros(ctx.ne), zeros(8)
    ctx.step(dev(u), dev(np.array([0.0])), dt, gk, stats)
    g = host(gk)
    g_ref = ref["gamma_k"]
    fin = np.isfinite(g_ref)
    borderline = (ref["curv"] > 0.5 * ref["noise"]) & (ref["curv"] < 2.0 * ref["noise"])
    assert np.array_equal(fin[~borderline], np.isfinite(g)[~borderline])
    both = fin & np.isfinite(g) & ~borderline
    # the two sides evaluate the right-hand side with different rounding: the
    # slopes differ by ~1e-14 of the term scale S, which in a quiet element is
    # a relative change rho_k of its increments, and gamma_k = -phi(0)/B'' moves
    # by ~4 rho_k gamma_k (phi(0) and B both quadratic in the increments)
    S = term_scale(O, ms, u)
    d3 = np.abs(du.reshape(ms.nv, ms.ne, ms.nd)).max(axis=2)  # [v, k]
    rho_k = (1e-14 * dt * S[:, None] / np.maximum(d3, 1e-300)).min(axis=0)
    tol = (2e-12 * np.maximum(1.0, g_ref[both]) + 1e-3 * ref["noise"][both] / ref["curv"][both]
           + 8.0 * rho_k[both] * g_ref[both])
    err = np.abs(g[both] - g_ref[both])
    w = np.argmax(err / tol)
    print(f"[stage-wise phi0 {name}] active {both.sum()} max |dgamma| {err.max():.2e} "
          f"bound of the difference form {(ref['noise'][both] / ref['curv'][both]).max():.2e}; "
          f"worst element: err {err[w]:.2e} tol {tol[w]:.2e} rho {rho_k[both][w]:.2e}")
    assert np.all(err <= tol), (err.max(), tol[np.argmax(err - tol)])
    assert ctx.sync_status()[0] == 0
