"""Pins of the oracle's Runge-Kutta tableaux, embedded error estimates and
error-controlled steps (CPU).

Fixed by: the order conditions of every rooted tree (enumerated here from
their recursive definition, independent of the oracle), the published node
vectors, the measured order of one step and of the error estimate on the
isentropic vortex, the estimate against the true error of the embedded
solution, the controller's step-count law steps ~ tol^(-1/(q+1)), and the
entropy statements of the relaxation modes on accepted steps.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

from paper_2003_08831_amd import inputs as I
from tests.oracle_helpers import orc_mesh

TABS = ["SSPRK33", "RK44", "BSRK43", "BSRK85"]


def rooted_trees(nmax):
    """All rooted trees up to nmax nodes, each a sorted tuple of subtrees."""
    by_order = {1: [()]}
    flat = [((), 1)]
    for n in range(2, nmax + 1):
        out = set()

        def forests(total, start, acc):
            if total == 0:
                out.add(tuple(sorted(acc)))
                return
            for idx in range(start, len(flat)):
                t, o = flat[idx]
                if o <= total:
                    forests(total - o, idx, acc + [t])

        forests(n - 1, 0, [])
        by_order[n] = sorted(out)
        flat += [(t, n) for t in by_order[n]]
    return by_order


def order_of(t):
    return 1 + sum(order_of(c) for c in t)


def density(t):
    return order_of(t) * math.prod(density(c) for c in t)


def stage_weights(A, t):
    """g(t) = elementwise product over the children c of A g(c); g(leaf) = 1."""
    g = np.ones(A.shape[0])
    for c in t:
        g = g * (A @ stage_weights(A, c))
    return g


def order_residuals(A, b, n):
    return [abs(b @ stage_weights(A, t) - 1.0 / density(t)) for t in rooted_trees(n)[n]]


def test_tree_enumeration_counts():
    # numbers of rooted trees with 1..7 nodes
    trees = rooted_trees(7)
    assert [len(trees[n]) for n in range(1, 8)] == [1, 1, 2, 4, 9, 20, 48]


@pytest.mark.parametrize("name", TABS)
def test_order_conditions(orc, name):
    T = orc.tableau(getattr(orc, name))
    A, b, bh, p, q = T["A"], T["b"], T["bhat"], T["p"], T["q"]
    assert np.all(np.triu(A) == 0.0)  # explicit
    assert np.all(b >= 0.0)  # the entropy estimate needs b_i >= 0
    for n in range(1, p + 1):
        assert max(order_residuals(A, b, n)) <= 1e-14, (name, n)
    assert max(order_residuals(A, b, p + 1)) > 1e-6  # not of order p + 1
    if q:
        for n in range(1, q + 1):
            assert max(order_residuals(A, bh, n)) <= 1e-14, (name, "embedded", n)
        assert max(order_residuals(A, bh, q + 1)) > 1e-6


def test_published_nodes_and_fsal(orc):
    F = Fraction
    c_bs3 = [F(0), F(1, 2), F(3, 4), F(1)]
    c_bs5 = [F(0), F(1, 6), F(2, 9), F(3, 7), F(2, 3), F(3, 4), F(1), F(1)]
    for name, cref in (("BSRK43", c_bs3), ("BSRK85", c_bs5)):
        T = orc.tableau(getattr(orc, name))
        np.testing.assert_allclose(T["c"], [float(x) for x in cref], rtol=0, atol=1e-15)
        # the last stage is evaluated at the higher-order solution, with zero weight
        np.testing.assert_allclose(T["A"][-1, :-1], T["b"][:-1], rtol=0, atol=0)
        assert T["b"][-1] == 0.0 and T["bhat"][-1] != 0.0


def _vortex(orc, nel=4, deg=3):
    ms = I.vortex_mesh(nel, deg)
    return ms, orc_mesh(orc, ms), I.vortex_state(ms)


def _reference(orc, m, u, dt, sub=64):
    """RK(4,4) with dt/sub substeps: a solution of the same semidiscrete ODE far
    more accurate than one step of any tableau here at dt."""
    y = u.copy()
    for _ in range(sub):
        du, _ = orc.rk_step(m, orc.RK44, y, dt / sub)
        y = y + du
    return y


@pytest.mark.parametrize("name", TABS)
def test_measured_step_order(orc, name):
    """Local error of one step ~ dt^(p+1); for the embedded pairs the estimate
    ~ dt^(q+1) and equals the true error of the embedded solution to leading
    order."""
    tab = getattr(orc, name)
    T = orc.tableau(tab)
    ms, m, u = _vortex(orc)
    # well inside the stability region (the CFL step is ~0.048 here): the
    # rates are asymptotic only for dt lambda << 1
    dt0 = orc.cfl_dt(m, u, 0.5)
    dts = [dt0 / 4, dt0 / 8]
    errs, ests, emb = [], [], []
    for dt in dts:
        ref = _reference(orc, m, u, dt)
        if T["q"]:
            du, _, e = orc.rk_step_err(m, tab, u, dt)
            ests.append(np.abs(e).max())
            emb.append(np.abs((u + du - e) - ref).max() / np.abs(e).max())
        else:
            du, _ = orc.rk_step(m, tab, u, dt)
        errs.append(np.abs(u + du - ref).max())
    rate = math.log2(errs[0] / errs[1])
    assert abs(rate - (T["p"] + 1)) <= 0.4, (name, rate, errs)
    if T["q"]:
        est_rate = math.log2(ests[0] / ests[1])
        assert abs(est_rate - (T["q"] + 1)) <= 0.4, (name, est_rate)
        # |true error of the embedded solution| / |estimate| -> 1, the
        # deviation (the higher-order solution's own error) shrinking ~ dt
        assert abs(emb[1] - 1.0) <= 0.25, (name, emb)
        if abs(emb[0] - 1.0) > 0.05:
            assert abs(emb[1] - 1.0) <= 0.7 * abs(emb[0] - 1.0), (name, emb)


def test_controller_factor_properties(orc):
    """err = 1 is accepted with the safety factor; smaller errors give larger
    steps up to the clip; the factor follows err^(-1/(q+1)) between the clips."""
    assert orc.adapt_factor(1.0, 2, True) == pytest.approx(0.9, rel=1e-15)
    assert orc.adapt_factor(0.0, 4, True) == 10.0
    assert orc.adapt_factor(1e30, 4, False) == 0.1
    f1, f2 = orc.adapt_factor(0.5, 2, True), orc.adapt_factor(0.5 / 8, 2, True)
    assert f2 / f1 == pytest.approx(2.0, rel=1e-14)  # 8^(1/3)
    assert orc.adapt_factor(2.0, 2, False) < orc.adapt_factor(2.0, 2, True)


def _adaptive_run(orc, m, u0, tab, tol, t_end, mode, max_attempts=4000):
    u, t, dt = u0.copy(), 0.0, 0.0
    acc = rej = 0
    hist = []
    while t < t_end - 1e-12 and acc + rej < max_attempts:
        if dt > 0.0:
            dt = min(dt, t_end - t)
        u_before = u.copy()
        r = orc.adaptive_step(m, tab, u, t, dt=dt, mode=mode, atol=tol, rtol=tol)
        assert r["rc"] == 0
        if r["accepted"]:
            acc += 1
            hist.append((u_before, r))
        else:
            rej += 1
            assert np.array_equal(u, u_before) and r["t"] == t
        t, dt = r["t"], r["dt_next"]
    return u, t, acc, rej, hist


def test_step_count_follows_tolerance(orc):
    """Error-controlled BSRK(4,3) over a fixed time: accepted steps scale as
    tol^(-1/(q+1)) = 10^(1/3) per decade, and the error against a fine
    reference shrinks with the tolerance."""
    ms, m, u0 = _vortex(orc)
    t_end = 2.0
    runs = {}
    # tolerances tight enough that accuracy, not stability, limits the step
    # (at 1e-4 the steps sit at the stability limit and get rejected there)
    for tol in (1e-6, 1e-7):
        u, t, acc, rej, _ = _adaptive_run(orc, m, u0, orc.BSRK43, tol, t_end,
                                          orc.RELAX_NONE)
        assert abs(t - t_end) <= 1e-12
        runs[tol] = (u, acc, rej)
    ratio = runs[1e-7][1] / runs[1e-6][1]
    assert 1.6 <= ratio <= 2.9, ratio
    ref = u0.copy()
    for _ in range(200):
        du, _ = orc.rk_step(m, orc.RK44, ref, t_end / 200)
        ref = ref + du
    e6, e7 = (np.abs(runs[tol][0] - ref).max() for tol in (1e-6, 1e-7))
    assert e7 < e6


@pytest.mark.parametrize("mode", ["RELAX_LOCAL", "RELAX_GLOBAL"])
def test_adaptive_relaxed_entropy(orc, mode):
    """Error-controlled BSRK(4,3) with an entropy-conservative surface flux:
    on every accepted step the local mode keeps each element's inequality
    eta_k(u_gamma) <= eta_k(u_old) + gamma deta_k, and the global mode keeps the
    total entropy to round-off."""
    ms = I.vortex_mesh(4, 3)
    m = orc_mesh(orc, ms, lambda_scale=0.0)
    u0 = I.vortex_state(ms)
    u, t, acc, rej, hist = _adaptive_run(orc, m, u0, orc.BSRK43, 1e-4, 1.0,
                                         getattr(orc, mode))
    assert acc >= 3
    eta0 = orc.elem_entropy(m, u0)
    sc = np.abs(eta0).sum()
    for u_old, r in hist:
        dt = r["dt"]
        du, deta, _ = orc.rk_step_err(m, orc.BSRK43, u_old, dt)
        u_new = u_old + r["gamma"] * du
        e_old, e_new = orc.elem_entropy(m, u_old), orc.elem_entropy(m, u_new)
        if mode == "RELAX_LOCAL":
            assert np.all(e_new <= e_old + r["gamma"] * deta + 64 * np.finfo(float).eps * sc)
        else:
            assert abs(e_new.sum() - e_old.sum()) <= 1e-13 * sc
    if mode == "RELAX_GLOBAL":
        assert abs(orc.elem_entropy(m, u).sum() - eta0.sum()) <= 1e-12 * sc
