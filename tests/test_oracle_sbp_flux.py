"""Pins of the oracle's SBP operators and pointwise fluxes (CPU only).

Each check is fixed by something other than the oracle's own formula: a
textbook matrix, numpy's Legendre routines, an exact quadrature, a calculus
identity or Tadmor's entropy-conservation condition.
"""
import json
import os

import numpy as np
import pytest

from paper_2003_08831_amd import inputs as I

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("deg", range(1, 8))
def test_lgl_nodes_match_numpy_legendre(orc, deg):
    x, w = orc.lgl(deg)
    np.testing.assert_allclose(x, I.lobatto_points(deg), atol=2e-15)


@pytest.mark.parametrize("deg", range(1, 8))
def test_sbp_property_and_quadrature(orc, deg):
    x, w = orc.lgl(deg)
    D = orc.dmat(deg)
    n = deg + 1
    Q = np.diag(w) @ D
    B = np.zeros((n, n))
    B[0, 0], B[-1, -1] = -1.0, 1.0
    assert np.abs(Q + Q.T - B).max() <= 5e-15
    # Lobatto quadrature is exact for degree <= 2p-1
    for k in range(2 * deg):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(w @ x ** k - exact) <= 5e-15
    # D differentiates polynomials of degree <= p exactly
    for k in range(deg + 1):
        d = k * x ** (k - 1) if k else np.zeros(n)
        np.testing.assert_allclose(D @ x ** k, d, atol=5e-13)
    np.testing.assert_allclose(D.sum(axis=1), 0.0, atol=1e-14)


def test_textbook_sbp_operators(orc):
    with open(os.path.join(GOLD, "sbp_textbook.json")) as f:
        gold = json.load(f)
    for case in gold["cases"]:
        deg = case["deg"]
        x, w = orc.lgl(deg)
        np.testing.assert_allclose(x, case["x"], atol=1e-15)
        np.testing.assert_allclose(w, case["w"], atol=1e-15)
        np.testing.assert_allclose(orc.dmat(deg), case["D"], atol=1e-14)


def _state(dim, gg, rho, v, p):
    return np.array([rho] + [rho * vi for vi in v]
                    + [p / (gg - 1) + 0.5 * rho * sum(vi * vi for vi in v)])


def _rand_states(dim, n, seed, gg=1.4):
    rng = np.random.Generator(np.random.PCG64(seed))
    for _ in range(n):
        yield _state(dim, gg, rng.uniform(0.2, 3.0), rng.uniform(-2, 2, dim),
                     rng.uniform(0.2, 3.0))


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_entropy_identities(orc, dim):
    gg = 1.4
    for u in _rand_states(dim, 200, 7 + dim):
        S = orc.entropy(dim, gg, u)
        w = orc.entropy_vars(dim, gg, u)
        # w.u - S = rho for S = -rho s/(gg-1)
        assert abs(w @ u - S - u[0]) <= 1e-13 * (abs(S) + abs(w @ u))
        # w = dS/du (central differences)
        for v in range(dim + 2):
            h = 1e-6 * max(1.0, abs(u[v]))
            e = np.zeros(dim + 2)
            e[v] = h
            fd = (orc.entropy(dim, gg, u + e) - orc.entropy(dim, gg, u - e)) / (2 * h)
            assert abs(fd - w[v]) <= 1e-7 * max(1.0, abs(w[v]))


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_physical_flux_special_states(orc, dim):
    gg = 1.4
    # fluid at rest: only the pressure acts, on the normal momentum
    u = _state(dim, gg, 1.3, [0.0] * dim, 0.7)
    for m in range(dim):
        f = orc.phys_flux(dim, gg, m, u)
        expect = np.zeros(dim + 2)
        expect[1 + m] = 0.7
        np.testing.assert_allclose(f, expect, atol=1e-15)
    # Galilean: uniform translation with velocity c in x carries u, plus p terms
    c = 0.8
    u = _state(dim, gg, 2.0, [c] + [0.0] * (dim - 1), 1.5)
    f = orc.phys_flux(dim, gg, 0, u)
    expect = c * u
    expect[1] += 1.5
    expect[-1] += 1.5 * c
    np.testing.assert_allclose(f, expect, rtol=1e-15)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_ec_flux_consistency_symmetry_tadmor(orc, dim):
    gg = 1.4
    rng = np.random.Generator(np.random.PCG64(11))
    states = list(_rand_states(dim, 400, 3 * dim))
    worst = 0.0
    for q in range(0, len(states), 2):
        uL = states[q]
        uR = states[q + 1] if q % 4 else uL * (1.0 + 1e-7 * rng.uniform(-1, 1, dim + 2))
        wL, wR = orc.entropy_vars(dim, gg, uL), orc.entropy_vars(dim, gg, uR)
        for m in range(dim):
            f = orc.ec_flux(dim, gg, m, uL, uR)
            np.testing.assert_allclose(f, orc.ec_flux(dim, gg, m, uR, uL), rtol=1e-14,
                                       atol=1e-15)
            np.testing.assert_allclose(orc.ec_flux(dim, gg, m, uL, uL),
                                       orc.phys_flux(dim, gg, m, uL), rtol=1e-14,
                                       atol=1e-14)
            # Tadmor: (w_R - w_L).f# = psi_R - psi_L, psi_m = rho v_m
            res = (wR - wL) @ f - (uR[1 + m] - uL[1 + m])
            scale = np.abs((wR - wL) * f).sum() + abs(uR[1 + m]) + abs(uL[1 + m])
            worst = max(worst, abs(res) / scale)
    assert worst <= 2e-14


def test_logmean(orc):
    rng = np.random.Generator(np.random.PCG64(5))
    # separated arguments: the definition (a-b)/(ln a - ln b) in extended precision
    for _ in range(500):
        a, b = rng.uniform(0.01, 100.0, 2)
        if abs(a / b - 1) < 0.1:
            continue
        la, lb = np.longdouble(a), np.longdouble(b)
        ref = (la - lb) / (np.log(la) - np.log(lb))
        assert abs(orc.logmean(a, b) - float(ref)) <= 2e-15 * float(ref)
    # equal arguments and the small-jump expansion of a h / ln(1+h)
    assert orc.logmean(3.0, 3.0) == 3.0
    for h0 in [1e-3, 1e-5, 1e-8, 1e-12]:
        a = 2.5
        b = a * (1 + h0)
        h = (np.longdouble(b) - np.longdouble(a)) / np.longdouble(a)  # the jump actually stored
        ref = float(np.longdouble(a) * (1 + h / 2 - h * h / 12 + h ** 3 / 24 - 19 * h ** 4 / 720))
        assert abs(orc.logmean(b, a) - ref) <= 4e-16 * a
