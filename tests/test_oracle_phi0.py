"""Pins of the oracle's stage-wise evaluation of phi_k(0) (CPU).

phi_k(0) = sum_i M w(u_old).du - deta_k is, by the definition of the RK
entropy estimate, equal to dt sum_i b_i sum_nodes M (w(u_old) - w(y^i)).k_i.
Fixed by: agreement with the difference form within that form's round-off
level, the leading-order closed form -dt^2/2 sum M f.(dw/du f) (from
sum_i b_i c_i = 1/2), the same closed form for perturbations of a uniform
state down to amplitudes where the difference form has lost its digits, and
the relaxation roots computed from it.
"""
import numpy as np
import pytest

from paper_2003_08831_amd import inputs as I
from tests.oracle_helpers import node_mass, orc_mesh


@pytest.mark.parametrize("tab", ["SSPRK33", "RK44", "BSRK43", "BSRK85"])
def test_stagewise_phi0_matches_difference_form(orc, tab):
    ms = I.MeshSpec(dim=2, deg=3, nel=(3, 3, 1), lo=(0, 0, 0), hi=(1, 1, 1))
    m = orc_mesh(orc, ms)
    u = I.random_state(ms, seed=5, smooth=True, rel=0.2, vmax=0.3)
    t = getattr(orc, tab)
    dt = orc.cfl_dt(m, u, 0.5)
    du, deta, a = orc.rk_step_a(m, t, u, dt)
    ref = orc.local_relaxation_solve(m, u, du, deta)
    assert np.all(np.abs(a - ref["phi0"]) <= ref["noise"]), np.abs(a - ref["phi0"]) / ref["noise"]
    assert np.all(a < 0.0)


def _jac_times(orc, ms, u, f, h=1e-6):
    """(dw/du) f per node by central differences of the entropy variables."""
    U = np.asarray(u).reshape(ms.nv, -1)
    F = np.asarray(f).reshape(ms.nv, -1)
    out = np.zeros_like(U)
    for n in range(U.shape[1]):
        wp = np.array(orc.entropy_vars(ms.dim, ms.gas_gamma, U[:, n] + h * F[:, n]))
        wm = np.array(orc.entropy_vars(ms.dim, ms.gas_gamma, U[:, n] - h * F[:, n]))
        out[:, n] = (wp - wm) / (2 * h)
    return out


def test_stagewise_phi0_leading_order_closed_form(orc):
    """phi_k(0) = -dt^2/2 sum_nodes M f.(dw/du) f + O(dt^3) for any RK method
    of order >= 2 (k_i = f + O(dt), y^i - u = c_i dt f + O(dt^2))."""
    ms = I.vortex_mesh(4, 3)
    m = orc_mesh(orc, ms)
    u = I.vortex_state(ms)
    f = orc.rhs(m, u)[0]
    Jf = _jac_times(orc, ms, u, f)
    F = f.reshape(ms.nv, -1)
    M = node_mass(orc, ms).reshape(-1)
    q = (F * Jf).sum(axis=0) * np.tile(M, ms.ne)
    lead = -0.5 * q.reshape(ms.ne, ms.nd).sum(axis=1)
    big = np.abs(lead) > 1e-3 * np.abs(lead).max()
    for tab in (orc.RK44, orc.BSRK85):
        devs = []
        for dt in (1e-3, 5e-4):
            _, _, a = orc.rk_step_a(m, tab, u, dt)
            devs.append(np.abs(a[big] / dt ** 2 / lead[big] - 1.0).max())
        assert devs[1] < 2e-3 and devs[1] < 0.7 * devs[0], devs  # -> 0 like dt


def test_stagewise_phi0_keeps_its_digits_near_uniform_flow(orc):
    """u = uniform + s * smooth perturbation, s from 1e-4 down to 1e-11: the
    stage-wise phi_k(0) keeps the same relative distance (the O(dt) term) from
    the leading-order closed form evaluated with the scheme's own f, while the
    difference form drifts and at s = 1e-12 is off by tens of percent."""
    ms = I.MeshSpec(dim=2, deg=3, nel=(3, 3, 1), lo=(0, 0, 0), hi=(1, 1, 1))
    m = orc_mesh(orc, ms)
    base = I.uniform_state(ms, vel=(0.3, -0.2, 0))
    pert = I.random_state(ms, seed=3, smooth=True, rel=0.2, vmax=0.3) - base
    dt = 0.1 * orc.cfl_dt(m, base, 0.5)
    M = np.tile(node_mass(orc, ms).reshape(-1), ms.ne)
    dev_acc, dev_naive = {}, {}
    for s in (1e-4, 1e-8, 1e-11, 1e-12):
        u = base + s * pert
        f = orc.rhs(m, u)[0]
        Jf = _jac_times(orc, ms, u, f, h=1e-4 / np.abs(f).max())
        lead = -0.5 * dt ** 2 * ((f.reshape(ms.nv, -1) * Jf).sum(axis=0) * M).reshape(
            ms.ne, ms.nd).sum(axis=1)
        du, deta, a = orc.rk_step_a(m, orc.RK44, u, dt)
        ref = orc.local_relaxation_solve(m, u, du, deta)
        dev_acc[s] = a / lead - 1.0
        dev_naive[s] = ref["phi0"] / lead - 1.0
    for s in (1e-8, 1e-11):
        assert np.abs(dev_acc[s] - dev_acc[1e-4]).max() <= 1e-3, s
    assert np.abs(dev_acc[1e-12]).max() <= 0.02
    assert np.abs(dev_naive[1e-12]).max() >= 0.1


def test_roots_from_stagewise_phi0(orc):
    """With phi(0) supplied the roots satisfy the element equations to the
    extended-precision level: r_k(gamma_k) - gamma_k (a_k - (A_k - deta_k))
    brackets zero, and they agree with the difference form's roots within that
    form's conditioning bound."""
    ms = I.vortex_mesh(4, 3)
    m = orc_mesh(orc, ms)
    u = I.vortex_state(ms)
    dt = orc.cfl_dt(m, u, 0.5)
    du, deta, a = orc.rk_step_a(m, orc.RK44, u, dt)
    acc = orc.local_relaxation_solve(m, u, du, deta, a=a)
    nai = orc.local_relaxation_solve(m, u, du, deta)
    assert acc["rc"] == 0 and nai["rc"] == 0
    fin = np.isfinite(nai["gamma_k"])
    assert np.array_equal(fin, np.isfinite(acc["gamma_k"]))
    tol = 2e-12 + nai["noise"][fin] / nai["curv"][fin]
    assert np.all(np.abs(acc["gamma_k"][fin] - nai["gamma_k"][fin]) <= tol)
    np.testing.assert_array_equal(acc["phi0"], a)
    # the supplied value enters phi exactly: phi(g) = a + B(g)/g changes sign at the root
    for k in np.flatnonzero(fin)[:8]:
        g = acc["gamma_k"][k]
        shift = a[k] - nai["phi0"][k]
        r_lo, _ = orc.relax_r(m, k, u, du, deta[k], g)
        r_hi, _ = orc.relax_r(m, k, u, du, deta[k], g * (1 + 4e-12))
        lvl = 1e-3 * nai["noise"][k] * g
        assert r_lo / g + shift <= lvl and r_hi / (g * (1 + 4e-12)) + shift >= -lvl
