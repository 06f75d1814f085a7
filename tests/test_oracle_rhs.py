"""Pins of the oracle's semidiscretization (CPU only): free-stream
preservation, conservation, entropy conservation of the EC volume term per
element, the exact LLF entropy-dissipation identity, the reduction of the
volume term to the collocation derivative, the BR1 identities and spatial
convergence on the isentropic vortex."""
import math

import numpy as np
import pytest

from paper_2003_08831_amd import inputs as I
from tests.oracle_helpers import face_weight, node_mass, orc_mesh, view

MESHES = [
    I.MeshSpec(dim=1, deg=3, nel=(7, 1, 1), lo=(0, 0, 0), hi=(1.3, 1, 1)),
    I.MeshSpec(dim=2, deg=3, nel=(3, 4, 1), lo=(0, -1, 0), hi=(1, 2, 1)),
    I.MeshSpec(dim=2, deg=4, nel=(2, 3, 1), lo=(0, 0, 0), hi=(1, 1, 1)),
    I.MeshSpec(dim=3, deg=2, nel=(2, 3, 2), lo=(0, 0, 0), hi=(1, 2, 1.5)),
    I.MeshSpec(dim=3, deg=3, nel=(2, 2, 2), lo=(0, 0, 0), hi=(1, 1, 1)),
]
IDS = [f"d{m.dim}p{m.deg}" for m in MESHES]


@pytest.mark.parametrize("ms", MESHES, ids=IDS)
def test_free_stream(orc, ms):
    m = orc_mesh(orc, ms)
    u = I.uniform_state(ms, rho=1.2, vel=(0.3, -0.4, 0.5), p=0.9)
    dudt, er = orc.rhs(m, u)
    assert np.abs(dudt).max() <= 1e-12
    assert np.abs(er).max() <= 1e-12


@pytest.mark.parametrize("ms", MESHES, ids=IDS)
@pytest.mark.parametrize("lam", [0.0, 1.0])
def test_conservation_and_entropy_balance(orc, ms, lam):
    m = orc_mesh(orc, ms, lambda_scale=lam)
    u = I.random_state(ms, seed=3)
    dudt, er = orc.rhs(m, u)
    M = node_mass(orc, ms)
    d = view(ms, dudt)
    scale = np.abs(d * M).sum()
    assert np.abs((d * M).sum(axis=(1, 2))).max() <= 1e-14 * scale
    # total entropy rate = -(interface dissipation), = 0 for the EC surface
    diss = orc.interface_dissipation(m, u)
    assert diss >= 0.0
    assert abs(er.sum() + diss) <= 1e-13 * (np.abs(er).sum() + diss + 1.0)
    if lam == 0.0:
        assert diss == 0.0


@pytest.mark.parametrize("ms", MESHES, ids=IDS)
def test_volume_term_element_identities(orc, ms):
    """Per element: sum_i M_i V_i and sum_i M_i w_i.V_i equal the face sums of
    f_m and of the entropy flux F_m = S v_m (no neighbours involved)."""
    m = orc_mesh(orc, ms)
    u = I.random_state(ms, seed=5)
    V = view(ms, orc.volume_term(m, u))
    U = view(ms, u)
    M = node_mass(orc, ms)
    gg = ms.gas_gamma
    for k in range(ms.ne):
        lhs_c = (V[:, k, :] * M).sum(axis=1)
        lhs_e = sum(M[i] * orc.entropy_vars(ms.dim, gg, U[:, k, i]) @ V[:, k, i]
                    for i in range(ms.nd))
        rhs_c = np.zeros(ms.nv)
        rhs_e = 0.0
        for i in range(ms.nd):
            ui = U[:, k, i]
            for mm in range(ms.dim):
                im = (i // ms.n ** mm) % ms.n
                sgn = 1.0 if im == ms.deg else (-1.0 if im == 0 else 0.0)
                if sgn == 0.0:
                    continue
                a = face_weight(orc, ms, i, mm)
                rhs_c += sgn * a * orc.phys_flux(ms.dim, gg, mm, ui)
                rhs_e += sgn * a * orc.entropy(ms.dim, gg, ui) * ui[1 + mm] / ui[0]
        sc = np.abs(V[:, k, :] * M).sum()
        np.testing.assert_allclose(lhs_c, rhs_c, atol=1e-13 * sc)
        assert abs(lhs_e - rhs_e) <= 1e-12 * (abs(rhs_e) + sc)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_central_volume_flux_is_exact_derivative(orc, dim):
    """With the central average as two-point flux, 2 D o F 1 = D f.  For
    constant v and p, rho affine in x: f is affine, so V_i is the exact
    derivative: V = c rho' (1, c e_x, |c|^2/2) in the x-direction."""
    ms = I.MeshSpec(dim=dim, deg=3, nel=(3, 2, 2)[:dim] + (1,) * (3 - dim),
                    lo=(0, 0, 0), hi=(1, 1, 1))
    m = orc_mesh(orc, ms, volume_flux=1)
    x = I.node_coords(ms)
    slope, c = 0.3, 0.7
    rho = 1.0 + slope * x[0]
    vel = [np.full_like(rho, c)] + [np.zeros_like(rho)] * (dim - 1)
    u = I.conserved(dim, ms.gas_gamma, rho, vel, np.full_like(rho, 0.8)).reshape(-1)
    V = view(ms, orc.volume_term(m, u))
    expect = np.zeros(ms.nv)
    expect[0] = c * slope
    expect[1] = c * c * slope
    expect[-1] = 0.5 * c ** 3 * slope
    for v in range(ms.nv):
        np.testing.assert_allclose(V[v], expect[v], atol=1e-13)


@pytest.mark.parametrize("ms", [MESHES[1], MESHES[3], MESHES[4]], ids=["d2p3", "d3p2", "d3p3"])
def test_br1_identities(orc, ms):
    ns = I.MeshSpec(dim=ms.dim, deg=ms.deg, nel=ms.nel, lo=ms.lo, hi=ms.hi, mu=0.05,
                    prandtl=0.72)
    m = orc_mesh(orc, ns)
    u = I.random_state(ns, seed=9, smooth=True, rel=0.1, vmax=0.3)
    # total viscous entropy rate: sum M w.Visc = -sum M theta.g <= 0
    dudt_ns, er_ns, vd = orc.rhs(m, u, want_visc=True)
    m_eu = orc_mesh(orc, I.MeshSpec(dim=ms.dim, deg=ms.deg, nel=ms.nel, lo=ms.lo, hi=ms.hi))
    dudt_eu, er_eu = orc.rhs(m_eu, u)
    visc_rate = er_ns.sum() - er_eu.sum()
    assert np.all(vd >= -1e-15)
    assert abs(visc_rate + vd.sum()) <= 1e-12 * vd.sum()
    # constant entropy variables: theta = 0 and no viscous term
    uf = I.uniform_state(ns, rho=1.1, vel=(0.2, 0.1, -0.3), p=0.9)
    assert np.abs(orc.br1_gradient(m, uf)).max() <= 1e-12
    d1, _ = orc.rhs(m, uf)
    assert np.abs(d1).max() <= 1e-12


def test_br1_gradient_exact_for_polynomials(orc):
    """theta is the exact gradient of w when w is a globally continuous
    polynomial of degree <= p: with rho = 1 + a x and p = rho (so that
    w_E = -1 is constant and w_1 = v), theta_x of the momentum component is v'."""
    ms = I.MeshSpec(dim=2, deg=3, nel=(3, 2, 1), lo=(0, 0, 0), hi=(1, 1, 1), mu=0.01)
    m = orc_mesh(orc, ms)
    x, y = I.node_coords(ms)
    # T = p/rho = 1 fixed, v_1 = 0.2 + 0.5 y + 0.1 x (affine, periodic break
    # avoided by checking an interior element pair only along x)
    rho = np.ones_like(x)
    v1 = 0.2 + 0.1 * np.sin(2 * math.pi * x)
    u = I.conserved(2, ms.gas_gamma, rho, [v1, np.zeros_like(x)], rho).reshape(-1)
    th = orc.br1_gradient(m, u).reshape(2, ms.nv, ms.ne, ms.nd)
    # w_1 = rho v_1 / p = v_1 ; d/dx v_1 = 0.2 pi cos(2 pi x) -- spectral accuracy only,
    # so check the y-derivative (exactly 0) and an x-derivative tolerance of the p=3 fit
    assert np.abs(th[1]).max() <= 1e-12
    err = np.abs(th[0, 1] - 0.2 * math.pi * np.cos(2 * math.pi * x)).max()
    assert err < 5e-2


@pytest.mark.slow
def test_vortex_spatial_convergence(orc):
    """p = 3 entropy-stable scheme on the isentropic vortex: density L2 error
    after t = 0.5 with RK(4,4) and a small step converges at about p + 1
    (the paper's p = 3 rates are 3.8 - 4.7)."""
    errs = []
    for nel in (4, 8, 16):
        ms = I.vortex_mesh(nel, 3)
        m = orc_mesh(orc, ms)
        u = I.vortex_state(ms)
        t, tend = 0.0, 0.5
        dt = 0.02 * 8 / nel
        nsteps = int(round(tend / dt))
        for _ in range(nsteps):
            du, _ = orc.rk_step(m, orc.RK44, u, dt)
            u += du
            t += dt
        ex = I.vortex_state(ms, t)
        M = node_mass(orc, ms)
        e = view(ms, u - ex)[0]
        errs.append(math.sqrt(((e ** 2) * M).sum() / 100.0))
    rates = [math.log(errs[i] / errs[i + 1], 2) for i in range(2)]
    assert rates[-1] > 3.3, (errs, rates)


def test_elem_max_speed_uniform_and_single_node(orc):
    """A uniform state has sum_m |v_m| + dim c in every element; raising the
    velocity at one node changes only its element's value."""
    import math as _m
    ms = I.tgv_mesh(nel=2, deg=2)
    u = I.uniform_state(ms, rho=1.3, vel=(0.3, -0.2, 0.1), p=0.9)
    m = orc_mesh(orc, ms)
    s = orc.elem_max_speed(m, u)
    c = _m.sqrt(1.4 * 0.9 / 1.3)
    np.testing.assert_allclose(s, 0.6 + 3 * c, rtol=1e-15)
    uv = view(ms, u).copy()
    k, i = 5, 7
    uv[1, k, i] *= 3.0  # rho v_1 tripled, energy kept: pressure drops
    rho, E = uv[0, k, i], uv[4, k, i]
    v = np.array([uv[1, k, i], uv[2, k, i], uv[3, k, i]]) / rho
    p = 0.4 * (E - 0.5 * rho * np.dot(v, v))
    s2 = orc.elem_max_speed(m, uv.reshape(-1))
    expect = np.abs(v).sum() + 3 * _m.sqrt(1.4 * p / rho)
    assert abs(s2[k] - max(expect, 0.6 + 3 * c)) <= 1e-15 * expect
    assert np.all(np.delete(s2, k) == s[0])
