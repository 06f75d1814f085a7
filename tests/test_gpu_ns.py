"""GPU parity of the Navier-Stokes (BR1 viscous) path against the CPU oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_2003_08831_amd import esrk  # noqa: E402
from paper_2003_08831_amd import inputs as I  # noqa: E402
from tests.gpu_helpers import ctx_for, dev, host, rhs_close, term_scale, zeros  # noqa: E402
from tests.oracle_helpers import node_mass, orc_mesh, view  # noqa: E402

pytestmark = pytest.mark.gpu

CASES = [
    ("d2p3", I.MeshSpec(dim=2, deg=3, nel=(5, 4, 1), lo=(0, 0, 0), hi=(1, 1.2, 1), mu=0.02),
     "smooth"),
    ("d2p2_rand", I.MeshSpec(dim=2, deg=2, nel=(3, 3, 1), lo=(0, 0, 0), hi=(1, 1, 1), mu=0.01),
     "rand"),
    ("d3p3_tgv", I.tgv_mesh(3, 3, mu=0.05), "tgv"),
    ("d3p4", I.MeshSpec(dim=3, deg=4, nel=(2, 3, 2), lo=(0, 0, 0), hi=(1, 1, 1), mu=0.01),
     "smooth"),
    ("d1p3", I.MeshSpec(dim=1, deg=3, nel=(11, 1, 1), lo=(0, 0, 0), hi=(1, 1, 1), mu=0.03),
     "smooth"),
    # 3-D p5: 216 nodes per element (four waves per block), nine MFMA row groups
    ("d3p5", I.MeshSpec(dim=3, deg=5, nel=(2, 2, 2), lo=(0, 0, 0), hi=(1, 1, 1), mu=0.01),
     "smooth"),
]
IDS = [c[0] for c in CASES]


def state(ms, kind, seed=1):
    if kind == "tgv":
        return I.tgv_state(ms, mach=0.3)
    return I.random_state(ms, seed=seed, smooth=(kind == "smooth"), rel=0.1, vmax=0.3)


def visc_scale(O, ms, u):
    """Scale of the viscous terms: (2/h)^2 |D|^2 mu times the entropy-variable
    spread, bounded through the oracle's own viscous right-hand side."""
    m_ns = orc_mesh(O, ms)
    m_eu = orc_mesh(O, I.MeshSpec(dim=ms.dim, deg=ms.deg, nel=ms.nel, lo=ms.lo, hi=ms.hi))
    d_ns, _ = O.rhs(m_ns, u)
    d_eu, _ = O.rhs(m_eu, u)
    return np.abs((d_ns - d_eu).reshape(ms.nv, -1)).max(axis=1)


@pytest.mark.parametrize("name,ms,kind", CASES, ids=IDS)
def test_rhs_ns_parity(name, ms, kind):
    u = state(ms, kind)
    m = orc_mesh(O, ms)
    ref, ref_eta, ref_vd = O.rhs(m, u, want_visc=True)
    ctx = ctx_for(ms)
    out, eta, vd = zeros(u.size), zeros(ctx.ne), zeros(ctx.ne)
    ctx.rhs_ns(dev(u), out, eta, vd)
    S = term_scale(O, ms, u) + 100.0 * visc_scale(O, ms, u)
    assert rhs_close(host(out), ref, ms, S) <= 1.0
    g_vd = host(vd)
    assert np.all(g_vd >= -1e-15 * np.abs(ref_vd).max())
    np.testing.assert_allclose(g_vd, ref_vd, rtol=1e-11, atol=1e-13 * np.abs(ref_vd).max())
    assert ctx.sync_status()[0] == 0


@pytest.mark.parametrize("name,ms,kind", [CASES[0], CASES[2], CASES[3]],
                         ids=["d2p3", "d3p3_tgv", "d3p4"])
def test_br1_identity_on_gpu(name, ms, kind):
    """The viscous part's entropy rate equals minus the viscous dissipation:
    sum M w.(dudt_ns - dudt_euler) = -sum_k diss_k <= 0, from the GPU outputs."""
    u = dev(state(ms, kind))
    ctx = ctx_for(ms)
    a, b = zeros(u.numel()), zeros(u.numel())
    ea, eb, vd = zeros(ctx.ne), zeros(ctx.ne), zeros(ctx.ne)
    ctx.rhs_ns(u, a, ea, vd)
    ctx.rhs_euler(u, b, eb)
    rate = host(ea).sum() - host(eb).sum()
    diss = host(vd).sum()
    assert diss > 0.0
    assert abs(rate + diss) <= 1e-10 * diss


@pytest.mark.parametrize("tab", [esrk.SSPRK33, esrk.RK44], ids=["ssprk33", "rk44"])
@pytest.mark.parametrize("name,ms,kind", [CASES[0], CASES[2]], ids=["d2p3", "d3p3_tgv"])
def test_ns_stage_chain_and_step_parity(tab, name, ms, kind):
    u = state(ms, kind, seed=2)
    m = orc_mesh(O, ms)
    dt = 0.5 * O.cfl_dt(m, u, 0.5)
    du_ref, deta_ref, ys, _, _ = O.rk_step(m, tab, u, dt, want_stages=True)
    S = term_scale(O, ms, u) + 100.0 * visc_scale(O, ms, u)
    ctx = ctx_for(ms, tableau=tab)
    s = O.tableau_stages(tab)
    ud = dev(u)
    bufs = [zeros(u.size), zeros(u.size)]
    du, deta = zeros(u.size), zeros(ctx.ne)
    yin = ud
    for i in range(s):
        yout = bufs[i % 2] if i < s - 1 else None
        ctx.rk_stage(i, dt, ud, yin, yout, du, deta)
        if yout is not None:
            assert rhs_close(host(yout), ys[i + 1], ms, dt * S) <= 1.0
        yin = yout
    assert rhs_close(host(du), du_ref, ms, dt * S, rel=1e-11) <= 1.0
    assert np.abs(host(deta) - deta_ref).max() <= 1e-10 * np.abs(deta_ref).max()
    # one whole relaxed step with the same fixed dt
    ref = O.local_relaxation_solve(m, u, du_ref, deta_ref)
    assert ref["rc"] == 0
    t = zeros(1)
    stats = zeros(8)
    ctx.step(ud, t, dt, None, stats)
    g = host(stats)[0]
    fin = np.isfinite(ref["gamma_k"])
    kmin = np.argmin(np.where(fin, ref["gamma_k"], np.inf))
    gtol = 2e-12 + ref["noise"][kmin] / ref["curv"][kmin] + 1e-9
    assert abs(g - ref["gamma"]) <= gtol
    assert ctx.sync_status()[0] == 0


@pytest.mark.parametrize("name,ms,kind", [CASES[0], CASES[2], CASES[3], CASES[5]],
                         ids=["d2p3", "d3p3_tgv", "d3p4", "d3p5"])
def test_ns_fp32_conservation(name, ms, kind):
    u = state(ms, kind)
    m = orc_mesh(O, ms)
    ref, _ = O.rhs(m, u)
    ctx = ctx_for(ms, precision=esrk.FP32_FLUX)
    out, eta, vd = zeros(u.size), zeros(ctx.ne), zeros(ctx.ne)
    ctx.rhs_ns(dev(u), out, eta, vd)
    g = view(ms, host(out))
    M = node_mass(O, ms)
    integ = (g * M).sum(axis=(1, 2))
    scale = (np.abs(g) * M).sum(axis=(1, 2))
    assert np.all(np.abs(integ) <= 1e-5 * scale)
    err = np.abs(g.reshape(ms.nv, -1) - ref.reshape(ms.nv, -1)).max(axis=1)
    assert np.all(err <= 5e-3 * np.abs(ref.reshape(ms.nv, -1)).max(axis=1) + 1e-6)
