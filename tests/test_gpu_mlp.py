"""GPU network kernels against the FP64 oracle, and the relaxation solve with a
learned or warm-start first trial point against the oracle's gamma_k.

The kernels compute in FP32; the oracle is evaluated on the same FP32-rounded
inputs, so the bounds below only cover FP32 arithmetic (about 2^-24 per
operation over sums of at most 32 terms per layer)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_2003_08831_amd import esrk, learn  # noqa: E402
from paper_2003_08831_amd import inputs as I  # noqa: E402
from tests.gpu_helpers import ctx_for, dev, host, zeros  # noqa: E402
from tests.oracle_helpers import orc_mesh  # noqa: E402
from tests.test_gpu_parity import check_gammas, make_state, relax_tolerance  # noqa: E402

pytestmark = pytest.mark.gpu

F32 = torch.float32


def rand_model(seed):
    """Network with nonzero biases (FP32-representable values, as float64)."""
    p = I.mlp_init(seed).astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(100 + seed))
    p[160:192] = rng.normal(scale=0.3, size=32)
    p[1216:1248] = rng.normal(scale=0.3, size=32)
    p[1280] = 0.1
    return p.astype(np.float32).astype(np.float64)


def rand_x(B, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.normal(size=(B, 5)).astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("B", [1, 63, 64, 1000, 4099])
def test_forward_parity(B):
    p = rand_model(1)
    X = rand_x(B, 2)
    ref = O.mlp_forward(p[:1281], X)
    y = zeros(B, F32)
    esrk.mlp_forward(dev(p, F32), dev(X, F32), y)
    err = np.abs(host(y).astype(np.float64) - ref).max()
    assert err <= 1e-5 * max(1.0, np.abs(ref).max()), err


@pytest.mark.parametrize("B", [1, 64, 300, 2000])
def test_grad_parity(B):
    p = rand_model(3)
    X = rand_x(B, 4)
    T = np.random.Generator(np.random.PCG64(5)).normal(size=B).astype(np.float32)
    g_ref, L_ref = O.mlp_grad(p[:1281], X, T.astype(np.float64))
    g = zeros(1281, F32)
    loss = zeros(1, F32)
    esrk.mlp_grad(dev(p, F32), dev(X, F32), dev(T, F32), g, loss)
    gg = host(g).astype(np.float64)
    assert np.abs(gg - g_ref).max() <= 1e-4 * np.abs(g_ref).max()
    assert abs(host(loss)[0] - L_ref) <= 1e-5 * L_ref


def test_adam_parity():
    rng = np.random.Generator(np.random.PCG64(6))
    p = rng.normal(size=1281).astype(np.float32).astype(np.float64)
    g = (rng.normal(size=1281) * 10.0 ** rng.uniform(-4, 1, size=1281))
    g = g.astype(np.float32).astype(np.float64)
    m = (0.1 * rng.normal(size=1281)).astype(np.float32).astype(np.float64)
    v = (0.01 * rng.uniform(size=1281) ** 2).astype(np.float32).astype(np.float64)
    pd, md, vd = dev(p, F32), dev(m, F32), dev(v, F32)
    lr, step = 1e-3, 5
    # FP32 rounding bounds from the size of the terms each update adds
    m_sc = 0.9 * np.abs(m) + 0.1 * np.abs(g)
    v_sc = 0.999 * v + 0.001 * g * g
    esrk.mlp_adam(pd, dev(g, F32), md, vd, step, lr)
    O.mlp_adam(p, g, m, v, step, lr)
    # (each constant and each operation rounds once: a few units of 2^-24)
    eps32 = 2.0 ** -24
    assert np.all(np.abs(host(md) - m) <= 6 * eps32 * m_sc)
    assert np.all(np.abs(host(vd) - v) <= 6 * eps32 * v_sc)
    c1, c2 = 1 - 0.9 ** step, 1 - 0.999 ** step
    # the step lr m_hat / (sqrt(v_hat) + eps) inherits those relative errors
    dstep = lr / (c1 * (np.sqrt(v / c2) + 1e-8)) * (
        6 * eps32 * m_sc + np.abs(m) * (3 * eps32 * v_sc / v + 8 * eps32))
    assert np.all(np.abs(host(pd) - p) <= 2 * eps32 * np.abs(p) + dstep)


def test_prepare_parity():
    rng = np.random.Generator(np.random.PCG64(8))
    B = 3001
    raw = np.stack([rng.normal(scale=1e-5, size=B), rng.normal(scale=3e-6, size=B),
                    rng.uniform(1e-3, 2e-3, size=B), rng.uniform(1.0, 2.0, size=B),
                    -rng.exponential(1e-7, size=B)], axis=1).astype(np.float32)
    q = rng.normal(loc=-0.3, scale=0.05, size=B)
    gamma = 1.0 + raw[:, 2].astype(np.float64) ** 2 * q
    model = np.zeros(1298, dtype=np.float32)
    md = dev(model, F32)
    xn, tn = zeros(B * 5, F32), zeros(B, F32)
    esrk.mlp_prepare(md, dev(raw, F32), xn, dev(gamma), tn, fit=True)
    ref_model, ref_x, ref_t = O.mlp_prepare(model.astype(np.float64), raw.astype(np.float64),
                                            gamma, fit=True)
    mg = host(md).astype(np.float64)
    np.testing.assert_allclose(mg[1281:], ref_model[1281:], rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(host(xn).reshape(B, 5), ref_x, atol=2e-5)
    np.testing.assert_allclose(host(tn), ref_t, atol=2e-5)
    # applying a fitted model without refitting gives the same inputs
    xn2 = zeros(B * 5, F32)
    esrk.mlp_prepare(md, dev(raw, F32), xn2, fit=False)
    assert torch.equal(xn, xn2)
    assert np.array_equal(host(md), mg.astype(np.float32))


def test_training_reduces_loss():
    """Student fitted to a teacher network's outputs by the GPU gradient and
    Adam kernels: the loss falls by more than 10x in 400 full-batch steps."""
    teacher = rand_model(11)
    X = rand_x(2048, 12)
    T = O.mlp_forward(teacher[:1281], X).astype(np.float32)
    student = dev(I.mlp_init(13), F32)
    Xd, Td = dev(X, F32), dev(T, F32)
    g, m, v = zeros(1281, F32), zeros(1281, F32), zeros(1281, F32)
    loss = zeros(1, F32)
    esrk.mlp_grad(student, Xd, Td, g, loss)
    L0 = float(host(loss)[0])
    for it in range(1, 401):
        esrk.mlp_grad(student, Xd, Td, g, loss)
        esrk.mlp_adam(student, g, m, v, it, 3e-3)
    esrk.mlp_grad(student, Xd, Td, g, loss)
    L1 = float(host(loss)[0])
    assert L1 < 0.1 * L0, (L0, L1)


RELAX_CASES = [
    ("d2p3_vortex", I.vortex_mesh(8, 3), "vortex"),
    ("d3p3_tgv", I.tgv_mesh(3, 3), "tgv"),
    ("d3p4", I.MeshSpec(dim=3, deg=4, nel=(3, 2, 3), lo=(0, 0, 0), hi=(1, 1, 1)), "smooth"),
    ("d2p5", I.MeshSpec(dim=2, deg=5, nel=(3, 3, 1), lo=(0, 0, 0), hi=(1, 1, 1)), "smooth"),
]


def _increment(ms, kind, tab=O.SSPRK33):
    u = make_state(ms, kind, seed=3)
    m = orc_mesh(O, ms)
    dt = O.cfl_dt(m, u, 0.5)
    du, deta = O.rk_step(m, tab, u, dt)
    return u, m, dt, du, deta


@pytest.mark.parametrize("name,ms,kind", RELAX_CASES, ids=[c[0] for c in RELAX_CASES])
def test_relaxation_with_model_features_and_gammas(name, ms, kind):
    u, m, dt, du, deta = _increment(ms, kind)
    ref = O.local_relaxation_solve(m, u, du, deta)
    assert ref["rc"] == 0
    ctx = ctx_for(ms)
    ud, dud, detad = dev(u), dev(du), dev(deta)
    feats = zeros(ctx.ne * 5, F32)
    gk, gam = zeros(ctx.ne), zeros(1)
    iters = torch.zeros(ctx.ne, dtype=torch.int32, device="cuda")
    vr = dev(np.linspace(-1e-3, 0.0, ctx.ne))
    # features only (no model): the plain solve
    ctx.local_relaxation_solve_ml(ud, dud, detad, dt, gk, gam, vr, None, feats, iters)
    check_gammas(host(gk), ref)
    f = host(feats).reshape(ctx.ne, 5).astype(np.float64)
    act = np.isfinite(ref["gamma_k"])
    np.testing.assert_array_equal(f[act, 0], deta.astype(np.float32)[act])
    d_eta = O.elem_entropy(m, u + du) - O.elem_entropy(m, u)
    eta_sc = np.abs(O.elem_entropy(m, u)).max()
    assert np.abs(f[act, 1] - d_eta[act]).max() <= 1e-6 * np.abs(d_eta).max() + 1e-13 * eta_sc
    assert np.all(f[act, 2] == np.float32(dt))
    np.testing.assert_allclose(f[act, 3], O.elem_max_speed(m, u)[act], rtol=1e-6)
    np.testing.assert_allclose(f[act, 4], (dt * host(vr))[act], rtol=1e-6, atol=1e-30)
    # with a (random, untrained) network and a badly scaled one: same gamma_k
    for shift in (0.0, 1e6, -1e6):
        p = rand_model(21).astype(np.float32)
        p[1281:1298] = 1.0
        p[1286:1291] = 0.0
        p[1296] = shift
        model = dev(p, F32)
        gk2 = zeros(ctx.ne)
        ctx.local_relaxation_solve_ml(ud, dud, detad, dt, gk2, gam, vr, model, None, iters)
        check_gammas(host(gk2), ref)
    # a warm start from the oracle's own roots: same gamma_k, few evaluations
    guess = dev(np.where(act, ref["gamma_k"], 1.0), F32)
    gk3 = zeros(ctx.ne)
    ctx.local_relaxation_solve(ud, dud, detad, gk3, gam, guess, iters)
    check_gammas(host(gk3), ref)
    assert ctx.sync_status()[0] == 0


def test_step_with_model_equals_plain_step():
    ms = I.vortex_mesh(8, 3)
    u = I.vortex_state(ms)
    ctx = ctx_for(ms)
    a, b = dev(u), dev(u)
    ta, tb = zeros(1), zeros(1)
    sa, sb = zeros(8), zeros(8)
    feats = torch.full((ctx.ne * 5,), float("nan"), dtype=F32, device="cuda")
    p = rand_model(31).astype(np.float32)
    p[1281:1298] = 1.0
    p[1286:1291] = 0.0
    p[1296] = 0.0
    model = dev(p, F32)
    m = orc_mesh(O, ms)
    for _ in range(5):
        # the oracle's roots on the same increment bound how far two root
        # solves with different trial points may land apart
        uh = host(a)
        du, deta = O.rk_step(m, O.SSPRK33, uh, O.cfl_dt(m, uh, 0.5))
        ref = O.local_relaxation_solve(m, uh, du, deta)
        fin = np.isfinite(ref["gamma_k"])
        kmin = np.argmin(np.where(fin, ref["gamma_k"], np.inf))
        tol = 2.0 * relax_tolerance(ref)[kmin]
        ctx.set_step_model(None, None)
        ctx.step(a, ta, 0.0, None, sa)
        ctx.set_step_model(model, feats)
        ctx.step(b, tb, 0.0, None, sb)
        ga, gb = host(sa), host(sb)
        assert abs(ga[0] - gb[0]) <= tol, (ga[0], gb[0], tol)
        # copy the state across so the two runs see the same increments
        b.copy_(a)
        tb.copy_(ta)
    ctx.set_step_model(None, None)
    f = host(feats).reshape(ctx.ne, 5)
    assert np.all(np.isfinite(f[:, 2:4]))
    assert ga[5] > 0 and gb[5] > 0
    assert ctx.sync_status()[0] == 0


def test_learned_guess_gain_report(capsys):
    """Collect samples from locally relaxed vortex steps, train, and report
    phi evaluations and solve time: plain first trial point, previous-step
    warm start and the network (each to the same tolerance)."""
    ms = I.vortex_mesh(8, 3)
    ctx = ctx_for(ms)
    u, t = dev(I.vortex_state(ms)), zeros(1)
    raw, g = learn.collect(ctx, u, t, 40)
    assert raw.shape[0] == g.shape[0] > 0
    model, hist = learn.train([(raw, g)], steps=300, batch=1024, lr=3e-3)
    assert np.isfinite(hist["train_final"]) and hist["train_final"] < 1.0
    res = learn.gain(ctx, u, t, 6, model)
    with capsys.disabled():
        print("\n[learned guess, vortex 8x8 p3]", hist["train_final"], hist["val_final"], res)
    for k in res:
        assert np.isfinite(res[k]["evals"]) and res[k]["evals"] >= 1.0
        assert res[k]["dgamma"] <= 1e-6
