"""Whole relaxed steps recorded into a HIP graph (esrk_run_graph) against the
same steps launched eagerly: bit-identical states, times and step statistics
on every replay, with the program's own eager work and synchronizations
between the replays."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2003_08831_amd import esrk  # noqa: E402
from paper_2003_08831_amd import inputs as I  # noqa: E402
from tests.gpu_helpers import ctx_for, dev, host, zeros  # noqa: E402

pytestmark = pytest.mark.gpu


def _eager(ms, u0, nsteps, mode, tableau):
    ctx = ctx_for(ms, tableau=tableau)
    ctx.set_relaxation_mode(mode)
    u, t, st = dev(u0), zeros(1), zeros(8)
    for _ in range(nsteps):
        ctx.step(u, t, 0.0, None, st)
    torch.cuda.synchronize()
    assert ctx.sync_status()[0] == 0
    return host(u), host(t), host(st)


@pytest.mark.parametrize("mode", [esrk.RELAX_LOCAL, esrk.RELAX_GLOBAL, esrk.RELAX_NONE],
                         ids=["local", "global", "none"])
@pytest.mark.parametrize("case", ["tgv_d3p3", "vortex_d2p3"])
def test_graph_replays_match_eager_steps(case, mode):
    if case == "tgv_d3p3":
        ms, tab = I.tgv_mesh(6, 3), esrk.RK44
        u0 = I.tgv_state(ms, 0.1)
    else:
        ms, tab = I.vortex_mesh(8, 3), esrk.SSPRK33
        u0 = I.vortex_state(ms)
    nsteps = 4
    ref = _eager(ms, u0, nsteps, mode, tab)
    ctx = ctx_for(ms, tableau=tab)
    ctx.set_relaxation_mode(mode)
    s = torch.cuda.Stream()
    u, t, st = dev(u0), zeros(1), zeros(8)
    u_start = dev(u0)
    for replay in range(3):
        with torch.cuda.stream(s):
            u.copy_(u_start)
            t.zero_()
            st.zero_()
            ctx.run_graph(u, t, nsteps, st, stream=s)
        s.synchronize()
        assert ctx.sync_status()[0] == 0
        assert np.array_equal(host(u), ref[0]), replay
        assert np.array_equal(host(t), ref[1]), replay
        assert np.array_equal(host(st), ref[2]), replay
        # eager work of the program between the replays
        junk = torch.randn(1 << 16, device="cuda").sum()
        torch.cuda.synchronize()
        del junk


def test_graph_rerecords_after_a_setting_changes():
    ms = I.tgv_mesh(4, 3)
    u0 = I.tgv_state(ms, 0.1)
    ref_local = _eager(ms, u0, 2, esrk.RELAX_LOCAL, esrk.RK44)
    ref_none = _eager(ms, u0, 2, esrk.RELAX_NONE, esrk.RK44)
    assert not np.array_equal(ref_local[0], ref_none[0])
    ctx = ctx_for(ms, tableau=esrk.RK44)
    s = torch.cuda.Stream()
    u, t = dev(u0), zeros(1)
    for mode, ref in ((esrk.RELAX_LOCAL, ref_local), (esrk.RELAX_NONE, ref_none)):
        ctx.set_relaxation_mode(mode)
        with torch.cuda.stream(s):
            u.copy_(dev(u0))
            t.zero_()
            ctx.run_graph(u, t, 2, None, stream=s)
        s.synchronize()
        assert np.array_equal(host(u), ref[0])


def test_graph_rejections():
    ms = I.tgv_mesh(4, 3)
    ctx = ctx_for(ms, tableau=esrk.BSRK43)
    s = torch.cuda.Stream()
    u, t = dev(I.tgv_state(ms, 0.1)), zeros(1)
    with pytest.raises(esrk.EsrkError) as e:
        ctx.run_graph(u, t, 1, None, stream=None)
    assert e.value.code == 1
    with pytest.raises(esrk.EsrkError) as e:
        ctx.run_graph(u, t, 0, None, stream=s)
    assert e.value.code == 1
    ctx.set_adaptive(1e-6, 1e-6)
    with pytest.raises(esrk.EsrkError) as e:
        ctx.run_graph(u, t, 1, None, stream=s)
    assert e.value.code == 7
