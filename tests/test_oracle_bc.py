"""Pins of the oracle's 1-D boundaries (CPU): Dirichlet exterior states that
equal the periodic neighbours reproduce the periodic right-hand side bit for
bit (so the boundary faces use the right side and node), a uniform state with
matching exterior states is stationary, the paper's shock-tube setup stays
admissible under relaxed steps; an outflow end is a Dirichlet end whose
exterior state is the interior trace, and with outflow ends the discrete
conservation law leaves exactly the physical fluxes of the two end traces."""
import numpy as np
import pytest

from paper_2003_08831_amd import inputs as I
from tests.oracle_helpers import orc_mesh


def _dirichlet_mesh(orc, ms, left, right, lambda_scale=1.0):
    return orc.mesh(ms.dim, ms.deg, ms.nel, ms.lo, ms.hi, gas_gamma=ms.gas_gamma,
                    lambda_scale=lambda_scale, dirichlet=(left, right))


@pytest.mark.parametrize("deg", [2, 3, 5])
def test_dirichlet_with_periodic_neighbour_states_is_periodic(orc, deg):
    ms = I.MeshSpec(dim=1, deg=deg, nel=(7, 1, 1), lo=(0, 0, 0), hi=(1.3, 1, 1))
    u = I.random_state(ms, seed=4, smooth=True)
    per = orc.rhs(orc_mesh(orc, ms), u)[0]
    U = u.reshape(ms.nv, -1)
    # the periodic left neighbour of the first node is the last node, and back
    dm = _dirichlet_mesh(orc, ms, U[:, -1], U[:, 0])
    dir_ = orc.rhs(dm, u)[0]
    assert np.array_equal(per, dir_)
    # other exterior states change only the two boundary elements
    dm2 = _dirichlet_mesh(orc, ms, U[:, -1] * 1.01, U[:, 0] * 0.99)
    d2 = (orc.rhs(dm2, u)[0] - per).reshape(ms.nv, ms.ne, ms.nd)
    assert np.abs(d2[:, 1:-1]).max() == 0.0
    assert np.abs(d2[:, 0]).max() > 0.0 and np.abs(d2[:, -1]).max() > 0.0


def test_uniform_state_with_matching_exterior_is_stationary(orc):
    ms = I.MeshSpec(dim=1, deg=3, nel=(9, 1, 1), lo=(0, 0, 0), hi=(1, 1, 1))
    u = I.uniform_state(ms, rho=1.3, vel=(0.4,), p=0.9)
    U = u.reshape(ms.nv, -1)
    k = orc.rhs(_dirichlet_mesh(orc, ms, U[:, 0], U[:, 0]), u)[0]
    assert np.abs(k).max() <= 1e-13 * np.abs(u).max() * 9 * 4 * 4


def test_sod_relaxed_steps_stay_admissible(orc):
    """The shock tube (1/8 of the paper's 128 elements, same p = 3, RK(4,4),
    dt = 5e-5) for 40 relaxed steps: every step solves, gamma stays near 1."""
    ms = I.sod_mesh(16, 3)
    u = I.sod_state(ms)
    m = _dirichlet_mesh(orc, ms, *I.end_states(ms, u))
    t = 0.0
    gams = []
    for _ in range(40):
        res = orc.step(m, orc.RK44, u, t, dt=5e-5)
        assert res["rc"] == 0
        t = res["t"]
        gams.append(res["gamma"])
    assert 0.9 < min(gams) <= max(gams) < 1.1


def _euler_flux_1d(q, gg):
    """Textbook 1-D Euler flux (rho v, rho v^2 + p, (E + p) v)."""
    rho, m, E = q
    v = m / rho
    p = (gg - 1.0) * (E - 0.5 * m * v)
    return np.array([m, m * v + p, (E + p) * v])


def test_outflow_is_dirichlet_with_the_interior_traces(orc):
    ms = I.MeshSpec(dim=1, deg=4, nel=(6, 1, 1), lo=(0, 0, 0), hi=(2.0, 1, 1))
    u = I.random_state(ms, seed=12, smooth=True)
    U = u.reshape(ms.nv, -1)
    out = orc.mesh(1, ms.deg, ms.nel, ms.lo, ms.hi, gas_gamma=ms.gas_gamma,
                   outflow=(True, True))
    dirt = _dirichlet_mesh(orc, ms, U[:, 0], U[:, -1])
    assert np.array_equal(orc.rhs(out, u)[0], orc.rhs(dirt, u)[0])
    # one outflow end, one Dirichlet end
    left = U[:, 0] * np.array([1.02, 0.9, 1.01])
    mix = orc.mesh(1, ms.deg, ms.nel, ms.lo, ms.hi, gas_gamma=ms.gas_gamma,
                   dirichlet=(left, None), outflow=(False, True))
    ref = orc.rhs(_dirichlet_mesh(orc, ms, left, U[:, -1]), u)[0]
    assert np.array_equal(orc.rhs(mix, u)[0], ref)


@pytest.mark.parametrize("deg", [1, 3, 5])
def test_outflow_conservation_leaves_the_end_fluxes(orc, deg):
    """Sum_i M_i du_i/dt = f(u at the left end) - f(u at the right end): the
    interior interface fluxes cancel (SBP), and an outflow end's interface
    flux is the physical flux of its own trace."""
    from tests.oracle_helpers import node_mass
    ms = I.MeshSpec(dim=1, deg=deg, nel=(8, 1, 1), lo=(-1, 0, 0), hi=(1.5, 1, 1))
    u = I.random_state(ms, seed=3 + deg, smooth=True)
    m = orc.mesh(1, ms.deg, ms.nel, ms.lo, ms.hi, gas_gamma=ms.gas_gamma,
                 outflow=(True, True))
    k = orc.rhs(m, u)[0].reshape(ms.nv, ms.ne, ms.nd)
    M = node_mass(orc, ms)
    total = np.einsum("vei,i->v", k, M)
    U = u.reshape(ms.nv, -1)
    expect = _euler_flux_1d(U[:, 0], ms.gas_gamma) - _euler_flux_1d(U[:, -1], ms.gas_gamma)
    scale = np.abs(np.einsum("vei,i->v", np.abs(k), M)).max()
    assert np.abs(total - expect).max() <= 1e-13 * scale


def test_uniform_state_with_outflow_ends_is_stationary(orc):
    ms = I.MeshSpec(dim=1, deg=3, nel=(9, 1, 1), lo=(0, 0, 0), hi=(1, 1, 1))
    u = I.uniform_state(ms, rho=0.7, vel=(-0.3,), p=1.4)
    m = orc.mesh(1, ms.deg, ms.nel, ms.lo, ms.hi, gas_gamma=ms.gas_gamma,
                 outflow=(True, True))
    k = orc.rhs(m, u)[0]
    assert np.abs(k).max() <= 1e-13 * np.abs(u).max() * 9 * 4 * 4
