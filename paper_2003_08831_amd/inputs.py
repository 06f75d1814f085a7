"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds input generators only: node coordinates of the mesh, the
analytic initial states and seeded random admissible states.  It contains none
of the scheme's arithmetic, imports neither the HIP library nor the oracle,
and both sides are fed from it.

Layout of every state: float64 array u[v, element, node] (flattened C order),
v in rho, rho*v_1..rho*v_dim, rho*E; elements lexicographic with x fastest;
nodes lexicographic over (deg+1)^dim with xi_1 fastest.

Node positions come from numpy's Legendre routines (the roots of P_p' plus the
end points): they are the mesh geometry at which initial states are sampled.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class MeshSpec:
    dim: int
    deg: int
    nel: tuple
    lo: tuple
    hi: tuple
    gas_gamma: float = 1.4
    gas_r: float = 1.0
    mu: float = 0.0
    prandtl: float = 0.72
    meta: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.deg + 1

    @property
    def nv(self):
        return self.dim + 2

    @property
    def nd(self):
        return self.n ** self.dim

    @property
    def ne(self):
        return int(np.prod(self.nel[: self.dim]))

    @property
    def N(self):
        return self.ne * self.nd


def lobatto_points(deg: int) -> np.ndarray:
    """Reference nodes on [-1, 1] from numpy.polynomial (roots of P_deg')."""
    c = np.zeros(deg + 1)
    c[-1] = 1.0
    inner = np.polynomial.legendre.legroots(np.polynomial.legendre.legder(c))
    return np.concatenate([[-1.0], np.sort(inner.real), [1.0]])


def node_coords(ms: MeshSpec) -> list:
    """Physical coordinates x_m[element, node] for m < dim."""
    xi = lobatto_points(ms.deg)
    n, dim = ms.n, ms.dim
    nel = list(ms.nel[:dim])
    h = [(ms.hi[m] - ms.lo[m]) / nel[m] for m in range(dim)]
    ke = np.arange(ms.ne)
    ki = np.arange(ms.nd)
    coords = []
    for m in range(dim):
        stride_e = int(np.prod(nel[:m])) if m else 1
        km = (ke // stride_e) % nel[m]
        im = (ki // (n ** m)) % n
        x = ms.lo[m] + (km[:, None] + 0.5 * (xi[im][None, :] + 1.0)) * h[m]
        coords.append(x)
    return coords


def conserved(dim, gg, rho, vel, p):
    """Pack primitive fields into u[v, ...]."""
    ke = 0.5 * rho * sum(v * v for v in vel)
    comps = [rho] + [rho * v for v in vel] + [p / (gg - 1.0) + ke]
    return np.stack([np.asarray(c, dtype=np.float64) for c in comps])


# ---------------------------------------------------------------- vortex ----
def vortex_fields(ms: MeshSpec, t: float = 0.0, eps: float = 5.0, mach: float = 0.5,
                  alpha: float = math.pi / 4.0, center=(0.0, 0.0)):
    """Isentropic vortex advected with the free stream (2-D).

    Free stream rho = 1, |U| = 1, p = 1/(gamma M^2), so c = 1/M.  The
    temperature ratio is T = 1 - eps^2 M^2 (gamma-1)/(8 pi^2) exp(G),
    rho = T^(1/(gamma-1)), p = p_inf rho T, with G = 1 - r^2 measured from the
    advected centre (nearest periodic image), and the swirl
      u1 = cos(a) - eps dy/(2 pi) exp(G/2),  u2 = sin(a) + eps dx/(2 pi) exp(G/2).
    """
    gg = ms.gas_gamma
    x, y = node_coords(ms)[:2]
    Lx = ms.hi[0] - ms.lo[0]
    Ly = ms.hi[1] - ms.lo[1]
    cx = center[0] + math.cos(alpha) * t
    cy = center[1] + math.sin(alpha) * t
    dx = x - cx
    dy = y - cy
    dx -= Lx * np.round(dx / Lx)
    dy -= Ly * np.round(dy / Ly)
    G = 1.0 - (dx * dx + dy * dy)
    T = 1.0 - eps * eps * mach * mach * (gg - 1.0) / (8.0 * math.pi ** 2) * np.exp(G)
    rho = T ** (1.0 / (gg - 1.0))
    p_inf = 1.0 / (gg * mach * mach)
    p = p_inf * rho * T
    u1 = math.cos(alpha) - eps * dy / (2.0 * math.pi) * np.exp(0.5 * G)
    u2 = math.sin(alpha) + eps * dx / (2.0 * math.pi) * np.exp(0.5 * G)
    return rho, [u1, u2], p


def vortex_mesh(nel: int = 8, deg: int = 3) -> MeshSpec:
    return MeshSpec(dim=2, deg=deg, nel=(nel, nel, 1), lo=(-5.0, -5.0, 0.0),
                    hi=(5.0, 5.0, 1.0), meta=dict(name="isentropic_vortex_2d"))


def vortex_state(ms: MeshSpec, t: float = 0.0) -> np.ndarray:
    rho, vel, p = vortex_fields(ms, t)
    return conserved(2, ms.gas_gamma, rho, vel, p).reshape(-1).copy()


# ------------------------------------------------------------ Taylor-Green ----
def tgv_mesh(nel: int = 16, deg: int = 3, mu: float = 0.0) -> MeshSpec:
    L = 2.0 * math.pi
    return MeshSpec(dim=3, deg=deg, nel=(nel, nel, nel), lo=(0.0, 0.0, 0.0),
                    hi=(L, L, L), mu=mu, prandtl=0.72,
                    meta=dict(name="taylor_green_3d"))


def tgv_state(ms: MeshSpec, mach: float = 0.1) -> np.ndarray:
    """Classical Taylor-Green vortex: rho = 1, V0 = L = 1,
    v = (sin x cos y cos z, -cos x sin y cos z, 0),
    p = 1/(gamma M^2) + (cos 2x + cos 2y)(cos 2z + 2)/16."""
    gg = ms.gas_gamma
    x, y, z = node_coords(ms)
    rho = np.ones_like(x)
    u1 = np.sin(x) * np.cos(y) * np.cos(z)
    u2 = -np.cos(x) * np.sin(y) * np.cos(z)
    u3 = np.zeros_like(x)
    p = 1.0 / (gg * mach * mach) + (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0) / 16.0
    return conserved(3, gg, rho, [u1, u2, u3], p).reshape(-1).copy()


# -------------------------------------------------------- Kelvin-Helmholtz ----
def kh_mesh(nel: int, deg: int = 3) -> MeshSpec:
    return MeshSpec(dim=2, deg=deg, nel=(nel, nel, 1), lo=(-1.0, -1.0, 0.0),
                    hi=(1.0, 1.0, 1.0), meta=dict(name="kelvin_helmholtz_2d"))


def kh_state(ms: MeshSpec, amp: float, k: int, delta: float = 1.0 / 15.0,
             sigma: float = 0.1) -> np.ndarray:
    """Shear layer on [-1,1]^2: B(y) = (tanh((y+1/2)/d) - tanh((y-1/2)/d))/2,
    rho = 1 + B (density ratio 2), u = -1/2 + B (shear +-0.5), p = 2.5,
    v = amp sin(2 pi k x) (exp(-(y-1/2)^2/s^2) + exp(-(y+1/2)^2/s^2))."""
    x, y = node_coords(ms)[:2]
    B = 0.5 * (np.tanh((y + 0.5) / delta) - np.tanh((y - 0.5) / delta))
    rho = 1.0 + B
    u1 = -0.5 + B
    u2 = amp * np.sin(2 * math.pi * k * x) * (np.exp(-((y - 0.5) / sigma) ** 2)
                                              + np.exp(-((y + 0.5) / sigma) ** 2))
    p = 2.5 * np.ones_like(x)
    return conserved(2, ms.gas_gamma, rho, [u1, u2], p).reshape(-1).copy()


def kh_batch_specs(nsims: int = 256, seed: int = 0):
    """Seeded batch recipe: elements per direction uniform in {16,32,48,64},
    amplitude log-uniform in [1e-3, 1e-1], wavenumber uniform in {1,2,3,4}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(nsims):
        nel = int(rng.choice([16, 32, 48, 64]))
        amp = float(10.0 ** rng.uniform(-3.0, -1.0))
        k = int(rng.integers(1, 5))
        out.append((nel, amp, k))
    return out


# ------------------------------------------------------- 1-D local gamma test ----
def local_gamma_1d_mesh(nel: int = 200, deg: int = 3) -> MeshSpec:
    return MeshSpec(dim=1, deg=deg, nel=(nel, 1, 1), lo=(-2.0, 0.0, 0.0),
                    hi=(2.0, 1.0, 1.0), meta=dict(name="local_gamma_1d"))


def local_gamma_1d_state(ms: MeshSpec) -> np.ndarray:
    """(rho, v, p) = (1 + cos(2 pi x)/2, 1/2, 1) for x < 0 and
    (1/2 + cos(2 pi x)/4, 1/2, 4/5) for x >= 0."""
    (x,) = node_coords(ms)[:1]
    left = x < 0.0
    rho = np.where(left, 1.0 + 0.5 * np.cos(2 * math.pi * x), 0.5 + 0.25 * np.cos(2 * math.pi * x))
    v = 0.5 * np.ones_like(x)
    p = np.where(left, 1.0, 0.8)
    return conserved(1, ms.gas_gamma, rho, [v], p).reshape(-1).copy()


# ------------------------------------------- 1-D problems with boundaries ----
def sod_mesh(nel: int = 128, deg: int = 3) -> MeshSpec:
    return MeshSpec(dim=1, deg=deg, nel=(nel, 1, 1), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                    meta=dict(name="sod_shock_tube"))


def sod_state(ms: MeshSpec) -> np.ndarray:
    """(rho, v, p) = (1, 0, 1) for x < 1/2, (1/8, 0, 1/10) for x >= 1/2."""
    (x,) = node_coords(ms)[:1]
    left = x < 0.5
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    return conserved(1, ms.gas_gamma, rho, [np.zeros_like(x)], p).reshape(-1).copy()


def shock_sine_mesh(nel: int = 256, deg: int = 3) -> MeshSpec:
    return MeshSpec(dim=1, deg=deg, nel=(nel, 1, 1), lo=(-5.0, 0.0, 0.0), hi=(5.0, 1.0, 1.0),
                    meta=dict(name="sine_shock_interaction"))


def shock_sine_state(ms: MeshSpec) -> np.ndarray:
    """(rho, v, p) = (1.515695, 0.523346, 1.805) for x < -4.5, else
    (1 + 0.1 sin(20 pi x), 0, 1)."""
    (x,) = node_coords(ms)[:1]
    left = x < -4.5
    rho = np.where(left, 1.515695, 1.0 + 0.1 * np.sin(20.0 * math.pi * x))
    v = np.where(left, 0.523346, 0.0)
    p = np.where(left, 1.805, 1.0)
    return conserved(1, ms.gas_gamma, rho, [v], p).reshape(-1).copy()


def end_states(ms: MeshSpec, u: np.ndarray):
    """Conserved states at the first and the last node of a 1-D mesh (the
    Lobatto nodes include the interval's ends): the Dirichlet exterior
    states that hold the initial boundary values."""
    U = np.asarray(u).reshape(ms.nv, -1)
    return U[:, 0].copy(), U[:, -1].copy()


# ------------------------------------------------------------ random states ----
def random_state(ms: MeshSpec, seed: int = 0, rel: float = 0.2, vmax: float = 0.5,
                 smooth: bool = False) -> np.ndarray:
    """Admissible random state: rho = 1 (1 + rel r), p = 1 (1 + rel r),
    v_m = vmax r with r uniform in [-1, 1] per node (or a random smooth field
    when smooth=True)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (ms.ne, ms.nd)
    if smooth:
        xs = node_coords(ms)

        def field():
            f = np.zeros(shape)
            for _ in range(3):
                ph = rng.uniform(0, 2 * math.pi)
                arg = ph
                for m in range(ms.dim):
                    L = ms.hi[m] - ms.lo[m]
                    arg = arg + 2 * math.pi * int(rng.integers(1, 3)) * xs[m] / L
                f += np.sin(arg) / 3.0
            return f
        r = [field() for _ in range(ms.dim + 2)]
    else:
        r = [rng.uniform(-1.0, 1.0, size=shape) for _ in range(ms.dim + 2)]
    rho = 1.0 + rel * r[0]
    p = 1.0 + rel * r[1]
    vel = [vmax * r[2 + m] for m in range(ms.dim)]
    return conserved(ms.dim, ms.gas_gamma, rho, vel, p).reshape(-1).copy()


def uniform_state(ms: MeshSpec, rho=1.0, vel=(0.3, -0.2, 0.1), p=1.0) -> np.ndarray:
    shape = (ms.ne, ms.nd)
    return conserved(ms.dim, ms.gas_gamma, np.full(shape, rho),
                     [np.full(shape, vel[m]) for m in range(ms.dim)],
                     np.full(shape, p)).reshape(-1).copy()


# Network for the first relaxation trial point: 5 -> 32 -> 32 -> 1.  Parameter
# layout W1[32][5], b1[32], W2[32][32], b2[32], w3[32], b3, then the input
# normalization scale[5], mean[5], std[5] and the output out_mean, out_std.
MLP_IN, MLP_H, MLP_TRAINED, MLP_MODEL = 5, 32, 1281, 1298


def mlp_init(seed: int = 0) -> np.ndarray:
    """Xavier-uniform weights, zero biases, identity normalization (float32)."""
    rng = np.random.default_rng(seed)
    p = np.zeros(MLP_MODEL, dtype=np.float64)

    def xavier(fan_out, fan_in):
        a = math.sqrt(6.0 / (fan_in + fan_out))
        return rng.uniform(-a, a, size=fan_out * fan_in)

    p[0:160] = xavier(MLP_H, MLP_IN)
    p[192:1216] = xavier(MLP_H, MLP_H)
    p[1248:1280] = xavier(1, MLP_H)
    p[1281:1286] = 1.0   # scale
    p[1291:1296] = 1.0   # std
    p[1297] = 1.0        # out_std
    return p.astype(np.float32)
