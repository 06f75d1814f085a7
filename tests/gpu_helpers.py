"""Shared plumbing of the GPU parity tests: device tensors, contexts built
from the same MeshSpec as the oracle meshes, and comparison helpers."""
import numpy as np
import torch

from paper_2003_08831_amd import esrk
from paper_2003_08831_amd import inputs as I

DEV = "cuda"


def ctx_for(ms: I.MeshSpec, precision=esrk.FP64, tableau=esrk.SSPRK33, lambda_scale=1.0,
            cfl=0.5, root_tol=1e-12, **kw):
    cfg = esrk.make_config(ms.dim, ms.deg, ms.nel, ms.lo, ms.hi, gas_gamma=ms.gas_gamma,
                           gas_r=ms.gas_r, mu=ms.mu, prandtl=ms.prandtl,
                           lambda_scale=lambda_scale, precision=precision, tableau=tableau,
                           cfl=cfl, root_tol=root_tol, **kw)
    return esrk.Context(cfg)


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def zeros(n, dtype=torch.float64):
    return torch.zeros(n, dtype=dtype, device=DEV)


def normwise(g, o, nv):
    """max over components of max|g - o| / max|o| (component-wise scale)."""
    g = np.asarray(g).reshape(nv, -1)
    o = np.asarray(o).reshape(nv, -1)
    out = []
    for v in range(nv):
        sc = np.abs(o[v]).max()
        out.append(np.abs(g[v] - o[v]).max() / (sc if sc > 0 else 1.0))
    return max(out)


def term_scale(O, ms, u):
    """Per-component scale of the terms the right-hand side sums before they
    cancel: max |f_v,m(u)| over nodes and directions, times the largest
    metric 2/h_m, times the largest row sum of |2 D| plus the interface lift
    1/w_0 (all from the oracle's own operators)."""
    U = np.asarray(u).reshape(ms.nv, -1)
    fmax = np.zeros(ms.nv)
    for i in range(U.shape[1]):
        for m in range(ms.dim):
            fmax = np.maximum(fmax, np.abs(O.phys_flux(ms.dim, ms.gas_gamma, m, U[:, i])))
    D = O.dmat(ms.deg)
    _, w = O.lgl(ms.deg)
    metric = max(2.0 * ms.nel[m] / (ms.hi[m] - ms.lo[m]) for m in range(ms.dim))
    opnorm = np.abs(2.0 * D).sum(axis=1).max() + 1.0 / w[0]
    return fmax * metric * opnorm * ms.dim


def term_scale_np(O, ms, u):
    """term_scale with max|f_v,m(u)| taken by numpy over all nodes at once (a
    tolerance scale, for meshes too large for the per-node oracle calls):
    f_m = [rho v_m, rho v_m v + p e_m, v_m (E + p)]."""
    U = np.asarray(u).reshape(ms.nv, -1)
    rho, E = U[0], U[-1]
    vel = U[1:1 + ms.dim] / rho
    p = (ms.gas_gamma - 1.0) * (E - 0.5 * rho * (vel ** 2).sum(axis=0))
    fmax = np.zeros(ms.nv)
    for m in range(ms.dim):
        f = [rho * vel[m]] + [rho * vel[m] * vel[k] + (p if k == m else 0.0)
                              for k in range(ms.dim)] + [vel[m] * (E + p)]
        fmax = np.maximum(fmax, np.array([np.abs(fv).max() for fv in f]))
    D = O.dmat(ms.deg)
    _, w = O.lgl(ms.deg)
    metric = max(2.0 * ms.nel[m] / (ms.hi[m] - ms.lo[m]) for m in range(ms.dim))
    opnorm = np.abs(2.0 * D).sum(axis=1).max() + 1.0 / w[0]
    return fmax * metric * opnorm * ms.dim


def rhs_close(g, o, ms, S, rel=1e-12, cond=1e-14):
    """Component-wise: |g - o| <= rel * max|o_v| + cond * S_v, where S_v is the
    term scale (FP64 evaluations of a cancelling sum differ by ~eps * S_v)."""
    g = np.asarray(g).reshape(ms.nv, -1)
    o = np.asarray(o).reshape(ms.nv, -1)
    worst = 0.0
    for v in range(ms.nv):
        tol = rel * np.abs(o[v]).max() + cond * S[v]
        worst = max(worst, np.abs(g[v] - o[v]).max() / tol)
    return worst
