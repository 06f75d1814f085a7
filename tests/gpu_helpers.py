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
