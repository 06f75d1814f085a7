"""Small helpers the oracle tests share: mesh construction and quadrature
masses assembled from the (separately pinned) Lobatto weights."""
import numpy as np

from paper_2003_08831_amd import inputs as I


def orc_mesh(orc, ms: I.MeshSpec, lambda_scale=1.0, volume_flux=0):
    return orc.mesh(ms.dim, ms.deg, ms.nel, ms.lo, ms.hi, gas_gamma=ms.gas_gamma,
                    gas_r=ms.gas_r, mu=ms.mu, prandtl=ms.prandtl,
                    lambda_scale=lambda_scale, volume_flux=volume_flux)


def node_mass(orc, ms: I.MeshSpec):
    _, w = orc.lgl(ms.deg)
    M = np.ones(ms.nd)
    for i in range(ms.nd):
        for m in range(ms.dim):
            h = (ms.hi[m] - ms.lo[m]) / ms.nel[m]
            M[i] *= 0.5 * h * w[(i // ms.n ** m) % ms.n]
    return M


def face_weight(orc, ms: I.MeshSpec, i, m):
    _, w = orc.lgl(ms.deg)
    a = 1.0
    for q in range(ms.dim):
        if q != m:
            h = (ms.hi[q] - ms.lo[q]) / ms.nel[q]
            a *= 0.5 * h * w[(i // ms.n ** q) % ms.n]
    return a


def view(ms: I.MeshSpec, u):
    return np.asarray(u).reshape(ms.nv, ms.ne, ms.nd)
