"""Element Hessians for the synthetic Newton systems (inputs only).

Stable Neo-Hookean volume energy in the form
``Psi(F) = mu/2 (|F|_F^2 - 3) - mu (J - 1) + lam/2 (J - 1)^2``
(the paper cites the Stable Neo-Hookean model for the volumetric term without
fixing a variant; this one is used for the synthetic systems only).  Each
12x12 element Hessian is projected to PSD by clamping eigenvalues at zero.
"""

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np


def lame(E, nu):
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return mu, lam


def _skew(v):
    z = np.zeros(v.shape[:-1] + (3, 3))
    z[..., 0, 1] = -v[..., 2]
    z[..., 0, 2] = v[..., 1]
    z[..., 1, 0] = v[..., 2]
    z[..., 1, 2] = -v[..., 0]
    z[..., 2, 0] = -v[..., 1]
    z[..., 2, 1] = v[..., 0]
    return z


def snh_dPsi_dF2(F, mu, lam):
    """9x9 Hessian of Psi w.r.t. vec(F) (column-major: index 3*col + row)."""
    f0, f1, f2 = F[..., :, 0], F[..., :, 1], F[..., :, 2]
    g = np.concatenate([np.cross(f1, f2), np.cross(f2, f0), np.cross(f0, f1)], axis=-1)
    J = np.einsum("...i,...i->...", f0, np.cross(f1, f2))
    HJ = np.zeros(F.shape[:-2] + (9, 9))
    s0, s1, s2 = _skew(f0), _skew(f1), _skew(f2)
    HJ[..., 0:3, 3:6] = -s2
    HJ[..., 0:3, 6:9] = s1
    HJ[..., 3:6, 0:3] = s2
    HJ[..., 3:6, 6:9] = -s0
    HJ[..., 6:9, 0:3] = -s1
    HJ[..., 6:9, 3:6] = s0
    H = mu * np.eye(9) + lam * g[..., :, None] * g[..., None, :]
    H += (lam * (J - 1.0) - mu)[..., None, None] * HJ
    return H, g, J


def snh_psi(F, mu, lam):
    J = np.linalg.det(F)
    return 0.5 * mu * (np.einsum("...ij,...ij->...", F, F) - 3.0) - mu * (J - 1.0) + 0.5 * lam * (J - 1.0) ** 2


def shape_gradients(rest, tets):
    """Per-tet ``D[4,3]`` with ``F = sum_a x_a D[a]^T`` and the rest volume."""
    X = rest[tets]
    Dm = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=-1)
    vol = np.abs(np.linalg.det(Dm)) / 6.0
    Dminv = np.linalg.inv(Dm)
    D = np.empty((tets.shape[0], 4, 3))
    D[:, 1:, :] = Dminv
    D[:, 0, :] = -Dminv.sum(axis=1)
    return D, vol


def deformation_gradient(x, tets, D):
    return np.einsum("nai,naj->nij", x[tets], D)


def snh_element_hessians(rest, x, tets, E, nu, chunk=16384):
    """PSD-projected 12x12 SNH Hessians (rest-volume weighted), per tet."""
    mu, lam = lame(E, nu)
    D, vol = shape_gradients(rest, tets)
    out = np.empty((tets.shape[0], 12, 12))

    def one(s):  # chunks are independent: the result does not depend on the thread count
        e = slice(s, min(s + chunk, tets.shape[0]))
        F = deformation_gradient(x, tets[e], D[e])
        H9, _, _ = snh_dPsi_dF2(F, mu, lam)
        d2 = H9.reshape(-1, 3, 3, 3, 3)  # [j, i, J, I]: vec index 3*col + row
        De = D[e]
        # K[(a,i),(b,I)] = sum_{j,J} D[a,j] D[b,J] d2[j,i,J,I]
        T = np.einsum("naj,njiJI->naiJI", De, d2)
        K = np.einsum("naiJI,nbJ->naibI", T, De).reshape(-1, 12, 12)
        K = 0.5 * (K + np.transpose(K, (0, 2, 1)))
        w, V = np.linalg.eigh(K)
        w = np.maximum(w, 0.0) * vol[e][:, None]
        out[e] = np.einsum("nij,nj,nkj->nik", V, w, V)

    starts = range(0, tets.shape[0], chunk)
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        list(ex.map(one, starts))
    return out, vol


def lumped_mass(tets, vol, n_nodes, density):
    m = np.zeros(n_nodes)
    np.add.at(m, tets.ravel(), np.repeat(density * vol / 4.0, 4))
    return m
