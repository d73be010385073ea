"""Stiff membrane coupled to affine bodies.

A flat square triangle sheet (``cells x cells`` squares, two triangles each)
carries

* the Hessian of the cubic inexact strain-limiting energy (Sec. 5,
  Eq. Stretch_Hessian) per triangle, evaluated at a seeded in-plane stretch
  ``F = [[1 + s_u, 0], [0, 1 + s_v], [0, 0]]``, ``s ~ U(0, max_stretch)``:
  with ``I5 = |F n|^2`` per direction ``n`` in ``{n_u, n_v}``,
  ``H_F = lambda' a_t * sum_n [3 (1 - 1/sqrt(I5)) (sqrt(I5) - 1) L_n (x) I3
  + 3 (I5 - 1) / I5^(3/2) f f^T]``, ``f = vec(F L_n)``, ``L_n = n n^T``,
  chained to the triangle's nodes through ``F = D_s D_m^-1``;
* a Gauss-Newton dihedral bending block per interior edge,
  ``k_b w_e grad(theta) grad(theta)^T`` with ``w_e = 3 |e|^2 / (A_1 + A_2)``,
  evaluated on the flat rest sheet (the gradient then points out of plane);
* lumped mass ``rho * thickness * area / 3`` per triangle corner.

Each affine body has 12 degrees of freedom ``q = [t, a_1, a_2, a_3]``
(translation and the columns of ``A``, four block rows; a point moves as
``t + A xbar``): the reduced mass ``sum_corners m_c J_c^T J_c``,
``J_c = [I3 | xbar_c,1 I3 | xbar_c,2 I3 | xbar_c,3 I3]``, plus the
PSD-clamped Hessian of the orthogonality energy
``kappa * vol * ||A A^T - I||_F^2`` at ``A = I + 1e-3 N(0, 1)``.  Each body is
coupled to ``per_body`` distinct random sheet nodes by a random PSD 15x15
block (12 body + 3 node degrees of freedom, ``Q diag(logU[1e2, 1e6]) Q^T``,
added unscaled, like the contact couplings of the cube workload).

``H = M + dt^2 (strain limiting + bending + orthogonality) + couplings``.
The node graph of the partition is the mesh connectivity, as for the cube's
contacts: triangle edges, bending pairs and the links among a body's own
block rows; the body-sheet couplings are left out of it (they are in ``H``).
"""

import numpy as np

from .bcsr import BlockSystem, assemble_bcsr, graph_from_edges, random_psd_block


def sheet(cells, size=1.0):
    """Rest positions (2D) and triangles of a ``cells x cells`` square grid;
    node (i, j) has id ``i * (cells + 1) + j``."""
    m = cells + 1
    i, j = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    X = np.stack([i.ravel(), j.ravel()], axis=1) * (size / cells)
    ci, cj = np.meshgrid(np.arange(cells), np.arange(cells), indexing="ij")
    v00 = (ci * m + cj).ravel()
    v10, v01, v11 = v00 + m, v00 + 1, v00 + m + 1
    tris = np.concatenate([np.stack([v00, v10, v11], axis=1), np.stack([v00, v11, v01], axis=1)])
    return X, tris


def interior_edges(tris):
    """(a, b, o1, o2, t1, t2) for every edge shared by two triangles: edge
    nodes a < b, the opposite node and the triangle on each side."""
    nt = tris.shape[0]
    loc = np.array([[0, 1, 2], [1, 2, 0], [2, 0, 1]])
    a = tris[:, loc[:, 0]].ravel()
    b = tris[:, loc[:, 1]].ravel()
    o = tris[:, loc[:, 2]].ravel()
    t = np.repeat(np.arange(nt), 3)
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    n = int(tris.max()) + 1
    key = lo.astype(np.int64) * n + hi
    order = np.argsort(key, kind="stable")
    key, lo, hi, o, t = key[order], lo[order], hi[order], o[order], t[order]
    pair = np.nonzero(key[1:] == key[:-1])[0]
    return lo[pair], hi[pair], o[pair], o[pair + 1], t[pair], t[pair + 1]


def strain_limiting_blocks(X, tris, s_u, s_v, lam, thickness):
    """3x3 blocks (k, l) of the per-triangle strain-limiting Hessian with
    respect to the triangle's node positions, as their diagonals
    (nt, 3, 3, 3) (with F stretched along the material axes every block is
    diagonal), and the triangle areas."""
    x0, x1, x2 = X[tris[:, 0]], X[tris[:, 1]], X[tris[:, 2]]
    Dm = np.stack([x1 - x0, x2 - x0], axis=2)  # (nt, 2, 2), columns = edges
    det = Dm[:, 0, 0] * Dm[:, 1, 1] - Dm[:, 0, 1] * Dm[:, 1, 0]
    area = 0.5 * np.abs(det)
    inv = np.empty_like(Dm)
    inv[:, 0, 0], inv[:, 1, 1] = Dm[:, 1, 1] / det, Dm[:, 0, 0] / det
    inv[:, 0, 1], inv[:, 1, 0] = -Dm[:, 0, 1] / det, -Dm[:, 1, 0] / det
    # F[:, c] = sum_k x_k beta_k[c]: beta_1 = row 0 of D_m^-1, beta_2 = row 1
    beta = np.stack([-(inv[:, 0, :] + inv[:, 1, :]), inv[:, 0, :], inv[:, 1, :]], axis=1)  # (nt, 3, 2)
    at = area * thickness
    Hn = []  # diagonals of H_u, H_v (f = vec(F L_n) has one nonzero entry, r, on the axis)
    for s, axis in ((s_u, 0), (s_v, 1)):
        r = 1.0 + s  # sqrt(I5)
        I5 = r * r
        c_iso = 3.0 * (1.0 - 1.0 / r) * (r - 1.0)
        c_rank = 3.0 * (I5 - 1.0) / I5 ** 1.5
        d = np.repeat(c_iso[:, None], 3, axis=1)
        d[:, axis] += c_rank * r * r
        Hn.append((lam * at)[:, None] * d)
    # block (k, l) = beta_k[0] beta_l[0] H_u + beta_k[1] beta_l[1] H_v
    wu = beta[:, :, None, 0] * beta[:, None, :, 0]
    wv = beta[:, :, None, 1] * beta[:, None, :, 1]
    return wu[..., None] * Hn[0][:, None, None] + wv[..., None] * Hn[1][:, None, None], area


def bending_blocks(X, area, edges, k_b):
    """Gauss-Newton dihedral blocks on the flat sheet over the nodes
    (o1, o2, a, b) of each interior edge: the out-of-plane entry of each
    3x3 block (the only nonzero one), (ne, 4, 4)."""
    a, b, o1, o2, t1, t2 = edges
    E = X[b] - X[a]
    le2 = np.einsum("ij,ij->i", E, E)
    le = np.sqrt(le2)
    A1, A2 = area[t1], area[t2]
    h1, h2 = 2.0 * A1 / le, 2.0 * A2 / le
    al1 = np.einsum("ij,ij->i", X[o1] - X[a], E) / le2
    al2 = np.einsum("ij,ij->i", X[o2] - X[a], E) / le2
    g = np.stack([1.0 / h1, 1.0 / h2, -((1.0 - al1) / h1 + (1.0 - al2) / h2), -(al1 / h1 + al2 / h2)], axis=1)
    w = k_b * 3.0 * le2 / (A1 + A2)
    return w[:, None, None] * g[:, :, None] * g[:, None, :]


def orthogonality_hessians(A, kappa_vol):
    """PSD-clamped Hessians (nb, 9, 9) of kappa_vol * ||A A^T - I||_F^2 with
    respect to vec(A) (columns of A stacked)."""
    nb = A.shape[0]
    B = A @ np.transpose(A, (0, 2, 1)) - np.eye(3)[None]
    H = np.empty((nb, 9, 9))
    for col in range(9):
        D = np.zeros((nb, 3, 3))
        D[:, col % 3, col // 3] = 1.0  # unit change of entry (row col % 3, column col // 3)
        dB = D @ np.transpose(A, (0, 2, 1)) + A @ np.transpose(D, (0, 2, 1))
        HD = 4.0 * kappa_vol[:, None, None] * (dB @ A + B @ D)
        H[:, :, col] = np.transpose(HD, (0, 2, 1)).reshape(nb, 9)  # vec, columns stacked
    H = 0.5 * (H + np.transpose(H, (0, 2, 1)))
    lam, Q = np.linalg.eigh(H)
    return (Q * np.maximum(lam, 0.0)[:, None, :]) @ np.transpose(Q, (0, 2, 1))


def membrane_system(
    cells,
    n_bodies,
    seed=0,
    per_body=16,
    size=1.0,
    thickness=1e-3,
    density=200.0,
    lam=5e6,
    max_stretch=0.08,
    k_b=1e-3,
    dt=0.01,
    body_side=0.05,
    body_density=1000.0,
    kappa=1e8,
):
    ss = np.random.SeedSequence(seed)
    s_stretch, s_bodies, s_attach, s_q, s_rhs = ss.spawn(5)
    X, tris = sheet(cells, size)
    Vs = X.shape[0]
    V = Vs + 4 * n_bodies
    nt = tris.shape[0]
    rs = np.random.default_rng(s_stretch)
    s_u = rs.uniform(0.0, max_stretch, nt)
    s_v = rs.uniform(0.0, max_stretch, nt)
    dt2 = dt * dt

    parts_r, parts_c, parts_b = [], [], []

    # strain limiting, 9 blocks per triangle
    Kd, area = strain_limiting_blocks(X, tris, s_u, s_v, lam, thickness)
    ka, kb = np.meshgrid(np.arange(3), np.arange(3), indexing="ij")
    ka, kb = ka.ravel(), kb.ravel()
    parts_r.append(tris[:, ka].ravel())
    parts_c.append(tris[:, kb].ravel())
    Kb = np.zeros((nt * 9, 3, 3))
    dg = (dt2 * Kd[:, ka, kb]).reshape(-1, 3)
    for c in range(3):
        Kb[:, c, c] = dg[:, c]
    parts_b.append(Kb)
    del Kd, dg

    # bending, 16 blocks per interior edge
    edges = interior_edges(tris)
    Bk = bending_blocks(X, area, edges, k_b)
    nodes4 = np.stack([edges[2], edges[3], edges[0], edges[1]], axis=1)
    ba, bb = np.meshgrid(np.arange(4), np.arange(4), indexing="ij")
    ba, bb = ba.ravel(), bb.ravel()
    parts_r.append(nodes4[:, ba].ravel())
    parts_c.append(nodes4[:, bb].ravel())
    Bb = np.zeros((Bk.shape[0] * 16, 3, 3))
    Bb[:, 2, 2] = (dt2 * Bk[:, ba, bb]).ravel()
    parts_b.append(Bb)
    del Bk

    # lumped sheet mass
    m_node = np.bincount(tris.ravel(), weights=np.repeat(density * thickness * area / 3.0, 3), minlength=Vs)
    parts_r.append(np.arange(Vs))
    parts_c.append(np.arange(Vs))
    parts_b.append(m_node[:, None, None] * np.eye(3)[None])

    meta = {
        "kind": "membrane_bodies",
        "cells": cells,
        "sheet_nodes": Vs,
        "triangles": nt,
        "bending_pairs": int(edges[0].size),
        "bodies": n_bodies,
        "per_body": per_body,
        "seed": seed,
    }
    if n_bodies:
        rb = np.random.default_rng(s_bodies)
        half = 0.5 * body_side
        corners = np.array([[sx, sy, sz] for sx in (-half, half) for sy in (-half, half) for sz in (-half, half)])
        vol = body_side ** 3
        m_c = body_density * vol / 8.0
        Mr = np.zeros((12, 12))
        for xb in corners:
            J = np.concatenate([np.eye(3)] + [xb[k] * np.eye(3) for k in range(3)], axis=1)
            Mr += m_c * J.T @ J
        A = np.eye(3)[None] + 1e-3 * rb.standard_normal((n_bodies, 3, 3))
        Ho = orthogonality_hessians(A, np.full(n_bodies, kappa * vol))
        Hb = np.broadcast_to(Mr, (n_bodies, 12, 12)).copy()
        Hb[:, 3:, 3:] += dt2 * Ho
        base = Vs + 4 * np.arange(n_bodies)
        pa, pb = np.meshgrid(np.arange(4), np.arange(4), indexing="ij")
        pa, pb = pa.ravel(), pb.ravel()
        parts_r.append((base[:, None] + pa[None]).ravel())
        parts_c.append((base[:, None] + pb[None]).ravel())
        parts_b.append(Hb.reshape(n_bodies, 4, 3, 4, 3).transpose(0, 1, 3, 2, 4)[:, pa, pb].reshape(-1, 3, 3))

        # couplings: body (4 block rows) + one sheet node, 15x15 each
        ra = np.random.default_rng(s_attach)
        attach = np.stack([ra.choice(Vs, size=per_body, replace=False) for _ in range(n_bodies)])
        rq = np.random.default_rng(s_q)
        C = np.stack([random_psd_block(rq, 15, 1e2, 1e6) for _ in range(n_bodies * per_body)])
        C = C.reshape(-1, 5, 3, 5, 3).transpose(0, 1, 3, 2, 4)  # (nc, 5, 5, 3, 3)
        ent = np.concatenate([np.repeat(base, per_body)[:, None] + np.arange(4)[None], attach.reshape(-1, 1)], axis=1)
        ea, eb = np.meshgrid(np.arange(5), np.arange(5), indexing="ij")
        ea, eb = ea.ravel(), eb.ravel()
        parts_r.append(ent[:, ea].ravel())
        parts_c.append(ent[:, eb].ravel())
        parts_b.append(C[:, ea, eb].reshape(-1, 3, 3))
        meta["attach"] = attach
    # positions (for the Morton ordering only): sheet nodes on the z = 0
    # plane; a body's four block rows at the centroid of the sheet nodes it
    # couples to, one body side above the sheet
    pos = np.zeros((V, 3))
    pos[:Vs, :2] = X[:, :2]
    if n_bodies:
        cen = X[attach][:, :, :2].mean(axis=1)
        for p4 in range(4):
            pos[base + p4, :2] = cen
            pos[base + p4, 2] = body_side
    meta["positions"] = pos

    all_r, all_c, all_b = np.concatenate(parts_r), np.concatenate(parts_c), np.concatenate(parts_b)
    del parts_r, parts_c, parts_b
    row_ptr, col_idx, val = assemble_bcsr(V, all_r, all_c, all_b)
    del all_r, all_c, all_b
    # node graph: triangle edges, bending pairs, links within each body
    gl = [tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]], np.stack([edges[2], edges[3]], axis=1)]
    if n_bodies:
        for p in range(4):
            for q in range(p + 1, 4):
                gl.append(np.stack([base + p, base + q], axis=1))
    gptr, gadj = graph_from_edges(V, np.concatenate(gl))
    b = np.random.default_rng(s_rhs).standard_normal(3 * V)
    meta["nnzb"] = int(col_idx.size)
    return BlockSystem(n=V, row_ptr=row_ptr, col_idx=col_idx, val=val, b=b, gptr=gptr, gadj=gadj, meta=meta)
