"""Contact Hessian lists on affine bodies resting on a sheet (inputs of the
two-level contact reduction only).

Contact nodes: the sheet's nodes (mesh nodes, block row = node id) and the 8
corners of every affine body (a cube of side ``body_side``; corner k of body
b is contact node ``Vs + 8 b + k``, with rest position ``xbar`` in the body
frame; the body's 12 DOFs are block rows ``Vs + 4 b .. Vs + 4 b + 3``, as in
the membrane + bodies system).  Each contact is a 12x12 PSD Hessian
``Q diag(logU(1e2, 1e6)) Q^T`` over four contact nodes, listed as its 16 3x3
node-pair blocks:
  * vertex-face: one body corner and a sheet triangle under the body;
  * edge-edge: two corners of one body and two of a neighbouring body.
A corner touches several triangles and a triangle several corners, so node
pairs repeat across contacts.
"""

import numpy as np

from .membrane import sheet


def psd_blocks(rng, n, dim, lo, hi):
    """``n`` blocks ``Q diag(s) Q^T``, Q Haar-orthogonal (QR with sign fix),
    ``s`` log-uniform in ``[lo, hi]`` (batched form of the random PSD block
    of the other workloads)."""
    A = rng.standard_normal((n, dim, dim))
    Q, R = np.linalg.qr(A)
    Q = Q * np.sign(np.diagonal(R, axis1=1, axis2=2))[:, None, :]
    s = np.exp(rng.uniform(np.log(lo), np.log(hi), size=(n, dim)))
    M = (Q * s[:, None, :]) @ np.swapaxes(Q, 1, 2)
    return 0.5 * (M + np.swapaxes(M, 1, 2))


def body_contacts(cells=512, n_bodies=2000, n_vf=200000, n_ee=40000, seed=1004, body_side=0.05, size=1.0):
    ss = np.random.SeedSequence(seed)
    s_pos, s_vf, s_ee, s_q = ss.spawn(4)
    X, tris = sheet(cells, size)
    Vs = X.shape[0]
    h = size / cells
    half = 0.5 * body_side
    corners = np.array([[sx, sy, sz] for sx in (-half, half) for sy in (-half, half) for sz in (-half, half)])
    n_nodes = Vs + 8 * n_bodies
    node_row = np.empty(n_nodes, dtype=np.int32)
    node_row[:Vs] = np.arange(Vs)
    node_row[Vs:] = Vs + 4 * np.repeat(np.arange(n_bodies), 8)
    is_body = np.zeros(n_nodes, dtype=np.int32)
    is_body[Vs:] = 1
    xbar = np.zeros((n_nodes, 3))
    xbar[Vs:] = np.tile(corners, (n_bodies, 1))
    # body centres over the sheet, in cell units away from the border
    rp = np.random.default_rng(s_pos)
    centre = rp.uniform(2, cells - 2, (n_bodies, 2)).astype(np.int64)
    quads = []
    # vertex-face: a bottom corner of a random body and one of the triangles
    # of the 2x2 cells under the body's centre
    rv = np.random.default_rng(s_vf)
    b = rv.integers(0, n_bodies, n_vf)
    k = rv.integers(0, 4, n_vf) * 2  # bottom corners (z = -half): k even
    ci = centre[b, 0] + rv.integers(-1, 1, n_vf)
    cj = centre[b, 1] + rv.integers(-1, 1, n_vf)
    tri = ci * cells + cj + rv.integers(0, 2, n_vf) * cells * cells  # either triangle of the cell
    quads.append(np.stack([Vs + 8 * b + k, tris[tri, 0], tris[tri, 1], tris[tri, 2]], axis=1))
    # edge-edge: two corners of a body and two of the next body in centre order
    re = np.random.default_rng(s_ee)
    order = np.lexsort((centre[:, 1], centre[:, 0]))
    i = re.integers(0, n_bodies - 1, n_ee)
    b1, b2 = order[i], order[i + 1]
    e1 = re.integers(0, 8, (n_ee, 2))
    e2 = re.integers(0, 8, (n_ee, 2))
    e1[:, 1] = np.where(e1[:, 1] == e1[:, 0], (e1[:, 0] + 1) % 8, e1[:, 1])
    e2[:, 1] = np.where(e2[:, 1] == e2[:, 0], (e2[:, 0] + 1) % 8, e2[:, 1])
    quads.append(np.stack([Vs + 8 * b1 + e1[:, 0], Vs + 8 * b1 + e1[:, 1], Vs + 8 * b2 + e2[:, 0],
                           Vs + 8 * b2 + e2[:, 1]], axis=1))
    quads = np.concatenate(quads)
    Hc = psd_blocks(np.random.default_rng(s_q), quads.shape[0], 12, 1e2, 1e6)
    Hc = Hc.reshape(-1, 4, 3, 4, 3).transpose(0, 1, 3, 2, 4)  # (n, 4, 4, 3, 3)
    a, bb = np.meshgrid(np.arange(4), np.arange(4), indexing="ij")
    a, bb = a.ravel(), bb.ravel()
    rows = quads[:, a].ravel().astype(np.int32)
    cols = quads[:, bb].ravel().astype(np.int32)
    blocks = Hc[:, a, bb].reshape(-1, 3, 3)
    return {
        "n_nodes": n_nodes,
        "n_dof_rows": Vs + 4 * n_bodies,
        "node_row": node_row,
        "node_is_body": is_body,
        "node_xbar": xbar,
        "rows": rows,
        "cols": cols,
        "blocks": blocks,
        "contacts": int(quads.shape[0]),
    }
