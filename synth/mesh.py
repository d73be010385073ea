"""Structured tetrahedral cube meshes (5 tets per cube, alternating split)."""

import numpy as np

# Local corner numbering of a unit cube: corner c = (cx, cy, cz) -> cx + 2*cy + 4*cz.
_C000, _C100, _C010, _C110, _C001, _C101, _C011, _C111 = range(8)

# Split A: the central tet joins the four "even" corners; the four "odd" corners
# each cut off a corner tet.  Split B is the mirror image.  Alternating A/B by
# cube parity makes every shared face carry the same diagonal on both sides.
_SPLIT_A = np.array(
    [
        [_C000, _C110, _C101, _C011],
        [_C100, _C000, _C110, _C101],
        [_C010, _C000, _C110, _C011],
        [_C001, _C000, _C101, _C011],
        [_C111, _C110, _C101, _C011],
    ],
    dtype=np.int64,
)
_SPLIT_B = np.array(
    [
        [_C100, _C010, _C001, _C111],
        [_C000, _C100, _C010, _C001],
        [_C110, _C100, _C010, _C111],
        [_C101, _C100, _C001, _C111],
        [_C011, _C010, _C001, _C111],
    ],
    dtype=np.int64,
)


def tet_cube(n, spacing=1.0):
    """Regular n x n x n grid of cubes split into 5 tets each.

    Returns ``(rest_positions[(n+1)^3, 3], tets[5 n^3, 4])``.  Node id is
    ``i + (n+1) * (j + (n+1) * k)`` for grid index (i, j, k).  Every tet is
    oriented with positive volume.
    """
    n = int(n)
    m = n + 1
    g = np.arange(m, dtype=np.float64) * spacing
    zz, yy, xx = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)

    ci, cj, ck = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    # sort cubes in (k, j, i) order so tets follow node numbering
    order = np.lexsort((ci, cj, ck))
    ci, cj, ck = ci[order], cj[order], ck[order]
    corners = np.empty((ci.size, 8), dtype=np.int64)
    for c in range(8):
        dx, dy, dz = c & 1, (c >> 1) & 1, (c >> 2) & 1
        corners[:, c] = (ci + dx) + m * ((cj + dy) + m * (ck + dz))
    parity = (ci + cj + ck) & 1
    tets = np.empty((ci.size, 5, 4), dtype=np.int64)
    a = parity == 0
    tets[a] = corners[a][:, _SPLIT_A]
    tets[~a] = corners[~a][:, _SPLIT_B]
    tets = tets.reshape(-1, 4)

    # orient: swap two vertices where the signed volume is negative
    d = pos[tets[:, 1:]] - pos[tets[:, :1]]
    vol = np.einsum("ij,ij->i", d[:, 0], np.cross(d[:, 1], d[:, 2]))
    neg = vol < 0
    tets[neg, 1], tets[neg, 2] = tets[neg, 2].copy(), tets[neg, 1].copy()
    return pos, tets


def mesh_edges(tets):
    """Unique undirected edges ``(a, b)`` with ``a < b`` of a tet mesh, sorted."""
    pairs = []
    for p in range(4):
        for q in range(p + 1, 4):
            pairs.append(tets[:, [p, q]])
    e = np.concatenate(pairs, axis=0)
    e.sort(axis=1)
    e = np.unique(e, axis=0)
    return e


def cube_surface_nodes(n):
    """Ids of the nodes on the boundary of the (n+1)^3 node grid, ascending."""
    m = n + 1
    k, j, i = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    on = (i == 0) | (i == n) | (j == 0) | (j == n) | (k == 0) | (k == n)
    return np.nonzero(on.ravel())[0].astype(np.int64)
