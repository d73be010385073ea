"""3x3-block BCSR assembly of element/contact contributions (inputs only)."""

from dataclasses import dataclass, field

import numpy as np


@dataclass
class BlockSystem:
    """An assembled SPD system ``H x = b`` in 3x3-block CSR form.

    ``row_ptr[n+1]`` / ``col_idx[nnzb]`` are int32 with ascending columns per
    row, both triangles stored, the diagonal block always present and
    ``val[b]`` the row-major 3x3 block.  ``H`` is bitwise symmetric:
    ``val[(j,i)] == val[(i,j)].T``.  ``gptr``/``gadj`` is the node graph the
    ordering partitions (the mesh edges; contacts are excluded, as they change
    between Newton steps).
    """

    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    val: np.ndarray
    b: np.ndarray
    gptr: np.ndarray
    gadj: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def nnzb(self):
        return int(self.col_idx.size)

    @property
    def ndof(self):
        return 3 * self.n

    def dense(self):
        """Dense ``3n x 3n`` copy (small systems only)."""
        n = self.n
        A = np.zeros((3 * n, 3 * n))
        for i in range(n):
            for p in range(self.row_ptr[i], self.row_ptr[i + 1]):
                j = self.col_idx[p]
                A[3 * i : 3 * i + 3, 3 * j : 3 * j + 3] = self.val[p]
        return A

    def scipy_bsr(self):
        import scipy.sparse as sp

        n = self.n
        return sp.bsr_matrix(
            (self.val, self.col_idx.astype(np.int64), self.row_ptr.astype(np.int64)),
            shape=(3 * n, 3 * n),
        )


def assemble_bcsr(n, rows, cols, blocks):
    """Sum 3x3 contributions ``blocks[k]`` at ``(rows[k], cols[k])`` into BCSR.

    The pattern of the contributions must be symmetric.  The result is made
    bitwise symmetric by mirroring: strictly-upper blocks overwrite their
    lower partners (transposed) and each diagonal block copies its upper
    scalar triangle onto its lower one.
    """
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    blocks = np.asarray(blocks, dtype=np.float64).reshape(-1, 9)
    keys = rows * n + cols
    order = np.argsort(keys, kind="stable")
    keys = keys[order]
    blocks = blocks[order]
    head = np.ones(keys.size, dtype=bool)
    head[1:] = keys[1:] != keys[:-1]
    starts = np.nonzero(head)[0]
    ukeys = keys[starts]
    val = np.add.reduceat(blocks, starts, axis=0).reshape(-1, 3, 3)
    r = ukeys // n
    c = ukeys % n

    # exact symmetry
    tkeys = c * n + r
    t = np.searchsorted(ukeys, tkeys)
    if np.any(t >= ukeys.size) or np.any(ukeys[np.minimum(t, ukeys.size - 1)] != tkeys):
        raise ValueError("contribution pattern is not symmetric")
    up = r < c
    val[t[up]] = np.transpose(val[up], (0, 2, 1))
    dg = r == c
    d = val[dg]
    iu = np.triu_indices(3, 1)
    d[:, iu[1], iu[0]] = d[:, iu[0], iu[1]]
    val[dg] = d

    counts = np.bincount(r, minlength=n)
    if np.any(np.bincount(r[dg], minlength=n) != 1):
        raise ValueError("every row needs its diagonal block")
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return row_ptr.astype(np.int32), c.astype(np.int32), np.ascontiguousarray(val)


def graph_from_edges(n, edges):
    """Symmetric CSR adjacency (ascending, no self loops) from an edge list."""
    edges = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    e = edges[edges[:, 0] != edges[:, 1]]
    a = np.concatenate([e[:, 0], e[:, 1]])
    b = np.concatenate([e[:, 1], e[:, 0]])
    key = np.unique(a * n + b)
    a = key // n
    b = key % n
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(a, minlength=n), out=ptr[1:])
    return ptr.astype(np.int32), b.astype(np.int32)


def random_psd_block(rng, dim, lo, hi):
    """``Q diag(s) Q^T`` with Q Haar-orthogonal (QR with sign fix) and
    ``s`` log-uniform in ``[lo, hi]``."""
    A = rng.standard_normal((dim, dim))
    Q, R = np.linalg.qr(A)
    Q = Q * np.sign(np.diag(R))[None, :]
    s = np.exp(rng.uniform(np.log(lo), np.log(hi), size=dim))
    M = (Q * s[None, :]) @ Q.T
    return 0.5 * (M + M.T)


def spd_system_from_edges(n, edges, seed, mass=1.0, lo=1e-1, hi=1e2):
    """SPD block system on a given node graph: ``mass * I`` plus one random
    PSD 6x6 coupling per edge; the node graph is the edge list."""
    edges = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    ss = np.random.SeedSequence(seed)
    s_vals, s_rhs = ss.spawn(2)
    rv = np.random.default_rng(s_vals)
    rows, cols, blks = list(range(n)), list(range(n)), [mass * np.eye(3)] * n
    for i, j in edges:
        B = random_psd_block(rv, 6, lo, hi)
        for a, u in enumerate((i, j)):
            for c, v in enumerate((i, j)):
                rows.append(u)
                cols.append(v)
                blks.append(B[3 * a : 3 * a + 3, 3 * c : 3 * c + 3])
    row_ptr, col_idx, val = assemble_bcsr(n, rows, cols, np.array(blks))
    gptr, gadj = graph_from_edges(n, edges)
    b = np.random.default_rng(s_rhs).standard_normal(3 * n)
    return BlockSystem(n=n, row_ptr=row_ptr, col_idx=col_idx, val=val, b=b, gptr=gptr, gadj=gadj,
                       meta={"kind": "edges_spd", "seed": seed})


def random_spd_system(n, n_pairs, seed, mass=1.0, lo=1e-1, hi=1e2, rhs=True, local=None):
    """Random SPD block system: ``mass * I`` plus random PSD 6x6 pair couplings.

    ``local`` (optional int) keeps pairs within that index distance so the
    pattern looks mesh-like.  The node graph is the coupling pattern.
    """
    ss = np.random.SeedSequence(seed)
    s_pairs, s_vals, s_rhs = ss.spawn(3)
    rp = np.random.default_rng(s_pairs)
    pairs = set()
    tries = 0
    while len(pairs) < n_pairs and n > 1 and tries < 100 * max(n_pairs, 1):
        tries += 1
        i = int(rp.integers(n))
        if local:
            j = i + int(rp.integers(-local, local + 1))
            if j < 0 or j >= n:
                continue
        else:
            j = int(rp.integers(n))
        if i == j:
            continue
        pairs.add((min(i, j), max(i, j)))
    pairs = sorted(pairs)
    rv = np.random.default_rng(s_vals)
    rows, cols, blks = [], [], []
    for i in range(n):
        rows.append(i)
        cols.append(i)
        blks.append(mass * np.eye(3))
    for i, j in pairs:
        B = random_psd_block(rv, 6, lo, hi)
        for a, u in enumerate((i, j)):
            for c, v in enumerate((i, j)):
                rows.append(u)
                cols.append(v)
                blks.append(B[3 * a : 3 * a + 3, 3 * c : 3 * c + 3])
    row_ptr, col_idx, val = assemble_bcsr(n, rows, cols, np.array(blks))
    gptr, gadj = graph_from_edges(n, np.array(pairs, dtype=np.int64).reshape(-1, 2))
    b = np.random.default_rng(s_rhs).standard_normal(3 * n) if rhs else np.zeros(3 * n)
    return BlockSystem(
        n=n,
        row_ptr=row_ptr,
        col_idx=col_idx,
        val=val,
        b=b,
        gptr=gptr,
        gadj=gadj,
        meta={"kind": "random_spd", "seed": seed, "pairs": len(pairs)},
    )
