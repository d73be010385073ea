"""Named synthetic Newton systems.

Each workload is a pure function of its parameters and seed:

* ``cube_system`` -- an ``n^3`` grid of unit cubes (5 tets each) with spacing
  ``h_x``, current nodes displaced by uniform noise of +-10 % of the spacing,
  ``H = M + dt^2 * sum_e PSD(K_e)`` with Stable Neo-Hookean element Hessians
  and lumped mass, optional contact-like couplings between surface-node pairs
  that are not mesh neighbours (each a random PSD 6x6 block
  ``Q diag(logU[1e2, 1e6]) Q^T``, added unscaled), and ``b ~ N(0, 1)``.
* ``config_small``  -- the 8^3 cube (729 nodes, 2560 tets, 2187 DOF),
  E = 1e5 Pa, nu = 0.4, no contacts.
* ``config_large``  -- the 48^3 cube (117,649 nodes, 552,960 tets,
  352,947 DOF), nu = 0.49, E in {1e4, 1e6, 1e8} Pa, 20,000 contact pairs.
* ``config_tiny``   -- 1^3 .. 4^3 cubes for brute-force checks.
* ``config_membrane`` -- a 512 x 512-cell triangle sheet (263,169 nodes)
  with strain-limiting and bending Hessians, coupled to 2,000 affine bodies
  (8,000 block rows) by random 15x15 blocks (``synth.membrane``).
"""

import numpy as np

from .bcsr import BlockSystem, assemble_bcsr, graph_from_edges, random_psd_block
from .fem import lumped_mass, snh_element_hessians
from .membrane import membrane_system
from .mesh import cube_surface_nodes, mesh_edges, tet_cube


def _contact_pairs(n, edges, n_pairs, rng, max_dist=2.0):
    """Unique surface-node pairs, not mesh-adjacent, rest-grid distance <= max_dist
    spacings, sampled uniformly without replacement."""
    m = n + 1
    surf = cube_surface_nodes(n)
    on = np.zeros(m ** 3, dtype=bool)
    on[surf] = True
    r = int(np.floor(max_dist))
    offs = []
    for dk in range(-r, r + 1):
        for dj in range(-r, r + 1):
            for di in range(-r, r + 1):
                if (di, dj, dk) <= (0, 0, 0):
                    continue  # keep one orientation of each offset
                if di * di + dj * dj + dk * dk <= max_dist * max_dist + 1e-12:
                    offs.append((di, dj, dk))
    si = surf % m
    sj = (surf // m) % m
    sk = surf // (m * m)
    cand = []
    for di, dj, dk in offs:
        ti, tj, tk = si + di, sj + dj, sk + dk
        ok = (ti >= 0) & (ti < m) & (tj >= 0) & (tj < m) & (tk >= 0) & (tk < m)
        t = ti + m * (tj + m * tk)
        ok &= on[np.where(ok, t, 0)]
        a, b = surf[ok], t[ok]
        cand.append(np.stack([np.minimum(a, b), np.maximum(a, b)], axis=1))
    cand = np.unique(np.concatenate(cand, axis=0), axis=0)
    ekey = set((edges[:, 0] * m ** 3 + edges[:, 1]).tolist())
    keep = np.array([(a * m ** 3 + b) not in ekey for a, b in cand], dtype=bool)
    cand = cand[keep]
    if n_pairs > cand.shape[0]:
        raise ValueError(f"only {cand.shape[0]} contact candidates for {n_pairs} pairs")
    pick = rng.choice(cand.shape[0], size=n_pairs, replace=False)
    pick.sort()
    return cand[pick], cand.shape[0]


def cube_system(
    n,
    E,
    nu,
    spacing=0.05,
    density=1000.0,
    dt=0.01,
    noise=0.1,
    n_contacts=0,
    seed=0,
    keep_blocks=False,
):
    ss = np.random.SeedSequence(seed)
    s_noise, s_rhs, s_pairs, s_q = ss.spawn(4)
    rest, tets = tet_cube(n, spacing)
    V = rest.shape[0]
    x = rest + np.random.default_rng(s_noise).uniform(-noise * spacing, noise * spacing, rest.shape)
    K, vol = snh_element_hessians(rest, x, tets, E, nu)
    mass = lumped_mass(tets, vol, V, density)
    edges = mesh_edges(tets)

    # element contributions: 16 blocks per tet
    nt = tets.shape[0]
    a_idx, b_idx = np.meshgrid(np.arange(4), np.arange(4), indexing="ij")
    a_idx, b_idx = a_idx.ravel(), b_idx.ravel()
    rows = tets[:, a_idx].ravel()
    cols = tets[:, b_idx].ravel()
    Kb = (dt * dt) * K.reshape(nt, 4, 3, 4, 3).transpose(0, 1, 3, 2, 4)
    blocks = Kb[:, a_idx, b_idx].reshape(-1, 3, 3)
    del K, Kb

    mrows = np.arange(V)
    mblocks = mass[:, None, None] * np.eye(3)[None]
    parts_r, parts_c, parts_b = [rows, mrows], [cols, mrows], [blocks, mblocks]

    meta = {
        "kind": "tet_cube",
        "cubes": n,
        "nodes": V,
        "tets": nt,
        "E": E,
        "nu": nu,
        "spacing": spacing,
        "density": density,
        "dt": dt,
        "noise": noise,
        "seed": seed,
        "mesh_edges": int(edges.shape[0]),
        "contacts": int(n_contacts),
        "positions": x,  # current node positions (V, 3)
    }
    if n_contacts:
        pairs, pool = _contact_pairs(n, edges, n_contacts, np.random.default_rng(s_pairs))
        rq = np.random.default_rng(s_q)
        cb = np.stack([random_psd_block(rq, 6, 1e2, 1e6) for _ in range(n_contacts)])
        cb = cb.reshape(-1, 2, 3, 2, 3).transpose(0, 1, 3, 2, 4)
        for u in range(2):
            for v in range(2):
                parts_r.append(pairs[:, u])
                parts_c.append(pairs[:, v])
                parts_b.append(cb[:, u, v])
        meta["contact_pool"] = int(pool)
    all_r, all_c, all_b = np.concatenate(parts_r), np.concatenate(parts_c), np.concatenate(parts_b)
    row_ptr, col_idx, val = assemble_bcsr(V, all_r, all_c, all_b)
    if keep_blocks:  # the unassembled block list (row, col, 3x3), in generation order
        meta["blocks"] = (all_r.astype(np.int32), all_c.astype(np.int32), all_b)
    gptr, gadj = graph_from_edges(V, edges)
    b = np.random.default_rng(s_rhs).standard_normal(3 * V)
    meta["nnzb"] = int(col_idx.size)
    return BlockSystem(n=V, row_ptr=row_ptr, col_idx=col_idx, val=val, b=b, gptr=gptr, gadj=gadj, meta=meta)


def config_tiny(n=2, E=1e5, nu=0.4, seed=999):
    return cube_system(n, E, nu, seed=seed)


def config_small(seed=1000):
    """8^3 cube, E = 1e5 Pa, nu = 0.4, no contacts."""
    return cube_system(8, 1e5, 0.4, seed=seed)


def config_large(E=1e6, seed=1001, n_contacts=20000, keep_blocks=False):
    """48^3 cube, nu = 0.49, given E, 20,000 contact-like pairs."""
    return cube_system(48, E, 0.49, n_contacts=n_contacts, seed=seed, keep_blocks=keep_blocks)


def config_membrane(cells=512, n_bodies=2000, seed=1003):
    """Stiff membrane plus affine bodies: 512^2 cells (263,169 nodes,
    524,288 triangles, 785,408 bending pairs), 2,000 bodies of 4 block rows,
    16 coupled sheet nodes each: 271,169 block rows."""
    return membrane_system(cells, n_bodies, seed=seed)


WORKLOADS = {
    "cube8": config_small,
    "cube48": config_large,
    "membrane512": config_membrane,
}
