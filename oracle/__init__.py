"""CPU oracle for the connectivity-enhanced MAS-preconditioned PCG solve.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product path
never calls it.  The arithmetic lives in ``oracle.c`` (plain C, FP64, single
thread, no FMA contraction); this module only marshals numpy arrays.
"""

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, NOT_CONVERGED, INVALID, NOT_SPD = 0, 1, -1, -2
DOT_SEQUENTIAL, DOT_COMPENSATED = 0, 1
MAX_LEVELS = 16


def build(force=True):
    """Compile ``oracle.c`` into ``liboracle.so`` (gcc, -O2, no FMA contraction)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    cmd = [
        "gcc",
        "-O2",
        "-std=c11",
        "-ffp-contract=off",
        "-fno-fast-math",
        "-fPIC",
        "-shared",
        "-Wall",
        "-o",
        _LIB + ".tmp",
        _SRC,
        "-lm",
    ]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None

_i = ctypes.c_int
_d = ctypes.c_double
_pi = ctypes.POINTER(ctypes.c_int)
_pd = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.orc_partition.argtypes = [_i, _pi, _pi, _i, _pi, _pi, _pi]
        L.orc_slots.argtypes = [_i, _pi, _i, _i, _pi, _pi]
        L.orc_mas_build.argtypes = [_i, _pi, _pi, _pd, _pi, _pi, _i, _i, _pi]
        L.orc_mas_build.restype = _vp
        L.orc_mas_build_parts.argtypes = [_i, _pi, _pi, _pd, _pi, _i, _i, _i, _pi]
        L.orc_mas_build_parts.restype = _vp
        L.orc_mas_free.argtypes = [_vp]
        for f in ("orc_mas_levels", "orc_mas_parts", "orc_mas_slack"):
            getattr(L, f).argtypes = [_vp]
        L.orc_mas_units.argtypes = [_vp, _i]
        L.orc_mas_domains.argtypes = [_vp, _i]
        L.orc_mas_get_map.argtypes = [_vp, _pi, _pi]
        L.orc_mas_get_sn.argtypes = [_vp, _i, _pi]
        L.orc_mas_get_domain_matrix.argtypes = [_vp, _i, _i, _pd]
        L.orc_mas_get_inverse.argtypes = [_vp, _i, _i, _pd]
        L.orc_mas_apply.argtypes = [_vp, _pd, _pd]
        L.orc_mas_perturb.argtypes = [_vp, _d, ctypes.c_ulonglong]
        L.orc_spmv.argtypes = [_i, _pi, _pi, _pd, _pd, _pd]
        L.orc_pcg.argtypes = [_i, _pi, _pi, _pd, _vp, _pd, _pd, _d, _i, _pi, _pd, _pd]
        L.orc_pcg_dots.argtypes = [_i, _pi, _pi, _pd, _vp, _pd, _pd, _d, _i, _i, _pi, _pd, _pd]
        L.orc_dot.argtypes = [_i, _pd, _pd, _i]
        L.orc_dot.restype = _d
        L.orc_adjoint_scatter.argtypes = [_i, _pi, _pi, _pd, _pd, _pd]
        L.orc_assemble.argtypes = [_i, ctypes.c_long, _pi, _pi, _pd, _pi, _pi, _pd]
        L.orc_assemble.restype = ctypes.c_long
        L.orc_abd_expand.argtypes = [_i, _pi, _pi, _pd, ctypes.c_long, _pi, _pi, _pd, _pi, _pi, _pd]
        L.orc_abd_expand.restype = ctypes.c_long
        _lib = L
    return _lib


def _ci(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_pi)


def _cd(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_pd)


def partition(V, gptr, gadj, N):
    """Returns ``(part[V], M, N_o)``."""
    gp, gpp = _ci(gptr)
    ga, gap = _ci(gadj if len(gadj) else np.zeros(1, np.int32))
    part = np.empty(V, np.int32)
    M, No = ctypes.c_int(), ctypes.c_int()
    s = lib().orc_partition(V, gpp, gap, N, part.ctypes.data_as(_pi), ctypes.byref(M), ctypes.byref(No))
    if s != OK:
        raise RuntimeError(f"orc_partition failed ({s})")
    return part, M.value, No.value


def slots(part, M, N):
    part, pp = _ci(part)
    V = part.size
    mp = np.empty(V, np.int32)
    rm = np.empty(M * N, np.int32)
    s = lib().orc_slots(V, pp, M, N, mp.ctypes.data_as(_pi), rm.ctypes.data_as(_pi))
    if s != OK:
        raise RuntimeError(f"orc_slots failed ({s})")
    return mp, rm


def spmv(row_ptr, col_idx, val, x):
    rp, rpp = _ci(row_ptr)
    ci, cip = _ci(col_idx)
    v, vp = _cd(np.asarray(val).reshape(-1))
    x, xp = _cd(x)
    n = rp.size - 1
    y = np.empty(3 * n)
    lib().orc_spmv(n, rpp, cip, vp, xp, y.ctypes.data_as(_pd))
    return y


def dot(a, b, mode=DOT_SEQUENTIAL):
    """a . b as the oracle's PCG forms it: ``DOT_SEQUENTIAL`` (ascending, working
    precision) or ``DOT_COMPENSATED`` (Dot2 of Ogita, Rump and Oishi)."""
    a, ap = _cd(a)
    b, bp = _cd(b)
    if a.size != b.size:
        raise ValueError("dot of vectors of different lengths")
    return lib().orc_dot(int(a.size), ap, bp, int(mode))


def adjoint_scatter(row_ptr, col_idx, lam, x):
    rp, rpp = _ci(row_ptr)
    ci, cip = _ci(col_idx)
    lam, lp = _cd(lam)
    x, xp = _cd(x)
    n = rp.size - 1
    out = np.empty((ci.size, 3, 3))
    lib().orc_adjoint_scatter(n, rpp, cip, lp, xp, out.ctypes.data_as(_pd))
    return out


def assemble(n, rows, cols, blocks):
    """BCSR (row_ptr, col_idx, val[nnzb, 3, 3]) of a block list: equal
    (row, col) blocks summed in list order."""
    r, rp = _ci(rows)
    c, cp = _ci(cols)
    b, bp = _cd(np.asarray(blocks, dtype=np.float64).reshape(-1))
    m = r.size
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    col_idx = np.zeros(max(m, 1), dtype=np.int32)
    val = np.zeros((max(m, 1), 3, 3))
    nb = lib().orc_assemble(int(n), m, rp, cp, bp, row_ptr.ctypes.data_as(_pi), col_idx.ctypes.data_as(_pi),
                            val.ctypes.data_as(_pd))
    if nb < 0:
        raise ValueError("block index out of range")
    return row_ptr, col_idx[:nb], val[:nb]


def abd_expand(node_row, node_is_body, node_xbar, rows, cols, blocks):
    """Contact blocks on affine bodies as DOF-block sub-blocks (J_r^T C J_c of
    every listed block, list order, Sec. 6.1): (rows, cols, blocks[n, 3, 3])."""
    nr, nrp = _ci(node_row)
    nb_, nbp = _ci(node_is_body)
    xb, xbp = _cd(np.asarray(node_xbar, dtype=np.float64).reshape(-1))
    r, rp = _ci(rows)
    c, cp = _ci(cols)
    b, bp = _cd(np.asarray(blocks, dtype=np.float64).reshape(-1))
    m = r.size
    out_r = np.zeros(16 * max(m, 1), dtype=np.int32)
    out_c = np.zeros(16 * max(m, 1), dtype=np.int32)
    out_b = np.zeros((16 * max(m, 1), 3, 3))
    k = lib().orc_abd_expand(int(nr.size), nrp, nbp, xbp, m, rp, cp, bp, out_r.ctypes.data_as(_pi),
                             out_c.ctypes.data_as(_pi), out_b.ctypes.data_as(_pd))
    if k < 0:
        raise ValueError("node index out of range")
    return out_r[:k], out_c[:k], out_b[:k]


class MAS:
    """The oracle's MAS preconditioner for one system.

    ``MAS(row_ptr, col_idx, val, N=16, max_levels=0, gptr=None, gadj=None)``
    partitions (graph or the pattern of H), builds the hierarchy and inverts
    every domain.  ``MAS.from_parts`` takes a given partition instead.
    """

    def __init__(self, row_ptr, col_idx, val, N=16, max_levels=0, gptr=None, gadj=None, part=None, M=None):
        self._rp, rpp = _ci(row_ptr)
        self._ci, cip = _ci(col_idx)
        self._val, vp = _cd(np.asarray(val).reshape(-1))
        self.V = self._rp.size - 1
        self.N = int(N)
        st = ctypes.c_int()
        if part is not None:
            pa, pap = _ci(part)
            self._h = lib().orc_mas_build_parts(self.V, rpp, cip, vp, pap, int(M), self.N, int(max_levels), ctypes.byref(st))
        else:
            if gptr is not None:
                gp, gpp = _ci(gptr)
                ga, gap = _ci(gadj if len(gadj) else np.zeros(1, np.int32))
            else:
                gpp = gap = None
            self._h = lib().orc_mas_build(self.V, rpp, cip, vp, gpp, gap, self.N, int(max_levels), ctypes.byref(st))
        self.status = st.value
        if not self._h:
            raise RuntimeError(f"orc_mas_build failed ({self.status})")

    @classmethod
    def from_parts(cls, row_ptr, col_idx, val, part, M, N, max_levels=0):
        return cls(row_ptr, col_idx, val, N=N, max_levels=max_levels, part=part, M=M)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_mas_free(h)
            self._h = None

    @property
    def levels(self):
        return lib().orc_mas_levels(self._h)

    @property
    def parts(self):
        return lib().orc_mas_parts(self._h)

    @property
    def slack(self):
        return lib().orc_mas_slack(self._h)

    def units(self, l):
        return lib().orc_mas_units(self._h, l)

    def domains(self, l):
        return lib().orc_mas_domains(self._h, l)

    def maps(self):
        mp = np.empty(self.V, np.int32)
        rm = np.empty(self.parts * self.N, np.int32)
        lib().orc_mas_get_map(self._h, mp.ctypes.data_as(_pi), rm.ctypes.data_as(_pi))
        return mp, rm

    def sn(self, l):
        out = np.empty(self.V, np.int32)
        lib().orc_mas_get_sn(self._h, l, out.ctypes.data_as(_pi))
        return out

    def domain_matrix(self, l, d):
        n3 = 3 * self.N
        out = np.empty((n3, n3))
        lib().orc_mas_get_domain_matrix(self._h, l, d, out.ctypes.data_as(_pd))
        return out

    def inverse(self, l, d):
        n3 = 3 * self.N
        out = np.empty((n3, n3))
        lib().orc_mas_get_inverse(self._h, l, d, out.ctypes.data_as(_pd))
        return out

    def perturb(self, eps, seed):
        """Scales every inverse entry by (1 + eps u), u ~ U[-1, 1) from
        SplitMix64 at (seed, entry index), keeping each inverse symmetric.
        Test infrastructure for the iteration-count contract only."""
        lib().orc_mas_perturb(self._h, float(eps), int(seed))

    def apply(self, r):
        r, rp_ = _cd(r)
        z = np.empty(3 * self.V)
        lib().orc_mas_apply(self._h, rp_, z.ctypes.data_as(_pd))
        return z

    def pcg(self, b, tol=1e-8, max_iter=10000, dots=DOT_SEQUENTIAL):
        """Returns ``(x, status, iterations, rel_residual, true_rel_residual)``;
        ``dots`` selects how the dot products are summed (see :func:`dot`)."""
        b, bp = _cd(b)
        x = np.empty(3 * self.V)
        it, rr, tr = ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
        s = lib().orc_pcg_dots(
            self.V,
            self._rp.ctypes.data_as(_pi),
            self._ci.ctypes.data_as(_pi),
            self._val.ctypes.data_as(_pd),
            self._h,
            bp,
            x.ctypes.data_as(_pd),
            float(tol),
            int(max_iter),
            int(dots),
            ctypes.byref(it),
            ctypes.byref(rr),
            ctypes.byref(tr),
        )
        return x, s, it.value, rr.value, tr.value
