"""Python front end of libmaspcg: argument marshalling over the C ABI.

PyTorch provides device memory (every tensor below lives on the current HIP
device) and the stream (torch's current stream); all arithmetic runs in the
library's HIP kernels.  Nothing here computes on the host.
"""

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import (
    MAS_F32,
    MAS_F64,
    MAS_INVALID_ARG,
    MAS_NOT_CONVERGED,
    MAS_OK,
    MAS_PRECISION_F64,
    MAS_PRECISION_MIXED,
    MasBcsr,
    MasInfo,
    MasOptions,
    PcgOptions,
    MasError,
    PcgResult,
    check,
)

_ALIGN = 256


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _need_cuda(t, name, dtype=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a HIP device tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class BlockMatrix:
    """3x3-block CSR matrix on the device (layout of include/mas_pcg.h)."""

    def __init__(self, row_ptr, col_idx, val):
        _need_cuda(row_ptr, "row_ptr", torch.int32)
        _need_cuda(col_idx, "col_idx", torch.int32)
        _need_cuda(val, "val")
        if val.dtype not in (torch.float64, torch.float32):
            raise ValueError("val must be float64 or float32")
        self.row_ptr, self.col_idx, self.val = row_ptr, col_idx, val
        self.n_rows = row_ptr.numel() - 1
        self.nnzb = col_idx.numel()
        if val.numel() != 9 * self.nnzb:
            raise ValueError("val must hold nnzb 3x3 blocks")

    @classmethod
    def from_numpy(cls, row_ptr, col_idx, val, device="cuda", dtype=torch.float64):
        return cls(
            torch.as_tensor(np.asarray(row_ptr, dtype=np.int32), device=device),
            torch.as_tensor(np.asarray(col_idx, dtype=np.int32), device=device),
            torch.as_tensor(np.ascontiguousarray(val).reshape(-1, 3, 3), device=device).to(dtype),
        )

    def c_struct(self):
        return MasBcsr(
            self.n_rows,
            self.nnzb,
            self.row_ptr.data_ptr(),
            self.col_idx.data_ptr(),
            self.val.data_ptr(),
            MAS_F32 if self.val.dtype == torch.float32 else MAS_F64,
        )


def bcsr_spmv(H, x, out=None):
    """y = H x (FP64 vectors, FP64 or FP32 blocks)."""
    _need_cuda(x, "x", torch.float64)
    if x.numel() != 3 * H.n_rows:
        raise ValueError("x must have 3 * n_rows entries")
    y = torch.empty_like(x) if out is None else out
    _need_cuda(y, "out", torch.float64)
    L = _lib.load()
    h = H.c_struct()
    check("bcsr_spmv", L.bcsr_spmv(ctypes.byref(h), _ptr(x), _ptr(y), _stream()))
    return y


def bcsr_assemble(n_rows, rows, cols, blocks, capacity=None):
    """BlockMatrix from a list of 3x3 blocks on the device (int32 rows / cols
    of shape [m], float64 blocks of shape [m, 3, 3] or [m, 9]): equal
    (row, col) blocks summed in list order.  capacity: output blocks to
    allocate (default m; a second call is made if the result needs more)."""
    _need_cuda(rows, "rows", torch.int32)
    _need_cuda(cols, "cols", torch.int32)
    _need_cuda(blocks, "blocks", torch.float64)
    m = rows.numel()
    if cols.numel() != m or blocks.numel() != 9 * m:
        raise ValueError("rows, cols and blocks must describe the same number of blocks")
    L = _lib.load()
    dev = rows.device
    need = int(L.bcsr_assemble_workspace_size(int(n_rows), m))
    ws = torch.empty(need + _ALIGN, dtype=torch.uint8, device=dev)
    wsp = (ws.data_ptr() + _ALIGN - 1) // _ALIGN * _ALIGN
    cap = m if capacity is None else int(capacity)
    for _ in range(2):
        row_ptr = torch.empty(int(n_rows) + 1, dtype=torch.int32, device=dev)
        col_idx = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        val = torch.empty((max(cap, 1), 3, 3), dtype=torch.float64, device=dev)
        nb = ctypes.c_int64(0)
        rc = L.bcsr_assemble(int(n_rows), m, _ptr(rows), _ptr(cols), _ptr(blocks), _ptr(row_ptr), _ptr(col_idx),
                             _ptr(val), cap, ctypes.byref(nb), ctypes.c_void_p(wsp), need, _stream())
        if rc == MAS_INVALID_ARG and nb.value > cap:
            cap = nb.value
            continue
        check("bcsr_assemble", rc)
        return BlockMatrix(row_ptr, col_idx[: nb.value], val[: nb.value])
    raise MasError("bcsr_assemble", MAS_INVALID_ARG)


def bcsr_assemble_noalloc(n_rows, rows, cols, blocks, row_ptr, col_idx, val):
    """bcsr_assemble into caller-allocated outputs, with the library's
    static device scratch instead of a workspace (no device allocation in
    the call).  row_ptr: int32 [n_rows + 1]; col_idx: int32 [capacity];
    val: float64 [capacity, 3, 3].  Returns the number of distinct blocks."""
    _need_cuda(rows, "rows", torch.int32)
    _need_cuda(cols, "cols", torch.int32)
    _need_cuda(blocks, "blocks", torch.float64)
    _need_cuda(row_ptr, "row_ptr", torch.int32)
    _need_cuda(col_idx, "col_idx", torch.int32)
    _need_cuda(val, "val", torch.float64)
    m = rows.numel()
    if cols.numel() != m or blocks.numel() != 9 * m:
        raise ValueError("rows, cols and blocks must describe the same number of blocks")
    if row_ptr.numel() != int(n_rows) + 1 or val.numel() != 9 * col_idx.numel():
        raise ValueError("row_ptr must hold n_rows + 1 entries and val 9 values per col_idx entry")
    nb = ctypes.c_int64(0)
    rc = _lib.load().bcsr_assemble_noalloc(int(n_rows), m, _ptr(rows), _ptr(cols), _ptr(blocks), _ptr(row_ptr),
                                           _ptr(col_idx), _ptr(val), col_idx.numel(), ctypes.byref(nb), _stream())
    check("bcsr_assemble_noalloc", rc)
    return int(nb.value)


def abd_contact_blocks(n_nodes, node_row, node_is_body, node_xbar, rows, cols, blocks, levels=2):
    """Contact blocks on affine bodies mapped to DOF blocks (two-level
    reduction, Sec. 6.1): returns (rows, cols, blocks[n, 3, 3]) on the
    device, ready for bcsr_assemble with the system's other blocks.
    node_row / node_is_body: int32 [n_nodes]; node_xbar: float64
    [n_nodes, 3]; rows / cols: int32 [m] node indices; blocks: float64
    [m, 3, 3]; levels: 2 (pairs reduced first) or 1 (every block mapped)."""
    for t, name, dt in ((node_row, "node_row", torch.int32), (node_is_body, "node_is_body", torch.int32),
                        (node_xbar, "node_xbar", torch.float64), (rows, "rows", torch.int32),
                        (cols, "cols", torch.int32), (blocks, "blocks", torch.float64)):
        _need_cuda(t, name, dt)
    m = rows.numel()
    L = _lib.load()
    dev = rows.device
    need = int(L.abd_contact_workspace_size(int(n_nodes), m))
    ws = torch.empty(need + _ALIGN, dtype=torch.uint8, device=dev)
    wsp = (ws.data_ptr() + _ALIGN - 1) // _ALIGN * _ALIGN
    cap = 16 * max(m, 1)
    out_r = torch.empty(cap, dtype=torch.int32, device=dev)
    out_c = torch.empty(cap, dtype=torch.int32, device=dev)
    out_b = torch.empty((cap, 3, 3), dtype=torch.float64, device=dev)
    n = ctypes.c_int64(0)
    rc = L.abd_contact_blocks(int(n_nodes), _ptr(node_row), _ptr(node_is_body), _ptr(node_xbar), m, _ptr(rows),
                              _ptr(cols), _ptr(blocks), int(levels), _ptr(out_r), _ptr(out_c), _ptr(out_b), cap,
                              ctypes.byref(n), ctypes.c_void_p(wsp), need, _stream())
    check("abd_contact_blocks", rc)
    k = n.value
    return out_r[:k], out_c[:k], out_b[:k]


class MasPcg:
    """MAS-preconditioned PCG for one sparsity pattern.

    ``MasPcg(row_ptr, col_idx, graph=None, domain_size=16, max_levels=0,
    precision="f64")`` runs the symbolic analysis on host copies of the
    pattern (numpy arrays or CPU tensors); ``graph=(g_ptr, g_adj)`` is the
    node graph to partition (default: the pattern of H).  ``partition=part``
    (an int array of node -> level-0 domain, e.g. ``morton_partition``)
    replaces the connectivity-aware partition.
    """

    def __init__(self, row_ptr, col_idx, graph=None, domain_size=16, max_levels=0, precision="f64", poison=False,
                 partition=None):
        """``poison=True`` fills a new workspace with 0xFF bytes (NaN doubles) so
        that any read of memory the library did not write shows up."""
        self._poison = poison
        L = _lib.load()
        self._L = L
        prec = {"f64": MAS_PRECISION_F64, "mixed": MAS_PRECISION_MIXED}[precision]
        self.precision = precision
        opts = MasOptions(int(domain_size), int(max_levels), prec, 0)
        h = ctypes.c_void_p()
        check("mas_create", L.mas_create(ctypes.byref(opts), ctypes.byref(h)))
        self._h = h
        rp = np.ascontiguousarray(np.asarray(row_ptr), dtype=np.int32)
        ci = np.ascontiguousarray(np.asarray(col_idx), dtype=np.int32)
        n = rp.size - 1
        if graph is not None:
            gp = np.ascontiguousarray(np.asarray(graph[0]), dtype=np.int32)
            ga = np.ascontiguousarray(np.asarray(graph[1]), dtype=np.int32)
            if ga.size == 0:
                ga = np.zeros(1, np.int32)
            gpp, gap = gp.ctypes.data_as(ctypes.c_void_p), ga.ctypes.data_as(ctypes.c_void_p)
        else:
            gpp = gap = None
        if partition is not None:
            part = np.ascontiguousarray(np.asarray(partition), dtype=np.int32)
            if part.size != n:
                raise ValueError("partition needs one domain id per node")
            check(
                "mas_analyze_partition",
                L.mas_analyze_partition(h, n, ci.size, rp.ctypes.data_as(ctypes.c_void_p),
                                        ci.ctypes.data_as(ctypes.c_void_p), part.ctypes.data_as(ctypes.c_void_p),
                                        int(part.max()) + 1 if part.size else 0),
            )
        else:
            check(
                "mas_analyze",
                L.mas_analyze(h, n, ci.size, rp.ctypes.data_as(ctypes.c_void_p), ci.ctypes.data_as(ctypes.c_void_p),
                              gpp, gap),
            )
        self.n_rows = n
        self.nnzb = int(ci.size)
        self._ws = None
        self._ws_ptr = 0

    def close(self):
        if getattr(self, "_h", None):
            self._L.mas_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    # ------------------------------------------------------------ queries
    def info(self):
        inf = MasInfo()
        check("mas_get_info", self._L.mas_get_info(self._h, ctypes.byref(inf)))
        lv = inf.levels
        return {
            "n_rows": inf.n_rows,
            "nnzb": inf.nnzb,
            "domain_size": inf.domain_size,
            "parts": inf.parts,
            "slack": inf.slack,
            "levels": lv,
            "units": list(inf.units[:lv]),
            "domains": list(inf.domains[:lv]),
            "coarse_nnzb": list(inf.coarse_nnzb[:lv]),
            "workspace_bytes": int(inf.workspace_bytes),
            "inverse_bytes": int(inf.inverse_bytes),
            "stored_blocks": int(inf.stored_blocks),
        }

    def ordering(self):
        """Host copies ``(map[V], remap[M*N], sn[levels, V])``."""
        inf = self.info()
        mp = np.empty(self.n_rows, np.int32)
        rm = np.empty(inf["parts"] * inf["domain_size"], np.int32)
        sn = np.empty((inf["levels"], self.n_rows), np.int32)
        check(
            "mas_get_ordering",
            self._L.mas_get_ordering(
                self._h, mp.ctypes.data_as(ctypes.c_void_p), rm.ctypes.data_as(ctypes.c_void_p), sn.ctypes.data_as(ctypes.c_void_p)
            ),
        )
        return mp, rm, sn

    def inverses(self, level, precision=None):
        """Host copy of level ``level``'s domain inverses after :meth:`build`:
        array [ndom, 3N, 3N] (zero rows/columns on unoccupied lanes).
        ``precision="mixed"`` reads the FP32 copy of a mixed handle."""
        inf = self.info()
        n = 3 * inf["domain_size"]
        out = np.empty((inf["domains"][level], n, n), np.float64)
        prec = {"f64": MAS_PRECISION_F64, "mixed": MAS_PRECISION_MIXED}[precision or "f64"]
        check("mas_get_inverses",
              self._L.mas_get_inverses(self._h, int(level), prec, out.ctypes.data_as(ctypes.c_void_p), _stream()))
        # stored column-major per domain: transpose to row-major (a no-op for exact symmetry)
        return out.transpose(0, 2, 1).copy()

    def hierarchy_device(self, device=None):
        """Supernode hierarchy rebuilt on the device from the analysed pattern.

        Returns ``(units[levels], sn[levels, V])`` in the layout of
        :meth:`info` / :meth:`ordering`; the construction runs in the library's
        kernels on torch's current stream (its scratch is a device tensor).
        """
        dev = torch.device("cuda") if device is None else torch.device(device)
        need = int(self._L.mas_hierarchy_workspace_size(self._h))
        if need == 0:
            raise MasError("mas_hierarchy_workspace_size", MAS_INVALID_ARG)
        ws = torch.empty(need + _ALIGN, dtype=torch.uint8, device=dev)
        base = (ws.data_ptr() + _ALIGN - 1) // _ALIGN * _ALIGN
        levels = ctypes.c_int32(0)
        units = np.zeros(_lib.MAS_MAX_LEVELS, np.int32)
        sn = np.empty((_lib.MAS_MAX_LEVELS, self.n_rows), np.int32)
        check(
            "mas_hierarchy_device",
            self._L.mas_hierarchy_device(
                self._h, ctypes.byref(levels), units.ctypes.data_as(ctypes.c_void_p),
                sn.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(base), ctypes.c_size_t(need), _stream()
            ),
        )
        L = levels.value
        return units[:L].copy(), sn[:L].copy()

    def hierarchy_rebuild(self, row_ptr, col_idx):
        """Supernode hierarchy of a new block pattern (device int32 row_ptr /
        col_idx in node order, e.g. after contacts changed) under the analysed
        partition, built on the device with no host round trip.

        Returns device tensors ``(units[MAS_MAX_LEVELS + 1], sn[MAS_MAX_LEVELS,
        V])``: ``units[0]`` is the level count (-1: an index outside the
        pattern), ``units[1 + l]`` the units of level l; ``sn[l, i]`` the unit
        of node i at level l (-1 past the last level).
        """
        _need_cuda(row_ptr, "row_ptr", torch.int32)
        _need_cuda(col_idx, "col_idx", torch.int32)
        if row_ptr.numel() != self.n_rows + 1:
            raise ValueError("row_ptr must have n_rows + 1 entries")
        dev = row_ptr.device
        need = int(self._L.mas_hierarchy_workspace_size(self._h))
        if need == 0:
            raise MasError("mas_hierarchy_workspace_size", MAS_INVALID_ARG)
        ws = torch.empty(need + _ALIGN, dtype=torch.uint8, device=dev)
        base = (ws.data_ptr() + _ALIGN - 1) // _ALIGN * _ALIGN
        units = torch.empty(_lib.MAS_MAX_LEVELS + 1, dtype=torch.int32, device=dev)
        sn = torch.empty((_lib.MAS_MAX_LEVELS, self.n_rows), dtype=torch.int32, device=dev)
        check("mas_hierarchy_rebuild",
              self._L.mas_hierarchy_rebuild(self._h, col_idx.numel(), _ptr(row_ptr), _ptr(col_idx), _ptr(units),
                                            _ptr(sn), ctypes.c_void_p(base), ctypes.c_size_t(need), _stream()))
        self._hier_ws = ws  # kept until the next call: the queued kernels use it
        return units, sn

    def replan(self, row_ptr, col_idx):
        """Every solver plan of a new block pattern (device int32 row_ptr /
        col_idx in node order, e.g. after contacts changed) derived on the
        device under the analysed partition; the next :meth:`build` takes a
        matrix of that pattern.  The scratch holding the plans is kept with
        the handle."""
        _need_cuda(row_ptr, "row_ptr", torch.int32)
        _need_cuda(col_idx, "col_idx", torch.int32)
        if row_ptr.numel() != self.n_rows + 1:
            raise ValueError("row_ptr must have n_rows + 1 entries")
        nnzb = col_idx.numel()
        need = int(self._L.mas_replan_workspace_size(self._h, nnzb))
        if need == 0:
            raise MasError("mas_replan_workspace_size", MAS_INVALID_ARG)
        ws = torch.empty(need + _ALIGN, dtype=torch.uint8, device=row_ptr.device)
        base = (ws.data_ptr() + _ALIGN - 1) // _ALIGN * _ALIGN
        check("mas_replan", self._L.mas_replan(self._h, nnzb, _ptr(row_ptr), _ptr(col_idx), ctypes.c_void_p(base),
                                               ctypes.c_size_t(need), _stream()))
        self._replan_ws = ws  # holds the plans until the handle is re-analysed or re-planned
        self.nnzb = int(nnzb)
        return self

    def timings(self):
        """Device ms of [coarse sums, inversion, H permute, PCG iterations] of the last calls."""
        out = (ctypes.c_double * 4)()
        check("mas_get_timings", self._L.mas_get_timings(self._h, out))
        return list(out)

    KERNEL_SLOTS = ("spmv", "update", "apply_coarse", "apply_level0", "level0_update", "residual", "permute_H",
                    "restrict")

    def set_kernel_timing(self, enable=True):
        check("mas_set_kernel_timing", self._L.mas_set_kernel_timing(self._h, int(bool(enable))))

    def kernel_timing(self):
        """{slot: (total_ms, launches)} accumulated since set_kernel_timing."""
        tot = (ctypes.c_double * 8)()
        cnt = (ctypes.c_int32 * 8)()
        check("mas_get_kernel_timing", self._L.mas_get_kernel_timing(self._h, tot, cnt))
        return {k: (tot[i], cnt[i]) for i, k in enumerate(self.KERNEL_SLOTS)}

    def workspace_size(self):
        return int(self._L.mas_workspace_size(self._h))

    # ------------------------------------------------------------- phases
    def _workspace(self, device):
        need = self.workspace_size()
        if self._ws is None or self._ws.numel() < need + _ALIGN or self._ws.device != device:
            self._ws = torch.empty(need + _ALIGN, dtype=torch.uint8, device=device)
            if self._poison:
                self._ws.fill_(255)
        base = self._ws.data_ptr()
        self._ws_ptr = (base + _ALIGN - 1) // _ALIGN * _ALIGN
        return self._ws_ptr, need

    def build(self, H):
        """Numeric phase on the device: coarse matrices and domain inverses."""
        if H.val.dtype != torch.float64:
            raise ValueError("mas_build needs FP64 values")
        ptr, need = self._workspace(H.val.device)
        h = H.c_struct()
        check("mas_build", self._L.mas_build(self._h, ctypes.byref(h), ctypes.c_void_p(ptr), need, _stream()))
        return self

    def apply(self, r, out=None):
        """z = M^-1 r."""
        _need_cuda(r, "r", torch.float64)
        z = torch.empty_like(r) if out is None else out
        check("mas_apply", self._L.mas_apply(self._h, _ptr(r), _ptr(z), _stream()))
        return z

    @staticmethod
    def _opts(tol, max_iter, x0_given, replace_every, check_every):
        return PcgOptions(float(tol), int(max_iter), int(x0_given), int(replace_every), int(check_every))

    @staticmethod
    def _result(res):
        return {
            "status": res.status,
            "iterations": res.iterations,
            "rel_residual": res.rel_residual,
            "true_rel_residual": res.true_rel_residual,
        }

    def solve(self, H, b, tol=1e-4, max_iter=10000, x0=None, out=None, replace_every=50, check_every=8, allow_not_converged=True):
        """Returns ``(x, result)``; raises MasError on failure."""
        _need_cuda(b, "b", torch.float64)
        x = out if out is not None else torch.empty_like(b)
        if x0 is not None:
            x.copy_(x0)
        opts = self._opts(tol, max_iter, x0 is not None, replace_every, check_every)
        res = PcgResult()
        h = H.c_struct()
        rc = self._L.pcg_solve(self._h, ctypes.byref(h), _ptr(b), _ptr(x), ctypes.byref(opts), ctypes.byref(res), _stream())
        check("pcg_solve", rc, (MAS_OK, MAS_NOT_CONVERGED) if allow_not_converged else (MAS_OK,))
        return x, self._result(res)

    def adjoint(self, H, x, dLdx, dLdH_dtype=torch.float64, want_dH=True, tol=1e-4, max_iter=10000, replace_every=50, check_every=8,
                allow_not_converged=True):
        """Returns ``(lambda = dL/db, dL/dH blocks or None, result)``; raises
        MasError on failure (also on MAS_NOT_CONVERGED when
        ``allow_not_converged`` is False)."""
        _need_cuda(x, "x", torch.float64)
        _need_cuda(dLdx, "dLdx", torch.float64)
        lam = torch.empty_like(dLdx)
        dH = None
        if want_dH:
            if dLdH_dtype not in (torch.float64, torch.float32):
                raise ValueError("dLdH_dtype must be float64 or float32")
            dH = torch.empty((H.nnzb, 3, 3), dtype=dLdH_dtype, device=x.device)
        opts = self._opts(tol, max_iter, 0, replace_every, check_every)
        res = PcgResult()
        h = H.c_struct()
        rc = self._L.pcg_adjoint(
            self._h,
            ctypes.byref(h),
            _ptr(x),
            _ptr(dLdx),
            _ptr(lam),
            _ptr(dH),
            MAS_F32 if dLdH_dtype == torch.float32 else MAS_F64,
            ctypes.byref(opts),
            ctypes.byref(res),
            _stream(),
        )
        check("pcg_adjoint", rc, (MAS_OK, MAS_NOT_CONVERGED) if allow_not_converged else (MAS_OK,))
        return lam, dH, self._result(res)
