"""ctypes declarations of the C ABI in include/mas_pcg.h (argument marshalling only)."""

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmaspcg.so")

MAS_OK = 0
MAS_NOT_CONVERGED = 1
MAS_INVALID_ARG = -1
MAS_NOT_SPD = -2
MAS_HIP_ERROR = -3
MAS_WORKSPACE_TOO_SMALL = -4
MAS_NOT_READY = -5
MAS_NOT_FINITE = -6

MAS_F64 = 0
MAS_F32 = 1
MAS_PRECISION_F64 = 0
MAS_PRECISION_MIXED = 1
MAS_MAX_LEVELS = 16
MAS_MAX_DOMAIN_SIZE = 40
MAS_NOALLOC_SCRATCH_BYTES = 64 << 20

SYMBOLS = (
    "mas_create",
    "mas_destroy",
    "mas_analyze",
    "mas_analyze_partition",
    "mas_morton_workspace_size",
    "mas_morton_partition",
    "mas_workspace_size",
    "mas_build",
    "mas_apply",
    "bcsr_spmv",
    "bcsr_assemble_workspace_size",
    "bcsr_assemble",
    "bcsr_assemble_noalloc",
    "abd_contact_workspace_size",
    "abd_contact_blocks",
    "pcg_solve",
    "pcg_adjoint",
    "mas_hierarchy_workspace_size",
    "mas_hierarchy_device",
    "mas_hierarchy_rebuild",
    "mas_replan_workspace_size",
    "mas_replan",
    "mas_get_info",
    "mas_get_ordering",
    "mas_get_inverses",
    "mas_get_timings",
    "mas_set_kernel_timing",
    "mas_get_kernel_timing",
    "mas_status_string",
)


class MasBcsr(ctypes.Structure):
    _fields_ = [
        ("n_rows", ctypes.c_int32),
        ("nnzb", ctypes.c_int32),
        ("row_ptr", ctypes.c_void_p),
        ("col_idx", ctypes.c_void_p),
        ("val", ctypes.c_void_p),
        ("dtype", ctypes.c_int32),
    ]


class MasOptions(ctypes.Structure):
    _fields_ = [
        ("domain_size", ctypes.c_int32),
        ("max_levels", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class PcgOptions(ctypes.Structure):
    _fields_ = [
        ("tol", ctypes.c_double),
        ("max_iter", ctypes.c_int32),
        ("x0_given", ctypes.c_int32),
        ("replace_every", ctypes.c_int32),
        ("check_every", ctypes.c_int32),
    ]


class PcgResult(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("iterations", ctypes.c_int32),
        ("rel_residual", ctypes.c_double),
        ("true_rel_residual", ctypes.c_double),
    ]


class MasInfo(ctypes.Structure):
    _fields_ = [
        ("n_rows", ctypes.c_int32),
        ("nnzb", ctypes.c_int32),
        ("domain_size", ctypes.c_int32),
        ("parts", ctypes.c_int32),
        ("slack", ctypes.c_int32),
        ("levels", ctypes.c_int32),
        ("units", ctypes.c_int32 * MAS_MAX_LEVELS),
        ("domains", ctypes.c_int32 * MAS_MAX_LEVELS),
        ("coarse_nnzb", ctypes.c_int32 * MAS_MAX_LEVELS),
        ("workspace_bytes", ctypes.c_int64),
        ("inverse_bytes", ctypes.c_int64),
        ("stored_blocks", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


_lib = None


class LibraryMissing(RuntimeError):
    pass


def load():
    """Loads libmaspcg.so; raises LibraryMissing if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing(
            f"{LIB_PATH} is missing: build it with paper_2411_06224_amd.build.build() (hipcc, gfx950)"
        )
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    P = ctypes.POINTER
    L.mas_create.argtypes = [P(MasOptions), P(vp)]
    L.mas_create.restype = ctypes.c_int
    L.mas_destroy.argtypes = [vp]
    L.mas_destroy.restype = None
    L.mas_analyze.argtypes = [vp, i32, i32, vp, vp, vp, vp]
    L.mas_analyze.restype = ctypes.c_int
    L.mas_analyze_partition.argtypes = [vp, i32, i32, vp, vp, vp, i32]
    L.mas_analyze_partition.restype = ctypes.c_int
    L.mas_morton_workspace_size.argtypes = [i32]
    L.mas_morton_workspace_size.restype = sz
    L.mas_morton_partition.argtypes = [i32, vp, i32, vp, vp, sz, vp]
    L.mas_morton_partition.restype = ctypes.c_int
    L.mas_workspace_size.argtypes = [vp]
    L.mas_workspace_size.restype = sz
    L.mas_build.argtypes = [vp, P(MasBcsr), vp, sz, vp]
    L.mas_build.restype = ctypes.c_int
    L.mas_apply.argtypes = [vp, vp, vp, vp]
    L.mas_apply.restype = ctypes.c_int
    L.bcsr_spmv.argtypes = [P(MasBcsr), vp, vp, vp]
    L.bcsr_spmv.restype = ctypes.c_int
    L.bcsr_assemble_workspace_size.argtypes = [i32, ctypes.c_int64]
    L.bcsr_assemble_workspace_size.restype = ctypes.c_size_t
    L.bcsr_assemble.argtypes = [i32, ctypes.c_int64, vp, vp, vp, vp, vp, vp, ctypes.c_int64, P(ctypes.c_int64), vp,
                                ctypes.c_size_t, vp]
    L.bcsr_assemble.restype = ctypes.c_int
    L.bcsr_assemble_noalloc.argtypes = [i32, ctypes.c_int64, vp, vp, vp, vp, vp, vp, ctypes.c_int64,
                                        P(ctypes.c_int64), vp]
    L.bcsr_assemble_noalloc.restype = ctypes.c_int
    L.abd_contact_workspace_size.argtypes = [i32, ctypes.c_int64]
    L.abd_contact_workspace_size.restype = ctypes.c_size_t
    L.abd_contact_blocks.argtypes = [i32, vp, vp, vp, ctypes.c_int64, vp, vp, vp, i32, vp, vp, vp, ctypes.c_int64,
                                     P(ctypes.c_int64), vp, ctypes.c_size_t, vp]
    L.abd_contact_blocks.restype = ctypes.c_int
    L.mas_hierarchy_workspace_size.argtypes = [vp]
    L.mas_hierarchy_workspace_size.restype = ctypes.c_size_t
    L.mas_hierarchy_device.argtypes = [vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    L.mas_hierarchy_device.restype = ctypes.c_int
    L.mas_hierarchy_rebuild.argtypes = [vp, ctypes.c_int64, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    L.mas_hierarchy_rebuild.restype = ctypes.c_int
    L.mas_replan_workspace_size.argtypes = [vp, ctypes.c_int64]
    L.mas_replan_workspace_size.restype = ctypes.c_size_t
    L.mas_replan.argtypes = [vp, ctypes.c_int64, vp, vp, vp, ctypes.c_size_t, vp]
    L.mas_replan.restype = ctypes.c_int
    L.pcg_solve.argtypes = [vp, P(MasBcsr), vp, vp, P(PcgOptions), P(PcgResult), vp]
    L.pcg_solve.restype = ctypes.c_int
    L.pcg_adjoint.argtypes = [vp, P(MasBcsr), vp, vp, vp, vp, i32, P(PcgOptions), P(PcgResult), vp]
    L.pcg_adjoint.restype = ctypes.c_int
    L.mas_get_info.argtypes = [vp, P(MasInfo)]
    L.mas_get_info.restype = ctypes.c_int
    L.mas_get_ordering.argtypes = [vp, vp, vp, vp]
    L.mas_get_ordering.restype = ctypes.c_int
    L.mas_get_inverses.argtypes = [vp, i32, i32, vp, vp]
    L.mas_get_inverses.restype = ctypes.c_int
    L.mas_get_timings.argtypes = [vp, P(ctypes.c_double)]
    L.mas_get_timings.restype = ctypes.c_int
    L.mas_set_kernel_timing.argtypes = [vp, ctypes.c_int]
    L.mas_set_kernel_timing.restype = ctypes.c_int
    L.mas_get_kernel_timing.argtypes = [vp, P(ctypes.c_double), P(ctypes.c_int32)]
    L.mas_get_kernel_timing.restype = ctypes.c_int
    L.mas_status_string.argtypes = [ctypes.c_int]
    L.mas_status_string.restype = ctypes.c_char_p
    _lib = L
    return L


def status_string(code):
    return load().mas_status_string(int(code)).decode()


class MasError(RuntimeError):
    def __init__(self, call, code):
        self.code = int(code)
        super().__init__(f"{call} failed: {status_string(code)} ({code})")


def check(call, code, allow=(MAS_OK,)):
    if code not in allow:
        raise MasError(call, code)
    return code
