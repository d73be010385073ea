"""MI355X-native MAS-preconditioned PCG (StiffGIPC, arXiv 2411.06224).

The solver is the C-ABI library ``libmaspcg.so`` (HIP kernels for gfx950 and
a C++ host planner, see include/mas_pcg.h); this package only marshals
arguments.  Importing it does not load the library; the first call does, and
fails loudly if the library has not been built.
"""

from ._lib import LibraryMissing, MasError, load
from .solver import BlockMatrix, MasPcg, abd_contact_blocks, bcsr_assemble, bcsr_assemble_noalloc, bcsr_spmv
from .autograd import MasPcgSolve, mas_pcg_solve
from .ordering import morton_partition

__all__ = [
    "BlockMatrix",
    "MasPcg",
    "bcsr_spmv",
    "bcsr_assemble",
    "bcsr_assemble_noalloc",
    "abd_contact_blocks",
    "MasPcgSolve",
    "mas_pcg_solve",
    "morton_partition",
    "LibraryMissing",
    "MasError",
    "load",
]
