"""Reference Morton ordering for the tests (numpy): the definition the
library's device partition (mas_morton_partition) must reproduce bit for
bit -- bounding box, 21-bit scaling ((x - lo) / extent) * (2^21 - 1)
rounded down, x/y/z bit interleave, order by code then node id, k-th node
to domain k / N.  Its codes are pinned against a bit-by-bit interleave."""

import numpy as np


def _spread3(v):
    """Spreads the low 21 bits of v so that bit i lands on bit 3 i."""
    v = v.astype(np.uint64) & np.uint64(0x1FFFFF)
    v = (v | (v << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
    v = (v | (v << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
    v = (v | (v << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
    v = (v | (v << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
    v = (v | (v << np.uint64(2))) & np.uint64(0x1249249249249249)
    return v


def morton_codes(positions):
    """63-bit Morton (Z-order) codes of 3-D points: each coordinate scaled to
    21 bits over the bounding box, bits interleaved x, y, z."""
    p = np.asarray(positions, dtype=np.float64).reshape(-1, 3)
    lo = p.min(axis=0)
    ext = np.maximum(p.max(axis=0) - lo, np.finfo(np.float64).tiny)
    q = np.floor((p - lo) / ext * ((1 << 21) - 1)).astype(np.int64)
    q = np.clip(q, 0, (1 << 21) - 1)
    return (_spread3(q[:, 0]) << np.uint64(2)) | (_spread3(q[:, 1]) << np.uint64(1)) | _spread3(q[:, 2])


def morton_partition(positions, domain_size=16):
    """Level-0 domains of ``domain_size`` consecutive nodes in Morton order of
    their positions (ties by node id): the domain ordering of the earlier MAS
    preconditioner that the connectivity-aware partition replaces (Sec. 4.1).
    Returns part[V]."""
    codes = morton_codes(positions)
    order = np.lexsort((np.arange(codes.size), codes))
    part = np.empty(codes.size, dtype=np.int32)
    part[order] = np.arange(codes.size) // domain_size
    return part
