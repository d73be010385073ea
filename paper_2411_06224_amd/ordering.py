"""Level-0 domain orderings for ``MasPcg(partition=...)`` computed by the
library (argument marshalling only)."""

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check

_ALIGN = 256


def morton_partition(positions, domain_size=16, device=None):
    """Level-0 domains of ``domain_size`` consecutive nodes in Morton order of
    their positions (ties by node id): the domain ordering of the earlier MAS
    preconditioner that the connectivity-aware partition replaces (Sec. 4.1),
    computed on the device by mas_morton_partition.  ``positions``: [V, 3]
    array or tensor.  Returns part[V] (numpy int32) for
    ``MasPcg(partition=...)``."""
    L = _lib.load()
    if device is None:
        device = positions.device if isinstance(positions, torch.Tensor) and positions.is_cuda else torch.device("cuda")
    pos = torch.as_tensor(positions, dtype=torch.float64, device=device).reshape(-1, 3).contiguous()
    n = pos.shape[0]
    need = int(L.mas_morton_workspace_size(n))
    ws = torch.empty(need + _ALIGN, dtype=torch.uint8, device=device)
    wsp = (ws.data_ptr() + _ALIGN - 1) // _ALIGN * _ALIGN
    part = torch.empty(n, dtype=torch.int32, device=device)
    stream = ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)
    rc = L.mas_morton_partition(n, ctypes.c_void_p(pos.data_ptr()), int(domain_size), ctypes.c_void_p(part.data_ptr()),
                                ctypes.c_void_p(wsp), need, stream)
    check("mas_morton_partition", rc)
    return part.cpu().numpy().astype(np.int32)
