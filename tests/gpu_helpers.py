"""Shared helpers of the GPU parity tests (HIP path through the C ABI)."""
import numpy as np
import pytest
import torch

gpu = pytest.mark.gpu


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2505_22168_amd as g
    g.load_library()
    return g


def gpu_list_triples(nl):
    """(i, j, Sx, Sy, Sz) of the device list as an int64 array [P,5]."""
    n = nl.n_pairs
    i = nl.rows()[:n].cpu().numpy()
    j = nl.j[:n].cpu().numpy().astype(np.int64)
    S = nl.shifts().cpu().numpy()
    return np.concatenate([i[:, None], j[:, None], S], 1)


def oracle_triples(onl):
    return np.concatenate([onl.i[:, None], onl.j[:, None], onl.S], 1)
