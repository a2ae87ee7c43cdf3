"""Helpers shared by the GPU tests: device buffers and one call of the client path."""
from __future__ import annotations

import numpy as np

import paper_2511_00737_amd as ep


def torch_cuda():
    import pytest
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def to_dev(a: np.ndarray):
    import torch
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).cuda()


def to_host_u32(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def hv_layout(h: np.ndarray, stride: int) -> np.ndarray:
    """int8 [Q][D] query hypervectors -> the library's [D][stride] layout (zero padding)."""
    Q, D = h.shape
    out = np.zeros((D, stride), dtype=np.int8)
    out[:, :Q] = h.T
    return out


def score_on_gpu(e: ep.Params, model_ct: np.ndarray, h: np.ndarray, gk=None, max_Q=None, tune=None):
    """Score ciphertexts uint32 [G][2][L][N] of query hypervectors h int8 [Q][D]; tune: keyword
    arguments of Session.tune (the kernel schedule)."""
    import torch
    Q = h.shape[0]
    s = ep.Session(e, to_dev(model_ct), to_dev(gk) if gk is not None else None, max_Q=max_Q or Q)
    try:
        if tune:
            s.tune(**tune)
        stride = s.hv_stride(Q)
        G = s.num_groups(Q)
        d_hv = to_dev(hv_layout(h, stride))
        d_out = torch.empty((G, 2, e.L, e.N), dtype=torch.int32, device="cuda")
        ep.ephdc_score_encrypted(s, d_hv, Q, d_out)
        torch.cuda.synchronize()
        return to_host_u32(d_out)
    finally:
        s.close()
