"""The scoring entry point that allocates nothing (its scratch is the library's static
per-GPU array), through the C ABI: two calls in a row, the second with fewer queries and
a different schedule, each bit-equal to ephdc_score_encrypted on the same inputs (itself
oracle-checked elsewhere) and, for the first, to the oracle."""
import ctypes

import numpy as np
import pytest

import paper_2511_00737_amd as ep
from oracle import bfv, pipeline
from oracle.params import Params as OParams, default_primes

from gpu_helpers import hv_layout, to_dev, to_host_u32, torch_cuda

pytestmark = pytest.mark.gpu


def _score(fn, s, h, Q):
    import torch
    d_hv = to_dev(hv_layout(h, s.hv_stride(Q)))
    out = torch.full((s.num_groups(Q), 2, s.prm.L, s.prm.N), -1, dtype=torch.int32, device="cuda")
    lib = ep.lib()
    st = getattr(lib, fn)(s.handle, ctypes.c_void_p(d_hv.data_ptr()), Q, ctypes.c_void_p(out.data_ptr()),
                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == ep.OK, lib.ephdc_last_error().decode()
    torch.cuda.synchronize()
    return to_host_u32(out)


@pytest.mark.parametrize("N,L,K,D,r", [(8192, 4, 7, 300, 1), (4096, 3, 2, 200, 1), (4096, 2, 3, 64, 4)])
def test_static_scratch_scoring_equals_workspace_scoring(N, L, K, D, r):
    torch_cuda()
    alpha, dnum = (1, 1) if r > 1 else (0, 0)
    primes = default_primes(N, L + alpha)
    kw = dict(N=N, q=tuple(primes[:L]), p=tuple(primes[L:]), F=64, D=D, K=K, r=r, dnum=dnum)
    o, e = OParams(**kw), ep.Params(**kw)
    rng = np.random.default_rng(N + D)
    C = rng.integers(-128, 128, (K, D)).astype(np.int8)
    sk = bfv.secret_key(o, 21)
    model = bfv.encrypt_model(o, sk, C, 21)
    gk64 = bfv.galois_keys(o, sk, 21) if r > 1 else None
    gk = gk64.astype(np.uint32) if r > 1 else None
    Q1, Q2 = 3 * o.B + 11, o.B // 2 + 1
    h1 = rng.choice(np.array([-1, 1], dtype=np.int8), (Q1, D))
    h2 = rng.choice(np.array([-1, 1], dtype=np.int8), (Q2, D))
    s = ep.Session(e, to_dev(model.astype(np.uint32)), to_dev(gk) if gk is not None else None, max_Q=Q1)
    try:
        a1 = _score("ephdc_score_encrypted_static", s, h1, Q1)
        b1 = _score("ephdc_score_encrypted", s, h1, Q1)
        s.tune(blocks=64, mode="fused")
        a2 = _score("ephdc_score_encrypted_static", s, h2, Q2)
        b2 = _score("ephdc_score_encrypted", s, h2, Q2)
    finally:
        s.close()
    assert np.array_equal(a1, b1)
    assert np.array_equal(a2, b2)
    assert np.array_equal(a1.astype(np.int64)[:1], pipeline.score_ciphertexts(o, model, h1, gk64, groups=[0]))


def test_static_scratch_rejects_a_call_larger_than_the_array():
    torch = torch_cuda()
    N, L = 16384, 8
    primes = default_primes(N, L)
    e = ep.Params(N=N, q=tuple(primes), F=64, D=16, K=2)
    model = torch.zeros((16, 2, L, N), dtype=torch.int32, device="cuda")
    s = ep.Session(e, model, max_Q=200000, workspace=None)
    try:
        Q = 200000
        s.tune(blocks=1024)  # 25 groups x 6 ranges x 8 limbs of partial sums: 157 MB
        d_hv = torch.zeros((16, s.hv_stride(Q)), dtype=torch.int8, device="cuda")
        out = torch.empty((s.num_groups(Q), 2, L, N), dtype=torch.int32, device="cuda")
        with pytest.raises(ep.EphdcError) as ei:
            ep.ephdc_score_encrypted_static(s, d_hv, Q, out)
        assert ei.value.status == ep.ERR_UNSUPPORTED
        assert "static scratch" in str(ei.value)
    finally:
        s.close()
