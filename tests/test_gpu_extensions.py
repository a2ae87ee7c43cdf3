"""HIP path vs the oracle for the method's variants (needs a gfx950 GPU): the HE-aware
scaling op of the multiply-accumulate, BGV and rounded-BFV model ciphertexts, plaintext
primes other than 65537 and the N = 2048 ring.  Every comparison is bit-exact."""
import numpy as np
import pytest

import paper_2511_00737_amd as ep
from oracle import bfv, hdc, pipeline
from oracle.params import Params as OParams, default_primes

from gpu_helpers import hv_layout, score_on_gpu, to_dev, to_host_u32, torch_cuda

pytestmark = pytest.mark.gpu


def make(N, L, D, K, **kw):
    primes = default_primes(N, L)
    args = dict(N=N, q=tuple(primes), F=64, D=D, K=K, **kw)
    o = OParams(**args)
    o.validate()
    return o, ep.Params(**args)


def values(rng, bits, shape):
    """Signed `bits`-bit values (bits = 1: +1 / -1), the paper's Q- and C-bit hypervectors."""
    if bits == 1:
        return rng.choice(np.array([-1, 1], dtype=np.int8), shape)
    return rng.integers(-(1 << (bits - 1)), 1 << (bits - 1), shape).astype(np.int8)


def scaled_scores(o, h, C):
    """Closed form of the scaled MAC: sum over blocks k of S_k * c^(n_k) mod t, S_k the exact
    dot products of block k, n_k = (complete blocks) - k scalings after a complete block k."""
    g, t = o.scale_every, o.t
    c = pow(2, -o.scale_shift, t)
    nfull = o.M // g
    want = np.zeros((h.shape[0], o.K), dtype=object)
    for k in range(-(-o.M // g)):
        blk = slice(k * g, min(o.M, (k + 1) * g))
        Sk = h[:, blk].astype(np.int64) @ C[:, blk].astype(np.int64).T
        want = want + Sk.astype(object) * pow(c, nfull - k if k < nfull else 0, t)
    want = np.array([[int(v) % t for v in row] for row in want], dtype=np.int64)
    return np.where(want > t // 2, want - t, want)


# (Q bits, C bits) of the paper's optimised settings (6, 2) and (8, 8), g = 512 as in the
# paper and smaller blocks; trailing partial blocks; split (64- and 32-bit sums) and fused paths
@pytest.mark.parametrize("N,L,t,qb,cb,D,g,s_,sched", [
    (4096, 3, 65537, 6, 2, 1029, 512, 13, None),
    (4096, 3, 65537, 8, 8, 200, 64, 12, dict(mode="fused", limb_group=3)),
    (8192, 4, 65537, 8, 8, 130, 32, 14, dict(values_per_thread=16)),
    (8192, 4, 114689, 6, 2, 97, 24, 5, dict(mode="fused", limb_group=2, values_per_thread=16)),
    (2048, 2, 40961, 8, 8, 300, 100, 3, None),
])
def test_scaling_op_matches_oracle(N, L, t, qb, cb, D, g, s_, sched):
    torch_cuda()
    o, e = make(N, L, D, K=2 if N == 2048 else 3, t=t, scale_every=g, scale_shift=s_)
    rng = np.random.default_rng(D + g)
    C = values(rng, cb, (o.K, D))
    h = values(rng, qb, (o.B + 37, D))  # two groups, the second ragged
    sk = bfv.secret_key(o, 9)
    model = bfv.encrypt_model(o, sk, C, 9)
    want = pipeline.score_ciphertexts(o, model, h)
    got = score_on_gpu(e, model.astype(np.uint32), h, tune=sched)
    assert np.array_equal(got.astype(np.int64), want)
    if t == 65537 and s_ >= 12:  # |c| = 2^(16-s): the noise stays far inside the budget
        sc, _ = ep.ephdc_decrypt_scores(e, sk.astype(np.int8), got, h.shape[0])
        assert np.array_equal(sc, scaled_scores(o, h, C))


@pytest.mark.parametrize("scheme", ["bgv", "bfv-r"])
@pytest.mark.parametrize("N,L,t", [(4096, 3, 65537), (2048, 2, 12289)])
def test_other_schemes_score_exactly(scheme, N, L, t):
    """BGV and rounded-BFV model ciphertexts (encrypted by the library, bit-exact with the
    oracle on the CPU): the device's ct x pt path gives the oracle's score ciphertexts, and
    they decrypt to the exact scores h . C mod t."""
    torch_cuda()
    o, e = make(N, L, 45, K=3, t=t, scheme=scheme)
    rng = np.random.default_rng(N + len(scheme))
    C = rng.integers(-128, 128, (o.K, o.D)).astype(np.int8)
    h = values(rng, 1, (2 * o.B + 5, o.D))
    sk, _ = ep.ephdc_keygen(e, 12)
    model = ep.ephdc_encrypt_model(e, sk, C, 13)
    assert np.array_equal(model.astype(np.int64), bfv.encrypt_model(o, sk.astype(np.int64), C, 13))
    got = score_on_gpu(e, model, h)
    assert np.array_equal(got.astype(np.int64), pipeline.score_ciphertexts(o, model.astype(np.int64), h))
    sc, am = ep.ephdc_decrypt_scores(e, sk, got, h.shape[0])
    assert np.array_equal(sc, hdc.scores_mod_t(h, C, t))
    assert np.array_equal(am, hdc.argmax(hdc.scores_int(h, C)))  # |h . C| <= 45 * 128 < t / 2: no wraps


@pytest.mark.parametrize("N,L,t,K,Q", [(2048, 2, 65537, 2, 1024), (2048, 3, 12289, 7, 700),
                                       (4096, 3, 40961, 2, 2049), (8192, 4, 114689, 7, 1300)])
def test_other_plaintext_primes_and_ring_2048(N, L, t, K, Q):
    """Batch encoding mod t for t other than 65537 (the slot root from the smallest
    generator of Z_t^*) and the N = 2048 transform shape: score ciphertexts bit-exact, the
    plaintexts of the batch-encode step, and decryption to h . C mod t."""
    torch = torch_cuda()
    o, e = make(N, L, 40, K=K, t=t)
    rng = np.random.default_rng(t + N)
    C = rng.integers(-128, 128, (o.K, o.D)).astype(np.int8)
    h = values(rng, 1, (Q, o.D))
    sk = bfv.secret_key(o, 14)
    model = bfv.encrypt_model(o, sk, C, 14)
    got = score_on_gpu(e, model.astype(np.uint32), h)
    assert np.array_equal(got.astype(np.int64), pipeline.score_ciphertexts(o, model, h))
    sc, _ = ep.ephdc_decrypt_scores(e, sk.astype(np.int8), got, Q)
    assert np.array_equal(sc, hdc.scores_mod_t(h, C, t))
    s = ep.Session(e, to_dev(model.astype(np.uint32)), max_Q=Q)
    try:
        d_hv = to_dev(hv_layout(h, s.hv_stride(Q)))
        G = s.num_groups(Q)
        for g, m in [(0, 0), (G - 1, o.M - 1)]:
            d_out = torch.empty((o.L, N), dtype=torch.int32, device="cuda")
            ep.ephdc_debug_plaintext(s, d_hv, Q, g, m, d_out)
            p = bfv.query_plaintext(o, h, g, m)
            got_p = to_host_u32(d_out).astype(np.int64)
            for l, q in enumerate(o.q):
                assert np.array_equal(got_p[l], p % q), (g, m, l)
    finally:
        s.close()


def test_calls_on_two_streams_share_one_workspace():
    """Two scoring calls on one session, enqueued back to back on two streams with different
    queries: the second waits for the first (they share the session's workspace), and both
    give the oracle's ciphertexts."""
    torch = torch_cuda()
    o, e = make(8192, 4, 64, K=7)
    rng = np.random.default_rng(15)
    C = rng.integers(-128, 128, (o.K, o.D)).astype(np.int8)
    sk = bfv.secret_key(o, 15)
    model = bfv.encrypt_model(o, sk, C, 15)
    Q = 2 * o.B
    h1, h2 = values(rng, 1, (Q, o.D)), values(rng, 1, (Q, o.D))
    s = ep.Session(e, to_dev(model.astype(np.uint32)), max_Q=Q)
    try:
        st1, st2 = torch.cuda.Stream(), torch.cuda.Stream()
        hv1 = to_dev(hv_layout(h1, s.hv_stride(Q)))
        hv2 = to_dev(hv_layout(h2, s.hv_stride(Q)))
        out1 = torch.empty((2, 2, o.L, o.N), dtype=torch.int32, device="cuda")
        out2 = torch.empty_like(out1)
        torch.cuda.synchronize()
        ep.ephdc_score_encrypted(s, hv1, Q, out1, stream=st1)
        ep.ephdc_score_encrypted(s, hv2, Q, out2, stream=st2)
        torch.cuda.synchronize()
        g1, g2 = to_host_u32(out1), to_host_u32(out2)
    finally:
        s.close()
    assert np.array_equal(g1.astype(np.int64), pipeline.score_ciphertexts(o, model, h1))
    assert np.array_equal(g2.astype(np.int64), pipeline.score_ciphertexts(o, model, h2))


def test_session_without_workspace_rejects_single_request_scoring():
    torch = torch_cuda()
    o, e = make(4096, 3, 16, K=2)
    model = np.zeros((o.M, 2, o.L, o.N), dtype=np.uint32)
    s = ep.Session(e, to_dev(model), max_Q=10, workspace=None)
    try:
        d_hv = torch.zeros((o.D, s.hv_stride(10)), dtype=torch.int8, device="cuda")
        d_out = torch.empty((1, 2, o.L, o.N), dtype=torch.int32, device="cuda")
        with pytest.raises(ep.EphdcError) as ei:
            ep.ephdc_score_encrypted(s, d_hv, 10, d_out)
        assert ei.value.status == ep.ERR_BUFFER
    finally:
        s.close()
    # a workspace one byte short of the minimum is refused at creation
    import ctypes
    c = e.c()
    need = ep.ephdc_workspace_bytes(e, 10)
    G = 1
    minimum = need - (min(G * o.M, (4 << 30) // (4 * o.N)) - G) * o.N * 4
    ws = torch.empty(minimum - 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(ep.EphdcError) as ei:
        ep.Session(e, to_dev(model), max_Q=10, workspace=ws)
    assert ei.value.status == ep.ERR_BUFFER
    ws = torch.empty(minimum, dtype=torch.uint8, device="cuda")
    ep.Session(e, to_dev(model), max_Q=10, workspace=ws).close()



@pytest.mark.parametrize("layout", ["contiguous", "subring"])
def test_scaling_op_in_batches(layout):
    """Batches whose requests mix scaled and unscaled models (one list launch serves both;
    in the subring layout the n-point kernels apply the weights), Q-bit queries encoded
    inside the batch, segment lengths shorter and longer than a scaling block, split and
    fused, unpacked and packed: every request equals the oracle's ciphertexts of its own
    query sequence (unpacked) or of its model's sequence (packed)."""
    import synth
    torch = torch_cuda()
    # (N, L, t, D, K, scale_every, scale_shift, Q bits, qshift)
    specs = [(4096, 3, 65537, 192, 3, 64, 12, 8, 4), (4096, 3, 65537, 128, 2, 0, 0, 1, 0),
             (8192, 4, 114689, 128, 2, 24, 5, 6, 6)]
    reqs_spec = [(0, 300), (1, 40), (2, 700), (0, 5), (2, 1), (1, 1200), (0, 900)]
    tenants, sessions = [], []
    for i, (N, L, t, D, K, g, s_, qb, qs) in enumerate(specs):
        o, e = make(N, L, D, K=K, t=t, scale_every=g, scale_shift=s_, qbits=qb, qshift=qs, layout=layout)
        C = values(np.random.default_rng(70 + i), 8, (K, D))
        sk = bfv.secret_key(o, 71 + i)
        model = bfv.encrypt_model(o, sk, C, 72 + i)
        base = synth.base_hypervectors(73 + i, o.F, D)
        tenants.append((o, model, base))
        mq = max(Q for ti, Q in reqs_spec if ti == i)
        sessions.append(ep.Session(e, to_dev(model.astype(np.uint32)), max_Q=mq))
    try:
        xs, hs = [], []
        for k, (ti, Q) in enumerate(reqs_spec):
            o, _, base = tenants[ti]
            xs.append(synth.uniform_features(200 + k, Q, o.F))
            hs.append(hdc.encode(xs[k], base, o.qbits, o.qshift))

        def requests(packed):
            out = []
            for k, (ti, Q) in enumerate(reqs_spec):
                o, _, base = tenants[ti]
                s = sessions[ti]
                d_out = torch.zeros((s.num_groups(Q) + (1 if packed else 0), 2, o.L, o.N), dtype=torch.int32,
                                    device="cuda")
                d_hv = None if packed else torch.empty((o.D, s.hv_stride(Q)), dtype=torch.int8, device="cuda")
                out.append(ep.Request(s, d_hv, Q, d_out, d_x=to_dev(xs[k]), d_base=to_dev(base)))
            return out

        reqs = requests(False)
        want = [pipeline.score_ciphertexts(tenants[ti][0], tenants[ti][1], hs[k])
                for k, (ti, _) in enumerate(reqs_spec)]
        b = ep.Batch(reqs)
        try:
            for mode, seg_len in (("split", 16), ("split", 1024), ("fused", 40)):
                b.tune(mode=mode, seg_len=seg_len, grid=300)
                for r in reqs:
                    r.d_score_ct.fill_(0)
                b.run()
                torch.cuda.synchronize()
                for k, r in enumerate(reqs):
                    assert np.array_equal(to_host_u32(r.d_score_ct).astype(np.int64), want[k]), (mode, seg_len, k)
        finally:
            b.close()
        preqs = requests(True)
        b = ep.Batch(preqs, packed=True)
        try:
            b.run()
            torch.cuda.synchronize()
            for k, ((ti, Q), r) in enumerate(zip(reqs_spec, preqs)):
                o, model, _ = tenants[ti]
                seq = np.concatenate([hs[j] for j, (tj, _) in enumerate(reqs_spec) if tj == ti])
                off, qf, nct = b.packing(k)
                got = to_host_u32(r.d_score_ct)[:nct].astype(np.int64)
                grp = list(range(off // o.B, off // o.B + nct))
                assert np.array_equal(got, pipeline.score_ciphertexts(o, model, seq, groups=grp)), ("packed", k)
        finally:
            b.close()
    finally:
        for s in sessions:
            s.close()
