"""Subring slot layout through the C ABI (needs a gfx950 GPU): the n-point batch-encoding and
MAC kernels (n = N/K') against the oracle word for word, against the N-point kernels of the
same session, with the scaling op, with the plaintext chunk split, with queries encoded on
the device, and in batches (whose list kernels run the N-point transforms)."""
import numpy as np
import pytest

import paper_2511_00737_amd as ep
import synth
from oracle import bfv, hdc, pipeline
from oracle.params import Params as OParams, default_primes

from gpu_helpers import hv_layout, to_dev, to_host_u32, torch_cuda

pytestmark = pytest.mark.gpu


def make(N, L, D, K, F=64, **kw):
    args = dict(N=N, q=tuple(default_primes(N, L)), F=F, D=D, K=K, layout="subring", **kw)
    o = OParams(**args)
    o.validate()
    return o, ep.Params(**args)


def values(rng, bits, shape):
    if bits == 1:
        return rng.choice(np.array([-1, 1], dtype=np.int8), shape)
    return rng.integers(-(1 << (bits - 1)), 1 << (bits - 1), shape).astype(np.int8)


def score(e, model, h, stride_offset=0, chunk_bytes=0):
    """Score ciphertexts of h through ephdc_score_encrypted; stride_offset > 0 places the
    hypervectors at a byte offset (not 16-byte aligned), which takes the N-point kernels."""
    torch = torch_cuda()
    Q = h.shape[0]
    s = ep.Session(e, to_dev(model.astype(np.uint32)), max_Q=Q)
    try:
        if chunk_bytes:
            s.set_chunk_bytes(chunk_bytes)
        stride = s.hv_stride(Q)
        lay = hv_layout(h, stride).reshape(-1)
        buf = torch.zeros(lay.size + 64, dtype=torch.int8, device="cuda")
        buf[stride_offset:stride_offset + lay.size] = to_dev(lay)
        d_hv = buf[stride_offset:stride_offset + lay.size]
        out = torch.empty((s.num_groups(Q), 2, e.L, e.N), dtype=torch.int32, device="cuda")
        ep.ephdc_score_encrypted(s, d_hv, Q, out)
        torch.cuda.synchronize()
        return to_host_u32(out).astype(np.int64)
    finally:
        s.close()


# (N, L, K, D, Q): n = N/K' of 4096 and 2048 (transforms across waves), 1024, 512 and 256
# (one wave each) under N = 2048, 4096 and 8192; ragged last groups; nine groups (MAC work
# items of eight groups, the second one ragged)
CASES = [(8192, 4, 7, 70, 2500), (8192, 4, 12, 33, 1100), (8192, 4, 26, 21, 300), (4096, 3, 3, 64, 1500),
         (4096, 3, 9, 40, 700), (2048, 2, 2, 50, 2100), (2048, 2, 5, 31, 600), (8192, 4, 2, 24, 5000),
         (4096, 3, 2, 40, 2100), (2048, 2, 8, 40, 2200)]


@pytest.mark.parametrize("N,L,K,D,Q", CASES)
def test_subring_scores_match_oracle(N, L, K, D, Q):
    o, e = make(N, L, D, K)
    rng = np.random.default_rng(N + K + D)
    C = values(rng, 8, (K, D))
    h = values(rng, 1, (Q, D))
    sk = bfv.secret_key(o, 3)
    model = bfv.encrypt_model(o, sk, C, 3)
    got = score(e, model, h)
    want = pipeline.score_ciphertexts(o, model, h)
    assert np.array_equal(got, want)
    sc, am = ep.ephdc_decrypt_scores(e, sk.astype(np.int8), got.astype(np.uint32), Q)
    assert np.array_equal(sc, hdc.scores_mod_t(h, C, o.t))


@pytest.mark.parametrize("N,L,K,D,Q", [(8192, 4, 7, 70, 2500), (4096, 3, 9, 40, 700), (2048, 2, 2, 50, 2100),
                                       (8192, 4, 2, 24, 5000)])
def test_subring_kernels_equal_the_n_point_kernels(N, L, K, D, Q):
    """The same session and queries through the N-point kernels (hypervectors at an odd
    byte offset) give the same ciphertexts, and so does a plaintext chunk of one plaintext
    per group (the MAC adding into stored sums chunk after chunk)."""
    o, e = make(N, L, D, K)
    rng = np.random.default_rng(5 * N + K)
    C = values(rng, 8, (K, D))
    h = values(rng, 4, (Q, D))
    sk = bfv.secret_key(o, 4)
    model = bfv.encrypt_model(o, sk, C, 4)
    fast = score(e, model, h)
    assert np.array_equal(fast, score(e, model, h, stride_offset=1))
    assert np.array_equal(fast, score(e, model, h, chunk_bytes=1))
    G = o.groups(Q)
    assert np.array_equal(fast[G - 1:], pipeline.score_ciphertexts(o, model, h, groups=[G - 1]))


@pytest.mark.parametrize("N,L,K,D,g,s_,qb", [(8192, 4, 7, 130, 32, 14, 8), (4096, 3, 3, 200, 64, 12, 6)])
def test_subring_with_scaling_op(N, L, K, D, g, s_, qb):
    o, e = make(N, L, D, K, scale_every=g, scale_shift=s_, qbits=qb)
    rng = np.random.default_rng(D + g)
    C = values(rng, 8, (K, D))
    h = values(rng, qb, (o.B + 77, D))
    sk = bfv.secret_key(o, 6)
    model = bfv.encrypt_model(o, sk, C, 6)
    assert np.array_equal(score(e, model, h), pipeline.score_ciphertexts(o, model, h))


def test_subring_queries_encoded_on_the_device():
    """Features -> ephdc_encode_queries (hypervectors of B = N/K' queries per group) ->
    subring scoring -> the oracle's scores."""
    torch = torch_cuda()
    o, e = make(8192, 4, 256, 7, F=128)
    Q = 1500
    x = synth.uniform_features(8, Q, o.F)
    base = synth.base_hypervectors(8, o.F, o.D)
    C = synth.class_hypervectors(8, o.K, o.D)
    sk = bfv.secret_key(o, 8)
    model = bfv.encrypt_model(o, sk, C, 8)
    s = ep.Session(e, to_dev(model.astype(np.uint32)), max_Q=Q)
    try:
        d_hv = torch.empty((o.D, s.hv_stride(Q)), dtype=torch.int8, device="cuda")
        ep.ephdc_encode_queries(s, to_dev(x), to_dev(base), Q, d_hv)
        out = torch.empty((s.num_groups(Q), 2, o.L, o.N), dtype=torch.int32, device="cuda")
        ep.ephdc_score_encrypted(s, d_hv, Q, out)
        torch.cuda.synchronize()
        got = to_host_u32(out)
    finally:
        s.close()
    h = hdc.encode(x, base)
    sc, _ = ep.ephdc_decrypt_scores(e, sk.astype(np.int8), got, Q)
    assert np.array_equal(sc, hdc.scores_mod_t(h, C, o.t))
    assert np.array_equal(got[1:].astype(np.int64), pipeline.score_ciphertexts(o, model, h, groups=[1]))


def test_subring_sessions_in_a_batch():
    """A batch mixing a subring session with a contiguous one (the list kernels gather
    through the scatter table): every request equals the oracle."""
    torch = torch_cuda()
    o1, e1 = make(4096, 3, 64, 3)
    args2 = dict(N=4096, q=tuple(default_primes(4096, 3)), F=64, D=64, K=3)
    o2, e2 = OParams(**args2), ep.Params(**args2)
    rng = np.random.default_rng(10)
    tenants = []
    for o, e in ((o1, e1), (o2, e2)):
        C = values(rng, 8, (o.K, o.D))
        sk = bfv.secret_key(o, 10)
        model = bfv.encrypt_model(o, sk, C, 10)
        tenants.append((o, e, model, ep.Session(e, to_dev(model.astype(np.uint32)), max_Q=2000)))
    try:
        reqs, want = [], []
        for k, (ti, Q) in enumerate([(0, 1500), (1, 700), (0, 3), (1, 2000)]):
            o, e, model, s = tenants[ti]
            h = values(rng, 1, (Q, o.D))
            d_hv = to_dev(hv_layout(h, s.hv_stride(Q)))
            out = torch.zeros((s.num_groups(Q), 2, o.L, o.N), dtype=torch.int32, device="cuda")
            reqs.append(ep.Request(s, d_hv, Q, out))
            want.append(pipeline.score_ciphertexts(o, model, h))
        b = ep.Batch(reqs)
        try:
            b.run()
            torch.cuda.synchronize()
        finally:
            b.close()
        for k, r in enumerate(reqs):
            assert np.array_equal(to_host_u32(r.d_score_ct).astype(np.int64), want[k]), k
    finally:
        for t in tenants:
            t[3].close()


def test_subring_batch_of_many_groups_on_one_model():
    """Eleven virtual groups of five requests on one subring model (MAC items of eight
    groups, the second ragged), packed and unpacked: every request equals its single-request
    ciphertexts, which equal the oracle's."""
    torch = torch_cuda()
    o, e = make(2048, 2, 40, 8)  # B = 256
    rng = np.random.default_rng(12)
    C = values(rng, 8, (o.K, o.D))
    sk = bfv.secret_key(o, 12)
    model = bfv.encrypt_model(o, sk, C, 12)
    s = ep.Session(e, to_dev(model.astype(np.uint32)), max_Q=1024)
    try:
        sizes = [256, 300, 700, 1000, 3]  # groups 1 + 2 + 3 + 4 + 1
        hs = [values(rng, 1, (Q, o.D)) for Q in sizes]
        reqs, single = [], []
        for h in hs:
            Q = h.shape[0]
            d_hv = to_dev(hv_layout(h, s.hv_stride(Q)))
            out = torch.zeros((s.num_groups(Q), 2, o.L, o.N), dtype=torch.int32, device="cuda")
            reqs.append(ep.Request(s, d_hv, Q, out))
            one = torch.empty_like(out)
            ep.ephdc_score_encrypted(s, d_hv, Q, one)
            single.append(one)
        b = ep.Batch(reqs)
        try:
            b.run()
            torch.cuda.synchronize()
        finally:
            b.close()
        for k, (r, one) in enumerate(zip(reqs, single)):
            assert torch.equal(r.d_score_ct, one), k
        assert np.array_equal(to_host_u32(single[3]).astype(np.int64), pipeline.score_ciphertexts(o, model, hs[3]))
        assert np.array_equal(to_host_u32(single[4]).astype(np.int64), pipeline.score_ciphertexts(o, model, hs[4]))
    finally:
        s.close()


def make_fold(N, L, D, K, r, dnum, alpha=2, F=64):
    primes = default_primes(N, L + alpha)
    args = dict(N=N, q=tuple(primes[:L]), p=tuple(primes[L:]), F=F, D=D, K=K, r=r, dnum=dnum, layout="subring")
    o = OParams(**args)
    o.validate()
    return o, ep.Params(**args)


def score_fold(e, model, gk, h, stride_offset=0):
    torch = torch_cuda()
    Q = h.shape[0]
    s = ep.Session(e, to_dev(model.astype(np.uint32)), to_dev(gk.astype(np.uint32)), max_Q=Q)
    try:
        stride = s.hv_stride(Q)
        lay = hv_layout(h, stride).reshape(-1)
        buf = torch.zeros(lay.size + 64, dtype=torch.int8, device="cuda")
        buf[stride_offset:stride_offset + lay.size] = to_dev(lay)
        out = torch.empty((s.num_groups(Q), 2, e.L, e.N), dtype=torch.int32, device="cuda")
        ep.ephdc_score_encrypted(s, buf[stride_offset:stride_offset + lay.size], Q, out)
        torch.cuda.synchronize()
        return to_host_u32(out).astype(np.int64)
    finally:
        s.close()


# (N, L, K, D, Q, r, dnum): folded subring layout, n = N/K' of 1024 and 256, D not a
# multiple of r, ragged last groups, five groups (work items of eight groups)
FOLD_CASES = [(4096, 3, 3, 37, 700, 4, 2), (8192, 4, 7, 30, 1500, 2, 2), (2048, 2, 2, 21, 300, 8, 2),
              (8192, 4, 26, 20, 300, 4, 4)]


@pytest.mark.parametrize("N,L,K,D,Q,r,dnum", FOLD_CASES)
def test_folded_subring_scores_match_oracle(N, L, K, D, Q, r, dnum):
    """Folded subring layout (n-point kernels, then rotate-and-sum with the layout's Galois
    elements): score ciphertexts word for word against the oracle, the same ciphertexts
    through the N-point kernels (hypervectors at an odd byte offset), exact decrypted scores."""
    o, e = make_fold(N, L, D, K, r, dnum)
    rng = np.random.default_rng(N + K + D + r)
    C = values(rng, 8, (K, D))
    h = values(rng, 1, (Q, D))
    sk = bfv.secret_key(o, 5)
    model = bfv.encrypt_model(o, sk, C, 5)
    gk = bfv.galois_keys(o, sk, 6)
    got = score_fold(e, model, gk, h)
    want = pipeline.score_ciphertexts(o, model, h, gk)
    assert np.array_equal(got, want)
    assert np.array_equal(score_fold(e, model, gk, h, stride_offset=3), want)
    sc, _ = ep.ephdc_decrypt_scores(e, sk.astype(np.int8), got.astype(np.uint32), Q)
    assert np.array_equal(sc, hdc.scores_mod_t(h, C, o.t))


def test_folded_subring_at_the_rotation_workload_shape():
    """N = 16384, 8 limbs + 2 special primes, 4 digits, K = 26 (K' = 32, n = 512), r = 8
    (64 queries per ciphertext): the last group matches the oracle bit for bit, every group
    equals the N-point kernels' result, and every score decrypts exactly."""
    N, L, K, D, Q, r = 16384, 8, 26, 40, 300, 8
    o, e = make_fold(N, L, D, K, r, dnum=4)
    rng = np.random.default_rng(26)
    C = values(rng, 8, (K, D))
    h = values(rng, 1, (Q, D))
    sk = bfv.secret_key(o, 7)
    model = bfv.encrypt_model(o, sk, C, 7)
    gk = bfv.galois_keys(o, sk, 8)
    got = score_fold(e, model, gk, h)
    G = o.groups(Q)
    want = pipeline.score_ciphertexts(o, model, h, gk, groups=[G - 1])
    assert np.array_equal(got[G - 1], want[0])
    assert np.array_equal(score_fold(e, model, gk, h, stride_offset=5), got)
    sc, _ = ep.ephdc_decrypt_scores(e, sk.astype(np.int8), got.astype(np.uint32), Q)
    assert np.array_equal(sc, hdc.scores_mod_t(h, C, o.t))


@pytest.mark.parametrize("layout", ["subring", "contiguous"])
def test_batch_encodes_queries_without_touching_padding(layout):
    """Batches that encode their queries on the device (HDC in the batch) write only the Q
    columns of a request's hypervectors: every batch encoding reads the other positions of
    the last group as zero.  Buffers filled with nonzero bytes beforehand still give the
    oracle's ciphertexts; packed, where the sequence's padding is not written either, every
    request still decrypts to its own exact scores."""
    torch = torch_cuda()
    from oracle import hdc as ohdc
    o, e = make_layout(2048, 2, 64, 3, 1, layout, F=48)  # the encoder takes D % 64 == 0
    rng = np.random.default_rng(14)
    C = values(rng, 8, (o.K, o.D))
    sk = bfv.secret_key(o, 14)
    model = bfv.encrypt_model(o, sk, C, 14)
    base = synth.base_hypervectors(14, o.F, o.D)
    d_base = to_dev(base)
    s = ep.Session(e, to_dev(model.astype(np.uint32)), max_Q=1200)
    sizes = [700, 3, 1100, 512]
    xs = [synth.uniform_features(20 + k, Q, o.F) for k, Q in enumerate(sizes)]
    hs = [ohdc.encode(x, base, o.qbits, o.qshift) for x in xs]
    try:
        reqs = []
        for Q, x in zip(sizes, xs):
            d_hv = torch.full((o.D, s.hv_stride(Q)), 77, dtype=torch.int8, device="cuda")
            out = torch.zeros((s.num_groups(Q), 2, o.L, o.N), dtype=torch.int32, device="cuda")
            reqs.append(ep.Request(s, d_hv, Q, out, d_x=to_dev(x), d_base=d_base))
        b = ep.Batch(reqs)
        try:
            b.run()
            torch.cuda.synchronize()
        finally:
            b.close()
        for k, (r, h) in enumerate(zip(reqs, hs)):
            Q = h.shape[0]
            assert (r.d_hv.cpu().numpy()[:, Q:] == 77).all(), k  # the padding columns were not written
            assert np.array_equal(to_host_u32(r.d_score_ct).astype(np.int64), pipeline.score_ciphertexts(o, model, h)), k
        # packed: one query sequence for the four requests
        preqs = []
        for Q, x in zip(sizes, xs):
            out = torch.zeros((s.num_groups(Q) + 1, 2, o.L, o.N), dtype=torch.int32, device="cuda")
            preqs.append(ep.Request(s, None, Q, out, d_x=to_dev(x), d_base=d_base))
        b = ep.Batch(preqs, packed=True)
        try:
            for rep in range(2):
                b.run()
                torch.cuda.synchronize()
                for k, (r, h) in enumerate(zip(preqs, hs)):
                    off, qf, nct = b.packing(k)
                    got = to_host_u32(r.d_score_ct)[:nct]
                    scores, _ = ep.ephdc_decrypt_scores_at(e, sk.astype(np.int8), got, qf, h.shape[0])
                    assert np.array_equal(scores, ohdc.scores_mod_t(h, C, o.t)), (rep, k)
        finally:
            b.close()
    finally:
        s.close()


def test_folded_subring_requests_in_batches():
    """Folded subring sessions in one batch with an unfolded one: their groups run through the
    subring models' n-point kernels, the finish kernel leaves the sums in each request's
    rotation workspace, and rotate-and-sum and the output transform follow per request.
    Unpacked (queries encoded beforehand), every request's ciphertexts equal the oracle's;
    packed (queries encoded in the batch), every request decrypts to its exact scores, over
    two runs of the batch."""
    torch = torch_cuda()
    from oracle import hdc as ohdc
    F = 48
    shapes = [(4096, 3, 3, 128, 2, 2), (2048, 2, 2, 64, 4, 2), (2048, 2, 5, 64, 1, 0)]  # N, L, K, D, r, dnum
    tenants = []
    for k, (N, L, K, D, r, dnum) in enumerate(shapes):
        if r > 1:
            o, e = make_fold(N, L, D, K, r, dnum, F=F)
        else:
            o, e = make(N, L, D, K, F=F)
        rng = np.random.default_rng(40 + k)
        C = values(rng, 8, (K, D))
        sk = bfv.secret_key(o, 40 + k)
        model = bfv.encrypt_model(o, sk, C, 40 + k)
        gk = bfv.galois_keys(o, sk, 50 + k) if r > 1 else None
        s = ep.Session(e, to_dev(model.astype(np.uint32)), to_dev(gk.astype(np.uint32)) if gk is not None else None,
                       max_Q=1500)
        base = synth.base_hypervectors(60 + k, F, D)
        tenants.append(dict(o=o, e=e, C=C, sk=sk, model=model, gk=gk, s=s, base=base, d_base=to_dev(base)))
    plan = [(0, 700), (1, 300), (2, 400), (0, 3), (1, 1000), (2, 30)]
    try:
        rng = np.random.default_rng(46)
        hs = [values(rng, 1, (Q, tenants[ti]["o"].D)) for ti, Q in plan]
        reqs = []
        for (ti, Q), h in zip(plan, hs):
            t = tenants[ti]
            out = torch.zeros((t["s"].num_groups(Q), 2, t["o"].L, t["o"].N), dtype=torch.int32, device="cuda")
            reqs.append(ep.Request(t["s"], to_dev(hv_layout(h, t["s"].hv_stride(Q))), Q, out))
        b = ep.Batch(reqs)
        try:
            b.run()
            torch.cuda.synchronize()
        finally:
            b.close()
        for k, ((ti, Q), h, r) in enumerate(zip(plan, hs, reqs)):
            t = tenants[ti]
            want = pipeline.score_ciphertexts(t["o"], t["model"], h, t["gk"])
            assert np.array_equal(to_host_u32(r.d_score_ct).astype(np.int64), want), k
        xs = [synth.uniform_features(70 + k, Q, F) for k, (ti, Q) in enumerate(plan)]
        preqs = []
        for (ti, Q), x in zip(plan, xs):
            t = tenants[ti]
            out = torch.zeros((t["s"].num_groups(Q) + 1, 2, t["o"].L, t["o"].N), dtype=torch.int32, device="cuda")
            preqs.append(ep.Request(t["s"], None, Q, out, d_x=to_dev(x), d_base=t["d_base"]))
        b = ep.Batch(preqs, packed=True)
        try:
            for rep in range(2):
                b.run()
                torch.cuda.synchronize()
                for k, ((ti, Q), x, r) in enumerate(zip(plan, xs, preqs)):
                    t = tenants[ti]
                    h = ohdc.encode(x, t["base"], t["o"].qbits, t["o"].qshift)
                    off, qf, nct = b.packing(k)
                    got = to_host_u32(r.d_score_ct)[:nct]
                    scores, _ = ep.ephdc_decrypt_scores_at(t["e"], t["sk"].astype(np.int8), got, qf, Q)
                    assert np.array_equal(scores, ohdc.scores_mod_t(h, t["C"], t["o"].t)), (rep, k)
        finally:
            b.close()
    finally:
        for t in tenants:
            t["s"].close()


def make_layout(N, L, D, K, r, layout, F=64):
    primes = default_primes(N, L + (2 if r > 1 else 0))
    args = dict(N=N, q=tuple(primes[:L]), F=F, D=D, K=K, r=r, layout=layout)
    if r > 1:
        args.update(p=tuple(primes[L:]), dnum=2)
    o = OParams(**args)
    o.validate()
    return o, ep.Params(**args)


@pytest.mark.parametrize("N,L,K,D,Q,r,layout", [(4096, 3, 3, 37, 700, 1, "subring"), (2048, 2, 2, 21, 300, 4, "subring"),
                                                (4096, 3, 3, 37, 700, 1, "contiguous"),
                                                (2048, 2, 2, 21, 300, 4, "contiguous")])
def test_single_request_reads_padding_as_zero(N, L, K, D, Q, r, layout):
    """The batch encoding of a single request (n-point kernels of the subring layout, N-point
    kernels of the contiguous one) reads the positions past Q of its last group as zero:
    nonzero bytes in the padding columns leave the ciphertexts equal to the oracle's (whose
    missing queries are zero)."""
    torch = torch_cuda()
    o, e = make_layout(N, L, D, K, r, layout)
    rng = np.random.default_rng(N + Q)
    C = values(rng, 8, (K, D))
    h = values(rng, 1, (Q, D))
    sk = bfv.secret_key(o, 8)
    model = bfv.encrypt_model(o, sk, C, 8)
    gk = bfv.galois_keys(o, sk, 9) if r > 1 else None
    s = ep.Session(e, to_dev(model.astype(np.uint32)), to_dev(gk.astype(np.uint32)) if gk is not None else None,
                   max_Q=Q)
    try:
        stride = s.hv_stride(Q)
        assert stride > Q
        lay = hv_layout(h, stride).reshape(D, stride).copy()
        lay[:, Q:] = 55
        out = torch.empty((s.num_groups(Q), 2, o.L, o.N), dtype=torch.int32, device="cuda")
        ep.ephdc_score_encrypted(s, to_dev(lay), Q, out)
        torch.cuda.synchronize()
        assert np.array_equal(to_host_u32(out).astype(np.int64), pipeline.score_ciphertexts(o, model, h, gk))
    finally:
        s.close()
