"""The workloads at their full sizes, in the launch configuration the benchmark times,
checked where the oracle can follow them: the tiny workload word for word; the plain-path
workload (N = 8192, 4 limbs, F = 2304, D = 4096, K = 7, 4096 queries) in both slot layouts
with sampled hypervectors, its whole last group word for word and every group decrypted
against the exact integer scores; the rotation and batching workloads, in both slot layouts
as well, as stated at their tests.

The encrypted model comes from the library's host-side encryption (bit-exact with the
oracle's on the CPU tests); every expected value here is computed by the oracle from it.
"""
import numpy as np
import pytest

import paper_2511_00737_amd as ep
import synth
from oracle import bfv, hdc, pipeline
from oracle.params import Params as OParams, default_primes

from gpu_helpers import to_dev, to_host_u32, torch_cuda

pytestmark = pytest.mark.gpu

N, L, F, D, K, Q = 8192, 4, 2304, 4096, 7, 4096


@pytest.mark.parametrize("layout", ["contiguous", "subring"])
def test_plain_workload_at_full_size_sampled(layout):
    """Both slot layouts; the subring session runs the n-point kernels (n = 1024, four full
    groups of 1024 queries) that the benchmark's headline line times."""
    torch = torch_cuda()
    primes = default_primes(N, L)
    o = OParams(N=N, q=tuple(primes), F=F, D=D, K=K, layout=layout)
    o.validate()
    e = ep.Params(N=N, q=tuple(primes), F=F, D=D, K=K, layout=layout)
    sk, _ = ep.ephdc_keygen(e, 0)
    C = synth.class_hypervectors(0, K, D)
    model = ep.ephdc_encrypt_model(e, sk, C, 0)
    x = synth.blob_images(0, Q)
    base = synth.base_hypervectors(0, F, D)

    s = ep.Session(e, to_dev(model), max_Q=Q)  # the benchmark's default schedule
    try:
        stride, G = s.hv_stride(Q), s.num_groups(Q)
        d_hv = torch.empty((D, stride), dtype=torch.int8, device="cuda")
        d_out = torch.empty((G, 2, L, N), dtype=torch.int32, device="cuda")
        ep.ephdc_encode_queries(s, to_dev(x), to_dev(base), Q, d_hv)
        ep.ephdc_score_encrypted(s, d_hv, Q, d_out)
        torch.cuda.synchronize()
        h = d_hv.cpu().numpy()[:, :Q].T.copy()
        assert not d_hv.cpu().numpy()[:, Q:].any()
        cts = to_host_u32(d_out).astype(np.int64)
    finally:
        s.close()

    # sampled queries: the oracle's HDC encoding
    rng = np.random.default_rng(8192)
    qs = np.sort(rng.choice(Q, 48, replace=False))
    assert np.array_equal(h[qs], hdc.encode(x[qs], base))

    # the whole last group (ragged in the contiguous layout), every word of both components
    # and all limbs, against
    # the oracle's multiply-accumulate over all 4096 model ciphertexts
    mdl = model.astype(np.int64)
    g = G - 1
    assert np.array_equal(cts[g], bfv.mac(o, mdl, h, g))

    # every query of every group decrypts to its exact score
    scores, _ = pipeline.decrypt_scores(o, sk.astype(np.int64), cts, Q)
    assert np.array_equal(scores, hdc.scores_mod_t(h, C, o.t))


def test_tiny_workload_at_full_size():
    """The tiny workload exactly (N = 4096, 3 limbs, F = 512 uniform features, D = 2048,
    K = 2, 64 queries, every input from seed 0), in the benchmark's launch configuration:
    every word of the score ciphertext against the oracle's, the oracle's HDC encoding of
    every query, decryption to h . C mod t and the argmax of the exact integer scores."""
    torch = torch_cuda()
    N1, L1, F1, D1, K1, Q1 = 4096, 3, 512, 2048, 2, 64
    primes = default_primes(N1, L1)
    o = OParams(N=N1, q=tuple(primes), F=F1, D=D1, K=K1)
    e = ep.Params(N=N1, q=tuple(primes), F=F1, D=D1, K=K1)
    x = synth.uniform_features(0, Q1, F1)
    base = synth.base_hypervectors(0, F1, D1)
    C = synth.class_hypervectors(0, K1, D1)
    sk = bfv.secret_key(o, 0)
    model = bfv.encrypt_model(o, sk, C, 0)
    s = ep.Session(e, to_dev(model.astype(np.uint32)), max_Q=Q1)
    try:
        stride, G = s.hv_stride(Q1), s.num_groups(Q1)
        d_hv = torch.empty((D1, stride), dtype=torch.int8, device="cuda")
        d_out = torch.empty((G, 2, L1, N1), dtype=torch.int32, device="cuda")
        ep.ephdc_encode_queries(s, to_dev(x), to_dev(base), Q1, d_hv)
        ep.ephdc_score_encrypted(s, d_hv, Q1, d_out)
        torch.cuda.synchronize()
        hv = d_hv.cpu().numpy()
        cts = to_host_u32(d_out).astype(np.int64)
    finally:
        s.close()
    h = hdc.encode(x, base)
    assert np.array_equal(hv[:, :Q1].T, h)
    assert not hv[:, Q1:].any()
    assert G == 1
    assert np.array_equal(cts, pipeline.score_ciphertexts(o, model, h))
    scores, am = pipeline.decrypt_scores(o, sk, cts, Q1)
    assert np.array_equal(scores, hdc.scores_mod_t(h, C, o.t))
    assert np.array_equal(am, hdc.argmax(hdc.scores_int(h, C)))
    sc2, am2 = ep.ephdc_decrypt_scores(e, sk.astype(np.int8), cts.astype(np.uint32), Q1)
    assert np.array_equal(sc2, scores) and np.array_equal(am2, am)


@pytest.mark.parametrize("layout", ["contiguous", "subring"])
def test_rotation_workload_at_full_size_sampled(layout):
    """The rotation workload at its full size (N = 16384, 8 limbs + 2 special primes,
    dnum = 4, r = 8, F = 2304, D = 10240, K = 26, 16384 queries: 211 groups in the
    contiguous layout, 256 of 64 queries in the folded subring layout, three rotate-and-sum
    steps each) in the benchmark's launch configuration: sampled
    hypervectors against the oracle's encoding, sampled groups decrypted by the oracle,
    and every query's scores equal to the exact integer scores mod t."""
    torch = torch_cuda()
    N, L, alpha, dnum, r, F, D, K, Q = 16384, 8, 2, 4, 8, 2304, 10240, 26, 16384
    primes = default_primes(N, L + alpha)
    kw = dict(N=N, q=tuple(primes[:L]), p=tuple(primes[L:]), F=F, D=D, K=K, r=r, dnum=dnum, layout=layout)
    o, e = OParams(**kw), ep.Params(**kw)
    o.validate()
    sk, gk = ep.ephdc_keygen(e, 0)
    C = synth.class_hypervectors(0, K, D)
    model = ep.ephdc_encrypt_model(e, sk, C, 0)
    x = synth.blob_images(0, Q)
    base = synth.base_hypervectors(0, F, D)

    s = ep.Session(e, to_dev(model), to_dev(gk), max_Q=Q)  # the benchmark's default schedule
    try:
        stride, G = s.hv_stride(Q), s.num_groups(Q)
        d_hv = torch.empty((D, stride), dtype=torch.int8, device="cuda")
        d_out = torch.empty((G, 2, L, N), dtype=torch.int32, device="cuda")
        ep.ephdc_encode_queries(s, to_dev(x), to_dev(base), Q, d_hv)
        ep.ephdc_score_encrypted(s, d_hv, Q, d_out)
        torch.cuda.synchronize()
        h = d_hv.cpu().numpy()[:, :Q].T.copy()
        cts = to_host_u32(d_out)
    finally:
        s.close()
    del d_hv, d_out

    rng = np.random.default_rng(16384)
    qs = np.sort(rng.choice(Q, 32, replace=False))
    assert np.array_equal(h[qs], hdc.encode(x[qs], base))

    want = hdc.scores_mod_t(h, C, o.t)
    # the oracle's decryption of sampled groups (first, last and four others)
    gs = sorted({0, G - 1, *rng.choice(G, 4, replace=False).tolist()})
    sko = sk.astype(np.int64)
    for g in gs:
        sc, _ = pipeline.decrypt_scores(o, sko, cts[g:g + 1].astype(np.int64), Q, groups=[g])
        lo, hi = g * o.B, min(Q, (g + 1) * o.B)
        assert np.array_equal(sc[lo:hi], want[lo:hi]), g
    # every group through the library's decryption
    scores, argmax = ep.ephdc_decrypt_scores(e, sk, cts, Q)
    assert np.array_equal(scores, want)
    assert np.array_equal(argmax, hdc.argmax(want))


@pytest.mark.parametrize("layout", ["contiguous", "subring"])
def test_batching_workload_at_full_size_sampled(layout):
    """The batching workload at its full size (256 requests of log-uniform sizes on six
    models, K in {2, 7} x D in {2048, 4096, 10240}, N = 8192, 4 limbs), in both slot layouts
    and the launch configuration the benchmark times: autotuned, graph-captured batches,
    unpacked and packed. The unpacked batch reproduces every request's single-request ciphertexts bit
    for bit; every request decrypts (unpacked, and packed at its offset) to the exact
    scores of its hypervectors, which match the oracle's encoding on sampled requests; the
    oracle decrypts sampled requests itself."""
    torch = torch_cuda()
    N, L, F, nreq = 8192, 4, 2304, 256
    models = [(K, D) for K in (2, 7) for D in (2048, 4096, 10240)]
    primes = default_primes(N, L)
    sizes, midx = synth.batch_mix(0, nreq, len(models))
    pool = synth.blob_images(0, 4096)
    d_pool = to_dev(pool)
    tenants = []
    for k, (K, D) in enumerate(models):
        e = ep.Params(N=N, q=tuple(primes), F=F, D=D, K=K, layout=layout)
        sk, _ = ep.ephdc_keygen(e, k)
        C = synth.class_hypervectors(k, K, D)
        sess = ep.Session(e, to_dev(ep.ephdc_encrypt_model(e, sk, C, k)), max_Q=4096)
        base = synth.base_hypervectors(0, F, D)
        tenants.append(dict(e=e, o=OParams(N=N, q=tuple(primes), F=F, D=D, K=K, layout=layout), sk=sk, C=C, s=sess,
                            base=base, d_base=to_dev(base)))
    try:
        reqs, offs = [], []
        for i in range(nreq):
            t, Q = tenants[int(midx[i])], int(sizes[i])
            off = (i * 977) % (4096 - Q + 1)
            d_hv = torch.empty((t["e"].D, t["s"].hv_stride(Q)), dtype=torch.int8, device="cuda")
            d_out = torch.empty((t["s"].num_groups(Q), 2, L, N), dtype=torch.int32, device="cuda")
            reqs.append(ep.Request(t["s"], d_hv, Q, d_out, d_x=d_pool[off:off + Q], d_base=t["d_base"]))
            offs.append(off)
        # single-request results first
        alone = []
        for r in reqs:
            ep.ephdc_encode_queries(r.session, r.d_x, r.d_base, r.Q, r.d_hv)
            ep.ephdc_score_encrypted(r.session, r.d_hv, r.Q, r.d_score_ct)
            alone.append(r.d_score_ct.clone())
        torch.cuda.synchronize()
        for r in reqs:
            r.d_score_ct.zero_()
        outs_p = [torch.zeros((r.d_score_ct.shape[0] + 1,) + tuple(r.d_score_ct.shape[1:]), dtype=torch.int32,
                              device="cuda") for r in reqs]
        torch.cuda.synchronize()
        stream = torch.cuda.Stream()
        batch = ep.Batch(reqs)
        batch.autotune(reps=1, stream=stream)
        batch.capture(stream)
        batch.run(stream)
        pbatch = ep.Batch([ep.Request(r.session, None, r.Q, o, d_x=r.d_x, d_base=r.d_base)
                           for r, o in zip(reqs, outs_p)], packed=True)
        pbatch.autotune(reps=1, stream=stream)
        pbatch.capture(stream)
        pbatch.run(stream)
        torch.cuda.synchronize()
        rng = np.random.default_rng(256)
        sampled = set(rng.choice(nreq, 6, replace=False).tolist())
        for i, (r, a) in enumerate(zip(reqs, alone)):
            assert torch.equal(r.d_score_ct, a), i
            t = tenants[int(midx[i])]
            h = r.d_hv.cpu().numpy()[:, :r.Q].T.copy()
            want = hdc.scores_mod_t(h, t["C"], 65537)
            cts = to_host_u32(r.d_score_ct)
            scores, _ = ep.ephdc_decrypt_scores(t["e"], t["sk"], cts, r.Q)
            assert np.array_equal(scores, want), i
            _, qf, nct = pbatch.packing(i)
            pscores, _ = ep.ephdc_decrypt_scores_at(t["e"], t["sk"], to_host_u32(outs_p[i])[:nct], qf, r.Q)
            assert np.array_equal(pscores, want), i
            if i in sampled:
                x = pool[offs[i]:offs[i] + r.Q]
                qs = np.unique(np.linspace(0, r.Q - 1, 8).astype(int))
                assert np.array_equal(h[qs], hdc.encode(x[qs], t["base"])), i
                osc, _ = pipeline.decrypt_scores(t["o"], t["sk"].astype(np.int64), cts.astype(np.int64), r.Q)
                assert np.array_equal(osc, want), i
    finally:
        for t in tenants:
            t["s"].close()


def test_served_tenant_of_the_serving_workload_shape():
    """One tenant of the serving workload's large half (N = 16384, 8 limbs + 2 special primes,
    dnum = 4, r = 4: two rotate-and-sum steps; F = 2304 blob images, K = 7, D = 2048) served
    together with an N = 8192 tenant's requests: its score ciphertext equals the oracle's
    word for word (multiply-accumulate and rotations), and every query decrypts to h . C mod t."""
    torch = torch_cuda()
    N, L, alpha, dnum, r, F5, D5, K5, Q5 = 16384, 8, 2, 4, 4, 2304, 2048, 7, 500
    primes = default_primes(N, L + alpha)
    kw = dict(N=N, q=tuple(primes[:L]), p=tuple(primes[L:]), F=F5, D=D5, K=K5, r=r, dnum=dnum)
    o, e = OParams(**kw), ep.Params(**kw)
    sk, gk = ep.ephdc_keygen(e, 50)
    C = synth.class_hypervectors(50, K5, D5)
    model = ep.ephdc_encrypt_model(e, sk, C, 50)
    base = synth.base_hypervectors(50, F5, D5)
    x = synth.blob_images(50, Q5)
    s = ep.Session(e, to_dev(model), to_dev(gk), max_Q=Q5, workspace=None)
    p2 = ep.Params(N=8192, q=tuple(default_primes(8192, 4)), F=F5, D=4096, K=7)
    sk2, _ = ep.ephdc_keygen(p2, 51)
    s2 = ep.Session(p2, to_dev(ep.ephdc_encrypt_model(p2, sk2, synth.class_hypervectors(51, 7, 4096), 51)),
                    max_Q=1024, workspace=None)
    base2 = to_dev(synth.base_hypervectors(51, F5, 4096))
    sv = ep.Server(8 << 30, streams=2, max_batch=8)
    try:
        t_big = sv.add_tenant(s, to_dev(base))
        t_small = sv.add_tenant(s2, base2)
        d_x = to_dev(x)
        out = torch.empty((s.num_groups(Q5), 2, L, N), dtype=torch.int32, device="cuda")
        others = []
        for k in range(3):
            xs = to_dev(synth.blob_images(60 + k, 700))
            o2 = torch.empty((s2.num_groups(700), 2, 4, 8192), dtype=torch.int32, device="cuda")
            others.append((sv.submit(t_small, xs, 700, o2), xs, o2))
        tk = sv.submit(t_big, d_x, Q5, out)
        sv.wait(0, timeout_s=300)
        assert sv.stats()["failed"] == 0 and sv.query(tk)[0] == 2
        cts = to_host_u32(out).astype(np.int64)
    finally:
        sv.close()
        s.close()
        s2.close()
    h = hdc.encode(x, base)
    assert o.groups(Q5) == 1
    want = pipeline.score_ciphertexts(o, model.astype(np.int64), h, gk.astype(np.int64))
    assert np.array_equal(cts, want)
    sc, am = ep.ephdc_decrypt_scores(e, sk, cts.astype(np.uint32), Q5)
    assert np.array_equal(sc, hdc.scores_mod_t(h, C, o.t))
