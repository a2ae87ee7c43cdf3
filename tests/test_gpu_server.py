"""Serving loop on the GPU (C ABI): requests of several tenants arriving while others run
are scored by continuous batches; each result equals the request scored alone, bit for
bit, and decrypts to the exact scores; admission respects the device-memory budget."""
import time

import numpy as np
import pytest

import paper_2511_00737_amd as ep
import synth
from oracle import bfv, hdc, pipeline
from oracle.params import Params as OParams, default_primes

from gpu_helpers import to_dev, to_host_u32, torch_cuda

pytestmark = pytest.mark.gpu

F = 64
# (N, L, K, D, r, alpha, dnum): two parameter sets with a folded model at N = 4096, one at
# N = 8192 and a folded model at N = 16384 (the 1024-thread transform shape)
TENANTS = [(4096, 3, 2, 64, 1, 0, 0), (4096, 3, 3, 128, 2, 1, 3), (8192, 4, 7, 64, 1, 0, 0),
           (16384, 3, 5, 64, 4, 1, 3)]


class Tenant:
    def __init__(self, i, N, L, K, D, r, alpha, dnum, max_Q):
        torch = torch_cuda()
        primes = default_primes(N, L + alpha)
        kw = dict(N=N, q=tuple(primes[:L]), p=tuple(primes[L:]), F=F, D=D, K=K, r=r, dnum=dnum)
        self.o, self.e = OParams(**kw), ep.Params(**kw)
        self.sk = bfv.secret_key(self.o, 80 + i)
        self.C = synth.class_hypervectors(81 + i, K, D)
        self.model = bfv.encrypt_model(self.o, self.sk, self.C, 82 + i)
        self.gk = bfv.galois_keys(self.o, self.sk, 83 + i) if r > 1 else None
        self.base = synth.base_hypervectors(84 + i, F, D)
        self.d_base = to_dev(self.base)
        self.s = ep.Session(self.e, to_dev(self.model.astype(np.uint32)),
                            to_dev(self.gk.astype(np.uint32)) if self.gk is not None else None, max_Q=max_Q)
        self.torch = torch

    def out(self, Q):
        return self.torch.zeros((self.s.num_groups(Q), 2, self.o.L, self.o.N), dtype=self.torch.int32, device="cuda")


@pytest.fixture(scope="module")
def tenants():
    ts = [Tenant(i, *t, max_Q=1500) for i, t in enumerate(TENANTS)]
    yield ts
    for t in ts:
        t.s.close()


def test_results_are_the_same_alone_and_in_the_mix(tenants):
    torch = tenants[0].torch
    rng = np.random.default_rng(2026)
    sv = ep.Server(1 << 30, streams=2, max_batch=8)
    try:
        ids = [sv.add_tenant(t.s, t.d_base) for t in tenants]
        jobs = []
        for k in range(40):
            ti = int(rng.integers(0, len(tenants)))
            Q = int(rng.integers(1, 1500))
            t = tenants[ti]
            x = synth.uniform_features(900 + k, Q, F)
            d_x, out = to_dev(x), t.out(Q)
            tk = sv.submit(ids[ti], d_x, Q, out)
            jobs.append((tk, ti, Q, x, d_x, out))
            if k % 5 == 4:
                time.sleep(0.002)  # later requests arrive while earlier batches run
        sv.wait(0, timeout_s=120)
        stats = sv.stats()
        assert stats["failed"] == 0 and stats["completed"] == 40 and stats["rejected"] == 0
        assert stats["batches"] >= 2 and stats["p99_ms"] >= stats["p50_ms"] > 0
        for tk, ti, Q, x, d_x, out in jobs:
            state, (ts, ta, td) = sv.query(tk)
            assert state == 2 and ts <= ta <= td
    finally:
        sv.close()
    # each request alone, through the single-request entry points
    for n, (tk, ti, Q, x, d_x, out) in enumerate(jobs):
        t = tenants[ti]
        d_hv = torch.empty((t.o.D, t.s.hv_stride(Q)), dtype=torch.int8, device="cuda")
        alone = t.out(Q)
        ep.ephdc_encode_queries(t.s, d_x, t.d_base, Q, d_hv)
        ep.ephdc_score_encrypted(t.s, d_hv, Q, alone)
        torch.cuda.synchronize()
        got = to_host_u32(out).astype(np.int64)
        assert np.array_equal(got, to_host_u32(alone).astype(np.int64)), n
        if n % 8 == 0:  # and against the oracle: exact scores, and the last group's ciphertext
            h = hdc.encode(x, t.base)
            scores, _ = pipeline.decrypt_scores(t.o, t.sk, got, Q)
            assert np.array_equal(scores, hdc.scores_mod_t(h, t.C, 65537)), n
            G = t.o.groups(Q)
            want = pipeline.score_ciphertexts(t.o, t.model, h, t.gk, groups=[G - 1])
            assert np.array_equal(got[G - 1], want[0]), n


def test_admission_by_device_memory(tenants):
    """A 64 MiB budget where one request of an N = 8192, D = 2048 tenant takes about 44 MiB
    (query hypervectors, partial sums, plaintext chunk): at most two fit at once, so the
    requests are admitted in several batches without ever exceeding the budget, and a
    request too large for the whole budget is rejected while the others complete."""
    torch = tenants[0].torch
    budget = 64 << 20
    primes = default_primes(8192, 4)
    prm = ep.Params(N=8192, q=tuple(primes), F=F, D=2048, K=2)
    sk, _ = ep.ephdc_keygen(prm, 7)
    C = synth.class_hypervectors(7, 2, 2048)
    base = synth.base_hypervectors(7, F, 2048)
    sess = ep.Session(prm, to_dev(ep.ephdc_encrypt_model(prm, sk, C, 7)), max_Q=4096)
    big_prm = ep.Params(N=8192, q=tuple(primes), F=F, D=8192, K=2)
    big = ep.Session(big_prm, torch.zeros((8192, 2, 4, 8192), dtype=torch.int32, device="cuda"), max_Q=4096)
    sv = ep.Server(budget, streams=2, max_batch=64)
    try:
        tid = sv.add_tenant(sess, to_dev(base))
        bid = sv.add_tenant(big, torch.zeros((F, 8192), dtype=torch.int8, device="cuda"))
        jobs = []
        for k in range(5):
            Q = 300 + 211 * k
            x = synth.uniform_features(1100 + k, Q, F)
            out = torch.zeros((sess.num_groups(Q), 2, 4, 8192), dtype=torch.int32, device="cuda")
            jobs.append((sv.submit(tid, to_dev(x), Q, out), Q, x, out))
        big_out = torch.zeros((big.num_groups(4096), 2, 4, 8192), dtype=torch.int32, device="cuda")
        btk = sv.submit(bid, torch.zeros((4096, F), dtype=torch.uint8, device="cuda"), 4096, big_out)
        sv.wait(0, timeout_s=120)
        assert sv.query(btk)[0] == -ep.ERR_OOM
        with pytest.raises(ep.EphdcError):
            sv.wait(btk)
        stats = sv.stats()
        assert stats["completed"] == 5 and stats["rejected"] == 1
        assert 0 < stats["peak_bytes"] <= budget and stats["batches"] >= 3
        for tk, Q, x, out in jobs:
            assert sv.query(tk)[0] == 2
            scores, _ = ep.ephdc_decrypt_scores(prm, sk, to_host_u32(out), Q)
            assert np.array_equal(scores, hdc.scores_mod_t(hdc.encode(x, base), C, 65537))
    finally:
        sv.close()
        sess.close()
        big.close()


def test_packed_serving_gives_each_request_its_scores(tenants):
    """With packing, requests of a tenant share ciphertexts; each request's output holds the
    ciphertexts with its queries, and decrypting them at its offset gives its own scores.
    The requests are submitted on a caller stream held by a chain of matrix products: the
    first batches wait for it on both server streams, so the rest queue and later batches
    take several requests of a tenant, which then share ciphertexts."""
    torch = tenants[0].torch
    rng = np.random.default_rng(77)
    specs = []
    for k in range(30):
        ti = int(rng.integers(0, len(tenants)))
        Q = int(rng.integers(1, 700))
        t = tenants[ti]
        x = synth.uniform_features(1300 + k, Q, F)
        out = torch.zeros((t.s.num_groups(Q) + 1, 2, t.o.L, t.o.N), dtype=torch.int32, device="cuda")
        specs.append((ti, Q, x, to_dev(x), out))
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    sv = ep.Server(1 << 30, streams=2, max_batch=16)
    try:
        sv.set_packing(True)
        ids = [sv.add_tenant(t.s, t.d_base) for t in tenants]
        with torch.cuda.stream(side):
            big = torch.randn((4096, 4096), device="cuda")
            for _ in range(16):
                big = big @ big
                big = big / big.abs().max()
            jobs = [(sv.submit(ids[ti], d_x, Q, out, stream=side), ti, Q, x, out) for ti, Q, x, d_x, out in specs]
        sv.wait(0, timeout_s=120)
        assert sv.stats()["completed"] == 30
        shared = 0
        for tk, ti, Q, x, out in jobs:
            t = tenants[ti]
            qf, nct = sv.result(tk)
            shared += qf > 0
            assert nct == (qf + Q - 1) // t.o.B + 1
            got = to_host_u32(out)[:nct]
            scores, _ = ep.ephdc_decrypt_scores_at(t.e, t.sk.astype(np.int8), got, qf, Q)
            assert np.array_equal(scores, hdc.scores_mod_t(hdc.encode(x, t.base), t.C, 65537)), tk
        assert shared > 0  # some requests did share a ciphertext with an earlier one
    finally:
        sv.close()


def test_submission_waits_for_the_callers_stream(tenants):
    """The features of each request are written by a kernel on the caller's stream that is
    still running when the request is submitted: the served result equals the request
    scored alone from the same features (the server waited for that stream)."""
    torch = tenants[0].torch
    t = tenants[2]  # N = 8192
    side = torch.cuda.Stream()
    sv = ep.Server(1 << 30, streams=2, max_batch=4)
    try:
        tid = sv.add_tenant(t.s, t.d_base)
        jobs = []
        for k in range(6):
            Q = 400 + 97 * k
            src = to_dev(synth.uniform_features(1300 + k, Q, F))
            d_x = torch.zeros((Q, F), dtype=torch.uint8, device="cuda")
            out = t.out(Q)
            torch.cuda.synchronize()
            with torch.cuda.stream(side):
                # a long kernel first, then the copy that writes d_x, all on `side`
                big = torch.randn((4096, 4096), device="cuda")
                for _ in range(8):
                    big = big @ big
                    big = big / big.abs().max()
                d_x.copy_(src)
                tk = sv.submit(tid, d_x, Q, out, stream=side)
            jobs.append((tk, Q, src, out))
        sv.wait(0, timeout_s=120)
        assert sv.stats()["failed"] == 0
    finally:
        sv.close()
    for tk, Q, src, out in jobs:
        d_hv = torch.empty((t.o.D, t.s.hv_stride(Q)), dtype=torch.int8, device="cuda")
        alone = t.out(Q)
        ep.ephdc_encode_queries(t.s, src, t.d_base, Q, d_hv)
        ep.ephdc_score_encrypted(t.s, d_hv, Q, alone)
        torch.cuda.synchronize()
        assert np.array_equal(to_host_u32(out), to_host_u32(alone))


def test_ticket_count_stays_bounded_over_thousands_of_requests(tenants):
    """3000 small requests, each released once done: the server's tracked tickets stay
    bounded by what is queued or running, and sampled results equal the request alone."""
    torch = tenants[0].torch
    t = tenants[0]  # N = 4096, D = 64
    sv = ep.Server(1 << 30, streams=2, max_batch=64)
    pool = to_dev(synth.uniform_features(1400, 64, F))
    try:
        tid = sv.add_tenant(t.s, t.d_base)
        live, peak, checks = [], 0, []
        for k in range(3000):
            Q = 1 + k % 37
            out = t.out(Q)
            tk = sv.submit(tid, pool[:Q], Q, out)
            live.append((tk, Q, out))
            if k % 100 == 99:
                sv.wait(tk, timeout_s=60)
                still = []
                for item in live:
                    if sv.query(item[0])[0] == 2:
                        if len(checks) < 5 and item[0] % 7 == 0:
                            checks.append(item)
                        sv.release(item[0])
                    else:
                        still.append(item)
                live = still
                peak = max(peak, int(sv.stats()["tickets"]))
        sv.wait(0, timeout_s=60)
        stats = sv.stats()
        assert stats["completed"] == 3000 and stats["failed"] == 0
        assert peak <= 200, peak
        for tk, Q, out in live:
            if sv.query(tk)[0] == 2:
                sv.release(tk)
        assert sv.stats()["tickets"] == 0
        with pytest.raises(ep.EphdcError):
            sv.query(checks[0][0])  # released
    finally:
        sv.close()
    for tk, Q, out in checks:
        d_hv = torch.empty((t.o.D, t.s.hv_stride(Q)), dtype=torch.int8, device="cuda")
        alone = t.out(Q)
        ep.ephdc_encode_queries(t.s, pool[:Q], t.d_base, Q, d_hv)
        ep.ephdc_score_encrypted(t.s, d_hv, Q, alone)
        torch.cuda.synchronize()
        assert np.array_equal(to_host_u32(out), to_host_u32(alone))


def test_serving_subring_tenants_unpacked_and_packed():
    """Tenants in the subring layout (scored per model as lists of virtual groups by the
    n-point kernels) beside a contiguous tenant on the same primes: unpacked, each request
    equals the request scored alone (and the oracle on a sample); packed, each decrypts at
    its offset to its exact scores."""
    torch = torch_cuda()
    specs = [(4096, 3, 3, 64, "subring"), (4096, 3, 2, 64, "contiguous"), (8192, 4, 7, 64, "subring")]
    ts = []
    for i, (N, L, K, D, lay) in enumerate(specs):
        kw = dict(N=N, q=tuple(default_primes(N, L)), F=F, D=D, K=K, layout=lay)
        o, e = OParams(**kw), ep.Params(**kw)
        sk = bfv.secret_key(o, 60 + i)
        C = synth.class_hypervectors(61 + i, K, D)
        model = bfv.encrypt_model(o, sk, C, 62 + i)
        base = synth.base_hypervectors(63 + i, F, D)
        ts.append(dict(o=o, e=e, sk=sk, C=C, model=model, base=base, d_base=to_dev(base),
                       s=ep.Session(e, to_dev(model.astype(np.uint32)), max_Q=1500)))
    try:
        for pack in (False, True):
            rng = np.random.default_rng(31 + pack)
            sv = ep.Server(1 << 30, streams=2, max_batch=8)
            try:
                if pack:
                    sv.set_packing(True)
                ids = [sv.add_tenant(t["s"], t["d_base"]) for t in ts]
                jobs = []
                for k in range(24):
                    ti = int(rng.integers(0, len(ts)))
                    Q = int(rng.integers(1, 1500))
                    t = ts[ti]
                    x = synth.uniform_features(1500 + k + 100 * pack, Q, F)
                    d_x = to_dev(x)
                    out = torch.zeros((t["s"].num_groups(Q) + (1 if pack else 0), 2, t["o"].L, t["o"].N),
                                      dtype=torch.int32, device="cuda")
                    jobs.append((sv.submit(ids[ti], d_x, Q, out), ti, Q, x, d_x, out))
                    if k % 6 == 5:
                        time.sleep(0.002)
                sv.wait(0, timeout_s=120)
                assert sv.stats()["completed"] == 24
                for n, (tk, ti, Q, x, d_x, out) in enumerate(jobs):
                    t = ts[ti]
                    h = hdc.encode(x, t["base"])
                    if pack:
                        qf, nct = sv.result(tk)
                        got = to_host_u32(out)[:nct]
                        scores, _ = ep.ephdc_decrypt_scores_at(t["e"], t["sk"].astype(np.int8), got, qf, Q)
                        assert np.array_equal(scores, hdc.scores_mod_t(h, t["C"], 65537)), n
                        continue
                    d_hv = torch.empty((t["o"].D, t["s"].hv_stride(Q)), dtype=torch.int8, device="cuda")
                    alone = torch.empty_like(out)
                    ep.ephdc_encode_queries(t["s"], d_x, t["d_base"], Q, d_hv)
                    ep.ephdc_score_encrypted(t["s"], d_hv, Q, alone)
                    torch.cuda.synchronize()
                    got = to_host_u32(out).astype(np.int64)
                    assert np.array_equal(got, to_host_u32(alone).astype(np.int64)), n
                    if n % 6 == 0:
                        G = t["o"].groups(Q)
                        want = pipeline.score_ciphertexts(t["o"], t["model"], h, groups=[G - 1])
                        assert np.array_equal(got[G - 1], want[0]), n
            finally:
                sv.close()
    finally:
        for t in ts:
            t["s"].close()
