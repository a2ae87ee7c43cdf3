"""Request batches through the C ABI (needs a gfx950 GPU): many requests of different sizes,
models (K, D, r) and ring dimensions scored by shared persistent launches give, request by
request, the oracle's score ciphertexts -- under every schedule, and on every replay of a
captured HIP graph."""
import numpy as np
import pytest

import paper_2511_00737_amd as ep
import synth
from oracle import bfv, hdc, pipeline
from oracle.params import Params as OParams, default_primes

from gpu_helpers import hv_layout, to_dev, to_host_u32, torch_cuda

pytestmark = pytest.mark.gpu

# (N, L, K, D, r, alpha, dnum): tenants sharing N = 4096 (one with a folded packing), and
# one at N = 8192, so the batch has two parameter sets
TENANTS = [(4096, 3, 2, 64, 1, 0, 0), (4096, 3, 5, 100, 1, 0, 0), (4096, 3, 3, 40, 4, 1, 3),
           (8192, 4, 7, 48, 1, 0, 0)]
# (tenant, Q, encode inside the batch)
REQUESTS = [(0, 1, True), (1, 7, False), (2, 300, False), (0, 1500, True), (3, 2500, False), (1, 3000, False),
            (2, 5, False), (3, 1, False), (0, 64, False)]
F = 64


class Tenant:
    def __init__(self, i, N, L, K, D, r, alpha, dnum):
        primes = default_primes(N, L + alpha)
        kw = dict(N=N, q=tuple(primes[:L]), p=tuple(primes[L:]), F=F, D=D, K=K, r=r, dnum=dnum)
        self.o, self.e = OParams(**kw), ep.Params(**kw)
        self.sk = bfv.secret_key(self.o, 20 + i)
        self.C = synth.class_hypervectors(30 + i, K, D)
        self.model = bfv.encrypt_model(self.o, self.sk, self.C, 40 + i)
        self.gk = bfv.galois_keys(self.o, self.sk, 50 + i) if r > 1 else None
        self.base = synth.base_hypervectors(60 + i, F, D)


@pytest.fixture(scope="module")
def world():
    torch = torch_cuda()
    tenants = [Tenant(i, *t) for i, t in enumerate(TENANTS)]
    sessions = []
    for i, t in enumerate(tenants):
        max_Q = max(Q for ti, Q, _ in REQUESTS if ti == i)
        sessions.append(ep.Session(t.e, to_dev(t.model.astype(np.uint32)),
                                   to_dev(t.gk.astype(np.uint32)) if t.gk is not None else None, max_Q=max_Q))
    reqs, want_h = [], []
    for k, (ti, Q, enc) in enumerate(REQUESTS):
        t, s = tenants[ti], sessions[ti]
        G = s.num_groups(Q)
        out = torch.zeros((G, 2, t.o.L, t.o.N), dtype=torch.int32, device="cuda")
        if enc:
            x = synth.uniform_features(70 + k, Q, F)
            h = hdc.encode(x, t.base)
            d_hv = torch.full((t.o.D, s.hv_stride(Q)), 99, dtype=torch.int8, device="cuda")
            reqs.append(ep.Request(s, d_hv, Q, out, d_x=to_dev(x), d_base=to_dev(t.base)))
        else:
            h = np.random.default_rng(k).choice(np.array([-1, 1], dtype=np.int8), (Q, t.o.D))
            reqs.append(ep.Request(s, to_dev(hv_layout(h, s.hv_stride(Q))), Q, out))
        want_h.append(h)
    # oracle, on the first and last groups of every request (all groups when few)
    want = []
    for (ti, Q, _), h in zip(REQUESTS, want_h):
        t = tenants[ti]
        G = t.o.groups(Q)
        groups = sorted({0, G - 1})
        want.append((groups, pipeline.score_ciphertexts(t.o, t.model, h, t.gk, groups=groups)))
    yield dict(torch=torch, tenants=tenants, sessions=sessions, reqs=reqs, h=want_h, want=want)
    for s in sessions:
        s.close()


def _outputs(w):
    w["torch"].cuda.synchronize()
    return [to_host_u32(r.d_score_ct).astype(np.int64) for r in w["reqs"]]


def _check(w, got, tag):
    for k, (g_out, (groups, want)) in enumerate(zip(got, w["want"])):
        for i, g in enumerate(groups):
            assert np.array_equal(g_out[g], want[i]), (tag, k, g)


def _clear(w):
    for r in w["reqs"]:
        r.d_score_ct.fill_(0)


def test_batch_matches_oracle_and_single_requests(world):
    w = world
    _clear(w)
    b = ep.Batch(w["reqs"])
    try:
        b.run()
        got = _outputs(w)
    finally:
        b.close()
    _check(w, got, "default")
    # hypervectors encoded inside the batch
    for (ti, Q, enc), r, h in zip(REQUESTS, w["reqs"], w["h"]):
        if enc:
            assert np.array_equal(r.d_hv.cpu().numpy()[:, :Q], h.T)
    # every group of every request equals the single-request path, and decrypts exactly
    torch = w["torch"]
    for k, ((ti, Q, _), r) in enumerate(zip(REQUESTS, w["reqs"])):
        t, s = w["tenants"][ti], w["sessions"][ti]
        one = torch.empty_like(r.d_score_ct)
        ep.ephdc_score_encrypted(s, r.d_hv, Q, one)
        torch.cuda.synchronize()
        assert np.array_equal(to_host_u32(one).astype(np.int64), got[k]), k
        scores, _ = pipeline.decrypt_scores(t.o, t.sk, got[k], Q)
        assert np.array_equal(scores, hdc.scores_mod_t(w["h"][k], t.C, 65537)), k


def test_score_many_matches_oracle(world):
    w = world
    _clear(w)
    ep.ephdc_score_many(w["reqs"])
    _check(w, _outputs(w), "score_many")


@pytest.mark.parametrize("mode", ["split", "fused"])
def test_every_batch_schedule_gives_the_same_bits(world, mode):
    w = world
    b = ep.Batch(w["reqs"])
    try:
        for vpt in (8,):
            for lg in (1,):
                for seg_len in (64, 1024):
                    for grid in (7, 512):
                        b.tune(mode=mode, values_per_thread=vpt, limb_group=lg, seg_len=seg_len, grid=grid)
                        _clear(w)
                        b.run()
                        _check(w, _outputs(w), (mode, vpt, lg, seg_len, grid))
    finally:
        b.close()


def test_limb_groups_and_shapes_at_n8192(world):
    """A batch of the N = 8192 tenant alone: every values-per-thread shape and limb group."""
    w = world
    idx = [k for k, (ti, _, _) in enumerate(REQUESTS) if ti == 3]
    reqs = [w["reqs"][k] for k in idx]
    b = ep.Batch(reqs)
    try:
        for mode in ("split", "fused"):
            for vpt in (8, 16):
                for lg in (1, 2, 4):
                    b.tune(mode=mode, values_per_thread=vpt, limb_group=lg, seg_len=32, grid=300)
                    for r in reqs:
                        r.d_score_ct.fill_(0)
                    b.run()
                    w["torch"].cuda.synchronize()
                    for k in idx:
                        got = to_host_u32(w["reqs"][k].d_score_ct).astype(np.int64)
                        groups, want = w["want"][k]
                        for i, g in enumerate(groups):
                            assert np.array_equal(got[g], want[i]), (mode, vpt, lg, k, g)
    finally:
        b.close()


def test_captured_graph_replays_match(world):
    """Every replay of the captured graph, with eager work on the same buffers between
    replays, reproduces the oracle's ciphertexts."""
    w = world
    torch = w["torch"]
    st = torch.cuda.Stream()
    b = ep.Batch(w["reqs"])
    try:
        b.tune(mode="split", seg_len=64, grid=256)
        b.capture(st)
        for rep in range(3):
            _clear(w)
            torch.cuda.synchronize()
            b.run(st)
            st.synchronize()
            _check(w, _outputs(w), ("replay", rep))
            # eager work between replays: a single-request score into the first output
            r0 = w["reqs"][0]
            ep.ephdc_score_encrypted(r0.session, r0.d_hv, r0.Q, r0.d_score_ct)
            torch.cuda.synchronize()
    finally:
        b.close()


def test_autotuner_keeps_a_valid_schedule(world):
    w = world
    b = ep.Batch(w["reqs"])
    try:
        sched, ms = b.autotune(reps=1)
        assert ms > 0 and sched["mode"] in ("split", "fused")
        _clear(w)
        b.run()
        _check(w, _outputs(w), ("autotuned", sched))
    finally:
        b.close()


# tenants whose D allows encoding inside the batch (D % 64 == 0), one of them folded (r = 2)
PACK_TENANTS = [(4096, 3, 2, 64, 1, 0, 0), (4096, 3, 3, 128, 2, 1, 3), (8192, 4, 7, 64, 1, 0, 0)]
PACK_REQUESTS = [(0, 300), (1, 7), (0, 1), (2, 700), (1, 333), (0, 2000), (2, 1), (1, 250), (0, 64), (2, 900)]


def test_packed_batch_matches_oracle():
    """Packing: requests of one session share ciphertexts.  Each request receives the
    ciphertexts of its session's query sequence that hold its queries -- equal bit for bit
    to the oracle's ciphertexts of the concatenated sequence -- and decrypting them at its
    offset gives exactly its own scores."""
    torch = torch_cuda()
    tenants = [Tenant(10 + i, *t) for i, t in enumerate(PACK_TENANTS)]
    sessions = []
    for i, t in enumerate(tenants):
        mq = max(Q for ti, Q in PACK_REQUESTS if ti == i)
        sessions.append(ep.Session(t.e, to_dev(t.model.astype(np.uint32)),
                                   to_dev(t.gk.astype(np.uint32)) if t.gk is not None else None, max_Q=mq))
    try:
        reqs, hs = [], []
        for k, (ti, Q) in enumerate(PACK_REQUESTS):
            t, s = tenants[ti], sessions[ti]
            x = synth.uniform_features(300 + k, Q, F)
            hs.append(hdc.encode(x, t.base))
            out = torch.zeros((s.num_groups(Q) + 1, 2, t.o.L, t.o.N), dtype=torch.int32, device="cuda")
            reqs.append(ep.Request(s, None, Q, out, d_x=to_dev(x), d_base=to_dev(t.base)))
        b = ep.Batch(reqs, packed=True)
        try:
            for rep in range(2):  # a second run reproduces the first
                for r in reqs:
                    r.d_score_ct.fill_(0)
                b.run()
                torch.cuda.synchronize()
                seq = {i: np.concatenate([hs[k] for k, (ti, _) in enumerate(PACK_REQUESTS) if ti == i])
                       for i in range(len(tenants))}
                for k, ((ti, Q), r) in enumerate(zip(PACK_REQUESTS, reqs)):
                    t = tenants[ti]
                    off, qf, nct = b.packing(k)
                    B = t.o.B
                    assert qf == off % B and nct == (off + Q - 1) // B - off // B + 1
                    got = to_host_u32(r.d_score_ct)[:nct]
                    want = pipeline.score_ciphertexts(t.o, t.model, seq[ti], t.gk,
                                                      groups=list(range(off // B, off // B + nct)))
                    assert np.array_equal(got.astype(np.int64), want), (rep, k)
                    scores, _ = ep.ephdc_decrypt_scores_at(t.e, t.sk.astype(np.int8), got, qf, Q)
                    assert np.array_equal(scores, hdc.scores_mod_t(hs[k], t.C, 65537)), (rep, k)
        finally:
            b.close()
    finally:
        for s in sessions:
            s.close()


def test_batch_at_n16384_with_rotations():
    """A batch whose parameter set is N = 16384 (the 1024-thread transform shape without an
    LDS table slot): two models, one folded (r = 4, two rotate-and-sum steps with key
    switching), requests with and without HDC encoding inside the batch. Unpacked, every
    request equals the single-request path bit for bit and the oracle on its groups;
    packed, every request decrypts at its offset to its exact scores."""
    torch = torch_cuda()
    specs = [(16384, 4, 5, 64, 4, 1, 2), (16384, 4, 2, 64, 1, 0, 0)]
    reqspec = [(0, 1, True), (0, 600, False), (1, 300, True), (1, 2000, False), (0, 150, True)]
    tenants = [Tenant(90 + i, *t) for i, t in enumerate(specs)]
    sessions = [ep.Session(t.e, to_dev(t.model.astype(np.uint32)),
                           to_dev(t.gk.astype(np.uint32)) if t.gk is not None else None, max_Q=2000)
                for t in tenants]
    try:
        reqs, hs = [], []
        for k, (ti, Q, enc) in enumerate(reqspec):
            t, s = tenants[ti], sessions[ti]
            out = torch.zeros((s.num_groups(Q), 2, t.o.L, t.o.N), dtype=torch.int32, device="cuda")
            if enc:
                x = synth.uniform_features(170 + k, Q, F)
                hs.append(hdc.encode(x, t.base))
                d_hv = torch.full((t.o.D, s.hv_stride(Q)), 99, dtype=torch.int8, device="cuda")
                reqs.append(ep.Request(s, d_hv, Q, out, d_x=to_dev(x), d_base=to_dev(t.base)))
            else:
                hs.append(np.random.default_rng(k).choice(np.array([-1, 1], dtype=np.int8), (Q, t.o.D)))
                reqs.append(ep.Request(s, to_dev(hv_layout(hs[-1], s.hv_stride(Q))), Q, out))
        b = ep.Batch(reqs)
        try:
            b.run()
            torch.cuda.synchronize()
            first = [r.d_score_ct.clone() for r in reqs]
            # the other shapes and paths of the list kernels give the same bits
            for mode, vpt, lg in (("split", 32, 1), ("fused", 16, 1), ("fused", 32, 2), ("split", 16, 2),
                                  ("split", 16, 4)):
                for r in reqs:
                    r.d_score_ct.fill_(0)
                b.tune(mode=mode, values_per_thread=vpt, limb_group=lg, seg_len=8, grid=300)
                b.run()
                torch.cuda.synchronize()
                for k, (r, f) in enumerate(zip(reqs, first)):
                    assert torch.equal(r.d_score_ct, f), (mode, vpt, lg, k)
        finally:
            b.close()
        for k, ((ti, Q, enc), r, h) in enumerate(zip(reqspec, reqs, hs)):
            t, s = tenants[ti], sessions[ti]
            got = to_host_u32(r.d_score_ct).astype(np.int64)
            if enc:
                assert np.array_equal(r.d_hv.cpu().numpy()[:, :Q], h.T), k
            one = torch.empty_like(r.d_score_ct)
            ep.ephdc_score_encrypted(s, r.d_hv, Q, one)
            torch.cuda.synchronize()
            assert np.array_equal(to_host_u32(one).astype(np.int64), got), k
            G = t.o.groups(Q)
            want = pipeline.score_ciphertexts(t.o, t.model, h, t.gk, groups=[G - 1])
            assert np.array_equal(got[G - 1], want[0]), k
            scores, _ = pipeline.decrypt_scores(t.o, t.sk, got, Q)
            assert np.array_equal(scores, hdc.scores_mod_t(h, t.C, 65537)), k
        # packed (the requests with features): requests of a model share ciphertexts
        enc = [k for k, (_, _, e) in enumerate(reqspec) if e]
        outs = [torch.zeros((reqs[k].d_score_ct.shape[0] + 1,) + tuple(reqs[k].d_score_ct.shape[1:]),
                            dtype=torch.int32, device="cuda") for k in enc]
        pb = ep.Batch([ep.Request(reqs[k].session, None, reqs[k].Q, o, d_x=reqs[k].d_x, d_base=reqs[k].d_base)
                       for k, o in zip(enc, outs)], packed=True)
        try:
            pb.run()
            torch.cuda.synchronize()
            for i, k in enumerate(enc):
                (ti, Q, _), h, t = reqspec[k], hs[k], tenants[reqspec[k][0]]
                _, qf, nct = pb.packing(i)
                got = to_host_u32(outs[i])[:nct]
                scores, _ = ep.ephdc_decrypt_scores_at(t.e, t.sk.astype(np.int8), got, qf, Q)
                assert np.array_equal(scores, hdc.scores_mod_t(h, t.C, 65537)), k
        finally:
            pb.close()
    finally:
        for s in sessions:
            s.close()
