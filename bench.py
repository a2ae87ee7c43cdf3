"""Benchmark of the EP-HDC client-side path on one MI355X.

One step = one request of the workload: HDC encoding of the queries (int8 MFMA) and
homomorphic scoring against the device-resident encrypted model (batch encoding, ct x pt
MAC, reduction, rotate-and-sum when the packing folds r > 1 blocks per row, and the output
transform), with every input already in HBM.
Prints one JSON line (see the keys below).

    python bench.py [--steps K] [--warmup W] [--workload c2|c1|c4] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import paper_2511_00737_amd as ep  # noqa: E402
import synth  # noqa: E402

METRIC = "encrypted HDC inferences/sec at N=8192 (batched vs plain GPU); p50/p99 latency"

WORKLOADS = {
    # small case the oracle finishes in seconds
    "c1": dict(N=4096, L=3, F=512, D=2048, K=2, Q=64, images=False,
               desc="BFV N=4096, 3x30-bit limbs, t=65537; HDC F=512 uniform uint8, D=2048, K=2; 64 queries"),
    # the metric's workload: plain method on the GPU, one request per launch
    "c2": dict(N=8192, L=4, F=2304, D=4096, K=7, Q=4096, images=True,
               desc="BFV N=8192, 4x30-bit limbs, t=65537; HDC F=2304 (48x48 Gaussian-blob images), "
                    "D=4096, K=7; 4096 queries per request, one request per launch"),
    # batching: 256 requests of log-uniform size over six models, scored together
    "c3": dict(N=8192, L=4, F=2304, requests=256, models=[(K, D) for K in (2, 7) for D in (2048, 4096, 10240)],
               desc="256 requests, sizes floor(exp(U[0, ln 4096])), each on one of six models "
                    "(K in {2, 7} x D in {2048, 4096, 10240}) at BFV N=8192, 4x30-bit limbs; HDC F=2304 "
                    "(48x48 Gaussian-blob images); one graph-captured batch of persistent launches, "
                    "autotuned schedule"),
    # serving: Poisson arrivals over 32 device-resident tenants, half at N = 8192 (the six
    # batching models) and half at N = 16384 with 8+2 limbs and r = 4 (two rotations)
    "c5": dict(serving=True, rate=2000.0, duration=5.0, qmax=512, tenants=32, F=2304,
               models=[(K, D) for K in (2, 7) for D in (2048, 4096, 10240)],
               desc="serving: Poisson arrivals, requests of U{1..512} queries, 32 tenants with device-resident "
                    "encrypted models (16 at BFV N=8192 / 4 limbs cycling K in {2, 7} x D in {2048, 4096, 10240}; "
                    "16 at N=16384 / 8+2 limbs, dnum=4, r=4 cycling the same (K, D)), HBM-budget admission, "
                    "continuous batching on 2 streams"),
    # detection from raw frames: 1080p frames, 64 x 64 windows at a stride of 8 pixels, HOG
    # features -> HDC encoding -> encrypted scoring at the paper's optimised ring (N = 2048)
    "detect": dict(detect=True, H=1080, W=1920, window=64, stride=8, N=2048, L=2, D=1024, K=2,
                   desc="1080x1920 synthetic frames, 64x64 windows at stride 8 (29824 windows, HOG F=1776), "
                        "HDC D=1024, K=2, BFV N=2048, 2x30-bit limbs, t=65537: frame -> HOG -> encode -> "
                        "score per step"),
    # findDmax sweep (design space exploration): N = 2048, two 24-bit limbs (Q about 2^48),
    # binary queries and 8-bit classes, K = 2 (the paper's Face task), per scheme and t
    "dmax": dict(dmax=True, N=2048, L=2, prime_bits=24, K=2, qbits=1, cbits=8, d_cap=4096, trials=8,
                 sweep={"bfv": [12289, 40961, 65537, 114689, 147457, 270337],
                        "bfv-r": [114689, 270337, 786433, 1179649, 1597441],
                        "bgv": [114689, 270337, 786433, 1179649, 1597441]},
                 desc="findDmax trials at N=2048, 2 x 24-bit primes, K=2, binary queries, 8-bit classes, "
                      "d_cap=4096: BFV, rounded BFV and BGV over t"),
    # large parameters: 8 ciphertext limbs + 2 special primes, hybrid key switching with 4
    # digits, 8 blocks folded per row (3 rotations per score ciphertext)
    "c4": dict(N=16384, L=8, alpha=2, dnum=4, r=8, F=2304, D=10240, K=26, Q=16384, images=True, cpu_sample_m=24,
               desc="BFV N=16384, 8x30-bit limbs + 2 special primes, dnum=4, t=65537; r=8 blocks per "
                    "row folded by 3 rotate-and-sum steps; HDC F=2304 (48x48 Gaussian-blob images), "
                    "D=10240, K=26; 16384 queries per request"),
}

# Peak of the integer VALU for 30-bit modular multiplication on MI355X: 256 CUs x 64 lanes
# x 2.4 GHz = 39.3 T 32-bit multiplies/s; a Shoup modular multiplication needs 3 of them.
MUL32_PEAK = 256 * 64 * 2.4e9
MODMUL_PEAK = MUL32_PEAK / 3
INT8_PEAK = 5.0e15  # dense int8 MFMA operations/s of MI355X
HBM_PEAK = 8.0e12  # HBM3E bytes/s of MI355X


def transform_mults(N: int) -> int:
    """Modular multiplications of one length-N negacyclic transform: (N/2) log2 N butterflies."""
    return (N // 2) * int(math.log2(N))


def algorithmic_modmuls(kernel: str, N: int, L: int, G: int, M: int) -> float:
    """Algorithmic modular multiplications of one launch over G groups x M plaintexts:
    batch encoding is one inverse transform mod t per plaintext; the MAC is L forward
    transforms plus 2L*N ct x pt products per plaintext (recomputed work not counted)."""
    enc = transform_mults(N)
    mac = L * transform_mults(N) + 2 * L * N
    per_pt = {"k_encode_pt": enc, "k_mac": mac, "k_score": enc + mac}[kernel]
    return float(G) * M * per_pt


# The sources that define each profiled kernel's code (its HIP file and the headers it uses).
KERNEL_SOURCES = {k: ("kernels_ntt.hip", "device_ntt.hpp", "kernel_common.hpp", "launch.hpp")
                  for k in ("k_mac", "k_encode_pt", "k_score", "k_finish", "k_mac_list", "k_encode_list")}
KERNEL_SOURCES["batch_unpacked"] = ("kernels_ntt.hip", "device_ntt.hpp", "kernel_common.hpp", "launch.hpp",
                                    "kernels_hdc.hip", "batch.hip")
KERNEL_SOURCES["k_hdc_encode"] = ("kernels_hdc.hip", "launch.hpp")
KERNEL_SOURCES["k_mac_sub"] = KERNEL_SOURCES["k_encode_sub"] = KERNEL_SOURCES["k_mac"]


def kernel_source_digest(kernel: str = "k_mac") -> str:
    """SHA-256 over the sources of `kernel`; a traffic figure is valid only for the code it was taken on."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2511_00737_amd", "csrc")
    for name in sorted(KERNEL_SOURCES[kernel]):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` recorded in profiles/<kernel>_<workload>_traffic.md by
    two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) scaled by a plain-copy calibration, or
    None when the file is missing or was taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    if fields.get("source_digest") != kernel_source_digest(kernel):
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _oracle_mac_worker(kw, D, C, m0, sample_m, seed, barrier, out):
    """One process of the all-cores oracle leg: the oracle's MAC of query group 0 over model
    ciphertexts m0 .. m0 + sample_m - 1 (encrypted here, untimed), timed after a barrier so
    that every process runs its MAC at the same time."""
    from oracle import bfv
    from oracle.params import Params as OParams
    o = OParams(D=D, **kw)
    s = bfv.secret_key(o, seed)
    model = bfv.encrypt_model(o, s, C, seed, ms=range(m0, m0 + sample_m))
    osub = OParams(D=sample_m * o.r, **kw)
    h = np.zeros((o.B, sample_m * o.r), dtype=np.int8)
    h[:16] = 1
    barrier.wait()
    t0 = time.time()
    bfv.mac(osub, model, h, 0)
    out.put((t0, time.time()))


def recorded_valu_issue(kernel: str, workload: str):
    """Fraction of SIMD cycles issuing a VALU instruction (SQ_INSTS_VALU * 4 / (SIMDs * cycles))
    recorded for `kernel` in profiles/sq_counters_<workload>.md, or None when missing or taken
    on different kernel sources."""
    path = os.path.join(ROOT, "profiles", f"sq_counters_{workload}.md")
    if not os.path.exists(path):
        return None
    digest, val = None, None
    for line in open(path):
        if line.startswith("- source_digest:"):
            digest = line.split(":", 1)[1].strip().strip("`")
        if line.startswith(f"- valu_issue_{kernel}:"):
            try:
                val = float(line.split(":", 1)[1].strip().strip("`"))
            except ValueError:
                val = None
    return val if digest == kernel_source_digest(kernel) else None


def cpu_baseline_all_cores(prm: ep.Params, C: np.ndarray, sample_m: int, t_hdc: float, t_rot: float):
    """The oracle on every host core: one process per core (spawned, single-threaded numpy),
    each timing the MAC of a different slice of sample_m model ciphertexts at the same time;
    the slices' plaintexts per second give inferences/s as in the single-core leg."""
    import multiprocessing as mp
    from oracle.params import Params as OParams
    kw = dict(N=prm.N, q=tuple(prm.q), p=tuple(prm.p), F=prm.F, K=prm.K, r=prm.r, dnum=prm.dnum,
              layout=prm.layout)
    o = OParams(D=prm.D, **kw)
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    nproc = max(1, min(cores, 16, o.M // sample_m))
    ctx = mp.get_context("spawn")
    barrier, out = ctx.Barrier(nproc), ctx.Queue()
    env_keep = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in env_keep:
        os.environ[k] = "1"
    procs = [ctx.Process(target=_oracle_mac_worker, args=(kw, prm.D, C, i * sample_m, sample_m, 0, barrier, out))
             for i in range(nproc)]
    try:
        for p in procs:
            p.start()
        spans = [out.get(timeout=600) for _ in procs]
        for p in procs:
            p.join()
    finally:
        for k, v in env_keep.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    wall = max(e for _, e in spans) - min(s_ for s_, _ in spans)
    pt_per_s = nproc * sample_m / wall
    t_group = o.M / pt_per_s + (t_rot + t_hdc * o.B) / nproc
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": o.B / t_group, "unit": "inferences/s", "cores": nproc, "kind": "oracle",
            "sample": f"{nproc} processes at once, each the oracle's ct x pt MAC of query group 0 over its own "
                      f"{sample_m} of the {o.M} model ciphertexts (plaintexts per second over the slowest "
                      f"process's span, scaled to the full model, HDC encoding and rotations added per core); "
                      f"host: {cores} usable cores of {os.cpu_count()}, {cpu}",
            "seconds": round(wall, 2)}


def cpu_baseline(w: dict, prm: ep.Params, x: np.ndarray, base: np.ndarray, C: np.ndarray, sample_m: int):
    """The oracle, timed on the host: HDC encoding of a few queries, the MAC of query group 0
    over the first `sample_m` model ciphertexts (scaled to the whole model) and, for folded
    packings, the rotate-and-sum of that group, turned into inferences/s."""
    from oracle import bfv, hdc
    from oracle.params import Params as OParams
    kw = dict(N=prm.N, q=tuple(prm.q), p=tuple(prm.p), F=prm.F, K=prm.K, r=prm.r, dnum=prm.dnum,
              layout=prm.layout)
    o = OParams(D=prm.D, **kw)
    s = bfv.secret_key(o, 0)
    sample_m = min(sample_m, o.M)
    osub = OParams(D=sample_m * o.r, **kw)
    model = bfv.encrypt_model(osub, s, C[:, :sample_m * o.r], 0)
    nq = 16
    t0 = time.perf_counter()
    h16 = hdc.encode(x[:nq], base)
    t_hdc = (time.perf_counter() - t0) / nq
    h = np.zeros((o.B, sample_m * o.r), dtype=np.int8)
    h[:nq] = h16[:, :sample_m * o.r]
    t0 = time.perf_counter()
    acc = bfv.mac(osub, model, h, 0)
    t_mac = time.perf_counter() - t0
    t_rot = 0.0
    if o.r > 1:
        gk = bfv.galois_keys(o, s, 0)
        t0 = time.perf_counter()
        bfv.rotate_and_sum(o, acc, gk)
        t_rot = time.perf_counter() - t0
    t_group = t_mac * o.M / sample_m + t_rot + t_hdc * o.B
    rot = f" and its rotate-and-sum ({o.log2r} rotations)" if o.r > 1 else ""
    one = {"value": o.B / t_group, "unit": "inferences/s", "cores": 1, "kind": "oracle",
           "sample": f"HDC encoding of {nq} queries, the ct x pt MAC of query group 0 "
                     f"({o.B} queries) over model ciphertexts 0..{sample_m - 1} of {o.M} "
                     f"scaled linearly to the full model{rot}; numpy, single thread "
                     f"(host has {os.cpu_count()} cores)",
           "seconds": round(t_mac + t_rot + t_hdc * nq, 2)}
    try:
        one["all_cores"] = cpu_baseline_all_cores(prm, C, sample_m, t_hdc, t_rot)
    except Exception as exc:  # the single-core figure stands on its own
        one["all_cores"] = {"error": repr(exc)}
    return one


def bench_batched(args, w) -> int:
    res = run_batched(args, w, "subring" if args.layout in ("auto", "subring") else "contiguous")
    if res is None:
        return 3
    print(json.dumps(res), flush=True)
    return 0


def profile_unpacked(args, w) -> int:
    """For counter runs: the batching workload's unpacked batch alone, enqueued launch by launch
    (no graph, no autotuner: the default schedule, which the autotuner keeps at this size),
    `--steps` runs after `--warmup`; prints ms per run.  Contiguous layout unless
    `--layout subring`."""
    import torch
    N, L, F, nreq = w["N"], w["L"], w["F"], w["requests"]
    layout = "subring" if args.layout == "subring" else "contiguous"
    primes = ep.default_primes(N, L)
    sizes, midx = synth.batch_mix(args.seed, nreq, len(w["models"]))
    dev = torch.device("cuda")
    d_pool = torch.from_numpy(synth.blob_images(args.seed, 4096)).to(dev)
    sessions, bases = [], []
    for k, (K, D) in enumerate(w["models"]):
        prm = ep.Params(N=N, q=tuple(primes), F=F, D=D, K=K, layout=layout)
        sk, _ = ep.ephdc_keygen(prm, args.seed + k)
        model = ep.ephdc_encrypt_model(prm, sk, synth.class_hypervectors(args.seed + k, K, D), args.seed + k)
        sessions.append(ep.Session(prm, torch.from_numpy(model.view(np.int32)).to(dev), max_Q=4096, workspace=None))
        bases.append(torch.from_numpy(synth.base_hypervectors(args.seed, F, D)).to(dev))
    reqs = []
    for i in range(nreq):
        s, Q = sessions[int(midx[i])], int(sizes[i])
        off = (i * 977) % (4096 - Q + 1)
        d_hv = torch.empty((s.prm.D, s.hv_stride(Q)), dtype=torch.int8, device=dev)
        d_out = torch.empty((s.num_groups(Q), 2, L, N), dtype=torch.int32, device=dev)
        reqs.append(ep.Request(s, d_hv, Q, d_out, d_x=d_pool[off:off + Q], d_base=bases[int(midx[i])]))
    batch = ep.Batch(reqs)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        batch.run(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch.run(stream)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / max(1, args.steps)
    print(json.dumps({"form": "unpacked batch, eager", "layout": layout, "runs": args.steps, "warmup": args.warmup,
                      "ms_per_run": round(ms, 4), "schedule": batch.schedule()}), flush=True)
    batch.close()
    for s in sessions:
        s.close()
    return 0


def request_modmuls(prm, G: int) -> float:
    """Algorithmic modular multiplications of scoring G groups of one request: the plaintexts'
    batch encoding, their transforms into every limb and the 2L*N ct x pt products each --
    N-point transforms in the contiguous layout, N/K'-point ones in the subring layout."""
    N, L, M = prm.N, prm.L, ep.ephdc_num_model_ct(prm)
    if prm.layout == "subring":
        n = N // (1 << (prm.K - 1).bit_length())
        return float(G) * M * ((1 + L) * transform_mults(n) + 2 * L * N)
    return algorithmic_modmuls("k_score", N, L, G, M)


def run_batched(args, w, layout: str = "contiguous"):
    """The batching workload: all requests scored by one graph-captured batch (persistent
    launches over a shared work list, schedule from the autotuner) against the plain form,
    the same requests one after another through the single-request entry points, in one slot
    layout.  Returns the result dict (None when a check fails)."""
    import torch
    N, L, F, nreq = w["N"], w["L"], w["F"], w["requests"]
    primes = ep.default_primes(N, L)
    seed = args.seed
    sizes, midx = synth.batch_mix(seed, nreq, len(w["models"]))
    t0 = time.perf_counter()
    pool = synth.blob_images(seed, 4096)
    dev = torch.device("cuda")
    d_pool = torch.from_numpy(pool).to(dev)
    tenants = []
    for k, (K, D) in enumerate(w["models"]):
        prm = ep.Params(N=N, q=tuple(primes), F=F, D=D, K=K, layout=layout)
        sk, _ = ep.ephdc_keygen(prm, seed + k)
        C = synth.class_hypervectors(seed + k, K, D)
        model = ep.ephdc_encrypt_model(prm, sk, C, seed + k)
        d_model = torch.from_numpy(model.view(np.int32)).to(dev)
        sess = ep.Session(prm, d_model, max_Q=4096)
        del d_model, model
        base = synth.base_hypervectors(seed, F, D)
        tenants.append(dict(prm=prm, sk=sk, C=C, sess=sess, d_base=torch.from_numpy(base).to(dev)))
    reqs = []
    for i in range(nreq):
        t = tenants[int(midx[i])]
        Q = int(sizes[i])
        s = t["sess"]
        off = (i * 977) % (4096 - Q + 1)
        d_hv = torch.empty((t["prm"].D, s.hv_stride(Q)), dtype=torch.int8, device=dev)
        d_out = torch.empty((s.num_groups(Q), 2, L, N), dtype=torch.int32, device=dev)
        reqs.append(ep.Request(s, d_hv, Q, d_out, d_x=d_pool[off:off + Q], d_base=t["d_base"]))
    torch.cuda.synchronize()
    print(f"[bench] c3: {nreq} requests, {int(sizes.sum())} queries, setup {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)

    # plain form: the requests one after another, one encode + one score call each
    stream = torch.cuda.Stream()

    def plain_step():
        for r in reqs:
            ep.ephdc_encode_queries(r.session, r.d_x, r.d_base, r.Q, r.d_hv, stream=stream)
            ep.ephdc_score_encrypted(r.session, r.d_hv, r.Q, r.d_score_ct, stream=stream)

    def timed(fn, steps):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            ev[k][0].record(stream)
            fn()
            ev[k][1].record(stream)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, np.array([a.elapsed_time(b) for a, b in ev])

    with torch.cuda.stream(stream):
        for _ in range(max(1, args.warmup)):
            plain_step()
        plain_wall, plain_lat = timed(plain_step, max(1, args.steps // 4))
        plain_out = [r.d_score_ct.clone() for r in reqs]

        batch = ep.Batch(reqs)
        t0 = time.perf_counter()
        sched, tuned_ms = batch.autotune(reps=2, stream=stream)
        t_tune = time.perf_counter() - t0
        print(f"[bench] c3: autotuned {sched} ({tuned_ms:.2f} ms/run) in {t_tune:.1f}s", file=sys.stderr, flush=True)
        batch.capture(stream)
        for _ in range(args.warmup):
            batch.run(stream)
        unpacked_wall, unpacked_lat = timed(lambda: batch.run(stream), max(1, args.steps // 2))
        # the same requests packed: one query sequence per model, shared ciphertexts
        outs_p = [torch.empty((r.d_score_ct.shape[0] + 1,) + tuple(r.d_score_ct.shape[1:]), dtype=torch.int32,
                              device=dev) for r in reqs]
        preqs = [ep.Request(r.session, None, r.Q, o, d_x=r.d_x, d_base=r.d_base) for r, o in zip(reqs, outs_p)]
        pbatch = ep.Batch(preqs, packed=True)
        t0 = time.perf_counter()
        psched, ptuned_ms = pbatch.autotune(reps=2, stream=stream)
        t_ptune = time.perf_counter() - t0
        print(f"[bench] c3 packed: autotuned {psched} ({ptuned_ms:.2f} ms/run) in {t_ptune:.1f}s",
              file=sys.stderr, flush=True)
        for _ in range(args.warmup):
            pbatch.run(stream)
        eager_wall, eager_lat = timed(lambda: pbatch.run(stream), max(1, args.steps // 2))
        pbatch.capture(stream)
        for _ in range(args.warmup):
            pbatch.run(stream)
        wall, lat = timed(lambda: pbatch.run(stream), args.steps)
    # the unpacked batch reproduces the plain form bit for bit; the packed one gives every
    # request its exact scores
    for r, p in zip(reqs, plain_out):
        if not torch.equal(r.d_score_ct, p):
            print("[bench] batched ciphertexts differ from the plain form", file=sys.stderr)
            return None
    for i in range(0, nreq, 16):
        r, t = reqs[i], tenants[int(midx[i])]
        hv = r.d_hv.cpu().numpy()[:, :r.Q].T.astype(np.float64)
        want = (hv @ t["C"].astype(np.float64).T).astype(np.int64) % 65537
        want = np.where(want > 32768, want - 65537, want)
        scores, _ = ep.ephdc_decrypt_scores(t["prm"], t["sk"], r.d_score_ct.cpu().numpy().view(np.uint32), r.Q)
        off, qf, nct = pbatch.packing(i)
        pscores, _ = ep.ephdc_decrypt_scores_at(t["prm"], t["sk"], outs_p[i][:nct].cpu().numpy().view(np.uint32),
                                                qf, r.Q)
        if not (np.array_equal(scores, want) and np.array_equal(pscores, want)):
            print("[bench] decrypted scores differ from h.C mod t", file=sys.stderr)
            return None
    total_q = int(sizes.sum())
    # algorithmic work of a step: plain and unpacked forms score every request in its own
    # ciphertexts (G_i = ceil(Q_i / B) groups each), the packed form one query sequence per model
    work_unpacked = 0.0
    for i in range(nreq):
        t = tenants[int(midx[i])]
        work_unpacked += request_modmuls(t["prm"], ep.ephdc_num_groups(t["prm"], int(sizes[i])))
    work_packed = 0.0
    for k, t in enumerate(tenants):
        Qk = int(sizes[midx == k].sum())
        if Qk:
            work_packed += request_modmuls(t["prm"], ep.ephdc_num_groups(t["prm"], Qk))

    def form(wall_s, lat_ms, work, desc, **extra):
        ms = wall_s * 1e3 / len(lat_ms)
        ach = work / (ms * 1e-3)
        return {"value": round(total_q / (ms * 1e-3), 1), "unit": "inferences/s", "ms_per_step": round(ms, 4),
                "latency_ms": {"p50": round(float(np.percentile(lat_ms, 50)), 4),
                               "p99": round(float(np.percentile(lat_ms, 99)), 4)},
                "roofline": {"bound": "alu", "kernel": "whole path of a step (batch encoding and MAC dominate)",
                             "achieved": round(ach / 1e12, 4), "peak": round(MODMUL_PEAK / 1e12, 4),
                             "unit": "Tmodmul/s", "frac": round(ach / MODMUL_PEAK, 4),
                             "per_step_modmuls": work},
                "form": desc, **extra}

    plain = form(plain_wall, plain_lat, work_unpacked,
                 "the requests one after another: an encode and a score call per request, no graph")
    unpacked = form(unpacked_wall, unpacked_lat, work_unpacked,
                    "one graph replay of persistent launches, every request in its own ciphertexts",
                    schedule=sched, autotune_s=round(t_tune, 1))
    packed = form(wall, lat, work_packed,
                  "one graph replay, the requests of each model sharing ciphertexts (one query sequence per model)",
                  schedule=psched, autotune_s=round(t_ptune, 1))
    packed_eager = form(eager_wall, eager_lat, work_packed, "the packed batch enqueued launch by launch, no graph")
    # HBM bytes of one unpacked run, recorded by counter runs of --profile-unpacked
    run_traffic = recorded_traffic("batch_unpacked", "c3" if layout == "contiguous" else "c3_subring")
    unpacked["roofline"]["traffic"] = run_traffic
    if run_traffic is not None:
        gbps = run_traffic / (unpacked["ms_per_step"] * 1e-3)
        unpacked["roofline"]["hbm_gbps"] = round(gbps / 1e9, 1)
        unpacked["roofline"]["hbm_frac"] = round(gbps / HBM_PEAK, 4)
    result = {
        "metric": METRIC, "value": packed["value"], "unit": "inferences/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": packed["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"c3: {w['desc']}", "requests": nreq, "queries_per_step": total_q,
                   "layout": layout},
        "latency_ms": packed["latency_ms"], "roofline": packed["roofline"],
        "plain": plain, "batched_unpacked": unpacked, "packed": packed, "packed_eager": packed_eager,
        "speedup_unpacked_vs_plain": round(unpacked["value"] / plain["value"], 3),
        "speedup_packed_vs_plain": round(packed["value"] / plain["value"], 3),
    }
    batch.close()
    pbatch.close()
    for t in tenants:
        t["sess"].close()
    return result


def bench_serving(args, w) -> int:
    """The serving workload: a Poisson trace replayed against the native serving loop.
    Requests are submitted at their arrival times (device-resident features); the report
    gives completed inferences/s over the run, submit-to-done latency p50/p99 and the time
    requests waited for admission, at the trace's rate and, with --rates, at lower ones."""
    import torch
    dev = torch.device("cuda")
    F, seed = w["F"], args.seed
    t0 = time.perf_counter()
    pool = torch.from_numpy(synth.blob_images(seed, w["qmax"])).to(dev)
    bases = {}
    tenants = []
    for k in range(w["tenants"]):
        K, D = w["models"][k % len(w["models"])]
        if k < w["tenants"] // 2:
            N, L, alpha, r, dnum = 8192, 4, 0, 1, 0
        else:
            N, L, alpha, r, dnum = 16384, 8, 2, 4, 4
        # every tenant in the subring layout (auto), the folded N = 16384 ones included
        layout = "subring" if args.layout in ("auto", "subring") else "contiguous"
        primes = ep.default_primes(N, L + alpha)
        prm = ep.Params(N=N, q=tuple(primes[:L]), p=tuple(primes[L:]), F=F, D=D, K=K, r=r, dnum=dnum,
                        layout=layout)
        sk, gk = ep.ephdc_keygen(prm, seed + 100 + k)
        C = synth.class_hypervectors(seed + 100 + k, K, D)
        model = ep.ephdc_encrypt_model(prm, sk, C, seed + 100 + k)
        d_model = torch.from_numpy(model.view(np.int32)).to(dev)
        d_gk = torch.from_numpy(gk.view(np.int32)).to(dev) if gk is not None else None
        sess = ep.Session(prm, d_model, d_gk, max_Q=w["qmax"], workspace=None)  # served only: no workspace
        del d_model, d_gk, model
        if D not in bases:
            bases[D] = torch.from_numpy(synth.base_hypervectors(seed, F, D)).to(dev)
        tenants.append(dict(prm=prm, sk=sk, C=C, sess=sess, base=bases[D]))
    torch.cuda.synchronize()
    model_bytes = sum(t["sess"].device_bytes for t in tenants)
    print(f"[bench] c5: {len(tenants)} tenants, {model_bytes / 2**30:.1f} GiB of sessions, "
          f"setup {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)

    def run(rate, duration, budget, pack=True):
        trace = synth.poisson_trace(seed, rate, duration, 1, w["qmax"], len(tenants))
        sv = ep.Server(budget, streams=2, max_batch=64)
        if pack:
            sv.set_packing(True)
        ids = [sv.add_tenant(t["sess"], t["base"]) for t in tenants]
        live, check, waits = {}, [], []
        torch.cuda.synchronize()
        start = time.perf_counter()
        for i, (ta, ti, Q) in enumerate(trace):
            delay = start + ta - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            t = tenants[ti]
            out = torch.empty((t["sess"].num_groups(Q) + (1 if pack else 0), 2, t["prm"].L, t["prm"].N),
                              dtype=torch.int32, device=dev)
            tk = sv.submit(ids[ti], pool[:Q], Q, out)
            live[tk] = (out, Q, ti)
            if i % 200 == 0:  # release finished requests now and then; keep a few to check
                for k in list(live):
                    st, (ts, tad, td) = sv.query(k)
                    if st != 2:
                        continue
                    waits.append(tad - ts)
                    item = live.pop(k)
                    if len(check) < 4 and k % 7 == 0:
                        # keep where its queries are, not the ticket: the server forgets the
                        # oldest unreleased tickets beyond its bound
                        check.append((sv.result(k), item))
                    sv.release(k)
        t_submitted = time.perf_counter() - start
        sv.wait(0, timeout_s=600)
        wall = time.perf_counter() - start
        stats = sv.stats()
        recent = list(live)[-4:]
        last = [(sv.result(k), live[k]) for k in recent]
        for tk in live:
            try:
                st, (ts, tad, td) = sv.query(tk)
            except ep.EphdcError:  # forgotten: beyond the server's bound of unreleased tickets
                continue
            if st == 2:
                waits.append(tad - ts)
        for (qf, nct), (out_k, q_k, ti_k) in check + last:
            t = tenants[ti_k]
            scores, _ = ep.ephdc_decrypt_scores_at(t["prm"], t["sk"], out_k[:nct].cpu().numpy().view(np.uint32), qf, q_k)
            hv = torch.empty((t["prm"].D, t["sess"].hv_stride(q_k)), dtype=torch.int8, device=dev)
            ep.ephdc_encode_queries(t["sess"], pool[:q_k], t["base"], q_k, hv)
            torch.cuda.synchronize()
            h = hv.cpu().numpy()[:, :q_k].T.astype(np.float64)
            want = (h @ t["C"].astype(np.float64).T).astype(np.int64) % 65537
            if not np.array_equal(scores, np.where(want > 32768, want - 65537, want)):
                raise RuntimeError("served scores differ from h.C mod t")
        sv.close()
        total_q = sum(q for _, _, q in trace)
        return {"rate_req_s": rate, "requests": len(trace), "queries": total_q,
                "offered_inferences_s": round(total_q / duration, 1),
                "value": round(total_q / wall, 1), "wall_s": round(wall, 3), "submit_s": round(t_submitted, 3),
                "p50_ms": round(stats["p50_ms"], 3), "p99_ms": round(stats["p99_ms"], 3),
                "admission_wait_ms_mean": round(1e3 * float(np.mean(waits)), 3) if waits else 0.0,
                "admission_wait_ms_p99": round(1e3 * float(np.percentile(waits, 99)), 3) if waits else 0.0,
                "rejected": int(stats["rejected"]), "batches": int(stats["batches"]),
                "mean_requests_per_batch": round(stats["mean_batch"], 2),
                "peak_request_bytes": int(stats["peak_bytes"]), "budget_bytes": int(stats["budget_bytes"]),
                "stable": wall <= duration * 1.2, "packing": pack}

    budget = 32 << 30
    main_run = run(w["rate"], args.duration or w["duration"], budget)
    print(f"[bench] c5 at {w['rate']} req/s: {main_run}", file=sys.stderr, flush=True)
    sweep = []
    for rate in [float(x) for x in args.rates.split(",") if x]:
        sweep.append(run(rate, args.duration or w["duration"], budget))
        print(f"[bench] c5 at {rate} req/s: {sweep[-1]}", file=sys.stderr, flush=True)
    unpacked = run(w["rate"], args.duration or w["duration"], budget, pack=False)
    print(f"[bench] c5 unpacked at {w['rate']} req/s: {unpacked}", file=sys.stderr, flush=True)
    result = {
        "metric": METRIC, "value": main_run["value"], "unit": "inferences/s", "n_gpus": 1,
        "steps": main_run["requests"], "warmup": 0, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"c5: {w['desc']}", "rate_req_s": w["rate"], "tenants": len(tenants),
                   "session_bytes": int(model_bytes),
                   "layouts": sorted({t["prm"].layout for t in tenants})},
        "latency_ms": {"p50": main_run["p50_ms"], "p99": main_run["p99_ms"]},
        "serving": main_run, "rate_sweep": sweep, "unpacked_at_same_rate": unpacked,
    }
    for t in tenants:
        t["sess"].close()
    print(json.dumps(result), flush=True)
    return 0


def bench_detect(args, w) -> int:
    """Object detection from raw frames on the client: per step one frame's sliding windows
    get their HOG feature maps, are HDC-encoded and scored against the encrypted model.
    inferences/s = windows per second; the HOG stage's HBM roofline is reported beside the
    scoring kernels'."""
    import torch
    from_frames = [synth.frame(args.seed + k, w["H"], w["W"]) for k in range(2)]
    H, W, win, st = w["H"], w["W"], w["window"], w["stride"]
    Q = ep.ephdc_hog_window_count(H, W, win, st)
    F = ep.ephdc_hog_feature_count(win)
    N, L, D, K = w["N"], w["L"], w["D"], w["K"]
    layout = "subring" if args.layout in ("auto", "subring") else "contiguous"
    prm = ep.Params(N=N, q=tuple(ep.default_primes(N, L)), F=F, D=D, K=K, layout=layout)
    base = synth.base_hypervectors(args.seed, F, D)
    C = synth.class_hypervectors(args.seed, K, D)
    sk, _ = ep.ephdc_keygen(prm, args.seed)
    model = ep.ephdc_encrypt_model(prm, sk, C, args.seed)
    dev = torch.device("cuda")
    sess = ep.Session(prm, torch.from_numpy(model.view(np.int32)).to(dev), max_Q=Q)
    d_frames = [torch.from_numpy(f).to(dev) for f in from_frames]
    d_base = torch.from_numpy(base).to(dev)
    d_ws = torch.empty(ep.ephdc_hog_workspace_bytes(H, W), dtype=torch.uint8, device=dev)
    d_x = torch.empty((Q, F), dtype=torch.uint8, device=dev)
    d_hv = torch.empty((D, sess.hv_stride(Q)), dtype=torch.int8, device=dev)
    G = sess.num_groups(Q)
    d_out = torch.empty((G, 2, L, N), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    hog_ev = []

    def step(k, timed=False):
        if timed:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
        ep.ephdc_hog_windows(d_frames[k % 2], win, st, d_x, d_workspace=d_ws)
        if timed:
            e1.record(stream)
            hog_ev.append((e0, e1))
        ep.ephdc_encode_queries(sess, d_x, d_base, Q, d_hv)
        ep.ephdc_score_encrypted(sess, d_hv, Q, d_out)

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    # throughput: the frames back to back between two synchronisations; then the same
    # frames with an event pair each for the latency percentiles, and again with the
    # session's kernel timers (and the HOG stage's events) for the per-stage times
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for k in range(args.steps):
        ev[k][0].record(stream)
        step(k)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    sess.profile(True)
    for k in range(args.steps):
        step(k, timed=True)
    torch.cuda.synchronize()
    prof = sess.profile_read()
    sess.profile(False)
    # check this launch configuration (after the timed passes, which follow the warm-up
    # directly): decrypted scores of every window of the last frame equal h . C mod t
    hv = d_hv.cpu().numpy()[:, :Q].T.astype(np.float64)
    scores, _ = ep.ephdc_decrypt_scores(prm, sk, d_out.cpu().numpy().view(np.uint32), Q)
    want = (hv @ C.astype(np.float64).T).astype(np.int64) % 65537
    if not np.array_equal(scores, np.where(want > 32768, want - 65537, want)):
        print("[bench] decrypted scores differ from h.C mod t", file=sys.stderr)
        return 3
    hog_ms = float(np.mean([a.elapsed_time(b) for a, b in hog_ev]))
    hog_bytes = H * W + Q * F  # frame read once, feature rows written once (histograms and blocks are small)
    M = ep.ephdc_num_model_ct(prm)
    mac_ms = prof["mac"][0] / max(1, prof["mac"][1])
    mac_ops = algorithmic_modmuls("k_mac", N, L, G, M) * args.steps / max(1, prof["mac"][1])
    n_sub = N // (1 << (K - 1).bit_length())
    if layout == "subring":
        # streaming MAC: the model once per launch's group tiles, the transformed plaintexts once
        tiles = -(-G // (8 if G > 4 else 4))
        mac_bytes = (tiles * M * 2 * L * N + G * M * L * n_sub + G * 2 * L * N) * 4.0 * args.steps / max(1, prof["mac"][1])
        mac_roof = {"bound": "hbm", "kernel": "k_mac_sub", "achieved": round(mac_bytes / (mac_ms * 1e-3) / 1e9, 1),
                    "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": round(mac_bytes / (mac_ms * 1e-3) / HBM_PEAK, 4),
                    "traffic": None, "algorithmic_bytes": mac_bytes, "avg_launch_ms": round(mac_ms, 4)}
    else:
        mac_roof = {"bound": "alu", "kernel": "k_mac", "achieved": round(mac_ops / (mac_ms * 1e-3) / 1e12, 4),
                    "peak": round(MODMUL_PEAK / 1e12, 4), "unit": "Tmodmul/s",
                    "frac": round(mac_ops / (mac_ms * 1e-3) / MODMUL_PEAK, 4), "traffic": None,
                    "avg_launch_ms": round(mac_ms, 4)}
    result = {
        "metric": "windows/s from raw frames (HOG + HDC encoding + encrypted scoring)",
        "value": round(Q * args.steps / wall, 1), "unit": "inferences/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(wall * 1e3 / args.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"detect: {w['desc']}", "windows_per_frame": Q, "features": F, "groups": G,
                   "layout": layout, "queries_per_ciphertext": ep.ephdc_queries_per_ct(prm)},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4), "p99": round(float(np.percentile(lat, 99)), 4)},
        "stages_ms_per_step": {"hog": round(hog_ms, 4),
                               **{k: round(v[0] / args.steps, 4) for k, v in prof.items() if v[1]}},
        "roofline": mac_roof,
        "roofline_hog": {"bound": "hbm", "kernel": "HOG cells + blocks + windows", "achieved":
                         round(hog_bytes / (hog_ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                         "frac": round(hog_bytes / (hog_ms * 1e-3) / HBM_PEAK, 4), "traffic": None,
                         "algorithmic_bytes": hog_bytes, "avg_ms": round(hog_ms, 4)},
        "paper": "7117.04 windows/s on one Ryzen 3970X core (Face, N=2^11, batch 1024, HOG and HDC encoding "
                 "included); other hardware and parameters",
    }
    sess.close()
    if not args.no_cpu_baseline:
        from oracle import hog as ohog, hdc as ohdc
        t0 = time.perf_counter()
        xo = ohog.window_features(from_frames[0], win, st)
        t_hog = time.perf_counter() - t0
        t0 = time.perf_counter()
        ohdc.encode(xo[:64], base)
        t_enc = (time.perf_counter() - t0) / 64
        cb = cpu_baseline(WORKLOADS["c2"], prm, xo[:16], base, C, 64)
        B = ep.ephdc_queries_per_ct(prm)
        t_group = B / cb["value"]  # oracle seconds per group of B windows, HDC encoding included
        per_win = t_hog / Q + t_group / B
        result["cpu_baseline"] = {"value": round(1.0 / per_win, 2), "unit": "inferences/s", "cores": 1,
                                  "kind": "oracle",
                                  "sample": f"oracle HOG of one whole frame ({t_hog:.2f}s for {Q} windows), and the "
                                            f"oracle's HDC encoding + MAC of one group over 64 of {M} model "
                                            f"ciphertexts scaled to the model; single thread",
                                  "seconds": round(t_hog + cb["seconds"], 2), "hdc_encode_s_per_window": t_enc}
    print(json.dumps(result), flush=True)
    return 0


def _primes_below(bound: int, N: int, count: int) -> list[int]:
    """The `count` largest primes below `bound` that are 1 mod 2N (trial division: the
    bounds used here are small)."""
    def is_prime(n):
        if n < 2 or n % 2 == 0:
            return n == 2
        f = 3
        while f * f <= n:
            if n % f == 0:
                return False
            f += 2
        return True
    out, k = [], (bound - 2) // (2 * N)
    while len(out) < count:
        if is_prime(k * 2 * N + 1):
            out.append(k * 2 * N + 1)
        k -= 1
    return out


def bench_dmax(args, w) -> int:
    """findDmax on the device over schemes and plaintext moduli: mean and spread of D_max per
    (scheme, t), the device's seconds per trial, and the oracle's seconds per trial on the
    host for the first setting (a bounded number of its prefixes)."""
    N, L, K = w["N"], w["L"], w["K"]
    q = tuple(_primes_below(1 << w["prime_bits"], N, L))
    rows = []
    t_all = time.perf_counter()
    trials = args.steps if args.steps != 20 else w["trials"]
    for scheme, ts in w["sweep"].items():
        for t in ts:
            prm = ep.Params(N=N, q=q, t=t, D=w["d_cap"], K=K, F=16, scheme=scheme, qbits=w["qbits"])
            t0 = time.perf_counter()
            d = ep.ephdc_find_dmax(prm, args.seed, trials, w["d_cap"], w["cbits"])
            dt = time.perf_counter() - t0
            rows.append({"scheme": scheme, "t": t, "log2_t": round(math.log2(t), 2), "mean": float(np.mean(d)),
                         "std": round(float(np.std(d)), 2), "min": int(d.min()), "max": int(d.max()),
                         "capped": int((d >= w["d_cap"]).sum()), "s_per_trial": round(dt / trials, 4)})
            print(f"[bench] dmax {scheme} t={t}: mean {rows[-1]['mean']:.1f} (min {d.min()}, max {d.max()}), "
                  f"{dt / trials:.3f} s/trial", file=sys.stderr, flush=True)
    wall = time.perf_counter() - t_all
    ntr = trials * len(rows)
    result = {"metric": "findDmax prefix evaluations/s (every D-term sum of a trial encrypted, decrypted and "
                        "checked; host encryption included)",
              "value": round(ntr * w["d_cap"] / wall, 1),
              "unit": "prefixes/s", "n_gpus": 1, "steps": ntr, "warmup": 0, "ms_per_step": round(wall * 1e3 / ntr, 2),
              "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
              "config": {"workload": f"dmax: {w['desc']}", "primes": list(q), "trials_per_setting": trials},
              "sweep": rows}
    if not args.no_cpu_baseline:
        from oracle import dmax as odmax
        from oracle.params import Params as OParams
        r0 = rows[0]
        cap = 64  # a bounded oracle trial: at most 64 prefixes (encryption of its model untimed)
        o = OParams(N=N, q=q, t=r0["t"], D=cap, K=K, F=8, scheme=r0["scheme"], qbits=w["qbits"])
        t0 = time.perf_counter()
        d0 = odmax.trial(o, args.seed, cap, w["cbits"])
        t_or = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": round(min(d0 + 1, cap) / t_or, 3), "unit": "prefixes/s", "cores": 1,
                                  "kind": "oracle",
                                  "sample": f"one oracle trial of the first setting ({r0['scheme']}, t={r0['t']}) "
                                            f"capped at {cap} prefixes (it evaluated {min(d0 + 1, cap)}; its model "
                                            f"encryption included); numpy and Python integers, single thread",
                                  "seconds": round(t_or, 2)}
    print(json.dumps(result), flush=True)
    return 0


def run_single(args, w, layout: str):
    """One single-request workload in one slot layout: the JSON fields of its line (without
    the batching leg and the CPU baseline), plus the inputs the CPU baseline samples."""
    import torch
    N, L, Q = w["N"], w["L"], w["Q"]
    alpha, r = w.get("alpha", 0), w.get("r", 1)
    primes = ep.default_primes(N, L + alpha)
    prm = ep.Params(N=N, q=tuple(primes[:L]), p=tuple(primes[L:]), F=w["F"], D=w["D"], K=w["K"], r=r,
                    dnum=w.get("dnum", 0), layout=layout)
    M = ep.ephdc_num_model_ct(prm)
    seed = args.seed
    t0 = time.perf_counter()
    x = synth.blob_images(seed, Q) if w["images"] else synth.uniform_features(seed, Q, w["F"])
    base = synth.base_hypervectors(seed, w["F"], w["D"])
    C = synth.class_hypervectors(seed, w["K"], w["D"])
    t_inputs = time.perf_counter() - t0
    t0 = time.perf_counter()
    sk, gk = ep.ephdc_keygen(prm, seed)
    model = ep.ephdc_encrypt_model(prm, sk, C, seed)
    t_encrypt = time.perf_counter() - t0
    print(f"[bench] {args.workload}: inputs {t_inputs:.1f}s, keygen+encrypt {t_encrypt:.1f}s (host)",
          file=sys.stderr, flush=True)

    dev = torch.device("cuda")
    d_model = torch.from_numpy(model.view(np.int32)).to(dev)
    d_gk = torch.from_numpy(gk.view(np.int32)).to(dev) if r > 1 else None
    sess = ep.Session(prm, d_model, d_gk, max_Q=Q)
    del d_model, d_gk, model
    if args.schedule:
        mode, vpt, lg, blocks = args.schedule.split(",")
        sess.tune(int(lg), int(blocks), int(vpt), mode)
    stride = sess.hv_stride(Q)
    G = sess.num_groups(Q)
    d_x = torch.from_numpy(x).to(dev)
    d_base = torch.from_numpy(base).to(dev)
    d_hv = torch.empty((prm.D, stride), dtype=torch.int8, device=dev)
    d_out = torch.empty((G, 2, L, N), dtype=torch.int32, device=dev)
    torch.cuda.synchronize()

    def step():
        ep.ephdc_encode_queries(sess, d_x, d_base, Q, d_hv)
        ep.ephdc_score_encrypted(sess, d_hv, Q, d_out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # throughput: the timed steps back to back between two synchronisations, with nothing
    # else on the stream (a timing event recorded between two steps stalls the GPU for tens
    # of microseconds); then the same steps with an event pair each for the latency
    # percentiles, and again with the session's kernel timers for the per-stage times
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for k in range(args.steps):
        ev[k][0].record(stream)
        step()
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    sess.profile(True)
    for k in range(args.steps):
        step()
    torch.cuda.synchronize()
    prof = sess.profile_read()
    sess.profile(False)
    # correctness check of this exact launch configuration (after the timed passes, so that
    # the timed steps follow the warm-up directly): decrypted scores of every query of the
    # last step equal the exact integer similarity (mod t) of the device-computed hypervectors
    out = d_out.cpu().numpy().view(np.uint32)
    hv = d_hv.cpu().numpy()[:, :Q].T.astype(np.float64)
    scores, _ = ep.ephdc_decrypt_scores(prm, sk, out, Q)
    want = (hv @ C.astype(np.float64).T).astype(np.int64) % 65537
    want = np.where(want > 32768, want - 65537, want)
    if not np.array_equal(scores, want):
        print("[bench] decrypted scores differ from h.C mod t", file=sys.stderr)
        return None
    ms_step = wall * 1e3 / args.steps
    value = Q * args.steps / wall

    def per_launch(kernel, stage):
        """(algorithmic modmuls of one launch, average launch ms): a step may cut the model
        range into several equal chunks, each one launch of the kernel."""
        tot_ms, n = prof[stage]
        per_step = algorithmic_modmuls(kernel, N, L, G, M)
        return per_step * args.steps / n, tot_ms / n

    split = prof["mac"][1] > 0
    kern, stage = ("k_mac", "mac") if split else ("k_score", "score")
    modmuls, k_ms = per_launch(kern, stage)
    achieved = modmuls / (k_ms * 1e-3)
    # subring layout with the n-point kernels (n = N/K' of 256..4096 under N = 2048..16384,
    # K' <= 32)
    Kp = 1 << (w["K"] - 1).bit_length() if layout == "subring" else w["K"]
    n_sub = N // Kp
    sub = layout == "subring" and 2048 <= N <= 16384 and 256 <= n_sub <= 4096 and 2 <= Kp <= 32

    def hbm(traffic, ms):
        """Achieved HBM bandwidth of a launch moving `traffic` bytes in `ms`, and its fraction of 8 TB/s."""
        if traffic is None:
            return {"hbm_gbps": None, "hbm_frac": None}
        return {"hbm_gbps": round(traffic / (ms * 1e-3) / 1e9, 1), "hbm_frac": round(traffic / (ms * 1e-3) / HBM_PEAK, 4)}
    result = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "inferences/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {w['desc']}", "queries_per_step": Q, "groups": G,
                   "queries_per_ciphertext": ep.ephdc_queries_per_ct(prm),
                   "model_ciphertexts": M, "rotations_per_group": int(math.log2(r)),
                   "layout": layout, "schedule": ("subring n=%d" % n_sub) if sub else ("split" if split else "fused")},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                       "p99": round(float(np.percentile(lat, 99)), 4)},
        "stages_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in prof.items() if v[1]},
        "launches_per_step": {k: v[1] // args.steps for k, v in prof.items() if v[1]},
        "roofline": {"bound": "alu", "kernel": kern, "achieved": round(achieved / 1e12, 4),
                     "peak": round(MODMUL_PEAK / 1e12, 4), "unit": "Tmodmul/s",
                     "frac": round(achieved / MODMUL_PEAK, 4),
                     "traffic": recorded_traffic(kern, args.workload),
                     "per_launch_modmuls": modmuls, "avg_launch_ms": round(k_ms, 4),
                     **hbm(recorded_traffic(kern, args.workload), k_ms),
                     "valu_issue": recorded_valu_issue(kern, args.workload)},
    }
    if sub:
        # the streaming MAC is bound by HBM: algorithmic bytes = the model once, the n-point
        # transforms of every (group, plaintext, limb) once, and the score sums once
        nl = prof["mac"][1] // args.steps
        mac_bytes = (M * 2 * L * N + G * M * L * n_sub + G * 2 * L * N) * 4.0 / nl
        mac_ms = prof["mac"][0] / prof["mac"][1]
        tr = recorded_traffic("k_mac_sub", args.workload)
        result["roofline"] = {"bound": "hbm", "kernel": "k_mac_sub", "achieved": round(mac_bytes / (mac_ms * 1e-3) / 1e9, 1),
                              "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                              "frac": round(mac_bytes / (mac_ms * 1e-3) / HBM_PEAK, 4), "traffic": tr,
                              "algorithmic_bytes": mac_bytes, "avg_launch_ms": round(mac_ms, 4),
                              **({"traffic_gbps": round(tr / (mac_ms * 1e-3) / 1e9, 1),
                                  "traffic_frac": round(tr / (mac_ms * 1e-3) / HBM_PEAK, 4)} if tr else {}),
                              "valu_issue": recorded_valu_issue("k_mac_sub", "subring_" + args.workload)}
        enc_ms = prof["encode_pt"][0] / prof["encode_pt"][1]
        enc_ops = G * M * (1 + L) * transform_mults(n_sub) / nl
        result["roofline_encode_pt"] = {"bound": "alu", "kernel": "k_encode_sub",
                                        "achieved": round(enc_ops / (enc_ms * 1e-3) / 1e12, 4),
                                        "peak": round(MODMUL_PEAK / 1e12, 4), "unit": "Tmodmul/s",
                                        "frac": round(enc_ops / (enc_ms * 1e-3) / MODMUL_PEAK, 4),
                                        "per_launch_modmuls": enc_ops, "avg_launch_ms": round(enc_ms, 4),
                                        "traffic": recorded_traffic("k_encode_sub", args.workload),
                                        **hbm(recorded_traffic("k_encode_sub", args.workload), enc_ms),
                                        "valu_issue": recorded_valu_issue("k_encode_sub", "subring_" + args.workload)}
    elif split:
        e_ops, e_ms = per_launch("k_encode_pt", "encode_pt")
        result["roofline_encode_pt"] = {"bound": "alu", "kernel": "k_encode_pt",
                                        "achieved": round(e_ops / (e_ms * 1e-3) / 1e12, 4),
                                        "frac": round(e_ops / (e_ms * 1e-3) / MODMUL_PEAK, 4),
                                        "avg_launch_ms": round(e_ms, 4),
                                        "traffic": recorded_traffic("k_encode_pt", args.workload),
                                        **hbm(recorded_traffic("k_encode_pt", args.workload), e_ms),
                                        "valu_issue": recorded_valu_issue("k_encode_pt", args.workload)}
    if prof["encode"][1]:
        # the HDC projection: 2*F*D int8 operations per query, against the dense int8 MFMA peak
        h_ms = prof["encode"][0] / prof["encode"][1]
        h_ops = 2.0 * Q * w["F"] * w["D"]
        result["roofline_hdc"] = {"bound": "mfma", "kernel": "k_hdc_encode",
                                  "achieved": round(h_ops / (h_ms * 1e-3) / 1e12, 2), "peak": INT8_PEAK / 1e12,
                                  "unit": "TOP/s", "frac": round(h_ops / (h_ms * 1e-3) / INT8_PEAK, 4),
                                  "traffic": recorded_traffic("k_hdc_encode", args.workload),
                                  "avg_launch_ms": round(h_ms, 4)}
    sess.close()
    del d_x, d_base, d_hv, d_out
    return result, prm, x, base, C


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-unpacked", action="store_true",
                    help="batching workload: only its unpacked batch, eager, default schedule (for counter runs)")
    ap.add_argument("--no-batched", action="store_true",
                    help="plain workload only: skip the batching workload's plain / batched / packed leg")
    ap.add_argument("--cpu-sample-m", type=int, default=0,
                    help="model ciphertexts in the oracle's timed sample (0: the workload's default)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--duration", type=float, default=0.0, help="serving: trace length in seconds")
    ap.add_argument("--schedule", default="", help="single-request workloads: mode,values_per_thread,limb_group,blocks "
                                                  "(e.g. split,16,1,512; empty keeps the session's default)")
    ap.add_argument("--rates", default="", help="serving: comma-separated extra arrival rates (req/s)")
    ap.add_argument("--layout", default="auto", choices=["auto", "contiguous", "subring"],
                    help="single-request workloads: slot layout of the queries (auto: the N = 8192 and "
                         "N = 16384 workloads in the subring layout, with the contiguous layout measured beside it)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 256 MiB device copy three times (calibrates FETCH_SIZE/WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the path shards by query group or model slice, "
              "but no multi-GPU run is part of this benchmark", file=sys.stderr)
        return 2

    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    if args.calibrate_copy:
        a = torch.empty(64 << 20, dtype=torch.int32, device="cuda").fill_(1)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 4, "copies": 3}))
        return 0
    w = WORKLOADS[args.workload]
    if "requests" in w:
        return profile_unpacked(args, w) if args.profile_unpacked else bench_batched(args, w)
    if w.get("serving"):
        return bench_serving(args, w)
    if w.get("dmax"):
        return bench_dmax(args, w)
    if w.get("detect"):
        return bench_detect(args, w)
    layouts = {"auto": ["subring", "contiguous"] if args.workload in ("c2", "c4") else ["contiguous"]}.get(
        args.layout, [args.layout])
    runs = []
    for lay in layouts:
        r = run_single(args, w, lay)
        if r is None:
            return 3
        runs.append(r)
    result, prm, x, base, C = runs[0]
    for other, *_ in runs[1:]:
        keep = ("value", "ms_per_step", "latency_ms", "stages_ms_per_step", "roofline", "roofline_encode_pt",
                "roofline_hdc", "config")
        result["layout_" + other["config"]["layout"]] = {k: other[k] for k in keep if k in other}
    if args.workload == "c2" and not args.no_batched:
        # the metric's other half: the batching workload at the same N and limbs, its requests
        # scored one after another (plain), as one unpacked batch and as one packed batch
        keys = ("config", "plain", "batched_unpacked", "packed", "packed_eager", "speedup_unpacked_vs_plain",
                "speedup_packed_vs_plain")
        for lay in layouts:
            b = run_batched(args, WORKLOADS["c3"], lay)
            if b is None:
                return 3
            result["batched" if lay == layouts[0] else "batched_" + lay] = {k: b[k] for k in keys}
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(w, prm, x, base, C, args.cpu_sample_m or w.get("cpu_sample_m", 256))
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
