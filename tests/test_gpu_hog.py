"""The detection front end on the device (sliding windows and their HOG feature maps)
against the oracle, byte for byte, and the client path from a raw frame to decrypted scores."""
import numpy as np
import pytest

import paper_2511_00737_amd as ep
import synth
from oracle import bfv, hdc, hog, pipeline
from oracle.params import Params as OParams, default_primes

from gpu_helpers import to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def hog_on_gpu(fr, window, stride):
    import torch
    H, W = fr.shape
    n = ep.ephdc_hog_window_count(H, W, window, stride)
    F = ep.ephdc_hog_feature_count(window)
    d_x = torch.full((n, F), 7, dtype=torch.uint8, device="cuda")
    ep.ephdc_hog_windows(to_dev(fr), window, stride, d_x)
    torch.cuda.synchronize()
    return d_x.cpu().numpy()


@pytest.mark.parametrize("H,W,window,stride,kind", [(64, 64, 64, 8, "noise"), (40, 48, 16, 8, "noise"),
                                                    (101, 77, 24, 16, "noise"), (96, 200, 48, 8, "frame"),
                                                    (240, 320, 64, 8, "frame"), (130, 130, 32, 24, "zero")])
def test_window_features_match_oracle(H, W, window, stride, kind):
    torch_cuda()
    rng = np.random.default_rng(H * W)
    if kind == "noise":
        fr = rng.integers(0, 256, (H, W)).astype(np.uint8)
    elif kind == "frame":
        fr = synth.frame(H + W, H, W, n_objects=6)
    else:
        fr = np.zeros((H, W), dtype=np.uint8)
    got = hog_on_gpu(fr, window, stride)
    want = hog.window_features(fr, window, stride)
    assert got.shape == want.shape
    assert np.array_equal(got, want)


def test_full_hd_frame_matches_oracle():
    """A 1080 x 1920 frame, 64 x 64 windows at a stride of 8 pixels: 29,824 windows of 1,776
    features, every byte equal to the oracle's."""
    torch_cuda()
    fr = synth.frame(0, 1080, 1920)
    got = hog_on_gpu(fr, 64, 8)
    want = hog.window_features(fr, 64, 8)
    assert got.shape == (29824, 1776)
    assert np.array_equal(got, want)


def test_frame_to_scores_on_the_client_path():
    """Frame -> HOG windows -> HDC encoding -> encrypted scoring (N = 2048, the paper's
    optimised ring, 2 limbs, K = 2) -> decryption: every window's scores equal h . C mod t with
    h the oracle's encoding of the oracle's HOG features."""
    torch = torch_cuda()
    fr = synth.frame(5, 160, 224, n_objects=8)
    window, stride = 64, 8
    x = hog.window_features(fr, window, stride)
    Q, F = x.shape
    N, L, D, K = 2048, 2, 256, 2
    q = tuple(default_primes(N, L))
    o = OParams(N=N, q=q, F=F, D=D, K=K)
    e = ep.Params(N=N, q=q, F=F, D=D, K=K)
    base = synth.base_hypervectors(5, F, D)
    C = synth.class_hypervectors(5, K, D)
    sk, _ = ep.ephdc_keygen(e, 5)
    model = ep.ephdc_encrypt_model(e, sk, C, 5)
    s = ep.Session(e, to_dev(model), max_Q=Q)
    try:
        d_x = torch.empty((Q, F), dtype=torch.uint8, device="cuda")
        ep.ephdc_hog_windows(to_dev(fr), window, stride, d_x)
        d_hv = torch.empty((D, s.hv_stride(Q)), dtype=torch.int8, device="cuda")
        ep.ephdc_encode_queries(s, d_x, to_dev(base), Q, d_hv)
        d_out = torch.empty((s.num_groups(Q), 2, L, N), dtype=torch.int32, device="cuda")
        ep.ephdc_score_encrypted(s, d_hv, Q, d_out)
        torch.cuda.synchronize()
        cts = d_out.cpu().numpy().view(np.uint32)
        hv = d_hv.cpu().numpy()
    finally:
        s.close()
    h = hdc.encode(x, base)
    assert np.array_equal(hv[:, :Q].T, h)
    sc, am = ep.ephdc_decrypt_scores(e, sk, cts, Q)
    assert np.array_equal(sc, hdc.scores_mod_t(h, C, o.t))
    assert np.array_equal(am, hdc.argmax(hdc.scores_int(h, C)))
    assert np.array_equal(cts[:1].astype(np.int64), pipeline.score_ciphertexts(o, model.astype(np.int64), h, groups=[0]))


def test_hog_argument_checks():
    torch = torch_cuda()
    assert ep.ephdc_hog_feature_count(20) == 0 and ep.ephdc_hog_window_count(64, 64, 64, 12) == 0
    fr = torch.zeros((64, 64), dtype=torch.uint8, device="cuda")
    x = torch.empty((1, 1776), dtype=torch.uint8, device="cuda")
    with pytest.raises(ep.EphdcError) as ei:
        ep.ephdc_hog_windows(fr, 64, 12, x)
    assert ei.value.status == ep.ERR_ARG
    with pytest.raises(ep.EphdcError) as ei:
        ep.ephdc_hog_windows(fr, 64, 8, x, d_workspace=torch.empty(16, dtype=torch.uint8, device="cuda"))
    assert ei.value.status == ep.ERR_BUFFER
