"""Python binding of libephdc: EP-HDC client-side encrypted HDC inference on MI355X.

A thin ctypes layer over the C ABI declared in include/ephdc.h.  Every entry point keeps
its C name and only marshals arguments: host arrays are numpy, device buffers are torch
tensors on the current HIP device (PyTorch is used for device memory and streams only).
All computation happens in the library's host C++ (server side) or HIP kernels (client
side).  Importing this module does not load the library; the first call does, and it
raises if the library has not been built (python -m paper_2511_00737_amd.build).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libephdc.so")

OK, ERR_ARG, ERR_PARAMS, ERR_BUFFER, ERR_HIP, ERR_NOKEY, ERR_OOM, ERR_UNSUPPORTED, ERR_TIMEOUT = range(9)
T_PLAIN = 65537


class EphdcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ephdc status {status}: {msg}")
        self.status = status


class _CParams(C.Structure):
    _fields_ = [("N", C.c_uint32), ("L", C.c_uint32), ("alpha", C.c_uint32), ("dnum", C.c_uint32),
                ("q", C.POINTER(C.c_uint32)), ("p", C.POINTER(C.c_uint32)), ("t", C.c_uint32),
                ("F", C.c_uint32), ("D", C.c_uint32), ("K", C.c_uint32), ("r", C.c_uint32),
                ("qbits", C.c_int32), ("qshift", C.c_uint32), ("scheme", C.c_uint32),
                ("scale_every", C.c_uint32), ("scale_shift", C.c_uint32), ("layout", C.c_uint32)]


SCHEMES = {"bfv": 0, "bfv-r": 1, "bgv": 2}
LAYOUTS = {"contiguous": 0, "subring": 1}


class _CRequest(C.Structure):
    _fields_ = [("session", C.c_void_p), ("d_x", C.c_void_p), ("d_base", C.c_void_p), ("d_hv", C.c_void_p),
                ("Q", C.c_uint32), ("d_score_ct", C.c_void_p)]


_lib = None


def lib() -> C.CDLL:
    """The loaded library (fails loudly when it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2511_00737_amd.build")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER(_CParams)
        u32p, i8p, u8p, i32p, u64p = (C.POINTER(C.c_uint32), C.POINTER(C.c_int8), C.POINTER(C.c_uint8),
                                      C.POINTER(C.c_int32), C.POINTER(C.c_uint64))
        sig = {
            "ephdc_last_error": (C.c_char_p, []),
            "ephdc_check_params": (C.c_int, [P]),
            "ephdc_queries_per_ct": (C.c_uint32, [P]),
            "ephdc_num_model_ct": (C.c_uint32, [P]),
            "ephdc_num_groups": (C.c_uint32, [P, C.c_uint32]),
            "ephdc_hv_stride": (C.c_uint32, [P, C.c_uint32]),
            "ephdc_galois_key_words": (C.c_size_t, [P]),
            "ephdc_default_primes": (C.c_int, [C.c_uint32, C.c_uint32, C.c_uint32, u32p]),
            "ephdc_gaussian_cdt": (C.c_int, [u64p]),
            "ephdc_keygen": (C.c_int, [P, C.c_uint64, i8p, u32p]),
            "ephdc_encrypt_model": (C.c_int, [P, i8p, i8p, C.c_uint64, u32p]),
            "ephdc_decrypt_scores": (C.c_int, [P, i8p, u32p, C.c_uint32, i32p, i32p]),
            "ephdc_decrypt_scores_at": (C.c_int, [P, i8p, u32p, C.c_uint32, C.c_uint32, i32p, i32p]),
            "ephdc_workspace_bytes": (C.c_size_t, [P, C.c_uint32]),
            "ephdc_session_create": (C.c_int, [P, C.c_void_p, C.c_size_t, C.c_void_p, C.c_size_t, C.c_uint32,
                                               C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]),
            "ephdc_session_destroy": (C.c_int, [C.c_void_p]),
            "ephdc_session_device_bytes": (C.c_size_t, [C.c_void_p]),
            "ephdc_encode_queries": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p,
                                               C.c_void_p]),
            "ephdc_score_encrypted": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p]),
            "ephdc_score_encrypted_static": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p,
                                                       C.c_void_p]),
            "ephdc_debug_plaintext": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32,
                                                C.c_void_p, C.c_void_p]),
            "ephdc_debug_polymul": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p,
                                              C.c_void_p]),
            "ephdc_find_dmax": (C.c_int, [P, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, i32p, C.c_void_p]),
            "ephdc_hog_feature_count": (C.c_uint32, [C.c_uint32]),
            "ephdc_hog_window_count": (C.c_uint32, [C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]),
            "ephdc_hog_workspace_bytes": (C.c_size_t, [C.c_uint32, C.c_uint32]),
            "ephdc_hog_windows": (C.c_int, [C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_void_p,
                                            C.c_size_t, C.c_void_p, C.c_void_p]),
            "ephdc_session_profile": (C.c_int, [C.c_void_p, C.c_int]),
            "ephdc_session_set_chunk_bytes": (C.c_int, [C.c_void_p, C.c_size_t]),
            "ephdc_session_tune": (C.c_int, [C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]),
            "ephdc_session_profile_read": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), u64p]),
            "ephdc_batch_create": (C.c_int, [C.POINTER(_CRequest), C.c_uint32, C.POINTER(C.c_void_p)]),
            "ephdc_batch_destroy": (C.c_int, [C.c_void_p]),
            "ephdc_batch_device_bytes": (C.c_size_t, [C.c_void_p]),
            "ephdc_batch_tune": (C.c_int, [C.c_void_p, u32p]),
            "ephdc_batch_schedule": (C.c_int, [C.c_void_p, u32p]),
            "ephdc_batch_autotune": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, u32p, C.POINTER(C.c_double)]),
            "ephdc_batch_run": (C.c_int, [C.c_void_p, C.c_void_p]),
            "ephdc_batch_capture": (C.c_int, [C.c_void_p, C.c_void_p]),
            "ephdc_score_many": (C.c_int, [C.POINTER(_CRequest), C.c_uint32, C.c_void_p]),
            "ephdc_batch_create_packed": (C.c_int, [C.POINTER(_CRequest), C.c_uint32, C.POINTER(C.c_void_p)]),
            "ephdc_batch_packing": (C.c_int, [C.c_void_p, C.c_uint32, u32p, u32p, u32p]),
            "ephdc_server_set_packing": (C.c_int, [C.c_void_p, C.c_int]),
            "ephdc_server_result": (C.c_int, [C.c_void_p, C.c_uint64, u32p, u32p]),
            "ephdc_server_create": (C.c_int, [C.c_size_t, C.c_uint32, C.c_uint32, C.POINTER(C.c_void_p)]),
            "ephdc_server_add_tenant": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, u32p]),
            "ephdc_server_submit": (C.c_int, [C.c_void_p, C.c_uint32, C.c_void_p, C.c_uint32, C.c_void_p,
                                              C.c_void_p, u64p]),
            "ephdc_server_release": (C.c_int, [C.c_void_p, C.c_uint64]),
            "ephdc_server_query": (C.c_int, [C.c_void_p, C.c_uint64, i32p, C.POINTER(C.c_double)]),
            "ephdc_server_wait": (C.c_int, [C.c_void_p, C.c_uint64, C.c_double]),
            "ephdc_server_stats": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
            "ephdc_server_destroy": (C.c_int, [C.c_void_p]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(st: int) -> None:
    if st != OK:
        raise EphdcError(st, lib().ephdc_last_error().decode())


def _ptr(a: np.ndarray, ctype):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(ctype))


# ------------------------------------------------------------------ parameters
@dataclass
class Params:
    """The ephdc_params struct (see include/ephdc.h)."""
    N: int
    q: tuple
    F: int
    D: int
    K: int
    r: int = 1
    p: tuple = ()
    dnum: int = 0
    t: int = T_PLAIN
    qbits: int = 1
    qshift: int = 0
    scheme: str = "bfv"     # "bfv", "bfv-r" (rounded scaling) or "bgv"
    scale_every: int = 0    # HE-aware scaling after every g accumulations (0: never)
    scale_shift: int = 0    # ... by the inverse of 2^scale_shift mod t
    layout: str = "contiguous"  # slot layout: "contiguous" or "subring"
    _keep: list = field(default_factory=list, repr=False, compare=False)

    @property
    def L(self) -> int:
        return len(self.q)

    @property
    def alpha(self) -> int:
        return len(self.p)

    def c(self) -> _CParams:
        qa = (C.c_uint32 * max(1, len(self.q)))(*self.q)
        pa = (C.c_uint32 * max(1, len(self.p)))(*self.p)
        self._keep[:] = [qa, pa]
        return _CParams(self.N, len(self.q), len(self.p), self.dnum, qa, pa, self.t, self.F, self.D, self.K,
                        self.r, self.qbits, self.qshift, SCHEMES[self.scheme], self.scale_every, self.scale_shift,
                        LAYOUTS[self.layout])


def default_primes(N: int, count: int, skip: int = 0) -> list[int]:
    out = np.zeros(count, dtype=np.uint32)
    _check(lib().ephdc_default_primes(N, count, skip, _ptr(out, C.c_uint32)))
    return [int(x) for x in out]


def ephdc_check_params(prm: Params) -> int:
    c = prm.c()
    return lib().ephdc_check_params(C.byref(c))


def ephdc_queries_per_ct(prm: Params) -> int:
    c = prm.c()
    return lib().ephdc_queries_per_ct(C.byref(c))


def ephdc_num_model_ct(prm: Params) -> int:
    c = prm.c()
    return lib().ephdc_num_model_ct(C.byref(c))


def ephdc_num_groups(prm: Params, Q: int) -> int:
    c = prm.c()
    return lib().ephdc_num_groups(C.byref(c), Q)


def ephdc_hv_stride(prm: Params, Q: int) -> int:
    c = prm.c()
    return lib().ephdc_hv_stride(C.byref(c), Q)


def ephdc_galois_key_words(prm: Params) -> int:
    c = prm.c()
    return lib().ephdc_galois_key_words(C.byref(c))


def ephdc_workspace_bytes(prm: Params, max_Q: int) -> int:
    c = prm.c()
    return lib().ephdc_workspace_bytes(C.byref(c), max_Q)


def ephdc_gaussian_cdt() -> list[int]:
    out = np.zeros(39, dtype=np.uint64)
    _check(lib().ephdc_gaussian_cdt(_ptr(out, C.c_uint64)))
    return [int(x) for x in out]


# ------------------------------------------------------------------ server side (host memory)
def ephdc_keygen(prm: Params, seed: int):
    """(sk int8 [N], galois_keys uint32 [log2 r][dnum][2][L+alpha][N] or None)."""
    c = prm.c()
    sk = np.zeros(prm.N, dtype=np.int8)
    nwords = lib().ephdc_galois_key_words(C.byref(c)) if prm.r > 1 else 0
    gk = np.zeros(nwords, dtype=np.uint32) if nwords else None
    _check(lib().ephdc_keygen(C.byref(c), seed, _ptr(sk, C.c_int8),
                              _ptr(gk, C.c_uint32) if gk is not None else None))
    if gk is not None:
        logr = prm.r.bit_length() - 1
        gk = gk.reshape(logr, prm.dnum, 2, prm.L + prm.alpha, prm.N)
    return sk, gk


def ephdc_encrypt_model(prm: Params, sk: np.ndarray, class_hv: np.ndarray, seed: int) -> np.ndarray:
    """Model ciphertexts uint32 [M][2][L][N], coefficient domain."""
    c = prm.c()
    M = lib().ephdc_num_model_ct(C.byref(c))
    out = np.zeros((M, 2, prm.L, prm.N), dtype=np.uint32)
    sk = np.ascontiguousarray(sk, dtype=np.int8)
    chv = np.ascontiguousarray(class_hv, dtype=np.int8)
    _check(lib().ephdc_encrypt_model(C.byref(c), _ptr(sk, C.c_int8), _ptr(chv, C.c_int8), seed,
                                     _ptr(out, C.c_uint32)))
    return out


def ephdc_decrypt_scores(prm: Params, sk: np.ndarray, score_ct: np.ndarray, Q: int):
    """(scores int32 [Q][K], argmax int32 [Q])."""
    c = prm.c()
    sc = np.zeros((Q, prm.K), dtype=np.int32)
    am = np.zeros(Q, dtype=np.int32)
    sk = np.ascontiguousarray(sk, dtype=np.int8)
    cts = np.ascontiguousarray(score_ct, dtype=np.uint32)
    _check(lib().ephdc_decrypt_scores(C.byref(c), _ptr(sk, C.c_int8), _ptr(cts, C.c_uint32), Q,
                                      _ptr(sc, C.c_int32), _ptr(am, C.c_int32)))
    return sc, am


def ephdc_decrypt_scores_at(prm: Params, sk: np.ndarray, score_ct: np.ndarray, q_first: int, Q: int):
    """Scores of queries q_first .. q_first+Q-1 of a ciphertext sequence (see the header)."""
    c = prm.c()
    sc = np.zeros((Q, prm.K), dtype=np.int32)
    am = np.zeros(Q, dtype=np.int32)
    sk = np.ascontiguousarray(sk, dtype=np.int8)
    cts = np.ascontiguousarray(score_ct, dtype=np.uint32)
    B = lib().ephdc_queries_per_ct(C.byref(c))
    need = -(-(q_first + Q) // B) * 2 * prm.L * prm.N
    if cts.size < need:
        raise EphdcError(ERR_BUFFER, f"score_ct holds {cts.size} words, needs {need}")
    _check(lib().ephdc_decrypt_scores_at(C.byref(c), _ptr(sk, C.c_int8), _ptr(cts, C.c_uint32), q_first, Q,
                                         _ptr(sc, C.c_int32), _ptr(am, C.c_int32)))
    return sc, am


# ------------------------------------------------------------------ client side (device memory)
def _stream(stream=None) -> int:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _dptr(t, nbytes: int | None = None) -> int:
    """Device address of a contiguous CUDA tensor holding at least `nbytes` bytes."""
    if not (t.is_cuda and t.is_contiguous()):
        raise EphdcError(ERR_ARG, "expected a contiguous device tensor")
    if nbytes is not None and t.numel() * t.element_size() < nbytes:
        raise EphdcError(ERR_BUFFER, f"device buffer holds {t.numel() * t.element_size()} bytes, needs {nbytes}")
    return t.data_ptr()


def _words(t) -> int:
    return t.numel() * t.element_size() // 4


class Session:
    """Owns an ephdc_session: device-resident evaluation-domain model and keys.

    workspace: True allocates a device tensor of ephdc_workspace_bytes(prm, max_Q) bytes
    (kept alive here and lent to the session); a uint8 device tensor is lent as given;
    None creates a session without one (batches, serving and the static-scratch entry
    point bring their own scratch)."""

    def __init__(self, prm: Params, d_model_ct, d_galois_keys=None, max_Q: int = 4096, stream=None,
                 workspace=True):
        import torch
        self.prm = prm
        self._c = prm.c()
        h = C.c_void_p()
        gk_ptr = _dptr(d_galois_keys) if d_galois_keys is not None else None
        gk_words = _words(d_galois_keys) if d_galois_keys is not None else 0
        if workspace is True:
            nbytes = lib().ephdc_workspace_bytes(C.byref(self._c), max_Q)
            if nbytes == 0:
                _check(lib().ephdc_check_params(C.byref(self._c)) or ERR_ARG)
            workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.workspace = workspace if workspace is not None and workspace is not False else None
        ws_ptr = _dptr(self.workspace) if self.workspace is not None else None
        ws_bytes = self.workspace.numel() * self.workspace.element_size() if self.workspace is not None else 0
        _check(lib().ephdc_session_create(C.byref(self._c), _dptr(d_model_ct), _words(d_model_ct), gk_ptr,
                                          gk_words, max_Q, ws_ptr, ws_bytes, _stream(stream), C.byref(h)))
        self.handle = h
        self.max_Q = max_Q

    def close(self) -> None:
        if self.handle:
            _check(lib().ephdc_session_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def device_bytes(self) -> int:
        return lib().ephdc_session_device_bytes(self.handle)

    def tune(self, limb_group: int = 0, blocks: int = 0, values_per_thread: int = 0, mode: str | None = None) -> None:
        """Schedule of the scoring kernel (see ephdc_session_tune); 0 / None keeps a setting."""
        m = {None: 0, "fused": 1, "split": 2}[mode]
        _check(lib().ephdc_session_tune(self.handle, limb_group, blocks, values_per_thread, m))

    def set_chunk_bytes(self, nbytes: int) -> None:
        """Bound on the split path's plaintext buffer (see ephdc_session_set_chunk_bytes)."""
        _check(lib().ephdc_session_set_chunk_bytes(self.handle, nbytes))

    def profile(self, enable: bool = True) -> None:
        """Bracket every kernel launch with HIP events on its stream (see ephdc_session_profile)."""
        _check(lib().ephdc_session_profile(self.handle, 1 if enable else 0))

    def profile_read(self):
        """{stage: (total ms, launches)} per kernel stage (see ephdc_session_profile_read); resets them."""
        ms = (C.c_double * 6)()
        cnt = np.zeros(6, dtype=np.uint64)
        _check(lib().ephdc_session_profile_read(self.handle, ms, _ptr(cnt, C.c_uint64)))
        names = ("score", "finish", "encode", "rotate", "encode_pt", "mac")
        return {n: (float(ms[i]), int(cnt[i])) for i, n in enumerate(names)}

    def hv_stride(self, Q: int) -> int:
        return lib().ephdc_hv_stride(C.byref(self._c), Q)

    def num_groups(self, Q: int) -> int:
        return lib().ephdc_num_groups(C.byref(self._c), Q)


def ephdc_session_create(prm: Params, d_model_ct, d_galois_keys=None, max_Q: int = 4096, stream=None,
                         workspace=True) -> Session:
    return Session(prm, d_model_ct, d_galois_keys, max_Q, stream, workspace)


def ephdc_session_destroy(s: Session) -> None:
    s.close()


def _sizes(s: Session, Q: int):
    p = s.prm
    stride = s.hv_stride(Q)
    return stride, p.D * stride, s.num_groups(Q) * 2 * p.L * p.N * 4


def ephdc_encode_queries(s: Session, d_x, d_base, Q: int, d_hv, stream=None) -> None:
    p = s.prm
    _, hv_bytes, _ = _sizes(s, Q)
    _check(lib().ephdc_encode_queries(s.handle, _dptr(d_x, Q * p.F), _dptr(d_base, p.F * p.D), Q,
                                      _dptr(d_hv, hv_bytes), _stream(stream)))


def ephdc_score_encrypted(s: Session, d_hv, Q: int, d_score_ct, stream=None) -> None:
    _, hv_bytes, out_bytes = _sizes(s, Q)
    _check(lib().ephdc_score_encrypted(s.handle, _dptr(d_hv, hv_bytes), Q, _dptr(d_score_ct, out_bytes),
                                       _stream(stream)))


def ephdc_score_encrypted_static(s: Session, d_hv, Q: int, d_score_ct, stream=None) -> None:
    """ephdc_score_encrypted with the library's static per-GPU scratch (allocates nothing)."""
    _, hv_bytes, out_bytes = _sizes(s, Q)
    _check(lib().ephdc_score_encrypted_static(s.handle, _dptr(d_hv, hv_bytes), Q, _dptr(d_score_ct, out_bytes),
                                              _stream(stream)))


def ephdc_debug_plaintext(s: Session, d_hv, Q: int, g: int, m: int, d_out, stream=None) -> None:
    p = s.prm
    _, hv_bytes, _ = _sizes(s, Q)
    _check(lib().ephdc_debug_plaintext(s.handle, _dptr(d_hv, hv_bytes), Q, g, m, _dptr(d_out, p.L * p.N * 4),
                                       _stream(stream)))


def ephdc_debug_polymul(s: Session, d_a, d_b, count: int, d_out, stream=None) -> None:
    nb = count * s.prm.N * 4
    _check(lib().ephdc_debug_polymul(s.handle, _dptr(d_a, nb), _dptr(d_b, nb), count, _dptr(d_out, nb),
                                     _stream(stream)))


def ephdc_find_dmax(prm: Params, seed: int, trials: int, d_cap: int, cbits: int = 8, stream=None) -> np.ndarray:
    """D_i of `trials` findDmax trials (int32 [trials]); see the header."""
    c = prm.c()
    out = np.zeros(trials, dtype=np.int32)
    _check(lib().ephdc_find_dmax(C.byref(c), seed, trials, d_cap, cbits, _ptr(out, C.c_int32), _stream(stream)))
    return out


# ------------------------------------------------------------------ detection front end
def ephdc_hog_feature_count(window: int) -> int:
    return lib().ephdc_hog_feature_count(window)


def ephdc_hog_window_count(H: int, W: int, window: int, stride: int) -> int:
    return lib().ephdc_hog_window_count(H, W, window, stride)


def ephdc_hog_workspace_bytes(H: int, W: int) -> int:
    return lib().ephdc_hog_workspace_bytes(H, W)


def ephdc_hog_windows(d_frame, window: int, stride: int, d_x, d_workspace=None, stream=None) -> None:
    """HOG features of every window of the uint8 [H][W] device frame into d_x (uint8
    [windows][features]); d_workspace: a device tensor of ephdc_hog_workspace_bytes(H, W)
    bytes, allocated here when None."""
    import torch
    H, W = int(d_frame.shape[0]), int(d_frame.shape[1])
    nws = lib().ephdc_hog_workspace_bytes(H, W)
    if d_workspace is None:
        d_workspace = torch.empty(max(nws, 1), dtype=torch.uint8, device=d_frame.device)
    need = ephdc_hog_window_count(H, W, window, stride) * ephdc_hog_feature_count(window)
    ws_bytes = d_workspace.numel() * d_workspace.element_size()
    _check(lib().ephdc_hog_windows(_dptr(d_frame, H * W), H, W, window, stride, _dptr(d_workspace), ws_bytes,
                                   _dptr(d_x, need), _stream(stream)))


# ------------------------------------------------------------------ request batches
@dataclass
class Request:
    """One client request of a batch (see ephdc_request): device tensors of the request."""
    session: "Session"
    d_hv: object
    Q: int
    d_score_ct: object
    d_x: object = None
    d_base: object = None


def _c_requests(reqs, packed: bool = False):
    arr = (_CRequest * len(reqs))()
    for i, r in enumerate(reqs):
        s, p = r.session, r.session.prm
        _, hv_bytes, out_bytes = _sizes(s, r.Q)
        if packed:  # one more ciphertext: the request's queries may straddle a boundary
            out_bytes += 2 * p.L * p.N * 4
        arr[i].session = s.handle
        arr[i].d_x = _dptr(r.d_x, r.Q * p.F) if r.d_x is not None else None
        arr[i].d_base = _dptr(r.d_base, p.F * p.D) if r.d_x is not None else None
        arr[i].d_hv = _dptr(r.d_hv, hv_bytes) if r.d_hv is not None else None
        arr[i].Q = r.Q
        arr[i].d_score_ct = _dptr(r.d_score_ct, out_bytes)
    return arr


class Batch:
    """Owns an ephdc_batch: the work lists of many requests scored by shared launches."""

    def __init__(self, reqs, packed: bool = False):
        self.reqs = list(reqs)  # keeps the sessions and tensors alive
        self.packed = packed
        arr = _c_requests(self.reqs, packed)
        h = C.c_void_p()
        create = lib().ephdc_batch_create_packed if packed else lib().ephdc_batch_create
        _check(create(arr, len(self.reqs), C.byref(h)))
        self.handle = h

    def packing(self, i: int):
        """(query_offset, q_first, n_ct) of request i of a packed batch (see the header)."""
        v = [C.c_uint32() for _ in range(3)]
        _check(lib().ephdc_batch_packing(self.handle, i, *[C.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def close(self) -> None:
        if self.handle:
            _check(lib().ephdc_batch_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def device_bytes(self) -> int:
        return lib().ephdc_batch_device_bytes(self.handle)

    def tune(self, mode: str | None = None, values_per_thread: int = 0, limb_group: int = 0, seg_len: int = 0,
             grid: int = 0) -> None:
        sc = np.array([{None: 0, "fused": 1, "split": 2}[mode], values_per_thread, limb_group, seg_len, grid],
                      dtype=np.uint32)
        _check(lib().ephdc_batch_tune(self.handle, _ptr(sc, C.c_uint32)))

    def schedule(self) -> dict:
        sc = np.zeros(5, dtype=np.uint32)
        _check(lib().ephdc_batch_schedule(self.handle, _ptr(sc, C.c_uint32)))
        return {"mode": {1: "fused", 2: "split"}[int(sc[0])], "values_per_thread": int(sc[1]),
                "limb_group": int(sc[2]), "seg_len": int(sc[3]), "grid": int(sc[4])}

    def autotune(self, reps: int = 2, stream=None):
        """(schedule dict, ms per run of the best schedule)."""
        sc = np.zeros(5, dtype=np.uint32)
        ms = C.c_double()
        _check(lib().ephdc_batch_autotune(self.handle, _stream(stream), reps, _ptr(sc, C.c_uint32), C.byref(ms)))
        return self.schedule(), ms.value

    def run(self, stream=None) -> None:
        _check(lib().ephdc_batch_run(self.handle, _stream(stream)))

    def capture(self, stream) -> None:
        """Capture the batch into a HIP graph on `stream` (a torch.cuda.Stream, not the null stream)."""
        _check(lib().ephdc_batch_capture(self.handle, _stream(stream)))


def ephdc_batch_create(reqs) -> Batch:
    return Batch(reqs)


def ephdc_score_many(reqs, stream=None) -> None:
    reqs = list(reqs)
    _check(lib().ephdc_score_many(_c_requests(reqs), len(reqs), _stream(stream)))


# ------------------------------------------------------------------ serving loop
class Server:
    """Owns an ephdc_server: tenants, a request queue and a native scheduler thread."""

    STATS = ("submitted", "completed", "rejected", "waiting", "in_flight", "batches", "mean_batch",
             "p50_ms", "p99_ms", "peak_bytes", "budget_bytes", "uptime_s", "failed", "tickets")

    def __init__(self, budget_bytes: int, streams: int = 2, max_batch: int = 0):
        h = C.c_void_p()
        _check(lib().ephdc_server_create(budget_bytes, streams, max_batch, C.byref(h)))
        self.handle = h
        self._keep = {}  # tenant sessions / bases and request buffers stay alive here
        self.pack = False

    def set_packing(self, enable: bool = True) -> None:
        """Requests of one tenant share ciphertexts within a batch (before the first submit)."""
        _check(lib().ephdc_server_set_packing(self.handle, 1 if enable else 0))
        self.pack = bool(enable)

    def result(self, ticket: int):
        """(q_first, n_ct) of a done request: where its queries sit in its output."""
        a, b = C.c_uint32(), C.c_uint32()
        _check(lib().ephdc_server_result(self.handle, ticket, C.byref(a), C.byref(b)))
        return a.value, b.value

    def add_tenant(self, session: "Session", d_base) -> int:
        p = session.prm
        t = C.c_uint32()
        _check(lib().ephdc_server_add_tenant(self.handle, session.handle, _dptr(d_base, p.F * p.D), C.byref(t)))
        self._keep[("tenant", t.value)] = (session, d_base)
        return t.value

    def submit(self, tenant: int, d_x, Q: int, d_score_ct, stream=None) -> int:
        """Queue a request; its kernels run after the work queued so far on `stream` (the
        current stream by default), which may still be writing d_x."""
        session = self._keep[("tenant", tenant)][0] if ("tenant", tenant) in self._keep else None
        if session is None:
            raise EphdcError(ERR_ARG, "unknown tenant")
        p = session.prm
        _, _, out_bytes = _sizes(session, Q)
        if self.pack:
            out_bytes += 2 * p.L * p.N * 4
        tk = C.c_uint64()
        _check(lib().ephdc_server_submit(self.handle, tenant, _dptr(d_x, Q * p.F), Q, _dptr(d_score_ct, out_bytes),
                                         _stream(stream), C.byref(tk)))
        self._keep[("req", tk.value)] = (d_x, d_score_ct)
        return tk.value

    def release(self, ticket: int) -> None:
        """Forget a finished ticket (and drop this wrapper's references to its tensors)."""
        _check(lib().ephdc_server_release(self.handle, ticket))
        self._keep.pop(("req", ticket), None)

    def query(self, ticket: int):
        """(state, (t_submit, t_admit, t_done)); state 0 waiting, 1 in flight, 2 done, <0 failed."""
        st = C.c_int32()
        tm = (C.c_double * 3)()
        _check(lib().ephdc_server_query(self.handle, ticket, C.byref(st), tm))
        return st.value, (tm[0], tm[1], tm[2])

    def wait(self, ticket: int = 0, timeout_s: float = 0.0) -> None:
        _check(lib().ephdc_server_wait(self.handle, ticket, timeout_s))

    def stats(self) -> dict:
        out = (C.c_double * 14)()
        _check(lib().ephdc_server_stats(self.handle, out))
        return {k: out[i] for i, k in enumerate(self.STATS)}

    def close(self) -> None:
        if self.handle:
            _check(lib().ephdc_server_destroy(self.handle))
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
