"""BFV over an RNS modulus, as used by EP-HDC (oracle; test infrastructure only).

The paper runs BFV (chosen over BGV for its noise behaviour, noise results)
through its HE library.  What the client-side method needs is stated in the
proposed method: the server encrypts the class hypervectors once with its
secret key and later decrypts the score ciphertexts; the client multiplies
plaintext query encodings into the encrypted model and adds (MulCP, AddCC).
The scheme details below are textbook BFV; where the paper is silent the
readings are:

* Ciphertext modulus Q = prod q_l (L primes), Delta = floor(Q / t).
* Secret-key encryption of mu (coefficients in [0, t)):
  ct = ([-a*s + e + Delta*mu]_Q, a), a uniform per limb, e Gaussian.  Limb l
  carries (Delta mod q_l) * mu.  Randomness: stream tag 5, ciphertext m uses
  draws from m*(L+1)*N: a for limb 0..L-1 (N draws each, coefficient order),
  then e (N draws).
* Plaintext of a query slot vector: mu = Encode(v), lifted to integers by the
  centred representative in (-t/2, t/2] and reduced into every limb.
* Decryption: x = [c0 + c1*s]_Q by exact CRT, mu = floor((2t*x + Q) / (2Q)) mod t.
* BFV with rounded scaling ("bfv-r"): the message term is round(Q*mu/t)
  instead of Delta*mu (the scaling many BFV libraries use); everything else,
  decryption included, is as in BFV.  Under Delta*mu a ct x pt product carries
  the extra error (Q mod t) * floor(mu*p/t), which the rounded scaling avoids.
* BGV (the noise study's comparison scheme; the paper keeps BFV): the message
  sits in the low bits and the error is scaled by t instead:
  ct = ([-a*s + t*e + mu~]_Q, a) with mu~ the centred representative of mu,
  and decryption is mu = ([c0 + c1*s]_Q, centred) mod t.  The ct x pt product,
  the accumulation and the scaling op are the same ring operations as in BFV.
* HE-aware scaling (BGV/BFV-aware quantisation): with g = scale_every > 0,
  after every g additions of the MAC the accumulator is multiplied by the
  plaintext scalar c = centred (2^s)^-1 mod t, so the plaintext becomes
  m * (2^s)^-1 mod t: the exact quotient m / 2^s whenever 2^s divides m.
* Rotations (fold factor r > 1 only; the paper's own packing needs none):
  the Galois automorphism X -> X^g, then hybrid key switching with dnum digits
  over the extended basis PQ (fast base conversion up, inner product with the
  switching keys, fast base conversion down and division by P).
"""
from __future__ import annotations

import math

import numpy as np

from . import ntt, prng, slots
from .arith import inv
from .layout import model_slots, query_slots, subring_gamma
from .params import Params


# --------------------------------------------------------------------------- keys
def secret_key(P: Params, seed: int) -> np.ndarray:
    """Ternary secret s, int64 [N] in {-1, 0, 1} (stream tag 4, draws 0..N-1)."""
    return prng.ternary(prng.draws(seed, prng.TAG_SECRET, 0, P.N))


def _mask_and_error(P: Params, moduli, seed: int, tag: int, start: int):
    """Uniform a (one poly per modulus) then one Gaussian error poly, from consecutive draws."""
    N = P.N
    a = np.stack([prng.uniform_mod(prng.draws(seed, tag, start + l * N, N), m)
                  for l, m in enumerate(moduli)])
    e = prng.gaussian(prng.draws(seed, tag, start + len(moduli) * N, N))
    return a, e


def encrypt(P: Params, s: np.ndarray, mu: np.ndarray, seed: int, index: int) -> np.ndarray:
    """Ciphertext int64 [2][L][N] of plaintext mu, using the draws reserved for ciphertext `index`."""
    L, N = P.L, P.N
    a, e = _mask_and_error(P, P.q, seed, prng.TAG_ENCRYPT, index * (L + 1) * N)
    ct = np.empty((2, L, N), dtype=np.int64)
    for l, q in enumerate(P.q):
        as_ = ntt.polymul(a[l], s % q, q)
        ct[0, l] = (-as_ + _message_term(P, e, mu, q)) % q
        ct[1, l] = a[l]
    return ct


def _message_term(P: Params, e: np.ndarray, mu: np.ndarray, q: int) -> np.ndarray:
    """e + Delta*mu (BFV), e + round(Q*mu/t) (BFV with rounded scaling) or t*e + centred(mu)
    (BGV), reduced mod q.  round(Q*mu/t) = Delta*mu + floor((2*r*mu + t) / (2t)), r = Q mod t."""
    if P.scheme == "bgv":
        return (P.t * e + slots.centered(mu, P.t)) % q
    out = (e + (P.Delta % q) * mu) % q
    if P.scheme == "bfv-r":
        r = P.Qmod % P.t
        out = (out + (2 * r * mu + P.t) // (2 * P.t)) % q
    return out


def model_plaintext(P: Params, C: np.ndarray, m: int) -> np.ndarray:
    """mu_m = Encode(slot vector of model ciphertext m), coefficients in [0, t)."""
    return slots.encode(model_slots(P, C, m), P.t)


def encrypt_model(P: Params, s: np.ndarray, C: np.ndarray, seed: int, ms=None,
                  chunk: int = 256) -> np.ndarray:
    """Model ciphertexts int64 [len(ms)][2][L][N] (all M when ms is None).

    Identical to calling encrypt() per ciphertext; consecutive ciphertexts are
    processed together because their draw windows are adjacent.
    """
    ms = list(range(P.M)) if ms is None else list(ms)
    L, N = P.L, P.N
    out = np.empty((len(ms), 2, L, N), dtype=np.int64)
    for i0 in range(0, len(ms), chunk):
        sel = ms[i0:i0 + chunk]
        mu = slots.encode(np.stack([model_slots(P, C, m) for m in sel]), P.t)
        u = np.stack([prng.draws(seed, prng.TAG_ENCRYPT, m * (L + 1) * N, (L + 1) * N)
                      for m in sel]).reshape(len(sel), L + 1, N)
        e = prng.gaussian(u[:, L])
        for l, q in enumerate(P.q):
            a = prng.uniform_mod(u[:, l], q)
            as_ = ntt.polymul(a, (s % q)[None, :], q)
            out[i0:i0 + len(sel), 0, l] = (-as_ + _message_term(P, e, mu, q)) % q
            out[i0:i0 + len(sel), 1, l] = a
    return out


def phase(P: Params, s: np.ndarray, ct: np.ndarray) -> np.ndarray:
    """x = [c0 + c1*s]_Q in [0, Q) as Python integers (exact CRT), object [N]."""
    Qm = P.Qmod
    x = [(ct[0, l] + ntt.polymul(ct[1, l], s % q, q)) % q for l, q in enumerate(P.q)]
    acc = np.zeros(P.N, dtype=object)
    for l, q in enumerate(P.q):
        Qhat = Qm // q
        acc = acc + x[l].astype(object) * ((Qhat * inv(Qhat, q)) % Qm)
    return acc % Qm


def decrypt(P: Params, s: np.ndarray, ct: np.ndarray) -> np.ndarray:
    """mu in [0, t) of a ciphertext int64 [2][L][N]."""
    Qm, t = P.Qmod, P.t
    acc = phase(P, s, ct)
    if P.scheme == "bgv":
        mu = np.array([(int(v) - Qm if int(v) > Qm // 2 else int(v)) % t for v in acc], dtype=np.int64)
        return mu
    mu = (2 * t * acc + Qm) // (2 * Qm) % t
    return mu.astype(np.int64)


def noise_margin_bits(P: Params, s: np.ndarray, ct: np.ndarray, mu: np.ndarray) -> float:
    """Bits left before decryption of ct would stop returning mu (the plaintext it should hold).

    BFV: log2(Delta/2) - log2 max |x - Delta*mu| (centred mod Q).  BGV: log2(Q/2) - log2 max |x|
    (centred mod Q), which measures the integer phase only while it has not wrapped, so a
    ciphertext that no longer decrypts to mu gets -inf.  x = [c0 + c1*s]_Q.
    """
    Qm = P.Qmod
    acc = phase(P, s, ct)
    if P.scheme == "bgv":
        err = [int(v) - Qm if int(v) > Qm // 2 else int(v) for v in acc]
        if any((e - int(m)) % P.t for e, m in zip(err, mu)):
            return -math.inf
        bound = Qm / 2
    else:
        err = [(int(v) - int(m) * P.Delta) % Qm for v, m in zip(acc, mu)]
        err = [v - Qm if v > Qm // 2 else v for v in err]
        bound = P.Delta / 2
    mx = max(abs(v) for v in err)
    return math.log2(bound) - (math.log2(mx) if mx else 0.0)


def noise_bits(P: Params, s: np.ndarray, ct: np.ndarray) -> float:
    """log2 of max |x - Delta*mu| over coefficients (the invariant noise of a ciphertext)."""
    Qm = P.Qmod
    x = [(ct[0, l] + ntt.polymul(ct[1, l], s % q, q)) % q for l, q in enumerate(P.q)]
    acc = np.zeros(P.N, dtype=object)
    for l, q in enumerate(P.q):
        Qhat = Qm // q
        acc = acc + x[l].astype(object) * ((Qhat * inv(Qhat, q)) % Qm)
    acc = acc % Qm
    mu = (2 * P.t * acc + Qm) // (2 * Qm) % P.t
    err = (acc - mu * P.Delta) % Qm
    err = [int(v) - Qm if int(v) > Qm // 2 else int(v) for v in err]
    mx = max(abs(v) for v in err)
    return math.log2(mx) if mx else 0.0


# --------------------------------------------------------------------------- ct x pt
def lift_centered(mu: np.ndarray, t: int) -> np.ndarray:
    """Integer representative of mu mod t in (-t/2, t/2]."""
    return slots.centered(mu, t)


def query_plaintext(P: Params, h: np.ndarray, g: int, m: int) -> np.ndarray:
    """Lifted plaintext (int64 [N], values in [-(t-1)/2, (t-1)/2]) of query group g, dimension block m."""
    return lift_centered(slots.encode(query_slots(P, h, g, m), P.t), P.t)


def mul_plain(P: Params, ct: np.ndarray, p: np.ndarray, moduli=None) -> np.ndarray:
    moduli = P.q if moduli is None else moduli
    out = np.empty_like(ct)
    for c in range(ct.shape[0]):
        for l, q in enumerate(moduli):
            out[c, l] = ntt.polymul(ct[c, l], p % q, q)
    return out


def mul_scalar(P: Params, ct: np.ndarray, c: int) -> np.ndarray:
    """ct * c for an integer plaintext scalar c (each residue times c mod q_l)."""
    out = np.empty_like(ct)
    for l, q in enumerate(P.q):
        out[:, l] = ct[:, l] * (c % q) % q
    return out


def mac(P: Params, model_ct: np.ndarray, h: np.ndarray, g: int, chunk: int = 256) -> np.ndarray:
    """acc_g = sum_m ct_m * p_(g,m) over all M model ciphertexts, int64 [2][L][N].

    Products are taken in the evaluation domain of each limb (ntt.forward) and
    summed there; within a run of additions the order of m does not matter (the
    sums are exact).  With scale_every = g_s > 0 the additions come in blocks of
    g_s model ciphertexts, and after every complete block the accumulator is
    multiplied by the scaling scalar (the multiplication commutes with the
    transform, so it is applied in the evaluation domain).
    """
    L, N, t = P.L, P.N, P.t
    acc = np.zeros((2, L, N), dtype=np.int64)
    blk = P.scale_every if P.scale_every else P.M
    for b0 in range(0, P.M, blk):
        b1 = min(P.M, b0 + blk)
        for m0 in range(b0, b1, chunk):
            ms = range(m0, min(b1, m0 + chunk))
            v = np.stack([query_slots(P, h, g, m) for m in ms])
            pt = lift_centered(slots.encode(v, t), t)
            for l, q in enumerate(P.q):
                ptf = ntt.forward(pt % q, q)
                for c in range(2):
                    ctf = ntt.forward(model_ct[m0:m0 + len(ms), c, l], q)
                    acc[c, l] = (acc[c, l] + (ctf * ptf % q).sum(axis=0)) % q
        if P.scale_every and b1 - b0 == P.scale_every:
            acc = mul_scalar(P, acc, P.scale_const)
    out = np.empty_like(acc)
    for l, q in enumerate(P.q):
        for c in range(2):
            out[c, l] = ntt.inverse(acc[c, l], q)
    return out


# --------------------------------------------------------------------------- automorphisms
def _automorphism_map(N: int, g: int):
    j = np.arange(N)
    dst = j * g % (2 * N)
    neg = dst >= N
    return np.where(neg, dst - N, dst), neg


def automorphism_int(a: np.ndarray, g: int) -> np.ndarray:
    """a(X) -> a(X^g) mod X^N + 1 for an integer polynomial: coefficient j goes to j*g mod 2N, negated past N."""
    dst, neg = _automorphism_map(a.shape[-1], g)
    out = np.zeros_like(a)
    out[..., dst] = np.where(neg, -a, a)
    return out


def automorphism(a: np.ndarray, g: int, moduli) -> np.ndarray:
    """The same map on residues: a is int64 [..., len(moduli), N]."""
    dst, neg = _automorphism_map(a.shape[-1], g)
    mods = np.asarray(moduli, dtype=np.int64).reshape((-1, 1))
    out = np.zeros_like(a)
    out[..., dst] = np.where(neg, (-a) % mods, a)
    return out


def galois_elements(P: Params) -> list[int]:
    """Galois elements g_i, i < log2 r, of rotate-and-sum.  Contiguous layout:
    3^(W * 2^i) mod 2N, which rotates each row left by W * 2^i slots.  Subring layout:
    gamma^(2^i) mod 2N with gamma = 1 + 2n/r (layout module docstring)."""
    if P.layout == "subring":
        return [pow(subring_gamma(P), 1 << i, 2 * P.N) for i in range(P.log2r)]
    return [pow(3, P.W << i, 2 * P.N) for i in range(P.log2r)]


def galois_keys(P: Params, s: np.ndarray, seed: int) -> np.ndarray:
    """Switching keys int64 [log2 r][dnum][2][L+alpha][N] (component 0 = b, 1 = a).

    Key (i, j): a uniform over all L+alpha moduli, e Gaussian (stream tag 6,
    draws from ((i*dnum + j) * (L+alpha+1)) * N), and
    b = -a*s + e + G_j * sigma_(g_i)(s), where G_j = P mod q_l for l in digit j
    and 0 on every other modulus (special primes included).
    """
    L, N, A = P.L, P.N, P.alpha
    mods = list(P.q) + list(P.p)
    out = np.empty((P.log2r, P.dnum, 2, L + A, N), dtype=np.int64)
    for i, g in enumerate(galois_elements(P)):
        s_rot = automorphism_int(s, g)
        for j, digit in enumerate(P.digits()):
            a, e = _mask_and_error(P, mods, seed, prng.TAG_GALOIS,
                                   (i * P.dnum + j) * (L + A + 1) * N)
            for l, m in enumerate(mods):
                b = (-ntt.polymul(a[l], s % m, m) + e) % m
                if l in digit:
                    b = (b + (P.Pmod % m) * (s_rot % m)) % m
                out[i, j, 0, l] = b
                out[i, j, 1, l] = a[l]
    return out


def mod_up(P: Params, d: np.ndarray, digit: list[int]) -> np.ndarray:
    """Extend the residues d[l] (l in digit, coefficient domain) to all L+alpha moduli.

    Fast base conversion without correction: for a modulus m outside the
    digit, y_m = sum_i [d_i * (Q_j/q_i)^-1]_(q_i) * (Q_j/q_i mod m) mod m.
    """
    mods = list(P.q) + list(P.p)
    Qj = 1
    for i in digit:
        Qj *= P.q[i]
    tvals = {i: d[i] * (inv(Qj // P.q[i], P.q[i])) % P.q[i] for i in digit}
    y = np.empty((len(mods), P.N), dtype=np.int64)
    for l, m in enumerate(mods):
        if l in digit:
            y[l] = d[l]
        else:
            acc = np.zeros(P.N, dtype=np.int64)
            for i in digit:
                acc = (acc + tvals[i] * ((Qj // P.q[i]) % m)) % m
            y[l] = acc
    return y


def mod_down(P: Params, x: np.ndarray) -> np.ndarray:
    """From PQ down to Q: out_l = (x_(q_l) - conv_P(x_P)) * P^-1 mod q_l (fast base conversion of the P part)."""
    L, A = P.L, P.alpha
    Pm = P.Pmod
    out = np.empty((L, P.N), dtype=np.int64)
    tv = [x[L + k] * inv(Pm // P.p[k], P.p[k]) % P.p[k] for k in range(A)]
    for l, q in enumerate(P.q):
        conv = np.zeros(P.N, dtype=np.int64)
        for k in range(A):
            conv = (conv + tv[k] * ((Pm // P.p[k]) % q)) % q
        out[l] = (x[l] - conv) % q * inv(Pm, q) % q
    return out


def key_switch(P: Params, c1: np.ndarray, ksk: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """(b', a') over Q with b' + a'*s = c1 * s' + small, for ksk = keys of one Galois element."""
    mods = list(P.q) + list(P.p)
    acc = np.zeros((2, len(mods), P.N), dtype=np.int64)
    for j, digit in enumerate(P.digits()):
        y = mod_up(P, c1, digit)
        for c in range(2):
            for l, m in enumerate(mods):
                acc[c, l] = (acc[c, l] + ntt.polymul(y[l], ksk[j, c, l], m)) % m
    return mod_down(P, acc[0]), mod_down(P, acc[1])


def rotate_and_sum(P: Params, ct: np.ndarray, gk: np.ndarray) -> np.ndarray:
    """For i < log2 r: ct <- ct + KeySwitch(sigma_(g_i)(ct)); block 0 then holds the sum of all blocks."""
    ct = ct.copy()
    for i, g in enumerate(galois_elements(P)):
        rot = automorphism(ct, g, P.q)
        b, a = key_switch(P, rot[1], gk[i])
        for l, q in enumerate(P.q):
            ct[0, l] = (ct[0, l] + rot[0, l] + b[l]) % q
            ct[1, l] = (ct[1, l] + a[l]) % q
    return ct
