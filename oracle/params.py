"""BFV + HDC parameter set of the oracle (test infrastructure only).

Symbols follow the paper's table of symbols: N is the polynomial degree (the
number of SIMD slots), t the plaintext modulus, D the hypervector dimension
and k (here K) the number of classes.  The ciphertext modulus is a product of
NTT-friendly primes (the paper leaves the modulus chain to its HE library);
the reading used here is: L primes q_l < 2^30 with q_l = 1 (mod 2N), passed in
explicitly, plus alpha special primes used only inside key switching.

Packing (EP-HDC, client-side HE): each query HV element goes to its own
plaintext and is replicated k times, so one ciphertext carries floor(N/k)
queries and D model ciphertexts are needed (Analysis / proposed method).
The fold factor r generalises this: r consecutive dimensions share one
ciphertext in r blocks of W = N/(2r) slots per row, and log2(r)
rotate-and-sum steps fold the blocks together.  r = 1 is the paper's packing.

Slot layout (the paper never fixes which slots a query occupies): "contiguous"
puts the K copies of a query in K consecutive slots of a row (B = floor(N/k),
the paper's batch size); "subring" puts them on one orbit of the subgroup
{h = 1 (mod 2N/K')} of Z_2N^* acting on the slot exponents, K' the power of two
at or above K, so that every query plaintext lies in Z_t[X^K'] (the K' - K extra
slots of an orbit carry the query value against zero model classes) and one
ciphertext holds B = N/(K' r) queries (layout.py states the slot map and the
Galois elements of its rotations).

The plaintext modulus t is any prime with t = 1 (mod 2N) (the paper sweeps
log2 t; its optimised settings use log2 t = 16 and 17, optimisation table).
The scheme is BFV (the paper's choice) or BGV (its comparison in the noise
study).  HE-aware quantisation (BGV/BFV-aware quantisation): with
scale_every = g > 0 the accumulator is multiplied by the inverse of
2^scale_shift mod t after every g ciphertext additions, which divides the
plaintext by 2^scale_shift whenever it is divisible.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from math import prod

from .arith import is_prime

T_DEFAULT = 65537


def default_primes(N: int, count: int, skip: int = 0, bound: int = 1 << 30) -> list[int]:
    """The `count` largest primes q < bound with q = 1 (mod 2N), after skipping `skip`, descending."""
    out = []
    k = (bound - 2) // (2 * N)
    while len(out) < count + skip:
        q = k * 2 * N + 1
        if q < bound and is_prime(q):
            out.append(q)
        k -= 1
    return out[skip:]


@dataclass(frozen=True)
class Params:
    N: int
    q: tuple
    t: int = T_DEFAULT
    F: int = 512
    D: int = 2048
    K: int = 2
    r: int = 1
    p: tuple = field(default_factory=tuple)  # special primes (key switching only)
    dnum: int = 0
    qbits: int = 1          # 1: binarise; 2..8: clamp(H >> qshift) to qbits signed bits
    qshift: int = 0
    scheme: str = "bfv"     # "bfv", "bfv-r" (rounded scaling) or "bgv"
    scale_every: int = 0    # g: scale after every g accumulations (0: never)
    scale_shift: int = 0    # s: the scale is the inverse of 2^s mod t
    layout: str = "contiguous"  # "contiguous" or "subring" (see the module docstring)

    # ---- derived sizes
    @property
    def L(self) -> int:
        return len(self.q)

    @property
    def alpha(self) -> int:
        return len(self.p)

    @property
    def W(self) -> int:
        """Block width: slots per block per row."""
        return self.N // (2 * self.r)

    @property
    def Kp(self) -> int:
        """Class slots per query: K (contiguous) or the power of two at or above K (subring)."""
        if self.layout == "subring":
            return 1 << (self.K - 1).bit_length()
        return self.K

    @property
    def Bq(self) -> int:
        """Queries per row of one ciphertext (contiguous layout)."""
        return self.W // self.K

    @property
    def n(self) -> int:
        """Orbits of the subring layout (N/K'): the length of its query plaintexts in X^K'."""
        return self.N // self.Kp

    @property
    def B(self) -> int:
        """Queries per ciphertext (two rows of Bq, or N/(K' r) groups of r orbits)."""
        if self.layout == "subring":
            return self.n // self.r
        return 2 * self.Bq

    @property
    def M(self) -> int:
        """Number of model ciphertexts."""
        return -(-self.D // self.r)

    def groups(self, Qn: int) -> int:
        return -(-Qn // self.B)

    @property
    def Qmod(self) -> int:
        return prod(self.q)

    @property
    def Pmod(self) -> int:
        return prod(self.p)

    @property
    def Delta(self) -> int:
        return self.Qmod // self.t

    @property
    def scale_const(self) -> int:
        """Centred representative of (2^s)^-1 mod t: the plaintext scalar of the scaling op."""
        c = pow(2, -self.scale_shift, self.t)
        return c - self.t if c > self.t // 2 else c

    @property
    def log2r(self) -> int:
        return self.r.bit_length() - 1

    @property
    def digit_size(self) -> int:
        return -(-self.L // self.dnum) if self.dnum else 0

    def digits(self) -> list[list[int]]:
        """Limb index sets I_j of the key-switching digits."""
        a = self.digit_size
        return [list(range(j * a, min((j + 1) * a, self.L))) for j in range(self.dnum)]

    def validate(self) -> None:
        N = self.N
        assert N >= 8 and N & (N - 1) == 0
        assert is_prime(self.t) and self.t % (2 * N) == 1
        assert self.scheme in ("bfv", "bfv-r", "bgv")
        assert self.scheme != "bgv" or self.r == 1  # BGV key switching is not implemented
        assert self.scale_every >= 0 and 0 <= self.scale_shift < 32
        allp = list(self.q) + list(self.p)
        assert len(set(allp)) == len(allp)
        for x in allp:
            assert x < (1 << 30) and x % (2 * N) == 1 and is_prime(x)
        assert self.r >= 1 and self.r & (self.r - 1) == 0
        assert self.layout in ("contiguous", "subring")
        assert self.layout == "contiguous" or self.B >= 2
        assert self.Bq >= 1
        if self.r > 1:
            assert self.dnum >= 1 and self.alpha >= 1
