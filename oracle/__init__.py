"""CPU oracle for EP-HDC client-side encrypted HDC inference.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
CPU statement of what the hot path computes.  Only the test suite, the smoke
check and the benchmark's CPU-baseline leg may import it; the library and its
Python binding never do, and nothing here is shared with the HIP code.

Precision: every value is an exact integer (numpy int64 for residues below
2^30, Python big integers for anything wider, e.g. CRT over the full modulus).

Modules, each citing the passage of the paper it restates:
  arith     primality, roots of unity, modular inverses (number theory helpers)
  prng      SplitMix64 in counter form and the three samplers
  ntt       negacyclic transform by evaluation, and polynomial products
  slots     SIMD slot map mod t: Encode / Decode (Preliminary: packing)
  hdc       random-projection encoding and binarisation (Preliminary: HDC)
  layout    EP-HDC slot packing of class and query hypervectors
  bfv       BFV key generation, encryption, decryption, ct x pt MAC,
            Galois automorphisms and hybrid key switching
  pipeline  the whole client-side path: queries -> encrypted score ciphertexts
  dmax      findDmax of the design-space exploration (Algorithm 1): the
            largest dimension whose encrypted dot product still decrypts
  hog       the detection front end: sliding windows over a frame and each
            window's HOG feature map (integer reading of Dalal-Triggs HOG)

Variants (BGV/BFV-aware quantisation and the noise study): any prime plaintext
modulus t = 1 (mod 2N); the schemes BFV, BFV with rounded scaling, and BGV; and
the scaling op (multiply by (2^s)^-1 mod t after every g accumulations).

Parity status: every function is pinned by tests under tests/ against
closed forms, brute force on tiny inputs, invariants or published values.
The key-switching output bits are pinned only through decryption
(a rotated, correctly decrypting ciphertext) and the stated formulas; there
is no published worked example of them.
"""
from . import arith, prng, ntt, slots, hdc, layout, bfv, pipeline, dmax, hog  # noqa: F401
from .params import Params, default_primes  # noqa: F401
