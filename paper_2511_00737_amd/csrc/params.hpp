// Parameter validation and the EP-HDC slot layout, shared by the host-side crypto and the
// session code of the library.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ephdc.h"
#include "host_math.hpp"

namespace ephdc {

// Thread-local error message behind ephdc_last_error().
void set_error(const std::string& msg);
ephdc_status fail(ephdc_status st, const std::string& msg);

struct ParamSet {
  uint32_t N = 0, L = 0, alpha = 0, dnum = 0, t = 0, F = 0, D = 0, K = 0, r = 0;
  uint32_t qbits = 1, qshift = 0;
  uint32_t scheme = EPHDC_BFV;              // EPHDC_BFV, EPHDC_BFV_ROUNDED or EPHDC_BGV
  uint32_t scale_every = 0, scale_shift = 0;  // HE-aware scaling: g and s (g = 0: off)
  uint32_t layout = EPHDC_LAYOUT_CONTIGUOUS;
  int logn = 0;
  std::vector<uint32_t> q, p;  // ciphertext primes, special primes

  uint32_t W() const { return N / (2 * r); }           // block width per row
  bool subring() const { return layout == EPHDC_LAYOUT_SUBRING; }
  uint32_t Kp() const { return subring() ? 1u << ilog2(K) : K; }  // class slots per query (ilog2 rounds up)
  uint32_t Bq() const { return W() / K; }              // queries per row (contiguous layout)
  uint32_t n() const { return N / Kp(); }               // orbits of the subring layout
  uint32_t B() const { return subring() ? n() / r : 2 * Bq(); }  // queries per ciphertext
  uint32_t M() const { return (D + r - 1) / r; }       // model ciphertexts
  uint32_t G(uint32_t Q) const { return (Q + B() - 1) / B(); }
  uint32_t log2r() const { return (uint32_t)ilog2(r); }
  uint32_t digit_size() const { return dnum ? (L + dnum - 1) / dnum : 0; }
  uint32_t nmod() const { return L + alpha; }
  uint32_t modulus(uint32_t i) const { return i < L ? q[i] : p[i - L]; }
  // Scaling op: full blocks of scale_every model ciphertexts (each followed by one scaling)
  // and the plaintext scalar, the centred representative of (2^scale_shift)^-1 mod t.
  uint32_t scale_blocks() const { return scale_every ? M() / scale_every : 0; }
  int64_t scale_const() const {
    const uint64_t c = powmod64(inv_mod(2, t), scale_shift, t);
    return c > t / 2 ? (int64_t)c - (int64_t)t : (int64_t)c;
  }

  // Validates and fills from the public struct; returns EPHDC_OK or an error (message set).
  ephdc_status load(const ephdc_params* prm);
};

// Odd exponent e_s in [0, 2N) of the evaluation point zeta^(e_s) of slot s:
// 3^s mod 2N for s < N/2, and -3^(s-N/2) mod 2N for the second half.
std::vector<uint32_t> slot_exponents(uint32_t N);

// Position of slot s in the bit-reversed evaluation order used by every transform of the
// library (position x holds the value at zeta^(2*brev(x)+1)).
std::vector<uint32_t> slot_positions(uint32_t N);

// For every transform position x: which query slot feeds it, packed as
// (query index inside the group) | (block u << 16), or 0xFFFFFFFF for a zero slot.
std::vector<uint32_t> query_scatter_table(const ParamSet& P);

// Slot index of (row rho, block u, query ql, class c).
inline uint32_t slot_index(const ParamSet& P, uint32_t rho, uint32_t u, uint32_t ql, uint32_t c) {
  return rho * (P.N / 2) + u * P.W() + ql * P.K + c;
}

// Slots of the subring layout.  With n = N/K' orbits of H = {h = 1 (mod 2n)} (orbit y: the
// exponents = 2*brev(y) + 1 mod 2n, position y of the n-point transform), block v of query
// ql < B = n/r takes orbit ql*r + v, and class c < K' of it is the exponent
// gamma^u * (e_ql + 2n*c) mod 2N, with gamma = 1 + 2n/r, e_ql = 2*brev(ql) + 1 over log2 B
// bits and u < r the power for which gamma^u * e_ql lies in orbit ql*r + v (u = 0 at
// v = 0).  The Galois elements gamma^(2^i) of rotate-and-sum then gather the r blocks of
// each class into block 0.
struct SubringSlots {
  std::vector<uint32_t> of_exp;  // odd exponent -> slot
  std::vector<uint32_t> u_of;    // [ql * r + v] -> u
  std::vector<uint64_t> gpow;    // gamma^u mod 2N, u < r
  uint32_t N = 0, n = 0, B = 0, r = 1;
  int logb = 0;
  explicit SubringSlots(const ParamSet& P);
  uint32_t slot_of(uint32_t ql, uint32_t c, uint32_t v = 0) const {
    const uint64_t e = (2ull * bitrev(ql, logb) + 1 + 2ull * n * c) % (2ull * N);
    return of_exp[gpow[u_of[(size_t)ql * r + v]] * e % (2ull * N)];
  }
};

// The model ciphertexts of ephdc_encrypt_model for a validated parameter set: class
// hypervectors int8 [K][D] -> uint32 [M][2][L][N], coefficient domain.
ephdc_status encrypt_model_host(const ParamSet& P, const int8_t* sk, const int8_t* class_hv, uint64_t seed,
                                uint32_t* model_ct);

// Galois element of rotate-and-sum step i: 3^(W * 2^i) mod 2N (contiguous layout: rotates
// each row by W * 2^i slots), or gamma^(2^i) mod 2N with gamma = 1 + 2n/r (subring layout).
inline uint32_t galois_element(const ParamSet& P, uint32_t i) {
  if (P.subring()) return (uint32_t)powmod64(1 + 2 * P.n() / P.r, 1ull << i, 2ull * P.N);
  return (uint32_t)powmod64(3, (uint64_t)P.W() << i, 2ull * P.N);
}

}  // namespace ephdc
