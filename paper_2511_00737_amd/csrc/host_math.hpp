// Host-side number theory, sampling and negacyclic transforms for the EP-HDC library.
//
// Used by the server-side calls (key generation, model encryption, decryption) and to
// build the device twiddle tables.  Everything is exact integer arithmetic on residues
// below 2^30 (products fit in 64 bits).
#pragma once

#include <array>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

namespace ephdc {

inline uint64_t mulmod64(uint64_t a, uint64_t b, uint64_t m) {
  return (uint64_t)((unsigned __int128)a * b % m);
}

inline uint64_t powmod64(uint64_t b, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  b %= m;
  while (e) {
    if (e & 1) r = mulmod64(r, b, m);
    b = mulmod64(b, b, m);
    e >>= 1;
  }
  return r;
}

// Deterministic Miller-Rabin for 64-bit integers (bases 2..37 suffice below 3.3e24).
inline bool is_prime_u64(uint64_t n) {
  static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return false;
  for (uint64_t p : bases) {
    if (n % p == 0) return n == p;
  }
  uint64_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) { d >>= 1; ++s; }
  for (uint64_t a : bases) {
    uint64_t x = powmod64(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool composite = true;
    for (int i = 1; i < s; ++i) {
      x = mulmod64(x, x, n);
      if (x == n - 1) { composite = false; break; }
    }
    if (composite) return false;
  }
  return true;
}

inline uint32_t inv_mod(uint64_t a, uint64_t m) {  // m prime
  return (uint32_t)powmod64(a % m, m - 2, m);
}

// Smallest generator of Z_q^* (q prime), then g^((q-1)/order).
inline uint32_t root_of_unity(uint32_t order, uint32_t q) {
  std::vector<uint64_t> f;
  uint64_t n = q - 1;
  for (uint64_t d = 2; d * d <= n; ++d) {
    if (n % d == 0) {
      f.push_back(d);
      while (n % d == 0) n /= d;
    }
  }
  if (n > 1) f.push_back(n);
  for (uint64_t g = 2;; ++g) {
    bool gen = true;
    for (uint64_t p : f) {
      if (powmod64(g, (q - 1) / p, q) == 1) { gen = false; break; }
    }
    if (gen) return (uint32_t)powmod64(g, (q - 1) / order, q);
  }
}

inline uint32_t bitrev(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) { r = (r << 1) | (x & 1); x >>= 1; }
  return r;
}

inline int ilog2(uint32_t x) {
  int b = 0;
  while ((1u << b) < x) ++b;
  return b;
}

// ------------------------------------------------------------------ SplitMix64, counter form
// Stream (seed, tag) has state s0 = seed ^ (tag << 32); draw n is the published SplitMix64
// finaliser applied to s0 + (n+1)*0x9E3779B97F4A7C15 (Steele, Lea, Flood, OOPSLA 2014).
enum : uint64_t { TAG_SECRET = 4, TAG_ENCRYPT = 5, TAG_GALOIS = 6 };

struct Stream {
  uint64_t s0;
  Stream(uint64_t seed, uint64_t tag) : s0(seed ^ (tag << 32)) {}
  uint64_t operator()(uint64_t n) const {
    uint64_t z = s0 + (n + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
};

// Discrete Gaussian sigma = 3.2 on [-19, 19]: T_k = round(2^53 * cumulative mass), T_19 = 2^53.
inline std::array<uint64_t, 39> gaussian_cdt() {
  const double sigma = 3.2;
  double rho[39];
  for (int i = -19; i <= 19; ++i) rho[i + 19] = std::exp(-(double)(i * i) / (2.0 * sigma * sigma));
  double total = 0.0;
  for (int i = 0; i < 39; ++i) total += rho[i];
  std::array<uint64_t, 39> T{};
  double acc = 0.0;
  for (int i = 0; i < 39; ++i) {
    acc += rho[i];
    T[i] = (uint64_t)std::nearbyint(acc / total * 9007199254740992.0);
  }
  T[38] = 1ull << 53;
  return T;
}

inline int gaussian_sample(uint64_t u, const std::array<uint64_t, 39>& T) {
  uint64_t x = u >> 11;
  int k = 0;
  while (x >= T[k]) ++k;  // T[38] = 2^53 > x always
  return k - 19;
}

// ------------------------------------------------------------------ host negacyclic transform
// Forward (Cooley-Tukey, natural in, bit-reversed out): position x holds a(w^(2*brev(x)+1)).
// Inverse (Gentleman-Sande) undoes it, including the 1/N factor.  Shoup multiplication
// with precomputed w' = floor(w * 2^32 / m); lazy values stay below 4m < 2^32.
struct HostNtt {
  uint32_t N = 0, m = 0, w = 0;
  int logn = 0;
  std::vector<uint32_t> fw, fwp, iw, iwp;  // bit-reversed powers of w and w^-1, with Shoup companions
  uint32_t ninv = 0, ninvp = 0;

  HostNtt() = default;
  HostNtt(uint32_t N_, uint32_t m_, uint32_t w_) : N(N_), m(m_), w(w_), logn(ilog2(N_)) {
    fw.resize(N); fwp.resize(N); iw.resize(N); iwp.resize(N);
    uint32_t winv = inv_mod(w, m);
    for (uint32_t k = 0; k < N; ++k) {
      uint32_t e = bitrev(k, logn);
      fw[k] = (uint32_t)powmod64(w, e, m);
      iw[k] = (uint32_t)powmod64(winv, e, m);
      fwp[k] = shoup(fw[k]);
      iwp[k] = shoup(iw[k]);
    }
    ninv = inv_mod(N, m);
    ninvp = shoup(ninv);
  }
  uint32_t shoup(uint32_t x) const { return (uint32_t)(((uint64_t)x << 32) / m); }
  uint32_t mul_shoup(uint32_t a, uint32_t x, uint32_t xp) const {  // result in [0, 2m)
    uint32_t qh = (uint32_t)(((uint64_t)a * xp) >> 32);
    return a * x - qh * m;
  }
  void forward(uint32_t* a) const {  // in [0, m) -> out [0, m)
    const uint32_t m2 = 2 * m;
    for (int s = 0; s < logn; ++s) {
      uint32_t half = N >> (s + 1);
      for (uint32_t blk = 0; blk < (1u << s); ++blk) {
        uint32_t wv = fw[(1u << s) + blk], wpv = fwp[(1u << s) + blk];
        uint32_t* x = a + blk * 2 * half;
        for (uint32_t j = 0; j < half; ++j) {
          uint32_t X = x[j] >= m2 ? x[j] - m2 : x[j];
          uint32_t T = mul_shoup(x[j + half], wv, wpv);
          x[j] = X + T;
          x[j + half] = X - T + m2;
        }
      }
    }
    for (uint32_t i = 0; i < N; ++i) {
      uint32_t v = a[i];
      if (v >= m2) v -= m2;
      if (v >= m) v -= m;
      a[i] = v;
    }
  }
  void inverse(uint32_t* a) const {  // in [0, m) -> out [0, m)
    const uint32_t m2 = 2 * m;
    for (int s = logn - 1; s >= 0; --s) {
      uint32_t half = N >> (s + 1);
      for (uint32_t blk = 0; blk < (1u << s); ++blk) {
        uint32_t wv = iw[(1u << s) + blk], wpv = iwp[(1u << s) + blk];
        uint32_t* x = a + blk * 2 * half;
        for (uint32_t j = 0; j < half; ++j) {
          uint32_t U = x[j], V = x[j + half];
          uint32_t S = U + V;
          if (S >= m2) S -= m2;
          x[j] = S;
          x[j + half] = mul_shoup(U - V + m2, wv, wpv);
        }
      }
    }
    for (uint32_t i = 0; i < N; ++i) {
      uint32_t v = mul_shoup(a[i], ninv, ninvp);
      if (v >= m) v -= m;
      a[i] = v;
    }
  }
};

// Primes used by the library (validated externally): the `count` largest primes below 2^30
// congruent to 1 mod 2N, after skipping `skip` of them, in descending order.
inline std::vector<uint32_t> default_primes(uint32_t N, uint32_t count, uint32_t skip) {
  std::vector<uint32_t> out;
  uint64_t step = 2ull * N;
  uint64_t k = ((1ull << 30) - 2) / step;
  while (out.size() < (size_t)count + skip && k > 0) {
    uint64_t q = k * step + 1;
    if (q < (1ull << 30) && is_prime_u64(q)) out.push_back((uint32_t)q);
    --k;
  }
  if (out.size() < (size_t)count + skip) return {};
  return std::vector<uint32_t>(out.begin() + skip, out.end());
}

}  // namespace ephdc
