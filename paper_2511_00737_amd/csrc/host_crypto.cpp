// Server side of EP-HDC: parameter checks, key generation, model encryption and decryption.
//
// The server owns the BFV secret key, encrypts the class hypervectors once and later
// decrypts the score ciphertexts the client returns (proposed method: client-side HE).
// All of it is exact integer arithmetic on the host; the heavy loops run on a pool of
// std::threads, one ciphertext (or key) per task, and every result is independent of
// the thread count because each task draws from its own fixed window of the stream.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <functional>
#include <memory>
#include <thread>

#include "params.hpp"

namespace ephdc {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

ephdc_status fail(ephdc_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

ephdc_status ParamSet::load(const ephdc_params* prm) {
  if (!prm) return fail(EPHDC_ERR_ARG, "params is NULL");
  N = prm->N; L = prm->L; alpha = prm->alpha; dnum = prm->dnum; t = prm->t;
  F = prm->F; D = prm->D; K = prm->K; r = prm->r; qshift = prm->qshift;
  scheme = prm->scheme; scale_every = prm->scale_every; scale_shift = prm->scale_shift;
  layout = prm->layout;
  if (prm->qbits < 1 || prm->qbits > 8) return fail(EPHDC_ERR_PARAMS, "qbits must be in [1, 8]");
  qbits = (uint32_t)prm->qbits;
  if (N < 8 || N > 32768 || (N & (N - 1))) return fail(EPHDC_ERR_PARAMS, "N must be a power of two in [8, 32768]");
  logn = ilog2(N);
  if (L < 1 || L > 16) return fail(EPHDC_ERR_PARAMS, "L must be in [1, 16]");
  if (alpha > 4) return fail(EPHDC_ERR_PARAMS, "alpha must be <= 4");
  if (!prm->q || (alpha && !prm->p)) return fail(EPHDC_ERR_ARG, "prime list is NULL");
  if (t < 257 || !is_prime_u64(t)) return fail(EPHDC_ERR_PARAMS, "t must be a prime >= 257");
  if (t % (2 * N) != 1) return fail(EPHDC_ERR_PARAMS, "t must be 1 mod 2N");
  if ((uint64_t)N * t >= (1ull << 32)) return fail(EPHDC_ERR_PARAMS, "N * t must be below 2^32");
  if (scheme > EPHDC_BGV) return fail(EPHDC_ERR_PARAMS, "scheme must be EPHDC_BFV, EPHDC_BFV_ROUNDED or EPHDC_BGV");
  if (scale_shift > 31) return fail(EPHDC_ERR_PARAMS, "scale_shift must be < 32");
  q.assign(prm->q, prm->q + L);
  p.assign(alpha ? prm->p : prm->q, alpha ? prm->p + alpha : prm->q);
  std::vector<uint32_t> all(q);
  all.insert(all.end(), p.begin(), p.end());
  for (size_t i = 0; i < all.size(); ++i) {
    uint32_t m = all[i];
    if (m >= (1u << 30)) return fail(EPHDC_ERR_PARAMS, "primes must be < 2^30");
    if (m % (2 * N) != 1) return fail(EPHDC_ERR_PARAMS, "prime " + std::to_string(m) + " is not 1 mod 2N");
    if (!is_prime_u64(m)) return fail(EPHDC_ERR_PARAMS, std::to_string(m) + " is not prime");
    if (m == t) return fail(EPHDC_ERR_PARAMS, "primes must differ from t");
    for (size_t j = 0; j < i; ++j)
      if (all[j] == m) return fail(EPHDC_ERR_PARAMS, "primes must be distinct");
  }
  if (K < 1 || D < 1 || F < 1) return fail(EPHDC_ERR_PARAMS, "F, D, K must be positive");
  if (r < 1 || (r & (r - 1))) return fail(EPHDC_ERR_PARAMS, "r must be a power of two");
  if (N / (2 * r) < K) return fail(EPHDC_ERR_PARAMS, "N/(2r) must be >= K (at least one query per row)");
  if (qshift > 31) return fail(EPHDC_ERR_PARAMS, "qshift must be <= 31");
  if (layout > EPHDC_LAYOUT_SUBRING) return fail(EPHDC_ERR_PARAMS, "layout must be contiguous or subring");
  if (subring() && (Kp() > N / 2 || B() < 2))
    return fail(EPHDC_ERR_PARAMS, "the subring layout needs N/(K' r) >= 2 (K' the power of two at or above K)");
  if (r > 1) {
    if (alpha < 1 || dnum < 1 || dnum > L) return fail(EPHDC_ERR_PARAMS, "r > 1 needs alpha >= 1 and 1 <= dnum <= L");
    if (scheme == EPHDC_BGV) return fail(EPHDC_ERR_PARAMS, "BGV takes r = 1 (no key switching)");
  }
  return EPHDC_OK;
}

std::vector<uint32_t> slot_exponents(uint32_t N) {
  std::vector<uint32_t> e(N);
  uint64_t g = 1;
  for (uint32_t s = 0; s < N / 2; ++s) {
    e[s] = (uint32_t)g;
    e[N / 2 + s] = (uint32_t)((2ull * N - g) % (2ull * N));
    g = g * 3 % (2ull * N);
  }
  return e;
}

std::vector<uint32_t> slot_positions(uint32_t N) {
  std::vector<uint32_t> e = slot_exponents(N), pos(N);
  int logn = ilog2(N);
  for (uint32_t s = 0; s < N; ++s) pos[s] = bitrev((e[s] - 1) / 2, logn);
  return pos;
}

SubringSlots::SubringSlots(const ParamSet& P)
    : of_exp(2 * P.N, 0), u_of((size_t)P.n(), 0), gpow(P.r), N(P.N), n(P.n()), B(P.B()), r(P.r), logb(ilog2(P.B())) {
  const std::vector<uint32_t> e = slot_exponents(P.N);
  for (uint32_t s = 0; s < P.N; ++s) of_exp[e[s]] = s;
  const uint64_t gamma = 1 + 2ull * n / r;
  const int logn = ilog2(n);
  for (uint32_t u = 0; u < r; ++u) {
    gpow[u] = powmod64(gamma, u, 2ull * N);
    const uint64_t gu = powmod64(gamma, u, 2ull * n);
    for (uint32_t ql = 0; ql < B; ++ql) {  // orbit of gamma^u * e_ql: block v = y - ql*r
      const uint64_t res = gu * (2ull * bitrev(ql, logb) + 1) % (2ull * n);
      const uint32_t y = bitrev((uint32_t)((res - 1) / 2), logn);
      u_of[y] = u;
    }
  }
}

std::vector<uint32_t> query_scatter_table(const ParamSet& P) {
  std::vector<uint32_t> pos = slot_positions(P.N);
  std::vector<uint32_t> tab(P.N, 0xFFFFFFFFu);
  if (P.subring()) {  // every slot of query ql's orbit carries its value
    const SubringSlots ss(P);
    for (uint32_t ql = 0; ql < P.B(); ++ql)
      for (uint32_t v = 0; v < P.r; ++v)
        for (uint32_t c = 0; c < P.Kp(); ++c) tab[pos[ss.slot_of(ql, c, v)]] = ql | (v << 16);
    return tab;
  }
  for (uint32_t rho = 0; rho < 2; ++rho)
    for (uint32_t u = 0; u < P.r; ++u)
      for (uint32_t ql = 0; ql < P.Bq(); ++ql)
        for (uint32_t c = 0; c < P.K; ++c)
          tab[pos[slot_index(P, rho, u, ql, c)]] = (rho * P.Bq() + ql) | (u << 16);
  return tab;
}

// ------------------------------------------------------------------ helpers
namespace {

void parallel_for(size_t n, const std::function<void(size_t)>& fn) {
  unsigned hw = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
  unsigned nt = (unsigned)std::min<size_t>(hw, n);
  if (nt <= 1) {
    for (size_t i = 0; i < n; ++i) fn(i);
    return;
  }
  std::atomic<size_t> next{0};
  std::vector<std::thread> pool;
  for (unsigned k = 0; k < nt; ++k)
    pool.emplace_back([&] {
      for (size_t i; (i = next.fetch_add(1)) < n;) fn(i);
    });
  for (auto& th : pool) th.join();
}

// Transforms for every modulus of the parameter set, plus t (with zeta = 3^((t-1)/2N),
// the root that fixes the slot map).
struct HostTables {
  std::vector<HostNtt> mod;  // L + alpha
  HostNtt tt;
  std::vector<uint32_t> pos;  // slot -> position
  explicit HostTables(const ParamSet& P) {
    for (uint32_t i = 0; i < P.nmod(); ++i) {
      uint32_t m = P.modulus(i);
      mod.emplace_back(P.N, m, root_of_unity(2 * P.N, m));
    }
    tt = HostNtt(P.N, P.t, root_of_unity(2 * P.N, P.t));
    pos = slot_positions(P.N);
  }
};

// Negacyclic a * b mod m with both operands given in the evaluation domain of `ntt`.
void pointwise(const HostNtt& ntt, const uint32_t* a, const uint32_t* b, uint32_t* out) {
  for (uint32_t i = 0; i < ntt.N; ++i) out[i] = (uint32_t)((uint64_t)a[i] * b[i] % ntt.m);
}

// Delta mod q_l with Delta = floor(Q/t): (-(Q mod t)) * t^-1 mod q_l, since Q = 0 mod q_l.
uint32_t delta_mod(const ParamSet& P, uint32_t l) {
  uint64_t rt = 1;
  for (uint32_t x : P.q) rt = rt * (x % P.t) % P.t;
  uint64_t ql = P.q[l];
  return (uint32_t)((ql - rt % ql) % ql * inv_mod(P.t, ql) % ql);
}

// Little-endian multi-word unsigned integers, just enough for exact CRT rounding.
struct Big {
  std::vector<uint32_t> w;
  static Big from(uint64_t v) { Big b; b.w = {(uint32_t)v, (uint32_t)(v >> 32)}; b.trim(); return b; }
  void trim() { while (!w.empty() && w.back() == 0) w.pop_back(); }
  Big mul(uint32_t k) const {
    Big r; uint64_t c = 0;
    for (uint32_t x : w) { uint64_t v = (uint64_t)x * k + c; r.w.push_back((uint32_t)v); c = v >> 32; }
    if (c) r.w.push_back((uint32_t)c);
    r.trim(); return r;
  }
  Big add(const Big& o) const {
    Big r; uint64_t c = 0; size_t n = std::max(w.size(), o.w.size());
    for (size_t i = 0; i < n; ++i) {
      uint64_t v = c + (i < w.size() ? w[i] : 0) + (i < o.w.size() ? o.w[i] : 0);
      r.w.push_back((uint32_t)v); c = v >> 32;
    }
    if (c) r.w.push_back((uint32_t)c);
    r.trim(); return r;
  }
  Big sub(const Big& o) const {  // requires *this >= o
    Big r; int64_t b = 0;
    for (size_t i = 0; i < w.size(); ++i) {
      int64_t v = (int64_t)w[i] - (i < o.w.size() ? o.w[i] : 0) - b;
      b = v < 0; if (v < 0) v += (1ll << 32);
      r.w.push_back((uint32_t)v);
    }
    r.trim(); return r;
  }
  uint32_t mod(uint32_t m) const {
    uint64_t r = 0;
    for (size_t i = w.size(); i-- > 0;) r = ((r << 32) | w[i]) % m;
    return (uint32_t)r;
  }
  int cmp(const Big& o) const {
    if (w.size() != o.w.size()) return w.size() < o.w.size() ? -1 : 1;
    for (size_t i = w.size(); i-- > 0;)
      if (w[i] != o.w[i]) return w[i] < o.w[i] ? -1 : 1;
    return 0;
  }
};

}  // namespace

}  // namespace ephdc

using namespace ephdc;

extern "C" {

const char* ephdc_last_error(void) { return g_last_error.c_str(); }

ephdc_status ephdc_check_params(const ephdc_params* prm) {
  ParamSet P;
  return P.load(prm);
}

uint32_t ephdc_queries_per_ct(const ephdc_params* prm) {
  ParamSet P;
  return P.load(prm) == EPHDC_OK ? P.B() : 0;
}

uint32_t ephdc_num_model_ct(const ephdc_params* prm) {
  ParamSet P;
  return P.load(prm) == EPHDC_OK ? P.M() : 0;
}

uint32_t ephdc_num_groups(const ephdc_params* prm, uint32_t Q) {
  ParamSet P;
  return P.load(prm) == EPHDC_OK ? P.G(Q) : 0;
}

uint32_t ephdc_hv_stride(const ephdc_params* prm, uint32_t Q) {
  ParamSet P;
  return P.load(prm) == EPHDC_OK ? P.G(Q) * P.B() : 0;
}

size_t ephdc_galois_key_words(const ephdc_params* prm) {
  ParamSet P;
  if (P.load(prm) != EPHDC_OK) return 0;
  return (size_t)P.log2r() * P.dnum * 2 * P.nmod() * P.N;
}

ephdc_status ephdc_default_primes(uint32_t N, uint32_t count, uint32_t skip, uint32_t* out) {
  if (!out) return fail(EPHDC_ERR_ARG, "out is NULL");
  if (N < 8 || (N & (N - 1))) return fail(EPHDC_ERR_ARG, "N must be a power of two >= 8");
  std::vector<uint32_t> v = default_primes(N, count, skip);
  if (v.size() != count) return fail(EPHDC_ERR_ARG, "not enough primes below 2^30");
  std::copy(v.begin(), v.end(), out);
  return EPHDC_OK;
}

ephdc_status ephdc_gaussian_cdt(uint64_t out[39]) {
  if (!out) return fail(EPHDC_ERR_ARG, "out is NULL");
  auto T = gaussian_cdt();
  std::copy(T.begin(), T.end(), out);
  return EPHDC_OK;
}

ephdc_status ephdc_keygen(const ephdc_params* prm, uint64_t seed, int8_t* sk, uint32_t* galois_keys) {
  ParamSet P;
  ephdc_status st = P.load(prm);
  if (st != EPHDC_OK) return st;
  if (!sk) return fail(EPHDC_ERR_ARG, "sk is NULL");
  const uint32_t N = P.N;
  Stream sec(seed, TAG_SECRET);
  for (uint32_t i = 0; i < N; ++i) sk[i] = (int8_t)((int)(sec(i) % 3) - 1);
  if (P.r == 1 || !galois_keys) {
    if (P.r > 1 && !galois_keys) return fail(EPHDC_ERR_NOKEY, "r > 1 needs a Galois key buffer");
    return EPHDC_OK;
  }
  HostTables H(P);
  const uint32_t nm = P.nmod(), steps = P.log2r(), dsz = P.digit_size();
  const auto cdt = gaussian_cdt();
  uint64_t Pmod[16];
  for (uint32_t l = 0; l < nm; ++l) {
    uint64_t m = P.modulus(l), acc = 1;
    for (uint32_t k = 0; k < P.alpha; ++k) acc = acc * (P.p[k] % m) % m;
    Pmod[l] = acc;
  }
  Stream gal(seed, TAG_GALOIS);
  parallel_for((size_t)steps * P.dnum, [&](size_t task) {
    uint32_t i = (uint32_t)(task / P.dnum), j = (uint32_t)(task % P.dnum);
    uint32_t g = galois_element(P, i);
    std::vector<int32_t> srot(N, 0);  // sigma_g(s) as an integer polynomial
    for (uint32_t k = 0; k < N; ++k) {
      uint64_t d = (uint64_t)k * g % (2ull * N);
      if (d < N) srot[d] = sk[k];
      else srot[d - N] = -sk[k];
    }
    uint64_t start = ((uint64_t)(i * P.dnum + j) * (nm + 1)) * N;
    std::vector<int32_t> e(N);
    for (uint32_t k = 0; k < N; ++k) e[k] = gaussian_sample(gal(start + (uint64_t)nm * N + k), cdt);
    std::vector<uint32_t> a(N), sv(N), as(N);
    for (uint32_t l = 0; l < nm; ++l) {
      const HostNtt& T = H.mod[l];
      const uint32_t m = T.m;
      for (uint32_t k = 0; k < N; ++k) a[k] = (uint32_t)(gal(start + (uint64_t)l * N + k) % m);
      for (uint32_t k = 0; k < N; ++k) sv[k] = sk[k] < 0 ? m - 1 : (uint32_t)sk[k];
      std::vector<uint32_t> A(a);
      T.forward(A.data());
      T.forward(sv.data());
      pointwise(T, A.data(), sv.data(), as.data());
      T.inverse(as.data());
      bool in_digit = l < P.L && l / dsz == j;
      uint32_t* b = galois_keys + ((((size_t)i * P.dnum + j) * 2 + 0) * nm + l) * N;
      uint32_t* aa = galois_keys + ((((size_t)i * P.dnum + j) * 2 + 1) * nm + l) * N;
      for (uint32_t k = 0; k < N; ++k) {
        uint64_t v = (uint64_t)(m - as[k]) + (e[k] < 0 ? m + e[k] : e[k]);
        if (in_digit) v += Pmod[l] * (uint64_t)(srot[k] < 0 ? m - 1 : (uint32_t)srot[k]) % m;
        b[k] = (uint32_t)(v % m);
        aa[k] = a[k];
      }
    }
  });
  return EPHDC_OK;
}

ephdc_status ephdc_encrypt_model(const ephdc_params* prm, const int8_t* sk, const int8_t* class_hv,
                                 uint64_t seed, uint32_t* model_ct) {
  ParamSet P;
  ephdc_status st = P.load(prm);
  if (st != EPHDC_OK) return st;
  if (!sk || !class_hv || !model_ct) return fail(EPHDC_ERR_ARG, "NULL buffer");
  return encrypt_model_host(P, sk, class_hv, seed, model_ct);
}

}  // extern "C"

namespace ephdc {

ephdc_status encrypt_model_host(const ParamSet& P, const int8_t* sk, const int8_t* class_hv, uint64_t seed,
                                uint32_t* model_ct) {
  HostTables H(P);
  const uint32_t N = P.N, L = P.L, M = P.M();
  const auto cdt = gaussian_cdt();
  std::vector<uint32_t> dl(L);
  uint64_t rt = 1;  // Q mod t (rounded BFV: round(Q*mu/t) = Delta*mu + floor((2*rt*mu + t) / 2t))
  for (uint32_t x : P.q) rt = rt * (x % P.t) % P.t;
  std::vector<std::vector<uint32_t>> S(L);  // secret key in each limb's evaluation domain
  for (uint32_t l = 0; l < L; ++l) {
    dl[l] = delta_mod(P, l);
    S[l].resize(N);
    for (uint32_t k = 0; k < N; ++k) S[l][k] = sk[k] < 0 ? P.q[l] - 1 : (uint32_t)sk[k];
    H.mod[l].forward(S[l].data());
  }
  Stream enc(seed, TAG_ENCRYPT);
  std::unique_ptr<SubringSlots> subring(P.subring() ? new SubringSlots(P) : nullptr);
  parallel_for(M, [&](size_t mi) {
    const uint32_t m = (uint32_t)mi;
    // slot vector of ciphertext m, placed at transform positions, then mu = Encode(v)
    std::vector<uint32_t> mu(N, 0);
    if (subring) {
      for (uint32_t u = 0; u < P.r && m * P.r + u < P.D; ++u)
        for (uint32_t ql = 0; ql < P.B(); ++ql)
          for (uint32_t c = 0; c < P.K; ++c) {
            int v = class_hv[(size_t)c * P.D + m * P.r + u];
            mu[H.pos[subring->slot_of(ql, c, u)]] = v < 0 ? (uint32_t)(P.t + v) : (uint32_t)v;
          }
    }
    for (uint32_t rho = 0; rho < 2 && !subring; ++rho)
      for (uint32_t u = 0; u < P.r; ++u) {
        uint32_t j = m * P.r + u;
        if (j >= P.D) continue;
        for (uint32_t ql = 0; ql < P.Bq(); ++ql)
          for (uint32_t c = 0; c < P.K; ++c) {
            int v = class_hv[(size_t)c * P.D + j];
            mu[H.pos[slot_index(P, rho, u, ql, c)]] = v < 0 ? (uint32_t)(P.t + v) : (uint32_t)v;
          }
      }
    H.tt.inverse(mu.data());
    const uint64_t start = (uint64_t)m * (L + 1) * N;
    std::vector<int32_t> e(N);
    for (uint32_t k = 0; k < N; ++k) e[k] = gaussian_sample(enc(start + (uint64_t)L * N + k), cdt);
    std::vector<uint32_t> a(N), as(N);
    for (uint32_t l = 0; l < L; ++l) {
      const HostNtt& T = H.mod[l];
      const uint32_t ql = T.m;
      for (uint32_t k = 0; k < N; ++k) a[k] = (uint32_t)(enc(start + (uint64_t)l * N + k) % ql);
      std::vector<uint32_t> A(a);
      T.forward(A.data());
      pointwise(T, A.data(), S[l].data(), as.data());
      T.inverse(as.data());
      uint32_t* c0 = model_ct + (((size_t)m * 2 + 0) * L + l) * N;
      uint32_t* c1 = model_ct + (((size_t)m * 2 + 1) * L + l) * N;
      for (uint32_t k = 0; k < N; ++k) {
        const uint64_t err = e[k] < 0 ? ql + e[k] : e[k];
        uint64_t msg;
        if (P.scheme == EPHDC_BGV) {  // t*e + centred(mu)
          const uint64_t mc = mu[k] > P.t / 2 ? ql - (P.t - mu[k]) : mu[k];
          msg = (err * P.t + mc) % ql;
        } else {  // e + Delta*mu, plus the rounding of Q*mu/t for the rounded variant
          msg = (err + (uint64_t)dl[l] * mu[k]) % ql;
          if (P.scheme == EPHDC_BFV_ROUNDED) msg += (2 * rt * mu[k] + P.t) / (2 * (uint64_t)P.t);
        }
        c0[k] = (uint32_t)(((uint64_t)(ql - as[k]) + msg) % ql);
        c1[k] = a[k];
      }
    }
  });
  return EPHDC_OK;
}

}  // namespace ephdc

extern "C" {

ephdc_status ephdc_decrypt_scores(const ephdc_params* prm, const int8_t* sk, const uint32_t* score_ct,
                                  uint32_t Q, int32_t* scores, int32_t* argmax) {
  return ephdc_decrypt_scores_at(prm, sk, score_ct, 0, Q, scores, argmax);
}

ephdc_status ephdc_decrypt_scores_at(const ephdc_params* prm, const int8_t* sk, const uint32_t* score_ct,
                                     uint32_t q_first, uint32_t Q, int32_t* scores, int32_t* argmax) {
  ParamSet P;
  ephdc_status st = P.load(prm);
  if (st != EPHDC_OK) return st;
  if (!sk || !score_ct || !scores) return fail(EPHDC_ERR_ARG, "NULL buffer");
  if (Q == 0) return EPHDC_OK;
  HostTables H(P);
  const uint32_t N = P.N, L = P.L, t = P.t;
  const uint32_t g_first = q_first / P.B(), G = P.G(q_first + Q) - g_first;
  // CRT constants: Qhat_l = Q/q_l (big), Qhat_l^-1 mod q_l, Q (big)
  std::vector<Big> Qhat(L);
  std::vector<uint32_t> Qhat_inv(L);
  Big Qbig = Big::from(1);
  for (uint32_t x : P.q) Qbig = Qbig.mul(x);
  for (uint32_t l = 0; l < L; ++l) {
    Big b = Big::from(1);
    uint64_t r = 1;
    for (uint32_t k = 0; k < L; ++k)
      if (k != l) { b = b.mul(P.q[k]); r = r * (P.q[k] % P.q[l]) % P.q[l]; }
    Qhat[l] = b;
    Qhat_inv[l] = inv_mod(r, P.q[l]);
  }
  const Big twoQ = Qbig.mul(2);
  const uint32_t Qmod_t = Qbig.mod(t);
  std::vector<std::vector<uint32_t>> S(L);
  for (uint32_t l = 0; l < L; ++l) {
    S[l].resize(N);
    for (uint32_t k = 0; k < N; ++k) S[l][k] = sk[k] < 0 ? P.q[l] - 1 : (uint32_t)sk[k];
    H.mod[l].forward(S[l].data());
  }
  std::unique_ptr<SubringSlots> subring(P.subring() ? new SubringSlots(P) : nullptr);
  parallel_for(G, [&](size_t gi) {
    const uint32_t g = g_first + (uint32_t)gi;
    std::vector<std::vector<uint32_t>> x(L, std::vector<uint32_t>(N));
    std::vector<uint32_t> tmp(N);
    for (uint32_t l = 0; l < L; ++l) {
      const HostNtt& T = H.mod[l];
      const uint32_t* c0 = score_ct + (((size_t)g * 2 + 0) * L + l) * N;
      const uint32_t* c1 = score_ct + (((size_t)g * 2 + 1) * L + l) * N;
      std::copy(c1, c1 + N, tmp.begin());
      T.forward(tmp.data());
      pointwise(T, tmp.data(), S[l].data(), x[l].data());
      T.inverse(x[l].data());
      for (uint32_t k = 0; k < N; ++k) x[l][k] = (uint32_t)(((uint64_t)x[l][k] + c0[k]) % T.m);
    }
    // mu = round(t*x/Q) mod t.  With y_l = x_l * Qhat_l^-1 mod q_l, t*x/Q equals
    // sum_l y_l*t/q_l minus a multiple of t; split y_l*t = a_l*q_l + b_l and round the
    // fraction sum_l b_l*Qhat_l / Q exactly with big integers.
    std::vector<uint32_t> mu(N);
    for (uint32_t k = 0; k < N && P.scheme == EPHDC_BGV; ++k) {
      // BGV: x = sum_l y_l * Qhat_l reduced mod Q, centred, then mod t
      Big X;
      for (uint32_t l = 0; l < L; ++l)
        X = X.add(Qhat[l].mul((uint32_t)((uint64_t)x[l][k] * Qhat_inv[l] % P.q[l])));
      while (X.cmp(Qbig) >= 0) X = X.sub(Qbig);
      const uint32_t xt = X.mod(t);
      mu[k] = X.mul(2).cmp(Qbig) > 0 ? (uint32_t)(((uint64_t)xt + t - Qmod_t) % t) : xt;
    }
    for (uint32_t k = 0; k < N && P.scheme != EPHDC_BGV; ++k) {
      uint64_t A = 0;
      Big Sf;
      for (uint32_t l = 0; l < L; ++l) {
        uint64_t y = (uint64_t)x[l][k] * Qhat_inv[l] % P.q[l];
        uint64_t yt = y * t;
        A += yt / P.q[l];
        Sf = Sf.add(Qhat[l].mul((uint32_t)(yt % P.q[l])));
      }
      Big X = Sf.mul(2).add(Qbig);
      uint64_t rnd = 0;
      while (X.cmp(twoQ) >= 0) { X = X.sub(twoQ); ++rnd; }
      mu[k] = (uint32_t)((A + rnd) % t);
    }
    H.tt.forward(mu.data());  // slot s now sits at position pos[s]
    const uint32_t B = P.B(), Bq = P.Bq();
    for (uint32_t qi = 0; qi < B; ++qi) {
      const uint32_t qg = g * B + qi;  // index in the ciphertext sequence
      if (qg < q_first) continue;
      if (qg >= q_first + Q) break;
      const uint32_t qq = qg - q_first;
      uint32_t rho = qi / Bq, ql = qi % Bq;
      int32_t best = 0;
      for (uint32_t c = 0; c < P.K; ++c) {
        uint32_t v = mu[H.pos[subring ? subring->slot_of(qi, c) : slot_index(P, rho, 0, ql, c)]];
        int32_t sc = v > t / 2 ? (int32_t)v - (int32_t)t : (int32_t)v;
        scores[(size_t)qq * P.K + c] = sc;
        if (c == 0 || sc > scores[(size_t)qq * P.K + best]) best = (int32_t)c;
      }
      if (argmax) argmax[qq] = best;
    }
  });
  return EPHDC_OK;
}

}  // extern "C"
