// findDmax on the device: the largest hypervector dimension D whose encrypted dot product
// still decrypts, per trial (EP-HDC design space exploration, Algorithm 1, procedure
// findDmax; noise study).
//
// A trial draws fresh keys, class values and query values, encrypts the D_cap model
// ciphertexts (server side, host) and then evaluates every prefix sum_{m < D} ct_m * p_m at
// once on the device instead of one D at a time:
//   1. batch encoding of the D_cap query plaintexts of group 0 (the scoring path's kernel);
//   2. per limb and chunk of model ciphertexts, running sums of the ct x pt products and
//      the decryption phase c0 + c1*s of every prefix (evaluation domain);
//   3. chunk offsets: each chunk's phases get the phase of all earlier chunks added;
//   4. the phases back to the coefficient domain, then decryption of every coefficient
//      (BFV: round(t*x/Q) mod t by exact RNS rounding; BGV: centred x mod t);
//   5. decoding to slots (forward transform mod t) and comparison with the running exact
//      dot products: the first prefix with a wrong slot ends the trial.
// The trial's D_i is the number of prefixes before the first wrong one (D_cap when none is).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "kernel_common.hpp"
#include "session.hpp"

namespace ephdc_dev {

struct DmaxArgs {
  const uint32_t* model;   // [D_cap][2][L][N] evaluation domain, Montgomery form
  const int32_t* pt;       // [D_cap][N] lifted query plaintexts (coefficient order)
  const uint32_t* skh;     // [L][N] secret key, evaluation domain, Montgomery form
  uint32_t* phase;         // [D_cap][L][N] decryption phases of the prefixes (evaluation domain)
  uint32_t* ends;          // [S][L][N] chunk-end phases, then their exclusive prefix sums
  const uint32_t* fwd_tw;  // [L][N] forward twiddles, Montgomery form
  const PrimeConst* pcs;   // [L]
  uint32_t L, dcap, chunk, S;
};

// Step 2: work item (chunk, limb).  Running sums acc_c in [0, 2q) of ct_m[c] * p_m over the
// chunk's ciphertexts; after each, the phase acc_0 + acc_1 * s of the prefix so far.
template <int LOGN, int LE>
__global__ __launch_bounds__((1 << LOGN) >> LE) void k_dmax_prefix(DmaxArgs a) {
  using S = Shape<LOGN, LE>;
  constexpr int E = S::E, N = S::N;
  LdsBufs b{0};
  const int tid = threadIdx.x;
  const uint32_t l = blockIdx.x % a.L, ch = blockIdx.x / a.L;
  const uint32_t m0 = ch * a.chunk, m1 = min(a.dcap, m0 + a.chunk);
  const PrimeConst pc = a.pcs[l];
  const uint32_t m2 = 2 * pc.m, eo = (uint32_t)tid * E * 4u, co = (uint32_t)tid * 4u;
  uint32_t sh[E], acc0[E], acc1[E], ph[E];
  const uint32_t* skl = a.skh + (size_t)l * N;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    sh[i] = ld_at(skl, eo + 4u * i);
    acc0[i] = acc1[i] = ph[i] = 0u;
  }
  for (uint32_t m = m0; m < m1; ++m) {
    const int32_t* ptm = a.pt + (size_t)m * N;
    uint32_t p[E];
#pragma unroll
    for (int i = 0; i < E; ++i) p[i] = pc.m + (uint32_t)ld_at(ptm, co + 4u * (uint32_t)(i * S::T));
    ntt_forward<LOGN, LE, false, true>(p, tid, a.fwd_tw + (size_t)l * N, pc, b);
    const uint32_t* ct0 = a.model + (((size_t)m * 2 + 0) * a.L + l) * N;
    const uint32_t* ct1 = a.model + (((size_t)m * 2 + 1) * a.L + l) * N;
    uint32_t* dst = a.phase + ((size_t)m * a.L + l) * N;
#pragma unroll
    for (int i = 0; i < E; ++i) {
      acc0[i] = csub(acc0[i] + mont_mul(ld_at(ct0, eo + 4u * i), p[i], pc.m, pc.mneg_inv), m2);
      acc1[i] = csub(acc1[i] + mont_mul(ld_at(ct1, eo + 4u * i), p[i], pc.m, pc.mneg_inv), m2);
      ph[i] = csub(csub(acc0[i] + mont_mul(acc1[i], sh[i], pc.m, pc.mneg_inv), m2), pc.m);
      st_at(dst, eo + 4u * i, ph[i]);
    }
  }
  uint32_t* end = a.ends + ((size_t)ch * a.L + l) * N;
#pragma unroll
  for (int i = 0; i < E; ++i) st_at(end, eo + 4u * i, ph[i]);
}

// Step 3a: exclusive prefix sums over chunks of the chunk-end phases, in place, one thread
// per (limb, position).
__global__ void k_dmax_scan_ends(uint32_t* ends, const PrimeConst* __restrict__ pcs, uint32_t L, uint32_t N,
                                 uint32_t S) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L * N) return;
  const uint32_t q = pcs[i / N].m;
  uint32_t run = 0;
  for (uint32_t ch = 0; ch < S; ++ch) {
    const uint32_t v = ends[(size_t)ch * L * N + i];
    ends[(size_t)ch * L * N + i] = run;
    run = csub(run + v, q);
  }
}

// Step 3b: the offset of a chunk added to the phases of its prefixes.
__global__ void k_dmax_add_offsets(uint32_t* phase, const uint32_t* __restrict__ ends,
                                   const PrimeConst* __restrict__ pcs, uint32_t L, uint32_t N, uint32_t chunk,
                                   uint32_t dcap) {
  const size_t total = (size_t)dcap * L * N;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const uint32_t m = (uint32_t)(i / ((size_t)L * N)), ln = (uint32_t)(i % ((size_t)L * N));
    const uint32_t ch = m / chunk;
    if (ch == 0) continue;
    phase[i] = csub(phase[i] + ends[(size_t)ch * L * N + ln], pcs[ln / N].m);
  }
}

// Constants of the exact decryption for L <= 2 limbs (Q < 2^60).
struct DecryptConst {
  uint32_t q[2];
  uint32_t qhat_inv[2];  // (Q/q_l)^-1 mod q_l
  uint64_t qhat[2];      // Q/q_l
  uint64_t Q;
  uint32_t t, L, bgv, Qmod_t;
  uint32_t q0_inv_mod_q1;  // Garner: q0^-1 mod q1 (L = 2)
};

// Step 4: decryption of every phase coefficient to mu in [0, t).
//   BFV: with y_l = x_l * (Q/q_l)^-1 mod q_l, t*x/Q = sum_l y_l*t/q_l minus a multiple of t;
//        split y_l*t = a_l*q_l + b_l, then mu = sum_l a_l + round(sum_l b_l*(Q/q_l) / Q) mod t
//        (the rounding term is 0, 1 or 2 and is found by comparisons, exactly).
//   BGV: x by Garner's reconstruction, centred, reduced mod t.
__global__ void k_dmax_decrypt(const uint32_t* __restrict__ phase, uint32_t* __restrict__ mu, DecryptConst c,
                               uint32_t N, size_t total) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const size_t m = i / N, k = i % N;
    const uint32_t x0 = phase[(m * c.L + 0) * N + k];
    const uint32_t x1 = c.L > 1 ? phase[(m * c.L + 1) * N + k] : 0u;
    uint32_t out;
    if (c.bgv) {
      uint64_t x = x0;
      if (c.L > 1) {
        const uint64_t d = ((uint64_t)x1 + c.q[1] - x0 % c.q[1]) % c.q[1];
        x = (uint64_t)x0 + (uint64_t)c.q[0] * (d * c.q0_inv_mod_q1 % c.q[1]);
      }
      const uint32_t xt = (uint32_t)(x % c.t);
      out = 2 * x > c.Q ? (uint32_t)(((uint64_t)xt + c.t - c.Qmod_t) % c.t) : xt;
    } else {
      uint64_t A = 0, Sf = 0;
      const uint32_t xs[2] = {x0, x1};
      for (uint32_t l = 0; l < c.L; ++l) {
        const uint64_t y = (uint64_t)xs[l] * c.qhat_inv[l] % c.q[l];
        const uint64_t yt = y * c.t;
        A += yt / c.q[l];
        Sf += (yt % c.q[l]) * c.qhat[l];
      }
      const uint64_t X = 2 * Sf + c.Q;
      const uint64_t rnd = (X >= 2 * c.Q ? 1u : 0u) + (X >= 4 * c.Q ? 1u : 0u);
      out = (uint32_t)((A + rnd) % c.t);
    }
    mu[i] = out;
  }
}

// Step 5: thread per slot position; the running exact dot product of the slot's query and
// class, compared with every prefix's decrypted slot until the first difference, whose
// prefix index goes to *fail (atomic minimum).
__global__ void k_dmax_compare(const uint32_t* __restrict__ slots, const uint32_t* __restrict__ tab,
                               const int8_t* __restrict__ cls, const int8_t* __restrict__ qry, uint32_t N,
                               uint32_t dcap, uint32_t t, uint32_t* fail) {
  const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= N) return;
  const uint32_t e = tab[x];
  const bool used = e != 0xFFFFFFFFu;
  const uint32_t qi = e >> 8, c = e & 0xFFu;
  int64_t acc = 0;
  for (uint32_t m = 0; m < dcap; ++m) {
    if (used) {
      acc += (int64_t)cls[(size_t)c * dcap + m] * qry[(size_t)qi * dcap + m];
      acc %= (int64_t)t;
    }
    const uint32_t want = (uint32_t)(acc < 0 ? acc + t : acc);
    if (slots[(size_t)m * N + x] != want) {
      atomicMin(fail, m);
      return;
    }
    if ((m & 63u) == 63u && __atomic_load_n(fail, __ATOMIC_RELAXED) <= m) return;
  }
}

}  // namespace ephdc_dev

namespace ephdc {

using namespace ephdc_dev;

namespace {

hipError_t launch_dmax_prefix(int logn, const DmaxArgs& a, hipStream_t st) {
  return dispatch(logn, [&](auto lnc, auto lec) {
    constexpr int LN = decltype(lnc)::value, LEv = decltype(lec)::value;
    static std::once_flag once;
    static hipError_t attr = hipSuccess;
    std::call_once(once, [] {
      attr = hipFuncSetAttribute((const void*)k_dmax_prefix<LN, LEv>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds_bytes<LN, LEv>());
    });
    if (attr != hipSuccess) return attr;
    k_dmax_prefix<LN, LEv><<<dim3(a.S * a.L), dim3(Shape<LN, LEv>::T), lds_bytes<LN, LEv>(), st>>>(a);
    return hipGetLastError();
  });
}

uint32_t sample_value(uint64_t u, uint32_t bits) {
  if (bits == 1) return (uint32_t)(2 * (u % 2)) - 1u;
  return (uint32_t)(u % (1ull << bits)) - (1u << (bits - 1));
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

ephdc_status dev_buf(DevBuf& b, size_t bytes, const char* what) {
  if (hipMalloc(&b.p, std::max<size_t>(bytes, 256)) != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();
    return fail(EPHDC_ERR_OOM, std::string("hipMalloc failed for ") + what);
  }
  return EPHDC_OK;
}

constexpr uint64_t kTagDmaxClass = 8, kTagDmaxQuery = 9;

}  // namespace

}  // namespace ephdc

using namespace ephdc;

extern "C" {

ephdc_status ephdc_find_dmax(const ephdc_params* prm, uint64_t seed, uint32_t trials, uint32_t d_cap,
                             uint32_t cbits, int32_t* dmax, void* stream) {
  if (!prm || !dmax) return fail(EPHDC_ERR_ARG, "NULL argument");
  if (trials == 0 || d_cap == 0) return fail(EPHDC_ERR_ARG, "trials and d_cap must be positive");
  if (cbits < 1 || cbits > 8) return fail(EPHDC_ERR_ARG, "cbits must be in [1, 8]");
  ephdc_params pp = *prm;
  pp.D = d_cap;
  pp.F = 16;
  pp.scale_every = 0;
  ParamSet P;
  ephdc_status st = P.load(&pp);
  if (st != EPHDC_OK) return st;
  if (P.r != 1 || P.subring())
    return fail(EPHDC_ERR_UNSUPPORTED, "findDmax uses the paper's packing (r = 1, contiguous layout)");
  if (P.L > 2) return fail(EPHDC_ERR_UNSUPPORTED, "findDmax decrypts on the device with L <= 2 limbs");
  if (P.K > 255) return fail(EPHDC_ERR_UNSUPPORTED, "findDmax takes K <= 255");
  if ((uint64_t)d_cap * P.B() >= (1ull << 31)) return fail(EPHDC_ERR_UNSUPPORTED, "d_cap * B must be < 2^31");
  hipStream_t hs = (hipStream_t)stream;
  const uint32_t N = P.N, L = P.L, B = P.B(), K = P.K;

  // decryption constants
  DecryptConst dc{};
  dc.L = L;
  dc.t = P.t;
  dc.bgv = P.scheme == EPHDC_BGV;
  dc.Q = 1;
  for (uint32_t l = 0; l < L; ++l) dc.Q *= P.q[l];
  for (uint32_t l = 0; l < L; ++l) {
    dc.q[l] = P.q[l];
    dc.qhat[l] = dc.Q / P.q[l];
    dc.qhat_inv[l] = inv_mod(dc.qhat[l] % P.q[l], P.q[l]);
  }
  dc.Qmod_t = (uint32_t)(dc.Q % P.t);
  dc.q0_inv_mod_q1 = L > 1 ? inv_mod(P.q[0], P.q[1]) : 0;
  // slot position -> (query, class) of group 0, or unused
  std::vector<uint32_t> pos = slot_positions(N), tab(N, 0xFFFFFFFFu);
  for (uint32_t rho = 0; rho < 2; ++rho)
    for (uint32_t ql = 0; ql < P.Bq(); ++ql)
      for (uint32_t c = 0; c < K; ++c) tab[pos[slot_index(P, rho, 0, ql, c)]] = ((rho * P.Bq() + ql) << 8) | c;
  // forward transform mod t (decoding) in Montgomery form, and the constants of t
  HostNtt Tt(N, P.t, root_of_unity(2 * N, P.t));
  std::vector<uint32_t> fwd_t(N);
  for (uint32_t k = 0; k < N; ++k) fwd_t[k] = (uint32_t)(((uint64_t)Tt.fw[k] << 32) % P.t);
  PrimeConst pct{};
  {
    uint32_t inv = 1;
    for (int i = 0; i < 5; ++i) inv *= 2u - P.t * inv;
    pct.m = P.t;
    pct.mneg_inv = 0u - inv;
    pct.r2 = (uint32_t)(((unsigned __int128)1 << 64) % P.t);
    pct.r1 = (uint32_t)((1ull << 32) % P.t);
  }

  // device buffers shared by the trials
  const uint32_t chunk = std::max<uint32_t>(16, (d_cap + 255) / 256);
  const uint32_t S = (d_cap + chunk - 1) / chunk;
  DevBuf d_model, d_hv, d_pt, d_sk, d_skh, d_phase, d_coef, d_ends, d_mu, d_slots, d_tab, d_cls, d_qry, d_fwdt,
      d_pct, d_fail;
  const size_t model_words = (size_t)d_cap * 2 * L * N;
  if ((st = dev_buf(d_model, model_words * 4, "model")) != EPHDC_OK ||
      (st = dev_buf(d_hv, (size_t)d_cap * B, "query hypervectors")) != EPHDC_OK ||
      (st = dev_buf(d_pt, (size_t)d_cap * N * 4, "plaintexts")) != EPHDC_OK ||
      (st = dev_buf(d_sk, (size_t)L * N * 4, "secret key")) != EPHDC_OK ||
      (st = dev_buf(d_skh, (size_t)L * N * 4, "secret key")) != EPHDC_OK ||
      (st = dev_buf(d_phase, (size_t)d_cap * L * N * 4, "phases")) != EPHDC_OK ||
      (st = dev_buf(d_coef, (size_t)d_cap * L * N * 4, "phases")) != EPHDC_OK ||
      (st = dev_buf(d_ends, (size_t)S * L * N * 4, "chunk ends")) != EPHDC_OK ||
      (st = dev_buf(d_mu, (size_t)d_cap * N * 4, "decryptions")) != EPHDC_OK ||
      (st = dev_buf(d_slots, (size_t)d_cap * N * 4, "slots")) != EPHDC_OK ||
      (st = dev_buf(d_tab, (size_t)N * 4, "slot table")) != EPHDC_OK ||
      (st = dev_buf(d_cls, (size_t)K * d_cap, "class values")) != EPHDC_OK ||
      (st = dev_buf(d_qry, (size_t)B * d_cap, "query values")) != EPHDC_OK ||
      (st = dev_buf(d_fwdt, (size_t)N * 4, "twiddles mod t")) != EPHDC_OK ||
      (st = dev_buf(d_pct, sizeof(PrimeConst), "constants of t")) != EPHDC_OK ||
      (st = dev_buf(d_fail, 4, "result")) != EPHDC_OK)
    return st;
  HIP_TRY(hipMemcpyAsync(d_tab.p, tab.data(), N * 4, hipMemcpyHostToDevice, hs), "copy");
  HIP_TRY(hipMemcpyAsync(d_fwdt.p, fwd_t.data(), N * 4, hipMemcpyHostToDevice, hs), "copy");
  HIP_TRY(hipMemcpyAsync(d_pct.p, &pct, sizeof pct, hipMemcpyHostToDevice, hs), "copy");

  std::vector<int8_t> sk(N), cls((size_t)K * d_cap), qry((size_t)B * d_cap), hv((size_t)d_cap * B);
  std::vector<uint32_t> model(model_words), skr((size_t)L * N);
  for (uint32_t tr = 0; tr < trials; ++tr) {
    const uint64_t sd = seed + tr;
    // inputs of the trial: secret key, class values [K][D_cap], query values [B][D_cap]
    const Stream sec(sd, TAG_SECRET), sc(sd, kTagDmaxClass), sq(sd, kTagDmaxQuery);
    for (uint32_t k = 0; k < N; ++k) sk[k] = (int8_t)((int)(sec(k) % 3) - 1);
    for (uint32_t m = 0; m < d_cap; ++m) {
      for (uint32_t c = 0; c < K; ++c) cls[(size_t)c * d_cap + m] = (int8_t)sample_value(sc((uint64_t)m * K + c), cbits);
      for (uint32_t q = 0; q < B; ++q) {
        const int8_t v = (int8_t)sample_value(sq((uint64_t)m * B + q), P.qbits);
        qry[(size_t)q * d_cap + m] = v;
        hv[(size_t)m * B + q] = v;
      }
    }
    for (uint32_t l = 0; l < L; ++l)
      for (uint32_t k = 0; k < N; ++k) skr[(size_t)l * N + k] = sk[k] < 0 ? P.q[l] - 1 : (uint32_t)sk[k];
    if ((st = encrypt_model_host(P, sk.data(), cls.data(), sd, model.data())) != EPHDC_OK) return st;
    HIP_TRY(hipMemcpyAsync(d_model.p, model.data(), model_words * 4, hipMemcpyHostToDevice, hs), "copy");
    HIP_TRY(hipMemcpyAsync(d_hv.p, hv.data(), hv.size(), hipMemcpyHostToDevice, hs), "copy");
    HIP_TRY(hipMemcpyAsync(d_sk.p, skr.data(), skr.size() * 4, hipMemcpyHostToDevice, hs), "copy");
    HIP_TRY(hipMemcpyAsync(d_cls.p, cls.data(), cls.size(), hipMemcpyHostToDevice, hs), "copy");
    HIP_TRY(hipMemcpyAsync(d_qry.p, qry.data(), qry.size(), hipMemcpyHostToDevice, hs), "copy");
    // the trial's session: evaluation-domain model and the transform tables
    ephdc_session* s = nullptr;
    if ((st = session_create(&pp, d_model.as<uint32_t>(), model_words, nullptr, 0, B, nullptr, 0, stream, false,
                             &s)) != EPHDC_OK)
      return st;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    // 1. query plaintexts of group 0
    ScoreArgs a{};
    a.hv = d_hv.as<int8_t>();
    a.scatter = s->d_scatter;
    a.inv_t = s->d_inv_t;
    a.pct = s->pct;
    a.pcs = s->d_pc;
    a.L = L;
    a.M = d_cap;
    a.D = d_cap;
    a.r = 1;
    a.hv_stride = B;
    a.B = B;
    a.G = 1;
    a.q_last = B;  // the trial's one group is full
    a.m_base = 0;
    a.m_len = d_cap;
    const uint32_t Se = std::min<uint32_t>(d_cap, 512);
    a.mchunk = (d_cap + Se - 1) / Se;
    a.pt = d_pt.as<int32_t>();
    chk(launch_encode_pt(P.logn, 0, a, (d_cap + a.mchunk - 1) / a.mchunk, hs));
    // the secret key in every limb's evaluation domain
    chk(launch_fwd_batch(P.logn, d_sk.as<uint32_t>(), d_skh.as<uint32_t>(), L, s->d_fwd, s->d_pc, L, 0, true, hs));
    // 2-3. prefix phases
    DmaxArgs da{s->d_model, d_pt.as<int32_t>(), d_skh.as<uint32_t>(), d_phase.as<uint32_t>(), d_ends.as<uint32_t>(),
                s->d_fwd, s->d_pc, L, d_cap, chunk, S};
    chk(launch_dmax_prefix(P.logn, da, hs));
    if (e == hipSuccess) {
      k_dmax_scan_ends<<<dim3((L * N + 255) / 256), dim3(256), 0, hs>>>(d_ends.as<uint32_t>(), s->d_pc, L, N, S);
      chk(hipGetLastError());
      k_dmax_add_offsets<<<dim3(2048), dim3(256), 0, hs>>>(d_phase.as<uint32_t>(), d_ends.as<uint32_t>(), s->d_pc, L,
                                                           N, chunk, d_cap);
      chk(hipGetLastError());
    }
    // 4. coefficient domain, decryption
    chk(launch_inv_batch(P.logn, d_phase.as<uint32_t>(), d_coef.as<uint32_t>(), (size_t)d_cap * L, s->d_inv, s->d_pc,
                         L, 0, hs));
    if (e == hipSuccess) {
      k_dmax_decrypt<<<dim3(2048), dim3(256), 0, hs>>>(d_coef.as<uint32_t>(), d_mu.as<uint32_t>(), dc, N,
                                                       (size_t)d_cap * N);
      chk(hipGetLastError());
    }
    // 5. slots, comparison with the exact running dot products
    chk(launch_fwd_batch(P.logn, d_mu.as<uint32_t>(), d_slots.as<uint32_t>(), d_cap, d_fwdt.as<uint32_t>(),
                         d_pct.as<PrimeConst>(), 1, 0, false, hs));
    const uint32_t none = 0xFFFFFFFFu;
    chk(hipMemcpyAsync(d_fail.p, &none, 4, hipMemcpyHostToDevice, hs));
    if (e == hipSuccess) {
      k_dmax_compare<<<dim3((N + 255) / 256), dim3(256), 0, hs>>>(d_slots.as<uint32_t>(), d_tab.as<uint32_t>(),
                                                                 d_cls.as<int8_t>(), d_qry.as<int8_t>(), N, d_cap,
                                                                 P.t, d_fail.as<uint32_t>());
      chk(hipGetLastError());
    }
    uint32_t first = none;
    chk(hipMemcpyAsync(&first, d_fail.p, 4, hipMemcpyDeviceToHost, hs));
    chk(hipStreamSynchronize(hs));
    (void)ephdc_session_destroy(s);
    if (e != hipSuccess) return hip_fail(e, "findDmax trial");
    dmax[tr] = (int32_t)std::min(first, d_cap);
  }
  return EPHDC_OK;
}

}  // extern "C"
