// Client side of the C ABI: sessions (device-resident evaluation-domain model, keys and
// tables), HDC encoding and homomorphic scoring.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "session.hpp"

using namespace ephdc;

namespace {

using ephdc::scale_op;

void drop_events(ephdc_session* s) {
  for (auto& v : s->ev) {
    for (auto& pr : v) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
    v.clear();
  }
}

// Records a start event for `stage` when profiling; returns the index to close with timed_end.
hipEvent_t timed_begin(ephdc_session* s, hipStream_t hs) {
  if (!s->profile) return nullptr;
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  (void)hipEventRecord(e, hs);
  return e;
}

void timed_end(ephdc_session* s, int stage, hipEvent_t start, hipStream_t hs) {
  if (!s->profile || !start) return;
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return;
  (void)hipEventRecord(e, hs);
  s->ev[stage].emplace_back(start, e);
}

void free_session(ephdc_session* s) {
  if (!s) return;
  drop_events(s);
  void* ptrs[] = {s->d_fwd, s->d_inv, s->d_inv_t, s->d_pc,   s->d_scatter,
                  s->d_model, s->d_gk, s->d_spow,  s->d_perm, s->d_ksc};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (s->done) (void)hipEventDestroy(s->done);
  delete s;
}

PrimeConst make_const(const HostNtt& T) {
  PrimeConst pc{};
  const uint32_t m = T.m;
  uint32_t inv = 1;  // m^-1 mod 2^32 by Newton iteration
  for (int i = 0; i < 5; ++i) inv *= 2u - m * inv;
  pc.m = m;
  pc.mneg_inv = (uint32_t)(0u - inv);
  pc.r2 = (uint32_t)(((unsigned __int128)1 << 64) % m);
  pc.r1 = (uint32_t)((1ull << 32) % m);
  pc.ninv_r = (uint32_t)(((uint64_t)T.ninv << 32) % m);
  pc.ninv_w1_r = (uint32_t)(((((uint64_t)T.ninv * T.iw[1]) % m) << 32) % m);
  return pc;
}

// Work decomposition of one scoring launch: G groups x S splits of the M model
// ciphertexts x nlg limb groups, aiming at kTargetBlocks workgroups.
struct Schedule {
  uint32_t G, S, mchunk;
};

Schedule schedule(const ephdc_session* s, uint32_t Q) {
  Schedule sc{};
  sc.G = s->P.G(Q);
  const uint32_t M = s->P.M();
  const uint32_t per = std::max<uint32_t>(1, sc.G * s->nlg);
  uint32_t S = std::max<uint32_t>(1, (s->target_blocks + per - 1) / per);
  S = std::min(S, M);
  sc.mchunk = (M + S - 1) / S;
  sc.S = (M + sc.mchunk - 1) / sc.mchunk;
  return sc;
}

ScoreArgs score_args(const ephdc_session* s, const int8_t* d_hv, uint32_t Q, const Schedule& sc,
                     const Workspace* ws) {
  const ParamSet& P = s->P;
  ScoreArgs a{};
  a.model = s->d_model;
  a.hv = d_hv;
  a.partial = ws ? ws->partial : nullptr;
  a.scatter = s->d_scatter;
  a.fwd_tw = s->d_fwd;
  a.inv_t = s->d_inv_t;
  a.pcs = s->d_pc;
  a.pct = s->pct;
  a.L = P.L;
  a.M = P.M();
  a.D = P.D;
  a.r = P.r;
  a.hv_stride = P.G(Q) * P.B();
  a.B = P.B();
  a.G = sc.G;
  a.q_last = Q ? Q - (P.G(Q) - 1) * P.B() : 0;
  a.S = sc.S;
  a.mchunk = sc.mchunk;
  a.NLG = s->nlg;
  a.m_base = 0;
  a.m_len = P.M();
  a.pt = ws ? ws->pt : nullptr;
  a.accumulate = 0;
  a.scale = scale_op(s);
  a.sub_logn = s->sub_logn;
  a.sub_logk = s->sub_logn ? (uint32_t)P.logn - s->sub_logn : 0;
  a.pct_sub = s->pct_sub;
  return a;
}

constexpr size_t kPtBytes = (size_t)4 << 30;  // default plaintext chunk of ephdc_workspace_bytes

// Split path: the model range is processed in chunks of m_len ciphertexts so that the
// lifted plaintexts of a chunk (G x m_len x N int32) fit the workspace's buffer; the MAC
// kernel of every chunk after the first adds into the stored partial sums.
hipError_t score_split(ephdc_session* s, ScoreArgs a, const Schedule& sc, size_t pt_cap, hipStream_t hs) {
  const ParamSet& P = s->P;
  const uint32_t M = P.M();
  if (sc.G > pt_cap) return hipErrorInvalidValue;  // cannot happen: cap >= G(max_Q) >= G
  const uint32_t mc = (uint32_t)std::max<size_t>(1, std::min<size_t>(M, pt_cap / sc.G));
  const uint32_t blocks_enc = std::max<uint32_t>(1, s->target_blocks);
  for (uint32_t base = 0; base < M; base += mc) {
    const uint32_t len = std::min(mc, M - base);
    ScoreArgs c = a;
    c.m_base = base;
    c.m_len = len;
    c.accumulate = base > 0;
    // encode: G x Se work items over the chunk
    uint32_t Se = std::max<uint32_t>(1, std::min(len, (blocks_enc + sc.G - 1) / sc.G));
    c.mchunk = (len + Se - 1) / Se;
    Se = (len + c.mchunk - 1) / c.mchunk;
    hipEvent_t t0 = timed_begin(s, hs);
    hipError_t e = launch_encode_pt(P.logn, (int)s->le, c, sc.G * Se, hs);
    if (e != hipSuccess) return e;
    timed_end(s, kStEncodePt, t0, hs);
    // MAC: G x S x nlg work items; the S splits of every chunk cover the chunk
    c.S = sc.S;
    c.mchunk = (len + sc.S - 1) / sc.S;
    t0 = timed_begin(s, hs);
    e = launch_mac(P.logn, (int)s->le, (int)s->lg, c, sc.G * sc.S * s->nlg, hs);
    if (e != hipSuccess) return e;
    timed_end(s, kStMac, t0, hs);
  }
  return hipSuccess;
}

// Subring layout: the batch-encoding kernel writes each query plaintext's n-point
// transforms for every limb (L*n words; a workspace that holds c N-word plaintexts holds
// c*N/(L*n) of them), then the streaming MAC reads the model once per chunk and group
// tile: work items of 512 evaluation positions x one limb x one to three tiles of four or
// eight groups x one split of the chunk, as many as fit the device at once.
hipError_t score_split_sub(ephdc_session* s, ScoreArgs a, uint32_t Q, size_t pt_cap, size_t partial_words,
                           Schedule& sc, hipStream_t hs) {
  const ParamSet& P = s->P;
  sc.G = P.G(Q);
  const uint32_t n = 1u << s->sub_logn;
  // the splits must fit the partial sums of the workspace and the smallest chunk the
  // plaintext buffer allows
  const size_t cap_pt = pt_cap * P.N / ((size_t)P.L * n);
  const size_t fit = partial_words / ((size_t)sc.G * 2 * P.L * P.N);
  sc.S = (uint32_t)std::max<size_t>(1, std::min<size_t>({sub_splits(P, sc.G), cap_pt / sc.G, fit}));
  a.G = sc.G;
  a.S = sc.S;
  return run_sub(s, a, pt_cap, s, hs);
}

uint2 shoup_pair(uint64_t w, uint32_t m) {
  w %= m;
  return make_uint2((uint32_t)w, (uint32_t)((w << 32) / m));
}

// Key-switching constants of every digit and modulus, laid out as KsConst describes:
// up_inv[L] | up_mul[dnum][ds][nmod] | down_inv[alpha] | down_mul[alpha][L] | pinv[L].
std::vector<uint2> ks_constants(const ParamSet& P) {
  const uint32_t L = P.L, A = P.alpha, dn = P.dnum, ds = P.digit_size(), nm = P.nmod();
  std::vector<uint2> c;
  c.reserve(L + (size_t)dn * ds * nm + A + (size_t)A * L + L);
  // Q_j / q_i reduced mod m: product of the other limbs of digit j
  auto qhat = [&](uint32_t j, uint32_t i, uint64_t m) {
    uint64_t v = 1 % m;
    for (uint32_t k = j * ds; k < std::min(L, (j + 1) * ds); ++k)
      if (k != i) v = mulmod64(v, P.q[k] % m, m);
    return v;
  };
  auto phat = [&](uint32_t kk, uint64_t m) {
    uint64_t v = 1 % m;
    for (uint32_t k = 0; k < A; ++k)
      if (k != kk) v = mulmod64(v, P.p[k] % m, m);
    return v;
  };
  for (uint32_t i = 0; i < L; ++i) c.push_back(shoup_pair(inv_mod(qhat(i / ds, i, P.q[i]), P.q[i]), P.q[i]));
  for (uint32_t j = 0; j < dn; ++j)
    for (uint32_t d = 0; d < ds; ++d)
      for (uint32_t m = 0; m < nm; ++m) {
        const uint32_t i = j * ds + d;
        const uint32_t mod = P.modulus(m);
        c.push_back(i < L ? shoup_pair(qhat(j, i, mod), mod) : make_uint2(0, 0));
      }
  for (uint32_t k = 0; k < A; ++k) c.push_back(shoup_pair(inv_mod(phat(k, P.p[k]), P.p[k]), P.p[k]));
  for (uint32_t k = 0; k < A; ++k)
    for (uint32_t i = 0; i < L; ++i) c.push_back(shoup_pair(phat(k, P.q[i]), P.q[i]));
  for (uint32_t i = 0; i < L; ++i) {
    uint64_t pm = 1;
    for (uint32_t k = 0; k < A; ++k) pm = mulmod64(pm, P.p[k] % P.q[i], P.q[i]);
    c.push_back(shoup_pair(inv_mod(pm, P.q[i]), P.q[i]));
  }
  return c;
}

// perm[i][x] = y with 2*brev(y)+1 = g_i * (2*brev(x)+1) mod 2N: evaluation position x of
// sigma_g(a) holds a at the point that sigma_g maps position x's point to.
std::vector<uint32_t> automorphism_perms(const ParamSet& P) {
  const uint32_t N = P.N, lg = P.logn, steps = P.log2r();
  std::vector<uint32_t> perm((size_t)steps * N);
  for (uint32_t i = 0; i < steps; ++i) {
    const uint64_t g = galois_element(P, i);
    for (uint32_t x = 0; x < N; ++x) {
      const uint64_t e = (g * (2ull * bitrev(x, lg) + 1)) % (2ull * N);
      perm[(size_t)i * N + x] = bitrev((uint32_t)((e - 1) / 2), lg);
    }
  }
  return perm;
}

}  // namespace

namespace ephdc {

uint32_t sub_splits(const ParamSet& P, uint32_t G) {
  const uint32_t per = mac_sub_items(P.N, P.L, G);
  const uint32_t S = std::max<uint32_t>(1, mac_sub_resident_blocks(G) / per);
  return std::min({S, P.M(), std::max<uint32_t>(1, kMaxBlocks / G)});
}

hipError_t run_sub(const ephdc_session* s, ScoreArgs a, size_t pt_cap, ephdc_session* timing, hipStream_t hs) {
  const ParamSet& P = s->P;
  const uint32_t M = P.M(), n = 1u << s->sub_logn, G = a.G, S = a.S;
  const uint32_t per = mac_sub_items(P.N, P.L, G);
  constexpr uint32_t kEncodeTransforms = 8192;
  const size_t cap = pt_cap * P.N / ((size_t)P.L * n);
  // the MAC's loads take 32-bit byte offsets from a round's first ciphertext: four
  // ciphertexts of transformed values (and of the model) must span less than 4 GiB
  if ((4 * (uint64_t)P.L * G + G) * n * 4 >= (1ull << 32) || 8ull * P.L * P.N * 4 >= (1ull << 32))
    return hipErrorInvalidValue;
  // chunks of mc ciphertexts; every chunk's MAC covers S splits (empty ones write or keep
  // their sums), so S <= mc keeps each split non-empty in full chunks
  const uint32_t mc = (uint32_t)std::max<size_t>(std::max<size_t>(1, S), std::min<size_t>(M, cap / G));
  if ((size_t)mc * G > cap && mc > 1) return hipErrorInvalidValue;  // cannot happen: cap >= G * S
  for (uint32_t base = 0; base < M; base += mc) {
    const uint32_t len = std::min(mc, M - base);
    ScoreArgs c = a;
    c.m_base = base;
    c.m_len = len;
    c.accumulate = base > 0;
    // batch encoding: about kEncodeTransforms transforms in flight, one per (group, split)
    uint32_t Se = std::max<uint32_t>(1, std::min(len, (kEncodeTransforms + G - 1) / G));
    c.mchunk = (len + Se - 1) / Se;
    Se = (len + c.mchunk - 1) / c.mchunk;
    hipEvent_t t0 = timing ? timed_begin(timing, hs) : nullptr;
    hipError_t e = launch_encode_sub((int)s->sub_logn, c, Se, hs);
    if (e != hipSuccess) return e;
    if (timing) timed_end(timing, kStEncodePt, t0, hs);
    c.mchunk = (len + S - 1) / S;
    t0 = timing ? timed_begin(timing, hs) : nullptr;
    e = launch_mac_sub(P.logn, (int)s->sub_logn, c, per * S, hs);
    if (e != hipSuccess) return e;
    if (timing) timed_end(timing, kStMac, t0, hs);
  }
  return hipSuccess;
}

ScoreArgs sub_group_args(const ephdc_session* s, const SubGroup* d_vg, uint32_t VG, uint32_t S, uint32_t* partial,
                         int32_t* pt) {
  const ParamSet& P = s->P;
  ScoreArgs a{};
  a.model = s->d_model;
  a.fwd_tw = s->d_fwd;
  a.inv_t = s->d_inv_t;
  a.pcs = s->d_pc;
  a.pct = s->pct;
  a.L = P.L;
  a.M = P.M();
  a.D = P.D;
  a.r = P.r;
  a.B = P.B();
  a.G = VG;
  a.S = S;
  a.NLG = P.L;
  a.m_len = P.M();
  a.partial = partial;
  a.pt = pt;
  a.scale = scale_op(s);
  a.sub_logn = s->sub_logn;
  a.sub_logk = (uint32_t)P.logn - s->sub_logn;
  a.pct_sub = s->pct_sub;
  a.vg = d_vg;
  return a;
}

size_t score_partial_words(const ephdc_session* s, uint32_t Q) {
  const Schedule sc = schedule(s, Q);
  const uint32_t S = s->sub_logn ? std::max(sc.S, sub_splits(s->P, sc.G)) : sc.S;
  return (size_t)sc.G * S * 2 * s->P.L * s->P.N;
}

ScaleOp scale_op(const ephdc_session* s) {
  ScaleOp so{};
  so.pow = s->d_spow;
  so.g = s->P.scale_every ? s->P.scale_every : 1;
  so.nb = s->P.scale_blocks();
  return so;
}

// Words of the rotation workspace for G groups: acc, R [G][2][L][N]; D [G][L][N];
// Y [G][dnum][nmod][N]; KS [G][2][nmod][N]; XP [G][2][alpha][N].
size_t rotate_words(const ParamSet& P, uint32_t G) {
  const size_t N = P.N;
  return (size_t)G * N * (4 * P.L + P.L + (size_t)P.dnum * P.nmod() + 2 * P.nmod() + 2 * P.alpha);
}

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct WsSizes {
  size_t partial_words, rot_words, gmax;
};

// G*S <= target/nlg + G for any schedule, so the partial sums cover every target up to
// kMaxBlocks workgroups.
WsSizes ws_sizes(const ParamSet& P, uint32_t max_Q) {
  WsSizes z;
  z.gmax = P.G(max_Q);
  z.partial_words = ((size_t)kMaxBlocks + z.gmax) * 2 * P.L * P.N;
  z.rot_words = P.r > 1 ? rotate_words(P, (uint32_t)z.gmax) : 0;
  return z;
}

}  // namespace

size_t workspace_min_bytes(const ParamSet& P, uint32_t max_Q) {
  const WsSizes z = ws_sizes(P, max_Q);
  return align256(z.partial_words * 4) + align256(z.rot_words * 4) + z.gmax * P.N * 4;
}

size_t workspace_default_bytes(const ParamSet& P, uint32_t max_Q) {
  const WsSizes z = ws_sizes(P, max_Q);
  const size_t cap = std::max<size_t>(z.gmax, std::min<size_t>(z.gmax * P.M(), kPtBytes / (4 * (size_t)P.N)));
  return align256(z.partial_words * 4) + align256(z.rot_words * 4) + cap * P.N * 4;
}

ephdc_status workspace_layout(const ParamSet& P, uint32_t max_Q, void* base, size_t bytes, Workspace* out) {
  const WsSizes z = ws_sizes(P, max_Q);
  if ((uintptr_t)base & 255) return fail(EPHDC_ERR_ARG, "the workspace must be 256-byte aligned");
  if (bytes < workspace_min_bytes(P, max_Q))
    return fail(EPHDC_ERR_BUFFER, "workspace of " + std::to_string(bytes) + " bytes, needs at least " +
                                      std::to_string(workspace_min_bytes(P, max_Q)) + " (ephdc_workspace_bytes)");
  char* p = static_cast<char*>(base);
  Workspace w;
  w.partial = reinterpret_cast<uint32_t*>(p);
  w.partial_words = z.partial_words;
  p += align256(z.partial_words * 4);
  w.rot = z.rot_words ? reinterpret_cast<uint32_t*>(p) : nullptr;
  p += align256(z.rot_words * 4);
  w.pt = reinterpret_cast<int32_t*>(p);
  w.pt_cap = (bytes - (size_t)(p - static_cast<char*>(base))) / (4 * (size_t)P.N);
  *out = w;
  return EPHDC_OK;
}

ephdc_status score_with(ephdc_session* s, const Workspace& ws, const int8_t* d_hv, uint32_t Q,
                        uint32_t* d_score_ct, hipStream_t hs) {
  const ParamSet& P = s->P;
  Schedule sc = schedule(s, Q);
  if ((size_t)sc.G * sc.S * 2 * P.L * P.N > ws.partial_words) return fail(EPHDC_ERR_BUFFER, "scratch too small");
  if ((uint64_t)P.D * P.G(Q) * P.B() >= (1ull << 31)) return fail(EPHDC_ERR_UNSUPPORTED, "D * hv stride must be < 2^31");
  // a call on another stream than the previous one waits for the previous one, whose
  // scratch it reuses
  if (s->done_set && s->done_stream != hs) HIP_TRY(hipStreamWaitEvent(hs, s->done, 0), "stream ordering");
  ScoreArgs a = score_args(s, d_hv, Q, sc, &ws);
  // the n-point kernels read each lane's queries as one aligned vector of E bytes
  const bool sub = s->sub_logn && ((uintptr_t)d_hv & 15) == 0;
  if (sub) {
    size_t cap = ws.pt_cap;
    if (s->pt_bytes) cap = std::max<size_t>(sc.G, std::min(cap, s->pt_bytes / (4 * (size_t)P.N)));
    HIP_TRY(score_split_sub(s, a, Q, cap, ws.partial_words, sc, hs), "subring score launch");
  } else if (s->split) {
    size_t cap = ws.pt_cap;
    if (s->pt_bytes) cap = std::max<size_t>(sc.G, std::min(cap, s->pt_bytes / (4 * (size_t)P.N)));
    HIP_TRY(score_split(s, a, sc, cap, hs), "split score launch");
  } else {
    hipEvent_t t0 = timed_begin(s, hs);
    HIP_TRY(launch_score(P.logn, (int)s->le, (int)s->lg, a, sc.G * sc.S * s->nlg, hs), "score launch");
    timed_end(s, kStFused, t0, hs);
  }
  if (P.r == 1) {
    hipEvent_t t1 = timed_begin(s, hs);
    HIP_TRY(launch_finish(P.logn, true, ws.partial, d_score_ct, sc.G, sc.S, P.L, s->d_inv, s->d_pc, hs),
            "finish launch");
    timed_end(s, kStFinish, t1, hs);
  } else {
    // r > 1: sum the partials in the evaluation domain, fold the r blocks of every row with
    // log2 r rotations, then return to the coefficient domain
    RotateArgs ra = rotate_args(s, ws.rot, sc.G);
    hipEvent_t t1 = timed_begin(s, hs);
    HIP_TRY(launch_finish(P.logn, false, ws.partial, ra.acc, sc.G, sc.S, P.L, s->d_inv, s->d_pc, hs),
            "finish launch");
    timed_end(s, kStFinish, t1, hs);
    hipEvent_t t2 = timed_begin(s, hs);
    for (uint32_t i = 0; i < P.log2r(); ++i) HIP_TRY(launch_rotate_step(P.logn, ra, i, hs), "rotate launch");
    HIP_TRY(launch_inv_batch(P.logn, ra.acc, d_score_ct, (size_t)sc.G * 2 * P.L, s->d_inv, s->d_pc, P.L, 0, hs),
            "output transform launch");
    timed_end(s, kStRotate, t2, hs);
  }
  HIP_TRY(hipEventRecord(s->done, hs), "completion event");
  s->done_stream = hs;
  s->done_set = true;
  return EPHDC_OK;
}

RotateArgs rotate_args(const ephdc_session* s, uint32_t* workspace, uint32_t G) {
  const ParamSet& P = s->P;
  const size_t N = P.N;
  RotateArgs r{};
  r.k = s->ks;
  r.k.G = G;
  r.perm = s->d_perm;
  r.ksk = s->d_gk;
  uint32_t* w = workspace;
  r.acc = w;  w += (size_t)G * 2 * P.L * N;
  r.R = w;    w += (size_t)G * 2 * P.L * N;
  r.D = w;    w += (size_t)G * P.L * N;
  r.Y = w;    w += (size_t)G * P.dnum * P.nmod() * N;
  r.KS = w;   w += (size_t)G * 2 * P.nmod() * N;
  r.XP = w;
  r.fwd_tw = s->d_fwd;
  r.inv_tw = s->d_inv;
  r.pcs = s->d_pc;
  return r;
}

}  // namespace ephdc

extern "C" {

size_t ephdc_workspace_bytes(const ephdc_params* prm, uint32_t max_Q) {
  ParamSet P;
  if (P.load(prm) != EPHDC_OK || max_Q == 0) return 0;
  return workspace_default_bytes(P, max_Q);
}

ephdc_status ephdc_session_create(const ephdc_params* prm, const uint32_t* d_model_ct, size_t model_words,
                                  const uint32_t* d_galois_keys, size_t gk_words, uint32_t max_Q,
                                  void* d_workspace, size_t ws_bytes, void* stream, ephdc_session** out) {
  return session_create(prm, d_model_ct, model_words, d_galois_keys, gk_words, max_Q, d_workspace, ws_bytes, stream,
                        true, out);
}

}  // extern "C"

ephdc_status ephdc::session_create(const ephdc_params* prm, const uint32_t* d_model_ct, size_t model_words,
                                   const uint32_t* d_galois_keys, size_t gk_words, uint32_t max_Q,
                                   void* d_workspace, size_t ws_bytes, void* stream, bool mac_primes,
                                   ephdc_session** out) {
  if (!out) return fail(EPHDC_ERR_ARG, "out is NULL");
  *out = nullptr;
  ParamSet P;
  ephdc_status st = P.load(prm);
  if (st != EPHDC_OK) return st;
  if (!d_model_ct) return fail(EPHDC_ERR_ARG, "model is NULL");
  if (!supported_logn(P.logn)) return fail(EPHDC_ERR_UNSUPPORTED, "kernels implement N in {2048, 4096, 8192, 16384}");
  for (uint32_t qi : P.q) {
    if (mac_primes && qi < (1u << 29))
      return fail(EPHDC_ERR_UNSUPPORTED, "the device kernels take ciphertext primes in [2^29, 2^30)");
    if (qi <= P.t) return fail(EPHDC_ERR_UNSUPPORTED, "the device kernels take ciphertext primes above t");
  }
  if (P.r > 1 && !d_galois_keys) return fail(EPHDC_ERR_NOKEY, "r > 1 needs Galois keys");
  if (max_Q == 0) return fail(EPHDC_ERR_ARG, "max_Q must be positive");
  if (model_words < (size_t)P.M() * 2 * P.L * P.N) return fail(EPHDC_ERR_BUFFER, "model buffer shorter than [M][2][L][N]");
  if (P.r > 1 && gk_words < (size_t)P.log2r() * P.dnum * 2 * P.nmod() * P.N)
    return fail(EPHDC_ERR_BUFFER, "Galois key buffer shorter than [log2 r][dnum][2][L+alpha][N]");
  Workspace ws;
  if (d_workspace && (st = workspace_layout(P, max_Q, d_workspace, ws_bytes, &ws)) != EPHDC_OK) return st;
  hipStream_t hs = (hipStream_t)stream;
  HIP_TRY(prepare_kernels(), "kernel setup");

  ephdc_session* s = new ephdc_session();
  s->P = P;
  s->max_Q = max_Q;
  s->ws = ws;
  s->has_ws = d_workspace != nullptr;
  if (hipEventCreateWithFlags(&s->done, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    s->done = nullptr;
    free_session(s);
    return fail(EPHDC_ERR_HIP, "event creation failed");
  }
  (void)hipGetDevice(&s->device);
  // default schedule (measured on MI355X at N = 8192, L = 4, 4096 queries): split path,
  // 8 values per thread, one limb per MAC work item; one MAC workgroup per compute unit
  // (256) from N = 8192 up, whose transform kernels hold one workgroup per CU, 512 below
  s->split = true;
  s->le = P.logn == 13 ? 3 : 0;
  s->lg = 1;
  s->nlg = P.L;
  s->target_blocks = P.logn >= 13 ? 256 : 512;

  const uint32_t N = P.N, nm = P.nmod();
  std::vector<uint32_t> fwd((size_t)nm * N), inv((size_t)nm * N), invt(N);
  std::vector<PrimeConst> pcs(nm);
  for (uint32_t i = 0; i < nm; ++i) {
    uint32_t m = P.modulus(i);
    HostNtt T(N, m, root_of_unity(2 * N, m));
    for (uint32_t k = 0; k < N; ++k) {
      fwd[(size_t)i * N + k] = (uint32_t)(((uint64_t)T.fw[k] << 32) % m);
      inv[(size_t)i * N + k] = (uint32_t)(((uint64_t)T.iw[k] << 32) % m);
    }
    pcs[i] = make_const(T);
  }
  {
    HostNtt Tt(N, P.t, root_of_unity(2 * N, P.t));
    for (uint32_t k = 0; k < N; ++k) invt[k] = (uint32_t)(((uint64_t)Tt.iw[k] << 32) % P.t);
    s->pct = make_const(Tt);
    if (P.subring()) {
      // n-point transforms of p~ in p(X) = p~(X^K'): the same tables (their first n words),
      // with n^-1 in the scaling stage of the inverse
      const uint32_t n = N / P.Kp();
      if (subring_kernels(P.logn, ilog2(n))) {
        s->sub_logn = (uint32_t)ilog2(n);
        s->pct_sub = s->pct;
        const uint64_t ninv = inv_mod(n, P.t);
        s->pct_sub.ninv_r = (uint32_t)((ninv << 32) % P.t);
        s->pct_sub.ninv_w1_r = (uint32_t)((((ninv * Tt.iw[1]) % P.t) << 32) % P.t);
      }
    }
  }
  std::vector<uint32_t> scatter = query_scatter_table(P);

  const size_t M = P.M();
  const size_t model_copy_words = M * 2 * P.L * N;
  const size_t key_words = P.r > 1 ? (size_t)P.log2r() * P.dnum * 2 * nm * N : 0;
  // scaling op: c^e * 2^32 mod q_l for e = 0 .. scale_blocks
  std::vector<uint32_t> spow;
  if (P.scale_every) {
    const uint32_t nb = P.scale_blocks();
    const int64_t c = P.scale_const();
    spow.resize((size_t)P.L * (nb + 1));
    for (uint32_t l = 0; l < P.L; ++l) {
      const uint64_t ql = P.q[l], cl = c < 0 ? ql - (uint64_t)(-c) % ql : (uint64_t)c % ql;
      uint64_t pw = 1;
      for (uint32_t e = 0; e <= nb; ++e, pw = mulmod64(pw, cl, ql)) spow[(size_t)l * (nb + 1) + e] = (uint32_t)((pw << 32) % ql);
    }
  }

  auto cleanup = [&](ephdc_status e) { free_session(s); return e; };
  if ((st = dev_alloc(s, &s->d_fwd, fwd.size(), "twiddles")) != EPHDC_OK) return cleanup(st);
  if ((st = dev_alloc(s, &s->d_inv, inv.size(), "twiddles")) != EPHDC_OK) return cleanup(st);
  if ((st = dev_alloc(s, &s->d_inv_t, invt.size(), "twiddles")) != EPHDC_OK) return cleanup(st);
  if ((st = dev_alloc(s, &s->d_pc, pcs.size(), "constants")) != EPHDC_OK) return cleanup(st);
  if ((st = dev_alloc(s, &s->d_scatter, scatter.size(), "scatter table")) != EPHDC_OK) return cleanup(st);
  if ((st = dev_alloc(s, &s->d_model, model_copy_words, "model")) != EPHDC_OK) return cleanup(st);
  if ((st = dev_alloc(s, &s->d_gk, key_words, "Galois keys")) != EPHDC_OK) return cleanup(st);
  if ((st = dev_alloc(s, &s->d_spow, spow.size(), "scaling constants")) != EPHDC_OK) return cleanup(st);
  std::vector<uint32_t> perm;
  std::vector<uint2> ksc;
  if (P.r > 1) {
    perm = automorphism_perms(P);
    ksc = ks_constants(P);
    if ((st = dev_alloc(s, &s->d_perm, perm.size(), "automorphism tables")) != EPHDC_OK) return cleanup(st);
    if ((st = dev_alloc(s, &s->d_ksc, ksc.size(), "key-switching constants")) != EPHDC_OK) return cleanup(st);
    KsConst& k = s->ks;
    const uint2* c = s->d_ksc;
    k.up_inv = c;    c += P.L;
    k.up_mul = c;    c += (size_t)P.dnum * P.digit_size() * nm;
    k.down_inv = c;  c += P.alpha;
    k.down_mul = c;  c += (size_t)P.alpha * P.L;
    k.pinv = c;
    k.L = P.L;
    k.alpha = P.alpha;
    k.dnum = P.dnum;
    k.ds = P.digit_size();
    k.nmod = nm;
  }

  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
  chk(hipMemcpyAsync(s->d_fwd, fwd.data(), fwd.size() * sizeof(uint32_t), hipMemcpyHostToDevice, hs));
  chk(hipMemcpyAsync(s->d_inv, inv.data(), inv.size() * sizeof(uint32_t), hipMemcpyHostToDevice, hs));
  chk(hipMemcpyAsync(s->d_inv_t, invt.data(), invt.size() * sizeof(uint32_t), hipMemcpyHostToDevice, hs));
  chk(hipMemcpyAsync(s->d_pc, pcs.data(), pcs.size() * sizeof(PrimeConst), hipMemcpyHostToDevice, hs));
  chk(hipMemcpyAsync(s->d_scatter, scatter.data(), scatter.size() * sizeof(uint32_t), hipMemcpyHostToDevice, hs));
  if (!spow.empty())
    chk(hipMemcpyAsync(s->d_spow, spow.data(), spow.size() * sizeof(uint32_t), hipMemcpyHostToDevice, hs));
  if (P.r > 1) {
    chk(hipMemcpyAsync(s->d_perm, perm.data(), perm.size() * sizeof(uint32_t), hipMemcpyHostToDevice, hs));
    chk(hipMemcpyAsync(s->d_ksc, ksc.data(), ksc.size() * sizeof(uint2), hipMemcpyHostToDevice, hs));
  }
  if (e == hipSuccess)
    e = launch_fwd_batch(P.logn, d_model_ct, s->d_model, M * 2 * P.L, s->d_fwd, s->d_pc, P.L, 0, true, hs);
  if (e == hipSuccess && key_words)
    e = launch_fwd_batch(P.logn, d_galois_keys, s->d_gk, key_words / N, s->d_fwd, s->d_pc, nm, 0, true, hs);
  if (e == hipSuccess) e = hipStreamSynchronize(hs);
  if (e != hipSuccess) {
    free_session(s);
    return hip_fail(e, "session setup");
  }
  *out = s;
  return EPHDC_OK;
}

extern "C" {

ephdc_status ephdc_session_destroy(ephdc_session* s) {
  if (!s) return fail(EPHDC_ERR_ARG, "session is NULL");
  // the session's own calls are done once its last scoring call is (setup was synchronous)
  if (s->done_set) (void)hipEventSynchronize(s->done);
  free_session(s);
  return EPHDC_OK;
}

size_t ephdc_session_device_bytes(const ephdc_session* s) { return s ? s->device_bytes : 0; }

ephdc_status ephdc_encode_queries(ephdc_session* s, const uint8_t* d_x, const int8_t* d_base, uint32_t Q,
                                  int8_t* d_hv, void* stream) {
  if (!s || !d_x || !d_base || !d_hv) return fail(EPHDC_ERR_ARG, "NULL argument");
  const ParamSet& P = s->P;
  if (Q == 0 || Q > s->max_Q) return fail(EPHDC_ERR_ARG, "Q must be in [1, max_Q]");
  if (P.F % 16 != 0 || P.D % 64 != 0) return fail(EPHDC_ERR_UNSUPPORTED, "encoding needs F % 16 == 0 and D % 64 == 0");
  if ((uint64_t)P.F * P.D >= (1ull << 31) || (uint64_t)Q * P.F >= (1ull << 31))
    return fail(EPHDC_ERR_UNSUPPORTED, "encoding needs F * D and Q * F below 2^31");
  if (((uintptr_t)d_x & 15) || ((uintptr_t)d_base & 3)) return fail(EPHDC_ERR_ARG, "x must be 16-byte and base 4-byte aligned");
  if ((uint64_t)P.D * P.G(Q) * P.B() >= (1ull << 31)) return fail(EPHDC_ERR_UNSUPPORTED, "D * hv stride must be < 2^31");
  hipStream_t hs = (hipStream_t)stream;
  hipEvent_t t0 = timed_begin(s, hs);
  HIP_TRY(launch_hdc_encode(d_x, d_base, d_hv, Q, P.F, P.D, P.G(Q) * P.B(), P.qbits, P.qshift, hs),
          "encode launch");
  timed_end(s, kStHdc, t0, hs);
  return EPHDC_OK;
}

ephdc_status ephdc_score_encrypted(ephdc_session* s, const int8_t* d_hv, uint32_t Q, uint32_t* d_score_ct,
                                   void* stream) {
  if (!s || !d_hv || !d_score_ct) return fail(EPHDC_ERR_ARG, "NULL argument");
  if (Q == 0 || Q > s->max_Q) return fail(EPHDC_ERR_ARG, "Q must be in [1, max_Q]");
  if (!s->has_ws) return fail(EPHDC_ERR_BUFFER, "the session was created without a workspace");
  return score_with(s, s->ws, d_hv, Q, d_score_ct, (hipStream_t)stream);
}

ephdc_status ephdc_session_tune(ephdc_session* s, uint32_t limb_group, uint32_t blocks, uint32_t values_per_thread,
                                uint32_t mode) {
  if (!s) return fail(EPHDC_ERR_ARG, "session is NULL");
  if (mode > 2) return fail(EPHDC_ERR_ARG, "mode must be 0 (keep), 1 (fused) or 2 (split)");
  if (mode) s->split = mode == 2;
  if (values_per_thread) {
    const int le = ilog2(values_per_thread);
    if ((1u << le) != values_per_thread || !supported_shape(s->P.logn, le))
      return fail(EPHDC_ERR_UNSUPPORTED, "no scoring kernel with that many values per thread for this N");
    s->le = (uint32_t)le;
  }
  if (limb_group) {
    if (limb_group > 4 || s->P.L % limb_group) return fail(EPHDC_ERR_ARG, "limb_group must divide L and be <= 4");
    if (limb_group == 3 && s->split) return fail(EPHDC_ERR_UNSUPPORTED, "the split path takes limb groups of 1, 2 or 4");
    s->lg = limb_group;
    s->nlg = s->P.L / limb_group;
  }
  if (blocks) {
    if (blocks > kMaxBlocks) return fail(EPHDC_ERR_ARG, "blocks must be <= 1024");
    s->target_blocks = blocks;
  }
  return EPHDC_OK;
}

ephdc_status ephdc_session_set_chunk_bytes(ephdc_session* s, size_t bytes) {
  if (!s) return fail(EPHDC_ERR_ARG, "session is NULL");
  s->pt_bytes = bytes;
  return EPHDC_OK;
}

ephdc_status ephdc_session_profile(ephdc_session* s, int enable) {
  if (!s) return fail(EPHDC_ERR_ARG, "session is NULL");
  s->profile = enable != 0;
  return EPHDC_OK;
}

ephdc_status ephdc_session_profile_read(ephdc_session* s, double ms[6], uint64_t count[6]) {
  if (!s || !ms || !count) return fail(EPHDC_ERR_ARG, "NULL argument");
  for (int k = 0; k < kStages; ++k) {
    ms[k] = 0.0;
    count[k] = 0;
    for (auto& pr : s->ev[k]) {
      HIP_TRY(hipEventSynchronize(pr.second), "event sync");
      float t = 0.f;
      HIP_TRY(hipEventElapsedTime(&t, pr.first, pr.second), "event time");
      ms[k] += t;
      ++count[k];
    }
  }
  drop_events(s);
  return EPHDC_OK;
}

ephdc_status ephdc_debug_plaintext(ephdc_session* s, const int8_t* d_hv, uint32_t Q, uint32_t g, uint32_t m,
                                   uint32_t* d_out, void* stream) {
  if (!s || !d_hv || !d_out) return fail(EPHDC_ERR_ARG, "NULL argument");
  const ParamSet& P = s->P;
  if (Q == 0 || g >= P.G(Q) || m >= P.M()) return fail(EPHDC_ERR_ARG, "g or m out of range");
  Schedule sc = schedule(s, Q);
  ScoreArgs a = score_args(s, d_hv, Q, sc, nullptr);
  HIP_TRY(launch_debug_plaintext(P.logn, a, g, m, d_out, (hipStream_t)stream), "debug launch");
  return EPHDC_OK;
}

ephdc_status ephdc_debug_polymul(ephdc_session* s, const uint32_t* d_a, const uint32_t* d_b, uint32_t count,
                                 uint32_t* d_out, void* stream) {
  if (!s || !d_a || !d_b || !d_out) return fail(EPHDC_ERR_ARG, "NULL argument");
  if (count == 0) return EPHDC_OK;
  const ParamSet& P = s->P;
  hipStream_t hs = (hipStream_t)stream;
  const size_t n = (size_t)count * P.N;
  uint32_t *ta = nullptr, *tb = nullptr;
  if (hipMalloc((void**)&ta, n * 4) != hipSuccess || hipMalloc((void**)&tb, n * 4) != hipSuccess) {
    if (ta) (void)hipFree(ta);
    (void)hipGetLastError();
    return fail(EPHDC_ERR_OOM, "debug buffers");
  }
  hipError_t e = launch_fwd_batch(P.logn, d_a, ta, count, s->d_fwd, s->d_pc, P.L, 0, true, hs);
  if (e == hipSuccess) e = launch_fwd_batch(P.logn, d_b, tb, count, s->d_fwd, s->d_pc, P.L, 0, false, hs);
  if (e == hipSuccess) e = launch_pointwise_mont(ta, tb, ta, n, P.N, s->d_pc, P.L, hs);
  if (e == hipSuccess) e = launch_inv_batch(P.logn, ta, d_out, count, s->d_inv, s->d_pc, P.L, 0, hs);
  if (e == hipSuccess) e = hipStreamSynchronize(hs);
  (void)hipFree(ta);
  (void)hipFree(tb);
  if (e != hipSuccess) return hip_fail(e, "debug polymul");
  return EPHDC_OK;
}

}  // extern "C"
