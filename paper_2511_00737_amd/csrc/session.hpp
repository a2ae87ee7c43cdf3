// Session state shared by the single-request entry points (session.hip) and the request
// lists of batches and the serving loop (batch.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <utility>
#include <vector>

#include "launch.hpp"
#include "params.hpp"

// Profiling stages (see ephdc_session_profile_read).
enum : int { kStFused = 0, kStFinish = 1, kStHdc = 2, kStRotate = 3, kStEncodePt = 4, kStMac = 5, kStages = 6 };

namespace ephdc {

// Device scratch of one scoring call, carved from a caller-owned buffer: partial sums of
// the work items, the rotation workspace (r > 1) and the split path's plaintext chunk.
struct Workspace {
  uint32_t* partial = nullptr;  // [G][S][2][L][N] partial accumulators
  size_t partial_words = 0;
  uint32_t* rot = nullptr;      // acc, R, D, Y, KS, XP for G(max_Q) groups (r > 1)
  int32_t* pt = nullptr;        // lifted plaintexts of one chunk [G][m_len][N]
  size_t pt_cap = 0;            // plaintexts the chunk buffer holds (>= G(max_Q))
};

}  // namespace ephdc

struct ephdc_session {
  ephdc::ParamSet P;
  int device = 0;
  uint32_t max_Q = 0;
  uint32_t lg = 1, nlg = 1;        // limbs per fused work item, number of limb groups
  uint32_t target_blocks = 256;    // workgroups per scoring launch the schedule aims at
  uint32_t le = 0;                 // log2 values per thread of the scoring kernel (0: default)
  bool split = false;              // batch-encode and MAC as two kernels (else one fused kernel)
  size_t pt_bytes = 0;             // bound on the plaintext chunk in bytes (0: all of the workspace's)
  // the caller's workspace (borrowed; none when the session is used only through batches,
  // the serving loop or the static-scratch entry point)
  ephdc::Workspace ws;
  bool has_ws = false;
  // the last scoring call's completion, so that a call on another stream waits for it
  hipEvent_t done = nullptr;
  hipStream_t done_stream = nullptr;
  bool done_set = false;
  // device memory owned by the session
  uint32_t* d_fwd = nullptr;       // [nmod][N] forward twiddles, Montgomery form (w * 2^32 mod m)
  uint32_t* d_inv = nullptr;       // [nmod][N] inverse twiddles, Montgomery form
  uint32_t* d_inv_t = nullptr;     // [N] inverse twiddles mod t, Montgomery form
  ephdc::PrimeConst* d_pc = nullptr;  // [nmod]
  uint32_t* d_scatter = nullptr;   // [N]
  uint32_t* d_model = nullptr;     // [M][2][L][N] evaluation domain, Montgomery form
  uint32_t* d_gk = nullptr;        // [log2r][dnum][2][nmod][N] evaluation domain, Montgomery form
  uint32_t* d_spow = nullptr;      // scaling op: [L][scale_blocks + 1] powers c^e * 2^32 mod q_l
  // rotate-and-sum (r > 1)
  uint32_t* d_perm = nullptr;      // [log2r][N] automorphism permutations of evaluation points
  uint2* d_ksc = nullptr;          // key-switching constants, pointed into by ks
  ephdc::KsConst ks{};
  ephdc::PrimeConst pct{};
  // subring layout with n-point kernels: log2 n (0: the N-point kernels) and the n-point
  // constants of t
  uint32_t sub_logn = 0;
  ephdc::PrimeConst pct_sub{};
  size_t device_bytes = 0;
  // kernel timing: pairs of events per stage, resolved when read
  bool profile = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[kStages];
};

namespace ephdc {

inline constexpr uint32_t kTargetBlocks = 256;  // one workgroup per CU on MI355X (256 CUs)
inline constexpr uint32_t kMaxBlocks = 1024;    // largest schedule target the scratch is sized for

inline ephdc_status hip_fail(hipError_t e, const char* what) {
  return fail(EPHDC_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                          \
  do {                                               \
    hipError_t _e = (expr);                          \
    if (_e != hipSuccess) return hip_fail(_e, what); \
  } while (0)

template <class T>
inline ephdc_status dev_alloc(ephdc_session* s, T** p, size_t count, const char* what) {
  if (count == 0) { *p = nullptr; return EPHDC_OK; }
  hipError_t e = hipMalloc((void**)p, count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(EPHDC_ERR_OOM, std::string("hipMalloc failed for ") + what);
  }
  s->device_bytes += count * sizeof(T);
  return EPHDC_OK;
}

// Workspace of ephdc_score_encrypted for batches of up to max_Q queries: the layout of a
// buffer of `bytes` bytes at `base` (EPHDC_ERR_BUFFER when it is too small), and the size
// ephdc_workspace_bytes reports (the minimum plus a plaintext chunk of up to 512 MiB).
size_t workspace_min_bytes(const ParamSet& P, uint32_t max_Q);
size_t workspace_default_bytes(const ParamSet& P, uint32_t max_Q);
ephdc_status workspace_layout(const ParamSet& P, uint32_t max_Q, void* base, size_t bytes, Workspace* out);

// ephdc_session_create; with mac_primes false, ciphertext primes below 2^29 (but above t)
// are accepted, for callers that use the transforms and the batch encoding but not the
// multiply-accumulate kernels, whose lazy bounds need primes of at least 2^29.
ephdc_status session_create(const ephdc_params* prm, const uint32_t* d_model_ct, size_t model_words,
                            const uint32_t* d_galois_keys, size_t gk_words, uint32_t max_Q, void* d_workspace,
                            size_t ws_bytes, void* stream, bool mac_primes, ephdc_session** out);

// Words of the partial sums that scoring Q queries takes under the session's schedule.
size_t score_partial_words(const ephdc_session* s, uint32_t Q);

// The scaling op of a session's parameters (pow == nullptr when scale_every is 0).
ScaleOp scale_op(const ephdc_session* s);

// The scoring of ephdc_score_encrypted with the scratch of `ws`.
ephdc_status score_with(ephdc_session* s, const Workspace& ws, const int8_t* d_hv, uint32_t Q,
                        uint32_t* d_score_ct, hipStream_t hs);

// Subring kernels (sessions with sub_logn > 0): splits of the model range for G groups,
// and one scoring pass over the groups of `a` (a.G groups, a.S splits; a.vg may map them to
// the queries of several requests) with a plaintext buffer of pt_cap N-word plaintexts,
// which must hold G * S of the kernels' transformed plaintexts.  `timing`: the session whose
// kernel timers record the launches, or nullptr.
uint32_t sub_splits(const ParamSet& P, uint32_t G);
hipError_t run_sub(const ephdc_session* s, ScoreArgs a, size_t pt_cap, ephdc_session* timing, hipStream_t hs);
ScoreArgs sub_group_args(const ephdc_session* s, const SubGroup* d_vg, uint32_t VG, uint32_t S, uint32_t* partial,
                         int32_t* pt);

// Rotation workspace and arguments for G groups of a folded (r > 1) session.
size_t rotate_words(const ParamSet& P, uint32_t G);
RotateArgs rotate_args(const ephdc_session* s, uint32_t* workspace, uint32_t G);

}  // namespace ephdc
