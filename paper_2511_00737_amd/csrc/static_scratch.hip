// Scoring without any device allocation: ephdc_score_encrypted with its scratch in a fixed
// array of the library's device code instead of the session's workspace.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "session.hpp"

using namespace ephdc;

// The scratch: one copy of this array per GPU (each at its own device address), held until
// the process ends.  Host code never passes its name to a kernel or a copy; its device
// address comes from hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) uint32_t scratch[kStaticScratchBytes / 4];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Device address of `device`'s copy of the scratch (the device must be current).
ephdc_status static_scratch(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return fail(EPHDC_ERR_UNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur), "hipGetDevice");
    if (cur != device) return fail(EPHDC_ERR_ARG, "the session's device must be the current device");
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return EPHDC_OK;
}

}  // namespace

extern "C" {

ephdc_status ephdc_score_encrypted_static(ephdc_session* s, const int8_t* d_hv, uint32_t Q, uint32_t* d_score_ct,
                                          void* stream) {
  if (!s || !d_hv || !d_score_ct) return fail(EPHDC_ERR_ARG, "NULL argument");
  if (Q == 0 || Q > s->max_Q) return fail(EPHDC_ERR_ARG, "Q must be in [1, max_Q]");
  const ParamSet& P = s->P;
  // this call's needs: the partial sums of the current schedule, the rotation workspace of
  // its groups and at least one plaintext per group for the split path's chunks
  const uint32_t G = P.G(Q);
  const size_t partial = align256(score_partial_words(s, Q) * 4);
  const size_t rot = P.r > 1 ? align256(rotate_words(P, G) * 4) : 0;
  const size_t need = partial + rot + (size_t)G * P.N * 4;
  if (need > kStaticScratchBytes)
    return fail(EPHDC_ERR_UNSUPPORTED, "this call needs " + std::to_string(need) +
                                           " bytes of scratch; the static scratch holds " +
                                           std::to_string(kStaticScratchBytes));
  void* base = nullptr;
  ephdc_status st = static_scratch(s->device, &base);
  if (st != EPHDC_OK) return st;
  Workspace w;
  char* p = static_cast<char*>(base);
  w.partial = reinterpret_cast<uint32_t*>(p);
  w.partial_words = partial / 4;
  p += partial;
  w.rot = rot ? reinterpret_cast<uint32_t*>(p) : nullptr;
  p += rot;
  w.pt = reinterpret_cast<int32_t*>(p);
  w.pt_cap = (kStaticScratchBytes - partial - rot) / (4 * (size_t)P.N);
  return score_with(s, w, d_hv, Q, d_score_ct, (hipStream_t)stream);
}

}  // extern "C"
