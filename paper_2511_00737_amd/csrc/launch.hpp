// Kernel argument blocks and host-side launchers of the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_ntt.hpp"

namespace ephdc_dev {

// Arguments of the fused scoring kernel (and the debug plaintext kernel).
struct ScoreArgs {
  const uint32_t* model;    // [M][2][L][N] evaluation domain, Montgomery form
  const int8_t* hv;         // [D][hv_stride] query hypervectors
  uint32_t* partial;        // [G][S][2][L][N] evaluation-domain partial sums
  const uint32_t* scatter;  // [N] slot source of every evaluation-side position
  const uint2* fwd_tw;      // [L+alpha][N] forward twiddles (w, w')
  const uint2* inv_t;       // [N] inverse twiddles mod t
  const PrimeConst* pcs;    // [L+alpha]
  PrimeConst pct;           // constants of t
  uint32_t tninv, tninvp;   // N^-1 mod t and Shoup companion
  uint32_t L, M, D, r, hv_stride, B, G, S, mchunk, NLG;
  // work covers model ciphertexts [m_base, m_base + m_len); splits cut that range
  uint32_t m_base, m_len;
  // split path: lifted plaintext coefficients [G][m_len][N] (int32 in (-t/2, t/2]) written
  // by the batch-encode kernel and read by the MAC kernel; with accumulate set, the MAC
  // kernel adds to the partial sums already stored instead of overwriting them
  int32_t* pt;
  uint32_t accumulate;
};

}  // namespace ephdc_dev

namespace ephdc {

using ephdc_dev::PrimeConst;
using ephdc_dev::ScoreArgs;

hipError_t prepare_kernels();
bool supported_logn(int logn);

hipError_t launch_fwd_batch(int logn, const uint32_t* in, uint32_t* out, size_t npolys, const uint2* tw,
                            const PrimeConst* pcs, uint32_t nlimb, uint32_t limb_base, bool mont,
                            hipStream_t st);
hipError_t launch_inv_batch(int logn, const uint32_t* in, uint32_t* out, size_t npolys, const uint2* itw,
                            const PrimeConst* pcs, uint32_t nlimb, uint32_t limb_base, hipStream_t st);
hipError_t launch_pointwise_mont(const uint32_t* a, const uint32_t* b, uint32_t* out, size_t n, uint32_t N,
                                 const PrimeConst* pcs, uint32_t nlimb, hipStream_t st);
hipError_t launch_score(int logn, int le, int lg, const ScoreArgs& a, uint32_t nblocks, hipStream_t st);
// split path: batch-encode every (g, m) plaintext of the launch into a.pt, then MAC
hipError_t launch_encode_pt(int logn, int le, const ScoreArgs& a, uint32_t nblocks, hipStream_t st);
hipError_t launch_mac(int logn, int le, int lg, const ScoreArgs& a, uint32_t nblocks, hipStream_t st);
bool supported_shape(int logn, int le);
hipError_t launch_finish(int logn, bool invert, const uint32_t* partial, uint32_t* out, uint32_t G, uint32_t S,
                         uint32_t L, const uint2* itw, const PrimeConst* pcs, hipStream_t st);
hipError_t launch_debug_plaintext(int logn, const ScoreArgs& a, uint32_t g, uint32_t m, uint32_t* out,
                                  hipStream_t st);

// HDC projection: hv[j][q] = quantise(sum_f (x[q][f]-128) * base[f][j]) for q < Q, 0 for Q <= q < stride.
hipError_t launch_hdc_encode(const uint8_t* x, const int8_t* base, int8_t* hv, uint32_t Q, uint32_t F,
                             uint32_t D, uint32_t stride, uint32_t qbits, uint32_t qshift, hipStream_t st);

}  // namespace ephdc
