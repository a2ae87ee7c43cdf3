// Kernel argument blocks and host-side launchers of the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_ntt.hpp"

namespace ephdc_dev {

// HE-aware scaling of the multiply-accumulate: after every g additions (model ciphertexts
// in order, nb complete blocks) the accumulator is multiplied by the plaintext scalar c.
// The product of ciphertext m is therefore weighted by c^e(m), e(m) = nb - floor(m/g) for
// m in a complete block and 0 in the trailing partial block; pow[l * (nb + 1) + e] holds
// c^e * 2^32 mod q_l (Montgomery form).  pow == nullptr: no scaling.
struct ScaleOp {
  const uint32_t* pow;
  uint32_t g, nb;
  __host__ __device__ uint32_t exponent(uint32_t m) const {
    const uint32_t b = m / g;
    return b < nb ? nb - b : 0u;
  }
};

// Where the queries of one (virtual) query group of the subring kernels come from: the
// group's first column in its request's hypervectors, their row pitch, and how many of the
// group's B query positions hold queries (the batch encoding reads the others as zero, so
// their columns need not be written).
struct SubGroup {
  const int8_t* hv;
  uint32_t stride, nq;
};

// Arguments of the fused scoring kernel (and the debug plaintext kernel).
struct ScoreArgs {
  const uint32_t* model;    // [M][2][L][N] evaluation domain, Montgomery form
  const int8_t* hv;         // [D][hv_stride] query hypervectors
  uint32_t* partial;        // [G][S][2][L][N] evaluation-domain partial sums
  const uint32_t* scatter;  // [N] slot source of every evaluation-side position
  const uint32_t* fwd_tw;   // [L+alpha][N] forward twiddles, Montgomery form
  const uint32_t* inv_t;    // [N] inverse twiddles mod t, Montgomery form
  const PrimeConst* pcs;    // [L+alpha]
  PrimeConst pct;           // constants of t
  uint32_t L, M, D, r, hv_stride, B, G, S, mchunk, NLG;
  // work covers model ciphertexts [m_base, m_base + m_len); splits cut that range
  uint32_t m_base, m_len;
  // split path: lifted plaintext coefficients [G][m_len][N] (int32 in (-t/2, t/2]) written
  // by the batch-encode kernel and read by the MAC kernel; with accumulate set, the MAC
  // kernel adds to the partial sums already stored instead of overwriting them
  int32_t* pt;
  uint32_t accumulate;
  // XCD-aware order of the MAC / fused work items (see XcdMap); xcd = 0: block = item
  uint32_t xcd, nitems;
  ScaleOp scale;
  // subring layout (sub_logn > 0): query plaintexts p(X) = p~(X^K'), K' = 2^sub_logk, of
  // n = 2^sub_logn coefficients; pt then holds their n-point transforms [G][m_len][L][n];
  // pct_sub holds the n-point constants of t
  uint32_t sub_logn, sub_logk;
  PrimeConst pct_sub;
  const SubGroup* vg;  // subring kernels: per group its queries (nullptr: hv + g * B, hv_stride)
  uint32_t q_last;     // queries in the last group (the others hold B; subring kernels: without vg)
};

// Workgroups are dispatched to the 8 XCDs of the chip round robin (workgroup d runs on XCD
// d % 8), and each XCD has its own L2.  Work items that read the same data (the limb items
// of one plaintext, the group items of one model range) are consecutive in item order, so
// with `on` set, XCD x takes the contiguous item range [x n / 8, (x + 1) n / 8): dispatch
// slot d holds item floor((d % 8) n / 8) + d / 8, and slots past the end of their range
// hold none.  The workgroups running at once on one XCD then work on neighbouring items
// and share their inputs in that XCD's L2, and every XCD gets n / 8 items (+-1).
struct XcdMap {
  uint32_t on, n;
  __host__ __device__ uint32_t item(uint32_t d) const {
    if (!on) return d < n ? d : 0xFFFFFFFFu;
    const uint64_t x = d & 7u, y = d >> 3;
    const uint64_t start = x * n / 8u, end = (x + 1u) * n / 8u;
    return start + y < end ? (uint32_t)(start + y) : 0xFFFFFFFFu;
  }
  // dispatch slots that cover every item
  __host__ __device__ uint32_t slots() const { return on ? 8u * ((n + 7u) / 8u) : n; }
};

// ---- request lists (many requests scored by one launch of each kernel)
// One request of a list.  `out` receives [G][2][L][N]: coefficient-domain score
// ciphertexts when r == 1, evaluation-domain sums (the input of rotate-and-sum) otherwise.
struct ReqDesc {
  const uint32_t* model;    // [M][2][L][N] evaluation domain, Montgomery form
  const int8_t* hv;         // [D][hv_stride]
  const uint32_t* scatter;  // [N] slot source table of the request's (K, r)
  uint32_t* out;
  uint32_t D, r, B, hv_stride;
  uint32_t Q;  // queries (the batch encoding reads later positions of the last group as zero)
  ScaleOp scale;
};

// A segment: model ciphertexts [m0, m1) of group g of request `req`; its plaintexts sit at
// plaintext index `pt` of the chunk buffer and its partial sums in slot `slot`.
struct Segment {
  uint32_t req, g, m0, m1, pt, slot;
};

// Output item: group g of request `req`, the sum of slots [slot0, slot0 + nslot).
struct FinishItem {
  uint32_t req, g, slot0, nslot;
};

struct TSideArgs {
  const uint32_t* inv_t;
  PrimeConst pct;
};

struct ListArgs {
  const ReqDesc* reqs;
  const Segment* segs;      // the segments of this launch
  uint32_t nseg, NLG, L;
  XcdMap xm;                // order of the MAC / fused items (nseg * NLG of them)
  const FinishItem* fin;
  uint32_t nfin;
  int32_t* pt;              // split path: lifted plaintexts of the launch's segments
  uint32_t* partial;        // [slots][2][L][N]
  const uint32_t* fwd_tw;
  const uint32_t* inv_tw;
  const PrimeConst* pcs;
  TSideArgs ts;
  uint32_t scaled;          // some request of the list carries the scaling op
};

// HDC encoding of many requests in one launch: per request its operands and layout, per
// 128 x 128 output tile its request and origin.
struct HdcReq {
  const uint8_t* x;
  const int8_t* base;
  int8_t* hv;  // first column of the request (rows of pitch `stride`)
  uint32_t Q, F, D, stride, ncols, qbits, qshift, pad;
};
struct HdcTile {
  uint32_t req, j0, q0, pad;
};

// One device-to-device copy of `words` 32-bit words (a multiple of 4, 16-byte aligned ends).
struct CopyRange {
  const uint32_t* src;
  uint32_t* dst;
  size_t words;
};

// Constants of hybrid key switching (Shoup pairs (w, floor(w*2^32/m)) for the modulus
// each multiplication is taken in).
struct KsConst {
  const uint2* up_inv;    // [L]: (Q_j/q_i)^-1 mod q_i, i in digit j
  const uint2* up_mul;    // [dnum][ds][nmod]: (Q_j/q_i) mod m
  const uint2* down_inv;  // [alpha]: (P/p_k)^-1 mod p_k
  const uint2* down_mul;  // [alpha][L]: (P/p_k) mod q_i
  const uint2* pinv;      // [L]: P^-1 mod q_i
  uint32_t L, alpha, dnum, ds, nmod, G;
};

// Buffers of the rotate-and-sum steps (all evaluation domain unless noted).
struct RotateArgs {
  KsConst k;
  const uint32_t* perm;    // [log2 r][N] automorphism permutations of evaluation points
  const uint32_t* ksk;     // [log2 r][dnum][2][nmod][N] switching keys, Montgomery form
  uint32_t* acc;           // [G][2][L][N] accumulators, updated in place
  uint32_t* R;             // [G][2][L][N] rotated accumulators
  uint32_t* D;             // [G][L][N] coefficient domain
  uint32_t* Y;             // [G][dnum][nmod][N]
  uint32_t* KS;            // [G][2][nmod][N]
  uint32_t* XP;            // [G][2][alpha][N] coefficient domain
  const uint32_t* fwd_tw;
  const uint32_t* inv_tw;
  const PrimeConst* pcs;
};

}  // namespace ephdc_dev

namespace ephdc {

using ephdc_dev::CopyRange;
using ephdc_dev::FinishItem;
using ephdc_dev::HdcReq;
using ephdc_dev::HdcTile;
using ephdc_dev::KsConst;
using ephdc_dev::ListArgs;
using ephdc_dev::ReqDesc;
using ephdc_dev::SubGroup;
using ephdc_dev::Segment;
using ephdc_dev::XcdMap;
using ephdc_dev::RotateArgs;

using ephdc_dev::PrimeConst;
using ephdc_dev::ScoreArgs;
using ephdc_dev::ScaleOp;

// Addressing of batched transforms: polynomial p is read from in + (p / in_per) * in_stride +
// (p % in_per) * N (likewise written); in_per / out_per = 0 means densely packed.
struct BatchMap {
  uint32_t in_per = 0, out_per = 0;
  size_t in_stride = 0, out_stride = 0;
};

// XCD-aware item order for n items (identity below 64 items).
XcdMap make_xcd_map(uint32_t n);

hipError_t prepare_kernels();
bool supported_logn(int logn);

hipError_t launch_fwd_batch(int logn, const uint32_t* in, uint32_t* out, size_t npolys, const uint32_t* tw,
                            const PrimeConst* pcs, uint32_t nlimb, uint32_t limb_base, bool mont,
                            hipStream_t st, const BatchMap& map = BatchMap{});
hipError_t launch_inv_batch(int logn, const uint32_t* in, uint32_t* out, size_t npolys, const uint32_t* itw,
                            const PrimeConst* pcs, uint32_t nlimb, uint32_t limb_base, hipStream_t st,
                            const BatchMap& map = BatchMap{});
hipError_t launch_pointwise_mont(const uint32_t* a, const uint32_t* b, uint32_t* out, size_t n, uint32_t N,
                                 const PrimeConst* pcs, uint32_t nlimb, hipStream_t st);
hipError_t launch_score(int logn, int le, int lg, const ScoreArgs& a, uint32_t nblocks, hipStream_t st);
// split path: batch-encode every (g, m) plaintext of the launch into a.pt, then MAC
hipError_t launch_encode_pt(int logn, int le, const ScoreArgs& a, uint32_t nblocks, hipStream_t st);
hipError_t launch_mac(int logn, int le, int lg, const ScoreArgs& a, uint32_t nblocks, hipStream_t st);
// subring layout: batch encoding with the n-point transforms of every limb (G groups x
// `splits` ranges of a.mchunk plaintexts), and the streaming MAC (position blocks x L x
// group tiles x S items)
bool subring_kernels(int logn, int sub_logn);
hipError_t launch_encode_sub(int sub_logn, const ScoreArgs& a, uint32_t splits, hipStream_t st);
hipError_t launch_mac_sub(int logn, int sub_logn, const ScoreArgs& a, uint32_t nblocks, hipStream_t st);
uint32_t mac_sub_resident_blocks(uint32_t G);  // streaming-MAC workgroups resident at once for G groups
uint32_t mac_sub_items(uint32_t N, uint32_t L, uint32_t G);  // streaming-MAC work items per split of G groups
bool supported_shape(int logn, int le);
hipError_t launch_finish(int logn, bool invert, const uint32_t* partial, uint32_t* out, uint32_t G, uint32_t S,
                         uint32_t L, const uint32_t* itw, const PrimeConst* pcs, hipStream_t st);
hipError_t launch_debug_plaintext(int logn, const ScoreArgs& a, uint32_t g, uint32_t m, uint32_t* out,
                                  hipStream_t st);

// Request lists: persistent launches over `grid` workgroups.
hipError_t launch_score_list(int logn, int le, int lg, const ListArgs& a, uint32_t grid, hipStream_t st);
hipError_t launch_encode_list(int logn, int le, const ListArgs& a, uint32_t grid, hipStream_t st);
hipError_t launch_mac_list(int logn, int le, int lg, const ListArgs& a, uint32_t grid, hipStream_t st);
hipError_t launch_finish_list(int logn, const ListArgs& a, hipStream_t st);

// One rotate-and-sum step (Galois element of step `step`): acc <- acc + KeySwitch(sigma(acc)).
hipError_t launch_rotate_step(int logn, const RotateArgs& r, uint32_t step, hipStream_t st);

// HDC encoding of many requests (one workgroup per tile) and copies of many ranges.
hipError_t launch_hdc_encode_list(const HdcReq* reqs, const HdcTile* tiles, uint32_t ntiles, hipStream_t st);
hipError_t launch_copy_list(const CopyRange* ranges, uint32_t n, size_t total_words, hipStream_t st);

// HDC projection: hv[j][q] = quantise(sum_f (x[q][f]-128) * base[f][j]) for q < Q, 0 for
// Q <= q < ncols (rows of pitch `stride`; ncols = 0 means the whole row).  Columns past
// ncols are not touched, so requests can be encoded side by side into one buffer.
hipError_t launch_hdc_encode(const uint8_t* x, const int8_t* base, int8_t* hv, uint32_t Q, uint32_t F,
                             uint32_t D, uint32_t stride, uint32_t qbits, uint32_t qshift, hipStream_t st,
                             uint32_t ncols = 0);

}  // namespace ephdc
