// HIP kernels of the scoring path: batched transforms, the fused batch-encode + ct x pt
// multiply-accumulate kernel, the partial-sum reduction and the debug entry kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "device_ntt.hpp"
#include "kernel_common.hpp"
#include "launch.hpp"

namespace ephdc_dev {

// ------------------------------------------------------------------ batched transforms
// One workgroup per polynomial; polynomial `poly` is taken mod modulus limb_base + poly % nlimb
// and sits at in + (poly / per) * stride + (poly % per) * N (likewise for the output), so
// that sub-arrays of interleaved buffers can be transformed in place or gathered.
struct PolyMap {
  uint32_t in_per, out_per;
  size_t in_stride, out_stride;
  __device__ __forceinline__ size_t in_off(size_t poly, int N) const {
    return (poly / in_per) * in_stride + (poly % in_per) * (size_t)N;
  }
  __device__ __forceinline__ size_t out_off(size_t poly, int N) const {
    return (poly / out_per) * out_stride + (poly % out_per) * (size_t)N;
  }
};

template <int LOGN, int LE>
__global__ __launch_bounds__((1 << LOGN) >> LE) void k_fwd_batch(const uint32_t* __restrict__ in,
                                                                  uint32_t* __restrict__ out,
                                                                  const uint32_t* __restrict__ fwd_tw,
                                                                  const PrimeConst* __restrict__ pcs,
                                                                  uint32_t nlimb, uint32_t limb_base, int mont,
                                                                  PolyMap pm) {
  using S = Shape<LOGN, LE>;
  LdsBufs b{0, 0, one_buffer<LOGN, LE>()};
  const int tid = threadIdx.x;
  const size_t poly = blockIdx.x;
  const uint32_t limb = limb_base + (uint32_t)(poly % nlimb);
  const PrimeConst pc = pcs[limb];
  const uint32_t* src = in + pm.in_off(poly, S::N);
  uint32_t v[S::E];
#pragma unroll
  for (int i = 0; i < S::E; ++i) v[i] = src[tid + i * S::T];
  ntt_forward<LOGN, LE>(v, tid, fwd_tw + (size_t)limb * S::N, pc, b);
  uint32_t* dst = out + pm.out_off(poly, S::N) + (size_t)tid * S::E;
#pragma unroll
  for (int i = 0; i < S::E; ++i) {
    uint32_t x = reduce4(v[i], pc.m);
    if (mont) x = csub(mont_mul(x, pc.r2, pc.m, pc.mneg_inv), pc.m);
    dst[i] = x;
  }
}

template <int LOGN, int LE>
__global__ __launch_bounds__((1 << LOGN) >> LE) void k_inv_batch(const uint32_t* __restrict__ in,
                                                                  uint32_t* __restrict__ out,
                                                                  const uint32_t* __restrict__ inv_tw,
                                                                  const PrimeConst* __restrict__ pcs,
                                                                  uint32_t nlimb, uint32_t limb_base, PolyMap pm) {
  using S = Shape<LOGN, LE>;
  LdsBufs b{0, 0, one_buffer<LOGN, LE>()};
  const int tid = threadIdx.x;
  const size_t poly = blockIdx.x;
  const uint32_t limb = limb_base + (uint32_t)(poly % nlimb);
  const PrimeConst pc = pcs[limb];
  const uint32_t* src = in + pm.in_off(poly, S::N) + (size_t)tid * S::E;
  uint32_t v[S::E];
#pragma unroll
  for (int i = 0; i < S::E; ++i) v[i] = src[i];
  ntt_inverse<LOGN, LE, true>(v, tid, inv_tw + (size_t)limb * S::N, pc, b);
  uint32_t* dst = out + pm.out_off(poly, S::N);
#pragma unroll
  for (int i = 0; i < S::E; ++i) dst[tid + i * S::T] = csub(v[i], pc.m);
}

// out = a * b (Montgomery: a in Montgomery form, b plain) mod the polynomial's modulus.
__global__ void k_pointwise_mont(const uint32_t* __restrict__ a, const uint32_t* __restrict__ b,
                                 uint32_t* __restrict__ out, size_t n, uint32_t N,
                                 const PrimeConst* __restrict__ pcs, uint32_t nlimb) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const PrimeConst& pc = pcs[(i / N) % nlimb];
    out[i] = csub(mont_mul(a[i], b[i], pc.m, pc.mneg_inv), pc.m);
  }
}

// The scatter table entry of register i of thread tid (position tid*E + i).  When the LDS
// plan has room, the table is staged once per workgroup after the exchange buffers,
// transposed to [i][tid] so that every read instruction touches consecutive words.
template <int LOGN, int LE>
__device__ __forceinline__ void stage_table(const uint32_t* __restrict__ scatter, int tid) {
  using S = Shape<LOGN, LE>;
  if constexpr (LdsPlan<LOGN, LE>::table_in_lds) {
    uint32_t* tbl = ephdc_lds + LdsPlan<LOGN, LE>::exchange_words;
#pragma unroll
    for (int i = 0; i < S::E; ++i) tbl[i * S::T + tid] = scatter[tid * S::E + i];
    lds_barrier();
  }
}

template <int LOGN, int LE>
__device__ __forceinline__ uint32_t table_entry(const uint32_t* __restrict__ scatter, int tid, int i) {
  using S = Shape<LOGN, LE>;
  if constexpr (LdsPlan<LOGN, LE>::table_in_lds) {
    return ephdc_lds[LdsPlan<LOGN, LE>::exchange_words + i * S::T + tid];
  } else {
    return scatter[tid * S::E + i];
  }
}

// ------------------------------------------------------------------ batch encoding
// Where the slot values of one query group come from: hypervector column block hvg (the
// group's first query), dimensions m*r + u < D, row pitch hv_stride.
struct QuerySrc {
  const int8_t* hvg;
  uint32_t D, r, hv_stride;
  uint32_t nq;  // queries of the group: later query positions read as zero
};

// Constants of the plaintext side (mod t).
using TSide = TSideArgs;

// Per position, from its scatter-table entry: the dimension offset u of the slot feeding it
// (all ones for an unused slot or a query position past the group's queries, which then
// reads as zero) and the byte offset of that slot's hv entry inside the group's block at
// m = 0.
template <int LOGN, int LE>
__device__ __forceinline__ void scatter_offsets(uint32_t (&du)[1 << LE], uint32_t (&off)[1 << LE],
                                                const uint32_t (&ent)[1 << LE], const QuerySrc& q) {
#pragma unroll
  for (int i = 0; i < (1 << LE); ++i) {
    const uint32_t e = ent[i];
    const bool none = e == 0xFFFFFFFFu || (e & 0xFFFFu) >= q.nq;
    du[i] = none ? 0xFFFFFFFFu : e >> 16;
    off[i] = none ? 0u : (e >> 16) * q.hv_stride + (e & 0xFFFFu);
  }
}

// Slot values of query plaintext (g, m) at this thread's evaluation-side positions
// tid*E + i (hv entry of dimension m*r + u, or 0 where that dimension or the slot does not
// exist; one uniform base and bound, no branch per value), then the inverse transform mod
// t, lazy (t < 2^17) and scaled by N^-1 in its last stage: mu in [0, t), coefficient
// layout tid + i*T.  TL: the inverse twiddles mod t are in the LDS table slot.
template <int LOGN, int LE, bool TL = false>
__device__ __forceinline__ void encode_query(uint32_t (&v)[1 << LE], const QuerySrc& q,
                                             const uint32_t (&du)[1 << LE], const uint32_t (&off)[1 << LE],
                                             const TSide& ts, uint32_t m, int tid, LdsBufs& b) {
  using S = Shape<LOGN, LE>;
  const uint32_t t = ts.pct.m;
  const uint32_t base = m * q.r * q.hv_stride, lim = q.D - m * q.r;  // m * r < D
#pragma unroll
  for (int i = 0; i < S::E; ++i) {
    const bool ok = du[i] < lim;
    const int h = ld_at(q.hvg, ok ? base + off[i] : 0u);
    const uint32_t val = (uint32_t)h + (t & (uint32_t)(h >> 31));  // h mod t
    v[i] = ok ? val : 0u;
  }
  ntt_inverse<LOGN, LE, true, true, TL>(v, tid, ts.inv_t, ts.pct, b);
#pragma unroll
  for (int i = 0; i < S::E; ++i) v[i] = csub(v[i], t);
}

// This thread's scatter-table entries (from the staged LDS copy when there is one).
template <int LOGN, int LE>
__device__ __forceinline__ void table_entries(uint32_t (&ent)[1 << LE], const uint32_t* __restrict__ scatter,
                                              int tid) {
#pragma unroll
  for (int i = 0; i < (1 << LE); ++i) ent[i] = table_entry<LOGN, LE>(scatter, tid, i);
}

// Centred lift of mu in [0, t) into Z_m: mu if mu <= t/2, else m - (t - mu).
__device__ __forceinline__ uint32_t lift(uint32_t mu, uint32_t t, uint32_t m) {
  return mu > (t >> 1) ? m - (t - mu) : mu;
}

// ------------------------------------------------------------------ scoring work items
// One MAC work item: model ciphertexts [m0, m1) of one query group, limbs [l0, l0 + LG),
// accumulated into the item's slot [2][L][N] (evaluation domain).
struct MacItem {
  const uint32_t* model;  // [M][2][L][N] evaluation domain, Montgomery form
  uint32_t* slot;         // partial sums of this item
  uint32_t L, m0, m1, l0;
  ScaleOp scale;          // HE-aware scaling (pow == nullptr: none)
};

// Weight of plaintext m in limb l under the scaling op: the transformed plaintext (values
// in [0, 4q)) is multiplied by c^e(m), back in [0, 2q).  The weights distribute the
// accumulator's scalings over its terms, which gives the same residues in any order of
// the additions and across work items.
template <int E>
__device__ __forceinline__ void apply_scale(uint32_t (&p)[E], const ScaleOp& so, uint32_t m, uint32_t l,
                                            const PrimeConst& pc) {
  if (so.pow == nullptr) return;
  const uint32_t e = so.exponent(m);
  if (e == 0) return;
  const uint32_t w = so.pow[l * (so.nb + 1) + e];
#pragma unroll
  for (int i = 0; i < E; ++i) p[i] = mont_mul(p[i], w, pc.m, pc.mneg_inv);
}

template <int LG, int E>
__device__ __forceinline__ void zero_acc(uint32_t (&acc)[2][LG][E]) {
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int li = 0; li < LG; ++li)
#pragma unroll
      for (int i = 0; i < E; ++i) acc[c][li][i] = 0;
}

template <int LOGN, int LE, int LG>
__device__ __forceinline__ void store_acc(const uint32_t (&acc)[2][LG][1 << LE], const MacItem& it,
                                          const PrimeConst* __restrict__ pcs, int tid) {
  using S = Shape<LOGN, LE>;
#pragma unroll
  for (int li = 0; li < LG; ++li) {
    const uint32_t l = it.l0 + li;
    const uint32_t mm = pcs[l].m;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      uint32_t* dst = it.slot + ((size_t)c * it.L + l) * S::N + (size_t)tid * S::E;
#pragma unroll
      for (int i = 0; i < S::E; ++i) dst[i] = csub(acc[c][li][i], mm);
    }
  }
}

// Fused item: for m in [m0, m1), batch-encode query plaintext (g, m), lift it into each
// limb of the group, transform it, and accumulate ct_m[c][l] * pt[l] for c in {0, 1}.
// Accumulators live in VGPRs for the whole range; the model values of a limb are requested
// before its transform so that their latency overlaps the transform.
template <int LOGN, int LE, int LG>
__device__ __forceinline__ void score_item(const MacItem& it, const QuerySrc& q, const uint32_t* __restrict__ scatter,
                                           const TSide& ts, const uint32_t* __restrict__ fwd_tw,
                                           const PrimeConst* __restrict__ pcs, int tid, LdsBufs& b) {
  using S = Shape<LOGN, LE>;
  constexpr int E = S::E, N = S::N;
  uint32_t acc[2][LG][E];
  zero_acc(acc);
  const uint32_t t = ts.pct.m;
  for (uint32_t m = it.m0; m < it.m1; ++m) {
    uint32_t mu[E], ent[E], du[E], off[E];
    table_entries<LOGN, LE>(ent, scatter, tid);
    scatter_offsets<LOGN, LE>(du, off, ent, q);
    encode_query<LOGN, LE>(mu, q, du, off, ts, m, tid, b);
#pragma unroll
    for (int li = 0; li < LG; ++li) {
      const uint32_t l = it.l0 + li;
      const PrimeConst pc = pcs[l];
      const uint32_t* ct0 = it.model + (((size_t)m * 2 + 0) * it.L + l) * N + (size_t)tid * E;
      const uint32_t* ct1 = it.model + (((size_t)m * 2 + 1) * it.L + l) * N + (size_t)tid * E;
      uint32_t c0[E], c1[E];
#pragma unroll
      for (int i = 0; i < E; ++i) {
        c0[i] = ct0[i];
        c1[i] = ct1[i];
      }
      uint32_t p[E];
#pragma unroll
      for (int i = 0; i < E; ++i) p[i] = lift(mu[i], t, pc.m);
      ntt_forward<LOGN, LE>(p, tid, fwd_tw + (size_t)l * N, pc, b);
      apply_scale(p, it.scale, m, l, pc);
      const uint32_t m2 = 2 * pc.m;
#pragma unroll
      for (int i = 0; i < E; ++i) {
        acc[0][li][i] = csub(acc[0][li][i] + mont_mul(c0[i], p[i], pc.m, pc.mneg_inv), m2);
        acc[1][li][i] = csub(acc[1][li][i] + mont_mul(c1[i], p[i], pc.m, pc.mneg_inv), m2);
      }
    }
  }
  store_acc<LOGN, LE, LG>(acc, it, pcs, tid);
}

// Batch encoding alone: query plaintexts (g, m) for m in [m0, m1), stored as centred lifts
// (int32 in (-t/2, t/2]), coefficient order, at dst + (m - m0) * N.  The table and output
// pointers are deliberately not __restrict__: that would let the compiler keep a global
// scatter table in registers across the loop and spill at 1024 threads.
// TL: the LDS table slot holds the inverse twiddles mod t (staged by the caller) instead
// of the scatter table, whose entries are then read from global memory.
template <int LOGN, int LE, bool TL = false>
__device__ __forceinline__ void encode_item(const QuerySrc& q, const uint32_t* scatter, const TSide& ts,
                                            uint32_t m0, uint32_t m1, int32_t* dst, int tid,
                                            LdsBufs& b) {
  using S = Shape<LOGN, LE>;
  const uint32_t t = ts.pct.m;
  // the item's scatter offsets, in registers for all of its plaintexts
  uint32_t ent[S::E], du[S::E], off[S::E];
  if constexpr (TL) {
#pragma unroll
    for (int i = 0; i < S::E; ++i) ent[i] = ld_at(scatter, (uint32_t)(tid * S::E + i) * 4u);
  } else {
    table_entries<LOGN, LE>(ent, scatter, tid);
  }
  scatter_offsets<LOGN, LE>(du, off, ent, q);
  for (uint32_t m = m0; m < m1; ++m) {
    uint32_t mu[S::E];
    encode_query<LOGN, LE, TL>(mu, q, du, off, ts, m, tid, b);
    int32_t* d = dst + (size_t)(m - m0) * S::N;
#pragma unroll
    for (int i = 0; i < S::E; ++i) d[tid + i * S::T] = mu[i] > (t >> 1) ? (int32_t)mu[i] - (int32_t)t : (int32_t)mu[i];
  }
}

// MAC alone: for m in [m0, m1), read the lifted plaintext (pt + (m - m0) * N), reduce it
// into each limb of the group, transform it and accumulate ct_m[c][l] * pt[l]; with
// accumulate set the item adds to the sums already in its slot.  With PF, the next
// plaintext and each limb's model values are requested ahead of the transform that
// precedes their use (more registers: used where the register budget allows it); the
// 32-bit form can request the next plaintext alone (PTPF).
template <int LOGN, int LE, int LG, bool PF, bool TL = false, bool PTPF = true, bool SC = false>
__device__ __forceinline__ void mac_item32(const MacItem& it, const int32_t* __restrict__ pt, bool accumulate,
                                         const uint32_t* __restrict__ fwd_tw, const PrimeConst* __restrict__ pcs,
                                         int tid, LdsBufs& b) {
  using S = Shape<LOGN, LE>;
  constexpr int E = S::E, N = S::N;
  // per-lane byte offsets inside one polynomial: evaluation layout (tid*E + i) for the model
  // and the sums, coefficient layout (tid + i*T) for the plaintexts
  const uint32_t eo = (uint32_t)tid * E * 4u, co = (uint32_t)tid * 4u;
  uint32_t acc[2][LG][E];
#pragma unroll
  for (int li = 0; li < LG; ++li)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const uint32_t* src = it.slot + ((size_t)c * it.L + it.l0 + li) * N;
#pragma unroll
      for (int i = 0; i < E; ++i) acc[c][li][i] = accumulate ? ld_at(src, eo + 4u * i) : 0u;
    }

  // PTPF: the next plaintext is requested a whole iteration ahead (it fits the registers of
  // every shape of the single-request kernel); the model values only with PF
  int32_t nxt[E];
  if (PTPF && it.m0 < it.m1) {
#pragma unroll
    for (int i = 0; i < E; ++i) nxt[i] = ld_at(pt, co + 4u * (uint32_t)(i * S::T));
  }
  for (uint32_t m = it.m0; m < it.m1; ++m) {
    const int32_t* ptm = pt + (size_t)(m - it.m0) * N;  // plaintext (g, m)
    int32_t cur[E];
    if constexpr (PTPF) {
#pragma unroll
      for (int i = 0; i < E; ++i) cur[i] = nxt[i];
      if (m + 1 < it.m1) {
#pragma unroll
        for (int i = 0; i < E; ++i) nxt[i] = ld_at(ptm + N, co + 4u * (uint32_t)(i * S::T));
      }
    } else {
#pragma unroll
      for (int i = 0; i < E; ++i) cur[i] = ld_at(ptm, co + 4u * (uint32_t)(i * S::T));
    }
#pragma unroll
    for (int li = 0; li < LG; ++li) {
      const uint32_t l = it.l0 + li;
      const PrimeConst pc = pcs[l];
      const uint32_t* ct0 = it.model + (((size_t)m * 2 + 0) * it.L + l) * N;
      const uint32_t* ct1 = it.model + (((size_t)m * 2 + 1) * it.L + l) * N;
      uint32_t c0[E], c1[E];
      if constexpr (PF) {
#pragma unroll
        for (int i = 0; i < E; ++i) {
          c0[i] = ld_at(ct0, eo + 4u * i);
          c1[i] = ld_at(ct1, eo + 4u * i);
        }
      }
      uint32_t p[E];
#pragma unroll
      for (int i = 0; i < E; ++i) p[i] = pc.m + (uint32_t)cur[i];  // |cur| <= t/2: in [0, 2m), = cur mod m
      ntt_forward<LOGN, LE, TL, true>(p, tid, fwd_tw + (size_t)l * N, pc, b);
      if constexpr (SC) apply_scale(p, it.scale, m, l, pc);
      if constexpr (!PF) {
#pragma unroll
        for (int i = 0; i < E; ++i) {
          c0[i] = ld_at(ct0, eo + 4u * i);
          c1[i] = ld_at(ct1, eo + 4u * i);
        }
      }
      const uint32_t m2 = 2 * pc.m;
#pragma unroll
      for (int i = 0; i < E; ++i) {
        acc[0][li][i] = csub(acc[0][li][i] + mont_mul(c0[i], p[i], pc.m, pc.mneg_inv), m2);
        acc[1][li][i] = csub(acc[1][li][i] + mont_mul(c1[i], p[i], pc.m, pc.mneg_inv), m2);
      }
    }
  }
  store_acc<LOGN, LE, LG>(acc, it, pcs, tid);
}

template <int LOGN, int LE, int LG, bool PF, bool TL = false, bool SC = false>
__device__ __forceinline__ void mac_item64(const MacItem& it, const int32_t* __restrict__ pt, bool accumulate,
                                         const uint32_t* __restrict__ fwd_tw, const PrimeConst* __restrict__ pcs,
                                         int tid, LdsBufs& b) {
  using S = Shape<LOGN, LE>;
  constexpr int E = S::E, N = S::N;
  // per-lane byte offsets inside one polynomial: evaluation layout (tid*E + i) for the model
  // and the sums, coefficient layout (tid + i*T) for the plaintexts
  const uint32_t eo = (uint32_t)tid * E * 4u, co = (uint32_t)tid * 4u;
  // Sums of (model in Montgomery form) x (plaintext, lazy in [0, 4m)) in 64 bits, folded
  // every second plaintext and reduced once at the end (fold64 / redc64); a stored partial
  // sum s re-enters as its Montgomery form s*2^32 mod m.
  uint64_t acc[2][LG][E];
#pragma unroll
  for (int li = 0; li < LG; ++li) {
    const PrimeConst pc = pcs[it.l0 + li];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const uint32_t* src = it.slot + ((size_t)c * it.L + it.l0 + li) * N;
#pragma unroll
      for (int i = 0; i < E; ++i)
        acc[c][li][i] = accumulate ? mont_mul(ld_at(src, eo + 4u * i), pc.r2, pc.m, pc.mneg_inv) : 0u;
    }
  }

  int32_t nxt[E];
  if (PF && it.m0 < it.m1) {
#pragma unroll
    for (int i = 0; i < E; ++i) nxt[i] = ld_at(pt, co + 4u * (uint32_t)(i * S::T));
  }
  for (uint32_t m = it.m0; m < it.m1; ++m) {
    const int32_t* ptm = pt + (size_t)(m - it.m0) * N;  // plaintext (g, m)
    int32_t cur[E];
    if constexpr (PF) {
#pragma unroll
      for (int i = 0; i < E; ++i) cur[i] = nxt[i];
      if (m + 1 < it.m1) {
#pragma unroll
        for (int i = 0; i < E; ++i) nxt[i] = ld_at(ptm + N, co + 4u * (uint32_t)(i * S::T));
      }
    } else {
#pragma unroll
      for (int i = 0; i < E; ++i) cur[i] = ld_at(ptm, co + 4u * (uint32_t)(i * S::T));
    }
    const bool fold = ((m - it.m0) & 1u) != 0u;
#pragma unroll
    for (int li = 0; li < LG; ++li) {
      const uint32_t l = it.l0 + li;
      const PrimeConst pc = pcs[l];
      const uint32_t* ct0 = it.model + (((size_t)m * 2 + 0) * it.L + l) * N;
      const uint32_t* ct1 = it.model + (((size_t)m * 2 + 1) * it.L + l) * N;
      uint32_t c0[E], c1[E];
      if constexpr (PF) {
#pragma unroll
        for (int i = 0; i < E; ++i) {
          c0[i] = ld_at(ct0, eo + 4u * i);
          c1[i] = ld_at(ct1, eo + 4u * i);
        }
      }
      uint32_t p[E];
#pragma unroll
      for (int i = 0; i < E; ++i) p[i] = pc.m + (uint32_t)cur[i];  // |cur| <= t/2: in [0, 2m), = cur mod m
      ntt_forward<LOGN, LE, TL, true>(p, tid, fwd_tw + (size_t)l * N, pc, b);
      if constexpr (SC) apply_scale(p, it.scale, m, l, pc);
      if constexpr (!PF) {
#pragma unroll
        for (int i = 0; i < E; ++i) {
          c0[i] = ld_at(ct0, eo + 4u * i);
          c1[i] = ld_at(ct1, eo + 4u * i);
        }
      }
#pragma unroll
      for (int i = 0; i < E; ++i) {
        acc[0][li][i] += (uint64_t)c0[i] * p[i];
        acc[1][li][i] += (uint64_t)c1[i] * p[i];
      }
      if (fold) {
#pragma unroll
        for (int i = 0; i < E; ++i) {
          acc[0][li][i] = fold64(acc[0][li][i], pc.r1);
          acc[1][li][i] = fold64(acc[1][li][i], pc.r1);
        }
      }
    }
  }
#pragma unroll
  for (int li = 0; li < LG; ++li) {
    const uint32_t l = it.l0 + li;
    const PrimeConst pc = pcs[l];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      uint32_t* dst = it.slot + ((size_t)c * it.L + l) * N;
#pragma unroll
      for (int i = 0; i < E; ++i) st_at(dst, eo + 4u * i, redc64(fold64(acc[c][li][i], pc.r1), pc.m, pc.mneg_inv));
    }
  }
}

// MAC alone: 64-bit lazy sums where 8 values per thread leave the registers for them,
// 32-bit sums of Montgomery products otherwise.
// SC: the work items may carry the scaling op (kernels without it keep their registers).
template <int LOGN, int LE, int LG, bool PF, bool TL = false, bool PTPF = true, bool SC = false>
__device__ __forceinline__ void mac_item(const MacItem& it, const int32_t* __restrict__ pt, bool accumulate,
                                         const uint32_t* __restrict__ fwd_tw, const PrimeConst* __restrict__ pcs,
                                         int tid, LdsBufs& b) {
  if constexpr (LE <= 3)
    mac_item64<LOGN, LE, LG, PF, TL, SC>(it, pt, accumulate, fwd_tw, pcs, tid, b);
  else
    mac_item32<LOGN, LE, LG, PF, TL, PTPF, SC>(it, pt, accumulate, fwd_tw, pcs, tid, b);
}

// ------------------------------------------------------------------ single-request kernels
// Work item w of a launch: limb group w % NLG, then group g, then split of the model range.
__device__ __forceinline__ TSide tside(const ScoreArgs& a) { return TSide{a.inv_t, a.pct}; }

__device__ __forceinline__ QuerySrc query_src(const ScoreArgs& a, uint32_t g) {
  return QuerySrc{a.hv + (size_t)g * a.B, a.D, a.r, a.hv_stride, g + 1 == a.G ? a.q_last : a.B};
}

template <int LOGN, int LG>
__device__ __forceinline__ MacItem single_item(const ScoreArgs& a, uint32_t w, uint32_t& g, uint32_t& split) {
  const uint32_t lgi = w % a.NLG, rest = w / a.NLG;
  g = rest % a.G;
  split = rest / a.G;
  MacItem it;
  it.model = a.model;
  it.slot = a.partial + ((size_t)g * a.S + split) * 2 * a.L * ((size_t)1 << LOGN);
  it.L = a.L;
  it.m0 = a.m_base + split * a.mchunk;
  it.m1 = min(a.m_base + a.m_len, it.m0 + a.mchunk);
  it.l0 = lgi * LG;
  it.scale = a.scale;
  return it;
}

template <int LOGN, int LE, int LG>
__global__ __launch_bounds__((1 << LOGN) >> LE) void k_score(ScoreArgs a) {
  const uint32_t w = XcdMap{a.xcd, a.nitems}.item(blockIdx.x);
  if (w == 0xFFFFFFFFu) return;  // a slot past the last item: the whole workgroup leaves
  LdsBufs b{0};
  const int tid = threadIdx.x;
  stage_table<LOGN, LE>(a.scatter, tid);
  uint32_t g, split;
  const MacItem it = single_item<LOGN, LG>(a, w, g, split);
  score_item<LOGN, LE, LG>(it, query_src(a, g), a.scatter, tside(a), a.fwd_tw, a.pcs, tid, b);
}

// Split path, batch encoding: work item (split, g) writes plaintexts (g, m) of the split's
// range to a.pt[g][m - m_base][:].
template <int LOGN, int LE>
__global__ __launch_bounds__((1 << LOGN) >> LE) void k_encode_pt(ScoreArgs a) {
  using S = Shape<LOGN, LE>;
  LdsBufs b{0};
  const int tid = threadIdx.x;
  const uint32_t g = blockIdx.x % a.G, split = blockIdx.x / a.G;
  const uint32_t m0 = a.m_base + split * a.mchunk;
  const uint32_t m1 = min(a.m_base + a.m_len, m0 + a.mchunk);
  int32_t* dst = a.pt + ((size_t)g * a.m_len + (m0 - a.m_base)) * S::N;
  if constexpr (LdsPlan<LOGN, LE>::table_in_lds) {
    stage_twiddles<LOGN, LE>(a.inv_t, tid);
    lds_barrier();
    encode_item<LOGN, LE, true>(query_src(a, g), a.scatter, tside(a), m0, m1, dst, tid, b);
  } else {
    encode_item<LOGN, LE>(query_src(a, g), a.scatter, tside(a), m0, m1, dst, tid, b);
  }
}

// Split path, MAC: work item (split, g, limb group) over the split's range of the chunk.
// A MAC item of one limb keeps that limb's forward twiddles in the LDS table slot (unused
// by the MAC kernels) for all of its plaintexts.
template <int LOGN, int LE, int LG>
constexpr bool mac_lds_twiddles() {
  return LG == 1 && LdsPlan<LOGN, LE>::table_in_lds;
}

template <int LOGN, int LE, int LG, bool PF, bool SC = false>
__global__ __launch_bounds__((1 << LOGN) >> LE) void k_mac(ScoreArgs a) {
  const uint32_t w = XcdMap{a.xcd, a.nitems}.item(blockIdx.x);
  if (w == 0xFFFFFFFFu) return;  // a slot past the last item: the whole workgroup leaves
  LdsBufs b{0};
  const int tid = threadIdx.x;
  uint32_t g, split;
  const MacItem it = single_item<LOGN, LG>(a, w, g, split);
  const int32_t* pt = a.pt + ((size_t)g * a.m_len + (it.m0 - a.m_base)) * ((size_t)1 << LOGN);
  if constexpr (mac_lds_twiddles<LOGN, LE, LG>()) {
    stage_twiddles<LOGN, LE>(a.fwd_tw + (size_t)it.l0 * ((size_t)1 << LOGN), tid);
    lds_barrier();
    mac_item<LOGN, LE, LG, PF, true, true, SC>(it, pt, a.accumulate != 0, a.fwd_tw, a.pcs, tid, b);
  } else {
    mac_item<LOGN, LE, LG, PF, false, true, SC>(it, pt, a.accumulate != 0, a.fwd_tw, a.pcs, tid, b);
  }
}

// Prefetching fits the register budget except for the 1024-thread shape of N = 16384.
template <int LOGN, int LE>
constexpr bool mac_prefetch() {
  return Shape<LOGN, LE>::T <= 512 || LE <= 3;
}

// ------------------------------------------------------------------ subring layout
// In the subring layout every query plaintext is p(X) = p~(X^K'), K' = N/n, so
//  * its batch encoding is the n-point inverse transform (root zeta^K') of its n orbit
//    values; block v of query ql of the group sits at n-point evaluation position
//    ql*r + v and holds dimension m*r + v (r = 1: a lane's inputs are E consecutive bytes
//    of the group's hypervector row);
//  * its transform mod q_l is the n-point forward transform of p~ (root psi^K'), and the
//    value at N-point evaluation position x is the n-point output at position x >> log2 K'.
// The n-point twiddle tables are the first n entries of the N-point ones (the bit reversal
// over log2 N bits of k < n is K' times the one over log2 n bits), and only the n^-1
// constants differ (pct_sub).  One wave runs one n-point transform (n = 64 E), all of its
// exchanges inside the wave's own LDS region.
//
// Two kernels: k_encode_sub turns each query plaintext into its L transformed n-point
// vectors (a.pt[m - m_base][l][blk][g][y mod ypi], weighted by the scaling op; in [0, q_l)
// for launches of more than four groups, else in [0, 2 q_l)), and
// k_mac_sub streams the model once: a work item owns a block of evaluation positions of one
// limb for up to four query groups.

// Streaming MAC work items: kSubThreads threads over 2 * kSubThreads evaluation positions,
// which read the n-point positions [blk * ypi, (blk + 1) * ypi) with ypi = 2 * kSubThreads / K'.
// The transformed plaintexts are stored [m - m_base][l][blk][g][ypi], so that the values an
// item reads for one ciphertext and its groups are contiguous.
constexpr int kSubThreads = 256;

// LDS offset of the wave-local exchange buffer inside an exchange plan (see exchange()).
template <int LOGN, int LE>
constexpr int local_exchange_offset() {
  return LdsPlan<LOGN, LE>::three ? 2 * Shape<LOGN, LE>::PADN : Shape<LOGN, LE>::PADN;
}

// Values per thread of the n-point batch-encoding transforms: one wave per transform up to
// n = 1024 (E = n/64), 16 values per thread above.
constexpr int sub_le(int ls) { return ls <= 10 ? ls - 6 : 4; }

// Threads of one batch-encoding workgroup: four one-wave transforms, or one transform of
// n/E threads (n = 2048, 4096) whose first exchanges cross waves.
template <int LOGn, int LEs>
constexpr int encode_sub_threads() {
  return Shape<LOGn, LEs>::T == 64 ? 256 : Shape<LOGn, LEs>::T;
}
template <int LOGn, int LEs>
constexpr size_t encode_sub_lds_bytes() {
  using S = Shape<LOGn, LEs>;
  return (S::T == 64 ? 4 * S::PADN : LdsPlan<LOGn, LEs>::exchange_words) * sizeof(uint32_t);
}

// Work item (split, group quad): transform j of the workgroup takes group TPW * quad + j
// and every plaintext of the split, so that the workgroup's stores of one plaintext fill
// the adjacent slots [blk][g .. g + TPW) of the MAC's layout at about the same time.
template <int LOGn, int LEs>
__global__ __launch_bounds__((encode_sub_threads<LOGn, LEs>())) void k_encode_sub(ScoreArgs a) {
  using S = Shape<LOGn, LEs>;
  constexpr int E = S::E, n = S::N;
  constexpr bool one_wave = S::T == 64;
  constexpr int TPW = encode_sub_threads<LOGn, LEs>() / S::T;  // transforms per workgroup
  const int lane = threadIdx.x % S::T, wave = threadIdx.x / S::T;
  LdsBufs b{0, one_wave ? wave * S::PADN - local_exchange_offset<LOGn, LEs>() : 0};
  const uint32_t nq = (a.G + TPW - 1) / TPW;
  const uint32_t g = blockIdx.x % nq * TPW + wave, split = blockIdx.x / nq;
  if (g >= a.G) return;  // a one-wave transform past the last group (no workgroup barrier follows)
  const uint32_t m0 = a.m_base + split * a.mchunk;
  const uint32_t m1 = min(a.m_base + a.m_len, m0 + a.mchunk);
  const uint32_t t = a.pct_sub.m, L = a.L;
  const uint32_t N = (uint32_t)n << a.sub_logk;
  // queries of the group (lane*E + i), rows of pitch `stride`
  const SubGroup sg = a.vg ? a.vg[g] : SubGroup{a.hv + (size_t)g * a.B, a.hv_stride, g + 1 == a.G ? a.q_last : a.B};
  const int8_t* hvg = sg.hv + (uint32_t)lane * E;
  // transformed plaintexts of the chunk: [m - m_base][l][blk][g][y mod ypi]; a lane's E
  // outputs lie in one block (E <= ypi for K' <= 32)
  uint32_t* dst = reinterpret_cast<uint32_t*>(a.pt) + (size_t)(m0 - a.m_base) * L * a.G * n;
  const uint32_t ypi = (2u * kSubThreads) >> a.sub_logk, y0 = (uint32_t)lane * E;
  const uint32_t lo = ((y0 / ypi) * a.G * ypi + g * ypi + y0 % ypi) * 4u;  // byte offset of the lane's outputs
  const bool full = a.G > 4;  // the MAC's eight-group tiles take fully reduced values
  const uint32_t r = a.r, lr = __builtin_ctz(r);
  for (uint32_t m = m0; m < m1; ++m) {
    uint32_t v[E];
    if (r == 1) {
      uint32_t w[E / 4];
      const int8_t* src = hvg + (size_t)m * sg.stride;
      if constexpr (E == 16) {
        const uint4 q = *reinterpret_cast<const uint4*>(src);
        w[0] = q.x; w[1] = q.y; w[2] = q.z; w[3] = q.w;
      } else if constexpr (E == 8) {
        const uint2 q = *reinterpret_cast<const uint2*>(src);
        w[0] = q.x; w[1] = q.y;
      } else {
        w[0] = *reinterpret_cast<const uint32_t*>(src);
      }
#pragma unroll
      for (int i = 0; i < E; ++i) {
        int h = (int)(w[i >> 2] << (24 - 8 * (i & 3))) >> 24;  // signed byte i
        if ((uint32_t)lane * E + i >= sg.nq) h = 0;              // no query at this position
        v[i] = (uint32_t)h + (t & (uint32_t)(h >> 31));           // h mod t
      }
    } else {
      // folded: position y holds query y >> log2 r at dimension m*r + (y mod r), zero past D
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const uint32_t y = (uint32_t)lane * E + i, j = m * r + (y & (r - 1));
        const int h = j < a.D && (y >> lr) < sg.nq ? (int)sg.hv[j * sg.stride + (y >> lr)] : 0;
        v[i] = (uint32_t)h + (t & (uint32_t)(h >> 31));
      }
    }
    ntt_inverse<LOGn, LEs, true, true>(v, lane, a.inv_t, a.pct_sub, b);
    int32_t c[E];  // centred lift, coefficient layout lane + i*T
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const uint32_t mu = csub(v[i], t);
      c[i] = mu > (t >> 1) ? (int32_t)mu - (int32_t)t : (int32_t)mu;
    }
    uint32_t* d = dst + (size_t)(m - m0) * L * a.G * n;
    for (uint32_t l = 0; l < L; ++l) {
      const PrimeConst pc = a.pcs[l];
#pragma unroll
      for (int i = 0; i < E; ++i) v[i] = pc.m + (uint32_t)c[i];  // |c| <= t/2: in [0, 2m), = c mod m
      ntt_forward<LOGn, LEs, false, true>(v, lane, a.fwd_tw + (size_t)l * N, pc, b);
      apply_scale(v, a.scale, m, l, pc);
#pragma unroll
      for (int i = 0; i < E; ++i) v[i] = csub(v[i], 2 * pc.m);
      if (full) {
#pragma unroll
        for (int i = 0; i < E; ++i) v[i] = csub(v[i], pc.m);
      }
      uint32_t* dl = d + (size_t)l * a.G * n;
#pragma unroll
      for (int i = 0; i < E; i += 4)
        st_at(reinterpret_cast<uint4*>(dl), lo + 4u * i, make_uint4(v[i], v[i + 1], v[i + 2], v[i + 3]));
    }
  }
}

typedef uint32_t v2u __attribute__((ext_vector_type(2)));

// Buffer resource for raw loads at a uniform address (no range limit): the base lives in
// scalar registers and every load adds a lane offset and a scalar offset, so no per-lane
// address arithmetic is needed.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t uniform_rsrc(const void* p) {
  const uint64_t a = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a), hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(((uint64_t)hi << 32) | lo), 0, -1, 0x00020000);
}

// MAC: work item (group tile, limb, position block, split).  Thread tid owns evaluation
// positions x0 = blk*512 + 2*tid and x0 + 1, which share the n-point value y = x0 >> log2 K'
// (K' >= 2), for the four or eight groups of its tile: per model ciphertext two words of c0
// and c1 and one transformed value per group, accumulated in 64-bit lazy sums.  The model
// word is below q < 2^30; the transformed value is below 2q for four-group tiles (a product
// below 2^61: four products fit above a folded sum, < 2^62 + 2^32) and below q for
// eight-group tiles (below 2^60: eight fit), so the sums fold every fourth or eighth
// ciphertext.  The loads run kSubDepth ciphertexts ahead through buffer resources at
// uniform bases; a tile's groups past the last one read the last group's values (their
// sums are not stored).  Tiles hold four groups, or eight when a launch scores more than
// four (batches, folded models).
constexpr int kSubDepth = 4;

template <int LOGKP, int kSubGroups>
__global__ __launch_bounds__(kSubThreads) void k_mac_sub(ScoreArgs a) {
  static_assert(LOGKP >= 1, "two positions per thread share one n-point value");
  constexpr int kFoldRounds = kSubGroups == 8 ? 2 : 1;
  static_assert(kSubDepth * kFoldRounds == (kSubGroups == 8 ? 8 : 4), "products between folds");
  const uint32_t N = (1u << a.sub_logn) << LOGKP, n = 1u << a.sub_logn, L = a.L;
  const uint32_t nblk = N / (2 * kSubThreads), ntile = (a.G + kSubGroups - 1) / kSubGroups;
  constexpr uint32_t ypi = (2u * kSubThreads) >> LOGKP;
  // item order: group tile, then limb, then position block, then split -- the tiles that
  // read one model slice are neighbours, and the XCD map runs neighbours on one XCD
  uint32_t w = XcdMap{a.xcd, a.nitems}.item(blockIdx.x);
  if (w == 0xFFFFFFFFu) return;  // a slot past the last item: the whole workgroup leaves
  const uint32_t tile = w % ntile;
  w /= ntile;
  const uint32_t l = w % L;
  w /= L;
  const uint32_t blk = w % nblk, split = w / nblk;
  const uint32_t g0 = tile * kSubGroups, ng = min((uint32_t)kSubGroups, a.G - g0);
  const uint32_t m0 = a.m_base + split * a.mchunk;
  const uint32_t m1 = min(a.m_base + a.m_len, m0 + a.mchunk);
  const uint32_t x0 = blk * 2 * kSubThreads + 2 * threadIdx.x, y = x0 >> LOGKP;
  const PrimeConst pc = a.pcs[l];
  // model words of (m, c): model + ((m * 2 + c) * L + l) * N + x0 (lane byte offset mo)
  const uint32_t* mod = a.model + (size_t)l * N;
  const uint32_t mo = x0 * 4u;
  const size_t mstride = (size_t)2 * L * N, cstride = (size_t)L * N;
  // transformed values of (g, m): pt + (((m - m_base) * L + l) * nblk + blk) * G * ypi +
  // g * ypi + y mod ypi (lane byte offset po)
  const uint32_t* pv = reinterpret_cast<const uint32_t*>(a.pt) + ((size_t)l * nblk + blk) * a.G * ypi + (size_t)g0 * ypi;
  const uint32_t po = (y % ypi) * 4u;
  const size_t pmstride = (size_t)L * a.G * n;

  uint64_t acc[kSubGroups][2][2];
#pragma unroll
  for (int k = 0; k < kSubGroups; ++k)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      uint32_t s0 = 0, s1 = 0;
      if (a.accumulate && (uint32_t)k < ng) {
        const uint32_t* src = a.partial + (((size_t)(g0 + k) * a.S + split) * 2 * L + (size_t)c * L + l) * N + x0;
        const uint2 s = *reinterpret_cast<const uint2*>(src);
        s0 = mont_mul(s.x, pc.r2, pc.m, pc.mneg_inv);
        s1 = mont_mul(s.y, pc.r2, pc.m, pc.mneg_inv);
      }
      acc[k][c][0] = s0;
      acc[k][c][1] = s1;
    }

  // byte strides of the loads: ciphertext m and component c of the model, plaintext m and
  // group k of the transformed values
  const uint32_t mb_ = (uint32_t)mstride * 4u, cb = (uint32_t)cstride * 4u, pb = (uint32_t)pmstride * 4u,
                 gb = ypi * 4u;
  struct Stage {
    v2u c0, c1;
    uint32_t p[kSubGroups];
  };
  // the loads of ciphertext d of a round: buffer resources at the round's uniform bases,
  // the lane's byte offset in a register and the ciphertext's and group's in scalars
  auto load = [&](Stage& st, const __amdgpu_buffer_rsrc_t& rm, const __amdgpu_buffer_rsrc_t& rp, int d) {
    st.c0 = __builtin_amdgcn_raw_buffer_load_b64(rm, mo, d * mb_, 0);
    st.c1 = __builtin_amdgcn_raw_buffer_load_b64(rm, mo, d * mb_ + cb, 0);
#pragma unroll
    for (int k = 0; k < kSubGroups; ++k)
      st.p[k] = __builtin_amdgcn_raw_buffer_load_b32(rp, po, d * pb + min((uint32_t)k, ng - 1) * gb, 0);
  };
  auto mac = [&](const Stage& st) {
#pragma unroll
    for (int k = 0; k < kSubGroups; ++k) {
      acc[k][0][0] += (uint64_t)st.c0.x * st.p[k];
      acc[k][0][1] += (uint64_t)st.c0.y * st.p[k];
      acc[k][1][0] += (uint64_t)st.c1.x * st.p[k];
      acc[k][1][1] += (uint64_t)st.c1.y * st.p[k];
    }
  };
  auto fold = [&] {
#pragma unroll
    for (int k = 0; k < kSubGroups; ++k)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        acc[k][c][0] = fold64(acc[k][c][0], pc.r1);
        acc[k][c][1] = fold64(acc[k][c][1], pc.r1);
      }
  };
  auto rsrc_model = [&](uint32_t m) { return uniform_rsrc(mod + (size_t)m * mstride); };
  auto rsrc_pt = [&](uint32_t m) { return uniform_rsrc(pv + (size_t)(m - a.m_base) * pmstride); };
  Stage ring[kSubDepth];
  uint32_t m = m0, round = 0;
  if (m < m1) {
    const auto rm = rsrc_model(m), rp = rsrc_pt(m);
#pragma unroll
    for (int d = 0; d < kSubDepth; ++d)
      if (m + d < m1) load(ring[d], rm, rp, d);
  }
  // full rounds whose next round is full too: each slot is used, then refilled for the
  // ciphertext kSubDepth ahead, without branches
  for (; m + 2 * kSubDepth <= m1; m += kSubDepth, ++round) {
    const auto rm = rsrc_model(m + kSubDepth), rp = rsrc_pt(m + kSubDepth);
#pragma unroll
    for (int d = 0; d < kSubDepth; ++d) {
      mac(ring[d]);
      load(ring[d], rm, rp, d);
    }
    if (round % kFoldRounds == kFoldRounds - 1) fold();
  }
  // the last one or two rounds
  for (; m < m1; m += kSubDepth, ++round) {
    const uint32_t next = m + kSubDepth;
    const auto rm = rsrc_model(next < m1 ? next : m), rp = rsrc_pt(next < m1 ? next : m);
#pragma unroll
    for (int d = 0; d < kSubDepth; ++d) {
      if (m + d < m1) mac(ring[d]);
      if (next + d < m1) load(ring[d], rm, rp, d);
    }
    if (round % kFoldRounds == kFoldRounds - 1) fold();
  }
#pragma unroll
  for (int k = 0; k < kSubGroups; ++k) {
    if ((uint32_t)k >= ng) break;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      uint32_t* dst = a.partial + (((size_t)(g0 + k) * a.S + split) * 2 * L + (size_t)c * L + l) * N + x0;
      *reinterpret_cast<uint2*>(dst) = make_uint2(redc64(fold64(acc[k][c][0], pc.r1), pc.m, pc.mneg_inv),
                                                  redc64(fold64(acc[k][c][1], pc.r1), pc.m, pc.mneg_inv));
    }
  }
}

// ------------------------------------------------------------------ request-list kernels
// Persistent kernels over the segments of many requests (one launch for all of them):
// workgroup w takes items w, w + gridDim.x, ...  Every request of a list shares N and the
// ciphertext moduli; K, D and the model differ, so the scatter table is restaged whenever
// the request's table changes.
template <int LOGN, int LE>
__device__ __forceinline__ void restage(const uint32_t* scatter, const uint32_t*& staged, int tid) {
  if (scatter != staged) {
    lds_barrier();  // every wave is done reading the previous table
    stage_table<LOGN, LE>(scatter, tid);
    staged = scatter;
  }
}

__device__ __forceinline__ QuerySrc query_src(const ReqDesc& r, uint32_t g) {
  return QuerySrc{r.hv + (size_t)g * r.B, r.D, r.r, r.hv_stride, min(r.B, r.Q - g * r.B)};
}

template <int LOGN, int LE, int LG>
__global__ __launch_bounds__((1 << LOGN) >> LE) void k_score_list(ListArgs a) {
  using S = Shape<LOGN, LE>;
  LdsBufs b{0};
  const int tid = threadIdx.x;
  const uint32_t* staged = nullptr;
  const uint32_t nd = a.xm.slots();
  for (uint32_t d = blockIdx.x; d < nd; d += gridDim.x) {
    const uint32_t w = a.xm.item(d);
    if (w == 0xFFFFFFFFu) continue;
    const Segment sg = a.segs[w / a.NLG];
    const ReqDesc r = a.reqs[sg.req];
    restage<LOGN, LE>(r.scatter, staged, tid);
    const MacItem it{r.model, a.partial + (size_t)sg.slot * 2 * a.L * S::N, a.L, sg.m0, sg.m1, (w % a.NLG) * LG,
                      r.scale};
    score_item<LOGN, LE, LG>(it, query_src(r, sg.g), r.scatter, a.ts, a.fwd_tw, a.pcs, tid, b);
  }
}

template <int LOGN, int LE>
__global__ __launch_bounds__((1 << LOGN) >> LE) void k_encode_list(ListArgs a) {
  using S = Shape<LOGN, LE>;
  LdsBufs b{0};
  const int tid = threadIdx.x;
  const uint32_t* staged = nullptr;
  if constexpr (LdsPlan<LOGN, LE>::table_in_lds) {  // one inverse table mod t for every request
    stage_twiddles<LOGN, LE>(a.ts.inv_t, tid);
    lds_barrier();
  }
  for (uint32_t w = blockIdx.x; w < a.nseg; w += gridDim.x) {
    const Segment sg = a.segs[w];
    const ReqDesc r = a.reqs[sg.req];
    int32_t* dst = a.pt + (size_t)sg.pt * S::N;
    if constexpr (LdsPlan<LOGN, LE>::table_in_lds) {
      encode_item<LOGN, LE, true>(query_src(r, sg.g), r.scatter, a.ts, sg.m0, sg.m1, dst, tid, b);
    } else {
      restage<LOGN, LE>(r.scatter, staged, tid);
      encode_item<LOGN, LE>(query_src(r, sg.g), r.scatter, a.ts, sg.m0, sg.m1, dst, tid, b);
    }
  }
}

template <int LOGN, int LE, int LG, bool PF, bool SC = false>
__global__ __launch_bounds__((1 << LOGN) >> LE) void k_mac_list(ListArgs a) {
  using S = Shape<LOGN, LE>;
  LdsBufs b{0};
  const int tid = threadIdx.x;
  const uint32_t nd = a.xm.slots();
  uint32_t staged_l = 0xFFFFFFFFu;  // limb whose twiddles the LDS table slot holds
  for (uint32_t d = blockIdx.x; d < nd; d += gridDim.x) {
    const uint32_t w = a.xm.item(d);
    if (w == 0xFFFFFFFFu) continue;
    const Segment sg = a.segs[w / a.NLG];
    const ReqDesc r = a.reqs[sg.req];
    const MacItem it{r.model, a.partial + (size_t)sg.slot * 2 * a.L * S::N, a.L, sg.m0, sg.m1, (w % a.NLG) * LG,
                      r.scale};
    if constexpr (mac_lds_twiddles<LOGN, LE, LG>()) {
      if (it.l0 != staged_l) {  // every request of a list shares the moduli and their tables
        lds_barrier();          // every wave is done with the previous limb's table
        stage_twiddles<LOGN, LE>(a.fwd_tw + (size_t)it.l0 * S::N, tid);
        lds_barrier();
        staged_l = it.l0;
      }
      mac_item<LOGN, LE, LG, PF, true, PF, SC>(it, a.pt + (size_t)sg.pt * S::N, false, a.fwd_tw, a.pcs, tid, b);
    } else {
      mac_item<LOGN, LE, LG, PF, false, PF, SC>(it, a.pt + (size_t)sg.pt * S::N, false, a.fwd_tw, a.pcs, tid, b);
    }
  }
}

// Finish of a request list: polynomial (c, l) of output item (request, g) sums the slots
// of the group's segments; requests with r = 1 are transformed to the coefficient domain,
// folded ones (r > 1) stay in the evaluation domain for their rotations.
template <int LOGN, int LE>
__global__ __launch_bounds__((1 << LOGN) >> LE) void k_finish_list(ListArgs a) {
  using S = Shape<LOGN, LE>;
  const int tid = threadIdx.x;
  const uint32_t poly = blockIdx.x % (2 * a.L), item = blockIdx.x / (2 * a.L);
  const uint32_t l = poly % a.L;
  const FinishItem f = a.fin[item];
  const ReqDesc r = a.reqs[f.req];
  const PrimeConst pc = a.pcs[l];
  uint32_t v[S::E];
#pragma unroll
  for (int i = 0; i < S::E; ++i) v[i] = 0;
  for (uint32_t sl = f.slot0; sl < f.slot0 + f.nslot; ++sl) {
    const uint32_t* src = a.partial + ((size_t)sl * 2 * a.L + poly) * S::N + (size_t)tid * S::E;
#pragma unroll
    for (int i = 0; i < S::E; ++i) v[i] = csub(v[i] + src[i], pc.m);
  }
  uint32_t* out = r.out + ((size_t)f.g * 2 * a.L + poly) * S::N;
  if (r.r == 1) {
    LdsBufs b{0};
    ntt_inverse<LOGN, LE, true>(v, tid, a.inv_tw + (size_t)l * S::N, pc, b);
#pragma unroll
    for (int i = 0; i < S::E; ++i) out[tid + i * S::T] = csub(v[i], pc.m);
  } else {
#pragma unroll
    for (int i = 0; i < S::E; ++i) out[(size_t)tid * S::E + i] = v[i];
  }
}

// Sum the S partial accumulators of every (g, c, l) (evaluation domain) and either store
// the sum (for the rotation steps) or transform it straight to the coefficient domain.
template <int LOGN, int LE, bool INVERT>
__global__ __launch_bounds__((1 << LOGN) >> LE) void k_finish(const uint32_t* __restrict__ partial,
                                                               uint32_t* __restrict__ out, uint32_t S_,
                                                               uint32_t L, const uint32_t* __restrict__ inv_tw,
                                                               const PrimeConst* __restrict__ pcs) {
  using S = Shape<LOGN, LE>;
  const int tid = threadIdx.x;
  const uint32_t poly = blockIdx.x;  // (g*2 + c)*L + l
  const uint32_t l = poly % L, gc = poly / L;
  const uint32_t c = gc % 2, g = gc / 2;
  const PrimeConst pc = pcs[l];
  uint32_t v[S::E];
#pragma unroll
  for (int i = 0; i < S::E; ++i) v[i] = 0;
  for (uint32_t sp = 0; sp < S_; ++sp) {
    const uint32_t* src = partial + ((((size_t)g * S_ + sp) * 2 + c) * L + l) * S::N + (size_t)tid * S::E;
#pragma unroll
    for (int i = 0; i < S::E; ++i) v[i] = csub(v[i] + src[i], pc.m);
  }
  if constexpr (INVERT) {
    LdsBufs b{0, 0, one_buffer<LOGN, LE>()};
    ntt_inverse<LOGN, LE, true>(v, tid, inv_tw + (size_t)l * S::N, pc, b);
    uint32_t* dst = out + (size_t)poly * S::N;
#pragma unroll
    for (int i = 0; i < S::E; ++i) dst[tid + i * S::T] = csub(v[i], pc.m);
  } else {
    uint32_t* dst = out + (size_t)poly * S::N + (size_t)tid * S::E;
#pragma unroll
    for (int i = 0; i < S::E; ++i) dst[i] = v[i];
  }
}

// Debug: the lifted query plaintext (g, m) in every limb, coefficient domain [L][N].
template <int LOGN, int LE>
__global__ __launch_bounds__((1 << LOGN) >> LE) void k_debug_plaintext(ScoreArgs a, uint32_t g, uint32_t m,
                                                                        uint32_t* __restrict__ out) {
  using S = Shape<LOGN, LE>;
  LdsBufs b{0};
  const int tid = threadIdx.x;
  stage_table<LOGN, LE>(a.scatter, tid);
  uint32_t mu[S::E], ent[S::E], du[S::E], off[S::E];
  const QuerySrc q = query_src(a, g);
  table_entries<LOGN, LE>(ent, a.scatter, tid);
  scatter_offsets<LOGN, LE>(du, off, ent, q);
  encode_query<LOGN, LE>(mu, q, du, off, tside(a), m, tid, b);
  for (uint32_t l = 0; l < a.L; ++l) {
    const uint32_t qm = a.pcs[l].m;
#pragma unroll
    for (int i = 0; i < S::E; ++i) out[(size_t)l * S::N + tid + i * S::T] = lift(mu[i], a.pct.m, qm);
  }
}

}  // namespace ephdc_dev

// ------------------------------------------------------------------ launchers
namespace ephdc {

using namespace ephdc_dev;

// Raises the dynamic-LDS limit of every kernel instantiation once per process.
template <int LOGN, int LE>
static hipError_t prepare_shape() {
  const int bytes = (int)lds_bytes<LOGN, LE>();
  hipError_t e = hipSuccess;
  auto set = [&](const void* f) {
    if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  };
  set((const void*)k_fwd_batch<LOGN, LE>);
  set((const void*)k_inv_batch<LOGN, LE>);
  set((const void*)k_score<LOGN, LE, 1>);
  set((const void*)k_score<LOGN, LE, 2>);
  set((const void*)k_score<LOGN, LE, 3>);
  set((const void*)k_score<LOGN, LE, 4>);
  set((const void*)k_encode_pt<LOGN, LE>);
  set((const void*)k_mac<LOGN, LE, 1, mac_prefetch<LOGN, LE>()>);
  set((const void*)k_mac<LOGN, LE, 2, mac_prefetch<LOGN, LE>()>);
  set((const void*)k_mac<LOGN, LE, 4, mac_prefetch<LOGN, LE>()>);
  set((const void*)k_mac<LOGN, LE, 1, mac_prefetch<LOGN, LE>(), true>);
  set((const void*)k_mac<LOGN, LE, 2, mac_prefetch<LOGN, LE>(), true>);
  set((const void*)k_mac<LOGN, LE, 4, mac_prefetch<LOGN, LE>(), true>);
  set((const void*)k_finish<LOGN, LE, true>);
  set((const void*)k_finish<LOGN, LE, false>);
  set((const void*)k_debug_plaintext<LOGN, LE>);
  set((const void*)k_score_list<LOGN, LE, 1>);
  set((const void*)k_score_list<LOGN, LE, 2>);
  set((const void*)k_score_list<LOGN, LE, 4>);
  set((const void*)k_encode_list<LOGN, LE>);
  set((const void*)k_mac_list<LOGN, LE, 1, mac_prefetch<LOGN, LE>()>);
  set((const void*)k_mac_list<LOGN, LE, 2, mac_prefetch<LOGN, LE>()>);
  set((const void*)k_mac_list<LOGN, LE, 4, mac_prefetch<LOGN, LE>()>);
  set((const void*)k_mac_list<LOGN, LE, 1, mac_prefetch<LOGN, LE>(), true>);
  set((const void*)k_mac_list<LOGN, LE, 2, mac_prefetch<LOGN, LE>(), true>);
  set((const void*)k_mac_list<LOGN, LE, 4, mac_prefetch<LOGN, LE>(), true>);
  set((const void*)k_finish_list<LOGN, LE>);
  return e;
}

// The subring batch-encoding kernels (one wave per n-point transform).
template <int LS>
static hipError_t prepare_sub() {
  constexpr int LE = sub_le(LS);
  return hipFuncSetAttribute((const void*)k_encode_sub<LS, LE>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)encode_sub_lds_bytes<LS, LE>());
}

hipError_t prepare_kernels() {
  static hipError_t once = [] {
    hipError_t ks = prepare_ks_kernels();
    if (ks != hipSuccess) return ks;
    hipError_t e = prepare_sub<8>();
    if (e == hipSuccess) e = prepare_sub<9>();
    if (e == hipSuccess) e = prepare_sub<10>();
    if (e == hipSuccess) e = prepare_sub<11>();
    if (e == hipSuccess) e = prepare_sub<12>();
    if (e == hipSuccess) e = prepare_shape<11, 3>();
    if (e == hipSuccess) e = prepare_shape<12, 3>();
    if (e == hipSuccess) e = prepare_shape<13, 3>();
    if (e == hipSuccess) e = prepare_shape<13, 4>();
    if (e == hipSuccess) e = prepare_shape<14, 4>();
    if (e == hipSuccess) e = prepare_shape<14, 5>();
    return e;
  }();
  return once;
}

bool supported_shape(int logn, int le) {
  return le == 0 || ((logn == 11 || logn == 12) && le == 3) || (logn == 13 && (le == 3 || le == 4)) ||
         (logn == 14 && (le == 4 || le == 5));
}

bool supported_logn(int logn) { return logn >= 11 && logn <= 14; }


static PolyMap make_map(const BatchMap& m, uint32_t N) {
  PolyMap pm;
  pm.in_per = m.in_per ? m.in_per : 1;
  pm.out_per = m.out_per ? m.out_per : 1;
  pm.in_stride = m.in_per ? m.in_stride : N;
  pm.out_stride = m.out_per ? m.out_stride : N;
  return pm;
}

hipError_t launch_fwd_batch(int logn, const uint32_t* in, uint32_t* out, size_t npolys, const uint32_t* tw,
                            const PrimeConst* pcs, uint32_t nlimb, uint32_t limb_base, bool mont,
                            hipStream_t st, const BatchMap& map) {
  if (npolys == 0) return hipSuccess;
  return dispatch(logn, [&](auto lnc, auto lec) {
    constexpr int LN = decltype(lnc)::value, LEv = decltype(lec)::value;
    const size_t sh = lds_bytes_one_transform<LN, LEv>();
    k_fwd_batch<LN, LEv><<<dim3((unsigned)npolys), dim3(Shape<LN, LEv>::T), sh, st>>>(
        in, out, tw, pcs, nlimb, limb_base, mont ? 1 : 0, make_map(map, 1u << LN));
    return hipGetLastError();
  });
}

hipError_t launch_inv_batch(int logn, const uint32_t* in, uint32_t* out, size_t npolys, const uint32_t* itw,
                            const PrimeConst* pcs, uint32_t nlimb, uint32_t limb_base, hipStream_t st,
                            const BatchMap& map) {
  if (npolys == 0) return hipSuccess;
  return dispatch(logn, [&](auto lnc, auto lec) {
    constexpr int LN = decltype(lnc)::value, LEv = decltype(lec)::value;
    const size_t sh = lds_bytes_one_transform<LN, LEv>();
    k_inv_batch<LN, LEv><<<dim3((unsigned)npolys), dim3(Shape<LN, LEv>::T), sh, st>>>(
        in, out, itw, pcs, nlimb, limb_base, make_map(map, 1u << LN));
    return hipGetLastError();
  });
}

hipError_t launch_pointwise_mont(const uint32_t* a, const uint32_t* b, uint32_t* out, size_t n, uint32_t N,
                                 const PrimeConst* pcs, uint32_t nlimb, hipStream_t st) {
  if (n == 0) return hipSuccess;
  unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 65536);
  k_pointwise_mont<<<dim3(blocks), dim3(256), 0, st>>>(a, b, out, n, N, pcs, nlimb);
  return hipGetLastError();
}

XcdMap make_xcd_map(uint32_t n) {
  XcdMap m{0, n};
#ifndef EPHDC_NO_XCD_ORDER
  m.on = n >= 64 ? 1u : 0u;
#endif
  return m;
}

hipError_t launch_score(int logn, int le, int lg, const ScoreArgs& a0, uint32_t nblocks, hipStream_t st) {
  if (nblocks == 0) return hipSuccess;
  ScoreArgs a = a0;
  const XcdMap xm = make_xcd_map(nblocks);
  a.xcd = xm.on;
  a.nitems = nblocks;
  return dispatch(logn, le, [&](auto lnc, auto lec) {
    constexpr int LN = decltype(lnc)::value, LEv = decltype(lec)::value;
    const dim3 grid(xm.slots()), block(Shape<LN, LEv>::T);
    const size_t sh = lds_bytes<LN, LEv>();
    switch (lg) {
      case 1: k_score<LN, LEv, 1><<<grid, block, sh, st>>>(a); break;
      case 2: k_score<LN, LEv, 2><<<grid, block, sh, st>>>(a); break;
      case 3: k_score<LN, LEv, 3><<<grid, block, sh, st>>>(a); break;
      case 4: k_score<LN, LEv, 4><<<grid, block, sh, st>>>(a); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  });
}

hipError_t launch_encode_pt(int logn, int le, const ScoreArgs& a, uint32_t nblocks, hipStream_t st) {
  if (nblocks == 0) return hipSuccess;
  return dispatch(logn, le, [&](auto lnc, auto lec) {
    constexpr int LN = decltype(lnc)::value, LEv = decltype(lec)::value;
    k_encode_pt<LN, LEv><<<dim3(nblocks), dim3(Shape<LN, LEv>::T), lds_bytes<LN, LEv>(), st>>>(a);
    return hipGetLastError();
  });
}

hipError_t launch_mac(int logn, int le, int lg, const ScoreArgs& a0, uint32_t nblocks, hipStream_t st) {
  if (nblocks == 0) return hipSuccess;
  ScoreArgs a = a0;
  const XcdMap xm = make_xcd_map(nblocks);
  a.xcd = xm.on;
  a.nitems = nblocks;
  return dispatch(logn, le, [&](auto lnc, auto lec) {
    constexpr int LN = decltype(lnc)::value, LEv = decltype(lec)::value;
    const dim3 grid(xm.slots()), block(Shape<LN, LEv>::T);
    const size_t sh = lds_bytes<LN, LEv>();
    constexpr bool P = mac_prefetch<LN, LEv>();
    const bool sc = a.scale.pow != nullptr;
    switch (lg * 2 + (sc ? 1 : 0)) {
      case 2: k_mac<LN, LEv, 1, P><<<grid, block, sh, st>>>(a); break;
      case 3: k_mac<LN, LEv, 1, P, true><<<grid, block, sh, st>>>(a); break;
      case 4: k_mac<LN, LEv, 2, P><<<grid, block, sh, st>>>(a); break;
      case 5: k_mac<LN, LEv, 2, P, true><<<grid, block, sh, st>>>(a); break;
      case 8: k_mac<LN, LEv, 4, P><<<grid, block, sh, st>>>(a); break;
      case 9: k_mac<LN, LEv, 4, P, true><<<grid, block, sh, st>>>(a); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  });
}

// Groups per streaming-MAC tile for a launch of G groups: four, or eight above four.
static uint32_t sub_tile(uint32_t G) { return G > 4 ? 8u : 4u; }

uint32_t mac_sub_items(uint32_t N, uint32_t L, uint32_t G) {
  const uint32_t gt = sub_tile(G);
  return (N / (2 * kSubThreads)) * L * ((G + gt - 1) / gt);
}

bool subring_kernels(int logn, int sub_logn) {
  return logn >= 11 && logn <= 14 && sub_logn >= 8 && sub_logn <= 12 && sub_logn < logn && logn - sub_logn <= 5;
}

template <class F>
hipError_t dispatch_sub(int sub_logn, F&& f) {
  switch (sub_logn) {
    case 8: return f(std::integral_constant<int, 8>{});
    case 9: return f(std::integral_constant<int, 9>{});
    case 10: return f(std::integral_constant<int, 10>{});
    case 11: return f(std::integral_constant<int, 11>{});
    case 12: return f(std::integral_constant<int, 12>{});
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_encode_sub(int sub_logn, const ScoreArgs& a, uint32_t splits, hipStream_t st) {
  if (splits == 0 || a.G == 0) return hipSuccess;
  return dispatch_sub(sub_logn, [&](auto lc) {
    constexpr int LS = decltype(lc)::value, LE = sub_le(LS);
    constexpr uint32_t TPW = encode_sub_threads<LS, LE>() / Shape<LS, LE>::T;
    const dim3 grid((a.G + TPW - 1) / TPW * splits);
    k_encode_sub<LS, LE><<<grid, dim3(encode_sub_threads<LS, LE>()), encode_sub_lds_bytes<LS, LE>(), st>>>(a);
    return hipGetLastError();
  });
}

uint32_t mac_sub_resident_blocks(uint32_t G) {
  auto count = [](const void* f) {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kSubThreads, 0) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return 1024u;
    return (uint32_t)std::max(1, per_cu * cus);
  };
  static const uint32_t n4 = count((const void*)k_mac_sub<3, 4>), n8 = count((const void*)k_mac_sub<3, 8>);
  return sub_tile(G) == 8 ? n8 : n4;
}

hipError_t launch_mac_sub(int logn, int sub_logn, const ScoreArgs& a0, uint32_t nblocks, hipStream_t st) {
  if (nblocks == 0) return hipSuccess;
  if (!subring_kernels(logn, sub_logn)) return hipErrorInvalidValue;
  ScoreArgs a = a0;
  const XcdMap xm = make_xcd_map(nblocks);
  a.xcd = xm.on;
  a.nitems = nblocks;
  const dim3 grid(xm.slots());
  const bool wide = sub_tile(a.G) == 8;
  switch ((logn - sub_logn) * 2 + (wide ? 1 : 0)) {
    case 2: k_mac_sub<1, 4><<<grid, dim3(kSubThreads), 0, st>>>(a); break;
    case 3: k_mac_sub<1, 8><<<grid, dim3(kSubThreads), 0, st>>>(a); break;
    case 4: k_mac_sub<2, 4><<<grid, dim3(kSubThreads), 0, st>>>(a); break;
    case 5: k_mac_sub<2, 8><<<grid, dim3(kSubThreads), 0, st>>>(a); break;
    case 6: k_mac_sub<3, 4><<<grid, dim3(kSubThreads), 0, st>>>(a); break;
    case 7: k_mac_sub<3, 8><<<grid, dim3(kSubThreads), 0, st>>>(a); break;
    case 8: k_mac_sub<4, 4><<<grid, dim3(kSubThreads), 0, st>>>(a); break;
    case 9: k_mac_sub<4, 8><<<grid, dim3(kSubThreads), 0, st>>>(a); break;
    case 10: k_mac_sub<5, 4><<<grid, dim3(kSubThreads), 0, st>>>(a); break;
    case 11: k_mac_sub<5, 8><<<grid, dim3(kSubThreads), 0, st>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_finish(int logn, bool invert, const uint32_t* partial, uint32_t* out, uint32_t G, uint32_t S_,
                         uint32_t L, const uint32_t* itw, const PrimeConst* pcs, hipStream_t st) {
  if (G == 0) return hipSuccess;
  return dispatch(logn, [&](auto lnc, auto lec) {
    constexpr int LN = decltype(lnc)::value, LEv = decltype(lec)::value;
    const dim3 grid(G * 2 * L), block(Shape<LN, LEv>::T);
    const size_t sh = lds_bytes_one_transform<LN, LEv>();
    if (invert)
      k_finish<LN, LEv, true><<<grid, block, sh, st>>>(partial, out, S_, L, itw, pcs);
    else
      k_finish<LN, LEv, false><<<grid, block, sh, st>>>(partial, out, S_, L, itw, pcs);
    return hipGetLastError();
  });
}

// Persistent list launches: the grid is rounded up to a multiple of 8 so that a workgroup
// stays on one XCD for all of its dispatch slots.
static uint32_t list_grid(uint32_t grid, uint32_t slots) {
  grid = std::min(grid, slots);
  return (grid + 7u) & ~7u;
}

hipError_t launch_score_list(int logn, int le, int lg, const ListArgs& a0, uint32_t grid, hipStream_t st) {
  if (grid == 0 || a0.nseg == 0) return hipSuccess;
  ListArgs a = a0;
  a.xm = make_xcd_map(a.nseg * a.NLG);
  grid = list_grid(grid, a.xm.slots());
  return dispatch(logn, le, [&](auto lnc, auto lec) {
    constexpr int LN = decltype(lnc)::value, LEv = decltype(lec)::value;
    const dim3 g(grid), block(Shape<LN, LEv>::T);
    const size_t sh = lds_bytes<LN, LEv>();
    switch (lg) {
      case 1: k_score_list<LN, LEv, 1><<<g, block, sh, st>>>(a); break;
      case 2: k_score_list<LN, LEv, 2><<<g, block, sh, st>>>(a); break;
      case 4: k_score_list<LN, LEv, 4><<<g, block, sh, st>>>(a); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  });
}

hipError_t launch_encode_list(int logn, int le, const ListArgs& a, uint32_t grid, hipStream_t st) {
  if (grid == 0 || a.nseg == 0) return hipSuccess;
  return dispatch(logn, le, [&](auto lnc, auto lec) {
    constexpr int LN = decltype(lnc)::value, LEv = decltype(lec)::value;
    k_encode_list<LN, LEv><<<dim3(grid), dim3(Shape<LN, LEv>::T), lds_bytes<LN, LEv>(), st>>>(a);
    return hipGetLastError();
  });
}

hipError_t launch_mac_list(int logn, int le, int lg, const ListArgs& a0, uint32_t grid, hipStream_t st) {
  if (grid == 0 || a0.nseg == 0) return hipSuccess;
  ListArgs a = a0;
  a.xm = make_xcd_map(a.nseg * a.NLG);
  grid = list_grid(grid, a.xm.slots());
  return dispatch(logn, le, [&](auto lnc, auto lec) {
    constexpr int LN = decltype(lnc)::value, LEv = decltype(lec)::value;
    const dim3 g(grid), block(Shape<LN, LEv>::T);
    const size_t sh = lds_bytes<LN, LEv>();
    constexpr bool P = mac_prefetch<LN, LEv>();
    switch (lg * 2 + (a.scaled ? 1 : 0)) {
      case 2: k_mac_list<LN, LEv, 1, P><<<g, block, sh, st>>>(a); break;
      case 3: k_mac_list<LN, LEv, 1, P, true><<<g, block, sh, st>>>(a); break;
      case 4: k_mac_list<LN, LEv, 2, P><<<g, block, sh, st>>>(a); break;
      case 5: k_mac_list<LN, LEv, 2, P, true><<<g, block, sh, st>>>(a); break;
      case 8: k_mac_list<LN, LEv, 4, P><<<g, block, sh, st>>>(a); break;
      case 9: k_mac_list<LN, LEv, 4, P, true><<<g, block, sh, st>>>(a); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  });
}

hipError_t launch_finish_list(int logn, const ListArgs& a, hipStream_t st) {
  if (a.nfin == 0) return hipSuccess;
  return dispatch(logn, [&](auto lnc, auto lec) {
    constexpr int LN = decltype(lnc)::value, LEv = decltype(lec)::value;
    k_finish_list<LN, LEv><<<dim3(a.nfin * 2 * a.L), dim3(Shape<LN, LEv>::T), lds_bytes<LN, LEv>(), st>>>(a);
    return hipGetLastError();
  });
}

hipError_t launch_debug_plaintext(int logn, const ScoreArgs& a, uint32_t g, uint32_t m, uint32_t* out,
                                  hipStream_t st) {
  return dispatch(logn, [&](auto lnc, auto lec) {
    constexpr int LN = decltype(lnc)::value, LEv = decltype(lec)::value;
    const size_t sh = lds_bytes<LN, LEv>();
    k_debug_plaintext<LN, LEv><<<dim3(1), dim3(Shape<LN, LEv>::T), sh, st>>>(a, g, m, out);
    return hipGetLastError();
  });
}

}  // namespace ephdc
