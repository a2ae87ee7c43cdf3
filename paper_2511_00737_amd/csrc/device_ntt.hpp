// Device-side modular arithmetic and register/LDS-resident negacyclic transforms for gfx950.
//
// Layout of one transform: N = 2^LOGN coefficients spread over T = N/E threads of a
// workgroup, E = 2^LE values per thread held in VGPRs.  The LOGN butterfly stages are
// grouped into passes of up to LE stages that run entirely in registers; between passes
// the values are exchanged through LDS (double-buffered, one barrier per exchange).
//
// Transform order (the library's evaluation domain): position x holds a(w^(2*brev(x)+1)).
// Register layouts:
//   coefficient side   thread tid holds positions tid + i*T   (i < E)  -- coalesced rows
//   evaluation side    thread tid holds positions tid*E + i   (i < E)  -- contiguous chunk
// The forward transform (Cooley-Tukey, Harvey lazy butterflies) maps the first to the
// second; the inverse (Gentleman-Sande) maps the second back to the first.
//
// Modular arithmetic (all moduli < 2^30, so lazy values below 4m fit in 32 bits):
//   Montgomery multiplication (R = 2^32): two 64-bit multiply-adds and one multiply, result
//   in [0, 2m) whenever a*b < m*2^32.  Twiddle tables and the N^-1 constants are stored in
//   Montgomery form (w*R mod m), so multiplying by them yields plain residues.
//   Shoup multiplication by a constant w with w' = floor(w*2^32/m): 3 multiplies and a
//   subtraction, result in [0, 2m) for any 32-bit input (used by the base conversions).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ephdc_dev {

struct PrimeConst {
  uint32_t m;         // modulus
  uint32_t mneg_inv;  // -m^-1 mod 2^32 (Montgomery)
  uint32_t r2;        // 2^64 mod m (to enter Montgomery form)
  uint32_t ninv_r;     // N^-1 * 2^32 mod m (Montgomery form)
  uint32_t ninv_w1_r;  // N^-1 * (first inverse twiddle) * 2^32 mod m
  uint32_t r1;         // 2^32 mod m (folds the high word of a 64-bit sum)
  uint32_t pad[2];
};

__device__ __forceinline__ uint32_t mul_shoup(uint32_t a, uint32_t w, uint32_t wp, uint32_t m) {
  const uint32_t qh = __umulhi(a, wp);
  return a * w - qh * m;
}

__device__ __forceinline__ uint32_t csub(uint32_t a, uint32_t m) { return a >= m ? a - m : a; }

// Global access at a uniform base plus a 32-bit byte offset: the form the scalar-base,
// vector-offset addressing mode takes (no 64-bit address arithmetic per lane).
template <class T>
__device__ __forceinline__ T ld_at(const T* base, uint32_t byte_off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}
template <class T>
__device__ __forceinline__ void st_at(T* base, uint32_t byte_off, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off) = v;
}

__device__ __forceinline__ uint32_t mont_mul(uint32_t a, uint32_t b, uint32_t m, uint32_t mneg_inv) {
  // (a*b + k*m) / 2^32 with k = (a*b mod 2^32) * (-m^-1): the low word of the sum is zero, so
  // the high word of one 64-bit multiply-add is the exact result (a*b + k*m < 2^63 whenever
  // a*b < 2^62).  In [0, 2m) for a*b < m*2^32.
  const uint64_t T = (uint64_t)a * b;
  const uint32_t k = (uint32_t)T * mneg_inv;
  return (uint32_t)(((uint64_t)k * m + T) >> 32);
}

// Full reduction of a lazy value in [0, 4m) to [0, m).
__device__ __forceinline__ uint32_t reduce4(uint32_t a, uint32_t m) { return csub(csub(a, 2 * m), m); }

// Lazy 64-bit multiply-accumulate for sums of products a*b with a < m, b < 4m (each below
// 2^62).  fold64 keeps the residue mod m and brings any sum below 2^64 back under
// 2^62 + 2^32 (hi * (2^32 mod m) + lo), so two products may be added between folds.
// redc64 ends the sum: for sums of Montgomery-form a (a*2^32 mod m) it returns the plain
// residue of sum a*b in [0, m).
__device__ __forceinline__ uint64_t fold64(uint64_t x, uint32_t r1) {
  return (uint64_t)(uint32_t)(x >> 32) * r1 + (uint32_t)x;
}
__device__ __forceinline__ uint32_t redc64(uint64_t x, uint32_t m, uint32_t mneg_inv) {
  // x < 2^62 + 2^32 after a fold: (x + k*m) / 2^32 < 2^31 + 2 < 4m, then two corrections
  const uint32_t k = (uint32_t)x * mneg_inv;
  return reduce4((uint32_t)(((uint64_t)k * m + x) >> 32), m);
}

template <int LOGN, int LE>
struct Shape {
  static constexpr int N = 1 << LOGN;
  static constexpr int E = 1 << LE;
  static constexpr int T = N / E;
  static constexpr int NFULL = LOGN / LE;
  static constexpr int REM = LOGN % LE;
  static constexpr int NPASS = NFULL + (REM ? 1 : 0);
  static constexpr int PADN = N + T;  // LDS words per exchange buffer: 64*E + 64 per wave
  static constexpr int s0(int p) { return p * LE; }
  static constexpr int k(int p) { return p < NFULL ? LE : REM; }
};

// Position handled by register i of thread tid during pass P.
// Pass P covers stages s0..s0+k-1; its butterfly groups have 2^k members at stride
// tmin = N >> (s0+k).  Thread tid takes groups tid + T*e (e < E/2^k), except in the last
// pass, where it takes the consecutive groups tid*E/2^k + e so that it ends up owning the
// contiguous chunk tid*E .. tid*E+E-1.
//
// The position is the bitwise OR of a part that depends only on tid and a part that
// depends only on i (their bit ranges never overlap), so every address derived from it by
// shifts and the LDS padding splits into a per-thread base plus a compile-time offset.
template <int LOGN, int LE, int P>
__host__ __device__ constexpr int tid_part(int tid) {
  using S = Shape<LOGN, LE>;
  constexpr int k = S::k(P);
  constexpr int tl = LOGN - S::s0(P) - k;  // log2(tmin)
  if constexpr (P == S::NPASS - 1) {
    return tid << LE;
  } else {
    return ((tid >> tl) << (tl + k)) | (tid & ((1 << tl) - 1));
  }
}

template <int LOGN, int LE, int P>
__host__ __device__ constexpr int i_part(int i) {
  using S = Shape<LOGN, LE>;
  constexpr int k = S::k(P);
  constexpr int tl = LOGN - S::s0(P) - k;
  if constexpr (P == S::NPASS - 1) {
    return i;
  } else {
    // group e of the thread is gamma = tid + T*e: its block index grows by T >> tl per e
    return ((((S::T >> tl) * (i >> k)) << (tl + k)) | ((i & ((1 << k) - 1)) << tl));
  }
}

// True when, in the layout of pass P, every wave owns exactly the contiguous block of
// positions [w*64*E, (w+1)*64*E): exchanges between two such layouts never cross waves.
template <int LOGN, int LE, int P>
__host__ __device__ constexpr bool wave_local() {
  using S = Shape<LOGN, LE>;
  constexpr int k = S::k(P);
  constexpr int tl = LOGN - S::s0(P) - k;
  if constexpr (P == S::NPASS - 1) {
    return true;  // x = tid*E + i
  } else {
    // x = ((tid >> tl) << (tl+k)) | (tid & (2^tl-1)) | i-part; the wave index tid >> 6 must equal
    // x >> (6 + LE) for every register, i.e. tl <= 6 and the group stride covers 64*E exactly
    return tl <= 6 && (6 - tl) + (tl + k) == 6 + LE && (S::E >> k) == 1;
  }
}

// LDS placement of an exchange.  A wave's block of positions is [64E*w, 64E*(w+1)), so
// position x splits into the wave part x >> B and the bits below B = 6 + LE.  Position x is
// stored at R*(x >> B) + sum over b < B of bit_b(x) * w[b], with R = 64E + 64 words per
// wave and per-bit weights w[b] chosen for the exchange.  The map is additive over bits,
// so it distributes over the disjoint tid / register parts of a position: the address is a
// per-thread base plus a compile-time offset.
//
// The LDS of gfx950 serves a wave's 32-bit accesses from 64 banks of 4 bytes.  For one
// register, the 64 lanes of a layout vary exactly six position bits (the lane bits), and
// the lanes hit 64 distinct banks when the six weights of those bits have distinct 2-adic
// valuations 0..5 mod 64.  The weights are found at compile time by a depth-first search
// over bits in increasing order: each weight is the smallest number above the sum of the
// previous ones (which keeps the map one-to-one) whose valuation is still free in the
// write layout and in the read layout it belongs to, and the sum must stay below R.  Every
// wave's image then lies in its own range [R*w, R*(w+1)) under every exchange's
// placement, which wave-local exchanges (no workgroup barrier) rely on.
constexpr int kMaxPadBits = 12;
struct Pad {
  int w[kMaxPadBits];
};
template <int LOGN, int LE>
__host__ __device__ constexpr int padx(const Pad& p, int x) {
  constexpr int B = 6 + LE, R = 64 * (1 << LE) + 64;
  int a = R * (x >> B);
  for (int b = 0; b < B; ++b) a += ((x >> b) & 1) * p.w[b];
  return a;
}
// The position bits that the 64 lanes of a wave vary in the layout of pass P.
template <int LOGN, int LE, int P>
__host__ __device__ constexpr int lane_bits() {
  int m = 0;
  for (int l = 0; l < 6; ++l) m |= tid_part<LOGN, LE, P>(1 << l);
  return m;
}
__host__ __device__ constexpr bool pad_search(int B, int R, int inW, int inR, int b, int pre, int usedW, int usedR,
                                              Pad& p) {
  if (b == B) return pre < R;
  const int lo = (1 << b) > pre + 1 ? (1 << b) : pre + 1;
  const bool bw = (inW >> b) & 1, br = (inR >> b) & 1;
  if (!bw && !br) {
    p.w[b] = lo;
    return pad_search(B, R, inW, inR, b + 1, pre + lo, usedW, usedR, p);
  }
  int tried = 0;
  for (int n = 0; n < 6; ++n) {  // free valuations, smallest resulting weight first
    int bv = -1, bwt = 0;
    for (int v = 0; v < 6; ++v) {
      if (((tried >> v) & 1) || (bw && ((usedW >> v) & 1)) || (br && ((usedR >> v) & 1))) continue;
      int m = (lo + (1 << v) - 1) >> v;
      if (!(m & 1)) ++m;
      if (bv < 0 || (m << v) < bwt) {
        bv = v;
        bwt = m << v;
      }
    }
    if (bv < 0) break;
    tried |= 1 << bv;
    p.w[b] = bwt;
    if (pad_search(B, R, inW, inR, b + 1, pre + bwt, bw ? usedW | (1 << bv) : usedW, br ? usedR | (1 << bv) : usedR,
                   p))
      return true;
  }
  return false;
}
template <int LOGN, int LE, int PF, int PT>
__host__ __device__ constexpr Pad exchange_pad() {
  Pad p{};
  constexpr int B = 6 + LE, R = 64 * (1 << LE) + 64;
  static_assert(B <= kMaxPadBits, "LDS placement has room for 12 position bits");
  const bool ok = pad_search(B, R, lane_bits<LOGN, LE, PF>(), lane_bits<LOGN, LE, PT>(), 0, 0, 0, 0, p);
  if (!ok) p.w[0] = -1;  // caught by the static_assert in exchange()
  return p;
}
// Bank-conflict excess of the layout of pass P under placement p: for each register, the
// number of lanes beyond one per bank (64 banks of 4 bytes, one wave).
template <int LOGN, int LE, int P>
__host__ __device__ constexpr int layout_conflicts(const Pad& p) {
  using S = Shape<LOGN, LE>;
  int total = 0;
  for (int i = 0; i < S::E; ++i) {
    int c64[64] = {};
    for (int lane = 0; lane < 64; ++lane) {
      const int addr = padx<LOGN, LE>(p, tid_part<LOGN, LE, P>(lane) | i_part<LOGN, LE, P>(i));
      if (++c64[addr & 63] > 1) ++total;
    }
  }
  return total;
}
// LDS plan of one workgroup.  Exchanges between two wave-local layouts stay inside one
// wave and use the wave's own region of the `local` buffer, with no workgroup barrier.
// When three buffers (and the scatter table) fit in the 160 KB of LDS, cross-wave
// exchanges alternate between g[0] and g[1] over all calls: a buffer is rewritten only
// after the barrier of the following cross-wave exchange has retired every read of its
// previous contents.  Otherwise they all use g[0] behind an extra leading barrier.
// Cross-wave and wave-local exchanges never share a buffer.
template <int LOGN, int LE>
struct LdsPlan {
  static constexpr int PADN = Shape<LOGN, LE>::PADN;
  static constexpr int N = Shape<LOGN, LE>::N;
  static constexpr bool three = (3 * PADN + N) * 4 <= 160 * 1024;
  static constexpr int exchange_words = three ? 3 * PADN : 2 * PADN;
  static constexpr bool table_in_lds = three;
  static constexpr int words = exchange_words + (table_in_lds ? N : 0);
};

// The dynamic LDS of every kernel.  Buffers are addressed as this symbol plus an integer
// offset so that every access compiles to an LDS (ds_*) instruction.
extern __shared__ uint32_t ephdc_lds[];

// Twiddles of pass P for this thread: for stage u of the pass, group e and sub-block v, the
// entry table[2^s + block] of the lower butterfly element, s = s0 + u.  Loaded in one go so
// that the loads can be issued ahead of the exchange that precedes the pass.
template <int LOGN, int LE, int P, class W = uint32_t>
struct Tw {
  using S = Shape<LOGN, LE>;
  static constexpr int k = S::k(P);
  static constexpr int G = S::E >> k;                 // groups per thread
  static constexpr int COUNT = G * ((1 << k) - 1);   // sum over stages of G * 2^u
  static constexpr int off(int u) { return G * ((1 << u) - 1); }
  W w[COUNT];
};

// TL: the table of this transform sits in LDS after the exchange buffers (staged by the
// caller); otherwise it is read from global memory.
template <int LOGN, int LE, int P, class W, bool TL = false>
__device__ __forceinline__ void load_tw(Tw<LOGN, LE, P, W>& t, int tid, const W* __restrict__ table) {
  using S = Shape<LOGN, LE>;
  using TW = Tw<LOGN, LE, P, W>;
  constexpr int k = TW::k;
  constexpr int s0 = S::s0(P);
  const int xt = (P == 0) ? 0 : tid_part<LOGN, LE, P>(tid);  // pass 0: blocks at stages < LE are uniform
  if constexpr (TL && P == S::NPASS - 1 && (TW::G << (k - 1)) >= 4) {
    // Last pass (x = tid*E + i): at stage u the thread's twiddles are the run of
    // R = G * 2^u consecutive words starting at 2^s + tid * R, read as 16-byte vectors, so
    // that a wave's lanes cover consecutive LDS bytes (no bank conflicts for R = 4).
#pragma unroll
    for (int u = 0; u < k; ++u) {
      const int s = s0 + u;
      constexpr int R0 = TW::G;
      const int R = R0 << u;
      const uint32_t w0 = LdsPlan<LOGN, LE>::exchange_words + (1u << s) + (uint32_t)tid * (uint32_t)R;
      if (R >= 4) {
#pragma unroll
        for (int j = 0; j < R; j += 4) {
          const uint4 q = *static_cast<const uint4*>(__builtin_assume_aligned(ephdc_lds + w0 + j, 16));
          t.w[TW::off(u) + j] = q.x;
          t.w[TW::off(u) + j + 1] = q.y;
          t.w[TW::off(u) + j + 2] = q.z;
          t.w[TW::off(u) + j + 3] = q.w;
        }
      } else {
#pragma unroll
        for (int j = 0; j < R; ++j) t.w[TW::off(u) + j] = ephdc_lds[w0 + j];
      }
    }
    return;
  }
#pragma unroll
  for (int u = 0; u < k; ++u) {
    const int s = s0 + u;
    const uint32_t lane = ((1u << s) + (uint32_t)(xt >> (LOGN - s))) * (uint32_t)sizeof(W);
#pragma unroll
    for (int e = 0; e < TW::G; ++e)
#pragma unroll
      for (int v = 0; v < (1 << u); ++v) {
        const int i = (e << k) | (v << (k - u));
        if constexpr (TL) {
          static_assert(sizeof(W) == 4 && LdsPlan<LOGN, LE>::table_in_lds, "LDS twiddles need the table slot");
          t.w[TW::off(u) + (e << u) + v] = ephdc_lds[LdsPlan<LOGN, LE>::exchange_words + lane / 4u +
                                                      (uint32_t)(i_part<LOGN, LE, P>(i) >> (LOGN - s))];
        } else {
          t.w[TW::off(u) + (e << u) + v] =
              ld_at(table, lane + (uint32_t)(i_part<LOGN, LE, P>(i) >> (LOGN - s)) * (uint32_t)sizeof(W));
        }
      }
  }
}

// Forward pass P: Cooley-Tukey butterflies, inputs and outputs in [0, 4m).  Twiddles are
// in Montgomery form (w * 2^32 mod m), so one table word per twiddle and the product
// Y * w mod m in [0, 2m) takes two 64-bit multiply-adds and one multiply.
// IN2M: the pass's inputs are already below 2m (the first stage needs no correction).
template <int LOGN, int LE, int P, bool IN2M = false>
__device__ __forceinline__ void fwd_pass(uint32_t (&v)[1 << LE], const Tw<LOGN, LE, P, uint32_t>& t,
                                         const PrimeConst& pc) {
  using S = Shape<LOGN, LE>;
  using TW = Tw<LOGN, LE, P, uint32_t>;
  constexpr int k = TW::k;
  const uint32_t m = pc.m, m2 = 2 * m;
#pragma unroll
  for (int u = 0; u < k; ++u) {
    const int h = 1 << (k - 1 - u);
#pragma unroll
    for (int i = 0; i < S::E; ++i) {
      if (i & h) continue;
      const int e = i >> k, vb = (i & ((1 << k) - 1)) >> (k - u);
      const uint32_t w = t.w[TW::off(u) + (e << u) + vb];
      const uint32_t X = (IN2M && u == 0) ? v[i] : csub(v[i], m2);
      const uint32_t T = mont_mul(v[i + h], w, m, pc.mneg_inv);  // Y < 4m, w < m
      v[i] = X + T;
      v[i + h] = X - T + m2;
    }
  }
}

// Inverse pass P: Gentleman-Sande butterflies, inputs and outputs in [0, 2m).  With SCALE,
// the last stage (s = 0) also multiplies by N^-1.
// TINY (moduli below 2^17, i.e. t = 65537): no reductions between stages.  Inputs are in
// [0, m); after d stages every value is below 2^d * m, so U + V needs no correction and
// U - V + m*2^d is non-negative; N * m < 2^32 keeps every value in range, and the Shoup
// multiplications (any 32-bit input) bring the twiddled half back to [0, 2m).  With SCALE
// the last stage's multiplications by N^-1 leave every output in [0, 2m).
template <int LOGN, int LE, int P, bool SCALE, bool TINY = false>
__device__ __forceinline__ void inv_pass(uint32_t (&v)[1 << LE], const Tw<LOGN, LE, P, uint32_t>& t,
                                         const PrimeConst& pc) {
  using S = Shape<LOGN, LE>;
  using TW = Tw<LOGN, LE, P, uint32_t>;
  constexpr int k = TW::k;
  constexpr int s0 = S::s0(P);
  static_assert(!TINY || SCALE, "the lazy inverse transform ends with the N^-1 scaling stage");
  const uint32_t m = pc.m, m2 = 2 * m;
#pragma unroll
  for (int u = k - 1; u >= 0; --u) {
    const int h = 1 << (k - 1 - u);
    const int d = LOGN - 1 - (s0 + u);  // stages already done
    const uint32_t K = TINY ? (m << d) : m2;
#pragma unroll
    for (int i = 0; i < S::E; ++i) {
      if (i & h) continue;
      const uint32_t U = v[i], V = v[i + h];
      if (SCALE && s0 + u == 0) {
        v[i] = mont_mul(U + V, pc.ninv_r, m, pc.mneg_inv);
        v[i + h] = mont_mul(U - V + K, pc.ninv_w1_r, m, pc.mneg_inv);
      } else {
        const int e = i >> k, vb = (i & ((1 << k) - 1)) >> (k - u);
        const uint32_t w = t.w[TW::off(u) + (e << u) + vb];
        v[i] = TINY ? U + V : csub(U + V, m2);
        v[i + h] = mont_mul(U - V + K, w, m, pc.mneg_inv);
      }
    }
  }
}

// Workgroup barrier that waits only for this wave's LDS (and scalar-memory) operations:
// vector-memory loads issued before it stay in flight.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Completion of this wave's own LDS operations (orders a wave-private write -> read).
__device__ __forceinline__ void lds_wave_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// Which cross-wave buffer the next cross-wave exchange uses (alternates in the
// three-buffer plan).
struct LdsBufs {
  int sel;
  int base = 0;      // word offset added to every exchange buffer (several transforms per workgroup)
  bool one = false;  // every exchange in one buffer, behind a workgroup barrier (see one_buffer())
};

// Kernels with one transform per workgroup and few registers may run every exchange in a
// single buffer (a barrier before each exchange) where the plan's two buffers would keep a
// CU to one workgroup: at N = 16384 two 1024-thread workgroups then share a CU, so one's
// memory phases overlap the other's transform.  The kernel's dynamic LDS is then PADN words.
template <int LOGN, int LE>
constexpr bool one_buffer() {
  constexpr int bytes = Shape<LOGN, LE>::PADN * 4;
  return !LdsPlan<LOGN, LE>::three && 4 * bytes > 160 * 1024 && 2 * bytes <= 160 * 1024;
}

template <int LOGN, int LE, int PF, int PT>
__device__ __forceinline__ void exchange(uint32_t (&v)[1 << LE], LdsBufs& b, int tid) {
  using S = Shape<LOGN, LE>;
  constexpr int P = S::PADN;
  constexpr bool local = wave_local<LOGN, LE, PF>() && wave_local<LOGN, LE, PT>();
  constexpr Pad pd = exchange_pad<LOGN, LE, PF, PT>();
  static_assert(pd.w[0] > 0, "no conflict-free LDS placement within 64E + 64 words per wave");
  static_assert(layout_conflicts<LOGN, LE, PF>(pd) == 0 && layout_conflicts<LOGN, LE, PT>(pd) == 0,
                "exchange layouts must hit 64 distinct banks per register");
  int off;
  if (b.one) {
    off = 0;
    lds_barrier();  // every wave has finished reading the previous exchange
  } else if constexpr (local) {
    off = LdsPlan<LOGN, LE>::three ? 2 * P : P;
  } else if constexpr (LdsPlan<LOGN, LE>::three) {
    off = b.sel * P;
    b.sel ^= 1;
  } else {
    off = 0;
    lds_barrier();  // every wave has finished reading the previous contents
  }
  off += b.base;
  uint32_t* wb = ephdc_lds + off + padx<LOGN, LE>(pd, tid_part<LOGN, LE, PF>(tid));
#pragma unroll
  for (int i = 0; i < S::E; ++i) wb[padx<LOGN, LE>(pd, i_part<LOGN, LE, PF>(i))] = v[i];
  if constexpr (local) lds_wave_sync();
  else lds_barrier();
  const uint32_t* rb = ephdc_lds + off + padx<LOGN, LE>(pd, tid_part<LOGN, LE, PT>(tid));
#pragma unroll
  for (int i = 0; i < S::E; ++i) v[i] = rb[padx<LOGN, LE>(pd, i_part<LOGN, LE, PT>(i))];
}

template <int LOGN, int LE, int P = 0, bool TL = false, bool IN2M = false>
__device__ __forceinline__ void ntt_forward_from(uint32_t (&v)[1 << LE], Tw<LOGN, LE, P, uint32_t>& tw, int tid,
                                                 const uint32_t* __restrict__ table, const PrimeConst& pc,
                                                 LdsBufs& b) {
  fwd_pass<LOGN, LE, P, IN2M && P == 0>(v, tw, pc);
  if constexpr (P + 1 < Shape<LOGN, LE>::NPASS) {
    Tw<LOGN, LE, P + 1, uint32_t> nt;
    load_tw<LOGN, LE, P + 1, uint32_t, TL>(nt, tid, table);  // in flight across the exchange
    exchange<LOGN, LE, P, P + 1>(v, b, tid);
    ntt_forward_from<LOGN, LE, P + 1, TL>(v, nt, tid, table, pc, b);
  }
}

// Forward transform: coefficient layout (tid + i*T) -> evaluation layout (tid*E + i); the
// table holds Montgomery-form twiddles.
// IN2M: every input is below 2m (otherwise below 4m).
template <int LOGN, int LE, bool TL = false, bool IN2M = false>
__device__ __forceinline__ void ntt_forward(uint32_t (&v)[1 << LE], int tid, const uint32_t* __restrict__ table,
                                            const PrimeConst& pc, LdsBufs& b) {
  Tw<LOGN, LE, 0, uint32_t> t0;
  load_tw<LOGN, LE, 0, uint32_t, TL>(t0, tid, table);
  ntt_forward_from<LOGN, LE, 0, TL, IN2M>(v, t0, tid, table, pc, b);
}

// Copies one transform's twiddle table (N words) into the LDS table slot; the caller
// brackets it with barriers (no wave may still read the previous table, and every wave
// must see the new one).
template <int LOGN, int LE>
__device__ __forceinline__ void stage_twiddles(const uint32_t* __restrict__ table, int tid) {
  using S = Shape<LOGN, LE>;
  static_assert(LdsPlan<LOGN, LE>::table_in_lds, "LDS twiddles need the table slot");
  uint32_t* dst = ephdc_lds + LdsPlan<LOGN, LE>::exchange_words;
#pragma unroll
  for (int i = 0; i < S::E; ++i) dst[i * S::T + tid] = ld_at(table, (uint32_t)(i * S::T + tid) * 4u);
}

template <int LOGN, int LE, bool SCALE, int P, bool TINY = false, bool TL = false>
__device__ __forceinline__ void ntt_inverse_from(uint32_t (&v)[1 << LE], Tw<LOGN, LE, P, uint32_t>& tw, int tid,
                                                 const uint32_t* __restrict__ table, const PrimeConst& pc,
                                                 LdsBufs& b) {
  inv_pass<LOGN, LE, P, SCALE, TINY>(v, tw, pc);
  if constexpr (P > 0) {
    Tw<LOGN, LE, P - 1, uint32_t> nt;
    load_tw<LOGN, LE, P - 1, uint32_t, TL>(nt, tid, table);
    exchange<LOGN, LE, P, P - 1>(v, b, tid);
    ntt_inverse_from<LOGN, LE, SCALE, P - 1, TINY, TL>(v, nt, tid, table, pc, b);
  }
}

// Inverse transform: evaluation layout (tid*E + i) -> coefficient layout (tid + i*T).
// TINY: lazy form for moduli below 2^17 (see inv_pass); inputs must be in [0, m).
template <int LOGN, int LE, bool SCALE, bool TINY = false, bool TL = false>
__device__ __forceinline__ void ntt_inverse(uint32_t (&v)[1 << LE], int tid, const uint32_t* __restrict__ table,
                                            const PrimeConst& pc, LdsBufs& b) {
  constexpr int PL = Shape<LOGN, LE>::NPASS - 1;
  Tw<LOGN, LE, PL, uint32_t> t0;
  load_tw<LOGN, LE, PL, uint32_t, TL>(t0, tid, table);
  ntt_inverse_from<LOGN, LE, SCALE, PL, TINY, TL>(v, t0, tid, table, pc, b);
}


}  // namespace ephdc_dev
