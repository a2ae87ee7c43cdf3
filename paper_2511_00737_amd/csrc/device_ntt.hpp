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
//   Shoup multiplication by a constant w with w' = floor(w*2^32/m): 3 integer multiplies,
//   result in [0, 2m).  Montgomery multiplication of two variables (R = 2^32): 4 multiplies,
//   result in [0, 2m) whenever a*b < m*2^32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ephdc_dev {

struct PrimeConst {
  uint32_t m;         // modulus
  uint32_t mneg_inv;  // -m^-1 mod 2^32 (Montgomery)
  uint32_t r2;        // 2^64 mod m (to enter Montgomery form)
  uint32_t ninv, ninvp;        // N^-1 mod m and Shoup companion
  uint32_t ninv_w1, ninv_w1p;  // N^-1 * (first inverse twiddle) and companion
  uint32_t pad;
};

__device__ __forceinline__ uint32_t mul_shoup(uint32_t a, uint32_t w, uint32_t wp, uint32_t m) {
  const uint32_t qh = __umulhi(a, wp);
  return a * w - qh * m;
}

__device__ __forceinline__ uint32_t csub(uint32_t a, uint32_t m) { return a >= m ? a - m : a; }

__device__ __forceinline__ uint32_t mont_mul(uint32_t a, uint32_t b, uint32_t m, uint32_t mneg_inv) {
  const uint64_t T = (uint64_t)a * b;
  const uint32_t lo = (uint32_t)T, hi = (uint32_t)(T >> 32);
  const uint32_t k = lo * mneg_inv;
  return hi + __umulhi(k, m) + (lo != 0u ? 1u : 0u);
}

// Full reduction of a lazy value in [0, 4m) to [0, m).
__device__ __forceinline__ uint32_t reduce4(uint32_t a, uint32_t m) { return csub(csub(a, 2 * m), m); }

template <int LOGN, int LE>
struct Shape {
  static constexpr int N = 1 << LOGN;
  static constexpr int E = 1 << LE;
  static constexpr int T = N / E;
  static constexpr int NFULL = LOGN / LE;
  static constexpr int REM = LOGN % LE;
  static constexpr int NPASS = NFULL + (REM ? 1 : 0);
  static constexpr int PADN = N + (N >> 5);  // LDS words per exchange buffer
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
__device__ __forceinline__ int tid_part(int tid) {
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

__host__ __device__ constexpr int lds_pad(int x) { return x + (x >> 5); }

// Forward pass P: Cooley-Tukey butterflies with twiddles tw[2^s + block] (= w^brev),
// inputs and outputs in [0, 4m).
template <int LOGN, int LE, int P>
__device__ __forceinline__ void fwd_pass(uint32_t (&v)[1 << LE], int tid, const uint2* __restrict__ tw,
                                         uint32_t m) {
  using S = Shape<LOGN, LE>;
  constexpr int k = S::k(P);
  constexpr int s0 = S::s0(P);
  const uint32_t m2 = 2 * m;
  const int xt = tid_part<LOGN, LE, P>(tid);
#pragma unroll
  for (int u = 0; u < k; ++u) {
    const int s = s0 + u;
    const int h = 1 << (k - 1 - u);
    const uint2* twb = tw + (1 << s) + (xt >> (LOGN - s));
#pragma unroll
    for (int i = 0; i < S::E; ++i) {
      if (i & h) continue;
      const uint2 w = twb[i_part<LOGN, LE, P>(i) >> (LOGN - s)];
      uint32_t X = csub(v[i], m2);
      const uint32_t Tm = mul_shoup(v[i + h], w.x, w.y, m);
      v[i] = X + Tm;
      v[i + h] = X - Tm + m2;
    }
  }
}

// Inverse pass P: Gentleman-Sande butterflies with twiddles itw[2^s + block] (= w^-brev),
// inputs and outputs in [0, 2m).  With SCALE, the last stage (s = 0) also multiplies by N^-1.
template <int LOGN, int LE, int P, bool SCALE>
__device__ __forceinline__ void inv_pass(uint32_t (&v)[1 << LE], int tid, const uint2* __restrict__ itw,
                                         const PrimeConst& pc) {
  using S = Shape<LOGN, LE>;
  constexpr int k = S::k(P);
  constexpr int s0 = S::s0(P);
  const uint32_t m = pc.m, m2 = 2 * m;
  const int xt = tid_part<LOGN, LE, P>(tid);
#pragma unroll
  for (int u = k - 1; u >= 0; --u) {
    const int s = s0 + u;
    const int h = 1 << (k - 1 - u);
    const uint2* twb = itw + (1 << s) + (xt >> (LOGN - s));
#pragma unroll
    for (int i = 0; i < S::E; ++i) {
      if (i & h) continue;
      const uint32_t U = v[i], V = v[i + h];
      if (SCALE && s == 0) {
        v[i] = mul_shoup(U + V, pc.ninv, pc.ninvp, m);
        v[i + h] = mul_shoup(U - V + m2, pc.ninv_w1, pc.ninv_w1p, m);
      } else {
        const uint2 w = twb[i_part<LOGN, LE, P>(i) >> (LOGN - s)];
        v[i] = csub(U + V, m2);
        v[i + h] = mul_shoup(U - V + m2, w.x, w.y, m);
      }
    }
  }
}

// Moves values from the register layout of pass PF to that of pass PT through LDS.
template <int LOGN, int LE, int PF, int PT>
__device__ __forceinline__ void exchange(uint32_t (&v)[1 << LE], uint32_t* __restrict__ buf, int tid) {
  using S = Shape<LOGN, LE>;
  uint32_t* wb = buf + lds_pad(tid_part<LOGN, LE, PF>(tid));
#pragma unroll
  for (int i = 0; i < S::E; ++i) wb[lds_pad(i_part<LOGN, LE, PF>(i))] = v[i];
  __syncthreads();
  const uint32_t* rb = buf + lds_pad(tid_part<LOGN, LE, PT>(tid));
#pragma unroll
  for (int i = 0; i < S::E; ++i) v[i] = rb[lds_pad(i_part<LOGN, LE, PT>(i))];
}

// Exchange buffers alternate on every exchange, across calls too, so one barrier per
// exchange suffices: a buffer is rewritten only after a later barrier has retired all
// reads of its previous contents.
struct LdsPair {
  uint32_t* b0;
  uint32_t* b1;
  int sel;
  __device__ __forceinline__ uint32_t* next() {
    uint32_t* p = sel ? b1 : b0;
    sel ^= 1;
    return p;
  }
};

// Makes a pointer opaque to the optimiser so that table loads stay inside the calling loop
// instead of being hoisted (and held in registers) across iterations.
template <class T>
__device__ __forceinline__ const T* opaque(const T* p) {
  asm volatile("" : "+s"(p));
  return p;
}

template <int LOGN, int LE, int P = 0>
__device__ __forceinline__ void ntt_forward(uint32_t (&v)[1 << LE], int tid, const uint2* __restrict__ tw,
                                            uint32_t m, LdsPair& lds) {
  if constexpr (P == 0) tw = opaque(tw);
  fwd_pass<LOGN, LE, P>(v, tid, tw, m);
  if constexpr (P + 1 < Shape<LOGN, LE>::NPASS) {
    exchange<LOGN, LE, P, P + 1>(v, lds.next(), tid);
    ntt_forward<LOGN, LE, P + 1>(v, tid, tw, m, lds);
  }
}

template <int LOGN, int LE, bool SCALE, int P = Shape<LOGN, LE>::NPASS - 1>
__device__ __forceinline__ void ntt_inverse(uint32_t (&v)[1 << LE], int tid, const uint2* __restrict__ itw,
                                            const PrimeConst& pc, LdsPair& lds) {
  if constexpr (P == Shape<LOGN, LE>::NPASS - 1) itw = opaque(itw);
  inv_pass<LOGN, LE, P, SCALE>(v, tid, itw, pc);
  if constexpr (P > 0) {
    exchange<LOGN, LE, P, P - 1>(v, lds.next(), tid);
    ntt_inverse<LOGN, LE, SCALE, P - 1>(v, tid, itw, pc, lds);
  }
}

}  // namespace ephdc_dev
