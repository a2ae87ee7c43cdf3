// Rotate-and-sum for folded packings (r > 1): Galois automorphisms in the evaluation domain
// and hybrid key switching (fast base conversion up to the extended basis, inner product
// with the switching keys, fast base conversion down and division by P).
//
// One rotation step on the accumulators acc[G][2][L][N] (evaluation domain, q limbs):
//   R        = sigma_g(acc)                      permutation of evaluation points
//   D        = iNTT(R[.][1])                     coefficient domain, for the digit split
//   Y[j][m]  = NTT_m(ModUp_j(D)), m not in I_j   fast base conversion, then transform
//   KS[c][m] = sum_j ksk[j][c][m] * (m in I_j ? R[1][m] : Y[j][m])
//   XP       = iNTT(KS[.][special limbs])
//   acc[c]  += (c == 0 ? R[0] : 0) + (KS[c][q limbs] - NTT(conv_P(XP[c]))) * P^-1
// All residues are exact, so the result is bit-identical to the coefficient-domain
// definition.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_ntt.hpp"
#include "kernel_common.hpp"
#include "launch.hpp"

namespace ephdc_dev {

// out[p][x] = in[p][perm[x]] for every polynomial p of the batch: grid (N / 256, npolys).
__global__ void k_automorph(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                            const uint32_t* __restrict__ perm, uint32_t N) {
  const size_t base = (size_t)blockIdx.y * N;
  const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  out[base + x] = in[base + perm[x]];
}

// Y[g][j][m] = NTT_m( sum_{i in I_j} [D[g][i] * (Q_j/q_i)^-1]_{q_i} * (Q_j/q_i mod m) ) for
// every modulus m outside digit j (blocks of moduli inside the digit exit at once).
template <int LOGN, int LE>
__global__ __launch_bounds__((1 << LOGN) >> LE) void k_modup_ntt(const uint32_t* __restrict__ D,
                                                                  uint32_t* __restrict__ Y, KsConst k,
                                                                  const uint32_t* __restrict__ fwd_tw,
                                                                  const PrimeConst* __restrict__ pcs) {
  using S = Shape<LOGN, LE>;
  const uint32_t m = blockIdx.x % k.nmod;
  const uint32_t j = (blockIdx.x / k.nmod) % k.dnum;
  const uint32_t g = blockIdx.x / (k.nmod * k.dnum);
  const uint32_t i0 = j * k.ds, i1 = min(k.L, i0 + k.ds);
  if (m >= i0 && m < i1) return;  // the digit's own limbs are taken from R directly
  LdsBufs b{0, 0, one_buffer<LOGN, LE>()};
  const int tid = threadIdx.x;
  const PrimeConst pm = pcs[m];
  const uint32_t m2 = 2 * pm.m;
  uint32_t v[S::E];
#pragma unroll
  for (int e = 0; e < S::E; ++e) v[e] = 0;
  for (uint32_t i = i0; i < i1; ++i) {
    const uint32_t qi = pcs[i].m;
    const uint2 inv = k.up_inv[i];
    const uint2 mul = k.up_mul[((size_t)j * k.ds + (i - i0)) * k.nmod + m];
    const uint32_t* src = D + ((size_t)g * k.L + i) * S::N + tid;
#pragma unroll
    for (int e = 0; e < S::E; ++e) {
      const uint32_t t = csub(mul_shoup(src[e * S::T], inv.x, inv.y, qi), qi);
      v[e] = csub(v[e] + mul_shoup(t, mul.x, mul.y, pm.m), m2);
    }
  }
#pragma unroll
  for (int e = 0; e < S::E; ++e) v[e] = csub(v[e], pm.m);
  ntt_forward<LOGN, LE>(v, tid, fwd_tw + (size_t)m * S::N, pm, b);
  uint32_t* dst = Y + (((size_t)g * k.dnum + j) * k.nmod + m) * S::N + (size_t)tid * S::E;
#pragma unroll
  for (int e = 0; e < S::E; ++e) dst[e] = reduce4(v[e], pm.m);
}

// KS[g][c][m] = sum_j ksk[j][c][m] (Montgomery form) * (m in I_j ? R[g][1][m] : Y[g][j][m]).
// Grid (N / 1024, G * nmod) of 256 threads; a thread takes four consecutive positions and
// both components, so each digit value is read once.
__global__ void k_ks_inner(const uint32_t* __restrict__ R, const uint32_t* __restrict__ Y,
                           const uint32_t* __restrict__ ksk, uint32_t* __restrict__ KS, KsConst k,
                           const PrimeConst* __restrict__ pcs, uint32_t N) {
  const uint32_t m = blockIdx.y % k.nmod, g = blockIdx.y / k.nmod;
  const uint32_t xo = (blockIdx.x * blockDim.x + threadIdx.x) * 16u;  // byte offset of 4 positions
  const PrimeConst pc = pcs[m];
  uint32_t a0[4] = {0, 0, 0, 0}, a1[4] = {0, 0, 0, 0};
  for (uint32_t j = 0; j < k.dnum; ++j) {
    const uint32_t i0 = j * k.ds, i1 = min(k.L, i0 + k.ds);
    const uint32_t* src = (m >= i0 && m < i1) ? R + (((size_t)g * 2 + 1) * k.L + m) * N
                                              : Y + (((size_t)g * k.dnum + j) * k.nmod + m) * N;
    const uint4 sv = ld_at(reinterpret_cast<const uint4*>(src), xo);
    const uint4 k0 = ld_at(reinterpret_cast<const uint4*>(ksk + (((size_t)j * 2 + 0) * k.nmod + m) * N), xo);
    const uint4 k1 = ld_at(reinterpret_cast<const uint4*>(ksk + (((size_t)j * 2 + 1) * k.nmod + m) * N), xo);
    const uint32_t sx[4] = {sv.x, sv.y, sv.z, sv.w}, kx0[4] = {k0.x, k0.y, k0.z, k0.w},
                   kx1[4] = {k1.x, k1.y, k1.z, k1.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      a0[e] = csub(a0[e] + mont_mul(kx0[e], sx[e], pc.m, pc.mneg_inv), 2 * pc.m);
      a1[e] = csub(a1[e] + mont_mul(kx1[e], sx[e], pc.m, pc.mneg_inv), 2 * pc.m);
    }
  }
  uint32_t* out0 = KS + (((size_t)g * 2 + 0) * k.nmod + m) * N;
  uint32_t* out1 = KS + (((size_t)g * 2 + 1) * k.nmod + m) * N;
  st_at(reinterpret_cast<uint4*>(out0), xo,
        make_uint4(csub(a0[0], pc.m), csub(a0[1], pc.m), csub(a0[2], pc.m), csub(a0[3], pc.m)));
  st_at(reinterpret_cast<uint4*>(out1), xo,
        make_uint4(csub(a1[0], pc.m), csub(a1[1], pc.m), csub(a1[2], pc.m), csub(a1[3], pc.m)));
}

template <int LOGN, int LE>
__global__ __launch_bounds__((1 << LOGN) >> LE) void k_moddown_ntt(const uint32_t* __restrict__ XP,
                                                                    const uint32_t* __restrict__ KS,
                                                                    const uint32_t* __restrict__ R,
                                                                    uint32_t* __restrict__ acc, KsConst k,
                                                                    const uint32_t* __restrict__ fwd_tw,
                                                                    const PrimeConst* __restrict__ pcs) {
  using S = Shape<LOGN, LE>;
  const uint32_t i = blockIdx.x % k.L;
  const uint32_t c = (blockIdx.x / k.L) % 2;
  const uint32_t g = blockIdx.x / (2 * k.L);
  LdsBufs b{0};
  const int tid = threadIdx.x;
  const PrimeConst pq = pcs[i];
  const uint32_t q2 = 2 * pq.m;
  // the operands of the last step, in the transform's output layout (positions tid*E + e):
  // requested together at the start, so that each lane's run is read in one burst and the
  // loads overlap the conversion and the transform
  const uint32_t off = (uint32_t)tid * S::E * 4u;
  const uint32_t* ks = KS + (((size_t)g * 2 + c) * k.nmod + i) * S::N;
  const uint32_t* r0 = R + (((size_t)g * 2 + 0) * k.L + i) * S::N;
  uint32_t* a = acc + (((size_t)g * 2 + c) * k.L + i) * S::N;
  uint32_t kv[S::E], av[S::E], rv[S::E];
#pragma unroll
  for (int e = 0; e < S::E; e += 4) {
    const uint4 x = ld_at(reinterpret_cast<const uint4*>(ks), off + 4u * e);
    const uint4 y = ld_at(reinterpret_cast<const uint4*>(a), off + 4u * e);
    kv[e] = x.x; kv[e + 1] = x.y; kv[e + 2] = x.z; kv[e + 3] = x.w;
    av[e] = y.x; av[e + 1] = y.y; av[e + 2] = y.z; av[e + 3] = y.w;
    uint4 z = make_uint4(0, 0, 0, 0);
    if (c == 0) z = ld_at(reinterpret_cast<const uint4*>(r0), off + 4u * e);
    rv[e] = z.x; rv[e + 1] = z.y; rv[e + 2] = z.z; rv[e + 3] = z.w;
  }
  uint32_t v[S::E];
#pragma unroll
  for (int e = 0; e < S::E; ++e) v[e] = 0;
  for (uint32_t kk = 0; kk < k.alpha; ++kk) {
    const uint32_t pk = pcs[k.L + kk].m;
    const uint2 inv = k.down_inv[kk];
    const uint2 mul = k.down_mul[(size_t)kk * k.L + i];
    const uint32_t* src = XP + (((size_t)g * 2 + c) * k.alpha + kk) * S::N + tid;
#pragma unroll
    for (int e = 0; e < S::E; ++e) {
      const uint32_t t = csub(mul_shoup(src[e * S::T], inv.x, inv.y, pk), pk);
      v[e] = csub(v[e] + mul_shoup(t, mul.x, mul.y, pq.m), q2);
    }
  }
#pragma unroll
  for (int e = 0; e < S::E; ++e) v[e] = csub(v[e], pq.m);
  ntt_forward<LOGN, LE>(v, tid, fwd_tw + (size_t)i * S::N, pq, b);
  const uint2 pinv = k.pinv[i];
#pragma unroll
  for (int e = 0; e < S::E; ++e) {
    const uint32_t conv = reduce4(v[e], pq.m);
    const uint32_t d = csub(mul_shoup(kv[e] + pq.m - conv, pinv.x, pinv.y, pq.m), pq.m);
    v[e] = csub(csub(av[e] + d, pq.m) + rv[e], pq.m);  // rv = 0 for c = 1
  }
#pragma unroll
  for (int e = 0; e < S::E; e += 4) st_at(reinterpret_cast<uint4*>(a), off + 4u * e, make_uint4(v[e], v[e + 1], v[e + 2], v[e + 3]));
}

}  // namespace ephdc_dev

namespace ephdc {

hipError_t prepare_ks_kernels() {
  hipError_t e = hipSuccess;
  auto shape = [&](auto lnc, auto lec) {
    constexpr int LN = decltype(lnc)::value, LEv = decltype(lec)::value;
    const int bytes = (int)lds_bytes<LN, LEv>();
    if (e == hipSuccess) e = hipFuncSetAttribute((const void*)k_modup_ntt<LN, LEv>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess) e = hipFuncSetAttribute((const void*)k_moddown_ntt<LN, LEv>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    return e;
  };
  for (int logn = 11; logn <= 14; ++logn) dispatch(logn, shape);
  return e;
}

hipError_t launch_rotate_step(int logn, const RotateArgs& r, uint32_t step, hipStream_t st) {
  const KsConst& k = r.k;
  const uint32_t N = 1u << logn;
  const size_t acc_polys = (size_t)k.G * 2 * k.L;
  if (N % 1024 != 0) return hipErrorInvalidValue;  // the grids below tile N by 256 and 1024
  // R = sigma_g(acc); the grid's second dimension counts polynomials, at most kMaxGridY a launch
  constexpr size_t kMaxGridY = 65535;
  hipError_t e = hipSuccess;
  for (size_t p0 = 0; p0 < acc_polys && e == hipSuccess; p0 += kMaxGridY) {
    const unsigned np = (unsigned)std::min(kMaxGridY, acc_polys - p0);
    k_automorph<<<dim3(N / 256, np), 256, 0, st>>>(r.acc + p0 * N, r.R + p0 * N, r.perm + (size_t)step * N, N);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return e;
  // D = iNTT(R[g][1][l]) for every group and limb
  BatchMap dmap;
  dmap.in_per = k.L;
  dmap.in_stride = (size_t)2 * k.L * N;
  e = launch_inv_batch(logn, r.R + (size_t)k.L * N, r.D, (size_t)k.G * k.L, r.inv_tw, r.pcs, k.L, 0, st, dmap);
  if (e != hipSuccess) return e;
  // Y = NTT(ModUp(D)) per digit and target modulus
  e = dispatch(logn, [&](auto lnc, auto lec) {
    constexpr int LN = decltype(lnc)::value, LEv = decltype(lec)::value;
    k_modup_ntt<LN, LEv><<<dim3(k.G * k.dnum * k.nmod), dim3(Shape<LN, LEv>::T), lds_bytes_one_transform<LN, LEv>(), st>>>(
        r.D, r.Y, k, r.fwd_tw, r.pcs);
    return hipGetLastError();
  });
  if (e != hipSuccess) return e;
  // KS = inner product with the switching keys of this step
  const uint32_t* ksk = r.ksk + (size_t)step * k.dnum * 2 * k.nmod * N;
  // groups in launches of at most kMaxGridY (group, modulus) pairs
  const uint32_t gstep = std::max<uint32_t>(1, (uint32_t)(kMaxGridY / k.nmod));
  for (uint32_t g0 = 0; g0 < k.G && e == hipSuccess; g0 += gstep) {
    const uint32_t ng = std::min(gstep, k.G - g0);
    k_ks_inner<<<dim3(N / 1024, ng * k.nmod), 256, 0, st>>>(
        r.R + (size_t)g0 * 2 * k.L * N, r.Y + (size_t)g0 * k.dnum * k.nmod * N, ksk, r.KS + (size_t)g0 * 2 * k.nmod * N,
        k, r.pcs, N);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return e;
  // XP = iNTT of the special limbs of KS
  BatchMap xmap;
  xmap.in_per = k.alpha;
  xmap.in_stride = (size_t)k.nmod * N;
  e = launch_inv_batch(logn, r.KS + (size_t)k.L * N, r.XP, (size_t)k.G * 2 * k.alpha, r.inv_tw, r.pcs, k.alpha,
                       k.L, st, xmap);
  if (e != hipSuccess) return e;
  // acc += rotated c0 + ModDown(KS)
  return dispatch(logn, [&](auto lnc, auto lec) {
    constexpr int LN = decltype(lnc)::value, LEv = decltype(lec)::value;
    k_moddown_ntt<LN, LEv><<<dim3(k.G * 2 * k.L), dim3(Shape<LN, LEv>::T), lds_bytes<LN, LEv>(), st>>>(
        r.XP, r.KS, r.R, r.acc, k, r.fwd_tw, r.pcs);
    return hipGetLastError();
  });
}

}  // namespace ephdc
