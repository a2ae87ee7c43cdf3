// HDC random-projection encoding on the int8 matrix cores of gfx950.
//
// hv[j][q] = quantise( sum_f (x[q][f] - 128) * base[f][j] ), an exact int8 x int8 -> int32
// contraction (|sum| <= F * 128 * 128 fits easily), computed as the product
// base^T (D x F) * (x - 128)^T (F x Q) with v_mfma_i32_16x16x64_i8, and written
// dimension-major so that the batch-encoding step reads one contiguous row per dimension.
//
// Tiling: a workgroup of 4 waves owns a 64 (dimensions) x 64 (queries) output tile and
// walks F in chunks of 64.  Both operands are staged in LDS with the contraction index
// contiguous (rows padded to 80 bytes); the base tile is transposed on the way in with
// 4x4 byte-block transposes in registers.  Each wave computes a 32 x 32 sub-tile as
// 2 x 2 MFMA tiles of 16 x 16.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "launch.hpp"

namespace ephdc_dev {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int HT = 64;      // tile edge
constexpr int HK = 64;      // contraction chunk
constexpr int PITCH = 80;   // LDS row pitch in bytes

// One 64 x 64 output tile (dimensions j0.., queries q0..).
__device__ __forceinline__ void hdc_tile(const uint8_t* __restrict__ x, const int8_t* __restrict__ base,
                                         int8_t* __restrict__ hv, uint32_t Q, uint32_t F, uint32_t D,
                                         uint32_t stride, uint32_t ncols, uint32_t qbits, uint32_t qshift,
                                         uint32_t j0, uint32_t q0) {
  __shared__ __attribute__((aligned(16))) uint8_t a_lds[HT * PITCH];  // [j][f]
  __shared__ __attribute__((aligned(16))) uint8_t b_lds[HT * PITCH];  // [q][f]
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wj = (wave >> 1) * 32, wq = (wave & 1) * 32;

  v4i acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4i{0, 0, 0, 0};

  const int jq = tid & 15, fq = tid >> 4;   // base tile: 4 dims x 4 features per thread
  const int xrow = tid >> 2, xch = tid & 3;  // feature tile: 16 bytes per thread

  for (uint32_t f0 = 0; f0 < F; f0 += HK) {
    // base[f0+4fq+a][j0+4jq .. +3] -> a_lds[j][f], transposing the 4x4 byte block
    uint32_t d[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const uint32_t f = f0 + 4 * fq + a;
      d[a] = f < F ? *reinterpret_cast<const uint32_t*>(base + (size_t)f * D + j0 + 4 * jq) : 0u;
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const uint32_t col = ((d[0] >> (8 * b)) & 0xFFu) | (((d[1] >> (8 * b)) & 0xFFu) << 8) |
                           (((d[2] >> (8 * b)) & 0xFFu) << 16) | (((d[3] >> (8 * b)) & 0xFFu) << 24);
      *reinterpret_cast<uint32_t*>(a_lds + (4 * jq + b) * PITCH + 4 * fq) = col;
    }
    // (x - 128) as int8 is x ^ 0x80
    {
      const uint32_t q = q0 + xrow, f = f0 + 16 * xch;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (q < Q && f < F) {
        v = *reinterpret_cast<const uint4*>(x + (size_t)q * F + f);
        v.x ^= 0x80808080u; v.y ^= 0x80808080u; v.z ^= 0x80808080u; v.w ^= 0x80808080u;
      }
      *reinterpret_cast<uint4*>(b_lds + xrow * PITCH + 16 * xch) = v;
    }
    __syncthreads();
    v4i av[2], bv[2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
      av[a] = *reinterpret_cast<const v4i*>(a_lds + (wj + 16 * a + (lane & 15)) * PITCH + 16 * (lane >> 4));
#pragma unroll
    for (int b = 0; b < 2; ++b)
      bv[b] = *reinterpret_cast<const v4i*>(b_lds + (wq + 16 * b + (lane & 15)) * PITCH + 16 * (lane >> 4));
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(av[a], bv[b], acc[a][b], 0, 0, 0);
    __syncthreads();
  }

  // lane holds rows 4*(lane/16)+i (dimensions) of column lane%16 (queries) of each 16x16 tile
  const int lo = -(1 << (qbits - 1)), hi = (1 << (qbits - 1)) - 1;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const uint32_t q = q0 + wq + 16 * b + (lane & 15);
      if (q >= ncols) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t j = j0 + wj + 16 * a + 4 * (lane >> 4) + i;
        const int H = acc[a][b][i];
        int h;
        if (q >= Q) h = 0;
        else if (qbits == 1) h = H >= 0 ? 1 : -1;
        else h = min(max(H >> qshift, lo), hi);
        hv[(size_t)j * stride + q] = (int8_t)h;
      }
    }
}

__global__ __launch_bounds__(256) void k_hdc_encode(const uint8_t* __restrict__ x, const int8_t* __restrict__ base,
                                                    int8_t* __restrict__ hv, uint32_t Q, uint32_t F, uint32_t D,
                                                    uint32_t stride, uint32_t ncols, uint32_t qbits, uint32_t qshift) {
  hdc_tile(x, base, hv, Q, F, D, stride, ncols, qbits, qshift, blockIdx.x * HT, blockIdx.y * HT);
}

// Many requests in one launch: workgroup w encodes tile tiles[w] of request reqs[tile.req].
__global__ __launch_bounds__(256) void k_hdc_encode_list(const HdcReq* __restrict__ reqs,
                                                         const HdcTile* __restrict__ tiles) {
  const HdcTile t = tiles[blockIdx.x];
  const HdcReq r = reqs[t.req];
  hdc_tile(r.x, r.base, r.hv, r.Q, r.F, r.D, r.stride, r.ncols, r.qbits, r.qshift, t.j0, t.q0);
}

// Copies of many word ranges in one launch (16-byte moves; every range is a multiple of
// 4 words and 16-byte aligned): workgroups stride over the ranges' 16-byte units.
__global__ __launch_bounds__(256) void k_copy_list(const CopyRange* __restrict__ ranges, uint32_t n) {
  for (uint32_t k = 0; k < n; ++k) {
    const CopyRange c = ranges[k];
    const uint4* src = reinterpret_cast<const uint4*>(c.src);
    uint4* dst = reinterpret_cast<uint4*>(c.dst);
    const size_t units = c.words / 4;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < units; i += (size_t)gridDim.x * blockDim.x)
      dst[i] = src[i];
  }
}

}  // namespace ephdc_dev

namespace ephdc {

hipError_t launch_hdc_encode_list(const HdcReq* reqs, const HdcTile* tiles, uint32_t ntiles, hipStream_t st) {
  if (ntiles == 0) return hipSuccess;
  ephdc_dev::k_hdc_encode_list<<<dim3(ntiles), dim3(256), 0, st>>>(reqs, tiles);
  return hipGetLastError();
}

hipError_t launch_copy_list(const CopyRange* ranges, uint32_t n, size_t total_words, hipStream_t st) {
  if (n == 0 || total_words == 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<size_t>(std::max<size_t>(1, total_words / 4 / 256 / (size_t)n), 1024);
  ephdc_dev::k_copy_list<<<dim3(grid), dim3(256), 0, st>>>(ranges, n);
  return hipGetLastError();
}

hipError_t launch_hdc_encode(const uint8_t* x, const int8_t* base, int8_t* hv, uint32_t Q, uint32_t F, uint32_t D,
                             uint32_t stride, uint32_t qbits, uint32_t qshift, hipStream_t st, uint32_t ncols) {
  if (ncols == 0 || ncols > stride) ncols = stride;
  if (ncols == 0) return hipSuccess;
  dim3 grid(D / ephdc_dev::HT, (ncols + ephdc_dev::HT - 1) / ephdc_dev::HT);
  ephdc_dev::k_hdc_encode<<<grid, dim3(256), 0, st>>>(x, base, hv, Q, F, D, stride, ncols, qbits, qshift);
  return hipGetLastError();
}

}  // namespace ephdc
