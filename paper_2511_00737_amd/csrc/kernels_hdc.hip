// HDC random-projection encoding on the int8 matrix cores of gfx950.
//
// hv[j][q] = quantise( sum_f (x[q][f] - 128) * base[f][j] ), an exact int8 x int8 -> int32
// contraction (|sum| <= F * 128 * 128 fits easily), computed as the product
// base^T (D x F) * (x - 128)^T (F x Q) with v_mfma_i32_16x16x64_i8, and written
// dimension-major so that the batch-encoding step reads one contiguous row per dimension.
//
// Tiling: a workgroup of 4 waves owns a 128 (dimensions) x 128 (queries) output tile and
// walks F in chunks of 64.  Both operands are staged in LDS with the contraction index
// contiguous, in 64-byte rows whose four 16-byte runs are XOR-swizzled by bits 2-3 of the
// row, so that the matrix-operand reads (16 rows, one run each) and the stores below touch
// 64 distinct banks.  The base tile is transposed on the way in with 4 x 4 byte-block
// transposes (v_perm) and placed at row 32*b + m for dimension 4*m + b, which spreads a
// wave's transposed stores over all banks too.  Global loads go through buffer resources
// whose range check returns zero past the end: features past F read zero base rows, so no
// load needs a branch, and whatever a row past D or Q holds only reaches outputs that are
// discarded or written as zero (tiles lying wholly past Q skip the contraction).  The next chunk's loads are issued before the current
// chunk's matrix work and consumed only at the next stage.  Each wave computes a 64 x 64
// quarter as 4 x 4 MFMA tiles of 16 x 16.  The LDS holds two chunks: chunk k is read from one
// buffer while chunk k + 1 is written to the other after the chunk's matrix instructions are
// issued, so each chunk needs one workgroup barrier.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "launch.hpp"

namespace ephdc_dev {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int HT = 128;     // tile edge (dimensions and queries)
constexpr int HK = 64;      // contraction chunk (bytes per LDS row)
constexpr int NT = 256;     // threads: 4 waves, each a 64 x 64 quarter of the tile
constexpr int SUB = HT / 2 / 16;  // 16 x 16 MFMA tiles per wave edge
constexpr uint32_t RSRC_WORD3 = 0x00020000u;  // raw (untyped) buffer access on gfx9-family parts

// byte offset of 16-byte run c of LDS row r
__device__ __forceinline__ int lds_at(int r, int c) { return r * HK + 16 * (c ^ ((r >> 2) & 3)); }

// Global operands of one contraction chunk, held in registers so that the next chunk's
// loads are in flight while the current chunk runs on the matrix cores.  QT: queries per
// tile (128 or 256).
template <int QT>
struct HdcStage {
  uint32_t d[2][4];     // base: two 4 x 4 byte blocks (4 features x 4 dimensions)
  uint4 xv[QT / 64];    // features: 16-byte runs (raw bytes; the offset is applied at the store)
};

struct HdcSrc {
  __amdgpu_buffer_rsrc_t x, base;  // x from row q0 on; base whole (F * D bytes)
  uint32_t F, D, j0;
};

template <int QT>
__device__ __forceinline__ void hdc_load(HdcStage<QT>& st, const HdcSrc& src, uint32_t f0, int tid) {
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int blk = tid + NT * k;
    // 32 dimension quads x 16 feature quads; 16 dimension quads per feature row across lanes
    const int jq = (blk & 15) + 16 * k, fq = (blk >> 4) & 15;
    const uint32_t j = src.j0 + 4 * jq;
#pragma unroll
    for (int a = 0; a < 4; ++a)
      st.d[k][a] = __builtin_amdgcn_raw_buffer_load_b32(src.base, (f0 + 4 * fq + a) * src.D + j, 0, 0);
  }
#pragma unroll
  for (int k = 0; k < QT / 64; ++k) {
    const int blk = tid + NT * k, row = blk >> 2, ch = blk & 3;  // QT queries x 4 runs of 16 features
    const v4i v = __builtin_amdgcn_raw_buffer_load_b128(src.x, row * src.F + f0 + 16 * ch, 0, 0);
    st.xv[k] = make_uint4(v[0], v[1], v[2], v[3]);
  }
}

// base rows [f][j] -> a_lds[32 * (j % 4) + j / 4][f] (4 x 4 byte-block transposes);
// features -> b_lds[q][f] as x - 128 (x ^ 0x80 on each byte)
template <int QT>
__device__ __forceinline__ void hdc_store(const HdcStage<QT>& st, uint8_t* a_lds, uint8_t* b_lds, int tid) {
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int blk = tid + NT * k;
    const int jq = (blk & 15) + 16 * k, fq = (blk >> 4) & 15;
    const uint32_t* d = st.d[k];
    const uint32_t lo01 = __builtin_amdgcn_perm(d[1], d[0], 0x05010400u);
    const uint32_t hi01 = __builtin_amdgcn_perm(d[1], d[0], 0x07030602u);
    const uint32_t lo23 = __builtin_amdgcn_perm(d[3], d[2], 0x05010400u);
    const uint32_t hi23 = __builtin_amdgcn_perm(d[3], d[2], 0x07030602u);
    const uint32_t col[4] = {__builtin_amdgcn_perm(lo23, lo01, 0x05040100u),
                             __builtin_amdgcn_perm(lo23, lo01, 0x07060302u),
                             __builtin_amdgcn_perm(hi23, hi01, 0x05040100u),
                             __builtin_amdgcn_perm(hi23, hi01, 0x07060302u)};
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) {
      const int r = 32 * bb + jq;
      *reinterpret_cast<uint32_t*>(a_lds + lds_at(r, fq >> 2) + 4 * (fq & 3)) = col[bb];
    }
  }
#pragma unroll
  for (int k = 0; k < QT / 64; ++k) {
    const int blk = tid + NT * k, row = blk >> 2, ch = blk & 3;
    uint4 v = st.xv[k];
    v.x ^= 0x80808080u; v.y ^= 0x80808080u; v.z ^= 0x80808080u; v.w ^= 0x80808080u;
    *reinterpret_cast<uint4*>(b_lds + lds_at(row, ch)) = v;
  }
}

// One 128 x QT output tile (dimensions j0.., queries q0..); each wave computes a 64 x QT/2
// quarter as 4 x QT/32 MFMA tiles.
template <int QT>
__device__ __forceinline__ void hdc_tile(const uint8_t* __restrict__ x, const int8_t* __restrict__ base,
                                         int8_t* __restrict__ hv, uint32_t Q, uint32_t F, uint32_t D,
                                         uint32_t stride, uint32_t ncols, uint32_t qbits, uint32_t qshift,
                                         uint32_t j0, uint32_t q0) {
  constexpr int SUBQ = QT / 2 / 16;
  // two LDS buffers per operand: chunk k is read from buffer k % 2 while chunk k + 1 is stored
  // into the other, so one barrier per chunk suffices
  __shared__ __attribute__((aligned(16))) uint8_t a_lds[2][HT * HK];  // [32 * (j % 4) + j / 4][f]
  __shared__ __attribute__((aligned(16))) uint8_t b_lds[2][QT * HK];  // [q][f]
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wj = (wave >> 1) * (HT / 2), wq = (wave & 1) * (QT / 2);

  HdcSrc src;
  // the resources must live in scalar registers: the row base and its length are uniform
  const uint64_t xa = reinterpret_cast<uint64_t>(x) + (uint64_t)q0 * F;
  const uint32_t xlo = __builtin_amdgcn_readfirstlane((uint32_t)xa), xhi = __builtin_amdgcn_readfirstlane((uint32_t)(xa >> 32));
  const uint32_t xbytes = __builtin_amdgcn_readfirstlane(q0 < Q ? (Q - q0) * F : 0u);
  src.x = __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(((uint64_t)xhi << 32) | xlo), 0, (int)xbytes, RSRC_WORD3);
  src.base = __builtin_amdgcn_make_buffer_rsrc(const_cast<int8_t*>(base), 0, (int)(F * D), RSRC_WORD3);
  src.F = F; src.D = D; src.j0 = j0;

  v4i acc[SUB][SUBQ];
#pragma unroll
  for (int a = 0; a < SUB; ++a)
#pragma unroll
    for (int b = 0; b < SUBQ; ++b) acc[a][b] = v4i{0, 0, 0, 0};

  // a tile whose queries all lie past Q (padding columns of the last query group) holds
  // zeros only: it skips the contraction and goes straight to the stores
  const uint32_t F_run = q0 < Q ? F : 0u;
  HdcStage<QT> st;
  if (F_run) {
    hdc_load(st, src, 0, tid);
    hdc_store(st, a_lds[0], b_lds[0], tid);
    if (HK < F) hdc_load(st, src, HK, tid);
  }
  int cur = 0;
  for (uint32_t f0 = 0; f0 < F_run; f0 += HK) {
    // buffer `cur` holds chunk f0 (stored by every wave), and every wave is done reading the
    // other buffer (chunk f0 - HK)
    __syncthreads();
    v4i av[SUB], bv[SUBQ];
#pragma unroll
    for (int a = 0; a < SUB; ++a)
      av[a] = *reinterpret_cast<const v4i*>(a_lds[cur] + lds_at(wj + 16 * a + (lane & 15), lane >> 4));
#pragma unroll
    for (int b = 0; b < SUBQ; ++b)
      bv[b] = *reinterpret_cast<const v4i*>(b_lds[cur] + lds_at(wq + 16 * b + (lane & 15), lane >> 4));
#pragma unroll
    for (int a = 0; a < SUB; ++a)
#pragma unroll
      for (int b = 0; b < SUBQ; ++b) acc[a][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(bv[b], av[a], acc[a][b], 0, 0, 0);
    // while the matrix cores work: chunk f0 + HK (loaded an iteration ago) into the other
    // buffer, and the loads of chunk f0 + 2 HK
    if (f0 + HK < F) {
      hdc_store(st, a_lds[cur ^ 1], b_lds[cur ^ 1], tid);
      if (f0 + 2 * HK < F) hdc_load(st, src, f0 + 2 * HK, tid);
    }
    cur ^= 1;
  }

  // The product is (x - 128) * base^T, so a lane holds queries 4*(lane/16) + i, i = 0..3, of
  // one base row (LDS row lane%16, i.e. dimension 4*(row % 32) + row / 32) in each 16 x 16
  // tile: four consecutive bytes of one hv row, stored as one word where aligned.
  const int lo = -(1 << (qbits - 1)), hi = (1 << (qbits - 1)) - 1;
#pragma unroll
  for (int a = 0; a < SUB; ++a) {
    const int r = wj + 16 * a + (lane & 15);
    const uint32_t j = j0 + 4 * (r & 31) + (r >> 5);
#pragma unroll
    for (int b = 0; b < SUBQ; ++b) {
      const uint32_t q = q0 + wq + 16 * b + 4 * (lane >> 4);
      if (j >= D || q >= ncols) continue;
      uint32_t w = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int H = acc[a][b][i];
        int h = qbits == 1 ? ((H >> 31) | 1) : min(max(H >> qshift, lo), hi);
        if (q + i >= Q) h = 0;
        w |= (uint32_t)(h & 0xFF) << (8 * i);
      }
      int8_t* dst = hv + (size_t)j * stride + q;
      if (q + 4 <= ncols && (reinterpret_cast<uintptr_t>(dst) & 3) == 0) {
        *reinterpret_cast<uint32_t*>(dst) = w;
      } else {
        for (int i = 0; i < 4 && q + i < ncols; ++i) dst[i] = (int8_t)(w >> (8 * i));
      }
    }
  }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_hdc_encode(const uint8_t* __restrict__ x, const int8_t* __restrict__ base,
                                                    int8_t* __restrict__ hv, uint32_t Q, uint32_t F, uint32_t D,
                                                    uint32_t stride, uint32_t ncols, uint32_t qbits, uint32_t qshift) {
  hdc_tile<2 * HT>(x, base, hv, Q, F, D, stride, ncols, qbits, qshift, blockIdx.x * HT, blockIdx.y * 2 * HT);
}

// Many requests in one launch: workgroup w encodes tile tiles[w] of request reqs[tile.req].
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_hdc_encode_list(const HdcReq* __restrict__ reqs,
                                                         const HdcTile* __restrict__ tiles) {
  const HdcTile t = tiles[blockIdx.x];
  const HdcReq r = reqs[t.req];
  hdc_tile<HT>(r.x, r.base, r.hv, r.Q, r.F, r.D, r.stride, r.ncols, r.qbits, r.qshift, t.j0, t.q0);
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
  dim3 grid((D + ephdc_dev::HT - 1) / ephdc_dev::HT, (ncols + 2 * ephdc_dev::HT - 1) / (2 * ephdc_dev::HT));
  ephdc_dev::k_hdc_encode<<<grid, dim3(256), 0, st>>>(x, base, hv, Q, F, D, stride, ncols, qbits, qshift);
  return hipGetLastError();
}

}  // namespace ephdc
