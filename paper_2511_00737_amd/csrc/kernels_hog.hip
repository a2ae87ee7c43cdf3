// The detection front end on the device: HOG feature maps of every sliding window of a
// frame (EP-HDC's driving example: windows slide over the frame left to right, row by
// row, and each window's HOG feature map is HDC-encoded as one query).
//
// Integer HOG (Dalal-Triggs layout, exact arithmetic): central-difference gradients with
// replicated borders, floor(sqrt) magnitudes, 9 unsigned orientation bins decided by exact
// integer tests against the boundary directions (round(2^14 cos 20k), round(2^14 sin 20k)),
// 8 x 8-pixel cells, 2 x 2-cell blocks L2-normalised with the clip at 0.2 scaled to byte 255
// (min(255, floor(1275 v / n)), n = floor(sqrt(sum v^2))), and
// cell-aligned windows whose features are their blocks in row order, padded with 128 (the
// HDC encoder's zero point) to a multiple of 16.
//
// The histograms and the normalised blocks are computed once per frame (windows at a
// stride of whole cells share them), then every window's feature row is a gather of
// contiguous 36-byte block runs: the last kernel is a word copy bound by its HBM writes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "params.hpp"

namespace ephdc_dev {

struct HogDirs {
  int c[8], s[8];  // boundary directions k = 1..8
};

// One wave per cell (lane = pixel of the 8 x 8 cell); four cells of one row per workgroup.
// The cell's 9 bin sums are wave reductions (order-free integer sums).
__global__ __launch_bounds__(256) void k_hog_cells(const uint8_t* __restrict__ frame, uint32_t H, uint32_t W,
                                                    uint32_t wc, uint32_t* __restrict__ hist, HogDirs dir) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t cx = blockIdx.x * 4 + (threadIdx.x >> 6), cy = blockIdx.y;
  if (cx >= wc) return;  // the whole wave leaves
  const uint32_t py = cy * 8 + (lane >> 3), px = cx * 8 + (lane & 7u);
  const uint32_t xl = px ? px - 1 : 0, xr = min(px + 1, W - 1);
  const uint32_t yu = py ? py - 1 : 0, yd = min(py + 1, H - 1);
  int gx = (int)frame[(size_t)py * W + xr] - (int)frame[(size_t)py * W + xl];
  int gy = (int)frame[(size_t)yd * W + px] - (int)frame[(size_t)yu * W + px];
  const int n = gx * gx + gy * gy;
  int r = (int)sqrtf((float)n);  // n < 2^17: within one of floor(sqrt(n)); corrected below
  r -= r * r > n;
  r += (r + 1) * (r + 1) <= n;
  if (gy < 0 || (gy == 0 && gx < 0)) {
    gx = -gx;
    gy = -gy;
  }
  int b = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) b += dir.c[k] * gy - dir.s[k] * gx >= 0;
  uint32_t mine = 0;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    uint32_t v = b == k ? (uint32_t)r : 0u;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == (uint32_t)k) mine = v;
  }
  if (lane < 9) hist[((size_t)cy * wc + cx) * 9 + lane] = mine;
}

// One thread per block: its 36 values and their clipped L2 normalisation to bytes, stored
// as 9 words.
__global__ __launch_bounds__(256) void k_hog_blocks(const uint32_t* __restrict__ hist, uint32_t hc, uint32_t wc,
                                                     uint32_t* __restrict__ blocks) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t nbx = wc - 1;
  if (i >= (hc - 1) * nbx) return;
  const uint32_t by = i / nbx, bx = i % nbx;
  uint32_t v[36];
  const uint32_t* c00 = hist + ((size_t)by * wc + bx) * 9;
  const uint32_t* c10 = hist + ((size_t)(by + 1) * wc + bx) * 9;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    v[k] = c00[k];
    v[9 + k] = c00[9 + k];
    v[18 + k] = c10[k];
    v[27 + k] = c10[9 + k];
  }
  uint64_t s2 = 0;  // below 36 * (64 * 361)^2 < 2^35
#pragma unroll
  for (int k = 0; k < 36; ++k) s2 += (uint64_t)v[k] * v[k];
  uint64_t n = (uint64_t)sqrt((double)s2);  // exact input; corrected to floor(sqrt(s2))
  n -= n * n > s2;
  n += (n + 1) * (n + 1) <= s2;
  uint32_t* dst = blocks + (size_t)i * 9;
#pragma unroll
  for (int w = 0; w < 9; ++w) {
    uint32_t word = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      word |= (n ? min(255u, (uint32_t)((1275ull * v[4 * w + j]) / n)) : 0u) << (8 * j);
    dst[w] = word;
  }
}

// One workgroup per window, one thread per output word: the window's row r of nb blocks is
// the contiguous run of nb * 9 words of block row (by + r) starting at block bx; the words
// past nb * nb * 9 are the padding (bytes 128).
__global__ __launch_bounds__(256) void k_hog_windows(const uint32_t* __restrict__ blocks, uint32_t nbx,
                                                      uint32_t nb, uint32_t fw, uint32_t nwx, uint32_t sc,
                                                      uint32_t* __restrict__ x) {
  const uint32_t win = blockIdx.x;
  const uint32_t wy = win / nwx, wx = win % nwx;  // window origin in strides
  const uint32_t feat_words = nb * nb * 9, row_words = nb * 9;
  const uint32_t* src = blocks + ((size_t)(wy * sc) * nbx + wx * sc) * 9;
  uint32_t* dst = x + (size_t)win * fw;
  for (uint32_t w = threadIdx.x; w < fw; w += blockDim.x) {
    uint32_t out = 0x80808080u;
    if (w < feat_words) {
      const uint32_t r = w / row_words, j = w - r * row_words;
      out = src[(size_t)r * nbx * 9 + j];
    }
    dst[w] = out;
  }
}

}  // namespace ephdc_dev

using namespace ephdc;
using namespace ephdc_dev;

namespace {

HogDirs hog_dirs() {
  HogDirs d{};
  const double pi = 3.14159265358979323846;
  for (int k = 1; k <= 8; ++k) {
    d.c[k - 1] = (int)std::lround(16384.0 * std::cos(pi * k / 9.0));
    d.s[k - 1] = (int)std::lround(16384.0 * std::sin(pi * k / 9.0));
  }
  return d;
}

bool hog_shape_ok(uint32_t H, uint32_t W, uint32_t window, uint32_t stride) {
  return window >= 16 && window % 8 == 0 && stride >= 8 && stride % 8 == 0 && H >= window && W >= window &&
         H <= 65536 && W <= 65536;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

uint32_t ephdc_hog_feature_count(uint32_t window) {
  if (window < 16 || window % 8) return 0;
  const uint32_t nb = window / 8 - 1;
  return (nb * nb * 36 + 15) / 16 * 16;
}

uint32_t ephdc_hog_window_count(uint32_t H, uint32_t W, uint32_t window, uint32_t stride) {
  if (!hog_shape_ok(H, W, window, stride)) return 0;
  return ((H - window) / stride + 1) * ((W - window) / stride + 1);
}

size_t ephdc_hog_workspace_bytes(uint32_t H, uint32_t W) {
  if (H < 16 || W < 16) return 0;
  const size_t hc = H / 8, wc = W / 8;
  return align256(hc * wc * 9 * 4) + (hc - 1) * (wc - 1) * 36;
}

ephdc_status ephdc_hog_windows(const uint8_t* d_frame, uint32_t H, uint32_t W, uint32_t window, uint32_t stride,
                               void* d_workspace, size_t ws_bytes, uint8_t* d_x, void* stream) {
  if (!d_frame || !d_workspace || !d_x) return fail(EPHDC_ERR_ARG, "NULL argument");
  if (!hog_shape_ok(H, W, window, stride))
    return fail(EPHDC_ERR_ARG, "window and stride must be multiples of 8 (window >= 16) and fit the frame");
  if (ws_bytes < ephdc_hog_workspace_bytes(H, W)) return fail(EPHDC_ERR_BUFFER, "HOG workspace too small");
  if (((uintptr_t)d_workspace & 255) || ((uintptr_t)d_x & 3))
    return fail(EPHDC_ERR_ARG, "the workspace must be 256-byte and x 4-byte aligned");
  hipStream_t hs = (hipStream_t)stream;
  const uint32_t hc = H / 8, wc = W / 8, nb = window / 8 - 1;
  const uint32_t F = ephdc_hog_feature_count(window), nwx = (W - window) / stride + 1;
  const uint64_t nwin = ephdc_hog_window_count(H, W, window, stride);
  uint32_t* hist = static_cast<uint32_t*>(d_workspace);
  uint32_t* blocks = reinterpret_cast<uint32_t*>(static_cast<char*>(d_workspace) + align256((size_t)hc * wc * 36));
  k_hog_cells<<<dim3((wc + 3) / 4, hc), dim3(256), 0, hs>>>(d_frame, H, W, wc, hist, hog_dirs());
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    const uint32_t nblk = (hc - 1) * (wc - 1);
    k_hog_blocks<<<dim3((nblk + 255) / 256), dim3(256), 0, hs>>>(hist, hc, wc, blocks);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    k_hog_windows<<<dim3((uint32_t)nwin), dim3(256), 0, hs>>>(blocks, wc - 1, nb, F / 4, nwx, stride / 8,
                                                              reinterpret_cast<uint32_t*>(d_x));
    e = hipGetLastError();
  }
  if (e != hipSuccess) return fail(EPHDC_ERR_HIP, std::string("HOG launch: ") + hipGetErrorString(e));
  return EPHDC_OK;
}

}  // extern "C"
