// Batched complex FFTs of whole grids in device memory.
//
// Grids that fit one LDS tile (H * W <= 16384, 2-D) are transformed by one
// workgroup each (row passes then column passes in LDS, one HBM read and one
// HBM write per element).  Larger grids (256 x 256, 256 x 128, 3-D volumes)
// take one pass per axis: each workgroup stages a 4096-element slab of lines
// in LDS, transforms it and writes it back.
#include "common.hpp"
#include "internal.hpp"

namespace dcsc {

constexpr int kAxisTile = 4096;
constexpr int kAxisThreads = 256;

// data: a batch of arrays [outer][L][inner]; transform along the middle axis.
// One block covers `bo` consecutive outer indices x L x `bi` consecutive inner
// indices (bo * L * bi == kAxisTile).
template <int L, int DIR>
__global__ __launch_bounds__(kAxisThreads) void k_fft_axis(float2* __restrict__ data, int64_t outer,
                                                          int64_t inner, int lbi, int lbo) {
  constexpr int T = kAxisTile, NT = kAxisThreads, LP = L + 1;
  __shared__ float2 tile[(T / L) * LP];
  __shared__ float2 tw[256];
  load_twiddles(tw);
  const int bi = 1 << lbi;
  const int64_t tiles_in = inner >> lbi;
  const int64_t t = blockIdx.x;
  const int64_t o0 = (t / tiles_in) << lbo;
  const int64_t i0 = (t % tiles_in) << lbi;
  // all of a thread's loads are issued before the first LDS store
  constexpr int EPT = T / NT;
  float2 v[EPT];
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int e = threadIdx.x + k * NT;
    const int b_in = e & (bi - 1);
    const int jj = (e >> lbi) & (L - 1);
    const int b_o = e >> lbi >> __builtin_ctz(L);
    v[k] = o0 + b_o < outer ? data[((o0 + b_o) * L + jj) * inner + i0 + b_in] : make_float2(0.f, 0.f);
  }
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int e = threadIdx.x + k * NT;
    const int b_in = e & (bi - 1);
    const int jj = (e >> lbi) & (L - 1);
    const int b_o = e >> lbi >> __builtin_ctz(L);
    tile[((b_o << lbi) + b_in) * LP + jj] = v[k];
  }
  __syncthreads();
  fft_lines<L, T, NT, DIR, 1, LP>(tile, tw);
  for (int e = threadIdx.x; e < T; e += NT) {
    const int b_in = e & (bi - 1);
    const int jj = (e >> lbi) & (L - 1);
    const int b_o = e >> lbi >> __builtin_ctz(L);
    if (o0 + b_o < outer) data[((o0 + b_o) * L + jj) * inner + i0 + b_in] = tile[((b_o << lbi) + b_in) * LP + jj];
  }
}

constexpr int tile_threads(int d) { return d >= 16384 ? 1024 : d <= 1024 ? 64 : d / 16; }

// One workgroup transforms one whole H x W grid in LDS.
template <int H, int W, int DIR>
__global__ __launch_bounds__(tile_threads(H * W)) void k_fft2d(float2* __restrict__ data) {
  constexpr int D = H * W, NT = tile_threads(D), WP = W + 1;
  __shared__ float2 tile[H * WP];
  __shared__ float2 tw[256];
  float2* g = data + (int64_t)blockIdx.x * D;
  load_twiddles(tw);
  {
    // all of a thread's loads are issued before the first LDS store
    constexpr int EPT = (D + NT - 1) / NT;
    float2 v[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int e = threadIdx.x + k * NT;
      if (e < D) v[k] = g[e];
    }
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int e = threadIdx.x + k * NT;
      if (e < D) tile[(e / W) * WP + (e % W)] = v[k];
    }
  }
  __syncthreads();
  fft2d_tile<H, W, WP, NT, DIR>(tile, tw);
  for (int e = threadIdx.x; e < D; e += NT) g[e] = tile[(e / W) * WP + (e % W)];
}

static int ilog2(int64_t v) {
  int l = 0;
  while ((int64_t(1) << l) < v) ++l;
  return l;
}

template <int DIR>
static hipError_t axis_pass(float2* data, int64_t outer, int L, int64_t inner, hipStream_t st) {
  const int ll = ilog2(L);
  int lbi = ilog2(inner);
  const int lt = ilog2(kAxisTile);
  if (lbi > lt - ll) lbi = lt - ll;
  const int lbo = lt - ll - lbi;
  const int64_t tiles = ((outer + (int64_t(1) << lbo) - 1) >> lbo) * (inner >> lbi);
  const dim3 grid((unsigned)tiles), block(kAxisThreads);
  switch (L) {
#define CASE(LL) \
  case LL: hipLaunchKernelGGL((k_fft_axis<LL, DIR>), grid, block, 0, st, data, outer, inner, lbi, lbo); break;
    CASE(2) CASE(4) CASE(8) CASE(16) CASE(32) CASE(64) CASE(128) CASE(256)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int DIR>
static bool tile_launch(float2* data, int64_t count, int h, int w, hipStream_t st) {
#define TL(HH, WW)                                                                                 \
  if (h == HH && w == WW) {                                                                        \
    hipLaunchKernelGGL((k_fft2d<HH, WW, DIR>), dim3((unsigned)count), dim3(tile_threads(HH * WW)), \
                       0, st, data);                                                               \
    return true;                                                                                   \
  }
  TL(16, 16) TL(16, 32) TL(16, 64) TL(16, 128) TL(16, 256)
  TL(32, 16) TL(32, 32) TL(32, 64) TL(32, 128) TL(32, 256)
  TL(64, 16) TL(64, 32) TL(64, 64) TL(64, 128) TL(64, 256)
  TL(128, 16) TL(128, 32) TL(128, 64) TL(128, 128)
  TL(256, 16) TL(256, 32) TL(256, 64)
#undef TL
  return false;
}

bool tile_supported(int h, int w) {
  const bool ph = h >= 16 && h <= 256 && (h & (h - 1)) == 0;
  const bool pw = w >= 16 && w <= 256 && (w & (w - 1)) == 0;
  return ph && pw && h * w <= kTileMax;
}

hipError_t fft_grids(float2* data, int64_t count, const int g[3], int dir, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int T = g[0], H = g[1], W = g[2];
  if (T == 1 && tile_supported(H, W)) {
    const bool ok = dir < 0 ? tile_launch<-1>(data, count, H, W, st) : tile_launch<1>(data, count, H, W, st);
    return ok ? hipGetLastError() : hipErrorInvalidValue;
  }
  hipError_t e;
  const int64_t hw = int64_t(H) * W;
  if (dir < 0) {
    if ((e = axis_pass<-1>(data, count * T * H, W, 1, st)) != hipSuccess) return e;
    if ((e = axis_pass<-1>(data, count * T, H, W, st)) != hipSuccess) return e;
    if (T > 1 && (e = axis_pass<-1>(data, count, T, hw, st)) != hipSuccess) return e;
  } else {
    if ((e = axis_pass<1>(data, count * T * H, W, 1, st)) != hipSuccess) return e;
    if ((e = axis_pass<1>(data, count * T, H, W, st)) != hipSuccess) return e;
    if (T > 1 && (e = axis_pass<1>(data, count, T, hw, st)) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace dcsc
