// Coding iteration for 2-D grids too large for one LDS tile (128 x 256,
// 256 x 128, 256 x 256): the map work of one ADMM iteration (back-projection
// D^T lambda, soft threshold, forward transform and reduction, see
// eq:Inference_solution) split into a row phase, a column phase and a row
// phase, so that every intermediate crosses HBM once each way:
//   rows inverse   buf[n][p] = row-IDFT of V = sum_j lam_j E_jp
//   columns        column-IDFT, soft-threshold step on the map pair (z in
//                  place, residual partials), column-DFT; buf in place
//   rows forward   row-DFT, times conj(E_jp), summed over the pairs of a
//                  group into part[n][g][j]
// Each workgroup stages a 4096-element tile (rows x W, or H x columns) in LDS
// and runs the same register hand-off passes as the single-tile kernel.
#include "common.hpp"
#include "internal.hpp"
#include "tiles.hpp"

namespace dcsc {

// Kernels: one item (tiles.hpp) per workgroup.

template <int W, int J>
__global__ __launch_bounds__(kSplitNT) void k_split_rows_inv(const float2* __restrict__ E,
                                                             const float2* __restrict__ lam,
                                                             float2* __restrict__ buf, int P, int H,
                                                             const int* __restrict__ stop) {
  if (stop && stop[0]) return;
  constexpr int RB = kSplitT / W, WP = tile_stride(W);
  __shared__ float2 tile[RB * WP];
  __shared__ float2 tw[256];
  load_twiddles(tw);
  // items (row chunk, pair)-major, images fastest, spread over the XCDs so
  // that the images of one XCD share rows of E in its L2
  const int N = (int)(gridDim.x / (unsigned)(P * (H / RB)));
  const int item = xcd_item((int)blockIdx.x, (int)gridDim.x);
  rows_inv_item<W, J>(tile, tw, item % N, (item / N) % P, item / N / P, E, lam, buf, P, H);
}

template <int H, int MODE>
__global__ __launch_bounds__(kSplitNT) void k_split_cols(float2* __restrict__ buf, float* __restrict__ z,
                                                         const float* zin,
                                                         float* __restrict__ theta, const int64_t* __restrict__ zoff,
                                                         const float* __restrict__ rho_cur, float beta,
                                                         double* __restrict__ rpart, int K, int P, int W,
                                                         const int* __restrict__ stop) {
  if (stop && stop[0]) return;
  constexpr int CB = kSplitT / H, WP = tile_stride(CB);
  __shared__ float2 tile[H * WP];
  __shared__ float2 tw[256];
  __shared__ double red[kSplitNT / 64];
  load_twiddles(tw);
  // column blocks fastest, in contiguous ranges per XCD: the two halves of
  // a 128-byte line of a map row (16 columns of 4 bytes each when H = 256)
  // are read by neighbouring blocks of one XCD, so the second finds the
  // line in that XCD's L2
  const int ncb = W / CB, item = xcd_item((int)blockIdx.x, (int)gridDim.x);
  cols_item<H, MODE>(tile, tw, red, item / ncb / P, (item / ncb) % P, item % ncb, ncb, buf, z, zin, theta, zoff,
                     rho_cur, beta, rpart, K, P, W);
}

template <int W, int J>
__global__ __launch_bounds__(kSplitNT) void k_split_rows_fwd(const float2* __restrict__ E,
                                                             const float2* __restrict__ buf,
                                                             float2* __restrict__ part, int P, int H, int ppg,
                                                             int ng, const int* __restrict__ stop) {
  if (stop && stop[0]) return;
  constexpr int RB = kSplitT / W, WP = tile_stride(W);
  __shared__ float2 tile[RB * WP];
  __shared__ float2 tw[256];
  load_twiddles(tw);
  const int N = (int)(gridDim.x / (unsigned)(ng * (H / RB)));
  const int item = xcd_item((int)blockIdx.x, (int)gridDim.x);  // as in the inverse row phase
  rows_fwd_item<W, J>(tile, tw, item % N, (item / N) % ng, item / N / ng, E, buf, part, P, H, ppg, ng);
}

// ================================================================== host

bool split_supported(int T, int H, int W) { return T == 1 && (H == 128 || H == 256) && (W == 128 || W == 256) && H * W > kTileMax; }

int split_col_blocks(const Plan& pl) { return pl.g[2] / (kSplitT / pl.g[1]); }

int split_row_blocks(const Plan& pl) { return pl.g[1] / (kSplitT / pl.g[2]); }

template <int J>
static hipError_t split_iter_j(const Plan& pl, const float2* E, const float2* lam, float2* buf, float* z,
                               float* theta, const float* rho, float beta, float2* part, double* rpart, int mode,
                               hipStream_t st, const int* stop, const float* zin) {
  const int H = pl.g[1], W = pl.g[2];
  const dim3 blk(kSplitNT);
  if (mode == 0) {
    const dim3 g1(split_row_blocks(pl) * pl.p * pl.n);
    if (W == 256) hipLaunchKernelGGL((k_split_rows_inv<256, J>), g1, blk, 0, st, E, lam, buf, pl.p, H, stop);
    else hipLaunchKernelGGL((k_split_rows_inv<128, J>), g1, blk, 0, st, E, lam, buf, pl.p, H, stop);
  }
  const dim3 g2(split_col_blocks(pl) * pl.p * pl.n);
  if (mode == 0) {
    if (H == 256)
      hipLaunchKernelGGL((k_split_cols<256, 0>), g2, blk, 0, st, buf, z, zin, theta, pl.zoff, rho, beta, rpart, pl.k,
                         pl.p, W, stop);
    else
      hipLaunchKernelGGL((k_split_cols<128, 0>), g2, blk, 0, st, buf, z, zin, theta, pl.zoff, rho, beta, rpart, pl.k,
                         pl.p, W, stop);
  } else {
    if (H == 256)
      hipLaunchKernelGGL((k_split_cols<256, 1>), g2, blk, 0, st, buf, z, nullptr, nullptr, pl.zoff, rho, 0.f, rpart,
                         pl.k, pl.p, W, stop);
    else
      hipLaunchKernelGGL((k_split_cols<128, 1>), g2, blk, 0, st, buf, z, nullptr, nullptr, pl.zoff, rho, 0.f, rpart,
                         pl.k, pl.p, W, stop);
  }
  const dim3 g3(split_row_blocks(pl) * pl.ng * pl.n);
  if (W == 256) hipLaunchKernelGGL((k_split_rows_fwd<256, J>), g3, blk, 0, st, E, buf, part, pl.p, H, pl.ppg, pl.ng, stop);
  else hipLaunchKernelGGL((k_split_rows_fwd<128, J>), g3, blk, 0, st, E, buf, part, pl.p, H, pl.ppg, pl.ng, stop);
  return hipGetLastError();
}

// mode 0: one ADMM map iteration; mode 1: forward transform and reduction of
// the given maps (z), l1 partials in rpart.
hipError_t split_maps(const Plan& pl, const float2* E, const float2* lam, float2* buf, float* z, float* theta,
                      const float* rho, float beta, float2* part, double* rpart, int mode, hipStream_t st,
                      const int* stop, const float* zin) {
  if (pl.j == 1) return split_iter_j<1>(pl, E, lam, buf, z, theta, rho, beta, part, rpart, mode, st, stop, zin);
  if (pl.j == 2) return split_iter_j<2>(pl, E, lam, buf, z, theta, rho, beta, part, rpart, mode, st, stop, zin);
  return split_iter_j<3>(pl, E, lam, buf, z, theta, rho, beta, part, rpart, mode, st, stop, zin);
}

}  // namespace dcsc
