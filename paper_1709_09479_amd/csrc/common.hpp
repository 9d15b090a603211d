// Device helpers shared by every kernel of the library: complex arithmetic,
// in-register DFTs of radix 2/4/8/16, a Stockham FFT over lines held in LDS,
// and deterministic block reductions.
//
// Transforms are unnormalised.  DIR = -1 is the forward DFT
// X[k] = sum_n x[n] exp(-2 pi i k n / L); DIR = +1 is the unscaled inverse.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dcsc {

// exp(-2 pi i m / 256), computed in float64 on the host and rounded once.
static __constant__ float2 c_tw256[256] = {
#include "twiddles.inc"
};

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float cabs2(float2 a) { return a.x * a.x + a.y * a.y; }

// multiply by DIR * i
template <int DIR>
__device__ __forceinline__ float2 mul_i(float2 a) {
  return DIR < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}

// multiply by (wr + DIR i wi)
template <int DIR>
__device__ __forceinline__ float2 mul_w(float2 a, float wr, float wi) {
  const float s = DIR < 0 ? -wi : wi;
  return make_float2(a.x * wr - a.y * s, a.x * s + a.y * wr);
}

constexpr float kC8 = 0.70710678118654752440f;   // cos(pi/4)
constexpr float kC16 = 0.92387953251128675613f;  // cos(pi/8)
constexpr float kS16 = 0.38268343236508977173f;  // sin(pi/8)

template <int DIR>
__device__ __forceinline__ void dft2(float2* v) {
  const float2 t = v[0];
  v[0] = cadd(t, v[1]);
  v[1] = csub(t, v[1]);
}

template <int DIR>
__device__ __forceinline__ void dft4(float2* v) {
  const float2 a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
  const float2 c = cadd(v[1], v[3]), d = mul_i<DIR>(csub(v[1], v[3]));
  v[0] = cadd(a, c);
  v[2] = csub(a, c);
  v[1] = cadd(b, d);
  v[3] = csub(b, d);
}

// natural order in and out: X[k] = E[k] + W^k O[k], X[k+4] = E[k] - W^k O[k]
template <int DIR>
__device__ __forceinline__ void dft8(float2* v) {
  float2 e[4] = {v[0], v[2], v[4], v[6]};
  float2 o[4] = {v[1], v[3], v[5], v[7]};
  dft4<DIR>(e);
  dft4<DIR>(o);
  o[1] = mul_w<DIR>(o[1], kC8, kC8);
  o[2] = mul_i<DIR>(o[2]);
  o[3] = mul_w<DIR>(o[3], -kC8, kC8);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = cadd(e[k], o[k]);
    v[k + 4] = csub(e[k], o[k]);
  }
}

template <int DIR>
__device__ __forceinline__ void dft16(float2* v) {
  float2 e[8], o[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    e[k] = v[2 * k];
    o[k] = v[2 * k + 1];
  }
  dft8<DIR>(e);
  dft8<DIR>(o);
  o[1] = mul_w<DIR>(o[1], kC16, kS16);
  o[2] = mul_w<DIR>(o[2], kC8, kC8);
  o[3] = mul_w<DIR>(o[3], kS16, kC16);
  o[4] = mul_i<DIR>(o[4]);
  o[5] = mul_w<DIR>(o[5], -kS16, kC16);
  o[6] = mul_w<DIR>(o[6], -kC8, kC8);
  o[7] = mul_w<DIR>(o[7], -kC16, kS16);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    v[k] = cadd(e[k], o[k]);
    v[k + 8] = csub(e[k], o[k]);
  }
}

template <int R, int DIR>
__device__ __forceinline__ void dft(float2* v) {
  if constexpr (R == 2) dft2<DIR>(v);
  else if constexpr (R == 4) dft4<DIR>(v);
  else if constexpr (R == 8) dft8<DIR>(v);
  else dft16<DIR>(v);
}

// Radix sequence per power-of-two length (2 .. 256).
constexpr int npasses(int L) { return L <= 16 ? 1 : 2; }
constexpr int radix_of(int L, int pass) {
  return L <= 16 ? L
       : L == 32 ? (pass == 0 ? 8 : 4)
       : L == 64 ? 8
       : L == 128 ? (pass == 0 ? 16 : 8)
       : 16;
}

// One Stockham pass (radix R, NS = product of the radices already applied)
// over B = T / L lines of length L held in LDS; element j of line b is at
// lds[b * SB + j * SL].  All NT threads of the block take part; the pass
// reads everything into registers, synchronises, writes, synchronises, so the
// transform runs in place.
template <int L, int T, int NT, int DIR, int SL, int SB, int PASS, int NS>
__device__ __forceinline__ void fft_pass(float2* lds, const float2* tw) {
  if constexpr (PASS < npasses(L)) {
    constexpr int R = radix_of(L, PASS);
    constexpr int B = T / L;
    constexpr int JOBS = T / R;
    constexpr int JPT = (JOBS + NT - 1) / NT;
    constexpr int LR = L / R;
    constexpr int TWSTEP = 256 / (NS * R);
    const int tid = threadIdx.x;
    float2 v[JPT][R];
#pragma unroll
    for (int q = 0; q < JPT; ++q) {
      const int job = tid + q * NT;
      if (JOBS % NT == 0 || job < JOBS) {
        const int b = job % B, j = job / B;
        const float2* src = lds + b * SB + j * SL;
#pragma unroll
        for (int r = 0; r < R; ++r) v[q][r] = src[r * LR * SL];
        if constexpr (NS > 1) {
          const int k = j % NS;
#pragma unroll
          for (int r = 1; r < R; ++r) {
            float2 w = tw[r * k * TWSTEP];
            if (DIR > 0) w.y = -w.y;
            v[q][r] = cmul(v[q][r], w);
          }
        }
        dft<R, DIR>(v[q]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < JPT; ++q) {
      const int job = tid + q * NT;
      if (JOBS % NT == 0 || job < JOBS) {
        const int b = job % B, j = job / B;
        const int k = j % NS;
        float2* dst = lds + b * SB + ((j / NS) * NS * R + k) * SL;
#pragma unroll
        for (int r = 0; r < R; ++r) dst[r * NS * SL] = v[q][r];
      }
    }
    __syncthreads();
    fft_pass<L, T, NT, DIR, SL, SB, PASS + 1, NS * R>(lds, tw);
  }
}

// B = T / L independent length-L transforms of lines in LDS.  The caller must
// have synchronised after writing the lines; the call ends synchronised.
template <int L, int T, int NT, int DIR, int SL, int SB>
__device__ __forceinline__ void fft_lines(float2* lds, const float2* tw) {
  fft_pass<L, T, NT, DIR, SL, SB, 0, 1>(lds, tw);
}

// 2-D transform of an H x W tile stored row-major with row stride WP.
template <int H, int W, int WP, int NT, int DIR>
__device__ __forceinline__ void fft2d_tile(float2* tile, const float2* tw) {
  fft_lines<W, H * W, NT, DIR, 1, WP>(tile, tw);
  fft_lines<H, H * W, NT, DIR, WP, 1>(tile, tw);
}

// ---------------------------------------------------------------------------
// Tile passes with explicit register hand-off.
//
// A 2-D tile of H x W complex values lives in LDS row-major with row stride
// WP.  Each axis of length L is transformed by plan_n(L) Stockham passes with
// radices plan_r(L, 0..) ("inverse order"); a forward transform uses the same
// radices in reverse order.  With that pairing the first pass of one
// transform reads exactly the register layout the last pass of the other
// leaves behind, so element-wise work between two transforms (and the global
// loads/stores feeding them) happens in registers without an LDS round trip.
constexpr int plan_n(int L) { return L <= 16 ? 1 : 2; }
constexpr int plan_r(int L, int i) {
  return L <= 16 ? L : L == 32 ? (i == 0 ? 8 : 4) : L == 64 ? 8 : L == 128 ? (i == 0 ? 8 : 16) : 16;
}

// One pass of radix R over the lines of a tile.  ROWS: lines are rows
// (address b * WP + pos); otherwise columns (address pos * WP + b).  JFAST:
// consecutive threads take consecutive positions j of one line; otherwise
// consecutive lines b.  NS: product of the radices already applied.
template <int L, int T, int NT, int DIR, int R_, int NS, bool JFAST, bool ROWS, int WP>
struct TilePass {
  static constexpr int R = R_;
  static constexpr int B = T / L, LR = L / R, JOBS = T / R;
  static constexpr int JPT = (JOBS + NT - 1) / NT;
  static constexpr bool FULL = (JOBS % NT) == 0;
  static constexpr int TWSTEP = 256 / (NS * R);
  __device__ static __forceinline__ bool job(int tid, int q, int& b, int& j) {
    const int jb = tid + q * NT;
    if (JFAST) {
      j = jb % LR;
      b = jb / LR;
    } else {
      b = jb % B;
      j = jb / B;
    }
    return FULL || jb < JOBS;
  }
  // one pad element after every 8 along a row; WP is the (odd) padded row
  // stride, so both lane-per-row and strided in-row accesses spread over banks
  __device__ static __forceinline__ int addr(int b, int pos) {
    return ROWS ? b * WP + pos + (pos >> 3) : pos * WP + b + (b >> 3);
  }
  __device__ static __forceinline__ int in_pos(int j, int r) { return j + r * LR; }
  __device__ static __forceinline__ int out_pos(int j, int r) { return (j / NS) * NS * R + (j % NS) + r * NS; }
  // read inputs from the tile, apply twiddles
  __device__ static __forceinline__ void load(int tid, const float2* tile, const float2* tw, float2 (&v)[JPT][R]) {
#pragma unroll
    for (int q = 0; q < JPT; ++q) {
      int b, j;
      if (!job(tid, q, b, j)) continue;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = tile[addr(b, in_pos(j, r))];
      if constexpr (NS > 1) {
        const int k = j % NS;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          float2 w = tw[r * k * TWSTEP];
          if (DIR > 0) w.y = -w.y;
          v[q][r] = cmul(v[q][r], w);
        }
      }
    }
  }
  __device__ static __forceinline__ void compute(int tid, float2 (&v)[JPT][R]) {
#pragma unroll
    for (int q = 0; q < JPT; ++q) {
      int b, j;
      if (job(tid, q, b, j)) dft<R, DIR>(v[q]);
    }
  }
  __device__ static __forceinline__ void store(int tid, float2* tile, const float2 (&v)[JPT][R]) {
#pragma unroll
    for (int q = 0; q < JPT; ++q) {
      int b, j;
      if (!job(tid, q, b, j)) continue;
#pragma unroll
      for (int r = 0; r < R; ++r) tile[addr(b, out_pos(j, r))] = v[q][r];
    }
  }
};

// The thread index as a value the compiler cannot treat as loop invariant:
// address arithmetic is then redone inside loops instead of being hoisted
// and held in registers across them.
__device__ __forceinline__ int opaque_tid() {
  int t = (int)threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// LDS -> LDS pass (in place; ends synchronised).
template <class P>
__device__ __forceinline__ void pass_lds(float2* tile, const float2* tw) {
  const int tid = opaque_tid();
  float2 v[P::JPT][P::R];
  P::load(tid, tile, tw, v);
  P::compute(tid, v);
  __syncthreads();
  P::store(tid, tile, v);
  __syncthreads();
}

// Register -> LDS pass (first pass of a transform, NS = 1).  Synchronises
// before writing (earlier readers of the tile) and after.
template <class P>
__device__ __forceinline__ void pass_from_regs(int tid, float2* tile, float2 (&v)[P::JPT][P::R]) {
  P::compute(tid, v);
  __syncthreads();
  P::store(tid, tile, v);
  __syncthreads();
}

// LDS -> register pass (last pass of a transform): outputs stay in v.
template <class P>
__device__ __forceinline__ void pass_to_regs(int tid, const float2* tile, const float2* tw, float2 (&v)[P::JPT][P::R]) {
  P::load(tid, tile, tw, v);
  P::compute(tid, v);
}

// Row stride of a padded W-wide tile (odd).
constexpr int tile_stride(int W) { return W + W / 8 + 1; }
// Pass types of the fused H x W tile transforms.
template <int H, int W, int NT, int WP>
struct TilePlan {
  static constexpr int T = H * W;
  static constexpr int NA = plan_n(W), NB = plan_n(H);
  static constexpr int A0 = plan_r(W, 0), AL = plan_r(W, NA - 1);
  static constexpr int B0 = plan_r(H, 0), BL = plan_r(H, NB - 1);
  // inverse: rows (A0 from registers [, AL]), then columns ([B0,] BL to registers)
  using InvRow0 = TilePass<W, T, NT, 1, A0, 1, true, true, WP>;
  using InvRow1 = TilePass<W, T, NT, 1, AL, A0, false, true, WP>;
  using InvCol0 = TilePass<H, T, NT, 1, B0, 1, false, false, WP>;
  using InvColL = TilePass<H, T, NT, 1, BL, H / BL, false, false, WP>;
  // forward: columns (BL from registers [, B0]), then rows ([AL,] A0 to registers)
  using FwdCol0 = TilePass<H, T, NT, -1, BL, 1, false, false, WP>;
  using FwdCol1 = TilePass<H, T, NT, -1, B0, BL, false, false, WP>;
  using FwdRow0 = TilePass<W, T, NT, -1, AL, 1, false, true, WP>;
  using FwdRowL = TilePass<W, T, NT, -1, A0, W / A0, true, true, WP>;
};

// Copy the twiddle table into LDS (caller synchronises before use).
__device__ __forceinline__ void load_twiddles(float2* tw_lds) {
  for (int i = threadIdx.x; i < 256; i += blockDim.x) tw_lds[i] = c_tw256[i];
}

// Sum of one double per thread over the block, in a fixed order.  Returns the
// total in thread 0 (other threads get an unspecified value).  `red` must hold
// blockDim.x / 64 doubles.
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 0; w < nw; ++w) t += red[w];
  }
  return t;
}

// Start of image n's code maps ([K][grid]) and of its image ([J][grid]).
__device__ __forceinline__ int64_t map_base(const int64_t* __restrict__ zoff, int n, int K, int64_t D) {
  return zoff ? zoff[n] : int64_t(n) * K * D;
}

// Work item of workgroup `id` of a 1-D grid of `total` workgroups when the
// items (in the caller's order) go to the 8 XCDs of the chip in contiguous
// ranges.  Workgroups are dispatched to the XCDs round-robin, so id % 8 names
// the XCD and id / 8 the position within its range.  A bijection on
// [0, total) for any total.
__device__ __forceinline__ int xcd_item(int id, int total) {
  constexpr int kXcd = 8;
  const int q = total / kXcd, r = total % kXcd;
  const int x = id % kXcd, s = id / kXcd;
  return x * q + (x < r ? x : r) + s;
}

// lam = (G + I/rho)^-1 r for one frequency.  J = 1 is a division; J > 1 is a
// Cholesky factorisation of the Hermitian positive-definite J x J block,
// carried out in float64.
template <int J>
__device__ __forceinline__ void dual_solve(const float2* __restrict__ Gf, float inv_rho, const float2* r,
                                           float2* lam) {
  if constexpr (J == 1) {
    const float den = Gf[0].x + inv_rho;
    lam[0] = make_float2(r[0].x / den, r[0].y / den);
  } else {
    double Lr[J][J], Li[J][J];
#pragma unroll
    for (int a = 0; a < J; ++a)
#pragma unroll
      for (int c = 0; c < J; ++c) Lr[a][c] = Li[a][c] = 0.0;
#pragma unroll
    for (int c = 0; c < J; ++c) {
      double s = (double)Gf[c * J + c].x + (double)inv_rho;
#pragma unroll
      for (int m = 0; m < c; ++m) s -= Lr[c][m] * Lr[c][m] + Li[c][m] * Li[c][m];
      const double lcc = sqrt(s);
      Lr[c][c] = lcc;
#pragma unroll
      for (int a = c + 1; a < J; ++a) {
        // L[a][c] = (A[a][c] - sum_m L[a][m] conj(L[c][m])) / L[c][c]
        double sr = Gf[a * J + c].x, si = Gf[a * J + c].y;
#pragma unroll
        for (int m = 0; m < c; ++m) {
          sr -= Lr[a][m] * Lr[c][m] + Li[a][m] * Li[c][m];
          si -= Li[a][m] * Lr[c][m] - Lr[a][m] * Li[c][m];
        }
        Lr[a][c] = sr / lcc;
        Li[a][c] = si / lcc;
      }
    }
    double yr[J], yi[J];
#pragma unroll
    for (int a = 0; a < J; ++a) {  // L y = r
      double sr = r[a].x, si = r[a].y;
#pragma unroll
      for (int m = 0; m < a; ++m) {
        sr -= Lr[a][m] * yr[m] - Li[a][m] * yi[m];
        si -= Lr[a][m] * yi[m] + Li[a][m] * yr[m];
      }
      yr[a] = sr / Lr[a][a];
      yi[a] = si / Lr[a][a];
    }
#pragma unroll
    for (int a = J - 1; a >= 0; --a) {  // L^H x = y
      double sr = yr[a], si = yi[a];
#pragma unroll
      for (int m = a + 1; m < J; ++m) {
        // conj(L[m][a]) * x[m]
        sr -= Lr[m][a] * yr[m] + Li[m][a] * yi[m];
        si -= Lr[m][a] * yi[m] - Li[m][a] * yr[m];
      }
      yr[a] = sr / Lr[a][a];
      yi[a] = si / Lr[a][a];
    }
#pragma unroll
    for (int a = 0; a < J; ++a) lam[a] = make_float2((float)yr[a], (float)yi[a]);
  }
}

__device__ __forceinline__ float soft_thresh(float u, float t) {
  const float a = fabsf(u) - t;
  return a > 0.0f ? copysignf(a, u) : 0.0f;
}

}  // namespace dcsc
