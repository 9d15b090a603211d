// Work items of the coding iteration as device functions: the fused
// single-tile map work, the three phases of the split path for larger 2-D
// grids and the per-frequency spectral step.  Each kernel of coding.hip and
// split.hip is one item per workgroup; the batched form (batched.hip) runs
// items of every grid class of a batch from one launch per phase.  An item
// takes its LDS (tile, twiddles, reduction scratch) from the caller; the
// twiddles must be loaded (load_twiddles) before the first item, and every
// item synchronises before its first write to the tile, so items can follow
// one another in a workgroup.
#pragma once
#include "common.hpp"

namespace dcsc {

constexpr int kSpecT = 256;     // threads (frequencies) of a spectral item
constexpr int kSplitT = 4096;   // complex elements per split-path tile
constexpr int kSplitNT = 256;   // threads of a split-path item

// Index of -f on the grid (T, H, W all powers of two).
__device__ __forceinline__ int64_t neg_index(int64_t fl, int T, int H, int W) {
  const int f = (int)fl;
  const int lw = __builtin_ctz(W), lh = __builtin_ctz(H);
  const int w = f & (W - 1), h = (f >> lw) & (H - 1), t = f >> (lw + lh);
  return (((((T - t) & (T - 1)) << lh) | ((H - h) & (H - 1))) << lw) | ((W - w) & (W - 1));
}

// Y(f) and Y(-f) for Y = sum_g part[n][g][j] (groups added in a fixed order
// by U interleaved accumulators, so that 2 U loads are in flight).
template <int U>
__device__ __forceinline__ void group_sums(const float2* __restrict__ part, int64_t stride_g, int ng, int64_t f,
                                           int64_t fn, float2& y, float2& ym) {
  float2 a[U], m[U];
#pragma unroll
  for (int u = 0; u < U; ++u) a[u] = m[u] = make_float2(0.f, 0.f);
  int g = 0;
  for (; g + U <= ng; g += U) {
    // all 2 U loads first: left to itself the scheduler interleaves each
    // load with its add through one register pair, one load in flight
    float2 va[U], vm[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const float2* pp = part + (g + u) * stride_g;
      va[u] = pp[f];
      vm[u] = pp[fn];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      a[u] = cadd(a[u], va[u]);
      m[u] = cadd(m[u], vm[u]);
    }
  }
  if (g < ng) {
    // the remaining groups the same way: every load from a valid group
    // (the last one for slots past ng), weighted by 1 or 0, which adds the
    // same bits as a plain sum
    float2 va[U], vm[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const float2* pp = part + min(g + u, ng - 1) * stride_g;
      va[u] = pp[f];
      vm[u] = pp[fn];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const float w = g + u < ng ? 1.f : 0.f;
      a[u] = make_float2(fmaf(w, va[u].x, a[u].x), fmaf(w, va[u].y, a[u].y));
      m[u] = make_float2(fmaf(w, vm[u].x, m[u].x), fmaf(w, vm[u].y, m[u].y));
    }
  }
#pragma unroll
  for (int h = U / 2; h > 0; h /= 2)
#pragma unroll
    for (int u = 0; u < h; ++u) {
      a[u] = cadd(a[u], a[u + h]);
      m[u] = cadd(m[u], m[u + h]);
    }
  y = a[0];
  ym = m[0];
}

// One block of kSpecT frequencies of image n after the forward pass of
// iteration i: yhat' = sym(sum_g part), Thhat' =
// G lam + (yhat' - yhat)/rho_i, partial sums of |Thhat' - Thhat|^2 (the dual
// residual by Parseval) and, when the step size is fixed, the next lam.  The
// thread of the lower index of each pair (f, -f) does both frequencies, so
// part is read once.
// U: group accumulators (2 U loads in flight); 16 pays where there are many
// groups (single-tile plans), 8 keeps registers low otherwise.
template <int J, int U>
__device__ __forceinline__ void spec_item(double* red, int blk, int n, int nblk, const float2* __restrict__ part,
                                          const float2* __restrict__ G, const float2* __restrict__ xh,
                                          float2* __restrict__ yh, float2* __restrict__ Th, float2* __restrict__ lam,
                                          const float* __restrict__ rho_cur, double* __restrict__ rdual, int ng, int T,
                                          int H, int W, int solve_next) {
  const int64_t D = int64_t(T) * H * W;
  const int64_t f = blk * (int64_t)kSpecT + threadIdx.x;
  double ds = 0.0;
  const int64_t fn = f < D ? neg_index(f, T, H, W) : 0;
  if (f < D && fn >= f) {  // the pair (f, -f) is handled once, by its lower index
    const float rho = rho_cur[n], inv_rho = 1.0f / rho;
    // the per-image spectra at f and -f do not depend on the group sums:
    // (for J = 1) their loads go out first
    float2 l0[J == 1 ? 2 : 1], y0[J == 1 ? 2 : 1], t0[J == 1 ? 2 : 1];
    if constexpr (J == 1) {
      const int64_t o = int64_t(n) * D;
      l0[0] = lam[o + f], y0[0] = yh[o + f], t0[0] = Th[o + f];
      l0[1] = lam[o + fn], y0[1] = yh[o + fn], t0[1] = Th[o + fn];
    }
    float2 ys[J];  // yhat' at f; at -f it is the conjugate
#pragma unroll
    for (int j = 0; j < J; ++j) {
      float2 y, ym;
      group_sums<U>(part + (int64_t(n) * ng * J + j) * D, int64_t(J) * D, ng, f, fn, y, ym);
      ys[j] = make_float2(0.5f * (y.x + ym.x), 0.5f * (y.y - ym.y));
    }
    for (int side = 0; side < (fn == f ? 1 : 2); ++side) {
      const int64_t ff = side ? fn : f;
      const float2* Gf = G + ff * J * J;
      float2 ynew[J], l[J], thn[J];
#pragma unroll
      for (int j = 0; j < J; ++j) {
        ynew[j] = side ? cconj(ys[j]) : ys[j];
        if constexpr (J == 1) l[j] = l0[side];
        else l[j] = lam[(int64_t(n) * J + j) * D + ff];
      }
#pragma unroll
      for (int j = 0; j < J; ++j) {
        float2 gl = make_float2(0.f, 0.f);
#pragma unroll
        for (int c = 0; c < J; ++c) gl = cadd(gl, cmul(Gf[j * J + c], l[c]));
        const int64_t o = (int64_t(n) * J + j) * D + ff;
        float2 yo, tho;
        if constexpr (J == 1) {
          yo = y0[side];
          tho = t0[side];
        } else {
          yo = yh[o];
          tho = Th[o];
        }
        thn[j] = make_float2(gl.x + (ynew[j].x - yo.x) * inv_rho, gl.y + (ynew[j].y - yo.y) * inv_rho);
        const double dx = (double)thn[j].x - tho.x, dy = (double)thn[j].y - tho.y;
        ds += dx * dx + dy * dy;
        yh[o] = ynew[j];
        Th[o] = thn[j];
      }
      if (solve_next) {
        float2 r[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
          const float2 x = xh[(int64_t(n) * J + j) * D + ff];
          r[j] = make_float2(thn[j].x + (ynew[j].x - x.x) * inv_rho, thn[j].y + (ynew[j].y - x.y) * inv_rho);
        }
        dual_solve<J>(Gf, inv_rho, r, l);
#pragma unroll
        for (int j = 0; j < J; ++j) lam[(int64_t(n) * J + j) * D + ff] = l[j];
      }
    }
  }
  const double t = block_sum(ds, red);
  if (threadIdx.x == 0) rdual[int64_t(n) * nblk + blk] = t;
}

// ------------------------------------------------------- fused tile kernel

// Threads per workgroup of the fused kernel: 32 elements per thread (512
// threads for the largest tiles).  J = 1 keeps its accumulator in
// registers; J > 1 writes each pair's spectrum, which k_accum reduces.
constexpr int fused_threads(int t, int j) {
  return j == 1 ? (t >= 16384 ? 1024 : (t / 32 < 64 ? 64 : t / 32))
                : (t >= 16384 ? 1024 : (t / 16 < 64 ? 64 : t / 16));
}

enum { kModeIter = 0, kModeForward = 1 };

// One workgroup per (pair group g, image n), handed out by xcd_item so that
// the workgroups of one XCD share pair groups (and their filter spectra in
// that XCD's L2) across the images.  kModeIter: for every pair p of
// the group, back-project lam (V = sum_j lam_j E_jp), inverse 2-D FFT, soft
// threshold step on the two maps (z updated in place, optional theta),
// forward 2-D FFT, and accumulate Y_j += C conj(E_jp).  kModeForward: only
// the forward FFT and accumulation of the given maps (plus l1 sums).
// The first pass of the inverse transform takes V straight from global
// memory, its last pass leaves D^T lam in registers for the soft threshold,
// whose result feeds the first forward pass from registers; the last forward
// pass leaves the spectrum in registers for the accumulation.
// part: J = 1 [N][ng][D] (the group's sum over its pairs); J > 1 [N][P][D]
// (each pair's spectrum C, reduced over the pairs by k_accum);
// rpart [N][ng] (sum (z'-z)^2, or sum |z| when forward).
template <int H, int W, int J, int MODE, int NT>
__device__ __forceinline__ void fused_item(float2* tile, const float2* tw, double* red, int n, int g,
                                           const float2* __restrict__ E, const float2* __restrict__ lam,
                                           float* __restrict__ z, float* __restrict__ theta,
                                           const int64_t* __restrict__ zoff, const float* __restrict__ rho_cur,
                                           float beta, float2* __restrict__ part, double* __restrict__ rpart, int K,
                                           int P, int ppg, int ng) {
  constexpr int D = H * W, WP = tile_stride(W);
#include "fused_body.inc"
}

// ------------------------------------------------ split path (large 2-D grids)

// ---------------------------------------------------------- rows inverse
template <int W, int J>
__device__ __forceinline__ void rows_inv_item(float2* tile, const float2* tw, int n, int p, int rc,
                                              const float2* __restrict__ E, const float2* __restrict__ lam,
                                              float2* __restrict__ buf, int P, int H) {
  constexpr int T = kSplitT, NT = kSplitNT, RB = T / W, WP = tile_stride(W);
  constexpr int A0 = plan_r(W, 0), AL = plan_r(W, 1);
  using P0 = TilePass<W, T, NT, 1, A0, 1, true, true, WP>;
  using P1 = TilePass<W, T, NT, 1, AL, A0, true, true, WP>;
  static_assert(plan_n(W) == 2, "two passes per row");
  const int64_t D = int64_t(H) * W, row0 = int64_t(rc) * RB;
  const float2* lamn = lam + int64_t(n) * J * D;
  const float2* Ep[J];
#pragma unroll
  for (int c = 0; c < J; ++c) Ep[c] = E + (int64_t(c) * P + p) * D;
  const int tid = opaque_tid();
  float2 v[P0::JPT][P0::R];
#pragma unroll
  for (int q = 0; q < P0::JPT; ++q) {
    int b, j;
    if (!P0::job(tid, q, b, j)) continue;
#pragma unroll
    for (int r = 0; r < P0::R; ++r) {
      const int64_t f = (row0 + b) * W + P0::in_pos(j, r);
      float2 s = make_float2(0.f, 0.f);
#pragma unroll
      for (int c = 0; c < J; ++c) s = cadd(s, cmul(lamn[c * D + f], Ep[c][f]));
      v[q][r] = s;
    }
  }
  pass_from_regs<P0>(tid, tile, v);
  float2 u[P1::JPT][P1::R];
  pass_to_regs<P1>(tid, tile, tw, u);
  float2* g = buf + (int64_t(n) * P + p) * D;
#pragma unroll
  for (int q = 0; q < P1::JPT; ++q) {
    int b, j;
    if (!P1::job(tid, q, b, j)) continue;
#pragma unroll
    for (int r = 0; r < P1::R; ++r) g[(row0 + b) * W + P1::out_pos(j, r)] = u[q][r];
  }
}


// ---------------------------------------------------------------- columns
// MODE 0 (iteration): column-IDFT, soft-threshold step, column-DFT; the
// codes are read from zin (the same layout as z; null: z itself, updated in
// place) and written to z.
// MODE 1 (forward only): the map pair enters from z, l1 partials.
// rpart[n][p * ncb + cb] (ncb column blocks): sum (z' - z)^2, or sum |z|.
template <int H, int MODE>
__device__ __forceinline__ void cols_item(float2* tile, const float2* tw, double* red, int n, int p, int cb, int ncb,
                                          float2* __restrict__ buf, float* __restrict__ z, const float* zin,
                                          float* __restrict__ theta, const int64_t* __restrict__ zoff,
                                          const float* __restrict__ rho_cur, float beta, double* __restrict__ rpart,
                                          int K, int P, int W) {
  constexpr int T = kSplitT, NT = kSplitNT, CB = T / H, WP = tile_stride(CB);
  constexpr int B0 = plan_r(H, 0), BL = plan_r(H, 1);
  using C0 = TilePass<H, T, NT, 1, B0, 1, false, false, WP>;
  using CL = TilePass<H, T, NT, 1, BL, H / BL, false, false, WP>;
  using F0 = TilePass<H, T, NT, -1, BL, 1, false, false, WP>;
  using F1 = TilePass<H, T, NT, -1, B0, BL, false, false, WP>;
  static_assert(CL::JPT == F0::JPT && CL::R == F0::R, "register hand-off mismatch");
  const int64_t D = int64_t(H) * W;
  const int c0 = cb * CB;
  float2* g = buf + (int64_t(n) * P + p) * D;
  const int ka = 2 * p, kb = 2 * p + 1;
  const bool hb = kb < K;
  const int64_t zbase = map_base(zoff, n, K, D);
  float* za = z + zbase + int64_t(ka) * D;
  float* zb = z + zbase + int64_t(hb ? kb : ka) * D;
  const float* zsrc = (MODE == 0 && zin) ? zin : z;
  const float* zia = zsrc + zbase + int64_t(ka) * D;
  const float* zib = zsrc + zbase + int64_t(hb ? kb : ka) * D;
  const int tid = opaque_tid();
  double rsum = 0.0;
  float2 v[F0::JPT][F0::R];
  if constexpr (MODE == 0) {
    const float rho = rho_cur[n], thr = rho * beta, inv_rho = 1.0f / rho, invD = 1.0f / (float)D;
    float2 a[C0::JPT][C0::R];
#pragma unroll
    for (int q = 0; q < C0::JPT; ++q) {
      int b, j;
      if (!C0::job(tid, q, b, j)) continue;
#pragma unroll
      for (int r = 0; r < C0::R; ++r) a[q][r] = g[int64_t(C0::in_pos(j, r)) * W + c0 + b];
    }
    pass_from_regs<C0>(tid, tile, a);
    pass_to_regs<CL>(tid, tile, tw, v);
    float* tha = theta ? theta + zbase + int64_t(ka) * D : nullptr;
    float* thb = theta ? theta + zbase + int64_t(hb ? kb : ka) * D : nullptr;
#pragma unroll
    for (int q = 0; q < CL::JPT; ++q) {
      int b, j;
      if (!CL::job(tid, q, b, j)) continue;
      float rs = 0.f;
#pragma unroll
      for (int r = 0; r < CL::R; ++r) {
        const int64_t f = int64_t(CL::out_pos(j, r)) * W + c0 + b;
        const float va = v[q][r].x * invD, vb = v[q][r].y * invD;
        const float a0 = zia[f], b0 = hb ? zib[f] : 0.f;
        const float a1 = soft_thresh(fmaf(-rho, va, a0), thr);
        const float b1 = hb ? soft_thresh(fmaf(-rho, vb, b0), thr) : 0.f;
        const float da = a1 - a0, db = b1 - b0;
        rs = fmaf(da, da, fmaf(db, db, rs));
        za[f] = a1;
        if (hb) zb[f] = b1;
        if (tha) {
          tha[f] = va + da * inv_rho;
          if (hb) thb[f] = vb + db * inv_rho;
        }
        v[q][r] = make_float2(a1, b1);
      }
      rsum += (double)rs;
    }
  } else {
#pragma unroll
    for (int q = 0; q < F0::JPT; ++q) {
      int b, j;
      if (!F0::job(tid, q, b, j)) continue;
#pragma unroll
      for (int r = 0; r < F0::R; ++r) {
        const int64_t f = int64_t(F0::in_pos(j, r)) * W + c0 + b;
        const float a0 = za[f], b0 = hb ? zb[f] : 0.f;
        rsum += (double)fabsf(a0) + (double)fabsf(b0);
        v[q][r] = make_float2(a0, b0);
      }
    }
  }
  pass_from_regs<F0>(tid, tile, v);
  float2 u[F1::JPT][F1::R];
  pass_to_regs<F1>(tid, tile, tw, u);
#pragma unroll
  for (int q = 0; q < F1::JPT; ++q) {
    int b, j;
    if (!F1::job(tid, q, b, j)) continue;
#pragma unroll
    for (int r = 0; r < F1::R; ++r) g[int64_t(F1::out_pos(j, r)) * W + c0 + b] = u[q][r];
  }
  const double tot = block_sum(rsum, red);
  if (threadIdx.x == 0) rpart[(int64_t(n) * P + p) * ncb + cb] = tot;
}


// ---------------------------------------------------------- rows forward
// part[n][g][j] rows of this tile = sum over the group's pairs of
// row-DFT(buf[n][p]) conj(E_jp); an empty group writes zeros.
template <int W, int J>
__device__ __forceinline__ void rows_fwd_item(float2* tile, const float2* tw, int n, int gi, int rc,
                                              const float2* __restrict__ E, const float2* __restrict__ buf,
                                              float2* __restrict__ part, int P, int H, int ppg, int ng) {
  constexpr int T = kSplitT, NT = kSplitNT, RB = T / W, WP = tile_stride(W);
  constexpr int A0 = plan_r(W, 0), AL = plan_r(W, 1);
  using Q0 = TilePass<W, T, NT, -1, AL, 1, true, true, WP>;
  using Q1 = TilePass<W, T, NT, -1, A0, AL, true, true, WP>;
  const int64_t D = int64_t(H) * W, row0 = int64_t(rc) * RB;
  const int p0 = gi * ppg, p1 = min(P, p0 + ppg);
  float2 acc[J][Q1::JPT][Q1::R];
#pragma unroll
  for (int c = 0; c < J; ++c)
#pragma unroll
    for (int q = 0; q < Q1::JPT; ++q)
#pragma unroll
      for (int r = 0; r < Q1::R; ++r) acc[c][q][r] = make_float2(0.f, 0.f);
  // The tile of the next pair and the filter spectra of this pair (J = 1)
  // are loaded before this pair's row transform, so that their latency
  // overlaps the transform instead of following it.
  auto load_tile = [&](int p, float2 (&v)[Q0::JPT][Q0::R]) {
    const int tid = opaque_tid();
    const float2* g = buf + (int64_t(n) * P + p) * D;
#pragma unroll
    for (int q = 0; q < Q0::JPT; ++q) {
      int b, j;
      if (!Q0::job(tid, q, b, j)) continue;
#pragma unroll
      for (int r = 0; r < Q0::R; ++r) v[q][r] = g[(row0 + b) * W + Q0::in_pos(j, r)];
    }
  };
  float2 v[Q0::JPT][Q0::R];
  if (p0 < p1) load_tile(p0, v);
  for (int p = p0; p < p1; ++p) {
    const int tid = opaque_tid();
    float2 e[J == 1 ? Q1::JPT : 1][J == 1 ? Q1::R : 1];
    float2 vn[J == 1 ? Q0::JPT : 1][J == 1 ? Q0::R : 1];
    if constexpr (J == 1) {
#pragma unroll
      for (int q = 0; q < Q1::JPT; ++q) {
        int b, j;
        if (!Q1::job(tid, q, b, j)) continue;
#pragma unroll
        for (int r = 0; r < Q1::R; ++r) e[q][r] = E[int64_t(p) * D + (row0 + b) * W + Q1::out_pos(j, r)];
      }
      if (p + 1 < p1) load_tile(p + 1, vn);
    }
    pass_from_regs<Q0>(tid, tile, v);
    float2 u[Q1::JPT][Q1::R];
    pass_to_regs<Q1>(tid, tile, tw, u);
#pragma unroll
    for (int q = 0; q < Q1::JPT; ++q) {
      int b, j;
      if (!Q1::job(tid, q, b, j)) continue;
#pragma unroll
      for (int r = 0; r < Q1::R; ++r) {
        if constexpr (J == 1) {
          acc[0][q][r] = cadd(acc[0][q][r], cmulc(u[q][r], e[q][r]));
        } else {
          const int64_t f = (row0 + b) * W + Q1::out_pos(j, r);
#pragma unroll
          for (int c = 0; c < J; ++c)
            acc[c][q][r] = cadd(acc[c][q][r], cmulc(u[q][r], E[(int64_t(c) * P + p) * D + f]));
        }
      }
    }
    if constexpr (J == 1) {
#pragma unroll
      for (int q = 0; q < Q0::JPT; ++q)
#pragma unroll
        for (int r = 0; r < Q0::R; ++r) v[q][r] = vn[q][r];
    } else if (p + 1 < p1) {
      load_tile(p + 1, v);
    }
  }
  const int tid = opaque_tid();
#pragma unroll
  for (int q = 0; q < Q1::JPT; ++q) {
    int b, j;
    if (!Q1::job(tid, q, b, j)) continue;
#pragma unroll
    for (int r = 0; r < Q1::R; ++r) {
      const int64_t f = (row0 + b) * W + Q1::out_pos(j, r);
#pragma unroll
      for (int c = 0; c < J; ++c) part[((int64_t(n) * ng + gi) * J + c) * D + f] = acc[c][q][r];
    }
  }
}


}  // namespace dcsc
