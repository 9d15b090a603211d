// Learning subproblem (eq:Learning_gamma .. eq:mu_update) with the CG of each
// multiplier step carried in a span of known vectors.
//
// The operator of eq:Learning_gamma is A = I + Z S^T W S Z^T with
// W = diag_k 1/(2 mu_k).  Every vector the CG of a learning call forms lies in
//     V = { a x + b gamma_0 + Z S^T w : a, b scalars, w in the filter space },
// gamma_0 the warm start: r_0 = -x - A gamma_0 is in V, and A maps V into V,
//     A(a x + b gamma_0 + Z S^T w) = a x + b gamma_0 + Z S^T (w + W h),
//     h = S Z^T (a x + b gamma_0 + Z S^T w) = a g_x + b g_0 + M w,
// with g_x = S Z^T x, g_0 = S Z^T gamma_0 and M = S Z^T Z S^T.  A vector of V
// is carried as (a, b, w, m = M w), per channel, and
//   <V, V'> = a a' |x|^2 + (a b' + b a') <x, gamma_0> + b b' |gamma_0|^2
//           + a <g_x, w'> + a' <g_x, w> + b <g_0, w'> + b' <g_0, w> + <w, m'>.
// M acts on the K x M1 x M2 filter space through lag correlations of the
// code maps,
//   (M w)_k(q) = sum_l sum_q' C_kl(q - q') w_l(q'),
//   C_kl(delta) = sum_n sum_s z_k^n(s) z_l^n(s + delta),  |delta_i| < M_i,
// and g_x, g_0 and the inner products of x and gamma_0 are lags of the same
// correlations with x_j and gamma_0,j taken as further maps.  A CG step then
// costs one product with M (K^2 (M1 M2)^2 multiply-adds per channel) in
// place of two passes over the N K H W code spectra; the filters
// d_k = -W_k S Z_k^T gamma = -W_k h_gamma (eq:Learning_Solution) need no
// pass, and gamma itself is formed once, after the last multiplier step.
// The CG iterates are those of the direct form in exact arithmetic.
//
// The correlations come from the float32 spectra of the direct form:
//   C_ab(delta) = 1/D sum_f conj(yhat_a(f)) yhat_b(f) e^{+2 pi i f.delta},
// summed over the rows f1 = 0 .. H/2 with weight 2 on the rows that stand
// for their mirror.  Everything after the spectra runs in float64: the
// expansion of <V, V> cancels (|r|^2 falls far below |x|^2 within a solve),
// which is harmless only when C, g_x, g_0 and the three inner products are
// the lag sums of one fixed set of spectra to float64 rounding.
#include <algorithm>

#include "common.hpp"
#include "internal.hpp"

namespace dcsc {

namespace {

constexpr int kTL = 8;           // maps per tile of the correlation table
constexpr int kNP = kTL * kTL;   // map pairs per tile pair
constexpr int kRF = 64;          // row frequencies per chunk of the row stage
constexpr size_t kRowsLds = size_t(kRF) * (kNP + 1) * 16;  // its R buffer (bytes)
constexpr int kSpanLds = 80 * 1024;  // LDS budget of one product workgroup (bytes): two per CU

// CG scalars per channel: the (a, b) coordinates of gamma (X), r, p, s and
// the previous step's |r|^2 and alpha.
enum { kAX, kBX, kAR, kBR, kAP, kBP, kAS, kBS, kGP, kALP, kNS };
enum { kModeSetup = 0, kModeInit = 1, kModeStep = 2, kModeDrec = 3 };

// Stride (doubles) of one (k, l) lag table, in memory and in the product
// kernel's LDS: at least E1 E2 and = M1 E2 mod 16, so that thread (l, q1) reads row
// entries at E2 (M1 l + q1) + const mod 16, i.e. consecutive threads hit
// distinct 8-byte bank pairs (E2 is odd).
__host__ __device__ constexpr int span_lag_stride(int M1, int M2) {
  const int E2 = 2 * M2 - 1, EE = (2 * M1 - 1) * E2;
  return EE + (((M1 * E2 - EE) % 16) + 16) % 16;
}

// Tile pair index t (A <= B, row-major over the upper triangle) -> (A, B).
__device__ __forceinline__ void tile_pair(int t, int LT, int& A, int& B) {
  A = 0;
  while (t >= LT - A) {
    t -= LT - A;
    ++A;
  }
  B = A + t;
}

// Twiddles of the row stage, T[f2][v] = e^{+2 pi i f2 v / W} for v < 16.
__global__ void l_cc_twiddles(double2* __restrict__ T, int W) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= W * 16) return;
  double s, c;
  sincospi(2.0 * (((i >> 4) * (i & 15)) & (W - 1)) / W, &s, &c);
  T[i] = make_double2(c, s);
}

// Row stage of the correlation table.  Workgroup (row f1, tile pair A <= B)
// forms R_ab(f1, f2) = sum_n conj(yhat_a^n) yhat_b^n for the 64 pairs of the
// tile pair and every f2, then
//   Tr_ab(f1, delta2) = sum_f2 R_ab(f1, f2) e^{+2 pi i f2 delta2 / W}
// for |delta2| < M2 (both signs from one set of products), kRF frequencies
// at a time.  Sum over images: wavefront w holds a 4 x 4 block of pairs, lane
// = frequency, and reads its 8 maps' spectra from memory straight into
// registers (each load of a wavefront is 64 consecutive frequencies), the
// next image's loads in flight while the current one is summed.  Lag sums:
// the chunk's R goes through LDS, lane = pair, wavefront w takes a quarter
// of the chunk's frequencies and all lags, with the twiddles the same for
// every lane (scalar loads); the four partial sums meet in LDS at the end.
template <int L>  // lag slots per pair: M2 <= L, L even
__global__ __launch_bounds__(256) void l_cc_rows(const float2* __restrict__ Zh, const float2* __restrict__ xh,
                                                 const float2* __restrict__ gh, const double2* __restrict__ T,
                                                 double2* __restrict__ Tr, int N, int K, int P, int J, int H, int W,
                                                 int M2, int LT, int NTP) {
  static_assert(L % 2 == 0 && L <= 16, "lag slots");
  static_assert(3 * 4 * (L / 2) * 64 <= 2 * kRF * (kNP + 1), "partial lag sums fit the R buffer");
  extern __shared__ double2 rl[];  // [kRF][kNP + 1]
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int item = xcd_item((int)blockIdx.x, (int)gridDim.x);
  const int f1 = item / NTP, tpi = item % NTP;
  int A, B;
  tile_pair(tpi, LT, A, B);
  const int64_t D = int64_t(H) * W;
  const int fm1 = (H - f1) & (H - 1);
  // The wavefront's maps, as 4 slots of two maps (2s, 2s + 1): slots 0, 1
  // are maps 4 qa .. 4 qa + 3 of tile A, slots 2, 3 maps 4 qb .. of tile B.
  // Code maps come as one pair spectrum and its mirror, x and gamma_0 maps
  // one value each.
  const int qa = wv >> 1, qb = wv & 1;
  const float2* bc[4];
  const float2* bm[4];
  const float2* b1[4];
  int64_t st0[4];
  int kind0[4];  // 0 none, 1 code pair, 2 x or gamma_0
  bool has1[4];
  const int64_t JD = int64_t(J) * D, PD = int64_t(P) * D;
  auto xg_row = [&](int a, int64_t row) -> const float2* {
    return (a < K + J ? xh + (a - K) * D : gh + (a - K - J) * D) + row;
  };
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int a0 = u < 2 ? A * kTL + 4 * qa + 2 * u : B * kTL + 4 * qb + 2 * (u - 2), a1 = a0 + 1;
    bc[u] = bm[u] = b1[u] = Zh;
    st0[u] = 0;
    kind0[u] = a0 < K ? 1 : (a0 < K + 2 * J ? 2 : 0);
    has1[u] = a1 >= K && a1 < K + 2 * J;
    if (kind0[u] == 1) {
      bc[u] = Zh + (a0 >> 1) * D + int64_t(f1) * W;
      bm[u] = Zh + (a0 >> 1) * D + int64_t(fm1) * W;
      st0[u] = PD;
    } else if (kind0[u] == 2) {
      bc[u] = xg_row(a0, int64_t(f1) * W);
      st0[u] = JD;
    }
    if (has1[u]) b1[u] = xg_row(a1, int64_t(f1) * W);
  }
  // A wavefront whose 4 slots are all code pairs sums, per pair of slots
  // (A slot s, B slot t) with spectra C, C' and mirrors Cm, Cm', the four
  // products
  //   S0 = conj(C) C', S1 = conj(C Cm'), S2 = Cm C', S3 = Cm conj(Cm')
  // over the images and forms the slots' four map pairs from them at the
  // end, exactly as the half sums (C + conj(Cm))/2 and -i (C - conj(Cm))/2
  // would give them; the other wavefronts form the maps' values per image
  // (in float64, the same half sums to float64 rounding).
  const bool pure = kind0[0] == 1 && kind0[1] == 1 && kind0[2] == 1 && kind0[3] == 1 && !has1[0] && !has1[1] &&
                    !has1[2] && !has1[3];
  double trc[L], tis[L], trs[L], tic[L];
#pragma unroll
  for (int v = 0; v < L; ++v) trc[v] = tis[v] = trs[v] = tic[v] = 0.0;
  for (int f2c = 0; f2c < W; f2c += kRF) {
    // lanes past W (W < kRF) repeat a frequency; their R is never read
    const int f2 = (f2c + lane) & (W - 1), fn = (W - f2) & (W - 1);
    double2 acc[4][4];  // R of pairs (4 qa + x, 4 qb + z)
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int z = 0; z < 4; ++z) acc[x][z] = make_double2(0.0, 0.0);
    if (pure) {
      double2 S[4][4];  // [2 s + t][product]
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int z = 0; z < 4; ++z) S[x][z] = make_double2(0.0, 0.0);
      // one base per image, advanced by P D, and per-lane byte offsets
      // into it: the loads of the 8 spectra take no address arithmetic
      unsigned oc[4], om[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        oc[u] = (unsigned)((bc[u] - Zh) + f2) * 8u;
        om[u] = (unsigned)((bm[u] - Zh) + fn) * 8u;
      }
      auto load = [&](float2(&lc)[4], float2(&lm)[4], int n) {
        const char* zb = reinterpret_cast<const char*>(Zh + n * PD);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          lc[u] = *reinterpret_cast<const float2*>(zb + oc[u]);
          lm[u] = *reinterpret_cast<const float2*>(zb + om[u]);
        }
      };
      auto mac = [&](const float2(&lc)[4], const float2(&lm)[4]) {
        double2 c[4], m[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          c[u] = make_double2(lc[u].x, lc[u].y);
          m[u] = make_double2(lm[u].x, lm[u].y);
        }
        // float32 values: every product is exact in float64
#pragma unroll
        for (int sa = 0; sa < 2; ++sa)
#pragma unroll
          for (int tb = 0; tb < 2; ++tb) {
            const double2 C = c[sa], Cm = m[sa], D2 = c[2 + tb], Dm = m[2 + tb];
            double2* q = S[2 * sa + tb];
            q[0].x = fma(C.y, D2.y, fma(C.x, D2.x, q[0].x));
            q[0].y = fma(-C.y, D2.x, fma(C.x, D2.y, q[0].y));
            q[1].x = fma(-C.y, Dm.y, fma(C.x, Dm.x, q[1].x));
            q[1].y = fma(-C.y, Dm.x, fma(-C.x, Dm.y, q[1].y));
            q[2].x = fma(-Cm.y, D2.y, fma(Cm.x, D2.x, q[2].x));
            q[2].y = fma(Cm.y, D2.x, fma(Cm.x, D2.y, q[2].y));
            q[3].x = fma(Cm.y, Dm.y, fma(Cm.x, Dm.x, q[3].x));
            q[3].y = fma(-Cm.x, Dm.y, fma(Cm.y, Dm.x, q[3].y));
          }
      };
      // Two named buffers: the next image's loads fly while one is summed.
      // Loads and sums of the loop body are unconditional (the last batch
      // may repeat image N - 1 and go unused): a load whose only use sits
      // under a branch is moved next to it, and the loads then wait.
      float2 la[4], ma[4], lb[4], mb[4];
      load(la, ma, 0);
      int n = 0;
      for (; n + 1 < N; n += 2) {
        load(lb, mb, n + 1);
        mac(la, ma);
        load(la, ma, min(n + 2, N - 1));
        mac(lb, mb);
      }
      if (n < N) mac(la, ma);  // odd N: image N - 1 is in la
      // with a = S0, b = S1, c = S2, d = S3 of slots s, t:
      //   R(2s, 2t) = (a + b + c + d)/4,       R(2s, 2t+1) = -i (a - b + c - d)/4,
      //   R(2s+1, 2t) = i (a + b - c - d)/4,   R(2s+1, 2t+1) = (a - b - c + d)/4
#pragma unroll
      for (int sa = 0; sa < 2; ++sa)
#pragma unroll
        for (int tb = 0; tb < 2; ++tb) {
          const double2* q = S[2 * sa + tb];
          const double2 ab = make_double2(q[0].x + q[1].x, q[0].y + q[1].y);
          const double2 am = make_double2(q[0].x - q[1].x, q[0].y - q[1].y);
          const double2 cd = make_double2(q[2].x + q[3].x, q[2].y + q[3].y);
          const double2 cm = make_double2(q[2].x - q[3].x, q[2].y - q[3].y);
          const double2 r00 = make_double2(ab.x + cd.x, ab.y + cd.y), r11 = make_double2(am.x - cm.x, am.y - cm.y);
          const double2 t01 = make_double2(am.x + cm.x, am.y + cm.y), t10 = make_double2(ab.x - cd.x, ab.y - cd.y);
          acc[2 * sa][2 * tb] = make_double2(0.25 * r00.x, 0.25 * r00.y);
          acc[2 * sa][2 * tb + 1] = make_double2(0.25 * t01.y, -0.25 * t01.x);
          acc[2 * sa + 1][2 * tb] = make_double2(-0.25 * t10.y, 0.25 * t10.x);
          acc[2 * sa + 1][2 * tb + 1] = make_double2(0.25 * r11.x, 0.25 * r11.y);
        }
    } else {
      float2 pc[4], pm[4], p1[4];
      auto issue = [&](int n) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          pc[u] = pm[u] = p1[u] = make_float2(0.f, 0.f);
          if (kind0[u] != 0) pc[u] = bc[u][n * st0[u] + f2];
          if (kind0[u] == 1) pm[u] = bm[u][n * st0[u] + fn];
          if (has1[u]) p1[u] = b1[u][n * JD + f2];
        }
      };
      issue(0);
      for (int n = 0; n < N; ++n) {
        double2 y[8];  // maps 4 qa .. 4 qa + 3 of A, then 4 qb .. 4 qb + 3 of B
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          double2 v0 = make_double2(pc[u].x, pc[u].y), v1 = make_double2(p1[u].x, p1[u].y);
          if (kind0[u] == 1) {
            // zhat_2p = (C + conj(C(-f)))/2, zhat_2p+1 = -i (C - conj(C(-f)))/2
            const double cx = pc[u].x, cy = pc[u].y, mx = pm[u].x, my = pm[u].y;
            v0 = make_double2(0.5 * (cx + mx), 0.5 * (cy - my));
            if (!has1[u]) v1 = make_double2(0.5 * (cy + my), -0.5 * (cx - mx));
          }
          y[2 * u] = v0;
          y[2 * u + 1] = v1;
        }
        if (n + 1 < N) issue(n + 1);
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int z = 0; z < 4; ++z) {
            const double2 a = y[x], b = y[4 + z];
            acc[x][z].x = fma(a.y, b.y, fma(a.x, b.x, acc[x][z].x));
            acc[x][z].y = fma(-a.y, b.x, fma(a.x, b.y, acc[x][z].y));
          }
      }
    }
    __syncthreads();  // the previous chunk's lag sums are done with rl
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int z = 0; z < 4; ++z) rl[lane * (kNP + 1) + (4 * qa + x) * kTL + 4 * qb + z] = acc[x][z];
    __syncthreads();
    const int nf = min(kRF, W - f2c);
    for (int e = 0; e < kRF / 4; ++e) {
      const int fl = wv * (kRF / 4) + e;
      if (fl >= nf) break;
      const double2 r = rl[fl * (kNP + 1) + lane];
      // all L slots: the table has 16 lags per frequency, and a slot past
      // M2 is never written out
      const double2* tf = T + (f2c + fl) * 16;
      double2 c[L];
#pragma unroll
      for (int v = 0; v < L; ++v) c[v] = tf[v];
#pragma unroll
      for (int v = 0; v < L; ++v) {
        trc[v] = fma(r.x, c[v].x, trc[v]);
        tis[v] = fma(r.y, c[v].y, tis[v]);
        trs[v] = fma(r.x, c[v].y, trs[v]);
        tic[v] = fma(r.y, c[v].x, tic[v]);
      }
    }
  }
  // the four wavefronts' partial sums, half of the lag slots at a time
  const int E2 = 2 * M2 - 1;
  double2* out = Tr + ((int64_t(f1) * NTP + tpi) * kNP + lane) * E2;
  double* red = reinterpret_cast<double*>(rl);  // [3][4][L / 2][64]
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    __syncthreads();
    if (wv > 0) {
#pragma unroll
      for (int vl = 0; vl < L / 2; ++vl) {
        const int v = h * (L / 2) + vl;
        double* rp = red + ((wv - 1) * 4 * (L / 2) + vl) * 64 + lane;
        rp[0] = trc[v];
        rp[(L / 2) * 64] = tis[v];
        rp[2 * (L / 2) * 64] = trs[v];
        rp[3 * (L / 2) * 64] = tic[v];
      }
    }
    __syncthreads();
    if (wv == 0) {
#pragma unroll
      for (int vl = 0; vl < L / 2; ++vl) {
        const int v = h * (L / 2) + vl;
        if (v >= M2) continue;
        double sc = trc[v], si = tis[v], ss = trs[v], sk = tic[v];
#pragma unroll
        for (int w = 0; w < 3; ++w) {
          const double* rp = red + (w * 4 * (L / 2) + vl) * 64 + lane;
          sc += rp[0];
          si += rp[(L / 2) * 64];
          ss += rp[2 * (L / 2) * 64];
          sk += rp[3 * (L / 2) * 64];
        }
        // R e^{+i theta} and R e^{-i theta}
        out[M2 - 1 + v] = make_double2(sc - si, ss + sk);
        if (v > 0) out[M2 - 1 - v] = make_double2(sc + si, sk - ss);
      }
    }
  }
}

// Column stage: C_ab(delta1, delta2) = 1/D sum_{f1 = 0}^{H/2} w(f1)
// Re[Tr_ab(f1, delta2) e^{+2 pi i f1 delta1 / H}], w = 1 on rows 0 and H/2,
// 2 elsewhere.  Each (pair, delta2) thread writes where its pair belongs:
// code-code pairs to C (and the mirror C_ba(-delta) = C_ab(delta)), code-x_j
// and code-gamma_0,j pairs on delta >= 0 to g_x and g_0, and the three
// delta = 0 values of x_j and gamma_0,j to s0 = [|x_j|^2, <x_j, gamma_0,j>,
// |gamma_0,j|^2].
__global__ __launch_bounds__(256) void l_cc_lags(const double2* __restrict__ Tr, double* __restrict__ C,
                                                 double* __restrict__ gx, double* __restrict__ g0,
                                                 double* __restrict__ s0, int K, int J, int H, int W, int M1,
                                                 int M2, int LT, int NTP) {
  // 64 (pair, delta2) items per workgroup, the canonical rows split over its
  // four wavefronts (more wavefronts in flight than one thread per item);
  // the partial sums meet in LDS
  __shared__ double2 tw[256];
  __shared__ double red[3][2][8][64];
  const int E2 = 2 * M2 - 1, MM = M1 * M2, EP = span_lag_stride(M1, M2);
  const int per = kNP * E2, bpt = (per + 63) / 64;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int tpi = blockIdx.x / bpt, idx = (blockIdx.x % bpt) * 64 + lane;
  for (int i = threadIdx.x; i < H; i += 256) {
    double s, c;
    sincospi(2.0 * i / H, &s, &c);
    tw[i] = make_double2(c, s);
  }
  __syncthreads();
  int A, B;
  tile_pair(tpi, LT, A, B);
  const int pi = idx / E2, e2 = idx % E2, d2 = e2 - (M2 - 1);
  const int a = A * kTL + (pi >> 3), b = B * kTL + (pi & 7), L = K + 2 * J;
  // what the pair feeds
  int kind = 0, j = 0;  // 1: C, 2: g_x, 3: g_0, 4..6: s0 rows
  if (idx < per && a < L && b < L && !(A == B && a > b)) {
    if (a < K && b < K) kind = 1;
    else if (a < K && b < K + J) kind = 2, j = b - K;
    else if (a < K) kind = 3, j = b - K - J;
    else if (a < K + J && b == a) kind = 4, j = a - K;
    else if (a < K + J && b == a + J) kind = 5, j = a - K;
    else if (a >= K + J && b == a) kind = 6, j = a - K - J;
    if ((kind >= 2 && d2 < 0) || (kind >= 4 && d2 != 0)) kind = 0;
  }
  double sc[16], ss[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) sc[v] = ss[v] = 0.0;
  if (kind != 0) {
    const double2* src = Tr + int64_t(tpi) * kNP * E2 + idx;
    const int64_t rstride = int64_t(NTP) * kNP * E2;
    for (int f1 = wv; f1 <= H / 2; f1 += 4) {
      const double2 t = src[f1 * rstride];
      const double wt = (f1 == 0 || f1 == H / 2) ? 1.0 : 2.0;
      const double tx = wt * t.x, ty = wt * t.y;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        if (v < M1) {
          const double2 c = tw[(f1 * v) & (H - 1)];
          sc[v] += tx * c.x;
          ss[v] += ty * c.y;
        }
      }
    }
  }
  // the four partial sums, eight lags at a time
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (h) __syncthreads();  // wavefront 0 is done with the first half
    if (wv > 0) {
#pragma unroll
      for (int vl = 0; vl < 8; ++vl) {
        red[wv - 1][0][vl][lane] = sc[8 * h + vl];
        red[wv - 1][1][vl][lane] = ss[8 * h + vl];
      }
    }
    __syncthreads();
    if (wv == 0) {
#pragma unroll
      for (int vl = 0; vl < 8; ++vl) {
#pragma unroll
        for (int w = 0; w < 3; ++w) {
          sc[8 * h + vl] += red[w][0][vl][lane];
          ss[8 * h + vl] += red[w][1][vl][lane];
        }
      }
    }
  }
  if (wv > 0 || kind == 0) return;
  const double invD = 1.0 / ((double)H * (double)W);
  if (kind == 1) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      if (v < M1) {
        const double cp = (sc[v] - ss[v]) * invD, cn = (sc[v] + ss[v]) * invD;  // delta1 = +v, -v
        C[(int64_t(a) * K + b) * EP + (M1 - 1 + v) * E2 + e2] = cp;
        if (v > 0) C[(int64_t(a) * K + b) * EP + (M1 - 1 - v) * E2 + e2] = cn;
        if (a != b) {
          C[(int64_t(b) * K + a) * EP + (M1 - 1 - v) * E2 + (E2 - 1 - e2)] = cp;
          if (v > 0) C[(int64_t(b) * K + a) * EP + (M1 - 1 + v) * E2 + (E2 - 1 - e2)] = cn;
        }
      }
    }
  } else if (kind <= 3) {
    double* dst = (kind == 2 ? gx : g0) + (int64_t(j) * K + a) * MM + d2;
#pragma unroll
    for (int v = 0; v < 16; ++v)
      if (v < M1) dst[v * M2] = (sc[v] - ss[v]) * invD;
  } else {
    s0[(kind - 4) * J + j] = (sc[0] - ss[0]) * invD;
  }
}

// dst[(i / seg) * dstride + i % seg] = src[i], i < count, by the workgroup:
// each thread issues its loads 32 at a time before it stores them.
__device__ __forceinline__ void stage_block(double* __restrict__ dst, const double* __restrict__ src, int count,
                                            int seg = 1, int dstride = 1) {
  constexpr int kB = 32;
  const int tid = threadIdx.x, bd = blockDim.x;
  for (int base = 0; base < count; base += kB * bd) {
    double v[kB];
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const int i = base + u * bd + tid;
      v[u] = i < count ? src[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const int i = base + u * bd + tid;
      if (i < count) dst[(i / seg) * dstride + i % seg] = v[u];
    }
  }
}

// Product with M for one (filter k, chunk of LCH input filters l):
//   Mt[k][lc][j][q] = sum_{l in chunk} sum_q' C_kl(q - q') t_l,j(q').
// One thread per (l, j, output row q1): with the support M1 x M2 fixed at
// compile time (MR rows; 0 = M1 known only at run time) the row loop is
// unrolled and every LDS read has a constant offset from the thread's two
// bases.  The chunk's rows are then summed in l order (in the LDS that held
// t).
template <int MR, int M2>
__global__ __launch_bounds__(256) void l_cc_apply(const double* __restrict__ C, const double* __restrict__ t,
                                                  double* __restrict__ Mt, int K, int J, int M1r, int LCH, int LC) {
  extern __shared__ double smem[];
  constexpr int E2 = 2 * M2 - 1;
  const int M1 = MR > 0 ? MR : M1r;
  const int MM = M1 * M2, EP = span_lag_stride(M1, M2);
  const int item = xcd_item((int)blockIdx.x, (int)gridDim.x);
  const int k = item / LC, lc = item % LC;
  const int l0 = lc * LCH, nl = min(LCH, K - l0);
  const int tid = threadIdx.x, bd = blockDim.x;
  double* Cs = smem;                   // [nl][EP]
  double* ts = Cs + LCH * EP;          // [J][LCH][MM], then the row sums [nl][J][MM]
  stage_block(Cs, C + (int64_t(k) * K + l0) * EP, nl * EP);
  for (int j = 0; j < J; ++j) stage_block(ts + j * LCH * MM, t + (int64_t(j) * K + l0) * MM, nl * MM);
  __syncthreads();
  const int ntask = nl * J * M1;
  const int q1 = tid % M1, lj = tid / M1;  // lj = l J + j
  double acc[M2];
#pragma unroll
  for (int q = 0; q < M2; ++q) acc[q] = 0.0;
  if (tid < ntask) {
    const int l = lj / J, j = lj - l * J;
    const double* tl = ts + (j * LCH + l) * MM;
    // output row q1 meets row q1 - q1' + M1 - 1 of C_kl at input row q1'
    const double* cb = Cs + l * EP + (q1 + M1 - 1) * E2;
    auto row = [&](int q1p) {
      double cr[E2], tr[M2];
#pragma unroll
      for (int e = 0; e < E2; ++e) cr[e] = cb[e - q1p * E2];
#pragma unroll
      for (int q = 0; q < M2; ++q) tr[q] = tl[q1p * M2 + q];
#pragma unroll
      for (int q2 = 0; q2 < M2; ++q2)
#pragma unroll
        for (int q2p = 0; q2p < M2; ++q2p) acc[q2] += cr[q2 - q2p + M2 - 1] * tr[q2p];
    };
    if constexpr (MR > 0) {
#pragma unroll
      for (int q1p = 0; q1p < MR; ++q1p) row(q1p);
    } else {
      for (int q1p = 0; q1p < M1; ++q1p) row(q1p);
    }
  }
  __syncthreads();  // every thread is done with ts
  double* red = ts;
  if (tid < ntask) {
#pragma unroll
    for (int q = 0; q < M2; ++q) red[lj * MM + q1 * M2 + q] = acc[q];
  }
  __syncthreads();
  const int JM = J * MM;
  for (int o = tid; o < JM; o += bd) {
    const int j = o / MM, q = o % MM;
    double s = 0.0;
    for (int l = 0; l < nl; ++l) s += red[(l * J + j) * MM + q];
    Mt[((int64_t(k) * LC + lc) * J + j) * MM + q] = s;
  }
}

struct SpanVecs {
  double *Xw, *Xm, *Rw, *Rm, *Pw, *Pm, *Sw, *Sm;
};

template <int J>
__device__ __forceinline__ double pickj(const double (&a)[J], int j) {
  double r = a[0];
#pragma unroll
  for (int i = 1; i < J; ++i)
    if (j == i) r = a[i];
  return r;
}

// Wavefront sum of x, returned to every lane (a fixed order).
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
  return __shfl(x, 0, 64);
}


// The vector updates of one multiplier step, one workgroup per filter k (its
// J x M1 x M2 entries of every vector).  Modes:
//   setup: gamma = gamma_0 (a, b, w, m) = (0, 1, 0, 0); t = W h_gamma; mu64 = mu.
//   init:  r = -x - A gamma from Mt = M t (t = W h_gamma); t = W h_r; dots of r.
//   step:  one CG step in the arrangement of Chronopoulos and Gear (as the
//          direct form): with gamma_r = |r|^2 and delta = <r, A r> =
//          |r|^2 + <h_r, W h_r>, beta = gamma_r / gamma_r', alpha =
//          gamma_r / (delta - beta gamma_r / alpha'); p = r + beta p,
//          s = A r + beta s, gamma += alpha p, r -= alpha s; t = W h_r;
//          dots of the new r.  With `drec` the multiplier step ends here.
//   drec:  d_k = -W_k h_gamma (eq:Learning_Solution), mu_k <- mu_k ||d_k||
//          (kept when the norm is 0, eq:mu_update); with `lastmu`
//          d_k <- d_k / max(1, ||d_k||); t = W h_gamma with the new mu.
// dots[k][4][J] holds the filter's share of <g_x, w_r>, <g_0, w_r>,
// <w_r, m_r> and <h_r, W h_r>; sc the CG scalars [kNS][J]; both are read
// from the previous launch's buffer and written to the other one.  The
// entries' loads are issued before the scalars are reduced; a thread holds
// J entries (J M1 M2 <= 256 J).
template <int J>
__global__ __launch_bounds__(256) void l_cc_update(int mode, int first, int drec, int lastmu,
                                                   const double* __restrict__ s0, const double* __restrict__ gx,
                                                   const double* __restrict__ g0, SpanVecs v, double* __restrict__ t,
                                                   const double* __restrict__ Mt, int LC,
                                                   const double* __restrict__ dots_in, double* __restrict__ dots_out,
                                                   const double* __restrict__ sc_in, double* __restrict__ sc_out,
                                                   double* __restrict__ mu64, float* __restrict__ mu,
                                                   float* __restrict__ d, int K, int MM) {
  constexpr int kUE = J;
  __shared__ double red[4][12];
  __shared__ double bc[2];
  const int k = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int JM = J * MM;
  const bool is_step = mode == kModeStep, is_init = mode == kModeInit;
  // ---- the previous launch's partial dots (step mode): this lane's
  // filters kk = lane, lane + 64, .. in batches of four; the first batch's
  // loads go out here, ahead of the entries', in every mode (dots_in is
  // valid workspace; only the step mode uses the values; a filter past K
  // loads the last one and adds 0)
  double dv[4][4][J];
  auto dots_batch = [&](int k0) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int kk = min(k0 + 64 * b + lane, K - 1);
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int j = 0; j < J; ++j) dv[b][q][j] = dots_in[(int64_t(kk) * 4 + q) * J + j];
    }
  };
  dots_batch(0);
  // ---- loads of this thread's entries
  double rw[kUE], rm[kUE], tv[kUE], mt[kUE], pw[kUE], pm[kUE], sw[kUE], sm[kUE], xw[kUE], xm[kUE], gxv[kUE],
      g0v[kUE];
  int jj[kUE];
  int64_t ii[kUE];
#pragma unroll
  for (int e = 0; e < kUE; ++e) {
    const int o = tid + 256 * e;
    jj[e] = o < JM ? o / MM : 0;
    ii[e] = (int64_t(jj[e]) * K + k) * MM + (o < JM ? o % MM : 0);
    rw[e] = rm[e] = tv[e] = mt[e] = pw[e] = pm[e] = sw[e] = sm[e] = xw[e] = xm[e] = gxv[e] = g0v[e] = 0.0;
    if (o >= JM) continue;
    const int64_t i = ii[e];
    g0v[e] = g0[i];
    if (mode == kModeSetup) continue;
    gxv[e] = gx[i];
    xm[e] = v.Xm[i];
    if (mode == kModeDrec) continue;
    xw[e] = v.Xw[i];
    tv[e] = t[i];
    if (is_step) {
      rw[e] = v.Rw[i];
      rm[e] = v.Rm[i];
      if (!first) {
        pw[e] = v.Pw[i];
        pm[e] = v.Pm[i];
        sw[e] = v.Sw[i];
        sm[e] = v.Sm[i];
      }
    }
    // M t summed over the input-filter chunks in chunk order
    const double* mp = Mt + (int64_t(k) * LC * J + jj[e]) * MM + (o % MM);
    const int64_t ms = int64_t(J) * MM;
    // eight chunks' loads at a time, all in flight together (a chunk past
    // LC loads the last one again and adds 0)
    double acc = 0.0;
    for (int lc = 0; lc < LC; lc += 8) {
      double a8[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) a8[u] = mp[min(lc + u, LC - 1) * ms];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += lc + u < LC ? a8[u] : 0.0;
    }
    mt[e] = acc;
  }
  // ---- scalars
  double sc[kNS][J];
#pragma unroll
  for (int j = 0; j < J; ++j)
#pragma unroll
    for (int f = 0; f < kNS; ++f) sc[f][j] = mode != kModeSetup ? sc_in[f * J + j] : 0.0;
  double al[J], be[J];
#pragma unroll
  for (int j = 0; j < J; ++j) al[j] = be[j] = 0.0;
  if (mode == kModeSetup) {
#pragma unroll
    for (int j = 0; j < J; ++j) sc[kBX][j] = 1.0;
    if (tid == 0) mu64[k] = (double)mu[k];
  } else if (is_init) {
#pragma unroll
    for (int j = 0; j < J; ++j) {
      sc[kAR][j] = -1.0 - sc[kAX][j];
      sc[kBR][j] = -sc[kBX][j];
    }
  } else if (is_step) {
    double ds[4][J];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int j = 0; j < J; ++j) ds[q][j] = 0.0;
    for (int k0 = 0; k0 < K; k0 += 256) {
      if (k0 > 0) dots_batch(k0);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const bool in = k0 + 64 * b + lane < K;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int j = 0; j < J; ++j) ds[q][j] += in ? dv[b][q][j] : 0.0;
      }
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const double a = sc[kAR][j], b = sc[kBR][j];
      const double S1 = wave_sum(ds[0][j]), S2 = wave_sum(ds[1][j]), S3 = wave_sum(ds[2][j]), S4 = wave_sum(ds[3][j]);
      const double gam = a * a * s0[j] + 2.0 * a * b * s0[J + j] + b * b * s0[2 * J + j] + 2.0 * a * S1 + 2.0 * b * S2 + S3;
      const double del = gam + S4;
      const double gp = first ? 0.0 : sc[kGP][j], ap = first ? 0.0 : sc[kALP][j];
      be[j] = gp > 0.0 ? gam / gp : 0.0;
      const double den = ap > 0.0 ? del - be[j] * gam / ap : del;
      al[j] = den > 0.0 ? gam / den : 0.0;
      // p = r + beta p, s = A r + beta s (A r has the coordinates of r)
      sc[kAP][j] = first ? a : a + be[j] * sc[kAP][j];
      sc[kBP][j] = first ? b : b + be[j] * sc[kBP][j];
      sc[kAS][j] = first ? a : a + be[j] * sc[kAS][j];
      sc[kBS][j] = first ? b : b + be[j] * sc[kBS][j];
      sc[kAX][j] += al[j] * sc[kAP][j];
      sc[kBX][j] += al[j] * sc[kBP][j];
      sc[kAR][j] = a - al[j] * sc[kAS][j];
      sc[kBR][j] = b - al[j] * sc[kBS][j];
      sc[kGP][j] = gam;
      sc[kALP][j] = al[j];
    }
  }
  const double wk = 0.5 / (mode == kModeSetup ? (double)mu[k] : mu64[k]);
  const bool with_dots = is_init || (is_step && !drec);
  double part[4][J];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int j = 0; j < J; ++j) part[q][j] = 0.0;
  // ---- updates
#pragma unroll
  for (int e = 0; e < kUE; ++e) {
    const int o = tid + 256 * e;
    if (o >= JM) continue;
    const int j = jj[e];
    const int64_t i = ii[e];
    if (mode == kModeSetup) {
      v.Xw[i] = 0.0;
      v.Xm[i] = 0.0;
      t[i] = wk * g0v[e];
      continue;
    }
    if (mode == kModeDrec) continue;
    double nrw, nrm;
    if (is_init) {
      nrw = -(xw[e] + tv[e]);
      nrm = -(xm[e] + mt[e]);
    } else {
      const double bej = pickj<J>(be, j), alj = pickj<J>(al, j);
      const double aw = rw[e] + tv[e], am = rm[e] + mt[e];  // A r
      double qpw = rw[e], qpm = rm[e], qsw = aw, qsm = am;
      if (!first) {
        qpw += bej * pw[e];
        qpm += bej * pm[e];
        qsw += bej * sw[e];
        qsm += bej * sm[e];
      }
      v.Pw[i] = qpw;
      v.Pm[i] = qpm;
      v.Sw[i] = qsw;
      v.Sm[i] = qsm;
      xw[e] += alj * qpw;
      xm[e] += alj * qpm;
      v.Xw[i] = xw[e];
      v.Xm[i] = xm[e];
      nrw = rw[e] - alj * qsw;
      nrm = rm[e] - alj * qsm;
    }
    v.Rw[i] = nrw;
    v.Rm[i] = nrm;
    if (!drec) {
      const double h = pickj<J>(sc[kAR], j) * gxv[e] + pickj<J>(sc[kBR], j) * g0v[e] + nrm, tn = wk * h;
      t[i] = tn;
#pragma unroll
      for (int q = 0; q < J; ++q) {
        if (q == j) {
          part[0][q] += gxv[e] * nrw;
          part[1][q] += g0v[e] * nrw;
          part[2][q] += nrw * nrm;
          part[3][q] += h * tn;
        }
      }
    }
  }
  if (with_dots) {
    // per-wavefront sums, then the four wavefronts in order
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const double w = wave_sum(part[q][j]);
        if (lane == 0) red[wid][q * 3 + j] = w;
      }
    __syncthreads();
    if (tid < 4 * J) {
      const int q = tid / J, j = tid % J;
      double tot = 0.0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += red[w][q * 3 + j];
      dots_out[(int64_t(k) * 4 + q) * J + j] = tot;
    }
  }
  if (drec || mode == kModeDrec) {
    double nn = 0.0, hv[kUE];
#pragma unroll
    for (int e = 0; e < kUE; ++e) {
      const int o = tid + 256 * e;
      hv[e] = 0.0;
      if (o >= JM) continue;
      const int j = jj[e];
      hv[e] = pickj<J>(sc[kAX], j) * gxv[e] + pickj<J>(sc[kBX], j) * g0v[e] + xm[e];
      const double dv = -wk * hv[e];
      nn += dv * dv;
    }
    const double tot = block_sum(nn, &red[0][0]);
    if (tid == 0) {
      const double nrm = sqrt(tot);
      const double mnew = nrm > 0.0 ? mu64[k] * nrm : mu64[k];
      mu64[k] = mnew;
      mu[k] = (float)mnew;
      bc[0] = nrm;
      bc[1] = mnew;
    }
    __syncthreads();
    const double nrm = bc[0], scale = lastmu ? 1.0 / fmax(1.0, nrm) : 1.0, wn = 0.5 / bc[1];
#pragma unroll
    for (int e = 0; e < kUE; ++e) {
      const int o = tid + 256 * e;
      if (o >= JM) continue;
      d[(int64_t(k) * J + jj[e]) * MM + (o % MM)] = (float)(-wk * hv[e] * scale);
      t[ii[e]] = wn * hv[e];
    }
  }
  if (k == 0 && tid == 0) {
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
      for (int f = 0; f < kNS; ++f) sc_out[f * J + j] = sc[f][j];
  }
}

// v = a_gamma xhat + b_gamma gamma_0hat over the full grids (the part of the
// final gamma outside Z S^T w).
__global__ void l_cc_vhat(const float2* __restrict__ xh, const float2* __restrict__ gh, float2* __restrict__ out,
                          const double* __restrict__ sc, int J, int64_t D) {
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int nj = blockIdx.y, j = nj % J;
  if (f >= D) return;
  const float a = (float)sc[kAX * J + j], b = (float)sc[kBX * J + j];
  const int64_t o = int64_t(nj) * D + f;
  const float2 x = xh[o], g = gh[o];
  out[o] = make_float2(a * x.x + b * g.x, a * x.y + b * g.y);
}

// U_k(f) = sum_m w_k(m) e^{-2 pi i f.m / D} at the canonical rows
// f1 = 0 .. H/2 (index f1 W + f2), written as one half (k = 2p: .x .y,
// k = 2p + 1: .z .w) of the pair-unpacked float4 table of pass B.  Four
// workgroups per (filter, channel), each forming the row DFT of the M1 rows
// of taps and a quarter of the column sums.
__global__ __launch_bounds__(256) void l_cc_uc(const double* __restrict__ Xw, float4* __restrict__ Uc, int K, int P,
                                               int J, int H, int W, int M1, int M2) {
  __shared__ float2 cs[16 * 256];
  __shared__ double2 twh[256], tww[256];
  __shared__ double wk[16 * 16];
  const int k = blockIdx.x, j = blockIdx.y, tid = threadIdx.x;
  const int MM = M1 * M2, nc = (H / 2 + 1) * W;
  for (int i = tid; i < MM; i += 256) wk[i] = Xw[(int64_t(j) * K + k) * MM + i];
  for (int i = tid; i < 256; i += 256) {
    double s, c;
    if (i < H) {
      sincospi(-2.0 * i / H, &s, &c);
      twh[i] = make_double2(c, s);
    }
    if (i < W) {
      sincospi(-2.0 * i / W, &s, &c);
      tww[i] = make_double2(c, s);
    }
  }
  __syncthreads();
  for (int e = tid; e < M1 * W; e += 256) {
    const int m1 = e / W, f2 = e % W;
    double re = 0.0, im = 0.0;
    for (int m2 = 0; m2 < M2; ++m2) {
      const double x = wk[m1 * M2 + m2];
      const double2 c = tww[(f2 * m2) & (W - 1)];
      re += x * c.x;
      im += x * c.y;
    }
    cs[m1 * W + f2] = make_float2((float)re, (float)im);
  }
  __syncthreads();
  float2* out = reinterpret_cast<float2*>(Uc + (int64_t(j) * P + (k >> 1)) * nc) + (k & 1);
  // the column stage's outputs are shared by the gridDim.z workgroups of
  // this (k, j), 256 at a time (each forms the small row stage itself)
  for (int i = blockIdx.z * 256 + tid; i < nc; i += 256 * gridDim.z) {
    const int f1 = i / W, f2 = i % W;
    double re = 0.0, im = 0.0;
    for (int m1 = 0; m1 < M1; ++m1) {
      const float2 a = cs[m1 * W + f2];
      const double2 c = twh[(f1 * m1) & (H - 1)];
      re += a.x * c.x - a.y * c.y;
      im += a.x * c.y + a.y * c.x;
    }
    out[2 * int64_t(i)] = make_float2((float)re, (float)im);
  }
}

// the odd filter slot of the last pair when K is odd
__global__ void l_cc_uc_zero(float4* __restrict__ Uc, int P, int nc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  if (i < nc) {
    float4* u = Uc + (int64_t(j) * P + (P - 1)) * nc + i;
    u->z = 0.f;
    u->w = 0.f;
  }
}

#define LJ_SPAN(KERNEL, J, grid, block, st, ...)                                            \
  do {                                                                                     \
    if ((J) == 1) hipLaunchKernelGGL(KERNEL<1>, grid, block, 0, st, __VA_ARGS__);          \
    else if ((J) == 2) hipLaunchKernelGGL(KERNEL<2>, grid, block, 0, st, __VA_ARGS__);     \
    else hipLaunchKernelGGL(KERNEL<3>, grid, block, 0, st, __VA_ARGS__);                   \
  } while (0)

struct SpanDims {
  int K, J, M1, M2, E1, E2, EE, MM, L, LT, NTP, Hc, LCH, LC, apply_threads;
};

SpanDims span_dims(const Plan& pl) {
  SpanDims s;
  s.K = pl.k;
  s.J = pl.j;
  s.M1 = pl.fs[1];
  s.M2 = pl.fs[2];
  s.E1 = 2 * s.M1 - 1;
  s.E2 = 2 * s.M2 - 1;
  s.EE = s.E1 * s.E2;
  s.MM = s.M1 * s.M2;
  s.L = s.K + 2 * s.J;
  s.LT = (s.L + kTL - 1) / kTL;
  s.NTP = s.LT * (s.LT + 1) / 2;
  s.Hc = pl.g[1] / 2 + 1;
  // a product workgroup holds LCH input filters: one thread per (l, j, row)
  const int per_l = (span_lag_stride(s.M1, s.M2) + s.J * s.MM) * (int)sizeof(double);
  s.LCH = std::max(1, std::min(s.K, std::min(kSpanLds / per_l, 256 / (s.J * s.M1))));
  s.LC = (s.K + s.LCH - 1) / s.LCH;
  s.apply_threads = std::min(256, 64 * ((s.LCH * s.J * s.M1 + 63) / 64));
  return s;
}

struct SpanWs {
  double2 *Tr, *T;
  double *C, *gx, *g0, *s0, *t, *Mt, *dots, *sc, *mu64;
  SpanVecs v;
};

size_t carve_span(const Plan& pl, void* base, SpanWs* w) {
  const SpanDims s = span_dims(pl);
  Carver c(base);
  const int64_t JKM = int64_t(s.J) * s.K * s.MM;
  w->Tr = c.take<double2>(int64_t(s.Hc) * s.NTP * kNP * s.E2);
  w->T = c.take<double2>(int64_t(pl.g[2]) * 16);
  w->C = c.take<double>(int64_t(s.K) * s.K * span_lag_stride(s.M1, s.M2));
  w->gx = c.take<double>(JKM);
  w->g0 = c.take<double>(JKM);
  w->s0 = c.take<double>(3 * s.J);
  double** vec[8] = {&w->v.Xw, &w->v.Xm, &w->v.Rw, &w->v.Rm, &w->v.Pw, &w->v.Pm, &w->v.Sw, &w->v.Sm};
  for (double** p : vec) *p = c.take<double>(JKM);
  w->t = c.take<double>(JKM);
  w->Mt = c.take<double>(int64_t(s.K) * s.LC * s.J * s.MM);
  w->dots = c.take<double>(2 * int64_t(s.K) * 4 * s.J);
  w->sc = c.take<double>(2 * kNS * s.J);
  w->mu64 = c.take<double>(s.K);
  return c.off;
}

}  // namespace

bool span_eligible(const Plan& pl) {
  const int H = pl.g[1], W = pl.g[2];
  if (pl.g[0] != 1 || H < 2 || W < 2 || H > 256 || W > 256) return false;
  if (pl.fs[1] < 1 || pl.fs[2] < 1 || pl.fs[1] > 16 || pl.fs[2] > 16 || pl.fs[1] > H || pl.fs[2] > W) return false;
  const SpanDims s = span_dims(pl);
  // the correlation tables stay below 2 GiB each, and one image's code
  // spectra below 4 GiB (the row stage addresses them with 32-bit offsets)
  const double tr = double(s.Hc) * s.NTP * kNP * s.E2 * 16.0, cc = double(s.K) * s.K * s.EE * 8.0;
  return tr < 2147483648.0 && cc < 2147483648.0 && double(pl.p) * H * W * 8.0 < 4294967296.0;
}

// Modelled time of one learning call in each form (seconds), with rates
// measured on the benchmark's call: the direct form streams the code
// spectra twice per CG step (about 4 TB/s on cache-resident sets) plus ~15 us
// of small launches; the span form builds the correlation table once (about
// 13e12 float64 multiply-adds/s counted as below, ~70 us for the column
// stage) and then costs one product with M (about 6e12 multiply-adds/s) and
// ~7 us per step.
bool span_preferred(const Plan& pl, int inner_iters, int cg_iters) {
  const SpanDims s = span_dims(pl);
  const double steps = double(inner_iters) * (cg_iters + 1);
  const double D = double(pl.g[1]) * pl.g[2];
  const double direct = steps * (2.0 * pl.n * pl.p * D * 8.0 / 4e12 + 15e-6);
  const double table = double(s.Hc) * pl.g[2] * s.NTP * kNP * (pl.n + s.M2) * 4.0 / 13e12 + 70e-6;
  const double span = table + steps * (double(s.J) * s.K * s.K * s.MM * s.MM / 6e12 + 7e-6);
  return span < direct;
}

size_t span_ws_bytes(const Plan& pl) {
  SpanWs w;
  return carve_span(pl, nullptr, &w);
}

hipError_t run_span(const Plan& pl, const float2* Zh, const float2* xh, const float2* gh, float2* vout, float4* Uc,
                    float* d, float* mu, int inner_iters, int cg_iters, void* span_ws, hipStream_t st) {
  SpanWs w;
  carve_span(pl, span_ws, &w);
  const SpanDims s = span_dims(pl);
  const int N = pl.n, H = pl.g[1], W = pl.g[2];
  hipLaunchKernelGGL(l_cc_twiddles, dim3((unsigned)((W * 16 + 255) / 256)), dim3(256), 0, st, w.T, W);
  {
    TraceScope trace(kTraceLearnSpanRows, st, true);
    hipEvent_t e0, e1;
    const bool tr = trace.events(&e0, &e1);
    const dim3 grid((unsigned)(s.NTP * s.Hc)), block(256);
#define SPAN_ROWS(L)                                                                                               \
  {                                                                                                                \
    static bool attr_set = false;                                                                                 \
    if (!attr_set) {                                                                                              \
      hipFuncSetAttribute(reinterpret_cast<const void*>(&l_cc_rows<L>), hipFuncAttributeMaxDynamicSharedMemorySize, \
                          (int)kRowsLds);                                                                         \
      attr_set = true;                                                                                            \
    }                                                                                                             \
    if (tr)                                                                                                       \
      hipExtLaunchKernelGGL(l_cc_rows<L>, grid, block, kRowsLds, st, e0, e1, 0, Zh, xh, gh, w.T, w.Tr, N, s.K,      \
                            pl.p, s.J, H, W, s.M2, s.LT, s.NTP);                                                 \
    else                                                                                                          \
      hipLaunchKernelGGL(l_cc_rows<L>, grid, block, kRowsLds, st, Zh, xh, gh, w.T, w.Tr, N, s.K, pl.p, s.J, H, W,   \
                         s.M2, s.LT, s.NTP);                                                                      \
  }
    switch ((s.M2 + 1) / 2) {
      case 1: SPAN_ROWS(2) break;
      case 2: SPAN_ROWS(4) break;
      case 3: SPAN_ROWS(6) break;
      case 4: SPAN_ROWS(8) break;
      case 5: SPAN_ROWS(10) break;
      case 6: SPAN_ROWS(12) break;
      case 7: SPAN_ROWS(14) break;
      default: SPAN_ROWS(16) break;
    }
#undef SPAN_ROWS
  }
  const int bpt = (kNP * s.E2 + 63) / 64;
  hipLaunchKernelGGL(l_cc_lags, dim3((unsigned)(s.NTP * bpt)), dim3(256), 0, st, w.Tr, w.C, w.gx, w.g0, w.s0, s.K,
                     s.J, H, W, s.M1, s.M2, s.LT, s.NTP);
  const size_t lds = size_t(s.LCH) * (span_lag_stride(s.M1, s.M2) + s.J * s.MM) * sizeof(double);
  auto apply = [&]() {
    TraceScope trace(kTraceLearnSpanApply, st, true);
    hipEvent_t e0, e1;
    const bool tr = trace.events(&e0, &e1);
    const dim3 grid((unsigned)(s.K * s.LC)), block((unsigned)s.apply_threads);
#define SPAN_APPLY_K(MR, M)                                                                                        \
  {                                                                                                                \
    static bool attr_set = false;                                                                                 \
    if (!attr_set) {                                                                                              \
      hipFuncSetAttribute(reinterpret_cast<const void*>(&l_cc_apply<MR, M>),                                       \
                          hipFuncAttributeMaxDynamicSharedMemorySize, kSpanLds);                                  \
      attr_set = true;                                                                                            \
    }                                                                                                             \
    if (tr)                                                                                                       \
      hipExtLaunchKernelGGL((l_cc_apply<MR, M>), grid, block, lds, st, e0, e1, 0, w.C, w.t, w.Mt, s.K, s.J, s.M1,  \
                            s.LCH, s.LC);                                                                         \
    else                                                                                                          \
      hipLaunchKernelGGL((l_cc_apply<MR, M>), grid, block, lds, st, w.C, w.t, w.Mt, s.K, s.J, s.M1, s.LCH, s.LC); \
  }
#define SPAN_APPLY(M)                   \
  case M:                               \
    if (s.M1 == M) SPAN_APPLY_K(M, M)   \
    else SPAN_APPLY_K(0, M)             \
    break;
    switch (s.M2) {
      SPAN_APPLY(1) SPAN_APPLY(2) SPAN_APPLY(3) SPAN_APPLY(4) SPAN_APPLY(5) SPAN_APPLY(6) SPAN_APPLY(7)
      SPAN_APPLY(8) SPAN_APPLY(9) SPAN_APPLY(10) SPAN_APPLY(11) SPAN_APPLY(12) SPAN_APPLY(13) SPAN_APPLY(14)
      SPAN_APPLY(15) SPAN_APPLY(16)
      default: break;
    }
#undef SPAN_APPLY_K
#undef SPAN_APPLY
  };
  int par = 0;
  auto update = [&](int mode, int first, int drec, int lastmu) {
    const int64_t dstride = int64_t(s.K) * 4 * s.J, sstride = int64_t(kNS) * s.J;
    LJ_SPAN(l_cc_update, s.J, dim3((unsigned)s.K), dim3(256), st, mode, first, drec, lastmu, w.s0, w.gx, w.g0, w.v,
            w.t, w.Mt, s.LC, w.dots + par * dstride, w.dots + (par ^ 1) * dstride, w.sc + par * sstride,
            w.sc + (par ^ 1) * sstride, w.mu64, mu, d, s.K, s.MM);
    par ^= 1;
  };
  update(kModeSetup, 0, 0, 0);
  for (int it = 0; it < inner_iters; ++it) {
    const int lastmu = it == inner_iters - 1 ? 1 : 0;
    if (cg_iters == 0) {
      update(kModeDrec, 0, 0, lastmu);
      continue;
    }
    apply();
    update(kModeInit, 0, 0, 0);
    for (int q = 0; q < cg_iters; ++q) {
      apply();
      update(kModeStep, q == 0 ? 1 : 0, q == cg_iters - 1 ? 1 : 0, lastmu);
    }
  }
  // gamma = a x + b gamma_0 + Z S^T w: the first two terms here, the last
  // through pass B
  const int64_t D = pl.dsz;
  hipLaunchKernelGGL(l_cc_vhat, dim3((unsigned)((D + 255) / 256), (unsigned)(N * s.J)), dim3(256), 0, st, xh, gh,
                     vout, w.sc + par * int64_t(kNS) * s.J, s.J, D);
  hipLaunchKernelGGL(l_cc_uc, dim3((unsigned)s.K, (unsigned)s.J, 4u), dim3(256), 0, st, w.v.Xw, Uc, s.K, pl.p, s.J, H, W,
                     s.M1, s.M2);
  if (s.K & 1) {
    const int nc = s.Hc * W;
    hipLaunchKernelGGL(l_cc_uc_zero, dim3((unsigned)((nc + 255) / 256), (unsigned)s.J), dim3(256), 0, st, Uc, pl.p,
                       nc);
  }
  return hipGetLastError();
}

}  // namespace dcsc
