// Batched coding of many images of uneven sizes (one call, shared filters).
//
// Images are grouped by padded grid (grid class); each class has the plan,
// workspace and per-image offset tables of the single-grid solver, so the
// codes stay in the caller's packed buffers.  After each class's set-up
// (spectra, first lam), every ADMM iteration of every class runs from five
// persistent launches, each over one work list that spans all classes (the
// coding problem separates over images, Sec. 3.1):
//   tiles     fused single-tile items (class, image, pair group)
//   rows_inv  split-path inverse row items (class, image, pair, row chunk)
//   cols      split-path column items (class, image, pair, column block)
//   rows_fwd  split-path forward row items (class, image, pair group, rows)
//   spec      spectral reduce + next dual solve (class, image, 256 freqs)
// The items are the device functions of the single-grid kernels (tiles.hpp)
// with each class's own grouping, so every image's codes are bit for bit
// those of the single-grid solver on its class.  A launch has as many
// workgroups as fit on the chip at once; the items of each class are split
// into eight contiguous chunks, chunk x of every class going to the
// workgroups of XCD x (workgroup x mod 8), which take them from a counter of
// their own XCD (relaxed atomics: items of one launch are independent).  The
// whole call can be captured once into a hipGraph and replayed; the
// pairs-per-workgroup grouping of each tile class comes from a measured
// search (csc_batch_autotune) or a heuristic.
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "internal.hpp"
#include "tiles.hpp"

namespace dcsc {

size_t run_code_ws(const Plan& pl);

constexpr int kChunk = 32;
constexpr int kXcds = 8;     // XCDs of the chip: workgroup i runs on XCD i mod 8
struct OffChunk {
  int64_t v[kChunk];
};

__global__ void k_set_table(int64_t* __restrict__ dst, OffChunk c, int count) {
  if ((int)threadIdx.x < count) dst[threadIdx.x] = c.v[threadIdx.x];
}

__global__ void k_fill_rho(float* __restrict__ dst, int n, float v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = v;
}

struct BatchClass {
  int h = 0, w = 0;
  std::vector<int> imgs;
  Plan pl;
  size_t off_tables = 0, off_rho = 0, off_ws = 0, ws_bytes = 0;
};

struct BatchPlan {
  int n = 0, k = 0, fs[2] = {0, 0};
  std::vector<BatchClass> cls;
  size_t off_ctr = 0;  // work-list counters: two sets of 8 (one per XCD), used alternately
  size_t total = 0;
};

static size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

static int plan_batch(const csc_batch* bt, BatchPlan* bp) {
  if (!bt || bt->abi_version != CSC_ABI_VERSION || bt->n < 1 || bt->k < 1) return CSC_EINVAL;
  if (!bt->grid || !bt->b_off || !bt->z_off) return CSC_EINVAL;
  bp->n = bt->n;
  bp->k = bt->k;
  bp->fs[0] = bt->fsupp[0];
  bp->fs[1] = bt->fsupp[1];
  std::map<std::pair<int, int>, std::vector<int>> groups;
  for (int i = 0; i < bt->n; ++i) {
    const int h = bt->grid[2 * i], w = bt->grid[2 * i + 1];
    if (bt->b_off[i] < 0 || bt->z_off[i] < 0) return CSC_EINVAL;
    groups[{h, w}].push_back(i);
  }
  size_t off = 0;
  int ci = 0;
  for (auto& kv : groups) {
    BatchClass c;
    c.h = kv.first.first;
    c.w = kv.first.second;
    c.imgs = kv.second;
    csc_shape s;
    memset(&s, 0, sizeof(s));
    s.abi_version = CSC_ABI_VERSION;
    s.n = (int)c.imgs.size();
    s.j = 1;
    s.k = bt->k;
    s.ndim = 2;
    s.grid[0] = c.h;
    s.grid[1] = c.w;
    s.fsupp[0] = bt->fsupp[0];
    s.fsupp[1] = bt->fsupp[1];
    const int rc = make_plan(&s, &c.pl);
    if (rc != CSC_OK) return rc;
    if (bt->ppg && bt->ppg[ci] > 0) set_grouping(&c.pl, bt->ppg[ci]);
    c.off_tables = off;
    off = align256(off + 2 * sizeof(int64_t) * c.imgs.size());
    c.off_rho = off;
    off = align256(off + sizeof(float) * c.imgs.size());
    c.off_ws = off;
    c.ws_bytes = run_code_ws(c.pl);
    off = align256(off + c.ws_bytes);
    bp->cls.push_back(c);
    ++ci;
  }
  bp->off_ctr = off;
  bp->total = align256(off + 2 * kXcds * sizeof(int));
  return CSC_OK;
}

static void upload_table(int64_t* dst, const std::vector<int64_t>& v, hipStream_t st) {
  for (size_t i = 0; i < v.size(); i += kChunk) {
    OffChunk c;
    const int cnt = (int)std::min<size_t>(kChunk, v.size() - i);
    for (int t = 0; t < cnt; ++t) c.v[t] = v[i + t];
    hipLaunchKernelGGL(k_set_table, dim3(1), dim3(kChunk), 0, st, dst + i, c, cnt);
  }
}

// ------------------------------------------------------- work lists

constexpr int kMaxCls = 24;  // grid classes per launch (every supported grid fits)

struct ItemCls {
  int h, w, n, p, ppg, ng;
  int items;  // items of the class in this launch
  const float2* E;
  const float2* G;
  const float2* xh;
  float2* yh;
  float2* Th;
  float2* lam;
  float2* part;
  float2* buf;
  double* rpart;
  double* rdual;
  const float* rho;
  const int64_t* zoff;
};

struct ItemLaunch {
  int ncls, k, solve_next;
  float beta;
  float* z;
  int* ctr;       // this launch's kXcds counters (zero at its start)
  int* ctr_next;  // the other set, zeroed here for the next launch
  ItemCls c[kMaxCls];
};

// The q-th item of XCD x's share: chunk x of class 0, then of class 1, ...
// Returns false past the end of the share.
__device__ __forceinline__ bool xcd_share_item(const ItemLaunch& L, int x, int q, int& cls, int& local) {
  for (int c = 0; c < L.ncls; ++c) {
    const int n = L.c[c].items;
    const int lo = (int)((int64_t(n) * x) / kXcds), hi = (int)((int64_t(n) * (x + 1)) / kXcds);
    if (q < hi - lo) {
      cls = c;
      local = lo + q;
      return true;
    }
    q -= hi - lo;
  }
  return false;
}

// Launches alternate between two counter sets: each one zeroes the set the
// next launch uses (the launch before it, which used that set, has ended).
__device__ __forceinline__ void clear_next_counters(const ItemLaunch& L) {
  if (blockIdx.x == 0 && threadIdx.x < kXcds) L.ctr_next[threadIdx.x] = 0;
}

// Next item of this workgroup's XCD; -1 when its share is done.
__device__ __forceinline__ int next_item(const ItemLaunch& L, int* slot, int& cls, int& local) {
  __syncthreads();  // the previous item's readers of *slot are done
  if (threadIdx.x == 0) *slot = atomicAdd(L.ctr + blockIdx.x % kXcds, 1);
  __syncthreads();
  const int q = *slot;
  return xcd_share_item(L, (int)(blockIdx.x % kXcds), q, cls, local) ? q : -1;
}

// Largest padded tile of the fused kernel over the supported grids.
constexpr int kTileLds = 256 * (64 + 64 / 8 + 1);
static_assert(kTileLds >= 128 * (128 + 128 / 8 + 1) && kTileLds >= 64 * (256 + 256 / 8 + 1), "tile LDS");

__global__ __launch_bounds__(1024) void kb_tiles(ItemLaunch L) {
  clear_next_counters(L);
  __shared__ float2 tile[kTileLds];
  __shared__ float2 tw[256];
  __shared__ double red[1024 / 64];
  __shared__ int slot;
  load_twiddles(tw);
  int c, local;
  while (next_item(L, &slot, c, local) >= 0) {
    const ItemCls& C = L.c[c];
    const int n = local % C.n, g = local / C.n;
#define TI(HH, WW)                                                                                                \
  if (C.h == HH && C.w == WW) {                                                                                   \
    fused_item<HH, WW, 1, kModeIter, 1024>(tile, tw, red, n, g, C.E, C.lam, L.z, nullptr, C.zoff, C.rho, L.beta,  \
                                           C.part, C.rpart, L.k, C.p, C.ppg, C.ng);                               \
    continue;                                                                                                     \
  }
    TI(16, 16) TI(16, 32) TI(16, 64) TI(16, 128) TI(16, 256)
    TI(32, 16) TI(32, 32) TI(32, 64) TI(32, 128) TI(32, 256)
    TI(64, 16) TI(64, 32) TI(64, 64) TI(64, 128) TI(64, 256)
    TI(128, 16) TI(128, 32) TI(128, 64) TI(128, 128)
    TI(256, 16) TI(256, 32) TI(256, 64)
#undef TI
  }
}

// the split path's tiles: rows x W (W = 128, 256) or H x columns
constexpr int kRowsLds = (kSplitT / 128) * (128 + 128 / 8 + 1);
constexpr int kColsLds = 256 * (16 + 16 / 8 + 1);
static_assert(kRowsLds >= (kSplitT / 256) * (256 + 256 / 8 + 1), "rows LDS");
static_assert(kColsLds >= 128 * (32 + 32 / 8 + 1), "cols LDS");

__global__ __launch_bounds__(kSplitNT) void kb_rows_inv(ItemLaunch L) {
  clear_next_counters(L);
  __shared__ float2 tile[kRowsLds];
  __shared__ float2 tw[256];
  __shared__ int slot;
  load_twiddles(tw);
  int c, local;
  while (next_item(L, &slot, c, local) >= 0) {
    const ItemCls& C = L.c[c];
    const int n = local % C.n, p = (local / C.n) % C.p, rc = local / C.n / C.p;
    if (C.w == 256) rows_inv_item<256, 1>(tile, tw, n, p, rc, C.E, C.lam, C.buf, C.p, C.h);
    else rows_inv_item<128, 1>(tile, tw, n, p, rc, C.E, C.lam, C.buf, C.p, C.h);
  }
}

__global__ __launch_bounds__(kSplitNT) void kb_cols(ItemLaunch L) {
  clear_next_counters(L);
  __shared__ float2 tile[kColsLds];
  __shared__ float2 tw[256];
  __shared__ double red[kSplitNT / 64];
  __shared__ int slot;
  load_twiddles(tw);
  int c, local;
  while (next_item(L, &slot, c, local) >= 0) {
    const ItemCls& C = L.c[c];
    const int ncb = C.w / (kSplitT / C.h);
    const int cb = local % ncb, p = (local / ncb) % C.p, n = local / ncb / C.p;
    if (C.h == 256)
      cols_item<256, 0>(tile, tw, red, n, p, cb, ncb, C.buf, L.z, nullptr, nullptr, C.zoff, C.rho, L.beta, C.rpart,
                        L.k, C.p, C.w);
    else
      cols_item<128, 0>(tile, tw, red, n, p, cb, ncb, C.buf, L.z, nullptr, nullptr, C.zoff, C.rho, L.beta, C.rpart,
                        L.k, C.p, C.w);
  }
}

__global__ __launch_bounds__(kSplitNT) void kb_rows_fwd(ItemLaunch L) {
  clear_next_counters(L);
  __shared__ float2 tile[kRowsLds];
  __shared__ float2 tw[256];
  __shared__ int slot;
  load_twiddles(tw);
  int c, local;
  while (next_item(L, &slot, c, local) >= 0) {
    const ItemCls& C = L.c[c];
    const int n = local % C.n, gi = (local / C.n) % C.ng, rc = local / C.n / C.ng;
    if (C.w == 256) rows_fwd_item<256, 1>(tile, tw, n, gi, rc, C.E, C.buf, C.part, C.p, C.h, C.ppg, C.ng);
    else rows_fwd_item<128, 1>(tile, tw, n, gi, rc, C.E, C.buf, C.part, C.p, C.h, C.ppg, C.ng);
  }
}

__global__ __launch_bounds__(kSpecT) void kb_spec(ItemLaunch L) {
  clear_next_counters(L);
  __shared__ double red[kSpecT / 64];
  __shared__ int slot;
  int c, local;
  while (next_item(L, &slot, c, local) >= 0) {
    const ItemCls& C = L.c[c];
    const int nblk = (C.h * C.w + kSpecT - 1) / kSpecT;
    // the accumulator count of the plain solver's choice for this class
    // (k_spec or k_spec_wide), so the batch equals it bit for bit
    if (C.ng > 8)
      spec_item<1, 16>(red, local % nblk, local / nblk, nblk, C.part, C.G, C.xh, C.yh, C.Th, C.lam, C.rho, C.rdual,
                       C.ng, 1, C.h, C.w, L.solve_next);
    else
      spec_item<1, 8>(red, local % nblk, local / nblk, nblk, C.part, C.G, C.xh, C.yh, C.Th, C.lam, C.rho, C.rdual,
                      C.ng, 1, C.h, C.w, L.solve_next);
  }
}

__global__ void k_zero_ints(int* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Resident workgroups of each launch (occupancy bound by LDS or threads).
static int device_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
  }
  return cus;
}

// Per-class tables, rho and plan with its offset tables.
static Plan class_setup(const BatchClass& c, const csc_batch* bt, float rho, char* ws, hipStream_t st) {
  const int nc = (int)c.imgs.size();
  int64_t* boff = reinterpret_cast<int64_t*>(ws + c.off_tables);
  int64_t* zoff = boff + nc;
  std::vector<int64_t> bo(nc), zo(nc);
  for (int i = 0; i < nc; ++i) {
    bo[i] = bt->b_off[c.imgs[i]];
    zo[i] = bt->z_off[c.imgs[i]];
  }
  upload_table(boff, bo, st);
  upload_table(zoff, zo, st);
  float* rho_c = reinterpret_cast<float*>(ws + c.off_rho);
  hipLaunchKernelGGL(k_fill_rho, dim3((nc + 255) / 256), dim3(256), 0, st, rho_c, nc, rho);
  Plan pl = c.pl;
  pl.boff = boff;
  pl.zoff = zoff;
  return pl;
}

// One class alone through the single-grid solver (the autotuner's timing).
static int enqueue_class(const BatchClass& c, const csc_batch* bt, const float* b, const float* d, float beta,
                         float rho, int iters, unsigned flags, float* z, char* ws, hipStream_t st) {
  const Plan pl = class_setup(c, bt, rho, ws, st);
  float* rho_c = reinterpret_cast<float*>(ws + c.off_rho);
  return run_code(pl, b, d, beta, rho_c, iters, flags & CSC_Z_ZERO, z, nullptr, nullptr, ws + c.off_ws, st);
}

// The whole batch: each class's set-up, then per iteration the five launches
// over the work lists of all classes.
static int enqueue_batch(const BatchPlan& bp, const csc_batch* bt, const float* b, const float* d, float beta,
                         float rho, int iters, unsigned flags, float* z, char* ws, hipStream_t st) {
  const int ncls = (int)bp.cls.size();
  ItemLaunch tiles{}, split{}, spec{};
  for (ItemLaunch* L : {&tiles, &split, &spec}) {
    L->k = bp.k;
    L->beta = beta;
    L->z = z;
  }
  std::vector<Plan> plans(ncls);
  for (int ci = 0; ci < ncls; ++ci) {
    const BatchClass& c = bp.cls[ci];
    plans[ci] = class_setup(c, bt, rho, ws, st);
    const Plan& pl = plans[ci];
    CodeWs w;
    carve_code(pl, ws + c.off_ws, &w);
    const float* rho_c = reinterpret_cast<const float*>(ws + c.off_rho);  // filled by class_setup
    if (code_prepare(pl, b, d, rho_c, flags & CSC_Z_ZERO, z, nullptr, iters > 0, w, st) != hipSuccess)
      return CSC_EHIP;
    ItemCls ic{};
    ic.h = c.h;
    ic.w = c.w;
    ic.n = pl.n;
    ic.p = pl.p;
    ic.ppg = pl.ppg;
    ic.ng = pl.ng;
    ic.E = w.E;
    ic.G = w.G;
    ic.xh = w.xh;
    ic.yh = w.yh;
    ic.Th = w.Th;
    ic.lam = w.lam;
    ic.part = w.part;
    ic.buf = w.buf;
    ic.rpart = w.rpri;
    ic.rdual = w.rdual;
    ic.rho = w.rho;
    ic.zoff = pl.zoff;
    if (pl.lds) {
      if (tiles.ncls >= kMaxCls) return CSC_EUNSUPPORTED;
      tiles.c[tiles.ncls++] = ic;
    } else if (pl.split) {
      if (split.ncls >= kMaxCls) return CSC_EUNSUPPORTED;
      split.c[split.ncls++] = ic;
    } else {
      return CSC_EUNSUPPORTED;
    }
    ic.items = pl.n * (int)((pl.dsz + kSpecT - 1) / kSpecT);
    spec.c[spec.ncls++] = ic;
  }
  for (int i = 0; i < tiles.ncls; ++i) tiles.c[i].items = tiles.c[i].n * tiles.c[i].ng;
  int* ctr = reinterpret_cast<int*>(ws + bp.off_ctr);
  hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, st, ctr, kXcds);
  int launch = 0;
  auto counters = [&](ItemLaunch& L) {
    L.ctr = ctr + (launch & 1) * kXcds;
    L.ctr_next = ctr + ((launch + 1) & 1) * kXcds;
    ++launch;
  };
  const int cus = device_cus();
  // workgroups of a launch: as many as fit at once (cap), at most one per
  // item, and a multiple of 8 (at least 8) so that every XCD share has some
  auto grid_for = [](const ItemLaunch& L, int64_t cap) {
    int64_t t = 0;
    for (int i = 0; i < L.ncls; ++i) t += L.c[i].items;
    const int64_t g = (std::min(t, cap) + kXcds - 1) / kXcds * kXcds;
    return dim3((unsigned)std::max<int64_t>(g, kXcds));
  };
  ItemLaunch ri = split, co = split, rf = split;
  for (int i = 0; i < split.ncls; ++i) {
    const ItemCls& C = split.c[i];
    const int rows = C.h / (kSplitT / C.w), cols = C.w / (kSplitT / C.h);
    ri.c[i].items = C.n * C.p * rows;
    co.c[i].items = C.n * C.p * cols;
    rf.c[i].items = C.n * C.ng * rows;
  }
  for (int it = 0; it < iters; ++it) {
    if (tiles.ncls) {
      counters(tiles);
      hipLaunchKernelGGL(kb_tiles, grid_for(tiles, cus), dim3(1024), 0, st, tiles);
    }
    if (split.ncls) {
      counters(ri);
      hipLaunchKernelGGL(kb_rows_inv, grid_for(ri, 4 * cus), dim3(kSplitNT), 0, st, ri);
      counters(co);
      hipLaunchKernelGGL(kb_cols, grid_for(co, 4 * cus), dim3(kSplitNT), 0, st, co);
      counters(rf);
      hipLaunchKernelGGL(kb_rows_fwd, grid_for(rf, 4 * cus), dim3(kSplitNT), 0, st, rf);
    }
    counters(spec);
    spec.solve_next = it < iters - 1 ? 1 : 0;
    hipLaunchKernelGGL(kb_spec, grid_for(spec, 8 * cus), dim3(kSpecT), 0, st, spec);
  }
  return hipGetLastError() == hipSuccess ? CSC_OK : CSC_EHIP;
}

struct BatchCall {
  const BatchPlan* bp;
  const csc_batch* bt;
  const float *b, *d;
  float beta, rho;
  int iters;
  unsigned flags;
  float* z;
  char* ws;
  hipStream_t st;
};

static int enqueue_batch_ctx(void* p) {
  BatchCall* c = static_cast<BatchCall*>(p);
  return enqueue_batch(*c->bp, c->bt, c->b, c->d, c->beta, c->rho, c->iters, c->flags, c->z, c->ws, c->st);
}

static std::vector<int64_t> batch_key(const csc_batch* bt, const float* b, const float* d, float beta, float rho,
                                      int iters, unsigned flags, float* z, void* ws, size_t ws_bytes,
                                      hipStream_t st) {
  int dev = 0;
  hipGetDevice(&dev);
  uint32_t bb, rr;
  memcpy(&bb, &beta, 4);
  memcpy(&rr, &rho, 4);
  std::vector<int64_t> k = {3, dev, (int64_t)(uintptr_t)b, (int64_t)(uintptr_t)d, (int64_t)(uintptr_t)z,
                            (int64_t)(uintptr_t)ws, (int64_t)ws_bytes, (int64_t)(uintptr_t)st, bb, rr, iters,
                            (int64_t)flags, bt->n, bt->k, bt->fsupp[0], bt->fsupp[1]};
  for (int i = 0; i < bt->n; ++i) {
    k.push_back(bt->grid[2 * i]);
    k.push_back(bt->grid[2 * i + 1]);
    k.push_back(bt->b_off[i]);
    k.push_back(bt->z_off[i]);
  }
  if (bt->ppg) {
    // one entry per class
    int ncls = 0;
    {
      BatchPlan tmp;
      if (plan_batch(bt, &tmp) == CSC_OK) ncls = (int)tmp.cls.size();
    }
    for (int c = 0; c < ncls; ++c) k.push_back(bt->ppg[c]);
  } else {
    k.push_back(-1);
  }
  return k;
}

}  // namespace dcsc

using namespace dcsc;

extern "C" {

size_t csc_batch_workspace_bytes(const csc_batch* batch) {
  BatchPlan bp;
  if (plan_batch(batch, &bp) != CSC_OK) return 0;
  return bp.total;
}

int csc_batch_classes(const csc_batch* batch, int32_t* grids, int32_t* counts, int max_classes) {
  BatchPlan bp;
  const int rc = plan_batch(batch, &bp);
  if (rc != CSC_OK) return rc;
  const int nc = (int)bp.cls.size();
  for (int i = 0; i < nc && i < max_classes; ++i) {
    if (grids) {
      grids[2 * i] = bp.cls[i].h;
      grids[2 * i + 1] = bp.cls[i].w;
    }
    if (counts) counts[i] = (int32_t)bp.cls[i].imgs.size();
  }
  return nc;
}

int csc_code_batched(const csc_batch* batch, const float* b, const float* d, float beta, float rho, int iters,
                     unsigned flags, float* z, void* ws, size_t ws_bytes, void* stream) {
  BatchPlan bp;
  int rc = plan_batch(batch, &bp);
  if (rc != CSC_OK) return rc;
  if (!b || !d || !z || iters < 0 || !(beta >= 0.0f) || !(rho > 0.0f)) return CSC_EINVAL;
  if (flags & ~(CSC_Z_ZERO | CSC_USE_GRAPH)) return CSC_EINVAL;
  if (!ws || ws_bytes < bp.total || (reinterpret_cast<uintptr_t>(ws) & 255u) != 0) return CSC_EWORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!(flags & CSC_USE_GRAPH) || st == nullptr)
    return enqueue_batch(bp, batch, b, d, beta, rho, iters, flags, z, static_cast<char*>(ws), st);
  BatchCall call{&bp, batch, b, d, beta, rho, iters, flags & ~CSC_USE_GRAPH, z, static_cast<char*>(ws), st};
  return graph_call(batch_key(batch, b, d, beta, rho, iters, flags, z, ws, ws_bytes, st), st, enqueue_batch_ctx,
                    &call);
}

int csc_batch_autotune(const csc_batch* batch, const float* b, const float* d, float beta, float rho, int iters,
                       float* z, void* ws, size_t ws_bytes, void* stream, int32_t* ppg_out, int max_classes) {
  BatchPlan bp;
  int rc = plan_batch(batch, &bp);
  if (rc != CSC_OK) return rc;
  if (!b || !d || !z || !ppg_out || iters < 1 || !(beta >= 0.0f) || !(rho > 0.0f)) return CSC_EINVAL;
  if ((int)bp.cls.size() > max_classes) return CSC_EINVAL;
  if (!ws || ws_bytes < bp.total || (reinterpret_cast<uintptr_t>(ws) & 255u) != 0) return CSC_EWORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return CSC_EHIP;
  static const int cand[] = {1, 2, 3, 4, 6, 8, 12, 16};
  for (int ci = 0; ci < (int)bp.cls.size(); ++ci) {
    BatchClass& c = bp.cls[ci];
    ppg_out[ci] = c.pl.ppg;
    if (!c.pl.lds && !c.pl.split) continue;
    float best = 1e30f;
    for (int cv : cand) {
      if (cv > c.pl.p) break;
      // the class alone, laid out from the start of the batch's workspace
      // with this grouping (fewer pairs per group need more partial
      // spectra); a grouping that does not fit is not tried
      BatchClass solo = c;
      set_grouping(&solo.pl, cv);
      const size_t nc = solo.imgs.size();
      solo.off_tables = 0;
      solo.off_rho = align256(2 * sizeof(int64_t) * nc);
      solo.off_ws = align256(solo.off_rho + sizeof(float) * nc);
      solo.ws_bytes = run_code_ws(solo.pl);
      if (solo.off_ws + solo.ws_bytes > ws_bytes) continue;
      // warm-up then timed run of this class alone
      rc = enqueue_class(solo, batch, b, d, beta, rho, iters, CSC_Z_ZERO, z, static_cast<char*>(ws), st);
      if (rc != CSC_OK) break;
      hipEventRecord(e0, st);
      rc = enqueue_class(solo, batch, b, d, beta, rho, iters, CSC_Z_ZERO, z, static_cast<char*>(ws), st);
      hipEventRecord(e1, st);
      if (rc != CSC_OK || hipEventSynchronize(e1) != hipSuccess) {
        rc = rc != CSC_OK ? rc : CSC_EHIP;
        break;
      }
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      if (ms < best) {
        best = ms;
        ppg_out[ci] = cv;
      }
    }
    if (rc != CSC_OK) break;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return rc;
}

}  // extern "C"
