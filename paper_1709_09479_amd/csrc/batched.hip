// Batched coding of many images of uneven sizes (one call, shared filters).
//
// Images are grouped by padded grid (grid class).  Each class runs the
// single-grid coding pipeline (fused single-tile kernel where the grid fits
// LDS, axis-pass FFTs otherwise) directly on the caller's packed buffers
// through per-image offset tables, so nothing is gathered or scattered.  The
// whole call -- per-class set-up spectra and every ADMM iteration of every
// class -- can be captured once into a hipGraph and replayed; the
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

namespace dcsc {

size_t run_code_ws(const Plan& pl);

constexpr int kChunk = 32;
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
  bp->total = off;
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

// Enqueue class `c` (or all classes when c < 0).
static int enqueue_batch(const BatchPlan& bp, const csc_batch* bt, const float* b, const float* d, float beta,
                         float rho, int iters, unsigned flags, float* z, char* ws, hipStream_t st, int only = -1) {
  for (int ci = 0; ci < (int)bp.cls.size(); ++ci) {
    if (only >= 0 && ci != only) continue;
    const BatchClass& c = bp.cls[ci];
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
    const int rc = run_code(pl, b, d, beta, rho_c, iters, flags & CSC_Z_ZERO, z, nullptr, nullptr, ws + c.off_ws, st);
    if (rc != CSC_OK) return rc;
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
      set_grouping(&c.pl, cv);
      // warm-up then timed run of this class alone
      rc = enqueue_batch(bp, batch, b, d, beta, rho, iters, CSC_Z_ZERO, z, static_cast<char*>(ws), st, ci);
      if (rc != CSC_OK) break;
      hipEventRecord(e0, st);
      rc = enqueue_batch(bp, batch, b, d, beta, rho, iters, CSC_Z_ZERO, z, static_cast<char*>(ws), st, ci);
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
