// C ABI entry points: argument validation (before anything is enqueued),
// planning, workspace sizing and dispatch to the coding / learning paths.
#include <string.h>

#include <map>
#include <cmath>
#include <mutex>
#include <vector>

#include "internal.hpp"

namespace dcsc {

size_t run_code_ws(const Plan& pl);
int run_objective(const Plan& pl, const float* b, const float* d, const float* z, float beta, double* out, void* ws,
                  hipStream_t st);
int run_learn(const Plan& pl, const float* b, const float* z, float* d, float* mu, float* gamma, int inner_iters,
              int cg_iters, unsigned flags, void* ws, hipStream_t st, float cg_tol = 0.0f,
              int* cg_counts = nullptr);
size_t run_learn_ws(const Plan& pl);
size_t run_diff_ws(const Plan& pl, int every);
int run_unrolled(const Plan& pl, const float* b, const float* d, float beta, const float* rho, int iters, int every,
                 float* z, float* ckpt, void* ws, hipStream_t st);
int run_backward(const Plan& pl, const float* b, const float* d, float beta, const float* rho, int iters, int every,
                 const float* ckpt, const float* zbar_in, float* dd, double* dbeta, void* ws, hipStream_t st);
int run_loss_grad(const Plan& pl, const float* b, const float* d, const float* z, float beta, double* loss,
                  float* zbar, float* dd, double* dbeta, void* ws, hipStream_t st);

static bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Resident workgroups per CU for a single-tile kernel of d complex elements
// (LDS bound: one tile of 8 bytes per element plus row padding).
static int tile_occupancy(int64_t d) {
  if (d >= 16384) return 1;
  if (d >= 8192) return 2;
  if (d >= 4096) return 4;
  return 8;
}

void set_grouping(Plan* p, int ppg_override) {
  if (!p->lds && !p->split) {
    p->ppg = 1;
    p->ng = 1;
    return;
  }
  int64_t ppg = ppg_override;
  if (ppg <= 0) {
    // fused: one workgroup per (group, image); split: row-phase workgroups
    // per (row chunk, group, image), about four resident per CU
    const int64_t units = int64_t(p->n) * p->p * (p->split ? split_row_blocks(*p) : 1);
    const int64_t slots = 256LL * (p->split ? 4 : tile_occupancy(p->dsz));
    ppg = (units + slots / 2) / slots;
  }
  if (ppg < 1) ppg = 1;
  if (ppg > p->p) ppg = p->p;
  p->ppg = (int)ppg;
  p->ng = (p->p + p->ppg - 1) / p->ppg;
}

int make_plan(const csc_shape* s, Plan* pl) {
  if (!s || s->abi_version != CSC_ABI_VERSION) return CSC_EINVAL;
  if (s->n < 1 || s->k < 1 || s->j < 1 || s->j > 3) return CSC_EINVAL;
  if (s->ndim != 2 && s->ndim != 3) return CSC_EINVAL;
  Plan p;
  p.n = s->n;
  p.j = s->j;
  p.k = s->k;
  p.p = (s->k + 1) / 2;
  p.nd = s->ndim;
  const int off = 3 - s->ndim;
  for (int a = 0; a < s->ndim; ++a) {
    p.g[off + a] = s->grid[a];
    p.fs[off + a] = s->fsupp[a];
  }
  for (int a = 0; a < 3; ++a) {
    if (!pow2(p.g[a])) return CSC_EINVAL;
    if (p.fs[a] < 1 || p.fs[a] > p.g[a]) return CSC_EINVAL;
  }
  if (p.g[1] < 8 || p.g[1] > 256 || p.g[2] < 8 || p.g[2] > 256) return CSC_EUNSUPPORTED;
  if (s->ndim == 3 && (p.g[0] < 2 || p.g[0] > 64)) return CSC_EUNSUPPORTED;
  p.dsz = int64_t(p.g[0]) * p.g[1] * p.g[2];
  p.msz = int64_t(p.fs[0]) * p.fs[1] * p.fs[2];
  p.lds = (p.g[0] == 1) && tile_supported(p.g[1], p.g[2]);
  p.split = !p.lds && split_supported(p.g[0], p.g[1], p.g[2]);
  p.vol = !p.lds && !p.split && vol_supported(p.g[0], p.g[1], p.g[2]);
  set_grouping(&p, 0);
  *pl = p;
  return CSC_OK;
}

int make_plan_flags(const csc_shape* s, unsigned flags, Plan* pl) {
  int rc = make_plan(s, pl);
  if (rc != CSC_OK) return rc;
  if (flags & CSC_NUCLEAR) {
    if (!nuclear_supported(pl->g[0], pl->g[1], pl->g[2])) return CSC_EUNSUPPORTED;
    // every map goes through the axis-by-axis transforms and the per-map
    // thresholding kernel
    pl->nuclear = true;
    pl->lds = false;
    pl->split = false;
    pl->ng = pl->ppg = 1;
  }
  return CSC_OK;
}

// Geometry the DCT-domain variant covers: 2-D, single-tile grids, filter
// quadrants of at most 16 x 16 taps.
static bool dct_plan_ok(const Plan& pl) {
  return pl.nd == 2 && dct_supported(pl.g[0], pl.g[1], pl.g[2]) && pl.fs[1] <= 16 && pl.fs[2] <= 16;
}

static int check_ws(void* ws, size_t have, size_t need) {
  if (need == 0) return CSC_OK;
  if (!ws || have < need || (reinterpret_cast<uintptr_t>(ws) & 255u) != 0) return CSC_EWORKSPACE;
  return CSC_OK;
}

// ------------------------------------------------------------ hipGraphs

namespace {
std::mutex g_graph_mu;
std::map<std::vector<int64_t>, hipGraphExec_t> g_graph_cache;
}  // namespace

int graph_call(const std::vector<int64_t>& key, hipStream_t st, int (*enqueue)(void*), void* ctx) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  auto it = g_graph_cache.find(key);
  if (it == g_graph_cache.end()) {
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return CSC_EHIP;
    const int rc = enqueue(ctx);
    const hipError_t ec = hipStreamEndCapture(st, &graph);
    if (rc != CSC_OK || ec != hipSuccess) {
      if (graph) hipGraphDestroy(graph);
      return rc != CSC_OK ? rc : CSC_EHIP;
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (ei != hipSuccess) return CSC_EHIP;
    if (g_graph_cache.size() >= 32) {
      hipGraphExecDestroy(g_graph_cache.begin()->second);
      g_graph_cache.erase(g_graph_cache.begin());
    }
    it = g_graph_cache.emplace(key, exec).first;
  }
  return hipGraphLaunch(it->second, st) == hipSuccess ? CSC_OK : CSC_EHIP;
}

static int64_t fbits(float v) {
  uint32_t u;
  memcpy(&u, &v, 4);
  return u;
}
static int64_t pbits(const void* p) { return (int64_t)(uintptr_t)p; }

static void shape_key(std::vector<int64_t>& k, const csc_shape* s) {
  int dev = 0;
  hipGetDevice(&dev);
  k.insert(k.end(), {dev, s->n, s->j, s->k, s->ndim, s->grid[0], s->grid[1], s->grid[2], s->fsupp[0], s->fsupp[1],
                     s->fsupp[2]});
}

// ------------------------------------------------------------- tracing

namespace {
constexpr int kTraceSlots = 8192;
std::mutex g_trace_mu;
bool g_trace_on = false;
int g_trace_every = 1;           // bracket every n-th launch of each class
int g_cls_seen[kTraceClasses];   // launches seen per class since enabling
std::vector<hipEvent_t> g_ev_start, g_ev_stop;
std::vector<int> g_ev_cls;
int g_ev_used = 0;
}  // namespace

TraceScope::TraceScope(int cls, hipStream_t st, bool own_launch)
    : cls_(cls), st_(st), slot_(-1), own_(own_launch) {
  std::lock_guard<std::mutex> lk(g_trace_mu);
  if (!g_trace_on || g_ev_used >= kTraceSlots) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st_, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  if (g_cls_seen[cls]++ % g_trace_every != 0) return;
  slot_ = g_ev_used++;
  g_ev_cls[slot_] = cls;
  if (!own_) hipEventRecord(g_ev_start[slot_], st_);
}

TraceScope::~TraceScope() {
  if (slot_ >= 0 && !own_) hipEventRecord(g_ev_stop[slot_], st_);
}

bool TraceScope::events(hipEvent_t* start, hipEvent_t* stop) const {
  if (slot_ < 0 || !own_) return false;
  std::lock_guard<std::mutex> lk(g_trace_mu);
  *start = g_ev_start[slot_];
  *stop = g_ev_stop[slot_];
  return true;
}

}  // namespace dcsc

// Scratch of csc_code_noalloc: one static array on every device the library
// runs on.  In host code `scratch` names a host-side stand-in, so the array's
// device address is looked up once per device (with that device current) and
// only that address is ever handed to kernels.
__device__ __align__(256) char scratch[CSC_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return CSC_EHIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return CSC_EHIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return CSC_OK;
}
}  // namespace

using namespace dcsc;

extern "C" {

int csc_abi_version(void) { return CSC_ABI_VERSION; }

int csc_check_finite(const float* x, int64_t n, int* flag, void* stream) {
  if (!flag || n < 0 || (n > 0 && !x)) return CSC_EINVAL;
  return launch_check_finite(x, n, flag, static_cast<hipStream_t>(stream)) == hipSuccess ? CSC_OK : CSC_EHIP;
}

int csc_trace_enable(int on) {
  if (on < 0) return CSC_EINVAL;
  std::lock_guard<std::mutex> lk(g_trace_mu);
  if (on && g_ev_start.empty()) {
    g_ev_start.resize(kTraceSlots);
    g_ev_stop.resize(kTraceSlots);
    g_ev_cls.resize(kTraceSlots);
    for (int i = 0; i < kTraceSlots; ++i) {
      if (hipEventCreate(&g_ev_start[i]) != hipSuccess || hipEventCreate(&g_ev_stop[i]) != hipSuccess) {
        g_ev_start.clear();
        g_ev_stop.clear();
        return CSC_EHIP;
      }
    }
  }
  g_trace_on = on != 0;
  if (on) {
    g_ev_used = 0;
    g_trace_every = on;
    for (int c = 0; c < kTraceClasses; ++c) g_cls_seen[c] = 0;
  }
  return CSC_OK;
}

int csc_trace_read(int cls, double* total_ms, int* count) {
  if (!total_ms || !count || cls < 0 || cls >= kTraceClasses) return CSC_EINVAL;
  std::lock_guard<std::mutex> lk(g_trace_mu);
  double tot = 0.0;
  int cnt = 0;
  for (int i = 0; i < g_ev_used; ++i) {
    if (g_ev_cls[i] != cls) continue;
    if (hipEventSynchronize(g_ev_stop[i]) != hipSuccess) return CSC_EHIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, g_ev_start[i], g_ev_stop[i]) != hipSuccess) return CSC_EHIP;
    tot += ms;
    ++cnt;
  }
  *total_ms = tot;
  *count = cnt;
  return CSC_OK;
}

const char* csc_strerror(int code) {
  switch (code) {
    case CSC_OK: return "success";
    case CSC_EINVAL: return "invalid argument or shape";
    case CSC_EWORKSPACE: return "workspace missing, too small or not 256-byte aligned";
    case CSC_EUNSUPPORTED: return "geometry not supported";
    case CSC_EHIP: return "HIP runtime error";
    case CSC_ENONFINITE: return "non-finite value (NaN or infinity) in a result";
    case CSC_ESCRATCH: return "problem needs more scratch than csc_code_noalloc's static array holds (64 MiB)";
    default: return "unknown error";
  }
}

size_t csc_workspace_bytes(const csc_shape* shape, int op, unsigned flags) {
  Plan pl;
  if (make_plan_flags(shape, op == CSC_OP_LEARN ? 0u : (flags & CSC_NUCLEAR), &pl) != CSC_OK) return 0;
  switch (op) {
    case CSC_OP_CODE:
    case CSC_OP_OBJECTIVE: return run_code_ws(pl);
    case CSC_OP_LEARN: return run_learn_ws(pl);
    case CSC_OP_DCT: return dct_plan_ok(pl) ? dct_ws_bytes(pl) : 0;
    default: return 0;
  }
}

int csc_code(const csc_shape* shape, const float* b, const float* d, float beta, float* rho, int iters,
             unsigned flags, float* z, float* theta, double* resid, void* ws, size_t ws_bytes, void* stream) {
  Plan pl;
  if (flags & ~(CSC_ADAPTIVE_RHO | CSC_Z_ZERO | CSC_THETA_ZERO | CSC_USE_GRAPH | CSC_NUCLEAR)) return CSC_EINVAL;
  int rc = make_plan_flags(shape, flags, &pl);
  if (rc != CSC_OK) return rc;
  if (!b || !d || !rho || !z || iters < 0 || !(beta >= 0.0f)) return CSC_EINVAL;
  if ((rc = check_ws(ws, ws_bytes, run_code_ws(pl))) != CSC_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const unsigned f = flags & ~(CSC_USE_GRAPH | CSC_NUCLEAR);
  if (!(flags & CSC_USE_GRAPH) || st == nullptr)
    return run_code(pl, b, d, beta, rho, iters, f, z, theta, resid, ws, st);
  struct Ctx {
    Plan* pl;
    const float *b, *d;
    float beta;
    float* rho;
    int iters;
    unsigned f;
    float *z, *theta;
    double* resid;
    void* ws;
    hipStream_t st;
  } c{&pl, b, d, beta, rho, iters, f, z, theta, resid, ws, st};
  std::vector<int64_t> key{1};
  shape_key(key, shape);
  key.insert(key.end(), {pbits(b), pbits(d), fbits(beta), pbits(rho), iters, (int64_t)flags, pbits(z), pbits(theta),
                         pbits(resid), pbits(ws), (int64_t)ws_bytes, pbits(st)});
  return graph_call(key, st,
                    [](void* p) -> int {
                      Ctx* c = static_cast<Ctx*>(p);
                      return run_code(*c->pl, c->b, c->d, c->beta, c->rho, c->iters, c->f, c->z, c->theta, c->resid,
                                      c->ws, c->st);
                    },
                    &c);
}

int csc_code_noalloc(const csc_shape* shape, const float* b, const float* d, float beta, float* rho, int iters,
                     unsigned flags, float* z, float* theta, double* resid, void* stream) {
  Plan pl;
  if (flags & ~(CSC_ADAPTIVE_RHO | CSC_Z_ZERO | CSC_THETA_ZERO | CSC_NUCLEAR)) return CSC_EINVAL;
  int rc = make_plan_flags(shape, flags, &pl);
  if (rc != CSC_OK) return rc;
  if (!b || !d || !rho || !z || iters < 0 || !(beta >= 0.0f)) return CSC_EINVAL;
  if (run_code_ws(pl) > CSC_NOALLOC_SCRATCH_BYTES) return CSC_ESCRATCH;
  void* ws = nullptr;
  if ((rc = scratch_address(&ws)) != CSC_OK) return rc;
  return run_code(pl, b, d, beta, rho, iters, flags & ~CSC_NUCLEAR, z, theta, resid, ws,
                  static_cast<hipStream_t>(stream));
}

int csc_learn(const csc_shape* shape, const float* b, const float* z, float* d, float* mu, float* gamma,
              int inner_iters, int cg_iters, unsigned flags, void* ws, size_t ws_bytes, void* stream) {
  Plan pl;
  int rc = make_plan(shape, &pl);
  if (rc != CSC_OK) return rc;
  if (!b || !z || !d || !mu || !gamma || inner_iters < 1 || cg_iters < 0) return CSC_EINVAL;
  if (flags & ~(CSC_GAMMA_ZERO | CSC_USE_GRAPH | CSC_LEARN_DIRECT | CSC_LEARN_SPAN)) return CSC_EINVAL;
  if ((flags & CSC_LEARN_DIRECT) && (flags & CSC_LEARN_SPAN)) return CSC_EINVAL;
  if ((rc = check_ws(ws, ws_bytes, run_learn_ws(pl))) != CSC_OK) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const unsigned f = flags & ~CSC_USE_GRAPH;
  if (!(flags & CSC_USE_GRAPH) || st == nullptr)
    return run_learn(pl, b, z, d, mu, gamma, inner_iters, cg_iters, f, ws, st);
  struct Ctx {
    Plan* pl;
    const float *b, *z;
    float *d, *mu, *gamma;
    int li, ci;
    unsigned f;
    void* ws;
    hipStream_t st;
  } c{&pl, b, z, d, mu, gamma, inner_iters, cg_iters, f, ws, st};
  std::vector<int64_t> key{2};
  shape_key(key, shape);
  key.insert(key.end(), {pbits(b), pbits(z), pbits(d), pbits(mu), pbits(gamma), inner_iters, cg_iters, (int64_t)f,
                         pbits(ws), (int64_t)ws_bytes, pbits(st)});
  return graph_call(key, st,
                    [](void* p) -> int {
                      Ctx* c = static_cast<Ctx*>(p);
                      return run_learn(*c->pl, c->b, c->z, c->d, c->mu, c->gamma, c->li, c->ci, c->f, c->ws, c->st);
                    },
                    &c);
}

int csc_code_tol(const csc_shape* shape, const float* b, const float* d, float beta, float* rho, int max_iters,
                 float tol, unsigned flags, float* z, float* theta, double* resid, int* iters_done, void* ws,
                 size_t ws_bytes, void* stream) {
  Plan pl;
  if (flags & ~(CSC_ADAPTIVE_RHO | CSC_Z_ZERO | CSC_THETA_ZERO | CSC_NUCLEAR)) return CSC_EINVAL;
  int rc = make_plan_flags(shape, flags, &pl);
  if (rc != CSC_OK) return rc;
  if (!b || !d || !rho || !z || max_iters < 0 || !(beta >= 0.0f) || !(tol > 0.0f) || !std::isfinite(tol))
    return CSC_EINVAL;
  if ((rc = check_ws(ws, ws_bytes, run_code_ws(pl))) != CSC_OK) return rc;
  return run_code(pl, b, d, beta, rho, max_iters, flags & ~CSC_NUCLEAR, z, theta, resid, ws,
                  static_cast<hipStream_t>(stream), tol, iters_done);
}

int csc_learn_tol(const csc_shape* shape, const float* b, const float* z, float* d, float* mu, float* gamma,
                  int inner_iters, int max_cg, float cg_tol, unsigned flags, int* cg_counts, void* ws,
                  size_t ws_bytes, void* stream) {
  Plan pl;
  int rc = make_plan(shape, &pl);
  if (rc != CSC_OK) return rc;
  if (!b || !z || !d || !mu || !gamma || inner_iters < 1 || max_cg < 0 || !(cg_tol >= 0.0f) ||
      !std::isfinite(cg_tol))
    return CSC_EINVAL;
  if (flags & ~CSC_GAMMA_ZERO) return CSC_EINVAL;
  if ((rc = check_ws(ws, ws_bytes, run_learn_ws(pl))) != CSC_OK) return rc;
  return run_learn(pl, b, z, d, mu, gamma, inner_iters, max_cg, flags, ws, static_cast<hipStream_t>(stream), cg_tol,
                   cg_counts);
}

int64_t csc_unrolled_record_floats(const csc_shape* shape) {
  Plan pl;
  if (make_plan(shape, &pl) != CSC_OK || pl.j != 1) return 0;
  return code_record_floats(pl);
}

size_t csc_unrolled_workspace_bytes(const csc_shape* shape, int every) {
  Plan pl;
  if (make_plan(shape, &pl) != CSC_OK || pl.j != 1 || every < 1) return 0;
  return run_diff_ws(pl, every);
}

static int diff_plan(const csc_shape* shape, Plan* pl) {
  int rc = make_plan(shape, pl);
  if (rc != CSC_OK) return rc;
  return pl->j == 1 ? CSC_OK : CSC_EUNSUPPORTED;
}

int csc_code_unrolled(const csc_shape* shape, const float* b, const float* d, float beta, const float* rho,
                      int iters, int every, float* z, float* ckpt, void* ws, size_t ws_bytes, void* stream) {
  Plan pl;
  int rc = diff_plan(shape, &pl);
  if (rc != CSC_OK) return rc;
  if (!b || !d || !rho || !z || iters < 0 || every < 1 || !(beta >= 0.0f)) return CSC_EINVAL;
  if ((rc = check_ws(ws, ws_bytes, run_diff_ws(pl, every))) != CSC_OK) return rc;
  return run_unrolled(pl, b, d, beta, rho, iters, every, z, ckpt, ws, static_cast<hipStream_t>(stream));
}

int csc_code_backward(const csc_shape* shape, const float* b, const float* d, float beta, const float* rho,
                      int iters, int every, const float* ckpt, const float* zbar, float* dd, double* dbeta, void* ws,
                      size_t ws_bytes, void* stream) {
  Plan pl;
  int rc = diff_plan(shape, &pl);
  if (rc != CSC_OK) return rc;
  if (!b || !d || !rho || !zbar || !dd || !dbeta || iters < 0 || every < 1 || !(beta >= 0.0f)) return CSC_EINVAL;
  if (iters > 0 && !ckpt) return CSC_EINVAL;
  if ((rc = check_ws(ws, ws_bytes, run_diff_ws(pl, every))) != CSC_OK) return rc;
  return run_backward(pl, b, d, beta, rho, iters, every, ckpt, zbar, dd, dbeta, ws, static_cast<hipStream_t>(stream));
}

int csc_loss_grad(const csc_shape* shape, const float* b, const float* d, const float* z, float beta, double* loss,
                  float* zbar, float* dd, double* dbeta, void* ws, size_t ws_bytes, void* stream) {
  Plan pl;
  int rc = diff_plan(shape, &pl);
  if (rc != CSC_OK) return rc;
  if (!b || !d || !z || !loss || !zbar || !dd || !dbeta || !(beta >= 0.0f)) return CSC_EINVAL;
  if ((rc = check_ws(ws, ws_bytes, run_diff_ws(pl, 1))) != CSC_OK) return rc;
  return run_loss_grad(pl, b, d, z, beta, loss, zbar, dd, dbeta, ws, static_cast<hipStream_t>(stream));
}

int csc_objective_reg(const csc_shape* shape, const float* b, const float* d, const float* z, float beta,
                      unsigned flags, double* out, void* ws, size_t ws_bytes, void* stream) {
  Plan pl;
  if (flags & ~CSC_NUCLEAR) return CSC_EINVAL;
  int rc = make_plan_flags(shape, flags, &pl);
  if (rc != CSC_OK) return rc;
  if (!b || !d || !z || !out || !(beta >= 0.0f)) return CSC_EINVAL;
  if ((rc = check_ws(ws, ws_bytes, run_code_ws(pl))) != CSC_OK) return rc;
  return run_objective(pl, b, d, z, beta, out, ws, static_cast<hipStream_t>(stream));
}

int csc_code_dct(const csc_shape* shape, const float* b, const float* q, float beta, float* rho, int iters,
                 unsigned flags, float* z, float* theta, double* resid, void* ws, size_t ws_bytes, void* stream) {
  Plan pl;
  int rc = make_plan(shape, &pl);
  if (rc != CSC_OK) return rc;
  if (!dct_plan_ok(pl)) return CSC_EUNSUPPORTED;
  if (!b || !q || !rho || !z || iters < 0 || !(beta >= 0.0f)) return CSC_EINVAL;
  if (flags & ~(CSC_ADAPTIVE_RHO | CSC_Z_ZERO | CSC_THETA_ZERO)) return CSC_EINVAL;
  if ((rc = check_ws(ws, ws_bytes, dct_ws_bytes(pl))) != CSC_OK) return rc;
  return run_code_dct(pl, b, q, beta, rho, iters, flags, z, theta, resid, ws, static_cast<hipStream_t>(stream));
}

int csc_objective_dct(const csc_shape* shape, const float* b, const float* q, const float* z, float beta,
                      double* out, void* ws, size_t ws_bytes, void* stream) {
  Plan pl;
  int rc = make_plan(shape, &pl);
  if (rc != CSC_OK) return rc;
  if (!dct_plan_ok(pl)) return CSC_EUNSUPPORTED;
  if (!b || !q || !z || !out || !(beta >= 0.0f)) return CSC_EINVAL;
  if ((rc = check_ws(ws, ws_bytes, dct_ws_bytes(pl))) != CSC_OK) return rc;
  return run_objective_dct(pl, b, q, z, beta, out, ws, static_cast<hipStream_t>(stream));
}

int csc_objective(const csc_shape* shape, const float* b, const float* d, const float* z, float beta, double* out,
                  void* ws, size_t ws_bytes, void* stream) {
  Plan pl;
  int rc = make_plan(shape, &pl);
  if (rc != CSC_OK) return rc;
  if (!b || !d || !z || !out || !(beta >= 0.0f)) return CSC_EINVAL;
  if ((rc = check_ws(ws, ws_bytes, run_code_ws(pl))) != CSC_OK) return rc;
  return run_objective(pl, b, d, z, beta, out, ws, static_cast<hipStream_t>(stream));
}

}  // extern "C"
