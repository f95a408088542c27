// C ABI of the batched HPS leaf library: argument checking, batch and
// scratch management, and the order of kernel launches.
//
// Memory: every device buffer a batch uses is allocated once, in
// hps_leaf_build (the Chebyshev tables, the stored X and h, per-leaf flags,
// and per-lane pass scratch sized for the largest mode: FP64 with a body-load
// column).  hps_leaf_condense and hps_leaf_recover never allocate or free, so
// they may be captured in a HIP graph after the batch is built.
// hps_leaf_condense_noalloc runs the same path with its pass scratch in a
// file-scope device array instead of the batch's.
//
// Concurrency: the order groups of a batch are dealt to up to kMaxLanes
// lanes (largest work first, each lane taking the next group while its sum
// of work is the smallest).  Each lane owns a side stream and its own pass
// scratch; a condense forks the lanes from the context stream with an event
// and joins them back, so groups of different orders overlap on the GPU
// (and in a captured graph the lanes become parallel branches).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/hps_leaf.h"
#include "hps_internal.h"

struct hps_ctx {
  hipStream_t stream;
  int device;
  bool timing = false;
  // events recorded around each launch while timing: (phase, start, stop)
  struct Rec {
    int phase;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
};

hipStream_t hps::ctx_stream(const hps_ctx *c) { return c->stream; }

namespace {

constexpr int kMaxLanes = 4;

struct Group {
  hps_leaf_desc d;
  hps::Geom geom;       // base pointers (leaf 0 of the group)
  int leaf0;            // first leaf in batch numbering
  size_t xt_off;        // offset of the group's Xt block (doubles)
  size_t h_off;         // offset of the group's h / f / ui block (doubles)
  size_t s_off;         // offset of the group's S block (doubles)
  size_t b_off;         // offset of the group's w / ub block (doubles)
  double *dtab;         // device: t [p], D [p*p], D2 [p*p]
  int tune_variant;     // see hps_batch_set_tuning
  int tune_ch;
  double work;          // algorithmic FLOP of the group (lane dealing)
};

// Device scratch of one pass over the leaves of a group: the LU work
// matrices, pivots and retire steps of the leaves in flight, and the
// refinement bookkeeping of those leaves (pass-local indexing).
struct Scratch {
  void *ws = nullptr;
  size_t ws_bytes = 0;
  int *piv = nullptr, *rstep = nullptr;
  size_t pr_elems = 0;      // ints in piv and in rstep
  int *conv = nullptr;      // [max_leaves]
  double *norms = nullptr;  // [max_leaves][kNormStride]
  int *list = nullptr;      // [max_leaves]
  int *count = nullptr;     // [1]
  size_t max_leaves = 0;
};

struct Lane {
  std::vector<int> groups;  // indices into hps_batch::groups, largest work first
  Scratch sc;
  void *mem = nullptr;      // the lane's single allocation (sc points into it)
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
};

hps_status from_hip(hipError_t e) {
  if (e == hipSuccess) return HPS_OK;
  if (e == hipErrorOutOfMemory) return HPS_ERR_OOM;
  return HPS_ERR_HIP;
}

#define HPS_TRY(expr)                         \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return from_hip(e_); \
  } while (0)

hipEvent_t take_event(hps_ctx *c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Runs `launch` (which enqueues on stream s), bracketed by events when the
// context is timing; timing only happens on the context stream.
template <typename F>
hipError_t timed(hps_ctx *c, hipStream_t s, int phase, F &&launch) {
  if (!c->timing || s != c->stream) return launch();
  hipEvent_t a = take_event(c), b = take_event(c);
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, s);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(b, s);
  if (e != hipSuccess) return e;
  c->recs.push_back({phase, a, b});
  return hipSuccess;
}

size_t env_workspace_bytes() {
  const char *s = std::getenv("HPS_WORKSPACE_MB");
  if (s && *s) {
    const long long mb = std::atoll(s);
    if (mb > 0) return (size_t)mb << 20;
  }
  return (size_t)32 << 30;  // 32 GiB of in-flight LU work matrices in total
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

struct hps_batch {
  hps_ctx *ctx = nullptr;
  std::vector<Group> groups;
  std::vector<Lane> lanes;
  hipEvent_t fork = nullptr;
  int nleaf = 0;
  size_t xt_total = 0, h_total = 0, s_total = 0, b_total = 0;
  double *Xt = nullptr;     // FP64 X^T of every leaf
  double *h = nullptr;      // FP64 h of every leaf
  bool have_h = false;
  bool have_x = false;
  int *info = nullptr;      // [nleaf] internal per-leaf status
  int *redo = nullptr;      // [nleaf] 1: condensed again in FP64 by the last condense
  int *redo_total = nullptr;  // [1] leaves redone by the last condense
  size_t ws_limit = 0;
  int last_refine = 0;
};

namespace {

size_t work_bytes_per_leaf(const hps::Geom &g, bool fp32) {
  return hps::leaf_tiles(g) * 256 * (fp32 ? 4 : 8);
}

hps::Geom make_geom(const hps_leaf_desc &d, const double *dtab, int nrhs) {
  hps::Geom g;
  g.p = d.p;
  g.m = d.p - 2;
  g.ni = g.m * g.m;
  g.nb = 4 * g.m;
  g.R = (g.ni + 15) / 16 * 16;
  g.RT = g.R / 16;
  g.nrhs = nrhs;
  g.CT = g.RT + (nrhs + 15) / 16;
  g.mdiv = (65536 + g.m - 1) / g.m;
  g.box = d.box;
  g.a11 = d.a11;
  g.a22 = d.a22;
  g.c1 = d.c1;
  g.c2 = d.c2;
  g.k2b = d.k2b;
  g.a12 = d.a12;
  g.D = dtab + d.p;
  g.D2 = dtab + d.p + (size_t)d.p * d.p;
  g.E = dtab + d.p + 2 * (size_t)d.p * d.p;
  g.tune_variant = 0;
  g.tune_ch = 0;
  return g;
}

hps::Geom make_geom(const Group &G, int nrhs) {
  hps::Geom g = make_geom(G.d, G.dtab, nrhs);
  g.tune_variant = G.tune_variant;
  g.tune_ch = G.tune_ch;
  return g;
}

// Geometry offset to leaf `l0` of its group.
hps::Geom shift(const hps::Geom &g, int l0) {
  hps::Geom s = g;
  const size_t pp = (size_t)g.p * g.p;
  s.box = g.box + 4 * (size_t)l0;
  if (g.a11) s.a11 = g.a11 + pp * l0;
  if (g.a22) s.a22 = g.a22 + pp * l0;
  if (g.c1) s.c1 = g.c1 + pp * l0;
  if (g.c2) s.c2 = g.c2 + pp * l0;
  if (g.k2b) s.k2b = g.k2b + pp * l0;
  if (g.a12) s.a12 = g.a12 + pp * l0;
  return s;
}

// Lays a Scratch over `bytes` of device memory at `base` for passes of at
// most `leaves` leaves of work matrices of `per` bytes and R rows.
Scratch carve(void *base, size_t bytes, size_t leaves, size_t per, int R) {
  Scratch s;
  char *p = (char *)base;
  size_t off = 0;
  auto take = [&](size_t n) {
    off = align_up(off, 256);
    char *q = p + off;
    off += n;
    return q;
  };
  s.ws = take(leaves * per);
  s.ws_bytes = leaves * per;
  s.piv = (int *)take(sizeof(int) * leaves * R);
  s.rstep = (int *)take(sizeof(int) * leaves * R);
  s.pr_elems = leaves * R;
  s.norms = (double *)take(sizeof(double) * hps::kNormStride * leaves);
  s.conv = (int *)take(sizeof(int) * leaves);
  s.list = (int *)take(sizeof(int) * leaves);
  s.count = (int *)take(sizeof(int) * 2);
  s.max_leaves = leaves;
  if (off > bytes) return Scratch();   // does not fit: empty
  return s;
}

size_t carve_bytes(size_t leaves, size_t per, int R) {
  return leaves * per + 2 * sizeof(int) * leaves * R + sizeof(double) * hps::kNormStride * leaves +
         2 * sizeof(int) * leaves + 2 * sizeof(int) + 8 * 256;
}

// Leaves per pass of group g for a condense / recover that needs `per`
// bytes of work matrix per leaf, within the scratch s.
int pass_leaves(const Scratch &s, const hps::Geom &g, size_t per, int nleaf) {
  if (!s.ws || per == 0) return 0;
  size_t n = s.ws_bytes / per;
  n = std::min(n, s.max_leaves);
  n = std::min(n, s.pr_elems / (size_t)g.R);
  n = std::min(n, (size_t)nleaf);
  if (n < (size_t)nleaf && n > 256) n -= n % 256;   // whole rounds over the CUs
  return (int)n;
}

hps_status sync_status(hps_batch *b, const int *info_dev, int n) {
  HPS_TRY(hipStreamSynchronize(b->ctx->stream));
  std::vector<int> h((size_t)n);
  if (n) HPS_TRY(hipMemcpy(h.data(), info_dev, sizeof(int) * n, hipMemcpyDeviceToHost));
  bool sing = false, nonf = false, nc = false;
  for (int v : h) {
    if (v > 0) sing = true;
    else if (v == -2) nonf = true;
    else if (v == -1) nc = true;
  }
  if (sing) return HPS_ERR_SINGULAR;
  if (nonf) return HPS_ERR_NONFINITE;
  if (nc) return HPS_ERR_NOT_CONVERGED;
  return HPS_OK;
}

struct CondenseArgs {
  bool fp32;
  double tol;
  int nref;
  const double *f;
  double *S;
  double *w;
};

// Steps a2-a6 for every leaf of group G on stream s, in passes that fit the
// scratch sc.
hps_status condense_group(hps_batch *b, const Group &G, const Scratch &sc, hipStream_t s,
                          const CondenseArgs &a) {
  const int extra = a.f ? 1 : 0;
  const hps::Geom g0 = make_geom(G, G.geom.nb + extra);
  const int chunk = pass_leaves(sc, g0, work_bytes_per_leaf(g0, a.fp32), G.d.nleaf);
  if (chunk < 1) return HPS_ERR_INVALID;
  for (int l0 = 0; l0 < G.d.nleaf; l0 += chunk) {
    const int n = std::min(chunk, G.d.nleaf - l0);
    const hps::Geom g = shift(g0, l0);
    const int gl = G.leaf0 + l0;
    const double *fc = a.f ? a.f + G.h_off + (size_t)l0 * g.ni : nullptr;
    double *Xt = b->Xt + G.xt_off + (size_t)l0 * g.nb * g.ni;
    double *hh = a.f ? b->h + G.h_off + (size_t)l0 * g.ni : nullptr;
    int *inf = b->info + gl;
    HPS_TRY(timed(b->ctx, s, 1, [&] {
      return hps::launch_factor(g, n, a.fp32, sc.ws, sc.piv, sc.rstep, inf, hps::RHS_CONDENSE, fc,
                                nullptr, s);
    }));
    hps::BackOut o;
    o.Xt = Xt;
    o.h = hh;
    o.ui = nullptr;
    o.norms = nullptr;
    o.skip = nullptr;
    o.mode = hps::BACK_STORE;
    HPS_TRY(timed(b->ctx, s, 2, [&] {
      return hps::launch_backsolve(g, n, a.fp32, sc.ws, sc.piv, sc.rstep, o, s);
    }));
    if (a.fp32) {
      // FP64 iterative refinement: residual -> stop test -> FP32 correction,
      // and one more residual after the last correction for the final test.
      int *conv = sc.conv;
      double *nrm = sc.norms;
      const double tl = a.tol > 0.0 ? a.tol : 1e-10;
      HPS_TRY(hps::launch_fill_int(conv, n, 0, s));
      o.mode = hps::BACK_ACCUM;
      o.skip = conv;
      o.norms = nrm;
      int nsol = 1;   // column chunks of the previous correction solve
      for (int it = 0; it <= a.nref; ++it) {
        if (it == a.nref && it > 0 && tl >= 1.0) break;  // no final test wanted
        const int nch = hps::refine_chunks(g, it);
        HPS_TRY(timed(b->ctx, s, 6, [&] {
          return hps::launch_residual(g, n, (float *)sc.ws, Xt, hh, fc, conv, nrm, nch, s);
        }));
        HPS_TRY(timed(b->ctx, s, 3, [&] {
          return hps::launch_convcheck(n, nrm, tl, conv, inf, it, it == a.nref ? 1 : 0, nch, nsol,
                                       s);
        }));
        if (it == a.nref) break;
        HPS_TRY(timed(b->ctx, s, 3, [&] {
          return hps::launch_refine_solve(g, n, sc.ws, sc.piv, sc.rstep, o, nch, s);
        }));
        nsol = hps::refine_solve_chunks(g, nch);
      }
      // Leaves the refinement could not bring to tol (A_ii too ill-conditioned
      // for an FP32 factorisation, e.g. near a leaf resonance) are condensed
      // again in FP64, reusing the FP32 work matrices, in passes of `cap`.
      HPS_TRY(hps::launch_fill_int(sc.count, 1, 0, s));
      HPS_TRY(timed(b->ctx, s, 3, [&] {
        return hps::launch_collect(n, inf, sc.list, sc.count, b->redo_total, b->redo + gl, s);
      }));
      const size_t per64 = work_bytes_per_leaf(g, false);
      const int cap = pass_leaves(sc, g, per64, n);
      if (cap < 1) return HPS_ERR_INVALID;
      hps::BackOut o64;
      o64.Xt = Xt;
      o64.h = hh;
      o64.ui = nullptr;
      o64.norms = nullptr;
      o64.skip = nullptr;
      o64.mode = hps::BACK_STORE;
      for (int s0 = 0; s0 < n; s0 += cap) {
        hps::Sel sel;
        sel.list = sc.list;
        sel.count = sc.count;
        sel.slot0 = s0;
        const int nb_ = std::min(cap, n - s0);
        HPS_TRY(timed(b->ctx, s, 7, [&] {
          return hps::launch_factor(g, nb_, false, sc.ws, sc.piv, sc.rstep, inf,
                                    hps::RHS_CONDENSE, fc, nullptr, s, sel);
        }));
        HPS_TRY(timed(b->ctx, s, 7, [&] {
          return hps::launch_backsolve(g, nb_, false, sc.ws, sc.piv, sc.rstep, o64, s, sel);
        }));
      }
    }
    HPS_TRY(timed(b->ctx, s, 4, [&] {
      return hps::launch_schur(g, n, Xt, hh, a.S + G.s_off + (size_t)l0 * g.nb * g.nb,
                               a.w ? a.w + G.b_off + (size_t)l0 * g.nb : nullptr, inf, s);
    }));
  }
  return HPS_OK;
}

// Re-form and re-factor every leaf of group G in FP64 and solve
// A_ii u_i = f_i - A_ib u_b, in passes that fit the scratch sc.
hps_status refactor_group(hps_batch *b, const Group &G, const Scratch &sc, hipStream_t s,
                          const double *ub, const double *f, double *ui) {
  const hps::Geom g0 = make_geom(G, 1);
  const int ch = pass_leaves(sc, g0, work_bytes_per_leaf(g0, false), G.d.nleaf);
  if (ch < 1) return HPS_ERR_INVALID;
  for (int l0 = 0; l0 < G.d.nleaf; l0 += ch) {
    const int n = std::min(ch, G.d.nleaf - l0);
    const hps::Geom g = shift(g0, l0);
    const double *fc = f ? f + G.h_off + (size_t)l0 * g.ni : nullptr;
    const double *uc = ub + G.b_off + (size_t)l0 * g.nb;
    int *inf = b->info + G.leaf0 + l0;
    HPS_TRY(timed(b->ctx, s, 5, [&] {
      return hps::launch_factor(g, n, false, sc.ws, sc.piv, sc.rstep, inf, hps::RHS_REFACTOR, fc,
                                uc, s);
    }));
    hps::BackOut o;
    o.Xt = nullptr;
    o.h = nullptr;
    o.ui = ui + G.h_off + (size_t)l0 * g.ni;
    o.norms = nullptr;
    o.skip = nullptr;
    o.mode = hps::BACK_UI;
    HPS_TRY(timed(b->ctx, s, 5, [&] {
      return hps::launch_backsolve(g, n, false, sc.ws, sc.piv, sc.rstep, o, s);
    }));
  }
  return HPS_OK;
}

// Runs `body(lane, stream)` for every lane: serially on the context stream
// when there is one lane or the context is timing (so that phase times stay
// attributable), else each lane on its own stream, forked from and joined
// back into the context stream.
template <typename F>
hps_status run_lanes(hps_batch *b, F &&body) {
  hipStream_t s0 = b->ctx->stream;
  const bool serial = b->lanes.size() == 1 || b->ctx->timing;
  if (serial) {
    for (Lane &L : b->lanes) {
      const hps_status st = body(L, s0);
      if (st != HPS_OK) return st;
    }
    return HPS_OK;
  }
  HPS_TRY(hipEventRecord(b->fork, s0));
  for (Lane &L : b->lanes) HPS_TRY(hipStreamWaitEvent(L.stream, b->fork, 0));
  hps_status first = HPS_OK;
  for (Lane &L : b->lanes) {
    const hps_status st = body(L, L.stream);
    if (st != HPS_OK && first == HPS_OK) first = st;
    // join even after a failure, so no branch is left dangling in a capture
    HPS_TRY(hipEventRecord(L.done, L.stream));
    HPS_TRY(hipStreamWaitEvent(s0, L.done, 0));
  }
  return first;
}

hps_status check_condense_args(hps_batch *b, hps_precision prec, int max_refine, const double *S,
                               const double *f) {
  if (!b || !S) return HPS_ERR_INVALID;
  if (prec != HPS_FP64 && prec != HPS_FP32_REFINE) return HPS_ERR_INVALID;
  if (max_refine < 0 || max_refine > 16) return HPS_ERR_INVALID;
  const bool fp32 = prec == HPS_FP32_REFINE;
  const int extra = f ? 1 : 0;
  for (const Group &G : b->groups) {
    // the FP32 path's structured residual has no mixed term
    if (fp32 && G.d.a12) return HPS_ERR_INVALID;
    if (hps::factor_lds_bytes(make_geom(G, G.geom.nb + extra), fp32) == 0) return HPS_ERR_INVALID;
  }
  return HPS_OK;
}

hps_status condense_prologue(hps_batch *b) {
  hipStream_t s = b->ctx->stream;
  HPS_TRY(hps::launch_fill_int(b->redo, b->nleaf, 0, s));
  HPS_TRY(hps::launch_fill_int(b->redo_total, 1, 0, s));
  return HPS_OK;
}

hps_status condense_epilogue(hps_batch *b, int nref, const double *f, int *info, int flags) {
  b->have_x = true;
  b->have_h = f != nullptr;
  b->last_refine = nref;
  hipStream_t s = b->ctx->stream;
  if (info) HPS_TRY(hps::launch_copy_info(b->info, info, b->nleaf, s));
  if (flags & HPS_SYNC) return sync_status(b, b->info, b->nleaf);
  return HPS_OK;
}

// --- the no-allocation variant's scratch --------------------------------
// The array itself is declared at file scope below the anonymous namespace;
// each device's address of it is taken once (hipGetSymbolAddress) and only
// that pointer is passed to kernels.
constexpr int kMaxDevices = 64;
void *g_scratch_ptr[kMaxDevices] = {nullptr};
hps_status noalloc_scratch(int device, void **out);

}  // namespace

// Pass scratch of hps_leaf_condense_noalloc: one array per GPU the library
// runs on (each device holds its own copy at its own address), kept until
// the process ends.  Host code never uses this name as an address.
static __device__ __align__(256) char scratch[HPS_NOALLOC_SCRATCH_BYTES];

namespace {

hps_status noalloc_scratch(int device, void **out) {
  if (device < 0 || device >= kMaxDevices) return HPS_ERR_INVALID;
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    HPS_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return HPS_OK;
}

}  // namespace

extern "C" {

const char *hps_status_string(hps_status s) {
  switch (s) {
    case HPS_OK: return "ok";
    case HPS_ERR_INVALID: return "invalid argument";
    case HPS_ERR_OOM: return "device out of memory";
    case HPS_ERR_HIP: return "HIP runtime error";
    case HPS_ERR_SINGULAR: return "exactly singular interior block (zero pivot)";
    case HPS_ERR_NOT_CONVERGED: return "iterative refinement did not converge";
    case HPS_ERR_NONFINITE: return "non-finite value in the result";
  }
  return "unknown status";
}

hps_status hps_ctx_create(void *stream, hps_ctx **out) {
  if (!out) return HPS_ERR_INVALID;
  *out = nullptr;
  hps_ctx *c = new (std::nothrow) hps_ctx;
  if (!c) return HPS_ERR_OOM;
  c->stream = (hipStream_t)stream;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return HPS_ERR_HIP;
  }
  // the no-allocation entry point's scratch address, taken once per device
  // at set-up with that device current
  void *p = nullptr;
  if (noalloc_scratch(c->device, &p) != HPS_OK) {
    delete c;
    return HPS_ERR_HIP;
  }
  *out = c;
  return HPS_OK;
}

hps_status hps_ctx_destroy(hps_ctx *ctx) {
  if (!ctx) return HPS_OK;
  // release everything, report the first failure
  hipError_t first = hipSuccess;
  auto keep = [&](hipError_t e) {
    if (first == hipSuccess) first = e;
  };
  for (auto &r : ctx->recs) {
    keep(hipEventDestroy(r.a));
    keep(hipEventDestroy(r.b));
  }
  for (hipEvent_t e : ctx->pool) keep(hipEventDestroy(e));
  delete ctx;
  return from_hip(first);
}

hps_status hps_ctx_set_timing(hps_ctx *ctx, int enable) {
  if (!ctx) return HPS_ERR_INVALID;
  ctx->timing = enable != 0;
  return HPS_OK;
}

hps_status hps_ctx_phase_times(hps_ctx *ctx, double *ms, int *launches) {
  if (!ctx) return HPS_ERR_INVALID;
  HPS_TRY(hipStreamSynchronize(ctx->stream));
  double acc[HPS_NPHASE] = {0};
  int cnt[HPS_NPHASE] = {0};
  hps_status st = HPS_OK;
  for (auto &r : ctx->recs) {
    float t = 0.0f;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) st = HPS_ERR_HIP;
    if (r.phase >= 0 && r.phase < HPS_NPHASE) {
      acc[r.phase] += t;
      cnt[r.phase] += 1;
    }
    ctx->pool.push_back(r.a);
    ctx->pool.push_back(r.b);
  }
  ctx->recs.clear();
  for (int i = 0; i < HPS_NPHASE; ++i) {
    if (ms) ms[i] = acc[i];
    if (launches) launches[i] = cnt[i];
  }
  return st;
}

hps_status hps_batch_destroy(hps_batch *b) {
  if (!b) return HPS_OK;
  hps_status st = HPS_OK;
  auto fr = [&](void *p) {
    if (p && hipFree(p) != hipSuccess) st = HPS_ERR_HIP;
  };
  for (Group &G : b->groups) fr(G.dtab);
  for (Lane &L : b->lanes) {
    fr(L.mem);
    if (L.stream && hipStreamDestroy(L.stream) != hipSuccess) st = HPS_ERR_HIP;
    if (L.done && hipEventDestroy(L.done) != hipSuccess) st = HPS_ERR_HIP;
  }
  if (b->fork && hipEventDestroy(b->fork) != hipSuccess) st = HPS_ERR_HIP;
  fr(b->Xt);
  fr(b->h);
  fr(b->info);
  fr(b->redo);
  fr(b->redo_total);
  delete b;
  return st;
}

hps_status hps_leaf_build(hps_ctx *ctx, const hps_leaf_desc *groups, int ngroups,
                          hps_batch **out) {
  if (!ctx || !groups || ngroups <= 0 || !out) return HPS_ERR_INVALID;
  *out = nullptr;
  long long total = 0;
  for (int i = 0; i < ngroups; ++i) {
    const hps_leaf_desc &d = groups[i];
    if (d.p < HPS_P_MIN || d.p > HPS_P_MAX || d.nleaf <= 0 || !d.box) return HPS_ERR_INVALID;
    total += d.nleaf;
  }
  if (total > (1LL << 30)) return HPS_ERR_INVALID;
  hps_batch *b = new (std::nothrow) hps_batch;
  if (!b) return HPS_ERR_OOM;
  b->ctx = ctx;
  b->ws_limit = env_workspace_bytes();
  int leaf0 = 0;
  hps_status st = HPS_OK;
  for (int i = 0; i < ngroups && st == HPS_OK; ++i) {
    Group G;
    G.d = groups[i];
    G.leaf0 = leaf0;
    G.dtab = nullptr;
    G.tune_variant = 0;
    G.tune_ch = 0;
    const int p = G.d.p;
    std::vector<double> tab(hps::cheb_table_size(p));
    hps::cheb_tables(p, tab.data(), tab.data() + p, tab.data() + p + (size_t)p * p,
                     tab.data() + p + 2 * (size_t)p * p);
    if (hipMalloc(&G.dtab, sizeof(double) * tab.size()) != hipSuccess) {
      st = HPS_ERR_OOM;
      break;
    }
    if (hipMemcpy(G.dtab, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice) !=
        hipSuccess) {
      (void)hipFree(G.dtab);   // the copy's failure is the error reported
      st = HPS_ERR_HIP;
      break;
    }
    G.geom = make_geom(G.d, G.dtab, 4 * (p - 2));
    const double ni = G.geom.ni, nb = G.geom.nb;
    G.work = G.d.nleaf * ((2.0 / 3.0) * ni * ni * ni + 2.0 * ni * ni * nb);
    G.xt_off = b->xt_total;
    G.h_off = b->h_total;
    G.s_off = b->s_total;
    G.b_off = b->b_total;
    b->xt_total += (size_t)G.d.nleaf * G.geom.nb * G.geom.ni;
    b->h_total += (size_t)G.d.nleaf * G.geom.ni;
    b->s_total += (size_t)G.d.nleaf * G.geom.nb * G.geom.nb;
    b->b_total += (size_t)G.d.nleaf * G.geom.nb;
    b->groups.push_back(G);
    leaf0 += G.d.nleaf;
  }
  b->nleaf = leaf0;
  if (st == HPS_OK) {
    if (hipMalloc(&b->Xt, sizeof(double) * b->xt_total) != hipSuccess ||
        hipMalloc(&b->h, sizeof(double) * b->h_total) != hipSuccess ||
        hipMalloc(&b->info, sizeof(int) * b->nleaf) != hipSuccess ||
        hipMalloc(&b->redo, sizeof(int) * b->nleaf) != hipSuccess ||
        hipMalloc(&b->redo_total, sizeof(int)) != hipSuccess)
      st = HPS_ERR_OOM;
  }
  if (st == HPS_OK) {
    // deal the groups to lanes: largest work first, to the least loaded lane
    // (HPS_LANES caps the lane count, 1 = one stream)
    int cap = kMaxLanes;
    if (const char *v = std::getenv("HPS_LANES")) {
      const int n = std::atoi(v);
      if (n >= 1 && n < cap) cap = n;
    }
    const int nl = std::min<int>(cap, (int)b->groups.size());
    b->lanes.resize(nl);
    std::vector<int> order(b->groups.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return b->groups[x].work > b->groups[y].work; });
    std::vector<double> load(nl, 0.0);
    for (int gi : order) {
      const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      b->lanes[k].groups.push_back(gi);
      load[k] += b->groups[gi].work;
    }
    // each lane's pass scratch, sized once for the largest mode: FP64 work
    // matrices with a body-load column (FP32 passes then fit twice the
    // leaves, whose bookkeeping is sized for that count).  The cap is shared
    // in proportion to the lanes' work, and a group that needs several
    // passes takes them in multiples of 256 leaves (whole rounds over the
    // CUs, so no pass ends with a lone partial round)
    double total_load = 0.0;
    for (double l : load) total_load += l;
    for (size_t li = 0; li < b->lanes.size(); ++li) {
      Lane &L = b->lanes[li];
      const double share = total_load > 0.0 ? load[li] / total_load : 1.0 / nl;
      const size_t lane_limit = std::max<size_t>((size_t)(share * (double)b->ws_limit), 1);
      size_t ws = 0, leaves = 0, prl = 0;
      for (int gi : L.groups) {
        const Group &G = b->groups[gi];
        const hps::Geom g = make_geom(G, G.geom.nb + 1);
        const size_t per64 = work_bytes_per_leaf(g, false);
        size_t n64 = std::min<size_t>(std::max<size_t>(1, lane_limit / per64), G.d.nleaf);
        if (n64 < (size_t)G.d.nleaf && n64 > 256) n64 -= n64 % 256;
        const size_t n32 = std::min<size_t>(2 * n64, G.d.nleaf);
        ws = std::max(ws, n64 * per64);
        leaves = std::max(leaves, n32);
        prl = std::max(prl, n32 * (size_t)g.R);
      }
      // carve with ws_bytes = ws and piv/rstep/bookkeeping for `leaves`
      const size_t bytes = ws + 2 * sizeof(int) * prl + sizeof(double) * hps::kNormStride * leaves +
                           2 * sizeof(int) * leaves + 2 * sizeof(int) + 8 * 256;
      if (hipMalloc(&L.mem, bytes) != hipSuccess) {
        st = HPS_ERR_OOM;
        break;
      }
      char *p = (char *)L.mem;
      size_t off = 0;
      auto take = [&](size_t n) {
        off = align_up(off, 256);
        char *q = p + off;
        off += n;
        return q;
      };
      L.sc.ws = take(ws);
      L.sc.ws_bytes = ws;
      L.sc.piv = (int *)take(sizeof(int) * prl);
      L.sc.rstep = (int *)take(sizeof(int) * prl);
      L.sc.pr_elems = prl;
      L.sc.norms = (double *)take(sizeof(double) * hps::kNormStride * leaves);
      L.sc.conv = (int *)take(sizeof(int) * leaves);
      L.sc.list = (int *)take(sizeof(int) * leaves);
      L.sc.count = (int *)take(sizeof(int) * 2);
      L.sc.max_leaves = leaves;
      if (nl > 1) {
        if (hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&L.done, hipEventDisableTiming) != hipSuccess) {
          st = HPS_ERR_HIP;
          break;
        }
      }
    }
    if (st == HPS_OK && nl > 1 &&
        hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess)
      st = HPS_ERR_HIP;
  }
  if (st != HPS_OK) {
    hps_batch_destroy(b);
    return st;
  }
  *out = b;
  return HPS_OK;
}

int hps_batch_nleaf(const hps_batch *b) { return b ? b->nleaf : -1; }

hps_status hps_batch_group_dims(const hps_batch *b, int g, int *p, int *nleaf, int *ni,
                                int *nb) {
  if (!b || g < 0 || g >= (int)b->groups.size()) return HPS_ERR_INVALID;
  const Group &G = b->groups[g];
  if (p) *p = G.d.p;
  if (nleaf) *nleaf = G.d.nleaf;
  if (ni) *ni = G.geom.ni;
  if (nb) *nb = G.geom.nb;
  return HPS_OK;
}

hps_status hps_leaf_nodes(hps_batch *b, int g, double *xy) {
  if (!b || !xy || g < 0 || g >= (int)b->groups.size()) return HPS_ERR_INVALID;
  const Group &G = b->groups[g];
  HPS_TRY(hps::launch_nodes(G.geom, G.d.nleaf, G.dtab, xy, b->ctx->stream));
  return HPS_OK;
}

hps_status hps_leaf_operator(hps_batch *b, int g, double *Aii, double *Aib, double *Abi,
                             double *Abb) {
  if (!b || g < 0 || g >= (int)b->groups.size()) return HPS_ERR_INVALID;
  const Group &G = b->groups[g];
  HPS_TRY(hps::launch_operator(G.geom, G.d.nleaf, Aii, Aib, Abi, Abb, b->ctx->stream));
  return HPS_OK;
}

hps_status hps_leaf_condense(hps_batch *b, hps_precision prec, double tol, int max_refine,
                             const double *f, double *S, double *w, int *info, int flags) {
  hps_status st = check_condense_args(b, prec, max_refine, S, f);
  if (st != HPS_OK) return st;
  const bool fp32 = prec == HPS_FP32_REFINE;
  const CondenseArgs a{fp32, tol, fp32 ? max_refine : 0, f, S, w};
  st = condense_prologue(b);
  if (st != HPS_OK) return st;
  st = run_lanes(b, [&](Lane &L, hipStream_t s) {
    for (int gi : L.groups) {
      const hps_status e = condense_group(b, b->groups[gi], L.sc, s, a);
      if (e != HPS_OK) return e;
    }
    return HPS_OK;
  });
  if (st != HPS_OK) return st;
  return condense_epilogue(b, a.nref, f, info, flags);
}

hps_status hps_leaf_condense_noalloc(hps_batch *b, hps_precision prec, double tol, int max_refine,
                                     const double *f, double *S, double *w, int *info, int flags) {
  hps_status st = check_condense_args(b, prec, max_refine, S, f);
  if (st != HPS_OK) return st;
  const bool fp32 = prec == HPS_FP32_REFINE;
  // every group must fit at least one leaf per pass (its FP64 redo too)
  for (const Group &G : b->groups) {
    const hps::Geom g = make_geom(G, G.geom.nb + (f ? 1 : 0));
    if (carve_bytes(1, work_bytes_per_leaf(g, false), g.R) > HPS_NOALLOC_SCRATCH_BYTES)
      return HPS_ERR_INVALID;
  }
  void *base = nullptr;
  st = noalloc_scratch(b->ctx->device, &base);
  if (st != HPS_OK) return st;
  const CondenseArgs a{fp32, tol, fp32 ? max_refine : 0, f, S, w};
  st = condense_prologue(b);
  if (st != HPS_OK) return st;
  hipStream_t s = b->ctx->stream;
  for (const Group &G : b->groups) {
    // the largest pass of this group's precision that fits the array
    const hps::Geom g = make_geom(G, G.geom.nb + (f ? 1 : 0));
    const size_t per = work_bytes_per_leaf(g, fp32);
    const size_t one = carve_bytes(1, per, g.R) - carve_bytes(0, per, g.R);
    const size_t n = std::min<size_t>(
        G.d.nleaf, (HPS_NOALLOC_SCRATCH_BYTES - carve_bytes(0, per, g.R)) / one);
    const Scratch sc = carve(base, HPS_NOALLOC_SCRATCH_BYTES, n, per, g.R);
    if (!sc.ws) return HPS_ERR_INVALID;
    st = condense_group(b, G, sc, s, a);
    if (st != HPS_OK) return st;
  }
  return condense_epilogue(b, a.nref, f, info, flags);
}

hps_status hps_leaf_recover(hps_batch *b, const double *ub, const double *f, double *ui,
                            int flags) {
  if (!b || !ub || !ui) return HPS_ERR_INVALID;
  hipStream_t s = b->ctx->stream;
  if (flags & HPS_RECOVER_REFACTOR) {
    hps_status st = run_lanes(b, [&](Lane &L, hipStream_t ls) {
      for (int gi : L.groups) {
        const hps_status e = refactor_group(b, b->groups[gi], L.sc, ls, ub, f, ui);
        if (e != HPS_OK) return e;
      }
      return HPS_OK;
    });
    if (st != HPS_OK) return st;
    if (flags & HPS_SYNC) return sync_status(b, b->info, b->nleaf);
    return HPS_OK;
  }
  if (!b->have_x) return HPS_ERR_INVALID;
  for (const Group &G : b->groups) {
    HPS_TRY(timed(b->ctx, s, 5, [&] {
      return hps::launch_recover(G.geom, G.d.nleaf, b->Xt + G.xt_off,
                                 b->have_h ? b->h + G.h_off : nullptr, ub + G.b_off,
                                 ui + G.h_off, s);
    }));
  }
  if (flags & HPS_SYNC) HPS_TRY(hipStreamSynchronize(s));
  return HPS_OK;
}

hps_status hps_batch_set_tuning(hps_batch *b, int g, int factor_variant, int chunk_cols) {
  if (!b || g < 0 || g >= (int)b->groups.size()) return HPS_ERR_INVALID;
  if (factor_variant < 0 || factor_variant > 4) return HPS_ERR_INVALID;
  if (chunk_cols < 0 || chunk_cols > 1024 || (chunk_cols & 15)) return HPS_ERR_INVALID;
  b->groups[g].tune_variant = factor_variant;
  b->groups[g].tune_ch = chunk_cols;
  return HPS_OK;
}

hps_status hps_batch_export(hps_batch *b, double *Xt, double *h) {
  if (!b || !b->have_x) return HPS_ERR_INVALID;
  hipStream_t s = b->ctx->stream;
  if (Xt)
    HPS_TRY(hipMemcpyAsync(Xt, b->Xt, sizeof(double) * b->xt_total, hipMemcpyDeviceToDevice, s));
  if (h) {
    if (b->have_h)
      HPS_TRY(hipMemcpyAsync(h, b->h, sizeof(double) * b->h_total, hipMemcpyDeviceToDevice, s));
    else
      HPS_TRY(hps::launch_fill_double(h, b->h_total, 0.0, s));
  }
  return HPS_OK;
}

hps_status hps_batch_redo_flags(hps_batch *b, int *flags) {
  if (!b || !flags) return HPS_ERR_INVALID;
  HPS_TRY(hps::launch_copy_info(b->redo, flags, b->nleaf, b->ctx->stream));
  return HPS_OK;
}

hps_status hps_batch_stats(const hps_batch *b, int *refine_steps, int *fp64_redo) {
  if (!b) return HPS_ERR_INVALID;
  if (refine_steps) *refine_steps = b->last_refine;
  if (fp64_redo) {
    int v = 0;
    HPS_TRY(hipStreamSynchronize(b->ctx->stream));
    HPS_TRY(hipMemcpy(&v, b->redo_total, sizeof(int), hipMemcpyDeviceToHost));
    *fp64_redo = v;
  }
  return HPS_OK;
}

int hps_batch_lanes(const hps_batch *b) { return b ? (int)b->lanes.size() : -1; }

}  // extern "C"
