// C ABI of the batched HPS leaf library: argument checking, batch and
// workspace management, and the order of kernel launches.
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

namespace {

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

// Runs `launch` on the context stream, bracketed by events when timing.
template <typename F>
hipError_t timed(hps_ctx *c, int phase, F &&launch) {
  if (!c->timing) return launch();
  hipEvent_t a = take_event(c), b = take_event(c);
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, c->stream);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(b, c->stream);
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
  return (size_t)16 << 30;  // 16 GiB of in-flight LU workspace
}

}  // namespace

struct hps_batch {
  hps_ctx *ctx = nullptr;
  std::vector<Group> groups;
  int nleaf = 0;
  size_t xt_total = 0, h_total = 0, s_total = 0, b_total = 0;
  double *Xt = nullptr;     // FP64 X^T of every leaf
  double *h = nullptr;      // FP64 h of every leaf
  bool have_h = false;
  bool have_x = false;
  int *info = nullptr;      // [nleaf] internal per-leaf status
  int *conv = nullptr;      // [nleaf] refinement converged flags
  double *norms = nullptr;  // [nleaf][kNormStride] refinement norms
  int *list = nullptr;      // [nleaf] leaves to redo in FP64
  int *count = nullptr;     // [2] length of list; leaves redone in FP64 by
                            //     the last condense
  void *ws = nullptr;       // LU work matrices of the leaves in flight
  size_t ws_bytes = 0;
  int *piv = nullptr, *rstep = nullptr;
  size_t pr_elems = 0;
  size_t ws_limit = 0;
  int last_refine = 0;
};

namespace {

size_t work_bytes_per_leaf(const hps::Geom &g, bool fp32) {
  return (size_t)g.RT * g.CT * 256 * (fp32 ? 4 : 8);
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
  g.box = d.box;
  g.a11 = d.a11;
  g.a22 = d.a22;
  g.c1 = d.c1;
  g.c2 = d.c2;
  g.k2b = d.k2b;
  g.D = dtab + d.p;
  g.D2 = dtab + d.p + (size_t)d.p * d.p;
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
  return s;
}

// Right-hand-side columns of the work matrix: the nb columns of A_ib plus
// f_i when present, or the single column f_i - A_ib u_b when re-factoring.
int rhs_cols(const Group &G, bool refactor, int extra) {
  return refactor ? 1 : G.geom.nb + extra;
}

hps_status ensure_workspace(hps_batch *b, bool refactor, int extra, bool fp32,
                            int *chunk_out) {
  // chunk size per group so that the in-flight work matrices fit ws_limit
  size_t need = 0, need_pr = 0;
  for (size_t gi = 0; gi < b->groups.size(); ++gi) {
    const Group &G = b->groups[gi];
    const hps::Geom g = make_geom(G, rhs_cols(G, refactor, extra));
    const size_t per = work_bytes_per_leaf(g, fp32);
    size_t chunk = std::max<size_t>(1, b->ws_limit / per);
    chunk = std::min<size_t>(chunk, (size_t)G.d.nleaf);
    chunk_out[gi] = (int)chunk;
    need = std::max(need, chunk * per);
    need_pr = std::max(need_pr, chunk * (size_t)g.R);
  }
  if (need > b->ws_bytes) {
    if (b->ws) HPS_TRY(hipFree(b->ws));
    b->ws = nullptr;
    b->ws_bytes = 0;
    HPS_TRY(hipMalloc(&b->ws, need));
    b->ws_bytes = need;
  }
  if (need_pr > b->pr_elems) {
    if (b->piv) HPS_TRY(hipFree(b->piv));
    if (b->rstep) HPS_TRY(hipFree(b->rstep));
    b->piv = b->rstep = nullptr;
    b->pr_elems = 0;
    HPS_TRY(hipMalloc(&b->piv, need_pr * sizeof(int)));
    HPS_TRY(hipMalloc(&b->rstep, need_pr * sizeof(int)));
    b->pr_elems = need_pr;
  }
  return HPS_OK;
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
  fr(b->Xt);
  fr(b->h);
  fr(b->info);
  fr(b->conv);
  fr(b->norms);
  fr(b->list);
  fr(b->count);
  fr(b->ws);
  fr(b->piv);
  fr(b->rstep);
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
    if (d.p < HPS_P_MIN || d.p > HPS_P_MAX || d.nleaf <= 0 || !d.box || d.a12)
      return HPS_ERR_INVALID;
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
    std::vector<double> tab((size_t)p + 2 * (size_t)p * p);
    hps::cheb_tables(p, tab.data(), tab.data() + p, tab.data() + p + (size_t)p * p);
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
        hipMalloc(&b->conv, sizeof(int) * b->nleaf) != hipSuccess ||
        hipMalloc(&b->norms, sizeof(double) * hps::kNormStride * b->nleaf) != hipSuccess ||
        hipMalloc(&b->list, sizeof(int) * b->nleaf) != hipSuccess ||
        hipMalloc(&b->count, 2 * sizeof(int)) != hipSuccess)
      st = HPS_ERR_OOM;
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
  if (!b || !S) return HPS_ERR_INVALID;
  if (prec != HPS_FP64 && prec != HPS_FP32_REFINE) return HPS_ERR_INVALID;
  if (max_refine < 0 || max_refine > 16) return HPS_ERR_INVALID;
  const bool fp32 = prec == HPS_FP32_REFINE;
  const int extra = f ? 1 : 0;
  std::vector<int> chunk(b->groups.size());
  for (const Group &G : b->groups)
    if (hps::factor_lds_bytes(make_geom(G, G.geom.nb + extra), fp32) == 0)
      return HPS_ERR_INVALID;
  hps_status st = ensure_workspace(b, false, extra, fp32, chunk.data());
  if (st != HPS_OK) return st;
  hipStream_t s = b->ctx->stream;
  const int nref = fp32 ? max_refine : 0;
  HPS_TRY(hps::launch_fill_int(b->count, 2, 0, s));
  for (size_t gi = 0; gi < b->groups.size(); ++gi) {
    const Group &G = b->groups[gi];
    const hps::Geom g0 = make_geom(G, G.geom.nb + extra);
    for (int l0 = 0; l0 < G.d.nleaf; l0 += chunk[gi]) {
      const int n = std::min(chunk[gi], G.d.nleaf - l0);
      const hps::Geom g = shift(g0, l0);
      const int gl = G.leaf0 + l0;
      const double *fc = f ? f + G.h_off + (size_t)l0 * g.ni : nullptr;
      double *Xt = b->Xt + G.xt_off + (size_t)l0 * g.nb * g.ni;
      double *hh = f ? b->h + G.h_off + (size_t)l0 * g.ni : nullptr;
      int *inf = b->info + gl;
      HPS_TRY(timed(b->ctx, 1, [&] {
        return hps::launch_factor(g, n, fp32, b->ws, b->piv, b->rstep, inf, hps::RHS_CONDENSE, fc,
                                  nullptr, s);
      }));
      hps::BackOut o;
      o.Xt = Xt;
      o.h = hh;
      o.ui = nullptr;
      o.norms = nullptr;
      o.skip = nullptr;
      o.mode = hps::BACK_STORE;
      HPS_TRY(timed(b->ctx, 2, [&] { return hps::launch_backsolve(g, n, fp32, b->ws, b->piv, b->rstep, o, s); }));
      if (fp32) {
        // FP64 iterative refinement: residual -> stop test -> FP32 correction,
        // and one more residual after the last correction for the final test.
        int *conv = b->conv + gl;
        double *nrm = b->norms + hps::kNormStride * (size_t)gl;
        const double tl = tol > 0.0 ? tol : 1e-10;
        HPS_TRY(hps::launch_fill_int(conv, n, 0, s));
        o.mode = hps::BACK_ACCUM;
        o.skip = conv;
        o.norms = nrm;
        int nsol = 1;   // column chunks of the previous correction solve
        for (int it = 0; it <= nref; ++it) {
          if (it == nref && it > 0 && tl >= 1.0) break;  // no final test wanted
          const int nch = hps::refine_chunks(g, it);
          HPS_TRY(timed(b->ctx, 6, [&] {
            return hps::launch_residual(g, n, (float *)b->ws, Xt, hh, fc, conv, nrm, nch, s);
          }));
          HPS_TRY(timed(b->ctx, 3, [&] {
            return hps::launch_convcheck(n, nrm, tl, conv, inf, it, it == nref ? 1 : 0, nch, nsol,
                                         s);
          }));
          if (it == nref) break;
          HPS_TRY(timed(b->ctx, 3, [&] {
            return hps::launch_refine_solve(g, n, b->ws, b->piv, b->rstep, o, nch, s);
          }));
          nsol = nch;
        }
        // Leaves the refinement could not bring to tol (A_ii too ill-conditioned
        // for an FP32 factorisation, e.g. near a leaf resonance) are condensed
        // again in FP64, reusing the FP32 workspace, in passes of `cap` leaves.
        HPS_TRY(hps::launch_fill_int(b->count, 1, 0, s));
        HPS_TRY(timed(b->ctx, 3, [&] { return hps::launch_collect(n, inf, b->list, b->count, b->count + 1, s); }));
        const size_t per64 = work_bytes_per_leaf(g, false);
        const int cap = (int)std::max<size_t>(1, std::min<size_t>(b->ws_bytes / per64, n));
        hps::BackOut o64;
        o64.Xt = Xt;
        o64.h = hh;
        o64.ui = nullptr;
        o64.norms = nullptr;
        o64.skip = nullptr;
        o64.mode = hps::BACK_STORE;
        for (int s0 = 0; s0 < n; s0 += cap) {
          hps::Sel sel;
          sel.list = b->list;
          sel.count = b->count;
          sel.slot0 = s0;
          const int nb_ = std::min(cap, n - s0);
          HPS_TRY(timed(b->ctx, 7, [&] {
            return hps::launch_factor(g, nb_, false, b->ws, b->piv, b->rstep, inf,
                                      hps::RHS_CONDENSE, fc, nullptr, s, sel);
          }));
          HPS_TRY(timed(b->ctx, 7, [&] {
            return hps::launch_backsolve(g, nb_, false, b->ws, b->piv, b->rstep, o64, s, sel);
          }));
        }
      }
      HPS_TRY(timed(b->ctx, 4, [&] {
        return hps::launch_schur(g, n, Xt, hh, S + G.s_off + (size_t)l0 * g.nb * g.nb,
                                 w ? w + G.b_off + (size_t)l0 * g.nb : nullptr, inf, s);
      }));
    }
  }
  b->have_x = true;
  b->have_h = f != nullptr;
  b->last_refine = nref;
  if (info) HPS_TRY(hps::launch_copy_info(b->info, info, b->nleaf, s));
  if (flags & HPS_SYNC) return sync_status(b, b->info, b->nleaf);
  return HPS_OK;
}

hps_status hps_leaf_recover(hps_batch *b, const double *ub, const double *f, double *ui,
                            int flags) {
  if (!b || !ub || !ui) return HPS_ERR_INVALID;
  hipStream_t s = b->ctx->stream;
  if (flags & HPS_RECOVER_REFACTOR) {
    std::vector<int> chunk(b->groups.size());
    hps_status st = ensure_workspace(b, true, 0, false, chunk.data());
    if (st != HPS_OK) return st;
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
      const Group &G = b->groups[gi];
      const hps::Geom g0 = make_geom(G, 1);
      const int ch = chunk[gi];
      for (int l0 = 0; l0 < G.d.nleaf; l0 += ch) {
        const int n = std::min(ch, G.d.nleaf - l0);
        const hps::Geom g = shift(g0, l0);
        const double *fc = f ? f + G.h_off + (size_t)l0 * g.ni : nullptr;
        const double *uc = ub + G.b_off + (size_t)l0 * g.nb;
        int *inf = b->info + G.leaf0 + l0;
        HPS_TRY(timed(b->ctx, 5, [&] {
          return hps::launch_factor(g, n, false, b->ws, b->piv, b->rstep, inf, hps::RHS_REFACTOR,
                                    fc, uc, s);
        }));
        hps::BackOut o;
        o.Xt = nullptr;
        o.h = nullptr;
        o.ui = ui + G.h_off + (size_t)l0 * g.ni;
        o.norms = nullptr;
        o.skip = nullptr;
        o.mode = hps::BACK_UI;
        HPS_TRY(timed(b->ctx, 5, [&] {
          return hps::launch_backsolve(g, n, false, b->ws, b->piv, b->rstep, o, s);
        }));
      }
    }
    if (flags & HPS_SYNC) return sync_status(b, b->info, b->nleaf);
    return HPS_OK;
  }
  if (!b->have_x) return HPS_ERR_INVALID;
  for (const Group &G : b->groups) {
    HPS_TRY(timed(b->ctx, 5, [&] {
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
  if (factor_variant < 0 || factor_variant > 3) return HPS_ERR_INVALID;
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

hps_status hps_batch_stats(const hps_batch *b, int *refine_steps, int *fp64_redo) {
  if (!b) return HPS_ERR_INVALID;
  if (refine_steps) *refine_steps = b->last_refine;
  if (fp64_redo) {
    int v[2] = {0, 0};
    HPS_TRY(hipStreamSynchronize(b->ctx->stream));
    HPS_TRY(hipMemcpy(v, b->count, sizeof(v), hipMemcpyDeviceToHost));
    *fp64_redo = v[1];
  }
  return HPS_OK;
}

}  // extern "C"
