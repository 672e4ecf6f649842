// Host side of the C ABI declared in include/rlgl.h.
//
// The context owns no device memory: the caller's workspace is carved into
// the cash buffers, the history, the frontier, the per-step record ring and
// the static pull plan.  A step is three launches (select, push, complete);
// rlgl_solve enqueues a batch of steps, reads the device status word once per
// batch and sizes the next batch from the observed contraction of the
// residual, so that the host synchronises a handful of times per solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/rlgl.h"
#include "rlgl_device.h"
#include "rlgl_kernels.hip"
#include "rlgl_lockstep.hip"
#include "rlgl_validate.hip"
#include "rlgl_small.hip"

using namespace rlgl;

namespace {

thread_local std::string g_err;

rlgl_status fail(rlgl_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(expr)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) return fail(RLGL_EHIP, "%s: %s", #expr, hipGetErrorString(e_));     \
  } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
// The workspace places the status word right after the three step records.
size_t records_bytes() { return align_up(sizeof(Rec) * 3, 256); }
size_t record_span() { return records_bytes() + sizeof(Glob); }

struct Layout {
  size_t cash0, cash1, hist, hist_lo, fr_rowstart, fr_eoff, fr_id, fr_scale, chunk_first, green_mask, delta, colt,
      hot_nodes, rec, glob,
      log, items, long_cols, long_acc, long_cnt, khist, tk_ckey, tk_cid, tk_hist, tk_cnt, tk_seg, total;
  size_t max_items, max_long;
  // relabelled layout
  size_t perm, old2new, nrowptr, ncol, nval, ncolptr, nrow, ncval;
};

// Upper bounds of the single-chain pull plan (pull_plan_host): a run ends
// because it is full (WL links or WCOLS columns) or because a long column
// follows; two consecutive runs hold more than WL links unless a column-count
// or long-column break separates them; pieces: nnz / WL + one per long column.
size_t pull_long_bound(long long nnz) { return (size_t)(nnz / (WL + 1) + 1); }
size_t pull_item_bound(long long n, long long nnz) {
  return 3 * (size_t)(nnz / WL + 2) + (size_t)(n / WCOLS + 2) + 2 * pull_long_bound(nnz) + 2;
}

Layout make_layout(long long n, long long nnz, int prec, bool has_csc, bool relabel = false, bool has_val = false,
                   bool topk = false) {
  Layout L{};
  const size_t cs = (prec == RLGL_FP64) ? 8 : 4;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes, 256);
    return at;
  };
  L.cash0 = take(cs * n);
  L.cash1 = has_csc ? take(cs * n) : L.cash0;
  L.hist = take(8 * n);  // double, or the float hi part
  L.hist_lo = (prec == RLGL_FP32C_KAHANH) ? take(4 * n) : 0;
  L.fr_rowstart = take(4 * n);
  L.fr_eoff = take(4 * n);
  L.fr_id = take(4 * n);
  L.fr_scale = take(cs * n);
  L.chunk_first = take(4 * (nnz / CH + 2));
  L.green_mask = take(n);
  L.delta = (prec == RLGL_FP64) ? 0 : take(8 * n);
  L.colt = take(4 * (size_t)nnz);
  L.hot_nodes = take(4 * (size_t)HOT_MAX);
  L.rec = take(sizeof(Rec) * 3);
  L.glob = take(sizeof(Glob));
  L.log = take(sizeof(StepLog) * LOG_STEPS);
  if (has_csc) {
    // upper bounds of the plan built in rlgl_create: a run ends because it is
    // full (WL links or WCOLS columns) or because a long column follows
    L.max_long = pull_long_bound(nnz);
    // runs: two consecutive runs hold more than WL links unless a column-count
    // or long-column break separates them; pieces: nnz / WL + one per long column
    L.max_items = pull_item_bound(n, nnz);
    L.items = take(sizeof(int4) * L.max_items);
    L.long_cols = take(4 * L.max_long);
    L.long_acc = take(8 * L.max_long);
    L.long_cnt = take(4 * L.max_long);
  }
  if (topk) {
    L.khist = take(4 * (size_t)3 * KH_STRIPES * KH_BINS);
    L.tk_ckey = take(8 * (size_t)n);
    L.tk_cid = take(4 * (size_t)n);
    L.tk_hist = take(4 * (size_t)TK_HIST_WORDS);
    L.tk_cnt = take(4 * (size_t)SEL_GRID);
    L.tk_seg = (prec == RLGL_FP64) ? 0 : take(4 * (size_t)TK_GRID * TK_LOW_BINS);
  }
  if (relabel) {
    const size_t vs = (prec == RLGL_FP64) ? 8 : 4;
    L.perm = take(4 * n);
    L.old2new = take(4 * n);
    L.nrowptr = take(4 * (n + 1));
    L.ncol = take(4 * (size_t)nnz);
    L.nval = has_val ? take(vs * (size_t)nnz) : 0;
    if (has_csc) {
      L.ncolptr = take(4 * (n + 1));
      L.nrow = take(4 * (size_t)nnz);
      L.ncval = has_val ? take(vs * (size_t)nnz) : 0;
    }
  }
  L.total = off + 256;
  return L;
}

bool valid_options(const rlgl_options *o, std::string &why) {
  if (o->sched < 0 || o->sched > 4) { why = "sched out of range"; return false; }
  if (!(o->r >= 1.0) || !std::isfinite(o->r)) { why = "r must be >= 1"; return false; }
  if (o->sched == RLGL_SCHED_TOPK && o->k < 1) { why = "k must be >= 1"; return false; }
  if (o->theta_period < 1) { why = "theta_period must be >= 1"; return false; }
  if (o->precision < 0 || o->precision > 2) { why = "precision out of range"; return false; }
  if (o->route < 0 || o->route > 2) { why = "route out of range"; return false; }
  if (!(o->pull_alpha >= 0.0)) { why = "pull_alpha must be >= 0"; return false; }
  if (o->check_period < 0) { why = "check_period must be >= 0"; return false; }
  if (o->refresh < 0) { why = "refresh must be >= 0"; return false; }
  if (o->relabel && (o->sched == RLGL_SCHED_TOPK || o->sched == RLGL_SCHED_PC)) {
    why = "relabel does not combine with TOPK or PC";
    return false;
  }
  return true;
}

const char *kernel_names[] = {"select", "push", "complete", "topk"};
enum { KS_SELECT = 0, KS_PUSH = 1, KS_COMPLETE = 2, KS_TOPK = 3, KS_N = 4 };

struct Launch {
  int kind;
  long long s;
  hipEvent_t a, b;
};

}  // namespace

struct rlgl_ctx {
  Dev d;
  hipStream_t stream;
  int prec;
  int hk;  // compensated history
  long long t;
  int grid_sel, grid_push, grid_cmp, grid_misc;
  int pull_wide;  // k_complete runs one workgroup of PULL_WIDE waves per CU (FP32 cash)
  int grid_pull;  // its grid: the workgroups that stay resident together
  Glob *host_glob;  // pinned
  Rec *host_rec;    // pinned, 3 records
  StepLog *host_log;
  bool prof;
  std::vector<Launch> launches;
  std::vector<hipEvent_t> free_events;
  int has_mask;
  int check_period;
  int refresh;
  long long refreshes;
  bool stale;  // host_rec / host_glob older than the device's (after a reset)
  bool khist_stale;  // the top-k histogram of the current record does not describe its cash
};

namespace {

hipEvent_t get_event(rlgl_ctx *c) {
  if (!c->free_events.empty()) {
    hipEvent_t e = c->free_events.back();
    c->free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

template <class F>
hipError_t timed(rlgl_ctx *c, int kind, long long s, F launch) {
  if (!c->prof) {
    launch();
    return hipGetLastError();
  }
  Launch L{kind, s, get_event(c), get_event(c)};
  (void)hipEventRecord(L.a, c->stream);
  launch();
  hipError_t e = hipGetLastError();
  (void)hipEventRecord(L.b, c->stream);
  c->launches.push_back(L);
  return e;
}

// k_complete and k_refresh come in variants by stored or implied link values
// and by whether the threshold's power mean needs sum |C|^r (r != 1).
template <class T, bool TK, int PW>
void launch_complete_w(rlgl_ctx *c, long long s, int force_all) {
  const Dev &d = c->d;
  const bool v = d.cval != nullptr, rp = d.r != 1.0;
  const int grid = c->grid_pull;
  if (v && rp) k_complete<T, true, true, TK, PW><<<grid, PW * 64, 0, c->stream>>>(d, s, force_all);
  else if (v) k_complete<T, true, false, TK, PW><<<grid, PW * 64, 0, c->stream>>>(d, s, force_all);
  else if (rp) k_complete<T, false, true, TK, PW><<<grid, PW * 64, 0, c->stream>>>(d, s, force_all);
  else k_complete<T, false, false, TK, PW><<<grid, PW * 64, 0, c->stream>>>(d, s, force_all);
}
template <class T, bool TK>
void launch_complete_tk(rlgl_ctx *c, long long s, int force_all) {
  if (sizeof(T) == 4 && c->pull_wide) launch_complete_w<float, TK, PULL_WIDE>(c, s, force_all);
  else launch_complete_w<T, TK, NWAVE>(c, s, force_all);
}
// The top-k rule needs the histogram of the keys the pass writes.
template <class T>
void launch_complete(rlgl_ctx *c, long long s, int force_all) {
  if (c->d.sched == SCHED_TOPK) launch_complete_tk<T, true>(c, s, force_all);
  else launch_complete_tk<T, false>(c, s, force_all);
}

// Workgroups of the k_complete variant launch_complete picks that fit one CU together.
template <bool TK>
const void *complete_wide_kernel(bool v, bool rp) {
  return v ? (rp ? (const void *)k_complete<float, true, true, TK, PULL_WIDE>
                 : (const void *)k_complete<float, true, false, TK, PULL_WIDE>)
           : (rp ? (const void *)k_complete<float, false, true, TK, PULL_WIDE>
                 : (const void *)k_complete<float, false, false, TK, PULL_WIDE>);
}
hipError_t complete_occupancy(const rlgl_ctx *c, int *per_cu) {
  const Dev &d = c->d;
  const bool v = d.cval != nullptr, rp = d.r != 1.0;
  if (c->pull_wide) {
    const void *w = d.sched == SCHED_TOPK ? complete_wide_kernel<true>(v, rp) : complete_wide_kernel<false>(v, rp);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, w, PULL_WIDE * 64, 0);
  }
  const void *f;
  if (d.sched == SCHED_TOPK) {
    if (c->prec == RLGL_FP64)
      f = v ? (rp ? (const void *)k_complete<double, true, true, true> : (const void *)k_complete<double, true, false, true>)
            : (rp ? (const void *)k_complete<double, false, true, true> : (const void *)k_complete<double, false, false, true>);
    else
      f = v ? (rp ? (const void *)k_complete<float, true, true, true> : (const void *)k_complete<float, true, false, true>)
            : (rp ? (const void *)k_complete<float, false, true, true> : (const void *)k_complete<float, false, false, true>);
  } else {
    if (c->prec == RLGL_FP64)
      f = v ? (rp ? (const void *)k_complete<double, true, true, false> : (const void *)k_complete<double, true, false, false>)
            : (rp ? (const void *)k_complete<double, false, true, false> : (const void *)k_complete<double, false, false, false>);
    else
      f = v ? (rp ? (const void *)k_complete<float, true, true, false> : (const void *)k_complete<float, true, false, false>)
            : (rp ? (const void *)k_complete<float, false, true, false> : (const void *)k_complete<float, false, false, false>);
  }
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, f, BLOCK, 0);
}

template <class T, int HK>
void launch_refresh(rlgl_ctx *c, long long t, int out) {
  const Dev &d = c->d;
  const bool v = d.cval != nullptr, rp = d.r != 1.0;
  if (v && rp) k_refresh<T, HK, true, true><<<c->grid_cmp, BLOCK, 0, c->stream>>>(d, t, out);
  else if (v) k_refresh<T, HK, true, false><<<c->grid_cmp, BLOCK, 0, c->stream>>>(d, t, out);
  else if (rp) k_refresh<T, HK, false, true><<<c->grid_cmp, BLOCK, 0, c->stream>>>(d, t, out);
  else k_refresh<T, HK, false, false><<<c->grid_cmp, BLOCK, 0, c->stream>>>(d, t, out);
}

hipError_t enqueue_step(rlgl_ctx *c, long long s, double eps, long long s_limit, int force_all) {
  const dim3 blk(BLOCK);
  const Dev &d = c->d;
  hipError_t e = hipSuccess;
  if (!force_all && d.sched == SCHED_TOPK) {
    e = timed(c, KS_TOPK, s, [&] {
      // the k-th largest |C| and the id bound among its ties: the bin of the
      // histogram the previous complete pass counted, its candidates, then a
      // radix select over them
      const bool dbl = c->prec == RLGL_FP64;
      if (c->khist_stale) {
        k_topk_hist_zero<<<8, 256, 0, c->stream>>>(d, s);
        if (dbl) k_topk_hist_full<double><<<c->grid_sel, BLOCK, 0, c->stream>>>(d, s);
        else k_topk_hist_full<float><<<c->grid_sel, BLOCK, 0, c->stream>>>(d, s);
        c->khist_stale = false;
      }
      if (!dbl) {
        // FP32 keys: the collecting pass counts the middle digit, one more
        // pass the low digit; the select pass fixes tau and the id bound
        k_topk_collect<float><<<d.tk_grid, BLOCK, 0, c->stream>>>(d, s);
        k_topk_narrow<<<d.tk_grid, BLOCK, 0, c->stream>>>(d, s);
        return;
      }
      // FP64 keys: the digits below bin B, then those of the ids (ids < 2^31)
      TkDigit dg[8];
      int nd = 0;
      for (int lo = 63 - KH_BITS; lo > 0;) {
        const int w = std::min(lo, KH_BITS);
        lo -= w;
        dg[nd++] = TkDigit{0, lo, w};
      }
      for (int lo = 31; lo > 0;) {
        const int w = std::min(lo, KH_BITS);
        lo -= w;
        dg[nd++] = TkDigit{1, lo, w};
      }
      const int pg = std::max(1, std::min(c->grid_sel, 256));
      k_topk_collect<double><<<d.tk_grid, BLOCK, 0, c->stream>>>(d, s);
      for (int p = 0; p <= nd; ++p) {
        const TkDigit prev = p > 0 ? dg[p - 1] : TkDigit{0, 0, 0};
        const TkDigit cur = p < nd ? dg[p] : TkDigit{1, 0, 0};
        k_topk_pass<double><<<p < nd ? pg : 1, BLOCK, 0, c->stream>>>(d, s, p, prev, cur);
      }
    });
    if (e != hipSuccess) return e;
  }
  e = timed(c, KS_SELECT, s, [&] {
    if (c->prec == RLGL_FP64) k_select<double, 0><<<c->grid_sel, blk, 0, c->stream>>>(d, s, eps, s_limit, force_all);
    else if (c->hk) k_select<float, 1><<<c->grid_sel, blk, 0, c->stream>>>(d, s, eps, s_limit, force_all);
    else k_select<float, 0><<<c->grid_sel, blk, 0, c->stream>>>(d, s, eps, s_limit, force_all);
  });
  if (e != hipSuccess) return e;
  // the select pulls every step of the all-green rule (and step 0) when the
  // CSC is given, so the push pass is not launched for them
  const bool pulls = d.colptr && (d.route == ROUTE_PULL || (d.route == ROUTE_AUTO && (force_all || d.sched == SCHED_ALL)));
  if (!pulls) {
    e = timed(c, KS_PUSH, s, [&] {
      if (c->prec == RLGL_FP64) k_push<double><<<c->grid_push, blk, 0, c->stream>>>(d, s);
      else k_push<float><<<c->grid_push, blk, 0, c->stream>>>(d, s);
    });
    if (e != hipSuccess) return e;
  }
  e = timed(c, KS_COMPLETE, s, [&] {
    if (c->prec == RLGL_FP64) launch_complete<double>(c, s, force_all);
    else launch_complete<float>(c, s, force_all);
  });
  return e;
}

rlgl_status read_back(rlgl_ctx *c) {
  if ((const char *)c->d.glob == (const char *)c->d.rec + records_bytes()) {
    HIP_TRY(hipMemcpyAsync(c->host_rec, c->d.rec, record_span(), hipMemcpyDeviceToHost, c->stream));
  } else {
    HIP_TRY(hipMemcpyAsync(c->host_glob, c->d.glob, sizeof(Glob), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(c->host_rec, c->d.rec, sizeof(Rec) * 3, hipMemcpyDeviceToHost, c->stream));
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->stale = false;
  c->t = c->host_glob->t;
  if (c->host_glob->bad)
    return fail(RLGL_EINVAL, "a kernel met a link index or plan entry outside its range: the graph breaks the "
                             "contract of rlgl_graph (rlgl_validate names the first violation)");
  return RLGL_OK;
}

void fill_info(rlgl_ctx *c, rlgl_step_info *info, int status) {
  if (!info) return;
  const long long t = c->t;
  const Rec &cur = c->host_rec[t % 3];
  const Rec &prv = c->host_rec[(t + 2) % 3];
  const Tot ct = host_totals(cur), pt = host_totals(prv);
  info->t = t;
  info->green = pt.green;
  info->green_total = cur.green_total;
  info->edges_pushed = cur.edges_total;
  info->l1_cash = ct.l1;
  info->h_sum = cur.hsum;
  info->resid = cur.hsum != 0.0 ? ct.l1 / std::fabs(cur.hsum) : INFINITY;
  info->theta = prv.theta;
  info->cash_sum = ct.csum;
  info->status = status;
  info->last_route = prv.mode;
}

rlgl_status reset_device(rlgl_ctx *c) {
  c->khist_stale = false;  // step 0 counts the histogram of C_1
  const Dev &d = c->d;
  const int gr = std::max(3, c->grid_misc);  // blocks 0..2 clear the three records
  if (c->prec == RLGL_FP64) k_reset<double, 0><<<gr, BLOCK, 0, c->stream>>>(d);
  else if (c->hk) k_reset<float, 1><<<gr, BLOCK, 0, c->stream>>>(d);
  else k_reset<float, 0><<<gr, BLOCK, 0, c->stream>>>(d);
  HIP_TRY(hipGetLastError());
  HIP_TRY(enqueue_step(c, 0, -1.0, 1, 1));  // step 0: all green, M_0 = (1/N) 1
  // step 0 always leaves t = 1; the host copies of the records are read
  // when a call first needs them
  c->t = 1;
  c->stale = true;
  return RLGL_OK;
}

// sync = false leaves the host copies stale (the caller reads back next).
rlgl_status do_refresh(rlgl_ctx *c, bool sync = true) {
  if (!c->d.colptr) return fail(RLGL_EINVAL, "refresh needs the CSC arrays");
  if (c->stale) {
    const rlgl_status st = read_back(c);
    if (st != RLGL_OK) return st;
  }
  const long long t = c->t;
  const int out = c->host_rec[t % 3].buf ^ 1;
  const Dev &d = c->d;
  k_refresh_prep<<<1, 64, 0, c->stream>>>(d, t);
  if (c->hk) k_refresh_pool<1><<<c->grid_misc, BLOCK, 0, c->stream>>>(d);
  else k_refresh_pool<0><<<c->grid_misc, BLOCK, 0, c->stream>>>(d);
  if (c->prec == RLGL_FP64) launch_refresh<double, 0>(c, t, out);
  else if (c->hk) launch_refresh<float, 1>(c, t, out);
  else launch_refresh<float, 0>(c, t, out);
  if (d.n_long > 0) {
    const int gl = std::max(1, std::min((d.n_long + BLOCK - 1) / BLOCK, NODE_GRID));
    if (c->prec == RLGL_FP64) k_refresh_long<double, 0><<<gl, BLOCK, 0, c->stream>>>(d, t, out);
    else if (c->hk) k_refresh_long<float, 1><<<gl, BLOCK, 0, c->stream>>>(d, t, out);
    else k_refresh_long<float, 0><<<gl, BLOCK, 0, c->stream>>>(d, t, out);
  }
  // with FP32 cash the refresh sources lived in the push accumulators
  if (d.rsrc == d.delta) k_zero_f64<<<c->grid_misc, BLOCK, 0, c->stream>>>(d.delta, d.n);
  k_refresh_done<<<1, 64, 0, c->stream>>>(d, t, out);
  HIP_TRY(hipGetLastError());
  ++c->refreshes;
  c->khist_stale = true;  // the rebuilt cash has no histogram of its own
  if (!sync) {
    c->stale = true;  // the refresh keeps t; the next read-back renews the copies
    return RLGL_OK;
  }
  return read_back(c);
}

rlgl_status status_of(int dev_status) {
  switch (dev_status) {
    case ST_ZERO_HISTORY: return RLGL_EZERO_HISTORY;
    case ST_NONFINITE: return RLGL_ENONFINITE;
    case ST_LIMIT: return RLGL_ENOT_CONVERGED;
    case ST_BAD_GRAPH: return RLGL_EINVAL;
    default: return RLGL_OK;
  }
}

// Relabelled layout (a1): states renumbered by decreasing out-degree, ties by
// id (a stable counting sort on the host, from the row pointers), and the CSR
// and CSC rewritten in the new numbering into the workspace by k_relabel_side.
// gi receives the relabelled graph; the context keeps the new -> old map.
rlgl_status relabel_graph(rlgl_ctx *c, const rlgl_graph *g, const Layout &L, char *w, rlgl_graph &gi) {
  const int n = g->n;
  Dev &d = c->d;
  std::vector<int> rp((size_t)n + 1), cp(g->csc_colptr ? (size_t)n + 1 : 0);
  HIP_TRY(hipMemcpyAsync(rp.data(), g->csr_rowptr, sizeof(int) * ((size_t)n + 1), hipMemcpyDeviceToHost, c->stream));
  if (g->csc_colptr)
    HIP_TRY(hipMemcpyAsync(cp.data(), g->csc_colptr, sizeof(int) * ((size_t)n + 1), hipMemcpyDeviceToHost,
                           c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (rp[0] != 0) return fail(RLGL_EINVAL, "csr_rowptr[0] must be 0");
  int maxdeg = 0;
  for (int i = 0; i < n; ++i) {
    const int dg = rp[i + 1] - rp[i];
    if (dg < 0) return fail(RLGL_EINVAL, "csr_rowptr decreases at %d", i);
    maxdeg = std::max(maxdeg, dg);
  }
  if (g->csc_colptr) {
    if (cp[0] != 0 || (long long)cp[n] != g->nnz) return fail(RLGL_EINVAL, "csc_colptr must run from 0 to nnz");
    for (int i = 0; i < n; ++i)
      if (cp[i + 1] < cp[i]) return fail(RLGL_EINVAL, "csc_colptr decreases at %d", i);
  }
  std::vector<int> new2old((size_t)n), old2new((size_t)n);
  if ((long long)maxdeg <= 4ll * n + 1024) {
    // counting sort by degree, largest first, stable in the id
    std::vector<long long> start((size_t)maxdeg + 2, 0);
    for (int i = 0; i < n; ++i) ++start[(size_t)(maxdeg - (rp[i + 1] - rp[i]))];
    long long acc = 0;
    for (auto &x : start) {
      const long long cnt = x;
      x = acc;
      acc += cnt;
    }
    for (int i = 0; i < n; ++i) new2old[(size_t)start[(size_t)(maxdeg - (rp[i + 1] - rp[i]))]++] = i;
  } else {
    for (int i = 0; i < n; ++i) new2old[i] = i;
    std::stable_sort(new2old.begin(), new2old.end(),
                     [&](int a, int b) { return rp[a + 1] - rp[a] > rp[b + 1] - rp[b]; });
  }
  for (int i = 0; i < n; ++i) old2new[new2old[i]] = i;
  std::vector<int> nrp((size_t)n + 1), ncp(g->csc_colptr ? (size_t)n + 1 : 0);
  nrp[0] = 0;
  for (int i = 0; i < n; ++i) nrp[i + 1] = nrp[i] + (rp[new2old[i] + 1] - rp[new2old[i]]);
  if (g->csc_colptr) {
    ncp[0] = 0;
    for (int i = 0; i < n; ++i) ncp[i + 1] = ncp[i] + (cp[new2old[i] + 1] - cp[new2old[i]]);
  }
  int *d_perm = (int *)(w + L.perm), *d_o2n = (int *)(w + L.old2new), *d_nrp = (int *)(w + L.nrowptr);
  HIP_TRY(hipMemcpyAsync(d_perm, new2old.data(), sizeof(int) * (size_t)n, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(d_o2n, old2new.data(), sizeof(int) * (size_t)n, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(d_nrp, nrp.data(), sizeof(int) * ((size_t)n + 1), hipMemcpyHostToDevice, c->stream));
  int *d_ncp = nullptr;
  if (g->csc_colptr) {
    d_ncp = (int *)(w + L.ncolptr);
    HIP_TRY(hipMemcpyAsync(d_ncp, ncp.data(), sizeof(int) * ((size_t)n + 1), hipMemcpyHostToDevice, c->stream));
  }
  const int grid = (int)std::max<long long>(1, std::min<long long>((g->nnz + BLOCK - 1) / BLOCK, 16384));
  int *ncol = (int *)(w + L.ncol);
  void *nval = g->csr_val ? (void *)(w + L.nval) : nullptr;
  if (c->prec == RLGL_FP64)
    k_relabel_side<double><<<grid, BLOCK, 0, c->stream>>>(n, g->csr_rowptr, g->csr_col, (const double *)g->csr_val,
                                                          d_perm, d_o2n, d_nrp, ncol, (double *)nval);
  else
    k_relabel_side<float><<<grid, BLOCK, 0, c->stream>>>(n, g->csr_rowptr, g->csr_col, (const float *)g->csr_val,
                                                         d_perm, d_o2n, d_nrp, ncol, (float *)nval);
  gi.csr_rowptr = d_nrp;
  gi.csr_col = ncol;
  gi.csr_val = nval;
  if (g->csc_colptr) {
    int *nrow = (int *)(w + L.nrow);
    void *ncval = g->csc_val ? (void *)(w + L.ncval) : nullptr;
    if (c->prec == RLGL_FP64)
      k_relabel_side<double><<<grid, BLOCK, 0, c->stream>>>(n, g->csc_colptr, g->csc_row,
                                                            (const double *)g->csc_val, d_perm, d_o2n, d_ncp, nrow,
                                                            (double *)ncval);
    else
      k_relabel_side<float><<<grid, BLOCK, 0, c->stream>>>(n, g->csc_colptr, g->csc_row, (const float *)g->csc_val,
                                                           d_perm, d_o2n, d_ncp, nrow, (float *)ncval);
    gi.csc_colptr = d_ncp;
    gi.csc_row = nrow;
    gi.csc_val = ncval;
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(c->stream));
  d.rowptr = gi.csr_rowptr;
  d.col = gi.csr_col;
  d.val = gi.csr_val;
  d.colptr = gi.csc_colptr;
  d.crow = gi.csc_row;
  d.cval = gi.csc_val;
  d.perm = d_perm;
  return RLGL_OK;
}

// The static plan of the single-chain pull from the CSC column pointers
// (host memory): RUN {k0, k1, p0, p1} (k0 >= 0) of whole columns with at most
// WL links and WCOLS columns, PIECE {-1 - slot, k, p0, p1} of at most WL links
// of a column with more than WL in-links (lng[slot] = k).  Every column is in
// exactly one run or is a long column, and every link in exactly one item.
bool pull_plan_host(const int *cp, int n, long long nnz, std::vector<int4> &items, std::vector<int> &lng,
                    std::string &why) {
  items.clear();
  lng.clear();
  if (n < 1 || cp[0] != 0 || (long long)cp[n] != nnz) {
    why = "csc_colptr[0] must be 0 and csc_colptr[n] = nnz";
    return false;
  }
  int run0 = -1, run_e = 0;
  auto flush = [&](int end) {
    if (run0 >= 0 && end > run0) items.push_back(make_int4(run0, end, cp[run0], cp[end]));
    run0 = -1;
    run_e = 0;
  };
  for (int k = 0; k < n; ++k) {
    const int dg = cp[k + 1] - cp[k];
    if (dg < 0) {
      why = "csc_colptr is not non-decreasing at " + std::to_string(k);
      return false;
    }
    if (dg > WL) {
      // a long column: pieces of WL links; the last one summed writes the column
      flush(k);
      const int slot = (int)lng.size();
      lng.push_back(k);
      for (int p = cp[k]; p < cp[k + 1]; p += WL)
        items.push_back(make_int4(-1 - slot, k, p, std::min(p + WL, cp[k + 1])));
      continue;
    }
    if (run0 >= 0 && (run_e + dg > WL || k - run0 >= WCOLS)) flush(k);
    if (run0 < 0) run0 = k;
    run_e += dg;
  }
  flush(n);
  // The pieces are spread evenly over the first three quarters of the runs:
  // a wave that sums a piece has two device-scope atomics in flight, which
  // costs little while the other waves keep their gathers going, but stalls
  // the pass when every wave takes a piece at once; the last column finished
  // leaves a quarter of the pass to hide behind.
  std::vector<int4> runs, pieces;
  for (const int4 &it : items) (it.x < 0 ? pieces : runs).push_back(it);
  const size_t span = (runs.size() * 3) / 4;
  items.clear();
  size_t r = 0;
  for (size_t q = 0; q < pieces.size(); ++q) {
    const size_t upto = span * (q + 1) / (pieces.size() + 1);
    while (r < upto) items.push_back(runs[r++]);
    items.push_back(pieces[q]);
  }
  while (r < runs.size()) items.push_back(runs[r++]);
  return true;
}

// Host-side construction of the static pull plan from the CSC column pointers.
rlgl_status build_plan(rlgl_ctx *c, const rlgl_graph *g, const Layout &L, char *ws) {
  const int n = g->n;
  std::vector<int> cp((size_t)n + 1);
  HIP_TRY(hipMemcpyAsync(cp.data(), g->csc_colptr, sizeof(int) * ((size_t)n + 1), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  std::vector<int4> items;
  std::vector<int> lng;
  std::string why;
  if (!pull_plan_host(cp.data(), n, g->nnz, items, lng, why)) return fail(RLGL_EINVAL, "%s", why.c_str());
  if (items.size() > L.max_items || lng.size() > L.max_long)
    return fail(RLGL_EINVAL, "pull plan exceeds its bound (internal)");
  if (!items.empty())
    HIP_TRY(hipMemcpyAsync(ws + L.items, items.data(), sizeof(int4) * items.size(), hipMemcpyHostToDevice, c->stream));
  if (!lng.empty())
    HIP_TRY(hipMemcpyAsync(ws + L.long_cols, lng.data(), sizeof(int) * lng.size(), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->d.items = (const int4 *)(ws + L.items);
  c->d.n_items = (int)items.size();
  c->d.long_cols = (const int *)(ws + L.long_cols);
  c->d.long_acc = (double *)(ws + L.long_acc);
  c->d.long_cnt = (int *)(ws + L.long_cnt);
  c->d.n_long = (int)lng.size();
  return RLGL_OK;
}

// Setup of the push route: the HOT_MAX destinations with the largest
// in-degrees (at least HOT_MIN_INDEG) get LDS accumulators, and a copy of
// the CSR columns tags them as -1 - slot.  In-degrees come from the CSC
// column pointers when given, else from a histogram of the CSR columns.
rlgl_status build_hot(rlgl_ctx *c, const rlgl_graph *g, const Layout &L, char *ws) {
  const int n = g->n;
  Dev &d = c->d;
  int *colt = (int *)(ws + L.colt);
  int *tmp = d.fr_id;  // n ints, free until the first push step
  std::vector<int> indeg((size_t)n);
  if (g->csc_colptr) {
    std::vector<int> cp((size_t)n + 1);
    HIP_TRY(hipMemcpyAsync(cp.data(), g->csc_colptr, sizeof(int) * ((size_t)n + 1), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (int k = 0; k < n; ++k) indeg[k] = cp[k + 1] - cp[k];
  } else {
    k_fill_int<<<c->grid_misc, BLOCK, 0, c->stream>>>(tmp, n, 0);
    if (g->nnz > 0) k_indegree<<<MAX_GRID, BLOCK, 0, c->stream>>>(d, tmp);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(indeg.data(), tmp, sizeof(int) * (size_t)n, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  std::vector<int> hot;
  for (int k = 0; k < n; ++k)
    if (indeg[k] >= HOT_MIN_INDEG) hot.push_back(k);
  std::sort(hot.begin(), hot.end(), [&](int a, int b) { return indeg[a] != indeg[b] ? indeg[a] > indeg[b] : a < b; });
  if ((int)hot.size() > HOT_MAX) hot.resize(HOT_MAX);
  d.n_hot = (int)hot.size();
  if (g->nnz > 0) {
    k_fill_int<<<c->grid_misc, BLOCK, 0, c->stream>>>(tmp, n, -1);
    if (!hot.empty()) {
      HIP_TRY(hipMemcpyAsync((void *)d.hot_nodes, hot.data(), sizeof(int) * hot.size(), hipMemcpyHostToDevice,
                             c->stream));
      k_scatter_slots<<<1, BLOCK, 0, c->stream>>>(d.hot_nodes, d.n_hot, tmp);
    }
    k_tag_columns<<<MAX_GRID, BLOCK, 0, c->stream>>>(d, colt, tmp);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(c->stream));
    d.colt = colt;
  }
  return RLGL_OK;
}

}  // namespace

extern "C" {

void rlgl_default_options(rlgl_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->sched = RLGL_SCHED_THRESHOLD;
  o->r = 1.0;
  o->k = 1;
  o->theta_period = 1;
  o->precision = RLGL_FP32C_FP64H;
  o->route = RLGL_ROUTE_AUTO;
  o->pull_alpha = 0.05;
  o->check_period = 0;
  o->record_green = 0;
  o->refresh = 1;
}

const char *rlgl_last_error(void) { return g_err.c_str(); }

size_t rlgl_validate_scratch_bytes(const rlgl_graph *g) {
  if (!g || g->n < 1) return 0;
  return sizeof(VHead) + align_up(4 * (size_t)g->n, 256);
}

rlgl_status rlgl_validate(const rlgl_graph *g, int32_t precision, void *dev_scratch, size_t scratch_bytes,
                          void *stream, double *max_row_dev) {
  if (!g) return fail(RLGL_EINVAL, "null graph");
  if (precision < 0 || precision > 2) return fail(RLGL_EINVAL, "precision out of range");
  const int n = g->n;
  const long long nnz = g->nnz;
  if (n < 1 || nnz < 0 || nnz >= (1ll << 31)) return fail(RLGL_EINVAL, "n or nnz out of range");
  if (!g->csr_rowptr || (nnz > 0 && !g->csr_col)) return fail(RLGL_EINVAL, "CSR arrays are NULL");
  if (g->csc_colptr && nnz > 0 && !g->csc_row) return fail(RLGL_EINVAL, "csc_row is NULL");
  if (!dev_scratch || scratch_bytes < rlgl_validate_scratch_bytes(g))
    return fail(RLGL_ENOMEM, "scratch smaller than rlgl_validate_scratch_bytes()");
  hipStream_t st = (hipStream_t)stream;
  VHead *h = (VHead *)dev_scratch;
  int *indeg = (int *)((char *)dev_scratch + sizeof(VHead));
  const int grid = std::max(1, std::min((n + BLOCK - 1) / BLOCK, MAX_GRID));
  const bool dbl = precision == RLGL_FP64;
  // values enter the link hashes only when both sides store them
  const int hv = (g->csr_val && g->csc_val) ? 1 : 0;
  const double tol = dbl ? 1e-12 : 1e-6;
  k_v_clear<<<grid, BLOCK, 0, st>>>(h, indeg, n);
  if (dbl)
    k_v_rows<double><<<grid, BLOCK, 0, st>>>(n, nnz, g->csr_rowptr, g->csr_col, (const double *)g->csr_val, hv, tol,
                                            h, indeg);
  else
    k_v_rows<float><<<grid, BLOCK, 0, st>>>(n, nnz, g->csr_rowptr, g->csr_col, (const float *)g->csr_val, hv, tol, h,
                                           indeg);
  if (g->csc_colptr) {
    if (dbl)
      k_v_cols<double><<<grid, BLOCK, 0, st>>>(n, nnz, g->csc_colptr, g->csc_row, (const double *)g->csc_val, hv, h,
                                              indeg);
    else
      k_v_cols<float><<<grid, BLOCK, 0, st>>>(n, nnz, g->csc_colptr, g->csc_row, (const float *)g->csc_val, hv, h,
                                             indeg);
  }
  HIP_TRY(hipGetLastError());
  VHead r{};
  HIP_TRY(hipMemcpyAsync(&r, h, sizeof(VHead), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (max_row_dev) *max_row_dev = __builtin_bit_cast(double, r.dev_bits);
  const unsigned int f = r.flags;
  if (f & VF_ROWPTR) return fail(RLGL_EINVAL, "csr_rowptr does not run from 0 to nnz without decreasing");
  if (f & VF_COL) return fail(RLGL_EINVAL, "a csr_col entry is outside [0, n)");
  if (f & VF_VAL) return fail(RLGL_EINVAL, "a csr_val entry is negative or not finite");
  if (f & VF_ROWSUM)
    return fail(RLGL_EINVAL, "a row of csr_val does not sum to 1 (max deviation %.3g, tolerance %.1g)",
                __builtin_bit_cast(double, r.dev_bits), tol);
  if (f & VF_COLPTR) return fail(RLGL_EINVAL, "csc_colptr does not run from 0 to nnz without decreasing");
  if (f & VF_ROW) return fail(RLGL_EINVAL, "a csc_row entry is outside [0, n)");
  if (f & VF_CVAL) return fail(RLGL_EINVAL, "a csc_val entry is negative or not finite");
  if (f & VF_INDEG) return fail(RLGL_EINVAL, "the CSC column lengths differ from the CSR in-degrees");
  if (g->csc_colptr && r.h_csr != r.h_csc)
    return fail(RLGL_EINVAL, "the CSC does not hold the same links%s as the CSR", hv ? " and values" : "");
  return RLGL_OK;
}

size_t rlgl_workspace_bytes(const rlgl_graph *g, const rlgl_options *o) {
  if (!g || !o || g->n < 1 || g->nnz < 0 || o->precision < 0 || o->precision > 2) return 0;
  return make_layout(g->n, g->nnz, o->precision, g->csc_colptr != nullptr, o->relabel != 0, g->csr_val != nullptr,
                     o->sched == RLGL_SCHED_TOPK)
      .total;
}

rlgl_status rlgl_create(const rlgl_graph *g, const rlgl_options *o, void *ws, size_t ws_bytes, void *stream,
                        rlgl_ctx **out) {
  if (!g || !o || !out) return fail(RLGL_EINVAL, "null argument");
  *out = nullptr;
  std::string why;
  if (!valid_options(o, why)) return fail(RLGL_EINVAL, "options: %s", why.c_str());
  if (g->n < 1) return fail(RLGL_EINVAL, "n must be >= 1");
  if (g->nnz < 0 || g->nnz >= (1ll << 31)) return fail(RLGL_EINVAL, "nnz must be in [0, 2^31)");
  if (!(g->damping > 0.0 && g->damping <= 1.0)) return fail(RLGL_EINVAL, "damping must be in (0, 1]");
  if (!g->csr_rowptr || (g->nnz > 0 && !g->csr_col)) return fail(RLGL_EINVAL, "CSR arrays missing");
  if (g->csc_colptr && (g->nnz > 0 && !g->csc_row)) return fail(RLGL_EINVAL, "csc_row missing");
  if (o->route == RLGL_ROUTE_PULL && !g->csc_colptr) return fail(RLGL_EINVAL, "pull routing needs the CSC arrays");
  if ((g->csr_val == nullptr) != (g->csc_colptr ? g->csc_val == nullptr : g->csr_val == nullptr))
    return fail(RLGL_EINVAL, "csr_val and csc_val must both be given or both be NULL");
  if (!ws) return fail(RLGL_EINVAL, "workspace is NULL");
  const Layout L = make_layout(g->n, g->nnz, o->precision, g->csc_colptr != nullptr, o->relabel != 0,
                               g->csr_val != nullptr, o->sched == RLGL_SCHED_TOPK);
  if (ws_bytes < L.total) return fail(RLGL_ENOMEM, "workspace too small: %zu < %zu", ws_bytes, L.total);

  rlgl_ctx *c = new (std::nothrow) rlgl_ctx();
  if (!c) return fail(RLGL_ENOMEM, "host allocation failed");
  c->stream = (hipStream_t)stream;
  c->prec = o->precision;
  c->hk = (o->precision == RLGL_FP32C_KAHANH);
  c->prof = false;
  char *w = (char *)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
  Dev &d = c->d;
  d.n = g->n;
  d.nnz = g->nnz;
  d.c = g->damping;
  d.rowptr = g->csr_rowptr;
  d.col = g->csr_col;
  d.val = g->csr_val;
  d.colptr = g->csc_colptr;
  d.crow = g->csc_row;
  d.cval = g->csc_val;
  d.sched = o->sched;
  d.r = o->r;
  d.k = o->k;
  d.theta_period = o->theta_period;
  d.route = g->csc_colptr ? o->route : RLGL_ROUTE_PUSH;
  d.pull_alpha = o->pull_alpha;
  d.seed = o->seed;
  d.green_in = nullptr;
  d.cash[0] = w + L.cash0;
  d.cash[1] = w + L.cash1;
  d.hist = w + L.hist;
  d.hist_lo = c->hk ? (float *)(w + L.hist_lo) : nullptr;
  d.fr_rowstart = (int *)(w + L.fr_rowstart);
  d.fr_eoff = (int *)(w + L.fr_eoff);
  d.fr_id = (int *)(w + L.fr_id);
  d.fr_scale = w + L.fr_scale;
  d.chunk_first = (int *)(w + L.chunk_first);
  d.green_mask = o->record_green ? (unsigned char *)(w + L.green_mask) : nullptr;
  d.delta = (o->precision == RLGL_FP64) ? nullptr : (double *)(w + L.delta);
  // the pull's per-node send values take the push frontier's scale array (a
  // step pulls or pushes, never both); the refresh's FP64 ones take the FP64
  // push accumulators, or that same array when the cash is FP64
  d.src = d.fr_scale;
  d.rsrc = (o->precision == RLGL_FP64) ? (double *)d.fr_scale : d.delta;
  d.colt = nullptr;
  d.hot_nodes = (const int *)(w + L.hot_nodes);
  d.n_hot = 0;
  c->has_mask = o->record_green != 0;
  c->check_period = o->check_period;
  c->refresh = g->csc_colptr ? o->refresh : 0;
  d.rec = (Rec *)(w + L.rec);
  d.glob = (Glob *)(w + L.glob);
  d.log = (StepLog *)(w + L.log);
  d.items = nullptr;
  d.n_items = 0;
  d.long_cols = nullptr;
  d.long_acc = nullptr;
  d.long_cnt = nullptr;
  d.n_long = 0;
  d.perm = nullptr;
  const bool topk = o->sched == RLGL_SCHED_TOPK;
  d.khist = topk ? (unsigned int *)(w + L.khist) : nullptr;
  d.tk_ckey = topk ? (unsigned long long *)(w + L.tk_ckey) : nullptr;
  d.tk_cid = topk ? (int *)(w + L.tk_cid) : nullptr;
  d.tk_hist = topk ? (unsigned int *)(w + L.tk_hist) : nullptr;
  d.tk_cnt = topk ? (int *)(w + L.tk_cnt) : nullptr;
  d.tk_seg = (topk && c->prec != RLGL_FP64) ? (unsigned int *)(w + L.tk_seg) : nullptr;
  c->khist_stale = false;

  const int tiles = (g->n + TILE - 1) / TILE;
  c->grid_sel = std::max(1, std::min(tiles, SEL_GRID));
  d.tk_grid = std::min(c->grid_sel, TK_GRID);  // workgroups of the collecting pass
  c->grid_push = (int)std::max<long long>(1, std::min<long long>((g->nnz + CH - 1) / CH, PUSH_GRID));
  c->grid_misc = std::max(1, std::min((g->n + BLOCK - 1) / BLOCK, NODE_GRID));

  rlgl_status st = RLGL_OK;
  // one pinned block mirrors the device's records followed by the status
  // word (their order in the workspace), so a read-back is one copy
  void *stage = nullptr;
  if (hipHostMalloc(&stage, record_span(), hipHostMallocDefault) != hipSuccess) {
    st = fail(RLGL_EHIP, "pinned host allocation failed");
  } else {
    c->host_rec = (Rec *)stage;
    c->host_glob = (Glob *)((char *)stage + records_bytes());
  }
  if (st == RLGL_OK) {
    int last = 0;
    if (hipMemcpyAsync(&last, g->csr_rowptr + g->n, sizeof(int), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
      st = fail(RLGL_EHIP, "reading csr_rowptr[n] failed");
    else if ((long long)last != g->nnz)
      st = fail(RLGL_EINVAL, "csr_rowptr[n] = %d differs from nnz = %lld", last, (long long)g->nnz);
  }
  rlgl_graph gi = *g;  // the graph the kernels see: the caller's, or its relabelled copy
  if (st == RLGL_OK && o->relabel) st = relabel_graph(c, g, L, w, gi);
  if (st == RLGL_OK && gi.csc_colptr) st = build_plan(c, &gi, L, w);
  if (st == RLGL_OK) st = build_hot(c, &gi, L, w);
  if (st == RLGL_OK) {
    // the pull's waves take items until the plan is done: one round of
    // workgroups, as many as stay resident together, keeps every wave's
    // one-item-ahead loads flowing from start to end
    // (FP32 cash: one workgroup of PULL_WIDE waves per CU, whose LDS stages
    // the send values of four times as many sources; the refresh keeps
    // four workgroups of NWAVE waves)
    int dev = 0, cus = 0, per_cu = 0, per_cu_w = 0;
    c->pull_wide = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) ||
        complete_occupancy(c, &per_cu) != hipSuccess || cus < 1 || per_cu < 1) {
      st = fail(RLGL_EHIP, "occupancy query failed");
    } else {
      c->grid_cmp = std::max({1, std::min(tiles, NODE_GRID), std::min(d.n_items, cus * per_cu)});
      c->grid_pull = c->grid_cmp;
      if (c->prec != RLGL_FP64 && gi.csc_colptr) {
        c->pull_wide = 1;
        if (complete_occupancy(c, &per_cu_w) != hipSuccess || per_cu_w < 1)
          st = fail(RLGL_EHIP, "occupancy query failed");
        else
          c->grid_pull = std::max(1, std::min(d.n_items > 0 ? d.n_items : 1, cus * per_cu_w));
      }
    }
  }
  if (st == RLGL_OK) st = reset_device(c);
  if (st != RLGL_OK) {
    rlgl_destroy(c);
    return st;
  }
  *out = c;
  return RLGL_OK;
}

void rlgl_destroy(rlgl_ctx *c) {
  if (!c) return;
  for (auto &L : c->launches) {
    (void)hipEventDestroy(L.a);
    (void)hipEventDestroy(L.b);
  }
  for (auto e : c->free_events) (void)hipEventDestroy(e);
  if (c->host_rec) (void)hipHostFree(c->host_rec);  // holds host_glob too
  delete c;
}

rlgl_status rlgl_reset(rlgl_ctx *c) {
  if (!c) return fail(RLGL_EINVAL, "null context");
  return reset_device(c);
}

rlgl_status rlgl_step(rlgl_ctx *c, int32_t nsteps, rlgl_step_info *info) {
  if (!c || nsteps < 0) return fail(RLGL_EINVAL, "bad argument");
  k_set_status<<<1, 64, 0, c->stream>>>(c->d.glob, 0);
  HIP_TRY(hipGetLastError());
  const long long s0 = c->t;
  for (long long s = s0; s < s0 + nsteps; ++s) HIP_TRY(enqueue_step(c, s, -1.0, s0 + nsteps, 0));
  rlgl_status st = read_back(c);
  if (st != RLGL_OK) return st;
  const int ds = c->host_glob->status;
  const rlgl_status rs = (ds == ST_ZERO_HISTORY || ds == ST_NONFINITE) ? status_of(ds) : RLGL_OK;
  fill_info(c, info, rs);
  if (rs != RLGL_OK) return fail(rs, "stopped at t = %lld (device status %d)", c->t, ds);
  return RLGL_OK;
}

rlgl_status rlgl_step_mask(rlgl_ctx *c, const uint8_t *dev_mask, rlgl_step_info *info) {
  if (!c || !dev_mask) return fail(RLGL_EINVAL, "null argument");
  if (c->d.perm) return fail(RLGL_EINVAL, "a caller-given green set needs the caller's numbering (relabel = 0)");
  k_set_status<<<1, 64, 0, c->stream>>>(c->d.glob, 0);
  HIP_TRY(hipGetLastError());
  // the kernels take the descriptor by value at launch, so the mask
  // schedule lives for this one step only
  const int sched = c->d.sched;
  c->d.sched = SCHED_MASK;
  c->d.green_in = (const unsigned char *)dev_mask;
  const long long s0 = c->t;
  const hipError_t e = enqueue_step(c, s0, -1.0, s0 + 1, 0);
  c->d.sched = sched;
  c->d.green_in = nullptr;
  c->khist_stale = true;  // that step's complete pass counted no histogram
  HIP_TRY(e);
  rlgl_status st = read_back(c);
  if (st != RLGL_OK) return st;
  const int ds = c->host_glob->status;
  const rlgl_status rs = (ds == ST_ZERO_HISTORY || ds == ST_NONFINITE) ? status_of(ds) : RLGL_OK;
  fill_info(c, info, rs);
  if (rs != RLGL_OK) return fail(rs, "stopped at t = %lld (device status %d)", c->t, ds);
  return RLGL_OK;
}

rlgl_status rlgl_solve(rlgl_ctx *c, double eps, int64_t max_steps, double *dev_pi, rlgl_step_info *info) {
  if (!c || max_steps < 0 || !(eps >= 0.0)) return fail(RLGL_EINVAL, "bad argument");
  k_set_status<<<1, 64, 0, c->stream>>>(c->d.glob, 0);
  HIP_TRY(hipGetLastError());
  const long long s_limit = c->t + max_steps;
  long long batch = c->check_period > 0 ? c->check_period : (c->d.sched == SCHED_MAXC ? 64 : 8);
  double prev_resid = -1.0;
  long long prev_t = c->t, refreshed_at = -1, last_refresh = c->t;
  int ds = 0;
  for (;;) {
    const long long s = c->t;
    long long nb = batch;
    if (s + nb > s_limit + 1) nb = s_limit + 1 - s;
    if (nb < 1) nb = 1;
    for (long long q = 0; q < nb; ++q) HIP_TRY(enqueue_step(c, s + q, eps, s_limit, 0));
    rlgl_status st = read_back(c);
    if (st != RLGL_OK) return st;
    ds = c->host_glob->status;
    if (ds == ST_CONVERGED && c->refresh > 0 && refreshed_at != c->t) {
      // accept the stop only on the cash rebuilt from the history; one step
      // is enqueued to re-run the stop test on it, and read back with it
      st = do_refresh(c, false);
      if (st != RLGL_OK) return st;
      refreshed_at = last_refresh = c->t;
      batch = 1;
      continue;
    }
    if (ds != 0) break;
    const Tot cur = host_totals(c->host_rec[c->t % 3]);
    const bool drift = std::fabs(cur.csum) > 0.5 * cur.l1;
    const bool periodic = c->refresh > 1 && c->t - last_refresh >= c->refresh;
    if (c->refresh > 0 && (drift || periodic) && refreshed_at != c->t) {
      st = do_refresh(c);
      if (st != RLGL_OK) return st;
      refreshed_at = last_refresh = c->t;
    }
    // size the next batch from the contraction seen so far
    const Rec &now = c->host_rec[c->t % 3];
    const double resid = now.hsum != 0.0 ? host_totals(now).l1 / std::fabs(now.hsum) : INFINITY;
    long long next = batch * 2;
    if (prev_resid > 0.0 && resid > 0.0 && resid < prev_resid && c->t > prev_t) {
      const double rate = std::pow(resid / prev_resid, 1.0 / (double)(c->t - prev_t));
      // steps until the stop test passes, plus the step that runs the test
      if (rate < 1.0 && resid > eps) next = (long long)std::ceil(std::log(eps / resid) / std::log(rate)) + 1;
    }
    if (c->d.sched == SCHED_MAXC) next = std::max(next, (long long)256);
    batch = std::max(1ll, std::min(next, 4096ll));
    if (c->check_period > 0) batch = c->check_period;
    prev_resid = resid;
    prev_t = c->t;
  }
  if (dev_pi) {
    if (c->hk) k_normalize<1><<<c->grid_misc, BLOCK, 0, c->stream>>>(c->d, dev_pi);
    else k_normalize<0><<<c->grid_misc, BLOCK, 0, c->stream>>>(c->d, dev_pi);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  const rlgl_status rs = (ds == ST_CONVERGED) ? RLGL_OK : status_of(ds);
  fill_info(c, info, rs);
  if (rs != RLGL_OK) return fail(rs, "solve stopped at t = %lld (device status %d)", c->t, ds);
  return RLGL_OK;
}

rlgl_status rlgl_refresh(rlgl_ctx *c, rlgl_step_info *info) {
  if (!c) return fail(RLGL_EINVAL, "null context");
  rlgl_status st = do_refresh(c);
  if (st != RLGL_OK) return st;
  fill_info(c, info, RLGL_OK);
  return RLGL_OK;
}

rlgl_status rlgl_get_state(rlgl_ctx *c, double *dC, double *dH, rlgl_step_info *info) {
  if (!c) return fail(RLGL_EINVAL, "null context");
  if (dC || dH) {
    if (c->prec == RLGL_FP64) k_export<double, 0><<<c->grid_misc, BLOCK, 0, c->stream>>>(c->d, dC, dH);
    else if (c->hk) k_export<float, 1><<<c->grid_misc, BLOCK, 0, c->stream>>>(c->d, dC, dH);
    else k_export<float, 0><<<c->grid_misc, BLOCK, 0, c->stream>>>(c->d, dC, dH);
    HIP_TRY(hipGetLastError());
  }
  rlgl_status st = read_back(c);
  if (st != RLGL_OK) return st;
  fill_info(c, info, RLGL_OK);
  return RLGL_OK;
}

rlgl_status rlgl_set_state(rlgl_ctx *c, const double *dC, const double *dH, double h_sum, int64_t t) {
  if (!c || !dC || !dH || t < 1) return fail(RLGL_EINVAL, "bad argument");
  const int buf = 0;
  k_prepare_import<<<3, 64, 0, c->stream>>>(c->d, t, buf);
  if (c->prec == RLGL_FP64) k_import<double, 0><<<c->grid_misc, BLOCK, 0, c->stream>>>(c->d, dC, dH, t, buf);
  else if (c->hk) k_import<float, 1><<<c->grid_misc, BLOCK, 0, c->stream>>>(c->d, dC, dH, t, buf);
  else k_import<float, 0><<<c->grid_misc, BLOCK, 0, c->stream>>>(c->d, dC, dH, t, buf);
  k_finish_import<<<1, 64, 0, c->stream>>>(c->d, t, h_sum);
  HIP_TRY(hipGetLastError());
  c->khist_stale = true;
  return read_back(c);
}

rlgl_status rlgl_get_green(rlgl_ctx *c, uint8_t *dmask) {
  if (!c || !dmask) return fail(RLGL_EINVAL, "bad argument");
  if (!c->has_mask) return fail(RLGL_EINVAL, "the context was created without record_green");
  if (c->d.perm) {
    k_export_mask<<<c->grid_misc, BLOCK, 0, c->stream>>>(c->d, dmask);
    HIP_TRY(hipGetLastError());
  } else {
    HIP_TRY(hipMemcpyAsync(dmask, c->d.green_mask, (size_t)c->d.n, hipMemcpyDeviceToDevice, c->stream));
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  return RLGL_OK;
}

rlgl_status rlgl_profile_enable(rlgl_ctx *c, int32_t on) {
  if (!c) return fail(RLGL_EINVAL, "null context");
  c->prof = on != 0;
  return RLGL_OK;
}

int32_t rlgl_profile_read(rlgl_ctx *c, rlgl_kernel_stat *out, int32_t max_entries) {
  if (!c || !out || max_entries < 0) return fail(RLGL_EINVAL, "bad argument");
  if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(RLGL_EHIP, "synchronize failed");
  std::vector<StepLog> log(LOG_STEPS);
  if (hipMemcpy(log.data(), c->d.log, sizeof(StepLog) * LOG_STEPS, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(RLGL_EHIP, "reading the step log failed");
  const double cs = (c->prec == RLGL_FP64) ? 8.0 : 4.0;
  const double vs = c->d.val ? cs : 0.0;
  const double hb = 16.0;  // history read-modify-write per green node
  const double n = (double)c->d.n, nnz = (double)c->d.nnz;
  double ms[KS_N] = {0}, bytes[KS_N] = {0}, touched[KS_N] = {0};
  long long cnt[KS_N] = {0}, links[KS_N] = {0};
  for (auto &L : c->launches) {
    const StepLog &lg = log[L.s % LOG_STEPS];
    if (lg.s != L.s) continue;  // launch of a step that never ran (after the stop) or fell off the ring
    const bool push = lg.mode == 0;
    const double ge = (double)lg.gedges;
    double b = 0.0, bt = 0.0;
    if (L.kind == KS_SELECT) {
      b = cs * n + (double)lg.green * (8.0 + hb);
      if (push) b += (double)lg.nfront * (4 + 4 + 4 + cs) + (double)lg.green * cs;
      else b += cs * n;  // what each node sends along its links in the pull
      bt = b;
    } else if (L.kind == KS_PUSH) {
      if (!push) continue;
      b = ge * (4.0 + vs + 2.0 * cs) + (double)lg.nfront * (8.0 + cs);
      bt = ge * (4.0 + vs + (c->d.delta ? 16.0 : 2.0 * cs)) + (double)lg.nfront * (12.0 + cs);
    } else if (L.kind == KS_COMPLETE) {
      if (push) {
        b = 2.0 * cs * n;
        bt = b + (c->d.delta ? 16.0 * n : 0.0);
      } else {
        // per link of a green node: source index, stored value, gathered
        // moved cash; per node: column pointer, cash read and write, moved cash
        b = ge * (4.0 + vs + cs) + n * (4.0 + 3.0 * cs);
        bt = nnz * (4.0 + vs + cs) + n * (4.0 + 3.0 * cs);
      }
    }
    float e = 0.f;
    (void)hipEventElapsedTime(&e, L.a, L.b);
    ms[L.kind] += e;
    bytes[L.kind] += b;
    touched[L.kind] += bt;
    links[L.kind] += (L.kind == KS_SELECT || L.kind == KS_TOPK) ? 0 : lg.gedges;
    cnt[L.kind] += 1;
  }
  for (auto &L : c->launches) {
    c->free_events.push_back(L.a);
    c->free_events.push_back(L.b);
  }
  c->launches.clear();
  int m = 0;
  for (int k = 0; k < KS_N && m < max_entries; ++k) {
    if (!cnt[k]) continue;
    std::memset(&out[m], 0, sizeof out[m]);
    std::snprintf(out[m].name, sizeof out[m].name, "%s", kernel_names[k]);
    out[m].launches = cnt[k];
    out[m].ms = ms[k];
    out[m].bytes = bytes[k];
    out[m].bytes_touched = touched[k];
    out[m].green_links = links[k];
    ++m;
  }
  return m;
}


// ------------------------------------------------------------ batched solves

}  // extern "C"

namespace {

// ---- the step-synchronous engine (shared by batched solves and the pool)

size_t ls_device_bytes(int cap) {
  return align_up(sizeof(LsChain) * (size_t)cap, 256) + align_up(sizeof(LsCtl) * (size_t)cap, 256) +
         align_up(sizeof(LsStripe) * LS_NS * (size_t)cap, 256) + align_up(4 * (4 * (size_t)cap + 3), 256) + 256;
}

struct LsEngine {
  hipStream_t stream = nullptr;
  int prec = 0, hk = 0, nt = 256, cap = 0;
  LsArgs args{};
  LsChain *d_chains = nullptr;
  int *d_lists = nullptr;  // act [cap] | tpre [cap+1] | wpre [cap+1] (pieces) | rpre [cap+1] (runs)
  int *h_lists = nullptr;  // pinned staging of d_lists
  LsCtl *h_ctl = nullptr;  // pinned [cap]
  unsigned int *h_done = nullptr;
  hipEvent_t staged = nullptr;
  bool staged_pending = false;
  int t_total = 0;
  int route_grid = 0;         // route workgroups the plan items are strided over; 0: one per item
  std::vector<LsChain> host;  // descriptors as on the device
  std::vector<int> act;
};

rlgl_status ls_init(LsEngine &E, char *ws, int cap, int prec, int sched, double r, int refresh, hipStream_t stream) {
  E.stream = stream;
  E.prec = prec;
  E.hk = prec == RLGL_FP32C_KAHANH;
  E.cap = cap;
  char *w = (char *)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char *p = w + off;
    off = align_up(off + bytes, 256);
    return p;
  };
  E.d_chains = (LsChain *)take(sizeof(LsChain) * (size_t)cap);
  LsArgs &a = E.args;
  a.chains = E.d_chains;
  a.ctl = (LsCtl *)take(sizeof(LsCtl) * (size_t)cap);
  a.stats = (LsStripe *)take(sizeof(LsStripe) * LS_NS * (size_t)cap);
  E.d_lists = (int *)take(4 * (4 * (size_t)cap + 3));
  a.done = (unsigned int *)take(256);
  a.act = E.d_lists;
  a.tpre = E.d_lists + cap;
  a.wpre = E.d_lists + 2 * cap + 1;
  a.rpre = E.d_lists + 3 * cap + 2;
  a.n_act = 0;
  a.w_total = 0;
  a.r_total = 0;
  a.sched = sched;
  a.refresh = refresh ? 1 : 0;
  a.r = r;
  E.host.assign((size_t)cap, LsChain{});
  HIP_TRY(hipHostMalloc((void **)&E.h_lists, 4 * (4 * (size_t)cap + 3), hipHostMallocDefault));
  HIP_TRY(hipHostMalloc((void **)&E.h_ctl, sizeof(LsCtl) * (size_t)cap, hipHostMallocDefault));
  HIP_TRY(hipHostMalloc((void **)&E.h_done, sizeof(unsigned int), hipHostMallocDefault));
  HIP_TRY(hipEventCreateWithFlags(&E.staged, hipEventDisableTiming));
  return RLGL_OK;
}

void ls_free(LsEngine &E) {
  if (E.staged) {
    (void)hipEventSynchronize(E.staged);
    (void)hipEventDestroy(E.staged);
  }
  if (E.h_lists) (void)hipHostFree(E.h_lists);
  if (E.h_ctl) (void)hipHostFree(E.h_ctl);
  if (E.h_done) (void)hipHostFree(E.h_done);
  E = LsEngine{};
}

// Makes `ids` the active slots (launch order: long columns of every chain
// first, then the runs, chain by chain in the order given).
rlgl_status ls_set_active(LsEngine &E, const std::vector<int> &ids) {
  if ((int)ids.size() > E.cap) return fail(RLGL_EINVAL, "active list longer than the engine capacity");
  if (E.staged_pending) HIP_TRY(hipEventSynchronize(E.staged));
  const int cap = E.cap, na = (int)ids.size();
  int *act = E.h_lists, *tp = E.h_lists + cap, *wp = E.h_lists + 2 * cap + 1, *rp = E.h_lists + 3 * cap + 2;
  long long tt = 0, tw = 0, tr = 0;
  for (int q = 0; q < na; ++q) {
    const LsChain &ch = E.host[ids[q]];
    act[q] = ids[q];
    tp[q] = (int)tt;
    wp[q] = (int)tw;
    rp[q] = (int)tr;
    tt += (ch.n + LS_TILE - 1) / LS_TILE;
    tw += ch.n_piece;
    tr += ch.n_run;
  }
  if (tt >= INT32_MAX || tw + tr >= INT32_MAX) return fail(RLGL_EINVAL, "active chains exceed the launch grid");
  tp[na] = (int)tt;
  wp[na] = (int)tw;
  rp[na] = (int)tr;
  HIP_TRY(hipMemcpyAsync(E.d_lists, E.h_lists, 4 * (4 * (size_t)cap + 3), hipMemcpyHostToDevice, E.stream));
  HIP_TRY(hipEventRecord(E.staged, E.stream));
  E.staged_pending = true;
  E.act = ids;
  E.args.n_act = na;
  E.args.w_total = (int)tw;
  E.args.r_total = (int)tr;
  E.t_total = (int)tt;
  return RLGL_OK;
}

template <class T, int HK>
void ls_launch(LsEngine &E) {
  const LsArgs &a = E.args;
  k_ls_select<T, HK><<<E.t_total, BLOCK, 0, E.stream>>>(a);
  const int items = a.w_total + a.r_total;
  if (items > 0 && E.route_grid <= 0) {
    // one workgroup per plan item
    if (E.nt == 512) k_ls_route<T, HK, 512><<<items, 512, 0, E.stream>>>(a);
    else k_ls_route<T, HK, 256><<<items, 256, 0, E.stream>>>(a);
  } else if (items > 0) {
    const int rg = std::min(items, E.route_grid);
    if (E.nt == 512) k_ls_route_strided<T, HK, 512><<<rg, 512, 0, E.stream>>>(a);
    else k_ls_route_strided<T, HK, 256><<<rg, 256, 0, E.stream>>>(a);
  }
  k_ls_control<T, HK><<<a.n_act, 64, 0, E.stream>>>(a);
}

rlgl_status ls_iterate(LsEngine &E, int count) {
  if (E.args.n_act == 0) return RLGL_OK;
  for (int i = 0; i < count; ++i) {
    if (E.prec == RLGL_FP64) ls_launch<double, 0>(E);
    else if (E.hk) ls_launch<float, 1>(E);
    else ls_launch<float, 0>(E);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(RLGL_EHIP, "lockstep launch: %s", hipGetErrorString(e));
  return RLGL_OK;
}

// Chain plan: the long columns (> CH links) first, as pieces of at most
// LS_PIECE links that add into long_acc[q] of the column's position q in
// long_cols, then runs of at most CH links and RUN_MAX_COLS columns.
// Returns false on a bad colptr.
bool chain_plan(const int *c, int n, int m, std::vector<int4> &items, std::vector<int> &long_cols,
                int &n_first, int &n_run, std::string &why) {
  if (c[0] != 0 || c[n] != m) {
    why = "csc_colptr must run from 0 to the link count";
    return false;
  }
  const size_t first = items.size();
  const size_t lfirst = long_cols.size();
  for (int q = 0; q < n; ++q) {
    const int dg = c[q + 1] - c[q];
    if (dg < 0) {
      why = "csc_colptr decreases";
      return false;
    }
    if (dg <= CH) continue;
    const int slot = (int)(long_cols.size() - lfirst);
    long_cols.push_back(q);
    for (int p = c[q]; p < c[q + 1]; p += LS_PIECE)
      items.push_back(make_int4(-1 - slot, q, p, std::min(p + LS_PIECE, c[q + 1])));
  }
  n_first = (int)(items.size() - first);
  int run0 = -1, run_e = 0;
  auto flush = [&](int end) {
    if (run0 >= 0 && end > run0) items.push_back(make_int4(run0, end, c[run0], c[end]));
    run0 = -1;
    run_e = 0;
  };
  for (int q = 0; q < n; ++q) {
    const int dg = c[q + 1] - c[q];
    if (dg > CH) {
      flush(q);
      continue;
    }
    if (run0 >= 0 && (run_e + dg > CH || q - run0 >= RUN_MAX_COLS)) flush(q);
    if (run0 < 0) run0 = q;
    run_e += dg;
  }
  flush(n);
  n_run = (int)(items.size() - first) - n_first;
  return true;
}

size_t long_col_bound(long long nnz) { return (size_t)(nnz / (CH + 1) + 1); }

size_t batch_item_bound(long long n, long long nnz) {
  // runs (see build_plan) plus the pieces of the columns longer than CH
  return 3 * (size_t)(nnz / CH + 2) + (size_t)(n / RUN_MAX_COLS + 2) + (size_t)(nnz / LS_PIECE + 1) +
         2 * long_col_bound(nnz);
}

// Per-chain outcome of a batched solve, gathered on the host.
struct ChainOut {
  long long t, edges;
  double resid, hsum;
  int status, green_steps;
  long long t0, t1;  // device wall clock at start and end of the chain's solve
};

struct BatchLayout {
  size_t cash0, cash1, src, hist, hist_lo, ls_items, long_cols, long_acc, order, queue, engine, total;
  size_t max_items, max_long;
  size_t nrowptr, ncolptr, nrow, perm;  // relabelled layout (0 without)
};

bool batch_layout(const rlgl_batch_graphs *g, const rlgl_batch_options *o, BatchLayout &L, std::string &why) {
  if (!g || !o || g->n_chains < 1 || !g->node_off || !g->edge_off) { why = "bad batch description"; return false; }
  if (o->precision < 0 || o->precision > 2) { why = "precision out of range"; return false; }
  if (g->node_off[0] != 0 || g->edge_off[0] != 0) { why = "node_off[0] and edge_off[0] must be 0"; return false; }
  const long long tn = g->node_off[g->n_chains];
  size_t items = 0, longs = 0;
  for (int k = 0; k < g->n_chains; ++k) {
    const long long n = g->node_off[k + 1] - g->node_off[k], m = g->edge_off[k + 1] - g->edge_off[k];
    if (n < 1 || n >= (1ll << 31) || m < 0 || m >= (1ll << 31)) { why = "chain sizes out of range"; return false; }
    items += batch_item_bound(n, m);
    longs += long_col_bound(m);
  }
  const size_t cs = (o->precision == RLGL_FP64) ? 8 : 4;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes, 256);
    return at;
  };
  L.cash0 = take(cs * tn);
  L.cash1 = take(cs * tn);
  L.src = take(cs * tn);
  L.hist = take(8 * tn);
  L.hist_lo = (o->precision == RLGL_FP32C_KAHANH) ? take(4 * tn) : 0;
  L.max_items = items;
  L.max_long = longs;
  L.ls_items = take(sizeof(int4) * items);
  L.long_cols = take(4 * longs);
  L.long_acc = take(8 * longs);
  L.order = take(4 * (size_t)g->n_chains);
  L.queue = take(256);
  L.engine = take(ls_device_bytes(g->n_chains));
  L.nrowptr = L.ncolptr = L.nrow = L.perm = 0;
  if (o->relabel) {
    const size_t rp_total = (size_t)tn + (size_t)g->n_chains;
    L.nrowptr = take(4 * rp_total);
    L.ncolptr = take(4 * rp_total);
    L.nrow = take(4 * (size_t)g->edge_off[g->n_chains]);
    L.perm = take(4 * (size_t)tn);
  }
  L.total = off + 256;
  return true;
}

}  // namespace

struct rlgl_batch {
  hipStream_t stream;
  int prec, hk, cus;
  int sched, refresh;
  double r;
  long long max_steps;
  int ls_nt, ls_per_cu, check_period;
  int relabel;
  double eps;
  double clock_khz;
  int n_chains;
  long long total_n;
  ChainOut *host_out;
  long long *host_t0;
  long long *dev_t0;
  unsigned int *dev_queue;
  std::vector<long long> node_off;
  std::vector<int> order;  // largest chain first
  int *dev_order;          // the same order on the device
  LsEngine E;
  double *ls_pi;           // output vector the lockstep descriptors point into
};

namespace {

rlgl_status batch_configure(rlgl_batch *b, const rlgl_batch_options &o) {
  if (o.engine != RLGL_BATCH_LOCKSTEP) return fail(RLGL_EINVAL, "engine must be RLGL_BATCH_LOCKSTEP");
  if (o.check_period < 1) return fail(RLGL_EINVAL, "check_period must be >= 1");
  if (o.wg_size != 256 && o.wg_size != 512) return fail(RLGL_EINVAL, "lockstep wg_size must be 256 or 512");
  if (o.wg_per_cu < 0 || o.wg_per_cu > 16) return fail(RLGL_EINVAL, "lockstep wg_per_cu must be in 0..16");
  b->ls_nt = o.wg_size;
  b->ls_per_cu = o.wg_per_cu;
  b->E.nt = o.wg_size;
  b->E.route_grid = b->cus * o.wg_per_cu;
  b->check_period = o.check_period;
  return RLGL_OK;
}

// Relabelled layout of every chain of a batch (a1): each chain's states
// renumbered by decreasing out-degree, ties by id (a stable counting sort on
// the host, from the row pointers), its row pointers rebuilt and its CSC
// rewritten by k_relabel_side into the workspace.  cp (host, the caller's
// column pointers of every chain) receives the new ones; the chain's new ->
// caller map stays in the workspace for the final pass.  The map the other
// way is only needed here and is kept in the send-value buffer, which no
// solve has used yet.
rlgl_status batch_relabel(rlgl_batch *b, const rlgl_batch_graphs *g, const BatchLayout &L, char *w,
                          std::vector<int> &cp, std::string &why) {
  const int nc = g->n_chains;
  const long long rp_total = b->total_n + nc;
  std::vector<int> rp((size_t)rp_total);
  HIP_TRY(hipMemcpyAsync(rp.data(), g->csr_rowptr, sizeof(int) * (size_t)rp_total, hipMemcpyDeviceToHost,
                         b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  std::vector<int> new2old((size_t)b->total_n), old2new((size_t)b->total_n), nrp((size_t)rp_total),
      ncp((size_t)rp_total);
  std::vector<long long> start;
  for (int k = 0; k < nc; ++k) {
    const long long no = g->node_off[k], ro = no + k;
    const int n = (int)(g->node_off[k + 1] - no);
    const int m = (int)(g->edge_off[k + 1] - g->edge_off[k]);
    const int *r = rp.data() + ro, *c = cp.data() + ro;
    if (c[0] != 0 || c[n] != m) {
      why = "chain " + std::to_string(k) + ": csc_colptr must run from 0 to the link count";
      return RLGL_EINVAL;
    }
    int maxdeg = 0;
    for (int i = 0; i < n; ++i) {
      const int dg = r[i + 1] - r[i];
      if (dg < 0 || c[i + 1] < c[i]) {
        why = "chain " + std::to_string(k) + ": csr_rowptr or csc_colptr decreases";
        return RLGL_EINVAL;
      }
      maxdeg = std::max(maxdeg, dg);
    }
    int *n2o = new2old.data() + no, *o2n = old2new.data() + no;
    if ((long long)maxdeg <= 4ll * n + 1024) {
      start.assign((size_t)maxdeg + 2, 0);
      for (int i = 0; i < n; ++i) ++start[(size_t)(maxdeg - (r[i + 1] - r[i]))];
      long long acc = 0;
      for (auto &x : start) {
        const long long cnt = x;
        x = acc;
        acc += cnt;
      }
      for (int i = 0; i < n; ++i) n2o[start[(size_t)(maxdeg - (r[i + 1] - r[i]))]++] = i;
    } else {
      for (int i = 0; i < n; ++i) n2o[i] = i;
      std::stable_sort(n2o, n2o + n, [&](int a, int c2) { return r[a + 1] - r[a] > r[c2 + 1] - r[c2]; });
    }
    for (int i = 0; i < n; ++i) o2n[n2o[i]] = i;
    int *nr = nrp.data() + ro, *nc2 = ncp.data() + ro;
    nr[0] = 0;
    nc2[0] = 0;
    for (int i = 0; i < n; ++i) {
      nr[i + 1] = nr[i] + (r[n2o[i] + 1] - r[n2o[i]]);
      nc2[i + 1] = nc2[i] + (c[n2o[i] + 1] - c[n2o[i]]);
    }
  }
  int *d_perm = (int *)(w + L.perm), *d_o2n = (int *)(w + L.src), *d_nrp = (int *)(w + L.nrowptr),
      *d_ncp = (int *)(w + L.ncolptr), *d_nrow = (int *)(w + L.nrow);
  HIP_TRY(hipMemcpyAsync(d_perm, new2old.data(), sizeof(int) * (size_t)b->total_n, hipMemcpyHostToDevice,
                         b->stream));
  HIP_TRY(hipMemcpyAsync(d_o2n, old2new.data(), sizeof(int) * (size_t)b->total_n, hipMemcpyHostToDevice,
                         b->stream));
  HIP_TRY(hipMemcpyAsync(d_nrp, nrp.data(), sizeof(int) * (size_t)rp_total, hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipMemcpyAsync(d_ncp, ncp.data(), sizeof(int) * (size_t)rp_total, hipMemcpyHostToDevice, b->stream));
  for (int k = 0; k < nc; ++k) {
    const long long no = g->node_off[k], ro = no + k, eo = g->edge_off[k];
    const int n = (int)(g->node_off[k + 1] - no);
    const long long m = g->edge_off[k + 1] - eo;
    if (m == 0) continue;
    const int grid = (int)std::max<long long>(1, std::min<long long>((m + BLOCK - 1) / BLOCK, 16384));
    k_relabel_side<float><<<grid, BLOCK, 0, b->stream>>>(n, g->csc_colptr + ro, g->csc_row + eo, (const float *)nullptr,
                                                         d_perm + no, d_o2n + no, d_ncp + ro, d_nrow + eo,
                                                         (float *)nullptr);
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(b->stream));
  cp.swap(ncp);
  return RLGL_OK;
}

__global__ void k_batch_start(unsigned int *queue, long long *t0) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *queue = 0u;
    *t0 = wall_clock64();
  }
}

rlgl_status lockstep_run(rlgl_batch *b, double *dev_pi) {
  LsEngine &E = b->E;
  if (dev_pi != b->ls_pi) {
    for (int k = 0; k < b->n_chains; ++k) E.host[k].pi = dev_pi + b->node_off[k];
    HIP_TRY(hipMemcpyAsync(E.d_chains, E.host.data(), sizeof(LsChain) * b->n_chains, hipMemcpyHostToDevice,
                           b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    b->ls_pi = dev_pi;
  }
  rlgl_status st = ls_set_active(E, b->order);
  if (st != RLGL_OK) return st;
  k_batch_start<<<1, 64, 0, b->stream>>>(b->dev_queue, b->dev_t0);
  k_ls_start<<<(b->n_chains + 255) / 256, 256, 0, b->stream>>>(E.d_chains, E.args.ctl, E.args.stats, b->dev_order,
                                                               b->n_chains, E.args.done);
  long long max_steps = 0;
  for (int k = 0; k < b->n_chains; ++k) max_steps = std::max(max_steps, E.host[k].max_steps);
  // every chain stops within max_steps green steps, step 0, one refresh per
  // step and the normalisation pass
  const long long limit = 2 * max_steps + 8;
  long long iters = 0;
  const int n = b->n_chains;
  unsigned int done_seen = 0;
  for (;;) {
    st = ls_iterate(E, b->check_period);
    if (st != RLGL_OK) return st;
    iters += b->check_period;
    HIP_TRY(hipMemcpyAsync(E.h_done, E.args.done, sizeof(unsigned int), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    if ((int)*E.h_done >= n) break;
    if (iters > limit) return fail(RLGL_EHIP, "lockstep batch did not finish within its step bound (internal)");
    // drop finished chains from the launch grids once an eighth of the active
    // ones have finished since the list was last built
    if ((size_t)(*E.h_done - done_seen) * 8 >= E.act.size()) {
      done_seen = *E.h_done;
      HIP_TRY(hipMemcpyAsync(E.h_ctl, E.args.ctl, sizeof(LsCtl) * n, hipMemcpyDeviceToHost, b->stream));
      HIP_TRY(hipStreamSynchronize(b->stream));
      std::vector<int> keep;
      keep.reserve(E.act.size());
      for (int k : E.act)
        if (E.h_ctl[k].mode != LS_DONE) keep.push_back(k);
      if (keep.size() < E.act.size()) {
        st = ls_set_active(E, keep);
        if (st != RLGL_OK) return st;
      }
    }
  }
  return RLGL_OK;
}

rlgl_status batch_run(rlgl_batch *b, double *dev_pi, float *ms) {
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  rlgl_status st = RLGL_OK;
  if (hipEventRecord(e0, b->stream) != hipSuccess) st = fail(RLGL_EHIP, "event record failed");
  if (st == RLGL_OK) st = lockstep_run(b, dev_pi);
  if (st == RLGL_OK && (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
    st = fail(RLGL_EHIP, "event wait failed");
  float t = 0.f;
  if (st == RLGL_OK) (void)hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st == RLGL_OK && ms) *ms = t;
  return st;
}

// Per-chain outcomes of the last solve, from the chains' control records.
rlgl_status batch_outcomes(rlgl_batch *b) {
  HIP_TRY(hipMemcpyAsync(b->E.h_ctl, b->E.args.ctl, sizeof(LsCtl) * b->n_chains, hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipMemcpyAsync(b->host_t0, b->dev_t0, sizeof(long long), hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  for (int k = 0; k < b->n_chains; ++k) {
    const LsCtl &c = b->E.h_ctl[k];
    ChainOut &o = b->host_out[k];
    o.t = c.t;
    o.edges = c.edges;
    o.resid = c.resid;
    o.hsum = c.hsum;
    o.status = c.status;
    o.green_steps = c.green_steps;
    o.t0 = c.t0;
    o.t1 = c.t1;
  }
  return RLGL_OK;
}

}  // namespace

namespace {
// Copies a plan out to the caller's host arrays (4 ints per item).
int64_t plan_out(const std::vector<int4> &items, const std::vector<int> &lng, int32_t *items_out, int64_t max_items,
                 int32_t *long_out, int64_t max_long) {
  if ((int64_t)items.size() > max_items || (int64_t)lng.size() > max_long) {
    fail(RLGL_ENOMEM, "plan needs %zu items and %zu long columns", items.size(), lng.size());
    return RLGL_ENOMEM;
  }
  if (items_out)
    for (size_t q = 0; q < items.size(); ++q) {
      items_out[4 * q] = items[q].x;
      items_out[4 * q + 1] = items[q].y;
      items_out[4 * q + 2] = items[q].z;
      items_out[4 * q + 3] = items[q].w;
    }
  if (long_out)
    for (size_t q = 0; q < lng.size(); ++q) long_out[q] = lng[q];
  return (int64_t)items.size();
}
}  // namespace

extern "C" {

int64_t rlgl_pull_plan(const int32_t *host_colptr, int32_t n, int64_t nnz, int32_t *items, int64_t max_items,
                       int32_t *long_cols, int64_t max_long, int64_t *n_long, int64_t *item_bound) {
  if (!host_colptr || n < 1 || nnz < 0 || nnz >= (1ll << 31) || max_items < 0 || max_long < 0 ||
      (max_items > 0 && !items) || (max_long > 0 && !long_cols))
    return fail(RLGL_EINVAL, "bad arguments to rlgl_pull_plan");
  std::vector<int4> it;
  std::vector<int> lng;
  std::string why;
  if (!pull_plan_host(host_colptr, n, nnz, it, lng, why)) return fail(RLGL_EINVAL, "%s", why.c_str());
  if (n_long) *n_long = (int64_t)lng.size();
  if (item_bound) *item_bound = (int64_t)pull_item_bound(n, nnz);
  return plan_out(it, lng, items, max_items, long_cols, max_long);
}

int64_t rlgl_batch_chain_plan(const int32_t *host_colptr, int32_t n, int64_t nnz, int32_t *items, int64_t max_items,
                              int32_t *long_cols, int64_t max_long, int64_t *n_long, int64_t *n_pieces,
                              int64_t *item_bound) {
  if (!host_colptr || n < 1 || nnz < 0 || nnz >= (1ll << 31) || max_items < 0 || max_long < 0 ||
      (max_items > 0 && !items) || (max_long > 0 && !long_cols))
    return fail(RLGL_EINVAL, "bad arguments to rlgl_batch_chain_plan");
  std::vector<int4> it;
  std::vector<int> lng;
  std::string why;
  int np = 0, nr = 0;
  if (!chain_plan(host_colptr, n, (int)nnz, it, lng, np, nr, why)) return fail(RLGL_EINVAL, "%s", why.c_str());
  if (n_long) *n_long = (int64_t)lng.size();
  if (n_pieces) *n_pieces = np;
  if (item_bound) *item_bound = (int64_t)batch_item_bound(n, nnz);
  return plan_out(it, lng, items, max_items, long_cols, max_long);
}


void rlgl_batch_default_options(rlgl_batch_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->sched = RLGL_SCHED_THRESHOLD;
  o->r = 1.0;
  o->precision = RLGL_FP32C_KAHANH;
  o->eps = 1e-7;
  o->max_steps = 100000;
  o->refresh = 1;
  o->wg_size = 256;
  o->wg_per_cu = 0;
  o->engine = RLGL_BATCH_LOCKSTEP;
  o->check_period = 8;
  o->relabel = 1;
}

size_t rlgl_batch_workspace_bytes(const rlgl_batch_graphs *g, const rlgl_batch_options *o) {
  BatchLayout L;
  std::string why;
  if (!batch_layout(g, o, L, why)) return 0;
  return L.total;
}

rlgl_status rlgl_batch_create(const rlgl_batch_graphs *g, const rlgl_batch_options *o, void *ws, size_t ws_bytes,
                              void *stream, rlgl_batch **out) {
  if (!g || !o || !out) return fail(RLGL_EINVAL, "null argument");
  *out = nullptr;
  BatchLayout L;
  std::string why;
  if (!batch_layout(g, o, L, why)) return fail(RLGL_EINVAL, "%s", why.c_str());
  if (o->sched != RLGL_SCHED_ALL && o->sched != RLGL_SCHED_THRESHOLD && o->sched != RLGL_SCHED_MAXC)
    return fail(RLGL_EINVAL, "batched solves support the ALL, THRESHOLD and MAXC schedules");
  if (!(o->r >= 1.0) || !std::isfinite(o->r) || !(o->eps >= 0.0) || o->max_steps < 0)
    return fail(RLGL_EINVAL, "bad r, eps or max_steps");
  if (!g->csr_rowptr || !g->csc_colptr || !g->csc_row || !g->damping)
    return fail(RLGL_EINVAL, "batched solves need the CSR row pointers, the CSC and the damping factors");
  if ((g->csr_val == nullptr) != (g->csc_val == nullptr)) return fail(RLGL_EINVAL, "csr_val/csc_val mismatch");
  if (!ws) return fail(RLGL_EINVAL, "workspace is NULL");
  if (ws_bytes < L.total) return fail(RLGL_ENOMEM, "workspace too small: %zu < %zu", ws_bytes, L.total);
  const int nc = g->n_chains;
  for (int k = 0; k < nc; ++k) {
    if (!(g->damping[k] > 0.0 && g->damping[k] <= 1.0)) return fail(RLGL_EINVAL, "damping of chain %d out of (0,1]", k);
    if (g->tol_l1 && !(g->tol_l1[k] >= 0.0)) return fail(RLGL_EINVAL, "tol_l1 of chain %d is negative", k);
    if (g->tol_l1 && g->damping[k] >= 1.0)
      return fail(RLGL_EINVAL, "chain %d: damping 1 has no L1 certificate for tol_l1 (give options.eps instead)", k);
  }

  rlgl_batch *b = new (std::nothrow) rlgl_batch();
  if (!b) return fail(RLGL_ENOMEM, "host allocation failed");
  b->stream = (hipStream_t)stream;
  b->prec = o->precision;
  b->hk = o->precision == RLGL_FP32C_KAHANH;
  b->n_chains = nc;
  b->total_n = g->node_off[nc];
  b->node_off.assign(g->node_off, g->node_off + nc + 1);
  b->ls_pi = nullptr;
  b->eps = o->eps;
  char *w = (char *)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
  b->sched = o->sched;
  b->r = o->r;
  b->max_steps = o->max_steps;
  b->refresh = o->refresh ? 1 : 0;
  b->dev_queue = (unsigned int *)(w + L.queue);
  b->dev_t0 = (long long *)(w + L.queue + 64);
  b->dev_order = (int *)(w + L.order);

  auto bail = [&](rlgl_status s) {
    rlgl_batch_destroy(b);
    return s;
  };
  int dev = 0, cus = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) ||
      hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev))
    return bail(fail(RLGL_EHIP, "device attribute query failed"));
  b->cus = std::max(cus, 1);
  b->clock_khz = khz > 0 ? khz : 100000.0;
  if (hipHostMalloc((void **)&b->host_out, sizeof(ChainOut) * nc, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&b->host_t0, sizeof(long long), hipHostMallocDefault) != hipSuccess)
    return bail(fail(RLGL_EHIP, "pinned host allocation failed"));
  rlgl_status st = ls_init(b->E, w + L.engine, nc, o->precision, o->sched, o->r, o->refresh, b->stream);
  if (st != RLGL_OK) return bail(st);

  // static plans: pieces of the long columns, then runs of at most CH in-links
  const long long rp_total = b->total_n + nc;
  std::vector<int> cp((size_t)rp_total);
  if (hipMemcpyAsync(cp.data(), g->csc_colptr, sizeof(int) * (size_t)rp_total, hipMemcpyDeviceToHost, b->stream) !=
          hipSuccess ||
      hipStreamSynchronize(b->stream) != hipSuccess)
    return bail(fail(RLGL_EHIP, "reading the column pointers failed"));
  b->relabel = o->relabel ? 1 : 0;
  if (b->relabel) {
    st = batch_relabel(b, g, L, w, cp, why);
    if (st != RLGL_OK) return bail(st == RLGL_EINVAL ? fail(st, "%s", why.c_str()) : st);
  }
  std::vector<int4> ls_items;
  std::vector<int> long_cols;
  std::vector<long long> size_of((size_t)nc);
  const size_t cs = (o->precision == RLGL_FP64) ? 8 : 4;
  for (int k = 0; k < nc; ++k) {
    const long long no = g->node_off[k], rp = no + k;
    const int n = (int)(g->node_off[k + 1] - no);
    const int m = (int)(g->edge_off[k + 1] - g->edge_off[k]);
    size_of[k] = (long long)m + n;
    int np = 0, nr2 = 0;
    const size_t li = ls_items.size(), lo = long_cols.size();
    if (!chain_plan(cp.data() + rp, n, m, ls_items, long_cols, np, nr2, why))
      return bail(fail(RLGL_EINVAL, "chain %d: %s", k, why.c_str()));
    LsChain &lc = b->E.host[k];
    if (b->relabel) {
      lc.rowptr = (const int *)(w + L.nrowptr) + rp;
      lc.colptr = (const int *)(w + L.ncolptr) + rp;
      lc.crow = (const int *)(w + L.nrow) + g->edge_off[k];
      lc.perm = (const int *)(w + L.perm) + no;
    } else {
      lc.rowptr = g->csr_rowptr + rp;
      lc.colptr = g->csc_colptr + rp;
      lc.crow = g->csc_row + g->edge_off[k];
      lc.perm = nullptr;
    }
    lc.items = (const int4 *)(w + L.ls_items) + li;
    lc.long_cols = (const int *)(w + L.long_cols) + lo;
    lc.long_acc = (double *)(w + L.long_acc) + lo;
    lc.n_long = (int)(long_cols.size() - lo);
    lc.cash0 = w + L.cash0 + cs * no;
    lc.cash1 = w + L.cash1 + cs * no;
    lc.src = w + L.src + cs * no;
    lc.hist = w + L.hist + (b->hk ? 4 : 8) * no;
    lc.hist_lo = b->hk ? (float *)(w + L.hist_lo) + no : nullptr;
    lc.pi = nullptr;
    lc.nnz = m;
    lc.max_steps = o->max_steps;
    lc.c = g->damping[k];
    lc.eps = g->tol_l1 ? g->tol_l1[k] * (1.0 - g->damping[k]) : o->eps;
    lc.n = n;
    lc.n_piece = np;
    lc.n_run = nr2;
  }
  if (ls_items.size() > L.max_items || long_cols.size() > L.max_long)
    return bail(fail(RLGL_EINVAL, "batch plan exceeds its bound (internal)"));
  b->order.resize((size_t)nc);
  for (int k = 0; k < nc; ++k) b->order[k] = k;
  std::stable_sort(b->order.begin(), b->order.end(), [&](int a, int c2) { return size_of[a] > size_of[c2]; });
  if ((!ls_items.empty() && hipMemcpyAsync(w + L.ls_items, ls_items.data(), sizeof(int4) * ls_items.size(),
                                           hipMemcpyHostToDevice, b->stream)) ||
      (!long_cols.empty() && hipMemcpyAsync(w + L.long_cols, long_cols.data(), 4 * long_cols.size(),
                                            hipMemcpyHostToDevice, b->stream)) ||
      hipMemcpyAsync(w + L.order, b->order.data(), sizeof(int) * nc, hipMemcpyHostToDevice, b->stream) ||
      hipStreamSynchronize(b->stream))
    return bail(fail(RLGL_EHIP, "uploading the batch plan failed"));
  st = batch_configure(b, *o);
  if (st != RLGL_OK) return bail(st);
  *out = b;
  return RLGL_OK;
}

rlgl_status rlgl_batch_solve(rlgl_batch *b, double *dev_pi, rlgl_chain_result *res, double *elapsed_ms) {
  if (!b || !dev_pi) return fail(RLGL_EINVAL, "bad argument");
  float ms = 0.f;
  rlgl_status st = batch_run(b, dev_pi, &ms);
  if (st != RLGL_OK) return st;
  if (elapsed_ms) *elapsed_ms = ms;
  st = batch_outcomes(b);
  if (st != RLGL_OK) return st;
  rlgl_status worst = RLGL_OK;
  const double us_per_tick = 1000.0 / b->clock_khz;
  for (int k = 0; k < b->n_chains; ++k) {
    const ChainOut &o = b->host_out[k];
    const rlgl_status cs = o.status == ST_CONVERGED ? RLGL_OK : status_of(o.status);
    if (cs != RLGL_OK && worst == RLGL_OK) worst = cs;
    if (res) {
      res[k].t = o.t;
      res[k].edges_pushed = o.edges;
      res[k].resid = o.resid;
      res[k].h_sum = o.hsum;
      res[k].status = cs;
      res[k].green_steps = o.green_steps;
      res[k].start_us = (double)(o.t0 - *b->host_t0) * us_per_tick;
      res[k].end_us = (double)(o.t1 - *b->host_t0) * us_per_tick;
    }
  }
  if (worst != RLGL_OK) return fail(worst, "at least one chain did not stop on its test");
  return RLGL_OK;
}

rlgl_status rlgl_batch_autotune(rlgl_batch *b, double *dev_pi, rlgl_batch_options *best) {
  if (!b || !dev_pi) return fail(RLGL_EINVAL, "bad argument");
  rlgl_batch_options cur;
  rlgl_batch_default_options(&cur);
  cur.sched = b->sched;
  cur.r = b->r;
  cur.precision = b->prec;
  cur.eps = b->eps;
  cur.max_steps = b->max_steps;
  cur.refresh = b->refresh;
  cur.check_period = b->check_period;
  cur.relabel = b->relabel;
  cur.engine = RLGL_BATCH_LOCKSTEP;
  cur.wg_size = b->ls_nt;
  cur.wg_per_cu = b->ls_per_cu;
  std::vector<rlgl_batch_options> cands;
  for (int nt : {256, 512})
    for (int pc : {0, 4, 8}) {
      rlgl_batch_options c = cur;
      c.engine = RLGL_BATCH_LOCKSTEP;
      c.wg_size = nt;
      c.wg_per_cu = pc;
      cands.push_back(c);
    }
  double best_ms = 1e300;
  rlgl_batch_options pick = cur;
  for (const rlgl_batch_options &c : cands) {
    if (batch_configure(b, c) != RLGL_OK) continue;
    float ms = 0.f;
    const rlgl_status st = batch_run(b, dev_pi, &ms);
    if (st != RLGL_OK) return st;
    if (ms < best_ms) {
      best_ms = ms;
      pick = c;
    }
  }
  const rlgl_status st = batch_configure(b, pick);
  if (st != RLGL_OK) return st;
  if (best) *best = pick;
  return RLGL_OK;
}

void rlgl_batch_destroy(rlgl_batch *b) {
  if (!b) return;
  ls_free(b->E);
  if (b->host_out) (void)hipHostFree(b->host_out);
  if (b->host_t0) (void)hipHostFree(b->host_t0);
  delete b;
}

}  // extern "C"

// ------------------------------------------------------------- serving pool

namespace {

enum { SLOT_FREE = 0, SLOT_UPLOADING = 1, SLOT_RUNNING = 2, SLOT_FINISHED = 3 };

struct PoolSlot {
  int state = SLOT_FREE;
  size_t off = 0, bytes = 0;  // arena block
  hipEvent_t ready = nullptr;
  char *stage = nullptr;      // page-locked copy of the plan and the long columns for the upload
  size_t stage_cap = 0;
  LsChain desc{};
  LsCtl final{};              // the chain's control record when it was collected
};

// Arena bytes of a chain: row and column pointers, CSC sources, plan, two
// cash buffers, the scaled source buffer, the history and pi_hat.
size_t pool_chain_bytes(int prec, long long n, long long nnz, size_t n_items, size_t n_long) {
  const size_t cs = (prec == RLGL_FP64) ? 8 : 4;
  size_t b = 0;
  b += align_up(4 * (size_t)(n + 1), 256) * 2;
  b += align_up(4 * (size_t)nnz, 256);
  b += align_up(sizeof(int4) * n_items + 4 * n_long, 256);
  b += align_up(8 * n_long, 256);
  b += align_up(cs * (size_t)n, 256) * 3;
  b += align_up(8 * (size_t)n, 256);  // double, or the float hi part
  if (prec == RLGL_FP32C_KAHANH) b += align_up(4 * (size_t)n, 256);
  b += align_up(8 * (size_t)n, 256);
  return b;
}

bool valid_pool_options(const rlgl_pool_options *o, std::string &why) {
  if (!o) { why = "null options"; return false; }
  if (o->sched != RLGL_SCHED_ALL && o->sched != RLGL_SCHED_THRESHOLD && o->sched != RLGL_SCHED_MAXC) {
    why = "the pool supports the ALL, THRESHOLD and MAXC schedules";
    return false;
  }
  if (!(o->r >= 1.0) || !std::isfinite(o->r)) { why = "r must be >= 1"; return false; }
  if (o->precision < 0 || o->precision > 2) { why = "precision out of range"; return false; }
  if (o->wg_size != 256 && o->wg_size != 512) { why = "wg_size must be 256 or 512"; return false; }
  if (o->max_chains < 1 || o->max_chains > (1 << 20)) { why = "max_chains out of range"; return false; }
  if (o->max_steps < 0) { why = "max_steps must be >= 0"; return false; }
  if (o->route_per_cu < 0 || o->route_per_cu > 16) { why = "route_per_cu must be in 0..16"; return false; }
  return true;
}

}  // namespace

struct rlgl_pool {
  rlgl_pool_options opt;
  hipStream_t stream = nullptr, copy = nullptr;
  LsEngine E;
  char *arena = nullptr;
  size_t arena_bytes = 0;
  std::vector<std::pair<size_t, size_t>> free_list;  // (offset, bytes), sorted, coalesced
  std::vector<PoolSlot> slots;
  std::vector<int> running;   // slots in the active list, admission order
  std::vector<int> finished;  // finished since the last poll
  bool dirty = false;
  bool in_flight = false;     // iterations enqueued by rlgl_pool_launch, not yet waited for
  hipEvent_t launched = nullptr;
  long long t_origin = 0;
  double clock_khz = 100000.0;
};

namespace {

bool arena_take(rlgl_pool *p, size_t bytes, size_t &off) {
  for (size_t q = 0; q < p->free_list.size(); ++q) {
    auto &f = p->free_list[q];
    if (f.second >= bytes) {
      off = f.first;
      f.first += bytes;
      f.second -= bytes;
      if (f.second == 0) p->free_list.erase(p->free_list.begin() + (long)q);
      return true;
    }
  }
  return false;
}

void arena_give(rlgl_pool *p, size_t off, size_t bytes) {
  auto &fl = p->free_list;
  auto it = std::lower_bound(fl.begin(), fl.end(), std::make_pair(off, (size_t)0));
  it = fl.insert(it, {off, bytes});
  // coalesce with the next and the previous block
  if (it + 1 != fl.end() && it->first + it->second == (it + 1)->first) {
    it->second += (it + 1)->second;
    fl.erase(it + 1);
  }
  if (it != fl.begin() && (it - 1)->first + (it - 1)->second == it->first) {
    (it - 1)->second += it->second;
    fl.erase(it);
  }
}

__global__ void k_wall_clock(long long *out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *out = wall_clock64();
}

}  // namespace

extern "C" {

void rlgl_pool_default_options(rlgl_pool_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->sched = RLGL_SCHED_THRESHOLD;
  o->r = 1.0;
  o->precision = RLGL_FP32C_KAHANH;
  o->refresh = 1;
  o->wg_size = 256;
  o->max_chains = 256;
  o->max_steps = 100000;
  o->route_per_cu = 8;
}

size_t rlgl_pool_workspace_bytes(const rlgl_pool_options *o, size_t arena_bytes) {
  std::string why;
  if (!valid_pool_options(o, why)) return 0;
  return ls_device_bytes(o->max_chains) + align_up(arena_bytes, 256) + 512;
}

size_t rlgl_pool_footprint(const rlgl_pool_options *o, int32_t n, int64_t nnz) {
  std::string why;
  if (!valid_pool_options(o, why) || n < 1 || nnz < 0) return 0;
  return pool_chain_bytes(o->precision, n, nnz, batch_item_bound(n, nnz), long_col_bound(nnz));
}

rlgl_status rlgl_pool_create(const rlgl_pool_options *o, void *ws, size_t ws_bytes, void *stream, rlgl_pool **out) {
  if (!out) return fail(RLGL_EINVAL, "null argument");
  *out = nullptr;
  std::string why;
  if (!valid_pool_options(o, why)) return fail(RLGL_EINVAL, "%s", why.c_str());
  if (!ws) return fail(RLGL_EINVAL, "workspace is NULL");
  const size_t ctl = ls_device_bytes(o->max_chains);
  if (ws_bytes < ctl + 512 + 256) return fail(RLGL_ENOMEM, "workspace too small for the pool's control records");
  rlgl_pool *p = new (std::nothrow) rlgl_pool();
  if (!p) return fail(RLGL_ENOMEM, "host allocation failed");
  auto bail = [&](rlgl_status s) {
    rlgl_pool_destroy(p);
    return s;
  };
  p->opt = *o;
  p->stream = (hipStream_t)stream;
  char *w = (char *)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
  const size_t lead = (size_t)(w - (char *)ws);
  rlgl_status st = ls_init(p->E, w, o->max_chains, o->precision, o->sched, o->r, o->refresh, p->stream);
  if (st != RLGL_OK) return bail(st);
  p->E.nt = o->wg_size;
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev))
      return bail(fail(RLGL_EHIP, "device attribute query failed"));
    p->E.route_grid = std::max(cus, 1) * o->route_per_cu;
  }
  p->arena = w + ctl;
  p->arena_bytes = (ws_bytes - lead - ctl) / 256 * 256;
  p->free_list.push_back({0, p->arena_bytes});
  p->slots.resize((size_t)o->max_chains);
  if (hipStreamCreateWithFlags(&p->copy, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(RLGL_EHIP, "creating the upload stream failed"));
  if (hipEventCreateWithFlags(&p->launched, hipEventDisableTiming) != hipSuccess)
    return bail(fail(RLGL_EHIP, "event creation failed"));
  for (PoolSlot &s : p->slots)
    if (hipEventCreateWithFlags(&s.ready, hipEventDisableTiming) != hipSuccess)
      return bail(fail(RLGL_EHIP, "event creation failed"));
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev))
    return bail(fail(RLGL_EHIP, "device attribute query failed"));
  p->clock_khz = khz > 0 ? khz : 100000.0;
  // device wall clock at creation: the origin of start_us / end_us
  long long *origin = (long long *)(p->E.args.done) + 8;
  k_wall_clock<<<1, 64, 0, p->stream>>>(origin);
  if (hipMemcpyAsync(&p->t_origin, origin, sizeof(long long), hipMemcpyDeviceToHost, p->stream) != hipSuccess ||
      hipStreamSynchronize(p->stream) != hipSuccess)
    return bail(fail(RLGL_EHIP, "reading the device clock failed"));
  *out = p;
  return RLGL_OK;
}

rlgl_status rlgl_pool_admit(rlgl_pool *p, const rlgl_request *q, int32_t *slot) {
  if (!p || !q || !slot) return fail(RLGL_EINVAL, "null argument");
  const long long n = q->n, m = q->nnz;
  if (n < 1 || m < 0 || m >= (1ll << 31)) return fail(RLGL_EINVAL, "request sizes out of range");
  if (!q->csr_rowptr || !q->csc_colptr || (m > 0 && !q->csc_row)) return fail(RLGL_EINVAL, "request arrays are NULL");
  if (!(q->damping > 0.0 && q->damping < 1.0))
    return fail(RLGL_EINVAL, "damping must be in (0, 1): a request stops on an L1 certificate, which c = 1 lacks");
  if (!(q->tol_l1 >= 0.0)) return fail(RLGL_EINVAL, "tol_l1 must be >= 0");
  const int32_t *rp = q->csr_rowptr;
  if (rp[0] != 0 || rp[n] != m) return fail(RLGL_EINVAL, "csr_rowptr must run from 0 to nnz");
  for (long long i = 0; i < n; ++i)
    if (rp[i + 1] < rp[i]) return fail(RLGL_EINVAL, "csr_rowptr decreases at %lld", i);
  int k = -1;
  for (int s = 0; s < (int)p->slots.size(); ++s)
    if (p->slots[s].state == SLOT_FREE) {
      k = s;
      break;
    }
  if (k < 0) return fail(RLGL_EBUSY, "no free slot");
  PoolSlot &S = p->slots[k];
  // the plan is built into the slot's page-locked staging buffer
  std::vector<int4> items;
  std::vector<int> longs;
  items.reserve(batch_item_bound(n, m));
  longs.reserve(long_col_bound(m));
  int np = 0, nr = 0;
  std::string why;
  if (!chain_plan(q->csc_colptr, (int)n, (int)m, items, longs, np, nr, why))
    return fail(RLGL_EINVAL, "%s", why.c_str());
  const int prec = p->opt.precision;
  const size_t bytes = pool_chain_bytes(prec, n, m, items.size(), longs.size());
  size_t off = 0;
  if (!arena_take(p, bytes, off)) return fail(RLGL_EBUSY, "no arena block of %zu bytes free", bytes);
  const size_t plan_bytes = sizeof(int4) * items.size() + 4 * longs.size();
  if (S.stage_cap < plan_bytes) {
    if (S.stage) (void)hipHostFree(S.stage);
    S.stage = nullptr;
    S.stage_cap = 0;
    const size_t cap = std::max(plan_bytes, (size_t)16384);
    if (hipHostMalloc((void **)&S.stage, cap, hipHostMallocDefault) != hipSuccess) {
      arena_give(p, off, bytes);
      return fail(RLGL_ENOMEM, "page-locked staging allocation failed");
    }
    S.stage_cap = cap;
  }
  std::memcpy(S.stage, items.data(), sizeof(int4) * items.size());
  std::memcpy(S.stage + sizeof(int4) * items.size(), longs.data(), 4 * longs.size());
  char *base = p->arena + off;
  size_t at = 0;
  auto take = [&](size_t b) {
    char *r = base + at;
    at += align_up(b, 256);
    return r;
  };
  const size_t cs = (prec == RLGL_FP64) ? 8 : 4;
  const bool hk = prec == RLGL_FP32C_KAHANH;
  LsChain &d = S.desc;
  d = LsChain{};
  int *d_rowptr = (int *)take(4 * (size_t)(n + 1));
  int *d_colptr = (int *)take(4 * (size_t)(n + 1));
  int *d_crow = (int *)take(4 * (size_t)m);
  int4 *d_items = (int4 *)take(plan_bytes);  // the plan, then the long columns
  d.rowptr = d_rowptr;
  d.colptr = d_colptr;
  d.crow = d_crow;
  d.items = d_items;
  d.long_cols = (const int *)(d_items + items.size());
  d.long_acc = (double *)take(8 * longs.size());
  d.n_long = (int)longs.size();
  d.cash0 = take(cs * (size_t)n);
  d.cash1 = take(cs * (size_t)n);
  d.src = take(cs * (size_t)n);
  d.hist = take(8 * (size_t)n);
  d.hist_lo = hk ? (float *)take(4 * (size_t)n) : nullptr;
  d.pi = (double *)take(8 * (size_t)n);
  d.nnz = m;
  d.max_steps = p->opt.max_steps;
  d.c = q->damping;
  d.eps = q->tol_l1 * (1.0 - q->damping);
  d.n = (int)n;
  d.n_piece = np;
  d.n_run = nr;
  hipError_t e = hipMemcpyAsync(d_rowptr, q->csr_rowptr, 4 * (size_t)(n + 1), hipMemcpyHostToDevice, p->copy);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_colptr, q->csc_colptr, 4 * (size_t)(n + 1), hipMemcpyHostToDevice, p->copy);
  if (e == hipSuccess && m > 0) e = hipMemcpyAsync(d_crow, q->csc_row, 4 * (size_t)m, hipMemcpyHostToDevice, p->copy);
  if (e == hipSuccess && plan_bytes > 0)
    e = hipMemcpyAsync(d_items, S.stage, plan_bytes, hipMemcpyHostToDevice, p->copy);
  if (e == hipSuccess) e = hipEventRecord(S.ready, p->copy);
  if (e != hipSuccess) {
    // let whatever was enqueued finish before the block can be reused
    (void)hipStreamSynchronize(p->copy);
    arena_give(p, off, bytes);
    return fail(RLGL_EHIP, "request upload: %s", hipGetErrorString(e));
  }
  S.off = off;
  S.bytes = bytes;
  S.state = SLOT_UPLOADING;
  *slot = k;
  return RLGL_OK;
}

rlgl_status rlgl_pool_launch(rlgl_pool *p, int32_t iterations) {
  if (!p || iterations < 0) return fail(RLGL_EINVAL, "bad argument");
  if (p->in_flight) return fail(RLGL_EINVAL, "iterations are already in flight (call rlgl_pool_wait)");
  // start the chains whose upload has landed
  for (int k = 0; k < (int)p->slots.size(); ++k) {
    PoolSlot &S = p->slots[k];
    if (S.state != SLOT_UPLOADING) continue;
    const hipError_t q = hipEventQuery(S.ready);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) return fail(RLGL_EHIP, "upload of slot %d: %s", k, hipGetErrorString(q));
    p->E.host[k] = S.desc;
    k_ls_admit<<<1, 64, 0, p->stream>>>(p->E.d_chains, p->E.args.ctl, p->E.args.stats, k, S.desc);
    S.state = SLOT_RUNNING;
    p->running.push_back(k);
    p->dirty = true;
  }
  HIP_TRY(hipGetLastError());
  if (p->dirty) {
    rlgl_status st = ls_set_active(p->E, p->running);
    if (st != RLGL_OK) return st;
    p->dirty = false;
  }
  if (!p->running.empty() && iterations > 0) {
    rlgl_status st = ls_iterate(p->E, iterations);
    if (st != RLGL_OK) return st;
    HIP_TRY(hipMemcpyAsync(p->E.h_ctl, p->E.args.ctl, sizeof(LsCtl) * p->slots.size(), hipMemcpyDeviceToHost,
                           p->stream));
    HIP_TRY(hipEventRecord(p->launched, p->stream));
    p->in_flight = true;
  }
  return RLGL_OK;
}

rlgl_status rlgl_pool_wait(rlgl_pool *p, int32_t *running) {
  if (!p) return fail(RLGL_EINVAL, "null pool");
  if (p->in_flight) {
    HIP_TRY(hipEventSynchronize(p->launched));
    p->in_flight = false;
    std::vector<int> keep;
    keep.reserve(p->running.size());
    for (int k : p->running) {
      if (p->E.h_ctl[k].mode == LS_DONE) {
        p->slots[k].final = p->E.h_ctl[k];
        p->slots[k].state = SLOT_FINISHED;
        p->finished.push_back(k);
      } else {
        keep.push_back(k);
      }
    }
    if (keep.size() != p->running.size()) {
      p->running.swap(keep);
      p->dirty = true;
    }
  }
  if (running) {
    int c = 0;
    for (const PoolSlot &S : p->slots) c += (S.state == SLOT_UPLOADING || S.state == SLOT_RUNNING);
    *running = c;
  }
  return RLGL_OK;
}

rlgl_status rlgl_pool_advance(rlgl_pool *p, int32_t iterations, int32_t *running) {
  const rlgl_status st = rlgl_pool_launch(p, iterations);
  if (st != RLGL_OK) return st;
  return rlgl_pool_wait(p, running);
}

int32_t rlgl_pool_poll(rlgl_pool *p, int32_t *slots, int32_t max_slots) {
  if (!p || (max_slots > 0 && !slots) || max_slots < 0) return fail(RLGL_EINVAL, "bad argument");
  const int m = std::min((int)p->finished.size(), (int)max_slots);
  for (int i = 0; i < m; ++i) slots[i] = p->finished[i];
  p->finished.erase(p->finished.begin(), p->finished.begin() + m);
  return m;
}

rlgl_status rlgl_pool_result(rlgl_pool *p, int32_t slot, rlgl_chain_result *r, const double **dev_pi) {
  if (!p || slot < 0 || slot >= (int)p->slots.size()) return fail(RLGL_EINVAL, "bad slot");
  const PoolSlot &S = p->slots[slot];
  if (S.state == SLOT_FREE) return fail(RLGL_EINVAL, "slot %d holds no chain", slot);
  if (S.state != SLOT_FINISHED) return fail(RLGL_EBUSY, "slot %d has not finished", slot);
  const LsCtl &c = S.final;
  if (r) {
    const double us = 1000.0 / p->clock_khz;
    r->t = c.t;
    r->edges_pushed = c.edges;
    r->resid = c.resid;
    r->h_sum = c.hsum;
    r->status = c.status == ST_CONVERGED ? RLGL_OK : status_of(c.status);
    r->green_steps = c.green_steps;
    r->start_us = (double)(c.t0 - p->t_origin) * us;
    r->end_us = (double)(c.t1 - p->t_origin) * us;
  }
  if (dev_pi) *dev_pi = S.desc.pi;
  return RLGL_OK;
}

rlgl_status rlgl_pool_release(rlgl_pool *p, int32_t slot) {
  if (!p || slot < 0 || slot >= (int)p->slots.size()) return fail(RLGL_EINVAL, "bad slot");
  PoolSlot &S = p->slots[slot];
  if (S.state == SLOT_FREE) return fail(RLGL_EINVAL, "slot %d holds no chain", slot);
  if (S.state != SLOT_FINISHED) return fail(RLGL_EBUSY, "slot %d is still uploading or running", slot);
  p->finished.erase(std::remove(p->finished.begin(), p->finished.end(), slot), p->finished.end());
  // the chain's kernels have all completed (it finished before the last
  // synchronisation of the pool's stream), so the block can be reused
  arena_give(p, S.off, S.bytes);
  S.state = SLOT_FREE;
  S.off = S.bytes = 0;
  return RLGL_OK;
}

void rlgl_pool_destroy(rlgl_pool *p) {
  if (!p) return;
  if (p->copy) {
    (void)hipStreamSynchronize(p->copy);
  }
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  for (PoolSlot &S : p->slots) {
    if (S.ready) (void)hipEventDestroy(S.ready);
    if (S.stage) (void)hipHostFree(S.stage);
  }
  if (p->copy) (void)hipStreamDestroy(p->copy);
  if (p->launched) (void)hipEventDestroy(p->launched);
  ls_free(p->E);
  delete p;
}

}  // extern "C"

// ------------------------------------------------------ one-workgroup solves

namespace {

struct SmallLayout {
  size_t rec, H, Q, total;
};

SmallLayout small_layout(long long n) {
  SmallLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes, 256);
    return at;
  };
  L.rec = take(sizeof(SmallRec));
  L.H = take(8 * (size_t)n);
  L.Q = take(8 * (size_t)n);
  L.total = off + 256;  // room to align the caller's pointer
  return L;
}

const void *small_kernel(int prec) {
  return prec == RLGL_FP64 ? (const void *)k_small<double> : (const void *)k_small<float>;
}

// Largest n whose cash fits in the LDS one workgroup may take on the current
// device, next to the kernel's own static LDS; 0 when the query fails.
// LDS bytes left to the one-workgroup kernel after its static arrays.
long long small_lds_budget(int prec) {
  int dev = 0, lds = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 0;
  hipFuncAttributes fa{};
  if (hipFuncGetAttributes(&fa, small_kernel(prec)) != hipSuccess) return 0;
  return (long long)lds - (long long)fa.sharedSizeBytes - 16;
}

int small_capacity(int prec) {
  const long long dyn = small_lds_budget(prec);
  const int cs = prec == RLGL_FP64 ? 8 : 4;
  return dyn > 0 ? (int)(dyn / cs) : 0;
}


// The workspace of rlgl_solve_small_static: a static device array of fixed
// size, one copy on every GPU the library runs on, held until the process
// ends.  Host code never passes the array's name to a kernel or a copy (on
// the host it stands for no device address); it uses the address that
// hipGetSymbolAddress returns, looked up once per device with that device
// current.
static __device__ __align__(256) unsigned char scratch[RLGL_SMALL_STATIC_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[MAX_DEVICES] = {};

rlgl_status static_scratch(char **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return fail(RLGL_EINVAL, "device %d beyond the library's table", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(RLGL_EHIP, "hipGetSymbolAddress returned no address for the static workspace");
    g_scratch_ptr[dev] = (char *)ptr;
  }
  *out = g_scratch_ptr[dev];
  return RLGL_OK;
}

rlgl_status small_solve(const rlgl_graph *g, const rlgl_options *o, double eps, int64_t max_steps, double *dev_pi,
                        char *ws, size_t ws_bytes, hipStream_t stream, rlgl_step_info *info) {
  if (!g || !o) return fail(RLGL_EINVAL, "null argument");
  std::string why;
  if (!valid_options(o, why)) return fail(RLGL_EINVAL, "options: %s", why.c_str());
  if (o->sched == RLGL_SCHED_TOPK) return fail(RLGL_EINVAL, "the one-workgroup solve has no top-k rule");
  if (g->n < 1) return fail(RLGL_EINVAL, "n must be >= 1");
  if (g->nnz < 0 || g->nnz >= (1ll << 31)) return fail(RLGL_EINVAL, "nnz must be in [0, 2^31)");
  if (!(g->damping > 0.0 && g->damping <= 1.0)) return fail(RLGL_EINVAL, "damping must be in (0, 1]");
  if (!g->csr_rowptr || !g->csc_colptr) return fail(RLGL_EINVAL, "the one-workgroup solve needs the CSR and the CSC");
  if (g->nnz > 0 && (!g->csr_col || !g->csc_row)) return fail(RLGL_EINVAL, "link arrays missing");
  if ((g->csr_val == nullptr) != (g->csc_val == nullptr))
    return fail(RLGL_EINVAL, "csr_val and csc_val must both be given or both be NULL");
  if (!(eps >= 0.0) || max_steps < 0) return fail(RLGL_EINVAL, "eps must be >= 0 and max_steps >= 0");
  const int cap = small_capacity(o->precision);
  if (g->n > cap) return fail(RLGL_EINVAL, "n = %d exceeds the one-workgroup capacity %d", g->n, cap);
  const SmallLayout L = small_layout(g->n);
  if (!ws) return fail(RLGL_EINVAL, "workspace is NULL");
  if (ws_bytes < L.total) return fail(RLGL_ENOMEM, "workspace too small: %zu < %zu", ws_bytes, L.total);
  char *w = (char *)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
  int ends[2] = {0, 0};
  HIP_TRY(hipMemcpyAsync(&ends[0], g->csr_rowptr + g->n, sizeof(int), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipMemcpyAsync(&ends[1], g->csc_colptr + g->n, sizeof(int), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  if ((long long)ends[0] != g->nnz || (long long)ends[1] != g->nnz)
    return fail(RLGL_EINVAL, "csr_rowptr[n] = %d and csc_colptr[n] = %d must equal nnz = %lld", ends[0], ends[1],
                (long long)g->nnz);

  SmallArgs a{};
  a.n = g->n;
  a.nnz = g->nnz;
  a.c = g->damping;
  a.rowptr = g->csr_rowptr;
  a.col = g->csr_col;
  a.colptr = g->csc_colptr;
  a.crow = g->csc_row;
  a.val = g->csr_val;
  a.cval = g->csc_val;
  a.sched = o->sched;
  a.r = o->r;
  a.theta_period = o->theta_period;
  a.seed = o->seed;
  a.refresh = o->refresh > 0 ? 1 : 0;
  a.eps = eps;
  a.max_steps = max_steps;
  a.H = (double *)(w + L.H);
  a.Q = (double *)(w + L.Q);
  a.rec = (SmallRec *)(w + L.rec);
  a.pi = dev_pi;
  const int cs = o->precision == RLGL_FP64 ? 8 : 4;
  size_t dyn = align_up((size_t)g->n * cs, 16);
  // the row pointers go into LDS after the cash when both fit
  const size_t with_rp = dyn + align_up(4 * ((size_t)g->n + 1), 16);
  a.rp_lds = (long long)with_rp <= small_lds_budget(o->precision) ? 1 : 0;
  if (a.rp_lds) dyn = with_rp;
  HIP_TRY(hipFuncSetAttribute(small_kernel(o->precision), hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn));
  if (o->precision == RLGL_FP64) k_small<double><<<1, SM_BLOCK, dyn, stream>>>(a);
  else k_small<float><<<1, SM_BLOCK, dyn, stream>>>(a);
  HIP_TRY(hipGetLastError());
  SmallRec r{};
  HIP_TRY(hipMemcpyAsync(&r, a.rec, sizeof r, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  const rlgl_status rs = (r.status == ST_CONVERGED) ? RLGL_OK : status_of(r.status);
  if (info) {
    info->t = r.t;
    info->green = r.green;
    info->green_total = r.green_total;
    info->edges_pushed = r.edges;
    info->l1_cash = r.l1;
    info->h_sum = r.hsum;
    info->resid = r.hsum != 0.0 ? r.l1 / std::fabs(r.hsum) : INFINITY;
    info->theta = r.theta;
    info->cash_sum = r.csum;
    info->status = rs;
    info->last_route = r.last_route;
  }
  if (r.status == ST_BAD_GRAPH)
    return fail(RLGL_EINVAL, "a row or column pointer or a link index of the graph is out of range");
  if (rs != RLGL_OK) return fail(rs, "one-workgroup solve stopped at t = %lld (device status %d)", r.t, r.status);
  return RLGL_OK;
}

}  // namespace

extern "C" {

int32_t rlgl_small_max_n(int32_t precision) {
  if (precision < 0 || precision > 2) return 0;
  return small_capacity(precision);
}

size_t rlgl_small_workspace_bytes(int32_t n) {
  if (n < 1) return 0;
  return small_layout(n).total;
}

rlgl_status rlgl_solve_small(const rlgl_graph *g, const rlgl_options *opt, double eps, int64_t max_steps,
                             double *dev_pi, void *dev_workspace, size_t ws_bytes, void *stream,
                             rlgl_step_info *info) {
  return small_solve(g, opt, eps, max_steps, dev_pi, (char *)dev_workspace, ws_bytes, (hipStream_t)stream, info);
}

}  // extern "C"

extern "C" {

rlgl_status rlgl_solve_small_static(const rlgl_graph *g, const rlgl_options *opt, double eps, int64_t max_steps,
                                    double *dev_pi, void *stream, rlgl_step_info *info) {
  if (!g) return fail(RLGL_EINVAL, "null argument");
  if (g->n < 1) return fail(RLGL_EINVAL, "n must be >= 1");
  const size_t need = small_layout(g->n).total;
  if (need > (size_t)RLGL_SMALL_STATIC_BYTES)
    return fail(RLGL_EINVAL, "n = %d needs %zu workspace bytes, beyond the static %zu", g->n, need,
                (size_t)RLGL_SMALL_STATIC_BYTES);
  char *ws = nullptr;
  const rlgl_status st = static_scratch(&ws);
  if (st != RLGL_OK) return st;
  return small_solve(g, opt, eps, max_steps, dev_pi, ws, (size_t)RLGL_SMALL_STATIC_BYTES, (hipStream_t)stream, info);
}

}  // extern "C"
