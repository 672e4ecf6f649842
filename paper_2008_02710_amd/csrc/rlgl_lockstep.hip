// Step-synchronous batched RLGL: every active chain advances one green-light
// step per iteration, and one iteration is three launches that span all of
// them at once:
//
//   k_ls_select  - one workgroup per tile of LS_TILE nodes of an active chain:
//                  green test on the snapshot C_t (Sec. 2.1, eq. (4)),
//                  H += M (eq. (5)), the restart pool T and sum M, and the
//                  scaled green mass M_j / outdeg(j) of every node into the
//                  chain's source buffer;
//   k_ls_route   - plan items (the pieces of the long columns of every
//                  chain first, then runs of at most CH links), one per
//                  workgroup or strided over a machine-sized grid: the CSC
//                  gather of eq. (6), C_{t+1}[k] = kept(k) + c sum_j src[j]
//                  + T/N, and the statistics of C_{t+1} (in the relabelled
//                  layout what the LS_HUB lowest-numbered states send is
//                  staged in LDS per item); a piece of a column with more
//                  than CH in-links adds its partial sum into the chain's
//                  FP64 long-column accumulator;
//   k_ls_control - one wave per active chain: finishes the long columns,
//                  adds up the chain's statistics,
//                  applies the stop test of Algorithm 1 step (7), the drift
//                  and stop-confirming FP64 refresh (eq. (7)), the step
//                  limit, and sets the threshold and the mode of the next
//                  iteration.
//
// A chain's state is its control record (mode, step, running H.1, ...) and
// LS_NS striped accumulators; the kernels of an iteration read the record and
// add into the stripes, the control kernel folds and clears them.  Chains
// that have stopped cost one record load per workgroup until the host drops
// them from the active list.  The link weights are implicit, 1/outdeg(j) in
// FP64, so the refresh that confirms a stop is exact to FP64 rounding (its
// scaled history H_j / outdeg(j) is gathered in FP64).  A batch may keep
// each chain in a relabelled layout (states renumbered by decreasing
// out-degree): every pass works in that numbering and only the final pass
// writes pi_hat back in the caller's.
#include "rlgl_device.h"

namespace rlgl {

constexpr int LS_NS = 16;       // stat stripes per chain
constexpr int LS_TILE = 1024;   // nodes per select workgroup (BLOCK threads x VPT)
constexpr int LS_PIECE = 4096;  // links per piece of a long column
constexpr int LS_HUB = 1024;    // FP32 send values staged per route item
static_assert(LS_TILE == BLOCK * VPT, "select tile");

enum : int { LS_IDLE = 0, LS_INIT = 1, LS_STEP = 2, LS_REFRESH = 3, LS_FINISH = 4, LS_DONE = 5 };

// Where a chain lives: chain-local node ids, device pointers.
struct LsChain {
  const int *rowptr;  // [n+1] CSR row pointers (out-degrees)
  const int *colptr;  // [n+1] CSC column pointers, 0-based
  const int *crow;    // [nnz] CSC sources
  const int4 *items;      // plan: n_piece pieces of long columns, then n_run runs
  const int *long_cols;   // [n_long] the columns with more than CH links
  double *long_acc;       // [n_long] their partial sums, zero between passes
  void *cash0, *cash1, *src;
  void *hist;
  float *hist_lo;
  double *pi;
  const int *perm;  // relabelled layout: [n] caller id of each state, else null
  long long nnz, max_steps;
  double c, eps;
  int n, n_piece, n_run, n_long;
};

// Per-chain control record, written by k_ls_control (and k_ls_select at step 0).
struct LsCtl {
  long long t, refreshed, edges, t0, t1;
  double theta, maxabs, hsum, hnorm, resid;
  int mode, buf, status, green_steps;
  int bad, pad_;  // a route met a link index or plan item outside its range
};

struct alignas(128) LsStripe {
  double l1, cs, sr;       // statistics of the cash vector a route pass produced
  unsigned long long mx;   // max |C| as the bits of a non-negative double
  double T, msum, dh, ge;  // select: restart pool, moved mass, |H| change, green links
};

struct LsArgs {
  const LsChain *chains;
  LsCtl *ctl;
  LsStripe *stats;
  const int *act;   // [n_act] active chain slots
  const int *tpre;  // [n_act+1] exclusive prefix of select tiles
  const int *wpre;  // [n_act+1] exclusive prefix of long-column pieces
  const int *rpre;  // [n_act+1] exclusive prefix of run items
  unsigned int *done;
  int n_act, w_total, r_total;
  int sched, refresh;
  double r;
};

// Largest a in [0, n_act) with pre[a] <= b, given pre[0] <= b < pre[n_act].
__device__ __forceinline__ int ls_find(const int *pre, int n_act, int b) {
  int lo = 0, hi = n_act;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <int HK>
__device__ __forceinline__ double ls_hist(const LsChain &ch, int i) {
  if (HK == 0) return ((const double *)ch.hist)[i];
  return (double)((const float *)ch.hist)[i] + (double)ch.hist_lo[i];
}

template <class T, int HK>
__global__ __launch_bounds__(BLOCK) void k_ls_select(LsArgs a) {
  const int ai = ls_find(a.tpre, a.n_act, blockIdx.x);
  const int k = a.act[ai];
  const int tile = blockIdx.x - a.tpre[ai];
  LsCtl *ctl = &a.ctl[k];
  const int mode = ctl->mode;
  if (mode != LS_INIT && mode != LS_STEP && mode != LS_REFRESH && mode != LS_FINISH) return;
  const LsChain ch = a.chains[k];
  const int n = ch.n;
  const double c = ch.c;
  const int *__restrict__ rowptr = ch.rowptr;
  const T *__restrict__ cur = (const T *)(ctl->buf ? ch.cash1 : ch.cash0);
  T *__restrict__ src = (T *)ch.src;
  double *H64 = (double *)ch.hist;
  float *Hhi = (float *)ch.hist;
  float *Hlo = ch.hist_lo;
  const double theta = ctl->theta, maxabs = ctl->maxabs, hsum = ctl->hsum;
  const int sched = a.sched;
  const T m0 = (T)(1.0 / (double)n);
  __shared__ double sh_red[4 * NWAVE];
  double aT = 0.0, aM = 0.0, aD = 0.0, aE = 0.0;
#pragma unroll
  for (int q = 0; q < VPT; ++q) {
    const int i = tile * LS_TILE + q * BLOCK + threadIdx.x;
    if (i >= n) continue;
    const int dg = rowptr[i + 1] - rowptr[i];
    if (mode == LS_FINISH) {
      ch.pi[ch.perm ? ch.perm[i] : i] = ls_hist<HK>(ch, i) / hsum;  // eq. (2), in the caller's numbering
    } else if (mode == LS_REFRESH) {
      // the FP64 scaled history H_j / outdeg(j) for the route, parked in the
      // output vector, which is not written before the final pass
      const double h = ls_hist<HK>(ch, i);
      aT += h * (dg > 0 ? 1.0 - c : 1.0);
      ch.pi[i] = dg > 0 ? h / (double)dg : 0.0;
    } else if (mode == LS_INIT) {
      // eq. (3): H_1 = M_0 = (1/N) 1, every node green
      if (HK == 0) {
        H64[i] = (double)m0;
      } else {
        Hhi[i] = (float)m0;
        Hlo[i] = 0.0f;
      }
      src[i] = dg > 0 ? (T)((double)m0 / (double)dg) : T(0);
      aM += (double)m0;
      aT += dg > 0 ? (1.0 - c) * (double)m0 : (double)m0;
      aE += (double)dg;
    } else {
      const T x = cur[i];
      const bool g = x != T(0) && is_green(x, i, sched, theta, maxabs, 0.0, -1);
      T s = T(0);
      if (g) {
        if (HK == 0) {
          const double h = H64[i], hn = h + (double)x;
          H64[i] = hn;
          aD += fabs(hn) - fabs(h);
        } else {
          // compensated (Kahan-Babuska) FP32 pair
          const float hi = Hhi[i], lo = Hlo[i], xf = (float)x;
          const float sum = hi + xf;
          const float comp = (fabsf(hi) >= fabsf(xf)) ? ((hi - sum) + xf) : ((xf - sum) + hi);
          const float lo2 = lo + comp;
          Hhi[i] = sum;
          Hlo[i] = lo2;
          aD += fabs((double)sum + (double)lo2) - fabs((double)hi + (double)lo);
        }
        aM += (double)x;
        aT += dg > 0 ? (1.0 - c) * (double)x : (double)x;
        aE += (double)dg;
        if (dg > 0) s = (T)((double)x / (double)dg);
      }
      src[i] = s;
    }
  }
  if (mode == LS_FINISH) return;
  const Red4 t4 = block_sum4(Red4{aT, aM, aD, aE}, sh_red);
  if (threadIdx.x == 0) {
    LsStripe *st = &a.stats[(size_t)k * LS_NS + tile % LS_NS];
    if (t4.a != 0.0) atomic_add_f64(&st->T, t4.a);
    if (t4.b != 0.0) atomic_add_f64(&st->msum, t4.b);
    if (t4.c != 0.0) atomic_add_f64(&st->dh, t4.c);
    if (t4.d != 0.0) atomic_add_f64(&st->ge, t4.d);
    if (mode == LS_INIT && tile == 0) ctl->t0 = wall_clock64();
  }
}

// One plan item of chain k (its index `local` in the chain's plan): step 0
// (C_1 = 0 - M_0 + M_0 P), a green-light step, or the refresh C_t = H_t P -
// H_t (eq. (7) with C_0 = 0) from the FP64 scaled history.  Adds the
// statistics of the written values to l1..mx.
template <class T, int HK, int NT, bool FRESH>
__device__ __forceinline__ void ls_item(const LsArgs &a, int k, int mode, int local, double off, ColLds<NT> &L,
                                        T *hub, double &l1, double &cs, double &sr, double &mx) {
  const LsChain ch = a.chains[k];
  const LsCtl *ctl = &a.ctl[k];
  const int n = ch.n;
  int *bad = &a.ctl[k].bad;
  const ColView g{ch.colptr, ch.crow, ch.rowptr, nullptr, n, 1, bad};
  const int buf = ctl->buf;
  const T *__restrict__ cur = (const T *)(buf ? ch.cash1 : ch.cash0);
  T *__restrict__ out = (T *)(buf ? ch.cash0 : ch.cash1);
  const T *__restrict__ src = (const T *)ch.src;
  const int4 item = ch.items[local];
  const bool refresh = mode == LS_REFRESH, init = mode == LS_INIT;
  const double *__restrict__ hs = ch.pi;
  const double m0 = (double)(T)(1.0 / (double)n);
  const double theta = ctl->theta, maxabs = ctl->maxabs;
  const int sched = a.sched;
  // What the LS_HUB lowest-numbered states send, staged in LDS for the item:
  // in the relabelled layout they are the chain's largest out-degrees (in the
  // caller's numbering they are no one in particular, and nothing is staged)
  const int hn = (!refresh && sizeof(T) == 4 && ch.perm) ? min(LS_HUB, n) : 0;
  if (hn > 0) {  // the same for the whole workgroup
    if (!FRESH) __syncthreads();  // the previous item's reads of the table are done
    for (int q = threadIdx.x; q < hn; q += NT) hub[q] = src[q];
    __syncthreads();
  }
  column_item<T, NT>(
      g, item,
      [&](int j) -> double {
        // a load at a clamped index and a select, not a branch per link; a
        // link outside [0, n) sends nothing and is reported
        const bool ok = (unsigned)j < (unsigned)n;
        if (!ok) *bad = 1;
        const unsigned int jc = ok ? (unsigned int)j : 0u;
        const double v = refresh ? hs[jc] : (double)(jc < (unsigned int)hn ? hub[jc] : src[jc]);
        return ok ? v : 0.0;
      },
      [&](int kk) -> double {
        if (init) return -m0;
        if (refresh) return -ls_hist<HK>(ch, kk);
        const T v = cur[kk];
        return is_green(v, kk, sched, theta, maxabs, 0.0, -1) ? 0.0 : (double)v;
      },
      ch.c, off, a.r, out, ch.long_acc, L, l1, cs, sr, mx);
}

// The pool T of chain k's pass from its select statistics (one wave adds the
// stripes), divided by N.
template <int NT>
__device__ __forceinline__ double ls_offset(const LsArgs &a, int k, double *sh) {
  if (threadIdx.x < 64) {
    double v = threadIdx.x < LS_NS ? a.stats[(size_t)k * LS_NS + threadIdx.x].T : 0.0;
    v = wave_sum(v);
    if (threadIdx.x == 0) *sh = v;
  }
  __syncthreads();
  return *sh / (double)a.chains[k].n;
}

template <int NT>
__device__ __forceinline__ void ls_fold(const LsArgs &a, int k, int stripe, double l1, double cs, double sr,
                                        double mx, ColLds<NT> &L) {
  constexpr int NW = NT / 64;
  const Red4 t4 = block_sum4<NW>(Red4{l1, cs, sr, 0.0}, L.red);
  const double bm = block_max<NW>(mx, L.red);
  if (threadIdx.x == 0) {
    LsStripe *st = &a.stats[(size_t)k * LS_NS + stripe];
    if (t4.a != 0.0) atomic_add_f64(&st->l1, t4.a);
    if (t4.b != 0.0) atomic_add_f64(&st->cs, t4.b);
    if (t4.c != 0.0) atomic_add_f64(&st->sr, t4.c);
    if (bm > 0.0) atomic_max_nonneg(&st->mx, bm);
  }
}

__device__ __forceinline__ bool ls_routes(int mode) { return mode == LS_INIT || mode == LS_STEP || mode == LS_REFRESH; }

// One workgroup per plan item.
template <class T, int HK, int NT>
__global__ __launch_bounds__(NT) void k_ls_route(LsArgs a) {
  __shared__ ColLds<NT> L;
  __shared__ double sh_T;
  __shared__ T s_hub[sizeof(T) == 4 ? LS_HUB : 1];
  const bool piece = (int)blockIdx.x < a.w_total;
  const int b = piece ? (int)blockIdx.x : (int)blockIdx.x - a.w_total;
  const int ai = ls_find(piece ? a.wpre : a.rpre, a.n_act, b);
  const int k = a.act[ai];
  const int mode = a.ctl[k].mode;
  if (!ls_routes(mode)) return;
  const int local = piece ? b - a.wpre[ai] : a.chains[k].n_piece + (b - a.rpre[ai]);
  const double off = ls_offset<NT>(a, k, &sh_T);
  double l1 = 0.0, cs = 0.0, sr = 0.0, mx = 0.0;
  ls_item<T, HK, NT, true>(a, k, mode, local, off, L, s_hub, l1, cs, sr, mx);
  ls_fold<NT>(a, k, local % LS_NS, l1, cs, sr, mx, L);
}

// Plan items strided over a machine-sized grid; the pool and the statistics
// are kept across consecutive items of one chain.
template <class T, int HK, int NT>
__global__ __launch_bounds__(NT) void k_ls_route_strided(LsArgs a) {
  __shared__ ColLds<NT> L;
  __shared__ double sh_T;
  __shared__ T s_hub[sizeof(T) == 4 ? LS_HUB : 1];
  const int total = a.w_total + a.r_total;
  const int stripe = blockIdx.x % LS_NS;
  int kc = -1, mode = LS_IDLE;  // chain of the previous item, its mode
  double off = 0.0;
  double l1 = 0.0, cs = 0.0, sr = 0.0, mx = 0.0;
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    const bool piece = it < a.w_total;
    const int b = piece ? it : it - a.w_total;
    const int ai = ls_find(piece ? a.wpre : a.rpre, a.n_act, b);
    const int k = a.act[ai];
    if (k != kc) {
      if (kc >= 0) {
        ls_fold<NT>(a, kc, stripe, l1, cs, sr, mx, L);
        l1 = cs = sr = mx = 0.0;
      }
      kc = k;
      mode = a.ctl[k].mode;
      if (ls_routes(mode)) off = ls_offset<NT>(a, k, &sh_T);
    }
    if (!ls_routes(mode)) continue;
    const int local = piece ? b - a.wpre[ai] : a.chains[k].n_piece + (b - a.rpre[ai]);
    ls_item<T, HK, NT, false>(a, k, mode, local, off, L, s_hub, l1, cs, sr, mx);
  }
  if (kc >= 0) ls_fold<NT>(a, kc, stripe, l1, cs, sr, mx, L);
}

// One wave per active chain.
template <class Tc, int HK>
__global__ __launch_bounds__(64) void k_ls_control(LsArgs a) {
  const int ai = blockIdx.x;
  if (ai >= a.n_act) return;
  const int k = a.act[ai];
  LsCtl *ctl = &a.ctl[k];
  const int mode = ctl->mode;
  if (mode == LS_IDLE || mode == LS_DONE) return;
  const int lane = threadIdx.x;
  LsStripe *st = &a.stats[(size_t)k * LS_NS];
  double l1 = 0, cs = 0, sr = 0, mx = 0, T = 0, ms = 0, dh = 0, ge = 0;
  if (lane < LS_NS) {
    const LsStripe &s = st[lane];
    l1 = s.l1;
    cs = s.cs;
    sr = s.sr;
    mx = __longlong_as_double((long long)s.mx);
    T = s.T;
    ms = s.msum;
    dh = s.dh;
    ge = s.ge;
  }
  T = wave_sum(T);
  const LsChain &ch = a.chains[k];
  if ((mode == LS_INIT || mode == LS_STEP || mode == LS_REFRESH) && ch.n_long > 0) {
    // the columns with more than CH links: x_k = kept(k) + c acc_k + T/N
    const int n = ch.n;
    const double off = T / (double)n, c = ch.c;
    const Tc *cur = (const Tc *)(ctl->buf ? ch.cash1 : ch.cash0);
    Tc *out = (Tc *)(ctl->buf ? ch.cash0 : ch.cash1);
    const double theta = ctl->theta, maxabs = ctl->maxabs;
    const double m0 = (double)(Tc)(1.0 / (double)n);
    for (int q = lane; q < ch.n_long; q += 64) {
      const int kk = ch.long_cols[q];
      const double acc = ch.long_acc[q];
      ch.long_acc[q] = 0.0;
      double kept;
      if (mode == LS_INIT) {
        kept = -m0;
      } else if (mode == LS_REFRESH) {
        kept = -ls_hist<HK>(ch, kk);
      } else {
        const Tc v = cur[kk];
        kept = is_green(v, kk, a.sched, theta, maxabs, 0.0, -1) ? 0.0 : (double)v;
      }
      const Tc x = (Tc)(kept + c * acc + off);
      out[kk] = x;
      fold_stats((double)x, a.r, l1, cs, sr, mx);
    }
  }
  l1 = wave_sum(l1);
  cs = wave_sum(cs);
  sr = wave_sum(sr);
  mx = wave_max(mx);
  ms = wave_sum(ms);
  dh = wave_sum(dh);
  ge = wave_sum(ge);
  if (lane < LS_NS) {
    LsStripe &s = st[lane];
    s.l1 = 0.0;
    s.cs = 0.0;
    s.sr = 0.0;
    s.mx = 0ull;
    s.T = 0.0;
    s.msum = 0.0;
    s.dh = 0.0;
    s.ge = 0.0;
  }
  if (lane != 0) return;
  if (mode == LS_FINISH) {
    ctl->mode = LS_DONE;
    ctl->t1 = wall_clock64();
    atomicAdd(a.done, 1u);
    return;
  }
  long long t = ctl->t, refreshed = ctl->refreshed;
  double hsum = ctl->hsum, hnorm = ctl->hnorm;
  if (mode == LS_INIT) {
    hsum = ms;
    hnorm = ms;
    ctl->edges = (long long)ge;
    t = 1;
  } else if (mode == LS_STEP) {
    hsum += ms;
    hnorm += dh;
    ctl->edges += (long long)ge;
    ctl->green_steps += 1;
    t += 1;
  } else {
    refreshed = t;
  }
  ctl->buf ^= 1;
  ctl->t = t;
  ctl->refreshed = refreshed;
  ctl->hsum = hsum;
  ctl->hnorm = hnorm;
  const double resid = l1 / fabs(hsum);
  ctl->resid = resid;
  int next = LS_STEP, status = 0;
  if (ctl->bad) {
    status = ST_BAD_GRAPH;
  } else if (!isfinite(l1) || !isfinite(hsum)) {
    status = ST_NONFINITE;
  } else if (fabs(hsum) <= 1e-300 || fabs(hsum) <= 1e-12 * hnorm) {
    status = ST_ZERO_HISTORY;
  } else {
    // FP32 rounding leaves C_t 1 != 0: once the drift is half of ||C_t||_1, or
    // before accepting a stop, the cash is rebuilt from H in FP64
    const bool drift = fabs(cs) > 0.5 * l1 && l1 > 0.0;
    const bool stop = t >= 2 && resid < ch.eps;
    if ((stop || drift) && a.refresh && refreshed != t) next = LS_REFRESH;
    else if (stop) status = ST_CONVERGED;
    else if (t - 1 >= ch.max_steps) status = ST_LIMIT;
  }
  if (status != 0) {
    ctl->status = status;
    if (status != ST_NONFINITE && status != ST_BAD_GRAPH && hsum != 0.0) {
      next = LS_FINISH;
    } else {
      next = LS_DONE;
      ctl->t1 = wall_clock64();
      atomicAdd(a.done, 1u);
    }
  } else if (next == LS_STEP) {
    ctl->theta = (a.sched == SCHED_THRESHOLD) ? (a.r == 1.0 ? l1 / (double)ch.n : pow(sr / (double)ch.n, 1.0 / a.r))
                                              : 0.0;
    ctl->maxabs = mx;
  }
  ctl->mode = next;
}

// Puts chains [0, count) of the slots in `ids` at the start of a solve: mode
// LS_INIT, counters cleared, stripes and long-column sums zeroed.
__global__ void k_ls_start(const LsChain *chains, LsCtl *ctl, LsStripe *stats, const int *ids, int count,
                           unsigned int *done) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q == 0) *done = 0u;
  if (q >= count) return;
  const int k = ids[q];
  const LsChain &ch = chains[k];
  for (int i = 0; i < ch.n_long; ++i) ch.long_acc[i] = 0.0;
  LsCtl z;
  z.t = 0;
  z.refreshed = -1;
  z.edges = 0;
  z.t0 = 0;
  z.t1 = 0;
  z.theta = 0.0;
  z.maxabs = 0.0;
  z.hsum = 0.0;
  z.hnorm = 0.0;
  z.resid = 0.0;
  z.mode = LS_INIT;
  z.buf = 0;
  z.status = 0;
  z.bad = 0;
  z.pad_ = 0;
  z.green_steps = 0;
  ctl[k] = z;
  for (int s = 0; s < LS_NS; ++s) {
    LsStripe &w = stats[(size_t)k * LS_NS + s];
    w.l1 = 0.0;
    w.cs = 0.0;
    w.sr = 0.0;
    w.mx = 0ull;
    w.T = 0.0;
    w.msum = 0.0;
    w.dh = 0.0;
    w.ge = 0.0;
  }
}

// Writes one chain's descriptor and starts it (pool admission).
__global__ void k_ls_admit(LsChain *chains, LsCtl *ctl, LsStripe *stats, int slot, LsChain ch) {
  for (int i = threadIdx.x; i < ch.n_long; i += blockDim.x) ch.long_acc[i] = 0.0;
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  chains[slot] = ch;
  LsCtl z;
  z.t = 0;
  z.refreshed = -1;
  z.edges = 0;
  z.t0 = 0;
  z.t1 = 0;
  z.theta = 0.0;
  z.maxabs = 0.0;
  z.hsum = 0.0;
  z.hnorm = 0.0;
  z.resid = 0.0;
  z.mode = LS_INIT;
  z.buf = 0;
  z.status = 0;
  z.bad = 0;
  z.pad_ = 0;
  z.green_steps = 0;
  ctl[slot] = z;
  for (int s = 0; s < LS_NS; ++s) {
    LsStripe &w = stats[(size_t)slot * LS_NS + s];
    w.l1 = 0.0;
    w.cs = 0.0;
    w.sr = 0.0;
    w.mx = 0ull;
    w.T = 0.0;
    w.msum = 0.0;
    w.dh = 0.0;
    w.ge = 0.0;
  }
}

template __global__ void k_ls_select<float, 0>(LsArgs);
template __global__ void k_ls_select<float, 1>(LsArgs);
template __global__ void k_ls_select<double, 0>(LsArgs);
template __global__ void k_ls_route<float, 0, 256>(LsArgs);
template __global__ void k_ls_route<float, 1, 256>(LsArgs);
template __global__ void k_ls_route<double, 0, 256>(LsArgs);
template __global__ void k_ls_route<float, 0, 512>(LsArgs);
template __global__ void k_ls_route<float, 1, 512>(LsArgs);
template __global__ void k_ls_route<double, 0, 512>(LsArgs);
template __global__ void k_ls_route_strided<float, 0, 256>(LsArgs);
template __global__ void k_ls_route_strided<float, 1, 256>(LsArgs);
template __global__ void k_ls_route_strided<double, 0, 256>(LsArgs);
template __global__ void k_ls_route_strided<float, 0, 512>(LsArgs);
template __global__ void k_ls_route_strided<float, 1, 512>(LsArgs);
template __global__ void k_ls_route_strided<double, 0, 512>(LsArgs);
template __global__ void k_ls_control<float, 0>(LsArgs);
template __global__ void k_ls_control<float, 1>(LsArgs);
template __global__ void k_ls_control<double, 0>(LsArgs);

}  // namespace rlgl
