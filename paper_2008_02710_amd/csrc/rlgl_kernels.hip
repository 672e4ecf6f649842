// Device side of the MI355X (gfx950) Red-Light-Green-Light solver.
//
// One green-light step t (Sec. 2.1, eqs. (4)-(6), Algorithm 1 steps (2)-(6))
// runs as three launches on the caller's stream:
//
//   k_select   - stop test of Algorithm 1 step (7) on C_t, threshold theta_t,
//                green test of every node on the snapshot C_t, H += M,
//                sum M, the restart pool T, and for push routing the
//                compaction of the green rows into a frontier (wave ballot +
//                block scan + one 64-bit atomic per tile).
//   k_push     - scatter c*P_ij*M_i along the CSR rows of the frontier
//                (edge-balanced: fixed chunks of links, the frontier row of
//                each link found by a search in LDS).  Pull steps skip it.
//   k_complete - push: adds the uniform restart share T/N to every node;
//                pull: gathers sum_j M_j c P_jk along the CSC columns into
//                the other cash buffer, M_j recomputed from the snapshot.
//                Both fold ||C_{t+1}||_1, sum C, sum |C|^r and max |C| into
//                the record of step t+1.
//
// All reductions are FP64.  Per-step scalars live in a ring of three device
// records indexed by t mod 3, so the host never touches them between steps:
// the kernels of step t read record t, accumulate into record t (select) or
// t+1 (complete), and select clears record t+1 before anyone uses it.  Block
// partial sums go to one of NSTRIPE stripes of a record (same-address atomics
// serialise), and readers add the stripes up with one wave.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rlgl_device.h"

namespace rlgl {

// ---------------------------------------------------------------- helpers

// Lane moves through DPP (the GFX9 encodings): row_shr:n shifts inside each
// row of 16 lanes, row_bcast:15 hands a row's last lane to the next row,
// row_bcast:31 hands lane 31 to rows 2 and 3, wave_shr:1 shifts the whole
// wave by one lane.  A lane with no source, or in a row the mask leaves out,
// reads 0.
constexpr int DPP_ROW_SHR1 = 0x111, DPP_ROW_SHR2 = 0x112, DPP_ROW_SHR4 = 0x114, DPP_ROW_SHR8 = 0x118;
constexpr int DPP_ROW_BCAST15 = 0x142, DPP_ROW_BCAST31 = 0x143, DPP_WAVE_SHR1 = 0x138;

template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_i32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xF, true);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned int lo = (unsigned int)dpp_i32<CTRL, ROWS>((int)(unsigned int)b);
  const unsigned int hi = (unsigned int)dpp_i32<CTRL, ROWS>((int)(unsigned int)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// One step of a segmented inclusive sum over the wave: the value from the
// lane the move names is added unless this lane already starts a segment.
template <int CTRL, int ROWS>
__device__ __forceinline__ void seg_scan_step(double &v, int &f) {
  const double yv = dpp_f64<CTRL, ROWS>(v);
  const int yf = dpp_i32<CTRL, ROWS>(f);
  if (!f) v += yv;
  f |= yf;
}

template <int CTRL, int ROWS>
__device__ __forceinline__ long long dpp_i64(long long v) {
  const unsigned long long b = (unsigned long long)v;
  const unsigned int lo = (unsigned int)dpp_i32<CTRL, ROWS>((int)(unsigned int)b);
  const unsigned int hi = (unsigned int)dpp_i32<CTRL, ROWS>((int)(unsigned int)(b >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ unsigned long long lane63_u64(unsigned long long b) {
  const unsigned int lo = (unsigned int)__builtin_amdgcn_readlane((int)(unsigned int)b, 63);
  const unsigned int hi = (unsigned int)__builtin_amdgcn_readlane((int)(unsigned int)(b >> 32), 63);
  return ((unsigned long long)hi << 32) | lo;
}

// Wave reductions through DPP moves (a lane with no source reads 0, so
// wave_max is for non-negative values); every lane receives the result.
__device__ __forceinline__ double wave_sum(double x) {
  x += dpp_f64<DPP_ROW_SHR1, 0xF>(x);
  x += dpp_f64<DPP_ROW_SHR2, 0xF>(x);
  x += dpp_f64<DPP_ROW_SHR4, 0xF>(x);
  x += dpp_f64<DPP_ROW_SHR8, 0xF>(x);
  x += dpp_f64<DPP_ROW_BCAST15, 0xA>(x);
  x += dpp_f64<DPP_ROW_BCAST31, 0xC>(x);
  return __longlong_as_double((long long)lane63_u64((unsigned long long)__double_as_longlong(x)));
}
__device__ __forceinline__ double wave_max(double x) {
  x = fmax(x, dpp_f64<DPP_ROW_SHR1, 0xF>(x));
  x = fmax(x, dpp_f64<DPP_ROW_SHR2, 0xF>(x));
  x = fmax(x, dpp_f64<DPP_ROW_SHR4, 0xF>(x));
  x = fmax(x, dpp_f64<DPP_ROW_SHR8, 0xF>(x));
  x = fmax(x, dpp_f64<DPP_ROW_BCAST15, 0xA>(x));
  x = fmax(x, dpp_f64<DPP_ROW_BCAST31, 0xC>(x));
  return __longlong_as_double((long long)lane63_u64((unsigned long long)__double_as_longlong(x)));
}
__device__ __forceinline__ long long wave_sum_ll(long long x) {
  x += dpp_i64<DPP_ROW_SHR1, 0xF>(x);
  x += dpp_i64<DPP_ROW_SHR2, 0xF>(x);
  x += dpp_i64<DPP_ROW_SHR4, 0xF>(x);
  x += dpp_i64<DPP_ROW_SHR8, 0xF>(x);
  x += dpp_i64<DPP_ROW_BCAST15, 0xA>(x);
  x += dpp_i64<DPP_ROW_BCAST31, 0xC>(x);
  return (long long)lane63_u64((unsigned long long)x);
}

// Block-wide sums of four doubles; every thread receives the result.
struct Red4 {
  double a, b, c, d;
};
template <int NW = NWAVE>
__device__ __forceinline__ Red4 block_sum4(Red4 v, double *sh /* 4*NW */) {
  v.a = wave_sum(v.a);
  v.b = wave_sum(v.b);
  v.c = wave_sum(v.c);
  v.d = wave_sum(v.d);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) {
    sh[w] = v.a;
    sh[NW + w] = v.b;
    sh[2 * NW + w] = v.c;
    sh[3 * NW + w] = v.d;
  }
  __syncthreads();
  Red4 r{0, 0, 0, 0};
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    r.a += sh[i];
    r.b += sh[NW + i];
    r.c += sh[2 * NW + i];
    r.d += sh[3 * NW + i];
  }
  __syncthreads();
  return r;
}
template <int NW = NWAVE>
__device__ __forceinline__ double block_max(double v, double *sh) {
  v = wave_max(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) sh[w] = v;
  __syncthreads();
  double r = sh[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) r = fmax(r, sh[i]);
  __syncthreads();
  return r;
}
__device__ __forceinline__ long long block_sum_ll(long long v, long long *sh) {
  v = wave_sum_ll(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) sh[w] = v;
  __syncthreads();
  long long r = 0;
#pragma unroll
  for (int i = 0; i < NWAVE; ++i) r += sh[i];
  __syncthreads();
  return r;
}
// Exclusive block scan of a 64-bit value; *total gets the block sum.
__device__ __forceinline__ unsigned long long block_excl_scan(unsigned long long x, unsigned long long *sh,
                                                              unsigned long long *total) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  unsigned long long inc = x;
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long y = __shfl_up(inc, o, 64);
    if (l >= o) inc += y;
  }
  if (l == 63) sh[w] = inc;
  __syncthreads();
  unsigned long long base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NWAVE; ++i) {
    const unsigned long long s = sh[i];
    if (i < w) base += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return base + inc - x;
}

__device__ __forceinline__ void atomic_add_f64(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add_cash(float *p, float v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add_cash(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_max_nonneg(unsigned long long *p, double v) {
  atomicMax(p, (unsigned long long)__double_as_longlong(v));
}
__device__ __forceinline__ double load_agent(const double *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ Acc *my_stripe(Rec *r) { return &r->acc[blockIdx.x % NSTRIPE]; }

// Totals of a record's stripes, computed by the first wave and broadcast.
__device__ Tot read_totals(const Rec *r, Tot *sh) {
  if (threadIdx.x < 64) {
    const int q = threadIdx.x;
    double l1 = 0, cs = 0, sr = 0, mx = 0, T = 0, ms = 0, dh = 0, hi = 0, hn = 0;
    long long gr = 0, ge = 0;
    if (q < NSTRIPE) {
      const Acc &a = r->acc[q];
      l1 = a.l1;
      cs = a.csum;
      sr = a.sumr;
      mx = __longlong_as_double((long long)a.maxabs_bits);
      T = a.T;
      ms = a.msum;
      dh = a.dhnorm;
      hi = a.hsum_import;
      hn = a.hnorm_import;
      gr = a.green;
      ge = a.gedges;
    }
    l1 = wave_sum(l1);
    cs = wave_sum(cs);
    sr = wave_sum(sr);
    mx = wave_max(mx);
    T = wave_sum(T);
    ms = wave_sum(ms);
    dh = wave_sum(dh);
    hi = wave_sum(hi);
    hn = wave_sum(hn);
    gr = wave_sum_ll(gr);
    ge = wave_sum_ll(ge);
    if (q == 0) *sh = Tot{l1, cs, sr, mx, T, ms, dh, hi, hn, gr, ge};
  }
  __syncthreads();
  const Tot t = *sh;
  __syncthreads();
  return t;
}

// Clears every stripe of a record (threads 0..NSTRIPE-1 of one block).
__device__ __forceinline__ void clear_stripes(Rec *r) {
  if (threadIdx.x < NSTRIPE) {
    Acc &a = r->acc[threadIdx.x];
    a.l1 = 0.0;
    a.csum = 0.0;
    a.sumr = 0.0;
    a.maxabs_bits = 0ull;
    a.T = 0.0;
    a.msum = 0.0;
    a.dhnorm = 0.0;
    a.green = 0;
    a.gedges = 0;
    a.hsum_import = 0.0;
    a.hnorm_import = 0.0;
  }
}

// Adds a block's statistics of a cash vector to its stripe of record r.
template <int NW = NWAVE>
// The waves' partials meet in LDS and wave 0 folds them with lane moves, so
// no thread holds the NW partials of all four sums at once.
__device__ __forceinline__ void fold_block_stats(Rec *r, double l1, double cs, double sr, double mx, double *sh) {
  static_assert(NW <= 64, "one lane of wave 0 per wave");
  l1 = wave_sum(l1);
  cs = wave_sum(cs);
  sr = wave_sum(sr);
  mx = wave_max(mx);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) {
    sh[w] = l1;
    sh[NW + w] = cs;
    sh[2 * NW + w] = sr;
    sh[3 * NW + w] = mx;
  }
  __syncthreads();
  if (w == 0) {
    const bool in = l < NW;
    const double a = wave_sum(in ? sh[l] : 0.0);
    const double b = wave_sum(in ? sh[NW + l] : 0.0);
    const double c = wave_sum(in ? sh[2 * NW + l] : 0.0);
    const double m = wave_max(in ? sh[3 * NW + l] : 0.0);
    if (l == 0) {
      Acc *acc = my_stripe(r);
      if (a != 0.0) atomic_add_f64(&acc->l1, a);
      if (b != 0.0) atomic_add_f64(&acc->csum, b);
      if (c != 0.0) atomic_add_f64(&acc->sumr, c);
      if (m > 0.0) atomic_max_nonneg(&acc->maxabs_bits, m);
    }
  }
  __syncthreads();
}

// RP = false: the caller knows r = 1 (no power sum, which keeps pow out of
// the register budget of the hot passes).
template <bool RP = true>
__device__ __forceinline__ void fold_stats(double x, double r, double &l1, double &cs, double &sr, double &mx) {
  const double a = fabs(x);
  l1 += a;
  cs += x;
  if (RP && r != 1.0) sr += pow(a, r);
  mx = fmax(mx, a);
}

// Green test of a node with cash v on the snapshot of step t.
// splitmix64 (Steele, Lea and Flood, 2014): output number `index` of the
// generator whose state starts at `seed` and advances by the golden gamma.
__device__ __forceinline__ unsigned long long splitmix64_at(unsigned long long seed, unsigned long long index) {
  unsigned long long z = seed + (index + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Green test of the node `id` with cash v on the snapshot C_t.  PC (RLGL_PC of
// Sec. 6, every node drawn at once): green with probability |v| / max |C_t|,
// the uniform draw being splitmix64 output t 2^32 + id, top 53 bits.
template <class T>
__device__ __forceinline__ bool is_green(T v, int id, int sched, double theta, double maxabs, double tau, int tie_id,
                                         unsigned long long seed = 0ull, long long t = 0,
                                         const unsigned char *mask = nullptr) {
  const double a = fabs((double)v);
  if (sched == SCHED_ALL) return true;
  if (sched == SCHED_MASK) return mask[id] != 0;  // the caller's green set
  if (sched == SCHED_THRESHOLD) return a >= theta;
  if (sched == SCHED_MAXC) return a == maxabs;
  if (sched == SCHED_PC) {
    if (!(maxabs > 0.0)) return false;
    const unsigned long long z = splitmix64_at(seed, ((unsigned long long)t << 32) + (unsigned int)id);
    const double u = (double)(z >> 11) * 0x1.0p-53;
    return u < a / maxabs;
  }
  return a > tau || (a == tau && id <= tie_id);  // top-k: k-th largest |C| and the id bound among its ties
}

__device__ __forceinline__ double inv_outdeg(const int *rowptr, int n, int j) {
  if ((unsigned)j >= (unsigned)n) return 0.0;
  const int dg = rowptr[j + 1] - rowptr[j];
  return dg > 0 ? 1.0 / (double)dg : 0.0;
}

template <int HK>
__device__ __forceinline__ double hist_at(const Dev &d, int j) {
  if (HK == 0) return ((const double *)d.hist)[j];
  return (double)((const float *)d.hist)[j] + (double)d.hist_lo[j];
}

// ------------------------------------------------------------------ select

// LDS of topk_fix_tau (defined with the top-k search below), which the select
// pass of a top-k step with FP32 keys calls to fix tau and the id bound.
struct TkFix {
  unsigned int h[TK_LOW_BINS];
  unsigned long long scan[NWAVE];
  int dig, seg, id;
  long long before, r;
};
__device__ __forceinline__ bool topk_fix_tau(const Dev &d, int G, TkFix &L, double *tau_out, int *tie_out);

template <class T, int HK>
__global__ __launch_bounds__(BLOCK) void k_select(Dev d, long long s, double eps, long long s_limit, int init) {
  Glob *g = d.glob;
  Rec *cur = &d.rec[s % 3];
  Rec *prv = &d.rec[(s + 2) % 3];
  Rec *nxt = &d.rec[(s + 1) % 3];

  __shared__ Tot sh_tot;
  __shared__ unsigned long long sh_scan[NWAVE];
  __shared__ double sh_red[4 * NWAVE];
  __shared__ long long sh_ll[NWAVE];
  __shared__ unsigned long long sh_base;

  // The node loads of this block's first tile depend on nothing the step's
  // scalars decide, so they are sent before the records are read.
  T *C = (T *)d.cash[cur->buf];
  const int n = d.n;
  const int ntiles = (n + TILE - 1) / TILE;
  T pv[VPT];
  int pr0[VPT], pr1[VPT];
  double ph[VPT];
  float plo[VPT];
  auto load_tile = [&](int tile) {
#pragma unroll
    for (int q = 0; q < VPT; ++q) {
      const int i = tile * TILE + q * BLOCK + threadIdx.x;
      const bool in = i < n;
      pv[q] = in ? C[i] : T(0);
      pr0[q] = in ? d.rowptr[i] : 0;
      pr1[q] = in ? d.rowptr[i + 1] : 0;
      if (HK == 0) {
        ph[q] = in ? ((const double *)d.hist)[i] : 0.0;
        plo[q] = 0.f;
      } else {
        ph[q] = in ? (double)((const float *)d.hist)[i] : 0.0;
        plo[q] = in ? d.hist_lo[i] : 0.f;
      }
    }
  };
  if ((int)blockIdx.x < ntiles) load_tile(blockIdx.x);
  if (sizeof(T) == 4 && !init && d.sched == SCHED_TOPK) {
    // the middle-digit counts of this step's top-k search, read only by
    // k_topk_narrow, start the next step at zero whatever this pass decides
    // (the low-digit ones, which it reads, are cleared by the next collect)
    for (int q = blockIdx.x * BLOCK + threadIdx.x; q < KH_STRIPES * KH_BINS; q += gridDim.x * BLOCK)
      d.tk_hist[q] = 0u;
  }
  if (g->status != 0) return;
  if (g->bad) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      g->status = ST_BAD_GRAPH;
      g->t = s;
    }
    return;
  }

  const Tot tot = read_totals(cur, &sh_tot);
  const double l1 = tot.l1, hsum = cur->hsum, hnorm = cur->hnorm;
  int st = 0;
  if (!init) {
    if (!isfinite(l1) || !isfinite(hsum)) st = ST_NONFINITE;
    else if (fabs(hsum) <= 1e-300 || fabs(hsum) <= 1e-12 * hnorm) st = ST_ZERO_HISTORY;
    else if (s >= 2 && l1 / fabs(hsum) < eps) st = ST_CONVERGED;
    else if (s >= s_limit) st = ST_LIMIT;
  }
  if (st != 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      g->status = st;
      g->t = s;
    }
    return;
  }

  const int sched = init ? SCHED_ALL : d.sched;
  double theta = 0.0;
  if (sched == SCHED_THRESHOLD) {
    if ((s - 1) % d.theta_period == 0)
      theta = (d.r == 1.0) ? l1 / (double)d.n : pow(tot.sumr / (double)d.n, 1.0 / d.r);
    else
      theta = prv->theta;
  }
  const double maxabs = tot.maxabs;
  double tau = cur->topk_tau;
  int tie_id = cur->topk_tie_id;
  if constexpr (sizeof(T) == 4) {
    if (sched == SCHED_TOPK) {
      // FP32 keys: every workgroup fixes tau and the id bound from what
      // k_topk_narrow counted (no launch of its own for one workgroup's work)
      __shared__ TkFix sh_fix;
      if (!topk_fix_tau(d, d.tk_grid, sh_fix, &tau, &tie_id)) {
        // the candidate lists do not hold what the histograms counted
        if (blockIdx.x == 0 && threadIdx.x == 0) {
          g->bad = 1;
          g->status = ST_BAD_GRAPH;
          g->t = s;
        }
        return;
      }
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        cur->topk_tau = tau;
        cur->topk_tie_id = tie_id;
      }
    }
  }
  // route: AUTO pulls when the previous step moved cash along at least
  // pull_alpha * nnz links (the log entry of step s-1)
  int mode;
  if (d.route == ROUTE_PUSH || d.colptr == nullptr) mode = 0;
  else if (d.route == ROUTE_PULL) mode = 1;
  else if (sched == SCHED_ALL) mode = 1;
  else mode = ((double)d.log[(s + LOG_STEPS - 1) % LOG_STEPS].gedges >= d.pull_alpha * (double)d.nnz) ? 1 : 0;

  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) {
      cur->theta = theta;
      cur->mode = mode;
      nxt->fr_pack = 0ull;
      nxt->ticket = 0u;
    }
    clear_stripes(nxt);
    if (d.khist && d.sched == SCHED_TOPK) {
      // the top-k histogram the complete pass of this step fills
      unsigned int *kh = d.khist + (size_t)((s + 1) % 3) * KH_STRIPES * KH_BINS;
      for (int q = threadIdx.x; q < KH_STRIPES * KH_BINS; q += BLOCK) kh[q] = 0u;
    }
  }

  const double c = d.c;

  double accT = 0.0, accM = 0.0, accDH = 0.0;
  long long accG = 0, accE = 0;

  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int base = tile * TILE;
    if (tile != (int)blockIdx.x) load_tile(tile);
    T v[VPT];
    int rs[VPT], deg[VPT];
    bool fr[VPT];
    unsigned int cnt = 0, edges = 0;
#pragma unroll
    for (int q = 0; q < VPT; ++q) {
      const int i = base + q * BLOCK + threadIdx.x;
      fr[q] = false;
      deg[q] = 0;
      rs[q] = 0;
      v[q] = T(0);
      const T x = pv[q];
      const bool gr = (i < n) && is_green(x, i, sched, theta, maxabs, tau, tie_id, d.seed, s, d.green_in);
      if (i < n) {
        if (d.green_mask) d.green_mask[i] = gr ? 1 : 0;
        T sent = T(0);  // pull: M_i P'_ij for each link i -> j (M_i itself with stored link values)
        if (gr) {
          ++accG;
          if (x != T(0)) {
            const int r0 = pr0[q];
            const int dg = pr1[q] - r0;
            if (d.cval) sent = x;
            else if (dg > 0) sent = (T)((double)x / (double)dg);
            // history: H_{t+1} = H_t + M_t (eq. (5))
            if (HK == 0) {
              double *H = (double *)d.hist;
              const double h = ph[q];
              const double hn = h + (double)x;
              H[i] = hn;
              accDH += fabs(hn) - fabs(h);
            } else {
              float *Hh = (float *)d.hist;
              float *Hl = d.hist_lo;
              const float hi = (float)ph[q], lo = plo[q], xf = (float)x;
              const float sum = hi + xf;
              const float comp = (fabsf(hi) >= fabsf(xf)) ? ((hi - sum) + xf) : ((xf - sum) + hi);
              const float lo2 = lo + comp;
              Hh[i] = sum;
              Hl[i] = lo2;
              accDH += fabs((double)sum + (double)lo2) - fabs((double)hi + (double)lo);
            }
            accM += (double)x;
            accT += (dg > 0) ? (1.0 - c) * (double)x : (double)x;
            accE += dg;
            if (mode == 0) {
              // C_t - M_t; the routed part arrives in k_push.  Step 0 starts
              // from C_0 = 0 while moving M_0 (held in C by k_reset): C_0 - M_0 = -M_0.
              C[i] = init ? -x : T(0);
              if (dg > 0) {
                fr[q] = true;
                v[q] = x;
                rs[q] = r0;
                deg[q] = dg;
                ++cnt;
                edges += (unsigned int)dg;
              }
            }
          }
        }
        if (mode == 1) ((T *)d.src)[i] = sent;
      }
    }
    if (mode == 0) {
      // frontier compaction: one 64-bit atomic per tile reserves both the
      // slots and the link range, so slot order and link order agree.
      unsigned long long tot2;
      const unsigned long long mine = ((unsigned long long)cnt << 32) | edges;
      const unsigned long long ex = block_excl_scan(mine, sh_scan, &tot2);
      if (threadIdx.x == 0) sh_base = tot2 ? atomicAdd(&cur->fr_pack, tot2) : 0ull;
      __syncthreads();
      const unsigned long long b = sh_base + ex;
      unsigned int slot = (unsigned int)(b >> 32);
      unsigned int eo = (unsigned int)(b & 0xffffffffu);
      __syncthreads();
#pragma unroll
      for (int q = 0; q < VPT; ++q) {
        if (fr[q]) {
          const int i = base + q * BLOCK + threadIdx.x;
          d.fr_rowstart[slot] = rs[q];
          d.fr_eoff[slot] = (int)eo;
          d.fr_id[slot] = i;
          double sc = c * (double)v[q];
          if (d.val == nullptr) sc /= (double)deg[q];
          ((T *)d.fr_scale)[slot] = (T)sc;
          // chunks whose first link lies in this row start at this slot
          const unsigned int first = (eo + CH - 1) / CH;
          const unsigned int last = (eo + (unsigned int)deg[q] - 1) / CH;
          for (unsigned int bch = first; bch <= last; ++bch) d.chunk_first[bch] = (int)slot;
          ++slot;
          eo += (unsigned int)deg[q];
        }
      }
    }
  }

  const Red4 r = block_sum4(Red4{accT, accM, accDH, 0.0}, sh_red);
  const long long gsum = block_sum_ll(accG, sh_ll);
  const long long esum = block_sum_ll(accE, sh_ll);
  if (threadIdx.x == 0) {
    Acc *a = my_stripe(cur);
    if (r.a != 0.0) atomic_add_f64(&a->T, r.a);
    if (r.b != 0.0) atomic_add_f64(&a->msum, r.b);
    if (r.c != 0.0) atomic_add_f64(&a->dhnorm, r.c);
    if (gsum) atomicAdd((unsigned long long *)&a->green, (unsigned long long)gsum);
    if (esum) atomicAdd((unsigned long long *)&a->gedges, (unsigned long long)esum);
  }
}

// -------------------------------------------------------------------- push

// The routed cash is summed in FP64: into C itself for FP64 cash, else into
// the delta array that complete folds into C with one rounding (adding many
// small amounts to a large FP32 value, as at an in-hub, loses them).  The
// destinations with the largest in-degrees are accumulated per workgroup in
// LDS and flushed once per workgroup: same-address global atomics serialise.
template <class T>
__global__ __launch_bounds__(BLOCK) void k_push(Dev d, long long s) {
  if (d.glob->status != 0) return;
  Rec *cur = &d.rec[s % 3];
  if (cur->mode != 0) return;
  const unsigned long long pk = cur->fr_pack;
  const int nent = (int)(pk >> 32);
  const int tot = (int)(pk & 0xffffffffu);
  if (tot == 0) return;
  double *__restrict__ D = d.delta ? d.delta : (double *)d.cash[cur->buf];
  const int *__restrict__ col = d.colt ? d.colt : d.col;
  const T *__restrict__ val = (const T *)d.val;
  const int nchunks = (tot + CH - 1) / CH;
  const int n_hot = d.n_hot;

  __shared__ int s_eoff[CH + 1];
  __shared__ int s_rs[CH + 1];
  __shared__ T s_sc[CH + 1];
  __shared__ double s_hot[HOT_MAX];
  for (int q = threadIdx.x; q < n_hot; q += BLOCK) s_hot[q] = 0.0;

  for (int b = blockIdx.x; b < nchunks; b += gridDim.x) {
    const int e0 = b * CH;
    const int e1 = min(tot, e0 + CH);
    const int j0 = d.chunk_first[b];
    const int j1 = (b + 1 < nchunks) ? d.chunk_first[b + 1] : nent - 1;
    // a chunk overlaps at most CH + 1 frontier rows (every row has a link);
    // anything else is a fault of the frontier, reported, never followed
    if (j0 < 0 || j1 >= nent || j1 < j0 || j1 - j0 + 1 > CH + 1) {
      d.glob->bad = 1;
      continue;
    }
    const int ne = j1 - j0 + 1;
    __syncthreads();
    for (int q = threadIdx.x; q < ne; q += BLOCK) {
      s_eoff[q] = d.fr_eoff[j0 + q];
      s_rs[q] = d.fr_rowstart[j0 + q];
      s_sc[q] = ((const T *)d.fr_scale)[j0 + q];
    }
    __syncthreads();
    for (int e = e0 + threadIdx.x; e < e1; e += BLOCK) {
      int lo = 0, hi = ne - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_eoff[mid] <= e) lo = mid;
        else hi = mid - 1;
      }
      const int idx = s_rs[lo] + (e - s_eoff[lo]);
      if ((unsigned long long)idx >= (unsigned long long)d.nnz) {
        d.glob->bad = 1;
        continue;
      }
      const int dst = col[idx];
      const double amt = val ? (double)s_sc[lo] * (double)val[idx] : (double)s_sc[lo];
      if (dst >= 0) {
        if (dst < d.n) atomic_add_f64(&D[dst], amt);
        else d.glob->bad = 1;  // a link outside [0, N): reported, never followed
      } else if (-1 - dst < n_hot) {
        atomicAdd(&s_hot[-1 - dst], amt);
      } else {
        d.glob->bad = 1;
      }
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < n_hot; q += BLOCK)
    if (s_hot[q] != 0.0) atomic_add_f64(&D[d.hot_nodes[q]], s_hot[q]);
}

// Setup: CSR columns with the hot destinations tagged (slot map in fr_id).
__global__ void k_tag_columns(Dev d, int *colt, const int *slot_of) {
  for (long long e = blockIdx.x * (long long)BLOCK + threadIdx.x; e < d.nnz; e += (long long)gridDim.x * BLOCK) {
    const int j = d.col[e];
    const int sl = ((unsigned)j < (unsigned)d.n) ? slot_of[j] : -1;
    colt[e] = sl >= 0 ? -1 - sl : j;
  }
}
__global__ void k_fill_int(int *p, int n, int v) {
  for (int i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) p[i] = v;
}
__global__ void k_scatter_slots(const int *hot, int n_hot, int *slot_of) {
  for (int q = blockIdx.x * BLOCK + threadIdx.x; q < n_hot; q += gridDim.x * BLOCK) slot_of[hot[q]] = q;
}
__global__ void k_indegree(Dev d, int *indeg) {
  for (long long e = blockIdx.x * (long long)BLOCK + threadIdx.x; e < d.nnz; e += (long long)gridDim.x * BLOCK) {
    const int j = d.col[e];
    if ((unsigned)j < (unsigned)d.n) atomicAdd(&indeg[j], 1);
  }
}

// ------------------------------------------------------------ top-k keys

template <class T>
__device__ __forceinline__ unsigned long long topk_key(T v) {
  if (sizeof(T) == 4) return (unsigned long long)__float_as_uint(fabsf((float)v));
  return (unsigned long long)__double_as_longlong(fabs((double)v));
}
template <class T>
__device__ __forceinline__ int kh_bin(T v) {
  return (int)(topk_key(v) >> (sizeof(T) == 4 ? 31 - KH_BITS : 63 - KH_BITS));
}
// Positions of the candidate list each collecting workgroup owns: a multiple
// of the workgroup size, so that the last one ends at or past n.
__device__ __forceinline__ int tk_segment(int n, int grid) {
  const int per = (n + grid - 1) / grid;
  return (per + BLOCK - 1) / BLOCK * BLOCK;
}
__device__ __forceinline__ unsigned int *khist_of(const Dev &d, long long s) {
  return d.khist + (size_t)(s % 3) * KH_STRIPES * KH_BINS;
}
// Adds one per active lane to h[bin] (bin < 2^BITS).  The lanes of a wave
// that share a bin are found with BITS ballots and counted by one atomic, so
// a histogram whose values crowd into a few bins costs one LDS atomic per
// distinct bin per wave instead of up to 64 on one address.  Every lane of
// the wave that is still executing must call it.
template <int BITS>
__device__ __forceinline__ void wave_hist_add(unsigned int *h, unsigned int bin, bool active) {
  unsigned long long same = __ballot(active);
#pragma unroll
  for (int b = 0; b < BITS; ++b) {
    const bool bit = (bin >> b) & 1u;
    const unsigned long long m = __ballot(bit);
    same &= bit ? m : ~m;
  }
  const int lane = threadIdx.x & 63;
  if (active && (same & ((1ull << lane) - 1ull)) == 0ull) atomicAdd(&h[bin], (unsigned int)__popcll(same));
}

// Adds a workgroup's LDS histogram to stripe blockIdx mod KH_STRIPES.
__device__ __forceinline__ void kh_flush(unsigned int *kh, const unsigned int *s_kh) {
  unsigned int *dst = kh + (size_t)(blockIdx.x % KH_STRIPES) * KH_BINS;
  for (int b = threadIdx.x; b < KH_BINS; b += blockDim.x)
    if (s_kh[b]) atomicAdd(&dst[b], s_kh[b]);
}
// The sum of the KH_STRIPES copies of a histogram into LDS (BLOCK threads):
// every load is sent before the first one is waited for.
__device__ __forceinline__ void kh_load(const unsigned int *kh, unsigned int *s_h) {
  constexpr int PB = KH_BINS / BLOCK;
  unsigned int c[PB];
#pragma unroll
  for (int u = 0; u < PB; ++u) c[u] = 0u;
#pragma unroll
  for (int q = 0; q < KH_STRIPES; ++q)
#pragma unroll
    for (int u = 0; u < PB; ++u) c[u] += kh[q * KH_BINS + u * BLOCK + threadIdx.x];
#pragma unroll
  for (int u = 0; u < PB; ++u) s_h[u * BLOCK + threadIdx.x] = c[u];
}

// ------------------------------------------------------- column gather pass
//
// Evaluates x_k = kept(k) + c * sum_{j in in(k)} moved(j) * P'_jk + off for
// every column k along the static plan and writes x_k to out, folding its
// statistics into record r.  P'_jk is the stored link value (or 1/outdeg(j)).
//
// Plan items: a RUN is a range of consecutive columns whose in-links (at most
// CH of them) are contiguous in the CSC arrays; one workgroup stages the CH
// contributions in LDS (coalesced index/value loads, 8 independent gathers
// per thread) and adds them up per column with a block-wide segmented scan,
// so every workgroup moves the same number of links whatever the degrees.
// A column with more than CH in-links is cut into PIECEs of CH links whose
// sums meet in long_acc; a later pass completes those columns (a
// last-workgroup ticket would cost every workgroup a device-scope fence).

struct Seg {
  double v;
  int f;  // a column starts inside the span
};
__device__ __forceinline__ Seg seg_op(Seg a, Seg b) { return Seg{b.f ? b.v : a.v + b.v, a.f | b.f}; }

// Item codes of a plan: RUN {k0, k1, p0, p1} with k0 >= 0; PIECE
// {-1 - slot, k, p0, p1} (one of several workgroups sharing a long column,
// summed into long_acc[slot]); WHOLE {ITEM_WHOLE, k, p0, p1} (a long column
// done by a single workgroup).
constexpr int ITEM_WHOLE = -2147483647 - 1;

// Graph view of one chain for the column pass.
struct ColView {
  const int *colptr, *crow, *rowptr;
  const void *cval;
  int n;
  int unit;  // moved(j) already holds M_j P'_jk: every link weight is 1
  int *bad;  // set when an item or a link index is out of range (may be null)
};

// LDS of the column pass over items of at most IC links and IK columns.
// Column starts as bits and column pointers as 16-bit offsets into the item.
template <int NT, int IC = CH, int IK = RUN_MAX_COLS>
struct ColLds {
  static_assert(IC <= 65535, "16-bit item offsets");
  double con[IC];              // contributions, then inclusive segmented sums
  unsigned int head[IC / 32];  // bit e: a column of the run starts at element e
  unsigned short cp[IK + 1];   // column pointers of the run, relative to p0, clamped into [0, ne]
  Seg wave[NT / 64];
  double red[4 * (NT / 64)];
};

// One plan item: adds c * sum_j moved(j) P'_jk + kept(k) + off into out[k]
// for the item's columns and folds the statistics of those values.
template <class T, int NT, int IC = CH, int IK = RUN_MAX_COLS, class Moved, class Kept>
__device__ __forceinline__ void column_item(const ColView &g, int4 item, Moved moved, Kept kept, double c,
                                            double off, double rr, T *__restrict__ out, double *long_acc,
                                            ColLds<NT, IC, IK> &L, double &l1, double &cs, double &sr,
                                            double &mx) {
  constexpr int NW = NT / 64;
  constexpr int U = IC / NT;                 // links per thread
  constexpr int KC = IK / NT;                // columns per thread
  static_assert(U >= 1 && KC >= 1 && U * NT == IC && KC * NT == IK, "item shape");
  static_assert(32 % U == 0 && IC % 32 == 0, "a thread's column-start bits lie in one word");
  const int *__restrict__ colptr = g.colptr;
  const int *__restrict__ crow = g.crow;
  const T *__restrict__ cval = (const T *)g.cval;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const bool unit = g.unit != 0;
  auto weight = [&](int p, int j) -> double {
    return unit ? 1.0 : (cval ? (double)cval[p] : inv_outdeg(g.rowptr, g.n, j));
  };
  // the item is the same for the whole workgroup: scalar registers
  item = make_int4(__builtin_amdgcn_readfirstlane(item.x), __builtin_amdgcn_readfirstlane(item.y),
                   __builtin_amdgcn_readfirstlane(item.z), __builtin_amdgcn_readfirstlane(item.w));
  if (item.x >= 0) {
    // RUN: every load below depends on the item alone
    const int k0 = item.x, k1 = item.y, p0 = item.z, p1 = item.w;
    const int ne = p1 - p0, ncol = k1 - k0;
    if (ne > IC || ne < 0 || ncol > IK || ncol < 0) {  // the plan never builds such an item
      if (g.bad) *g.bad = 1;
      return;
    }
    __syncthreads();
    int jj[U];
    double ww[U];
    // loads clamped into the item (no per-thread branch); past its end the
    // source is -1 and the weight 0
    const int elast = max(ne - 1, 0);
    const int *__restrict__ rows = (ne > 0) ? crow + p0 : colptr;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = u * NT + tid;
      const int j = rows[min(e, elast)];
      jj[u] = (e < ne) ? j : -1;
      ww[u] = 0.0;
      if (cval && !unit && ne > 0) {
        const double v = (double)cval[p0 + min(e, elast)];
        ww[u] = (e < ne) ? v : 0.0;
      }
    }
    double kv[KC];
#pragma unroll
    for (int m = 0; m < KC; ++m) {
      const int q = m * NT + tid;
      kv[m] = (q < ncol) ? kept(k0 + q) : 0.0;
    }
    for (int q = tid; q <= ncol; q += NT) L.cp[q] = (unsigned short)min(max(colptr[k0 + q] - p0, 0), ne);
    for (int q = tid; q < IC / 32; q += NT) L.head[q] = 0u;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = u * NT + tid;
      if (e < ne) {
        const double w = unit ? 1.0 : (cval ? ww[u] : inv_outdeg(g.rowptr, g.n, jj[u]));
        L.con[e] = moved(jj[u]) * w;
      }
    }
    __syncthreads();
    for (int q = tid; q < ncol; q += NT) {
      const int a = L.cp[q];
      if (a < L.cp[q + 1]) atomicOr(&L.head[a >> 5], 1u << (a & 31));  // a < ne <= IC
    }
    __syncthreads();
    // segmented inclusive scan: thread t owns elements [t*U, t*U+U)
    double loc[U];
    int first_head = U;
    Seg run{0.0, 0};
    const unsigned int hbits = L.head[(tid * U) >> 5] >> ((tid * U) & 31);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = tid * U + u;
      const double x = (e < ne) ? L.con[e] : 0.0;
      const int h = (e < ne) ? (int)((hbits >> u) & 1u) : 0;
      if (h && first_head == U) first_head = u;
      run = h ? Seg{x, 1} : Seg{run.v + x, run.f};
      loc[u] = run.v;
    }
    Seg inc = run;
    seg_scan_step<DPP_ROW_SHR1, 0xF>(inc.v, inc.f);
    seg_scan_step<DPP_ROW_SHR2, 0xF>(inc.v, inc.f);
    seg_scan_step<DPP_ROW_SHR4, 0xF>(inc.v, inc.f);
    seg_scan_step<DPP_ROW_SHR8, 0xF>(inc.v, inc.f);
    seg_scan_step<DPP_ROW_BCAST15, 0xA>(inc.v, inc.f);
    seg_scan_step<DPP_ROW_BCAST31, 0xC>(inc.v, inc.f);
    if (lane == 63) L.wave[wv] = inc;
    // exclusive value: the inclusive one of the lane before (lane 0 reads 0)
    const Seg ex{dpp_f64<DPP_WAVE_SHR1, 0xF>(inc.v), dpp_i32<DPP_WAVE_SHR1, 0xF>(inc.f)};
    __syncthreads();
    Seg wbase{0.0, 0};
    for (int q = 0; q < wv; ++q) wbase = seg_op(wbase, L.wave[q]);
    const Seg carry = seg_op(wbase, ex);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = tid * U + u;
      if (e < ne) L.con[e] = (u < first_head) ? carry.v + loc[u] : loc[u];
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < KC; ++m) {
      const int q = m * NT + tid;
      if (q < ncol) {
        const int a = L.cp[q], b = L.cp[q + 1];
        const double acc = (b > a) ? L.con[b - 1] : 0.0;
        const T x = (T)(kv[m] + c * acc + off);
        out[k0 + q] = x;
        fold_stats((double)x, rr, l1, cs, sr, mx);
      }
    }
  } else {
    // PIECE or WHOLE: a strided walk over [p0, p1) of one column
    const int k = item.y, pb = item.z, pe = item.w;
    double acc = 0.0;
    for (int p0 = pb; p0 < pe; p0 += IC) {
      int jj[U];
      double ww[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int p = p0 + u * NT + tid;
        jj[u] = (p < pe) ? crow[p] : -1;
        ww[u] = (p < pe) ? weight(p, jj[u]) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (jj[u] >= 0) acc += moved(jj[u]) * ww[u];
    }
    const Red4 t4 = block_sum4<NW>(Red4{acc, 0, 0, 0}, L.red);
    if (tid == 0) {
      if (item.x == ITEM_WHOLE) {
        const T x = (T)(kept(k) + c * t4.a + off);
        out[k] = x;
        fold_stats((double)x, rr, l1, cs, sr, mx);
      } else {
        atomic_add_f64(&long_acc[-1 - item.x], t4.a);
      }
    }
  }
}

// Wave-level column pass of one chain.  Every wave takes plan items on its
// own (no workgroup barrier inside the item loop): a RUN {k0, k1, p0, p1} of
// whole columns holding at most WL links and WCOLS columns, or a PIECE
// {-1 - slot, k, p0, p1} of at most WL links of a longer column, whose sum
// goes to long_acc[slot]: with FUSE the piece that completes the column's
// link count writes the column, otherwise a later pass does (long_finish).
//
// The loads of an item (its CSC sources, column pointers and, with STAGEK,
// the raw cash values its kept part needs) are issued coalesced into
// registers one item ahead, right after the current item's gathers, so they
// travel while the wave sums that item and the wait for the gathers does not
// include them; at the top of the next round they are parked in the wave's
// LDS.
//
// In a RUN, lane l owns the WU consecutive links [l*WU, l*WU + WU) of the
// item and gathers what their sources send.  Lane q marks the last link of
// column q in LDS, so each lane reads which of its links end a column (and
// which column) with WU/4 LDS loads, then walks its links without branches:
// a column that both starts and ends among them stores its sum at once; the
// sum of the leading part of its first column (which may have started in an
// earlier lane) waits for the carry, the sum of the trailing part goes into
// a segmented scan across the lanes, whose exclusive value is that carry.
// Then lane q writes column q of the item: x_k = kept(k) + c * sum_k + off
// (columns without in-links have sum 0).
__device__ __forceinline__ void wave_lds_fence() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_wave_barrier();
}

template <class T, class S, bool VAL, bool STAGEK, bool RP, bool FUSE, bool KH = false, int PW = NWAVE, class Keep>
__device__ __forceinline__ void wave_pull(const Dev &d, const S *__restrict__ src, const T *__restrict__ kraw,
                                          Keep keep, double off, T *__restrict__ out, Rec *r,
                                          unsigned int *s_kh = nullptr) {
  static_assert(!FUSE || STAGEK, "finishing long columns reads their raw values");
  const T *__restrict__ kraw_t = kraw;
  constexpr int KW = STAGEK ? (int)(sizeof(T) / 4) : 0;      // dwords per staged raw value
  constexpr int NCP = (WCOLS + 1 + 63) / 64;                 // column pointers per lane
  constexpr int NK = STAGEK ? (WCOLS * KW + 63) / 64 : 1;    // staged raw dwords per lane
  __shared__ int s_row[PW][WL];
  // stored link values of the item, parked like its sources
  // (with stored values a wave's column sums share its value buffer: the
  // values are read out of it before the first sum is written, and the next
  // item is parked only after the last sum is read)
  __shared__ __align__(16) T s_val[VAL ? PW : 1][VAL ? WL : 1];
  __shared__ int s_cp[PW][NCP * 64];
  __shared__ unsigned int s_kr[PW][NK * 64];
  __shared__ double s_sum[VAL ? 1 : PW][WCOLS + 64];
  static_assert(!VAL || WL * sizeof(T) >= (WCOLS + 64) * sizeof(double), "sums fit the value buffer");
  __shared__ double sh_red[4 * PW];
  // What the HOTK lowest-numbered sources send, staged once per workgroup
  // in the relabelled layout, where they are the states of largest
  // out-degree: their gathers (about a fifth of the links on R-MAT, half on
  // the Chung-Lu graphs) read LDS instead of L2.  In the caller's numbering
  // (always so under top-k) the lowest ids are no one in particular, and
  // nothing is staged.  FP32 send values only, as many as leave room for the
  // other LDS arrays of four workgroups of NWAVE waves per CU, or of one of
  // PULL_WIDE waves.
  static_assert(PW == NWAVE || PW == PULL_WIDE, "two workgroup widths");
  constexpr int HOTK = (sizeof(S) != 4 || KH) ? 1
                       : PW == NWAVE ? (VAL ? HOT_SRC_VAL : HOT_SRC)
                                     : (VAL ? HOT_WIDE_VAL : HOT_WIDE);
  __shared__ S s_hot[HOTK];
  const int hk = (sizeof(S) == 4 && !KH && d.perm) ? min(HOTK, d.n) : 0;
  for (int q = threadIdx.x; q < hk; q += PW * 64) s_hot[q] = src[q];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  int *row = s_row[wv];
  T *valw = s_val[VAL ? wv : 0];
  int *cp = s_cp[wv];
  unsigned int *kr = s_kr[wv];
  double *sum = VAL ? (double *)s_val[wv] : s_sum[wv];
  const int n = d.n, n_items = d.n_items;
  const double c = d.c, rr = d.r;
  const int *__restrict__ colptr = d.colptr;
  const int *__restrict__ crow = d.crow;
  const T *__restrict__ cval = (const T *)d.cval;
  const unsigned int *__restrict__ kw = (const unsigned int *)kraw;
  double l1 = 0.0, cs = 0.0, sr = 0.0, mx = 0.0;
  const int e0 = lane * WU;
  const int stride = (int)gridDim.x * PW;
  const int4 none = make_int4(-1, 0, 0, 0);

  // registers of the item fetched ahead
  int pr[WU] = {}, pc[NCP] = {};
  T pv[VAL ? WU : 1] = {};
  unsigned int pk[NK] = {};
  // The item is the same for the whole wave (scalar registers); every lane
  // loads at an index clamped into the item, so no load sits behind a
  // per-lane branch, and the lanes past the item's end take their fill
  // value only when the item is parked (a select at fetch time would wait
  // for the loads there).
  // Every fetch sends the same loads whatever the item (an empty item reads
  // the first column pointer, which every graph has), so the waits below
  // count exactly the loads sent after the ones they wait for.
  auto fetch = [&](int4 item) {
    // item-relative bases (uniform) keep the per-lane offsets 32-bit
    const int ne = item.w - item.z;
    const int *__restrict__ rows = (ne > 0) ? crow + item.z : colptr;
    const int elast = max(ne - 1, 0);
#pragma unroll
    for (int u = 0; u < WU; ++u) pr[u] = rows[(unsigned int)min(u * 64 + lane, elast)];
    if (VAL) {
      // the item's link values, coalesced like its sources (an empty item
      // reads the first column pointer's bytes, which every graph has)
      const T *__restrict__ vs = (ne > 0) ? cval + item.z : (const T *)colptr;
#pragma unroll
      for (int u = 0; u < WU; ++u) pv[u] = vs[(unsigned int)min(u * 64 + lane, elast)];
    }
    const bool run = item.x >= 0;  // a run: 1 <= ncol <= WCOLS
    const int k0 = run ? item.x : 0, ncol = run ? item.y - item.x : 0;
    const int *__restrict__ cps = colptr + k0;
#pragma unroll
    for (int q = 0; q < NCP; ++q) pc[q] = cps[(unsigned int)min(q * 64 + lane, ncol)];
    if (STAGEK) {
      const unsigned int *__restrict__ kws = kw + (size_t)k0 * KW;
      const int klast = max(ncol * KW - 1, 0);
#pragma unroll
      for (int q = 0; q < NK; ++q) pk[q] = kws[(unsigned int)min(q * 64 + lane, klast)];
    }
  };
  // The wave's items of 64 consecutive rounds are loaded at once, lane r
  // holding round base + r, and each round's item is read out of its lane
  // into scalar registers: no round waits for an item load (a per-round load
  // would have to be waited for together with the vector loads before it).
  const int it0 = (int)blockIdx.x * PW + wv;
  int4 ilist = none;
  int ibase = 0;
  auto load_items = [&](int round0) {
    const int i = it0 + (round0 + lane) * stride;
    ilist = (i < n_items) ? d.items[i] : none;
    ibase = round0;
    // wait here, on this rare path, not where the rounds read the list
    asm volatile("" : "+v"(ilist.x), "+v"(ilist.y), "+v"(ilist.z), "+v"(ilist.w));
  };
  auto item_of = [&](int round) -> int4 {
    if (round - ibase >= 64) load_items(round);
    const int r = round - ibase;
    return make_int4(__builtin_amdgcn_readlane(ilist.x, r), __builtin_amdgcn_readlane(ilist.y, r),
                     __builtin_amdgcn_readlane(ilist.z, r), __builtin_amdgcn_readlane(ilist.w, r));
  };

  // FUSE: the piece that brings its column's link count (long_cnt) to the
  // column's in-degree finishes the column.  Device-scope atomics on one
  // address are carried out at one place for the whole device; a piece takes
  // its count only after its add has returned, and the finishing piece swaps
  // the sum out only after its count has returned, so the swap comes after
  // every piece's add.  Each of the two round trips overlaps the wave's next
  // item: piece pa has its add in flight, piece pb its count.
  struct Piece {
    int slot, k, ne, deg;
    T raw;
    double before;
    int seen;
  } pa{}, pb{};
  bool has_a = false, has_b = false;
  double piece_sum = 0.0;
  auto advance = [&]() {
    if (has_b) {
      if (lane == 0 && pb.seen + pb.ne == pb.deg) {
        const double sum = __hip_atomic_exchange(&d.long_acc[pb.slot], 0.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&d.long_cnt[pb.slot], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const T y = (T)(keep(pb.raw, pb.k) + c * sum + off);
        out[pb.k] = y;
        fold_stats<RP>((double)y, rr, l1, cs, sr, mx);
        if (KH) atomicAdd(&s_kh[kh_bin(y)], 1u);
      }
      has_b = false;
    }
    if (has_a) {
      pb = pa;
      if (lane == 0) {
        asm volatile("" ::"v"(pa.before) : "memory");
        pb.seen = __hip_atomic_fetch_add(&d.long_cnt[pa.slot], pa.ne, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      has_a = false;
      has_b = true;
    }
  };

  int it = it0, round = 0;
  load_items(0);
  int4 cur = item_of(0);
  // an item the plan cannot have built is not followed, and reported
  int badl = 0;
  auto valid = [&](int4 item) {
    const int ne = item.w - item.z;
    bool ok = ne >= 0 && ne <= WL;
    ok = ok && (item.x < 0 || (item.y - item.x >= 1 && item.y - item.x <= WCOLS));
    badl |= ok ? 0 : 1;
    return ok;
  };
  if (it < n_items) fetch(valid(cur) ? cur : none);
  for (; it < n_items; it += stride, ++round) {
    // park the fetched item in LDS, then send the next one's loads
    const int4 item = valid(cur) ? cur : none;
    {
      const int p0 = item.z, ne = item.w - item.z, ncol = item.y - item.x;
      const bool run = item.x >= 0;
#pragma unroll
      for (int u = 0; u < WU; ++u) row[u * 64 + lane] = (u * 64 + lane < ne) ? pr[u] : -1;
      if (VAL) {
#pragma unroll
        for (int u = 0; u < WU; ++u) valw[u * 64 + lane] = pv[u];
      }
#pragma unroll
      for (int q = 0; q < NCP; ++q) cp[q * 64 + lane] = (run && q * 64 + lane <= ncol) ? pc[q] - p0 : 0;
      if (STAGEK) {
#pragma unroll
        for (int q = 0; q < NK; ++q) kr[q * 64 + lane] = (run && q * 64 + lane < ncol * KW) ? pk[q] : 0u;
      }
    }
    wave_lds_fence();
    const int ne = item.w - item.z;
    static_assert(WU % 4 == 0, "lanes read their links four at a time");
    int jj[WU];
#pragma unroll
    for (int h = 0; h < WU; h += 4) {
      const int4 a = *(const int4 *)&row[e0 + h];
      jj[h] = a.x; jj[h + 1] = a.y; jj[h + 2] = a.z; jj[h + 3] = a.w;
    }
    // The item's gathers are sent before the next item's loads: loads
    // complete in the order they were sent, so waiting for the gathers then
    // never waits for the next item's stream.
    S xr[WU];
    bool ok[WU];
#pragma unroll
    for (int u = 0; u < WU; ++u) {
      // jj is -1 past the item's end; a link outside [0, N) sends nothing
      // and is reported
      const unsigned int j = (unsigned int)jj[u];
      ok[u] = j < (unsigned int)n;
      badl |= (e0 + u < item.w - item.z && !ok[u]) ? 1 : 0;
      xr[u] = (j < (unsigned int)hk) ? s_hot[j] : src[ok[u] ? j : 0u];
    }
    // this lane's link values, parked with the item
    T wr[WU];
    if (VAL) {
#pragma unroll
      for (int u = 0; u < WU; ++u) wr[u] = valw[e0 + u];
    }
    asm volatile("" ::: "memory");
    // the next round's item (none past the end: its loads read element 0)
    const int4 nxt = item_of(round + 1);
    fetch(valid(nxt) ? nxt : none);
    S x[WU];
    double w[WU];
#pragma unroll
    for (int u = 0; u < WU; ++u) {
      asm volatile("" : "+v"(xr[u]));  // the wait for the gather stays here
      x[u] = ok[u] ? xr[u] : S(0);
      w[u] = 1.0;
      if (VAL) w[u] = (e0 + u < ne) ? (double)wr[u] : 1.0;
    }
    if (item.x >= 0) {
      const int k0 = item.x, ncol = item.y - item.x;
      // Mark the last link of every column that has one with the column's
      // index (row[] is free once jj holds this lane's sources; LDS
      // operations of one wave take effect in program order).
      static_assert(WCOLS <= 64, "one lane per column of a run");
#pragma unroll
      for (int h = 0; h < WU; h += 4) *(int4 *)&row[e0 + h] = make_int4(-1, -1, -1, -1);
      if (lane < ncol) {
        sum[lane] = 0.0;  // stays 0 for a column without in-links
        const int b0 = cp[lane], b1 = cp[lane + 1];
        if (b1 > b0) row[b1 - 1] = lane;
      }
      wave_lds_fence();
      int ec[WU];
#pragma unroll
      for (int h = 0; h < WU; h += 4) {
        const int4 a = *(const int4 *)&row[e0 + h];
        ec[h] = a.x; ec[h + 1] = a.y; ec[h + 2] = a.z; ec[h + 3] = a.w;
      }
      // Walk the lane's links: the sum up to its first column end is the
      // head of that column (f), later ends close columns that lie wholly in
      // the lane; links past ne send 0 and end no column.
      // Branch-free: a link that closes no column inside the lane stores to
      // the lane's own spare slot (sum[WCOLS + lane]).
      double acc = 0.0, head = 0.0;
      int ended = 0, f = 0;
#pragma unroll
      for (int u = 0; u < WU; ++u) {
        acc += (double)x[u] * w[u];
        const int q = ec[u];
        const bool e = q >= 0;
        sum[(e && ended) ? q : WCOLS + lane] = acc;
        const bool first = e && !ended;
        head = first ? acc : head;
        f = first ? q : f;
        ended |= (int)e;
        acc = e ? 0.0 : acc;
      }
      // inclusive segmented scan of the trailing sums (a lane with a column
      // end starts a segment); its exclusive value is the carry
      double iv = acc;
      int fl = ended;
      seg_scan_step<DPP_ROW_SHR1, 0xF>(iv, fl);
      seg_scan_step<DPP_ROW_SHR2, 0xF>(iv, fl);
      seg_scan_step<DPP_ROW_SHR4, 0xF>(iv, fl);
      seg_scan_step<DPP_ROW_SHR8, 0xF>(iv, fl);
      seg_scan_step<DPP_ROW_BCAST15, 0xA>(iv, fl);
      seg_scan_step<DPP_ROW_BCAST31, 0xC>(iv, fl);
      const double carry = dpp_f64<DPP_WAVE_SHR1, 0xF>(iv);
      if (ended) sum[f] = carry + head;
      wave_lds_fence();
      T *__restrict__ outs = out + k0;
      if (lane < ncol) {  // ncol <= WCOLS <= 64: one column per lane
        const int q = lane;
        const double kv = STAGEK ? keep(((const T *)kr)[q], k0 + q) : keep(T(0), k0 + q);
        const T y = (T)(kv + c * sum[q] + off);
        outs[(unsigned)q] = y;
        fold_stats<RP>((double)y, rr, l1, cs, sr, mx);
        if (KH) atomicAdd(&s_kh[kh_bin(y)], 1u);
      }
    } else if (ne > 0) {
      double acc = 0.0;
#pragma unroll
      for (int u = 0; u < WU; ++u) acc += (double)x[u] * w[u];
      acc = wave_sum(acc);
      if (!FUSE) {
        if (lane == 0) atomic_add_f64(&d.long_acc[-1 - item.x], acc);
      } else {
        piece_sum = acc;
      }
    }
    if (FUSE) {
      advance();
      if (item.x < 0 && ne > 0) {
        // the piece's add goes out now; its count follows one item later
        pa.slot = -1 - item.x;
        pa.k = item.y;
        pa.ne = ne;
        pa.deg = colptr[pa.k + 1] - colptr[pa.k];
        if (lane == 0) {
          pa.raw = kraw_t[pa.k];
          pa.before =
              __hip_atomic_fetch_add(&d.long_acc[pa.slot], piece_sum, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        has_a = true;
      }
    }
    wave_lds_fence();  // this item's LDS reads are done before the next park
    cur = nxt;
  }
  if (FUSE) {
    advance();
    advance();
  }
  if (badl) d.glob->bad = 1;
  fold_block_stats<PW>(r, l1, cs, sr, mx, sh_red);
}

// ----------------------------------------------------------------- complete

// PW waves per workgroup: NWAVE (four workgroups per CU) or PULL_WIDE (one
// workgroup per CU, whose pull stages the send values of four times as many
// sources in LDS).
template <class T, bool VAL, bool RP, bool TK, int PW = NWAVE>
__global__ __launch_bounds__(PW * 64, PW == NWAVE ? 4 : 1) void k_complete(Dev d, long long s, int init) {
  constexpr int NT = PW * 64;
  Glob *g = d.glob;
  if (g->status != 0) return;
  Rec *cur = &d.rec[s % 3];
  Rec *nxt = &d.rec[(s + 1) % 3];
  __shared__ Tot sh_tot;
  __shared__ double sh_red[4 * PW];
  // TK: the top-k histogram of C_{t+1}'s keys, counted as they are written
  __shared__ unsigned int s_kh[TK ? KH_BINS : 1];
  if (TK) {
    for (int b = threadIdx.x; b < KH_BINS; b += NT) s_kh[b] = 0u;
    __syncthreads();
  }
  const Tot tot = read_totals(cur, &sh_tot);
  const int n = d.n;
  const double off = tot.T / (double)n;  // uniform restart share of eq. (6)
  const int mode = cur->mode;
  const double r = d.r;

  if (mode == 0) {
    double l1 = 0.0, cs = 0.0, sr = 0.0, mx = 0.0;
    T *C = (T *)d.cash[cur->buf];
    double *D = d.delta;
    const int ntiles = (n + NT * VPT - 1) / (NT * VPT);
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
#pragma unroll
      for (int q = 0; q < VPT; ++q) {
        const int i = tile * NT * VPT + q * NT + threadIdx.x;
        if (i < n) {
          double x = (double)C[i] + off;
          if (D) {
            x += D[i];
            D[i] = 0.0;
          }
          const T y = (T)x;
          C[i] = y;
          fold_stats<RP>((double)y, r, l1, cs, sr, mx);
          if (TK) atomicAdd(&s_kh[kh_bin(y)], 1u);
        }
      }
    }
    fold_block_stats<PW>(nxt, l1, cs, sr, mx, sh_red);
  } else {
    const int sched = init ? SCHED_ALL : d.sched;
    const double theta = cur->theta;
    const double maxabs = tot.maxabs;
    const double tau = cur->topk_tau;
    const int tie_id = cur->topk_tie_id;
    const T *__restrict__ Cc = (const T *)d.cash[cur->buf];
    T *__restrict__ Cn = (T *)d.cash[cur->buf ^ 1];
    // the kept part C_t - M_t of node k from its cash v
    auto keep = [&](T v, int k) -> double {
      if (init) return -(double)v;  // step 0: C_0 - M_0 with C_0 = 0
      return is_green(v, k, sched, theta, maxabs, tau, tie_id, d.seed, s, d.green_in) ? 0.0 : (double)v;
    };
    // what the sources send was written by select (zero off the green set;
    // links outside [0, N) are ignored)
    wave_pull<T, T, VAL, true, RP, true, TK, PW>(d, (const T *)d.src, Cc, keep, off, Cn, nxt, s_kh);
  }
  if (TK) {
    __syncthreads();
    kh_flush(khist_of(d, s + 1), s_kh);
  }

  if (blockIdx.x == 0 && threadIdx.x == 0) {
    nxt->hsum = cur->hsum + tot.msum;
    nxt->hnorm = cur->hnorm + tot.dhnorm;
    nxt->edges_total = cur->edges_total + tot.gedges;
    nxt->green_total = cur->green_total + (init ? 0 : tot.green);
    nxt->buf = (mode == 0) ? cur->buf : (cur->buf ^ 1);
    g->t = s + 1;
    StepLog *lg = &d.log[s % LOG_STEPS];
    lg->s = s;
    lg->mode = mode;
    lg->green = tot.green;
    lg->gedges = tot.gedges;
    lg->nfront = (long long)(cur->fr_pack >> 32);
  }
}

// Completes the long columns once all their pieces have been added to
// long_acc: x_k = kept(k) + c * acc + off, then resets
// long_acc for the next pass and folds the statistics of the x_k.
// kept(k, q) may use what the caller loaded ahead for the column at q.
template <class T, class Kept>
__device__ __forceinline__ void long_finish(const Dev &d, Kept kept, double off, T *__restrict__ out, Rec *r) {
  __shared__ double sh_red[4 * NWAVE];
  double l1 = 0.0, cs = 0.0, sr = 0.0, mx = 0.0;
  for (int q = blockIdx.x * BLOCK + threadIdx.x; q < d.n_long; q += gridDim.x * BLOCK) {
    const int k = d.long_cols[q];
    const double acc = d.long_acc[q];
    d.long_acc[q] = 0.0;
    const T x = (T)(kept(k, q) + d.c * acc + off);
    out[k] = x;
    fold_stats((double)x, d.r, l1, cs, sr, mx);
  }
  fold_block_stats(r, l1, cs, sr, mx, sh_red);
}

template <class T, int HK>
__global__ __launch_bounds__(BLOCK) void k_refresh_long(Dev d, long long t, int out_buf) {
  auto kept = [&](int k, int) -> double { return -hist_at<HK>(d, k); };
  long_finish<T>(d, kept, d.glob->rpool / (double)d.n, (T *)d.cash[out_buf], &d.rec[t % 3]);
}

// -------------------------------------------------- top-k threshold search
//
// The k-th largest |C| of the snapshot C_t (tau) and the largest node id that
// still fits among the nodes with |C| = tau, so that green = |C| > tau or
// (|C| = tau and id <= tie_id) selects exactly k nodes ordered by |C|
// descending, then id ascending.  Non-negative floats order as their bits
// (the key).
//
//  1. The pass that writes C_t (k_complete of step t-1) also counts the top
//     KH_BITS bits of every key in a per-workgroup LDS histogram, added into
//     KH_STRIPES global copies (same-address atomics serialise).  After a
//     refresh or an import, k_topk_hist_full counts them instead.
//  2. k_topk_collect (one pass over C_t): every workgroup finds the bin B that
//     holds the k-th key from the histogram and copies the keys of bin B and
//     their ids into its own segment of the candidate list, in node order.
//     With FP32 keys it also counts their next KH_BITS bits.
//  3. FP32 keys: k_topk_narrow counts the last bits of the keys in one more
//     pass over the candidates, and every workgroup of the select pass fixes
//     tau and the id bound from those counts (below).  FP64 keys: k_topk_pass,
//     a few short radix passes over the candidates, KH_BITS bits of the key at
//     a time, then of the ids among the keys equal to tau.

__global__ void k_topk_hist_zero(Dev d, long long s) {
  unsigned int *kh = khist_of(d, s);
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < KH_STRIPES * KH_BINS; q += gridDim.x * blockDim.x)
    kh[q] = 0u;
}

template <class T>
__global__ __launch_bounds__(BLOCK) void k_topk_hist_full(Dev d, long long s) {
  if (d.glob->status != 0) return;
  __shared__ unsigned int s_kh[KH_BINS];
  for (int b = threadIdx.x; b < KH_BINS; b += BLOCK) s_kh[b] = 0u;
  __syncthreads();
  const T *C = (const T *)d.cash[d.rec[s % 3].buf];
  for (int base = blockIdx.x * BLOCK; base < d.n; base += gridDim.x * BLOCK) {
    const int i = base + threadIdx.x;
    wave_hist_add<KH_BITS>(s_kh, i < d.n ? (unsigned int)kh_bin(C[i]) : 0u, i < d.n);
  }
  __syncthreads();
  kh_flush(khist_of(d, s), s_kh);
}

// The digit of a histogram in taking order (keys: largest first; ids:
// smallest first) at which the running count reaches rem, and the count taken
// before it.  Every thread of a BLOCK-wide workgroup calls it and receives
// the result; `h` holds nb <= KH_BINS counts (LDS).
__device__ __forceinline__ void pick_digit(const unsigned int *h, int nb, bool ascending, long long rem, int *dig,
                                           long long *before, unsigned long long *sh_scan, int *sh_dig,
                                           long long *sh_before) {
  constexpr int PER = KH_BINS / BLOCK;
  unsigned int cnt[PER];
  unsigned long long mine = 0;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int q = threadIdx.x * PER + u;  // position in taking order
    const int b = ascending ? q : nb - 1 - q;
    cnt[u] = (q < nb) ? h[b] : 0u;
    mine += cnt[u];
  }
  unsigned long long total;
  unsigned long long run = block_excl_scan(mine, sh_scan, &total);
  if (threadIdx.x == 0) *sh_dig = -1;
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int q = threadIdx.x * PER + u;
    if (q < nb && run < (unsigned long long)rem && run + cnt[u] >= (unsigned long long)rem) {
      *sh_dig = ascending ? q : nb - 1 - q;
      *sh_before = (long long)run;
    }
    run += cnt[u];
  }
  __syncthreads();
  *dig = *sh_dig;
  *before = *sh_before;
  __syncthreads();
}

// Finds the bin B of the k-th key from the histogram the complete pass
// counted and appends every node of bin B (key, id) to the candidate list;
// leaves the radix state (prefix, rem) for the first pass over them.
template <class T>
__global__ __launch_bounds__(BLOCK) void k_topk_collect(Dev d, long long s) {
  Glob *g = d.glob;
  if (g->status != 0) return;
  constexpr int KB = sizeof(T) == 4 ? 31 : 63;  // key bits
  __shared__ unsigned int s_h[KH_BINS];
  __shared__ unsigned long long sh_scan[NWAVE];
  __shared__ int sh_dig;
  __shared__ long long sh_before;
  const unsigned int *kh = khist_of(d, s);
  const long long want = d.k < (long long)d.n ? d.k : (long long)d.n;
  // workgroup b owns the nodes [b S, (b + 1) S) and writes their candidates
  // to the same positions of the list (no shared counter), in node order;
  // tk_cnt[b] says how many.  The values of its first TK_PRE tiles are
  // loaded before the bin is known, so they travel with the histogram.
  const T *C = (const T *)d.cash[d.rec[s % 3].buf];
  const int S = tk_segment(d.n, gridDim.x);
  const int b0 = blockIdx.x * S, b1 = min(d.n, b0 + S);
  constexpr int TK_PRE = 4;
  T pre[TK_PRE][VPT];
#pragma unroll
  for (int r = 0; r < TK_PRE; ++r)
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
      // a load at an index clamped into [0, n) and a select, no branch
      const int i = b0 + r * TILE + u * BLOCK + threadIdx.x;
      const T x = C[(unsigned int)min(i, b1 - 1)];
      pre[r][u] = (i < b1) ? x : T(0);
    }
  kh_load(kh, s_h);
  // FP64 keys: the first pass counts into buffer 0.  FP32 keys: this pass
  // counts the next digit into the KH_STRIPES copies at tk_hist itself, which
  // the previous step's select pass (or the reset) left at zero, and clears
  // the low-digit counts that select pass read, for k_topk_narrow.
  constexpr bool NEXT = sizeof(T) == 4;
  if (!NEXT)
    for (int q = blockIdx.x * BLOCK + threadIdx.x; q < KH_BINS; q += gridDim.x * BLOCK) d.tk_hist[q] = 0u;
  else if (blockIdx.x == 0)
    for (int q = threadIdx.x; q < TK_LOW_BINS; q += BLOCK) d.tk_hist[KH_STRIPES * KH_BINS + q] = 0u;
  __syncthreads();
  int B;
  long long above;
  pick_digit(s_h, KH_BINS, false, want, &B, &above, sh_scan, &sh_dig, &sh_before);
  if (B < 0) {
    // the histogram does not describe C_t (it counts fewer than k keys)
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      g->bad = 1;
      g->tk_rem[0] = 0;
    }
    return;
  }
  if (NEXT) {
    for (int b = threadIdx.x; b < KH_BINS; b += BLOCK) s_h[b] = 0u;
    __syncthreads();
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    g->tk_pref[0] = (unsigned long long)B << (KB - KH_BITS);
    g->tk_rem[0] = want - above;  // keys of bin B still to take, >= 1
    g->tk_done = 0;
  }
  unsigned long long *ckey = d.tk_ckey + b0;
  int *cid = d.tk_cid + b0;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const unsigned long long below = (1ull << lane) - 1ull;
  // VPT nodes per thread between two barriers, listed in node order
  __shared__ int sh_wc[VPT][NWAVE];
  int filled = 0;
  // one tile of VPT nodes per thread (a uniform call: it holds barriers)
  auto tile = [&](int base, const T (&v)[VPT]) {
    bool hit[VPT];
    unsigned long long bal[VPT];
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
      const int i = base + u * BLOCK + threadIdx.x;
      hit[u] = i < b1 && kh_bin(v[u]) == B;
      bal[u] = __ballot(hit[u]);
      if (lane == 0) sh_wc[u][wv] = __popcll(bal[u]);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
      int off = filled, tot = 0;
      for (int w = 0; w < NWAVE; ++w) {
        off += (w < wv) ? sh_wc[u][w] : 0;
        tot += sh_wc[u][w];
      }
      const unsigned long long key = topk_key(v[u]);
      if (hit[u]) {
        const int slot = off + __popcll(bal[u] & below);
        ckey[slot] = key;
        cid[slot] = base + u * BLOCK + threadIdx.x;
      }
      // (bal is the same on every lane: the whole wave enters or none)
      if (NEXT && bal[u]) wave_hist_add<KH_BITS>(s_h, (unsigned int)(key >> TK_LOW_BITS) & (KH_BINS - 1u), hit[u]);
      filled += tot;
    }
    __syncthreads();
  };
#pragma unroll
  for (int r = 0; r < TK_PRE; ++r)
    if (b0 + r * TILE < b1) tile(b0 + r * TILE, pre[r]);
  for (int base = b0 + TK_PRE * TILE; base < b1; base += TILE) {
    T v[VPT];
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
      const int i = base + u * BLOCK + threadIdx.x;
      v[u] = (i < b1) ? C[i] : T(0);
    }
    tile(base, v);
  }
  if (threadIdx.x == 0) d.tk_cnt[blockIdx.x] = filled;
  if (NEXT) kh_flush(d.tk_hist, s_h);  // stripe blockIdx mod KH_STRIPES
}

// FP32 keys (31 bits: the histogram's KH_BITS, a middle digit of KH_BITS, a
// low digit of TK_LOW_BITS).  k_topk_narrow: every workgroup picks the middle
// digit from the counts k_topk_collect made, then compacts the candidates of
// its own segment that match the key so far (in place and in node order) and
// counts their low digit, into the global low-digit histogram and into its
// segment's row of tk_seg.  topk_fix_tau, in every workgroup of the select
// pass, picks the low digit, which completes tau; if only some of the keys
// equal to tau are taken, the segment rows say which segment holds the last
// one taken, and a scan of that segment's compacted list in node order finds
// its id.  (A last-workgroup ticket in place of that redundant work would need
// a device-scope fence in every workgroup of k_topk_narrow, which writes back
// the XCD's whole L2.)
__device__ __forceinline__ unsigned int *tk_low_hist(const Dev &d) { return d.tk_hist + KH_STRIPES * KH_BINS; }

__global__ __launch_bounds__(BLOCK) void k_topk_narrow(Dev d, long long s) {
  Glob *g = d.glob;
  if (g->status != 0) return;
  __shared__ unsigned int s_h[KH_BINS];
  __shared__ unsigned long long sh_scan[NWAVE];
  __shared__ int sh_dig;
  __shared__ long long sh_before;
  __shared__ int sh_wc[NWAVE];
  const unsigned long long pref0 = g->tk_pref[0];
  const long long rem0 = g->tk_rem[0];
  if (rem0 <= 0) return;  // k_topk_collect found no bin (reported there)
  // the segment's first BLOCK entries are loaded before the digit is known,
  // so they travel with the histogram (at an index clamped into the list:
  // the last segments may start past its end; only entries below cnt are
  // used)
  const int S = tk_segment(d.n, gridDim.x);
  const int cnt = d.tk_cnt[blockIdx.x];
  unsigned long long *ckey = d.tk_ckey + (size_t)blockIdx.x * S;
  int *cid = d.tk_cid + (size_t)blockIdx.x * S;
  const size_t q0 = min((size_t)blockIdx.x * S + threadIdx.x, (size_t)d.n - 1);
  const unsigned long long key0 = d.tk_ckey[q0];
  const int id0 = d.tk_cid[q0];
  kh_load(d.tk_hist, s_h);
  __syncthreads();
  int A;
  long long beforeA;
  pick_digit(s_h, KH_BINS, false, rem0, &A, &beforeA, sh_scan, &sh_dig, &sh_before);
  if (A < 0) {
    // fewer candidates than the histogram of C_t promised
    if (threadIdx.x == 0) g->bad = 1;
    return;
  }
  const long long remA = rem0 - beforeA;
  const unsigned long long prefA = pref0 | ((unsigned long long)A << TK_LOW_BITS);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    g->tk_pref[1] = prefA;
    g->tk_rem[1] = remA;
  }
  for (int b = threadIdx.x; b < TK_LOW_BINS; b += BLOCK) s_h[b] = 0u;
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int filled = 0;
  // Every thread holds its entry before the barrier below, and an entry moves
  // only to a position at or before its own, so no entry is overwritten
  // before it is read.
  for (int c0 = 0; c0 < cnt; c0 += BLOCK) {
    const int q = c0 + threadIdx.x;
    const bool in = q < cnt;
    const unsigned long long key = in ? (c0 == 0 ? key0 : ckey[q]) : 0ull;
    const int id = in ? (c0 == 0 ? id0 : cid[q]) : 0;
    const bool hit = in && (key >> TK_LOW_BITS) == (prefA >> TK_LOW_BITS);
    const unsigned long long bal = __ballot(hit);
    if (lane == 0) sh_wc[wv] = __popcll(bal);
    __syncthreads();
    int off = filled, tot = 0;
    for (int w = 0; w < NWAVE; ++w) {
      off += (w < wv) ? sh_wc[w] : 0;
      tot += sh_wc[w];
    }
    if (hit) {
      const int slot = off + __popcll(bal & ((1ull << lane) - 1ull));
      ckey[slot] = key;
      cid[slot] = id;
    }
    wave_hist_add<TK_LOW_BITS>(s_h, (unsigned int)key & (TK_LOW_BINS - 1u), hit);
    filled += tot;
    __syncthreads();
  }
  unsigned int *hlow = tk_low_hist(d);
  unsigned int *seg = d.tk_seg + (size_t)blockIdx.x * TK_LOW_BINS;
  for (int b = threadIdx.x; b < TK_LOW_BINS; b += BLOCK) {
    seg[b] = s_h[b];
    if (s_h[b]) atomicAdd(&hlow[b], s_h[b]);
  }
  if (threadIdx.x == 0) d.tk_cnt[blockIdx.x] = filled;
}

static_assert(TK_GRID <= BLOCK, "topk_fix_tau reads one segment row per thread");
// FP32 keys, after k_topk_narrow: picks the low digit from the low-digit
// histogram, which completes tau, and the id bound among the keys equal to
// tau (segment rows, then a scan of the segment's compacted list in node
// order).  Every thread of the BLOCK-wide workgroup calls it and receives
// the result; false when the lists do not hold what the histograms counted.
__device__ __forceinline__ bool topk_fix_tau(const Dev &d, int G, TkFix &L, double *tau_out, int *tie_out) {
  const Glob *g = d.glob;
  const unsigned long long prefA = g->tk_pref[1];
  const long long remA = g->tk_rem[1];
  const unsigned int *hlow = tk_low_hist(d);
  for (int b = threadIdx.x; b < TK_LOW_BINS; b += BLOCK) L.h[b] = hlow[b];
  __syncthreads();
  int Bl;
  long long beforeB;
  pick_digit(L.h, TK_LOW_BINS, false, remA, &Bl, &beforeB, L.scan, &L.dig, &L.before);
  if (Bl < 0) return false;
  const unsigned long long tau = prefA | (unsigned long long)Bl;
  const long long remB = remA - beforeB;  // keys equal to tau still to take, >= 1
  int tie = 0x7fffffff;                    // every key equal to tau is taken
  if (remB < (long long)L.h[Bl]) {
    // the segment that holds the remB-th key equal to tau, in node order
    const unsigned long long mine =
        (int)threadIdx.x < G ? (unsigned long long)d.tk_seg[(size_t)threadIdx.x * TK_LOW_BINS + Bl] : 0ull;
    unsigned long long total;
    const unsigned long long run = block_excl_scan(mine, L.scan, &total);
    if (threadIdx.x == 0) L.seg = -1;
    __syncthreads();
    if ((int)threadIdx.x < G && run < (unsigned long long)remB && run + mine >= (unsigned long long)remB) {
      L.seg = threadIdx.x;
      L.r = remB - (long long)run;
    }
    __syncthreads();
    const int sb = L.seg;
    if (sb < 0) return false;
    // thread t scans the strip [t L, (t + 1) L) of the segment's list
    const long long r = L.r;
    const int S = tk_segment(d.n, G);
    const int m = d.tk_cnt[sb];
    const unsigned long long *kk = d.tk_ckey + (size_t)sb * S;
    const int *ii = d.tk_cid + (size_t)sb * S;
    const int strip = (m + BLOCK - 1) / BLOCK;
    const int q0 = min(m, (int)threadIdx.x * strip), q1 = min(m, q0 + strip);
    unsigned long long own = 0;
    for (int q = q0; q < q1; ++q) own += (kk[q] == tau) ? 1ull : 0ull;
    unsigned long long tot2;
    const unsigned long long before = block_excl_scan(own, L.scan, &tot2);
    if (threadIdx.x == 0) L.id = -1;
    __syncthreads();
    if (before < (unsigned long long)r && before + own >= (unsigned long long)r) {
      long long left = r - (long long)before;
      for (int q = q0; q < q1; ++q)
        if (kk[q] == tau && --left == 0) {
          L.id = ii[q];
          break;
        }
    }
    __syncthreads();
    tie = L.id;
    if (tie < 0) return false;
  }
  *tau_out = (double)__uint_as_float((unsigned int)tau);
  *tie_out = tie;
  return true;
}

// One digit of the radix select over the candidates: the digits of the key
// below bin B from the top (largest first), then the digits of the node ids
// among the keys equal to tau (smallest first).  Pass p first picks digit
// p - 1 from the histogram pass p - 1 counted (every workgroup the same way),
// then counts digit p among the candidates that match the digits fixed so
// far.  `prev` / `cur`: {is_id, lo, width} of those digits (cur.width = 0:
// the last pass, which only picks and writes tau and the id bound).
struct TkDigit {
  int is_id, lo, width;
};

template <class T>
__global__ __launch_bounds__(BLOCK) void k_topk_pass(Dev d, long long s, int p, TkDigit prev, TkDigit cur) {
  Glob *g = d.glob;
  if (g->status != 0) return;
  if (g->tk_done) return;  // tau and the id bound are written already
  __shared__ unsigned int s_h[KH_BINS];
  __shared__ unsigned long long sh_scan[NWAVE];
  __shared__ int sh_dig;
  __shared__ long long sh_before;
  __shared__ int s_pre[SEL_GRID + 1];
  unsigned long long pref = g->tk_pref[p & 1];
  long long rem = g->tk_rem[p & 1];
  unsigned long long tau = g->tk_tau;
  if (p == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
    g->tk_pref[1] = pref;  // the state pass 1 starts from, before its pick
    g->tk_rem[1] = rem;
  }
  if (p > 0) {
    const unsigned int *hp = d.tk_hist + (size_t)((p - 1) % 3) * KH_BINS;
    for (int b = threadIdx.x; b < KH_BINS; b += BLOCK) s_h[b] = hp[b];
    __syncthreads();
    int dig;
    long long before;
    pick_digit(s_h, 1 << prev.width, prev.is_id != 0, rem, &dig, &before, sh_scan, &sh_dig, &sh_before);
    pref |= (unsigned long long)dig << prev.lo;
    rem -= before;
    if (!prev.is_id && cur.is_id) {
      // the key is complete: tau; the ids come next, unless every key equal
      // to tau is taken (then no id bound is needed)
      tau = pref;
      pref = 0ull;
      if ((long long)s_h[dig] == rem) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
          Rec *r = &d.rec[s % 3];
          r->topk_tau = sizeof(T) == 4 ? (double)__uint_as_float((unsigned int)tau)
                                       : __longlong_as_double((long long)tau);
          r->topk_tie_id = 0x7fffffff;
          g->tk_done = 1;
        }
        return;
      }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      g->tk_pref[(p + 1) & 1] = pref;
      g->tk_rem[(p + 1) & 1] = rem;
      g->tk_tau = tau;
    }
  }
  if (cur.width == 0) {
    // the last pass: pref is the id bound among the ties of tau
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      Rec *r = &d.rec[s % 3];
      r->topk_tau = sizeof(T) == 4 ? (double)__uint_as_float((unsigned int)tau) : __longlong_as_double((long long)tau);
      r->topk_tie_id = (int)pref;
    }
    return;
  }
  // the buffer pass p + 1 counts into (pass p - 2's, read by pass p - 1)
  unsigned int *hz = d.tk_hist + (size_t)((p + 1) % 3) * KH_BINS;
  for (int q = blockIdx.x * BLOCK + threadIdx.x; q < KH_BINS; q += gridDim.x * BLOCK) hz[q] = 0u;
  for (int b = threadIdx.x; b < KH_BINS; b += BLOCK) s_h[b] = 0u;
  __syncthreads();
  const int hi = cur.lo + cur.width;
  const unsigned long long dmask = (1ull << cur.width) - 1ull;
  // the candidates sit in segments of S positions, tk_cnt[b] of them filled:
  // candidate number q is in the segment whose prefix count covers it
  const int S = tk_segment(d.n, d.tk_grid);
  const int G = d.tk_grid;
  for (int b = threadIdx.x; b < G; b += BLOCK) s_pre[b + 1] = d.tk_cnt[b];
  __syncthreads();
  if (threadIdx.x == 0) {
    s_pre[0] = 0;
    for (int b = 1; b <= G; ++b) s_pre[b] += s_pre[b - 1];
  }
  __syncthreads();
  const int m = s_pre[G];
  for (int base = blockIdx.x * BLOCK; base < m; base += gridDim.x * BLOCK) {
    const int q = base + threadIdx.x;
    bool take = q < m;
    unsigned long long x = 0ull;
    if (take) {
      int lo = 0, up = G;  // s_pre[lo] <= q < s_pre[up]
      while (up - lo > 1) {
        const int mid = (lo + up) >> 1;
        if (s_pre[mid] <= q) lo = mid;
        else up = mid;
      }
      const int e = lo * S + (q - s_pre[lo]);
      const unsigned long long key = d.tk_ckey[e];
      x = cur.is_id ? (unsigned long long)(unsigned int)d.tk_cid[e] : key;
      take = (!cur.is_id || key == tau) && (x >> hi) == (pref >> hi);
    }
    wave_hist_add<KH_BITS>(s_h, (unsigned int)((x >> cur.lo) & dmask), take);
  }
  __syncthreads();
  unsigned int *hc = d.tk_hist + (size_t)(p % 3) * KH_BINS;
  for (int b = threadIdx.x; b < KH_BINS; b += BLOCK)
    if (s_h[b]) atomicAdd(&hc[b], s_h[b]);
}

// ------------------------------------------------------------------ refresh
//
// Rebuilds the cash of state t from the history alone.  With C_0 = 0 the
// balance identity of Sec. 2.2 (eq. (7)) reads H_t + C_t = H_t P, so
// C_t = H_t P - H_t; it is evaluated in FP64 along the CSC columns and rounded
// once to the cash type.  This removes the rounding that FP32 routing leaves
// in C (whose exact sum is zero) without changing the method's trajectory.

__global__ void k_refresh_prep(Dev d, long long t) {
  if (blockIdx.x != 0) return;
  Rec *cur = &d.rec[t % 3];
  if (threadIdx.x < NSTRIPE) {
    Acc &a = cur->acc[threadIdx.x];
    a.l1 = 0.0;
    a.csum = 0.0;
    a.sumr = 0.0;
    a.maxabs_bits = 0ull;
  }
  if (threadIdx.x == 0) {
    d.glob->rpool = 0.0;
    d.glob->ticket = 0u;
  }
}

template <int HK>
__global__ __launch_bounds__(BLOCK) void k_refresh_pool(Dev d) {
  const int n = d.n;
  const double c = d.c;
  double acc = 0.0;
  __shared__ double sh_red[4 * NWAVE];
  for (int j = blockIdx.x * BLOCK + threadIdx.x; j < n; j += gridDim.x * BLOCK) {
    const int dg = d.rowptr[j + 1] - d.rowptr[j];
    const double h = hist_at<HK>(d, j);
    acc += h * (dg == 0 ? 1.0 : 1.0 - c);
    // H_j P'_jk per link j -> k (H_j itself with stored link values)
    d.rsrc[j] = d.cval ? h : (dg > 0 ? h / (double)dg : 0.0);
  }
  const Red4 r = block_sum4(Red4{acc, 0, 0, 0}, sh_red);
  if (threadIdx.x == 0 && r.a != 0.0) atomic_add_f64(&d.glob->rpool, r.a);
}

template <class T, int HK, bool VAL, bool RP>
__global__ __launch_bounds__(BLOCK, 4) void k_refresh(Dev d, long long t, int out_buf) {
  Rec *cur = &d.rec[t % 3];
  const int n = d.n;
  const double off = d.glob->rpool / (double)n;
  auto keep = [&](T, int k) -> double { return -hist_at<HK>(d, k); };
  wave_pull<T, double, VAL, false, RP, false>(d, d.rsrc, (const T *)nullptr, keep, off, (T *)d.cash[out_buf], cur);
}

// Clears an FP64 array (the push accumulators after the refresh used them).
__global__ __launch_bounds__(BLOCK) void k_zero_f64(double *p, int n) {
  for (int i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) p[i] = 0.0;
}

__global__ void k_refresh_done(Dev d, long long t, int out_buf) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  d.rec[t % 3].buf = out_buf;
  d.glob->status = d.glob->bad ? ST_BAD_GRAPH : 0;
}

// ------------------------------------------------------------ init / misc

template <class T, int HK>
__global__ __launch_bounds__(BLOCK) void k_reset(Dev d) {
  const int n = d.n;
  const T m0 = (T)(1.0 / (double)n);
  T *C = (T *)d.cash[0];
  for (int i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) {
    if (d.delta) d.delta[i] = 0.0;
    C[i] = m0;  // holds M_0 = (1/N) 1 until step 0 moves it
    if (HK == 0) {
      ((double *)d.hist)[i] = 0.0;
    } else {
      ((float *)d.hist)[i] = 0.0f;
      d.hist_lo[i] = 0.0f;
    }
  }
  if (blockIdx.x < 3) {
    Rec *r = &d.rec[blockIdx.x];
    clear_stripes(r);
    if (threadIdx.x == 0) {
      r->hsum = 0.0;
      r->hnorm = 0.0;
      r->edges_total = 0;
      r->green_total = 0;
      r->buf = 0;
      r->mode = 0;
      r->theta = 0.0;
      r->fr_pack = 0ull;
      r->ticket = 0u;
      r->topk_tau = 0.0;
      r->topk_tie_id = -1;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    d.glob->status = 0;
    d.glob->bad = 0;
    d.glob->tk_tau = 0ull;
    d.glob->t = 0;
    d.glob->ticket = 0u;
    d.glob->rpool = 0.0;
  }
  if (d.tk_hist)
    for (int q = blockIdx.x * BLOCK + threadIdx.x; q < TK_HIST_WORDS; q += gridDim.x * BLOCK) d.tk_hist[q] = 0u;
  for (int q = blockIdx.x * BLOCK + threadIdx.x; q < d.n_long; q += gridDim.x * BLOCK) {
    d.long_acc[q] = 0.0;
    if (d.long_cnt) d.long_cnt[q] = 0;
  }
  for (int q = blockIdx.x * BLOCK + threadIdx.x; q < LOG_STEPS; q += gridDim.x * BLOCK) {
    d.log[q].s = -1;
    d.log[q].gedges = 0;
  }
}

__global__ void k_set_status(Glob *g, int st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) g->status = st;
}

template <int HK>
__global__ __launch_bounds__(BLOCK) void k_normalize(Dev d, double *pi) {
  const long long t = d.glob->t;
  const double hs = d.rec[t % 3].hsum;
  const int n = d.n;
  for (int i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) {
    pi[d.perm ? d.perm[i] : i] = hist_at<HK>(d, i) / hs;  // pi_hat_t = H_t / (H_t 1), eq. (2)
  }
}

template <class T, int HK>
__global__ __launch_bounds__(BLOCK) void k_export(Dev d, double *Cout, double *Hout) {
  const long long t = d.glob->t;
  const T *C = (const T *)d.cash[d.rec[t % 3].buf];
  const int n = d.n;
  for (int i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) {
    const int o = d.perm ? d.perm[i] : i;
    if (Cout) Cout[o] = (double)C[i];
    if (Hout) Hout[o] = hist_at<HK>(d, i);
  }
}

// Green mask of the last step in the caller's numbering.
__global__ __launch_bounds__(BLOCK) void k_export_mask(Dev d, unsigned char *out) {
  for (int i = blockIdx.x * BLOCK + threadIdx.x; i < d.n; i += gridDim.x * BLOCK)
    out[d.perm ? d.perm[i] : i] = d.green_mask[i];
}

// Relabelled copy of one side of the graph (CSR or CSC): new row i is old row
// new2old[i], its ids mapped through old2new (ids outside [0, n) are kept, so
// the kernels still ignore them).  One thread per link of the new layout; the
// new row of link p is found by a binary search of the new row pointers, so a
// hub row is spread over many threads.
template <class V>
__global__ __launch_bounds__(BLOCK) void k_relabel_side(int n, const int *ptr, const int *idx, const V *val,
                                                        const int *new2old, const int *old2new, const int *nptr,
                                                        int *nidx, V *nval) {
  const int m = nptr[n];
  for (int p = blockIdx.x * BLOCK + threadIdx.x; p < m; p += gridDim.x * BLOCK) {
    int lo = 0, hi = n;  // nptr[lo] <= p < nptr[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (nptr[mid] <= p) lo = mid;
      else hi = mid;
    }
    const int src = ptr[new2old[lo]] + (p - nptr[lo]);
    const int j = idx[src];
    nidx[p] = ((unsigned)j < (unsigned)n) ? old2new[j] : j;
    if (val) nval[p] = val[src];
  }
}

// Imports (C, H) at index t and refolds the statistics of C_t into record t.
template <class T, int HK>
__global__ __launch_bounds__(BLOCK) void k_import(Dev d, const double *Cin, const double *Hin, long long t,
                                                   int buf) {
  Rec *cur = &d.rec[t % 3];
  T *C = (T *)d.cash[buf];
  const int n = d.n;
  const double r = d.r;
  double l1 = 0, cs = 0, sr = 0, mx = 0, hs = 0, hn = 0;
  __shared__ double sh_red[4 * NWAVE];
  for (int i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) {
    if (d.delta) d.delta[i] = 0.0;
    const int o = d.perm ? d.perm[i] : i;
    const T x = (T)Cin[o];
    C[i] = x;
    fold_stats((double)x, r, l1, cs, sr, mx);
    const double h = Hin[o];
    if (HK == 0) {
      ((double *)d.hist)[i] = h;
      hs += h;
      hn += fabs(h);
    } else {
      const float hi = (float)h;
      const float lo = (float)(h - (double)hi);
      ((float *)d.hist)[i] = hi;
      d.hist_lo[i] = lo;
      hs += (double)hi + (double)lo;
      hn += fabs((double)hi + (double)lo);
    }
  }
  const Red4 b = block_sum4(Red4{hs, hn, 0, 0}, sh_red);
  if (threadIdx.x == 0) {
    Acc *a = my_stripe(cur);
    atomic_add_f64(&a->hsum_import, b.a);
    atomic_add_f64(&a->hnorm_import, b.b);
  }
  fold_block_stats(cur, l1, cs, sr, mx, sh_red);
}

__global__ void k_prepare_import(Dev d, long long t, int buf) {
  if (blockIdx.x >= 3) return;
  Rec *r = &d.rec[blockIdx.x];
  clear_stripes(r);
  if (threadIdx.x == 0) {
    r->hsum = 0.0;
    r->hnorm = 0.0;
    r->edges_total = 0;
    r->green_total = 0;
    r->fr_pack = 0ull;
    r->ticket = 0u;
    r->mode = 0;
    r->theta = 0.0;
    r->topk_tau = 0.0;
    r->topk_tie_id = -1;
    r->buf = buf;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    d.log[(t + LOG_STEPS - 1) % LOG_STEPS].gedges = d.nnz;  // the AUTO router sees a dense previous step
    d.glob->status = 0;
    d.glob->bad = 0;
    d.glob->t = t;
  }
}

__global__ void k_finish_import(Dev d, long long t, double h_sum) {
  __shared__ Tot sh_tot;
  Rec *cur = &d.rec[t % 3];
  const Tot tot = read_totals(cur, &sh_tot);
  if (threadIdx.x == 0) {
    cur->hsum = isnan(h_sum) ? tot.hsum_import : h_sum;
    cur->hnorm = tot.hnorm_import;
  }
}

// ------------------------------------------------------- explicit instances

template __global__ void k_select<float, 0>(Dev, long long, double, long long, int);
template __global__ void k_select<float, 1>(Dev, long long, double, long long, int);
template __global__ void k_select<double, 0>(Dev, long long, double, long long, int);
template __global__ void k_push<float>(Dev, long long);
template __global__ void k_push<double>(Dev, long long);
template __global__ void k_complete<float, false, false, false>(Dev, long long, int);
template __global__ void k_complete<float, false, false, true>(Dev, long long, int);
template __global__ void k_complete<float, false, true, false>(Dev, long long, int);
template __global__ void k_complete<float, false, true, true>(Dev, long long, int);
template __global__ void k_complete<float, true, false, false>(Dev, long long, int);
template __global__ void k_complete<float, true, false, true>(Dev, long long, int);
template __global__ void k_complete<float, true, true, false>(Dev, long long, int);
template __global__ void k_complete<float, true, true, true>(Dev, long long, int);
template __global__ void k_complete<float, false, false, false, PULL_WIDE>(Dev, long long, int);
template __global__ void k_complete<float, false, false, true, PULL_WIDE>(Dev, long long, int);
template __global__ void k_complete<float, false, true, false, PULL_WIDE>(Dev, long long, int);
template __global__ void k_complete<float, false, true, true, PULL_WIDE>(Dev, long long, int);
template __global__ void k_complete<float, true, false, false, PULL_WIDE>(Dev, long long, int);
template __global__ void k_complete<float, true, false, true, PULL_WIDE>(Dev, long long, int);
template __global__ void k_complete<float, true, true, false, PULL_WIDE>(Dev, long long, int);
template __global__ void k_complete<float, true, true, true, PULL_WIDE>(Dev, long long, int);
template __global__ void k_complete<double, false, false, false>(Dev, long long, int);
template __global__ void k_complete<double, false, false, true>(Dev, long long, int);
template __global__ void k_complete<double, false, true, false>(Dev, long long, int);
template __global__ void k_complete<double, false, true, true>(Dev, long long, int);
template __global__ void k_complete<double, true, false, false>(Dev, long long, int);
template __global__ void k_complete<double, true, false, true>(Dev, long long, int);
template __global__ void k_complete<double, true, true, false>(Dev, long long, int);
template __global__ void k_complete<double, true, true, true>(Dev, long long, int);
template __global__ void k_refresh_long<float, 0>(Dev, long long, int);
template __global__ void k_refresh_long<float, 1>(Dev, long long, int);
template __global__ void k_refresh_long<double, 0>(Dev, long long, int);
template __global__ void k_topk_hist_full<float>(Dev, long long);
template __global__ void k_topk_hist_full<double>(Dev, long long);
template __global__ void k_topk_collect<float>(Dev, long long);
template __global__ void k_topk_collect<double>(Dev, long long);
template __global__ void k_topk_pass<double>(Dev, long long, int, TkDigit, TkDigit);
template __global__ void k_refresh_pool<0>(Dev);
template __global__ void k_refresh_pool<1>(Dev);
template __global__ void k_refresh<float, 0, false, false>(Dev, long long, int);
template __global__ void k_refresh<float, 0, false, true>(Dev, long long, int);
template __global__ void k_refresh<float, 0, true, false>(Dev, long long, int);
template __global__ void k_refresh<float, 0, true, true>(Dev, long long, int);
template __global__ void k_refresh<float, 1, false, false>(Dev, long long, int);
template __global__ void k_refresh<float, 1, false, true>(Dev, long long, int);
template __global__ void k_refresh<float, 1, true, false>(Dev, long long, int);
template __global__ void k_refresh<float, 1, true, true>(Dev, long long, int);
template __global__ void k_refresh<double, 0, false, false>(Dev, long long, int);
template __global__ void k_refresh<double, 0, false, true>(Dev, long long, int);
template __global__ void k_refresh<double, 0, true, false>(Dev, long long, int);
template __global__ void k_refresh<double, 0, true, true>(Dev, long long, int);
template __global__ void k_reset<float, 0>(Dev);
template __global__ void k_reset<float, 1>(Dev);
template __global__ void k_reset<double, 0>(Dev);
template __global__ void k_normalize<0>(Dev, double *);
template __global__ void k_normalize<1>(Dev, double *);
template __global__ void k_export<float, 0>(Dev, double *, double *);
template __global__ void k_export<float, 1>(Dev, double *, double *);
template __global__ void k_export<double, 0>(Dev, double *, double *);
template __global__ void k_import<float, 0>(Dev, const double *, const double *, long long, int);
template __global__ void k_import<float, 1>(Dev, const double *, const double *, long long, int);
template __global__ void k_import<double, 0>(Dev, const double *, const double *, long long, int);
template __global__ void k_relabel_side<float>(int, const int *, const int *, const float *, const int *,
                                               const int *, const int *, int *, float *);
template __global__ void k_relabel_side<double>(int, const int *, const int *, const double *, const int *,
                                                const int *, const int *, int *, double *);

}  // namespace rlgl
