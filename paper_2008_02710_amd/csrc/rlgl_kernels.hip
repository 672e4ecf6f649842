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
//                the other cash buffer.  Both fold ||C_{t+1}||_1, sum C,
//                sum |C|^r and max |C| into the record of step t+1.
//
// All reductions are FP64.  Per-step scalars live in a ring of three device
// records indexed by t mod 3, so the host never has to touch them between
// steps: the kernels of step t read record t, accumulate into record t (select)
// or t+1 (complete), and select clears record t+1 before anyone uses it.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rlgl_device.h"

namespace rlgl {

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ double wave_sum(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}
__device__ __forceinline__ double wave_max(double x) {
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
  return x;
}
__device__ __forceinline__ long long wave_sum_ll(long long x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Block-wide sums of four doubles; every thread receives the result.
struct Red4 {
  double a, b, c, d;
};
__device__ __forceinline__ Red4 block_sum4(Red4 v, double *sh /* 4*NWAVE */) {
  v.a = wave_sum(v.a);
  v.b = wave_sum(v.b);
  v.c = wave_sum(v.c);
  v.d = wave_sum(v.d);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) {
    sh[w] = v.a;
    sh[NWAVE + w] = v.b;
    sh[2 * NWAVE + w] = v.c;
    sh[3 * NWAVE + w] = v.d;
  }
  __syncthreads();
  Red4 r{0, 0, 0, 0};
#pragma unroll
  for (int i = 0; i < NWAVE; ++i) {
    r.a += sh[i];
    r.b += sh[NWAVE + i];
    r.c += sh[2 * NWAVE + i];
    r.d += sh[3 * NWAVE + i];
  }
  __syncthreads();
  return r;
}
__device__ __forceinline__ double block_max(double v, double *sh) {
  v = wave_max(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) sh[w] = v;
  __syncthreads();
  double r = sh[0];
#pragma unroll
  for (int i = 1; i < NWAVE; ++i) r = fmax(r, sh[i]);
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

// Green test of node i with cash v on the snapshot of step t.
template <class T>
__device__ __forceinline__ bool is_green(T v, int sched, double theta, double maxabs) {
  const double a = fabs((double)v);
  if (sched == SCHED_ALL) return true;
  if (sched == SCHED_THRESHOLD) return a >= theta;
  if (sched == SCHED_MAXC) return a == maxabs;
  return a > theta;  // top-k: resolved into a strict bound plus explicit ties by the caller
}

// Top-k keys: |C| as the bits of a non-negative double, ties by smaller id.
template <class T>
__device__ __forceinline__ bool topk_green(T v, int i, double tau, int tie_limit_id) {
  const double a = fabs((double)v);
  return a > tau || (a == tau && i <= tie_limit_id);
}

__device__ __forceinline__ double pow_r(double a, double r) { return r == 1.0 ? a : pow(a, r); }

// ------------------------------------------------------------------ select

template <class T, int HK>
__global__ __launch_bounds__(BLOCK) void k_select(Dev d, long long s, double eps, long long s_limit, int force_all) {
  Glob *g = d.glob;
  if (g->status != 0) return;
  Rec *cur = &d.rec[s % 3];
  Rec *prv = &d.rec[(s + 2) % 3];
  Rec *nxt = &d.rec[(s + 1) % 3];

  const double l1 = cur->l1, hsum = cur->hsum, hnorm = cur->hnorm;
  int st = 0;
  if (s >= 1) {
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

  const int sched = force_all ? SCHED_ALL : d.sched;
  double theta = 0.0;
  if (sched == SCHED_THRESHOLD) {
    if ((s - 1) % d.theta_period == 0)
      theta = (d.r == 1.0) ? l1 / (double)d.n : pow(cur->sumr / (double)d.n, 1.0 / d.r);
    else
      theta = prv->theta;
  }
  const double maxabs = __longlong_as_double((long long)cur->maxabs_bits);
  double tau = 0.0;
  int tie_id = -1;
  if (sched == SCHED_TOPK) {
    tau = cur->topk_tau;
    tie_id = cur->topk_tie_id;
  }
  int mode;
  if (d.route == ROUTE_PUSH || d.colptr == nullptr) mode = 0;
  else if (d.route == ROUTE_PULL) mode = 1;
  else if (sched == SCHED_ALL) mode = 1;
  else mode = ((double)prv->gedges >= d.pull_alpha * (double)d.nnz) ? 1 : 0;

  if (blockIdx.x == 0 && threadIdx.x == 0) {
    cur->theta = theta;
    cur->mode = mode;
    nxt->l1 = 0.0;
    nxt->csum = 0.0;
    nxt->sumr = 0.0;
    nxt->maxabs_bits = 0ull;
    nxt->T = 0.0;
    nxt->msum = 0.0;
    nxt->dhnorm = 0.0;
    nxt->fr_pack = 0ull;
    nxt->green = 0;
    nxt->gedges = 0;
    nxt->ticket = 0u;
  }

  T *C = (T *)d.cash[cur->buf];
  const int n = d.n;
  const double c = d.c;
  const int ntiles = (n + TILE - 1) / TILE;

  __shared__ unsigned long long sh_scan[NWAVE];
  __shared__ double sh_red[4 * NWAVE];
  __shared__ long long sh_ll[NWAVE];
  __shared__ unsigned long long sh_base;

  double accT = 0.0, accM = 0.0, accDH = 0.0;
  long long accG = 0, accE = 0;

  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int base = tile * TILE;
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
      if (i < n) {
        const T x = C[i];
        const bool gr = (sched == SCHED_TOPK) ? topk_green(x, i, tau, tie_id) : is_green(x, sched, theta, maxabs);
        if (d.green_mask) d.green_mask[i] = gr ? 1 : 0;
        if (gr) {
          ++accG;
          if (x != T(0)) {
            const int r0 = d.rowptr[i];
            const int dg = d.rowptr[i + 1] - r0;
            // history: H_{t+1} = H_t + M_t (eq. (5))
            if (HK == 0) {
              double *H = (double *)d.hist;
              const double h = H[i];
              const double hn = h + (double)x;
              H[i] = hn;
              accDH += fabs(hn) - fabs(h);
            } else {
              float *Hh = (float *)d.hist;
              float *Hl = d.hist_lo;
              const float hi = Hh[i], lo = Hl[i], xf = (float)x;
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
              C[i] = force_all ? -x : T(0);
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
      }
    }
    if (mode == 0) {
      // frontier compaction: one 64-bit atomic per tile reserves both the
      // slots and the link range, so slot order and link order agree.
      unsigned long long tot;
      const unsigned long long mine = ((unsigned long long)cnt << 32) | edges;
      const unsigned long long ex = block_excl_scan(mine, sh_scan, &tot);
      if (threadIdx.x == 0) sh_base = tot ? atomicAdd(&cur->fr_pack, tot) : 0ull;
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
    if (r.a != 0.0) atomic_add_f64(&cur->T, r.a);
    if (r.b != 0.0) atomic_add_f64(&cur->msum, r.b);
    if (r.c != 0.0) atomic_add_f64(&cur->dhnorm, r.c);
    if (gsum) atomicAdd((unsigned long long *)&cur->green, (unsigned long long)gsum);
    if (esum) atomicAdd((unsigned long long *)&cur->gedges, (unsigned long long)esum);
  }
}

// -------------------------------------------------------------------- push

template <class T>
__global__ __launch_bounds__(BLOCK) void k_push(Dev d, long long s) {
  if (d.glob->status != 0) return;
  Rec *cur = &d.rec[s % 3];
  if (cur->mode != 0) return;
  const unsigned long long pk = cur->fr_pack;
  const int nent = (int)(pk >> 32);
  const int tot = (int)(pk & 0xffffffffu);
  if (tot == 0) return;
  T *C = (T *)d.cash[cur->buf];
  const int *__restrict__ col = d.col;
  const T *__restrict__ val = (const T *)d.val;
  const int nchunks = (tot + CH - 1) / CH;

  __shared__ int s_eoff[CH + 1];
  __shared__ int s_rs[CH + 1];
  __shared__ T s_sc[CH + 1];

  for (int b = blockIdx.x; b < nchunks; b += gridDim.x) {
    const int e0 = b * CH;
    const int e1 = min(tot, e0 + CH);
    const int j0 = d.chunk_first[b];
    const int j1 = (b + 1 < nchunks) ? d.chunk_first[b + 1] : nent - 1;
    // a chunk overlaps at most CH + 1 frontier rows (every row has a link)
    if (j0 < 0 || j1 >= nent || j1 < j0 || j1 - j0 + 1 > CH + 1) continue;
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
      if ((unsigned long long)idx >= (unsigned long long)d.nnz) continue;
      const int dst = col[idx];
      if ((unsigned)dst >= (unsigned)d.n) continue;  // links outside [0, N) are ignored
      const T amt = val ? s_sc[lo] * val[idx] : s_sc[lo];
      atomic_add_cash(&C[dst], amt);
    }
  }
}

// ----------------------------------------------------------------- complete

template <class T>
__device__ __forceinline__ void fold_stats(double x, double r, double &l1, double &cs, double &sr, double &mx) {
  const double a = fabs(x);
  l1 += a;
  cs += x;
  if (r != 1.0) sr += pow(a, r);
  mx = fmax(mx, a);
}

template <class T>
__device__ __forceinline__ double inv_outdeg(const Dev &d, int j) {
  if ((unsigned)j >= (unsigned)d.n) return 0.0;
  const int dg = d.rowptr[j + 1] - d.rowptr[j];
  return dg > 0 ? 1.0 / (double)dg : 0.0;
}

template <class T>
__global__ __launch_bounds__(BLOCK) void k_complete(Dev d, long long s, int force_all) {
  Glob *g = d.glob;
  if (g->status != 0) return;
  Rec *cur = &d.rec[s % 3];
  Rec *nxt = &d.rec[(s + 1) % 3];
  const int n = d.n;
  const double c = d.c;
  const double off = cur->T / (double)n;  // uniform restart share of eq. (6)
  const int mode = cur->mode;
  const double r = d.r;
  double l1 = 0.0, cs = 0.0, sr = 0.0, mx = 0.0;

  __shared__ double sh_red[4 * NWAVE];
  __shared__ double s_con[CH];
  __shared__ int s_last;

  if (mode == 0) {
    T *C = (T *)d.cash[cur->buf];
    const int ntiles = (n + TILE - 1) / TILE;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
#pragma unroll
      for (int q = 0; q < VPT; ++q) {
        const int i = tile * TILE + q * BLOCK + threadIdx.x;
        if (i < n) {
          const T x = (T)((double)C[i] + off);
          C[i] = x;
          fold_stats<T>((double)x, r, l1, cs, sr, mx);
        }
      }
    }
  } else {
    const int sched = force_all ? SCHED_ALL : d.sched;
    const double theta = cur->theta;
    const double maxabs = __longlong_as_double((long long)cur->maxabs_bits);
    const double tau = cur->topk_tau;
    const int tie_id = cur->topk_tie_id;
    const T *__restrict__ Cc = (const T *)d.cash[cur->buf];
    T *__restrict__ Cn = (T *)d.cash[cur->buf ^ 1];
    const int *__restrict__ colptr = d.colptr;
    const int *__restrict__ crow = d.crow;
    const T *__restrict__ cval = (const T *)d.cval;
    auto moved = [&](int j) -> double {
      if ((unsigned)j >= (unsigned)n) return 0.0;  // links outside [0, N) are ignored
      const T v = Cc[j];
      const bool gr = (sched == SCHED_TOPK) ? topk_green(v, j, tau, tie_id) : is_green(v, sched, theta, maxabs);
      return gr ? (double)v : 0.0;
    };
    auto kept = [&](int k) -> double {
      const T v = Cc[k];
      if (force_all) return -(double)v;  // step 0: C_0 - M_0 with C_0 = 0
      const bool gr = (sched == SCHED_TOPK) ? topk_green(v, k, tau, tie_id) : is_green(v, sched, theta, maxabs);
      return gr ? 0.0 : (double)v;
    };
    const int nitems = d.n_items;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
      const int4 item = d.items[it];
      if (item.x == ITEM_SHORT) {
        const int k0 = item.y, k1 = item.z;
        const int p0 = colptr[k0], p1 = colptr[k1];
        if (p1 - p0 > CH || p1 < p0) continue;  // the plan never builds such an item
        __syncthreads();
        for (int p = p0 + threadIdx.x; p < p1; p += BLOCK) {
          const int j = crow[p];
          const double m = moved(j);
          const double w = cval ? (double)cval[p] : inv_outdeg<T>(d, j);
          s_con[p - p0] = m * w;
        }
        __syncthreads();
        for (int k = k0 + threadIdx.x; k < k1; k += BLOCK) {
          const int a = colptr[k] - p0, b = colptr[k + 1] - p0;
          double acc = 0.0;
          for (int q = a; q < b; ++q) acc += s_con[q];
          const T x = (T)(kept(k) + c * acc + off);
          Cn[k] = x;
          fold_stats<T>((double)x, r, l1, cs, sr, mx);
        }
      } else if (item.x == ITEM_MEDIUM) {
        const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
        if (w < item.z) {
          const int k = d.med_cols[item.y + w];
          const int p0 = colptr[k], p1 = colptr[k + 1];
          double acc = 0.0;
          for (int p = p0 + lane; p < p1; p += 64) {
            const int j = crow[p];
            const double wgt = cval ? (double)cval[p] : inv_outdeg<T>(d, j);
            acc += moved(j) * wgt;
          }
          acc = wave_sum(acc);
          if (lane == 0) {
            const T x = (T)(kept(k) + c * acc + off);
            Cn[k] = x;
            fold_stats<T>((double)x, r, l1, cs, sr, mx);
          }
        }
      } else {  // ITEM_LONG piece: partial sum of one long column
        const int slot = item.y;
        const int k = d.long_cols[slot];
        const int p0 = item.z;
        const int p1 = min(item.w, colptr[k + 1]);
        double acc = 0.0;
        for (int p = p0 + threadIdx.x; p < p1; p += BLOCK) {
          const int j = crow[p];
          const double wgt = cval ? (double)cval[p] : inv_outdeg<T>(d, j);
          acc += moved(j) * wgt;
        }
        const Red4 t4 = block_sum4(Red4{acc, 0, 0, 0}, sh_red);
        if (threadIdx.x == 0) atomic_add_f64(&d.long_acc[slot], t4.a);
      }
    }
    // The last block to finish completes the long columns.
    if (d.n_long > 0) {
      __threadfence();
      __syncthreads();
      if (threadIdx.x == 0) s_last = (atomicAdd(&cur->ticket, 1u) == gridDim.x - 1);
      __syncthreads();
      if (s_last) {
        __threadfence();
        for (int q = threadIdx.x; q < d.n_long; q += BLOCK) {
          const int k = d.long_cols[q];
          const double acc = load_agent(&d.long_acc[q]);
          d.long_acc[q] = 0.0;
          const T x = (T)(kept(k) + c * acc + off);
          Cn[k] = x;
          fold_stats<T>((double)x, r, l1, cs, sr, mx);
        }
      }
    }
  }

  const Red4 t4 = block_sum4(Red4{l1, cs, sr, 0.0}, sh_red);
  const double bm = block_max(mx, sh_red);
  if (threadIdx.x == 0) {
    if (t4.a != 0.0) atomic_add_f64(&nxt->l1, t4.a);
    if (t4.b != 0.0) atomic_add_f64(&nxt->csum, t4.b);
    if (t4.c != 0.0) atomic_add_f64(&nxt->sumr, t4.c);
    if (bm > 0.0) atomic_max_nonneg(&nxt->maxabs_bits, bm);
    if (blockIdx.x == 0) {
      nxt->hsum = cur->hsum + cur->msum;
      nxt->hnorm = cur->hnorm + cur->dhnorm;
      nxt->edges_total = cur->edges_total + cur->gedges;
      nxt->green_total = cur->green_total + (s >= 1 ? cur->green : 0);
      nxt->buf = (mode == 0) ? cur->buf : (cur->buf ^ 1);
      g->t = s + 1;
      StepLog *lg = &d.log[s % LOG_STEPS];
      lg->s = s;
      lg->mode = mode;
      lg->green = cur->green;
      lg->gedges = cur->gedges;
      lg->nfront = (long long)(cur->fr_pack >> 32);
    }
  }
}

// -------------------------------------------------- top-k threshold search
//
// k_topk finds, for the snapshot C_t, the k-th largest |C| (tau) and the
// largest node id that still fits among the nodes with |C| = tau, so that
// green = |C| > tau or (|C| = tau and id <= tie_id) selects exactly k nodes
// ordered by |C| descending, then id ascending.  One block, bitwise radix
// search on the 63-bit pattern of |C| as a double, then a search on ids.
template <class T>
__global__ __launch_bounds__(1024) void k_topk(Dev d, long long s) {
  if (d.glob->status != 0) return;
  Rec *cur = &d.rec[s % 3];
  const T *C = (const T *)d.cash[cur->buf];
  const int n = d.n;
  const long long k = d.k < (long long)n ? d.k : (long long)n;
  __shared__ unsigned long long sh_cnt[1024 / 64];
  __shared__ unsigned long long sh_prefix;
  auto block_count = [&](auto pred) -> unsigned long long {
    unsigned long long c = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) c += pred(i) ? 1ull : 0ull;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) sh_cnt[threadIdx.x >> 6] = c;
    __syncthreads();
    unsigned long long t = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh_cnt[w];
    __syncthreads();
    return t;
  };
  auto keyof = [&](int i) -> unsigned long long {
    return (unsigned long long)__double_as_longlong(fabs((double)C[i]));
  };
  // largest pattern P such that #(key >= P) >= k: bitwise from the top
  if (threadIdx.x == 0) sh_prefix = 0ull;
  __syncthreads();
  for (int bit = 62; bit >= 0; --bit) {
    const unsigned long long cand = sh_prefix | (1ull << bit);
    const unsigned long long c = block_count([&](int i) { return keyof(i) >= cand; });
    if (threadIdx.x == 0 && c >= (unsigned long long)k) sh_prefix = cand;
    __syncthreads();
  }
  const unsigned long long tau_bits = sh_prefix;
  const unsigned long long above = block_count([&](int i) { return keyof(i) > tau_bits; });
  const long long need = k - (long long)above;  // >= 1 ties to take
  // smallest id bound I such that #(key == tau, id <= I) >= need
  if (threadIdx.x == 0) sh_prefix = 0ull;
  __syncthreads();
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = lo + (hi - lo) / 2;
    const unsigned long long c = block_count([&](int i) { return i <= mid && keyof(i) == tau_bits; });
    if (c >= (unsigned long long)need) hi = mid;
    else lo = mid + 1;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    cur->topk_tau = __longlong_as_double((long long)tau_bits);
    cur->topk_tie_id = lo;
  }
}

// ------------------------------------------------------------------ refresh
//
// Rebuilds the cash of state t from the history alone.  With C_0 = 0 the
// balance identity of Sec. 2.2 (eq. (7)) reads H_t + C_t = H_t P, so
// C_t = H_t P - H_t; it is evaluated in FP64 along the CSC columns and rounded
// once to the cash type.  This removes the rounding that FP32 routing leaves
// in C (whose exact sum is zero) without changing the method's trajectory.

__global__ void k_refresh_prep(Dev d, long long t) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Rec *cur = &d.rec[t % 3];
  cur->l1 = 0.0;
  cur->csum = 0.0;
  cur->sumr = 0.0;
  cur->maxabs_bits = 0ull;
  d.glob->rpool = 0.0;
  d.glob->ticket = 0u;
}

template <int HK>
__device__ __forceinline__ double hist_at(const Dev &d, int j) {
  if (HK == 0) return ((const double *)d.hist)[j];
  return (double)((const float *)d.hist)[j] + (double)d.hist_lo[j];
}

template <int HK>
__global__ __launch_bounds__(BLOCK) void k_refresh_pool(Dev d) {
  const int n = d.n;
  const double c = d.c;
  double acc = 0.0;
  __shared__ double sh_red[4 * NWAVE];
  for (int j = blockIdx.x * BLOCK + threadIdx.x; j < n; j += gridDim.x * BLOCK) {
    const bool dangling = d.rowptr[j + 1] == d.rowptr[j];
    acc += hist_at<HK>(d, j) * (dangling ? 1.0 : 1.0 - c);
  }
  const Red4 r = block_sum4(Red4{acc, 0, 0, 0}, sh_red);
  if (threadIdx.x == 0 && r.a != 0.0) atomic_add_f64(&d.glob->rpool, r.a);
}

template <class T, int HK>
__global__ __launch_bounds__(BLOCK) void k_refresh(Dev d, long long t, int out_buf) {
  Rec *cur = &d.rec[t % 3];
  const int n = d.n;
  const double c = d.c;
  const double off = d.glob->rpool / (double)n;
  const double r = d.r;
  T *__restrict__ Cn = (T *)d.cash[out_buf];
  const int *__restrict__ colptr = d.colptr;
  const int *__restrict__ crow = d.crow;
  const T *__restrict__ cval = (const T *)d.cval;
  double l1 = 0.0, cs = 0.0, sr = 0.0, mx = 0.0;
  __shared__ double sh_red[4 * NWAVE];
  __shared__ double s_con[CH];
  __shared__ int s_last;
  auto hin = [&](int j) -> double { return ((unsigned)j < (unsigned)n) ? hist_at<HK>(d, j) : 0.0; };
  const int nitems = d.n_items;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int4 item = d.items[it];
    if (item.x == ITEM_SHORT) {
      const int k0 = item.y, k1 = item.z;
      const int p0 = colptr[k0], p1 = colptr[k1];
      if (p1 - p0 > CH || p1 < p0) continue;
      __syncthreads();
      for (int p = p0 + threadIdx.x; p < p1; p += BLOCK) {
        const int j = crow[p];
        const double w = cval ? (double)cval[p] : inv_outdeg<T>(d, j);
        s_con[p - p0] = hin(j) * w;
      }
      __syncthreads();
      for (int k = k0 + threadIdx.x; k < k1; k += BLOCK) {
        const int a = colptr[k] - p0, b = colptr[k + 1] - p0;
        double acc = 0.0;
        for (int q = a; q < b; ++q) acc += s_con[q];
        const T x = (T)(c * acc + off - hin(k));
        Cn[k] = x;
        fold_stats<T>((double)x, r, l1, cs, sr, mx);
      }
    } else if (item.x == ITEM_MEDIUM) {
      const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
      if (w < item.z) {
        const int k = d.med_cols[item.y + w];
        double acc = 0.0;
        for (int p = colptr[k] + lane; p < colptr[k + 1]; p += 64) {
          const int j = crow[p];
          acc += hin(j) * (cval ? (double)cval[p] : inv_outdeg<T>(d, j));
        }
        acc = wave_sum(acc);
        if (lane == 0) {
          const T x = (T)(c * acc + off - hin(k));
          Cn[k] = x;
          fold_stats<T>((double)x, r, l1, cs, sr, mx);
        }
      }
    } else {
      const int slot = item.y;
      const int k = d.long_cols[slot];
      const int p1 = min(item.w, colptr[k + 1]);
      double acc = 0.0;
      for (int p = item.z + threadIdx.x; p < p1; p += BLOCK) {
        const int j = crow[p];
        acc += hin(j) * (cval ? (double)cval[p] : inv_outdeg<T>(d, j));
      }
      const Red4 t4 = block_sum4(Red4{acc, 0, 0, 0}, sh_red);
      if (threadIdx.x == 0) atomic_add_f64(&d.long_acc[slot], t4.a);
    }
  }
  if (d.n_long > 0) {
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_last = (atomicAdd(&d.glob->ticket, 1u) == gridDim.x - 1);
    __syncthreads();
    if (s_last) {
      __threadfence();
      for (int q = threadIdx.x; q < d.n_long; q += BLOCK) {
        const int k = d.long_cols[q];
        const double acc = load_agent(&d.long_acc[q]);
        d.long_acc[q] = 0.0;
        const T x = (T)(c * acc + off - hin(k));
        Cn[k] = x;
        fold_stats<T>((double)x, r, l1, cs, sr, mx);
      }
    }
  }
  const Red4 t4 = block_sum4(Red4{l1, cs, sr, 0.0}, sh_red);
  const double bm = block_max(mx, sh_red);
  if (threadIdx.x == 0) {
    if (t4.a != 0.0) atomic_add_f64(&cur->l1, t4.a);
    if (t4.b != 0.0) atomic_add_f64(&cur->csum, t4.b);
    if (t4.c != 0.0) atomic_add_f64(&cur->sumr, t4.c);
    if (bm > 0.0) atomic_max_nonneg(&cur->maxabs_bits, bm);
  }
}

__global__ void k_refresh_done(Dev d, long long t, int out_buf) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  d.rec[t % 3].buf = out_buf;
  d.glob->status = 0;
}

// ------------------------------------------------------------ init / misc

template <class T, int HK>
__global__ __launch_bounds__(BLOCK) void k_reset(Dev d) {
  const int n = d.n;
  const T m0 = (T)(1.0 / (double)n);
  T *C = (T *)d.cash[0];
  for (int i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) {
    C[i] = m0;  // holds M_0 = (1/N) 1 until step 0 moves it
    if (HK == 0) {
      ((double *)d.hist)[i] = 0.0;
    } else {
      ((float *)d.hist)[i] = 0.0f;
      d.hist_lo[i] = 0.0f;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x < 3) {
    Rec *r = &d.rec[threadIdx.x];
    r->l1 = threadIdx.x == 0 ? 1.0 : 0.0;
    r->csum = 0.0;
    r->sumr = 0.0;
    r->maxabs_bits = 0ull;
    r->hsum = 0.0;
    r->hnorm = 0.0;
    r->edges_total = 0;
    r->green_total = 0;
    r->buf = 0;
    r->mode = 0;
    r->theta = 0.0;
    r->T = 0.0;
    r->msum = 0.0;
    r->dhnorm = 0.0;
    r->fr_pack = 0ull;
    r->green = 0;
    r->gedges = 0;
    r->ticket = 0u;
    r->topk_tau = 0.0;
    r->topk_tie_id = -1;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    d.glob->status = 0;
    d.glob->t = 0;
    d.glob->ticket = 0u;
    d.glob->rpool = 0.0;
  }
  for (int q = blockIdx.x * BLOCK + threadIdx.x; q < d.n_long; q += gridDim.x * BLOCK) d.long_acc[q] = 0.0;
  for (int q = blockIdx.x * BLOCK + threadIdx.x; q < LOG_STEPS; q += gridDim.x * BLOCK) d.log[q].s = -1;
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
    double h;
    if (HK == 0) h = ((const double *)d.hist)[i];
    else h = (double)((const float *)d.hist)[i] + (double)d.hist_lo[i];
    pi[i] = h / hs;  // pi_hat_t = H_t / (H_t 1), eq. (2)
  }
}

template <class T, int HK>
__global__ __launch_bounds__(BLOCK) void k_export(Dev d, double *Cout, double *Hout) {
  const long long t = d.glob->t;
  const T *C = (const T *)d.cash[d.rec[t % 3].buf];
  const int n = d.n;
  for (int i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) {
    if (Cout) Cout[i] = (double)C[i];
    if (Hout) {
      if (HK == 0) Hout[i] = ((const double *)d.hist)[i];
      else Hout[i] = (double)((const float *)d.hist)[i] + (double)d.hist_lo[i];
    }
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
    const T x = (T)Cin[i];
    C[i] = x;
    fold_stats<T>((double)x, r, l1, cs, sr, mx);
    const double h = Hin[i];
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
  const Red4 a = block_sum4(Red4{l1, cs, sr, hs}, sh_red);
  const Red4 b = block_sum4(Red4{hn, 0, 0, 0}, sh_red);
  const double bm = block_max(mx, sh_red);
  if (threadIdx.x == 0) {
    atomic_add_f64(&cur->l1, a.a);
    atomic_add_f64(&cur->csum, a.b);
    atomic_add_f64(&cur->sumr, a.c);
    atomic_add_f64(&cur->hsum_import, a.d);
    atomic_add_f64(&cur->hnorm, b.a);
    if (bm > 0.0) atomic_max_nonneg(&cur->maxabs_bits, bm);
  }
}

__global__ void k_prepare_import(Dev d, long long t, int buf) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int q = 0; q < 3; ++q) {
    Rec *r = &d.rec[q];
    r->l1 = 0.0;
    r->csum = 0.0;
    r->sumr = 0.0;
    r->maxabs_bits = 0ull;
    r->hsum = 0.0;
    r->hsum_import = 0.0;
    r->hnorm = 0.0;
    r->T = 0.0;
    r->msum = 0.0;
    r->dhnorm = 0.0;
    r->fr_pack = 0ull;
    r->green = 0;
    r->gedges = 0;
    r->ticket = 0u;
    r->mode = 0;
    r->theta = 0.0;
    r->topk_tau = 0.0;
    r->topk_tie_id = -1;
  }
  Rec *cur = &d.rec[t % 3];
  cur->buf = buf;
  cur->edges_total = 0;
  cur->green_total = 0;
  d.rec[(t + 2) % 3].gedges = d.nnz;  // the AUTO router sees a dense previous step
  d.glob->status = 0;
  d.glob->t = t;
}

__global__ void k_finish_import(Dev d, long long t, double h_sum) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Rec *cur = &d.rec[t % 3];
  cur->hsum = isnan(h_sum) ? cur->hsum_import : h_sum;
}

// ------------------------------------------------------- explicit instances

template __global__ void k_select<float, 0>(Dev, long long, double, long long, int);
template __global__ void k_select<float, 1>(Dev, long long, double, long long, int);
template __global__ void k_select<double, 0>(Dev, long long, double, long long, int);
template __global__ void k_push<float>(Dev, long long);
template __global__ void k_push<double>(Dev, long long);
template __global__ void k_complete<float>(Dev, long long, int);
template __global__ void k_complete<double>(Dev, long long, int);
template __global__ void k_topk<float>(Dev, long long);
template __global__ void k_topk<double>(Dev, long long);
template __global__ void k_reset<float, 0>(Dev);
template __global__ void k_reset<float, 1>(Dev);
template __global__ void k_reset<double, 0>(Dev);
template __global__ void k_refresh_pool<0>(Dev);
template __global__ void k_refresh_pool<1>(Dev);
template __global__ void k_refresh<float, 0>(Dev, long long, int);
template __global__ void k_refresh<float, 1>(Dev, long long, int);
template __global__ void k_refresh<double, 0>(Dev, long long, int);
template __global__ void k_normalize<0>(Dev, double *);
template __global__ void k_normalize<1>(Dev, double *);
template __global__ void k_export<float, 0>(Dev, double *, double *);
template __global__ void k_export<float, 1>(Dev, double *, double *);
template __global__ void k_export<double, 0>(Dev, double *, double *);
template __global__ void k_import<float, 0>(Dev, const double *, const double *, long long, int);
template __global__ void k_import<float, 1>(Dev, const double *, const double *, long long, int);
template __global__ void k_import<double, 0>(Dev, const double *, const double *, long long, int);

}  // namespace rlgl
