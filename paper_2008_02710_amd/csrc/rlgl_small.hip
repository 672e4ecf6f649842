// A whole RLGL solve of a small chain in one workgroup (one launch).
//
// For chains whose cash vector fits in one workgroup's LDS (N up to about
// 20,000 states in FP64 on gfx950), the step-to-step dependence of
// Algorithm 1 makes a multi-launch solve latency-bound: every step waits for
// the whole previous step.  Here one workgroup of 512 threads runs step 0,
// the green-light steps, the stop test and the normalisation pi_hat = H/(H 1)
// without leaving the kernel; C lives in LDS, the history H and the moved
// cash in the caller's workspace (L2-resident at these sizes), and workgroup
// barriers are the only synchronisation.
//
// Two routes per step (eq. (6), C_{t+1} = C_t - M_t + M_t P):
//   * list route, for RLGL_MaxC (Sec. 6): the maximisers are collected in LDS
//     (from per-thread records the previous step's share pass kept, or by a
//     scan) and wave 0 moves their cash in increasing node order, link by
//     link along the CSR rows (the lanes load a green node's links together;
//     the adds are made in link order, or all at once when they are equal),
//     then the restart share is added to every node.  With FP64 cash this is
//     the operation order of the plain serial method (C -= M for every green
//     node, then the links of each green node in turn, then the uniform
//     share), so the cash vector equals the serial one bit for bit and so
//     does the green set of every step.
//   * column route, for every other rule (and MaxC ties beyond the list's
//     capacity): every green node publishes c P'_ij M_i (or M_i with stored
//     values), and each column k sums C_k - M_k plus its in-links in
//     increasing source order (the CSC order), then the share.  Only the
//     restart pool is summed in another order than the serial one.
// The FP32-cash variant rounds each node once per column route (FP64 sums);
// its list route rounds once per link, and a stop is accepted only on the
// cash rebuilt from the history, C_t = H_t P - H_t (eq. (7)), when refresh is
// set.
#include <type_traits>

#include "rlgl_device.h"

namespace rlgl {

constexpr int SM_BLOCK = 512;             // threads of the one workgroup (8 waves; about 215 VGPRs, no spills)
constexpr int SM_NW = SM_BLOCK / 64;
constexpr int SM_LIST = 512;              // green nodes the list route takes
constexpr int SM_BATCH = 8;               // in-links of a column whose loads are sent together
constexpr int SM_UNROLL = 8;              // nodes per thread whose LDS loads are sent together

// Result record of a small solve (in the workspace).
struct SmallRec {
  long long t, green, green_total, edges;
  double l1, hsum, csum, theta;
  int status, last_route;
};

struct SmallArgs {
  int n;
  long long nnz;
  double c;
  const int *rowptr, *col, *colptr, *crow;
  const void *val, *cval;  // stored link values (cash type) or both null: 1/outdeg
  int sched;
  double r;
  int theta_period;
  unsigned long long seed;
  int refresh;  // FP32 cash: accept a stop only on the cash rebuilt from H
  int rp_lds;   // the CSR row pointers are copied into LDS after the cash (they fit)
  double eps;
  long long max_steps;
  double *H;  // [n] history
  double *Q;  // [n] what each node sends along one of its links this step
  SmallRec *rec;
  double *pi;  // [n] output or null
};

// Block sums of three doubles and the maximum of a fourth (non-negative);
// every thread receives them.  Two barriers.
struct Red3M {
  double a, b, c, m;
};
__device__ __forceinline__ Red3M small_reduce(Red3M v, double *sh /* 4 * SM_NW */) {
  v.a = wave_sum(v.a);
  v.b = wave_sum(v.b);
  v.c = wave_sum(v.c);
  v.m = wave_max(v.m);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) {
    sh[w] = v.a;
    sh[SM_NW + w] = v.b;
    sh[2 * SM_NW + w] = v.c;
    sh[3 * SM_NW + w] = v.m;
  }
  __syncthreads();
  Red3M r{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < SM_NW; ++i) {
    r.a += sh[i];
    r.b += sh[SM_NW + i];
    r.c += sh[2 * SM_NW + i];
    r.m = fmax(r.m, sh[3 * SM_NW + i]);
  }
  __syncthreads();
  return r;
}

__device__ __forceinline__ long long small_sum_ll(long long v, long long *sh) {
  v = wave_sum_ll(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) sh[w] = v;
  __syncthreads();
  long long r = 0;
#pragma unroll
  for (int i = 0; i < SM_NW; ++i) r += sh[i];
  __syncthreads();
  return r;
}

// A double of lane q (uniform q) on every lane.
__device__ __forceinline__ double rd_lane(double v, int q) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned int)(b & 0xffffffffll), q);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), q);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}

template <class T>
__global__ __launch_bounds__(SM_BLOCK) void k_small(SmallArgs a) {
#pragma clang fp contract(off)
  extern __shared__ __align__(16) unsigned char sm_dyn[];
  T *C = (T *)sm_dyn;
  __shared__ double s_red[4 * SM_NW];
  __shared__ long long s_ll[SM_NW];
  __shared__ int s_list[SM_LIST];
  // list route: each green node's moved cash, out-degree and first link
  __shared__ double s_lm[SM_LIST];
  __shared__ int s_ld[SM_LIST], s_lr[SM_LIST];
  __shared__ int s_cnt;
  __shared__ int s_ovf;  // a thread holds more than two maximisers
  __shared__ double s_out[4];  // list route: moved sum, restart pool, change of ||H||_1
  __shared__ long long s_edges;
  __shared__ int s_bad;  // a pointer or link index outside its range was met

  const int tid = threadIdx.x;
  const int n = a.n;
  const double c = a.c;
  const int *__restrict__ rowptr = a.rowptr;
  const int *__restrict__ colptr = a.colptr;
  const int *__restrict__ crow = a.crow;
  const T *__restrict__ cval = (const T *)a.cval;
  double *__restrict__ H = a.H;
  double *__restrict__ Q = a.Q;
  const bool stored = a.cval != nullptr;
  const bool fp32 = sizeof(T) == 4;

  const long long nnz = a.nnz;
  // Pointers and link indices are checked where they are read: a value
  // outside its range is skipped and reported (status ST_BAD_GRAPH), never
  // followed.
  auto deg = [&](int i) -> int {
    const int r0 = rowptr[i], r1 = rowptr[i + 1];
    if (r0 < 0 || r1 < r0 || (long long)r1 > nnz) {
      s_bad = 1;
      return 0;
    }
    return r1 - r0;
  };
  // c P'_ij M_i for implied link values (the product in the serial order:
  // (c w) m), M_i itself with stored ones (the link value is applied per link)
  auto sent = [&](double m, int d) -> double {
    if (m == 0.0 || d == 0) return 0.0;
    if (stored) return m;
    const double cw = c * (1.0 / (double)d);
    return cw * m;
  };
  // Column route: C_k <- (C_k - M_k) + sum_{j in in(k)} c P'_jk M_j + share,
  // the in-links in CSC order (increasing source); Q holds what each source
  // sends.  Folds the statistics of the new cash.
  double l1p, csp, srp, mxp;
  const bool rp = a.r != 1.0;
  auto fold = [&](double x) {
    const double ax = fabs(x);
    l1p += ax;
    csp += x;
    if (rp) srp += pow(ax, a.r);
    mxp = fmax(mxp, ax);
  };
  auto column_pass = [&](auto kept, double share) {
    l1p = csp = srp = mxp = 0.0;
    for (int k = tid; k < n; k += SM_BLOCK) {
      double acc = kept(k);
      int p0 = colptr[k], p1 = colptr[k + 1];
      if (p0 < 0 || p1 < p0 || (long long)p1 > nnz) {
        s_bad = 1;
        p1 = p0;
      }
      for (int p = p0; p < p1; p += SM_BATCH) {
        // the batch's loads are independent: sent together, added in order
        int jj[SM_BATCH];
        double qq[SM_BATCH], ww[SM_BATCH];
#pragma unroll
        for (int u = 0; u < SM_BATCH; ++u) {
          jj[u] = (p + u < p1) ? crow[p + u] : -1;
          if (p + u < p1 && (unsigned)jj[u] >= (unsigned)n) {
            s_bad = 1;
            jj[u] = -1;
          }
        }
#pragma unroll
        for (int u = 0; u < SM_BATCH; ++u) {
          qq[u] = (jj[u] >= 0) ? Q[jj[u]] : 0.0;
          ww[u] = (stored && jj[u] >= 0) ? (double)cval[p + u] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < SM_BATCH; ++u) {
          if (qq[u] != 0.0) {
            double add = qq[u];
            if (stored) {
              const double cw = c * ww[u];
              add = cw * qq[u];
            }
            acc = acc + add;
          }
        }
      }
      const T y = (T)(acc + share);
      C[k] = y;
      fold((double)y);
    }
  };

  // ---- step 0 (eq. (3), then eqs. (5)-(6) with G_0 = [N], M_0 = (1/N) 1)
  if (tid == 0) {
    s_bad = 0;
    s_ovf = 0;
    s_cnt = 0;
  }
  // the list route reads each green node's row pointers from this copy
  int *s_rp = (int *)(sm_dyn + (((size_t)n * sizeof(T) + 15) & ~(size_t)15));
  if (a.rp_lds)
    for (int i = tid; i <= n; i += SM_BLOCK) s_rp[i] = rowptr[i];
  __syncthreads();
  const double m0 = 1.0 / (double)n;
  long long edges = 0;
  for (int i = tid; i < n; i += SM_BLOCK) {
    const int d = deg(i);
    H[i] = m0;
    Q[i] = sent(m0, d);
    if (d > 0) edges += d;
  }
  edges = small_sum_ll(edges, s_ll);
  if (tid == 0) {
    // H_1 1 and the restart pool of M_0 summed in node order, as the serial method does
    double s = 0.0, pool = 0.0;
    for (int i = 0; i < n; ++i) {
      s += m0;
      pool += (deg(i) > 0) ? (1.0 - c) * m0 : m0;
    }
    s_out[0] = s;
    s_out[1] = pool;
  }
  __syncthreads();
  double hsum = s_out[0];
  double hnorm = hsum;
  column_pass([&](int) { return -m0; }, s_out[1] / (double)n);

  long long t = 1, green = 0, green_total = 0, refreshed_at = -1;
  // MaxC: the pass that adds the restart share also keeps, per thread, its
  // largest |C| and the nodes that hold it (up to two); `tracked` says they
  // describe the cash the next step selects from
  bool tracked = false;
  double tmax = -1.0;
  int tidx0 = -1, tidx1 = -1, tcnt = 0;
  int status = ST_RUNNING, last_route = ROUTE_PULL;
  double theta = 0.0, l1 = 0.0, csum = 0.0;
  // l1 and max after a list-route step with FP64 cash and r = 1 (the other
  // sums are zero there): one exchange and one barrier; the exchange buffer
  // alternates with the step, and the route's barrier lies between a read of
  // one buffer and the next write of it
  __shared__ double s_r2[2][2 * SM_NW];
  for (;;) {
    Red3M st;
    if (tracked && !fp32 && !rp) {
      const double lw = wave_sum(l1p), mw = wave_max(mxp);
      double *b2 = s_r2[t & 1];
      if ((tid & 63) == 0) {
        b2[tid >> 6] = lw;
        b2[SM_NW + (tid >> 6)] = mw;
      }
      __syncthreads();
      st = Red3M{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int i = 0; i < SM_NW; ++i) {
        st.a += b2[i];
        st.m = fmax(st.m, b2[SM_NW + i]);
      }
    } else {
      st = small_reduce(Red3M{l1p, csp, srp, mxp}, s_red);
    }
    l1 = st.a;
    csum = st.b;
    const double maxabs = st.m;
    if (s_bad) {
      status = ST_BAD_GRAPH;
      break;
    }
    if (!isfinite(l1) || !isfinite(hsum)) {
      status = ST_NONFINITE;
      break;
    }
    if (fabs(hsum) <= 1e-300 || fabs(hsum) <= 1e-12 * hnorm) {
      status = ST_ZERO_HISTORY;
      break;
    }
    const bool stop = t >= 2 && l1 / fabs(hsum) < a.eps;
    const bool drift = fp32 && fabs(csum) > 0.5 * l1;
    if (fp32 && a.refresh && (stop || drift) && refreshed_at != t) {
      // C_t = H_t P - H_t in FP64 (eq. (7) with C_0 = 0), rounded once
      double pool = 0.0;
      for (int j = tid; j < n; j += SM_BLOCK) {
        const int d = deg(j);
        const double h = H[j];
        Q[j] = sent(h, d);
        pool += (d > 0) ? (1.0 - c) * h : h;
      }
      pool = small_reduce(Red3M{pool, 0.0, 0.0, 0.0}, s_red).a;
      column_pass([&](int k) { return -H[k]; }, pool / (double)n);
      tracked = false;
      refreshed_at = t;
      continue;
    }
    if (stop) {
      status = ST_CONVERGED;
      break;
    }
    if (t - 1 >= a.max_steps) {
      status = ST_LIMIT;
      break;
    }
    if (a.sched == SCHED_THRESHOLD && (t - 1) % a.theta_period == 0)
      theta = (a.r == 1.0) ? l1 / (double)n : pow(st.c / (double)n, 1.0 / a.r);

    // ---- list route (RLGL_MaxC)
    bool listed = false;
    if (a.sched == SCHED_MAXC) {
      if (tracked) {
        // the maximisers from the per-thread records (s_cnt was cleared by
        // the pass that made them); a thread that holds more than two falls
        // back to the scan below
        if (tmax == maxabs) {
          if (tcnt > 2) {
            s_ovf = 1;
          } else {
            const int q = atomicAdd(&s_cnt, tcnt);
            if (q < SM_LIST) s_list[q] = tidx0;
            if (tcnt == 2 && q + 1 < SM_LIST) s_list[q + 1] = tidx1;
          }
        }
        __syncthreads();
      }
      const bool scan = !tracked || s_ovf;
      if (scan) {
        __syncthreads();  // every thread has read s_ovf
        if (tid == 0) {
          s_cnt = 0;
          s_ovf = 0;
        }
        __syncthreads();
      }
      // SM_UNROLL independent LDS loads per thread before the first is used
      for (int base = 0; scan && base < n; base += SM_BLOCK * SM_UNROLL) {
        double v[SM_UNROLL];
#pragma unroll
        for (int u = 0; u < SM_UNROLL; ++u) {
          // an index clamped into [0, n): no load waits behind a branch
          const int i = base + u * SM_BLOCK + tid;
          const double x = fabs((double)C[min(i, n - 1)]);
          v[u] = (i < n) ? x : -1.0;
        }
#pragma unroll
        for (int u = 0; u < SM_UNROLL; ++u) {
          if (v[u] == maxabs) {
            const int q = atomicAdd(&s_cnt, 1);
            if (q < SM_LIST) s_list[q] = base + u * SM_BLOCK + tid;
          }
        }
      }
      if (scan) __syncthreads();
      const int ng = s_cnt;
      if (ng <= SM_LIST) {
        listed = true;
        if (tid < 64) {
          // Wave 0 routes the list.  Loads are made by the lanes together;
          // every update of the cash and of the sums is made one at a time in
          // the serial order, from values read out of the lanes.
          const int lane = tid;
          if (lane == 0) {
            // increasing node order (insertion sort; the list is usually one node)
            for (int q = 1; q < ng; ++q) {
              const int v = s_list[q];
              int p = q - 1;
              while (p >= 0 && s_list[p] > v) {
                s_list[p + 1] = s_list[p];
                --p;
              }
              s_list[p + 1] = v;
            }
          }
          wave_lds_fence();
          double msum = 0.0, pool = 0.0, dh = 0.0;
          long long e = 0;
          // The history of the first 64 listed nodes is loaded here and
          // updated after the links are routed (H takes no part in moving the
          // cash), so its round trip overlaps theirs.
          const int nq0 = min(64, ng);
          const int li0 = min(max(s_list[min(lane, max(nq0 - 1, 0))], 0), n - 1);  // in [0, n) whatever the list
          const double h00 = H[li0];
          // M_t from the snapshot: every green node's cash leaves before any
          // arrives (the nodes of the list are distinct)
          for (int q0 = 0; q0 < ng; q0 += 64) {
            const int nq = min(64, ng - q0);
            double lm = 0.0;
            if (lane < nq) {
              const int li = s_list[q0 + lane];
              lm = (double)C[li];
              C[li] = (T)((double)C[li] - lm);
              s_lm[q0 + lane] = lm;
              const int r0 = a.rp_lds ? s_rp[li] : rowptr[li];
              const int r1 = a.rp_lds ? s_rp[li + 1] : rowptr[li + 1];
              const bool okr = r0 >= 0 && r1 >= r0 && (long long)r1 <= nnz;
              if (!okr) s_bad = 1;
              s_ld[q0 + lane] = okr ? r1 - r0 : 0;
              s_lr[q0 + lane] = r0;
            }
            for (int q = 0; q < nq; ++q) msum += rd_lane(lm, q);
          }
          wave_lds_fence();
          for (int q = 0; q < ng; ++q) {
            const double m = s_lm[q];
            if (m == 0.0) continue;
            const int d = s_ld[q];
            const int r0 = s_lr[q];
            if (d == 0) {
              pool += m;
              continue;
            }
            e += d;
            for (int b = 0; b < d; b += 64) {
              const int nb = min(64, d - b);
              int lk = -1;
              double ladd = 0.0;
              if (lane < nb) {
                const int p = r0 + b + lane;
                const double w = a.val ? (double)((const T *)a.val)[p] : 1.0 / (double)d;
                const double cw = c * w;
                ladd = cw * m;
                lk = a.col[p];
                if ((unsigned)lk >= (unsigned)n) {
                  s_bad = 1;
                  lk = -1;
                }
              }
              // FP64 cash and one value on every link of the chunk: the adds
              // are equal, so the lanes may make them in any order (an LDS
              // atomic for a node linked twice); otherwise one at a time in
              // link order
              const double a0 = rd_lane(ladd, 0);
              if (!fp32 && __ballot(lane < nb && ladd != a0) == 0ull) {
                if (lk >= 0) atomicAdd((double *)&C[lk], ladd);
              } else {
                for (int u = 0; u < nb; ++u) {
                  const int k = __builtin_amdgcn_readlane(lk, u);
                  const double add = rd_lane(ladd, u);
                  if (k >= 0 && lane == 0) C[k] = (T)((double)C[k] + add);
                }
              }
              wave_lds_fence();
            }
            pool += (1.0 - c) * m;
          }
          // H_{t+1} = H_t + M_t on the listed nodes (eq. (5)), and the change
          // of ||H||_1 summed in list order
          for (int q0 = 0; q0 < ng; q0 += 64) {
            const int nq = min(64, ng - q0);
            double ldh = 0.0;
            if (lane < nq) {
              const int li = s_list[q0 + lane];
              const double h0 = (q0 == 0) ? h00 : H[li];
              const double h1 = h0 + s_lm[q0 + lane];
              H[li] = h1;
              ldh = fabs(h1) - fabs(h0);
            }
            for (int q = 0; q < nq; ++q) dh += rd_lane(ldh, q);
          }
          if (lane == 0) {
            s_out[0] = msum;
            s_out[1] = pool;
            s_out[2] = dh;
            s_edges = e;
          }
        }
        __syncthreads();
        const double share = s_out[1] / (double)n;
        hsum = hsum + s_out[0];
        hnorm += s_out[2];
        edges += s_edges;
        green = ng;
        l1p = csp = srp = mxp = 0.0;
        tmax = -1.0;
        tcnt = 0;
        if (tid == 0) s_cnt = 0;  // every thread read it before the barrier above
        // C_k + share for every node, with the statistics of fold() (the sum
        // of C only where the drift test needs it, FP32 cash; the maximum is
        // tmax) and the per-thread maximisers.  Whole chunks of SM_UNROLL
        // nodes per thread carry no bounds test, so their loads are all sent
        // before the first is used; the power sum is a separate instance.
        auto share_pass = [&](auto rpow) {
          constexpr bool RPW = decltype(rpow)::value;
          auto one = [&](double v, int k) {
            const T y = (T)(v + share);
            C[k] = y;
            const double ay = fabs((double)y);
            l1p += ay;
            if (fp32) csp += (double)y;
            if (RPW) srp += pow(ay, a.r);
            const bool gt = ay > tmax, eq = ay == tmax;
            tidx1 = (eq && tcnt == 1) ? k : tidx1;
            tcnt = gt ? 1 : (eq ? tcnt + 1 : tcnt);
            tidx0 = gt ? k : tidx0;
            tmax = gt ? ay : tmax;
          };
          int base = 0;
          for (; base + SM_BLOCK * SM_UNROLL <= n; base += SM_BLOCK * SM_UNROLL) {
            double v[SM_UNROLL];
#pragma unroll
            for (int u = 0; u < SM_UNROLL; ++u) v[u] = (double)C[base + u * SM_BLOCK + tid];
#pragma unroll
            for (int u = 0; u < SM_UNROLL; ++u) one(v[u], base + u * SM_BLOCK + tid);
          }
          for (int k = base + tid; k < n; k += SM_BLOCK) one((double)C[k], k);
        };
        if (rp) share_pass(std::true_type{});
        else share_pass(std::false_type{});
        mxp = fmax(tmax, 0.0);
        tracked = true;
        last_route = ROUTE_PUSH;
      }
    }

    // ---- column route
    if (!listed) {
      double msum = 0.0, pool = 0.0, dh = 0.0;
      long long e = 0, g = 0;
      for (int i = tid; i < n; i += SM_BLOCK) {
        const T v = C[i];
        const bool gr = is_green(v, i, a.sched, theta, maxabs, 0.0, -1, a.seed, t);
        const double m = gr ? (double)v : 0.0;
        const int d = deg(i);
        Q[i] = sent(m, d);
        g += gr ? 1 : 0;
        if (m != 0.0) {
          const double h0 = H[i];
          const double h1 = h0 + m;
          H[i] = h1;
          dh += fabs(h1) - fabs(h0);
          e += d;
          C[i] = (T)((double)v - m);
        }
        msum += m;
        pool += (d > 0) ? (1.0 - c) * m : m;
      }
      const Red3M r = small_reduce(Red3M{msum, pool, dh, 0.0}, s_red);
      e = small_sum_ll(e, s_ll);
      g = small_sum_ll(g, s_ll);
      hsum = hsum + r.a;
      hnorm += r.c;
      edges += e;
      green = g;
      column_pass([&](int k) { return (double)C[k]; }, r.b / (double)n);
      tracked = false;
      last_route = ROUTE_PULL;
    }
    green_total += green;
    ++t;
    // no barrier here: the reduction that opens the next step has one before
    // any thread reads what this step wrote
  }

  if (!fp32 && tracked) {
    // the last pass was the list route's, which leaves out the sum of C
    double cs = 0.0;
    for (int k = tid; k < n; k += SM_BLOCK) cs += (double)C[k];
    csum = small_reduce(Red3M{cs, 0.0, 0.0, 0.0}, s_red).a;
  }
  if (a.pi && (status == ST_CONVERGED || status == ST_LIMIT)) {
    for (int i = tid; i < n; i += SM_BLOCK) a.pi[i] = H[i] / hsum;  // pi_hat_t = H_t / (H_t 1), eq. (2)
  }
  if (tid == 0) {
    SmallRec *o = a.rec;
    o->t = t;
    o->green = green;
    o->green_total = green_total;
    o->edges = edges;
    o->l1 = l1;
    o->hsum = hsum;
    o->csum = csum;
    o->theta = a.sched == SCHED_THRESHOLD ? theta : 0.0;
    o->status = status;
    o->last_route = last_route;
  }
}

template __global__ void k_small<double>(SmallArgs);
template __global__ void k_small<float>(SmallArgs);

}  // namespace rlgl
