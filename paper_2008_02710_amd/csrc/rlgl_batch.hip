// Batched RLGL: many independent chains in one persistent launch.
//
// The grid is sized to the machine (workgroups per CU x CUs).  Every
// workgroup takes the next chain from a device queue (chains are ordered by
// decreasing link count on the host, so the longest solves start first) and
// runs that chain's whole solve - step 0, the green-light steps, the stop
// test, the FP64 refresh that confirms a stop and the normalisation - with
// workgroup barriers only.  Nothing crosses workgroups but the queue ticket,
// so no device-scope fence is ever issued.  A chain's cash sits in two
// ping-pong buffers; the route is the CSC gather of the single-chain pull
// (column_item), its columns packed into runs of at most CH links.
#include "rlgl_device.h"

namespace rlgl {

struct ChainDesc {
  long long node_off;  // first node in the concatenated state vectors
  long long rp_off;    // first entry of the chain's row/column pointers (node_off + chain index)
  long long edge_off;  // first link in the concatenated link arrays
  int n, nnz;
  int item_off, n_items;
  double c;
  double eps;          // stop threshold on ||C_t||_1 / |H_t 1|
};

struct ChainOut {
  long long t, edges;
  double resid, hsum;
  int status, green_steps;
  long long t0, t1;    // device wall clock at start and end of the chain's solve
};

struct BatchDev {
  int n_chains;
  int sched;
  double r;
  long long max_steps;
  int refresh;
  const ChainDesc *chains;
  const int *order;
  ChainOut *out;
  const int *rowptr, *col, *colptr, *crow;
  const void *val, *cval;
  const int4 *items;
  void *cash0, *cash1, *hist;
  float *hist_lo;
  unsigned int *queue;
  double *pi;
};

template <int NW>
__device__ __forceinline__ double block_sum1(double v, double *sh) {
  return block_sum4<NW>(Red4{v, 0, 0, 0}, sh).a;
}

template <class T, int HK, int NT>
__device__ void batch_chain(const BatchDev &b, int k, ColLds<NT> &L) {
  constexpr int NW = NT / 64;
  const ChainDesc cd = b.chains[k];
  const long long t_start = wall_clock64();
  const int n = cd.n;
  const double c = cd.c;
  const double rr = b.r;
  const int tid = threadIdx.x;
  const int *__restrict__ rowptr = b.rowptr + cd.rp_off;
  __shared__ int s_bad;  // a link index or plan item outside its range
  if (tid == 0) s_bad = 0;
  __syncthreads();
  const ColView g{b.colptr + cd.rp_off, b.crow + cd.edge_off, rowptr,
                  b.cval ? (const void *)((const T *)b.cval + cd.edge_off) : nullptr, n, 0, &s_bad};
  T *Ca = (T *)b.cash0 + cd.node_off;
  T *Cb = (T *)b.cash1 + cd.node_off;
  double *H64 = (double *)b.hist + cd.node_off;
  float *Hhi = (float *)b.hist + cd.node_off;
  float *Hlo = b.hist_lo ? b.hist_lo + cd.node_off : nullptr;
  const int4 *items = b.items + cd.item_off;
  auto hist = [&](int i) -> double { return HK == 0 ? H64[i] : (double)Hhi[i] + (double)Hlo[i]; };
  auto deg = [&](int i) -> int { return rowptr[i + 1] - rowptr[i]; };

  // statistics of the cash vector produced by a route pass
  double l1, cs, sr, mx;
  auto route = [&](auto moved, auto kept, double off, T *out) {
    double a = 0.0, bb = 0.0, cc = 0.0, m = 0.0;
    for (int it = 0; it < cd.n_items; ++it)
      column_item<T, NT>(g, items[it], moved, kept, c, off, rr, out, nullptr, L, a, bb, cc, m);
    const Red4 s4 = block_sum4<NW>(Red4{a, bb, cc, 0.0}, L.red);
    l1 = s4.a;
    cs = s4.b;
    sr = s4.c;
    mx = block_max<NW>(m, L.red);
  };

  // step 0 (eq. (3), then eqs. (5)-(6) with G_0 = [N] and M_0 = (1/N) 1)
  const T m0 = (T)(1.0 / (double)n);
  double accT = 0.0, accM = 0.0;
  for (int i = tid; i < n; i += NT) {
    if (HK == 0) {
      H64[i] = (double)m0;
    } else {
      Hhi[i] = (float)m0;
      Hlo[i] = 0.0f;
    }
    accM += (double)m0;
    accT += deg(i) > 0 ? (1.0 - c) * (double)m0 : (double)m0;
  }
  const Red4 s0 = block_sum4<NW>(Red4{accT, accM, 0, 0}, L.red);
  double hsum = s0.b, hnorm = s0.b;
  long long edges = cd.nnz;
  // a link outside [0, n) sends nothing and is reported
  auto in_range = [&](int j) -> bool {
    const bool ok = (unsigned)j < (unsigned)n;
    if (!ok) s_bad = 1;
    return ok;
  };
  route([&](int j) -> double { return in_range(j) ? (double)m0 : 0.0; },
        [&](int) -> double { return -(double)m0; }, s0.a / (double)n, Ca);
  T *cur = Ca, *oth = Cb;
  long long t = 1, refreshed = -1;
  int status = 0, green_steps = 0;
  double resid = 0.0;

  for (;;) {
    resid = l1 / fabs(hsum);
    if (s_bad) { status = ST_BAD_GRAPH; break; }
    if (!isfinite(l1) || !isfinite(hsum)) { status = ST_NONFINITE; break; }
    if (fabs(hsum) <= 1e-300 || fabs(hsum) <= 1e-12 * hnorm) { status = ST_ZERO_HISTORY; break; }
    // the rounding of FP32 cash leaves C_t 1 != 0; once that drift is half of
    // ||C_t||_1 the cash is rebuilt from the history, as before a stop
    const bool drift = fabs(cs) > 0.5 * l1 && l1 > 0.0;
    if ((t >= 2 && resid < cd.eps) || (drift && b.refresh && refreshed != t)) {
      if (b.refresh && refreshed != t) {
        // confirm the stop on C_t = H_t P - H_t (eq. (7) with C_0 = 0), in FP64
        double pool = 0.0;
        for (int i = tid; i < n; i += NT) pool += hist(i) * (deg(i) > 0 ? 1.0 - c : 1.0);
        pool = block_sum1<NW>(pool, L.red);
        route([&](int j) -> double { return in_range(j) ? hist(j) : 0.0; },
              [&](int kk) -> double { return -hist(kk); }, pool / (double)n, oth);
        T *tmp = cur;
        cur = oth;
        oth = tmp;
        refreshed = t;
        continue;
      }
      status = ST_CONVERGED;
      break;
    }
    if (t - 1 >= b.max_steps) { status = ST_LIMIT; break; }
    double theta = 0.0;
    if (b.sched == SCHED_THRESHOLD) theta = (rr == 1.0) ? l1 / (double)n : pow(sr / (double)n, 1.0 / rr);
    const double maxabs = mx;
    const int sched = b.sched;
    auto green = [&](T v) -> bool { return is_green(v, 0, sched, theta, maxabs, 0.0, -1); };
    // select (eqs. (4)-(5)): H += M for the green nodes, pool and moved mass
    double aT = 0.0, aM = 0.0, aD = 0.0, aE = 0.0;
    for (int i = tid; i < n; i += NT) {
      const T x = cur[i];
      if (x != T(0) && green(x)) {
        const int dg = deg(i);
        if (HK == 0) {
          const double h = H64[i], hn = h + (double)x;
          H64[i] = hn;
          aD += fabs(hn) - fabs(h);
        } else {
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
      }
    }
    const Red4 s1 = block_sum4<NW>(Red4{aT, aM, aD, aE}, L.red);
    hsum += s1.b;
    hnorm += s1.c;
    edges += (long long)s1.d;
    ++green_steps;
    // route (eq. (6)) by the CSC gather, M_j recomputed from the snapshot
    const T *cc = cur;
    route([&](int j) -> double {
            if (!in_range(j)) return 0.0;
            const T v = cc[j];
            return green(v) ? (double)v : 0.0;
          },
          [&](int kk) -> double {
            const T v = cc[kk];
            return green(v) ? 0.0 : (double)v;
          },
          s1.a / (double)n, oth);
    T *tmp = cur;
    cur = oth;
    oth = tmp;
    ++t;
  }
  if (status != ST_NONFINITE && status != ST_BAD_GRAPH && hsum != 0.0)
    for (int i = tid; i < n; i += NT) b.pi[cd.node_off + i] = hist(i) / hsum;  // eq. (2)
  if (tid == 0) {
    ChainOut o;
    o.t = t;
    o.edges = edges;
    o.resid = resid;
    o.hsum = hsum;
    o.status = status;
    o.green_steps = green_steps;
    o.t0 = t_start;
    o.t1 = wall_clock64();
    b.out[k] = o;
  }
}

template <class T, int HK, int NT>
__global__ __launch_bounds__(NT) void k_batch(BatchDev b) {
  __shared__ ColLds<NT> L;
  __shared__ int sh_k;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) sh_k = (int)atomicAdd(b.queue, 1u);
    __syncthreads();
    const int q = sh_k;
    if (q >= b.n_chains) break;
    batch_chain<T, HK, NT>(b, b.order[q], L);
  }
}

__global__ void k_batch_reset(unsigned int *queue) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *queue = 0u;
}

template __global__ void k_batch<float, 0, 256>(BatchDev);
template __global__ void k_batch<float, 0, 512>(BatchDev);
template __global__ void k_batch<float, 0, 1024>(BatchDev);
template __global__ void k_batch<float, 1, 256>(BatchDev);
template __global__ void k_batch<float, 1, 512>(BatchDev);
template __global__ void k_batch<float, 1, 1024>(BatchDev);
template __global__ void k_batch<double, 0, 256>(BatchDev);
template __global__ void k_batch<double, 0, 512>(BatchDev);
template __global__ void k_batch<double, 0, 1024>(BatchDev);

}  // namespace rlgl
