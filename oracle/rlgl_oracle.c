/*
 * Reference oracle for the Red-Light-Green-Light (RLGL) method of
 * Avrachenkov, Brown and Litvak, "Red Light Green Light Method for Solving
 * Large Markov Chains" (J. Sci. Comput. 93:18, 2022; arXiv 2008.02710).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, serial, FP64 statement of
 * what the method computes.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header, table
 * or helper with the HIP library, and the HIP library never calls it.
 *
 * Every function follows the paper's notation:
 *   N states, transition matrix P (row-stochastic), cash C_t, moved cash M_t,
 *   history H_t, green set G_t, estimate pi_hat_t = H_t / (H_t 1).
 *
 * The chain.  The caller gives the link matrix W as CSR (rowptr/col/val) and a
 * damping factor c in (0,1].  The transition matrix is the Google matrix of
 * Sec. 3.2 (the PageRank example after the Dobrushin coefficient),
 *     P = c W + (1-c)/N 1 1^T,
 * and a row of W with no stored entry (a dangling node; the paper is silent
 * about them) is read as the uniform row 1/N.  Duplicate (i,j) entries add up.
 * val == NULL means every stored entry of row i weighs 1/outdeg(i).
 *
 * Readings of the paper taken here (each one is listed with its reason in the
 * design notes of the repository):
 *   - M_0 is uniform 1/N unless the caller passes another M_0 (Sec. 2.1).
 *   - all green moves of a step use the cash snapshot C_t (eq. (4)-(6)).
 *   - the stop test is the one of Algorithm 1, step (7), applied for t >= 2:
 *     ||C_t||_1 / |H_t 1| < eps.
 *   - RLGL_MaxC (Sec. 6) greens every node whose |C| equals max_j |C_j|.
 *   - the threshold rule of RLGL_Theta (Sec. 6) is applied to all nodes at
 *     once: G_t = { i : |C_t,i| >= theta_t }, theta_t = (sum_j |C_t,j|^r / N)^(1/r)
 *     recomputed every theta_period steps.
 *   - top-k (not in the paper) orders by |C| descending, then node id ascending.
 *   - RLGL_PC (Sec. 6) is drawn for all nodes at once: node i is green with
 *     probability |C_t,i| / max_j |C_t,j|, its uniform draw taken from
 *     splitmix64 at counter t 2^32 + i (the synchronous form of the Poisson
 *     clock the paper mentions, normalised by the largest cash).
 *   - H_t 1 counts as zero when |H_t 1| <= 1e-300 or |H_t 1| <= 1e-12 ||H_t||_1
 *     (the restart case of Sec. 2.1 and Example 1).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_ALL = 0, ORC_THRESHOLD = 1, ORC_TOPK = 2, ORC_MAXC = 3, ORC_PC = 4 };
enum {
  ORC_OK = 0,
  ORC_EINVAL = -1,
  ORC_ENOMEM = -2,
  ORC_EZERO_HISTORY = -4,
  ORC_ENOT_CONVERGED = -5,
  ORC_ENONFINITE = -6
};

typedef struct {
  int32_t n;
  const int64_t *rowptr; /* n+1 entries */
  const int32_t *col;    /* rowptr[n] entries */
  const double *val;     /* rowptr[n] entries, or NULL for 1/outdeg */
  double c;              /* damping, 0 < c <= 1 */
} orc_chain;

typedef struct {
  int64_t t;            /* index of the final state C_t, H_t */
  int64_t steps;        /* green-light steps taken after step 0 */
  int64_t green_total;  /* sum over steps t >= 1 of |G_t| */
  int64_t edges_pushed; /* stored links of green nodes that moved non-zero cash, step 0 included */
  double l1_cash;       /* ||C_t||_1 */
  double h_sum;         /* H_t 1 */
  double resid;         /* ||C_t||_1 / |H_t 1| */
  double theta;         /* last threshold used (THRESHOLD), else 0 */
  double cash_sum;      /* C_t 1 */
  int32_t status;
} orc_info;

static int64_t outdeg(const orc_chain *ch, int32_t i) { return ch->rowptr[i + 1] - ch->rowptr[i]; }

/* out += M P, with P the chain described above.  This is the product M_t P of
 * the cash recursion (eq. (6)): each node i splits M_i into c*W_ij*M_i along
 * its stored links and (1-c)*M_i into the uniform restart; a dangling node
 * sends all of M_i to the uniform restart. */
void orc_route(const orc_chain *ch, const double *M, double *out) {
  const int32_t n = ch->n;
  double pool = 0.0;
  for (int32_t i = 0; i < n; ++i) {
    const double m = M[i];
    if (m == 0.0) continue;
    const int64_t d = outdeg(ch, i);
    if (d == 0) {
      pool += m;
      continue;
    }
    for (int64_t e = ch->rowptr[i]; e < ch->rowptr[i + 1]; ++e) {
      const double w = ch->val ? ch->val[e] : 1.0 / (double)d;
      out[ch->col[e]] += ch->c * w * m;
    }
    pool += (1.0 - ch->c) * m;
  }
  const double share = pool / (double)n;
  for (int32_t j = 0; j < n; ++j) out[j] += share;
}

/* Threshold of RLGL_Theta (Sec. 6): the power mean of order r of |C_t|. */
double orc_theta(int32_t n, const double *C, double r) {
  double s = 0.0;
  if (r == 1.0) {
    for (int32_t j = 0; j < n; ++j) s += fabs(C[j]);
    return s / (double)n;
  }
  for (int32_t j = 0; j < n; ++j) s += pow(fabs(C[j]), r);
  return pow(s / (double)n, 1.0 / r);
}

/* qsort comparator for top-k: |C| descending, then id ascending. */
static const double *g_topk_c;
static int topk_cmp(const void *a, const void *b) {
  const int32_t i = *(const int32_t *)a, j = *(const int32_t *)b;
  const double ai = fabs(g_topk_c[i]), aj = fabs(g_topk_c[j]);
  if (ai > aj) return -1;
  if (ai < aj) return 1;
  return (i < j) ? -1 : (i > j);
}

/* splitmix64 (Steele, Lea and Flood, OOPSLA 2014): output number `index`
 * (0-based) of the generator whose state starts at `seed` and advances by the
 * golden gamma 0x9E3779B97F4A7C15 before each output. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t index) {
  uint64_t z = seed + (index + 1u) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* RLGL_PC (Sec. 6) with every node drawn at once: node i is green at step t
 * with probability |C_t,i| / max_j |C_t,j|.  Its uniform draw is
 * u = (splitmix64 output number t 2^32 + i, shifted right by 11) 2^-53, and it
 * is green iff u < |C_t,i| / max_j |C_t,j| (both in FP64).  A node of maximal
 * |C| is always green; zero cash never is. */
int64_t orc_select_pc(int32_t n, const double *C, uint64_t seed, int64_t t, uint8_t *mask) {
  double mx = 0.0;
  int64_t cnt = 0;
  for (int32_t i = 0; i < n; ++i)
    if (fabs(C[i]) > mx) mx = fabs(C[i]);
  for (int32_t i = 0; i < n; ++i) {
    mask[i] = 0;
    if (mx > 0.0) {
      const uint64_t z = orc_splitmix64(seed, ((uint64_t)t << 32) + (uint64_t)i);
      const double u = (double)(z >> 11) * 0x1.0p-53;
      mask[i] = u < fabs(C[i]) / mx;
    }
    cnt += mask[i];
  }
  return cnt;
}

/* Green-light set G_t chosen from the cash snapshot C_t.  Writes mask[i] in
 * {0,1} and returns |G_t|.  theta is used by ORC_THRESHOLD only, k by
 * ORC_TOPK only.  Returns -1 on a bad argument. */
int64_t orc_select(int32_t n, const double *C, int32_t sched, double theta, int64_t k, uint8_t *mask) {
  int64_t cnt = 0;
  if (sched == ORC_ALL) {
    for (int32_t i = 0; i < n; ++i) mask[i] = 1;
    return n;
  }
  if (sched == ORC_THRESHOLD) {
    for (int32_t i = 0; i < n; ++i) {
      mask[i] = fabs(C[i]) >= theta;
      cnt += mask[i];
    }
    return cnt;
  }
  if (sched == ORC_MAXC) {
    double mx = 0.0;
    for (int32_t i = 0; i < n; ++i)
      if (fabs(C[i]) > mx) mx = fabs(C[i]);
    for (int32_t i = 0; i < n; ++i) {
      mask[i] = fabs(C[i]) == mx;
      cnt += mask[i];
    }
    return cnt;
  }
  if (sched == ORC_TOPK) {
    if (k < 1) return -1;
    int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!idx) return -1;
    for (int32_t i = 0; i < n; ++i) idx[i] = i;
    g_topk_c = C;
    qsort(idx, (size_t)n, sizeof(int32_t), topk_cmp);
    memset(mask, 0, (size_t)n);
    for (int64_t q = 0; q < k && q < n; ++q) mask[idx[q]] = 1;
    free(idx);
    return k < n ? k : n;
  }
  return -1;
}

/* Step 0 of Algorithm 1 (eq. (3), then eqs. (5) and (6) with G_0 = [N]):
 * C_0 = 0, H_0 = 0, H_1 = M_0, C_1 = C_0 - M_0 + M_0 P.
 * M0 == NULL means the uniform M_0 = (1/N) 1.  Writes C = C_1, H = H_1 and
 * returns H_1 1 in *hsum; *edges gets the links used by step 0. */
void orc_init(const orc_chain *ch, const double *M0, double *C, double *H, double *hsum, int64_t *edges) {
  const int32_t n = ch->n;
  double s = 0.0;
  int64_t e = 0;
  for (int32_t i = 0; i < n; ++i) {
    const double m = M0 ? M0[i] : 1.0 / (double)n;
    H[i] = m;
    C[i] = -m;
    s += m;
    if (m != 0.0) e += outdeg(ch, i);
  }
  orc_route(ch, H, C); /* H_1 = M_0 at this point */
  *hsum = s;
  *edges = e;
}

/* One step t >= 1 (eqs. (4)-(6)) for the green set in mask:
 * M_t = C_t I(G_t), H_{t+1} = H_t + M_t, C_{t+1} = C_t - M_t + M_t P.
 * M is caller scratch of n doubles.  Returns sum_i M_t,i through *msum and
 * adds the links used to *edges. */
void orc_step(const orc_chain *ch, const uint8_t *mask, double *C, double *H, double *hsum, int64_t *edges,
              double *M) {
  const int32_t n = ch->n;
  double s = 0.0;
  int64_t e = 0;
  for (int32_t i = 0; i < n; ++i) {
    M[i] = mask[i] ? C[i] : 0.0;
    if (M[i] != 0.0) e += outdeg(ch, i);
  }
  for (int32_t i = 0; i < n; ++i) {
    H[i] += M[i];
    C[i] -= M[i];
    s += M[i];
  }
  orc_route(ch, M, C);
  *hsum += s;
  *edges += e;
}

static double l1norm(int32_t n, const double *x) {
  double s = 0.0;
  for (int32_t i = 0; i < n; ++i) s += fabs(x[i]);
  return s;
}

/* Algorithm 1 run to its stop test.  Returns the status; pi_out (n doubles)
 * receives pi_hat_t = H_t / (H_t 1) whenever H_t 1 is usable.  C_out and H_out
 * (n doubles each, may be NULL) receive the final C_t and H_t. */
int32_t orc_solve(const orc_chain *ch, const double *M0, int32_t sched, double r, int64_t k, int32_t theta_period,
                  double eps, int64_t max_steps, uint64_t seed, double *pi_out, double *C_out, double *H_out,
                  orc_info *info) {
  const int32_t n = ch->n;
  if (n <= 0 || !(ch->c > 0.0 && ch->c <= 1.0) || theta_period < 1 || !(r >= 1.0)) return ORC_EINVAL;
  double *C = (double *)malloc(sizeof(double) * (size_t)n);
  double *H = (double *)malloc(sizeof(double) * (size_t)n);
  double *M = (double *)malloc(sizeof(double) * (size_t)n);
  uint8_t *mask = (uint8_t *)malloc((size_t)n);
  if (!C || !H || !M || !mask) {
    free(C); free(H); free(M); free(mask);
    return ORC_ENOMEM;
  }
  double hsum = 0.0, theta = 0.0, l1 = 0.0, resid = 0.0;
  int64_t edges = 0, green_total = 0, t = 1;
  int32_t status = ORC_OK;
  orc_init(ch, M0, C, H, &hsum, &edges);
  for (;;) {
    l1 = l1norm(n, C);
    const double hn = l1norm(n, H);
    if (!isfinite(l1) || !isfinite(hsum)) { status = ORC_ENONFINITE; break; }
    if (fabs(hsum) <= 1e-300 || fabs(hsum) <= 1e-12 * hn) { status = ORC_EZERO_HISTORY; break; }
    resid = l1 / fabs(hsum);
    if (t >= 2 && resid < eps) { status = ORC_OK; break; }
    if (t - 1 >= max_steps) { status = ORC_ENOT_CONVERGED; break; }
    if (sched == ORC_THRESHOLD && (t - 1) % theta_period == 0) theta = orc_theta(n, C, r);
    const int64_t g = (sched == ORC_PC) ? orc_select_pc(n, C, seed, t, mask) : orc_select(n, C, sched, theta, k, mask);
    if (g < 0) { status = ORC_EINVAL; break; }
    green_total += g;
    orc_step(ch, mask, C, H, &hsum, &edges, M);
    ++t;
  }
  if (pi_out && status != ORC_EINVAL && hsum != 0.0 && isfinite(hsum))
    for (int32_t i = 0; i < n; ++i) pi_out[i] = H[i] / hsum;
  if (C_out) memcpy(C_out, C, sizeof(double) * (size_t)n);
  if (H_out) memcpy(H_out, H, sizeof(double) * (size_t)n);
  if (info) {
    double cs = 0.0;
    for (int32_t i = 0; i < n; ++i) cs += C[i];
    info->t = t;
    info->steps = t - 1;
    info->green_total = green_total;
    info->edges_pushed = edges;
    info->l1_cash = l1;
    info->h_sum = hsum;
    info->resid = resid;
    info->theta = (sched == ORC_THRESHOLD) ? theta : 0.0;
    info->cash_sum = cs;
    info->status = status;
  }
  free(C); free(H); free(M); free(mask);
  return status;
}

/* Power iteration, the reference method of Sec. 6 and the all-green special
 * case of Sec. 2.3.1: x_0 = (1/N) 1, x_{k+1} = x_k P, stopped when
 * ||x_{k+1} - x_k||_1 <= tol.  x_out receives the last iterate. */
int32_t orc_power_iteration(const orc_chain *ch, double tol, int64_t max_iter, double *x_out, int64_t *iters) {
  const int32_t n = ch->n;
  if (n <= 0) return ORC_EINVAL;
  double *x = (double *)malloc(sizeof(double) * (size_t)n);
  double *y = (double *)malloc(sizeof(double) * (size_t)n);
  if (!x || !y) { free(x); free(y); return ORC_ENOMEM; }
  for (int32_t i = 0; i < n; ++i) x[i] = 1.0 / (double)n;
  int32_t status = ORC_ENOT_CONVERGED;
  int64_t it = 0;
  while (it < max_iter) {
    memset(y, 0, sizeof(double) * (size_t)n);
    orc_route(ch, x, y);
    ++it;
    double d = 0.0;
    for (int32_t i = 0; i < n; ++i) d += fabs(y[i] - x[i]);
    double *tmp = x; x = y; y = tmp;
    if (!isfinite(d)) { status = ORC_ENONFINITE; break; }
    if (d <= tol) { status = ORC_OK; break; }
  }
  memcpy(x_out, x, sizeof(double) * (size_t)n);
  if (iters) *iters = it;
  free(x); free(y);
  return status;
}

/* Algorithm 2 (Gauss-Southwell for PageRank, GSo-PR, Sec. 2.4), the
 * positive-cash special case of RLGL: C_1 = (1-c) s, H_1 = 0; step t moves the
 * largest cash C_t,k (ties: the smallest k) along c P,
 *   H_{t+1} = H_t + C_t,k e_k,  C_{t+1} = C_t - C_t,k e_k (I - c P),
 * until ||C_t||_1 < eps (t >= 2).  P is the chain's link matrix W (a row with
 * no stored link is uniform); the restart is carried by s (uniform when NULL).
 * pi_hat_t = H_t.  Writes H_t and C_t, *steps gets the moves made and *edges the
 * links they used. */
int32_t orc_gso_pr(const orc_chain *ch, const double *s, double eps, int64_t max_steps, double *H, double *C,
                   int64_t *steps, int64_t *edges) {
  const int32_t n = ch->n;
  if (n <= 0 || !(ch->c > 0.0 && ch->c < 1.0)) return ORC_EINVAL;
  const double c = ch->c;
  for (int32_t i = 0; i < n; ++i) {
    C[i] = (1.0 - c) * (s ? s[i] : 1.0 / (double)n);
    H[i] = 0.0;
  }
  int64_t t = 1, e = 0;
  int32_t status = ORC_ENOT_CONVERGED;
  for (;;) {
    const double l1 = l1norm(n, C);
    if (!isfinite(l1)) { status = ORC_ENONFINITE; break; }
    if (t >= 2 && l1 < eps) { status = ORC_OK; break; }
    if (t - 1 >= max_steps) break;
    int32_t k = 0;
    for (int32_t i = 1; i < n; ++i)
      if (C[i] > C[k]) k = i;
    const double m = C[k];
    H[k] += m;
    C[k] -= m;
    const int64_t d = outdeg(ch, k);
    if (d == 0) {
      for (int32_t j = 0; j < n; ++j) C[j] += c * m / (double)n;
    } else {
      for (int64_t q = ch->rowptr[k]; q < ch->rowptr[k + 1]; ++q)
        C[ch->col[q]] += c * m * (ch->val ? ch->val[q] : 1.0 / (double)d);
      e += d;
    }
    ++t;
  }
  if (steps) *steps = t - 1;
  if (edges) *edges = e;
  return status;
}

/* The same power iteration with its product x P taken column by column on
 * every host core (OpenMP): a CPU baseline, not a reference.  It builds the
 * transpose of W once; each y_k = c sum_j x_j W_jk + pool / N, the pool as in
 * orc_route.  *threads_used receives the thread count. */
int32_t orc_power_iteration_omp(const orc_chain *ch, double tol, int64_t max_iter, double *x_out, int64_t *iters,
                                int32_t *threads_used) {
  const int32_t n = ch->n;
  if (n <= 0) return ORC_EINVAL;
  const int64_t m = ch->rowptr[n];
  int64_t *cp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  int32_t *rw = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
  double *wv = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
  double *x = (double *)malloc(sizeof(double) * (size_t)n);
  double *y = (double *)malloc(sizeof(double) * (size_t)n);
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  if (!cp || !rw || !wv || !x || !y || !fill) {
    free(cp); free(rw); free(wv); free(x); free(y); free(fill);
    return ORC_ENOMEM;
  }
  for (int64_t e = 0; e < m; ++e) cp[ch->col[e] + 1] += 1;
  for (int32_t k = 0; k < n; ++k) cp[k + 1] += cp[k];
  for (int32_t k = 0; k < n; ++k) fill[k] = cp[k];
  for (int32_t i = 0; i < n; ++i) {
    const int64_t d = outdeg(ch, i);
    for (int64_t e = ch->rowptr[i]; e < ch->rowptr[i + 1]; ++e) {
      const int64_t q = fill[ch->col[e]]++;
      rw[q] = i;
      wv[q] = ch->val ? ch->val[e] : 1.0 / (double)d;
    }
  }
  for (int32_t i = 0; i < n; ++i) x[i] = 1.0 / (double)n;
  int32_t status = ORC_ENOT_CONVERGED;
  int64_t it = 0;
  int32_t used = 1;
  const double c = ch->c;
  while (it < max_iter) {
    double pool = 0.0;
#pragma omp parallel for reduction(+ : pool) schedule(static)
    for (int32_t i = 0; i < n; ++i) pool += (outdeg(ch, i) > 0 ? 1.0 - c : 1.0) * x[i];
    const double share = pool / (double)n;
    double d = 0.0;
#pragma omp parallel for reduction(+ : d) schedule(dynamic, 4096)
    for (int32_t k = 0; k < n; ++k) {
      double acc = 0.0;
      for (int64_t q = cp[k]; q < cp[k + 1]; ++q) acc += x[rw[q]] * wv[q];
      y[k] = c * acc + share;
      d += fabs(y[k] - x[k]);
    }
#pragma omp parallel
    {
#pragma omp single
      used = omp_get_num_threads();
    }
    ++it;
    double *tmp = x; x = y; y = tmp;
    if (!isfinite(d)) { status = ORC_ENONFINITE; break; }
    if (d <= tol) { status = ORC_OK; break; }
  }
  memcpy(x_out, x, sizeof(double) * (size_t)n);
  if (iters) *iters = it;
  if (threads_used) *threads_used = used;
  free(cp); free(rw); free(wv); free(x); free(y); free(fill);
  return status;
}

/* ||pi - pi P||_1, the residual of Sec. 6 ("until ||pi_t - pi_t P||_1 < eps"). */
double orc_residual(const orc_chain *ch, const double *pi) {
  const int32_t n = ch->n;
  double *y = (double *)calloc((size_t)n, sizeof(double));
  if (!y) return NAN;
  orc_route(ch, pi, y);
  double s = 0.0;
  for (int32_t i = 0; i < n; ++i) s += fabs(pi[i] - y[i]);
  free(y);
  return s;
}
