/*
 * Seeded synthetic graph generators and sparse-layout builders.
 *
 * This file holds no arithmetic of the RLGL method: it only draws random
 * graphs and lays them out as CSR (out-links) and CSC (in-links).  Both the
 * reference oracle and the HIP library are fed from what it produces.
 *
 * Randomness is counter-based: every draw is splitmix64 applied to
 * (stream key, counter), so results are independent of the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}
static inline uint64_t stream_key(uint64_t seed, uint64_t stream) {
  return mix64(mix64(seed + 0x632be59bd9b4e019ULL) ^ (stream * 0x9e3779b97f4a7c15ULL + 0x1234567ULL));
}
static inline uint64_t draw(uint64_t key, uint64_t i) { return mix64(key + (i + 1) * 0x9e3779b97f4a7c15ULL); }
static inline double unit53(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }

/* out[i] = Poisson(lam) + add, one inverse-transform draw per node. */
void wl_poisson(int64_t n, double lam, int32_t add, uint64_t seed, uint64_t stream, int32_t *out) {
  const uint64_t key = stream_key(seed, stream);
  const double p0 = exp(-lam);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    const double u = unit53(draw(key, (uint64_t)i));
    double p = p0, F = p0;
    int32_t k = 0;
    while (u > F && k < 100000) {
      ++k;
      p *= lam / (double)k;
      F += p;
      if (p == 0.0) break;
    }
    out[i] = k + add;
  }
}

/* out[e] uniform in [0, n) */
void wl_uniform_int(int64_t m, int64_t n, uint64_t seed, uint64_t stream, int32_t *out) {
  const uint64_t key = stream_key(seed, stream);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    const uint64_t x = draw(key, (uint64_t)e);
    out[e] = (int32_t)(((x >> 32) * (uint64_t)n) >> 32);
  }
}

/* out[e] uniform doubles in [0,1) */
void wl_uniform01(int64_t m, uint64_t seed, uint64_t stream, double *out) {
  const uint64_t key = stream_key(seed, stream);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) out[e] = unit53(draw(key, (uint64_t)e));
}

/* m draws from the distribution whose cumulative sums (non-decreasing,
 * cdf[nw-1] > 0) are given: index of the first cdf entry above u*cdf[nw-1]. */
void wl_categorical(int64_t nw, const double *cdf, int64_t m, uint64_t seed, uint64_t stream, int32_t *out) {
  const uint64_t key = stream_key(seed, stream);
  const double total = cdf[nw - 1];
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    const double u = unit53(draw(key, (uint64_t)e)) * total;
    int64_t lo = 0, hi = nw - 1;
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if (cdf[mid] > u) hi = mid; else lo = mid + 1;
    }
    out[e] = (int32_t)lo;
  }
}

/* Uniform random permutation of 0..n-1 (Fisher-Yates, serial). */
void wl_permutation(int64_t n, uint64_t seed, uint64_t stream, int32_t *perm) {
  const uint64_t key = stream_key(seed, stream);
  for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
  for (int64_t i = n - 1; i > 0; --i) {
    const uint64_t x = draw(key, (uint64_t)i);
    const int64_t j = (int64_t)(((x >> 32) * (uint64_t)(i + 1)) >> 32);
    const int32_t t = perm[i];
    perm[i] = perm[j];
    perm[j] = t;
  }
}

/* R-MAT edges (Graph500 style, no noise): each of `scale` levels picks a
 * quadrant with probabilities (a, b, c, 1-a-b-c); quadrant b sets the
 * destination bit, c the source bit, d both.  Two 32-bit uniforms per draw. */
void wl_rmat(int32_t scale, int64_t m, double a, double b, double c, uint64_t seed, uint64_t stream,
             int32_t *src, int32_t *dst) {
  const uint64_t key = stream_key(seed, stream);
  const double ab = a + b, abc = a + b + c;
  const int64_t per_edge = (scale + 1) / 2;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    uint32_t s = 0, d = 0;
    for (int32_t lev = 0; lev < scale; ++lev) {
      const uint64_t x = draw(key, (uint64_t)(e * per_edge + lev / 2));
      const uint32_t half = (lev & 1) ? (uint32_t)(x >> 32) : (uint32_t)x;
      const double u = (double)half * (1.0 / 4294967296.0);
      uint32_t sb, db;
      if (u < a) { sb = 0; db = 0; }
      else if (u < ab) { sb = 0; db = 1; }
      else if (u < abc) { sb = 1; db = 0; }
      else { sb = 1; db = 1; }
      s = (s << 1) | sb;
      d = (d << 1) | db;
    }
    src[e] = (int32_t)s;
    dst[e] = (int32_t)d;
  }
}

/* x[e] = perm[x[e]] */
void wl_relabel(int64_t m, const int32_t *perm, int32_t *x) {
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) x[e] = perm[x[e]];
}

/* Stable counting sort of an edge list by `key`: ptr[n+1] gets the segment
 * offsets, other[] the second endpoint in segment order, and order[] (if not
 * NULL) the original edge index.  Edges keep their input order inside a
 * segment. */
int wl_bucket(int64_t n, int64_t m, const int32_t *key, const int32_t *other, int64_t *ptr, int32_t *other_out,
              int64_t *order) {
  memset(ptr, 0, sizeof(int64_t) * (size_t)(n + 1));
  for (int64_t e = 0; e < m; ++e) {
    const int32_t k = key[e];
    if (k < 0 || k >= n) return -1;
    ptr[k + 1]++;
  }
  for (int64_t i = 0; i < n; ++i) ptr[i + 1] += ptr[i];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  if (!fill) return -2;
  memcpy(fill, ptr, sizeof(int64_t) * (size_t)n);
  for (int64_t e = 0; e < m; ++e) {
    const int64_t p = fill[key[e]]++;
    other_out[p] = other[e];
    if (order) order[p] = e;
  }
  free(fill);
  return 0;
}

/* CSR -> CSC: colptr[n+1], row[nnz] (source of each in-link) and perm[nnz]
 * (position of that link in the CSR arrays), stable in CSR order. */
int wl_transpose(int64_t n, const int64_t *rowptr, const int32_t *col, int64_t *colptr, int32_t *row,
                 int64_t *perm) {
  const int64_t m = rowptr[n];
  memset(colptr, 0, sizeof(int64_t) * (size_t)(n + 1));
  for (int64_t e = 0; e < m; ++e) {
    if (col[e] < 0 || col[e] >= n) return -1;
    colptr[col[e] + 1]++;
  }
  for (int64_t i = 0; i < n; ++i) colptr[i + 1] += colptr[i];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  if (!fill) return -2;
  memcpy(fill, colptr, sizeof(int64_t) * (size_t)n);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      const int64_t p = fill[col[e]]++;
      row[p] = (int32_t)i;
      perm[p] = e;
    }
  free(fill);
  return 0;
}
