// Debug check of a chain's arrays before a solve.  The method needs P to be a
// stochastic matrix (Sec. 2: the rows of W sum to one), the CSR to describe
// W, and the CSC, when given, to be the transpose of the same links.  Every
// read below is bounds-checked against n and nnz, so arrays that break the
// contract are reported, never followed out of range.
#include "rlgl_device.h"

namespace rlgl {

enum : unsigned int {
  VF_ROWPTR = 1u,        // csr_rowptr not non-decreasing from 0 to nnz
  VF_COL = 2u,           // a csr_col outside [0, n)
  VF_VAL = 4u,           // a csr_val negative or non-finite
  VF_ROWSUM = 8u,        // a row with links whose values do not sum to 1
  VF_COLPTR = 16u,       // csc_colptr not non-decreasing from 0 to nnz
  VF_ROW = 32u,          // a csc_row outside [0, n)
  VF_INDEG = 64u,        // a column's CSC length differs from its CSR in-degree
  VF_CVAL = 128u,        // a csc_val negative or non-finite
};

struct alignas(256) VHead {
  unsigned int flags;
  unsigned int pad;
  unsigned long long dev_bits;  // max |row sum - 1| as the bits of a non-negative double
  unsigned long long h_csr;     // sum of link hashes over the CSR
  unsigned long long h_csc;     // the same over the CSC
};

// Hash of a link (i, j) and the bit pattern of its value (0 when values are
// not compared): the splitmix64 finaliser of the packed pair, offset by the value.
__device__ __forceinline__ unsigned long long link_hash(unsigned int i, unsigned int j, unsigned long long vb) {
  unsigned long long z = (((unsigned long long)i << 32) | j) + vb * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <class V>
__device__ __forceinline__ unsigned long long value_bits(V v) {
  if (sizeof(V) == 8) return (unsigned long long)__double_as_longlong((double)v);
  return (unsigned long long)(unsigned int)__float_as_uint((float)v);
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}
__device__ __forceinline__ unsigned int wave_or(unsigned int x) {
  for (int o = 32; o > 0; o >>= 1) x |= __shfl_xor(x, o, 64);
  return x;
}

__device__ __forceinline__ void vhead_fold(VHead *h, unsigned int fl, double dev, unsigned long long hs, bool csc) {
  fl = wave_or(fl);
  dev = wave_max(dev);
  hs = wave_sum_u64(hs);
  if ((threadIdx.x & 63) == 0) {
    if (fl) atomicOr(&h->flags, fl);
    if (dev > 0.0) atomic_max_nonneg(&h->dev_bits, dev);
    if (hs) atomicAdd(csc ? &h->h_csc : &h->h_csr, hs);
  }
}

__global__ __launch_bounds__(BLOCK) void k_v_clear(VHead *h, int *indeg, int n) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *h = VHead{};
  for (int i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) indeg[i] = 0;
}

// One thread per row: structure, value range, row sum, in-degree histogram,
// link hashes.
template <class V>
__global__ __launch_bounds__(BLOCK) void k_v_rows(int n, long long nnz, const int *rowptr, const int *col,
                                                   const V *val, int hash_vals, double tol, VHead *h, int *indeg) {
  unsigned int fl = 0;
  double dev = 0.0;
  unsigned long long hs = 0;
  for (int i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) {
    const long long a = rowptr[i], b = rowptr[i + 1];
    if ((i == 0 && a != 0) || (i == n - 1 && b != nnz) || a > b || a < 0 || b > nnz) {
      fl |= VF_ROWPTR;
      continue;
    }
    double sum = 0.0;
    for (long long e = a; e < b; ++e) {
      const int j = col[e];
      unsigned long long vb = 0;
      if (val) {
        const double v = (double)val[e];
        if (!(v >= 0.0) || !isfinite(v)) fl |= VF_VAL;
        sum += v;
        if (hash_vals) vb = value_bits(val[e]);
      }
      if ((unsigned)j >= (unsigned)n) {
        fl |= VF_COL;
        continue;
      }
      atomicAdd(&indeg[j], 1);
      hs += link_hash((unsigned)i, (unsigned)j, vb);
    }
    if (val && b > a) {
      const double d = fabs(sum - 1.0);
      if (!(d <= tol)) fl |= VF_ROWSUM;
      dev = fmax(dev, isfinite(d) ? d : 1e300);
    }
  }
  vhead_fold(h, fl, dev, hs, false);
}

// One thread per column: structure, in-degree against the CSR histogram,
// value range, link hashes.
template <class V>
__global__ __launch_bounds__(BLOCK) void k_v_cols(int n, long long nnz, const int *colptr, const int *crow,
                                                   const V *cval, int hash_vals, VHead *h, const int *indeg) {
  unsigned int fl = 0;
  unsigned long long hs = 0;
  for (int k = blockIdx.x * BLOCK + threadIdx.x; k < n; k += gridDim.x * BLOCK) {
    const long long a = colptr[k], b = colptr[k + 1];
    if ((k == 0 && a != 0) || (k == n - 1 && b != nnz) || a > b || a < 0 || b > nnz) {
      fl |= VF_COLPTR;
      continue;
    }
    if (b - a != (long long)indeg[k]) fl |= VF_INDEG;
    for (long long e = a; e < b; ++e) {
      const int i = crow[e];
      unsigned long long vb = 0;
      if (cval) {
        const double v = (double)cval[e];
        if (!(v >= 0.0) || !isfinite(v)) fl |= VF_CVAL;
        if (hash_vals) vb = value_bits(cval[e]);
      }
      if ((unsigned)i >= (unsigned)n) {
        fl |= VF_ROW;
        continue;
      }
      hs += link_hash((unsigned)i, (unsigned)k, vb);
    }
  }
  vhead_fold(h, fl, 0.0, hs, true);
}

template __global__ void k_v_rows<float>(int, long long, const int *, const int *, const float *, int, double,
                                         VHead *, int *);
template __global__ void k_v_rows<double>(int, long long, const int *, const int *, const double *, int, double,
                                          VHead *, int *);
template __global__ void k_v_cols<float>(int, long long, const int *, const int *, const float *, int, VHead *,
                                         const int *);
template __global__ void k_v_cols<double>(int, long long, const int *, const int *, const double *, int, VHead *,
                                          const int *);

}  // namespace rlgl
