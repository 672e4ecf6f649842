// Shared definitions of the device kernels and the host side of the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rlgl {

constexpr int BLOCK = 256;          // threads per workgroup (4 waves of 64)
constexpr int NWAVE = BLOCK / 64;
constexpr int VPT = 4;              // nodes per thread in node-parallel passes
constexpr int TILE = BLOCK * VPT;   // nodes per tile
constexpr int CH = 2048;            // links per push/pull chunk
constexpr int SHORT_MAX = 64;       // pull: in-degree handled by the thread-per-column path
constexpr int LONG_COL_MIN = 4096;      // pull: in-degree split across several workgroups
constexpr int LOG_STEPS = 4096;     // ring of per-step records kept for profiling
constexpr int MAX_GRID = 2048;

enum { SCHED_ALL = 0, SCHED_THRESHOLD = 1, SCHED_TOPK = 2, SCHED_MAXC = 3 };
enum { ROUTE_PUSH = 0, ROUTE_PULL = 1, ROUTE_AUTO = 2 };
enum { ST_RUNNING = 0, ST_CONVERGED = 1, ST_LIMIT = 2, ST_ZERO_HISTORY = -4, ST_NONFINITE = -6 };
enum { ITEM_SHORT = 0, ITEM_MEDIUM = 1, ITEM_LONG = 2 };

// Scalars of step t (record t mod 3).  The statistics describe C_t and are
// folded in by step t-1; the accumulators are folded in by step t itself.
struct alignas(256) Rec {
  // statistics of C_t and H_t
  double l1;                 // ||C_t||_1
  double csum;               // C_t 1
  double sumr;               // sum |C_t|^r (r != 1)
  unsigned long long maxabs_bits;  // max |C_t| as double bits
  double hsum;               // H_t 1
  double hsum_import;        // sum of an imported H
  double hnorm;              // ||H_t||_1
  long long edges_total;     // edge-pushes of steps 0..t-1
  long long green_total;     // |G| summed over steps 1..t-1
  int buf;                   // cash buffer that holds C_t
  int mode;                  // 0 push, 1 pull (set by select of step t)
  double theta;              // threshold used by step t
  double topk_tau;           // top-k: k-th largest |C_t|
  int topk_tie_id;           // top-k: largest id taken among ties at tau
  unsigned int ticket;       // last-block detection in k_complete
  // accumulators of step t
  double T;                  // restart pool: sum_G M_i (1 - c [outdeg_i > 0])
  double msum;               // sum_G M_i
  double dhnorm;             // change of ||H||_1
  unsigned long long fr_pack;  // frontier rows << 32 | frontier links
  long long green;           // |G_t|
  long long gedges;          // links of green nodes with non-zero cash
};

struct Glob {
  int status;
  unsigned int ticket;       // last-block detection in k_refresh
  long long t;               // index of the current state
  double rpool;              // refresh: sum_j H_j (1 - c [outdeg_j > 0])
};

struct StepLog {
  long long s, green, gedges, nfront;
  int mode, pad;
};

// Everything a kernel needs, passed by value.
struct Dev {
  int n;
  long long nnz;
  double c;
  const int *rowptr;
  const int *col;
  const void *val;
  const int *colptr;
  const int *crow;
  const void *cval;
  // options
  int sched;
  double r;
  long long k;
  int theta_period;
  int route;
  double pull_alpha;
  // workspace
  void *cash[2];
  void *hist;        // double[n], or float[n] (hi part) for the compensated history
  float *hist_lo;    // float[n] low part of the compensated history
  int *fr_rowstart;
  int *fr_eoff;
  int *fr_id;
  void *fr_scale;
  int *chunk_first;
  unsigned char *green_mask;
  Rec *rec;
  Glob *glob;
  StepLog *log;
  // static pull plan
  const int4 *items;
  int n_items;
  const int *med_cols;
  const int *long_cols;
  double *long_acc;
  int n_long;
};

}  // namespace rlgl
