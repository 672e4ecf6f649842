// Shared definitions of the device kernels and the host side of the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rlgl {

constexpr int BLOCK = 256;          // threads per workgroup (4 waves of 64)
constexpr int NWAVE = BLOCK / 64;
constexpr int VPT = 4;              // nodes per thread in node-parallel passes
constexpr int TILE = BLOCK * VPT;   // nodes per tile
constexpr int CH = 2048;            // links per push chunk and per batched pull item
constexpr int RUN_MAX_COLS = 1024; // batched pull: columns per run item (4 per thread)
constexpr int WU = 8;               // single-chain pull: links per lane of a wave item
constexpr int WL = 64 * WU;         // single-chain pull: links per run item and per long-column piece
constexpr int WCOLS = 64;           // single-chain pull: columns per run item
constexpr int HOT_SRC = 6144;       // single-chain pull: send values of the lowest-numbered sources held in LDS
constexpr int HOT_SRC_VAL = 4096;   // the same when the pull parks stored link values (LDS budget of four
                                    // workgroups per CU)
// The same with one workgroup of PULL_WIDE waves per CU (the LDS of a whole CU):
constexpr int PULL_WIDE = 16;
constexpr int HOT_WIDE = 24576, HOT_WIDE_VAL = 20480;
constexpr int KH_BITS = 11;         // top-k: bits of the |C| key counted by the pass that writes C
constexpr int KH_BINS = 1 << KH_BITS;
constexpr int KH_STRIPES = 4;       // global copies of the top-k histogram
constexpr int TK_GRID = 256;        // top-k: workgroups of the collecting pass at most (one segment each)
constexpr int TK_LOW_BITS = 31 - 2 * KH_BITS;  // FP32 keys: bits below the histogram's and the next digit's
constexpr int TK_LOW_BINS = 1 << TK_LOW_BITS;
// top-k pass histograms: FP64 keys, three digit buffers; FP32 keys, the
// middle digit in KH_STRIPES copies and the low digit
constexpr int TK_HIST_WORDS = (3 > KH_STRIPES ? 3 : KH_STRIPES) * KH_BINS + TK_LOW_BINS;
constexpr int LOG_STEPS = 4096;     // ring of per-step records kept for profiling
constexpr int MAX_GRID = 2048;      // edge-parallel launches
constexpr int NODE_GRID = 512;      // node-parallel launches (2 workgroups per CU)
constexpr int SEL_GRID = 1024;      // select launches (4 workgroups per CU, one tile each at N = 2^20)
constexpr int HOT_MAX = 2048;       // push: destinations privatised in LDS (FP64) per workgroup
constexpr int HOT_MIN_INDEG = 256;  // push: in-degree from which a destination is privatised
constexpr int PUSH_GRID = 512;      // push launches (hot partials flushed once per workgroup)
// Same-address atomics serialise (~13 ns each on MI355X), so every block
// folds its partial sums into one of NSTRIPE cache-line-sized stripes
// (block b -> stripe b mod NSTRIPE); readers add the stripes up.
constexpr int NSTRIPE = 32;

enum { SCHED_ALL = 0, SCHED_THRESHOLD = 1, SCHED_TOPK = 2, SCHED_MAXC = 3, SCHED_PC = 4 };
// a step whose green set the caller gives as a byte mask (rlgl_step_mask)
constexpr int SCHED_MASK = 5;
enum { ROUTE_PUSH = 0, ROUTE_PULL = 1, ROUTE_AUTO = 2 };
// ST_BAD_GRAPH: a kernel met a row/column pointer or link index outside its
// range (the caller's graph breaks the contract); reported as RLGL_EINVAL.
enum { ST_RUNNING = 0, ST_CONVERGED = 1, ST_LIMIT = 2, ST_BAD_GRAPH = -1, ST_ZERO_HISTORY = -4, ST_NONFINITE = -6 };

// One stripe of the FP64 accumulators of a record.
struct alignas(128) Acc {
  // statistics of C_t (folded in by the step that produced C_t)
  double l1;                        // ||C_t||_1
  double csum;                      // C_t 1
  double sumr;                      // sum |C_t|^r (r != 1)
  unsigned long long maxabs_bits;   // max |C_t| as the bits of a non-negative double
  // accumulators of step t (folded in by select of step t)
  double T;                         // restart pool: sum_G M_i (1 - c [outdeg_i > 0])
  double msum;                      // sum_G M_i
  double dhnorm;                    // change of ||H||_1
  long long green;                  // |G_t|
  long long gedges;                 // links of green nodes with non-zero cash
  // sums of an imported state
  double hsum_import;
  double hnorm_import;
};

// Totals of the stripes.
struct Tot {
  double l1, csum, sumr, maxabs, T, msum, dhnorm, hsum_import, hnorm_import;
  long long green, gedges;
};

// Scalars of step t (record t mod 3).
struct alignas(256) Rec {
  double hsum;                // H_t 1
  double hnorm;               // ||H_t||_1
  long long edges_total;      // edge-pushes of steps 0..t-1
  long long green_total;      // |G| summed over steps 1..t-1
  int buf;                    // cash buffer that holds C_t
  int mode;                   // 0 push, 1 pull (set by select of step t)
  double theta;               // threshold used by step t
  double topk_tau;            // top-k: k-th largest |C_t|
  int topk_tie_id;            // top-k: largest id taken among ties at tau
  unsigned int ticket;        // last-block detection in k_complete
  unsigned long long fr_pack; // frontier rows << 32 | frontier links (one reservation per tile)
  Acc acc[NSTRIPE];
};

struct Glob {
  int status;
  unsigned int ticket;        // last-block detection in k_refresh
  int bad;                    // a kernel met a link index or plan item outside its range (sticky)
  int pad_;
  long long t;                // index of the current state
  double rpool;               // refresh: sum_j H_j (1 - c [outdeg_j > 0])
  // top-k: the histogram bin that holds the k-th key, the keys of that bin
  // still to take, and the length of its candidate list
  unsigned long long tk_pref[2];  // radix state of the passes (double-buffered by pass parity)
  long long tk_rem[2];
  unsigned long long tk_tau;      // the k-th key, once its digits are fixed
  int tk_done;  // tau and the id bound of the running top-k select are written
  unsigned int pad2_;
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
  unsigned long long seed;  // SCHED_PC draws
  const unsigned char *green_in;  // SCHED_MASK: the caller's green set, one byte per node
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
  double *delta;         // push with FP32 cash: FP64 sums of the routed cash, folded into C by complete
  void *src;             // pull: what each node sends along one of its links this step (cash type, n)
  double *rsrc;          // refresh: what each node's history sends along one link (FP64, n)
  const int *colt;       // push: CSR columns with hot destinations tagged as -1 - slot
  const int *hot_nodes;  // push: node of each hot slot
  int n_hot;
  Rec *rec;
  Glob *glob;
  StepLog *log;
  // static pull plan
  const int4 *items;
  int n_items;
  const int *long_cols;
  double *long_acc;
  int *long_cnt;  // links of each long column summed so far in the running pass (0 between passes)
  int n_long;
  // relabelled layout: internal index -> caller's id (NULL: the caller's numbering)
  const int *perm;
  // top-k: histograms of the top key bits per record, candidate keys and ids
  unsigned int *khist;         // [3][KH_STRIPES][KH_BINS]
  unsigned long long *tk_ckey;  // [n]
  int *tk_cid;                  // [n]
  unsigned int *tk_hist;        // [TK_HIST_WORDS] digit histograms of the passes over the candidates
  int *tk_cnt;                  // [tk_grid] candidates each collecting workgroup found
  unsigned int *tk_seg;         // FP32 keys: [tk_grid][TK_LOW_BINS] low-digit histograms per segment
  int tk_grid;                  // workgroups of the collecting pass
};

// Host-side sum of the stripes (same order as the device).
inline Tot host_totals(const Rec &r) {
  Tot t{};
  for (int q = 0; q < NSTRIPE; ++q) {
    const Acc &a = r.acc[q];
    t.l1 += a.l1;
    t.csum += a.csum;
    t.sumr += a.sumr;
    double m;
    __builtin_memcpy(&m, &a.maxabs_bits, sizeof m);
    t.maxabs = m > t.maxabs ? m : t.maxabs;
    t.T += a.T;
    t.msum += a.msum;
    t.dhnorm += a.dhnorm;
    t.hsum_import += a.hsum_import;
    t.hnorm_import += a.hnorm_import;
    t.green += a.green;
    t.gedges += a.gedges;
  }
  return t;
}

}  // namespace rlgl
