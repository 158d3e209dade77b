// Host-side objects of the AA-PDHG runtime (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <chrono>
#include <memory>
#include <string>
#include <vector>

#include "../../include/aapdhg.h"
#include "aapdhg_internal.h"
#include "kernels.h"

namespace aapdhg {

struct Error {
  aapdhg_status status;
  std::string msg;
  Error(aapdhg_status s, const char* fmt, ...);
};

void hip_check(hipError_t e, const char* what);
void default_options(aapdhg_options* o);
extern thread_local std::string g_thread_error;
// Stream of the calling thread's set-up work in Problem::create (uploads,
// scaling, power iteration): nullptr is the default stream; the server's
// admission thread sets its copy stream.
extern thread_local hipStream_t g_setup_stream;

// Owning device allocation.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf();
  void release();
  void alloc(size_t nbytes, const char* what);
  void upload(const void* src, size_t nbytes, const char* what);
  void zero(const char* what);
};

struct Problem;

// A named host range for profilers (roctx; seen with rocprofv3 --marker-trace,
// free when no tool is attached): create, solve and serving epochs.
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePush(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

// The device work tables of a set of LPs that advance in the same launches.
struct LaunchSet {
  static constexpr int MAX_STATUS = 65536;
  static constexpr int64_t MAX_LOOP_PASSES = 65535;  // per launch of the persistent loop kernel
  std::vector<Problem*> members;
  LaunchTables t;
  DevBuf d_lps, d_llp, d_chunks, d_blocksA, d_blocksB, d_dblocks, d_splits, d_rec, d_dpart, d_dcnt, d_splitpart,
      d_splitcnt, d_tiles, d_status, d_wgs, d_looplps, d_sync, d_bc, d_err, d_pwpart, d_pwcnt, d_pwrec, d_gpart,
      d_gcnt;
  int* h_status = nullptr;  // pinned, 2 x MAX_STATUS
  int64_t last_epochs = 0;
  std::vector<double> finish_s;  // per member: seconds into run_to_completion when seen stopped
  ~LaunchSet();
  void build(const std::vector<Problem*>& lps);
  void enqueue_passes(hipStream_t st, int64_t iters);
  // enqueue passes with events around the launches and wait.  Persistent
  // kernel: ms4 = {1, ms of the one launch, passes, 1}; three launches per
  // pass: ms4 = {0, mean ms of A, of B, of C}.
  void timed_passes(hipStream_t st, int64_t iters, double* ms4);
  void check_loop_error(hipStream_t st);
  // tag base of the next persistent launch: the launch count times 65536, so
  // that (launch, pass) tags of published decisions never repeat between
  // consecutive launches (passes per launch stay below 65536)
  unsigned int launch_seq = 0;
  unsigned int next_tag() { return (++launch_seq) << 16; }
  void enqueue_eval(hipStream_t st);
  // Epochs of loop passes until every member has stopped (or the time
  // limit).  With compact_below > 0 it returns as soon as at most that many
  // members are still running (compacted is then set and the others' finish
  // times stay -1).  Times count from *t0 when given.
  double run_to_completion(hipStream_t st, int epoch, double time_limit_s, int compact_below = 0,
                           const std::chrono::steady_clock::time_point* t0 = nullptr);
  bool compacted = false;
  size_t device_bytes() const;
  // three-launch passes captured in a HIP graph and replayed (some member
  // asked for it and the set is not persistent)
  bool use_graph = false;
  hipGraphExec_t graph_exec = nullptr;
  int64_t graph_passes = 0;
  void build_graph(int64_t iters);
  void drop_graph();
};

// One LP: host copies of the data as solved, its device arrays and state.
struct Problem {
  aapdhg_options opt{};
  int m = 0, n = 0, N = 0, nnz = 0;
  bool fp64 = false;
  bool started = false;
  bool pending_init = false;  // start point set, init step (k = 0) not yet enqueued
  bool in_batch = false;
  double qnorm = 0.0, cnorm = 0.0, norm_est = 0.0;
  double last_solve_seconds = 0.0;
  // host data (after scaling and rounding)
  std::vector<int> rowptr, colidx, colptr, rowidx;
  std::vector<double> val, valT, c, q, lo, hi, dhat, d_row, d_col;
  std::vector<uint8_t> rowtype;
  // work tables (LP-local indices)
  std::vector<Chunk> chunksA, chunksB;
  std::vector<SplitRow> splitsA, splitsB;
  int npartsA = 0, npartsB = 0;
  std::vector<MixTile> tiles;
  // device data
  DevBuf d_rowptr, d_colidx, d_val, d_colptr, d_rowidx, d_valT, d_rmapA, d_rmapB, d_c, d_lo, d_hi, d_q, d_dhat,
      d_rowtype;
  DevBuf d_u[2], d_g[2], d_xbar, d_hist_dG, d_hist_W, d_lam, d_sc, d_desc, d_xfer;
  DevBuf d_anchor;  // iterate of the last primal-weight check (when the update is on)
  DevBuf d_rsum;    // restarted PDHG: sum of the epoch's iterates
  DevBuf d_scale;   // d_col then d_row, for results written to device memory (made on first use)
  DevBuf d_pptr, d_pidx, d_pval, d_part, d_pchunk;  // column panels of the dual product
  bool panels = false;
  int pcoff[MAX_PANELS + 1] = {};
  std::vector<Chunk> chunksBp;  // dual pass in a launch of its own with panels: 256-row chunks
  int row_weight = 4;           // chunk cost model: entries a row counts beyond its own
  std::vector<int> dev_ptrA, dev_ptrB;  // row pointers of the device row orders (host copies)
  LPDesc desc{};
  Scalars sc_init{};
  std::unique_ptr<LaunchSet> solo;

  ~Problem();
  void create(int32_t m, int32_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
              const double* val, const double* c, const double* q, const double* l, const double* u,
              const uint8_t* row_type, const aapdhg_options* opt);
  void fill_desc();
  void set_gram_mode();
  double power_norm();
  void reset_host_state();
  void enqueue_reset(hipStream_t st);
  void enqueue_init(hipStream_t st);
  void iterate_noalloc(hipStream_t st, int64_t iters);
  void read_scalars(Scalars& s);
  void download(const void* dev, size_t len, double* host, hipStream_t st);
  void upload_vec(void* dev, const double* host, size_t len, hipStream_t st);
  void result(double* x, double* y, double* lam, aapdhg_info* info, bool run_eval);
  void get_state(double* u, double* u_prev, double* g_prev, double* dG, double* W, int64_t* meta, double* gram);
  void get_weights(double* anchor, double* w);
  void scale_on_device();
  void result_device(double* x, double* y, double* lam, aapdhg_info* info, hipStream_t st);
  void set_weights(const double* anchor, const double* w);
  void set_state(const double* u, const double* u_prev, const double* g_prev, const double* dG, const double* W,
                 const int64_t* meta, const double* gram);
  size_t device_bytes() const;
  void rebuild_tables();
  // autotuner (tuner.cpp): row_weight, chunks_per_block and loop_kernel
  // from the tuning cache, or timed on the device and stored there
  void autotune();
  std::string tune_key() const;
  double time_candidate();
};

}  // namespace aapdhg
