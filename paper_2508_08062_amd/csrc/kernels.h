// Launchers of the HIP kernels (kernels.hip), used by the host runtime.
#pragma once

#include <hip/hip_runtime.h>

#include "aapdhg_internal.h"

namespace aapdhg {

// Device tables of one launch set: the LPs that advance together.
struct LaunchTables {
  bool fp64 = false;
  int mt = 4;  // memory bound of the kernel instantiation (>= every member's m_A)
  const LPDesc* lps = nullptr;
  const LaunchLP* llp = nullptr;
  int nlps = 0;
  const Chunk* chunks = nullptr;  // both passes
  const BlockWork* blocksA = nullptr;
  int nblocksA = 0;
  const BlockWork* blocksB = nullptr;
  int nblocksB = 0;
  int nleaves = 0;
  const DecideBlock* dblocks = nullptr;
  int ndblocks = 0;
  const SplitRow* splits = nullptr;
  double* rec = nullptr;
  double* dpart = nullptr;
  unsigned int* dcnt = nullptr;
  double* splitpart = nullptr;
  unsigned int* splitcnt = nullptr;
  const MixTile* tiles = nullptr;
  int ntiles = 0;
  double* pwpart = nullptr;       // [tiles][2] weight-check partial sums
  unsigned int* pwcnt = nullptr;  // [LPs] weight-check arrivals
  double* gpart = nullptr;        // [tiles][gram_partials_per_tile(mt)] Gram-launch partials
  unsigned int* gcnt = nullptr;   // [LPs] Gram-launch arrivals
  bool gram = false;  // some LP of the table forms its Gram matrix on demand (the Gram launch runs)
  bool dots = true;   // some LP of the table needs the per-pass dots in the three-launch passes
  // persistent loop kernel (when the set fits the resident workgroups)
  bool panels = false;  // the one LP of the table has column panels for its dual product
  bool persistent = false;
  bool ext = false;  // some LP of the table uses the primal-weight update or restarts
  const LoopWG* wgs = nullptr;
  int nwgs = 0;
  const LoopLP* looplps = nullptr;
  LoopSync* sync = nullptr;
  BcastMsg* bc = nullptr;
  double* pwrec = nullptr;  // [workgroups][2] weight-check partial sums
  int* err = nullptr;
  unsigned long long timeout_ticks = 0;
};

// One loop pass (passes A, B, the decisions D and, in MODE_ITER, the Gram
// launch and the mix C) for every LP of the table.  With ev != nullptr,
// events ev[0..3] are recorded before A, after A, after D and after C on the
// same stream.
hipError_t launch_loop_pass(const LaunchTables& t, hipStream_t st, int mode, hipEvent_t* ev = nullptr);
// `passes` loop passes of every LP of the table in one cooperative launch of
// the persistent loop kernel (t.persistent must be set), after a Gram refresh
// of the LPs whose three-launch passes left G and rhs stale.
hipError_t launch_loop(const LaunchTables& t, hipStream_t st, long long passes, unsigned int tag0);
// Gram refresh: G and rhs of the live slots of every LP of the table whose
// scalars say they are stale (no work for the others).
hipError_t launch_gram_refresh(const LaunchTables& t, hipStream_t st);
// Doubles per mix tile of the Gram launch's partials for memory bound mt.
int gram_partials_per_tile(int mt);
// Workgroups of the persistent loop kernel that fit on the device at once.
int loop_capacity(bool fp64, int mt, bool ext);
// Workgroups of pass A (pass 0) or pass B (pass 1) of the three-launch path
// that the device holds at once (0 if the query fails), for the kernel with
// (dots) or without the per-pass dots of the new difference column.
int pass_capacity(bool fp64, int mt, int pass, bool dots);
hipError_t launch_start_point(const LPDesc& d, bool fp64, hipStream_t st);
// Zero `bytes` (a multiple of 4) of device memory with a fill kernel on `st`.
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);

// Scratch of the no-allocation entry point: a file-scope device array of
// STATIC_SCRATCH_BYTES per device, held until the process ends.  *out
// receives its address on the current device (looked up once per device).
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)2 << 20;
constexpr int MAX_DEVICES = 64;
hipError_t static_scratch(void** out);

// Scaling of K before the solve: ruiz_iters Ruiz sweeps, then (pock_chambolle)
// one Pock-Chambolle step with alpha = 1, on the float64 CSR values `val`;
// the factors are divided into drow[m] and dcol[n].  cptr/cperm: the CSC
// order of the entries (positions in the CSR), for the column sums.
// Work: rfac[m], cfac[n], cmax[n].
struct ScalingArgs {
  int m = 0, n = 0;
  const int* rowptr = nullptr;
  const int* colidx = nullptr;
  double* val = nullptr;
  const int* cptr = nullptr;
  const int* cperm = nullptr;
  double* rfac = nullptr;
  double* cfac = nullptr;
  unsigned long long* cmax = nullptr;
  double* drow = nullptr;
  double* dcol = nullptr;
  int ruiz_iters = 0;
  bool pock_chambolle = false;
};
hipError_t launch_scaling(const ScalingArgs& s, hipStream_t st);
// x[n], y[m], lambda[n] (float64, device; any may be null) from the iterate u
// and the reduced costs lam of type T (fp64: double, else float), unscaled by
// scale = (d_col[n], d_row[m]).
hipError_t launch_unscale(const void* u, const void* lam, const double* scale, bool fp64, int n, int m, double* x,
                          double* y, double* lo, hipStream_t st);
// Power iteration on K^T K from the SplitMix64 start vector of `seed`;
// est[0..iters] receives ||K^T K v|| of each step (the square of the ||K||
// estimate).  work holds 2n + m + 1024 doubles.
hipError_t launch_power_iteration(const LPDesc& d, bool fp64, int iters, unsigned long long seed, double* work,
                                  double* est, hipStream_t st);
hipError_t launch_gather_status(const LPDesc* lps, int count, int* out, hipStream_t st);
hipError_t launch_time_limit(const LPDesc* lps, int count, hipStream_t st);
hipError_t launch_to_f64(const void* src, bool fp64, double* dst, size_t len, hipStream_t st);
hipError_t launch_from_f64(const double* src, void* dst, bool fp64, size_t len, hipStream_t st);

}  // namespace aapdhg
