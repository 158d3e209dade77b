// Host runtime of the AA-PDHG library: C ABI entry points, input validation,
// set-up (CSR/CSC copies, Ruiz equilibration, D-hat, step size), the work
// tables of the kernels, the epoch driver, results and checkpoints.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "../../include/aapdhg.h"
#include "aapdhg_internal.h"
#include "kernels.h"
#include "runtime.h"

namespace aapdhg {

thread_local std::string g_thread_error;
thread_local hipStream_t g_setup_stream = nullptr;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

Error::Error(aapdhg_status s, const char* fmt, ...) : status(s) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  msg = buf;
}

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    if (e == hipErrorOutOfMemory) throw Error(AAPDHG_E_NOMEM, "%s: out of device memory", what);
    throw Error(AAPDHG_E_HIP, "%s: %s", what, hipGetErrorString(e));
  }
}

// ---------------------------------------------------------------------------
// device buffers
// ---------------------------------------------------------------------------

DevBuf::~DevBuf() { release(); }
void DevBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}
void DevBuf::alloc(size_t nbytes, const char* what) {
  release();
  if (nbytes == 0) nbytes = 8;
  hip_check(hipMalloc(&p, nbytes), what);
  bytes = nbytes;
}
void DevBuf::upload(const void* src, size_t nbytes, const char* what) {
  alloc(nbytes, what);
  if (!src || !nbytes) return;
  if (g_setup_stream) {
    hip_check(hipMemcpyAsync(p, src, nbytes, hipMemcpyHostToDevice, g_setup_stream), what);
    hip_check(hipStreamSynchronize(g_setup_stream), what);  // src may be a temporary
  } else {
    hip_check(hipMemcpy(p, src, nbytes, hipMemcpyHostToDevice), what);
  }
}
void DevBuf::zero(const char* what) {
  if (!p) return;
  if (g_setup_stream) {
    hip_check(launch_zero(p, bytes & ~(size_t)3, g_setup_stream), what);
    hip_check(hipStreamSynchronize(g_setup_stream), what);
  } else {
    hip_check(hipMemset(p, 0, bytes), what);
  }
}

// Copy device memory to the host on the set-up stream (see g_setup_stream).
static void setup_download(void* dst, const void* src, size_t nbytes, const char* what) {
  if (!nbytes) return;
  if (g_setup_stream) {
    hip_check(hipMemcpyAsync(dst, src, nbytes, hipMemcpyDeviceToHost, g_setup_stream), what);
    hip_check(hipStreamSynchronize(g_setup_stream), what);
  } else {
    hip_check(hipMemcpy(dst, src, nbytes, hipMemcpyDeviceToHost), what);
  }
}

// ---------------------------------------------------------------------------
// options
// ---------------------------------------------------------------------------

void default_options(aapdhg_options* o) {
  std::memset(o, 0, sizeof *o);
  o->variant = AAPDHG_VARIANT_AA;
  o->precision = 0;
  o->memory = 10;
  o->D = 10.0;
  o->eps_sg = 1.0;
  o->beta = 1.0;
  o->eta = 1e-10;
  o->cs = 0.2;
  o->kappa_bar = 1e8;
  o->tau = 0.0;
  o->sigma = 0.0;
  o->tol = 1e-4;
  o->max_iter = 100000;
  o->time_limit_s = 0.0;
  o->kkt_every = 64;
  o->dhat_mode = 1;
  o->ruiz_iters = 0;
  o->power_iters = 200;
  o->epoch = 256;
  o->chunks_per_block = 0;
  o->loop_kernel = 0;
  o->pw_period = 0;
  o->pw_theta = 0.5;
  o->pw_eps_zero = 1e-10;
  o->pw_omega0 = 0.0;
  o->pw_rho = 0.0;
  o->sg_div = 1.0;
  o->pw_dhat = 1;
  o->restart_period = 75;
  o->prep_device = 2;
  o->pock_chambolle = 0;
  o->angle_mode = 0;
  o->length_floor = 0;
  o->graph = 0;
  o->autotune = 0;
  o->gram_mode = 0;
  o->seed = 0;
}

static void check_options(const aapdhg_options& o) {
  if (o.variant < 0 || o.variant > 3) throw Error(AAPDHG_E_ARG, "variant must be 0, 1, 2 or 3");
  if (o.prep_device < 0 || o.prep_device > 2) throw Error(AAPDHG_E_ARG, "prep_device must be 0, 1 or 2");
  if (o.pock_chambolle != 0 && o.pock_chambolle != 1) throw Error(AAPDHG_E_ARG, "pock_chambolle must be 0 or 1");
  if (o.angle_mode != 0 && o.angle_mode != 1) throw Error(AAPDHG_E_ARG, "angle_mode must be 0 or 1");
  if (o.length_floor != 0 && o.length_floor != 1) throw Error(AAPDHG_E_ARG, "length_floor must be 0 or 1");
  if (o.graph != 0 && o.graph != 1) throw Error(AAPDHG_E_ARG, "graph must be 0 or 1");
  if (o.autotune != 0 && o.autotune != 1) throw Error(AAPDHG_E_ARG, "autotune must be 0 or 1");
  if (o.gram_mode < 0 || o.gram_mode > 2) throw Error(AAPDHG_E_ARG, "gram_mode must be 0, 1 or 2");
  if (o.variant == AAPDHG_VARIANT_RPDHG && o.restart_period < 1)
    throw Error(AAPDHG_E_ARG, "restart_period must be >= 1 for restarted PDHG");
  if (o.precision != 0 && o.precision != 1) throw Error(AAPDHG_E_ARG, "precision must be 0 or 1");
  if (o.memory < 1 || o.memory > MAXM) throw Error(AAPDHG_E_ARG, "memory must be in [1, %d]", MAXM);
  if (!(o.D >= 0.0)) throw Error(AAPDHG_E_ARG, "D must be >= 0");
  if (!(o.eps_sg > 0.0) || !std::isfinite(o.eps_sg)) throw Error(AAPDHG_E_ARG, "eps_sg must be > 0");
  if (!(o.beta > 0.0 && o.beta <= 1.0)) throw Error(AAPDHG_E_ARG, "beta must be in (0, 1]");
  if (!(o.eta >= 0.0) || !std::isfinite(o.eta)) throw Error(AAPDHG_E_ARG, "eta must be >= 0");
  if (!(o.cs > 0.0 && o.cs <= 1.0)) throw Error(AAPDHG_E_ARG, "cs must be in (0, 1]");
  if (!(o.kappa_bar > 0.0)) throw Error(AAPDHG_E_ARG, "kappa_bar must be > 0");
  if (!(o.tol >= 0.0)) throw Error(AAPDHG_E_ARG, "tol must be >= 0");
  if (o.max_iter < 0) throw Error(AAPDHG_E_ARG, "max_iter must be >= 0");
  if (o.kkt_every < 0) throw Error(AAPDHG_E_ARG, "kkt_every must be >= 0");
  if (o.dhat_mode < 0 || o.dhat_mode > 2) throw Error(AAPDHG_E_ARG, "dhat_mode must be 0, 1 or 2");
  if (o.ruiz_iters < 0 || o.ruiz_iters > 1000) throw Error(AAPDHG_E_ARG, "ruiz_iters must be in [0, 1000]");
  if (o.power_iters < 1 || o.power_iters > 100000) throw Error(AAPDHG_E_ARG, "power_iters must be in [1, 100000]");
  if (o.epoch < 1 || o.epoch > 1000000) throw Error(AAPDHG_E_ARG, "epoch must be in [1, 1e6]");
  if (o.chunks_per_block < 0 || o.chunks_per_block > 4096) throw Error(AAPDHG_E_ARG, "chunks_per_block must be in [0, 4096]");
  if (o.loop_kernel < 0 || o.loop_kernel > 1) throw Error(AAPDHG_E_ARG, "loop_kernel must be 0 or 1");
  if (o.wait_limit_us < 0) throw Error(AAPDHG_E_ARG, "wait_limit_us must be >= 0");
  if (!std::isfinite(o.tau) || !std::isfinite(o.sigma)) throw Error(AAPDHG_E_ARG, "tau and sigma must be finite");
  if (o.pw_period < 0) throw Error(AAPDHG_E_ARG, "pw_period must be >= 0");
  if (!(o.pw_theta >= 0.0 && o.pw_theta <= 1.0)) throw Error(AAPDHG_E_ARG, "pw_theta must be in [0, 1]");
  if (!(o.pw_eps_zero > 0.0) || !std::isfinite(o.pw_eps_zero)) throw Error(AAPDHG_E_ARG, "pw_eps_zero must be > 0");
  if (!std::isfinite(o.pw_omega0)) throw Error(AAPDHG_E_ARG, "pw_omega0 must be finite");
  if (!std::isfinite(o.pw_rho)) throw Error(AAPDHG_E_ARG, "pw_rho must be finite");
  if (o.pw_dhat != 0 && o.pw_dhat != 1) throw Error(AAPDHG_E_ARG, "pw_dhat must be 0 or 1");
  if (!(o.sg_div > 0.0) || !std::isfinite(o.sg_div)) throw Error(AAPDHG_E_ARG, "sg_div must be > 0");
}

// ---------------------------------------------------------------------------
// work tables of one LP
// ---------------------------------------------------------------------------

static int pow2floor(int v) {
  int p = 1;
  while (p * 2 <= v) p *= 2;
  return p;
}

constexpr int LONG_ROW = 128;  // rows above this length leave the multi-row chunks
constexpr int64_t PANEL_MIN_NNZ = 1 << 22;  // column panels for the dual product from 4M entries
constexpr int64_t PREP_DEVICE_NNZ = 1 << 20;  // automatic scaling on the device from 1M entries

// Order of the rows of one pass on the device: rows of at most LONG_ROW
// entries keep their original order (their epilogue accesses stay
// coalesced), longer rows follow by decreasing length so that a few of them
// can share a workgroup, and rows longer than a chunk come last.  rmap[pos]
// is the original row at position pos; ptr2/idx2/val2 are the matrix with its
// rows in that order.
static void reorder_rows(const std::vector<int>& ptr, const std::vector<int>& idx, const std::vector<double>& v,
                         int R, std::vector<int>& rmap, std::vector<int>& ptr2, std::vector<int>& idx2,
                         std::vector<double>& v2) {
  rmap.clear();
  std::vector<int> longr, split;
  for (int r = 0; r < R; ++r) {
    const int len = ptr[r + 1] - ptr[r];
    if (len <= LONG_ROW) rmap.push_back(r);
    else if (len <= CHUNK_NNZ) longr.push_back(r);
    else split.push_back(r);
  }
  std::stable_sort(longr.begin(), longr.end(),
                   [&](int a, int b) { return ptr[a + 1] - ptr[a] > ptr[b + 1] - ptr[b]; });
  rmap.insert(rmap.end(), longr.begin(), longr.end());
  rmap.insert(rmap.end(), split.begin(), split.end());
  ptr2.assign(R + 1, 0);
  idx2.resize(idx.size());
  v2.resize(v.size());
  for (int pos = 0; pos < R; ++pos) {
    const int r = rmap[pos];
    const int len = ptr[r + 1] - ptr[r];
    ptr2[pos + 1] = ptr2[pos] + len;
    std::copy(idx.begin() + ptr[r], idx.begin() + ptr[r + 1], idx2.begin() + ptr2[pos]);
    std::copy(v.begin() + ptr[r], v.begin() + ptr[r + 1], v2.begin() + ptr2[pos]);
  }
}

// Cut the positions [0, R) of a reordered matrix into chunks (see Chunk):
//  - runs of short rows form multi-row chunks of at most CHUNK_ROWS rows and
//    CHUNK_NNZ entries, weighted so that short rows (whose epilogue
//    dominates) do not crowd a chunk: each row counts row_weight entries
//    beyond its own (4 by default; the autotuner may choose another);
//  - longer rows are grouped by up to four (one wave each), at most CHUNK_NNZ
//    entries per group; a group of one is reduced by the whole workgroup;
//  - a row with more than CHUNK_NNZ entries is split into parts of SPLIT_NNZ.
static void build_chunks(const std::vector<int>& ptr, int R, std::vector<Chunk>& chunks,
                         std::vector<SplitRow>& splits, int& nparts_total, int row_weight) {
  const int ROW_WEIGHT = row_weight;
  chunks.clear();
  splits.clear();
  nparts_total = 0;
  int r = 0;
  while (r < R) {
    const int len = ptr[r + 1] - ptr[r];
    if (len > CHUNK_NNZ) {
      const int np = (len + SPLIT_NNZ - 1) / SPLIT_NNZ;
      SplitRow sr{};
      sr.row = r;
      sr.nparts = np;
      sr.part0 = nparts_total;
      const int sid = (int)splits.size();
      splits.push_back(sr);
      nparts_total += np;
      for (int p = 0; p < np; ++p) {
        Chunk c{};
        c.kind = 1;
        c.r0 = r;
        c.r1 = r + 1;
        c.k0 = ptr[r] + p * SPLIT_NNZ;
        c.k1 = std::min(ptr[r + 1], c.k0 + SPLIT_NNZ);
        c.tpr = p;
        c.split = sid;
        chunks.push_back(c);
      }
      ++r;
      continue;
    }
    const int r0 = r;
    int nnz = 0;
    if (len > LONG_ROW) {
      while (r < R && r - r0 < BLOCK / 64) {
        const int l2 = ptr[r + 1] - ptr[r];
        if (l2 <= LONG_ROW || l2 > CHUNK_NNZ || nnz + l2 > CHUNK_NNZ) break;
        nnz += l2;
        ++r;
      }
      Chunk c{};
      c.kind = 0;
      c.r0 = r0;
      c.r1 = r;
      c.k0 = ptr[r0];
      c.k1 = ptr[r];
      c.tpr = r - r0 == 1 ? BLOCK : 64;
      chunks.push_back(c);
      continue;
    }
    while (r < R && r - r0 < CHUNK_ROWS) {
      const int l2 = ptr[r + 1] - ptr[r];
      if (l2 > LONG_ROW) break;
      if (nnz + l2 > CHUNK_NNZ) break;
      if (nnz + l2 + ROW_WEIGHT * (r - r0 + 1) > CHUNK_NNZ + ROW_WEIGHT * 64 && r > r0) break;
      nnz += l2;
      ++r;
    }
    const int nrows = r - r0;
    Chunk c{};
    c.kind = 0;
    c.r0 = r0;
    c.r1 = r;
    c.k0 = ptr[r0];
    c.k1 = ptr[r];
    c.tpr = nrows >= BLOCK ? 1 : std::min(64, pow2floor(BLOCK / nrows));
    chunks.push_back(c);
  }
}

// ---------------------------------------------------------------------------
// problem creation
// ---------------------------------------------------------------------------

template <typename T>
static void upload_as(DevBuf& b, const std::vector<double>& v, const char* what) {
  std::vector<T> tmp(v.begin(), v.end());
  b.upload(tmp.data(), tmp.size() * sizeof(T), what);
}

Problem::~Problem() = default;

void Problem::create(int32_t m_, int32_t n_, int64_t nnz_, const int64_t* row_ptr, const int32_t* col_idx,
                     const double* val_, const double* c_, const double* q_, const double* l_, const double* u_,
                     const uint8_t* row_type, const aapdhg_options* opt_) {
  TraceRange tr("aapdhg create");
  if (opt_) opt = *opt_; else default_options(&opt);
  check_options(opt);
  if (m_ < 1 || n_ < 1) throw Error(AAPDHG_E_ARG, "m and n must be >= 1 (m=%d n=%d)", m_, n_);
  if (nnz_ < 0 || nnz_ >= (int64_t)1 << 31) throw Error(AAPDHG_E_ARG, "nnz must be in [0, 2^31)");
  if ((int64_t)m_ + n_ >= (int64_t)1 << 31) throw Error(AAPDHG_E_ARG, "m + n too large");
  if (!row_ptr || (!col_idx && nnz_) || (!val_ && nnz_) || !c_ || !q_ || !l_ || !u_ || !row_type)
    throw Error(AAPDHG_E_ARG, "null input array");
  m = m_;
  n = n_;
  nnz = (int)nnz_;
  N = m + n;
  fp64 = opt.precision == 1;
  // ---- validate and copy, sorting each row by column ----
  if (row_ptr[0] != 0 || row_ptr[m] != nnz_) throw Error(AAPDHG_E_ARG, "row_ptr[0] must be 0 and row_ptr[m] must be nnz");
  rowptr.assign(m + 1, 0);
  for (int i = 0; i < m; ++i) {
    if (row_ptr[i + 1] < row_ptr[i]) throw Error(AAPDHG_E_ARG, "row_ptr decreases at row %d", i);
    rowptr[i + 1] = (int)row_ptr[i + 1];
  }
  colidx.resize(nnz);
  val.resize(nnz);
  {
    std::vector<std::pair<int, double>> tmp;
    for (int i = 0; i < m; ++i) {
      tmp.clear();
      for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
        const int j = col_idx[q];
        if (j < 0 || j >= n) throw Error(AAPDHG_E_ARG, "column index %d out of range at row %d", j, i);
        if (!std::isfinite(val_[q])) throw Error(AAPDHG_E_ARG, "non-finite matrix value at row %d", i);
        tmp.emplace_back(j, val_[q]);
      }
      std::sort(tmp.begin(), tmp.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
      for (size_t t = 0; t < tmp.size(); ++t) {
        if (t > 0 && tmp[t].first == tmp[t - 1].first) throw Error(AAPDHG_E_ARG, "repeated column %d in row %d", tmp[t].first, i);
        colidx[rowptr[i] + t] = tmp[t].first;
        val[rowptr[i] + t] = tmp[t].second;
      }
    }
  }
  c.assign(c_, c_ + n);
  q.assign(q_, q_ + m);
  lo.assign(l_, l_ + n);
  hi.assign(u_, u_ + n);
  rowtype.assign(row_type, row_type + m);
  for (int j = 0; j < n; ++j) {
    if (!std::isfinite(c[j])) throw Error(AAPDHG_E_ARG, "non-finite c[%d]", j);
    if (std::isnan(lo[j]) || std::isnan(hi[j]) || lo[j] > hi[j] || lo[j] == INFINITY || hi[j] == -INFINITY)
      throw Error(AAPDHG_E_ARG, "invalid bounds at column %d", j);
  }
  for (int i = 0; i < m; ++i) {
    if (!std::isfinite(q[i])) throw Error(AAPDHG_E_ARG, "non-finite q[%d]", i);
    if (rowtype[i] > 1) throw Error(AAPDHG_E_ARG, "row_type[%d] must be 0 or 1", i);
  }
  // ---- Ruiz equilibration and the Pock-Chambolle step (preconditioning of
  // Section 5.2): on the device or the host (prep_device; automatic: the
  // device from PREP_DEVICE_NNZ entries, where its set-up pays off); both
  // apply the same operations in the same order to every entry ----
  d_row.assign(m, 1.0);
  d_col.assign(n, 1.0);
  const bool scale = opt.ruiz_iters > 0 || opt.pock_chambolle;
  const bool on_device = opt.prep_device == 1 || (opt.prep_device == 2 && (int64_t)nnz >= PREP_DEVICE_NNZ);
  if (scale && on_device) {
    scale_on_device();
  } else if (scale) {
    std::vector<double> rmax(m), cmax(n), r(m), s(n);
    for (int it = 0; it < opt.ruiz_iters; ++it) {
      std::fill(rmax.begin(), rmax.end(), 0.0);
      std::fill(cmax.begin(), cmax.end(), 0.0);
      for (int i = 0; i < m; ++i)
        for (int qq = rowptr[i]; qq < rowptr[i + 1]; ++qq) {
          const double a = std::fabs(val[qq]);
          rmax[i] = std::max(rmax[i], a);
          cmax[colidx[qq]] = std::max(cmax[colidx[qq]], a);
        }
      for (int i = 0; i < m; ++i) r[i] = std::sqrt(rmax[i] > 0.0 ? rmax[i] : 1.0);
      for (int j = 0; j < n; ++j) s[j] = std::sqrt(cmax[j] > 0.0 ? cmax[j] : 1.0);
      for (int i = 0; i < m; ++i)
        for (int qq = rowptr[i]; qq < rowptr[i + 1]; ++qq) val[qq] = val[qq] / (r[i] * s[colidx[qq]]);
      for (int i = 0; i < m; ++i) d_row[i] = d_row[i] / r[i];
      for (int j = 0; j < n; ++j) d_col[j] = d_col[j] / s[j];
    }
    if (opt.pock_chambolle) {
      // alpha = 1: row and column absolute sums, rows in index order
      std::vector<double> rs(m, 0.0), cs(n, 0.0);
      for (int i = 0; i < m; ++i)
        for (int qq = rowptr[i]; qq < rowptr[i + 1]; ++qq) {
          rs[i] += std::fabs(val[qq]);
          cs[colidx[qq]] += std::fabs(val[qq]);
        }
      for (int i = 0; i < m; ++i) r[i] = std::sqrt(rs[i] > 0.0 ? rs[i] : 1.0);
      for (int j = 0; j < n; ++j) s[j] = std::sqrt(cs[j] > 0.0 ? cs[j] : 1.0);
      for (int i = 0; i < m; ++i)
        for (int qq = rowptr[i]; qq < rowptr[i + 1]; ++qq) val[qq] = val[qq] / (r[i] * s[colidx[qq]]);
      for (int i = 0; i < m; ++i) d_row[i] = d_row[i] / r[i];
      for (int j = 0; j < n; ++j) d_col[j] = d_col[j] / s[j];
    }
  }
  if (scale) {
    for (int j = 0; j < n; ++j) {
      c[j] = c[j] * d_col[j];
      lo[j] = lo[j] / d_col[j];
      hi[j] = hi[j] / d_col[j];
    }
    for (int i = 0; i < m; ++i) q[i] = q[i] * d_row[i];
  }
  // ---- round to the working precision (the LP the device holds) ----
  if (!fp64) {
    auto r32 = [](std::vector<double>& v) {
      for (auto& x : v) x = (double)(float)x;
    };
    r32(val);
    r32(c);
    r32(q);
    r32(lo);
    r32(hi);
  }
  // ---- CSC copy (CSR of K^T), rows in increasing order within each column ----
  colptr.assign(n + 1, 0);
  for (int qq = 0; qq < nnz; ++qq) colptr[colidx[qq] + 1]++;
  for (int j = 0; j < n; ++j) colptr[j + 1] += colptr[j];
  rowidx.resize(nnz);
  valT.resize(nnz);
  {
    std::vector<int> fill(colptr.begin(), colptr.end() - 1);
    for (int i = 0; i < m; ++i)
      for (int qq = rowptr[i]; qq < rowptr[i + 1]; ++qq) {
        const int dst = fill[colidx[qq]]++;
        rowidx[dst] = i;
        valT[dst] = val[qq];
      }
  }
  // ---- D-hat (Remark se:Dhat_construction): x part from columns, y part from rows ----
  dhat.assign(N, 1.0);
  if (opt.dhat_mode != 0) {
    std::vector<double> cm(n, 0.0), rm(m, 0.0);
    for (int i = 0; i < m; ++i)
      for (int qq = rowptr[i]; qq < rowptr[i + 1]; ++qq) {
        const double a = std::fabs(val[qq]);
        rm[i] = std::max(rm[i], a);
        cm[colidx[qq]] = std::max(cm[colidx[qq]], a);
      }
    for (int j = 0; j < n; ++j) dhat[j] = std::sqrt(std::max(cm[j], 1e-10));
    for (int i = 0; i < m; ++i) dhat[n + i] = std::sqrt(std::max(rm[i], 1e-10));
    if (opt.dhat_mode == 2)
      for (auto& v : dhat) v = 1.0 / v;
  }
  qnorm = 0.0;
  for (double v : q) qnorm += v * v;
  qnorm = std::sqrt(qnorm);
  cnorm = 0.0;
  for (double v : c) cnorm += v * v;
  cnorm = std::sqrt(cnorm);
  // ---- device row orders and work tables ----
  std::vector<int> rmapA, rmapB, ptrA, idxA, ptrB, idxB;
  std::vector<double> valA, valB;
  reorder_rows(colptr, rowidx, valT, n, rmapA, ptrA, idxA, valA);
  reorder_rows(rowptr, colidx, val, m, rmapB, ptrB, idxB, valB);
  dev_ptrA = ptrA;
  dev_ptrB = ptrB;
  build_chunks(ptrA, n, chunksA, splitsA, npartsA, row_weight);
  build_chunks(ptrB, m, chunksB, splitsB, npartsB, row_weight);
  tiles.clear();
  for (int e = 0; e < N; e += MIX_TILE) {
    MixTile t{};
    t.e0 = e;
    t.e1 = std::min(N, e + MIX_TILE);
    tiles.push_back(t);
  }
  // ---- device copies ----
  const size_t ts = fp64 ? 8 : 4;
  d_rowptr.upload(ptrB.data(), ptrB.size() * 4, "rowptr");
  d_colidx.upload(idxB.data(), idxB.size() * 4, "colidx");
  d_colptr.upload(ptrA.data(), ptrA.size() * 4, "colptr");
  d_rowidx.upload(idxA.data(), idxA.size() * 4, "rowidx");
  d_rmapA.upload(rmapA.data(), rmapA.size() * 4, "column order");
  d_rmapB.upload(rmapB.data(), rmapB.size() * 4, "row order");
  if (fp64) {
    upload_as<double>(d_val, valB, "val");
    upload_as<double>(d_valT, valA, "valT");
    upload_as<double>(d_c, c, "c");
    upload_as<double>(d_lo, lo, "l");
    upload_as<double>(d_hi, hi, "u");
    upload_as<double>(d_q, q, "q");
    upload_as<double>(d_dhat, dhat, "dhat");
  } else {
    upload_as<float>(d_val, valB, "val");
    upload_as<float>(d_valT, valA, "valT");
    upload_as<float>(d_c, c, "c");
    upload_as<float>(d_lo, lo, "l");
    upload_as<float>(d_hi, hi, "u");
    upload_as<float>(d_q, q, "q");
    upload_as<float>(d_dhat, dhat, "dhat");
  }
  d_rowtype.upload(rowtype.data(), rowtype.size(), "rowtype");
  // ---- column panels of the dual product for large LPs without split rows:
  // the workgroups of panel p gather only the 1/np of x_bar it covers,
  // which stays in the L2s of the XCDs that run them ----
  const int np = panel_count(fp64);
  panels = (int64_t)nnz >= PANEL_MIN_NNZ && splitsB.empty() && n >= np * 1024;
  if (panels) {
    std::vector<int> pptr((size_t)np * (m + 1), 0), pidx(nnz);
    std::vector<double> pval(nnz);
    auto panel_of = [&](int col) { return (int)((int64_t)col * np / n); };
    std::vector<int64_t> cnt(np, 0);
    for (int q = 0; q < nnz; ++q) cnt[panel_of(idxB[q])]++;
    std::vector<int64_t> base(np + 1, 0);
    for (int p = 0; p < np; ++p) base[p + 1] = base[p] + cnt[p];
    std::vector<int64_t> fill(base.begin(), base.end() - 1);
    for (int r = 0; r < m; ++r) {
      for (int p = 0; p < np; ++p) pptr[(size_t)p * (m + 1) + r] = (int)fill[p];
      for (int q = ptrB[r]; q < ptrB[r + 1]; ++q) {
        const int p = panel_of(idxB[q]);
        pidx[fill[p]] = idxB[q];
        pval[fill[p]] = valB[q];
        ++fill[p];
      }
    }
    for (int p = 0; p < np; ++p) pptr[(size_t)p * (m + 1) + m] = (int)fill[p];
    d_pptr.upload(pptr.data(), pptr.size() * 4, "panel pointers");
    d_pidx.upload(pidx.data(), pidx.size() * 4, "panel indices");
    if (fp64)
      upload_as<double>(d_pval, pval, "panel values");
    else
      upload_as<float>(d_pval, pval, "panel values");
    d_part.alloc((size_t)2 * np * m * 8, "panel sums");
    // chunks of each panel for k_panel: consecutive rows, at most PANEL_ROWS
    // of them and CHUNK_NNZ entries; each listed as (first row, first entry),
    // the list of a panel closed by (m, the panel's end)
    std::vector<int> pchunk;
    int nlist = 0;
    for (int p = 0; p < np; ++p) {
      pcoff[p] = nlist;
      const int* pp = pptr.data() + (size_t)p * (m + 1);
      int r = 0;
      while (r < m) {
        pchunk.push_back(r);
        pchunk.push_back(pp[r]);
        ++nlist;
        int rows = 0, ent = 0;
        while (r < m && rows < PANEL_ROWS) {
          const int len = pp[r + 1] - pp[r];
          if (rows > 0 && ent + len > CHUNK_NNZ) break;
          ent += len;
          ++rows;
          ++r;
        }
      }
      pchunk.push_back(m);
      pchunk.push_back(pp[m]);
      ++nlist;
    }
    pcoff[np] = nlist;
    d_pchunk.upload(pchunk.data(), pchunk.size() * 4, "panel chunks");
    // the dual epilogue then only adds panel sums: chunks of BLOCK rows
    chunksBp.clear();
    for (int r = 0; r < m; r += BLOCK) {
      Chunk c{};
      c.kind = 0;
      c.r0 = r;
      c.r1 = std::min(m, r + BLOCK);
      c.k0 = ptrB[c.r0];
      c.k1 = ptrB[c.r1];
      c.tpr = 1;
      chunksBp.push_back(c);
    }
  }
  for (int p = 0; p < 2; ++p) {
    d_u[p].alloc(N * ts, "u");
    d_u[p].zero("u");
    d_g[p].alloc(N * ts, "g");
    d_g[p].zero("g");
  }
  d_xbar.alloc(n * ts, "xbar");
  d_hist_dG.alloc((size_t)opt.memory * N * ts, "history dG");
  d_hist_dG.zero("history dG");
  d_hist_W.alloc((size_t)opt.memory * N * ts, "history W");
  d_hist_W.zero("history W");
  d_lam.alloc(n * ts, "lambda");
  d_sc.alloc(sizeof(Scalars), "scalars");
  d_xfer.alloc((size_t)N * 8, "transfer buffer");
  if (opt.pw_period > 0) d_anchor.alloc(N * ts, "primal-weight anchor");
  if (opt.variant == AAPDHG_VARIANT_RPDHG) d_rsum.alloc(N * 8, "restart epoch sum");
  fill_desc();
  // ---- step size (Section 5.1): tau = sigma = 0.9 / ||K||_2 by power iteration ----
  norm_est = power_norm();
  if (!(norm_est > 0.0)) {
    // the iteration found nothing: K = 0, or (measure zero for a random start)
    // a start in the null space of K; the Frobenius norm bounds ||K||_2 above
    double f2 = 0.0;
    for (const double v : val) f2 += v * v;
    norm_est = std::sqrt(f2);
  }
  if (opt.tau <= 0.0 || opt.sigma <= 0.0) {
    if (!(norm_est > 0.0)) {
      opt.tau = opt.sigma = 1.0;  // K = 0: any step satisfies the assumption
    } else {
      opt.tau = opt.sigma = 0.9 / norm_est;
    }
  } else if (norm_est > 0.0 && opt.tau * opt.sigma * norm_est * norm_est >= 1.0) {
    throw Error(AAPDHG_E_ARG, "tau * sigma * ||K||^2 = %g must be < 1 (||K|| ~ %g)",
                opt.tau * opt.sigma * norm_est * norm_est, norm_est);
  }
  fill_desc();
  set_gram_mode();
  d_desc.upload(&desc, sizeof desc, "descriptor");
  solo = std::make_unique<LaunchSet>();
  std::vector<Problem*> one{this};
  solo->build(one);
  reset_host_state();
  if (opt.autotune) autotune();
}

// The work tables again, after row_weight or the launch options changed:
// the multi-row chunks of both passes and the LP's own launch set.
void Problem::rebuild_tables() {
  build_chunks(dev_ptrA, n, chunksA, splitsA, npartsA, row_weight);
  build_chunks(dev_ptrB, m, chunksB, splitsB, npartsB, row_weight);
  set_gram_mode();
  solo = std::make_unique<LaunchSet>();
  std::vector<Problem*> one{this};
  solo->build(one);
}

// Whether the three-launch passes form the Gram matrix on demand (option
// gram_mode; by default only for an LP that the persistent kernel cannot
// take by itself, by the rule LaunchSet::build applies to a set of one).
void Problem::set_gram_mode() {
  bool lazy = opt.gram_mode == 2;
  if (opt.gram_mode == 0) {
    bool alone = opt.loop_kernel == 0;
    if (alone) {
      const bool ext = opt.pw_period > 0 || opt.variant == AAPDHG_VARIANT_RPDHG;
      const int cap = loop_capacity(fp64, std::max(1, opt.memory), ext);
      const long long need = (long long)std::max(chunksA.size(), chunksB.size());
      alone = cap >= 1 && need <= 2LL * cap;
    }
    lazy = !alone;
  }
  desc.lazy_gram = lazy ? 1 : 0;
}

void Problem::fill_desc() {
  std::memset(&desc, 0, sizeof desc);
  desc.m = m;
  desc.n = n;
  desc.N = N;
  desc.M = opt.memory;
  desc.variant = opt.variant;
  desc.kkt_every = opt.kkt_every;
  desc.max_iter = opt.max_iter;
  desc.tau = opt.tau;
  desc.sigma = opt.sigma;
  if (opt.pw_omega0 > 0.0 && opt.tau > 0.0 && opt.sigma > 0.0) {
    // tau = gamma / omega^0, sigma = gamma omega^0 with gamma = sqrt(tau sigma)
    const double gam = std::sqrt(opt.tau * opt.sigma);
    desc.tau = gam / opt.pw_omega0;
    desc.sigma = gam * opt.pw_omega0;
  }
  desc.beta = opt.beta;
  desc.D = opt.D;
  desc.eps_sg = opt.eps_sg;
  desc.eta = opt.eta;
  desc.cs = opt.cs;
  desc.kappa_bar = opt.kappa_bar;
  desc.angle_mode = opt.angle_mode;
  desc.length_floor = opt.length_floor;
  desc.tol = opt.tol;
  desc.sg_div = opt.sg_div;
  desc.pw_period = opt.pw_period;
  desc.pw_dhat = opt.pw_dhat;
  desc.pw_theta = opt.pw_theta;
  desc.pw_eps0 = opt.pw_eps_zero;
  desc.pw_rho = opt.pw_rho;
  desc.anchor = d_anchor.p;
  desc.restart = opt.variant == AAPDHG_VARIANT_RPDHG ? opt.restart_period : 0;
  desc.rsum = (double*)d_rsum.p;
  desc.rowptr = (const int*)d_rowptr.p;
  desc.colidx = (const int*)d_colidx.p;
  desc.val = d_val.p;
  desc.colptr = (const int*)d_colptr.p;
  desc.rowidx = (const int*)d_rowidx.p;
  desc.valT = d_valT.p;
  desc.rmapA = (const int*)d_rmapA.p;
  desc.rmapB = (const int*)d_rmapB.p;
  desc.c = d_c.p;
  desc.lo = d_lo.p;
  desc.hi = d_hi.p;
  desc.q = d_q.p;
  desc.dhat = d_dhat.p;
  desc.rowtype = (const unsigned char*)d_rowtype.p;
  desc.u[0] = d_u[0].p;
  desc.u[1] = d_u[1].p;
  desc.g[0] = d_g[0].p;
  desc.g[1] = d_g[1].p;
  desc.xbar = d_xbar.p;
  desc.dG = d_hist_dG.p;
  desc.W = d_hist_W.p;
  desc.lam = d_lam.p;
  desc.sc = (Scalars*)d_sc.p;
  desc.panels = panels ? panel_count(fp64) : 0;
  desc.pptr = (const int*)d_pptr.p;
  desc.pidx = (const int*)d_pidx.p;
  desc.pval = d_pval.p;
  desc.part = (double*)d_part.p;
  desc.pchunk = (const int*)d_pchunk.p;
  for (int p = 0; p <= MAX_PANELS; ++p) desc.pcoff[p] = pcoff[p];
}

// The scaling loops of create() on the device: the CSR (float64 values) and
// the CSC order of its entries go up, the scaled values and the factors come
// back.
void Problem::scale_on_device() {
  std::vector<int> cptr(n + 1, 0), cperm(nnz);
  for (int qq = 0; qq < nnz; ++qq) cptr[colidx[qq] + 1]++;
  for (int j = 0; j < n; ++j) cptr[j + 1] += cptr[j];
  {
    std::vector<int> fill(cptr.begin(), cptr.end() - 1);
    for (int i = 0; i < m; ++i)
      for (int qq = rowptr[i]; qq < rowptr[i + 1]; ++qq) cperm[fill[colidx[qq]]++] = qq;
  }
  DevBuf b_rowptr, b_colidx, b_val, b_cptr, b_cperm, b_rfac, b_cfac, b_cmax, b_drow, b_dcol;
  b_rowptr.upload(rowptr.data(), rowptr.size() * 4, "scaling rowptr");
  b_colidx.upload(colidx.data(), std::max<size_t>(colidx.size(), 1) * 4, "scaling colidx");
  b_val.upload(val.data(), std::max<size_t>(val.size(), 1) * 8, "scaling values");
  b_cptr.upload(cptr.data(), cptr.size() * 4, "scaling column pointers");
  b_cperm.upload(cperm.data(), std::max<size_t>(cperm.size(), 1) * 4, "scaling column order");
  b_rfac.alloc((size_t)m * 8, "row factors");
  b_cfac.alloc((size_t)n * 8, "column factors");
  b_cmax.alloc((size_t)n * 8, "column maxima");
  b_drow.upload(d_row.data(), (size_t)m * 8, "d_row");
  b_dcol.upload(d_col.data(), (size_t)n * 8, "d_col");
  ScalingArgs a;
  a.m = m;
  a.n = n;
  a.rowptr = (const int*)b_rowptr.p;
  a.colidx = (const int*)b_colidx.p;
  a.val = (double*)b_val.p;
  a.cptr = (const int*)b_cptr.p;
  a.cperm = (const int*)b_cperm.p;
  a.rfac = (double*)b_rfac.p;
  a.cfac = (double*)b_cfac.p;
  a.cmax = (unsigned long long*)b_cmax.p;
  a.drow = (double*)b_drow.p;
  a.dcol = (double*)b_dcol.p;
  a.ruiz_iters = opt.ruiz_iters;
  a.pock_chambolle = opt.pock_chambolle != 0;
  hip_check(launch_scaling(a, g_setup_stream), "scaling launch");
  setup_download(val.data(), b_val.p, (size_t)nnz * 8, "scaled values");
  setup_download(d_row.data(), b_drow.p, (size_t)m * 8, "d_row");
  setup_download(d_col.data(), b_dcol.p, (size_t)n * 8, "d_col");
}

double Problem::power_norm() {
  DevBuf work, est;
  work.alloc(((size_t)2 * n + m + 1024) * 8, "power iteration work");
  est.alloc(((size_t)opt.power_iters + 1) * 8, "power iteration estimates");
  hip_check(launch_power_iteration(desc, fp64, opt.power_iters, opt.seed, (double*)work.p, (double*)est.p,
                                   g_setup_stream),
            "power iteration launch");
  std::vector<double> e(opt.power_iters + 1);
  setup_download(e.data(), est.p, e.size() * 8, "power iteration result");
  return std::sqrt(std::max(0.0, e.back()));
}

size_t Problem::device_bytes() const {
  size_t b = 0;
  const DevBuf* bufs[] = {&d_pptr, &d_pidx, &d_pval, &d_part, &d_pchunk,
                          &d_rowptr, &d_colidx, &d_val, &d_colptr, &d_rowidx, &d_valT, &d_rmapA, &d_rmapB, &d_c, &d_lo, &d_hi,
                          &d_q, &d_dhat, &d_rowtype, &d_u[0], &d_u[1], &d_g[0], &d_g[1], &d_xbar, &d_hist_dG,
                          &d_hist_W, &d_lam, &d_sc, &d_desc, &d_xfer, &d_anchor, &d_rsum, &d_scale};
  for (auto* p : bufs) b += p->bytes;
  if (solo) b += solo->device_bytes();
  return b;
}

void Problem::reset_host_state() {
  std::memset(&sc_init, 0, sizeof sc_init);
  sc_init.k = 0;
  sc_init.status = ST_RUNNING;
  sc_init.branch = BR_NONE;
  sc_init.nlive = 0;
  sc_init.newslot = 0;
  sc_init.qnorm = qnorm;
  sc_init.cnorm = cnorm;
  // primal weight (Alg 7): tau = gstep / omega, sigma = gstep * omega; the
  // given (or estimated) steps are used as they are until the first update
  sc_init.gstep = std::sqrt(opt.tau * opt.sigma);
  sc_init.omega = opt.pw_omega0 > 0.0 ? opt.pw_omega0 : std::sqrt(opt.sigma / opt.tau);
  sc_init.tau = opt.pw_omega0 > 0.0 ? sc_init.gstep / sc_init.omega : opt.tau;
  sc_init.sigma = opt.pw_omega0 > 0.0 ? sc_init.gstep * sc_init.omega : opt.sigma;
  sc_init.dha[0] = sc_init.dha[1] = 1.0;
  sc_init.dhb[0] = sc_init.dhb[1] = 0.0;
  sc_init.pw_updates = 0;
  sc_init.faa_empty = 0;
  sc_init.gram_ok = 1;  // empty memory
  sc_init.pw_flag = 0;
  sc_init.pw_blend = 0;
}

void Problem::enqueue_reset(hipStream_t st) {
  hip_check(hipMemcpyAsync(d_sc.p, &sc_init, sizeof sc_init, hipMemcpyHostToDevice, st), "reset scalars");
  hip_check(launch_start_point(desc, fp64, st), "start point");
  started = true;
  pending_init = true;
}

// The passes of aapdhg_iterate with the per-pass scratch of the launch
// tables (partial-sum records, decision partials and counters, split,
// weight-check and Gram-launch partials and counters and, for the persistent
// kernel, its barrier counters, published decisions, weight-check partials
// and error word) in
// the library's static device array instead of the handle's buffers.
// Nothing is allocated: the array's used range is cleared by a fill kernel
// on `st`, then the passes are enqueued.
void Problem::iterate_noalloc(hipStream_t st, int64_t iters) {
  void* base = nullptr;
  hip_check(static_scratch(&base), "static scratch address");
  LaunchSet& L = *solo;
  LaunchTables t = L.t;
  size_t off = 0;
  auto take = [&](const DevBuf& b) -> void* {
    if (!b.p) return nullptr;
    void* p = (char*)base + off;
    off += (b.bytes + 255) & ~(size_t)255;
    return p;
  };
  t.rec = (double*)take(L.d_rec);
  t.dpart = (double*)take(L.d_dpart);
  t.dcnt = (unsigned int*)take(L.d_dcnt);
  t.splitpart = (double*)take(L.d_splitpart);
  t.splitcnt = (unsigned int*)take(L.d_splitcnt);
  t.pwpart = (double*)take(L.d_pwpart);
  t.pwcnt = (unsigned int*)take(L.d_pwcnt);
  t.gpart = (double*)take(L.d_gpart);
  t.gcnt = (unsigned int*)take(L.d_gcnt);
  if (t.persistent) {
    t.sync = (LoopSync*)take(L.d_sync);
    t.bc = (BcastMsg*)take(L.d_bc);
    t.err = (int*)take(L.d_err);
    t.pwrec = (double*)take(L.d_pwrec);
  }
  if (off > STATIC_SCRATCH_BYTES)
    throw Error(AAPDHG_E_ARG, "this LP needs %zu bytes of pass scratch; the no-allocation entry point has %zu",
                off, STATIC_SCRATCH_BYTES);
  hip_check(launch_zero(base, off, st), "clear static scratch");
  if (!started) enqueue_reset(st);
  if (pending_init && iters > 0) {  // the init step is the first pass
    hip_check(launch_loop_pass(t, st, MODE_ITER), "initial pass");
    pending_init = false;
    --iters;
  }
  if (t.persistent) {
    for (int64_t done = 0; done < iters;) {
      const int64_t np = std::min<int64_t>(iters - done, LaunchSet::MAX_LOOP_PASSES);
      hip_check(launch_loop(t, st, np, L.next_tag()), "loop launch");
      done += np;
    }
    return;
  }
  for (int64_t it = 0; it < iters; ++it) hip_check(launch_loop_pass(t, st, MODE_ITER), "loop pass");
}

// Alg 2 set-up: u^1 = T u^0, g^0 and ||g^0|| (the pass with k = 0), on the
// LP's own three-launch tables.
void Problem::enqueue_init(hipStream_t st) {
  if (!pending_init) return;
  hip_check(launch_loop_pass(solo->t, st, MODE_ITER), "initial pass");
  pending_init = false;
}

// ---------------------------------------------------------------------------
// launch sets
// ---------------------------------------------------------------------------

LaunchSet::~LaunchSet() {
  drop_graph();
  if (h_status) (void)hipHostFree(h_status);
}

void LaunchSet::drop_graph() {
  if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
  graph_exec = nullptr;
  graph_passes = 0;
}

// Capture `iters` three-launch loop passes on a private stream and
// instantiate the graph; replays run the same kernels with the same
// arguments (every table and state they read is in device memory).
void LaunchSet::build_graph(int64_t iters) {
  drop_graph();
  hipStream_t cap = nullptr;
  hip_check(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "capture stream");
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t el = hipSuccess;
    for (int64_t it = 0; it < iters && el == hipSuccess; ++it) el = launch_loop_pass(t, cap, MODE_ITER);
    e = hipStreamEndCapture(cap, &g);
    if (el != hipSuccess) e = el;
  }
  (void)hipStreamDestroy(cap);
  if (e == hipSuccess) e = hipGraphInstantiate(&graph_exec, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess) graph_exec = nullptr;
  hip_check(e, "graph capture of the loop passes");
  graph_passes = iters;
}

size_t LaunchSet::device_bytes() const {
  size_t b = 0;
  const DevBuf* bufs[] = {&d_lps, &d_llp, &d_chunks, &d_blocksA, &d_blocksB, &d_dblocks, &d_splits, &d_rec,
                          &d_dpart, &d_dcnt, &d_splitpart, &d_splitcnt, &d_tiles, &d_status, &d_wgs, &d_looplps,
                          &d_sync, &d_bc, &d_err, &d_pwpart, &d_pwcnt, &d_pwrec, &d_gpart, &d_gcnt};
  for (auto* p : bufs) b += p->bytes;
  return b;
}

void LaunchSet::build(const std::vector<Problem*>& lps) {
  drop_graph();
  members = lps;
  const int count = (int)lps.size();
  if (count == 0) throw Error(AAPDHG_E_ARG, "empty launch set");
  if (count > MAX_STATUS) throw Error(AAPDHG_E_ARG, "at most %d problems per batch", MAX_STATUS);
  std::vector<LPDesc> descs;
  std::vector<LaunchLP> llp(count);
  std::vector<Chunk> chunks;
  std::vector<BlockWork> bA, bB;
  std::vector<DecideBlock> dblocks;
  std::vector<SplitRow> splits;
  std::vector<MixTile> tl;
  t = LaunchTables{};
  t.fp64 = lps[0]->fp64;
  int mt = 1;
  for (auto* p : lps) mt = std::max(mt, p->opt.memory);
  // The persistent loop kernel pays off while every resident workgroup has
  // about one chunk per pass (then each workgroup owns one chunk); larger
  // sets use three launches per pass, which the hardware balances.
  bool want = true;
  long long need = 0;
  for (auto* p : lps) {
    want &= p->opt.loop_kernel == 0;
    need += (long long)std::max(p->chunksA.size(), p->chunksB.size());
  }
  bool ext = false;
  for (auto* p : lps) ext |= p->opt.pw_period > 0 || p->opt.variant == AAPDHG_VARIANT_RPDHG;
  const int cap = want ? loop_capacity(lps[0]->fp64, mt, ext) : 0;
  const bool persist = cap >= count && need <= 2LL * cap;
  int parts = 0;
  // per LP and pass: chunks, split rows, workgroups; leaves are the
  // workgroups followed by the split rows
  struct PassInfo {
    int b0, nb;   // workgroups in bA / bB (multi-row units)
    int bend;     // end of the LP's units (split parts follow the multi-row units)
    int s0, ns;   // split rows
    int leaf0;    // first leaf record
  };
  std::vector<PassInfo> info(2 * count);
  int nleaves = 0;
  for (int i = 0; i < count; ++i) {
    Problem* p = lps[i];
    if (p->fp64 != t.fp64) throw Error(AAPDHG_E_ARG, "all problems of a batch must share the precision");
    mt = std::max(mt, p->opt.memory);
    descs.push_back(p->desc);
    if (count > 1) descs.back().panels = 0;  // panels run only in a launch of their own
    for (int pass = 0; pass < 2; ++pass) {
      const auto& pc = pass == 0 ? p->chunksA : (count == 1 && p->panels ? p->chunksBp : p->chunksB);
      const auto& ps = pass == 0 ? p->splitsA : p->splitsB;
      const int np = pass == 0 ? p->npartsA : p->npartsB;
      auto& bw = pass == 0 ? bA : bB;
      PassInfo& pi = info[2 * i + pass];
      const int c_off = (int)chunks.size();
      pi.s0 = (int)splits.size();
      pi.ns = (int)ps.size();
      for (auto sr : ps) {
        sr.part0 += parts;
        splits.push_back(sr);
      }
      parts += np;
      for (auto c : pc) {
        c.lp = i;
        if (c.kind == 1) c.split += pi.s0;
        chunks.push_back(c);
      }
      const int nch = (int)pc.size();
      int cpb = p->opt.chunks_per_block;
      if (cpb <= 0) {
        // group the LP's chunks so that its workgroups of the pass fit on the
        // device at once, in one round (the pass B kernel holds fewer per CU);
        // the count depends on the LP's own options only, so the LP's
        // reduction order is the same alone and in any batch
        int pcap = pass_capacity(p->fp64, p->opt.memory, pass, p->desc.lazy_gram == 0);
        if (pcap <= 0) pcap = 1024;
        cpb = std::max(1, (nch + pcap - 1) / pcap);
      }
      if (persist) cpb = 1;
      // workgroups: runs of up to cpb multi-row chunks (leaves, listed first),
      // then one workgroup per split-row part (no leaf of their own)
      pi.b0 = (int)bw.size();
      for (int c = 0; c < nch;) {
        if (pc[c].kind == 1) {
          ++c;
          continue;
        }
        BlockWork w{};
        w.lp = i;
        w.kind = 0;
        w.c0 = c_off + c;
        int e = c;
        while (e < nch && e - c < cpb && pc[e].kind == 0) ++e;
        w.c1 = c_off + e;
        bw.push_back(w);
        c = e;
      }
      pi.nb = (int)bw.size() - pi.b0;
      for (int c = 0; c < nch; ++c) {
        if (pc[c].kind != 1) continue;
        BlockWork w{};
        w.lp = i;
        w.kind = 1;
        w.c0 = w.c1 = c_off + c;
        w.leaf = -1;
        bw.push_back(w);
      }
      pi.bend = (int)bw.size();
      pi.leaf0 = nleaves;
      nleaves += pi.nb + pi.ns;
    }
    const int t0 = (int)tl.size();
    for (auto x : p->tiles) {
      x.sc = p->desc.sc;
      x.lp = i;
      x.t0 = t0;
      x.nt = (int)p->tiles.size();
      tl.push_back(x);
    }
  }
  // records and decision workgroups: every LP's records (its primal-pass
  // workgroups and split columns, then its dual-pass workgroups and split
  // rows) are added by DECIDE_RECORDS-position workgroups of the decision launch
  for (int i = 0; i < count; ++i) {
    PassInfo& pa = info[2 * i];
    PassInfo& pb = info[2 * i + 1];
    for (int b = 0; b < pa.nb; ++b) bA[pa.b0 + b].leaf = pa.leaf0 + b;
    for (int q = 0; q < pa.ns; ++q) splits[pa.s0 + q].leaf = pa.leaf0 + pa.nb + q;
    for (int b = 0; b < pb.nb; ++b) bB[pb.b0 + b].leaf = pb.leaf0 + b;
    for (int q = 0; q < pb.ns; ++q) splits[pb.s0 + q].leaf = pb.leaf0 + pb.nb + q;
    LaunchLP& L = llp[i];
    L.leafA = pa.leaf0;
    L.nA = pa.nb + pa.ns;
    L.leafB = pb.leaf0;
    L.nB = pb.nb + pb.ns;
    const int total = L.nA + L.nB;
    L.blk0 = (int)dblocks.size();
    L.nblk = std::max(1, (total + DECIDE_RECORDS - 1) / DECIDE_RECORDS);
    for (int g = 0; g < L.nblk; ++g) {
      DecideBlock d{};
      d.sc = lps[i]->desc.sc;
      d.lp = i;
      d.r0 = g * DECIDE_RECORDS;
      d.r1 = std::min(total, (g + 1) * DECIDE_RECORDS);
      d.slot = L.blk0 + g;
      d.leafA = L.leafA;
      d.nA = L.nA;
      d.leafB = L.leafB;
      d.blk0 = L.blk0;
      d.nblk = L.nblk;
      dblocks.push_back(d);
    }
  }
  t.mt = mt;
  t.ext = ext;
  t.panels = count == 1 && lps[0]->panels;
  t.nlps = count;
  d_lps.upload(descs.data(), descs.size() * sizeof(LPDesc), "lp table");
  d_llp.upload(llp.data(), llp.size() * sizeof(LaunchLP), "lp roots");
  d_chunks.upload(chunks.data(), chunks.size() * sizeof(Chunk), "chunks");
  d_blocksA.upload(bA.data(), bA.size() * sizeof(BlockWork), "workgroups A");
  d_blocksB.upload(bB.data(), bB.size() * sizeof(BlockWork), "workgroups B");
  d_dblocks.upload(dblocks.data(), dblocks.size() * sizeof(DecideBlock), "decision workgroups");
  d_splits.upload(splits.data(), std::max<size_t>(splits.size(), 1) * sizeof(SplitRow), "splits");
  d_rec.alloc((size_t)std::max(nleaves, 1) * NDOT * 8, "partial records");
  d_rec.zero("partial records");
  d_dpart.alloc(dblocks.size() * NDOT * 8, "decision partials");
  d_dcnt.alloc((size_t)count * 4, "decision counters");
  d_dcnt.zero("decision counters");
  d_splitpart.alloc((size_t)std::max(parts, 1) * 2 * 8, "split partials");
  d_splitcnt.alloc(std::max<size_t>(splits.size(), 1) * 4, "split counters");
  d_splitcnt.zero("split counters");
  d_tiles.upload(tl.data(), tl.size() * sizeof(MixTile), "mix tiles");
  d_pwpart.alloc(std::max<size_t>(tl.size(), 1) * 2 * 8, "weight-check partials");
  d_pwcnt.alloc((size_t)count * 4, "weight-check counters");
  d_pwcnt.zero("weight-check counters");
  d_gpart.alloc(std::max<size_t>(tl.size(), 1) * gram_partials_per_tile(mt) * 8, "Gram partials");
  d_gcnt.alloc((size_t)count * 4, "Gram counters");
  d_gcnt.zero("Gram counters");
  d_status.alloc(count * 4, "status");
  if (!h_status) hip_check(hipHostMalloc((void**)&h_status, sizeof(int) * 2 * MAX_STATUS, hipHostMallocDefault), "pinned status");
  t.lps = (const LPDesc*)d_lps.p;
  t.llp = (const LaunchLP*)d_llp.p;
  t.chunks = (const Chunk*)d_chunks.p;
  t.blocksA = (const BlockWork*)d_blocksA.p;
  t.nblocksA = (int)bA.size();
  t.blocksB = (const BlockWork*)d_blocksB.p;
  t.nblocksB = (int)bB.size();
  t.nleaves = nleaves;
  t.dblocks = (const DecideBlock*)d_dblocks.p;
  t.ndblocks = (int)dblocks.size();
  t.splits = (const SplitRow*)d_splits.p;
  t.rec = (double*)d_rec.p;
  t.dpart = (double*)d_dpart.p;
  t.dcnt = (unsigned int*)d_dcnt.p;
  t.splitpart = (double*)d_splitpart.p;
  t.splitcnt = (unsigned int*)d_splitcnt.p;
  t.tiles = (const MixTile*)d_tiles.p;
  t.ntiles = (int)tl.size();
  t.pwpart = (double*)d_pwpart.p;
  t.pwcnt = (unsigned int*)d_pwcnt.p;
  t.gpart = (double*)d_gpart.p;
  t.gcnt = (unsigned int*)d_gcnt.p;
  // the Gram launch serves the LPs that form the Gram matrix on demand; the
  // pass kernels form the per-pass dots when some LP needs them
  t.gram = false;
  t.dots = false;
  for (auto* p : lps) {
    const bool aa = p->opt.variant == AAPDHG_VARIANT_AA || p->opt.variant == AAPDHG_VARIANT_FAA;
    t.gram |= aa && p->desc.lazy_gram != 0;
    t.dots |= p->desc.lazy_gram == 0;
  }

  // ---- persistent loop kernel: a group of resident workgroups per LP ----
  t.persistent = false;
  use_graph = false;
  for (auto* p : lps) use_graph |= p->opt.graph != 0;
  if (!persist) return;
  use_graph = false;
  // cost of a unit (one chunk): a chunk's dependent chain of loads costs
  // about as much as 3000 gathered entries
  auto unit_weight = [&](const BlockWork& w) -> double {
    const Chunk& ch = chunks[w.c0];
    return 3000.0 + (double)(ch.k1 - ch.k0) + (w.kind == 1 ? 0.0 : 2.0 * (ch.r1 - ch.r0));
  };
  std::vector<double> wlp(count);
  std::vector<int> umax(count), G(count);
  double wtot = 0.0;
  for (int i = 0; i < count; ++i) {
    double wa = 0.0, wb = 0.0;
    for (int u = info[2 * i].b0; u < info[2 * i].bend; ++u) wa += unit_weight(bA[u]);
    for (int u = info[2 * i + 1].b0; u < info[2 * i + 1].bend; ++u) wb += unit_weight(bB[u]);
    wlp[i] = std::max(wa, wb);
    umax[i] = std::max(info[2 * i].bend - info[2 * i].b0, info[2 * i + 1].bend - info[2 * i + 1].b0);
    wtot += wlp[i];
  }
  int gsum = 0;
  for (int i = 0; i < count; ++i) {
    // with room, rank 0 (which takes the decisions) gets no CSR unit
    const int nb = info[2 * i + 1].bend - info[2 * i + 1].b0;
    G[i] = need + count <= cap ? std::max(1, std::max(umax[i], nb + 1))
                               : std::max(1, std::min(umax[i], (int)std::floor((double)cap * wlp[i] / wtot)));
    gsum += G[i];
  }
  while (gsum > cap) {  // trim the largest groups
    int big = 0;
    for (int i = 1; i < count; ++i)
      if (G[i] > G[big]) big = i;
    --G[big];
    --gsum;
  }
  // units of rank j: a contiguous run, cut by cumulative weight
  auto assign = [&](const std::vector<BlockWork>& bw, int u0, int u1, int g, std::vector<int>& first, int skip) {
    first.assign(g + 1, u1);
    if (u1 - u0 <= g - skip) {  // one unit per workgroup, none for the first `skip` ranks
      for (int q = 0; q <= g; ++q) first[q] = std::min(u1, u0 + std::max(0, q - skip));
      return;
    }
    double tot = 0.0;
    for (int u = u0; u < u1; ++u) tot += unit_weight(bw[u]);
    double cum = 0.0;
    int rank_prev = -1;
    for (int u = u0; u < u1; ++u) {
      const double w = unit_weight(bw[u]);
      const int r = std::min(g - 1, (int)((cum + 0.5 * w) * g / tot));
      for (int q = rank_prev + 1; q <= r; ++q) first[q] = u;
      rank_prev = std::max(rank_prev, r);
      cum += w;
    }
    for (int q = rank_prev + 1; q <= g; ++q) first[q] = u1;
  };
  std::vector<LoopWG> wgs;
  std::vector<LoopLP> llps(count);
  std::vector<int> fa, fb;
  for (int i = 0; i < count; ++i) {
    const PassInfo& pa = info[2 * i];
    const PassInfo& pb = info[2 * i + 1];
    assign(bA, pa.b0, pa.bend, G[i], fa, 0);
    assign(bB, pb.b0, pb.bend, G[i], fb, 1);
    for (int j = 0; j < G[i]; ++j) {
      LoopWG w{};
      w.lp = i;
      w.rank = j;
      w.a0 = fa[j];
      w.a1 = fa[j + 1];
      w.b0 = fb[j];
      w.b1 = fb[j + 1];
      wgs.push_back(w);
    }
    llps[i].nwg = G[i];
    llps[i].wg0 = (int)wgs.size() - G[i];
    llps[i].leaf0 = pa.leaf0;
    llps[i].nleafA = pa.nb + pa.ns;
    llps[i].nleaf = pb.leaf0 + pb.nb + pb.ns - pa.leaf0;
  }
  d_wgs.upload(wgs.data(), wgs.size() * sizeof(LoopWG), "loop workgroups");
  d_looplps.upload(llps.data(), llps.size() * sizeof(LoopLP), "loop groups");
  d_sync.alloc(sizeof(LoopSync) * (size_t)count, "loop counters");
  d_bc.alloc(sizeof(BcastMsg) * (size_t)count, "loop decisions");
  d_bc.zero("loop decisions");
  d_err.alloc(sizeof(int), "loop error word");
  d_err.zero("loop error word");
  d_pwrec.alloc(wgs.size() * 2 * 8, "loop weight-check partials");
  int dev = 0, khz = 0;
  hip_check(hipGetDevice(&dev), "device");
  hip_check(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev), "wall clock rate");
  long long wait_us = 0;
  for (auto* p : lps) wait_us = std::max<long long>(wait_us, p->opt.wait_limit_us);
  if (wait_us == 0) wait_us = 4000000;
  // wall-clock ticks: khz per millisecond
  t.timeout_ticks = std::max<unsigned long long>(1ull, (unsigned long long)std::max(khz, 1) * (unsigned long long)wait_us / 1000ull);
  t.wgs = (const LoopWG*)d_wgs.p;
  t.nwgs = (int)wgs.size();
  t.looplps = (const LoopLP*)d_looplps.p;
  t.sync = (LoopSync*)d_sync.p;
  t.bc = (BcastMsg*)d_bc.p;
  t.pwrec = (double*)d_pwrec.p;
  t.err = (int*)d_err.p;
  t.persistent = true;
}

// Raise if a wait of the persistent loop kernel gave up (the LPs it served
// were stopped with status NUMERICAL).
void LaunchSet::check_loop_error(hipStream_t st) {
  if (!t.persistent) return;
  int e = 0;
  hip_check(hipMemcpyAsync(&e, d_err.p, sizeof e, hipMemcpyDeviceToHost, st), "loop error word");
  hip_check(hipStreamSynchronize(st), "loop error sync");
  if (e != 0) {
    d_err.zero("loop error word");
    throw Error(AAPDHG_E_HIP, "a wait of the persistent loop kernel timed out");
  }
}

void LaunchSet::enqueue_passes(hipStream_t st, int64_t iters) {
  if (t.persistent) {
    for (int64_t done = 0; done < iters;) {
      const int64_t np = std::min<int64_t>(iters - done, MAX_LOOP_PASSES);
      hip_check(launch_loop(t, st, np, next_tag()), "loop launch");
      done += np;
    }
    return;
  }
  if (use_graph && iters > 1) {
    if (graph_passes != iters) build_graph(iters);
    hip_check(hipGraphLaunch(graph_exec, st), "graph launch");
    return;
  }
  for (int64_t it = 0; it < iters; ++it) hip_check(launch_loop_pass(t, st, MODE_ITER), "loop pass");
}

void LaunchSet::timed_passes(hipStream_t st, int64_t iters, double* ms4) {
  if (iters < 1) throw Error(AAPDHG_E_ARG, "iters must be >= 1");
  if (t.persistent) {
    if (iters > MAX_LOOP_PASSES) throw Error(AAPDHG_E_ARG, "at most %d passes per timed launch", (int)MAX_LOOP_PASSES);
    hipEvent_t ev[2];
    for (auto& e : ev) hip_check(hipEventCreate(&e), "event");
    hip_check(hipEventRecord(ev[0], st), "event record");
    hip_check(launch_loop(t, st, iters, next_tag()), "loop launch");
    hip_check(hipEventRecord(ev[1], st), "event record");
    hip_check(hipStreamSynchronize(st), "timed sync");
    float ms = 0.f;
    hip_check(hipEventElapsedTime(&ms, ev[0], ev[1]), "event time");
    for (auto& e : ev) (void)hipEventDestroy(e);
    ms4[0] = 1.0;
    ms4[1] = ms;
    ms4[2] = (double)iters;
    ms4[3] = 1.0;
    return;
  }
  double* ms3 = ms4 + 1;
  ms4[0] = 0.0;
  std::vector<hipEvent_t> ev((size_t)iters * 4);
  for (auto& e : ev) hip_check(hipEventCreate(&e), "event");
  for (int64_t it = 0; it < iters; ++it) hip_check(launch_loop_pass(t, st, MODE_ITER, &ev[(size_t)it * 4]), "loop pass");
  hip_check(hipStreamSynchronize(st), "timed sync");
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t it = 0; it < iters; ++it)
    for (int q = 0; q < 3; ++q) {
      float ms = 0.f;
      hip_check(hipEventElapsedTime(&ms, ev[(size_t)it * 4 + q], ev[(size_t)it * 4 + q + 1]), "event time");
      acc[q] += ms;
    }
  for (auto& e : ev) (void)hipEventDestroy(e);
  for (int q = 0; q < 3; ++q) ms3[q] = acc[q] / (double)iters;
}

void LaunchSet::enqueue_eval(hipStream_t st) { hip_check(launch_loop_pass(t, st, MODE_EVAL), "evaluation pass"); }

// Run epochs until every member has stopped.  The status of epoch e is read
// while epoch e+1 is already queued, so the device does not wait for the host.
double LaunchSet::run_to_completion(hipStream_t st, int epoch, double time_limit_s, int compact_below,
                                    const std::chrono::steady_clock::time_point* t0p) {
  TraceRange tr("aapdhg solve");
  const auto t0 = t0p ? *t0p : std::chrono::steady_clock::now();
  compacted = false;
  const int count = t.nlps;
  hipEvent_t ev[2];
  hip_check(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming), "event");
  hip_check(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming), "event");
  int slot = 0;
  bool pending = false;
  int pend_slot = 0;
  bool done = false;
  int64_t epochs = 0;
  finish_s.assign(count, -1.0);
  while (!done) {
    roctxMark("aapdhg epoch");
    enqueue_passes(st, epoch);
    hip_check(launch_gather_status(t.lps, count, (int*)d_status.p, st), "status gather");
    hip_check(hipMemcpyAsync(h_status + slot * MAX_STATUS, d_status.p, count * 4, hipMemcpyDeviceToHost, st), "status copy");
    hip_check(hipEventRecord(ev[slot], st), "event record");
    ++epochs;
    if (pending) {
      hip_check(hipEventSynchronize(ev[pend_slot]), "event wait");
      int nrun = 0;
      const double now = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      for (int i = 0; i < count; ++i) {
        const bool run = h_status[pend_slot * MAX_STATUS + i] == ST_RUNNING;
        nrun += run ? 1 : 0;
        if (!run && finish_s[i] < 0.0) finish_s[i] = now;  // seen stopped at this status read
      }
      if (nrun == 0) done = true;
      if (nrun > 0 && nrun <= compact_below) {
        compacted = true;  // the caller continues with the running members only
        done = true;
      }
    }
    pending = true;
    pend_slot = slot;
    slot ^= 1;
    const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (!done && time_limit_s > 0.0 && el > time_limit_s) {
      hip_check(launch_time_limit(t.lps, count, st), "time limit");
      done = true;
    }
  }
  hip_check(hipStreamSynchronize(st), "solve sync");
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  last_epochs = epochs;
  const double total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (!compacted)
    for (auto& f : finish_s)
      if (f < 0.0) f = total;
  check_loop_error(st);
  return total;
}

// ---------------------------------------------------------------------------
// results
// ---------------------------------------------------------------------------

void Problem::read_scalars(Scalars& s) {
  hip_check(hipMemcpy(&s, d_sc.p, sizeof s, hipMemcpyDeviceToHost), "read scalars");
}

void Problem::download(const void* dev, size_t len, double* host, hipStream_t st) {
  hip_check(launch_to_f64(dev, fp64, (double*)d_xfer.p, len, st), "convert");
  hip_check(hipMemcpyAsync(host, d_xfer.p, len * 8, hipMemcpyDeviceToHost, st), "download");
  hip_check(hipStreamSynchronize(st), "download sync");
}

void Problem::upload_vec(void* dev, const double* host, size_t len, hipStream_t st) {
  hip_check(hipMemcpyAsync(d_xfer.p, host, len * 8, hipMemcpyHostToDevice, st), "upload");
  hip_check(launch_from_f64((const double*)d_xfer.p, dev, fp64, len, st), "convert");
  hip_check(hipStreamSynchronize(st), "upload sync");
}

static void fill_info(const Scalars& s, double secs, aapdhg_info* info) {
  std::memset(info, 0, sizeof *info);
  info->term = s.status;
  info->iters = s.k;
  info->aa_steps = s.i_aa;
  info->pdhg_steps = s.j_pdhg;
  info->primal_obj = s.pobj;
  info->dual_obj = s.dobj;
  info->r_gap = s.r_g;
  info->r_pri = s.r_p;
  info->r_dual = s.r_d;
  info->kkt = s.kkt;
  info->gnorm = s.gnorm;
  info->g0norm = s.n0;
  info->solve_seconds = secs;
  info->step_tau = s.tau;
  info->step_sigma = s.sigma;
  info->omega = s.omega;
  info->pw_updates = s.pw_updates;
  info->faa_empty = s.faa_empty;
}

// Results into caller device memory: the evaluation pass at the current
// iterate, then x, y, lambda unscaled and converted to float64 on `st`.
void Problem::result_device(double* x, double* y, double* lam, aapdhg_info* info, hipStream_t st) {
  hip_check(hipDeviceSynchronize(), "result sync");
  if (!started) throw Error(AAPDHG_E_STATE, "no solve has been run on this handle");
  solo->enqueue_eval(nullptr);
  hip_check(hipStreamSynchronize(nullptr), "evaluation sync");
  Scalars s;
  read_scalars(s);
  if (!d_scale.p) {
    std::vector<double> sc(N);
    std::copy(d_col.begin(), d_col.end(), sc.begin());
    std::copy(d_row.begin(), d_row.end(), sc.begin() + n);
    d_scale.upload(sc.data(), sc.size() * 8, "scaling factors");
  }
  hip_check(launch_unscale(d_u[(int)(s.k & 1)].p, d_lam.p, (const double*)d_scale.p, fp64, n, m, x, y, lam, st),
            "unscale launch");
  if (info) {
    fill_info(s, last_solve_seconds, info);
    info->gram_on_demand = desc.lazy_gram;
  }
}

void Problem::result(double* x, double* y, double* lam, aapdhg_info* info, bool run_eval) {
  hip_check(hipDeviceSynchronize(), "result sync");
  if (!started) throw Error(AAPDHG_E_STATE, "no solve has been run on this handle");
  if (run_eval) {
    solo->enqueue_eval(nullptr);
    hip_check(hipStreamSynchronize(nullptr), "evaluation sync");
  }
  Scalars s;
  read_scalars(s);
  const int par = (int)(s.k & 1);
  const size_t ts = fp64 ? 8 : 4;
  std::vector<double> u(N);
  download(d_u[par].p, N, u.data(), nullptr);
  if (x)
    for (int j = 0; j < n; ++j) x[j] = u[j] * d_col[j];
  if (y)
    for (int i = 0; i < m; ++i) y[i] = u[n + i] * d_row[i];
  if (lam) {
    std::vector<double> l(n);
    download(d_lam.p, n, l.data(), nullptr);
    for (int j = 0; j < n; ++j) lam[j] = l[j] / d_col[j];
  }
  (void)ts;
  if (info) {
    fill_info(s, last_solve_seconds, info);
    info->gram_on_demand = desc.lazy_gram;
  }
}

// primal-weight state: see aapdhg_get_weights in aapdhg.h
void Problem::get_weights(double* anchor, double* w) {
  hip_check(hipDeviceSynchronize(), "weight sync");
  Scalars s;
  read_scalars(s);
  if (w) {
    const double v[AAPDHG_WEIGHT_WORDS] = {s.omega,  s.gstep,  s.tau,    s.sigma,   s.dha[0],
                                           s.dha[1], s.dhb[0], s.dhb[1], (double)s.pw_updates, (double)s.pw_flag};
    std::memcpy(w, v, sizeof v);
  }
  if (anchor) {
    if (!d_anchor.p) throw Error(AAPDHG_E_STATE, "the primal-weight update is off (pw_period = 0): no anchor");
    download(d_anchor.p, N, anchor, nullptr);
  }
}

void Problem::set_weights(const double* anchor, const double* w) {
  if (!w) throw Error(AAPDHG_E_ARG, "set_weights needs the weight words");
  if (!(w[0] > 0.0) || !(w[1] > 0.0) || !(w[2] > 0.0) || !(w[3] > 0.0) || !(w[8] >= 0.0) ||
      (w[9] != 0.0 && w[9] != 1.0))
    throw Error(AAPDHG_E_ARG, "invalid primal-weight state");
  hip_check(hipDeviceSynchronize(), "weight sync");
  if (anchor) {
    if (!d_anchor.p) throw Error(AAPDHG_E_STATE, "the primal-weight update is off (pw_period = 0): no anchor");
    upload_vec(d_anchor.p, anchor, N, nullptr);
  }
  Scalars s;
  read_scalars(s);
  s.omega = w[0];
  s.gstep = w[1];
  s.tau = w[2];
  s.sigma = w[3];
  s.dha[0] = w[4];
  s.dha[1] = w[5];
  s.dhb[0] = w[6];
  s.dhb[1] = w[7];
  s.pw_updates = (long long)w[8];
  s.pw_flag = (int)w[9];
  hip_check(hipMemcpy(d_sc.p, &s, sizeof s, hipMemcpyHostToDevice), "write scalars");
}

// checkpoint layout: see aapdhg_get_state in aapdhg.h
void Problem::get_state(double* u, double* u_prev, double* g_prev, double* dG, double* W, int64_t* meta,
                        double* gram) {
  hip_check(hipDeviceSynchronize(), "state sync");
  // G and rhs as the persistent kernel keeps them (three-launch passes leave them stale)
  hip_check(launch_gram_refresh(solo->t, nullptr), "Gram refresh");
  hip_check(hipDeviceSynchronize(), "state sync");
  Scalars s;
  read_scalars(s);
  const int par = (int)(s.k & 1);
  if (u) download(d_u[par].p, N, u, nullptr);
  if (u_prev) download(d_u[par ^ 1].p, N, u_prev, nullptr);
  if (g_prev) download(d_g[par ^ 1].p, N, g_prev, nullptr);
  const size_t ts = fp64 ? 8 : 4;
  for (int sl = 0; sl < opt.memory; ++sl) {
    if (dG) download((char*)d_hist_dG.p + (size_t)sl * N * ts, N, dG + (size_t)sl * N, nullptr);
    if (W) download((char*)d_hist_W.p + (size_t)sl * N * ts, N, W + (size_t)sl * N, nullptr);
  }
  if (meta) {
    std::memset(meta, 0, sizeof(int64_t) * (8 + 2 * MAXM));
    meta[0] = s.k;
    meta[1] = s.status;
    meta[2] = s.i_aa;
    meta[3] = s.j_pdhg;
    meta[4] = s.nlive;
    meta[5] = s.newslot;
    meta[6] = s.branch;
    meta[7] = s.nmix;
    for (int t = 0; t < MAXM; ++t) meta[8 + t] = s.live[t];
    for (int t = 0; t < s.nmix && t < MAXM; ++t) meta[8 + MAXM + t] = s.mixslot[t];
  }
  if (gram) {
    std::memcpy(gram, s.G, sizeof s.G);
    std::memcpy(gram + MAXM * MAXM, s.rhs, sizeof s.rhs);
    std::memcpy(gram + MAXM * MAXM + MAXM, s.du2, sizeof s.du2);
    gram[MAXM * MAXM + 2 * MAXM] = s.n0;
    gram[MAXM * MAXM + 2 * MAXM + 1] = s.gnorm;
    for (int t = 0; t < MAXM; ++t) gram[MAXM * MAXM + 2 * MAXM + 2 + t] = t < s.nmix ? s.gamma[t] : 0.0;
  }
}

void Problem::set_state(const double* u, const double* u_prev, const double* g_prev, const double* dG,
                        const double* W, const int64_t* meta, const double* gram) {
  if (!meta || !gram || !u || !u_prev || !g_prev || !dG || !W)
    throw Error(AAPDHG_E_ARG, "set_state needs every buffer");
  hip_check(hipDeviceSynchronize(), "state sync");
  Scalars s = sc_init;
  s.k = meta[0];
  s.status = (int)meta[1];
  s.i_aa = meta[2];
  s.j_pdhg = meta[3];
  s.nlive = (int)meta[4];
  s.newslot = (int)meta[5];
  if (s.k < 1 || s.nlive < 0 || s.nlive > opt.memory || s.newslot < 0 || s.newslot >= opt.memory)
    throw Error(AAPDHG_E_ARG, "invalid state metadata");
  for (int t = 0; t < MAXM; ++t) s.live[t] = (int)meta[8 + t];
  for (int t = 0; t < s.nlive; ++t)
    if (s.live[t] < 0 || s.live[t] >= opt.memory) throw Error(AAPDHG_E_ARG, "invalid live slot");
  std::memcpy(s.G, gram, sizeof s.G);
  std::memcpy(s.rhs, gram + MAXM * MAXM, sizeof s.rhs);
  std::memcpy(s.du2, gram + MAXM * MAXM + MAXM, sizeof s.du2);
  s.n0 = gram[MAXM * MAXM + 2 * MAXM];
  s.gnorm = gram[MAXM * MAXM + 2 * MAXM + 1];
  s.branch = BR_PDHG;
  const int par = (int)(s.k & 1);
  upload_vec(d_u[par].p, u, N, nullptr);
  upload_vec(d_u[par ^ 1].p, u_prev, N, nullptr);
  upload_vec(d_g[par ^ 1].p, g_prev, N, nullptr);
  const size_t ts = fp64 ? 8 : 4;
  for (int sl = 0; sl < opt.memory; ++sl) {
    upload_vec((char*)d_hist_dG.p + (size_t)sl * N * ts, dG + (size_t)sl * N, N, nullptr);
    upload_vec((char*)d_hist_W.p + (size_t)sl * N * ts, W + (size_t)sl * N, N, nullptr);
  }
  hip_check(hipMemcpy(d_sc.p, &s, sizeof s, hipMemcpyHostToDevice), "write scalars");
  started = true;
  pending_init = false;
}

}  // namespace aapdhg

// ===========================================================================
// C ABI
// ===========================================================================

using namespace aapdhg;

struct aapdhg_problem {
  Problem p;
  std::string err;
  // aapdhg_solve runs its epochs on this thread; every other call on the
  // handle waits for it first (hguard)
  std::thread solver;
  aapdhg_status solve_status = AAPDHG_OK;
  std::string solve_msg;
  void join() {
    if (solver.joinable()) solver.join();
  }
};

struct aapdhg_batch {
  std::vector<aapdhg_problem*> members;
  LaunchSet set;
  std::string err;
};

template <typename F>
static aapdhg_status guard(std::string* err, F&& f) {
  try {
    f();
    return AAPDHG_OK;
  } catch (const Error& e) {
    if (err) *err = e.msg;
    g_thread_error = e.msg;
    return e.status;
  } catch (const std::bad_alloc&) {
    if (err) *err = "host allocation failed";
    g_thread_error = "host allocation failed";
    return AAPDHG_E_NOMEM;
  } catch (const std::exception& e) {
    if (err) *err = e.what();
    g_thread_error = e.what();
    return AAPDHG_E_ARG;
  }
}

// Entry points on a handle: wait for a solve in flight, then run f; a
// failure of that solve is reported by the first call after it.
template <typename F>
static aapdhg_status hguard(aapdhg_t h, F&& f) {
  h->join();
  if (h->solve_status != AAPDHG_OK) {
    const aapdhg_status s = h->solve_status;
    h->err = h->solve_msg;
    g_thread_error = h->solve_msg;
    h->solve_status = AAPDHG_OK;
    return s;
  }
  return guard(&h->err, std::forward<F>(f));
}

extern "C" {

void aapdhg_default_options(aapdhg_options* o) {
  if (o) default_options(o);
}

aapdhg_status aapdhg_create(int32_t m, int32_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                            const double* val, const double* c, const double* q, const double* l, const double* u,
                            const uint8_t* row_type, const aapdhg_options* opt, aapdhg_t* out) {
  if (!out) {
    g_thread_error = "out is NULL";
    return AAPDHG_E_ARG;
  }
  *out = nullptr;
  auto* h = new (std::nothrow) aapdhg_problem;
  if (!h) {
    g_thread_error = "host allocation failed";
    return AAPDHG_E_NOMEM;
  }
  aapdhg_status st = guard(nullptr, [&] { h->p.create(m, n, nnz, row_ptr, col_idx, val, c, q, l, u, row_type, opt); });
  if (st != AAPDHG_OK) {
    delete h;
    return st;
  }
  *out = h;
  return AAPDHG_OK;
}

aapdhg_status aapdhg_create_device(int32_t m, int32_t n, int64_t nnz, const int64_t* row_ptr,
                                   const int32_t* col_idx, const double* val, const double* c, const double* q,
                                   const double* l, const double* u, const uint8_t* row_type,
                                   const aapdhg_options* opt, void* stream, aapdhg_t* out) {
  if (!out) {
    g_thread_error = "out is NULL";
    return AAPDHG_E_ARG;
  }
  *out = nullptr;
  std::vector<int64_t> hp;
  std::vector<int32_t> hi;
  std::vector<double> hv, hc, hq, hl, hu;
  std::vector<uint8_t> ht;
  const aapdhg_status st0 = guard(nullptr, [&] {
    if (m < 1 || n < 1) throw Error(AAPDHG_E_ARG, "m and n must be >= 1 (m=%d n=%d)", m, n);
    if (nnz < 0 || nnz >= (int64_t)1 << 31) throw Error(AAPDHG_E_ARG, "nnz must be in [0, 2^31)");
    if (!row_ptr || (!col_idx && nnz) || (!val && nnz) || !c || !q || !l || !u || !row_type)
      throw Error(AAPDHG_E_ARG, "null input array");
    hipStream_t s = (hipStream_t)stream;
    // every range must lie inside one device allocation (checked before any
    // host buffer is sized): a short buffer is an argument error here rather
    // than a read past its end
    auto in_range = [&](const void* src, size_t bytes, const char* what) {
      if (!bytes) return;
      hipDeviceptr_t base = nullptr;
      size_t size = 0;
      if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)src) != hipSuccess || !base) {
        (void)hipGetLastError();
        throw Error(AAPDHG_E_ARG, "%s: not device memory", what);
      }
      if ((const char*)src + bytes > (const char*)base + size)
        throw Error(AAPDHG_E_ARG, "%s: the allocation ends before the %zu bytes the sizes imply", what, bytes);
    };
    const size_t M = m, Nn = n, Z = (size_t)nnz;
    in_range(row_ptr, (M + 1) * 8, "row_ptr");
    in_range(col_idx, Z * 4, "col_idx");
    in_range(val, Z * 8, "val");
    in_range(c, Nn * 8, "c");
    in_range(q, M * 8, "q");
    in_range(l, Nn * 8, "l");
    in_range(u, Nn * 8, "u");
    in_range(row_type, M, "row_type");
    hp.resize(M + 1);
    hi.resize(Z);
    hv.resize(Z);
    hc.resize(Nn);
    hl.resize(Nn);
    hu.resize(Nn);
    hq.resize(M);
    ht.resize(M);
    auto get = [&](void* dst, const void* src, size_t bytes, const char* what) {
      if (bytes) hip_check(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s), what);
    };
    get(hp.data(), row_ptr, hp.size() * 8, "row_ptr from device");
    get(hi.data(), col_idx, hi.size() * 4, "col_idx from device");
    get(hv.data(), val, hv.size() * 8, "val from device");
    get(hc.data(), c, hc.size() * 8, "c from device");
    get(hq.data(), q, hq.size() * 8, "q from device");
    get(hl.data(), l, hl.size() * 8, "l from device");
    get(hu.data(), u, hu.size() * 8, "u from device");
    get(ht.data(), row_type, ht.size(), "row_type from device");
    hip_check(hipStreamSynchronize(s), "device input sync");
  });
  if (st0 != AAPDHG_OK) return st0;
  return aapdhg_create(m, n, nnz, hp.data(), hi.data(), hv.data(), hc.data(), hq.data(), hl.data(), hu.data(),
                       ht.data(), opt, out);
}

aapdhg_status aapdhg_result_device(aapdhg_t h, double* x, double* y, double* lambda, aapdhg_info* info,
                                   void* stream) {
  if (!h) return AAPDHG_E_ARG;
  return hguard(h, [&] { h->p.result_device(x, y, lambda, info, (hipStream_t)stream); });
}

aapdhg_status aapdhg_solve(aapdhg_t h, void* stream) {
  if (!h) return AAPDHG_E_ARG;
  return hguard(h, [&] {
    if (h->p.in_batch) throw Error(AAPDHG_E_STATE, "problem belongs to a live batch");
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    hip_check(hipGetDevice(&dev), "device");
    h->p.enqueue_reset(st);
    h->p.enqueue_init(st);
    // the epochs are enqueued by a thread of the handle: the call returns
    // at once; termination is decided on the device (the status each pass
    // leaves in the LP's scalars), the thread only stops enqueuing
    h->solver = std::thread([h, st, dev] {
      h->solve_status = guard(&h->solve_msg, [&] {
        hip_check(hipSetDevice(dev), "solve device");
        h->p.last_solve_seconds = h->p.solo->run_to_completion(st, h->p.opt.epoch, h->p.opt.time_limit_s);
      });
    });
  });
}

aapdhg_status aapdhg_wait(aapdhg_t h) {
  if (!h) return AAPDHG_E_ARG;
  return hguard(h, [] {});
}

aapdhg_status aapdhg_iterate(aapdhg_t h, void* stream, int64_t iters) {
  if (!h) return AAPDHG_E_ARG;
  return hguard(h, [&] {
    if (iters < 0) throw Error(AAPDHG_E_ARG, "iters must be >= 0");
    if (h->p.in_batch) throw Error(AAPDHG_E_STATE, "problem belongs to a live batch");
    hipStream_t st = (hipStream_t)stream;
    if (!h->p.started) h->p.enqueue_reset(st);
    if (h->p.pending_init && iters > 0) {  // the init step is the first pass
      h->p.enqueue_init(st);
      --iters;
    }
    h->p.solo->enqueue_passes(st, iters);
  });
}

aapdhg_status aapdhg_iterate_noalloc(aapdhg_t h, void* stream, int64_t iters) {
  if (!h) return AAPDHG_E_ARG;
  return hguard(h, [&] {
    if (iters < 0) throw Error(AAPDHG_E_ARG, "iters must be >= 0");
    if (h->p.in_batch) throw Error(AAPDHG_E_STATE, "problem belongs to a live batch");
    h->p.iterate_noalloc((hipStream_t)stream, iters);
  });
}

aapdhg_status aapdhg_iterate_timed(aapdhg_t h, void* stream, int64_t iters, double* ms4) {
  if (!h || !ms4) return AAPDHG_E_ARG;
  return hguard(h, [&] {
    if (h->p.in_batch) throw Error(AAPDHG_E_STATE, "problem belongs to a live batch");
    hipStream_t st = (hipStream_t)stream;
    if (!h->p.started) h->p.enqueue_reset(st);
    h->p.enqueue_init(st);
    h->p.solo->timed_passes(st, iters, ms4);
  });
}

aapdhg_status aapdhg_reset(aapdhg_t h, void* stream) {
  if (!h) return AAPDHG_E_ARG;
  return hguard(h, [&] { h->p.enqueue_reset((hipStream_t)stream); });
}

aapdhg_status aapdhg_result(aapdhg_t h, double* x, double* y, double* lambda, aapdhg_info* info) {
  if (!h) return AAPDHG_E_ARG;
  return hguard(h, [&] { h->p.result(x, y, lambda, info, true); });
}

aapdhg_status aapdhg_get_state(aapdhg_t h, double* u, double* u_prev, double* g_prev, double* dG, double* W,
                               int64_t* meta, double* gram) {
  if (!h) return AAPDHG_E_ARG;
  return hguard(h, [&] { h->p.get_state(u, u_prev, g_prev, dG, W, meta, gram); });
}

aapdhg_status aapdhg_set_state(aapdhg_t h, const double* u, const double* u_prev, const double* g_prev,
                               const double* dG, const double* W, const int64_t* meta, const double* gram) {
  if (!h) return AAPDHG_E_ARG;
  return hguard(h, [&] { h->p.set_state(u, u_prev, g_prev, dG, W, meta, gram); });
}

aapdhg_status aapdhg_get_weights(aapdhg_t h, double* anchor, double* w) {
  if (!h) return AAPDHG_E_ARG;
  return hguard(h, [&] { h->p.get_weights(anchor, w); });
}

aapdhg_status aapdhg_set_weights(aapdhg_t h, const double* anchor, const double* w) {
  if (!h) return AAPDHG_E_ARG;
  return hguard(h, [&] { h->p.set_weights(anchor, w); });
}

aapdhg_status aapdhg_get_dims(aapdhg_t h, int32_t* m, int32_t* n, int64_t* nnz, double* tau, double* sigma) {
  if (!h) return AAPDHG_E_ARG;
  h->join();
  if (m) *m = h->p.m;
  if (n) *n = h->p.n;
  if (nnz) *nnz = h->p.nnz;
  if (tau) *tau = h->p.opt.tau;
  if (sigma) *sigma = h->p.opt.sigma;
  return AAPDHG_OK;
}

aapdhg_status aapdhg_get_scaling(aapdhg_t h, double* d_row, double* d_col) {
  if (!h) return AAPDHG_E_ARG;
  h->join();
  if (d_row) std::copy(h->p.d_row.begin(), h->p.d_row.end(), d_row);
  if (d_col) std::copy(h->p.d_col.begin(), h->p.d_col.end(), d_col);
  return AAPDHG_OK;
}

aapdhg_status aapdhg_destroy(aapdhg_t h) {
  if (!h) return AAPDHG_E_ARG;
  h->join();
  (void)hipDeviceSynchronize();
  delete h;
  return AAPDHG_OK;
}

const char* aapdhg_last_error(aapdhg_t h) {
  if (h) return h->err.c_str();
  return g_thread_error.c_str();
}

aapdhg_status aapdhg_batch_create(int32_t count, const aapdhg_t* problems, aapdhg_batch_t* out) {
  if (!out || !problems || count < 1) {
    g_thread_error = "invalid batch arguments";
    return AAPDHG_E_ARG;
  }
  *out = nullptr;
  auto* b = new (std::nothrow) aapdhg_batch;
  if (!b) return AAPDHG_E_NOMEM;
  aapdhg_status st = guard(nullptr, [&] {
    std::vector<Problem*> ps;
    for (int i = 0; i < count; ++i) {
      if (!problems[i]) throw Error(AAPDHG_E_ARG, "problem %d is NULL", i);
      problems[i]->join();  // a solve of its own in flight finishes first
      if (problems[i]->p.in_batch) throw Error(AAPDHG_E_STATE, "problem %d already belongs to a batch", i);
      for (int j = 0; j < i; ++j)
        if (problems[j] == problems[i]) throw Error(AAPDHG_E_ARG, "problem %d appears twice", i);
      ps.push_back(&problems[i]->p);
      b->members.push_back(problems[i]);
    }
    b->set.build(ps);
    for (auto* p : ps) p->in_batch = true;
  });
  if (st != AAPDHG_OK) {
    delete b;
    return st;
  }
  *out = b;
  return AAPDHG_OK;
}

aapdhg_status aapdhg_batch_solve(aapdhg_batch_t b, void* stream) {
  if (!b) return AAPDHG_E_ARG;
  return guard(&b->err, [&] {
    hipStream_t st = (hipStream_t)stream;
    int epoch = 1 << 30;
    double tl = 0.0;
    for (auto* h : b->members) {
      h->p.enqueue_reset(st);
      h->p.enqueue_init(st);
      epoch = std::min(epoch, h->p.opt.epoch);
      tl = std::max(tl, h->p.opt.time_limit_s);
    }
    // Members stop at different passes: once at most half of a set of 8 or
    // more is still running, the running members continue in a launch set of
    // their own (a small set fits the persistent loop kernel), so the passes
    // of the last stragglers do not pay for the launches of finished LPs.
    const auto t0 = std::chrono::steady_clock::now();
    const size_t nm = b->members.size();
    std::vector<double> fin(nm, -1.0);
    std::vector<size_t> idx(nm);
    for (size_t i = 0; i < nm; ++i) idx[i] = i;
    LaunchSet* cur = &b->set;
    std::unique_ptr<LaunchSet> sub;
    double total = 0.0;
    for (;;) {
      const int count = cur->t.nlps;
      const int below = count >= 8 ? count / 2 : 0;
      double left = 0.0;
      if (tl > 0.0) left = std::max(1e-9, tl - std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
      total = cur->run_to_completion(st, epoch, left, below, &t0);
      std::vector<Problem*> running;
      std::vector<size_t> ridx;
      for (int j = 0; j < count; ++j) {
        if (cur->finish_s[j] >= 0.0) {
          fin[idx[j]] = cur->finish_s[j];
        } else {
          running.push_back(&b->members[idx[j]]->p);
          ridx.push_back(idx[j]);
        }
      }
      if (!cur->compacted || running.empty()) break;
      auto next = std::make_unique<LaunchSet>();
      next->build(running);
      sub = std::move(next);
      cur = sub.get();
      idx = ridx;
    }
    for (size_t i = 0; i < nm; ++i) b->members[i]->p.last_solve_seconds = fin[i] >= 0.0 ? fin[i] : total;
  });
}

aapdhg_status aapdhg_batch_iterate(aapdhg_batch_t b, void* stream, int64_t iters) {
  if (!b) return AAPDHG_E_ARG;
  return guard(&b->err, [&] {
    if (iters < 0) throw Error(AAPDHG_E_ARG, "iters must be >= 0");
    hipStream_t st = (hipStream_t)stream;
    for (auto* h : b->members) {
      if (!h->p.started) h->p.enqueue_reset(st);
      h->p.enqueue_init(st);
    }
    b->set.enqueue_passes(st, iters);
  });
}

aapdhg_status aapdhg_batch_iterate_timed(aapdhg_batch_t b, void* stream, int64_t iters, double* ms4) {
  if (!b || !ms4) return AAPDHG_E_ARG;
  return guard(&b->err, [&] {
    hipStream_t st = (hipStream_t)stream;
    for (auto* h : b->members) {
      if (!h->p.started) h->p.enqueue_reset(st);
      h->p.enqueue_init(st);
    }
    b->set.timed_passes(st, iters, ms4);
  });
}

aapdhg_status aapdhg_batch_result(aapdhg_batch_t b, int32_t i, double* x, double* y, double* lambda,
                                  aapdhg_info* info) {
  if (!b) return AAPDHG_E_ARG;
  if (i < 0 || i >= (int32_t)b->members.size()) {
    g_thread_error = "batch member index out of range";
    return AAPDHG_E_ARG;
  }
  return aapdhg_result(b->members[i], x, y, lambda, info);
}

aapdhg_status aapdhg_batch_destroy(aapdhg_batch_t b) {
  if (!b) return AAPDHG_E_ARG;
  (void)hipDeviceSynchronize();
  for (auto* h : b->members) h->p.in_batch = false;
  delete b;
  return AAPDHG_OK;
}

}  // extern "C"
