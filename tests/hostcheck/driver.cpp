// Host-logic driver for the sanitizer build (AddressSanitizer + UBSan): the C
// ABI on ragged, empty, long-row, long-column and invalid LPs, batches, the
// no-allocation pass entry, checkpoints, device-memory entry points and the
// server's admission and retirement, against the CPU stand-in of the HIP
// runtime (hip_stub.cpp), whose kernels do nothing.  Exits 0 and prints
// "hostcheck ok" when every call returned what it should.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <random>
#include <thread>
#include <vector>

#include <hip/hip_runtime.h>

#include "aapdhg.h"

static int g_fail = 0;
#define CHECK(cond)                                                      \
  do {                                                                   \
    if (!(cond)) {                                                       \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      ++g_fail;                                                          \
    }                                                                    \
  } while (0)

// Allocation failure on demand, on this thread only: while g_fail_at is
// nonzero, operator new throws std::bad_alloc for requests of at least that
// many bytes (the library's host copies of a submission go through it).
static thread_local size_t g_fail_at = 0;
void* operator new(size_t sz) {
  if (g_fail_at && sz >= g_fail_at) throw std::bad_alloc();
  if (void* p = std::malloc(sz ? sz : 1)) return p;
  throw std::bad_alloc();
}
void* operator new(size_t sz, const std::nothrow_t&) noexcept {
  if (g_fail_at && sz >= g_fail_at) return nullptr;
  return std::malloc(sz ? sz : 1);
}
void operator delete(void* p) noexcept { std::free(p); }
void operator delete(void* p, size_t) noexcept { std::free(p); }
void operator delete(void* p, const std::nothrow_t&) noexcept { std::free(p); }

struct LP {
  int m = 0, n = 0;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  std::vector<double> val, c, q, l, u;
  std::vector<uint8_t> rt;
  int64_t nnz() const { return rowptr.back(); }
};

// rows of the given lengths, distinct random columns in random order
static LP make_lp(int n, const std::vector<int>& lens, unsigned seed) {
  LP p;
  std::mt19937 rng(seed);
  p.m = (int)lens.size();
  p.n = n;
  p.rowptr.push_back(0);
  std::vector<int> perm(n);
  for (int j = 0; j < n; ++j) perm[j] = j;
  for (int i = 0; i < p.m; ++i) {
    const int L = std::min(lens[i], n);
    for (int k = 0; k < L; ++k) std::swap(perm[k], perm[k + rng() % (n - k)]);
    for (int k = 0; k < L; ++k) {
      p.col.push_back(perm[k]);
      p.val.push_back(1.0 + (double)(rng() % 7) - 3.0 + 0.25);
    }
    p.rowptr.push_back((int64_t)p.col.size());
  }
  for (int j = 0; j < n; ++j) {
    p.c.push_back((double)(rng() % 5) - 2.0);
    const int kind = j % 3;
    p.l.push_back(kind == 2 ? -INFINITY : 0.0);
    p.u.push_back(kind == 0 ? 1.0 : INFINITY);
  }
  for (int i = 0; i < p.m; ++i) {
    p.q.push_back((double)(rng() % 3));
    p.rt.push_back((uint8_t)(i % 2));
  }
  return p;
}

static aapdhg_status create(const LP& p, const aapdhg_options* o, aapdhg_t* h) {
  return aapdhg_create(p.m, p.n, p.nnz(), p.rowptr.data(), p.col.data(), p.val.data(), p.c.data(), p.q.data(),
                       p.l.data(), p.u.data(), p.rt.data(), o, h);
}

static void exercise(const LP& p, aapdhg_options o) {
  aapdhg_t h = nullptr;
  CHECK(create(p, &o, &h) == AAPDHG_OK);
  if (!h) {
    std::fprintf(stderr, "create: %s\n", aapdhg_last_error(nullptr));
    return;
  }
  CHECK(aapdhg_iterate(h, nullptr, 3) == AAPDHG_OK);
  CHECK(aapdhg_iterate_noalloc(h, nullptr, 2) == AAPDHG_OK);
  double ms4[4];
  CHECK(aapdhg_iterate_timed(h, nullptr, 2, ms4) == AAPDHG_OK);
  std::vector<double> x(p.n), y(p.m), lam(p.n);
  aapdhg_info info;
  CHECK(aapdhg_result(h, x.data(), y.data(), lam.data(), &info) == AAPDHG_OK);
  const int M = o.memory, N = p.m + p.n;
  std::vector<double> uu(N), up(N), gp(N), dG((size_t)M * N), W((size_t)M * N),
      gram(AAPDHG_MAX_MEMORY * AAPDHG_MAX_MEMORY + 3 * AAPDHG_MAX_MEMORY + 2);
  std::vector<int64_t> meta(8 + 2 * AAPDHG_MAX_MEMORY);
  CHECK(aapdhg_get_state(h, uu.data(), up.data(), gp.data(), dG.data(), W.data(), meta.data(), gram.data()) ==
        AAPDHG_OK);
  meta[0] = 5;  // a valid k
  CHECK(aapdhg_set_state(h, uu.data(), up.data(), gp.data(), dG.data(), W.data(), meta.data(), gram.data()) ==
        AAPDHG_OK);
  meta[4] = M + 1;  // more live slots than the memory holds
  CHECK(aapdhg_set_state(h, uu.data(), up.data(), gp.data(), dG.data(), W.data(), meta.data(), gram.data()) ==
        AAPDHG_E_ARG);
  std::vector<double> dr(p.m), dc(p.n);
  CHECK(aapdhg_get_scaling(h, dr.data(), dc.data()) == AAPDHG_OK);
  CHECK(aapdhg_solve(h, nullptr) == AAPDHG_OK);
  CHECK(aapdhg_result(h, x.data(), y.data(), nullptr, &info) == AAPDHG_OK);
  CHECK(aapdhg_reset(h, nullptr) == AAPDHG_OK);
  CHECK(aapdhg_destroy(h) == AAPDHG_OK);
}

int main() {
  aapdhg_options o;
  aapdhg_default_options(&o);
  o.tau = o.sigma = 0.5;
  o.max_iter = 100;
  o.epoch = 8;

  // ragged: empty rows, a row split into parts (> 2048 entries), long rows
  // sharing a workgroup, one-entry rows; the last columns stay empty
  std::vector<int> lens;
  for (int i = 0; i < 300; ++i) lens.push_back(i % 7 == 0 ? 0 : 1 + i % 9);
  lens[5] = 5000;
  lens[6] = 1500;
  lens[7] = 300;
  lens[8] = 130;
  LP rag = make_lp(6000, lens, 1);
  exercise(rag, o);
  // float64, FAA, primal weights, restarts, Ruiz on the host and on the device, every loop kernel
  aapdhg_options o2 = o;
  o2.precision = 1;
  o2.variant = AAPDHG_VARIANT_FAA;
  o2.memory = 16;
  o2.loop_kernel = 1;
  exercise(rag, o2);
  aapdhg_options o3 = o;
  o3.pw_period = 4;
  o3.ruiz_iters = 10;
  o3.prep_device = 0;
  exercise(rag, o3);
  o3.prep_device = 1;
  o3.pock_chambolle = 1;
  o3.variant = AAPDHG_VARIANT_RPDHG;
  exercise(rag, o3);
  // captured passes and the autotuner (its cache in the working directory)
  aapdhg_options o4 = o;
  o4.graph = 1;
  o4.autotune = 1;
  o4.loop_kernel = 1;
  setenv("AAPDHG_TUNE_CACHE", "hostcheck_tune.txt", 1);
  exercise(rag, o4);
  exercise(rag, o4);  // the second takes the cached choice
  // the Gram matrix on demand for every three-launch set, and on every pass
  aapdhg_options o5 = o;
  o5.gram_mode = 2;
  exercise(rag, o5);
  o5.gram_mode = 1;
  o5.loop_kernel = 1;
  exercise(rag, o5);
  // transposed shape: columns longer than a chunk in the CSC pass
  std::vector<int> tall(4000, 3);
  LP tl = make_lp(40, tall, 2);
  exercise(tl, o);
  // no entries at all
  LP empty = make_lp(50, std::vector<int>(20, 0), 3);
  exercise(empty, o);
  // large enough for column panels (>= 4M entries, no row over 2048)
  LP big = make_lp(40000, std::vector<int>(10500, 400), 4);
  exercise(big, o);

  // invalid inputs
  {
    LP bad = make_lp(100, std::vector<int>(10, 5), 5);
    aapdhg_t h = nullptr;
    LP b1 = bad;
    b1.col[3] = 100;  // column out of range
    CHECK(create(b1, &o, &h) == AAPDHG_E_ARG && !h);
    LP b2 = bad;
    b2.col[1] = b2.col[0];  // repeated column in a row
    CHECK(create(b2, &o, &h) == AAPDHG_E_ARG);
    LP b3 = bad;
    b3.rowptr[4] = b3.rowptr[3] - 1;  // decreasing row pointers
    CHECK(create(b3, &o, &h) == AAPDHG_E_ARG);
    LP b4 = bad;
    b4.l[0] = 2.0;  // l > u (column 0 has u = 1)
    CHECK(create(b4, &o, &h) == AAPDHG_E_ARG);
    LP b5 = bad;
    b5.c[0] = NAN;
    CHECK(create(b5, &o, &h) == AAPDHG_E_ARG);
    LP b6 = bad;
    b6.rt[0] = 7;
    CHECK(create(b6, &o, &h) == AAPDHG_E_ARG);
    aapdhg_options ob = o;
    ob.memory = 0;
    CHECK(create(bad, &ob, &h) == AAPDHG_E_ARG);
    ob = o;
    ob.length_floor = 2;
    CHECK(create(bad, &ob, &h) == AAPDHG_E_ARG);
    ob.length_floor = 0;
    ob.gram_mode = 3;
    CHECK(create(bad, &ob, &h) == AAPDHG_E_ARG);
    CHECK(aapdhg_create(0, 5, 0, bad.rowptr.data(), nullptr, nullptr, bad.c.data(), bad.q.data(), bad.l.data(),
                        bad.u.data(), bad.rt.data(), &o, &h) == AAPDHG_E_ARG);
    CHECK(aapdhg_last_error(nullptr)[0] != '\0');
  }

  // device-memory entry points (stand-in device memory is host memory)
  {
    LP p = make_lp(500, std::vector<int>(80, 6), 6);
    auto dev = [](const void* src, size_t bytes) {
      void* d = nullptr;
      hipMalloc(&d, bytes);
      hipMemcpy(d, src, bytes, hipMemcpyHostToDevice);
      return d;
    };
    void* drp = dev(p.rowptr.data(), p.rowptr.size() * 8);
    void* dci = dev(p.col.data(), p.col.size() * 4);
    void* dva = dev(p.val.data(), p.val.size() * 8);
    void* dc = dev(p.c.data(), p.c.size() * 8);
    void* dq = dev(p.q.data(), p.q.size() * 8);
    void* dl = dev(p.l.data(), p.l.size() * 8);
    void* du = dev(p.u.data(), p.u.size() * 8);
    void* drt = dev(p.rt.data(), p.rt.size());
    aapdhg_t h = nullptr;
    CHECK(aapdhg_create_device(p.m, p.n, p.nnz(), (int64_t*)drp, (int32_t*)dci, (double*)dva, (double*)dc,
                               (double*)dq, (double*)dl, (double*)du, (uint8_t*)drt, &o, nullptr, &h) == AAPDHG_OK);
    // a host pointer is refused
    aapdhg_t h2 = nullptr;
    CHECK(aapdhg_create_device(p.m, p.n, p.nnz(), p.rowptr.data(), (int32_t*)dci, (double*)dva, (double*)dc,
                               (double*)dq, (double*)dl, (double*)du, (uint8_t*)drt, &o, nullptr, &h2) == AAPDHG_E_ARG);
    if (h) {
      CHECK(aapdhg_iterate(h, nullptr, 2) == AAPDHG_OK);
      void* dx = nullptr;
      hipMalloc(&dx, (size_t)p.n * 8);
      aapdhg_info info;
      CHECK(aapdhg_result_device(h, (double*)dx, nullptr, nullptr, &info, nullptr) == AAPDHG_OK);
      hipFree(dx);
      CHECK(aapdhg_destroy(h) == AAPDHG_OK);
    }
    for (void* d : {drp, dci, dva, dc, dq, dl, du, drt}) hipFree(d);
  }

  // batches of uneven LPs
  {
    std::vector<LP> lps;
    for (int i = 0; i < 6; ++i) lps.push_back(make_lp(300 + 200 * i, std::vector<int>(100 + 50 * i, 4 + i), 10 + i));
    lps[2] = rag;
    std::vector<aapdhg_t> hs;
    for (auto& p : lps) {
      aapdhg_t h = nullptr;
      CHECK(create(p, &o, &h) == AAPDHG_OK);
      hs.push_back(h);
    }
    aapdhg_batch_t b = nullptr;
    CHECK(aapdhg_batch_create((int)hs.size(), hs.data(), &b) == AAPDHG_OK);
    if (b) {
      CHECK(aapdhg_batch_iterate(b, nullptr, 3) == AAPDHG_OK);
      double ms4[4];
      CHECK(aapdhg_batch_iterate_timed(b, nullptr, 2, ms4) == AAPDHG_OK);
      CHECK(aapdhg_batch_solve(b, nullptr) == AAPDHG_OK);
      aapdhg_info info;
      std::vector<double> x(lps[3].n);
      CHECK(aapdhg_batch_result(b, 3, x.data(), nullptr, nullptr, &info) == AAPDHG_OK);
      CHECK(aapdhg_batch_result(b, 6, nullptr, nullptr, nullptr, &info) == AAPDHG_E_ARG);
      CHECK(aapdhg_batch_destroy(b) == AAPDHG_OK);
    }
    for (auto h : hs) aapdhg_destroy(h);
  }

  // server: admission, epochs, retirement, a request beyond the budget
  {
    aapdhg_server_t s = nullptr;
    CHECK(aapdhg_server_start((size_t)64 << 20, 4, &o, nullptr, nullptr, &s) == AAPDHG_OK);
    std::vector<uint64_t> tickets;
    std::vector<LP> reqs;
    for (int i = 0; i < 7; ++i) reqs.push_back(make_lp(200 + 30 * i, std::vector<int>(60 + 10 * i, 5), 20 + i));
    reqs.push_back(make_lp(2000000, std::vector<int>(3000, 1000), 30));  // too large for the budget
    for (auto& p : reqs) {
      uint64_t t = 0;
      CHECK(aapdhg_server_submit(s, p.m, p.n, p.nnz(), p.rowptr.data(), p.col.data(), p.val.data(), p.c.data(),
                                 p.q.data(), p.l.data(), p.u.data(), p.rt.data(), &t) == AAPDHG_OK);
      tickets.push_back(t);
    }
    int done = 0, failed = 0;
    for (int spin = 0; spin < 20000 && done + failed < (int)tickets.size(); ++spin) {
      for (size_t i = 0; i < tickets.size(); ++i) {
        if (!tickets[i]) continue;
        std::vector<double> x(reqs[i].n), y(reqs[i].m);
        aapdhg_info info;
        double ta = 0, td = 0;
        const aapdhg_status st = aapdhg_server_poll(s, tickets[i], &info, x.data(), y.data(), &ta, &td);
        if (st == AAPDHG_PENDING) continue;
        if (st == AAPDHG_OK) ++done; else ++failed;
        tickets[i] = 0;
      }
    }
    CHECK(done == 7 && failed == 1);
    // a submission whose host copy of the values cannot be allocated fails with
    // E_NOMEM, frees what it had copied, and the server goes on admitting
    {
      const LP& p = reqs[6];
      uint64_t t = 0;
      g_fail_at = (size_t)p.nnz() * sizeof(double);
      const aapdhg_status st = aapdhg_server_submit(s, p.m, p.n, p.nnz(), p.rowptr.data(), p.col.data(),
                                                    p.val.data(), p.c.data(), p.q.data(), p.l.data(),
                                                    p.u.data(), p.rt.data(), &t);
      g_fail_at = 0;
      CHECK(st == AAPDHG_E_NOMEM);
      CHECK(std::strstr(aapdhg_last_error(nullptr), "allocation") != nullptr);
      CHECK(aapdhg_server_submit(s, p.m, p.n, p.nnz(), p.rowptr.data(), p.col.data(), p.val.data(), p.c.data(),
                                 p.q.data(), p.l.data(), p.u.data(), p.rt.data(), &t) == AAPDHG_OK);
      aapdhg_status ps = AAPDHG_PENDING;
      std::vector<double> x(p.n), y(p.m);
      for (int spin = 0; spin < 20000 && ps == AAPDHG_PENDING; ++spin) {
        ps = aapdhg_server_poll(s, t, nullptr, x.data(), y.data(), nullptr, nullptr);
        if (ps == AAPDHG_PENDING) std::this_thread::sleep_for(std::chrono::milliseconds(1));
      }
      CHECK(ps == AAPDHG_OK);
    }
    int64_t stats[6];
    CHECK(aapdhg_server_stats(s, stats) == AAPDHG_OK);
    CHECK(aapdhg_server_poll(s, 999999, nullptr, nullptr, nullptr, nullptr, nullptr) == AAPDHG_E_ARG);
    CHECK(aapdhg_server_stop(s) == AAPDHG_OK);
  }

  if (g_fail) {
    std::fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  std::printf("hostcheck ok\n");
  return 0;
}
