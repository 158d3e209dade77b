// HIP kernels of the AA-PDHG / FAA-PDHG hot path for gfx950 (MI355X).
//
// One loop pass of Alg 2 / Alg 3 is three launches over a table of work items
// that may mix many LPs:
//   pass A  primal: w = K^T y by CSC gather, x_hat = P_X(x - tau (c - w)),
//           x_bar = 2 x_hat - x, g_x = x_hat - x, history column x-part and its
//           dot products, KKT sums at u^k (eq. pdhg; Alg 2 memory lines;
//           Remark re:constrcution-termi-con)
//   pass B  dual: v = K x_bar by CSR gather, y_hat = P_Y(y + sigma (q - v)),
//           g_y, history y-part and dots; the last block of each LP reduces all
//           partial sums in a fixed order and takes the decisions of the pass
//           in float64 (termination, memory update, safeguard, filters, the
//           m x m least-squares solve)
//   pass C  mix: u^{k+1} = P(u^k + beta D-hat g^k - sum_t gamma_t W_t) on
//           Anderson steps (W = dU + beta D-hat dG, so this is u^k - H^k g^k).
// A PDHG step needs no pass C: passes A/B already wrote u_hat^{k+1} into the
// buffer of the next iterate.
//
// Reductions are deterministic: every partial sum has a fixed place and is
// added in a fixed order, so a run is bitwise repeatable and an LP's iterates
// do not depend on which other LPs share the launch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "aapdhg_internal.h"
#include "kernels.h"

namespace aapdhg {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

// One DPP data-movement step on the two 32-bit halves of a double (VALU only).
// With every row enabled each lane reads a valid source lane and no old value
// is kept; with rows masked off (row broadcasts) those lanes return 0.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_mov(double v) {
  if constexpr (ROWMASK == 0xF) {
    const int lo = __builtin_amdgcn_mov_dpp((int)__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
  } else {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)__double2loint(v), CTRL, ROWMASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)__double2hiint(v), CTRL, ROWMASK, 0xF, false);
    return __hiloint2double(hi, lo);
  }
}

// Sum over the 64 lanes of a wave, returned to every lane.  A fixed sequence
// of DPP steps: pairs, quads, half rows and rows (all lanes of a 16-lane row
// then hold the row sum), then row 0 into row 1, row 2 into row 3, rows 0-1
// into rows 2-3; lane 63 ends with the total.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_mov<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v += dpp_mov<0x141, 0xF>(v);  // row_half_mirror
  v += dpp_mov<0x140, 0xF>(v);  // row_mirror
  v += dpp_mov<0x142, 0xA>(v);  // row_bcast:15
  v += dpp_mov<0x143, 0xC>(v);  // row_bcast:31
  const int lo = __builtin_amdgcn_readlane((int)__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane((int)__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// Block-wide sum of one value per thread; the result is valid in thread 0.
// Fixed butterfly inside each wave, then the four wave sums in wave order.
__device__ __forceinline__ double block_sum(double v, double* s_tmp) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) s_tmp[wv] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = ((s_tmp[0] + s_tmp[1]) + s_tmp[2]) + s_tmp[3];
  return r;
}

// Cross-block data (partial sums, counters) inside one kernel: stores and
// loads at agent scope go straight to the device-coherent level for just those
// words, so no fence has to write back or invalidate a whole L2.  A writer
// waits for its stores to complete (vmcnt 0) before it bumps the counter; the
// block that sees the final count reads the words back at agent scope.
__device__ __forceinline__ void st_agent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_agent(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Coherent load of cross-block data that the compiler may keep in flight with
// others (a buffer load with the sc1 cache policy).
__device__ __forceinline__ double ld_coh(const double* base, int idx) {
  const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(base), 0, 0x7fffffff, 0x00020000);
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, idx * 8, 0, 16));
}
// A value the same in every lane (a chunk bound from a table), made known to
// the compiler as such, so that a test on it branches once for the wave.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Sum of base[first + i * stride] for i = 0 .. count - 1, added in that
// order, with U coherent loads issued together: a loop that adds each value
// as it is loaded waits for every load on its own.  The loads past count read
// the last value again and are not added, so the sum is the plain in-order
// one bit for bit.
template <int U>
__device__ __forceinline__ double ordered_sum_coh(const double* base, int first, int stride, int count) {
  double s = 0.0;
  for (int i0 = 0; i0 < count; i0 += U) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = ld_coh(base, first + (i0 + u < count ? i0 + u : count - 1) * stride);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i0 + u < count) s += v[u];
  }
  return s;
}
__device__ __forceinline__ void wait_stores() {
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's stores are complete
}
// Count one arrival; true for the block that arrives last (thread 0 only).
__device__ __forceinline__ bool arrive(unsigned int* cnt, unsigned int total) {
  wait_stores();
  const unsigned int prev = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return prev == total - 1u;
}
__device__ __forceinline__ void reset_counter(unsigned int* cnt) {
  __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ T clampT(T v, T lo, T hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

__device__ __forceinline__ double proj_lambda(double lam, bool lf, bool uf) {
  // eq. lambda-case: {0} both infinite, R- only u finite, R+ only l finite, R both finite
  if (!lf && !uf) return 0.0;
  if (!lf) return lam < 0.0 ? lam : 0.0;
  if (!uf) return lam > 0.0 ? lam : 0.0;
  return lam;
}

// ---------------------------------------------------------------------------
// decisions of a loop pass (one thread of the last block of an LP)
// ---------------------------------------------------------------------------

// The decisions of a loop pass run on the 64 lanes of one wave, on LDS data.
// Values read from LDS by every lane are uniform; lane 0 writes scalars.  LDS
// instructions of one wave complete in order, so a value written by one lane
// is seen by every lane's later read.

// Orders one wave's LDS writes before its later reads by other lanes: LDS
// instructions of a wave complete in order; this keeps the compiler from
// moving or caching accesses across the point.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
}

// LDS workspace of the decisions.
struct SolveWork {
  double A[MAXM * MAXM];
  double gam[MAXM];
  double fn[MAXM], gdiag[MAXM], b[MAXM], e2[MAXM];
  int live[MAXM], ord[MAXM], keep[MAXM];
  int nl, nk, kk, pad;
  bool dep[MAXM];
};

// Cholesky A = L L^T of the n x n matrix in A (row-major, stride MAXM, lower
// part), right-looking: step j scales column j and updates the trailing
// triangle, so every entry receives its updates in the order of a
// column-by-column factorisation.  With gdiag != nullptr a pivot that is not
// above 1e-28 gdiag[j] marks column j dependent (zero column, dep[j] = true)
// and the factorisation continues; without it such a pivot fails.  With
// seq_cs > 0 (and gdiag, fn) a column j >= 1 whose r_jj / fn[j] is below
// seq_cs is marked dependent as well, so later columns are measured against
// the columns kept so far only.
__device__ bool wave_chol(double* A, int n, int lane, const double* gdiag, bool* dep, double seq_cs = 0.0,
                          const double* fn = nullptr) {
  for (int j = 0; j < n; ++j) {
    const double piv = A[j * MAXM + j];
    bool isdep = false;
    if (gdiag) {
      isdep = !(piv > 1e-28 * gdiag[j]) || !isfinite(piv);
      if (!isdep && seq_cs > 0.0 && j > 0) isdep = !(sqrt(piv) / fn[j] >= seq_cs);
    } else if (!(piv > 0.0) || !isfinite(piv)) {
      return false;
    }
    const double r = isdep ? 0.0 : sqrt(piv);
    wave_sync();
    if (lane == 0) {
      A[j * MAXM + j] = r;
      if (gdiag) dep[j] = isdep;
    }
    for (int i = j + 1 + lane; i < n; i += 64) A[i * MAXM + j] = isdep ? 0.0 : A[i * MAXM + j] / r;
    wave_sync();
    const int mm = n - j - 1;
    const int np = mm * (mm + 1) / 2;
    for (int p = lane; p < np; p += 64) {
      int a = (int)((sqrtf(8.0f * (float)p + 1.0f) - 1.0f) * 0.5f);
      while ((a + 1) * (a + 2) / 2 <= p) ++a;
      while (a * (a + 1) / 2 > p) --a;
      const int b = p - a * (a + 1) / 2;
      const int i = j + 1 + a, k = j + 1 + b;
      A[i * MAXM + k] -= A[i * MAXM + j] * A[k * MAXM + j];
    }
    wave_sync();
  }
  return true;
}

// Solve L L^T x = b with the factor from wave_chol (b overwritten by x).
__device__ void wave_chol_solve(const double* L, double* b, int n, int lane) {
  for (int i = 0; i < n; ++i) {
    const double bi = b[i] / L[i * MAXM + i];
    wave_sync();
    if (lane == 0) b[i] = bi;
    for (int k = i + 1 + lane; k < n; k += 64) b[k] -= L[k * MAXM + i] * bi;
    wave_sync();
  }
  for (int i = n - 1; i >= 0; --i) {
    const double bi = b[i] / L[i * MAXM + i];
    wave_sync();
    if (lane == 0) b[i] = bi;
    for (int k = lane; k < i; k += 64) b[k] -= L[i * MAXM + k] * bi;
    wave_sync();
  }
}

// gamma for the history columns `slots` (oldest first): (G + shift I) gamma = rhs.
__device__ bool solve_gamma(const Scalars* sc, const int* slots, int n, double shift, SolveWork* w, int lane) {
  for (int q = lane; q < n * n; q += 64) {
    const int a = q / n, b = q - a * n;
    if (b <= a) w->A[a * MAXM + b] = sc->G[slots[a] * MAXM + slots[b]] + (a == b ? shift : 0.0);
  }
  if (lane < n) w->gam[lane] = sc->rhs[slots[lane]];
  wave_sync();
  if (!wave_chol(w->A, n, lane, nullptr, nullptr)) return false;
  wave_chol_solve(w->A, w->gam, n, lane);
  bool ok = true;
  for (int a = 0; a < n; ++a) ok &= isfinite(w->gam[a]);
  return ok;
}

// FAA filters (Alg 3 lines Reverse..Reverse; Alg 4 AngleFilter, Alg 5
// LengthFilter with the bounds of Lemma le:RK-1bound1).  w->live holds nl
// slots oldest first; on return it holds the survivors, oldest first, and the
// count is returned.  The R factor of the reversed history comes from the
// Gram (R^T R = F^T F): r_ii^2 is the squared distance of column i from the
// span of the newer columns.
__device__ int faa_filter(const LPDesc& d, const Scalars* sc, int nl, SolveWork* w, int lane) {
  int* ord = w->ord;  // newest first (Reverse)
  if (lane < nl) {
    ord[lane] = w->live[nl - 1 - lane];
  }
  for (int q = lane; q < nl * nl; q += 64) {
    const int a = q / nl, b = q - a * nl;
    const int oa = w->live[nl - 1 - a], ob = w->live[nl - 1 - b];
    if (b <= a) w->A[a * MAXM + b] = sc->G[oa * MAXM + ob];
    if (a == b) {
      w->gdiag[a] = sc->G[oa * MAXM + oa];
      w->fn[a] = sqrt(w->gdiag[a] > 0.0 ? w->gdiag[a] : 0.0);
    }
  }
  wave_sync();
  wave_chol(w->A, nl, lane, w->gdiag, w->dep, d.angle_mode ? d.cs : 0.0, w->fn);
  // AngleFilter: the newest column is always kept; column i >= 2 is removed
  // when |r_ii| / ||f_i|| < c_s (a zero or dependent column is removed).
  // With angle_mode 1 the factorisation above already skipped the removed
  // columns, so r_ii is the distance from the span of the kept ones.
  bool keepme = false;
  if (lane < nl) {
    const double rii = w->dep[lane] ? 0.0 : w->A[lane * MAXM + lane];
    keepme = lane == 0 || (w->fn[lane] > 0.0 && rii / w->fn[lane] >= d.cs);
  }
  const unsigned long long bal = __ballot(keepme);
  const int nk = __popcll(bal);
  if (keepme) w->keep[__popcll(bal & ((1ull << lane) - 1ull))] = lane;
  wave_sync();
  // LengthFilter on the kept columns (newest first, 1-based j in the lemma)
  const double cs = d.cs, ct = sqrt(1.0 - cs * cs);
  if (lane < nk) {
    const int jj = lane;
    w->e2[jj] = sc->du2[ord[w->keep[jj]]];
    const double fj2 = w->fn[w->keep[jj]] * w->fn[w->keep[jj]];
    if (jj == 0) {
      w->b[jj] = 1.0 / fj2;
    } else {
      const int j = jj + 1;
      const double f12 = w->fn[w->keep[0]] * w->fn[w->keep[0]];
      double tot = ct * ct * pow(ct + cs, 2.0 * (j - 2)) / (f12 * pow(cs, 2.0 * (j - 2)));
      for (int i = 2; i <= j - 1; ++i) {
        const double fi2 = w->fn[w->keep[i - 1]] * w->fn[w->keep[i - 1]];
        tot += ct * ct * pow(ct + cs, 2.0 * (j - i - 1)) / (fi2 * pow(cs, 2.0 * (j - i)));
      }
      tot += 1.0 / fj2;
      w->b[jj] = tot / (cs * cs);
    }
  }
  wave_sync();
  if (lane == 0) {
    int kk = nk;
    const double kb2 = d.kappa_bar * d.kappa_bar;
    while (kk >= 1) {
      double se = 0.0, sb = 0.0;
      for (int j = 0; j < kk; ++j) {
        se += w->e2[j];
        sb += w->b[j];
      }
      if (se * sb <= kb2) break;
      --kk;
    }
    // reading of Alg 5 when no k passes: none kept (floor 0) or the newest (floor 1)
    if (kk < d.length_floor && nk > 0) kk = d.length_floor;
    w->kk = kk;
  }
  wave_sync();
  const int kk = w->kk;
  // survivors: first kk kept columns (newest first) -> oldest first
  if (lane < kk) w->live[lane] = ord[w->keep[kk - 1 - lane]];
  wave_sync();
  return kk;
}

// Decisions of loop pass k, on the summed records f: KKT test, memory update,
// safeguard, Anderson coefficients (Alg 2) or filters (Alg 3).  Every lane of
// one wave calls it; sc points at an LDS copy of the LP's scalars.
// D-hat after a primal-weight update (remark on the primal-weight form):
// (1 - alpha) diag(1/omega, omega) + alpha diag(D-hat_1 / omega, D-hat_2 omega),
// kept as coefficients of the construction's D-hat: dha[p] D-hat_0 + dhb[p]
// on the x part (p = 0) and the y part (p = 1).
__device__ __forceinline__ void dhat_coeffs(double alpha, double omega, double* dha, double* dhb) {
  dha[0] = alpha / omega;
  dhb[0] = (1.0 - alpha) / omega;
  dha[1] = alpha * omega;
  dhb[1] = (1.0 - alpha) * omega;
}

// Alg 7 from the squared distances of x^k and y^k to the iterate of the last
// check: true when both exceed epsilon_zero; then omega is smoothed in log
// space and tau = gstep / omega, sigma = gstep * omega.
__device__ __forceinline__ bool pw_decide(const LPDesc& d, double dx2, double dy2, double gstep, double& omega,
                                          double& tau, double& sigma) {
  const double dx = sqrt(dx2), dy = sqrt(dy2);
  if (!(dx > d.pw_eps0 && dy > d.pw_eps0)) return false;
  omega = exp(d.pw_theta * log(dy / dx) + (1.0 - d.pw_theta) * log(omega));
  tau = gstep / omega;
  sigma = gstep * omega;
  return true;
}

// The end of a loop pass, once its branch is known: the mix coefficients, the
// live slots, the slot of the next difference pair and the counters.
__device__ void finish_pass(const LPDesc& d, Scalars* sc, SolveWork* w, bool aa, int nmix, int nl, long long k,
                            long long i_aa, int lane) {
  const bool L0 = lane == 0;
  wave_sync();
  if (lane < nmix) {
    sc->mixslot[lane] = w->live[lane];
    sc->gamma[lane] = w->gam[lane];
  }
  if (lane < nl) sc->live[lane] = w->live[lane];
  // slot for the next difference pair: the lowest free one, else the oldest
  unsigned int used = lane < nl ? 1u << w->live[lane] : 0u;
#pragma unroll
  for (int off = 1; off < MAXM; off <<= 1) used |= __shfl_xor(used, off, 64);
  used = __shfl(used, 0, 64);  // lanes 0..MAXM-1 hold every live slot
  const unsigned int freem = ~used & ((1u << d.M) - 1u);
  const int ns = (nl < d.M && freem != 0u) ? __ffs(freem) - 1 : w->live[0];
  wave_sync();
  if (L0) {
    sc->nmix = nmix;
    if (aa) {
      sc->branch = BR_AA;
      sc->i_aa = i_aa + 1;
    } else {
      sc->branch = BR_PDHG;
      sc->j_pdhg += 1;
    }
    sc->nlive = nl;
    sc->newslot = ns;
    sc->k = k + 1;
  }
}

// The decisions of a loop pass (wave 0 of one workgroup), from the summed
// records f.  With lazy set (three-launch path) the records carry no dots of
// the new difference column with the stored ones: G and rhs are left stale,
// and a pass whose safeguard test passes with a non-empty memory ends with
// branch BR_GRAM, for the Gram launch to finish (gram_decide).
template <int MT>
__device__ void final_step(const LPDesc& d, Scalars* sc, const double* f, bool eval, bool kkt, bool init,
                           SolveWork* w, int lane, bool lazy) {
  using DT = Dot<MT>;
  const bool L0 = lane == 0;
  double kktv = 0.0;
  if (kkt) {
    // Remark re:constrcution-termi-con: relative gap, primal and dual infeasibility
    const double pobj = f[DT::KA0];
    const double dobj = f[DT::KB0] + f[DT::KA1];
    const double rg = fabs(dobj - pobj) / (1.0 + fabs(dobj) + fabs(pobj));
    const double rp = sqrt(f[DT::KB1]) / (1.0 + sc->qnorm);
    const double rd = sqrt(f[DT::KA2]) / (1.0 + sc->cnorm);
    kktv = fmax(rg, fmax(rp, rd));
    if (L0) {
      sc->pobj = pobj;
      sc->dobj = dobj;
      sc->r_g = rg;
      sc->r_p = rp;
      sc->r_d = rd;
      sc->kkt = kktv;
      sc->kkt_k = sc->k;
    }
  }
  if (eval) return;
  const double gnorm = sqrt(f[DT::GG]);
  const double gprev = sc->gnorm;  // ||g^{k-1}||
  const long long k = sc->k;
  const double n0 = sc->n0;
  const long long i_aa = sc->i_aa;
  wave_sync();
  if (L0) sc->gnorm = gnorm;
  if (init) {  // Alg 2 set-up: g^0 = u^1 - u^0
    if (L0) {
      sc->n0 = gnorm;
      if (!isfinite(gnorm)) {
        sc->status = ST_NUMERICAL;
        sc->branch = BR_NONE;
      } else if (gnorm == 0.0) {
        sc->status = ST_CONVERGED;  // u^0 is a fixed point
        sc->branch = BR_NONE;
      } else {
        sc->branch = BR_PDHG;
        sc->k = 1;
      }
    }
    return;
  }
  if (k > d.max_iter || (kkt && kktv <= d.tol) || !isfinite(gnorm)) {
    if (L0) {
      sc->status = k > d.max_iter ? ST_ITER_LIMIT : (kkt && kktv <= d.tol) ? ST_CONVERGED : ST_NUMERICAL;
      sc->branch = BR_NONE;
    }
    return;
  }
  // memory update (both branches): the pair written this pass goes to newslot
  const int s = sc->newslot;
  const int nl_old = sc->nlive;
  const bool pw_reset = sc->pw_flag != 0;
  wave_sync();
  if (L0) sc->pw_blend = 0;
  if (pw_reset) {
    // the weight changed before this pass (Alg 7): the memory was reset and
    // the pair of this pass, which joins residuals of two maps, is not kept;
    // D-hat is re-blended with alpha from the residual decrease
    if (L0) {
      w->nl = 0;
      sc->pw_flag = 0;
      if (d.pw_dhat) {
        const double rho = (gprev - gnorm) / fmax(gprev, d.pw_eps0);
        const bool dec = rho > d.pw_rho;
        dhat_coeffs(dec ? 0.1 : 0.9, sc->omega, sc->dha, sc->dhb);
        sc->pw_blend = dec ? 2 : 1;
      }
    }
  }
  if (!pw_reset && !lazy && lane < nl_old) {
    const int slot = sc->live[lane];
    if (slot != s) {  // the oldest column is replaced
      const double gv = f[DT::G + lane];
      sc->G[s * MAXM + slot] = gv;
      sc->G[slot * MAXM + s] = gv;
      sc->rhs[slot] += gv;  // <dG[slot], g^k> = <dG[slot], g^{k-1}> + <dG[slot], dg_new>
    }
  }
  if (!pw_reset) {
    // live slots without the replaced one, oldest first, then the new pair
    const int slot = lane < nl_old ? sc->live[lane] : -1;
    const bool keep = lane < nl_old && slot != s;
    const unsigned long long bal = __ballot(keep);
    if (keep) w->live[__popcll(bal & ((1ull << lane) - 1ull))] = slot;
    if (L0) {
      const int nk = __popcll(bal);
      w->live[nk] = s;
      w->nl = nk + 1;
      if (!lazy) {
        sc->G[s * MAXM + s] = f[DT::DGDG];
        sc->rhs[s] = f[DT::DGG];
      }
      sc->du2[s] = f[DT::DU2];
    }
  }
  if (lazy && L0) sc->gram_ok = 0;
  wave_sync();
  int nl = w->nl;

  bool aa = false;
  int nmix = 0;
  if (d.variant == V_AA || d.variant == V_FAA) {
    // safeguard (Alg 2): ||g^k|| <= D ||g^0|| (i^k / c + 1)^{-(1+eps)}, c = 1 in
    // Alg 2 (Iter_AA / c otherwise); ties accelerate.  The bound changes only
    // with i^k: computed once per Anderson step
    double thr = sc->thr;
    if (sc->thr_i != i_aa + 1) {
      thr = d.D * n0 * pow((double)i_aa / d.sg_div + 1.0, -(1.0 + d.eps_sg));
      wave_sync();
      if (L0) {
        sc->thr = thr;
        sc->thr_i = i_aa + 1;
      }
    }
    if (gnorm <= thr && lazy && nl > 0) {
      // the Gram launch forms G and rhs of the live slots and finishes the pass
      wave_sync();
      if (lane < nl) sc->live[lane] = w->live[lane];
      if (L0) {
        sc->nlive = nl;
        sc->branch = BR_GRAM;
      }
      return;
    }
    if (gnorm <= thr) {
      if (d.variant == V_AA) {
        if (nl == 0) {
          aa = true;  // empty memory (after a weight update): u_AA = u^k + beta D-hat g^k
        } else if (solve_gamma(sc, w->live, nl, d.eta, w, lane)) {
          aa = true;
          nmix = nl;
        }
      } else {
        const int nl_in = nl;
        nl = faa_filter(d, sc, nl, w, lane);  // the survivors become the memory
        if (nl == 0) {
          aa = true;  // no history left: u_AA = u^k + beta D-hat g^k
          if (L0 && nl_in > 0) sc->faa_empty += 1;
        } else if (solve_gamma(sc, w->live, nl, 0.0, w, lane)) {
          aa = true;
          nmix = nl;
        }
      }
    }
  }
  finish_pass(d, sc, w, aa, nmix, nl, k, i_aa, lane);
}

// The pending decisions of a pass left with branch BR_GRAM (wave 0 of the
// last workgroup of the Gram launch), once G and rhs hold the Gram matrix of
// the live slots and their dots with g^k: the regularised solve of Alg 2, or
// the filters and the least-squares solve of Alg 3, then the end of the pass.
__device__ void gram_decide(const LPDesc& d, Scalars* sc, SolveWork* w, int lane) {
  const int nl_in = sc->nlive;
  if (lane < nl_in) w->live[lane] = sc->live[lane];
  wave_sync();
  int nl = nl_in;
  bool aa = false;
  int nmix = 0;
  if (d.variant == V_AA) {
    if (solve_gamma(sc, w->live, nl, d.eta, w, lane)) {
      aa = true;
      nmix = nl;
    }
  } else {
    nl = faa_filter(d, sc, nl, w, lane);  // the survivors become the memory
    if (nl == 0) {
      aa = true;  // no history left: u_AA = u^k + beta D-hat g^k
      if (lane == 0) sc->faa_empty += 1;
    } else if (solve_gamma(sc, w->live, nl, 0.0, w, lane)) {
      aa = true;
      nmix = nl;
    }
  }
  finish_pass(d, sc, w, aa, nmix, nl, sc->k, sc->i_aa, lane);
  // G and rhs of the kept slots are current (rhs against g^k, the residual
  // before the new iteration index)
  if (lane == 0) sc->gram_ok = 1;
}

// ---------------------------------------------------------------------------
// pass A (PASS = 0, columns of K via CSC) and pass B (PASS = 1, rows via CSR)
// ---------------------------------------------------------------------------

// Data that other workgroups of the same launch write, read and written at
// agent scope (buffer instructions with the sc1 policy) without a fence.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t coh_rsrc(const void* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, 0x7fffffff, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T ldc(const T* base, int i) {
  if constexpr (sizeof(T) == 8) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(coh_rsrc(base), i * 8, 0, 16));
  } else {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(coh_rsrc(base), i * 4, 0, 16));
  }
}
template <typename T>
__device__ __forceinline__ void stc(T* base, int i, T v) {
  if constexpr (sizeof(T) == 8) {
    using B64 = decltype(__builtin_amdgcn_raw_buffer_load_b64(coh_rsrc(base), 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(B64, v), coh_rsrc(base), i * 8, 0, 16);
  } else {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), coh_rsrc(base), i * 4, 0, 16);
  }
}

// Inputs of one row's (or column's) epilogue, loaded before anything is stored
// so that the loads of a thread's rows and of the SpMV are in flight together.
template <typename T, int MT>
struct RowIn {
  T u, up, gp, cq, lo, hi, dh;
  unsigned char ge;
  T hv[MT];
};

// What every workgroup of an LP needs to know about the pass it works on.
struct PassView {
  long long k;
  int nl, s_new;
  int ndot;  // stored columns the new difference column is dotted with (nl, or 0 on the three-launch path)
  const int* live;  // live history slots, oldest first (LDS)
  bool eval, init, kkt, hist_on, skip0;
  bool restart_now;  // restarted PDHG: this pass ends an epoch
  // tau, sigma (primal weight) and the D-hat coefficients a_x, a_y, b_x, b_y
  // of this pass, six consecutive doubles (LDS in the loop kernel)
  const double* steps;
};

__device__ __forceinline__ PassView make_view(const LPDesc& d, long long k, int nl, int s_new, const int* live,
                                              bool eval, const double* steps) {
  PassView v;
  v.steps = steps;
  v.k = k;
  v.nl = nl;
  v.ndot = nl;
  v.s_new = s_new;
  v.live = live;
  v.eval = eval;
  v.init = !eval && k == 0;
  v.kkt = eval || (!v.init && d.kkt_every > 0 && (k % d.kkt_every) == 0);
  v.hist_on = !eval && !v.init;
  v.restart_now = !eval && d.restart > 0 && (k + 1) % d.restart == 0;
  // a full memory replaces its oldest column: that column takes no dots
  v.skip0 = nl > 0 && live[0] == s_new;
  return v;
}

// One pass over one LP.  COH is set inside the persistent loop kernel, where
// other workgroups of the launch read what this one writes: the iterates and
// x_bar are written and read at agent scope.  Everything else of a row is
// read and written only by the workgroup that owns the row, except for split
// rows, which are finished by whichever part arrives last: their epilogue
// (row_coh) reads and writes everything of the row at agent scope.  EXT: the
// extended loop features may be on: step sizes and D-hat that change during
// the solve (primal-weight update) and restarts (restarted PDHG); without it
// tau, sigma and D-hat are the LP's fixed values and there are no restarts.
template <typename T, int MT, int PASS, bool COH, bool EXT>
struct PassCtx {
  using DT = Dot<MT>;
  static constexpr int NPAN = panel_count(sizeof(T) == 8);  // column panels of the dual product
  const LPDesc* dp;
  PassView v;
  int n, N;
  const T* ucur;  // u^k
  T* unext;       // u^{k-1} on entry, u_hat^{k+1} on exit
  T* gcur;
  const T* gprev;
  T* dG;
  T* W;
  T* xbar;
  const T* dhat;
  const int* ptr;
  const int* idx;
  const T* val;
  const int* rmap;
  const T* gv1;  // pass A gathers y^k; pass B gathers x_bar (and x^k for KKT)
  const T* gv2;
  const T* cq;
  const T* lov;
  const T* hiv;
  const unsigned char* rtype;
  double beta, tau, sigma;
  double dh_a, dh_b;  // D-hat of this pass's part: dh_a D-hat_0 + dh_b
  bool two;

  __device__ __forceinline__ PassCtx(const LPDesc* d, const PassView& pv) : dp(d), v(pv) {
    n = d->n;
    N = d->N;
    const int par = (int)(pv.k & 1);
    ucur = (const T*)d->u[par];
    unext = (T*)d->u[par ^ 1];
    gcur = (T*)d->g[par];
    gprev = (const T*)d->g[par ^ 1];
    dG = (T*)d->dG;
    W = (T*)d->W;
    xbar = (T*)d->xbar;
    dhat = (const T*)d->dhat;
    ptr = PASS == 0 ? d->colptr : d->rowptr;
    idx = PASS == 0 ? d->rowidx : d->colidx;
    val = (const T*)(PASS == 0 ? d->valT : d->val);
    rmap = PASS == 0 ? d->rmapA : d->rmapB;
    gv1 = PASS == 0 ? ucur + n : (pv.eval ? ucur : (const T*)xbar);
    gv2 = ucur;
    cq = (const T*)(PASS == 0 ? d->c : d->q);
    lov = (const T*)d->lo;
    hiv = (const T*)d->hi;
    rtype = d->rowtype;
    beta = d->beta;
    if constexpr (EXT) {
      tau = pv.steps[0];
      sigma = pv.steps[1];
      dh_a = pv.steps[2 + PASS];
      dh_b = pv.steps[4 + PASS];
    } else {
      tau = d->tau;
      sigma = d->sigma;
      dh_a = 1.0;
      dh_b = 0.0;
    }
    two = PASS == 1 && pv.kkt && !pv.eval;
  }

  __device__ __forceinline__ T gather(const T* gv, int i) const {
    if constexpr (COH) return ldc(gv, i);
    return gv[i];
  }
  __device__ __forceinline__ T ld(const T* p, int i, bool c) const {
    if constexpr (COH) {
      if (c) return ldc(p, i);
    }
    return p[i];
  }
  __device__ __forceinline__ void st(T* p, int i, T x, bool c) const {
    if constexpr (COH) {
      if (c) {
        stc(p, i, x);
        return;
      }
    }
    p[i] = x;
  }

  // ---- epilogue, part 1: loads ----
  __device__ __forceinline__ void load_row(int r, RowIn<T, MT>& in, bool row_coh) const {
    const int e = PASS == 0 ? r : n + r;
    // iterates are always written at agent scope in the loop kernel (other
    // workgroups gather them), so they are read back the same way
    in.u = ld(ucur, e, true);
    in.cq = cq[r];
    if (PASS == 0) {
      in.lo = lov[r];
      in.hi = hiv[r];
    } else {
      in.ge = rtype[r];
    }
    if (v.hist_on) {
      in.up = ld(unext, e, true);
      in.gp = ld(gprev, e, row_coh);
      in.dh = dhat[e];
#pragma unroll
      for (int t = 0; t < MT; ++t)
        if (t < v.ndot && !(t == 0 && v.skip0)) in.hv[t] = ld(dG + (size_t)v.live[t] * N, e, row_coh);
    }
  }

  // ---- epilogue, part 2: eq. pdhg update, residual, history, dots, KKT sums ----
  __device__ __forceinline__ void finish_row(int r, const RowIn<T, MT>& in, double s1, double s2, double* accv,
                                             bool row_coh) const {
    const int e = PASS == 0 ? r : n + r;
    T g = (T)0;
    if (!v.eval) {
      T nx;
      if (PASS == 0) {
        // x_hat = P_X(x - tau (c - K^T y)), x_bar = 2 x_hat - x
        nx = clampT((T)((double)in.u - tau * ((double)in.cq - s1)), in.lo, in.hi);
        st(xbar, r, (T)(2.0 * (double)nx - (double)in.u), true);
      } else {
        // y_hat = P_Y(y + sigma (q - K x_bar))
        nx = (T)((double)in.u + sigma * ((double)in.cq - s1));
        if (in.ge && nx < (T)0) nx = (T)0;
      }
      g = (T)((double)nx - (double)in.u);
      st(gcur, e, g, row_coh);
      T nu = nx;  // the next iterate
      if constexpr (EXT) {
        if (dp->restart > 0) {
          // restarted PDHG: add the PDHG point to the epoch's sum; the last
          // pass of an epoch moves to the epoch's average and clears the sum
          double* rs = dp->rsum;
          const bool rc = COH && row_coh;
          const double sum = (rc ? ldc((const double*)rs, e) : rs[e]) + (double)nx;
          double keep = sum;
          if (v.restart_now) {
            nu = (T)(sum / (double)dp->restart);
            keep = 0.0;
          }
          if (rc) stc(rs, e, keep); else rs[e] = keep;
        }
      }
      st(unext, e, nu, true);
      accv[DT::GG] += (double)g * (double)g;
    }
    if (v.hist_on) {
      // memory pair of this pass: dg = g^k - g^{k-1}, du = u^k - u^{k-1}
      const T dgT = (T)((double)g - (double)in.gp);
      const T duT = (T)((double)in.u - (double)in.up);
      const double dg = (double)dgT, du = (double)duT, gd = (double)g;
      st(dG + (size_t)v.s_new * N, e, dgT, row_coh);
      const double dh = EXT ? dh_a * (double)in.dh + dh_b : (double)in.dh;
      st(W + (size_t)v.s_new * N, e, (T)(du + beta * dh * dg), row_coh);
      accv[DT::DGDG] += dg * dg;
      accv[DT::DGG] += dg * gd;
      accv[DT::DU2] += du * du;
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        if (t < v.ndot && !(t == 0 && v.skip0)) {
          const double hv = (double)in.hv[t];
          accv[DT::G + t] += dg * hv;
        }
      }
    }
    if (v.kkt) {
      if (PASS == 0) {
        const bool lf = isfinite((double)in.lo), uf = isfinite((double)in.hi);
        const double cj = (double)in.cq;
        const double lamv = proj_lambda(cj - s1, lf, uf);
        accv[DT::KA0] += cj * (double)in.u;
        accv[DT::KA1] += (lf ? (double)in.lo * fmax(lamv, 0.0) : 0.0) - (uf ? (double)in.hi * fmax(-lamv, 0.0) : 0.0);
        const double rd = cj - s1 - lamv;
        accv[DT::KA2] += rd * rd;
        if (v.eval) ((T*)dp->lam)[r] = (T)lamv;
      } else {
        const double kx = v.eval ? s1 : s2;  // (K x^k)_i
        const double qi = (double)in.cq;
        accv[DT::KB0] += qi * (double)in.u;
        double res = qi - kx;
        if (in.ge && res < 0.0) res = 0.0;
        accv[DT::KB1] += res * res;
      }
    }
  }

  // ---- multi-row chunk: stage products in LDS, reduce rows, epilogue ----
  // CACHED: the chunk's column indices (cidx), this thread's original row
  // (crow) and its row's range in the chunk (ca0, ca1) come from LDS, where
  // the persistent kernel keeps the one chunk a workgroup owns.
  // Pass B of an LP with column panels (three-launch path): the row sums come
  // from k_panel, so each chunk of the run is BLOCK rows, one per thread, with
  // no matrix work.  RB chunks are loaded together (their loads in flight at
  // once) and then finished in chunk order, so each thread adds its rows'
  // dots in the same order as one chunk at a time.
  template <int RB>
  __device__ __forceinline__ void panel_rows(const Chunk* chunks, int c0, int c1, double* acc) const {
    const int tid = threadIdx.x;
    const int m = dp->m;
    for (int c = c0; c < c1; c += RB) {
      RowIn<T, MT> rin[RB];
      double s1[RB], s2[RB];
      int row[RB];
      bool has[RB];
#pragma unroll
      for (int j = 0; j < RB; ++j) {
        s1[j] = 0.0;
        s2[j] = 0.0;
        row[j] = 0;
        has[j] = false;
        if (c + j < c1) {
          const Chunk ch = chunks[c + j];
          const int r = ch.r0 + tid;
          has[j] = r < ch.r1;
          if (has[j]) {
            row[j] = rmap[r];
            load_row(row[j], rin[j], false);
#pragma unroll
            for (int p = 0; p < NPAN; ++p) s1[j] += dp->part[(size_t)p * m + r];
            if (two) {
#pragma unroll
              for (int p = 0; p < NPAN; ++p) s2[j] += dp->part[(size_t)(NPAN + p) * m + r];
            }
          }
        }
      }
#pragma unroll
      for (int j = 0; j < RB; ++j)
        if (has[j]) finish_row(row[j], rin[j], s1[j], s2[j], acc, false);
    }
  }

  template <bool CACHED>
  __device__ __forceinline__ void multi_chunk(const Chunk& ch, double* acc, double* s_prod, double* s_tmp,
                                              const int* cidx = nullptr, const int* crow = nullptr,
                                              const int* ca0 = nullptr, const int* ca1 = nullptr) const {
    constexpr int UNR = CHUNK_NNZ / BLOCK;  // staged entries per thread
    const int tid = threadIdx.x;
    const int r0 = ch.r0, r1 = ch.r1, kb = ch.k0, ke = ch.k1, tpr = ch.tpr;
    const bool blockmode = tpr == BLOCK;
    const int grp = blockmode ? 0 : tid / tpr;
    const int lane_r = blockmode ? tid : tid % tpr;
    const int r = r0 + grp;  // this thread group's position (at most one)
    const bool has_row = r < r1 && (!blockmode || tid == 0);
    int row = 0;  // its original row
    if (has_row) row = CACHED ? crow[tid] : rmap[r];
    if (!COH && PASS == 1 && dp->panels) {
      // the row sums were formed by k_panel: add the panels in order
      if (has_row && lane_r == 0) {
        RowIn<T, MT> rin;
        load_row(row, rin, false);
        const int m = dp->m;
        double sum1 = 0.0, sum2 = 0.0;
#pragma unroll
        for (int p = 0; p < NPAN; ++p) sum1 += dp->part[(size_t)p * m + r];
        if (two) {
#pragma unroll
          for (int p = 0; p < NPAN; ++p) sum2 += dp->part[(size_t)(NPAN + p) * m + r];
        }
        finish_row(row, rin, sum1, sum2, acc, false);
      }
      return;
    }
    // Every load of the chunk is made, positions past its end reading its
    // last entry (their products are not staged): a load under a bounds test
    // of its own is waited for before the next one is issued, which the
    // persistent kernel, one wave per SIMD, cannot hide.  ne is the same for
    // the whole workgroup; an empty chunk gathers entry 0 (m, n >= 1).
    const bool ne = uni(ke) > uni(kb);
    int ci[UNR];
    T vv[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int o = tid + u * BLOCK;
      const int oc = kb + o < ke ? o : ke - 1 - kb;
      ci[u] = 0;
      vv[u] = (T)0;
      if (ne) {
        if constexpr (COH) {
          ci[u] = CACHED ? cidx[oc] : idx[kb + oc];
          vv[u] = val[kb + oc];
        } else {
          // a launch streams the matrix once: non-temporal, so the gathered
          // vector keeps its place in L2
          ci[u] = __builtin_nontemporal_load(&idx[kb + oc]);
          vv[u] = __builtin_nontemporal_load(&val[kb + oc]);
        }
      }
    }
    int a0 = 0, a1 = 0;
    RowIn<T, MT> rin;
    if (r < r1) {
      a0 = CACHED ? ca0[tid] : ptr[r] - kb;
      a1 = CACHED ? ca1[tid] : ptr[r + 1] - kb;
      if (has_row && lane_r == 0) load_row(row, rin, false);
    }
    double sum1 = 0.0, sum2 = 0.0;
    const int nsweep = two ? 2 : 1;
    for (int sw = 0; sw < nsweep; ++sw) {
      const T* gv = sw == 0 ? gv1 : gv2;
      T gg[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) gg[u] = gather(gv, ci[u]);
      __syncthreads();  // s_prod is free
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int q = tid + u * BLOCK;
        if (kb + q < ke) s_prod[q] = (double)vv[u] * (double)gg[u];
      }
      __syncthreads();
      double sres;
      if (blockmode) {
        double s = 0.0;
        for (int q = a0 + tid; q < a1; q += BLOCK) s += s_prod[q];
        sres = block_sum(s, s_tmp);
      } else {
        // four independent partial sums keep several LDS reads in flight
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int q = a0 + lane_r;
        for (; q + 3 * tpr < a1; q += 4 * tpr) {
          s0 += s_prod[q];
          s1 += s_prod[q + tpr];
          s2 += s_prod[q + 2 * tpr];
          s3 += s_prod[q + 3 * tpr];
        }
        for (; q < a1; q += tpr) s0 += s_prod[q];
        double s = (s0 + s1) + (s2 + s3);
        for (int off = 1; off < tpr; off <<= 1) s += __shfl_xor(s, off, 64);
        sres = s;
      }
      if (sw == 0) sum1 = sres; else sum2 = sres;
    }
    if (has_row && lane_r == 0) finish_row(row, rin, sum1, sum2, acc, false);
  }

  // ---- one part of a split row: partial sums; the last part to arrive
  // finishes the row and writes its record.  True in that workgroup.
  __device__ __forceinline__ bool split_part(const Chunk& ch, const SplitRow* splits, double* splitpart,
                                             unsigned int* splitcnt, double* rec, double* s_tmp, double* s_racc,
                                             int* s_own) const {
    constexpr int UNR = CHUNK_NNZ / BLOCK;
    const int tid = threadIdx.x;
    const SplitRow sr = splits[ch.split];
    const int kb = ch.k0, ke = ch.k1, part = ch.tpr;
    double s1 = 0.0, s2 = 0.0;
    for (int base = kb; base < ke; base += UNR * BLOCK) {
      int ci[UNR];
      T vv[UNR], g1[UNR], g2[UNR];
      // every load is made (positions past the part's end read its last
      // entry) and the values past the end are then set to zero
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int q = base + tid + u * BLOCK;
        const int qc = q < ke ? q : ke - 1;
        ci[u] = COH ? idx[qc] : __builtin_nontemporal_load(&idx[qc]);
        vv[u] = COH ? val[qc] : __builtin_nontemporal_load(&val[qc]);
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) g1[u] = gather(gv1, ci[u]);
      if (two) {
#pragma unroll
        for (int u = 0; u < UNR; ++u) g2[u] = gather(gv2, ci[u]);
      } else {
#pragma unroll
        for (int u = 0; u < UNR; ++u) g2[u] = (T)0;
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const bool ok = base + tid + u * BLOCK < ke;
        vv[u] = ok ? vv[u] : (T)0;
        g1[u] = ok ? g1[u] : (T)0;
        g2[u] = ok ? g2[u] : (T)0;
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        s1 += (double)vv[u] * (double)g1[u];
        s2 += (double)vv[u] * (double)g2[u];
      }
    }
    s1 = block_sum(s1, s_tmp);
    s2 = block_sum(s2, s_tmp);
    if (tid == 0) {
      st_agent(&splitpart[2 * (sr.part0 + part) + 0], s1);
      st_agent(&splitpart[2 * (sr.part0 + part) + 1], s2);
      *s_own = arrive(&splitcnt[ch.split], (unsigned)sr.nparts);
    }
    __syncthreads();
    if (!*s_own) return false;
    if (tid == 0) {
      reset_counter(&splitcnt[ch.split]);
      RowIn<T, MT> in;
      const int row = rmap[sr.row];
      load_row(row, in, true);
      // the parts' sums in part order
      const double t1 = ordered_sum_coh<16>(splitpart, 2 * sr.part0 + 0, 2, sr.nparts);
      const double t2 = ordered_sum_coh<16>(splitpart, 2 * sr.part0 + 1, 2, sr.nparts);
      for (int q = 0; q < DT::COUNT; ++q) s_racc[q] = 0.0;
      finish_row(row, in, t1, t2, s_racc, true);
      double* rp = rec + (size_t)sr.leaf * NDOT;
      for (int q = 0; q < DT::COUNT; ++q) st_agent(&rp[q], s_racc[q]);
    }
    return true;
  }
};

// The record of one workgroup: the sums of its threads' C values, in a fixed
// order.  Lanes are first added in groups of GL (DPP: pairs, quads and, for
// GL = 8, half rows), every group's C sums go to LDS (s_buf, free on entry),
// then PARTS threads per value add NG / PARTS groups each in order and finish
// with DPP over their PARTS lanes.  With lane0_only the caller guarantees
// that only lane 0 of each wave holds non-zero sums (one row per wave or per
// workgroup): the four wave values are then added in order.
template <int MT>
__device__ __forceinline__ void write_record(double* acc, double (*s_red)[NDOT], double* out, bool lane0_only,
                                             double* s_buf) {
  constexpr int C = Dot<MT>::COUNT;
  constexpr int GL = 64 * C <= CHUNK_NNZ ? 4 : 8;  // lanes per group
  constexpr int NG = BLOCK / GL;                    // groups of the workgroup
  constexpr int PARTS = 8 * C <= BLOCK ? 8 : 4;     // threads per value in the second stage
  constexpr int PER = NG / PARTS;                   // groups per thread
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (lane0_only) {
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < C; ++q) s_red[wv][q] = acc[q];
    }
    __syncthreads();
    if (tid < C) st_agent(&out[tid], ((s_red[0][tid] + s_red[1][tid]) + s_red[2][tid]) + s_red[3][tid]);
    return;
  }
#pragma unroll
  for (int q = 0; q < C; ++q) acc[q] += dpp_mov<0xB1, 0xF>(acc[q]);  // pairs
#pragma unroll
  for (int q = 0; q < C; ++q) acc[q] += dpp_mov<0x4E, 0xF>(acc[q]);  // quads
  if (GL == 8) {
#pragma unroll
    for (int q = 0; q < C; ++q) acc[q] += dpp_mov<0x141, 0xF>(acc[q]);  // half rows
  }
  __syncthreads();  // s_buf is free
  if ((tid & (GL - 1)) == 0) {
#pragma unroll
    for (int q = 0; q < C; ++q) s_buf[(tid / GL) * C + q] = acc[q];
  }
  __syncthreads();
  const int q = tid / PARTS, part = tid % PARTS;
  double v = 0.0;
  if (q < C) {
#pragma unroll
    for (int g = 0; g < PER; ++g) v += s_buf[(part * PER + g) * C + q];
  }
  v += dpp_mov<0xB1, 0xF>(v);
  v += dpp_mov<0x4E, 0xF>(v);
  if (PARTS == 8) v += dpp_mov<0x141, 0xF>(v);
  if (q < C && part == 0) st_agent(&out[q], v);
}

// DOTS: some LP of the launch takes the per-pass dots of the new difference
// column with the stored ones (gram_mode); without it they are compiled out.
template <typename T, int MT, int PASS, bool DOTS>
__global__ __launch_bounds__(BLOCK) void k_pass(PassArgs a) {
  using DT = Dot<MT>;
  __shared__ double s_prod[CHUNK_NNZ];
  __shared__ double s_red[BLOCK / 64][NDOT];
  __shared__ double s_racc[NDOT];  // dot sums of one split row
  __shared__ double s_tmp[4];
  __shared__ int s_live[MAXM];
  __shared__ int s_own;

  const int tid = threadIdx.x;
  const BlockWork bw = a.blocks[blockIdx.x];
  const LPDesc* dp = a.lps + bw.lp;
  Scalars* sc = dp->sc;
  const bool eval = a.mode == MODE_EVAL;
  if (!eval && sc->status != ST_RUNNING) return;
  if (tid < MAXM) s_live[tid] = sc->live[tid];
  __syncthreads();
  PassView v = make_view(*dp, sc->k, sc->nlive, sc->newslot, s_live, eval, &sc->tau);
  // an LP that forms its Gram matrix on demand takes no dots with the stored columns
  if (!DOTS || dp->lazy_gram) v.ndot = 0;
  const PassCtx<T, MT, PASS, false, true> P(dp, v);

  if (bw.kind == 1) {
    const Chunk ch = a.chunks[bw.c0];
    P.split_part(ch, a.splits, a.splitpart, a.splitcnt, a.rec, s_tmp, s_racc, &s_own);
    return;
  }

  double acc[DT::COUNT];
#pragma unroll
  for (int q = 0; q < DT::COUNT; ++q) acc[q] = 0.0;
  bool lane0 = true;  // every chunk of the unit has one row per wave or workgroup
  if (PASS == 1 && dp->panels) {
    P.template panel_rows<2>(a.chunks, bw.c0, bw.c1, acc);
    lane0 = false;
  } else {
    for (int c = bw.c0; c < bw.c1; ++c) {
      const Chunk ch = a.chunks[c];
      lane0 &= ch.tpr >= 64;
      P.template multi_chunk<false>(ch, acc, s_prod, s_tmp);
    }
  }
  write_record<MT>(acc, s_red, a.rec + (size_t)bw.leaf * NDOT, lane0, s_prod);
}

// Decisions of a loop pass on the three-launch path, after pass B: every LP's
// records of both passes are added in a fixed order and its last workgroup
// runs final_step.  Workgroup b adds positions [r0, r1) of its LP's record
// list (thread (t, q) adds value q of positions r0 + t, r0 + t + PT, ... in
// order; then the PT sums of each value in order) into partial b; the last
// of the LP's workgroups to arrive adds the LP's partials in order.  The
// records were written by the previous launches, so only the partials need
// agent-scope stores and an arrival count.
template <typename T, int MT>
__global__ __launch_bounds__(BLOCK) void k_decide(PassArgs a) {
  using DT = Dot<MT>;
  constexpr int C = DT::COUNT;
  constexpr int PT = BLOCK / C;  // positions read at once
  __shared__ double s_part[BLOCK];
  __shared__ double s_fin[NDOT];
  __shared__ int s_live[MAXM];
  __shared__ int s_flag;
  __shared__ SolveWork s_work;
  __shared__ Scalars s_sc;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const DecideBlock db = a.dblocks[blockIdx.x];
  const LPDesc* dp = a.lps + db.lp;
  Scalars* sc = db.sc;
  const bool eval = a.mode == MODE_EVAL;
  // the LP's scalars (the decisions run on an LDS copy), loaded together with
  // the records; nothing in this launch writes them before its last workgroup
  constexpr int SW = sizeof(Scalars) / 8;
  constexpr int SPT = (SW + BLOCK - 1) / BLOCK;
  unsigned long long* gsc = reinterpret_cast<unsigned long long*>(sc);
  unsigned long long* lsc = reinterpret_cast<unsigned long long*>(&s_sc);
  unsigned long long sreg[SPT];
#pragma unroll
  for (int i = 0; i < SPT; ++i) sreg[i] = tid + i * BLOCK < SW ? gsc[tid + i * BLOCK] : 0ull;
  const int t = tid / C, q = tid - (tid / C) * C;
  double s = 0.0;
  if (t < PT) {
    // positions r0 + t, r0 + t + PT, ... added in order, RB loads issued
    // together (those past r1 read position p0 again and are not added)
    constexpr int RB = 16;
    for (int p0 = db.r0 + t; p0 < db.r1; p0 += RB * PT) {
      double v[RB];
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        const int p = p0 + u * PT < db.r1 ? p0 + u * PT : p0;
        const int rix = p < db.nA ? db.leafA + p : db.leafB + (p - db.nA);
        v[u] = a.rec[(size_t)rix * NDOT + q];
      }
#pragma unroll
      for (int u = 0; u < RB; ++u)
        if (p0 + u * PT < db.r1) s += v[u];
    }
  }
#pragma unroll
  for (int i = 0; i < SPT; ++i)
    if (tid + i * BLOCK < SW) lsc[tid + i * BLOCK] = sreg[i];
  s_part[tid] = s;
  __syncthreads();
  if (!eval && s_sc.status != ST_RUNNING) return;
  double part = 0.0;
  if (tid < C) {
    for (int tt = 0; tt < PT; ++tt) part += s_part[tt * C + tid];
  }
  if (db.nblk > 1) {
    if (tid < C) st_agent(&a.dpart[(size_t)db.slot * NDOT + tid], part);
    __syncthreads();
    if (wv == 0) {
      wait_stores();
      if (tid == 0) s_flag = arrive(&a.dcnt[db.lp], (unsigned)db.nblk);
    }
    __syncthreads();
    if (!s_flag) return;
    if (tid == 0) reset_counter(&a.dcnt[db.lp]);
    if (tid < C) {
      s_fin[tid] = ordered_sum_coh<16>(a.dpart, db.blk0 * NDOT + tid, NDOT, db.nblk);
    }
  } else if (tid < C) {
    s_fin[tid] = 0.0 + part;  // the ordered sum of the one partial
  }
  if (tid < MAXM) s_live[tid] = s_sc.live[tid];
  __syncthreads();
  const PassView v = make_view(*dp, s_sc.k, s_sc.nlive, s_sc.newslot, s_live, eval, &s_sc.tau);
  if (wv == 0) final_step<MT>(*dp, &s_sc, s_fin, eval, v.kkt, v.init, &s_work, lane, dp->lazy_gram != 0);
  __syncthreads();
  for (int w = tid; w < SW; w += BLOCK) gsc[w] = lsc[w];
}

// ---------------------------------------------------------------------------
// Gram launch (three-launch path): the history's Gram matrix on demand
// ---------------------------------------------------------------------------
//
// The passes of the three-launch path leave out the dots of each new
// difference column with the stored ones: those would read the whole history
// on every pass, while Anderson steps are a small share of the passes.  When
// a pass's safeguard test passes with a non-empty memory, its decisions are
// left pending (branch BR_GRAM); this launch then forms, from the stored
// columns, G = dG_L^T dG_L and r = dG_L^T g^k for the live slots L (Alg 2's
// Gram matrix and right-hand side) and the LP's last workgroup takes the
// step's decisions (gram_decide).  With refresh set it only brings G and
// r = dG_L^T g^{k-1} up to date for LPs whose passes left them stale, before
// the persistent kernel, which updates them pass by pass, takes the LPs over,
// or before they are read back.
// Workgroup b takes mix tile b (one tile each: on the passes that need nothing
// every workgroup reads the LP's scalars once and exits, all at the same
// time).  A tile's entries are added per thread in entry order, then within
// each wave (fixed DPP sequence) and over the four waves in order; the tile's
// values are stored value-major.  The workgroup that finishes the LP's last
// tile adds each value's partials in a fixed order (per LP): with at most 64
// tiles, one wave per value (lane l holds tile l) and its DPP sum; with more,
// lane l of the value's wave first adds tiles l, l + 64, ... in order.  The
// partials are read with many loads in flight: this sum is the serial tail of
// an Anderson step.  Values: G[a][b] for a <= b < MT at a MT - a (a - 1) / 2 + (b - a),
// then r[a] at MT (MT + 1) / 2 + a.
template <int MT>
__host__ __device__ constexpr int gram_values() {
  return MT * (MT + 1) / 2 + MT;
}

// Block-wide sums of the NV values of acc[] (fixed order: DPP within each
// wave, then the waves in order) into out[0..NV).
template <int NV>
__device__ __forceinline__ void block_sums(const double* acc, double (*s_red)[NV], double* out) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  constexpr int NW = BLOCK / 64;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    const double v = wave_sum(acc[q]);
    if (lane == 0) s_red[wv][q] = v;
  }
  __syncthreads();
  for (int q = tid; q < NV; q += BLOCK) {
    double v = s_red[0][q];
#pragma unroll
    for (int w = 1; w < NW; ++w) v += s_red[w][q];
    out[q] = v;
  }
  __syncthreads();
}

template <typename T, int MT>
__global__ __launch_bounds__(BLOCK) void k_gram(GramArgs a) {
  constexpr int NG = MT * (MT + 1) / 2;
  constexpr int NV = gram_values<MT>();
  __shared__ double s_red[BLOCK / 64][NV];
  __shared__ double s_val[NV];
  __shared__ int s_live[MAXM];
  __shared__ int s_flag;
  __shared__ SolveWork s_work;
  __shared__ Scalars s_sc;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int tix = blockIdx.x;
  const MixTile tl = a.tiles[tix];
  const LPDesc& d = a.lps[tl.lp];
  Scalars* sc = tl.sc;
  if (a.refresh) {
    if (sc->gram_ok != 0 || sc->nlive == 0) return;
  } else if (sc->status != ST_RUNNING || sc->branch != BR_GRAM) {
    return;
  }
  const int nl = sc->nlive;
  const long long k = sc->k;
  if (tid < MAXM) s_live[tid] = sc->live[tid];
  __syncthreads();
  // the residual of the last finished pass: g^k while its decisions are
  // pending, g^{k-1} once they are taken
  const T* __restrict__ g = (const T*)d.g[(int)((a.refresh ? k - 1 : k) & 1)];
  const T* __restrict__ dG = (const T*)d.dG;
  const size_t N = (size_t)d.N;
  // offsets of the live columns (uniform, from the scalars).  Every column
  // load is made and the unused ones masked (a load under a condition of its
  // own would be waited for before the next); those read the first live
  // column again.
  size_t col[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t) col[t] = (size_t)sc->live[t < nl ? t : 0] * N;
  double acc[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) acc[q] = 0.0;
  for (int e = tl.e0 + tid; e < tl.e1; e += BLOCK) {
    T hv[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) hv[t] = dG[col[t] + e];
    const double gv = (double)g[e];
    double h[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) h[t] = t < nl ? (double)hv[t] : 0.0;
    int q = 0;
#pragma unroll
    for (int i = 0; i < MT; ++i) {
#pragma unroll
      for (int j = i; j < MT; ++j) acc[q++] += h[i] * h[j];
    }
#pragma unroll
    for (int i = 0; i < MT; ++i) acc[NG + i] += h[i] * gv;
  }
  block_sums<NV>(acc, s_red, s_val);
  const int j = tix - tl.t0;
  double* part = a.gpart + (size_t)tl.t0 * NV;
  for (int q = tid; q < NV; q += BLOCK) st_agent(&part[(size_t)q * tl.nt + j], s_val[q]);
  wait_stores();
  __syncthreads();
  if (tid == 0) s_flag = arrive(&a.gcnt[tl.lp], (unsigned)tl.nt);
  __syncthreads();
  if (!s_flag) return;
  // ---- the LP's last tile: the sums over its tiles, then the decisions ----
  if (tid == 0) reset_counter(&a.gcnt[tl.lp]);
  constexpr int SW = sizeof(Scalars) / 8;
  unsigned long long* gsc = reinterpret_cast<unsigned long long*>(sc);
  unsigned long long* lsc = reinterpret_cast<unsigned long long*>(&s_sc);
  for (int w = tid; w < SW; w += BLOCK) lsc[w] = gsc[w];
  if (tl.nt <= 64) {
    // few tiles: wave w adds values w, w + 4, ... (lane l holds tile l), DPP
    // sum; the wave's loads are issued together first (lanes past the tiles
    // and values past NV read an existing partial, which is not used)
    constexpr int NW = BLOCK / 64;
    constexpr int QPW = (NV + NW - 1) / NW;
    const int tl_lane = lane < tl.nt ? lane : 0;
    double pv[QPW];
#pragma unroll
    for (int i = 0; i < QPW; ++i) {
      const int q = wv + i * NW;
      pv[i] = ld_coh(part, (q < NV ? q : 0) * tl.nt + tl_lane);
    }
#pragma unroll
    for (int i = 0; i < QPW; ++i) {
      const int q = wv + i * NW;
      const double v = wave_sum(lane < tl.nt ? pv[i] : 0.0);
      if (q < NV && lane == 0) s_val[q] = v;
    }
    __syncthreads();
  } else {
    // many tiles: wave w adds values w, w + 4, ...; lane l adds tiles l,
    // l + 64, ... of the value in order (24 loads issued together), then the
    // DPP sum over the lanes
    for (int q = wv; q < NV; q += BLOCK / 64) {
      const int cnt = lane < tl.nt ? (tl.nt - lane + 63) / 64 : 0;
      const double v = wave_sum(ordered_sum_coh<24>(part, q * tl.nt + lane, 64, cnt));
      if (lane == 0) s_val[q] = v;
    }
    __syncthreads();
  }
  if (tid < NV) {
    // value tid -> (row, column) of G, or the row of r
    int ia = -1, ib = -1;
    if (tid >= NG) {
      ia = tid - NG;
    } else {
      int q = tid, i = 0;
      while (q >= MT - i) {
        q -= MT - i;
        ++i;
      }
      ia = i;
      ib = i + q;
    }
    const double v = s_val[tid];
    if (ib < 0) {
      if (ia < nl) s_sc.rhs[s_live[ia]] = v;
    } else if (ia < nl && ib < nl) {
      s_sc.G[s_live[ia] * MAXM + s_live[ib]] = v;
      s_sc.G[s_live[ib] * MAXM + s_live[ia]] = v;
    }
  }
  __syncthreads();
  if (wv == 0) {
    if (a.refresh) {
      if (lane == 0) s_sc.gram_ok = 1;
    } else {
      gram_decide(d, &s_sc, &s_work, lane);
    }
  }
  __syncthreads();
  for (int w = tid; w < SW; w += BLOCK) gsc[w] = lsc[w];
}

// ---------------------------------------------------------------------------
// persistent loop kernel: many loop passes of Alg 2 / Alg 3 in one launch
// ---------------------------------------------------------------------------
//
// Every LP of the launch owns a group of workgroups (all resident: the launch
// is cooperative).  A workgroup always works on the same units of the CSC and
// CSR passes, so the rows it finishes (iterate, residual, history) stay its
// own from pass to pass; only the gathered vectors, x_bar, the records and
// the decisions cross workgroups, at agent scope.  Per pass:
//   phase A over the workgroup's CSC units, group barrier,
//   phase B over its CSR units, arrival;
//   rank 0 of the group adds the records of both phases in a fixed order,
//   takes the decisions (final_step) and publishes them;
//   on Anderson steps every workgroup mixes the entries it owns, then a group
//   barrier (the next phase A gathers the new y); with EXT, when the next
//   iteration is a primal-weight check (Alg 7), the same traversal adds the
//   distances to the anchor and every workgroup takes the weight decision
//   from the group's sums after that barrier.
// EXT = false compiles the primal-weight and restart paths out: the kernel of
// plain AA-PDHG / FAA-PDHG / PDHG sets keeps its registers for the passes.
// Every wait is bounded: after the wait limit (four seconds unless the
// options set it), or once another workgroup of the LP has given up, it
// returns false, the group leaves the loop and the launch reports the failure
// in *err.

__device__ __forceinline__ unsigned int ld_u32(const unsigned int* p) {
  return __hip_atomic_load(const_cast<unsigned int*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wave 0 only: wait until the NSUB sub-counters at `sub` add up to at least
// `target` (lane q < NSUB reads sub-counter q).
__device__ bool wait_sum_geq(const unsigned int* sub, unsigned int target, unsigned int* abortw,
                             unsigned long long ticks) {
  const int lane = threadIdx.x & 63;
  const unsigned long long t0 = wall_clock64();
  for (unsigned int it = 0;; ++it) {
    unsigned int v = lane < NSUB ? ld_u32(sub + lane * SUB_STRIDE) : 0u;
#pragma unroll
    for (int off = 1; off < NSUB; off <<= 1) v += __shfl_xor(v, off, 64);
    if (__shfl(v, 0, 64) >= target) return true;
    if ((it & 15u) == 15u) {
      const unsigned int ab = __shfl(lane == 0 ? ld_u32(abortw) : 0u, 0, 64);
      if (ab != 0u) return false;
      if (wall_clock64() - t0 > ticks) {
        if (lane == 0) __hip_atomic_store(abortw, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return false;
      }
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// Count this workgroup's arrival on its sub-counter (thread 0 only).
__device__ __forceinline__ void arrive_sub(unsigned int* sub, int rank) {
  __hip_atomic_fetch_add(sub + (rank % NSUB) * SUB_STRIDE, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Group barrier: every wave's stores complete, one arrival per workgroup,
// wait for `target` arrivals.  Every thread calls it.
__device__ __forceinline__ bool group_barrier(unsigned int* sub, int rank, unsigned int target, unsigned int* abortw,
                                              unsigned long long ticks, int* s_ok) {
  wait_stores();
  __syncthreads();
  if (threadIdx.x == 0) arrive_sub(sub, rank);
  if (threadIdx.x < 64) {
    const bool ok = wait_sum_geq(sub, target, abortw, ticks);
    if (threadIdx.x == 0) *s_ok = ok ? 1 : 0;
  }
  __syncthreads();
  return *s_ok != 0;
}

// Fixed-order sum of records: thread (q, s) adds records s, s + S, ... of
// slot q; the S partial sums are then added in order (and, with `add`, to
// what s_fin holds).
template <int MT>
__device__ __forceinline__ void reduce_records(const double* rec, int nrec, double* s_part, double* s_fin,
                                               bool add) {
  constexpr int C = Dot<MT>::COUNT;
  constexpr int QW = C <= 32 ? 32 : 64;
  constexpr int S = BLOCK / QW;
  constexpr int BATCH = 32;  // loads of one thread in flight together
  const int tid = threadIdx.x, q = tid % QW, s = tid / QW;
  double sum = 0.0;
  if (q < C) {
    for (int r0 = s; r0 < nrec; r0 += S * BATCH) {
      double v[BATCH];
#pragma unroll
      for (int j = 0; j < BATCH; ++j) {
        const int r = r0 + j * S;
        v[j] = r < nrec ? ld_coh(rec, r * NDOT + q) : 0.0;
      }
#pragma unroll
      for (int j = 0; j < BATCH; ++j) sum += v[j];
    }
  }
  s_part[tid] = sum;
  __syncthreads();
  if (tid < C) {
    double f = 0.0;
    for (int t = 0; t < S; ++t) f += s_part[t * QW + tid];
    s_fin[tid] = add ? s_fin[tid] + f : f;
  }
  __syncthreads();
}

// The entries of u a workgroup of the loop kernel owns: the columns of its
// CSC units, the rows of its CSR units (threads stride over them) and the
// split rows whose part 0 it holds (thread 0).  f(e, coh): coh is set for
// split rows, whose row data another workgroup may have written.
template <typename F>
__device__ __forceinline__ void for_owned(const LoopArgs& a, const LoopWG& wg, const LPDesc* dp, F&& f) {
  const int n = dp->n;
  for (int pass = 0; pass < 2; ++pass) {
    const BlockWork* bws = pass == 0 ? a.blocksA : a.blocksB;
    const int u0 = pass == 0 ? wg.a0 : wg.b0, u1 = pass == 0 ? wg.a1 : wg.b1;
    const int* rmap = pass == 0 ? dp->rmapA : dp->rmapB;
    const int off = pass == 0 ? 0 : n;
    for (int u = u0; u < u1; ++u) {
      const BlockWork bw = bws[u];
      if (bw.kind == 1) {
        const Chunk ch = a.chunks[bw.c0];
        if (ch.tpr == 0 && threadIdx.x == 0) f(off + rmap[a.splits[ch.split].row], true);
        continue;
      }
      for (int c = bw.c0; c < bw.c1; ++c) {
        const Chunk ch = a.chunks[c];
        for (int pos = ch.r0 + (int)threadIdx.x; pos < ch.r1; pos += BLOCK) f(off + rmap[pos], false);
      }
    }
  }
}

// One traversal of the entries this workgroup owns after the decisions of a
// pass (iterates at agent scope).  With `mix`: the Anderson mix of Alg 2,
// u^{k+1} = P(u^k + beta D-hat g^k - sum_t gamma_t W_t).  With `check` (Alg 7
// at the top of the next iteration): the squared distances of the new iterate
// to the anchor, x part in *sx and y part in *sy (per thread); the anchor then
// takes the new iterate.
template <typename T, bool EXT>
__device__ __forceinline__ void mix_owned(const LoopArgs& a, const LoopWG& wg, const LPDesc* dp, const Bcast& bc,
                                          bool mix, bool check, double* sx, double* sy) {
  const int par = (int)((bc.k - 1) & 1);  // the pass that decided was k-1
  const T* ucur = (const T*)dp->u[par];
  T* unext = (T*)dp->u[par ^ 1];
  const T* g = (const T*)dp->g[par];
  const T* W = (const T*)dp->W;
  const T* dhat = (const T*)dp->dhat;
  const T* lov = (const T*)dp->lo;
  const T* hiv = (const T*)dp->hi;
  T* anc = (T*)dp->anchor;
  const int n = dp->n, N = dp->N, nmix = bc.nmix;
  const double beta = dp->beta;
  double x2 = 0.0, y2 = 0.0;
  for_owned(a, wg, dp, [&](int e, bool c) {
    T r;
    if (mix) {
      double dh = (double)dhat[e];
      if constexpr (EXT) {
        const int p = e < n ? 0 : 1;
        dh = bc.dha[p] * dh + bc.dhb[p];
      }
      double v = (double)ldc(ucur, e) + beta * dh * (double)(c ? ldc(g, e) : g[e]);
      for (int t = 0; t < nmix; ++t) {
        const T* wc = W + (size_t)bc.mixslot[t] * N;
        v -= bc.gamma[t] * (double)(c ? ldc(wc, e) : wc[e]);
      }
      r = (T)v;
      if (e < n) {
        r = clampT(r, lov[e], hiv[e]);
      } else if (dp->rowtype[e - n] != 0 && r < (T)0) {
        r = (T)0;
      }
      stc(unext, e, r);
    } else {
      r = ldc((const T*)unext, e);  // a PDHG step: the new iterate is the PDHG point already written
    }
    if (EXT && check) {
      const double dd = (double)r - (double)anc[e];
      if (e < n) x2 += dd * dd; else y2 += dd * dd;
      anc[e] = r;
    }
  });
  *sx = x2;
  *sy = y2;
}

// A workgroup that owns exactly one multi-row chunk in a pass keeps it in LDS
// for the whole launch.
struct ChunkCache {
  int on;
  int leaf;
  Chunk ch;
  int idx[CHUNK_NNZ];  // column indices of the chunk's entries
  int row[BLOCK];      // original row of each thread's row group
  int a0[BLOCK], a1[BLOCK];
};

template <int PASS>
__device__ __forceinline__ void fill_cache(const LoopArgs& a, const LPDesc* dp, int u0, int u1, ChunkCache* cc) {
  const int tid = threadIdx.x;
  const BlockWork* bws = PASS == 0 ? a.blocksA : a.blocksB;
  bool on = false;
  BlockWork bw{};
  if (u1 - u0 == 1) {
    bw = bws[u0];
    on = bw.kind == 0 && bw.c1 - bw.c0 == 1;
  }
  if (tid == 0) cc->on = on ? 1 : 0;
  if (!on) return;
  const Chunk ch = a.chunks[bw.c0];
  if (tid == 0) {
    cc->ch = ch;
    cc->leaf = bw.leaf;
  }
  const int* ptr = PASS == 0 ? dp->colptr : dp->rowptr;
  const int* idx = PASS == 0 ? dp->rowidx : dp->colidx;
  const int* rmap = PASS == 0 ? dp->rmapA : dp->rmapB;
  for (int q = tid; q < ch.k1 - ch.k0; q += BLOCK) cc->idx[q] = idx[ch.k0 + q];
  const bool blockmode = ch.tpr == BLOCK;
  const int r = ch.r0 + (blockmode ? 0 : tid / ch.tpr);
  cc->row[tid] = r < ch.r1 ? rmap[r] : 0;
  cc->a0[tid] = r < ch.r1 ? ptr[r] - ch.k0 : 0;
  cc->a1[tid] = r < ch.r1 ? ptr[r + 1] - ch.k0 : 0;
}

template <typename T, int MT, int PASS, bool EXT>
__device__ __forceinline__ void loop_units(const LoopArgs& a, const LPDesc* dp, const PassView& v, int u0, int u1,
                                           double* s_prod, double (*s_red)[NDOT], double* s_tmp, double* s_racc,
                                           int* s_own, const ChunkCache* cc) {
  using DT = Dot<MT>;
  const PassCtx<T, MT, PASS, true, EXT> P(dp, v);
  if (cc->on) {
    double acc[DT::COUNT];
#pragma unroll
    for (int q = 0; q < DT::COUNT; ++q) acc[q] = 0.0;
    P.template multi_chunk<true>(cc->ch, acc, s_prod, s_tmp, cc->idx, cc->row, cc->a0, cc->a1);
    write_record<MT>(acc, s_red, a.rec + (size_t)cc->leaf * NDOT, cc->ch.tpr >= 64, s_prod);
    return;
  }
  const BlockWork* bws = PASS == 0 ? a.blocksA : a.blocksB;
  for (int u = u0; u < u1; ++u) {
    const BlockWork bw = bws[u];
    if (bw.kind == 1) {
      P.split_part(a.chunks[bw.c0], a.splits, a.splitpart, a.splitcnt, a.rec, s_tmp, s_racc, s_own);
      __syncthreads();  // s_own, s_racc and s_tmp are reused
      continue;
    }
    double acc[DT::COUNT];
#pragma unroll
    for (int q = 0; q < DT::COUNT; ++q) acc[q] = 0.0;
    bool lane0 = true;
    for (int c = bw.c0; c < bw.c1; ++c) {
      const Chunk ch = a.chunks[c];
      lane0 &= ch.tpr >= 64;
      P.template multi_chunk<false>(ch, acc, s_prod, s_tmp);
    }
    write_record<MT>(acc, s_red, a.rec + (size_t)bw.leaf * NDOT, lane0, s_prod);
  }
}

// Wave 0 of rank 0: publish the decisions of a pass as tagged words, in
// every copy of the message (see BcastMsg).
__device__ __forceinline__ void publish_decisions(const Bcast& b, unsigned long long* msg, unsigned int tag) {
  const int lane = threadIdx.x & 63;
  unsigned int pay = 0;
  if (lane == 0) {
    pay = (unsigned)b.status | (unsigned)b.branch << 4 | (unsigned)b.nmix << 8 | (unsigned)b.nlive << 16 |
          (unsigned)b.newslot << 24;
  } else if (lane <= 4) {
    const int* src = lane <= 2 ? b.live : b.mixslot;
    const int base = ((lane - 1) & 1) * 8;
    for (int t = 0; t < 8; ++t) pay |= ((unsigned)src[base + t] & 15u) << (4 * t);
  } else if (lane < 5 + 2 * MAXM) {
    const int t = (lane - 5) >> 1;
    const double gv = b.gamma[t];
    pay = ((lane - 5) & 1) ? (unsigned)__double2hiint(gv) : (unsigned)__double2loint(gv);
  } else if (lane == 5 + 2 * MAXM) {
    pay = (unsigned)b.blend;
  }
  if (lane < BC_WORDS) {
    const unsigned long long wv = (unsigned long long)pay | (unsigned long long)tag << 32;
    for (int c = 0; c < BC_COPIES; ++c) stc(reinterpret_cast<double*>(msg + 64 * c), lane, __builtin_bit_cast(double, wv));
  }
}

// Wave 0 of the other ranks: wait until every word carries `tag`, then
// unpack into b (k becomes k_next).  Bounded like every wait.
__device__ bool read_decisions(Bcast& b, const unsigned long long* msg, unsigned int tag, long long k_next,
                               unsigned int* abortw, unsigned long long ticks) {
  const int lane = threadIdx.x & 63;
  const unsigned long long t0 = wall_clock64();
  unsigned long long wv = 0;
  for (unsigned int it = 0;; ++it) {
    if (lane < BC_WORDS) wv = __builtin_bit_cast(unsigned long long, ldc(reinterpret_cast<const double*>(msg), lane));
    const bool stale = lane < BC_WORDS && (unsigned int)(wv >> 32) != tag;
    if (__ballot(stale) == 0ull) break;
    if ((it & 15u) == 15u) {
      const unsigned int ab = __shfl(lane == 0 ? ld_u32(abortw) : 0u, 0, 64);
      if (ab != 0u) return false;
      if (wall_clock64() - t0 > ticks) {
        if (lane == 0) __hip_atomic_store(abortw, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return false;
      }
    }
    __builtin_amdgcn_s_sleep(1);
  }
  const unsigned int pay = (unsigned int)wv;
  const unsigned int w0 = __shfl(pay, 0, 64);
  if (lane == 0) {
    b.k = k_next;
    b.status = (int)(w0 & 15u);
    b.branch = (int)((w0 >> 4) & 15u);
    b.nmix = (int)((w0 >> 8) & 255u);
    b.nlive = (int)((w0 >> 16) & 255u);
    b.newslot = (int)(w0 >> 24);
  }
  const unsigned int l0 = __shfl(pay, 1, 64), l1 = __shfl(pay, 2, 64);
  const unsigned int m0 = __shfl(pay, 3, 64), m1 = __shfl(pay, 4, 64);
  const unsigned int glo = __shfl(pay, 5 + 2 * (lane & (MAXM - 1)), 64);
  const unsigned int ghi = __shfl(pay, 6 + 2 * (lane & (MAXM - 1)), 64);
  const unsigned int bl = __shfl(pay, 5 + 2 * MAXM, 64);
  if (lane == 0) b.blend = (int)bl;
  if (lane < MAXM) {
    const unsigned int lw = lane < 8 ? l0 : l1, mw = lane < 8 ? m0 : m1;
    b.live[lane] = (int)((lw >> (4 * (lane & 7))) & 15u);
    b.mixslot[lane] = (int)((mw >> (4 * (lane & 7))) & 15u);
    b.gamma[lane] = __hiloint2double((int)ghi, (int)glo);
  }
  return true;
}

template <typename T, int MT, bool EXT>
__global__ __launch_bounds__(BLOCK) void k_loop(LoopArgs a) {
  __shared__ double s_prod[CHUNK_NNZ];
  __shared__ double s_red[BLOCK / 64][NDOT];
  __shared__ double s_fin[NDOT];
  __shared__ double s_racc[NDOT];
  __shared__ double s_tmp[4];
  __shared__ double s_part[BLOCK];
  __shared__ int s_own;
  __shared__ int s_ok;
  __shared__ Bcast s_bc;
  __shared__ SolveWork s_work;
  __shared__ Scalars s_sc;
  __shared__ ChunkCache s_cc[2];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const LoopWG wg = a.wgs[blockIdx.x];
  const LPDesc* dp = a.lps + wg.lp;
  const LoopLP L = a.llp[wg.lp];
  LoopSync* sy = a.sync + wg.lp;
  Scalars* sc = dp->sc;
  // Scalars change only at the end of the launch (rank 0 writes them back
  // after every workgroup of the group has passed the first barrier).
  if (sc->status != ST_RUNNING || sc->k < 1) return;
  const bool root = wg.rank == 0;
  if (tid == 0) {
    s_bc.k = sc->k;
    s_bc.status = sc->status;
    s_bc.branch = sc->branch;
    s_bc.nmix = 0;
    s_bc.nlive = sc->nlive;
    s_bc.newslot = sc->newslot;
    s_bc.blend = 0;
    s_bc.omega = sc->omega;
    s_bc.tau = sc->tau;
    s_bc.sigma = sc->sigma;
    s_bc.dha[0] = sc->dha[0];
    s_bc.dha[1] = sc->dha[1];
    s_bc.dhb[0] = sc->dhb[0];
    s_bc.dhb[1] = sc->dhb[1];
  }
  if (tid < MAXM) s_bc.live[tid] = sc->live[tid];
  constexpr int SW = sizeof(Scalars) / 8;
  unsigned long long* gsc = reinterpret_cast<unsigned long long*>(sc);
  unsigned long long* lsc = reinterpret_cast<unsigned long long*>(&s_sc);
  if (root)
    for (int q = tid; q < SW; q += BLOCK) lsc[q] = gsc[q];
  fill_cache<0>(a, dp, wg.a0, wg.a1, &s_cc[0]);
  fill_cache<1>(a, dp, wg.b0, wg.b1, &s_cc[1]);
  __syncthreads();

  unsigned long long* msg = a.bc[wg.lp].w;
  const unsigned long long ticks = a.timeout_ticks;
  unsigned int nbar = 0;
  bool ok = true;
  for (long long it = 0; it < a.max_passes; ++it) {
    const PassView v = make_view(*dp, s_bc.k, s_bc.nlive, s_bc.newslot, s_bc.live, false, &s_bc.tau);
    // ---- phase A: K^T y and the primal update ----
    loop_units<T, MT, 0, EXT>(a, dp, v, wg.a0, wg.a1, s_prod, s_red, s_tmp, s_racc, &s_own, &s_cc[0]);
    ++nbar;
    if (!group_barrier(sy->bar, wg.rank, nbar * (unsigned)L.nwg, &sy->abort, ticks, &s_ok)) {
      ok = false;
      break;
    }
    // ---- phase B: K x_bar and the dual update ----
    loop_units<T, MT, 1, EXT>(a, dp, v, wg.b0, wg.b1, s_prod, s_red, s_tmp, s_racc, &s_own, &s_cc[1]);
    wait_stores();
    __syncthreads();
    if (tid == 0) arrive_sub(sy->arr, wg.rank);
    const unsigned int done = (unsigned int)(it + 1);
    if (root) {
      // ---- decisions of the pass ----
      // the CSC records are complete since the barrier: add them while the
      // CSR phase finishes elsewhere
      reduce_records<MT>(a.rec + (size_t)L.leaf0 * NDOT, L.nleafA, s_part, s_fin, false);
      if (tid < 64) {
        const bool okw = wait_sum_geq(sy->arr, done * (unsigned)L.nwg, &sy->abort, ticks);
        if (tid == 0) s_ok = okw ? 1 : 0;
      }
      __syncthreads();
      if (!s_ok) {
        ok = false;
        break;
      }
      reduce_records<MT>(a.rec + (size_t)(L.leaf0 + L.nleafA) * NDOT, L.nleaf - L.nleafA, s_part, s_fin, true);
      if (wv == 0) final_step<MT>(*dp, &s_sc, s_fin, false, v.kkt, false, &s_work, lane, false);
      __syncthreads();
      if (tid == 0) {
        s_bc.k = s_sc.k;
        s_bc.status = s_sc.status;
        s_bc.branch = s_sc.branch;
        s_bc.nmix = s_sc.nmix;
        s_bc.nlive = s_sc.nlive;
        s_bc.newslot = s_sc.newslot;
        if (EXT) {
          s_bc.blend = s_sc.pw_blend;
          for (int p = 0; p < 2; ++p) {
            s_bc.dha[p] = s_sc.dha[p];
            s_bc.dhb[p] = s_sc.dhb[p];
          }
        }
      }
      if (tid < MAXM) {
        s_bc.live[tid] = s_sc.live[tid];
        s_bc.mixslot[tid] = s_sc.mixslot[tid];
        s_bc.gamma[tid] = s_sc.gamma[tid];
      }
      __syncthreads();
      if (tid < 64) publish_decisions(s_bc, msg, a.tag0 + done);
    } else {
      if (tid < 64) {
        const bool okw = read_decisions(s_bc, msg + 64 * (wg.rank % BC_COPIES), a.tag0 + done, s_bc.k + 1, &sy->abort, ticks);
        if (tid == 0) s_ok = okw ? 1 : 0;
      }
      if (EXT && tid == 0 && s_ok && s_bc.blend != 0)  // the D-hat re-blend rank 0 made in final_step
        dhat_coeffs(s_bc.blend == 2 ? 0.1 : 0.9, s_bc.omega, s_bc.dha, s_bc.dhb);
      __syncthreads();
      if (!s_ok) {
        ok = false;
        break;
      }
    }
    if (s_bc.status != ST_RUNNING) break;
    const bool mix = s_bc.branch == BR_AA;
    const bool check = EXT && dp->pw_period > 0 && s_bc.k % dp->pw_period == 0;
    if (mix || check) {
      // the mix of an AA step and/or the distances of Alg 7's check, then a
      // group barrier (the next phase A gathers the new y; the check's sums
      // are complete)
      double sx, sy2;
      mix_owned<T, EXT>(a, wg, dp, s_bc, mix, check, &sx, &sy2);
      if (check) {
        sx = block_sum(sx, s_tmp);
        sy2 = block_sum(sy2, s_tmp);
        if (tid == 0) {
          st_agent(&a.pwrec[2 * blockIdx.x], sx);
          st_agent(&a.pwrec[2 * blockIdx.x + 1], sy2);
        }
      }
      ++nbar;
      if (!group_barrier(sy->bar, wg.rank, nbar * (unsigned)L.nwg, &sy->abort, ticks, &s_ok)) {
        ok = false;
        break;
      }
      if (check) {
        // every workgroup adds the group's sums in the same order and takes
        // the same decision; rank 0 keeps it in the LP's scalars
        if (tid < 64) {
          double px = 0.0, py = 0.0;
          for (int r = lane; r < L.nwg; r += 64) {
            px += ld_coh(a.pwrec, 2 * (L.wg0 + r));
            py += ld_coh(a.pwrec, 2 * (L.wg0 + r) + 1);
          }
          px = wave_sum(px);
          py = wave_sum(py);
          if (tid == 0) {
            double om = s_bc.omega, ta = s_bc.tau, si = s_bc.sigma;
            if (pw_decide(*dp, px, py, sc->gstep, om, ta, si)) {
              s_bc.omega = om;
              s_bc.tau = ta;
              s_bc.sigma = si;
              s_bc.nlive = 0;
              s_bc.newslot = 0;
              if (root) {
                s_sc.omega = om;
                s_sc.tau = ta;
                s_sc.sigma = si;
                s_sc.nlive = 0;
                s_sc.newslot = 0;
                s_sc.pw_flag = 1;
                s_sc.pw_updates += 1;
              }
            }
          }
        }
        __syncthreads();
      }
    }
  }
  if (!ok && tid == 0) __hip_atomic_store(a.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (root) {
    __syncthreads();
    if (!ok && tid == 0) {
      s_sc.status = ST_NUMERICAL;
      s_sc.branch = BR_NONE;
    }
    __syncthreads();
    for (int q = tid; q < SW; q += BLOCK) gsc[q] = lsc[q];
  }
}

// ---------------------------------------------------------------------------
// column panels of the dual product (large LPs): row sums per panel
// ---------------------------------------------------------------------------

// Workgroup b works on panel b % NP (NP = panel_count): workgroups are dealt
// to the eight XCDs in turn, so each XCD gathers from one 1/NP slice of x_bar
// (with 4 panels XCDs p and p + 4 share panel p), which stays in its L2.  A
// workgroup takes every (gridDim / NP)-th chunk of its panel:
// stages the chunk's products in LDS (eight gathers in flight per thread),
// then each thread adds the entries of up to four rows in order.  Writes
// part[0][p][r] (x_bar, or x^k when evaluating) and, on KKT passes,
// part[1][p][r] (x^k).  The chunk table holds each chunk's first row and
// first entry, so a chunk's loads depend on one table read; the indices,
// values and row ranges of the next chunk are loaded while the current one
// is summed.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_panel(const LPDesc* lps, int mode) {
  constexpr int UNR = CHUNK_NNZ / BLOCK;
  constexpr int RPT = PANEL_ROWS / BLOCK;
  __shared__ double s_p[CHUNK_NNZ];
  const LPDesc& d = lps[0];
  const Scalars* sc = d.sc;
  const bool eval = mode == MODE_EVAL;
  if (!eval && sc->status != ST_RUNNING) return;
  const long long k = sc->k;
  const bool init = !eval && k == 0;
  const bool kkt = eval || (!init && d.kkt_every > 0 && (k % d.kkt_every) == 0);
  const T* ucur = (const T*)d.u[(int)(k & 1)];
  const T* __restrict__ gv1 = eval ? ucur : (const T*)d.xbar;
  const T* __restrict__ gv2 = ucur;
  const bool two = kkt && !eval;
  const int tid = threadIdx.x;
  constexpr int NP = panel_count(sizeof(T) == 8);
  const int p = blockIdx.x % NP;
  const int j = blockIdx.x / NP, nj = gridDim.x / NP;
  const int m = d.m;
  const int* __restrict__ ptr = d.pptr + (size_t)p * (m + 1);
  const int* __restrict__ idx = d.pidx;
  const T* __restrict__ val = (const T*)d.pval;
  const int* __restrict__ cst = d.pchunk + 2 * d.pcoff[p];  // (first row, first entry) per chunk
  const int nch = d.pcoff[p + 1] - d.pcoff[p] - 1;
  double* __restrict__ out1 = d.part + (size_t)p * m;
  double* __restrict__ out2 = d.part + (size_t)(NP + p) * m;
  // the chunk's loads: column indices, values and this thread's row ranges
  int ci[UNR], ra[RPT], rb[RPT];
  T vv[UNR];
  auto load = [&](int c, int* lci, T* lvv, int* lra, int* lrb) {
    const int r0 = cst[2 * c], kb = cst[2 * c + 1];
    const int r1 = cst[2 * c + 2], ke = cst[2 * c + 3];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int q = kb + tid + u * BLOCK;
      lci[u] = q < ke ? idx[q] : 0;
      lvv[u] = q < ke ? val[q] : (T)0;
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = r0 + tid + i * BLOCK;
      lra[i] = r < r1 ? ptr[r] - kb : 0;
      lrb[i] = r < r1 ? ptr[r + 1] - kb : 0;
    }
  };
  int c = j;
  if (c >= nch) return;
  load(c, ci, vv, ra, rb);
  for (;;) {
    const int r0 = cst[2 * c], kb = cst[2 * c + 1];
    const int r1 = cst[2 * c + 2], ke = cst[2 * c + 3];
    T g1[UNR], g2[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const bool ok = kb + tid + u * BLOCK < ke;
      g1[u] = ok ? gv1[ci[u]] : (T)0;
      g2[u] = (ok && two) ? gv2[ci[u]] : (T)0;
    }
    // products of this chunk into registers, then the next chunk's loads
    double pr1[UNR], pr2[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      pr1[u] = (double)vv[u] * (double)g1[u];
      pr2[u] = (double)vv[u] * (double)g2[u];
    }
    int sra[RPT], srb[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      sra[i] = ra[i];
      srb[i] = rb[i];
    }
    const int cn = c + nj;
    if (cn < nch) load(cn, ci, vv, ra, rb);
    // one sweep per gathered vector (the second only on KKT passes)
    for (int sw = 0; sw < (two ? 2 : 1); ++sw) {
      __syncthreads();  // the previous sums are done with the LDS
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int q = tid + u * BLOCK;
        if (kb + q < ke) s_p[q] = sw == 0 ? pr1[u] : pr2[u];
      }
      __syncthreads();
      double* out = sw == 0 ? out1 : out2;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int r = r0 + tid + i * BLOCK;
        if (r < r1) {
          double a = 0.0;
          for (int q = sra[i]; q < srb[i]; ++q) a += s_p[q];
          out[r] = a;
        }
      }
    }
    if (cn >= nch) break;
    c = cn;
  }
}

// Pass C: the Anderson mix of Alg 2 on AA steps, and the weight check of
// Alg 7 when the next iteration k is a multiple of U_P: every tile adds the
// squared distances of its entries of u^k to the anchor (which then takes
// u^k); the last tile of the LP to arrive adds the tiles' sums in order and
// updates the weight, the step sizes and the memory in the LP's scalars.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_mix(MixArgs a) {
  __shared__ double s_gam[MAXM];
  __shared__ int s_slot[MAXM];
  __shared__ double s_tmp[4];
  __shared__ int s_last;
  const MixTile tl = a.tiles[blockIdx.x];
  const LPDesc& d = a.lps[tl.lp];
  Scalars* sc = tl.sc;
  if (sc->status != ST_RUNNING) return;
  const bool mix = sc->branch == BR_AA;
  const bool check = d.pw_period > 0 && sc->k % d.pw_period == 0;
  if (!mix && !check) return;
  const int par = (int)((sc->k - 1) & 1);  // the pass that decided was k-1
  const T* ucur = (const T*)d.u[par];
  T* unext = (T*)d.u[par ^ 1];  // u^k once the mix is done
  const int n = d.n, N = d.N;
  if (mix) {
    const int nmix = sc->nmix;
    if (threadIdx.x < MAXM) {
      s_gam[threadIdx.x] = sc->gamma[threadIdx.x];
      s_slot[threadIdx.x] = sc->mixslot[threadIdx.x];
    }
    __syncthreads();
    const T* g = (const T*)d.g[par];
    const T* W = (const T*)d.W;
    const T* dhat = (const T*)d.dhat;
    const double dha[2] = {sc->dha[0], sc->dha[1]}, dhb[2] = {sc->dhb[0], sc->dhb[1]};
    for (int e = tl.e0 + threadIdx.x; e < tl.e1; e += BLOCK) {
      const int p = e < n ? 0 : 1;
      const double dh = dha[p] * (double)dhat[e] + dhb[p];
      double v = (double)ucur[e] + d.beta * dh * (double)g[e];
      for (int t = 0; t < nmix; ++t) v -= s_gam[t] * (double)W[(size_t)s_slot[t] * N + e];
      T r = (T)v;
      if (e < n) {
        r = clampT(r, ((const T*)d.lo)[e], ((const T*)d.hi)[e]);
      } else if (d.rowtype[e - n] != 0 && r < (T)0) {
        r = (T)0;
      }
      unext[e] = r;
    }
  }
  if (!check) return;
  T* anc = (T*)d.anchor;
  double x2 = 0.0, y2 = 0.0;
  for (int e = tl.e0 + threadIdx.x; e < tl.e1; e += BLOCK) {
    const T v = unext[e];
    const double dd = (double)v - (double)anc[e];
    if (e < n) x2 += dd * dd; else y2 += dd * dd;
    anc[e] = v;
  }
  x2 = block_sum(x2, s_tmp);
  y2 = block_sum(y2, s_tmp);
  if (threadIdx.x == 0) {
    st_agent(&a.pwpart[2 * blockIdx.x], x2);
    st_agent(&a.pwpart[2 * blockIdx.x + 1], y2);
    s_last = arrive(&a.pwcnt[tl.lp], (unsigned)tl.nt) ? 1 : 0;
  }
  __syncthreads();
  if (!s_last || threadIdx.x >= 64) return;
  const int lane = threadIdx.x;
  if (lane == 0) reset_counter(&a.pwcnt[tl.lp]);
  double px = 0.0, py = 0.0;
  for (int t = lane; t < tl.nt; t += 64) {
    px += ld_coh(a.pwpart, 2 * (tl.t0 + t));
    py += ld_coh(a.pwpart, 2 * (tl.t0 + t) + 1);
  }
  px = wave_sum(px);
  py = wave_sum(py);
  if (lane == 0) {
    double om = sc->omega, ta = sc->tau, si = sc->sigma;
    if (pw_decide(d, px, py, sc->gstep, om, ta, si)) {
      sc->omega = om;
      sc->tau = ta;
      sc->sigma = si;
      sc->nlive = 0;
      sc->newslot = 0;
      sc->pw_flag = 1;
      sc->pw_updates += 1;
    }
  }
}

// ---------------------------------------------------------------------------
// set-up kernels
// ---------------------------------------------------------------------------

// u^0 = (clip(0, l, u), 0); the weight check's anchor starts at u^0 and the
// restart epoch's sum at 0
template <typename T>
__global__ void k_start_point(LPDesc d) {
  T* u0 = (T*)d.u[0];
  T* anc = (T*)d.anchor;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < d.N; e += gridDim.x * blockDim.x) {
    const T v = e < d.n ? clampT((T)0, ((const T*)d.lo)[e], ((const T*)d.hi)[e]) : (T)0;
    u0[e] = v;
    if (anc) anc[e] = v;
    if (d.rsum) d.rsum[e] = 0.0;
  }
}

// y = A x for CSR (ptr, idx, val), one wave per row, float64 vectors.
template <typename T>
__global__ void k_spmv_wave(const int* ptr, const int* idx, const T* val, const int* rmap, const double* x,
                            double* y, int rows) {
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int nw = (gridDim.x * blockDim.x) >> 6;
  for (int r = wave; r < rows; r += nw) {
    double s = 0.0;
    for (int q = ptr[r] + lane; q < ptr[r + 1]; q += 64) s += (double)val[q] * x[idx[q]];
    s = wave_sum(s);
    if (lane == 0) y[rmap[r]] = s;
  }
}

__global__ void k_sqnorm_part(const double* x, int len, double* part) {
  __shared__ double s_tmp[4];
  double s = 0.0;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < len; e += gridDim.x * blockDim.x) s += x[e] * x[e];
  s = block_sum(s, s_tmp);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// x = z / ||z|| with ||z||^2 = sum of nparts partials: thread t adds partials
// t, t + BLOCK, ... in order, then the block's fixed butterfly, so every block
// gets the same value; block 0 records ||z|| in est[slot].
__global__ void k_normalize(const double* z, double* x, int len, const double* part, int nparts, double* est, int slot) {
  __shared__ double s_norm;
  __shared__ double s_tmp[4];
  double s = 0.0;
  for (int p = threadIdx.x; p < nparts; p += BLOCK) s += part[p];
  s = block_sum(s, s_tmp);
  if (threadIdx.x == 0) {
    s_norm = sqrt(s);
    if (blockIdx.x == 0) est[slot] = s_norm;
  }
  __syncthreads();
  const double nz = s_norm;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < len; e += gridDim.x * blockDim.x) x[e] = nz > 0.0 ? z[e] / nz : 0.0;
}

// Start vector of the power iteration: x[j] = 2u - 1 with u the top 53 bits
// of output j of SplitMix64 (Steele, Lea and Flood, 2014) started at state
// `seed`, i.e. the mix of seed + (j + 1) * 0x9E3779B97F4A7C15, as a fraction
// of 2^53.
__global__ void k_fill_start(double* x, int len, unsigned long long seed) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < len; e += gridDim.x * blockDim.x) {
    unsigned long long z = seed + ((unsigned long long)e + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    x[e] = 2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0;
  }
}

// Copy the status word of every LP of a launch table into out[].
__global__ void k_gather_status(const LPDesc* lps, int count, int* out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) out[i] = lps[i].sc->status;
}

// Time limit reached: running LPs stop at their current iterate.
__global__ void k_time_limit(const LPDesc* lps, int count) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
    Scalars* sc = lps[i].sc;
    if (sc->status == ST_RUNNING) {
      sc->status = ST_TIME_LIMIT;
      sc->branch = BR_NONE;
    }
  }
}

// float64 <-> T conversions for host transfers
template <typename S, typename D>
__global__ void k_convert(const S* src, D* dst, size_t len) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < len; e += (size_t)gridDim.x * blockDim.x) dst[e] = (D)src[e];
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------

constexpr int PANEL_BLOCKS = 1024;  // workgroups of the panel kernel (4 per CU: every one resident)

template <typename T, int MT>
static hipError_t launch_passes_mt(const LaunchTables& t, hipStream_t st, int mode, hipEvent_t* ev) {
  PassArgs pa{};
  pa.lps = t.lps;
  pa.llp = t.llp;
  pa.chunks = t.chunks;
  pa.dblocks = t.dblocks;
  pa.splits = t.splits;
  pa.rec = t.rec;
  pa.dpart = t.dpart;
  pa.dcnt = t.dcnt;
  pa.splitpart = t.splitpart;
  pa.splitcnt = t.splitcnt;
  pa.nleaves = t.nleaves;
  pa.mode = mode;
  pa.blocks = t.blocksA;
  if (ev) (void)hipEventRecord(ev[0], st);
  if (t.nblocksA > 0) {
    if (t.dots)
      hipLaunchKernelGGL((k_pass<T, MT, 0, true>), dim3(t.nblocksA), dim3(BLOCK), 0, st, pa);
    else
      hipLaunchKernelGGL((k_pass<T, MT, 0, false>), dim3(t.nblocksA), dim3(BLOCK), 0, st, pa);
  }
  if (ev) (void)hipEventRecord(ev[1], st);
  if (t.panels) hipLaunchKernelGGL((k_panel<T>), dim3(PANEL_BLOCKS), dim3(BLOCK), 0, st, t.lps, mode);
  pa.blocks = t.blocksB;
  if (t.nblocksB > 0) {
    if (t.dots)
      hipLaunchKernelGGL((k_pass<T, MT, 1, true>), dim3(t.nblocksB), dim3(BLOCK), 0, st, pa);
    else
      hipLaunchKernelGGL((k_pass<T, MT, 1, false>), dim3(t.nblocksB), dim3(BLOCK), 0, st, pa);
  }
  if (t.ndblocks > 0) hipLaunchKernelGGL((k_decide<T, MT>), dim3(t.ndblocks), dim3(BLOCK), 0, st, pa);
  if (ev) (void)hipEventRecord(ev[2], st);
  if (mode == MODE_ITER && t.ntiles > 0) {
    if (t.gram) {
      const GramArgs ga{t.lps, t.tiles, t.gpart, t.gcnt, 0};
      hipLaunchKernelGGL((k_gram<T, MT>), dim3(t.ntiles), dim3(BLOCK), 0, st, ga);
    }
    MixArgs ma{t.lps, t.tiles, t.pwpart, t.pwcnt};
    hipLaunchKernelGGL((k_mix<T>), dim3(t.ntiles), dim3(BLOCK), 0, st, ma);
  }
  if (ev) (void)hipEventRecord(ev[3], st);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_passes_t(const LaunchTables& t, hipStream_t st, int mode, hipEvent_t* ev) {
  if (t.mt <= 4) return launch_passes_mt<T, 4>(t, st, mode, ev);
  if (t.mt <= 8) return launch_passes_mt<T, 8>(t, st, mode, ev);
  if (t.mt <= 10) return launch_passes_mt<T, 10>(t, st, mode, ev);
  return launch_passes_mt<T, 16>(t, st, mode, ev);
}

hipError_t launch_loop_pass(const LaunchTables& t, hipStream_t st, int mode, hipEvent_t* ev) {
  return t.fp64 ? launch_passes_t<double>(t, st, mode, ev) : launch_passes_t<float>(t, st, mode, ev);
}

// the memory bounds the kernels are instantiated for
static int mt_bucket(int mt) { return mt <= 4 ? 4 : mt <= 8 ? 8 : mt <= 10 ? 10 : 16; }

int gram_partials_per_tile(int mt) {
  switch (mt_bucket(mt)) {
    case 4: return gram_values<4>();
    case 8: return gram_values<8>();
    case 10: return gram_values<10>();
    default: return gram_values<16>();
  }
}

template <typename T>
static hipError_t gram_refresh_t(const LaunchTables& t, hipStream_t st) {
  if (t.ntiles <= 0 || !t.gram) return hipSuccess;
  const GramArgs ga{t.lps, t.tiles, t.gpart, t.gcnt, 1};
  const dim3 grid(t.ntiles);
  switch (mt_bucket(t.mt)) {
    case 4: hipLaunchKernelGGL((k_gram<T, 4>), grid, dim3(BLOCK), 0, st, ga); break;
    case 8: hipLaunchKernelGGL((k_gram<T, 8>), grid, dim3(BLOCK), 0, st, ga); break;
    case 10: hipLaunchKernelGGL((k_gram<T, 10>), grid, dim3(BLOCK), 0, st, ga); break;
    default: hipLaunchKernelGGL((k_gram<T, 16>), grid, dim3(BLOCK), 0, st, ga); break;
  }
  return hipGetLastError();
}

hipError_t launch_gram_refresh(const LaunchTables& t, hipStream_t st) {
  return t.fp64 ? gram_refresh_t<double>(t, st) : gram_refresh_t<float>(t, st);
}

template <typename T, bool EXT>
static const void* loop_kernel_mt(int mt) {
  if (mt <= 4) return reinterpret_cast<const void*>(&k_loop<T, 4, EXT>);
  if (mt <= 8) return reinterpret_cast<const void*>(&k_loop<T, 8, EXT>);
  if (mt <= 10) return reinterpret_cast<const void*>(&k_loop<T, 10, EXT>);
  return reinterpret_cast<const void*>(&k_loop<T, 16, EXT>);
}

static const void* loop_kernel_for(bool fp64, int mt, bool ext) {
  if (fp64) return ext ? loop_kernel_mt<double, true>(mt) : loop_kernel_mt<double, false>(mt);
  return ext ? loop_kernel_mt<float, true>(mt) : loop_kernel_mt<float, false>(mt);
}

template <typename T, int PASS, bool DOTS>
static const void* pass_kernel_mt(int mt) {
  if (mt <= 4) return reinterpret_cast<const void*>(&k_pass<T, 4, PASS, DOTS>);
  if (mt <= 8) return reinterpret_cast<const void*>(&k_pass<T, 8, PASS, DOTS>);
  if (mt <= 10) return reinterpret_cast<const void*>(&k_pass<T, 10, PASS, DOTS>);
  return reinterpret_cast<const void*>(&k_pass<T, 16, PASS, DOTS>);
}

template <typename T, bool DOTS>
static const void* pass_kernel_for(int mt, int pass) {
  return pass == 0 ? pass_kernel_mt<T, 0, DOTS>(mt) : pass_kernel_mt<T, 1, DOTS>(mt);
}

int pass_capacity(bool fp64, int mt, int pass, bool dots) {
  int dev = 0, cus = 0, nb = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const void* k = fp64 ? (dots ? pass_kernel_for<double, true>(mt, pass) : pass_kernel_for<double, false>(mt, pass))
                       : (dots ? pass_kernel_for<float, true>(mt, pass) : pass_kernel_for<float, false>(mt, pass));
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, BLOCK, 0) != hipSuccess) return 0;
  return nb * cus;
}

int loop_capacity(bool fp64, int mt, bool ext) {
  int dev = 0, cus = 0, coop = 0, nb = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, loop_kernel_for(fp64, mt, ext), BLOCK, 0) != hipSuccess)
    return 0;
  return nb * cus;
}

// Zero `words` 32-bit words at p (a fill kernel rather than a memset, so that
// the clear is an ordinary kernel node when a caller captures the stream).
__global__ void k_zero_u32(unsigned int* p, size_t words) {
  for (size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x; i < words; i += (size_t)gridDim.x * BLOCK) p[i] = 0u;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
  const size_t words = bytes / 4;
  if (words == 0) return hipSuccess;
  const size_t blocks = (words + BLOCK - 1) / BLOCK;
  hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)(blocks < 1024 ? blocks : 1024)), dim3(BLOCK), 0, st,
                     (unsigned int*)p, words);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// scratch of the no-allocation entry point (aapdhg_iterate_noalloc)
// ---------------------------------------------------------------------------
//
// One array per device, alive until the process ends.  Host code never uses
// the array's name as an address: static_scratch() looks the device address
// up once per device (with that device current) and hands it out.
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

hipError_t static_scratch(void** out) {
  static std::mutex mu;
  static void* addr[MAX_DEVICES] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *out = addr[dev];
  return hipSuccess;
}

hipError_t launch_loop(const LaunchTables& t, hipStream_t st, long long passes, unsigned int tag0) {
  LoopArgs la{};
  la.lps = t.lps;
  la.llp = t.looplps;
  la.wgs = t.wgs;
  la.blocksA = t.blocksA;
  la.blocksB = t.blocksB;
  la.chunks = t.chunks;
  la.splits = t.splits;
  la.rec = t.rec;
  la.splitpart = t.splitpart;
  la.splitcnt = t.splitcnt;
  la.sync = t.sync;
  la.bc = t.bc;
  la.pwrec = t.pwrec;
  la.err = t.err;
  la.max_passes = passes;
  la.timeout_ticks = t.timeout_ticks;
  la.tag0 = tag0;
  hipError_t e = launch_gram_refresh(t, st);
  if (e != hipSuccess) return e;
  e = launch_zero(t.sync, sizeof(LoopSync) * (size_t)t.nlps, st);
  if (e != hipSuccess) return e;
  void* args[] = {&la};
  return hipLaunchCooperativeKernel(loop_kernel_for(t.fp64, t.mt, t.ext), dim3(t.nwgs), dim3(BLOCK), args, 0, st);
}

hipError_t launch_start_point(const LPDesc& d, bool fp64, hipStream_t st) {
  const int grid = (d.N + BLOCK - 1) / BLOCK < 4096 ? (d.N + BLOCK - 1) / BLOCK : 4096;
  if (fp64)
    hipLaunchKernelGGL(k_start_point<double>, dim3(grid > 0 ? grid : 1), dim3(BLOCK), 0, st, d);
  else
    hipLaunchKernelGGL(k_start_point<float>, dim3(grid > 0 ? grid : 1), dim3(BLOCK), 0, st, d);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// scaling of K before the solve (Ruiz sweeps, Pock-Chambolle step), float64
// CSR values in place; d_row and d_col collect the factors
// ---------------------------------------------------------------------------

// Row i: r_i = sqrt(max_j |K_ij|) and the column maxima by 64-bit atomic max
// of the absolute values' bit patterns (non-negative doubles order like their
// bits, so the maxima are exact whatever the order).
__global__ void k_ruiz_max(const int* rowptr, const int* colidx, const double* val, int m, double* rfac,
                           unsigned long long* cmax) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
    double rm = 0.0;
    for (int q = rowptr[i]; q < rowptr[i + 1]; ++q) {
      const double a = fabs(val[q]);
      rm = fmax(rm, a);
      atomicMax(&cmax[colidx[q]], (unsigned long long)__double_as_longlong(a));
    }
    rfac[i] = sqrt(rm > 0.0 ? rm : 1.0);
  }
}

__global__ void k_max_to_fac(const unsigned long long* cmax, int n, double* cfac) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    const double c = __longlong_as_double((long long)cmax[j]);
    cfac[j] = sqrt(c > 0.0 ? c : 1.0);
  }
}

// Pock-Chambolle with alpha = 1: the factor of row i (of column j) is the
// square root of its absolute sum, one wave per row (per column, through the
// CSC order cperm), lanes strided then the fixed butterfly.
__global__ void k_pc_rows(const int* rowptr, const double* val, int m, double* rfac) {
  const int lane = threadIdx.x & 63;
  const int w = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, nw = (gridDim.x * blockDim.x) >> 6;
  for (int i = w; i < m; i += nw) {
    double s = 0.0;
    for (int q = rowptr[i] + lane; q < rowptr[i + 1]; q += 64) s += fabs(val[q]);
    s = wave_sum(s);
    if (lane == 0) rfac[i] = sqrt(s > 0.0 ? s : 1.0);
  }
}

__global__ void k_pc_cols(const int* cptr, const int* cperm, const double* val, int n, double* cfac) {
  const int lane = threadIdx.x & 63;
  const int w = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, nw = (gridDim.x * blockDim.x) >> 6;
  for (int j = w; j < n; j += nw) {
    double s = 0.0;
    for (int q = cptr[j] + lane; q < cptr[j + 1]; q += 64) s += fabs(val[cperm[q]]);
    s = wave_sum(s);
    if (lane == 0) cfac[j] = sqrt(s > 0.0 ? s : 1.0);
  }
}

// K_ij / (r_i s_j) and d_row /= r (thread per row), d_col /= s.
__global__ void k_apply_scale(const int* rowptr, const int* colidx, double* val, int m, const double* rfac,
                              const double* cfac, double* drow) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
    const double r = rfac[i];
    for (int q = rowptr[i]; q < rowptr[i + 1]; ++q) val[q] = val[q] / (r * cfac[colidx[q]]);
    drow[i] = drow[i] / r;
  }
}

__global__ void k_div_by(double* d, const double* f, int len) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < len; e += gridDim.x * blockDim.x) d[e] = d[e] / f[e];
}

// Results in the caller's variables, float64: x = d_col x_s, y = d_row y_s,
// lambda = lambda_s / d_col (scale = d_col then d_row); any output may be null.
template <typename T>
__global__ void k_unscale(const T* u, const T* lam, const double* scale, int n, int m, double* x, double* y,
                          double* lo) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n + m; e += gridDim.x * blockDim.x) {
    if (e < n) {
      if (x) x[e] = (double)u[e] * scale[e];
      if (lo) lo[e] = (double)lam[e] / scale[e];
    } else if (y) {
      y[e - n] = (double)u[e] * scale[e];
    }
  }
}

hipError_t launch_unscale(const void* u, const void* lam, const double* scale, bool fp64, int n, int m, double* x,
                          double* y, double* lo, hipStream_t st) {
  const int grid = std::min(4096, (n + m + BLOCK - 1) / BLOCK);
  if (fp64)
    hipLaunchKernelGGL(k_unscale<double>, dim3(grid), dim3(BLOCK), 0, st, (const double*)u, (const double*)lam,
                       scale, n, m, x, y, lo);
  else
    hipLaunchKernelGGL(k_unscale<float>, dim3(grid), dim3(BLOCK), 0, st, (const float*)u, (const float*)lam,
                       scale, n, m, x, y, lo);
  return hipGetLastError();
}

hipError_t launch_scaling(const ScalingArgs& s, hipStream_t st) {
  const int gr = std::min(4096, (s.m + BLOCK - 1) / BLOCK);
  const int gc = std::min(4096, (s.n + BLOCK - 1) / BLOCK);
  for (int it = 0; it < s.ruiz_iters; ++it) {
    hipError_t e = hipMemsetAsync(s.cmax, 0, (size_t)s.n * 8, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ruiz_max, dim3(gr), dim3(BLOCK), 0, st, s.rowptr, s.colidx, (const double*)s.val, s.m,
                       s.rfac, s.cmax);
    hipLaunchKernelGGL(k_max_to_fac, dim3(gc), dim3(BLOCK), 0, st, (const unsigned long long*)s.cmax, s.n, s.cfac);
    hipLaunchKernelGGL(k_apply_scale, dim3(gr), dim3(BLOCK), 0, st, s.rowptr, s.colidx, s.val, s.m,
                       (const double*)s.rfac, (const double*)s.cfac, s.drow);
    hipLaunchKernelGGL(k_div_by, dim3(gc), dim3(BLOCK), 0, st, s.dcol, (const double*)s.cfac, s.n);
  }
  if (s.pock_chambolle) {
    const int wr = std::min(4096, (s.m + 3) / 4), wc = std::min(4096, (s.n + 3) / 4);  // 4 waves per block
    hipLaunchKernelGGL(k_pc_rows, dim3(wr), dim3(BLOCK), 0, st, s.rowptr, (const double*)s.val, s.m, s.rfac);
    hipLaunchKernelGGL(k_pc_cols, dim3(wc), dim3(BLOCK), 0, st, s.cptr, s.cperm, (const double*)s.val, s.n, s.cfac);
    hipLaunchKernelGGL(k_apply_scale, dim3(gr), dim3(BLOCK), 0, st, s.rowptr, s.colidx, s.val, s.m,
                       (const double*)s.rfac, (const double*)s.cfac, s.drow);
    hipLaunchKernelGGL(k_div_by, dim3(gc), dim3(BLOCK), 0, st, s.dcol, (const double*)s.cfac, s.n);
  }
  return hipGetLastError();
}

hipError_t launch_power_iteration(const LPDesc& d, bool fp64, int iters, unsigned long long seed, double* work,
                                  double* est, hipStream_t st) {
  // work: v[n], z[n], w[m], part[1024]
  const int n = d.n, m = d.m;
  double* v = work;
  double* z = work + n;
  double* w = work + 2 * (size_t)n;
  double* part = work + 2 * (size_t)n + m;
  const int nparts = 1024;
  const int gridv = 1024;
  const int gridr = 2048;
  hipLaunchKernelGGL(k_fill_start, dim3(gridv), dim3(BLOCK), 0, st, v, n, seed);
  hipLaunchKernelGGL(k_sqnorm_part, dim3(nparts), dim3(BLOCK), 0, st, (const double*)v, n, part);
  hipLaunchKernelGGL(k_normalize, dim3(gridv), dim3(BLOCK), 0, st, (const double*)v, v, n, (const double*)part, nparts, est, 0);
  for (int it = 0; it < iters; ++it) {
    if (fp64) {
      hipLaunchKernelGGL(k_spmv_wave<double>, dim3(gridr), dim3(BLOCK), 0, st, d.rowptr, d.colidx, (const double*)d.val, d.rmapB, (const double*)v, w, m);
      hipLaunchKernelGGL(k_spmv_wave<double>, dim3(gridr), dim3(BLOCK), 0, st, d.colptr, d.rowidx, (const double*)d.valT, d.rmapA, (const double*)w, z, n);
    } else {
      hipLaunchKernelGGL(k_spmv_wave<float>, dim3(gridr), dim3(BLOCK), 0, st, d.rowptr, d.colidx, (const float*)d.val, d.rmapB, (const double*)v, w, m);
      hipLaunchKernelGGL(k_spmv_wave<float>, dim3(gridr), dim3(BLOCK), 0, st, d.colptr, d.rowidx, (const float*)d.valT, d.rmapA, (const double*)w, z, n);
    }
    hipLaunchKernelGGL(k_sqnorm_part, dim3(nparts), dim3(BLOCK), 0, st, (const double*)z, n, part);
    hipLaunchKernelGGL(k_normalize, dim3(gridv), dim3(BLOCK), 0, st, (const double*)z, v, n, (const double*)part, nparts, est, 1 + it);
  }
  return hipGetLastError();
}

hipError_t launch_gather_status(const LPDesc* lps, int count, int* out, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_status, dim3((count + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, st, lps, count, out);
  return hipGetLastError();
}

hipError_t launch_time_limit(const LPDesc* lps, int count, hipStream_t st) {
  hipLaunchKernelGGL(k_time_limit, dim3((count + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, st, lps, count);
  return hipGetLastError();
}

hipError_t launch_to_f64(const void* src, bool fp64, double* dst, size_t len, hipStream_t st) {
  if (len == 0) return hipSuccess;
  const size_t g = (len + BLOCK - 1) / BLOCK;
  const int grid = g < 4096 ? (int)g : 4096;
  if (fp64)
    hipLaunchKernelGGL((k_convert<double, double>), dim3(grid), dim3(BLOCK), 0, st, (const double*)src, dst, len);
  else
    hipLaunchKernelGGL((k_convert<float, double>), dim3(grid), dim3(BLOCK), 0, st, (const float*)src, dst, len);
  return hipGetLastError();
}

hipError_t launch_from_f64(const double* src, void* dst, bool fp64, size_t len, hipStream_t st) {
  if (len == 0) return hipSuccess;
  const size_t g = (len + BLOCK - 1) / BLOCK;
  const int grid = g < 4096 ? (int)g : 4096;
  if (fp64)
    hipLaunchKernelGGL((k_convert<double, double>), dim3(grid), dim3(BLOCK), 0, st, src, (double*)dst, len);
  else
    hipLaunchKernelGGL((k_convert<double, float>), dim3(grid), dim3(BLOCK), 0, st, src, (float*)dst, len);
  return hipGetLastError();
}

}  // namespace aapdhg
