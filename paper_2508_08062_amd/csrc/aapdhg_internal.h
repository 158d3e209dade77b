// Device-side data layout shared by the HIP kernels and the host runtime of
// the AA-PDHG library.  Nothing here is part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace aapdhg {

constexpr int MAXM = 16;          // largest Anderson memory
constexpr int BLOCK = 256;        // threads per workgroup (4 wave64)
constexpr int CHUNK_NNZ = 2048;   // nnz staged in LDS by one multi-row chunk
constexpr int CHUNK_ROWS = 256;   // rows of one multi-row chunk (one per thread at most)
constexpr int ROWS_PER_THREAD = CHUNK_ROWS / BLOCK;
constexpr int SPLIT_NNZ = 8192;   // nnz per part of a split (very long) row
constexpr int DECIDE_RECORDS = 256;  // records added by one workgroup of the decision launch
constexpr int MIX_TILE = 2048;    // elements per block of the mix pass
constexpr int NDOT = 2 * MAXM + 16;  // stride of one partial-sum record (doubles)
// Column panels of the dual product: 4 in float32 (each x_bar slice, 2 MB on
// the 1M x 2M LP, taken by two XCDs), 8 in float64 (one slice per XCD, so that
// a slice still fits an XCD's L2).
constexpr int MAX_PANELS = 8;
__host__ __device__ constexpr int panel_count(bool fp64) { return fp64 ? 8 : 4; }
constexpr int PANEL_ROWS = 1024;  // rows of one panel chunk (four per thread)

// Partial-sum record: MT = memory bound of the kernel instantiation.
//   [0, MT)  <dg_new, dG[live t]>, the new row of the Gram matrix
//   MT+0 <dg,dg>  MT+1 <dg,g>  MT+2 <g,g>  MT+3 <du,du>
//   MT+4..MT+6  KKT sums of the primal pass: c.x, l.lam+ - u.lam-, ||c-K^T y-lam||^2
//   MT+7..MT+8  KKT sums of the dual pass: q.y, ||primal residual||^2
// Both passes fill disjoint KKT slots, so the records of a loop pass are
// simply added.  The right-hand sides <dG[t], g^k> need no sums of their own:
// g^k = g^{k-1} + dg_new, so <dG[t], g^k> = <dG[t], g^{k-1}> + <dG[t], dg_new>.
template <int MT>
struct Dot {
  static constexpr int G = 0, DGDG = MT, DGG = MT + 1, GG = MT + 2, DU2 = MT + 3, KA0 = MT + 4,
                       KA1 = MT + 5, KA2 = MT + 6, KB0 = MT + 7, KB1 = MT + 8, COUNT = MT + 9;
};

enum Status : int { ST_CONVERGED = 0, ST_ITER_LIMIT = 1, ST_TIME_LIMIT = 2, ST_NUMERICAL = 3, ST_RUNNING = 4 };
// BR_GRAM: the safeguard test of the pass passed with a non-empty memory on
// the three-launch path; the Gram launch forms the history's Gram matrix and
// finishes the pass (the branch is then BR_AA or BR_PDHG).
enum Branch : int { BR_NONE = 0, BR_PDHG = 1, BR_AA = 2, BR_GRAM = 3 };
enum Variant : int { V_PDHG = 0, V_AA = 1, V_FAA = 2, V_RPDHG = 3 };
enum Mode : int { MODE_ITER = 0, MODE_EVAL = 1 };

// Per-LP iteration state, written only by the single block that finishes a
// loop pass (or by host set-up while the device is idle).
struct alignas(256) Scalars {
  long long k;       // index of the current iterate u^k (0 before the init step)
  long long i_aa;    // Anderson steps taken
  long long j_pdhg;  // PDHG steps taken
  long long kkt_k;   // iteration of the last KKT evaluation
  int status;        // Status
  int branch;        // Branch of the last loop pass
  int nlive;         // live history slots
  int newslot;       // slot that receives the next difference pair
  int live[MAXM];    // live slots, oldest first
  int nmix;          // slots used by the pending mix
  int mixslot[MAXM];
  int pad0[3];
  double n0;         // ||g^0||
  double gnorm;      // ||g^k||
  double G[MAXM * MAXM];  // Gram of the history columns, by physical slot
  double rhs[MAXM];       // <dG[slot], g^k>
  double du2[MAXM];       // ||du[slot]||^2
  double gamma[MAXM];     // mixing coefficients for mixslot[]
  double pobj, dobj, r_g, r_p, r_d, kkt;
  double qnorm, cnorm;
  double thr;             // safeguard bound for i^k = thr_i - 1 (valid when thr_i == i^k + 1)
  long long thr_i;
  // primal weight (Alg 7): tau = gstep / omega, sigma = gstep * omega
  double omega, gstep, tau, sigma;
  // D-hat in use: dha[p] * D-hat_0 + dhb[p] on the x part (p = 0) and the y part (p = 1)
  double dha[2], dhb[2];
  long long pw_updates;   // accepted weight updates
  int pw_flag;            // 1: the weight changed before this pass (memory reset pending)
  int pw_blend;           // set by the pass that re-blended D-hat: 1 alpha = 0.9, 2 alpha = 0.1
  long long faa_empty;    // FAA steps whose filters kept no column
  // 1: G and rhs hold the Gram matrix of the live slots and <dG[slot], g^{k-1}>.
  // The persistent kernel keeps them so from pass to pass; the passes of the
  // three-launch path leave them stale (0) and form them only for Anderson
  // steps (the Gram launch), or when a refresh asks for them.
  int gram_ok;
  int pad1;
};

// Per-LP immutable description (device copy).  Vectors of length N = n + m
// hold the x part first and the y part at offset n.
struct LPDesc {
  int m, n, N, M;
  int variant, kkt_every;
  long long max_iter;
  double tau, sigma, beta, D, eps_sg, eta, cs, kappa_bar, tol;
  double sg_div;  // c of the Iter_AA / c safeguard
  // primal-weight update (Alg 7): period U_P (0 = off), theta, epsilon_zero,
  // the residual-decrease threshold of the D-hat re-blend, re-blend on/off
  int pw_period, pw_dhat;
  double pw_theta, pw_eps0, pw_rho;
  void* anchor;  // u at the last weight check (length N), when pw_period > 0
  // restarted PDHG: epoch length R (0 = no restarts) and the sum of the
  // epoch's iterates so far (length N, float64)
  int restart;
  int angle_mode;  // FAA angle filter: 0 one factorisation, 1 refreshed after each removal
  int length_floor;  // FAA length filter keeps at least this many columns (0 or 1)
  // 1: the three-launch passes leave out the dots of the new difference column
  // with the stored ones; G and rhs are formed by the Gram launch when a step
  // needs them (the persistent kernel keeps them pass by pass either way)
  int lazy_gram;
  double* rsum;
  const int* rowptr;  // CSR of K, rows in the order rmapB
  const int* colidx;
  const void* val;
  const int* colptr;  // CSC of K (CSR of K^T), columns in the order rmapA
  const int* rowidx;
  const void* valT;
  const int* rmapA;   // original column at each position of the CSC
  const int* rmapB;   // original row at each position of the CSR
  const void* c;
  const void* lo;
  const void* hi;
  const void* q;
  const void* dhat;  // length N
  const unsigned char* rowtype;
  void* u[2];  // iterates, by parity of k
  void* g[2];  // residuals, by parity of k
  void* xbar;  // 2 x_hat - x (length n)
  void* dG;    // history [M][N]
  void* W;     // dU + beta D-hat dG, [M][N]
  void* lam;   // reduced costs written by the evaluation pass (length n)
  Scalars* sc;
  // Column panels of the CSR (large LPs in launches of their own): the
  // entries of row position r whose column lies in panel p are
  // [pptr[p (m+1) + r], pptr[p (m+1) + r + 1]) of pidx / pval; part holds the
  // panel row sums [2][panels][m] (x_bar, and x^k on KKT passes).
  int panels;  // 0 or panel_count(the LP's precision)
  const int* pptr;
  const int* pidx;
  const void* pval;
  double* part;
  // panel p's chunks (<= PANEL_ROWS rows, <= CHUNK_NNZ entries each): chunk
  // c < pcoff[p+1] - pcoff[p] - 1 starts at row pchunk[2 (pcoff[p] + c)] and
  // entry pchunk[2 (pcoff[p] + c) + 1]; the list of each panel ends with
  // (m, the panel's last entry + 1)
  const int* pchunk;
  int pcoff[MAX_PANELS + 1];
};

// One workgroup's share of an SpMV pass.  "Rows" are columns of K in the
// primal pass (CSC) and rows of K in the dual pass (CSR); r0, r1 and split
// rows are positions in the pass's row order (rmapA / rmapB).
struct Chunk {
  int lp;     // index into the launch's LP table
  int kind;   // 0: multi-row (rows [r0,r1), nnz [k0,k1) staged in LDS); 1: part of a split row
  int r0, r1;
  int k0, k1;
  int tpr;    // multi: threads per row (1..64, or BLOCK for a single row); split: part index
  int split;  // split: global split-row index
  int pad[4];
};

// One workgroup of the decision launch (three-launch path): positions
// [r0, r1) of its LP's record list (the LP's primal-pass records [leafA,
// leafA + nA), then its dual-pass records from leafB), summed into partial
// `slot`; the LP's partials are [blk0, blk0 + nblk).  The LP's scalars and
// record ranges are copied here so that the launch's first loads depend on
// this entry alone.
struct DecideBlock {
  Scalars* sc;
  int lp;
  int r0, r1;
  int slot;
  int leafA, nA, leafB;
  int blk0, nblk;
  int pad;
};

struct SplitRow {
  int row;      // pass-local row
  int nparts;
  int part0;    // first slot in the split partial buffer
  int leaf;     // record that receives the row's dot sums (written by the last part)
  int pad[4];
};

// One workgroup of an SpMV pass.  kind 0: the multi-row chunks [c0, c1) of
// one LP, streamed in order, whose dot sums go to record `leaf`; kind 1: the
// split-row part in chunk c0 (its row's sums go to the split row's record).
struct BlockWork {
  int lp;
  int kind;
  int c0, c1;
  int leaf;
  int pad[3];
};

// Per-LP entry of a launch table: its records (primal pass [leafA, leafA +
// nA), dual pass [leafB, leafB + nB)) and its workgroups of the decision
// launch [blk0, blk0 + nblk) (their partials have the same indices).
struct LaunchLP {
  int leafA, nA, leafB, nB;
  int blk0, nblk;
  int pad[2];
};

struct MixTile {
  Scalars* sc;  // the LP's scalars (the launches' first check reads them)
  int lp;
  int e0, e1;
  int t0, nt;  // the LP's tiles: [t0, t0 + nt)
  int pad;
};

// Everything a pass kernel needs; passed by value.
struct PassArgs {
  const LPDesc* lps;
  const LaunchLP* llp;
  const BlockWork* blocks;
  const Chunk* chunks;
  const DecideBlock* dblocks;
  const SplitRow* splits;
  double* rec;          // [nleaves][NDOT] partial-sum records
  double* dpart;        // [decision workgroups][NDOT] partial sums of the records
  unsigned int* dcnt;   // [LPs] arrivals of the decision workgroups
  double* splitpart;    // [split parts][2]
  unsigned int* splitcnt;  // [split rows]
  int nleaves;          // leaf records of both passes (workgroups and split rows)
  int mode;
};

// The Gram launch (three-launch path): one workgroup per mix tile.  Partials
// of an LP are stored value-major: value q of the LP's tile j (of nt) at
// gpart[t0 * nv + q * nt + j], with t0 the LP's first tile and nv the values
// per tile of the launch's memory bound.
struct GramArgs {
  const LPDesc* lps;
  const MixTile* tiles;
  double* gpart;
  unsigned int* gcnt;    // [LPs] arrivals
  int refresh;           // 1: only bring G and rhs up to date where gram_ok is 0
};

struct MixArgs {
  const LPDesc* lps;
  const MixTile* tiles;
  double* pwpart;        // [tiles][2]: squared distances to the anchor (weight checks)
  unsigned int* pwcnt;   // [LPs] arrivals of the weight check
};

// ---- persistent loop kernel ----

// One workgroup of the persistent loop kernel: its LP, its rank in the LP's
// group, and the units (BlockWork entries) it handles in the CSC pass
// [a0, a1) and in the CSR pass [b0, b1), for the whole launch.
struct LoopWG {
  int lp;
  int rank;
  int a0, a1;
  int b0, b1;
  int pad[2];
};

// Per-LP entry: the size of its workgroup group and its partial-sum records
// (the leaves of both passes, [leaf0, leaf0 + nleaf)).
struct LoopLP {
  int nwg;
  int leaf0;
  int nleaf;   // records of both passes
  int nleafA;  // of which the CSC pass's come first
  int wg0;     // the group's workgroups are [wg0, wg0 + nwg)
  int pad[3];
};

// Per-LP counters of one launch (zeroed before the launch).  Arrivals are
// spread over NSUB counters 128 bytes apart (workgroup rank modulo NSUB), so
// that the atomics of a group do not queue on one address; a waiter adds the
// NSUB counters.
constexpr int NSUB = 8;
constexpr int SUB_STRIDE = 32;  // unsigned ints between sub-counters
struct alignas(256) LoopSync {
  unsigned int bar[NSUB * SUB_STRIDE];  // group-barrier arrivals
  unsigned int arr[NSUB * SUB_STRIDE];  // arrivals after the CSR phase
  unsigned int abort;                   // set when a wait gave up
  unsigned int pad[63];
};

// Decisions of a pass as every workgroup of the group keeps them (LDS).
struct Bcast {
  long long k;
  int status, branch, nmix, nlive, newslot, blend;
  int mixslot[MAXM];
  int live[MAXM];
  double gamma[MAXM];
  double omega, tau, sigma;  // step sizes in use (primal weight)
  double dha[2], dhb[2];     // D-hat in use
};
// The passes read tau, sigma, dha and dhb as six consecutive doubles from
// either struct.
static_assert(offsetof(Bcast, dhb) == offsetof(Bcast, tau) + 4 * sizeof(double), "step words");
static_assert(offsetof(Scalars, dhb) == offsetof(Scalars, tau) + 4 * sizeof(double), "step words");

// The decisions as rank 0 publishes them: BC_WORDS 64-bit words, each a
// 32-bit payload (low half) and the 32-bit tag of the pass (high half), so a
// reader that sees every tag of its pass has the whole message in one read.
//   word 0: status | branch << 4 | nmix << 8 | nlive << 16 | newslot << 24
//   words 1-2: live slots, 4 bits each; words 3-4: mix slots, 4 bits each
//   words 5 .. 5 + 2 MAXM: gamma, low and high halves
//   word 5 + 2 MAXM: D-hat re-blend of the pass (0 none, 1 alpha = 0.9, 2 alpha = 0.1)
constexpr int BC_WORDS = 6 + 2 * MAXM;
// Rank 0 writes BC_COPIES copies of the message; the other ranks poll copy
// (rank % BC_COPIES), which spreads their polling over four copies.
constexpr int BC_COPIES = 4;
struct alignas(256) BcastMsg {
  unsigned long long w[64 * BC_COPIES];
};

struct LoopArgs {
  const LPDesc* lps;
  const LoopLP* llp;
  const LoopWG* wgs;
  const BlockWork* blocksA;
  const BlockWork* blocksB;
  const Chunk* chunks;
  const SplitRow* splits;
  double* rec;
  double* splitpart;
  unsigned int* splitcnt;
  double* pwrec;  // [workgroups][2]: squared distances to the anchor (weight checks)
  LoopSync* sync;
  BcastMsg* bc;
  int* err;  // set to 1 when a wait gave up
  long long max_passes;
  unsigned int tag0;  // tag of pass 0 of this launch (the pass number is added)
  unsigned long long timeout_ticks;  // bound of one wait, in wall-clock ticks
};

}  // namespace aapdhg
