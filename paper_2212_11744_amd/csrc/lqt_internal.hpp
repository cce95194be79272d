// Internal interfaces between the host API (validation, workspace planning, dispatch) and the
// kernel translation units.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/lqt.h"

#include <cstddef>
#include <cstdint>

namespace lqt {

constexpr int kMaxLevels = 40;
constexpr int kThreads = 64;  // one wavefront per workgroup: spreads small grids over all CUs

// Problem arrays of one call, type-erased (element type given by the dtype of the call).
struct KProb {
  int nx, nu, T, n, batch;
  int F_sampled, L_sampled, has_c;
  const void *t, *F, *L, *c, *Q, *R, *r, *Qf, *rf, *x0;
  const void* consts;  // per-problem prepared constants (see consts_count)
  // Ragged mode (batched solve of problems with uneven horizons): seg != nullptr.  The nseg
  // problems are concatenated into one horizon of T blocks (batch = 1): problem i owns blocks
  // seg[i] .. seg[i+1] - 2 and block seg[i+1] - 1 is a separator element (A = 0, b = x0 of
  // problem i + 1, C = 0, eta = Qf_i rf_i, J = Qf_i).  t has T rows (row g = left end of block g),
  // samples of problem i start at sample 2n (seg[i] - i) + i, constant F, L and Q, R, Qf, rf, x0
  // are per problem, and outputs have T rows (row g = boundary g; no row for the end of the last
  // separator).
  const int64_t* seg = nullptr;
  int nseg = 0;
  // Time-invariant path (lqt_dims.lti): per-problem shared element parts and response tables.
  int lti = 0;
};

// Per-problem table of the time-invariant path (values of the call dtype): A - I [nx*nx],
// C and J packed upper [ns each], then V[j] and W[j] for the 2n+1 samples j of a block
// ([nx][nx] each, row-major): b = sum_j V[j] r_j, eta = sum_j W[j] r_j.
__host__ __device__ inline long lti_off_V(int nx) { return (long)nx * nx + nx * (nx + 1); }
__host__ __device__ inline long lti_off_W(int nx, int n) {
  return lti_off_V(nx) + (2L * n + 1) * nx * nx;
}
__host__ __device__ inline long lti_count(int nx, int n) {
  return lti_off_V(nx) + 2 * (2L * n + 1) * nx * nx;
}

// Index of the problem owning block (or boundary) g in ragged mode: the largest i with
// seg[i] <= g, clamped to [0, nseg - 1].
__device__ inline int seg_find(const int64_t* seg, int nseg, long g) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (seg[mid] <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Per-problem constants prepared once per call by the prep kernel (values of the call dtype):
//   G = L R^{-1} L^T [nx*nx], Lc = L W [nx*nu] with W = chol(R)^{-T} (so G = Lc Lc^T),
//   Kc = R^{-1} L^T [nu*nx], W [nu*nu], Rinv [nu*nu].  G, Lc, Kc only when L is constant.
__host__ __device__ inline int consts_off_G(int, int) { return 0; }
__host__ __device__ inline int consts_off_Lc(int nx, int) { return nx * nx; }
__host__ __device__ inline int consts_off_Kc(int nx, int nu) { return nx * nx + nx * nu; }
__host__ __device__ inline int consts_off_W(int nx, int nu) { return nx * nx + 2 * nx * nu; }
__host__ __device__ inline int consts_off_Rinv(int nx, int nu) { return nx * nx + 2 * nx * nu + nu * nu; }
__host__ __device__ inline int consts_count(int nx, int nu) { return nx * nx + 2 * nx * nu + 2 * nu * nu; }

// Tree shape of the scans: n[0] = T blocks; level 1 has ceil(T / 4) nodes (4 blocks per lane);
// level l + 1 has ceil(n[l] / 256) nodes (4 nodes per lane, 64 lanes per wave) while n[l] > 256;
// level `levels` (<= 256 nodes) is swept by one wavefront.
// Blocks per tile of the element layout (include/lqt.h) and of every tiled record array.
constexpr int kEltTile = 512;
constexpr int kLaneChunk = 4;
constexpr int kWaveSpan = 256;
constexpr int kLbGroupTiles = 64;  // tiles per group record of the single-pass scans
// Blocks per lane of the single-pass scans (a tile is one wave: 64 lanes), chosen from the
// horizon.  A longer chunk costs serial steps per lane; more tiles cost look-back depth (about
// log2 of the tiles in flight, in Lemma 7 combinations) and, beyond the ~1024 waves resident at
// once, another round of tiles.  Measured on the FP64 point mass (value scan, 512-block element
// tiles): 1 block per lane is best up to 2^11 blocks, 2 up to 2^14, 4 up to 2^17 (2^16: 78 us vs
// 84 with 2 and 87 with 8), 8 from 2^18 on (2^18: 110 us vs 122 with 4; 2^20: 315 us vs 407;
// 16 per lane, one round of resident tiles at 2^20, is slower again: 402 us).
// The trajectory scan keeps its lanes' block maps in registers and stops at 4.  The records are
// laid out for one block per lane, so they hold any chunk's tiles.
constexpr int kScanMaxVChunk = 8, kScanMaxTChunk = 4;
inline int scan_chunk(long T, int cmax) {
  const int c = T <= (1L << 11) ? 1 : T <= (1L << 14) ? 2 : T <= (1L << 17) ? 4 : 8;
  return c < cmax ? c : cmax;
}
// Trajectory scan (measured on the same workload): 1 block per lane up to 2^14 blocks (2^14:
// 25.7 us vs 28.8 with 4), 2 at 2^15 (28.5 vs 29.7), 4 (its maximum) from 2^16 on (2^16: 32.9 vs
// 35.3 with 2; 2^20: 193 vs 266).
inline int traj_chunk(long T) {
  return T <= (1L << 14) ? 1 : T <= (1L << 15) ? 2 : kScanMaxTChunk;
}

struct Tree {
  int levels = 0;
  long n[kMaxLevels + 1] = {};
};

Tree plan_tree(long T);

// Records of one single-pass scan with decoupled look-back (lookback.hpp), for `batch` problems
// of G tiles and NG = ceil(G / 64) groups each.  ctr, tflag and gflag are consecutive words (one
// clear covers them); payloads hold value q of record r at [q * G + r] (tiles) or [q * NG + r]
// (groups) per problem.
struct LbRecs {
  unsigned* ctr = nullptr;    // [batch] tile counters
  unsigned* tflag = nullptr;  // [batch][G] status words of the tiles
  unsigned* gflag = nullptr;  // [batch][NG] status words of the groups
  void* tagg = nullptr;       // [batch][NMAP][G] tile aggregates
  void* tst = nullptr;        // [batch][NST][G] inclusive states of the tiles
  void* gagg = nullptr;       // [batch][NMAP][NG] group aggregates
  void* gst = nullptr;        // [batch][NST][NG] inclusive states of the groups
  long G = 0, NG = 0;
  long nwords = 0;            // ctr .. end of gflag
};

// Workspace pointers of one call (all per-level arrays hold `batch` problems back to back, each in
// tiles of 512 items).
struct Work {
  void* consts = nullptr;
  LbRecs lbv, lbt;                   // single-pass value and trajectory scans (per-lane path)
  void* vtup[kMaxLevels + 1] = {};   // value tree: tuples at level l >= 1
  void* vval[kMaxLevels + 1] = {};   // value tree: (packed S, v) at right ends of level-l nodes
  void* vpart[kMaxLevels + 1] = {};  // value tree: lane partials of the wave trees above level l
  void* tmap[kMaxLevels + 1] = {};   // trajectory tree: affine maps at level l
  void* tx[kMaxLevels + 1] = {};     // trajectory tree: x at left ends of level-l nodes
  void* tpart[kMaxLevels + 1] = {};  // trajectory tree: lane partials above level l
  void* elts = nullptr;              // elements when the caller gives none (lqt_solve)
  void* gsamp = nullptr;             // adjoint with sampled L: G(t) at every sample
  unsigned* wq_done = nullptr;       // wave path: status words and counter of the queue solve
  long wq_words = 0;
  void* bmap = nullptr;              // wave path, solve: every block's map ([batch][T][nx^2 + nx])
  // canary mode (lqt_debug_canary): a 256-byte slot after every region, filled by check_ws and
  // checked at the end of the call; canary_res: the index of the first changed slot
  static constexpr int kMaxCanaries = 160;
  unsigned* canary[kMaxCanaries] = {};
  int ncanary = 0;
  int* canary_res = nullptr;
  bool canary_armed = false;
  // adjoint
  void* lmap[kMaxLevels + 1] = {};   // lambda scan: maps, states, lane partials per level
  void* lst[kMaxLevels + 1] = {};
  void* lpart[kMaxLevels + 1] = {};
  void* cmap[kMaxLevels + 1] = {};   // (Sbar, vbar) scan
  void* cst[kMaxLevels + 1] = {};
  void* cpart[kMaxLevels + 1] = {};
  void* lam = nullptr;               // lambda_k, [batch][T+1][nx]
  void* bnd = nullptr;               // adjoints of block-boundary samples, [batch][T][2][nx]
  void* wsum = nullptr;              // per-wave sums of the Q and G adjoints
  void* ckpt = nullptr;              // RK4 step start values of every block (nullptr: recompute)
  void* lti = nullptr;               // time-invariant path tables, [batch][lti_count]
  int* flag = nullptr;               // finite check: set to 1 when an output is NaN or Inf
};

// Largest n_steps for which the adjoint keeps the RK4 step start values of every block in the
// workspace (above it they are recomputed from the block's start).
constexpr int kCkptMaxSteps = 16;

// Kernel launchers of one (nx, nu, dtype) instantiation.  Each returns hipGetLastError().
struct Ops {
  hipError_t (*prep)(const KProb&, void* consts, hipStream_t);
  hipError_t (*build)(const KProb&, void* elts, hipStream_t);
  // single-pass scans: values S, v of every boundary; trajectory x, u (u nullable)
  // (chunk: blocks per lane, 1, 2, 4 or 8 (value) / 4 (trajectory); see scan_chunk)
  hipError_t (*vscan)(const KProb&, const void* elts, void* S, void* v, const LbRecs&, int chunk,
                      hipStream_t);
  hipError_t (*tscan)(const KProb&, const void* elts, const void* S, const void* v, void* x,
                      void* u, const LbRecs&, int chunk, hipStream_t);
  // level 1 of the node products (4 blocks per lane), for the Method 2 tree
  hipError_t (*vreduce0)(const KProb&, const void* elts, void* lvl1, long n1, hipStream_t);
  // time-invariant path: response tables, then the elements from them
  hipError_t (*lti_prep)(const KProb&, void* tab, hipStream_t);
  hipError_t (*lti_build)(const KProb&, const void* tab, void* elts, hipStream_t);
  // elements from the forward conditional ODEs (Theorem 9)
  hipError_t (*build_fwd)(const KProb&, void* elts, hipStream_t);
  // Method 2 trajectory: forward prefix scan of (C, z) over the node products
  hipError_t (*m2_up)(const KProb&, const void* src, long n_src, void* part, void* dst, long n_dst,
                      hipStream_t);
  hipError_t (*m2_top)(const KProb&, const void* tup, long n, void* st, hipStream_t);
  hipError_t (*m2_down)(const KProb&, const void* tup, long n_child, const void* part,
                        const void* st_par, long n_par, void* st_child, hipStream_t);
  hipError_t (*m2_bottom)(const KProb&, const void* elts, const void* S, const void* v,
                          const void* st1, long n1, void* x, void* u, hipStream_t);
  // (Method 2's tree levels use the value-tree arrays vtup, vpart, vval of Work)
  // values inside the blocks at the n T + 1 RK4 nodes
  hipError_t (*dense)(const KProb&, const void* S, const void* v, const void* x, void* Sd,
                      void* vd, void* xd, void* ud, hipStream_t);
  // elements with every block split: Theorem 9 on the first half, Theorem 8 on the second
  hipError_t (*build_split)(const KProb&, void* elts, hipStream_t);
  // elements (constant coefficients) plus the RK4 step start values the adjoint re-linearises at
  hipError_t (*build_ckpt)(const KProb&, void* elts, void* ckpt, hipStream_t);
  // value and trajectory scans in one launch over a work queue (records lbv, lbt cleared; value chunk
  // cv = 1, 4 or 8 blocks per lane, trajectory chunk queue_tchunk(cv))
  // the constants prep and, in the same launch, the zeroing of both single-pass scans' status
  // words (the full solve: one launch less)
  hipError_t (*prep_clear)(const KProb&, void* consts, const LbRecs& a, const LbRecs& b,
                           hipStream_t);
  hipError_t (*scan_queue)(const KProb&, const void* elts, void* S, void* v, void* x, void* u,
                             const LbRecs& lbv, const LbRecs& lbt, int cv, hipStream_t);
};

// Adjoint kernels (lqt_adjoint.hip) of one (nx, nu, dtype) instantiation.
struct AdjOps {
  hipError_t (*lam_bottom)(const KProb&, const void* elts, const void* S, const void* v,
                           const void* xbar, void* maps1, long n1, hipStream_t);
  hipError_t (*lam_up)(const KProb&, const void* src, long n_src, void* part, void* dst,
                       long n_dst, hipStream_t);
  hipError_t (*lam_top)(const KProb&, const void* xbar, const void* src, long n, void* out,
                        hipStream_t);
  hipError_t (*lam_down)(const KProb&, const void* src, long n_child, const void* part,
                         const void* st_par, long n_par, void* st_child, hipStream_t);
  hipError_t (*cong_bottom)(const KProb&, const void* elts, const void* S, const void* v,
                            const void* x, const void* xbar, const void* lam1, long n1, void* lam,
                            void* maps1, void* dx0, hipStream_t);
  hipError_t (*cong_up)(const KProb&, const void* src, long n_src, void* part, void* dst,
                        long n_dst, hipStream_t);
  hipError_t (*cong_top)(const KProb&, const void* src, long n, void* out, hipStream_t);
  hipError_t (*cong_down)(const KProb&, const void* src, long n_child, const void* part,
                          const void* st_par, long n_par, void* st_child, hipStream_t);
  hipError_t (*elem)(const KProb&, void* elts, const void* S, const void* v, const void* x,
                     const void* lam, const void* sv1, long n1, void* dQf, void* drf,
                     hipStream_t);
  // ckpt_ready: the step start values are already in ckpt (written by Ops::build_ckpt)
  hipError_t (*rk4)(const KProb&, const void* abar, void* dr, void* bnd, void* wsum, void* ckpt,
                    bool ckpt_ready, void* gsamp, hipStream_t);
  hipError_t (*finish)(const KProb&, const void* bnd, void* dr, const void* wsum, void* dQ,
                       void* dR, hipStream_t);
};

// FP64 adjoint instantiations for 1 <= nu <= nx <= 4; nullptr otherwise.
const AdjOps* adj_ops(int nx, int nu, int dtype);

// Build shards.  The per-lane and wave sources hold many template instantiations, so each is
// compiled several times (with -DLQT_SHARD=i, i < the shard count below) and every object keeps
// only the instantiations of its shard; the shard functions return nullptr for the sizes they do
// not hold, and the dispatchers (lane_ops, wave_*) ask every shard.
constexpr int kLaneShards = 4;
constexpr int kWaveShards = 8;
// Shard of a per-lane instantiation: (nx, nu) numbered 0..9 in (nx, nu) order, FP32 after FP64.
__host__ __device__ constexpr int lane_shard(int nx, int nu, bool f32) {
  return ((nx * (nx - 1)) / 2 + nu - 1 + (f32 ? 10 : 0)) % kLaneShards;
}
__host__ __device__ constexpr int wave_shard(int nx, bool f32) {
  return (2 * (nx - 5) + (f32 ? 1 : 0)) % kWaveShards;
}
template <int S>
const Ops* lane_ops_shard(int nx, int nu, int dtype);

// Instantiations for 1 <= nu <= nx <= 4 (one tuple per lane); nullptr if not available.
const Ops* lane_ops(int nx, int nu, int dtype);

// Wavefront-per-tuple path (lqt_wave.hip) for any nx <= 16: one wavefront per block or tree
// node, matrices in LDS.  Its trees reduce wcs[l] nodes per wave at level l: n[0] = T,
// n[l + 1] = ceil(n[l] / wcs[l]) while n[l] > wcs[l] (wcs[0] = wc, above kWaveUpperChunk).  Tree nodes are records ([batch][n[l]][record]):
// tuples (NE values, element order), values (S full, v: nx^2 + nx), maps (P = Psi - I, q:
// nx^2 + nx), states (nx).
struct WTree {
  int levels = 0;
  int wc = 8;                     // blocks per wave at the bottom (= wcs[0])
  int wcs[kMaxLevels + 1] = {};   // wcs[l]: nodes of level l per node of level l + 1
  long n[kMaxLevels + 1] = {};
};
// Upper levels branch by kWaveUpperChunk whatever the bottom chunk: their node counts are small,
// so the serial chain of a wave (wcs[l] combinations or folds) is what they cost.
constexpr int kWaveUpperChunk = 4;
WTree wave_tree(long T, int wc);
// The wave path's solve after the element build in one launch over a work queue: the stages of
// the two trees (4 levels + 1 of them) and where their items start; done: one status word per
// item, then the item counter (total + 1 words, zero before the launch).
constexpr int kWqMaxLevels = 16;
struct WQueue {
  int levels = 0, nst = 0;
  int wcs[kWqMaxLevels + 1] = {};  // branching of every level (WTree::wcs)
  long total = 0;
  long n[kWqMaxLevels + 1] = {};      // nodes per problem at level l (n[0] = T)
  long start[4 * kWqMaxLevels + 1] = {};
  int kind[4 * kWqMaxLevels + 1] = {};
  int level[4 * kWqMaxLevels + 1] = {};
  unsigned* done = nullptr;
  void* bmap = nullptr;  // per-block maps (Work::bmap)
  void* vtup[kWqMaxLevels + 1] = {};
  void* vval[kWqMaxLevels + 1] = {};
  void* tmap[kWqMaxLevels + 1] = {};
  void* tx[kWqMaxLevels + 1] = {};
};
// The queue of a tree (pointers from w; false if the tree is deeper than kWqMaxLevels).
bool wave_queue(const WTree& t, long batch, const Work& w, WQueue* q);
// Launchers of one wave-path instantiation (state size, dtype).
struct WaveFns {
  hipError_t (*build)(const KProb&, void* elts, hipStream_t);
  hipError_t (*value)(const KProb&, const WTree&, const Work&, const void* elts, void* S, void* v,
                      void* maps1, hipStream_t);
  hipError_t (*traj)(const KProb&, const WTree&, const Work&, const void* elts, const void* S,
                     const void* v, void* x, void* u, bool maps_ready, hipStream_t);
  // both trees in one launch (q.done cleared)
  hipError_t (*solve_queue)(const KProb&, const WQueue& q, const void* elts, void* S, void* v,
                            void* x, void* u, hipStream_t);
  hipError_t (*build_fwd)(const KProb&, void* elts, hipStream_t);    // Theorem 9
  hipError_t (*build_split)(const KProb&, void* elts, hipStream_t);  // split blocks
  // Method 2 trajectory (node products in w.vtup, prefix records in w.vpart)
  hipError_t (*method2)(const KProb&, const WTree&, const Work&, const void* elts, const void* S,
                        const void* v, void* x, void* u, hipStream_t);
  hipError_t (*dense)(const KProb&, const void* S, const void* v, const void* x, void* Sd,
                      void* vd, void* xd, void* ud, hipStream_t);  // values inside the blocks
  // time-invariant path: the table of a problem (lti_count values), then the elements
  hipError_t (*lti_prep)(const KProb&, void* tab, hipStream_t);
  hipError_t (*lti_build)(const KProb&, const void* tab, void* elts, hipStream_t);
};
template <int S>
const WaveFns* wave_fns_shard(int nx, int dtype);
hipError_t wave_build(const KProb& kp, int dtype, void* elts, hipStream_t s);
hipError_t wave_build_fwd(const KProb& kp, int dtype, void* elts, hipStream_t s);
hipError_t wave_build_split(const KProb& kp, int dtype, void* elts, hipStream_t s);
hipError_t wave_method2(const KProb& kp, int dtype, const WTree& t, const Work& w,
                        const void* elts, const void* S, const void* v, void* x, void* u,
                        hipStream_t s);
hipError_t wave_lti(const KProb& kp, int dtype, void* tab, void* elts, hipStream_t s);
hipError_t wave_dense(const KProb& kp, int dtype, const void* S, const void* v, const void* x,
                      void* Sd, void* vd, void* xd, void* ud, hipStream_t s);
hipError_t wave_value(const KProb& kp, int dtype, const WTree& t, const Work& w, const void* elts,
                      void* S, void* v, void* maps1, hipStream_t s);
hipError_t wave_traj(const KProb& kp, int dtype, const WTree& t, const Work& w, const void* elts,
                     const void* S, const void* v, void* x, void* u, bool maps_ready,
                     hipStream_t s);
hipError_t wave_solve_queue(const KProb& kp, int dtype, const WQueue& q, const void* elts, void* S,
                            void* v, void* x, void* u, hipStream_t s);

// Options of a full solve: the number of nodes per wave of the wave path's trees.
struct SolveOpts {
  int wave_chunk = 8;
  // Per-lane path: 0 runs the value and trajectory scans as two launches (chunks from
  // scan_chunk); 1, 4 or 8 runs both in one work-queue launch with that value chunk.
  // Wave path: nonzero runs both trees in one work-queue launch (wave_queue).
  int queue_chunk = 0;
};

// Zeroes the counter and status words of a single-pass scan (before every launch; the full solve
// clears both of its scans' words in its constants launch, Ops::prep_clear).
hipError_t lb_clear(const LbRecs& r, hipStream_t s);

// Trajectory chunk of the work-queue scans for value chunk cv.
inline int queue_tchunk(int cv) { return cv < 4 ? cv : 4; }

// Workspace layout of one call (lqt_api.hip); the layout for wave_chunk wc also serves any larger
// chunk.  nconsts: problems whose per-problem constants are prepared.
// ws_elts: a solve keeps its elements in the workspace (false when the caller provides them).
// keep_maps: on the wave path, room for every block's closed-loop map (Work::bmap).
size_t layout(const lqt_dims* d, lqt_call call, char* base, Work* w, int wc, long nconsts,
              bool ws_elts = true, bool keep_maps = true);

// Prep, element build, value scan and trajectory scan for validated arguments.
lqt_status run_solve(const lqt_dims* d, const KProb& kp, const Work& w, void* elts, void* S,
                     void* v, void* x, void* u, const SolveOpts& o, hipStream_t stream);

// Record / clear the calling thread's last error (lqt_last_error).
// Simulated failures (lqt_debug_fail_launch): every checked HIP call's status passes through
// debug_gate; debug_gate_note() names a failure the gate produced (and forgets it).
hipError_t debug_gate(hipError_t e);
const char* debug_gate_note();
lqt_status set_error(lqt_status st, const char* msg);
lqt_status clear_error();

// Prep kernel (any nx, nu <= 16).
hipError_t launch_prep(const KProb& kp, int dtype, void* consts, hipStream_t stream);

}  // namespace lqt
