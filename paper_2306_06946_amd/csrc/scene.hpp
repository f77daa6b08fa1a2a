// The scene object behind the opaque icr_scene handle, and the host-side
// launchers of every kernel family.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "common.hpp"

namespace icr {

// Device allocations owned by a scene; freed together.
struct Arena {
  std::vector<void *> ptrs;
  size_t bytes = 0;
  template <class T>
  T *alloc(size_t count) {
    if (count == 0) count = 1;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) throw HipError(e, "hipMalloc(" + std::to_string(count * sizeof(T)) + " bytes)");
    ptrs.push_back(p);
    bytes += count * sizeof(T);
    return static_cast<T *>(p);
  }
  template <class T>
  T *upload(const std::vector<T> &v, hipStream_t st) {
    T *p = alloc<T>(v.size());
    if (!v.empty()) ICR_HIP(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
    return p;
  }
  void release() {
    for (void *p : ptrs) (void)hipFree(p);
    ptrs.clear();
    bytes = 0;
  }
};

// Per-level host summary used to size grids.
struct LevelInfo {
  int first = 0, count = 0;   // into level_sup
  int max_n3 = 0;             // max DOF columns of a supernode
  int max_f3 = 0;             // max front order
  int max_b3 = 0;             // max below rows (DOF)
  long long max_f2 = 0;       // max f^2
  int max_rows_tiles = 0;     // max ceil(n3/64)
  int max_below_tiles = 0;    // max ceil(b3/64)
  int a_first = 0, a_count = 0;   // A-scatter entries of the level
  int child_rank_max = 0;
  int fwd_split_diag = 1, fwd_split_off = 1;   // k-chunks of the split single-RHS forward products
  int srhs_off[3] = {0, 0, 0}, srhs_cnt[3] = {0, 0, 0};   // single-RHS task lists (SR_*) of the level
};
// single-RHS task lists per level: (supernode of the level, block): forward
// diagonal (64 rows of n_s), forward below rows (64 of b_s), backward (16
// columns of n_s)
enum { SR_FWD_DIAG = 0, SR_FWD_OFF = 1, SR_BWD = 2 };

struct Mesh {
  int N = 0, T = 0, n = 0, nnzb = 0;
  double rho = 0, alpha = 0, beta = 0, h = 0, grav[3] = {0, 0, 0};
  std::vector<double> nodes;
  std::vector<int> tets;
  std::vector<uint8_t> fixed;
  MeshGraph graph;
  // device
  double *d_nodes = nullptr, *d_E = nullptr, *d_nu = nullptr;
  int *d_tets = nullptr;
  uint8_t *d_fixed = nullptr;
  int *d_bsr_ptr = nullptr, *d_bsr_col = nullptr, *d_bsr_row = nullptr;
  int *d_contrib_ptr = nullptr, *d_contrib = nullptr;  // per block: (tet*16 + a*4 + b)
  int *d_nt_ptr = nullptr, *d_nt = nullptr;            // node -> tets
  double *d_Ke = nullptr, *d_vol = nullptr, *d_mass = nullptr, *d_K = nullptr, *d_A = nullptr;
  int *d_err = nullptr;
};

struct Factor {
  Symbolic sym;
  std::vector<SupDev> sup;
  std::vector<LevelInfo> levels;
  SupDev *d_sup = nullptr;
  int *d_rows = nullptr, *d_child = nullptr, *d_invmap_off = nullptr, *d_invmap = nullptr;
  int *d_level_sup = nullptr, *d_perm = nullptr, *d_iperm = nullptr, *d_sup_of_node = nullptr;
  AScatter *d_ascat = nullptr;
  double *d_front = nullptr, *d_linv = nullptr, *d_x1 = nullptr;
  long long front_elems = 0, linv_elems = 0, x1_elems = 0;
  int *d_err = nullptr;
  double flops = 0, ms = 0;
  long long nnzL = 0;
  int max_front = 0;
  // multi-RHS arenas (grown on demand)
  int nc_cap = 0;
  double *d_X = nullptr, *d_Z = nullptr, *d_Wp = nullptr, *d_fpos = nullptr;
  int *d_keys = nullptr, *d_order = nullptr, *d_pos = nullptr, *d_lohi = nullptr, *d_cerr = nullptr;
  // Z f in column chunks: tasks (supernode, first row, first column, partial offset)
  // multi-RHS product tasks per (height level, kind), built on the device
  // from the contact ranges: (supernode, tile row << 16 | tile column)
  int2 *d_rhs_tasks = nullptr;
  int *d_rhs_off = nullptr, *d_rhs_cnt = nullptr, *d_level_first = nullptr;
  std::vector<int> rhs_off, rhs_cap;   // first entry and capacity of each list
  int4 *d_zf_tasks = nullptr;
  int n_zf_tasks = 0, n_zf_sum_tasks = 0;   // the first n_zf_sum_tasks tasks have chunk 0
  double *d_zf_part = nullptr;
  Arena rhs_arena;
  long long x_elems = 0, z_elems = 0;   // sizes of the X and Z arenas
  // mixed-precision multi-RHS solve: FP32 copies of the fronts and L_ss^-1,
  // FP32 X and Z, FP64 residual (laid out like Z)
  Arena fac32_arena, mixed_arena;
  bool have32 = false;
  int mixed_cap = 0;   // nc_cap the mixed arena was sized for
  float *d_front32 = nullptr, *d_linv32 = nullptr, *d_X32 = nullptr, *d_Z32 = nullptr;
  double *d_R = nullptr;
  // single-RHS work vectors (permuted)
  double *d_y = nullptr;
  // partial sums of the split forward products, the single-RHS task lists
  double *d_fwd_part = nullptr;
  int2 *d_srhs_tasks = nullptr;
};

// Work buffers of the PGS kernels: start gaps g [m], the compact coupling
// block (pgs_wss_elems() doubles) and a 2-int control block.
struct PgsWork {
  double *g = nullptr, *Wss = nullptr;
  double *gnSet = nullptr, *swn = nullptr;   // per contact: normal gap at the set's start state, sqrt(W~_nn)
  int *Sidx = nullptr, *nS = nullptr;         // first active set (ascending contact ids) and its size
  double *rec = nullptr, *gS = nullptr;       // its records and gaps (sets of at most 128 contacts)
  int *ctl = nullptr;                         // 4 control words
  // block Gauss-Seidel of sets beyond the chains (only when n_c > 512; NULL:
  // the single-workgroup sweep continues instead)
  // (records of all contacts, blocked diagonal couplings, the change lists of
  // two blocks, sync words)
  double *recAll = nullptr, *Wblk = nullptr, *dl = nullptr;
  int *chg = nullptr, *csync = nullptr;
};

struct Contacts {
  int count = 0;                 // candidates
  std::vector<int> nodes;
  int *d_cand = nullptr;
  double *d_mu_node = nullptr;   // friction per node (0 if not a candidate)
  int nc_cap = 0;
  int *d_nodes_c = nullptr;      // selected contact nodes of the current step
  double *d_mu = nullptr, *d_pfree = nullptr, *d_pstart = nullptr, *d_p = nullptr;
  double *d_C = nullptr, *d_Cprev = nullptr, *d_delta = nullptr, *d_dk = nullptr;
  double *d_lam = nullptr, *d_f = nullptr, *d_WH = nullptr, *d_W = nullptr;
  float *d_WH32 = nullptr, *d_W32 = nullptr;   // FP32 storage of the mixed-precision step
  PgsWork pgs;
  int8_t *d_status = nullptr;
  int *d_sweeps = nullptr;       // per Newton iteration
  double *d_eps = nullptr;
  Arena arena;
};

// Pair contacts between two bodies (icr_set_pairs): points of body 1
// against points of body 2, p = x_1 - x_2 (weights of body-2 nodes
// negative), each with a fixed normal; they come first in every step's
// contact list.
struct Pairs {
  int count = 0;            // pairs
  int nu = 0;               // their distinct nodes
  std::vector<int> nodes;   // those nodes, ascending
  std::vector<int> idx;     // per slot: index into nodes, or -1
  std::vector<double> w;    // per slot weight (0 for unused slots)
  int *d_slot_node = nullptr;   // [count*4] node id or -1
  double *d_w = nullptr, *d_normal = nullptr, *d_mu = nullptr, *d_force = nullptr;
  int *d_nodes = nullptr, *d_csr_ptr = nullptr, *d_csr_slot = nullptr;   // node -> slots naming it
  Arena arena;
  // per step size (n_contacts): node list of the W_H build, expansion maps,
  // nodal W_N, node forces
  int step_nc = 0;
  int *d_unodes = nullptr, *d_idx = nullptr;
  double *d_wexp = nullptr, *d_WN = nullptr, *d_fu = nullptr;
  Arena step_arena;
};


// Per-step parameters kept in device memory, so a captured step graph can be
// replayed: the obstacle and the time at the start of the step.
struct StepCtx {
  icr_obstacle obs;
  double t0;
  double h;
};

// One scene's Newton loop in the batched launch (k_newton_batch): sizes, its
// step options and device pointers into the scene (fast scheme, FP64, no
// pair contacts, n_c <= kPgsWaveMax).
struct NewtonTask {
  int nc, n_newton, max_sweeps, j_inner;
  double tol, h;
  const StepCtx *ctx;
  const double *WH, *pfree, *pstart, *mu;
  double *W, *p, *f, *C, *dk, *lam, *eps;
  double *g, *Wss, *gnSet, *swn;   // PGS work (PgsWork of the scene)
  int8_t *status;
  int *sweeps, *ctl;
};
constexpr int kNewtonBatchMax = 64;   // scenes per batched launch
struct NewtonBatchIdx {               // the table entries of one launch
  int n;
  int idx[kNewtonBatchMax];
};

struct State {
  StepCtx *d_ctx = nullptr;
  unsigned long long *d_stamps = nullptr;   // device-clock phase stamps of the last timed step
  icr_obstacle obs_host{};      // last obstacle written to d_ctx
  bool obs_valid = false;
  double *d_q = nullptr, *d_v = nullptr, *d_qrest = nullptr;
  double *d_b = nullptr, *d_dvfree = nullptr, *d_qfree = nullptr, *d_sol = nullptr;
  double *d_node_force = nullptr;   // world-frame force per node from the previous step
  int *d_prev_nodes = nullptr;
  int *d_prev_nc = nullptr;   // contacts of the previous step (device: a captured step graph reads it)
  double t = 0;
};

}  // namespace icr

// A captured icr_step launch sequence and the options it was captured for.
struct StepGraph {
  bool valid = false;
  icr_step_opts key{};
  long epoch = -1;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    valid = false;
  }
};

struct icr_scene {
  hipStream_t stream = nullptr;
  int device = 0;
  std::string err;
  bool assembled = false, factored = false, has_candidates = false, stepped = false;
  icr::Mesh mesh;
  icr::Factor fac;
  icr::Contacts con;
  icr::Pairs pairs;
  icr::State st;
  icr::Arena mesh_arena, fac_arena, state_arena;
  // mapped contacts of icr_build_WH: distinct nodes, slot indices, nodal W_N
  icr::Arena map_arena;
  int map_nc_cap = 0, map_nu_cap = 0;
  int *d_map_nodes = nullptr, *d_map_idx = nullptr;
  double *d_map_WN = nullptr;
  int last_nc = 0;
  bool last_mixed = false;   // the last step kept W_H in FP32
  int last_build_nc = 0;   // contact count of the last multi-RHS forward solve (Z valid for it)
  long epoch = 0;          // bumped whenever device buffers are (re)allocated
  int clock_khz = 0;       // device wall-clock rate used by the phase stamps
  StepGraph sg;
  // second stream of the multi-RHS solve: the W_H products of a tree level
  // run there while the main stream goes on with the next level's solve
  bool overlap = true;
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

namespace icr {

// k_fem.hip
void launch_element_matrices(icr_scene *s);
void launch_assemble_blocks(icr_scene *s);
void launch_free_rhs(icr_scene *s, const double *q, const double *v, double *b);
void launch_axpy_qfree(icr_scene *s);
void launch_integrate(icr_scene *s);

// k_factor.hip
void run_numeric_factor(icr_scene *s);

// k_solve.hip
void single_rhs_solve(icr_scene *s, const double *b, double *x);
// x = A^-1 H^T f for the contacts of the last build_WH_device call (reuses Z).
void contact_force_solve(icr_scene *s, const double *f, double *x);
void ensure_rhs_capacity(icr_scene *s, int nc);
void launch_fill(icr_scene *s, double *x, long n, double v);
void launch_widen(icr_scene *s, const float *x, double *y, long n);   // y = (double) x
void launch_narrow(icr_scene *s, const double *x, float *y, long n);  // y = (float) x
// W_H = H A^-1 H^T, or J A^-1 J^T with J = C H when per-contact frames
// [nc*9] are given (the standard rebuild of Algorithm 2).
void build_WH_device(icr_scene *s, int nc, const int *node_ids, double *WH, bool validate,
                     const double *frames = nullptr);
// Mixed precision: Z by FP32 MFMA solves, `refine` steps of iterative
// refinement with the residual P H^T - L Z formed in FP64, W_H = Z^T Z in
// FP64, written as FP32 (WH32) and/or FP64 (WH64).  Needs ensure_mixed.
void ensure_mixed(icr_scene *s);
void build_WH_mixed(icr_scene *s, int nc, const int *node_ids, int refine, float *WH32, double *WH64);
// W_H of mapped contacts from the nodal W_N of their distinct nodes:
// idx [nc*4] slot -> index into those nodes (-1 unused), w [nc*4] weights.
void launch_wh_expand(hipStream_t st, int nc, int nu, const int *idx, const double *w, const double *WN, double *WH);

// k_contact.hip
void launch_select_contacts(icr_scene *s, int nc);
void launch_directions(icr_scene *s, int nc, bool first);
void launch_set_ctx(icr_scene *s, const icr_obstacle *obs, const double *t0);
void launch_stamp(icr_scene *s, int slot);
// W and W_H stored as double, or as float (the mixed-precision step: every
// sum is still taken in FP64)
template <class TW>
void launch_update_W(hipStream_t st, int nc, const TW *WH, const double *C, TW *W);
constexpr int kPgsMaxContacts = 4096;
constexpr int kMaxNewton = 256;   // Newton iterations per step (per-iteration sweeps, eps, stamps)
// Layout of the PGS work buffers: per-contact records of kPgsRecWidth
// doubles, the blocked coupling matrix of an active set of up to kPgsWaveMax
// contacts in 3x3 blocks of kPgsBlk doubles, padded to pgs_wave_pad contacts.
constexpr int kPgsRecWidth = 22;
constexpr int kPgsWaveMax = 512;
constexpr int kPgsBlk = 10;
// 64 contacts per register slot, two slots per chain wave beyond 64 contacts
__host__ __device__ constexpr inline int pgs_wave_pad(int nS) { return nS <= 64 ? 64 : 128 * ((nS + 127) / 128); }
// doubles of the blocked coupling matrix of an active set (n_c contacts)
constexpr inline size_t pgs_wss_elems(int nc) {
  return (size_t)(nc < kPgsWaveMax ? nc : kPgsWaveMax) * pgs_wave_pad(nc < kPgsWaveMax ? nc : kPgsWaveMax) * kPgsBlk;
}
// doubles of the prepared records (and gaps) of a first active set
constexpr inline size_t pgs_rec_elems(int nc) { return (size_t)(nc < kPgsWaveMax ? nc : kPgsWaveMax) * kPgsRecWidth; }
// Block Gauss-Seidel over the whole GPU (sets beyond kPgsWaveMax contacts):
// blocks of kPgsCoopB contacts, each block's couplings padded like a wave set.
constexpr int kPgsCoopB = 128;
constexpr int kPgsCoopSync = 256;   // ints of sync words
constexpr inline size_t pgs_coop_blk_elems(int nc) {
  return (size_t)((nc + kPgsCoopB - 1) / kPgsCoopB) * kPgsCoopB * kPgsCoopB * kPgsBlk;
}
void pgs_prepare();   // kernel attributes (dynamic LDS), once per device; call outside graph capture
// The Newton loops of the scenes tasks[ids.idx[0..n)] (device table), one
// workgroup each, in one launch on stream st.
void launch_newton_batch(hipStream_t st, const NewtonTask *tasks, const NewtonBatchIdx &ids);
int coop_grid();      // workgroups of the cooperative large-set PGS on this device (0: not available)
void launch_pgs_per_constraint(hipStream_t st, int nc, const StepCtx *ctx, const double *WH, const double *pfree,
                               const double *p, const double *pstart, const double *mu, double h, double *f,
                               double *Cm, double *lam, int8_t *status, int max_sweeps, double tol, int j_inner,
                               int *sweeps_dev, double *eps_dev, const PgsWork &wk);
template <class TW>
void launch_pgs(hipStream_t st, int nc, const TW *W, const double *d, const double *mu, double h,
                double *lam, int8_t *status, int max_sweeps, double tol, int j_inner, int *sweeps_dev,
                double *eps_dev, const PgsWork &wk);
void launch_world_force(hipStream_t st, int nc, const double *C, const double *lam, double *f);
// f = C^T lambda and the proximity update p = p_free + h^2 W_H f (Eq. 31) in one launch
template <class TW>
void launch_world_force_proximity(hipStream_t st, int nc, const double *Cm, const double *lam, double *f,
                                  const TW *WH, const double *p_free, double h, double *p);
template <class TW>
void launch_proximity(hipStream_t st, int nc, const TW *WH, const double *p_free, const double *f, double h,
                      double *p);
// World-frame forces of this step's contacts become the next step's warm
// start (previous contacts cleared), then the step time advances.
void launch_store_forces(icr_scene *s, int nc);
// pair contacts of a step (first pairs.count contacts) and the node list of its W_H build
void launch_pair_points(icr_scene *s, int nc);
// fu = H_w^T f on the nodes of the step's W_H build
void launch_node_forces(icr_scene *s, int nc, const double *f, double *fu);
void launch_standard_proximity(icr_scene *s, int nc);

}  // namespace icr
