// Internal host-side structures of the solver library.
#pragma once
#include <hip/hip_runtime.h>

#include <chrono>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/fsi_mg.h"
#include "fsi_kernels.h"

namespace fsi {

struct Error {
  fsi_status code;
  std::string msg;
  Error(fsi_status c, std::string m) : code(c), msg(std::move(m)) {}
};

void set_error(const std::string &m);
void hip_check(hipError_t e, const char *what);
int pick_lpr(int64_t nnz, int64_t nrows);

struct DevCsr {
  int n = 0, m = 0, nnz = 0, lpr = 8;
  int *rowptr = nullptr, *col = nullptr;
  double *val = nullptr;
  float *val32 = nullptr;
  CsrView<double> v64() const { return CsrView<double>{n, m, nnz, rowptr, col, val}; }
  CsrView<float> v32() const { return CsrView<float>{n, m, nnz, rowptr, col, val32}; }
};

struct Level {
  int n = 0;
  DevCsr J, P, R;
  // Schwarz patches
  int npatch = 0, mmax = 0, ntask = 0;
  int64_t sum_m = 0, sum_m2 = 0, sum_om = 0, total_owned = 0, boff_total = 0, woff_total = 0;
  std::vector<int64_t> h_ptr, h_boff;
  int64_t blk_base = 0;   // offset of this level's blocks in the shared scratch
  int64_t pm_base = 0;    // offset of this level's pivot arrays (sum of m over earlier levels)
  std::vector<int32_t> h_dof;
  std::vector<uint8_t> h_owned, h_kind;
  int *d_pm = nullptr, *d_po = nullptr, *d_dof = nullptr, *d_out_off = nullptr,
      *d_own_local = nullptr, *d_out_idx = nullptr, *d_task_patch = nullptr,
      *d_task_row0 = nullptr, *d_row_patch = nullptr, *d_row_local = nullptr,
      *d_unowned = nullptr;
  int n_unowned = 0;
  int64_t *d_pdof_off = nullptr, *d_woff = nullptr, *d_boff = nullptr;
  // 16-bit owned rows in groups of four columns (columns padded to m4 = a
  // multiple of 4): per patch offsets, and the storage's length
  int64_t *d_woff16 = nullptr;
  int64_t woff16_total = 0;
  // block extraction map (launch_extract_map): nslots (entry, position) pairs
  int64_t ext_nslots = 0;
  int *d_ext_src = nullptr, *d_ext_dst = nullptr;
  int64_t *d_ext_slot_off = nullptr;
  // solid blocks apart (solid_precision / refine_sweeps): owned rows in FP32
  // (ntask_s tasks, offsets woff into Ws), or full FP32 inverses (nftask
  // packing tasks over all rows, offsets woff_full into Wfull) applied with
  // refinement sweeps; nref refined blocks with local CSR rows of B_k
  int ntask_s = 0, nref = 0, nftask = 0;
  int64_t woff_solid = 0, wfull_total = 0, full_rows = 0;
  int *d_task_patch_s = nullptr, *d_task_row0_s = nullptr, *d_po_full = nullptr,
      *d_full_off = nullptr, *d_full_local = nullptr, *d_ftask_patch = nullptr, *d_ftask_row0 = nullptr,
      *d_ref_patch = nullptr, *d_ref_src = nullptr, *d_own_dof = nullptr;
  int64_t *d_woff_full = nullptr;
  float *yref0 = nullptr, *yref1 = nullptr, *gref = nullptr, *rhoref = nullptr;   // refined rows' vectors
  int *d_ref_growptr = nullptr, *d_ref_gcol = nullptr;   // the refined blocks as one CSR (rows, columns)
  float *bref = nullptr;                                  // its values (FP32, gathered at refactor)
  int ref_nnz = 0, ref_lpr = 8;
  float *Ws = nullptr, *Wfull32 = nullptr, *Wscale_full = nullptr;
  uint16_t *Wfull16 = nullptr;
  double *W64 = nullptr;
  float *W32 = nullptr;
  uint16_t *W16 = nullptr;
  float *Wscale = nullptr, *Cscale = nullptr;
  int w16_kind = 0;
  // ILU(0) of the fluid blocks (fluid_ilu): the nilu blocks, their rows'
  // L/U patterns, the factors' positions in the dense blocks (level-relative)
  // and values (FP64, or FP32 in a mixed hierarchy)
  int nilu = 0, ilu_max_entries = 0;
  int64_t ilu_nl = 0, ilu_nu = 0, ilu_rows = 0;
  int *d_ilu_patch = nullptr, *d_ilu_row0 = nullptr, *d_ilu_lptr = nullptr, *d_ilu_uptr = nullptr,
      *d_ilu_cptr = nullptr, *d_ilu_lpos = nullptr, *d_ilu_upos = nullptr, *d_ilu_dpos = nullptr,
      *d_ilu_flev = nullptr, *d_ilu_flev_off = nullptr, *d_ilu_blev = nullptr, *d_ilu_blev_off = nullptr;
  int16_t *d_ilu_lcol = nullptr, *d_ilu_ucol = nullptr, *d_ilu_crow = nullptr, *d_ilu_frow = nullptr,
          *d_ilu_brow = nullptr;
  uint32_t *d_ilu_mask = nullptr;
  int64_t *d_ilu_moff = nullptr;
  double *ilu_l64 = nullptr, *ilu_u64 = nullptr, *ilu_d64 = nullptr;
  float *ilu_l32 = nullptr, *ilu_u32 = nullptr, *ilu_d32 = nullptr;
  // device Galerkin product (fsi_mg_galerkin), on levels >= 1: T = J P on
  // its pattern (prepared at the first call), and the positions of the next
  // coarser level's Dirichlet diagonals; the Dirichlet rows of this level
  // when the input flags them
  // Galerkin products as gathers: for every entry q of T = J P (then of the
  // coarse operator R T), its contributions t in [ptr[q], ptr[q+1]) are
  // w[t] * x[idx[t]], x the variable operand's values (J, then T), w the
  // constant one's (P, then R), listed in the order a row-by-column product
  // sums them
  int *d_gt_ptr = nullptr, *d_gt_idx = nullptr, *d_gc_ptr = nullptr, *d_gc_idx = nullptr, *d_cdir_pos = nullptr;
  double *d_gt_w = nullptr, *d_gc_w = nullptr, *d_t_val = nullptr;
  int64_t gt_n = 0, gc_n = 0;
  int n_cdir = 0;
  std::vector<int> h_dir;
  bool dir_known = false;
  // coarsest level: row-major inverse
  double *C0 = nullptr;
  // work vectors
  double *r = nullptr, *e = nullptr, *s = nullptr;
  float *r32 = nullptr, *e32 = nullptr, *s32 = nullptr;
};

// Caching device allocator for the server: freed blocks are kept (by size)
// and handed out again, so serving never calls hipFree (which synchronises
// the device); everything is released when the pool is destroyed.
struct DevicePool {
  std::mutex mu;
  std::multimap<size_t, void *> free_blocks;
  std::vector<void *> all;
  int64_t allocated = 0, in_use = 0, peak_in_use = 0;   // bytes: hipMalloc'd, handed out, most handed out
  void *get(size_t bytes, size_t *got);
  void put(void *p, size_t bytes);
  ~DevicePool();
};

// Device allocations owned by one object: from the pool when there is one,
// else hipMalloc/hipFree.
struct DevList {
  DevicePool *pool = nullptr;
  std::vector<std::pair<void *, size_t>> v;
};

struct Krylov {
  int m = 0;
  double *V = nullptr, *Z = nullptr, *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr,
         *y = nullptr, *h1 = nullptr, *partial = nullptr, *npart = nullptr,
         *nrm = nullptr, *flags = nullptr, *scal = nullptr, *w = nullptr;
  double *pinned = nullptr;       // 8 doubles of host-coherent pinned memory (a pool slot)
  double *pinned_dev = nullptr;   // its device address
  hipEvent_t ev_done = nullptr;   // recorded after a phase's D2H copy, polled by the host
  std::vector<hipGraphExec_t> step_graphs;   // Arnoldi step j as one graph (use_graph)
  int graph_side = -1, graph_orth = -1;      // the solve variant the step graphs hold
  DevList owned;
};

struct GraphKey {
  const double *r;
  double *z;
  bool operator<(const GraphKey &o) const { return r < o.r || (r == o.r && z < o.z); }
};

// a block above kMaxPatch dofs, inverted on its own by the Gauss-Jordan chain
struct LargeBlock {
  int q;            // index in the all-level block tables (status)
  int m;            // its dofs
  int64_t boff;     // its offset in the block scratch
  int64_t poff;     // its offset in the permutation arrays
};
struct MG {
  int nlevels = 0;
  int device = 0;                 // HIP device current at setup
  double *static_ws = nullptr;    // that device's static Krylov workspace (fsi_fgmres_solve_noalloc)
  bool mixed = false;
  fsi_mg_opts opts{};
  // blocks above kMaxPatch dofs (left out of the batched inversion): the
  // padded FP64 working copy (large_ld columns), the FP64 inverse of the mixed
  // forms before its cast, the identity dof map and the chain's int work
  std::vector<LargeBlock> large;
  int large_mmax = 0;
  int64_t large_ld = 0;
  double *large_A = nullptr, *large_C = nullptr;
  int *large_iota = nullptr, *large_iwork = nullptr;
  std::vector<Level> lv;
  DevList owned;
  hipStream_t own_stream = nullptr;
  bool own_side = true;   // side_stream created by the handle (else borrowed)
  Krylov kry;
  std::map<GraphKey, hipGraphExec_t> graphs;
  double setup_ms = 0.0;
  // persistent setup scratch: dense blocks, pivot status, coarse dense matrix, GJ work
  double *blk_scratch = nullptr, *dense_scratch = nullptr, *gj_work = nullptr;
  int *status = nullptr, *status0 = nullptr;
  int64_t blk_total = 0;
  int64_t *all_boff = nullptr, *all_poff = nullptr;
  int *all_pm = nullptr;
  int *gj_perm = nullptr, *gj_used = nullptr;   // pivot permutations of the block inverses
  int64_t dense_ld = 0;                         // leading dimension of the coarse dense matrix
  // coarsest operator split (CoarseSplit): nf free dofs inverted densely, nd
  // diagonal-only dofs by a reciprocal
  int coarse_nf = 0, coarse_nd = 0;
  int *coarse_fpos = nullptr, *coarse_dlist = nullptr;
  int npatch_all = 0, mmax_all = 1;
  int gj_variant = 0;     // batched Gauss-Jordan kernel variant (GjVariant, 0 = by size)
  int gj_grid = 0;        // its workgroups, and their block lists (gj_schedule)
  int *gj_sched = nullptr;
  std::vector<int> h_all_pm;   // block sizes of all levels, in the batched order
  hipStream_t side_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipGraphExec_t coarse_graph = nullptr;   // the coarsest inversion's launch chain, replayed per refactor
  // event timing of the finest-level Schwarz kernel
  bool prof_on = false;
  size_t prof_used = 0, prof_gj_used = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev, prof_gj_ev;   // Schwarz (finest), batched inversion
  bool galerkin_ready = false;   // the device Galerkin product's patterns are prepared
};

extern thread_local std::string g_last_error;

// pool (may be NULL): device memory from the caching allocator; side_st (may
// be NULL): a borrowed second stream for the coarsest inversion
MG *mg_setup(const fsi_level *levels, int nlevels, const fsi_mg_opts *opts, hipStream_t user_st,
             hipStream_t own_st, DevicePool *pool = nullptr, hipStream_t side_st = nullptr);
void destroy_mg(MG *mg);
void validate_levels(const fsi_level *levels, int nlevels, const fsi_mg_opts *opts);
void validate_levels_light(const fsi_level *levels, int nlevels, const fsi_mg_opts *opts);
void apply_vcycle(MG &mg, const double *r, double *z, hipStream_t st);
void run_vcycle(MG &mg, const double *r, double *z, hipStream_t st);
fsi_status fgmres(MG &mg, const double *b, double *x, const fsi_krylov_opts &ko, fsi_solve_info *info,
                  hipStream_t st, Krylov *ws = nullptr);
RasView ras_view(const Level &L);
void ensure_krylov(MG &mg, int m);
void clear_graphs(MG &mg);
double *pinned_slot_acquire();
void pinned_slot_release(double *s);
void refactor(MG &mg, hipStream_t st);
// coarse operators R J P on the device from the finest values (fsi_mg_galerkin)
void galerkin(MG &mg, hipStream_t st);
void release_setup_scratch(MG &mg);

// GMRES(m) as a host state machine over the device work (section "Details on
// the iterative solver").  RIGHT: flexible GMRES, z_j = M^{-1} v_j kept, the
// monitored residual is |b - J x|.  LEFT: GMRES on M^{-1} J, the monitored
// residual is |M^{-1}(b - J x)| and the reference of the stopping rule is its
// initial value; a final phase computes the true residual |b - J x|.
struct FgmresRun {
  enum Phase { kFirst, kIter, kCheck, kFinal, kDone };
  MG *mg = nullptr;
  Krylov *K = nullptr;            // the workspace: mg->kry, or a caller-bound one (no graphs)
  const double *b = nullptr;
  double *x = nullptr;
  fsi_krylov_opts ko{};
  hipStream_t st = nullptr;
  Phase phase = kDone;
  bool left = false, twice = true, graphs = false;
  double bnorm = 0.0, ref = 0.0, beta = 0.0, beta0 = 0.0, est = 0.0, true_res = 0.0;
  int iters = 0, restarts = 0, j = 0, k = 0, limit = 0, nhist = 0;
  bool fixed = false, converged = false;
  std::chrono::steady_clock::time_point t0;
  // ws: NULL (the handle's own workspace, allocated on first use, steps
  // replayed from graphs when use_graph) or a workspace bound by
  // bind_krylov (no allocation, no graphs)
  void start(MG &mg, const double *b, double *x, const fsi_krylov_opts &ko, hipStream_t st,
             Krylov *ws = nullptr);
  void enqueue();
  // a step split around a V-cycle applied by the caller (phase kIter):
  // enqueue_step_pre, then z = M^{-1} vin into vout on any stream ordered
  // between the two, then enqueue_step_post
  void enqueue_step_pre(const double **vin, double **vout);
  void enqueue_step_post();
  bool complete();
  void fill_info(fsi_solve_info *info) const;
 private:
  void enqueue_residual();
  void enqueue_true_residual();
  void enqueue_step();
  void finish_cycle();
  bool finish();
  void add_hist(double v);
};
void validate_krylov(const fsi_krylov_opts &ko);
// V-cycles of several systems in batched launches (z = M^{-1} r each, r != z);
// the systems must be batch_compatible with each other
struct BatchItem {
  MG *mg;
  const double *r;
  double *z;
};
bool batch_compatible(const MG &a, const MG &b);
void batched_vcycle(const std::vector<BatchItem> &items, hipStream_t st);
// doubles of device memory the Krylov buffers of an n-row system with restart m take
int64_t krylov_doubles(int n, int m);
// points the buffers of K into base (krylov_doubles(n, m) doubles, 256-byte
// aligned); the pinned slot and the event are the handle's (acquired at setup)
void bind_krylov(Krylov &K, const MG &mg, double *base, int n, int m);

}  // namespace fsi
