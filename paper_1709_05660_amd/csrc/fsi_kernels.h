// Internal launch interface of the gfx950 kernels (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

namespace fsi {

constexpr int kWave = 64;
constexpr int kMaxPatch = 800;      // largest Schwarz block of the batched inversion, ILU and refinement
constexpr int kMaxLargePatch = 6144;   // larger blocks: one Gauss-Jordan chain each (equal to kMaxCoarse)

// CSR on the device: int32 offsets and columns (sizes checked at upload).
template <typename T>
struct CsrView {
  int nrows, ncols, nnz;
  const int *rowptr, *col;
  const T *val;
};

// ---- sparse operators (a4, a6): y = A x | y = r - A x | y += A x
enum SpmvMode { kSpmvSet = 0, kSpmvResid = 1, kSpmvAdd = 2 };
template <typename T>
void launch_spmv(const CsrView<T> &A, const T *x, const T *r, T *y, int mode, int lanes_per_row,
                 hipStream_t st);

// ---- setup (a1, a2, a3)
void launch_fill_f64(double *x, int64_t n, double v, hipStream_t st);
// extraction map of a level (built once): for every slot, one CSR entry of a
// block row (slots of row t start at slot_off[t]), the entry's index src and
// its position dst in the level's blocks (row-major B_k at boff[k]), -1 when
// its column lies outside the block; dst < 2^31 (checked on the host)
void launch_extract_map(const CsrView<double> &J, const int *pm, const int64_t *pdof_off,
                        const int *dof, const int64_t *boff, int64_t total_rows,
                        const int *row_patch, const int *row_local, const int64_t *slot_off,
                        int *src, int *dst, hipStream_t st);
// B_k = J[I_k, I_k] through the map (blocks zero-filled beforehand), in
// FP64 or rounded to FP32
void launch_extract(const double *val, int64_t nslots, const int *src, const int *dst,
                    double *blocks, hipStream_t st);
void launch_extract(const double *val, int64_t nslots, const int *src, const int *dst,
                    float *blocks, hipStream_t st);
// Gauss-Jordan inverse of every block, one workgroup per block (m <= 1024),
// rows never exchanged: Binv[i][c] = S[perm[i]][used[c]] with S left in the
// block and perm/used at poff[k]; status[k] = 0 ok, else 1 + failing step
// kernel variants (panel width x threads), chosen by the autotuner: NB 16
// on 256 or 512 threads, NB 32 on 512 with the panel in LDS (m <= 512), and
// a wide panel read back from the block itself (NB 32 for m <= 512, 24 for
// m <= 1024, 512 threads), and NB 24 on 512 threads with the panel in LDS
// (where m 25 doubles fit beside the static LDS, m <= ~790).  An
// unsupported or zero variant falls back to the first that fits of NB 32
// pairs, NB 32, NB 24 (both with the LDS panel) and NB 16 on 256 threads
// Paired panels (k_gj_paired, blocks up to 512 dofs): two panels of NB 32
// (one row per thread) factored in turn, the rest of the block updated once
// per pair.
enum GjVariant { kGjAuto = 0, kGj16x256 = 1, kGj16x512 = 2, kGj32x512 = 3, kGjWideG = 4, kGj24x512 = 5,
                 kGjP32x512 = 6,
                 // FP32 working matrices (mixed forms): panel width x threads (x rows per thread)
                 kGjF64x512 = 11, kGjF32x512 = 12, kGjF32x256 = 13, kGjF32x512r2 = 14, kGjF48x512r2 = 15,
                 kGjPF32x512 = 16 };
bool gj_variant_ok(int variant, int mmax);
bool gj_variant_f32(int variant);
// workgroups of the batched inversion for npatch blocks (the fewest rounds
// over the compute units), and the host-built schedule: grid + 1 offsets
// into the block list that follows them (grid + 1 + npatch ints)
int gj_batched_grid(int npatch);
std::vector<int> gj_schedule(const int *pm, int npatch, int grid);
// ev0/ev1 (optional): events recorded at the kernel's own start and end
void launch_gj_batched(double *blocks, const int64_t *boff, const int *pm, const int64_t *poff,
                       int *perm, int *used, int npatch, int mmax, int *status, int grid,
                       const int *sched, hipStream_t st, int variant = kGjAuto,
                       hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// the same elimination on FP32 blocks (the working matrices of the mixed
// forms), on the FP32 matrix cores
void launch_gj_batched_f32(float *blocks, const int64_t *boff, const int *pm, const int64_t *poff,
                           int *perm, int *used, int npatch, int mmax, int *status, int grid,
                           const int *sched, hipStream_t st, int variant = kGjAuto,
                           hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// The coarsest operator's dofs split into D, whose row and column hold only
// the diagonal entry (Dirichlet rows of a symmetrically eliminated
// operator), and the free rest F: the operator is diag(a_D) + A_FF up to
// ordering, and so is its inverse.  fpos[i]: position of dof i in F, -1 in
// D; dlist: the nd dofs of D; rowptr/val: the operator's CSR on the device
// (a_dd is the single entry of row d).
struct CoarseSplit {
  int n = 0, nd = 0;
  const int *fpos = nullptr, *dlist = nullptr, *rowptr = nullptr;
  const double *val = nullptr;
};
// inverse of the coarsest operator written row-major (n x n) to C0: the
// dense F x F block A (leading dimension ld, nf <= kMaxCoarse, overwritten)
// by Gauss-Jordan, 1 / a_dd on D; iwork: 2 nf ints; status[0] = 0 ok, else
// 1 + failing step (the steps of D follow the nf of F)
constexpr int kMaxCoarse = 6144;
void launch_fill_i32(int *x, int n, int v, hipStream_t st);
// x[i] = i for i < n
void launch_iota_i32(int *x, int n, hipStream_t st);
// dst[i ld + j] = (double) src[i m + j] for i, j < m (a block into a padded FP64 copy)
template <typename TS>
void launch_copy_block(const TS *src, int m, double *dst, int64_t ld, hipStream_t st);
void gj_coarse(double *A, int nf, int64_t ld, const CoarseSplit &cs, double *C0, int *status,
               int *iwork, hipStream_t st);
// Owned rows of Binv_k, column-major per (patch, 64 owned rows) task: task
// (k, r0) with nr = min(64, o_k - r0) rows holds entry (c, r) at
// W[woff_k + r0 m_k + c nr + r - r0]; optional FP32/16-bit copies; the
// inverted blocks in FP64 or FP32 (TB).  With woff16, the 16-bit copy groups
// four columns per row instead: with m4 = m_k rounded up to a multiple of 4,
// entry (c, r) at W16[woff16_k + r0 m4 + (c / 4) 4 nr + 4 (r - r0) + c % 4]
// (the padding columns are never written: the caller zeroes them once)
template <typename TB>
void launch_pack_owned(const TB *blocks, const int64_t *boff, const int *pm, const int *po,
                       const int64_t *woff, const int *own_off, const int *own_local,
                       const int *task_patch, const int *task_row0, int ntask, double *W64,
                       float *W32, uint16_t *W16, int w16_kind, float *wscale,
                       const int64_t *pdof_off, const float *cscale, const int *perm,
                       const int64_t *woff16, hipStream_t st);
// 16-bit storage: per-column scales of the owned rows of every block inverse
template <typename TB>
void launch_colscale(const TB *blocks, const int64_t *boff, const int *pm, const int *po,
                     const int *own_off, const int *own_local, const int64_t *pdof_off,
                     const int *task_patch, const int *task_row0, int ntask, int64_t total_cols,
                     float *cscale, const int *perm, int mmax, hipStream_t st, bool first = true,
                     bool last = true);

// ---- smoother (a5): e[out] += omega * W_k s[I_k] for every owned row
//      (16-bit: W_k = diag(rs) W16 diag(cs), two-sided scaling)
struct RasView {
  int ntask;
  const int *task_patch, *task_row0;
  const int *pm, *po;
  const int64_t *pdof_off, *woff;   // 16-bit storage: the grouped layout's offsets (woff16)
  const int *dof, *out_off, *out_idx;
  const float *cscale;   // 16-bit storage: column scales (per patch dof), else null
  const int *unowned;    // the dofs no patch owns (nunowned of them)
  int nunowned;
  int mmax;              // the largest block (the gathered vector's LDS, sized at launch)
};
// e[owned dofs] (+= when add, else =) omega * (owned rows of B_k^{-1}) s_k; with
// add false (a zero initial correction) the dofs no patch owns are set to 0,
// so e needs no clearing.  ev0/ev1: optional events recorded at the
// finest-level kernel's start and end
void launch_ras_f64(const RasView &v, const double *W, const double *s, double *e, double omega,
                    bool finest, bool add, hipStream_t st, hipEvent_t ev0 = nullptr,
                    hipEvent_t ev1 = nullptr);
void launch_ras_f32(const RasView &v, const float *W, const float *s, float *e, float omega,
                    bool finest, bool add, hipStream_t st, hipEvent_t ev0 = nullptr,
                    hipEvent_t ev1 = nullptr);
void launch_ras_16(const RasView &v, const uint16_t *W, int w16_kind, const float *wscale,
                   const float *s, float *e, float omega, bool finest, bool add, hipStream_t st,
                   hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// ---- refined local solves of the solid blocks (mixed forms): per block k,
// g = s[I_k], y = W~ g, then `sweeps` times y += W~ (g - B_k y) with
// B_k = J[I_k, I_k] in FP32, and e[owned] (+)= omega y.  B: all refined
// blocks as one FP32 CSR matrix over their rows (row full_off[k] + i of block
// k, columns in the same numbering), applied by the SpMV with lpr lanes per
// row; gfull, rho: vectors of the refined rows.  W~: every row of the inverse
// (FP32, or 16-bit with row scales rscale at full_off[k] and column scales
// cscale at pdof_off[k]) in the packing's task layout (rows in chunks of 64,
// column-major inside a chunk) at woff_full[k]; the ntask (block, 64 rows)
// tasks of all refined blocks; own_dof[full_off[k] + i]: the global dof that
// row i writes, -1 when block k does not own it.  y0, y1: two scratch vectors
// of the refined rows (full_off totals).  With add false the dofs no patch
// owns are also cleared.  1 + sweeps launches.
struct RefineView {
  int ntask, w16_kind, lpr;
  const int *task_patch, *task_row0, *pm, *dof, *full_off, *own_dof;
  const int64_t *pdof_off, *woff_full;
  CsrView<float> B;
  float *gfull, *rho;
  const float *rscale, *cscale;
  const int *unowned;
  int nunowned;
};
// out[q] = val[src[q]] (the refined blocks' values, refreshed at each refactor)
void launch_gather_f32(const float *val, const int *src, int n, float *out, hipStream_t st);
void launch_ras_refine(const RefineView &v, const float *W32, const uint16_t *W16, const float *s, float *e,
                       float omega, bool add, int sweeps, float *y0, float *y1, hipStream_t st);

// ---- ILU(0) local solves of the fluid blocks (fluid_ilu): per ILU block b
// (patch patch[b], m rows, index r = row0[b] + k for its row or column k),
// L (unit lower) and U (upper) on the block's pattern, U's diagonal apart.
// L's rows: columns lcol[lptr[r] .. lptr[r + 1]) (< k); U's rows: ucol[uptr[r]
// .. uptr[r + 1]) (> k); L's columns: rows crow[cptr[r] .. cptr[r + 1])
// (> k); local indices.  The factorization uses U's rows and L's columns
// with the pattern as a bit mask (m x m bits at word moff[b]).  The
// substitutions go level by level: the block's rows sorted by forward level
// are frow[row0[b] ..), level f spanning frow[flev[f] .. flev[f + 1]) for f
// in [flev_off[b], flev_off[b + 1]) (a row's L columns all lie in earlier
// levels); backward levels likewise (brow, blev, blev_off; U columns in
// earlier levels).  frow/brow hold local row numbers.
struct IluView {
  int nblk;
  const int *patch, *row0;
  const int *pm, *dof, *out_off, *own_local, *out_idx;
  const int64_t *pdof_off, *boff;
  const int *lptr, *uptr, *cptr;
  const int16_t *lcol, *ucol, *crow;
  const int16_t *frow, *brow;
  const int *flev, *flev_off, *blev, *blev_off;
  const uint32_t *mask;
  const int64_t *moff;
  const int *unowned;
  int nunowned;
  int max_entries;   // entries of the largest single factor (L or U) of any block (LDS staging when they fit)
};
// in place on the dense blocks B_k (row-major at boff[k]; FP64 or FP32),
// zero off the pattern on entry; status[status_base + patch] = 0, or 1 + the
// step whose pivot is zero or not finite
template <typename T>
void launch_ilu_factor(const IluView &v, T *blocks, int *status, int status_base, hipStream_t st);
// out[q] = (V) blocks[pos[q]] for q < n (the factors' values, compacted)
template <typename T, typename V>
void launch_ilu_gather(const T *blocks, const int *pos, int64_t n, V *out, hipStream_t st);
// e[owned dofs of every ILU block] (+)= omega (L U)^{-1} s[I_k] (lval, uval:
// the L and U values in row order; udiag: U's diagonal by row); with clear
// (and add false) also e[unowned] = 0 (when no other Schwarz launch of the
// level does)
template <typename V>
void launch_ilu_apply(const IluView &v, const V *lval, const V *uval, const V *udiag, const V *s, V *e,
                      V omega, bool add, bool clear, hipStream_t st);

// ---- Galerkin product on the device: out[q] = sum of x[idx[t]] * w[t] over
// t in [ptr[q], ptr[q+1]) in list order, for q < n (a sparse product C = A B
// on C's given pattern, its terms listed once on the host; entries that no
// term reaches are 0).  add_at: val[pos[t]] += v for t < n (Dirichlet
// diagonals).
void launch_gather_dot(int n, const int *ptr, const int *idx, const double *w, const double *x, double *out,
                       hipStream_t st);
void launch_add_at(double *val, const int *pos, int n, double v, hipStream_t st);

// ---- coarsest solve (a7): y = W x, W row-major n x n FP64
void launch_dense_gemv(const double *W, int n, const double *x, double *y, hipStream_t st);

// ---- measurement: plain streaming read of n doubles (x 16-byte aligned, n
// even); out receives kStreamReadBlocks partial sums
constexpr int kStreamReadBlocks = 1024;
void launch_stream_read(const double *x, int64_t n, double *out, hipStream_t st);

// ---- batches: one launch applies an operation to up to kMaxBatch
// independent systems (the server's co-resident systems), each entry on
// workgroups [blk0[s], blk0[s + 1]) with the arithmetic of its single launch.
// The launchers split longer lists and group entries by the single launch's
// template shape (lanes per row, waves per Schwarz workgroup).
constexpr int kMaxBatch = 16;
template <typename T>
struct SpmvItem {
  CsrView<T> A;
  const T *x, *r;
  T *y;
};
template <typename T>
struct SpmvBatch {
  int count, mode;
  int blk0[kMaxBatch + 1];
  SpmvItem<T> it[kMaxBatch];
};
// lpr[i]: the lanes per row of entry i (as launch_spmv takes it)
template <typename T>
void launch_spmv_batch(const SpmvItem<T> *items, const int *lpr, int count, int mode, hipStream_t st);
template <typename WT, typename VT>
struct RasItem {
  RasView v;
  const WT *W;
  int w16_kind;
  const float *wscale;
  const VT *s;
  VT *e;
};
template <typename WT, typename VT>
struct RasBatch {
  int count;
  int blk0[kMaxBatch + 1];
  RasItem<WT, VT> it[kMaxBatch];
};
void launch_ras_batch_f64(const RasItem<double, double> *items, int count, double omega, bool add,
                          hipStream_t st);
void launch_ras_batch_f32(const RasItem<float, float> *items, int count, float omega, bool add,
                          hipStream_t st);
void launch_ras_batch_16(const RasItem<uint16_t, float> *items, int count, float omega, bool add,
                         hipStream_t st);
struct GemvItem {
  const double *W;
  int n;
  const double *x;
  double *y;
};
struct GemvBatch {
  int count;
  int blk0[kMaxBatch + 1];
  GemvItem it[kMaxBatch];
};
void launch_dense_gemv_batch(const GemvItem *items, int count, hipStream_t st);
template <typename A, typename B>
struct CastItem {
  const A *x;
  B *y;
  int n;
};
template <typename A, typename B>
struct CastBatch {
  int count;
  int blk0[kMaxBatch + 1];
  CastItem<A, B> it[kMaxBatch];
};
template <typename A, typename B>
void launch_cast_batch(const CastItem<A, B> *items, int count, hipStream_t st);

// ---- vectors
void launch_cast_d2f(const double *x, float *y, int n, hipStream_t st);
void launch_cast_f2d(const float *x, double *y, int n, hipStream_t st);
void launch_fill_f32(float *x, int64_t n, float v, hipStream_t st);
void launch_axpy_f64(int n, double a, const double *x, double *y, hipStream_t st);
void launch_copy_f64(int n, const double *x, double *y, hipStream_t st);

// ---- Krylov (a8, a9)
// Reductions over n rows use krylov_blocks(n) row chunks of at most
// kKrylovChunk rows; chunk sums are stored as partial[i * nblk + chunk].
constexpr int kKrylovThreads = 512;
constexpr int kKrylovWaves = kKrylovThreads / 64;
constexpr int kKrylovChunk = 2048;
constexpr int kMaxKrylovCols = 64;
inline int krylov_blocks(int n) { return std::max(256, (n + kKrylovChunk - 1) / kKrylovChunk); }
// h[i] = V[:, i]^T w, i < k <= kMaxKrylovCols (V column-major, leading dimension
// ldv); partial holds krylov_blocks(n) * k doubles
void launch_kdot(int n, const double *V, int64_t ldv, int k, const double *w, double *partial,
                 double *h, hipStream_t st);
// Orthogonalisation of Arnoldi step j (k = j + 1 basis vectors V) by classical
// Gram-Schmidt applied twice (twice) or once, and its Givens column, in four
// launches (three for one pass): h1 = V^T w; w -= V h1; [h2 = V^T w; w -= V h2;
// h1 += h2;]
// H[:, j] = h1, H[j + 1, j] = |w|, previous rotations then a new one on H[:, j]
// and g; flags[0] = |g[j + 1]|, flags[1] = breakdown, scal[0] = |w|;
// v_next = w / |w| (untouched when |w| == 0).  partial holds
// 2 * krylov_blocks(n) * kMaxKrylovCols doubles, npart krylov_blocks(n).
// host_out (device address of host-coherent pinned memory, or NULL): flags[0],
// flags[1] are written to host_out[0..1], then host_out[2] = 1 (ready).
void launch_arnoldi_orth(int n, const double *V, int64_t ldv, int k, double *w, double *partial,
                         double *h1, double *npart, double *v_next, double *H, int ldh, int j,
                         double *cs, double *sn, double *g, double *flags, double *scal,
                         double *host_out, hipStream_t st, bool twice = true);
// y = H^{-1} g (upper triangular k x k), then x += Z y
void launch_backsolve(const double *H, int ldh, const double *g, int k, double *y, hipStream_t st);
void launch_zupdate(int n, const double *Z, int64_t ldz, int k, const double *y, double *x,
                    hipStream_t st);
// v = r / beta with beta = sqrt(nrm2[0]); g = [beta, 0...]
void launch_start_cycle(int n, const double *r, const double *nrm2, double *v, double *g, int m,
                        hipStream_t st);

}  // namespace fsi

namespace fsi {
// the F x F block (see CoarseSplit), dense row-major with leading dimension
// ld, from CSR (zero-filled beforehand)
void launch_csr_to_dense(const CsrView<double> &A, const int *fpos, double *dense, int64_t ld,
                         hipStream_t st);
}  // namespace fsi
