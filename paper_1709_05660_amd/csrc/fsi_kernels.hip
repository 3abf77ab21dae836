// gfx950 kernels of the FSI multigrid/FGMRES hot path.
//
// Memory-bound steps (SpMV residuals, transfers, Schwarz applications,
// coarsest solve, Krylov vector work) are written for coalesced HBM access
// with 64-wide wavefronts.  The dense inversions of the setup live in
// fsi_gj.hip.
#include "fsi_kernels.h"

#include <hip/hip_bf16.h>
#include <hip/hip_ext.h>
#include <hip/hip_fp16.h>

#include <algorithm>
#include <mutex>
#include <type_traits>
#include <cmath>

namespace fsi {

static inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// ------------------------------------------------------------------ SpMV
// Sum over a group of LPR consecutive lanes, the total in every lane of the
// group: DPP within rows of 16 lanes (quad swaps, then the half-row and row
// mirrors), cross-lane shuffles only for groups of 32 and 64.
template <typename T, int LPR>
__device__ __forceinline__ T group_sum(T v) {
  auto dpp = [](T x, auto ctrl) {
    if constexpr (sizeof(T) == 8) {
      const long long b = __double_as_longlong(x);
      const int lo = __builtin_amdgcn_update_dpp((int)b, (int)b, decltype(ctrl)::value, 0xF, 0xF, false);
      const int hi = __builtin_amdgcn_update_dpp((int)(b >> 32), (int)(b >> 32), decltype(ctrl)::value, 0xF, 0xF, false);
      return (T)__longlong_as_double(((long long)hi << 32) | (unsigned)lo);
    } else {
      return (T)__int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(x), __float_as_int(x),
                                                            decltype(ctrl)::value, 0xF, 0xF, false));
    }
  };
  if constexpr (LPR >= 2) v += dpp(v, std::integral_constant<int, 0xB1>{});   // quad_perm [1,0,3,2]
  if constexpr (LPR >= 4) v += dpp(v, std::integral_constant<int, 0x4E>{});   // quad_perm [2,3,0,1]
  if constexpr (LPR >= 8) v += dpp(v, std::integral_constant<int, 0x141>{});  // row_half_mirror
  if constexpr (LPR >= 16) v += dpp(v, std::integral_constant<int, 0x140>{}); // row_mirror
  if constexpr (LPR >= 32) v += __shfl_xor(v, 16, 64);
  if constexpr (LPR >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

// LPR lanes per row; each lane takes the row's entries lane, lane + LPR, ...
// four at a time (their column and value loads issued together), summing
// in the same order as a one-at-a-time loop.  Whole rows leave together, so
// every group reduces with all its lanes active.
// blk: the workgroup's index among the operator's own workgroups (256 threads)
template <typename T, int LPR>
__device__ __forceinline__ void spmv_body(int blk, int nrows, const int *__restrict__ rowptr,
                                          const int *__restrict__ col, const T *__restrict__ val,
                                          const T *__restrict__ x, const T *__restrict__ r,
                                          T *__restrict__ y, int mode) {
  const int gid = blk * 256 + threadIdx.x;
  const int row = gid / LPR;
  const int lane = gid % LPR;
  const bool live = row < nrows;
  T acc = 0;
  if (live) {
    const int beg = rowptr[row], end = rowptr[row + 1];
    int p = beg + lane;
    for (; p + 3 * LPR < end; p += 4 * LPR) {
      const int c0 = col[p], c1 = col[p + LPR], c2 = col[p + 2 * LPR], c3 = col[p + 3 * LPR];
      const T v0 = val[p], v1 = val[p + LPR], v2 = val[p + 2 * LPR], v3 = val[p + 3 * LPR];
      acc += v0 * x[c0];
      acc += v1 * x[c1];
      acc += v2 * x[c2];
      acc += v3 * x[c3];
    }
    for (; p < end; p += LPR) acc += val[p] * x[col[p]];
  }
  acc = group_sum<T, LPR>(acc);
  if (live && lane == 0) {
    if (mode == kSpmvSet)
      y[row] = acc;
    else if (mode == kSpmvResid)
      y[row] = r[row] - acc;
    else
      y[row] += acc;
  }
}
template <typename T, int LPR>
__global__ __launch_bounds__(256) void k_spmv(int nrows, const int *__restrict__ rowptr,
                                              const int *__restrict__ col,
                                              const T *__restrict__ val, const T *__restrict__ x,
                                              const T *__restrict__ r, T *__restrict__ y,
                                              int mode) {
  spmv_body<T, LPR>(blockIdx.x, nrows, rowptr, col, val, x, r, y, mode);
}

// the batch entry of workgroup b: blk0[s] <= b < blk0[s + 1] (count <= kMaxBatch)
__device__ __forceinline__ int batch_entry(const int *blk0, int count, int b) {
  int s = 0;
  while (s + 1 < count && blk0[s + 1] <= b) ++s;
  return s;
}

// one operator per entry of the batch, each on its own workgroups
template <typename T, int LPR>
__global__ __launch_bounds__(256) void k_spmv_batch(SpmvBatch<T> B) {
  const int s = batch_entry(B.blk0, B.count, blockIdx.x);
  const SpmvItem<T> &it = B.it[s];
  spmv_body<T, LPR>(blockIdx.x - B.blk0[s], it.A.nrows, it.A.rowptr, it.A.col, it.A.val, it.x, it.r,
                    it.y, B.mode);
}

template <typename T>
void launch_spmv_batch(const SpmvItem<T> *items, const int *lpr, int count, int mode, hipStream_t st) {
  for (int L : {2, 4, 8, 16, 32, 64}) {
    SpmvBatch<T> B;
    B.mode = mode;
    B.count = 0;
    B.blk0[0] = 0;
    auto flush = [&] {
      if (B.count == 0 || B.blk0[B.count] == 0) {
        B.count = 0;
        return;
      }
      const int grid = B.blk0[B.count];
#define FSI_SPMVB_CASE(LL) \
  case LL:                 \
    k_spmv_batch<T, LL><<<grid, 256, 0, st>>>(B); break;
      switch (L) {
        FSI_SPMVB_CASE(2)
        FSI_SPMVB_CASE(4)
        FSI_SPMVB_CASE(8)
        FSI_SPMVB_CASE(16)
        FSI_SPMVB_CASE(32)
        FSI_SPMVB_CASE(64)
      }
#undef FSI_SPMVB_CASE
      B.count = 0;
    };
    for (int i = 0; i < count; ++i) {
      // the single launch's lanes per row (unknown values run with 8, as there)
      const int li = (lpr[i] == 2 || lpr[i] == 4 || lpr[i] == 16 || lpr[i] == 32 || lpr[i] == 64) ? lpr[i] : 8;
      if (li != L || items[i].A.nrows == 0) continue;
      B.it[B.count] = items[i];
      B.blk0[B.count + 1] = B.blk0[B.count] + cdiv((int64_t)items[i].A.nrows * L, 256);
      if (++B.count == kMaxBatch) flush();
    }
    flush();
  }
}
template void launch_spmv_batch<double>(const SpmvItem<double> *, const int *, int, int, hipStream_t);
template void launch_spmv_batch<float>(const SpmvItem<float> *, const int *, int, int, hipStream_t);

template <typename T>
void launch_spmv(const CsrView<T> &A, const T *x, const T *r, T *y, int mode, int lpr,
                 hipStream_t st) {
  if (A.nrows == 0) return;
  const int64_t threads = (int64_t)A.nrows * lpr;
  const int grid = cdiv(threads, 256);
#define FSI_SPMV_CASE(L) \
  case L:                \
    k_spmv<T, L><<<grid, 256, 0, st>>>(A.nrows, A.rowptr, A.col, A.val, x, r, y, mode); break;
  switch (lpr) {
    FSI_SPMV_CASE(2)
    FSI_SPMV_CASE(4)
    FSI_SPMV_CASE(8)
    FSI_SPMV_CASE(16)
    FSI_SPMV_CASE(32)
    FSI_SPMV_CASE(64)
    default:
      k_spmv<T, 8><<<cdiv((int64_t)A.nrows * 8, 256), 256, 0, st>>>(A.nrows, A.rowptr, A.col,
                                                                      A.val, x, r, y, mode);
  }
#undef FSI_SPMV_CASE
}
template void launch_spmv<double>(const CsrView<double> &, const double *, const double *,
                                  double *, int, int, hipStream_t);
template void launch_spmv<float>(const CsrView<float> &, const float *, const float *, float *,
                                 int, int, hipStream_t);

// ------------------------------------------------------------------ fills / casts
__global__ void k_fill_f64(double *x, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}
__global__ void k_fill_f32(float *x, int64_t n, float v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}
void launch_fill_f64(double *x, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return;
  k_fill_f64<<<std::min<int64_t>(cdiv(n, 256), 4096), 256, 0, st>>>(x, n, v);
}
void launch_fill_f32(float *x, int64_t n, float v, hipStream_t st) {
  if (n <= 0) return;
  k_fill_f32<<<std::min<int64_t>(cdiv(n, 256), 4096), 256, 0, st>>>(x, n, v);
}
__global__ void k_cast_d2f(const double *x, float *y, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (float)x[i];
}
__global__ void k_cast_f2d(const float *x, double *y, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (double)x[i];
}
// elementwise conversions of a batch of vectors (256 entries per workgroup)
template <typename A, typename Bt>
__global__ __launch_bounds__(256) void k_cast_batch(CastBatch<A, Bt> B) {
  const int s = batch_entry(B.blk0, B.count, blockIdx.x);
  const int i = (blockIdx.x - B.blk0[s]) * 256 + threadIdx.x;
  if (i < B.it[s].n) B.it[s].y[i] = (Bt)B.it[s].x[i];
}
template <typename A, typename Bt>
void launch_cast_batch(const CastItem<A, Bt> *items, int count, hipStream_t st) {
  CastBatch<A, Bt> B;
  B.count = 0;
  B.blk0[0] = 0;
  auto flush = [&] {
    if (B.count && B.blk0[B.count]) k_cast_batch<A, Bt><<<B.blk0[B.count], 256, 0, st>>>(B);
    B.count = 0;
  };
  for (int i = 0; i < count; ++i) {
    if (items[i].n <= 0) continue;
    B.it[B.count] = items[i];
    B.blk0[B.count + 1] = B.blk0[B.count] + cdiv(items[i].n, 256);
    if (++B.count == kMaxBatch) flush();
  }
  flush();
}
template void launch_cast_batch<double, float>(const CastItem<double, float> *, int, hipStream_t);
template void launch_cast_batch<float, double>(const CastItem<float, double> *, int, hipStream_t);

void launch_cast_d2f(const double *x, float *y, int n, hipStream_t st) {
  if (n > 0) k_cast_d2f<<<cdiv(n, 256), 256, 0, st>>>(x, y, n);
}
void launch_cast_f2d(const float *x, double *y, int n, hipStream_t st) {
  if (n > 0) k_cast_f2d<<<cdiv(n, 256), 256, 0, st>>>(x, y, n);
}
__global__ void k_axpy_f64(int n, double a, const double *x, double *y) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += a * x[i];
}
__global__ void k_copy_f64(int n, const double *x, double *y) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i];
}
void launch_axpy_f64(int n, double a, const double *x, double *y, hipStream_t st) {
  if (n > 0) k_axpy_f64<<<cdiv(n, 256), 256, 0, st>>>(n, a, x, y);
}
void launch_copy_f64(int n, const double *x, double *y, hipStream_t st) {
  if (n > 0) k_copy_f64<<<cdiv(n, 256), 256, 0, st>>>(n, x, y);
}

// ------------------------------------------------------------------ block extraction
// Extraction map, built once at setup: one wave per (patch, local row); each
// slot (one CSR entry of the row, slots of row t from slot_off[t]) records the
// entry's index and its position in the level's blocks, found by a binary
// search of its column in the sorted dof list, or -1 outside the patch.
__global__ __launch_bounds__(256) void k_extract_map(int nrows_total, const int *__restrict__ row_patch,
                                                     const int *__restrict__ row_local,
                                                     const int *__restrict__ pm,
                                                     const int64_t *__restrict__ pdof_off,
                                                     const int *__restrict__ dof,
                                                     const int64_t *__restrict__ boff,
                                                     const int *__restrict__ rowptr,
                                                     const int *__restrict__ col,
                                                     const int64_t *__restrict__ slot_off,
                                                     int *__restrict__ src, int *__restrict__ dst) {
  const int t = blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (t >= nrows_total) return;
  const int k = row_patch[t];
  const int i = row_local[t];
  const int m = pm[k];
  const int *d = dof + pdof_off[k];
  const int g = d[i];
  const int64_t base = boff[k] + (int64_t)i * m;
  const int64_t s0 = slot_off[t];
  for (int p = rowptr[g] + lane; p < rowptr[g + 1]; p += 64) {
    const int c = col[p];
    int lo = 0, hi = m - 1, at = -1;
    while (lo <= hi) {
      const int mid = (lo + hi) >> 1;
      const int v = d[mid];
      if (v == c) {
        at = mid;
        break;
      }
      if (v < c)
        lo = mid + 1;
      else
        hi = mid - 1;
    }
    src[s0 + (p - rowptr[g])] = p;
    dst[s0 + (p - rowptr[g])] = at < 0 ? -1 : (int)(base + at);
  }
}

void launch_extract_map(const CsrView<double> &J, const int *pm, const int64_t *pdof_off,
                        const int *dof, const int64_t *boff, int64_t total_rows,
                        const int *row_patch, const int *row_local, const int64_t *slot_off,
                        int *src, int *dst, hipStream_t st) {
  if (total_rows == 0) return;
  k_extract_map<<<cdiv(total_rows, 4), 256, 0, st>>>((int)total_rows, row_patch, row_local, pm,
                                                      pdof_off, dof, boff, J.rowptr, J.col,
                                                      slot_off, src, dst);
}

// B_k = J[I_k, I_k]: one thread per slot of the map (FP32 blocks: the values
// rounded to single precision, the working matrices of the mixed forms)
template <typename TB>
__global__ __launch_bounds__(256) void k_extract(int64_t nslots, const int *__restrict__ src,
                                                 const int *__restrict__ dst,
                                                 const double *__restrict__ val,
                                                 TB *__restrict__ blocks) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nslots) return;
  const int q = dst[e];
  if (q >= 0) blocks[q] = (TB)val[src[e]];
}

void launch_extract(const double *val, int64_t nslots, const int *src, const int *dst,
                    double *blocks, hipStream_t st) {
  if (nslots == 0) return;
  k_extract<<<(unsigned)((nslots + 255) / 256), 256, 0, st>>>(nslots, src, dst, val, blocks);
}
void launch_extract(const double *val, int64_t nslots, const int *src, const int *dst,
                    float *blocks, hipStream_t st) {
  if (nslots == 0) return;
  k_extract<<<(unsigned)((nslots + 255) / 256), 256, 0, st>>>(nslots, src, dst, val, blocks);
}

// ------------------------------------------------------------------ packing of owned rows
__device__ inline uint16_t to_bf16(float f) {
  __hip_bfloat16 h = __float2bfloat16(f);
  return *reinterpret_cast<uint16_t *>(&h);
}
__device__ inline uint16_t to_fp16(float f) {
  __half h = __float2half(f);
  return *reinterpret_cast<uint16_t *>(&h);
}
__device__ inline float from_bf16(uint16_t u) {
  return __uint_as_float(((uint32_t)u) << 16);
}
__device__ inline float from_fp16(uint16_t u) {
  __half h = *reinterpret_cast<__half *>(&u);
  return __half2float(h);
}

// The Gauss-Jordan result S holds every block inverse up to its pivot
// permutations: Binv[i][c] = S[perm[i]][used[c]], equivalently physical
// column p of S is logical column perm[p] (per-patch arrays at pdof_off[k]).

// Column scales of the owned rows of every block inverse (16-bit storage):
// cs[c] = max over owned rows r of |Binv[r][c]| (cscale zeroed beforehand).
// One workgroup per (patch, 64 owned rows): the rows are read contiguously,
// the maxima meet in LDS (float bit patterns order like the non-negative
// values) and then in cscale.
template <typename TB>
__global__ __launch_bounds__(256) void k_colscale(const TB *__restrict__ blocks,
                                                  const int64_t *__restrict__ boff,
                                                  const int *__restrict__ pm,
                                                  const int *__restrict__ po,
                                                  const int *__restrict__ own_off,
                                                  const int *__restrict__ own_local,
                                                  const int64_t *__restrict__ pdof_off,
                                                  const int *__restrict__ task_patch,
                                                  const int *__restrict__ task_row0, float *cscale,
                                                  const int *__restrict__ perm) {
  extern __shared__ unsigned cmax[];   // the largest block's columns (sized at launch)
  const int k = task_patch[blockIdx.x], r0 = task_row0[blockIdx.x];
  const int m = pm[k], nr = min(64, po[k] - r0);
  const int *pk = perm + pdof_off[k];
  const TB *B = blocks + boff[k];
  for (int c = threadIdx.x; c < m; c += blockDim.x) cmax[c] = 0u;
  __syncthreads();
  for (int r = 0; r < nr; ++r) {
    const TB *row = B + (int64_t)pk[own_local[own_off[k] + r0 + r]] * m;
    for (int p = threadIdx.x; p < m; p += blockDim.x)
      atomicMax(&cmax[pk[p]], __float_as_uint((float)fabs((double)row[p])));
  }
  __syncthreads();
  for (int c = threadIdx.x; c < m; c += blockDim.x)
    atomicMax(reinterpret_cast<unsigned *>(cscale + pdof_off[k]) + c, cmax[c]);
}
// columns with no nonzero owned entry get scale 1
__global__ void k_scale_fix(float *cs, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n && !(cs[i] > 0.0f)) cs[i] = 1.0f;
}
template <typename TB>
void launch_colscale(const TB *blocks, const int64_t *boff, const int *pm, const int *po,
                     const int *own_off, const int *own_local, const int64_t *pdof_off,
                     const int *task_patch, const int *task_row0, int ntask, int64_t total_cols,
                     float *cscale, const int *perm, int mmax, hipStream_t st, bool first, bool last) {
  if (first) launch_fill_f32(cscale, total_cols, 0.0f, st);
  if (ntask)
    k_colscale<<<ntask, 256, sizeof(unsigned) * mmax, st>>>(blocks, boff, pm, po, own_off, own_local, pdof_off,
                                                            task_patch, task_row0, cscale, perm);
  if (last) k_scale_fix<<<cdiv(total_cols, 256), 256, 0, st>>>(cscale, total_cols);
}

// Owned rows of Binv_k in task-contiguous column-major order: the rows of
// task (k, r0) (nr = min(64, o - r0) rows) occupy W_k[r0 m ...], entry (c, r)
// at W_k[r0 m + c nr + r - r0], so one Schwarz workgroup streams one
// contiguous region.  One workgroup per (patch, 64 owned rows), 64 physical
// columns p of S at a time: the
// rows' segments are read in order into an LDS tile, and column p is written
// to logical column c = perm[p] with consecutive owned rows in consecutive
// lanes, so both the reads and the stores are contiguous.  16-bit storage:
// row r is stored divided by cs[c] and by its row scale, the largest
// |Binv[r][c]| / cs[c] of the row.
template <typename TB>
__global__ __launch_bounds__(256) void k_pack_owned(const TB *__restrict__ blocks,
                                                    const int64_t *__restrict__ boff,
                                                    const int *__restrict__ pm,
                                                    const int *__restrict__ po,
                                                    const int64_t *__restrict__ woff,
                                                    const int *__restrict__ own_off,
                                                    const int *__restrict__ own_local,
                                                    const int *__restrict__ task_patch,
                                                    const int *__restrict__ task_row0, double *W64,
                                                    float *W32, uint16_t *W16, int w16_kind,
                                                    float *wscale, const int64_t *__restrict__ pdof_off,
                                                    const float *__restrict__ cscale,
                                                    const int *__restrict__ perm,
                                                    const int64_t *__restrict__ woff16) {
  __shared__ double tile[64][65];
  __shared__ int64_t rowoff[64];
  __shared__ double rsc[64];
  const int k = task_patch[blockIdx.x], r0 = task_row0[blockIdx.x];
  const int m = pm[k], o = po[k], nr = min(64, o - r0);
  const int *pk = perm + pdof_off[k];
  const TB *B = blocks + boff[k];
  const float *cs = W16 ? cscale + pdof_off[k] : nullptr;
  const int tid = threadIdx.x;
  if (tid < 64) rowoff[tid] = tid < nr ? (int64_t)pk[own_local[own_off[k] + r0 + tid]] * m : 0;
  __syncthreads();
  if (W16) {
    const int r = tid >> 2, sub = tid & 3;   // 4 threads per row
    double mx = 0.0;
    if (r < nr) {
#pragma unroll 8
      for (int p = sub; p < m; p += 4) mx = fmax(mx, fabs((double)B[rowoff[r] + p]) / (double)cs[pk[p]]);
    }
    mx = fmax(mx, __shfl_xor(mx, 1, 4));
    mx = fmax(mx, __shfl_xor(mx, 2, 4));
    if (mx == 0.0) mx = 1.0;
    if (sub == 0 && r < nr) {
      rsc[r] = mx;
      wscale[own_off[k] + r0 + r] = (float)mx;
    }
    __syncthreads();
  }
  const int64_t wk = woff[k] + (int64_t)r0 * m;
  const int m4 = (m + 3) & ~3;
  const int64_t wk16 = woff16 ? woff16[k] + (int64_t)r0 * m4 : 0;
  for (int q0 = 0; q0 < m; q0 += 64) {
    // all 16 loads of a thread in flight together; clamped addresses (the
    // entries past the block are never stored)
    double vals[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int idx = tid + 256 * u;
      vals[u] = (double)B[rowoff[min(idx >> 6, nr - 1)] + min(q0 + (idx & 63), m - 1)];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int idx = tid + 256 * u;
      tile[idx >> 6][idx & 63] = vals[u];
    }
    __syncthreads();
    for (int idx = tid; idx < 64 * 64; idx += 256) {
      const int p = idx >> 6, r = idx & 63;
      if (r < nr && q0 + p < m) {
        const int c = pk[q0 + p];
        const double v = tile[r][p];
        const int64_t dst = wk + (int64_t)c * nr + r;
        if (W64) W64[dst] = v;
        if (W32) W32[dst] = (float)v;
        if (W16) {
          const float q = (float)(v / ((double)cs[c] * rsc[r]));
          const int64_t d16 = woff16 ? wk16 + (int64_t)(c >> 2) * (nr * 4) + r * 4 + (c & 3) : dst;
          W16[d16] = w16_kind == 1 ? to_bf16(q) : to_fp16(q);
        }
      }
    }
    __syncthreads();
  }
}
template <typename TB>
void launch_pack_owned(const TB *blocks, const int64_t *boff, const int *pm, const int *po,
                       const int64_t *woff, const int *own_off, const int *own_local,
                       const int *task_patch, const int *task_row0, int ntask, double *W64,
                       float *W32, uint16_t *W16, int w16_kind, float *wscale,
                       const int64_t *pdof_off, const float *cscale, const int *perm,
                       const int64_t *woff16, hipStream_t st) {
  if (ntask == 0) return;
  k_pack_owned<<<ntask, 256, 0, st>>>(blocks, boff, pm, po, woff, own_off, own_local, task_patch,
                                      task_row0, W64, W32, W16, w16_kind, wscale, pdof_off, cscale,
                                      perm, woff16);
}
#define FSI_PACK_INST(TB)                                                                            \
  template void launch_colscale<TB>(const TB *, const int64_t *, const int *, const int *, const int *, \
                                    const int *, const int64_t *, const int *, const int *, int,       \
                                    int64_t, float *, const int *, int, hipStream_t, bool, bool);      \
  template void launch_pack_owned<TB>(const TB *, const int64_t *, const int *, const int *,           \
                                      const int64_t *, const int *, const int *, const int *,          \
                                      const int *, int, double *, float *, uint16_t *, int, float *,   \
                                      const int64_t *, const float *, const int *, const int64_t *,    \
                                      hipStream_t);
FSI_PACK_INST(double)
FSI_PACK_INST(float)
#undef FSI_PACK_INST

// ------------------------------------------------------------------ restricted Schwarz
// One workgroup per (patch, 64 owned rows).  The patch's residual entries
// are gathered once into LDS; each of the NWV waves accumulates its share
// of the columns of the task's owned rows of B_k^{-1} (stored column-major
// per task, so the workgroup's rows are one contiguous region and one step
// over a column is one coalesced load of the task's rows, eight loads in
// flight per lane), the partial sums meet in LDS and lane r of the first
// wave adds omega times row r to its owned dof (or stores it, when add is 0:
// a zero initial correction; the workgroups then also clear the dofs no patch
// owns, a slice each).  Levels with few tasks use more waves per
// workgroup (a shorter chain of loads per wave).  TAG only names the
// finest-level launch.
__device__ inline float w16val(uint16_t v, int kind) {
  return kind == 1 ? from_bf16(v) : from_fp16(v);
}

template <typename WT, typename AT, bool IS16>
__device__ inline AT wload(const WT *w, int64_t idx, int kind) {
  if constexpr (IS16)
    return (AT)w16val(w[idx], kind);
  else
    return (AT)w[idx];
}

// 16-bit storage: four consecutive columns of a row sit side by side (group
// g = c / 4 of a task holds its nr rows x 4 columns row by row, columns padded
// with zeros to a multiple of 4), so each lane loads 8 bytes per group and one
// wave load is 512 contiguous bytes; CH groups (4 CH columns) in flight per
// lane, one chunk ahead (16 groups measured slower than 8: 17.0 against
// 15.2 us on the 2D finest level).  KIND 1: bf16, 2: fp16.
template <int KIND>
__device__ __forceinline__ float4 w16x4(uint2 q) {
  if constexpr (KIND == 1)
    return make_float4(__uint_as_float(q.x << 16), __uint_as_float(q.x & 0xffff0000u),
                       __uint_as_float(q.y << 16), __uint_as_float(q.y & 0xffff0000u));
  else
    return make_float4(from_fp16((uint16_t)(q.x & 0xffffu)), from_fp16((uint16_t)(q.x >> 16)),
                       from_fp16((uint16_t)(q.y & 0xffffu)), from_fp16((uint16_t)(q.y >> 16)));
}
template <int KIND, int NWV, int CH = 8>
__device__ __forceinline__ void ras_body16(int task, const RasView &v, const uint16_t *__restrict__ W,
                                           const float *__restrict__ wscale, const float *__restrict__ s,
                                           float *__restrict__ e, float omega, int add) {
  extern __shared__ __align__(16) unsigned char ras_lds[];
  float *xs = reinterpret_cast<float *>(ras_lds);   // the patch's m4 columns (sized at launch)
  __shared__ float red[NWV - 1][64];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int k = v.task_patch[task];
  const int r0 = v.task_row0[task];
  const int m = v.pm[k], o = v.po[k];
  const int m4 = (m + 3) & ~3, ng = m4 >> 2;
  const int *d = v.dof + v.pdof_off[k];
  const int row = r0 + lane;
  const bool live = row < o;
  const int share = (ng + NWV - 1) / NWV;
  const int g0 = wave * share, g1 = min(ng, g0 + share);
  const int nr = min(64, o - r0);
  const uint2 *w = reinterpret_cast<const uint2 *>(W + v.woff[k] + (int64_t)r0 * m4) + (live ? lane : nr - 1);
  // clamped to the wave's own last group: the prefetch past the end of the
  // range re-reads that group (cached) instead of the next wave's columns
  const int glast = max(g1 - 1, 0);
  auto loadc = [&](int g, uint2(&wv)[CH]) {
#pragma unroll
    for (int u = 0; u < CH; ++u) wv[u] = w[(int64_t)min(g + u, glast) * nr];
  };
  uint2 cur[CH];
  loadc(min(g0, glast), cur);
  const float *cs = v.cscale + v.pdof_off[k];
  for (int c = threadIdx.x; c < m4; c += 64 * NWV) xs[c] = c < m ? s[d[c]] * cs[c] : 0.0f;
  if (!add)
    for (int i = task * 64 * NWV + threadIdx.x; i < v.nunowned; i += v.ntask * 64 * NWV) e[v.unowned[i]] = 0.0f;
  __syncthreads();
  float a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  auto fma4 = [&](float &acc, uint2 q, int g) {
    const float4 wv = w16x4<KIND>(q);
    const float4 x = *reinterpret_cast<const float4 *>(&xs[4 * g]);
    acc += (wv.x * x.x + wv.y * x.y) + (wv.z * x.z + wv.w * x.w);
  };
  int g = g0;
  for (; g + CH <= g1; g += CH) {
    uint2 nxt[CH];
    loadc(g + CH, nxt);
#pragma unroll
    for (int u = 0; u < CH; ++u) fma4(a[u & 7], cur[u], g + u);
#pragma unroll
    for (int u = 0; u < CH; ++u) cur[u] = nxt[u];
  }
  // the last partial chunk (already loaded in cur), in group order; unrolled
  // with a predicate so that cur stays in registers
#pragma unroll
  for (int u = 0; u < CH; ++u)
    if (g + u < g1) fma4(a[0], cur[u], g + u);
  float acc = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  if (wave > 0) red[wave - 1][lane] = acc;
  __syncthreads();
  if (wave == 0 && live) {
#pragma unroll
    for (int q = 0; q < NWV - 1; ++q) acc += red[q][lane];
    acc *= wscale[v.out_off[k] + row];
    const int gd = v.out_idx[v.out_off[k] + row];
    const float upd = omega * acc;
    e[gd] = add ? e[gd] + upd : upd;
  }
}

// task: the workgroup's task of v (v.ntask workgroups per operator); FP64 or
// FP32 storage (16-bit storage: ras_body16)
template <typename WT, typename VT, typename AT, bool IS16, int NWV>
__device__ __forceinline__ void ras_body(int task, const RasView &v, const WT *__restrict__ W,
                                         int w16_kind, const float *__restrict__ wscale,
                                         const VT *__restrict__ s, VT *__restrict__ e, AT omega,
                                         int add) {
  extern __shared__ __align__(16) unsigned char ras_lds[];
  AT *xs = reinterpret_cast<AT *>(ras_lds);   // the patch's m columns (sized at launch)
  __shared__ AT red[NWV - 1][64];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int k = v.task_patch[task];
  const int r0 = v.task_row0[task];
  const int m = v.pm[k], o = v.po[k];
  const int *d = v.dof + v.pdof_off[k];
  const int row = r0 + lane;
  const bool live = row < o;
  const int share = (m + NWV - 1) / NWV;
  const int c0 = wave * share, c1 = min(m, c0 + share);
  // this wave's columns stream 8 at a time, one chunk ahead of the one being
  // summed; the first chunk is issued before the residual gather so that no
  // workgroup starts with an idle memory pipe.  Addresses are clamped to the
  // wave's own last column (never summed twice): the prefetch past the end of
  // the range re-reads that cached column instead of fetching the next wave's
  // columns a second time
  const int nr = min(64, o - r0);
  const WT *w = W + v.woff[k] + (int64_t)r0 * m + (live ? lane : nr - 1);
  const int clast = max(c1 - 1, 0);
  auto load8 = [&](int c, AT(&wv)[8]) {
#pragma unroll
    for (int u = 0; u < 8; ++u) wv[u] = wload<WT, AT, IS16>(w, (int64_t)min(c + u, clast) * nr, w16_kind);
  };
  AT cur[8];
  load8(min(c0, clast), cur);
  for (int c = threadIdx.x; c < m; c += 64 * NWV) xs[c] = (AT)s[d[c]];
  if (!add)
    for (int i = task * 64 * NWV + threadIdx.x; i < v.nunowned; i += v.ntask * 64 * NWV)
      e[v.unowned[i]] = (VT)0;
  __syncthreads();
  AT a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int c = c0;
  for (; c + 8 <= c1; c += 8) {
    AT nxt[8];
    load8(c + 8, nxt);
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += cur[u] * xs[c + u];
#pragma unroll
    for (int u = 0; u < 8; ++u) cur[u] = nxt[u];
  }
  // the last partial chunk (already loaded in cur), in column order
  for (int u = 0; c + u < c1; ++u) a[0] += cur[u] * xs[c + u];
  AT acc = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  if (wave > 0) red[wave - 1][lane] = acc;
  __syncthreads();
  if (wave == 0 && live) {
#pragma unroll
    for (int q = 0; q < NWV - 1; ++q) acc += red[q][lane];
    const int g = v.out_idx[v.out_off[k] + row];
    const VT upd = (VT)(omega * acc);
    e[g] = add ? e[g] + upd : upd;
  }
}
template <typename WT, typename VT, typename AT, bool IS16, int TAG, int NWV>
__global__ __launch_bounds__(64 * NWV) void k_ras(RasView v, const WT *__restrict__ W,
                                                  int w16_kind, const float *__restrict__ wscale,
                                                  const VT *__restrict__ s,
                                                  VT *__restrict__ e, AT omega, int add) {
  if constexpr (IS16) {
    if (w16_kind == 1)
      ras_body16<1, NWV>(blockIdx.x, v, W, wscale, s, e, omega, add);
    else
      ras_body16<2, NWV>(blockIdx.x, v, W, wscale, s, e, omega, add);
  } else {
    ras_body<WT, VT, AT, IS16, NWV>(blockIdx.x, v, W, w16_kind, wscale, s, e, omega, add);
  }
}
// the Schwarz steps of a batch of systems (one level each), each on its own tasks
template <typename WT, typename VT, typename AT, bool IS16, int NWV>
__global__ __launch_bounds__(64 * NWV) void k_ras_batch(RasBatch<WT, VT> B, AT omega, int add) {
  const int s = batch_entry(B.blk0, B.count, blockIdx.x);
  const RasItem<WT, VT> &it = B.it[s];
  if constexpr (IS16) {
    if (it.w16_kind == 1)
      ras_body16<1, NWV>(blockIdx.x - B.blk0[s], it.v, it.W, it.wscale, it.s, it.e, omega, add);
    else
      ras_body16<2, NWV>(blockIdx.x - B.blk0[s], it.v, it.W, it.wscale, it.s, it.e, omega, add);
  } else {
    ras_body<WT, VT, AT, IS16, NWV>(blockIdx.x - B.blk0[s], it.v, it.W, it.w16_kind, it.wscale, it.s, it.e,
                                    omega, add);
  }
}

static int ras_waves(int ntask);

// out[q] = val[src[q]]: the refined blocks' entries of the FP32 operator
__global__ void k_gather_f32(const float *__restrict__ val, const int *__restrict__ src, int n,
                             float *__restrict__ out) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q < n) out[q] = val[src[q]];
}
void launch_gather_f32(const float *val, const int *src, int n, float *out, hipStream_t st) {
  if (n > 0) k_gather_f32<<<cdiv(n, 256), 256, 0, st>>>(val, src, n, out);
}
// Refined local solves of the solid blocks (see RefineView), with the work
// layout of k_ras: one workgroup per (block, 64 rows) task of every row of
// the stored inverse, NWV waves splitting its columns.  MODE 0: y_out = W~ g
// with g = s[I_k] (the first task of each block also keeps g).  MODE 1, a
// refinement sweep after the block SpMV rho = g - B y_in:
// y_out = y_in + W~ rho for its rows; the last sweep writes
// omega y_out to the owned dofs of e instead (stores when add is 0, and then
// also clears the dofs no patch owns).  16-bit storage: the gathered vector is
// multiplied by the column scales, each row's sum by its row scale.
template <typename WT, bool IS16, int NWV, int MODE>
__global__ __launch_bounds__(64 * NWV) void k_refine(RefineView v, const WT *__restrict__ W,
                                                     const float *__restrict__ s,
                                                     const float *__restrict__ y_in,
                                                     float *__restrict__ y_out, float *__restrict__ e,
                                                     float omega, int add, int last) {
  __shared__ float xs[kMaxPatch];
  __shared__ float red[NWV - 1][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int k = v.task_patch[blockIdx.x], r0 = v.task_row0[blockIdx.x];
  const int m = v.pm[k], fo = v.full_off[k];
  const int *d = v.dof + v.pdof_off[k];
  const int row = r0 + lane;
  const bool live = row < m;
  const int nr = min(64, m - r0);
  const int share = (m + NWV - 1) / NWV;
  const int c0 = wave * share, c1 = min(m, c0 + share);
  const WT *w = W + v.woff_full[k] + (int64_t)r0 * m + (live ? lane : nr - 1);
  auto load8 = [&](int c, float(&wv)[8]) {
#pragma unroll
    for (int u = 0; u < 8; ++u) wv[u] = wload<WT, float, IS16>(w, (int64_t)min(c + u, m - 1) * nr, v.w16_kind);
  };
  float cur[8];
  load8(min(c0, m - 1), cur);
  const float *cs = IS16 ? v.cscale + v.pdof_off[k] : nullptr;
  for (int c = threadIdx.x; c < m; c += 64 * NWV) {
    float g;
    if constexpr (MODE == 0) {
      g = s[d[c]];
      if (r0 == 0) v.gfull[fo + c] = g;   // the block's right-hand side, for the residual
    } else {
      g = v.rho[fo + c];                   // g - B_k y_in, from the block SpMV
    }
    xs[c] = IS16 ? g * cs[c] : g;
  }
  if (MODE == 1 && last && !add)
    for (int i = blockIdx.x * 64 * NWV + threadIdx.x; i < v.nunowned; i += gridDim.x * 64 * NWV)
      e[v.unowned[i]] = 0.0f;
  __syncthreads();
  float a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int c = c0;
  for (; c + 8 <= c1; c += 8) {
    float nxt[8];
    load8(c + 8, nxt);
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += cur[u] * xs[c + u];
#pragma unroll
    for (int u = 0; u < 8; ++u) cur[u] = nxt[u];
  }
  for (int u = 0; c + u < c1; ++u) a[0] += cur[u] * xs[c + u];
  float acc = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  if (wave > 0) red[wave - 1][lane] = acc;
  __syncthreads();
  if (wave == 0 && live) {
#pragma unroll
    for (int q = 0; q < NWV - 1; ++q) acc += red[q][lane];
    if constexpr (IS16) acc *= v.rscale[fo + row];
    if constexpr (MODE == 0) {
      y_out[fo + row] = acc;
    } else {
      const float yn = y_in[fo + row] + acc;
      if (!last) {
        y_out[fo + row] = yn;
      } else {
        const int gd = v.own_dof[fo + row];
        if (gd >= 0) e[gd] = add ? e[gd] + omega * yn : omega * yn;
      }
    }
  }
}

template <typename WT, bool IS16, int NWV>
static void refine_nw(const RefineView &v, const WT *W, const float *s, float *e, float omega, bool add,
                      int sweeps, float *y0, float *y1, hipStream_t st) {
  k_refine<WT, IS16, NWV, 0><<<v.ntask, 64 * NWV, 0, st>>>(v, W, s, nullptr, y0, e, omega, (int)add, 0);
  for (int sw = 0; sw < sweeps; ++sw) {
    launch_spmv(v.B, y0, v.gfull, v.rho, kSpmvResid, v.lpr, st);
    k_refine<WT, IS16, NWV, 1><<<v.ntask, 64 * NWV, 0, st>>>(v, W, s, y0, y1, e, omega, (int)add,
                                                            sw + 1 == sweeps);
    std::swap(y0, y1);
  }
}
template <typename WT, bool IS16>
static void refine_any(const RefineView &v, const WT *W, const float *s, float *e, float omega, bool add,
                       int sweeps, float *y0, float *y1, hipStream_t st) {
  switch (ras_waves(v.ntask)) {
    case 4: refine_nw<WT, IS16, 4>(v, W, s, e, omega, add, sweeps, y0, y1, st); break;
    case 8: refine_nw<WT, IS16, 8>(v, W, s, e, omega, add, sweeps, y0, y1, st); break;
    default: refine_nw<WT, IS16, 16>(v, W, s, e, omega, add, sweeps, y0, y1, st);
  }
}
void launch_ras_refine(const RefineView &v, const float *W32, const uint16_t *W16, const float *s, float *e,
                       float omega, bool add, int sweeps, float *y0, float *y1, hipStream_t st) {
  if (v.ntask == 0 || sweeps < 1) return;
  if (W16)
    refine_any<uint16_t, true>(v, W16, s, e, omega, add, sweeps, y0, y1, st);
  else
    refine_any<float, false>(v, W32, s, e, omega, add, sweeps, y0, y1, st);
}

// ev0/ev1 (optional, finest level): timing events recorded at the kernel's
// own start and end (hipExtLaunchKernelGGL), not around its launch
static int ras_waves(int ntask) { return ntask >= 1024 ? 4 : (ntask >= 256 ? 8 : 16); }

// dynamic LDS of a Schwarz launch: the gathered vector of the largest block
// (16-bit storage: padded to a multiple of 4 columns)
template <typename AT>
static size_t ras_lds_bytes(int mmax) {
  return sizeof(AT) * (size_t)((std::max(mmax, 1) + 3) & ~3);
}
template <typename WT, typename VT, typename AT, bool IS16, int NWV>
static void launch_ras_nw(const RasView &v, const WT *W, int w16_kind, const float *wscale,
                          const VT *s, VT *e, AT omega, bool finest, bool add, hipStream_t st,
                          hipEvent_t ev0, hipEvent_t ev1) {
  const size_t lds = ras_lds_bytes<AT>(v.mmax);
  if (finest)
    hipExtLaunchKernelGGL(k_ras<WT, VT, AT, IS16, 1, NWV>, dim3(v.ntask), dim3(64 * NWV), lds, st,
                          ev0, ev1, 0, v, W, w16_kind, wscale, s, e, omega, (int)add);
  else
    k_ras<WT, VT, AT, IS16, 0, NWV><<<v.ntask, 64 * NWV, lds, st>>>(v, W, w16_kind, wscale, s, e,
                                                                   omega, (int)add);
}
template <typename WT, typename VT, typename AT, bool IS16>
static void launch_ras_any(const RasView &v, const WT *W, int w16_kind, const float *wscale,
                           const VT *s, VT *e, AT omega, bool finest, bool add, hipStream_t st,
                           hipEvent_t ev0, hipEvent_t ev1) {
  if (v.ntask == 0) return;
  switch (ras_waves(v.ntask)) {
    case 4:
      launch_ras_nw<WT, VT, AT, IS16, 4>(v, W, w16_kind, wscale, s, e, omega, finest, add, st, ev0, ev1);
      break;
    case 8:
      launch_ras_nw<WT, VT, AT, IS16, 8>(v, W, w16_kind, wscale, s, e, omega, finest, add, st, ev0, ev1);
      break;
    default:
      launch_ras_nw<WT, VT, AT, IS16, 16>(v, W, w16_kind, wscale, s, e, omega, finest, add, st, ev0,
                                          ev1);
  }
}
void launch_ras_f64(const RasView &v, const double *W, const double *s, double *e, double omega,
                    bool finest, bool add, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  launch_ras_any<double, double, double, false>(v, W, 0, nullptr, s, e, omega, finest, add, st,
                                                ev0, ev1);
}
void launch_ras_f32(const RasView &v, const float *W, const float *s, float *e, float omega,
                    bool finest, bool add, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  launch_ras_any<float, float, float, false>(v, W, 0, nullptr, s, e, omega, finest, add, st, ev0,
                                             ev1);
}
void launch_ras_16(const RasView &v, const uint16_t *W, int w16_kind, const float *wscale,
                   const float *s, float *e, float omega, bool finest, bool add, hipStream_t st,
                   hipEvent_t ev0, hipEvent_t ev1) {
  launch_ras_any<uint16_t, float, float, true>(v, W, w16_kind, wscale, s, e, omega, finest, add,
                                               st, ev0, ev1);
}

// batched Schwarz steps: entries grouped by the waves per workgroup that a
// single launch of the same level would use (the same arithmetic per system)
template <typename WT, typename VT, typename AT, bool IS16>
static void launch_ras_batch_t(const RasItem<WT, VT> *items, int count, AT omega, bool add, hipStream_t st) {
  for (int nw : {4, 8, 16}) {
    RasBatch<WT, VT> B;
    B.count = 0;
    B.blk0[0] = 0;
    auto flush = [&] {
      const int grid = B.count ? B.blk0[B.count] : 0;
      if (grid > 0) {
        int mmax = 1;
        for (int q = 0; q < B.count; ++q) mmax = std::max(mmax, B.it[q].v.mmax);
        const size_t lds = ras_lds_bytes<AT>(mmax);
        if (nw == 4)
          k_ras_batch<WT, VT, AT, IS16, 4><<<grid, 256, lds, st>>>(B, omega, (int)add);
        else if (nw == 8)
          k_ras_batch<WT, VT, AT, IS16, 8><<<grid, 512, lds, st>>>(B, omega, (int)add);
        else
          k_ras_batch<WT, VT, AT, IS16, 16><<<grid, 1024, lds, st>>>(B, omega, (int)add);
      }
      B.count = 0;
    };
    for (int i = 0; i < count; ++i) {
      if (items[i].v.ntask == 0 || ras_waves(items[i].v.ntask) != nw) continue;
      B.it[B.count] = items[i];
      B.blk0[B.count + 1] = B.blk0[B.count] + items[i].v.ntask;
      if (++B.count == kMaxBatch) flush();
    }
    flush();
  }
}
void launch_ras_batch_f64(const RasItem<double, double> *items, int count, double omega, bool add,
                          hipStream_t st) {
  launch_ras_batch_t<double, double, double, false>(items, count, omega, add, st);
}
void launch_ras_batch_f32(const RasItem<float, float> *items, int count, float omega, bool add,
                          hipStream_t st) {
  launch_ras_batch_t<float, float, float, false>(items, count, omega, add, st);
}
void launch_ras_batch_16(const RasItem<uint16_t, float> *items, int count, float omega, bool add,
                         hipStream_t st) {
  launch_ras_batch_t<uint16_t, float, float, true>(items, count, omega, add, st);
}

// ------------------------------------------------------------------ ILU(0) of fluid blocks
// a failed attribute call must not leave its error for the next launch check
static inline void hip_ok_or_clear(hipError_t e) {
  if (e != hipSuccess) (void)hipGetLastError();
}

// Right-looking elimination on the dense block with the pattern as a mask,
// one workgroup per block: step k updates a_ij -= (a_ik / a_kk) a_kj at the
// pattern positions (i, j) with i, j > k, a_ik and a_kj in the pattern (the
// L rows of column k times the U columns of row k, spread over the
// threads), then scales the L column.  Every a_ij receives its updates in
// ascending k, the order of the row-by-row formulation.
template <typename T>
__global__ __launch_bounds__(256) void k_ilu_factor(IluView v, T *__restrict__ blocks, int *__restrict__ status,
                                                    int status_base) {
  const int b = blockIdx.x, tid = threadIdx.x;
  const int k = v.patch[b], m = v.pm[k], r0 = v.row0[b];
  T *A = blocks + v.boff[k];
  const uint32_t *mk = v.mask + v.moff[b];
  int fail = 0;
  for (int kk = 0; kk < m; ++kk) {
    const T akk = A[(int64_t)kk * m + kk];
    if (!(akk != (T)0) || !isfinite((double)akk)) {
      fail = kk + 1;
      break;
    }
    const int ua = v.uptr[r0 + kk], nu = v.uptr[r0 + kk + 1] - ua;
    const int ca = v.cptr[r0 + kk], nl = v.cptr[r0 + kk + 1] - ca;
    for (int t = tid; t < nl * nu; t += 256) {
      const int i = v.crow[ca + t / nu], j = v.ucol[ua + t % nu];
      const int64_t bit = (int64_t)i * m + j;
      if ((mk[bit >> 5] >> (bit & 31)) & 1u) {
        const T l = A[(int64_t)i * m + kk] / akk;
        A[(int64_t)i * m + j] -= l * A[(int64_t)kk * m + j];
      }
    }
    __threadfence_block();
    __syncthreads();
    for (int t = tid; t < nl; t += 256) {
      const int64_t q = (int64_t)v.crow[ca + t] * m + kk;
      A[q] = A[q] / akk;
    }
    __threadfence_block();
    __syncthreads();
  }
  if (tid == 0) status[status_base + k] = fail;
}
template <typename T>
void launch_ilu_factor(const IluView &v, T *blocks, int *status, int status_base, hipStream_t st) {
  if (v.nblk > 0) k_ilu_factor<T><<<v.nblk, 256, 0, st>>>(v, blocks, status, status_base);
}
template void launch_ilu_factor<double>(const IluView &, double *, int *, int, hipStream_t);
template void launch_ilu_factor<float>(const IluView &, float *, int *, int, hipStream_t);

template <typename T, typename V>
__global__ void k_ilu_gather(const T *__restrict__ blocks, const int *__restrict__ pos, int64_t n,
                             V *__restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q < n) out[q] = (V)blocks[pos[q]];
}
template <typename T, typename V>
void launch_ilu_gather(const T *blocks, const int *pos, int64_t n, V *out, hipStream_t st) {
  if (n > 0) k_ilu_gather<T, V><<<cdiv(n, 256), 256, 0, st>>>(blocks, pos, n, out);
}
template void launch_ilu_gather<double, double>(const double *, const int *, int64_t, double *, hipStream_t);
template void launch_ilu_gather<float, float>(const float *, const int *, int64_t, float *, hipStream_t);

// Forward then backward substitution of one ILU block per workgroup (256
// threads), level by level: the rows of a level depend only on earlier
// levels, so up to 32 rows of a level run side by side, eight lanes per row
// summing its products (in a fixed order: lane-strided partial sums, then a
// fixed butterfly), with one barrier per level (measured: the sweeps in one
// wave with wave-level ordering instead, eight rows at a time, were slower).
// STAGE: each sweep's factor (L for the forward sweep, then U for the
// backward one: values and 16-bit columns) is first copied to LDS by the
// whole workgroup, four loads in flight per thread; else the factors are read
// from memory.
template <typename V, bool STAGE>
__global__ __launch_bounds__(256) void k_ilu_apply(IluView v, const V *__restrict__ lval, const V *__restrict__ uval,
                                                   const V *__restrict__ udiag, const V *__restrict__ s,
                                                   V *__restrict__ e, V omega, int add, int clear) {
  extern __shared__ __align__(16) unsigned char ilu_lds[];
  __shared__ V y[kMaxPatch];
  __shared__ V dg[kMaxPatch];
  __shared__ int lp[kMaxPatch + 1], upp[kMaxPatch + 1];
  __shared__ int16_t fr[kMaxPatch], br[kMaxPatch];
  __shared__ int16_t fl[kMaxPatch + 1], bl[kMaxPatch + 1];   // level starts (local)
  const int b = blockIdx.x, tid = threadIdx.x;
  const int k = v.patch[b], m = v.pm[k], r0 = v.row0[b];
  const int *d = v.dof + v.pdof_off[k];
  const int la = v.lptr[r0], ua = v.uptr[r0];
  const int f0 = v.flev_off[b], nf = v.flev_off[b + 1] - f0;
  const int b0 = v.blev_off[b], nb = v.blev_off[b + 1] - b0;
  for (int t = tid; t <= nf; t += 256) fl[t] = (int16_t)(v.flev[f0 + t] - r0);
  for (int t = tid; t <= nb; t += 256) bl[t] = (int16_t)(v.blev[b0 + t] - r0);
  for (int c = tid; c < m; c += 256) {
    y[c] = s[d[c]];
    dg[c] = udiag[r0 + c];
    fr[c] = v.frow[r0 + c];
    br[c] = v.brow[r0 + c];
  }
  for (int c = tid; c <= m; c += 256) {
    lp[c] = v.lptr[r0 + c] - la;
    upp[c] = v.uptr[r0 + c] - ua;
  }
  if (clear && !add)
    for (int i = b * 256 + tid; i < v.nunowned; i += v.nblk * 256) e[v.unowned[i]] = (V)0;
  const V *Lv = lval + la, *Uv = uval + ua;
  const int16_t *Lc = v.lcol + la, *Uc = v.ucol + ua;
  V *sv = reinterpret_cast<V *>(ilu_lds);
  // one factor's n values and columns into LDS (values, then the columns)
  auto stage = [&](const V *gv, const int16_t *gc, int n, const V *&lv, const int16_t *&lc) {
    int16_t *sc = reinterpret_cast<int16_t *>(sv + n);
    for (int q0 = tid; q0 < n; q0 += 256 * 4) {
      V a[4];
      int16_t c[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = min(q0 + 256 * u, n - 1);
        a[u] = gv[q];
        c[u] = gc[q];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (q0 + 256 * u < n) {
          sv[q0 + 256 * u] = a[u];
          sc[q0 + 256 * u] = c[u];
        }
    }
    lv = sv;
    lc = sc;
  };
  if constexpr (STAGE) stage(Lv, Lc, v.lptr[r0 + m] - la, Lv, Lc);
  __syncthreads();
  const int grp = tid >> 3, sub = tid & 7;
  for (int f = 0; f < nf; ++f) {
    const int a = fl[f], z = fl[f + 1];
    for (int base = a; base < z; base += 32) {
      const int rr = base + grp;
      int row = 0;
      V acc = 0;
      if (rr < z) {
        row = fr[rr];
        for (int q = lp[row] + sub; q < lp[row + 1]; q += 8) acc += Lv[q] * y[Lc[q]];
      }
      acc = group_sum<V, 8>(acc);
      if (rr < z && sub == 0) y[row] -= acc;
    }
    __syncthreads();
  }
  if constexpr (STAGE) {
    stage(Uv, Uc, v.uptr[r0 + m] - ua, Uv, Uc);   // the forward sweep's reads ended at its last barrier
    __syncthreads();
  }
  for (int f = 0; f < nb; ++f) {
    const int a = bl[f], z = bl[f + 1];
    for (int base = a; base < z; base += 32) {
      const int rr = base + grp;
      int row = 0;
      V acc = 0;
      if (rr < z) {
        row = br[rr];
        for (int q = upp[row] + sub; q < upp[row + 1]; q += 8) acc += Uv[q] * y[Uc[q]];
      }
      acc = group_sum<V, 8>(acc);
      if (rr < z && sub == 0) y[row] = (y[row] - acc) / dg[row];
    }
    __syncthreads();
  }
  for (int t = v.out_off[k] + tid; t < v.out_off[k + 1]; t += 256) {
    const int g = v.out_idx[t];
    const V u = omega * y[v.own_local[t]];
    e[g] = add ? e[g] + u : u;
  }
}
template <typename V>
void launch_ilu_apply(const IluView &v, const V *lval, const V *uval, const V *udiag, const V *s, V *e,
                      V omega, bool add, bool clear, hipStream_t st) {
  if (v.nblk == 0) return;
  // staged when the larger factor of every block fits beside the kernel's
  // static LDS (about 26 KB in FP64)
  constexpr size_t kStageMax = 128 * 1024;
  const size_t stage = (size_t)v.max_entries * (sizeof(V) + sizeof(int16_t));
  if (stage <= kStageMax) {
    static std::once_flag attr;   // raise the dynamic LDS limit once per instance (setup threads race here)
    std::call_once(attr, [] {
      hip_ok_or_clear(hipFuncSetAttribute((const void *)k_ilu_apply<V, true>,
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)kStageMax));
    });
    k_ilu_apply<V, true><<<v.nblk, 256, stage, st>>>(v, lval, uval, udiag, s, e, omega, (int)add, (int)clear);
  } else {
    k_ilu_apply<V, false><<<v.nblk, 256, 0, st>>>(v, lval, uval, udiag, s, e, omega, (int)add, (int)clear);
  }
}
template void launch_ilu_apply<double>(const IluView &, const double *, const double *, const double *,
                                       const double *, double *, double, bool, bool, hipStream_t);
template void launch_ilu_apply<float>(const IluView &, const float *, const float *, const float *,
                                      const float *, float *, float, bool, bool, hipStream_t);

// ------------------------------------------------------------------ Galerkin product
// out[q] = sum over t in [ptr[q], ptr[q+1]) of x[idx[t]] * w[t], in list order
// (one thread per output entry)
__global__ __launch_bounds__(256) void k_gather_dot(int n, const int *__restrict__ ptr, const int *__restrict__ idx,
                                                    const double *__restrict__ w, const double *__restrict__ x,
                                                    double *__restrict__ out) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= n) return;
  double acc = 0.0;
  for (int t = ptr[q]; t < ptr[q + 1]; ++t) acc += x[idx[t]] * w[t];
  out[q] = acc;
}
void launch_gather_dot(int n, const int *ptr, const int *idx, const double *w, const double *x, double *out,
                       hipStream_t st) {
  if (n > 0) k_gather_dot<<<cdiv(n, 256), 256, 0, st>>>(n, ptr, idx, w, x, out);
}
__global__ void k_add_at(double *val, const int *pos, int n, double v) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t < n) val[pos[t]] += v;
}
void launch_add_at(double *val, const int *pos, int n, double v, hipStream_t st) {
  if (n > 0) k_add_at<<<cdiv(n, 256), 256, 0, st>>>(val, pos, n, v);
}

// ------------------------------------------------------------------ coarsest solve GEMV
// y = W x with W row-major: one wave per row streams the row (64 consecutive
// doubles per load, four loads in flight), then a fixed butterfly
__device__ __forceinline__ void gemv_rows_body(int blk, const double *__restrict__ W, int n,
                                               const double *__restrict__ x, double *__restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int row = blk * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const double *w = W + (int64_t)row * n;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int c = lane;
  for (; c + 192 < n; c += 256) {
    a0 += w[c] * x[c];
    a1 += w[c + 64] * x[c + 64];
    a2 += w[c + 128] * x[c + 128];
    a3 += w[c + 192] * x[c + 192];
  }
  for (; c < n; c += 64) a0 += w[c] * x[c];
  double acc = (a0 + a1) + (a2 + a3);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) y[row] = acc;
}
__global__ __launch_bounds__(256) void k_gemv_rows(const double *__restrict__ W, int n,
                                                   const double *__restrict__ x,
                                                   double *__restrict__ y) {
  gemv_rows_body(blockIdx.x, W, n, x, y);
}
__global__ __launch_bounds__(256) void k_gemv_batch(GemvBatch B) {
  const int s = batch_entry(B.blk0, B.count, blockIdx.x);
  gemv_rows_body(blockIdx.x - B.blk0[s], B.it[s].W, B.it[s].n, B.it[s].x, B.it[s].y);
}
void launch_dense_gemv(const double *W, int n, const double *x, double *y, hipStream_t st) {
  if (n > 0) k_gemv_rows<<<cdiv(n, 4), 256, 0, st>>>(W, n, x, y);
}
void launch_dense_gemv_batch(const GemvItem *items, int count, hipStream_t st) {
  GemvBatch B;
  B.count = 0;
  B.blk0[0] = 0;
  auto flush = [&] {
    if (B.count && B.blk0[B.count]) k_gemv_batch<<<B.blk0[B.count], 256, 0, st>>>(B);
    B.count = 0;
  };
  for (int i = 0; i < count; ++i) {
    if (items[i].n <= 0) continue;
    B.it[B.count] = items[i];
    B.blk0[B.count + 1] = B.blk0[B.count] + cdiv(items[i].n, 4);
    if (++B.count == kMaxBatch) flush();
  }
  flush();
}

// Arnoldi column j (one thread): H[:, j] = h, |w| and breakdown test, the
// previous rotations, a new one, and g
__device__ void givens_column(double *H, int ldh, int j, const double *h, const double *nrm2,
                              double *cs, double *sn, double *g, double *flags, double *scal) {
  const double hn = sqrt(nrm2[0]);
  double hh = 0.0;
  for (int i = 0; i <= j; ++i) {
    H[i + (int64_t)j * ldh] = h[i];
    hh += h[i] * h[i];
  }
  H[j + 1 + (int64_t)j * ldh] = hn;
  const int breakdown = hn <= 1e-14 * sqrt(hh);
  for (int i = 0; i < j; ++i) {
    const double a = H[i + (int64_t)j * ldh], b = H[i + 1 + (int64_t)j * ldh];
    H[i + (int64_t)j * ldh] = cs[i] * a + sn[i] * b;
    H[i + 1 + (int64_t)j * ldh] = -sn[i] * a + cs[i] * b;
  }
  const double a = H[j + (int64_t)j * ldh], b = H[j + 1 + (int64_t)j * ldh];
  const double den = hypot(a, b);
  cs[j] = a / den;
  sn[j] = b / den;
  H[j + (int64_t)j * ldh] = den;
  H[j + 1 + (int64_t)j * ldh] = 0.0;
  g[j + 1] = -sn[j] * g[j];
  g[j] = cs[j] * g[j];
  flags[0] = fabs(g[j + 1]);
  flags[1] = breakdown ? 1.0 : 0.0;
  scal[0] = hn;
}
// ------------------------------------------------------------------ Krylov reductions
// Every reduction over the n rows runs on krylov_blocks(n) fixed row chunks:
// a chunk's sum, formed in a fixed order, goes to partial[i * nblk + chunk].
// The kernel that needs the totals adds the chunk sums in a fixed order, in
// every workgroup (a few KB read from L2 each), so no separate reduction
// launch and no cross-workgroup signalling is needed, and every sum has one
// order for a given n: runs are reproducible.

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// out[i] = sum over the nblk chunk sums of column i, i < k <= kMaxKrylovCols.
// Wave w takes columns w, w + kKrylovWaves, ...; lane l adds chunks l, l + 64,
// ... in order, then a fixed butterfly.  All loads are issued before the adds.
__device__ __forceinline__ void finish_cols(const double *__restrict__ partial, int nblk, int k,
                                            double *out) {
  constexpr int C = (kMaxKrylovCols + kKrylovWaves - 1) / kKrylovWaves;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (wave >= k) return;
  double s[C];
#pragma unroll
  for (int c = 0; c < C; ++c) s[c] = 0.0;
#pragma unroll 4
  for (int b0 = 0; b0 < nblk; b0 += 64) {
    const bool ok = b0 + lane < nblk;
    const int b = ok ? b0 + lane : nblk - 1;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int i = min(wave + kKrylovWaves * c, k - 1);
      const double v = partial[(int64_t)i * nblk + b];
      s[c] += ok ? v : 0.0;
    }
  }
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const double t = wave_sum(s[c]);
    if (lane == 0 && wave + kKrylovWaves * c < k) out[wave + kKrylovWaves * c] = t;
  }
}

__device__ __forceinline__ void chunk_range(int n, int &r0, int &r1) {
  const int chunk = (n + gridDim.x - 1) / gridDim.x;
  r0 = min(n, (int)blockIdx.x * chunk);
  r1 = min(n, r0 + chunk);
}

// chunk sums of V[:, i]^T w for i < k, one wave per column (w from global, or
// from LDS indexed from the chunk's first row)
template <bool WLDS>
__device__ __forceinline__ void chunk_dots(const double *__restrict__ V, int64_t ldv, int k,
                                           const double *w, int r0, int r1,
                                           double *__restrict__ partial) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nblk = gridDim.x;
  for (int i = wave; i < k; i += kKrylovWaves) {
    const double *Vi = V + (int64_t)i * ldv;
    double acc = 0.0;
    for (int r = r0 + lane; r < r1; r += 64) acc += Vi[r] * (WLDS ? w[r - r0] : w[r]);
    acc = wave_sum(acc);
    if (lane == 0) partial[(int64_t)i * nblk + blockIdx.x] = acc;
  }
}

// w -= V h on the chunk's rows (h in LDS; sum over the columns in order), the
// new rows also kept in LDS (ws, when given); returns this thread's sum of squares
__device__ __forceinline__ double chunk_update(const double *__restrict__ V, int64_t ldv, int k,
                                               const double *hs, double *__restrict__ w, int r0,
                                               int r1, double *ws) {
  double nacc = 0.0;
  for (int r = r0 + threadIdx.x; r < r1; r += kKrylovThreads) {
    double s = 0.0;
    for (int i = 0; i < k; ++i) s += V[(int64_t)i * ldv + r] * hs[i];
    const double nv = w[r] - s;
    w[r] = nv;
    if (ws) ws[r - r0] = nv;
    nacc += nv * nv;
  }
  return nacc;
}

// partial <- chunk sums of V[:, 0..k)^T w
__global__ __launch_bounds__(kKrylovThreads) void k_kdot(int n, const double *__restrict__ V,
                                                         int64_t ldv, int k,
                                                         const double *__restrict__ w,
                                                         double *__restrict__ partial) {
  int r0, r1;
  chunk_range(n, r0, r1);
  chunk_dots<false>(V, ldv, k, w, r0, r1, partial);
}
__global__ __launch_bounds__(kKrylovThreads) void k_kfinish(const double *__restrict__ partial,
                                                            int nblk, int k,
                                                            double *__restrict__ h) {
  finish_cols(partial, nblk, k, h);
}
void launch_kdot(int n, const double *V, int64_t ldv, int k, const double *w, double *partial,
                 double *h, hipStream_t st) {
  const int nb = krylov_blocks(n);
  k_kdot<<<nb, kKrylovThreads, 0, st>>>(n, V, ldv, k, w, partial);
  k_kfinish<<<1, kKrylovThreads, 0, st>>>(partial, nb, k, h);
}

// h1 = sum of pin's chunk sums (block 0 stores it); w -= V h1; pout <- chunk
// sums of V^T w
__global__ __launch_bounds__(kKrylovThreads) void k_kupdate_dot(
    int n, const double *__restrict__ V, int64_t ldv, int k, const double *__restrict__ pin,
    double *__restrict__ h1, double *__restrict__ w, double *__restrict__ pout) {
  __shared__ double hs[kMaxKrylovCols];
  __shared__ double ws[kKrylovChunk];
  int r0, r1;
  chunk_range(n, r0, r1);
  finish_cols(pin, gridDim.x, k, hs);
  __syncthreads();
  if (blockIdx.x == 0 && (int)threadIdx.x < k) h1[threadIdx.x] = hs[threadIdx.x];
  (void)chunk_update(V, ldv, k, hs, w, r0, r1, ws);
  __syncthreads();
  chunk_dots<true>(V, ldv, k, ws, r0, r1, pout);
}

// h2 = sum of pin's chunk sums (block 0: h1 += h2, or h1 = h2 when the pass
// is the only one, SET); w -= V h2; npart <- chunk sums of w^2
template <bool SET>
__global__ __launch_bounds__(kKrylovThreads) void k_kupdate_norm(
    int n, const double *__restrict__ V, int64_t ldv, int k, const double *__restrict__ pin,
    double *__restrict__ h1, double *__restrict__ w, double *__restrict__ npart) {
  __shared__ double hs[kMaxKrylovCols];
  __shared__ double red[kKrylovWaves];
  int r0, r1;
  chunk_range(n, r0, r1);
  finish_cols(pin, gridDim.x, k, hs);
  __syncthreads();
  if (blockIdx.x == 0 && (int)threadIdx.x < k) h1[threadIdx.x] = SET ? hs[threadIdx.x] : h1[threadIdx.x] + hs[threadIdx.x];
  const double nacc = wave_sum(chunk_update(V, ldv, k, hs, w, r0, r1, nullptr));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = nacc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kKrylovWaves; ++q) t += red[q];
    npart[blockIdx.x] = t;
  }
}

// |w|^2 from npart; block 0 forms Arnoldi column j and its rotations; every
// block writes its chunk of v_{j+1} = w / |w| (unless |w| == 0)
__global__ __launch_bounds__(kKrylovThreads) void k_kgivens_scale(
    int n, const double *__restrict__ npart, const double *__restrict__ w, double *__restrict__ v,
    double *H, int ldh, int j, const double *h1, double *cs, double *sn, double *g,
    double *flags, double *scal, double *host_out) {
  __shared__ double nrm2[1];
  int r0, r1;
  chunk_range(n, r0, r1);
  finish_cols(npart, gridDim.x, 1, nrm2);
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    givens_column(H, ldh, j, h1, nrm2, cs, sn, g, flags, scal);
    if (host_out) {
      host_out[0] = flags[0];
      host_out[1] = flags[1];
      __threadfence_system();
      host_out[2] = 1.0;   // ready: the host polls this after clearing it
    }
  }
  const double hn = sqrt(nrm2[0]);
  if (hn > 0.0)
    for (int r = r0 + threadIdx.x; r < r1; r += kKrylovThreads) v[r] = w[r] / hn;
}

void launch_arnoldi_orth(int n, const double *V, int64_t ldv, int k, double *w, double *partial,
                         double *h1, double *npart, double *v_next, double *H, int ldh, int j,
                         double *cs, double *sn, double *g, double *flags, double *scal,
                         double *host_out, hipStream_t st, bool twice) {
  const int nb = krylov_blocks(n);
  double *p1 = partial, *p2 = partial + (int64_t)nb * kMaxKrylovCols;
  k_kdot<<<nb, kKrylovThreads, 0, st>>>(n, V, ldv, k, w, p1);
  if (twice) {
    k_kupdate_dot<<<nb, kKrylovThreads, 0, st>>>(n, V, ldv, k, p1, h1, w, p2);
    k_kupdate_norm<false><<<nb, kKrylovThreads, 0, st>>>(n, V, ldv, k, p2, h1, w, npart);
  } else {
    k_kupdate_norm<true><<<nb, kKrylovThreads, 0, st>>>(n, V, ldv, k, p1, h1, w, npart);
  }
  k_kgivens_scale<<<nb, kKrylovThreads, 0, st>>>(n, npart, w, v_next, H, ldh, j, h1, cs, sn, g,
                                                 flags, scal, host_out);
}

__global__ void k_backsolve(const double *H, int ldh, const double *g, int k, double *y) {
  if (threadIdx.x != 0) return;
  for (int i = k - 1; i >= 0; --i) {
    double s = g[i];
    for (int l = i + 1; l < k; ++l) s -= H[i + (int64_t)l * ldh] * y[l];
    y[i] = s / H[i + (int64_t)i * ldh];
  }
}
void launch_backsolve(const double *H, int ldh, const double *g, int k, double *y,
                      hipStream_t st) {
  k_backsolve<<<1, 64, 0, st>>>(H, ldh, g, k, y);
}
__global__ void k_zupdate(int n, const double *__restrict__ Z, int64_t ldz, int k,
                          const double *__restrict__ y, double *__restrict__ x) {
  __shared__ double ys[64];
  if ((int)threadIdx.x < k) ys[threadIdx.x] = y[threadIdx.x];
  __syncthreads();
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double s = 0.0;
  for (int i = 0; i < k; ++i) s += Z[(int64_t)i * ldz + r] * ys[i];
  x[r] += s;
}
void launch_zupdate(int n, const double *Z, int64_t ldz, int k, const double *y, double *x,
                    hipStream_t st) {
  k_zupdate<<<cdiv(n, 256), 256, 0, st>>>(n, Z, ldz, k, y, x);
}
__global__ void k_start_cycle(int n, const double *r, const double *nrm2, double *v, double *g,
                              int m) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const double beta = sqrt(nrm2[0]);
  if (i < n) v[i] = r[i] / beta;
  if (i <= m) g[i] = (i == 0) ? beta : 0.0;
}
void launch_start_cycle(int n, const double *r, const double *nrm2, double *v, double *g, int m,
                        hipStream_t st) {
  k_start_cycle<<<cdiv(std::max(n, m + 1), 256), 256, 0, st>>>(n, r, nrm2, v, g, m);
}

// ------------------------------------------------------------------ measurement
// Streaming read of n doubles with 16-byte loads, eight in flight per lane
// over a grid-stride loop; block b writes its partial sum to out[b].  It is
// the device's plain read rate that the HBM-bound kernels are compared with.
// each workgroup streams its own contiguous chunk (a grid-stride pattern over
// the whole buffer reads about 10 % slower on this device)
__global__ __launch_bounds__(256) void k_stream_read(const double2 *__restrict__ x, int64_t n2,
                                                     double *__restrict__ out) {
  __shared__ double red[4];
  const int64_t chunk = (n2 + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = (int64_t)blockIdx.x * chunk;
  const int64_t b1 = b0 + chunk < n2 ? b0 + chunk : n2;
  int64_t i = b0 + threadIdx.x;
  double s = 0.0;
  for (; i + 7 * 256 < b1; i += 8 * 256) {
    double2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = x[i + u * 256];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u].x + v[u].y;
  }
  for (; i < b1; i += 256) s += x[i].x + x[i].y;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}
void launch_stream_read(const double *x, int64_t n, double *out, hipStream_t st) {
  if (n >= 2)
    k_stream_read<<<kStreamReadBlocks, 256, 0, st>>>(reinterpret_cast<const double2 *>(x), n / 2,
                                                     out);
}

}  // namespace fsi
