// gfx950 kernels of the FSI multigrid/FGMRES hot path.
//
// Memory-bound steps (SpMV residuals, transfers, Schwarz applications,
// coarsest solve, Krylov vector work) are written for coalesced HBM access
// with 64-wide wavefronts; the dense block inversion (setup) is a blocked
// Gauss-Jordan elimination with the pivot panel staged in LDS.
#include "fsi_kernels.h"

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <algorithm>
#include <cmath>

namespace fsi {

static inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// ------------------------------------------------------------------ SpMV
template <typename T, int LPR>
__global__ __launch_bounds__(256) void k_spmv(int nrows, const int *__restrict__ rowptr,
                                              const int *__restrict__ col,
                                              const T *__restrict__ val, const T *__restrict__ x,
                                              const T *__restrict__ r, T *__restrict__ y,
                                              int mode) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int row = gid / LPR;
  const int lane = gid % LPR;
  if (row >= nrows) return;  // whole lane group leaves together
  const int beg = rowptr[row], end = rowptr[row + 1];
  T acc = 0;
  for (int p = beg + lane; p < end; p += LPR) acc += val[p] * x[col[p]];
#pragma unroll
  for (int off = LPR / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, LPR);
  if (lane == 0) {
    if (mode == kSpmvSet)
      y[row] = acc;
    else if (mode == kSpmvResid)
      y[row] = r[row] - acc;
    else
      y[row] += acc;
  }
}

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
// One wave per (patch, local row): every nonzero of the CSR row whose column
// belongs to the patch lands at its position (binary search in the sorted dof list).
__global__ __launch_bounds__(256) void k_extract(int nrows_total, const int *__restrict__ row_patch,
                                                 const int *__restrict__ row_local,
                                                 const int *__restrict__ pm,
                                                 const int64_t *__restrict__ pdof_off,
                                                 const int *__restrict__ dof,
                                                 const int64_t *__restrict__ boff,
                                                 const int *__restrict__ rowptr,
                                                 const int *__restrict__ col,
                                                 const double *__restrict__ val,
                                                 double *__restrict__ blocks) {
  const int t = blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (t >= nrows_total) return;
  const int k = row_patch[t];
  const int i = row_local[t];
  const int m = pm[k];
  const int *d = dof + pdof_off[k];
  const int g = d[i];
  double *B = blocks + boff[k] + (int64_t)i * m;
  for (int p = rowptr[g] + lane; p < rowptr[g + 1]; p += 64) {
    const int c = col[p];
    int lo = 0, hi = m - 1;
    while (lo <= hi) {
      const int mid = (lo + hi) >> 1;
      const int v = d[mid];
      if (v == c) {
        B[mid] = val[p];
        break;
      }
      if (v < c)
        lo = mid + 1;
      else
        hi = mid - 1;
    }
  }
}

void launch_extract(const CsrView<double> &J, int npatch, const int *pm, const int64_t *pdof_off,
                    const int *dof, const int64_t *boff, double *blocks, int64_t total_rows,
                    const int *row_patch, const int *row_local, hipStream_t st) {
  (void)npatch;
  if (total_rows == 0) return;
  k_extract<<<cdiv(total_rows, 4), 256, 0, st>>>((int)total_rows, row_patch, row_local, pm,
                                                  pdof_off, dof, boff, J.rowptr, J.col, J.val,
                                                  blocks);
}

// ------------------------------------------------------------------ Gauss-Jordan inversion
// In-place Gauss-Jordan with partial pivoting (largest |a|, lowest row on
// ties), blocked by panels of NB pivot columns.  For a panel starting at p0:
//  1. the m x w panel is processed step by step (pivot search over the rows
//     not yet used, row swap, scaling of the pivot row, elimination of every
//     other row, the pivot column replaced by the inverse column);
//  2. every other column v receives the panel's row swaps and then the
//     accumulated transform v <- (v with pivot rows zeroed) + Pn v[pivot rows],
//     a rank-w update;
// finally the columns are un-permuted in reverse order of the row swaps.

struct Argmax {
  double v;
  int i;
};
__device__ inline Argmax better(Argmax a, Argmax b) {
  if (b.v > a.v || (b.v == a.v && b.i < a.i)) return b;
  return a;
}
__device__ inline Argmax wave_argmax(Argmax a) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    Argmax b;
    b.v = __shfl_xor(a.v, off, 64);
    b.i = __shfl_xor(a.i, off, 64);
    a = better(a, b);
  }
  return a;
}

// Panel pivot steps executed by ONE wavefront: lane l owns the panel rows
// i = l, l + 64, ...; the pivot search is a shuffle argmax; the pivot-row
// swap, the broadcast of the pivot row and the updates are LDS accesses of
// that single wave, which the LDS serves in program order, so a step needs
// no workgroup barrier.  Panel element (i, c) at P[i * ps + c].  TC >= 0:
// the step's pivot column is the compile-time TC of a full-width panel.
template <int NB, int TC>
__device__ __forceinline__ int pivot_step(double *P, int ps, int m, int p0, int w, int t_rt,
                                          int *swaps) {
  constexpr bool FULL = TC >= 0;
  const int t = FULL ? TC : t_rt;
  const int lane = threadIdx.x & 63;
  const int p = p0 + t;
  Argmax best{-1.0, 0x7fffffff};
  for (int i = p + lane; i < m; i += 64) {
    const double a = fabs(P[i * ps + t]);
    best = better(best, Argmax{a != a ? INFINITY : a, i});
  }
  best = wave_argmax(best);
  if (!(best.v > 0.0) || isinf(best.v)) return p + 1;
  const int piv = best.i;
  if (lane == 0) swaps[p] = piv;
  if (piv != p && lane < (FULL ? NB : w)) {
    const double a = P[p * ps + lane];
    P[p * ps + lane] = P[piv * ps + lane];
    P[piv * ps + lane] = a;
  }
  const double d = 1.0 / P[p * ps + t];
  double prow[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) prow[c] = ((FULL || c < w) && c != t) ? P[p * ps + c] * d : 0.0;
  for (int i = lane; i < m; i += 64) {
    double *row = P + i * ps;
    double v[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) v[c] = (FULL || c < w) ? row[c] : 0.0;
    if (i == p) {
#pragma unroll
      for (int c = 0; c < NB; ++c) v[c] = (c == t) ? d : prow[c];
    } else {
      const double f = FULL ? v[FULL ? TC : 0] : row[t];
#pragma unroll
      for (int c = 0; c < NB; ++c) v[c] = (c == t) ? -f * d : v[c] - f * prow[c];
    }
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (FULL || c < w) row[c] = v[c];
  }
  return 0;
}

template <int NB, int T>
__device__ __forceinline__ int full_steps(double *P, int ps, int m, int p0, int *swaps) {
  if constexpr (T < NB) {
    const int f = pivot_step<NB, T>(P, ps, m, p0, NB, T, swaps);
    if (f) return f;
    return full_steps<NB, T + 1>(P, ps, m, p0, swaps);
  } else {
    return 0;
  }
}

template <int NB>
__device__ int panel_wave(double *P, int ps, int m, int p0, int w, int *swaps) {
  if (w == NB) return full_steps<NB, 0>(P, ps, m, p0, swaps);
  for (int t = 0; t < w; ++t) {
    const int f = pivot_step<NB, -1>(P, ps, m, p0, w, t, swaps);
    if (f) return f;
  }
  return 0;
}

// The panel's row swaps (p0+t <-> swaps[p0+t], in order) as one permutation
// of at most 2 w rows: dst[k] receives the old row src[k].  One thread.
template <int NB>
__device__ int row_permutation(const int *swaps, int p0, int w, int *dst, int *src, int *pos,
                               int *cur) {
  int cnt = 0;
  auto slot = [&](int r) {
    for (int q = 0; q < cnt; ++q)
      if (pos[q] == r) return q;
    pos[cnt] = r;
    cur[cnt] = r;
    return cnt++;
  };
  for (int t = 0; t < w; ++t) {
    const int a = slot(p0 + t), b = slot(swaps[p0 + t]);
    const int tmp = cur[a];
    cur[a] = cur[b];
    cur[b] = tmp;
  }
  int n = 0;
  for (int q = 0; q < cnt; ++q)
    if (cur[q] != pos[q]) {
      dst[n] = pos[q];
      src[n] = cur[q];
      ++n;
    }
  return n;
}

// One workgroup per block (all smoothing levels in one launch); the m x NB
// panel lives in LDS, its pivot steps run on the first wave, then all waves
// apply the rank-w update to the other columns over (column, chunk of NB
// rows) items: all rows but the pivot chunk first, then the pivot chunk
// (whose old values are the update's right factor X).  Each item issues its
// 2 NB loads before its FMAs.
template <int NB, int NT>
__global__ __launch_bounds__(NT) void k_gj_batched(double *blocks, const int64_t *boff,
                                                   const int *pm, int *status) {
  extern __shared__ double lds[];
  __shared__ int swaps[kMaxPatch];
  __shared__ int s_flag[1], s_nperm[1], s_dst[2 * NB], s_src[2 * NB], s_pos[2 * NB], s_cur[2 * NB];
  const int k = blockIdx.x;
  const int m = pm[k];
  double *A = blocks + boff[k];
  constexpr int PS = NB + 1;                // padded row stride: lane-owned rows hit distinct banks
  double *P = lds;                          // m x NB, row-major, stride PS
  const int tid = threadIdx.x;
  const int nchunk = (m + NB - 1) / NB;
  int fail = 0;
  for (int p0 = 0; p0 < m && !fail; p0 += NB) {
    const int w = min(NB, m - p0);
    const int rstep = NT / w;
    if (tid < rstep * w)
      for (int i = tid / w, c = tid % w; i < m; i += rstep) P[i * PS + c] = A[i * m + p0 + c];
    __syncthreads();
    if (tid < 64) {
      const int f = panel_wave<NB>(P, PS, m, p0, w, swaps);
      if (tid == 0) s_flag[0] = f;
    }
    __syncthreads();
    fail = s_flag[0];
    if (fail) break;
    if (tid < rstep * w)
      for (int i = tid / w, c = tid % w; i < m; i += rstep) A[i * m + p0 + c] = P[i * PS + c];
    const int ncol = m - w;
    if (tid == 0) s_nperm[0] = row_permutation<NB>(swaps, p0, w, s_dst, s_src, s_pos, s_cur);
    __syncthreads();
    // row swaps of this panel on the other columns: independent loads, then stores
    const int nperm = s_nperm[0];
    for (int q = tid; q < ncol; q += NT) {
      const int j = q < p0 ? q : q + w;
      double vals[2 * NB];
#pragma unroll
      for (int k2 = 0; k2 < 2 * NB; ++k2) vals[k2] = (k2 < nperm) ? A[(int64_t)s_src[k2] * m + j] : 0.0;
#pragma unroll
      for (int k2 = 0; k2 < 2 * NB; ++k2)
        if (k2 < nperm) A[(int64_t)s_dst[k2] * m + j] = vals[k2];
    }
    __threadfence_block();
    __syncthreads();
    const int cp = p0 / NB;
    for (int pass = 0; pass < 2; ++pass) {
      const int nitem = pass == 0 ? ncol * (nchunk - 1) : ncol;
      // item -> (chunk, column); the division happens once per item, not per FMA
      for (int it = tid; it < nitem; it += NT) {
        int chunk = pass == 0 ? it / ncol : cp;
        if (pass == 0 && chunk >= cp) ++chunk;
        const int q = it - (pass == 0 ? (it / ncol) * ncol : 0);
        const int j = q < p0 ? q : q + w;
        const int i0 = chunk * NB, i1 = min(m, i0 + NB);
        double X[NB], Ac[NB];
#pragma unroll
        for (int t = 0; t < NB; ++t) X[t] = (t < w) ? A[(int64_t)(p0 + t) * m + j] : 0.0;
#pragma unroll
        for (int u = 0; u < NB; ++u) Ac[u] = (pass == 0 && i0 + u < i1) ? A[(int64_t)(i0 + u) * m + j] : 0.0;
#pragma unroll
        for (int u = 0; u < NB; ++u) {
          if (i0 + u < i1) {
            const double *Pi = P + (i0 + u) * PS;
            double acc = Ac[u];
#pragma unroll
            for (int t = 0; t < NB; ++t) acc += Pi[t] * X[t];
            A[(int64_t)(i0 + u) * m + j] = acc;
          }
        }
      }
      __threadfence_block();
      __syncthreads();
    }
  }
  if (!fail) {
    for (int i = tid; i < m; i += NT) {
      double *Ai = A + (int64_t)i * m;
      for (int p = m - 1; p >= 0; --p) {
        const int sw = swaps[p];
        if (sw != p) {
          const double a = Ai[p];
          Ai[p] = Ai[sw];
          Ai[sw] = a;
        }
      }
    }
  }
  if (tid == 0) status[k] = fail;
}

// panel width: 16 keeps the rank-w update's operands in registers (no spills)
int gj_panel_width(int mmax) {
  const int64_t budget = 150 * 1024;
  if ((int64_t)mmax * 17 * 8 <= budget) return 16;
  return 8;
}

template <int NB>
static void launch_gj_nb(double *blocks, const int64_t *boff, const int *pm, int npatch, int mmax,
                         int *status, hipStream_t st) {
  const size_t shm = (size_t)mmax * (NB + 1) * sizeof(double);
  (void)hipFuncSetAttribute((const void *)k_gj_batched<NB, 512>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  k_gj_batched<NB, 512><<<npatch, 512, shm, st>>>(blocks, boff, pm, status);
}

void launch_gj_batched(double *blocks, const int64_t *boff, const int *pm, int npatch, int mmax,
                       int *status, hipStream_t st, int nb_req) {
  if (npatch == 0) return;
  int nb = gj_panel_width(mmax);
  if (nb_req == 8 || (nb_req == 16 && (int64_t)mmax * 17 * 8 <= 150 * 1024)) nb = nb_req;
  if (nb == 16)
    launch_gj_nb<16>(blocks, boff, pm, npatch, mmax, status, st);
  else
    launch_gj_nb<8>(blocks, boff, pm, npatch, mmax, status, st);
}

// ---- large single matrix (coarsest operator): the panel lives in LDS
// (column-major, contiguous pivot searches), one workgroup; the same kernel
// applies the panel's row swaps to the other columns and copies their pivot
// rows to X; the rank-w update then runs on many workgroups.
template <int NB>
__global__ __launch_bounds__(512) void k_gj_large_panel(double *A, int n, int p0, int w, int *swaps,
                                                         double *X, int *status) {
  extern __shared__ double lds[];
  __shared__ int s_flag[1], s_nperm[1], s_dst[2 * NB], s_src[2 * NB], s_pos[2 * NB], s_cur[2 * NB];
  if (status[0]) return;
  constexpr int PS = NB + 1;                // padded row stride (bank spread)
  double *P = lds;                          // n x NB, row-major, stride PS
  const int tid = threadIdx.x;
  const int rstep = 512 / w;
  if (tid < rstep * w)
    for (int i = tid / w, c = tid % w; i < n; i += rstep) P[i * PS + c] = A[(int64_t)i * n + p0 + c];
  __syncthreads();
  if (tid < 64) {
    const int f = panel_wave<NB>(P, PS, n, p0, w, swaps);
    if (tid == 0) s_flag[0] = f;
  }
  __syncthreads();
  if (s_flag[0]) {
    if (tid == 0) status[0] = s_flag[0];
    return;
  }
  if (tid < rstep * w)
    for (int i = tid / w, c = tid % w; i < n; i += rstep) A[(int64_t)i * n + p0 + c] = P[i * PS + c];
  if (tid == 0) s_nperm[0] = row_permutation<NB>(swaps, p0, w, s_dst, s_src, s_pos, s_cur);
  __syncthreads();
  const int nperm = s_nperm[0];
  for (int j = tid; j < n; j += 512) {
    if (j >= p0 && j < p0 + w) continue;
    double vals[2 * NB];
#pragma unroll
    for (int k2 = 0; k2 < 2 * NB; ++k2) vals[k2] = (k2 < nperm) ? A[(int64_t)s_src[k2] * n + j] : 0.0;
#pragma unroll
    for (int k2 = 0; k2 < 2 * NB; ++k2)
      if (k2 < nperm) A[(int64_t)s_dst[k2] * n + j] = vals[k2];
    for (int t = 0; t < w; ++t) X[(int64_t)t * n + j] = A[(int64_t)(p0 + t) * n + j];
  }
}
// rows split over blockIdx.y, columns over threads
template <int NB>
__global__ __launch_bounds__(256) void k_gj_large_update(double *A, int n, int p0, int w,
                                                         const double *X, const int *status) {
  if (status[0]) return;
  __shared__ double Pn[64 * NB];
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i0 = blockIdx.y * 64;
  const int i1 = min(n, i0 + 64);
  for (int idx = threadIdx.x; idx < (i1 - i0) * w; idx += blockDim.x) {
    const int i = idx / w, t = idx % w;
    Pn[i * NB + t] = A[(int64_t)(i0 + i) * n + p0 + t];
  }
  __syncthreads();
  if (j >= n || (j >= p0 && j < p0 + w)) return;
  double Xr[NB];
#pragma unroll
  for (int t = 0; t < NB; ++t) Xr[t] = (t < w) ? X[(int64_t)t * n + j] : 0.0;
  for (int i = i0; i < i1; i += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      v[u] = (i + u < i1 && !(i + u >= p0 && i + u < p0 + w)) ? A[(int64_t)(i + u) * n + j] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (i + u < i1) {
        double acc = v[u];
#pragma unroll
        for (int t = 0; t < NB; ++t) acc += Pn[(i + u - i0) * NB + t] * Xr[t];
        A[(int64_t)(i + u) * n + j] = acc;
      }
    }
  }
}
__global__ void k_gj_large_unpermute(double *A, int n, const int *swaps, const int *status) {
  if (status[0]) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double *Ai = A + (int64_t)i * n;
  for (int p = n - 1; p >= 0; --p) {
    const int sw = swaps[p];
    if (sw != p) {
      const double a = Ai[p];
      Ai[p] = Ai[sw];
      Ai[sw] = a;
    }
  }
}

template <int NB>
static void gj_large_nb(double *A, int n, int *status_dev, double *work, hipStream_t st) {
  int *swaps = reinterpret_cast<int *>(work);
  double *X = work + n;
  const size_t shm = (size_t)(NB + 1) * n * sizeof(double);
  (void)hipFuncSetAttribute((const void *)k_gj_large_panel<NB>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  for (int p0 = 0; p0 < n; p0 += NB) {
    const int w = std::min(NB, n - p0);
    k_gj_large_panel<NB><<<1, 512, shm, st>>>(A, n, p0, w, swaps, X, status_dev);
    dim3 grid(cdiv(n, 256), cdiv(n, 64));
    k_gj_large_update<NB><<<grid, 256, 0, st>>>(A, n, p0, w, X, status_dev);
  }
  k_gj_large_unpermute<<<cdiv(n, 256), 256, 0, st>>>(A, n, swaps, status_dev);
}

// work: n ints (swaps, in n doubles) + 16 n doubles (X)
void gj_large(double *A, int n, int *status_dev, double *work, hipStream_t st) {
  const int64_t budget = 150 * 1024;
  if ((int64_t)n * 17 * 8 <= budget)
    gj_large_nb<16>(A, n, status_dev, work, st);
  else if ((int64_t)n * 9 * 8 <= budget)
    gj_large_nb<8>(A, n, status_dev, work, st);
  else
    gj_large_nb<4>(A, n, status_dev, work, st);
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

// one wave per owned row: W[c * o + r] = Binv[own_local[r]][c]; 16-bit rows scaled by max |.|
__global__ __launch_bounds__(256) void k_pack_owned(const double *__restrict__ blocks,
                                                    const int64_t *__restrict__ boff,
                                                    const int *__restrict__ pm,
                                                    const int *__restrict__ po,
                                                    const int64_t *__restrict__ woff,
                                                    const int *__restrict__ own_off,
                                                    const int *__restrict__ own_local,
                                                    int64_t total_owned,
                                                    const int *__restrict__ orow_patch,
                                                    const int *__restrict__ orow_r, double *W64,
                                                    float *W32, uint16_t *W16, int w16_kind,
                                                    float *wscale, const int64_t *__restrict__ pdof_off,
                                                    const float *__restrict__ cscale) {
  const int64_t t = blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (t >= total_owned) return;
  const int k = orow_patch[t];
  const int r = orow_r[t];
  const int m = pm[k], o = po[k];
  const double *row = blocks + boff[k] + (int64_t)own_local[own_off[k] + r] * m;
  const float *cs = W16 ? cscale + pdof_off[k] : nullptr;
  double mx = 0.0;
  if (W16) {
    for (int c = lane; c < m; c += 64) mx = fmax(mx, fabs(row[c]) / (double)cs[c]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    if (mx == 0.0) mx = 1.0;
    if (lane == 0) wscale[own_off[k] + r] = (float)mx;
  }
  for (int c = lane; c < m; c += 64) {
    const int64_t dst = woff[k] + (int64_t)c * o + r;
    const double v = row[c];
    if (W64) W64[dst] = v;
    if (W32) W32[dst] = (float)v;
    if (W16) {
      const float q = (float)(v / ((double)cs[c] * mx));
      W16[dst] = w16_kind == 1 ? to_bf16(q) : to_fp16(q);
    }
  }
}

// column scales of the owned rows of every block inverse: cs = max_r |Binv[own_r][c]|
__global__ void k_colscale(const double *__restrict__ blocks, const int64_t *__restrict__ boff,
                           const int *__restrict__ pm, const int *__restrict__ po,
                           const int *__restrict__ own_off, const int *__restrict__ own_local,
                           const int64_t *__restrict__ pdof_off, int64_t total_cols,
                           const int *__restrict__ col_patch, const int *__restrict__ col_local,
                           float *cscale) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= total_cols) return;
  const int k = col_patch[t], c = col_local[t];
  const int m = pm[k], o = po[k];
  const double *B = blocks + boff[k];
  double mx = 0.0;
  for (int r = 0; r < o; ++r) mx = fmax(mx, fabs(B[(int64_t)own_local[own_off[k] + r] * m + c]));
  cscale[pdof_off[k] + c] = mx > 0.0 ? (float)mx : 1.0f;
}
void launch_colscale(const double *blocks, const int64_t *boff, const int *pm, const int *po,
                     const int *own_off, const int *own_local, const int64_t *pdof_off,
                     int64_t total_cols, const int *col_patch, const int *col_local, float *cscale,
                     hipStream_t st) {
  if (total_cols == 0) return;
  k_colscale<<<cdiv(total_cols, 256), 256, 0, st>>>(blocks, boff, pm, po, own_off, own_local,
                                                     pdof_off, total_cols, col_patch, col_local,
                                                     cscale);
}

void launch_pack_owned(const double *blocks, const int64_t *boff, const int *pm, const int *po,
                       const int64_t *woff, const int *own_off, const int *own_local, int npatch,
                       int64_t total_owned, const int *orow_patch, const int *orow_r, double *W64,
                       float *W32, uint16_t *W16, int w16_kind, float *wscale,
                       const int64_t *pdof_off, const float *cscale, hipStream_t st) {
  (void)npatch;
  if (total_owned == 0) return;
  k_pack_owned<<<cdiv(total_owned, 4), 256, 0, st>>>(blocks, boff, pm, po, woff, own_off,
                                                      own_local, total_owned, orow_patch, orow_r,
                                                      W64, W32, W16, w16_kind, wscale, pdof_off,
                                                      cscale);
}

__global__ void k_transpose(const double *A, int n, double *W) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  const int r = (int)(idx % n), c = (int)(idx / n);
  W[idx] = A[(int64_t)r * n + c];  // W[c * n + r] = A[r][c]
}
void launch_transpose_colmajor(const double *A, int n, double *W, hipStream_t st) {
  k_transpose<<<cdiv((int64_t)n * n, 256), 256, 0, st>>>(A, n, W);
}

// ------------------------------------------------------------------ restricted Schwarz
// One workgroup per (patch, 64 owned rows).  The patch's residual entries
// are gathered once into LDS; each of the four waves accumulates its quarter
// of the columns of the owned rows of B_k^{-1} (stored column-major, so one
// step over a column is one coalesced 64-row load, eight loads in flight per
// lane), the partial sums meet in LDS and lane r of the first wave adds
// omega times row r to its owned dof.  TAG only names the finest-level launch.
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

template <typename WT, typename VT, typename AT, bool IS16, int TAG>
__global__ __launch_bounds__(256) void k_ras(RasView v, const WT *__restrict__ W, int w16_kind,
                                             const float *__restrict__ wscale,
                                             const VT *__restrict__ s, VT *__restrict__ e,
                                             AT omega) {
  __shared__ AT xs[kMaxPatch];
  __shared__ AT red[3][64];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int task = blockIdx.x;
  const int k = v.task_patch[task];
  const int r0 = v.task_row0[task];
  const int m = v.pm[k], o = v.po[k];
  const int *d = v.dof + v.pdof_off[k];
  if constexpr (IS16) {
    const float *cs = v.cscale + v.pdof_off[k];
    for (int c = threadIdx.x; c < m; c += 256) xs[c] = (AT)s[d[c]] * (AT)cs[c];
  } else {
    for (int c = threadIdx.x; c < m; c += 256) xs[c] = (AT)s[d[c]];
  }
  __syncthreads();
  const int row = r0 + lane;
  const int quarter = (m + 3) >> 2;
  const int c0 = wave * quarter, c1 = min(m, c0 + quarter);
  AT acc = 0;
  if (row < o) {
    const WT *w = W + v.woff[k] + row;
    AT a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int c = c0;
    for (; c + 8 <= c1; c += 8) {
      AT wv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) wv[u] = wload<WT, AT, IS16>(w, (int64_t)(c + u) * o, w16_kind);
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] += wv[u] * xs[c + u];
    }
    for (; c < c1; ++c) a[0] += wload<WT, AT, IS16>(w, (int64_t)c * o, w16_kind) * xs[c];
    acc = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  }
  if (wave > 0) red[wave - 1][lane] = acc;
  __syncthreads();
  if (wave == 0 && row < o) {
    acc = ((acc + red[0][lane]) + red[1][lane]) + red[2][lane];
    if constexpr (IS16) acc *= (AT)wscale[v.out_off[k] + row];
    const int g = v.out_idx[v.out_off[k] + row];
    e[g] = e[g] + (VT)(omega * acc);
  }
}

void launch_ras_f64(const RasView &v, const double *W, const double *s, double *e, double omega,
                    bool finest, hipStream_t st) {
  if (v.ntask == 0) return;
  if (finest)
    k_ras<double, double, double, false, 1><<<v.ntask, 256, 0, st>>>(v, W, 0, nullptr, s, e, omega);
  else
    k_ras<double, double, double, false, 0><<<v.ntask, 256, 0, st>>>(v, W, 0, nullptr, s, e, omega);
}
void launch_ras_f32(const RasView &v, const float *W, const float *s, float *e, float omega,
                    bool finest, hipStream_t st) {
  if (v.ntask == 0) return;
  if (finest)
    k_ras<float, float, float, false, 1><<<v.ntask, 256, 0, st>>>(v, W, 0, nullptr, s, e, omega);
  else
    k_ras<float, float, float, false, 0><<<v.ntask, 256, 0, st>>>(v, W, 0, nullptr, s, e, omega);
}
void launch_ras_16(const RasView &v, const uint16_t *W, int w16_kind, const float *wscale,
                   const float *s, float *e, float omega, bool finest, hipStream_t st) {
  if (v.ntask == 0) return;
  if (finest)
    k_ras<uint16_t, float, float, true, 1><<<v.ntask, 256, 0, st>>>(v, W, w16_kind, wscale, s, e, omega);
  else
    k_ras<uint16_t, float, float, true, 0><<<v.ntask, 256, 0, st>>>(v, W, w16_kind, wscale, s, e, omega);
}

// ------------------------------------------------------------------ coarsest solve GEMV
constexpr int kGemvSplit = 8;
__global__ __launch_bounds__(256) void k_gemv_partial(const double *__restrict__ W, int n,
                                                      const double *__restrict__ x,
                                                      double *__restrict__ partial) {
  __shared__ double red[4][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = blockIdx.x * 64 + lane;
  const int chunk = (n + kGemvSplit - 1) / kGemvSplit;
  const int c0 = blockIdx.y * chunk, c1 = min(n, c0 + chunk);
  double acc = 0.0;
  if (row < n)
    for (int c = c0 + wave; c < c1; c += 4) acc += W[(int64_t)c * n + row] * x[c];
  red[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && row < n)
    partial[(int64_t)blockIdx.y * n + row] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}
__global__ void k_gemv_finish(const double *partial, int n, double *y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int q = 0; q < kGemvSplit; ++q) s += partial[(int64_t)q * n + i];
  y[i] = s;
}
void launch_dense_gemv(const double *W, int n, const double *x, double *y, double *partial,
                       hipStream_t st) {
  dim3 grid(cdiv(n, 64), kGemvSplit);
  k_gemv_partial<<<grid, 256, 0, st>>>(W, n, x, partial);
  k_gemv_finish<<<cdiv(n, 256), 256, 0, st>>>(partial, n, y);
}

// ------------------------------------------------------------------ Krylov reductions
__device__ inline double block_sum_256(double v, double *sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ __launch_bounds__(256) void k_mdot(int n, const double *__restrict__ V, int64_t ldv,
                                              int k, const double *__restrict__ w,
                                              double *__restrict__ partial, int ldp) {
  __shared__ double sh[4];
  const int chunk = (n + kMdotBlocks - 1) / kMdotBlocks;
  const int r0 = blockIdx.x * chunk, r1 = min(n, r0 + chunk);
  for (int i = 0; i < k; ++i) {
    const double *Vi = V + (int64_t)i * ldv;
    double acc = 0.0;
    for (int r = r0 + threadIdx.x; r < r1; r += 256) acc += Vi[r] * w[r];
    const double s = block_sum_256(acc, sh);
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * ldp + i] = s;
  }
}
void launch_mdot(int n, const double *V, int64_t ldv, int k, const double *w, double *partial,
                 int ldp, hipStream_t st) {
  k_mdot<<<kMdotBlocks, 256, 0, st>>>(n, V, ldv, k, w, partial, ldp);
}
__global__ void k_mdot_finish(const double *partial, int ldp, int k, double *out, int acc) {
  const int i = threadIdx.x;
  if (i >= k) return;
  double s = 0.0;
  for (int b = 0; b < kMdotBlocks; ++b) s += partial[(int64_t)b * ldp + i];
  out[i] = acc ? out[i] + s : s;
}
void launch_mdot_finish(const double *partial, int ldp, int k, double *out, int accumulate,
                        hipStream_t st) {
  k_mdot_finish<<<1, 64, 0, st>>>(partial, ldp, k, out, accumulate);
}

__global__ __launch_bounds__(256) void k_mupdate(int n, const double *__restrict__ V, int64_t ldv,
                                                 int k, const double *__restrict__ h,
                                                 double *__restrict__ w,
                                                 double *__restrict__ norm_partial) {
  __shared__ double sh[4];
  __shared__ double hs[64];
  if (threadIdx.x < k) hs[threadIdx.x] = h[threadIdx.x];
  __syncthreads();
  const int chunk = (n + kMdotBlocks - 1) / kMdotBlocks;
  const int r0 = blockIdx.x * chunk, r1 = min(n, r0 + chunk);
  double nacc = 0.0;
  for (int r = r0 + threadIdx.x; r < r1; r += 256) {
    double s = 0.0;
    for (int i = 0; i < k; ++i) s += V[(int64_t)i * ldv + r] * hs[i];
    const double nv = w[r] - s;
    w[r] = nv;
    nacc += nv * nv;
  }
  if (norm_partial) {
    const double t = block_sum_256(nacc, sh);
    if (threadIdx.x == 0) norm_partial[blockIdx.x] = t;
  }
}
void launch_mupdate(int n, const double *V, int64_t ldv, int k, const double *h, double *w,
                    double *norm_partial, hipStream_t st) {
  k_mupdate<<<kMdotBlocks, 256, 0, st>>>(n, V, ldv, k, h, w, norm_partial);
}

// single thread: Arnoldi column bookkeeping and Givens rotations
__global__ void k_givens(double *H, int ldh, int j, const double *h, const double *nrm2,
                         double *cs, double *sn, double *g, double *flags, double *scal) {
  if (threadIdx.x != 0) return;
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
void launch_givens(double *H, int ldh, int j, const double *h, const double *nrm2, double *cs,
                   double *sn, double *g, double *flags, double *scal, hipStream_t st) {
  k_givens<<<1, 64, 0, st>>>(H, ldh, j, h, nrm2, cs, sn, g, flags, scal);
}
__global__ void k_scale_to(int n, const double *w, const double *scal, double *v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const double hn = scal[0];
  if (i < n && hn > 0.0) v[i] = w[i] / hn;
}
void launch_scale_to(int n, const double *w, const double *scal, double *v, hipStream_t st) {
  k_scale_to<<<cdiv(n, 256), 256, 0, st>>>(n, w, scal, v);
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
  if (threadIdx.x < k) ys[threadIdx.x] = y[threadIdx.x];
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

}  // namespace fsi

namespace fsi {
__global__ void k_csr_to_dense(int n, const int *rowptr, const int *col, const double *val,
                               double *A) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  for (int p = rowptr[r]; p < rowptr[r + 1]; ++p) A[(int64_t)r * n + col[p]] = val[p];
}
void launch_csr_to_dense(const CsrView<double> &A, double *dense, hipStream_t st) {
  if (A.nrows > 0)
    k_csr_to_dense<<<cdiv(A.nrows, 256), 256, 0, st>>>(A.nrows, A.rowptr, A.col, A.val, dense);
}
}  // namespace fsi
