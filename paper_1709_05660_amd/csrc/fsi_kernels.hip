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

// Panel phase on a panel P (row stride ps) of m rows and w columns whose
// column t corresponds to pivot p0 + t.  fcol: m scratch doubles.  Executed
// by one workgroup of nthr threads.  Returns 0 or 1 + failing pivot.
template <int NTHR>
__device__ int panel_phase(double *P, int ps, int m, int p0, int w, double *fcol, int *swaps,
                           Argmax *red, int *s_flag) {
  const int tid = threadIdx.x;
  for (int t = 0; t < w; ++t) {
    const int p = p0 + t;
    Argmax best{-1.0, 0x7fffffff};
    for (int i = p + tid; i < m; i += NTHR) {
      const double a = fabs(P[(int64_t)i * ps + t]);
      best = better(best, Argmax{a != a ? INFINITY : a, i});
    }
    best = wave_argmax(best);
    if ((tid & 63) == 0) red[tid >> 6] = best;
    __syncthreads();
    if (tid == 0) {
      Argmax b = red[0];
      for (int q = 1; q < NTHR / 64; ++q) b = better(b, red[q]);
      swaps[p] = b.i;
      s_flag[0] = (!(b.v > 0.0) || isinf(b.v)) ? p + 1 : 0;
    }
    __syncthreads();
    if (s_flag[0]) return s_flag[0];
    const int piv = swaps[p];
    if (piv != p) {
      for (int c = tid; c < w; c += NTHR) {
        const double a = P[(int64_t)p * ps + c];
        P[(int64_t)p * ps + c] = P[(int64_t)piv * ps + c];
        P[(int64_t)piv * ps + c] = a;
      }
    }
    __syncthreads();
    const double d = 1.0 / P[(int64_t)p * ps + t];
    for (int i = tid; i < m; i += NTHR) fcol[i] = P[(int64_t)i * ps + t];
    __syncthreads();
    for (int c = tid; c < w; c += NTHR)
      P[(int64_t)p * ps + c] = (c == t) ? d : P[(int64_t)p * ps + c] * d;
    __syncthreads();
    for (int64_t idx = tid; idx < (int64_t)m * w; idx += NTHR) {
      const int i = (int)(idx / w);
      const int c = (int)(idx % w);
      if (i == p) continue;
      const double f = fcol[i];
      P[(int64_t)i * ps + c] = (c == t) ? -f * d : P[(int64_t)i * ps + c] - f * P[(int64_t)p * ps + c];
    }
    __syncthreads();
  }
  return 0;
}

template <int NB>
__global__ __launch_bounds__(256) void k_gj_batched(double *blocks, const int64_t *boff,
                                                    const int *pm, int *status) {
  extern __shared__ double lds[];
  __shared__ int swaps[kMaxPatch];
  __shared__ Argmax red[4];
  __shared__ int s_flag[1];
  const int k = blockIdx.x;
  const int m = pm[k];
  double *A = blocks + boff[k];
  double *P = lds;             // m x NB panel
  double *fcol = lds + (int64_t)m * NB;
  const int tid = threadIdx.x;
  int fail = 0;
  for (int p0 = 0; p0 < m && !fail; p0 += NB) {
    const int w = min(NB, m - p0);
    for (int64_t idx = tid; idx < (int64_t)m * w; idx += 256) {
      const int i = (int)(idx / w), c = (int)(idx % w);
      P[i * NB + c] = A[(int64_t)i * m + p0 + c];
    }
    __syncthreads();
    fail = panel_phase<256>(P, NB, m, p0, w, fcol, swaps, red, s_flag);
    if (fail) break;
    for (int64_t idx = tid; idx < (int64_t)m * w; idx += 256) {
      const int i = (int)(idx / w), c = (int)(idx % w);
      A[(int64_t)i * m + p0 + c] = P[i * NB + c];
    }
    // rank-w update of the other columns (threads own columns: coalesced rows)
    for (int j = tid; j < m; j += 256) {
      if (j >= p0 && j < p0 + w) continue;
      double X[NB];
#pragma unroll
      for (int t = 0; t < NB; ++t) {
        if (t < w) {
          const int pr = p0 + t, sw = swaps[pr];
          if (sw != pr) {
            const double a = A[(int64_t)pr * m + j];
            A[(int64_t)pr * m + j] = A[(int64_t)sw * m + j];
            A[(int64_t)sw * m + j] = a;
          }
        }
      }
#pragma unroll
      for (int t = 0; t < NB; ++t) X[t] = (t < w) ? A[(int64_t)(p0 + t) * m + j] : 0.0;
      for (int i = 0; i < m; ++i) {
        double acc = (i >= p0 && i < p0 + w) ? 0.0 : A[(int64_t)i * m + j];
        const double *Pi = P + i * NB;
#pragma unroll
        for (int t = 0; t < NB; ++t) acc += Pi[t] * X[t];
        A[(int64_t)i * m + j] = acc;
      }
    }
    __threadfence_block();
    __syncthreads();
  }
  if (!fail) {
    // un-permute columns in reverse order of the row swaps (threads own rows)
    for (int i = tid; i < m; i += 256) {
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

int gj_panel_width(int mmax) {
  const int64_t budget = 150 * 1024;
  if ((int64_t)mmax * 33 * 8 <= budget) return 32;
  if ((int64_t)mmax * 17 * 8 <= budget) return 16;
  return 8;
}

void launch_gj_batched(double *blocks, const int64_t *boff, const int *pm, int npatch, int mmax,
                       int *status, hipStream_t st) {
  if (npatch == 0) return;
  const int nb = gj_panel_width(mmax);
  const size_t shm = (size_t)mmax * (nb + 1) * sizeof(double);
  if (nb == 32) {
    (void)hipFuncSetAttribute((const void *)k_gj_batched<32>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)shm);
    k_gj_batched<32><<<npatch, 256, shm, st>>>(blocks, boff, pm, status);
  } else if (nb == 16) {
    (void)hipFuncSetAttribute((const void *)k_gj_batched<16>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)shm);
    k_gj_batched<16><<<npatch, 256, shm, st>>>(blocks, boff, pm, status);
  } else {
    (void)hipFuncSetAttribute((const void *)k_gj_batched<8>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)shm);
    k_gj_batched<8><<<npatch, 256, shm, st>>>(blocks, boff, pm, status);
  }
}

// ---- large single matrix (coarsest operator): panel in global memory, many
// workgroups for the rank-w update.
constexpr int kLargeNB = 16;
__global__ __launch_bounds__(1024) void k_gj_large_panel(double *A, int n, int p0, int w,
                                                         double *fcol, int *swaps, int *status) {
  __shared__ Argmax red[16];
  __shared__ int s_flag[1];
  if (status[0]) return;
  const int f = panel_phase<1024>(A + p0, n, n, p0, w, fcol, swaps, red, s_flag);
  if (threadIdx.x == 0 && f) status[0] = f;
}
// apply the panel's swaps to the non-panel columns and copy the pivot rows to X (w x n)
__global__ void k_gj_large_swap(double *A, int n, int p0, int w, const int *swaps, double *X,
                                const int *status) {
  if (status[0]) return;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n || (j >= p0 && j < p0 + w)) return;
  for (int t = 0; t < w; ++t) {
    const int pr = p0 + t, sw = swaps[pr];
    if (sw != pr) {
      const double a = A[(int64_t)pr * n + j];
      A[(int64_t)pr * n + j] = A[(int64_t)sw * n + j];
      A[(int64_t)sw * n + j] = a;
    }
  }
  for (int t = 0; t < w; ++t) X[(int64_t)t * n + j] = A[(int64_t)(p0 + t) * n + j];
}
// rows split over blockIdx.y, columns over threads
__global__ __launch_bounds__(256) void k_gj_large_update(double *A, int n, int p0, int w,
                                                         const double *X, const int *status) {
  if (status[0]) return;
  __shared__ double Pn[64 * kLargeNB];
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i0 = blockIdx.y * 64;
  const int i1 = min(n, i0 + 64);
  for (int idx = threadIdx.x; idx < (i1 - i0) * w; idx += blockDim.x) {
    const int i = idx / w, t = idx % w;
    Pn[i * kLargeNB + t] = A[(int64_t)(i0 + i) * n + p0 + t];
  }
  __syncthreads();
  if (j >= n || (j >= p0 && j < p0 + w)) return;
  double Xr[kLargeNB];
#pragma unroll
  for (int t = 0; t < kLargeNB; ++t) Xr[t] = (t < w) ? X[(int64_t)t * n + j] : 0.0;
  for (int i = i0; i < i1; ++i) {
    double acc = (i >= p0 && i < p0 + w) ? 0.0 : A[(int64_t)i * n + j];
#pragma unroll
    for (int t = 0; t < kLargeNB; ++t) acc += Pn[(i - i0) * kLargeNB + t] * Xr[t];
    A[(int64_t)i * n + j] = acc;
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

// work: n (fcol) + n (swaps as int, stored in doubles' space) + kLargeNB * n (X)
void gj_large(double *A, int n, int *status_dev, double *work, hipStream_t st) {
  double *fcol = work;
  int *swaps = reinterpret_cast<int *>(work + n);
  double *X = work + 2 * (int64_t)n;
  for (int p0 = 0; p0 < n; p0 += kLargeNB) {
    const int w = std::min(kLargeNB, n - p0);
    k_gj_large_panel<<<1, 1024, 0, st>>>(A, n, p0, w, fcol, swaps, status_dev);
    k_gj_large_swap<<<cdiv(n, 256), 256, 0, st>>>(A, n, p0, w, swaps, X, status_dev);
    dim3 grid(cdiv(n, 256), cdiv(n, 64));
    k_gj_large_update<<<grid, 256, 0, st>>>(A, n, p0, w, X, status_dev);
  }
  k_gj_large_unpermute<<<cdiv(n, 256), 256, 0, st>>>(A, n, swaps, status_dev);
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
                                                    float *wscale) {
  const int64_t t = blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (t >= total_owned) return;
  const int k = orow_patch[t];
  const int r = orow_r[t];
  const int m = pm[k], o = po[k];
  const double *row = blocks + boff[k] + (int64_t)own_local[own_off[k] + r] * m;
  double mx = 0.0;
  if (W16) {
    for (int c = lane; c < m; c += 64) mx = fmax(mx, fabs(row[c]));
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
    if (W16) W16[dst] = w16_kind == 1 ? to_bf16((float)(v / mx)) : to_fp16((float)(v / mx));
  }
}

void launch_pack_owned(const double *blocks, const int64_t *boff, const int *pm, const int *po,
                       const int64_t *woff, const int *own_off, const int *own_local, int npatch,
                       int64_t total_owned, const int *orow_patch, const int *orow_r, double *W64,
                       float *W32, uint16_t *W16, int w16_kind, float *wscale, hipStream_t st) {
  (void)npatch;
  if (total_owned == 0) return;
  k_pack_owned<<<cdiv(total_owned, 4), 256, 0, st>>>(blocks, boff, pm, po, woff, own_off,
                                                      own_local, total_owned, orow_patch, orow_r,
                                                      W64, W32, W16, w16_kind, wscale);
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
// One wave per (patch, 64 owned rows): the patch's residual entries are
// gathered into the wave's LDS slice, then each lane accumulates one owned
// row of B_k^{-1} (stored column-major, so a step over a column is one
// coalesced 64-row load) and adds omega times it to its owned dof.
template <typename WT>
__device__ inline float w16val(WT v, int kind);
template <>
__device__ inline float w16val<uint16_t>(uint16_t v, int kind) {
  return kind == 1 ? from_bf16(v) : from_fp16(v);
}

template <typename WT, typename VT, typename AT, bool IS16>
__global__ __launch_bounds__(256) void k_ras(RasView v, const WT *__restrict__ W, int w16_kind,
                                             const float *__restrict__ wscale,
                                             const VT *__restrict__ s, VT *__restrict__ e,
                                             AT omega) {
  __shared__ AT xs[4][kMaxPatch];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int task = blockIdx.x * 4 + wave;
  const bool valid = task < v.ntask;
  int k = 0, r0 = 0, m = 0, o = 0;
  if (valid) {
    k = v.task_patch[task];
    r0 = v.task_row0[task];
    m = v.pm[k];
    o = v.po[k];
    const int *d = v.dof + v.pdof_off[k];
    for (int c = lane; c < m; c += 64) xs[wave][c] = (AT)s[d[c]];
  }
  __syncthreads();
  if (!valid) return;
  const int row = r0 + lane;
  if (row >= o) return;
  const WT *w = W + v.woff[k] + row;
  const AT *x = xs[wave];
  AT a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  int c = 0;
  for (; c + 4 <= m; c += 4) {
    AT w0, w1, w2, w3;
    if constexpr (IS16) {
      w0 = w16val<WT>(w[(int64_t)c * o], w16_kind);
      w1 = w16val<WT>(w[(int64_t)(c + 1) * o], w16_kind);
      w2 = w16val<WT>(w[(int64_t)(c + 2) * o], w16_kind);
      w3 = w16val<WT>(w[(int64_t)(c + 3) * o], w16_kind);
    } else {
      w0 = (AT)w[(int64_t)c * o];
      w1 = (AT)w[(int64_t)(c + 1) * o];
      w2 = (AT)w[(int64_t)(c + 2) * o];
      w3 = (AT)w[(int64_t)(c + 3) * o];
    }
    a0 += w0 * x[c];
    a1 += w1 * x[c + 1];
    a2 += w2 * x[c + 2];
    a3 += w3 * x[c + 3];
  }
  for (; c < m; ++c) {
    AT wv;
    if constexpr (IS16)
      wv = w16val<WT>(w[(int64_t)c * o], w16_kind);
    else
      wv = (AT)w[(int64_t)c * o];
    a0 += wv * x[c];
  }
  AT acc = (a0 + a1) + (a2 + a3);
  if constexpr (IS16) acc *= (AT)wscale[v.out_off[k] + row];
  const int g = v.out_idx[v.out_off[k] + row];
  e[g] = e[g] + (VT)(omega * acc);
}

void launch_ras_f64(const RasView &v, const double *W, const double *s, double *e, double omega,
                    hipStream_t st) {
  if (v.ntask == 0) return;
  k_ras<double, double, double, false><<<cdiv(v.ntask, 4), 256, 0, st>>>(v, W, 0, nullptr, s, e,
                                                                          omega);
}
void launch_ras_f32(const RasView &v, const float *W, const float *s, float *e, float omega,
                    hipStream_t st) {
  if (v.ntask == 0) return;
  k_ras<float, float, float, false><<<cdiv(v.ntask, 4), 256, 0, st>>>(v, W, 0, nullptr, s, e,
                                                                       omega);
}
void launch_ras_16(const RasView &v, const uint16_t *W, int w16_kind, const float *wscale,
                   const float *s, float *e, float omega, hipStream_t st) {
  if (v.ntask == 0) return;
  k_ras<uint16_t, float, float, true><<<cdiv(v.ntask, 4), 256, 0, st>>>(v, W, w16_kind, wscale,
                                                                         s, e, omega);
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
