// gfx950 Gauss-Jordan inversions of the setup: the explicit inverses of the
// Schwarz blocks B_k of every smoothing level (one workgroup per block, all
// levels in one launch) and of the coarsest operator (one workgroup factors
// each pivot panel, a grid of workgroups applies it to the other columns).
//
// Both are the same blocked right-looking Gauss-Jordan elimination with
// partial pivoting (largest magnitude among the rows not yet used as pivots,
// compared to 39 significant bits, lowest row on ties).  A panel of NB pivot
// columns is factored with its rows held in registers: thread t holds rows
// t, t + NT, ...  A pivot step costs one workgroup barrier: each wave reduces
// its candidates' keys (magnitude and row in one double) with DPP, publishes
// its best candidate row in LDS (double-buffered by step parity), and every
// thread then takes the best of the waves' keys and eliminates that row from
// its own rows.
//
// Rows are never exchanged.  The pivot row of step s is recorded as
// perm[s], the step at which row i served as pivot as used[i], and the
// stored result S is the inverse up to these two permutations,
//     inv(A)[k][c] = S[perm[k]][used[c]],
// which the consumers (the owned-row packing, the coarse transpose) apply
// as they read S.  A factored panel PC (rows of S in the panel's columns)
// acts on every other column j by
//     A[i][j] <- [i is not a pivot row of the panel] A[i][j]
//                + sum_t PC[i][t] X[t][j],
// where X[t][j] is the panel's t-th pivot row before the update.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cfloat>
#include <climits>
#include <cmath>
#include <functional>
#include <queue>
#include <vector>

#include "fsi_kernels.h"

namespace fsi {

static inline int cdivg(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

constexpr int kNoRow = 0x7fffffff;

// DPP move of a double to a fresh register (full EXEC, every row written)
template <int CTRL>
__device__ __forceinline__ double mov_dpp_f64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// DPP move of a double (full EXEC); rows outside ROWS keep their own value
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp_f64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp((int)b, (int)b, CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(b >> 32), (int)(b >> 32), CTRL, ROWS, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double readlane_f64(double x, int l) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// DPP controls: quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_ror 4, row_ror 8,
// row_bcast 15 (lane 15 of each row into the next row), row_bcast 31 (lane 31
// into rows 2 and 3)
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppRor4 = 0x124, kDppRor8 = 0x128;
constexpr int kDppBcast15 = 0x142, kDppBcast31 = 0x143;

// Pivot keys.  A candidate row i with entry a in the pivot column is keyed
// by |a| with its lowest 13 mantissa bits replaced by 8191 - i (rows are
// below 8192): keys order by |a| to 39 significant bits, then by the lowest
// row, and a plain fmax reduces them (positive doubles order as their bit
// patterns).  A non-finite |a| keys as the largest finite double, which
// fails the step; rows that are not candidates carry -1.
constexpr long long kKeyMask = (1LL << 13) - 1;
__device__ __forceinline__ double pivot_key(double a, int i) {
  double x = fabs(a);
  if (!(x <= DBL_MAX)) x = DBL_MAX;   // NaN or infinite
  return __longlong_as_double((__double_as_longlong(x) & ~kKeyMask) | (kKeyMask - i));
}
__device__ __forceinline__ int key_row(double k) {
  return (int)(kKeyMask - (__double_as_longlong(k) & kKeyMask));
}
__device__ __forceinline__ double key_value(double k) {
  return __longlong_as_double(__double_as_longlong(k) & ~kKeyMask);
}

// max of two pivot keys.  Keys are never NaN, so with RAW the plain
// instruction is used (fmax first quiets possible signalling NaNs of both
// operands); the asm statement limits the scheduler, so kernels whose panel
// already fills most registers keep fmax.
template <bool RAW>
__device__ __forceinline__ double key_max(double a, double b) {
  if constexpr (RAW) {
    double r;
    asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
  } else {
    return fmax(a, b);
  }
}

// wave-wide maximum of a key, the same value in every lane: DPP inside each
// row of 16 lanes, then row broadcasts carry the running maximum into the
// last row, whose lane 63 is read.  Requires all 64 lanes active.
template <bool RAW>
__device__ __forceinline__ double wave_max(double v) {
  v = key_max<RAW>(v, mov_dpp_f64<kDppXor1>(v));
  v = key_max<RAW>(v, mov_dpp_f64<kDppXor2>(v));
  v = key_max<RAW>(v, mov_dpp_f64<kDppRor4>(v));
  v = key_max<RAW>(v, mov_dpp_f64<kDppRor8>(v));
  v = key_max<RAW>(v, dpp_f64<kDppBcast15, 0xA>(v));   // rows 1, 3: max with rows 0, 2
  v = key_max<RAW>(v, dpp_f64<kDppBcast31, 0xC>(v));   // rows 2, 3: max with row 1
  return readlane_f64(v, 63);
}

// 1 / a from the hardware reciprocal refined by two Newton steps: within an
// ulp of the rounded quotient for 2^-1021 <= |a| <= 2^1021 (outside that range
// the result may be 0 or NaN; such a pivot leaves the block unusable anyway)
__device__ __forceinline__ double recip(double a) {
  double x = __builtin_amdgcn_rcp(a);
  x = fma(x, fma(-a, x, 1.0), x);
  x = fma(x, fma(-a, x, 1.0), x);
  return x;
}

// LDS of the pivot steps: one candidate row (with the reciprocal of its
// pivot-column entry and its key) per wave and step parity, and the panel's
// pivot rows in step order.
template <int NB, int NW, typename T = double>
struct PivotLds {
  T row[2][NW][NB];
  double key[2][NW];
  T dinv[2][NW];
  int piv[NB];
};

// 1 / a in single precision: the hardware reciprocal and one Newton step
__device__ __forceinline__ float recip(float a) {
  float x = __builtin_amdgcn_rcpf(a);
  return fmaf(x, fmaf(-a, x, 1.0f), x);
}

// One pivot step on column t of the panel held in v (see reg_panel).
// Returns 0 or 1 + the failing step, uniformly.  RAW: see key_max.
// T: the element type of the rows (double, or float for the mixed forms'
// working matrices); the keys are doubles in both cases (a float magnitude
// converts exactly and leaves the low mantissa bits to the row number).
template <int NB, int R, int NT, bool RAW, typename T>
__device__ __forceinline__ int pivot_step(T (&v)[R][NB], int (&stp)[R], int m, int p0, int t,
                                          int col, PivotLds<NB, NT / 64, T> &sh, int &mypiv) {
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int buf = t & 1;
  double key = -1.0;   // this lane's best key and its signed pivot-column entry
  T sv = 1;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int i = tid + q * NT;
    if (i < m && stp[q] < 0) {
      const double kq = pivot_key((double)v[q][col], i);
      if (kq > key) {
        key = kq;
        sv = v[q][col];
      }
    }
  }
  // every lane inverts its own candidate while the wave reduction runs;
  // the winner publishes its row and reciprocal
  const T dl = recip(sv);
  const double wkey = wave_max<RAW>(key);
  if (wkey >= 0.0 && key == wkey) {
    const int i = key_row(key);
#pragma unroll
    for (int q = 0; q < R; ++q)
      if (tid + q * NT == i) {
#pragma unroll
        for (int c = 0; c < NB; ++c) sh.row[buf][wave][c] = v[q][c];
      }
    sh.dinv[buf][wave] = dl;
  }
  if (lane == 0) sh.key[buf][wave] = wkey;
  __syncthreads();
  // the waves' keys combined by a tree
  double kk[NW];
#pragma unroll
  for (int k = 0; k < NW; ++k) kk[k] = sh.key[buf][k];
#pragma unroll
  for (int s2 = 1; s2 < NW; s2 <<= 1)
#pragma unroll
    for (int k = 0; k + s2 < NW; k += 2 * s2) kk[k] = key_max<RAW>(kk[k], kk[k + s2]);
  const double gkey = kk[0];
  const double gv = key_value(gkey);
  if (!(gkey >= 0.0) || !(gv > 0.0) || gv >= key_value(pivot_key(DBL_MAX, 0))) return p0 + t + 1;
  const int gi = key_row(gkey);
  const int gw = (gi % NT) >> 6;
  if (tid == 0) sh.piv[t] = gi;
  if (tid == t) mypiv = gi;
  const T *prow = sh.row[buf][gw];
  const T d = sh.dinv[buf][gw];
  // every row is eliminated with one FMA per column, v - (f d) prow, then
  // the one lane holding the pivot row overwrites it with prow d (a branch
  // of one lane instead of a select on every row)
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const T fd = v[q][col] * d;
#pragma unroll
    for (int c = 0; c < NB; ++c) v[q][c] = c == col ? -fd : v[q][c] - fd * prow[c];
  }
#pragma unroll
  for (int q = 0; q < R; ++q)
    if (tid + q * NT == gi) {
#pragma unroll
      for (int c = 0; c < NB; ++c) v[q][c] = c == col ? d : prow[c] * d;
      stp[q] = p0 + t;
    }
  return 0;
}

// Factors the panel of columns [p0, p0 + w) of an m-row matrix whose rows
// tid + q * NT sit in v[q][0..NB) (columns beyond w are zero; rows beyond m
// are never candidates); stp[q] is the step at which that row became a
// pivot (< 0: not yet; rows beyond m carry kNoRow).  Thread t receives the
// pivot row of step t in mypiv.  RAW: see key_max.  UNR: the NB steps are
// unrolled and step t works on the static column t.  Otherwise the step loop
// is rolled: the current pivot column is always v[q][0] and each step
// rotates the row left by one column (every register index stays static),
// the columns being back in order after NB rotations.  Called by all NT
// threads.  Returns 0, or 1 + the step whose pivot is zero or not finite
// (the same value in every thread).
template <int NB, int R, int NT, bool UNR, bool RAW, typename T>
__device__ __forceinline__ int reg_panel(T (&v)[R][NB], int (&stp)[R], int m, int p0, int w,
                                         PivotLds<NB, NT / 64, T> &sh, int &mypiv) {
  if constexpr (UNR) {
#pragma unroll
    for (int t = 0; t < NB; ++t)
      if (t < w) {
        const int f = pivot_step<NB, R, NT, RAW, T>(v, stp, m, p0, t, t, sh, mypiv);
        if (f) return f;
      }
  } else {
    for (int t = 0; t < NB; ++t) {
      if (t < w) {
        const int f = pivot_step<NB, R, NT, RAW, T>(v, stp, m, p0, t, 0, sh, mypiv);
        if (f) return f;
      }
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const T h = v[q][0];
#pragma unroll
        for (int c = 0; c + 1 < NB; ++c) v[q][c] = v[q][c + 1];
        v[q][NB - 1] = h;
      }
    }
  }
  return 0;
}

// ------------------------------------------------------------------ batched blocks
typedef double dx4 __attribute__((ext_vector_type(4)));
typedef float fx4 __attribute__((ext_vector_type(4)));
constexpr int kPrefetch = 4;   // row tiles in flight per wave in the updates

// The 16x16x4 matrix-core product of each element type.  Operand layouts are
// the same (A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k); the output
// tile differs: the FP64 instruction holds D[i][j] in lane j + 16 (i % 4),
// register i / 4, the FP32 one in lane j + 16 (i / 4), register i % 4.
template <typename T>
struct Mfma16;
template <>
struct Mfma16<double> {
  typedef dx4 acc;
  static __device__ __forceinline__ acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int r, int kq) { return r * 4 + kq; }
};
template <>
struct Mfma16<float> {
  typedef fx4 acc;
  static __device__ __forceinline__ acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int r, int kq) { return kq * 4 + r; }
};

// T: FP64 (the plain form) or FP32 (the mixed forms: the working matrix and
// the matrix-core products in single precision, the pivot keys in double).
// One workgroup of NT threads per block at a time (m <= NT R), looping
// over the blocks the schedule gives it: sched[0..grid] are offsets into
// the block list sched[grid + 1 ..] (see gj_schedule).  Per panel: factor in
// registers, store the panel to the block and to LDS (stride NB + 1), then
// apply it to the other columns on the matrix cores: each wave owns whole
// 16-column tiles, reads its tiles' X (the pivot rows' old values) first and
// then updates every 16-row tile, pivot rows included, with
// v_mfma_f64_16x16x4f64 (A: PC rows, B: X; operand layouts: A[i][k] in lane
// i + 16 k, B[k][j] in lane j + 16 k, D[i][j] in lane j + 16 (i % 4),
// register i / 4), the tiles' loads issued kPrefetch tiles ahead.  The block array is padded by NB doubles at its end:
// a panel slice is loaded whole from its row base.  GPC: the update reads
// the panel from the block's own panel columns (just written, in L2)
// instead of an LDS copy, so NB = 32 needs no LDS of m (NB + 1) doubles.
template <typename T, int NB, int R, int NT, bool UNR, bool GPC>
__global__ __launch_bounds__(NT) void k_gj_batched(T *__restrict__ blocks,
                                                    const int64_t *__restrict__ boff,
                                                    const int *__restrict__ pm,
                                                    const int64_t *__restrict__ poff,
                                                    int *__restrict__ perm_all,
                                                    int *__restrict__ used_all,
                                                    int *__restrict__ status,
                                                    const int *__restrict__ sched) {
  typedef Mfma16<T> MM;
  typedef typename MM::acc acc;
  constexpr int PS = NB + 1, KC = NB / 4;
  extern __shared__ __align__(16) unsigned char gj_dyn_lds[];
  T *PC = reinterpret_cast<T *>(gj_dyn_lds);
  __shared__ PivotLds<NB, NT / 64, T> sh;
  __shared__ short s_used[R * NT];   // step numbers < 1024, or -1
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int jl = lane & 15, kq = lane >> 4;
  const int *list = sched + gridDim.x + 1;
  for (int t = sched[blockIdx.x]; t < sched[blockIdx.x + 1]; ++t) {
    const int k = list[t];
    const int m = pm[k];
    T *A = blocks + boff[k];
    int *perm = perm_all + poff[k];
    for (int i = tid; i < m; i += NT) s_used[i] = -1;
    __syncthreads();
    int fail = 0;
    for (int p0 = 0; p0 < m; p0 += NB) {
      const int w = min(NB, m - p0);
      T v[R][NB];
      int stp[R];
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int i = tid + q * NT;
        stp[q] = i < m ? s_used[i] : kNoRow;
        const T *row = A + min(i, m - 1) * m + p0;
#pragma unroll
        for (int c = 0; c < NB; ++c) v[q][c] = row[c];
      }
#pragma unroll
      for (int q = 0; q < R; ++q)
#pragma unroll
        for (int c = 0; c < NB; ++c)
          if (c >= w) v[q][c] = 0;
      int mypiv = 0;   // unused here: the update reads the pivots from LDS
      fail = reg_panel<NB, R, NT, UNR, false>(v, stp, m, p0, w, sh, mypiv);
      if (fail) break;
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int i = tid + q * NT;
        if (i < m) {
#pragma unroll
          for (int c = 0; c < NB; ++c) {
            if (c < w) A[i * m + p0 + c] = v[q][c];
            if constexpr (!GPC) PC[i * PS + c] = v[q][c];
          }
          if (stp[q] >= p0) s_used[i] = (short)stp[q];
        }
      }
      __threadfence_block();
      __syncthreads();
      if (tid < w) perm[p0 + tid] = sh.piv[tid];
      const int mp = m - w;
      const int nct = (mp + 15) >> 4, nrt = (m + 15) >> 4;
      for (int ct = wave; ct < nct; ct += NT / 64) {
        const int q = ct * 16 + jl;
        const bool colok = q < mp;
        const int j = colok ? (q < p0 ? q : q + w) : 0;
        // X: clamped loads issued together, zeroed outside the panel
        T bx[KC];
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) bx[kk] = A[sh.piv[min(kk * 4 + kq, w - 1)] * m + j];
#pragma unroll
        for (int kk = 0; kk < KC; ++kk)
          if (!(colok && kk * 4 + kq < w)) bx[kk] = 0;
        // every load unconditional at a clamped address (prefetches past the
        // last tile repeat it), so no load waits on a branch; the pivot rows
        // and the rows past m are zeroed where the tile is used
        auto load_tile = [&](int rt) {
          acc c;
#pragma unroll
          for (int r = 0; r < 4; ++r) c[r] = A[min(rt * 16 + MM::row(r, kq), m - 1) * m + j];
          return c;
        };
        acc ring[kPrefetch];
#pragma unroll
        for (int u = 0; u < kPrefetch; ++u) ring[u] = load_tile(min(u, nrt - 1));
        for (int rt0 = 0; rt0 < nrt; rt0 += kPrefetch) {
#pragma unroll
          for (int u = 0; u < kPrefetch; ++u) {
            const int rt = rt0 + u;
            acc c = ring[u];
            ring[u] = load_tile(min(rt + kPrefetch, nrt - 1));
            if (rt < nrt) {
              int su[4];
              T a[KC];
              const int ia = rt * 16 + jl;
#pragma unroll
              for (int r = 0; r < 4; ++r) su[r] = s_used[min(rt * 16 + MM::row(r, kq), m - 1)];
#pragma unroll
              for (int kk = 0; kk < KC; ++kk) {
                if constexpr (GPC) {
                  // clamped to the panel's last column, zeroed beyond it
                  const T x = A[min(ia, m - 1) * m + p0 + min(kk * 4 + kq, w - 1)];
                  a[kk] = kk * 4 + kq < w ? x : (T)0;
                } else {
                  a[kk] = PC[min(ia, m - 1) * PS + kk * 4 + kq];
                }
              }
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int i = rt * 16 + MM::row(r, kq);
                if (!(colok && i < m && (su[r] < p0 || su[r] >= p0 + w))) c[r] = 0;
              }
#pragma unroll
              for (int kk = 0; kk < KC; ++kk) c = MM::mma(ia < m ? a[kk] : (T)0, bx[kk], c);
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int i = rt * 16 + MM::row(r, kq);
                if (colok && i < m) A[i * m + j] = c[r];
              }
            }
          }
        }
      }
      __threadfence_block();
      __syncthreads();
    }
    // a failed block publishes the identity permutation, so that the packing
    // (which runs before the host reads the status) stays inside the block
    __syncthreads();
    for (int i = tid; i < m; i += NT) {
      used_all[poff[k] + i] = fail ? i : s_used[i];
      if (fail) perm[i] = i;
    }
    if (tid == 0) status[k] = fail;
    __syncthreads();
  }
}

// Applies a factored panel (steps [kb, kb + kw), its columns in the block,
// pivot rows xrows[0..kw)) to a set of columns of an m x m block: the
// columns [c_lo, c_lo + cn) when inside, else every column outside that
// range.  Each wave owns the 16-row tiles wave, wave + NW, ... (at most RT)
// and holds their panel rows (the A operand) in registers for the whole
// update.  The columns go by chunks of CW; the chunk's X (the pivot rows'
// old values) sits in LDS (Xs: two buffers of 4 KCX x CW, the next chunk's
// read from the block while the current one is computed), and every wave
// loads all its C tiles of the chunk, zeroes the pivot rows and accumulates
// on the matrix cores.  One barrier per chunk.  Called by all NT threads
// (the early return for an empty column set is uniform); ends with a barrier
// when it updates anything.
template <typename T, int KCX, int NT, int RT, int CW>
__device__ __forceinline__ void gj_apply_rows(T *__restrict__ A, int m, int kb, int kw, const int *xrows,
                                              int c_lo, int cn, bool inside, const short *s_used, T *Xs) {
  typedef Mfma16<T> MM;
  typedef typename MM::acc acc;
  constexpr int NW = NT / 64, NCT = CW / 16, KR = 4 * KCX, XE = (KR * CW + NT - 1) / NT;
  static_assert(RT * KCX <= 64, "the panel rows of a wave's tiles must fit in registers");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int jl = lane & 15, kq = lane >> 4;
  const int mp = inside ? cn : m - cn;
  if (mp <= 0) return;   // no column to update (a block of at most 2 NB dofs)
  const int nrt = (m + 15) >> 4;
  auto col = [&](int q) { return inside ? c_lo + q : (q < c_lo ? q : q + cn); };
  T ah[RT][KCX];
  unsigned keep = 0;   // bit 4 u + r: C row r of tile u is kept (exists, not a pivot row of the panel)
#pragma unroll
  for (int u = 0; u < RT; ++u) {
    const int rt = wave + NW * u;
    const int ia = min(rt * 16 + jl, m - 1);
#pragma unroll
    for (int kk = 0; kk < KCX; ++kk) {
      const T x = A[ia * m + kb + min(kk * 4 + kq, kw - 1)];
      ah[u][kk] = (rt * 16 + jl < m && kk * 4 + kq < kw) ? x : (T)0;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = rt * 16 + MM::row(r, kq);
      const int su = s_used[min(i, m - 1)];
      if (i < m && (su < kb || su >= kb + kw)) keep |= 1u << (4 * u + r);
    }
  }
  // this thread's share of a chunk's X: element e = tid + x NT is (t, c) =
  // (e / CW, e % CW); clamped loads, zeroed outside
  auto load_x = [&](int q0, T (&xv)[XE]) {
#pragma unroll
    for (int x = 0; x < XE; ++x) {
      const int e = tid + x * NT, t = e / CW, q = q0 + e % CW;
      const T v = A[xrows[min(t, kw - 1)] * m + col(min(q, mp - 1))];
      xv[x] = (e < KR * CW && t < kw && q < mp) ? v : (T)0;
    }
  };
  auto store_x = [&](int buf, const T (&xv)[XE]) {
#pragma unroll
    for (int x = 0; x < XE; ++x) {
      const int e = tid + x * NT;
      if (e < KR * CW) Xs[buf * KR * CW + e] = xv[x];
    }
  };
  {
    T xv[XE];
    load_x(0, xv);
    store_x(0, xv);
  }
  __syncthreads();
  int buf = 0;
  for (int q0 = 0; q0 < mp; q0 += CW, buf ^= 1) {
    int jc[NCT];
    bool cok[NCT];
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
      const int q = q0 + ct * 16 + jl;
      cok[ct] = q < mp;
      jc[ct] = cok[ct] ? col(q) : c_lo;
    }
    acc c[RT][NCT];
#pragma unroll
    for (int u = 0; u < RT; ++u)
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          c[u][ct][r] = A[min((wave + NW * u) * 16 + MM::row(r, kq), m - 1) * m + jc[ct]];
    // the next chunk's X: its columns are not touched by this chunk
    const bool more = q0 + CW < mp;
    T xv[XE];
    if (more) load_x(q0 + CW, xv);
    const T *X = Xs + buf * KR * CW;
#pragma unroll
    for (int u = 0; u < RT; ++u) {
      if (wave + NW * u >= nrt) continue;
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) {
        acc cc = c[u][ct];
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (!((keep >> (4 * u + r)) & 1u)) cc[r] = 0;
#pragma unroll
        for (int kk = 0; kk < KCX; ++kk) cc = MM::mma(ah[u][kk], X[(kk * 4 + kq) * CW + ct * 16 + jl], cc);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = (wave + NW * u) * 16 + MM::row(r, kq);
          if (cok[ct] && i < m) A[i * m + jc[ct]] = cc[r];
        }
      }
    }
    if (more) store_x(buf ^ 1, xv);
    __syncthreads();
  }
}

// The batched inversion with paired panels: two panels of NB columns are
// factored one after the other, each applied at once only to the other's
// columns, and the pair then acts on the rest of the block as one panel of
// 2 NB columns (its pivot rows' old values as X).  The block is streamed once
// per 2 NB pivots instead of once per NB, with the same matrix-core work;
// the result is the same elimination up to rounding (the rest columns take
// the pair's two rank-NB products as one sum).  Schedule, layouts and
// outputs as k_gj_batched.
template <typename T, int NB, int R, int NT>
__global__ __launch_bounds__(NT) void k_gj_paired(T *__restrict__ blocks, const int64_t *__restrict__ boff,
                                                  const int *__restrict__ pm, const int64_t *__restrict__ poff,
                                                  int *__restrict__ perm_all, int *__restrict__ used_all,
                                                  int *__restrict__ status, const int *__restrict__ sched) {
  constexpr int KC = NB / 4;
  __shared__ PivotLds<NB, NT / 64, T> sh;
  __shared__ short s_used[R * NT];
  __shared__ int piv2[2 * NB];
  constexpr int CW = 16, RT = (R * NT / 16 + NT / 64 - 1) / (NT / 64);
  __shared__ T Xs[2 * 2 * NB * CW];
  const int tid = threadIdx.x;
  const int *list = sched + gridDim.x + 1;
  for (int t = sched[blockIdx.x]; t < sched[blockIdx.x + 1]; ++t) {
    const int k = list[t];
    const int m = pm[k];
    T *A = blocks + boff[k];
    int *perm = perm_all + poff[k];
    for (int i = tid; i < m; i += NT) s_used[i] = -1;
    __syncthreads();
    int fail = 0;
    for (int P0 = 0; P0 < m && !fail; P0 += 2 * NB) {
      const int W = min(2 * NB, m - P0);
      for (int sub = 0; sub < 2; ++sub) {
        const int p0 = P0 + sub * NB;
        if (p0 >= P0 + W) break;
        const int w = min(NB, P0 + W - p0);
        T v[R][NB];
        int stp[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int i = tid + q * NT;
          stp[q] = i < m ? s_used[i] : kNoRow;
          const T *row = A + min(i, m - 1) * m + p0;
#pragma unroll
          for (int c = 0; c < NB; ++c) v[q][c] = row[c];
        }
#pragma unroll
        for (int q = 0; q < R; ++q)
#pragma unroll
          for (int c = 0; c < NB; ++c)
            if (c >= w) v[q][c] = 0;
        int mypiv = 0;
        fail = reg_panel<NB, R, NT, true, false>(v, stp, m, p0, w, sh, mypiv);
        if (fail) break;
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int i = tid + q * NT;
          if (i < m) {
#pragma unroll
            for (int c = 0; c < NB; ++c)
              if (c < w) A[i * m + p0 + c] = v[q][c];
            if (stp[q] >= p0) s_used[i] = (short)stp[q];
          }
        }
        __threadfence_block();
        __syncthreads();
        if (tid < w) {
          perm[p0 + tid] = sh.piv[tid];
          piv2[sub * NB + tid] = sh.piv[tid];
        }
        // the pair's other columns: the second panel's after the first, the
        // first's after the second
        const int o0 = sub == 0 ? P0 + NB : P0, on = sub == 0 ? W - NB : NB;
        if (on > 0) gj_apply_rows<T, KC, NT, RT, CW>(A, m, p0, w, sh.piv, o0, on, true, s_used, Xs);
        __threadfence_block();
        __syncthreads();
      }
      if (fail) break;
      // the rest of the block: one update by the pair's 2 NB columns
      gj_apply_rows<T, 2 * KC, NT, RT, CW>(A, m, P0, W, piv2, P0, W, false, s_used, Xs);
      __threadfence_block();
      __syncthreads();
    }
    __syncthreads();
    for (int i = tid; i < m; i += NT) {
      used_all[poff[k] + i] = fail ? i : s_used[i];
      if (fail) perm[i] = i;
    }
    if (tid == 0) status[k] = fail;
    __syncthreads();
  }
}

static size_t gj_batched_lds(int mmax, int nb, size_t elem = sizeof(double)) {
  return (size_t)mmax * (nb + 1) * elem;
}

// static LDS of a kernel instance, queried once per instance (-1: the query failed)
template <typename T, int NB, int R, int NT, bool UNR = true>
static int64_t gj_static_lds() {
  static const int64_t v = [] {
    hipFuncAttributes a;
    return hipFuncGetAttributes(&a, (const void *)k_gj_batched<T, NB, R, NT, UNR, false>) == hipSuccess
               ? (int64_t)a.sharedSizeBytes
               : (int64_t)-1;
  }();
  return v;
}
// the LDS panel (m rows of NB + 1 elements) fits beside the static LDS
template <typename T, int NB, int R, int NT, bool UNR = true>
static bool gj_lds_fits(int mmax) {
  const int64_t st = gj_static_lds<T, NB, R, NT, UNR>();
  return mmax <= R * NT && st >= 0 && st + (int64_t)gj_batched_lds(mmax, NB, sizeof(T)) <= 160 * 1024;
}

template <typename T, int NB, int R, int NT>
static bool gj_paired_fits(int mmax) {
  static const int64_t st = [] {
    hipFuncAttributes a;
    return hipFuncGetAttributes(&a, (const void *)k_gj_paired<T, NB, R, NT>) == hipSuccess
               ? (int64_t)a.sharedSizeBytes
               : (int64_t)-1;
  }();
  return mmax <= R * NT && st >= 0 && st <= 160 * 1024;
}

bool gj_variant_ok(int variant, int mmax) {
  switch (variant) {
    case kGjP32x512:
      return gj_paired_fits<double, 32, 1, 512>(mmax);
    case kGjPF32x512:
      return gj_paired_fits<float, 32, 1, 512>(mmax);
    case kGj16x256:
    case kGj16x512:
      return mmax <= 1024;
    case kGj32x512:   // one row per thread, and the LDS panel next to the static LDS
      return mmax <= 512 && gj_batched_lds(mmax, 32) <= 140 * 1024;
    case kGjWideG:    // panel read from the block itself: no LDS of m
      return mmax <= 1024;
    case kGj24x512:   // two rows per thread, the LDS panel next to the static LDS
      return gj_lds_fits<double, 24, 2, 512>(mmax);
    case kGjF64x512:
      return gj_lds_fits<float, 64, 1, 512, false>(mmax);
    case kGjF32x512:
      return gj_lds_fits<float, 32, 1, 512>(mmax);
    case kGjF32x256:
      return gj_lds_fits<float, 32, 2, 256>(mmax);
    case kGjF32x512r2:
      return gj_lds_fits<float, 32, 2, 512>(mmax);
    case kGjF48x512r2:
      return gj_lds_fits<float, 48, 2, 512, false>(mmax);
    default:
      return false;
  }
}

bool gj_variant_f32(int variant) { return variant >= kGjF64x512; }

int gj_batched_grid(int npatch) {
  // as many workgroups as the fewest rounds over the compute units need:
  // the rest of the device stays free for the coarsest inversion
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  ncu = std::max(ncu, 1);
  npatch = std::max(npatch, 1);
  const int rounds = (npatch + ncu - 1) / ncu;
  return (npatch + rounds - 1) / rounds;
}

std::vector<int> gj_schedule(const int *pm, int npatch, int grid) {
  // longest processing time first: blocks by decreasing m^3 (the update
  // work), each to the workgroup with the least work so far (ties: lowest
  // index), so mixed block sizes do not leave one workgroup two large ones
  std::vector<int> order(npatch);
  for (int k = 0; k < npatch; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return pm[a] > pm[b]; });
  typedef std::pair<double, int> Load;
  std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
  for (int g = 0; g < grid; ++g) heap.push(Load(0.0, g));
  std::vector<std::vector<int>> per(grid);
  for (int k : order) {
    Load l = heap.top();
    heap.pop();
    per[l.second].push_back(k);
    const double m = pm[k];
    heap.push(Load(l.first + m * m * m, l.second));
  }
  std::vector<int> out(grid + 1 + npatch);
  out[0] = 0;
  for (int g = 0; g < grid; ++g) out[g + 1] = out[g] + (int)per[g].size();
  for (int g = 0; g < grid; ++g)
    std::copy(per[g].begin(), per[g].end(), out.begin() + grid + 1 + out[g]);
  return out;
}

template <int NB, int R, int NT, bool UNR, bool GPC = false, typename T>
static void launch_gj_nbr(T *blocks, const int64_t *boff, const int *pm, const int64_t *poff,
                          int *perm, int *used, int grid, const int *sched, int mmax, int *status,
                          hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr) {
  const size_t shm = GPC ? 0 : gj_batched_lds(mmax, NB, sizeof(T));
  if (shm)
    (void)hipFuncSetAttribute((const void *)k_gj_batched<T, NB, R, NT, UNR, GPC>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  // with events: recorded at the kernel's own start and end
  hipExtLaunchKernelGGL(k_gj_batched<T, NB, R, NT, UNR, GPC>, dim3(grid), dim3(NT), shm, st, ev0, ev1, 0,
                        blocks, boff, pm, poff, perm, used, status, sched);
}

template <int NB, int R, int NT, typename T>
static void launch_gj_paired(T *blocks, const int64_t *boff, const int *pm, const int64_t *poff, int *perm,
                             int *used, int grid, const int *sched, int mmax, int *status, hipStream_t st,
                             hipEvent_t ev0, hipEvent_t ev1) {
  (void)mmax;
  hipExtLaunchKernelGGL(k_gj_paired<T, NB, R, NT>, dim3(grid), dim3(NT), 0, st, ev0, ev1, 0, blocks, boff, pm,
                        poff, perm, used, status, sched);
}

void launch_gj_batched(double *blocks, const int64_t *boff, const int *pm, const int64_t *poff,
                       int *perm, int *used, int npatch, int mmax, int *status, int grid,
                       const int *sched, hipStream_t st, int variant, hipEvent_t ev0, hipEvent_t ev1) {
  if (npatch == 0) return;
  if (!gj_variant_ok(variant, mmax))
    variant = gj_variant_ok(kGjP32x512, mmax)  ? kGjP32x512
              : gj_variant_ok(kGj32x512, mmax) ? kGj32x512
              : gj_variant_ok(kGj24x512, mmax) ? kGj24x512
                                               : kGj16x256;
  const bool small = mmax <= 512;
  // NB 16 on 256 threads: one wave per SIMD, the per-step work common to a
  // wave shared by more rows; on 512 threads: twice the waves, so twice the
  // update loads in flight per compute unit.  NB 32 (24 for two rows per
  // thread, the most that stays in registers): 1/2 (2/3) of the update
  // traffic of NB 16, the panel in LDS or read from the block.
  if (variant == kGjP32x512)
    launch_gj_paired<32, 1, 512>(blocks, boff, pm, poff, perm, used, grid, sched, mmax, status, st, ev0, ev1);
  else if (variant == kGj32x512)
    launch_gj_nbr<32, 1, 512, true>(blocks, boff, pm, poff, perm, used, grid, sched, mmax, status, st, ev0, ev1);
  else if (variant == kGjWideG && small)
    launch_gj_nbr<32, 1, 512, true, true>(blocks, boff, pm, poff, perm, used, grid, sched, mmax,
                                          status, st, ev0, ev1);
  else if (variant == kGjWideG)
    launch_gj_nbr<24, 2, 512, true, true>(blocks, boff, pm, poff, perm, used, grid, sched, mmax,
                                          status, st, ev0, ev1);
  else if (variant == kGj24x512)
    launch_gj_nbr<24, 2, 512, true>(blocks, boff, pm, poff, perm, used, grid, sched, mmax, status,
                                    st, ev0, ev1);
  else if (variant == kGj16x512 && small)
    launch_gj_nbr<16, 1, 512, true>(blocks, boff, pm, poff, perm, used, grid, sched, mmax, status, st, ev0, ev1);
  else if (variant == kGj16x512)
    launch_gj_nbr<16, 2, 512, true>(blocks, boff, pm, poff, perm, used, grid, sched, mmax, status, st, ev0, ev1);
  else if (small)
    launch_gj_nbr<16, 2, 256, true>(blocks, boff, pm, poff, perm, used, grid, sched, mmax, status, st, ev0, ev1);
  else
    launch_gj_nbr<16, 4, 256, true>(blocks, boff, pm, poff, perm, used, grid, sched, mmax, status, st, ev0, ev1);
}

// FP32 working matrices (the mixed forms): paired NB 32 panels on 512
// threads (blocks up to 512 dofs, the panel read back from the block), NB 64
// on 512 threads (one row per thread), NB 32 on 512 or on 256 threads (two
// rows per thread: two workgroups fit a compute unit), NB 32 or 48 on 512
// threads with two rows per thread (blocks up to 1024 dofs), these with the
// panel in LDS.  An unsupported variant falls back to the first that fits of
// paired NB 32, NB 64, NB 32, NB 48 and NB 32 with two rows per thread.
void launch_gj_batched_f32(float *blocks, const int64_t *boff, const int *pm, const int64_t *poff,
                           int *perm, int *used, int npatch, int mmax, int *status, int grid,
                           const int *sched, hipStream_t st, int variant, hipEvent_t ev0,
                           hipEvent_t ev1) {
  if (npatch == 0) return;
  if (!gj_variant_f32(variant) || !gj_variant_ok(variant, mmax)) {
    variant = kGjF32x512r2;
    for (int v : {kGjPF32x512, kGjF64x512, kGjF32x512, kGjF48x512r2, kGjF32x512r2})
      if (gj_variant_ok(v, mmax)) {
        variant = v;
        break;
      }
  }
  switch (variant) {
    case kGjPF32x512:
      launch_gj_paired<32, 1, 512>(blocks, boff, pm, poff, perm, used, grid, sched, mmax, status, st, ev0, ev1);
      break;
    case kGjF64x512:
      launch_gj_nbr<64, 1, 512, false>(blocks, boff, pm, poff, perm, used, grid, sched, mmax, status, st, ev0, ev1);
      break;
    case kGjF32x512:
      launch_gj_nbr<32, 1, 512, true>(blocks, boff, pm, poff, perm, used, grid, sched, mmax, status, st, ev0, ev1);
      break;
    case kGjF32x256:
      launch_gj_nbr<32, 2, 256, true>(blocks, boff, pm, poff, perm, used, grid, sched, mmax, status, st, ev0, ev1);
      break;
    case kGjF48x512r2:
      launch_gj_nbr<48, 2, 512, false>(blocks, boff, pm, poff, perm, used, grid, sched, mmax, status, st, ev0, ev1);
      break;
    default:
      launch_gj_nbr<32, 2, 512, true>(blocks, boff, pm, poff, perm, used, grid, sched, mmax, status, st, ev0, ev1);
      break;
  }
}

// ------------------------------------------------------------------ coarsest operator
// A: n x n row-major with leading dimension ld (a multiple of 16 doubles).
__global__ void k_fill_i32(int *x, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}
void launch_fill_i32(int *x, int n, int v, hipStream_t st) {
  if (n > 0) k_fill_i32<<<cdivg(n, 256), 256, 0, st>>>(x, n, v);
}

// The coarse matrix's panel [p0, p0 + w) into registers: rows tid + q NT,
// loaded whole from their base (p0 + NB <= ld: ld is a multiple of 16 and
// NB divides 16; 16-byte accesses since ld and p0 are multiples of 2); rows
// beyond n repeat row n - 1 and are never candidates.
template <int NB, int R, int NT>
__device__ __forceinline__ void cgj_load(const double *__restrict__ A, int n, int64_t ld, int p0,
                                         int w, const int *__restrict__ used, double (&v)[R][NB],
                                         int (&stp)[R]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int i = tid + q * NT;
    stp[q] = i < n ? used[i] : kNoRow;
    const double2 *row = reinterpret_cast<const double2 *>(A + (int64_t)min(i, n - 1) * ld + p0);
#pragma unroll
    for (int c = 0; c < NB / 2; ++c) {
      const double2 x = row[c];
      v[q][2 * c] = x.x;
      v[q][2 * c + 1] = x.y;
    }
  }
#pragma unroll
  for (int q = 0; q < R; ++q)
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c >= w) v[q][c] = 0.0;
}

// Factors the loaded panel (all NT threads of the workgroup), stores it,
// marks its pivot rows in used[] and writes perm[p0 ...] from the threads
// that hold them (no barrier after the stores).  On failure status[0] =
// 1 + the failing step.
template <int NB, int R, int NT>
__device__ __forceinline__ void cgj_factor(double *__restrict__ A, int n, int64_t ld, int p0,
                                           int w, int *__restrict__ perm, int *__restrict__ used,
                                           int *__restrict__ status, PivotLds<NB, NT / 64> &sh,
                                           double (&v)[R][NB], int (&stp)[R]) {
  const int tid = threadIdx.x;
  int mypiv = 0;
  const int f = reg_panel<NB, R, NT, true, true>(v, stp, n, p0, w, sh, mypiv);
  if (f) {
    if (tid == 0) status[0] = f;
    return;
  }
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int i = tid + q * NT;
    if (i < n) {
      double *row = A + (int64_t)i * ld + p0;
      if (w == NB) {
        double2 *row2 = reinterpret_cast<double2 *>(row);
#pragma unroll
        for (int c = 0; c < NB / 2; ++c) row2[c] = make_double2(v[q][2 * c], v[q][2 * c + 1]);
      } else {
#pragma unroll
        for (int c = 0; c < NB; ++c)
          if (c < w) row[c] = v[q][c];
      }
      if (stp[q] >= p0) used[i] = stp[q];
    }
  }
  if (tid < w) perm[p0 + tid] = mypiv;
}

template <int NB, int R, int NT>
__global__ __launch_bounds__(NT) void k_cgj_panel(double *__restrict__ A, int n, int64_t ld,
                                                  int p0, int w, int *__restrict__ perm,
                                                  int *__restrict__ used,
                                                  int *__restrict__ status) {
  __shared__ PivotLds<NB, NT / 64> sh;
  if (status[0]) return;
  double v[R][NB];
  int stp[R];
  cgj_load<NB, R, NT>(A, n, ld, p0, w, used, v, stp);
  cgj_factor<NB, R, NT>(A, n, ld, p0, w, perm, used, status, sh, v, stp);
}

// Applies the factored panel [p0, p0 + w) to one tile of 16 of the columns
// outside it (taken in order, skipping the panel).  The workgroup's waves
// read the tile's X (pivot rows' old values) into registers, meet at a
// barrier, then update the tile's 16-row tiles round-robin on the matrix
// cores (operand layouts as in the batched kernel); no other workgroup
// touches the tile.
template <int NB, int NT>
__device__ __forceinline__ void cgj_update_tile(double *__restrict__ A, int n, int64_t ld, int p0,
                                                int w, int ct, const int *__restrict__ perm,
                                                const int *__restrict__ used) {
  constexpr int KC = (NB + 3) / 4, NWV = NT / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int jl = lane & 15, kq = lane >> 4;
  const int mp = n - w;
  const int q = ct * 16 + jl;
  const bool colok = q < mp;
  const int j = colok ? (q < p0 ? q : q + w) : 0;
  // X: pivot rows' old values, clamped loads issued together (perm, then A)
  int pr[KC];
#pragma unroll
  for (int kk = 0; kk < KC; ++kk) pr[kk] = perm[p0 + min(kk * 4 + kq, w - 1)];
  double bx[KC];
#pragma unroll
  for (int kk = 0; kk < KC; ++kk) bx[kk] = A[pr[kk] * ld + j];
#pragma unroll
  for (int kk = 0; kk < KC; ++kk)
    if (!(colok && kk * 4 + kq < w)) bx[kk] = 0.0;
  __syncthreads();
  const int nrt = (n + 15) >> 4;
  // clamped addresses: no load waits on another; the pivot rows, the rows
  // past n and the columns past the panel are zeroed where the tile is used
  struct Tile {
    dx4 c;
    int u[4];
    double a[KC];
  };
  auto load_tile = [&](int rt) {
    Tile T;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = min(rt * 16 + r * 4 + kq, n - 1);
      T.c[r] = A[i * ld + j];
      T.u[r] = used[i];
    }
    const int ia = min(rt * 16 + jl, n - 1);
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) T.a[kk] = A[ia * ld + p0 + min(kk * 4 + kq, NB - 1)];
    return T;
  };
  // prefetches are unconditional (past the last tile they repeat it), so no
  // load waits on a branch
  Tile ring[kPrefetch];
#pragma unroll
  for (int u = 0; u < kPrefetch; ++u) ring[u] = load_tile(min(wave + NWV * u, nrt - 1));
  for (int rt0 = wave; rt0 < nrt; rt0 += NWV * kPrefetch) {
#pragma unroll
    for (int u = 0; u < kPrefetch; ++u) {
      const int rt = rt0 + NWV * u;
      Tile T = ring[u];
      ring[u] = load_tile(min(rt + NWV * kPrefetch, nrt - 1));
      if (rt < nrt) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = rt * 16 + r * 4 + kq;
          if (!(colok && i < n && (T.u[r] < p0 || T.u[r] >= p0 + w))) T.c[r] = 0.0;
        }
        const bool arow = rt * 16 + jl < n;
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) {
          const double a = (arow && kk * 4 + kq < NB) ? T.a[kk] : 0.0;
          T.c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bx[kk], T.c, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = rt * 16 + r * 4 + kq;
          if (colok && i < n) A[i * ld + j] = T.c[r];
        }
      }
    }
  }
}

// Update of the compressed column tile p0 / 16, which holds the next
// panel, by the factored panel [p0, p0 + w), for every row that is not one
// of the panel's pivot rows (those are read here as X and finished by the
// factoring workgroup of k_cgj_step); 64 rows per workgroup, 4 threads per
// row, 4 columns each.  The critical path between two panels is then this
// short launch and the factorization, not a whole-tile update.
template <int NB>
__global__ __launch_bounds__(256) void k_cgj_next(double *__restrict__ A, int n, int64_t ld, int p0,
                                                  int w, const int *__restrict__ perm,
                                                  const int *__restrict__ used,
                                                  const int *__restrict__ status) {
  __shared__ double X[NB][16];   // the pivot rows' values in the tile, staged once
  if (status[0]) return;
  const int tid = threadIdx.x, mp = n - w, q00 = (p0 / 16) * 16;
  // this thread's row: panel values (whole 16-byte pairs: p0 + NB <= ld) and
  // its 4 tile entries, all loads issued before the X staging (clamped
  // addresses; what lies outside is never stored)
  const int i = blockIdx.x * 64 + (tid >> 2);
  const int ic = min(i, n - 1);
  const int s = used[ic];
  const int e0 = (tid & 3) * 4;
  double *Ai = A + ic * ld;
  double pc[NB];
  const double2 *pc2 = reinterpret_cast<const double2 *>(Ai + p0);
#pragma unroll
  for (int c = 0; c < NB / 2; ++c) {
    const double2 x = pc2[c];
    pc[2 * c] = x.x;
    pc[2 * c + 1] = x.y;
  }
  int jj[4];
  double a[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int q = min(q00 + e0 + e, mp - 1);
    jj[e] = q < p0 ? q : q + w;
    a[e] = Ai[jj[e]];
  }
  if (tid < 16 * NB) {
    const int t = tid >> 4, q = q00 + (tid & 15);
    const int qc = min(q, mp - 1);
    const double x = A[perm[p0 + min(t, w - 1)] * ld + (qc < p0 ? qc : qc + w)];
    X[t][tid & 15] = (t < w && q < mp) ? x : 0.0;
  }
  __syncthreads();
  if (i >= n || (s >= p0 && s < p0 + w)) return;
#pragma unroll
  for (int t = 0; t < NB; ++t)
    if (t >= w) pc[t] = 0.0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    double acc = a[e];
#pragma unroll
    for (int t = 0; t < NB; ++t) acc += pc[t] * X[t][e0 + e];
    if (q00 + e0 + e < mp) Ai[jj[e]] = acc;
  }
}

// One launch per panel [p0, p0 + w).  Every workgroup but one updates one
// compressed column tile with the panel.  The workgroup of tile p0 / 16
// (which holds the next panel; k_cgj_next has updated its other rows)
// computes the panel's pivot rows in that tile, then factors the next
// panel.  Concurrent readers of used[] only test membership in
// [p0, p0 + w), which the factorization never changes (it sets entries that
// were -1 to steps >= p0 + w); it writes only its own tile and
// perm[p0 + w ...].
template <int NB, int R, int NT>
__global__ __launch_bounds__(NT) void k_cgj_step(double *__restrict__ A, int n, int64_t ld,
                                                 int p0, int w, int *__restrict__ perm,
                                                 int *__restrict__ used,
                                                 int *__restrict__ status) {
  __shared__ PivotLds<NB, NT / 64> sh;
  if (status[0]) return;
  const int pn = p0 + w;
  if (pn >= n || (int)blockIdx.x != p0 / 16) {
    cgj_update_tile<NB, NT>(A, n, ld, p0, w, blockIdx.x, perm, used);
    return;
  }
  // the next panel's loads go out first; meanwhile the panel's pivot rows in
  // this tile are computed, new A[r_s][j] = sum_t PC[r_s][t] X[t][j] with X
  // the pivot rows' old values (all read before any is written), stored to
  // the block and patched into the loaded rows through LDS
  __shared__ double fix[NB][16];
  const int tid = threadIdx.x, mp = n - w, ct = p0 / 16, wn = min(NB, n - pn);
  double v[R][NB];
  int stp[R];
  cgj_load<NB, R, NT>(A, n, ld, pn, wn, used, v, stp);
  double val = 0.0;
  int64_t dst = -1;
  if (tid < 16 * w) {
    // clamped loads issued together: the panel's pivot rows, then this
    // thread's pivot-row panel values and the pivot rows' tile column
    const int sidx = tid >> 4, q = ct * 16 + (tid & 15);
    const int qc = min(q, mp - 1);
    const int j = qc < p0 ? qc : qc + w;
    int pv[NB];
#pragma unroll
    for (int t = 0; t < NB; ++t) pv[t] = perm[p0 + min(t, w - 1)];
    const double2 *pr2 = reinterpret_cast<const double2 *>(A + pv[sidx] * ld + p0);
    double prv[NB], xa[NB];
#pragma unroll
    for (int c = 0; c < NB / 2; ++c) {
      const double2 x = pr2[c];
      prv[2 * c] = x.x;
      prv[2 * c + 1] = x.y;
    }
#pragma unroll
    for (int t = 0; t < NB; ++t) xa[t] = A[pv[t] * ld + j];
#pragma unroll
    for (int t = 0; t < NB; ++t)
      if (t < w) val += prv[t] * xa[t];
    if (q < mp) dst = pv[sidx] * ld + j;
    else val = 0.0;
    fix[sidx][tid & 15] = val;
  }
  __syncthreads();
  if (dst >= 0) A[dst] = val;
  const int e0 = p0 - ct * 16;   // the next panel's first column within the tile
#pragma unroll
  for (int q = 0; q < R; ++q)
    if (stp[q] >= p0 && stp[q] < p0 + w) {
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < wn) v[q][c] = fix[stp[q] - p0][e0 + c];
    }
  cgj_factor<NB, R, NT>(A, n, ld, pn, wn, perm, used, status, sh, v, stp);
}

// C0[k * n + c] = inv(A)[k][c] (row-major, the dense GEMV layout): on F x F
// S[perm[fk]][used[fc]], on the diagonal of D 1 / a_kk (the row's single
// entry), zero elsewhere
__global__ void k_cgj_finish(const double *__restrict__ S, int n, int64_t ld,
                             const int *__restrict__ perm, const int *__restrict__ used,
                             const int *__restrict__ fpos, const int *__restrict__ rowptr,
                             const double *__restrict__ val, const int *__restrict__ status,
                             double *__restrict__ C0) {
  if (status[0]) return;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (c >= n) return;
  const int fk = fpos[k], fc = fpos[c];
  double x = 0.0;
  if (fk >= 0 && fc >= 0)
    x = S[perm[fk] * ld + used[fc]];
  else if (k == c)
    x = 1.0 / val[rowptr[k]];
  C0[(int64_t)k * n + c] = x;
}

// the diagonal entries of D: a zero or non-finite one is reported as step
// nf + (its index in dlist) when the free block itself inverted (one
// workgroup; the smallest failing index wins)
__global__ __launch_bounds__(256) void k_cgj_dcheck(const int *__restrict__ dlist, int nd, int nf,
                                                    const int *__restrict__ rowptr,
                                                    const double *__restrict__ val,
                                                    int *__restrict__ status) {
  __shared__ int smin[256];
  int mine = INT_MAX;
  for (int t = threadIdx.x; t < nd; t += 256) {
    const double a = val[rowptr[dlist[t]]];
    if (!(a != 0.0 && fabs(a) <= DBL_MAX)) mine = min(mine, t);
  }
  smin[threadIdx.x] = mine;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) smin[threadIdx.x] = min(smin[threadIdx.x], smin[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0 && status[0] == 0 && smin[0] != INT_MAX) status[0] = 1 + nf + smin[0];
}

template <int NB, int R, int NT>
static void gj_coarse_nb(double *A, int n, int64_t ld, int *perm, int *used, int *status,
                         hipStream_t st) {
  k_cgj_panel<NB, R, NT><<<1, NT, 0, st>>>(A, n, ld, 0, std::min(NB, n), perm, used, status);
  for (int p0 = 0; p0 < n; p0 += NB) {
    const int w = std::min(NB, n - p0);
    if (n <= w) break;
    if (p0 + w < n) k_cgj_next<NB><<<cdivg(n, 64), 256, 0, st>>>(A, n, ld, p0, w, perm, used, status);
    k_cgj_step<NB, R, NT><<<cdivg(n - w, 16), NT, 0, st>>>(A, n, ld, p0, w, perm, used, status);
  }
}

void gj_coarse(double *A, int nf, int64_t ld, const CoarseSplit &cs, double *C0, int *status,
               int *iwork, hipStream_t st) {
  int *perm = iwork, *used = iwork + nf;
  if (nf > 0) {
    k_fill_i32<<<cdivg(nf, 256), 256, 0, st>>>(used, nf, -1);
    // (panel width, rows per thread, threads): 512 threads, the panel rows in
    // registers without spilling
    if (nf <= 512)
      gj_coarse_nb<16, 1, 512>(A, nf, ld, perm, used, status, st);
    else if (nf <= 1024)
      gj_coarse_nb<16, 2, 512>(A, nf, ld, perm, used, status, st);
    else if (nf <= 1536)
      gj_coarse_nb<16, 3, 512>(A, nf, ld, perm, used, status, st);
    else if (nf <= 3072)
      gj_coarse_nb<8, 6, 512>(A, nf, ld, perm, used, status, st);
    else if (nf <= 4096)   // 8 columns, 8 rows a thread: 188 registers, no spill (10 rows spill)
      gj_coarse_nb<8, 8, 512>(A, nf, ld, perm, used, status, st);
    else
      gj_coarse_nb<4, 12, 512>(A, nf, ld, perm, used, status, st);
  }
  if (cs.nd > 0)
    k_cgj_dcheck<<<1, 256, 0, st>>>(cs.dlist, cs.nd, nf, cs.rowptr, cs.val, status);
  k_cgj_finish<<<dim3(cdivg(cs.n, 256), cs.n), 256, 0, st>>>(A, cs.n, ld, perm, used, cs.fpos,
                                                             cs.rowptr, cs.val, status, C0);
}

__global__ void k_iota_i32(int *x, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) x[i] = i;
}
void launch_iota_i32(int *x, int n, hipStream_t st) {
  if (n > 0) k_iota_i32<<<cdivg(n, 256), 256, 0, st>>>(x, n);
}
template <typename TS>
__global__ void k_copy_block(const TS *__restrict__ src, int m, double *__restrict__ dst, int64_t ld) {
  const int j = blockIdx.x * 256 + threadIdx.x, i = blockIdx.y;
  if (j < m) dst[(int64_t)i * ld + j] = (double)src[(int64_t)i * m + j];
}
template <typename TS>
void launch_copy_block(const TS *src, int m, double *dst, int64_t ld, hipStream_t st) {
  if (m > 0) k_copy_block<TS><<<dim3(cdivg(m, 256), m), 256, 0, st>>>(src, m, dst, ld);
}
template void launch_copy_block<double>(const double *, int, double *, int64_t, hipStream_t);
template void launch_copy_block<float>(const float *, int, double *, int64_t, hipStream_t);

// one wave per row of F, its lanes over the row's entries
__global__ __launch_bounds__(256) void k_csr_to_dense(int n, int64_t ld, const int *rowptr,
                                                      const int *col, const double *val,
                                                      const int *fpos, double *A) {
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= n) return;
  const int fr = fpos[r];
  if (fr < 0) return;
  const int lane = threadIdx.x & 63;
  for (int p = rowptr[r] + lane; p < rowptr[r + 1]; p += 64) {
    const int fc = fpos[col[p]];
    if (fc >= 0) A[fr * ld + fc] = val[p];
  }
}
void launch_csr_to_dense(const CsrView<double> &A, const int *fpos, double *dense, int64_t ld,
                         hipStream_t st) {
  if (A.nrows > 0)
    k_csr_to_dense<<<cdivg(A.nrows, 4), 256, 0, st>>>(A.nrows, ld, A.rowptr, A.col, A.val, fpos,
                                                      dense);
}

}  // namespace fsi
