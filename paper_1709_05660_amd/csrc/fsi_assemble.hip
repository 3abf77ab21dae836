// Device assembly of the finest residual and its exact Jacobian, and the
// Newton loop on the device (include/fsi_assembly.h).
//
// One workgroup per (element of one colour, range of Jacobian columns).  The
// element residual's rows are sums over quadrature points of test functions
// weighted by a few coefficients per point; the workgroup differentiates
// those coefficients along each of its columns' local dofs (one-direction
// dual numbers: value and derivative), then contracts them with the
// test-function tables and adds the element Jacobian's entries into the CSR
// values at positions found once, when the assembly is created.  Elements of
// one colour share no node, so every entry is written once per launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <vector>

#include "../../include/fsi_assembly.h"
#include "fsi_internal.h"

namespace fsi {

// ------------------------------------------------------------ one-direction duals
struct D1 {
  double v, g;
};
__device__ __forceinline__ D1 dc(double c) { return {c, 0.0}; }
__device__ __forceinline__ D1 operator+(D1 a, D1 b) { return {a.v + b.v, a.g + b.g}; }
__device__ __forceinline__ D1 operator-(D1 a, D1 b) { return {a.v - b.v, a.g - b.g}; }
__device__ __forceinline__ D1 operator-(D1 a) { return {-a.v, -a.g}; }
__device__ __forceinline__ D1 operator*(D1 a, D1 b) { return {a.v * b.v, a.g * b.v + a.v * b.g}; }
__device__ __forceinline__ D1 operator*(double s, D1 b) { return {s * b.v, s * b.g}; }
__device__ __forceinline__ D1 operator+(D1 a, double c) { return {a.v + c, a.g}; }
__device__ __forceinline__ D1 operator/(D1 a, D1 b) {
  const double q = a.v / b.v;
  return {q, (a.g - q * b.g) / b.v};
}

struct AsmView {
  int ne, ndof, ncolor;
  const int *l2g, *tgt, *color_ptr, *color_elems, *rowptr, *col;
  const uint8_t *solid, *dir;
  const double *N, *dN, *psi, *w, *yprev;
  double vol, mu, rho, mu_s, dt, rho_s;
  int transient;
};

template <int DIM>
struct Shape {
  static constexpr int NA = DIM == 3 ? 27 : 9, NP = DIM + 1, NL = 2 * DIM * NA + NP, NQ = DIM == 3 ? 27 : 9;
};

// fields of one state at one quadrature point (as the host builder's Kin)
template <int DIM, typename V>
struct KinD {
  V Gd[DIM][DIM], F[DIM][DIM], Fi[DIM][DIM], det, pq, uq[DIM], dq[DIM], gu[DIM][DIM];
};

// The sums over the element's nodes at one quadrature point: the reference
// gradients of displacement and velocity, velocity, displacement and
// pressure.  They are linear in the element state, and a thread's dual state
// differs from the element's value by one unit entry (its local dof), so the
// value sums are taken once per element and point and shared through LDS, and
// each thread adds its single-term derivative; only the nonlinear part
// (deformation gradient, determinant, inverse, stresses) runs in duals.
template <int DIM>
struct Sums {
  // per point: Gd[c][j], Gu[c][j], uq[c], dq[c], pq
  static constexpr int GD = 0, GU = DIM * DIM, UQ = 2 * DIM * DIM, DQ = UQ + DIM, PQ = DQ + DIM, NS = PQ + 1;
};

// sum s of point q for the element state ye
template <int DIM>
__device__ __forceinline__ double point_sum(const double *sN, const double *sdN, const double *spsi, const double *ye,
                                            int q, int s) {
  constexpr int NA = Shape<DIM>::NA, NP = Shape<DIM>::NP;
  using S = Sums<DIM>;
  const double *Nq = sN + q * NA, *dNq = sdN + q * NA * DIM;
  double acc = 0.0;
  if (s < S::UQ) {
    const int c = (s % (DIM * DIM)) / DIM, j = s % DIM;
    const double *yc = ye + (s < S::GU ? c : DIM + c) * NA;
    for (int a = 0; a < NA; ++a) acc += dNq[a * DIM + j] * yc[a];
  } else if (s < S::PQ) {
    const double *yc = ye + (s < S::DQ ? DIM + s - S::UQ : s - S::DQ) * NA;
    for (int a = 0; a < NA; ++a) acc += Nq[a] * yc[a];
  } else {
    for (int j = 0; j < NP; ++j) acc += spsi[q * NP + j] * ye[2 * DIM * NA + j];
  }
  return acc;
}

// the rest of the kinematics from the gradients (F = I + Gd, its determinant
// and inverse, and for the fluid the velocity gradient in current coordinates
// gu = Gu F^{-1}); uq, dq and pq are set by the caller
template <int DIM, typename V>
__device__ __forceinline__ void kin_finish(const V (&Gd)[DIM][DIM], const V (&Gu)[DIM][DIM], bool fluid,
                                           KinD<DIM, V> &k) {
#pragma unroll
  for (int c = 0; c < DIM; ++c)
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      k.Gd[c][j] = Gd[c][j];
      k.F[c][j] = c == j ? Gd[c][j] + 1.0 : Gd[c][j];
    }
  if constexpr (DIM == 2) {
    k.det = k.F[0][0] * k.F[1][1] - k.F[0][1] * k.F[1][0];
    k.Fi[0][0] = k.F[1][1] / k.det;
    k.Fi[1][1] = k.F[0][0] / k.det;
    k.Fi[0][1] = -(k.F[0][1] / k.det);
    k.Fi[1][0] = -(k.F[1][0] / k.det);
  } else {
    V cof[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
        cof[i][j] = k.F[i1][j1] * k.F[i2][j2] - k.F[i1][j2] * k.F[i2][j1];
      }
    k.det = k.F[0][0] * cof[0][0] + k.F[0][1] * cof[0][1] + k.F[0][2] * cof[0][2];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) k.Fi[i][j] = cof[j][i] / k.det;
  }
  if (!fluid) return;
#pragma unroll
  for (int c = 0; c < DIM; ++c)
#pragma unroll
    for (int b = 0; b < DIM; ++b) {
      V s = V{};
#pragma unroll
      for (int j = 0; j < DIM; ++j) s = s + Gu[c][j] * k.Fi[j][b];
      k.gu[c][b] = s;
    }
}

// kinematics of the state at t_n from its shared sums
template <int DIM>
__device__ __forceinline__ void kin_value(const double *S, bool fluid, KinD<DIM, double> &k) {
  using SS = Sums<DIM>;
  double Gd[DIM][DIM], Gu[DIM][DIM];
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      Gd[c][j] = S[SS::GD + c * DIM + j];
      Gu[c][j] = S[SS::GU + c * DIM + j];
    }
    k.uq[c] = S[SS::UQ + c];
    k.dq[c] = S[SS::DQ + c];
  }
  k.pq = S[SS::PQ];
  kin_finish<DIM>(Gd, Gu, fluid, k);
}

// kinematics of the current state differentiated along local dof jd: the
// shared value sums plus the one term that dof contributes to each
template <int DIM>
__device__ __forceinline__ void kin_dual(const double *S, const double *Nq, const double *dNq, const double *ps,
                                         int jd, bool fluid, KinD<DIM, D1> &k) {
  constexpr int NA = Shape<DIM>::NA;
  using SS = Sums<DIM>;
  const bool isd = jd < DIM * NA, isv = !isd && jd < 2 * DIM * NA, isp = jd >= 2 * DIM * NA;
  const int tc = isd ? jd / NA : (isv ? (jd - DIM * NA) / NA : -1);
  const int ta = isp ? 0 : jd % NA;
  const double nq = Nq[ta], pp = isp ? ps[jd - 2 * DIM * NA] : 0.0;
  double dn[DIM];
#pragma unroll
  for (int j = 0; j < DIM; ++j) dn[j] = dNq[ta * DIM + j];
  D1 Gd[DIM][DIM], Gu[DIM][DIM];
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
      Gd[c][j] = {S[SS::GD + c * DIM + j], isd && c == tc ? dn[j] : 0.0};
      Gu[c][j] = {S[SS::GU + c * DIM + j], isv && c == tc ? dn[j] : 0.0};
    }
    k.uq[c] = {S[SS::UQ + c], isv && c == tc ? nq : 0.0};
    k.dq[c] = {S[SS::DQ + c], isd && c == tc ? nq : 0.0};
  }
  k.pq = {S[SS::PQ], pp};
  kin_finish<DIM>(Gd, Gu, fluid, k);
}

// structural coupling of local row lr with local column lc (the builder's rule)
__device__ __forceinline__ bool coupled_d(int dim, int na, bool solid, bool transient, int lr, int lc) {
  const int nd = dim * na;
  const int rblk = lr < nd ? 0 : (lr < 2 * nd ? 1 : 2);
  const int cblk = lc < nd ? 0 : (lc < 2 * nd ? 1 : 2);
  const int rc = (lr % nd) / na, cc = (lc % nd) / na;
  if (!solid) {
    if (rblk == 0) return true;
    if (rblk == 1) return cblk == 0 && rc == cc;
    return cblk != 2;
  }
  if (rblk == 0) return cblk != 1 || (transient && rc == cc);
  if (rblk == 1) return (cblk == 1 || (transient && cblk == 0)) && rc == cc;
  return cblk == 0;
}

// Every element residual row is a sum over the quadrature points of one test
// function (N_a, or psi_j for the pressure rows) and its reference gradient
// weighted by a few per-point coefficients: for the momentum rows of
// component c the coefficients of N_a and of dN_a/dX_j, likewise for the mesh
// motion (fluid) or kinematic (solid) rows, and one coefficient for the
// pressure rows.  Their derivatives along a local dof follow from the
// point's dual kinematics; the element Jacobian is then the contraction of
// the test-function tables with these derivatives.
template <int DIM>
struct Terms {
  static constexpr int K = 1 + DIM;   // N_a, dN_a/dX_0 .. dN_a/dX_{DIM-1}
  static constexpr int MOM = 0, MESH = DIM * K, PR = 2 * DIM * K, NK = PR + 1;
};

// The coefficients of one point for one column of the element: their
// derivatives along local dof jd, or with value set their values (the
// residual), the formulas of the host builder (steady, or one Crank-Nicolson
// step when sums0, the sums of the state at t_n, is given).
template <int DIM>
__device__ __forceinline__ void point_terms(const AsmView &v, bool solid, const double *sums, const double *sums0,
                                            const double *Nq, const double *dNq, const double *ps, double w, int jd,
                                            bool value, double *out) {
  using T = Terms<DIM>;
  const bool cn = sums0 != nullptr;
  const double dt = v.dt, rho = v.rho, mu = v.mu;
  const double k_ale = 1.0 / v.vol;
  KinD<DIM, D1> k1;
  kin_dual<DIM>(sums, Nq, dNq, ps, jd, !solid, k1);
  // per-point quantities of the rows: momentum (S, Tm), mesh motion /
  // kinematics (A), continuity / incompressibility (Pr)
  D1 S[DIM], Tm[DIM][DIM], A[DIM], Pr;
  double Tm0[DIM][DIM];
  bool with_S = true;
  if (!solid) {
    D1 sig1[DIM][DIM];
    for (int c = 0; c < DIM; ++c)
      for (int b = 0; b < DIM; ++b) {
        sig1[c][b] = mu * (k1.gu[c][b] + k1.gu[b][c]);
        if (b == c) sig1[c][b] = sig1[c][b] - k1.pq;
      }
    const D1 wJ1 = w * k1.det;
    if (!cn) {
      for (int c = 0; c < DIM; ++c) {
        D1 t = dc(0.0);
        for (int b = 0; b < DIM; ++b) t = t + k1.gu[c][b] * k1.uq[b];
        S[c] = rho * (wJ1 * t);
        for (int j = 0; j < DIM; ++j) {
          D1 t2 = dc(0.0);
          for (int b = 0; b < DIM; ++b) t2 = t2 + sig1[c][b] * k1.Fi[j][b];
          Tm[c][j] = wJ1 * t2;
          Tm0[c][j] = 0.0;
        }
      }
    } else {
      KinD<DIM, double> k0;
      kin_value<DIM>(sums0, true, k0);
      double sig0[DIM][DIM];
      for (int c = 0; c < DIM; ++c)
        for (int b = 0; b < DIM; ++b) {
          sig0[c][b] = mu * (k0.gu[c][b] + k0.gu[b][c]);
          if (b == c) sig0[c][b] -= k0.pq;
        }
      const double wJ0 = w * k0.det;
      D1 wq[DIM], Gw[DIM][DIM];
      for (int c = 0; c < DIM; ++c) {
        wq[c] = (1.0 / dt) * k1.dq[c] + (-k0.dq[c] / dt);
        for (int j = 0; j < DIM; ++j) Gw[c][j] = (1.0 / dt) * k1.Gd[c][j] + (-k0.Gd[c][j] / dt);
      }
      D1 divw1 = dc(0.0), divw0 = dc(0.0);
      for (int c = 0; c < DIM; ++c)
        for (int j = 0; j < DIM; ++j) {
          divw1 = divw1 + Gw[c][j] * k1.Fi[j][c];
          divw0 = divw0 + k0.Fi[j][c] * Gw[c][j];
        }
      for (int c = 0; c < DIM; ++c) {
        D1 t1 = -(divw1 * k1.uq[c]);
        for (int b = 0; b < DIM; ++b) t1 = t1 + k1.gu[c][b] * k1.uq[b] - k1.gu[c][b] * wq[b];
        t1 = (0.5 * rho) * t1 + (rho / dt) * k1.uq[c];
        D1 t2 = (-k0.uq[c]) * divw0;
        for (int b = 0; b < DIM; ++b) t2 = t2 + k0.gu[c][b] * k0.uq[b] + (-k0.gu[c][b]) * wq[b];
        t2 = (0.5 * rho) * t2 + (-(rho / dt) * k0.uq[c]);
        S[c] = wJ1 * t1 + wJ0 * t2;
        for (int j = 0; j < DIM; ++j) {
          D1 s1 = dc(0.0);
          double c0 = 0.0;
          for (int b = 0; b < DIM; ++b) {
            s1 = s1 + sig1[c][b] * k1.Fi[j][b];
            c0 += sig0[c][b] * k0.Fi[j][b];
          }
          Tm[c][j] = 0.5 * (wJ1 * s1);
          Tm0[c][j] = 0.5 * wJ0 * c0;
        }
      }
    }
    for (int c = 0; c < DIM; ++c) A[c] = dc(0.0);   // the mesh motion uses Gd directly
    D1 div = dc(0.0);
    for (int c = 0; c < DIM; ++c) div = div + k1.gu[c][c];
    Pr = wJ1 * div;
  } else {
    // Piola stress J sigma F^{-T}, sigma = -p I + mu_s F F^T
    D1 sig[DIM][DIM];
    for (int c = 0; c < DIM; ++c)
      for (int b = 0; b < DIM; ++b) {
        D1 s = dc(0.0);
        for (int j = 0; j < DIM; ++j) s = s + k1.F[c][j] * k1.F[b][j];
        sig[c][b] = v.mu_s * s;
        if (b == c) sig[c][b] = sig[c][b] - k1.pq;
      }
    for (int c = 0; c < DIM; ++c)
      for (int b = 0; b < DIM; ++b) {
        D1 s = dc(0.0);
        for (int j = 0; j < DIM; ++j) s = s + sig[c][j] * k1.Fi[b][j];
        Tm[c][b] = k1.det * s;
        Tm0[c][b] = 0.0;
      }
    with_S = cn;
    if (cn) {
      KinD<DIM, double> k0;
      kin_value<DIM>(sums0, false, k0);
      double sg0[DIM][DIM];
      for (int c = 0; c < DIM; ++c)
        for (int b = 0; b < DIM; ++b) {
          double s = 0.0;
          for (int j = 0; j < DIM; ++j) s += k0.F[c][j] * k0.F[b][j];
          sg0[c][b] = v.mu_s * s - (b == c ? k0.pq : 0.0);
        }
      for (int c = 0; c < DIM; ++c) {
        for (int b = 0; b < DIM; ++b) {
          double s = 0.0;
          for (int j = 0; j < DIM; ++j) s += sg0[c][j] * k0.Fi[b][j];
          Tm0[c][b] = k0.det * s;
        }
        S[c] = (v.rho_s / dt) * (k1.det * k1.uq[c] + (-k0.det * k0.uq[c]));
        A[c] = (-1.0 / dt) * k1.dq[c] + 0.5 * k1.uq[c] + (k0.dq[c] / dt + 0.5 * k0.uq[c]);
      }
    } else {
      for (int c = 0; c < DIM; ++c) {
        S[c] = dc(0.0);
        A[c] = k1.uq[c];
      }
    }
    Pr = k1.det + (-1.0);
  }
  const double half = (solid && cn) ? 0.5 : 1.0;
  auto put = [&](int i, D1 x) { out[i] = value ? x.v : x.g; };
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    if (!solid) {
      put(T::MOM + c * T::K, S[c]);
      put(T::MESH + c * T::K, dc(0.0));
#pragma unroll
      for (int j = 0; j < DIM; ++j) {
        put(T::MOM + c * T::K + 1 + j, Tm[c][j] + Tm0[c][j]);
        put(T::MESH + c * T::K + 1 + j, (w * k_ale) * k1.Gd[c][j]);
      }
    } else {
      put(T::MOM + c * T::K, with_S ? w * S[c] : dc(0.0));
      put(T::MESH + c * T::K, w * A[c]);
#pragma unroll
      for (int j = 0; j < DIM; ++j) {
        put(T::MOM + c * T::K + 1 + j, (half * w) * (Tm[c][j] + Tm0[c][j]));
        put(T::MESH + c * T::K + 1 + j, dc(0.0));
      }
    }
  }
  put(T::PR, solid ? w * Pr : Pr);
}

// Assembly of one element, columns [c0, c0 + DC) of its Jacobian, column NL
// standing for the residual.  Phase 1: the point sums of the element state
// (and of the state at t_n).  Phase 2: the coefficients of every (column,
// point) pair into LDS.  Phase 3: each thread contracts one row's test
// function with CPT columns' coefficients and adds the results at the
// positions the map gives (-1: not stored).  Elements of one colour share no
// node, so no two threads of a launch add to one entry.
template <int DIM, int DC, int CPT, int NT>
__global__ __launch_bounds__(NT) void k_assemble(AsmView v, const double *__restrict__ y, double *__restrict__ r,
                                                 double *__restrict__ jval, const int *__restrict__ map, int cbase,
                                                 int nsplit) {
  constexpr int NA = Shape<DIM>::NA, NP = Shape<DIM>::NP, NL = Shape<DIM>::NL, NQ = Shape<DIM>::NQ;
  constexpr int NS = Sums<DIM>::NS, NK = Terms<DIM>::NK, K = Terms<DIM>::K;
  static_assert(DC % CPT == 0, "columns per thread must divide the columns per block");
  __shared__ double ye[NL], ye0[NL];
  __shared__ int tg[NL];
  __shared__ double sN[NQ * NA], sdN[NQ * NA * DIM], spsi[NQ * NP], sw[NQ];
  __shared__ double sums[NQ * NS], sums0[NQ * NS];
  __shared__ double terms[DC * NQ * NK];
  const int e = v.color_elems[cbase + blockIdx.x / nsplit];
  const int c0 = (blockIdx.x % nsplit) * DC;
  const bool solid = v.solid[e] != 0;
  for (int i = threadIdx.x; i < NL; i += NT) {
    const int g = v.l2g[(int64_t)e * NL + i];
    tg[i] = v.tgt[(int64_t)e * NL + i];
    ye[i] = y[g];
    ye0[i] = v.transient ? v.yprev[g] : 0.0;
  }
  for (int i = threadIdx.x; i < NQ * NA; i += NT) sN[i] = v.N[i];
  for (int i = threadIdx.x; i < NQ * NA * DIM; i += NT) sdN[i] = v.dN[i];
  for (int i = threadIdx.x; i < NQ * NP; i += NT) spsi[i] = v.psi[i];
  for (int i = threadIdx.x; i < NQ; i += NT) sw[i] = v.w[i];
  __syncthreads();
  for (int i = threadIdx.x; i < NQ * NS; i += NT) {
    sums[i] = point_sum<DIM>(sN, sdN, spsi, ye, i / NS, i % NS);
    if (v.transient) sums0[i] = point_sum<DIM>(sN, sdN, spsi, ye0, i / NS, i % NS);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < DC * NQ; i += NT) {
    const int cl = i / NQ, q = i % NQ, col = c0 + cl;
    if (col > NL) continue;
    point_terms<DIM>(v, solid, sums + q * NS, v.transient ? sums0 + q * NS : nullptr, sN + q * NA,
                     sdN + q * NA * DIM, spsi + q * NP, sw[q], col == NL ? 0 : col, col == NL, terms + i * NK);
  }
  __syncthreads();
  for (int it = threadIdx.x; it < NL * (DC / CPT); it += NT) {
    const int lr = it % NL, cg = (it / NL) * CPT;
    // the row's test function: offset of its coefficients, node, and how many
    int off, a, nk;
    if (lr < 2 * DIM * NA) {
      const int blk = lr / (DIM * NA), c = (lr % (DIM * NA)) / NA;
      off = (blk == 0 ? Terms<DIM>::MOM : Terms<DIM>::MESH) + c * K;
      a = lr % NA;
      nk = K;
    } else {
      off = Terms<DIM>::PR;
      a = lr - 2 * DIM * NA;
      nk = 1;
    }
    double acc[CPT];
#pragma unroll
    for (int k = 0; k < CPT; ++k) acc[k] = 0.0;
    for (int q = 0; q < NQ; ++q) {
      const double *tq = terms + (cg * NQ + q) * NK + off;
      if (nk == 1) {
        const double f = spsi[q * NP + a];
#pragma unroll
        for (int k = 0; k < CPT; ++k) acc[k] += f * tq[k * NQ * NK];
      } else {
        double f[K];
        f[0] = sN[q * NA + a];
#pragma unroll
        for (int j = 0; j < DIM; ++j) f[1 + j] = sdN[(q * NA + a) * DIM + j];
#pragma unroll
        for (int k = 0; k < CPT; ++k)
#pragma unroll
          for (int j = 0; j < K; ++j) acc[k] += f[j] * tq[k * NQ * NK + j];
      }
    }
    const int tr = tg[lr];
    const int *mrow = map + ((int64_t)e * NL + lr) * NL;
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      const int col = c0 + cg + k;
      if (col < NL) {
        const int pos = mrow[col];
        if (pos >= 0) jval[pos] += acc[k];
      } else if (col == NL && tr >= 0) {
        r[tr] += acc[k];
      }
    }
  }
}

// CSR position of every (element, local row, local column) entry of the
// element Jacobian that the assembly stores, else -1: rows without a target,
// Dirichlet rows and columns, and structurally uncoupled pairs are not stored.
__global__ void k_asm_map(AsmView v, int dim, int na, int nl, int64_t total, int *map) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= total) return;
  const int64_t el = idx / nl;
  const int e = (int)(el / nl), lr = (int)(el % nl), jd = (int)(idx % nl);
  const int tr = v.tgt[(int64_t)e * nl + lr], gc = v.l2g[(int64_t)e * nl + jd];
  int pos = -1;
  if (tr >= 0 && !v.dir[tr] && !v.dir[gc] && coupled_d(dim, na, v.solid[e] != 0, v.transient != 0, lr, jd)) {
    int lo = v.rowptr[tr], hi = v.rowptr[tr + 1];
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (v.col[mid] < gc)
        lo = mid + 1;
      else
        hi = mid;
    }
    if (lo < v.rowptr[tr + 1] && v.col[lo] == gc) pos = lo;
  }
  map[idx] = pos;
}

// Dirichlet rows: r = y - g and a unit diagonal
__global__ void k_dirichlet_rows(const int *rows, const int *diag, int n, const double *y, const double *gval,
                                 double *r, double *jval) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  const int i = rows[t];
  r[i] = y[i] - gval[t];
  jval[diag[t]] = 1.0;
}
// Dirichlet dofs set to their values
__global__ void k_set_dirichlet(const int *rows, const double *gval, int n, double *y) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[rows[i]] = gval[i];
}

__global__ void k_neg_free(const double *r, const uint8_t *dir, int n, double *b) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) b[i] = dir[i] ? 0.0 : -r[i];
}

// device memory of the assembler: plain allocations owned here, freed when
// the assembler is destroyed or when its creation fails part way
struct AsmMem {
  std::vector<void *> v;
  AsmMem() = default;
  AsmMem(const AsmMem &) = delete;
  AsmMem &operator=(const AsmMem &) = delete;
  ~AsmMem() {
    if (!v.empty()) (void)hipDeviceSynchronize();   // no kernel of a failed creation still reads them
    for (void *p : v) (void)hipFree(p);
  }
  template <typename T>
  T *alloc(int64_t n) {
    void *p = nullptr;
    if (n <= 0) return nullptr;
    if (hipMalloc(&p, sizeof(T) * (size_t)n) != hipSuccess) throw Error(FSI_E_OOM, "device allocation");
    v.push_back(p);
    return static_cast<T *>(p);
  }
  template <typename T>
  T *up(const T *h, int64_t n) {
    T *d = alloc<T>(n);
    if (n > 0) hip_check(hipMemcpy(d, h, sizeof(T) * (size_t)n, hipMemcpyHostToDevice), "H2D");
    return d;
  }
};

struct Assembly {
  AsmView v{};
  int dim = 2, nnz = 0;
  std::vector<int> h_color_ptr;
  int ndir = 0;
  int *d_dir_rows = nullptr, *d_dir_diag = nullptr;
  double *d_dir_val = nullptr;
  double *b = nullptr, *x = nullptr, *r = nullptr, *partial = nullptr, *nrm = nullptr;
  double *yprev = nullptr;   // the state at t_n of a time step (the view reads it), else null
  int *map = nullptr;        // CSR positions of the element Jacobians' entries (ne x nl x nl), -1 if not stored
  AsmMem mem;
};

template <int DIM, int DC, int CPT, int NT>
static void launch_assemble_dim(Assembly &A, const double *y, double *r, double *jval, hipStream_t st) {
  constexpr int NL = Shape<DIM>::NL;
  const int nsplit = (NL + 1 + DC - 1) / DC;   // the element's columns and the residual
  for (int c = 0; c < A.v.ncolor; ++c) {
    const int n = A.h_color_ptr[c + 1] - A.h_color_ptr[c];
    if (n > 0)
      k_assemble<DIM, DC, CPT, NT>
          <<<n * nsplit, NT, 0, st>>>(A.v, y, r, jval, A.map, A.h_color_ptr[c], nsplit);
  }
}

static void assemble(Assembly &A, const double *y, double *r, double *jval, hipStream_t st) {
  launch_fill_f64(r, A.v.ndof, 0.0, st);
  launch_fill_f64(jval, A.nnz, 0.0, st);
  if (A.dim == 2)
    launch_assemble_dim<2, 40, 10, 192>(A, y, r, jval, st);   // the whole element in one workgroup
  else
    launch_assemble_dim<3, 16, 8, 256>(A, y, r, jval, st);
  if (A.ndir)
    k_dirichlet_rows<<<(A.ndir + 255) / 256, 256, 0, st>>>(A.d_dir_rows, A.d_dir_diag, A.ndir, y, A.d_dir_val, r,
                                                            jval);
  hip_check(hipGetLastError(), "assembly launch");
}

static Assembly *create(const fsi_element_data &ed, const fsi_csr &J, hipStream_t st) {
  if ((ed.dim != 2 && ed.dim != 3) || ed.ne < 1 || !ed.l2g || !ed.tgt || !ed.solid || !ed.color_ptr ||
      !ed.color_elems || !ed.N || !ed.dN || !ed.psi || !ed.w || !ed.dirichlet || !ed.dval)
    throw Error(FSI_E_INVALID, "element data incomplete");
  const int na = ed.dim == 3 ? 27 : 9, nl = 2 * ed.dim * na + ed.dim + 1, nq = ed.dim == 3 ? 27 : 9;
  if (ed.na != na || ed.nl != nl || ed.nq != nq || ed.np != ed.dim + 1 || J.nrows != ed.ndof || J.ncols != ed.ndof ||
      !J.rowptr || !J.colind || J.nnz >= ((int64_t)1 << 31) || ed.ndof >= ((int64_t)1 << 31))
    throw Error(FSI_E_INVALID, "element data and pattern sizes do not match");
  std::unique_ptr<Assembly> A(new Assembly());
  A->dim = ed.dim;
  A->nnz = (int)J.nnz;
  A->h_color_ptr.assign(ed.color_ptr, ed.color_ptr + ed.ncolor + 1);
  for (int64_t q = 0; q < (int64_t)ed.ne * nl; ++q)
    if (ed.l2g[q] < 0 || ed.l2g[q] >= ed.ndof || ed.tgt[q] < -1 || ed.tgt[q] >= ed.ndof)
      throw Error(FSI_E_INVALID, "element data: a dof out of range");
  if (A->h_color_ptr.front() != 0 || A->h_color_ptr.back() != ed.ne)
    throw Error(FSI_E_INVALID, "element data: colours do not list every element");
  AsmMem &M = A->mem;
  AsmView &v = A->v;
  v.ne = ed.ne;
  v.ndof = (int)ed.ndof;
  v.ncolor = ed.ncolor;
  v.l2g = M.up(ed.l2g, (int64_t)ed.ne * nl);
  v.tgt = M.up(ed.tgt, (int64_t)ed.ne * nl);
  v.color_ptr = M.up(ed.color_ptr, ed.ncolor + 1);
  v.color_elems = M.up(ed.color_elems, ed.ne);
  std::vector<int32_t> rp(J.nrows + 1);
  for (int64_t i = 0; i <= J.nrows; ++i) rp[i] = (int32_t)J.rowptr[i];
  v.rowptr = M.up(rp.data(), J.nrows + 1);
  v.col = M.up(J.colind, J.nnz);
  v.solid = M.up(ed.solid, ed.ne);
  v.dir = M.up(ed.dirichlet, ed.ndof);
  v.N = M.up(ed.N, (int64_t)nq * na);
  v.dN = M.up(ed.dN, (int64_t)nq * na * ed.dim);
  v.psi = M.up(ed.psi, (int64_t)nq * (ed.dim + 1));
  v.w = M.up(ed.w, nq);
  v.transient = ed.y_prev ? 1 : 0;
  A->yprev = ed.y_prev ? M.up(ed.y_prev, ed.ndof) : nullptr;
  v.yprev = A->yprev;
  v.vol = ed.vol;
  v.mu = ed.mu;
  v.rho = ed.rho;
  v.mu_s = ed.mu_s;
  v.dt = ed.dt;
  v.rho_s = ed.rho_s;
  std::vector<int> drows, ddiag;
  std::vector<double> dvals;
  for (int64_t i = 0; i < ed.ndof; ++i)
    if (ed.dirichlet[i]) {
      const int32_t *a = J.colind + J.rowptr[i], *b = J.colind + J.rowptr[i + 1];
      const int32_t *f = std::lower_bound(a, b, (int32_t)i);
      if (f == b || *f != i) throw Error(FSI_E_INVALID, "a Dirichlet row of the pattern holds no diagonal");
      drows.push_back((int)i);
      ddiag.push_back((int)(f - J.colind));
      dvals.push_back(ed.dval[i]);
    }
  A->ndir = (int)drows.size();
  A->d_dir_rows = M.up(drows.data(), (int64_t)drows.size());
  A->d_dir_diag = M.up(ddiag.data(), (int64_t)ddiag.size());
  A->d_dir_val = M.up(dvals.data(), (int64_t)dvals.size());
  const int n = (int)ed.ndof;
  A->b = M.alloc<double>(n);
  A->x = M.alloc<double>(n);
  A->r = M.alloc<double>(n);
  A->partial = M.alloc<double>(krylov_blocks(n));
  A->nrm = M.alloc<double>(4);
  const int64_t nmap = (int64_t)ed.ne * nl * nl;
  A->map = M.alloc<int>(nmap);
  k_asm_map<<<(unsigned)((nmap + 255) / 256), 256, 0, st>>>(v, ed.dim, na, nl, nmap, A->map);
  hip_check(hipGetLastError(), "assembly map");
  hip_check(hipStreamSynchronize(st), "assembly map");
  return A.release();
}

static double dev_norm(Assembly &A, const double *x, int n, hipStream_t st) {
  launch_kdot(n, x, n, 1, x, A.partial, A.nrm, st);
  double h = 0.0;
  hip_check(hipMemcpyAsync(&h, A.nrm, sizeof(double), hipMemcpyDeviceToHost, st), "D2H norm");
  hip_check(hipStreamSynchronize(st), "norm");
  return std::sqrt(h);
}

static fsi_status newton(Assembly &A, MG &mg, double *y, const fsi_newton_opts &no, const fsi_krylov_opts &ko,
                         fsi_newton_info *info, hipStream_t st) {
  Level &F = mg.lv.back();
  if (F.n != A.v.ndof || F.J.nnz != A.nnz) throw Error(FSI_E_INVALID, "the handle's finest pattern is not the assembly's");
  if (no.max_newton < 1 || !(no.tol > 0.0)) throw Error(FSI_E_INVALID, "invalid Newton options");
  fsi_newton_info inf{};
  const int n = A.v.ndof;
  fsi_status st_out = FSI_NOT_CONVERGED;
  for (int k = 0; k < no.max_newton; ++k) {
    assemble(A, y, A.r, F.J.val, st);   // the finest values go straight into the handle
    const double rn = dev_norm(A, A.r, n, st);
    if (k == 0) inf.res0 = rn;
    inf.res_last = rn;
    k_neg_free<<<(n + 255) / 256, 256, 0, st>>>(A.r, A.v.dir, n, A.b);
    galerkin(mg, st);
    refactor(mg, st);
    fsi_krylov_opts kk = ko;
    kk.x0_nonzero = 0;
    fsi_solve_info si{};
    const fsi_status s = fgmres(mg, A.b, A.x, kk, &si, st);
    if (s < 0) return s;
    inf.krylov_iters += si.iters;
    launch_axpy_f64(n, 1.0, A.x, y, st);
    const double en = dev_norm(A, A.x, n, st), yn = dev_norm(A, y, n, st);
    inf.steps = k + 1;
    inf.last_update = yn > 0 ? en / yn : en;
    if (en <= no.tol * yn) {
      inf.converged = 1;
      st_out = FSI_OK;
      break;
    }
  }
  if (info) *info = inf;
  return st_out;
}

// Crank-Nicolson steps: the current state becomes the state at t_n, Newton
// from it gives the state at t_{n+1}
static fsi_status cn_steps(Assembly &A, MG &mg, double *y, int nsteps, const fsi_newton_opts &no,
                           const fsi_krylov_opts &ko, fsi_newton_info *info, hipStream_t st) {
  if (!A.v.transient || !A.yprev) throw Error(FSI_E_INVALID, "the assembly holds no state at t_n (a steady problem)");
  if (nsteps < 1) throw Error(FSI_E_INVALID, "nsteps < 1");
  for (int k = 0; k < nsteps; ++k) {
    hip_check(hipMemcpyAsync(A.yprev, y, sizeof(double) * A.v.ndof, hipMemcpyDeviceToDevice, st), "state at t_n");
    fsi_newton_info inf{};
    const fsi_status r = newton(A, mg, y, no, ko, &inf, st);
    if (info) info[k] = inf;
    if (r != FSI_OK) return r;
  }
  return FSI_OK;
}

// full multigrid: Newton on each mesh, coarsest first, each mesh started from
// the prolongation of the previous mesh's iterate (relative to a base state
// that carries the boundary values, when one is given)
static fsi_status fmg(int nlev, Assembly *const *A, MG *const *M, double *const *y, const double *const *base,
                      const int32_t *caps, const fsi_newton_opts &no, const fsi_krylov_opts &ko,
                      fsi_newton_info *info, hipStream_t st) {
  for (int j = 0; j < nlev; ++j) {
    if (!A[j] || !M[j] || !y[j] || (base && !base[j])) throw Error(FSI_E_INVALID, "null handle or vector");
    if (caps && caps[j] < 1) throw Error(FSI_E_INVALID, "a Newton step limit below 1");
    if (M[j]->lv.back().n != A[j]->v.ndof) throw Error(FSI_E_INVALID, "a handle's finest size is not its assembly's");
    if (j > 0 && (M[j]->nlevels < 2 || M[j]->lv[M[j]->nlevels - 2].n != A[j - 1]->v.ndof))
      throw Error(FSI_E_INVALID, "mesh j-1 is not the level below the finest of handle j");
  }
  fsi_status out = FSI_NOT_CONVERGED;
  for (int j = 0; j < nlev; ++j) {
    Assembly &a = *A[j];
    MG &mg = *M[j];
    if (j > 0) {
      const Level &F = mg.lv.back();
      const int nc = A[j - 1]->v.ndof;
      if (base) launch_axpy_f64(nc, -1.0, base[j - 1], y[j - 1], st);
      launch_spmv(F.P.v64(), y[j - 1], (const double *)nullptr, y[j], kSpmvSet, F.P.lpr, st);
      if (base) {
        launch_axpy_f64(nc, 1.0, base[j - 1], y[j - 1], st);
        launch_axpy_f64(a.v.ndof, 1.0, base[j], y[j], st);
      }
      if (a.ndir) k_set_dirichlet<<<(a.ndir + 255) / 256, 256, 0, st>>>(a.d_dir_rows, a.d_dir_val, a.ndir, y[j]);
      hip_check(hipGetLastError(), "fmg prolongation");
    }
    fsi_newton_opts o = no;
    if (caps) o.max_newton = caps[j];
    fsi_newton_info inf{};
    const fsi_status s = newton(a, mg, y[j], o, ko, &inf, st);
    if (info) info[j] = inf;
    if (s < 0) return s;
    if (j + 1 == nlev) out = s;
  }
  return out;
}

}  // namespace fsi

using namespace fsi;

extern "C" {

fsi_status fsi_assembly_create(const fsi_element_data *ed, const fsi_csr *J, void *hip_stream,
                               struct fsi_assembly **out) {
  try {
    if (!ed || !J || !out) throw Error(FSI_E_INVALID, "null argument");
    *out = reinterpret_cast<fsi_assembly *>(create(*ed, *J, (hipStream_t)hip_stream));
    return FSI_OK;
  } catch (const Error &e) {
    set_error(e.msg);
    return e.code;
  }
}

fsi_status fsi_assembly_run(struct fsi_assembly *h, const double *y_dev, double *r_dev, double *jval_dev,
                            void *hip_stream) {
  try {
    Assembly *A = reinterpret_cast<Assembly *>(h);
    if (!A || !y_dev || !r_dev || !jval_dev) throw Error(FSI_E_INVALID, "null argument");
    assemble(*A, y_dev, r_dev, jval_dev, (hipStream_t)hip_stream);
    return FSI_OK;
  } catch (const Error &e) {
    set_error(e.msg);
    return e.code;
  }
}

fsi_status fsi_newton_solve(struct fsi_assembly *h, struct fsi_mg *mh, double *y_dev, const fsi_newton_opts *nopts,
                            const fsi_krylov_opts *kopts, fsi_newton_info *info, void *hip_stream) {
  try {
    Assembly *A = reinterpret_cast<Assembly *>(h);
    MG *mg = reinterpret_cast<MG *>(mh);
    if (!A || !mg || !y_dev || !nopts || !kopts) throw Error(FSI_E_INVALID, "null argument");
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : mg->own_stream;
    return newton(*A, *mg, y_dev, *nopts, *kopts, info, st);
  } catch (const Error &e) {
    set_error(e.msg);
    return e.code;
  }
}

fsi_status fsi_cn_steps(struct fsi_assembly *h, struct fsi_mg *mh, double *y_dev, int32_t nsteps,
                        const fsi_newton_opts *nopts, const fsi_krylov_opts *kopts, fsi_newton_info *info,
                        void *hip_stream) {
  try {
    Assembly *A = reinterpret_cast<Assembly *>(h);
    MG *mg = reinterpret_cast<MG *>(mh);
    if (!A || !mg || !y_dev || !nopts || !kopts) throw Error(FSI_E_INVALID, "null argument");
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : mg->own_stream;
    return cn_steps(*A, *mg, y_dev, nsteps, *nopts, *kopts, info, st);
  } catch (const Error &e) {
    set_error(e.msg);
    return e.code;
  }
}

fsi_status fsi_fmg_solve(int32_t nlev, struct fsi_assembly *const *a, struct fsi_mg *const *mg,
                         double *const *y_dev, const double *const *base_dev, const int32_t *max_newton,
                         const fsi_newton_opts *nopts, const fsi_krylov_opts *kopts, fsi_newton_info *info,
                         void *hip_stream) {
  try {
    if (nlev < 1 || !a || !mg || !y_dev || !nopts || !kopts) throw Error(FSI_E_INVALID, "null argument or nlev < 1");
    if (nopts->max_newton < 1 || !(nopts->tol > 0.0)) throw Error(FSI_E_INVALID, "invalid Newton options");
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : (mg[0] ? reinterpret_cast<MG *>(mg[0])->own_stream : nullptr);
    return fmg(nlev, reinterpret_cast<Assembly *const *>(a), reinterpret_cast<MG *const *>(mg), y_dev, base_dev,
               max_newton, *nopts, *kopts, info, st);
  } catch (const Error &e) {
    set_error(e.msg);
    return e.code;
  }
}

fsi_status fsi_assembly_destroy(struct fsi_assembly *h) {
  Assembly *A = reinterpret_cast<Assembly *>(h);
  if (!A) return FSI_OK;
  (void)hipDeviceSynchronize();
  delete A;   // frees its device memory
  return FSI_OK;
}

}  // extern "C"
