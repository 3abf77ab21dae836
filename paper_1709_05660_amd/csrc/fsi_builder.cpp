// Host-side problem builder (see include/fsi_problem.h): structured mesh,
// Q2/P1disc spaces, monolithic ALE residual (steady, or one Crank-Nicolson
// time step) with its exact Jacobian by forward-mode dual numbers, transfers,
// Galerkin products and patches.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/fsi_problem.h"

namespace fsib {

struct Err : std::runtime_error {
  using std::runtime_error::runtime_error;
};

// ------------------------------------------------------------ dual numbers
template <int N>
struct Dual {
  double v;
  double g[N];
};
template <int N>
inline void dzero(Dual<N> &a) {
  a.v = 0.0;
  std::memset(a.g, 0, sizeof a.g);
}
template <int N>
inline void dconst(Dual<N> &a, double c) {
  dzero(a);
  a.v = c;
}
// a += s * b
template <int N>
inline void daxpy(Dual<N> &a, double s, const Dual<N> &b) {
  a.v += s * b.v;
  for (int i = 0; i < N; ++i) a.g[i] += s * b.g[i];
}
// r = a * b
template <int N>
inline void dmul(Dual<N> &r, const Dual<N> &a, const Dual<N> &b) {
  r.v = a.v * b.v;
  for (int i = 0; i < N; ++i) r.g[i] = a.g[i] * b.v + a.v * b.g[i];
}
// a += b * c
template <int N>
inline void dfma(Dual<N> &a, const Dual<N> &b, const Dual<N> &c) {
  a.v += b.v * c.v;
  for (int i = 0; i < N; ++i) a.g[i] += b.g[i] * c.v + b.v * c.g[i];
}
// a -= b * c
template <int N>
inline void dfms(Dual<N> &a, const Dual<N> &b, const Dual<N> &c) {
  a.v -= b.v * c.v;
  for (int i = 0; i < N; ++i) a.g[i] -= b.g[i] * c.v + b.v * c.g[i];
}
// r = a / b
template <int N>
inline void ddiv(Dual<N> &r, const Dual<N> &a, const Dual<N> &b) {
  const double inv = 1.0 / b.v;
  const double q = a.v * inv;
  r.v = q;
  for (int i = 0; i < N; ++i) r.g[i] = (a.g[i] - q * b.g[i]) * inv;
}

// ------------------------------------------------------------ mesh
enum { NF = 0, NS = 1, NI = 2 };  // node classes: fluid-only, solid-only, interface

struct Mesh {
  int dim = 2, n[3] = {1, 1, 1}, g2[3] = {1, 1, 1};
  double L[3] = {1, 1, 1}, h[3] = {1, 1, 1};
  int ne = 0, N2 = 0, na = 0, npe = 0, p_off = 0, ndof = 0;
  std::vector<uint8_t> solid;   // per element
  std::vector<int> enodes;      // ne * na, local node a = (ax, ay, az) x fastest
  std::vector<uint8_t> ncls;    // per Q2 node
  std::vector<uint8_t> dir;     // per dof
  std::vector<double> dval;     // per dof
  int node(int I, int J, int K) const { return I + g2[0] * (J + g2[1] * K); }
  void grid(int nd, int &I, int &J, int &K) const {
    I = nd % g2[0];
    J = (nd / g2[0]) % g2[1];
    K = nd / (g2[0] * g2[1]);
  }
  int elem(int ex, int ey, int ez) const { return ex + n[0] * (ey + n[1] * ez); }
  int d_dof(int c, int nd) const { return c * N2 + nd; }
  int u_dof(int c, int nd) const { return (dim + c) * N2 + nd; }
  int p_dof(int e, int j) const { return p_off + npe * e + j; }
};

static double inflow(const Mesh &M, double u_peak, double y, double z) {
  double v = u_peak * 4.0 * y * (M.L[1] - y) / (M.L[1] * M.L[1]);
  if (M.dim == 3) v *= 4.0 * z * (M.L[2] - z) / (M.L[2] * M.L[2]);
  return v;
}

static Mesh make_mesh(const fsi_problem_spec &s, int nx, int ny, int nz) {
  Mesh M;
  M.dim = s.dim;
  M.n[0] = nx;
  M.n[1] = ny;
  M.n[2] = s.dim == 3 ? nz : 1;
  M.L[0] = s.lx;
  M.L[1] = s.ly;
  M.L[2] = s.lz;
  for (int d = 0; d < 3; ++d) {
    M.h[d] = d < s.dim ? M.L[d] / M.n[d] : 1.0;
    M.g2[d] = d < s.dim ? 2 * M.n[d] + 1 : 1;
  }
  M.ne = M.n[0] * M.n[1] * M.n[2];
  M.N2 = M.g2[0] * M.g2[1] * M.g2[2];
  M.na = s.dim == 3 ? 27 : 9;
  M.npe = s.dim + 1;
  M.p_off = 2 * s.dim * M.N2;
  M.ndof = M.p_off + M.npe * M.ne;
  M.solid.assign(M.ne, 0);
  M.enodes.resize((size_t)M.ne * M.na);
  const int az_n = s.dim == 3 ? 3 : 1;
  for (int ez = 0; ez < M.n[2]; ++ez)
    for (int ey = 0; ey < M.n[1]; ++ey)
      for (int ex = 0; ex < M.n[0]; ++ex) {
        const int e = M.elem(ex, ey, ez);
        const double c[3] = {(ex + 0.5) * M.h[0], (ey + 0.5) * M.h[1], (ez + 0.5) * M.h[2]};
        bool in = true;
        for (int d = 0; d < s.dim; ++d) in = in && c[d] > s.solid_lo[d] && c[d] < s.solid_hi[d];
        M.solid[e] = in ? 1 : 0;
        int a = 0;
        for (int kz = 0; kz < az_n; ++kz)
          for (int ky = 0; ky < 3; ++ky)
            for (int kx = 0; kx < 3; ++kx)
              M.enodes[(size_t)e * M.na + a++] =
                  M.node(2 * ex + kx, 2 * ey + ky, s.dim == 3 ? 2 * ez + kz : 0);
      }
  std::vector<uint8_t> hs(M.N2, 0), hf(M.N2, 0);
  for (int e = 0; e < M.ne; ++e)
    for (int a = 0; a < M.na; ++a) (M.solid[e] ? hs : hf)[M.enodes[(size_t)e * M.na + a]] = 1;
  M.ncls.resize(M.N2);
  for (int i = 0; i < M.N2; ++i) M.ncls[i] = (hs[i] && hf[i]) ? NI : (hs[i] ? NS : NF);
  // Dirichlet: d = 0 on the outer boundary; u on inflow (profile) and walls (0)
  M.dir.assign(M.ndof, 0);
  M.dval.assign(M.ndof, 0.0);
  for (int i = 0; i < M.N2; ++i) {
    int I, J, K;
    M.grid(i, I, J, K);
    const bool lox = I == 0, hix = I == M.g2[0] - 1;
    bool wall = J == 0 || J == M.g2[1] - 1;
    if (s.dim == 3) wall = wall || K == 0 || K == M.g2[2] - 1;
    const bool bnd = lox || hix || wall;
    for (int c = 0; c < s.dim; ++c) {
      if (bnd) M.dir[M.d_dof(c, i)] = 1;
      if (lox || wall) {
        M.dir[M.u_dof(c, i)] = 1;
        if (c == 0 && lox && !wall)
          M.dval[M.u_dof(0, i)] = inflow(M, s.u_peak, J * M.h[1] / 2, K * M.h[2] / 2);
      }
    }
  }
  return M;
}

// ------------------------------------------------------------ quadrature tables
struct Tab {
  int nq = 0, na = 0, npe = 0, dim = 2;
  std::vector<double> N, dN, psi, w;  // N[q*na+a], dN[(q*na+a)*dim+k], psi[q*npe+j], w[q]
  double vol = 1.0;
};

static Tab make_tab(const Mesh &M) {
  Tab T;
  T.dim = M.dim;
  T.na = M.na;
  T.npe = M.npe;
  const double gp[3] = {0.5 * (1.0 - std::sqrt(0.6)), 0.5, 0.5 * (1.0 + std::sqrt(0.6))};
  const double gw[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
  auto b = [](int a, double t) {
    return a == 0 ? (2 * t - 1) * (t - 1) : (a == 1 ? 4 * t * (1 - t) : t * (2 * t - 1));
  };
  auto db = [](int a, double t) { return a == 0 ? 4 * t - 3 : (a == 1 ? 4 - 8 * t : 4 * t - 1); };
  const int q3 = M.dim == 3 ? 3 : 1;
  T.nq = 9 * q3;
  T.N.resize(T.nq * T.na);
  T.dN.resize(T.nq * T.na * M.dim);
  T.psi.resize(T.nq * T.npe);
  T.w.resize(T.nq);
  T.vol = M.h[0] * M.h[1] * (M.dim == 3 ? M.h[2] : 1.0);
  int q = 0;
  for (int qz = 0; qz < q3; ++qz)
    for (int qy = 0; qy < 3; ++qy)
      for (int qx = 0; qx < 3; ++qx, ++q) {
        const int qi[3] = {qx, qy, qz};
        double t[3];
        double wq = 1.0;
        for (int d = 0; d < M.dim; ++d) {
          t[d] = gp[qi[d]];
          wq *= gw[qi[d]] * M.h[d];
        }
        T.w[q] = wq;
        int a = 0;
        for (int az = 0; az < q3; ++az)
          for (int ay = 0; ay < 3; ++ay)
            for (int ax = 0; ax < 3; ++ax, ++a) {
              const int ai[3] = {ax, ay, az};
              double v = 1.0;
              for (int d = 0; d < M.dim; ++d) v *= b(ai[d], t[d]);
              T.N[q * T.na + a] = v;
              for (int k = 0; k < M.dim; ++k) {
                double g = 1.0;
                for (int d = 0; d < M.dim; ++d) g *= (d == k) ? db(ai[d], t[d]) / M.h[d] : b(ai[d], t[d]);
                T.dN[(q * T.na + a) * M.dim + k] = g;
              }
            }
        T.psi[q * T.npe] = 1.0;
        for (int d = 0; d < M.dim; ++d) T.psi[q * T.npe + 1 + d] = 2.0 * t[d] - 1.0;
      }
  return T;
}

// ------------------------------------------------------------ element kernel
// Plain-double forms of the dual helpers: the state at t_n of a time step is a
// constant of the Jacobian and runs through the same kinematics code.
inline void dzero(double &a) { a = 0.0; }
inline void dconst(double &a, double c) { a = c; }
inline void daxpy(double &a, double s, double b) { a += s * b; }
inline void dmul(double &r, double a, double b) { r = a * b; }
inline void dfma(double &a, double b, double c) { a += b * c; }
inline void dfms(double &a, double b, double c) { a -= b * c; }
inline void ddiv(double &r, double a, double b) { r = a / b; }
inline void dneg(double &a) { a = -a; }
inline void dscale(double &a, double s) { a *= s; }
inline void dshift(double &a, double c) { a += c; }
template <int N>
inline void dneg(Dual<N> &a) {
  a.v = -a.v;
  for (int i = 0; i < N; ++i) a.g[i] = -a.g[i];
}
template <int N>
inline void dscale(Dual<N> &a, double s) {
  a.v *= s;
  for (int i = 0; i < N; ++i) a.g[i] *= s;
}
// a += c for a constant c
template <int N>
inline void dshift(Dual<N> &a, double c) {
  a.v += c;
}

// fields of one state at one quadrature point
template <int DIM, typename V>
struct Kin {
  V Gd[DIM][DIM], F[DIM][DIM], Fi[DIM][DIM], det, pq, uq[DIM], dq[DIM], gu[DIM][DIM];
};

// grad_hat d, F = I + grad_hat d, J = det F, F^{-1} by cofactors, p, u and d
// at the point and, for a fluid element, the Eulerian velocity gradient
// grad u = grad_hat u F^{-1}
template <int DIM, int NA, int NP, typename V, class FD, class FU, class FP>
static void kinematics(const double *Nq, const double *dNq, const double *ps, FD D, FU U, FP Pp,
                       bool fluid, Kin<DIM, V> &k) {
  for (int c = 0; c < DIM; ++c)
    for (int j = 0; j < DIM; ++j) {
      dzero(k.Gd[c][j]);
      for (int a = 0; a < NA; ++a) daxpy(k.Gd[c][j], dNq[a * DIM + j], D(c, a));
      k.F[c][j] = k.Gd[c][j];
      if (c == j) dshift(k.F[c][j], 1.0);
    }
  if constexpr (DIM == 2) {
    dmul(k.det, k.F[0][0], k.F[1][1]);
    dfms(k.det, k.F[0][1], k.F[1][0]);
    ddiv(k.Fi[0][0], k.F[1][1], k.det);
    ddiv(k.Fi[1][1], k.F[0][0], k.det);
    ddiv(k.Fi[0][1], k.F[0][1], k.det);
    ddiv(k.Fi[1][0], k.F[1][0], k.det);
    dneg(k.Fi[0][1]);
    dneg(k.Fi[1][0]);
  } else {
    V cof[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
        dmul(cof[i][j], k.F[i1 % DIM][j1 % DIM], k.F[i2 % DIM][j2 % DIM]);
        dfms(cof[i][j], k.F[i1 % DIM][j2 % DIM], k.F[i2 % DIM][j1 % DIM]);
      }
    dmul(k.det, k.F[0][0], cof[0][0]);
    dfma(k.det, k.F[0][1], cof[0][1]);
    dfma(k.det, k.F[0][2 % DIM], cof[0][2]);
    for (int i = 0; i < DIM; ++i)
      for (int j = 0; j < DIM; ++j) ddiv(k.Fi[i][j], cof[j][i], k.det);
  }
  dconst(k.pq, 0.0);
  for (int j = 0; j < NP; ++j) daxpy(k.pq, ps[j], Pp(j));
  for (int c = 0; c < DIM; ++c) {
    dzero(k.uq[c]);
    dzero(k.dq[c]);
    for (int a = 0; a < NA; ++a) {
      daxpy(k.uq[c], Nq[a], U(c, a));
      daxpy(k.dq[c], Nq[a], D(c, a));
    }
  }
  if (!fluid) return;
  V Gu[DIM][DIM];
  for (int c = 0; c < DIM; ++c)
    for (int j = 0; j < DIM; ++j) {
      dzero(Gu[c][j]);
      for (int a = 0; a < NA; ++a) daxpy(Gu[c][j], dNq[a * DIM + j], U(c, a));
    }
  for (int c = 0; c < DIM; ++c)
    for (int b = 0; b < DIM; ++b) {
      dzero(k.gu[c][b]);
      for (int j = 0; j < DIM; ++j) dfma(k.gu[c][b], Gu[c][j], k.Fi[j][b]);
    }
}

// fluid Cauchy stress -p I + mu (grad u + grad u^T) and, for the solid, the
// first Piola stress J sigma F^{-T} with sigma = -p I + mu_s F F^T
template <int DIM, typename V>
static void fluid_stress(const Kin<DIM, V> &k, double mu, V (&sig)[DIM][DIM]) {
  for (int c = 0; c < DIM; ++c)
    for (int b = 0; b < DIM; ++b) {
      dzero(sig[c][b]);
      daxpy(sig[c][b], mu, k.gu[c][b]);
      daxpy(sig[c][b], mu, k.gu[b][c]);
      if (b == c) daxpy(sig[c][b], -1.0, k.pq);
    }
}
template <int DIM, typename V>
static void piola(const Kin<DIM, V> &k, double mu_s, V (&P)[DIM][DIM]) {
  V sig[DIM][DIM], t;
  for (int c = 0; c < DIM; ++c)
    for (int b = 0; b < DIM; ++b) {
      dzero(sig[c][b]);
      for (int j = 0; j < DIM; ++j) dfma(sig[c][b], k.F[c][j], k.F[b][j]);
      dscale(sig[c][b], mu_s);
      if (b == c) daxpy(sig[c][b], -1.0, k.pq);
    }
  for (int c = 0; c < DIM; ++c)
    for (int b = 0; b < DIM; ++b) {
      dzero(t);
      for (int j = 0; j < DIM; ++j) dfma(t, sig[c][j], k.Fi[b][j]);
      dmul(P[c][b], k.det, t);
    }
}

// Local dofs: [d_c(a)] c-major, [u_c(a)], [p_j]; local rows: [mom_c(a)], [aux_c(a)], [pres_j].
template <int DIM, int NL>
struct ElemOut {
  Dual<NL> rows[NL];
};

// Local residual rows of one element with their derivatives in the element's
// dofs.  Steady form when ye0 is null; otherwise one Crank-Nicolson step from
// the state ye0 at t_n to ye at t_{n+1} (section "Discretization of the
// operator formulation"): fluid momentum (rho/dt)(J1 u1 - J0 u0) phi plus half
// of each of -rho div(w) u phi + rho ((u - w).grad) u phi + sigma : grad phi
// on the configurations of t_{n+1} and t_n, mesh velocity w = (d1 - d0)/dt;
// continuity and mesh motion at t_{n+1}; solid momentum (rho_s/dt)(J1 u1 -
// J0 u0) phi plus half of each Piola term; incompressibility at t_{n+1};
// kinematics -(d1 - d0)/dt + (u1 + u0)/2 against phi.
template <int DIM, int NL>
static void element(const Mesh &, const Tab &T, const fsi_problem_spec &s, bool solid, const double *ye,
                    const double *ye0, ElemOut<DIM, NL> &out, bool want_grad) {
  constexpr int NA = DIM == 3 ? 27 : 9;
  constexpr int NP = DIM + 1;
  using DN = Dual<NL>;
  static_assert(NL == 2 * DIM * NA + NP, "local size");
  for (int r = 0; r < NL; ++r) dzero(out.rows[r]);
  thread_local std::vector<DN> dofs;
  dofs.resize(NL);
  for (int i = 0; i < NL; ++i) {
    dconst(dofs[i], ye[i]);
    if (want_grad) dofs[i].g[i] = 1.0;
  }
  auto D = [&](int c, int a) -> const DN & { return dofs[c * NA + a]; };
  auto U = [&](int c, int a) -> const DN & { return dofs[(DIM + c) * NA + a]; };
  auto Pp = [&](int j) -> const DN & { return dofs[2 * DIM * NA + j]; };
  auto D0 = [&](int c, int a) { return ye0[c * NA + a]; };
  auto U0 = [&](int c, int a) { return ye0[(DIM + c) * NA + a]; };
  auto P0 = [&](int j) { return ye0[2 * DIM * NA + j]; };
  const bool cn = ye0 != nullptr;
  const double dt = s.dt;
  DN *mom = out.rows, *aux = out.rows + DIM * NA, *pres = out.rows + 2 * DIM * NA;
  const double k_ale = 1.0 / T.vol;
  Kin<DIM, DN> k1;
  Kin<DIM, double> k0;
  DN sig1[DIM][DIM], Tm[DIM][DIM], S[DIM], t1, t2;
  double sig0[DIM][DIM];
  for (int q = 0; q < T.nq; ++q) {
    const double *Nq = &T.N[q * NA];
    const double *dNq = &T.dN[q * NA * DIM];
    const double *ps = &T.psi[q * NP];
    const double w = T.w[q];
    kinematics<DIM, NA, NP>(Nq, dNq, ps, D, U, Pp, !solid, k1);
    if (cn) kinematics<DIM, NA, NP>(Nq, dNq, ps, D0, U0, P0, !solid, k0);
    if (!solid) {
      fluid_stress(k1, s.mu, sig1);
      DN wJ1;
      dconst(wJ1, 0.0);
      daxpy(wJ1, w, k1.det);
      if (!cn) {
        // rho ((u . grad) u) and sigma against grad phi, weighted by w J
        for (int c = 0; c < DIM; ++c) {
          dzero(t1);
          for (int b = 0; b < DIM; ++b) dfma(t1, k1.gu[c][b], k1.uq[b]);
          dmul(S[c], wJ1, t1);
          dscale(S[c], s.rho);
          for (int j = 0; j < DIM; ++j) {
            dzero(t2);
            for (int b = 0; b < DIM; ++b) dfma(t2, sig1[c][b], k1.Fi[j][b]);
            dmul(Tm[c][j], wJ1, t2);
          }
        }
      } else {
        fluid_stress(k0, s.mu, sig0);
        const double wJ0 = w * k0.det;
        DN wq[DIM], Gw[DIM][DIM], divw1, divw0;
        for (int c = 0; c < DIM; ++c) {
          dzero(wq[c]);
          daxpy(wq[c], 1.0 / dt, k1.dq[c]);
          dshift(wq[c], -k0.dq[c] / dt);
          for (int j = 0; j < DIM; ++j) {
            dzero(Gw[c][j]);
            daxpy(Gw[c][j], 1.0 / dt, k1.Gd[c][j]);
            dshift(Gw[c][j], -k0.Gd[c][j] / dt);
          }
        }
        dzero(divw1);
        dzero(divw0);
        for (int c = 0; c < DIM; ++c)
          for (int j = 0; j < DIM; ++j) {
            dfma(divw1, Gw[c][j], k1.Fi[j][c]);
            daxpy(divw0, k0.Fi[j][c], Gw[c][j]);
          }
        for (int c = 0; c < DIM; ++c) {
          // t_{n+1}: (rho/dt) u1 + rho/2 (-div(w) u1 + grad u1 (u1 - w))
          dzero(t1);
          dfms(t1, divw1, k1.uq[c]);
          for (int b = 0; b < DIM; ++b) {
            dfma(t1, k1.gu[c][b], k1.uq[b]);
            dfms(t1, k1.gu[c][b], wq[b]);
          }
          dscale(t1, 0.5 * s.rho);
          daxpy(t1, s.rho / dt, k1.uq[c]);
          dmul(S[c], wJ1, t1);
          // t_n: -(rho/dt) u0 + rho/2 (-div(w) u0 + grad u0 (u0 - w))
          dzero(t2);
          daxpy(t2, -k0.uq[c], divw0);
          for (int b = 0; b < DIM; ++b) {
            dshift(t2, k0.gu[c][b] * k0.uq[b]);
            daxpy(t2, -k0.gu[c][b], wq[b]);
          }
          dscale(t2, 0.5 * s.rho);
          dshift(t2, -(s.rho / dt) * k0.uq[c]);
          daxpy(S[c], wJ0, t2);
          // half of each stress term
          for (int j = 0; j < DIM; ++j) {
            dzero(t2);
            double c0 = 0.0;
            for (int b = 0; b < DIM; ++b) {
              dfma(t2, sig1[c][b], k1.Fi[j][b]);
              c0 += sig0[c][b] * k0.Fi[j][b];
            }
            dmul(Tm[c][j], wJ1, t2);
            dscale(Tm[c][j], 0.5);
            dshift(Tm[c][j], 0.5 * wJ0 * c0);
          }
        }
      }
      for (int c = 0; c < DIM; ++c)
        for (int a = 0; a < NA; ++a) {
          DN &R = mom[c * NA + a];
          daxpy(R, Nq[a], S[c]);
          for (int j = 0; j < DIM; ++j) daxpy(R, dNq[a * DIM + j], Tm[c][j]);
          DN &A = aux[c * NA + a];
          for (int b = 0; b < DIM; ++b) daxpy(A, w * k_ale * dNq[a * DIM + b], k1.Gd[c][b]);
        }
      dzero(t1);
      for (int c = 0; c < DIM; ++c) daxpy(t1, 1.0, k1.gu[c][c]);
      dmul(t2, wJ1, t1);
      for (int j = 0; j < NP; ++j) daxpy(pres[j], ps[j], t2);
    } else {
      piola(k1, s.mu_s, Tm);
      double P0m[DIM][DIM] = {};
      if (cn) piola(k0, s.mu_s, P0m);
      const double half = cn ? 0.5 : 1.0;
      for (int c = 0; c < DIM; ++c) {
        // (rho_s/dt)(J1 u1 - J0 u0) in a time step
        if (cn) {
          dmul(S[c], k1.det, k1.uq[c]);
          dshift(S[c], -k0.det * k0.uq[c]);
          dscale(S[c], s.rho_s / dt);
        }
        // kinematics: u (steady), -(d1 - d0)/dt + (u1 + u0)/2 (time step)
        dzero(t1);
        if (cn) {
          daxpy(t1, -1.0 / dt, k1.dq[c]);
          daxpy(t1, 0.5, k1.uq[c]);
          dshift(t1, k0.dq[c] / dt + 0.5 * k0.uq[c]);
        } else {
          daxpy(t1, 1.0, k1.uq[c]);
        }
        for (int a = 0; a < NA; ++a) {
          DN &R = mom[c * NA + a];
          if (cn) daxpy(R, w * Nq[a], S[c]);
          for (int b = 0; b < DIM; ++b) {
            daxpy(R, half * w * dNq[a * DIM + b], Tm[c][b]);
            if (cn) dshift(R, half * w * dNq[a * DIM + b] * P0m[c][b]);
          }
          daxpy(aux[c * NA + a], w * Nq[a], t1);
        }
      }
      dconst(t1, -1.0);
      daxpy(t1, 1.0, k1.det);
      for (int j = 0; j < NP; ++j) daxpy(pres[j], w * ps[j], t1);
    }
  }
}

// Structural coupling of local row lr with local column lc.  A time step adds
// the solid momentum's mass term on the same velocity component and the
// kinematics' time difference on the same displacement component (the blocks
// that vanish only in the steady case, section "Structure of the Jacobian").
static bool coupled(int dim, int na, bool solid, bool transient, int lr, int lc) {
  const int nd = dim * na;
  const int rblk = lr < nd ? 0 : (lr < 2 * nd ? 1 : 2);   // mom, aux, pres
  const int cblk = lc < nd ? 0 : (lc < 2 * nd ? 1 : 2);   // d, u, p
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

// global target row of local row lr of element e (-1: dropped)
static int target_row(const Mesh &M, int e, int lr) {
  const int nd = M.dim * M.na;
  if (lr >= 2 * nd) return M.p_dof(e, lr - 2 * nd);
  const bool aux = lr >= nd;
  const int c = (lr % nd) / M.na, a = lr % M.na;
  const int nodeid = M.enodes[(size_t)e * M.na + a];
  const int cls = M.ncls[nodeid];
  if (M.solid[e]) return aux ? M.u_dof(c, nodeid) : M.d_dof(c, nodeid);
  if (cls == NF) return aux ? M.d_dof(c, nodeid) : M.u_dof(c, nodeid);
  return aux ? -1 : M.d_dof(c, nodeid);  // interface node in a fluid element
}

static int local_col_dof(const Mesh &M, int e, int lc) {
  const int nd = M.dim * M.na;
  if (lc >= 2 * nd) return M.p_dof(e, lc - 2 * nd);
  const int c = (lc % nd) / M.na, a = lc % M.na;
  const int nodeid = M.enodes[(size_t)e * M.na + a];
  return lc < nd ? M.d_dof(c, nodeid) : M.u_dof(c, nodeid);
}

struct Csr {
  int nrows = 0, ncols = 0;
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<double> v;
};

// sparsity from the structural rule, then values by element colouring
template <int DIM, int NL>
static void assemble(const Mesh &M, const fsi_problem_spec &s, const std::vector<double> &y,
                     const std::vector<double> *y_prev, std::vector<double> &r, Csr *J) {
  const bool tr = y_prev != nullptr;
  constexpr int NA = DIM == 3 ? 27 : 9;
  const Tab T = make_tab(M);
  std::vector<std::vector<int>> loc(M.ne);
  auto l2g = [&](int e, std::vector<int> &g) {
    g.resize(NL);
    for (int lc = 0; lc < NL; ++lc) g[lc] = local_col_dof(M, e, lc);
  };
  r.assign(M.ndof, 0.0);
  if (J) {
    std::vector<std::vector<int32_t>> rows(M.ndof);
    std::vector<int> g;
    for (int e = 0; e < M.ne; ++e) {
      l2g(e, g);
      for (int lr = 0; lr < NL; ++lr) {
        const int t = target_row(M, e, lr);
        if (t < 0 || M.dir[t]) continue;
        for (int lc = 0; lc < NL; ++lc)
          if (coupled(DIM, NA, M.solid[e], tr, lr, lc) && !M.dir[g[lc]]) rows[t].push_back(g[lc]);
      }
    }
    for (int i = 0; i < M.ndof; ++i)
      if (M.dir[i]) rows[i].push_back(i);
    J->nrows = J->ncols = M.ndof;
    J->rp.assign(M.ndof + 1, 0);
    for (int i = 0; i < M.ndof; ++i) {
      auto &v = rows[i];
      std::sort(v.begin(), v.end());
      v.erase(std::unique(v.begin(), v.end()), v.end());
      J->rp[i + 1] = J->rp[i] + (int64_t)v.size();
    }
    J->ci.resize(J->rp[M.ndof]);
    J->v.assign(J->rp[M.ndof], 0.0);
    for (int i = 0; i < M.ndof; ++i) {
      std::copy(rows[i].begin(), rows[i].end(), J->ci.begin() + J->rp[i]);
      if (M.dir[i]) J->v[J->rp[i]] = 1.0;
    }
  }
  // element colouring: (ex, ey, ez) parities; same colour => no shared node
  const int ncol = DIM == 3 ? 8 : 4;
  for (int color = 0; color < ncol; ++color) {
    std::vector<int> els;
    for (int e = 0; e < M.ne; ++e) {
      const int ex = e % M.n[0], ey = (e / M.n[0]) % M.n[1], ez = e / (M.n[0] * M.n[1]);
      if ((ex & 1) + 2 * (ey & 1) + 4 * (ez & 1) == color) els.push_back(e);
    }
#pragma omp parallel
    {
      std::unique_ptr<ElemOut<DIM, NL>> out(new ElemOut<DIM, NL>());
      std::vector<int> g;
      std::vector<double> ye(NL), ye0(tr ? NL : 0);
#pragma omp for schedule(dynamic, 4)
      for (size_t ii = 0; ii < els.size(); ++ii) {
        const int e = els[ii];
        for (int lc = 0; lc < NL; ++lc) ye[lc] = y[local_col_dof(M, e, lc)];
        if (tr)
          for (int lc = 0; lc < NL; ++lc) ye0[lc] = (*y_prev)[local_col_dof(M, e, lc)];
        element<DIM, NL>(M, T, s, M.solid[e], ye.data(), tr ? ye0.data() : nullptr, *out, J != nullptr);
        for (int lr = 0; lr < NL; ++lr) {
          const int t = target_row(M, e, lr);
          if (t < 0) continue;
          r[t] += out->rows[lr].v;
          if (!J || M.dir[t]) continue;
          const int64_t a = J->rp[t], b = J->rp[t + 1];
          for (int lc = 0; lc < NL; ++lc) {
            if (!coupled(DIM, NA, M.solid[e], tr, lr, lc)) continue;
            const int gc = local_col_dof(M, e, lc);
            if (M.dir[gc]) continue;
            const int64_t pos = std::lower_bound(J->ci.begin() + a, J->ci.begin() + b, gc) - J->ci.begin();
            J->v[pos] += out->rows[lr].g[lc];
          }
        }
      }
    }
  }
  for (int i = 0; i < M.ndof; ++i)
    if (M.dir[i]) r[i] = y[i] - M.dval[i];
}

// ------------------------------------------------------------ state
// S_c / max|S_c| at the Q2 nodes, c = 0..dim-1, with
// S_c = sum_{k,l(,m)=1..K} a_{c,k,l(,m)} / (k^2+l^2(+m^2)) prod sin(k pi x / L)
static std::vector<std::vector<double>> fourier_shapes(const Mesh &M, const fsi_problem_spec &s) {
  const int K = s.kmax;
  const int nmodes = (int)std::lround(std::pow((double)K, s.dim));
  std::vector<std::vector<double>> out(s.dim);
  for (int c = 0; c < s.dim; ++c) {
    std::vector<double> &S = out[c];
    S.assign(M.N2, 0.0);
    for (int i = 0; i < M.N2; ++i) {
      int I, J, Kz;
      M.grid(i, I, J, Kz);
      const double x[3] = {I * M.h[0] / 2, J * M.h[1] / 2, Kz * M.h[2] / 2};
      double acc = 0.0;
      for (int md = 0; md < nmodes; ++md) {
        int kk[3] = {1, 1, 1}, rem = md;
        for (int d = s.dim - 1; d >= 0; --d) {
          kk[d] = rem % K + 1;
          rem /= K;
        }
        double t = s.coeffs[(size_t)c * nmodes + md];
        double den = 0.0;
        for (int d = 0; d < s.dim; ++d) den += kk[d] * kk[d];
        t /= den;
        for (int d = 0; d < s.dim; ++d) t *= std::sin(kk[d] * M_PI * x[d] / M.L[d]);
        acc += t;
      }
      S[i] = acc;
    }
    double mx = 0.0;
    for (double v : S) mx = std::max(mx, std::fabs(v));
    for (double &v : S) v /= mx;
  }
  return out;
}

// Seeded linearisation state: d = 0, fluid-only velocities carry the inflow
// profile plus amp * S_c / max|S_c|, solid pressure mu_s (stress-free solid),
// Dirichlet dofs their boundary values.  For a time step this is the state at
// t_n and y1 (the Newton iterate at t_{n+1}) moves every free displacement by
// amp_d * S_c / max|S_c|.
static std::vector<double> make_state(const Mesh &M, const fsi_problem_spec &s, std::vector<double> *y1) {
  std::vector<double> y(M.ndof, 0.0);
  const auto shapes = fourier_shapes(M, s);
  for (int c = 0; c < s.dim; ++c)
    for (int i = 0; i < M.N2; ++i) {
      double u = 0.0;
      if (M.ncls[i] == NF) {
        int I, J, Kz;
        M.grid(i, I, J, Kz);
        u = s.amp * shapes[c][i];
        if (c == 0) u += inflow(M, s.u_peak, J * M.h[1] / 2, Kz * M.h[2] / 2);
      }
      y[M.u_dof(c, i)] = u;
    }
  for (int e = 0; e < M.ne; ++e)
    if (M.solid[e]) y[M.p_dof(e, 0)] = s.mu_s;
  for (int i = 0; i < M.ndof; ++i)
    if (M.dir[i]) y[i] = M.dval[i];
  if (y1) {
    *y1 = y;
    for (int c = 0; c < s.dim; ++c)
      for (int i = 0; i < M.N2; ++i) {
        const int dd = M.d_dof(c, i);
        if (!M.dir[dd]) (*y1)[dd] += s.amp_d * shapes[c][i];
      }
  }
  return y;
}

// ------------------------------------------------------------ transfers
// coarse Q2 nodes and weights for fine Q2 grid index I (1D)
static int q2w(int I, int nc, int *idx, double *w) {
  int ec = std::min(I / 4, nc - 1);
  const int loc = I - 4 * ec;  // 0..4 quarter steps
  static const double tab[5][3] = {{1, 0, 0},
                                   {0.375, 0.75, -0.125},
                                   {0, 1, 0},
                                   {-0.125, 0.75, 0.375},
                                   {0, 0, 1}};
  int k = 0;
  for (int a = 0; a < 3; ++a)
    if (tab[loc][a] != 0.0) {
      idx[k] = 2 * ec + a;
      w[k] = tab[loc][a];
      ++k;
    }
  return k;
}

// row types: 0 ALE, 1 SM, 2 IM, 3 FM, 4 KS, 5 PF, 6 PS
static int row_type(const Mesh &M, int dof) {
  if (dof >= M.p_off) return M.solid[(dof - M.p_off) / M.npe] ? 6 : 5;
  const int field = dof / M.N2, nd = dof % M.N2;
  const bool dslot = field < M.dim;
  const int cls = M.ncls[nd];
  if (dslot) return cls == NF ? 0 : (cls == NS ? 1 : 2);
  return cls == NF ? 3 : 4;
}
static bool compatible(int tc, int tf) {
  const bool mc = tc >= 1 && tc <= 3, mf = tf >= 1 && tf <= 3;
  if (mc || mf) return mc && mf;
  return tc == tf;
}

struct Trip {
  int r, c;
  double v;
};
static Csr from_trips(int nr, int nc, std::vector<Trip> &t) {
  std::sort(t.begin(), t.end(), [](const Trip &a, const Trip &b) { return a.r < b.r || (a.r == b.r && a.c < b.c); });
  Csr A;
  A.nrows = nr;
  A.ncols = nc;
  A.rp.assign(nr + 1, 0);
  for (size_t i = 0; i < t.size(); ++i) {
    if (i > 0 && t[i].r == t[i - 1].r && t[i].c == t[i - 1].c) {
      A.v.back() += t[i].v;
      continue;
    }
    A.ci.push_back(t[i].c);
    A.v.push_back(t[i].v);
    A.rp[t[i].r + 1]++;
  }
  for (int i = 0; i < nr; ++i) A.rp[i + 1] += A.rp[i];
  return A;
}

// P (fine x coarse) and R (coarse x fine)
static void transfers(const Mesh &F, const Mesh &C, Csr &P, Csr &R) {
  std::vector<Trip> tp, tr;
  const int dim = F.dim;
  for (int j = 0; j < F.N2; ++j) {
    int I[3];
    F.grid(j, I[0], I[1], I[2]);
    int idx[3][3];
    double w[3][3];
    int cnt[3] = {1, 1, 1};
    for (int d = 0; d < 3; ++d) {
      if (d < dim) {
        cnt[d] = q2w(I[d], C.n[d], idx[d], w[d]);
      } else {
        idx[d][0] = 0;
        w[d][0] = 1.0;
      }
    }
    for (int a = 0; a < cnt[0]; ++a)
      for (int b = 0; b < cnt[1]; ++b)
        for (int c3 = 0; c3 < cnt[2]; ++c3) {
          const int ci = C.node(idx[0][a], idx[1][b], idx[2][c3]);
          const double wt = w[0][a] * w[1][b] * w[2][c3];
          for (int f = 0; f < 2 * dim; ++f) {
            const int fd = f * F.N2 + j, cd = f * C.N2 + ci;
            if (!F.dir[fd] && !C.dir[cd]) tp.push_back({fd, cd, wt});
          }
          for (int comp = 0; comp < dim; ++comp)
            for (int sf = 0; sf < 2; ++sf)
              for (int sc = 0; sc < 2; ++sc) {
                const int fr = (sf * dim + comp) * F.N2 + j, cr = (sc * dim + comp) * C.N2 + ci;
                if (F.dir[fr] || C.dir[cr]) continue;
                if (compatible(row_type(C, cr), row_type(F, fr))) tr.push_back({cr, fr, wt});
              }
        }
  }
  // P1disc: child coefficients b0 = a0 + sum_d s_d a_d / 2, b_d = a_d / 2
  for (int e = 0; e < F.ne; ++e) {
    const int ex = e % F.n[0], ey = (e / F.n[0]) % F.n[1], ez = e / (F.n[0] * F.n[1]);
    const int ix[3] = {ex, ey, ez};
    const int E = C.elem(ex / 2, ey / 2, dim == 3 ? ez / 2 : 0);
    auto add = [&](int fr, int cc, double v) {
      tp.push_back({fr, cc, v});
      tr.push_back({cc, fr, v});
    };
    add(F.p_dof(e, 0), C.p_dof(E, 0), 1.0);
    for (int d = 0; d < dim; ++d) {
      const double sgn = (ix[d] % 2 == 0) ? -1.0 : 1.0;
      add(F.p_dof(e, 0), C.p_dof(E, 1 + d), 0.5 * sgn);
      add(F.p_dof(e, 1 + d), C.p_dof(E, 1 + d), 0.5);
    }
  }
  P = from_trips(F.ndof, C.ndof, tp);
  R = from_trips(C.ndof, F.ndof, tr);
}

// C = A * B (Gustavson, row-parallel)
static Csr spgemm(const Csr &A, const Csr &B) {
  Csr Cm;
  Cm.nrows = A.nrows;
  Cm.ncols = B.ncols;
  std::vector<std::vector<int32_t>> cols(A.nrows);
  std::vector<std::vector<double>> vals(A.nrows);
#pragma omp parallel
  {
    std::vector<double> acc(B.ncols, 0.0);
    std::vector<int> mark(B.ncols, -1);
    std::vector<int32_t> list;
#pragma omp for schedule(dynamic, 64)
    for (int i = 0; i < A.nrows; ++i) {
      list.clear();
      for (int64_t p = A.rp[i]; p < A.rp[i + 1]; ++p) {
        const int k = A.ci[p];
        const double a = A.v[p];
        for (int64_t q = B.rp[k]; q < B.rp[k + 1]; ++q) {
          const int c = B.ci[q];
          if (mark[c] != i) {
            mark[c] = i;
            acc[c] = 0.0;
            list.push_back(c);
          }
          acc[c] += a * B.v[q];
        }
      }
      std::sort(list.begin(), list.end());
      cols[i] = list;
      vals[i].resize(list.size());
      for (size_t t = 0; t < list.size(); ++t) vals[i][t] = acc[list[t]];
    }
  }
  Cm.rp.assign(A.nrows + 1, 0);
  for (int i = 0; i < A.nrows; ++i) Cm.rp[i + 1] = Cm.rp[i] + (int64_t)cols[i].size();
  Cm.ci.resize(Cm.rp[A.nrows]);
  Cm.v.resize(Cm.rp[A.nrows]);
  for (int i = 0; i < A.nrows; ++i) {
    std::copy(cols[i].begin(), cols[i].end(), Cm.ci.begin() + Cm.rp[i]);
    std::copy(vals[i].begin(), vals[i].end(), Cm.v.begin() + Cm.rp[i]);
  }
  return Cm;
}

// identity at Dirichlet rows (rows/columns of R J P are zero there)
static void set_dirichlet_diag(Csr &A, const std::vector<uint8_t> &dir) {
  std::vector<Trip> t;
  for (int i = 0; i < A.nrows; ++i) {
    for (int64_t p = A.rp[i]; p < A.rp[i + 1]; ++p) t.push_back({i, A.ci[p], A.v[p]});
    if (dir[i]) t.push_back({i, i, 1.0});
  }
  A = from_trips(A.nrows, A.ncols, t);
}

// ------------------------------------------------------------ patches
struct Patches {
  std::vector<int64_t> ptr;
  std::vector<int32_t> dof;
  std::vector<uint8_t> owned, kind;
};

static Patches make_patches(const Mesh &M, int p) {
  for (int d = 0; d < M.dim; ++d)
    if (M.n[d] % p) throw Err("mesh not divisible by the patch size");
  const int nb[3] = {M.n[0] / p, M.n[1] / p, M.dim == 3 ? M.n[2] / p : 1};
  std::vector<std::vector<int32_t>> solid_l, fluid_l;
  for (int bz = 0; bz < nb[2]; ++bz)
    for (int by = 0; by < nb[1]; ++by)
      for (int bx = 0; bx < nb[0]; ++bx) {
        std::vector<int32_t> sd, fd;
        const int zr = M.dim == 3 ? p : 1;
        for (int kz = 0; kz < zr; ++kz)
          for (int ky = 0; ky < p; ++ky)
            for (int kx = 0; kx < p; ++kx) {
              const int e = M.elem(bx * p + kx, by * p + ky, M.dim == 3 ? bz * p + kz : 0);
              auto &dst = M.solid[e] ? sd : fd;
              for (int a = 0; a < M.na; ++a) {
                const int nd = M.enodes[(size_t)e * M.na + a];
                for (int c = 0; c < M.dim; ++c) {
                  dst.push_back(M.d_dof(c, nd));
                  dst.push_back(M.u_dof(c, nd));
                }
              }
              for (int j = 0; j < M.npe; ++j) dst.push_back(M.p_dof(e, j));
            }
        for (auto *v : {&sd, &fd}) {
          std::sort(v->begin(), v->end());
          v->erase(std::unique(v->begin(), v->end()), v->end());
          v->erase(std::remove_if(v->begin(), v->end(), [&](int32_t d) { return M.dir[d] != 0; }),
                   v->end());
        }
        if (!sd.empty()) solid_l.push_back(sd);
        if (!fd.empty()) fluid_l.push_back(fd);
      }
  Patches P;
  P.ptr.push_back(0);
  std::vector<uint8_t> taken(M.ndof, 0);
  auto emit = [&](const std::vector<int32_t> &v, uint8_t kind) {
    for (int32_t d : v) {
      P.dof.push_back(d);
      P.owned.push_back(taken[d] ? 0 : 1);
      taken[d] = 1;
    }
    P.kind.push_back(kind);
    P.ptr.push_back((int64_t)P.dof.size());
  };
  for (auto &v : solid_l) emit(v, 1);
  for (auto &v : fluid_l) emit(v, 0);
  return P;
}

// ------------------------------------------------------------ problem
struct Problem {
  fsi_problem_spec spec;
  std::vector<double> coeffs;
  std::vector<Mesh> meshes;  // coarsest first
  std::vector<Csr> J, P, R;
  std::vector<Patches> patches;
  std::vector<double> y, b;
  std::vector<double> y_prev;  // state at t_n of a time step (empty: steady)
  // the finest level's element data (fsi_problem_element_data)
  std::vector<int32_t> l2g, tgt, color_ptr, color_elems;
  Tab tab;
};

static void residual_jacobian(const Mesh &M, const fsi_problem_spec &s, const std::vector<double> &y,
                              const std::vector<double> *y_prev, std::vector<double> &r, Csr *J) {
  if (M.dim == 2)
    assemble<2, 39>(M, s, y, y_prev, r, J);
  else
    assemble<3, 166>(M, s, y, y_prev, r, J);
}

static Problem *build(const fsi_problem_spec &s0) {
  if (s0.dim != 2 && s0.dim != 3) throw Err("dim must be 2 or 3");
  if (s0.levels < 1 || s0.patch < 1 || s0.kmax < 1 || !s0.coeffs) throw Err("invalid spec");
  if (s0.transient && !(s0.dt > 0.0 && std::isfinite(s0.dt) && s0.rho_s >= 0.0 && std::isfinite(s0.amp_d)))
    throw Err("a time step needs dt > 0, rho_s >= 0 and a finite amp_d");
  std::unique_ptr<Problem> pb(new Problem());
  pb->spec = s0;
  const int nmodes = (int)std::lround(std::pow((double)s0.kmax, s0.dim));
  pb->coeffs.assign(s0.coeffs, s0.coeffs + (size_t)s0.dim * nmodes);
  pb->spec.coeffs = pb->coeffs.data();
  const fsi_problem_spec &s = pb->spec;
  const int L = s.levels;
  const int f = 1 << (L - 1);
  const int nf[3] = {s.nx, s.ny, s.dim == 3 ? s.nz : 1};
  for (int d = 0; d < s.dim; ++d)
    if (nf[d] % f || (L > 1 && (nf[d] / f) < 1)) throw Err("mesh not divisible by 2^(levels-1)");
  for (int l = 0; l < L; ++l) {
    const int sc = 1 << (L - 1 - l);
    Mesh M = make_mesh(s, s.nx / sc, s.ny / sc, s.dim == 3 ? s.nz / sc : 1);
    // the solid box must be element-aligned on every level
    for (int d = 0; d < s.dim; ++d)
      for (double x : {s.solid_lo[d], s.solid_hi[d]}) {
        if (x <= 0.0 || x >= M.L[d]) continue;
        const double q = x / M.h[d];
        if (std::fabs(q - std::round(q)) > 1e-9) throw Err("solid box not element-aligned on a level");
      }
    pb->meshes.push_back(std::move(M));
  }
  const Mesh &Fm = pb->meshes.back();
  const std::vector<double> *yp = nullptr;
  if (s.transient) {
    pb->y_prev = make_state(Fm, s, &pb->y);
    yp = &pb->y_prev;
  } else {
    pb->y = make_state(Fm, s, nullptr);
  }
  pb->J.resize(L);
  pb->P.resize(L);
  pb->R.resize(L);
  std::vector<double> r;
  residual_jacobian(Fm, s, pb->y, yp, r, &pb->J[L - 1]);
  pb->b.resize(Fm.ndof);
  for (int i = 0; i < Fm.ndof; ++i) pb->b[i] = Fm.dir[i] ? 0.0 : -r[i];
  for (int l = L - 1; l >= 1; --l) {
    transfers(pb->meshes[l], pb->meshes[l - 1], pb->P[l], pb->R[l]);
    Csr JP = spgemm(pb->J[l], pb->P[l]);
    pb->J[l - 1] = spgemm(pb->R[l], JP);
    set_dirichlet_diag(pb->J[l - 1], pb->meshes[l - 1].dir);
  }
  pb->patches.resize(L);
  for (int l = 1; l < L; ++l) pb->patches[l] = make_patches(pb->meshes[l], s.patch);
  // element data of the finest level, colours by element parity as the assembly's
  const int nl = 2 * Fm.dim * Fm.na + Fm.npe;
  pb->l2g.resize((size_t)Fm.ne * nl);
  pb->tgt.resize((size_t)Fm.ne * nl);
  for (int e = 0; e < Fm.ne; ++e)
    for (int q = 0; q < nl; ++q) {
      pb->l2g[(size_t)e * nl + q] = local_col_dof(Fm, e, q);
      pb->tgt[(size_t)e * nl + q] = target_row(Fm, e, q);
    }
  const int ncol = Fm.dim == 3 ? 8 : 4;
  pb->color_ptr.assign(1, 0);
  for (int color = 0; color < ncol; ++color) {
    for (int e = 0; e < Fm.ne; ++e) {
      const int ex = e % Fm.n[0], ey = (e / Fm.n[0]) % Fm.n[1], ez = e / (Fm.n[0] * Fm.n[1]);
      if ((ex & 1) + 2 * (ey & 1) + 4 * (ez & 1) == color) pb->color_elems.push_back(e);
    }
    pb->color_ptr.push_back((int32_t)pb->color_elems.size());
  }
  pb->tab = make_tab(Fm);
  return pb.release();
}

static fsi_csr view(const Csr &A) {
  fsi_csr c;
  c.nrows = A.nrows;
  c.ncols = A.ncols;
  c.nnz = (int64_t)A.ci.size();
  c.rowptr = A.rp.data();
  c.colind = A.ci.data();
  c.val = A.v.data();
  return c;
}

thread_local std::string last_msg;

}  // namespace fsib

using namespace fsib;

extern "C" {

fsi_status fsi_problem_build(const fsi_problem_spec *spec, struct fsi_problem **out) {
  if (!spec || !out) return FSI_E_INVALID;
  try {
    *out = reinterpret_cast<fsi_problem *>(build(*spec));
    return FSI_OK;
  } catch (const std::exception &e) {
    last_msg = e.what();
    *out = nullptr;
    return FSI_E_INVALID;
  }
}

const char *fsi_problem_last_error(void) { return last_msg.c_str(); }

int32_t fsi_problem_nlevels(const struct fsi_problem *p) {
  return p ? (int32_t)reinterpret_cast<const Problem *>(p)->meshes.size() : 0;
}

fsi_status fsi_problem_levels(const struct fsi_problem *hp, fsi_level *levels) {
  const Problem *p = reinterpret_cast<const Problem *>(hp);
  if (!p || !levels) return FSI_E_INVALID;
  for (size_t l = 0; l < p->meshes.size(); ++l) {
    fsi_level &L = levels[l];
    std::memset(&L, 0, sizeof L);
    L.J = view(p->J[l]);
    L.dirichlet = p->meshes[l].dir.data();
    if (l > 0) {
      L.P = view(p->P[l]);
      L.R = view(p->R[l]);
      const Patches &pt = p->patches[l];
      L.patches.npatch = (int32_t)pt.kind.size();
      L.patches.ptr = pt.ptr.data();
      L.patches.dof = pt.dof.data();
      L.patches.owned = pt.owned.data();
      L.patches.kind = pt.kind.data();
    }
  }
  return FSI_OK;
}

fsi_status fsi_problem_vectors(const struct fsi_problem *hp, const double **b, const double **y,
                               int64_t *n) {
  const Problem *p = reinterpret_cast<const Problem *>(hp);
  if (!p) return FSI_E_INVALID;
  if (b) *b = p->b.data();
  if (y) *y = p->y.data();
  if (n) *n = (int64_t)p->b.size();
  return FSI_OK;
}

fsi_status fsi_problem_dirichlet(const struct fsi_problem *hp, int32_t level, const uint8_t **flags) {
  const Problem *p = reinterpret_cast<const Problem *>(hp);
  if (!p || !flags || level < 0 || level >= (int32_t)p->meshes.size()) return FSI_E_INVALID;
  *flags = p->meshes[level].dir.data();
  return FSI_OK;
}

fsi_status fsi_problem_residual(const struct fsi_problem *hp, const double *y, double *r) {
  const Problem *p = reinterpret_cast<const Problem *>(hp);
  if (!p || !y || !r) return FSI_E_INVALID;
  const Mesh &M = p->meshes.back();
  std::vector<double> yy(y, y + M.ndof), rr;
  residual_jacobian(M, p->spec, yy, p->spec.transient ? &p->y_prev : nullptr, rr, nullptr);
  std::copy(rr.begin(), rr.end(), r);
  return FSI_OK;
}

fsi_status fsi_problem_element_data(const struct fsi_problem *hp, fsi_element_data *out) {
  const Problem *p = reinterpret_cast<const Problem *>(hp);
  if (!p || !out) return FSI_E_INVALID;
  const Mesh &M = p->meshes.back();
  fsi_element_data &d = *out;
  d.dim = M.dim;
  d.ne = M.ne;
  d.na = M.na;
  d.np = M.npe;
  d.nl = 2 * M.dim * M.na + M.npe;
  d.nq = p->tab.nq;
  d.ncolor = (int32_t)p->color_ptr.size() - 1;
  d.ndof = M.ndof;
  d.l2g = p->l2g.data();
  d.tgt = p->tgt.data();
  d.solid = M.solid.data();
  d.color_ptr = p->color_ptr.data();
  d.color_elems = p->color_elems.data();
  d.N = p->tab.N.data();
  d.dN = p->tab.dN.data();
  d.psi = p->tab.psi.data();
  d.w = p->tab.w.data();
  d.vol = p->tab.vol;
  d.dirichlet = M.dir.data();
  d.dval = M.dval.data();
  d.y_prev = p->spec.transient ? p->y_prev.data() : nullptr;
  d.mu = p->spec.mu;
  d.rho = p->spec.rho;
  d.mu_s = p->spec.mu_s;
  d.dt = p->spec.dt;
  d.rho_s = p->spec.rho_s;
  return FSI_OK;
}

fsi_status fsi_problem_destroy(struct fsi_problem *hp) {
  delete reinterpret_cast<Problem *>(hp);
  return FSI_OK;
}

}  // extern "C"
