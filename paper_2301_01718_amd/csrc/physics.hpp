// Rusanov fluxes and their exact derivatives (first-order finite volume).
//
// Burgers: f(u) = u^2/2, wave speed |u|.  Euler (Sec. 3.1, eq. euler):
// conservative (rho, rho u, rho v, E), p = (gamma - 1)(E - (rho u^2 + rho v^2)/2),
// wave speed |u_n| + c, c = sqrt(gamma p / rho).
// F(qL, qR) = (f(qL) + f(qR))/2 - alpha/2 (qR - qL), alpha = max(sL, sR),
// a tie sL = sR takes the left branch and |x| at x = 0 the + branch.
//
// The flux values are evaluated with contraction off and in a fixed operation
// order, so that the residual is reproducible bit for bit.
#pragma once

#include "common.hpp"

namespace hs {

// ------------------------------------------------------------------ Burgers
__device__ inline double burgers_flux(double uL, double uR) {
#pragma clang fp contract(off)
  const double aL = uL >= 0.0 ? uL : -uL;
  const double aR = uR >= 0.0 ? uR : -uR;
  const double a = aL >= aR ? aL : aR;
  return 0.25 * (uL * uL + uR * uR) - (0.5 * a) * (uR - uL);
}

// dF/duL and dF/duR.
__device__ inline void burgers_flux_d(double uL, double uR, double& dL, double& dR) {
  const double aL = uL >= 0.0 ? uL : -uL;
  const double aR = uR >= 0.0 ? uR : -uR;
  const bool left = aL >= aR;
  const double a = left ? aL : aR;
  const double daL = left ? (uL >= 0.0 ? 1.0 : -1.0) : 0.0;
  const double daR = left ? 0.0 : (uR >= 0.0 ? 1.0 : -1.0);
  const double jump = uR - uL;
  dL = 0.5 * uL + 0.5 * a - 0.5 * daL * jump;
  dR = 0.5 * uR - 0.5 * a - 0.5 * daR * jump;
}

// -------------------------------------------------------------------- Euler
struct EulerPhys {
  double f[4];
  double un, c;
};

// Physical flux along x (normal = 0) or y (normal = 1).
__device__ inline EulerPhys euler_phys(const double q[4], double gamma, int normal) {
#pragma clang fp contract(off)
  EulerPhys r;
  const double rho = q[0], mx = q[1], my = q[2], en = q[3];
  const double u = mx / rho;
  const double v = my / rho;
  const double p = (gamma - 1.0) * (en - 0.5 * (mx * u + my * v));
  r.c = sqrt(gamma * p / rho);
  if (normal == 0) {
    r.un = u;
    r.f[0] = mx;
    r.f[1] = mx * u + p;
    r.f[2] = my * u;
    r.f[3] = (en + p) * u;
  } else {
    r.un = v;
    r.f[0] = my;
    r.f[1] = mx * v;
    r.f[2] = my * v + p;
    r.f[3] = (en + p) * v;
  }
  return r;
}

__device__ inline void euler_flux(const double qL[4], const double qR[4], double gamma, int normal,
                                  double F[4]) {
#pragma clang fp contract(off)
  const EulerPhys L = euler_phys(qL, gamma, normal);
  const EulerPhys R = euler_phys(qR, gamma, normal);
  const double sL = (L.un >= 0.0 ? L.un : -L.un) + L.c;
  const double sR = (R.un >= 0.0 ? R.un : -R.un) + R.c;
  const double a = sL >= sR ? sL : sR;
#pragma unroll
  for (int k = 0; k < 4; ++k) F[k] = 0.5 * (L.f[k] + R.f[k]) - (0.5 * a) * (qR[k] - qL[k]);
}

// Flux Jacobian A = df/dq (row-major 4x4) and the gradient of the wave speed
// s = |u_n| + c with respect to q.
__device__ inline void euler_jac(const double q[4], double gamma, int normal, double A[16],
                                 double ds[4], double& s) {
  const double rho = q[0], mx = q[1], my = q[2], en = q[3];
  const double u = mx / rho, v = my / rho;
  const double g1 = gamma - 1.0;
  const double k = 0.5 * (u * u + v * v);
  const double p = g1 * (en - 0.5 * (mx * u + my * v));
  const double c = sqrt(gamma * p / rho);
  const double H = (en + p) / rho;
  const double un = normal == 0 ? u : v;
  if (normal == 0) {
    const double r[16] = {0.0, 1.0, 0.0, 0.0,
                          g1 * k - u * u, (3.0 - gamma) * u, -g1 * v, g1,
                          -u * v, v, u, 0.0,
                          u * (g1 * k - H), H - g1 * u * u, -g1 * u * v, gamma * u};
#pragma unroll
    for (int i = 0; i < 16; ++i) A[i] = r[i];
  } else {
    const double r[16] = {0.0, 0.0, 1.0, 0.0,
                          -u * v, v, u, 0.0,
                          g1 * k - v * v, -g1 * u, (3.0 - gamma) * v, g1,
                          v * (g1 * k - H), -g1 * u * v, H - g1 * v * v, gamma * v};
#pragma unroll
    for (int i = 0; i < 16; ++i) A[i] = r[i];
  }
  const double sg = un >= 0.0 ? 1.0 : -1.0;
  const double cf = gamma / (2.0 * c * rho);
  double dc[4] = {cf * (g1 * k - p / rho), cf * (-g1 * u), cf * (-g1 * v), cf * g1};
  double dun[4] = {-un / rho, 0.0, 0.0, 0.0};
  dun[normal == 0 ? 1 : 2] = 1.0 / rho;
#pragma unroll
  for (int i = 0; i < 4; ++i) ds[i] = sg * dun[i] + dc[i];
  s = (un >= 0.0 ? un : -un) + c;
}

// dF/dqL and dF/dqR (row-major 4x4 each) of the Rusanov flux.
__device__ inline void euler_flux_d(const double qL[4], const double qR[4], double gamma, int normal,
                                    double DL[16], double DR[16]) {
  double AL[16], AR[16], dsL[4], dsR[4], sL, sR;
  euler_jac(qL, gamma, normal, AL, dsL, sL);
  euler_jac(qR, gamma, normal, AR, dsR, sR);
  const bool left = sL >= sR;
  const double a = left ? sL : sR;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double jump = qR[r] - qL[r];
#pragma unroll
    for (int col = 0; col < 4; ++col) {
      const double daL = left ? dsL[col] : 0.0;
      const double daR = left ? 0.0 : dsR[col];
      const double id = r == col ? 1.0 : 0.0;
      DL[r * 4 + col] = 0.5 * AL[r * 4 + col] + 0.5 * a * id - 0.5 * jump * daL;
      DR[r * 4 + col] = 0.5 * AR[r * 4 + col] - 0.5 * a * id - 0.5 * jump * daR;
    }
  }
}

// ---------------------------------------------------------- per-cell stencil
// Gathers the state of a cell and its four face neighbours (ghosts applied)
// from a full-size, component-major vector.
template <int NC>
struct Stencil {
  double c[NC];
  double nb[4][NC];
  int idx[4];   // neighbour cell, the cell itself (extrapolation ghost) or -1 (inflow ghost)
  int self;
};

template <int NC>
__device__ inline void load_stencil(const Grid& g, const double* __restrict__ q, int cell,
                                    Stencil<NC>& st) {
  int i, j;
  cell_ij(g, cell, i, j);
  const int ndir = g.kind == HS_BURGERS_1D ? 2 : 4;
  st.self = cell;
#pragma unroll
  for (int a = 0; a < NC; ++a) st.c[a] = q[a * g.ncell + cell];
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    if (d >= ndir) {
      st.idx[d] = cell;
#pragma unroll
      for (int a = 0; a < NC; ++a) st.nb[d][a] = st.c[a];
      continue;
    }
    const int nb = neighbour(g, i, j, d);
    st.idx[d] = nb;
#pragma unroll
    for (int a = 0; a < NC; ++a) st.nb[d][a] = nb < 0 ? g.inflow : q[a * g.ncell + nb];
  }
}

// Residual of one cell: R = (q - q_prev) + lx (F_E - F_W) [+ ly (F_N - F_S)].
template <int NC>
__device__ inline void cell_residual(const Grid& g, const Stencil<NC>& st, const double* qp,
                                     double R[NC]) {
#pragma clang fp contract(off)
  if constexpr (NC == 1) {
    const double fw = burgers_flux(st.nb[0][0], st.c[0]);
    const double fe = burgers_flux(st.c[0], st.nb[1][0]);
    double r = (st.c[0] - qp[0]) + g.lx * (fe - fw);
    if (g.kind != HS_BURGERS_1D) {
      const double fs = burgers_flux(st.nb[2][0], st.c[0]);
      const double fn = burgers_flux(st.c[0], st.nb[3][0]);
      r = r + g.ly * (fn - fs);
    }
    R[0] = r;
  } else {
    double fw[4], fe[4], fs[4], fn[4];
    euler_flux(st.nb[0], st.c, g.gamma, 0, fw);
    euler_flux(st.c, st.nb[1], g.gamma, 0, fe);
    euler_flux(st.nb[2], st.c, g.gamma, 1, fs);
    euler_flux(st.c, st.nb[3], g.gamma, 1, fn);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      double r = (st.c[a] - qp[a]) + g.lx * (fe[a] - fw[a]);
      R[a] = r + g.ly * (fn[a] - fs[a]);
    }
  }
}

// Residual plus the Jacobian row of one cell: D (NC x NC, row-major) and the
// four neighbour blocks O[d].  Derivatives with respect to a ghost that copies
// the cell are folded into D; those with respect to the inflow constant are
// dropped, and O[d] is then zero.
template <int NC>
__device__ inline void cell_jacobian(const Grid& g, const Stencil<NC>& st, double D[NC * NC],
                                     double O[4][NC * NC]) {
  const int ndir = g.kind == HS_BURGERS_1D ? 2 : 4;
#pragma unroll
  for (int e = 0; e < NC * NC; ++e) {
    D[e] = (e % (NC + 1) == 0) ? 1.0 : 0.0;
#pragma unroll
    for (int d = 0; d < 4; ++d) O[d][e] = 0.0;
  }
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    if (d >= ndir) continue;
    const double lam = d < 2 ? g.lx : g.ly;
    // face between (left, right); the cell is the right state for W/S, left for E/N
    const bool cell_is_left = (d == 1 || d == 3);
    const double sign = cell_is_left ? 1.0 : -1.0;   // + lam F_E, - lam F_W
    double Dc[NC * NC], Dn[NC * NC];                  // d/d(cell state), d/d(neighbour state)
    if constexpr (NC == 1) {
      double dL, dR;
      if (cell_is_left) {
        burgers_flux_d(st.c[0], st.nb[d][0], dL, dR);
        Dc[0] = dL; Dn[0] = dR;
      } else {
        burgers_flux_d(st.nb[d][0], st.c[0], dL, dR);
        Dc[0] = dR; Dn[0] = dL;
      }
    } else {
      const int normal = d < 2 ? 0 : 1;
      if (cell_is_left) euler_flux_d(st.c, st.nb[d], g.gamma, normal, Dc, Dn);
      else euler_flux_d(st.nb[d], st.c, g.gamma, normal, Dn, Dc);
    }
    const bool fold = st.idx[d] == st.self;       // ghost copies the cell
#pragma unroll
    for (int e = 0; e < NC * NC; ++e) {
      D[e] += sign * lam * Dc[e];
      const double on = sign * lam * Dn[e];
      if (st.idx[d] < 0) continue;                 // inflow constant
      if (fold) D[e] += on;
      else O[d][e] += on;
    }
  }
}

// Inverse of a small row-major NC x NC matrix (NC = 4: adjugate; otherwise
// Gauss-Jordan with partial pivoting).
template <int NC>
__device__ inline void small_inverse(const double A[NC * NC], double X[NC * NC]) {
  if constexpr (NC == 1) {
    X[0] = 1.0 / A[0];
  } else if constexpr (NC == 4) {
    // adjugate / determinant, the cofactors from complementary 2 x 2 minors of
    // the top and bottom row pairs (Laplace expansion): static indexing, so
    // the block stays in registers (the blocks inverted here are the
    // diagonally dominated Newton-Jacobian blocks; the relaxation only needs
    // an accurate inverse, the converged Newton state does not depend on it)
    const double a00 = A[0], a01 = A[1], a02 = A[2], a03 = A[3], a10 = A[4], a11 = A[5], a12 = A[6], a13 = A[7];
    const double a20 = A[8], a21 = A[9], a22 = A[10], a23 = A[11], a30 = A[12], a31 = A[13], a32 = A[14],
                 a33 = A[15];
    const double s0 = a00 * a11 - a10 * a01, s1 = a00 * a12 - a10 * a02, s2 = a00 * a13 - a10 * a03;
    const double s3 = a01 * a12 - a11 * a02, s4 = a01 * a13 - a11 * a03, s5 = a02 * a13 - a12 * a03;
    const double c5 = a22 * a33 - a32 * a23, c4 = a21 * a33 - a31 * a23, c3 = a21 * a32 - a31 * a22;
    const double c2 = a20 * a33 - a30 * a23, c1 = a20 * a32 - a30 * a22, c0 = a20 * a31 - a30 * a21;
    const double inv = 1.0 / (s0 * c5 - s1 * c4 + s2 * c3 + s3 * c2 - s4 * c1 + s5 * c0);
    X[0] = (a11 * c5 - a12 * c4 + a13 * c3) * inv;
    X[1] = (-a01 * c5 + a02 * c4 - a03 * c3) * inv;
    X[2] = (a31 * s5 - a32 * s4 + a33 * s3) * inv;
    X[3] = (-a21 * s5 + a22 * s4 - a23 * s3) * inv;
    X[4] = (-a10 * c5 + a12 * c2 - a13 * c1) * inv;
    X[5] = (a00 * c5 - a02 * c2 + a03 * c1) * inv;
    X[6] = (-a30 * s5 + a32 * s2 - a33 * s1) * inv;
    X[7] = (a20 * s5 - a22 * s2 + a23 * s1) * inv;
    X[8] = (a10 * c4 - a11 * c2 + a13 * c0) * inv;
    X[9] = (-a00 * c4 + a01 * c2 - a03 * c0) * inv;
    X[10] = (a30 * s4 - a31 * s2 + a33 * s0) * inv;
    X[11] = (-a20 * s4 + a21 * s2 - a23 * s0) * inv;
    X[12] = (-a10 * c3 + a11 * c1 - a12 * c0) * inv;
    X[13] = (a00 * c3 - a01 * c1 + a02 * c0) * inv;
    X[14] = (-a30 * s3 + a31 * s1 - a32 * s0) * inv;
    X[15] = (a20 * s3 - a21 * s1 + a22 * s0) * inv;
  } else {
    double M[NC][2 * NC];
#pragma unroll
    for (int r = 0; r < NC; ++r)
#pragma unroll
      for (int c = 0; c < 2 * NC; ++c) M[r][c] = c < NC ? A[r * NC + c] : (c - NC == r ? 1.0 : 0.0);
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      int piv = k;
      double best = fabs(M[k][k]);
#pragma unroll
      for (int r = k + 1; r < NC; ++r)
        if (fabs(M[r][k]) > best) { best = fabs(M[r][k]); piv = r; }
#pragma unroll
      for (int c = 0; c < 2 * NC; ++c) {   // swap rows k and piv
        const double t = M[k][c];
        M[k][c] = M[piv][c];
        M[piv][c] = t;
      }
      const double inv = 1.0 / M[k][k];
#pragma unroll
      for (int c = 0; c < 2 * NC; ++c) M[k][c] *= inv;
#pragma unroll
      for (int r = 0; r < NC; ++r) {
        if (r == k) continue;
        const double f = M[r][k];
#pragma unroll
        for (int c = 0; c < 2 * NC; ++c) M[r][c] -= f * M[k][c];
      }
    }
#pragma unroll
    for (int r = 0; r < NC; ++r)
#pragma unroll
      for (int c = 0; c < NC; ++c) X[r * NC + c] = M[r][NC + c];
  }
}

}  // namespace hs
