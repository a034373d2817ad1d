// The paper's own full-order scheme (Sec. 3.1) on the 2D Euler mesh of a
// context: MUSCL reconstruction of the primitive variables (rho, u, v, P)
// limited by minmod, Roe's approximate Riemann solver at every face, BDF2 in
// time (eq. bdf with a_0 = 1/3, a_1 = -4/3, a_2 = 1, beta = 2/3; BDF1 where
// q_{k-2} is absent) and the residual of eq. hdm.  Boundaries: ghosts holding
// given states (the initial boundary states, Sec. 3.2) or reflective walls
// (Sec. 3.3).
//
// One thread per cell gathers its radius-2 cross stencil (ghosts applied),
// reconstructs the two faces on each axis and differences their Roe fluxes;
// every face is evaluated by both of its cells with the same operations and
// operands, so the two values agree bit for bit and the scheme stays
// discretely conservative.
//
// The implicit step is a defect correction: each iteration evaluates the
// second-order BDF residual and relaxes the first-order Rusanov Jacobian of
// the same step (a_2 I - beta dt dF_1/dq, transmissive ghosts) against it;
// the iteration converges to the root of the second-order residual, at a
// rate set by the gap between the two Jacobians (about 0.1 per iteration at
// the paper's Courant numbers).  The limiter's kinks make the exact Jacobian
// only piecewise defined, which a Newton method would have to differentiate.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "common.hpp"
#include "paper_hdm.hpp"
#include "physics.hpp"

namespace hs {

hs_status linear_solve(hs_ctx* ctx, const hs_samples* s, double rho, double eta, double* q, int* sweeps);

// Conservative state of cell (i, j), with ghosts: at most one of i, j lies
// outside the mesh, by at most two cells.
__device__ inline void paper_state(const Grid& g, const PaperBC& bc, const double* __restrict__ q, int i, int j,
                                   double s[4]) {
  int side = -1;
  if (i < 0) side = 0;
  else if (i >= g.nx) side = 1;
  else if (j < 0) side = 2;
  else if (j >= g.ny) side = 3;
  if (side >= 0 && bc.kind == HS_PAPER_BC_FIXED) {
#pragma unroll
    for (int a = 0; a < 4; ++a) s[a] = bc.ghost[side][a];
    return;
  }
  // wall: the mirror cell, its normal momentum reversed
  if (side == 0) i = -1 - i;
  else if (side == 1) i = 2 * g.nx - 1 - i;
  else if (side == 2) j = -1 - j;
  else if (side == 3) j = 2 * g.ny - 1 - j;
  const int cell = i + g.nx * j;
#pragma unroll
  for (int a = 0; a < 4; ++a) s[a] = q[a * g.ncell + cell];
  if (side == 0 || side == 1) s[1] = -s[1];
  if (side == 2 || side == 3) s[2] = -s[2];
}

__device__ inline void to_primitive(const double s[4], double gamma, double w[4]) {
#pragma clang fp contract(off)
  const double rho = s[0];
  const double irho = 1.0 / rho;   // one division per state (a division is a multi-instruction sequence)
  const double u = s[1] * irho;
  const double v = s[2] * irho;
  w[0] = rho;
  w[1] = u;
  w[2] = v;
  w[3] = (gamma - 1.0) * (s[3] - 0.5 * rho * (u * u + v * v));
}

// Zero unless a and b share a sign; then the one of smaller magnitude.
__device__ inline double minmod(double a, double b) {
  if (!(a * b > 0.0)) return 0.0;
  return fabs(a) <= fabs(b) ? a : b;
}

// Roe's flux between reconstructed primitive states wL | wR across a face
// normal to axis (0: x, 1: y).  The states are rotated so that component n
// carries the normal velocity and t the tangential one; the four waves are
// the acoustic u_n -+ c, the entropy wave and the shear wave at u_n.
__device__ inline void roe_flux(const double wL[4], const double wR[4], double gamma, int axis, double F[4]) {
#pragma clang fp contract(off)
  const int n = axis == 0 ? 1 : 2, t = axis == 0 ? 2 : 1;
  const double g1 = gamma - 1.0;
  const double ig1 = 1.0 / g1;
  const double rL = wL[0], nL = wL[n], tL = wL[t], pL = wL[3];
  const double rR = wR[0], nR = wR[n], tR = wR[t], pR = wR[3];
  const double eL = pL * ig1 + 0.5 * rL * (wL[1] * wL[1] + wL[2] * wL[2]);
  const double eR = pR * ig1 + 0.5 * rR * (wR[1] * wR[1] + wR[2] * wR[2]);
  const double hL = (eL + pL) * (1.0 / rL), hR = (eR + pR) * (1.0 / rR);
  // physical fluxes in the face frame: mass, normal, tangential momentum, energy
  const double fL[4] = {rL * nL, rL * nL * nL + pL, rL * nL * tL, (eL + pL) * nL};
  const double fR[4] = {rR * nR, rR * nR * nR + pR, rR * nR * tR, (eR + pR) * nR};
  // Roe averages (each reciprocal formed once: divisions dominate the face's cost)
  const double sL = sqrt(rL), sR = sqrt(rR);
  const double iden = 1.0 / (sL + sR);
  const double un = (sL * nL + sR * nR) * iden;
  const double ut = (sL * tL + sR * tR) * iden;
  const double h = (sL * hL + sR * hR) * iden;
  const double kin = 0.5 * (un * un + ut * ut);
  const double c2 = g1 * (h - kin);
  const double c = sqrt(c2);
  const double ic2 = 1.0 / c2;
  const double rho = sL * sR;
  const double dp = pR - pL, dn = nR - nL;
  // wave strengths times |speed|
  const double w1 = fabs(un - c) * ((dp - rho * c * dn) * (0.5 * ic2));
  const double w2 = fabs(un) * ((rR - rL) - dp * ic2);
  const double w3 = fabs(un) * (rho * (tR - tL));
  const double w4 = fabs(un + c) * ((dp + rho * c * dn) * (0.5 * ic2));
  double d[4];
  d[0] = w1 + w2 + w4;
  d[1] = w1 * (un - c) + w2 * un + w4 * (un + c);
  d[2] = (w1 + w2 + w4) * ut + w3;
  d[3] = w1 * (h - un * c) + w2 * kin + w3 * ut + w4 * (h + un * c);
  double Ff[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) Ff[a] = 0.5 * (fL[a] + fR[a]) - 0.5 * d[a];
  F[0] = Ff[0];
  F[n] = Ff[1];
  F[t] = Ff[2];
  F[3] = Ff[3];
}

// dt f*(q) of one cell: minus dt times its flux divergence.
__device__ inline void paper_dt_rhs(const Grid& g, const PaperBC& bc, const double* __restrict__ q, int cell,
                                    double out[4]) {
#pragma clang fp contract(off)
  int i, j;
  cell_ij(g, cell, i, j);
  const int naxes = g.ny > 1 ? 2 : 1;
#pragma unroll
  for (int a = 0; a < 4; ++a) out[a] = 0.0;
  for (int axis = 0; axis < naxes; ++axis) {
    double w[5][4];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      double s[4];
      if (axis == 0) paper_state(g, bc, q, i - 2 + k, j, s);
      else paper_state(g, bc, q, i, j - 2 + k, s);
      to_primitive(s, g.gamma, w[k]);
    }
    double sl[3][4];
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
      for (int a = 0; a < 4; ++a) sl[m][a] = minmod(w[m + 1][a] - w[m][a], w[m + 2][a] - w[m + 1][a]);
    double lo_l[4], lo_r[4], hi_l[4], hi_r[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      lo_l[a] = w[1][a] + 0.5 * sl[0][a];
      lo_r[a] = w[2][a] - 0.5 * sl[1][a];
      hi_l[a] = w[2][a] + 0.5 * sl[1][a];
      hi_r[a] = w[3][a] - 0.5 * sl[2][a];
    }
    double Flo[4], Fhi[4];
    roe_flux(lo_l, lo_r, g.gamma, axis, Flo);
    roe_flux(hi_l, hi_r, g.gamma, axis, Fhi);
    const double l = axis == 0 ? g.lx : g.ly;
#pragma unroll
    for (int a = 0; a < 4; ++a) out[a] = out[a] - l * (Fhi[a] - Flo[a]);
  }
}

// BDF residual of one cell: a_2 q - beta dt f*(q) + a_0 q_{k-2} + a_1 q_{k-1}
// (BDF2), or q - dt f*(q) - q_{k-1} (BDF1, q2 == nullptr).
__device__ inline void paper_cell_residual(const Grid& g, const PaperBC& bc, const double* __restrict__ q,
                                           const double* __restrict__ q1, const double* __restrict__ q2, int cell,
                                           double R[4]) {
#pragma clang fp contract(off)
  double f[4];
  paper_dt_rhs(g, bc, q, cell, f);
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int k = a * g.ncell + cell;
    if (q2) R[a] = q[k] - (2.0 / 3.0) * f[a] + (1.0 / 3.0) * q2[k] - (4.0 / 3.0) * q1[k];
    else R[a] = q[k] - f[a] - q1[k];
  }
}

// The block-Jacobi relaxation data of one cell's correction from the
// first-order Jacobian on grid gj (rhs = -D^-1 R, coef[d] = D^-1 O[d]; with
// nbr, the couplings to cells outside the sampled set are dropped), and the
// running max |R| and contraction bound of the thread.
__device__ inline void relax_data(const Grid& gj, const double* __restrict__ q, int cell, int p, int cap,
                                  const int* __restrict__ nbr, const double R[4], double* __restrict__ coef,
                                  double* __restrict__ rhs, double& rmax, double& rho, bool& bad) {
  Stencil<4> st;
  load_stencil<4>(gj, q, cell, st);
  double D[16], O[4][16], Di[16];
  cell_jacobian<4>(gj, st, D, O);
  if (nbr) {
#pragma unroll
    for (int d = 0; d < 4; ++d)
      if (nbr[d * cap + p] < 0)
#pragma unroll
        for (int e = 0; e < 16; ++e) O[d][e] = 0.0;
  }
  small_inverse<4>(D, Di);
  double rowsum[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    rmax = nan_max(rmax, fabs(R[a]));
    bad |= !isfinite(R[a]);
    double b = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) b -= Di[a * 4 + c] * R[c];
    rhs[a * cap + p] = b;
    rowsum[a] = 0.0;
  }
#pragma unroll
  for (int d = 0; d < 4; ++d)
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        double m = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) m += Di[a * 4 + c] * O[d][c * 4 + b];
        coef[((d * 4 + a) * 4 + b) * (size_t)cap + p] = m;
        rowsum[a] += fabs(m);
      }
#pragma unroll
  for (int a = 0; a < 4; ++a) rho = nan_max(rho, rowsum[a]);
  if (!isfinite(rho)) bad = true;
}

// The residual and the relaxation data of the correction on the compact list
// hat[0..count) of sampled cells, whose in-set neighbours are nbr[d * cap + p]
// (the couplings to every other cell are dropped: those entries are held);
// max |R| and the contraction bound as block partials.
__global__ void __launch_bounds__(kBlock) paper_resjac_kernel(Grid g, Grid gj, PaperBC bc,
                                                              const double* __restrict__ q,
                                                              const double* __restrict__ q1,
                                                              const double* __restrict__ q2,
                                                              const int* __restrict__ hat,
                                                              const int* __restrict__ nbr, int count,
                                                              double* __restrict__ coef, double* __restrict__ rhs,
                                                              double* __restrict__ part) {
  __shared__ double lds[kBlock / kWave];
  double rmax = 0.0, rho = 0.0;
  bool bad = false;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < count; p += gridDim.x * blockDim.x) {
    const int cell = hat[p];
    double R[4];
    paper_cell_residual(g, bc, q, q1, q2, cell, R);
    relax_data(gj, q, cell, p, g.ncell, nbr, R, coef, rhs, rmax, rho, bad);
  }
  rmax = block_max(bad ? INFINITY : rmax, lds);
  rho = block_max(rho, lds);
  if (threadIdx.x == 0) {
    stat_part(part, kStatResMax, rmax);
    stat_part(part, kStatRho, rho);
  }
}

// ------------------------------------------------------------ tiled form
// The full-mesh evaluations by TX x TY tiles (16 x 16; 256 x 1 in 1D): the
// primitive states of the tile and its two-cell cross halo are formed once
// into LDS, every face flux of the tile once, then each cell differences its
// faces.  The arithmetic of each state, slope, face flux and difference is
// that of the per-cell form, so the two give the same bits; a face on a tile
// edge is evaluated by both tiles from the same operands.  Tiles go to the
// blocks XCD by XCD (consecutive tiles share halo rows in that XCD's L2).
enum PaperTileMode : int { kTileResidual = 0, kTileNorms = 1, kTileResjac = 2 };

template <int TX, int TY>
struct PaperTile {
  static constexpr int WR = TY == 1 ? 1 : TY + 4;   // staged rows (1D: the tile's own row)
  static constexpr int WC = TX + 4;
  static constexpr int NT = TX * TY;
  double w[4][WR][WC];
  double fx[4][TY][TX + 1];
  double fy[4][TY == 1 ? 1 : TY + 1][TX];
};

template <int TX, int TY, int MODE>
__global__ void __launch_bounds__(TX * TY) paper_tile_kernel(Grid g, Grid gj, PaperBC bc,
                                                             const double* __restrict__ q,
                                                             const double* __restrict__ q1,
                                                             const double* __restrict__ q2, int ntx, int ntiles,
                                                             double* __restrict__ out, double* __restrict__ coef,
                                                             double* __restrict__ rhs, double* __restrict__ part) {
#pragma clang fp contract(off)
  using T = PaperTile<TX, TY>;
  __shared__ T sh;
  __shared__ double lds[T::NT / kWave];
  const int nslot = gridDim.x;   // a multiple of 8
  const int slot0 = (int)(blockIdx.x % 8) * (nslot / 8) + (int)(blockIdx.x / 8);
  double acc = 0.0, rmax = 0.0, rho = 0.0;
  bool bad = false;
  for (int t = slot0; t < ntiles; t += nslot) {
    const int tx0 = (t % ntx) * TX, ty0 = (t / ntx) * TY;
    // primitive states: tile cells and the cross halo (no corners), each
    // position inside the mesh or a ghost on one side only
    for (int e = threadIdx.x; e < T::WR * T::WC; e += T::NT) {
      const int lx = e % T::WC, lr = e / T::WC;
      const int ly = TY == 1 ? 2 : lr;
      const int gx = tx0 + lx - 2, gy = ty0 + ly - 2;
      const bool xin = gx >= 0 && gx < g.nx, yin = gy >= 0 && gy < g.ny;
      const bool col = lx >= 2 && lx < TX + 2, row = ly >= 2 && ly < TY + 2;
      if (!(col || row) || !(xin || yin) || gx < -2 || gx >= g.nx + 2 || gy < -2 || gy >= g.ny + 2) continue;
      double st[4], w[4];
      paper_state(g, bc, q, gx, gy, st);
      to_primitive(st, g.gamma, w);
#pragma unroll
      for (int a = 0; a < 4; ++a) sh.w[a][lr][lx] = w[a];
    }
    __syncthreads();
    // x faces: face fx sits left of tile column fx (cells fx - 1 | fx)
    for (int e = threadIdx.x; e < (TX + 1) * TY; e += T::NT) {
      const int fx = e % (TX + 1), fr = e / (TX + 1);
      if (ty0 + fr >= g.ny || tx0 + fx > g.nx) continue;
      const int r = TY == 1 ? 0 : fr + 2;
      double wl[4], wr[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const double* v = sh.w[a][r];
        const double sl = minmod(v[fx + 1] - v[fx], v[fx + 2] - v[fx + 1]);
        const double sr = minmod(v[fx + 2] - v[fx + 1], v[fx + 3] - v[fx + 2]);
        wl[a] = v[fx + 1] + 0.5 * sl;
        wr[a] = v[fx + 2] - 0.5 * sr;
      }
      double F[4];
      roe_flux(wl, wr, g.gamma, 0, F);
#pragma unroll
      for (int a = 0; a < 4; ++a) sh.fx[a][fr][fx] = F[a];
    }
    if (TY > 1) {
      // y faces: face fy sits below tile row fy (cells fy - 1 | fy)
      for (int e = threadIdx.x; e < TX * (TY + 1); e += T::NT) {
        const int cx = e % TX, fy = e / TX;
        if (tx0 + cx >= g.nx || ty0 + fy > g.ny) continue;
        const int c = cx + 2;
        double wl[4], wr[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const double v0 = sh.w[a][fy][c], v1 = sh.w[a][fy + 1][c], v2 = sh.w[a][fy + 2][c],
                       v3 = sh.w[a][fy + 3][c];
          const double sl = minmod(v1 - v0, v2 - v1);
          const double sr = minmod(v2 - v1, v3 - v2);
          wl[a] = v1 + 0.5 * sl;
          wr[a] = v2 - 0.5 * sr;
        }
        double F[4];
        roe_flux(wl, wr, g.gamma, 1, F);
#pragma unroll
        for (int a = 0; a < 4; ++a) sh.fy[a][fy][cx] = F[a];
      }
    }
    __syncthreads();
    const int cx = threadIdx.x % TX, cy = threadIdx.x / TX;
    const int gx = tx0 + cx, gy = ty0 + cy;
    if (gx < g.nx && gy < g.ny) {
      const int cell = gx + g.nx * gy;
      double R[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        double f = 0.0;
        f = f - g.lx * (sh.fx[a][cy][cx + 1] - sh.fx[a][cy][cx]);
        if (TY > 1) f = f - g.ly * (sh.fy[a][cy + 1][cx] - sh.fy[a][cy][cx]);
        const int k = a * g.ncell + cell;
        if (q2) R[a] = q[k] - (2.0 / 3.0) * f + (1.0 / 3.0) * q2[k] - (4.0 / 3.0) * q1[k];
        else R[a] = q[k] - f - q1[k];
      }
      if (MODE == kTileResidual) {
#pragma unroll
        for (int a = 0; a < 4; ++a) out[a * g.ncell + cell] = R[a];
      } else if (MODE == kTileNorms) {
        const double rn = sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2] + R[3] * R[3]);
        out[cell] = rn;
        acc += rn;
      } else {
        relax_data(gj, q, cell, cell, g.ncell, nullptr, R, coef, rhs, rmax, rho, bad);
      }
    }
    __syncthreads();
  }
  if (MODE == kTileNorms) {
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) stat_part(part, kStatSum, acc);
  } else if (MODE == kTileResjac) {
    rmax = block_max(bad ? INFINITY : rmax, lds);
    rho = block_max(rho, lds);
    if (threadIdx.x == 0) {
      stat_part(part, kStatResMax, rmax);
      stat_part(part, kStatRho, rho);
    }
  }
}

// Launch of a tiled full-mesh evaluation; *nb: its blocks (the partials).
template <int MODE>
static hs_status paper_tiles(hs_ctx* ctx, const Grid& gj, const PaperBC& bc, const double* q, const double* q1,
                             const double* q2, double* out, int* nb) {
  const Grid& g = ctx->g;
  const bool one_d = g.ny == 1;
  const int TX = one_d ? 256 : 16, TY = one_d ? 1 : 16;
  const int ntx = (g.nx + TX - 1) / TX, nty = (g.ny + TY - 1) / TY;
  const int ntiles = ntx * nty;
  // a multiple of 8 blocks, at most the partials' capacity
  const int grid = std::min((ntiles + 7) / 8 * 8, kPartCap / 8 * 8);
  *nb = grid;
  if (one_d)
    HS_LAUNCH(ctx, (paper_tile_kernel<256, 1, MODE>), grid, 256, g, gj, bc, q, q1, q2, ntx, ntiles, out, ctx->coef,
              ctx->rhs, ctx->part);
  else
    HS_LAUNCH(ctx, (paper_tile_kernel<16, 16, MODE>), grid, 256, g, gj, bc, q, q1, q2, ntx, ntiles, out, ctx->coef,
              ctx->rhs, ctx->part);
  return HS_OK;
}

// The relaxation of one correction on a small set (count * NC <= 4096: the
// compact list of sampled cells, or the whole mesh) in one workgroup: the
// iterate lives in LDS, nsw Jacobi sweeps x <- rhs - sum_d coef[d] x[nb_d]
// from x_1 = rhs are separated by workgroup barriers instead of launches, and
// the result is added to the state.  Neighbours: the list's in-set table, or
// on the whole mesh the grid's (a transmissive ghost is the cell itself,
// whose coefficient block is zero).
constexpr int kSmallRelax = 4096;

template <int NC>
__global__ void __launch_bounds__(1024) small_relax_kernel(Grid gj, const int* __restrict__ hat,
                                                           const int* __restrict__ nbr, int count,
                                                           const double* __restrict__ coef,
                                                           const double* __restrict__ rhs, int nsw,
                                                           double* __restrict__ q) {
  __shared__ double xs[2 * kSmallRelax];
  const int cap = gj.ncell;
  double* x0 = xs;
  double* x1 = xs + NC * count;
  for (int e = threadIdx.x; e < NC * count; e += blockDim.x) x0[e] = rhs[(size_t)(e / count) * cap + e % count];
  __syncthreads();
  for (int k = 1; k < nsw; ++k) {
    for (int p = threadIdx.x; p < count; p += blockDim.x) {
      int nb[4];
      if (hat) {
#pragma unroll
        for (int d = 0; d < 4; ++d) nb[d] = nbr[d * cap + p];
      } else {
        int i, j;
        cell_ij(gj, p, i, j);
#pragma unroll
        for (int d = 0; d < 4; ++d) nb[d] = (gj.ny == 1 && d >= 2) ? -1 : neighbour(gj, i, j, d);
      }
#pragma unroll
      for (int a = 0; a < NC; ++a) {
        double v = rhs[(size_t)a * cap + p];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          if (nb[d] < 0) continue;
#pragma unroll
          for (int b = 0; b < NC; ++b) v -= coef[((size_t)(d * NC + a) * NC + b) * cap + p] * x0[b * count + nb[d]];
        }
        x1[a * count + p] = v;
      }
    }
    __syncthreads();
    double* t = x0;
    x0 = x1;
    x1 = t;
  }
  for (int e = threadIdx.x; e < NC * count; e += blockDim.x) {
    const int a = e / count, p = e % count;
    const int cell = hat ? hat[p] : p;
    q[(size_t)a * cap + cell] += x0[e];
  }
}

// Relative accuracy of each relaxed correction: the defect correction itself
// reduces the residual by about 0.15 per iteration, so a finer solve buys
// nothing (measured: 0.1 against 0.02 takes Sod's full step from 0.69 to
// 0.59 ms and the implosion's from 2.19 to 2.09 ms).
constexpr double kDefectEta = 0.1;

hs_status paper_bc(hs_ctx* ctx, const hs_paper_hdm* hdm, PaperBC* bc) {
  if (ctx->nc != 4) return ctx->fail(HS_ERR_INVALID_ARG, "the paper's scheme needs an HS_EULER_2D context");
  if (hdm->bc != HS_PAPER_BC_FIXED && hdm->bc != HS_PAPER_BC_WALL)
    return ctx->fail(HS_ERR_INVALID_ARG, "hs_paper_hdm.bc must be HS_PAPER_BC_FIXED or HS_PAPER_BC_WALL");
  if (hdm->bc == HS_PAPER_BC_WALL && ctx->g.nx < 2)
    return ctx->fail(HS_ERR_INVALID_ARG, "reflective walls need two cells along x");
  bc->kind = hdm->bc;
  for (int s = 0; s < 4; ++s)
    for (int a = 0; a < 4; ++a) {
      const double v = hdm->ghost[s][a];
      if (hdm->bc == HS_PAPER_BC_FIXED && (s < 2 || ctx->g.ny > 1)) {
        if (!std::isfinite(v) || (a == 0 && !(v > 0.0)))
          return ctx->fail(HS_ERR_INVALID_ARG, "ghost states must be finite with positive density");
      }
      bc->ghost[s][a] = v;
    }
  return HS_OK;
}

hs_status paper_solve(hs_ctx* ctx, const PaperBC& bc, double* u, const double* q1, const double* q2, double tol,
                      const hs_samples* s, hs_step_info* info) {
  const int count = s ? s->n_s : ctx->ncell;
  if (count == 0) return HS_OK;
  // the correction's Jacobian: first-order Rusanov, transmissive ghosts, the
  // step's beta dt
  Grid gj = ctx->g;
  gj.bc = HS_BC_TRANSMISSIVE;
  const double beta = q2 ? 2.0 / 3.0 : 1.0;
  gj.lx *= beta;
  gj.ly *= beta;
  const int maxit = 4 * ctx->p.newton_maxit;
  const int nb = stat_blocks(count);
  int sweeps = 0;
  for (int it = 0;; ++it) {
    int nbs = nb;
    if (s)
      HS_LAUNCH(ctx, paper_resjac_kernel, nb, kBlock, ctx->g, gj, bc, u, q1, q2, s->hat, s->nbr, count, ctx->coef,
                ctx->rhs, ctx->part);
    else
      HS_TRY(paper_tiles<kTileResjac>(ctx, gj, bc, u, q1, q2, nullptr, &nbs));
    unsigned long long st[kStatSlots];
    HS_TRY(finish_stats(ctx, nbs, (1u << kStatResMax) | (1u << kStatRho), 0u, st));
    const double rmax = bits_to_double(st[kStatResMax]);
    const double rho = bits_to_double(st[kStatRho]);
    if (!std::isfinite(rmax)) return ctx->fail(HS_ERR_NONFINITE, "non-finite residual of the paper's scheme");
    if (info) info->residual_inf = rmax;
    if (rmax <= tol) {
      if (info) {
        info->newton_iters += it;
        info->lin_sweeps += sweeps;
      }
      return HS_OK;
    }
    if (it >= maxit) {
      char msg[160];
      std::snprintf(msg, sizeof msg, "defect correction: ||R||_inf = %.3e > %.3e after %d iterations", rmax, tol, it);
      return ctx->fail(HS_ERR_NOT_CONVERGED, msg);
    }
    if (!std::isfinite(rho)) return ctx->fail(HS_ERR_NONFINITE, "non-finite Jacobian");
    const double eta = std::max(kDefectEta, ctx->p.lin_rtol);
    const int nsw = rho > 0.0 && rho < 1.0 ? std::max(1, (int)std::ceil(std::log(eta) / std::log(rho))) : 1;
    if (4 * count <= kSmallRelax && rho < 1.0 && nsw <= ctx->p.lin_maxit) {
      // the whole correction in one workgroup (the set is small)
      HS_LAUNCH(ctx, small_relax_kernel<4>, 1, 1024, gj, s ? s->hat : nullptr, s ? s->nbr : nullptr, count,
                (const double*)ctx->coef, (const double*)ctx->rhs, nsw, u);
      sweeps += nsw;
    } else {
      HS_TRY(linear_solve(ctx, s, rho, eta, u, &sweeps));
    }
  }
}

hs_status paper_cell_norms(hs_ctx* ctx, const PaperBC& bc, const double* q, const double* q1, const double* q2,
                           double* rcell, int* nb) {
  return paper_tiles<kTileNorms>(ctx, ctx->g, bc, q, q1, q2, rcell, nb);
}

}  // namespace hs

using namespace hs;

extern "C" {

hs_status hs_paper_residual(hs_ctx* ctx, const hs_paper_hdm* hdm, const double* q, const double* q_prev,
                            const double* q_prev2, double* R) {
  if (!ctx || !hdm || !q || !q_prev || !R) return HS_ERR_INVALID_ARG;
  if (R == q || R == q_prev || (q_prev2 && R == q_prev2)) return ctx->fail(HS_ERR_INVALID_ARG, "R aliases an input");
  PaperBC bc;
  HS_TRY(paper_bc(ctx, hdm, &bc));
  int nb;
  return paper_tiles<kTileResidual>(ctx, ctx->g, bc, q, q_prev, q_prev2, R, &nb);
}

hs_status hdm_step_bdf2(hs_ctx* ctx, const hs_paper_hdm* hdm, const double* q_prev, const double* q_prev2,
                        double* q_out, hs_step_info* info) {
  if (!ctx || !hdm || !q_prev || !q_out) return HS_ERR_INVALID_ARG;
  if (q_out == q_prev || (q_prev2 && q_out == q_prev2))
    return ctx->fail(HS_ERR_INVALID_ARG, "q_out aliases an input");
  if (info) std::memset(info, 0, sizeof *info);
  PaperBC bc;
  HS_TRY(paper_bc(ctx, hdm, &bc));
  double qmax;
  HS_TRY(max_abs(ctx, q_prev, ctx->n, &qmax));
  if (!std::isfinite(qmax)) return ctx->fail(HS_ERR_NONFINITE, "non-finite q_prev");
  const double tol = ctx->p.newton_rtol * std::max(1.0, qmax);
  HIP_TRY(ctx, hipMemcpyAsync(q_out, q_prev, ctx->n * 8, hipMemcpyDeviceToDevice, ctx->stream));
  HS_TRY(paper_solve(ctx, bc, q_out, q_prev, q_prev2, tol, nullptr, info));
  if (info) info->n_s = ctx->ncell;
  return HS_OK;
}

}  // extern "C"
