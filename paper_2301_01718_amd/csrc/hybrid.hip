// Hybrid snapshot step (eq. hybrid; the hybrid branch of Alg. 1):
//   A6  gappy-POD fit on the sampled rows with a truncated pseudo-inverse
//       (eq. red_coord with the fit rows = hat-S), and the subiterations of
//       Sec. 2.3.2 between the restricted Newton solve and the fit;
//   A7  reconstruction psi + Phi y of the unsampled entries (eq. rom_approx);
//   A8  residual-gated Shapiro filters (Sec. 2.3.4);
//   A4  reconstruction-error indicator of the filtered snapshot (Sec. 2.3.3).
//
// The fit factorises the gathered Gram matrix Phi_S^T Phi_S (FP64 MFMA) once
// per step: a Jacobi eigendecomposition gives the truncated pseudo-inverse
// G+ (singular values of Phi_S below rcond_fit * sigma_max dropped).  Every
// subiteration then costs two passes over the gathered rows: y0 = G+ Phi_S^T d
// and one refinement step y = y0 + G+ Phi_S^T (d - Phi_S y0).  The Gram's
// eigenvalues carry about eps lambda_max of absolute error, so the cut is
// never placed below kFitEigFloor lambda_max (sigma ratio 1.2e-7): a gathered
// basis more ill-conditioned than that has no resolvable trailing directions
// in the Gram, and the step reports its condition number (the fits of the
// workloads measure kappa <= 1e3).
constexpr double kFitEigFloor = 64 * 2.220446049250313e-16;
#include "dense.hpp"
#include "paper_hdm.hpp"
#include "physics.hpp"

#include <algorithm>
#include <cstring>
#include <mutex>

namespace hs {

// Gathered rows of Phi at the dofs of hat-S cells (all components): thread
// (r, q) holds row r and columns q, q + 4, ... of the chunk.
template <typename TP>
struct GatherLoader {
  const TP* Phi;
  long long n;
  int m, nc, ncell, ns;
  const int* hat;
  struct Regs {
    double v[kMaxBasis / 4];
  };
  __device__ void init(Regs&) const {}
  __device__ void prefetch(long long row0, Regs& R) const {
    const int r = threadIdx.x % kChunk;
    const long long row = row0 + r;
    long long dof = -1;
    if (row < (long long)nc * ns) {
      const int a = (int)(row / ns), p = (int)(row % ns);
      dof = (long long)a * ncell + hat[p];
      if (dof >= n) dof = -1;   // a caller's fit point outside the state: no row
    }
#pragma unroll
    for (int i = 0; i < kMaxBasis / 4; ++i) {
      const int j = threadIdx.x / kChunk + 4 * i;
      R.v[i] = (dof >= 0 && j < m) ? (double)Phi[(size_t)j * n + dof] : 0.0;
    }
  }
  __device__ void commit(long long, const Regs& R, double* X, int ldx, int wp) const {
    const int r = threadIdx.x % kChunk;
#pragma unroll
    for (int i = 0; i < kMaxBasis / 4; ++i) {
      const int j = threadIdx.x / kChunk + 4 * i;
      if (j < wp) X[r * ldx + j] = R.v[i];
    }
  }
};

// The Cholesky route of the pseudo-inverse is taken while its bound on
// lambda_max / lambda_min of the Gram stays below this (kappa(Phi_S) < 1e3):
// the inverse is then good to kappa^2 eps = 1e-10 and the fit's refinement
// step removes that; more ill-conditioned fits take the eigen route.
constexpr double kCholMaxRatio = 1e6;

// For a well-conditioned Gram the truncated pseudo-inverse is the inverse:
// G = L L^T (Cholesky), G^-1 = L^-T L^-1.  Taken when the Cholesky succeeds
// and ||G||_F ||G^-1||_F (an upper bound on lambda_max / lambda_min) stays
// below 1 / cut, so that no eigenvalue can lie under the cut.  Returns false
// (nothing written) otherwise.  Every thread of the block calls it.
__device__ bool pinv_by_cholesky(const double* A, double* L, double* Li, int lda, int m, double cut,
                                 double* __restrict__ Gp, double* __restrict__ misc,
                                 unsigned long long* __restrict__ stats) {
#pragma clang fp contract(off)
  __shared__ int bad;
  __shared__ double lds[256 / kWave];
  const int t = threadIdx.x, nt = blockDim.x;
  if (t == 0) bad = 0;
  __syncthreads();
  for (int k = 0; k < m; ++k) {
    // every thread forms l_kk from the same sums (same bits), then its entry
    double dk = A[k * lda + k];
    for (int j = 0; j < k; ++j) dk -= L[k * lda + j] * L[k * lda + j];
    const double lkk = sqrt(dk);
    for (int i = k + t; i < m; i += nt) {
      if (i == k) {
        L[k * lda + k] = lkk;
        if (!(dk > 0.0)) bad = 1;
      } else {
        double sacc = A[i * lda + k];
        for (int j = 0; j < k; ++j) sacc -= L[i * lda + j] * L[k * lda + j];
        L[i * lda + k] = sacc / lkk;
      }
    }
    __syncthreads();
    if (bad) return false;
  }
  // L^-1, one column per thread (forward substitution)
  if (t < m) {
    const int c = t;
    Li[c * lda + c] = 1.0 / L[c * lda + c];
    for (int i = c + 1; i < m; ++i) {
      double sacc = 0.0;
      for (int k = c; k < i; ++k) sacc += L[i * lda + k] * Li[k * lda + c];
      Li[i * lda + c] = -sacc / L[i * lda + i];
    }
  }
  __syncthreads();
  // G^-1 = L^-T L^-1 (into L's upper part is not needed: straight to Gp) and
  // the Frobenius norms of G and G^-1
  double fa = 0.0, fi = 0.0;
  for (int e = t; e < m * m; e += nt) {
    const int r = e / m, c = e % m;
    double sacc = 0.0;
    for (int k = r > c ? r : c; k < m; ++k) sacc += Li[k * lda + r] * Li[k * lda + c];
    Gp[e] = sacc;
    fi += sacc * sacc;
    fa += A[r * lda + c] * A[r * lda + c];
  }
  fa = block_sum(fa, lds);
  fi = block_sum(fi, lds);
  __shared__ int ok;
  if (t == 0) {
    const double kb = sqrt(fa) * sqrt(fi);     // >= lambda_max / lambda_min
    ok = kb * cut < 1.0 && kb < kCholMaxRatio;
    if (ok) {
      misc[1] = m;
      misc[2] = sqrt(kb);                      // >= kappa(Phi_S)
      stats[kStatFitRank] = dbits((double)m);
      stats[kStatFitCond] = dbits(misc[2]);
    }
  }
  __syncthreads();
  return ok != 0;
}

// Truncated pseudo-inverse of the m x m Gram: G+ = sum_{kept} v v^T / lambda
// (or the inverse, when a Cholesky shows that nothing is cut).
__global__ void __launch_bounds__(256) pinv_kernel(const double* __restrict__ G, int m, double rcond,
                                                  double* __restrict__ Gp, double* __restrict__ misc,
                                                  unsigned long long* __restrict__ stats, int use_chol) {
#pragma clang fp contract(off)
  __shared__ double A[kMaxBasis * (kMaxBasis + 1)], V[kMaxBasis * (kMaxBasis + 1)];
  __shared__ double lam[kMaxBasis];
  __shared__ int order[kMaxBasis];
  __shared__ int rank;
  const int lda = kMaxBasis + 1;
  const int t = threadIdx.x;
  for (int e = t; e < m * m; e += blockDim.x) A[(e / m) * lda + e % m] = G[e];
  __syncthreads();
  {
    __shared__ double Li[kMaxBasis * (kMaxBasis + 1)];
    // (m <= 8 keeps the eigen route: pinv_small_kernel computes the same
    // pseudo-inverse in registers and is checked against this one)
    if (use_chol && m > 8 && pinv_by_cholesky(A, V, Li, lda, m, fmax(rcond * rcond, kFitEigFloor), Gp, misc, stats))
      return;
  }
  jacobi_eig_wave(A, V, lda, m, lam, order, 40);
  if (t == 0) {
    int k = 0;
    const double lmax = lam[0];
    const double cut = fmax(rcond * rcond, kFitEigFloor) * lmax;
    for (int i = 0; i < m; ++i)
      if (lmax > 0.0 && lam[i] > cut) k = i + 1;
    rank = k;
    misc[1] = k;
    misc[2] = k > 0 ? sqrt(lmax / lam[k - 1]) : 0.0;
    stats[kStatFitRank] = dbits((double)k);
    stats[kStatFitCond] = dbits(misc[2]);
  }
  __syncthreads();
  for (int e = t; e < m * m; e += blockDim.x) {
    const int r = e / m, c = e % m;
    double s = 0.0;
    for (int i = 0; i < rank; ++i) s += V[r * lda + order[i]] * V[c * lda + order[i]] / lam[i];
    Gp[e] = s;
  }
}

// The same truncated pseudo-inverse for m <= 8 in one wave with the matrix in
// registers: lane 8 i + j holds A[i][j] and V[i][j].  Each round every lane
// fetches the entries of its row pair and of its 2 x 2 block by cross-lane
// reads, forms the row pair's rotation, reads its column pair's from lane
// (j, j) and updates its own entry, so a round has no LDS round trip and no
// barrier.  Schedule, thresholds, rotation formulas and
// update order are those of jacobi_eig_wave, so the result is the same to the
// bit (both round every product and sum on its own).  Launch: one block of
// 64 threads.
__device__ inline int rr_partner(int x, int r, int np) {   // 0 <= r < np - 1
  const int np1 = np - 1;
  if (x >= np) return x;
  if (x == np1) return r;
  int y = 2 * r - x;
  if (y < 0) y += np1;
  if (y >= np1) y -= np1;
  return y == x ? np1 : y;
}

__global__ void __launch_bounds__(64) pinv_small_kernel(const double* __restrict__ G, int m, double rcond,
                                                       double* __restrict__ Gp, double* __restrict__ misc,
                                                       unsigned long long* __restrict__ stats) {
#pragma clang fp contract(off)
  constexpr int D = 8;
  __shared__ double Vs[D * (D + 1)];
  __shared__ double lam[D];
  __shared__ int order[D];
  const int l = threadIdx.x, i = l / D, j = l % D;
  const bool in = i < m && j < m;
  double a = in ? G[i * m + j] : 0.0;
  double v = (in && i == j) ? 1.0 : 0.0;
  // atol = eps * sum_i |a_ii| in index order, the same in every lane
  double tr = 0.0;
  for (int k = 0; k < m; ++k) tr += fabs(__shfl(a, k * D + k, kWave));
  const double atol = 2.2e-16 * tr;
  const int np = (m + 1) & ~1;
  const double nt2 = (double)m * 2.2e-16;
  for (int sweep = 0; sweep < 40; ++sweep) {
    int big = 0;
    for (int r = 0; r < np - 1; ++r) {
      const int pi = rr_partner(i, r, np), pj = rr_partner(j, r, np);
      const int rp = min(i, pi), rq = max(i, pi), cp = min(j, pj), cq = max(j, pj);
      // entries of the row pair and of this lane's 2 x 2 block (padding lanes
      // hold zeros; the indices are < 8)
      const double app = __shfl(a, rp * D + rp, kWave), aqq = __shfl(a, rq * D + rq, kWave);
      const double apq = __shfl(a, rp * D + rq, kWave);
      const double a00 = __shfl(a, rp * D + cp, kWave), a01 = __shfl(a, rp * D + cq, kWave);
      const double a10 = __shfl(a, rq * D + cp, kWave), a11 = __shfl(a, rq * D + cq, kWave);
      const double vo = __shfl(v, i * D + (j == cp ? cq : cp), kWave);
      // rotation of the row pair (c = 1, s = 0 if none); lane (j, j) holds the
      // one of this lane's column pair
      double ck = 1.0, sk = 0.0;
      if (rq < m) {
        const double lim2 = fabs(app) * fabs(aqq);
        const double apq2 = apq * apq;
        if (fabs(apq) > atol && apq2 > (2.2e-16 * 2.2e-16) * lim2) {
          const double d = 0.5 * (aqq - app);
          const double tt = (d >= 0.0 ? apq : -apq) / (fabs(d) + sqrt(d * d + apq2));
          ck = rsqrt(1.0 + tt * tt);
          sk = tt * ck;
          if (apq2 > nt2 * nt2 * lim2) big = 1;
        }
      }
      const double cl = __shfl(ck, j * D + j, kWave), sl = __shfl(sk, j * D + j, kWave);
      const bool rqv = rq < m, cqv = cq < m;
      const double x01 = cqv ? a01 : 0.0, x10 = rqv ? a10 : 0.0, x11 = (rqv && cqv) ? a11 : 0.0;
      // rows, then columns (the order of jacobi_eig_wave)
      const double b00 = ck * a00 - sk * x10, b01 = ck * x01 - sk * x11;
      const double b10 = sk * a00 + ck * x10, b11 = sk * x01 + ck * x11;
      if (i == rp) a = j == cp ? cl * b00 - sl * b01 : sl * b00 + cl * b01;
      else a = j == cp ? cl * b10 - sl * b11 : sl * b10 + cl * b11;
      if (sl != 0.0) v = j == cp ? cl * v - sl * vo : sl * vo + cl * v;
      if (!in) a = 0.0, v = 0.0;
    }
    if (!__any(big)) break;
  }
  if (in) Vs[i * (D + 1) + j] = v;
  // stable descending order of the diagonal (cross-lane reads by all lanes)
  const int ld = min(l, D - 1);
  const double li = __shfl(a, ld * D + ld, kWave);
  int rk = 0;
  for (int k = 0; k < m; ++k) {
    const double lk = __shfl(a, k * D + k, kWave);
    rk += (lk > li) || (lk == li && k < l);
  }
  if (l < m) {
    lam[rk] = li;
    order[rk] = l;
  }
  __syncthreads();
  int rank = 0;
  const double lmax = lam[0];
  const double cut = fmax(rcond * rcond, kFitEigFloor) * lmax;
  for (int k = 0; k < m; ++k)
    if (lmax > 0.0 && lam[k] > cut) rank = k + 1;
  if (l == 0) {
    misc[1] = rank;
    misc[2] = rank > 0 ? sqrt(lmax / lam[rank - 1]) : 0.0;
    stats[kStatFitRank] = dbits((double)rank);
    stats[kStatFitCond] = dbits(misc[2]);
  }
  if (in) {
    double s = 0.0;
    for (int k = 0; k < rank; ++k) s += Vs[i * (D + 1) + order[k]] * Vs[j * (D + 1) + order[k]] / lam[k];
    Gp[i * m + j] = s;
  }
}

// Partial projections Phi_rows^T d over rows (gathered if hat != nullptr):
// mode 0: d = u - psi; mode 1: d = u - psi - Phi_row y0.
template <int MP, typename TP>
__global__ void __launch_bounds__(256) project_kernel(const TP* __restrict__ Phi, long long n, int m,
                                                      int nc, int ncell, const int* __restrict__ hat, int ns,
                                                      const double* __restrict__ u, const double* __restrict__ psi,
                                                      const double* __restrict__ y0, int mode,
                                                      double* __restrict__ part) {
  __shared__ double yl[MP];
  __shared__ double wsum[4][MP];
  for (int j = threadIdx.x; j < MP; j += blockDim.x) yl[j] = (mode == 1 && j < m) ? y0[j] : 0.0;
  __syncthreads();
  double acc[MP];
#pragma unroll
  for (int j = 0; j < MP; ++j) acc[j] = 0.0;
  const long long rows = hat ? (long long)nc * ns : n;
  for (long long row = blockIdx.x * (long long)blockDim.x + threadIdx.x; row < rows;
       row += (long long)gridDim.x * blockDim.x) {
    long long dof = row;
    if (hat) dof = (row / ns) * (long long)ncell + hat[row % ns];
    if (dof < 0 || dof >= n) continue;   // a caller's fit point outside the state: no row
    double ph[MP];
#pragma unroll
    for (int j = 0; j < MP; ++j) ph[j] = j < m ? (double)Phi[(size_t)j * n + dof] : 0.0;
    double d = u[dof] - psi[dof];
    if (mode == 1) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < MP; ++j) s += ph[j] * yl[j];
      d -= s;
    }
#pragma unroll
    for (int j = 0; j < MP; ++j) acc[j] += ph[j] * d;
  }
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
#pragma unroll
  for (int j = 0; j < MP; ++j) {
    const double v = wave_sum(acc[j]);
    if (lane == 0) wsum[wave][j] = v;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < m; j += blockDim.x)
    part[(size_t)blockIdx.x * MP + j] = ((wsum[0][j] + wsum[1][j]) + wsum[2][j]) + wsum[3][j];
}

// Reduce the projection partials and apply the pseudo-inverse.  Wave v sums
// the partials of coefficients v, v + 4, ... (lanes stride the blocks in a
// fixed order, then a fixed shuffle tree).
// mode 0: y0 = G+ b.  mode 1: y = y0 + G+ b, ||y - y_prev|| to misc[0], y_prev = y.
__global__ void __launch_bounds__(256) project_finish_kernel(const double* __restrict__ part, int nb, int mp,
                                                             int m, const double* __restrict__ Gp, int mode,
                                                             double* __restrict__ y0, double* __restrict__ y,
                                                             double* __restrict__ yprev, double* __restrict__ misc,
                                                             int first, unsigned long long* __restrict__ stats) {
  __shared__ double b[kMaxBasis], ynew[kMaxBasis];
  const int t = threadIdx.x;
  const int lane = t % kWave, wave = t / kWave, nw = blockDim.x / kWave;
  for (int j = wave; j < m; j += nw) {
    double s = 0.0;
    for (int k = lane; k < nb; k += kWave) s += part[(size_t)k * mp + j];
    s = wave_sum(s);
    if (lane == 0) b[j] = s;
  }
  __syncthreads();
  if (t < m) {
    double s = 0.0;
    for (int c = 0; c < m; ++c) s += Gp[t * m + c] * b[c];
    if (mode == 0) y0[t] = s;
    else ynew[t] = y0[t] + s;
  }
  __syncthreads();
  if (mode == 1 && t == 0) {
    double d2 = 0.0;
    for (int i = 0; i < m; ++i) {
      const double d = ynew[i] - yprev[i];
      d2 += d * d;
    }
    misc[0] = first ? INFINITY : sqrt(d2);
    if (stats) stats[kStatDy] = dbits(misc[0]);
  }
  __syncthreads();
  if (mode == 1 && t < m) {
    y[t] = ynew[t];
    yprev[t] = ynew[t];
  }
}

// u <- psi + Phi y on the dofs of the listed cells.
template <typename TP>
__global__ void ring_update_kernel(const TP* __restrict__ Phi, long long n, int m, int nc, int ncell,
                                   const int* __restrict__ cells, int nl, const double* __restrict__ psi,
                                   const double* __restrict__ y, double* __restrict__ u) {
  __shared__ double yl[kMaxBasis];
  if (threadIdx.x < m) yl[threadIdx.x] = y[threadIdx.x];
  __syncthreads();
  const long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (k >= (long long)nc * nl) return;
  const long long dof = (k / nl) * (long long)ncell + cells[k % nl];
  double s = 0.0;
  for (int j = 0; j < m; ++j) s += (double)Phi[(size_t)j * n + dof] * yl[j];
  u[dof] = psi[dof] + s;
}

// rho_r = psi_r + sum_j Phi_rj y_j (the one expression every kernel that
// reconstructs uses, so that they agree to the bit).
template <typename TP>
__device__ inline double recon_value(const TP* __restrict__ Phi, long long n, int m, const double* __restrict__ psi,
                                     const double* yl, long long r) {
  double s = 0.0;
  for (int j = 0; j < m; ++j) s += (double)Phi[(size_t)j * n + r] * yl[j];
  return psi[r] + s;
}

// rho = psi + Phi y everywhere; gamma = u on hat-S cells, rho elsewhere.
// With mask == nullptr only rho is written.
template <typename TP>
__global__ void recon_kernel(const TP* __restrict__ Phi, long long n, int m, int ncell,
                             const double* __restrict__ psi, const double* __restrict__ y,
                             const uint8_t* __restrict__ mask, const double* __restrict__ u,
                             double* __restrict__ gamma, double* __restrict__ rho) {
  __shared__ double yl[kMaxBasis];
  if (threadIdx.x < m) yl[threadIdx.x] = y[threadIdx.x];
  __syncthreads();
  const long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (r >= n) return;
  const double rr = recon_value(Phi, n, m, psi, yl, r);
  rho[r] = rr;
  if (mask) gamma[r] = mask[r % ncell] ? u[r] : rr;
}

__global__ void eye_kernel(double* __restrict__ A, int m) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < m * m) A[e] = (e / m == e % m) ? 1.0 : 0.0;
}

// max_abs_partials (hdm.hip): per-block maxima of |x| in slot kStatQMax.
hs_status max_abs_partials(hs_ctx* ctx, const double* x, long long n, int* nb);

// max |gamma| of every workgroup alike, from the nbq partials of
// max_abs_partials (a maximum is exact in any order).
__device__ inline double block_qmax(const double* __restrict__ qpart, int nbq) {
  __shared__ double lds[kBlock / kWave];
  __shared__ double qmax;
  double qm = 0.0;
  for (int b = threadIdx.x; b < nbq; b += blockDim.x) qm = nan_max(qm, qpart[kStatQMax * kPartCap + b]);
  qm = block_max(qm, lds);
  if (threadIdx.x == 0) qmax = qm;
  __syncthreads();
  return qmax;
}

// The cell's error sum_c d_c^2 (d_c = gamma - rho of component c), flushed to
// 0 below floor2.
__device__ inline double cell_error(double e, double floor2) { return e < floor2 ? 0.0 : e; }
__device__ inline double add_square(double e, double d, int a) {
#pragma clang fp contract(off)
  return a == 0 ? d * d : e + d * d;
}

// eps_cell = sum_c (gamma - rho)^2, flushed to 0 below fl^2 with
// fl = floor_rel * max(1, max |gamma|).
__global__ void indicator_kernel(int ncell, int nc, const double* __restrict__ gamma,
                                 const double* __restrict__ rho, double floor_rel,
                                 const double* __restrict__ qpart, int nbq, double* __restrict__ eps) {
#pragma clang fp contract(off)
  const double qmax = block_qmax(qpart, nbq);
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  const double fl = floor_rel * fmax(1.0, qmax);
  const double floor2 = fl * fl;
  double e = 0.0;
  for (int a = 0; a < nc; ++a) e = add_square(e, gamma[(size_t)a * ncell + c] - rho[(size_t)a * ncell + c], a);
  eps[c] = cell_error(e, floor2);
}

// The same indicator with rho = psi + Phi y formed in place (no rho buffer).
template <typename TP>
__global__ void indicator_direct_kernel(int ncell, int nc, const double* __restrict__ gamma, const TP* __restrict__ Phi,
                                        const double* __restrict__ psi, const double* __restrict__ y, int m,
                                        double floor_rel, const double* __restrict__ qpart, int nbq,
                                        double* __restrict__ eps) {
#pragma clang fp contract(off)
  __shared__ double yl[kMaxBasis];
  if (threadIdx.x < m) yl[threadIdx.x] = y[threadIdx.x];
  const double qmax = block_qmax(qpart, nbq);   // its barrier also publishes yl
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  const long long n = (long long)nc * ncell;
  const double fl = floor_rel * fmax(1.0, qmax);
  const double floor2 = fl * fl;
  double e = 0.0;
  for (int a = 0; a < nc; ++a) {
    const long long r = (long long)a * ncell + c;
    e = add_square(e, gamma[r] - recon_value(Phi, n, m, psi, yl, r), a);
  }
  eps[c] = cell_error(e, floor2);
}

// ----------------------------------------------------------------- filter
// S_n = I - (-delta^2/4)^n at one point, from the 2n+1 values load(-n..n)
// along one axis (centre load(0)): n nested second differences
// -(a - 2b + c)/4, subtracted from the centre.  Every filter kernel goes
// through this function, so the arithmetic is the same everywhere.
template <int N, typename Load>
__device__ inline double shapiro_point(Load load) {
#pragma clang fp contract(off)
  double v[2 * N + 1];
#pragma unroll
  for (int s = -N; s <= N; ++s) v[s + N] = load(s);
  const double centre = v[N];
#pragma unroll
  for (int lev = 0; lev < N; ++lev)
#pragma unroll
    for (int s = 0; s + 2 < 2 * (N - lev) + 1; ++s) v[s] = -(v[s] - 2.0 * v[s + 1] + v[s + 2]) / 4.0;
  return centre - v[0];
}

template <typename Load>
__device__ inline double shapiro_any(int nord, Load load) {
  if (nord == 1) return shapiro_point<1>(load);
  if (nord == 2) return shapiro_point<2>(load);
  return shapiro_point<3>(load);
}

// out = S_n in along one axis (periodic wrap or repetition of the boundary value).
__global__ void shapiro_kernel(Grid g, const double* __restrict__ in, double* __restrict__ out, int axis,
                               int nord) {
  const long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (k >= (long long)g.nc * g.ncell) return;
  const int a = (int)(k / g.ncell), cell = (int)(k % g.ncell);
  int i, j;
  cell_ij(g, cell, i, j);
  const int len = axis == 0 ? g.nx : g.ny;
  const int x0 = axis == 0 ? i : j;
  const bool per = g.bc == HS_BC_PERIODIC;
  const double* src = in + (size_t)a * g.ncell;
  out[k] = shapiro_any(nord, [&](int s) {
    int x = x0 + s;
    if (per) x = wrap_index(x, len);
    else x = x < 0 ? 0 : (x >= len ? len - 1 : x);
    return src[axis == 0 ? x + g.nx * j : i + g.nx * x];
  });
}

// rcell = cellwise 2-norm of R(q); block partial sums of rcell to part.
template <int NC>
__global__ void cellres_kernel(Grid g, const double* __restrict__ q, const double* __restrict__ qp,
                               double* __restrict__ rcell, double* __restrict__ part) {
#pragma clang fp contract(off)
  __shared__ double lds[kBlock / kWave];
  const int cell = blockIdx.x * blockDim.x + threadIdx.x;
  double rn = 0.0;
  if (cell < g.ncell) {
    Stencil<NC> st;
    load_stencil<NC>(g, q, cell, st);
    double p[NC], R[NC];
#pragma unroll
    for (int a = 0; a < NC; ++a) p[a] = qp[a * g.ncell + cell];
    cell_residual<NC>(g, st, p, R);
    double s = R[0] * R[0];
#pragma unroll
    for (int a = 1; a < NC; ++a) s = s + R[a] * R[a];
    rn = sqrt(s);
    rcell[cell] = rn;
  }
  const double bs = block_sum(rn, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = bs;
}

__global__ void sum_finish_kernel(const double* __restrict__ part, int nb, double* __restrict__ out) {
  __shared__ double lds[kBlock / kWave];
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) s += part[b];
  s = block_sum(s, lds);
  if (threadIdx.x == 0) *out = s;
}

// Replay of a recorded pass: merged = mask ? gf : cur.
__global__ void mask_blend_kernel(long long n, int ncell, const double* __restrict__ cur,
                                  const double* __restrict__ gf, const uint8_t* __restrict__ mask,
                                  double* __restrict__ merged) {
  const long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (r >= n) return;
  merged[r] = mask[r % ncell] ? gf[r] : cur[r];
}

// ------------------------------------------------------ fused filter pass
// One pass of the residual-gated filter (Sec. 2.3.4) per TX x TY tile, with
// the state read once from HBM instead of once per stage:
//   A  the current state on the tile + an H = n_max + 2 halo (staged in LDS);
//   B  S_x A on the tile + a 2-cell ring of columns, all staged rows;
//   G  S_y B on the tile + a 2-cell ring (1D: G = B);
//   M  the gate on the tile + a 1-cell ring: G where the cell residual norm of
//      G is below r (the norm of the current state), else A;
//   r2 the cell residual norm of M on the tile.
// The filter differences are nested in the order of shapiro_kernel and the
// residual is cell_residual on the same values, so G, the decisions, M and
// r2 are bit-identical to the unfused passes; ring cells are recomputed by
// the neighbouring tiles with the same arithmetic.  Out-of-domain positions
// of a non-periodic grid hold the clamped state (the filter's boundary
// repetition); the residual stencils follow the ghost rules of neighbour().
// Per block: the kept count and the sum of r2 go to the statistics partials.
constexpr int kFiltHalo = 5;

template <int NC, int TX, int TY>
struct FiltCfg {
  static constexpr bool ONE_D = TY == 1;
  static constexpr int H = kFiltHalo;
  static constexpr int AW = TX + 2 * H, AH = ONE_D ? 1 : TY + 2 * H;
  static constexpr int BW = TX + 4, BH = AH;
  static constexpr int GW = TX + 4, GH = ONE_D ? 1 : TY + 4;
  static constexpr int MW = TX + 2, MH = ONE_D ? 1 : TY + 2;
};

__device__ inline int wrap_or_clamp(int u, int len, bool per) {
  if (per) return wrap_index(u, len);
  return u < 0 ? 0 : (u >= len ? len - 1 : u);
}

// Stencil of the cell at unwrapped position (ux, uy) (inside the domain, or
// any position on a periodic grid) from an LDS array arr[a * stride + pos]
// whose position (0, 0) is the unwrapped point (ox, oy), row width w.
template <int NC>
__device__ inline void lds_stencil(const Grid& g, const double* arr, int stride, int ox, int oy, int w, int ux,
                                   int uy, Stencil<NC>& st) {
  const bool per = g.bc == HS_BC_PERIODIC;
  const int ndir = g.kind == HS_BURGERS_1D ? 2 : 4;
  const int pc = (uy - oy) * w + (ux - ox);
#pragma unroll
  for (int a = 0; a < NC; ++a) st.c[a] = arr[a * stride + pc];
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    if (d >= ndir) {
#pragma unroll
      for (int a = 0; a < NC; ++a) st.nb[d][a] = st.c[a];
      continue;
    }
    const int vx = ux + (d == 0 ? -1 : (d == 1 ? 1 : 0));
    const int vy = uy + (d == 2 ? -1 : (d == 3 ? 1 : 0));
    const bool inside = per || (vx >= 0 && vx < g.nx && vy >= 0 && vy < g.ny);
    if (inside) {
      const int pn = (vy - oy) * w + (vx - ox);
#pragma unroll
      for (int a = 0; a < NC; ++a) st.nb[d][a] = arr[a * stride + pn];
    } else {
      const bool inflow = neighbour(g, ux, uy, d) < 0;
#pragma unroll
      for (int a = 0; a < NC; ++a) st.nb[d][a] = inflow ? g.inflow : st.c[a];
    }
  }
}

// Device state of the filter loop (orders o, passes within an order it): the
// finisher of each pass advances it exactly as the host loop would, so the
// next pass can be enqueued before the host has read the decision.
struct FiltCtl {
  int o, it, parity, done, passes, kept;   // parity 1: the current state is in the spare buffer
  double sum_r;                            // l1 sum of the current state's residual norms
};

// The gate kernel's view of that state (ctl == nullptr: a host-driven pass).
// Device-driven pass k reads the state of pass k - 1 from ctl[(k - 1) & 1],
// advances it with that pass's kept count and residual sum (reduced from its
// partials by every workgroup alike) and stores it to ctl[k & 1]; workgroup 0
// posts the record of pass k - 1.  Pass 0 runs the initial state ctl[0].
struct FiltSpec {
  FiltCtl* ctl = nullptr;
  double* state[2] = {nullptr, nullptr};   // gamma, spare
  double* norms[2] = {nullptr, nullptr};   // r, r2
  int orders[4] = {0, 0, 0, 0};
  int pass = 0, nb = 0;                    // k; partial count of every pass
  int first = 1;                           // host-driven pass: the first of its order (every tile computed)
  int n_orders = 0, jfmax = 0;
  double eps_f = 0.0;
  unsigned long long* stats = nullptr;     // kStatCount / kStatSum of pass k - 1
  PostSlot post{};                         // the record of pass k - 1 (k >= 1)
};

// Partial slots of device pass k (alternating, so pass k + 1 reads them while
// writing its own).
__host__ __device__ inline int filt_count_slot(int k) { return (k & 1) ? kStatFiltCount1 : kStatCount; }
__host__ __device__ inline int filt_sum_slot(int k) { return (k & 1) ? kStatFiltSum1 : kStatSum; }

// One step of the filter loop after a pass that kept `kept` cells and left
// the l1 residual sum `sum`, as the host loop takes it (no cell kept: next
// order; else swap the buffers, and stop the order when the relative
// decrease falls below eps_f or after jfmax passes).
__device__ inline FiltCtl filt_advance(FiltCtl c, long long kept, double sum, int n_orders, int jfmax,
                                       double eps_f) {
#pragma clang fp contract(off)
  c.passes += 1;
  c.kept += (int)kept;
  if (kept == 0) {
    c.o += 1;
    c.it = 0;
  } else {
    c.parity ^= 1;
    const double dec = (c.sum_r - sum) / c.sum_r;
    c.sum_r = sum;
    c.it += 1;
    if (dec < eps_f || c.it >= jfmax) {
      c.o += 1;
      c.it = 0;
    }
  }
  if (c.o >= n_orders) c.done = 1;
  return c;
}

template <int NC, int TX, int TY>
__global__ void __launch_bounds__(kBlock) filter_gate_kernel(
    Grid g, int ntx, int ntiles, int nord, const double* __restrict__ cur, const double* __restrict__ qp,
    const double* __restrict__ r, double* __restrict__ merged, double* __restrict__ r2,
    uint8_t* __restrict__ keep_out, double* __restrict__ part, const FiltSpec fs) {
#pragma clang fp contract(off)
  using C = FiltCfg<NC, TX, TY>;
  constexpr bool ONE_D = C::ONE_D;
  constexpr int H = C::H, AW = C::AW, AH = C::AH, BW = C::BW, BH = C::BH, GW = C::GW, GH = C::GH;
  constexpr int MW = C::MW, MH = C::MH;
  constexpr int RA = AW * AH, RB = BW * BH, RG = GW * GH, RM = MW * MH;
  static_assert(ONE_D || RM <= RB, "the gate's merged state reuses the S_x buffer");
  __shared__ double sA[NC * RA];
  __shared__ double sB[NC * RB];
  __shared__ double sG[ONE_D ? 1 : NC * RG];
  __shared__ double sM1[ONE_D ? NC * RM : 1];
  __shared__ uint8_t sK[RM];
  __shared__ double lds[kBlock / kWave];
  double* G = ONE_D ? sB : sG;
  const int gstride = ONE_D ? RB : RG;
  double* M = ONE_D ? sM1 : sB;
  const bool per = g.bc == HS_BC_PERIODIC;
  double rsum = 0.0;
  int kept = 0;
  // Partial slots alternate with the pass index, so that a pass reads the
  // per-tile results of the previous one while writing its own.
  int pass = fs.pass;
  int cslot = filt_count_slot(pass), sslot = filt_sum_slot(pass);
  bool all = fs.first != 0;
  if (fs.ctl != nullptr) {
    // the pass the device state asks for, or none once the loop is done
    const int k = fs.pass;
    FiltCtl c = fs.ctl[k == 0 ? 0 : (k - 1) & 1];
    if (k > 0) {
      // pass k - 1's kept count and residual sum: the same strided order and
      // tree in every workgroup (and as finish_stats reduces them)
      __shared__ unsigned long long rec[8];
      const FiltCtl c0 = c;
      double cnt = 0.0, sum = 0.0;
      if (!c0.done) {
        const int cs = filt_count_slot(k - 1), ss = filt_sum_slot(k - 1);
        for (int b = threadIdx.x; b < fs.nb; b += blockDim.x) {
          cnt = cnt + part[cs * kPartCap + b];
          sum = sum + part[ss * kPartCap + b];
        }
        cnt = block_sum(cnt, lds);
        sum = block_sum(sum, lds);
        __shared__ double bc[2];   // thread 0's results to the workgroup
        if (threadIdx.x == 0) {
          bc[0] = cnt;
          bc[1] = sum;
        }
        __syncthreads();
        cnt = bc[0];
        sum = bc[1];
        c = filt_advance(c0, (long long)cnt, sum, fs.n_orders, fs.jfmax, fs.eps_f);
      }
      if (blockIdx.x == 0) {
        if (threadIdx.x == 0) {
          fs.ctl[k & 1] = c;
          const bool ran = !c0.done;
          if (ran) {
            fs.stats[kStatCount] = dbits(cnt);
            fs.stats[kStatSum] = dbits(sum);
          }
          rec[0] = ran ? (unsigned long long)(long long)cnt : 0ull;
          rec[1] = ran ? dbits(sum) : 0ull;
          rec[2] = (unsigned long long)c.done;
          rec[3] = (unsigned long long)c.parity;
          rec[4] = (unsigned long long)c.passes;
          rec[5] = (unsigned long long)c.kept;
          rec[6] = ran ? 1ull : 0ull;
        }
        __syncthreads();
        if (threadIdx.x < kWave) post_words(reinterpret_cast<const uint32_t*>(rec), 14, fs.post.dst, fs.post.tagp,
                                            fs.post.tag);
      }
    }
    if (c.done) return;
    cslot = filt_count_slot(k);
    sslot = filt_sum_slot(k);
    all = k == 0 || c.it == 0;
    nord = fs.orders[c.o];
    cur = fs.state[c.parity];
    merged = fs.state[c.parity ^ 1];
    r = fs.norms[c.parity];
    r2 = fs.norms[c.parity ^ 1];
  }

  // Within an order, pass k can change a cell (its state, its gate decision
  // or its residual norm) only if a cell within the halo H changed in pass
  // k - 1, and H is less than a tile: pass k computes only the tiles next to
  // (or being) a tile that kept a cell in pass k - 1.  Every other tile is
  // unchanged in both state and norm buffers (by induction over the passes;
  // the first pass of an order computes every tile) and carries its
  // residual-sum partial forward, the sum of the same values in the same
  // order.  One tile per workgroup is needed for the per-tile partials.
  const bool track = !all && (int)gridDim.x == ntiles;
  bool carried = false;
  double carry_sum = 0.0;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int X0 = (tile % ntx) * TX, Y0 = ONE_D ? 0 : (tile / ntx) * TY;
    if (track) {
      // thread i < 9 reads neighbour tile i's kept count of pass k - 1
      int hit = 0;
      if (threadIdx.x < (ONE_D ? 3 : 9)) {
        const int tx = tile % ntx, ty = tile / ntx, nty = ntiles / ntx;
        int ux = tx + (int)(threadIdx.x % 3) - 1, uy = ONE_D ? 0 : ty + (int)(threadIdx.x / 3) - 1;
        if (per) {
          ux = (ux + ntx) % ntx;
          uy = (uy + nty) % nty;
        }
        if (ux >= 0 && ux < ntx && uy >= 0 && uy < nty)
          hit = part[filt_count_slot(pass - 1) * kPartCap + uy * ntx + ux] > 0.0;
      }
      if (!__syncthreads_or(hit)) {
        carried = true;
        carry_sum = part[filt_sum_slot(pass - 1) * kPartCap + tile];
        if (keep_out) {
          for (int p = threadIdx.x; p < TX * TY; p += kBlock) {
            const int ux = X0 + p % TX, uy = Y0 + p / TX;
            if (ux < g.nx && uy < g.ny) keep_out[ux + g.nx * uy] = 0;
          }
        }
        continue;
      }
    }
    // A: the current state, wrapped or clamped
    for (int p = threadIdx.x; p < RA; p += kBlock) {
      const int ax = p % AW, ay = p / AW;
      const int x = wrap_or_clamp(X0 - H + ax, g.nx, per);
      const int y = ONE_D ? 0 : wrap_or_clamp(Y0 - H + ay, g.ny, per);
#pragma unroll
      for (int a = 0; a < NC; ++a) sA[a * RA + p] = cur[(size_t)a * g.ncell + x + (size_t)g.nx * y];
    }
    __syncthreads();
    // B = S_x A (columns X0-2 .. X0+TX+1)
    for (int p = threadIdx.x; p < RB; p += kBlock) {
      const int bx = p % BW, by = p / BW;
      const int c0 = by * AW + bx + H - 2;
#pragma unroll
      for (int a = 0; a < NC; ++a) {
        const double* src = sA + a * RA + c0;
        sB[a * RB + p] = shapiro_any(nord, [&](int s) { return src[s]; });
      }
    }
    __syncthreads();
    if constexpr (!ONE_D) {
      // G = S_y B (rows Y0-2 .. Y0+TY+1)
      for (int p = threadIdx.x; p < RG; p += kBlock) {
        const int gx = p % GW, gy = p / GW;
        const int c0 = (gy + H - 2) * BW + gx;
#pragma unroll
        for (int a = 0; a < NC; ++a) {
          const double* src = sB + a * RB + c0;
          sG[a * RG + p] = shapiro_any(nord, [&](int s) { return src[s * BW]; });
        }
      }
      __syncthreads();
    }
    // gate on the tile + 1 ring
    for (int p = threadIdx.x; p < RM; p += kBlock) {
      const int mx = p % MW, my = p / MW;
      const int ux = X0 - 1 + mx, uy = ONE_D ? 0 : Y0 - 1 + my;
      uint8_t keep = 0;
      if (per || (ux >= 0 && ux < g.nx && uy >= 0 && uy < g.ny)) {
        const int cell = wrap_or_clamp(ux, g.nx, per) + g.nx * (ONE_D ? 0 : wrap_or_clamp(uy, g.ny, per));
        Stencil<NC> st;
        lds_stencil<NC>(g, G, gstride, X0 - 2, ONE_D ? 0 : Y0 - 2, GW, ux, uy, st);
        double pv[NC], R[NC];
#pragma unroll
        for (int a = 0; a < NC; ++a) pv[a] = qp[(size_t)a * g.ncell + cell];
        cell_residual<NC>(g, st, pv, R);
        double s = R[0] * R[0];
#pragma unroll
        for (int a = 1; a < NC; ++a) s = s + R[a] * R[a];
        keep = sqrt(s) < r[cell];
        const int pa = (uy - (ONE_D ? 0 : Y0 - H)) * AW + (ux - (X0 - H));
#pragma unroll
        for (int a = 0; a < NC; ++a) M[a * RM + p] = keep ? st.c[a] : sA[a * RA + pa];
      }
      sK[p] = keep;
    }
    __syncthreads();
    // the merged state, its residual norm and the decisions on the tile
    for (int p = threadIdx.x; p < TX * TY; p += kBlock) {
      const int lx = p % TX, ly = p / TX;
      const int ux = X0 + lx, uy = Y0 + ly;
      if (ux >= g.nx || uy >= g.ny) continue;
      const int cell = ux + g.nx * uy;
      Stencil<NC> st;
      lds_stencil<NC>(g, M, RM, X0 - 1, ONE_D ? 0 : Y0 - 1, MW, ux, uy, st);
      double pv[NC], R[NC];
#pragma unroll
      for (int a = 0; a < NC; ++a) pv[a] = qp[(size_t)a * g.ncell + cell];
      cell_residual<NC>(g, st, pv, R);
      double s = R[0] * R[0];
#pragma unroll
      for (int a = 1; a < NC; ++a) s = s + R[a] * R[a];
      const double rn = sqrt(s);
      r2[cell] = rn;
      rsum += rn;
#pragma unroll
      for (int a = 0; a < NC; ++a) merged[(size_t)a * g.ncell + cell] = st.c[a];
      const uint8_t keep = sK[(ONE_D ? 0 : (ly + 1) * MW) + lx + 1];
      if (keep_out) keep_out[cell] = keep;
      kept += keep;
    }
    __syncthreads();
  }
  if (carried) {
    if (threadIdx.x == 0) {
      stat_part(part, sslot, carry_sum);
      stat_part(part, cslot, 0.0);
    }
    return;
  }
  const double bs = block_sum(rsum, lds);
  const int bk = block_sum_int(kept, reinterpret_cast<int*>(lds));
  if (threadIdx.x == 0) {
    stat_part(part, sslot, bs);
    stat_part(part, cslot, (double)bk);
  }
}

// Initial state of the device-driven filter loop (one workgroup of kBlock):
// the l1 sum of the input state's residual norms reduced from the nb block
// partials of cellres_kernel as sum_finish_kernel reduces them (same order,
// same tree), also stored to the statistics slot kStatSum0.
__global__ void filt_init_kernel(FiltCtl* ctl, const double* __restrict__ part, int nb,
                                 unsigned long long* __restrict__ stats, int done) {
  __shared__ double lds[kBlock / kWave];
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) s += part[b];
  s = block_sum(s, lds);
  if (threadIdx.x == 0) {
    stats[kStatSum0] = dbits(s);
    FiltCtl c;
    c.o = 0;
    c.it = 0;
    c.parity = 0;
    c.done = done;
    c.passes = 0;
    c.kept = 0;
    c.sum_r = s;
    *ctl = c;
  }
}

// Tile of the fused filter pass (must match the instantiations in filter_pass).
static void filter_tile(const hs_ctx* ctx, int* tx, int* ty) {
  if (ctx->g.kind == HS_BURGERS_1D) { *tx = 512; *ty = 1; }
  else if (ctx->nc == 1) { *tx = 32; *ty = 32; }
  else { *tx = 16; *ty = 16; }
}

// One gated pass: merged (the next state), r2, keep_out; kept count and sum
// of r2 to the statistics slots kStatCount / kStatSum (enqueued only).
static hs_status filter_gate_launch(hs_ctx* ctx, const double* cur, const double* q_prev, const double* r, int nord,
                                    double* merged, double* r2, uint8_t* keep_out, const FiltSpec& fs, int* nb_out) {
  int tx, ty;
  filter_tile(ctx, &tx, &ty);
  const int ntx = (ctx->g.nx + tx - 1) / tx;
  const int ntiles = ntx * ((ctx->g.ny + ty - 1) / ty);
  const int nb = std::min(ntiles, kPartCap);
  FiltSpec f = fs;
  f.nb = nb;   // every pass of a grid has the same partial count
  HS_TRY(prof_begin(ctx, HS_PROF_FILTER));
  if (ctx->g.kind == HS_BURGERS_1D)
    HS_LAUNCH(ctx, (filter_gate_kernel<1, 512, 1>), nb, kBlock, ctx->g, ntx, ntiles, nord, cur, q_prev, r, merged,
              r2, keep_out, ctx->part, f);
  else if (ctx->nc == 1)
    HS_LAUNCH(ctx, (filter_gate_kernel<1, 32, 32>), nb, kBlock, ctx->g, ntx, ntiles, nord, cur, q_prev, r, merged,
              r2, keep_out, ctx->part, f);
  else
    HS_LAUNCH(ctx, (filter_gate_kernel<4, 16, 16>), nb, kBlock, ctx->g, ntx, ntiles, nord, cur, q_prev, r, merged,
              r2, keep_out, ctx->part, f);
  // a full pass reads the state, q_prev and r once and writes merged, r2 and
  // the decisions; a later pass of an order computes only the tiles near the
  // previous pass's changes (decided on the device), counted as no bytes (with
  // one pass per order every pass is the first of its order)
  const bool full = fs.ctl ? (fs.pass == 0 || fs.jfmax == 1) : fs.first != 0;
  HS_TRY(prof_end(ctx, HS_PROF_FILTER,
                  full ? (double)ctx->ncell * (8.0 * ctx->nc * 3 + 8.0 * 2 + (keep_out ? 1.0 : 0.0)) : 0.0));
  *nb_out = nb;
  return HS_OK;
}

// One host-driven gated pass (index pass within the step, first: the first of
// its order): merged (the next state), r2, keep_out; the kept count and the
// sum of r2 come back in *kept, *sum (st: every statistics slot).
static hs_status filter_pass(hs_ctx* ctx, const double* cur, const double* q_prev, const double* r, int nord,
                             double* merged, double* r2, uint8_t* keep_out, int pass, bool first,
                             unsigned long long* st, long long* kept, double* sum) {
  int nb;
  FiltSpec fs;
  fs.pass = pass;
  fs.first = first ? 1 : 0;
  HS_TRY(filter_gate_launch(ctx, cur, q_prev, r, nord, merged, r2, keep_out, fs, &nb));
  const int cs = filt_count_slot(pass), ss = filt_sum_slot(pass);
  HS_TRY(finish_stats(ctx, nb, 0u, (1u << cs) | (1u << ss), st));
  *kept = (long long)bits_to_double(st[cs]);
  *sum = bits_to_double(st[ss]);
  return HS_OK;
}

// Cell residual norms of q to rcell; their l1 sum is left as *nb block
// partials in ctx->red.
static hs_status cell_residual_partials(hs_ctx* ctx, const double* q, const double* q_prev, double* rcell,
                                        int* nb_out) {
  const int nb = blocks_for(ctx->ncell);
  if (nb > kRedBlocks * 64) return ctx->fail(HS_ERR_SHAPE, "grid too large for the reduction buffer");
  HS_TRY(prof_begin(ctx, HS_PROF_CELLRES));
  if (ctx->nc == 1) HS_LAUNCH(ctx, cellres_kernel<1>, nb, kBlock, ctx->g, q, q_prev, rcell, ctx->red);
  else HS_LAUNCH(ctx, cellres_kernel<4>, nb, kBlock, ctx->g, q, q_prev, rcell, ctx->red);
  HS_TRY(prof_end(ctx, HS_PROF_CELLRES, (double)ctx->ncell * (16.0 * ctx->nc + 8.0)));
  *nb_out = nb;
  return HS_OK;
}

hs_status cell_residual_launch(hs_ctx* ctx, const double* q, const double* q_prev, double* rcell, int slot) {
  int nb;
  HS_TRY(cell_residual_partials(ctx, q, q_prev, rcell, &nb));
  HS_LAUNCH(ctx, sum_finish_kernel, 1, kBlock, ctx->red, nb, reinterpret_cast<double*>(ctx->stats + slot));
  return HS_OK;
}

hs_status cell_residual_norm(hs_ctx* ctx, const double* q, const double* q_prev, double* rcell,
                             double* sum_out) {
  const int nb = blocks_for(ctx->ncell);
  if (nb > kRedBlocks * 64) return ctx->fail(HS_ERR_SHAPE, "grid too large for the reduction buffer");
  HS_TRY(prof_begin(ctx, HS_PROF_CELLRES));
  if (ctx->nc == 1) HS_LAUNCH(ctx, cellres_kernel<1>, nb, kBlock, ctx->g, q, q_prev, rcell, ctx->red);
  else HS_LAUNCH(ctx, cellres_kernel<4>, nb, kBlock, ctx->g, q, q_prev, rcell, ctx->red);
  // reads q and q_prev (neighbours counted once), writes one norm per cell
  HS_TRY(prof_end(ctx, HS_PROF_CELLRES, (double)ctx->ncell * (16.0 * ctx->nc + 8.0)));
  double* slot = ctx->small + kSmMisc + 8;
  HS_LAUNCH(ctx, sum_finish_kernel, 1, kBlock, ctx->red, nb, slot);
  return readback(ctx, slot, sizeof(double), sum_out);
}

static hs_status filter_apply(hs_ctx* ctx, const double* in, double* out, int nord) {
  const long long n = ctx->n;
  const int nb = blocks_for(n);
  if (ctx->g.kind == HS_BURGERS_1D) {
    HS_LAUNCH(ctx, shapiro_kernel, nb, kBlock, ctx->g, in, out, 0, nord);
  } else {
    HS_LAUNCH(ctx, shapiro_kernel, nb, kBlock, ctx->g, in, ctx->R, 0, nord);
    HS_LAUNCH(ctx, shapiro_kernel, nb, kBlock, ctx->g, (const double*)ctx->R, out, 1, nord);
  }
  return HS_OK;
}

// One host synchronisation per pass: the gate's kept count and the l1 sum of
// the merged state's cell residual norms are read together (when nothing was
// kept the merged state equals the current one, so the sum is unchanged).
// The norms carry over from one filter order to the next (same state).
// The filter loop driven by the device state (no recording): the host keeps
// two passes enqueued beyond the last record it has read (pass k + 1 posts
// the record of pass k), and stops enqueueing once a record says the loop is
// done (the pass that posted it then did nothing).
static hs_status run_filter_device(hs_ctx* ctx, double* gamma, const double* q_prev, const hs_hybrid_params* hp,
                                   hs_step_info* info) {
  FiltCtl* ctl = reinterpret_cast<FiltCtl*>(ctx->small + kSmFilt);   // two slots
  int nbr;
  HS_TRY(cell_residual_partials(ctx, gamma, q_prev, ctx->rcell, &nbr));
  HS_LAUNCH(ctx, filt_init_kernel, 1, kBlock, ctl, (const double*)ctx->red, nbr, ctx->stats, 0);
  FiltSpec fs;
  fs.ctl = ctl;
  fs.state[0] = gamma;
  fs.state[1] = ctx->gtmp;
  fs.norms[0] = ctx->rcell;
  fs.norms[1] = ctx->rcell2;
  for (int o = 0; o < hp->n_orders; ++o) fs.orders[o] = hp->filter_orders[o];
  fs.n_orders = hp->n_orders;
  fs.jfmax = hp->jfmax;
  fs.eps_f = hp->eps_f;
  fs.stats = ctx->stats;
  const long long max_passes = (long long)hp->n_orders * hp->jfmax;
  long long enqueued = 0;
  // pass k = enqueued; for k >= 1 it posts the record of pass k - 1 to *p
  auto enqueue = [&](PostSlot* p) -> hs_status {
    int nb;
    fs.pass = (int)enqueued;
    fs.post = p ? (*p = post_slot(ctx)) : PostSlot{};
    // the pointers and the order come from the device state
    HS_TRY(filter_gate_launch(ctx, gamma, q_prev, ctx->rcell, 1, ctx->gtmp, ctx->rcell2, nullptr, fs, &nb));
    ++enqueued;
    return HS_OK;
  };
  // one record is outstanding at a time: that of pass k, posted by pass k + 1
  // (running or queued), while pass k + 2 is enqueued once it is read
  PostSlot pend;
  HS_TRY(enqueue(nullptr));
  HS_TRY(enqueue(&pend));
  unsigned long long rec[8];
  for (;;) {
    HS_TRY(await_post(ctx, pend, rec, 7 * sizeof(unsigned long long)));
    if (rec[2]) break;
    if (enqueued > max_passes) return ctx->fail(HS_ERR_INVALID_ARG, "filter loop ran past its pass bound");
    HS_TRY(enqueue(&pend));
  }
  if (info) {
    info->filter_passes += (int)rec[4];
    info->filter_kept += (int)rec[5];
  }
  if (rec[3]) HIP_TRY(ctx, hipMemcpyAsync(gamma, ctx->gtmp, ctx->n * 8, hipMemcpyDeviceToDevice, ctx->stream));
  return HS_OK;
}

hs_status run_filter(hs_ctx* ctx, double* gamma, const double* q_prev, const hs_hybrid_params* hp,
                     hs_step_info* info, hs_htape* record) {
  if (!record) {
    if (hp->n_orders <= 0 || hp->jfmax <= 0) return HS_OK;
    return run_filter_device(ctx, gamma, q_prev, hp, info);
  }
  if (record) {
    if ((long long)hp->n_orders * hp->jfmax > kMaxPasses)
      return ctx->fail(HS_ERR_INVALID_ARG, "taped step: more filter passes possible than the tape holds");
    record->npass = 0;
  }
  double* cur = gamma;
  double* spare = ctx->gtmp;
  double* r = ctx->rcell;
  double* r2 = ctx->rcell2;
  bool have_sum = false;
  double sum_r = 0.0;
  if (hp->n_orders > 0 && hp->jfmax > 0) HS_TRY(cell_residual_launch(ctx, cur, q_prev, r, kStatSum0));
  int pass = 0;
  for (int o = 0; o < hp->n_orders; ++o) {
    const int nord = hp->filter_orders[o];
    for (int it = 1; it <= hp->jfmax; ++it) {
      uint8_t* keep_out = record ? record->masks + (size_t)record->npass * ctx->ncell : nullptr;
      unsigned long long st[kStatSlots];
      long long kept;
      double sum_new;
      HS_TRY(filter_pass(ctx, cur, q_prev, r, nord, spare, r2, keep_out, pass, it == 1, st, &kept, &sum_new));
      ++pass;
      if (!have_sum) {
        sum_r = bits_to_double(st[kStatSum0]);
        have_sum = true;
      }
      if (info) {
        info->filter_passes += 1;
        info->filter_kept += (int)kept;
      }
      if (kept == 0) break;
      if (record) record->passes[record->npass++] = nord;
      std::swap(cur, spare);
      std::swap(r, r2);
      const double dec = (sum_r - sum_new) / sum_r;
      sum_r = sum_new;
      if (dec < hp->eps_f) break;
    }
  }
  if (cur != gamma)
    HIP_TRY(ctx, hipMemcpyAsync(gamma, cur, ctx->n * 8, hipMemcpyDeviceToDevice, ctx->stream));
  return HS_OK;
}

// The recorded filter passes applied without gating.
static hs_status replay_filter(hs_ctx* ctx, double* gamma, const hs_htape* tape, hs_step_info* info) {
  double* cur = gamma;
  double* spare = ctx->gtmp;
  for (int k = 0; k < tape->npass; ++k) {
    HS_TRY(filter_apply(ctx, cur, ctx->gf, tape->passes[k]));
    HS_LAUNCH(ctx, mask_blend_kernel, blocks_for(ctx->n), kBlock, (long long)ctx->n, ctx->ncell, cur, ctx->gf,
              tape->masks + (size_t)k * ctx->ncell, spare);
    std::swap(cur, spare);
    if (info) info->filter_passes += 1;
  }
  if (cur != gamma)
    HIP_TRY(ctx, hipMemcpyAsync(gamma, cur, ctx->n * 8, hipMemcpyDeviceToDevice, ctx->stream));
  return HS_OK;
}

// ------------------------------------------------------------- fit helpers
static int pad16(int m) { return (m + 15) / 16 * 16; }

template <typename TP>
static hs_status launch_project_t(hs_ctx* ctx, const TP* Phi, int m, const int* hat, int ns, const double* u,
                                  const double* psi, const double* y0, int mode, int nb, int nc) {
  const long long n = ctx->n;
  switch (pad16(m)) {
    case 16: HS_LAUNCH(ctx, (project_kernel<16, TP>), nb, kBlock, Phi, n, m, nc, ctx->ncell, hat, ns, u, psi, y0, mode, ctx->red); break;
    case 32: HS_LAUNCH(ctx, (project_kernel<32, TP>), nb, kBlock, Phi, n, m, nc, ctx->ncell, hat, ns, u, psi, y0, mode, ctx->red); break;
    case 48: HS_LAUNCH(ctx, (project_kernel<48, TP>), nb, kBlock, Phi, n, m, nc, ctx->ncell, hat, ns, u, psi, y0, mode, ctx->red); break;
    default: HS_LAUNCH(ctx, (project_kernel<64, TP>), nb, kBlock, Phi, n, m, nc, ctx->ncell, hat, ns, u, psi, y0, mode, ctx->red); break;
  }
  return HS_OK;
}

// Phi is double (HS_FP64) or float (HS_MIXED_FP32).  The rows are every
// component of the listed cells, or (nc = 1) the listed entries themselves.
static hs_status launch_project(hs_ctx* ctx, const void* Phi, int prec, int m, const int* hat, int ns,
                                const double* u, const double* psi, const double* y0, int mode, int* nb_out,
                                int nc = -1) {
  if (nc < 0) nc = ctx->nc;
  const long long rows = hat ? (long long)nc * ns : ctx->n;
  const int nb = (int)std::max<long long>(1, std::min<long long>((rows + kBlock - 1) / kBlock, 512));
  *nb_out = nb;
  if (prec == HS_MIXED_FP32)
    return launch_project_t(ctx, (const float*)Phi, m, hat, ns, u, psi, y0, mode, nb, nc);
  return launch_project_t(ctx, (const double*)Phi, m, hat, ns, u, psi, y0, mode, nb, nc);
}

template <typename TP>
static hs_status launch_ring(hs_ctx* ctx, const TP* Phi, int m, const hs_samples* s, const double* psi,
                             const double* y, double* u) {
  HS_LAUNCH(ctx, ring_update_kernel<TP>, blocks_for((long long)ctx->nc * s->l), kBlock, Phi, (long long)ctx->n, m,
            ctx->nc, ctx->ncell, s->tilde, s->l, psi, y, u);
  return HS_OK;
}

template <typename TP>
static hs_status launch_recon(hs_ctx* ctx, const TP* Phi, int m, const double* psi, const double* y,
                              const uint8_t* mask, const double* u, double* gamma, double* rho) {
  HS_LAUNCH(ctx, recon_kernel<TP>, blocks_for(ctx->n), kBlock, Phi, (long long)ctx->n, m, ctx->ncell, psi, y, mask,
            u, gamma, rho);
  return HS_OK;
}

static hs_status ring_update(hs_ctx* ctx, const void* Phi, int prec, int m, const hs_samples* s, const double* psi,
                             const double* y, double* u) {
  if (prec == HS_MIXED_FP32) return launch_ring(ctx, (const float*)Phi, m, s, psi, y, u);
  return launch_ring(ctx, (const double*)Phi, m, s, psi, y, u);
}

static hs_status reconstruct(hs_ctx* ctx, const void* Phi, int prec, int m, const double* psi, const double* y,
                             const uint8_t* mask, const double* u, double* gamma, double* rho) {
  if (prec == HS_MIXED_FP32) return launch_recon(ctx, (const float*)Phi, m, psi, y, mask, u, gamma, rho);
  return launch_recon(ctx, (const double*)Phi, m, psi, y, mask, u, gamma, rho);
}

// Gram of the (gathered) rows and its truncated pseudo-inverse (FP64 MFMA on
// the basis entries in either storage precision).
template <typename TP>
static hs_status launch_fit_gram(hs_ctx* ctx, const TP* Phi, int m, const int* hat, int ns, int nb, int wp,
                                 long long rows, int nc) {
  GatherLoader<TP> ld{Phi, (long long)ctx->n, m, nc, ctx->ncell, ns, hat};
  const size_t lds = (size_t)kChunk * (wp + 1) * sizeof(double);
  hipLaunchKernelGGL(gram_kernel<GatherLoader<TP>>, dim3(nb), dim3(256), lds, ctx->stream, ld, rows, wp, ctx->red);
  HIP_TRY(ctx, hipGetLastError());
  return HS_OK;
}

static hs_status fit_factor(hs_ctx* ctx, const void* Phi, int prec, int m, const int* hat, int ns, double rcond,
                            int nc = -1) {
  if (nc < 0) nc = ctx->nc;
  const int wp = pad16(m);
  const long long rows = hat ? (long long)nc * ns : ctx->n;
  const long long nchunks = (rows + kChunk - 1) / kChunk;
  const int nb = (int)std::max<long long>(1, std::min<long long>(nchunks, 512));
  if (prec == HS_MIXED_FP32) HS_TRY(launch_fit_gram(ctx, (const float*)Phi, m, hat, ns, nb, wp, rows, nc));
  else HS_TRY(launch_fit_gram(ctx, (const double*)Phi, m, hat, ns, nb, wp, rows, nc));
  HS_LAUNCH(ctx, gram_reduce_kernel, m * m, kBlock, ctx->red, nb, wp, m, ctx->small + kSmG);
  if (ctx->small_pinv && m >= 1 && m <= 8)
    HS_LAUNCH(ctx, pinv_small_kernel, 1, kWave, ctx->small + kSmG, m, rcond, ctx->small + kSmGp,
              ctx->small + kSmMisc, ctx->stats);
  else
    HS_LAUNCH(ctx, pinv_kernel, 1, 256, ctx->small + kSmG, m, rcond, ctx->small + kSmGp, ctx->small + kSmMisc,
              ctx->stats, ctx->fit_chol);
  return HS_OK;
}

// y = pinv fit of (u - psi) on the rows, with one refinement step.
static hs_status fit_solve(hs_ctx* ctx, const void* Phi, int prec, int m, const int* hat, int ns, const double* u,
                           const double* psi, int first, int nc = -1) {
  double* sm = ctx->small;
  int nb;
  HS_TRY(launch_project(ctx, Phi, prec, m, hat, ns, u, psi, nullptr, 0, &nb, nc));
  HS_LAUNCH(ctx, project_finish_kernel, 1, 256, ctx->red, nb, pad16(m), m, sm + kSmGp, 0, sm + kSmY0, sm + kSmY,
            sm + kSmYPrev, sm + kSmMisc, first, (unsigned long long*)nullptr);
  HS_TRY(launch_project(ctx, Phi, prec, m, hat, ns, u, psi, sm + kSmY0, 1, &nb, nc));
  HS_LAUNCH(ctx, project_finish_kernel, 1, 256, ctx->red, nb, pad16(m), m, sm + kSmGp, 1, sm + kSmY0, sm + kSmY,
            sm + kSmYPrev, sm + kSmMisc, first, ctx->stats);
  return HS_OK;
}

// mode: -1 plain step, HS_TAPE_RECORD, HS_TAPE_REPLAY (see the header).
static hs_status hybrid_impl(hs_ctx* ctx, const double* q_prev, const void* Phi, const double* psi, int m,
                             const hs_samples* s, const hs_hybrid_params* hp, double* q_out, double* eps_out,
                             double* y_out, hs_step_info* info, hs_htape* tape, int mode,
                             const int32_t* fit_points = nullptr, int32_t n_fit = 0) {
  if (!ctx) return HS_ERR_INVALID_ARG;
  // HS_BASIS_PENDING: the basis is still being formed on the context's
  // second stream; it is completed after the first Newton solve, and on
  // every early return by the guard
  const bool pending = m == HS_BASIS_PENDING;
  struct PendingGuard {
    hs_ctx* c;
    bool active;
    ~PendingGuard() {
      int32_t me;
      if (active && c->aux_pending) (void)basis_finish_pending(c, &me);
    }
  } guard{ctx, pending};
  if (!q_prev || !Phi || !psi || !hp || !q_out) return HS_ERR_INVALID_ARG;
  if (q_out == q_prev || q_out == psi || (const void*)q_out == Phi) return HS_ERR_INVALID_ARG;
  const bool replay = mode == HS_TAPE_REPLAY;
  if (mode >= 0 && (!tape || tape->ctx != ctx)) return HS_ERR_INVALID_ARG;
  if (replay) {
    if (!tape->recorded) return ctx->fail(HS_ERR_INVALID_ARG, "replay of a tape that holds no recorded step");
    s = tape->s;
  }
  if (pending && (replay || !ctx->aux_pending))
    return ctx->fail(HS_ERR_INVALID_ARG, "HS_BASIS_PENDING needs an asynchronous basis update in flight");
  if (!s || s->ctx != ctx) return HS_ERR_INVALID_ARG;
  if (!pending && (m < 1 || m > ctx->p.m_max)) return ctx->fail(HS_ERR_RANK, "empty basis");
  if (hp->jmax < 1 || hp->n_orders < 0 || hp->n_orders > 4 || !(hp->rcond_fit > 0) || !(hp->eps_y >= 0))
    return HS_ERR_INVALID_ARG;
  for (int o = 0; o < hp->n_orders; ++o)
    if (hp->filter_orders[o] < 1 || hp->filter_orders[o] > 3) return HS_ERR_INVALID_ARG;
  const int prec = hp->precision;
  if (prec != HS_FP64 && prec != HS_MIXED_FP32) return HS_ERR_INVALID_ARG;
  if (s->n_s == 0) return ctx->fail(HS_ERR_RANK, "empty sampled set");
  if (n_fit < 0 || n_fit > ctx->n || (n_fit > 0 && !fit_points)) return ctx->fail(HS_ERR_INVALID_ARG, "fit points");
  if (n_fit > 0 && mode >= 0) return ctx->fail(HS_ERR_INVALID_ARG, "a taped step fits over the sampled cells");
  // the fit's rows: every entry of the sampled cells, or the given entries
  const int* frows = n_fit > 0 ? fit_points : s->hat;
  const int nfr = n_fit > 0 ? n_fit : s->n_s;
  const int fnc = n_fit > 0 ? 1 : ctx->nc;
  hs_step_info local{};
  hs_step_info* inf = info ? info : &local;
  std::memset(inf, 0, sizeof *inf);
  inf->n_s = s->n_s;
  inf->l = s->l;
  const int jmax = replay ? tape->J : hp->jmax;
  if (replay) {
    const size_t need = (size_t)jmax * ctx->n;
    if (tape->us_cap < need) {
      if (tape->us) HIP_TRY(ctx, hipFree(tape->us));
      tape->us = nullptr;
      tape->us_cap = 0;
      if (hipMalloc((void**)&tape->us, need * 8) != hipSuccess)
        return ctx->fail(HS_ERR_OOM, "tape: no memory for the subiteration states");
      tape->us_cap = need;
    }
  }

  double* u = ctx->u;
  double* sm = ctx->small;
  // max |q_prev| (Newton tolerance) and the fit factorisation, read together
  // (with a pending basis the factorisation follows the first Newton solve);
  // with the device decision they come back with the first Newton
  // iteration, whose sweep launch forms the tolerance from the same value
  HS_TRY(max_abs_launch(ctx, q_prev, ctx->n));
  HIP_TRY(ctx, hipMemcpyAsync(u, q_prev, ctx->n * 8, hipMemcpyDeviceToDevice, ctx->stream));
  if (!pending) HS_TRY(fit_factor(ctx, Phi, prec, m, frows, nfr, hp->rcond_fit, fnc));
  unsigned long long st[kStatSlots];
  double primed[3];
  bool have_primed = false;
  const bool ctrl = newton_ctrl_ok(ctx, s) && ctx->p.newton_rtol > 0.0;
  if (ctrl) {
    int dev_total = 0;
    HS_TRY(newton_first_ctrl(ctx, u, q_prev, 0.0, s, 0, 0.0, st, &dev_total, true));
    primed[0] = bits_to_double(st[kStatResMax]);
    primed[1] = bits_to_double(st[kStatRho]);
    primed[2] = dev_total;
    have_primed = true;
  } else {
    HS_TRY(read_stats(ctx, st));
  }
  const double qmax = bits_to_double(st[kStatQMax]);
  if (!std::isfinite(qmax)) return ctx->fail(HS_ERR_NONFINITE, "non-finite q_prev");
  const double tol = ctx->p.newton_rtol * std::max(1.0, qmax);
  auto fit_stats = [&]() -> hs_status {
    inf->fit_rank = (int)bits_to_double(st[kStatFitRank]);
    inf->fit_cond = bits_to_double(st[kStatFitCond]);
    return inf->fit_rank == 0 ? ctx->fail(HS_ERR_RANK, "rank-zero fit") : HS_OK;
  };
  if (!pending) HS_TRY(fit_stats());

  // Subiterations.  The stop test on ||y_j - y_{j-1}|| is read together with
  // the residual of the next Newton solve's first iteration, launched
  // speculatively (it changes no state, so it is simply dropped on a stop).
  bool fit_check = false;   // the fit factorised after the pending basis: its rank still to read
  for (int j = 1; j <= jmax; ++j) {
    HS_TRY(newton_solve(ctx, u, q_prev, tol, s, inf, have_primed ? primed : nullptr));
    have_primed = false;   // consumed: a replayed subiteration launches its own first iteration
    if (pending && j == 1) {
      int32_t me = 0;
      guard.active = false;
      HS_TRY(basis_finish_pending(ctx, &me));
      if (me < 1 || me > ctx->p.m_max) return ctx->fail(HS_ERR_RANK, "empty basis");
      m = me;
      // its rank and condition come back with this subiteration's decision
      HS_TRY(fit_factor(ctx, Phi, prec, m, frows, nfr, hp->rcond_fit, fnc));
      fit_check = true;
    }
    if (replay)
      HIP_TRY(ctx, hipMemcpyAsync(tape->us + (size_t)(j - 1) * ctx->n, u, ctx->n * 8, hipMemcpyDeviceToDevice,
                                  ctx->stream));
    HS_TRY(fit_solve(ctx, Phi, prec, m, frows, nfr, u, psi, j == 1, fnc));
    if (s->l > 0) HS_TRY(ring_update(ctx, Phi, prec, m, s, psi, sm + kSmY, u));
    inf->subiters = j;
    if (replay) continue;
    const bool more = j < jmax;
    // with the device decision, the next solve's first sweeps start at once
    // unless the device's stop test (the same as below) ends the loop
    int dev_total = 0;
    if (more && ctrl) HS_TRY(newton_first_ctrl(ctx, u, q_prev, tol, s, j >= 2, hp->eps_y, st, &dev_total));
    else if (more) HS_TRY(newton_first_launch(ctx, u, q_prev, s, st));
    else HS_TRY(read_stats(ctx, st));
    if (fit_check) {
      fit_check = false;
      HS_TRY(fit_stats());
    }
    const double dy = bits_to_double(st[kStatDy]);
    inf->dy_last = dy;
    if (!more || (j >= 2 && dy < hp->eps_y)) break;
    primed[0] = bits_to_double(st[kStatResMax]);
    primed[1] = bits_to_double(st[kStatRho]);
    primed[2] = dev_total;
    have_primed = true;
  }
  if (replay) {
    HIP_TRY(ctx, hipMemcpyAsync(tape->gp, sm + kSmGp, (size_t)m * m * 8, hipMemcpyDeviceToDevice, ctx->stream));
    tape->m = m;
    tape->precision = prec;
  }
  HS_TRY(prof_begin(ctx, HS_PROF_RECON));
  HS_TRY(reconstruct(ctx, Phi, prec, m, psi, sm + kSmY, s->mask, u, q_out, ctx->rho));
  // reads m columns of Phi, psi, u and the mask; writes gamma and rho
  const double phi_bytes = prec == HS_MIXED_FP32 ? 4.0 : 8.0;
  HS_TRY(prof_end(ctx, HS_PROF_RECON, (double)ctx->n * (phi_bytes * m + 32.0) + (double)ctx->ncell));
  if (replay) HS_TRY(replay_filter(ctx, q_out, tape, inf));
  else HS_TRY(run_filter(ctx, q_out, q_prev, hp, inf, mode == HS_TAPE_RECORD ? tape : nullptr));
  if (eps_out) {
    int nbq;
    HS_TRY(max_abs_partials(ctx, q_out, ctx->n, &nbq));
    HS_LAUNCH(ctx, indicator_kernel, blocks_for(ctx->ncell), kBlock, ctx->ncell, ctx->nc, q_out, ctx->rho,
              hp->floor_rel, (const double*)ctx->part, nbq, eps_out);
  }
  if (y_out) HIP_TRY(ctx, hipMemcpyAsync(y_out, sm + kSmY, m * 8, hipMemcpyDeviceToDevice, ctx->stream));
  if (mode == HS_TAPE_RECORD) {
    HS_TRY(hs_samples_set(ctx, tape->s, s->hat, s->n_s));
    tape->J = inf->subiters;
    tape->recorded = true;
    tape->replayed = false;
  }
  if (replay) tape->replayed = true;
  // outputs complete in stream order: no wait for the work after the last decision
  return HS_OK;
}

// ------------------------------------------- Gauss-Newton subiterations
// Rows of the misfit's Jacobian A = Phi_S + X (X = J_S^-1 J_T Phi_T, column
// j at X + j N in the compact layout a ncell + p of the sampled list): the
// gathered rows of Phi plus those of X, for the Gram A^T A on MFMA.
struct GnLoader {
  const double* Phi;
  const double* X;
  long long n;
  int m, nc, ncell, ns;
  const int* hat;
  struct Regs {
    double v[kMaxBasis / 4];
  };
  __device__ void init(Regs&) const {}
  __device__ void prefetch(long long row0, Regs& R) const {
    const int r = threadIdx.x % kChunk;
    const long long row = row0 + r;
    long long dof = -1, xo = 0;
    if (row < (long long)nc * ns) {
      const int a = (int)(row / ns), p = (int)(row % ns);
      dof = (long long)a * ncell + hat[p];
      xo = (long long)a * ncell + p;
    }
#pragma unroll
    for (int i = 0; i < kMaxBasis / 4; ++i) {
      const int j = threadIdx.x / kChunk + 4 * i;
      R.v[i] = (dof >= 0 && j < m) ? Phi[(size_t)j * n + dof] + X[(size_t)j * n + xo] : 0.0;
    }
  }
  __device__ void commit(long long, const Regs& R, double* Xl, int ldx, int wp) const {
    const int r = threadIdx.x % kChunk;
#pragma unroll
    for (int i = 0; i < kMaxBasis / 4; ++i) {
      const int j = threadIdx.x / kChunk + 4 * i;
      if (j < wp) Xl[r * ldx + j] = R.v[i];
    }
  }
};

// out = D^-1 J_T phi on the sampled list: for each sampled cell the
// Jacobian blocks of its neighbours outside the sampled set (the ring; a
// ghost that copies the cell is part of D, an inflow ghost is constant)
// applied to column phi of the basis, then the cell's diagonal block
// inverted (the right-hand side of the relaxation of J_S x = J_T phi).
template <int NC>
__global__ void __launch_bounds__(kBlock) gn_coupling_kernel(Grid g, const double* __restrict__ u,
                                                             const int* __restrict__ hat,
                                                             const int* __restrict__ nbr, int count,
                                                             const double* __restrict__ phi,
                                                             double* __restrict__ out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= count) return;
  const int cap = g.ncell;
  const int cell = hat[p];
  Stencil<NC> st;
  load_stencil<NC>(g, u, cell, st);
  double D[NC * NC], O[4][NC * NC], Di[NC * NC];
  cell_jacobian<NC>(g, st, D, O);
  small_inverse<NC>(D, Di);
  double b[NC];
#pragma unroll
  for (int a = 0; a < NC; ++a) b[a] = 0.0;
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const int nb = st.idx[d];
    if (nbr[d * cap + p] >= 0 || nb < 0 || nb == cell) continue;
#pragma unroll
    for (int a = 0; a < NC; ++a)
#pragma unroll
      for (int c = 0; c < NC; ++c) b[a] += O[d][a * NC + c] * phi[(size_t)c * g.ncell + nb];
  }
#pragma unroll
  for (int a = 0; a < NC; ++a) {
    double v = 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) v += Di[a * NC + c] * b[c];
    out[(size_t)a * cap + p] = v;
  }
}

// Per-block partials of -A^T r over the sampled rows, r = Phi_S y - (u_S - psi_S).
template <int MP>
__global__ void __launch_bounds__(256) gn_grad_kernel(const double* __restrict__ Phi, const double* __restrict__ X,
                                                      long long n, int m, int nc, int ncell,
                                                      const int* __restrict__ hat, int ns,
                                                      const double* __restrict__ u,
                                                      const double* __restrict__ psi,
                                                      const double* __restrict__ y, double* __restrict__ part) {
  __shared__ double yl[MP];
  __shared__ double wsum[4][MP];
  for (int j = threadIdx.x; j < MP; j += blockDim.x) yl[j] = j < m ? y[j] : 0.0;
  __syncthreads();
  double acc[MP];
#pragma unroll
  for (int j = 0; j < MP; ++j) acc[j] = 0.0;
  const long long rows = (long long)nc * ns;
  for (long long row = blockIdx.x * (long long)blockDim.x + threadIdx.x; row < rows;
       row += (long long)gridDim.x * blockDim.x) {
    const long long a = row / ns, p = row % ns;
    const long long dof = a * ncell + hat[p], xo = a * ncell + p;
    double ph[MP];
    double r = 0.0;
#pragma unroll
    for (int j = 0; j < MP; ++j) {
      ph[j] = j < m ? Phi[(size_t)j * n + dof] : 0.0;
      r += ph[j] * yl[j];
    }
    r -= u[dof] - psi[dof];
#pragma unroll
    for (int j = 0; j < MP; ++j) acc[j] -= (j < m ? ph[j] + X[(size_t)j * n + xo] : 0.0) * r;
  }
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
#pragma unroll
  for (int j = 0; j < MP; ++j) {
    const double v = wave_sum(acc[j]);
    if (lane == 0) wsum[wave][j] = v;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < m; j += blockDim.x)
    part[(size_t)blockIdx.x * MP + j] = ((wsum[0][j] + wsum[1][j]) + wsum[2][j]) + wsum[3][j];
}

// One Gauss-Newton subiteration's step after the partial solve in u: the
// relaxation data of the sampled Jacobian at u, X by m relaxed solves into
// work, A^T A and its pseudo-inverse, y <- y - (A^T A)^+ A^T r; ||dy|| to the
// statistics.
template <int NC>
static hs_status gn_step(hs_ctx* ctx, const double* Phi, int m, const hs_samples* s, const double* psi,
                         const double* q_prev, double rcond, double* work, hs_step_info* inf) {
  double* sm = ctx->small;
  const long long n = ctx->n;
  unsigned long long st[kStatSlots];
  HS_TRY(newton_first_launch(ctx, ctx->u, q_prev, s, st));
  const double rho = bits_to_double(st[kStatRho]);
  for (int k = 0; k < m; ++k) {
    HS_LAUNCH(ctx, gn_coupling_kernel<NC>, blocks_for(s->n_s), kBlock, ctx->g, (const double*)ctx->u, s->hat,
              s->nbr, s->n_s, Phi + (size_t)k * n, ctx->adj);
    int sweeps = 0;
    HS_TRY(relax_solve(ctx, s, ctx->coef, ctx->adj, rho, ctx->p.lin_rtol, work + (size_t)k * n, &sweeps));
    inf->lin_sweeps += sweeps;
  }
  // A^T A on MFMA and its pseudo-inverse (rank and condition to the statistics)
  const int wp = pad16(m);
  const long long rows = (long long)NC * s->n_s;
  const long long nchunks = (rows + kChunk - 1) / kChunk;
  const int nb = (int)std::max<long long>(1, std::min<long long>(nchunks, 512));
  GnLoader ld{Phi, work, n, m, NC, ctx->ncell, s->n_s, s->hat};
  const size_t lds = (size_t)kChunk * (wp + 1) * sizeof(double);
  hipLaunchKernelGGL(gram_kernel<GnLoader>, dim3(nb), dim3(256), lds, ctx->stream, ld, rows, wp, ctx->red);
  HIP_TRY(ctx, hipGetLastError());
  HS_LAUNCH(ctx, gram_reduce_kernel, m * m, kBlock, ctx->red, nb, wp, m, sm + kSmG);
  if (ctx->small_pinv && m <= 8)
    HS_LAUNCH(ctx, pinv_small_kernel, 1, kWave, sm + kSmG, m, rcond, sm + kSmGp, sm + kSmMisc, ctx->stats);
  else
    HS_LAUNCH(ctx, pinv_kernel, 1, 256, sm + kSmG, m, rcond, sm + kSmGp, sm + kSmMisc, ctx->stats, ctx->fit_chol);
  // y0 = y_prev = y; y = y0 + G+ (-A^T r)
  HIP_TRY(ctx, hipMemcpyAsync(sm + kSmY0, sm + kSmY, m * 8, hipMemcpyDeviceToDevice, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(sm + kSmYPrev, sm + kSmY, m * 8, hipMemcpyDeviceToDevice, ctx->stream));
  const int nbg = (int)std::max<long long>(1, std::min<long long>((rows + kBlock - 1) / kBlock, 512));
  switch (wp) {
    case 16: HS_LAUNCH(ctx, gn_grad_kernel<16>, nbg, 256, Phi, (const double*)work, n, m, NC, ctx->ncell, s->hat, s->n_s, (const double*)ctx->u, psi, (const double*)(sm + kSmY), ctx->red); break;
    case 32: HS_LAUNCH(ctx, gn_grad_kernel<32>, nbg, 256, Phi, (const double*)work, n, m, NC, ctx->ncell, s->hat, s->n_s, (const double*)ctx->u, psi, (const double*)(sm + kSmY), ctx->red); break;
    case 48: HS_LAUNCH(ctx, gn_grad_kernel<48>, nbg, 256, Phi, (const double*)work, n, m, NC, ctx->ncell, s->hat, s->n_s, (const double*)ctx->u, psi, (const double*)(sm + kSmY), ctx->red); break;
    default: HS_LAUNCH(ctx, gn_grad_kernel<64>, nbg, 256, Phi, (const double*)work, n, m, NC, ctx->ncell, s->hat, s->n_s, (const double*)ctx->u, psi, (const double*)(sm + kSmY), ctx->red); break;
  }
  HS_LAUNCH(ctx, project_finish_kernel, 1, 256, ctx->red, nbg, wp, m, sm + kSmGp, 1, sm + kSmY0, sm + kSmY,
            sm + kSmYPrev, sm + kSmMisc, 0, ctx->stats);
  return HS_OK;
}

// The hybrid step with Gauss-Newton subiterations on the reduced coordinates
// (the first iterate is the paper's first subiteration); FP64 basis.
static hs_status hybrid_gn_impl(hs_ctx* ctx, const double* q_prev, const double* Phi, const double* psi, int m,
                                const hs_samples* s, const hs_hybrid_params* hp, double* work, double* q_out,
                                double* eps_out, double* y_out, hs_step_info* info) {
  if (!ctx || !q_prev || !Phi || !psi || !hp || !q_out || !s || !work) return HS_ERR_INVALID_ARG;
  if (q_out == q_prev || q_out == psi || q_out == Phi || s->ctx != ctx) return HS_ERR_INVALID_ARG;
  if (m < 1 || m > ctx->p.m_max) return ctx->fail(HS_ERR_RANK, "empty basis");
  if (hp->precision != HS_FP64) return ctx->fail(HS_ERR_INVALID_ARG, "Gauss-Newton subiterations need an FP64 basis");
  if (hp->jmax < 1 || hp->n_orders < 0 || hp->n_orders > 4 || !(hp->rcond_fit > 0) || !(hp->eps_y >= 0))
    return HS_ERR_INVALID_ARG;
  for (int o = 0; o < hp->n_orders; ++o)
    if (hp->filter_orders[o] < 1 || hp->filter_orders[o] > 3) return HS_ERR_INVALID_ARG;
  if (s->n_s == 0) return ctx->fail(HS_ERR_RANK, "empty sampled set");
  hs_step_info local{};
  hs_step_info* inf = info ? info : &local;
  std::memset(inf, 0, sizeof *inf);
  inf->n_s = s->n_s;
  inf->l = s->l;
  double* u = ctx->u;
  double* sm = ctx->small;
  HS_TRY(max_abs_launch(ctx, q_prev, ctx->n));
  HIP_TRY(ctx, hipMemcpyAsync(u, q_prev, ctx->n * 8, hipMemcpyDeviceToDevice, ctx->stream));
  HS_TRY(fit_factor(ctx, Phi, HS_FP64, m, s->hat, s->n_s, hp->rcond_fit));
  unsigned long long st[kStatSlots];
  HS_TRY(read_stats(ctx, st));
  const double qmax = bits_to_double(st[kStatQMax]);
  if (!std::isfinite(qmax)) return ctx->fail(HS_ERR_NONFINITE, "non-finite q_prev");
  const double tol = ctx->p.newton_rtol * std::max(1.0, qmax);
  inf->fit_rank = (int)bits_to_double(st[kStatFitRank]);
  inf->fit_cond = bits_to_double(st[kStatFitCond]);
  if (inf->fit_rank == 0) return ctx->fail(HS_ERR_RANK, "rank-zero fit");
  // the first iterate: the paper's first subiteration
  HS_TRY(newton_solve(ctx, u, q_prev, tol, s, inf));
  HS_TRY(fit_solve(ctx, Phi, HS_FP64, m, s->hat, s->n_s, u, psi, 1));
  inf->subiters = 1;
  for (int j = 2; j <= hp->jmax; ++j) {
    if (s->l > 0) HS_TRY(ring_update(ctx, Phi, HS_FP64, m, s, psi, sm + kSmY, u));
    HS_TRY(newton_solve(ctx, u, q_prev, tol, s, inf));
    if (ctx->nc == 1) HS_TRY(gn_step<1>(ctx, Phi, m, s, psi, q_prev, hp->rcond_fit, work, inf));
    else HS_TRY(gn_step<4>(ctx, Phi, m, s, psi, q_prev, hp->rcond_fit, work, inf));
    HS_TRY(read_stats(ctx, st));
    inf->subiters = j;
    inf->dy_last = bits_to_double(st[kStatDy]);
    if (!std::isfinite(inf->dy_last)) return ctx->fail(HS_ERR_NONFINITE, "non-finite Gauss-Newton step");
    if (inf->dy_last < hp->eps_y) break;
  }
  // the sampled values consistent with the final coordinates
  if (s->l > 0) HS_TRY(ring_update(ctx, Phi, HS_FP64, m, s, psi, sm + kSmY, u));
  HS_TRY(newton_solve(ctx, u, q_prev, tol, s, inf));
  HS_TRY(reconstruct(ctx, Phi, HS_FP64, m, psi, sm + kSmY, s->mask, u, q_out, ctx->rho));
  HS_TRY(run_filter(ctx, q_out, q_prev, hp, inf, nullptr));
  if (eps_out) {
    int nbq;
    HS_TRY(max_abs_partials(ctx, q_out, ctx->n, &nbq));
    HS_LAUNCH(ctx, indicator_kernel, blocks_for(ctx->ncell), kBlock, ctx->ncell, ctx->nc, q_out, ctx->rho,
              hp->floor_rel, (const double*)ctx->part, nbq, eps_out);
  }
  if (y_out) HIP_TRY(ctx, hipMemcpyAsync(y_out, sm + kSmY, m * 8, hipMemcpyDeviceToDevice, ctx->stream));
  return hs_sync(ctx);
}

// ------------------------------------------ the paper's full-order scheme
// Gate of one filter pass with precomputed norms: keep the filtered value
// where its cell residual norm rf is below r (all components), count the kept
// cells (kStatCount partials, as doubles).
__global__ void __launch_bounds__(kBlock) paper_gate_kernel(int ncell, const double* __restrict__ r,
                                                            const double* __restrict__ rf,
                                                            const double* __restrict__ gf, double* __restrict__ cur,
                                                            uint8_t* __restrict__ keep_out, double* __restrict__ part) {
  __shared__ double lds[kBlock / kWave];
  double kept = 0.0;
  for (int cell = blockIdx.x * blockDim.x + threadIdx.x; cell < ncell; cell += gridDim.x * blockDim.x) {
    const bool keep = rf[cell] < r[cell];
    if (keep) {
#pragma unroll
      for (int a = 0; a < 4; ++a) cur[(size_t)a * ncell + cell] = gf[(size_t)a * ncell + cell];
      kept += 1.0;
    }
    if (keep_out) keep_out[cell] = keep ? 1 : 0;
  }
  kept = block_sum(kept, lds);
  if (threadIdx.x == 0) stat_part(part, kStatCount, kept);
}

// The residual-gated filters of Sec. 2.3.4 with the paper scheme's cell
// residual norms (the loop of run_filter, host-driven: one read-back per pass).
static hs_status paper_filter(hs_ctx* ctx, const PaperBC& bc, double* gamma, const double* q1, const double* q2,
                              const hs_hybrid_params* hp, hs_step_info* info) {
  if (hp->n_orders <= 0 || hp->jfmax <= 0) return HS_OK;
  double* r = ctx->rcell;
  double* rf = ctx->rcell2;
  int nb;
  unsigned long long st[kStatSlots];
  HS_TRY(paper_cell_norms(ctx, bc, gamma, q1, q2, r, &nb));
  HS_TRY(finish_stats(ctx, nb, 0u, 1u << kStatSum, st));
  double sum_r = bits_to_double(st[kStatSum]);
  for (int o = 0; o < hp->n_orders; ++o) {
    const int nord = hp->filter_orders[o];
    for (int it = 1; it <= hp->jfmax; ++it) {
      HS_TRY(filter_apply(ctx, gamma, ctx->gf, nord));
      HS_TRY(paper_cell_norms(ctx, bc, ctx->gf, q1, q2, rf, &nb));
      HS_LAUNCH(ctx, paper_gate_kernel, stat_blocks(ctx->ncell), kBlock, ctx->ncell, (const double*)r,
                (const double*)rf, (const double*)ctx->gf, gamma, (uint8_t*)nullptr, ctx->part);
      HS_TRY(paper_cell_norms(ctx, bc, gamma, q1, q2, r, &nb));
      HS_TRY(finish_stats(ctx, nb, 0u, (1u << kStatCount) | (1u << kStatSum), st));
      const long long kept = (long long)bits_to_double(st[kStatCount]);
      if (info) {
        info->filter_passes += 1;
        info->filter_kept += (int)kept;
      }
      if (kept == 0) break;
      const double sum_new = bits_to_double(st[kStatSum]);
      const double dec = (sum_r - sum_new) / sum_r;
      sum_r = sum_new;
      if (dec < hp->eps_f) break;
    }
  }
  return HS_OK;
}

// One hybrid step with the paper's scheme: the subiterations of hybrid_impl
// with the BDF residual (q2: q_{k-2}) in the partial solve and the filter
// gate.  The residual of a sampled cell reads two cells along each axis, so
// after every fit all unsampled entries take psi + Phi y (a superset of the
// cells that residual reads).
static hs_status hybrid_paper_impl(hs_ctx* ctx, const hs_paper_hdm* hdm, const double* q_prev, const double* q_prev2,
                                   const void* Phi, const double* psi, int m, const hs_samples* s,
                                   const int32_t* fit_points, int32_t n_fit, const hs_hybrid_params* hp,
                                   double* q_out, double* eps_out, double* y_out, hs_step_info* info) {
  if (!ctx || !hdm || !q_prev || !Phi || !psi || !hp || !q_out || !s) return HS_ERR_INVALID_ARG;
  if (q_out == q_prev || q_out == psi || (const void*)q_out == Phi || (q_prev2 && q_out == q_prev2))
    return ctx->fail(HS_ERR_INVALID_ARG, "q_out aliases an input");
  if (s->ctx != ctx) return HS_ERR_INVALID_ARG;
  if (ctx->p.bc != HS_BC_TRANSMISSIVE)
    return ctx->fail(HS_ERR_INVALID_ARG, "the paper's hybrid step needs a context with HS_BC_TRANSMISSIVE");
  PaperBC bc;
  HS_TRY(paper_bc(ctx, hdm, &bc));
  if (m < 1 || m > ctx->p.m_max) return ctx->fail(HS_ERR_RANK, "empty basis");
  if (hp->jmax < 1 || hp->n_orders < 0 || hp->n_orders > 4 || !(hp->rcond_fit > 0) || !(hp->eps_y >= 0))
    return HS_ERR_INVALID_ARG;
  for (int o = 0; o < hp->n_orders; ++o)
    if (hp->filter_orders[o] < 1 || hp->filter_orders[o] > 3) return HS_ERR_INVALID_ARG;
  const int prec = hp->precision;
  if (prec != HS_FP64 && prec != HS_MIXED_FP32) return HS_ERR_INVALID_ARG;
  if (s->n_s == 0) return ctx->fail(HS_ERR_RANK, "empty sampled set");
  if (n_fit < 0 || n_fit > ctx->n || (n_fit > 0 && !fit_points)) return ctx->fail(HS_ERR_INVALID_ARG, "fit points");
  // the fit's rows: every entry of the sampled cells, or the given entries
  const int* frows = n_fit > 0 ? fit_points : s->hat;
  const int nfr = n_fit > 0 ? n_fit : s->n_s;
  const int fnc = n_fit > 0 ? 1 : ctx->nc;
  hs_step_info local{};
  hs_step_info* inf = info ? info : &local;
  std::memset(inf, 0, sizeof *inf);
  inf->n_s = s->n_s;
  inf->l = ctx->ncell - s->n_s;
  double* u = ctx->u;
  double* u_next = ctx->gtmp;
  double* sm = ctx->small;
  HS_TRY(max_abs_launch(ctx, q_prev, ctx->n));
  HIP_TRY(ctx, hipMemcpyAsync(u, q_prev, ctx->n * 8, hipMemcpyDeviceToDevice, ctx->stream));
  HS_TRY(fit_factor(ctx, Phi, prec, m, frows, nfr, hp->rcond_fit, fnc));
  unsigned long long st[kStatSlots];
  HS_TRY(read_stats(ctx, st));
  const double qmax = bits_to_double(st[kStatQMax]);
  if (!std::isfinite(qmax)) return ctx->fail(HS_ERR_NONFINITE, "non-finite q_prev");
  const double tol = ctx->p.newton_rtol * std::max(1.0, qmax);
  inf->fit_rank = (int)bits_to_double(st[kStatFitRank]);
  inf->fit_cond = bits_to_double(st[kStatFitCond]);
  if (inf->fit_rank == 0) return ctx->fail(HS_ERR_RANK, "rank-zero fit");
  for (int j = 1; j <= hp->jmax; ++j) {
    HS_TRY(paper_solve(ctx, bc, u, q_prev, q_prev2, tol, s, inf));
    HS_TRY(fit_solve(ctx, Phi, prec, m, frows, nfr, u, psi, j == 1, fnc));
    // unsampled entries (the ring among them) = psi + Phi y; rho = psi + Phi y
    HS_TRY(reconstruct(ctx, Phi, prec, m, psi, sm + kSmY, s->mask, u, u_next, ctx->rho));
    std::swap(u, u_next);
    inf->subiters = j;
    HS_TRY(read_stats(ctx, st));
    const double dy = bits_to_double(st[kStatDy]);
    inf->dy_last = dy;
    if (j >= 2 && dy < hp->eps_y) break;
  }
  HIP_TRY(ctx, hipMemcpyAsync(q_out, u, ctx->n * 8, hipMemcpyDeviceToDevice, ctx->stream));
  HS_TRY(paper_filter(ctx, bc, q_out, q_prev, q_prev2, hp, inf));
  if (eps_out) {
    int nbq;
    HS_TRY(max_abs_partials(ctx, q_out, ctx->n, &nbq));
    HS_LAUNCH(ctx, indicator_kernel, blocks_for(ctx->ncell), kBlock, ctx->ncell, ctx->nc, q_out, ctx->rho,
              hp->floor_rel, (const double*)ctx->part, nbq, eps_out);
  }
  if (y_out) HIP_TRY(ctx, hipMemcpyAsync(y_out, sm + kSmY, m * 8, hipMemcpyDeviceToDevice, ctx->stream));
  return HS_OK;
}

}  // namespace hs

using namespace hs;

extern "C" {


hs_status hs_filter(hs_ctx* ctx, const double* gamma_in, const double* q_prev, const hs_hybrid_params* hp,
                    double* gamma_out, hs_step_info* info) {
  if (!ctx || !gamma_in || !q_prev || !hp || !gamma_out || gamma_out == q_prev) return HS_ERR_INVALID_ARG;
  if (hp->n_orders < 0 || hp->n_orders > 4 || hp->jfmax < 0) return HS_ERR_INVALID_ARG;
  for (int o = 0; o < hp->n_orders; ++o)
    if (hp->filter_orders[o] < 1 || hp->filter_orders[o] > 3) return HS_ERR_INVALID_ARG;
  if (info) std::memset(info, 0, sizeof *info);
  if (gamma_out != gamma_in)
    HIP_TRY(ctx, hipMemcpyAsync(gamma_out, gamma_in, ctx->n * 8, hipMemcpyDeviceToDevice, ctx->stream));
  HS_TRY(run_filter(ctx, gamma_out, q_prev, hp, info));
  return hs_sync(ctx);
}

hs_status hs_indicator_full(hs_ctx* ctx, const double* gamma, const void* Phi, const double* psi, int32_t m,
                            double floor_rel, int32_t precision, double* eps, double* y_out) {
  if (!ctx || !gamma || !Phi || !psi || !eps) return HS_ERR_INVALID_ARG;
  if (m < 1 || m > ctx->p.m_max) return HS_ERR_INVALID_ARG;
  if (precision != HS_FP64 && precision != HS_MIXED_FP32) return HS_ERR_INVALID_ARG;
  double* sm = ctx->small;
  int nb;
  HS_TRY(launch_project(ctx, Phi, precision, m, nullptr, 0, gamma, psi, nullptr, 0, &nb));
  // y = Phi^T (gamma - psi): G+ = I
  HS_LAUNCH(ctx, eye_kernel, blocks_for(m * m), kBlock, sm + kSmGp, m);
  HS_LAUNCH(ctx, project_finish_kernel, 1, 256, ctx->red, nb, pad16(m), m, sm + kSmGp, 0, sm + kSmY0, sm + kSmY,
            sm + kSmYPrev, sm + kSmMisc, 1, (unsigned long long*)nullptr);
  HS_TRY(reconstruct(ctx, Phi, precision, m, psi, sm + kSmY0, nullptr, nullptr, nullptr, ctx->rho));
  int nbq;
  HS_TRY(max_abs_partials(ctx, gamma, ctx->n, &nbq));
  HS_LAUNCH(ctx, indicator_kernel, blocks_for(ctx->ncell), kBlock, ctx->ncell, ctx->nc, gamma, ctx->rho, floor_rel,
            (const double*)ctx->part, nbq, eps);
  if (y_out) HIP_TRY(ctx, hipMemcpyAsync(y_out, sm + kSmY0, m * 8, hipMemcpyDeviceToDevice, ctx->stream));
  return hs_sync(ctx);
}

hs_status rom_hybrid_step(hs_ctx* ctx, const double* q_prev, const void* Phi, const double* psi, int32_t m,
                          const hs_samples* s, const hs_hybrid_params* hp, double* q_out, double* eps_out,
                          double* y_out, hs_step_info* info) {
  return hybrid_impl(ctx, q_prev, Phi, psi, m, s, hp, q_out, eps_out, y_out, info, nullptr, -1);
}

hs_status rom_hybrid_step_gn(hs_ctx* ctx, const double* q_prev, const double* Phi, const double* psi, int32_t m,
                             const hs_samples* s, const hs_hybrid_params* hp, double* work, double* q_out,
                             double* eps_out, double* y_out, hs_step_info* info) {
  return hybrid_gn_impl(ctx, q_prev, Phi, psi, m, s, hp, work, q_out, eps_out, y_out, info);
}

hs_status rom_hybrid_step_bdf2(hs_ctx* ctx, const hs_paper_hdm* hdm, const double* q_prev, const double* q_prev2,
                               const void* Phi, const double* psi, int32_t m, const hs_samples* s,
                               const int32_t* fit_points, int32_t n_fit, const hs_hybrid_params* hp,
                               double* q_out, double* eps_out, double* y_out, hs_step_info* info) {
  return hybrid_paper_impl(ctx, hdm, q_prev, q_prev2, Phi, psi, m, s, fit_points, n_fit, hp, q_out, eps_out, y_out,
                           info);
}

hs_status rom_hybrid_step_fit(hs_ctx* ctx, const double* q_prev, const void* Phi, const double* psi, int32_t m,
                              const hs_samples* s, const int32_t* fit_points, int32_t n_fit,
                              const hs_hybrid_params* hp, double* q_out, double* eps_out, double* y_out,
                              hs_step_info* info) {
  return hybrid_impl(ctx, q_prev, Phi, psi, m, s, hp, q_out, eps_out, y_out, info, nullptr, -1, fit_points, n_fit);
}

hs_status rom_hybrid_step_taped(hs_ctx* ctx, const double* q_prev, const void* Phi, const double* psi,
                                int32_t m, const hs_samples* s, const hs_hybrid_params* hp, double* q_out,
                                double* eps_out, hs_step_info* info, hs_htape* tape, int32_t mode) {
  if (mode != HS_TAPE_RECORD && mode != HS_TAPE_REPLAY) return HS_ERR_INVALID_ARG;
  return hybrid_impl(ctx, q_prev, Phi, psi, m, s, hp, q_out, eps_out, nullptr, info, tape, mode);
}

hs_status hs_htape_create(hs_ctx* ctx, hs_htape** out) {
  if (!ctx || !out) return HS_ERR_INVALID_ARG;
  hs_htape* t = new hs_htape();
  t->ctx = ctx;
  hs_status st = hs_samples_create(ctx, &t->s);
  if (st == HS_OK && hipMalloc((void**)&t->masks, (size_t)kMaxPasses * ctx->ncell) != hipSuccess) st = HS_ERR_OOM;
  if (st == HS_OK && hipMalloc((void**)&t->gp, (size_t)kMaxBasis * kMaxBasis * 8) != hipSuccess) st = HS_ERR_OOM;
  if (st != HS_OK) {
    hs_htape_destroy(t);
    return ctx->fail(st, "tape allocation failed");
  }
  *out = t;
  return HS_OK;
}

hs_status hs_htape_info(const hs_htape* t, int32_t* J, int32_t* npass, int32_t* passes, uint8_t* masks) {
  if (!t) return HS_ERR_INVALID_ARG;
  hs_ctx* ctx = t->ctx;
  if (!t->recorded) return ctx->fail(HS_ERR_INVALID_ARG, "tape holds no recorded step");
  if (J) *J = t->J;
  if (npass) *npass = t->npass;
  if (passes)
    for (int k = 0; k < t->npass; ++k) passes[k] = t->passes[k];
  if (masks && t->npass > 0) {
    HIP_TRY(ctx, hipMemcpyAsync(masks, t->masks, (size_t)t->npass * ctx->ncell, hipMemcpyDeviceToDevice,
                                ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  }
  return HS_OK;
}

hs_status hs_htape_samples(hs_htape* t, hs_samples** out) {
  if (!t || !out) return HS_ERR_INVALID_ARG;
  *out = t->s;
  return HS_OK;
}

hs_status hs_htape_destroy(hs_htape* t) {
  if (!t) return HS_ERR_INVALID_ARG;
  if (t->s) hs_samples_destroy(t->s);
  if (t->masks) (void)hipFree(t->masks);
  if (t->us) (void)hipFree(t->us);
  if (t->gp) (void)hipFree(t->gp);
  delete t;
  return HS_OK;
}

}  // extern "C"

// ------------------------------------------- indicator without allocation
// hs_indicator_full_noalloc keeps its working memory in one file-scope device
// array (each GPU the library runs on holds its own copy until the process
// ends).  Host code never passes the array's name to a kernel: the device
// address is looked up once per device with hipGetSymbolAddress and kept.
// Layout (doubles): projection partials (kProjBlocks x 64), the identity
// (64 x 64), y and the finish kernel's bookkeeping (4 x 64), the max-|gamma|
// partials (slot kStatQMax of a kStatSlots x kPartCap statistics block).
namespace hs {
constexpr int kProjBlocks = 512;
constexpr size_t kNoAllocPart = 0;
constexpr size_t kNoAllocEye = kNoAllocPart + (size_t)kProjBlocks * kMaxBasis;
constexpr size_t kNoAllocY = kNoAllocEye + (size_t)kMaxBasis * kMaxBasis;
constexpr size_t kNoAllocStats = kNoAllocY + 4 * kMaxBasis;
constexpr size_t kNoAllocDoubles = kNoAllocStats + (size_t)(kStatQMax + 1) * kPartCap;
constexpr int kNoAllocMaxDevices = 64;
}  // namespace hs

static __device__ __align__(256) double scratch[hs::kNoAllocDoubles];

namespace hs {
static std::mutex g_noalloc_mu;
static double* g_noalloc_ptr[kNoAllocMaxDevices] = {nullptr};

// The device address of this device's scratch array (looked up on the first
// call on each device, with that device current).
static hs_status noalloc_scratch(double** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return HS_ERR_HIP;
  if (dev < 0 || dev >= kNoAllocMaxDevices) return HS_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HS_ERR_HIP;
    g_noalloc_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_noalloc_ptr[dev];
  return HS_OK;
}

#define HS_NA_LAUNCH(stream, kernel, grid, block, ...)                               \
  do {                                                                               \
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, stream, __VA_ARGS__);     \
    if (hipGetLastError() != hipSuccess) return HS_ERR_HIP;                          \
  } while (0)

// Per-block maxima of |x| into slot kStatQMax of a statistics block (a
// maximum is exact in any order, so these equal max_abs_partials' values).
__global__ void noalloc_max_abs_kernel(const double* __restrict__ x, long long n, double* __restrict__ part) {
  __shared__ double lds[kBlock / kWave];
  double mx = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    mx = nan_max(mx, fabs(x[i]));
  mx = block_max(mx, lds);
  if (threadIdx.x == 0) stat_part(part, kStatQMax, mx);
}

template <typename TP>
static hs_status indicator_noalloc_t(hipStream_t st, double* sc, int ncell, int nc, const double* gamma,
                                     const TP* Phi, const double* psi, int m, double floor_rel, double* eps,
                                     double* y_out) {
  const long long n = (long long)nc * ncell;
  const int nb = (int)std::max<long long>(1, std::min<long long>((n + kBlock - 1) / kBlock, kProjBlocks));
  double* part = sc + kNoAllocPart;
  double* eye = sc + kNoAllocEye;
  double* y = y_out ? y_out : sc + kNoAllocY;
  double* misc = sc + kNoAllocY + kMaxBasis;
  double* stats = sc + kNoAllocStats;
  // y = Phi^T (gamma - psi): the projection partials of every block, then
  // their fixed-order sum applied to the identity (the same kernels and
  // order as hs_indicator_full)
  switch (pad16(m)) {
    case 16: HS_NA_LAUNCH(st, (project_kernel<16, TP>), nb, kBlock, Phi, n, m, nc, ncell, (const int*)nullptr, 0, gamma, psi, (const double*)nullptr, 0, part); break;
    case 32: HS_NA_LAUNCH(st, (project_kernel<32, TP>), nb, kBlock, Phi, n, m, nc, ncell, (const int*)nullptr, 0, gamma, psi, (const double*)nullptr, 0, part); break;
    case 48: HS_NA_LAUNCH(st, (project_kernel<48, TP>), nb, kBlock, Phi, n, m, nc, ncell, (const int*)nullptr, 0, gamma, psi, (const double*)nullptr, 0, part); break;
    default: HS_NA_LAUNCH(st, (project_kernel<64, TP>), nb, kBlock, Phi, n, m, nc, ncell, (const int*)nullptr, 0, gamma, psi, (const double*)nullptr, 0, part); break;
  }
  HS_NA_LAUNCH(st, eye_kernel, blocks_for(m * m), kBlock, eye, m);
  HS_NA_LAUNCH(st, project_finish_kernel, 1, 256, (const double*)part, nb, pad16(m), m, (const double*)eye, 0, y,
               misc + kMaxBasis, misc + 2 * kMaxBasis, misc, 1, (unsigned long long*)nullptr);
  const int nbq = blocks_for(n, kBlock, 1024);
  HS_NA_LAUNCH(st, noalloc_max_abs_kernel, nbq, kBlock, gamma, n, stats);
  HS_NA_LAUNCH(st, (indicator_direct_kernel<TP>), blocks_for(ncell), kBlock, ncell, nc, gamma, Phi, psi,
               (const double*)y, m, floor_rel, (const double*)stats, nbq, eps);
  return HS_OK;
}
#undef HS_NA_LAUNCH
}  // namespace hs

extern "C" hs_status hs_indicator_full_noalloc(void* hip_stream, int32_t ncell, int32_t ncomp, const double* gamma,
                                               const void* Phi, const double* psi, int32_t m, double floor_rel,
                                               int32_t precision, double* eps, double* y_out) {
  using namespace hs;
  if (!gamma || !Phi || !psi || !eps) return HS_ERR_INVALID_ARG;
  if (ncomp != 1 && ncomp != 4) return HS_ERR_INVALID_ARG;
  if (precision != HS_FP64 && precision != HS_MIXED_FP32) return HS_ERR_INVALID_ARG;
  if (!(floor_rel >= 0.0)) return HS_ERR_INVALID_ARG;
  // the scratch array is sized for m <= 64 and at most 2^31 - 1 entries
  if (m < 1 || m > kMaxBasis || ncell < 1 || (long long)ncomp * ncell >= (1LL << 31)) return HS_ERR_SHAPE;
  double* sc = nullptr;
  HS_TRY(noalloc_scratch(&sc));
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (precision == HS_MIXED_FP32)
    return indicator_noalloc_t(st, sc, ncell, ncomp, gamma, (const float*)Phi, psi, m, floor_rel, eps, y_out);
  return indicator_noalloc_t(st, sc, ncell, ncomp, gamma, (const double*)Phi, psi, m, floor_rel, eps, y_out);
}
