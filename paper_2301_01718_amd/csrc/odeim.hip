// Oversampled empirical interpolation points of a basis (eq. odeim; Alg. 1:
// P_{k+1} = ODEIM_{n_p}(Phi_{k+1})): n_p entries of the state vector whose
// rows of Phi serve the fit of eq. red_coord.
//
// The first m points are QDEIM's, the pivots of a column-pivoted QR of
// Phi^T: step j takes the row phi_i whose component orthogonal to the rows
// already taken is longest, |phi_i|^2 - sum_k (q_k^T phi_i)^2 with q_k an
// orthonormal basis of the taken rows.  Each further point maximises a lower
// bound of the smallest eigenvalue of the sampled Gram M + phi phi^T
// (M = Phi_P^T Phi_P; l_1 <= l_2 its two smallest eigenvalues, u_1 the
// eigenvector of l_1, g = l_2 - l_1):
//   gain = (g + |phi|^2 - sqrt((g + |phi|^2)^2 - 4 g (u_1^T phi)^2)) / 2,
// and (u_1^T phi)^2 when m = 1.  Ties go to the lowest index.
//
// Every step is one pass over Phi (one thread per row, the row's m entries
// in registers, a block argmax) and a one-wave pick that reduces the
// partials in a fixed order, marks the point, extends the orthonormal basis
// or the Gram, and (from the m-th point on) diagonalises the m x m Gram by
// cyclic Jacobi in LDS.  m <= 16.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "common.hpp"

namespace hs {

constexpr int kOdeimMax = 16;

// Layout of the small state (doubles) in ctx->small beyond the fit's slots.
struct OdeimState {
  double q[kOdeimMax][kOdeimMax];   // orthonormal basis of the QDEIM rows (q[k][.])
  double M[kOdeimMax][kOdeimMax];   // Gram of the taken rows
  double u1[kOdeimMax];             // eigenvector of the smallest eigenvalue
  double lam1, gap;                 // smallest eigenvalue, gap to the next (< 0: m = 1)
  int nq;                           // QDEIM rows taken
};

__device__ inline void argmax_merge(double& v, int& i, double v2, int i2) {
  if (v2 > v || (v2 == v && i2 < i)) {
    v = v2;
    i = i2;
  }
}

// Scores of every row not taken; per block (max score, its lowest index).
__global__ void __launch_bounds__(kBlock) odeim_score_kernel(const double* __restrict__ Phi, long long n, int m,
                                                             int qdeim, const OdeimState* __restrict__ st,
                                                             const uint8_t* __restrict__ taken,
                                                             double* __restrict__ pval, int* __restrict__ pidx) {
  __shared__ double q[kOdeimMax][kOdeimMax];
  __shared__ double u1[kOdeimMax];
  __shared__ double sv[kBlock / kWave];
  __shared__ int si[kBlock / kWave];
  const int nq = st->nq;
  for (int e = threadIdx.x; e < kOdeimMax * kOdeimMax; e += blockDim.x) q[e / kOdeimMax][e % kOdeimMax] = st->q[e / kOdeimMax][e % kOdeimMax];
  if (threadIdx.x < kOdeimMax) u1[threadIdx.x] = st->u1[threadIdx.x];
  __syncthreads();
  const double gap = st->gap;
  double best = -INFINITY;
  int bi = 0x7fffffff;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    if (taken[i]) continue;
    double ph[kOdeimMax];
#pragma unroll
    for (int j = 0; j < kOdeimMax; ++j) ph[j] = j < m ? Phi[(size_t)j * n + i] : 0.0;
    double nrm = 0.0;
#pragma unroll
    for (int j = 0; j < kOdeimMax; ++j) nrm += ph[j] * ph[j];
    double score;
    if (qdeim) {
      double pr = 0.0;
      for (int k = 0; k < nq; ++k) {
        double d = 0.0;
#pragma unroll
        for (int j = 0; j < kOdeimMax; ++j) d += q[k][j] * ph[j];
        pr += d * d;
      }
      score = nrm - pr;
    } else {
      double a = 0.0;
#pragma unroll
      for (int j = 0; j < kOdeimMax; ++j) a += u1[j] * ph[j];
      if (gap < 0.0) {
        score = a * a;
      } else {
        const double s = gap + nrm;
        score = 0.5 * (s - sqrt(fmax(s * s - 4.0 * gap * a * a, 0.0)));
      }
    }
    argmax_merge(best, bi, score, (int)i);
  }
  // wave then block argmax
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const double v2 = __shfl_xor(best, o, kWave);
    const int i2 = __shfl_xor(bi, o, kWave);
    argmax_merge(best, bi, v2, i2);
  }
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  if (lane == 0) {
    sv[wave] = best;
    si[wave] = bi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x / kWave); ++w) argmax_merge(best, bi, sv[w], si[w]);
    pval[blockIdx.x] = best;
    pidx[blockIdx.x] = bi;
  }
}

// One wave: reduce the partials (lanes stride the blocks, then a lane tree;
// ties to the lowest index), take the point, extend the orthonormal basis of
// the QDEIM rows or the Gram, and from the m-th point on diagonalise the Gram
// by cyclic Jacobi in LDS (each rotation's rows and columns updated by m
// lanes) for l_1, the gap and u_1.
__global__ void __launch_bounds__(kWave) odeim_pick_kernel(const double* __restrict__ Phi, long long n, int m,
                                                           int qdeim, int slot, int nb,
                                                           const double* __restrict__ pval,
                                                           const int* __restrict__ pidx, OdeimState* st,
                                                           uint8_t* __restrict__ taken, int32_t* __restrict__ points) {
  __shared__ double A[kOdeimMax][kOdeimMax + 1], V[kOdeimMax][kOdeimMax + 1];
  __shared__ double ph[kOdeimMax], rot[2];
  __shared__ int pick;
  const int t = threadIdx.x;
  double best = -INFINITY;
  int bi = 0x7fffffff;
  for (int b = t; b < nb; b += kWave) argmax_merge(best, bi, pval[b], pidx[b]);
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const double v2 = __shfl_xor(best, o, kWave);
    const int i2 = __shfl_xor(bi, o, kWave);
    argmax_merge(best, bi, v2, i2);
  }
  if (t == 0) {
    if (bi < 0 || bi >= n) bi = 0;   // no candidate left (cannot happen for n_p <= n)
    pick = bi;
    taken[bi] = 1;
    points[slot] = bi;
  }
  __syncthreads();
  const int p0 = pick;
  if (t < m) ph[t] = Phi[(size_t)t * n + p0];
  __syncthreads();
  if (qdeim && t == 0) {
    // Gram-Schmidt of the row against the basis, twice, then normalise
    double v[kOdeimMax];
    for (int j = 0; j < m; ++j) v[j] = ph[j];
    for (int pass = 0; pass < 2; ++pass)
      for (int k = 0; k < st->nq; ++k) {
        double d = 0.0;
        for (int j = 0; j < m; ++j) d += st->q[k][j] * v[j];
        for (int j = 0; j < m; ++j) v[j] -= d * st->q[k][j];
      }
    double nv = 0.0;
    for (int j = 0; j < m; ++j) nv += v[j] * v[j];
    nv = sqrt(nv);
    for (int j = 0; j < m; ++j) st->q[st->nq][j] = nv > 0.0 ? v[j] / nv : 0.0;
    st->nq += 1;
  }
  if (t < m)
    for (int j = 0; j < m; ++j) st->M[t][j] += ph[t] * ph[j];
  __syncthreads();
  if (slot + 1 < m) return;
  if (t < m)
    for (int j = 0; j < m; ++j) {
      A[t][j] = st->M[t][j];
      V[t][j] = t == j ? 1.0 : 0.0;
    }
  __syncthreads();
  // sweeps until one applies no rotation: an off-diagonal entry is rotated
  // away unless it is below 1e-16 of the geometric mean of its diagonal pair
  // (the eigenvalues then carry errors of second order in it)
  __shared__ int nrot;
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (t == 0) nrot = 0;
    __syncthreads();
    for (int p = 0; p < m - 1; ++p)
      for (int r = p + 1; r < m; ++r) {
        if (t == 0) {
          const double apr = A[p][r];
          double c = 1.0, sn = 0.0;
          if (fabs(apr) > 1e-16 * sqrt(fabs(A[p][p] * A[r][r]))) {
            const double theta = (A[r][r] - A[p][p]) / (2.0 * apr);
            const double tt = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(tt * tt + 1.0);
            sn = tt * c;
            nrot += 1;
          }
          rot[0] = c;
          rot[1] = sn;
        }
        __syncthreads();
        const double c = rot[0], sn = rot[1];
        if (sn != 0.0) {
          if (t < m) {
            const double akp = A[t][p], akr = A[t][r];
            A[t][p] = c * akp - sn * akr;
            A[t][r] = sn * akp + c * akr;
            const double vkp = V[t][p], vkr = V[t][r];
            V[t][p] = c * vkp - sn * vkr;
            V[t][r] = sn * vkp + c * vkr;
          }
          __syncthreads();
          if (t < m) {
            const double apk = A[p][t], ark = A[r][t];
            A[p][t] = c * apk - sn * ark;
            A[r][t] = sn * apk + c * ark;
          }
        }
        __syncthreads();
      }
    if (nrot == 0) break;
    __syncthreads();
  }
  if (t == 0) {
    int i1 = 0;
    for (int i = 1; i < m; ++i)
      if (A[i][i] < A[i1][i1]) i1 = i;
    double l2 = INFINITY;
    for (int i = 0; i < m; ++i)
      if (i != i1 && A[i][i] < l2) l2 = A[i][i];
    st->lam1 = A[i1][i1];
    st->gap = m > 1 ? l2 - A[i1][i1] : -1.0;
    for (int j = 0; j < m; ++j) st->u1[j] = V[j][i1];
  }
}

__global__ void odeim_init_kernel(OdeimState* st, uint8_t* taken, long long n) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) taken[i] = 0;
  if (i < kOdeimMax * kOdeimMax) {
    st->q[i / kOdeimMax][i % kOdeimMax] = 0.0;
    st->M[i / kOdeimMax][i % kOdeimMax] = 0.0;
  }
  if (i < kOdeimMax) st->u1[i] = 0.0;
  if (i == 0) {
    st->nq = 0;
    st->lam1 = 0.0;
    st->gap = -1.0;
  }
}

// ODEIM state after the fit's slots of ctx->small (16 x 64 x 64 doubles).
constexpr size_t kSmOdeim = 15 * kMaxBasis * kMaxBasis;

}  // namespace hs

using namespace hs;

extern "C" {

hs_status hs_odeim(hs_ctx* ctx, const double* Phi, int32_t m, int32_t n_p, int32_t* points) {
  if (!ctx || !Phi || !points) return HS_ERR_INVALID_ARG;
  if (m < 1 || m > kOdeimMax || m > ctx->p.m_max)
    return ctx->fail(HS_ERR_INVALID_ARG, "hs_odeim: 1 <= m <= min(16, m_max)");
  if (n_p < m || n_p > ctx->n) return ctx->fail(HS_ERR_INVALID_ARG, "hs_odeim: m <= n_p <= N");
  static_assert(sizeof(OdeimState) <= kMaxBasis * kMaxBasis * sizeof(double), "ODEIM state exceeds its slot");
  OdeimState* st = reinterpret_cast<OdeimState*>(ctx->small + kSmOdeim);
  uint8_t* taken = reinterpret_cast<uint8_t*>(ctx->ibuf);   // N bytes (ibuf holds 4 (ncell + 8192) >= N)
  double* pval = ctx->red;
  int* pidx = reinterpret_cast<int*>(ctx->red + kRedBlocks);
  const long long n = ctx->n;
  const int nb = blocks_for(n, kBlock, kRedBlocks);
  HS_LAUNCH(ctx, odeim_init_kernel, blocks_for(std::max<long long>(n, kOdeimMax * kOdeimMax)), kBlock, st, taken,
            n);
  for (int k = 0; k < n_p; ++k) {
    const int qd = k < m ? 1 : 0;
    HS_LAUNCH(ctx, odeim_score_kernel, nb, kBlock, Phi, n, (int)m, qd, (const OdeimState*)st,
              (const uint8_t*)taken, pval, pidx);
    HS_LAUNCH(ctx, odeim_pick_kernel, 1, kWave, Phi, n, (int)m, qd, k, nb, (const double*)pval, (const int*)pidx,
              st, taken, points);
  }
  return HS_OK;
}

}  // extern "C"
