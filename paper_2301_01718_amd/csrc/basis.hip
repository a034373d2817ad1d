// POD basis update (A9): reference state and POD_m of the snapshot window
// (eq. mean, eq. pod; the basis-update branch of Alg. 1).
//
// The first pass over the window forms, row by row, both window means (the
// centring state psi_k over the first w snapshots and psi_{k+1} over the last
// w), the centred row of X = [gamma_j - psi_k] and accumulates the Gram
// matrix X^T X on FP64 MFMA.  That Gram only serves as a preconditioner: its
// eigenvalues carry about eps sigma_0^2 of absolute error, so singular values
// below about 1e-8 sigma_0 (the POD cut) have no digits in it.  A shifted
// pivoted Cholesky factor C1 of it is inverted, and the second pass forms the
// Gram of X C1^-1 from the data, whose truncated pivoted Cholesky factor R2
// gives X = Q R, R = R2 C1, with R accurate to the rounding of X itself
// (X not squared).  One-sided Jacobi on R^T gives the right singular vectors
// V and sigma; the third pass forms Phi = X V_m diag(1/sigma_m), the left
// singular vectors, again on MFMA.  Traffic: three reads of the window and
// one write of Phi.
// Kernels using the window staging must run with 256 threads (four waves).
#include "dense.hpp"

#include <algorithm>
#include <cstring>

namespace hs {

// Wave-private window chunks.  A wave owns 16 consecutive rows: lane l holds
// row l % 16 of the snapshots l / 16, l / 16 + 4, ... (at most 17 per lane),
// so each load instruction reads a 128-byte run of four snapshots.  The
// window means of a row are lane-group sums combined by two fixed shuffles;
// the centred rows go to a wave-private LDS region (16 rows), from which the
// MFMA operands are read.  There is no workgroup barrier in the loop, and the
// small register footprint lets about six waves per SIMD hide the latency.
constexpr int kWaveRows = 16;                 // rows per wave chunk

// Snapshot pointers come from a table, so the compiler cannot tell they
// address global memory and would use flat loads, which also count against
// the LDS wait counter.  The cast makes them global loads.
typedef const __attribute__((address_space(1))) double* gptr_t;

// The window's snapshot addresses, passed by value as a kernel argument (no
// upload of a device table before the launch).
struct SnapTable {
  const double* p[kMaxBasis + 1];
};

template <int PER>
struct LaneSnaps {
  gptr_t p[PER];   // this lane's snapshots l / 16 + 4 i (clamped to the last one)
  double v[PER];
};

template <int PER>
__device__ inline void lane_snaps_init(const SnapTable& snaps, int nsnap, LaneSnaps<PER>& L) {
  const int g = (threadIdx.x % kWave) / 16;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int j = g + 4 * i;
    L.p[i] = (gptr_t)snaps.p[j < nsnap ? j : nsnap - 1];
  }
}

// Loads this lane's values of its row (branch-free: all loads in flight
// together; rows past n read row n - 1, snapshots past nsnap the last one,
// both zeroed afterwards).
template <int PER>
__device__ inline void lane_snaps_load(LaneSnaps<PER>& L, int nsnap, long long n, long long row) {
  const int g = (threadIdx.x % kWave) / 16;
  const bool ok = row < n;
  const long long rr = ok ? row : n - 1;
#pragma unroll
  for (int i = 0; i < PER; ++i) L.v[i] = L.p[i][rr];
#pragma unroll
  for (int i = 0; i < PER; ++i) L.v[i] = (ok && g + 4 * i < nsnap) ? L.v[i] : 0.0;
}

// Window means with the sum correctly rounded (reproducible to the bit by
// any implementation that rounds the sum correctly, whatever its order):
// each lane keeps its values' sum as an unevaluated pair hi + lo with Knuth's
// error-free TwoSum, the four lane groups of a row combine their pairs, and
// hi + lo is rounded once.  The pair is exact as long as the accumulated low
// parts add without rounding (values of a row within a few binades of each
// other); otherwise it differs from the exact sum by about eps^2 of it, which
// changes the rounded result only when the exact sum lies that close to a
// rounding boundary.
__device__ inline void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Pair sum over the four lane groups of a row.  Each combination is
// symmetric in its two operands (the rounded sum and its exact error do not
// depend on the order, and lo_a + lo_b == lo_b + lo_a), so all four groups
// hold the same bits.
__device__ inline double group_sum_exact(double hi, double lo) {
#pragma unroll
  for (int o = 16; o <= 32; o *= 2) {
    const double h2 = __shfl_xor(hi, o, kWave), l2 = __shfl_xor(lo, o, kWave);
    double s, e;
    two_sum(hi, h2, s, e);
    hi = s;
    lo = (lo + l2) + e;
  }
  return hi + lo;
}

// The row's centring state (mean of the first w snapshots); psi_new (mean of
// the last w) is written by the lanes of group 0.
template <int PER>
__device__ inline double lane_snaps_centre(const LaneSnaps<PER>& L, int nsnap, int w, long long row, long long n,
                                           double* __restrict__ psi_new) {
  const int g = (threadIdx.x % kWave) / 16;
  const int off = nsnap - w;
  double ch = 0.0, cl = 0.0, nh = 0.0, nl = 0.0;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int j = g + 4 * i;
    double e;
    two_sum(ch, j < w ? L.v[i] : 0.0, ch, e);
    cl += e;
    two_sum(nh, (j >= off && j < nsnap) ? L.v[i] : 0.0, nh, e);
    nl += e;
  }
  const double c = group_sum_exact(ch, cl);
  const double nw = group_sum_exact(nh, nl);
  if (psi_new && g == 0 && row < n) psi_new[row] = nw / (double)w;
  return c / (double)w;
}

// X[r][j - off] = v_j - c into the wave's region (kWaveRows x ldx).  Values
// with no column (j < off, j >= nsnap) go to the spare column wp, which no
// product reads; columns w .. wp - 1 are zeroed once per kernel.
template <int PER>
__device__ inline void lane_snaps_store(const LaneSnaps<PER>& L, double c, int nsnap, int w, int wp, double* xs,
                                        int ldx) {
  const int lane = threadIdx.x % kWave, g = lane / 16, r = lane % 16;
  const int off = nsnap - w;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int j = g + 4 * i;
    const int col = (j >= off && j < nsnap) ? j - off : wp;
    xs[r * ldx + col] = L.v[i] - c;
  }
}

// Orders this wave's LDS accesses around its region (the region is private
// to the wave, whose LDS instructions execute in order; this stops the
// compiler from moving them across).
__device__ inline void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Window Gram G = X^T X (upper tiles ti <= tj of 16 x 16) and psi_new.  Each
// wave accumulates its chunks' tiles in registers; the four waves' tiles are
// summed in a fixed order into the block partial part[blockIdx.x] (wp x wp).
// Block: 4 waves; dynamic LDS: 4 regions of kWaveRows x (wp + 1) (the cross-
// wave sum reuses them at the end).
template <int NS>
__global__ void __launch_bounds__(256) window_gram_kernel(const SnapTable snaps, int nsnap,
                                                          int w, long long n, int wp, double* __restrict__ psi_new,
                                                          double* __restrict__ part) {
  extern __shared__ double sh[];
  constexpr int NT = (NS - 1) / 16;              // tile rows of the padded Gram
  constexpr int NTILES = NT * (NT + 1) / 2;
  constexpr int PER = (NS + 3) / 4;
  static_assert(NTILES * 256 <= 4 * kWaveRows * NS, "the cross-wave sum reuses the regions");
  const int ldx = wp + 1;
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  double* xs = sh + wv * kWaveRows * ldx;
  for (int e = lane; e < kWaveRows * ldx; e += kWave) xs[e] = 0.0;
  double4_t acc[NTILES];
#pragma unroll
  for (int t = 0; t < NTILES; ++t) acc[t] = (double4_t){0.0, 0.0, 0.0, 0.0};
  LaneSnaps<PER> L;
  lane_snaps_init<PER>(snaps, nsnap, L);
  const long long nchunks = (n + kWaveRows - 1) / kWaveRows;
  const long long nwaves = gridDim.x * 4LL;
  for (long long ch = blockIdx.x * 4LL + wv; ch < nchunks; ch += nwaves) {
    const long long row = ch * kWaveRows + lane % 16;
    lane_snaps_load<PER>(L, nsnap, n, row);
    const double c = lane_snaps_centre<PER>(L, nsnap, w, row, n, psi_new);
    wave_lds_fence();
    lane_snaps_store<PER>(L, c, nsnap, w, wp, xs, ldx);
    wave_lds_fence();
    // per k-step the NT column blocks x_t = X[k][16 t + l % 16] serve as
    // both operands: A = X^T (A[r][k] = X[k][16 ti + r]), B[k][c] = X[k][16 tj + c];
    // the tiles of a k-step are independent, the k-steps are not unrolled
    // (fewer live registers, more resident waves)
#pragma unroll 1
    for (int k0 = 0; k0 < kWaveRows; k0 += 4) {
      const int k = k0 + lane / 16;
      double x[NT];
#pragma unroll
      for (int tb = 0; tb < NT; ++tb) x[tb] = xs[k * ldx + tb * 16 + lane % 16];
      int t = 0;
#pragma unroll
      for (int ti = 0; ti < NT; ++ti)
#pragma unroll
        for (int tj = ti; tj < NT; ++tj, ++t) acc[t] = mfma_f64(x[ti], x[tj], acc[t]);
    }
  }
  // rows past n were zeroed and centred with their (zero) mean: they add nothing
  __syncthreads();
  double* red = sh;
  for (int q = 0; q < 4; ++q) {
    if (wv == q) {
#pragma unroll
      for (int t = 0; t < NTILES; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int e = t * 256 + i * kWave + lane;
          red[e] = q == 0 ? acc[t][i] : red[e] + acc[t][i];
        }
    }
    __syncthreads();
  }
  double* out = part + (size_t)blockIdx.x * wp * wp;
  for (int e = threadIdx.x; e < NTILES * 256; e += blockDim.x) {
    const int t = e / 256, i = (e % 256) / kWave, l = e % kWave;
    int ti = 0, tt = t;
    while (tt >= NT - ti) {
      tt -= NT - ti;
      ++ti;
    }
    const int tj = ti + tt;
    const int r = ti * 16 + l / 16 + 4 * i, cc = tj * 16 + l % 16;
    out[r * wp + cc] = red[e];
  }
}

// Sum over each aligned group of 8 lanes, in every lane of the group, by DPP
// moves (quad xor 1, quad xor 2, half-row mirror): register-to-register,
// without the LDS round trip of a lane shuffle.
template <int CTRL>
__device__ inline double dpp_double(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ inline double group8_sum(double x) {
  x += dpp_double<0xB1>(x);    // quad_perm [1, 0, 3, 2]
  x += dpp_double<0x4E>(x);    // quad_perm [2, 3, 0, 1]
  x += dpp_double<0x141>(x);   // row_half_mirror: lane i <-> 7 - i within 8
  return x;
}

template <int CTRL>
__device__ inline int dpp_int(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
}

// Largest v over the wave with its lane's index id (ties to the lower id),
// returned in every lane: a butterfly within each row of 16 lanes by DPP
// moves (quad xor 1, quad xor 2, half-row mirror, row mirror), then the four
// row results read as uniform values.
__device__ inline double wave_argmax(double v, int id, int& arg) {
#define HS_ARGMAX_STEP(CTRL)                                  \
  {                                                           \
    const double ov = dpp_double<CTRL>(v);                    \
    const int oi = dpp_int<CTRL>(id);                         \
    if (ov > v || (ov == v && oi < id)) { v = ov; id = oi; }  \
  }
  HS_ARGMAX_STEP(0xB1)
  HS_ARGMAX_STEP(0x4E)
  HS_ARGMAX_STEP(0x141)
  HS_ARGMAX_STEP(0x140)
#undef HS_ARGMAX_STEP
  double best = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 0),
                                 __builtin_amdgcn_readlane(__double2loint(v), 0));
  int bi = __builtin_amdgcn_readlane(id, 0);
#pragma unroll
  for (int r = 1; r < 4; ++r) {
    const double rv = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 16 * r),
                                       __builtin_amdgcn_readlane(__double2loint(v), 16 * r));
    const int ri = __builtin_amdgcn_readlane(id, 16 * r);
    if (rv > best || (rv == best && ri < bi)) { best = rv; bi = ri; }
  }
  arg = bi;
  return best;
}

// Pivoted Cholesky of the symmetric w x w matrix A (stride lda, w <= 64):
// A = P L L^T P^T + S, stopped once the largest remaining diagonal entry is at
// most tol (S is what remains).  Right-looking, block parallel: per step one
// wave picks the pivot (the largest remaining diagonal, ties to the lowest
// index), every row forms its multiplier l_i = A[i][p] / sqrt(A[p][p]) (the
// multipliers go to L in the original row order), and the block subtracts
// l l^T from the trailing matrix in place; three barriers per step.  Outputs:
// L (zeroed by the caller) with rows in pivot order (row q <-> index
// perm[q]) and columns 0 .. rank - 1; perm is a full permutation (rows never
// pivoted follow in increasing index).  A is overwritten.  Every thread of
// the block (256 threads) calls it; buf holds 2 * kMaxBasis doubles of LDS.
__device__ __forceinline__ void block_pivoted_cholesky(double* A, int lda, int w, double tol, double* L,
                                                       double* buf, int* perm, int* rank) {
  const int t = threadIdx.x;
  __shared__ int s_piv, s_done[kMaxBasis];
  __shared__ double s_best;
  if (t < kMaxBasis) s_done[t] = t >= w;
  __syncthreads();
  int k = 0;
  for (; k < w; ++k) {
    if (t < kWave) {
      int p;
      const double best = wave_argmax(s_done[t] ? -INFINITY : A[t * lda + t], t, p);
      if (t == 0) {
        s_piv = p;
        s_best = best;
      }
    }
    __syncthreads();
    const int p = s_piv;
    const double best = s_best;
    if (!(best > tol)) break;
    const double lkk = sqrt(best);
    if (t < w) {
      const double li = s_done[t] ? 0.0 : (t == p ? lkk : A[t * lda + p] / lkk);
      buf[t] = li;
      L[t * lda + k] = li;
    }
    __syncthreads();
    // rows t / 64, t / 64 + 4, ..., column t % 64 (no integer division by w)
    // (unrolled, so that every row's loads are in flight together)
    if ((t & 63) < w) {
      const int j = t & 63;
      const double lj = buf[j];
#pragma unroll
      for (int u = 0; u < kMaxBasis / 4; ++u) {
        const int i = (t >> 6) + 4 * u;
        if (i < w) A[i * lda + j] -= buf[i] * lj;
      }
    }
    if (t == 0) {
      s_done[p] = 1;
      perm[k] = p;
    }
    __syncthreads();
  }
  // the rows never pivoted take the remaining positions in index order
  if (t < kWave) {
    const bool rest = t < w && !s_done[t];
    const unsigned long long mask = __ballot(rest);
    if (rest) perm[k + __popcll(mask & ((1ull << t) - 1ull))] = t;
  }
  __syncthreads();
  // rows of L into pivot order (through registers: at most 16 entries per thread)
  const int r = k;
  const int c = t & 63;
  double tmp[kMaxBasis / 4];
#pragma unroll
  for (int u = 0; u < kMaxBasis / 4; ++u) {
    const int q = (t >> 6) + 4 * u;
    tmp[u] = (q < w && c < r) ? L[perm[q] * lda + c] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kMaxBasis / 4; ++u) {
    const int q = (t >> 6) + 4 * u;
    if (q < w && c < r) L[q * lda + c] = tmp[u];
  }
  if (t == 0) *rank = r;
  __syncthreads();
}

// 1/sqrt(x) for x > 1e-290 from the hardware estimate and two Newton steps
// (the library form also rescales denormals and handles infinities); the
// rotations below need c^2 (1 + t^2) = 1 to rounding, not a correctly
// rounded square root.
__device__ inline double rsqrt_newton(double x) {
#pragma clang fp contract(fast)
  double r = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  r = r * (1.5 - hx * r * r);
  r = r * (1.5 - hx * r * r);
  return r;
}

// 1/x from the hardware estimate and two Newton steps (x > 1e-290).
__device__ inline double rcp_newton(double x) {
#pragma clang fp contract(fast)
  double r = __builtin_amdgcn_rcp(x);
  r = r * (2.0 - x * r);
  r = r * (2.0 - x * r);
  return r;
}

// One-sided Jacobi on the columns of B (w rows x r columns; column p at
// B[p * ldb], rows contiguous): rotate
// column pairs until they are orthogonal, so that B W = U Sigma with U the
// left singular vectors of B and Sigma its singular values (the column norms
// afterwards).  Pairs are scheduled round robin; each pair is one group of 8
// lanes (dot products reduced by DPP moves), one barrier per round.  A pair is
// rotated when |b_p.b_q| > sqrt(w) eps |b_p||b_q| (the rounding level of a
// length-w dot product); sweeps stop once no pair exceeds w eps, so rounding
// noise cannot keep them going.  Block of 256 threads (up to 32 pairs).  With
// ldb = 8 (mod 16) doubles a group's eight lanes read one half of the LDS
// banks, the half set by the parity of its column.
template <int NR>
__device__ __forceinline__ void block_jacobi_columns(double* B, int ldb, int w, int r, int* sched, int* rotated_p) {
  const int t = threadIdx.x;
  const double tol_rot = sqrt((double)w) * 2.2e-16, tol_conv = (double)w * 2.2e-16;
  const int np = (r + 1) & ~1;
  const int P = np / 2;
  const int grp = t / 8, gl = t % 8;
  int& rotated = *rotated_p;
  // the round-robin schedule, once (sched: LDS of (kMaxBasis - 1) kMaxBasis / 2
  // ints): round rd pairs (p, q) of group grp
  for (int e = t; e < (np - 1) * P; e += blockDim.x) {
    const int rd = e / P, g = e % P;
    int p, q;
    if (g == 0) {
      p = rd % (np - 1);
      q = np - 1;
    } else {
      p = (rd + g) % (np - 1);
      q = (rd - g + (np - 1)) % (np - 1);
    }
    if (p > q) { const int x = p; p = q; q = x; }
    sched[e] = p | (q << 8);
  }
  __syncthreads();
  for (int sweep = 0; sweep < 60 && r > 1; ++sweep) {
    if (t == 0) rotated = 0;
    __syncthreads();
    for (int rd = 0; rd < np - 1; ++rd) {
      if (grp < P) {
        const int pq = sched[rd * P + grp];
        const int p = pq & 0xFF, q = pq >> 8;
        if (q < r) {
          // rows gl, gl + 8, ... (8 NR >= w rows: rows past w are zero, so
          // the loads and stores need no branch and are all in flight together)
          double xs[NR], ys[NR];
#pragma unroll
          for (int i = 0; i < NR; ++i) {
            const int k = gl + 8 * i;
            xs[i] = B[p * ldb + k];
            ys[i] = B[q * ldb + k];
          }
          double aa = 0.0, bb = 0.0, gg = 0.0;
#pragma unroll
          for (int i = 0; i < NR; ++i) {
            aa += xs[i] * xs[i];
            bb += ys[i] * ys[i];
            gg += xs[i] * ys[i];
          }
          aa = group8_sum(aa);
          bb = group8_sum(bb);
          gg = group8_sum(gg);
          // rotation when |g| > tol sqrt(a b), tested on squares; with
          // d = b - a, e = 2 g: t = sign(d) e / (|d| + sqrt(d^2 + e^2)) (the
          // smaller root of t^2 + 2 (d / e) t - 1 = 0), c = 1 / sqrt(1 + t^2)
          const double ab = aa * bb;
          if (aa > 0.0 && bb > 0.0 && gg * gg > tol_rot * tol_rot * ab) {
            const double dd = bb - aa, ee = 2.0 * gg;
            const double x2 = dd * dd + ee * ee;
            double tt, c;
            if (x2 > 1e-290 && x2 < 1e290) {
              const double h = x2 * rsqrt_newton(x2);
              tt = (dd >= 0.0 ? ee : -ee) * rcp_newton(fabs(dd) + h);
              c = rsqrt_newton(1.0 + tt * tt);
            } else {
              tt = (dd >= 0.0 ? ee : -ee) / (fabs(dd) + sqrt(x2));
              c = rsqrt(1.0 + tt * tt);
            }
            const double sn = c * tt;
#pragma unroll
            for (int i = 0; i < NR; ++i) {
              const int k = gl + 8 * i;
              B[p * ldb + k] = c * xs[i] - sn * ys[i];
              B[q * ldb + k] = sn * xs[i] + c * ys[i];
            }
            if (gl == 0 && gg * gg > tol_conv * tol_conv * ab) rotated = 1;
          }
        }
      }
      __syncthreads();
    }
    if (!rotated) break;
    __syncthreads();
  }
}

// The thin SVD of the window deviations X (N x w) is taken from a triangular
// factor R with R^T R = X^T X up to rounding of X itself (X = Q R, Q not
// formed), in two window passes:
//  stage 1: the window Gram G1 = X^T X (first pass) is factored by pivoted
//           Cholesky, stopped at the shift s1 = kShift1 trace(G1); the
//           remaining diagonal is set to sqrt(s1) (the factor is completed to
//           an invertible C1 = U1 P^T, U1 upper triangular).  C1 only has to
//           precondition X: the directions whose energy lies below s1 (where
//           G1 carries no digits) are scaled up to O(1) instead of dropped.
//  stage 2: the Gram of Y = X C1^-1 is formed from the data (second pass,
//           X C1^-1 computed on the fly), factored by pivoted Cholesky with
//           rank truncation at kTrunc2 trace(G2): Y = Q2 R2 + (dropped noise),
//           so X = Q2 R with R = R2 C1.
// The singular values of X above sqrt(s1) keep a relative accuracy of about
// eps (the directions in Y are O(1)); below it, of about eps s1 / sigma^2,
// which at the POD cut (sigma = 1e-8 sigma_0) is about 1e-10 relative.  A
// Gram alone resolves sigma only down to about sqrt(eps) sigma_0.
constexpr double kShift1 = 1e-13;
constexpr double kTrunc2 = 1e-15;

// Stage 1 (one block of 256 threads): C1 (w x w, row stride kMaxBasis) and its
// inverse T1 = P U1^-1 (wp x wp, zero padded, the operand of the second pass).
__global__ void __launch_bounds__(256) basis_prec_kernel(const double* __restrict__ G, int w, int wp,
                                                        double* __restrict__ T1, double* __restrict__ C1) {
  // one workgroup on a latency-bound chain, sharing its compute unit with the
  // main stream's kernels: its waves take issue priority there
  __builtin_amdgcn_s_setprio(3);
  constexpr int lda = kMaxBasis + 1;
  __shared__ double A[kMaxBasis * lda];   // G1, then the columns of U1^-1
  __shared__ double L[kMaxBasis * lda];   // completed Cholesky factor L1 = U1^T (pivot order)
  __shared__ double buf[2 * kMaxBasis];
  __shared__ int perm[kMaxBasis];
  __shared__ int rank;
  __shared__ double s1;
  const int t = threadIdx.x, nt = blockDim.x;
  if ((t & 63) < w)
    for (int i = t >> 6; i < w; i += nt >> 6) A[i * lda + (t & 63)] = G[i * w + (t & 63)];
  for (int e = t; e < kMaxBasis * lda; e += nt) L[e] = 0.0;
  __syncthreads();
  if (t == 0) {
    double tr = 0.0;
    for (int i = 0; i < w; ++i) tr += fabs(A[i * lda + i]);
    s1 = tr > 0.0 ? kShift1 * tr : 1.0;   // an all-zero window: any invertible C1 will do
  }
  __syncthreads();
  block_pivoted_cholesky(A, lda, w, s1, L, buf, perm, &rank);
  const int r = rank;
  for (int k = r + t; k < w; k += nt) L[k * lda + k] = sqrt(s1);
  __syncthreads();
  // U1^-1 by right-looking back substitution on all columns at once: U1 X = I
  // with U1[i][k] = L[k][i]; X builds up in A (row i final once step i has
  // divided it by U1[i][i], rows above i updated by U1[k][i] X[i][.])
  if ((t & 63) < w)
    for (int i = t >> 6; i < w; i += nt >> 6) A[i * lda + (t & 63)] = i == (t & 63) ? 1.0 : 0.0;
  __syncthreads();
  for (int i = w - 1; i >= 0; --i) {
    if (t >= i && t < w) A[i * lda + t] /= L[i * lda + i];
    __syncthreads();
    // rows t / 64, t / 64 + 4, ... < i, column i + t % 64 (no integer division)
    const int c = i + (t & 63);
    if (c < w) {
      const double xc = A[i * lda + c];
#pragma unroll
      for (int u = 0; u < kMaxBasis / 4; ++u) {
        const int k = (t >> 6) + 4 * u;
        if (k < i) A[k * lda + c] -= L[i * lda + k] * xc;
      }
    }
    __syncthreads();
  }
  // T1[perm[i]][c] = (U1^-1)[i][c]; C1[i][perm[k]] = U1[i][k] = L[k][i]
  __shared__ int iperm[kMaxBasis];
  if (t < w) iperm[perm[t]] = t;
  __syncthreads();
  for (int e = t; e < wp * wp; e += nt) {
    const int rr = e / wp, c = e % wp;
    const int i = rr < w ? iperm[rr] : w;
    T1[e] = (c < w && i <= c) ? A[i * lda + c] : 0.0;
  }
  for (int e = t; e < w * w; e += nt) {
    const int i = e / w, c = e % w;
    C1[i * kMaxBasis + perm[c]] = c >= i ? L[c * lda + i] : 0.0;
  }
}

// Stage 2 and the small SVD (one block of 256 threads): R = R2 C1 from the
// truncated pivoted Cholesky of G2, then one-sided Jacobi on the columns of
// R^T (w x r2): R^T W = V Sigma, V the right singular vectors of R and so of
// X, Sigma its singular values.  Outputs sigma (w, descending, zeros past
// r2), m_eff = #{i < m : sigma_i > tau sigma_0} and the formation matrix
// T = V_m diag(1/sigma_m) (w x mp, zero padded), each column's sign making
// the largest-magnitude entry of v_i positive (lowest index on ties).
__global__ void __launch_bounds__(256) basis_svd_kernel(const double* __restrict__ G2,
                                                       const double* __restrict__ C1, int w, int m,
                                                       double tau, double* __restrict__ sigma,
                                                       double* __restrict__ T, int mp,
                                                       int* __restrict__ m_eff_out) {
  __builtin_amdgcn_s_setprio(3);   // as in the preconditioner kernel
  constexpr int lda = kMaxBasis + 1;
  constexpr int ldb = kMaxBasis + 8;
  __shared__ double A[kMaxBasis * ldb];   // G2 (stride lda), then R by rows (the columns of R^T, stride ldb)
  __shared__ double L[kMaxBasis * lda];   // pivoted Cholesky factor of G2, then V
  __shared__ double Cs[kMaxBasis * kMaxBasis];   // C1 (its rows are read in pivot order)
  __shared__ double d[2 * kMaxBasis], lam[kMaxBasis];
  __shared__ int perm[kMaxBasis], order[kMaxBasis];
  __shared__ int sched[(kMaxBasis - 1) * (kMaxBasis / 2)];
  __shared__ int rank, meff, rotated;
  __shared__ double tol;
  const int t = threadIdx.x, nt = blockDim.x;
  for (int e = t; e < kMaxBasis * lda; e += nt) L[e] = 0.0;
  for (int e = t; e < w * kMaxBasis; e += nt) Cs[e] = C1[e];
  if ((t & 63) < w)
    for (int i = t >> 6; i < w; i += nt >> 6) A[i * lda + (t & 63)] = G2[i * w + (t & 63)];
  __syncthreads();
  if (t == 0) {
    double tr = 0.0;
    for (int i = 0; i < w; ++i) tr += fabs(A[i * lda + i]);
    tol = kTrunc2 * tr;
  }
  __syncthreads();
  block_pivoted_cholesky(A, lda, w, tol, L, d, perm, &rank);
  const int r = rank;
  for (int e = t; e < kMaxBasis * ldb; e += nt) A[e] = 0.0;   // rows past w of R^T stay zero
  __syncthreads();
  // R[i][j] = sum_k R2[i][k] C1[perm[k]][j], R2[i][k] = L2[k][i] (zero for
  // k < i and for i >= r), on MFMA in 16 x 16 tiles; row i of R is column i
  // of R^T, stored at A[i * ldb]
  {
    const int lane = t % kWave, wv = t / kWave;
    const int nti = (r + 15) / 16, ntj = (w + 15) / 16;
    for (int tt = wv; tt < nti * ntj; tt += nt / kWave) {
      const int ti = tt / ntj, tj = tt % ntj;
      double4_t acc = (double4_t){0.0, 0.0, 0.0, 0.0};
      for (int k0 = 0; k0 < w; k0 += 4) {
        const int k = k0 + lane / 16;
        const int i = ti * 16 + lane % 16, j = tj * 16 + lane % 16;
        const double av = k < w ? L[k * lda + i] : 0.0;
        const double bv = (k < w && j < w) ? Cs[perm[k] * kMaxBasis + j] : 0.0;
        acc = mfma_f64(av, bv, acc);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = ti * 16 + lane / 16 + 4 * q, j = tj * 16 + lane % 16;
        if (i < r && j < w) A[i * ldb + j] = acc[q];
      }
    }
  }
  __syncthreads();
  switch ((w + 7) / 8) {
    case 1: block_jacobi_columns<1>(A, ldb, w, r, sched, &rotated); break;
    case 2: block_jacobi_columns<2>(A, ldb, w, r, sched, &rotated); break;
    case 3: block_jacobi_columns<3>(A, ldb, w, r, sched, &rotated); break;
    case 4: block_jacobi_columns<4>(A, ldb, w, r, sched, &rotated); break;
    case 5: block_jacobi_columns<5>(A, ldb, w, r, sched, &rotated); break;
    case 6: block_jacobi_columns<6>(A, ldb, w, r, sched, &rotated); break;
    case 7: block_jacobi_columns<7>(A, ldb, w, r, sched, &rotated); break;
    default: block_jacobi_columns<8>(A, ldb, w, r, sched, &rotated); break;
  }
  // squared singular values: column norms, in descending order (stable rank sort)
  if (t < r) {
    double s2 = 0.0;
    for (int k = 0; k < w; ++k) s2 += A[t * ldb + k] * A[t * ldb + k];
    d[t] = s2;
  }
  __syncthreads();
  if (t < r) {
    const double li = d[t];
    int rk = 0;
    for (int j = 0; j < r; ++j) rk += (d[j] > li) || (d[j] == li && j < t);
    lam[rk] = li;
    order[rk] = t;
  }
  __syncthreads();
  if (t == 0) {
    const double s0 = r > 0 ? sqrt(fmax(lam[0], 0.0)) : 0.0;
    int me = 0;
    for (int i = 0; i < w; ++i) {
      const double si = i < r ? sqrt(fmax(lam[i], 0.0)) : 0.0;
      sigma[i] = si;
      if (i < m && s0 > 0.0 && si > tau * s0) me = i + 1;
    }
    meff = me;
    *m_eff_out = me;
  }
  __syncthreads();
  // V[:, i] = (R^T W)[:, order[i]] / sigma_i
  for (int e = t; e < w * meff; e += nt) {
    const int row = e / meff, i = e % meff;
    L[row * lda + i] = A[order[i] * ldb + row] / sqrt(lam[i]);
  }
  __syncthreads();
  for (int i = t; i < mp; i += nt) {
    if (i < meff) {
      int best = 0;
      double bv = -1.0;
      for (int rr = 0; rr < w; ++rr) {
        const double a = fabs(L[rr * lda + i]);
        if (a > bv) { bv = a; best = rr; }
      }
      const double sg = L[best * lda + i] >= 0.0 ? 1.0 : -1.0;
      const double inv = sg / sqrt(lam[i]);
      for (int rr = 0; rr < kMaxBasis; ++rr) T[rr * mp + i] = rr < w ? L[rr * lda + i] * inv : 0.0;
    } else {
      for (int rr = 0; rr < kMaxBasis; ++rr) T[rr * mp + i] = 0.0;
    }
  }
}

// Second window pass: the Gram of Y = X T1 (T1 = C1^-1, wp x wp), X centred
// on the fly as in the first pass.  Per wave chunk: Y = X T1 on MFMA (as in
// the formation pass), Y back into the wave's LDS region in place of X, then
// Y^T Y accumulated as in the first pass.  Block: 4 waves; dynamic LDS: T1
// (wp x (wp + 1)), then 4 regions of kWaveRows x (wp + 1).
template <int NS>
__global__ void __launch_bounds__(256) window_pgram_kernel(const SnapTable snaps, int nsnap, int w, long long n,
                                                           const double* __restrict__ T1, int wp,
                                                           double* __restrict__ part) {
  extern __shared__ double sh[];
  constexpr int NT = (NS - 1) / 16;
  constexpr int NTILES = NT * (NT + 1) / 2;
  constexpr int PER = (NS + 3) / 4;
  const int ldx = wp + 1, ldt = wp + 1;
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  double* Ts = sh;
  double* xs = sh + wp * ldt + wv * kWaveRows * ldx;
  for (int e = threadIdx.x; e < wp * wp; e += blockDim.x) Ts[(e / wp) * ldt + e % wp] = T1[e];
  for (int e = lane; e < kWaveRows * ldx; e += kWave) xs[e] = 0.0;
  __syncthreads();
  double4_t acc[NTILES];
#pragma unroll
  for (int t = 0; t < NTILES; ++t) acc[t] = (double4_t){0.0, 0.0, 0.0, 0.0};
  LaneSnaps<PER> L;
  lane_snaps_init<PER>(snaps, nsnap, L);
  const long long nchunks = (n + kWaveRows - 1) / kWaveRows;
  const long long nwaves = gridDim.x * 4LL;
  for (long long ch = blockIdx.x * 4LL + wv; ch < nchunks; ch += nwaves) {
    const long long row = ch * kWaveRows + lane % 16;
    lane_snaps_load<PER>(L, nsnap, n, row);
    const double c = lane_snaps_centre<PER>(L, nsnap, w, row, n, nullptr);
    wave_lds_fence();
    lane_snaps_store<PER>(L, c, nsnap, w, wp, xs, ldx);
    wave_lds_fence();
    // Y tile mb: lane holds Y[lane % 16][16 mb + lane / 16 + 4 i]
    double4_t yv[NT];
#pragma unroll
    for (int mb = 0; mb < NT; ++mb) {
      yv[mb] = (double4_t){0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
      for (int k0 = 0; k0 + 1 < NS; k0 += 4) {
        const int k = k0 + lane / 16;
        const double a = Ts[k * ldt + mb * 16 + lane % 16];   // A = T1^T: A[c][k] = T1[k][c]
        const double b = xs[(lane % 16) * ldx + k];           // B[k][r] = X[r][k]
        yv[mb] = mfma_f64(a, b, yv[mb]);
      }
    }
    wave_lds_fence();
#pragma unroll
    for (int mb = 0; mb < NT; ++mb)
#pragma unroll
      for (int i = 0; i < 4; ++i) xs[(lane % 16) * ldx + mb * 16 + lane / 16 + 4 * i] = yv[mb][i];
    wave_lds_fence();
#pragma unroll 1
    for (int k0 = 0; k0 < kWaveRows; k0 += 4) {
      const int k = k0 + lane / 16;
      double x[NT];
#pragma unroll
      for (int tb = 0; tb < NT; ++tb) x[tb] = xs[k * ldx + tb * 16 + lane % 16];
      int t = 0;
#pragma unroll
      for (int ti = 0; ti < NT; ++ti)
#pragma unroll
        for (int tj = ti; tj < NT; ++tj, ++t) acc[t] = mfma_f64(x[ti], x[tj], acc[t]);
    }
  }
  __syncthreads();
  double* red = sh;
  for (int q = 0; q < 4; ++q) {
    if (wv == q) {
#pragma unroll
      for (int t = 0; t < NTILES; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int e = t * 256 + i * kWave + lane;
          red[e] = q == 0 ? acc[t][i] : red[e] + acc[t][i];
        }
    }
    __syncthreads();
  }
  double* out = part + (size_t)blockIdx.x * wp * wp;
  for (int e = threadIdx.x; e < NTILES * 256; e += blockDim.x) {
    const int t = e / 256, i = (e % 256) / kWave, l = e % kWave;
    int ti = 0, tt = t;
    while (tt >= NT - ti) {
      tt -= NT - ti;
      ++ti;
    }
    const int tj = ti + tt;
    const int r = ti * 16 + l / 16 + 4 * i, cc = tj * 16 + l % 16;
    out[r * wp + cc] = red[e];
  }
}

// Phi = X T for rows of the window (centred on the fly), on MFMA, in
// wave-private chunks as the Gram pass.  C^T = T^T X^T so that each 16-lane
// group writes 16 consecutive rows of one column of Phi.  Block: 4 waves;
// dynamic LDS: T (wp x (mp + 1)), then 4 regions of kWaveRows x (wp + 1).
// TP = double, or float for the FP32 master copy (rounded once on store).
// meff is read from device memory (the eigen kernel's output), so the pass can
// be enqueued before the host learns m_eff.
template <int NS, typename TP>
__global__ void __launch_bounds__(256) basis_form_kernel(const SnapTable snaps, int nsnap,
                                                         int w, long long n, const double* __restrict__ T,
                                                         int mp, int wp, const int* __restrict__ meff_d,
                                                         TP* __restrict__ Phi) {
  extern __shared__ double sh[];
  constexpr int PER = (NS + 3) / 4;
  const int meff = *meff_d;
  const int ldx = wp + 1, ldt = mp + 1;
  double* Ts = sh;
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  double* xs = sh + wp * ldt + wv * kWaveRows * ldx;
  for (int e = threadIdx.x; e < wp * mp; e += blockDim.x) Ts[(e / mp) * ldt + e % mp] = T[e];
  for (int e = lane; e < kWaveRows * ldx; e += kWave) xs[e] = 0.0;
  __syncthreads();
  LaneSnaps<PER> L;
  lane_snaps_init<PER>(snaps, nsnap, L);
  const long long nchunks = (n + kWaveRows - 1) / kWaveRows;
  const long long nwaves = gridDim.x * 4LL;
  for (long long ch = blockIdx.x * 4LL + wv; ch < nchunks; ch += nwaves) {
    const long long row = ch * kWaveRows + lane % 16;
    lane_snaps_load<PER>(L, nsnap, n, row);
    const double c = lane_snaps_centre<PER>(L, nsnap, w, row, n, nullptr);
    wave_lds_fence();
    lane_snaps_store<PER>(L, c, nsnap, w, wp, xs, ldx);
    wave_lds_fence();
    for (int mb = 0; mb * 16 < meff; ++mb) {
      double4_t acc = (double4_t){0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
      for (int k0 = 0; k0 + 1 < NS; k0 += 4) {
        const int k = k0 + lane / 16;
        const double a = Ts[k * ldt + mb * 16 + lane % 16];              // A = T^T: A[c][k] = T[k][c]
        const double b = xs[(lane % 16) * ldx + k];                      // B[k][r] = X[r][k]
        acc = mfma_f64(a, b, acc);
      }
      const long long orow = ch * kWaveRows + lane % 16;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int col = mb * 16 + lane / 16 + 4 * i;
        if (col < meff && orow < n) Phi[(size_t)col * n + orow] = (TP)acc[i];
      }
    }
  }
}

// Workgroups of 256 threads of kernel fn (dynamic LDS lds) that the device
// holds at once: a window pass launched with exactly that many workgroups
// runs in one resident round, every wave with the same share of chunks.
static int resident_blocks(const hs_ctx* ctx, const void* fn, size_t lds) {
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, 256, lds) != hipSuccess || per < 1) per = 1;
  return per * ctx->num_cu;
}

// Enqueue the whole update on the context's current stream; m_eff stays on
// the device (meff_d) until read back.
static hs_status basis_enqueue(hs_ctx* ctx, const double* const* snaps, int32_t nsnap, int32_t w, int32_t m,
                               double tau_pod, int32_t precision, void* Phi_out, double* psi_out,
                               double* sigma_out) {
  if (!ctx || !snaps || !Phi_out || !psi_out || !sigma_out) return HS_ERR_INVALID_ARG;
  if (w < 2 || w > ctx->p.w_max || (nsnap != w && nsnap != w + 1)) return HS_ERR_INVALID_ARG;
  if (m < 1 || m > ctx->p.m_max || m > w) return HS_ERR_INVALID_ARG;
  if (!(tau_pod >= 0.0 && tau_pod < 1.0)) return HS_ERR_INVALID_ARG;
  if (precision != HS_FP64 && precision != HS_MIXED_FP32) return HS_ERR_INVALID_ARG;
  if (ctx->n >= (1LL << 29)) return ctx->fail(HS_ERR_SHAPE, "basis_update: more than 2^29 entries per snapshot");
  for (int j = 0; j < nsnap; ++j)
    if (!snaps[j]) return HS_ERR_INVALID_ARG;
  SnapTable tab{};
  for (int j = 0; j < nsnap; ++j) tab.p[j] = snaps[j];
  const long long n = ctx->n;
  const int wp = (w + 15) / 16 * 16;
  const int mp = (m + 15) / 16 * 16;
  // four waves per workgroup, each on 16-row chunks; the Gram pass keeps
  // three workgroups per compute unit resident (registers), so its grid is
  // one resident round (768), which also bounds the partials it leaves
  const long long nchunks = (n + kWaveRows - 1) / kWaveRows;
  const int nb = (int)std::min<long long>((nchunks + 3) / 4, 768);
  const int nbf = (int)std::min<long long>((nchunks + 3) / 4, kRedBlocks);
  int nb_pgram = nb;
  const size_t glds = (size_t)4 * kWaveRows * (wp + 1) * sizeof(double);
  const size_t flds = ((size_t)wp * (mp + 1) + (size_t)4 * kWaveRows * (wp + 1)) * sizeof(double);
  if (flds > (size_t)ctx->max_lds)
    return ctx->fail(HS_ERR_SHAPE, "basis_update: window and rank need more LDS than a workgroup has");
  HS_TRY(prof_begin(ctx, HS_PROF_BASIS_GRAM));
  switch (wp) {
    case 16: hipLaunchKernelGGL(window_gram_kernel<17>, dim3(nb), dim3(256), glds, ctx->stream, tab, nsnap, w, n, wp, psi_out, ctx->red); break;
    case 32: hipLaunchKernelGGL(window_gram_kernel<33>, dim3(nb), dim3(256), glds, ctx->stream, tab, nsnap, w, n, wp, psi_out, ctx->red); break;
    case 48: hipLaunchKernelGGL(window_gram_kernel<49>, dim3(nb), dim3(256), glds, ctx->stream, tab, nsnap, w, n, wp, psi_out, ctx->red); break;
    default: hipLaunchKernelGGL(window_gram_kernel<65>, dim3(nb), dim3(256), glds, ctx->stream, tab, nsnap, w, n, wp, psi_out, ctx->red); break;
  }
  HIP_TRY(ctx, hipGetLastError());
  // reads every snapshot of the window once, writes psi_{k+1}
  HS_TRY(prof_end(ctx, HS_PROF_BASIS_GRAM, 8.0 * (double)n * (nsnap + 1)));
  double* G = ctx->small + kSmBasG;
  double* G2 = ctx->small + kSmBasG2;
  double* T1 = ctx->small + kSmBasT1;
  double* C1 = ctx->small + kSmBasC1;
  double* T = ctx->small + kSmBasT;
  int* meff_d = reinterpret_cast<int*>(ctx->small + kSmBasMeff);
  HS_LAUNCH(ctx, gram_reduce_kernel, w * w, kBlock, ctx->red, nb, wp, w, G);
  HS_LAUNCH(ctx, basis_prec_kernel, 1, 256, (const double*)G, w, wp, T1, C1);
  // second pass: Gram of X T1 (reads every window snapshot once)
  const size_t plds = ((size_t)wp * (wp + 1) + (size_t)4 * kWaveRows * (wp + 1)) * sizeof(double);
  if (plds > (size_t)ctx->max_lds)
    return ctx->fail(HS_ERR_SHAPE, "basis_update: window needs more LDS than a workgroup has");
  HS_TRY(prof_begin(ctx, HS_PROF_BASIS_PGRAM));
  {
    // the pass holds more registers than the Gram pass (two workgroups per
    // compute unit instead of three): its grid is its own resident round
    const void* fn = wp == 16 ? (const void*)window_pgram_kernel<17>
                   : wp == 32 ? (const void*)window_pgram_kernel<33>
                   : wp == 48 ? (const void*)window_pgram_kernel<49> : (const void*)window_pgram_kernel<65>;
    const int nbp = (int)std::min<long long>({(nchunks + 3) / 4, (long long)resident_blocks(ctx, fn, plds), 768LL});
    switch (wp) {
      case 16: hipLaunchKernelGGL(window_pgram_kernel<17>, dim3(nbp), dim3(256), plds, ctx->stream, tab, nsnap, w, n, (const double*)T1, wp, ctx->red); break;
      case 32: hipLaunchKernelGGL(window_pgram_kernel<33>, dim3(nbp), dim3(256), plds, ctx->stream, tab, nsnap, w, n, (const double*)T1, wp, ctx->red); break;
      case 48: hipLaunchKernelGGL(window_pgram_kernel<49>, dim3(nbp), dim3(256), plds, ctx->stream, tab, nsnap, w, n, (const double*)T1, wp, ctx->red); break;
      default: hipLaunchKernelGGL(window_pgram_kernel<65>, dim3(nbp), dim3(256), plds, ctx->stream, tab, nsnap, w, n, (const double*)T1, wp, ctx->red); break;
    }
    nb_pgram = nbp;
  }
  HIP_TRY(ctx, hipGetLastError());
  HS_TRY(prof_end(ctx, HS_PROF_BASIS_PGRAM, 8.0 * (double)n * nsnap));
  HS_LAUNCH(ctx, gram_reduce_kernel, w * w, kBlock, ctx->red, nb_pgram, wp, w, G2);
  HS_LAUNCH(ctx, basis_svd_kernel, 1, 256, (const double*)G2, (const double*)C1, w, m, tau_pod, sigma_out, T, mp,
            meff_d);
  HS_TRY(prof_begin(ctx, HS_PROF_BASIS_FORM));
#define HS_FORM(NSV)                                                                                            \
  do {                                                                                                          \
    if (precision == HS_MIXED_FP32)                                                                             \
      hipLaunchKernelGGL((basis_form_kernel<NSV, float>), dim3(nbf), dim3(256), flds, ctx->stream, tab, nsnap, w, n, \
                         (const double*)T, mp, wp, (const int*)meff_d, (float*)Phi_out);                       \
    else                                                                                                        \
      hipLaunchKernelGGL((basis_form_kernel<NSV, double>), dim3(nbf), dim3(256), flds, ctx->stream, tab, nsnap, w, \
                         n, (const double*)T, mp, wp, (const int*)meff_d, (double*)Phi_out);                   \
  } while (0)
  switch (wp) {
    case 16: HS_FORM(17); break;
    case 32: HS_FORM(33); break;
    case 48: HS_FORM(49); break;
    default: HS_FORM(65); break;
  }
#undef HS_FORM
  HIP_TRY(ctx, hipGetLastError());
  // the measurement ends with the kernel; its bytes need m_eff (set on completion)
  const size_t before = ctx->prof_bytes.size();
  HS_TRY(prof_end(ctx, HS_PROF_BASIS_FORM, 0.0));
  const int idx = ctx->prof_bytes.size() > before ? (int)before : -1;
  ctx->pending_form = {n, nsnap, precision == HS_MIXED_FP32 ? 4.0 : 8.0, idx};
  return HS_OK;
}

// m_eff of the enqueued update (waits for the stream it ran on); closes the
// formation pass's measurement with its algorithmic bytes.
static hs_status basis_complete(hs_ctx* ctx, int32_t* m_eff) {
  int* meff_d = reinterpret_cast<int*>(ctx->small + kSmBasMeff);
  int me = 0;
  HS_TRY(readback(ctx, meff_d, sizeof(int), &me));
  *m_eff = me;
  ctx->basis_meff = me;
  // reads every snapshot of the window once, writes m_eff columns of Phi
  const auto& f = ctx->pending_form;
  if (f.prof_idx >= 0 && f.prof_idx < (int)ctx->prof_bytes.size())
    ctx->prof_bytes[f.prof_idx] = (double)f.n * (8.0 * f.nsnap + f.phi_bytes * me);
  return HS_OK;
}

}  // namespace hs

using namespace hs;

extern "C" hs_status basis_update(hs_ctx* ctx, const double* const* snaps, int32_t nsnap, int32_t w, int32_t m,
                                  double tau_pod, int32_t precision, void* Phi_out, double* psi_out,
                                  double* sigma_out, int32_t* m_eff) {
  if (!ctx || !m_eff) return HS_ERR_INVALID_ARG;
  if (ctx->aux_pending) return ctx->fail(HS_ERR_INVALID_ARG, "an asynchronous basis update is in flight");
  HS_TRY(basis_enqueue(ctx, snaps, nsnap, w, m, tau_pod, precision, Phi_out, psi_out, sigma_out));
  return basis_complete(ctx, m_eff);
}

extern "C" hs_status basis_update_async(hs_ctx* ctx, const double* const* snaps, int32_t nsnap, int32_t w,
                                        int32_t m, double tau_pod, int32_t precision, void* Phi_out,
                                        double* psi_out, double* sigma_out) {
  if (!ctx) return HS_ERR_INVALID_ARG;
  if (ctx->aux_pending) return ctx->fail(HS_ERR_INVALID_ARG, "an asynchronous basis update is in flight");
  // the update starts after everything enqueued on the context's stream so far
  HIP_TRY(ctx, hipEventRecord(ctx->aux_ready, ctx->stream));
  HIP_TRY(ctx, hipStreamWaitEvent(ctx->aux, ctx->aux_ready, 0));
  hipStream_t main = ctx->stream;
  ctx->stream = ctx->aux;
  const hs_status st = basis_enqueue(ctx, snaps, nsnap, w, m, tau_pod, precision, Phi_out, psi_out, sigma_out);
  ctx->stream = main;
  if (st != HS_OK) {
    (void)hipStreamSynchronize(ctx->aux);
    return st;
  }
  ctx->aux_pending = true;
  return HS_OK;
}

namespace hs {
hs_status basis_finish_pending(hs_ctx* ctx, int32_t* m_eff) {
  if (!ctx->aux_pending) return ctx->fail(HS_ERR_INVALID_ARG, "no asynchronous basis update in flight");
  ctx->aux_pending = false;
  hipStream_t main = ctx->stream;
  ctx->stream = ctx->aux;
  const hs_status st = basis_complete(ctx, m_eff);
  ctx->stream = main;
  return st;
}
}  // namespace hs

extern "C" hs_status basis_update_finish(hs_ctx* ctx, int32_t* m_eff) {
  if (!ctx || !m_eff) return HS_ERR_INVALID_ARG;
  return basis_finish_pending(ctx, m_eff);
}

extern "C" hs_status hs_basis_m_eff(hs_ctx* ctx, int32_t* m_eff) {
  if (!ctx || !m_eff) return HS_ERR_INVALID_ARG;
  if (ctx->aux_pending) return ctx->fail(HS_ERR_INVALID_ARG, "a basis update is still in flight");
  *m_eff = ctx->basis_meff;
  return HS_OK;
}
