// Tall-skinny dense kernels on FP64 MFMA (v_mfma_f64_16x16x4f64) and the
// one-wave symmetric Jacobi eigensolver used for the small (<= 64 x 64)
// problems of the basis update and of the gappy fit.
//
// MFMA operand layout (16x16x4, wave64): lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; accumulator element i of lane l is
// C[l / 16 + 4 i][l % 16] (measured on gfx950 with a known product).
#pragma once

#include "common.hpp"

namespace hs {

typedef double double4_t __attribute__((ext_vector_type(4)));

__device__ inline double4_t mfma_f64(double a, double b, double4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kChunk = 64;   // rows staged per LDS chunk

// Gram G = X^T X of a tall matrix whose rows are produced by a Loader into
// LDS (kChunk rows x ldx, zero padded), accumulated over all chunks of this
// block; the block's partial wp x wp matrix goes to part[blockIdx.x].
//   Loader::init(regs) loads per-block constants (e.g. pointers) once;
//   Loader::prefetch(chunk_row0, regs) issues the loads of a chunk into
//   registers; Loader::commit(chunk_row0, regs, X /*LDS kChunk x ldx*/) writes
//   the rows.  The next chunk's loads are in flight during the products.
// Block: 256 threads = 4 waves; G is symmetric, so only the nt (nt + 1) / 2
// tiles with ti <= tj are formed; wave v owns tiles t = v, v + 4, ... of them.
template <class Loader>
__global__ void __launch_bounds__(256) gram_kernel(Loader ld, long long nrows, int wp,
                                                   double* __restrict__ part) {
  extern __shared__ double X[];   // kChunk x (wp + 1)
  const int ldx = wp + 1;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int nt = wp / 16;
  const int ntiles = nt * (nt + 1) / 2;
  // upper-triangle tile t -> (ti, tj), ti <= tj, row by row
  auto tile_of = [nt](int t, int& ti, int& tj) {
    int i = 0;
    while (t >= nt - i) {
      t -= nt - i;
      ++i;
    }
    ti = i;
    tj = i + t;
  };
  double4_t acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = (double4_t){0.0, 0.0, 0.0, 0.0};
  const long long nchunks = (nrows + kChunk - 1) / kChunk;
  typename Loader::Regs R;
  ld.init(R);
  long long ch = blockIdx.x;
  if (ch < nchunks) ld.prefetch(ch * kChunk, R);
  for (; ch < nchunks; ch += gridDim.x) {
    __syncthreads();
    ld.commit(ch * kChunk, R, X, ldx, wp);
    __syncthreads();
    if (ch + gridDim.x < nchunks) ld.prefetch((ch + gridDim.x) * kChunk, R);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int tile = wave + 4 * t;
      if (tile >= ntiles) break;
      int ti, tj;
      tile_of(tile, ti, tj);
#pragma unroll 4
      for (int k0 = 0; k0 < kChunk; k0 += 4) {
        const int k = k0 + lane / 16;
        const double a = X[k * ldx + ti * 16 + lane % 16];   // A = X^T: A[r][k] = X[k][ti*16 + r]
        const double b = X[k * ldx + tj * 16 + lane % 16];   // B[k][c] = X[k][tj*16 + c]
        acc[t] = mfma_f64(a, b, acc[t]);
      }
    }
  }
  double* out = part + (size_t)blockIdx.x * wp * wp;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int tile = wave + 4 * t;
    if (tile >= ntiles) break;
    int ti, tj;
    tile_of(tile, ti, tj);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = ti * 16 + lane / 16 + 4 * i, c = tj * 16 + lane % 16;
      out[r * wp + c] = acc[t][i];
    }
  }
}

// Sum nb partial wp x wp matrices; one block per entry of the w x w result
// (row-major, leading dimension w), a fixed strided order and a fixed tree.
// Entries below the diagonal tiles are read from their mirror image (only
// tiles with ti <= tj are formed), so G is exactly symmetric off the
// diagonal tiles.
static __global__ void gram_reduce_kernel(const double* __restrict__ part, int nb, int wp, int w,
                                          double* __restrict__ G) {
  __shared__ double lds[kBlock / kWave];
  const int e = blockIdx.x;
  int r = e / w, c = e % w;
  if (r / 16 > c / 16) {
    const int x = r;
    r = c;
    c = x;
  }
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) s += part[(size_t)b * wp * wp + r * wp + c];
  s = block_sum(s, lds);
  if (threadIdx.x == 0) G[e] = s;
}

// ---------------------------------------------------------------- Jacobi
// Symmetric eigendecomposition A = V diag(lam) V^T of an n x n matrix (n <= 64)
// by cyclic Jacobi with round-robin parallel ordering (any block size that is
// a multiple of 64).  A pair is rotated only if its off-diagonal entry exceeds
// both eps * sqrt(|a_pp a_qq|) and eps * trace|A|: below the latter an entry
// is rounding noise that cannot move any eigenvalue by more than rounding.
// Sweeps stop once no entry exceeds n eps sqrt(|a_pp a_qq|).  On
// return lam is sorted in descending order with V's columns permuted alike.
// A (n x n, row-major) is overwritten.  LDS: A, V (64 x 65 each).
__device__ inline void jacobi_eig_wave(double* A, double* V, int lda, int n, double* lam, int* order,
                                       int max_sweeps) {
  // every product and sum rounded on its own (no contraction), so that the
  // register variant for m <= 8 takes the same rotations to the bit
#pragma clang fp contract(off)
  const int t = threadIdx.x;
  const int nt = blockDim.x;
  for (int i = t; i < n * lda; i += nt) V[i] = 0.0;
  __syncthreads();
  if (t < n) V[t * lda + t] = 1.0;
  __syncthreads();
  const int np = (n + 1) & ~1;     // even number of players
  __shared__ double cs[32], sn[32];
  __shared__ int pp[32], qq[32];
  __shared__ int rotated;
  __shared__ double atol;
  if (t == 0) {
    double tr = 0.0;
    for (int i = 0; i < n; ++i) tr += fabs(A[i * lda + i]);
    atol = 2.2e-16 * tr;
  }
  __syncthreads();
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (t == 0) rotated = 0;
    __syncthreads();
    for (int r = 0; r < np - 1; ++r) {
      if (t < np / 2) {
        int p, q;
        if (t == 0) {
          p = r % (np - 1);
          q = np - 1;
        } else {
          p = (r + t) % (np - 1);
          q = (r - t + (np - 1)) % (np - 1);
        }
        if (p > q) { const int x = p; p = q; q = x; }
        double c = 1.0, s = 0.0;
        if (q < n) {
          // thresholds on squares (no square root), and the rotation with one
          // square root, one division and one reciprocal square root:
          // t = sign(d) e / (|d| + sqrt(d^2 + e^2)), d = (a_qq - a_pp) / 2,
          // e = a_pq, is tan(theta) of the rotation that zeroes a_pq
          const double apq = A[p * lda + q];
          const double app = A[p * lda + p], aqq = A[q * lda + q];
          const double lim2 = fabs(app) * fabs(aqq);
          const double apq2 = apq * apq;
          if (fabs(apq) > atol && apq2 > (2.2e-16 * 2.2e-16) * lim2) {
            const double d = 0.5 * (aqq - app);
            const double tt = (d >= 0.0 ? apq : -apq) / (fabs(d) + sqrt(d * d + apq2));
            c = rsqrt(1.0 + tt * tt);
            s = tt * c;
            // rotations at the rounding level do not keep the sweeps going
            const double nt2 = (double)n * 2.2e-16;
            if (apq2 > nt2 * nt2 * lim2) rotated = 1;
          }
        }
        pp[t] = p; qq[t] = q; cs[t] = c; sn[t] = s;
      }
      __shared__ int any;
      if (t == 0) any = 0;
      __syncthreads();
      if (t < np / 2 && sn[t] != 0.0) any = 1;
      __syncthreads();
      if (any) {
        // A <- J^T A J on the disjoint 2x2 blocks (rows of pair k, columns of pair l)
        const int P = np / 2;
        for (int b = t; b < P * P; b += nt) {
          const int k = b / P, l = b % P;
          if (sn[k] == 0.0 && sn[l] == 0.0) continue;
          const int rp = pp[k], rq = qq[k], cp = pp[l], cq = qq[l];
          const bool rqv = rq < n, cqv = cq < n;
          double a00 = A[rp * lda + cp];
          double a01 = cqv ? A[rp * lda + cq] : 0.0;
          double a10 = rqv ? A[rq * lda + cp] : 0.0;
          double a11 = (rqv && cqv) ? A[rq * lda + cq] : 0.0;
          const double ck = cs[k], sk = sn[k], cl = cs[l], sl = sn[l];
          // rows
          double b00 = ck * a00 - sk * a10, b01 = ck * a01 - sk * a11;
          double b10 = sk * a00 + ck * a10, b11 = sk * a01 + ck * a11;
          // columns
          a00 = cl * b00 - sl * b01;
          a01 = sl * b00 + cl * b01;
          a10 = cl * b10 - sl * b11;
          a11 = sl * b10 + cl * b11;
          A[rp * lda + cp] = a00;
          if (cqv) A[rp * lda + cq] = a01;
          if (rqv) A[rq * lda + cp] = a10;
          if (rqv && cqv) A[rq * lda + cq] = a11;
        }
        // V <- V J
        for (int e = t; e < P * n; e += nt) {
          const int l = e / n, row = e % n;
          if (sn[l] == 0.0) continue;
          const int p = pp[l], q = qq[l];
          const double c = cs[l], s = sn[l];
          const double vp = V[row * lda + p], vq = V[row * lda + q];
          V[row * lda + p] = c * vp - s * vq;
          V[row * lda + q] = s * vp + c * vq;
        }
      }
      __syncthreads();
    }
    if (!rotated) break;
    __syncthreads();
  }
  // stable descending order by rank: rank_i = #{j: l_j > l_i} + #{j < i: l_j == l_i}
  if (t < n) {
    const double li = A[t * lda + t];
    int rk = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = A[j * lda + j];
      rk += (lj > li) || (lj == li && j < t);
    }
    lam[rk] = li;
    order[rk] = t;
  }
  __syncthreads();
}

}  // namespace hs
