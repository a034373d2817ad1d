// POD basis update (A9): reference state and POD_m of the snapshot window
// (eq. mean, eq. pod; the basis-update branch of Alg. 1).
//
// One pass over the window forms, row by row, both window means (the
// centring state psi_k over the first w snapshots and psi_{k+1} over the last
// w), the centred row of X = [gamma_j - psi_k] and accumulates the Gram
// matrix X^T X on FP64 MFMA.  A one-wave Jacobi eigensolver gives
// X^T X = V diag(sigma^2) V^T; a second pass forms Phi = X V_m diag(1/sigma_m),
// the left singular vectors, again on MFMA.  The traffic is two reads of the
// window and one write of Phi (the method-of-snapshots minimum).
#include "dense.hpp"

#include <algorithm>
#include <cstring>

namespace hs {

constexpr int kMaxSnaps = kMaxBasis + 1;
constexpr int kRawLd = kMaxSnaps + 1;   // LDS leading dimension of the raw snapshot tile

// Stage the rows row0 .. row0+63 of all nsnap snapshots into LDS (raw[r][j]),
// every thread issuing independent coalesced loads, then let one thread per
// row form the two window means by sequential sums in snapshot order.
__device__ inline void stage_window(const double* const* __restrict__ snaps, int nsnap, int w, long long n,
                                    long long row0, double* raw, double* centre, double* psi_new) {
  for (int idx = threadIdx.x; idx < kChunk * nsnap; idx += blockDim.x) {
    const int r = idx % kChunk, j = idx / kChunk;
    const long long row = row0 + r;
    raw[r * kRawLd + j] = row < n ? snaps[j][row] : 0.0;
  }
  __syncthreads();
  if (threadIdx.x < kChunk) {
    const int r = threadIdx.x;
    const double* x = raw + r * kRawLd;
    double c = 0.0, nw = 0.0;
    for (int j = 0; j < w; ++j) c += x[j];
    for (int j = nsnap - w; j < nsnap; ++j) nw += x[j];
    c = c / (double)w;
    nw = nw / (double)w;
    centre[r] = c;
    if (psi_new && row0 + r < n) psi_new[row0 + r] = nw;
  }
  __syncthreads();
}

// Row loader of the centred window; also writes psi_new for its rows.
struct WindowLoader {
  const double* const* snaps;   // device table of nsnap pointers
  int nsnap, w;
  long long n;
  double* psi_new;
  __device__ void load(long long row0, double* X, int ldx, int wp) const {
    __shared__ double raw[kChunk * kRawLd];
    __shared__ double centre[kChunk];
    stage_window(snaps, nsnap, w, n, row0, raw, centre, psi_new);
    const int off = nsnap - w;
    for (int idx = threadIdx.x; idx < kChunk * wp; idx += blockDim.x) {
      const int r = idx / wp, j = idx % wp;
      X[r * ldx + j] = j < w ? raw[r * kRawLd + off + j] - centre[r] : 0.0;
    }
  }
};

// Eigen-decomposition of G (w x w) and the formation matrix
// T = V_m diag(1/sigma) (w x mp, zero padded), sigma (w), m_eff.
__global__ void __launch_bounds__(256) basis_eig_kernel(const double* __restrict__ G, int w, int m,
                                                       double tau, double* __restrict__ sigma,
                                                       double* __restrict__ T, int mp,
                                                       int* __restrict__ m_eff_out) {
  __shared__ double A[kMaxBasis * (kMaxBasis + 1)], V[kMaxBasis * (kMaxBasis + 1)];
  __shared__ double lam[kMaxBasis];
  __shared__ int order[kMaxBasis];
  __shared__ int meff;
  const int lda = kMaxBasis + 1;
  const int t = threadIdx.x;
  for (int e = t; e < w * w; e += blockDim.x) A[(e / w) * lda + e % w] = G[e];
  __syncthreads();
  jacobi_eig_wave(A, V, lda, w, lam, order, 40);
  if (t == 0) {
    const double s0 = sqrt(fmax(lam[0], 0.0));
    int me = 0;
    for (int i = 0; i < w; ++i) {
      const double si = sqrt(fmax(lam[i], 0.0));
      sigma[i] = si;
      if (i < m && s0 > 0.0 && si > tau * s0) me = i + 1;
    }
    meff = me;
    *m_eff_out = me;
  }
  __syncthreads();
  // T[:, i] = sign_i * V[:, order[i]] / sigma_i, sign making the largest |entry| positive
  for (int i = t; i < mp; i += blockDim.x) {
    if (i < meff) {
      const int col = order[i];
      int best = 0;
      double bv = -1.0;
      for (int r = 0; r < w; ++r) {
        const double a = fabs(V[r * lda + col]);
        if (a > bv) { bv = a; best = r; }
      }
      const double sg = V[best * lda + col] >= 0.0 ? 1.0 : -1.0;
      const double inv = sg / sqrt(lam[i]);
      for (int r = 0; r < kMaxBasis; ++r) T[r * mp + i] = r < w ? V[r * lda + col] * inv : 0.0;
    } else {
      for (int r = 0; r < kMaxBasis; ++r) T[r * mp + i] = 0.0;
    }
  }
}

// Phi = X T for rows of the window (centred on the fly), on MFMA.
// C^T = T^T X^T so that each 16-lane group writes 16 consecutive rows of one
// column of Phi.
__global__ void __launch_bounds__(256) basis_form_kernel(const double* const* __restrict__ snaps, int nsnap,
                                                         int w, long long n, const double* __restrict__ T,
                                                         int mp, int wp, int meff, double* __restrict__ Phi) {
  __shared__ double raw[kChunk * kRawLd];
  __shared__ double Ts[kMaxBasis * (kMaxBasis + 1)];
  __shared__ double centre[kChunk];
  const int ldx = kMaxBasis + 1;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  for (int e = threadIdx.x; e < wp * mp; e += blockDim.x) Ts[(e / mp) * ldx + e % mp] = T[(e / mp) * mp + e % mp];
  const int off = nsnap - w;
  const long long nchunks = (n + kChunk - 1) / kChunk;
  for (long long ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    const long long row0 = ch * kChunk;
    __syncthreads();
    stage_window(snaps, nsnap, w, n, row0, raw, centre, nullptr);
    // centre the X columns in place (raw[r][off + j] -> x_j - centre)
    for (int idx = threadIdx.x; idx < kChunk * wp; idx += blockDim.x) {
      const int r = idx / wp, j = idx % wp;
      raw[r * kRawLd + off + j] = j < w ? raw[r * kRawLd + off + j] - centre[r] : 0.0;
    }
    __syncthreads();
    const int rb = wave;   // 16 rows per wave
    for (int mb = 0; mb * 16 < mp; ++mb) {
      double4_t acc = (double4_t){0.0, 0.0, 0.0, 0.0};
      for (int k0 = 0; k0 < wp; k0 += 4) {
        const int k = k0 + lane / 16;
        const double a = Ts[k * ldx + mb * 16 + lane % 16];                 // A = T^T: A[c][k] = T[k][c]
        const double b = raw[(rb * 16 + lane % 16) * kRawLd + off + k];     // B[k][r] = X[r][k]
        acc = mfma_f64(a, b, acc);
      }
      const long long orow = row0 + rb * 16 + lane % 16;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int col = mb * 16 + lane / 16 + 4 * i;
        if (col < meff && orow < n) Phi[(size_t)col * n + orow] = acc[i];
      }
    }
  }
}

}  // namespace hs

using namespace hs;

extern "C" hs_status basis_update(hs_ctx* ctx, const double* const* snaps, int32_t nsnap, int32_t w, int32_t m,
                                  double tau_pod, int32_t precision, double* Phi_out, double* psi_out,
                                  double* sigma_out, int32_t* m_eff) {
  if (!ctx || !snaps || !Phi_out || !psi_out || !sigma_out || !m_eff) return HS_ERR_INVALID_ARG;
  if (w < 2 || w > ctx->p.w_max || (nsnap != w && nsnap != w + 1)) return HS_ERR_INVALID_ARG;
  if (m < 1 || m > ctx->p.m_max || m > w) return HS_ERR_INVALID_ARG;
  if (!(tau_pod >= 0.0 && tau_pod < 1.0)) return HS_ERR_INVALID_ARG;
  if (precision != HS_FP64) return ctx->fail(HS_ERR_INVALID_ARG, "basis_update: only HS_FP64 in this build");
  for (int j = 0; j < nsnap; ++j)
    if (!snaps[j]) return HS_ERR_INVALID_ARG;
  // pointer table to device memory through the pinned staging area
  std::memcpy(ctx->hstage, snaps, nsnap * sizeof(double*));
  HIP_TRY(ctx, hipMemcpyAsync(ctx->ptab, ctx->hstage, nsnap * sizeof(double*), hipMemcpyHostToDevice, ctx->stream));
  const double* const* tab = const_cast<const double* const*>(ctx->ptab);
  const long long n = ctx->n;
  const int wp = (w + 15) / 16 * 16;
  const int mp = (m + 15) / 16 * 16;
  const long long nchunks = (n + kChunk - 1) / kChunk;
  const int nb = (int)std::min<long long>(nchunks, 512);
  WindowLoader ld{tab, nsnap, w, n, psi_out};
  const size_t lds = (size_t)kChunk * (wp + 1) * sizeof(double);
  HS_TRY(prof_begin(ctx, HS_PROF_BASIS_GRAM));
  hipLaunchKernelGGL(gram_kernel<WindowLoader>, dim3(nb), dim3(256), lds, ctx->stream, ld, n, wp, ctx->red);
  HIP_TRY(ctx, hipGetLastError());
  // reads every snapshot of the window once, writes psi_{k+1}
  HS_TRY(prof_end(ctx, HS_PROF_BASIS_GRAM, 8.0 * (double)n * (nsnap + 1)));
  double* G = ctx->small;
  double* T = ctx->small + kMaxBasis * kMaxBasis;
  int* meff_d = reinterpret_cast<int*>(ctx->small + 3 * kMaxBasis * kMaxBasis);
  HS_LAUNCH(ctx, gram_reduce_kernel, w * w, kBlock, ctx->red, nb, wp, w, G);
  HS_LAUNCH(ctx, basis_eig_kernel, 1, 256, G, w, m, tau_pod, sigma_out, T, mp, meff_d);
  int me = 0;
  HS_TRY(readback(ctx, meff_d, sizeof(int), &me));
  *m_eff = me;
  if (me == 0) return HS_OK;
  HS_TRY(prof_begin(ctx, HS_PROF_BASIS_FORM));
  HS_LAUNCH(ctx, basis_form_kernel, nb, 256, tab, nsnap, w, n, T, mp, wp, me, Phi_out);
  // reads every snapshot of the window once, writes m_eff columns of Phi
  HS_TRY(prof_end(ctx, HS_PROF_BASIS_FORM, 8.0 * (double)n * (nsnap + me)));
  return HS_OK;
}
