// POD basis update (A9): reference state and POD_m of the snapshot window
// (eq. mean, eq. pod; the basis-update branch of Alg. 1).
//
// One pass over the window forms, row by row, both window means (the
// centring state psi_k over the first w snapshots and psi_{k+1} over the last
// w), the centred row of X = [gamma_j - psi_k] and accumulates the Gram
// matrix X^T X on FP64 MFMA.  A pivoted Cholesky reduction to the numerical
// rank and a Jacobi eigensolver on the reduced matrix give
// X^T X = V diag(sigma^2) V^T; a second pass forms Phi = X V_m diag(1/sigma_m),
// the left singular vectors, again on MFMA.  The traffic is two reads of the
// window and one write of Phi (the method-of-snapshots minimum).
// Kernels using the window staging must run with 256 threads (four waves).
#include "dense.hpp"

#include <algorithm>
#include <cstring>

namespace hs {

constexpr int kMaxSnaps = kMaxBasis + 1;
constexpr int kPerWave = (kMaxSnaps + 3) / 4;   // snapshots each of the four waves loads

// Rows row0 .. row0+63 of the window in registers: lane = row, wave q holds
// snapshots q, q+4, ... (wave-uniform pointers).  window_prefetch only issues
// the loads, so a kernel can start the next chunk's loads before it computes
// on the current one; window_commit waits for them.
struct WindowRegs {
  const double* p[kPerWave];   // this wave's snapshot pointers (loaded once per block)
  double v[kPerWave];
};

__device__ inline void window_init(const double* const* __restrict__ snaps, int nsnap, WindowRegs& R) {
  const int q = __builtin_amdgcn_readfirstlane(threadIdx.x / kChunk);
#pragma unroll
  for (int i = 0; i < kPerWave; ++i) {
    const int j = q + 4 * i;
    R.p[i] = j < nsnap ? snaps[j] : nullptr;
  }
}

// Snapshot pointers come from a device table, so the compiler cannot tell
// they address global memory and would use flat loads, which also count
// against the LDS wait counter: the first LDS wait of the commit would then
// drain every prefetched load.  The cast makes them global loads.
typedef const __attribute__((address_space(1))) double* gptr_t;

__device__ inline void window_prefetch(int nsnap, long long n, long long row0, WindowRegs& R) {
  const int lane = threadIdx.x % kChunk;
  const int q = __builtin_amdgcn_readfirstlane(threadIdx.x / kChunk);
  const long long row = row0 + lane;
  const bool ok = row < n;
#pragma unroll
  for (int i = 0; i < kPerWave; ++i) {
    const int j = q + 4 * i;
    R.v[i] = (j < nsnap && ok) ? ((gptr_t)R.p[i])[row] : 0.0;
  }
}

// Centred rows into X (64 x ldx, LDS): X[r][j] = snap[off + j][row0 + r] -
// centre[r] for j < w, 0 for w <= j < wp.  The centring state (mean of the
// first w snapshots) and psi_new (mean of the last w) are summed per wave over
// its snapshots and the four partial sums combined in a fixed order.  Needs
// 256 threads; the caller synchronises before reading X.
__device__ inline void window_commit(const WindowRegs& R, int nsnap, int w, long long n, long long row0, double* X,
                                     int ldx, int wp, double* psi_new) {
  __shared__ double part_c[4][kChunk], part_n[4][kChunk], centre[kChunk];
  const int lane = threadIdx.x % kChunk;
  const int q = __builtin_amdgcn_readfirstlane(threadIdx.x / kChunk);
  const long long row = row0 + lane;
  const bool ok = row < n;
  const int off = nsnap - w;
  double c = 0.0, nw = 0.0;
#pragma unroll
  for (int i = 0; i < kPerWave; ++i) {
    const int j = q + 4 * i;
    if (j < w) c += R.v[i];
    if (j >= off && j < nsnap) nw += R.v[i];
  }
  part_c[q][lane] = c;
  part_n[q][lane] = nw;
  __syncthreads();
  if (threadIdx.x < kChunk) {
    const double cc = ((part_c[0][lane] + part_c[1][lane]) + part_c[2][lane]) + part_c[3][lane];
    const double nn = ((part_n[0][lane] + part_n[1][lane]) + part_n[2][lane]) + part_n[3][lane];
    centre[lane] = cc / (double)w;
    if (psi_new && ok) psi_new[row] = nn / (double)w;
  }
  __syncthreads();
  const double ce = centre[lane];
#pragma unroll
  for (int i = 0; i < kPerWave; ++i) {
    const int j = q + 4 * i;
    if (j >= off && j < nsnap) X[lane * ldx + (j - off)] = ok ? R.v[i] - ce : 0.0;
  }
  for (int j = w + q; j < wp; j += 4) X[lane * ldx + j] = 0.0;
}

// Row loader of the centred window; also writes psi_new for its rows.
struct WindowLoader {
  const double* const* snaps;   // device table of nsnap pointers
  int nsnap, w;
  long long n;
  double* psi_new;
  using Regs = WindowRegs;
  __device__ void init(Regs& R) const { window_init(snaps, nsnap, R); }
  __device__ void prefetch(long long row0, Regs& R) const { window_prefetch(nsnap, n, row0, R); }
  __device__ void commit(long long row0, const Regs& R, double* X, int ldx, int wp) const {
    window_commit(R, nsnap, w, n, row0, X, ldx, wp, psi_new);
  }
};

// Eigen-decomposition of the window Gram G (w x w, PSD) and the formation
// matrix T = V_m diag(1/sigma) (w x mp, zero padded), sigma (w), m_eff.
//  1. pivoted Cholesky G = P L L^T P^T + S, stopped when the largest remaining
//     diagonal entry is below eps * trace(G) (S is then below the rounding
//     level of G itself), giving L (w x r), r = numerical rank;
//  2. one-sided Jacobi on the columns of L: L W = U Sigma (U orthonormal), so
//     G = P U Sigma^2 U^T P^T without forming L^T L;
//  3. eigenvectors of G: V = P U; singular values sigma.
// One block of 256 threads.
__global__ void __launch_bounds__(256) basis_eig_kernel(const double* __restrict__ G, int w, int m,
                                                       double tau, double* __restrict__ sigma,
                                                       double* __restrict__ T, int mp,
                                                       int* __restrict__ m_eff_out) {
  constexpr int lda = kMaxBasis + 1;
  __shared__ double A[kMaxBasis * lda];   // G, then the eigenvectors V
  __shared__ double L[kMaxBasis * lda];   // pivoted Cholesky factor (permuted rows), then L W
  __shared__ double d[kMaxBasis], lam[kMaxBasis];
  __shared__ int perm[kMaxBasis], order[kMaxBasis];
  __shared__ int rank, piv, meff;
  __shared__ double tolc;
  const int t = threadIdx.x, nt = blockDim.x;
  for (int e = t; e < w * w; e += nt) A[(e / w) * lda + e % w] = G[e];
  for (int e = t; e < kMaxBasis * lda; e += nt) L[e] = 0.0;
  __syncthreads();
  if (t < w) {
    d[t] = A[t * lda + t];
    perm[t] = t;
  }
  if (t == 0) {
    double tr = 0.0;
    for (int i = 0; i < w; ++i) tr += fabs(A[i * lda + i]);
    tolc = 2.2e-16 * tr;
    rank = 0;
  }
  __syncthreads();
  // 1. pivoted Cholesky (rows of L in pivot order: row i <-> index perm[i])
  for (int k = 0; k < w; ++k) {
    if (t < kWave) {
      // pivot: largest remaining diagonal, ties to the lowest position (w <= 64: one wave)
      double best = (t >= k && t < w) ? d[perm[t]] : -INFINITY;
      int p = t;
      for (int o = kWave / 2; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, kWave);
        const int op = __shfl_xor(p, o, kWave);
        if (ob > best || (ob == best && op < p)) { best = ob; p = op; }
      }
      if (t == 0) {
        piv = best > tolc ? p : -1;
        if (piv >= 0) rank = k + 1;
      }
    }
    __syncthreads();
    if (piv < 0) break;
    if (piv != k) {   // swap pivot rows k <-> piv of perm and of L's first k columns
      if (t < k) {
        const double x = L[k * lda + t];
        L[k * lda + t] = L[piv * lda + t];
        L[piv * lda + t] = x;
      }
      __syncthreads();
      if (t == 0) {
        const int x = perm[k];
        perm[k] = perm[piv];
        perm[piv] = x;
      }
      __syncthreads();
    }
    const double lkk = sqrt(d[perm[k]]);
    for (int i = k + t; i < w; i += nt) {
      if (i == k) {
        L[k * lda + k] = lkk;
        continue;
      }
      double sacc = A[perm[i] * lda + perm[k]];
      double s4[4] = {0.0, 0.0, 0.0, 0.0};
      int j = 0;
      for (; j + 8 <= k; j += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) s4[u % 4] += L[i * lda + j + u] * L[k * lda + j + u];
      }
      for (; j < k; ++j) s4[0] += L[i * lda + j] * L[k * lda + j];
      sacc -= ((s4[0] + s4[1]) + s4[2]) + s4[3];
      const double lik = sacc / lkk;
      L[i * lda + k] = lik;
      d[perm[i]] -= lik * lik;
    }
    __syncthreads();
  }
  const int r = rank;
  // 2. one-sided Jacobi on the columns of L (w x r): rotate column pairs until
  //    they are orthogonal; then L W = U Sigma with the left singular vectors
  //    U of L, i.e. the eigenvectors of G (in pivot row order), and sigma^2
  //    the eigenvalues.  Pairs are scheduled round robin; each pair is one
  //    group of 8 lanes (dot products reduced by shuffles), one barrier per
  //    round.  A pair is rotated when |a_p.a_q| > sqrt(w) eps |a_p||a_q| (the
  //    rounding level of a length-w dot product); sweeps stop once no pair
  //    exceeds w eps, so rounding noise cannot keep them going.
  {
    const double tol_rot = sqrt((double)w) * 2.2e-16, tol_conv = (double)w * 2.2e-16;
    const int np = (r + 1) & ~1;
    const int P = np / 2;
    const int grp = t / 8, gl = t % 8;
    __shared__ int rotated;
    for (int sweep = 0; sweep < 60 && r > 1; ++sweep) {
      if (t == 0) rotated = 0;
      __syncthreads();
      for (int rd = 0; rd < np - 1; ++rd) {
        if (grp < P) {
          int p, q;
          if (grp == 0) {
            p = rd % (np - 1);
            q = np - 1;
          } else {
            p = (rd + grp) % (np - 1);
            q = (rd - grp + (np - 1)) % (np - 1);
          }
          if (p > q) { const int x = p; p = q; q = x; }
          if (q < r) {
            // rows gl, gl + 8, ... (w <= 64: at most 8 per lane, all loads in flight together)
            double xs[8], ys[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
              const int k = gl + 8 * i;
              xs[i] = k < w ? L[k * lda + p] : 0.0;
              ys[i] = k < w ? L[k * lda + q] : 0.0;
            }
            double aa = 0.0, bb = 0.0, gg = 0.0;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
              aa += xs[i] * xs[i];
              bb += ys[i] * ys[i];
              gg += xs[i] * ys[i];
            }
#pragma unroll
            for (int o = 4; o > 0; o >>= 1) {
              aa += __shfl_xor(aa, o, kWave);
              bb += __shfl_xor(bb, o, kWave);
              gg += __shfl_xor(gg, o, kWave);
            }
            const double lim = sqrt(aa * bb);
            if (aa > 0.0 && bb > 0.0 && fabs(gg) > tol_rot * lim) {
              const double zeta = (bb - aa) / (2.0 * gg);
              const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
              const double c = 1.0 / sqrt(1.0 + tt * tt), sn = c * tt;
#pragma unroll
              for (int i = 0; i < 8; ++i) {
                const int k = gl + 8 * i;
                if (k < w) {
                  L[k * lda + p] = c * xs[i] - sn * ys[i];
                  L[k * lda + q] = sn * xs[i] + c * ys[i];
                }
              }
              if (gl == 0 && fabs(gg) > tol_conv * lim) rotated = 1;
            }
          }
        }
        __syncthreads();
      }
      if (!rotated) break;
      __syncthreads();
    }
  }
  // eigenvalues: squared column norms, in descending order (stable rank sort)
  if (t < r) {
    double s2 = 0.0;
    for (int k = 0; k < w; ++k) s2 += L[k * lda + t] * L[k * lda + t];
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
  // 3. sigma, m_eff
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
  // V[:, i] = P L[:, order[i]] / sqrt(lam_i) in original index order (stored in A)
  for (int e = t; e < w * meff; e += nt) {
    const int row = e / meff, i = e % meff;
    A[perm[row] * lda + i] = L[row * lda + order[i]] / sqrt(lam[i]);
  }
  __syncthreads();
  // T[:, i] = sign_i V[:, i] / sigma_i, the sign making the largest |entry| positive
  for (int i = t; i < mp; i += nt) {
    if (i < meff) {
      int best = 0;
      double bv = -1.0;
      for (int rr = 0; rr < w; ++rr) {
        const double a = fabs(A[rr * lda + i]);
        if (a > bv) { bv = a; best = rr; }
      }
      const double sg = A[best * lda + i] >= 0.0 ? 1.0 : -1.0;
      const double inv = sg / sqrt(lam[i]);
      for (int rr = 0; rr < kMaxBasis; ++rr) T[rr * mp + i] = rr < w ? A[rr * lda + i] * inv : 0.0;
    } else {
      for (int rr = 0; rr < kMaxBasis; ++rr) T[rr * mp + i] = 0.0;
    }
  }
}

// Phi = X T for rows of the window (centred on the fly), on MFMA.
// C^T = T^T X^T so that each 16-lane group writes 16 consecutive rows of one
// column of Phi.  The next chunk's loads are in flight during the products.
// 256 threads; dynamic LDS: X (kChunk x (wp + 1)) then T (wp x (mp + 1)).
// TP = double, or float for the FP32 master copy (rounded once on store).
// meff is read from device memory (the eigen kernel's output), so the pass can
// be enqueued before the host learns m_eff.
template <typename TP>
__global__ void __launch_bounds__(256) basis_form_kernel(const double* const* __restrict__ snaps, int nsnap,
                                                         int w, long long n, const double* __restrict__ T,
                                                         int mp, int wp, const int* __restrict__ meff_d,
                                                         TP* __restrict__ Phi) {
  extern __shared__ double sh[];
  const int meff = *meff_d;
  const int ldx = wp + 1, ldt = mp + 1;
  double* X = sh;
  double* Ts = sh + kChunk * ldx;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  for (int e = threadIdx.x; e < wp * mp; e += blockDim.x) Ts[(e / mp) * ldt + e % mp] = T[e];
  const long long nchunks = (n + kChunk - 1) / kChunk;
  // two register buffers: the loads of the chunk after next are in flight
  // while the current chunk is committed and multiplied
  WindowRegs Ra, Rb;
  window_init(snaps, nsnap, Ra);
  window_init(snaps, nsnap, Rb);
  const long long G = gridDim.x;
  auto process = [&](WindowRegs& R, long long ch) {
    const long long row0 = ch * kChunk;
    __syncthreads();
    window_commit(R, nsnap, w, n, row0, X, ldx, wp, nullptr);
    __syncthreads();
    if (ch + 2 * G < nchunks) window_prefetch(nsnap, n, (ch + 2 * G) * kChunk, R);
    const int rb = wave;   // 16 rows per wave
    for (int mb = 0; mb * 16 < mp; ++mb) {
      if (mb * 16 >= meff) break;
      double4_t acc = (double4_t){0.0, 0.0, 0.0, 0.0};
      for (int k0 = 0; k0 < wp; k0 += 4) {
        const int k = k0 + lane / 16;
        const double a = Ts[k * ldt + mb * 16 + lane % 16];     // A = T^T: A[c][k] = T[k][c]
        const double b = X[(rb * 16 + lane % 16) * ldx + k];    // B[k][r] = X[r][k]
        acc = mfma_f64(a, b, acc);
      }
      const long long orow = row0 + rb * 16 + lane % 16;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int col = mb * 16 + lane / 16 + 4 * i;
        if (col < meff && orow < n) Phi[(size_t)col * n + orow] = (TP)acc[i];
      }
    }
  };
  long long ch = blockIdx.x;
  if (ch < nchunks) window_prefetch(nsnap, n, ch * kChunk, Ra);
  if (ch + G < nchunks) window_prefetch(nsnap, n, (ch + G) * kChunk, Rb);
  for (; ch < nchunks; ch += 2 * G) {
    process(Ra, ch);
    if (ch + G < nchunks) process(Rb, ch + G);
  }
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
  const int nb = (int)std::min<long long>(nchunks, kRedBlocks);
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
  HS_TRY(prof_begin(ctx, HS_PROF_BASIS_FORM));
  const size_t flds = ((size_t)kChunk * (wp + 1) + (size_t)wp * (mp + 1)) * sizeof(double);
  if (precision == HS_MIXED_FP32)
    hipLaunchKernelGGL(basis_form_kernel<float>, dim3(nb), dim3(256), flds, ctx->stream, tab, nsnap, w, n,
                       (const double*)T, mp, wp, (const int*)meff_d, (float*)Phi_out);
  else
    hipLaunchKernelGGL(basis_form_kernel<double>, dim3(nb), dim3(256), flds, ctx->stream, tab, nsnap, w, n,
                       (const double*)T, mp, wp, (const int*)meff_d, (double*)Phi_out);
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
  int* meff_d = reinterpret_cast<int*>(ctx->small + 3 * kMaxBasis * kMaxBasis);
  int me = 0;
  HS_TRY(readback(ctx, meff_d, sizeof(int), &me));
  *m_eff = me;
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

extern "C" hs_status basis_update_finish(hs_ctx* ctx, int32_t* m_eff) {
  if (!ctx || !m_eff) return HS_ERR_INVALID_ARG;
  if (!ctx->aux_pending) return ctx->fail(HS_ERR_INVALID_ARG, "no asynchronous basis update in flight");
  ctx->aux_pending = false;
  hipStream_t main = ctx->stream;
  ctx->stream = ctx->aux;
  const hs_status st = basis_complete(ctx, m_eff);
  ctx->stream = main;
  return st;
}
