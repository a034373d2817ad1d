// Discrete adjoint of one time step with every decision of the forward run
// frozen (schedule, sampled sets, subiteration count J, filter masks, basis):
//
//   full step (eq. hdm): R(gamma_k; gamma_{k-1}) = 0 with dR/dgamma_{k-1} = -I,
//     so lambda_{k-1} = J(gamma_k)^{-T} lambda_k;
//   hybrid step (eq. hybrid, Sec. 2.3.2, Sec. 2.3.4): the forward is, for
//     j = 1..J, a restricted solve R_S(v_j, t_j; p) = 0 on hat-S (t_1 = p on
//     the ring tilde-S), the fit y_j = A+ (v_j - psi_S) with A = Phi on the
//     hat-S rows, t_{j+1} = psi_T + Phi_T y_J; then gamma = psi + Phi y_J off
//     hat-S, v_J on it, and the frozen filter passes g <- M S g + (I - M) g.
//     Reverse mode runs these in the opposite order: the transposed passes
//     S^T M g + (I - M) g, y-bar = Phi^T g on the unsampled rows, and per
//     subiteration (last first) y-bar_j += Phi_T^T t-bar_{j+1},
//     v-bar_j += A+^T y-bar_j = Phi_S G+ y-bar_j, mu = J_S(u_j)^{-T} v-bar_j,
//     p-bar_S += mu, t-bar_j = -J_ST(u_j)^T mu; finally p-bar_T += t-bar_1.
//
// Transposed Jacobian blocks: cell p's row of J^T holds, for every stencil
// neighbour c, the transpose of the block that c's residual has for p,
// i.e. sum over the faces d of c that see p of O_c[d]^T.  The kernels
// recompute those blocks from the neighbour's stencil (no stored Jacobian),
// and the transposed system is relaxed with the same block-Jacobi sweeps as
// the forward Newton corrections (the iteration matrix D^{-T} O^T has the
// spectrum of the forward one).
#include "physics.hpp"

#include <algorithm>
#include <cstring>

namespace hs {

// Relative accuracy of every transposed solve (max norm).
constexpr double kAdjointRtol = 1e-12;

// Sum of the blocks O_c[d] of cell c's Jacobian over the faces d whose
// neighbour is `target` (several faces when a periodic line is short).
template <int NC>
__device__ inline void coupling_block(const Grid& g, const double* __restrict__ q, int c, int target,
                                      double B[NC * NC]) {
  Stencil<NC> st;
  load_stencil<NC>(g, q, c, st);
  double D[NC * NC], O[4][NC * NC];
  cell_jacobian<NC>(g, st, D, O);
#pragma unroll
  for (int e = 0; e < NC * NC; ++e) B[e] = 0.0;
#pragma unroll
  for (int d = 0; d < 4; ++d)
    if (st.idx[d] == target)
#pragma unroll
      for (int e = 0; e < NC * NC; ++e) B[e] += O[d][e];
}

// Relaxation data of the transposed system J^T x = v on the full mesh
// (hat == nullptr, count = ncell) or on the compact list hat with neighbour
// table nbr: coef[(e, a, b)] = (D_p^{-T} B_e^T)[a][b] for the distinct
// neighbour in direction e (0 for repeats, ghosts and cells outside the
// list), rhs = D_p^{-T} v_p; the max-norm contraction bound to part[Rho].
template <int NC>
__global__ void __launch_bounds__(kBlock) adj_coef_kernel(Grid g, const double* __restrict__ q, const int* __restrict__ hat,
                                const int* __restrict__ nbr, int count, int cap, const double* __restrict__ v,
                                double* __restrict__ coef, double* __restrict__ rhs, double* __restrict__ part) {
  __shared__ double lds[kBlock / kWave];
  double rho = 0.0;
  const int ndir = g.kind == HS_BURGERS_1D ? 2 : 4;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < count; p += gridDim.x * blockDim.x) {
    const int cell = hat ? hat[p] : p;
    int i, j;
    cell_ij(g, cell, i, j);
    double Di[NC * NC];
    {
      Stencil<NC> st;
      load_stencil<NC>(g, q, cell, st);
      double D[NC * NC], O[4][NC * NC];
      cell_jacobian<NC>(g, st, D, O);
      small_inverse<NC>(D, Di);
    }
    double rowsum[NC];
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      double b = 0.0;
#pragma unroll
      for (int k = 0; k < NC; ++k) b += Di[k * NC + a] * v[k * cap + p];
      rhs[a * cap + p] = b;
      rowsum[a] = 0.0;
    }
    int seen[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      int c = -1, key = -1;
      if (e < ndir) {
        if (hat) {
          key = nbr[e * cap + p];
          c = key >= 0 ? hat[key] : -1;
        } else {
          c = neighbour(g, i, j, e);
          if (c == cell) c = -1;
          key = c;
        }
      }
      for (int f = 0; f < e; ++f)
        if (key >= 0 && seen[f] == key) key = -1, c = -1;
      seen[e] = key;
      double B[NC * NC];
      if (c >= 0) coupling_block<NC>(g, q, c, cell, B);
#pragma unroll
      for (int a = 0; a < NC; ++a)
#pragma unroll
        for (int b = 0; b < NC; ++b) {
          double mv = 0.0;
          if (c >= 0) {
#pragma unroll
            for (int k = 0; k < NC; ++k) mv += Di[k * NC + a] * B[b * NC + k];
          }
          coef[((e * NC + a) * NC + b) * (size_t)cap + p] = mv;
          rowsum[a] += fabs(mv);
        }
    }
#pragma unroll
    for (int a = 0; a < NC; ++a) rho = nan_max(rho, rowsum[a]);
    if (!isfinite(rho)) rho = INFINITY;
  }
  rho = block_max(rho, lds);
  if (threadIdx.x == 0) stat_part(part, kStatRho, rho);
}

// t-bar on the ring: tb[t] = -sum over the distinct hat-S neighbours s of the
// ring cell of B_s^T mu[s], with B_s the block of s's residual for the ring
// cell (pos maps a cell to its hat-S index, -1 outside).
template <int NC>
__global__ void __launch_bounds__(kBlock) ring_coupling_kernel(Grid g, const double* __restrict__ q, const int* __restrict__ tilde, int l,
                                     const int* __restrict__ pos, const double* __restrict__ mu, int cap,
                                     double* __restrict__ tb) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= l) return;
  const int cell = tilde[t];
  int i, j;
  cell_ij(g, cell, i, j);
  const int ndir = g.kind == HS_BURGERS_1D ? 2 : 4;
  double acc[NC];
#pragma unroll
  for (int a = 0; a < NC; ++a) acc[a] = 0.0;
  int seen[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    int s = -1;
    if (e < ndir) {
      s = neighbour(g, i, j, e);
      if (s == cell) s = -1;
    }
    for (int f = 0; f < e; ++f)
      if (s >= 0 && seen[f] == s) s = -1;
    seen[e] = s;
    const int ps = s >= 0 ? pos[s] : -1;
    if (ps < 0) continue;
    double B[NC * NC];
    coupling_block<NC>(g, q, s, cell, B);
#pragma unroll
    for (int a = 0; a < NC; ++a)
#pragma unroll
      for (int b = 0; b < NC; ++b) acc[a] -= B[b * NC + a] * mu[b * cap + ps];
  }
#pragma unroll
  for (int a = 0; a < NC; ++a) tb[a * cap + t] = acc[a];
}

// Correlation weights of (-delta^2/4)^n for offsets -n..n (symmetric).
__device__ inline double shapiro_weight(int n, int k) {
  const int a = k < 0 ? -k : k;
  if (n == 1) {
    const double w[2] = {0.5, -0.25};
    return w[a];
  }
  if (n == 2) {
    const double w[3] = {6.0 / 16.0, -4.0 / 16.0, 1.0 / 16.0};
    return w[a];
  }
  const double w[4] = {20.0 / 64.0, -15.0 / 64.0, 6.0 / 64.0, -1.0 / 64.0};
  return w[a];
}

// One transposed filter pass along an axis: out = S^T h with h = mask . in
// (mask == nullptr: h = in), S = I - K E (E extends the line by n values,
// periodic wrap or repetition of the end value).  With comb != nullptr the
// output is S^T h + (1 - cmask) . comb (the untouched part of a gated pass).
__global__ void shapiro_t_kernel(Grid g, const double* __restrict__ in, const uint8_t* __restrict__ mask,
                                 double* __restrict__ out, int axis, int n, const double* __restrict__ comb,
                                 const uint8_t* __restrict__ cmask) {
  const long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (k >= (long long)g.nc * g.ncell) return;
  const int a = (int)(k / g.ncell), cell = (int)(k % g.ncell);
  int i, j;
  cell_ij(g, cell, i, j);
  const int len = axis == 0 ? g.nx : g.ny;
  const int x0 = axis == 0 ? i : j;
  auto at = [&](int x) {
    const int cc = axis == 0 ? x + g.nx * j : i + g.nx * x;
    const double v = in[(size_t)a * g.ncell + cc];
    return mask ? (mask[cc] ? v : 0.0) : v;
  };
  double acc = at(x0);
  if (g.bc == HS_BC_PERIODIC) {
    // the source cell x0 - k of weight c_k lands on x0 for every k
    for (int s = -n; s <= n; ++s) {
      int x = x0 - s;
      x = wrap_index(x, len);
      acc -= shapiro_weight(n, s) * at(x);
    }
  } else {
    // source x contributes c_k for every k with clamp(x + k) == x0
    for (int x = x0 - n; x <= x0 + n; ++x) {
      if (x < 0 || x >= len) continue;
      double w = 0.0;
      for (int s = -n; s <= n; ++s) {
        int y = x + s;
        y = y < 0 ? 0 : (y >= len ? len - 1 : y);
        if (y == x0) w += shapiro_weight(n, s);
      }
      if (w != 0.0) acc -= w * at(x);
    }
  }
  if (comb && !cmask[cell]) acc += comb[k];
  out[k] = acc;
}

// Partial sums Phi^T x over rows: the listed cells (all components, x in the
// compact layout x[a * cap + p]) or, with list == nullptr, every row whose cell
// is not flagged in skip (x in the state layout).
template <int MP>
__global__ void __launch_bounds__(256) adj_project_kernel(const double* __restrict__ Phi, long long n, int m,
                                                          int nc, int ncell, const int* __restrict__ list,
                                                          int count, const uint8_t* __restrict__ skip,
                                                          const double* __restrict__ x, double* __restrict__ part) {
  __shared__ double wsum[4][MP];
  double acc[MP];
#pragma unroll
  for (int c = 0; c < MP; ++c) acc[c] = 0.0;
  const long long rows = list ? (long long)nc * count : n;
  for (long long row = blockIdx.x * (long long)blockDim.x + threadIdx.x; row < rows;
       row += (long long)gridDim.x * blockDim.x) {
    long long dof = row;
    double xv;
    if (list) {
      const long long a = row / count, p = row % count;
      dof = a * ncell + list[p];
      xv = x[a * ncell + p];
    } else {
      if (skip && skip[row % ncell]) continue;
      xv = x[row];
    }
#pragma unroll
    for (int c = 0; c < MP; ++c)
      if (c < m) acc[c] += Phi[(size_t)c * n + dof] * xv;
  }
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
#pragma unroll
  for (int c = 0; c < MP; ++c) {
    const double v = wave_sum(acc[c]);
    if (lane == 0) wsum[wave][c] = v;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < m; c += blockDim.x)
    part[(size_t)blockIdx.x * MP + c] = ((wsum[0][c] + wsum[1][c]) + wsum[2][c]) + wsum[3][c];
}

// out = add + sum of the partials (fixed order); z = Gp out if Gp != nullptr.
__global__ void __launch_bounds__(256) adj_project_finish_kernel(const double* __restrict__ part, int nb, int mp,
                                                                 int m, const double* __restrict__ add,
                                                                 double* __restrict__ out,
                                                                 const double* __restrict__ Gp,
                                                                 double* __restrict__ z) {
  __shared__ double b[kMaxBasis];
  const int t = threadIdx.x;
  const int lane = t % kWave, wave = t / kWave, nw = blockDim.x / kWave;
  for (int c = wave; c < m; c += nw) {
    double s = 0.0;
    for (int k = lane; k < nb; k += kWave) s += part[(size_t)k * mp + c];
    s = wave_sum(s);
    if (lane == 0) b[c] = (add ? add[c] : 0.0) + s;
  }
  __syncthreads();
  if (t < m) {
    out[t] = b[t];
    if (Gp) {
      double s = 0.0;
      for (int c = 0; c < m; ++c) s += Gp[t * m + c] * b[c];
      z[t] = s;
    }
  }
}

// out[a * cap + p] = (add ? add[a * cap + p] : 0) + sum_c Phi[dof, c] z[c] on the listed cells.
__global__ void adj_expand_kernel(const double* __restrict__ Phi, long long n, int m, int nc, int ncell,
                                  const int* __restrict__ list, int count, const double* __restrict__ z,
                                  const double* __restrict__ add, double* __restrict__ out) {
  __shared__ double zl[kMaxBasis];
  if (threadIdx.x < m) zl[threadIdx.x] = z[threadIdx.x];
  __syncthreads();
  const long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (k >= (long long)nc * count) return;
  const long long a = k / count, p = k % count;
  const long long dof = a * ncell + list[p];
  double s = 0.0;
  for (int c = 0; c < m; ++c) s += Phi[(size_t)c * n + dof] * zl[c];
  const long long o = a * ncell + p;
  out[o] = (add ? add[o] : 0.0) + s;
}

// Compact gather x[a * cap + p] = v[a * ncell + list[p]] and scatter-add
// v[a * ncell + list[p]] += x[a * cap + p] (cells of a list are distinct).
__global__ void gather_kernel(int nc, int ncell, const int* __restrict__ list, int count,
                              const double* __restrict__ v, double* __restrict__ x) {
  const long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (k >= (long long)nc * count) return;
  const long long a = k / count, p = k % count;
  x[a * ncell + p] = v[a * ncell + list[p]];
}

__global__ void scatter_add_kernel(int nc, int ncell, const int* __restrict__ list, int count,
                                   const double* __restrict__ x, double* __restrict__ v) {
  const long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (k >= (long long)nc * count) return;
  const long long a = k / count, p = k % count;
  v[a * ncell + list[p]] += x[a * ncell + p];
}

// v[dof] -= x[a * cap + p] on the listed cells; out[i] = g[i] off the cells
// flagged in mask, 0 on them.
__global__ void scatter_sub_kernel(int nc, int ncell, const int* __restrict__ list, int count,
                                   const double* __restrict__ x, double* __restrict__ v) {
  const long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (k >= (long long)nc * count) return;
  const long long a = k / count, p = k % count;
  v[a * ncell + list[p]] -= x[a * ncell + p];
}

__global__ void unmasked_copy_kernel(long long n, int ncell, const uint8_t* __restrict__ mask,
                                     const double* __restrict__ g, double* __restrict__ out) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) out[i] = mask[i % ncell] ? 0.0 : g[i];
}

__global__ void zero_kernel(double* __restrict__ x, long long n) {
  const long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (k < n) x[k] = 0.0;
}

// ------------------------------------------------------------------- host
static int pad16(int m) { return (m + 15) / 16 * 16; }

static hs_status project(hs_ctx* ctx, const double* Phi, int m, const int* list, int count, const uint8_t* skip,
                         const double* x, const double* add, double* out, const double* Gp, double* z) {
  const long long rows = list ? (long long)ctx->nc * count : ctx->n;
  const int nb = (int)std::max<long long>(1, std::min<long long>((rows + kBlock - 1) / kBlock, 512));
  const int mp = pad16(m);
  const long long n = ctx->n;
  switch (mp) {
    case 16: HS_LAUNCH(ctx, adj_project_kernel<16>, nb, kBlock, Phi, n, m, ctx->nc, ctx->ncell, list, count, skip, x, ctx->red); break;
    case 32: HS_LAUNCH(ctx, adj_project_kernel<32>, nb, kBlock, Phi, n, m, ctx->nc, ctx->ncell, list, count, skip, x, ctx->red); break;
    case 48: HS_LAUNCH(ctx, adj_project_kernel<48>, nb, kBlock, Phi, n, m, ctx->nc, ctx->ncell, list, count, skip, x, ctx->red); break;
    default: HS_LAUNCH(ctx, adj_project_kernel<64>, nb, kBlock, Phi, n, m, ctx->nc, ctx->ncell, list, count, skip, x, ctx->red); break;
  }
  HS_LAUNCH(ctx, adj_project_finish_kernel, 1, 256, ctx->red, nb, mp, m, add, out, Gp, z);
  return HS_OK;
}

// Transposed relaxation data at state q, then the solve into x (compact).
static hs_status transposed_solve(hs_ctx* ctx, const double* q, const hs_samples* s, const double* v, double* x,
                                  int* sweeps) {
  const int* hat = s ? s->hat : nullptr;
  const int* nbr = s ? s->nbr : nullptr;
  const int count = s ? s->n_s : ctx->ncell;
  const int nbs = stat_blocks(count);
  if (ctx->nc == 1)
    HS_LAUNCH(ctx, adj_coef_kernel<1>, nbs, kBlock, ctx->g, q, hat, nbr, count, ctx->ncell, v, ctx->coef, ctx->rhs,
              ctx->part);
  else
    HS_LAUNCH(ctx, adj_coef_kernel<4>, nbs, kBlock, ctx->g, q, hat, nbr, count, ctx->ncell, v, ctx->coef, ctx->rhs,
              ctx->part);
  unsigned long long st[kStatSlots];
  HS_TRY(finish_stats(ctx, nbs, 1u << kStatRho, 0u, st));
  const double rho = bits_to_double(st[kStatRho]);
  if (!std::isfinite(rho)) return ctx->fail(HS_ERR_NONFINITE, "non-finite transposed Jacobian");
  return relax_solve(ctx, s, ctx->coef, ctx->rhs, rho, kAdjointRtol, x, sweeps);
}

}  // namespace hs

using namespace hs;

extern "C" {

hs_status hdm_step_adjoint(hs_ctx* ctx, const double* q_out, const double* lam_in, double* lam_out,
                           hs_step_info* info) {
  if (!ctx || !q_out || !lam_in || !lam_out || lam_out == q_out) return HS_ERR_INVALID_ARG;
  if (info) std::memset(info, 0, sizeof *info);
  const double* v = lam_in;
  if (lam_out == lam_in) {
    HIP_TRY(ctx, hipMemcpyAsync(ctx->adj, lam_in, ctx->n * 8, hipMemcpyDeviceToDevice, ctx->stream));
    v = ctx->adj;
  }
  int sweeps = 0;
  HS_TRY(transposed_solve(ctx, q_out, nullptr, v, lam_out, &sweeps));
  if (info) info->lin_sweeps = sweeps;
  return hs_sync(ctx);
}

hs_status rom_hybrid_step_adjoint_psi(hs_ctx* ctx, const double* Phi, int32_t m, const hs_htape* tape,
                                      const double* lam_in, double* lam_out, double* lam_psi, hs_step_info* info) {
  if (!ctx || !Phi || !tape || !lam_in || !lam_out || tape->ctx != ctx) return HS_ERR_INVALID_ARG;
  if (lam_psi && (lam_psi == lam_in || lam_psi == lam_out)) return HS_ERR_INVALID_ARG;
  if (!tape->replayed) return ctx->fail(HS_ERR_INVALID_ARG, "adjoint needs a replayed tape");
  if (m != tape->m) return ctx->fail(HS_ERR_INVALID_ARG, "basis size differs from the replayed step");
  if (tape->precision != HS_FP64) return ctx->fail(HS_ERR_INVALID_ARG, "adjoint needs an FP64 basis");
  const hs_samples* s = tape->s;
  const int ncell = ctx->ncell, nc = ctx->nc;
  const long long N = ctx->n;
  const int nbN = blocks_for(N);
  if (info) std::memset(info, 0, sizeof *info);

  // (1) transposed filter passes, last first; g ends in buf[cur]
  double* buf[3] = {ctx->adj, ctx->gf, ctx->gtmp};
  int cur = 0;
  HIP_TRY(ctx, hipMemcpyAsync(buf[0], lam_in, N * 8, hipMemcpyDeviceToDevice, ctx->stream));
  for (int k = tape->npass - 1; k >= 0; --k) {
    const uint8_t* mk = tape->masks + (size_t)k * ncell;
    const int nord = tape->passes[k];
    double* gin = buf[cur];
    double* tmp = buf[(cur + 1) % 3];
    double* gout = buf[(cur + 2) % 3];
    if (ctx->g.kind == HS_BURGERS_1D) {
      HS_LAUNCH(ctx, shapiro_t_kernel, nbN, kBlock, ctx->g, gin, mk, gout, 0, nord, gin, mk);
    } else {
      // S = S_y S_x, so S^T = S_x^T S_y^T
      HS_LAUNCH(ctx, shapiro_t_kernel, nbN, kBlock, ctx->g, gin, mk, tmp, 1, nord, (const double*)nullptr,
                (const uint8_t*)nullptr);
      HS_LAUNCH(ctx, shapiro_t_kernel, nbN, kBlock, ctx->g, (const double*)tmp, (const uint8_t*)nullptr, gout, 0,
                nord, gin, mk);
    }
    cur = (cur + 2) % 3;
    if (info) info->filter_passes += 1;
  }
  double* g = buf[cur];
  double* vbar0 = buf[(cur + 1) % 3];   // compact over hat-S
  double* tbar = buf[(cur + 2) % 3];    // compact over tilde-S
  double* vbar = ctx->u;                // compact over hat-S
  double* mu = ctx->rho;                // compact over hat-S
  double* sm = ctx->small;

  // (2) reconstruction transpose: y-bar = Phi^T g off hat-S; v-bar = g on hat-S;
  // psi-bar = g off hat-S (psi + Phi y there)
  HS_TRY(project(ctx, Phi, m, nullptr, 0, s->mask, g, nullptr, sm + kSmAdjY0, nullptr, nullptr));
  HS_LAUNCH(ctx, gather_kernel, blocks_for((long long)nc * s->n_s), kBlock, nc, ncell, s->hat, s->n_s,
            (const double*)g, vbar0);
  HS_LAUNCH(ctx, zero_kernel, nbN, kBlock, lam_out, N);
  if (lam_psi) HS_LAUNCH(ctx, unmasked_copy_kernel, nbN, kBlock, N, ncell, (const uint8_t*)s->mask, (const double*)g,
                         lam_psi);

  // (3) subiterations in reverse
  int sweeps = 0;
  for (int j = tape->J - 1; j >= 0; --j) {
    const bool last = j == tape->J - 1;
    const double* uj = tape->us + (size_t)j * N;
    // t_{j+1} = psi on the ring + Phi y_j: its adjoint also goes to psi-bar
    if (lam_psi && !last && s->l > 0)
      HS_LAUNCH(ctx, scatter_add_kernel, blocks_for((long long)nc * s->l), kBlock, nc, ncell, s->tilde, s->l,
                (const double*)tbar, lam_psi);
    if (last)
      HS_LAUNCH(ctx, adj_project_finish_kernel, 1, 256, sm + kSmAdjY0, 1, 64, m, (const double*)nullptr,
                sm + kSmAdjY, (const double*)tape->gp, sm + kSmAdjZ);
    else
      HS_TRY(project(ctx, Phi, m, s->tilde, s->l, nullptr, tbar, nullptr, sm + kSmAdjY, tape->gp, sm + kSmAdjZ));
    HS_LAUNCH(ctx, adj_expand_kernel, blocks_for((long long)nc * s->n_s), kBlock, Phi, N, m, nc, ncell, s->hat,
              s->n_s, (const double*)(sm + kSmAdjZ), last ? (const double*)vbar0 : (const double*)nullptr, vbar);
    if (lam_psi) {
      // y_j = A^+ (v_j - psi on hat-S): psi-bar -= (A^+)^T y-bar = Phi_S z there
      HS_LAUNCH(ctx, adj_expand_kernel, blocks_for((long long)nc * s->n_s), kBlock, Phi, N, m, nc, ncell, s->hat,
                s->n_s, (const double*)(sm + kSmAdjZ), (const double*)nullptr, ctx->R);
      HS_LAUNCH(ctx, scatter_sub_kernel, blocks_for((long long)nc * s->n_s), kBlock, nc, ncell, s->hat, s->n_s,
                (const double*)ctx->R, lam_psi);
    }
    HS_TRY(transposed_solve(ctx, uj, s, vbar, mu, &sweeps));
    HS_LAUNCH(ctx, scatter_add_kernel, blocks_for((long long)nc * s->n_s), kBlock, nc, ncell, s->hat, s->n_s,
              (const double*)mu, lam_out);
    if (s->l > 0) {
      if (nc == 1)
        HS_LAUNCH(ctx, ring_coupling_kernel<1>, blocks_for(s->l), kBlock, ctx->g, uj, s->tilde, s->l, s->pos,
                  (const double*)mu, ncell, tbar);
      else
        HS_LAUNCH(ctx, ring_coupling_kernel<4>, blocks_for(s->l), kBlock, ctx->g, uj, s->tilde, s->l, s->pos,
                  (const double*)mu, ncell, tbar);
    }
  }
  if (s->l > 0)
    HS_LAUNCH(ctx, scatter_add_kernel, blocks_for((long long)nc * s->l), kBlock, nc, ncell, s->tilde, s->l,
              (const double*)tbar, lam_out);
  if (info) {
    info->lin_sweeps = sweeps;
    info->subiters = tape->J;
    info->n_s = s->n_s;
    info->l = s->l;
  }
  return hs_sync(ctx);
}

hs_status rom_hybrid_step_adjoint(hs_ctx* ctx, const double* Phi, int32_t m, const hs_htape* tape,
                                  const double* lam_in, double* lam_out, hs_step_info* info) {
  return rom_hybrid_step_adjoint_psi(ctx, Phi, m, tape, lam_in, lam_out, nullptr, info);
}

}  // extern "C"
