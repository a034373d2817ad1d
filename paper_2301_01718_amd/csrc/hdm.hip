// Full-order model: context lifetime, residual (A1), Jacobian products (A2)
// and the Newton solve (A3) of the backward-Euler HDM (eq. hdm), on the full
// mesh or restricted to a compact list of sampled cells (eq. partial_hdm2).
//
// Linear systems are solved by (block-)Jacobi relaxation: per cell the
// iteration is delta <- b - sum_X M_X delta[X] with M_X = D^{-1} O_X and
// b = -D^{-1} R.  The residual/Jacobian kernel also returns the contraction
// bound rho = max_cells max_rows sum |M_X|.  When rho < 1 the sweep count
// ceil(log(eta) / log(rho)) guarantees the requested accuracy eta of each
// Newton correction in the max norm without any reduction inside the sweeps
// (the scalar Burgers systems).  Otherwise (Euler, whose components have very
// different scales, so the max-norm bound is loose although the iteration
// contracts) the sweeps run in batches and stop on the fixed-point difference.
// eta follows the residual (inexact Newton), floored at lin_rtol.
#include "physics.hpp"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>

namespace hs {

// ----------------------------------------------------------- small kernels
__global__ void fill_u64_kernel(unsigned long long* p, int n, unsigned long long v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void max_abs_kernel(const double* __restrict__ x, long long n, double* __restrict__ part) {
  __shared__ double lds[kBlock / kWave];
  double m = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    m = nan_max(m, fabs(x[i]));
  m = block_max(m, lds);
  if (threadIdx.x == 0) stat_part(part, kStatQMax, m);
}

// Read-backs go through a host buffer that the device writes directly
// (pinned, coherent, mapped): one wave stores the words, fences at system
// scope and then stores the tag; the host spins on the tag instead of waiting
// for a copy engine and the stream's completion signal.
constexpr size_t kPinBytes = 65536;

__global__ void post_kernel(const uint32_t* __restrict__ src, int words, uint32_t* dst, uint32_t* tagp,
                            unsigned tag) {
  post_words(src, words, dst, tagp, tag);
}

// One block: reduce the partials of the flagged slots (fixed strided order and
// a fixed tree) and store them as bit patterns in the stats slots; with dst,
// the first wave then posts all slots to the host buffer.
__global__ void finish_stats_kernel(const double* __restrict__ part, int nb, unsigned max_mask,
                                    unsigned sum_mask, unsigned long long* __restrict__ stats, uint32_t* dst,
                                    uint32_t* tagp, unsigned tag) {
  __shared__ double lds[kBlock / kWave];
  __shared__ unsigned long long sv[kStatSlots];   // all slots, as posted
  if (threadIdx.x < kStatSlots) sv[threadIdx.x] = stats[threadIdx.x];
  const unsigned mask = max_mask | sum_mask;
  // the partials of every flagged slot are loaded together (per slot the
  // order is the strided one and the tree below is fixed)
  double v[kStatSlots];
#pragma unroll
  for (int slot = 0; slot < kStatSlots; ++slot) v[slot] = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
#pragma unroll
    for (int slot = 0; slot < kStatSlots; ++slot) {
      if (!((mask >> slot) & 1u)) continue;
      const double x = part[slot * kPartCap + b];
      v[slot] = ((max_mask >> slot) & 1u) ? nan_max(v[slot], x) : v[slot] + x;
    }
  }
#pragma unroll
  for (int slot = 0; slot < kStatSlots; ++slot) {
    if (!((mask >> slot) & 1u)) continue;
    const double r = ((max_mask >> slot) & 1u) ? block_max(v[slot], lds) : block_sum(v[slot], lds);
    if (threadIdx.x == 0) {
      stats[slot] = dbits(r);
      sv[slot] = dbits(r);
    }
  }
  if (dst == nullptr) return;
  __syncthreads();
  if (threadIdx.x < kWave) post_words(reinterpret_cast<const uint32_t*>(sv), kStatSlots * 2, dst, tagp, tag);
}

static unsigned next_tag(hs_ctx* ctx) {
  ctx->pin_tag = ctx->pin_tag + 1u == 0u ? 1u : ctx->pin_tag + 1u;
  return ctx->pin_tag;
}

static uint32_t* pin_tag_dev(hs_ctx* ctx) {
  return reinterpret_cast<uint32_t*>(static_cast<char*>(ctx->dpin) + kPinBytes);
}

// The read-back ring after the main area: kPostSlots slots of kSlotBytes
// (data, then the tag word at kPostWords).
constexpr int kPostSlots = 8;
constexpr size_t kSlotBytes = 256;
constexpr size_t kRingOffset = kPinBytes + 256;

// Spin until the tag arrives at t; after 20 ms fall back to a blocking wait
// on the stream (a long queue ahead, or an error to report).
static hs_status await_tag_at(hs_ctx* ctx, const volatile uint32_t* t, unsigned tag) {
  const auto start = std::chrono::steady_clock::now();
  for (unsigned spin = 1;; ++spin) {
    if (*t == tag) break;
    if ((spin & 1023u) == 0u && std::chrono::steady_clock::now() - start > std::chrono::milliseconds(20)) {
      HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
      if (*t != tag) return ctx->fail(HS_ERR_HIP, "read-back: the device did not deliver the result");
      break;
    }
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  return HS_OK;
}

static hs_status await_tag(hs_ctx* ctx, unsigned tag) {
  return await_tag_at(
      ctx, reinterpret_cast<const volatile uint32_t*>(static_cast<const char*>(ctx->hpin) + kPinBytes), tag);
}

PostSlot post_slot(hs_ctx* ctx) {
  PostSlot p;
  p.slot = (int)(ctx->post_next++ % kPostSlots);
  char* base = static_cast<char*>(ctx->dpin) + kRingOffset + (size_t)p.slot * kSlotBytes;
  p.dst = reinterpret_cast<uint32_t*>(base);
  p.tagp = reinterpret_cast<uint32_t*>(base) + kPostWords;
  p.tag = next_tag(ctx);
  return p;
}

hs_status await_post(hs_ctx* ctx, const PostSlot& p, void* out, size_t bytes) {
  if (bytes > kPostWords * 4) return ctx->fail(HS_ERR_INVALID_ARG, "post larger than a ring slot");
  const char* base = static_cast<const char*>(ctx->hpin) + kRingOffset + (size_t)p.slot * kSlotBytes;
  HS_TRY(await_tag_at(ctx, reinterpret_cast<const volatile uint32_t*>(base) + kPostWords, p.tag));
  std::memcpy(out, base, bytes);
  return HS_OK;
}

hs_status readback(hs_ctx* ctx, const void* dsrc, size_t bytes, void* hdst) {
  if (bytes > kPinBytes) return ctx->fail(HS_ERR_INVALID_ARG, "readback too large");
  if (bytes % 4 != 0 || reinterpret_cast<uintptr_t>(dsrc) % 4 != 0)
    return ctx->fail(HS_ERR_INVALID_ARG, "readback of a non-word-aligned range");
  const unsigned tag = next_tag(ctx);
  HS_LAUNCH(ctx, post_kernel, 1, kWave, static_cast<const uint32_t*>(dsrc), (int)(bytes / 4),
            static_cast<uint32_t*>(ctx->dpin), pin_tag_dev(ctx), tag);
  HS_TRY(await_tag(ctx, tag));
  std::memcpy(hdst, ctx->hpin, bytes);
  return HS_OK;
}

hs_status prof_begin(hs_ctx* ctx, int cls) {
  if (ctx->prof_class != cls || cls == 0) return HS_OK;
  if (ctx->prof_used + 2 > ctx->prof_ev.size()) {
    for (int k = 0; k < 64; ++k) {
      hipEvent_t e;
      HIP_TRY(ctx, hipEventCreate(&e));
      ctx->prof_ev.push_back(e);
    }
  }
  HIP_TRY(ctx, hipEventRecord(ctx->prof_ev[ctx->prof_used], ctx->stream));
  return HS_OK;
}

hs_status prof_end(hs_ctx* ctx, int cls, double bytes) {
  if (ctx->prof_class != cls || cls == 0) return HS_OK;
  HIP_TRY(ctx, hipEventRecord(ctx->prof_ev[ctx->prof_used + 1], ctx->stream));
  ctx->prof_used += 2;
  ctx->prof_bytes.push_back(bytes);
  return HS_OK;
}

hs_status zero_stats(hs_ctx* ctx) {
  HS_LAUNCH(ctx, fill_u64_kernel, 1, 64, ctx->stats, (int)kStatSlots, 0ull);
  return HS_OK;
}

hs_status read_stats(hs_ctx* ctx, unsigned long long* out) {
  return readback(ctx, ctx->stats, kStatSlots * sizeof(unsigned long long), out);
}

hs_status finish_stats(hs_ctx* ctx, int nb, unsigned max_mask, unsigned sum_mask, unsigned long long* out) {
  if (!out) {
    HS_LAUNCH(ctx, finish_stats_kernel, 1, kBlock, ctx->part, nb, max_mask, sum_mask, ctx->stats, nullptr,
              nullptr, 0u);
    return HS_OK;
  }
  const unsigned tag = next_tag(ctx);
  HS_LAUNCH(ctx, finish_stats_kernel, 1, kBlock, ctx->part, nb, max_mask, sum_mask, ctx->stats,
            static_cast<uint32_t*>(ctx->dpin), pin_tag_dev(ctx), tag);
  HS_TRY(await_tag(ctx, tag));
  std::memcpy(out, ctx->hpin, kStatSlots * sizeof(unsigned long long));
  return HS_OK;
}

// The per-block maxima of |x| only (slot kStatQMax of ctx->part, *nb of them),
// for a kernel that reduces them itself.
hs_status max_abs_partials(hs_ctx* ctx, const double* x, long long n, int* nb) {
  *nb = blocks_for(n, kBlock, 1024);
  HS_LAUNCH(ctx, max_abs_kernel, *nb, kBlock, x, n, ctx->part);
  return HS_OK;
}

hs_status max_abs_launch(hs_ctx* ctx, const double* x, long long n) {
  int nb;
  HS_TRY(max_abs_partials(ctx, x, n, &nb));
  return finish_stats(ctx, nb, 1u << kStatQMax, 0u);
}

hs_status max_abs(hs_ctx* ctx, const double* x, long long n, double* out) {
  const int nb = blocks_for(n, kBlock, 1024);
  HS_LAUNCH(ctx, max_abs_kernel, nb, kBlock, x, n, ctx->part);
  unsigned long long st[kStatSlots];
  HS_TRY(finish_stats(ctx, nb, 1u << kStatQMax, 0u, st));
  *out = bits_to_double(st[kStatQMax]);
  return HS_OK;
}

// ------------------------------------------------------------ dense blocks
// --------------------------------------------------------- residual kernel
template <int NC>
__global__ void residual_kernel(Grid g, const double* __restrict__ q, const double* __restrict__ qp,
                                double* __restrict__ R) {
  const int cell = blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= g.ncell) return;
  Stencil<NC> st;
  load_stencil<NC>(g, q, cell, st);
  double p[NC], r[NC];
#pragma unroll
  for (int a = 0; a < NC; ++a) p[a] = qp[a * g.ncell + cell];
  cell_residual<NC>(g, st, p, r);
#pragma unroll
  for (int a = 0; a < NC; ++a) R[a * g.ncell + cell] = r[a];
}

// The same residual with each thread marching down K rows of one column (a
// block covers 256 columns): the column's K + 2 states along y are loaded
// once and kept in registers, so of the five stencil loads per cell only the
// two along x remain (hits in the lines the wave's own loads bring in).  The
// stencil values, and so the arithmetic, are the per-cell kernel's.  Rows past
// the mesh (a ragged last band) are skipped.
template <int NC, int K>
__global__ void __launch_bounds__(256) residual_col_kernel(Grid g, const double* __restrict__ q,
                                                           const double* __restrict__ qp, double* __restrict__ R) {
  const int i = blockIdx.x * 256 + threadIdx.x, j0 = blockIdx.y * K;
  if (i >= g.nx || j0 >= g.ny) return;
  const int kn = min(K, g.ny - j0);
  const int c_dn = neighbour(g, i, j0, 2), c_up = neighbour(g, i, j0 + kn - 1, 3);
  // w[s]: the state below the band (s = 0), its rows (1..kn), the state above it (kn + 1)
  double w[K + 2][NC];
  double pv[K][NC];
#pragma unroll
  for (int s = 0; s < K + 2; ++s) {
    const int c = s == 0 ? c_dn : (s <= kn ? i + g.nx * (j0 + s - 1) : (s == kn + 1 ? c_up : -1));
#pragma unroll
    for (int a = 0; a < NC; ++a) w[s][a] = c >= 0 ? q[(size_t)a * g.ncell + c] : 0.0;
  }
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int a = 0; a < NC; ++a) pv[k][a] = k < kn ? qp[(size_t)a * g.ncell + i + g.nx * (j0 + k)] : 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (k >= kn) break;
    const int j = j0 + k, cell = i + g.nx * j;
    Stencil<NC> st;
    st.self = cell;
#pragma unroll
    for (int a = 0; a < NC; ++a) st.c[a] = w[k + 1][a];
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const int nb = neighbour(g, i, j, d);
      st.idx[d] = nb;
#pragma unroll
      for (int a = 0; a < NC; ++a) st.nb[d][a] = nb < 0 ? g.inflow : q[(size_t)a * g.ncell + nb];
    }
    st.idx[2] = neighbour(g, i, j, 2);
    st.idx[3] = neighbour(g, i, j, 3);
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      st.nb[2][a] = w[k][a];
      st.nb[3][a] = w[k + 2][a];
    }
    double r[NC];
    cell_residual<NC>(g, st, pv[k], r);
#pragma unroll
    for (int a = 0; a < NC; ++a) R[(size_t)a * g.ncell + cell] = r[a];
  }
}

// c = a + b, one element per thread: the streaming reference.
__global__ void __launch_bounds__(kBlock) stream_add_kernel(long long n, const double* __restrict__ a,
                                                            const double* __restrict__ b, double* __restrict__ c) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e < n) c[e] = a[e] + b[e];
}

// out = J(q) v
template <int NC>
__global__ void __launch_bounds__(kBlock) jvp_kernel(Grid g, const double* __restrict__ q, const double* __restrict__ v,
                           double* __restrict__ out) {
  const int cell = blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= g.ncell) return;
  Stencil<NC> st;
  load_stencil<NC>(g, q, cell, st);
  double D[NC * NC], O[4][NC * NC];
  cell_jacobian<NC>(g, st, D, O);
  double acc[NC];
#pragma unroll
  for (int a = 0; a < NC; ++a) {
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < NC; ++b) s += D[a * NC + b] * v[b * g.ncell + cell];
    acc[a] = s;
  }
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    const int nb = st.idx[d];
    if (nb < 0 || nb == cell) continue;
#pragma unroll
    for (int a = 0; a < NC; ++a)
#pragma unroll
      for (int b = 0; b < NC; ++b) acc[a] += O[d][a * NC + b] * v[b * g.ncell + nb];
  }
#pragma unroll
  for (int a = 0; a < NC; ++a) out[a * g.ncell + cell] = acc[a];
}

// Residual + Jacobi iteration data on the full mesh (hat == nullptr) or on the
// compact list hat[0..count) whose in-set neighbours are nbr[d * cap + p].
template <int NC>
__global__ void __launch_bounds__(kBlock) resjac_kernel(Grid g, const double* __restrict__ q, const double* __restrict__ qp,
                              const int* __restrict__ hat, const int* __restrict__ nbr, int count,
                              int cap, double* __restrict__ coef, double* __restrict__ rhs,
                              double* __restrict__ part) {
  __shared__ double lds[kBlock / kWave];
  double rmax = 0.0, rho = 0.0;
  bool bad = false;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < count; p += gridDim.x * blockDim.x) {
    const int cell = hat ? hat[p] : p;
    Stencil<NC> st;
    load_stencil<NC>(g, q, cell, st);
    double pv[NC], R[NC];
#pragma unroll
    for (int a = 0; a < NC; ++a) pv[a] = qp[a * g.ncell + cell];
    cell_residual<NC>(g, st, pv, R);
    double D[NC * NC], O[4][NC * NC];
    cell_jacobian<NC>(g, st, D, O);
    if (hat) {
#pragma unroll
      for (int d = 0; d < 4; ++d)
        if (nbr[d * cap + p] < 0)
#pragma unroll
          for (int e = 0; e < NC * NC; ++e) O[d][e] = 0.0;   // fixed (tilde-S) or ghost value
    }
    double Di[NC * NC];
    small_inverse<NC>(D, Di);
    double rowsum[NC];
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      rmax = nan_max(rmax, fabs(R[a]));
      bad |= !isfinite(R[a]);
      double b = 0.0;
#pragma unroll
      for (int c = 0; c < NC; ++c) b -= Di[a * NC + c] * R[c];
      rhs[a * cap + p] = b;
      rowsum[a] = 0.0;
    }
#pragma unroll
    for (int d = 0; d < 4; ++d) {
#pragma unroll
      for (int a = 0; a < NC; ++a)
#pragma unroll
        for (int b = 0; b < NC; ++b) {
          double m = 0.0;
#pragma unroll
          for (int c = 0; c < NC; ++c) m += Di[a * NC + c] * O[d][c * NC + b];
          coef[((d * NC + a) * NC + b) * (size_t)cap + p] = m;
          rowsum[a] += fabs(m);
        }
    }
#pragma unroll
    for (int a = 0; a < NC; ++a) rho = nan_max(rho, rowsum[a]);
    if (!isfinite(rho)) bad = true;
  }
  rmax = block_max(bad ? INFINITY : rmax, lds);
  rho = block_max(rho, lds);
  if (threadIdx.x == 0) {
    stat_part(part, kStatResMax, rmax);
    stat_part(part, kStatRho, rho);
  }
}

// ------------------------------------------------------------ Newton solve
hs_status linear_solve(hs_ctx* ctx, const hs_samples* s, double rho, double eta, double* q, int* sweeps);

template <int NC>
static hs_status resjac_launch(hs_ctx* ctx, const double* q, const double* q_prev, const hs_samples* s,
                               unsigned long long* st, bool finish = true) {
  const int* hat = s ? s->hat : nullptr;
  const int* nbr = s ? s->nbr : nullptr;
  const int count = s ? s->n_s : ctx->ncell;
  const int nbs = stat_blocks(count);
  HS_TRY(prof_begin(ctx, HS_PROF_RESJAC));
  HS_LAUNCH(ctx, resjac_kernel<NC>, nbs, kBlock, ctx->g, q, q_prev, hat, nbr, count, ctx->ncell, ctx->coef,
            ctx->rhs, ctx->part);
  // reads: state of the cell (+ 4 neighbours, counted once), q_prev, the
  // list entries; writes: 4 NC x NC relaxation blocks and the NC-vector b
  HS_TRY(prof_end(ctx, HS_PROF_RESJAC,
                  (double)count * (8.0 * NC * 2 + 8.0 * (4 * NC * NC + NC) + (hat ? 4.0 * 5 : 0.0))));
  if (!finish) return HS_OK;
  return finish_stats(ctx, nbs, (1u << kStatResMax) | (1u << kStatRho), 0u, st);
}

// One Newton iteration's residual/Jacobian whose decision is taken on the
// device by the first sweep launch (NewtonCtrl): that launch runs while the
// host reads the decision back.  *total: the correction's sweep count (<= 0:
// no sweeps ran).
template <int NC>
static hs_status resjac_ctrl(hs_ctx* ctx, double* q, const double* q_prev, double tol, const hs_samples* s,
                             unsigned long long* st, int* total, int sub_check = 0, double eps_y = 0.0,
                             bool tol_from_qmax = false) {
  HS_TRY(resjac_launch<NC>(ctx, q, q_prev, s, nullptr, false));
  NewtonCtrl c;
  c.sub_check = sub_check;
  c.eps_y = eps_y;
  if (tol_from_qmax) c.rtol_qmax = ctx->p.newton_rtol;
  c.part = ctx->part;
  c.nb = stat_blocks(s ? s->n_s : ctx->ncell);
  c.tol = tol;
  c.scale = std::max(1.0, tol / ctx->p.newton_rtol);
  c.lin_rtol = ctx->p.lin_rtol;
  c.lin_maxit = ctx->p.lin_maxit;
  c.stats = ctx->stats;
  c.dst = static_cast<uint32_t*>(ctx->dpin);
  c.tagp = pin_tag_dev(ctx);
  c.tag = next_tag(ctx);
  const size_t pidx = ctx->prof_bytes.size();
  HS_TRY(prof_begin(ctx, HS_PROF_SWEEP));
  HS_TRY(relax_first_ctrl(ctx, s, q, c));
  HS_TRY(prof_end(ctx, HS_PROF_SWEEP, 0.0));
  HS_TRY(await_tag(ctx, c.tag));
  std::memcpy(st, ctx->hpin, kStatSlots * sizeof(unsigned long long));
  *total = (int)(long long)st[kStatSweeps];
  // a launch that ran sweeps moved a launch's algorithmic bytes
  if (*total > 0 && ctx->prof_bytes.size() > pidx) ctx->prof_bytes[pidx] = sweep_launch_bytes(ctx, s);
  return HS_OK;
}

hs_status newton_first_ctrl(hs_ctx* ctx, double* q, const double* q_prev, double tol, const hs_samples* s,
                            int sub_check, double eps_y, unsigned long long* st, int* total, bool tol_from_qmax) {
  if (!newton_ctrl_ok(ctx, s)) return ctx->fail(HS_ERR_INVALID_ARG, "device Newton decision needs scalar tiles");
  if (tol_from_qmax && !(ctx->p.newton_rtol > 0.0))
    return ctx->fail(HS_ERR_INVALID_ARG, "tolerance from max |q_prev| needs newton_rtol > 0");
  return resjac_ctrl<1>(ctx, q, q_prev, tol, s, st, total, sub_check, eps_y, tol_from_qmax);
}

hs_status newton_first_launch(hs_ctx* ctx, const double* q, const double* q_prev, const hs_samples* s,
                              unsigned long long* st) {
  if (ctx->nc == 1) return resjac_launch<1>(ctx, q, q_prev, s, st);
  return resjac_launch<4>(ctx, q, q_prev, s, st);
}

template <int NC>
static hs_status newton_impl(hs_ctx* ctx, double* q, const double* q_prev, double tol,
                             const hs_samples* s, hs_step_info* info, const double* primed) {
  const int maxit = ctx->p.newton_maxit;
  const double lin_rtol = ctx->p.lin_rtol;
  int sweeps_total = 0;
  const bool ctrl = newton_ctrl_ok(ctx, s);
  for (int it = 0;; ++it) {
    double rmax, rho;
    int dev_total = 0;
    if (it == 0 && primed) {
      rmax = primed[0];
      rho = primed[1];
      dev_total = (int)primed[2];
    } else {
      unsigned long long st[kStatSlots];
      if (ctrl) HS_TRY(resjac_ctrl<NC>(ctx, q, q_prev, tol, s, st, &dev_total));
      else HS_TRY(resjac_launch<NC>(ctx, q, q_prev, s, st));
      rmax = bits_to_double(st[kStatResMax]);
      rho = bits_to_double(st[kStatRho]);
    }
    if (!std::isfinite(rmax))
      return ctx->fail(HS_ERR_NONFINITE, "non-finite residual in Newton solve");
    if (info) {
      info->residual_inf = rmax;
    }
    if (rmax <= tol) {
      if (info) {
        info->newton_iters += it;
        info->lin_sweeps += sweeps_total;
      }
      return HS_OK;
    }
    if (it >= maxit) {
      char msg[160];
      std::snprintf(msg, sizeof msg, "Newton: ||R||_inf = %.3e > %.3e after %d iterations", rmax, tol, it);
      return ctx->fail(HS_ERR_NOT_CONVERGED, msg);
    }
    if (!std::isfinite(rho)) return ctx->fail(HS_ERR_NONFINITE, "non-finite Jacobian");
    if (dev_total > 0) {
      // the device chose a fixed-count correction and its first launch ran
      // min(S, total - 1) sweeps from x_1 = rhs into d0 (or onto q)
      const int first = std::min(tile_sweeps(ctx, s), dev_total - 1);
      if (dev_total - 1 > first)
        HS_TRY(relax_sweeps(ctx, s, ctx->coef, ctx->rhs, ctx->d0, dev_total - 1 - first, q, false, nullptr));
      sweeps_total += dev_total;
      continue;
    }
    // Inexact Newton: the correction needs relative accuracy eta ~ ||R|| (the
    // quadratic term is of that size anyway) and never beyond what brings the
    // next residual to a tenth of the tolerance; lin_rtol is the floor.
    const double scale = std::max(1.0, tol / ctx->p.newton_rtol);
    const double eta = std::min(0.1, std::max(lin_rtol, std::max(rmax / scale, 0.1 * tol / rmax)));
    HS_TRY(linear_solve(ctx, s, rho, eta, q, &sweeps_total));
  }
}

// x[a * cap + p] = src[a * cap + p] for p < count (compact layout).
__global__ void copy_compact_kernel(int nc, int count, int cap, const double* __restrict__ src,
                                    double* __restrict__ dst) {
  const long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (k >= (long long)nc * count) return;
  const long long a = k / count, p = k % count;
  dst[a * cap + p] = src[a * cap + p];
}

// Relaxation of the system whose data (ctx->coef, rhs) is loaded, to relative
// accuracy eta in the max norm; the sweeps start from x_1 = rhs.  With q the
// solution is added to the state q (Newton update), otherwise written to x
// (compact layout).  rho < 1 with a sweep count within lin_maxit: that many
// sweeps (rho^nsw <= eta); otherwise batches of 8 with the stop test on the
// fixed-point difference and the rate estimated from successive batches
// (error <= r / (1 - r) * ||x_{k+1} - x_k||).
static hs_status linear_solve_impl(hs_ctx* ctx, const hs_samples* s, const double* rhs, double rho, double eta,
                                   double* q, double* x, int* sweeps) {
  int nsw = 1;
  if (rho > 0.0 && rho < 1.0) nsw = std::max(1, (int)std::ceil(std::log(eta) / std::log(rho)));
  const double* last = rhs;
  int used;
  if (rho < 1.0 && nsw <= ctx->p.lin_maxit) {
    HS_TRY(relax_sweeps(ctx, s, ctx->coef, rhs, rhs, nsw - 1, q, false, &last));
    used = nsw;
  } else {
    constexpr int kBatch = 8;
    int k = 1;
    double prev_diff = -1.0, rate = 0.9;
    bool conv = false;
    while (k < ctx->p.lin_maxit) {
      const int b = std::min(kBatch, ctx->p.lin_maxit - k);
      const double* nxt;
      HS_TRY(relax_sweeps(ctx, s, ctx->coef, rhs, last, b, nullptr, true, &nxt));
      last = nxt;
      k += b;
      const int nb = use_tiles(ctx, s) ? (s ? s->ntiles : ctx->ntx * ctx->nty) : blocks_for(s ? s->n_s : ctx->ncell);
      unsigned long long st[kStatSlots];
      HS_TRY(finish_stats(ctx, nb, (1u << kStatDiff) | (1u << kStatDnorm), 0u, st));
      const double diff = bits_to_double(st[kStatDiff]);
      const double dn = bits_to_double(st[kStatDnorm]);
      if (!std::isfinite(diff)) return ctx->fail(HS_ERR_NONFINITE, "non-finite relaxation iterate");
      if (prev_diff > 0.0 && diff > 0.0) rate = std::min(0.99, std::pow(diff / prev_diff, 1.0 / b));
      prev_diff = diff;
      if (diff == 0.0 || (rate < 1.0 && rate / (1.0 - rate) * diff <= eta * dn)) {
        conv = true;
        break;
      }
    }
    used = k;
    if (!conv) return ctx->fail(HS_ERR_NOT_CONVERGED, "block-Jacobi relaxation did not converge");
    if (q) HS_TRY(relax_sweeps(ctx, s, ctx->coef, rhs, last, 0, q, false, nullptr));
  }
  if (x) {
    const int count = s ? s->n_s : ctx->ncell;
    if (last != x)
      HS_LAUNCH(ctx, (copy_compact_kernel), blocks_for((long long)ctx->nc * count), kBlock, ctx->nc, count,
                ctx->ncell, last, x);
  }
  if (sweeps) *sweeps += used;
  return HS_OK;
}

hs_status linear_solve(hs_ctx* ctx, const hs_samples* s, double rho, double eta, double* q, int* sweeps) {
  return linear_solve_impl(ctx, s, ctx->rhs, rho, eta, q, nullptr, sweeps);
}

hs_status relax_solve(hs_ctx* ctx, const hs_samples* s, const double* coef, const double* rhs, double rho,
                      double eta, double* x, int* sweeps) {
  if ((s ? s->n_s : ctx->ncell) == 0) return HS_OK;
  if (coef != ctx->coef) return ctx->fail(HS_ERR_INVALID_ARG, "relaxation data must be in the context");
  return linear_solve_impl(ctx, s, rhs, rho, eta, nullptr, x, sweeps);
}

hs_status newton_solve(hs_ctx* ctx, double* q, const double* q_prev, double tol, const hs_samples* s,
                       hs_step_info* info, const double* primed) {
  if (s && s->n_s == 0) return HS_OK;
  if (ctx->nc == 1) return newton_impl<1>(ctx, q, q_prev, tol, s, info, primed);
  return newton_impl<4>(ctx, q, q_prev, tol, s, info, primed);
}

}  // namespace hs

using namespace hs;

// ================================================================ C ABI
extern "C" {

const char* hs_status_string(hs_status s) {
  switch (s) {
    case HS_OK: return "ok";
    case HS_ERR_INVALID_ARG: return "invalid argument";
    case HS_ERR_SHAPE: return "shape beyond capacity";
    case HS_ERR_NOT_CONVERGED: return "not converged";
    case HS_ERR_RANK: return "rank deficient";
    case HS_ERR_NONFINITE: return "non-finite value";
    case HS_ERR_HIP: return "HIP runtime error";
    case HS_ERR_OOM: return "out of device memory";
    default: return "unknown status";
  }
}

const char* hs_last_error(const hs_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

static hs_status alloc(hs_ctx* ctx, void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes < 256 ? 256 : bytes);
  if (e != hipSuccess) return ctx->fail(HS_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
  return HS_OK;
}

hs_status hs_destroy(hs_ctx* ctx) {
  if (!ctx) return HS_ERR_INVALID_ARG;
  void* bufs[] = {ctx->u,    ctx->R,     ctx->rhs,    ctx->d0,  ctx->d1,    ctx->coef, ctx->rho,
                  ctx->gf,   ctx->gtmp,  ctx->rcell,  ctx->rcell2, ctx->red, ctx->small, ctx->stats,
                  ctx->ibuf, ctx->part, ctx->adj};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  for (hipEvent_t e : ctx->prof_ev) (void)hipEventDestroy(e);
  if (ctx->aux) {
    (void)hipStreamSynchronize(ctx->aux);
    (void)hipStreamDestroy(ctx->aux);
  }
  if (ctx->aux_ready) (void)hipEventDestroy(ctx->aux_ready);
  if (ctx->hpin) (void)hipHostFree(ctx->hpin);
  delete ctx;
  return HS_OK;
}

hs_status hs_create(const hs_problem* pr, void* stream, hs_ctx** out) {
  if (!pr || !out) return HS_ERR_INVALID_ARG;
  *out = nullptr;
  if (pr->kind < HS_BURGERS_1D || pr->kind > HS_EULER_2D) return HS_ERR_INVALID_ARG;
  if (pr->bc < HS_BC_INFLOW_OUTFLOW || pr->bc > HS_BC_TRANSMISSIVE) return HS_ERR_INVALID_ARG;
  if (pr->nx < 1 || pr->ny < 1 || (pr->kind == HS_BURGERS_1D && pr->ny != 1)) return HS_ERR_INVALID_ARG;
  if (pr->bc == HS_BC_INFLOW_OUTFLOW && pr->kind != HS_BURGERS_1D) return HS_ERR_INVALID_ARG;
  if (!(pr->dx > 0) || !(pr->dt > 0) || (pr->kind != HS_BURGERS_1D && !(pr->dy > 0))) return HS_ERR_INVALID_ARG;
  if (pr->m_max < 1 || pr->m_max > kMaxBasis || pr->w_max < 1 || pr->w_max > kMaxBasis) return HS_ERR_INVALID_ARG;
  if ((long long)pr->nx * pr->ny > (1ll << 28)) return HS_ERR_SHAPE;

  hs_ctx* ctx = new hs_ctx();
  ctx->p = *pr;
  if (ctx->p.newton_rtol <= 0) ctx->p.newton_rtol = 1e-13;
  if (ctx->p.newton_maxit <= 0) ctx->p.newton_maxit = 30;
  if (ctx->p.lin_rtol <= 0 || ctx->p.lin_rtol >= 1) ctx->p.lin_rtol = 1e-10;
  if (ctx->p.lin_maxit <= 0) ctx->p.lin_maxit = 400;
  ctx->stream = static_cast<hipStream_t>(stream);
  (void)hipGetDevice(&ctx->device);
  if (hipDeviceGetAttribute(&ctx->max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device) != hipSuccess)
    ctx->max_lds = 65536;
  if (hipDeviceGetAttribute(&ctx->num_cu, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess ||
      ctx->num_cu < 1)
    ctx->num_cu = 256;
  ctx->nc = pr->kind == HS_EULER_2D ? 4 : 1;
  ctx->ncell = pr->nx * pr->ny;
  ctx->n = ctx->nc * ctx->ncell;
  ctx->nnb = 4;
  Grid& g = ctx->g;
  g.nx = pr->nx;
  g.ny = pr->ny;
  g.ncell = ctx->ncell;
  g.nc = ctx->nc;
  g.kind = pr->kind;
  g.bc = pr->bc;
  g.lx = pr->dt / pr->dx;
  g.ly = pr->kind == HS_BURGERS_1D ? 0.0 : pr->dt / pr->dy;
  g.gamma = pr->gamma;
  g.inflow = pr->inflow;
  {
    int l = 0;
    while ((1LL << l) < (long long)g.nx) ++l;
    g.nx_shift = 32 + l;
    g.nx_mul = (unsigned long long)((((unsigned __int128)1 << g.nx_shift) + (unsigned)g.nx - 1) / (unsigned)g.nx);
  }
  set_tile_geometry(ctx, pr);

  const size_t N = ctx->n, NC = ctx->ncell, nc = ctx->nc;
  hs_status st = HS_OK;
  auto A = [&](void** p, size_t bytes) {
    if (st == HS_OK) st = alloc(ctx, p, bytes);
  };
  A((void**)&ctx->u, N * 8);
  A((void**)&ctx->R, N * 8);
  A((void**)&ctx->rhs, N * 8);
  A((void**)&ctx->d0, N * 8);
  A((void**)&ctx->d1, N * 8);
  A((void**)&ctx->coef, 4 * nc * nc * NC * 8);
  A((void**)&ctx->rho, N * 8);
  A((void**)&ctx->gf, N * 8);
  A((void**)&ctx->gtmp, N * 8);
  A((void**)&ctx->rcell, NC * 8);
  A((void**)&ctx->rcell2, NC * 8);
  A((void**)&ctx->red, (size_t)kRedBlocks * kMaxBasis * kMaxBasis * 8);
  A((void**)&ctx->small, 16 * kMaxBasis * kMaxBasis * 8);
  A((void**)&ctx->stats, kStatSlots * 8);
  A((void**)&ctx->ibuf, (NC + 8192) * 4);
  A((void**)&ctx->adj, N * 8);
  A((void**)&ctx->part, (size_t)kStatSlots * kPartCap * 8);
  if (st == HS_OK) {
    if (hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->aux_ready, hipEventDisableTiming) != hipSuccess)
      st = ctx->fail(HS_ERR_HIP, "stream/event creation");
  }
  if (st == HS_OK) {
    const size_t pin = kRingOffset + kPostSlots * kSlotBytes;
    hipError_t e = hipHostMalloc(&ctx->hpin, pin, hipHostMallocCoherent | hipHostMallocMapped);
    if (e == hipSuccess) e = hipHostGetDevicePointer(&ctx->dpin, ctx->hpin, 0);
    if (e == hipSuccess) std::memset(ctx->hpin, 0, pin);
    if (e != hipSuccess) st = ctx->fail(HS_ERR_OOM, "hipHostMalloc");
  }
  if (st != HS_OK) {
    hs_destroy(ctx);
    return st;
  }
  *out = ctx;
  return HS_OK;
}

hs_status hs_prof_enable(hs_ctx* ctx, int32_t cls) {
  if (!ctx || cls < HS_PROF_NONE || cls > HS_PROF_STREAM) return HS_ERR_INVALID_ARG;
  ctx->prof_class = cls;
  ctx->prof_used = 0;
  ctx->prof_bytes.clear();
  return HS_OK;
}

hs_status hs_prof_read(hs_ctx* ctx, double* total_ms, int32_t* launches, double* bytes) {
  if (!ctx || !total_ms || !launches || !bytes) return HS_ERR_INVALID_ARG;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  double ms = 0.0, b = 0.0;
  for (size_t k = 0; k + 1 < ctx->prof_used; k += 2) {
    float e = 0.f;
    HIP_TRY(ctx, hipEventElapsedTime(&e, ctx->prof_ev[k], ctx->prof_ev[k + 1]));
    ms += e;
  }
  for (double x : ctx->prof_bytes) b += x;
  *total_ms = ms;
  *launches = (int32_t)(ctx->prof_used / 2);
  *bytes = b;
  ctx->prof_used = 0;
  ctx->prof_bytes.clear();
  return HS_OK;
}

hs_status hs_set_option(hs_ctx* ctx, int32_t option, int64_t value) {
  if (!ctx) return HS_ERR_INVALID_ARG;
  if (option == HS_OPT_TILED_SWEEPS && value >= 0 && value <= 2) {
    ctx->tiled = (int)value;
    return HS_OK;
  }
  if (option == HS_OPT_FIT_CHOLESKY && (value == 0 || value == 1)) {
    ctx->fit_chol = (int)value;
    return HS_OK;
  }
  if (option == HS_OPT_SMALL_PINV && (value == 0 || value == 1)) {
    ctx->small_pinv = (int)value;
    return HS_OK;
  }
  return HS_ERR_INVALID_ARG;
}

hs_status hs_sync(hs_ctx* ctx) {
  if (!ctx) return HS_ERR_INVALID_ARG;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return HS_OK;
}

hs_status hs_stream_add(hs_ctx* ctx, const double* a, const double* b, double* c, int64_t n) {
  if (!ctx || !a || !b || !c || n < 0 || n > (1LL << 38) || c == a || c == b) return HS_ERR_INVALID_ARG;
  if (n == 0) return HS_OK;
  HS_TRY(prof_begin(ctx, HS_PROF_STREAM));
  HS_LAUNCH(ctx, stream_add_kernel, (unsigned)((n + kBlock - 1) / kBlock), kBlock, (long long)n, a, b, c);
  return prof_end(ctx, HS_PROF_STREAM, 24.0 * (double)n);
}

hs_status hs_residual(hs_ctx* ctx, const double* q, const double* q_prev, double* R) {
  if (!ctx || !q || !q_prev || !R) return HS_ERR_INVALID_ARG;
  const int nb = blocks_for(ctx->ncell);
  HS_TRY(prof_begin(ctx, HS_PROF_RESIDUAL));
  // Column bands pay on large 2D meshes (measured, same bits: 2D Burgers
  // 4096^2 with 4 rows 103 -> 76 us; Euler 2048^2 with 2 rows 115 -> 99 us,
  // 512^2 9.3 -> 8.8 us); on 2D Burgers up to 1024^2 one cell per thread is
  // about 5 % faster.
  const Grid& g = ctx->g;
  const dim3 bands1((g.nx + 255) / 256, (g.ny + 3) / 4), bands4((g.nx + 255) / 256, (g.ny + 1) / 2);
  if (ctx->nc == 1 && g.ny > 1 && ctx->ncell > (1 << 20))
    HS_LAUNCH(ctx, (residual_col_kernel<1, 4>), bands1, 256, g, q, q_prev, R);
  else if (ctx->nc == 1)
    HS_LAUNCH(ctx, residual_kernel<1>, nb, kBlock, g, q, q_prev, R);
  else if (g.ny > 1 && ctx->ncell >= (1 << 18))
    HS_LAUNCH(ctx, (residual_col_kernel<4, 2>), bands4, 256, g, q, q_prev, R);
  else
    HS_LAUNCH(ctx, residual_kernel<4>, nb, kBlock, g, q, q_prev, R);
  // reads q and q_prev once, writes R
  return prof_end(ctx, HS_PROF_RESIDUAL, 24.0 * ctx->n);
}

hs_status hs_jvp(hs_ctx* ctx, const double* q, const double* v, double* out) {
  if (!ctx || !q || !v || !out) return HS_ERR_INVALID_ARG;
  const int nb = blocks_for(ctx->ncell);
  if (ctx->nc == 1) HS_LAUNCH(ctx, jvp_kernel<1>, nb, kBlock, ctx->g, q, v, out);
  else HS_LAUNCH(ctx, jvp_kernel<4>, nb, kBlock, ctx->g, q, v, out);
  return HS_OK;
}

hs_status hdm_step(hs_ctx* ctx, const double* q_prev, double* q_out, hs_step_info* info) {
  if (!ctx || !q_prev || !q_out || q_prev == q_out) return HS_ERR_INVALID_ARG;
  if (info) std::memset(info, 0, sizeof *info);
  double qmax;
  HS_TRY(max_abs(ctx, q_prev, ctx->n, &qmax));
  if (!std::isfinite(qmax)) return ctx->fail(HS_ERR_NONFINITE, "non-finite q_prev");
  const double tol = ctx->p.newton_rtol * std::max(1.0, qmax);
  HIP_TRY(ctx, hipMemcpyAsync(q_out, q_prev, ctx->n * 8, hipMemcpyDeviceToDevice, ctx->stream));
  HS_TRY(newton_solve(ctx, q_out, q_prev, tol, nullptr, info));
  if (info) info->n_s = ctx->ncell;
  return HS_OK;
}

}  // extern "C"
