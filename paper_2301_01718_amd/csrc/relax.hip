// Block-Jacobi relaxation sweeps with temporal blocking in LDS.
//
// One sweep is x_new = b - sum_X M_X x_old[X] per cell (the relaxation of the
// Newton correction, and of the transposed systems of the adjoint).  A
// launch of the tiled kernel covers up to S sweeps: a workgroup stages one
// tile of the grid plus an S-cell halo (periodic wrap where the grid wraps),
// keeps its cells' M_X and b in registers, and runs the sweeps in LDS; the
// region whose values are exact shrinks by one cell per sweep, so after s <= S
// sweeps the tile itself holds the exact iterate.  On a sampled set the
// active tiles are those holding a sampled cell; other cells of a tile carry
// no unknown (their value stays 0 and no sampled cell reads it, exactly as in
// the compact list form).  Per cell the products are accumulated in the
// order of the compact-list sweep, so both give the same iterates bit for bit.
// Per launch each region cell is read once instead of once per sweep; tiles
// are used where they are dense (the full mesh, compact sampled sets).
#include "physics.hpp"

#include <algorithm>

namespace hs {

// Threads per tile of the scalar 2D kernels.  A sampled set activates a few
// hundred 16 x 16 tiles, fewer workgroups than the chip holds: 512 threads
// (two region cells each) give a launch twice the waves of 256 (sampled-set
// sweeps 367 -> 306 us per hybrid step on 1024^2).  The full mesh's 32 x 32
// tiles take 1024 threads (three region cells each, 60 registers instead of
// 177; full step 0.42 -> 0.37 ms).  Euler's 4 x 4 blocks keep 256 threads
// (more threads per tile leave fewer registers per thread and spill).
constexpr int kSweepThreadsSet = 512;
constexpr int kSweepThreadsMesh = 1024;

template <int NC, int TSX, int TSY, int S, int NT>
struct TileCfg {
  static constexpr int RW = TSX + 2 * S;
  static constexpr int RH = TSY == 1 ? 1 : TSY + 2 * S;
  static constexpr int R = RW * RH;
  static constexpr int CPT = (R + NT - 1) / NT;   // region cells per thread
};

// The sweep count of a Newton correction (0: none here, converged or
// non-finite; -1: the batch form), as the host computes it: inexact Newton
// accuracy eta from the residual, rho^nsw <= eta.
__device__ inline int newton_sweeps(double rmax, double rho, const NewtonCtrl& c) {
  if (!isfinite(rmax) || rmax <= c.tol || !isfinite(rho)) return 0;
  const double eta = fmin(0.1, fmax(c.lin_rtol, fmax(rmax / c.scale, 0.1 * c.tol / rmax)));
  int nsw = 1;
  if (rho > 0.0 && rho < 1.0) {
    const double k = ceil(log(eta) / log(rho));
    nsw = k > (double)c.lin_maxit ? c.lin_maxit + 1 : max(1, (int)k);
  }
  return (rho < 1.0 && nsw <= c.lin_maxit) ? nsw : -1;
}

// tiles: active tile ids (nullptr: tile = blockIdx.x); pos/nbr: compact index
// of a cell and of its in-set neighbours (nullptr: full mesh, index = cell).
// xin: iterate before the launch (compact layout x[a * cap + p]); the result
// goes to xout, or is added to the state q when q != nullptr.  With record,
// max |x_last - x_prev| and max |x_last| of the tile go to the statistics.
// With ctl.part the launch first takes the Newton decision (NewtonCtrl): nsw
// and q then follow from it, and block 0 posts the statistics to the host.
// The grid is ntiles rounded up to a multiple of 8 workgroups, in an
// XCD-aware order: workgroups are dealt to the eight XCDs round robin (block b
// runs on XCD b % 8), so block b takes tile slot (b % 8) per + b / 8 and each
// XCD sweeps a contiguous run of the (row-ordered) tile list, whose staged
// halos overlap and are then read from that XCD's own L2.
template <int NC, int TSX, int TSY, int S, bool COEF_REG, int NT>
__global__ void __launch_bounds__(NT) tile_sweep_kernel(
    Grid g, const int* __restrict__ tiles, int ntiles, int ntx, const int* __restrict__ pos,
    const int* __restrict__ nbr, int cap, const double* __restrict__ coef, const double* __restrict__ rhs,
    const double* __restrict__ xin, double* __restrict__ xout, double* __restrict__ q, int nsw, int record,
    double* __restrict__ part, const NewtonCtrl ctl) {
  using C = TileCfg<NC, TSX, TSY, S, NT>;
  constexpr int RW = C::RW, RH = C::RH, R = C::R, CPT = C::CPT;
  constexpr bool ONE_D = TSY == 1;
  constexpr int NDIR = ONE_D ? 2 : 4;
  __shared__ double xs[2][NC][R];
  __shared__ double lds[NT / kWave];
  __shared__ int s_total;
  if (ctl.part != nullptr) {
    // every block reduces the same partials (max: exact in any order)
    double rm = 0.0, rh = 0.0;
    for (int b = threadIdx.x; b < ctl.nb; b += NT) {
      rm = nan_max(rm, ctl.part[kStatResMax * kPartCap + b]);
      rh = nan_max(rh, ctl.part[kStatRho * kPartCap + b]);
    }
    rm = block_max(rm, lds);
    rh = block_max(rh, lds);
    if (threadIdx.x == 0) {
      NewtonCtrl c = ctl;
      if (c.rtol_qmax > 0.0) {
        // the tolerance the host forms from the same max |q_prev|
        const double qm = __longlong_as_double((long long)ctl.stats[kStatQMax]);
        c.tol = c.rtol_qmax * fmax(1.0, qm);
        c.scale = fmax(1.0, c.tol / c.rtol_qmax);
      }
      const double dy = __longlong_as_double((long long)ctl.stats[kStatDy]);
      const int total = (c.sub_check && dy < c.eps_y) ? 0 : newton_sweeps(rm, rh, c);
      s_total = total;
      if (blockIdx.x == 0) {
        ctl.stats[kStatResMax] = dbits(rm);
        ctl.stats[kStatRho] = dbits(rh);
        ctl.stats[kStatSweeps] = (unsigned long long)(long long)total;
      }
    }
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x < kWave)
      post_words(reinterpret_cast<const uint32_t*>(ctl.stats), kStatSlots * 2, ctl.dst, ctl.tagp, ctl.tag);
    const int total = s_total;
    if (total <= 0) return;
    nsw = min(S, total - 1);
    if (total - 1 > S) q = nullptr;
  }
  const int slot = (int)(blockIdx.x % 8) * (int)(gridDim.x / 8) + (int)(blockIdx.x / 8);
  if (slot >= ntiles) return;
  const int tile = tiles ? tiles[slot] : slot;
  const int tx = tile % ntx, ty = tile / ntx;
  const int i0 = tx * TSX - S, j0 = ONE_D ? 0 : ty * TSY - S;
  const bool per = g.bc == HS_BC_PERIODIC;

  // Which cells a launch of nsw <= S sweeps touches: before sweep k the
  // values at distance >= k from the region edge are exact, and only the
  // tile (distance >= S) is kept, so sweep k updates the cells at distance
  // >= lo + 1 + k (lo = S - nsw) and cells nearer the edge than lo are never
  // read.  Cells outside the set carry no unknown: never updated (their value
  // stays 0, and no set cell reads them).
  const int lo = S - nsw;
  // Staging, with the loads of a kind issued together: (1) the region cells
  // (wrapped, or -1 outside the domain) and their distance to the region
  // edge; (2) their compact indices; (3) iterate, right-hand side and
  // coefficients of the cells that need them.
  int pidx[CPT];
  int cells[CPT];
  int dist[CPT];
  unsigned vmask[CPT];
  double rh[CPT][NC];
  double x0[CPT][NC];
  double cf[COEF_REG ? CPT : 1][COEF_REG ? 4 * NC * NC : 1];
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int r = threadIdx.x + c * NT;
    int cell = -1, dd = -1;
    if (r < R) {
      const int rx = r % RW, ry = r / RW;
      dd = min(rx, RW - 1 - rx);
      if (!ONE_D) dd = min(dd, min(ry, RH - 1 - ry));
      int gi = i0 + rx, gj = j0 + ry;
      if (per) {
        gi = wrap_index(gi, g.nx);
        gj = ONE_D ? 0 : wrap_index(gj, g.ny);
        cell = gi + g.nx * gj;
      } else if (gi >= 0 && gi < g.nx && gj >= 0 && gj < g.ny) {
        cell = gi + g.nx * gj;
      }
    }
    cells[c] = cell;
    dist[c] = dd;
  }
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    int p = -1;
    if (cells[c] >= 0 && dist[c] >= lo) p = pos ? pos[cells[c]] : cells[c];
    pidx[c] = p;
  }
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
#pragma unroll
    for (int a = 0; a < NC; ++a) x0[c][a] = 0.0;
    if (pidx[c] >= 0) {
#pragma unroll
      for (int a = 0; a < NC; ++a) x0[c][a] = xin[a * cap + pidx[c]];
    }
  }
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int p = pidx[c];
    unsigned v = 0u;
#pragma unroll
    for (int a = 0; a < NC; ++a) rh[c][a] = 0.0;
    if (p >= 0 && dist[c] > lo) {
#pragma unroll
      for (int d = 0; d < NDIR; ++d) {
        bool ok;
        if (pos) {
          ok = nbr[d * cap + p] >= 0;
        } else {
          int ci, cj;
          cell_ij(g, cells[c], ci, cj);
          const int nb = neighbour(g, ci, cj, d);
          ok = nb >= 0 && nb != cells[c];
        }
        v |= ok ? (1u << d) : 0u;
      }
#pragma unroll
      for (int a = 0; a < NC; ++a) rh[c][a] = rhs[a * cap + p];
      if constexpr (COEF_REG) {
#pragma unroll
        for (int e = 0; e < 4 * NC * NC; ++e) cf[c][e] = coef[(size_t)e * cap + p];
      }
    }
    vmask[c] = v;
  }
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int r = threadIdx.x + c * NT;
    if (r >= R) continue;
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      xs[0][a][r] = x0[c][a];
      xs[1][a][r] = x0[c][a];
    }
  }
  __syncthreads();

  // Neighbour directions that a cell reads: in-set neighbours inside the
  // staged region (at the region edge a cell's value is no longer needed).
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int r = threadIdx.x + c * NT;
    const int rx = r % RW, ry = r / RW;
    unsigned v = vmask[c];
    if (rx == 0) v &= ~1u;
    if (rx == RW - 1) v &= ~2u;
    if (!ONE_D) {
      if (ry == 0) v &= ~4u;
      if (ry == RH - 1) v &= ~8u;
    }
    vmask[c] = v;
  }

  // The sweeps, branch-free per updated cell so that all LDS reads of a
  // sweep are in flight together: every direction reads an in-region value
  // (the cell's own where the direction is off) and the update is kept by a
  // select, so the accumulation is the compact-list sweep's, operation for
  // operation.
  int cur = 0;
  for (int k = 0; k < nsw; ++k) {
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int r = threadIdx.x + c * NT;
      if (pidx[c] < 0 || dist[c] < lo + 1 + k) continue;
      const int pp = pidx[c];
      double acc[NC];
#pragma unroll
      for (int a = 0; a < NC; ++a) acc[a] = rh[c][a];
#pragma unroll
      for (int d = 0; d < NDIR; ++d) {
        const bool on = (vmask[c] >> d) & 1u;
        const int off = d == 0 ? -1 : (d == 1 ? 1 : (d == 2 ? -RW : RW));
        const int nr = on ? r + off : r;
        double t[NC];
#pragma unroll
        for (int a = 0; a < NC; ++a) {
          t[a] = acc[a];
#pragma unroll
          for (int b = 0; b < NC; ++b) {
            const int e = (d * NC + a) * NC + b;
            double m;
            if constexpr (COEF_REG) m = cf[c][e];
            else m = coef[(size_t)e * cap + pp];
            t[a] -= m * xs[cur][b][nr];
          }
        }
#pragma unroll
        for (int a = 0; a < NC; ++a) acc[a] = on ? t[a] : acc[a];
      }
#pragma unroll
      for (int a = 0; a < NC; ++a) xs[cur ^ 1][a][r] = acc[a];
    }
    __syncthreads();
    cur ^= 1;
  }

  double diff = 0.0, dn = 0.0;
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int r = threadIdx.x + c * NT;
    if (r >= R || pidx[c] < 0) continue;
    const int rx = r % RW, ry = r / RW;
    const int li = rx - S, lj = ONE_D ? 0 : ry - S;
    if (li < 0 || li >= TSX || lj < 0 || lj >= TSY) continue;
    if (tx * TSX + li >= g.nx || ty * TSY + lj >= g.ny) continue;   // ragged last tile
    const int p = pidx[c];
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      const double x = xs[cur][a][r];
      if (q) q[a * g.ncell + cells[c]] += x;
      else xout[a * cap + p] = x;
      if (record) {
        diff = nan_max(diff, fabs(x - xs[cur ^ 1][a][r]));
        dn = nan_max(dn, fabs(x));
      }
    }
  }
  if (record) {
    diff = block_max(diff, lds);
    dn = block_max(dn, lds);
    if (threadIdx.x == 0) {
      part[kStatDiff * kPartCap + slot] = diff;
      part[kStatDnorm * kPartCap + slot] = dn;
    }
  }
}

// Compact-list sweep (the same iteration, one sweep per launch); used for
// scattered sampled sets, when the tiled form is switched off, or when the
// grid holds more tiles than the statistics capacity.
template <int NC, bool FINAL, bool RECORD>
__global__ void list_sweep_kernel(Grid g, const int* __restrict__ hat, const int* __restrict__ nbr, int count,
                                  int cap, const double* __restrict__ coef, const double* __restrict__ rhs,
                                  const double* __restrict__ dold, double* __restrict__ dnew,
                                  double* __restrict__ q, double* __restrict__ part) {
  __shared__ double lds[kBlock / kWave];
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  double diff = 0.0, dn = 0.0;
  if (p < count) {
    const int ndir = g.kind == HS_BURGERS_1D ? 2 : 4;
    double acc[NC];
#pragma unroll
    for (int a = 0; a < NC; ++a) acc[a] = rhs[a * cap + p];
    int i = 0, j = 0, cell = p;
    if (hat) cell = hat[p];
    else cell_ij(g, p, i, j);
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      if (d >= ndir) break;
      int nb;
      if (hat) {
        nb = nbr[d * cap + p];
        if (nb < 0) continue;
      } else {
        nb = neighbour(g, i, j, d);
        if (nb < 0 || nb == cell) continue;
      }
#pragma unroll
      for (int a = 0; a < NC; ++a)
#pragma unroll
        for (int b = 0; b < NC; ++b)
          acc[a] -= coef[((d * NC + a) * NC + b) * (size_t)cap + p] * dold[b * cap + nb];
    }
    if (FINAL) {
#pragma unroll
      for (int a = 0; a < NC; ++a) q[a * g.ncell + cell] += acc[a];
    } else {
#pragma unroll
      for (int a = 0; a < NC; ++a) {
        dnew[a * cap + p] = acc[a];
        if (RECORD) {
          diff = nan_max(diff, fabs(acc[a] - dold[a * cap + p]));
          dn = nan_max(dn, fabs(acc[a]));
        }
      }
    }
  }
  if (RECORD) {
    diff = block_max(diff, lds);
    dn = block_max(dn, lds);
    if (threadIdx.x == 0) {
      stat_part(part, kStatDiff, diff);
      stat_part(part, kStatDnorm, dn);
    }
  }
}

template <int NC>
__global__ void add_list_kernel(Grid g, const int* __restrict__ hat, int count, int cap,
                                const double* __restrict__ d, double* __restrict__ q) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= count) return;
  const int cell = hat ? hat[p] : p;
#pragma unroll
  for (int a = 0; a < NC; ++a) q[a * g.ncell + cell] += d[a * cap + p];
}

// ------------------------------------------------------------------- host
template <int NC, int TSX, int TSY, int S, bool CR, int NT = kBlock>
static hs_status launch_tiles(hs_ctx* ctx, const hs_samples* s, int ntiles, const double* coef,
                              const double* rhs, const double* xin, double* xout, double* q, int k, bool record,
                              const NewtonCtrl& ctl = NewtonCtrl{}) {
  HS_LAUNCH(ctx, (tile_sweep_kernel<NC, TSX, TSY, S, CR, NT>), (ntiles + 7) / 8 * 8, NT, ctx->g,
            s ? s->tiles : nullptr, ntiles, s ? ctx->sntx : ctx->ntx, s ? s->pos : nullptr, s ? s->nbr : nullptr,
            ctx->ncell, coef, rhs, xin, xout, q, k, record ? 1 : 0, ctx->part, ctl);
  return HS_OK;
}

// Tiles pay unless the set is scattered: every region cell of an active tile
// is staged and swept, so a set that activates many tiles while filling few
// of their cells is relaxed over its compact list instead.  A tiled launch
// costs about one list sweep while doing up to S = 8 sweeps, and its work
// grows with the staged cells (4x the tile cells for 16 x 16, S = 8): tiles
// are used down to a quarter of the active tiles' cells sampled.
// Euler's 4 x 4 blocks stay on the compact list unless tiles are forced: a
// tile cannot hold their 64 coefficients per cell in registers, re-reads them
// every sweep and runs one wave per SIMD (512^2: full step 8.2 ms tiled,
// 1.4 ms over the list).
bool use_tiles(const hs_ctx* ctx, const hs_samples* s) {
  const int ntiles = s ? s->ntiles : ctx->ntx * ctx->nty;
  if (ctx->tiled == 0 || ntiles <= 0 || ntiles > kPartCap) return false;
  if (ctx->tiled == 2) return true;
  if (ctx->nc != 1) return false;
  if (!s) return true;
  return 4.0 * s->n_s >= (double)ntiles * ctx->stile_x * ctx->stile_y;
}

bool newton_ctrl_ok(const hs_ctx* ctx, const hs_samples* s) { return ctx->nc == 1 && use_tiles(ctx, s); }

// A sweep launch reads the relaxation blocks, b and the iterate once and
// writes the new iterate.
double sweep_launch_bytes(const hs_ctx* ctx, const hs_samples* s) {
  const int count = s ? s->n_s : ctx->ncell;
  return (double)count * (8.0 * (4 * ctx->nc * ctx->nc + ctx->nc) + 16.0 * ctx->nc);
}

hs_status relax_first_ctrl(hs_ctx* ctx, const hs_samples* s, double* q, const NewtonCtrl& c) {
  if (!newton_ctrl_ok(ctx, s)) return ctx->fail(HS_ERR_INVALID_ARG, "device Newton decision needs scalar tiles");
  const int ntiles = s ? s->ntiles : ctx->ntx * ctx->nty;
  const double* in = ctx->rhs;
  double* out = ctx->d0;
  const double* coef = ctx->coef;
  const double* rhs = ctx->rhs;
  if (ctx->g.kind == HS_BURGERS_1D && s)
    return launch_tiles<1, 256, 1, 8, true>(ctx, s, ntiles, coef, rhs, in, out, q, 0, false, c);
  if (ctx->g.kind == HS_BURGERS_1D)
    return launch_tiles<1, 1024, 1, 8, true>(ctx, s, ntiles, coef, rhs, in, out, q, 0, false, c);
  if (s)
    return launch_tiles<1, 16, 16, 8, true, kSweepThreadsSet>(ctx, s, ntiles, coef, rhs, in, out, q, 0, false, c);
  return launch_tiles<1, 32, 32, 8, true, kSweepThreadsMesh>(ctx, s, ntiles, coef, rhs, in, out, q, 0, false, c);
}

int tile_sweeps(const hs_ctx* ctx, const hs_samples* s) {
  if (!use_tiles(ctx, s)) return 1;
  return s ? ctx->stile_s : ctx->tile_s;
}

hs_status relax_sweeps(hs_ctx* ctx, const hs_samples* s, const double* coef, const double* rhs,
                       const double* xin, int nsweeps, double* q, bool record, const double** xlast) {
  const int count = s ? s->n_s : ctx->ncell;
  const int cap = ctx->ncell;
  const Grid& g = ctx->g;
  const int NC = ctx->nc;
  if (nsweeps <= 0) {
    if (q) {
      if (NC == 1) HS_LAUNCH(ctx, add_list_kernel<1>, blocks_for(count), kBlock, g, s ? s->hat : nullptr, count, cap, xin, q);
      else HS_LAUNCH(ctx, add_list_kernel<4>, blocks_for(count), kBlock, g, s ? s->hat : nullptr, count, cap, xin, q);
    }
    if (xlast) *xlast = xin;
    return HS_OK;
  }
  const int ntiles = s ? s->ntiles : ctx->ntx * ctx->nty;
  const bool tiled = use_tiles(ctx, s);
  const double* in = xin;
  int left = nsweeps;
  while (left > 0) {
    const int k = tiled ? std::min(left, s ? ctx->stile_s : ctx->tile_s) : 1;
    const bool last = k == left;
    double* out = in == ctx->d0 ? ctx->d1 : ctx->d0;
    double* qq = last ? q : nullptr;
    const bool rec = last && record;
    HS_TRY(prof_begin(ctx, HS_PROF_SWEEP));
    if (tiled) {
      if (g.kind == HS_BURGERS_1D && s)
        HS_TRY((launch_tiles<1, 256, 1, 8, true>(ctx, s, ntiles, coef, rhs, in, out, qq, k, rec)));
      else if (g.kind == HS_BURGERS_1D)
        HS_TRY((launch_tiles<1, 1024, 1, 8, true>(ctx, s, ntiles, coef, rhs, in, out, qq, k, rec)));
      else if (NC == 1 && s)
        HS_TRY((launch_tiles<1, 16, 16, 8, true, kSweepThreadsSet>(ctx, s, ntiles, coef, rhs, in, out, qq, k, rec)));
      else if (NC == 1)
        HS_TRY((launch_tiles<1, 32, 32, 8, true, kSweepThreadsMesh>(ctx, s, ntiles, coef, rhs, in, out, qq, k, rec)));
      else
        HS_TRY((launch_tiles<4, 16, 16, 4, false>(ctx, s, ntiles, coef, rhs, in, out, qq, k, rec)));
    } else {
      const int nb = blocks_for(count);
      if (rec && nb > kPartCap) return ctx->fail(HS_ERR_SHAPE, "relaxation grid beyond the statistics capacity");
      const int* hat = s ? s->hat : nullptr;
      const int* nbr = s ? s->nbr : nullptr;
#define HS_SWEEP(NCV)                                                                                         \
  do {                                                                                                        \
    if (qq)                                                                                                   \
      HS_LAUNCH(ctx, (list_sweep_kernel<NCV, true, false>), nb, kBlock, g, hat, nbr, count, cap, coef, rhs, in, \
                out, qq, ctx->part);                                                                          \
    else if (rec)                                                                                             \
      HS_LAUNCH(ctx, (list_sweep_kernel<NCV, false, true>), nb, kBlock, g, hat, nbr, count, cap, coef, rhs, in, \
                out, qq, ctx->part);                                                                          \
    else                                                                                                      \
      HS_LAUNCH(ctx, (list_sweep_kernel<NCV, false, false>), nb, kBlock, g, hat, nbr, count, cap, coef, rhs,   \
                in, out, qq, ctx->part);                                                                      \
  } while (0)
      if (NC == 1) HS_SWEEP(1);
      else HS_SWEEP(4);
#undef HS_SWEEP
    }
    HS_TRY(prof_end(ctx, HS_PROF_SWEEP, sweep_launch_bytes(ctx, s)));
    left -= k;
    in = out;
  }
  if (xlast) *xlast = q ? nullptr : in;
  return HS_OK;
}

// Tile geometry (must match the instantiations above): the full mesh uses
// large tiles; sampled sets, which cluster along fronts and fill only part
// of a tile, use smaller ones so that a launch has enough workgroups.
void tile_geometry(const hs_problem* pr, int nc, bool sampled, int* tx, int* ty, int* s) {
  if (pr->kind == HS_BURGERS_1D) { *tx = sampled ? 256 : 1024; *ty = 1; *s = 8; }
  else if (nc == 1) { *tx = sampled ? 16 : 32; *ty = sampled ? 16 : 32; *s = 8; }
  else { *tx = 16; *ty = 16; *s = 4; }
}

void set_tile_geometry(hs_ctx* ctx, const hs_problem* pr) {
  tile_geometry(pr, ctx->nc, false, &ctx->tile_x, &ctx->tile_y, &ctx->tile_s);
  ctx->ntx = (ctx->g.nx + ctx->tile_x - 1) / ctx->tile_x;
  ctx->nty = (ctx->g.ny + ctx->tile_y - 1) / ctx->tile_y;
  tile_geometry(pr, ctx->nc, true, &ctx->stile_x, &ctx->stile_y, &ctx->stile_s);
  ctx->sntx = (ctx->g.nx + ctx->stile_x - 1) / ctx->stile_x;
  ctx->snty = (ctx->g.ny + ctx->stile_y - 1) / ctx->stile_y;
}

}  // namespace hs
