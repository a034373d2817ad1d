// Internal definitions shared by the HIP translation units of libhsrom.
// Not part of the public interface (see include/hsrom.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "hsrom.h"

namespace hs {

constexpr int kBlock = 256;          // threads per block for streaming kernels
constexpr int kWave = 64;            // CDNA wavefront width
constexpr int kMaxBasis = 64;        // m_max, w_max limit (one workgroup small solves)
constexpr int kRedBlocks = 1024;     // upper bound on blocks of a reduction pass

// Problem geometry and constants passed by value to every kernel.
struct Grid {
  int nx, ny, ncell, nc, kind, bc;
  double lx, ly, gamma, inflow;
  unsigned long long nx_mul;   // ceil(2^nx_shift / nx), for cell / nx by a multiply
  int nx_shift;                // 32 + ceil(log2 nx)
};

// Small statistics slots (uint64 bit patterns of non-negative doubles, so an
// integer atomicMax is an exact, order-independent maximum).
enum StatSlot : int {
  kStatResMax = 0,     // max |R|
  kStatRho = 1,        // Jacobi contraction bound
  kStatQMax = 2,       // max |q_prev|
  kStatNonFinite = 3,  // != 0 if a non-finite residual was met
  kStatCount = 4,      // generic integer counter
  kStatDiff = 5,       // max |delta_new - delta_old| of a recorded sweep
  kStatDnorm = 6,      // max |delta_new| of a recorded sweep
  kStatFitRank = 8,    // rank of the fit's pseudo-inverse
  kStatFitCond = 9,    // its condition number
  kStatDy = 10,        // ||y_j - y_{j-1}|| of the last subiteration
  kStatSum0 = 11,      // l1 sum of the cell residual norms before a filter order
  kStatSum = 12,       // the same after a filter pass
  kStatSweeps = 13,    // sweeps of the Newton correction decided on the device (integer; -1: batch form)
  kStatFiltCount1 = 14,  // kept count and residual sum of a device-driven filter pass with an odd
  kStatFiltSum1 = 15,    // index (partials only: even passes use kStatCount / kStatSum)
  kStatSlots = 16
};

constexpr int kPartCap = 4096;   // max blocks of a kernel that reports statistics

}  // namespace hs

// ------------------------------------------------------------------ context
struct hs_ctx {
  hs_problem p{};
  hs::Grid g{};
  int nc = 1, ncell = 0, n = 0, nnb = 4;   // nnb: stencil neighbours per cell
  hipStream_t stream = nullptr;
  hipStream_t aux = nullptr;        // library-owned stream of basis_update_async (default priority)
  hipEvent_t aux_ready = nullptr;   // recorded on stream, waited on by aux
  bool aux_pending = false;         // an asynchronous basis update is in flight
  int basis_meff = 0;               // m_eff of the last completed basis update
  struct { long long n; int nsnap; double phi_bytes; int prof_idx; } pending_form{0, 0, 8.0, -1};
  int device = 0;
  int max_lds = 65536;               // LDS bytes a workgroup may use on this device
  int num_cu = 256;                  // compute units of the device
  std::string err;

  // device workspaces (allocated once at create)
  double* u = nullptr;        // N  working state (hybrid step)
  double* R = nullptr;        // N  residual / scratch
  double* rhs = nullptr;      // N  Jacobi right-hand side b = -D^{-1} R
  double* d0 = nullptr;       // N  Jacobi iterate
  double* d1 = nullptr;       // N  Jacobi iterate
  double* coef = nullptr;     // nnb * nc * nc * ncell : M_X = D^{-1} O_X
  double* rho = nullptr;      // N  reconstruction psi + Phi y
  double* gf = nullptr;       // N  filtered state
  double* gtmp = nullptr;     // N  filter scratch / merged state
  double* rcell = nullptr;    // ncell cell residual norms
  double* rcell2 = nullptr;   // ncell cell residual norms
  double* adj = nullptr;      // N  adjoint work vector
  // tiled relaxation: tile_x x tile_y cells per tile, up to tile_s sweeps per
  // launch; ntx x nty tiles cover the grid; tiled: 0 = one sweep per launch
  // over the compact cell list, 1 = tiles where dense enough, 2 = tiles always
  int tile_x = 0, tile_y = 0, tile_s = 0, ntx = 0, nty = 0;
  // the same for sampled sets (smaller tiles: a set fills a few of them)
  int stile_x = 0, stile_y = 0, stile_s = 0, sntx = 0, snty = 0;
  int tiled = 1;
  // fit pseudo-inverse for m <= 8: 1 = one wave in registers, 0 = LDS routine
  int small_pinv = 1;
  int fit_chol = 1;           // HS_OPT_FIT_CHOLESKY
  double* red = nullptr;      // reduction partials (kRedBlocks * 64 * 64 doubles)
  double* small = nullptr;    // small dense matrices and vectors (16 * 64 * 64 doubles)
  unsigned long long* stats = nullptr;   // kStatSlots
  double* part = nullptr;     // per-block partial statistics: kStatSlots x kPartCap
  int* ibuf = nullptr;        // integer scratch (ncell + 1024)
  void* hpin = nullptr;       // host read-back buffer (64 KiB + tag word): pinned, coherent, mapped
  void* dpin = nullptr;       // its device address
  unsigned pin_tag = 0;       // last tag published into it
  unsigned post_next = 0;     // next slot of the read-back ring

  // kernel timing (hs_prof_enable)
  int prof_class = 0;
  std::vector<hipEvent_t> prof_ev;   // start/stop pairs
  std::vector<double> prof_bytes;
  size_t prof_used = 0;

  hs_status fail(hs_status s, const std::string& msg) {
    err = msg;
    return s;
  }
};

struct hs_samples {
  hs_ctx* ctx = nullptr;
  int ncell = 0;
  int n_g = 0, n_s = 0, l = 0;
  uint8_t* gmask = nullptr;   // ncell, G
  uint8_t* mask = nullptr;    // ncell, hat-S
  uint8_t* tmask = nullptr;   // ncell, tilde-S
  uint8_t* dtmp = nullptr;    // ncell, dilation scratch
  int32_t* hat = nullptr;     // ncell capacity, sorted hat-S cells
  int32_t* tilde = nullptr;   // ncell capacity, sorted tilde-S cells
  int32_t* pos = nullptr;     // ncell, compact index of a hat-S cell or -1
  int32_t* nbr = nullptr;     // 4 * ncell, compact index of each stencil neighbour in hat-S or -1
  int32_t* scan = nullptr;    // scan scratch
  int32_t* scan3 = nullptr;   // block sums of the three set compactions, then their totals
  uint8_t* tflag = nullptr;   // per tile of the context's tiling: holds a hat-S cell
  int32_t* tiles = nullptr;   // active tile ids (ntiles)
  int ntiles = 0;
};

// A hybrid step's frozen decisions (and, after a replay, its internal states).
constexpr int kMaxPasses = 64;
struct hs_htape {
  hs_ctx* ctx = nullptr;
  hs_samples* s = nullptr;    // copy of the sampled set
  int J = 0;                  // subiterations
  int npass = 0;              // applied filter passes
  int passes[kMaxPasses] = {0};   // filter order n of each applied pass
  uint8_t* masks = nullptr;   // kMaxPasses x ncell kept-cell masks
  double* us = nullptr;       // J x N states after each subiteration's Newton solve (replay)
  size_t us_cap = 0;          // capacity of us in doubles
  double* gp = nullptr;       // fit pseudo-inverse (m x m, replay)
  int m = 0;
  int precision = HS_FP64;    // basis precision of the replay
  bool recorded = false, replayed = false;
};

// Layout of ctx->small (offsets in doubles).
constexpr int kSmG = 0;                 // Gram (m x m)
constexpr int kSmGp = 4096;             // pseudo-inverse (m x m)
constexpr int kSmY0 = 12288;            // y0
constexpr int kSmY = 12288 + 64;        // y
constexpr int kSmYPrev = 12288 + 128;   // previous y
constexpr int kSmMisc = 12288 + 192;    // [0] = ||dy||, [1] = rank, [2] = cond, [8] = residual sum
constexpr int kSmAdjY = 12288 + 256;    // adjoint: y-bar of the current subiteration
constexpr int kSmAdjZ = 12288 + 320;    // adjoint: G+ y-bar
constexpr int kSmAdjY0 = 12288 + 384;   // adjoint: y-bar from the reconstruction
constexpr int kSmFilt = 12288 + 448;    // device state of the filter loop (FiltCtl)
// basis_update's matrices (its own region: the update may run on the second
// stream while the main stream uses the fit's entries above)
constexpr int kSmBasG = 8 * 4096;       // window Gram X^T X (w x w)
constexpr int kSmBasG2 = 9 * 4096;      // Gram of the preconditioned window (w x w)
constexpr int kSmBasT1 = 10 * 4096;     // preconditioner inverse (wp x wp)
constexpr int kSmBasC1 = 11 * 4096;     // preconditioner (w x w, stride 64)
constexpr int kSmBasT = 12 * 4096;      // formation matrix (w x mp)
constexpr int kSmBasMeff = 13 * 4096;   // m_eff (int)

// ----------------------------------------------------------------- helpers
#define HS_TRY(expr)                     \
  do {                                   \
    hs_status _s = (expr);               \
    if (_s != HS_OK) return _s;          \
  } while (0)

#define HIP_TRY(ctx, expr)                                                            \
  do {                                                                                \
    hipError_t _e = (expr);                                                           \
    if (_e != hipSuccess)                                                             \
      return (ctx)->fail(HS_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

#define HS_LAUNCH(ctx, kernel, grid, block, ...)                                        \
  do {                                                                                  \
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, (ctx)->stream, __VA_ARGS__); \
    hipError_t _e = hipGetLastError();                                                  \
    if (_e != hipSuccess)                                                               \
      return (ctx)->fail(HS_ERR_HIP, std::string("launch " #kernel ": ") + hipGetErrorString(_e)); \
  } while (0)

namespace hs {

inline int blocks_for(long long n, int per_block = kBlock, int cap = 1 << 30) {
  long long b = (n + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return static_cast<int>(b);
}

inline double bits_to_double(unsigned long long b) {
  double d;
  static_assert(sizeof(d) == sizeof(b), "");
  __builtin_memcpy(&d, &b, sizeof d);
  return d;
}

// ------------------------------------------------------- device utilities
__device__ inline unsigned long long dbits(double d) { return __double_as_longlong(d); }

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// max(a, b), NaN if either is NaN (fmax returns the other operand, so a
// maximum taken with it would hide a NaN from the finiteness checks).
__device__ inline double nan_max(double a, double b) { return a != a ? a : (b != b ? b : fmax(a, b)); }

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = nan_max(v, __shfl_xor(v, o, kWave));
  return v;
}

__device__ inline int wave_sum_int(int v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Block-wide sum with a fixed tree (deterministic for a fixed block size).
// The result is valid in thread 0.  lds needs blockDim.x / 64 doubles.
__device__ inline double block_sum(double v, double* lds) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  const int nw = blockDim.x / kWave;
  if (l == 0) lds[w] = v;
  __syncthreads();
  double r = 0.0;
  if (w == 0) {
    r = (l < nw) ? lds[l] : 0.0;
    r = wave_sum(r);
  }
  __syncthreads();
  return r;
}

__device__ inline double block_max(double v, double* lds) {
  v = wave_max(v);
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  const int nw = blockDim.x / kWave;
  if (l == 0) lds[w] = v;
  __syncthreads();
  double r = 0.0;
  if (w == 0) {
    r = (l < nw) ? lds[l] : 0.0;
    r = wave_max(r);
  }
  __syncthreads();
  return r;
}

__device__ inline int block_sum_int(int v, int* lds) {
  v = wave_sum_int(v);
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  const int nw = blockDim.x / kWave;
  if (l == 0) lds[w] = v;
  __syncthreads();
  int r = 0;
  if (w == 0) {
    r = (l < nw) ? lds[l] : 0;
    r = wave_sum_int(r);
  }
  __syncthreads();
  return r;
}

// Record max(|x|) of non-negative x into a stats slot.
__device__ inline void stat_max(unsigned long long* slot, double x) {
  atomicMax(slot, dbits(x));
}

// Per-block partial of a statistic: part[slot * kPartCap + block].  A finish
// kernel reduces the partials (no same-address atomics across blocks).
// Row j = cell / nx and column i = cell % nx by a multiply and a shift (a
// runtime division costs about 20 VALU instructions): with l = ceil(log2 nx)
// and m = ceil(2^(32+l) / nx), floor(cell m / 2^(32+l)) is the exact
// quotient for every 0 <= cell < 2^31.
__device__ inline void cell_ij(const Grid& g, int cell, int& i, int& j) {
  j = (int)(((unsigned long long)(unsigned)cell * g.nx_mul) >> g.nx_shift);
  i = cell - j * g.nx;
}

// u wrapped into [0, len) on a periodic axis.  Every halo and stencil offset
// here lies within one period of the range, where one conditional add or
// subtract does it (a runtime remainder costs about 20 VALU instructions);
// the remainder serves anything farther.
__device__ inline int wrap_index(int u, int len) {
  if (u >= -len && u < 2 * len) return u < 0 ? u + len : (u >= len ? u - len : u);
  return ((u % len) + len) % len;
}

__device__ inline void stat_part(double* part, int slot, double v) {
  part[slot * kPartCap + blockIdx.x] = v;
}

// Read-back to the host buffer (pinned, coherent, mapped): one wave stores the
// words, fences at system scope (its stores are complete once the fence has
// waited for them) and then stores the tag the host spins on.
__device__ inline void post_words(const uint32_t* src, int words, uint32_t* dst, uint32_t* tagp, unsigned tag) {
  for (int i = threadIdx.x; i < words; i += kWave) dst[i] = src[i];
  __threadfence_system();
  if (threadIdx.x == 0) *(volatile uint32_t*)tagp = tag;
}

// ---------------------------------------------------------- grid helpers
// Neighbour of cell (i, j) across a face.  dir: 0 = W, 1 = E, 2 = S, 3 = N.
// Returns the neighbour cell, the cell itself for a zeroth-order-extrapolation
// ghost, or -1 for the constant inflow ghost (1D left boundary).
__device__ inline int neighbour(const Grid& g, int i, int j, int dir) {
  const bool per = g.bc == HS_BC_PERIODIC;
  if (dir < 2) {
    int ii = dir == 0 ? i - 1 : i + 1;
    if (ii < 0) {
      if (per) ii = g.nx - 1;
      else if (g.bc == HS_BC_INFLOW_OUTFLOW) return -1;
      else ii = 0;
    } else if (ii >= g.nx) {
      ii = per ? 0 : g.nx - 1;
    }
    return ii + g.nx * j;
  }
  int jj = dir == 2 ? j - 1 : j + 1;
  if (jj < 0) jj = per ? g.ny - 1 : 0;
  else if (jj >= g.ny) jj = per ? 0 : g.ny - 1;
  return i + g.nx * jj;
}

// Whether the neighbour across face dir is a distinct real cell (its state is
// an independent unknown) rather than a ghost that copies the cell itself.
__device__ inline bool neighbour_is_other(const Grid& g, int cell, int nb) {
  return nb >= 0 && nb != cell;
}

}  // namespace hs

// ------------------------------------------ cross-translation-unit internals
namespace hs {
hs_status readback(hs_ctx* ctx, const void* dsrc, size_t bytes, void* hdst);
hs_status zero_stats(hs_ctx* ctx);
hs_status read_stats(hs_ctx* ctx, unsigned long long* out /* kStatSlots */);
// Reduce the per-block partials of the slots in max_mask (max) and sum_mask
// (sum) over nb blocks into the stats slots (bit patterns of the doubles).
// With out, the same launch also delivers all stats slots to the host
// (read_stats in one step).
hs_status finish_stats(hs_ctx* ctx, int nb, unsigned max_mask, unsigned sum_mask,
                       unsigned long long* out = nullptr);
inline int stat_blocks(long long n) { return blocks_for(n, kBlock, kPartCap); }
hs_status max_abs(hs_ctx* ctx, const double* x, long long n, double* out);
// Newton on the full mesh (s == nullptr) or on a sampled set.  primed: the
// first iteration's residual/Jacobian was already launched on q by
// newton_first_launch or newton_first_ctrl, and {max |R|, rho, the device's
// sweep count (0: none ran)} were read back (else nullptr).
hs_status newton_solve(hs_ctx* ctx, double* q, const double* q_prev, double tol,
                       const hs_samples* s, hs_step_info* info, const double* primed = nullptr);
// Residual, Jacobian relaxation data and the ResMax/Rho statistics at q;
// with st all stats slots are read back as well (else enqueued only).
// The same with the decision on the device (newton_ctrl_ok): the first sweep
// launch also applies the subiteration stop test when sub_check is set (the
// host applies it to the same ||dy|| from the posted stats); *total as in the
// primed array.
hs_status newton_first_ctrl(hs_ctx* ctx, double* q, const double* q_prev, double tol, const hs_samples* s,
                            int sub_check, double eps_y, unsigned long long* st, int* total,
                            bool tol_from_qmax = false);
hs_status newton_first_launch(hs_ctx* ctx, const double* q, const double* q_prev, const hs_samples* s,
                              unsigned long long* st);
// max |x| into the QMax statistics slot (enqueued only).
hs_status max_abs_launch(hs_ctx* ctx, const double* x, long long n);
hs_status cell_residual_norm(hs_ctx* ctx, const double* q, const double* q_prev, double* rcell,
                             double* sum_out);
// The same, enqueued only: the sum goes to the statistics slot `slot`.
hs_status cell_residual_launch(hs_ctx* ctx, const double* q, const double* q_prev, double* rcell, int slot);
hs_status run_filter(hs_ctx* ctx, double* gamma, const double* q_prev, const hs_hybrid_params* hp,
                     hs_step_info* info, hs_htape* record = nullptr);
// Solve the linear system whose relaxation data (coef, rhs layout [.. * ncell + p])
// is given, to relative accuracy eta; result in x (same layout).  rho is the
// max-norm contraction bound of the relaxation (>= 1: monitored batches).
hs_status relax_solve(hs_ctx* ctx, const hs_samples* s, const double* coef, const double* rhs, double rho,
                      double eta, double* x, int* sweeps);
// Relaxation sweeps k0+1 .. k0+nsweeps on the full mesh (s == nullptr) or the
// sampled set s, starting from the iterate xin (compact layout).  With q the
// final iterate is added to the state q (Newton update); otherwise *xlast
// points to it (one of ctx->d0 / ctx->d1, or xin if nsweeps == 0).  With
// record, the last sweep reports max |x_k - x_{k-1}| and max |x_k|.
hs_status relax_sweeps(hs_ctx* ctx, const hs_samples* s, const double* coef, const double* rhs,
                       const double* xin, int nsweeps, double* q, bool record, const double** xlast);
// The Newton decision taken by the first tiled sweep launch of an iteration
// (scalar problems): it reduces the residual/Jacobian partials (ResMax, Rho),
// tests convergence, chooses the sweep count of the correction exactly as the
// host would (inexact Newton, rho^nsw <= eta), runs the first sweeps of it and
// posts the stats (with kStatSweeps) to the host; the host then enqueues the
// remaining sweeps.  total <= 0 (converged, non-finite, or the batch form):
// the launch changes nothing but the stats.
struct NewtonCtrl {
  const double* part = nullptr;   // nullptr: an ordinary launch
  int nb = 0;                     // resjac blocks
  double tol = 0.0, scale = 1.0, lin_rtol = 0.0;
  int lin_maxit = 0;
  int sub_check = 0;       // also the subiteration stop test: no sweeps when ||y_j - y_{j-1}|| < eps_y
  double eps_y = 0.0;
  double rtol_qmax = 0.0;  // > 0: tol = rtol_qmax max(1, max |q_prev|) from the statistics (tol, scale unused)
  unsigned long long* stats = nullptr;
  uint32_t* dst = nullptr;
  uint32_t* tagp = nullptr;
  unsigned tag = 0;
};
// A slot of the host read-back ring: posts that may be in flight while the
// host reads an earlier one (the filter loop runs one pass ahead).
struct PostSlot {
  uint32_t* dst = nullptr;    // device address of the slot's data (kPostWords words)
  uint32_t* tagp = nullptr;   // device address of its tag word
  unsigned tag = 0;
  int slot = 0;
};
constexpr int kPostWords = 32;
PostSlot post_slot(hs_ctx* ctx);
// Waits for the slot's tag, then copies bytes (<= 4 kPostWords) of its data.
hs_status await_post(hs_ctx* ctx, const PostSlot& p, void* out, size_t bytes);
// Whether the Newton decision can run in the first sweep launch on s.
bool newton_ctrl_ok(const hs_ctx* ctx, const hs_samples* s);
// That launch: sweeps from x_1 = rhs into ctx->d0, or onto q when they are all.
hs_status relax_first_ctrl(hs_ctx* ctx, const hs_samples* s, double* q, const NewtonCtrl& c);
// Algorithmic bytes of one sweep launch on s (nullptr: the full mesh).
double sweep_launch_bytes(const hs_ctx* ctx, const hs_samples* s);
// Tile shape and sweeps per launch of the full mesh (sampled = false) or of
// sampled sets; set_tile_geometry fills both into the context.
void tile_geometry(const hs_problem* pr, int nc, bool sampled, int* tx, int* ty, int* s);
void set_tile_geometry(hs_ctx* ctx, const hs_problem* pr);
// Whether the relaxation on s (nullptr: full mesh) runs in tiles, and the
// sweeps per tiled launch.
bool use_tiles(const hs_ctx* ctx, const hs_samples* s);
// Completes the asynchronous basis update in flight (its m_eff to *m_eff).
hs_status basis_finish_pending(hs_ctx* ctx, int32_t* m_eff);
int tile_sweeps(const hs_ctx* ctx, const hs_samples* s);
// Bracket one launch of kernel class cls with events (no-op unless enabled).
hs_status prof_begin(hs_ctx* ctx, int cls);
hs_status prof_end(hs_ctx* ctx, int cls, double bytes);
}  // namespace hs
