// Sampling sets (A5): from the per-cell reconstruction error to G, the
// sampled set hat-S = dilate(G), its face-neighbour ring tilde-S and the
// compact lists used by the restricted kernels (Sec. 2.3.3 and the set
// operations of Alg. 1).
//
// G is the n_g largest errors with ties to the lower cell index.  The n_g-th
// largest value is found by an 8-pass, 8-bit radix select on the IEEE bit
// patterns of the errors (for non-negative doubles the unsigned integer order
// is the numeric order), so the result is exact and independent of any
// floating-point summation.  Integer histograms use LDS atomics (exact).
#include "physics.hpp"

#include <algorithm>
#include <cmath>

namespace hs {

constexpr int kScanItems = 4;                          // items per thread in a scan block
constexpr int kScanTile = kBlock * kScanItems;         // 1024 items per block

struct SelectState {
  unsigned long long prefix;   // digits of the threshold key fixed so far
  long long k;                 // rank still to place within the current bucket
};

__global__ void count_positive_kernel(const double* __restrict__ eps, int n, double* __restrict__ part) {
  __shared__ int lds[kBlock / kWave];
  int c = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) c += eps[i] > 0.0;
  c = block_sum_int(c, lds);
  if (threadIdx.x == 0) stat_part(part, kStatCount, (double)c);
}

__global__ void radix_hist_kernel(const double* __restrict__ eps, int n, const SelectState* st, int shift,
                                  unsigned int* __restrict__ hist) {
  __shared__ unsigned int h[256];
  for (int t = threadIdx.x; t < 256; t += blockDim.x) h[t] = 0;
  __syncthreads();
  const unsigned long long himask = shift >= 56 ? 0ull : (~0ull << (shift + 8));
  const unsigned long long pre = st->prefix & himask;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double e = eps[i];
    if (!(e > 0.0)) continue;
    const unsigned long long key = dbits(e);
    if ((key & himask) == pre) atomicAdd(&h[(key >> shift) & 255u], 1u);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < 256; t += blockDim.x)
    if (h[t]) atomicAdd(&hist[t], h[t]);
}

// One block of 256 threads: choose the digit that holds the k-th largest key.
__global__ void radix_pick_kernel(SelectState* st, int shift, unsigned int* __restrict__ hist) {
  __shared__ unsigned long long above[257];
  const int t = threadIdx.x;   // digit t
  if (t == 0) {
    // suffix sums from the largest digit down (256 terms, one thread: exact and cheap)
    unsigned long long s = 0;
    above[256] = 0;
    for (int d = 255; d >= 0; --d) {
      above[d] = s;            // count of keys with digit > d
      s += hist[d];
    }
  }
  __syncthreads();
  const long long k = st->k;
  const unsigned long long a = above[t], c = hist[t];
  __syncthreads();
  if (c > 0 && (long long)a < k && k <= (long long)(a + c)) {
    st->prefix |= (unsigned long long)t << shift;
    st->k = k - (long long)a;
  }
  __syncthreads();
  hist[t] = 0;
}

// gmask = key > K, emask = key == K (candidates for the remaining ties).
__global__ void mark_kernel(const double* __restrict__ eps, int n, const SelectState* st,
                            uint8_t* __restrict__ gmask, uint8_t* __restrict__ emask) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double e = eps[i];
  const unsigned long long K = st->prefix;
  const unsigned long long key = e > 0.0 ? dbits(e) : 0ull;
  gmask[i] = (e > 0.0) && key > K;
  emask[i] = (e > 0.0) && key == K;
}

// ------------------------------------------------------------- block scan
// Exclusive scan of per-block totals, then per-element ranks.
__global__ void flag_count_kernel(const uint8_t* __restrict__ f, int n, int* __restrict__ bsum) {
  __shared__ int lds[kBlock / kWave];
  const int base = blockIdx.x * kScanTile;
  int c = 0;
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    const int i = base + r * kBlock + threadIdx.x;
    if (i < n) c += f[i] != 0;
  }
  c = block_sum_int(c, lds);
  if (threadIdx.x == 0) bsum[blockIdx.x] = c;
}

// Single block: exclusive scan of nb block sums in place; total to bsum[nb].
__global__ void scan_bsums_kernel(int* __restrict__ bsum, int nb) {
  __shared__ int carry;
  __shared__ int wsum[kBlock / kWave];
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < nb; base += kBlock) {
    const int i = base + threadIdx.x;
    const int v = i < nb ? bsum[i] : 0;
    // inclusive wave scan
    int x = v;
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int y = __shfl_up(x, o, kWave);
      if (lane >= o) x += y;
    }
    if (lane == kWave - 1) wsum[w] = x;
    __syncthreads();
    int woff = 0;
    for (int k = 0; k < w; ++k) woff += wsum[k];
    const int incl = x + woff + carry;
    if (i < nb) bsum[i] = incl - v;
    __syncthreads();
    if (threadIdx.x == kBlock - 1) carry = incl;
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[nb] = carry;
}

// Rank of each set flag within its block (exclusive), plus the block offset.
__device__ inline int block_exclusive_rank(int flag, int* wsum) {
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  int x = flag;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  if (lane == kWave - 1) wsum[w] = x;
  __syncthreads();
  int woff = 0;
  for (int k = 0; k < w; ++k) woff += wsum[k];
  __syncthreads();
  return x - flag + woff;
}

// Compaction: list[offset] = i for every set flag, pos[i] = offset or -1.
__global__ void compact_kernel(const uint8_t* __restrict__ f, int n, const int* __restrict__ bsum,
                               int* __restrict__ list, int* __restrict__ pos) {
  __shared__ int wsum[kBlock / kWave];
  __shared__ int run;
  if (threadIdx.x == 0) run = 0;
  __syncthreads();
  const int base = blockIdx.x * kScanTile;
  const int off = bsum[blockIdx.x];
  for (int r = 0; r < kScanItems; ++r) {
    const int i = base + r * kBlock + threadIdx.x;
    const int flag = (i < n) && f[i];
    const int rank = block_exclusive_rank(flag, wsum);
    const int o = off + run + rank;
    if (i < n) {
      if (flag) list[o] = i;
      if (pos) pos[i] = flag ? o : -1;
    }
    __syncthreads();
    if (threadIdx.x == kBlock - 1) run += rank + flag;
    __syncthreads();
  }
}

// Ties: keep the first k equal keys (by cell index) in G.
__global__ void tie_keep_kernel(const uint8_t* __restrict__ emask, int n, const int* __restrict__ bsum,
                                const SelectState* st, uint8_t* __restrict__ gmask) {
  __shared__ int wsum[kBlock / kWave];
  __shared__ int run;
  if (threadIdx.x == 0) run = 0;
  __syncthreads();
  const long long k = st->k;
  const int base = blockIdx.x * kScanTile;
  const int off = bsum[blockIdx.x];
  for (int r = 0; r < kScanItems; ++r) {
    const int i = base + r * kBlock + threadIdx.x;
    const int flag = (i < n) && emask[i];
    const int rank = block_exclusive_rank(flag, wsum);
    if (flag && (long long)(off + run + rank) < k) gmask[i] = 1;
    __syncthreads();
    if (threadIdx.x == kBlock - 1) run += rank + flag;
    __syncthreads();
  }
}

// ------------------------------------------------------------- set growth
// Chebyshev dilation along one axis (0 = x, 1 = y) by radius h.
__global__ void dilate_kernel(Grid g, const uint8_t* __restrict__ in, uint8_t* __restrict__ out, int axis,
                              int h) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.ncell) return;
  const int i = c % g.nx, j = c / g.nx;
  const bool per = g.bc == HS_BC_PERIODIC;
  const int n = axis == 0 ? g.nx : g.ny;
  const int x0 = axis == 0 ? i : j;
  uint8_t v = 0;
  for (int d = -h; d <= h && !v; ++d) {
    int x = x0 + d;
    if (x < 0 || x >= n) {
      if (!per) continue;
      x = ((x % n) + n) % n;
    }
    v |= axis == 0 ? in[x + g.nx * j] : in[i + g.nx * x];
  }
  out[c] = v;
}

// tilde-S: face neighbours of hat-S that are not in hat-S.
__global__ void ring_kernel(Grid g, const uint8_t* __restrict__ mask, uint8_t* __restrict__ tmask) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.ncell) return;
  if (mask[c]) {
    tmask[c] = 0;
    return;
  }
  const int i = c % g.nx, j = c / g.nx;
  const bool per = g.bc == HS_BC_PERIODIC;
  const int ndir = g.kind == HS_BURGERS_1D ? 2 : 4;
  uint8_t v = 0;
  for (int d = 0; d < ndir; ++d) {
    int ii = i + (d == 0 ? -1 : d == 1 ? 1 : 0);
    int jj = j + (d == 2 ? -1 : d == 3 ? 1 : 0);
    if (ii < 0 || ii >= g.nx || jj < 0 || jj >= g.ny) {
      if (!per) continue;
      ii = (ii + g.nx) % g.nx;
      jj = (jj + g.ny) % g.ny;
    }
    v |= mask[ii + g.nx * jj];
  }
  tmask[c] = v;
}

// Neighbour table of the compact sampled list: compact index of each face
// neighbour that is itself sampled, else -1 (ghosts, tilde-S cells).
__global__ void nbr_table_kernel(Grid g, const int* __restrict__ hat, int ns, int cap,
                                 const int* __restrict__ pos, int* __restrict__ nbr) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ns) return;
  const int cell = hat[p];
  const int i = cell % g.nx, j = cell / g.nx;
  const int ndir = g.kind == HS_BURGERS_1D ? 2 : 4;
  for (int d = 0; d < 4; ++d) {
    int v = -1;
    if (d < ndir) {
      const int nb = neighbour(g, i, j, d);
      if (nb >= 0 && nb != cell) v = pos[nb];
    }
    nbr[d * cap + p] = v;
  }
}

__global__ void scatter_mask_kernel(const int* __restrict__ list, int n, int ncell, uint8_t* __restrict__ mask) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int c = list[p];
  if (c >= 0 && c < ncell) mask[c] = 1;   // out-of-range entries are dropped (count check fails)
}

// Flag the tile of every listed cell (all writers store the same value).
__global__ void tile_flag_kernel(Grid g, const int* __restrict__ hat, int ns, int tx, int ty, int ntx,
                                 uint8_t* __restrict__ tflag) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ns) return;
  const int cell = hat[p];
  const int i = cell % g.nx, j = cell / g.nx;
  tflag[(j / ty) * ntx + i / tx] = 1;
}

__global__ void fill_u8_kernel(uint8_t* p, int n, uint8_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void init_state_kernel(SelectState* st, long long k) {
  st->prefix = 0ull;
  st->k = k;
}

// ------------------------------------------------------------------- host
// The select state lives after the block sums in the scan buffer, 8-byte aligned.
static size_t state_offset(int n) { return ((size_t)n / kScanTile + 32) & ~(size_t)1; }

static hs_status scan_blocks(hs_ctx* ctx, const uint8_t* flags, int n, int* bsum) {
  const int nb = blocks_for(n, kScanTile);
  HS_LAUNCH(ctx, flag_count_kernel, nb, kBlock, flags, n, bsum);
  HS_LAUNCH(ctx, scan_bsums_kernel, 1, kBlock, bsum, nb);
  return HS_OK;
}

// Compact n flags into list (and pos); returns the count on the host.
static hs_status compact(hs_ctx* ctx, hs_samples* s, const uint8_t* flags, int n, int* list, int* pos,
                         int* count) {
  const int nb = blocks_for(n, kScanTile);
  HS_TRY(scan_blocks(ctx, flags, n, s->scan));
  HS_LAUNCH(ctx, compact_kernel, nb, kBlock, flags, n, s->scan, list, pos);
  return readback(ctx, s->scan + nb, sizeof(int), count);
}

// hat mask -> tilde mask, both lists, pos and the neighbour table.
static hs_status finish_sets(hs_ctx* ctx, hs_samples* s) {
  const int n = s->ncell;
  const int nb = blocks_for(n);
  HS_LAUNCH(ctx, ring_kernel, nb, kBlock, ctx->g, s->mask, s->tmask);
  HS_TRY(compact(ctx, s, s->mask, n, s->hat, s->pos, &s->n_s));
  HS_TRY(compact(ctx, s, s->tmask, n, s->tilde, nullptr, &s->l));
  if (s->n_s > 0)
    HS_LAUNCH(ctx, nbr_table_kernel, blocks_for(s->n_s), kBlock, ctx->g, s->hat, s->n_s, n, s->pos, s->nbr);
  // active tiles of the tiled relaxation
  const int nt = ctx->ntx * ctx->nty;
  HS_LAUNCH(ctx, fill_u8_kernel, blocks_for(nt), kBlock, s->tflag, nt, (uint8_t)0);
  if (s->n_s > 0)
    HS_LAUNCH(ctx, tile_flag_kernel, blocks_for(s->n_s), kBlock, ctx->g, s->hat, s->n_s, ctx->tile_x,
              ctx->tile_y, ctx->ntx, s->tflag);
  HS_TRY(compact(ctx, s, s->tflag, nt, s->tiles, nullptr, &s->ntiles));
  return HS_OK;
}

}  // namespace hs

using namespace hs;

extern "C" {

hs_status hs_samples_create(hs_ctx* ctx, hs_samples** out) {
  if (!ctx || !out) return HS_ERR_INVALID_ARG;
  hs_samples* s = new hs_samples();
  s->ctx = ctx;
  s->ncell = ctx->ncell;
  const size_t n = ctx->ncell;
  void** bufs[] = {(void**)&s->gmask, (void**)&s->mask, (void**)&s->tmask, (void**)&s->dtmp};
  bool ok = true;
  for (void** b : bufs) ok = ok && hipMalloc(b, n + 64) == hipSuccess;
  ok = ok && hipMalloc((void**)&s->hat, n * 4 + 64) == hipSuccess;
  ok = ok && hipMalloc((void**)&s->tilde, n * 4 + 64) == hipSuccess;
  ok = ok && hipMalloc((void**)&s->pos, n * 4 + 64) == hipSuccess;
  ok = ok && hipMalloc((void**)&s->nbr, 4 * n * 4 + 64) == hipSuccess;
  const size_t nt = (size_t)ctx->ntx * ctx->nty;
  ok = ok && hipMalloc((void**)&s->tflag, nt + 64) == hipSuccess;
  ok = ok && hipMalloc((void**)&s->tiles, nt * 4 + 64) == hipSuccess;
  ok = ok && hipMalloc((void**)&s->scan, (n / kScanTile + 64) * 4 + sizeof(SelectState) + 64) == hipSuccess;
  if (!ok) {
    hs_samples_destroy(s);
    return ctx->fail(HS_ERR_OOM, "hipMalloc (samples)");
  }
  *out = s;
  return HS_OK;
}

hs_status hs_samples_destroy(hs_samples* s) {
  if (!s) return HS_ERR_INVALID_ARG;
  void* bufs[] = {s->gmask, s->mask, s->tmask, s->dtmp, s->hat, s->tilde, s->pos, s->nbr, s->scan,
                  s->tflag, s->tiles};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  delete s;
  return HS_OK;
}

hs_status hs_samples_counts(const hs_samples* s, int32_t* counts) {
  if (!s || !counts) return HS_ERR_INVALID_ARG;
  counts[0] = s->n_g;
  counts[1] = s->n_s;
  counts[2] = s->l;
  return HS_OK;
}

hs_status sample_select(hs_ctx* ctx, const double* eps, const hs_sample_params* sp, hs_samples* s) {
  if (!ctx || !eps || !sp || !s || s->ctx != ctx) return HS_ERR_INVALID_ARG;
  if (sp->halo < 0 || sp->halo > 8) return HS_ERR_INVALID_ARG;
  if (sp->rule == HS_RULE_FRACTION) {
    if (!(sp->fraction >= 0.0 && sp->fraction <= 1.0)) return HS_ERR_INVALID_ARG;
  } else if (sp->rule == HS_RULE_RRE) {
    return ctx->fail(HS_ERR_INVALID_ARG, "the RRE rule is not available in this build");
  } else {
    return HS_ERR_INVALID_ARG;
  }
  const int n = ctx->ncell;
  const int nb = blocks_for(n);
  // n_g = min(ceil(f * ncell), #{eps > 0})
  const int nbp = blocks_for(n, kBlock, 1024);
  HS_LAUNCH(ctx, count_positive_kernel, nbp, kBlock, eps, n, ctx->part);
  HS_TRY(finish_stats(ctx, nbp, 0u, 1u << kStatCount));
  unsigned long long st[kStatSlots];
  HS_TRY(read_stats(ctx, st));
  const long long npos = (long long)bits_to_double(st[kStatCount]);
  const long long want = (long long)std::ceil(sp->fraction * (double)n);
  const long long ng = std::min(want, npos);
  s->n_g = (int)ng;

  SelectState* state = reinterpret_cast<SelectState*>(s->scan + state_offset(n));
  unsigned int* hist = reinterpret_cast<unsigned int*>(ctx->ibuf);
  if (ng == 0) {
    HS_LAUNCH(ctx, fill_u8_kernel, nb, kBlock, s->gmask, n, (uint8_t)0);
  } else {
    HS_LAUNCH(ctx, fill_u8_kernel, blocks_for(256 * sizeof(unsigned int)), kBlock,
              reinterpret_cast<uint8_t*>(hist), (int)(256 * sizeof(unsigned int)), (uint8_t)0);
    HS_LAUNCH(ctx, init_state_kernel, 1, 1, state, ng);
    for (int shift = 56; shift >= 0; shift -= 8) {
      HS_LAUNCH(ctx, radix_hist_kernel, blocks_for(n, kBlock, 2048), kBlock, eps, n, state, shift, hist);
      HS_LAUNCH(ctx, radix_pick_kernel, 1, 256, state, shift, hist);
    }
    HS_LAUNCH(ctx, mark_kernel, nb, kBlock, eps, n, state, s->gmask, s->dtmp);
    HS_TRY(scan_blocks(ctx, s->dtmp, n, s->scan));
    HS_LAUNCH(ctx, tie_keep_kernel, blocks_for(n, kScanTile), kBlock, s->dtmp, n, s->scan, state, s->gmask);
  }
  // hat-S = dilate(G): x, then y
  const uint8_t* src = s->gmask;
  if (ctx->g.kind == HS_BURGERS_1D) {
    HS_LAUNCH(ctx, dilate_kernel, nb, kBlock, ctx->g, src, s->mask, 0, sp->halo);
  } else {
    HS_LAUNCH(ctx, dilate_kernel, nb, kBlock, ctx->g, src, s->dtmp, 0, sp->halo);
    HS_LAUNCH(ctx, dilate_kernel, nb, kBlock, ctx->g, s->dtmp, s->mask, 1, sp->halo);
  }
  return finish_sets(ctx, s);
}

hs_status hs_samples_set(hs_ctx* ctx, hs_samples* s, const int32_t* hat, int32_t n_s) {
  if (!ctx || !s || s->ctx != ctx || n_s < 0 || n_s > ctx->ncell || (n_s > 0 && !hat))
    return HS_ERR_INVALID_ARG;
  const int n = ctx->ncell;
  HS_LAUNCH(ctx, fill_u8_kernel, blocks_for(n), kBlock, s->mask, n, (uint8_t)0);
  if (n_s > 0) HS_LAUNCH(ctx, scatter_mask_kernel, blocks_for(n_s), kBlock, hat, n_s, n, s->mask);
  HS_TRY(finish_sets(ctx, s));
  if (s->n_s != n_s) return ctx->fail(HS_ERR_INVALID_ARG, "hat list has duplicates or out-of-range cells");
  s->n_g = n_s;
  return HS_OK;
}

hs_status hs_samples_export(hs_ctx* ctx, const hs_samples* s, int32_t* hat, int32_t* tilde, uint8_t* mask) {
  if (!ctx || !s) return HS_ERR_INVALID_ARG;
  if (hat && s->n_s) HIP_TRY(ctx, hipMemcpyAsync(hat, s->hat, s->n_s * 4, hipMemcpyDeviceToDevice, ctx->stream));
  if (tilde && s->l) HIP_TRY(ctx, hipMemcpyAsync(tilde, s->tilde, s->l * 4, hipMemcpyDeviceToDevice, ctx->stream));
  if (mask) HIP_TRY(ctx, hipMemcpyAsync(mask, s->mask, s->ncell, hipMemcpyDeviceToDevice, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return HS_OK;
}

}  // extern "C"
