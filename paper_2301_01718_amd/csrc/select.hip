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
// The RRE rule (eq. rre) first finds n_g with the same radix walk carrying
// exact fixed-point sums of the errors instead of counts.
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

// #{eps > 0} and max eps (per-block partials).
__global__ void count_positive_kernel(const double* __restrict__ eps, int n, double* __restrict__ part) {
  __shared__ int lds[kBlock / kWave];
  __shared__ double ldm[kBlock / kWave];
  int c = 0;
  double mx = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double e = eps[i];
    c += e > 0.0;
    mx = fmax(mx, e > 0.0 ? e : 0.0);
  }
  c = block_sum_int(c, lds);
  mx = block_max(mx, ldm);
  if (threadIdx.x == 0) {
    stat_part(part, kStatCount, (double)c);
    stat_part(part, kStatQMax, mx);
  }
}

// --------------------------------------------------------------- RRE rule
// eq. rre in integers: every error is encoded in 64-bit fixed point relative
// to the largest, q = floor(eps 2^(63 - emax)) (2^emax <= max eps <
// 2^(emax+1)), and all sums of q are exact integers (32-bit halves summed in
// 64-bit integers, integer atomics), so the decision RRE(n_g) >= delta does
// not depend on any summation order.  Comparisons S >= delta T are made as
// S 2^dsh >= dnum T with delta = dnum 2^-dsh, in 256-bit integers.  The
// encoding drops less than one unit of 2^(emax - 63) per error, so n_g is the
// one eq. rre gives with exact sums unless the exact ratio at the crossing
// lies within (n_g + N) 2^(emax - 63) / sum(eps) of delta; delta >= 1 is
// decided exactly (every positive error).
struct U256 {
  unsigned long long w[4];
};

__device__ inline U256 u256_small(unsigned long long lo, unsigned long long hi32sum) {
  // lo + hi32sum * 2^32
  U256 r{{0, 0, 0, 0}};
  r.w[0] = lo;
  const unsigned long long a = hi32sum << 32, b = hi32sum >> 32;
  r.w[0] += a;
  r.w[1] = b + (r.w[0] < a ? 1ull : 0ull);
  return r;
}

__device__ inline U256 u256_add(const U256& a, const U256& b) {
  U256 r;
  unsigned long long c = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const unsigned long long s = a.w[i] + b.w[i];
    const unsigned long long c1 = s < a.w[i];
    r.w[i] = s + c;
    const unsigned long long c2 = r.w[i] < s;
    c = c1 | c2;
  }
  return r;
}

__device__ inline U256 u256_shl(const U256& a, int sh) {   // 0 <= sh < 256
  U256 r{{0, 0, 0, 0}};
  const int ws = sh / 64, bs = sh % 64;
  for (int i = 3; i >= ws; --i) {
    unsigned long long v = a.w[i - ws] << bs;
    if (bs && i - ws - 1 >= 0) v |= a.w[i - ws - 1] >> (64 - bs);
    r.w[i] = v;
  }
  return r;
}

__device__ inline U256 u256_mul64(const U256& a, unsigned long long m) {
  U256 r{{0, 0, 0, 0}};
  unsigned long long carry = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const unsigned long long lo = a.w[i] * m, hi = __umul64hi(a.w[i], m);
    r.w[i] = lo + carry;
    carry = hi + (r.w[i] < lo ? 1ull : 0ull);
  }
  return r;
}

__device__ inline bool u256_ge(const U256& a, const U256& b) {
  for (int i = 3; i >= 0; --i)
    if (a.w[i] != b.w[i]) return a.w[i] > b.w[i];
  return true;
}

__device__ inline unsigned long long fixed_q(double e, int emax) {
  if (!(e > 0.0)) return 0ull;
  const unsigned long long b = dbits(e);
  const int ex = (int)(b >> 52);
  unsigned long long M = b & ((1ull << 52) - 1ull);
  int x;
  if (ex == 0) {
    x = -1074;                 // subnormal: e = M 2^-1074
  } else {
    M |= 1ull << 52;           // e = M 2^(ex - 1075)
    x = ex - 1075;
  }
  const int sh = x + 63 - emax;
  if (sh >= 0) return M << sh;
  if (sh <= -64) return 0ull;
  return M >> (-sh);
}

struct RreState {
  unsigned long long prefix;    // digits of the crossing key fixed so far
  long long count_above;        // keys above the prefix bucket
  U256 s_above;                 // sum of q above the prefix bucket
  U256 target;                  // dnum * T
  unsigned long long tot_lo, tot_hi;   // T = tot_lo + tot_hi 2^32
  long long ng;                 // result
  int dsh;
  int emax;
};

__global__ void rre_total_kernel(const double* __restrict__ eps, int n, int emax, RreState* st) {
  __shared__ unsigned long long slo[kBlock / kWave], shi[kBlock / kWave];
  unsigned long long lo = 0, hi = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const unsigned long long q = fixed_q(eps[i], emax);
    lo += q & 0xffffffffull;
    hi += q >> 32;
  }
  for (int o = kWave / 2; o > 0; o >>= 1) {
    lo += __shfl_xor(lo, o, kWave);
    hi += __shfl_xor(hi, o, kWave);
  }
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  if (lane == 0) {
    slo[w] = lo;
    shi[w] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long a = 0, b = 0;
    for (int k = 0; k < (int)(blockDim.x / kWave); ++k) {
      a += slo[k];
      b += shi[k];
    }
    atomicAdd(&st->tot_lo, a);
    atomicAdd(&st->tot_hi, b);
  }
}

__global__ void rre_init_kernel(RreState* st, unsigned long long dnum, int dsh, int emax) {
  const U256 T = u256_small(st->tot_lo, st->tot_hi);
  st->target = u256_mul64(T, dnum);
  st->dsh = dsh;
  st->emax = emax;
  st->prefix = 0ull;
  st->count_above = 0;
  st->s_above = U256{{0, 0, 0, 0}};
  st->ng = 0;
}

// Per digit of the keys under the current prefix: count and the exact sum
// of q (two 64-bit integer halves).
__global__ void rre_hist_kernel(const double* __restrict__ eps, int n, const RreState* st, int shift,
                                unsigned int* __restrict__ cnt, unsigned long long* __restrict__ slo,
                                unsigned long long* __restrict__ shi) {
  __shared__ unsigned int c[256];
  __shared__ unsigned long long l[256], h[256];
  for (int t = threadIdx.x; t < 256; t += blockDim.x) {
    c[t] = 0;
    l[t] = 0;
    h[t] = 0;
  }
  __syncthreads();
  const unsigned long long himask = shift >= 56 ? 0ull : (~0ull << (shift + 8));
  const unsigned long long pre = st->prefix & himask;
  const int emax = st->emax;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double e = eps[i];
    if (!(e > 0.0)) continue;
    const unsigned long long key = dbits(e);
    if ((key & himask) != pre) continue;
    const int d = (int)((key >> shift) & 255u);
    const unsigned long long q = fixed_q(e, emax);
    atomicAdd(&c[d], 1u);
    atomicAdd(&l[d], q & 0xffffffffull);
    atomicAdd(&h[d], q >> 32);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < 256; t += blockDim.x) {
    if (c[t]) {
      atomicAdd(&cnt[t], c[t]);
      atomicAdd(&slo[t], l[t]);
      atomicAdd(&shi[t], h[t]);
    }
  }
}

// One thread: walk the digits from the largest down, adding bucket sums to
// the running sum above, and fix the digit whose bucket crosses the target;
// then clear the histograms.
__global__ void rre_pick_kernel(RreState* st, int shift, unsigned int* __restrict__ cnt,
                                unsigned long long* __restrict__ slo, unsigned long long* __restrict__ shi) {
  if (threadIdx.x == 0) {
    U256 acc = st->s_above;
    long long ca = st->count_above;
    for (int d = 255; d >= 0; --d) {
      if (cnt[d] == 0) continue;
      const U256 nxt = u256_add(acc, u256_small(slo[d], shi[d]));
      if (u256_ge(u256_shl(nxt, st->dsh), st->target)) {
        st->prefix |= (unsigned long long)d << shift;
        break;
      }
      acc = nxt;
      ca += cnt[d];
    }
    st->s_above = acc;
    st->count_above = ca;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < 256; t += blockDim.x) {
    cnt[t] = 0;
    slo[t] = 0;
    shi[t] = 0;
  }
}

// The crossing key K is fixed; its tied keys all carry q_K.  n_g = count
// above K + the smallest t with (S_above + t q_K) 2^dsh >= dnum T.
__global__ void rre_final_kernel(RreState* st, long long ties) {
  const unsigned long long K = st->prefix;
  const unsigned long long qk = fixed_q(__longlong_as_double((long long)K), st->emax);
  long long lo = 1, hi = ties > 0 ? ties : 1;
  while (lo < hi) {
    const long long mid = lo + (hi - lo) / 2;
    const U256 v = u256_add(st->s_above, u256_mul64(U256{{qk, 0, 0, 0}}, (unsigned long long)mid));
    if (u256_ge(u256_shl(v, st->dsh), st->target)) hi = mid;
    else lo = mid + 1;
  }
  st->ng = st->count_above + lo;
}

// Number of keys equal to K (the last pass's bucket, counted again).
__global__ void count_key_kernel(const double* __restrict__ eps, int n, const RreState* st,
                                 unsigned int* __restrict__ out) {
  __shared__ int lds[kBlock / kWave];
  int c = 0;
  const unsigned long long K = st->prefix;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double e = eps[i];
    c += (e > 0.0) && dbits(e) == K;
  }
  c = block_sum_int(c, lds);
  if (threadIdx.x == 0 && c) atomicAdd(out, (unsigned int)c);
}

// Exclusive prefix sum of a per-thread count within its block.
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

// Keys whose digit is shared by many lanes of a wave (the exponent digits of
// errors that span a few binades) are counted once per wave: up to four
// rounds in which the first pending lane's digit is matched across the wave
// and added with its lane count; the remaining lanes add one each.
__device__ inline void wave_hist_add(unsigned int* h, unsigned d, bool pending) {
  const int lane = threadIdx.x % kWave;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const unsigned long long act = __ballot(pending);
    if (act == 0ull) return;
    const int leader = __ffsll((long long)act) - 1;
    const unsigned dl = __shfl(d, leader, kWave);
    const bool match = pending && d == dl;
    const unsigned long long mm = __ballot(match);
    if (lane == leader) atomicAdd(&h[dl], (unsigned)__popcll(mm));
    pending = pending && !match;
  }
  if (pending) atomicAdd(&h[d], 1u);
}

// The global histogram has kHistCopies copies, a block adding into copy
// blockIdx % kHistCopies: the blocks' additions to a common digit (all the
// keys of one binade) would otherwise serialise on one address.
constexpr int kHistCopies = 8;

constexpr int kHistWords = kHistCopies * 256;   // one histogram buffer
constexpr int kRadixBlocks = 512;               // workgroups of a digit pass

// The digit of the previous pass, taken by every workgroup of 256 threads
// from that pass's histogram buffer (thread t on digit 255 - t): the
// exclusive prefix over t counts the keys with a larger digit, and the
// bucket holding the k-th largest key fixes the digit.  Returns the state
// after that digit (the same in every workgroup).
// With ngd != nullptr (the first digit, whose histogram holds every positive
// key) the rank is first capped at #{eps > 0}: n_g = min(k, #{eps > 0}) of
// the fraction rule, stored to *ngd by workgroup 0.
__device__ inline SelectState radix_pick(const unsigned int* __restrict__ hist, int shift, SelectState s,
                                         int* wsum, SelectState* sh, long long* ngd = nullptr) {
  const int d = 255 - (int)threadIdx.x;
  int c = 0;
#pragma unroll
  for (int k = 0; k < kHistCopies; ++k) c += (int)hist[k * 256 + d];
  if (threadIdx.x == 0) *sh = s;
  const int above = block_exclusive_rank(c, wsum);
  if (ngd != nullptr) {
    __shared__ long long npos;
    if (threadIdx.x == 255) npos = (long long)above + c;
    __syncthreads();
    if (s.k > npos) s.k = npos;
    if (threadIdx.x == 0) {
      sh->k = s.k;
      if (blockIdx.x == 0) *ngd = s.k;
    }
    __syncthreads();
  }
  if (c > 0 && (long long)above < s.k && s.k <= (long long)above + c) {
    sh->prefix = s.prefix | ((unsigned long long)d << shift);
    sh->k = s.k - above;
  }
  __syncthreads();
  const SelectState r = *sh;
  __syncthreads();
  return r;
}

// Digit pass p (shift 56 - 8p) of the radix select, 256 threads: the digit
// of pass p - 1 from its buffer, the state after it (workgroup 0 stores it
// for pass p + 1), then this pass's histogram of the keys that share the
// fixed digits.  Buffers rotate over three: pass p fills p % 3, reads
// (p - 1) % 3 and clears (p + 1) % 3, which the pass before it read and the
// pass after it fills.  States alternate over two slots.
__global__ void __launch_bounds__(256) radix_pass_kernel(const double* __restrict__ eps, int n,
                                                         SelectState* __restrict__ st2, int p,
                                                         unsigned int* __restrict__ hist3,
                                                         long long* __restrict__ ngd) {
  __shared__ unsigned int h[256];
  __shared__ int wsum[256 / kWave];
  __shared__ SelectState sh;
  const int shift = 56 - 8 * p;
  h[threadIdx.x] = 0;
  unsigned int* nxt = hist3 + ((p + 1) % 3) * kHistWords;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < kHistWords; i += gridDim.x * 256) nxt[i] = 0u;
  SelectState s = st2[(p + 1) % 2];
  if (p > 0) s = radix_pick(hist3 + ((p - 1) % 3) * kHistWords, shift + 8, s, wsum, &sh, p == 1 ? ngd : nullptr);
  if (blockIdx.x == 0 && threadIdx.x == 0) st2[p % 2] = s;
  __syncthreads();
  const unsigned long long himask = shift >= 56 ? 0ull : (~0ull << (shift + 8));
  const unsigned long long pre = s.prefix & himask;
  const int stride = gridDim.x * 256;
  // the trip count is uniform across a wave (every lane takes part in the ballots)
  for (int base = blockIdx.x * 256; base < n; base += stride) {
    const int i = base + threadIdx.x;
    const double e = i < n ? eps[i] : 0.0;
    const unsigned long long key = dbits(e);
    const bool take = e > 0.0 && (key & himask) == pre;
    wave_hist_add(h, (unsigned)(key >> shift) & 255u, take);
  }
  __syncthreads();
  unsigned int* copy = hist3 + (p % 3) * kHistWords + (blockIdx.x % kHistCopies) * 256;
  if (h[threadIdx.x]) atomicAdd(&copy[threadIdx.x], h[threadIdx.x]);
}

// The last digit (pass 7's buffer), then gmask = key > K and emask = key == K
// (candidates for the remaining ties) on the workgroup's scan tile of
// kScanTile cells, whose emask count goes to bsum[blockIdx.x] for the tie
// scan; workgroup 0 stores the final state in slot 0 for the tie pass.
// 256 threads, one workgroup per scan tile.
__global__ void __launch_bounds__(256) radix_mark_kernel(const double* __restrict__ eps, int n,
                                                         SelectState* __restrict__ st2,
                                                         const unsigned int* __restrict__ hist3,
                                                         const long long* __restrict__ ngd,
                                                         uint8_t* __restrict__ gmask, uint8_t* __restrict__ emask,
                                                         int* __restrict__ bsum) {
  __shared__ int wsum[256 / kWave];
  __shared__ int lds[256 / kWave];
  __shared__ SelectState sh;
  const SelectState s = radix_pick(hist3 + (7 % 3) * kHistWords, 0, st2[7 % 2], wsum, &sh);
  if (blockIdx.x == 0 && threadIdx.x == 0) st2[0] = s;
  const unsigned long long K = s.prefix;
  const bool any = *ngd > 0;   // n_g = 0: nothing is marked
  const int base = blockIdx.x * kScanTile;
  int c = 0;
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    const int i = base + r * 256 + threadIdx.x;
    if (i < n) {
      const double e = eps[i];
      const unsigned long long key = e > 0.0 ? dbits(e) : 0ull;
      const bool tie = any && (e > 0.0) && key == K;
      gmask[i] = any && (e > 0.0) && key > K;
      emask[i] = tie;
      c += tie;
    }
  }
  c = block_sum_int(c, lds);
  if (threadIdx.x == 0) bsum[blockIdx.x] = c;
}

// ------------------------------------------------------------- block scan
// Exclusive scan of per-block totals, then per-element ranks.
// Single block: exclusive scan of nb block sums in place; total to bsum[nb].
__device__ inline void scan_bsums_block(int* __restrict__ bsum, int nb) {
  __shared__ int carry;
  __shared__ int wsum[kBlock / kWave];
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < nb; base += kBlock) {
    const int i = base + threadIdx.x;
    const int v = i < nb ? bsum[i] : 0;
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

__global__ void scan_bsums_kernel(int* __restrict__ bsum, int nb) { scan_bsums_block(bsum, nb); }

// Compaction: list[offset] = i for every set flag, pos[i] = offset or -1.
// Block b of a stream compaction: list[rank] = i for the flagged i of its
// tile (bsum: exclusive scan of the tiles' counts); pos[i] = rank or -1.
__device__ inline void compact_block(const uint8_t* __restrict__ f, int n, const int* __restrict__ bsum,
                                     int* __restrict__ list, int* __restrict__ pos, int b) {
  __shared__ int wsum[kBlock / kWave];
  __shared__ int run;
  if (threadIdx.x == 0) run = 0;
  __syncthreads();
  const int base = b * kScanTile;
  const int off = bsum[b];
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
  int i, j;
  cell_ij(g, c, i, j);
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
// (It also clears the nt tile flags that tile_flag_mask_kernel sets next.)
__global__ void ring_kernel(Grid g, const uint8_t* __restrict__ mask, uint8_t* __restrict__ tmask,
                            uint8_t* __restrict__ tflag, int nt) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < nt) tflag[c] = 0;
  if (c >= g.ncell) return;
  if (mask[c]) {
    tmask[c] = 0;
    return;
  }
  int i, j;
  cell_ij(g, c, i, j);
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
  int i, j;
  cell_ij(g, cell, i, j);
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

__global__ void fill_u8_kernel(uint8_t* p, int n, uint8_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// The tiles that hold a hat-S cell, from the mask (the same set as from the
// list, available before the list is compacted).
__global__ void tile_flag_mask_kernel(Grid g, const uint8_t* __restrict__ mask, int tx, int ty, int ntx,
                                      uint8_t* __restrict__ tflag) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.ncell || !mask[c]) return;
  int i, j;
  cell_ij(g, c, i, j);
  tflag[(j / ty) * ntx + i / tx] = 1;
}

// Three flag arrays compacted together: the block counts of all three in one
// launch, the scans of the three block-sum arrays in another (one workgroup
// each), then a compaction per array and one read-back of the three totals.
struct Flags3 {
  const uint8_t* f[3];
  int n[3];
  int nb[3];     // blocks_for(n, kScanTile)
  int* bsum[3];  // nb + 1 entries each
};

__global__ void flag_count3_kernel(Flags3 fl, int* __restrict__ ticket) {
  __shared__ int lds[kBlock / kWave];
  if (blockIdx.x == 0 && threadIdx.x == 0) *ticket = 0;   // for scan_bsums3_kernel
  int a = 0, b = blockIdx.x;
  if (b >= fl.nb[0]) {
    b -= fl.nb[0];
    a = 1;
    if (b >= fl.nb[1]) {
      b -= fl.nb[1];
      a = 2;
    }
  }
  const uint8_t* f = fl.f[a];
  const int n = fl.n[a];
  const int base = b * kScanTile;
  int c = 0;
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    const int i = base + r * kBlock + threadIdx.x;
    if (i < n) c += f[i] != 0;
  }
  c = block_sum_int(c, lds);
  if (threadIdx.x == 0) fl.bsum[a][b] = c;
}

// The three compactions of the sets (hat-S with positions, tilde-S, active
// tiles) in one launch: blocks [0, nb0) take array 0, the next nb1 array 1,
// the rest array 2 (the split of flag_count3_kernel).
struct Lists3 {
  int* list[3];
  int* pos0;
};

__global__ void compact3_kernel(Flags3 fl, Lists3 out) {
  int a = 0, b = blockIdx.x;
  if (b >= fl.nb[0]) {
    b -= fl.nb[0];
    a = 1;
    if (b >= fl.nb[1]) {
      b -= fl.nb[1];
      a = 2;
    }
  }
  compact_block(fl.f[a], fl.n[a], fl.bsum[a], out.list[a], a == 0 ? out.pos0 : nullptr, b);
}

// Workgroup a scans array a's block sums; the totals also go to totals[a],
// and n_g (when ngd is given) to totals[3].  The last of the three
// workgroups to finish (ticket at totals[4], cleared by flag_count3_kernel)
// posts totals[0..3] to the host, so the sizes are read while the
// compactions behind this kernel run.
__global__ void scan_bsums3_kernel(Flags3 fl, int* __restrict__ totals, const long long* __restrict__ ngd,
                                   PostSlot post) {
  __shared__ int last;
  const int a = blockIdx.x;
  scan_bsums_block(fl.bsum[a], fl.nb[a]);
  if (threadIdx.x == 0) {
    totals[a] = fl.bsum[a][fl.nb[a]];
    if (a == 0) totals[3] = ngd ? (int)*ngd : 0;
    __threadfence();   // this workgroup's totals before its ticket
    last = atomicAdd(&totals[4], 1) == (int)gridDim.x - 1;
    if (last) __threadfence();   // the other workgroups' totals after their tickets
  }
  __syncthreads();
  if (!last) return;
  __shared__ uint32_t words[4];
  if (threadIdx.x < 4) words[threadIdx.x] = (uint32_t)__hip_atomic_load(&totals[threadIdx.x], __ATOMIC_RELAXED,
                                                                         __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  if (threadIdx.x < kWave) post_words(words, 4, post.dst, post.tagp, post.tag);
}

// One block of 256 threads: the state before the first digit (slot 1) of a
// selection of rank k (capped at #{eps > 0} by the first digit pick, which
// also stores n_g), and a cleared first histogram buffer.
__global__ void init_state_kernel(SelectState* st2, long long k, unsigned int* __restrict__ hist3) {
#pragma unroll
  for (int c = 0; c < kHistCopies; ++c) hist3[c * 256 + threadIdx.x] = 0u;
  if (threadIdx.x == 0) {
    st2[1].prefix = 0ull;
    st2[1].k = k;
  }
}

// ------------------------------------------------------------------- host
// The select state lives after the block sums in the scan buffer, 8-byte aligned.
static size_t state_offset(int n) { return ((size_t)n / kScanTile + 32) & ~(size_t)1; }

// n_g of the RRE rule (exact fixed-point sums), given #{eps > 0} and max eps.
static hs_status rre_count(hs_ctx* ctx, const double* eps, int n, double delta, long long npos, double emx,
                           long long* ng) {
  if (npos == 0) { *ng = 0; return HS_OK; }
  // RRE(n) reaches 1 only with every positive error in the sum, and never exceeds it
  if (delta >= 1.0) { *ng = npos; return HS_OK; }
  if (!(delta > std::ldexp(1.0, -64))) { *ng = 1; return HS_OK; }   // the largest q alone exceeds delta T
  int de;
  const double dm = std::frexp(delta, &de);                 // delta = dm 2^de, 0.5 <= dm < 1
  const unsigned long long dnum = (unsigned long long)std::ldexp(dm, 53);
  const int dsh = 53 - de;                                  // delta = dnum 2^-dsh, dsh <= 117
  const int emax = std::ilogb(emx);
  // scratch in the integer buffer: histograms (8-byte aligned) and the state
  unsigned char* base = reinterpret_cast<unsigned char*>(ctx->ibuf) + 8192;
  unsigned int* cnt = reinterpret_cast<unsigned int*>(base);
  unsigned long long* slo = reinterpret_cast<unsigned long long*>(base + 1024);
  unsigned long long* shi = reinterpret_cast<unsigned long long*>(base + 3072);
  RreState* rs = reinterpret_cast<RreState*>(base + 5120);
  unsigned int* ties = reinterpret_cast<unsigned int*>(base + 5120 + 256);
  const int bytes = 5120 + 256 + 64;
  HS_LAUNCH(ctx, fill_u8_kernel, blocks_for(bytes), kBlock, base, bytes, (uint8_t)0);
  HS_LAUNCH(ctx, rre_total_kernel, blocks_for(n, kBlock, 1024), kBlock, eps, n, emax, rs);
  HS_LAUNCH(ctx, rre_init_kernel, 1, 1, rs, dnum, dsh, emax);
  for (int shift = 56; shift >= 0; shift -= 8) {
    HS_LAUNCH(ctx, rre_hist_kernel, blocks_for(n, kBlock, 2048), kBlock, eps, n, rs, shift, cnt, slo, shi);
    HS_LAUNCH(ctx, rre_pick_kernel, 1, 256, rs, shift, cnt, slo, shi);
  }
  HS_LAUNCH(ctx, count_key_kernel, blocks_for(n, kBlock, 1024), kBlock, eps, n, rs, ties);
  unsigned int nt;
  HS_TRY(readback(ctx, ties, sizeof nt, &nt));
  HS_LAUNCH(ctx, rre_final_kernel, 1, 1, rs, (long long)nt);
  long long r;
  HS_TRY(readback(ctx, &rs->ng, sizeof r, &r));
  *ng = std::min(r, npos);
  return HS_OK;
}

// hat mask -> tilde mask, both lists, pos, the neighbour table and the
// active tiles of the tiled relaxation; one read-back for the three counts.
static hs_status finish_sets(hs_ctx* ctx, hs_samples* s, const long long* ngd = nullptr) {
  const int n = s->ncell;
  const int nb = blocks_for(n);
  const int nt = ctx->sntx * ctx->snty;
  // the ring's grid covers the tile flags (nt <= n)
  HS_LAUNCH(ctx, ring_kernel, nb, kBlock, ctx->g, s->mask, s->tmask, s->tflag, nt);
  HS_LAUNCH(ctx, tile_flag_mask_kernel, nb, kBlock, ctx->g, s->mask, ctx->stile_x, ctx->stile_y, ctx->sntx,
            s->tflag);
  Flags3 fl;
  const uint8_t* flags[3] = {s->mask, s->tmask, s->tflag};
  const int lens[3] = {n, n, nt};
  const size_t region = (size_t)n / kScanTile + 64;
  for (int a = 0; a < 3; ++a) {
    fl.f[a] = flags[a];
    fl.n[a] = lens[a];
    fl.nb[a] = blocks_for(lens[a], kScanTile);
    fl.bsum[a] = s->scan3 + a * region;
  }
  int* totals = s->scan3 + 3 * region;   // 4 totals and the scan's ticket
  HS_LAUNCH(ctx, flag_count3_kernel, fl.nb[0] + fl.nb[1] + fl.nb[2], kBlock, fl, totals + 4);
  const PostSlot ps = post_slot(ctx);
  HS_LAUNCH(ctx, scan_bsums3_kernel, 3, kBlock, fl, totals, ngd, ps);
  const Lists3 lists{{s->hat, s->tilde, s->tiles}, s->pos};
  HS_LAUNCH(ctx, compact3_kernel, fl.nb[0] + fl.nb[1] + fl.nb[2], kBlock, fl, lists);
  int cnt[4];
  HS_TRY(await_post(ctx, ps, cnt, sizeof cnt));
  s->n_s = cnt[0];
  s->l = cnt[1];
  s->ntiles = cnt[2];
  if (ngd) s->n_g = cnt[3];
  if (s->n_s > 0)
    HS_LAUNCH(ctx, nbr_table_kernel, blocks_for(s->n_s), kBlock, ctx->g, s->hat, s->n_s, n, s->pos, s->nbr);
  return HS_OK;
}

// mask[point % ncell] = 1 for entries of the state vector (points < nc ncell).
__global__ void point_cells_kernel(const int32_t* __restrict__ points, int np, int ncell, long long n,
                                   uint8_t* __restrict__ mask) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const int p = points[i];
  if (p >= 0 && p < n) mask[p % ncell] = 1;
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
  const size_t nt = (size_t)ctx->sntx * ctx->snty;
  ok = ok && hipMalloc((void**)&s->tflag, nt + 64) == hipSuccess;
  ok = ok && hipMalloc((void**)&s->tiles, nt * 4 + 64) == hipSuccess;
  ok = ok && hipMalloc((void**)&s->scan, (n / kScanTile + 64) * 4 + sizeof(SelectState) + 64) == hipSuccess;
  ok = ok && hipMalloc((void**)&s->scan3, (3 * (n / kScanTile + 64) + 64) * 4) == hipSuccess;
  if (!ok) {
    hs_samples_destroy(s);
    return ctx->fail(HS_ERR_OOM, "hipMalloc (samples)");
  }
  *out = s;
  return HS_OK;
}

hs_status hs_samples_destroy(hs_samples* s) {
  if (!s) return HS_ERR_INVALID_ARG;
  void* bufs[] = {s->gmask, s->mask, s->tmask, s->dtmp, s->hat, s->tilde, s->pos, s->nbr, s->scan, s->scan3,
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
    if (!std::isfinite(sp->delta)) return HS_ERR_INVALID_ARG;
  } else {
    return HS_ERR_INVALID_ARG;
  }
  const int n = ctx->ncell;
  const int nb = blocks_for(n);
  const int nbp = blocks_for(n, kBlock, 1024);
  SelectState* state = reinterpret_cast<SelectState*>(s->scan + state_offset(n));
  long long* ngd = reinterpret_cast<long long*>(state + 2);
  unsigned int* hist = reinterpret_cast<unsigned int*>(ctx->ibuf);
  long long k;   // the rank the digit passes look for
  if (sp->rule == HS_RULE_FRACTION) {
    // n_g = min(ceil(f * ncell), #{eps > 0}): the first digit pick caps the
    // rank at the positive count of its histogram and stores n_g, read back
    // with the set sizes
    k = (long long)std::ceil(sp->fraction * (double)n);
  } else {
    HS_LAUNCH(ctx, count_positive_kernel, nbp, kBlock, eps, n, ctx->part);
    unsigned long long st[kStatSlots];
    HS_TRY(finish_stats(ctx, nbp, 1u << kStatQMax, 1u << kStatCount, st));
    const long long npos = (long long)bits_to_double(st[kStatCount]);
    const double emx = bits_to_double(st[kStatQMax]);
    HS_TRY(rre_count(ctx, eps, n, sp->delta, npos, emx, &k));
  }
  const int rb = blocks_for(n, 256, kRadixBlocks);
  HS_LAUNCH(ctx, init_state_kernel, 1, 256, state, k, hist);
  for (int p = 0; p < 8; ++p) HS_LAUNCH(ctx, radix_pass_kernel, rb, 256, eps, n, state, p, hist, ngd);
  // the mark pass also counts each scan tile's tie candidates
  const int nbs = blocks_for(n, kScanTile);
  HS_LAUNCH(ctx, radix_mark_kernel, nbs, 256, eps, n, state, hist, (const long long*)ngd, s->gmask, s->dtmp,
            s->scan);
  HS_LAUNCH(ctx, scan_bsums_kernel, 1, kBlock, s->scan, nbs);
  HS_LAUNCH(ctx, tie_keep_kernel, blocks_for(n, kScanTile), kBlock, s->dtmp, n, s->scan, state, s->gmask);
  // hat-S = dilate(G): x, then y
  const uint8_t* src = s->gmask;
  if (ctx->g.kind == HS_BURGERS_1D) {
    HS_LAUNCH(ctx, dilate_kernel, nb, kBlock, ctx->g, src, s->mask, 0, sp->halo);
  } else {
    HS_LAUNCH(ctx, dilate_kernel, nb, kBlock, ctx->g, src, s->dtmp, 0, sp->halo);
    HS_LAUNCH(ctx, dilate_kernel, nb, kBlock, ctx->g, s->dtmp, s->mask, 1, sp->halo);
  }
  return finish_sets(ctx, s, ngd);
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

hs_status hs_samples_add_points(hs_ctx* ctx, hs_samples* s, const int32_t* points, int32_t n_p) {
  if (!ctx || !s || s->ctx != ctx || n_p < 0 || (n_p > 0 && !points)) return HS_ERR_INVALID_ARG;
  if (n_p == 0) return HS_OK;
  HS_LAUNCH(ctx, point_cells_kernel, blocks_for(n_p), kBlock, points, n_p, ctx->ncell, (long long)ctx->n, s->mask);
  const int n_g = s->n_g;
  HS_TRY(finish_sets(ctx, s));
  s->n_g = n_g;
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
