// Algorithm 1 as one call, and its adjoint (the trajectory part of the
// boundary): hs_traj_forward runs the whole schedule of full and hybrid
// steps with the sampling and basis updates after each step, recording every
// decision the adjoint keeps frozen (the step schedule, the sampled sets, J,
// the filter passes and their kept-cell masks, the bases) and a checkpoint of
// the state every K steps; hs_traj_backward walks the checkpointed segments
// backwards, replays each segment from its checkpoint (checking that the
// replay reproduces the next checkpoint bit for bit) and applies the step
// adjoints in reverse order.
//
// Schedule (Alg. 1): full steps for k + 1 <= w and k mod z == 0, and
// wherever no sampled set or basis exists; a hybrid step whose Newton solve
// does not converge or whose fit has rank zero is redone as a full step.
// After step k (k >= w - 1, step k + 1 not full, k < N_t): the indicator of
// gamma_k (from the hybrid step itself, or with the latest basis after a full
// step) selects the sampled set of step k + 1, and the basis and reference
// state are rebuilt from the window of the last w + 1 snapshots.
#include "common.hpp"

#include <cstring>
#include <map>
#include <vector>

namespace hs {

__global__ void differ_kernel(const double* __restrict__ a, const double* __restrict__ b, long long n,
                              int* __restrict__ flag) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    // bit patterns: equal values that differ in sign of zero or NaN payload count as different
    if (__double_as_longlong(a[i]) != __double_as_longlong(b[i])) {
      atomicOr(flag, 1);
      return;
    }
  }
}

__global__ void zero_int_kernel(int* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

// y += x; and y = x / w (acc == 0) or y += x / w (acc == 1): the share of a
// psi adjoint that goes to one of the w snapshots psi averages.
__global__ void axpy_kernel(long long n, const double* __restrict__ x, double* __restrict__ y) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] += x[i];
}

__global__ void share_kernel(long long n, const double* __restrict__ x, double w, double* __restrict__ y, int acc) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] = acc ? y[i] + x[i] / w : x[i] / w;
}

}  // namespace hs

struct hs_tape {
  hs_ctx* ctx = nullptr;
  hs_traj_params p{};
  bool recorded = false;
  std::vector<double*> ring;   // w + 2 snapshot slots
  double* eps = nullptr;       // ncell
  double* sigma = nullptr;     // w_max
  int* flag = nullptr;         // replay check
  hs_samples* samples = nullptr;
  struct Basis {
    double* Phi = nullptr;
    double* psi = nullptr;
    int m = 0;
    int k_update = 0;              // the step the update followed: psi averages gamma_{k-w+1} .. gamma_k
  };
  std::vector<Basis> bases;        // one per basis update
  std::vector<int> kind;           // per step 1..steps (index k): 0 full, 1 hybrid
  std::vector<int> bver;           // basis version of a hybrid step (-1: none)
  std::vector<hs_htape*> ht;       // per hybrid step (nullptr otherwise)
  std::map<int, double*> ckpt;     // checkpoints (step -> state)
  std::vector<double*> seg;        // K + 1 segment states (backward)
  double* lam[2] = {nullptr, nullptr};
  double* lam_psi = nullptr;       // a hybrid step's psi adjoint (backward through psi)
  std::vector<double*> pool;       // spare N-vectors for the pending psi contributions
};

namespace hs {

static void tape_release_run(hs_tape* t) {
  for (auto& b : t->bases) {
    if (b.Phi) (void)hipFree(b.Phi);
    if (b.psi) (void)hipFree(b.psi);
  }
  t->bases.clear();
  for (hs_htape* h : t->ht)
    if (h) hs_htape_destroy(h);
  t->ht.clear();
  for (auto& kv : t->ckpt) (void)hipFree(kv.second);
  t->ckpt.clear();
  for (double* s : t->seg) (void)hipFree(s);
  for (double* s : t->pool) (void)hipFree(s);
  t->pool.clear();
  if (t->lam_psi) (void)hipFree(t->lam_psi);
  t->lam_psi = nullptr;
  t->seg.clear();
  t->kind.clear();
  t->bver.clear();
  t->recorded = false;
}

static hs_status dalloc(hs_ctx* ctx, void** p, size_t bytes) {
  if (hipMalloc(p, bytes) != hipSuccess) {
    *p = nullptr;
    return ctx->fail(HS_ERR_OOM, "trajectory tape: device allocation failed");
  }
  return HS_OK;
}

static hs_status dcopy(hs_ctx* ctx, double* dst, const double* src, long long n) {
  HIP_TRY(ctx, hipMemcpyAsync(dst, src, (size_t)n * 8, hipMemcpyDeviceToDevice, ctx->stream));
  return HS_OK;
}

static bool full_by_schedule(int k, int w, int z) { return k + 1 <= w || k % z == 0; }
static bool wants_update(int k, int w, int z, int steps) { return k >= w - 1 && (k + 1) % z != 0 && k < steps; }

static hs_status check_params(hs_ctx* ctx, const hs_traj_params* p) {
  if (!p) return HS_ERR_INVALID_ARG;
  if (p->steps < 1 || p->checkpoint_every < 1 || p->z < 1) return HS_ERR_INVALID_ARG;
  if (p->w < 2 || p->w > ctx->p.w_max || p->m < 1 || p->m > ctx->p.m_max || p->m > p->w) return HS_ERR_INVALID_ARG;
  if (p->hybrid.precision != HS_FP64)
    return ctx->fail(HS_ERR_INVALID_ARG, "the trajectory adjoint runs on an FP64 basis");
  if (p->psi_adjoint != 0 && p->psi_adjoint != 1) return HS_ERR_INVALID_ARG;
  return HS_OK;
}

}  // namespace hs

using namespace hs;

extern "C" {

hs_status hs_tape_create(hs_ctx* ctx, hs_tape** out) {
  if (!ctx || !out) return HS_ERR_INVALID_ARG;
  *out = new hs_tape();
  (*out)->ctx = ctx;
  return HS_OK;
}

hs_status hs_tape_destroy(hs_tape* t) {
  if (!t) return HS_ERR_INVALID_ARG;
  tape_release_run(t);
  for (double* s : t->ring) (void)hipFree(s);
  if (t->eps) (void)hipFree(t->eps);
  if (t->sigma) (void)hipFree(t->sigma);
  if (t->flag) (void)hipFree(t->flag);
  for (double* l : t->lam)
    if (l) (void)hipFree(l);
  if (t->samples) hs_samples_destroy(t->samples);
  delete t;
  return HS_OK;
}

hs_status hs_traj_forward(hs_ctx* ctx, const double* q0, const hs_traj_params* params, hs_tape* t, double* qT) {
  if (!ctx || !q0 || !t || !qT || t->ctx != ctx) return HS_ERR_INVALID_ARG;
  HS_TRY(check_params(ctx, params));
  const hs_traj_params p = *params;
  const long long n = ctx->n;
  tape_release_run(t);
  t->p = p;
  // the snapshot ring and the per-run buffers (kept across runs while the
  // window length allows)
  const int nslot = p.w + 2;
  while ((int)t->ring.size() < nslot) {
    double* s = nullptr;
    HS_TRY(dalloc(ctx, (void**)&s, (size_t)n * 8));
    t->ring.push_back(s);
  }
  if (!t->eps) HS_TRY(dalloc(ctx, (void**)&t->eps, (size_t)ctx->ncell * 8));
  if (!t->sigma) HS_TRY(dalloc(ctx, (void**)&t->sigma, (size_t)kMaxBasis * 8));
  if (!t->flag) HS_TRY(dalloc(ctx, (void**)&t->flag, sizeof(int)));
  if (!t->samples) HS_TRY(hs_samples_create(ctx, &t->samples));
  t->kind.assign(p.steps + 1, 0);
  t->bver.assign(p.steps + 1, -1);
  t->ht.assign(p.steps + 1, nullptr);
  auto slot = [&](int k) { return t->ring[k % nslot]; };

  HS_TRY(dcopy(ctx, slot(0), q0, n));
  {
    double* c0 = nullptr;
    HS_TRY(dalloc(ctx, (void**)&c0, (size_t)n * 8));
    t->ckpt[0] = c0;
    HS_TRY(dcopy(ctx, c0, q0, n));
  }
  int cur = -1;            // current basis version
  bool have_samples = false;
  for (int k = 1; k <= p.steps; ++k) {
    const double* prev = slot(k - 1);
    double* out = slot(k);
    bool hybrid = !full_by_schedule(k, p.w, p.z) && have_samples && cur >= 0 && t->bases[cur].m > 0;
    if (hybrid) {
      hs_htape* h = nullptr;
      HS_TRY(hs_htape_create(ctx, &h));
      const hs_tape::Basis& b = t->bases[cur];
      const hs_status st = rom_hybrid_step_taped(ctx, prev, b.Phi, b.psi, b.m, t->samples, &p.hybrid, out, t->eps,
                                                 nullptr, h, HS_TAPE_RECORD);
      if (st == HS_OK) {
        t->ht[k] = h;
        t->bver[k] = cur;
      } else {
        hs_htape_destroy(h);
        if (st != HS_ERR_NOT_CONVERGED && st != HS_ERR_RANK) return st;
        hybrid = false;    // redone as a full step
      }
    }
    if (!hybrid) HS_TRY(hdm_step(ctx, prev, out, nullptr));
    t->kind[k] = hybrid ? 1 : 0;
    if (k % p.checkpoint_every == 0 || k == p.steps) {
      double* c = nullptr;
      HS_TRY(dalloc(ctx, (void**)&c, (size_t)n * 8));
      t->ckpt[k] = c;
      HS_TRY(dcopy(ctx, c, out, n));
    }
    have_samples = false;
    if (wants_update(k, p.w, p.z, p.steps)) {
      const bool sample = k >= p.w && cur >= 0 && t->bases[cur].m > 0;
      if (sample && !hybrid) {
        const hs_tape::Basis& b = t->bases[cur];
        HS_TRY(hs_indicator_full(ctx, out, b.Phi, b.psi, b.m, p.hybrid.floor_rel, HS_FP64, t->eps, nullptr));
      }
      // the new basis from the window gamma_{k-w} .. gamma_k (gamma_0 .. gamma_{w-1} at k = w - 1)
      const int lo = k >= p.w ? k - p.w : 0;
      std::vector<const double*> win;
      for (int j = lo; j <= k; ++j) win.push_back(slot(j));
      hs_tape::Basis nb;
      nb.k_update = k;
      HS_TRY(dalloc(ctx, (void**)&nb.Phi, (size_t)n * p.m * 8));
      HS_TRY(dalloc(ctx, (void**)&nb.psi, (size_t)n * 8));
      t->bases.push_back(nb);
      hs_tape::Basis& b = t->bases.back();
      HS_TRY(basis_update(ctx, win.data(), (int)win.size(), p.w, p.m, p.tau_pod, HS_FP64, b.Phi, b.psi, t->sigma,
                          &b.m));
      cur = (int)t->bases.size() - 1;
      if (sample) {
        HS_TRY(sample_select(ctx, t->eps, &p.sample, t->samples));
        int32_t cnt[3];
        HS_TRY(hs_samples_counts(t->samples, cnt));
        have_samples = cnt[1] > 0;
      }
    }
  }
  HS_TRY(dcopy(ctx, qT, slot(p.steps), n));
  t->recorded = true;
  return hs_sync(ctx);
}

hs_status hs_traj_backward(hs_ctx* ctx, hs_tape* t, const double* lam_T, double* lam_0) {
  if (!ctx || !t || !lam_T || !lam_0 || t->ctx != ctx) return HS_ERR_INVALID_ARG;
  if (!t->recorded) return ctx->fail(HS_ERR_INVALID_ARG, "hs_traj_backward: the tape holds no forward run");
  const hs_traj_params& p = t->p;
  const long long n = ctx->n;
  const int K = p.checkpoint_every;
  while ((int)t->seg.size() < K + 1) {
    double* s = nullptr;
    HS_TRY(dalloc(ctx, (void**)&s, (size_t)n * 8));
    t->seg.push_back(s);
  }
  for (double*& l : t->lam)
    if (!l) HS_TRY(dalloc(ctx, (void**)&l, (size_t)n * 8));
  double* lam = t->lam[0];
  double* lam2 = t->lam[1];
  HS_TRY(dcopy(ctx, lam, lam_T, n));
  // through psi: a hybrid step's psi adjoint is held, divided by w, for each
  // snapshot its psi averages, and added to that snapshot's adjoint when the
  // backward pass reaches it (snapshot index -> accumulated contribution)
  const bool through_psi = p.psi_adjoint != 0;
  std::map<int, double*> pending;
  if (through_psi && !t->lam_psi) HS_TRY(dalloc(ctx, (void**)&t->lam_psi, (size_t)n * 8));
  auto take = [&](double** out) -> hs_status {
    if (!t->pool.empty()) {
      *out = t->pool.back();
      t->pool.pop_back();
      return HS_OK;
    }
    return dalloc(ctx, (void**)out, (size_t)n * 8);
  };
  auto settle = [&](int j) -> hs_status {   // adds the contributions to gamma_j into lam
    auto it = pending.find(j);
    if (it == pending.end()) return HS_OK;
    HS_LAUNCH(ctx, axpy_kernel, blocks_for(n, kBlock, 1024), kBlock, n, (const double*)it->second, lam);
    t->pool.push_back(it->second);
    pending.erase(it);
    return HS_OK;
  };
  const int last0 = ((p.steps - 1) / K) * K;
  for (int s0 = last0; s0 >= 0; s0 -= K) {
    const int s1 = std::min(s0 + K, p.steps);
    // replay the segment from its checkpoint (the tapes keep each hybrid
    // step's internal states for its adjoint)
    const double* q = t->ckpt.at(s0);
    for (int k = s0 + 1; k <= s1; ++k) {
      double* out = t->seg[k - s0];
      if (t->kind[k] == 0) {
        HS_TRY(hdm_step(ctx, q, out, nullptr));
      } else {
        const hs_tape::Basis& b = t->bases[t->bver[k]];
        HS_TRY(rom_hybrid_step_taped(ctx, q, b.Phi, b.psi, b.m, nullptr, &p.hybrid, out, nullptr, nullptr, t->ht[k],
                                     HS_TAPE_REPLAY));
      }
      q = out;
    }
    HS_LAUNCH(ctx, zero_int_kernel, 1, 1, t->flag);
    HS_LAUNCH(ctx, differ_kernel, blocks_for(n, kBlock, 1024), kBlock, q, t->ckpt.at(s1), n, t->flag);
    int differ = 0;
    HS_TRY(readback(ctx, t->flag, sizeof(int), &differ));
    if (differ)
      return ctx->fail(HS_ERR_INVALID_ARG, "hs_traj_backward: a segment replay did not reproduce its checkpoint "
                                           "(inputs or basis changed since hs_traj_forward)");
    // the step adjoints in reverse order
    for (int k = s1; k > s0; --k) {
      if (through_psi) HS_TRY(settle(k));
      if (t->kind[k] == 0) {
        HS_TRY(hdm_step_adjoint(ctx, t->seg[k - s0], lam, lam2, nullptr));
      } else {
        const hs_tape::Basis& b = t->bases[t->bver[k]];
        if (!through_psi) {
          HS_TRY(rom_hybrid_step_adjoint(ctx, b.Phi, b.m, t->ht[k], lam, lam2, nullptr));
        } else {
          HS_TRY(rom_hybrid_step_adjoint_psi(ctx, b.Phi, b.m, t->ht[k], lam, lam2, t->lam_psi, nullptr));
          for (int j = b.k_update - p.w + 1; j <= b.k_update; ++j) {
            auto it = pending.find(j);
            if (it == pending.end()) {
              double* buf = nullptr;
              HS_TRY(take(&buf));
              HS_LAUNCH(ctx, share_kernel, blocks_for(n, kBlock, 1024), kBlock, n, (const double*)t->lam_psi,
                        (double)p.w, buf, 0);
              pending[j] = buf;
            } else {
              HS_LAUNCH(ctx, share_kernel, blocks_for(n, kBlock, 1024), kBlock, n, (const double*)t->lam_psi,
                        (double)p.w, it->second, 1);
            }
          }
        }
      }
      std::swap(lam, lam2);
    }
  }
  if (through_psi) {
    HS_TRY(settle(0));
    if (!pending.empty()) return ctx->fail(HS_ERR_INVALID_ARG, "hs_traj_backward: a psi contribution was not settled");
  }
  HS_TRY(dcopy(ctx, lam_0, lam, n));
  return hs_sync(ctx);
}

hs_status hs_tape_step(const hs_tape* t, int32_t k, int32_t* kind, int32_t* basis, hs_htape** htape) {
  if (!t || !t->recorded || k < 1 || k > t->p.steps) return HS_ERR_INVALID_ARG;
  if (kind) *kind = t->kind[k];
  if (basis) *basis = t->bver[k];
  if (htape) *htape = t->ht[k];
  return HS_OK;
}

hs_status hs_tape_basis(hs_ctx* ctx, const hs_tape* t, int32_t version, double* Phi_out, double* psi_out,
                        int32_t* m) {
  if (!ctx || !t || !t->recorded || version < 0 || version >= (int)t->bases.size()) return HS_ERR_INVALID_ARG;
  const hs_tape::Basis& b = t->bases[version];
  if (m) *m = b.m;
  if (Phi_out && b.m > 0) HS_TRY(dcopy(ctx, Phi_out, b.Phi, (long long)ctx->n * b.m));
  if (psi_out) HS_TRY(dcopy(ctx, psi_out, b.psi, ctx->n));
  return hs_sync(ctx);
}

hs_status hs_tape_checkpoint(hs_ctx* ctx, const hs_tape* t, int32_t k, double* q_out) {
  if (!ctx || !t || !t->recorded || !q_out) return HS_ERR_INVALID_ARG;
  auto it = t->ckpt.find(k);
  if (it == t->ckpt.end()) return HS_ERR_INVALID_ARG;
  HS_TRY(dcopy(ctx, q_out, it->second, ctx->n));
  return hs_sync(ctx);
}

}  // extern "C"
