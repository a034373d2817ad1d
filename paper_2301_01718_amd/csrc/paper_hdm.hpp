// The paper's full-order scheme (Sec. 3.1): what the hybrid step shares with
// the full step (paper_hdm.hip).
#pragma once

#include "common.hpp"

namespace hs {

struct PaperBC {
  int kind;              // HS_PAPER_BC_FIXED or HS_PAPER_BC_WALL
  double ghost[4][4];    // FIXED: states outside the left, right, bottom, top boundaries
};

// Checks the call's boundary data against the context (an Euler mesh).
hs_status paper_bc(hs_ctx* ctx, const hs_paper_hdm* hdm, PaperBC* bc);

// Defect correction of the BDF residual (q2 == nullptr: BDF1) for the entries
// of u on the sampled set s (s == nullptr: the whole mesh), every other entry
// of u held, until ||R||_inf <= tol on those cells.  Adds the corrections'
// count and sweeps to info (may be null) and sets info->residual_inf.
hs_status paper_solve(hs_ctx* ctx, const PaperBC& bc, double* u, const double* q1, const double* q2, double tol,
                      const hs_samples* s, hs_step_info* info);

// rcell[cell] = 2-norm over the components of the BDF residual of q; the
// per-block sums of rcell go to the kStatSum partials (*nb blocks).
hs_status paper_cell_norms(hs_ctx* ctx, const PaperBC& bc, const double* q, const double* q1, const double* q2,
                           double* rcell, int* nb);

}  // namespace hs
