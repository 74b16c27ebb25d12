// Declarations of the two-level aggregation multigrid (mg.hip).
#pragma once

#include "laph_host.h"

namespace laph {

constexpr int kMgMaxVec = 16;       // near-null vectors at most (32 coarse components per site)
constexpr int kMgMaxRestart = 16;   // outer GCR directions at most

// Geometry and validity of an aggregate shape for the context's lattice.
laph_status mg_geometry(const Ctx &c, int nvec, const int block[4], MgGeom &g);
// Bytes of the multigrid buffer: basis (nv full FP64 fields) + coarse matrix + flag.
size_t mg_state_bytes(const Ctx &c, const MgGeom &g);
// Workspace of the setup: two canonical copies of the near-null vectors plus the
// batched solver that relaxes them (null_passes > 0).
size_t mg_setup_workspace_bytes(const Ctx &c, const MgGeom &g, int null_passes);
// Setup on the attached buffer: relax V0 (canonical, nv fields) by null_passes
// inverse-iteration solves, block-orthonormalise, build D_c = P^dagger D P.
laph_status mg_setup(Ctx &c, int mass_idx, const MgGeom &g, const double *V0, int null_passes, double null_tol,
                     char *state, size_t state_bytes, char *work, size_t work_bytes);
// Canonical readback of the basis; coarse matrix copy.
laph_status mg_basis_canonical(const Ctx &c, double *out);
// R f / P c on canonical fields (work: n full internal FP64 fields)
laph_status mg_restrict_canonical(const Ctx &c, double *cvec, const double *f, int n, char *work);
laph_status mg_prolong_canonical(const Ctx &c, double *f, const double *cvec, int n, char *work);
laph_status mg_coarse_apply(const Ctx &c, double *out, const double *in, int n);
// Batched solve of D x = b (canonical, full lattice) by GCR preconditioned with one
// multigrid cycle per iteration.
// run: the attached multigrid with the call's cycle parameters (smooth_iters,
// coarse_iters, coarse_tol, restart, maxiter).
size_t mg_solve_workspace_bytes(const Ctx &c, int nrhs, int restart);
laph_status mg_solve(Ctx &c, const MgState &run, double *X, const double *B, int nrhs, double tol,
                     laph_rhs_stats *stats, char *work, size_t work_bytes);

// One building block of the multigrid cycle (tests): what 0: D in FP32; 1: the smoother;
// 2: the cycle; 4: D in FP64 (canonical fields in and out); 3: the coarse solve (coarse
// vectors); 5, 6: the GCR directions Z, W after run.maxiter iterations ([restart][n] fields).
laph_status mg_component(Ctx &c, const MgState &run, int what, double *out, const double *in, int n, char *work,
                         size_t work_bytes);

}  // namespace laph
