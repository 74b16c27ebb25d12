// Declarations of reduce.hip: fixed-order FP64 reductions and the streaming copy.
#pragma once

#include "laph_host.h"

namespace laph {

// block partials of the mass-gradient dot product (the scratch holds
// kGradBlocks partials and one result)
constexpr int kGradBlocks = 2048;
constexpr size_t kGradScratchDoubles = kGradBlocks + 1;

// out[r * 3 + q] = sum of the nsb stage partials of RHS r and quantity q < nq
laph_status sum_stage_partials(const Ctx &c, const double *partials, int pstride, int nsb, int nrhs, int nq,
                               double *out);
// *g_host = -sum Re(conj(Z_i) X_i) over n_complex elements (synchronises the stream)
laph_status mass_gradient(const Ctx &c, double *g_host, const double *Z, const double *X, size_t n_complex,
                          double *scratch);
// dst = src (bytes a multiple of 16) reps times after one warm copy; average ms per copy
laph_status stream_copy(const Ctx &c, void *dst, const void *src, size_t bytes, int reps, double *ms_host);

}  // namespace laph
