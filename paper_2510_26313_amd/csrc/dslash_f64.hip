// F64 instantiations of the even-odd stencil stages (kept in their own
// translation unit so the three precisions compile in parallel).
#include "dslash_lds.h"

namespace laph {
bool launch_stage_f64(const StageSpec &s, const StageArgs &a, hipStream_t st) { return launch_p<F64>(s, a, st); }
bool launch_stage_lds_f64(const StageSpec &s, const StageArgs &a, hipStream_t st) {
    return launch_lds_p<F64>(s, a, st);
}
}  // namespace laph
