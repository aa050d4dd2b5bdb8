// Kernels of the fcc6 spline (see lsp_dispatch.h).
#include "lsp_dispatch.h"

namespace lsp {
hipError_t launch_eval_fcc6(const EvalArgs& a) { return launch_kind<kFcc6>(a); }
}  // namespace lsp
