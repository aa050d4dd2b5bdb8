// Kernels of the tricubic spline (see lsp_dispatch.h).
#include "lsp_dispatch.h"

namespace lsp {
hipError_t launch_eval_tricubic(const EvalArgs& a) { return launch_kind<kTricubic>(a); }
}  // namespace lsp
