// Kernels of the tricubic spline (see lsp_dispatch.h).
#include "lsp_dispatch.h"

namespace lsp {
template hipError_t launch_eval<kTricubic>(const EvalArgs& a);
}  // namespace lsp
