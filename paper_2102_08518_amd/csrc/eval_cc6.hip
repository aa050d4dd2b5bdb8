// Kernels of the cc6 spline (see lsp_dispatch.h).
#include "lsp_dispatch.h"

namespace lsp {
template hipError_t launch_eval<kCc6>(const EvalArgs& a);
}  // namespace lsp
