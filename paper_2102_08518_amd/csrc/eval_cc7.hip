// Kernels of the cc7 spline (see lsp_dispatch.h).
#include "lsp_dispatch.h"

namespace lsp {
template hipError_t launch_eval<kCc7>(const EvalArgs& a);
}  // namespace lsp
