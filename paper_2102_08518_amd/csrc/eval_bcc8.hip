// Kernels of the bcc8 spline (see lsp_dispatch.h).
#include "lsp_dispatch.h"

namespace lsp {
template hipError_t launch_eval<kBcc8>(const EvalArgs& a);
}  // namespace lsp
