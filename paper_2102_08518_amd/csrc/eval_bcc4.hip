// Kernels of the bcc4 spline (see lsp_dispatch.h).
#include "lsp_dispatch.h"

namespace lsp {
template hipError_t launch_eval<kBcc4>(const EvalArgs& a);
}  // namespace lsp
