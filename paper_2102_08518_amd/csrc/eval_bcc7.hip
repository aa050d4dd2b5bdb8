// Kernels of the bcc7 spline (see lsp_dispatch.h).
#include "lsp_dispatch.h"

namespace lsp {
template hipError_t launch_eval<kBcc7>(const EvalArgs& a);
}  // namespace lsp
