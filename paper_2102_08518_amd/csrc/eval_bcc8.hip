// Kernels of the bcc8 spline (see lsp_dispatch.h).
#include "lsp_dispatch.h"

namespace lsp {
hipError_t launch_eval_bcc8(const EvalArgs& a) { return launch_kind<kBcc8>(a); }
}  // namespace lsp
