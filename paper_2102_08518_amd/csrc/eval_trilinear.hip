// Kernels of the trilinear spline (see lsp_dispatch.h).
#include "lsp_dispatch.h"

namespace lsp {
template hipError_t launch_eval<kTrilinear>(const EvalArgs& a);
}  // namespace lsp
