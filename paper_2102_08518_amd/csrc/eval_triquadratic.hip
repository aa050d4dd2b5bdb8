// Kernels of the triquadratic spline (see lsp_dispatch.h).
#include "lsp_dispatch.h"

namespace lsp {
template hipError_t launch_eval<kTriquadratic>(const EvalArgs& a);
}  // namespace lsp
