// Instantiation of the line kernel's forward step variants (both precisions).
#include "line_kernel.h"

namespace mr {
namespace line {
template hipError_t launch_line<double, FWD>(mr_ctx*, LineArgs<double>, hipStream_t);
template hipError_t launch_line<float, FWD>(mr_ctx*, LineArgs<float>, hipStream_t);
}  // namespace line
}  // namespace mr
