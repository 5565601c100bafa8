// Instantiation of the line kernel's reverse step at n = 0 variants (both precisions).
#include "line_kernel.h"

namespace mr {
namespace line {
template hipError_t launch_line<double, BWD0>(mr_ctx*, LineArgs<double>, hipStream_t);
template hipError_t launch_line<float, BWD0>(mr_ctx*, LineArgs<float>, hipStream_t);
}  // namespace line
}  // namespace mr
