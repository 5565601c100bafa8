// Instantiation of the line kernel's reverse-step variants (FP32).
#include "line_kernel.h"

namespace mr {
namespace line {
template hipError_t launch_line<float, BWD>(mr_ctx*, LineArgs<float>, hipStream_t);
}  // namespace line
}  // namespace mr
