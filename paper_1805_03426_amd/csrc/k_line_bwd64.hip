// Instantiation of the line kernel's reverse-step variants (FP64).
#include "line_kernel.h"

namespace mr {
namespace line {
template hipError_t launch_line<double, BWD>(mr_ctx*, LineArgs<double>, hipStream_t);
}  // namespace line
}  // namespace mr
