// Counting kernels for walks of any depth: seven levels below a pair node through the
// nested recursion, deeper ones (k > 10) through the framed walk dfs_deep.
#include "count_kernels.h"

namespace arb {
ARB_COUNT_DEPTH_UNIT(8)
}  // namespace arb
