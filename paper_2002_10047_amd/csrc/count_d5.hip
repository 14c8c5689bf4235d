// Counting kernels whose bitmap recursion goes at most 5 level(s) below a pair node.
#include "count_kernels.h"

namespace arb {
ARB_COUNT_DEPTH_UNIT(5)
}  // namespace arb
