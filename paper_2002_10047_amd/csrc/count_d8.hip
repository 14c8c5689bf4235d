// Counting kernels whose bitmap recursion goes at most 8 level(s) below a pair node.
#include "count_kernels.h"

namespace arb {
ARB_COUNT_DEPTH_UNIT(8)
}  // namespace arb
