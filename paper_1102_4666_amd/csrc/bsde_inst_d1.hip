// bsde_inst_d1.hip -- path kernels for d = 1: eta in {2, 3, 4, 5, 6, 8},
// FP32 and FP64 paths; the Dupire-type volatility at eta = 4.
// Also the path kernels of the kernel operator of Section 3.2.
#include "bsde_path.h"

namespace bsde {
#define SETS_D1(X)                                                             \
    X(2, 10, kPrecBoth, false) X(3, 10, kPrecBoth, false)                      \
    X(4, 10, kPrecBoth, true) X(5, 10, kPrecBoth, false)                       \
    X(6, 10, kPrecBoth, false) X(8, 10, kPrecBoth, false)
BSDE_DEFINE_DIMENSION(1, SETS_D1)
BSDE_DEFINE_KERNEL_OP(1)
} // namespace bsde
