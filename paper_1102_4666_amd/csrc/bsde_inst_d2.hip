// bsde_inst_d2.hip -- path kernels for d = 2: eta in {2, 3, 4, 5}, FP32 and
// FP64 paths; the Dupire-type volatility at eta = 3.
// Also the path kernels of the kernel operator of Section 3.2.
#include "bsde_path.h"

namespace bsde {
#define SETS_D2(X)                                                             \
    X(2, 10, kPrecBoth, false) X(3, 10, kPrecBoth, true)                       \
    X(4, 10, kPrecBoth, false) X(5, 10, kPrecBoth, false)
BSDE_DEFINE_DIMENSION(2, SETS_D2)
BSDE_DEFINE_KERNEL_OP(2)
} // namespace bsde
