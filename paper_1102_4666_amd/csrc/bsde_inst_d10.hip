// bsde_inst_d10.hip -- path kernels for d = 10, FP32 paths only (the FP64
// form does not fit the register file): total degree eta in {2, 3}, and the
// hyperbolic set eta = 5, q = 0.6 (p = 221) of the paper's d = 10 runs.
#include "bsde_path.h"

namespace bsde {
#define SETS_D10(X) X(2, 10, false, false) X(3, 10, false, false) X(5, 6, false, false)
BSDE_DEFINE_DIMENSION(10, SETS_D10)
} // namespace bsde
