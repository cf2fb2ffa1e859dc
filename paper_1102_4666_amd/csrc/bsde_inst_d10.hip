// bsde_inst_d10.hip -- path kernels for d = 10, FP32 paths only (the FP64
// form does not fit the register file): total degree eta in {2, 3}.  The
// hyperbolic sets of the paper's d = 10 runs are in bsde_inst_d10h.hip.
#include "bsde_path.h"

namespace bsde {
#define SETS_D10(X) X(2, 10, false, false) X(3, 10, false, false)
BSDE_DEFINE_DIMENSION(10, SETS_D10)
} // namespace bsde
