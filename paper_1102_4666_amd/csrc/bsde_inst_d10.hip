// bsde_inst_d10.hip -- path kernels for d = 10 with FP32 paths: total
// degree eta in {2, 3}.  FP64 paths are in bsde_inst_d10d.hip, the
// hyperbolic sets of the paper's d = 10 runs in bsde_inst_d10q5.hip,
// bsde_inst_d10q6.hip and bsde_inst_d10q7.hip.
#include "bsde_path.h"

namespace bsde {
#define SETS_D10(X) X(2, 10, kPrecF32, false) X(3, 10, kPrecF32, false)
BSDE_DEFINE_DIMENSION(10, SETS_D10)
} // namespace bsde
