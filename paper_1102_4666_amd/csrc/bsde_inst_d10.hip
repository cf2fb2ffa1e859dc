// bsde_inst_d10.hip -- path kernels for d = 10: eta in {2, 3}, FP32 paths
// only (the FP64 form does not fit the register file).
#include "bsde_path.h"

namespace bsde {
#define SETS_D10(X) X(2, false, false) X(3, false, false)
BSDE_DEFINE_DIMENSION(10, SETS_D10)
} // namespace bsde
