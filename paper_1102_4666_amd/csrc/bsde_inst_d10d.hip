// bsde_inst_d10d.hip -- path kernels for d = 10 with FP64 paths: total
// degree eta in {2, 3}, constant and bump volatility.  A translation unit of
// its own so that it compiles beside the FP32 ones (bsde_inst_d10.hip).
#include "bsde_path.h"

namespace bsde {
#define SETS_D10D(X) X(2, 10, kPrecF64, false) X(3, 10, kPrecF64, false)
BSDE_DEFINE_DIMENSION_NAMED(10, 10d, SETS_D10D)
} // namespace bsde
