// bsde_inst_d10q7.hip -- path kernels for d = 10 on the hyperbolic index set
// of eq. hyper_set (Section 4.2) with eta = 5, q = 0.7 (p = 386).  FP32
// paths only.  Each hyperbolic set is a translation unit of its own so
// that the sets compile side by side.
#include "bsde_path.h"

namespace bsde {
#define SETS_D10Q7(X) X(5, 7, kPrecF32, false)
BSDE_DEFINE_DIMENSION_NAMED(10, 10q7, SETS_D10Q7)
} // namespace bsde
