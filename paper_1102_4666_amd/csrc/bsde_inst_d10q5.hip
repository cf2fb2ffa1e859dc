// bsde_inst_d10q5.hip -- path kernels for d = 10 on the hyperbolic index set
// of eq. hyper_set (Section 4.2) with eta = 5, q = 0.5 (p = 111).  FP32
// paths only.  Each hyperbolic set is a translation unit of its own so
// that the sets compile side by side.
#include "bsde_path.h"

namespace bsde {
#define SETS_D10Q5(X) X(5, 5, kPrecF32, false)
BSDE_DEFINE_DIMENSION_NAMED(10, 10q5, SETS_D10Q5)
} // namespace bsde
