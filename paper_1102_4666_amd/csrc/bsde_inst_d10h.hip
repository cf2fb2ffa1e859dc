// bsde_inst_d10h.hip -- path kernels for d = 10 on the hyperbolic index
// sets of eq. hyper_set (Section 4.2) with eta = 5: q = 0.5 (p = 111),
// q = 0.6 (p = 221, the paper's d = 10 runs) and q = 0.7 (p = 386).  FP32
// paths only.  A translation unit of its own so that it compiles beside
// the total-degree d = 10 kernels.
#include "bsde_path.h"

namespace bsde {
#define SETS_D10H(X) X(5, 5, false, false) X(5, 6, false, false) X(5, 7, false, false)
BSDE_DEFINE_DIMENSION_NAMED(10, 10h, SETS_D10H)
} // namespace bsde
