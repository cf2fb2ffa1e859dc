// bsde_inst_d10q6.hip -- path kernels for d = 10 on the hyperbolic index set
// of eq. hyper_set (Section 4.2) with q = 0.6: eta = 5 (p = 221, the
// paper's d = 10 runs) and eta = 4 (p = 100, the sparser set the paper's
// d = 10 study sets beside it).  FP32 paths only.  Each hyperbolic set is a
// translation unit of its own so that the sets compile side by side.
#include "bsde_path.h"

namespace bsde {
#define SETS_D10Q6(X) X(4, 6, kPrecF32, false) X(5, 6, kPrecF32, false)
BSDE_DEFINE_DIMENSION_NAMED(10, 10q6, SETS_D10Q6)
} // namespace bsde
