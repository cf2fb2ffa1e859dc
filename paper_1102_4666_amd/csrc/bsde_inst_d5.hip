// bsde_inst_d5.hip -- path kernels for d = 5: eta in {2, 3}, FP32 and FP64
// paths, all volatility kinds (the Dupire-type one for the paper's d = 5
// runs of Section 6).
#include "bsde_path.h"

namespace bsde {
#define SETS_D5(X) X(2, 10, kPrecBoth, true) X(3, 10, kPrecBoth, true)
BSDE_DEFINE_DIMENSION(5, SETS_D5)
} // namespace bsde
