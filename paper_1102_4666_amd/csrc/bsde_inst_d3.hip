// bsde_inst_d3.hip -- path kernels for d = 3: eta in {2, 3, 4}, FP32 and
// FP64 paths.
#include "bsde_path.h"

namespace bsde {
#define SETS_D3(X)                                                             \
    X(2, 10, kPrecBoth, false) X(3, 10, kPrecBoth, false)                      \
    X(4, 10, kPrecBoth, false)
BSDE_DEFINE_DIMENSION(3, SETS_D3)
} // namespace bsde
