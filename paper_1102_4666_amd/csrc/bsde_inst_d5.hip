// bsde_inst_d5.hip -- path kernels for d = 5 (eta in {2, 3}).
#include "bsde_path.h"

namespace bsde {

hipError_t launch_path_d5(int eta, bool fp32, int blocks, hipStream_t s,
                           const PathParams &prm, const double *pts,
                           const void *gamma, double *partial)
{
    BSDE_PATH_CASE(5, 2)
    BSDE_PATH_CASE(5, 3)
    return hipErrorInvalidValue;
}

// multi-indices of the kernels' basis, in the kernels' order
int index_table_d5(int eta, int8_t *nu, int cap)
{
    if (eta == 2) {
        constexpr auto &t = Basis<6, 2>::tab;
        constexpr int P = Basis<6, 2>::P;
        if (nu && cap >= P)
            for (int l = 0; l < P; ++l)
                for (int v = 0; v < 6; ++v) nu[l * 6 + v] = t.nu[l][v];
        return P;
    }
    if (eta == 3) {
        constexpr auto &t = Basis<6, 3>::tab;
        constexpr int P = Basis<6, 3>::P;
        if (nu && cap >= P)
            for (int l = 0; l < P; ++l)
                for (int v = 0; v < 6; ++v) nu[l * 6 + v] = t.nu[l][v];
        return P;
    }
    return 0;
}

} // namespace bsde
