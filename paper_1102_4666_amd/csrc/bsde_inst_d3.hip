// bsde_inst_d3.hip -- path kernels for d = 3 (eta in {2, 3, 4}).
#include "bsde_path.h"

namespace bsde {

hipError_t launch_path_d3(int eta, bool fp32, int blocks, hipStream_t s,
                           const PathParams &prm, const double *pts,
                           const void *gamma, double *partial)
{
    BSDE_PATH_CASE(3, 2)
    BSDE_PATH_CASE(3, 3)
    BSDE_PATH_CASE(3, 4)
    return hipErrorInvalidValue;
}

// multi-indices of the kernels' basis, in the kernels' order
int index_table_d3(int eta, int8_t *nu, int cap)
{
    if (eta == 2) {
        constexpr auto &t = Basis<4, 2>::tab;
        constexpr int P = Basis<4, 2>::P;
        if (nu && cap >= P)
            for (int l = 0; l < P; ++l)
                for (int v = 0; v < 4; ++v) nu[l * 4 + v] = t.nu[l][v];
        return P;
    }
    if (eta == 3) {
        constexpr auto &t = Basis<4, 3>::tab;
        constexpr int P = Basis<4, 3>::P;
        if (nu && cap >= P)
            for (int l = 0; l < P; ++l)
                for (int v = 0; v < 4; ++v) nu[l * 4 + v] = t.nu[l][v];
        return P;
    }
    if (eta == 4) {
        constexpr auto &t = Basis<4, 4>::tab;
        constexpr int P = Basis<4, 4>::P;
        if (nu && cap >= P)
            for (int l = 0; l < P; ++l)
                for (int v = 0; v < 4; ++v) nu[l * 4 + v] = t.nu[l][v];
        return P;
    }
    return 0;
}

} // namespace bsde
