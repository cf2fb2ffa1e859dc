// bsde_inst_d1.hip -- path kernels for d = 1 (eta in {2, 3, 4, 5, 6, 8}).
#include "bsde_path.h"

namespace bsde {

hipError_t launch_path_d1(int eta, bool fp32, int blocks, hipStream_t s,
                           const PathParams &prm, const double *pts,
                           const void *gamma, double *partial)
{
    BSDE_PATH_CASE(1, 2)
    BSDE_PATH_CASE(1, 3)
    BSDE_PATH_CASE(1, 4)
    BSDE_PATH_CASE(1, 5)
    BSDE_PATH_CASE(1, 6)
    BSDE_PATH_CASE(1, 8)
    return hipErrorInvalidValue;
}

// multi-indices of the kernels' basis, in the kernels' order
int index_table_d1(int eta, int8_t *nu, int cap)
{
    if (eta == 2) {
        constexpr auto &t = Basis<2, 2>::tab;
        constexpr int P = Basis<2, 2>::P;
        if (nu && cap >= P)
            for (int l = 0; l < P; ++l)
                for (int v = 0; v < 2; ++v) nu[l * 2 + v] = t.nu[l][v];
        return P;
    }
    if (eta == 3) {
        constexpr auto &t = Basis<2, 3>::tab;
        constexpr int P = Basis<2, 3>::P;
        if (nu && cap >= P)
            for (int l = 0; l < P; ++l)
                for (int v = 0; v < 2; ++v) nu[l * 2 + v] = t.nu[l][v];
        return P;
    }
    if (eta == 4) {
        constexpr auto &t = Basis<2, 4>::tab;
        constexpr int P = Basis<2, 4>::P;
        if (nu && cap >= P)
            for (int l = 0; l < P; ++l)
                for (int v = 0; v < 2; ++v) nu[l * 2 + v] = t.nu[l][v];
        return P;
    }
    if (eta == 5) {
        constexpr auto &t = Basis<2, 5>::tab;
        constexpr int P = Basis<2, 5>::P;
        if (nu && cap >= P)
            for (int l = 0; l < P; ++l)
                for (int v = 0; v < 2; ++v) nu[l * 2 + v] = t.nu[l][v];
        return P;
    }
    if (eta == 6) {
        constexpr auto &t = Basis<2, 6>::tab;
        constexpr int P = Basis<2, 6>::P;
        if (nu && cap >= P)
            for (int l = 0; l < P; ++l)
                for (int v = 0; v < 2; ++v) nu[l * 2 + v] = t.nu[l][v];
        return P;
    }
    if (eta == 8) {
        constexpr auto &t = Basis<2, 8>::tab;
        constexpr int P = Basis<2, 8>::P;
        if (nu && cap >= P)
            for (int l = 0; l < P; ++l)
                for (int v = 0; v < 2; ++v) nu[l * 2 + v] = t.nu[l][v];
        return P;
    }
    return 0;
}

} // namespace bsde
