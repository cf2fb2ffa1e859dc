// bsde_inst_d2.hip -- path kernels for d = 2 (eta in {2, 3, 4, 5}).
#include "bsde_path.h"

namespace bsde {

hipError_t launch_path_d2(int eta, bool fp32, int blocks, hipStream_t s,
                           const PathParams &prm, const double *pts,
                           const void *gamma, double *partial)
{
    BSDE_PATH_CASE(2, 2)
    BSDE_PATH_CASE(2, 3)
    BSDE_PATH_CASE(2, 4)
    BSDE_PATH_CASE(2, 5)
    return hipErrorInvalidValue;
}

// multi-indices of the kernels' basis, in the kernels' order
int index_table_d2(int eta, int8_t *nu, int cap)
{
    if (eta == 2) {
        constexpr auto &t = Basis<3, 2>::tab;
        constexpr int P = Basis<3, 2>::P;
        if (nu && cap >= P)
            for (int l = 0; l < P; ++l)
                for (int v = 0; v < 3; ++v) nu[l * 3 + v] = t.nu[l][v];
        return P;
    }
    if (eta == 3) {
        constexpr auto &t = Basis<3, 3>::tab;
        constexpr int P = Basis<3, 3>::P;
        if (nu && cap >= P)
            for (int l = 0; l < P; ++l)
                for (int v = 0; v < 3; ++v) nu[l * 3 + v] = t.nu[l][v];
        return P;
    }
    if (eta == 4) {
        constexpr auto &t = Basis<3, 4>::tab;
        constexpr int P = Basis<3, 4>::P;
        if (nu && cap >= P)
            for (int l = 0; l < P; ++l)
                for (int v = 0; v < 3; ++v) nu[l * 3 + v] = t.nu[l][v];
        return P;
    }
    if (eta == 5) {
        constexpr auto &t = Basis<3, 5>::tab;
        constexpr int P = Basis<3, 5>::P;
        if (nu && cap >= P)
            for (int l = 0; l < P; ++l)
                for (int v = 0; v < 3; ++v) nu[l * 3 + v] = t.nu[l][v];
        return P;
    }
    return 0;
}

hipError_t launch_batch_d2(int eta, bool fp32, bool bump, int blocks,
                            hipStream_t s, const BatchTileDesc *probs,
                            int nprob, const long long *tile_begin,
                            unsigned int *counter)
{
    BSDE_BATCH_CASE(2, 2)
    BSDE_BATCH_CASE(2, 3)
    BSDE_BATCH_CASE(2, 4)
    BSDE_BATCH_CASE(2, 5)
    return hipErrorInvalidValue;
}

// blocks of the batched kernel resident per CU
int batch_occupancy_d2(int eta, bool fp32, bool bump)
{
    int nb = 0;
#define OCC(E, R, V)                                                           \
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(                        \
        &nb, batch_path_kernel<2, E, R, V>, kBlock, 0)
    if (eta == 2) {
        if (fp32 && bump) OCC(2, float, kVolBump);
        else if (fp32) OCC(2, float, kVolConst);
        else if (bump) OCC(2, double, kVolBump);
        else OCC(2, double, kVolConst);
    }
    if (eta == 3) {
        if (fp32 && bump) OCC(3, float, kVolBump);
        else if (fp32) OCC(3, float, kVolConst);
        else if (bump) OCC(3, double, kVolBump);
        else OCC(3, double, kVolConst);
    }
    if (eta == 4) {
        if (fp32 && bump) OCC(4, float, kVolBump);
        else if (fp32) OCC(4, float, kVolConst);
        else if (bump) OCC(4, double, kVolBump);
        else OCC(4, double, kVolConst);
    }
    if (eta == 5) {
        if (fp32 && bump) OCC(5, float, kVolBump);
        else if (fp32) OCC(5, float, kVolConst);
        else if (bump) OCC(5, double, kVolBump);
        else OCC(5, double, kVolConst);
    }
#undef OCC
    return nb;
}

} // namespace bsde
