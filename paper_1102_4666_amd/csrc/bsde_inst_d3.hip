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

hipError_t launch_batch_d3(int eta, bool fp32, bool bump, int blocks,
                            hipStream_t s, const BatchTileDesc *probs,
                            int nprob, const long long *tile_begin,
                            unsigned int *counter)
{
    BSDE_BATCH_CASE(3, 2)
    BSDE_BATCH_CASE(3, 3)
    BSDE_BATCH_CASE(3, 4)
    return hipErrorInvalidValue;
}

// blocks of the batched kernel resident per CU
int batch_occupancy_d3(int eta, bool fp32, bool bump)
{
    int nb = 0;
#define OCC(E, R, V)                                                           \
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(                        \
        &nb, batch_path_kernel<3, E, R, V>, kBlock, 0)
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
#undef OCC
    return nb;
}

} // namespace bsde
