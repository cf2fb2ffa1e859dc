// bsde_inst_d10.hip -- path kernels for d = 10 (eta in {2, 3}), FP32 paths only.
#include "bsde_path.h"

namespace bsde {

hipError_t launch_path_d10(int eta, bool fp32, int blocks, hipStream_t s,
                           const PathParams &prm, const double *pts,
                           const void *gamma, double *partial)
{
    BSDE_PATH_CASE_FP32(10, 2)
    BSDE_PATH_CASE_FP32(10, 3)
    return hipErrorInvalidValue;
}

// multi-indices of the kernels' basis, in the kernels' order
int index_table_d10(int eta, int8_t *nu, int cap)
{
    if (eta == 2) {
        constexpr auto &t = Basis<11, 2>::tab;
        constexpr int P = Basis<11, 2>::P;
        if (nu && cap >= P)
            for (int l = 0; l < P; ++l)
                for (int v = 0; v < 11; ++v) nu[l * 11 + v] = t.nu[l][v];
        return P;
    }
    if (eta == 3) {
        constexpr auto &t = Basis<11, 3>::tab;
        constexpr int P = Basis<11, 3>::P;
        if (nu && cap >= P)
            for (int l = 0; l < P; ++l)
                for (int v = 0; v < 11; ++v) nu[l * 11 + v] = t.nu[l][v];
        return P;
    }
    return 0;
}

hipError_t launch_batch_d10(int eta, bool fp32, bool bump, int blocks,
                            hipStream_t s, const BatchTileDesc *probs,
                            int nprob, const long long *tile_begin,
                            unsigned int *counter)
{
    BSDE_BATCH_CASE_FP32(10, 2)
    BSDE_BATCH_CASE_FP32(10, 3)
    return hipErrorInvalidValue;
}

// blocks of the batched kernel resident per CU
int batch_occupancy_d10(int eta, bool fp32, bool bump)
{
    int nb = 0;
#define OCC(E, R, V)                                                           \
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(                        \
        &nb, batch_path_kernel<10, E, R, V>, kBlock, 0)
    if (eta == 2) {
        if (bump) OCC(2, float, kVolBump);
        else OCC(2, float, kVolConst);
    }
    if (eta == 3) {
        if (bump) OCC(3, float, kVolBump);
        else OCC(3, float, kVolConst);
    }
#undef OCC
    return nb;
}

} // namespace bsde
