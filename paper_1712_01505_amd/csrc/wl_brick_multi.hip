// wl_brick_multi.hip -- the brick walk with several right-hand sides per
// workgroup (wl_brick.h, MULTI = 1), instantiated here for every storage
// precision, apart from the one-right-hand-side kernels.
#include "wl_brick.h"

namespace wl {

template <int P, int DAG>
static hipError_t brick_multi_d(const StencilParams &p, const BrickGeom &g, dim3 grid, dim3 block, size_t smem,
                                hipStream_t st)
{
    if (!p.apply) {
        if (p.red != RED_NONE)
            return hipErrorInvalidValue;
        return brick_go1<P, DAG, RED_NONE, 0, 1>(grid, block, smem, p, g, st);
    }
    if (p.apply == 3) {  // the residual aux - D in (FP64 / FP32)
        if constexpr (P == F64 || P == F32) {
            if (p.red == RED_NONE)
                return brick_go1<P, DAG, RED_NONE, 3, 1>(grid, block, smem, p, g, st);
            if (p.red == RED_NORM)
                return brick_go1<P, DAG, RED_NORM, 3, 1>(grid, block, smem, p, g, st);
        }
        return hipErrorInvalidValue;
    }
    if (p.apply != 1)
        return hipErrorInvalidValue;
    switch (p.red) {
    case RED_NONE: return brick_go1<P, DAG, RED_NONE, 1, 1>(grid, block, smem, p, g, st);
    case RED_NORM: return brick_go1<P, DAG, RED_NORM, 1, 1>(grid, block, smem, p, g, st);
    case RED_DOTV: return brick_go1<P, DAG, RED_DOTV, 1, 1>(grid, block, smem, p, g, st);
    case RED_DOTIN_NORM: return brick_go1<P, DAG, RED_DOTIN_NORM, 1, 1>(grid, block, smem, p, g, st);
    case RED_BICG: return brick_go1<P, DAG, RED_BICG, 1, 1>(grid, block, smem, p, g, st);
    case RED_SR: return brick_go1<P, DAG, RED_SR, 1, 1>(grid, block, smem, p, g, st);
    default: return hipErrorInvalidValue;
    }
}

template <int P>
hipError_t brick_multi_dispatch(int dagger, const StencilParams &p, const BrickGeom &g, dim3 grid, dim3 block,
                                size_t smem, hipStream_t st)
{
    return dagger ? brick_multi_d<P, 1>(p, g, grid, block, smem, st) : brick_multi_d<P, 0>(p, g, grid, block, smem, st);
}

template hipError_t brick_multi_dispatch<F64>(int, const StencilParams &, const BrickGeom &, dim3, dim3, size_t,
                                              hipStream_t);
template hipError_t brick_multi_dispatch<F32>(int, const StencilParams &, const BrickGeom &, dim3, dim3, size_t,
                                              hipStream_t);
template hipError_t brick_multi_dispatch<BF16S>(int, const StencilParams &, const BrickGeom &, dim3, dim3, size_t,
                                                hipStream_t);
template hipError_t brick_multi_dispatch<F16S>(int, const StencilParams &, const BrickGeom &, dim3, dim3, size_t,
                                               hipStream_t);

}  // namespace wl
