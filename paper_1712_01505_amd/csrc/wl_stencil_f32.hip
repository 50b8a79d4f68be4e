// wl_stencil_f32.hip -- the stencil and multi-lattice kernels instantiated
// for f32 storage (one translation unit per precision keeps the build parallel).
#include "wl_stencil_kern.h"

namespace wl {
template hipError_t launch_stencil_p<F32>(int, const LaunchCfg &, const StencilParams &, hipStream_t);
template const void *multi_kernel_p<F32>(int, int, int, bool);
}  // namespace wl
