// wl_stencil_f16.hip -- the stencil and multi-lattice kernels instantiated
// for f16 storage (one translation unit per precision keeps the build parallel).
#include "wl_stencil_kern.h"

namespace wl {
template hipError_t launch_stencil_p<F16S>(int, const LaunchCfg &, const StencilParams &, hipStream_t);
template const void *multi_kernel_p<F16S>(int, int, int, bool);
}  // namespace wl
