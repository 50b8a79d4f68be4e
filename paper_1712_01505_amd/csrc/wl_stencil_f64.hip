// wl_stencil_f64.hip -- the stencil and multi-lattice kernels instantiated
// for f64 storage (one translation unit per precision keeps the build parallel).
#include "wl_stencil_kern.h"

namespace wl {
template hipError_t launch_stencil_p<F64>(int, const LaunchCfg &, const StencilParams &, hipStream_t);
template const void *multi_kernel_p<F64>(int, int, int, bool);
}  // namespace wl
