// wl_stencil_bf16.hip -- the stencil and multi-lattice kernels instantiated
// for bf16 storage (one translation unit per precision keeps the build parallel).
#include "wl_stencil_kern.h"

namespace wl {
template hipError_t launch_stencil_p<BF16S>(int, const LaunchCfg &, const StencilParams &, hipStream_t);
template const void *multi_kernel_p<BF16S>(int, int, int, bool);
}  // namespace wl
