// The persistent ragged kernel with ABFT mode 1.
#include "tfft_ragged_kernel.hpp"

namespace tfft {

RaggedKernel ragged_kernel_ft1() { return make_ragged_kernel<1>(); }

}  // namespace tfft
