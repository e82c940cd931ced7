// The persistent ragged kernel with ABFT mode 1.
#include "tfft_ragged_kernel.hpp"

namespace tfft {

RaggedKernel ragged_kernel_ft1(int waves) {
    return waves == 3 ? make_ragged_kernel<1, true>() : make_ragged_kernel<1, false>();
}

}  // namespace tfft
