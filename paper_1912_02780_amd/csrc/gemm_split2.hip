// bf16-plane instantiations of the MFMA contraction kernel, 2 planes per operand.
#include "gemm_split.hpp"

namespace dtrg {

void launch_gemm_split2(const KArgs& a, dim3 grid, int out, int tile, int tag, hipStream_t s) {
    if (out == 0) launch_split_tag<2, 0>(a, grid, tile, tag, s);
    else if (out == 1) launch_split_tag<2, 1>(a, grid, tile, tag, s);
    else launch_split_tag<2, 2>(a, grid, tile, tag, s);
}

}  // namespace dtrg
