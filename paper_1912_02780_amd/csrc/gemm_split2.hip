// bf16-plane instantiations of the MFMA contraction kernel, 2 planes per operand.
#include "gemm_split.hpp"

namespace dtrg {

void launch_gemm_split2(const KArgs& a, dim3 grid, int out, int tile, int tag, bool akm, bool bkm, hipStream_t s) {
    launch_split_np<2>(a, grid, out, tile, tag, akm, bkm, s);
}

}  // namespace dtrg
