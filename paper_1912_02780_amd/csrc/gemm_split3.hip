// bf16-plane instantiations of the MFMA contraction kernel, 3 planes per operand.
#include "gemm_split.hpp"

namespace dtrg {

void launch_gemm_split2(const KArgs& a, dim3 grid, int out, int tile, int tag, bool akm, bool bkm, hipStream_t s);

void launch_gemm_split(const KArgs& a, dim3 grid, int np, int out, int tile, int tag, bool akm, bool bkm,
                       hipStream_t s) {
    DTRG_REQUIRE(np == 2 || np == 3, DTRG_EINVAL, "split contraction: 2 or 3 planes");
    if (np == 2) launch_gemm_split2(a, grid, out, tile, tag, akm, bkm, s);
    else launch_split_np<3>(a, grid, out, tile, tag, akm, bkm, s);
}

}  // namespace dtrg
