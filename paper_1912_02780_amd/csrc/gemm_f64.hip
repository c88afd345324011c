// FP64 instantiations of the MFMA contraction kernel.
#include "gemm_kernels.hpp"

namespace dtrg {

void launch_gemm_f64(const KArgs& a, dim3 grid, bool akm, bool bkm, int tag, bool big, hipStream_t s) {
    if (big) launch_mfma4<double, double, 128, 128, 16, 4, 2>(a, grid, akm, bkm, tag, s);
    else launch_mfma4<double, double, 64, 64, 16>(a, grid, akm, bkm, 0, s);
}

}  // namespace dtrg
