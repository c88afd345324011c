// FP32 instantiations of the MFMA contraction kernel.
#include "gemm_kernels.hpp"

namespace dtrg {

void launch_gemm_f32(const KArgs& a, dim3 grid, bool akm, bool bkm, int tag, bool big, bool out_f64, hipStream_t s) {
    if (out_f64) {
        if (big) launch_mfma4<float, double, 128, 128, 16>(a, grid, akm, bkm, tag, s);
        else launch_mfma4<float, double, 64, 64, 16>(a, grid, akm, bkm, 0, s);
    } else {
        if (big) launch_mfma4<float, float, 128, 128, 16>(a, grid, akm, bkm, tag, s);
        else launch_mfma4<float, float, 64, 64, 16>(a, grid, akm, bkm, 0, s);
    }
}

}  // namespace dtrg
