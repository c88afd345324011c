// Split-bf16 (three products) instantiations of the MFMA contraction kernel.
#include "gemm_kernels.hpp"

namespace dtrg {

void launch_gemm_bf16x3(const KArgs& a, dim3 grid, bool akm, bool bkm, int tag, bool big, bool out_f64,
                        hipStream_t s) {
    if (out_f64) {
        if (big) launch_bf16x3<double, 128, 128>(a, grid, akm, bkm, tag, s);
        else launch_bf16x3<double, 64, 64>(a, grid, akm, bkm, 0, s);
    } else {
        if (big) launch_bf16x3<float, 128, 128>(a, grid, akm, bkm, tag, s);
        else launch_bf16x3<float, 64, 64>(a, grid, akm, bkm, 0, s);
    }
}

}  // namespace dtrg
