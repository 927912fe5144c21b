// BF16 GEMM tile configuration REG_128x128_W2x2 (128 x 128 tile, register-staged loader, 4 waves of 64x64),
// instantiated for BF16 and e4m3 weights.  One translation unit per
// configuration so the build compiles them in parallel.
#include "gemm_kernels.hpp"

namespace vl {

hipError_t gemm_launch_cfg6(const bf16_t* A, int lda, const void* B, int ldb, bool b_fp8,
                               int M, int N, int K, int op, const EpiArgs& e, hipStream_t s) {
  if (b_fp8) return launch_bf16<128, 128, 2, 2, true>(A, lda, B, ldb, M, N, K, op, e, s);
  return launch_bf16<128, 128, 2, 2, false>(A, lda, B, ldb, M, N, K, op, e, s);
}

}  // namespace vl
