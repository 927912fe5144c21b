// BF16 GEMM tile configuration DL_256x256_W4x2 (256 x 256 tile, 8 waves, 64x128 outputs per wave),
// instantiated for BF16 and e4m3 weights.  One translation unit per
// configuration so the build compiles them in parallel.
#include "gemm_kernels.hpp"

namespace vl {

hipError_t gemm_launch_cfg1(const bf16_t* A, int lda, const void* B, int ldb, bool b_fp8,
                               int M, int N, int K, int op, const EpiArgs& e, hipStream_t s) {
  if (b_fp8) return launch_bf16_dl<256, 256, 4, 2, true>(A, lda, B, ldb, M, N, K, op, e, s);
  return launch_bf16_dl<256, 256, 4, 2, false>(A, lda, B, ldb, M, N, K, op, e, s);
}

}  // namespace vl
