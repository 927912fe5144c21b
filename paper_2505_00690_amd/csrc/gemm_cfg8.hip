// BF16 GEMM tile configuration DL3_160x256_W1x8 (160 x 256 tile, 8 waves side by
// side along N, 160x32 outputs per wave; 5/8 of the 256 x 256 tile, for
// N = 1024 products whose 256 x 256 tile count leaves the last round on 256
// CUs mostly idle; small enough for a three-stage LDS ring, i.e. loads two
// K tiles ahead, which matters when the activations come from HBM),
// instantiated for BF16 and e4m3 weights.  One translation unit per
// configuration so the build compiles them in parallel.
#include "gemm_kernels.hpp"

namespace vl {

hipError_t gemm_launch_cfg8(const bf16_t* A, int lda, const void* B, int ldb, bool b_fp8,
                               int M, int N, int K, int op, const EpiArgs& e, hipStream_t s) {
  if (b_fp8) return launch_bf16_dl<160, 256, 1, 8, true, 2, 3>(A, lda, B, ldb, M, N, K, op, e, s);
  return launch_bf16_dl<160, 256, 1, 8, false, 2, 3>(A, lda, B, ldb, M, N, K, op, e, s);
}

}  // namespace vl
