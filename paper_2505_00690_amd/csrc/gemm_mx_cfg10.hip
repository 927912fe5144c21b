// MXFP8 GEMM tile configuration MX_192x256_W2x4 (192 x 256 tile, 2 x 4 waves).
// One translation unit per configuration so the build compiles them in
// parallel.
#include "gemm_mx.hpp"

namespace vl {

hipError_t gemm_mx_launch_cfg10(const uint8_t* A, const uint8_t* SA, const uint8_t* B,
                               const uint8_t* SB, int M, int N, int K, int op, const EpiArgs& e,
                               hipStream_t s) {
  return launch_mx<192, 256, 2, 4>(A, SA, B, SB, M, N, K, op, e, s);
}

}  // namespace vl
