// MXFP8 GEMM tile configuration MX_128x256_W2x4 (128 x 256 tile, 2 x 4 waves).
// One translation unit per configuration so the build compiles them in
// parallel.
#include "gemm_mx.hpp"

namespace vl {

hipError_t gemm_mx_launch_cfg11(const uint8_t* A, const uint8_t* SA, const uint8_t* B,
                               const uint8_t* SB, int M, int N, int K, int op, const EpiArgs& e,
                               hipStream_t s) {
  return launch_mx<128, 256, 2, 4>(A, SA, B, SB, M, N, K, op, e, s);
}

}  // namespace vl
