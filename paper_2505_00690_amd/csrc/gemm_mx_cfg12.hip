// MXFP8 GEMM tile configuration MX_128x128_W2x2 (128 x 128 tile, 2 x 2 waves).
// One translation unit per configuration so the build compiles them in
// parallel.
#include "gemm_mx.hpp"

namespace vl {

hipError_t gemm_mx_launch_cfg12(const uint8_t* A, const uint8_t* SA, const uint8_t* B,
                               const uint8_t* SB, int M, int N, int K, int op, const EpiArgs& e,
                               hipStream_t s) {
  return launch_mx<128, 128, 2, 2>(A, SA, B, SB, M, N, K, op, e, s);
}

}  // namespace vl
