// MXFP8 GEMM tile configuration MX_160x256_W1x8 (160 x 256 tile, 1 x 8 waves).
// One translation unit per configuration so the build compiles them in
// parallel.
#include "gemm_mx.hpp"

namespace vl {

hipError_t gemm_mx_launch_cfg9(const uint8_t* A, const uint8_t* SA, const uint8_t* B,
                               const uint8_t* SB, int M, int N, int K, int op, const EpiArgs& e,
                               hipStream_t s) {
  return launch_mx<160, 256, 1, 8>(A, SA, B, SB, M, N, K, op, e, s);
}

}  // namespace vl
