// Dense contractions C[M,N] = A[M,K] . B[N,K]^T with fused epilogues: the
// configuration table, the tile heuristics and the launchers, plus the FP32
// kernels.
//
// BF16 path (kernels in gemm_kernels.hpp): v_mfma_f32_32x32x16_bf16 on
// gfx950.  A workgroup owns a BM x BN output tile and walks K in steps of 64
// through a ring of two or three LDS stages filled by direct-to-LDS loads
// (buffer_load ... lds, 16 bytes per lane) issued one or two K steps ahead.
// LDS rows are 64 BF16 (128 B) whose eight 16-byte chunks are permuted by
// XOR with (r ^ (r >> 3)) & 7, so the operand reads of an MFMA are free of
// bank conflicts.  Output tiles are dealt XCD by XCD.  The epilogue stages
// each 32-row slab of a wave's tile through LDS and stores rows whole.  All
// configurations accumulate K in the same order, so they agree bitwise; the
// per-configuration instantiations live in gemm_cfg*.hip / gemm_mx_cfg*.hip.
//
// FP32 path: LDS-tiled FMA kernel (64 x 64 tile, 4 x 4 per thread), the plain
// FP32 baseline; and a few-rows FP32 kernel for the heads' small products
// (pooled rows or embeddings against the projection or the texts).
#include "gemm_kernels.hpp"

namespace vl {

// ------------------------------------------------- BF16 GEMM configurations
hipError_t gemm_launch_cfg0(const bf16_t*, int, const void*, int, bool, int, int, int, int,
                               const EpiArgs&, hipStream_t);
hipError_t gemm_launch_cfg1(const bf16_t*, int, const void*, int, bool, int, int, int, int,
                               const EpiArgs&, hipStream_t);
hipError_t gemm_launch_cfg2(const bf16_t*, int, const void*, int, bool, int, int, int, int,
                               const EpiArgs&, hipStream_t);
hipError_t gemm_launch_cfg3(const bf16_t*, int, const void*, int, bool, int, int, int, int,
                               const EpiArgs&, hipStream_t);
hipError_t gemm_launch_cfg4(const bf16_t*, int, const void*, int, bool, int, int, int, int,
                               const EpiArgs&, hipStream_t);
hipError_t gemm_launch_cfg5(const bf16_t*, int, const void*, int, bool, int, int, int, int,
                               const EpiArgs&, hipStream_t);
hipError_t gemm_launch_cfg6(const bf16_t*, int, const void*, int, bool, int, int, int, int,
                               const EpiArgs&, hipStream_t);
hipError_t gemm_launch_cfg7(const bf16_t*, int, const void*, int, bool, int, int, int, int,
                               const EpiArgs&, hipStream_t);
hipError_t gemm_launch_cfg8(const bf16_t*, int, const void*, int, bool, int, int, int, int,
                               const EpiArgs&, hipStream_t);

// ------------------------------------------------ MXFP8 GEMM configurations
hipError_t gemm_mx_launch_cfg9(const uint8_t*, const uint8_t*, const uint8_t*, const uint8_t*,
                               int, int, int, int, const EpiArgs&, hipStream_t);
hipError_t gemm_mx_launch_cfg10(const uint8_t*, const uint8_t*, const uint8_t*, const uint8_t*,
                                int, int, int, int, const EpiArgs&, hipStream_t);
hipError_t gemm_mx_launch_cfg11(const uint8_t*, const uint8_t*, const uint8_t*, const uint8_t*,
                                int, int, int, int, const EpiArgs&, hipStream_t);
hipError_t gemm_mx_launch_cfg12(const uint8_t*, const uint8_t*, const uint8_t*, const uint8_t*,
                                int, int, int, int, const EpiArgs&, hipStream_t);

const char* gemm_cfg_name(int cfg) {
  static const char* names[N_GEMM_CFGS] = {"DL_256x256_W2x4", "DL_256x256_W4x2", "DL_256x256_W2x2", "DL_128x128_W2x2", "DL_256x128_W2x2", "DL_128x256_W2x2", "REG_128x128_W2x2", "DL_192x256_W2x4",
                                           "DL3_160x256_W1x8", "MX_160x256_W1x8", "MX_192x256_W2x4", "MX_128x256_W2x4", "MX_128x128_W2x2"};
  return cfg >= 0 && cfg < N_GEMM_CFGS ? names[cfg] : "unknown";
}

int gemm_cfg_heuristic(int M, int N, int K, bool b_fp8) {
  (void)K;
  (void)b_fp8;
  // Estimated time in units of one 256 x 256 tile on one CU: rounds of tiles
  // over the 256 CUs times the relative tile time (area / relative
  // efficiency, from measurements on gfx950).  Small grids fall back to
  // 128 x 128 tiles.
  struct C { int cfg, bm, bn; double eff; };
  static const C cands[] = {{CFG_DL_256x256_W2x4, 256, 256, 1.0},
                            {CFG_DL_192x256_W2x4, 192, 256, 0.9},
                            {CFG_DL3_160x256_W1x8, 160, 256, 0.85},
                            {CFG_DL_128x128_W2x2, 128, 128, 0.55}};
  int best = CFG_DL_128x128_W2x2;
  double best_t = 1e300;
  for (const C& c : cands) {
    const long tiles = (long)((M + c.bm - 1) / c.bm) * ((N + c.bn - 1) / c.bn);
    const double t = (double)((tiles + 255) / 256) * (c.bm * c.bn) / (65536.0 * c.eff);
    if (t < best_t) { best_t = t; best = c.cfg; }
  }
  return best;
}

hipError_t gemm_bf16(const bf16_t* A, int lda, const void* B, int ldb, bool b_fp8, int M, int N,
                     int K, int op, int cfg, const EpiArgs& e, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  if (b_fp8 && op == OP_PATCH) return hipErrorInvalidValue;
  if (cfg < 0 || cfg >= N_BF16_CFGS) cfg = gemm_cfg_heuristic(M, N, K, b_fp8);
  // The register-staged kernel has no producer side of the LayerNorm
  // folding, reads no device row count and has no GELU-backward form; its
  // direct-to-LDS counterpart gives the same bits.
  if (cfg == CFG_REG_128x128_W2x2 && (e.u_out || e.m_dev || op == OP_DGELU))
    cfg = CFG_DL_128x128_W2x2;
  switch (cfg) {
    case 0: return gemm_launch_cfg0(A, lda, B, ldb, b_fp8, M, N, K, op, e, s);
    case 1: return gemm_launch_cfg1(A, lda, B, ldb, b_fp8, M, N, K, op, e, s);
    case 2: return gemm_launch_cfg2(A, lda, B, ldb, b_fp8, M, N, K, op, e, s);
    case 3: return gemm_launch_cfg3(A, lda, B, ldb, b_fp8, M, N, K, op, e, s);
    case 4: return gemm_launch_cfg4(A, lda, B, ldb, b_fp8, M, N, K, op, e, s);
    case 5: return gemm_launch_cfg5(A, lda, B, ldb, b_fp8, M, N, K, op, e, s);
    case 6: return gemm_launch_cfg6(A, lda, B, ldb, b_fp8, M, N, K, op, e, s);
    case 7: return gemm_launch_cfg7(A, lda, B, ldb, b_fp8, M, N, K, op, e, s);
    case 8: return gemm_launch_cfg8(A, lda, B, ldb, b_fp8, M, N, K, op, e, s);
  }
  return hipErrorInvalidValue;
}

int gemm_mx_cfg_heuristic(int M, int N, int K) {
  (void)K;
  // Same model as the BF16 heuristic, with the relative tile efficiencies
  // measured for the MXFP8 kernel on gfx950.
  struct C { int cfg, bm, bn; double eff; };
  static const C cands[] = {{CFG_MX_192x256_W2x4, 192, 256, 1.0},
                            {CFG_MX_160x256_W1x8, 160, 256, 0.95},
                            {CFG_MX_128x256_W2x4, 128, 256, 0.85},
                            {CFG_MX_128x128_W2x2, 128, 128, 0.6}};
  int best = CFG_MX_128x128_W2x2;
  double best_t = 1e300;
  for (const C& c : cands) {
    const long tiles = (long)((M + c.bm - 1) / c.bm) * ((N + c.bn - 1) / c.bn);
    const double t = (double)((tiles + 255) / 256) * (c.bm * c.bn) / (65536.0 * c.eff);
    if (t < best_t) { best_t = t; best = c.cfg; }
  }
  return best;
}

hipError_t gemm_mx(const uint8_t* A, const uint8_t* SA, const uint8_t* B, const uint8_t* SB,
                   int M, int N, int K, int op, int cfg, const EpiArgs& e, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  if (K % 128 || N % 32) return hipErrorInvalidValue;
  if (!gemm_cfg_is_mx(cfg)) cfg = gemm_mx_cfg_heuristic(M, N, K);
  switch (cfg) {
    case CFG_MX_160x256_W1x8: return gemm_mx_launch_cfg9(A, SA, B, SB, M, N, K, op, e, s);
    case CFG_MX_192x256_W2x4: return gemm_mx_launch_cfg10(A, SA, B, SB, M, N, K, op, e, s);
    case CFG_MX_128x256_W2x4: return gemm_mx_launch_cfg11(A, SA, B, SB, M, N, K, op, e, s);
    case CFG_MX_128x128_W2x2: return gemm_mx_launch_cfg12(A, SA, B, SB, M, N, K, op, e, s);
  }
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------ FP32 FMA GEMM
template <int OP>
__global__ __launch_bounds__(256) void k_gemm_f32(const float* __restrict__ A, int lda,
                                                  const float* __restrict__ B, int ldb, int M,
                                                  int N, int K, EpiArgs e) {
  constexpr int EPI = OpEpi<OP>::kind;
  constexpr int T = 64, KS = 16;
  __shared__ float sA[2][KS][T + 4];
  __shared__ float sB[2][KS][T + 4];
  const int tid = threadIdx.x;
  const int m0 = blockIdx.x * T, n0 = blockIdx.y * T;
  // loader: row = tid / 4, k4 = (tid % 4) * 4
  const int lrow = tid >> 2, lk = (tid & 3) * 4;
  const float* pa = A + (size_t)min(m0 + lrow, M - 1) * lda + lk;
  const float* pb = B + (size_t)min(n0 + lrow, N - 1) * ldb + lk;
  const int tm = tid >> 4, tn = tid & 15;
  float acc[4][4] = {};
  float4 ra = *reinterpret_cast<const float4*>(pa);
  float4 rb = *reinterpret_cast<const float4*>(pb);
  auto st = [&](int buf) {
    sA[buf][lk + 0][lrow] = ra.x; sA[buf][lk + 1][lrow] = ra.y;
    sA[buf][lk + 2][lrow] = ra.z; sA[buf][lk + 3][lrow] = ra.w;
    sB[buf][lk + 0][lrow] = rb.x; sB[buf][lk + 1][lrow] = rb.y;
    sB[buf][lk + 2][lrow] = rb.z; sB[buf][lk + 3][lrow] = rb.w;
  };
  st(0);
  __syncthreads();
  const int KT = K / KS;
  for (int kt = 0; kt < KT; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < KT) {
      ra = *reinterpret_cast<const float4*>(pa + (kt + 1) * KS);
      rb = *reinterpret_cast<const float4*>(pb + (kt + 1) * KS);
    }
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const float4 a = *reinterpret_cast<const float4*>(&sA[cur][k][tm * 4]);
      const float4 b = *reinterpret_cast<const float4*>(&sB[cur][k][tn * 4]);
      const float av[4] = {a.x, a.y, a.z, a.w};
      const float bv[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(av[i], bv[j], acc[i][j]);
    }
    if (kt + 1 < KT) st(cur ^ 1);
    __syncthreads();
  }
  const int n = n0 + tn * 4;
  if (n >= N) return;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + tm * 4 + i;
    if (m < M) epi_store4<EPI, false>(e, m, n, acc[i][0], acc[i][1], acc[i][2], acc[i][3]);
  }
}

hipError_t gemm_f32(const float* A, int lda, const float* B, int ldb, int M, int N, int K,
                    int op, const EpiArgs& e, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  dim3 grid((M + 63) / 64, (N + 63) / 64), block(256);
#define VL_GEMM_CASE(OP)                                                                    \
  case OP:                                                                                  \
    hipLaunchKernelGGL(k_gemm_f32<OP>, grid, block, 0, s, A, lda, B, ldb, M, N, K, e); break;
  switch (op) {
    VL_GEMM_CASE(OP_PATCH)
    VL_GEMM_CASE(OP_QKV)
    VL_GEMM_CASE(OP_OPROJ)
    VL_GEMM_CASE(OP_FC1)
    VL_GEMM_CASE(OP_FC2)
    VL_GEMM_CASE(OP_LOGITS)
    VL_GEMM_CASE(OP_FC1_PRE)
    default: return hipErrorInvalidValue;
  }
#undef VL_GEMM_CASE
  return hipGetLastError();
}

// ------------------------------------------------ FP32 GEMM with few A rows
// The small products of the heads (logits of a few images against many
// texts, projections of pooled rows): A has few rows and B is the large
// operand, so 64x64 tiles leave most CUs idle.  A workgroup owns 8 rows of A
// (staged in LDS in K chunks) and 32 columns; thread (kq, column) sums its
// column's products with the 8 rows over the float4 chunks kq, kq + 8, kq +
// 16, ... of K, and the 8 partial sums of an output are added in kq order.
// Every output is computed the same way whatever M is, so a row's result does
// not depend on the other rows of the batch.
constexpr int FR_M = 8, FR_N = 32, FR_KQ = 8, FR_KC = 512;

template <int OP>
__global__ __launch_bounds__(256) void k_gemm_f32_rows(const float* __restrict__ A, int lda,
                                                       const float* __restrict__ B, int ldb,
                                                       int M, int N, int K, EpiArgs e) {
  constexpr int EPI = OpEpi<OP>::kind;
  __shared__ float4 sA[FR_M][FR_KC / 4];
  __shared__ float sP[FR_KQ][FR_M][FR_N + 1];
  const int tid = threadIdx.x;
  const int nl = tid & (FR_N - 1), kq = tid >> 5;
  const int nbn = (N + FR_N - 1) / FR_N;      // one-dimensional grid: no limit on M
  const int m0 = (int)(blockIdx.x / nbn) * FR_M, n0 = (int)(blockIdx.x % nbn) * FR_N;
  const float* brow = B + (size_t)min(n0 + nl, N - 1) * ldb;
  float acc[FR_M];
#pragma unroll
  for (int r = 0; r < FR_M; ++r) acc[r] = 0.f;
  constexpr int NB = FR_KC / 4 / FR_KQ;   // B chunks per thread and K chunk
  for (int k0 = 0; k0 < K; k0 += FR_KC) {
    const int nc = min(FR_KC, K - k0) / 4;   // float4 chunks in this K chunk
    // All of this thread's B loads of the K chunk are issued first, so their
    // latencies overlap one another and the A staging.
    float4 b[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int c = kq + FR_KQ * i;
      b[i] = c < nc ? *reinterpret_cast<const float4*>(brow + k0 + 4 * c)
                    : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    __syncthreads();                          // readers of the previous chunk are done
    for (int i = tid; i < FR_M * nc; i += 256) {
      const int r = i / nc, c = i - r * nc;
      sA[r][c] = *reinterpret_cast<const float4*>(A + (size_t)min(m0 + r, M - 1) * lda + k0 + 4 * c);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int c = kq + FR_KQ * i;
      if (c >= nc) break;
#pragma unroll
      for (int r = 0; r < FR_M; ++r) {
        const float4 a = sA[r][c];
        acc[r] = fmaf(a.x, b[i].x, acc[r]);
        acc[r] = fmaf(a.y, b[i].y, acc[r]);
        acc[r] = fmaf(a.z, b[i].z, acc[r]);
        acc[r] = fmaf(a.w, b[i].w, acc[r]);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < FR_M; ++r) sP[kq][r][nl] = acc[r];
  __syncthreads();
  if (tid >= FR_M * FR_N / 4) return;
  const int r = tid / (FR_N / 4), nq = (tid % (FR_N / 4)) * 4;
  const int m = m0 + r, n = n0 + nq;
  if (m >= M || n >= N) return;
  float v[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    float t = sP[0][r][nq + j];
#pragma unroll
    for (int q = 1; q < FR_KQ; ++q) t += sP[q][r][nq + j];
    v[j] = t;
  }
  epi_store4<EPI, false>(e, m, n, v[0], v[1], v[2], v[3]);
}

hipError_t gemm_f32_rows(const float* A, int lda, const float* B, int ldb, int M, int N, int K,
                         int op, const EpiArgs& e, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  const int64_t blocks = (int64_t)((N + FR_N - 1) / FR_N) * ((M + FR_M - 1) / FR_M);
  if (blocks > INT32_MAX) return hipErrorInvalidValue;
  dim3 grid((unsigned)blocks), block(256);
#define VL_GEMM_CASE(OP)                                                                   \
  case OP:                                                                                 \
    hipLaunchKernelGGL(k_gemm_f32_rows<OP>, grid, block, 0, s, A, lda, B, ldb, M, N, K, e); \
    break;
  switch (op) {
    VL_GEMM_CASE(OP_QKV)
    VL_GEMM_CASE(OP_OPROJ)
    VL_GEMM_CASE(OP_FC1)
    VL_GEMM_CASE(OP_FC2)
    VL_GEMM_CASE(OP_LOGITS)
    default: return hipErrorInvalidValue;
  }
#undef VL_GEMM_CASE
  return hipGetLastError();
}

}  // namespace vl
