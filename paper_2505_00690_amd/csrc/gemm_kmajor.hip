// K-major BF16 GEMM for weight gradients (training backward).
//
// A weight gradient sums over tokens: dW[m][n] = sum_t G[t][m] X[t][n], with
// the output gradient G [T, M] and the layer input X [T, N] both stored
// token-major (the contraction index is the row).  The block GEMMs take
// K-contiguous operands; this kernel takes both operands K-major instead, so
// no transposed copies are needed: 64-row K tiles of A and B stream into LDS
// by direct-to-LDS loads (row-major, 512-byte rows), and each MFMA fragment
// (8 K values of one row m or n) comes from two gfx950 LDS transpose reads
// (ds_read_b64_tr_b16), which give lane (column c, half g) K rows
// 16jj + 4g + 0..3 and 16jj + 8 + 4g + 0..3 of its column.  A and B use the
// same K order, so each MFMA contracts matching pairs.
#include "gemm_kernels.hpp"

namespace vl {

namespace {

constexpr int KM_T = 256;   // tile side (M and N)
constexpr int KM_K = 64;    // K rows per LDS tile
constexpr int KM_ROWB = KM_T * 2;            // bytes per K row of a tile
constexpr int KM_BYTES = KM_K * KM_ROWB;     // one operand tile, 32 KB

// Chunk c (16 bytes) of K row r of a tile sits at position c ^ f(r).  Rows
// of 512 bytes all start at bank 0, and one 32-lane pass of transpose reads
// covers K rows 4t .. 4t+3 at four consecutive chunks each: f(r) = 4 (r & 3)
// puts those 16 (row, chunk) pairs in 16 distinct 16-byte bank groups.
__device__ __forceinline__ int km_f(int r) { return (r & 3) << 2; }

typedef short s16x4k __attribute__((ext_vector_type(4)));

// Fragment at LDS byte address `a` (a lane's offset for its column block and
// K sub-step already added): two transpose reads, K rows +0..3 and +8..11.
__device__ __forceinline__ bf16x8 km_frag(uint32_t a) {
  typedef __attribute__((address_space(3))) s16x4k lds_s16x4;
  const s16x4k v0 = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)(uintptr_t)a);
  const s16x4k v1 =
      __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)(uintptr_t)(a + 8 * KM_ROWB));
  u32x4 vk;
  vk[0] = __builtin_bit_cast(u32x2, v0).x; vk[1] = __builtin_bit_cast(u32x2, v0).y;
  vk[2] = __builtin_bit_cast(u32x2, v1).x; vk[3] = __builtin_bit_cast(u32x2, v1).y;
  return __builtin_bit_cast(bf16x8, vk);
}

}  // namespace

// C = alpha A^T B + beta over K rows [z kc, z kc + kc) of split z = grid y,
// written FP32 at out + z zstride ([M, ldo]).  A [K, lda], B [K, ldb] BF16,
// rows >= k_valid read as zero.  8 waves, 2 x 4 of 128 x 64 outputs.
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2))) void
k_gemm_bf16_kmajor(const bf16_t* __restrict__ A, int lda, const bf16_t* __restrict__ B, int ldb,
                   int K, int k_valid, int gm, int gn, EpiArgs e) {
  __shared__ __attribute__((aligned(1024))) char smem[2 * 2 * KM_BYTES];   // [stage][A | B]
  const int kbeg = blockIdx.y * e.kc, kend = min(K, kbeg + e.kc);
  float* out = static_cast<float*>(e.out) + blockIdx.y * e.zstride;
  int tm, tn;
  xcd_tile(gm, gn, 8, &tm, &tn);
  const int m0 = tm * KM_T, n0 = tn * KM_T;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 2, wn = wave & 3;
  const int l32 = lane & 31, g = lane >> 5;
  const uint32_t lds0 = lds_offset(smem);

  // Loads: per operand tile 32 instructions of 1 KB (two K rows); wave w
  // issues pairs 4w .. 4w+3; lane l takes row l / 32 of the pair and physical
  // chunk l % 32, i.e. logical chunk (l % 32) ^ f(row).
  auto issue = [&](int st, int k0) {
    const int rows_left = max(0, k_valid - k0);
    const i32x4 ra = buffer_rsrc(A + (size_t)k0 * lda, (uint64_t)rows_left * lda * 2);
    const i32x4 rb = buffer_rsrc(B + (size_t)k0 * ldb, (uint64_t)rows_left * ldb * 2);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int pair = 4 * wave + j;
      const int row = 2 * pair + (lane >> 5);
      const int lc = (lane & 31) ^ km_f(row);
      const uint32_t lo = lds0 + st * 2 * KM_BYTES + pair * 1024;
      dma16(ra, lo, row * lda * 2 + (m0 + 8 * lc) * 2, 0);
      dma16(rb, lo + KM_BYTES, row * ldb * 2 + (n0 + 8 * lc) * 2, 0);
    }
  };

  // This lane's transpose-read offsets within a tile at K sub-step 0.  A
  // 16-lane group reads K rows 4 (group / 2) + i / 4 (i = lane % 16) and
  // columns 32 blk + 16 (group % 2) + 4 (i % 4) .. +3, i.e. logical chunk
  // 4 blk + c8 with c8 < 4, stored at (4 blk + c8) ^ f(row) =
  // 4 (blk ^ (row & 3)) + c8.  Rows 8 and 16 further keep row & 3.
  const int grp = lane >> 4, li = lane & 15;
  const int krow = 4 * (grp >> 1) + (li >> 2);
  const int col = 16 * (grp & 1) + 4 * (li & 3);
  const int xr = krow & 3;
  const int lbase = krow * KM_ROWB + ((col >> 3) << 4) + (col & 7) * 2;
  int offA[4], offB[2];
#pragma unroll
  for (int b = 0; b < 4; ++b) offA[b] = lbase + (((4 * wm + b) ^ xr) << 6);
#pragma unroll
  for (int a = 0; a < 2; ++a) offB[a] = lbase + (((2 * wn + a) ^ xr) << 6);

  f32x16 acc[4][2];
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[b][a][r] = 0.f;

  const int nk = (kend - kbeg + KM_K - 1) / KM_K;
  if (nk <= 0) return;   // (a split past K: no launch makes one)
  bf16x8 fa0[4], fb0[2], fa1[4], fb1[2];
  auto ldfrag = [&](bf16x8* fa, bf16x8* fb, int st, int kk) {
    const uint32_t tA = lds0 + st * 2 * KM_BYTES + kk * 16 * KM_ROWB, tB = tA + KM_BYTES;
#pragma unroll
    for (int b = 0; b < 4; ++b) fa[b] = km_frag(tA + offA[b]);
#pragma unroll
    for (int a = 0; a < 2; ++a) fb[a] = km_frag(tB + offB[a]);
  };
  auto mma = [&](const bf16x8* fa, const bf16x8* fb) {
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a)
        acc[b][a] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[b], fb[a], acc[b][a], 0, 0, 0);
  };
  // One MFMA, then two LDS reads (one fragment of the next sub-step), six
  // times; the last two MFMAs carry none.
  auto interleave = [&]() {
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
  };

  // Two stages: tile t+1 loads while tile t is read.  The barrier at the
  // end of step t makes tile t+1 visible and frees stage t for tile t+2; the
  // last sub-step's MFMAs of tile t run after it, overlapping the first reads
  // of tile t+1.
  issue(0, kbeg);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  lds_barrier();
  ldfrag(fa0, fb0, 0, 0);
  for (int t = 0; t < nk; ++t) {
    const int cur = t & 1, nxt = cur ^ 1;
    if (t + 1 < nk) issue(nxt, kbeg + (t + 1) * KM_K);
    ldfrag(fa1, fb1, cur, 1);
    mma(fa0, fb0);
    interleave();
    ldfrag(fa0, fb0, cur, 2);
    mma(fa1, fb1);
    interleave();
    ldfrag(fa1, fb1, cur, 3);
    mma(fa0, fb0);
    interleave();
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // this wave's loads of tile t+1
    lds_barrier();
    // (after the last tile these read a stage that is never used)
    ldfrag(fa0, fb0, nxt, 0);
    mma(fa1, fb1);
    interleave();
  }
  // acc[b][a][r] = C[m][n], m = m0 + 128 wm + 32 b + 8 (r / 4) + 4 g + r % 4,
  // n = n0 + 64 wn + 32 a + l32: 32 consecutive columns per row and store.
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = m0 + 128 * wm + 32 * b + 8 * (r >> 2) + 4 * g + (r & 3);
        const int n = n0 + 64 * wn + 32 * a + l32;
        out[(size_t)m * e.ldo + n] = e.alpha * acc[b][a][r] + e.beta;
      }
}

hipError_t gemm_bf16_kmajor(const bf16_t* A, int lda, const bf16_t* B, int ldb, int M, int N,
                            int K, int k_valid, const EpiArgs& e, hipStream_t s) {
  if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
  if (M % KM_T || N % KM_T || K % KM_K || e.kc <= 0 || e.kc % KM_K || lda % 8 || ldb % 8 ||
      lda < M || ldb < N || k_valid > K)
    return hipErrorInvalidValue;
  const int gm = M / KM_T, gn = N / KM_T;
  dim3 grid(gm * gn, (K + e.kc - 1) / e.kc), block(512);
  hipLaunchKernelGGL(k_gemm_bf16_kmajor, grid, block, 0, s, A, lda, B, ldb, K, k_valid, gm, gn,
                     e);
  return hipGetLastError();
}

}  // namespace vl
