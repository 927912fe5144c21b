// Dense contractions (kernel templates) C[M,N] = A[M,K] . B[N,K]^T with
// fused epilogues: bias, GELU, residual add, patch-embedding class-token and
// position add, per-row weight scales (e4m3 weights), the folded-LayerNorm
// forms and split-K partial products.
//
// k_gemm_bf16_dl (the kernel every BF16 configuration uses but one):
// direct-to-LDS tile loads into a two- or three-stage ring, chunk swizzle
// (r ^ (r >> 3)) & 7, one LDS fragment read interleaved with each MFMA, the
// last K sub-step's MFMAs issued after the barrier, XCD-aware tile order, and
// an LDS-staged epilogue that stores whole rows.  k_gemm_bf16: the older
// register-staged kernel (configuration REG_128x128), kept as a reference
// configuration.  Both give the same bits.
// BF16 / FP32 GEMM kernel templates shared by the per-configuration
// translation units (gemm_cfg_*.hip) and the FP32 unit (gemm.hip).
#pragma once


#include "kernels.hpp"

namespace vl {

// ---------------------------------------------------------------- epilogue
enum EpiKind { EPI_BIAS, EPI_BIAS_GELU, EPI_BIAS_RESID, EPI_PATCH, EPI_SCALE_BIAS, EPI_BIAS_F32,
               EPI_DGELU };
template <int OP>
struct OpEpi {
  static constexpr int kind = OP == OP_PATCH ? EPI_PATCH
                              : OP == OP_QKV ? EPI_BIAS
                              : OP == OP_FC1 ? EPI_BIAS_GELU
                              : OP == OP_LOGITS ? EPI_SCALE_BIAS
                              : OP == OP_FC1_PRE ? EPI_BIAS_F32
                              : OP == OP_DGELU ? EPI_DGELU
                                                : EPI_BIAS_RESID;
};

// LayerNorm-folded output (consumer side, see EpiArgs): one formula shared
// by every kernel so all tile configurations agree bitwise.
__device__ __forceinline__ float ln_fold1(float v, float ws, float c1, float c2, float mu,
                                          float rstd) {
  return __builtin_fmaf(rstd, __builtin_fmaf(v, ws, -(mu * c1)), c2);
}

// GELU backward of four columns (OP_DGELU): dz = dg (Phi(z) + z phi(z)) and,
// with out2, g = GELU(z), Phi from the forward's polynomial (so g has the
// forward's bits), phi = exp(-z^2 / 2) / sqrt(2 pi); both stored as BF16.
__device__ __forceinline__ void dgelu_store4(const EpiArgs& e, int m, int n, float4 dg,
                                             float4 z) {
  const float zz[4] = {z.x, z.y, z.z, z.w}, dd[4] = {dg.x, dg.y, dg.z, dg.w};
  float dz[4], gg[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float c = phi_poly(zz[j]);
    const float ph =
        0.3989422804014327f * __builtin_amdgcn_exp2f(-0.72134752044448170f * zz[j] * zz[j]);
    dz[j] = dd[j] * (c + zz[j] * ph);
    gg[j] = zz[j] * c;
  }
  const size_t o = (size_t)m * e.ldo + n;
  u32x2 pk;
  pk.x = pack_bf16x2(dz[0], dz[1]);
  pk.y = pack_bf16x2(dz[2], dz[3]);
  *reinterpret_cast<u32x2*>(static_cast<bf16_t*>(e.out) + o) = pk;
  if (e.out2) {
    pk.x = pack_bf16x2(gg[0], gg[1]);
    pk.y = pack_bf16x2(gg[2], gg[3]);
    *reinterpret_cast<u32x2*>(static_cast<bf16_t*>(e.out2) + o) = pk;
  }
}

// BF16 GELU of an FP32 pre-activation into out2 (OP_FC1_PRE with out2).
__device__ __forceinline__ void gelu_out2_store4(const EpiArgs& e, int m, int n, float4 y) {
  u32x2 pk;
  pk.x = pack_bf16x2(gelu_poly(y.x), gelu_poly(y.y));
  pk.y = pack_bf16x2(gelu_poly(y.z), gelu_poly(y.w));
  *reinterpret_cast<u32x2*>(static_cast<bf16_t*>(e.out2) + (size_t)m * e.ldo + n) = pk;
}

template <int EPI, bool OUT_BF16>
__device__ __forceinline__ void epi_store4(const EpiArgs& e, int m, int n, float v0, float v1,
                                           float v2, float v3) {
  float v[4] = {v0, v1, v2, v3};
  if (EPI == EPI_DGELU) {
    dgelu_store4(e, m, n, make_float4(v[0], v[1], v[2], v[3]),
                 *reinterpret_cast<const float4*>(e.aux + (size_t)m * e.ldo + n));
    return;
  }
  if (EPI == EPI_SCALE_BIAS) {
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = e.alpha * v[j] + e.beta;
    *reinterpret_cast<float4*>(static_cast<float*>(e.out) + (size_t)m * e.ldo + n) =
        make_float4(v[0], v[1], v[2], v[3]);
    if (e.out2) {   // BF16 copy
      u32x2 pk;
      pk.x = pack_bf16x2(v[0], v[1]);
      pk.y = pack_bf16x2(v[2], v[3]);
      *reinterpret_cast<u32x2*>(static_cast<bf16_t*>(e.out2) + (size_t)m * e.ldo + n) = pk;
    }
    return;
  }
  float4 ws = make_float4(1.f, 1.f, 1.f, 1.f);
  if (e.wscale) ws = *reinterpret_cast<const float4*>(e.wscale + n);
  if (EPI == EPI_PATCH) {
    v[0] *= ws.x; v[1] *= ws.y; v[2] *= ws.z; v[3] *= ws.w;
    const int2 ti = e.tok_info[m];
    float* X = static_cast<float*>(e.out) + (size_t)m * e.ldo + n;
    float4 add;
    if (ti.y == 0) {
      const float4 c = *reinterpret_cast<const float4*>(e.cls + n);
      const float4 p = *reinterpret_cast<const float4*>(e.pos + n);
      add = make_float4(c.x + p.x, c.y + p.y, c.z + p.z, c.w + p.w);
    } else {
      const ImgDesc d = e.imgs[ti.x];
      const int g0 = e.base_grid;
      const int pidx = ti.y - 1;
      const int r = pidx / d.gw, q = pidx - r * d.gw;
      float sy = ((float)r + 0.5f) * (float)g0 / (float)d.gh - 0.5f;
      float sx = ((float)q + 0.5f) * (float)g0 / (float)d.gw - 0.5f;
      sy = fminf(fmaxf(sy, 0.f), (float)(g0 - 1));
      sx = fminf(fmaxf(sx, 0.f), (float)(g0 - 1));
      const int y0 = (int)sy, x0 = (int)sx;
      const int y1 = min(y0 + 1, g0 - 1), x1 = min(x0 + 1, g0 - 1);
      const float wy = sy - (float)y0, wx = sx - (float)x0;
      const int D = e.ldo;
      const float4 p00 = *reinterpret_cast<const float4*>(e.pos + (size_t)(1 + y0 * g0 + x0) * D + n);
      const float4 p01 = *reinterpret_cast<const float4*>(e.pos + (size_t)(1 + y0 * g0 + x1) * D + n);
      const float4 p10 = *reinterpret_cast<const float4*>(e.pos + (size_t)(1 + y1 * g0 + x0) * D + n);
      const float4 p11 = *reinterpret_cast<const float4*>(e.pos + (size_t)(1 + y1 * g0 + x1) * D + n);
      const float4 b = *reinterpret_cast<const float4*>(e.bias + n);
      const float a00 = (1.f - wy) * (1.f - wx), a01 = (1.f - wy) * wx;
      const float a10 = wy * (1.f - wx), a11 = wy * wx;
      add.x = b.x + a00 * p00.x + a01 * p01.x + a10 * p10.x + a11 * p11.x;
      add.y = b.y + a00 * p00.y + a01 * p01.y + a10 * p10.y + a11 * p11.y;
      add.z = b.z + a00 * p00.z + a01 * p01.z + a10 * p10.z + a11 * p11.z;
      add.w = b.w + a00 * p00.w + a01 * p01.w + a10 * p10.w + a11 * p11.w;
    }
    *reinterpret_cast<float4*>(X) = make_float4(v[0] + add.x, v[1] + add.y, v[2] + add.z,
                                                v[3] + add.w);
    return;
  }
  // acc * weight scale + bias as one fused operation (scale 1 without
  // per-row weight scales); the staged epilogue of the direct-to-LDS kernel
  // does the same, so every configuration agrees bitwise.
  if ((EPI == EPI_BIAS || EPI == EPI_BIAS_GELU) && e.row_stats) {
    const float2 st = *reinterpret_cast<const float2*>(e.row_stats + 2 * (size_t)m);
    const float4 a = *reinterpret_cast<const float4*>(e.c1 + n);
    const float4 c = *reinterpret_cast<const float4*>(e.c2 + n);
    v[0] = ln_fold1(v[0], ws.x, a.x, c.x, st.x, st.y);
    v[1] = ln_fold1(v[1], ws.y, a.y, c.y, st.x, st.y);
    v[2] = ln_fold1(v[2], ws.z, a.z, c.z, st.x, st.y);
    v[3] = ln_fold1(v[3], ws.w, a.w, c.w, st.x, st.y);
  } else {
    const float4 b = *reinterpret_cast<const float4*>(e.bias + n);
    v[0] = __builtin_fmaf(v[0], ws.x, b.x); v[1] = __builtin_fmaf(v[1], ws.y, b.y);
    v[2] = __builtin_fmaf(v[2], ws.z, b.z); v[3] = __builtin_fmaf(v[3], ws.w, b.w);
  }
  if (EPI == EPI_BIAS_RESID) {
    float4* X = reinterpret_cast<float4*>(static_cast<float*>(e.out) + (size_t)m * e.ldo + n);
    float4 x = e.resid_in ? *reinterpret_cast<const float4*>(e.resid_in + (size_t)m * e.ldo + n)
                          : *X;
    x.x += v[0]; x.y += v[1]; x.z += v[2]; x.w += v[3];
    *X = x;
    return;
  }
  if (EPI == EPI_BIAS_F32) {
    const float4 y = make_float4(v[0], v[1], v[2], v[3]);
    *reinterpret_cast<float4*>(static_cast<float*>(e.out) + (size_t)m * e.ldo + n) = y;
    if (e.out2) gelu_out2_store4(e, m, n, y);
    return;
  }
  if (EPI == EPI_BIAS_GELU) {
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = OUT_BF16 ? gelu_poly(v[j]) : gelu_erf(v[j]);
  }
  if (OUT_BF16) {
    u32x2 pk;
    pk.x = pack_bf16x2(v[0], v[1]);
    pk.y = pack_bf16x2(v[2], v[3]);
    *reinterpret_cast<u32x2*>(static_cast<bf16_t*>(e.out) + (size_t)m * e.ldo + n) = pk;
  } else {
    *reinterpret_cast<float4*>(static_cast<float*>(e.out) + (size_t)m * e.ldo + n) =
        make_float4(v[0], v[1], v[2], v[3]);
  }
}

// ------------------------------------------------------------ BF16 MFMA GEMM
constexpr int BK = 64;  // K step (BF16 elements) per LDS tile

// LDS tile layout: rows of 64 BF16 (128 B); the eight 16-byte chunks of row r
// are permuted by XOR with f(r) = (r ^ (r >> 3)) & 7.  An MFMA operand read
// takes one chunk from each of 32 consecutive rows; f makes any 8 consecutive
// rows hit 8 distinct chunk positions and any 16 consecutive rows hit 16
// distinct (row parity, chunk) positions, i.e. distinct banks whether the
// LDS serves 8 lanes over 32 banks or 16 lanes over 64 banks per pass.
__device__ __forceinline__ int swz_f(int row) { return (row ^ (row >> 3)) & 7; }
__device__ __forceinline__ int swz(int row, int chunk) {  // element offset in a tile
  return row * BK + ((chunk ^ swz_f(row)) << 3);
}

template <int BM, int BN, int WGM, int WGN, bool B_FP8, int OP>
__global__ __launch_bounds__(WGM* WGN * 64) void k_gemm_bf16(
    const bf16_t* __restrict__ A, int lda, const void* __restrict__ Bv, int ldb, int M,
    int N, int K, EpiArgs e) {
  constexpr int EPI = OpEpi<OP>::kind;
  constexpr bool OUT_BF16 = OP == OP_QKV || OP == OP_FC1;
  constexpr int NT = WGM * WGN * 64;
  constexpr int WM = BM / WGM;   // activation rows per wave
  constexpr int WN = BN / WGN;   // output columns per wave
  constexpr int TM = WM / 32;
  constexpr int TN = WN / 32;
  constexpr int CA = BM * 8 / NT;                      // 16-B chunks of A per thread
  constexpr int CB = B_FP8 ? BN * 4 / NT : BN * 8 / NT;  // 16-B chunks of B per thread
  static_assert(CA * NT == BM * 8, "A tile / threads");
  static_assert(CB >= 1, "B tile / threads");

  __shared__ __attribute__((aligned(16))) bf16_t sA[2][BM * BK];
  __shared__ __attribute__((aligned(16))) bf16_t sB[2][BN * BK];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  const int m0 = blockIdx.x * BM;
  const int n0 = blockIdx.y * BN;

  // This thread's 16-B chunks: chunk c = tid + i*NT sits in tile row
  // c / 8 (A, BF16 B) or c / 4 (e4m3 B) and chunk column c % 8 (c % 4).
  // Rows past M / N are clamped to the last row (loaded, never stored).
  constexpr int RA = NT / 8;                       // row stride between i's
  constexpr int RB = B_FP8 ? NT / 4 : NT / 8;
  const int a_row0 = tid >> 3, a_kc = tid & 7;
  const int b_row0 = B_FP8 ? (tid >> 2) : (tid >> 3);
  const int b_kc = B_FP8 ? (tid & 3) : (tid & 7);
  const bf16_t* Ab = A + (size_t)m0 * lda;
  const char* Bb = static_cast<const char*>(Bv) + (size_t)n0 * ldb * (B_FP8 ? 1 : 2);
  const int a_lim = M - 1 - m0, b_lim = N - 1 - n0;

  u32x4 ra[CA], rb[CB];
  auto load_tile = [&](int k0) {
#pragma unroll
    for (int i = 0; i < CA; ++i) {
      const int row = min(a_row0 + i * RA, a_lim);
      ra[i] = *reinterpret_cast<const u32x4*>(Ab + row * lda + k0 + a_kc * 8);
    }
#pragma unroll
    for (int i = 0; i < CB; ++i) {
      const int row = min(b_row0 + i * RB, b_lim);
      if (B_FP8)
        rb[i] = *reinterpret_cast<const u32x4*>(Bb + row * ldb + k0 + b_kc * 16);
      else
        rb[i] = *reinterpret_cast<const u32x4*>(Bb + 2 * (row * ldb + k0 + b_kc * 8));
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int i = 0; i < CA; ++i)
      *reinterpret_cast<u32x4*>(&sA[buf][swz(a_row0 + i * RA, a_kc)]) = ra[i];
#pragma unroll
    for (int i = 0; i < CB; ++i) {
      const int row = b_row0 + i * RB;
      if (B_FP8) {
        u32x4 lo, hi;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const uint32_t x = rb[i][w];
          const uint32_t h0 = e4m3_to_bf16_bits(x & 0xFF) | (e4m3_to_bf16_bits((x >> 8) & 0xFF) << 16);
          const uint32_t h1 = e4m3_to_bf16_bits((x >> 16) & 0xFF) | (e4m3_to_bf16_bits(x >> 24) << 16);
          if (w < 2) { lo[2 * w] = h0; lo[2 * w + 1] = h1; }
          else { hi[2 * (w - 2)] = h0; hi[2 * (w - 2) + 1] = h1; }
        }
        *reinterpret_cast<u32x4*>(&sB[buf][swz(row, 2 * b_kc)]) = lo;
        *reinterpret_cast<u32x4*>(&sB[buf][swz(row, 2 * b_kc + 1)]) = hi;
      } else {
        *reinterpret_cast<u32x4*>(&sB[buf][swz(row, b_kc)]) = rb[i];
      }
    }
  };

  f32x16 acc[TN][TM];
#pragma unroll
  for (int a = 0; a < TN; ++a)
#pragma unroll
    for (int b = 0; b < TM; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;

  const int l32 = lane & 31, g = lane >> 5;
  const int KT = K / BK;
  load_tile(0);
  store_tile(0);
  __syncthreads();
  for (int kt = 0; kt < KT; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < KT) load_tile((kt + 1) * BK);
    const bf16_t* tA = sA[cur];
    const bf16_t* tB = sB[cur];
#pragma unroll
    for (int kk = 0; kk < BK / 16; ++kk) {
      bf16x8 fw[TN], fx[TM];
#pragma unroll
      for (int a = 0; a < TN; ++a)
        fw[a] = *reinterpret_cast<const bf16x8*>(&tB[swz(wn * WN + a * 32 + l32, 2 * kk + g)]);
#pragma unroll
      for (int b = 0; b < TM; ++b)
        fx[b] = *reinterpret_cast<const bf16x8*>(&tA[swz(wm * WM + b * 32 + l32, 2 * kk + g)]);
#pragma unroll
      for (int a = 0; a < TN; ++a)
#pragma unroll
        for (int b = 0; b < TM; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fw[a], fx[b], acc[a][b], 0, 0, 0);
    }
    if (kt + 1 < KT) store_tile(cur ^ 1);
    __syncthreads();
  }

  // Epilogue: acc[a][b][r] is C[m, n] with m = row of lane, n = 8(r/4)+4g+r%4.
#pragma unroll
  for (int b = 0; b < TM; ++b) {
    const int m = m0 + wm * WM + b * 32 + l32;
    if (m >= M) continue;
#pragma unroll
    for (int a = 0; a < TN; ++a) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int n = n0 + wn * WN + a * 32 + 8 * q + 4 * g;
        if (n < N)
          epi_store4<EPI, OUT_BF16>(e, m, n, acc[a][b][4 * q + 0], acc[a][b][4 * q + 1],
                                    acc[a][b][4 * q + 2], acc[a][b][4 * q + 3]);
      }
    }
  }
}

// ------------------------------------------- BF16 MFMA GEMM, direct-to-LDS
// Same contraction and epilogues, for BF16 weights.  Tiles are fetched with
// buffer_load ... lds (16 bytes per lane straight into LDS, no staging
// registers): one wave instruction fills 8 tile rows (1 KB), lane l taking
// row l/8 and physical chunk l%8, i.e. logical chunk (l%8) ^ (l/8) under the
// row-XOR swizzle.  Buffer resources are bounded by the matrix end, so rows
// past M / N read as zero.  Output tiles are assigned XCD by XCD: workgroup
// ids are dealt round-robin to the 8 XCDs, so a contiguous range of tiles is
// given to each XCD and walked in groups of GROUP_M row tiles, letting the
// tiles resident on one XCD share A rows and B rows in its L2.
__device__ __forceinline__ void xcd_tile_of(int bid, int gm, int gn, int group_m, int* tm,
                                            int* tn) {
  const int total = gm * gn;
  const int xcd = bid & 7, local = bid >> 3;
  const int q = total >> 3, r = total & 7;
  const int id = xcd * q + min(xcd, r) + local;
  const int per_group = group_m * gn;
  const int g = id / per_group;
  const int first = g * group_m;
  const int gsz = min(gm - first, group_m);
  const int w = id - g * per_group;
  *tm = first + w % gsz;
  *tn = w / gsz;
}
__device__ __forceinline__ void xcd_tile(int gm, int gn, int group_m, int* tm, int* tn) {
  xcd_tile_of(blockIdx.x, gm, gn, group_m, tm, tn);
}

// e4m3 B tiles: rows of 64 bytes (BK codes) whose four 16-byte chunks are
// XOR-swizzled by (row >> 2) & 3; a fragment read takes 8 codes (ds_read_b64)
// and widens them with v_cvt_scalef32_pk_bf16_fp8 (scale 1: exact).
__device__ __forceinline__ int swz8(int row, int kk, int g) {  // byte offset in an e4m3 tile
  return row * BK + ((kk ^ ((row >> 2) & 3)) << 4) + (g << 3);
}

template <int BM, int BN, int WGM, int WGN, bool B_FP8, int OP, int RPM, int ST>
__global__ __launch_bounds__(WGM* WGN * 64)
__attribute__((amdgpu_waves_per_eu(WGM * WGN / 4, WGM * WGN / 4))) void k_gemm_bf16_dl(
    const bf16_t* __restrict__ A, int lda, const void* __restrict__ Bv, int ldb, int M, int N,
    int K, int gm, int gn, EpiArgs e) {
  constexpr int EPI = OpEpi<OP>::kind;
  constexpr bool OUT_BF16 = OP == OP_QKV || OP == OP_FC1;
  constexpr int NW = WGM * WGN;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int TM = WM / 32, TN = WN / 32;
  static_assert(WM % 32 == 0 && WN % 32 == 0, "wave tile must be whole 32x32 blocks");
  constexpr int BROWS = B_FP8 ? 16 : 8;               // B rows per load instruction
  // Load instructions per wave per tile (the last round may cover only some
  // waves when the row groups do not divide evenly; that test is
  // wave-uniform).
  constexpr int GA = BM / 8, GB = BN / BROWS;  // row groups of A / B per tile
  constexpr int IA = (GA + NW - 1) / NW, IB = (GB + NW - 1) / NW;
  static_assert(GA * 8 == BM && GB * BROWS == BN, "tile rows / load groups");
  constexpr int BES = B_FP8 ? 1 : 2;                    // bytes per B element

  // One LDS arena: a ring of ST operand tile pairs during the K loop, then
  // per-wave epilogue staging slabs (32 rows x WN FP32 each).
  static_assert(ST == 2 || ST == 3, "two or three K tiles in flight");
  constexpr int LDS_AB = ST * (BM * BK * 2 + BN * BK * BES);
  constexpr int LDS_EPI = NW * 32 * WN * 4;
  __shared__ __attribute__((aligned(1024))) char smem[LDS_AB > LDS_EPI ? LDS_AB : LDS_EPI];
  bf16_t(*sA)[BM * BK] = reinterpret_cast<bf16_t(*)[BM * BK]>(smem);
  uint8_t(*sB)[BN * BK * BES] = reinterpret_cast<uint8_t(*)[BN * BK * BES]>(smem + ST * BM * BK * 2);

  if (EPI == EPI_SCALE_BIAS && e.kc > 0) {   // split-K: this split's K columns
    const int k0 = blockIdx.y * e.kc;
    A += k0;
    Bv = static_cast<const char*>(Bv) + (size_t)k0 * BES;
    K = min(e.kc, K - k0);
    e.out = static_cast<float*>(e.out) + blockIdx.y * e.zstride;
  }
  if (e.m_dev) {   // capacity launch: the live row count comes from the device
    M = *e.m_dev;
    gm = (M + BM - 1) / BM;
    if (!xcd_live(blockIdx.x, gm * gn)) return;
  }
  int tm_, tn_;
  xcd_tile(gm, gn, 8, &tm_, &tn_);
  const int m0 = tm_ * BM, n0 = tn_ * BN;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WGN, wn = wave % WGN;

  const i32x4 ra = buffer_rsrc(A + (size_t)m0 * lda, (uint64_t)(M - m0) * lda * 2);
  const i32x4 rb = buffer_rsrc(static_cast<const char*>(Bv) + (size_t)n0 * ldb * BES,
                               (uint64_t)(N - n0) * ldb * BES);
  // Lane's place inside an 8-row group g8: row 8*g8 + l/8, physical chunk
  // l%8, hence logical chunk (l%8) ^ f(row) = (l%8) ^ (l/8) ^ (g8%8).
  const int lrow = lane >> 3, lchunk = (lane & 7) ^ (lane >> 3);
  const int a_off = lrow * lda * 2;
  // e4m3 B: 16-row groups, lane row l/4, physical chunk l%4, logical chunk
  // (l%4) ^ ((l/16)%4).
  const int b_off = B_FP8 ? (lane >> 2) * ldb + (((lane & 3) ^ ((lane >> 4) & 3)) << 4)
                          : lrow * ldb * 2;

  const uint32_t ldsA = lds_offset(&sA[0][0]), ldsB = lds_offset(&sB[0][0]);
  auto issue = [&](int buf, int k0) {
#pragma unroll
    for (int i = 0; i < IA; ++i) {
      const int grp = wave + i * NW;  // 8-row group index
      if (GA % NW != 0 && grp >= GA) break;
      dma16(ra, ldsA + (buf * BM * BK + grp * 8 * BK) * 2,
            a_off + grp * 8 * lda * 2 + ((lchunk ^ (grp & 7)) << 4), k0 * 2);
    }
#pragma unroll
    for (int i = 0; i < IB; ++i) {
      const int grp = wave + i * NW;
      if (GB % NW != 0 && grp >= GB) break;
      dma16(rb, ldsB + (buf * BN * BK + grp * BROWS * BK) * BES,
            b_off + grp * BROWS * ldb * BES + (B_FP8 ? 0 : ((lchunk ^ (grp & 7)) << 4)),
            k0 * BES);
    }
  };

  f32x16 acc[TN][TM];
#pragma unroll
  for (int a = 0; a < TN; ++a)
#pragma unroll
    for (int b = 0; b < TM; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;

  const int l32 = lane & 31, g = lane >> 5;
  const int KT = K / BK;
  // Fragments of K sub-step kk (16 K values) of the current tile.  Each
  // fragment row's byte offset in a tile buffer is precomputed with the
  // swizzle and the lane's half g folded in: BF16 chunk (2kk + g) ^ f(row)
  // of a 128-byte row is (offset ^ (kk << 5)); e4m3 chunk kk ^ f8(row) of a
  // 64-byte row is (offset ^ (kk << 4)).
  // Row r0 + 32b has the chunk permutation of row r0 + 32 (b & 1) (the
  // swizzles depend on the row modulo 64), so the offset of fragment b is
  // one of two per-lane bases plus an immediate of 32b rows: two live
  // registers per operand instead of one per fragment.
  int pA[2], pB[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int ra = wm * WM + j * 32 + l32, rb = wn * WN + j * 32 + l32;
    pA[j] = (wm * WM + l32) * (BK * 2) + ((g ^ swz_f(ra)) << 4);
    pB[j] = B_FP8 ? (wn * WN + l32) * BK + (((rb >> 2) & 3) << 4) + (g << 3)
                  : (wn * WN + l32) * (BK * 2) + ((g ^ swz_f(rb)) << 4);
  }
  bf16x8 fw0[TN], fx0[TM], fw1[TN], fx1[TM];
  auto ldfrag = [&](bf16x8* fw, bf16x8* fx, int buf, int kk) {
    const char* tA = reinterpret_cast<const char*>(sA[buf]);
    const char* tB = reinterpret_cast<const char*>(sB[buf]);
#pragma unroll
    for (int a = 0; a < TN; ++a) {
      if (B_FP8) {
        const u32x2 c8 =
            *reinterpret_cast<const u32x2*>(tB + (pB[a & 1] ^ (kk << 4)) + a * 32 * BK);
        typedef __bf16 b2 __attribute__((ext_vector_type(2)));
        const b2 h0 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(c8.x, 1.0f, false);
        const b2 h1 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(c8.x, 1.0f, true);
        const b2 h2 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(c8.y, 1.0f, false);
        const b2 h3 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(c8.y, 1.0f, true);
        bf16x8 f;
        f[0] = h0[0]; f[1] = h0[1]; f[2] = h1[0]; f[3] = h1[1];
        f[4] = h2[0]; f[5] = h2[1]; f[6] = h3[0]; f[7] = h3[1];
        fw[a] = f;
      } else {
        fw[a] = *reinterpret_cast<const bf16x8*>(tB + (pB[a & 1] ^ (kk << 5)) + a * 32 * BK * 2);
      }
    }
#pragma unroll
    for (int b = 0; b < TM; ++b)
      fx[b] = *reinterpret_cast<const bf16x8*>(tA + (pA[b & 1] ^ (kk << 5)) + b * 32 * BK * 2);
  };
  auto mma = [&](const bf16x8* fw, const bf16x8* fx) {
#pragma unroll
    for (int a = 0; a < TN; ++a)
#pragma unroll
      for (int b = 0; b < TM; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fw[a], fx[b], acc[a][b], 0, 0, 0);
  };
  // One MFMA, RPM LDS reads (1 when RPM does not divide the fragment count),
  // ... then the remaining MFMAs: all of the next
  // sub-step's reads are in flight early in the current one.
  constexpr int NF = TN + TM, NM = TN * TM;
  constexpr int RPM_ = NF % RPM == 0 ? RPM : 1;
  constexpr int NG = NF / RPM_;  // MFMAs that carry reads
  auto interleave = [&]() {
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, RPM_, 0);
    }
    if (NM > NG) __builtin_amdgcn_sched_group_barrier(0x008, NM - NG, 0);
  };

  // Loads of one tile by this wave (fewer for the waves past the last full
  // round of row groups); with three stages the wait before a barrier leaves
  // exactly the next tile's loads in flight.
  const int n_ld = (GA % NW == 0 || wave < GA % NW ? IA : IA - 1) +
                   (GB % NW == 0 || wave < GB % NW ? IB : IB - 1);
  auto wait_all_but_one_tile = [&]() {
    if (n_ld == IA + IB) asm volatile("s_waitcnt vmcnt(%0)" ::"n"(IA + IB) : "memory");
    else if (n_ld == IA + IB - 1) asm volatile("s_waitcnt vmcnt(%0)" ::"n"(IA + IB - 1) : "memory");
    else asm volatile("s_waitcnt vmcnt(%0)" ::"n"(IA + IB - 2) : "memory");
  };

  // Pipeline across tiles: the last sub-step's MFMAs of tile kt run after the
  // barrier, overlapping the first LDS reads of tile kt+1, so the matrix
  // cores do not drain at every barrier.  Loads run ST - 1 tiles ahead.
  issue(0, 0);
  if (ST == 3 && KT > 1) {
    issue(1, BK);
    wait_all_but_one_tile();
  } else {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  }
  lds_barrier();
  ldfrag(fw0, fx0, 0, 0);
  for (int kt = 0; kt < KT; ++kt) {
    const int cur = ST == 2 ? (kt & 1) : kt % 3;
    const int nxt = ST == 2 ? (cur ^ 1) : (cur == 2 ? 0 : cur + 1);
    if (kt + ST - 1 < KT) issue(ST == 2 ? nxt : (nxt == 2 ? 0 : nxt + 1), (kt + ST - 1) * BK);
    ldfrag(fw1, fx1, cur, 1);
    mma(fw0, fx0);
    interleave();
    ldfrag(fw0, fx0, cur, 2);
    mma(fw1, fx1);
    interleave();
    ldfrag(fw1, fx1, cur, 3);
    mma(fw0, fx0);
    interleave();
    // Tile kt+1 must have landed (the stage being filled for kt+2 held tile
    // kt-1, whose readers all passed the previous barrier).
    if (ST == 3 && kt + 2 < KT) wait_all_but_one_tile();
    else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    lds_barrier();
    // (On the last tile these reads fetch stale fragments that are never
    // used; reading unconditionally keeps the accumulators out of a branch.)
    ldfrag(fw0, fx0, nxt, 0);
    mma(fw1, fx1);
    interleave();
  }

  // Epilogue.  The accumulator layout gives each lane one row and 4-column
  // groups spread over the wave tile, so direct stores would touch 32 rows
  // per instruction.  Instead each 32-row slab of the wave's tile goes
  // through a wave-private LDS slab (row r's 16-byte chunks XOR-permuted by
  // r & 15, or by (r >> 1) & 7 for 8-chunk rows: the 16 lanes of one LDS
  // pass hit distinct banks both when writing a column of rows and when
  // reading along a row) and is
  // read back row-major: consecutive lanes own consecutive 16-byte column
  // chunks, so bias / residual loads and output stores are full-line
  // accesses, and each lane's columns (hence its bias) stay fixed.
  lds_barrier();  // all waves are done with the operand tiles
  constexpr int CPR = WN / 4;    // 16-byte FP32 chunks per staged row
  static_assert(CPR >= 8 && 64 % CPR == 0, "staging layout needs WN in {32, 64, 128}");
  auto sw = [](int r) { return CPR >= 16 ? (r & 15) : ((r >> 1) & 7); };
  constexpr int RPP = 64 / CPR;  // rows per read-back pass
  constexpr int NP = 32 / RPP;   // passes per slab
  constexpr int NB = NP < 8 ? NP : 8;  // passes per batch of global loads
  float* stage = reinterpret_cast<float*>(smem) + wave * 32 * WN;
  const int rc = lane % CPR, rr = lane / CPR;
  const int n = n0 + wn * WN + 4 * rc;
  const bool n_ok = n < N;
  float4 bias4 = make_float4(0.f, 0.f, 0.f, 0.f), ws4 = make_float4(1.f, 1.f, 1.f, 1.f);
  // LayerNorm folding: consumer constants c1 / c2 (c2 in place of the bias),
  // or the producer's next-LayerNorm gain (in bias4's place: unused there).
  const bool fold_in = (EPI == EPI_BIAS || EPI == EPI_BIAS_GELU) && e.row_stats != nullptr;
  const bool fold_out = EPI == EPI_BIAS_RESID && e.u_out != nullptr;
  float4 c14 = make_float4(0.f, 0.f, 0.f, 0.f), g4 = c14;
  if (EPI != EPI_PATCH && EPI != EPI_SCALE_BIAS && EPI != EPI_DGELU && n_ok) {
    if (fold_in) {
      c14 = *reinterpret_cast<const float4*>(e.c1 + n);
      bias4 = *reinterpret_cast<const float4*>(e.c2 + n);
    } else {
      bias4 = *reinterpret_cast<const float4*>(e.bias + n);
    }
    if (fold_out) g4 = *reinterpret_cast<const float4*>(e.u_gamma + n);
    if (e.wscale) ws4 = *reinterpret_cast<const float4*>(e.wscale + n);
  }
  // The residual (or z) rows of a slab: with one batch of loads per slab,
  // slab b+1's are issued before slab b's stores, so waiting for them does
  // not also wait for those stores to complete (the vector memory counter
  // counts loads and stores in issue order).
  constexpr bool XLOAD = EPI == EPI_BIAS_RESID || EPI == EPI_DGELU;
  constexpr bool XNEXT = XLOAD && NB == NP;
  const float* xsrc = EPI == EPI_DGELU ? e.aux
                      : e.resid_in     ? e.resid_in
                                       : static_cast<const float*>(e.out);
  float4 xn[NB];
  auto load_x = [&](int b, float4 (&dst)[NB]) {
#pragma unroll
    for (int p = 0; p < NB; ++p) {
      const int m = m0 + wm * WM + b * 32 + rr + p * RPP;
      if (m < M && n_ok) dst[p] = *reinterpret_cast<const float4*>(xsrc + (size_t)m * e.ldo + n);
    }
  };
  if (XNEXT) load_x(0, xn);
#pragma unroll
  for (int b = 0; b < TM; ++b) {
#pragma unroll
    for (int a = 0; a < TN; ++a)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = a * 8 + 2 * q + g;  // columns a*32 + 8q + 4g .. +3
        *reinterpret_cast<float4*>(stage + l32 * WN + ((c ^ sw(l32)) << 2)) =
            make_float4(acc[a][b][4 * q + 0], acc[a][b][4 * q + 1], acc[a][b][4 * q + 2],
                        acc[a][b][4 * q + 3]);
      }
    const int mb = m0 + wm * WM + b * 32 + rr;
#pragma unroll
    for (int p0 = 0; p0 < NP; p0 += NB) {
      float4 v[NB], x[NB];
#pragma unroll
      for (int p = 0; p < NB; ++p) {
        const int row = (p0 + p) * RPP + rr;
        v[p] = *reinterpret_cast<const float4*>(stage + row * WN + ((rc ^ sw(row)) << 2));
      }
      if (XNEXT) {   // this slab's rows, then the next slab's
#pragma unroll
        for (int p = 0; p < NB; ++p) x[p] = xn[p];
        if (b + 1 < TM) load_x(b + 1, xn);
      } else if (XLOAD) {   // the residual, or z
#pragma unroll
        for (int p = 0; p < NB; ++p) {
          const int m = mb + (p0 + p) * RPP;
          if (m < M && n_ok) x[p] = *reinterpret_cast<const float4*>(xsrc + (size_t)m * e.ldo + n);
        }
      }
      // LayerNorm-folded consumer: the batch's row statistics, loaded
      // together so their latencies overlap.
      float2 rs[NB];
      if (EPI == EPI_BIAS || EPI == EPI_BIAS_GELU) {
        if (fold_in) {
#pragma unroll
          for (int p = 0; p < NB; ++p) {
            const int m = min(mb + (p0 + p) * RPP, M - 1);
            rs[p] = *reinterpret_cast<const float2*>(e.row_stats + 2 * (size_t)m);
          }
        }
      }
#pragma unroll
      for (int p = 0; p < NB; ++p) {
        const int m = mb + (p0 + p) * RPP;
        if (m >= M || !n_ok) continue;
        if (EPI == EPI_PATCH) {
          epi_store4<EPI, OUT_BF16>(e, m, n, v[p].x, v[p].y, v[p].z, v[p].w);
          continue;
        }
        if (EPI == EPI_SCALE_BIAS) {
          const float4 y = make_float4(e.alpha * v[p].x + e.beta, e.alpha * v[p].y + e.beta,
                                       e.alpha * v[p].z + e.beta, e.alpha * v[p].w + e.beta);
          *reinterpret_cast<float4*>(static_cast<float*>(e.out) + (size_t)m * e.ldo + n) = y;
          if (e.out2) {   // BF16 copy
            u32x2 pk;
            pk.x = pack_bf16x2(y.x, y.y);
            pk.y = pack_bf16x2(y.z, y.w);
            *reinterpret_cast<u32x2*>(static_cast<bf16_t*>(e.out2) + (size_t)m * e.ldo + n) = pk;
          }
          continue;
        }
        if (EPI == EPI_DGELU) {
          dgelu_store4(e, m, n, v[p], x[p]);
          continue;
        }
        float4 y;
        if (fold_in) {
          const float2 st = rs[p];
          y = make_float4(ln_fold1(v[p].x, ws4.x, c14.x, bias4.x, st.x, st.y),
                          ln_fold1(v[p].y, ws4.y, c14.y, bias4.y, st.x, st.y),
                          ln_fold1(v[p].z, ws4.z, c14.z, bias4.z, st.x, st.y),
                          ln_fold1(v[p].w, ws4.w, c14.w, bias4.w, st.x, st.y));
        } else {
          y = make_float4(__builtin_fmaf(v[p].x, ws4.x, bias4.x),
                          __builtin_fmaf(v[p].y, ws4.y, bias4.y),
                          __builtin_fmaf(v[p].z, ws4.z, bias4.z),
                          __builtin_fmaf(v[p].w, ws4.w, bias4.w));
        }
        if (EPI == EPI_BIAS_RESID) {
          const float4 xn = make_float4(x[p].x + y.x, x[p].y + y.y, x[p].z + y.z, x[p].w + y.w);
          *reinterpret_cast<float4*>(static_cast<float*>(e.out) + (size_t)m * e.ldo + n) = xn;
          if (fold_out) {
            // u = bf16(x * gamma) and the (mean, M2) of the row's 32-column
            // group, which the 8 consecutive lanes rc = 8j .. 8j+7 hold
            // (all with the same row, so all active together).
            u32x2 pk;
            pk.x = pack_bf16x2(xn.x * g4.x, xn.y * g4.y);
            pk.y = pack_bf16x2(xn.z * g4.z, xn.w * g4.w);
            *reinterpret_cast<u32x2*>(e.u_out + (size_t)m * e.ldo + n) = pk;
            float sm = (xn.x + xn.y) + (xn.z + xn.w);
            sm += __shfl_xor(sm, 1, 64);
            sm += __shfl_xor(sm, 2, 64);
            sm += __shfl_xor(sm, 4, 64);
            const float mg = sm * (1.f / 32.f);
            const float d0 = xn.x - mg, d1 = xn.y - mg, d2 = xn.z - mg, d3 = xn.w - mg;
            float q = (d0 * d0 + d1 * d1) + (d2 * d2 + d3 * d3);
            q += __shfl_xor(q, 1, 64);
            q += __shfl_xor(q, 2, 64);
            q += __shfl_xor(q, 4, 64);
            if ((rc & 7) == 0)   // group-major: consecutive rows are adjacent
              *reinterpret_cast<float2*>(e.part_stats + ((size_t)(n >> 5) * M + m) * 2) =
                  make_float2(mg, q);
          }
          continue;
        }
        if (EPI == EPI_BIAS_F32) {
          *reinterpret_cast<float4*>(static_cast<float*>(e.out) + (size_t)m * e.ldo + n) = y;
          if (e.out2) gelu_out2_store4(e, m, n, y);
          continue;
        }
        if (EPI == EPI_BIAS_GELU) {
          y.x = gelu_poly(y.x); y.y = gelu_poly(y.y);
          y.z = gelu_poly(y.z); y.w = gelu_poly(y.w);
        }
        u32x2 pk;
        pk.x = pack_bf16x2(y.x, y.y);
        pk.y = pack_bf16x2(y.z, y.w);
        *reinterpret_cast<u32x2*>(static_cast<bf16_t*>(e.out) + (size_t)m * e.ldo + n) = pk;
      }
    }
  }
}



template <int BM, int BN, int WGM, int WGN, bool B_FP8, int RPM = 2, int ST = 2>
static hipError_t launch_bf16_dl(const bf16_t* A, int lda, const void* B, int ldb, int M,
                                 int N, int K, int op, const EpiArgs& e, hipStream_t s) {
  const int gm = (M + BM - 1) / BM, gn = (N + BN - 1) / BN;
  dim3 grid(gm * gn, op == OP_LOGITS && e.kc > 0 ? (K + e.kc - 1) / e.kc : 1),
      block(WGM * WGN * 64);
#define VL_GEMM_CASE(OP)                                                                  \
  case OP:                                                                                \
    hipLaunchKernelGGL((k_gemm_bf16_dl<BM, BN, WGM, WGN, B_FP8, OP, RPM, ST>), grid, block, \
                       0, s, A, lda, B, ldb, M, N, K, gm, gn, e);                         \
    break;
  switch (op) {
    VL_GEMM_CASE(OP_PATCH)
    VL_GEMM_CASE(OP_QKV)
    VL_GEMM_CASE(OP_OPROJ)
    VL_GEMM_CASE(OP_FC1)
    VL_GEMM_CASE(OP_FC2)
    VL_GEMM_CASE(OP_LOGITS)
    VL_GEMM_CASE(OP_FC1_PRE)
    VL_GEMM_CASE(OP_DGELU)
    default: return hipErrorInvalidValue;
  }
#undef VL_GEMM_CASE
  return hipGetLastError();
}


template <int BM, int BN, int WGM, int WGN, bool B_FP8>
static hipError_t launch_bf16(const bf16_t* A, int lda, const void* B, int ldb, int M, int N,
                              int K, int op, const EpiArgs& e, hipStream_t s) {
  dim3 grid((M + BM - 1) / BM, (N + BN - 1) / BN);
  dim3 block(WGM * WGN * 64);
#define VL_GEMM_CASE(OP)                                                                   \
  case OP:                                                                                 \
    hipLaunchKernelGGL((k_gemm_bf16<BM, BN, WGM, WGN, B_FP8, OP>), grid, block, 0, s, A, lda, \
                       B, ldb, M, N, K, e);                                                \
    break;
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

}  // namespace vl
