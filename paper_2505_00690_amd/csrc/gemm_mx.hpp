// MX-FP8 GEMM (OCP Microscaling Formats v1.0, MXFP8 with e4m3 elements):
// C[M,N] = A[M,K] . B[N,K]^T where both operands are e4m3 codes with one
// E8M0 scale (2^(e-127)) per 32 consecutive K elements of a row, applied
// inside v_mfma_scale_f32_32x32x64_f8f6f4 on gfx950.
//
// Tiles: rows of 128 K bytes, the same size, direct-to-LDS load pattern and
// chunk swizzle as the BF16 tiles (k_gemm_bf16_dl), so per K tile the load,
// LDS and MFMA-cycle budgets match the BF16 kernel while the MFMAs cover twice
// the K.  One K tile = two MFMA K steps of 64.  Operand lane layout of the
// MFMA (checked on the hardware with an in-bounds probe): lane l holds row
// l % 32; its 32 bytes are K [16g, 16g+16) then K [32+16g, 32+16g+16) of the
// 64-wide step (g = l / 32); its scale byte applies to K block g (32 wide).
//
// Scales are stored block-major, [K/128][rows][4] bytes, with the four blocks
// of a (row, K tile) in the order 0, 2, 1, 3: the 16-bit half g of that word
// then holds blocks g and 2 + g, i.e. the lane's scale for K steps 0 and 1,
// selected by the MFMA's (immediate) byte select.  A K tile's scales for a
// tile's rows are contiguous and load with the operand tiles.
#pragma once

#include "gemm_kernels.hpp"

namespace vl {

typedef int32_t i32x8 __attribute__((ext_vector_type(8)));
constexpr int MXK = 128;  // K elements (bytes) per LDS tile

// Wait until at most n of this wave's global loads are outstanding (n is
// wave-uniform; s_waitcnt takes an immediate).
__device__ __forceinline__ void wait_vm_le(int n) {
  switch (n) {
    case 0: asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); break;
    case 1: asm volatile("s_waitcnt vmcnt(1)" ::: "memory"); break;
    case 2: asm volatile("s_waitcnt vmcnt(2)" ::: "memory"); break;
    case 3: asm volatile("s_waitcnt vmcnt(3)" ::: "memory"); break;
    case 4: asm volatile("s_waitcnt vmcnt(4)" ::: "memory"); break;
    case 5: asm volatile("s_waitcnt vmcnt(5)" ::: "memory"); break;
    case 6: asm volatile("s_waitcnt vmcnt(6)" ::: "memory"); break;
    case 7: asm volatile("s_waitcnt vmcnt(7)" ::: "memory"); break;
    case 8: asm volatile("s_waitcnt vmcnt(8)" ::: "memory"); break;
    case 9: asm volatile("s_waitcnt vmcnt(9)" ::: "memory"); break;
    case 10: asm volatile("s_waitcnt vmcnt(10)" ::: "memory"); break;
    case 11: asm volatile("s_waitcnt vmcnt(11)" ::: "memory"); break;
    case 12: asm volatile("s_waitcnt vmcnt(12)" ::: "memory"); break;
    case 13: asm volatile("s_waitcnt vmcnt(13)" ::: "memory"); break;
    case 14: asm volatile("s_waitcnt vmcnt(14)" ::: "memory"); break;
    case 15: asm volatile("s_waitcnt vmcnt(15)" ::: "memory"); break;
    default: asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); break;
  }
}

template <int BM, int BN, int WGM, int WGN, int OP, int ST>
__global__ __launch_bounds__(WGM* WGN * 64)
__attribute__((amdgpu_waves_per_eu(WGM * WGN / 4, WGM * WGN / 4))) void k_gemm_mx(
    const uint8_t* __restrict__ A, const uint8_t* __restrict__ SA, const uint8_t* __restrict__ B,
    const uint8_t* __restrict__ SB, int M, int N, int K, int gm, int gn, EpiArgs e) {
  constexpr int EPI = OpEpi<OP>::kind;
  constexpr int NW = WGM * WGN;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int TM = WM / 32, TN = WN / 32;
  static_assert(WM % 32 == 0 && WN % 32 == 0, "wave tile must be whole 32x32 blocks");
  constexpr int GA = BM / 8, GB = BN / 8;          // 8-row groups per tile
  constexpr int IA = (GA + NW - 1) / NW, IB = (GB + NW - 1) / NW;
  static_assert(BM * 4 <= 1024 && BN * 4 <= 1024, "one load instruction per scale tile");
  static_assert(ST >= 2 && ST <= 4, "two to four K tiles in the LDS ring");
  constexpr int TILE_A = BM * MXK, TILE_B = BN * MXK, TILE_S = 1024;
  constexpr int LDS_AB = ST * (TILE_A + TILE_B + 2 * TILE_S);
  constexpr int LDS_EPI = NW * 32 * WN * 4;
  __shared__ __attribute__((aligned(1024))) char smem[LDS_AB > LDS_EPI ? LDS_AB : LDS_EPI];
  char* const sA = smem;
  char* const sB = smem + ST * TILE_A;
  char* const sSA = smem + ST * (TILE_A + TILE_B);
  char* const sSB = sSA + ST * TILE_S;

  int tm_, tn_;
  xcd_tile(gm, gn, 8, &tm_, &tn_);
  const int m0 = tm_ * BM, n0 = tn_ * BN;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WGN, wn = wave % WGN;
  const int KT = K / MXK;

  const i32x4 ra = buffer_rsrc(A + (size_t)m0 * K, (uint64_t)(M - m0) * K);
  const i32x4 rb = buffer_rsrc(B + (size_t)n0 * K, (uint64_t)(N - n0) * K);
  const i32x4 rsa = buffer_rsrc(SA, (uint64_t)KT * M * 4);
  const i32x4 rsb = buffer_rsrc(SB, (uint64_t)KT * N * 4);
  const int lrow = lane >> 3, lchunk = (lane & 7) ^ (lane >> 3);
  const uint32_t ldsA = lds_offset(sA), ldsB = lds_offset(sB);
  const uint32_t ldsSA = lds_offset(sSA), ldsSB = lds_offset(sSB);
  auto issue = [&](int buf, int kt) {
    const int k0 = kt * MXK;
#pragma unroll
    for (int i = 0; i < IA; ++i) {
      const int grp = wave + i * NW;
      if (GA % NW != 0 && grp >= GA) break;
      dma16(ra, ldsA + buf * TILE_A + grp * 8 * MXK,
            (grp * 8 + lrow) * K + ((lchunk ^ (grp & 7)) << 4), k0);
    }
#pragma unroll
    for (int i = 0; i < IB; ++i) {
      const int grp = wave + i * NW;
      if (GB % NW != 0 && grp >= GB) break;
      dma16(rb, ldsB + buf * TILE_B + grp * 8 * MXK,
            (grp * 8 + lrow) * K + ((lchunk ^ (grp & 7)) << 4), k0);
    }
    // Scale words of this K tile for the tile's rows (lanes past the rows
    // fetch neighbouring words into the unused rest of the 1 KB slot).
    // (offsets below 2^32: checked by the launcher)
    if (wave == 0)
      dma16(rsa, ldsSA + buf * TILE_S, (int)(((uint32_t)kt * M + m0) * 4u + lane * 16), 0);
    if (wave == NW - 1)
      dma16(rsb, ldsSB + buf * TILE_S, (int)(((uint32_t)kt * N + n0) * 4u + lane * 16), 0);
  };

  f32x16 acc[TN][TM];
#pragma unroll
  for (int a = 0; a < TN; ++a)
#pragma unroll
    for (int b = 0; b < TM; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;

  const int l32 = lane & 31, g = lane >> 5;
  // Fragment row byte offsets: logical chunk c = 4kk + 2h + g of a 128-byte
  // row sits at chunk c ^ f(row); with the lane's g and f folded in, the
  // offset for (kk, h) is base ^ ((4kk + 2h) << 4).
  int offA[TM], offB[TN];
#pragma unroll
  for (int b = 0; b < TM; ++b) {
    const int row = wm * WM + b * 32 + l32;
    offA[b] = row * MXK + ((g ^ swz_f(row)) << 4);
  }
#pragma unroll
  for (int a = 0; a < TN; ++a) {
    const int row = wn * WN + a * 32 + l32;
    offB[a] = row * MXK + ((g ^ swz_f(row)) << 4);
  }
  struct Frag {
    i32x8 w[TN], x[TM];
    int sw[TN], sx[TM];
  };
  Frag f0, f1;
  auto ldfrag = [&](Frag& f, int buf, int kk) {
    const char* tA = sA + buf * TILE_A;
    const char* tB = sB + buf * TILE_B;
    const char* tSA = sSA + buf * TILE_S;
    const char* tSB = sSB + buf * TILE_S;
#pragma unroll
    for (int a = 0; a < TN; ++a) {
      const u32x4 lo = *reinterpret_cast<const u32x4*>(tB + (offB[a] ^ ((4 * kk) << 4)));
      const u32x4 hi = *reinterpret_cast<const u32x4*>(tB + (offB[a] ^ ((4 * kk + 2) << 4)));
      f.w[a] = i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
      f.sw[a] = *reinterpret_cast<const uint16_t*>(tSB + (wn * WN + a * 32 + l32) * 4 + 2 * g);
    }
#pragma unroll
    for (int b = 0; b < TM; ++b) {
      const u32x4 lo = *reinterpret_cast<const u32x4*>(tA + (offA[b] ^ ((4 * kk) << 4)));
      const u32x4 hi = *reinterpret_cast<const u32x4*>(tA + (offA[b] ^ ((4 * kk + 2) << 4)));
      f.x[b] = i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
      f.sx[b] = *reinterpret_cast<const uint16_t*>(tSA + (wm * WM + b * 32 + l32) * 4 + 2 * g);
    }
  };
  // (weights are the MFMA's first operand, so lanes own activation rows and
  // the epilogue layout is the BF16 kernel's)
  auto mma0 = [&](const Frag& f) {
#pragma unroll
    for (int a = 0; a < TN; ++a)
#pragma unroll
      for (int b = 0; b < TM; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
            f.w[a], f.x[b], acc[a][b], 0, 0, 0, f.sw[a], 0, f.sx[b]);
  };
  auto mma1 = [&](const Frag& f) {
#pragma unroll
    for (int a = 0; a < TN; ++a)
#pragma unroll
      for (int b = 0; b < TM; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
            f.w[a], f.x[b], acc[a][b], 0, 0, 1, f.sw[a], 1, f.sx[b]);
  };
  constexpr int NF = 2 * (TN + TM) + (TN + TM), NM = TN * TM;  // reads: 2 per fragment + scale
  auto interleave = [&]() {
    constexpr int NG = NF < NM ? NF : NM;
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, (NF + NG - 1) / NG, 0);
    }
    if (NM > NG) __builtin_amdgcn_sched_group_barrier(0x008, NM - NG, 0);
  };

  // Global loads of one K tile by this wave: its operand row groups, plus
  // the scale tile for waves 0 (A) and NW - 1 (B).  Loads complete in issue
  // order, so "at most k tiles outstanding" is vmcnt <= k * n_ld.
  const int n_ld = (GA % NW == 0 || wave < GA % NW ? IA : IA - 1) +
                   (GB % NW == 0 || wave < GB % NW ? IB : IB - 1) + (wave == 0) +
                   (wave == NW - 1);
  // Loads run ST - 1 tiles ahead.  Tile kt + ST - 1 goes into the stage of
  // tile kt - 1, whose readers all passed the barrier of iteration kt - 1.
  for (int i = 0; i < ST - 1 && i < KT; ++i) issue(i, i);
  wait_vm_le(n_ld * (KT - 1 < ST - 2 ? KT - 1 : ST - 2));
  lds_barrier();
  ldfrag(f0, 0, 0);
  int cur = 0;
  for (int kt = 0; kt < KT; ++kt) {
    const int nxt = cur + 1 == ST ? 0 : cur + 1;
    if (kt + ST - 1 < KT) issue(cur == 0 ? ST - 1 : cur - 1, kt + ST - 1);
    ldfrag(f1, cur, 1);
    mma0(f0);
    interleave();
    // tile kt + 1 must have landed; later tiles may still be in flight
    const int ahead = KT - 2 - kt < ST - 2 ? KT - 2 - kt : ST - 2;
    wait_vm_le(ahead > 0 ? n_ld * ahead : 0);
    lds_barrier();
    ldfrag(f0, nxt, 0);   // next tile (stale on the last; never used)
    mma1(f1);
    interleave();
    cur = nxt;
  }

  // Epilogue: as in k_gemm_bf16_dl (scales were applied inside the MFMA).
  lds_barrier();
  constexpr int CPR = WN / 4;
  static_assert(CPR >= 8 && 64 % CPR == 0, "staging layout needs WN in {32, 64, 128}");
  static_assert(OP == OP_QKV || OP == OP_OPROJ || OP == OP_FC1 || OP == OP_FC2, "MXFP8 ops");
  auto swe = [](int r) { return CPR >= 16 ? (r & 15) : ((r >> 1) & 7); };
  constexpr int RPP = 64 / CPR;
  constexpr int NP = 32 / RPP;
  constexpr int NB = NP < 8 ? NP : 8;
  float* stage = reinterpret_cast<float*>(smem) + wave * 32 * WN;
  const int rc = lane % CPR, rr = lane / CPR;
  const int n = n0 + wn * WN + 4 * rc;
  const bool n_ok = n < N;
  float4 bias4 = make_float4(0.f, 0.f, 0.f, 0.f);
  if (n_ok) bias4 = *reinterpret_cast<const float4*>(e.bias + n);
  // Residual rows: slab b+1's are loaded before slab b's stores, so waiting
  // for them does not wait for those stores too (loads and stores share the
  // vector memory counter, in issue order).
  constexpr bool XNEXT = EPI == EPI_BIAS_RESID && NB == NP;
  float4 xn[NB];
  auto load_x = [&](int b, float4 (&dst)[NB]) {
#pragma unroll
    for (int p = 0; p < NB; ++p) {
      const int m = m0 + wm * WM + b * 32 + rr + p * RPP;
      if (m < M && n_ok)
        dst[p] = *reinterpret_cast<const float4*>(static_cast<const float*>(e.out) +
                                                  (size_t)m * e.ldo + n);
    }
  };
  if (XNEXT) load_x(0, xn);
#pragma unroll
  for (int b = 0; b < TM; ++b) {
#pragma unroll
    for (int a = 0; a < TN; ++a)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = a * 8 + 2 * q + g;
        *reinterpret_cast<float4*>(stage + l32 * WN + ((c ^ swe(l32)) << 2)) =
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
        v[p] = *reinterpret_cast<const float4*>(stage + row * WN + ((rc ^ swe(row)) << 2));
      }
      if (XNEXT) {
#pragma unroll
        for (int p = 0; p < NB; ++p) x[p] = xn[p];
        if (b + 1 < TM) load_x(b + 1, xn);
      } else if (EPI == EPI_BIAS_RESID) {
#pragma unroll
        for (int p = 0; p < NB; ++p) {
          const int m = mb + (p0 + p) * RPP;
          if (m < M && n_ok)
            x[p] = *reinterpret_cast<const float4*>(static_cast<const float*>(e.out) +
                                                    (size_t)m * e.ldo + n);
        }
      }
#pragma unroll
      for (int p = 0; p < NB; ++p) {
        const int m = mb + (p0 + p) * RPP;
        float4 y = make_float4(v[p].x + bias4.x, v[p].y + bias4.y, v[p].z + bias4.z,
                               v[p].w + bias4.w);
        if (OP == OP_FC1) {
          // GELU, then MXFP8 for the next GEMM: the 8 lanes of a 32-column
          // block share its amax (rows and column blocks are uniformly in
          // or out of range within such a group, so all lanes take part).
          y.x = gelu_poly(y.x); y.y = gelu_poly(y.y);
          y.z = gelu_poly(y.z); y.w = gelu_poly(y.w);
          const float amax =
              max8(fmaxf(fmaxf(fabsf(y.x), fabsf(y.y)), fmaxf(fabsf(y.z), fabsf(y.w))));
          const uint32_t sb = mx_scale_byte(amax);
          const uint32_t q = mx_pack4(y.x, y.y, y.z, y.w, mx_inv_scale(sb));
          if (m < M && n_ok) {
            *reinterpret_cast<uint32_t*>(static_cast<uint8_t*>(e.out) + (size_t)m * e.ldo + n) = q;
            if ((rc & 7) == 0) e.out_scale[mx_scale_off(m, n, e.scale_rows)] = (uint8_t)sb;
          }
          continue;
        }
        if (m >= M || !n_ok) continue;
        if (EPI == EPI_BIAS_RESID) {
          *reinterpret_cast<float4*>(static_cast<float*>(e.out) + (size_t)m * e.ldo + n) =
              make_float4(x[p].x + y.x, x[p].y + y.y, x[p].z + y.z, x[p].w + y.w);
          continue;
        }
        u32x2 pk;
        pk.x = pack_bf16x2(y.x, y.y);
        pk.y = pack_bf16x2(y.z, y.w);
        *reinterpret_cast<u32x2*>(static_cast<bf16_t*>(e.out) + (size_t)m * e.ldo + n) = pk;
      }
    }
  }
}

template <int BM, int BN, int WGM, int WGN, int ST = 2>
static hipError_t launch_mx(const uint8_t* A, const uint8_t* SA, const uint8_t* B,
                            const uint8_t* SB, int M, int N, int K, int op, const EpiArgs& e,
                            hipStream_t s) {
  if (K % MXK || N % 32) return hipErrorInvalidValue;
  // scale offsets are 32-bit buffer offsets (plus one 1 KB load past a row run)
  if ((uint64_t)(K / MXK) * ((uint64_t)(M > N ? M : N) + 256) * 4 >= (1ull << 32))
    return hipErrorInvalidValue;
  const int gm = (M + BM - 1) / BM, gn = (N + BN - 1) / BN;
  dim3 grid(gm * gn), block(WGM * WGN * 64);
#define VL_MX_CASE(OP)                                                                  \
  case OP:                                                                              \
    hipLaunchKernelGGL((k_gemm_mx<BM, BN, WGM, WGN, OP, ST>), grid, block, 0, s, A, SA, B, SB, \
                       M, N, K, gm, gn, e);                                             \
    break;
  switch (op) {
    VL_MX_CASE(OP_QKV)
    VL_MX_CASE(OP_OPROJ)
    VL_MX_CASE(OP_FC1)
    VL_MX_CASE(OP_FC2)
    default: return hipErrorInvalidValue;
  }
#undef VL_MX_CASE
  return hipGetLastError();
}

}  // namespace vl
