// Multi-head self-attention over a packed, variable-length token stream
// (scaled dot-product attention, Vaswani et al. 2017, Sec. 3.2.1 Eq. 1;
// attention is restricted to the tokens of one image).
//
// BF16 kernel (flash-style, MFMA).  A workgroup of four waves owns up to
// 128 queries of one (image, head); each wave owns 32 queries.  Key and value
// tiles of 64 tokens stream through a three-stage LDS ring by direct-to-LDS
// loads issued two tiles ahead; both are kept row-major (token x head dim,
// 16-byte chunks of a row XOR-permuted by a function of the row so the
// operand reads below are bank-conflict free).  Scores are computed
// transposed, S^T = K Q^T (v_mfma_f32_32x32x16_bf16), so a lane owns one
// query and 16 of the 32 keys of an MFMA block: row max and row sum of the
// online softmax are in-lane reductions plus one exchange with lane^32.  The
// output is accumulated transposed too, O^T += V^T P^T: P^T goes to the MFMA
// straight from the score registers (rounded to BF16) and the V^T operand is
// read from the row-major value tile with the LDS transpose read
// (ds_read_b64_tr_b16), which hands each lane one head-dim column at four
// tokens.  Softmax statistics stay in FP32; exponentials are exp2 of
// log2(e)-prescaled scores, and the running max is only raised when a tile
// exceeds it by more than 2^8 (the normaliser cancels the reference point;
// this bounds every exponential by 2^8 and makes rescaling rare).
//
// FP32 kernel: one thread per query, K/V tiles of 32 tokens in LDS, online
// softmax per tile; the plain FP32 baseline.
#include <type_traits>

#include "kernels.hpp"

namespace vl {

constexpr int ATT_Q = 128;   // queries per workgroup
constexpr int ATT_KV = 64;   // keys per LDS tile
constexpr int ATT_ST = 3;    // LDS ring stages
constexpr float ATT_TAU = 8.f;  // lazy-rescale threshold (log2 units)

// Row-major K / V tile of 64 tokens x HD BF16 (HD/8 16-byte chunks per row),
// chunk c of row r stored at position c ^ f(r).  Key tiles: f(r) =
// (r ^ (r >> 3)) & 7 for HD = 64, (r >> 2) & 3 for HD = 32, so 16
// consecutive rows read at one logical chunk (the K operand) hit distinct
// banks.  Value tiles: f(r) = r & 7 for HD = 64, no permutation for HD = 32;
// the four consecutive rows of one transpose read then hit distinct banks,
// and f depends only on r mod 8, so a lane's read offsets for all 16-row
// groups differ by immediates.
template <int HD, bool VALUE>
struct KvTile {
  static constexpr int NCH = HD / 8;
  static constexpr int ROWB = HD * 2;
  static constexpr int BYTES = 64 * ROWB;
  __device__ static int f(int r) {
    if (VALUE) return NCH == 8 ? (r & 7) : 0;
    return NCH == 8 ? ((r ^ (r >> 3)) & 7) : ((r >> 2) & 3);
  }
  __device__ static int off(int r, int chunk) { return r * ROWB + ((chunk ^ f(r)) << 4); }
};

typedef short s16x4 __attribute__((ext_vector_type(4)));

// MX = false: O is BF16 [T, D].  MX = true: O is MXFP8 for the output
// projection, codes [T, D] (out) and scales [D/128][T][4] (out_scale); a
// 32-column block of a head lies in one lane pair (lane, lane ^ 32).
// Work items are dealt XCD by XCD (xcd_linear): each XCD is given a
// contiguous range of (head, query block) items, in which the query blocks
// of one (image, head) are consecutive and share that image's key and value
// rows in the XCD's L2.

template <int HD, bool MX>
__global__ __launch_bounds__(256) void k_attn_bf16(const bf16_t* __restrict__ qkv,
                                                   void* __restrict__ out,
                                                   uint8_t* __restrict__ out_scale, int T_rows,
                                                   const ImgDesc* __restrict__ imgs,
                                                   const AttnItem* __restrict__ items,
                                                   int heads, int causal,
                                                   const BatchCounts* __restrict__ bc,
                                                   float* __restrict__ lse_out) {
  using T = KvTile<HD, false>;
  using TV = KvTile<HD, true>;
  constexpr int RPI = 1024 / T::ROWB;          // tile rows per 1 KB load instruction
  constexpr int LPW = ATT_KV / RPI / 4;        // K (and V) load instructions per wave
  static_assert(LPW >= 1 && LPW * RPI * 4 == ATT_KV, "tile / waves");
  __shared__ __attribute__((aligned(1024))) char sK[ATT_ST][T::BYTES];
  __shared__ __attribute__((aligned(1024))) char sV[ATT_ST][T::BYTES];

  int n_items = gridDim.x / heads, total = gridDim.x;
  if (bc) {   // capacity launch: the live item count comes from the device
    n_items = bc->n_items;
    total = n_items * heads;
    if (!xcd_live(blockIdx.x, total)) return;
  }
  const int wi = xcd_linear(blockIdx.x, total);
  const AttnItem it = items[wi % n_items];
  const int h = wi / n_items;
  const ImgDesc dsc = imgs[it.img];
  const int N = dsc.ntok;
  const int D = heads * HD;
  const int ld = 3 * D;
  const bf16_t* base = qkv + (size_t)dsc.tok_start * ld;
  const bf16_t* Qp = base + h * HD;

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l32 = lane & 31, g = lane >> 5;
  const int qw = it.q0 + wave * 32;            // first query of this wave
  const bool wave_active = qw < N;
  const int q = qw + l32;                      // this lane's query
  const int qc = min(q, N - 1);

  // Q^T operand fragments: lane (query, g) holds Q[q][16c + 8g .. +7].
  bf16x8 qf[HD / 16];
#pragma unroll
  for (int c = 0; c < HD / 16; ++c)
    qf[c] = *reinterpret_cast<const bf16x8*>(Qp + (size_t)qc * ld + 16 * c + 8 * g);
  // Wait for Q here with a wait the compiler sees (vmcnt(0)): otherwise its
  // wait-count pass, unaware of the direct-to-LDS loads below, keeps
  // waiting for Q at the score MFMAs of every tile and drains the prefetch.
  __builtin_amdgcn_s_waitcnt(0x0F70);

  // Direct-to-LDS loads: instruction i of this wave fills tile rows
  // R = (wave * LPW + i) * RPI ..; lane l takes row R + l / NCH and physical
  // chunk l % NCH, i.e. logical chunk (l % NCH) ^ f(row).  Rows past the
  // image read as zero (buffer bound).
  const i32x4 rk = buffer_rsrc(base + D + h * HD, (uint64_t)N * ld * 2);
  const i32x4 rv = buffer_rsrc(base + 2 * D + h * HD, (uint64_t)N * ld * 2);
  int goffK[LPW], goffV[LPW];
#pragma unroll
  for (int i = 0; i < LPW; ++i) {
    const int row = (wave * LPW + i) * RPI + lane / T::NCH;
    goffK[i] = row * ld * 2 + (((lane % T::NCH) ^ T::f(row)) << 4);
    goffV[i] = row * ld * 2 + (((lane % T::NCH) ^ TV::f(row)) << 4);
  }
  const uint32_t ldsK = lds_offset(&sK[0][0]), ldsV = lds_offset(&sV[0][0]);
  auto issue = [&](int kt, int st) {
    const int kb = kt * ATT_KV * ld * 2;
#pragma unroll
    for (int i = 0; i < LPW; ++i) {
      const uint32_t lo = st * T::BYTES + (wave * LPW + i) * 1024;
      dma16(rk, ldsK + lo, goffK[i] + kb, 0);
      dma16(rv, ldsV + lo, goffV[i] + kb, 0);
    }
  };

  // K operand (scores): lane reads row 32kb + l32, logical chunk 2c + g.
  int koff[2][HD / 16];
#pragma unroll
  for (int kb = 0; kb < 2; ++kb)
#pragma unroll
    for (int c = 0; c < HD / 16; ++c) koff[kb][c] = T::off(32 * kb + l32, 2 * c + g);
  // V^T operand: per 16-key chunk jj and 32-column block a, two transpose
  // reads.  Within each 16-lane group (g = group / 2, column half dh =
  // group % 2) lane i supplies the 8 bytes at token 16jj + 8hf + 4g + i/4
  // (hf = 0, 1 for the two reads), columns 32a + 16dh + 4(i%4) .. +3, and
  // receives column 32a + 16dh + i at the four tokens 16jj + 8hf + 4g +
  // (0..3): the same token order as the P^T fragment below.  With the value
  // tile's permutation the offset is vbase[a] + (16jj + 8hf) * row bytes.
  const int grp = lane >> 4, li = lane & 15;
  const int tg = grp >> 1, dh = grp & 1;
  int vbase[HD / 32];
#pragma unroll
  for (int a = 0; a < HD / 32; ++a) {
    const int col = 32 * a + 16 * dh + 4 * (li & 3);
    vbase[a] = TV::off(4 * tg + (li >> 2), col >> 3) + (col & 7) * 2;
  }

  const float sl2 = 1.4426950408889634f / sqrtf((float)HD);  // log2(e)/sqrt(d)
  float m_run = -INFINITY, l_run = 0.f;   // reference max (log2 units), sum
  f32x16 o[HD / 32];
#pragma unroll
  for (int a = 0; a < HD / 32; ++a)
#pragma unroll
    for (int r = 0; r < 16; ++r) o[a][r] = 0.f;

  // Causal: query q sees keys 0..q, so this workgroup needs keys below its
  // last query only.
  const int kv_end = causal ? min(N, it.q0 + ATT_Q) : N;
  const int KT = (kv_end + ATT_KV - 1) / ATT_KV;
  // One key tile; the ring stage is a compile-time constant so every LDS
  // address is a per-lane base plus an immediate.
  auto tile = [&](auto stage, int kt) {
    constexpr int st = decltype(stage)::value;
    // Tile kt must have landed; tile kt+1's loads may stay in flight.
    if (kt + 1 < KT) asm volatile("s_waitcnt vmcnt(%0)" ::"n"(2 * LPW) : "memory");
    else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    lds_barrier();
    // Stage (st+2)%3 held tile kt-1, whose readers all passed the barrier.
    if (kt + 2 < KT) issue(kt + 2, (st + 2) % ATT_ST);
    if (!wave_active) return;
    // With the causal mask a tile whose first key follows every query of the
    // wave contributes nothing (all its probabilities are 0); the wave only
    // keeps the ring moving for the other waves.
    if (causal && kt * ATT_KV > qw + 31) return;
    const char* tK = sK[st];
    // S^T blocks: s[kb][r] = S[key 32kb + 8(r/4) + 4g + r%4][query].
    f32x16 s[2];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
#pragma unroll
      for (int r = 0; r < 16; ++r) s[kb][r] = 0.f;
#pragma unroll
      for (int c = 0; c < HD / 16; ++c) {
        const bf16x8 kf = *reinterpret_cast<const bf16x8*>(tK + koff[kb][c]);
        s[kb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(kf, qf[c], s[kb], 0, 0, 0);
      }
    }
    // All V^T fragments of the tile, read while the softmax runs.
    bf16x8 vf[4][HD / 32];
#pragma unroll
    for (int jj = 0; jj < 4; ++jj)
#pragma unroll
      for (int a = 0; a < HD / 32; ++a) {
        typedef __attribute__((address_space(3))) s16x4 lds_s16x4;
        const uint32_t vb = ldsV + st * TV::BYTES + vbase[a] + 16 * jj * TV::ROWB;
        const s16x4 v0 = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)(uintptr_t)vb);
        const s16x4 v1 =
            __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)(uintptr_t)(vb + 8 * TV::ROWB));
        u32x4 vk;
        vk[0] = __builtin_bit_cast(u32x2, v0).x; vk[1] = __builtin_bit_cast(u32x2, v0).y;
        vk[2] = __builtin_bit_cast(u32x2, v1).x; vk[3] = __builtin_bit_cast(u32x2, v1).y;
        vf[jj][a] = __builtin_bit_cast(bf16x8, vk);
      }
    const int kbase = kt * ATT_KV;
    // keys past the sequence, and with a causal mask keys after the query
    // (every query keeps key 0, so no row is ever fully masked)
    const int kmax = causal ? min(N - 1, q) : N - 1;
    if (kbase + ATT_KV - 1 > (causal ? min(N - 1, qw) : N - 1)) {
#pragma unroll
      for (int kb = 0; kb < 2; ++kb)
#pragma unroll
        for (int r = 0; r < 16; ++r)
          if (kbase + kb * 32 + 8 * (r >> 2) + 4 * g + (r & 3) > kmax) s[kb][r] = -INFINITY;
    }
    // Row max: three-input maxima (inline so no NaN-quieting copies are
    // inserted; scores are never NaN).
    float mt = s[0][0];
#pragma unroll
    for (int i = 1; i < 31; i += 2) {
      const float x = s[i >> 4][i & 15], y = s[(i + 1) >> 4][(i + 1) & 15];
      asm("v_max3_f32 %0, %1, %2, %3" : "=v"(mt) : "v"(mt), "v"(x), "v"(y));
    }
    asm("v_max_f32 %0, %1, %2" : "=v"(mt) : "v"(mt), "v"(s[1][15]));
    mt = fmaxf(mt, __shfl_xor(mt, 32, 64)) * sl2;
    if (__any(mt > m_run + ATT_TAU)) {
      const float m_new = fmaxf(m_run, mt);
      const float alpha = __builtin_amdgcn_exp2f(m_run - m_new);
      l_run *= alpha;
#pragma unroll
      for (int a = 0; a < HD / 32; ++a)
#pragma unroll
        for (int r = 0; r < 16; ++r) o[a][r] *= alpha;
      m_run = m_new;
    }
    const float nm = -m_run;
    float ls0 = 0.f, ls1 = 0.f;
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float p = __builtin_amdgcn_exp2f(fmaf(s[kb][r], sl2, nm));
        s[kb][r] = p;
        if (r & 1) ls1 += p; else ls0 += p;
      }
    l_run += ls0 + ls1;
    // O^T += V^T P^T over four 16-key chunks jj; chunk jj = 2kb + hh uses
    // s[kb][8hh .. 8hh+7]: keys 16jj + 8(e/4) + 4g + e%4 for element e.
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int kb = jj >> 1, hh = jj & 1;
      u32x4 pk;
#pragma unroll
      for (int w = 0; w < 4; ++w)
        pk[w] = pack_bf16x2(s[kb][8 * hh + 2 * w], s[kb][8 * hh + 2 * w + 1]);
      const bf16x8 pf = __builtin_bit_cast(bf16x8, pk);
#pragma unroll
      for (int a = 0; a < HD / 32; ++a)
        o[a] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(vf[jj][a], pf, o[a], 0, 0, 0);
    }
  };

  issue(0, 0);
  if (KT > 1) issue(1, 1);
  for (int kt = 0; kt < KT; kt += ATT_ST) {
    tile(std::integral_constant<int, 0>(), kt);
    if (kt + 1 < KT) tile(std::integral_constant<int, 1>(), kt + 1);
    if (kt + 2 < KT) tile(std::integral_constant<int, 2>(), kt + 2);
  }
  if (!wave_active || q >= N) return;
  const float lt = l_run + __shfl_xor(l_run, 32, 64);
  const float inv = 1.f / lt;
  if (lse_out && g == 0) lse_out[(size_t)(dsc.tok_start + q) * heads + h] = m_run + log2f(lt);
  if constexpr (MX) {
    const int row = dsc.tok_start + q;
    uint8_t* op = static_cast<uint8_t*>(out) + (size_t)row * D + h * HD;
#pragma unroll
    for (int a = 0; a < HD / 32; ++a) {
      // |o * inv| is largest where |o| is (rounding is monotonic).
      float am = 0.f;
#pragma unroll
      for (int r = 0; r < 16; ++r) am = fmaxf(am, fabsf(o[a][r]));
      am = fmaxf(am, __shfl_xor(am, 32, 64)) * inv;
      const uint32_t sb = mx_scale_byte(am);
      const float si = mx_inv_scale(sb);
#pragma unroll
      for (int rq = 0; rq < 4; ++rq) {
        const int d = a * 32 + 8 * rq + 4 * g;
        *reinterpret_cast<uint32_t*>(op + d) =
            mx_pack4(o[a][4 * rq + 0] * inv, o[a][4 * rq + 1] * inv, o[a][4 * rq + 2] * inv,
                     o[a][4 * rq + 3] * inv, si);
      }
      if (g == 0) out_scale[mx_scale_off(row, h * HD + a * 32, T_rows)] = (uint8_t)sb;
    }
    return;
  }
  bf16_t* op = static_cast<bf16_t*>(out) + (size_t)(dsc.tok_start + q) * D + h * HD;
#pragma unroll
  for (int a = 0; a < HD / 32; ++a)
#pragma unroll
    for (int rq = 0; rq < 4; ++rq) {
      const int d = a * 32 + 8 * rq + 4 * g;
      u32x2 pk;
      pk.x = pack_bf16x2(o[a][4 * rq + 0] * inv, o[a][4 * rq + 1] * inv);
      pk.y = pack_bf16x2(o[a][4 * rq + 2] * inv, o[a][4 * rq + 3] * inv);
      *reinterpret_cast<u32x2*>(op + d) = pk;
    }
}

// ------------------------------------------------ BF16, K/V resident in LDS
// For images of 129 .. 64 NT tokens at head width 64: one workgroup of eight
// waves per (image, head) loads that head's keys and values into LDS once (NT
// tiles of 64 tokens, 16 KB per tile pair; NT = 10 fills the 160 KB) and
// runs every query of the image against them, 32 queries per wave at a time.
// The first pass (queries 0 .. 255) consumes the tiles as they land, loads
// issued two tiles ahead as in the streaming kernel; later passes find all
// tiles resident.  Each query's arithmetic (score MFMAs, lazy rescale,
// exponentials, P^T V^T MFMAs, in key-tile order) is the streaming kernel's,
// so the outputs are bitwise the same; what changes is that keys and values
// cross from L2 into LDS once per (image, head) instead of once per
// 128-query block.
constexpr int RES_W = 8;   // waves per resident workgroup

template <int NT, bool MX>
__global__ __launch_bounds__(RES_W * 64) void k_attn_bf16_res(
    const bf16_t* __restrict__ qkv, void* __restrict__ out, uint8_t* __restrict__ out_scale,
    int T_rows, const ImgDesc* __restrict__ imgs, const int* __restrict__ res_imgs, int heads,
    const BatchCounts* __restrict__ bc, float* __restrict__ lse_out) {
  constexpr int HD = 64;
  using T = KvTile<HD, false>;
  using TV = KvTile<HD, true>;
  constexpr int RPI = 1024 / T::ROWB;          // tile rows per 1 KB load instruction
  constexpr int LPW = ATT_KV / RPI / RES_W;    // K (and V) load instructions per wave per tile
  static_assert(LPW >= 1 && LPW * RPI * RES_W == ATT_KV, "tile / waves");
  __shared__ __attribute__((aligned(1024))) char sK[NT][T::BYTES];
  __shared__ __attribute__((aligned(1024))) char sV[NT][T::BYTES];

  int n_res = gridDim.x / heads, total = gridDim.x;
  if (bc) {   // capacity launch: the live image count comes from the device
    n_res = bc->n_res;
    total = n_res * heads;
    if (!xcd_live(blockIdx.x, total)) return;
  }
  const int wi = xcd_linear(blockIdx.x, total);
  const int img = res_imgs[wi % n_res];
  const int h = wi / n_res;
  const ImgDesc dsc = imgs[img];
  const int N = dsc.ntok;
  const int D = heads * HD;
  const int ld = 3 * D;
  const bf16_t* base = qkv + (size_t)dsc.tok_start * ld;
  const bf16_t* Qp = base + h * HD;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l32 = lane & 31, g = lane >> 5;

  const i32x4 rk = buffer_rsrc(base + D + h * HD, (uint64_t)N * ld * 2);
  const i32x4 rv = buffer_rsrc(base + 2 * D + h * HD, (uint64_t)N * ld * 2);
  int goffK[LPW], goffV[LPW];
#pragma unroll
  for (int i = 0; i < LPW; ++i) {
    const int row = (wave * LPW + i) * RPI + lane / T::NCH;
    goffK[i] = row * ld * 2 + (((lane % T::NCH) ^ T::f(row)) << 4);
    goffV[i] = row * ld * 2 + (((lane % T::NCH) ^ TV::f(row)) << 4);
  }
  const uint32_t ldsK = lds_offset(&sK[0][0]), ldsV = lds_offset(&sV[0][0]);
  auto issue = [&](int kt) {
    const int kb = kt * ATT_KV * ld * 2;
#pragma unroll
    for (int i = 0; i < LPW; ++i) {
      const uint32_t lo = kt * T::BYTES + (wave * LPW + i) * 1024;
      dma16(rk, ldsK + lo, goffK[i] + kb, 0);
      dma16(rv, ldsV + lo, goffV[i] + kb, 0);
    }
  };
  int koff[2][HD / 16];
#pragma unroll
  for (int kb = 0; kb < 2; ++kb)
#pragma unroll
    for (int c = 0; c < HD / 16; ++c) koff[kb][c] = T::off(32 * kb + l32, 2 * c + g);
  const int grp = lane >> 4, li = lane & 15;
  const int tg = grp >> 1, dh = grp & 1;
  int vbase[HD / 32];
#pragma unroll
  for (int a = 0; a < HD / 32; ++a) {
    const int col = 32 * a + 16 * dh + 4 * (li & 3);
    vbase[a] = TV::off(4 * tg + (li >> 2), col >> 3) + (col & 7) * 2;
  }
  const float sl2 = 1.4426950408889634f / sqrtf((float)HD);
  const int KT = (N + ATT_KV - 1) / ATT_KV;    // <= NT (checked by the launcher)

  // One 32-query chunk of this wave against key tile kt (resident in slot kt).
  auto tile = [&](int kt, const bf16x8* qf, f32x16* o, float& m_run, float& l_run, int q) {
    const char* tK = sK[kt];
    f32x16 s[2];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
#pragma unroll
      for (int r = 0; r < 16; ++r) s[kb][r] = 0.f;
#pragma unroll
      for (int c = 0; c < HD / 16; ++c) {
        const bf16x8 kf = *reinterpret_cast<const bf16x8*>(tK + koff[kb][c]);
        s[kb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(kf, qf[c], s[kb], 0, 0, 0);
      }
    }
    bf16x8 vf[4][HD / 32];
#pragma unroll
    for (int jj = 0; jj < 4; ++jj)
#pragma unroll
      for (int a = 0; a < HD / 32; ++a) {
        typedef __attribute__((address_space(3))) s16x4 lds_s16x4;
        const uint32_t vb = ldsV + kt * TV::BYTES + vbase[a] + 16 * jj * TV::ROWB;
        const s16x4 v0 = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)(uintptr_t)vb);
        const s16x4 v1 =
            __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)(uintptr_t)(vb + 8 * TV::ROWB));
        u32x4 vk;
        vk[0] = __builtin_bit_cast(u32x2, v0).x; vk[1] = __builtin_bit_cast(u32x2, v0).y;
        vk[2] = __builtin_bit_cast(u32x2, v1).x; vk[3] = __builtin_bit_cast(u32x2, v1).y;
        vf[jj][a] = __builtin_bit_cast(bf16x8, vk);
      }
    const int kbase = kt * ATT_KV;
    if (kbase + ATT_KV - 1 > N - 1) {
#pragma unroll
      for (int kb = 0; kb < 2; ++kb)
#pragma unroll
        for (int r = 0; r < 16; ++r)
          if (kbase + kb * 32 + 8 * (r >> 2) + 4 * g + (r & 3) > N - 1) s[kb][r] = -INFINITY;
    }
    float mt = s[0][0];
#pragma unroll
    for (int i = 1; i < 31; i += 2) {
      const float x = s[i >> 4][i & 15], y = s[(i + 1) >> 4][(i + 1) & 15];
      asm("v_max3_f32 %0, %1, %2, %3" : "=v"(mt) : "v"(mt), "v"(x), "v"(y));
    }
    asm("v_max_f32 %0, %1, %2" : "=v"(mt) : "v"(mt), "v"(s[1][15]));
    mt = fmaxf(mt, __shfl_xor(mt, 32, 64)) * sl2;
    if (__any(mt > m_run + ATT_TAU)) {
      const float m_new = fmaxf(m_run, mt);
      const float alpha = __builtin_amdgcn_exp2f(m_run - m_new);
      l_run *= alpha;
#pragma unroll
      for (int a = 0; a < HD / 32; ++a)
#pragma unroll
        for (int r = 0; r < 16; ++r) o[a][r] *= alpha;
      m_run = m_new;
    }
    const float nm = -m_run;
    float ls0 = 0.f, ls1 = 0.f;
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float p = __builtin_amdgcn_exp2f(fmaf(s[kb][r], sl2, nm));
        s[kb][r] = p;
        if (r & 1) ls1 += p; else ls0 += p;
      }
    l_run += ls0 + ls1;
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int kb = jj >> 1, hh = jj & 1;
      u32x4 pk;
#pragma unroll
      for (int w = 0; w < 4; ++w)
        pk[w] = pack_bf16x2(s[kb][8 * hh + 2 * w], s[kb][8 * hh + 2 * w + 1]);
      const bf16x8 pf = __builtin_bit_cast(bf16x8, pk);
#pragma unroll
      for (int a = 0; a < HD / 32; ++a)
        o[a] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(vf[jj][a], pf, o[a], 0, 0, 0);
    }
  };
  auto store = [&](const f32x16* o, float m_run, float l_run, int q) {
    const float lt = l_run + __shfl_xor(l_run, 32, 64);
    if (q >= N) return;
    const float inv = 1.f / lt;
    if (lse_out && g == 0) lse_out[(size_t)(dsc.tok_start + q) * heads + h] = m_run + log2f(lt);
    if constexpr (MX) {
      const int row = dsc.tok_start + q;
      uint8_t* op = static_cast<uint8_t*>(out) + (size_t)row * D + h * HD;
#pragma unroll
      for (int a = 0; a < HD / 32; ++a) {
        float am = 0.f;
#pragma unroll
        for (int r = 0; r < 16; ++r) am = fmaxf(am, fabsf(o[a][r]));
        am = fmaxf(am, __shfl_xor(am, 32, 64)) * inv;
        const uint32_t sb = mx_scale_byte(am);
        const float si = mx_inv_scale(sb);
#pragma unroll
        for (int rq = 0; rq < 4; ++rq) {
          const int d = a * 32 + 8 * rq + 4 * g;
          *reinterpret_cast<uint32_t*>(op + d) =
              mx_pack4(o[a][4 * rq + 0] * inv, o[a][4 * rq + 1] * inv, o[a][4 * rq + 2] * inv,
                       o[a][4 * rq + 3] * inv, si);
        }
        if (g == 0) out_scale[mx_scale_off(row, h * HD + a * 32, T_rows)] = (uint8_t)sb;
      }
    } else {
      bf16_t* op = static_cast<bf16_t*>(out) + (size_t)(dsc.tok_start + q) * D + h * HD;
#pragma unroll
      for (int a = 0; a < HD / 32; ++a)
#pragma unroll
        for (int rq = 0; rq < 4; ++rq) {
          const int d = a * 32 + 8 * rq + 4 * g;
          u32x2 pk;
          pk.x = pack_bf16x2(o[a][4 * rq + 0] * inv, o[a][4 * rq + 1] * inv);
          pk.y = pack_bf16x2(o[a][4 * rq + 2] * inv, o[a][4 * rq + 3] * inv);
          *reinterpret_cast<u32x2*>(op + d) = pk;
        }
    }
  };
  auto load_q = [&](bf16x8* qf, int q) {
    const int qc = min(q, N - 1);
#pragma unroll
    for (int c = 0; c < HD / 16; ++c)
      qf[c] = *reinterpret_cast<const bf16x8*>(Qp + (size_t)qc * ld + 16 * c + 8 * g);
  };

  // Pass 1: queries 0 .. 255 (chunk = wave) while the tiles arrive.
  {
    bf16x8 qf[HD / 16];
    const int q = 32 * wave + l32;
    const bool active = 32 * wave < N;
    load_q(qf, q);
    // Q has landed before the tile loads are issued (a wait the compiler
    // sees, so it does not wait for Q again at every tile's MFMAs).
    __builtin_amdgcn_s_waitcnt(0x0F70);
    issue(0);
    if (KT > 1) issue(1);
    float m_run = -INFINITY, l_run = 0.f;
    f32x16 o[HD / 32];
#pragma unroll
    for (int a = 0; a < HD / 32; ++a)
#pragma unroll
      for (int r = 0; r < 16; ++r) o[a][r] = 0.f;
    for (int kt = 0; kt < KT; ++kt) {
      if (kt + 1 < KT) asm volatile("s_waitcnt vmcnt(%0)" ::"n"(2 * LPW) : "memory");
      else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      lds_barrier();
      if (kt + 2 < KT) issue(kt + 2);
      if (active) tile(kt, qf, o, m_run, l_run, q);
    }
    if (active) store(o, m_run, l_run, q);
  }
  // Later passes: every tile resident; chunks RES_W .. of 32 queries.
  for (int c0 = 32 * RES_W; c0 < N; c0 += 32 * RES_W) {
    const int qw = c0 + 32 * wave;
    if (qw >= N) break;
    const int q = qw + l32;
    bf16x8 qf[HD / 16];
    load_q(qf, q);
    float m_run = -INFINITY, l_run = 0.f;
    f32x16 o[HD / 32];
#pragma unroll
    for (int a = 0; a < HD / 32; ++a)
#pragma unroll
      for (int r = 0; r < 16; ++r) o[a][r] = 0.f;
    for (int kt = 0; kt < KT; ++kt) tile(kt, qf, o, m_run, l_run, q);
    store(o, m_run, l_run, q);
  }
}

// Images the resident kernel takes: more tokens than one 128-query block
// (fewer already read their keys once) and at most 64 NT with NT = 10.
constexpr int RES_MIN_TOKENS = ATT_Q + 1, RES_MAX_TILES = 10;

template <bool MX>
static hipError_t launch_res(const bf16_t* qkv, void* out, uint8_t* out_scale, int T,
                             const ImgDesc* imgs, const int* res_imgs, int n_res, int max_tiles,
                             int heads, hipStream_t s, const BatchCounts* bc, float* lse_out) {
  dim3 grid(n_res * heads), block(RES_W * 64);
  if (max_tiles <= 4)
    hipLaunchKernelGGL((k_attn_bf16_res<4, MX>), grid, block, 0, s, qkv, out, out_scale, T, imgs,
                       res_imgs, heads, bc, lse_out);
  else if (max_tiles <= 6)
    hipLaunchKernelGGL((k_attn_bf16_res<6, MX>), grid, block, 0, s, qkv, out, out_scale, T, imgs,
                       res_imgs, heads, bc, lse_out);
  else if (max_tiles <= 8)
    hipLaunchKernelGGL((k_attn_bf16_res<8, MX>), grid, block, 0, s, qkv, out, out_scale, T, imgs,
                       res_imgs, heads, bc, lse_out);
  else if (max_tiles <= RES_MAX_TILES)
    hipLaunchKernelGGL((k_attn_bf16_res<RES_MAX_TILES, MX>), grid, block, 0, s, qkv, out,
                       out_scale, T, imgs, res_imgs, heads, bc, lse_out);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t attention_bf16_resident(const bf16_t* qkv, void* out, uint8_t* out_scale, bool mx,
                                   int T, const ImgDesc* imgs, const int* res_imgs, int n_res,
                                   int max_tiles, int heads, int head_dim, hipStream_t s,
                                   const BatchCounts* bc, float* lse_out) {
  if (n_res <= 0) return hipSuccess;
  if (head_dim != 64) return hipErrorInvalidValue;
  return mx ? launch_res<true>(qkv, out, out_scale, T, imgs, res_imgs, n_res, max_tiles, heads, s,
                               bc, nullptr)
            : launch_res<false>(qkv, out, out_scale, T, imgs, res_imgs, n_res, max_tiles, heads,
                                s, bc, lse_out);
}

// ----------------------------------------------------------------- FP32
constexpr int F32_KV = 32;

template <int HD>
__global__ __launch_bounds__(ATT_Q) void k_attn_f32(const float* __restrict__ qkv,
                                                    float* __restrict__ out,
                                                    const ImgDesc* __restrict__ imgs,
                                                    const AttnItem* __restrict__ items,
                                                    int heads, int causal) {
  __shared__ float sK[F32_KV][HD];
  __shared__ float sV[F32_KV][HD];
  const AttnItem it = items[blockIdx.x];
  const int h = blockIdx.y;
  const ImgDesc dsc = imgs[it.img];
  const int N = dsc.ntok;
  const int D = heads * HD, ld = 3 * D;
  const float* base = qkv + (size_t)dsc.tok_start * ld;
  const int tid = threadIdx.x;
  const int q = it.q0 + tid;
  const int qc = min(q, N - 1);
  float qv[HD], o[HD];
#pragma unroll
  for (int d = 0; d < HD; d += 4) {
    const float4 x = *reinterpret_cast<const float4*>(base + (size_t)qc * ld + h * HD + d);
    qv[d] = x.x; qv[d + 1] = x.y; qv[d + 2] = x.z; qv[d + 3] = x.w;
    o[d] = o[d + 1] = o[d + 2] = o[d + 3] = 0.f;
  }
  const float sc = 1.f / sqrtf((float)HD);
  float m_run = -INFINITY, l_run = 0.f;
  const int kv_end = causal ? min(N, it.q0 + ATT_Q) : N;
  const int kmax = causal ? min(N - 1, q) : N - 1;   // last key this query sees
  for (int k0 = 0; k0 < kv_end; k0 += F32_KV) {
    __syncthreads();
    for (int idx = tid; idx < F32_KV * HD / 4; idx += ATT_Q) {
      const int key = idx / (HD / 4), d = (idx % (HD / 4)) * 4;
      const int kk = min(k0 + key, N - 1);
      *reinterpret_cast<float4*>(&sK[key][d]) =
          *reinterpret_cast<const float4*>(base + (size_t)kk * ld + D + h * HD + d);
      *reinterpret_cast<float4*>(&sV[key][d]) =
          *reinterpret_cast<const float4*>(base + (size_t)kk * ld + 2 * D + h * HD + d);
    }
    __syncthreads();
    float s[F32_KV];
    float mt = -INFINITY;
#pragma unroll
    for (int j = 0; j < F32_KV; ++j) {
      float a = 0.f;
#pragma unroll
      for (int d = 0; d < HD; ++d) a = fmaf(qv[d], sK[j][d], a);
      s[j] = (k0 + j <= kmax) ? a * sc : -INFINITY;
      mt = fmaxf(mt, s[j]);
    }
    const float m_new = fmaxf(m_run, mt);
    const float alpha = expf(m_run - m_new);
    l_run *= alpha;
#pragma unroll
    for (int d = 0; d < HD; ++d) o[d] *= alpha;
#pragma unroll
    for (int j = 0; j < F32_KV; ++j) {
      const float p = expf(s[j] - m_new);
      l_run += p;
#pragma unroll
      for (int d = 0; d < HD; ++d) o[d] = fmaf(p, sV[j][d], o[d]);
    }
    m_run = m_new;
  }
  if (q >= N) return;
  const float inv = 1.f / l_run;
  float* op = out + (size_t)(dsc.tok_start + q) * D + h * HD;
#pragma unroll
  for (int d = 0; d < HD; d += 4)
    *reinterpret_cast<float4*>(op + d) =
        make_float4(o[d] * inv, o[d + 1] * inv, o[d + 2] * inv, o[d + 3] * inv);
}

// ------------------------------------------------ attention pooling (MAP)
// One learned query per head over all tokens of an image: s_j = q_h . K_jh /
// sqrt(d), p = softmax_j(s), O_h = sum_j p_j V_jh (FP32 arithmetic).  kv is
// [T, 2D] with K in columns 0..D-1 and V in D..2D-1, BF16 or FP32.  One
// workgroup of 256 threads per (image, head): scores in LDS, then 256/d
// groups of d threads sum strided token subsets of p_j V_j.
template <typename TKV>
__global__ __launch_bounds__(256) void k_map_attn(const TKV* __restrict__ kv,
                                                  const float* __restrict__ q,
                                                  const ImgDesc* __restrict__ imgs, int heads,
                                                  int hd, float* __restrict__ out) {
  __shared__ float sp[1025];
  __shared__ float sq[64];
  __shared__ float red[4];
  __shared__ float part[256];
  const ImgDesc d = imgs[blockIdx.x];
  const int h = blockIdx.y, tid = threadIdx.x;
  const int N = d.ntok, D = heads * hd, ld = 2 * D;
  auto ld_f = [](const TKV* p) {
    if constexpr (sizeof(TKV) == 2) return bf16_bits_to_f32(*reinterpret_cast<const uint16_t*>(p));
    else return static_cast<float>(*p);
  };
  if (tid < hd) sq[tid] = q[h * hd + tid];
  __syncthreads();
  const TKV* base = kv + (size_t)d.tok_start * ld;
  const float sc = 1.f / sqrtf((float)hd);
  float mx = -INFINITY;
  for (int j = tid; j < N; j += 256) {
    const TKV* kr = base + (size_t)j * ld + h * hd;
    float a = 0.f;
    for (int c = 0; c < hd; ++c) a = fmaf(sq[c], ld_f(kr + c), a);
    sp[j] = a * sc;
    mx = fmaxf(mx, a * sc);
  }
  mx = wave_max(mx);
  if ((tid & 63) == 0) red[tid >> 6] = mx;
  __syncthreads();
  mx = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  __syncthreads();
  float sum = 0.f;
  for (int j = tid; j < N; j += 256) {
    const float p = expf(sp[j] - mx);
    sp[j] = p;
    sum += p;
  }
  sum = wave_sum(sum);
  if ((tid & 63) == 0) red[tid >> 6] = sum;
  __syncthreads();
  sum = (red[0] + red[1]) + (red[2] + red[3]);
  const int G = 256 / hd, grp = tid / hd, c = tid % hd;
  float acc = 0.f;
  if (grp < G)
    for (int j = grp; j < N; j += G) acc = fmaf(sp[j], ld_f(base + (size_t)j * ld + D + h * hd + c), acc);
  part[tid] = acc;
  __syncthreads();
  if (tid < hd) {
    float o = 0.f;
    for (int g = 0; g < G; ++g) o += part[g * hd + tid];
    out[(size_t)blockIdx.x * D + h * hd + tid] = o / sum;
  }
}

hipError_t map_attention(const void* kv, bool kv_bf16, const float* q, const ImgDesc* imgs,
                         int n_imgs, int heads, int head_dim, float* out, hipStream_t s) {
  if (n_imgs <= 0) return hipSuccess;
  if (head_dim > 64 || 256 % head_dim) return hipErrorInvalidValue;
  dim3 grid(n_imgs, heads), block(256);
  if (kv_bf16)
    hipLaunchKernelGGL(k_map_attn<bf16_t>, grid, block, 0, s, static_cast<const bf16_t*>(kv), q,
                       imgs, heads, head_dim, out);
  else
    hipLaunchKernelGGL(k_map_attn<float>, grid, block, 0, s, static_cast<const float*>(kv), q,
                       imgs, heads, head_dim, out);
  return hipGetLastError();
}

hipError_t attention_bf16(const bf16_t* qkv, bf16_t* o, const ImgDesc* imgs,
                          const AttnItem* items, int n_items, int heads, int head_dim,
                          bool causal, hipStream_t s, const BatchCounts* bc, float* lse_out) {
  if (n_items <= 0) return hipSuccess;
  dim3 grid(n_items * heads), block(256);
  if (head_dim == 64)
    hipLaunchKernelGGL((k_attn_bf16<64, false>), grid, block, 0, s, qkv, o, nullptr, 0, imgs,
                       items, heads, (int)causal, bc, lse_out);
  else if (head_dim == 32)
    hipLaunchKernelGGL((k_attn_bf16<32, false>), grid, block, 0, s, qkv, o, nullptr, 0, imgs,
                       items, heads, (int)causal, bc, lse_out);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t attention_bf16_mx(const bf16_t* qkv, uint8_t* codes, uint8_t* scales, int T,
                             const ImgDesc* imgs, const AttnItem* items, int n_items,
                             int heads, int head_dim, bool causal, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  dim3 grid(n_items * heads), block(256);
  if (head_dim == 64)
    hipLaunchKernelGGL((k_attn_bf16<64, true>), grid, block, 0, s, qkv, codes, scales, T, imgs,
                       items, heads, (int)causal, nullptr, nullptr);
  else if (head_dim == 32)
    hipLaunchKernelGGL((k_attn_bf16<32, true>), grid, block, 0, s, qkv, codes, scales, T, imgs,
                       items, heads, (int)causal, nullptr, nullptr);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t attention_f32(const float* qkv, float* o, const ImgDesc* imgs,
                         const AttnItem* items, int n_items, int heads, int head_dim,
                         bool causal, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  dim3 grid(n_items, heads), block(ATT_Q);
  if (head_dim == 64)
    hipLaunchKernelGGL(k_attn_f32<64>, grid, block, 0, s, qkv, o, imgs, items, heads,
                       (int)causal);
  else if (head_dim == 32)
    hipLaunchKernelGGL(k_attn_f32<32>, grid, block, 0, s, qkv, o, imgs, items, heads,
                       (int)causal);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace vl
