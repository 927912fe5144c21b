// Multi-head self-attention over a packed, variable-length token stream
// (scaled dot-product attention, Vaswani et al. 2017, Sec. 3.2.1 Eq. 1;
// attention is restricted to the tokens of one image).
//
// BF16 kernel (flash-style, MFMA).  A workgroup of four waves owns up to
// 128 queries of one (image, head); each wave owns 32 queries.  Keys and
// values stream through LDS in tiles of 64 tokens (double buffered, the next
// tile's global loads issued before the current tile's MFMAs).  Scores are
// computed transposed, S^T = K Q^T (v_mfma_f32_32x32x16_bf16), so a lane owns
// one query and 16 of the 32 keys of an MFMA block: the row max and row sum of
// the online softmax are in-lane reductions plus one exchange with lane^32.
// The output is accumulated transposed too, O^T += V^T P^T, so P^T is fed to
// the MFMA straight from the score registers (rounded to BF16) and the
// per-query rescale factor is lane-local.  V is written to LDS transposed
// (d-major) for that operand.  Softmax statistics stay in FP32; exponentials
// are exp2 of log2(e)-prescaled scores.
//
// FP32 kernel: one thread per query, K/V tiles of 32 tokens in LDS, online
// softmax per tile; the plain FP32 baseline.
#include "kernels.hpp"

namespace vl {

constexpr int ATT_Q = 128;   // queries per workgroup
constexpr int ATT_KV = 64;   // keys per LDS tile

// sK[key][HD]: 16-B chunks of a row swizzled; for HD = 64 by
// (key ^ (key >> 3)) & 7, which keeps 8 (or 16) consecutive keys read at one
// logical chunk on distinct banks; for HD = 32 by key & 3.
template <int HD>
__device__ __forceinline__ int k_off(int key, int chunk) {
  constexpr int NC = HD / 8;
  const int f = NC == 8 ? ((key ^ (key >> 3)) & 7) : (key & (NC - 1));
  return key * HD + ((chunk ^ f) << 3);
}
// sVt[d][64 keys]: 16-B chunks of a row swizzled by (d ^ (d >> 3)) & 7, so
// both the transposing stores (8 rows d = 8c + e at one key) and the
// fragment reads (32 consecutive rows d at one key chunk) spread over banks.
__device__ __forceinline__ int vt_off(int d, int key) {
  return d * ATT_KV + ((((key >> 3) ^ ((d ^ (d >> 3)) & 7))) << 3) + (key & 7);
}

template <int HD>
__global__ __launch_bounds__(256) void k_attn_bf16(const bf16_t* __restrict__ qkv,
                                                   bf16_t* __restrict__ out,
                                                   const ImgDesc* __restrict__ imgs,
                                                   const AttnItem* __restrict__ items,
                                                   int heads) {
  constexpr int NCH = HD / 8;                  // 16-B chunks per row of one head
  constexpr int KLOADS = ATT_KV * NCH / 256;   // K chunks per thread
  constexpr int VTHREADS = 32 * NCH;           // threads staging V: key pair x chunk
  static_assert(KLOADS >= 1 && VTHREADS <= 256, "tile / threads");
  // Three-stage K / V ring: while tile kt's softmax and P.V run, tile kt+1
  // is read for the next scores and tile kt+2 is being staged.
  __shared__ __attribute__((aligned(16))) bf16_t sK[3][ATT_KV * HD];
  __shared__ __attribute__((aligned(16))) bf16_t sVt[3][HD * ATT_KV];

  const AttnItem it = items[blockIdx.x];
  const int h = blockIdx.y;
  const ImgDesc dsc = imgs[it.img];
  const int N = dsc.ntok;
  const int D = heads * HD;
  const int ld = 3 * D;
  const bf16_t* base = qkv + (size_t)dsc.tok_start * ld;
  const bf16_t* Qp = base + h * HD;
  const bf16_t* Kp = base + D + h * HD;
  const bf16_t* Vp = base + 2 * D + h * HD;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l32 = lane & 31, g = lane >> 5;
  const int qw = it.q0 + wave * 32;           // first query of this wave
  const bool wave_active = qw < N;
  const int q = qw + l32;                      // this lane's query
  const int qc = min(q, N - 1);

  // Q^T operand fragments: lane (query, g) holds Q[q][16c + 8g .. +7].
  bf16x8 qf[HD / 16];
#pragma unroll
  for (int c = 0; c < HD / 16; ++c)
    qf[c] = *reinterpret_cast<const bf16x8*>(Qp + (size_t)qc * ld + 16 * c + 8 * g);

  // Staging: K chunk id = tid + i*256 -> key id / NCH, chunk id % NCH.
  // V: thread (key pair vp = tid / NCH, chunk vc = tid % NCH) loads rows
  // 2vp and 2vp+1 (coalesced: NCH consecutive lanes cover a row) and stores
  // them transposed as 32-bit key pairs.
  const int vp = tid / NCH, vc = tid % NCH;
  u32x4 rk[KLOADS], rv0, rv1;
  auto load_kv = [&](int kbase) {
#pragma unroll
    for (int i = 0; i < KLOADS; ++i) {
      const int id = tid + i * 256;
      const int key = min(kbase + id / NCH, N - 1);
      rk[i] = *reinterpret_cast<const u32x4*>(Kp + (size_t)key * ld + (id % NCH) * 8);
    }
    if (tid < VTHREADS) {
      const int k0 = min(kbase + 2 * vp, N - 1), k1 = min(kbase + 2 * vp + 1, N - 1);
      rv0 = *reinterpret_cast<const u32x4*>(Vp + (size_t)k0 * ld + vc * 8);
      rv1 = *reinterpret_cast<const u32x4*>(Vp + (size_t)k1 * ld + vc * 8);
    }
  };
  auto store_kv = [&](int buf) {
#pragma unroll
    for (int i = 0; i < KLOADS; ++i) {
      const int id = tid + i * 256;
      *reinterpret_cast<u32x4*>(&sK[buf][k_off<HD>(id / NCH, id % NCH)]) = rk[i];
    }
    if (tid < VTHREADS) {
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const uint32_t a = rv0[w], b = rv1[w];
        // element 2w (low halves) and 2w+1 (high halves) of the chunk
        *reinterpret_cast<uint32_t*>(&sVt[buf][vt_off(vc * 8 + 2 * w, 2 * vp)]) =
            (a & 0xFFFFu) | (b << 16);
        *reinterpret_cast<uint32_t*>(&sVt[buf][vt_off(vc * 8 + 2 * w + 1, 2 * vp)]) =
            (a >> 16) | (b & 0xFFFF0000u);
      }
    }
  };

  const float sl2 = 1.4426950408889634f / sqrtf((float)HD);  // log2(e)/sqrt(d)
  float m_run = -INFINITY, l_run = 0.f;   // running max (log2 units) and sum
  f32x16 o[HD / 32];
#pragma unroll
  for (int a = 0; a < HD / 32; ++a)
#pragma unroll
    for (int r = 0; r < 16; ++r) o[a][r] = 0.f;

  // S^T blocks of one key tile: s[kb][r] = S[key kb*32 + 8(r/4) + 4g + r%4][query].
  auto scores = [&](const bf16_t* tK, f32x16* s) {
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
#pragma unroll
      for (int r = 0; r < 16; ++r) s[kb][r] = 0.f;
#pragma unroll
      for (int c = 0; c < HD / 16; ++c) {
        const bf16x8 kf = *reinterpret_cast<const bf16x8*>(&tK[k_off<HD>(kb * 32 + l32, 2 * c + g)]);
        s[kb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(kf, qf[c], s[kb], 0, 0, 0);
      }
    }
  };

  // Software pipeline: the scores of tile kt+1 are issued to the matrix
  // cores before the softmax of tile kt runs on the vector ALUs (the two are
  // independent), then P.V of tile kt.
  const int KT = (N + ATT_KV - 1) / ATT_KV;
  load_kv(0);
  store_kv(0);
  if (KT > 1) {
    load_kv(ATT_KV);
    store_kv(1);
  }
  __syncthreads();
  f32x16 s_cur[2], s_nxt[2];
  if (wave_active) scores(sK[0], s_cur);
  for (int kt = 0; kt < KT; ++kt) {
    const int cur = kt % 3;
    if (kt + 2 < KT) load_kv((kt + 2) * ATT_KV);
    if (wave_active) {
      if (kt + 1 < KT) scores(sK[(kt + 1) % 3], s_nxt);
      const bf16_t* tV = sVt[cur];
      f32x16* s = s_cur;
      const int kbase = kt * ATT_KV;
      if (kbase + ATT_KV > N) {            // keys past the image: excluded
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
#pragma unroll
          for (int r = 0; r < 16; ++r)
            if (kbase + kb * 32 + 8 * (r >> 2) + 4 * g + (r & 3) >= N) s[kb][r] = -INFINITY;
      }
      float mt = s[0][0];
#pragma unroll
      for (int kb = 0; kb < 2; ++kb)
#pragma unroll
        for (int r = 0; r < 16; ++r) mt = fmaxf(mt, s[kb][r]);
      mt = fmaxf(mt, __shfl_xor(mt, 32, 64));
      const float m_new = fmaxf(m_run, mt * sl2);
      const float nm = -m_new;
      if (__any(m_new != m_run)) {         // rescale only when some max moved
        const float alpha = __builtin_amdgcn_exp2f(m_run - m_new);
        l_run *= alpha;
#pragma unroll
        for (int a = 0; a < HD / 32; ++a)
#pragma unroll
          for (int r = 0; r < 16; ++r) o[a][r] *= alpha;
      }
      m_run = m_new;
      float ls = 0.f;
#pragma unroll
      for (int kb = 0; kb < 2; ++kb)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const float p = __builtin_amdgcn_exp2f(fmaf(s[kb][r], sl2, nm));
          s[kb][r] = p;
          ls += p;
        }
      l_run += ls;
      // O^T += V^T P^T over four 16-key chunks j; chunk j = 2kb + hh uses
      // s[kb][8hh .. 8hh+7]: keys 16j + 8(e/4) + 4g + e%4 for element e.
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int kb = j >> 1, hh = j & 1;
        u32x4 pk;
#pragma unroll
        for (int w = 0; w < 4; ++w)
          pk[w] = pack_bf16x2(s[kb][8 * hh + 2 * w], s[kb][8 * hh + 2 * w + 1]);
        const bf16x8 pf = __builtin_bit_cast(bf16x8, pk);
#pragma unroll
        for (int a = 0; a < HD / 32; ++a) {
          const int d = a * 32 + l32;
          const u32x2 v0 = *reinterpret_cast<const u32x2*>(&tV[vt_off(d, 16 * j + 4 * g)]);
          const u32x2 v1 = *reinterpret_cast<const u32x2*>(&tV[vt_off(d, 16 * j + 8 + 4 * g)]);
          u32x4 vk;
          vk[0] = v0.x; vk[1] = v0.y; vk[2] = v1.x; vk[3] = v1.y;
          o[a] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, vk), pf, o[a],
                                                         0, 0, 0);
        }
      }
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) s_cur[kb] = s_nxt[kb];
    }
    // Stage kt+2 overwrites the buffer of tile kt-1, last read before the
    // previous barrier.
    if (kt + 2 < KT) store_kv((kt + 2) % 3);
    __syncthreads();
  }
  if (!wave_active || q >= N) return;
  const float lt = l_run + __shfl_xor(l_run, 32, 64);
  const float inv = 1.f / lt;
  bf16_t* op = out + (size_t)(dsc.tok_start + q) * D + h * HD;
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

// ----------------------------------------------------------------- FP32
constexpr int F32_KV = 32;

template <int HD>
__global__ __launch_bounds__(ATT_Q) void k_attn_f32(const float* __restrict__ qkv,
                                                    float* __restrict__ out,
                                                    const ImgDesc* __restrict__ imgs,
                                                    const AttnItem* __restrict__ items,
                                                    int heads) {
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
  for (int k0 = 0; k0 < N; k0 += F32_KV) {
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
      s[j] = (k0 + j < N) ? a * sc : -INFINITY;
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

hipError_t attention_bf16(const bf16_t* qkv, bf16_t* o, const ImgDesc* imgs,
                          const AttnItem* items, int n_items, int heads, int head_dim,
                          hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  dim3 grid(n_items, heads), block(256);
  if (head_dim == 64)
    hipLaunchKernelGGL(k_attn_bf16<64>, grid, block, 0, s, qkv, o, imgs, items, heads);
  else if (head_dim == 32)
    hipLaunchKernelGGL(k_attn_bf16<32>, grid, block, 0, s, qkv, o, imgs, items, heads);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t attention_f32(const float* qkv, float* o, const ImgDesc* imgs,
                         const AttnItem* items, int n_items, int heads, int head_dim,
                         hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  dim3 grid(n_items, heads), block(ATT_Q);
  if (head_dim == 64)
    hipLaunchKernelGGL(k_attn_f32<64>, grid, block, 0, s, qkv, o, imgs, items, heads);
  else if (head_dim == 32)
    hipLaunchKernelGGL(k_attn_f32<32>, grid, block, 0, s, qkv, o, imgs, items, heads);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace vl
