// Row and elementwise kernels: LayerNorm, patch gathering, class-token
// pooling with projection and L2 normalisation, scoring heads, and the
// weight preparation done once per model.
#include <algorithm>

#include "kernels.hpp"

namespace vl {

// ---------------------------------------------------------------- LayerNorm
// LayerNorm (Ba et al. 2016, Sec. 3): mean and biased variance of each row,
// computed in FP32 with two passes over registers.  One wave per row.
template <int NPER, bool OUT_BF16>
__global__ __launch_bounds__(256) void k_layernorm(const float* __restrict__ x,
                                                   const float* __restrict__ gm,
                                                   const float* __restrict__ bt, float eps,
                                                   void* __restrict__ y, int M,
                                                   const BatchCounts* __restrict__ bc) {
  constexpr int D = NPER * 64;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (bc) M = bc->T;   // capacity launch: live rows
  if (row >= M) return;
  const float* xr = x + (size_t)row * D;
  float v[NPER];
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < NPER; ++i) {
    v[i] = xr[lane + 64 * i];
    s += v[i];
  }
  const float mean = wave_sum(s) * (1.f / D);
  float q = 0.f;
#pragma unroll
  for (int i = 0; i < NPER; ++i) {
    v[i] -= mean;
    q += v[i] * v[i];
  }
  const float rstd = rsqrtf(wave_sum(q) * (1.f / D) + eps);
#pragma unroll
  for (int i = 0; i < NPER; ++i) {
    const int c = lane + 64 * i;
    const float o = v[i] * rstd * gm[c] + bt[c];
    if (OUT_BF16)
      static_cast<bf16_t*>(y)[(size_t)row * D + c] = (bf16_t)f32_to_bf16_bits(o);
    else
      static_cast<float*>(y)[(size_t)row * D + c] = o;
  }
}

template <int NPER>
static void launch_ln(const float* x, const float* g, const float* b, float eps, void* y,
                      bool y_bf16, int M, hipStream_t s, const BatchCounts* bc) {
  dim3 grid((M + 3) / 4), block(256);
  if (y_bf16)
    hipLaunchKernelGGL((k_layernorm<NPER, true>), grid, block, 0, s, x, g, b, eps, y, M, bc);
  else
    hipLaunchKernelGGL((k_layernorm<NPER, false>), grid, block, 0, s, x, g, b, eps, y, M, bc);
}

hipError_t layernorm_rows(const float* x, const float* g, const float* b, float eps, void* y,
                          bool y_bf16, int M, int D, hipStream_t s, const BatchCounts* bc) {
  if (M <= 0) return hipSuccess;
  switch (D / 64) {
    case 2: launch_ln<2>(x, g, b, eps, y, y_bf16, M, s, bc); break;
    case 4: launch_ln<4>(x, g, b, eps, y, y_bf16, M, s, bc); break;
    case 6: launch_ln<6>(x, g, b, eps, y, y_bf16, M, s, bc); break;
    case 8: launch_ln<8>(x, g, b, eps, y, y_bf16, M, s, bc); break;
    case 10: launch_ln<10>(x, g, b, eps, y, y_bf16, M, s, bc); break;
    case 12: launch_ln<12>(x, g, b, eps, y, y_bf16, M, s, bc); break;
    case 14: launch_ln<14>(x, g, b, eps, y, y_bf16, M, s, bc); break;
    case 16: launch_ln<16>(x, g, b, eps, y, y_bf16, M, s, bc); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ------------------------------------------------- LayerNorm folding pieces
// The first block's LayerNorm in folded form: row statistics as k_layernorm
// takes them (FP32, two passes over registers), written as (mean, rstd),
// and u = bf16(x * g).  One wave per row.
template <int NPER>
__global__ __launch_bounds__(256) void k_ln_fold(const float* __restrict__ x,
                                                 const float* __restrict__ gm, float eps,
                                                 bf16_t* __restrict__ u,
                                                 float* __restrict__ st, int M) {
  constexpr int D = NPER * 64;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= M) return;
  const float* xr = x + (size_t)row * D;
  float v[NPER];
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < NPER; ++i) {
    v[i] = xr[lane + 64 * i];
    s += v[i];
  }
  const float mean = wave_sum(s) * (1.f / D);
  float q = 0.f;
#pragma unroll
  for (int i = 0; i < NPER; ++i) {
    const float d = v[i] - mean;
    q += d * d;
  }
  const float rstd = rsqrtf(wave_sum(q) * (1.f / D) + eps);
#pragma unroll
  for (int i = 0; i < NPER; ++i) {
    const int c = lane + 64 * i;
    u[(size_t)row * D + c] = (bf16_t)f32_to_bf16_bits(v[i] * gm[c]);
  }
  if (lane == 0) *reinterpret_cast<float2*>(st + 2 * (size_t)row) = make_float2(mean, rstd);
}

hipError_t ln_fold_rows(const float* x, const float* g, float eps, bf16_t* u, float* row_stats,
                        int M, int D, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  dim3 grid((M + 3) / 4), block(256);
#define VL_LNF(N)                                                                       \
  case N:                                                                               \
    hipLaunchKernelGGL(k_ln_fold<N>, grid, block, 0, s, x, g, eps, u, row_stats, M); break;
  switch (D / 64) {
    VL_LNF(2) VL_LNF(4) VL_LNF(6) VL_LNF(8) VL_LNF(10) VL_LNF(12) VL_LNF(14) VL_LNF(16)
    default: return hipErrorInvalidValue;
  }
#undef VL_LNF
  return hipGetLastError();
}

// Row statistics from G = D/32 equal-size column groups' (mean_g, M2_g),
// stored group-major ([G][M] pairs): mean = sum_g mean_g / G and M2 =
// sum_g M2_g + 32 sum_g (mean_g - mean)^2 (the exact combination of
// equal-size groups); then rstd = 1 / sqrt(M2 / D + eps).  Eight lanes per
// row, lane j taking groups j, j + 8, ... in order, the lanes' sums added
// in a fixed butterfly order.
__global__ __launch_bounds__(256) void k_ln_stats(const float* __restrict__ parts, int M, int G,
                                                  float eps, float* __restrict__ st) {
  const int row = blockIdx.x * 32 + (threadIdx.x >> 3), j = threadIdx.x & 7;
  const float2* pr = reinterpret_cast<const float2*>(parts) + min(row, M - 1);
  float sm = 0.f;
  for (int g = j; g < G; g += 8) sm += pr[(size_t)g * M].x;
  sm += __shfl_xor(sm, 1, 64);
  sm += __shfl_xor(sm, 2, 64);
  sm += __shfl_xor(sm, 4, 64);
  const float mean = sm / (float)G;
  float t = 0.f;
  for (int g = j; g < G; g += 8) {
    const float2 v = pr[(size_t)g * M];
    const float d = v.x - mean;
    t += fmaf(32.f, d * d, v.y);
  }
  t += __shfl_xor(t, 1, 64);
  t += __shfl_xor(t, 2, 64);
  t += __shfl_xor(t, 4, 64);
  if (row < M && j == 0)
    *reinterpret_cast<float2*>(st + 2 * (size_t)row) =
        make_float2(mean, rsqrtf(t / (float)(32 * G) + eps));
}

hipError_t ln_stats_from_parts(const float* parts, int M, int D, float eps, float* row_stats,
                               hipStream_t s) {
  if (M <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ln_stats, dim3((M + 31) / 32), dim3(256), 0, s, parts, M, D / 32, eps,
                     row_stats);
  return hipGetLastError();
}

// c1[n] = sum_k g[k] W[n,k], c2[n] = sum_k b[k] W[n,k] + bias[n] with W the
// GEMM's weights (BF16, or e4m3 codes times the row scale), FP32 sums in a
// fixed order.  One workgroup per output row.
template <bool FP8>
__global__ __launch_bounds__(256) void k_ln_consts(const void* __restrict__ w,
                                                   const float* __restrict__ ws,
                                                   const float* __restrict__ g,
                                                   const float* __restrict__ b,
                                                   const float* __restrict__ bias, int K,
                                                   float* __restrict__ c1,
                                                   float* __restrict__ c2) {
  __shared__ float red[4];
  const int n = blockIdx.x;
  float a = 0.f, c = 0.f;
  for (int k = threadIdx.x; k < K; k += 256) {
    float wv;
    if (FP8)
      wv = bf16_bits_to_f32(e4m3_to_bf16_bits(static_cast<const uint8_t*>(w)[(size_t)n * K + k]));
    else
      wv = bf16_bits_to_f32(static_cast<const bf16_t*>(w)[(size_t)n * K + k]);
    a = fmaf(g[k], wv, a);
    c = fmaf(b[k], wv, c);
  }
  auto sum = [](float x, float y) { return x + y; };
  a = block_reduce(a, red, sum);
  c = block_reduce(c, red, sum);
  if (threadIdx.x == 0) {
    const float sc = FP8 ? ws[n] : 1.f;
    c1[n] = a * sc;
    c2[n] = fmaf(c, sc, bias[n]);
  }
}

hipError_t ln_fold_consts(const void* w, bool w_fp8, const float* wscale, const float* g,
                          const float* b, const float* bias, int N, int K, float* c1, float* c2,
                          hipStream_t s) {
  if (w_fp8)
    hipLaunchKernelGGL(k_ln_consts<true>, dim3(N), dim3(256), 0, s, w, wscale, g, b, bias, K, c1,
                       c2);
  else
    hipLaunchKernelGGL(k_ln_consts<false>, dim3(N), dim3(256), 0, s, w, wscale, g, b, bias, K, c1,
                       c2);
  return hipGetLastError();
}

// LayerNorm with an MXFP8 output (the A operand of the next GEMM): as above,
// but each lane holds float4 chunks lane + 64 i of the row, so a 32-column
// MX block is 8 adjacent lanes.  D % 128 == 0, so the chunks in range form
// whole 8-lane groups.
template <int NV4>
__global__ __launch_bounds__(256) void k_layernorm_mx(const float* __restrict__ x,
                                                      const float* __restrict__ gm,
                                                      const float* __restrict__ bt, float eps,
                                                      uint8_t* __restrict__ codes,
                                                      uint8_t* __restrict__ scales, int M,
                                                      int D) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= M) return;
  const int nch = D >> 2;
  const float4* xr = reinterpret_cast<const float4*>(x + (size_t)row * D);
  float4 v[NV4];
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < NV4; ++i) {
    const int ch = lane + 64 * i;
    v[i] = ch < nch ? xr[ch] : make_float4(0.f, 0.f, 0.f, 0.f);
    s += (v[i].x + v[i].y) + (v[i].z + v[i].w);
  }
  const float mean = wave_sum(s) / (float)D;
  float q = 0.f;
#pragma unroll
  for (int i = 0; i < NV4; ++i) {
    if (lane + 64 * i >= nch) continue;
    v[i].x -= mean; v[i].y -= mean; v[i].z -= mean; v[i].w -= mean;
    q += (v[i].x * v[i].x + v[i].y * v[i].y) + (v[i].z * v[i].z + v[i].w * v[i].w);
  }
  const float rstd = rsqrtf(wave_sum(q) / (float)D + eps);
#pragma unroll
  for (int i = 0; i < NV4; ++i) {
    const int ch = lane + 64 * i;
    if (64 * i >= nch) break;  // wave-uniform
    float4 g4 = make_float4(0.f, 0.f, 0.f, 0.f), b4 = g4;
    if (ch < nch) {
      g4 = reinterpret_cast<const float4*>(gm)[ch];
      b4 = reinterpret_cast<const float4*>(bt)[ch];
    }
    const float o0 = v[i].x * rstd * g4.x + b4.x, o1 = v[i].y * rstd * g4.y + b4.y;
    const float o2 = v[i].z * rstd * g4.z + b4.z, o3 = v[i].w * rstd * g4.w + b4.w;
    const float amax = max8(fmaxf(fmaxf(fabsf(o0), fabsf(o1)), fmaxf(fabsf(o2), fabsf(o3))));
    const uint32_t sb = mx_scale_byte(amax);
    const uint32_t w = mx_pack4(o0, o1, o2, o3, mx_inv_scale(sb));
    if (ch < nch) {
      reinterpret_cast<uint32_t*>(codes + (size_t)row * D)[ch] = w;
      if ((lane & 7) == 0) scales[mx_scale_off(row, 4 * ch, M)] = (uint8_t)sb;
    }
  }
}

hipError_t layernorm_rows_mx(const float* x, const float* g, const float* b, float eps,
                             uint8_t* codes, uint8_t* scales, int M, int D, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  if (D % 128 || D > 1024) return hipErrorInvalidValue;
  dim3 grid((M + 3) / 4), block(256);
  switch ((D + 255) / 256) {
    case 1: hipLaunchKernelGGL(k_layernorm_mx<1>, grid, block, 0, s, x, g, b, eps, codes, scales, M, D); break;
    case 2: hipLaunchKernelGGL(k_layernorm_mx<2>, grid, block, 0, s, x, g, b, eps, codes, scales, M, D); break;
    case 3: hipLaunchKernelGGL(k_layernorm_mx<3>, grid, block, 0, s, x, g, b, eps, codes, scales, M, D); break;
    case 4: hipLaunchKernelGGL(k_layernorm_mx<4>, grid, block, 0, s, x, g, b, eps, codes, scales, M, D); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ------------------------------------------------------- token embedding
// Text sequences: X[t] = tok_emb[id(t)] + pos[i] for token i of a sequence
// (row-gather of the learned tables), plus tok_info[t] = (sequence, i).  A
// descriptor's pix_off is the offset of its ids in the packed id stream.
// Grid (token within sequence, sequence); one workgroup of 64 lanes per
// token, float4 columns.  Ids are clamped into [0, vocab) so a bad id cannot
// read outside the table.
__global__ __launch_bounds__(64) void k_text_embed(const int32_t* __restrict__ ids,
                                                   const ImgDesc* __restrict__ seqs,
                                                   const float* __restrict__ tok_emb,
                                                   const float* __restrict__ pos, int vocab,
                                                   int D, float* __restrict__ X,
                                                   int2* __restrict__ tok_info) {
  const ImgDesc d = seqs[blockIdx.y];
  const int i = blockIdx.x;
  if (i >= d.ntok) return;
  const int t = d.tok_start + i;                     // row in this part's X
  const int id = min(max(ids[d.pix_off + i], 0), vocab - 1);  // ids: whole batch
  const float4* er = reinterpret_cast<const float4*>(tok_emb + (size_t)id * D);
  const float4* pr = reinterpret_cast<const float4*>(pos + (size_t)i * D);
  float4* xr = reinterpret_cast<float4*>(X + (size_t)t * D);
  for (int c = threadIdx.x; c < D / 4; c += 64) {
    const float4 a = er[c], b = pr[c];
    xr[c] = make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
  }
  if (threadIdx.x == 0) tok_info[t] = make_int2((int)blockIdx.y, i);
}

hipError_t text_embed(const int32_t* ids, const ImgDesc* seqs, int n_seqs, int max_len,
                      const float* tok_emb, const float* pos, int vocab, int D, float* X,
                      int2* tok_info, hipStream_t s) {
  if (n_seqs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_text_embed, dim3(max_len, n_seqs), dim3(64), 0, s, ids, seqs, tok_emb, pos,
                     vocab, D, X, tok_info);
  return hipGetLastError();
}

// ------------------------------------------------------------------ im2col
// Token row t of image i: zeros for the class token, otherwise the patch's
// raw pixels in (channel, row-in-patch, column-in-patch) order followed by
// zero padding to kpad.  One wave per token; blockIdx.y is the image.
template <bool OUT_BF16>
__global__ __launch_bounds__(256) void k_im2col(const float* __restrict__ pix,
                                                const ImgDesc* __restrict__ imgs, int chans,
                                                int patch, int kpad, void* __restrict__ out,
                                                int2* __restrict__ tok_info,
                                                const BatchCounts* __restrict__ bc) {
  if (bc) {   // capacity launch: live images and the call's pixel buffer
    if ((int)blockIdx.y >= bc->n) return;
    pix = bc->pix;
  }
  const ImgDesc d = imgs[blockIdx.y];
  const int tok = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (tok >= d.ntok) return;
  const int t = d.tok_start + tok;
  if (lane == 0) tok_info[t] = make_int2(blockIdx.y, tok);
  const int pp = patch * patch, kreal = chans * pp;
  int r = 0, q = 0;
  if (tok > 0) {
    r = (tok - 1) / d.gw;
    q = (tok - 1) - r * d.gw;
  }
  const float* src = pix + d.pix_off;
  // (c, a, b) of this lane's k, advanced by 64 per step with carries
  // instead of two integer divisions per element.
  int c = lane / pp, a = lane - c * pp;
  int b = a % patch;
  a /= patch;
  const int dc = 64 / pp, drem = 64 - dc * pp;
  const int da = drem / patch, db = drem - da * patch;
  for (int k = lane; k < kpad; k += 64) {
    float v = 0.f;
    if (tok > 0 && k < kreal)
      v = src[(size_t)c * d.H * d.W + (size_t)(r * patch + a) * d.W + q * patch + b];
    if (OUT_BF16)
      static_cast<bf16_t*>(out)[(size_t)t * kpad + k] = (bf16_t)f32_to_bf16_bits(v);
    else
      static_cast<float*>(out)[(size_t)t * kpad + k] = v;
    b += db;
    a += da;
    c += dc;
    if (b >= patch) { b -= patch; ++a; }
    if (a >= patch) { a -= patch; ++c; }
  }
}

hipError_t im2col(const float* pix, const ImgDesc* imgs, int n_imgs, int max_ntok, int chans,
                  int patch, int kpad, void* out, bool out_bf16, int2* tok_info, hipStream_t s,
                  const BatchCounts* bc) {
  if (n_imgs <= 0) return hipSuccess;
  dim3 grid((max_ntok + 3) / 4, n_imgs), block(256);
  if (out_bf16)
    hipLaunchKernelGGL(k_im2col<true>, grid, block, 0, s, pix, imgs, chans, patch, kpad, out,
                       tok_info, bc);
  else
    hipLaunchKernelGGL(k_im2col<false>, grid, block, 0, s, pix, imgs, chans, patch, kpad, out,
                       tok_info, bc);
  return hipGetLastError();
}

// ----------------------------------------------------- pool + LN + proj + L2
// Pooling, final LayerNorm (ViT Eq. 4), bias-free projection and L2
// normalisation, FP32.  The pooled row is a sequence's first (the image class
// token) or, with pool_last, its last (the text end-of-text token).
//
// Final LayerNorm of each sequence's pooled row into z [n, D]: one workgroup
// per sequence, FP32 statistics with the biased variance.  The projection of
// all pooled rows is then one few-rows GEMM, which reads the projection
// matrix once per 8 sequences.
__global__ __launch_bounds__(256) void k_pool_ln(const float* __restrict__ x,
                                                 const ImgDesc* __restrict__ imgs,
                                                 const float* __restrict__ gm,
                                                 const float* __restrict__ bt, float eps, int D,
                                                 float* __restrict__ z, int pool_last,
                                                 const BatchCounts* __restrict__ bc) {
  __shared__ float red[4];
  if (bc && (int)blockIdx.x >= bc->n) return;   // capacity launch: live sequences
  const int tid = threadIdx.x;
  const ImgDesc d = imgs[blockIdx.x];
  const float* xr = x + (size_t)(d.tok_start + (pool_last ? d.ntok - 1 : 0)) * D;
  float* zr = z + (size_t)blockIdx.x * D;
  float s = 0.f;
  for (int c = tid; c < D; c += 256) s += xr[c];
  const float mean = block_reduce(s, red, [](float a, float b) { return a + b; }) / D;
  float q = 0.f;
  for (int c = tid; c < D; c += 256) {
    const float v = xr[c] - mean;
    q += v * v;
  }
  const float rstd = rsqrtf(block_reduce(q, red, [](float a, float b) { return a + b; }) / D + eps);
  for (int c = tid; c < D; c += 256) zr[c] = (xr[c] - mean) * rstd * gm[c] + bt[c];
}

// Row-wise division by the L2 norm (clamped at 1e-12).  One wave per row.
__global__ __launch_bounds__(256) void k_l2_normalise(const float* __restrict__ e,
                                                      float* __restrict__ out, int rows, int P,
                                                      const BatchCounts* __restrict__ bc) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (bc) {   // capacity launch: live rows, written to the call's output
    rows = bc->n;
    out = bc->emb;
  }
  if (row >= rows) return;
  const float* er = e + (size_t)row * P;
  float n2 = 0.f;
  for (int c = lane; c < P; c += 64) n2 += er[c] * er[c];
  const float inv = 1.f / fmaxf(sqrtf(wave_sum(n2)), 1e-12f);
  for (int c = lane; c < P; c += 64) out[(size_t)row * P + c] = er[c] * inv;
}

hipError_t pool_project(const float* x, const ImgDesc* imgs, int n_imgs, const float* g,
                        const float* b, float eps, const float* proj, int D, int P,
                        bool pool_last, float* z, float* e_tmp, float* emb, hipStream_t s,
                        const BatchCounts* bc) {
  if (n_imgs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pool_ln, dim3(n_imgs), dim3(256), 0, s, x, imgs, g, b, eps, D, z,
                     (int)pool_last, bc);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  // e_tmp = z . proj^T (the projection has no bias)
  EpiArgs ep;
  ep.out = e_tmp; ep.ldo = P;
  // (with bc, rows past the live count project unwritten z rows; no output
  // depends on them)
  err = gemm_f32_rows(z, D, proj, D, n_imgs, P, D, OP_LOGITS, ep, s);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_l2_normalise, dim3((n_imgs + 3) / 4), dim3(256), 0, s, e_tmp, emb, n_imgs,
                     P, bc);
  return hipGetLastError();
}

hipError_t l2_normalise_rows(const float* e, float* out, int rows, int P, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_l2_normalise, dim3((rows + 3) / 4), dim3(256), 0, s, e, out, rows, P,
                     nullptr);
  return hipGetLastError();
}

// ------------------------------------------------------------- score heads
// In place over logit rows: CLIP head = softmax over the row (texts), SigLIP
// head = sigmoid of each logit.  top1 = lowest column index of the maximum.
__global__ __launch_bounds__(256) void k_score_rows(float* __restrict__ sc,
                                                    int32_t* __restrict__ top1, int cols,
                                                    int head) {
  __shared__ float rv[4];
  __shared__ int ri[4];
  __shared__ float red[4];
  float* row = sc + (size_t)blockIdx.x * cols;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  float best = -INFINITY;
  int bi = 0x7fffffff;
  for (int c = tid; c < cols; c += 256) {
    const float v = row[c];
    if (v > best) { best = v; bi = c; }   // c increases: first max kept
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const float ov = __shfl_xor(best, o, 64);
    const int oi = __shfl_xor(bi, o, 64);
    if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
  }
  if (lane == 0) { rv[w] = best; ri[w] = bi; }
  __syncthreads();
  best = rv[0]; bi = ri[0];
  for (int k = 1; k < 4; ++k)
    if (rv[k] > best || (rv[k] == best && ri[k] < bi)) { best = rv[k]; bi = ri[k]; }
  if (top1 && tid == 0) top1[blockIdx.x] = bi;
  if (head == 0) {
    float s = 0.f;
    for (int c = tid; c < cols; c += 256) s += expf(row[c] - best);
    s = block_reduce(s, red, [](float a, float b) { return a + b; });
    const float inv = 1.f / s;
    for (int c = tid; c < cols; c += 256) row[c] = expf(row[c] - best) * inv;
  } else {
    for (int c = tid; c < cols; c += 256) row[c] = 1.f / (1.f + expf(-row[c]));
  }
}

hipError_t score_rows(float* scores, int32_t* top1, int rows, int cols, int head,
                      hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_score_rows, dim3(rows), dim3(256), 0, s, scores, top1, cols, head);
  return hipGetLastError();
}

// -------------------------------------------------------- weight preparation
__global__ void k_convert_bf16(const float* __restrict__ src, bf16_t* __restrict__ dst,
                               size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    dst[i] = (bf16_t)f32_to_bf16_bits(src[i]);
}

hipError_t convert_bf16(const float* src, bf16_t* dst, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const size_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_convert_bf16, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256),
                     0, s, src, dst, n);
  return hipGetLastError();
}

// OCP e4m3fn encoding (OFP8 rev 1.0, Sec. 5.1) of an FP32 value, round to
// nearest even, saturating at +-448.  Below 2^-6 the step is 2^-9
// (subnormal codes 0..7; 8 lands on the smallest normal code 0x08).
__device__ __forceinline__ uint32_t f32_to_e4m3(float y) {
  const uint32_t sign = (__float_as_uint(y) >> 24) & 0x80u;
  const float a = fminf(fabsf(y), 448.f);
  if (a < 0.015625f) return sign | (uint32_t)rintf(a * 512.f);
  int ex;
  const float f = frexpf(a, &ex);      // a = f * 2^ex, f in [0.5, 1)
  int E = ex - 1;                      // a in [2^E, 2^(E+1))
  uint32_t mq = (uint32_t)rintf((2.f * f - 1.f) * 8.f);
  if (mq == 8u) { E += 1; mq = 0u; }
  return sign | ((uint32_t)(E + 7) << 3) | mq;
}

// Per-output-row quantiser: s = max|row| / 448 (1 for an all-zero row),
// code = e4m3(w / s).  One workgroup per row.
__global__ __launch_bounds__(256) void k_quant_e4m3(const float* __restrict__ src,
                                                    uint8_t* __restrict__ dst,
                                                    float* __restrict__ scales, int cols) {
  __shared__ float red[4];
  const float* r = src + (size_t)blockIdx.x * cols;
  float m = 0.f;
  for (int c = threadIdx.x; c < cols; c += 256) m = fmaxf(m, fabsf(r[c]));
  m = block_reduce(m, red, [](float a, float b) { return fmaxf(a, b); });
  float s = m / 448.f;
  if (!(s > 0.f)) s = 1.f;
  if (threadIdx.x == 0) scales[blockIdx.x] = s;
  for (int c = threadIdx.x; c < cols; c += 256)
    dst[(size_t)blockIdx.x * cols + c] = (uint8_t)f32_to_e4m3(r[c] / s);
}

hipError_t quantise_e4m3_rows(const float* src, uint8_t* dst, float* scales, int rows, int cols,
                              hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_quant_e4m3, dim3(rows), dim3(256), 0, s, src, dst, scales, cols);
  return hipGetLastError();
}

// FP32 -> BF16 as the kernels round: method 0 the integer round-to-nearest-
// even of the bit pattern (LayerNorm outputs, weights, activations written
// one value at a time), method 1 the packed conversion instruction
// (v_cvt_pk_bf16_f32: GEMM epilogues, attention probabilities); n even.
template <int METHOD>
__global__ __launch_bounds__(256) void k_bf16_round(const float* __restrict__ src,
                                                    uint32_t* __restrict__ dst, size_t n2) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n2; i += (size_t)gridDim.x * 256) {
    const float2 v = reinterpret_cast<const float2*>(src)[i];
    dst[i] = METHOD == 0 ? (f32_to_bf16_bits(v.x) | (f32_to_bf16_bits(v.y) << 16))
                         : pack_bf16x2(v.x, v.y);
  }
}

hipError_t bf16_round(const float* src, bf16_t* dst, size_t n, int method, hipStream_t s) {
  const size_t n2 = n / 2;
  if (n2 == 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<size_t>((n2 + 255) / 256, 65536);
  if (method == 0)
    hipLaunchKernelGGL(k_bf16_round<0>, dim3(blocks), dim3(256), 0, s, src,
                       reinterpret_cast<uint32_t*>(dst), n2);
  else
    hipLaunchKernelGGL(k_bf16_round<1>, dim3(blocks), dim3(256), 0, s, src,
                       reinterpret_cast<uint32_t*>(dst), n2);
  return hipGetLastError();
}

// MXFP8 encoding of FP32 rows (weights at model creation, or any caller's
// rows): thread i encodes the four values 4i .. 4i+3 of the flattened
// [rows, cols] array; cols % 128 == 0, so an aligned group of 8 threads is
// one 32-value block of one row, and a group is wholly in or out of range.
__global__ void k_mx_quant(const float* __restrict__ src, uint8_t* __restrict__ codes,
                           uint8_t* __restrict__ scales, int rows, int cols) {
  const size_t n4 = (size_t)rows * cols / 4;
  const int c4 = cols / 4;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
       i += (size_t)gridDim.x * blockDim.x) {
    const float4 v = reinterpret_cast<const float4*>(src)[i];
    const float amax = max8(fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
    const uint32_t sb = mx_scale_byte(amax);
    reinterpret_cast<uint32_t*>(codes)[i] = mx_pack4(v.x, v.y, v.z, v.w, mx_inv_scale(sb));
    if ((i & 7) == 0) {
      const int r = (int)(i / c4), c = 4 * (int)(i % c4);
      scales[mx_scale_off(r, c, rows)] = (uint8_t)sb;
    }
  }
}

hipError_t mx_quantise_rows(const float* src, uint8_t* codes, uint8_t* scales, int rows,
                            int cols, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  if (cols <= 0 || cols % 128) return hipErrorInvalidValue;
  const size_t n4 = (size_t)rows * cols / 4;
  const size_t blocks = (n4 + 255) / 256;
  hipLaunchKernelGGL(k_mx_quant, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0,
                     s, src, codes, scales, rows, cols);
  return hipGetLastError();
}

// Normalisation folded into the patch embedding: W'[d,c,a,b] = W / std_c,
// b'[d] = b[d] - sum_{c,a,b} W[d,c,a,b] * mean_c / std_c.  Output rows are
// padded with zeros to kpad columns.  One workgroup per output channel d.
__global__ __launch_bounds__(256) void k_fold_patch(const float* __restrict__ w,
                                                    const float* __restrict__ b, float4 mean,
                                                    float4 stdv, int chans, int pp, int kpad,
                                                    float* __restrict__ w32,
                                                    bf16_t* __restrict__ w16,
                                                    float* __restrict__ bout) {
  __shared__ float red[4];
  const int d = blockIdx.x;
  const int kreal = chans * pp;
  const float* wr = w + (size_t)d * kreal;
  float acc = 0.f;
  for (int k = threadIdx.x; k < kpad; k += 256) {
    float v = 0.f;
    if (k < kreal) {
      const int c = k / pp;
      const float sd = c == 0 ? stdv.x : (c == 1 ? stdv.y : (c == 2 ? stdv.z : stdv.w));
      const float mu = c == 0 ? mean.x : (c == 1 ? mean.y : (c == 2 ? mean.z : mean.w));
      v = wr[k] / sd;
      acc = fmaf(v, mu, acc);
    }
    if (w32) w32[(size_t)d * kpad + k] = v;
    if (w16) w16[(size_t)d * kpad + k] = (bf16_t)f32_to_bf16_bits(v);
  }
  acc = block_reduce(acc, red, [](float a, float c) { return a + c; });
  if (threadIdx.x == 0) bout[d] = b[d] - acc;
}

hipError_t fold_patch_weights(const float* w, const float* b, const float* mean,
                              const float* stdv, int chans, int D, int patch, int kpad,
                              float* w_f32, bf16_t* w_bf16, float* b_out, hipStream_t s) {
  if (chans < 1 || chans > 4) return hipErrorInvalidValue;
  float mu[4] = {0.f, 0.f, 0.f, 0.f}, sd[4] = {1.f, 1.f, 1.f, 1.f};
  for (int c = 0; c < chans; ++c) { mu[c] = mean[c]; sd[c] = stdv[c]; }
  hipLaunchKernelGGL(k_fold_patch, dim3(D), dim3(256), 0, s, w, b,
                     make_float4(mu[0], mu[1], mu[2], mu[3]), make_float4(sd[0], sd[1], sd[2], sd[3]),
                     chans, patch * patch, kpad, w_f32, w_bf16, b_out);
  return hipGetLastError();
}

hipError_t copy_f32(const float* src, float* dst, size_t n, hipStream_t s) {
  return hipMemcpyAsync(dst, src, n * sizeof(float), hipMemcpyDeviceToDevice, s);
}

}  // namespace vl
