// Kernels of contrastive training through the image tower: the pieces the
// training forward adds (the FC1 activation taken from a kept FP32
// pre-activation) and the backward pass -- the chain rule of each forward
// definition:
//   L2 normalisation  e_hat = e / |e|:  de = (de_hat - e_hat <e_hat, de_hat>) / |e|
//   LayerNorm (Ba et al. 2016, Sec. 3):  dx = rstd (dxh - mean(dxh) - xh mean(dxh xh)),
//       dxh = dy * gamma;  dgamma = sum dy xh,  dbeta = sum dy
//   GELU (Hendrycks & Gimpel 2016):  GELU'(z) = Phi(z) + z phi(z)
//   attention (Vaswani et al. 2017, Eq. 1):  dV = P^T dO,  dP = dO V^T,
//       dS = P (dP - rowsum(dO O)),  dQ = dS K / sqrt(d),  dK = dS^T Q / sqrt(d)
//   patch embedding / class token / position table (ViT Eq. 1).
// The products of the linear layers run on the GEMM kernels (gemm.hip);
// here are the transposes that feed them, the deterministic column sums of
// the bias and LayerNorm gradients (per-block partial sums added in a fixed
// order), the attention backward and the head / embedding pieces.
#include <type_traits>

#include "kernels.hpp"

namespace vl {

template <typename T>
__device__ __forceinline__ float ldf(const T* p, size_t i);
template <>
__device__ __forceinline__ float ldf<float>(const float* p, size_t i) { return p[i]; }
template <>
__device__ __forceinline__ float ldf<bf16_t>(const bf16_t* p, size_t i) {
  return bf16_bits_to_f32(p[i]);
}
template <typename T>
__device__ __forceinline__ void stf(T* p, size_t i, float v);
template <>
__device__ __forceinline__ void stf<float>(float* p, size_t i, float v) { p[i] = v; }
template <>
__device__ __forceinline__ void stf<bf16_t>(bf16_t* p, size_t i, float v) {
  p[i] = (bf16_t)f32_to_bf16_bits(v);
}

// ------------------------------------------------------------- transposes
// out[c][r] = in[r][c] for r < rows, 0 for rows <= r < ld_out (the zero K
// padding of a weight-gradient GEMM), c < cols.  32 x 32 tiles through LDS.
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_transpose(const TI* __restrict__ in, int rows, int cols,
                                                   int ld_in, TO* __restrict__ out, int ld_out) {
  __shared__ float t[32][33];
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int k = ty; k < 32; k += 8) {
    const int r = r0 + k, c = c0 + tx;
    t[k][tx] = (r < rows && c < cols) ? ldf(in, (size_t)r * ld_in + c) : 0.f;
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int c = c0 + k, r = r0 + tx;
    if (c < cols && r < ld_out) stf(out, (size_t)c * ld_out + r, t[tx][k]);
  }
}

// BF16 output, 64 x 64 tiles: each thread moves 8 consecutive elements (16
// bytes of BF16 out, 16 or 32 bytes in) per access; the tile waits in LDS as
// BF16 rows padded by 8 elements.  Used when cols % 8 == 0, ld_in % 8 == 0,
// ld_out % 8 == 0 and both pointers are 16-byte aligned.
// With part (the row-block partials of colsum, kColRows = 64 rows per
// block): part[blockIdx.y][c] = the sum of the input column c over the
// tile's rows in ascending order, from the values as given (FP32 input before
// its BF16 rounding), as k_colsum_part forms it.
// With copy (FP32 input): also the input rounded to BF16 in its own layout
// ([rows, ld_in]), from the same loads.
template <typename TI>
__global__ __launch_bounds__(256) void k_transpose64(const TI* __restrict__ in, int rows, int cols,
                                                     int ld_in, bf16_t* __restrict__ out,
                                                     int ld_out, float* __restrict__ part,
                                                     bf16_t* __restrict__ copy) {
  static_assert(kColRows == 64, "one partial per 64-row tile");
  __shared__ __attribute__((aligned(16))) uint16_t t[64][72];
  __shared__ float tf[sizeof(TI) == 4 ? 64 : 1][65];   // FP32 input as given, for the sums
  const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
  const int tid = threadIdx.x;
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
    const int r = (tid >> 3) + 32 * pass, cc = (tid & 7) * 8;
    const int gr = r0 + r, gc = c0 + cc;
    u32x4 v = {0u, 0u, 0u, 0u};
    if (gr < rows && gc < cols) {   // cols % 8 == 0: the 8 columns are all in range
      if constexpr (sizeof(TI) == 2) {
        v = *reinterpret_cast<const u32x4*>(in + (size_t)gr * ld_in + gc);
      } else {
        const float4 a = *reinterpret_cast<const float4*>(in + (size_t)gr * ld_in + gc);
        const float4 b = *reinterpret_cast<const float4*>(in + (size_t)gr * ld_in + gc + 4);
        v[0] = pack_bf16x2(a.x, a.y); v[1] = pack_bf16x2(a.z, a.w);
        v[2] = pack_bf16x2(b.x, b.y); v[3] = pack_bf16x2(b.z, b.w);
        if (copy) *reinterpret_cast<u32x4*>(copy + (size_t)gr * ld_in + gc) = v;
        if (part) {
          const float f[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
          for (int j = 0; j < 8; ++j) tf[r][cc + j] = f[j];
        }
      }
    }
    *reinterpret_cast<u32x4*>(&t[r][cc]) = v;
  }
  __syncthreads();
  if (part && tid < 64 && c0 + tid < cols) {   // rows past the matrix are not added
    const int nr = min(64, rows - r0);
    float acc = 0.f;
    for (int r = 0; r < nr; ++r)
      acc += sizeof(TI) == 4 ? tf[sizeof(TI) == 4 ? r : 0][tid]
                             : bf16_bits_to_f32(t[r][tid]);
    part[(size_t)blockIdx.y * cols + c0 + tid] = acc;
  }
  if (out == nullptr) return;   // partials (and the copy) only
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
    const int c = (tid >> 3) + 32 * pass, rr = (tid & 7) * 8;
    const int gc = c0 + c, gr = r0 + rr;
    if (gc >= cols || gr >= ld_out) continue;   // ld_out % 8 == 0: all 8 rows in range
    u32x4 v;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      v[j] = (uint32_t)t[rr + 2 * j][c] | ((uint32_t)t[rr + 2 * j + 1][c] << 16);
    *reinterpret_cast<u32x4*>(out + (size_t)gc * ld_out + gr) = v;
  }
}

hipError_t transpose_rows(const void* in, bool in_bf16, int rows, int cols, int ld_in, void* out,
                          bool out_bf16, int ld_out, hipStream_t s, float* colsum_part,
                          bf16_t* copy_bf16) {
  if (cols <= 0 || ld_out <= 0) return hipSuccess;
  // (no output: a pass for the column-sum partials or the copy alone)
  if (!out && (!out_bf16 || (!colsum_part && !copy_bf16))) return hipErrorInvalidValue;
  const bool al16 = (reinterpret_cast<uintptr_t>(in) % 16 == 0) &&
                    (reinterpret_cast<uintptr_t>(out) % 16 == 0);
  if (out_bf16 && al16 && cols % 8 == 0 && ld_in % 8 == 0 && ld_out % 8 == 0) {
    // the partials need every row block of the input to be a row of blocks
    if (colsum_part && (ld_out + 63) / 64 < (rows + 63) / 64) return hipErrorInvalidValue;
    if (copy_bf16 && (in_bf16 || (ld_out + 63) / 64 < (rows + 63) / 64 ||
                      reinterpret_cast<uintptr_t>(copy_bf16) % 16))
      return hipErrorInvalidValue;
    dim3 grid((cols + 63) / 64, (ld_out + 63) / 64), block(256);
    if (in_bf16)
      hipLaunchKernelGGL(k_transpose64<bf16_t>, grid, block, 0, s, static_cast<const bf16_t*>(in),
                         rows, cols, ld_in, static_cast<bf16_t*>(out), ld_out, colsum_part,
                         nullptr);
    else
      hipLaunchKernelGGL(k_transpose64<float>, grid, block, 0, s, static_cast<const float*>(in),
                         rows, cols, ld_in, static_cast<bf16_t*>(out), ld_out, colsum_part,
                         copy_bf16);
    return hipGetLastError();
  }
  if (colsum_part || copy_bf16 || !out) return hipErrorInvalidValue;
  dim3 grid((cols + 31) / 32, (ld_out + 31) / 32), block(256);
  if (in_bf16 && out_bf16)
    hipLaunchKernelGGL((k_transpose<bf16_t, bf16_t>), grid, block, 0, s,
                       static_cast<const bf16_t*>(in), rows, cols, ld_in,
                       static_cast<bf16_t*>(out), ld_out);
  else if (!in_bf16 && out_bf16)
    hipLaunchKernelGGL((k_transpose<float, bf16_t>), grid, block, 0, s,
                       static_cast<const float*>(in), rows, cols, ld_in,
                       static_cast<bf16_t*>(out), ld_out);
  else if (!in_bf16 && !out_bf16)
    hipLaunchKernelGGL((k_transpose<float, float>), grid, block, 0, s,
                       static_cast<const float*>(in), rows, cols, ld_in,
                       static_cast<float*>(out), ld_out);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// ------------------------------------------------------------ column sums
// part[b][c] = sum of in[r][c] over the rows r of block b (kColRows rows,
// ascending), skipping class-token rows when tok is given; then out[c] =
// sum over b ascending.  Fixed order: the result does not depend on timing.
// Four adjacent columns per thread (one 16- or 8-byte load per row).
__device__ __forceinline__ float4 ld4(const float* p) { return *reinterpret_cast<const float4*>(p); }
__device__ __forceinline__ float4 ld4(const bf16_t* p) {
  const u32x2 v = *reinterpret_cast<const u32x2*>(p);
  return make_float4(bf16_bits_to_f32(v.x & 0xFFFFu), bf16_bits_to_f32(v.x >> 16),
                     bf16_bits_to_f32(v.y & 0xFFFFu), bf16_bits_to_f32(v.y >> 16));
}

template <typename T>
__global__ __launch_bounds__(256) void k_colsum_part(const T* __restrict__ in, int R, int C,
                                                     int ld, const int2* __restrict__ tok,
                                                     float* __restrict__ part) {
  const int c = 4 * (blockIdx.x * 256 + threadIdx.x);
  if (c >= C) return;
  const int r0 = blockIdx.y * kColRows, r1 = min(R, r0 + kColRows);
  float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int r = r0; r < r1; ++r) {
    if (tok && tok[r].y == 0) continue;
    const float4 v = ld4(in + (size_t)r * ld + c);
    s.x += v.x; s.y += v.y; s.z += v.z; s.w += v.w;
  }
  *reinterpret_cast<float4*>(part + (size_t)blockIdx.y * C + c) = s;
}

// Final pass: 4 columns per workgroup, 64 phases per column (many small
// workgroups: the partials are few, so the pass is latency-bound); phase k
// sums the partials b = k, k + 64, ... in ascending order, then the 64 phase
// sums are added in phase order.  blockIdx.y = 1 takes a second partial array
// of the same shape (part2 -> out2) in the same launch.
__global__ __launch_bounds__(256) void k_colsum_final(const float* __restrict__ part0, int nb,
                                                      int C, float* __restrict__ out0,
                                                      const float* __restrict__ part2,
                                                      float* __restrict__ out2) {
  const float* part = blockIdx.y ? part2 : part0;
  float* out = blockIdx.y ? out2 : out0;
  __shared__ float red[64][5];
  const int cl = threadIdx.x & 3, ph = threadIdx.x >> 2;
  const int c = blockIdx.x * 4 + cl;
  float s = 0.f;
  if (c < C)
    for (int b = ph; b < nb; b += 64) s += part[(size_t)b * C + c];
  red[ph][cl] = s;
  __syncthreads();
  if (ph == 0 && c < C) {
    float t = 0.f;
    for (int k = 0; k < 64; ++k) t += red[k][cl];
    out[c] = t;
  }
}

hipError_t colsum_final(const float* part, int nb, int C, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_colsum_final, dim3((C + 3) / 4), dim3(256), 0, s, part, nb, C, out,
                     nullptr, nullptr);
  return hipGetLastError();
}

// Two column sums of [nb, C] partial arrays in one launch.
static hipError_t colsum_final2(const float* part, const float* part2, int nb, int C,
                                float* out, float* out2, hipStream_t s) {
  hipLaunchKernelGGL(k_colsum_final, dim3((C + 3) / 4, 2), dim3(256), 0, s, part, nb, C, out,
                     part2, out2);
  return hipGetLastError();
}

hipError_t colsum(const void* in, bool in_bf16, int R, int C, int ld, const int2* tok,
                  float* part, float* out, hipStream_t s) {
  const int nb = (R + kColRows - 1) / kColRows;
  if (nb <= 0 || C % 4 || ld % 4) return hipErrorInvalidValue;
  dim3 grid((C / 4 + 255) / 256, nb), block(256);
  if (in_bf16)
    hipLaunchKernelGGL(k_colsum_part<bf16_t>, grid, block, 0, s, static_cast<const bf16_t*>(in),
                       R, C, ld, tok, part);
  else
    hipLaunchKernelGGL(k_colsum_part<float>, grid, block, 0, s, static_cast<const float*>(in), R,
                       C, ld, tok, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return colsum_final(part, nb, C, out, s);
}

// -------------------------------------------------------- LayerNorm backward
// dx[r] += LN'(x[r]) dy[r] for rows r of [R, D] (statistics recomputed from x
// in FP32 as the forward takes them), and per-block partial sums of
// dgamma (dy * xh) and dbeta (dy) over the block's kLnRows rows.  One wave
// per row; the four waves' partials are added in wave order.
template <int NPER>
__global__ __launch_bounds__(256) void k_ln_bwd(const float* __restrict__ x,
                                                const float* __restrict__ gm,
                                                const float* __restrict__ dy, float eps,
                                                float* __restrict__ dx, int R,
                                                float* __restrict__ pg, float* __restrict__ pb) {
  constexpr int D = NPER * 64;
  __shared__ float sg[4][D], sb[4][D];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float ag[NPER], ab[NPER];
#pragma unroll
  for (int i = 0; i < NPER; ++i) ag[i] = ab[i] = 0.f;
  for (int rr = w; rr < kLnRows; rr += 4) {
    const int r = blockIdx.x * kLnRows + rr;
    if (r >= R) break;
    const float* xr = x + (size_t)r * D;
    const float* dr = dy + (size_t)r * D;
    float v[NPER], d[NPER];
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
    float a = 0.f, b = 0.f;
#pragma unroll
    for (int i = 0; i < NPER; ++i) {
      const int c = lane + 64 * i;
      const float xh = v[i] * rstd;
      const float g = dr[c];
      const float dxh = g * gm[c];
      ag[i] += g * xh;
      ab[i] += g;
      a += dxh;
      b += dxh * xh;
      v[i] = xh;
      d[i] = dxh;
    }
    a = wave_sum(a) * (1.f / D);
    b = wave_sum(b) * (1.f / D);
    float* o = dx + (size_t)r * D;
#pragma unroll
    for (int i = 0; i < NPER; ++i) {
      const int c = lane + 64 * i;
      o[c] += rstd * (d[i] - a - v[i] * b);
    }
  }
#pragma unroll
  for (int i = 0; i < NPER; ++i) {
    sg[w][lane + 64 * i] = ag[i];
    sb[w][lane + 64 * i] = ab[i];
  }
  __syncthreads();
  for (int c = threadIdx.x; c < D; c += 256) {
    pg[(size_t)blockIdx.x * D + c] = (sg[0][c] + sg[1][c]) + (sg[2][c] + sg[3][c]);
    pb[(size_t)blockIdx.x * D + c] = (sb[0][c] + sb[1][c]) + (sb[2][c] + sb[3][c]);
  }
}

hipError_t layernorm_backward(const float* x, const float* g, const float* dy, float eps,
                              float* dx, int R, int D, float* pg, float* pb, float* dgamma,
                              float* dbeta, hipStream_t s) {
  const int nb = (R + kLnRows - 1) / kLnRows;
  if (nb <= 0) return hipErrorInvalidValue;
  dim3 grid(nb), block(256);
#define VL_LNB(N)                                                                              \
  case N:                                                                                      \
    hipLaunchKernelGGL(k_ln_bwd<N>, grid, block, 0, s, x, g, dy, eps, dx, R, pg, pb); break;
  switch (D / 64) {
    VL_LNB(2) VL_LNB(4) VL_LNB(6) VL_LNB(8) VL_LNB(10) VL_LNB(12) VL_LNB(14) VL_LNB(16)
    default: return hipErrorInvalidValue;
  }
#undef VL_LNB
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return colsum_final2(pg, pb, nb, D, dgamma, dbeta, s);
}

// ------------------------------------------------------------------- GELU
// Training forward: the FC1 activation from the kept FP32 pre-activation z,
// exactly as the inference FC1 epilogue forms it (the polynomial Phi rounded
// to BF16 pairs, or erf in FP32), so both forwards agree bitwise.
template <bool OUT_BF16>
__global__ __launch_bounds__(256) void k_gelu_fwd(const float* __restrict__ z, void* __restrict__ g,
                                                  size_t n2) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n2) return;
  const float2 v = reinterpret_cast<const float2*>(z)[i];
  if (OUT_BF16)
    static_cast<uint32_t*>(g)[i] = pack_bf16x2(gelu_poly(v.x), gelu_poly(v.y));
  else
    static_cast<float2*>(g)[i] = make_float2(gelu_erf(v.x), gelu_erf(v.y));
}

hipError_t gelu_forward(const float* z, void* g, bool g_bf16, size_t n, hipStream_t s) {
  const size_t n2 = n / 2;  // n is even (the MLP width is a multiple of 128)
  dim3 grid((unsigned)((n2 + 255) / 256)), block(256);
  if (g_bf16) hipLaunchKernelGGL(k_gelu_fwd<true>, grid, block, 0, s, z, g, n2);
  else hipLaunchKernelGGL(k_gelu_fwd<false>, grid, block, 0, s, z, g, n2);
  return hipGetLastError();
}

// Backward: dz = dg (Phi(z) + z phi(z)), and the activation itself again
// (g, as the forward formed it) for the weight gradient of FC2.  Two
// elements per thread.  BF16 models take Phi from the forward's polynomial
// (so g has the forward's bits) and phi = exp(-z^2/2) / sqrt(2 pi) from the
// hardware base-2 exponential; FP32 models the erf form.
template <typename T>
__global__ __launch_bounds__(256) void k_gelu_bwd(const float* __restrict__ dg,
                                                  const float* __restrict__ z, T* __restrict__ dz,
                                                  T* __restrict__ g, size_t n2) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n2) return;
  constexpr bool BF = sizeof(T) == 2;
  const float2 v = reinterpret_cast<const float2*>(z)[i];
  const float2 d = reinterpret_cast<const float2*>(dg)[i];
  float c[2], ph[2];
  const float vv[2] = {v.x, v.y};
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    if (BF) {
      c[j] = phi_poly(vv[j]);
      // exp(-z^2/2) = 2^(-z^2 log2(e) / 2)
      ph[j] = 0.3989422804014327f * __builtin_amdgcn_exp2f(-0.72134752044448170f * vv[j] * vv[j]);
    } else {
      c[j] = 0.5f * (1.0f + erff(vv[j] * 0.70710678118654752f));
      ph[j] = 0.3989422804014327f * expf(-0.5f * vv[j] * vv[j]);
    }
  }
  const float dz0 = d.x * (c[0] + v.x * ph[0]), dz1 = d.y * (c[1] + v.y * ph[1]);
  if (BF) {
    reinterpret_cast<uint32_t*>(dz)[i] = pack_bf16x2(dz0, dz1);
    reinterpret_cast<uint32_t*>(g)[i] = pack_bf16x2(v.x * c[0], v.y * c[1]);
  } else {
    reinterpret_cast<float2*>(dz)[i] = make_float2(dz0, dz1);
    reinterpret_cast<float2*>(g)[i] = make_float2(gelu_erf(v.x), gelu_erf(v.y));
  }
}

hipError_t gelu_backward(const float* dg, const float* z, void* dz, void* g, bool bf16, size_t n,
                         hipStream_t s) {
  const size_t n2 = n / 2;  // n is even (the MLP width is a multiple of 128)
  dim3 grid((unsigned)((n2 + 255) / 256)), block(256);
  if (bf16)
    hipLaunchKernelGGL(k_gelu_bwd<bf16_t>, grid, block, 0, s, dg, z, static_cast<bf16_t*>(dz),
                       static_cast<bf16_t*>(g), n2);
  else
    hipLaunchKernelGGL(k_gelu_bwd<float>, grid, block, 0, s, dg, z, static_cast<float*>(dz),
                       static_cast<float*>(g), n2);
  return hipGetLastError();
}

// ------------------------------------------------------- attention backward
// Tiles of 64 queries x 64 keys of one (image, head).  Thread t of a 256-wide
// workgroup owns row t / 4 of the tile and the quarter t % 4 of its columns;
// scores are recomputed from Q and K in FP32 (BF16 operands are widened).
// dq pass: per 64-query block, first the row maximum and sum of
// exponentials over all keys (log-sum-exp), then dQ; it also writes the
// log-sum-exp and D = rowsum(dO * O) for the dk/dv pass, which walks all
// query blocks per 64-key block.  No atomics: every output has one writer.
constexpr int AB = 64;

template <typename T, int HD>
__global__ __launch_bounds__(256) void k_attn_bwd_dq(const T* __restrict__ qkv,
                                                     const T* __restrict__ o,
                                                     const float* __restrict__ dO,
                                                     const ImgDesc* __restrict__ imgs,
                                                     const AttnItem* __restrict__ items, int heads,
                                                     T* __restrict__ dqkv, float* __restrict__ lse,
                                                     float* __restrict__ dsum) {
  constexpr int LD = HD + 1, KQ = HD / 4;
  __shared__ float sQ[AB][LD], sdO[AB][LD], sK[AB][LD], sV[AB][LD], sS[AB][AB + 1];
  const AttnItem it = items[blockIdx.x];
  const int h = blockIdx.y;
  const ImgDesc d = imgs[it.img];
  const int N = d.ntok, base = d.tok_start;
  const int DM = heads * HD, D3 = 3 * DM;
  const float scale = 1.0f / sqrtf((float)HD);
  const int tid = threadIdx.x, r = tid >> 2, cq = tid & 3;
  const int nq = min(AB, N - it.q0);
  for (int i = tid; i < AB * HD; i += 256) {
    const int rr = i / HD, k = i - rr * HD;
    const bool ok = rr < nq;
    const size_t row = (size_t)(base + it.q0 + rr);
    sQ[rr][k] = ok ? ldf(qkv, row * D3 + h * HD + k) : 0.f;
    sdO[rr][k] = ok ? dO[row * DM + h * HD + k] : 0.f;
    sV[rr][k] = ok ? ldf(o, row * DM + h * HD + k) : 0.f;   // O, for D
  }
  __syncthreads();
  float dsv = 0.f;
#pragma unroll
  for (int k = 0; k < KQ; ++k) dsv += sdO[r][cq * KQ + k] * sV[r][cq * KQ + k];
  dsv += __shfl_xor(dsv, 1);
  dsv += __shfl_xor(dsv, 2);
  __syncthreads();
  auto load_kv = [&](int k0, int nk, bool with_v) {
    for (int i = tid; i < AB * HD; i += 256) {
      const int rr = i / HD, k = i - rr * HD;
      const size_t row = (size_t)(base + k0 + rr);
      sK[rr][k] = rr < nk ? ldf(qkv, row * D3 + DM + h * HD + k) : 0.f;
      if (with_v) sV[rr][k] = rr < nk ? ldf(qkv, row * D3 + 2 * DM + h * HD + k) : 0.f;
    }
  };
  // pass 1: log-sum-exp of the row over all keys of the image
  float mrow = -INFINITY, lrow = 0.f;
  for (int k0 = 0; k0 < N; k0 += AB) {
    const int nk = min(AB, N - k0);
    load_kv(k0, nk, false);
    __syncthreads();
    float sc[16];
    float tmax = -INFINITY;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int c = cq * 16 + j;
      float a = 0.f;
#pragma unroll
      for (int k = 0; k < HD; ++k) a += sQ[r][k] * sK[c][k];
      sc[j] = c < nk ? a * scale : -INFINITY;
      tmax = fmaxf(tmax, sc[j]);
    }
    tmax = fmaxf(tmax, __shfl_xor(tmax, 1));
    tmax = fmaxf(tmax, __shfl_xor(tmax, 2));
    const float mnew = fmaxf(mrow, tmax);
    float ts = 0.f;
#pragma unroll
    for (int j = 0; j < 16; ++j) ts += expf(sc[j] - mnew);
    ts += __shfl_xor(ts, 1);
    ts += __shfl_xor(ts, 2);
    lrow = lrow * expf(mrow - mnew) + ts;
    mrow = mnew;
    __syncthreads();
  }
  const float lse_r = mrow + logf(lrow);
  // pass 2: dS and dQ
  float dq[KQ];
#pragma unroll
  for (int k = 0; k < KQ; ++k) dq[k] = 0.f;
  for (int k0 = 0; k0 < N; k0 += AB) {
    const int nk = min(AB, N - k0);
    load_kv(k0, nk, true);
    __syncthreads();
#pragma unroll 4
    for (int j = 0; j < 16; ++j) {
      const int c = cq * 16 + j;
      float a = 0.f, b = 0.f;
#pragma unroll
      for (int k = 0; k < HD; ++k) {
        a += sQ[r][k] * sK[c][k];
        b += sdO[r][k] * sV[c][k];
      }
      const float p = c < nk ? expf(a * scale - lse_r) : 0.f;
      sS[r][c] = p * (b - dsv);
    }
    __syncthreads();
    for (int c = 0; c < nk; ++c) {
      const float ds = sS[r][c];
#pragma unroll
      for (int k = 0; k < KQ; ++k) dq[k] += ds * sK[c][cq * KQ + k];
    }
    __syncthreads();
  }
  if (r < nq) {
    const size_t row = (size_t)(base + it.q0 + r);
#pragma unroll
    for (int k = 0; k < KQ; ++k) stf(dqkv, row * D3 + h * HD + cq * KQ + k, dq[k] * scale);
    if (cq == 0) {
      lse[row * heads + h] = lse_r;
      dsum[row * heads + h] = dsv;
    }
  }
}

template <typename T, int HD>
__global__ __launch_bounds__(256) void k_attn_bwd_dkv(const T* __restrict__ qkv,
                                                      const float* __restrict__ dO,
                                                      const ImgDesc* __restrict__ imgs,
                                                      const AttnItem* __restrict__ items, int heads,
                                                      const float* __restrict__ lse,
                                                      const float* __restrict__ dsum,
                                                      T* __restrict__ dqkv) {
  constexpr int LD = HD + 1, KQ = HD / 4;
  __shared__ float sK[AB][LD], sV[AB][LD], sQ[AB][LD], sdO[AB][LD];
  __shared__ float sP[AB][AB + 1], sDS[AB][AB + 1], sL[AB], sD[AB];
  const AttnItem it = items[blockIdx.x];   // it.q0: first key of the block
  const int h = blockIdx.y;
  const ImgDesc d = imgs[it.img];
  const int N = d.ntok, base = d.tok_start;
  const int DM = heads * HD, D3 = 3 * DM;
  const float scale = 1.0f / sqrtf((float)HD);
  const int tid = threadIdx.x, c = tid >> 2, rq = tid & 3;
  const int nk = min(AB, N - it.q0);
  for (int i = tid; i < AB * HD; i += 256) {
    const int rr = i / HD, k = i - rr * HD;
    const size_t row = (size_t)(base + it.q0 + rr);
    sK[rr][k] = rr < nk ? ldf(qkv, row * D3 + DM + h * HD + k) : 0.f;
    sV[rr][k] = rr < nk ? ldf(qkv, row * D3 + 2 * DM + h * HD + k) : 0.f;
  }
  float dk[KQ], dv[KQ];
#pragma unroll
  for (int k = 0; k < KQ; ++k) dk[k] = dv[k] = 0.f;
  for (int q0 = 0; q0 < N; q0 += AB) {
    const int nq = min(AB, N - q0);
    for (int i = tid; i < AB * HD; i += 256) {
      const int rr = i / HD, k = i - rr * HD;
      const size_t row = (size_t)(base + q0 + rr);
      sQ[rr][k] = rr < nq ? ldf(qkv, row * D3 + h * HD + k) : 0.f;
      sdO[rr][k] = rr < nq ? dO[row * DM + h * HD + k] : 0.f;
    }
    if (tid < AB) {
      const size_t row = (size_t)(base + q0 + tid);
      sL[tid] = tid < nq ? lse[row * heads + h] : 0.f;
      sD[tid] = tid < nq ? dsum[row * heads + h] : 0.f;
    }
    __syncthreads();
#pragma unroll 4
    for (int j = 0; j < 16; ++j) {
      const int r = rq * 16 + j;
      float a = 0.f, b = 0.f;
#pragma unroll
      for (int k = 0; k < HD; ++k) {
        a += sQ[r][k] * sK[c][k];
        b += sdO[r][k] * sV[c][k];
      }
      const bool ok = r < nq && c < nk;
      const float p = ok ? expf(a * scale - sL[r]) : 0.f;
      sP[c][r] = p;
      sDS[c][r] = p * (b - sD[r]);
    }
    __syncthreads();
    for (int r = 0; r < nq; ++r) {
      const float p = sP[c][r], ds = sDS[c][r];
#pragma unroll
      for (int k = 0; k < KQ; ++k) {
        dv[k] += p * sdO[r][rq * KQ + k];
        dk[k] += ds * sQ[r][rq * KQ + k];
      }
    }
    __syncthreads();
  }
  if (c < nk) {
    const size_t row = (size_t)(base + it.q0 + c);
#pragma unroll
    for (int k = 0; k < KQ; ++k) {
      stf(dqkv, row * D3 + DM + h * HD + rq * KQ + k, dk[k] * scale);
      stf(dqkv, row * D3 + 2 * DM + h * HD + rq * KQ + k, dv[k]);
    }
  }
}

// ---- MFMA form (BF16 models).  v_mfma_f32_32x32x16_bf16 computes
// C[i][j] += sum_k A[i][k] B[j][k] over 16 values of k: lane (l32, g) gives
// A[l32][8g + e] and B[l32][8g + e] (e = 0..7) and receives column j = l32,
// rows i = 8(r/4) + 4g + r%4 (r = 0..15) of C.  Hence an accumulator whose
// rows run over a contraction index serves directly as a B operand (rows
// 16hh + {4g .. 4g+3, 8+4g .. 8+4g+3} of a 32-row block are its elements
// 8hh .. 8hh+7), provided the A operand supplies the same eight rows: the
// gfx950 LDS transpose read gives exactly that from a row-major tile (the
// forward attention kernel's value-operand read).
//
// dq kernel (below): four waves own 128 queries, key / value tiles stream
// through LDS; dS^T = P^T (dP^T - D) and dQ^T += K^T dS^T with K^T read
// transposed from the key tile.  dkv kernel: four waves own 128 keys (lane:
// one key, K and V rows in registers); per 64-query tile (Q and dO in LDS)
// S = Q K^T, dP = dO V^T, P, dS, then dV^T += dO^T P and dK^T += Q^T dS with
// dO^T and Q^T read transposed.  FP32 accumulation; P and dS rounded to BF16
// as MFMA operands; dO rounded to BF16 where it is an MFMA operand.
template <int HD>
struct TrTile {   // row-major 64 x HD BF16 tile; chunk c of row r at c ^ f(r)
  static constexpr int NCH = HD / 8;
  static constexpr int ROWB = HD * 2;
  static constexpr int BYTES = 64 * ROWB;
  __device__ static int f(int r) { return NCH == 8 ? (r & 7) : 0; }
  __device__ static int off(int r, int chunk) { return r * ROWB + ((chunk ^ f(r)) << 4); }
};

typedef short s16x4b __attribute__((ext_vector_type(4)));

// This lane's offset, within a TrTile, of its transposed-operand reads for
// 32-column block a and 16-row chunk 0 (chunk jj adds 16 jj rows: the
// permutation depends on the row modulo 8 only).
template <int HD>
__device__ __forceinline__ uint32_t tr_lane_off(int a, int lane) {
  using TT = TrTile<HD>;
  const int grp = lane >> 4, li = lane & 15;
  const int col = 32 * a + 16 * (grp & 1) + 4 * (li & 3);
  return TT::off(4 * (grp >> 1) + (li >> 2), col >> 3) + (col & 7) * 2;
}

// Transposed operand at LDS byte address `addr` (a lane's tr_lane_off plus
// the tile and 16-row chunk): rows +0..3 and +8..11 of the lane's column.
template <int HD>
__device__ __forceinline__ bf16x8 tr_read(uint32_t addr) {
  typedef __attribute__((address_space(3))) s16x4b lds_s16x4;
  const s16x4b v0 = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)(uintptr_t)addr);
  const s16x4b v1 = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
      (lds_s16x4*)(uintptr_t)(addr + 8 * TrTile<HD>::ROWB));
  u32x4 vk;
  vk[0] = __builtin_bit_cast(u32x2, v0).x; vk[1] = __builtin_bit_cast(u32x2, v0).y;
  vk[2] = __builtin_bit_cast(u32x2, v1).x; vk[3] = __builtin_bit_cast(u32x2, v1).y;
  return __builtin_bit_cast(bf16x8, vk);
}

__device__ __forceinline__ bf16x8 pack8(const f32x16& c, int hh) {
  u32x4 pk;
#pragma unroll
  for (int w = 0; w < 4; ++w) pk[w] = pack_bf16x2(c[8 * hh + 2 * w], c[8 * hh + 2 * w + 1]);
  return __builtin_bit_cast(bf16x8, pk);
}

__device__ __forceinline__ bf16x8 f32x8_to_bf16(float4 a, float4 b) {
  u32x4 pk;
  pk[0] = pack_bf16x2(a.x, a.y); pk[1] = pack_bf16x2(a.z, a.w);
  pk[2] = pack_bf16x2(b.x, b.y); pk[3] = pack_bf16x2(b.z, b.w);
  return __builtin_bit_cast(bf16x8, pk);
}

// Value tile of the dQ kernel (read by rows only): chunk c of row r at
// c ^ f(r), f chosen so 16 consecutive rows read at one logical chunk hit
// distinct banks.
template <int HD>
struct RowTile {
  static constexpr int NCH = HD / 8;
  static constexpr int ROWB = HD * 2;
  static constexpr int BYTES = 64 * ROWB;
  __device__ static int f(int r) { return NCH == 8 ? ((r ^ (r >> 3)) & 7) : ((r >> 2) & 3); }
  __device__ static int off(int r, int chunk) { return r * ROWB + ((chunk ^ f(r)) << 4); }
};

constexpr int BWD_Q = 128;   // queries per dQ workgroup (four waves of 32)
constexpr int BWD_ST = 3;    // key / value tile ring stages of the dQ kernel

// dQ kernel: four waves own 128 queries of one (image, head), a lane one
// query (B operands Q and dO of its row in registers).  Key and value tiles
// of 64 tokens stream through a three-stage LDS ring by direct-to-LDS loads
// issued two tiles ahead (rows past the image read as zero).  Per tile:
// S^T = K Q^T, dP^T = V dO^T, P = exp2(S log2(e) / sqrt(d) - lse),
// dS^T = P^T (dP^T - D), dQ^T += K^T dS^T with K^T read transposed from the
// key tile.  Work items are dealt XCD by XCD (the query blocks of one
// (image, head) share its keys and values in one L2).  LSE_IN: lse2_io holds
// each query's log-sum-exp (log2 units, from the forward) and is only read;
// otherwise a first pass over the keys forms and writes it.  Also writes D =
// rowsum(dO O) per query.
template <int HD, bool LSE_IN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_attn_bwd_dq_mfma(const bf16_t* __restrict__ qkv,
                                                          const bf16_t* __restrict__ o,
                                                          const float* __restrict__ dO,
                                                          const ImgDesc* __restrict__ imgs,
                                                          const AttnItem* __restrict__ items,
                                                          int heads, bf16_t* __restrict__ dqkv,
                                                          float* __restrict__ lse2_io,
                                                          float* __restrict__ dsum_out) {
  using TK = TrTile<HD>;
  using TV = RowTile<HD>;
  constexpr int NC = HD / 16, NA = HD / 32;
  constexpr int RPI = 1024 / TK::ROWB;     // tile rows per 1 KB direct-to-LDS load
  constexpr int LPW = 64 / RPI / 4;        // key (and value) loads per wave and tile
  static_assert(LPW >= 1 && LPW * RPI * 4 == 64, "tile / waves");
  __shared__ __attribute__((aligned(1024))) char sK[BWD_ST][TK::BYTES];
  __shared__ __attribute__((aligned(1024))) char sV[BWD_ST][TV::BYTES];
  const int total = gridDim.x, n_items = total / heads;
  const int wi = xcd_linear(blockIdx.x, total);
  const AttnItem it = items[wi % n_items];
  const int h = wi / n_items;
  const ImgDesc dsc = imgs[it.img];
  const int N = dsc.ntok, DM = heads * HD, ld3 = 3 * DM;
  const bf16_t* base = qkv + (size_t)dsc.tok_start * ld3 + h * HD;
  const int tid = threadIdx.x, lane = tid & 63, l32 = lane & 31, g = lane >> 5;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: LDS bases
  const int qw = it.q0 + 32 * wave;
  const bool wave_active = qw < N;
  const int q = qw + l32;
  const bool qok = q < N;
  const int qc = min(q, N - 1);
  const size_t qrow = (size_t)dsc.tok_start + qc;
  bf16x8 qf[NC], df[NC];
  float dsv = 0.f;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int col = 16 * c + 8 * g;
    qf[c] = *reinterpret_cast<const bf16x8*>(base + (size_t)qc * ld3 + col);
    const float4* dp = reinterpret_cast<const float4*>(dO + qrow * DM + h * HD + col);
    float4 x0 = dp[0], x1 = dp[1];
    if (!qok) x0 = x1 = make_float4(0.f, 0.f, 0.f, 0.f);
    df[c] = f32x8_to_bf16(x0, x1);
    const bf16_t* op = o + qrow * DM + h * HD + col;
    const float xs[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
#pragma unroll
    for (int e = 0; e < 8; ++e) dsv += xs[e] * bf16_bits_to_f32(op[e]);
  }
  dsv += __shfl_xor(dsv, 32, 64);
  const float sl2 = 1.4426950408889634f / sqrtf((float)HD);
  // pass 1 (no log-sum-exp given): each query's log-sum-exp of its scaled
  // scores (log2 units), key fragments straight from global memory
  float lse2;
  if constexpr (LSE_IN) {
    lse2 = lse2_io[qrow * heads + h];
  } else {
    float m = -INFINITY, l = 0.f;
    for (int k0 = 0; k0 < N; k0 += 64) {
      f32x16 s[2];
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
#pragma unroll
        for (int r = 0; r < 16; ++r) s[kb][r] = 0.f;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const bf16x8 kf = *reinterpret_cast<const bf16x8*>(
              base + DM + (size_t)min(k0 + 32 * kb + l32, N - 1) * ld3 + 16 * c + 8 * g);
          s[kb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(kf, qf[c], s[kb], 0, 0, 0);
        }
      }
      float mt = -INFINITY;
#pragma unroll
      for (int kb = 0; kb < 2; ++kb)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int key = k0 + 32 * kb + 8 * (r >> 2) + 4 * g + (r & 3);
          s[kb][r] = key < N ? s[kb][r] * sl2 : -INFINITY;
          mt = fmaxf(mt, s[kb][r]);
        }
      mt = fmaxf(mt, __shfl_xor(mt, 32, 64));
      const float mn = fmaxf(m, mt);
      float ts = 0.f;
#pragma unroll
      for (int kb = 0; kb < 2; ++kb)
#pragma unroll
        for (int r = 0; r < 16; ++r) ts += exp2f(s[kb][r] - mn);
      l = l * exp2f(m - mn) + ts;
      m = mn;
    }
    lse2 = m + log2f(l + __shfl_xor(l, 32, 64));
  }
  // Wait for the operands above with a wait the compiler sees, so its
  // wait-count pass does not hold the ring's loads back for them later.
  __builtin_amdgcn_s_waitcnt(0x0F70);

  // Direct-to-LDS loads: instruction i of this wave fills tile rows
  // R = (wave LPW + i) RPI ..; lane l takes row R + l / NCH and physical
  // chunk l % NCH, i.e. logical chunk (l % NCH) ^ f(row).
  const i32x4 rk = buffer_rsrc(base + DM, (uint64_t)N * ld3 * 2);
  const i32x4 rv = buffer_rsrc(base + 2 * DM, (uint64_t)N * ld3 * 2);
  int goffK[LPW], goffV[LPW];
#pragma unroll
  for (int i = 0; i < LPW; ++i) {
    const int row = (wave * LPW + i) * RPI + lane / TK::NCH;
    goffK[i] = row * ld3 * 2 + (((lane % TK::NCH) ^ TK::f(row)) << 4);
    goffV[i] = row * ld3 * 2 + (((lane % TV::NCH) ^ TV::f(row)) << 4);
  }
  const uint32_t ldsK = lds_offset(&sK[0][0]), ldsV = lds_offset(&sV[0][0]);
  auto issue = [&](int kt, int st) {
    const int kb = kt * 64 * ld3 * 2;
#pragma unroll
    for (int i = 0; i < LPW; ++i) {
      const uint32_t lo = st * TK::BYTES + (wave * LPW + i) * 1024;
      dma16(rk, ldsK + lo, goffK[i] + kb, 0);
      dma16(rv, ldsV + lo, goffV[i] + kb, 0);
    }
  };
  // Row-operand offsets: lane reads row 32kb + l32, logical chunk 2c + g.
  int koff[2][NC], voff[2][NC];
#pragma unroll
  for (int kb = 0; kb < 2; ++kb)
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      koff[kb][c] = TK::off(32 * kb + l32, 2 * c + g);
      voff[kb][c] = TV::off(32 * kb + l32, 2 * c + g);
    }

  uint32_t trK[NA];   // K^T reads: per-lane base, plus stage and chunk immediates
#pragma unroll
  for (int a = 0; a < NA; ++a) trK[a] = ldsK + tr_lane_off<HD>(a, lane);
  f32x16 dq[NA];
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int r = 0; r < 16; ++r) dq[a][r] = 0.f;
  const int KT = (N + 63) / 64;
  auto tile = [&](auto stage, int kt) {
    constexpr int st = decltype(stage)::value;
    // Tile kt must have landed; tile kt+1's loads may stay in flight.
    if (kt + 1 < KT) asm volatile("s_waitcnt vmcnt(%0)" ::"n"(2 * LPW) : "memory");
    else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    lds_barrier();
    // Stage (st+2)%3 held tile kt-1, whose readers all passed the barrier.
    if (kt + 2 < KT) issue(kt + 2, (st + 2) % BWD_ST);
    if (!wave_active) return;
    const char* tK = sK[st];
    const char* tV = sV[st];
    const int k0 = kt * 64;
    // The 64 keys as two halves of 32 (fewer live registers): half kb gives
    // the 16-key chunks jj = 2kb, 2kb + 1 of dQ^T += K^T dS^T.
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
      f32x16 s, dp;
#pragma unroll
      for (int r = 0; r < 16; ++r) s[r] = dp[r] = 0.f;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const bf16x8 kf = *reinterpret_cast<const bf16x8*>(tK + koff[kb][c]);
        s = __builtin_amdgcn_mfma_f32_32x32x16_bf16(kf, qf[c], s, 0, 0, 0);
        const bf16x8 vf = *reinterpret_cast<const bf16x8*>(tV + voff[kb][c]);
        dp = __builtin_amdgcn_mfma_f32_32x32x16_bf16(vf, df[c], dp, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int key = k0 + 32 * kb + 8 * (r >> 2) + 4 * g + (r & 3);
        // (a key past the image has a zero row, score 0; its p could
        // overflow for a very negative log-sum-exp, so it is selected away)
        const float p = key < N ? __builtin_amdgcn_exp2f(fmaf(s[r], sl2, -lse2)) : 0.f;
        s[r] = p * (dp[r] - dsv);
      }
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
        const bf16x8 dsf = pack8(s, hh);
#pragma unroll
        for (int a = 0; a < NA; ++a)
          dq[a] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              tr_read<HD>(trK[a] + st * TK::BYTES + 16 * (2 * kb + hh) * TK::ROWB), dsf, dq[a],
              0, 0, 0);
      }
    }
  };
  issue(0, 0);
  if (KT > 1) issue(1, 1);
  for (int kt = 0; kt < KT; kt += BWD_ST) {
    tile(std::integral_constant<int, 0>(), kt);
    if (kt + 1 < KT) tile(std::integral_constant<int, 1>(), kt + 1);
    if (kt + 2 < KT) tile(std::integral_constant<int, 2>(), kt + 2);
  }
  if (!qok) return;
  const float scale = 1.0f / sqrtf((float)HD);
  const size_t row = (size_t)dsc.tok_start + q;
  bf16_t* out = dqkv + row * ld3 + h * HD;
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int rq = 0; rq < 4; ++rq) {
      u32x2 pk;
      pk.x = pack_bf16x2(dq[a][4 * rq + 0] * scale, dq[a][4 * rq + 1] * scale);
      pk.y = pack_bf16x2(dq[a][4 * rq + 2] * scale, dq[a][4 * rq + 3] * scale);
      *reinterpret_cast<u32x2*>(out + a * 32 + 8 * rq + 4 * g) = pk;
    }
  if (g == 0) {
    if (!LSE_IN) lse2_io[row * heads + h] = lse2;
    dsum_out[row * heads + h] = dsv;
  }
}

// dK/dV kernel: four waves own 128 keys of one (image, head), a lane one key
// (K and V rows of its key in registers, the A-side operands of S and dP).
// dO in BF16 (dO_b [T, DM]).  Query and dO tiles of 64 tokens, with their
// log-sum-exp and D values, stream through a three-stage LDS ring by
// direct-to-LDS loads issued two tiles ahead (rows past the image read as
// zero).  Work items are dealt XCD by XCD.
// (Head width 64 keeps ~180 registers live: two waves per SIMD; 32: three.)
template <int HD>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(HD == 64 ? 2 : 3))) void
k_attn_bwd_dkv_mfma(const bf16_t* __restrict__ qkv, const bf16_t* __restrict__ dO_b,
                    const ImgDesc* __restrict__ imgs, const AttnItem* __restrict__ items,
                    int heads, const float* __restrict__ lse2, const float* __restrict__ dsum,
                    bf16_t* __restrict__ dqkv) {
  using TT = TrTile<HD>;
  constexpr int NC = HD / 16, NA = HD / 32;
  constexpr int RPI = 1024 / TT::ROWB;   // tile rows per 1 KB direct-to-LDS load
  constexpr int LPW = 64 / RPI / 4;      // query (and dO) loads per wave and tile
  static_assert(LPW >= 1 && LPW * RPI * 4 == 64, "tile / waves");
  __shared__ __attribute__((aligned(1024))) char sQ[BWD_ST][TT::BYTES];
  __shared__ __attribute__((aligned(1024))) char sdO[BWD_ST][TT::BYTES];
  __shared__ __attribute__((aligned(256))) float sL[BWD_ST][64];
  __shared__ __attribute__((aligned(256))) float sD[BWD_ST][64];
  const int total = gridDim.x, n_items = total / heads;
  const int wi = xcd_linear(blockIdx.x, total);
  const AttnItem it = items[wi % n_items];   // it.q0: first key of the block
  const int h = wi / n_items;
  const ImgDesc dsc = imgs[it.img];
  const int N = dsc.ntok, DM = heads * HD, ld3 = 3 * DM;
  const bf16_t* base = qkv + (size_t)dsc.tok_start * ld3 + h * HD;
  const bf16_t* dbase = dO_b + (size_t)dsc.tok_start * DM + h * HD;
  const int tid = threadIdx.x, lane = tid & 63, l32 = lane & 31, g = lane >> 5;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: LDS bases
  const int kw = it.q0 + 32 * wave;
  const bool wave_active = kw < N;
  const int k = kw + l32;
  const bool kok = k < N;
  const int kc = min(k, N - 1);
  bf16x8 kf[NC], vf[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    kf[c] = *reinterpret_cast<const bf16x8*>(base + DM + (size_t)kc * ld3 + 16 * c + 8 * g);
    vf[c] = *reinterpret_cast<const bf16x8*>(base + 2 * DM + (size_t)kc * ld3 + 16 * c + 8 * g);
  }
  // Wait for K and V with a wait the compiler sees, so its wait-count pass
  // does not hold the ring's loads back for them later.
  __builtin_amdgcn_s_waitcnt(0x0F70);
  const float sl2 = 1.4426950408889634f / sqrtf((float)HD);
  f32x16 dv[NA], dk[NA];
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int r = 0; r < 16; ++r) dv[a][r] = dk[a][r] = 0.f;
  // Load i of wave w fills rows RPI (LPW w + i) .. +RPI-1; lane l takes row
  // l / NCH of them and physical chunk l % NCH, i.e. logical chunk
  // (l % NCH) ^ f(row).  Wave 0 also loads the tile's 64 log-sum-exp and D
  // values (one per lane, stride `heads`).
  const i32x4 rq = buffer_rsrc(base, (uint64_t)N * ld3 * 2);
  const i32x4 rd = buffer_rsrc(dbase, (uint64_t)N * DM * 2);
  const size_t lbase = (size_t)dsc.tok_start * heads + h;
  const i32x4 rl = buffer_rsrc(lse2 + lbase, (uint64_t)N * heads * 4);
  const i32x4 rs = buffer_rsrc(dsum + lbase, (uint64_t)N * heads * 4);
  int goffQ[LPW], goffD[LPW];
#pragma unroll
  for (int i = 0; i < LPW; ++i) {
    const int row = (wave * LPW + i) * RPI + lane / TT::NCH;
    const int chunk = (lane % TT::NCH) ^ TT::f(row);
    goffQ[i] = row * ld3 * 2 + chunk * 16;
    goffD[i] = row * DM * 2 + chunk * 16;
  }
  const uint32_t ldsQ0 = lds_offset(&sQ[0][0]), ldsO0 = lds_offset(&sdO[0][0]);
  const uint32_t ldsL0 = lds_offset(&sL[0][0]), ldsD0 = lds_offset(&sD[0][0]);
  // Per-lane read offsets within a tile: rows (query half qb adds 32 rows,
  // which keep the permutation) and transposed reads (plus immediates).
  int roff[NC];
  uint32_t trb[NA];
#pragma unroll
  for (int c = 0; c < NC; ++c) roff[c] = TT::off(l32, 2 * c + g);
#pragma unroll
  for (int a = 0; a < NA; ++a) trb[a] = tr_lane_off<HD>(a, lane);
  auto issue = [&](int qt, int st) {
    const int q0 = qt * 64;
#pragma unroll
    for (int i = 0; i < LPW; ++i) {
      const uint32_t lo = st * TT::BYTES + (wave * LPW + i) * 1024;
      dma16(rq, ldsQ0 + lo, goffQ[i] + q0 * ld3 * 2, 0);
      dma16(rd, ldsO0 + lo, goffD[i] + q0 * DM * 2, 0);
    }
    if (wave == 0) {
      dma4(rl, ldsL0 + st * 256, (q0 + lane) * heads * 4, 0);
      dma4(rs, ldsD0 + st * 256, (q0 + lane) * heads * 4, 0);
    }
  };
  const int QT = (N + 63) / 64;
  auto tile = [&](auto stage, int qt) {
    constexpr int st = decltype(stage)::value;
    // Tile qt must have landed; tile qt+1's loads may stay in flight.
    if (qt + 1 < QT) {
      if (wave == 0) asm volatile("s_waitcnt vmcnt(%0)" ::"n"(2 * LPW + 2) : "memory");
      else asm volatile("s_waitcnt vmcnt(%0)" ::"n"(2 * LPW) : "memory");
    } else {
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    }
    lds_barrier();
    // Stage (st+2)%3 held tile qt-1, whose readers all passed the barrier.
    if (qt + 2 < QT) issue(qt + 2, (st + 2) % BWD_ST);
    if (!wave_active) return;
    const char* tQ = sQ[st];
    const char* tO = sdO[st];
    const float* cL = sL[st];
    const float* cD = sD[st];
    // The 64 queries as two halves of 32 (fewer live registers): for half qb,
    // s[r] = S[query q0 + qi][key k], qi = 32qb + 8(r/4) + 4g + r%4, then its
    // two 16-query chunks jj = 2qb, 2qb + 1 of dV^T += dO^T P, dK^T += Q^T dS.
#pragma unroll
    for (int qb = 0; qb < 2; ++qb) {
      f32x16 sc, dp;
#pragma unroll
      for (int r = 0; r < 16; ++r) sc[r] = dp[r] = 0.f;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int ro = roff[c] + 32 * qb * TT::ROWB;
        const bf16x8 qa = *reinterpret_cast<const bf16x8*>(tQ + ro);
        sc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(qa, kf[c], sc, 0, 0, 0);
        const bf16x8 da = *reinterpret_cast<const bf16x8*>(tO + ro);
        dp = __builtin_amdgcn_mfma_f32_32x32x16_bf16(da, vf[c], dp, 0, 0, 0);
      }
      // No masks: query rows past the image read as zero (Q, dO, the
      // log-sum-exp and D), so their p is 1 and their dS 0, and both meet
      // zero dO and Q rows; a lane past the last key holds key N-1's rows
      // (p <= 1) and its dK / dV are not stored.
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int qi = 32 * qb + 8 * (r >> 2) + 4 * g + (r & 3);
        const float p = __builtin_amdgcn_exp2f(fmaf(sc[r], sl2, -cL[qi]));
        sc[r] = p;
        dp[r] = p * (dp[r] - cD[qi]);
      }
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
        const int jj = 2 * qb + hh;
        const bf16x8 pf = pack8(sc, hh);
        const bf16x8 dsf = pack8(dp, hh);
#pragma unroll
        for (int a = 0; a < NA; ++a) {
          const uint32_t o = trb[a] + st * TT::BYTES + 16 * jj * TT::ROWB;
          dv[a] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(tr_read<HD>(ldsO0 + o), pf, dv[a], 0,
                                                          0, 0);
          dk[a] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(tr_read<HD>(ldsQ0 + o), dsf, dk[a], 0,
                                                          0, 0);
        }
      }
    }
  };
  issue(0, 0);
  if (QT > 1) issue(1, 1);
  for (int qt = 0; qt < QT; qt += BWD_ST) {
    tile(std::integral_constant<int, 0>(), qt);
    if (qt + 1 < QT) tile(std::integral_constant<int, 1>(), qt + 1);
    if (qt + 2 < QT) tile(std::integral_constant<int, 2>(), qt + 2);
  }
  if (!kok) return;
  const float scale = 1.0f / sqrtf((float)HD);
  bf16_t* out = dqkv + ((size_t)dsc.tok_start + k) * ld3 + h * HD;
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int rq4 = 0; rq4 < 4; ++rq4) {
      u32x2 pk;
      pk.x = pack_bf16x2(dk[a][4 * rq4 + 0] * scale, dk[a][4 * rq4 + 1] * scale);
      pk.y = pack_bf16x2(dk[a][4 * rq4 + 2] * scale, dk[a][4 * rq4 + 3] * scale);
      *reinterpret_cast<u32x2*>(out + DM + a * 32 + 8 * rq4 + 4 * g) = pk;
      pk.x = pack_bf16x2(dv[a][4 * rq4 + 0], dv[a][4 * rq4 + 1]);
      pk.y = pack_bf16x2(dv[a][4 * rq4 + 2], dv[a][4 * rq4 + 3]);
      *reinterpret_cast<u32x2*>(out + 2 * DM + a * 32 + 8 * rq4 + 4 * g) = pk;
    }
}

template <int HD>
static void launch_attn_bwd_mfma(const void* qkv, const void* o, const float* dO,
                                 const ImgDesc* imgs, const AttnItem* items64, int n_items64,
                                 const AttnItem* items128, int n_items128, int heads, void* dqkv,
                                 float* lse, float* dsum, hipStream_t s, bool lse_given,
                                 const bf16_t* dO_bf16) {
  dim3 gq(n_items128 * heads), bq(256);
  if (lse_given)
    hipLaunchKernelGGL((k_attn_bwd_dq_mfma<HD, true>), gq, bq, 0, s,
                       static_cast<const bf16_t*>(qkv), static_cast<const bf16_t*>(o), dO, imgs,
                       items128, heads, static_cast<bf16_t*>(dqkv), lse, dsum);
  else
    hipLaunchKernelGGL((k_attn_bwd_dq_mfma<HD, false>), gq, bq, 0, s,
                       static_cast<const bf16_t*>(qkv), static_cast<const bf16_t*>(o), dO, imgs,
                       items128, heads, static_cast<bf16_t*>(dqkv), lse, dsum);
  hipLaunchKernelGGL(k_attn_bwd_dkv_mfma<HD>, gq, bq, 0, s, static_cast<const bf16_t*>(qkv),
                     dO_bf16, imgs, items128, heads, lse, dsum, static_cast<bf16_t*>(dqkv));
}

template <typename T, int HD>
static void launch_attn_bwd(const void* qkv, const void* o, const float* dO, const ImgDesc* imgs,
                            const AttnItem* items, int n_items, int heads, void* dqkv, float* lse,
                            float* dsum, hipStream_t s) {
  dim3 grid(n_items, heads), block(256);
  hipLaunchKernelGGL((k_attn_bwd_dq<T, HD>), grid, block, 0, s, static_cast<const T*>(qkv),
                     static_cast<const T*>(o), dO, imgs, items, heads, static_cast<T*>(dqkv), lse,
                     dsum);
  hipLaunchKernelGGL((k_attn_bwd_dkv<T, HD>), grid, block, 0, s, static_cast<const T*>(qkv), dO,
                     imgs, items, heads, lse, dsum, static_cast<T*>(dqkv));
}

hipError_t attention_backward(const void* qkv, const void* o, bool bf16, const float* dO,
                              const ImgDesc* imgs, const AttnItem* items64, int n_items,
                              const AttnItem* items128, int n_items128, int heads, int head_dim,
                              void* dqkv, float* lse, float* dsum, hipStream_t s, bool lse_given,
                              const bf16_t* dO_bf16) {
  if (n_items <= 0) return hipSuccess;
  if ((lse_given || dO_bf16) && !bf16) return hipErrorInvalidValue;
  if (bf16 && (!dO_bf16 || !items128 || n_items128 <= 0)) return hipErrorInvalidValue;
  if (head_dim == 64) {
    if (bf16)
      launch_attn_bwd_mfma<64>(qkv, o, dO, imgs, items64, n_items, items128, n_items128, heads,
                               dqkv, lse, dsum, s, lse_given, dO_bf16);
    else launch_attn_bwd<float, 64>(qkv, o, dO, imgs, items64, n_items, heads, dqkv, lse, dsum, s);
  } else if (head_dim == 32) {
    if (bf16)
      launch_attn_bwd_mfma<32>(qkv, o, dO, imgs, items64, n_items, items128, n_items128, heads,
                               dqkv, lse, dsum, s, lse_given, dO_bf16);
    else launch_attn_bwd<float, 32>(qkv, o, dO, imgs, items64, n_items, heads, dqkv, lse, dsum, s);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ------------------------------------------------------ pooling head backward
// One workgroup per image: from the kept pre-normalisation embedding e and
// the embedding gradient, de; the class token's final LayerNorm recomputed
// (z, xh); dz = W_p^T de; the class row of dX; and the image's terms of the
// final LayerNorm's parameter gradients (dz * xh, dz), summed over images
// afterwards in image order.  D <= 1024 (four columns per thread), P <= 1024.
__global__ __launch_bounds__(256) void k_pool_bwd(const float* __restrict__ X,
                                                  const ImgDesc* __restrict__ imgs,
                                                  const float* __restrict__ e,
                                                  const float* __restrict__ demb,
                                                  const float* __restrict__ proj,
                                                  const float* __restrict__ gm,
                                                  const float* __restrict__ bt, float eps, int D,
                                                  int P, float* __restrict__ de_out,
                                                  float* __restrict__ z_out,
                                                  float* __restrict__ dX, float* __restrict__ pg,
                                                  float* __restrict__ pb) {
  __shared__ float red[4];
  __shared__ float sde[1024];
  const int i = blockIdx.x, tid = threadIdx.x;
  const float* er = e + (size_t)i * P;
  const float* dr = demb + (size_t)i * P;
  auto sum = [](float a, float b) { return a + b; };
  float n2 = 0.f, dot = 0.f;
  for (int p = tid; p < P; p += 256) {
    n2 += er[p] * er[p];
    dot += er[p] * dr[p];
  }
  n2 = block_reduce(n2, red, sum);
  dot = block_reduce(dot, red, sum);
  const float inv = 1.f / fmaxf(sqrtf(n2), 1e-12f);
  const float ehd = dot * inv;   // <e_hat, d e_hat>
  for (int p = tid; p < P; p += 256) {
    const float v = (dr[p] - er[p] * inv * ehd) * inv;
    sde[p] = v;
    de_out[(size_t)i * P + p] = v;
  }
  __syncthreads();
  const ImgDesc d = imgs[i];
  const float* xr = X + (size_t)d.tok_start * D;
  float s = 0.f;
  for (int c = tid; c < D; c += 256) s += xr[c];
  const float mean = block_reduce(s, red, sum) / D;
  float q = 0.f;
  for (int c = tid; c < D; c += 256) {
    const float v = xr[c] - mean;
    q += v * v;
  }
  const float rstd = rsqrtf(block_reduce(q, red, sum) / D + eps);
  float xh[4], dz[4];
  float a = 0.f, b = 0.f;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = tid + 256 * j;
    xh[j] = dz[j] = 0.f;
    if (c >= D) continue;
    xh[j] = (xr[c] - mean) * rstd;
    z_out[(size_t)i * D + c] = xh[j] * gm[c] + bt[c];
    float acc = 0.f;
    for (int p = 0; p < P; ++p) acc += proj[(size_t)p * D + c] * sde[p];
    dz[j] = acc;
    const float dxh = acc * gm[c];
    a += dxh;
    b += dxh * xh[j];
  }
  a = block_reduce(a, red, sum) / D;
  b = block_reduce(b, red, sum) / D;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = tid + 256 * j;
    if (c >= D) continue;
    dX[(size_t)d.tok_start * D + c] = rstd * (dz[j] * gm[c] - a - xh[j] * b);
    pg[(size_t)i * D + c] = dz[j] * xh[j];
    pb[(size_t)i * D + c] = dz[j];
  }
}

// dW_p[p][c] = sum over images (ascending) of de[i][p] z[i][c].
__global__ __launch_bounds__(256) void k_outer_sum(const float* __restrict__ de,
                                                   const float* __restrict__ z, int n, int P,
                                                   int D, float* __restrict__ out) {
  const int c = blockIdx.x * 256 + threadIdx.x, p = blockIdx.y;
  if (c >= D) return;
  float s = 0.f;
  for (int i = 0; i < n; ++i) s += de[(size_t)i * P + p] * z[(size_t)i * D + c];
  out[(size_t)p * D + c] = s;
}

hipError_t pool_backward(const float* X, const ImgDesc* imgs, int n, const float* e,
                         const float* demb, const float* proj, const float* g, const float* b,
                         float eps, int D, int P, float* de, float* z, float* dX, float* pg,
                         float* pb, float* part, float* d_proj, float* d_lnf_g, float* d_lnf_b,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_pool_bwd, dim3(n), dim3(256), 0, s, X, imgs, e, demb, proj, g, b, eps, D,
                     P, de, z, dX, pg, pb);
  hipLaunchKernelGGL(k_outer_sum, dim3((D + 255) / 256, P), dim3(256), 0, s, de, z, n, P, D,
                     d_proj);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  if ((err = colsum(pg, false, n, D, D, nullptr, part, d_lnf_g, s)) != hipSuccess) return err;
  return colsum(pb, false, n, D, D, nullptr, part, d_lnf_b, s);
}

hipError_t outer_sum(const float* a, const float* b, int n, int P, int D, float* out,
                     hipStream_t s) {
  if (n <= 0 || P <= 0 || D <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_outer_sum, dim3((D + 255) / 256, P), dim3(256), 0, s, a, b, n, P, D, out);
  return hipGetLastError();
}

// ------------------------------------------- attention-pooling head backward
// L2 normalisation and projection of the pooled rows: per image, from e
// [n, P] (before normalisation) and dL/d(e_hat) demb: de = (demb - e_hat
// <e_hat, demb>) / |e| and dz = W_p^T de [n, D] (W_p [P, D]).  P <= 1024.
__global__ __launch_bounds__(256) void k_l2proj_bwd(const float* __restrict__ e,
                                                    const float* __restrict__ demb,
                                                    const float* __restrict__ proj, int D, int P,
                                                    float* __restrict__ de_out,
                                                    float* __restrict__ dz) {
  __shared__ float red[4];
  __shared__ float sde[1024];
  const int i = blockIdx.x, tid = threadIdx.x;
  const float* er = e + (size_t)i * P;
  const float* dr = demb + (size_t)i * P;
  auto sum = [](float a, float b) { return a + b; };
  float n2 = 0.f, dot = 0.f;
  for (int p = tid; p < P; p += 256) {
    n2 += er[p] * er[p];
    dot += er[p] * dr[p];
  }
  n2 = block_reduce(n2, red, sum);
  dot = block_reduce(dot, red, sum);
  const float inv = 1.f / fmaxf(sqrtf(n2), 1e-12f);
  const float ehd = dot * inv;   // <e_hat, d e_hat>
  for (int p = tid; p < P; p += 256) {
    const float v = (dr[p] - er[p] * inv * ehd) * inv;
    sde[p] = v;
    de_out[(size_t)i * P + p] = v;
  }
  __syncthreads();
  for (int c = tid; c < D; c += 256) {
    float acc = 0.f;
    for (int p = 0; p < P; ++p) acc += proj[(size_t)p * D + c] * sde[p];
    dz[(size_t)i * D + c] = acc;
  }
}

hipError_t l2proj_backward(const float* e, const float* demb, const float* proj, int n, int D,
                           int P, float* de, float* dz, hipStream_t s) {
  if (n <= 0 || P > 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_l2proj_bwd, dim3(n), dim3(256), 0, s, e, demb, proj, D, P, de, dz);
  return hipGetLastError();
}

// One query per head over an image's tokens (the pooling head): with p =
// softmax(q_h k_t / sqrt(d)) over the image's tokens t, D = dO_h . o_h,
// dV_t = p_t dO_h, dS_t = p_t (dO_h . v_t - D), dK_t = dS_t q_h / sqrt(d),
// dq_h = sum_t dS_t k_t / sqrt(d).  One workgroup per (image, head); scores
// and dS in LDS (images of up to 4096 tokens), FP32 throughout; dK / dV
// written in kv's element type into dkv [T, 2D] = [dK | dV].
template <typename T>
__global__ __launch_bounds__(256) void k_map_attn_bwd(const T* __restrict__ kv,
                                                      const float* __restrict__ q,
                                                      const float* __restrict__ o,
                                                      const float* __restrict__ dO,
                                                      const ImgDesc* __restrict__ imgs, int heads,
                                                      int hd, T* __restrict__ dkv,
                                                      float* __restrict__ dq) {
  constexpr int kMaxN = 4096;
  __shared__ float sq[64], sdo[64], red[4];
  __shared__ float sp[kMaxN], sds[kMaxN];
  const int i = blockIdx.x, h = blockIdx.y, tid = threadIdx.x;
  const ImgDesc dsc = imgs[i];
  const int N = dsc.ntok, D = heads * hd, ld = 2 * D;
  const T* base = kv + (size_t)dsc.tok_start * ld + h * hd;
  T* obase = dkv + (size_t)dsc.tok_start * ld + h * hd;
  const float scale = 1.f / sqrtf((float)hd);
  if (tid < hd) {
    sq[tid] = q[h * hd + tid];
    sdo[tid] = dO[(size_t)i * D + h * hd + tid];
  }
  __syncthreads();
  auto sum = [](float a, float b) { return a + b; };
  auto mx = [](float a, float b) { return fmaxf(a, b); };
  float dd = tid < hd ? sdo[tid] * o[(size_t)i * D + h * hd + tid] : 0.f;
  const float Dsum = block_reduce(dd, red, sum);
  auto ld_f = [](const T* p) {
    if constexpr (sizeof(T) == 2) return bf16_bits_to_f32(*reinterpret_cast<const uint16_t*>(p));
    else return static_cast<float>(*p);
  };
  auto st_f = [](T* p, float v) {
    if constexpr (sizeof(T) == 2) *reinterpret_cast<uint16_t*>(p) = (uint16_t)f32_to_bf16_bits(v);
    else *p = v;
  };
  float m = -INFINITY;
  for (int t = tid; t < N; t += 256) {
    const T* kr = base + (size_t)t * ld;
    float acc = 0.f;
    for (int j = 0; j < hd; ++j) acc += sq[j] * ld_f(kr + j);
    const float sc = acc * scale;
    sp[t] = sc;
    m = fmaxf(m, sc);
  }
  m = block_reduce(m, red, mx);
  float l = 0.f;
  for (int t = tid; t < N; t += 256) {
    const float e = expf(sp[t] - m);
    sp[t] = e;
    l += e;
  }
  l = block_reduce(l, red, sum);
  const float il = 1.f / l;
  for (int t = tid; t < N; t += 256) {
    const float p = sp[t] * il;
    const T* vr = base + D + (size_t)t * ld;
    float dp = 0.f;
    for (int j = 0; j < hd; ++j) dp += sdo[j] * ld_f(vr + j);
    const float ds = p * (dp - Dsum);
    sds[t] = ds;
    T* kr = obase + (size_t)t * ld;
    for (int j = 0; j < hd; ++j) {
      st_f(kr + j, ds * sq[j] * scale);
      st_f(kr + D + j, p * sdo[j]);
    }
  }
  __syncthreads();
  for (int j = tid; j < hd; j += 256) {
    float acc = 0.f;
    for (int t = 0; t < N; ++t) acc += sds[t] * ld_f(base + (size_t)t * ld + j);
    dq[(size_t)i * D + h * hd + j] = acc * scale;
  }
}

hipError_t map_attention_backward(const void* kv, bool kv_bf16, const float* q, const float* o,
                                  const float* dO, const ImgDesc* imgs, int n, int max_ntok,
                                  int heads, int hd, void* dkv, float* dq, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (hd > 64 || max_ntok > 4096) return hipErrorInvalidValue;
  dim3 grid(n, heads), block(256);
  if (kv_bf16)
    hipLaunchKernelGGL(k_map_attn_bwd<bf16_t>, grid, block, 0, s, static_cast<const bf16_t*>(kv),
                       q, o, dO, imgs, heads, hd, static_cast<bf16_t*>(dkv), dq);
  else
    hipLaunchKernelGGL(k_map_attn_bwd<float>, grid, block, 0, s, static_cast<const float*>(kv), q,
                       o, dO, imgs, heads, hd, static_cast<float*>(dkv), dq);
  return hipGetLastError();
}

// ------------------------------------------------- token embedding backward
// Position table rows (images at the base grid, so token j of every image
// uses row j): dpos[j] = sum over images of dX[tok_start + j]; row 0 is also
// the class token's gradient.
__global__ __launch_bounds__(256) void k_pos_grad(const float* __restrict__ dX,
                                                  const ImgDesc* __restrict__ imgs, int n, int D,
                                                  float* __restrict__ dpos,
                                                  float* __restrict__ dcls) {
  const int c = blockIdx.x * 256 + threadIdx.x, j = blockIdx.y;
  if (c >= D) return;
  float s = 0.f;
  for (int i = 0; i < n; ++i) s += dX[(size_t)(imgs[i].tok_start + j) * D + c];
  dpos[(size_t)j * D + c] = s;
  if (j == 0) dcls[c] = s;
}

// Patch weights: the forward multiplies raw pixels by W / std (folded), so
// dW[d][k] = (dWf[d][k] - mean_c db[d]) / std_c with c = k / (P*P), where dWf
// is the gradient of the folded weights and db that of the patch bias.
__global__ __launch_bounds__(256) void k_patch_w_grad(const float* __restrict__ dwf, int kpad,
                                                      const float* __restrict__ db, ChanNorm cn,
                                                      int kpe, int pp, int D,
                                                      float* __restrict__ out) {
  const int k = blockIdx.x * 256 + threadIdx.x, dd = blockIdx.y;
  if (k >= kpe || dd >= D) return;
  const int c = k / pp;
  out[(size_t)dd * kpe + k] = (dwf[(size_t)dd * kpad + k] - cn.mean[c] * db[dd]) / cn.std[c];
}

hipError_t embed_backward(const float* dX, const ImgDesc* imgs, int n, int D, int rows_pos,
                          const float* dwf, int kpad, const float* db, ChanNorm cn, int kpe,
                          int pp, float* d_pos, float* d_cls, float* d_patch_w, hipStream_t s) {
  hipLaunchKernelGGL(k_pos_grad, dim3((D + 255) / 256, rows_pos), dim3(256), 0, s, dX, imgs, n, D,
                     d_pos, d_cls);
  hipLaunchKernelGGL(k_patch_w_grad, dim3((kpe + 255) / 256, D), dim3(256), 0, s, dwf, kpad, db,
                     cn, kpe, pp, D, d_patch_w);
  return hipGetLastError();
}

// ------------------------------------------------------------------- misc
__global__ __launch_bounds__(256) void k_sum_splits(const float* __restrict__ part, int splits,
                                                    size_t n, float* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int z = 0; z < splits; ++z) s += part[(size_t)z * n + i];
  out[i] = s;
}

// Four consecutive elements per lane (16-byte loads and stores); the sum of
// each element runs over the splits in the same ascending order as above.
__global__ __launch_bounds__(256) void k_sum_splits4(const float4* __restrict__ part, int splits,
                                                     size_t n4, float4* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n4) return;
  float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll 4
  for (int z = 0; z < splits; ++z) {
    const float4 v = part[(size_t)z * n4 + i];
    s.x += v.x;
    s.y += v.y;
    s.z += v.z;
    s.w += v.w;
  }
  out[i] = s;
}

hipError_t sum_splits(const float* part, int splits, size_t n, float* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const bool vec = n % 4 == 0 && reinterpret_cast<uintptr_t>(part) % 16 == 0 &&
                   reinterpret_cast<uintptr_t>(out) % 16 == 0;
  if (vec) {
    const size_t n4 = n / 4;
    hipLaunchKernelGGL(k_sum_splits4, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, s,
                       reinterpret_cast<const float4*>(part), splits, n4,
                       reinterpret_cast<float4*>(out));
  } else {
    hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, part,
                       splits, n, out);
  }
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_fill_zero(float* __restrict__ p, size_t n) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

hipError_t fill_zero(float* p, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace vl
