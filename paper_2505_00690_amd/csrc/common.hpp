// Shared device-side types and helpers for the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vl {

typedef uint16_t bf16_t;  // BF16 bit pattern
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// FP32 -> BF16, round to nearest even (inputs are finite).
__device__ __forceinline__ uint32_t f32_to_bf16_bits(float x) {
  uint32_t b = __float_as_uint(x);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return b >> 16;
}
// Two FP32 -> packed BF16 pair, round to nearest even (v_cvt_pk_bf16_f32).
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
  const f32x2 v = {lo, hi};
  const bf16x2 h = __builtin_convertvector(v, bf16x2);
  return __builtin_bit_cast(uint32_t, h);
}
__device__ __forceinline__ float bf16_bits_to_f32(uint32_t h) {
  return __uint_as_float(h << 16);
}

// OCP e4m3fn code (byte) -> BF16 bits.  Exact: every e4m3 value has a BF16
// representation.  Normal codes (exponent field e >= 1) map to BF16 exponent
// e + 120 with the 3 significand bits shifted up by 4; subnormal codes
// (e == 0) are m * 2^-9.
__device__ __forceinline__ uint32_t e4m3_to_bf16_bits(uint32_t b) {
  uint32_t s = (b & 0x80u) << 8;
  uint32_t mag = b & 0x7Fu;
  uint32_t r;
  if (mag >= 8u) {
    r = (mag << 4) + 0x3C00u;
  } else {
    r = __float_as_uint((float)mag * 0.001953125f) >> 16;
  }
  return s | r;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

// GELU(x) = x * Phi(x) = x/2 * (1 + erf(x / sqrt 2)), exact-erf form.
__device__ __forceinline__ float gelu_erf(float x) {
  return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f));
}

// GELU(x) = x * Phi(x) for the BF16-output epilogue, with all-FMA-pipe
// arithmetic: Phi(x) - 1/2 ~= t * P(t^2), t = x clamped to [-4.5, 4.5], P an
// even-power polynomial of degree 8 in t^2 (coefficients from
// fit_gelu_poly.py; |error| of Phi <= 2.5e-5 including the clamp, i.e. a
// relative GELU error far below the BF16 rounding of the output), evaluated
// as x * (1/2 + t P(t^2)).  The FP32 path keeps erff.
// Phi(x) = 1/2 + t P(t^2) as above (the GELU backward uses it too).
__device__ __forceinline__ float phi_poly(float x) {
  const float t = __builtin_amdgcn_fmed3f(x, -4.5f, 4.5f);
  const float u = t * t;
  float p = 3.806312210e-11f;
  p = fmaf(p, u, -4.002815412e-09f);
  p = fmaf(p, u, 1.846330520e-07f);
  p = fmaf(p, u, -4.960022125e-06f);
  p = fmaf(p, u, 8.727943350e-05f);
  p = fmaf(p, u, -1.076754532e-03f);
  p = fmaf(p, u, 9.729534388e-03f);
  p = fmaf(p, u, -6.624048948e-02f);
  p = fmaf(p, u, 3.988665044e-01f);
  return fmaf(t, p, 0.5f);
}
__device__ __forceinline__ float gelu_poly(float x) { return x * phi_poly(x); }

// ------------- MXFP8 blocks (OCP Microscaling Formats (MX) Specification v1.0)
// 32 consecutive values along K share one E8M0 scale 2^X (byte X + 127) and
// are stored as e4m3 codes of v / 2^X.  X = floor(log2 amax) - 8 (8 is the
// largest e4m3 exponent), clamped below at -127; for an FP32 amax that is its
// biased exponent field minus 8.  v / 2^X then lies below 512 in magnitude
// and is saturated at 448 before rounding to nearest even.
//
// Scale layout of an [R, K] operand: block-major, [K/128][R][4] bytes, the
// four blocks of a 128-wide K tile in the order 0, 2, 1, 3, so a GEMM loads a
// K tile's scales for consecutive rows as one contiguous run and the 16-bit
// half g of a word holds the scales of blocks g and 2 + g.
__device__ __forceinline__ uint32_t mx_scale_byte(float amax) {
  const int e = (int)((__float_as_uint(amax) >> 23) & 0xFFu);
  return (uint32_t)(e > 8 ? e - 8 : 0);
}
// 2^-X for scale byte sb (always a normal FP32 value for sb <= 253).
__device__ __forceinline__ float mx_inv_scale(uint32_t sb) {
  return __uint_as_float((254u - sb) << 23);
}
// Four values times inv -> four e4m3 codes (byte i = value i), saturating,
// round to nearest even (v_cvt_pk_fp8_f32).
__device__ __forceinline__ uint32_t mx_pack4(float a, float b, float c, float d, float inv) {
  a = __builtin_amdgcn_fmed3f(a * inv, -448.f, 448.f);
  b = __builtin_amdgcn_fmed3f(b * inv, -448.f, 448.f);
  c = __builtin_amdgcn_fmed3f(c * inv, -448.f, 448.f);
  d = __builtin_amdgcn_fmed3f(d * inv, -448.f, 448.f);
  uint32_t w = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(c, d, (int)w, true);
}
// Byte offset of the scale of row r, column c in an operand of R rows.
__device__ __forceinline__ size_t mx_scale_off(int r, int c, int R) {
  const int b = (c >> 5) & 3;
  return ((size_t)(c >> 7) * R + r) * 4 + (((b & 1) << 1) | (b >> 1));
}
// Maximum over the 8 lanes of an aligned group of 8 (DPP within rows).
__device__ __forceinline__ float max8(float v) {
  v = fmaxf(v, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true)));
  v = fmaxf(v, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, true)));
  v = fmaxf(v, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x141, 0xF, 0xF, true)));
  return v;
}

// ------------------------------------------------ direct-to-LDS loads (gfx950)
// buffer_load_dwordx4 ... lds: 16 bytes per lane go from global memory
// straight into LDS (no VGPR round trip).  The buffer resource bounds the
// access: offsets at or past num_records read as zero.
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

// LDS byte offset of a __shared__ object.  A generic pointer into LDS is the
// shared aperture base (high 32 bits) plus the LDS offset (low 32 bits), so
// truncation yields the offset without the null check an address-space cast
// would add.
__device__ __forceinline__ uint32_t lds_offset(const void* p) {
  return static_cast<uint32_t>(reinterpret_cast<uintptr_t>(p));
}

// One 16-byte-per-lane direct-to-LDS load: lane i's 16 bytes from
// rsrc + voffset + soffset land at LDS byte lds + 16 i (lds and soffset
// wave-uniform).  Issued as inline assembly so the compiler's wait-count pass
// does not treat it as an LDS store and force vmcnt(0) before every later LDS
// read; the kernels wait for these loads themselves (s_waitcnt vmcnt(n)
// before their barrier).
__device__ __forceinline__ void dma16(i32x4 rsrc, uint32_t lds, int voffset, int soffset) {
  asm volatile("s_mov_b32 m0, %0\n\tbuffer_load_dwordx4 %1, %2, %3 offen lds"
               :
               : "s"(lds), "v"(voffset), "s"(rsrc), "s"(soffset)
               : "memory", "m0");
}

// The same with 4 bytes per lane: lane i's dword lands at LDS byte lds + 4 i.
__device__ __forceinline__ void dma4(i32x4 rsrc, uint32_t lds, int voffset, int soffset) {
  asm volatile("s_mov_b32 m0, %0\n\tbuffer_load_dword %1, %2, %3 offen lds"
               :
               : "s"(lds), "v"(voffset), "s"(rsrc), "s"(soffset)
               : "memory", "m0");
}

// Workgroup barrier without the compiler's memory fence (which would also
// wait for every outstanding global load): LDS reads of this wave are
// drained first, global-to-LDS loads are waited for explicitly by callers.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

__device__ __forceinline__ i32x4 buffer_rsrc(const void* base, uint64_t bytes) {
  const uint64_t p = reinterpret_cast<uint64_t>(base);
  i32x4 r;
  r[0] = (int32_t)(uint32_t)(p & 0xffffffffu);
  r[1] = (int32_t)(uint32_t)(p >> 32);        // stride 0
  r[2] = (int32_t)(uint32_t)(bytes > 0xffffffffull ? 0xffffffffull : bytes);
  r[3] = 0x00020000;
  r[0] = __builtin_amdgcn_readfirstlane(r[0]);
  r[1] = __builtin_amdgcn_readfirstlane(r[1]);
  r[2] = __builtin_amdgcn_readfirstlane(r[2]);
  return r;
}

// Reduction over a 256-thread workgroup (4 waves) with `op`; every thread
// gets the result.  red: 4 floats of LDS.  Safe to call back to back (the
// first barrier waits for the previous call's readers).
template <typename Op>
__device__ __forceinline__ float block_reduce(float v, float* red, Op op) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = op(v, __shfl_xor(v, o, 64));
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  v = op(op(red[0], red[1]), op(red[2], red[3]));
  return v;
}

// Workgroup ids are dealt round-robin to the 8 XCDs, and a kernel that gives
// each XCD a contiguous range of `total` items hands XCD x total / 8 of them,
// plus one when x < total % 8.  When the grid has more workgroups than
// `total` (a launch sized for a capacity), the live workgroups of XCD x are
// those with bid / 8 below that count, and all of them exist in any grid of
// at least `total` workgroups.
__device__ __forceinline__ bool xcd_live(int bid, int total) {
  const int xcd = bid & 7, local = bid >> 3;
  return local < (total >> 3) + (xcd < (total & 7) ? 1 : 0);
}

// The position of workgroup bid in an order that gives each XCD a contiguous
// range of `total` items: XCD x takes items x * (total / 8) + min(x, total %
// 8) onwards, in the order its workgroups arrive.
__device__ __forceinline__ int xcd_linear(int bid, int total) {
  const int xcd = bid & 7, local = bid >> 3;
  const int q = total >> 3, r = total & 7;
  return xcd * q + min(xcd, r) + local;
}

}  // namespace vl
