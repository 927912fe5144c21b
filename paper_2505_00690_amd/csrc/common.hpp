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

// The same GELU with erf from Abramowitz & Stegun, Handbook of Mathematical
// Functions, formula 7.1.26 (|error of erf| <= 1.5e-7): for z >= 0,
// erf(z) = 1 - (a1 t + a2 t^2 + a3 t^3 + a4 t^4 + a5 t^5) exp(-z^2),
// t = 1 / (1 + p z), odd extension for z < 0.  Branch-free, one reciprocal
// and one exp2; in FP32 the GELU error stays below 5e-7 absolute, far under
// the BF16 rounding of the outputs it feeds.  Used where the GEMM output is
// BF16; the FP32 path keeps erff.
__device__ __forceinline__ float gelu_as7126(float x) {
  const float z = x * 0.70710678118654752f;
  const float az = fabsf(z);
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, az, 1.0f));
  float poly = fmaf(1.061405429f, t, -1.453152027f);
  poly = fmaf(poly, t, 1.421413741f);
  poly = fmaf(poly, t, -0.284496736f);
  poly = fmaf(poly, t, 0.254829592f);
  poly *= t;
  const float e = __builtin_amdgcn_exp2f(-(az * az) * 1.4426950408889634f);
  const float erf_abs = fmaf(-poly, e, 1.0f);
  const float erf_z = __builtin_copysignf(erf_abs, z);
  return 0.5f * x * (1.0f + erf_z);
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

}  // namespace vl
