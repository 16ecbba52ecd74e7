// fp16 vector types and the hi / lo fp16 split used to run FP32-accurate products on
// the fp16 matrix cores: x = hi + lo with hi = x rounded to fp16 and lo = (x - hi)
// rounded, about 2^-22 relative.  Products of halves are exact in fp32, so
// hi*hi + hi*lo + lo*hi accumulated in fp32 matches an fp32 product sum to ~1e-7
// relative.
#pragma once

namespace rsv {

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef float float2_t __attribute__((ext_vector_type(2)));
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef float float4_a4 __attribute__((ext_vector_type(4), aligned(4)));  // 4-byte-aligned loads

// The residuals x - hi are taken by mixed-precision FMAs straight from the packed
// halves (-hi * 1 + x, exact since hi is x rounded to 11 bits), which saves the two
// conversions back to fp32.
__device__ __forceinline__ void split2(float a, float b, half2_t& hi, half2_t& lo) {
  const float2_t x = {a, b};
  hi = __builtin_convertvector(x, half2_t);
  float ra, rb;
  asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(ra) : "v"(hi), "v"(a));
  asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(rb) : "v"(hi), "v"(b));
  lo = __builtin_convertvector(float2_t{ra, rb}, half2_t);
}

// fp16 hi / lo split of four costs: c = hi + lo to about 2^-22 relative.
__device__ __forceinline__ void split4(const float4_t& c, half4_t& hi, half4_t& lo) {
  half2_t h0, l0, h1, l1;
  split2(c[0], c[1], h0, l0);
  split2(c[2], c[3], h1, l1);
  hi[0] = h0[0]; hi[1] = h0[1]; hi[2] = h1[0]; hi[3] = h1[1];
  lo[0] = l0[0]; lo[1] = l0[1]; lo[2] = l1[0]; lo[3] = l1[1];
}

}  // namespace rsv
