// FP32 -> BF16 and FP32 -> FP16 conversions, round to nearest with ties to
// even, written on the FP32 bit pattern.  The matrix-core stencil rounds its
// operands with these so that the rounding rule is exactly the documented
// one: values first rounded to FP32, then to the 16-bit format.  (A plain
// cast chain double -> float -> half may be carried out as one rounding from
// double, which differs on FP32 values that sit exactly on a 16-bit tie.)
// Host-compilable so that a CPU test can check them bit for bit.
#pragma once

#if defined(__HIPCC__)
#define MRHS_RND_QUAL __host__ __device__ __forceinline__
#else
#define MRHS_RND_QUAL inline
#endif

namespace mrhs {

MRHS_RND_QUAL unsigned short bf16_rne_bits(unsigned u) {
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

MRHS_RND_QUAL unsigned short f16_rne_bits(unsigned u) {
  const unsigned sign = (u >> 16) & 0x8000u;
  const unsigned a = u & 0x7fffffffu;
  if (a >= 0x7f800000u) return (unsigned short)(sign | 0x7c00u | (a > 0x7f800000u ? 0x200u : 0u));
  if (a >= 0x477ff000u) return (unsigned short)(sign | 0x7c00u);  // >= 65520 rounds to infinity
  if (a < 0x38800000u) {                                         // below 2^-14: subnormal or zero
    const unsigned e = a >> 23;
    if (e < 102u) return (unsigned short)sign;  // below 2^-25 (2^-25 itself ties to 0)
    const unsigned m = (a & 0x7fffffu) | 0x800000u;
    const unsigned s = 126u - e;  // k = m / 2^s in units of 2^-24, s in [14, 24]
    unsigned k = m >> s;
    const unsigned rem = m & ((1u << s) - 1u), half = 1u << (s - 1u);
    if (rem > half || (rem == half && (k & 1u))) ++k;
    return (unsigned short)(sign | k);
  }
  unsigned r = a - 0x38000000u;  // rebias the exponent from 127 to 15
  r += 0xfffu + ((r >> 13) & 1u);
  return (unsigned short)(sign | (r >> 13));
}

}  // namespace mrhs
