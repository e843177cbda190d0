// Exact arithmetic on residues modulo p, 2 < p < 2^31, in 32-bit lanes.
//
// Sums of two residues stay below 2^32 because p < 2^31 (the reason the
// paper picks primes below 2^31, Sec. 3.5), so one conditional subtraction
// reduces them; min(s, s - p) is that subtraction without a branch (if
// s < p, s - p wraps above 2^31 > s).
//
// Products by a per-instance constant c use Shoup's precomputed-quotient
// method (V. Shoup, NTL MulModPrecon; D. Harvey, "Faster arithmetic for
// number-theoretic transforms", J. Symb. Comp. 2014): with c' = floor(c 2^32
// / p), r = c x - floor(c' x / 2^32) p lies in [0, 2p).
//
// Products of two variable residues (the read-out dot product) use
// Montgomery reduction (P. Montgomery, Math. Comp. 44, 1985) with R = 2^32:
// redc(x * y) = x y R^{-1} mod p, so one operand is kept premultiplied by R.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cs {

__device__ __forceinline__ uint32_t add_mod(uint32_t a, uint32_t b, uint32_t p) {
  uint32_t s = a + b;
  return min(s, s - p);
}

__device__ __forceinline__ uint32_t sub_mod(uint32_t a, uint32_t b, uint32_t p) {
  uint32_t d = a - b;
  return min(d, d + p);
}

// c * x mod p, c < p, cs = floor(c * 2^32 / p), any x < 2^32.
__device__ __forceinline__ uint32_t mul_shoup(uint32_t x, uint32_t c, uint32_t cs, uint32_t p) {
  uint32_t qh = __umulhi(cs, x);
  uint32_t r = c * x - qh * p;
  return min(r, r - p);
}

// x * y * 2^-32 mod p for x, y < p; pinv = -p^{-1} mod 2^32.
__device__ __forceinline__ uint32_t mul_redc(uint32_t x, uint32_t y, uint32_t p, uint32_t pinv) {
  uint32_t tlo = x * y;
  uint32_t thi = __umulhi(x, y);
  uint32_t mq = tlo * pinv;
  uint32_t mh = __umulhi(mq, p);
  // tlo + low(mq p) is 0 mod 2^32; it carries out exactly when tlo != 0.
  uint32_t r = thi + mh + (tlo != 0u ? 1u : 0u);
  return min(r, r - p);
}

}  // namespace cs
