// FF_mul on the FP64 units: an alternative instruction mix for the
// Montgomery product.
//
// The paper finds the INT32 pipes of its GPUs saturated by FF_mul while the
// floating-point pipes sit idle, and leaves their use open (Sections IV-B,
// IV-C and V-C).  This is that variant for gfx950: every partial product of
// the Montgomery multiplication is computed on v_fma_f64 instead of
// v_mad_u64_u32, with the operands cut into 48-bit limbs (six limbs, 288
// bits) so that each limb product is below 2^96 and fits the error-free
// product transformation of a fused multiply-add (Ogita, Rump and Oishi,
// "Accurate sum and dot product", SIAM J. Sci. Comput. 2005; applied to
// multiprecision modular multiplication on GPUs by Emmart, Zheng and Weems,
// "Faster modular exponentiation using double precision floating point
// arithmetic on the GPU", ARITH 2018).
//
// Accumulation.  Each column of the product scan keeps two doubles: H, pinned
// to the binade [2^100, 2^101) by starting at C = 2^100, so that every fused
// multiply-add H' = fma(x, y, H) rounds to a multiple of 2^48; and L, which
// collects what each rounding dropped.  One partial product x y (x, y < 2^48)
// is four instructions:
//     H' = fma(x, y, H);  d = H' - H  (exact);  e = fma(x, y, -d)  (exact,
//     |e| <= 2^47);  L = L + e  (exact while |L| < 2^53);  H = H'
// and the column's value is (H - C) + L.  A column holds at most 12 products
// (six of a b, six of m p), so H stays below C + 0.75 2^100 and |L| below
// 2^53 with the carry from the previous column.
//
// Reduction.  Montgomery reduction in radix 2^48 interleaved with the product
// scan (finely integrated product scanning, as the integer FF_mul): the digit
// m_k = (column_k mod 2^48) p' mod 2^48, p' = -p^-1 mod 2^48, is itself one
// error-free product.  The result is a b 2^-288 mod p, in [0, 2p) before the
// final conditional subtraction: with R' = 2^288 the second operand must be
// held as y 2^288 mod p (plans that use this multiplier store their tables
// that way), so that the product of data in the 2^256 Montgomery form and
// such a table entry is again in the 2^256 form.
//
// Every step is exact: the result equals the integer FF_mul's, bit for bit.
#pragma once
#include <cstdint>

#include "field.hpp"

namespace zk {

constexpr int kF64Limbs = 6;
constexpr int kF64Bits = 48;

// 48-bit limb j of the 256-bit value given as eight 32-bit words.
constexpr __host__ __device__ uint64_t limb48(const uint32_t w[kLimbs], int j) {
  const int lo = kF64Bits * j;
  uint64_t r = 0;
  for (int b = 0; b < kF64Bits; ++b) {
    const int bit = lo + b;
    if (bit < 32 * kLimbs && ((w[bit / 32] >> (bit % 32)) & 1u)) r |= 1ull << b;
  }
  return r;
}

// -p^-1 mod 2^48 by Newton's iteration x <- x (2 - p x), which doubles the
// number of correct low bits each step (p is odd, so x = 1 is right mod 2).
template <class F>
constexpr uint64_t f64_pinv() {
  const uint64_t mask = (1ull << kF64Bits) - 1;
  const uint64_t p0 = limb48(F::P, 0);
  uint64_t x = 1;
  for (int i = 0; i < 6; ++i) x = (x * (2 - p0 * x)) & mask;
  return (0 - x) & mask;
}

namespace f64 {

constexpr double kC = 1267650600228229401496703205376.0;  // 2^100
constexpr double kBeta = 281474976710656.0;               // 2^48
constexpr double kInvBeta = 1.0 / 281474976710656.0;      // 2^-48 (exact)
constexpr double kTwo52 = 4503599627370496.0;             // 2^52

// An integer below 2^52 as a double: the bit pattern of 2^52 + v, minus 2^52.
__host__ __device__ __forceinline__ double u52_to_double(uint64_t v) {
  return __builtin_bit_cast(double, 0x4330000000000000ull | v) - kTwo52;
}
// An integer-valued double in [0, 2^52) back to its bits.
__host__ __device__ __forceinline__ uint64_t double_to_u52(double d) {
  return __builtin_bit_cast(uint64_t, d + kTwo52) & ((1ull << 52) - 1);
}

__host__ __device__ __forceinline__ void split(const Fe& a, double x[kF64Limbs]) {
  const uint64_t m16 = 0xffffull;
  x[0] = u52_to_double((uint64_t)a.v[0] | ((uint64_t)a.v[1] & m16) << 32);
  x[1] = u52_to_double((uint64_t)(a.v[1] >> 16) | (uint64_t)a.v[2] << 16);
  x[2] = u52_to_double((uint64_t)a.v[3] | ((uint64_t)a.v[4] & m16) << 32);
  x[3] = u52_to_double((uint64_t)(a.v[4] >> 16) | (uint64_t)a.v[5] << 16);
  x[4] = u52_to_double((uint64_t)a.v[6] | ((uint64_t)a.v[7] & m16) << 32);
  x[5] = u52_to_double((uint64_t)(a.v[7] >> 16));
}

// Add x y to the column (H, L) exactly.
__host__ __device__ __forceinline__ void acc(double x, double y, double& H, double& L) {
  const double h = __builtin_fma(x, y, H);
  const double d = h - H;
  const double e = __builtin_fma(x, y, -d);
  L += e;
  H = h;
}

// v mod 2^48 for an integer-valued double v (|v| < 2^53): in [0, 2^48).
__host__ __device__ __forceinline__ double mod_beta(double v, double& quot) {
  quot = __builtin_floor(v * kInvBeta);
  return __builtin_fma(-kBeta, quot, v);
}

}  // namespace f64

// a b 2^-288 mod p, canonical.  a < 2^256, b < p.
template <class F>
__host__ __device__ __forceinline__ Fe mul_f64(const Fe& a, const Fe& b) {
  using namespace f64;
  constexpr double pinv = (double)f64_pinv<F>();
  constexpr double P0 = (double)limb48(F::P, 0), P1 = (double)limb48(F::P, 1), P2 = (double)limb48(F::P, 2),
                   P3 = (double)limb48(F::P, 3), P4 = (double)limb48(F::P, 4), P5 = (double)limb48(F::P, 5);
  const double P[kF64Limbs] = {P0, P1, P2, P3, P4, P5};
  double x[kF64Limbs], y[kF64Limbs], m[kF64Limbs], r[kF64Limbs];
  split(a, x);
  split(b, y);
  double carry = 0;
#pragma unroll
  for (int k = 0; k < 2 * kF64Limbs; ++k) {
    double H = kC, L = carry;
#pragma unroll
    for (int i = 0; i < kF64Limbs; ++i) {
      const int j = k - i;
      if (j >= 0 && j < kF64Limbs) acc(x[i], y[j], H, L);
    }
#pragma unroll
    for (int i = 0; i < kF64Limbs; ++i) {
      const int j = k - i;
      if (i < k && j >= 0 && j < kF64Limbs) acc(m[i], P[j], H, L);
    }
    if (k < kF64Limbs) {
      // digit m_k zeroes this column mod 2^48; the column's value is
      // (H - C) + L with H - C a multiple of 2^48, so only L matters
      double q;
      const double lm = mod_beta(L, q);
      double ph = kC, pl = 0;
      acc(lm, pinv, ph, pl);  // lm p' = (ph - C) + pl with ph - C = 0 mod 2^48
      double q2;
      m[k] = mod_beta(pl, q2);
      acc(m[k], P[0], H, L);
      carry = (H - kC) * kInvBeta + L * kInvBeta;  // both exact integers
    } else {
      double q;
      r[k - kF64Limbs] = mod_beta(L, q);
      carry = (H - kC) * kInvBeta + q;
    }
  }
  // r < 2p < 2^256: repack six 48-bit limbs into eight 32-bit words
  uint64_t u[kF64Limbs];
#pragma unroll
  for (int i = 0; i < kF64Limbs; ++i) u[i] = double_to_u52(r[i]);
  uint32_t t[kLimbs];
  t[0] = (uint32_t)u[0];
  t[1] = (uint32_t)(u[0] >> 32) | (uint32_t)(u[1] << 16);
  t[2] = (uint32_t)(u[1] >> 16);
  t[3] = (uint32_t)u[2];
  t[4] = (uint32_t)(u[2] >> 32) | (uint32_t)(u[3] << 16);
  t[5] = (uint32_t)(u[3] >> 16);
  t[6] = (uint32_t)u[4];
  t[7] = (uint32_t)(u[4] >> 32) | (uint32_t)(u[5] << 16);
  return reduce_once<F>(t);
}

// BLS12-381 Fr with every product on the FP64 multiplier.  Plans of this
// variant hold their tables (the second operand of every product) as
// y 2^288 mod p; data stays in the 2^256 Montgomery form.
struct Bls12_381FrF64 : Bls12_381Fr {
  static constexpr bool kAltMul = true;
  __host__ __device__ static __forceinline__ Fe mul(const Fe& a, const Fe& b) { return mul_f64<Bls12_381Fr>(a, b); }
};

}  // namespace zk
