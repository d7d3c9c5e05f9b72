// Prime-field arithmetic for 255-bit scalar fields on gfx950.
//
// An element is eight 32-bit limbs, little-endian (limb 0 least
// significant), in Montgomery form with R = 2^256, canonical in [0, p).
//
// The paper's finite-field layer (Section IV-B) names the operations used by
// the NTT butterflies: FF_add, FF_sub and FF_mul, with FF_mul and FF_sqr
// taking almost all of the NTT's time.  It attributes most of the add/sub
// latency to the branches that decide the conditional reduction (Section
// IV-B and the micro-architecture analysis of Section IV-C); here every
// reduction is a branchless borrow-select, so the lanes of a wavefront never
// diverge.
//
// FF_mul on the device is Montgomery multiplication in the finely integrated
// product scanning (FIPS) order of Koc, Acar and Kaliski, "Analyzing and
// comparing Montgomery multiplication algorithms" (IEEE Micro, 1996): the
// 512-bit product and the reduction m * p are accumulated column by column in
// a 64-bit accumulator plus a small overflow counter.  Each 32x32-bit partial
// product is one v_mad_u64_u32 whose carry-out goes straight into the counter
// with v_addc_co_u32, so a column costs two instructions per partial product
// and no compare/select.  On gfx950 v_mad_u64_u32 issues at the full VALU
// rate, so instruction count, not multiplier throughput, sets the cost.
//
// The portable CIOS form (mul_portable) runs on the host for plan-time
// constants; both forms compute the same canonical result.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <type_traits>

namespace zk {

constexpr int kLimbs = 8;

// A field type may bring its own Montgomery multiplier (F::kAltMul = true,
// F::mul(a, b)): mul and mul_k below then call it instead of the integer
// FIPS product (field_f64.hpp uses this for the FP64 variant).
template <class F, class = void>
struct HasAltMul : std::false_type {};
template <class F>
struct HasAltMul<F, std::void_t<decltype(F::kAltMul)>> : std::bool_constant<F::kAltMul> {};

// BLS12-381 scalar field Fr.  2-adicity 32; 7 generates the multiplicative group.
struct Bls12_381Fr {
  static constexpr uint32_t P[kLimbs] = {0x00000001u, 0xffffffffu, 0xfffe5bfeu, 0x53bda402u,
                                         0x09a1d805u, 0x3339d808u, 0x299d7d48u, 0x73eda753u};
  static constexpr uint32_t INV = 0xffffffffu;  // -p^{-1} mod 2^32
  static constexpr int TWO_ADICITY = 32;
  static constexpr uint32_t GENERATOR = 7;
  static constexpr int ID = 1;
};

// BN254 scalar field Fr.  2-adicity 28; 5 generates the multiplicative group.
struct Bn254Fr {
  static constexpr uint32_t P[kLimbs] = {0xf0000001u, 0x43e1f593u, 0x79b97091u, 0x2833e848u,
                                         0x8181585du, 0xb85045b6u, 0xe131a029u, 0x30644e72u};
  static constexpr uint32_t INV = 0xefffffffu;
  static constexpr int TWO_ADICITY = 28;
  static constexpr uint32_t GENERATOR = 5;
  static constexpr int ID = 2;
};

// BLS12-377 scalar field (the curve of the paper's other workloads); like
// BLS12-381 Fr its lowest limb is 1, so INV = -1 mod 2^32.
struct Bls12_377Fr {
  static constexpr uint32_t P[kLimbs] = {0x00000001u, 0x0a118000u, 0xd0000001u, 0x59aa76feu,
                                         0x5c37b001u, 0x60b44d1eu, 0x9a2ca556u, 0x12ab655eu};
  static constexpr uint32_t INV = 0xffffffffu;
  static constexpr int TWO_ADICITY = 47;
  static constexpr uint32_t GENERATOR = 22;
  static constexpr int ID = 3;
};

struct __align__(16) Fe {
  uint32_t v[kLimbs];
};

__host__ __device__ __forceinline__ Fe fe_zero() {
  Fe r;
#pragma unroll
  for (int j = 0; j < kLimbs; ++j) r.v[j] = 0;
  return r;
}

// ---------------------------------------------------------------------------
// FF_add / FF_sub (branchless)

// a + b mod p, inputs canonical.  a + b < 2p < 2^256 for both fields, so the
// sum fits in eight limbs; subtract p and keep the difference unless it
// borrowed.  The limb chains use the add/sub-with-carry builtins, which lower
// to v_add_co_u32 / v_addc_co_u32 (v_sub_co / v_subb_co) chains on gfx950.
template <class F>
__host__ __device__ __forceinline__ Fe add(const Fe& a, const Fe& b) {
  Fe s, d;
  unsigned int c = 0, br = 0;
#pragma unroll
  for (int j = 0; j < kLimbs; ++j) s.v[j] = __builtin_addc(a.v[j], b.v[j], c, &c);
#pragma unroll
  for (int j = 0; j < kLimbs; ++j) d.v[j] = __builtin_subc(s.v[j], F::P[j], br, &br);
#pragma unroll
  for (int j = 0; j < kLimbs; ++j) d.v[j] = br ? s.v[j] : d.v[j];
  return d;
}

// a - b mod p, inputs canonical: subtract, then add p back under the borrow
// mask.
template <class F>
__host__ __device__ __forceinline__ Fe sub(const Fe& a, const Fe& b) {
  Fe d;
  unsigned int br = 0, c = 0;
#pragma unroll
  for (int j = 0; j < kLimbs; ++j) d.v[j] = __builtin_subc(a.v[j], b.v[j], br, &br);
  const uint32_t mask = 0u - br;
#pragma unroll
  for (int j = 0; j < kLimbs; ++j) d.v[j] = __builtin_addc(d.v[j], F::P[j] & mask, c, &c);
  return d;
}

// 2p as eight limbs (p < 2^255 for all three fields).
template <class F>
struct TwoP {
  static constexpr uint32_t limb(int j) { return (F::P[j] << 1) | (j ? F::P[j - 1] >> 31 : 0u); }
  static constexpr uint32_t V[kLimbs] = {limb(0), limb(1), limb(2), limb(3), limb(4), limb(5), limb(6), limb(7)};
};

// Lazy FF_add / FF_sub on [0, 2p): a, b < 2p in, result < 2p out.  The sum
// a + b < 4p can exceed 2^256 (BLS12-381 Fr has p > 2^254), so its carry-out
// takes part in the choice: subtract 2p when the sum carried out or the
// subtraction did not borrow.
template <class F>
__host__ __device__ __forceinline__ Fe add_lazy(const Fe& a, const Fe& b) {
  Fe s, d;
  unsigned int c = 0, br = 0;
#pragma unroll
  for (int j = 0; j < kLimbs; ++j) s.v[j] = __builtin_addc(a.v[j], b.v[j], c, &c);
#pragma unroll
  for (int j = 0; j < kLimbs; ++j) d.v[j] = __builtin_subc(s.v[j], TwoP<F>::V[j], br, &br);
  const bool keep = br & (c ^ 1u);
#pragma unroll
  for (int j = 0; j < kLimbs; ++j) d.v[j] = keep ? s.v[j] : d.v[j];
  return d;
}

// a - b, plus 2p when it borrowed: a - b lies in (-2p, 2p).
template <class F>
__host__ __device__ __forceinline__ Fe sub_lazy(const Fe& a, const Fe& b) {
  Fe d;
  unsigned int br = 0, c = 0;
#pragma unroll
  for (int j = 0; j < kLimbs; ++j) d.v[j] = __builtin_subc(a.v[j], b.v[j], br, &br);
  const uint32_t mask = 0u - br;
#pragma unroll
  for (int j = 0; j < kLimbs; ++j) d.v[j] = __builtin_addc(d.v[j], TwoP<F>::V[j] & mask, c, &c);
  return d;
}

// t < 2p in eight limbs -> t mod p.
template <class F>
__host__ __device__ __forceinline__ Fe reduce_once(const uint32_t t[kLimbs]) {
  Fe r, d;
  unsigned int br = 0;
#pragma unroll
  for (int j = 0; j < kLimbs; ++j) d.v[j] = __builtin_subc(t[j], F::P[j], br, &br);
#pragma unroll
  for (int j = 0; j < kLimbs; ++j) r.v[j] = br ? t[j] : d.v[j];
  return r;
}

// x < 2p -> x mod p.
template <class F>
__host__ __device__ __forceinline__ Fe canon(const Fe& x) {
  return reduce_once<F>(x.v);
}

// ---------------------------------------------------------------------------
// FF_mul, portable CIOS (host; also valid on the device)

// Montgomery product a b 2^-256 mod p in CIOS order with the multiplication
// and reduction loops fused.  Both moduli have a top limb below 2^31 - 1, so
// the running value never needs a ninth limb.
template <class F>
__host__ __device__ __forceinline__ Fe mul_portable(const Fe& a, const Fe& b) {
  uint32_t t[kLimbs];
#pragma unroll
  for (int j = 0; j < kLimbs; ++j) t[j] = 0;
#pragma unroll
  for (int i = 0; i < kLimbs; ++i) {
    const uint32_t bi = b.v[i];
    uint64_t x = (uint64_t)a.v[0] * bi + t[0];
    uint32_t A = (uint32_t)(x >> 32);
    const uint32_t t0 = (uint32_t)x;
    const uint32_t m = t0 * F::INV;
    uint64_t y = (uint64_t)m * F::P[0] + t0;
    uint32_t C = (uint32_t)(y >> 32);
#pragma unroll
    for (int j = 1; j < kLimbs; ++j) {
      x = (uint64_t)a.v[j] * bi + t[j] + A;
      A = (uint32_t)(x >> 32);
      y = (uint64_t)m * F::P[j] + (uint32_t)x + C;
      C = (uint32_t)(y >> 32);
      t[j - 1] = (uint32_t)y;
    }
    t[kLimbs - 1] = C + A;
  }
  return reduce_once<F>(t);
}

// ---------------------------------------------------------------------------
// FF_mul, device FIPS

#if defined(__HIP_DEVICE_COMPILE__)
// 64-bit acc + a * b with the carry-out of the 64-bit addition returned as a
// lane mask.  Register-only arithmetic; no memory operand.
__device__ __forceinline__ uint64_t mad_co_vv(uint32_t a, uint32_t b, uint64_t c, uint64_t& co) {
  uint64_t r;
  asm("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(r), "=s"(co) : "v"(a), "v"(b), "v"(c));
  return r;
}
// Same, with b wave-uniform (an SGPR operand, e.g. a modulus limb).
__device__ __forceinline__ uint64_t mad_co_vs(uint32_t a, uint32_t b, uint64_t c, uint64_t& co) {
  uint64_t r;
  asm("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(r), "=s"(co) : "v"(a), "s"(b), "v"(c));
  return r;
}
// Ordered (volatile) forms for mul_k: the compiler keeps volatile asm in
// source order, which is how the K chains stay interleaved.  Each chain keeps
// one SGPR pair for its carry mask for the whole product ("+s": the multiply-
// add writes it, the carry add reads it and writes its own, unused, carry-out
// back into it), so consecutive instructions of different chains never write
// the same SGPRs: two VALU writes of one SGPR pair back to back need a wait
// state on gfx950, which the compiler otherwise pays with an s_nop before
// almost every instruction of the product.
__device__ __forceinline__ uint64_t mad_co_vv_ord(uint32_t a, uint32_t b, uint64_t c, uint64_t& co) {
  uint64_t r;
  asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(r), "+s"(co) : "v"(a), "v"(b), "v"(c));
  return r;
}
__device__ __forceinline__ uint64_t mad_co_vs_ord(uint32_t a, uint32_t b, uint64_t c, uint64_t& co) {
  uint64_t r;
  asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(r), "+s"(co) : "v"(a), "s"(b), "v"(c));
  return r;
}
__device__ __forceinline__ uint32_t add_carry_ord(uint32_t x, uint64_t& co) {
  uint32_t r;
  asm volatile("v_addc_co_u32_e64 %0, %1, %2, 0, %1" : "=v"(r), "+s"(co) : "v"(x));
  return r;
}
// 0 - x with the borrow (x != 0) left in co, ordered like the forms above.
__device__ __forceinline__ uint32_t neg_borrow_ord(uint32_t x, uint64_t& co) {
  uint32_t r;
  asm volatile("v_sub_co_u32_e64 %0, %1, 0, %2" : "=v"(r), "+s"(co) : "v"(x));
  return r;
}
// x + (carry bit of this lane)
__device__ __forceinline__ uint32_t add_carry(uint32_t x, uint64_t ci) {
  uint32_t r;
  uint64_t unused;
  asm("v_addc_co_u32_e64 %0, %1, %2, 0, %3" : "=v"(r), "=s"(unused) : "v"(x), "s"(ci));
  return r;
}

template <class F, bool CANON = true>
__device__ __forceinline__ Fe mul(const Fe& a, const Fe& b) {
  if constexpr (HasAltMul<F>::value) return F::mul(a, b);
  uint32_t m[kLimbs], r[kLimbs];
  uint64_t acc = 0;  // current column, low 64 bits
  uint32_t hi = 0;   // overflow count of the current column
#define ZK_TERM(x, y)                 \
  {                                   \
    uint64_t co;                      \
    acc = mad_co_vv(x, y, acc, co);   \
    hi = add_carry(hi, co);           \
  }
#define ZK_TERM_P(x, y)               \
  {                                   \
    uint64_t co;                      \
    acc = mad_co_vs(x, y, acc, co);   \
    hi = add_carry(hi, co);           \
  }
  // Columns 0..7: the reduction digit m_i is chosen so that column i becomes
  // 0 mod 2^32 and is shifted out.
#pragma unroll
  for (int i = 0; i < kLimbs; ++i) {
#pragma unroll
    for (int j = 0; j < i; ++j) {
      ZK_TERM(a.v[j], b.v[i - j]);
      ZK_TERM_P(m[j], F::P[i - j]);
    }
    ZK_TERM(a.v[i], b.v[0]);
    if constexpr (F::P[0] == 1u) {
      // see mul_k: the digit's product is a borrow
      uint64_t co;
      uint32_t lo;
      asm("v_sub_co_u32_e64 %0, %1, 0, %2" : "=v"(m[i]), "=s"(co) : "v"((uint32_t)acc));
      asm("v_addc_co_u32_e64 %0, %1, %2, 0, %3" : "=v"(lo), "=s"(co) : "v"((uint32_t)(acc >> 32)), "s"(co));
      hi = add_carry(hi, co);
      acc = ((uint64_t)hi << 32) | lo;
    } else {
      m[i] = (uint32_t)acc * F::INV;
      ZK_TERM_P(m[i], F::P[0]);
      acc = (acc >> 32) | ((uint64_t)hi << 32);
    }
    hi = 0;
  }
  // Columns 8..15 hold the result.
#pragma unroll
  for (int i = kLimbs; i < 2 * kLimbs; ++i) {
#pragma unroll
    for (int j = i - (kLimbs - 1); j < kLimbs; ++j) {
      ZK_TERM(a.v[j], b.v[i - j]);
      ZK_TERM_P(m[j], F::P[i - j]);
    }
    r[i - kLimbs] = (uint32_t)acc;
    acc = (acc >> 32) | ((uint64_t)hi << 32);
    hi = 0;
  }
#undef ZK_TERM
#undef ZK_TERM_P
  // the result is below 2p; CANON = false leaves it there (see mul_k)
  if constexpr (CANON) return reduce_once<F>(r);
  Fe o;
#pragma unroll
  for (int j = 0; j < kLimbs; ++j) o.v[j] = r[j];
  return o;
}
// K independent Montgomery products r[k] = a[k] b[k], computed column by
// column in lock step.  Each column of one product is a serial chain
// (v_mad_u64_u32 -> v_mad_u64_u32 through the accumulator, v_addc through
// the counter); emitting the K chains' instructions alternately gives every
// instruction K-1 independent instructions of distance from the one it
// waits for, which hides the issue latency the single chain exposes and
// removes the carry-hazard wait states.  The result of each product is
// identical to mul().
//
// Moduli with p = 1 mod 2^32 (BLS12-381 Fr, BLS12-377 Fr: -p^-1 = -1 mod
// 2^32) make the reduction digit m_i = -c mod 2^32 for a column c, and
// c + m_i p_0 = c + m_i has a zero low word with a carry into bit 32 exactly
// when c mod 2^32 != 0.  The digit's multiply-add and carry count then become
// one subtraction whose borrow is that carry, added to the column's high word
// as it becomes the next column's low word, which also saves the register
// move of the shift.
//
// Lazy reduction (CANON = false): before its final subtraction the
// Montgomery product is (a b + m p) / 2^256 < a b / 2^256 + p < b + p, so for
// any eight-limb a and a canonical b (b < p: every table entry and constant)
// it is below 2p, and the subtraction can be left out.  Data in the NTT
// passes stays in [0, 2p) this way (add_lazy / sub_lazy below keep that
// range) and is made canonical once, where it leaves the computation.
template <class F, int K, bool CANON = true>
__device__ __forceinline__ void mul_k(Fe* r, const Fe* a, const Fe* b) {
  if constexpr (HasAltMul<F>::value) {
#pragma unroll
    for (int k = 0; k < K; ++k) r[k] = F::mul(a[k], b[k]);
    return;
  }
  uint32_t m[K][kLimbs], t[K][kLimbs];
  uint64_t acc[K], co[K];
  uint32_t hi[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    acc[k] = 0;
    hi[k] = 0;
    co[k] = 0;
  }
#define ZK_TERMS(X, Y, MADFN)                                        \
  {                                                                  \
    _Pragma("unroll") for (int k = 0; k < K; ++k) acc[k] = MADFN(X, Y, acc[k], co[k]); \
    _Pragma("unroll") for (int k = 0; k < K; ++k) hi[k] = add_carry_ord(hi[k], co[k]);  \
  }
#pragma unroll
  for (int i = 0; i < kLimbs; ++i) {
#pragma unroll
    for (int j = 0; j < i; ++j) {
      ZK_TERMS(a[k].v[j], b[k].v[i - j], mad_co_vv_ord);
      ZK_TERMS(m[k][j], F::P[i - j], mad_co_vs_ord);
    }
    ZK_TERMS(a[k].v[i], b[k].v[0], mad_co_vv_ord);
    if constexpr (F::P[0] == 1u) {
      uint32_t lo[K];
#pragma unroll
      for (int k = 0; k < K; ++k) m[k][i] = neg_borrow_ord((uint32_t)acc[k], co[k]);
#pragma unroll
      for (int k = 0; k < K; ++k) lo[k] = add_carry_ord((uint32_t)(acc[k] >> 32), co[k]);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        hi[k] = add_carry_ord(hi[k], co[k]);
        acc[k] = ((uint64_t)hi[k] << 32) | lo[k];
        hi[k] = 0;
      }
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) m[k][i] = (uint32_t)acc[k] * F::INV;
      ZK_TERMS(m[k][i], F::P[0], mad_co_vs_ord);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        acc[k] = (acc[k] >> 32) | ((uint64_t)hi[k] << 32);
        hi[k] = 0;
      }
    }
  }
#pragma unroll
  for (int i = kLimbs; i < 2 * kLimbs; ++i) {
#pragma unroll
    for (int j = i - (kLimbs - 1); j < kLimbs; ++j) {
      ZK_TERMS(a[k].v[j], b[k].v[i - j], mad_co_vv_ord);
      ZK_TERMS(m[k][j], F::P[i - j], mad_co_vs_ord);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      t[k][i - kLimbs] = (uint32_t)acc[k];
      acc[k] = (acc[k] >> 32) | ((uint64_t)hi[k] << 32);
      hi[k] = 0;
    }
  }
#undef ZK_TERMS
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if constexpr (CANON) {
      r[k] = reduce_once<F>(t[k]);
    } else {
#pragma unroll
      for (int j = 0; j < kLimbs; ++j) r[k].v[j] = t[k][j];
    }
  }
}
#else
// Host compilation pass: device code is parsed but never emitted here.
template <class F, bool CANON = true>
__host__ __device__ inline Fe mul(const Fe& a, const Fe& b) {
  return mul_portable<F>(a, b);
}
template <class F, int K, bool CANON = true>
__host__ __device__ inline void mul_k(Fe* r, const Fe* a, const Fe* b) {
  for (int k = 0; k < K; ++k) r[k] = mul_portable<F>(a[k], b[k]);
}
#endif

// ---------------------------------------------------------------------------
// Host-side helpers for plan-time constants (plain integers <-> Montgomery).

template <class F>
inline Fe fe_from_u32(uint32_t x) {
  Fe r = fe_zero();
  r.v[0] = x;
  return r;
}

// 2^256 mod p, i.e. the Montgomery form of 1, by 256 modular doublings of 1.
template <class F>
inline Fe mont_one() {
  Fe x = fe_from_u32<F>(1);
  for (int i = 0; i < 256; ++i) x = add<F>(x, x);
  return x;
}

// 2^512 mod p: 256 more doublings.
template <class F>
inline Fe mont_r2() {
  Fe x = mont_one<F>();
  for (int i = 0; i < 256; ++i) x = add<F>(x, x);
  return x;
}

template <class F>
inline Fe to_mont(const Fe& plain) {
  return mul_portable<F>(plain, mont_r2<F>());
}

template <class F>
inline Fe from_mont(const Fe& m) {
  return mul_portable<F>(m, fe_from_u32<F>(1));
}

// base^e (Montgomery in and out); e given as eight 32-bit limbs.
template <class F>
inline Fe pow_mont(const Fe& base, const uint32_t e[kLimbs]) {
  Fe r = mont_one<F>();
  for (int i = 255; i >= 0; --i) {
    r = mul_portable<F>(r, r);
    if ((e[i / 32] >> (i % 32)) & 1u) r = mul_portable<F>(r, base);
  }
  return r;
}

template <class F>
inline Fe pow_mont_u64(const Fe& base, uint64_t e) {
  uint32_t ew[kLimbs] = {(uint32_t)e, (uint32_t)(e >> 32), 0, 0, 0, 0, 0, 0};
  return pow_mont<F>(base, ew);
}

// a^(p-2) = a^-1 (Fermat), Montgomery in and out.
template <class F>
inline Fe inv_mont(const Fe& a) {
  uint32_t e[kLimbs];
  uint32_t br = 2;
  for (int j = 0; j < kLimbs; ++j) {
    uint64_t t = (uint64_t)F::P[j] - br;
    e[j] = (uint32_t)t;
    br = (uint32_t)(t >> 32) & 1u;
  }
  return pow_mont<F>(a, e);
}

// Primitive 2^log2n-th root of unity g^((p-1)/2^log2n) in Montgomery form.
template <class F>
inline Fe root_of_unity(int log2n) {
  uint32_t e[kLimbs];
  for (int j = 0; j < kLimbs; ++j) e[j] = F::P[j];
  e[0] -= 1;
  for (int s = 0; s < log2n; ++s)
    for (int j = 0; j < kLimbs; ++j) e[j] = (e[j] >> 1) | (j + 1 < kLimbs ? e[j + 1] << 31 : 0u);
  return pow_mont<F>(to_mont<F>(fe_from_u32<F>(F::GENERATOR)), e);
}

}  // namespace zk
