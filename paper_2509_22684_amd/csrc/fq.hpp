// The base field of BLS12-381 G1, F_q (381-bit q), for the MSM kernels.
//
// An element is twelve 32-bit limbs, little-endian, in Montgomery form with
// R = 2^384.  Inside the kernels elements are kept in [0, 2q) (lazy
// reduction: 4q < 2^384, so a Montgomery product of two such elements is
// below 2q without a final subtraction, and sums and differences reduce
// modulo 2q); canon() brings one to [0, q) where it leaves the device.
// FF_mul is the same finely integrated product scanning as the scalar
// fields' (field.hpp): each 32x32-bit partial product is one v_mad_u64_u32
// into a 64-bit column accumulator whose carry-out feeds a v_addc_co_u32
// column counter, 2 N^2 = 288 of each per product; K independent products
// (mul2, mul3, mul4) interleave column by column, each chain keeping its own
// carry SGPR pair.  FF_add / FF_sub are branchless carry chains with a
// borrow-select.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace zk {
namespace fq {

constexpr int kN = 12;

// q = (x0 - 1)^2 (x0^4 - x0^2 + 1) / 3 + x0, x0 = -0xd201000000010000.
constexpr uint32_t kQ[kN] = {0xffffaaabu, 0xb9feffffu, 0xb153ffffu, 0x1eabfffeu, 0xf6b0f624u, 0x6730d2a0u,
                             0xf38512bfu, 0x64774b84u, 0x434bacd7u, 0x4b1ba7b6u, 0x397fe69au, 0x1a0111eau};
constexpr uint32_t k2Q[kN] = {0xffff5556u, 0x73fdffffu, 0x62a7ffffu, 0x3d57fffdu, 0xed61ec48u, 0xce61a541u,
                              0xe70a257eu, 0xc8ee9709u, 0x869759aeu, 0x96374f6cu, 0x72ffcd34u, 0x340223d4u};
constexpr uint32_t kInv = 0xfffcfffdu;  // -q^-1 mod 2^32
// 2^384 mod q: the Montgomery form of 1.
constexpr uint32_t kOne[kN] = {0x0002fffdu, 0x76090000u, 0xc40c0002u, 0xebf4000bu, 0x53c758bau, 0x5f489857u,
                               0x70525745u, 0x77ce5853u, 0xa256ec6du, 0x5c071a97u, 0xfa80e493u, 0x15f65ec3u};

struct __align__(16) Fq {
  uint32_t v[kN];
};

__device__ __forceinline__ Fq zero() {
  Fq r;
#pragma unroll
  for (int j = 0; j < kN; ++j) r.v[j] = 0;
  return r;
}

__device__ __forceinline__ Fq one() {
  Fq r;
#pragma unroll
  for (int j = 0; j < kN; ++j) r.v[j] = kOne[j];
  return r;
}

// a = 0 mod q, for a in [0, 2q): a is 0 or q.
__device__ __forceinline__ bool is_zero(const Fq& a) {
  uint32_t o = 0, oq = 0;
#pragma unroll
  for (int j = 0; j < kN; ++j) {
    o |= a.v[j];
    oq |= a.v[j] ^ kQ[j];
  }
  return o == 0 || oq == 0;
}

// a in [0, 2q) to [0, q).
__device__ __forceinline__ Fq canon(const Fq& a) {
  Fq d;
  unsigned int br = 0;
#pragma unroll
  for (int j = 0; j < kN; ++j) d.v[j] = __builtin_subc(a.v[j], kQ[j], br, &br);
#pragma unroll
  for (int j = 0; j < kN; ++j) d.v[j] = br ? a.v[j] : d.v[j];
  return d;
}

// a + b mod 2q (a, b in [0, 2q); a + b < 4q < 2^384).
__device__ __forceinline__ Fq add(const Fq& a, const Fq& b) {
  Fq s, d;
  unsigned int c = 0, br = 0;
#pragma unroll
  for (int j = 0; j < kN; ++j) s.v[j] = __builtin_addc(a.v[j], b.v[j], c, &c);
#pragma unroll
  for (int j = 0; j < kN; ++j) d.v[j] = __builtin_subc(s.v[j], k2Q[j], br, &br);
#pragma unroll
  for (int j = 0; j < kN; ++j) d.v[j] = br ? s.v[j] : d.v[j];
  return d;
}

// a - b mod 2q (a, b in [0, 2q)).
__device__ __forceinline__ Fq sub(const Fq& a, const Fq& b) {
  Fq d;
  unsigned int br = 0, c = 0;
#pragma unroll
  for (int j = 0; j < kN; ++j) d.v[j] = __builtin_subc(a.v[j], b.v[j], br, &br);
  const uint32_t mask = 0u - br;
#pragma unroll
  for (int j = 0; j < kN; ++j) d.v[j] = __builtin_addc(d.v[j], k2Q[j] & mask, c, &c);
  return d;
}

__device__ __forceinline__ Fq dbl(const Fq& a) { return add(a, a); }

#if defined(__HIP_DEVICE_COMPILE__)
__device__ __forceinline__ uint64_t mad_vv(uint32_t a, uint32_t b, uint64_t c, uint64_t& co) {
  uint64_t r;
  asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(r), "+s"(co) : "v"(a), "v"(b), "v"(c));
  return r;
}
__device__ __forceinline__ uint64_t mad_vs(uint32_t a, uint32_t b, uint64_t c, uint64_t& co) {
  uint64_t r;
  asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(r), "+s"(co) : "v"(a), "s"(b), "v"(c));
  return r;
}
__device__ __forceinline__ uint32_t addc(uint32_t x, uint64_t& co) {
  uint32_t r;
  asm volatile("v_addc_co_u32_e64 %0, %1, %2, 0, %1" : "=v"(r), "+s"(co) : "v"(x));
  return r;
}

// K independent Montgomery products r[k] = a[k] b[k] 2^-384 mod q, column by
// column in lock step (see the file comment).
template <int K>
__device__ __forceinline__ void mul_k(Fq* r, const Fq* a, const Fq* b) {
  uint32_t m[K][kN], t[K][kN];
  uint64_t acc[K], co[K];
  uint32_t hi[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    acc[k] = 0;
    hi[k] = 0;
    co[k] = 0;
  }
#define ZK_FQ_TERMS(X, Y, MADFN)                                                  \
  {                                                                               \
    _Pragma("unroll") for (int k = 0; k < K; ++k) acc[k] = MADFN(X, Y, acc[k], co[k]); \
    _Pragma("unroll") for (int k = 0; k < K; ++k) hi[k] = addc(hi[k], co[k]);     \
  }
#pragma unroll
  for (int i = 0; i < kN; ++i) {
#pragma unroll
    for (int j = 0; j < i; ++j) {
      ZK_FQ_TERMS(a[k].v[j], b[k].v[i - j], mad_vv);
      ZK_FQ_TERMS(m[k][j], kQ[i - j], mad_vs);
    }
    ZK_FQ_TERMS(a[k].v[i], b[k].v[0], mad_vv);
#pragma unroll
    for (int k = 0; k < K; ++k) m[k][i] = (uint32_t)acc[k] * kInv;
    ZK_FQ_TERMS(m[k][i], kQ[0], mad_vs);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      acc[k] = (acc[k] >> 32) | ((uint64_t)hi[k] << 32);
      hi[k] = 0;
    }
  }
#pragma unroll
  for (int i = kN; i < 2 * kN; ++i) {
#pragma unroll
    for (int j = i - (kN - 1); j < kN; ++j) {
      ZK_FQ_TERMS(a[k].v[j], b[k].v[i - j], mad_vv);
      ZK_FQ_TERMS(m[k][j], kQ[i - j], mad_vs);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      t[k][i - kN] = (uint32_t)acc[k];
      acc[k] = (acc[k] >> 32) | ((uint64_t)hi[k] << 32);
      hi[k] = 0;
    }
  }
#undef ZK_FQ_TERMS
  // t < 2q for a, b < 2q: left there (lazy reduction)
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int j = 0; j < kN; ++j) r[k].v[j] = t[k][j];
}
#else
// Host compilation pass: device code is parsed but never emitted here.
template <int K>
__device__ inline void mul_k(Fq* r, const Fq* a, const Fq* b) {
  for (int k = 0; k < K; ++k) r[k] = a[k];
  (void)b;
}
#endif

__device__ __forceinline__ Fq mul(const Fq& a, const Fq& b) {
  Fq r;
  mul_k<1>(&r, &a, &b);
  return r;
}
__device__ __forceinline__ void mul2(Fq& r0, const Fq& a0, const Fq& b0, Fq& r1, const Fq& a1, const Fq& b1) {
  Fq a[2] = {a0, a1}, b[2] = {b0, b1}, r[2];
  mul_k<2>(r, a, b);
  r0 = r[0];
  r1 = r[1];
}
// Three and four independent products, interleaved: more instructions in
// flight for the reduction's lone waves, where one product's chain of
// dependent multiply-adds would otherwise wait on its own latency.
__device__ __forceinline__ void mul3(Fq& r0, const Fq& a0, const Fq& b0, Fq& r1, const Fq& a1, const Fq& b1, Fq& r2,
                                     const Fq& a2, const Fq& b2) {
  Fq a[3] = {a0, a1, a2}, b[3] = {b0, b1, b2}, r[3];
  mul_k<3>(r, a, b);
  r0 = r[0];
  r1 = r[1];
  r2 = r[2];
}
__device__ __forceinline__ void mul4(Fq& r0, const Fq& a0, const Fq& b0, Fq& r1, const Fq& a1, const Fq& b1, Fq& r2,
                                     const Fq& a2, const Fq& b2, Fq& r3, const Fq& a3, const Fq& b3) {
  Fq a[4] = {a0, a1, a2, a3}, b[4] = {b0, b1, b2, b3}, r[4];
  mul_k<4>(r, a, b);
  r0 = r[0];
  r1 = r[1];
  r2 = r[2];
  r3 = r[3];
}
__device__ __forceinline__ Fq sqr(const Fq& a) { return mul(a, a); }

// a^-1 = a^(q-2) (Fermat), left-to-right square-and-multiply; a != 0.
__device__ __forceinline__ Fq inverse(const Fq& a) {
  // q - 2 differs from q only in the lowest limb (q mod 2^32 >= 2)
  Fq r = one();
#pragma unroll 1
  for (int i = 32 * kN - 1; i >= 0; --i) {
    r = sqr(r);
    const uint32_t e = (i < 32) ? kQ[0] - 2u : kQ[i / 32];
    if ((e >> (i % 32)) & 1u) r = mul(r, a);
  }
  return r;
}

}  // namespace fq
}  // namespace zk
