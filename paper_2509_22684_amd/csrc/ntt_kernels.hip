// Auxiliary kernels (table generation, pointwise quotient, validation) and
// the pass dispatcher.  The pass kernels themselves are instantiated per
// field and in-register radix in ntt_pass_<field>_e<k>.hip so they compile in
// parallel.
#include <algorithm>

#include "field_f64.hpp"
#include "ntt_kernels.hpp"
#include "ntt_pass_impl.hpp"

namespace zk {

hipError_t launch_pass_bls_e3(int log_r, int log_tile, const PassArgs& a, hipStream_t s);
hipError_t launch_pass_bls_e2(int log_r, int log_tile, const PassArgs& a, hipStream_t s);
hipError_t launch_pass_bls_e1(int log_r, int log_tile, const PassArgs& a, hipStream_t s);
hipError_t launch_pass_bn_e3(int log_r, int log_tile, const PassArgs& a, hipStream_t s);
hipError_t launch_pass_bn_e2(int log_r, int log_tile, const PassArgs& a, hipStream_t s);
hipError_t launch_pass_bn_e1(int log_r, int log_tile, const PassArgs& a, hipStream_t s);
hipError_t launch_pass_b377_e3(int log_r, int log_tile, const PassArgs& a, hipStream_t s);
hipError_t launch_pass_b377_e2(int log_r, int log_tile, const PassArgs& a, hipStream_t s);
hipError_t launch_pass_b377_e1(int log_r, int log_tile, const PassArgs& a, hipStream_t s);
hipError_t launch_pass_bls_f64_e2(int log_r, int log_tile, const PassArgs& a, hipStream_t s);

namespace {
using detail::load_fe;
using detail::store_fe;

// ---------------------------------------------------------------------------
// Table generation, pointwise quotient, validation

template <class F>
__global__ void __launch_bounds__(256) gen_kernel(GenArgs g) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.count) return;
  uint64_t e = t;
  if (g.mode == kGenPassTwiddle) e = g.mult * (t / g.ns) * (t % g.ns);
  Fe x = g.scale;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t d = (uint32_t)(e >> (8 * k)) & 255u;
    if (d) x = mul<F>(x, g.levels[256 * k + d]);
  }
  store_fe(g.out, t, x);
}

template <class F>
__global__ void __launch_bounds__(256) quotient_pointwise_kernel(const Fe* __restrict__ a, const Fe* __restrict__ b,
                                                                  const Fe* c, Fe* out, Fe zinv, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Fe ab = mul<F>(load_fe(a, i), load_fe(b, i));
  store_fe(out, i, mul<F>(sub<F>(ab, load_fe(c, i)), zinv));
}

template <class F>
__global__ void __launch_bounds__(256) validate_kernel(const Fe* __restrict__ x, uint64_t n, uint32_t* count) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Fe v = load_fe(x, i);
  uint32_t br = 0;
#pragma unroll
  for (int j = 0; j < kLimbs; ++j) {
    uint64_t s = (uint64_t)v.v[j] - F::P[j] - br;
    br = (uint32_t)(s >> 32) & 1u;
  }
  if (!br) atomicAdd(count, 1u);  // v >= p
}

template <class F, int VARIANT>
__global__ void __launch_bounds__(256) field_mul_kernel(const Fe* __restrict__ a, const Fe* __restrict__ b,
                                                         Fe* __restrict__ out, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Fe x = load_fe(a, i), y = load_fe(b, i);
  if constexpr (VARIANT == 2) {  // the pass kernels' lazy, ordered product
    Fe r;
    mul_k<F, 1, false>(&r, &x, &y);
    store_fe(out, i, r);
  } else {
    store_fe(out, i, VARIANT == 1 ? mul_f64<F>(x, y) : mul<F>(x, y));
  }
}

inline uint32_t blocks_for(uint64_t n, uint32_t per) { return (uint32_t)((n + per - 1) / per); }

}  // namespace

hipError_t launch_pass(int field, int log_r, int log_tile, int log_e, const PassArgs& a, hipStream_t s) {
  if (field == Bls12_381Fr::ID) {
    if (log_e == 3) return launch_pass_bls_e3(log_r, log_tile, a, s);
    if (log_e == 2) return launch_pass_bls_e2(log_r, log_tile, a, s);
    if (log_e == 1) return launch_pass_bls_e1(log_r, log_tile, a, s);
  } else if (field == Bn254Fr::ID) {
    if (log_e == 3) return launch_pass_bn_e3(log_r, log_tile, a, s);
    if (log_e == 2) return launch_pass_bn_e2(log_r, log_tile, a, s);
    if (log_e == 1) return launch_pass_bn_e1(log_r, log_tile, a, s);
  } else if (field == Bls12_377Fr::ID) {
    if (log_e == 3) return launch_pass_b377_e3(log_r, log_tile, a, s);
    if (log_e == 2) return launch_pass_b377_e2(log_r, log_tile, a, s);
    if (log_e == 1) return launch_pass_b377_e1(log_r, log_tile, a, s);
  } else if (field == kFieldBls12_381Fp64) {
    if (log_e == 2) return launch_pass_bls_f64_e2(log_r, log_tile, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_field_mul(int field, int variant, const Fe* a, const Fe* b, Fe* out, uint64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (variant < 0 || variant > 2) return hipErrorInvalidValue;
  const dim3 grid(blocks_for(n, 256)), block(256);
#define ZK_FIELD_MUL(FT)                                                                          \
  if (variant == 0) hipLaunchKernelGGL((field_mul_kernel<FT, 0>), grid, block, 0, s, a, b, out, n); \
  else if (variant == 1) hipLaunchKernelGGL((field_mul_kernel<FT, 1>), grid, block, 0, s, a, b, out, n); \
  else hipLaunchKernelGGL((field_mul_kernel<FT, 2>), grid, block, 0, s, a, b, out, n);
  if (field == Bls12_381Fr::ID) {
    ZK_FIELD_MUL(Bls12_381Fr)
  } else if (field == Bn254Fr::ID) {
    ZK_FIELD_MUL(Bn254Fr)
  } else if (field == Bls12_377Fr::ID) {
    ZK_FIELD_MUL(Bls12_377Fr)
  } else {
    return hipErrorInvalidValue;
  }
#undef ZK_FIELD_MUL
  return hipGetLastError();
}

hipError_t launch_gen(int field, const GenArgs& g, hipStream_t s) {
  if (g.count == 0) return hipSuccess;
  const dim3 grid(blocks_for(g.count, 256)), block(256);
  if (field == Bls12_381Fr::ID) hipLaunchKernelGGL(gen_kernel<Bls12_381Fr>, grid, block, 0, s, g);
  else if (field == Bn254Fr::ID) hipLaunchKernelGGL(gen_kernel<Bn254Fr>, grid, block, 0, s, g);
  else if (field == Bls12_377Fr::ID) hipLaunchKernelGGL(gen_kernel<Bls12_377Fr>, grid, block, 0, s, g);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_quotient_pointwise(int field, const Fe* a, const Fe* b, const Fe* c, Fe* out, Fe zinv, uint64_t n,
                                     hipStream_t s) {
  if (n == 0) return hipSuccess;
  const dim3 grid(blocks_for(n, 256)), block(256);
  if (field == Bls12_381Fr::ID)
    hipLaunchKernelGGL(quotient_pointwise_kernel<Bls12_381Fr>, grid, block, 0, s, a, b, c, out, zinv, n);
  else if (field == Bn254Fr::ID)
    hipLaunchKernelGGL(quotient_pointwise_kernel<Bn254Fr>, grid, block, 0, s, a, b, c, out, zinv, n);
  else if (field == Bls12_377Fr::ID)
    hipLaunchKernelGGL(quotient_pointwise_kernel<Bls12_377Fr>, grid, block, 0, s, a, b, c, out, zinv, n);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// Device-to-host copy on the compute units: pinned host memory is mapped into
// the device's address space, so workgroups can store to it directly.  A DMA
// copy in the other direction then runs at the same time (both directions of
// the link busy at once), which two DMA copies on separate streams did not.
__global__ void __launch_bounds__(256) copy_out_kernel(uint4* __restrict__ dst, const uint4* __restrict__ src,
                                                       uint64_t nvec) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvec; i += stride) dst[i] = src[i];
}

hipError_t launch_copy_out(void* host_dst, const void* dev_src, uint64_t bytes, hipStream_t s) {
  const uint64_t nvec = bytes / 16;
  if (nvec == 0) return hipSuccess;
  const uint32_t blocks = (uint32_t)std::min<uint64_t>(256, (nvec + 255) / 256);
  hipLaunchKernelGGL(copy_out_kernel, dim3(blocks), dim3(256), 0, s, static_cast<uint4*>(host_dst),
                     static_cast<const uint4*>(dev_src), nvec);
  return hipGetLastError();
}

hipError_t launch_validate(int field, const Fe* x, uint64_t n, uint32_t* d_count, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const dim3 grid(blocks_for(n, 256)), block(256);
  if (field == Bls12_381Fr::ID) hipLaunchKernelGGL(validate_kernel<Bls12_381Fr>, grid, block, 0, s, x, n, d_count);
  else if (field == Bn254Fr::ID) hipLaunchKernelGGL(validate_kernel<Bn254Fr>, grid, block, 0, s, x, n, d_count);
  else if (field == Bls12_377Fr::ID)
    hipLaunchKernelGGL(validate_kernel<Bls12_377Fr>, grid, block, 0, s, x, n, d_count);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace zk
