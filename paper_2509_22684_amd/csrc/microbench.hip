// Micro-benchmarks of the units the NTT's rooflines are drawn on: the
// all-CU issue rate of single VALU instruction kinds (the 32x32->64
// multiply-add v_mad_u64_u32 that FF_mul is built from, its carry add, a
// plain 32-bit add and the FP64 FMA), the rate of one FIPS column step (a
// multiply-add and the carry add it feeds), the rate of whole Montgomery
// products, and the HBM bandwidth of a streaming copy.  The paper's
// roofline analysis (Section IV-C) places its NTT kernels against the INT32
// throughput of the GPU; on gfx950 that denominator is measured here rather
// than taken from a data sheet.
//
// Every ALU kernel runs CHAINS independent dependency chains per lane so
// that the issue rate, not the latency of one chain, is measured, and folds
// the chains into one value per lane that it stores, so nothing is dead.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "../../include/zkntt.h"
#include "field.hpp"
#include "field_f64.hpp"

namespace zk {
namespace {

constexpr int kChains = 8;
constexpr int kUnroll = 8;  // chain steps per loop iteration
constexpr int kThreads = 256;

template <int KIND>
__global__ void __launch_bounds__(kThreads) rate_kernel(uint32_t iters, uint32_t seed, uint64_t* __restrict__ out) {
  const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t a = seed ^ (gid * 0x9e3779b9u), b = a * 0x85ebca6bu + 1u;
  uint64_t acc[kChains];
  uint32_t lo[kChains];
  double d[kChains];
  // Carry masks: one SGPR pair per chain, live to the end, so consecutive
  // instructions of different chains never write the same SGPRs (two VALU
  // writes of one SGPR pair back to back cost a wait state on gfx950).
  uint64_t co[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) {
    acc[k] = (uint64_t)(a + k) << 7;
    lo[k] = b + 3u * (uint32_t)k;
    d[k] = (double)(a & 0xffff) * 0.5 + k;
    co[k] = 0;
  }
  const double x = 1.0000001, y = 0.9999999;
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
      for (int k = 0; k < kChains; ++k) {
        if constexpr (KIND == ZK_MB_MAD_U64_U32) {
          asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(acc[k]), "+s"(co[k]) : "v"(a), "v"(b));
        } else if constexpr (KIND == ZK_MB_FMA_F64) {
          asm volatile("v_fma_f64 %0, %1, %2, %0" : "+v"(d[k]) : "v"(x), "v"(y));
        } else if constexpr (KIND == ZK_MB_ADD_U32) {
          asm volatile("v_add_u32 %0, %1, %0" : "+v"(lo[k]) : "v"(a));
        } else if constexpr (KIND == ZK_MB_ADDC_U32) {
          asm volatile("v_add_co_u32 %0, %1, %2, %0" : "+v"(lo[k]), "+s"(co[k]) : "v"(a));
          asm volatile("v_addc_co_u32_e64 %0, %1, %2, %0, %1" : "+v"(lo[k]), "+s"(co[k]) : "v"(b));
        } else if constexpr (KIND == ZK_MB_MAD_ADDC) {
          // one FIPS column step: acc += a b with its carry-out counted
          asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(acc[k]), "+s"(co[k]) : "v"(a), "v"(b));
          asm volatile("v_addc_co_u32_e64 %0, %1, %0, 0, %1" : "+v"(lo[k]), "+s"(co[k]));
        } else if constexpr (KIND == ZK_MB_MAD_FMA) {
          // an integer multiply-add and an independent FP64 FMA: whether the
          // two share one issue slot or can run side by side
          asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(acc[k]), "+s"(co[k]) : "v"(a), "v"(b));
          asm volatile("v_fma_f64 %0, %1, %2, %0" : "+v"(d[k]) : "v"(x), "v"(y));
        } else if constexpr (KIND == ZK_MB_MAD_ADD) {
          asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(acc[k]), "+s"(co[k]) : "v"(a), "v"(b));
          asm volatile("v_add_u32 %0, %1, %0" : "+v"(lo[k]) : "v"(a));
        }
      }
    }
  }
  uint64_t r = 0;
#pragma unroll
  for (int k = 0; k < kChains; ++k) {
    r ^= acc[k] + lo[k] + co[k];
    r ^= (uint64_t)__double_as_longlong(d[k]);
  }
  out[gid] = r;
}

// Montgomery products of the NTT's field, K interleaved per thread (the pass
// kernels interleave 2 to 4): x_k <- x_k y_k.
template <class F, int K, bool CANON = true>
__global__ void __launch_bounds__(kThreads) ffmul_kernel(uint32_t iters, uint32_t seed, uint64_t* __restrict__ out) {
  const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
  Fe x[K], y[K];
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int j = 0; j < kLimbs; ++j) {
      // below p: the top limb stays under every modulus' top limb
      x[k].v[j] = (j == kLimbs - 1) ? (seed + gid + (uint32_t)k) & 0x0fffffffu : seed * 2654435761u + gid * (j + 1);
      y[k].v[j] = (j == kLimbs - 1) ? (gid * 7u + (uint32_t)k) & 0x0fffffffu : gid * 40503u + (uint32_t)(j * k);
    }
  for (uint32_t it = 0; it < iters; ++it) mul_k<F, K, CANON>(x, x, y);
  uint64_t r = 0;
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int j = 0; j < kLimbs; ++j) r = r * 31 + x[k].v[j];
  out[gid] = r;
}

// The same on the FP64 multiplier (three independent products per trip).
__global__ void __launch_bounds__(kThreads) ffmul_f64_kernel(uint32_t iters, uint32_t seed,
                                                             uint64_t* __restrict__ out) {
  const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
  Fe x[3], y[3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int j = 0; j < kLimbs; ++j) {
      x[k].v[j] = (j == kLimbs - 1) ? (seed + gid + (uint32_t)k) & 0x0fffffffu : seed * 2654435761u + gid * (j + 1);
      y[k].v[j] = (j == kLimbs - 1) ? (gid * 7u + (uint32_t)k) & 0x0fffffffu : gid * 40503u + (uint32_t)(j * k);
    }
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 3; ++k) x[k] = mul_f64<Bls12_381Fr>(x[k], y[k]);
  }
  uint64_t r = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int j = 0; j < kLimbs; ++j) r = r * 31 + x[k].v[j];
  out[gid] = r;
}

__global__ void __launch_bounds__(kThreads) copy_kernel(uint4* __restrict__ dst, const uint4* __restrict__ src,
                                                        uint64_t nvec) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvec; i += stride) dst[i] = src[i];
}

}  // namespace
}  // namespace zk

extern "C" int zk_microbench(int kind, uint32_t iters, void* d_buf, size_t buf_bytes, void* stream, int reps,
                             double* ops_per_s, float* ms_per_launch) {
  using namespace zk;
  if (!d_buf || !ops_per_s || !ms_per_launch || reps < 1) return ZK_EINVAL;
  if ((reinterpret_cast<uintptr_t>(d_buf) & 255u) != 0) return ZK_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return ZK_EDEVICE;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return ZK_EDEVICE;
  // eight 256-thread workgroups per CU (32 waves, 8 per SIMD); the products
  // run at the pass kernels' occupancy, four waves per SIMD
  const bool ffmul = kind == ZK_MB_FFMUL_BLS12_381 || kind == ZK_MB_FFMUL_K2 || kind == ZK_MB_FFMUL_K4 ||
                     kind == ZK_MB_FFMUL_F64 || kind == ZK_MB_FFMUL_LAZY || kind == ZK_MB_FFMUL_BN254;
  const uint32_t blocks = (uint32_t)cus * (ffmul ? 4u : 8u);
  const uint64_t lanes = (uint64_t)blocks * kThreads;
  double ops = 0;  // per launch
  auto launch = [&]() -> hipError_t {
    uint64_t* out = static_cast<uint64_t*>(d_buf);
    switch (kind) {
      case ZK_MB_MAD_U64_U32:
        hipLaunchKernelGGL(rate_kernel<ZK_MB_MAD_U64_U32>, dim3(blocks), dim3(kThreads), 0, s, iters, 7u, out);
        break;
      case ZK_MB_FMA_F64:
        hipLaunchKernelGGL(rate_kernel<ZK_MB_FMA_F64>, dim3(blocks), dim3(kThreads), 0, s, iters, 7u, out);
        break;
      case ZK_MB_ADD_U32:
        hipLaunchKernelGGL(rate_kernel<ZK_MB_ADD_U32>, dim3(blocks), dim3(kThreads), 0, s, iters, 7u, out);
        break;
      case ZK_MB_ADDC_U32:
        hipLaunchKernelGGL(rate_kernel<ZK_MB_ADDC_U32>, dim3(blocks), dim3(kThreads), 0, s, iters, 7u, out);
        break;
      case ZK_MB_MAD_ADDC:
        hipLaunchKernelGGL(rate_kernel<ZK_MB_MAD_ADDC>, dim3(blocks), dim3(kThreads), 0, s, iters, 7u, out);
        break;
      case ZK_MB_MAD_FMA:
        hipLaunchKernelGGL(rate_kernel<ZK_MB_MAD_FMA>, dim3(blocks), dim3(kThreads), 0, s, iters, 7u, out);
        break;
      case ZK_MB_MAD_ADD:
        hipLaunchKernelGGL(rate_kernel<ZK_MB_MAD_ADD>, dim3(blocks), dim3(kThreads), 0, s, iters, 7u, out);
        break;
      case ZK_MB_FFMUL_BLS12_381:
        hipLaunchKernelGGL((ffmul_kernel<Bls12_381Fr, 3>), dim3(blocks), dim3(kThreads), 0, s, iters, 7u, out);
        break;
      case ZK_MB_FFMUL_K2:
        hipLaunchKernelGGL((ffmul_kernel<Bls12_381Fr, 2>), dim3(blocks), dim3(kThreads), 0, s, iters, 7u, out);
        break;
      case ZK_MB_FFMUL_K4:
        hipLaunchKernelGGL((ffmul_kernel<Bls12_381Fr, 4>), dim3(blocks), dim3(kThreads), 0, s, iters, 7u, out);
        break;
      case ZK_MB_FFMUL_LAZY:
        hipLaunchKernelGGL((ffmul_kernel<Bls12_381Fr, 3, false>), dim3(blocks), dim3(kThreads), 0, s, iters, 7u, out);
        break;
      case ZK_MB_FFMUL_BN254:
        hipLaunchKernelGGL((ffmul_kernel<Bn254Fr, 3>), dim3(blocks), dim3(kThreads), 0, s, iters, 7u, out);
        break;
      case ZK_MB_FFMUL_F64:
        hipLaunchKernelGGL(ffmul_f64_kernel, dim3(blocks), dim3(kThreads), 0, s, iters, 7u, out);
        break;
      case ZK_MB_COPY: {
        const uint64_t nvec = buf_bytes / 32;  // half the buffer read, half written
        hipLaunchKernelGGL(copy_kernel, dim3(blocks), dim3(kThreads), 0, s,
                           reinterpret_cast<uint4*>(static_cast<char*>(d_buf) + nvec * 16),
                           static_cast<const uint4*>(d_buf), nvec);
        break;
      }
      default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
  };
  switch (kind) {
    case ZK_MB_MAD_U64_U32:
    case ZK_MB_FMA_F64:
    case ZK_MB_ADD_U32:
    case ZK_MB_MAD_ADDC:
      ops = (double)lanes * iters * kUnroll * kChains;  // instructions (MAD+ADDC: column steps)
      break;
    case ZK_MB_ADDC_U32:
    case ZK_MB_MAD_FMA:
    case ZK_MB_MAD_ADD:
      ops = (double)lanes * iters * kUnroll * kChains * 2;  // two instructions per step
      break;
    case ZK_MB_FFMUL_BLS12_381:
    case ZK_MB_FFMUL_F64:
    case ZK_MB_FFMUL_LAZY:
    case ZK_MB_FFMUL_BN254:
      ops = (double)lanes * iters * 3;
      break;
    case ZK_MB_FFMUL_K2:
      ops = (double)lanes * iters * 2;
      break;
    case ZK_MB_FFMUL_K4:
      ops = (double)lanes * iters * 4;
      break;
    case ZK_MB_COPY:
      ops = (double)(buf_bytes / 32) * 32;  // bytes read + written
      break;
    default:
      return ZK_EINVAL;
  }
  if (kind != ZK_MB_COPY && buf_bytes < lanes * sizeof(uint64_t)) return ZK_EINVAL;
  if (kind == ZK_MB_COPY && buf_bytes < 64) return ZK_EINVAL;
  if (launch() != hipSuccess) return ZK_EDEVICE;  // warm-up
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return ZK_EDEVICE;
  int rc = ZK_OK;
  if (hipEventRecord(e0, s) != hipSuccess) rc = ZK_EDEVICE;
  for (int r = 0; r < reps && rc == ZK_OK; ++r)
    if (launch() != hipSuccess) rc = ZK_EDEVICE;
  if (rc == ZK_OK && hipEventRecord(e1, s) != hipSuccess) rc = ZK_EDEVICE;
  float ms = 0;
  if (rc == ZK_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
    rc = ZK_EDEVICE;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != ZK_OK) return rc;
  *ms_per_launch = ms / (float)reps;
  *ops_per_s = ops / (*ms_per_launch * 1e-3);
  return ZK_OK;
}
