// Persistent batched NTT kernel: many independent transforms of uneven sizes
// and both fields in one launch.
//
// The paper finds GPU NTTs run as short, bursty kernels with launch
// parameters that fit some sizes badly (Section IV-A: the energy comparison of
// Table III and the radix-256 schedule whose last kernel launches 16M
// two-thread blocks); Section V-A asks for autotuning of such parameters.  Here a
// batch of jobs becomes one work list of (job, pass, tile) items, ordered
// pass-major (every job's pass 0 tiles, then every pass 1 tile, ...), with
// larger jobs first inside a pass.  A grid of persistent workgroups pops items
// from an atomic counter.  An item of pass p waits until all tiles of its
// job's pass p-1 are done; because items are popped in list order, every tile
// it waits for was popped earlier by a running workgroup, so the wait always
// ends.  The wait is also bounded: past `spin_limit` polls the workgroup sets
// the error flag and every workgroup exits, so a fault cannot hang the device.
//
// Each tile runs the same pass_tile code as the single-transform kernels, so
// a job's result is bit-identical to its stand-alone transform.
#include "ntt_batch.hpp"
#include "ntt_pass_impl.hpp"

namespace zk {
namespace {

constexpr int kBatchThreads = 256;
constexpr int kBatchLdsSlots = (1 << 11) + (1 << 11) / 8;

__device__ __forceinline__ uint32_t load_acquire(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Inlined (not a call) so that log_r and log_tile stay wave-uniform scalars
// and every branch around the tile's barriers is a uniform scalar branch.
template <class F>
__device__ __forceinline__ void run_tile(const PassArgs& a, int log_r, int log_tile, uint32_t tile, Fe* lds) {
  const uint32_t t = threadIdx.x;
  if (log_tile == 11) {
    switch (log_r) {
      case 5: detail::pass_tile<F, 5, 11, 3>(a, tile, lds, t, true); return;
      case 6: detail::pass_tile<F, 6, 11, 3>(a, tile, lds, t, true); return;
      case 7: detail::pass_tile<F, 7, 11, 3>(a, tile, lds, t, true); return;
      case 8: detail::pass_tile<F, 8, 11, 3>(a, tile, lds, t, true); return;
      case 11: detail::pass_tile<F, 11, 11, 3>(a, tile, lds, t, true); return;
      default: return;
    }
  }
  if (log_tile == 10 && log_r == 10) {
    // 128 threads cover the tile; the upper half shadows the lower half.
    detail::pass_tile<F, 10, 10, 3>(a, tile, lds, t & 127u, t < 128u);
  }
}

// Pointwise quotient step on one tile: 2^11 elements, 8 per thread, lanes on
// consecutive elements.
template <class F>
__device__ __forceinline__ void run_pointwise(const PointwiseArgs& pw, uint32_t tile) {
  const uint64_t base = ((uint64_t)tile << kPointwiseTileLog) + threadIdx.x;
#pragma unroll
  for (int e = 0; e < (1 << kPointwiseTileLog) / kBatchThreads; ++e) {
    const uint64_t i = base + (uint64_t)e * kBatchThreads;
    if (i < pw.n) {
      const Fe ab = mul<F>(detail::load_fe(pw.a, i), detail::load_fe(pw.b, i));
      detail::store_fe(pw.out, i, mul<F>(sub<F>(ab, detail::load_fe(pw.c, i)), pw.zinv));
    }
  }
}

__global__ void __launch_bounds__(kBatchThreads) ntt_batch_kernel(const BatchJob* __restrict__ jobs,
                                                                 const BatchItem* __restrict__ items,
                                                                 uint32_t nitems, uint32_t* ctl) {
  __shared__ Fe lds[kBatchLdsSlots];
  __shared__ uint32_t s_item;
  __shared__ uint32_t s_abort;
  uint32_t* head = ctl + kCtlHead;
  uint32_t* error = ctl + kCtlError;
  const uint32_t spin_limit = ctl[kCtlSpinLimit];
  uint32_t* done = ctl + kCtlDone;

  // Every loop exit and branch below depends only on values made
  // wave-uniform with readfirstlane, so the loop stays a uniform loop and all
  // threads reach each barrier together.  (Were the exits derived from plain
  // LDS reads, the compiler could treat them as divergent and restructure the
  // loop so that thread 0 finishes its queue work after the other threads
  // have already passed the next barrier.)
  for (;;) {
    if (threadIdx.x == 0) {
      s_item = atomicAdd(head, 1u);
      s_abort = load_acquire(error);
    }
    __syncthreads();
    const uint32_t it = __builtin_amdgcn_readfirstlane(s_item);
    const uint32_t abort = __builtin_amdgcn_readfirstlane(s_abort);
    __syncthreads();
    if (abort != 0 || it >= nitems) break;

    const uint32_t job_id = __builtin_amdgcn_readfirstlane(items[it].job);
    const uint32_t pass = __builtin_amdgcn_readfirstlane(items[it].pass);
    const uint32_t tile = __builtin_amdgcn_readfirstlane(items[it].tile);
    const BatchJob& job = jobs[job_id];
    if (pass > 0) {
      if (threadIdx.x == 0) {
        const uint32_t need = job.pass[pass - 1].tiles;
        const uint32_t* cnt = done + job_id * kMaxBatchPasses + (pass - 1);
        if (spin_limit == 0) {
          atomicOr(error, 1u);  // test hook: every dependency wait fails at once
        } else {
          uint32_t spins = 0;
          while (load_acquire(cnt) < need) {
            __builtin_amdgcn_s_sleep(2);
            if (++spins > spin_limit) {
              atomicOr(error, 1u);
              break;
            }
          }
        }
        s_abort = load_acquire(error);
      }
      __syncthreads();
      const uint32_t failed = __builtin_amdgcn_readfirstlane(s_abort);
      if (failed != 0) break;
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    const uint32_t kind = __builtin_amdgcn_readfirstlane(job.kind);
    const uint32_t field = __builtin_amdgcn_readfirstlane(job.field);
    if (kind == kJobPointwise) {
      if (field == Bls12_381Fr::ID) run_pointwise<Bls12_381Fr>(job.pw, tile);
      else run_pointwise<Bn254Fr>(job.pw, tile);
    } else {
      const BatchPass& bp = job.pass[pass];
      const int log_r = __builtin_amdgcn_readfirstlane(bp.log_r);
      const int log_tile = __builtin_amdgcn_readfirstlane(bp.log_tile);
      if (field == Bls12_381Fr::ID) run_tile<Bls12_381Fr>(bp.args, log_r, log_tile, tile, lds);
      else run_tile<Bn254Fr>(bp.args, log_r, log_tile, tile, lds);
    }

    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // this thread's stores are visible device-wide
    __syncthreads();                                     // ... for every thread of the tile
    if (threadIdx.x == 0) {
      __hip_atomic_fetch_add(done + job_id * kMaxBatchPasses + pass, 1u, __ATOMIC_RELEASE,
                             __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Zero the queue head, the error flag and the completion counters (a kernel
// rather than a memset so the sequence can live in a graph).
__global__ void __launch_bounds__(256) ntt_batch_reset_kernel(uint32_t* ctl, uint32_t ndone) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    ctl[kCtlHead] = 0;
    ctl[kCtlError] = 0;
  }
  if (i < ndone) ctl[kCtlDone + i] = 0;
}

}  // namespace

bool batch_shape_supported(int log_r, int log_tile) {
  if (log_tile == 11) return (log_r >= 5 && log_r <= 8) || log_r == 11;
  return log_tile == 10 && log_r == 10;
}

hipError_t launch_batch(const BatchJob* jobs, const BatchItem* items, uint32_t nitems, uint32_t* ctl,
                        uint32_t njobs, uint32_t grid, hipStream_t s) {
  const uint32_t ndone = njobs * kMaxBatchPasses;
  hipLaunchKernelGGL(ntt_batch_reset_kernel, dim3((ndone + 255) / 256 + 1), dim3(256), 0, s, ctl, ndone);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (nitems == 0 || grid == 0) return hipSuccess;
  hipLaunchKernelGGL(ntt_batch_kernel, dim3(grid), dim3(kBatchThreads), 0, s, jobs, items, nitems, ctl);
  return hipGetLastError();
}

int batch_workgroups_per_cu() { return 1; }  // registers: one 256-thread workgroup per CU

}  // namespace zk
