// Persistent batched NTT kernel: many independent transforms of uneven sizes
// and both fields in one launch.
//
// The paper finds GPU NTTs run as short, bursty kernels with launch
// parameters that fit some sizes badly (Section IV-A: the energy comparison of
// Table III and the radix-256 schedule whose last kernel launches 16M
// two-thread blocks); Section V-A asks for autotuning of such parameters.  Here a
// batch of jobs becomes work queues of (job, pass, tile) items, each queue
// pass-major (its jobs' pass 0 tiles, then their pass 1 tiles, ...), larger
// jobs first.  A grid of persistent workgroups drains the queues.
//
// XCD locality.  MI355X has eight XCDs, each with its own L2; the L2s are not
// coherent with each other inside a kernel, so passing data between
// workgroups on different XCDs needs an L2 writeback at the producer and an
// L2 invalidate at the consumer (agent-scope release/acquire), which measured
// slower than the transforms themselves when done once per tile.  Instead a
// queue is claimed by one XCD (the owner word holds the XCC id read from the
// hardware register) and only that XCD's workgroups pop from it, so every
// tile of a job runs under one L2.  Producer and consumer then synchronise as
// workgroups sharing an L2 do: the producer waits for its stores to complete
// (the vector L1 writes through to L2) before counting the tile done, and
// the consumer invalidates its CU's L1 after the count is reached.
// Workgroups claim a new queue only when their XCD's queues have nothing
// left to pop, which balances the XCDs dynamically.
//
// Progress.  An item of pass p waits until all tiles of its job's pass p-1
// are done.  Items of a queue are popped in order by running workgroups, so
// every tile a waiting item depends on was popped earlier by a workgroup
// that is running it: the wait always ends.  It is also bounded: past
// `spin_limit` polls the workgroup sets the error flag and every workgroup
// exits, so a fault cannot hang the device.  The last workgroup to exit
// checks that every item ran.
//
// Each tile computes exactly what the single-transform pass kernels compute,
// so a job's result is bit-identical to its stand-alone transform.
#include "ntt_batch.hpp"
#include "ntt_pass_impl.hpp"

namespace zk {
namespace {

// Tiles of 2^kBatchTileLog elements computed with the radix-4 register
// schedule: four elements per thread.
constexpr int kBatchLogE = 2;
constexpr int kBatchThreads = (1 << kBatchTileLog) >> kBatchLogE;
constexpr int kBatchLdsSlots = (1 << kBatchTileLog) + (1 << kBatchTileLog) / 8;
constexpr int kBatchWgsPerCu = 163840 / (kBatchLdsSlots * 32);  // LDS limit
// Products interleaved per group in the batch tile body: two and three fit
// 128 VGPRs without spills (four spills 28); two measured faster.
constexpr int kDynGroup = 2;

// Control words are read and written with relaxed device-scope atomics.
__device__ __forceinline__ uint32_t load_relaxed(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t xcc_id() {
  // HW_REG_XCC_ID (hardware register 20), bits [3:0]
  return __builtin_amdgcn_s_getreg((20) | (0 << 6) | ((4 - 1) << 11));
}

// Release of a finished tile to workgroups under the same L2: every thread's
// stores have completed at L2 once its memory counters drain.
__device__ __forceinline__ void release_to_l2() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0);
}

// Acquire of tiles released under the same L2: drop this CU's L1 lines so
// the loads that follow read L2.
__device__ __forceinline__ void acquire_from_l2() {
  asm volatile("buffer_inv sc0" ::: "memory");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// One tile of one pass with the pass shape taken at run time: J columns x R
// points (R = 2^log_r, J R = 2^log_tile), four points per thread, radix-4
// register rounds and, when log_r is odd, a final radix-2 round.  The
// arithmetic is that of pass_tile with LOG_E = 2 step for step (same loads,
// same twiddle exponents, same butterflies in the same order), so the bytes
// equal those of the stand-alone kernels; only the index arithmetic is
// computed at run time, so the persistent loop holds one tile body per field
// and its register allocation is that of a single shape.  Threads t >=
// 2^(log_tile - 2) shadow thread t mod 2^(log_tile - 2) and store nothing.
// log_r and log_tile are wave-uniform; 2 <= log_r <= log_tile <= 11.  (Batch
// jobs never carry kPassPostPointwise: the pointwise step is a job of its own.)
// Like the pass kernels it keeps the data in [0, 2p) inside the tile and
// stores canonical values, so the stored bytes are the same.
template <class F>
__device__ __forceinline__ void tile_dyn(const PassArgs& a, int log_r, int log_tile, uint32_t tile, Fe* lds) {
  using detail::lds_slot;
  using detail::load_fe;
  using detail::sfor;
  const int log_threads = log_tile - 2;
  const bool writer = threadIdx.x < (1u << log_threads);
  const uint32_t t = threadIdx.x & ((1u << log_threads) - 1);
  const int log_j = log_tile - log_r;
  const uint32_t J = 1u << log_j;
  const uint32_t c = t & (J - 1);
  const uint32_t q = t >> log_j;
  const uint32_t R = 1u << log_r;
  const uint32_t quarter = R >> 2;  // threads per column
  const uint64_t n = 1ull << a.log_n;
  const uint64_t ns = 1ull << a.log_ns;
  const uint64_t j = (uint64_t)tile * J + c;
  const uint32_t log_stride = a.log_n - log_r;

  // round 0 is radix 4: thread q holds points q + e R/4
  Fe v[4];
  const bool rev = a.flags & kPassReverseIn;
  sfor<4>([&](auto e_) {
    constexpr int e = decltype(e_)::value;
    const uint64_t idx = j + ((uint64_t)(q + e * quarter) << log_stride);
    v[e] = load_fe(a.in, rev ? ((n - idx) & (n - 1)) : idx);
  });
  Fe w[4];
  if (a.flags & kPassPreTable) {
    sfor<4>([&](auto e_) {
      constexpr int e = decltype(e_)::value;
      w[e] = load_fe(a.pre_table, j + ((uint64_t)(q + e * quarter) << log_stride));
    });
    detail::mul_many<F, 4, kDynGroup>(v, w);
  }
  if (a.tw_pass) {
    sfor<4>([&](auto e_) {
      constexpr int e = decltype(e_)::value;
      w[e] = load_fe(a.tw_pass, ((uint64_t)(q + e * quarter) << a.log_ns) + (j & (ns - 1)));
    });
    detail::mul_many<F, 4, kDynGroup>(v, w);
  } else if (a.tw_hi) {
    // two points at a time, as in pass_tile, to keep the register peak down
    const uint64_t jm = j & (ns - 1);
    const uint32_t log_mult = a.log_n - a.log_ns - log_r;
    const uint64_t lo_mask = (1ull << a.log_lo) - 1;
    sfor<2>([&](auto h_) {
      constexpr int h = decltype(h_)::value;
      Fe hi[2], lo[2];
      sfor<2>([&](auto k_) {
        constexpr int e = 2 * h + decltype(k_)::value;
        const uint64_t ex = ((uint64_t)(q + e * quarter) * jm) << log_mult;
        hi[e - 2 * h] = load_fe(a.tw_hi, ex >> a.log_lo);
        lo[e - 2 * h] = load_fe(a.tw_lo, ex & lo_mask);
      });
      detail::mul_many<F, 2, 2, true>(hi, lo);  // canonical: the factor of the next product
      detail::mul_many<F, 2, 2>(v + 2 * h, hi);
    });
  }

  const int r4 = log_r >> 1;  // radix-4 rounds
  const bool odd = log_r & 1;
  for (int rho = 0; rho < r4; ++rho) {
    const int log_nsr = 2 * rho;
    const uint32_t nsr = 1u << log_nsr;
    if (rho > 0) {
      sfor<4>([&](auto e_) {
        constexpr int e = decltype(e_)::value;
        v[e] = lds[lds_slot((q + e * quarter) * J + c)];
      });
      // in-tile twiddles w_{4 Nsr}^(s (q mod Nsr)) for s = 1, 2, 3
      const uint32_t im = q & (nsr - 1);
      const int log_step = log_r - log_nsr - 2;  // R / (Nsr 4)
      Fe ws[3];
      sfor<3>([&](auto k_) {
        constexpr int k = decltype(k_)::value;
        ws[k] = load_fe(a.tw_r, ((k + 1) * im) << log_step);
      });
      detail::mul_many<F, 3, kDynGroup>(v + 1, ws);
    }
    Fe W[2];
    W[0] = load_fe(a.tw_r, 0);
    W[1] = load_fe(a.tw_r, quarter);  // w_4
    detail::dft_regs<F, 2, 0>(v, W);
    const bool last = !odd && rho == r4 - 1;
    if (!last) {
      if (rho > 0) __syncthreads();
      if (writer) {
        sfor<4>([&](auto e_) {
          constexpr int e = decltype(e_)::value;
          const uint32_t o = ((q >> log_nsr) << (log_nsr + 2)) + (q & (nsr - 1)) + e * nsr;
          lds[lds_slot(o * J + c)] = v[e];
        });
      }
      __syncthreads();
    }
  }
  if (odd) {
    // final radix-2 round: thread q owns slots i = q + g R/4 (g < 2), each
    // taking points i and i + R/2
    const int log_nsr = 2 * r4;
    const uint32_t nsr = 1u << log_nsr;
    const uint32_t half = R >> 1;
    sfor<4>([&](auto e_) {
      constexpr int e = decltype(e_)::value;
      const uint32_t i = q + (e >> 1) * quarter;
      v[e] = lds[lds_slot((i + (e & 1) * half) * J + c)];
    });
    Fe ys[2], ws[2];
    sfor<2>([&](auto g_) {
      constexpr int g = decltype(g_)::value;
      const uint32_t im = (q + g * quarter) & (nsr - 1);
      ys[g] = v[2 * g + 1];
      ws[g] = load_fe(a.tw_r, im);  // w_{2 Nsr}^im = tw_r[im R / (2 Nsr)], and R = 2 Nsr here
    });
    detail::mul_many<F, 2, kDynGroup>(ys, ws);
    v[1] = ys[0];
    v[3] = ys[1];
    Fe W[1];
    W[0] = load_fe(a.tw_r, 0);
    detail::dft_regs<F, 1, 0>(v, W);
    detail::dft_regs<F, 1, 2>(v, W);
  }

  // output r_out of column j goes to (j / Ns) Ns R + (j mod Ns) + r_out Ns
  const uint64_t base = ((j >> a.log_ns) << (a.log_ns + log_r)) + (j & (ns - 1));
  auto out_index = [&](int e) -> uint64_t {
    const uint32_t r_out = odd ? q + (e >> 1) * quarter + (e & 1) * (R >> 1) : q + e * quarter;
    return base + ((uint64_t)r_out << a.log_ns);
  };
  if (a.flags & kPassPostTable) {
    sfor<4>([&](auto e_) {
      constexpr int e = decltype(e_)::value;
      w[e] = load_fe(a.post_table, out_index(e));
    });
    detail::mul_many<F, 4, kDynGroup>(v, w);
  }
  if (a.flags & kPassPostConst) {
    sfor<4>([&](auto e_) {
      constexpr int e = decltype(e_)::value;
      w[e] = a.post_const;
    });
    detail::mul_many<F, 4, kDynGroup>(v, w);
  }
  if (writer) {  // canonical out, as the pass kernels
    sfor<4>([&](auto e_) {
      constexpr int e = decltype(e_)::value;
      detail::store_fe(a.out, out_index(e), canon<F>(v[e]));
    });
  }
}

// Pointwise quotient step on one tile: 2^11 elements, lanes on consecutive
// elements.
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

// Shared state of the persistent loop.
struct QueueCtl {
  const BatchJob* __restrict__ jobs;
  const BatchItem* __restrict__ items;
  const BatchQueue* __restrict__ queues;
  uint32_t* ctl;
  uint32_t spin_limit;
  uint32_t me;  // this XCD's owner tag: XCC id + 1
};

// Workgroup-shared scratch of the loop; values read back from it are made
// wave-uniform with readfirstlane, so every branch of the loop is uniform and
// all threads reach each barrier together.  (Were the exits derived from
// plain LDS reads, the compiler could treat them as divergent and
// restructure the loop so that thread 0 finishes its queue work after the
// other threads have passed the next barrier.)
struct LoopShared {
  uint32_t item;
  uint32_t abort;
  uint32_t pick;
};

constexpr uint32_t kNone = 0xffffffffu;

__device__ __forceinline__ uint32_t* queue_head(uint32_t* ctl, uint32_t q) { return ctl + kCtlQueues + 2 * q; }
__device__ __forceinline__ uint32_t* queue_owner(uint32_t* ctl, uint32_t q) { return ctl + kCtlQueues + 2 * q + 1; }

// A queue in [lo, hi) for this XCD to pop from: one it owns with items left,
// else one it claims now; kNone when every queue of the range is claimed and
// this XCD's are exhausted.  Wave 0 scans the queues a lane each.
__device__ __forceinline__ uint32_t find_queue(const QueueCtl& c, uint32_t lo, uint32_t hi, LoopShared* sh) {
  if (threadIdx.x < 64) {
    const uint32_t q = lo + threadIdx.x;
    const bool valid = q < hi;
    uint32_t pick = kNone;
    for (;;) {
      const uint32_t owner = valid ? load_relaxed(queue_owner(c.ctl, q)) : kNone;
      const uint32_t head = valid ? load_relaxed(queue_head(c.ctl, q)) : kNone;
      const uint32_t size = valid ? c.queues[q].size : 0;
      const uint64_t mine = __ballot(valid && owner == c.me && head < size);
      if (mine) {
        pick = lo + (uint32_t)(__ffsll((unsigned long long)mine) - 1);
        break;
      }
      const uint64_t free_q = __ballot(valid && owner == 0);
      if (!free_q) break;
      const uint32_t lane = (uint32_t)(__ffsll((unsigned long long)free_q) - 1);
      bool won = false;
      if (threadIdx.x == lane) {
        uint32_t expected = 0;
        won = __hip_atomic_compare_exchange_strong(queue_owner(c.ctl, q), &expected, c.me, __ATOMIC_RELAXED,
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      if (__ballot(won)) {
        pick = lo + lane;
        break;
      }
      // another XCD claimed that queue first; scan again (each queue is
      // claimed once, so this ends)
    }
    if (threadIdx.x == 0) sh->pick = pick;
  }
  __syncthreads();
  const uint32_t pick = __builtin_amdgcn_readfirstlane(sh->pick);
  __syncthreads();
  return pick;
}

// Pop the next index of queue q for the whole workgroup; kNone once the error
// flag is set.
__device__ __forceinline__ uint32_t pop(const QueueCtl& c, uint32_t q, LoopShared* sh) {
  if (threadIdx.x == 0) {
    sh->item = atomicAdd(queue_head(c.ctl, q), 1u);
    sh->abort = load_relaxed(c.ctl + kCtlError);
  }
  __syncthreads();
  const uint32_t it = __builtin_amdgcn_readfirstlane(sh->item);
  const uint32_t abort = __builtin_amdgcn_readfirstlane(sh->abort);
  __syncthreads();
  return abort != 0 ? kNone : it;
}

// Run one item; false if its dependency wait failed.
template <class F>
__device__ __forceinline__ bool run_item(const QueueCtl& c, uint32_t it, Fe* lds, LoopShared* sh) {
  const uint32_t job_id = __builtin_amdgcn_readfirstlane(c.items[it].job);
  const uint32_t pass = __builtin_amdgcn_readfirstlane(c.items[it].pass);
  const uint32_t tile = __builtin_amdgcn_readfirstlane(c.items[it].tile);
  const BatchJob& job = c.jobs[job_id];
  uint32_t* done = c.ctl + kCtlDone + job_id * kMaxBatchPasses;
  if (pass > 0) {
    if (threadIdx.x == 0) {
      const uint32_t need = job.pass[pass - 1].tiles;
      if (c.spin_limit == 0) {
        atomicOr(c.ctl + kCtlError, kBatchErrWait);  // test hook: every dependency wait fails at once
      } else {
        uint32_t spins = 0;
        while (load_relaxed(done + pass - 1) < need) {
          __builtin_amdgcn_s_sleep(2);
          if (++spins > c.spin_limit) {
            atomicOr(c.ctl + kCtlError, kBatchErrWait);
            break;
          }
        }
      }
      sh->abort = load_relaxed(c.ctl + kCtlError);
    }
    __syncthreads();
    const uint32_t failed = __builtin_amdgcn_readfirstlane(sh->abort);
    if (failed != 0) return false;
    acquire_from_l2();
  }
  const uint32_t kind = __builtin_amdgcn_readfirstlane(job.kind);
  if (kind == kJobPointwise) {
    run_pointwise<F>(job.pw, tile);
  } else {
    const BatchPass& bp = job.pass[pass];
    const int log_r = __builtin_amdgcn_readfirstlane(bp.log_r);
    const int log_tile = __builtin_amdgcn_readfirstlane(bp.log_tile);
    tile_dyn<F>(bp.args, log_r, log_tile, tile, lds);
  }
  release_to_l2();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_fetch_add(done + pass, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return true;
}

// Drain this XCD's share of queues [lo, hi), all on field F, counting the
// items run in `ran`; false once the error flag stops the batch.  Each field
// has its own loop so that each loop body is register-allocated for one
// field's arithmetic alone.
template <class F>
__device__ __forceinline__ bool drain(const QueueCtl& c, uint32_t lo, uint32_t hi, Fe* lds, LoopShared* sh,
                                      uint32_t& ran) {
  uint32_t q = find_queue(c, lo, hi, sh);
  while (q != kNone) {
    const uint32_t k = pop(c, q, sh);
    if (k == kNone) return false;
    if (k < c.queues[q].size) {
      if (!run_item<F>(c, c.queues[q].base + k, lds, sh)) return false;
      ++ran;
    } else {
      q = find_queue(c, lo, hi, sh);
    }
  }
  return true;
}

__global__ void __launch_bounds__(kBatchThreads, kBatchWgsPerCu * kBatchThreads / 256)
    ntt_batch_kernel(const BatchJob* __restrict__ jobs, const BatchItem* __restrict__ items,
                     const BatchQueue* __restrict__ queues, uint32_t q_end0, uint32_t q_end1, uint32_t q_end2,
                     uint32_t nitems, uint32_t* ctl) {
  __shared__ Fe lds[kBatchLdsSlots];
  __shared__ LoopShared sh;
  const QueueCtl c{jobs, items, queues, ctl, ctl[kCtlSpinLimit],
                   (uint32_t)__builtin_amdgcn_readfirstlane(xcc_id()) + 1u};
  // Items run by this workgroup, added to the shared count once at exit: a
  // device-scope atomic on one word per item serialised every item of the
  // batch behind it.
  uint32_t ran = 0;
  if (drain<Bls12_381Fr>(c, 0, q_end0, lds, &sh, ran) && drain<Bn254Fr>(c, q_end0, q_end1, lds, &sh, ran))
    drain<Bls12_377Fr>(c, q_end1, q_end2, lds, &sh, ran);

  // The last workgroup out checks that every item ran (acquire-release on
  // the exit count orders each workgroup's item count before its exit).
  __syncthreads();
  if (threadIdx.x == 0) {
    if (ran) __hip_atomic_fetch_add(ctl + kCtlItemsDone, ran, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t exited = __hip_atomic_fetch_add(ctl + kCtlExited, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (exited + 1 == gridDim.x && load_relaxed(ctl + kCtlItemsDone) != nitems)
      atomicOr(ctl + kCtlError, kBatchErrIncomplete);
  }
}

// Zero the control words (a kernel rather than a memset so the sequence can
// live in a graph); the poll limit is kept.
__global__ void __launch_bounds__(256) ntt_batch_reset_kernel(uint32_t* ctl, uint32_t nwords) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nwords && i != kCtlSpinLimit) ctl[i] = 0;
}

}  // namespace

bool batch_shape_supported(int log_r, int log_tile) {
  return log_r >= 2 && log_r <= log_tile && log_tile <= kBatchTileLog;
}

hipError_t launch_batch(const BatchJob* jobs, const BatchItem* items, const BatchQueue* queues,
                        const uint32_t nq_end[3], uint32_t nitems, uint32_t* ctl, uint32_t njobs, uint32_t grid,
                        hipStream_t s) {
  const uint32_t nwords = kCtlDone + njobs * kMaxBatchPasses;
  hipLaunchKernelGGL(ntt_batch_reset_kernel, dim3((nwords + 255) / 256), dim3(256), 0, s, ctl, nwords);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (nitems == 0 || grid == 0) return hipSuccess;
  hipLaunchKernelGGL(ntt_batch_kernel, dim3(grid), dim3(kBatchThreads), 0, s, jobs, items, queues, nq_end[0],
                     nq_end[1], nq_end[2], nitems, ctl);
  return hipGetLastError();
}

int batch_workgroups_per_cu() { return kBatchWgsPerCu; }

}  // namespace zk
