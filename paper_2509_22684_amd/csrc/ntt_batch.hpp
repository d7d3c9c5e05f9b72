// Batched persistent NTT launch: device descriptors and launch helper
// (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "ntt_kernels.hpp"

namespace zk {

constexpr int kMaxBatchPasses = 4;

// One pass of one job: the same arguments a stand-alone launch would get.
struct BatchPass {
  PassArgs args;
  int32_t log_r;
  int32_t log_tile;
  uint32_t tiles;  // workgroup tiles in this pass
  uint32_t pad;
};

// out_i = (a_i b_i - c_i) zinv for i < n, in tiles of 2^11 elements.
struct PointwiseArgs {
  const Fe* a;
  const Fe* b;
  const Fe* c;
  Fe* out;
  Fe zinv;
  uint64_t n;
  uint64_t pad;
};

enum BatchJobKind : uint32_t { kJobTransform = 0, kJobPointwise = 1 };

struct BatchJob {
  BatchPass pass[kMaxBatchPasses];
  PointwiseArgs pw;
  uint32_t field;
  uint32_t npasses;  // transform: passes; pointwise: 1
  uint32_t kind;     // BatchJobKind
  uint32_t pad;
};

// Batch tiles: 2^11 elements, 512 threads of four elements, two workgroups
// per CU (the LDS limit).  Multi-pass jobs run in tiles of this size; jobs up
// to this size run whole in one tile.  (2^10-element tiles, the stand-alone
// default, measured slower here: twice the items, each with its queue pop,
// dependency check and completion count.)
#ifndef ZK_BATCH_TILE_LOG
#define ZK_BATCH_TILE_LOG 11
#endif
constexpr int kBatchTileLog = ZK_BATCH_TILE_LOG;
constexpr int kPointwiseTileLog = kBatchTileLog;

struct BatchItem {
  uint32_t job;
  uint32_t pass;
  uint32_t tile;
  uint32_t pad;
};

// A work queue: items [base, base + size) of the item array, all from jobs
// on one field, pass-major.  Every job's items sit in exactly one queue, and
// a queue is drained by the workgroups of the one XCD that claims it.
struct BatchQueue {
  uint32_t base;
  uint32_t size;
  uint32_t field;
  uint32_t pad;
};

// A job whose tiles exceed this fraction of the batch's tiles (1 / XCDs)
// would be the batch's critical path on one XCD; such jobs run instead as
// their own pass launches (all XCDs), ahead of the persistent kernel.
constexpr int kXcds = 8;

// Per field at most 32 queues: one wave scans a field's queues at once, a
// lane per queue.  Three fields.
constexpr int kMaxLocalQueues = 32;
constexpr int kMaxQueues = 3 * kMaxLocalQueues;

// Control words in device memory: error flag, poll limit of a dependency
// wait, count of exited workgroups, count of finished items, then per queue a
// pop counter and an owner word (0 = unclaimed, else XCC id + 1), then one
// completion counter per (job, pass).
enum : uint32_t {
  kCtlError = 0,
  kCtlSpinLimit = 1,
  kCtlExited = 2,
  kCtlItemsDone = 3,
  kCtlQueues = 4,
  kCtlDone = kCtlQueues + 2 * kMaxQueues
};

// Error flag values.
enum : uint32_t { kBatchErrWait = 1, kBatchErrIncomplete = 2 };

bool batch_shape_supported(int log_r, int log_tile);
int batch_workgroups_per_cu();

// Reset the control words of njobs jobs, then launch `grid` persistent
// workgroups over the queues: queues [0, nq_end[0]) hold BLS12-381 Fr work,
// [nq_end[0], nq_end[1]) BN254 Fr work, [nq_end[1], nq_end[2]) BLS12-377 Fr
// work; nitems items in all.
hipError_t launch_batch(const BatchJob* jobs, const BatchItem* items, const BatchQueue* queues,
                        const uint32_t nq_end[3], uint32_t nitems, uint32_t* ctl, uint32_t njobs, uint32_t grid,
                        hipStream_t s);

}  // namespace zk
