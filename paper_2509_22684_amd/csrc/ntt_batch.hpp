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

constexpr int kPointwiseTileLog = 11;

struct BatchItem {
  uint32_t job;
  uint32_t pass;
  uint32_t tile;
  uint32_t pad;
};

// Control words in device memory: queue head, error flag, the poll limit of
// a dependency wait, then one completion counter per (job, pass).
enum : uint32_t { kCtlHead = 0, kCtlError = 1, kCtlSpinLimit = 2, kCtlDone = 4 };

bool batch_shape_supported(int log_r, int log_tile);
int batch_workgroups_per_cu();

// Reset the control words of njobs jobs, then launch `grid` persistent
// workgroups over `nitems` items, of which items [0, nfirst) belong to
// BLS12-381 Fr jobs and the rest to BN254 Fr jobs.
hipError_t launch_batch(const BatchJob* jobs, const BatchItem* items, uint32_t nitems, uint32_t nfirst,
                        uint32_t* ctl, uint32_t njobs, uint32_t grid, hipStream_t s);

}  // namespace zk
