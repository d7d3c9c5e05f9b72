// MSM launch helpers (internal); see msm.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace zk {
namespace msm {

constexpr int kPointWords = 24;  // affine point: x, y as 12 limbs each
constexpr int kXyzzWords = 48;   // X, Y, ZZ, ZZZ

// Everything one MSM launch touches; the buffers are slices of the caller's
// workspace (sizes in msm_workspace_bytes).
struct MsmLaunch {
  const uint32_t* table;    // windows x n affine points: 2^(c w) P_i
  const uint32_t* scalars;  // n x 8 limbs, Montgomery form over BLS12-381 Fr
  uint64_t n;
  int c;                    // window bits
  int windows;
  uint32_t slices;          // lanes per bucket in the accumulation
  uint32_t chunk;           // partials summed per lane in the reduction
  uint16_t* digits;         // windows x n
  uint32_t* counts;         // 2^c
  uint32_t* offsets;        // 2^c + 1
  uint32_t* ranks;          // windows x n: an entry's place in its bucket
  uint32_t* entries;        // windows x n
  uint32_t* partial;        // 2^c x slices XYZZ
  uint32_t* buckets;        // 2^c XYZZ
  uint32_t* level_a;        // c x ceil(2^c / chunk) XYZZ
  uint32_t* level_b;        // same
  uint32_t* result;         // one XYZZ point
};

// table[w n + i] = 2^(c w) P_i for points first .. first + count of n;
// scratch: count x windows x 60 words.
hipError_t launch_precompute(const uint32_t* pts, uint64_t n, uint64_t first, uint64_t count, int c, int windows,
                             uint32_t* table, uint32_t* scratch, hipStream_t s);
hipError_t launch_msm(const MsmLaunch& m, hipStream_t s);

}  // namespace msm
}  // namespace zk
