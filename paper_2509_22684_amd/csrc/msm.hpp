// MSM launch helpers (internal); see msm.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace zk {
namespace msm {

constexpr int kPointWords = 24;  // affine point: x, y as 12 limbs each
constexpr int kXyzzWords = 48;   // X, Y, ZZ, ZZZ
constexpr uint32_t kChunk = 8;         // buckets per chunk in the reduction by bits
constexpr uint32_t kLevel0Lanes = 64;  // level-0 lanes summed per result in the reduction by bits
constexpr uint32_t kLevel0Chunks = 2;  // chunks per level-0 lane

// Everything one MSM launch touches; the buffers are slices of the caller's
// workspace (sizes in msm_workspace_bytes).
struct MsmLaunch {
  const uint32_t* table;    // windows x n affine points: 2^(c w) P_i
  const uint32_t* scalars;  // n x 8 limbs, Montgomery form over BLS12-381 Fr
  uint64_t n;
  int c;                    // window bits
  int windows;
  uint32_t per_group;       // scalars per histogram group, per_group x windows <= 65535
  uint32_t groups;          // ceil(n / per_group)
  uint32_t lanes;           // accumulation lanes (accumulate_lanes)
  uint32_t kmin;            // fewest sorted entries per lane
  uint16_t* digits;         // windows x n
  uint16_t* ranks;          // windows x n: an entry's place among its group's entries of its bucket
  uint32_t* hist;           // groups x 2^c
  uint32_t* counts;         // 2^c
  uint32_t* offsets;        // 2^c + 1
  uint32_t* entries;        // windows x n
  uint32_t* head;           // lanes XYZZ
  uint32_t* tail;           // lanes XYZZ
  uint32_t* big;            // max_big_buckets(lanes) bucket indices
  uint32_t* big_count;      // one word
  uint32_t* buckets;        // 2^c XYZZ
  uint32_t* chunk_sums;     // ceil(2^c / kChunk) XYZZ
  uint32_t* level_a;        // c x ceil(ceil(2^c / kChunk) / (kLevel0Lanes kLevel0Chunks)) XYZZ
  uint32_t* level_b;        // c XYZZ
  uint32_t* result;         // one XYZZ point
};

// table[w n + i] = 2^(c w) P_i for points first .. first + count of n;
// scratch: count x windows x 60 words.
hipError_t launch_precompute(const uint32_t* pts, uint64_t n, uint64_t first, uint64_t count, int c, int windows,
                             uint32_t* table, uint32_t* scratch, hipStream_t s);
// A combine lane adds at most kCombineSerial runs' heads; a bucket spanning
// more runs is listed for a workgroup.  Such buckets own more than
// kCombineSerial run starts each, so at most lanes / kCombineSerial + 1.
constexpr uint32_t kCombineSerial = 16;
inline uint32_t max_big_buckets(uint32_t lanes) { return lanes / kCombineSerial + 1u; }

// Accumulation lanes that are resident on the current device at once.
hipError_t accumulate_lanes(uint32_t* lanes);
hipError_t launch_msm(const MsmLaunch& m, hipStream_t s);

}  // namespace msm
}  // namespace zk
