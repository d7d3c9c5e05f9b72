// Device kernels of the NTT library and their launch helpers (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "field.hpp"

namespace zk {

// Flags of one global pass.
enum PassFlags : uint32_t {
  kPassReverseIn = 1u,   // first pass: read input index (n - idx) mod n
  kPassPreTable = 2u,    // first pass: multiply input idx by pre_table[idx]
  kPassPostTable = 4u,   // last pass: multiply output k by post_table[k]
  kPassPostConst = 8u,   // last pass: multiply every output by post_const
  kPassPostPointwise = 16u,  // last pass: out_k = (pw_a[k] pw_b[k] - out_k) post_const
};

// Arguments of one global radix-R Stockham pass over n = 2^log_n elements.
// The pass reads columns j + r (n/R) for r < R, multiplies element r of
// column j by the inter-pass twiddle w_{Ns R}^(r (j mod Ns)), runs an R-point
// DFT, and writes output r of column j to (j / Ns) Ns R + (j mod Ns) + r Ns,
// where Ns = 2^log_ns is the product of the radices of the earlier passes.
//
// Inter-pass twiddles come either from tw_pass, a table [r][j mod Ns] read in
// the same order as the data, or (tw_pass null, tw_hi non-null) from two
// small tables: w_n^e = tw_hi[e >> log_lo] * tw_lo[e mod 2^log_lo] with
// e = (n / (Ns R)) r (j mod Ns), one extra multiplication per element.
struct PassArgs {
  const Fe* in;
  Fe* out;
  const Fe* tw_pass;     // [r * Ns + (j mod Ns)], null on the first pass
  const Fe* tw_r;        // w_R^k for k < R
  const Fe* tw_lo;       // w_n^k, k < 2^log_lo (two-level mode)
  const Fe* tw_hi;       // w_n^(k 2^log_lo)    (two-level mode)
  const Fe* pre_table;   // see kPassPreTable
  const Fe* post_table;  // see kPassPostTable
  const Fe* pw_a;        // see kPassPostPointwise
  const Fe* pw_b;
  Fe post_const;         // see kPassPostConst, kPassPostPointwise
  uint32_t log_n;
  uint32_t log_ns;
  uint32_t flags;
  uint32_t log_lo;
  // Grouped launch (grp_jobs > 0): one launch runs this pass for grp_jobs
  // transforms of one plan, 2^log_grp_tiles tiles each; workgroup b takes
  // tile b mod 2^log_grp_tiles of job b / 2^log_grp_tiles, reading
  // grp_in[job] and writing grp_out[job] in place of in and out.
  const Fe* const* grp_in;
  Fe* const* grp_out;
  uint32_t grp_jobs;
  uint32_t log_grp_tiles;
};

// Shapes the pass kernels are instantiated for: tiles of 2^10 or 2^11
// elements with 2^3 .. 2^9 points per column, tiles of 2^8 elements with
// 2^3 .. 2^7 points per column (two or four elements per thread only), or
// one tile holding a whole transform of up to 2^11 points.
inline bool pass_shape_supported(int log_r, int log_tile, int log_e = 2) {
  if (log_tile == 11) return (log_r >= 3 && log_r <= 9) || log_r == 11;
  if (log_tile == 10 && log_r >= 3 && log_r <= 9) return true;
  if (log_tile == 8 && log_r >= 3 && log_r <= 7 && log_e <= 2) return true;
  return log_tile == log_r && log_r >= 0 && log_r <= 10;
}

// Kernel field id of BLS12-381 Fr with products on the FP64 multiplier
// (field_f64.hpp); launch_pass takes it like a field id.
constexpr int kFieldBls12_381Fp64 = 101;

// out_i = a_i b_i 2^-256 mod p (variant 0, the integer FIPS product) or
// a_i b_i 2^-288 mod p (variant 1, the FP64 product), for i < n.
hipError_t launch_field_mul(int field, int variant, const Fe* a, const Fe* b, Fe* out, uint64_t n, hipStream_t s);

// Launch one pass; log_r + log_j = log_tile.  Returns hipSuccess or the
// launch error.
hipError_t launch_pass(int field, int log_r, int log_tile, int log_e, const PassArgs& a, hipStream_t s);

// Table generation: out[t] = scale * base^e(t) for t < count, with
// e(t) = t (kGenPowers) or e(t) = mult * (t / ns) * (t mod ns) (kGenPassTwiddle).
// base^e is assembled from four 256-entry level tables held in `levels`
// (levels[256 k + d] = base^(d 256^k)), so e must be below 2^32.
enum GenMode : uint32_t { kGenPowers = 0, kGenPassTwiddle = 1 };
struct GenArgs {
  Fe* out;
  const Fe* levels;
  Fe scale;
  uint64_t count;
  uint64_t ns;
  uint64_t mult;
  uint32_t mode;
};
hipError_t launch_gen(int field, const GenArgs& g, hipStream_t s);

// E_i = (A_i B_i - C_i) * zinv, written to out (may alias c).
hipError_t launch_quotient_pointwise(int field, const Fe* a, const Fe* b, const Fe* c, Fe* out, Fe zinv, uint64_t n,
                                     hipStream_t s);

// Count elements with limbs >= p (non-canonical) into *d_count (device u32).
hipError_t launch_validate(int field, const Fe* x, uint64_t n, uint32_t* d_count, hipStream_t s);

// bytes (a multiple of 16) from device memory to pinned host memory, by a
// kernel rather than a DMA engine.
hipError_t launch_copy_out(void* host_dst, const void* dev_src, uint64_t bytes, hipStream_t s);

}  // namespace zk
