// Pass kernels for BLS12-381 Fr with radix-4 in-register butterflies.
#include "ntt_pass_impl.hpp"

namespace zk {
hipError_t launch_pass_bls_e2(int log_r, int log_tile, const PassArgs& a, hipStream_t s) {
  return detail::dispatch_shape<Bls12_381Fr, 2>(log_r, log_tile, a, s);
}
}  // namespace zk
