// Pass kernels for BN254 Fr with radix-4 in-register butterflies.
#include "ntt_pass_impl.hpp"

namespace zk {
hipError_t launch_pass_bn_e2(int log_r, int log_tile, const PassArgs& a, hipStream_t s) {
  return detail::dispatch_shape<Bn254Fr, 2>(log_r, log_tile, a, s);
}
}  // namespace zk
