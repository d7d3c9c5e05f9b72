// Pass kernels for BLS12-377 Fr with radix-8 in-register butterflies.
#include "ntt_pass_impl.hpp"

namespace zk {
hipError_t launch_pass_b377_e3(int log_r, int log_tile, const PassArgs& a, hipStream_t s) {
  return detail::dispatch_shape<Bls12_377Fr, 3>(log_r, log_tile, a, s);
}
}  // namespace zk
