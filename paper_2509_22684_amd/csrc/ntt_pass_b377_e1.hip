// Pass kernels for BLS12-377 Fr with radix-2 in-register butterflies.
#include "ntt_pass_impl.hpp"

namespace zk {
hipError_t launch_pass_b377_e1(int log_r, int log_tile, const PassArgs& a, hipStream_t s) {
  return detail::dispatch_shape<Bls12_377Fr, 1>(log_r, log_tile, a, s);
}
}  // namespace zk
