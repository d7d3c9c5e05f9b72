// Pass kernels for BLS12-381 Fr with radix-4 in-register butterflies and
// every product on the FP64 multiplier (field_f64.hpp).
#include "field_f64.hpp"
#include "ntt_pass_impl.hpp"

namespace zk {
hipError_t launch_pass_bls_f64_e2(int log_r, int log_tile, const PassArgs& a, hipStream_t s) {
  return detail::dispatch_shape<Bls12_381FrF64, 2>(log_r, log_tile, a, s);
}
}  // namespace zk
