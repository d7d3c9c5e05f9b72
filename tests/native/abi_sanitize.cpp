// Driver for the C ABI's host-side paths under AddressSanitizer and
// UndefinedBehaviorSanitizer: argument checks that return before any device
// call, schedule resolution and registration, table-size queries, the error
// message buffer, from several threads at once.  Needs no GPU.
#include <cstdio>
#include <cstring>
#include <thread>
#include <vector>

#include "zkntt.h"

static int bad = 0;
#define CHECK(c)                                                  \
  do {                                                            \
    if (!(c)) {                                                   \
      std::fprintf(stderr, "FAIL %s:%d %s\n", __FILE__, __LINE__, #c); \
      ++bad;                                                      \
    }                                                             \
  } while (0)

static void host_paths(int t) {
  for (int rep = 0; rep < 200; ++rep) {
    ntt_plan_opts in{}, out{};
    CHECK(ntt_plan_resolve_opts(1, 24, nullptr, &out) == ZK_OK);
    CHECK(out.log2_radix != 0 && out.log2_tile != 0);
    in.log2_tile = 12;
    CHECK(ntt_plan_resolve_opts(1, 20, &in, &out) == ZK_EUNSUPPORTED);
    CHECK(std::strlen(zk_last_error()) > 0);
    in = ntt_plan_opts{};
    in.flags = 2;
    CHECK(ntt_plan_resolve_opts(2, 20, &in, &out) == ZK_EUNSUPPORTED);  // FP64 products: BLS12-381 only
    CHECK(ntt_plan_table_bytes(1, 33, nullptr) == 0);
    CHECK(ntt_plan_table_bytes(3, (uint32_t)(10 + (t + rep) % 30), nullptr) > 0);
    ntt_plan_opts reg{};
    reg.log2_radix = 2;
    reg.log2_pass_radix = (uint32_t)(6 + (t + rep) % 4);
    CHECK(ntt_tuning_register(1, (uint32_t)(12 + t), &reg) == ZK_OK);
    CHECK(ntt_tuning_register(1, 40, &reg) == ZK_EUNSUPPORTED);
    // null and misaligned arguments are refused before any device call
    CHECK(ntt_forward(nullptr, nullptr, nullptr, nullptr, nullptr) == ZK_EINVAL);
    CHECK(ntt_forward_noalloc(nullptr, nullptr, nullptr, nullptr) == ZK_EINVAL);
    CHECK(quotient_poly(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == ZK_EINVAL);
    CHECK(zk_copy_to_host(nullptr, nullptr, 16, nullptr) == ZK_EINVAL);
    CHECK(zk_copy_to_host(reinterpret_cast<void*>(256), reinterpret_cast<void*>(512), 24, nullptr) == ZK_EINVAL);
    CHECK(ntt_batch_create_jobs(nullptr, nullptr, 0, 0) == ZK_EINVAL);
    CHECK(ntt_batch_status(nullptr) == ZK_EINVAL);
    CHECK(msm_bases_create(nullptr, nullptr, 0, 0, nullptr) == ZK_EINVAL);
    msm_bases* mb = nullptr;
    CHECK(msm_bases_create(&mb, nullptr, 16, 0, nullptr) == ZK_EINVAL && mb == nullptr);
    CHECK(msm_compute(nullptr, nullptr, nullptr, nullptr, nullptr) == ZK_EINVAL);
    CHECK(zk_field_mul(9, 0, nullptr, nullptr, nullptr, 1, nullptr) == ZK_EUNSUPPORTED);
    CHECK(zk_field_mul(1, 0, nullptr, nullptr, nullptr, 1, nullptr) == ZK_EINVAL);
    CHECK(ntt_workspace_bytes(nullptr) == 0 && quotient_workspace_bytes(nullptr) == 0);
  }
}

int main() {
  std::vector<std::thread> th;
  for (int t = 0; t < 4; ++t) th.emplace_back(host_paths, t);
  for (auto& x : th) x.join();
  ntt_tuning_clear();
  std::printf(bad ? "ABI sanitizer driver: %d failures\n" : "ABI sanitizer driver: ok\n", bad);
  return bad ? 1 : 0;
}
