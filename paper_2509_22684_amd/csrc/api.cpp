// C ABI of the NTT library: plans, transforms and the quotient chain.
//
// A plan fixes the field and n = 2^log2n, derives the primitive root of unity
// w_n = g^((p-1)/n) (g the smallest generator), and builds in device memory:
//   * the inter-pass twiddle table of every pass but the first, laid out
//     [r][j mod Ns] so that it streams coalesced beside the data it scales;
//   * a w_R table for each radix R used by a pass (in-tile twiddles);
//   * the coset tables g^k, n^-1 g^-k and n^-1 g^k (k < n) used to fuse the
//     coset shifts and the 1/n scaling into the first or last pass.
// Tables are generated on the device from four 256-entry level tables of the
// base computed on the host, so plan creation costs milliseconds even at
// n = 2^24.
//
// Transforms are sequences of Stockham passes (ntt_pass_impl.hpp, one
// translation unit per field and register radix); the inverse runs the
// forward passes on the index-reversed input, since
// sum_i X_i w^(-ij) = sum_i X_(-i mod n) w^(ij), and scales by 1/n on the
// last pass.  Batches (ntt_batch.hip) reuse the plans' tables and pass
// arguments.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/zkntt.h"
#include "field.hpp"
#include "msm.hpp"
#include "ntt_batch.hpp"
#include "ntt_kernels.hpp"

using zk::Fe;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? ZK_ENOMEM : ZK_EDEVICE;
}

// kInverseRaw and kForwardShifted split the quotient's INTT-then-coset-NTT
// differently: the inverse without its 1/n scaling, then the forward NTT
// with g^k / n applied as it loads its input.
enum Kind { kForward, kInverse, kCosetForward, kCosetInverse, kInverseToCoset, kInverseRaw, kForwardShifted };

struct PassDesc {
  int log_r;
  int log_tile;
  uint32_t log_ns;
  Fe* tw_pass;  // null on the first pass
  Fe* tw_r;
};

}  // namespace

struct ntt_plan {
  int field = 0;
  uint32_t log_n = 0;
  uint64_t n = 0;
  int log_e = 2;
  uint32_t flags = 0;
  int device = 0;
  std::vector<PassDesc> passes;
  std::vector<void*> owned;  // device allocations
  size_t device_bytes = 0;
  Fe n_inv{};        // 1/n, Montgomery
  Fe n_inv_op{};     // 1/n as the second operand of the plan's multiplier
  Fe zinv{};         // 1/(g^n - 1), Montgomery
  int kfield = 0;    // field id the pass kernels are launched for
  bool fp64 = false; // products on the FP64 multiplier (tables held as y 2^288)
  uint32_t twiddle_mode = 1;      // 1 table per pass, 2 two-level
  uint32_t max_log_r = 8;         // stages per global pass
  uint32_t log_tile = 10;         // elements per workgroup tile of a multi-pass transform, log2
  Fe* tw_lo = nullptr;            // two-level mode: w_n^k, k < 2^log_lo
  Fe* tw_hi = nullptr;            //                 w_n^(k 2^log_lo)
  uint32_t log_lo = 0;
  Fe* coset_fwd = nullptr;        // g^k
  Fe* coset_inv = nullptr;        // n^-1 g^-k
  Fe* inv_to_coset = nullptr;     // n^-1 g^k
  uint32_t* d_count = nullptr;    // validation counter
  std::mutex validate_mu;
  // quotient_poly up to 2^kQuotientForkMaxLog: A's and B's chains run on two
  // side streams forked from the caller's stream and joined back
  hipStream_t qside[2] = {nullptr, nullptr};
  hipEvent_t qfork = nullptr;
  hipEvent_t qjoin[2] = {nullptr, nullptr};
  std::mutex quotient_mu;  // one fork/join sequence at a time per plan
  ntt_plan_opts opts{};    // the resolved schedule
};

namespace {

template <class F>
struct Host {
  // levels[256 k + d] = base^(d 256^k), k < 4, d < 256
  static std::vector<Fe> levels(const Fe& base) {
    std::vector<Fe> lv(1024);
    Fe step = base;
    for (int k = 0; k < 4; ++k) {
      Fe x = zk::mont_one<F>();
      for (int d = 0; d < 256; ++d) {
        lv[256 * k + d] = x;
        x = zk::mul_portable<F>(x, step);
      }
      step = x;  // step^256
    }
    return lv;
  }
};

struct TableBuilder {
  ntt_plan* p;
  hipStream_t s = nullptr;
  std::vector<void*> scratch;

  int alloc(Fe** out, uint64_t count) {
    void* d = nullptr;
    hipError_t e = hipMalloc(&d, count * sizeof(Fe));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(plan table)");
    p->owned.push_back(d);
    p->device_bytes += count * sizeof(Fe);
    *out = static_cast<Fe*>(d);
    return ZK_OK;
  }

  template <class F>
  int generate(Fe* out, uint64_t count, const Fe& base, const Fe& scale, uint32_t mode, uint64_t ns,
               uint64_t mult) {
    std::vector<Fe> lv = Host<F>::levels(base);
    void* d_lv = nullptr;
    hipError_t e = hipMalloc(&d_lv, lv.size() * sizeof(Fe));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(level table)");
    scratch.push_back(d_lv);
    e = hipMemcpy(d_lv, lv.data(), lv.size() * sizeof(Fe), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(level table)");
    zk::GenArgs g{};
    g.out = out;
    g.levels = static_cast<const Fe*>(d_lv);
    g.scale = scale;
    g.count = count;
    g.ns = ns ? ns : 1;
    g.mult = mult;
    g.mode = mode;
    e = zk::launch_gen(F::ID, g, s);
    if (e != hipSuccess) return hip_fail(e, "table generation launch");
    return ZK_OK;
  }

  ~TableBuilder() {
    if (!scratch.empty()) {
      (void)hipDeviceSynchronize();
      for (void* d : scratch) (void)hipFree(d);
    }
  }
};

void free_plan(ntt_plan* p) {
  if (!p) return;
  for (int i = 0; i < 2; ++i) {
    if (p->qside[i]) (void)hipStreamDestroy(p->qside[i]);
    if (p->qjoin[i]) (void)hipEventDestroy(p->qjoin[i]);
  }
  if (p->qfork) (void)hipEventDestroy(p->qfork);
  for (void* d : p->owned) (void)hipFree(d);
  delete p;
}

// Plans whose quotient chain runs A's and B's transforms on side streams.
constexpr uint32_t kQuotientForkMaxLog = 22;
bool quotient_forks(const ntt_plan* p) { return p->log_n <= kQuotientForkMaxLog; }

// Split log_n into passes of at most max_log_r stages each, larger radices
// first (a single pass covers n up to the tile size in one tile).
std::vector<int> split_passes(uint32_t log_n, uint32_t max_log_r, uint32_t log_tile) {
  std::vector<int> r;
  if (log_n <= log_tile) {
    r.push_back((int)log_n);
    return r;
  }
  // a column of a multi-pass tile holds fewer points than the tile
  max_log_r = std::min(max_log_r, log_tile - 1);
  const int P = (int)((log_n + max_log_r - 1) / max_log_r);
  const int base = (int)log_n / P, extra = (int)log_n % P;
  for (int k = 0; k < P; ++k) r.push_back(base + (k < extra ? 1 : 0));
  return r;
}

template <class F>
int build_plan(ntt_plan* p) {
  TableBuilder tb{p};
  const uint32_t L = p->log_n;
  const Fe w_n = zk::root_of_unity<F>((int)L);
  const Fe one = zk::mont_one<F>();
  const Fe g = zk::to_mont<F>(zk::fe_from_u32<F>(F::GENERATOR));
  const Fe g_inv = zk::inv_mont<F>(g);
  p->n_inv = zk::inv_mont<F>(zk::pow_mont_u64<F>(zk::add<F>(one, one), L));
  // Second operands of the pass kernels' products (every table entry, 1/n):
  // y 2^256 mod p for the integer multiplier, y 2^288 mod p for the FP64 one
  // (R = 2^288 there), i.e. scaled by 2^32 in the Montgomery form.
  Fe opscale = one;
  if (p->fp64) {
    Fe two32 = zk::fe_zero();
    two32.v[1] = 1;
    opscale = zk::to_mont<F>(two32);
  }
  p->n_inv_op = zk::mul_portable<F>(p->n_inv, opscale);
  {
    Fe gn = g;
    for (uint32_t i = 0; i < L; ++i) gn = zk::mul_portable<F>(gn, gn);  // g^n
    p->zinv = zk::inv_mont<F>(zk::sub<F>(gn, one));
  }

  std::vector<int> radices = split_passes(L, p->max_log_r, p->log_tile);
  uint32_t log_ns = 0;
  Fe* tw_r_by_log[33] = {nullptr};
  for (size_t k = 0; k < radices.size(); ++k) {
    PassDesc d{};
    d.log_r = radices[k];
    d.log_tile = (L <= p->log_tile) ? (int)L : (int)p->log_tile;
    d.log_ns = log_ns;
    if (!zk::pass_shape_supported(d.log_r, d.log_tile, p->log_e))
      return fail(ZK_EUNSUPPORTED, "no pass kernel for a radix-2^" + std::to_string(d.log_r) +
                                       " pass; choose a larger log2_pass_radix");
    if (!tw_r_by_log[d.log_r]) {
      const uint64_t R = 1ull << d.log_r;
      Fe* t = nullptr;
      if (int rc = tb.alloc(&t, R)) return rc;
      Fe w_r = w_n;  // w_R = w_n^(n/R)
      for (uint32_t i = 0; i < L - (uint32_t)d.log_r; ++i) w_r = zk::mul_portable<F>(w_r, w_r);
      if (int rc = tb.generate<F>(t, R, w_r, opscale, zk::kGenPowers, 1, 0)) return rc;
      tw_r_by_log[d.log_r] = t;
    }
    d.tw_r = tw_r_by_log[d.log_r];
    if (k > 0 && p->twiddle_mode == 1) {
      const uint64_t ns = 1ull << log_ns, R = 1ull << d.log_r;
      const uint64_t count = ns * R;
      if (int rc = tb.alloc(&d.tw_pass, count)) return rc;
      // entry r * Ns + j' = w_n^((n / (Ns R)) r j')
      if (int rc = tb.generate<F>(d.tw_pass, count, w_n, opscale, zk::kGenPassTwiddle, ns, p->n >> (log_ns + d.log_r)))
        return rc;
    }
    p->passes.push_back(d);
    log_ns += (uint32_t)d.log_r;
  }

  if (radices.size() > 1 && p->twiddle_mode == 2) {
    // two-level inter-pass twiddles: w_n^e = hi[e >> log_lo] * lo[e mod 2^log_lo]
    p->log_lo = (L + 1) / 2;
    const uint64_t nlo = 1ull << p->log_lo, nhi = 1ull << (L - p->log_lo);
    if (int rc = tb.alloc(&p->tw_lo, nlo)) return rc;
    if (int rc = tb.generate<F>(p->tw_lo, nlo, w_n, opscale, zk::kGenPowers, 1, 0)) return rc;
    Fe w_step = w_n;
    for (uint32_t i = 0; i < p->log_lo; ++i) w_step = zk::mul_portable<F>(w_step, w_step);
    if (int rc = tb.alloc(&p->tw_hi, nhi)) return rc;
    if (int rc = tb.generate<F>(p->tw_hi, nhi, w_step, opscale, zk::kGenPowers, 1, 0)) return rc;
  }

  // Coset tables.
  if (int rc = tb.alloc(&p->coset_fwd, p->n)) return rc;
  if (int rc = tb.generate<F>(p->coset_fwd, p->n, g, opscale, zk::kGenPowers, 1, 0)) return rc;
  if (int rc = tb.alloc(&p->coset_inv, p->n)) return rc;
  if (int rc = tb.generate<F>(p->coset_inv, p->n, g_inv, p->n_inv_op, zk::kGenPowers, 1, 0)) return rc;
  if (int rc = tb.alloc(&p->inv_to_coset, p->n)) return rc;
  if (int rc = tb.generate<F>(p->inv_to_coset, p->n, g, p->n_inv_op, zk::kGenPowers, 1, 0)) return rc;

  {
    void* d = nullptr;
    hipError_t e = hipMalloc(&d, 256);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(counter)");
    p->owned.push_back(d);
    p->d_count = static_cast<uint32_t*>(d);
  }
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "plan table generation");
  return ZK_OK;
}

// Tuned schedules registered by the caller (the autotuner's database):
// ntt_plan_create fills every zero option from here before falling back to
// the built-in defaults.
struct TuningRegistry {
  std::mutex mu;
  std::map<std::pair<int, uint32_t>, ntt_plan_opts> opts;
};
TuningRegistry& tuning_registry() {
  static TuningRegistry* r = new TuningRegistry();  // never destroyed: plans may be created at exit
  return *r;
}

int field_adicity(int field) {
  if (field == ZK_FIELD_BLS12_381_FR) return zk::Bls12_381Fr::TWO_ADICITY;
  if (field == ZK_FIELD_BN254_FR) return zk::Bn254Fr::TWO_ADICITY;
  if (field == ZK_FIELD_BLS12_377_FR) return zk::Bls12_377Fr::TWO_ADICITY;
  return 0;
}

int check_opts(const ntt_plan_opts& o) {
  if (o.twiddle_mode > 2) return fail(ZK_EUNSUPPORTED, "twiddle_mode must be 0, 1 or 2");
  if (o.log2_pass_radix && (o.log2_pass_radix < 4 || o.log2_pass_radix > 9))
    return fail(ZK_EUNSUPPORTED, "log2_pass_radix must be 0 or 4..9");
  if (o.log2_radix > 3) return fail(ZK_EUNSUPPORTED, "log2_radix must be 0, 1, 2 or 3");
  if (!(o.log2_tile == 0 || o.log2_tile == 8 || o.log2_tile == 10 || o.log2_tile == 11))
    return fail(ZK_EUNSUPPORTED, "log2_tile must be 0, 8, 10 or 11");
  if (o.flags & ~(ZK_FLAG_VALIDATE | ZK_FLAG_FFMUL_FP64)) return fail(ZK_EUNSUPPORTED, "unknown flag bits");
  return ZK_OK;
}

// The schedule a plan for (field, log2n) runs: every zero field of `in`
// from the registered tuned schedule, then from the built-in defaults.
int resolve_opts(int field, uint32_t log2n, const ntt_plan_opts* in, ntt_plan_opts* out) {
  const int adicity = field_adicity(field);
  if (!adicity) return fail(ZK_EUNSUPPORTED, "unknown field id " + std::to_string(field));
  if (log2n > (uint32_t)adicity)
    return fail(ZK_EUNSUPPORTED, "log2n " + std::to_string(log2n) + " exceeds the field's 2-adicity " +
                                     std::to_string(adicity));
  ntt_plan_opts o{};
  if (in) o = *in;
  if (int rc = check_opts(o)) return rc;
  if (o.flags & ZK_FLAG_FFMUL_FP64) {
    // the FP64 multiplier is built for BLS12-381 Fr with radix-4 rounds
    if (field != ZK_FIELD_BLS12_381_FR)
      return fail(ZK_EUNSUPPORTED, "ZK_FLAG_FFMUL_FP64 is available for BLS12-381 Fr only");
    if (o.log2_radix && o.log2_radix != 2)
      return fail(ZK_EUNSUPPORTED, "ZK_FLAG_FFMUL_FP64 runs radix-4 register rounds (log2_radix 0 or 2)");
    o.log2_radix = 2;
  }
  {
    TuningRegistry& reg = tuning_registry();
    std::lock_guard<std::mutex> lock(reg.mu);
    auto it = reg.opts.find({field, log2n});
    if (it != reg.opts.end()) {
      const ntt_plan_opts& t = it->second;
      if (!o.twiddle_mode) o.twiddle_mode = t.twiddle_mode;
      if (!o.log2_radix) o.log2_radix = t.log2_radix;
      if (!o.log2_tile) o.log2_tile = t.log2_tile;
      if (!o.log2_pass_radix) o.log2_pass_radix = t.log2_pass_radix;
    }
  }
  // Built-in defaults.  Register radix: radix-2 rounds (two elements per
  // thread, twice the threads per tile) up to 2^18, where a transform has
  // too few tiles to fill the chip and more waves per tile shorten each
  // pass; radix-4 above, where every CU is busy and fewer instructions per
  // element win.  Pass depth: up to 2^18 two passes of at most 2^9 points (a
  // third pass would cost another launch or, in a batch, another round of
  // tiles and dependency waits); above, passes of at most 2^8 points, which
  // measured fastest at 2^24.
  // Tile: 2^8 elements for radix-2 transforms of 2^10 to 2^16 points (they
  // do not fill the chip; smaller tiles spread a pass over four times the
  // workgroups: 2^12 in 24 us against 33 us with 2^10-element tiles), 2^10
  // otherwise (the pass split under 2^8 tiles, passes of at most 2^7 points,
  // would add a pass to batched jobs).
  if (!o.twiddle_mode) o.twiddle_mode = 1;
  if (!o.log2_radix) o.log2_radix = log2n <= 18 ? 1 : 2;
  if (!o.log2_tile) o.log2_tile = (log2n >= 10 && log2n <= 16 && o.log2_radix == 1) ? 8 : 10;
  if (!o.log2_pass_radix) o.log2_pass_radix = log2n <= 18 ? 9 : 8;
  if (o.log2_tile == 8 && o.log2_radix == 3 && log2n > 8)
    return fail(ZK_EUNSUPPORTED, "2^8-element tiles take two or four elements per thread (log2_radix 1 or 2)");
  *out = o;
  return ZK_OK;
}

bool aligned(const void* ptr) { return (reinterpret_cast<uintptr_t>(ptr) & 255u) == 0; }

// [a, a + na) and [b, b + nb) share a byte.
bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return na && nb && x < y + nb && y < x + na;
}

int check_device(const ntt_plan* p) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != p->device) return fail(ZK_EINVAL, "the current HIP device is not the plan's device");
  return ZK_OK;
}

int validate_input(ntt_plan* p, const void* x, hipStream_t s) {
  // The check reads its count back to the host and waits for the stream,
  // which a stream being captured into a graph cannot do.
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t ce = hipStreamIsCapturing(s, &cs);
  if (ce != hipSuccess) return hip_fail(ce, "hipStreamIsCapturing");
  if (cs != hipStreamCaptureStatusNone)
    return fail(ZK_EINVAL, "ZK_FLAG_VALIDATE needs a host synchronisation and cannot run under stream capture");
  std::lock_guard<std::mutex> lock(p->validate_mu);
  hipError_t e = hipMemsetAsync(p->d_count, 0, sizeof(uint32_t), s);
  if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync(counter)");
  e = zk::launch_validate(p->field, static_cast<const Fe*>(x), p->n, p->d_count, s);
  if (e != hipSuccess) return hip_fail(e, "validate launch");
  uint32_t bad = 0;
  e = hipMemcpyAsync(&bad, p->d_count, sizeof bad, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "validate readback");
  if (bad) return fail(ZK_EINVAL, std::to_string(bad) + " input elements are not canonical (>= p)");
  return ZK_OK;
}

// Arguments of pass k of a transform of `kind`: pass 0 reads `in`, the last
// pass writes `out`, and the passes in between alternate between the
// workspace and `out` (pass k writes work when k is even).  With an odd
// number of passes the last one reads and writes `out` in place, which is
// safe because the last pass writes exactly the elements each tile reads.
zk::PassArgs make_pass_args(const ntt_plan* p, Kind kind, size_t k, const void* in, void* out, void* work) {
  const size_t P = p->passes.size();
  const PassDesc& d = p->passes[k];
  zk::PassArgs a{};
  a.in = static_cast<const Fe*>(k == 0 ? in : (k % 2 == 1 ? work : out));
  a.out = static_cast<Fe*>(k + 1 == P ? out : (k % 2 == 0 ? work : out));
  a.tw_pass = d.tw_pass;
  a.tw_r = d.tw_r;
  if (k > 0 && !d.tw_pass) {
    a.tw_lo = p->tw_lo;
    a.tw_hi = p->tw_hi;
    a.log_lo = p->log_lo;
  }
  a.log_n = p->log_n;
  a.log_ns = d.log_ns;
  a.flags = 0;
  if (k == 0) {
    if (kind == kInverse || kind == kCosetInverse || kind == kInverseToCoset || kind == kInverseRaw)
      a.flags |= zk::kPassReverseIn;
    if (kind == kCosetForward) {
      a.flags |= zk::kPassPreTable;
      a.pre_table = p->coset_fwd;
    } else if (kind == kForwardShifted) {
      a.flags |= zk::kPassPreTable;
      a.pre_table = p->inv_to_coset;
    }
  }
  if (k + 1 == P) {
    if (kind == kInverse) {
      a.flags |= zk::kPassPostConst;
      a.post_const = p->n_inv_op;
    } else if (kind == kCosetInverse) {
      a.flags |= zk::kPassPostTable;
      a.post_table = p->coset_inv;
    } else if (kind == kInverseToCoset) {
      a.flags |= zk::kPassPostTable;
      a.post_table = p->inv_to_coset;
    }
  }
  return a;
}

// events: optional array of P + 1 events recorded before each pass and
// after the last one on stream s.
int run_transform(const ntt_plan* p, Kind kind, const void* in, void* out, void* work, hipStream_t s,
                  hipEvent_t* events = nullptr) {
  const size_t P = p->passes.size();
  for (size_t k = 0; k < P; ++k) {
    if (events) {
      hipError_t e = hipEventRecord(events[k], s);
      if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    }
    const PassDesc& d = p->passes[k];
    const zk::PassArgs a = make_pass_args(p, kind, k, in, out, work);
    hipError_t e = zk::launch_pass(p->kfield, d.log_r, d.log_tile, p->log_e, a, s);
    if (e != hipSuccess) return hip_fail(e, "NTT pass launch");
  }
  if (events) {
    hipError_t e = hipEventRecord(events[P], s);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  }
  return ZK_OK;
}

size_t workspace_elems(const ntt_plan* p) { return p->passes.size() >= 2 ? p->n : 0; }

// Forward NTT of `in` whose last pass also applies the quotient's pointwise
// step with the coset evaluations a and b: out = (a b - NTT(in)) / (g^n - 1).
int run_forward_pointwise(const ntt_plan* p, const void* in, void* out, void* work, const Fe* a, const Fe* b,
                          hipStream_t s) {
  const size_t P = p->passes.size();
  for (size_t k = 0; k < P; ++k) {
    const PassDesc& d = p->passes[k];
    zk::PassArgs args = make_pass_args(p, kForwardShifted, k, in, out, work);
    if (k + 1 == P) {
      args.flags |= zk::kPassPostPointwise;
      args.pw_a = a;
      args.pw_b = b;
      args.post_const = p->zinv;
    }
    hipError_t e = zk::launch_pass(p->field, d.log_r, d.log_tile, p->log_e, args, s);
    if (e != hipSuccess) return hip_fail(e, "NTT pass launch");
  }
  return ZK_OK;
}

int transform_entry(const ntt_plan* p, Kind kind, const void* in, void* out, void* work, void* stream) {
  if (!p) return fail(ZK_EINVAL, "null plan");
  if (!in || !out) return fail(ZK_EINVAL, "null vector pointer");
  if (!aligned(in) || !aligned(out)) return fail(ZK_EINVAL, "vector pointers must be 256-byte aligned");
  if (workspace_elems(p)) {
    if (!work) return fail(ZK_EINVAL, "this plan needs a workspace (ntt_workspace_bytes)");
    if (!aligned(work)) return fail(ZK_EINVAL, "workspace must be 256-byte aligned");
    const size_t vb = p->n * sizeof(Fe), wb = workspace_elems(p) * sizeof(Fe);
    if (overlaps(work, wb, in, vb) || overlaps(work, wb, out, vb))
      return fail(ZK_EINVAL, "workspace must not overlap the vectors");
  }
  if (in != out && overlaps(in, p->n * sizeof(Fe), out, p->n * sizeof(Fe)))
    return fail(ZK_EINVAL, "in and out must be the same buffer or not overlap");
  if (int rc = check_device(p)) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (p->flags & ZK_FLAG_VALIDATE) {
    if (int rc = validate_input(const_cast<ntt_plan*>(p), in, s)) return rc;
  }
  return run_transform(p, kind, in, out, work, s);
}

// Workspace of ntt_forward_noalloc: a file-scope device array, so that the
// call allocates nothing.  Each device holds its own copy at its own address;
// host code reaches it only through the address hipGetSymbolAddress returns
// for that device (the array's name in host code is not a device address).
constexpr uint64_t kNoAllocWorkElems = 1ull << 20;  // 32 MiB: ping-pong vector of n <= 2^20

}  // namespace

static __device__ __align__(256) Fe noalloc_scratch[kNoAllocWorkElems];

namespace {

struct ScratchAddrs {
  std::mutex mu;
  std::vector<void*> by_device;
};
ScratchAddrs& scratch_addrs() {
  static ScratchAddrs* s = new ScratchAddrs();  // never destroyed
  return *s;
}

// The scratch array's address on device `dev` (which must be current),
// looked up once per device.
int scratch_address(int dev, void** out) {
  ScratchAddrs& sa = scratch_addrs();
  std::lock_guard<std::mutex> lock(sa.mu);
  if ((size_t)dev >= sa.by_device.size()) sa.by_device.resize((size_t)dev + 1, nullptr);
  if (!sa.by_device[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(noalloc_scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e, "hipGetSymbolAddress(noalloc_scratch)");
    sa.by_device[dev] = ptr;
  }
  *out = sa.by_device[dev];
  return ZK_OK;
}

}  // namespace

extern "C" {

int ntt_plan_create(ntt_plan** out, int field, uint32_t log2n, const ntt_plan_opts* opts) {
  if (!out) return fail(ZK_EINVAL, "null output pointer");
  *out = nullptr;
  ntt_plan_opts o{};
  if (int rc = resolve_opts(field, log2n, opts, &o)) return rc;

  ntt_plan* p = new (std::nothrow) ntt_plan();
  if (!p) return fail(ZK_ENOMEM, "host allocation failed");
  p->field = field;
  p->log_n = log2n;
  p->n = 1ull << log2n;
  p->log_e = (int)o.log2_radix;
  p->flags = o.flags;
  p->twiddle_mode = o.twiddle_mode;
  p->max_log_r = o.log2_pass_radix;
  p->log_tile = o.log2_tile;
  p->opts = o;
  p->fp64 = (o.flags & ZK_FLAG_FFMUL_FP64) != 0;
  p->kfield = p->fp64 ? zk::kFieldBls12_381Fp64 : field;
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) {
    free_plan(p);
    return hip_fail(e, "hipGetDevice");
  }
  int rc = field == ZK_FIELD_BLS12_381_FR ? build_plan<zk::Bls12_381Fr>(p)
           : field == ZK_FIELD_BN254_FR    ? build_plan<zk::Bn254Fr>(p)
                                           : build_plan<zk::Bls12_377Fr>(p);
  if (rc) {
    free_plan(p);
    return rc;
  }
  if (quotient_forks(p)) {
    e = hipEventCreateWithFlags(&p->qfork, hipEventDisableTiming);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
      e = hipStreamCreateWithFlags(&p->qside[i], hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&p->qjoin[i], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
      free_plan(p);
      return hip_fail(e, "quotient side streams");
    }
  }
  *out = p;
  return ZK_OK;
}

void ntt_plan_destroy(ntt_plan* p) { free_plan(p); }

int ntt_tuning_register(int field, uint32_t log2n, const ntt_plan_opts* opts) {
  if (!opts) return fail(ZK_EINVAL, "null options");
  const int adicity = field_adicity(field);
  if (!adicity) return fail(ZK_EUNSUPPORTED, "unknown field id " + std::to_string(field));
  if (log2n > (uint32_t)adicity) return fail(ZK_EUNSUPPORTED, "log2n exceeds the field's 2-adicity");
  if (int rc = check_opts(*opts)) return rc;
  if (opts->flags) return fail(ZK_EINVAL, "a tuned schedule carries no flags");
  TuningRegistry& reg = tuning_registry();
  std::lock_guard<std::mutex> lock(reg.mu);
  reg.opts[{field, log2n}] = *opts;
  return ZK_OK;
}

void ntt_tuning_clear(void) {
  TuningRegistry& reg = tuning_registry();
  std::lock_guard<std::mutex> lock(reg.mu);
  reg.opts.clear();
}

int ntt_plan_resolve_opts(int field, uint32_t log2n, const ntt_plan_opts* opts, ntt_plan_opts* resolved) {
  if (!resolved) return fail(ZK_EINVAL, "null output pointer");
  return resolve_opts(field, log2n, opts, resolved);
}

size_t ntt_plan_table_bytes(int field, uint32_t log2n, const ntt_plan_opts* opts) {
  ntt_plan_opts o{};
  if (resolve_opts(field, log2n, opts, &o) != ZK_OK) return 0;
  // the allocations build_plan makes for this schedule
  const std::vector<int> radices = split_passes(log2n, o.log2_pass_radix, o.log2_tile);
  const int log_tile = log2n <= o.log2_tile ? (int)log2n : (int)o.log2_tile;
  uint64_t elems = 0;
  bool seen[33] = {false};
  uint32_t log_ns = 0;
  for (size_t k = 0; k < radices.size(); ++k) {
    if (!zk::pass_shape_supported(radices[k], log_tile, (int)o.log2_radix)) {
      fail(ZK_EUNSUPPORTED, "no pass kernel for a radix-2^" + std::to_string(radices[k]) + " pass");
      return 0;
    }
    if (!seen[radices[k]]) elems += 1ull << radices[k];
    seen[radices[k]] = true;
    if (k > 0 && o.twiddle_mode == 1) elems += (1ull << log_ns) << radices[k];
    log_ns += (uint32_t)radices[k];
  }
  if (radices.size() > 1 && o.twiddle_mode == 2) {
    const uint32_t log_lo = (log2n + 1) / 2;
    elems += (1ull << log_lo) + (1ull << (log2n - log_lo));
  }
  elems += 3ull << log2n;  // coset tables
  return elems * sizeof(Fe);
}

int ntt_plan_get_opts(const ntt_plan* p, ntt_plan_opts* out) {
  if (!p || !out) return fail(ZK_EINVAL, "null argument");
  *out = p->opts;
  return ZK_OK;
}

size_t ntt_workspace_bytes(const ntt_plan* p) { return p ? workspace_elems(p) * sizeof(Fe) : 0; }

size_t ntt_plan_device_bytes(const ntt_plan* p) { return p ? p->device_bytes : 0; }

int ntt_plan_passes(const ntt_plan* p) { return p ? (int)p->passes.size() : 0; }

int ntt_forward(const ntt_plan* p, const void* d_in, void* d_out, void* d_work, void* stream) {
  return transform_entry(p, kForward, d_in, d_out, d_work, stream);
}

int ntt_forward_noalloc(const ntt_plan* p, const void* d_in, void* d_out, void* stream) {
  if (!p) return fail(ZK_EINVAL, "null plan");
  if (workspace_elems(p) > kNoAllocWorkElems)
    return fail(ZK_EUNSUPPORTED, "ntt_forward_noalloc holds a workspace of at most 2^20 elements (n <= 2^20); "
                                 "this plan needs " + std::to_string(workspace_elems(p)));
  void* work = nullptr;
  if (workspace_elems(p)) {
    if (int rc = check_device(p)) return rc;
    if (int rc = scratch_address(p->device, &work)) return rc;
  }
  return transform_entry(p, kForward, d_in, d_out, work, stream);
}

int ntt_inverse(const ntt_plan* p, const void* d_in, void* d_out, void* d_work, void* stream) {
  return transform_entry(p, kInverse, d_in, d_out, d_work, stream);
}

int ntt_coset_forward(const ntt_plan* p, const void* d_in, void* d_out, void* d_work, void* stream) {
  return transform_entry(p, kCosetForward, d_in, d_out, d_work, stream);
}

int ntt_coset_inverse(const ntt_plan* p, const void* d_in, void* d_out, void* d_work, void* stream) {
  return transform_entry(p, kCosetInverse, d_in, d_out, d_work, stream);
}

size_t quotient_workspace_bytes(const ntt_plan* p) {
  return p ? (2 * p->n + (quotient_forks(p) ? 3 : 1) * workspace_elems(p)) * sizeof(Fe) : 0;
}

int quotient_poly(const ntt_plan* p, const void* d_A, const void* d_B, const void* d_C, void* d_H, void* d_work,
                  void* stream) {
  if (!p) return fail(ZK_EINVAL, "null plan");
  if (p->fp64) return fail(ZK_EUNSUPPORTED, "the quotient chain runs on the integer multiplier only");
  if (!d_A || !d_B || !d_C || !d_H || !d_work) return fail(ZK_EINVAL, "null pointer");
  if (!aligned(d_A) || !aligned(d_B) || !aligned(d_C) || !aligned(d_H) || !aligned(d_work))
    return fail(ZK_EINVAL, "pointers must be 256-byte aligned");
  {
    const size_t vb = p->n * sizeof(Fe), wb = quotient_workspace_bytes(p);
    for (const void* x : {d_A, d_B, d_C, static_cast<const void*>(d_work)})
      if (overlaps(d_H, vb, x, x == d_work ? wb : vb))
        return fail(ZK_EINVAL, "H must not overlap A, B, C or the workspace");
    for (const void* x : {d_A, d_B, d_C})
      if (overlaps(d_work, wb, x, vb)) return fail(ZK_EINVAL, "the workspace must not overlap A, B or C");
  }
  if (int rc = check_device(p)) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (p->flags & ZK_FLAG_VALIDATE) {
    for (const void* x : {d_A, d_B, d_C})
      if (int rc = validate_input(const_cast<ntt_plan*>(p), x, s)) return rc;
  }
  Fe* t1 = static_cast<Fe*>(d_work);
  Fe* t2 = t1 + p->n;
  const size_t ws = workspace_elems(p);
  Fe* w = ws ? t2 + p->n : nullptr;
  Fe* H = static_cast<Fe*>(d_H);
  if (quotient_forks(p)) {
    // Up to 2^kQuotientForkMaxLog one transform does not fill the chip: A's
    // and B's INTT->NTT chains run on two side streams beside C's INTT, each
    // with its own workspace, and C's forward NTT with the pointwise step
    // waits for both.  Same kernels and arguments, so the same bytes.
    std::lock_guard<std::mutex> lock(const_cast<ntt_plan*>(p)->quotient_mu);
    hipError_t e = hipEventRecord(p->qfork, s);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipStreamWaitEvent(p->qside[i], p->qfork, 0);
    if (e != hipSuccess) return hip_fail(e, "quotient fork");
    const void* src[2] = {d_A, d_B};
    Fe* dst[2] = {t1, t2};
    int rc = ZK_OK;
    for (int i = 0; i < 2 && rc == ZK_OK; ++i) {
      Fe* wi = ws ? w + (size_t)(i + 1) * ws : nullptr;
      rc = run_transform(p, kInverseRaw, src[i], dst[i], wi, p->qside[i]);
      if (rc == ZK_OK) rc = run_transform(p, kForwardShifted, dst[i], dst[i], wi, p->qside[i]);
    }
    if (rc == ZK_OK) rc = run_transform(p, kInverseRaw, d_C, H, w, s);
    // join both side streams into s in every case, so that whatever was
    // queued on them is ordered before later work on s, also after an error
    for (int i = 0; i < 2; ++i) {
      e = hipEventRecord(p->qjoin[i], p->qside[i]);
      if (e == hipSuccess) e = hipStreamWaitEvent(s, p->qjoin[i], 0);
      if (e != hipSuccess && rc == ZK_OK) rc = hip_fail(e, "quotient join");
    }
    if (rc != ZK_OK) return rc;
    if (int rc = run_forward_pointwise(p, H, H, w, t1, t2, s)) return rc;
    return run_transform(p, kCosetInverse, H, H, w, s);
  }
  // Each of A, B, C: INTT without its 1/n, then a forward NTT that multiplies
  // coefficient k by g^k / n as its first pass loads it: evaluations on
  // g<w>.  (Scaling in the forward's first pass rather than the inverse's
  // last pass puts the product where the pass has no inter-pass twiddle.)
  // The last pass of C's forward NTT also applies the pointwise step
  // (A B - C) / (g^n - 1), so H holds the quotient's coset values without a
  // separate pass over memory.
  const void* src[3] = {d_A, d_B, d_C};
  Fe* dst[3] = {t1, t2, H};
  for (int v = 0; v < 3; ++v) {
    if (int rc = run_transform(p, kInverseRaw, src[v], dst[v], w, s)) return rc;
    if (v < 2) {
      if (int rc = run_transform(p, kForwardShifted, dst[v], dst[v], w, s)) return rc;
    } else if (int rc = run_forward_pointwise(p, H, H, w, t1, t2, s)) {
      return rc;
    }
  }
  return run_transform(p, kCosetInverse, H, H, w, s);
}

int quotient_coset_evals(const ntt_plan* p, const void* d_in, void* d_out, void* d_work, void* stream) {
  if (p && p->fp64) return fail(ZK_EUNSUPPORTED, "the quotient chain runs on the integer multiplier only");
  if (int rc = transform_entry(p, kInverseRaw, d_in, d_out, d_work, stream)) return rc;
  return run_transform(p, kForwardShifted, d_out, d_out, d_work, static_cast<hipStream_t>(stream));
}

int quotient_pointwise(const ntt_plan* p, const void* d_A, const void* d_B, const void* d_C, void* d_out,
                       void* stream) {
  if (!p) return fail(ZK_EINVAL, "null plan");
  if (p->fp64) return fail(ZK_EUNSUPPORTED, "the quotient chain runs on the integer multiplier only");
  if (!d_A || !d_B || !d_C || !d_out) return fail(ZK_EINVAL, "null pointer");
  if (!aligned(d_A) || !aligned(d_B) || !aligned(d_C) || !aligned(d_out))
    return fail(ZK_EINVAL, "pointers must be 256-byte aligned");
  if (int rc = check_device(p)) return rc;
  hipError_t e = zk::launch_quotient_pointwise(p->field, static_cast<const Fe*>(d_A), static_cast<const Fe*>(d_B),
                                               static_cast<const Fe*>(d_C), static_cast<Fe*>(d_out), p->zinv, p->n,
                                               static_cast<hipStream_t>(stream));
  return e == hipSuccess ? ZK_OK : hip_fail(e, "pointwise launch");
}

int zk_copy_to_host(void* host_dst, const void* dev_src, size_t bytes, void* stream) {
  if (!host_dst || !dev_src) return fail(ZK_EINVAL, "null pointer");
  if (bytes % 16 || reinterpret_cast<uintptr_t>(host_dst) % 16 || reinterpret_cast<uintptr_t>(dev_src) % 16)
    return fail(ZK_EINVAL, "bytes and both pointers must be multiples of 16");
  hipPointerAttribute_t ha{}, da{};
  hipError_t e = hipPointerGetAttributes(&ha, host_dst);
  if (e != hipSuccess || ha.type != hipMemoryTypeHost) {
    (void)hipGetLastError();
    return fail(ZK_EINVAL, "destination must be pinned host memory (hipHostMalloc)");
  }
  void* mapped = nullptr;  // the destination's address as the device sees it
  e = hipHostGetDevicePointer(&mapped, host_dst, 0);
  if (e != hipSuccess || !mapped) {
    (void)hipGetLastError();
    return fail(ZK_EINVAL, "destination is not mapped for the device");
  }
  e = hipPointerGetAttributes(&da, dev_src);
  if (e != hipSuccess || da.type != hipMemoryTypeDevice) {
    (void)hipGetLastError();
    return fail(ZK_EINVAL, "source must be device memory");
  }
  e = zk::launch_copy_out(mapped, dev_src, bytes, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? ZK_OK : hip_fail(e, "copy-out launch");
}

int ntt_profile_passes(const ntt_plan* p, int kind, const void* d_in, void* d_out, void* d_work, void* stream,
                       float* ms_per_pass, int max_passes) {
  if (!p || !ms_per_pass) return fail(ZK_EINVAL, "null argument");
  if (kind < 0 || kind > 3) return fail(ZK_EINVAL, "kind must be 0..3");
  const int P = (int)p->passes.size();
  if (max_passes < P) return fail(ZK_EINVAL, "ms_per_pass holds fewer entries than the plan has passes");
  if (!d_in || !d_out) return fail(ZK_EINVAL, "null vector pointer");
  if (!aligned(d_in) || !aligned(d_out)) return fail(ZK_EINVAL, "vector pointers must be 256-byte aligned");
  if (workspace_elems(p) && (!d_work || !aligned(d_work) || d_work == d_in || d_work == d_out))
    return fail(ZK_EINVAL, "this plan needs a distinct, aligned workspace");
  if (int rc = check_device(p)) return rc;
  std::vector<hipEvent_t> ev(P + 1, nullptr);
  int rc = ZK_OK;
  for (auto& e : ev) {
    hipError_t h = hipEventCreate(&e);
    if (h != hipSuccess) {
      rc = hip_fail(h, "hipEventCreate");
      break;
    }
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!rc) rc = run_transform(p, static_cast<Kind>(kind), d_in, d_out, d_work, s, ev.data());
  if (!rc) {
    hipError_t h = hipEventSynchronize(ev[P]);
    for (int k = 0; k < P && h == hipSuccess; ++k) h = hipEventElapsedTime(&ms_per_pass[k], ev[k], ev[k + 1]);
    if (h != hipSuccess) rc = hip_fail(h, "pass timing");
  }
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  return rc ? rc : P;
}

int zk_field_mul(int field, int variant, const void* d_a, const void* d_b, void* d_out, uint64_t n, void* stream) {
  if (!field_adicity(field)) return fail(ZK_EUNSUPPORTED, "unknown field id " + std::to_string(field));
  if (variant < 0 || variant > 2)
    return fail(ZK_EUNSUPPORTED, "variant must be 0 (integer), 1 (FP64) or 2 (integer, lazy)");
  if (n && (!d_a || !d_b || !d_out)) return fail(ZK_EINVAL, "null pointer");
  if ((n && (!aligned(d_a) || !aligned(d_b) || !aligned(d_out))))
    return fail(ZK_EINVAL, "pointers must be 256-byte aligned");
  hipError_t e = zk::launch_field_mul(field, variant, static_cast<const Fe*>(d_a), static_cast<const Fe*>(d_b),
                                      static_cast<Fe*>(d_out), n, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? ZK_OK : hip_fail(e, "field multiplication launch");
}

const char* zk_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches

// Work of a batch run as ordinary launches ahead of the persistent kernel
// (see batch_build): a pointwise job, or a group of transforms of one plan
// and kind, one grouped pass launch per pass.
struct DirectWork {
  const ntt_plan* plan;
  bool pointwise;
  const void* in;  // pointwise operands
  const void* in2;
  const void* in3;
  void* out;
  std::vector<zk::PassArgs> pass;  // grouped transforms
  std::vector<size_t> ptr_off;     // per pass: offset of its in pointers in the batch's pointer array
  size_t lane = 0;                 // side stream it runs on
};

struct ntt_batch {
  int device = 0;
  std::vector<DirectWork> direct;
  uint32_t njobs = 0;
  uint32_t nitems = 0;
  uint32_t nq_end[3] = {0, 0, 0};  // end of each field's queues: BLS12-381, BN254, BLS12-377
  uint32_t grid = 0;
  void* d_mem = nullptr;  // descriptor block from the pool
  size_t d_mem_bytes = 0;
  // Batches without a graph keep their descriptor image in the block's pinned
  // host twin and upload it on the stream of their first launch, so that
  // creating one never waits for the device; each of their launches also
  // copies the error word back to the twin (status_host) on the launch
  // stream.  The uploaded bytes; upload still to do; status in the twin.
  void* h_mem = nullptr;
  size_t upload_bytes = 0;
  mutable bool upload_pending = false;
  mutable bool status_on_host = false;
  uint32_t* status_host = nullptr;
  hipEvent_t done_ev = nullptr;  // recorded on the launch stream after every launch
  bool launched = false;
  zk::BatchJob* d_jobs = nullptr;
  zk::BatchItem* d_items = nullptr;
  zk::BatchQueue* d_queues = nullptr;
  uint32_t* d_ctl = nullptr;
  hipStream_t capture_stream = nullptr;
  // side streams for the direct work, forked from and joined back into the
  // launch stream (none when the launch stream alone has all the work)
  std::vector<hipStream_t> sides;
  std::vector<hipEvent_t> joins;
  hipEvent_t fork_ev = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

constexpr uint32_t kDefaultSpinLimit = 1u << 22;
// Queues per field by default: 16 measured fastest on the 64-job workload
// (0.81 ms against 0.84 ms with 32 and 0.88-0.90 ms with 4 or 8).
constexpr size_t kQueuesPerField = 16;

size_t batch_work_elems(const ntt_plan* const* plans, int njobs) {
  size_t total = 0;
  for (int k = 0; k < njobs; ++k)
    if (plans[k]) total += workspace_elems(plans[k]);
  return total;
}

// Side streams and their events are recycled between batches (creating
// them costs more host time than the rest of a small batch's set-up, and the
// serving loop builds a batch per tick).  A batch holds its own while it
// lives; free ones stay until the process ends.
struct SidePool {
  std::mutex mu;
  std::vector<std::pair<int, hipStream_t>> streams;  // (device, stream)
  std::vector<std::pair<int, hipEvent_t>> events;
};
SidePool& side_pool() {
  static SidePool* pool = new SidePool();  // never destroyed: outlives every batch
  return *pool;
}

hipError_t take_stream(int dev, hipStream_t* out) {
  SidePool& sp = side_pool();
  {
    std::lock_guard<std::mutex> lock(sp.mu);
    for (size_t i = 0; i < sp.streams.size(); ++i)
      if (sp.streams[i].first == dev) {
        *out = sp.streams[i].second;
        sp.streams.erase(sp.streams.begin() + (long)i);
        return hipSuccess;
      }
  }
  return hipStreamCreateWithFlags(out, hipStreamNonBlocking);
}

hipError_t take_event(int dev, hipEvent_t* out) {
  SidePool& sp = side_pool();
  {
    std::lock_guard<std::mutex> lock(sp.mu);
    for (size_t i = 0; i < sp.events.size(); ++i)
      if (sp.events[i].first == dev) {
        *out = sp.events[i].second;
        sp.events.erase(sp.events.begin() + (long)i);
        return hipSuccess;
      }
  }
  return hipEventCreateWithFlags(out, hipEventDisableTiming);
}

void give_back(int dev, const std::vector<hipStream_t>& streams, const std::vector<hipEvent_t>& events) {
  SidePool& sp = side_pool();
  std::lock_guard<std::mutex> lock(sp.mu);
  for (hipStream_t x : streams)
    if (x) sp.streams.emplace_back(dev, x);
  for (hipEvent_t x : events)
    if (x) sp.events.emplace_back(dev, x);
}

// A synchronous copy on a pooled non-blocking stream: ordered after nothing
// but itself, so it never waits for work the caller has queued elsewhere.
hipError_t copy_on_own_stream(int dev, void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
  if (bytes == 0) return hipSuccess;
  hipStream_t xs = nullptr;
  hipError_t e = take_stream(dev, &xs);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(dst, src, bytes, kind, xs);
  if (e == hipSuccess) e = hipStreamSynchronize(xs);
  give_back(dev, {xs}, {});
  return e;
}

// Device memory for batch descriptors is recycled the same way: hipFree
// waits for the whole device, so a serving loop that destroyed each tick's
// batch with it would stall every stream of the device once per tick.
// Blocks are powers of two from 64 KiB; a batch takes the smallest free
// block that fits (one block per batch) and returns it on destruction.
struct DescPool {
  std::mutex mu;
  struct Block {
    int dev;
    size_t bytes;
    void* ptr;
    hipEvent_t last_use;  // recorded after the last launch of the batch that held it, or null
    void* host;           // pinned host twin of the same size, made on first need, or null
  };
  std::vector<Block> free_blocks;
};
DescPool& desc_pool() {
  static DescPool* pool = new DescPool();  // never destroyed: outlives every batch
  return *pool;
}

size_t desc_block_bytes(size_t need) {
  size_t b = 64 << 10;
  while (b < need) b <<= 1;
  return b;
}

hipError_t take_desc(int dev, size_t need, void** out, size_t* got, void** host) {
  DescPool& dp = desc_pool();
  const size_t want = desc_block_bytes(need);
  {
    std::lock_guard<std::mutex> lock(dp.mu);
    size_t best = dp.free_blocks.size();
    for (size_t i = 0; i < dp.free_blocks.size(); ++i) {
      const DescPool::Block& bl = dp.free_blocks[i];
      if (bl.dev == dev && bl.bytes >= want && (best == dp.free_blocks.size() || bl.bytes < dp.free_blocks[best].bytes))
        best = i;
    }
    if (best < dp.free_blocks.size()) {
      const DescPool::Block bl = dp.free_blocks[best];
      dp.free_blocks.erase(dp.free_blocks.begin() + (long)best);
      *out = bl.ptr;
      *got = bl.bytes;
      *host = bl.host;
      hipError_t e = hipSuccess;
      if (bl.last_use) {
        // the batch that held the block may still run if it was destroyed
        // early; its descriptors are overwritten only once it is done
        e = hipEventSynchronize(bl.last_use);
        give_back(dev, {}, {bl.last_use});
      }
      return e;
    }
  }
  *got = want;
  *host = nullptr;
  return hipMalloc(out, want);
}

void give_desc(int dev, size_t bytes, void* ptr, hipEvent_t last_use, void* host) {
  if (!ptr) return;
  DescPool& dp = desc_pool();
  std::lock_guard<std::mutex> lock(dp.mu);
  dp.free_blocks.push_back(DescPool::Block{dev, bytes, ptr, last_use, host});
}

void free_batch(ntt_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
  std::vector<hipEvent_t> evs(b->joins);
  evs.push_back(b->fork_ev);
  give_back(b->device, b->sides, evs);
  give_desc(b->device, b->d_mem_bytes, b->d_mem, b->launched ? b->done_ev : nullptr, b->h_mem);
  if (!b->launched && b->done_ev) give_back(b->device, {}, {b->done_ev});
  delete b;
}

// Everything one launch of the batch does: the counter reset and the
// persistent kernel on s and the direct work on side streams, forked from s
// before and joined into s after, so that they all run at the same time
// (the persistent grid then leaves room for the pass kernels).
int batch_enqueue(const ntt_batch* b, hipStream_t s) {
  if (b->upload_pending) {
    // ordered before everything below on s, and through the fork on the
    // side streams
    hipError_t e = hipMemcpyAsync(b->d_mem, b->h_mem, b->upload_bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "batch descriptor upload");
    b->upload_pending = false;
  }
  if (!b->sides.empty()) {
    hipError_t e = hipEventRecord(b->fork_ev, s);
    for (hipStream_t x : b->sides)
      if (e == hipSuccess) e = hipStreamWaitEvent(x, b->fork_ev, 0);
    if (e != hipSuccess) return hip_fail(e, "batch fork");
  }
  int rc = ZK_OK;
  hipError_t e = zk::launch_batch(b->d_jobs, b->d_items, b->d_queues, b->nq_end, b->nitems, b->d_ctl, b->njobs,
                                  b->grid, s);
  if (e != hipSuccess) rc = hip_fail(e, "batch launch");
  for (size_t k = 0; k < b->direct.size() && rc == ZK_OK; ++k) {
    const DirectWork& d = b->direct[k];
    hipStream_t ds = b->sides.empty() ? s : b->sides[d.lane];
    if (d.pointwise) {
      e = zk::launch_quotient_pointwise(d.plan->field, static_cast<const Fe*>(d.in), static_cast<const Fe*>(d.in2),
                                        static_cast<const Fe*>(d.in3), static_cast<Fe*>(d.out), d.plan->zinv,
                                        d.plan->n, ds);
      if (e != hipSuccess) rc = hip_fail(e, "pointwise launch");
      continue;
    }
    for (size_t q = 0; q < d.pass.size() && rc == ZK_OK; ++q) {
      const PassDesc& pd = d.plan->passes[q];
      e = zk::launch_pass(d.plan->field, pd.log_r, pd.log_tile, 2, d.pass[q], ds);
      if (e != hipSuccess) rc = hip_fail(e, "grouped pass launch");
    }
  }
  // join every side stream into s, also after an error, so that whatever was
  // queued on them is ordered before later work on s
  for (size_t i = 0; i < b->sides.size(); ++i) {
    e = hipEventRecord(b->joins[i], b->sides[i]);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, b->joins[i], 0);
    if (e != hipSuccess && rc == ZK_OK) rc = hip_fail(e, "batch join");
  }
  return rc;
}

bool op_to_kind(int op, Kind* k) {
  switch (op) {
    case ZK_OP_FORWARD: *k = kForward; return true;
    case ZK_OP_INVERSE: *k = kInverse; return true;
    case ZK_OP_COSET_FORWARD: *k = kCosetForward; return true;
    case ZK_OP_COSET_INVERSE: *k = kCosetInverse; return true;
    case ZK_OP_INVERSE_TO_COSET: *k = kInverseToCoset; return true;
    default: return false;
  }
}

int batch_build(ntt_batch** out, const ntt_batch_job* specs, int njobs, bool capture,
                size_t queues_per_field = kQueuesPerField, bool all_direct = false) {
  if (!out) return fail(ZK_EINVAL, "null output pointer");
  *out = nullptr;
  if (njobs < 0 || (njobs > 0 && !specs)) return fail(ZK_EINVAL, "bad job array");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");

  std::vector<zk::BatchJob> jobs(njobs);
  std::vector<Kind> kinds(njobs, kForward);
  for (int k = 0; k < njobs; ++k) {
    const ntt_batch_job& sp = specs[k];
    const ntt_plan* p = sp.plan;
    if (!p) return fail(ZK_EINVAL, "null plan in batch job " + std::to_string(k));
    if (p->fp64) return fail(ZK_EUNSUPPORTED, "batches run on the integer multiplier only");
    if (p->device != dev) return fail(ZK_EINVAL, "batch plans must live on the current device");
    zk::BatchJob& J = jobs[k];
    std::memset(&J, 0, sizeof J);
    J.field = (uint32_t)p->field;
    if (sp.op == ZK_OP_QUOTIENT_POINTWISE) {
      if (!sp.in || !sp.in2 || !sp.in3 || !sp.out) return fail(ZK_EINVAL, "pointwise job needs in, in2, in3, out");
      if (!aligned(sp.in) || !aligned(sp.in2) || !aligned(sp.in3) || !aligned(sp.out))
        return fail(ZK_EINVAL, "batch buffers must be 256-byte aligned");
      J.kind = zk::kJobPointwise;
      J.npasses = 1;
      J.pw.a = static_cast<const Fe*>(sp.in);
      J.pw.b = static_cast<const Fe*>(sp.in2);
      J.pw.c = static_cast<const Fe*>(sp.in3);
      J.pw.out = static_cast<Fe*>(sp.out);
      J.pw.zinv = p->zinv;
      J.pw.n = p->n;
      J.pass[0].tiles = (uint32_t)((p->n + (1u << zk::kPointwiseTileLog) - 1) >> zk::kPointwiseTileLog);
      continue;
    }
    Kind kind;
    if (!op_to_kind(sp.op, &kind)) return fail(ZK_EINVAL, "unknown batch op " + std::to_string(sp.op));
    kinds[k] = kind;
    if (!sp.in || !sp.out || !aligned(sp.in) || !aligned(sp.out))
      return fail(ZK_EINVAL, "batch buffers must be non-null and 256-byte aligned");
    if (p->passes.size() > (size_t)zk::kMaxBatchPasses) return fail(ZK_EUNSUPPORTED, "too many passes for a batch");
    // The batch picks its own tile: the whole vector up to 2^kBatchTileLog
    // elements, else tiles of that size (what its workgroups hold).  A pass's
    // arguments and tables do not depend on the tile.
    const int batch_tile = (int)std::min<uint32_t>(p->log_n, zk::kBatchTileLog);
    for (const PassDesc& d : p->passes)
      if (!zk::batch_shape_supported(d.log_r, batch_tile))
        return fail(ZK_EUNSUPPORTED, "batched launches need n >= 4 and passes of at most 2^" +
                                         std::to_string(zk::kBatchTileLog) + " points");
    if (workspace_elems(p)) {
      if (!sp.work || !aligned(sp.work)) return fail(ZK_EINVAL, "batch job needs an aligned workspace");
      const size_t vb = p->n * sizeof(Fe), wb = workspace_elems(p) * sizeof(Fe);
      if (overlaps(sp.work, wb, sp.in, vb) || overlaps(sp.work, wb, sp.out, vb))
        return fail(ZK_EINVAL, "workspace must not overlap the vectors");
    }
    J.kind = zk::kJobTransform;
    J.npasses = (uint32_t)p->passes.size();
    for (size_t q = 0; q < p->passes.size(); ++q) {
      J.pass[q].args = make_pass_args(p, kind, q, sp.in, sp.out, sp.work);
      J.pass[q].log_r = p->passes[q].log_r;
      J.pass[q].log_tile = batch_tile;
      J.pass[q].tiles = (uint32_t)(p->n >> batch_tile);
    }
  }
  int cus = 0;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
  // Transforms of equal plans and kind form groups.  The persistent kernel
  // keeps each job on one XCD, and its run-time-shape tile body issues at
  // about half the rate of the pass kernels; a group that fills the chip can
  // instead run as ordinary pass launches, one per pass for all its jobs
  // (grouped launches), ahead of the persistent kernel in the same stream.
  // Which groups do is chosen greedily on a time estimate, with constants
  // measured on MI355X: the grouped launches take, per pass, a launch gap
  // plus rounds of pass tiles over the chip; the persistent kernel takes the
  // larger of its items spread over all its workgroups and its largest job
  // alone on one XCD.  A group moves while that lowers the estimated total.
  // A pointwise job runs on its own when it is more than an eighth of the
  // batch.
  auto load = [&](int k) {
    uint64_t t = 0;
    for (uint32_t q = 0; q < jobs[k].npasses; ++q) t += jobs[k].pass[q].tiles;
    return t;
  };
  uint64_t total = 0;
  for (int k = 0; k < njobs; ++k) total += load(k);
  // Plans with equal field, size and pass schedule hold equal tables, so a
  // group may span several such plans and run on the first one's tables.
  // Grouped launches fill the chip, so they use radix-4 register rounds
  // whatever the plans' register radix (the tables and bytes are the same).
  std::vector<std::vector<int>> groups;  // in order of first appearance
  {
    auto same = [&](int a, int b) {
      const ntt_plan* x = specs[a].plan;
      const ntt_plan* y = specs[b].plan;
      return kinds[a] == kinds[b] && x->field == y->field && x->log_n == y->log_n &&
             x->max_log_r == y->max_log_r && x->log_tile == y->log_tile && x->twiddle_mode == y->twiddle_mode;
    };
    for (int k = 0; k < njobs; ++k) {
      if (jobs[k].kind != zk::kJobTransform) continue;
      size_t g = 0;
      while (g < groups.size() && !same(groups[g][0], k)) ++g;
      if (g == groups.size()) groups.emplace_back();
      groups[g].push_back(k);
    }
  }
  std::vector<bool> direct(njobs, false);
  for (int k = 0; k < njobs; ++k)
    if (jobs[k].kind == zk::kJobPointwise) direct[k] = all_direct || load(k) * zk::kXcds > total;
  constexpr double kLaunchUs = 4.0;      // gap between dependent launches
  constexpr double kRoundUs = 40.0;      // one round of 2^10-element pass tiles, 4 per CU
  constexpr double kBatchItemUs = 70.0;  // one 2^11-element item of the persistent kernel
  const double batch_slots = (double)cus * zk::batch_workgroups_per_cu();
  const size_t G = groups.size();
  std::vector<double> grouped_us(G), group_items(G), alone_us(G);
  for (size_t g = 0; g < G; ++g) {
    const ntt_plan* p = specs[groups[g][0]].plan;
    const int log_tile = p->passes[0].log_tile;
    const uint64_t tiles = (p->n >> log_tile) * groups[g].size();  // per pass, at the plan's tile
    const double slots = (double)cus * (log_tile >= 11 ? 2 : 4);
    const double round_us = kRoundUs * std::ldexp(1.0, log_tile - 10);  // a round's work scales with the tile
    grouped_us[g] = (double)p->passes.size() * (kLaunchUs + std::ceil((double)tiles / slots) * round_us);
    group_items[g] = (double)(load(groups[g][0]) * groups[g].size());
    alone_us[g] = (double)load(groups[g][0]) * kBatchItemUs / (batch_slots / zk::kXcds);
  }
  double other_items = 0, other_alone = 0;  // persistent work outside the groups
  for (int k = 0; k < njobs; ++k)
    if (jobs[k].kind == zk::kJobPointwise && !direct[k]) {
      other_items += (double)load(k);
      other_alone = std::max(other_alone, (double)load(k) * kBatchItemUs / (batch_slots / zk::kXcds));
    }
  std::vector<bool> moved(G, false);
  auto estimate = [&](size_t flip) {
    double t = 0, it = other_items, alone = other_alone;
    for (size_t g = 0; g < G; ++g) {
      if (moved[g] != (g == flip)) {
        t += grouped_us[g];
      } else {
        it += group_items[g];
        alone = std::max(alone, alone_us[g]);
      }
    }
    return t + (it > 0 ? std::max(it * kBatchItemUs / batch_slots, alone) : 0.0);
  };
  if (all_direct) std::fill(moved.begin(), moved.end(), true);
  for (double best = estimate(G); !all_direct;) {
    size_t pick = G;
    for (size_t g = 0; g < G; ++g) {
      if (moved[g]) continue;
      const double t = estimate(g);
      if (t < best) {
        best = t;
        pick = g;
      }
    }
    if (pick == G) break;
    moved[pick] = true;
  }
  std::vector<std::vector<int>> direct_groups;
  for (size_t g = 0; g < G; ++g) {
    if (!moved[g]) continue;
    const ntt_plan* p = specs[groups[g][0]].plan;
    // one launch holds at most 2^31 workgroups
    const size_t per_launch = std::max<size_t>(1, (1ull << 31) / (p->n >> p->passes[0].log_tile));
    for (size_t i = 0; i < groups[g].size(); i += per_launch)
      direct_groups.emplace_back(groups[g].begin() + i,
                                 groups[g].begin() + std::min(groups[g].size(), i + per_launch));
    for (int k : groups[g]) direct[k] = true;
  }

  // Work queues of the other jobs.  Per field, jobs are dealt largest first
  // to the least loaded of up to queues_per_field queues; queues are listed
  // heaviest first, BLS12-381 queues, then BN254, then BLS12-377, and each queue
  // lists its items pass-major, larger jobs first.
  std::vector<zk::BatchItem> items;
  std::vector<zk::BatchQueue> queues;
  uint32_t nq_end[3] = {0, 0, 0};
  const uint32_t field_order[3] = {(uint32_t)zk::Bls12_381Fr::ID, (uint32_t)zk::Bn254Fr::ID,
                                   (uint32_t)zk::Bls12_377Fr::ID};
  for (int fi = 0; fi < 3; ++fi) {
    const uint32_t field = field_order[fi];
    std::vector<int> fj;
    for (int k = 0; k < njobs; ++k)
      if (jobs[k].field == field && !direct[k]) fj.push_back(k);
    std::stable_sort(fj.begin(), fj.end(), [&](int a, int b) { return load(a) > load(b); });
    const size_t nq = std::min<size_t>(fj.size(), queues_per_field);
    std::vector<std::vector<int>> qjobs(nq);
    std::vector<uint64_t> qload(nq, 0);
    for (int k : fj) {
      const size_t q = (size_t)(std::min_element(qload.begin(), qload.end()) - qload.begin());
      qjobs[q].push_back(k);  // jobs arrive largest first, so each queue's list is too
      qload[q] += load(k);
    }
    std::vector<size_t> qorder(nq);
    for (size_t q = 0; q < nq; ++q) qorder[q] = q;
    std::stable_sort(qorder.begin(), qorder.end(), [&](size_t a, size_t b) { return qload[a] > qload[b]; });
    for (size_t q : qorder) {
      zk::BatchQueue bq{(uint32_t)items.size(), 0, field, 0};
      for (int pass = 0; pass < zk::kMaxBatchPasses; ++pass)
        for (int k : qjobs[q])
          if ((uint32_t)pass < jobs[k].npasses)
            for (uint32_t t = 0; t < jobs[k].pass[pass].tiles; ++t)
              items.push_back(zk::BatchItem{(uint32_t)k, (uint32_t)pass, t, 0});
      bq.size = (uint32_t)items.size() - bq.base;
      queues.push_back(bq);
    }
    nq_end[fi] = (uint32_t)queues.size();
  }

  ntt_batch* b = new (std::nothrow) ntt_batch();
  if (!b) return fail(ZK_ENOMEM, "host allocation failed");
  b->device = dev;
  b->njobs = (uint32_t)njobs;
  b->nitems = (uint32_t)items.size();
  for (int fi = 0; fi < 3; ++fi) b->nq_end[fi] = nq_end[fi];
  // Direct work; the grouped launches' per-job vector pointers go to one
  // device array, `ptrs`, in and out lists for each pass of each group.
  std::vector<uintptr_t> ptrs;
  for (int k = 0; k < njobs; ++k)
    if (direct[k] && jobs[k].kind == zk::kJobPointwise) {
      const ntt_batch_job& sp = specs[k];
      b->direct.push_back(DirectWork{sp.plan, true, sp.in, sp.in2, sp.in3, sp.out, {}, {}});
    }
  for (const std::vector<int>& g : direct_groups) {
    const ntt_plan* p = specs[g[0]].plan;
    DirectWork d{p, false, nullptr, nullptr, nullptr, nullptr, {}, {}};
    for (size_t q = 0; q < p->passes.size(); ++q) {
      const ntt_batch_job& s0 = specs[g[0]];
      zk::PassArgs a = make_pass_args(p, kinds[g[0]], q, s0.in, s0.out, s0.work);
      a.grp_jobs = (uint32_t)g.size();
      a.log_grp_tiles = p->log_n - (uint32_t)p->passes[q].log_tile;
      d.ptr_off.push_back(ptrs.size());
      for (int k : g)
        ptrs.push_back(reinterpret_cast<uintptr_t>(make_pass_args(p, kinds[k], q, specs[k].in, specs[k].out, specs[k].work).in));
      for (int k : g)
        ptrs.push_back(reinterpret_cast<uintptr_t>(make_pass_args(p, kinds[k], q, specs[k].in, specs[k].out, specs[k].work).out));
      d.pass.push_back(a);
    }
    b->direct.push_back(std::move(d));
  }
  // Next to direct work the persistent kernel takes one workgroup per CU,
  // leaving LDS and wave slots for the pass kernels beside it (below: half
  // of that when its items can wait).
  const bool beside = !b->direct.empty() && !items.empty();
  b->grid = (uint32_t)std::min<size_t>(items.size(), (size_t)cus * (beside ? 1 : zk::batch_workgroups_per_cu()));
  // Direct work goes to up to kSideStreams side streams, dealt largest first
  // (by tiles over all passes) to the least loaded, so that groups too small
  // to fill the chip alone run at the same time.
  constexpr size_t kSideStreams = 3;
  const size_t nsides = std::min(kSideStreams, b->direct.size());
  if (nsides > 1 || beside) {
    std::vector<size_t> order(b->direct.size());
    std::vector<uint64_t> work(b->direct.size(), 0), lane_load(nsides, 0);
    for (size_t i = 0; i < order.size(); ++i) {
      order[i] = i;
      const DirectWork& d = b->direct[i];
      work[i] = d.pointwise ? (d.plan->n >> 10) : (d.plan->n >> d.plan->passes[0].log_tile) * d.pass.size() *
                                                       std::max<uint32_t>(1, d.pass.empty() ? 1 : d.pass[0].grp_jobs);
    }
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t c) { return work[a] > work[c]; });
    for (size_t i : order) {
      const size_t l = (size_t)(std::min_element(lane_load.begin(), lane_load.end()) - lane_load.begin());
      b->direct[i].lane = l;
      lane_load[l] += work[i];
    }
    // Beside direct work whose longest lane takes longer than the persistent
    // kernel would on half the CUs, the persistent kernel gets half the CUs:
    // its items have slack, and the freed slots go to the direct pass
    // launches, whose chain of dependent passes is then the batch's critical
    // path.  (64-job batch: 0.512-0.520 against 0.543 ms; below half the
    // CUs it measured flat.)  Lane times use the estimate above; the
    // persistent kernel's is allowed twice the longest lane's, since that
    // estimate counts a pass alone on the chip.
    if (beside) {
      std::vector<double> lane_us(nsides, 0.0);
      for (const DirectWork& d : b->direct) {
        if (d.pointwise) continue;
        const int log_tile = d.plan->passes[0].log_tile;
        const double tiles = (double)(d.plan->n >> log_tile) * std::max<uint32_t>(1, d.pass[0].grp_jobs);
        const double slots = (double)cus * (log_tile >= 11 ? 2 : 4);
        lane_us[d.lane] += (double)d.pass.size() *
                           (kLaunchUs + std::ceil(tiles / slots) * kRoundUs * std::ldexp(1.0, log_tile - 10));
      }
      const double longest = *std::max_element(lane_us.begin(), lane_us.end());
      const uint32_t half = (uint32_t)std::max(1, cus / 2);
      if ((double)items.size() * kBatchItemUs / half <= 2.0 * longest)
        b->grid = std::min<uint32_t>(b->grid, half);
    }
    b->sides.assign(nsides, nullptr);
    b->joins.assign(nsides, nullptr);
    e = take_event(dev, &b->fork_ev);
    for (size_t i = 0; i < nsides && e == hipSuccess; ++i) {
      e = take_stream(dev, &b->sides[i]);
      if (e == hipSuccess) e = take_event(dev, &b->joins[i]);
    }
    if (e != hipSuccess) {
      free_batch(b);
      return hip_fail(e, "batch side streams");
    }
  }
  e = take_event(dev, &b->done_ev);
  if (e != hipSuccess) {
    b->done_ev = nullptr;
    free_batch(b);
    return hip_fail(e, "batch event");
  }
  const size_t jobs_bytes = ((sizeof(zk::BatchJob) * jobs.size() + 255) / 256) * 256;
  const size_t items_bytes = ((sizeof(zk::BatchItem) * items.size() + 255) / 256) * 256;
  const size_t queues_bytes = ((sizeof(zk::BatchQueue) * queues.size() + 255) / 256) * 256;
  const size_t ctl_words = zk::kCtlDone + (size_t)njobs * zk::kMaxBatchPasses;
  const size_t ctl_bytes = ((ctl_words * sizeof(uint32_t) + 255) / 256) * 256;
  // (the 256-byte-aligned word past the descriptors holds the status in the
  // host twin)
  e = take_desc(dev, jobs_bytes + items_bytes + queues_bytes + ctl_bytes + ptrs.size() * sizeof(uintptr_t) + 512,
                &b->d_mem, &b->d_mem_bytes, &b->h_mem);
  if (e != hipSuccess) {
    b->d_mem = nullptr;
    free_batch(b);
    return hip_fail(e, "hipMalloc(batch)");
  }
  char* base = static_cast<char*>(b->d_mem);
  b->d_jobs = reinterpret_cast<zk::BatchJob*>(base);
  b->d_items = reinterpret_cast<zk::BatchItem*>(base + jobs_bytes);
  b->d_queues = reinterpret_cast<zk::BatchQueue*>(base + jobs_bytes + items_bytes);
  b->d_ctl = reinterpret_cast<uint32_t*>(base + jobs_bytes + items_bytes + queues_bytes);
  uintptr_t* d_ptrs = reinterpret_cast<uintptr_t*>(base + jobs_bytes + items_bytes + queues_bytes + ctl_bytes);
  for (DirectWork& d : b->direct)
    for (size_t q = 0; q < d.pass.size(); ++q) {
      d.pass[q].grp_in = reinterpret_cast<const Fe* const*>(d_ptrs + d.ptr_off[q]);
      d.pass[q].grp_out = reinterpret_cast<Fe* const*>(d_ptrs + d.ptr_off[q] + d.pass[q].grp_jobs);
    }
  // All descriptors in one host image of the block, uploaded with one copy
  // on a stream of the library's own (a copy on the null stream could be
  // ordered after work the caller has queued on other streams).
  const size_t used = jobs_bytes + items_bytes + queues_bytes + ctl_bytes + ptrs.size() * sizeof(uintptr_t);
  std::vector<char> image(used, 0);
  if (!jobs.empty()) std::memcpy(image.data(), jobs.data(), sizeof(zk::BatchJob) * jobs.size());
  if (!items.empty()) std::memcpy(image.data() + jobs_bytes, items.data(), sizeof(zk::BatchItem) * items.size());
  if (!queues.empty())
    std::memcpy(image.data() + jobs_bytes + items_bytes, queues.data(), sizeof(zk::BatchQueue) * queues.size());
  {
    std::vector<uint32_t> ctl(ctl_words, 0);
    ctl[zk::kCtlSpinLimit] = kDefaultSpinLimit;
    std::memcpy(image.data() + jobs_bytes + items_bytes + queues_bytes, ctl.data(), ctl_words * sizeof(uint32_t));
  }
  if (!ptrs.empty())
    std::memcpy(image.data() + jobs_bytes + items_bytes + queues_bytes + ctl_bytes, ptrs.data(),
                ptrs.size() * sizeof(uintptr_t));
  if (capture) {
    e = copy_on_own_stream(dev, b->d_mem, image.data(), used, hipMemcpyHostToDevice);
  } else {
    // Without a graph the image waits in the block's pinned twin (made once
    // per pooled block) and goes up on the first launch's stream.
    if (!b->h_mem) e = hipHostMalloc(&b->h_mem, b->d_mem_bytes, hipHostMallocDefault);
    if (e == hipSuccess) {
      std::memcpy(b->h_mem, image.data(), used);
      b->upload_bytes = used;
      b->upload_pending = true;
      b->status_host = reinterpret_cast<uint32_t*>(static_cast<char*>(b->h_mem) + (used + 255) / 256 * 256);
    } else {
      b->h_mem = nullptr;
    }
  }
  if (e != hipSuccess) {
    free_batch(b);
    return hip_fail(e, "batch descriptor upload");
  }
  if (capture) {
    // One graph: the direct jobs' passes, the counter reset kernel and the
    // persistent kernel.
    e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      const int rc = batch_enqueue(b, b->capture_stream);
      e = hipStreamEndCapture(b->capture_stream, &b->graph);
      if (rc != ZK_OK) {
        free_batch(b);
        return rc;
      }
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      free_batch(b);
      return hip_fail(e, "batch graph capture");
    }
  }
  *out = b;
  return ZK_OK;
}

// Forward NTTs in place: job k transforms d_bufs[k] with its own slice of
// the workspace.
int forward_specs(std::vector<ntt_batch_job>* specs, const ntt_plan* const* plans, void* const* d_bufs, int njobs,
                  void* d_work) {
  if (njobs < 0 || (njobs > 0 && (!plans || !d_bufs))) return fail(ZK_EINVAL, "bad job arrays");
  const size_t need = njobs > 0 ? batch_work_elems(plans, njobs) : 0;
  if (need && (!d_work || !aligned(d_work))) return fail(ZK_EINVAL, "batch needs an aligned workspace");
  Fe* work = static_cast<Fe*>(d_work);
  specs->resize(njobs);
  for (int k = 0; k < njobs; ++k) {
    ntt_batch_job& sp = (*specs)[k];
    std::memset(&sp, 0, sizeof sp);
    sp.plan = plans[k];
    sp.op = ZK_OP_FORWARD;
    sp.in = d_bufs[k];
    sp.out = d_bufs[k];
    if (plans[k] && workspace_elems(plans[k])) {
      sp.work = work;
      work += workspace_elems(plans[k]);
    }
  }
  return ZK_OK;
}

}  // namespace

extern "C" {

size_t ntt_batch_workspace_bytes(const ntt_plan* const* plans, int njobs) {
  return (plans && njobs > 0) ? batch_work_elems(plans, njobs) * sizeof(Fe) : 0;
}

int ntt_batch_create(ntt_batch** out, const ntt_plan* const* plans, void* const* d_bufs, int njobs, void* d_work) {
  std::vector<ntt_batch_job> specs;
  if (int rc = forward_specs(&specs, plans, d_bufs, njobs, d_work)) return rc;
  return batch_build(out, specs.data(), njobs, true);
}

int ntt_batch_create_jobs(ntt_batch** out, const ntt_batch_job* jobs, int njobs, int flags) {
  if (flags & ~(ZK_BATCH_GRAPH | ZK_BATCH_DIRECT | ZK_BATCH_QUEUES_MASK))
    return fail(ZK_EUNSUPPORTED, "unknown batch flag bits");
  const size_t q = (size_t)((flags & ZK_BATCH_QUEUES_MASK) >> ZK_BATCH_QUEUES_SHIFT);
  if (q > (size_t)zk::kMaxLocalQueues) return fail(ZK_EUNSUPPORTED, "at most 32 queues per field");
  return batch_build(out, jobs, njobs, (flags & ZK_BATCH_GRAPH) != 0, q ? q : kQueuesPerField,
                     (flags & ZK_BATCH_DIRECT) != 0);
}

// After every launch: the event that tells when the batch's descriptors
// are free for reuse.
int mark_launched(const ntt_batch* b, hipStream_t s) {
  hipError_t e = hipEventRecord(b->done_ev, s);
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord(batch)");
  const_cast<ntt_batch*>(b)->launched = true;
  return ZK_OK;
}

int ntt_batch_launch(const ntt_batch* b, void* stream) {
  if (!b) return fail(ZK_EINVAL, "null batch");
  if (!b->exec) return fail(ZK_EINVAL, "batch was created without a graph; use ntt_batch_launch_eager");
  hipError_t e = hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch(batch)");
  b->status_on_host = false;
  return mark_launched(b, static_cast<hipStream_t>(stream));
}

int ntt_batch_launch_eager(const ntt_batch* b, void* stream) {
  if (!b) return fail(ZK_EINVAL, "null batch");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (int rc = batch_enqueue(b, s)) return rc;
  b->status_on_host = false;
  if (b->status_host) {
    // the error word follows the launch to the pinned twin, so that the
    // status is read without a copy that could queue behind other streams
    hipError_t e = hipMemcpyAsync(b->status_host, b->d_ctl + zk::kCtlError, sizeof(uint32_t),
                                  hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "batch status copy");
    b->status_on_host = true;
  }
  return mark_launched(b, s);
}

int ntt_batch_status(const ntt_batch* b) {
  if (!b) return fail(ZK_EINVAL, "null batch");
  uint32_t err = 0;
  if (b->status_on_host) {
    err = *static_cast<volatile const uint32_t*>(b->status_host);
  } else {
    hipError_t e = copy_on_own_stream(b->device, &err, b->d_ctl + zk::kCtlError, sizeof err, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "batch status readback");
  }
  if (err & zk::kBatchErrWait)
    return fail(ZK_EDEVICE, "a batched dependency wait exceeded its poll limit; outputs are invalid");
  if (err) return fail(ZK_EDEVICE, "the batch ended with items not run; outputs are invalid");
  return ZK_OK;
}

int ntt_batch_set_spin_limit(ntt_batch* b, uint32_t polls) {
  if (!b) return fail(ZK_EINVAL, "null batch");
  if (b->upload_pending) {  // still in the host image: set it there
    const size_t off = reinterpret_cast<char*>(b->d_ctl + zk::kCtlSpinLimit) - static_cast<char*>(b->d_mem);
    std::memcpy(static_cast<char*>(b->h_mem) + off, &polls, sizeof polls);
    return ZK_OK;
  }
  hipError_t e = copy_on_own_stream(b->device, b->d_ctl + zk::kCtlSpinLimit, &polls, sizeof polls,
                                    hipMemcpyHostToDevice);
  return e == hipSuccess ? ZK_OK : hip_fail(e, "batch spin limit");
}

int ntt_batch_items(const ntt_batch* b) { return b ? (int)b->nitems : 0; }

int ntt_batch_grid(const ntt_batch* b) { return b ? (int)b->grid : 0; }

void ntt_batch_destroy(ntt_batch* b) { free_batch(b); }

int ntt_batch_forward(const ntt_plan* const* plans, void* const* d_bufs, int njobs, void* d_work, void* stream) {
  std::vector<ntt_batch_job> specs;
  if (int rc = forward_specs(&specs, plans, d_bufs, njobs, d_work)) return rc;
  ntt_batch* b = nullptr;
  int rc = batch_build(&b, specs.data(), njobs, false);
  if (rc) return rc;
  rc = ntt_batch_launch_eager(b, stream);
  if (!rc) {
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    rc = e == hipSuccess ? ntt_batch_status(b) : hip_fail(e, "batch synchronise");
  }
  free_batch(b);
  return rc;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Multi-scalar multiplication (BLS12-381 G1)

struct msm_bases {
  int device = 0;
  uint64_t n = 0;
  int c = 0;
  int windows = 0;
  uint32_t per_group = 1;  // scalars per histogram group
  uint32_t groups = 1;
  uint32_t lanes = 1;      // accumulation lanes
  uint32_t kmin = 32;      // fewest sorted entries per accumulation lane
  void* table = nullptr;
};

namespace {

constexpr int kScalarBits = 255;  // BLS12-381 Fr elements are below 2^255

struct MsmLayout {
  size_t digits, ranks, hist, counts, offsets, entries, head, tail, big, big_count, buckets, chunk_sums, level_a,
      level_b, total;
};

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

MsmLayout msm_layout(const msm_bases* b) {
  MsmLayout L{};
  const size_t nb = size_t(1) << b->c;
  const size_t entries = (size_t)b->windows * b->n;
  const size_t T = (nb + zk::msm::kChunk - 1) / zk::msm::kChunk;
  const size_t per = (size_t)zk::msm::kLevel0Lanes * zk::msm::kLevel0Chunks;
  const size_t T0 = (T + per - 1) / per;
  const size_t xyzz = zk::msm::kXyzzWords * sizeof(uint32_t);
  size_t off = 0;
  L.digits = off;
  off += round256(entries * sizeof(uint16_t));
  L.ranks = off;
  off += round256(entries * sizeof(uint16_t));
  L.hist = off;
  off += round256((size_t)b->groups * nb * sizeof(uint32_t));
  L.counts = off;
  off += round256(nb * sizeof(uint32_t));
  L.offsets = off;
  off += round256((nb + 1) * sizeof(uint32_t));
  L.entries = off;
  off += round256(entries * sizeof(uint32_t));
  L.head = off;
  off += round256((size_t)b->lanes * xyzz);
  L.tail = off;
  off += round256((size_t)b->lanes * xyzz);
  L.big = off;
  off += round256((size_t)zk::msm::max_big_buckets(b->lanes) * sizeof(uint32_t));
  L.big_count = off;
  off += round256(sizeof(uint32_t));
  L.buckets = off;
  off += round256(nb * xyzz);
  L.chunk_sums = off;
  off += round256(T * xyzz);
  L.level_a = off;
  off += round256((size_t)b->c * T0 * xyzz);
  L.level_b = off;
  off += round256((size_t)b->c * xyzz);
  L.total = off;
  return L;
}

}  // namespace

extern "C" {

int msm_bases_create(msm_bases** out, const void* d_points, uint64_t n, uint32_t window_bits, void* stream) {
  if (!out) return fail(ZK_EINVAL, "null output pointer");
  *out = nullptr;
  if (n == 0) return fail(ZK_EINVAL, "an MSM needs at least one point");
  if (!d_points || !aligned(d_points)) return fail(ZK_EINVAL, "points must be non-null and 256-byte aligned");
  if (window_bits > 16) return fail(ZK_EUNSUPPORTED, "window_bits must be 0 (automatic) or 1..16");
  int c = (int)window_bits;
  if (!c) {
    int lg = 0;
    while ((1ull << (lg + 1)) <= n) ++lg;
    c = std::max(4, std::min(16, lg - 2));
  }
  const int windows = (kScalarBits + c - 1) / c;
  if ((uint64_t)windows * n >= (1ull << 32)) return fail(ZK_EUNSUPPORTED, "too many points for this window size");
  msm_bases* b = new (std::nothrow) msm_bases();
  if (!b) return fail(ZK_ENOMEM, "host allocation failed");
  hipError_t e = hipGetDevice(&b->device);
  if (e != hipSuccess) {
    delete b;
    return hip_fail(e, "hipGetDevice");
  }
  b->n = n;
  b->c = c;
  b->windows = windows;
  // histogram groups: per_group x windows digits, each bucket's count in a
  // group below 2^16
  b->per_group = (uint32_t)std::min<uint64_t>(n, 65535u / (uint32_t)windows);
  b->groups = (uint32_t)((n + b->per_group - 1) / b->per_group);
  // accumulation lanes: the resident ones, fewer when the entries are few
  e = zk::msm::accumulate_lanes(&b->lanes);
  if (e != hipSuccess) {
    delete b;
    return hip_fail(e, "accumulation occupancy");
  }
  b->lanes = (uint32_t)std::max<uint64_t>(
      1, std::min<uint64_t>(b->lanes, ((uint64_t)windows * n + b->kmin - 1) / b->kmin));
  const size_t table_bytes = (size_t)windows * n * zk::msm::kPointWords * sizeof(uint32_t);
  e = hipMalloc(&b->table, table_bytes);
  if (e != hipSuccess) {
    delete b;
    return hip_fail(e, "hipMalloc(MSM table)");
  }
  // the precomputation's XYZZ scratch, a chunk of points at a time
  const uint64_t chunk_pts = std::min<uint64_t>(n, 1ull << 18);
  void* scratch = nullptr;
  e = hipMalloc(&scratch, (size_t)chunk_pts * windows * 60 * sizeof(uint32_t));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint32_t* pts = static_cast<const uint32_t*>(d_points);
  uint32_t* table = static_cast<uint32_t*>(b->table);
  for (uint64_t lo = 0; lo < n && e == hipSuccess; lo += chunk_pts)
    e = zk::msm::launch_precompute(pts, n, lo, std::min<uint64_t>(chunk_pts, n - lo), c, windows, table,
                                   static_cast<uint32_t*>(scratch), s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (scratch) (void)hipFree(scratch);
  if (e != hipSuccess) {
    (void)hipFree(b->table);
    delete b;
    return hip_fail(e, "MSM precomputation");
  }
  *out = b;
  return ZK_OK;
}

void msm_bases_destroy(msm_bases* b) {
  if (!b) return;
  if (b->table) (void)hipFree(b->table);
  delete b;
}

uint64_t msm_bases_count(const msm_bases* b) { return b ? b->n : 0; }

int msm_bases_window_bits(const msm_bases* b) { return b ? b->c : 0; }

size_t msm_bases_device_bytes(const msm_bases* b) {
  return b ? (size_t)b->windows * b->n * zk::msm::kPointWords * sizeof(uint32_t) : 0;
}

size_t msm_workspace_bytes(const msm_bases* b) { return b ? msm_layout(b).total : 0; }

int msm_compute(const msm_bases* b, const void* d_scalars, void* d_result, void* d_work, void* stream) {
  if (!b) return fail(ZK_EINVAL, "null bases");
  if (!d_scalars || !d_result || !d_work) return fail(ZK_EINVAL, "null pointer");
  if (!aligned(d_scalars) || !aligned(d_result) || !aligned(d_work))
    return fail(ZK_EINVAL, "pointers must be 256-byte aligned");
  const MsmLayout L = msm_layout(b);
  {
    const size_t sb = b->n * 8 * sizeof(uint32_t), rb = zk::msm::kXyzzWords * sizeof(uint32_t);
    if (overlaps(d_work, L.total, d_scalars, sb) || overlaps(d_result, rb, d_scalars, sb) ||
        overlaps(d_result, rb, d_work, L.total))
      return fail(ZK_EINVAL, "scalars, result and workspace must not overlap");
  }
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != b->device) return fail(ZK_EINVAL, "the current HIP device is not the bases' device");
  char* w = static_cast<char*>(d_work);
  zk::msm::MsmLaunch m{};
  m.table = static_cast<const uint32_t*>(b->table);
  m.scalars = static_cast<const uint32_t*>(d_scalars);
  m.n = b->n;
  m.c = b->c;
  m.windows = b->windows;
  m.per_group = b->per_group;
  m.groups = b->groups;
  m.lanes = b->lanes;
  m.kmin = b->kmin;
  m.digits = reinterpret_cast<uint16_t*>(w + L.digits);
  m.ranks = reinterpret_cast<uint16_t*>(w + L.ranks);
  m.hist = reinterpret_cast<uint32_t*>(w + L.hist);
  m.counts = reinterpret_cast<uint32_t*>(w + L.counts);
  m.offsets = reinterpret_cast<uint32_t*>(w + L.offsets);
  m.entries = reinterpret_cast<uint32_t*>(w + L.entries);
  m.head = reinterpret_cast<uint32_t*>(w + L.head);
  m.tail = reinterpret_cast<uint32_t*>(w + L.tail);
  m.big = reinterpret_cast<uint32_t*>(w + L.big);
  m.big_count = reinterpret_cast<uint32_t*>(w + L.big_count);
  m.buckets = reinterpret_cast<uint32_t*>(w + L.buckets);
  m.chunk_sums = reinterpret_cast<uint32_t*>(w + L.chunk_sums);
  m.level_a = reinterpret_cast<uint32_t*>(w + L.level_a);
  m.level_b = reinterpret_cast<uint32_t*>(w + L.level_b);
  m.result = static_cast<uint32_t*>(d_result);
  e = zk::msm::launch_msm(m, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? ZK_OK : hip_fail(e, "MSM launch");
}

}  // extern "C"
