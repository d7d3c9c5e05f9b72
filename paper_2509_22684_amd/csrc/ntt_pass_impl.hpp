// NTT pass kernels for gfx950.
//
// The transform follows the paper's description of GPU NTTs (Section II-B):
// radix-2 Cooley-Tukey butterflies, with a block of threads performing a
// radix-2^k sub-transform through on-chip shared memory and several stages
// processed per batch.  Here each workgroup runs one radix-R "pass" of a
// Stockham (self-sorting) decomposition over a tile of J columns x R points:
//
//   * global memory is touched once per pass, by coalesced loads of J
//     consecutive columns (J x 32 bytes per row) and coalesced stores, so no
//     separate bit-reversal or shuffle pass exists and input and output are
//     in natural order;
//   * inside the tile, every thread keeps E = 2^LOG_E elements in registers
//     (E = 4 by default, 2 or 8 by plan option) and runs radix-E DIT
//     butterflies on them; rounds are separated by one exchange through LDS
//     (padded so 32-byte elements do not conflict on banks);
//   * the twiddles between passes come from a table laid out in the order
//     the pass reads its data ([r][j mod Ns]), so they stream coalesced
//     alongside it; in-tile twiddles come from a small w_R table.
//
// All arithmetic is exact and branchless (see field.hpp).  Inside a pass the
// data stays in [0, 2p) (lazy reduction: no final subtraction in the
// products, butterflies that keep that range); every pass stores canonical
// values, so buffers between passes and outputs hold canonical elements.
#pragma once
#include <utility>

#include "ntt_kernels.hpp"

namespace zk {
namespace detail {

constexpr __host__ __device__ int imin(int a, int b) { return a < b ? a : b; }

// Vectors, tables and plan data all live in device global memory; the
// address-space cast lets pointers loaded from descriptors (the batch kernel)
// use global rather than flat instructions, whose completion would also hold
// up LDS waits.
typedef unsigned int U32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const U32x4 GlobalCU4;
typedef __attribute__((address_space(1))) uint32_t GlobalU32;

// Two 16-byte loads per element; limbs are taken out one by one and stores go
// limb by limb (the compiler merges them into two 16-byte stores), which
// leaves the register allocator free to place each limb on its own.
__device__ __forceinline__ Fe load_fe(const Fe* __restrict__ p, uint64_t i) {
  GlobalCU4* q = (GlobalCU4*)(uintptr_t)(p + i);
  const U32x4 lo = q[0], hi = q[1];
  Fe r;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    r.v[k] = lo[k];
    r.v[4 + k] = hi[k];
  }
  return r;
}

__device__ __forceinline__ void store_fe(Fe* __restrict__ p, uint64_t i, const Fe& x) {
  GlobalU32* q = (GlobalU32*)(uintptr_t)(p + i);
#pragma unroll
  for (int k = 0; k < 8; ++k) q[k] = x.v[k];
}

// LDS slot of element e of a tile: one pad slot after every 8 elements, so
// lanes writing elements 8 apart land 9 slots (288 bytes) apart and spread
// over all banks.
__device__ __forceinline__ uint32_t lds_slot(uint32_t e) { return e + (e >> 3); }

constexpr __host__ __device__ int bitrev_ct(int x, int bits) {
  int r = 0;
  for (int b = 0; b < bits; ++b) r |= ((x >> b) & 1) << (bits - 1 - b);
  return r;
}

// Compile-time loop: fn(std::integral_constant<int, i>) for i < N, so every
// register-array index below is a constant and the arrays stay in VGPRs.
template <class Fn, int... I>
__device__ __forceinline__ void sfor_impl(Fn& fn, std::integer_sequence<int, I...>) {
  (fn(std::integral_constant<int, I>{}), ...);
}
template <int N, class Fn>
__device__ __forceinline__ void sfor(Fn&& fn) {
  sfor_impl(fn, std::make_integer_sequence<int, N>{});
}

// Independent products run GROUP at a time, interleaved (mul_k).  More
// products in flight hide more latency but hold more registers: with the
// 128-VGPR budget of four waves per SIMD, threads holding eight elements
// interleave two products, threads holding four interleave three (measured
// fastest on MI355X against two and four, which spills), and threads holding
// two interleave up to four.
template <int EL>
constexpr int mul_group() {
  return EL >= 8 ? 2 : EL == 4 ? 3 : 4;
}

// x[k] = x[k] w[k] for k < N, in interleaved groups of GROUP products.  The
// w[k] are canonical (tables, constants); the products are left in [0, 2p)
// (lazy reduction, field.hpp) unless CANON.
template <class F, int N, int GROUP, bool CANON = false>
__device__ __forceinline__ void mul_many(Fe* x, const Fe* w) {
  constexpr int G = N / GROUP, REST = N % GROUP;
  sfor<G>([&](auto g_) {
    constexpr int g = decltype(g_)::value;
    mul_k<F, GROUP, CANON>(x + GROUP * g, x + GROUP * g, w + GROUP * g);
  });
  if constexpr (REST == 1) {
    // a lone product keeps the reorderable form, which the scheduler can
    // overlap with surrounding loads and LDS traffic
    x[GROUP * G] = mul<F, CANON>(x[GROUP * G], w[GROUP * G]);
  } else if constexpr (REST > 1) {
    mul_k<F, REST, CANON>(x + GROUP * G, x + GROUP * G, w + GROUP * G);
  }
}

// In-register DFT of E = 2^LOGE points (natural order in and out) on
// v[OFF .. OFF + E): bit-reversed renaming, then log2 E radix-2 DIT stages
// with butterflies (x, y) -> (x + w y, x - w y).  W[k] = w_E^k for k < E/2.
// The multiplications of one stage are independent and run interleaved.
// Points in [0, 2p) in and out (lazy reduction).
template <class F, int LOGE, int OFF, int N>
__device__ __forceinline__ void dft_regs(Fe (&v)[N], const Fe* W) {
  constexpr int GROUP = mul_group<N>();
  constexpr int E = 1 << LOGE;
  if constexpr (E > 1) {
    Fe a[E];
    sfor<E>([&](auto s_) {
      constexpr int s = decltype(s_)::value;
      a[s] = v[OFF + bitrev_ct(s, LOGE)];
    });
    sfor<LOGE>([&](auto st_) {
      constexpr int st = decltype(st_)::value;
      constexpr int half = 1 << st;  // butterflies pair elements half apart
      // butterfly u has twiddle index t = u mod half; t != 0 needs a product
      constexpr int NM = (E / 2) - (E / 2) / half;
      if constexpr (NM > 0) {
        Fe ys[NM], ws[NM];
        sfor<E / 2>([&](auto u_) {
          constexpr int u = decltype(u_)::value;
          constexpr int t = u & (half - 1);
          constexpr int b = (u >> st) << (st + 1);
          constexpr int k = u - (u / half) - 1;  // rank among the t != 0 butterflies
          if constexpr (t != 0) {
            ys[k] = a[b + t + half];
            ws[k] = W[t << (LOGE - 1 - st)];
          }
        });
        mul_many<F, NM, GROUP>(ys, ws);
        sfor<E / 2>([&](auto u_) {
          constexpr int u = decltype(u_)::value;
          constexpr int t = u & (half - 1);
          constexpr int b = (u >> st) << (st + 1);
          constexpr int k = u - (u / half) - 1;
          if constexpr (t != 0) a[b + t + half] = ys[k];
        });
      }
      sfor<E / 2>([&](auto u_) {
        constexpr int u = decltype(u_)::value;
        constexpr int t = u & (half - 1);
        constexpr int b = (u >> st) << (st + 1);
        const Fe x = a[b + t];
        const Fe y = a[b + t + half];
        a[b + t] = add_lazy<F>(x, y);
        a[b + t + half] = sub_lazy<F>(x, y);
      });
    });
    sfor<E>([&](auto s_) {
      constexpr int s = decltype(s_)::value;
      v[OFF + s] = a[s];
    });
  }
}

template <int LOG_R, int LOG_TILE, int LOG_E>
struct PassShape {
  static constexpr int R = 1 << LOG_R;
  static constexpr int LOG_J = LOG_TILE - LOG_R;
  static constexpr int J = 1 << LOG_J;
  static constexpr int LE = imin(LOG_E, LOG_R);  // log2 elements per thread
  static constexpr int EL = 1 << LE;
  static constexpr int THREADS = (1 << LOG_TILE) / EL;
  static constexpr int ROUNDS = LOG_R == 0 ? 0 : (LOG_R + LE - 1) / LE;
  static constexpr int LDS_SLOTS = ROUNDS > 1 ? (1 << LOG_TILE) + (1 << LOG_TILE) / 8 : 1;
  static constexpr int SLOT_STRIDE = R / EL;  // threads per column
  // Workgroups of this tile that fit a CU's 160 KiB of LDS (multi-pass tiles;
  // single-pass shapes keep two), and the waves per SIMD the register
  // allocation aims for so that they all stay resident: WGS * THREADS / 256.
  static constexpr int LDS_BYTES = LDS_SLOTS * 32;
  static constexpr int WGS = LOG_R == LOG_TILE ? 2 : imin(4, 163840 / LDS_BYTES);
  static constexpr int MIN_WAVES = WGS * THREADS >= 256 ? WGS * THREADS / 256 : 1;
  // log2 radix of in-tile round rho: full LE except possibly the last
  static constexpr int round_log(int rho) { return imin(LE, LOG_R - rho * LE); }
  // Wave-major slot numbering (see pass_tile): with four elements per thread,
  // whole waves per column group and a multiple of four waves, every wave
  // holds slots q of one residue mod 4, so the twiddles of in-tile round 1,
  // w^(s (q mod 4)), are all 1 for a whole wave out of four.
  static constexpr int WAVES = THREADS / 64;
  static constexpr bool WAVE_Q = EL == 4 && THREADS >= 256 && WAVES % 4 == 0 && J <= 64 && LOG_R >= 4;
};

// One in-tile round rho (radix Er = 2^LR, earlier in-tile radices' product
// Nsr = 2^(rho LE)).  Thread q of column c owns slots i = q + g (R / EL) for
// g < EL / Er; slot i takes points i + s (R / Er), s < Er.  Round 0 works on
// the registers as loaded; later rounds read the tile from LDS and apply the
// in-tile twiddles w_{Nsr Er}^(s (i mod Nsr)).  All rounds but the last write
// their outputs (i / Nsr) Nsr Er + (i mod Nsr) + s Nsr back to LDS.
template <class F, int LOG_R, int LOG_TILE, int LOG_E, int RHO, int N>
__device__ __forceinline__ void tile_round(Fe (&v)[N], Fe* lds, const Fe* __restrict__ tw_r, uint32_t c,
                                           uint32_t q, bool writer) {
  using S = PassShape<LOG_R, LOG_TILE, LOG_E>;
  constexpr int LOG_NSR = RHO * S::LE;
  constexpr int LR = S::round_log(RHO);
  constexpr int ER = 1 << LR;
  constexpr int NSR = 1 << LOG_NSR;
  constexpr bool LAST = RHO + 1 == S::ROUNDS;

  if constexpr (RHO > 0) {
    sfor<S::EL>([&](auto e_) {
      constexpr int e = decltype(e_)::value;
      const uint32_t i = q + (e / ER) * S::SLOT_STRIDE;
      const uint32_t idx = i + (e % ER) * (S::R / ER);
      v[e] = lds[lds_slot(idx * S::J + c)];
    });
    // in-tile twiddles of the points with s = e mod Er != 0, interleaved
    constexpr int NM = S::EL - S::EL / ER;
    // In round 1 with wave-major slots, q mod 4 is the same on a whole wave,
    // and the wave with q mod 4 = 0 would multiply by w^0 = 1: it skips the
    // products (the result is the same bytes).
    bool twiddle = true;
    if constexpr (S::WAVE_Q && RHO == 1 && ER == 4) twiddle = __builtin_amdgcn_readfirstlane(q & 3u) != 0;
    if (twiddle) {
      Fe ys[NM], ws[NM];
      sfor<S::EL>([&](auto e_) {
        constexpr int e = decltype(e_)::value;
        constexpr int s = e % ER;
        constexpr int k = e - e / ER - 1;  // rank among the s != 0 points
        if constexpr (s != 0) {
          const uint32_t im = (q + (e / ER) * S::SLOT_STRIDE) & (NSR - 1);
          ys[k] = v[e];
          ws[k] = tw_r[(S::R / (NSR * ER)) * s * im];
        }
      });
      mul_many<F, NM, mul_group<S::EL>()>(ys, ws);
      sfor<S::EL>([&](auto e_) {
        constexpr int e = decltype(e_)::value;
        constexpr int k = e - e / ER - 1;
        if constexpr (e % ER != 0) v[e] = ys[k];
      });
    }
  }
  Fe W[ER / 2 > 0 ? ER / 2 : 1];
  sfor<ER / 2>([&](auto k_) {
    constexpr int k = decltype(k_)::value;
    W[k] = tw_r[k * (S::R / ER)];  // w_Er^k, wave-uniform
  });
  sfor<S::EL / ER>([&](auto g_) {
    constexpr int g = decltype(g_)::value;
    dft_regs<F, LR, g * ER>(v, W);
  });

  if constexpr (!LAST) {
    if constexpr (RHO > 0) __syncthreads();  // every thread has read this round's inputs
    if (writer) {
      sfor<S::EL>([&](auto e_) {
        constexpr int e = decltype(e_)::value;
        const uint32_t i = q + (e / ER) * S::SLOT_STRIDE;
        const uint32_t o = (i >> LOG_NSR) * (NSR * ER) + (i & (NSR - 1)) + (e % ER) * NSR;
        lds[lds_slot(o * S::J + c)] = v[e];
      });
    }
    __syncthreads();
    tile_round<F, LOG_R, LOG_TILE, LOG_E, RHO + 1>(v, lds, tw_r, c, q, writer);
  }
}

// One tile of one pass: J columns x R points.  `t` is the thread's index
// within the tile (t < THREADS); threads with `writer` false shadow thread t
// (same loads and arithmetic) but store nothing, so a workgroup wider than
// the tile still reaches every barrier.  `lds` holds LDS_SLOTS elements.
template <class F, int LOG_R, int LOG_TILE, int LOG_E>
__device__ __forceinline__ void pass_tile(const PassArgs& a, uint64_t tile, Fe* lds, uint32_t t, bool writer) {
  using S = PassShape<LOG_R, LOG_TILE, LOG_E>;
  // Thread t of the tile handles column c and slot q.  Lanes of a wave take
  // the J columns fastest (so global accesses stay in J x 32-byte runs); the
  // slots either follow the thread index (q = t / J) or, with wave-major
  // numbering, take the wave index as their lowest bits (q = w + WAVES k).
  const uint32_t c = t & (S::J - 1);  // column within the tile
  uint32_t q;                         // slot within the column
  if constexpr (S::WAVE_Q) {
    q = (t >> 6) + S::WAVES * ((t & 63) >> S::LOG_J);
  } else {
    q = t >> S::LOG_J;
  }
  const uint64_t n = 1ull << a.log_n;
  const uint64_t ns = 1ull << a.log_ns;
  const uint64_t j = tile * S::J + c;           // global column, < n / R
  const uint32_t log_stride = a.log_n - LOG_R;  // column stride n / R

  // Round 0 reads its points r = i + s (R / Er0) straight from global memory.
  constexpr int ER0 = 1 << S::round_log(0);
  Fe v[S::EL];
  auto point0 = [&](int e) -> uint64_t { return q + (e / ER0) * S::SLOT_STRIDE + (e % ER0) * (S::R / ER0); };
  const bool rev = a.flags & kPassReverseIn;
  sfor<S::EL>([&](auto e_) {
    constexpr int e = decltype(e_)::value;
    const uint64_t idx = j + (point0(e) << log_stride);
    v[e] = load_fe(a.in, rev ? ((n - idx) & (n - 1)) : idx);
  });
  Fe w[S::EL];  // per-point factors, multiplied in interleaved groups
  if (a.flags & kPassPreTable) {
    sfor<S::EL>([&](auto e_) {
      constexpr int e = decltype(e_)::value;
      w[e] = load_fe(a.pre_table, j + (point0(e) << log_stride));
    });
    mul_many<F, S::EL, mul_group<S::EL>()>(v, w);
  }
  if (a.tw_pass) {  // inter-pass twiddle w_{Ns R}^(r (j mod Ns)), table [r][j mod Ns]
    sfor<S::EL>([&](auto e_) {
      constexpr int e = decltype(e_)::value;
      w[e] = load_fe(a.tw_pass, (point0(e) << a.log_ns) + (j & (ns - 1)));
    });
    mul_many<F, S::EL, mul_group<S::EL>()>(v, w);
  } else if (a.tw_hi) {  // the same twiddle from the two-level tables
    // Two points at a time: holding both factors of every point at once
    // (2 EL elements on top of the data) made this branch the kernel's
    // register peak and spilled registers in every pass, table mode included.
    const uint64_t jm = j & (ns - 1);
    const uint32_t log_mult = a.log_n - a.log_ns - LOG_R;
    const uint64_t lo_mask = (1ull << a.log_lo) - 1;
    constexpr int CH = S::EL >= 2 ? 2 : 1;
    sfor<S::EL / CH>([&](auto h_) {
      constexpr int h = decltype(h_)::value;
      Fe hi[CH], lo[CH];
      sfor<CH>([&](auto k_) {
        constexpr int k = decltype(k_)::value;
        const uint64_t ex = (point0(CH * h + k) * jm) << log_mult;
        hi[k] = load_fe(a.tw_hi, ex >> a.log_lo);
        lo[k] = load_fe(a.tw_lo, ex & lo_mask);
      });
      mul_many<F, CH, CH, true>(hi, lo);  // canonical: the factor of the next product
      mul_many<F, CH, CH>(v + CH * h, hi);
    });
  }

  if constexpr (S::ROUNDS > 0) tile_round<F, LOG_R, LOG_TILE, LOG_E, 0>(v, lds, a.tw_r, c, q, writer);

  // The last round leaves output r_out = i + s (R / Er) of column j in
  // v[g Er + s]; it goes to (j / Ns) Ns R + (j mod Ns) + r_out Ns.
  constexpr int ERL = S::ROUNDS == 0 ? 1 : 1 << S::round_log(S::ROUNDS - 1);
  const uint64_t base = ((j >> a.log_ns) << (a.log_ns + LOG_R)) + (j & (ns - 1));
  auto out_index = [&](int e) -> uint64_t {
    const uint64_t r_out = q + (e / ERL) * S::SLOT_STRIDE + (e % ERL) * (S::R / ERL);
    return base + (r_out << a.log_ns);
  };
  if (a.flags & kPassPostTable) {
    Fe w[S::EL];
    sfor<S::EL>([&](auto e_) {
      constexpr int e = decltype(e_)::value;
      w[e] = load_fe(a.post_table, out_index(e));
    });
    mul_many<F, S::EL, mul_group<S::EL>()>(v, w);
  }
  if (a.flags & kPassPostConst) {
    Fe w[S::EL];
    sfor<S::EL>([&](auto e_) {
      constexpr int e = decltype(e_)::value;
      w[e] = a.post_const;
    });
    mul_many<F, S::EL, mul_group<S::EL>()>(v, w);
  }
  if (a.flags & kPassPostPointwise) {
    // the quotient's pointwise step fused into the last pass of the third
    // coset NTT: (A B - C) / (g^n - 1) with C this pass's output, one
    // element at a time (this runs once per quotient).  Where the tile has
    // LDS, the elements wait there (it is free after the last round) and
    // come back one by one, so the step's operands never sit beside all of
    // v: their register peak would otherwise be the whole kernel's and
    // spill in every pass.
    if constexpr (S::LDS_SLOTS >= S::THREADS * S::EL) {
      __syncthreads();  // every thread has read its last round's inputs
      sfor<S::EL>([&](auto e_) {
        constexpr int e = decltype(e_)::value;
        lds[lds_slot(t * S::EL + e)] = v[e];
      });
      sfor<S::EL>([&](auto e_) {
        constexpr int e = decltype(e_)::value;
        const uint64_t k = out_index(e);
        const Fe ab = mul<F>(load_fe(a.pw_a, k), load_fe(a.pw_b, k));
        const Fe r = mul<F>(sub_lazy<F>(ab, lds[lds_slot(t * S::EL + e)]), a.post_const);
        if (writer) store_fe(a.out, k, r);
      });
      return;
    } else {
      sfor<S::EL>([&](auto e_) {
        constexpr int e = decltype(e_)::value;
        const uint64_t k = out_index(e);
        const Fe ab = mul<F>(load_fe(a.pw_a, k), load_fe(a.pw_b, k));
        v[e] = mul<F>(sub_lazy<F>(ab, v[e]), a.post_const);
      });
    }
  }
  if (writer) {  // canonical out of every pass
    sfor<S::EL>([&](auto e_) {
      constexpr int e = decltype(e_)::value;
      store_fe(a.out, out_index(e), canon<F>(v[e]));
    });
  }
}

template <class F, int LOG_R, int LOG_TILE, int LOG_E>
__global__ void __launch_bounds__((PassShape<LOG_R, LOG_TILE, LOG_E>::THREADS),
                                  (PassShape<LOG_R, LOG_TILE, LOG_E>::MIN_WAVES))
    ntt_pass_kernel(PassArgs a) {
  using S = PassShape<LOG_R, LOG_TILE, LOG_E>;
  __shared__ Fe lds[S::LDS_SLOTS];
  uint32_t tile = blockIdx.x;
  if (a.grp_jobs) {
    const uint32_t job = blockIdx.x >> a.log_grp_tiles;
    tile = blockIdx.x & ((1u << a.log_grp_tiles) - 1u);
    a.in = a.grp_in[job];
    a.out = a.grp_out[job];
  }
  pass_tile<F, LOG_R, LOG_TILE, LOG_E>(a, tile, lds, threadIdx.x, true);
}

}  // namespace detail
}  // namespace zk

namespace zk {
namespace detail {

template <class F, int LOG_R, int LOG_TILE, int LOG_E>
hipError_t launch_one(const PassArgs& a, hipStream_t s) {
  using S = PassShape<LOG_R, LOG_TILE, LOG_E>;
  const uint64_t tiles = ((1ull << a.log_n) >> LOG_TILE) * (a.grp_jobs ? a.grp_jobs : 1u);
  hipLaunchKernelGGL((ntt_pass_kernel<F, LOG_R, LOG_TILE, LOG_E>), dim3((uint32_t)tiles), dim3(S::THREADS), 0, s, a);
  return hipGetLastError();
}

// Multi-pass tiles of 2^11 or 2^10 elements with radix 2^3 .. 2^9 per pass,
// 2^8-element tiles with radix 2^3 .. 2^8 for two or four elements per
// thread (small transforms spread over more CUs), and single-pass transforms
// of up to 2^11 points held in one tile.  Keep in step with
// pass_shape_supported().
template <class F, int LOG_E>
hipError_t dispatch_shape(int log_r, int log_tile, const PassArgs& a, hipStream_t s) {
  if constexpr (LOG_E <= 2) {
    if (log_tile == 8 && log_r < 8) {
      switch (log_r) {
        case 3: return launch_one<F, 3, 8, LOG_E>(a, s);
        case 4: return launch_one<F, 4, 8, LOG_E>(a, s);
        case 5: return launch_one<F, 5, 8, LOG_E>(a, s);
        case 6: return launch_one<F, 6, 8, LOG_E>(a, s);
        case 7: return launch_one<F, 7, 8, LOG_E>(a, s);
        default: break;
      }
    }
  }
  if (log_tile == 10 && log_r < 10) {
    switch (log_r) {
      case 3: return launch_one<F, 3, 10, LOG_E>(a, s);
      case 4: return launch_one<F, 4, 10, LOG_E>(a, s);
      case 5: return launch_one<F, 5, 10, LOG_E>(a, s);
      case 6: return launch_one<F, 6, 10, LOG_E>(a, s);
      case 7: return launch_one<F, 7, 10, LOG_E>(a, s);
      case 8: return launch_one<F, 8, 10, LOG_E>(a, s);
      case 9: return launch_one<F, 9, 10, LOG_E>(a, s);
      default: break;
    }
  }
  if (log_tile == 11) {
    switch (log_r) {
      case 3: return launch_one<F, 3, 11, LOG_E>(a, s);
      case 4: return launch_one<F, 4, 11, LOG_E>(a, s);
      case 5: return launch_one<F, 5, 11, LOG_E>(a, s);
      case 6: return launch_one<F, 6, 11, LOG_E>(a, s);
      case 7: return launch_one<F, 7, 11, LOG_E>(a, s);
      case 8: return launch_one<F, 8, 11, LOG_E>(a, s);
      case 9: return launch_one<F, 9, 11, LOG_E>(a, s);
      case 11: return launch_one<F, 11, 11, LOG_E>(a, s);
      default: break;
    }
  }
  if (log_tile == log_r) {
    switch (log_r) {
      case 0: return launch_one<F, 0, 0, LOG_E>(a, s);
      case 1: return launch_one<F, 1, 1, LOG_E>(a, s);
      case 2: return launch_one<F, 2, 2, LOG_E>(a, s);
      case 3: return launch_one<F, 3, 3, LOG_E>(a, s);
      case 4: return launch_one<F, 4, 4, LOG_E>(a, s);
      case 5: return launch_one<F, 5, 5, LOG_E>(a, s);
      case 6: return launch_one<F, 6, 6, LOG_E>(a, s);
      case 7: return launch_one<F, 7, 7, LOG_E>(a, s);
      case 8: return launch_one<F, 8, 8, LOG_E>(a, s);
      case 9: return launch_one<F, 9, 9, LOG_E>(a, s);
      case 10: return launch_one<F, 10, 10, LOG_E>(a, s);
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace detail
}  // namespace zk
