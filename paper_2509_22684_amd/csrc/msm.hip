// Multi-scalar multiplication on BLS12-381 G1: Q = sum_i s_i P_i.
//
// MSM is the paper's other dominant proving kernel (Section II-A, Fig. 4(a));
// the libraries it measures compute it with Pippenger's bucket method and
// their cost is counted in point additions and doublings (Table V).  This is
// the bucket method laid out for MI355X:
//
// * Fixed bases with per-window multiples.  The points of a Groth16 MSM are
//   the proving key's, fixed across proofs, so msm_bases_create stores, for
//   c-bit windows w = 0 .. W-1, the affine multiples 2^(c w) P_i (W n points:
//   1.5 GiB at n = 2^20, c = 16, small next to 288 GB of HBM).  A scalar's
//   window digits then all index one set of 2^c - 1 buckets, and the
//   window-by-window Horner combination, a chain of W c point doublings that
//   no amount of parallelism shortens, disappears from every MSM.
// * Counting sort of (digit, point) pairs: per-workgroup histograms in LDS
//   (each entry keeps its rank within its group and bucket), a prefix over
//   the groups per bucket, one scan over the buckets, and a scatter put the
//   points of each bucket next to each other, with no global atomics.
// * Bucket accumulation: the sorted entries are cut into equal runs, one per
//   lane, across bucket boundaries; a lane adds its run's points into XYZZ
//   accumulators with mixed (XYZZ + affine) additions, 8 multiplications
//   and 2 squarings each in four rounds of independent products, and the
//   segments at the runs' ends then combine per bucket.  XYZZ coordinates
//   (x = X / ZZ, y = Y / ZZZ) keep additions free of inversions.
// * Bucket reduction by bits: sum_k k B_k = sum_b 2^b G_b with
//   G_b = sum of the buckets whose index has bit b set.  The G_b are
//   independent reductions (chunk sums formed once, chunks per lane, then
//   trees in LDS), and the c terms 2^b G_b are doubled in parallel and
//   summed by a tree: a critical path of a few dozen point operations,
//   where the running-sum method is a serial chain of 2^(c+1) additions.
//
// Field arithmetic: fq.hpp (12 x 32-bit limbs, Montgomery FIPS products).
// Scalars arrive as the NTT library's Montgomery limbs over BLS12-381 Fr and
// are converted with one product by 1.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "field.hpp"
#include "fq.hpp"
#include "msm.hpp"

namespace zk {
namespace msm {
namespace {

using fq::Fq;

struct Affine {
  Fq x, y;
};
struct Xyzz {
  Fq X, Y, ZZ, ZZZ;
};

__device__ __forceinline__ Xyzz infinity() {
  Xyzz r;
  r.X = fq::one();
  r.Y = fq::one();
  r.ZZ = fq::zero();
  r.ZZZ = fq::zero();
  return r;
}

__device__ __forceinline__ bool is_inf(const Xyzz& p) { return fq::is_zero(p.ZZ); }

__device__ __forceinline__ Xyzz from_affine(const Affine& a) {
  Xyzz r;
  r.X = a.x;
  r.Y = a.y;
  r.ZZ = fq::one();
  r.ZZZ = fq::one();
  return r;
}

// 2 P in XYZZ (y^2 = x^3 + b, a = 0): U = 2Y, V = U^2, W = U V, S = X V,
// M = 3 X^2; X3 = M^2 - 2S, Y3 = M (S - X3) - W Y, ZZ3 = V ZZ, ZZZ3 = W ZZZ.
// Infinity (ZZ = 0) and points with Y = 0 give ZZ3 = 0.
// The products run in three rounds of independent ones (2, 4, 3).
__device__ __forceinline__ Xyzz dbl(const Xyzz& p) {
  const Fq U = fq::dbl(p.Y);
  Fq V, XX;
  fq::mul2(V, U, U, XX, p.X, p.X);
  const Fq M = fq::add(fq::dbl(XX), XX);
  Fq W, S, MM;
  Xyzz r;
  fq::mul4(W, U, V, S, p.X, V, MM, M, M, r.ZZ, V, p.ZZ);
  r.X = fq::sub(MM, fq::dbl(S));
  Fq t, WY;
  fq::mul3(t, M, fq::sub(S, r.X), WY, W, p.Y, r.ZZZ, W, p.ZZZ);
  r.Y = fq::sub(t, WY);
  return r;
}

// 2 A for an affine point: U = 2y, V = U^2, W = U V, S = x V, M = 3 x^2;
// X3 = M^2 - 2S, Y3 = M (S - X3) - W y, ZZ3 = V, ZZZ3 = W.
__device__ __forceinline__ Xyzz dbl_affine(const Affine& a) {
  const Fq U = fq::dbl(a.y);
  Fq V, XX;
  fq::mul2(V, U, U, XX, a.x, a.x);
  Fq W, S;
  fq::mul2(W, U, V, S, a.x, V);
  const Fq M = fq::add(fq::dbl(XX), XX);
  Xyzz r;
  r.X = fq::sub(fq::sqr(M), fq::dbl(S));
  Fq t, WY;
  fq::mul2(t, M, fq::sub(S, r.X), WY, W, a.y);
  r.Y = fq::sub(t, WY);
  r.ZZ = V;
  r.ZZZ = W;
  return r;
}

// P + A with A affine: U2 = x2 ZZ1, S2 = y2 ZZZ1, P = U2 - X1, R = S2 - Y1,
// PP = P^2, PPP = P PP, Q = X1 PP; X3 = R^2 - PPP - 2Q,
// Y3 = R (Q - X3) - Y1 PPP, ZZ3 = ZZ1 PP, ZZZ3 = ZZZ1 PPP.  P = 0 means
// x-coordinates agree: the points are equal (double A) or opposite
// (infinity).
__device__ __forceinline__ Xyzz add_mixed(const Xyzz& p, const Affine& a) {
  if (is_inf(p)) return from_affine(a);
  Fq U2, S2;
  fq::mul2(U2, a.x, p.ZZ, S2, a.y, p.ZZZ);
  const Fq P = fq::sub(U2, p.X);
  const Fq R = fq::sub(S2, p.Y);
  if (fq::is_zero(P)) return fq::is_zero(R) ? dbl_affine(a) : infinity();
  Fq PP, RR;
  fq::mul2(PP, P, P, RR, R, R);
  Fq PPP, Qx;
  fq::mul2(PPP, P, PP, Qx, p.X, PP);
  Xyzz r;
  r.X = fq::sub(fq::sub(RR, PPP), fq::dbl(Qx));
  Fq t, YP;
  fq::mul4(t, R, fq::sub(Qx, r.X), YP, p.Y, PPP, r.ZZ, p.ZZ, PP, r.ZZZ, p.ZZZ, PPP);
  r.Y = fq::sub(t, YP);
  return r;
}

// P1 + P2, both XYZZ: U1 = X1 ZZ2, U2 = X2 ZZ1, S1 = Y1 ZZZ2, S2 = Y2 ZZZ1,
// P = U2 - U1, R = S2 - S1, PP = P^2, PPP = P PP, Q = U1 PP;
// X3 = R^2 - PPP - 2Q, Y3 = R (Q - X3) - S1 PPP, ZZ3 = ZZ1 ZZ2 PP,
// ZZZ3 = ZZZ1 ZZZ2 PPP.
// The 14 products run in four rounds of independent ones (4, 2, 4, 4).
__device__ __forceinline__ Xyzz add(const Xyzz& p, const Xyzz& q) {
  if (is_inf(p)) return q;
  if (is_inf(q)) return p;
  Fq U1, U2, S1, S2;
  fq::mul4(U1, p.X, q.ZZ, U2, q.X, p.ZZ, S1, p.Y, q.ZZZ, S2, q.Y, p.ZZZ);
  const Fq P = fq::sub(U2, U1);
  const Fq R = fq::sub(S2, S1);
  if (fq::is_zero(P)) return fq::is_zero(R) ? dbl(p) : infinity();
  Fq PP, RR;
  fq::mul2(PP, P, P, RR, R, R);
  Fq PPP, Qx, z2, z3;
  fq::mul4(PPP, P, PP, Qx, U1, PP, z2, p.ZZ, q.ZZ, z3, p.ZZZ, q.ZZZ);
  Xyzz r;
  r.X = fq::sub(fq::sub(RR, PPP), fq::dbl(Qx));
  Fq t, SP;
  fq::mul4(t, R, fq::sub(Qx, r.X), SP, S1, PPP, r.ZZ, z2, PP, r.ZZZ, z3, PPP);
  r.Y = fq::sub(t, SP);
  return r;
}

__device__ __forceinline__ Affine load_affine(const uint32_t* __restrict__ pts, uint64_t i) {
  const uint4* q = reinterpret_cast<const uint4*>(pts + 24 * i);
  Affine a;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const uint4 u = q[k], w = q[3 + k];
    a.x.v[4 * k] = u.x, a.x.v[4 * k + 1] = u.y, a.x.v[4 * k + 2] = u.z, a.x.v[4 * k + 3] = u.w;
    a.y.v[4 * k] = w.x, a.y.v[4 * k + 1] = w.y, a.y.v[4 * k + 2] = w.z, a.y.v[4 * k + 3] = w.w;
  }
  return a;
}

__device__ __forceinline__ void store_affine(uint32_t* __restrict__ pts, uint64_t i, const Affine& a) {
#pragma unroll
  for (int k = 0; k < fq::kN; ++k) {
    pts[24 * i + k] = a.x.v[k];
    pts[24 * i + 12 + k] = a.y.v[k];
  }
}

__device__ __forceinline__ Xyzz load_xyzz(const uint32_t* __restrict__ p, uint64_t i) {
  Xyzz r;
#pragma unroll
  for (int k = 0; k < fq::kN; ++k) {
    r.X.v[k] = p[48 * i + k];
    r.Y.v[k] = p[48 * i + 12 + k];
    r.ZZ.v[k] = p[48 * i + 24 + k];
    r.ZZZ.v[k] = p[48 * i + 36 + k];
  }
  return r;
}

__device__ __forceinline__ void store_xyzz(uint32_t* __restrict__ p, uint64_t i, const Xyzz& a) {
#pragma unroll
  for (int k = 0; k < fq::kN; ++k) {
    p[48 * i + k] = a.X.v[k];
    p[48 * i + 12 + k] = a.Y.v[k];
    p[48 * i + 24 + k] = a.ZZ.v[k];
    p[48 * i + 36 + k] = a.ZZZ.v[k];
  }
}

// ---------------------------------------------------------------------------
// Precomputation: table[w n + i] = 2^(c w) P_i, affine.  One lane per point
// walks the windows with c doublings each, keeping the XYZZ multiples in
// `scratch`, then turns all W of them affine with one inversion (prefix
// products of the ZZZ, Fermat inversion, back-substitution; 1/ZZ = (ZZ/ZZZ)^2).

// Points first .. first + count of n; scratch holds `count` points' rows.
__global__ void __launch_bounds__(128) precompute_kernel(const uint32_t* __restrict__ pts, uint64_t n,
                                                         uint64_t first, uint64_t count, int c, int windows,
                                                         uint32_t* __restrict__ table,
                                                         uint32_t* __restrict__ scratch) {
  const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const uint64_t i = first + k;
  const Affine a = load_affine(pts, i);
  store_affine(table, i, a);
  if (windows == 1) return;
  // scratch rows of this point: windows x (XYZZ, prefix product of ZZZ)
  uint32_t* my = scratch + k * windows * 60;
  Xyzz p = from_affine(a);
  Fq pre = fq::one();
  for (int w = 1; w < windows; ++w) {
    for (int d = 0; d < c; ++d) p = dbl(p);
    store_xyzz(my, w, p);  // 48-word slots at 48 w ...
    pre = fq::mul(pre, p.ZZZ);
#pragma unroll
    for (int k = 0; k < fq::kN; ++k) my[48 * windows + 12 * w + k] = pre.v[k];
  }
  Fq inv = fq::inverse(pre);  // 1 / prod_w ZZZ_w
  for (int w = windows - 1; w >= 1; --w) {
    const Xyzz q = load_xyzz(my, w);
    Fq prev;
    if (w > 1) {
#pragma unroll
      for (int k = 0; k < fq::kN; ++k) prev.v[k] = my[48 * windows + 12 * (w - 1) + k];
    } else {
      prev = fq::one();
    }
    Fq t, nxt;
    fq::mul2(t, inv, prev, nxt, inv, q.ZZZ);  // t = 1 / ZZZ_w; inv <- 1 / prod_{v<w} ZZZ_v
    inv = nxt;
    const Fq iz = fq::mul(q.ZZ, t);  // 1 / Z
    const Fq izz = fq::sqr(iz);      // 1 / ZZ
    Affine r;
    fq::mul2(r.x, q.X, izz, r.y, q.Y, t);
    store_affine(table, (uint64_t)w * n + i, r);
  }
}

// ---------------------------------------------------------------------------
// Digits and counting sort.

// Scalar k of n from the Montgomery form: s = S 2^-256 (a product by 1).
__device__ __forceinline__ Fe scalar_plain(const uint32_t* __restrict__ sc, uint64_t i) {
  Fe s, one;
#pragma unroll
  for (int j = 0; j < kLimbs; ++j) {
    s.v[j] = sc[8 * i + j];
    one.v[j] = j == 0 ? 1u : 0u;
  }
  return mul<Bls12_381Fr>(s, one);
}

// Bits [c w, c w + c) of s.  The limbs are picked by unrolled selects, not
// by a run-time index, so s stays in registers.
__device__ __forceinline__ uint32_t digit(const Fe& s, int c, int w) {
  const int lo = c * w;
  const int word = lo >> 5, sh = lo & 31;
  uint32_t w0 = 0u, w1 = 0u;
#pragma unroll
  for (int k = 0; k < kLimbs; ++k) {
    w0 = k == word ? s.v[k] : w0;
    w1 = k == word + 1 ? s.v[k] : w1;
  }
  const uint64_t bits = ((uint64_t)w1 << 32) | w0;
  return (uint32_t)(bits >> sh) & ((1u << c) - 1u);
}

// Counting sort without global atomics.  Workgroup g takes scalars
// [g B, g B + B) with B windows <= 65535, so that each bucket's count in the
// group fits 16 bits: the group's histogram lives in LDS as 16-bit halves of
// 32-bit words (2^c x 2 bytes, at most 128 KiB), and each digit's LDS
// increment returns its rank among the group's digits of that bucket.
// hist[g 2^c + d] = the group's count of digit d.
constexpr int kHistThreads = 1024;
constexpr uint32_t kHistWords = 1u << 15;  // 2^16 16-bit counters

__global__ void __launch_bounds__(kHistThreads) hist_kernel(const uint32_t* __restrict__ sc, uint64_t n, int c,
                                                            int windows, uint32_t per_group,
                                                            uint16_t* __restrict__ digits, uint16_t* __restrict__ ranks,
                                                            uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[kHistWords];
  const uint32_t nb = 1u << c, words = (nb + 1) / 2;
  const uint32_t t = threadIdx.x;
  for (uint32_t k = t; k < words; k += kHistThreads) h[k] = 0u;
  __syncthreads();
  const uint64_t first = (uint64_t)blockIdx.x * per_group;
  for (uint32_t k = t; k < per_group; k += kHistThreads) {
    const uint64_t i = first + k;
    if (i >= n) break;
    const Fe s = scalar_plain(sc, i);
    for (int w = 0; w < windows; ++w) {
      const uint32_t d = digit(s, c, w);
      const uint64_t e = (uint64_t)w * n + i;
      digits[e] = (uint16_t)d;
      if (d) {
        const uint32_t sh = (d & 1u) * 16u;
        ranks[e] = (uint16_t)(atomicAdd(&h[d >> 1], 1u << sh) >> sh);
      }
    }
  }
  __syncthreads();
  uint32_t* row = hist + (uint64_t)blockIdx.x * nb;
  for (uint32_t d = t; d < nb; d += kHistThreads) row[d] = (h[d >> 1] >> ((d & 1u) * 16u)) & 0xFFFFu;
}

// Per bucket d: hist[g 2^c + d] <- the counts of d in groups before g, and
// counts[d] = the total.
__global__ void __launch_bounds__(256) column_scan_kernel(uint32_t* __restrict__ hist, uint32_t nb, uint32_t groups,
                                                          uint32_t* __restrict__ counts) {
  const uint32_t d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= nb) return;
  uint32_t run = 0;
  for (uint32_t g = 0; g < groups; ++g) {
    const uint64_t k = (uint64_t)g * nb + d;
    const uint32_t v = hist[k];
    hist[k] = run;
    run += v;
  }
  counts[d] = run;
}

// Exclusive scan of counts[0 .. nb) into offsets[0 .. nb] (offsets[nb] =
// total), nb = 2^c <= 2^16.  One workgroup of 1024 threads; thread t keeps
// the run [t per, t per + per) of counts in registers (per <= 64; 16-byte
// loads and stores when per is a multiple of 4), and a tree over the runs'
// sums in LDS gives each run its start.
constexpr uint32_t kScanThreads = 1024, kScanPer = 64;

__global__ void __launch_bounds__(kScanThreads) scan_kernel(const uint32_t* __restrict__ counts, uint32_t nb,
                                                            uint32_t* __restrict__ offsets,
                                                            uint32_t* __restrict__ big_count) {
  __shared__ uint32_t part[kScanThreads];
  const uint32_t t = threadIdx.x;
  const uint32_t per = (nb + kScanThreads - 1) / kScanThreads;
  const uint32_t lo = t * per;
  const bool vec = (per & 3u) == 0;
  uint32_t v[kScanPer];
#pragma unroll
  for (uint32_t q = 0; q < kScanPer / 4; ++q) {
    if (vec && 4 * q < per) {
      const uint4 u = reinterpret_cast<const uint4*>(counts + lo)[q];
      v[4 * q] = u.x, v[4 * q + 1] = u.y, v[4 * q + 2] = u.z, v[4 * q + 3] = u.w;
    } else {
#pragma unroll
      for (uint32_t r = 0; r < 4; ++r) {
        const uint32_t j = 4 * q + r;
        v[j] = !vec && j < per && lo + j < nb ? counts[lo + j] : 0u;
      }
    }
  }
  uint32_t s = 0;
#pragma unroll
  for (uint32_t j = 0; j < kScanPer; ++j) s += j < per ? v[j] : 0u;
  part[t] = s;
  __syncthreads();
  for (uint32_t off = 1; off < kScanThreads; off <<= 1) {
    const uint32_t x = t >= off ? part[t - off] : 0u;
    __syncthreads();
    part[t] += x;
    __syncthreads();
  }
  uint32_t run = part[t] - s;  // exclusive prefix of this run
#pragma unroll
  for (uint32_t j = 0; j < kScanPer; ++j) {
    const uint32_t x = v[j];
    v[j] = run;
    run += j < per ? x : 0u;
  }
#pragma unroll
  for (uint32_t q = 0; q < kScanPer / 4; ++q) {
    if (vec && 4 * q < per) {
      reinterpret_cast<uint4*>(offsets + lo)[q] = make_uint4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
    } else {
#pragma unroll
      for (uint32_t r = 0; r < 4; ++r) {
        const uint32_t j = 4 * q + r;
        if (!vec && j < per && lo + j < nb) offsets[lo + j] = v[j];
      }
    }
  }
  if (t == kScanThreads - 1) offsets[nb] = part[kScanThreads - 1];
  if (t == 0) *big_count = 0u;  // the combine step's list of large buckets starts empty
}

// entries[offsets[d] + (earlier groups' count of d) + rank] = w n + i for
// every nonzero digit d: one thread per entry, no atomics.  Workgroup L takes
// window L mod W of scalar block L / W, so that the workgroups in flight at
// once read the histogram rows of a few groups, which stay in L2.
__global__ void __launch_bounds__(256) scatter_kernel(const uint16_t* __restrict__ digits,
                                                      const uint16_t* __restrict__ ranks, uint64_t n, int windows,
                                                      uint32_t per_group, uint32_t nb,
                                                      const uint32_t* __restrict__ hist,
                                                      const uint32_t* __restrict__ offsets,
                                                      uint32_t* __restrict__ entries) {
  const uint32_t w = blockIdx.x % (uint32_t)windows, blk = blockIdx.x / (uint32_t)windows;
  const uint64_t i = (uint64_t)blk * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t e = (uint64_t)w * n + i;
  const uint32_t d = digits[e];
  if (d) entries[offsets[d] + hist[(i / per_group) * nb + d] + ranks[e]] = (uint32_t)e;
}

// ---------------------------------------------------------------------------
// Bucket accumulation, balanced over lanes.  The E sorted entries are cut
// into runs of K = max(kmin, ceil(E / lanes)) consecutive positions, one run
// per lane, whatever the bucket sizes: every lane does the same number of
// mixed additions, and the grid is sized to the device's resident waves, so
// that the accumulation is one round of equal lanes.  A run crosses bucket
// boundaries: lane j keeps one accumulator per bucket segment of its run and
// stores the segment containing the run's first position in head[j], the one
// containing its last position (when it is another) in tail[j], and every
// segment between them, a whole bucket, straight into buckets[d].

__device__ __forceinline__ uint32_t lane_span(uint32_t E, uint32_t lanes, uint32_t kmin) {
  return max(kmin, (uint32_t)(((uint64_t)E + lanes - 1) / lanes));
}

constexpr uint32_t kAccumulateThreads = 128;

__global__ void __launch_bounds__(kAccumulateThreads) accumulate_kernel(const uint32_t* __restrict__ table,
                                                         const uint32_t* __restrict__ entries,
                                                         const uint32_t* __restrict__ offsets, uint32_t nb,
                                                         uint32_t lanes, uint32_t kmin, uint32_t* __restrict__ head,
                                                         uint32_t* __restrict__ tail,
                                                         uint32_t* __restrict__ buckets) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= lanes) return;
  const uint32_t E = offsets[nb];
  const uint32_t K = lane_span(E, lanes, kmin);
  const uint64_t start = (uint64_t)j * K;
  if (start >= E) return;
  const uint32_t lo_pos = (uint32_t)start;
  const uint32_t end = (uint32_t)min<uint64_t>(start + K, E);
  // the bucket holding position lo_pos: offsets[cur] <= lo_pos < offsets[cur + 1]
  uint32_t lo = 0, hi = nb;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (offsets[mid] <= lo_pos) lo = mid; else hi = mid;
  }
  uint32_t cur = lo, next = offsets[cur + 1];
  bool first = true;
  Xyzz acc = infinity();
  for (uint32_t k = lo_pos; k < end; ++k) {
    if (k == next) {  // bucket cur ends before position k
      if (first) store_xyzz(head, j, acc); else store_xyzz(buckets, cur, acc);
      first = false;
      acc = infinity();
      do {
        ++cur;
        next = offsets[cur + 1];
      } while (next <= k);  // skip empty buckets
    }
    acc = add_mixed(acc, load_affine(table, entries[k]));
  }
  if (first) store_xyzz(head, j, acc); else store_xyzz(tail, j, acc);
}

// Bucket d from the lanes' segments: the segment in the lane holding its
// first position (that lane's head or tail), plus the heads of the lanes
// that start inside it.  A bucket that begins and ends strictly inside one
// lane's run was stored by that lane; an empty bucket is infinity.  A bucket
// spanning more than kCombineSerial runs (skewed scalars: many equal
// digits) is listed in big[] for big_combine_kernel instead of being summed
// by one lane.

__global__ void __launch_bounds__(128) combine_kernel(const uint32_t* __restrict__ offsets, uint32_t nb,
                                                      uint32_t lanes, uint32_t kmin,
                                                      const uint32_t* __restrict__ head,
                                                      const uint32_t* __restrict__ tail,
                                                      uint32_t* __restrict__ buckets, uint32_t* __restrict__ big,
                                                      uint32_t* __restrict__ big_count) {
  const uint32_t d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= nb) return;
  const uint32_t lo = offsets[d], hi = offsets[d + 1];
  if (lo == hi) {
    store_xyzz(buckets, d, infinity());
    return;
  }
  const uint32_t E = offsets[nb];
  const uint32_t K = lane_span(E, lanes, kmin);
  const uint32_t jl = lo / K, jh = (hi - 1) / K;
  if (jh - jl > kCombineSerial) {
    big[atomicAdd(big_count, 1u)] = d;
    return;
  }
  const uint64_t run_end = min<uint64_t>((uint64_t)(jl + 1) * K, E);
  Xyzz acc;
  if (lo == jl * K) acc = load_xyzz(head, jl);
  else if (hi >= run_end) acc = load_xyzz(tail, jl);
  else return;
  for (uint32_t j = jl + 1; j <= jh; ++j) acc = add(acc, load_xyzz(head, j));
  store_xyzz(buckets, d, acc);
}

// Tree sum in LDS of the workgroup's points p[t] (t < blockDim.x, a power of
// two): log2(blockDim.x) rounds of pairwise additions.  Returns the total in
// every thread.
__device__ __forceinline__ Xyzz lds_tree_sum(const Xyzz& p, Xyzz* sh) {
  const uint32_t t = threadIdx.x;
  sh[t] = p;
  __syncthreads();
  for (uint32_t half = blockDim.x >> 1; half > 0; half >>= 1) {
    if (t < half) sh[t] = add(sh[t], sh[t + half]);
    __syncthreads();
  }
  return sh[0];
}

// A listed bucket (workgroup b takes big[b] while b < *big_count): its
// first segment (it spans more than one run, so that is the head or the
// tail of its first lane) and the heads of the runs inside it, summed by
// kBigThreads lanes with strided shares and a tree.  At most
// lanes / kCombineSerial + 1 buckets can be listed.
constexpr int kBigThreads = 256;

__global__ void __launch_bounds__(kBigThreads) big_combine_kernel(const uint32_t* __restrict__ offsets, uint32_t nb,
                                                                  uint32_t lanes, uint32_t kmin,
                                                                  const uint32_t* __restrict__ head,
                                                                  const uint32_t* __restrict__ tail,
                                                                  const uint32_t* __restrict__ big,
                                                                  const uint32_t* __restrict__ big_count,
                                                                  uint32_t* __restrict__ buckets) {
  __shared__ Xyzz sh[kBigThreads];
  if (blockIdx.x >= *big_count) return;  // the same for every thread of the workgroup
  const uint32_t d = big[blockIdx.x];
  const uint32_t lo = offsets[d], hi = offsets[d + 1];
  const uint32_t E = offsets[nb];
  const uint32_t K = lane_span(E, lanes, kmin);
  const uint32_t jl = lo / K, jh = (hi - 1) / K;
  Xyzz acc = infinity();
  if (threadIdx.x == 0) acc = lo == jl * K ? load_xyzz(head, jl) : load_xyzz(tail, jl);
  for (uint32_t j = jl + 1 + threadIdx.x; j <= jh; j += kBigThreads) acc = add(acc, load_xyzz(head, j));
  const Xyzz total = lds_tree_sum(acc, sh);
  if (threadIdx.x == 0) store_xyzz(buckets, d, total);
}

// ---------------------------------------------------------------------------
// Reduction by bits.  Buckets are grouped in chunks of kChunk consecutive
// indices.  For a bit b at or above the chunk's bits, bit b is the same for
// every bucket of chunk t (it is bit b - 3 of t), so its share of G_b is the
// whole chunk sum S_t or nothing: S_t is computed once, for all those bits.

// S_t = the sum of the buckets of chunk t.  kChunkLanes lanes share a chunk,
// each adding kChunk / kChunkLanes of its buckets, and a tree in LDS joins
// their sums: three point additions in sequence instead of seven.  (Having
// the same lanes also form the low bits' shares, with a different sum per
// lane, made the rounds divergent and took three times as long.)
constexpr uint32_t kChunkLanes = 4;
constexpr uint32_t kChunkThreads = 64;

__global__ void __launch_bounds__(kChunkThreads) chunk_sum_kernel(const uint32_t* __restrict__ buckets, uint32_t nb,
                                                                  uint32_t* __restrict__ sums) {
  __shared__ Xyzz sh[kChunkThreads];
  const uint32_t g = blockIdx.x * kChunkThreads + threadIdx.x;
  const uint32_t t = g / kChunkLanes, q = g % kChunkLanes;
  const uint32_t T = (nb + kChunk - 1) / kChunk;
  constexpr uint32_t per = kChunk / kChunkLanes;
  Xyzz acc = infinity();
  if (t < T)
    for (uint32_t d = t * kChunk + q * per; d < min(nb, t * kChunk + (q + 1) * per); ++d)
      acc = add(acc, load_xyzz(buckets, d));
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (uint32_t half = kChunkLanes / 2; half > 0; half >>= 1) {
    if (q < half) sh[threadIdx.x] = add(sh[threadIdx.x], sh[threadIdx.x + half]);
    __syncthreads();
  }
  if (q == 0 && t < T) store_xyzz(sums, t, sh[threadIdx.x]);
}

// Level 0: lane (b, u) holds the share of G_b of chunks t = u C .. u C + C - 1
// (C = kLevel0Chunks): below the chunks' bits, the sum of their buckets with
// bit b set (at most kChunk / 2 per chunk); above, the sums S_t of the
// chunks with bit b set.  A workgroup of kLevel0Lanes lanes of one bit sums
// them by a tree: out[b * ceil(T / (kLevel0Lanes C)) + blockIdx.x].  Two
// chunks per lane keep one wave per SIMD, where a point addition's latency
// is shortest.
__global__ void __launch_bounds__(kLevel0Lanes) bits_level0_kernel(const uint32_t* __restrict__ buckets,
                                                                   const uint32_t* __restrict__ sums, uint32_t nb,
                                                                   uint32_t* __restrict__ out) {
  __shared__ Xyzz sh[kLevel0Lanes];
  const uint32_t T = (nb + kChunk - 1) / kChunk;
  const uint32_t b = blockIdx.y, u = blockIdx.x * kLevel0Lanes + threadIdx.x;
  Xyzz acc = infinity();
  for (uint32_t t = u * kLevel0Chunks; t < min(T, (u + 1) * kLevel0Chunks); ++t) {
    if ((1u << b) < kChunk) {
      for (uint32_t d = t * kChunk; d < min(nb, (t + 1) * kChunk); ++d)
        if ((d >> b) & 1u) acc = add(acc, load_xyzz(buckets, d));
    } else if (((t * kChunk) >> b) & 1u) {
      acc = add(acc, load_xyzz(sums, t));
    }
  }
  const Xyzz total = lds_tree_sum(acc, sh);
  if (threadIdx.x == 0) store_xyzz(out, (uint64_t)b * gridDim.x + blockIdx.x, total);
}

// G_b for b = blockIdx.x: the sum of the `len` level-0 results of bit b,
// kReduceThreads lanes each summing a strided share, then a tree.
constexpr int kReduceThreads = 64;  // one wave: at most 2^16 / (8 * 128) = 64 level-0 results per bit
__global__ void __launch_bounds__(kReduceThreads) reduce_bit_kernel(const uint32_t* __restrict__ in, uint32_t len,
                                                                    uint32_t* __restrict__ out) {
  __shared__ Xyzz sh[kReduceThreads];
  const uint32_t b = blockIdx.x;
  Xyzz acc = infinity();
  for (uint32_t k = threadIdx.x; k < len; k += blockDim.x) acc = add(acc, load_xyzz(in, (uint64_t)b * len + k));
  const Xyzz total = lds_tree_sum(acc, sh);
  if (threadIdx.x == 0) store_xyzz(out, b, total);
}

// result = sum_b 2^b G_b (b < c <= 16): lane b doubles G_b b times, then a
// tree sums the c scaled points.
__global__ void __launch_bounds__(16) final_kernel(const uint32_t* __restrict__ G, int c, uint32_t* __restrict__ res) {
  __shared__ Xyzz sh[16];
  const int b = (int)threadIdx.x;
  Xyzz p = infinity();
  if (b < c) {
    p = load_xyzz(G, (uint64_t)b);
    for (int k = 0; k < b; ++k) p = dbl(p);
  }
  Xyzz total = lds_tree_sum(p, sh);
  if (threadIdx.x == 0) {
    // the result leaves the device canonical
    total.X = fq::canon(total.X);
    total.Y = fq::canon(total.Y);
    total.ZZ = fq::canon(total.ZZ);
    total.ZZZ = fq::canon(total.ZZZ);
    store_xyzz(res, 0, total);
  }
}

inline uint32_t blocks(uint64_t n, uint32_t per) { return (uint32_t)((n + per - 1) / per); }

}  // namespace

hipError_t launch_precompute(const uint32_t* pts, uint64_t n, uint64_t first, uint64_t count, int c, int windows,
                             uint32_t* table, uint32_t* scratch, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(precompute_kernel, dim3(blocks(count, 128)), dim3(128), 0, s, pts, n, first, count, c, windows,
                     table, scratch);
  return hipGetLastError();
}

hipError_t accumulate_lanes(uint32_t* lanes) {
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(accumulate_kernel),
                                                     kAccumulateThreads, 0);
  if (e != hipSuccess) return e;
  *lanes = (uint32_t)std::max(1, cus * std::max(1, per_cu)) * kAccumulateThreads;
  return hipSuccess;
}

hipError_t launch_msm(const MsmLaunch& m, hipStream_t s) {
  const uint32_t nb = 1u << m.c;  // bucket 0 unused
  hipError_t e;
  // counting sort: group histograms, their column prefixes, bucket offsets,
  // then the scatter
  hipLaunchKernelGGL(hist_kernel, dim3(m.groups), dim3(kHistThreads), 0, s, m.scalars, m.n, m.c, m.windows,
                     m.per_group, m.digits, m.ranks, m.hist);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(column_scan_kernel, dim3(blocks(nb, 256)), dim3(256), 0, s, m.hist, nb, m.groups, m.counts);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(kScanThreads), 0, s, m.counts, nb, m.offsets, m.big_count);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(scatter_kernel, dim3(blocks(m.n, 256) * (uint32_t)m.windows), dim3(256), 0, s, m.digits,
                     m.ranks, m.n, m.windows, m.per_group, nb, m.hist, m.offsets, m.entries);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // bucket sums: equal runs of sorted entries per lane, then the runs'
  // boundary segments into their buckets
  hipLaunchKernelGGL(accumulate_kernel, dim3(blocks(m.lanes, kAccumulateThreads)), dim3(kAccumulateThreads), 0, s,
                     m.table, m.entries, m.offsets, nb, m.lanes, m.kmin, m.head, m.tail, m.buckets);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(combine_kernel, dim3(blocks(nb, 128)), dim3(128), 0, s, m.offsets, nb, m.lanes, m.kmin, m.head,
                     m.tail, m.buckets, m.big, m.big_count);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(big_combine_kernel, dim3(max_big_buckets(m.lanes)), dim3(kBigThreads), 0, s, m.offsets, nb,
                     m.lanes, m.kmin, m.head, m.tail, m.big, m.big_count, m.buckets);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // reduction by bits
  const uint32_t T = (nb + kChunk - 1) / kChunk;
  hipLaunchKernelGGL(chunk_sum_kernel, dim3(blocks((uint64_t)T * kChunkLanes, kChunkThreads)), dim3(kChunkThreads), 0,
                     s, m.buckets, nb, m.chunk_sums);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const uint32_t T0 = blocks(T, kLevel0Lanes * kLevel0Chunks);  // level-0 results per bit
  hipLaunchKernelGGL(bits_level0_kernel, dim3(T0, m.c), dim3(kLevel0Lanes), 0, s, m.buckets, m.chunk_sums, nb,
                     m.level_a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // each bit's level-0 results into G_b, then sum_b 2^b G_b
  hipLaunchKernelGGL(reduce_bit_kernel, dim3(m.c), dim3(kReduceThreads), 0, s, m.level_a, T0, m.level_b);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(final_kernel, dim3(1), dim3(16), 0, s, m.level_b, m.c, m.result);
  return hipGetLastError();
}

}  // namespace msm
}  // namespace zk
