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
// * Counting sort of (digit, point) pairs: a histogram of the digits (each
//   entry keeps its rank in its bucket), one scan, and a scatter without
//   atomics put the points of each bucket next to each other.
// * Bucket accumulation: each bucket's points are split into S slices; one
//   lane adds a slice's points into an XYZZ accumulator with mixed
//   (XYZZ + affine) additions, 8 multiplications and 2 squarings each; the
//   slices then combine.  XYZZ coordinates (x = X / ZZ, y = Y / ZZZ) keep
//   additions free of inversions.
// * Bucket reduction by bits: sum_k k B_k = sum_b 2^b G_b with
//   G_b = sum of the buckets whose index has bit b set.  The G_b are
//   independent reductions (chunks of buckets per lane, then a tree in LDS
//   per bit), and the c terms 2^b G_b are doubled in parallel and summed by a
//   tree: a critical path of a few dozen point operations, where the
//   running-sum method is a serial chain of 2^(c+1) additions.
//
// Field arithmetic: fq.hpp (12 x 32-bit limbs, Montgomery FIPS products).
// Scalars arrive as the NTT library's Montgomery limbs over BLS12-381 Fr and
// are converted with one product by 1.
#include <hip/hip_runtime.h>

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
__device__ __forceinline__ Xyzz dbl(const Xyzz& p) {
  const Fq U = fq::dbl(p.Y);
  Fq V, XX;
  fq::mul2(V, U, U, XX, p.X, p.X);
  Fq W, S;
  fq::mul2(W, U, V, S, p.X, V);
  const Fq M = fq::add(fq::dbl(XX), XX);
  Xyzz r;
  r.X = fq::sub(fq::sqr(M), fq::dbl(S));
  Fq t, WY;
  fq::mul2(t, M, fq::sub(S, r.X), WY, W, p.Y);
  r.Y = fq::sub(t, WY);
  fq::mul2(r.ZZ, V, p.ZZ, r.ZZZ, W, p.ZZZ);
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
  const Fq PP = fq::sqr(P);
  Fq PPP, Qx;
  fq::mul2(PPP, P, PP, Qx, p.X, PP);
  Xyzz r;
  r.X = fq::sub(fq::sub(fq::sqr(R), PPP), fq::dbl(Qx));
  Fq t, YP;
  fq::mul2(t, R, fq::sub(Qx, r.X), YP, p.Y, PPP);
  r.Y = fq::sub(t, YP);
  fq::mul2(r.ZZ, p.ZZ, PP, r.ZZZ, p.ZZZ, PPP);
  return r;
}

// P1 + P2, both XYZZ: U1 = X1 ZZ2, U2 = X2 ZZ1, S1 = Y1 ZZZ2, S2 = Y2 ZZZ1,
// P = U2 - U1, R = S2 - S1, PP = P^2, PPP = P PP, Q = U1 PP;
// X3 = R^2 - PPP - 2Q, Y3 = R (Q - X3) - S1 PPP, ZZ3 = ZZ1 ZZ2 PP,
// ZZZ3 = ZZZ1 ZZZ2 PPP.
__device__ __forceinline__ Xyzz add(const Xyzz& p, const Xyzz& q) {
  if (is_inf(p)) return q;
  if (is_inf(q)) return p;
  Fq U1, U2, S1, S2;
  fq::mul2(U1, p.X, q.ZZ, U2, q.X, p.ZZ);
  fq::mul2(S1, p.Y, q.ZZZ, S2, q.Y, p.ZZZ);
  const Fq P = fq::sub(U2, U1);
  const Fq R = fq::sub(S2, S1);
  if (fq::is_zero(P)) return fq::is_zero(R) ? dbl(p) : infinity();
  const Fq PP = fq::sqr(P);
  Fq PPP, Qx;
  fq::mul2(PPP, P, PP, Qx, U1, PP);
  Xyzz r;
  r.X = fq::sub(fq::sub(fq::sqr(R), PPP), fq::dbl(Qx));
  Fq t, SP;
  fq::mul2(t, R, fq::sub(Qx, r.X), SP, S1, PPP);
  r.Y = fq::sub(t, SP);
  Fq z2, z3;
  fq::mul2(z2, p.ZZ, q.ZZ, z3, p.ZZZ, q.ZZZ);
  fq::mul2(r.ZZ, z2, PP, r.ZZZ, z3, PPP);
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

__device__ __forceinline__ uint32_t digit(const Fe& s, int c, int w) {
  const int lo = c * w;
  const int word = lo >> 5, sh = lo & 31;
  uint64_t bits = s.v[word];
  if (word + 1 < kLimbs) bits |= (uint64_t)s.v[word + 1] << 32;
  return (uint32_t)(bits >> sh) & ((1u << c) - 1u);
}

// digits[w n + i] = window w of scalar i; for each nonzero digit d the entry
// takes the next rank of bucket d (the histogram count before its increment),
// so the scatter needs no atomics of its own.
__global__ void __launch_bounds__(256) digits_kernel(const uint32_t* __restrict__ sc, uint64_t n, int c, int windows,
                                                     uint16_t* __restrict__ digits, uint32_t* __restrict__ ranks,
                                                     uint32_t* __restrict__ counts) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Fe s = scalar_plain(sc, i);
  for (int w = 0; w < windows; ++w) {
    const uint32_t d = digit(s, c, w);
    const uint64_t e = (uint64_t)w * n + i;
    digits[e] = (uint16_t)d;
    if (d) ranks[e] = atomicAdd(counts + d, 1u);
  }
}

// Exclusive scan of counts[0 .. nb) into offsets[0 .. nb] (offsets[nb] =
// total).  One workgroup of 1024 threads, each summing a contiguous run.
__global__ void __launch_bounds__(1024) scan_kernel(const uint32_t* __restrict__ counts, uint32_t nb,
                                                    uint32_t* __restrict__ offsets) {
  __shared__ uint32_t part[1024];
  const uint32_t t = threadIdx.x;
  const uint32_t per = (nb + 1023) / 1024;
  const uint32_t lo = t * per, hi = min(nb, lo + per);
  uint32_t s = 0;
  for (uint32_t k = lo; k < hi; ++k) s += counts[k];
  part[t] = s;
  __syncthreads();
  for (uint32_t off = 1; off < 1024; off <<= 1) {
    const uint32_t v = t >= off ? part[t - off] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint32_t run = part[t] - s;  // exclusive prefix of this run
  for (uint32_t k = lo; k < hi; ++k) {
    offsets[k] = run;
    run += counts[k];
  }
  if (t == 1023) offsets[nb] = part[1023];
}

// entries[offsets[d] + rank] = w n + i for every nonzero digit d: one
// thread per entry, no atomics.
__global__ void __launch_bounds__(256) scatter_kernel(const uint16_t* __restrict__ digits,
                                                      const uint32_t* __restrict__ ranks, uint64_t count,
                                                      const uint32_t* __restrict__ offsets,
                                                      uint32_t* __restrict__ entries) {
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  const uint32_t d = digits[e];
  if (d) entries[offsets[d] + ranks[e]] = (uint32_t)e;
}

// ---------------------------------------------------------------------------
// Bucket accumulation: lane (bucket d, slice s) adds the points of slice s of
// bucket d; partial[d * S + s] = that sum (XYZZ).

__global__ void __launch_bounds__(128) accumulate_kernel(const uint32_t* __restrict__ table,
                                                         const uint32_t* __restrict__ entries,
                                                         const uint32_t* __restrict__ offsets, uint32_t nb,
                                                         uint32_t slices, uint32_t* __restrict__ partial) {
  const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (uint64_t)nb * slices) return;
  const uint32_t d = (uint32_t)(g / slices), s = (uint32_t)(g % slices);
  const uint32_t lo = offsets[d], hi = offsets[d + 1];
  const uint32_t len = hi - lo;
  const uint32_t a = lo + (uint32_t)((uint64_t)len * s / slices);
  const uint32_t b = lo + (uint32_t)((uint64_t)len * (s + 1) / slices);
  Xyzz acc = infinity();
  for (uint32_t k = a; k < b; ++k) acc = add_mixed(acc, load_affine(table, entries[k]));
  store_xyzz(partial, g, acc);
}

// ---------------------------------------------------------------------------
// Reduction by bits.  Level 0: lane (b, t) sums, over buckets d of chunk t
// (chunk = `chunk` consecutive bucket indices, 8: a lane adds at most 8
// buckets, the chunk's all when bit b lies above the chunk's bits) with bit
// b of d set, the S slices of those buckets; out[b * T + t].

__global__ void __launch_bounds__(128) bits_level0_kernel(const uint32_t* __restrict__ partial, uint32_t nb,
                                                          uint32_t slices, int c, uint32_t chunk,
                                                          uint32_t* __restrict__ out) {
  const uint32_t T = (nb + chunk - 1) / chunk;
  const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (uint64_t)c * T) return;
  const uint32_t b = (uint32_t)(g / T), t = (uint32_t)(g % T);
  Xyzz acc = infinity();
  const uint32_t lo = t * chunk, hi = min(nb, lo + chunk);
  for (uint32_t d = lo; d < hi; ++d) {
    if (!((d >> b) & 1u)) continue;
    for (uint32_t s = 0; s < slices; ++s) acc = add(acc, load_xyzz(partial, (uint64_t)d * slices + s));
  }
  store_xyzz(out, g, acc);
}

__global__ void __launch_bounds__(128) sum_level_kernel(const uint32_t* __restrict__ in, uint32_t groups,
                                                        uint32_t len, uint32_t chunk, uint32_t* __restrict__ out) {
  // `groups` groups of `len` partials each; out: groups x ceil(len / chunk)
  const uint32_t T = (len + chunk - 1) / chunk;
  const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (uint64_t)groups * T) return;
  const uint32_t grp = (uint32_t)(g / T), t = (uint32_t)(g % T);
  Xyzz acc = infinity();
  const uint32_t lo = t * chunk, hi = min(len, lo + chunk);
  for (uint32_t k = lo; k < hi; ++k) acc = add(acc, load_xyzz(in, (uint64_t)grp * len + k));
  store_xyzz(out, g, acc);
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

// G_b for b = blockIdx.x: the sum of `len` partials of bit b, 512 lanes each
// summing a strided share, then a tree (96 KiB of LDS).
constexpr int kReduceThreads = 512;
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
  const Xyzz total = lds_tree_sum(p, sh);
  if (threadIdx.x == 0) store_xyzz(res, 0, total);
}

__global__ void __launch_bounds__(256) zero_kernel(uint32_t* __restrict__ p, uint64_t words) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < words) p[i] = 0;
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

hipError_t launch_msm(const MsmLaunch& m, hipStream_t s) {
  const uint32_t nb = 1u << m.c;  // bucket 0 unused
  hipError_t e;
  // counts
  hipLaunchKernelGGL(zero_kernel, dim3(blocks(nb, 256)), dim3(256), 0, s, m.counts, (uint64_t)nb);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (m.n) {
    hipLaunchKernelGGL(digits_kernel, dim3(blocks(m.n, 256)), dim3(256), 0, s, m.scalars, m.n, m.c, m.windows,
                       m.digits, m.ranks, m.counts);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, m.counts, nb, m.offsets);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (m.n) {
    const uint64_t count = (uint64_t)m.windows * m.n;
    hipLaunchKernelGGL(scatter_kernel, dim3(blocks(count, 256)), dim3(256), 0, s, m.digits, m.ranks, count, m.offsets,
                       m.entries);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const uint64_t lanes = (uint64_t)nb * m.slices;
  hipLaunchKernelGGL(accumulate_kernel, dim3(blocks(lanes, 128)), dim3(128), 0, s, m.table, m.entries, m.offsets, nb,
                     m.slices, m.partial);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // each bucket's slices into one point
  hipLaunchKernelGGL(sum_level_kernel, dim3(blocks(nb, 128)), dim3(128), 0, s, m.partial, nb, m.slices, m.slices,
                     m.buckets);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // reduction by bits
  uint32_t T = (nb + m.chunk - 1) / m.chunk;
  hipLaunchKernelGGL(bits_level0_kernel, dim3(blocks((uint64_t)m.c * T, 128)), dim3(128), 0, s, m.buckets, nb, 1u,
                     m.c, m.chunk, m.level_a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // each bit's partials into G_b, then sum_b 2^b G_b
  hipLaunchKernelGGL(reduce_bit_kernel, dim3(m.c), dim3(kReduceThreads), 0, s, m.level_a, T, m.level_b);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(final_kernel, dim3(1), dim3(16), 0, s, m.level_b, m.c, m.result);
  return hipGetLastError();
}

}  // namespace msm
}  // namespace zk
