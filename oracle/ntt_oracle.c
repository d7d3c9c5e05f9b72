/*
 * CPU oracle for the NTT family and the Groth16 quotient chain.
 *
 * TEST INFRASTRUCTURE ONLY: the product library never includes, links or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do (through oracle/coracle.py).  It shares no header, table or
 * constant with the HIP library and derives every constant it uses (roots of
 * unity, coset powers, inverses, Montgomery factors) from the modulus and the
 * generator.
 *
 * What it computes (paper, Section II-B): the NTT maps a = [a_0 .. a_{n-1}]
 * to A with A_i = sum_j a_j w^(i j), w a primitive n-th root of unity,
 * computed with the radix-2 Cooley-Tukey butterfly, n/2 butterflies in each
 * of log2(n) stages (Fig. 4(b)).  The quotient chain (Section II, Fig. 3;
 * seven NTTs per proof, Section IV-A) interleaves forward and inverse
 * transforms with elementwise products.
 *
 * Arithmetic: plain residues in [0, p) held in four 64-bit limbs.  Products
 * are 512-bit schoolbook products reduced with Barrett's method (Menezes, van
 * Oorschot and Vanstone, Handbook of Applied Cryptography, Algorithm 14.42,
 * base b = 2^64, k = 4).  Montgomery form appears only at the boundary:
 * inputs y are read as y * 2^-256 mod p and outputs written as x * 2^256 mod p.
 *
 * Parallelism: each butterfly stage is split across POSIX threads; the
 * stages themselves run one after another.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

typedef struct {
  uint64_t w[4];
} fe; /* residue in [0, p), little-endian 64-bit words */

typedef struct {
  fe p;
  uint64_t mu[5]; /* floor(2^512 / p) */
  fe g;           /* multiplicative generator */
  int two_adicity;
  fe r_mod; /* 2^256 mod p */
  fe r_inv; /* 2^-256 mod p */
} field;

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -3 };

/* ------------------------------------------------------------------------ */
/* multi-word helpers                                                         */

static int geq4(const uint64_t *a, const uint64_t *b) {
  for (int i = 3; i >= 0; --i) {
    if (a[i] != b[i]) return a[i] > b[i];
  }
  return 1;
}

/* a -= b over n words; returns the borrow */
static uint64_t subn(uint64_t *a, const uint64_t *b, int n) {
  uint64_t borrow = 0;
  for (int i = 0; i < n; ++i) {
    u128 d = (u128)a[i] - b[i] - borrow;
    a[i] = (uint64_t)d;
    borrow = (uint64_t)(d >> 64) & 1u;
  }
  return borrow;
}

/* a += b over n words; returns the carry */
static uint64_t addn(uint64_t *a, const uint64_t *b, int n) {
  uint64_t carry = 0;
  for (int i = 0; i < n; ++i) {
    u128 s = (u128)a[i] + b[i] + carry;
    a[i] = (uint64_t)s;
    carry = (uint64_t)(s >> 64);
  }
  return carry;
}

/* out[0 .. na+nb) = a * b, schoolbook */
static void muln(uint64_t *out, const uint64_t *a, int na, const uint64_t *b, int nb) {
  memset(out, 0, sizeof(uint64_t) * (size_t)(na + nb));
  for (int i = 0; i < na; ++i) {
    uint64_t carry = 0;
    for (int j = 0; j < nb; ++j) {
      u128 t = (u128)a[i] * b[j] + out[i + j] + carry;
      out[i + j] = (uint64_t)t;
      carry = (uint64_t)(t >> 64);
    }
    out[i + nb] = carry;
  }
}

/* Barrett reduction of x < 2^512 (eight words) modulo p (HAC 14.42). */
static fe barrett(const field *F, const uint64_t x[8]) {
  uint64_t q2[10], r2full[10], r1[5], r2[5];
  /* q1 = floor(x / b^(k-1)) = x[3..7]; q2 = q1 * mu */
  muln(q2, x + 3, 5, F->mu, 5);
  /* q3 = floor(q2 / b^(k+1)) = q2[5..9]; r2 = q3 * p mod b^(k+1) */
  muln(r2full, q2 + 5, 5, F->p.w, 4);
  memcpy(r2, r2full, sizeof r2);
  memcpy(r1, x, sizeof r1); /* r1 = x mod b^(k+1) */
  subn(r1, r2, 5);          /* r = r1 - r2 mod b^(k+1) */
  uint64_t p5[5] = {F->p.w[0], F->p.w[1], F->p.w[2], F->p.w[3], 0};
  for (;;) {
    /* while r >= p: r -= p  (at most twice) */
    int ge = r1[4] != 0 || geq4(r1, F->p.w);
    if (!ge) break;
    subn(r1, p5, 5);
  }
  fe r;
  memcpy(r.w, r1, sizeof r.w);
  return r;
}

static fe fmul(const field *F, fe a, fe b) {
  uint64_t x[8];
  muln(x, a.w, 4, b.w, 4);
  return barrett(F, x);
}

static fe fadd(const field *F, fe a, fe b) {
  fe r = a;
  uint64_t carry = addn(r.w, b.w, 4);
  if (carry || geq4(r.w, F->p.w)) subn(r.w, F->p.w, 4);
  return r;
}

static fe fsub(const field *F, fe a, fe b) {
  fe r = a;
  if (subn(r.w, b.w, 4)) addn(r.w, F->p.w, 4);
  return r;
}

static fe fe_small(uint64_t v) {
  fe r = {{v, 0, 0, 0}};
  return r;
}

/* a^e, e given as four 64-bit words, square-and-multiply from the top bit */
static fe fpow(const field *F, fe a, const uint64_t e[4]) {
  fe r = fe_small(1);
  for (int i = 255; i >= 0; --i) {
    r = fmul(F, r, r);
    if ((e[i / 64] >> (i % 64)) & 1u) r = fmul(F, r, a);
  }
  return r;
}

static fe fpow_u64(const field *F, fe a, uint64_t e) {
  uint64_t ew[4] = {e, 0, 0, 0};
  return fpow(F, a, ew);
}

/* Fermat: a^(p-2) */
static fe finv(const field *F, fe a) {
  uint64_t e[4];
  memcpy(e, F->p.w, sizeof e);
  uint64_t two[4] = {2, 0, 0, 0};
  subn(e, two, 4);
  return fpow(F, a, e);
}

/* w_n = g^((p-1)/n), n = 2^log2n <= 2^two_adicity */
static fe root_of_unity(const field *F, int log2n) {
  uint64_t e[4];
  memcpy(e, F->p.w, sizeof e);
  e[0] -= 1; /* p is odd, no borrow */
  for (int s = 0; s < log2n; ++s) {
    for (int i = 0; i < 4; ++i) e[i] = (e[i] >> 1) | (i < 3 ? e[i + 1] << 63 : 0);
  }
  return fpow(F, F->g, e);
}

/* ------------------------------------------------------------------------ */
/* field set-up                                                               */

static void parse_hex(uint64_t w[4], const char *hex) {
  memset(w, 0, sizeof(uint64_t) * 4);
  size_t len = strlen(hex);
  for (size_t i = 0; i < len; ++i) {
    char c = hex[len - 1 - i];
    uint64_t v = (c >= '0' && c <= '9') ? (uint64_t)(c - '0') : (uint64_t)((c | 32) - 'a' + 10);
    w[i / 16] |= v << (4 * (i % 16));
  }
}

static void field_init(field *F, const char *p_hex, uint64_t generator, int two_adicity) {
  memset(F, 0, sizeof *F);
  parse_hex(F->p.w, p_hex);
  F->g = fe_small(generator);
  F->two_adicity = two_adicity;
  /* mu = floor(2^512 / p) by binary long division */
  uint64_t rem[5] = {0, 0, 0, 0, 0}, p5[5] = {F->p.w[0], F->p.w[1], F->p.w[2], F->p.w[3], 0};
  memset(F->mu, 0, sizeof F->mu);
  for (int bit = 512; bit >= 0; --bit) {
    /* rem = 2 rem + (bit of 2^512) */
    for (int i = 4; i > 0; --i) rem[i] = (rem[i] << 1) | (rem[i - 1] >> 63);
    rem[0] = (rem[0] << 1) | (bit == 512 ? 1u : 0u);
    int ge = rem[4] != 0 || geq4(rem, F->p.w);
    if (ge) {
      subn(rem, p5, 5);
      if (bit / 64 < 5) F->mu[bit / 64] |= (uint64_t)1 << (bit % 64); /* quotient < 2^260 */
    }
  }
  uint64_t x[8] = {0, 0, 0, 0, 1, 0, 0, 0}; /* 2^256 */
  F->r_mod = barrett(F, x);
  F->r_inv = finv(F, F->r_mod);
}

static field g_fields[4];
static pthread_once_t g_once = PTHREAD_ONCE_INIT;

static void fields_init(void) {
  field_init(&g_fields[1], "73eda753299d7d483339d80809a1d80553bda402fffe5bfeffffffff00000001", 7, 32);
  field_init(&g_fields[2], "30644e72e131a029b85045b68181585d2833e84879b9709143e1f593f0000001", 5, 28);
  field_init(&g_fields[3], "12ab655e9a2ca55660b44d1e5c37b00159aa76fed00000010a11800000000001", 22, 47);
}

static const field *get_field(int id) {
  pthread_once(&g_once, fields_init);
  return (id >= 1 && id <= 3) ? &g_fields[id] : NULL;
}

/* ------------------------------------------------------------------------ */
/* parallel loop                                                              */

typedef void (*range_fn)(void *ctx, size_t lo, size_t hi);
typedef struct {
  range_fn fn;
  void *ctx;
  size_t lo, hi;
} range_job;

static void *range_thread(void *arg) {
  range_job *j = (range_job *)arg;
  j->fn(j->ctx, j->lo, j->hi);
  return NULL;
}

#define MAX_THREADS 256

static void parallel_for(size_t n, int nthreads, range_fn fn, void *ctx) {
  if (nthreads > MAX_THREADS) nthreads = MAX_THREADS;
  if (nthreads <= 1 || n < 4096) {
    fn(ctx, 0, n);
    return;
  }
  pthread_t th[MAX_THREADS];
  range_job jobs[MAX_THREADS];
  int started = 0;
  for (int t = 0; t < nthreads; ++t) {
    jobs[t].fn = fn;
    jobs[t].ctx = ctx;
    jobs[t].lo = n * (size_t)t / (size_t)nthreads;
    jobs[t].hi = n * (size_t)(t + 1) / (size_t)nthreads;
    if (t == 0) continue;
    if (pthread_create(&th[t], NULL, range_thread, &jobs[t]) != 0) {
      range_thread(&jobs[t]); /* run inline if a thread cannot start */
      jobs[t].fn = NULL;
    }
    started = t;
  }
  range_thread(&jobs[0]);
  for (int t = 1; t <= started; ++t) {
    if (jobs[t].fn) pthread_join(th[t], NULL);
  }
}

/* ------------------------------------------------------------------------ */
/* boundary conversion                                                        */

static fe load_limbs(const uint32_t *y) {
  fe r;
  for (int i = 0; i < 4; ++i) r.w[i] = (uint64_t)y[2 * i] | ((uint64_t)y[2 * i + 1] << 32);
  return r;
}

static void store_limbs(uint32_t *y, fe x) {
  for (int i = 0; i < 4; ++i) {
    y[2 * i] = (uint32_t)x.w[i];
    y[2 * i + 1] = (uint32_t)(x.w[i] >> 32);
  }
}

typedef struct {
  const field *F;
  const uint32_t *in;
  uint32_t *out;
  fe *x;
} conv_ctx;

static void from_mont_range(void *c, size_t lo, size_t hi) {
  conv_ctx *k = (conv_ctx *)c;
  for (size_t i = lo; i < hi; ++i) {
    uint64_t prod[8];
    fe y = load_limbs(k->in + 8 * i);
    muln(prod, y.w, 4, k->F->r_inv.w, 4); /* y < 2^256, so the product is < 2^512 */
    k->x[i] = barrett(k->F, prod);
  }
}

static void to_mont_range(void *c, size_t lo, size_t hi) {
  conv_ctx *k = (conv_ctx *)c;
  for (size_t i = lo; i < hi; ++i) store_limbs(k->out + 8 * i, fmul(k->F, k->x[i], k->F->r_mod));
}

static void from_mont(const field *F, const uint32_t *in, fe *x, size_t n, int nt) {
  conv_ctx c = {F, in, NULL, x};
  parallel_for(n, nt, from_mont_range, &c);
}

static void to_mont(const field *F, const fe *x, uint32_t *out, size_t n, int nt) {
  conv_ctx c = {F, NULL, out, (fe *)x};
  parallel_for(n, nt, to_mont_range, &c);
}

/* ------------------------------------------------------------------------ */
/* powers and scalings                                                        */

typedef struct {
  const field *F;
  fe base;
  fe scale;
  fe *x; /* x[i] *= scale * base^i, or x[i] = base^i when mode == 1 */
  int mode;
} pow_ctx;

static void pow_range(void *c, size_t lo, size_t hi) {
  pow_ctx *k = (pow_ctx *)c;
  const field *F = k->F;
  fe cur = fmul(F, k->scale, fpow_u64(F, k->base, (uint64_t)lo));
  for (size_t i = lo; i < hi; ++i) {
    if (k->mode == 1) k->x[i] = cur;
    else k->x[i] = fmul(F, k->x[i], cur);
    cur = fmul(F, cur, k->base);
  }
}

/* x[i] *= scale * base^i */
static void scale_by_powers(const field *F, fe *x, size_t n, fe base, fe scale, int nt) {
  pow_ctx c = {F, base, scale, x, 0};
  parallel_for(n, nt, pow_range, &c);
}

/* tab[i] = base^i */
static void fill_powers(const field *F, fe *tab, size_t n, fe base, int nt) {
  pow_ctx c = {F, base, fe_small(1), tab, 1};
  parallel_for(n, nt, pow_range, &c);
}

/* ------------------------------------------------------------------------ */
/* radix-2 Cooley-Tukey                                                       */

typedef struct {
  const field *F;
  fe *x;
  const fe *tw; /* w^k, k < n/2 */
  size_t half;  /* m / 2 */
  size_t tstride; /* n / m */
} stage_ctx;

static void stage_range(void *c, size_t lo, size_t hi) {
  stage_ctx *k = (stage_ctx *)c;
  const field *F = k->F;
  for (size_t t = lo; t < hi; ++t) {
    size_t j = t % k->half;
    size_t b = (t / k->half) * 2 * k->half;
    fe u = k->x[b + j];
    fe v = fmul(F, k->tw[j * k->tstride], k->x[b + j + k->half]);
    k->x[b + j] = fadd(F, u, v);
    k->x[b + j + k->half] = fsub(F, u, v);
  }
}

static size_t bitrev(size_t i, int bits) {
  size_t r = 0;
  for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1u) << (bits - 1 - b);
  return r;
}

/* In-place NTT with root w of order n = 2^log2n, natural order in and out:
 * bit-reverse, then stages m = 2, 4, .., n with butterflies
 * (x, y) -> (x + w_m^j y, x - w_m^j y), w_m = w^(n/m). */
static int ntt_inplace(const field *F, fe *x, int log2n, fe w, int nt) {
  size_t n = (size_t)1 << log2n;
  for (size_t i = 0; i < n; ++i) {
    size_t r = bitrev(i, log2n);
    if (r > i) {
      fe t = x[i];
      x[i] = x[r];
      x[r] = t;
    }
  }
  if (n < 2) return ORC_OK;
  fe *tw = (fe *)malloc(sizeof(fe) * (n / 2));
  if (!tw) return ORC_ENOMEM;
  fill_powers(F, tw, n / 2, w, nt);
  for (int s = 1; s <= log2n; ++s) {
    size_t m = (size_t)1 << s;
    stage_ctx c = {F, x, tw, m / 2, n / m};
    parallel_for(n / 2, nt, stage_range, &c);
  }
  free(tw);
  return ORC_OK;
}

enum { K_FORWARD = 0, K_INVERSE = 1, K_COSET_FORWARD = 2, K_COSET_INVERSE = 3 };

/* Apply one of the four transforms to plain residues in place. */
static int transform_plain(const field *F, fe *x, int log2n, int kind, int nt) {
  size_t n = (size_t)1 << log2n;
  fe w = root_of_unity(F, log2n);
  fe one = fe_small(1);
  int rc;
  switch (kind) {
    case K_FORWARD:
      return ntt_inplace(F, x, log2n, w, nt);
    case K_INVERSE:
      rc = ntt_inplace(F, x, log2n, finv(F, w), nt);
      if (rc) return rc;
      scale_by_powers(F, x, n, one, finv(F, fe_small(n)), nt);
      return ORC_OK;
    case K_COSET_FORWARD:
      scale_by_powers(F, x, n, F->g, one, nt);
      return ntt_inplace(F, x, log2n, w, nt);
    case K_COSET_INVERSE:
      rc = ntt_inplace(F, x, log2n, finv(F, w), nt);
      if (rc) return rc;
      scale_by_powers(F, x, n, finv(F, F->g), finv(F, fe_small(n)), nt);
      return ORC_OK;
    default:
      return ORC_EINVAL;
  }
}

static int check_args(const field *F, int log2n) {
  if (!F) return ORC_EINVAL;
  if (log2n < 0 || log2n > F->two_adicity || log2n > 40) return ORC_EINVAL;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* exported entry points (ctypes)                                             */

/* One transform of n = 2^log2n Montgomery-form elements (8 x u32 limbs each).
 * kind: 0 forward, 1 inverse, 2 coset forward (shift g), 3 coset inverse. */
int orc_transform(int field_id, int log2n, int kind, const uint32_t *in, uint32_t *out, int nthreads) {
  const field *F = get_field(field_id);
  int rc = check_args(F, log2n);
  if (rc) return rc;
  size_t n = (size_t)1 << log2n;
  fe *x = (fe *)malloc(sizeof(fe) * n);
  if (!x) return ORC_ENOMEM;
  from_mont(F, in, x, n, nthreads);
  rc = transform_plain(F, x, log2n, kind, nthreads);
  if (!rc) to_mont(F, x, out, n, nthreads);
  free(x);
  return rc;
}

typedef struct {
  const field *F;
  fe *a, *b, *c;
  fe zinv;
} pw_ctx;

static void pointwise_range(void *k_, size_t lo, size_t hi) {
  pw_ctx *k = (pw_ctx *)k_;
  for (size_t i = lo; i < hi; ++i) {
    fe t = fsub(k->F, fmul(k->F, k->a[i], k->b[i]), k->c[i]);
    k->a[i] = fmul(k->F, t, k->zinv);
  }
}

/* Groth16 quotient chain: for X in {A, B, C}: X' = cosetNTT(INTT(X));
 * E = (A' B' - C') (g^n - 1)^-1; H = cosetINTT(E).  Montgomery in and out. */
int orc_quotient(int field_id, int log2n, const uint32_t *A, const uint32_t *B, const uint32_t *C, uint32_t *H,
                 int nthreads) {
  const field *F = get_field(field_id);
  int rc = check_args(F, log2n);
  if (rc) return rc;
  size_t n = (size_t)1 << log2n;
  fe *a = (fe *)malloc(sizeof(fe) * n), *b = (fe *)malloc(sizeof(fe) * n), *c = (fe *)malloc(sizeof(fe) * n);
  if (!a || !b || !c) {
    free(a);
    free(b);
    free(c);
    return ORC_ENOMEM;
  }
  const uint32_t *src[3] = {A, B, C};
  fe *dst[3] = {a, b, c};
  for (int v = 0; v < 3 && !rc; ++v) {
    from_mont(F, src[v], dst[v], n, nthreads);
    rc = transform_plain(F, dst[v], log2n, K_INVERSE, nthreads);
    if (!rc) rc = transform_plain(F, dst[v], log2n, K_COSET_FORWARD, nthreads);
  }
  if (!rc) {
    fe zh = fsub(F, fpow_u64(F, F->g, (uint64_t)n), fe_small(1)); /* Z_H on the coset: g^n - 1 */
    pw_ctx k = {F, a, b, c, finv(F, zh)};
    parallel_for(n, nthreads, pointwise_range, &k);
    rc = transform_plain(F, a, log2n, K_COSET_INVERSE, nthreads);
  }
  if (!rc) to_mont(F, a, H, n, nthreads);
  free(a);
  free(b);
  free(c);
  return rc;
}

typedef struct {
  const field *F;
  const fe *coeffs;
  size_t n;
  const fe *pts;
  fe *vals;
} horner_ctx;

static void horner_range(void *k_, size_t lo, size_t hi) {
  horner_ctx *k = (horner_ctx *)k_;
  for (size_t q = lo; q < hi; ++q) {
    fe acc = fe_small(0);
    for (size_t j = k->n; j-- > 0;) acc = fadd(k->F, fmul(k->F, acc, k->pts[q]), k->coeffs[j]);
    k->vals[q] = acc;
  }
}

/* vals[q] = sum_j coeffs[j] w^(idx[q] j) by Horner's rule, w the n-th root;
 * coefficients and values in Montgomery form.  Independent of any NTT code. */
int orc_eval_at_roots(int field_id, int log2n, const uint32_t *coeffs, const uint64_t *idx, int count,
                      uint32_t *vals, int nthreads) {
  const field *F = get_field(field_id);
  int rc = check_args(F, log2n);
  if (rc) return rc;
  if (count < 0) return ORC_EINVAL;
  size_t n = (size_t)1 << log2n;
  fe *x = (fe *)malloc(sizeof(fe) * n);
  fe *pts = (fe *)malloc(sizeof(fe) * (size_t)(count + 1));
  fe *out = (fe *)malloc(sizeof(fe) * (size_t)(count + 1));
  if (!x || !pts || !out) {
    free(x);
    free(pts);
    free(out);
    return ORC_ENOMEM;
  }
  from_mont(F, coeffs, x, n, nthreads);
  fe w = root_of_unity(F, log2n);
  for (int q = 0; q < count; ++q) pts[q] = fpow_u64(F, w, idx[q] % n);
  horner_ctx k = {F, x, n, pts, out};
  /* parallel over points: one point per slot */
  if (nthreads > 1 && count > 1) {
    pthread_t th[MAX_THREADS];
    range_job jobs[MAX_THREADS];
    int nt = nthreads < count ? nthreads : count;
    if (nt > MAX_THREADS) nt = MAX_THREADS;
    int ok[MAX_THREADS];
    for (int t = 0; t < nt; ++t) {
      jobs[t].fn = horner_range;
      jobs[t].ctx = &k;
      jobs[t].lo = (size_t)count * (size_t)t / (size_t)nt;
      jobs[t].hi = (size_t)count * (size_t)(t + 1) / (size_t)nt;
      ok[t] = pthread_create(&th[t], NULL, range_thread, &jobs[t]) == 0;
      if (!ok[t]) range_thread(&jobs[t]);
    }
    for (int t = 0; t < nt; ++t)
      if (ok[t]) pthread_join(th[t], NULL);
  } else {
    horner_range(&k, 0, (size_t)count);
  }
  to_mont(F, out, vals, (size_t)count, 1);
  free(x);
  free(pts);
  free(out);
  return ORC_OK;
}

/* Elementwise field operations on plain residues (8 x u32 limbs), for
 * checking this file's arithmetic against Python integers.
 * op: 0 add, 1 sub, 2 mul, 3 inverse of a, 4 a^e with e = b (as integer). */
int orc_field_op(int field_id, int op, const uint32_t *a, const uint32_t *b, uint32_t *out, int count) {
  const field *F = get_field(field_id);
  if (!F || count < 0) return ORC_EINVAL;
  for (int i = 0; i < count; ++i) {
    fe x = load_limbs(a + 8 * i), y = load_limbs(b + 8 * i), r;
    switch (op) {
      case 0: r = fadd(F, x, y); break;
      case 1: r = fsub(F, x, y); break;
      case 2: r = fmul(F, x, y); break;
      case 3: r = finv(F, x); break;
      case 4: r = fpow(F, x, y.w); break;
      default: return ORC_EINVAL;
    }
    store_limbs(out + 8 * i, r);
  }
  return ORC_OK;
}

/* The oracle's own constants, for the pins: which = 0 modulus, 1 mu (five
 * words, 40 bytes), 2 2^256 mod p, 3 root of order 2^log2n. */
int orc_constant(int field_id, int which, int log2n, uint32_t *out) {
  const field *F = get_field(field_id);
  if (!F) return ORC_EINVAL;
  switch (which) {
    case 0: store_limbs(out, F->p); return ORC_OK;
    case 1:
      for (int i = 0; i < 5; ++i) {
        out[2 * i] = (uint32_t)F->mu[i];
        out[2 * i + 1] = (uint32_t)(F->mu[i] >> 32);
      }
      return ORC_OK;
    case 2: store_limbs(out, F->r_mod); return ORC_OK;
    case 3: /* any order up to the 2-adicity: no vector of that size is made */
      if (log2n < 0 || log2n > F->two_adicity) return ORC_EINVAL;
      store_limbs(out, root_of_unity(F, log2n));
      return ORC_OK;
    default: return ORC_EINVAL;
  }
}
