/*
 * Driver for running the C oracle (oracle/ntt_oracle.c) under host
 * sanitizers (AddressSanitizer + UndefinedBehaviorSanitizer, or
 * ThreadSanitizer): transforms, round trips, the quotient chain, Horner
 * evaluations and field operations over the three fields, at sizes below
 * and above the point where the oracle splits stages over threads, with 1, 3
 * and 8 threads.  Exit status 0 when every round trip and consistency check
 * holds; the sanitizers abort on any memory error, data race or undefined
 * behaviour they see.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_transform(int field_id, int log2n, int kind, const uint32_t *in, uint32_t *out, int nthreads);
int orc_quotient(int field_id, int log2n, const uint32_t *A, const uint32_t *B, const uint32_t *C, uint32_t *H,
                 int nthreads);
int orc_eval_at_roots(int field_id, int log2n, const uint32_t *coeffs, const uint64_t *idx, int count,
                      uint32_t *vals, int nthreads);
int orc_field_op(int field_id, int op, const uint32_t *a, const uint32_t *b, uint32_t *out, int count);

/* small canonical inputs: limb 0 only, so every value is below every modulus */
static void fill(uint32_t *x, size_t n, uint32_t seed) {
  uint64_t s = seed * 0x9e3779b97f4a7c15ull + 1;
  memset(x, 0, n * 32);
  for (size_t i = 0; i < n; ++i) {
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    x[8 * i] = (uint32_t)(s >> 33);
    x[8 * i + 1] = (uint32_t)(s >> 7) & 0xffffu;
  }
}

static int check(int cond, const char *what, int field, int log2n, int nt) {
  if (!cond) fprintf(stderr, "FAIL %s field %d 2^%d threads %d\n", what, field, log2n, nt);
  return cond ? 0 : 1;
}

int main(void) {
  int bad = 0;
  const int threads[3] = {1, 3, 8};
  for (int field = 1; field <= 3; ++field) {
    for (int log2n = 0; log2n <= 14; log2n += (log2n < 12 ? 3 : 1)) {
      const size_t n = (size_t)1 << log2n;
      uint32_t *x = malloc(n * 32), *y = malloc(n * 32), *z = malloc(n * 32), *ref = malloc(n * 32);
      fill(x, n, (uint32_t)(field * 100 + log2n));
      for (int t = 0; t < 3; ++t) {
        const int nt = threads[t];
        bad += check(orc_transform(field, log2n, 0, x, y, nt) == 0, "forward", field, log2n, nt);
        if (t == 0) memcpy(ref, y, n * 32);
        bad += check(memcmp(ref, y, n * 32) == 0, "thread count changes the result", field, log2n, nt);
        bad += check(orc_transform(field, log2n, 1, y, z, nt) == 0, "inverse", field, log2n, nt);
        bad += check(memcmp(x, z, n * 32) == 0, "inverse round trip", field, log2n, nt);
        bad += check(orc_transform(field, log2n, 2, x, y, nt) == 0, "coset forward", field, log2n, nt);
        bad += check(orc_transform(field, log2n, 3, y, z, nt) == 0, "coset inverse", field, log2n, nt);
        bad += check(memcmp(x, z, n * 32) == 0, "coset round trip", field, log2n, nt);
      }
      if (log2n <= 13) {
        uint32_t *B = malloc(n * 32), *C = malloc(n * 32);
        fill(B, n, 7);
        fill(C, n, 8);
        bad += check(orc_quotient(field, log2n, x, B, C, y, 3) == 0, "quotient", field, log2n, 3);
        bad += check(orc_quotient(field, log2n, x, B, C, z, 8) == 0, "quotient", field, log2n, 8);
        bad += check(memcmp(y, z, n * 32) == 0, "quotient thread counts", field, log2n, 8);
        free(B);
        free(C);
      }
      /* Horner evaluations at roots equal the forward transform's entries */
      uint64_t idx[4] = {0, n > 1 ? 1 : 0, n / 2, n - 1};
      uint32_t vals[4 * 8];
      bad += check(orc_transform(field, log2n, 0, x, y, 8) == 0, "forward", field, log2n, 8);
      bad += check(orc_eval_at_roots(field, log2n, x, idx, 4, vals, 3) == 0, "horner", field, log2n, 3);
      for (int k = 0; k < 4; ++k) bad += check(memcmp(vals + 8 * k, y + 8 * idx[k], 32) == 0, "horner value", field, log2n, 3);
      /* field operations: (a + b) - b = a, a * 1 (Montgomery one from add) */
      uint32_t *s = malloc(n * 32);
      bad += check(orc_field_op(field, 0, x, z, s, (int)n) == 0, "add", field, log2n, 1);
      bad += check(orc_field_op(field, 1, s, z, y, (int)n) == 0, "sub", field, log2n, 1);
      bad += check(memcmp(x, y, n * 32) == 0, "add then sub", field, log2n, 1);
      bad += check(orc_field_op(field, 2, x, z, s, (int)n) == 0, "mul", field, log2n, 1);
      free(s);
      free(x);
      free(y);
      free(z);
      free(ref);
    }
  }
  /* argument checks */
  uint32_t one[8] = {1};
  bad += check(orc_transform(2, 29, 0, one, one, 1) != 0, "size beyond 2-adicity refused", 2, 29, 1);
  bad += check(orc_transform(9, 2, 0, one, one, 1) != 0, "unknown field refused", 9, 2, 1);
  printf(bad ? "oracle sanitizer driver: %d failures\n" : "oracle sanitizer driver: ok\n", bad);
  return bad ? 1 : 0;
}
