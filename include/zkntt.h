/*
 * zkntt: Number-Theoretic Transforms and the Groth16 quotient chain over
 * 255-bit scalar fields, on AMD Instinct MI355X (gfx950).
 *
 * What the calls compute (ZKProphet, arXiv 2509.22684):
 *   - The NTT maps a vector a = [a_0 .. a_{n-1}] of field elements to A with
 *     A_i = sum_j a_j w^(i j), w a primitive n-th root of unity; the inverse
 *     transform (INTT) undoes it (Section II-C, "Number-Theoretic Transform").
 *   - The Groth16 prover derives the quotient polynomial h from the witness
 *     polynomials with forward and inverse NTTs interleaved with elementwise
 *     operations (Section II-A and Fig. 2); a proof runs seven NTTs
 *     (Section IV-A).
 *
 * Conventions fixed by this library where the paper leaves a choice open:
 *   - n = 2^log2n, 0 <= log2n <= 2-adicity of the field (32 for BLS12-381 Fr,
 *     28 for BN254 Fr).  n = 1 is the identity transform.
 *   - w_n = g^((p-1)/n) with g the smallest multiplicative generator
 *     (g = 7 for BLS12-381 Fr, g = 5 for BN254 Fr).
 *   - Natural order in and out for every call.
 *   - Coset transforms evaluate on g * <w_n>: coefficient j is multiplied by
 *     g^j before the forward transform (and by g^-j after the inverse one).
 *
 * Data layout (every vector argument):
 *   - n elements, element i at bytes [32 i, 32 i + 32) of the buffer.
 *   - An element is eight 32-bit limbs, little-endian (limb 0 least
 *     significant), holding the Montgomery form x * 2^256 mod p of the value
 *     x, canonical in [0, p).  Outputs are canonical.  Inputs outside [0, p)
 *     are a caller error; with ZK_FLAG_VALIDATE the call checks them.
 *   - Buffers are device memory (hipMalloc or equivalent), 256-byte aligned;
 *     a misaligned pointer returns ZK_EINVAL.
 *
 * Ownership and concurrency:
 *   - The caller owns every buffer passed in.  A plan owns its device tables
 *     (twiddles, coset powers) and frees them in ntt_plan_destroy.
 *   - A plan is immutable after ntt_plan_create; calls on one plan may run
 *     concurrently on different streams when each has its own workspace.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     All calls are asynchronous on that stream; errors during kernel
 *     execution surface at the caller's synchronisation.
 *
 * Errors: every call returns a zk_status; nothing aborts and no exception
 * crosses this interface.  zk_last_error() returns a message for the
 * calling thread's most recent failure.
 */
#ifndef ZKNTT_H
#define ZKNTT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ntt_plan ntt_plan;

typedef enum { ZK_FIELD_BLS12_381_FR = 1, ZK_FIELD_BN254_FR = 2 } zk_field;

typedef enum {
  ZK_OK = 0,
  ZK_EINVAL = -1,       /* bad argument: null/misaligned pointer, non-canonical input */
  ZK_EUNSUPPORTED = -2, /* size beyond the field's 2-adicity, unknown field or option */
  ZK_ENOMEM = -3,       /* a device allocation failed */
  ZK_EDEVICE = -4       /* a HIP runtime call or kernel launch failed */
} zk_status;

/* Plan options.  Zero in any field selects the tuned default. */
typedef struct {
  uint32_t twiddle_mode; /* 0 default, 1 precomputed tables in HBM */
  uint32_t log2_radix;   /* radix of the in-register butterflies: 0 default, 1 (radix-2), 2, 3 */
  uint32_t log2_tile;    /* elements per workgroup tile, log2: 0 default (11), 8..11 */
  uint32_t flags;        /* ZK_FLAG_* */
} ntt_plan_opts;

#define ZK_FLAG_VALIDATE 1u /* check that inputs are canonical (adds a device-to-host sync) */

/* Create a plan for n = 2^log2n transforms over `field` on the current HIP
 * device: derives the root of unity and builds its twiddle and coset tables
 * in device memory.  opts may be NULL.  On success *out owns the plan. */
int ntt_plan_create(ntt_plan **out, int field, uint32_t log2n, const ntt_plan_opts *opts);
void ntt_plan_destroy(ntt_plan *p);

/* Bytes of device workspace ntt_* calls on this plan need (0: none). */
size_t ntt_workspace_bytes(const ntt_plan *p);
/* Bytes of device memory held by the plan's tables. */
size_t ntt_plan_device_bytes(const ntt_plan *p);
/* Number of global passes (kernel launches) one transform takes. */
int ntt_plan_passes(const ntt_plan *p);

/* Forward NTT: out_i = sum_j in_j w^(i j)  (Section II-C).
 * d_in may equal d_out.  d_work: ntt_workspace_bytes(p) bytes, or NULL when
 * that is 0; it must not overlap d_in or d_out. */
int ntt_forward(const ntt_plan *p, const void *d_in, void *d_out, void *d_work, void *stream);

/* Inverse NTT: out_j = n^-1 sum_i in_i w^(-i j).  Same buffer rules. */
int ntt_inverse(const ntt_plan *p, const void *d_in, void *d_out, void *d_work, void *stream);

/* Coset forward NTT: out_i = sum_j in_j (g w^i)^j, the evaluations of the
 * polynomial with coefficients in_j on the coset g<w>. */
int ntt_coset_forward(const ntt_plan *p, const void *d_in, void *d_out, void *d_work, void *stream);

/* Coset inverse NTT: coefficients from evaluations on g<w>:
 * out_j = g^-j n^-1 sum_i in_i w^(-i j). */
int ntt_coset_inverse(const ntt_plan *p, const void *d_in, void *d_out, void *d_work, void *stream);

/* Bytes of device workspace quotient_poly needs. */
size_t quotient_workspace_bytes(const ntt_plan *p);

/* Groth16 quotient chain (Section II-A, Fig. 2; seven NTTs, Section IV-A).
 * A, B, C are evaluations on <w> (natural order).  With a, b, c their
 * interpolating polynomials, computes on the coset g<w>
 *   E_i = (a(g w^i) b(g w^i) - c(g w^i)) / (g^n - 1)
 * (Z_H(x) = x^n - 1 takes the constant value g^n - 1 on the coset) and
 * returns in H the n coefficients of the polynomial with those coset values:
 *   H = cosetINTT( (cosetNTT(INTT A) . cosetNTT(INTT B) - cosetNTT(INTT C)) / (g^n - 1) ).
 * A, B, C are not modified; H must not overlap them or d_work. */
int quotient_poly(const ntt_plan *p, const void *d_A, const void *d_B, const void *d_C, void *d_H,
                  void *d_work, void *stream);

/* Measurement helper: run one transform (kind 0 forward, 1 inverse, 2 coset
 * forward, 3 coset inverse; same buffer rules as the calls above) with a HIP
 * event recorded on `stream` before each pass and after the last, wait for
 * it, and store each pass's duration in ms_per_pass[0 .. passes).  Returns
 * the number of passes (> 0) or a zk_status.  Synchronises the stream. */
int ntt_profile_passes(const ntt_plan *p, int kind, const void *d_in, void *d_out, void *d_work, void *stream,
                       float *ms_per_pass, int max_passes);

/* Thread-local description of the calling thread's last failure. */
const char *zk_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ZKNTT_H */
