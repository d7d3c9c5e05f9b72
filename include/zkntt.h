/*
 * zkntt: Number-Theoretic Transforms and the Groth16 quotient chain over
 * 253- to 255-bit scalar fields (BLS12-381 Fr, BN254 Fr and BLS12-377 Fr, the
 * curve of the paper's other workloads), on AMD Instinct MI355X (gfx950).
 *
 * What the calls compute (ZKProphet, arXiv 2509.22684):
 *   - The NTT maps a vector a = [a_0 .. a_{n-1}] of field elements to A with
 *     A_i = sum_j a_j w^(i j), w a primitive n-th root of unity; the inverse
 *     transform (INTT) undoes it (Section II-B, "Number-Theoretic Transform").
 *   - The Groth16 prover derives the quotient polynomial h from the witness
 *     polynomials with forward and inverse NTTs interleaved with elementwise
 *     operations (Section II and Fig. 3); a proof runs seven NTTs
 *     (Section IV-A).
 *
 * Conventions fixed by this library where the paper leaves a choice open:
 *   - n = 2^log2n, 0 <= log2n <= 2-adicity of the field (32 for BLS12-381 Fr,
 *     28 for BN254 Fr, 47 for BLS12-377 Fr).  n = 1 is the identity transform.
 *   - w_n = g^((p-1)/n) with g the smallest multiplicative generator
 *     (g = 7 for BLS12-381 Fr, g = 5 for BN254 Fr, g = 22 for BLS12-377 Fr).
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

typedef enum { ZK_FIELD_BLS12_381_FR = 1, ZK_FIELD_BN254_FR = 2, ZK_FIELD_BLS12_377_FR = 3 } zk_field;

typedef enum {
  ZK_OK = 0,
  ZK_EINVAL = -1,       /* bad argument: null/misaligned pointer, non-canonical input */
  ZK_EUNSUPPORTED = -2, /* size beyond the field's 2-adicity, unknown field or option */
  ZK_ENOMEM = -3,       /* a device allocation failed */
  ZK_EDEVICE = -4       /* a HIP runtime call or kernel launch failed */
} zk_status;

/* Plan options.  Zero in any schedule field selects the tuned schedule
 * registered for (field, log2n) with ntt_tuning_register (the autotuner's
 * measurements; the Python binding registers its database before it creates
 * a plan), else the built-in default noted beside the field.  Every schedule
 * computes the same bytes. */
typedef struct {
  uint32_t twiddle_mode;    /* 0 default; 1 one precomputed table per pass in HBM;
                               2 two small tables and one extra multiplication per element */
  uint32_t log2_radix;      /* radix of the in-register butterflies: 0 default (1, radix-2, up to
                               n = 2^18; 2 above), 1 (radix-2), 2 or 3 */
  uint32_t log2_tile;       /* elements per workgroup tile of a multi-pass transform, log2:
                               0 default (8 for radix-2 transforms of n = 2^10 .. 2^16,
                               else 10); 8 (small transforms over more CUs; register
                               radix 2 or 4 only, passes of at most 2^7 points); 10; or
                               11 (twice the LDS, half the workgroups per CU) */
  uint32_t flags;           /* ZK_FLAG_* */
  uint32_t log2_pass_radix; /* most butterfly stages fused into one global pass: 0 default (9 up to
                               n = 2^18, so at most two passes there; 8 above), 4..9 */
} ntt_plan_opts;

#define ZK_FLAG_VALIDATE 1u /* check that inputs are canonical (adds a device-to-host sync, so calls on a
                               stream that is being captured into a graph return ZK_EINVAL) */
#define ZK_FLAG_FFMUL_FP64 2u /* every product of the transforms on the FP64 units (v_fma_f64, 48-bit
                                 limbs, error-free product transformations) instead of v_mad_u64_u32:
                                 the paper's open question of using the floating-point pipes for FF_mul
                                 (Sections IV-B, V-C).  Same bytes.  BLS12-381 Fr, radix-4 register
                                 rounds, ntt_forward / ntt_inverse / ntt_coset_* only (the quotient
                                 calls and batches return ZK_EUNSUPPORTED on such a plan). */

/* Create a plan for n = 2^log2n transforms over `field` on the current HIP
 * device: derives the root of unity and builds its twiddle and coset tables
 * in device memory.  opts may be NULL.  On success *out owns the plan. */
int ntt_plan_create(ntt_plan **out, int field, uint32_t log2n, const ntt_plan_opts *opts);
void ntt_plan_destroy(ntt_plan *p);

/* Tuned schedules (Section V-A of the paper asks that such launch parameters
 * be adapted to the GPU rather than picked by hand).  ntt_tuning_register
 * records the schedule the autotuner measured fastest for (field, log2n) in
 * a process-wide table; later ntt_plan_create calls fill each zero option
 * field from it.  opts->flags must be 0.  Thread-safe; host only (no device
 * call).  ntt_tuning_clear empties the table. */
int ntt_tuning_register(int field, uint32_t log2n, const ntt_plan_opts *opts);
void ntt_tuning_clear(void);
/* The schedule ntt_plan_create would use for these arguments (zero fields
 * resolved), without creating a plan: host only, no device needed.  opts may
 * be NULL.  Same errors as ntt_plan_create's argument checks. */
int ntt_plan_resolve_opts(int field, uint32_t log2n, const ntt_plan_opts *opts, ntt_plan_opts *resolved);
/* The resolved schedule of an existing plan. */
int ntt_plan_get_opts(const ntt_plan *p, ntt_plan_opts *out);
/* Bytes of device tables ntt_plan_create would allocate for these
 * arguments (what ntt_plan_device_bytes reports for the plan), computed on
 * the host without creating the plan or touching the device; 0 if the
 * arguments are unsupported (zk_last_error says why).  For admission
 * control: a caller can budget a plan before it exists. */
size_t ntt_plan_table_bytes(int field, uint32_t log2n, const ntt_plan_opts *opts);

/* Bytes of device workspace ntt_* calls on this plan need (0: none). */
size_t ntt_workspace_bytes(const ntt_plan *p);
/* Bytes of device memory held by the plan's tables. */
size_t ntt_plan_device_bytes(const ntt_plan *p);
/* Number of global passes (kernel launches) one transform takes. */
int ntt_plan_passes(const ntt_plan *p);

/* Forward NTT: out_i = sum_j in_j w^(i j)  (Section II-B).
 * d_in may equal d_out; otherwise they must not overlap.  d_work:
 * ntt_workspace_bytes(p) bytes, or NULL when that is 0; it must not overlap
 * d_in or d_out (ZK_EINVAL; the byte ranges are compared). */
int ntt_forward(const ntt_plan *p, const void *d_in, void *d_out, void *d_work, void *stream);

/* ntt_forward without a workspace argument and without any allocation, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  The library keeps
 * a fixed workspace of 2^20 elements (32 MiB) per device for it, held until
 * the process ends; plans whose ntt_workspace_bytes exceeds that (n > 2^20)
 * return ZK_EUNSUPPORTED.  Same result and buffer rules as ntt_forward.
 * Every call on one device shares that workspace and leaves its contents
 * behind: calls that may overlap in time on one device (different streams,
 * or threads enqueuing without ordering) race and must be serialised by the
 * caller. */
int ntt_forward_noalloc(const ntt_plan *p, const void *d_in, void *d_out, void *stream);

/* Inverse NTT: out_j = n^-1 sum_i in_i w^(-i j).  Same buffer rules. */
int ntt_inverse(const ntt_plan *p, const void *d_in, void *d_out, void *d_work, void *stream);

/* Coset forward NTT: out_i = sum_j in_j (g w^i)^j, the evaluations of the
 * polynomial with coefficients in_j on the coset g<w>. */
int ntt_coset_forward(const ntt_plan *p, const void *d_in, void *d_out, void *d_work, void *stream);

/* Coset inverse NTT: coefficients from evaluations on g<w>:
 * out_j = g^-j n^-1 sum_i in_i w^(-i j). */
int ntt_coset_inverse(const ntt_plan *p, const void *d_in, void *d_out, void *d_work, void *stream);

/* Bytes of device workspace quotient_poly needs (up to n = 2^22 it holds
 * three transform workspaces, so that A's and B's transforms can run at the
 * same time as C's). */
size_t quotient_workspace_bytes(const ntt_plan *p);

/* Groth16 quotient chain (Section II, Fig. 3; seven NTTs, Section IV-A).
 * A, B, C are evaluations on <w> (natural order).  With a, b, c their
 * interpolating polynomials, computes on the coset g<w>
 *   E_i = (a(g w^i) b(g w^i) - c(g w^i)) / (g^n - 1)
 * (Z_H(x) = x^n - 1 takes the constant value g^n - 1 on the coset) and
 * returns in H the n coefficients of the polynomial with those coset values:
 *   H = cosetINTT( (cosetNTT(INTT A) . cosetNTT(INTT B) - cosetNTT(INTT C)) / (g^n - 1) ).
 * A, B, C are not modified; H must not overlap them or d_work, and d_work
 * must not overlap A, B or C (ZK_EINVAL; the byte ranges are compared).
 * Up to n = 2^22 the transforms of A and B run on two streams of the plan,
 * forked from `stream` and joined back into it before C's forward NTT, so
 * the call still completes in the order of `stream`; calls on one plan from
 * several threads are serialised while they enqueue. */
int quotient_poly(const ntt_plan *p, const void *d_A, const void *d_B, const void *d_C, void *d_H,
                  void *d_work, void *stream);

/* The stages of quotient_poly, for callers that interleave them with other
 * work (e.g. start on A while B and C are still being copied to the device):
 * quotient_poly(A, B, C, H) equals, byte for byte,
 *   quotient_coset_evals(A -> T1); quotient_coset_evals(B -> T2);
 *   quotient_coset_evals(C -> T3); quotient_pointwise(T1, T2, T3 -> H);
 *   ntt_coset_inverse(H -> H).
 *
 * quotient_coset_evals: out = cosetNTT(INTT(in)), the values on g<w> of the
 * polynomial that takes the values `in` on <w> (the INTT runs without its
 * 1/n, and the forward NTT multiplies coefficient j by g^j / n as its first
 * pass loads it).  in may equal out; d_work as for ntt_forward.
 * quotient_pointwise: out_i = (A_i B_i - C_i) / (g^n - 1) for i < n, each
 * element read before it is written, so out may equal any input. */
int quotient_coset_evals(const ntt_plan *p, const void *d_in, void *d_out, void *d_work, void *stream);
int quotient_pointwise(const ntt_plan *p, const void *d_A, const void *d_B, const void *d_C, void *d_out,
                       void *stream);

/* Copy `bytes` (a multiple of 16; both pointers 16-byte aligned) from device
 * memory to pinned host memory (hipHostMalloc) with a kernel, asynchronously
 * on `stream`.  For host-resident jobs whose GPU work moves data both ways
 * (the paper finds transfers exceed the NTT itself, Section IV-A): a DMA
 * upload and this download keep both directions of the link busy at once,
 * where two DMA copies in opposite directions measured as one after the
 * other.  ZK_EINVAL if host_dst is not pinned, mapped host memory or dev_src
 * is not device memory. */
int zk_copy_to_host(void *host_dst, const void *dev_src, size_t bytes, void *stream);

/* ------------------------------------------------------------------------
 * Batches: many independent forward NTTs of uneven sizes and any field in
 * one persistent launch.  GPU NTTs run as short, bursty kernels with launch
 * shapes that fit some sizes badly (Section IV-A; Section V-A asks for
 * autotuning of such parameters); a batch deals its jobs' tiles into work
 * queues (pass-major within a queue) that a grid of persistent workgroups
 * drains.  Each queue is claimed by one XCD, so all tiles of a job run under
 * one L2.  Transforms of equal plans (field, size, schedule) and kind form
 * groups; a group whose tiles fill the chip, or whose jobs would be the
 * critical path on one XCD, runs instead as grouped pass launches (one
 * launch per pass for all jobs of the group) over the whole chip; the choice
 * follows a time estimate made when the batch is created.  A pointwise job
 * larger than an eighth of the batch runs as its own launch the same way.
 * Such launches go to up to three side streams of the batch, forked from the
 * launch stream before the persistent kernel and joined into it after (in
 * the graph: parallel branches), so the call still completes in stream
 * order on the stream it was given.
 * Every tile is computed exactly as in the stand-alone transform, so results
 * are byte-identical to ntt_forward.
 *
 * Jobs need n >= 4 and at most 4 global passes (ZK_EUNSUPPORTED otherwise);
 * the batch computes every tile with its own radix-4 register schedule,
 * whatever register radix the plan uses (the bytes are the same).
 * The batch binds the plans, buffers and workspace it was created with: they
 * must stay valid until ntt_batch_destroy.  Launches of one batch
 * must not overlap (they share the batch's queue counters).
 * ------------------------------------------------------------------------ */
typedef struct ntt_batch ntt_batch;

/* Bytes of device workspace for a batch of these plans (ping-pong buffers of
 * the multi-pass jobs). */
size_t ntt_batch_workspace_bytes(const ntt_plan *const *plans, int njobs);

/* Build the device work list for jobs k < njobs (forward NTT of d_bufs[k] in
 * place with plans[k]) and capture its launch (a counter-reset kernel and the
 * persistent kernel) into a HIP graph.  Synchronous. */
int ntt_batch_create(ntt_batch **out, const ntt_plan *const *plans, void *const *d_bufs, int njobs,
                     void *d_work);

/* General batches: each job is one transform of any kind, or the pointwise
 * step of the quotient chain.  Transform jobs follow the buffer rules of the
 * single calls (in may equal out; work: ntt_workspace_bytes(plan) bytes of
 * its own, distinct from in/out and from every other job's work).  Jobs run
 * concurrently: no job may write a buffer another job of the same batch
 * reads or writes. */
typedef enum {
  ZK_OP_FORWARD = 0,
  ZK_OP_INVERSE = 1,
  ZK_OP_COSET_FORWARD = 2,
  ZK_OP_COSET_INVERSE = 3,
  ZK_OP_INVERSE_TO_COSET = 4,     /* INTT then coefficient j times g^j: a coset NTT's input */
  ZK_OP_QUOTIENT_POINTWISE = 5    /* out_i = (in_i in2_i - in3_i) / (g^n - 1); out may equal in3 */
} zk_op;

typedef struct {
  const ntt_plan *plan; /* field and size (pointwise: n and g) */
  int32_t op;           /* zk_op */
  int32_t reserved;
  const void *in;
  const void *in2;      /* pointwise only */
  const void *in3;      /* pointwise only */
  void *out;
  void *work;           /* transform workspace, or NULL when the plan needs none */
} ntt_batch_job;

#define ZK_BATCH_GRAPH 1 /* capture the launch into a HIP graph (ntt_batch_launch) */
/* Every job as pass launches (transforms of equal plans grouped, pointwise
 * steps on their own): no persistent kernel, whose large workgroups can wait
 * long for room on CUs that other streams' pass kernels keep filling. */
#define ZK_BATCH_DIRECT 2
/* Work queues per field, 1..32 (0: 16).  Jobs are dealt largest first to the
 * least-loaded queue and each queue runs on one XCD: more queues balance the
 * XCDs more finely, fewer put more independent jobs in each queue so that a
 * tile waiting on its job's previous pass is rarer. */
#define ZK_BATCH_QUEUES_SHIFT 8
#define ZK_BATCH_QUEUES_MASK (0x3f << ZK_BATCH_QUEUES_SHIFT)
#define ZK_BATCH_QUEUES(q) ((int)(q) << ZK_BATCH_QUEUES_SHIFT)

/* Without ZK_BATCH_GRAPH the call does not wait for the device: the work
 * list stays in pinned host memory and is uploaded on the stream of the
 * first ntt_batch_launch_eager.  With it, the work list is uploaded and the
 * graph captured before the call returns. */
int ntt_batch_create_jobs(ntt_batch **out, const ntt_batch_job *jobs, int njobs, int flags);

/* Replay the batch's graph on `stream`: one persistent launch runs all jobs. */
int ntt_batch_launch(const ntt_batch *b, void *stream);

/* The same two kernels launched directly on `stream`, without the graph
 * (after the work list's upload on its first call; each call also copies
 * the batch's error word to host memory on `stream`). */
int ntt_batch_launch_eager(const ntt_batch *b, void *stream);

/* After the stream of the last launch has been synchronised: ZK_OK, or
 * ZK_EDEVICE if a dependency wait exceeded its poll limit (the kernel then
 * stops early) or the launch ended with items not run; the outputs are then
 * invalid.  After an eager launch this reads host memory only; after a graph
 * launch it copies the error word synchronously. */
int ntt_batch_status(const ntt_batch *b);

/* Poll limit of one dependency wait (default 2^22).  0 makes every
 * dependency wait fail at once (a test hook for the error path).  Synchronous
 * once the work list is on the device; before an eager batch's first launch
 * it only updates the pending host copy. */
int ntt_batch_set_spin_limit(ntt_batch *b, uint32_t polls);

/* Work items (tiles) the persistent kernel drains (jobs run as grouped or
 * direct launches are not counted) and persistent workgroups per launch. */
int ntt_batch_items(const ntt_batch *b);
int ntt_batch_grid(const ntt_batch *b);

/* Frees the batch.  Its device descriptors go back to a per-process pool
 * of the library (hipFree would wait for the whole device); a later batch
 * reuses them only after the last launch of this one has completed, so a
 * batch may be destroyed while its launch is still running. */
void ntt_batch_destroy(ntt_batch *b);

/* One-shot: build, launch without a graph, synchronise `stream`, check the
 * status and free the batch. */
int ntt_batch_forward(const ntt_plan *const *plans, void *const *d_bufs, int njobs, void *d_work, void *stream);

/* Measurement helper: run one transform (kind 0 forward, 1 inverse, 2 coset
 * forward, 3 coset inverse; same buffer rules as the calls above) with a HIP
 * event recorded on `stream` before each pass and after the last, wait for
 * it, and store each pass's duration in ms_per_pass[0 .. passes).  Returns
 * the number of passes (> 0) or a zk_status.  Synchronises the stream. */
int ntt_profile_passes(const ntt_plan *p, int kind, const void *d_in, void *d_out, void *d_work, void *stream,
                       float *ms_per_pass, int max_passes);

/* ------------------------------------------------------------------------
 * Multi-scalar multiplication on BLS12-381 G1: Q = sum_i s_i P_i, the
 * paper's other dominant proving kernel (Section II-A, Fig. 4(a); Table V
 * counts its point operations).  Pippenger's bucket method with XYZZ
 * accumulators, over fixed bases (the proving key's points) whose per-window
 * multiples are precomputed once.
 *
 * Layouts (device memory, 256-byte aligned):
 *   - a point: 24 32-bit limbs, x then y, each 12 little-endian limbs of the
 *     Montgomery form v 2^384 mod q (q the 381-bit base field prime), affine,
 *     canonical; the bases must lie in the order-r subgroup (r the BLS12-381
 *     scalar field modulus), not at infinity;
 *   - a scalar: 8 limbs, the Montgomery form s 2^256 mod r over BLS12-381 Fr,
 *     as every NTT call of this library reads and writes them (so an NTT or
 *     quotient output feeds an MSM directly);
 *   - the result: 48 limbs, XYZZ coordinates (X, Y, ZZ, ZZZ) in the same
 *     Montgomery form with x = X / ZZ and y = Y / ZZZ; ZZ = 0 is the point at
 *     infinity.  (Affine coordinates would need one field inversion, a serial
 *     chain the caller can run wherever it likes.)
 * ------------------------------------------------------------------------ */
typedef struct msm_bases msm_bases;

/* Precompute, for c-bit windows w < W = ceil(255 / c), the multiples
 * 2^(c w) P_i of the n points (W n affine points of device memory, held by
 * the bases); window_bits = c, 0 = chosen from n (16 from n = 2^18).
 * Synchronous (waits for `stream`).  ZK_EINVAL: null, misaligned or n = 0;
 * ZK_EUNSUPPORTED: window_bits > 16 or W n >= 2^32. */
int msm_bases_create(msm_bases **out, const void *d_points, uint64_t n, uint32_t window_bits, void *stream);
void msm_bases_destroy(msm_bases *b);
uint64_t msm_bases_count(const msm_bases *b);
int msm_bases_window_bits(const msm_bases *b);
size_t msm_bases_device_bytes(const msm_bases *b);
/* Bytes of workspace msm_compute needs: the sort arrays, one bucket
 * histogram per group of 65535 / W scalars, and the bucket sums, with one
 * accumulator pair per accumulation lane (as many lanes as the bases' device
 * keeps resident at once). */
size_t msm_workspace_bytes(const msm_bases *b);
/* d_result = sum_i s_i P_i for the n scalars at d_scalars; asynchronous on
 * `stream`.  d_work: msm_workspace_bytes(b) bytes; concurrent calls need
 * their own workspace.  Inputs are not modified.  ZK_EINVAL: null or
 * misaligned pointers, scalars, result and workspace overlapping (byte
 * ranges), or a current device other than the one the bases live on. */
int msm_compute(const msm_bases *b, const void *d_scalars, void *d_result, void *d_work, void *stream);

/* Measurement helper: the all-CU rate of the units the NTT's rooflines are
 * drawn on (the paper places its NTT kernels on the GPU's INT32 roofline,
 * Section IV-C).  One warm-up launch, then `reps` launches timed with HIP
 * events on `stream`; synchronises the stream.
 *   ZK_MB_MAD_U64_U32      v_mad_u64_u32 instructions/s (8 independent chains per lane)
 *   ZK_MB_FMA_F64          v_fma_f64 instructions/s
 *   ZK_MB_ADD_U32          v_add_u32 instructions/s
 *   ZK_MB_ADDC_U32         v_add_co_u32 + v_addc_co_u32 instructions/s (carry chains)
 *   ZK_MB_MAD_ADDC         FIPS column steps/s (v_mad_u64_u32 plus the v_addc_co_u32 of its carry)
 *   ZK_MB_FFMUL_BLS12_381  Montgomery products/s over BLS12-381 Fr (three interleaved per thread,
 *                          four waves per SIMD, like the pass kernels); ZK_MB_FFMUL_K2 and
 *                          ZK_MB_FFMUL_K4 interleave two and four
 *   ZK_MB_FFMUL_F64        Montgomery products/s over BLS12-381 Fr on the FP64 multiplier
 *                          (three per thread, four waves per SIMD)
 *   ZK_MB_FFMUL_LAZY       as ZK_MB_FFMUL_BLS12_381 without the final conditional subtraction
 *                          (operands and results in [0, 2p), as in the NTT passes)
 *   ZK_MB_FFMUL_BN254      as ZK_MB_FFMUL_BLS12_381 over BN254 Fr (a modulus whose lowest
 *                          limb is not 1: the reduction digit costs a full multiply-add)
 *   ZK_MB_MAD_FMA          instructions/s of v_mad_u64_u32 and v_fma_f64 interleaved (independent)
 *   ZK_MB_MAD_ADD          instructions/s of v_mad_u64_u32 and v_add_u32 interleaved (independent)
 *   ZK_MB_COPY             bytes/s read plus written by a streaming copy of the
 *                          first half of d_buf into its second half
 * `iters`: loop trips per thread (ALU kinds; ignored by the copy).  d_buf:
 * 256-byte aligned device memory of buf_bytes; the ALU kinds store one
 * 8-byte value per launched thread (256 CUs x 2048 threads: 4 MiB) and
 * return ZK_EINVAL if it is smaller.  Writes the rate to *ops_per_s and the
 * mean launch time to *ms_per_launch. */
typedef enum {
  ZK_MB_MAD_U64_U32 = 0,
  ZK_MB_FMA_F64 = 1,
  ZK_MB_ADD_U32 = 2,
  ZK_MB_ADDC_U32 = 3,
  ZK_MB_MAD_ADDC = 4,
  ZK_MB_FFMUL_BLS12_381 = 5,
  ZK_MB_COPY = 6,
  ZK_MB_FFMUL_K2 = 7,
  ZK_MB_FFMUL_K4 = 8,
  ZK_MB_MAD_FMA = 9,
  ZK_MB_MAD_ADD = 10,
  ZK_MB_FFMUL_F64 = 11,
  ZK_MB_FFMUL_LAZY = 12,
  ZK_MB_FFMUL_BN254 = 13
} zk_microbench_kind;
int zk_microbench(int kind, uint32_t iters, void *d_buf, size_t buf_bytes, void *stream, int reps,
                  double *ops_per_s, float *ms_per_launch);

/* Element-wise Montgomery product, for checking the multipliers on their
 * own: out_i = a_i b_i 2^-256 mod p with variant 0 (the integer FIPS product
 * of every transform), a_i b_i 2^-288 mod p with variant 1 (the FP64
 * product of ZK_FLAG_FFMUL_FP64 plans, whose radix is 2^288).  Variant 2 is
 * the product the transforms' butterflies use, without its final
 * subtraction: out_i is congruent to a_i b_i 2^-256 and lies in [0, 2p) for
 * any eight-limb a_i and canonical b_i.  Inputs canonical (variant 2: b
 * only), 256-byte aligned device arrays of n elements; asynchronous on
 * `stream`.  out may equal a or b.  ZK_EUNSUPPORTED for another variant. */
int zk_field_mul(int field, int variant, const void *d_a, const void *d_b, void *d_out, uint64_t n, void *stream);

/* Thread-local description of the calling thread's last failure. */
const char *zk_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ZKNTT_H */
