/*
 * ntt.h -- C ABI of the MI355X negacyclic NTT library (libntt.so).
 *
 * What is computed (NTTSuite, "Twiddle Factors" paragraph, Eq. 1 and 3, with
 * the negacyclic twist and the inverse made explicit):
 *   psi_l     = c^((q_l - 1) / 2N), c the smallest quadratic non-residue mod q_l
 *               (a primitive 2N-th root of unity; the paper leaves g unnamed)
 *   forward   X_k = sum_{j<N} x_j psi^((2k+1) j)          mod q_l,  k = 0..N-1
 *   inverse   x_j = N^-1 psi^-j sum_{k<N} X_k psi^(-2jk)   mod q_l
 *   pointwise Z_k = X_k Y_k                                mod q_l
 * so that inverse(pointwise(forward(a), forward(b))) is the product of a and b
 * in Z_q[x]/(x^N + 1). Results are exact (integer arithmetic); every output is
 * canonical in [0, q_l).
 *
 * Data layout: contiguous row-major [batch][L][N] words, limb l of every
 * polynomial reduced mod moduli[l]. Words are uint64_t, or uint32_t for plans
 * created with NTT_WORD32. The spectrum is in natural order k = 0..N-1 unless
 * the plan has NTT_ORDER_BITREV, in which case position i holds X[brv(i)]
 * (brv reverses log2(N) bits); inverse() consumes the order forward()
 * produces, and pointwise() works in either.
 *
 * Ownership: the caller owns every data buffer (device pointers, e.g. from
 * hipMalloc or a framework tensor) and the stream. A plan owns its device
 * twiddle tables (about 16N bytes per limb and direction for 64-bit words)
 * and, for natural-order spectra with N >= 2^15, a scratch buffer of
 * batch*L*N words per stream it is used on; ntt_plan_destroy frees both.
 * Plans live on the device that was current when they were created.
 *
 * Asynchrony and errors: ntt_forward / ntt_inverse / ntt_pointwise_mul only
 * enqueue work on `stream` (a hipStream_t; NULL is the default stream) and
 * return NTT_OK; argument errors are detected before anything is enqueued and
 * returned as negative codes. Inputs must be canonical (in [0, q_l)); other
 * values give unspecified (but in-bounds) results, or NTT_ERR_RANGE with
 * NTT_DEBUG_CHECK. The functions are
 * thread-safe for concurrent use of one plan on different streams.
 *
 * Allocation failures: every device and pinned-host allocation the library
 * makes is checked; a failed one makes the call return NTT_ERR_NOMEM (a
 * creating call returns NULL with that code) after freeing what the call had
 * allocated, with nothing enqueued. The pool's pinned copy of a table falls
 * back to pageable host memory instead. For testing, the environment variable
 * NTT_FAIL_ALLOC=k makes the k-th allocation counted from when the variable
 * took its current value fail.
 */
#ifndef NTT_H
#define NTT_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define NTT_OK 0
#define NTT_ERR_ARG (-1)         /* null pointer, zero count, unknown flag     */
#define NTT_ERR_N (-2)           /* N not a power of two in [2, 2^17]          */
#define NTT_ERR_MODULUS (-3)     /* q not prime, 2N does not divide q-1, or q  */
                                 /* too large (>= 2^61; >= 2^30 with WORD32)   */
#define NTT_ERR_NOMEM (-4)       /* device or host allocation failed           */
#define NTT_ERR_HIP (-5)         /* a HIP call or kernel launch failed         */
#define NTT_ERR_BUDGET (-6)      /* server: job larger than the whole budget   */
#define NTT_ERR_UNSUPPORTED (-7) /* no kernel for this shape/variant           */
#define NTT_ERR_STATE (-8)       /* unknown ticket, or object shut down        */
#define NTT_ERR_TIMEOUT (-9)     /* wait timed out; the job is still pending   */
#define NTT_ERR_SCRATCH (-10)    /* ntt_forward_noalloc: the call needs more   */
                                 /* scratch than NTT_NOALLOC_SCRATCH_BYTES     */
#define NTT_ERR_RANGE (-11)      /* NTT_DEBUG_CHECK: an input word is not      */
                                 /* canonical (not below its limb's modulus)   */

/* ---- plan flags ---------------------------------------------------------- */
#define NTT_WORD32 0x1u          /* uint32_t words, every q_l < 2^30            */
#define NTT_ORDER_BITREV 0x2u    /* spectrum in bit-reversed order              */
#define NTT_CYCLIC 0x4u          /* the cyclic transform of Eq. 3 instead:      */
                                 /*   X_k = sum_j x_j omega^(jk), omega = c^((q-1)/N), */
                                 /*   inverse with N^-1; needs N | q-1          */
#define NTT_DEBUG_CHECK 0x8u     /* check the canonical-input precondition: each */
                                 /*   call first scans its inputs, synchronizes */
                                 /*   the stream and returns NTT_ERR_RANGE (with */
                                 /*   nothing else enqueued) if a word is not    */
                                 /*   below its modulus. Also turned on for every */
                                 /*   plan by the environment variable           */
                                 /*   NTT_DEBUG_CHECK=1. For debugging: it makes  */
                                 /*   the calls synchronous and is not for graph */
                                 /*   capture.                                    */

/* ---- kernel variants (for tuning and measurement) ------------------------- */
#define NTT_PATH_AUTO 0          /* library default for (N, word)               */
#define NTT_PATH_TINY 1          /* N < 16: one thread per transform            */
#define NTT_PATH_LDS 2           /* whole transform in one workgroup's LDS      */
#define NTT_PATH_FOURSTEP 3      /* column pass + row pass (N = N1 x N2)        */
/* The paper's algorithm variants (cyclic plans, natural order only): one
 * kernel launch per stage over global memory, canonical arithmetic (Alg. 4-5),
 * for comparison with the fused paths. */
#define NTT_PATH_PAPER_DIT 4      /* Alg. 1: bit_reverse, stages 1..L in place   */
#define NTT_PATH_PAPER_DIF 5      /* Alg. 2: stages L..1 in place, bit_reverse   */
#define NTT_PATH_PAPER_PEASE 6    /* Alg. 3: constant geometry, copy per stage   */
#define NTT_PATH_PAPER_PEASE_NC 7 /* Pease_nc: constant geometry, arrays swapped */
#define NTT_PATH_PAPER_STOCKHAM 8 /* Stockham autosort: two arrays, no bit_reverse */

typedef struct ntt_plan ntt_plan;

/* Create a plan for length N = 2^n (2 <= N <= 2^17) and L moduli. Each modulus
 * must be prime with 2N | q-1 and q < 2^61 (q < 2^30 with NTT_WORD32); the
 * array is copied. Computes psi_l, the twiddle tables and their Shoup
 * companions floor(w * 2^64 / q) (the paper's tw_h, Alg. 5) on the host and
 * uploads them. Synchronous. Returns NULL on error (see ntt_last_error). */
ntt_plan* ntt_plan_create(uint32_t N, const uint64_t* moduli, uint32_t L);

/* As ntt_plan_create with NTT_* flags and optional per-limb roots: psi may be
 * NULL (default root above) or L values, each a primitive 2N-th root of unity
 * mod q_l (checked: psi^N == q_l - 1), or with NTT_CYCLIC a primitive N-th
 * root omega (checked: omega^(N/2) == q_l - 1). */
ntt_plan* ntt_plan_create_ex(uint32_t N, const uint64_t* moduli, uint32_t L, uint32_t flags,
                             const uint64_t* psi);

void ntt_plan_destroy(ntt_plan* plan);

/* Forward negacyclic NTT of `batch` polynomials, in place on d_data
 * ([batch][L][N] words on the plan's device). Asynchronous on stream. */
int ntt_forward(const ntt_plan* plan, void* d_data, uint32_t batch, void* stream);

/* Inverse NTT (including the N^-1 scaling), in place. Asynchronous. On the
 * four-step path the result is written with streaming (nontemporal) stores,
 * which do not keep it in the caches: nothing in the transform reads it again,
 * and the caches stay with what the next kernels read. */
int ntt_inverse(const ntt_plan* plan, void* d_data, uint32_t batch, void* stream);

/* d_c = d_a * d_b elementwise mod q_l over [batch][L][N]; d_c may alias d_a
 * or d_b (exactly, not partially). Asynchronous. */
int ntt_pointwise_mul(const ntt_plan* plan, const void* d_a, const void* d_b, void* d_c,
                      uint32_t batch, void* stream);

/* d_c = inverse(d_a * d_b): the pointwise product followed by the inverse
 * NTT (the usual last two steps of a negacyclic polynomial product). On the
 * four-step path the product is computed inside the first inverse kernel, so
 * the product is never written to memory; elsewhere it is the two calls in a
 * row. d_c may alias d_a or d_b (exactly). Asynchronous. */
int ntt_pointwise_mul_inverse(const ntt_plan* plan, const void* d_a, const void* d_b, void* d_c,
                              uint32_t batch, void* stream);

/* Product of coefficient-domain polynomials, for `batch` pairs of [L][N]
 * polynomials d_a, d_b: d_c = a * b in Z_q[x]/(x^N + 1) per limb (mod
 * x^N - 1 for NTT_CYCLIC plans), i.e. inverse(pointwise(forward(a),
 * forward(b))) without handing the spectra back. At four-step sizes the two
 * forward row passes, the product and the first inverse pass are one kernel,
 * so the spectra never reach HBM. d_a and d_b are not modified; d_c may be
 * d_a or d_b. The plan keeps a workspace of 2 * batch * L * N words per
 * stream. The spectrum-order flag of the plan does not apply (inputs and
 * output are coefficients); a paper-variant plan uses the library's default
 * variant. Asynchronous. */
int ntt_polymul(const ntt_plan* plan, const void* d_a, const void* d_b, void* d_c, uint32_t batch, void* stream);

/* One kernel of a four-step transform, for timing and profiling: stage 0 is
 * the first kernel (forward: column pass, data -> scratch; inverse: row pass,
 * data -> scratch), stage 1 the second (scratch -> data). Running stage 0 then
 * stage 1 on the same stream equals ntt_forward / ntt_inverse. Returns
 * NTT_ERR_UNSUPPORTED unless the plan's variant is NTT_PATH_FOURSTEP. */
int ntt_forward_stage(const ntt_plan* plan, void* d_data, uint32_t batch, int stage, void* stream);
/* Same for ntt_pointwise_mul_inverse: stage 0 is the fused product + first
 * inverse kernel (d_a, d_b -> scratch), stage 1 the second (scratch -> d_c).
 * The intermediate is the row transform of the Montgomery product
 * a*b*2^-w mod q (w = 64, or 32 with NTT_WORD32); stage 1 multiplies 2^w back
 * in with its last stage, so the two stages together equal the fused call. */
int ntt_pointwise_mul_inverse_stage(const ntt_plan* plan, const void* d_a, const void* d_b, void* d_c,
                                    uint32_t batch, int stage, void* stream);
int ntt_inverse_stage(const ntt_plan* plan, void* d_data, uint32_t batch, int stage, void* stream);

/* Plan queries: the root used for each limb (L values: psi, or omega for
 * NTT_CYCLIC plans) and the variant. */
int ntt_plan_get_psi(const ntt_plan* plan, uint64_t* psi_out);
int ntt_plan_get_variant(const ntt_plan* plan, int* path, int* log_n1);

/* Select the kernel variant of a plan: path NTT_PATH_*, and for
 * NTT_PATH_FOURSTEP the column length 2^log_n1 (6 <= log_n1, log2(N)-log_n1
 * <= 9). The NTT_PATH_PAPER_* variants need an NTT_CYCLIC plan in natural
 * order; Pease and Stockham use scratch like the four-step path. Not safe
 * while other threads use the plan. */
int ntt_plan_set_variant(ntt_plan* plan, int path, int log_n1);

/* Quotient flavour of the 64-bit Shoup product: 0 (default) estimates
 * floor(y * w' / 2^64) from three of the four 32x32 partial products (off by
 * at most 2, lazy bound 4q); 1 computes it exactly (lazy bound 2q). Exact is
 * available on NTT_PATH_FOURSTEP only; kept for measurement. */
int ntt_plan_set_quotient(ntt_plan* plan, int exact);

/* Row passes of NTT_PATH_FOURSTEP; every setting computes the same transform
 * (the negacyclic NTT of Sec. 2, or the cyclic one of NTT_CYCLIC plans).
 * A twisted row pass: after the column stages, row r of the N1 x N2 matrix
 * is the residue of the input modulo x^N2 - b_r^N2, with b_r = psi^(2 brv(r)
 * + 1) (omega^brv(r) for cyclic plans). The row's transform is then a cyclic
 * NTT of length N2, whose twiddles are the same for every row and are kept
 * in LDS, of the row multiplied elementwise by b_r^j (the twist). The library
 * runs it split: the first register phase with the row's own twiddles (N2/16
 * or fewer, staged in LDS), then the twist, which at that point takes one
 * factor b_r^c per thread (a few when the first phase is short), then the
 * cyclic phases; the inverse runs the same steps backwards. A row then reads
 * about N2/8 table entries instead of N2. Its tables (N + N2 twiddle entries
 * per limb, direction and split) are built when the plan is created, or this
 * call or ntt_plan_set_variant selects them, for the plan's own split; a call
 * that the tuning table sends to another split builds that split's tables on
 * its first use (host work of about 10 ms per limb at N = 2^17, spread over
 * up to 16 threads). A merged row pass runs the row stages of the
 * merged-twiddle transform, whose twiddles differ from row to row and are read
 * from global memory between butterflies.
 * mask: NTT_ROW_TWIST_FWD and/or NTT_ROW_TWIST_INV select the twisted form
 * for that direction, the rest are merged; the default is both
 * (NTT_ROW_TWIST_DEFAULT): on MI355X the two forms are within a few percent
 * of each other timed alone, but the twisted ones move less memory and make a
 * step of two ciphertexts' product on two streams about 6% faster.
 * Applies to ntt_forward, ntt_inverse,
 * ntt_pointwise_mul_inverse and their _stage forms; a stage run in one
 * setting composes with the other stage run in another (the forward
 * intermediate is the same column pass output, and the inverse intermediates
 * agree modulo q within the range the column pass accepts). ntt_polymul,
 * batches and the server use the merged form. Returns NTT_ERR_ARG for other mask bits. Not
 * safe while other threads use the plan. */
#define NTT_ROW_TWIST_FWD 1
#define NTT_ROW_TWIST_INV 2
#define NTT_ROW_TWIST_DEFAULT (NTT_ROW_TWIST_FWD | NTT_ROW_TWIST_INV)
int ntt_plan_set_row_twist(ntt_plan* plan, int mask);

/* Scratch a natural-order four-step call of `batch` polynomials needs (bytes;
 * 0 when the chosen variant works in place). The plan allocates it. */
size_t ntt_workspace_bytes(const ntt_plan* plan, uint32_t batch);

/* ntt_forward for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, and harnesses that forbid
 * hipMalloc. Same arguments, transform and asynchrony as ntt_forward, but the
 * four-step intermediate lives in a fixed device array that the library
 * holds on each GPU it runs on (NTT_NOALLOC_SCRATCH_BYTES, 64 MiB, kept until
 * the process ends) instead of the plan's per-stream scratch, and the call
 * makes no allocation of any kind. That is enough for natural-order spectra
 * of batch * L * N <= 2^23 words, e.g. 4 polynomials of 24 limbs at N = 2^16.
 * Errors: NTT_ERR_SCRATCH when ntt_workspace_bytes(plan, batch) exceeds the
 * array; NTT_ERR_UNSUPPORTED for the paper's per-stage variants (their tables
 * are built on first use); the argument errors of ntt_forward. Where the
 * twisted forward row pass would need tables the plan has not built, the
 * merged one (the same transform) runs instead.
 * Calls that need no scratch (LDS-resident sizes, bit-reversed spectra) use
 * none. Every call on one GPU shares that GPU's array and the array keeps the
 * last call's contents (each call writes the whole intermediate before it
 * reads it back, so nothing needs clearing): calls that can overlap on one GPU
 * (on different streams, or from several threads) race and must be ordered by
 * the caller. */
#define NTT_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int ntt_forward_noalloc(const ntt_plan* plan, void* d_data, uint32_t batch, void* stream);

/* The row forms (NTT_ROW_TWIST_* mask) and the column passes' values per
 * thread (log2; 3 or 4 for 64-bit four-step calls, else 0) that a call with
 * `batch` polynomials would run with (after tuning). */
int ntt_plan_get_row_form(const ntt_plan* plan, uint32_t batch, int* row_twist, int* log_values);

/* The variant a call with `batch` polynomials would run (after tuning). */
int ntt_plan_get_variant_for(const ntt_plan* plan, uint32_t batch, int* path, int* log_n1, int* exact);
/* Columns per tile of the four-step column passes a call on `batch`
 * polynomials runs with: 16 or 32 (64-bit words, as tuned), 32 (32-bit
 * words), 0 off the four-step path. */
int ntt_plan_get_col_tile(const ntt_plan* plan, uint32_t batch, int* columns);

/* Thread-local code of the last failed call that returns a pointer, and a
 * static description of any code. */
int ntt_last_error(void);
void ntt_set_last_error(int code);
const char* ntt_strerror(int code);

/* ---- autotuner ------------------------------------------------------------
 * Times every kernel variant the library has for (N, word size, `items`
 * transforms per call) on the current GPU: the LDS-resident kernel, each
 * four-step split N1 x N2, and for 64-bit words both quotient flavours, 8
 * or 16 values per thread (so 2 or 1 threads per 16 values of a column) and
 * 16 or 32 columns per tile in the column passes; `reps` timed calls each after two warm-up calls, with
 * HIP events on a private stream. For a four-step winner it then times each
 * direction's row pass merged and twisted and keeps the faster. The winner
 * goes into a process-wide table that plans in automatic mode (the default)
 * and batches consult per call, keyed by (word, log2 N, log2 items); a plan
 * uses the tuned row forms until ntt_plan_set_row_twist fixes its own. The
 * table is saved and loaded as JSON tagged with the GPU architecture. At its
 * first plan, batch or server creation a process loads the file named by
 * NTT_TUNE_CACHE, or, if that variable is unset, tune_<arch>.json next to
 * libntt.so (an empty NTT_TUNE_CACHE loads nothing).
 * The timed calls rotate over copies of the batch (512 MiB in all, at most
 * 64 copies) so that each reads its data from memory rather than the caches.
 * Synchronous; allocates those copies of items*N words while it runs. */
typedef struct {
  int32_t path;       /* NTT_PATH_* */
  int32_t log_n1;     /* four-step column length log2 */
  int32_t exact;      /* 64-bit quotient flavour */
  float us_per_call;  /* measured time of the winner */
  int32_t row_twist;  /* four-step: NTT_ROW_TWIST_* mask of the faster row forms; -1 otherwise */
  int32_t lv_col;     /* four-step, 64-bit: log2 values per thread of the column passes (4), 0 = default (3) */
  int32_t col_tile;   /* four-step, 64-bit: columns per column-pass tile (32), 0 = default (16) */
} ntt_tune_choice;
int ntt_autotune(uint32_t N, uint32_t flags, uint32_t items, uint32_t reps, ntt_tune_choice* best);
int ntt_tune_save(const char* path);
int ntt_tune_load(const char* path);  /* NTT_ERR_STATE if the file is for another arch */
int ntt_tune_clear(void);

/* ---- batched executor ---------------------------------------------------------
 * Many polynomials of different N (16 <= N <= 2^17) and limb counts,
 * transformed by one ntt_batch_run: each job is one polynomial, [L][N]
 * contiguous 64-bit words at d_data, limb l reduced mod moduli[l] (q < 2^61,
 * prime, 2N | q-1). Items (polynomial, limb) are bucketed by (N, op); each
 * bucket runs the tuned (or default) variant; the buckets' kernels are
 * captured once, at creation, into one hipGraph (the buckets as parallel
 * branches; with NTT_BATCH_SERIAL one after another, the largest first), so a
 * run is a single hipGraphLaunch. Twiddle tables come from a process-wide pool
 * keyed by (device, q, N) and stay resident. The batch owns its descriptor
 * table, four-step scratch and graph; the caller owns the job buffers, which
 * must stay valid (the graph holds their addresses). Natural-order spectra. */
#define NTT_JOB_FORWARD 0u
#define NTT_JOB_INVERSE 1u
typedef struct {
  uint32_t N;                 /* transform length */
  uint32_t L;                 /* limbs */
  uint32_t op;                /* NTT_JOB_FORWARD or NTT_JOB_INVERSE */
  uint32_t reserved;
  const uint64_t* moduli;     /* L moduli (host; read during create) */
  void* d_data;               /* [L][N] words on the device, in place */
} ntt_job_desc;
typedef struct ntt_batch ntt_batch;
typedef struct {
  uint32_t items, buckets, kernels, uses_graph;
  uint64_t scratch_bytes, twiddle_pool_bytes;
} ntt_batch_info;
#define NTT_BATCH_NO_GRAPH 0x1u  /* launch the kernels directly on each run */
#define NTT_BATCH_BRANCHES 0x2u  /* the graph holds the buckets as parallel branches,
                                    forked from and joined to the run's stream: the
                                    default, so this flag changes nothing */
#define NTT_BATCH_SERIAL 0x4u    /* the graph holds the buckets one after another,
                                    largest first (not with NTT_BATCH_BRANCHES) */
ntt_batch* ntt_batch_create(const ntt_job_desc* jobs, uint32_t n_jobs, uint32_t flags);
int ntt_batch_run(ntt_batch* batch, void* stream);
int ntt_batch_get_info(const ntt_batch* batch, ntt_batch_info* info);
void ntt_batch_destroy(ntt_batch* batch);

/* ---- serving loop ---------------------------------------------------------------
 * Continuous batching of requests on device-resident polynomials ([L][N]
 * 64-bit words, 16 <= N <= 2^17, 1 <= L <= 256, natural order):
 *   NTT_REQ_NTT      d_out = forward(d_a)
 *   NTT_REQ_INTT     d_out = inverse(d_a)
 *   NTT_REQ_POLYMUL  d_out = d_a * d_b in Z_q[x]/(x^N + 1) (two forward
 *                    NTTs, pointwise product, inverse NTT)
 * d_a and d_b are not modified unless d_out equals one of them (in place);
 * partial overlaps are not allowed. A scheduler thread admits queued jobs in
 * arrival order whenever one of n_streams device streams is free and the
 * job's working memory (an operand copy for POLYMUL, four-step scratch for
 * N >= 2^14) and the twiddle tables of its (q, N) pairs that are not resident
 * yet (32N + 72 bytes each) fit in the server's hbm_budget_bytes arena, after
 * evicting resident tables no admitted job uses (least recently used first);
 * a job that cannot fit alone is refused with NTT_ERR_BUDGET; jobs admitted
 * together run as one batch (descriptor table + one launch per (phase, N)),
 * up to max_batch_items (polynomial, limb) transforms per batch. Latency is
 * measured from submit to the scheduler observing completion. With
 * NTT_SERVER_SIMULATE nothing touches a device: each batch completes after
 * simulate_ns_per_item per item (for testing the scheduler). The caller owns
 * all request buffers and must keep them valid until the ticket completes.
 * The server owns its arena, streams and descriptor buffers. submit/wait/
 * stats are thread-safe; destroy drains queued work first. */
#define NTT_REQ_NTT 0u
#define NTT_REQ_INTT 1u
#define NTT_REQ_POLYMUL 2u
#define NTT_SERVER_SIMULATE 0x1u
typedef struct {
  uint32_t op, N, L, reserved;
  const uint64_t* moduli;  /* host, L values, read during submit */
  const void* d_a;
  const void* d_b;         /* NTT_REQ_POLYMUL only */
  void* d_out;
} ntt_request;
typedef struct {
  size_t hbm_budget_bytes;
  uint32_t n_streams;        /* 1..64 */
  uint32_t max_batch_items;
  uint32_t flags;
  uint32_t reserved;
  double simulate_ns_per_item;
} ntt_server_config;
typedef struct {
  uint64_t submitted, completed, failed, rejected, queued;
  uint64_t batches, items, ntts;   /* ntts: forward + inverse transforms done */
  uint64_t admission_stalls;       /* times a free slot waited for arena space */
  uint64_t peak_bytes;             /* largest arena use */
  uint32_t max_inflight_batches, reserved;
  double p50_us, p99_us, mean_us, max_us;
  double wall_s, busy_s;           /* since creation or reset; busy = a batch in flight */
  uint64_t table_bytes;            /* twiddle tables resident in the arena now      */
  uint64_t table_uploads;          /* tables made resident (uploaded)               */
  uint64_t table_evictions;        /* unreferenced tables evicted for space         */
} ntt_server_stats;
typedef struct ntt_server ntt_server;
ntt_server* ntt_server_create(const ntt_server_config* cfg);
int ntt_server_submit(ntt_server* server, const ntt_request* req, uint64_t* ticket);
/* NTT_OK when the job finished (then the ticket is forgotten), the job's
 * error code if it failed, NTT_ERR_TIMEOUT if still pending after timeout_us
 * (< 0: wait forever), NTT_ERR_STATE for an unknown ticket. */
int ntt_server_wait(ntt_server* server, uint64_t ticket, int64_t timeout_us);
int ntt_server_get_stats(ntt_server* server, ntt_server_stats* stats);
int ntt_server_reset_stats(ntt_server* server);
void ntt_server_destroy(ntt_server* server);

/* ---- HE steps on either side of the transform ---------------------------------
 * The paper motivates the NTT by homomorphic encryption (Introduction) and
 * names further HE primitives as its future work (Conclusion). These are the
 * two steps that surround the transform in an RNS HE multiplication, with the
 * standard definitions of that literature. Same ownership, asynchrony and
 * canonical-input rules as above; 64-bit words only for the conversions.
 *
 * Ciphertext tensor product in the NTT domain (the first step of a
 * ciphertext-ciphertext product): for each of `batch` pairs of two-component
 * ciphertexts d_a, d_b [batch][2][L][N] (words of the plan's width), writes
 * d_d [batch][3][L][N] with, elementwise mod q_l,
 *   d0 = a0*b0,  d1 = a0*b1 + a1*b0,  d2 = a1*b1
 * so that (a0 + a1 s)(b0 + b1 s) = d0 + d1 s + d2 s^2. d_d must not overlap
 * d_a or d_b. The plan supplies N, L and the moduli; any spectrum order. */
int ntt_tensor_product(const ntt_plan* plan, const void* d_a, const void* d_b, void* d_d, uint32_t batch,
                       void* stream);

/* Fast RNS basis conversion (Bajard, Eynard, Hasan, Zucca, SAC 2016) from a
 * source basis s_0..s_{L-1} (product S) to a target basis t_0..t_{K-1}, on
 * coefficient-domain residues. With shat_i = S / s_i,
 *   conv(x)_j = sum_i [x_i shat_i^-1 mod s_i] shat_i  mod t_j,
 * the residues mod t_j of X + alpha S, where X in [0, S) has residues x_i and
 * 0 <= alpha < L (alpha depends on the coefficient). ModUp in key switching
 * is this conversion; ModDown (Cheon, Han, Kim, Kim, Song, SAC 2018) divides
 * by S, from y over the target basis and x over the source basis:
 *   moddown(x, y)_j = (y_j - conv(x)_j) S^-1  mod t_j.
 * A conversion plan holds the constants (shat_i^-1 mod s_i, the K x L matrix
 * shat_i mod t_j, S^-1 mod t_j) on the device current at creation.
 *   N       coefficients per polynomial: even, 2 <= N <= 2^28
 *   src, L  source primes, 1 <= L <= 64, each < 2^61 (host array, copied)
 *   dst, K  target primes, 1 <= K <= 4096, each < 2^61; all L + K distinct
 * Returns NULL and sets ntt_last_error() to NTT_ERR_ARG, NTT_ERR_N,
 * NTT_ERR_MODULUS (not prime, too large, repeated), NTT_ERR_NOMEM or
 * NTT_ERR_HIP on failure. */
typedef struct ntt_bconv ntt_bconv;
ntt_bconv* ntt_bconv_create(uint32_t N, const uint64_t* src, uint32_t L, const uint64_t* dst, uint32_t K);
void ntt_bconv_destroy(ntt_bconv* conv);
int ntt_bconv_get_info(const ntt_bconv* conv, uint32_t* N, uint32_t* L, uint32_t* K);
/* d_out [batch][K][N] = conv(d_x [batch][L][N]). d_out must not overlap d_x.
 * Device pointers 16-byte aligned (NTT_ERR_ARG otherwise). */
int ntt_base_conv(const ntt_bconv* conv, const void* d_x, void* d_out, uint32_t batch, void* stream);
/* d_out [batch][K][N] = moddown(d_x [batch][L][N], d_y [batch][K][N]).
 * d_out may be d_y (in place) but must not overlap d_x. 16-byte aligned. */
int ntt_mod_down(const ntt_bconv* conv, const void* d_x, const void* d_y, void* d_out, uint32_t batch,
                 void* stream);

#ifdef __cplusplus
}
#endif
#endif /* NTT_H */
