/*
 * pir.h -- C ABI of libpir, the GPU hot path of single-server RLWE PIR:
 * the first-dimension database scan of poly-HE folding and the negacyclic
 * NTT/INTT that feed and drain it, for AMD Instinct MI355X (gfx950).
 *
 * What is computed (paper: Sec. 3.2, poly-HE folding steps 5 and 6; Sec. 4,
 * "INT32 modular GEMM"; Sec. 2.3, RNS and NTT).  The server holds a database
 * of R x C plaintext polynomials DB[i][j] in R_p = Z_p[X]/(X^N+1).  A query is
 * R RLWE ciphertexts ct_i = (a_i, b_i) in R_Q^2, Q = q_0 * ... * q_{K-1}.  The
 * answer is, for every column j,
 *
 *      answer_j = sum_i DB[i][j] * ct_i        in R_Q^2,
 *
 * computed per RNS prime q_k in NTT form, where it becomes, for every slot t,
 * an exact modular matrix product Y_t = D_t^T * Q_t (mod q_k) of shape
 * (C x R) * (R x 2B) for a batch of B queries.
 *
 * Conventions shared by every call.
 *  - Residues are uint32 in [0, q_k).  A polynomial is stored as K rows of N
 *    residues, one row per prime ("[K][N]", RNS matrix of Sec. 2.3).
 *  - NTT form: slot t of the transform of a(X) mod q_k holds
 *    a(psi_k^(2*brv(t)+1)) mod q_k, brv = bit reversal over log2(N) bits, and
 *    psi_k = the smallest integer x >= 2 with x^N = -1 (mod q_k).  The inverse
 *    transform includes the factor N^-1.
 *  - A ciphertext is [2][K][N]: component 0 = a, component 1 = b (App. A.2).
 *  - Query layout [B][R][2][K][N]; answer layout [B][C][2][K][N].
 *  - The database lift maps a byte v to the residue v (unsigned lift).
 *  - Pointers documented "device" must point to device memory of the context's
 *    GPU; "host" to host memory.  The caller owns every buffer it passes.
 *  - Every call that takes a stream is asynchronous on that stream (a
 *    hipStream_t passed as void*; NULL = the null stream).  Buffers must stay
 *    valid until the stream has passed the work.
 *  - Errors: every call returns a pir_status.  On error nothing useful is
 *    guaranteed in the outputs; pir_last_error(ctx) describes the failure.
 *    No C++ exception crosses this boundary.
 *  - A context is not thread-safe: use one context per host thread.
 *  - Calls that use the context workspace (documented below) share one
 *    buffer: work enqueued by such calls on different streams must not run at
 *    the same time (use one stream, or order the streams with events).
 */
#ifndef PIR_H_
#define PIR_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIR_MAX_PRIMES 4
#define PIR_MIN_LOG2_N 10
#define PIR_MAX_LOG2_N 12
#define PIR_PRIME_BITS 28 /* every q_k < 2^28 */
#define PIR_MAX_R 32768u  /* rows: bounds the exact int32 limb sums */
#define PIR_MAX_C 65536u

typedef enum {
  PIR_OK = 0,
  PIR_ERR_INVALID_ARG = 1,   /* null pointer, size out of range, bad layout */
  PIR_ERR_UNSUPPORTED = 2,   /* parameters outside what the kernels handle */
  PIR_ERR_OUT_OF_MEMORY = 3, /* a device or host allocation failed */
  PIR_ERR_BUDGET = 4,        /* the context's HBM budget would be exceeded */
  PIR_ERR_DEVICE = 5,        /* a HIP runtime call failed */
  PIR_ERR_NOT_READY = 6      /* asked for a result that is not available yet */
} pir_status;

typedef void *pir_stream; /* hipStream_t */

typedef struct pir_ctx pir_ctx; /* one per device: tables, workspace, budget */
typedef struct pir_db pir_db;   /* device-resident NTT-form database */

/* RNS parameters (Sec. 2.3; prime rule of App. A, "RNS prime selection").
 * N = 2^log2_n with 10 <= log2_n <= 12; 1 <= n_primes <= 4; each primes[k]
 * prime, < 2^28, = 1 (mod 2N), all distinct; p = 2^plain_log2 with
 * 1 <= plain_log2 <= 32 (database bytes are plaintext coefficients and are
 * lifted as they are; ring packing scales by Delta = floor(Q / p)). */
typedef struct {
  uint32_t log2_n;
  uint32_t n_primes;
  uint32_t primes[PIR_MAX_PRIMES];
  uint32_t plain_log2;
} pir_params;

/* Human-readable name of a status code (static storage). */
const char *pir_status_string(pir_status s);

/* Library version string (static storage). */
const char *pir_version(void);

/* The `count` largest primes q < 2^bound_log2 with q = 1 (mod 2^(log2_n+1)),
 * in descending order (App. A, RNS prime selection).  Host only; `out` is a
 * host array of `count` entries.  INVALID_ARG if log2_n > 20, bound_log2 > 31,
 * count == 0 or too few primes exist. */
pir_status pir_find_primes(uint32_t log2_n, uint32_t count, uint32_t bound_log2,
                           uint32_t *out);

/* Validate `params`; on success write psi_k (the NTT root, see above) for each
 * prime into `psi_out` (host, n_primes entries; may be NULL).  Host only. */
pir_status pir_params_check(const pir_params *params, uint32_t *psi_out);

/* Create a context on HIP device `device`.  `hbm_budget_bytes` caps the device
 * memory the context may hold (databases + workspace); 0 = no cap beyond the
 * device.  *out receives the context; release it with pir_ctx_destroy. */
pir_status pir_ctx_create(int device, size_t hbm_budget_bytes, pir_ctx **out);

/* Release the context (after freeing its databases).  Waits for the device. */
void pir_ctx_destroy(pir_ctx *ctx);

/* Text of the last error on `ctx` (valid until the next call on it); with
 * ctx == NULL, the last failure of a call that had no context (this thread). */
const char *pir_last_error(const pir_ctx *ctx);

/* Device bytes the context holds right now (databases + workspace). */
size_t pir_ctx_device_bytes(const pir_ctx *ctx);

/* Make the context's workspace at least `bytes` large now, so that later
 * calls of that size allocate nothing.  Synchronizes the device when it grows. */
pir_status pir_ctx_reserve(pir_ctx *ctx, size_t bytes);

/* ---- offline database transform (Sec. 2.4 plaintext bloating; Sec. 3.2
 * step 5; Sec. 4.2 layout transposition; Sec. 4.3 fused RNS decomposition).
 * Lifts every byte of `raw` ([R][C][N] uint8, row-major: row i, column j,
 * coefficient n) into Z_{q_k} for every prime, applies the forward NTT, and
 * stores the result in the library's scan layout (slot-major, limb-planar
 * tiles; opaque).  `raw` is device memory if raw_is_device != 0, else host
 * memory (copied in slabs through pinned staging).  1 <= R <= PIR_MAX_R,
 * 1 <= C <= PIR_MAX_C.  The database holds R_pad*C_pad*N*K*4 + 65536 bytes
 * of device memory (R_pad = R rounded up to 64, C_pad = C rounded up to 8; the
 * last 64 KiB are padding that the batched scan may read but never uses);
 * BUDGET if that exceeds the context's budget.  The call returns after `raw` has been
 * consumed (it synchronizes `stream`), so the caller may free `raw` at once.
 * *out receives the database; release it with pir_db_free. */
pir_status pir_db_load_ntt(pir_ctx *ctx, const pir_params *params, const uint8_t *raw,
                           int raw_is_device, uint32_t R, uint32_t C, pir_stream stream,
                           pir_db **out);

/* Shape and size of a loaded database (any output pointer may be NULL). */
pir_status pir_db_info(const pir_db *db, pir_params *params, uint32_t *R, uint32_t *C,
                       size_t *device_bytes);

/* Read back NTT-form database polynomials in canonical layout: rows
 * [i0, i0+ni) x columns [j0, j0+nj) into `out` (device, [ni][nj][K][N] uint32).
 * For checking the offline transform against an independent one. */
pir_status pir_db_read_ntt(pir_ctx *ctx, const pir_db *db, uint32_t i0, uint32_t ni,
                           uint32_t j0, uint32_t nj, uint32_t *out, pir_stream stream);

/* Release a database's device memory (waits for the device). */
void pir_db_free(pir_db *db);

/* ---- forward / inverse negacyclic NTT of queries and answers (Sec. 2.3; Sec. 4.3),
 * in place on `polys` (device, [n_polys][K][N] uint32, residues < q_k).
 * The inverse includes N^-1.  Values >= q_k give unspecified results (never an
 * out-of-bounds access). */
pir_status pir_ntt(pir_ctx *ctx, const pir_params *params, uint32_t *polys, size_t n_polys,
                   pir_stream stream);
pir_status pir_intt(pir_ctx *ctx, const pir_params *params, uint32_t *polys, size_t n_polys,
                    pir_stream stream);

/* ---- answer drain with modulus switching: inverse NTT fused with it (Sec. 4.3 fuses the
 * modulus reduction into the inverse NTT; Sec. 3.6 ends the online answer with
 * it; App. D.5 bounds its error).  For each of n_polys answer polynomials in
 * NTT form, answer_ntt[p][k][t] (device, [n_polys][K][N] uint32 residues in
 * [0, q_k), K = params->n_primes), the inverse NTT per prime gives residues
 * of coefficient x in [0, Q), Q = q_0 q_1 (or q_0); out[p][t] (device,
 * [n_polys][N] uint32) receives the nearest integer to x * 2^bits / Q,
 * reduced mod 2^bits (Q is odd, so there are no ties).  The paper's target
 * is bits = 29.  answer_ntt is not modified; out must not overlap it.
 * Asynchronous on `stream`.  Errors: INVALID_ARG (NULL buffers with
 * n_polys > 0, bits outside [1, 32], bad params), UNSUPPORTED (more than two
 * primes).  Timed as the INTT stage when profiling is on. */
pir_status pir_intt_modswitch(pir_ctx *ctx, const pir_params *params, const uint32_t *answer_ntt,
                              size_t n_polys, uint32_t bits, uint32_t *out, pir_stream stream);

/* ---- scalar-HE database GEMM mod 2^32 (Sec. 4.1: an INT8 database times
 * INT32 query words on the matrix engines, four byte-wise products shifted
 * and added mod 2^32; Sec. 2: the online step of SimplePIR with multi-client
 * batching).  pir_sdb_load copies an int8 database db[D1][D0] (row-major,
 * host or device memory per db_is_device; the caller may free it once the
 * call returns) into device tiles of ceil(D1/32)*32 x D0_pad bytes, D0_pad =
 * D0 rounded up to 256 (1 byte per entry).  1 <= D1 <= PIR_SDB_MAX_D1,
 * 1 <= D0 <= PIR_SDB_MAX_D0 (every int32 partial sum of the product is then
 * exact), at most 2^40 bytes of tiles.  Errors: INVALID_ARG, OUT_OF_MEMORY,
 * BUDGET, DEVICE.
 * pir_sdb_mul: query device uint32 [B][D0], out device uint32 [B][D1],
 *   out[b][r] = sum_c db[r][c] * query[b][c]  (mod 2^32),
 * 1 <= B <= PIR_MAX_BATCH; uses 32 KiB x ceil(D0/256) x ceil(B/32) of
 * context workspace for the split queries.  Asynchronous on `stream`; timed as the
 * pack and scan stages when profiling is on.  pir_sdb_free waits for the
 * device and releases the tiles. */
#define PIR_SDB_MAX_D0 131071u
#define PIR_SDB_MAX_D1 (1u << 26)
typedef struct pir_sdb pir_sdb;
pir_status pir_sdb_load(pir_ctx *ctx, const int8_t *db, int db_is_device, uint32_t D1,
                        uint32_t D0, pir_stream stream, pir_sdb **out);
pir_status pir_sdb_mul(pir_ctx *ctx, const pir_sdb *db, const uint32_t *query, uint32_t B,
                       uint32_t *out, pir_stream stream);
void pir_sdb_free(pir_sdb *db);


/* ---- the scan in NTT form (Sec. 3.2 step 6; Sec. 4 INT32 modular GEMM).
 * query_ntt: device [B][R][2][K][N], NTT form; answer_ntt: device
 * [B][C][2][K][N], NTT form, fully overwritten:
 *   answer[b][j][c][k][t] = sum_i D_k[i][j][t] * query[b][i][c][k][t] (mod q_k).
 * 1 <= B <= PIR_MAX_BATCH.  For B > 1 uses context workspace of about
 * B*R_pad*2*K*N (query tiles) + B*C*2*K*N*4 (answers in scan order) bytes,
 * grown on demand. */
#define PIR_MAX_BATCH 256u
pir_status pir_db_mul(pir_ctx *ctx, const pir_db *db, const uint32_t *query_ntt, uint32_t B,
                      uint32_t *answer_ntt, pir_stream stream);

/* ---- fused batch over several databases (Sec. 2.5 multi-client
 * batching; Sec. 4.4 stream-wise buffering).  For every job: forward NTT of
 * its queries, the scan, inverse NTT of its answers -- coefficient form in and
 * out.  Jobs may name different databases (different N, R, C); the scans of
 * all jobs run in one launch.  query_coeff: device [B][R][2][K][N] (left
 * unchanged).  switch_bits = 0: answer_coeff is device [B][C][2][K][N]
 * (coefficient form).  switch_bits in [1, 32]: the drain is the fused inverse
 * NTT and modulus switch of pir_intt_modswitch, and answer_coeff is device
 * [B][C][2][N] words mod 2^switch_bits (K <= 2, else UNSUPPORTED); the NTT-form
 * answers then take B*C*2*K*N*4 bytes of context workspace. */
typedef struct {
  const pir_db *db;
  uint32_t B;
  const uint32_t *query_coeff;
  uint32_t *answer_coeff;
  uint32_t switch_bits;
} pir_job;

pir_status pir_answer_batch(pir_ctx *ctx, const pir_job *jobs, size_t n_jobs,
                            pir_stream stream);

/* ---- pir_answer_batch without any device allocation.  For callers that
 * cannot allocate device memory: code under HIP graph capture, serving loops
 * and harnesses that forbid hipMalloc.  Same jobs, layouts, results and
 * errors as pir_answer_batch, but its workspace (the NTT-form queries, the
 * query tiles, the scan-order answers and the unswitched answers) lives in a
 * fixed device array of PIR_STATIC_SCRATCH_BYTES that the library holds on
 * every GPU it runs on until the process ends, instead of the context's
 * growable workspace.  Calls no allocating routine.  A job list whose
 * workspace exceeds that size (for instance B*R*2*K*N*4 > 64 MiB for one
 * batch-1 job) returns PIR_ERR_BUDGET before anything is enqueued.  Every
 * call on one GPU shares that GPU's array, from any context: calls that
 * overlap on one GPU (different streams, host threads or contexts) race and
 * must be ordered by the caller.  Stage profiling (pir_profile_*) does not
 * time these calls.  PIR_ERR_DEVICE if the array's address could not be
 * taken when the context was created. */
#define PIR_STATIC_SCRATCH_BYTES (64u << 20)
pir_status pir_answer_batch_static(pir_ctx *ctx, const pir_job *jobs, size_t n_jobs,
                                   pir_stream stream);

/* ---- ring packing of LWE ciphertexts into RLWE ciphertexts (App. C.1,
 * Eq. tiptoe-rp; Sec. 3.5 "Massive parallelism": H C + (0 | G) as
 * (#RNS N)-parallel ceil(D1/N) x 2B x n modular GEMMs over NTT-form
 * polynomials).  The LWE ciphertexts of a client are the rows of (A, b):
 * A is D1 x n over Z_p (the same for every client: SimplePIR's hint), b its
 * D1 offsets, p = 2^params->plain_log2.  Cut into C' = ceil(D1/N) chunks of
 * N rows, chunk r packs into one RLWE ciphertext
 *     (0, Delta iota(b_r)) + sum_{i<n} iota(A_{r,i}) ct_i      in R_Q^2,
 * iota(v) = sum_j v_j X^j, A_{r,i}[j] = A[r N + j][i] (zero past D1),
 * Delta = floor(Q / p), values of Z_p lifted unsigned, ct_i the client's
 * special ciphertext encrypting its LWE secret entry s_i; it decrypts to
 * iota(b_r + A_r s) mod p.
 * pir_pack_load: the offline transform of A ([D1][n] uint32, row-major, each
 * entry < 2^32; host or device per a_is_device) into an opaque hint H held
 * like a database of n rows and C' columns (pir_db_info reports R = n,
 * C = C'); 1 <= n <= PIR_MAX_R, C' <= PIR_MAX_C.  Uses about 2 x D1 n 4
 * bytes of temporary device memory; synchronizes `stream`; release H with
 * pir_db_free.  Errors: INVALID_ARG, UNSUPPORTED, BUDGET, OUT_OF_MEMORY,
 * DEVICE.
 * pir_pack: for B clients (1 <= B <= PIR_MAX_BATCH), special_coeff device
 * [B][n][2][K][N] (coefficient form, residues < q_k, left unchanged), lwe_b
 * device [B][D1] uint32 (< 2^32), out device [B][C'][2][K][N] coefficient
 * form, or with switch_bits in [1, 32] (K <= 2) the fused modulus switch of
 * pir_intt_modswitch into [B][C'][2][N] words.  Asynchronous on `stream`;
 * uses context workspace as pir_answer_batch does for one job, plus
 * B C' K N 4 bytes for NTT(Delta iota(b)).  INVALID_ARG for a database that
 * was not loaded by pir_pack_load. */
pir_status pir_pack_load(pir_ctx *ctx, const pir_params *params, const uint32_t *A, int a_is_device,
                         uint32_t D1, uint32_t n, pir_stream stream, pir_db **out);
pir_status pir_pack(pir_ctx *ctx, const pir_db *H, uint32_t B, const uint32_t *special_coeff,
                    const uint32_t *lwe_b, uint32_t *out, uint32_t switch_bits, pir_stream stream);

/* ---- query expansion (ExpPack: Sec. 3.5 "Expansion-based ring packing",
 * App. C.2) and RGSW folding (Sec. 3.2 step 7; Sec. 3.6 step 7).
 *
 * Gadget (both calls): a coefficient of Z_Q, Q = q0 q1 (one or two primes), is
 * recombined by CRT, centred to (-Q/2, Q/2] and written in n_digits balanced
 * digits of base 2^base_log (the low ones in [-2^(base_log-1),
 * 2^(base_log-1)), the top one taking the rest); g_d = 2^(base_log d).
 * Requires 2^(base_log n_digits) >= Q, 1 <= base_log <= 30,
 * 1 <= n_digits <= PIR_MAX_DIGITS, and one or two primes (else UNSUPPORTED).
 * Ciphertexts are (a, b) with phase a s + b, layout [2][K][N] coefficient form,
 * residues < q_k.
 *
 * pir_expand_keys_load: the key-switching keys of B clients, keys
 * [B][levels][n_digits][2][K][N] coefficient form (host or device per
 * keys_is_device): key j of a client switches from s(X^(N/2^j + 1)) to s, row
 * d = (a_d, -a_d s + e_d + g_d s(X^(N/2^j + 1))).  They are copied and held in
 * NTT form (B levels n_digits 2 K N 4 bytes) until pir_expand_keys_free.
 * 1 <= levels <= log2 N.  A host copy is complete on return; a device source
 * must stay valid until `stream` passes the load.
 *
 * pir_expand: every client's ciphertext ct_coeff [B][2][K][N] of
 * sum_i m_i X^i becomes out [B][n][2][K][N], output i encrypting the constant
 * m_i (1 <= n <= N): the input is multiplied by 2^-l mod q_k (l =
 * ceil(log2 n), at least 1, at most the keys' levels) and taken through l
 * levels of the recursive expansion; at level j each ciphertext c becomes
 * c + Subs(c, N/2^j + 1) at its own index k and c' + Subs(c', N/2^j + 1),
 * c' = c X^(-2^j), at index k + 2^j, Subs = automorphism X -> X^g then key
 * switch.  out feeds pir_pack's special ciphertexts directly.  Asynchronous on
 * `stream`; uses context workspace of about
 * B (2 min(2^(l-1), n) 2 + n (n_digits + 2)) K N 4 bytes.
 *
 * pir_fold: for each of B clients, selects one of D = 2^L ciphertexts
 * cts_coeff [B][D][2][K][N] with L RGSW ciphertexts rgsw_coeff
 * [B][L][2 n_digits][2][K][N] (coefficient form; row d = (a_d + m g_d, -a_d s +
 * e_d), row n_digits + d = (a_d', -a_d' s + e_d' + m g_d), m the index bit):
 * round j replaces entries (2i, 2i + 1) by ct_2i + RGSW_j [x] (ct_2i+1 - ct_2i),
 * the external product being sum_d D_d(a) row_d + D_d(b) row_{n_digits + d}.
 * out [B][2][K][N].  D = 1 copies.  Asynchronous on `stream`; context
 * workspace about B (L 2 n_digits 2 + D/2 (6 + 2 n_digits)) K N 4 bytes.
 * Errors: INVALID_ARG, UNSUPPORTED, BUDGET, OUT_OF_MEMORY, DEVICE. */
#define PIR_MAX_DIGITS 16u
typedef struct pir_keys pir_keys;
pir_status pir_expand_keys_load(pir_ctx *ctx, const pir_params *params, const uint32_t *keys,
                                int keys_is_device, uint32_t B, uint32_t levels,
                                uint32_t base_log, uint32_t n_digits, pir_stream stream,
                                pir_keys **out);
void pir_expand_keys_free(pir_keys *keys);
pir_status pir_expand(pir_ctx *ctx, const pir_keys *keys, const uint32_t *ct_coeff, uint32_t n,
                      uint32_t *out, pir_stream stream);
pir_status pir_fold(pir_ctx *ctx, const pir_params *params, const uint32_t *cts_coeff, uint32_t D,
                    const uint32_t *rgsw_coeff, uint32_t base_log, uint32_t n_digits, uint32_t B,
                    uint32_t *out, pir_stream stream);

/* ---- batch steady state: a job list captured once into a HIP graph.
 * pir_plan_create records what pir_answer_batch(jobs) enqueues (all kernel
 * launches, with the scan variants chosen at that moment) into a graph with
 * a workspace of its own; pir_plan_launch replays it on `stream` with no
 * host-side decoding.  The buffers named by the jobs are baked in: refill the
 * query buffers between launches to answer new queries.  The jobs' databases
 * must outlive the plan.  pir_plan_destroy waits for the device. */
typedef struct pir_plan pir_plan;

pir_status pir_plan_create(pir_ctx *ctx, const pir_job *jobs, size_t n_jobs, pir_stream stream,
                           pir_plan **out);
pir_status pir_plan_launch(pir_plan *plan, pir_stream stream);
void pir_plan_destroy(pir_plan *plan);

/* ---- tuning of the scan.  Several kernel variants compute the same
 * exact result with different tile shapes, unroll depths and load policies.
 * The context remembers one variant per (N, K, R, C, B); without a choice a
 * fixed default is used.  Results never depend on the variant. */

/* Number of scan variants for batch size B (host only). */
uint32_t pir_scan_variants(uint32_t B);

/* Use variant `index` (< pir_scan_variants(B)) for databases shaped like `db`
 * at batch size B. */
pir_status pir_scan_select(pir_ctx *ctx, const pir_db *db, uint32_t B, uint32_t index);

/* Name of the kernel ("k_scan_b1", "k_scan_b1r" or "k_scan_mfma") that a
 * single-job scan of `db` at batch size B launches with the context's current
 * choice (for profiles and reports).  The string is static; NULL for a NULL
 * context or database or B outside [1, PIR_MAX_BATCH]. */
const char *pir_scan_kernel(const pir_ctx *ctx, const pir_db *db, uint32_t B);

/* Autotune: time every variant for `db` at batch size B on `stream` (on
 * workspace contents; values do not affect timing), keep the fastest, and wait
 * for the stream.  If `report` is not NULL it receives up to report_len bytes
 * of "index:kind/jbw/unr/nt=ms;" entries and the chosen index. */
pir_status pir_tune(pir_ctx *ctx, const pir_db *db, uint32_t B, pir_stream stream, char *report,
                    size_t report_len);

/* Autotune the fused scan launches of pir_answer_batch for this job list:
 * times every variant on the whole list (values do not affect timing) and
 * keeps the fastest for later calls with jobs of the same shapes in the same
 * order.  Waits for `stream`.  `report` as for pir_tune. */
pir_status pir_tune_batch(pir_ctx *ctx, const pir_job *jobs, size_t n_jobs, pir_stream stream,
                          char *report, size_t report_len);

/* ---- continuous-batching server (Sec. 2.5 multi-client batching;
 * Sec. 4.4 stream-wise buffering).  The database's K*N (prime, slot) pairs are
 * cut into n_chunks ranges [K N c / n_chunks, K N (c+1) / n_chunks) scanned
 * round-robin, one range per step.  A query
 * is admitted at a step boundary into a free column slot (forward NTT and
 * limb packing into its own columns), takes part in every step's scan launch
 * with all other active queries, and finishes after n_chunks steps: inverse
 * NTT, copy to its answer buffer, completion event.  A query's answer is the
 * same bytes alone or among others.  State per column slot: query limbs
 * (R_pad*2*K*N bytes) and an answer (C*2*K*N*4 bytes); max_batch is lowered
 * to what the context's HBM budget admits (BUDGET if not even one fits). */
typedef struct pir_server pir_server;

pir_status pir_server_create(pir_ctx *ctx, const pir_db *db, uint32_t max_batch, uint32_t n_chunks,
                             pir_server **out);
void pir_server_destroy(pir_server *srv);

/* Queue a query (device [R][2][K][N], coefficient form) whose answer goes to
 * answer_coeff (device [C][2][K][N]).  Launches nothing.  Both buffers must
 * stay valid until the ticket reports done. */
pir_status pir_server_submit(pir_server *srv, const uint32_t *query_coeff, uint32_t *answer_coeff,
                             uint64_t *ticket);

/* One step on `stream`: admit queued queries into free slots, scan the next
 * range for all active queries, finish queries that completed their lap.
 * Asynchronous.  *admitted / *finished (may be NULL) count this step's events.
 * Steps of one server share its state (query columns, answers, the admission
 * scratch): give every step the same stream, or order the streams. */
pir_status pir_server_step(pir_server *srv, pir_stream stream, uint32_t *admitted,
                           uint32_t *finished);

/* *done = 1 once the ticket's answer is in its buffer (reported once; the
 * ticket is then forgotten), else 0.  INVALID_ARG for unknown tickets;
 * DEVICE (reported once) for a ticket whose answer drain could not be
 * launched.  A step whose admission or scan launch fails returns DEVICE and
 * leaves the failed query queued and the range unscanned, so stepping again
 * retries it. */
pir_status pir_server_poll(pir_server *srv, uint64_t ticket, int *done);

/* Admission limit after the budget, queries active and queued, next range. */
pir_status pir_server_info(const pir_server *srv, uint32_t *max_batch, uint32_t *active,
                           uint32_t *queued, uint32_t *next_chunk);

/* Capacity planning on the host (no device): the largest batch <= max_batch
 * whose server state -- query limbs of every column slot, the answer state of
 * every slot, one admission's NTT scratch -- fits in budget_bytes beside
 * held_bytes already held (budget 0 = no cap), for a database of R x C
 * polynomials under `params`.  *admitted = 0 if not even one fits;
 * *state_bytes (may be NULL) receives that batch's state size.  This is the
 * limit pir_server_create applies. */
pir_status pir_server_capacity(const pir_params *params, uint32_t R, uint32_t C, size_t held_bytes,
                               size_t budget_bytes, uint32_t max_batch, uint32_t *admitted,
                               size_t *state_bytes);

/* The server's schedule run on the host with a stand-in executor (no device),
 * for tests and capacity planning.  n_slots = K*N slots cut into n_chunks
 * ranges (1 <= n_chunks <= n_slots); submits[s] queries are submitted before
 * step s (s < n_steps), numbered 0.. in submission order; n_queries = their
 * sum.  For each query: admit_step, admit_slot (column slot) and finish_step
 * (UINT32_MAX if it did not happen within n_steps).  cover (host,
 * [n_queries][n_slots], may be NULL) counts how often each slot was scanned
 * while the query was active: exactly 1 everywhere for a finished query. */
pir_status pir_server_simulate(uint32_t max_batch, uint32_t n_slots, uint32_t n_chunks,
                               const uint32_t *submits, uint32_t n_steps, uint32_t n_queries,
                               uint32_t *admit_step, uint32_t *admit_slot, uint32_t *finish_step,
                               uint32_t *cover);

/* ---- measurement: per-stage kernel time with HIP events (off by default).
 * While enabled, pir_db_mul and pir_answer_batch time each profiled stage with
 * a pair of HIP events on the call's stream: the scan's launch records them
 * itself at the kernel's start and end (no marker commands between kernels);
 * the other stages record them on the stream around their launches, which
 * leaves a few microseconds idle between kernels.  pir_profile_read waits for
 * the recorded events and returns the summed elapsed time (ms) and the number
 * of launches of `stage` since profiling was (re-)enabled.  Enabling resets
 * the sums.  Graph captures (pir_plan_create) never record events. */
typedef enum {
  PIR_STAGE_NTT = 0,  /* forward NTT of queries */
  PIR_STAGE_PACK = 1, /* query transposition into scan tiles */
  PIR_STAGE_SCAN = 2, /* the database scan */
  PIR_STAGE_INTT = 3, /* inverse NTT of answers */
  PIR_STAGE_UNPACK = 4, /* answer transposition out of scan order (B > 1) */
  PIR_N_STAGES = 5
} pir_stage;

/* enable != 0: time every stage; 0: off. */
pir_status pir_profile_enable(pir_ctx *ctx, int enable);
/* Time only the stages whose bit (1 << stage) is set in mask (0: off).
 * INVALID_ARG for bits at or above PIR_N_STAGES. */
pir_status pir_profile_stages(pir_ctx *ctx, uint32_t mask);
pir_status pir_profile_read(pir_ctx *ctx, uint32_t stage, double *total_ms, uint64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* PIR_H_ */
