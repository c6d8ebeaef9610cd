/*
 * ldpcx.h -- C-ABI of libldpcx, batched LDPC decoding on AMD Instinct MI355X (gfx950).
 *
 * The calls follow the paper's statement of the decoding problem (Algs. 1 and
 * 2: input H, the iteration cap I_max and the channel observation y; output
 * the decision c-hat, sought such that c-hat H^T = 0 or the cap is reached;
 * sec. 2.1: H is a sparse M x N matrix over GF(2^p), code size (N, K) with
 * K = N - M).  Binary codes (g = 2) are decoded with min-sum variants, codes
 * over GF(g), g = 2^p <= 256, with the Min-Max algorithm (Alg. 2).
 *
 * Conventions for every call:
 *   - Pointers documented as "device" must point to memory of the current HIP
 *     device (e.g. a torch tensor's data_ptr()); "host" pointers are ordinary
 *     CPU memory.  The caller owns every input/output buffer; the library owns
 *     code handles, internal workspaces and servers.
 *   - `stream` is a hipStream_t passed as void* (NULL = the legacy default
 *     stream).  Decode calls are stream-ordered and asynchronous: they return
 *     once the work is enqueued; buffers must stay valid until it completes.
 *   - Arguments are validated on the host before anything is enqueued.  Every
 *     call returns an ldpcx_status; no C++ exception crosses the ABI.  The
 *     last error message of the calling thread is available from
 *     ldpcx_last_error().  A device fault surfaces as LDPCX_E_DEVICE at the
 *     next call that synchronises.
 *   - Code handles are immutable after creation and may be shared between
 *     threads and streams.
 *   - Integer semantics are fixed and identical on every code path: results
 *     are bit-exact functions of the inputs (see ldpcx_decode_params).
 */
#ifndef LDPCX_H
#define LDPCX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LDPCX_OK = 0,
    LDPCX_E_INVAL = -1,       /* bad argument or malformed code description */
    LDPCX_E_NOMEM = -2,       /* device or host allocation failed */
    LDPCX_E_DEVICE = -3,      /* HIP runtime error (launch failure, device fault) */
    LDPCX_E_UNSUPPORTED = -4, /* valid request outside what the kernels implement */
    LDPCX_E_BUDGET = -5,      /* server: request cannot fit the memory budget */
    LDPCX_E_CANCELLED = -6,   /* server: request was cancelled */
    LDPCX_E_TIMEOUT = -7,     /* server: wait timed out (request still pending) */
    LDPCX_E_NOTFOUND = -8     /* server: unknown ticket */
} ldpcx_status;

enum { LDPCX_SCHED_FLOODING = 0, LDPCX_SCHED_LAYERED = 1, LDPCX_SCHED_AUTO = 2 };
enum { LDPCX_RULE_MS = 0, LDPCX_RULE_NMS = 1, LDPCX_RULE_OMS = 2, LDPCX_RULE_MINMAX = 3, LDPCX_RULE_SPA = 4 };

typedef struct ldpcx_code ldpcx_code;

/* Description of a parity-check matrix H (host memory; copied by ldpcx_code_create).
 *   g          field size: 2 for binary codes, else 2^p with 4 <= g <= 256.
 *   prim_poly  primitive polynomial of GF(g), bit i = coefficient of x^i (e.g. 0x43 for
 *              x^6 + x + 1); ignored when g == 2.  Field elements use the polynomial basis
 *              of sec. 2.1 (element x encodes the polynomial whose coefficients are x's bits).
 *   n, m       number of variable nodes (columns, symbols) and check nodes (rows).
 *   row_ptr    [m + 1] CSR row offsets, row_ptr[0] = 0.
 *   col_idx    [row_ptr[m]] column of each nonzero, strictly ascending inside a row.
 *   h_val      [row_ptr[m]] nonzero GF(g) coefficient of each entry; NULL when g == 2.
 *   z          layer size for the binary layered schedule: rows [l*z, (l+1)*z) form layer
 *              l and must touch pairwise disjoint columns; m % z == 0.  0 = no layer
 *              structure.  Ignored for g > 2 (see the Min-Max layers under schedule).
 *   k_info     information symbols per codeword used for throughput accounting (n - m).
 * Limits: every check degree in [2, 14] for g == 2 (in [2, 16] for g > 2); n, m >= 1. */
typedef struct {
    int32_t g;
    uint32_t prim_poly;
    int32_t n, m;
    const int32_t *row_ptr;
    const int32_t *col_idx;
    const uint8_t *h_val;
    int32_t z;
    int32_t k_info;
} ldpcx_code_desc;

/* Decoding parameters.
 *   max_iters   I_max >= 0.
 *   early_stop  1: iteration k first tests the syndrome of the decision of iteration
 *               k - 1 and stops the codeword when it is zero (Alg. 2); 0: always run
 *               max_iters iterations (fixed-iteration throughput mode).
 *   schedule    FLOODING (two-phase, Alg. 2), LAYERED (rows of one layer in parallel,
 *               layers in ascending order; binary codes with z > 0 or z == 0 meaning
 *               row by row; Min-Max over GF(4)..GF(64): layers from a greedy colouring
 *               of the checks in ascending order, each check in the lowest layer holding
 *               no check that shares a variable with it, and each check's incoming
 *               alphas formed by eq. (14) from the betas as they stand when its layer
 *               runs), or AUTO (the autotuner picks; ldpcx_decode reports the schedule
 *               used).  The FFT-SPA decoder and GF(128)/GF(256) run FLOODING only.
 *   rule        MS / NMS / OMS for g == 2, MINMAX for g > 2.
 *   nms_num, nms_shift   NMS magnitude f(m) = (nms_num * m) >> nms_shift (0.75 = 3, 2);
 *               a factor in [0, 1]: 0 <= nms_num <= 2^nms_shift, nms_shift <= 6
 *               (LDPCX_E_INVAL otherwise), so that f(m) <= m <= msg_max.
 *   oms_offset  OMS magnitude f(m) = max(m - oms_offset, 0).
 *   msg_max     binary variable-to-check message saturation, 1..127 (default 127).
 * Binary arithmetic: channel LLRs L are int8, positive favours bit 0.  Check-to-
 * variable message r_mn = prod_{n' != n} sgn(q_mn') * f(min_{n' != n} |q_mn'|),
 * sgn(0) = +1; a posteriori Lambda_n = L_n + sum_m r_mn (exact, 16 bit, in both
 * schedules: the layered update is Lambda_n <- Lambda_n - r_old + r_new); the check
 * node sees q_mn = clamp(Lambda_n - r_mn, +-msg_max); decision c_n = [Lambda_n < 0].
 * Min-Max arithmetic (eqs. (7)-(15)): messages int16, sums in 32 bit, alpha clamped
 * to nb_msg_max (0 = 32767, the 16-bit decoder; 127 gives the 8-bit message variant of
 * sec. 5, whose channel vectors are clipped to the same range: gamma'(x) =
 * min(gamma(x), nb_msg_max) is used wherever gamma appears); decision = lowest x
 * minimising gamma'_n(x) + sum_m beta_mn(x).  nb_msg_max is ignored for binary codes.
 * FFT-SPA arithmetic (Alg. 1, rule SPA, flooding; GF(4)..GF(64) with check and variable
 * degrees <= 16, GF(128) and GF(256) with degrees <= 4; gamma is the same symbol-cost
 * input): probabilities in Q24 (2^24 = 1),
 * channel p = norm(W(gamma)) with W(c) = round(2^24 exp(-c/4)); eq. (3) with the
 * Walsh-Hadamard transform exact in integers, products qmul(a, b) = floor((a b + 2^23)
 * / 2^24) in ascending edge order, inverse = transform (its sums in 64 bits) then
 * floor(. / g) clamped at 0;
 * eqs. (5)-(6) with norm(z)(x) = floor((z(x) R + 2^21) / 2^22), R = floor(2^46 /
 * sum z) (p_n when sum z = 0); decision = lowest x maximising p_n(x) times every
 * incoming message; permutation and stop rule as for Min-Max. */
typedef struct {
    int32_t max_iters;
    int32_t early_stop;
    int32_t schedule;
    int32_t rule;
    int32_t nms_num;
    int32_t nms_shift;
    int32_t oms_offset;
    int32_t msg_max;
    int32_t nb_msg_max;
} ldpcx_decode_params;

/* Validate `desc`, build the library's device structures (CSR/CSC, layer table, GF
 * tables) on the current device and return an opaque handle in *out.
 * Errors: LDPCX_E_INVAL (malformed H: unsorted or repeated columns, zero or out-of-range
 * coefficient, bad layer size, check degree < 2), LDPCX_E_UNSUPPORTED (degrees above the
 * limits), LDPCX_E_NOMEM, LDPCX_E_DEVICE. */
ldpcx_status ldpcx_code_create(const ldpcx_code_desc *desc, ldpcx_code **out);

/* Release a code handle (synchronises the device first).  NULL is accepted. */
ldpcx_status ldpcx_code_destroy(ldpcx_code *code);

/* Sizes of a code handle (host pointers, any may be NULL). */
ldpcx_status ldpcx_code_info(const ldpcx_code *code, int32_t *n, int32_t *m, int32_t *nnz,
                             int32_t *g, int32_t *max_dc, int32_t *max_dv);

/* Decode `batch` independent codewords (Algs. 2 / min-sum; the multicodeword mapping of
 * sec. 4: every codeword is an independent decoder).
 *   llr          device, g == 2: int8 [batch][n] channel LLRs;
 *                g > 2: int16 [batch][n][g] channel vectors gamma_n(x) = ln(p(eta)/p(x))
 *                quantised (Alg. 2 initialisation), entries in [0, 32767] with minimum 0
 *                over x (gamma_n(eta) = 0 at the most likely symbol eta; the decoders of
 *                codes whose variables all have degree 2 rely on it).
 *   hard         device, g == 2: uint8 [batch][ceil(n/8)], bit j of codeword b is bit
 *                (j % 8) (LSB first) of byte j / 8; padding bits are 0.
 *                g > 2: uint8 [batch][n] decided symbols.
 *   syndrome_ok  device uint8 [batch]: 1 when the final decision satisfies every check.
 *   iters        device int16 [batch]: iterations performed (0 when the channel decision
 *                already satisfied H and early_stop is on).
 *   schedule_used host int32*, may be NULL: the schedule actually run.
 * batch == 0 is a no-op.  The library may allocate a workspace on `stream` (stream-ordered
 * allocator). */
ldpcx_status ldpcx_decode(const ldpcx_code *code, const ldpcx_decode_params *params, int32_t batch,
                          const void *llr, void *hard, uint8_t *syndrome_ok, int16_t *iters,
                          int32_t *schedule_used, void *stream);

/* Same as ldpcx_decode, and additionally writes the final message state in canonical
 * CSR edge order (edge e = position in col_idx), for bit-exact comparison of every message:
 *   g == 2: msg_a = int8 q [batch][nnz] (q_e = clamp(Lambda - r_e)), msg_b = int8 r
 *           [batch][nnz], msg_c = int16 Lambda [batch][n].
 *   g > 2:  msg_a = int16 alpha [batch][nnz][g], msg_b = int16 beta [batch][nnz][g],
 *           msg_c unused (may be NULL); rule SPA: int32 Q24 u and v' [batch][nnz][g].
 * All message pointers are device memory.  Before the first iteration beta = r = 0. */
ldpcx_status ldpcx_debug_dump(const ldpcx_code *code, const ldpcx_decode_params *params,
                              int32_t batch, const void *llr, void *hard, uint8_t *syndrome_ok,
                              int16_t *iters, void *msg_a, void *msg_b, void *msg_c, void *stream);

/* Allocation-free variant of ldpcx_decode, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * Same arguments, layouts and results as ldpcx_decode (bit for bit), on the plan
 * ldpcx_decode would use.  The call allocates nothing: no hipMalloc, no stream-ordered
 * allocation, no graph capture.  Decoders that need a workspace take it from one static
 * device array of LDPCX_NOALLOC_SCRATCH_BYTES per GPU, held from the first call on that
 * GPU until the process ends; the batch then runs as consecutive chunks on `stream`
 * whose workspaces fit the array.  Every call on one GPU shares that GPU's array, so calls
 * that overlap on one GPU (other streams or threads, without ordering between them)
 * race and give wrong results: the caller serialises them.  Errors as ldpcx_decode, plus
 * LDPCX_E_UNSUPPORTED when the workspace of the smallest chunk the decoder allows (one
 * group of 256 codewords for long binary codes, one codeword otherwise) exceeds the array. */
#define LDPCX_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
ldpcx_status ldpcx_decode_noalloc(const ldpcx_code *code, const ldpcx_decode_params *params, int32_t batch,
                                  const void *llr, void *hard, uint8_t *syndrome_ok, int16_t *iters,
                                  int32_t *schedule_used, void *stream);

/* One job of a ragged batch: `batch` codewords of `code` with their own parameters and
 * buffers (same layouts as ldpcx_decode). */
typedef struct {
    const ldpcx_code *code;
    ldpcx_decode_params params;
    int32_t batch;
    const void *llr;
    void *hard;
    uint8_t *syndrome_ok;
    int16_t *iters;
} ldpcx_job;

/* Decode a ragged batch of jobs over different codes and sizes on `stream` (the
 * multicodeword mapping of sec. 4: independent decoders).  Jobs whose state fits one
 * workgroup run as items of the persistent kernel, with per-codeword early termination
 * inside: quasi-cyclic binary codes (2 x npairs codewords per item), other binary codes
 * held in LDS (cpw codewords per item), Min-Max over GF(4)..GF(64) whose messages of one
 * codeword fit a workgroup's LDS and that have at least 32 checks (one codeword per
 * item, every message in LDS) and FFT-SPA codes of the LDS-resident family (one group of
 * codewords per item).  Workgroups claim items longest first from a device counter
 * (one atomic add per item, never a wait for another workgroup), so the load stays
 * balanced when codewords stop early.  The kernel runs as up to five launches on the
 * stream, one per kind of item (binary; Min-Max of check degree <= 4, with or without
 * stored alphas; Min-Max of larger check degree; FFT-SPA), each with the occupancy its
 * own registers and LDS allow.  Jobs whose
 * state does not fit a workgroup (binary codes in the interleaved layout, GF(128) and
 * GF(256), larger codewords, FFT-SPA wave kernels) are gathered per (code, parameters,
 * resolved schedule) into one batch each and decoded by that batch's own launch
 * sequence on the same stream, after the persistent kernel.  Results are identical to
 * calling ldpcx_decode on each job; AUTO schedules are resolved per job as in
 * ldpcx_decode.  The library allocates stream-ordered scratch for the item tables and
 * the gathered batches and frees it on the stream. */
ldpcx_status ldpcx_decode_ragged(const ldpcx_job *jobs, int32_t njobs, void *stream);

/* Autotune the launch configuration of (code, params, batch) by timing the candidate
 * configurations on `stream` (synchronous).  The choice is cached per (code, params,
 * batch class) and used by later decode calls; when params->schedule is AUTO the
 * schedule is tuned too.  *chosen_schedule (may be NULL) receives the schedule and
 * *best_us (may be NULL) the measured time of the winner in microseconds. */
ldpcx_status ldpcx_tune(const ldpcx_code *code, const ldpcx_decode_params *params, int32_t batch,
                        int32_t *chosen_schedule, float *best_us, void *stream);

/* Launch configuration that the next decode of (code, params, batch) would use:
 * kernel family (0 = LDS-resident binary, 1 = interleaved binary, 2 = Min-Max (interleaved
 * up to GF(64), lanes over entries above), 4 = FFT-SPA (one wave per node and group of
 * codewords, lanes over entries; codewords per workgroup reports codewords per wave of
 * the check-node kernel), 5 = Min-Max
 * with one group of 64 codewords per workgroup and its messages in LDS (GF(4)..GF(64),
 * codes whose alpha and beta for 64 codewords fit 160 KB; 256, 512 or 1024 threads),
 * 6 = FFT-SPA with cw_per_wg codewords per workgroup and every vector in LDS, all
 * iterations in one launch (check and variable degrees <= 4, the vectors of cw_per_wg
 * codewords within 160 KB; 256, 512 or 1024 threads), 7 = Min-Max with one codeword per
 * workgroup, every message in LDS and the lanes over the field entries, all iterations
 * in one launch (GF(4)..GF(64), the messages of one codeword within 160 KB, stored in
 * signed 16 bits, or in 8 bits when nb_msg_max <= 255, which needs costs >= 0 as the
 * input contract states; without stored alphas when every variable has degree 2 and
 * each 64-lane group of threads holds at most two checks; a multiple of 64 threads up to
 * 1024, at most 256 used for check degrees above 4; both schedules),
 * 3 = packed two-codewords-per-lane binary for quasi-cyclic codes, available
 * when every layer of z rows consists of z x z circulant blocks, at most 16 layers and
 * 8 blocks per layer; threads = z * cw_per_wg / 2 * layers is its flooding kernel with the
 * layers in parallel), codewords per workgroup (family 1: codewords per launch
 * sequence; larger batches run as consecutive slices), threads per workgroup. */
ldpcx_status ldpcx_plan_info(const ldpcx_code *code, const ldpcx_decode_params *params,
                             int32_t batch, int32_t *family, int32_t *cw_per_wg,
                             int32_t *threads);

/* Pin the launch configuration used for (code, params, batch class) instead of the
 * default or tuned one.  family as in ldpcx_plan_info; cw_per_wg and threads are used by
 * family 0 (threads a multiple of 64 in [64, 1024]); cw_per_wg by family 3 (even, the
 * pairs' rows at most 512 threads; threads = z * cw_per_wg / 2 * layers selects the
 * flooding kernel with the layers in parallel when z * cw_per_wg / 2 is a multiple of 64
 * and the product at most 1024, else threads is ignored) and by family 1 (slice size, rounded up to a multiple
 * of 128 and capped by the batch and the 31-bit offset limit).  The pinned plan must be able to
 * run the requested schedule (LDPCX_E_UNSUPPORTED otherwise; families 1, 4 and 6 are
 * flooding only, families 2, 5 and 7 run the layered schedule up to GF(64)); family 5
 * takes threads = 256, 512 or 1024, family 7 a multiple of 64 up to 1024, family 6
 * cw_per_wg in [1, 64] and threads = 256, 512 or 1024.  Results never depend on the
 * plan. */
ldpcx_status ldpcx_plan_set(ldpcx_code *code, const ldpcx_decode_params *params, int32_t batch,
                            int32_t family, int32_t cw_per_wg, int32_t threads);

/* Measurement aid (no passage of the paper): run `blocks` workgroups of 256 threads
 * on `stream`, every lane doing `iters` rounds of 8 independent chains of one packed
 * 16-bit add and one packed 16-bit max (16 VALU wave instructions per round and
 * wave).  The caller times it to measure the device's VALU issue rate, the peak that
 * the integer rooflines are quoted against.  LDPCX_E_INVAL for non-positive sizes. */
ldpcx_status ldpcx_valu_probe(int32_t blocks, int32_t iters, void *stream);

/* ------------------------------------------------------------------ serving */
typedef struct ldpcx_server ldpcx_server;

/* Serving.  Sec. 4 lets every decoder start as soon as its codewords are available
 * instead of waiting for a full batch; the server does that on one GPU by admitting
 * requests into launches while earlier launches still run.
 *
 * Serving modes.
 *   CONTINUOUS: whenever one of the `max_inflight` launch slots is free and requests
 *     wait, the scheduler admits waiting codewords in arrival order while the free
 *     budget allows (a request that only partly fits is split at a codeword boundary)
 *     and launches them on the slot's stream: consecutive chunks of short codes as ONE
 *     ragged batch (ldpcx_decode_ragged: workgroup-local codes in its persistent
 *     kernel, small flooding Min-Max chunks gathered per code), capped at about 1.5 ms
 *     of estimated device time; a chunk of a long code (interleaved decoder), of
 *     FFT-SPA, of layered Min-Max or of more than 64 Min-Max codewords as a launch of
 *     its own (the plain decoder's launch sequence, parallel over checks).  Requests
 *     that arrive while launches are in flight are admitted into the next free slot
 *     without waiting for those launches to end, so their work overlaps on the device.
 *   PER_REQUEST: the one-code-per-launch baseline: one request (or budget-sized
 *     chunk of it) per launch through the plain decoder, one launch at a time, in
 *     arrival order.
 * Decoded results never depend on the mode, the mix or the chunking: every codeword
 * gets exactly what ldpcx_decode gives it alone. */
enum { LDPCX_SERVE_CONTINUOUS = 0, LDPCX_SERVE_PER_REQUEST = 1 };

typedef struct {
    size_t hbm_budget;     /* device bytes admitted work may hold at once: inputs, outputs
                            * and decoder workspaces of every chunk in flight */
    int32_t max_inflight;  /* launch slots (streams) in flight at once, >= 1 (PER_REQUEST: 1) */
    int32_t mode;          /* LDPCX_SERVE_* */
    int32_t max_launch_cw; /* cap on codewords per launch, 0 = only the budget caps it */
} ldpcx_server_config;

/* Create a server on the current device with its scheduler thread.  The code handles
 * of submitted requests stay resident on the device (they are the caller's handles;
 * keep them alive while requests use them).  LDPCX_E_INVAL for a bad configuration,
 * LDPCX_E_DEVICE when streams or events cannot be created. */
ldpcx_status ldpcx_server_create(const ldpcx_server_config *cfg, ldpcx_server **out);

/* Submit a request: `batch` codewords of `code` in HOST buffers with the layouts of
 * ldpcx_decode (llr_host read when the request is admitted, outputs written when it
 * completes; all must stay valid until then, or until a cancel returns).  Returns at
 * once with a ticket (thread-safe).  LDPCX_E_BUDGET when one codeword alone does not
 * fit the budget; parameter errors as ldpcx_decode.  batch = 0 completes at once. */
ldpcx_status ldpcx_server_submit(ldpcx_server *srv, const ldpcx_code *code,
                                 const ldpcx_decode_params *params, int32_t batch,
                                 const void *llr_host, void *hard_host, uint8_t *syndrome_ok_host,
                                 int16_t *iters_host, uint64_t *ticket);

/* *done = 1 when the request finished (its host outputs are complete). */
ldpcx_status ldpcx_server_poll(ldpcx_server *srv, uint64_t ticket, int32_t *done);

/* Block until the request finishes or `timeout_ms` elapses (< 0: no limit).  Returns the
 * request's final status (LDPCX_OK, LDPCX_E_CANCELLED, LDPCX_E_DEVICE ...) and releases
 * the ticket (a later poll or wait on it gives LDPCX_E_NOTFOUND), or LDPCX_E_TIMEOUT
 * and keeps it.  Timing of the request (submit, first admission into a launch,
 * completion with its outputs in host memory) is returned in microseconds since
 * server creation when the pointers are not NULL. */
ldpcx_status ldpcx_server_wait(ldpcx_server *srv, uint64_t ticket, int32_t timeout_ms,
                               double *t_submit_us, double *t_admit_us, double *t_done_us);

/* Cancel a request that has not completed: chunks still queued are dropped, chunks in
 * flight finish on the device but their outputs are discarded; the request completes
 * at once with LDPCX_E_CANCELLED and its host buffers are no longer touched.  Cancelling
 * a completed request is a no-op. */
ldpcx_status ldpcx_server_cancel(ldpcx_server *srv, uint64_t ticket);

/* Counters: requests completed, codewords decoded, launches, peak bytes admitted
 * (any pointer may be NULL). */
ldpcx_status ldpcx_server_stats(ldpcx_server *srv, uint64_t *completed, uint64_t *codewords,
                                uint64_t *launches, uint64_t *peak_bytes);

/* Cancel pending requests, wait for launches in flight, stop the scheduler thread
 * and free the server.  Tickets not yet waited on become invalid. */
ldpcx_status ldpcx_server_destroy(ldpcx_server *srv);

/* Message of the last failing call on this thread ("" if none). */
const char *ldpcx_last_error(void);

/* Library version string. */
const char *ldpcx_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LDPCX_H */
