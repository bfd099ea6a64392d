/*
 * epi.h -- C ABI of the MI355X (gfx950) exhaustive k-order epistasis scanner.
 *
 * The library enumerates every combination of `order` SNPs out of M, builds
 * each combination's contingency table (3^order genotype cells x {cases,
 * controls}) from bit-packed per-genotype, per-class individual masks with
 * bitwise AND and population count, scores every table by mutual information
 * and keeps the best `top_k` combinations.
 *
 * Paper (Ponte-Fernandez, Gonzalez-Dominguez, Martin, "A SIMD algorithm for
 * the detection of epistatic interactions of any order"):
 *   - genotype tables: Section 2.1 (one bit per individual, one row per
 *     genotype, cases and controls in separate subtables);
 *   - contingency tables: Section 2.2 (popcount of the AND of rows; the last
 *     level is fused with the popcount and never stored);
 *   - score: Section 2.3, Equations 1-3 (MI = H(X) + H(Y) - H(X,Y), natural
 *     logarithm, probabilities over all individuals, empty cells skipped);
 *   - exploration: Section 2.4, Algorithm 1 (every combination of the order
 *     exactly once; only the highest-MI combinations are kept), orders 2-8
 *     and every order up to a bound in one pass (epi_scan_orders);
 *   - segmented exploration: Section 3.4, Algorithm 2 (tables of a block
 *     counted first, then scored; EPI_BLOCK_SEGMENTED);
 *   - the steps as separate passes (epi_genotype_tables,
 *     epi_contingency_tables, epi_mutual_information), which Section 4
 *     times one by one.
 *
 * Conventions shared by every call:
 *   - Every function returns EPI_OK (0) or a negative EPI_E* status; no C++
 *     exception, abort or exit crosses this boundary.  epi_last_error()
 *     returns a message for the calling thread's most recent failure.
 *   - Genotypes are uint8 in {0,1,2}: homozygous dominant, heterozygous,
 *     homozygous recessive (the three genotype-table rows of Section 2.1).
 *     Phenotypes are uint8: 1 = case, 0 = control.
 *   - Host pointers are borrowed only for the duration of the call.  Device
 *     pointers (the *_device variants) must be readable by the context's
 *     device and stay valid until the call returns.
 *   - `stream` arguments are hipStream_t values passed as void*; NULL selects
 *     the context's own stream.  Work is ordered after prior work on that
 *     stream.
 *   - Results are ordered best first: larger MI, then the lexicographically
 *     smaller combination (ascending SNP indices).
 *   - A contingency table is returned as 2 x 3^order uint32 counts: cases
 *     first, then controls; cell index x = sum_t g_t * 3^(order-1-t), first
 *     SNP most significant (the row index i*3+j used when a SNP is added to a
 *     genotype table, Section 2.1).
 *   - Scores are float32 values of MI in nats.
 */
#ifndef EPI_H
#define EPI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define EPI_OK 0
#define EPI_EINVAL (-1)       /* invalid argument or input value            */
#define EPI_ENOMEM (-2)       /* device memory budget or allocation failed  */
#define EPI_EDEVICE (-3)      /* HIP runtime error                          */
#define EPI_EUNSUPPORTED (-4) /* valid request outside the built limits     */
#define EPI_ENOTREADY (-5)    /* result not available yet                   */
#define EPI_ENOTFOUND (-6)    /* unknown dataset / scan / batch / request   */

/* ---- limits -------------------------------------------------------------- */
#define EPI_MIN_ORDER 2
#define EPI_MAX_ORDER 8
/* Largest order the server accepts (its per-request result blocks are sized
 * for it). */
#define EPI_SERVE_MAX_ORDER 5
#define EPI_MAX_TOP_K 256
/* A combination is keyed by its indices packed big-endian into 64 bits with
 * floor(64/order) bits each, so M may not exceed 2^floor(64/order)
 * (order 5: M <= 4096). */

typedef struct epi_ctx epi_ctx;

/* Message of the calling thread's last failed call ("" if none).  The pointer
 * stays valid until the thread's next call into the library. */
const char *epi_last_error(void);

/* Library version string. */
const char *epi_version(void);

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device`.  `hbm_budget_bytes` caps the
 * device memory the context may hold at once (datasets + scan buffers);
 * 0 = 90% of the device's free memory at creation.  *out receives the
 * handle.  Errors: EINVAL (bad device / null out), EDEVICE. */
int epi_create(int32_t device, uint64_t hbm_budget_bytes, epi_ctx **out);

/* Wait for all work of the context, then free every dataset, scan, batch and
 * server it owns.  NULL is accepted. */
int epi_destroy(epi_ctx *ctx);

/* Device memory currently held by the context and its budget, in bytes. */
int epi_memory(epi_ctx *ctx, uint64_t *used_bytes, uint64_t *budget_bytes);

/* ---- datasets (Section 2.1: genotype tables) ---------------------------- */

/* Pack a dataset into device-resident genotype masks.
 * geno: host, M rows of N genotypes, row stride `ld` bytes (ld >= N).
 * pheno: host, N phenotypes.  Individuals keep their input order within each
 * class.  The packed masks stay on the device until epi_unload/epi_destroy.
 * Errors: EINVAL (M < 1, N < 2, ld < N, a genotype not in {0,1,2}, a
 * phenotype not in {0,1}, no case or no control), ENOMEM, EDEVICE.
 * *dataset_id receives the handle. */
int epi_load_genotypes(epi_ctx *ctx, const uint8_t *geno, int64_t ld, const uint8_t *pheno, int32_t M,
                       int32_t N, int32_t *dataset_id);

/* Same as epi_load_genotypes with geno/pheno in device memory (e.g. torch
 * tensors).  Synchronises `stream` once to validate the input. */
int epi_load_genotypes_device(epi_ctx *ctx, const uint8_t *d_geno, int64_t ld, const uint8_t *d_pheno,
                              int32_t M, int32_t N, void *stream, int32_t *dataset_id);

/* Repack new genotypes and phenotypes into an existing dataset, from device
 * memory, asynchronously on `stream` (no allocation, no synchronisation).
 * d_geno must hold the dataset's M rows of N genotypes (row stride ld >= N)
 * and d_pheno its N phenotypes with the dataset's number of cases; the
 * library cannot see the size of a device buffer, so a smaller buffer is
 * read past its end.  The values are checked on the device while they are
 * packed: a genotype outside {0,1,2}, a phenotype outside {0,1} or a
 * different number of cases makes the results call of every scan of the
 * dataset that runs after this repack (epi_results, epi_batch_results,
 * epi_server_results) fail with EINVAL, until a repack with valid input.
 * Errors: ENOTFOUND, EINVAL (null pointer, ld < N). */
int epi_repack_device(epi_ctx *ctx, int32_t dataset_id, const uint8_t *d_geno, int64_t ld,
                      const uint8_t *d_pheno, void *stream);

/* Free a dataset: waits for device work of scans and batches that still read
 * it (a batch that names it can no longer run).  EINVAL while a server
 * request on it is queued or running (its memory stays valid until the
 * request is done). */
int epi_unload(epi_ctx *ctx, int32_t dataset_id);

/* Shape of a dataset and the device bytes it holds. */
int epi_dataset_info(epi_ctx *ctx, int32_t dataset_id, int32_t *M, int32_t *N, int32_t *n_cases,
                     uint64_t *device_bytes);

/* ---- scans (Algorithm 1 + Sections 2.2-2.3) ----------------------------- */

typedef struct {
    int32_t dataset_id;
    int32_t order; /* EPI_MIN_ORDER..EPI_MAX_ORDER */
    int32_t top_k; /* 1..EPI_MAX_TOP_K */
    int32_t reserved; /* must be 0 */
} epi_scan_desc;

/* Start one exhaustive scan of `order` over a dataset, keeping the best
 * `top_k` combinations (plain launch).  Asynchronous on `stream`; poll with
 * epi_query or block with epi_wait.  *scan_id receives the handle.
 * Errors: ENOTFOUND (dataset), EINVAL (order < 2 or > M, top_k < 1),
 * EUNSUPPORTED (order > EPI_MAX_ORDER, top_k > EPI_MAX_TOP_K, M too large
 * for the order's key width), ENOMEM, EDEVICE. */
int epi_scan(epi_ctx *ctx, int32_t dataset_id, int32_t order, int32_t top_k, void *stream,
             int32_t *scan_id);

/* Start n scans as ONE persistent launch fed by a device-side work queue,
 * captured once into a HIP graph.  scan_ids[i] receives the handle of
 * descs[i]; each behaves like a scan from epi_scan.  Same errors as
 * epi_scan, checked for every descriptor before anything is launched. */
int epi_scan_batch(epi_ctx *ctx, const epi_scan_desc *descs, int32_t n, void *stream, int32_t *scan_ids);

/* Every order from 2 to max_order in one pass (a search up to a given
 * combination size): one scan per order, launched together as by
 * epi_scan_batch; scan_ids[o - 2] receives the scan of order o, each waited
 * for, read and released on its own.  The order-2 results are scored by the
 * pair sub-table pass that the order-3 (or order-4) scan runs anyway, so the
 * pairs are counted once.  Errors as epi_scan for each order (EINVAL for
 * max_order < 2 or above M, EUNSUPPORTED above EPI_MAX_ORDER). */
int epi_scan_orders(epi_ctx *ctx, int32_t dataset_id, int32_t max_order, int32_t top_k, void *stream,
                    int32_t *scan_ids);

/* *done = 1 when the scan's results are ready, else 0. */
int epi_query(epi_ctx *ctx, int32_t scan_id, int32_t *done);

/* Block until the scan's results are ready. */
int epi_wait(epi_ctx *ctx, int32_t scan_id);

/* Copy a finished scan's results into caller buffers.
 * combos: capacity * order int32 (ascending SNP indices per row);
 * scores: capacity float (MI, nats); tables: nullable, capacity * 2 *
 * 3^order uint32.  *n_written = min(capacity, top_k, C(M, order)).
 * Errors: ENOTFOUND, ENOTREADY (not finished; call epi_wait), EINVAL. */
int epi_results(epi_ctx *ctx, int32_t scan_id, int32_t capacity, int32_t *combos, float *scores,
                uint32_t *tables, int32_t *n_written);

/* Device timings of a finished scan in milliseconds (HIP events on the
 * scan's stream): ms[0] whole scan, ms[1] sub-table pass, ms[2] main
 * counting/scoring kernel, ms[3] top-K merge + result tables.  Entries that
 * do not apply (or scans run inside a batch graph) are -1. */
int epi_scan_timing(epi_ctx *ctx, int32_t scan_id, float ms[4]);

/* Number of combinations C(M, order) of a scan and the kernel variant it ran
 * (0 = per-combination generic kernel, 1 = order-2 reduced-cell kernel,
 * 2 = order-3 reduced-cell kernel) and its prefix block. */
int epi_scan_info(epi_ctx *ctx, int32_t scan_id, uint64_t *n_combinations, int32_t *variant,
                  int32_t *prefix_block);

/* Free a scan's buffers (waits for it first). */
int epi_release(epi_ctx *ctx, int32_t scan_id);

/* ---- completeness check (Algorithm 1: every combination exactly once;
 *      Section 2.2: each with its contingency table) ---------------------- */

/* Start a scan exactly as epi_scan does (same kernel choice, same results,
 * read with epi_wait / epi_results / epi_release), with the checking build
 * of its counting kernels: they also count every combination they score and
 * add up a digest of it and its table.  For a combination c_1 < ... < c_k
 * with table T[class][x] (class 0 = cases, x the cell index of epi_results)
 *   h = mix64(... mix64(mix64(c_1 + 1) + c_2 + 1) ... + c_k + 1),
 *   s = sum over class, x of T[class][x] * mix64(2 x + class + 1),
 *   contribution = mix64(h XOR s),
 * all modulo 2^64, mix64 being the output function of SplitMix64 (Steele,
 * Lea and Flood, 2014).  The scan's digest is the sum of the contributions,
 * independent of the order of the visit, so it can be compared with a
 * count-and-digest of every combination computed any other way.  Slower
 * than epi_scan (it is a check, not the production path).  Errors as
 * epi_scan. */
int epi_scan_check(epi_ctx *ctx, int32_t dataset_id, int32_t order, int32_t top_k, void *stream,
                   int32_t *scan_id);

/* Count of combinations scored and their digest, of a finished scan started
 * by epi_scan_check.  Errors: ENOTFOUND, ENOTREADY (not finished), EINVAL
 * (a scan not started by epi_scan_check, null output). */
int epi_scan_digest(epi_ctx *ctx, int32_t scan_id, uint64_t *n_scored, uint64_t *digest);

/* ---- allocation-free scan ------------------------------------------------ */

/* Bytes of the scratch array that every device holds for epi_scan_noalloc,
 * from the library's load until the process ends (128 MiB). */
#define EPI_NOALLOC_SCRATCH_BYTES 134217728

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  The same
 * scan as epi_scan (same combinations, scores and tables), enqueued on
 * `stream` (NULL: the context's) without allocating anything: no hipMalloc,
 * hipFree, pinned host memory or events.  Every intermediate buffer (work
 * queues, candidate lists, pair and triplet sub-tables, descriptor tables the
 * context has not cached yet, the result block) is carved from the device's
 * scratch array of EPI_NOALLOC_SCRATCH_BYTES.  Outputs are caller-owned
 * device buffers, written when the stream reaches the scan's end:
 *   d_combos: top_k * order int32, d_scores: top_k float,
 *   d_tables: nullable, top_k * 2 * 3^order uint32 (layout of epi_results),
 *   d_n: one int32, the number of results (min(top_k, C(M, order))), or -1
 *        when the dataset's last packing had invalid input.
 * The call returns once the work is enqueued; synchronise the stream before
 * reading the outputs.  Every call on a device shares that device's array and
 * it keeps the last call's contents (each call clears what must start at
 * zero), so calls that overlap on one device race: serialise them (one
 * stream, or a wait between them).  Served-style kernel choice: the fused
 * kernels (segmented pins are ignored), and order 4 by reduced cells only
 * when its sub-tables fit in half the array (else all cells; same results).
 * Errors: as epi_scan, and EUNSUPPORTED when the scan's buffers exceed the
 * array (the pair sub-table alone takes 32 C(M, 2) bytes at orders 3-4; order
 * 3 at M = 1000 takes about 25 MB in all). */
int epi_scan_noalloc(epi_ctx *ctx, int32_t dataset_id, int32_t order, int32_t top_k, void *stream,
                     int32_t *d_combos, float *d_scores, uint32_t *d_tables, int32_t *d_n);

/* ---- re-runnable batches ------------------------------------------------- */

/* Build a batch of n scans once: work queue, per-scan buffers and (if
 * use_graph) a captured HIP graph of the whole launch sequence.  Run it with
 * epi_batch_run any number of times; each run overwrites the results.
 * persistent = 1: all scans in one persistent launch (what epi_scan_batch
 * does); 0: back-to-back plain launches, one per scan. */
int epi_batch_create(epi_ctx *ctx, const epi_scan_desc *descs, int32_t n, int32_t persistent,
                     int32_t use_graph, int32_t *batch_id);
int epi_batch_run(epi_ctx *ctx, int32_t batch_id, void *stream);
int epi_batch_wait(epi_ctx *ctx, int32_t batch_id);
/* Results of scan `index` of the batch; same layout as epi_results. */
int epi_batch_results(epi_ctx *ctx, int32_t batch_id, int32_t index, int32_t capacity, int32_t *combos,
                      float *scores, uint32_t *tables, int32_t *n_written);
/* Device milliseconds of the batch's last run (events around the run). */
int epi_batch_timing(epi_ctx *ctx, int32_t batch_id, float *ms);
int epi_batch_destroy(epi_ctx *ctx, int32_t batch_id);

/* ---- autotuner ----------------------------------------------------------- */

/* Counting kernels by prefix block (the number of first SNPs a work item
 * shares; Section 2.4 reuses such prefixes of the enumeration):
 *   order 2: 2, 4, 8 -- popcount kernels; 16 (EPI_BLOCK_MFMA_FP4) -- the four
 *            reduced pair cells as 0/1 matrix products on the matrix cores
 *            (the order-3 products below without the middle SNP's mask;
 *            datasets with fewer than 2^22 individuals);
 *   order 3: 1, 2, 4, 8 -- popcount kernels (Section 2.2: AND + popcount);
 *            16 (EPI_BLOCK_MFMA_FP4) -- the reduced cells as 0/1 matrix
 *            products on the matrix cores, 4-bit float operands (1.0 = 0x2),
 *            exact float32 sums (datasets with fewer than 2^22 individuals);
 *            32 (EPI_BLOCK_MFMA_I8) -- the same products with 8-bit integer
 *            operands and int32 sums (never chosen by the autotuner: it
 *            moves twice the operand bytes of the 4-bit form for the same
 *            products);
 *            48 (EPI_BLOCK_MFMA_FP4_2J) -- the 4-bit products with two
 *            consecutive middle SNPs per work item, so each operand load
 *            feeds twice the products; the control steps' products are
 *            scaled by 2^(T-2) (the matrix instruction's exponent scale), so
 *            one float accumulator holds 4 n(cases) + 2^T n(controls), T = 2
 *            + the bit width of the case count: only for datasets where
 *            4 n_cases + 2^T n_controls < 2^24 (e.g. up to 2047 individuals
 *            per class).
 * Every kernel produces the same integers and therefore the same results.
 * Plain scans on the matrix-core blocks with at least 64 work items per wave
 * first run a pilot pass: one work item per wave, from the middle of the
 * scan, whose best screening sums, lowered by the screen's error bound, go
 * into the scan's score histogram; the K-th best of those is a lower bound
 * of the final K-th best score, which every wave of the scan then starts
 * from (same results, fewer combinations scored exactly while the bound
 * rises). */
#define EPI_BLOCK_MFMA_FP4 16
#define EPI_BLOCK_MFMA_I8 32
#define EPI_BLOCK_MFMA_FP4_2J 48
/* Any order: the segmented exploration of Section 3.4 (Algorithm 2).  Each
 * wave counts the full 2 x 3^k tables of a block of 64 combinations into a
 * device buffer, then scores the block (the fused kernels score each table as
 * it is counted).  Same results; the buffer takes 2 x 3^k x 256 bytes per
 * wave of the launch (order 8: 3.4 MB).  Block 0 restores the built-in
 * choice for the order.  Served requests (epi_server_*) always use the fused
 * kernels. */
#define EPI_BLOCK_SEGMENTED 64
/* Orders 4-8: the per-combination kernel that counts all 3^order cells of a
 * combination's table with AND + popcount (Section 2.2 as written).  It is
 * the built-in choice from order 5 on; order 4 uses the reduced-cell kernel
 * (the cells with genotypes 0 and 1 counted, the others by
 * inclusion-exclusion from the pair and triplet sub-tables) when its
 * triplet sub-table fits, and this block pins the all-cell kernel instead. */
#define EPI_BLOCK_ALL_CELLS 81

/* Time every counting kernel of `order` on the dataset's own scan and
 * remember the fastest for datasets of the same size bucket (the same
 * power-of-two buckets of 32-bit words per SNP row and of the number of
 * SNPs).
 * The candidates are the blocks listed above: order 2 prefix blocks 2, 4, 8
 * and EPI_BLOCK_MFMA_FP4;
 * order 3 blocks 1, 2, 4, 8, EPI_BLOCK_MFMA_FP4 and EPI_BLOCK_MFMA_FP4_2J;
 * order 4 the reduced-cell
 * kernel (reported as 0), EPI_BLOCK_ALL_CELLS and EPI_BLOCK_SEGMENTED;
 * orders 5-8 EPI_BLOCK_ALL_CELLS and EPI_BLOCK_SEGMENTED.  Each is timed on
 * eight slices of work items spread evenly over the whole scan (each about
 * 8 items per wave of the launch, or an eighth of the scan if that is less)
 * and its time divided by the
 * combinations those items score (counted on the host), so kernels whose
 * items hold different numbers of combinations compare fairly.  The choice
 * is also written to the cache file named by EPI_TUNE_CACHE (if set).  Scans
 * (plain, batched and served) use tuned choices automatically; untuned
 * shapes use built-in defaults (order 3: the matrix-core kernel where
 * available).  *choice receives the chosen block. */
int epi_autotune(epi_ctx *ctx, int32_t dataset_id, int32_t order, int32_t *choice);

/* The candidates of the last epi_autotune of `order` for the dataset's size
 * bucket and their measured cost in nanoseconds per scored combination, in
 * the order they were timed: blocks[i], ns_per_combination[i] for i <
 * min(capacity, *n_candidates).  Errors: ENOTFOUND (no such autotune),
 * EINVAL. */
int epi_autotune_report(epi_ctx *ctx, int32_t dataset_id, int32_t order, int32_t capacity, int32_t *blocks,
                        double *ns_per_combination, int32_t *n_candidates);

/* Pin the counting kernel for `order` on datasets of the same bucket as
 * `dataset_id`, as if the autotuner had chosen `block` (one of the blocks
 * listed above; orders above 3 take EPI_BLOCK_SEGMENTED, EPI_BLOCK_ALL_CELLS
 * and 0).  EPI_BLOCK_MFMA_I8 builds the dataset's integer
 * operand copies on the context stream and waits for them (no other work on
 * the dataset may be in flight).  EPI_EINVAL for a block not listed for the
 * order, EPI_EUNSUPPORTED for a matrix-core block on a dataset with 2^22
 * individuals or more and for EPI_BLOCK_MFMA_FP4_2J on one whose class sizes
 * do not fit its accumulator, EPI_ENOMEM if the copies do not fit. */
int epi_set_prefix_block(epi_ctx *ctx, int32_t dataset_id, int32_t order, int32_t block);

/* ---- the steps of the method as separate passes ------------------------- */

/* Each of these takes n combinations of `order` SNP indices of a resident
 * dataset on the device (int32 [n][order]; any indices in [0, M), in any
 * order), runs on the context stream and returns when it is done;
 * *kernel_ms (may be null) receives the kernel's time.  Output buffers are
 * device memory owned by the caller.  EPI_EINVAL for an order outside the
 * listed range, a null buffer, or an index outside [0, M) (that
 * combination's output is left unwritten), EPI_ENOTFOUND for an unknown
 * dataset, EPI_EDEVICE for a HIP error.  n = 0 does nothing. */

/* Genotype tables (Section 2.1; Algorithm 1 builds them one SNP at a time):
 * for each combination, row x for each of the 3^order genotype combinations
 * (x in base 3, the first SNP's genotype the leading digit) is the set of
 * individuals with those genotypes, cases then controls, as bitsets.
 * d_rows: uint32 [n][3^order][W], W = W0 + W1 with W0 = 4 ceil(n_cases / 128)
 * and W1 = 4 ceil(n_controls / 128); bit b of word w < W0 is case 32 w + b,
 * bit b of word W0 + w is control 32 w + b (each class in input order); bits
 * past a class's size are 0.  order 1 .. EPI_MAX_ORDER. */
int epi_genotype_tables(epi_ctx *ctx, int32_t dataset_id, int32_t order, const int32_t *d_combos, uint64_t n,
                        uint32_t *d_rows, float *kernel_ms);

/* Contingency tables (Section 2.2): d_tables uint32 [n][2][3^order], class 0
 * = cases, the cell order of the genotype tables (and of epi_results).
 * order 2 .. EPI_MAX_ORDER. */
int epi_contingency_tables(epi_ctx *ctx, int32_t dataset_id, int32_t order, const int32_t *d_combos, uint64_t n,
                           uint32_t *d_tables, float *kernel_ms);

/* Mutual information (Section 2.3, Equation 1, natural logarithm) of n
 * contingency tables of the dataset, uint32 [n][2][3^order] on the device,
 * into d_mi (double [n], device).  It is the exact fixed-point sum the scans
 * rank by, scaled to nats, so it matches a scan's score of the same
 * combination to the float rounding of that score.  EPI_EINVAL if a table's
 * classes do not sum to the dataset's class sizes (its d_mi entry is NaN).
 * order 2 .. EPI_MAX_ORDER. */
int epi_mutual_information(epi_ctx *ctx, int32_t dataset_id, int32_t order, const uint32_t *d_tables, uint64_t n,
                           double *d_mi, float *kernel_ms);

/* ---- serving: continuous batching -------------------------------------- */

typedef struct {
    int32_t max_active;        /* requests resident on the device at once (>= 1) */
    int32_t rounds_in_flight;  /* launch rounds on the device at once: 1 = the host
                                * reads a round's results before it builds the next
                                * (new requests join at the next round); 2 = it
                                * builds and enqueues the next round while the
                                * device runs the current one (no device idle
                                * between rounds; a request that arrives meanwhile
                                * waits one round more); 0 = 2 while the next round
                                * is short, else 1.  EINVAL outside 0..2. */
    uint64_t request_budget;   /* device bytes for request buffers (0 = ctx budget) */
} epi_server_config;

/* Start a server thread that admits requests by device-memory footprint and
 * runs every admitted request's work as slices of shared persistent launches
 * (continuous batching: requests join and leave between launch rounds). */
int epi_server_start(epi_ctx *ctx, const epi_server_config *cfg, int32_t *server_id);

/* Enqueue a scan request on a resident dataset; thread-safe, non-blocking.
 * Same argument checks as epi_scan, and EUNSUPPORTED for an order above
 * EPI_SERVE_MAX_ORDER. */
int epi_server_submit(epi_ctx *ctx, int32_t server_id, int32_t dataset_id, int32_t order, int32_t top_k,
                      int32_t *request_id);

/* *state: 0 queued, 1 admitted (on the device), 2 done. */
int epi_server_poll(epi_ctx *ctx, int32_t server_id, int32_t request_id, int32_t *state);

/* Results of a finished request (layout as epi_results) and its latency in
 * milliseconds from submission to results ready (nullable).  The request is
 * freed after this call.  Errors: ENOTREADY, ENOTFOUND. */
int epi_server_results(epi_ctx *ctx, int32_t server_id, int32_t request_id, int32_t capacity,
                       int32_t *combos, float *scores, uint32_t *tables, int32_t *n_written,
                       double *latency_ms);

/* Counters: [0] requests done, [1] launch rounds, [2] combos*individuals done,
 * [3] peak request bytes, [4] peak concurrently admitted requests. */
int epi_server_stats(epi_ctx *ctx, int32_t server_id, uint64_t out[5]);

/* Finish all submitted requests, then stop the server thread. */
int epi_server_stop(epi_ctx *ctx, int32_t server_id);

#ifdef __cplusplus
}
#endif

#endif /* EPI_H */
