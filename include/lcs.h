/*
 * lcs.h -- C ABI of an MI355X (gfx950) engine for the longest common
 * subsequence of two strings, following the grid-graph method of
 * "Parallel Longest Common SubSequence Analysis In Chapel" (arXiv 2309.09072),
 * itself a variant of Lu and Lin's first parallel algorithm.
 *
 * Problem (Section I): two strings over a finite alphabet in; the length of a
 * longest common subsequence and one such subsequence (a "witness") out.
 *
 * Method (Section II): the LCS is the heaviest path from the top-left to the
 * bottom-right vertex of the grid graph whose diagonal edges (weight 1) sit
 * where the symbols match (Section II-A, Fig. 1).  For a horizontal strip of
 * rows, the breakout matrix D(i, j) holds the leftmost bottom-row column that a
 * path of weight j can reach from top-row column i (Section II-B-1).  Strips of
 * base_rows rows are built by appending rows with per-symbol next-match tables
 * (the base case of Section II-B-3) or, with identical results, from a combed
 * seaweed permutation of the strip (single pairs and staged batches); adjacent
 * strips are merged with the combine equation of
 * Section II-B-1 up to the whole grid, the length is read off the top matrix,
 * and the witness comes from the cross vertices found by a recursive midpoint
 * search (Sections II-C to II-E).
 *
 * Conventions shared by every call:
 *   - a is the ROW string (length m), b the COLUMN string (length n).  Symbols
 *     are uint8 codes 0..alphabet-1.  Swapping a and b leaves the length
 *     unchanged but may change the witness.
 *   - Columns and breakouts are 0-indexed vertex columns 0..n.  "Unreachable"
 *     (the paper's infinity) is stored as n + 1.
 *   - The caller owns every device buffer (inputs, outputs, workspace); the
 *     library never allocates or frees device memory.  Workspaces are plain
 *     device allocations of the size the planning call reports.
 *   - Device work is enqueued on the caller's HIP stream (a hipStream_t passed
 *     as void*, NULL = the null stream) and is asynchronous unless stated.
 *     Device outputs are valid once that stream has been synchronised.
 *   - Every call returns an int32 status: LCS_OK or a negative LCS_E_* code.
 *     No C++ exception or abort crosses this interface.
 *   - A plan, batch or server handle is not thread-safe; distinct handles are
 *     independent.
 */
#ifndef LCS_H_
#define LCS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
#define LCS_OK 0
#define LCS_E_INVAL (-1)     /* bad argument: null pointer, size or alphabet out of range */
#define LCS_E_TOO_BIG (-2)   /* sizes exceed the plan, or an index would not fit in int32 */
#define LCS_E_WORKSPACE (-3) /* workspace smaller than required */
#define LCS_E_HIP (-4)       /* a HIP runtime call or kernel launch failed */
#define LCS_E_SYMBOL (-5)    /* a symbol >= alphabet was found on the device */
#define LCS_E_CAPACITY (-6)  /* witness output buffer too small */
#define LCS_E_STATE (-7)     /* call out of order (e.g. length before any build) */
#define LCS_E_NOMEM (-8)     /* host memory allocation failed */
#define LCS_E_BUDGET (-9)    /* serving: request does not fit the memory budget */
#define LCS_E_AGAIN (-10)    /* serving: queue full, try again after polling */

/* Human-readable name of a status code (static storage, never NULL). */
const char *lcs_status_string(int32_t status);

/* ============================================================ single pair */

typedef struct lcs_plan_s *lcs_plan_t;

typedef struct lcs_plan_desc {
    int32_t max_m;     /* largest row-string length the plan accepts, >= 0 */
    int32_t max_n;     /* largest column-string length, >= 0 */
    int32_t alphabet;  /* number of symbol codes, 1..256 */
    int32_t base_rows; /* rows per base strip (Section II-B-3 generalised to
                          base_rows rows): 16, 32, 64, 128, 256, 512 or 1024;
                          0 selects by the sizes built (rows = max_m and
                          columns = max_n, or the shorter and longer of the two
                          with LCS_PLAN_ORIENT): 1024 from 8192 rows, 512 from
                          4096 rows with 8192 columns, 256 from 4096 rows, else
                          64 */
    int32_t tile;      /* vertices per search tile of the combine: power of two
                          in 4..32; 0 selects the default (32) */
    uint32_t flags;    /* 0 or an OR of LCS_PLAN_PROFILE, LCS_PLAN_ORIENT */
} lcs_plan_desc;

#define LCS_PLAN_PROFILE 1u /* record HIP events around every kernel of a build/trace */
#define LCS_PLAN_ORIENT 2u  /* when m > n, build the problem of reversed b (rows) against
                               reversed a (columns): the recursion depth follows the
                               shorter string (Section II-C: depth grows with log m).
                               The length is the same, and the witness is mapped back
                               to a's and b's indices: the canonical witness of the
                               reversed, transposed problem is the canonical witness of
                               (a, b) read backwards.  lcs_semilocal is then not
                               available (LCS_E_STATE) and lcs_dist_view shows the
                               matrices of the problem that was built. */

/*
 * Plan the breakout-matrix recursion for strings up to max_m x max_n.
 * On success *out receives a new plan (host memory only) and *workspace_bytes
 * the exact device workspace size needed by lcs_dist_build for the largest
 * sizes: every level of the strip recursion (all kept for the trace), a
 * sentinel row per matrix, the next-match tables and search/trace scratch.
 * Errors: LCS_E_INVAL (null pointer, negative size, alphabet outside 1..256,
 * unsupported base_rows or tile), LCS_E_TOO_BIG (a matrix would have 2^30 or
 * more cells, or max_n >= 2^24 - 2), LCS_E_NOMEM.
 */
int32_t lcs_plan(const lcs_plan_desc *desc, lcs_plan_t *out, size_t *workspace_bytes);

/* Workspace size for one pair of exact sizes (m, n) <= the plan's maxima. */
int32_t lcs_plan_workspace(lcs_plan_t plan, int32_t m, int32_t n, size_t *workspace_bytes);

/* The plan's descriptor with its defaults resolved (base_rows and tile as the
 * builds use them) written to *out.  Errors: LCS_E_INVAL (null pointer). */
int32_t lcs_plan_describe(lcs_plan_t plan, lcs_plan_desc *out);

/* Release a plan (host memory only; the workspace stays the caller's). */
int32_t lcs_plan_destroy(lcs_plan_t plan);

/*
 * Build every breakout matrix of the strip recursion for the pair (a, b):
 * the per-symbol next-match tables (Section II-B-3 base case; the trace reads
 * them), the base strips of base_rows rows (from each strip's seaweed
 * combing: the breakout rows that appending the rows one at a time with those
 * tables gives), then the combine equation of Section II-B-1 level by
 * level up to the whole grid, whose argmin search follows the monotone-matrix
 * property of Section II-B-1 (Alg. 1 and Alg. 2 for every tile-th vertex,
 * bracketed searches in between), and finally the LCS length.
 *   a, b       device pointers to m and n symbol codes (may be NULL when the
 *              length is 0).
 *   workspace  device pointer, at least lcs_plan_workspace(plan, m, n) bytes,
 *              256-byte aligned.  It must stay allocated and untouched while
 *              lcs_length / lcs_trace / lcs_dist_view use this build.
 * m = 0 or n = 0 is legal: no device work, length 0.
 * Errors: LCS_E_INVAL, LCS_E_TOO_BIG (m or n above the plan's maxima),
 * LCS_E_WORKSPACE, LCS_E_HIP.  A symbol >= alphabet is only detected on the
 * device and reported as LCS_E_SYMBOL by the next lcs_length or lcs_trace.
 */
int32_t lcs_dist_build(lcs_plan_t plan, const uint8_t *a, int32_t m, const uint8_t *b, int32_t n,
                       void *workspace, size_t workspace_bytes, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same as
 * lcs_dist_build, with the workspace taken from a device array that the
 * library holds itself, LCS_NOALLOC_WORKSPACE_BYTES long, one copy on each GPU
 * it runs on (the current device's copy is used; the stream must belong to
 * it), kept until the process ends.  It allocates nothing and calls no
 * allocating routine.  Every call on a GPU shares that GPU's array: calls that
 * overlap on one GPU race, and the build's matrices stay readable by
 * lcs_length, lcs_trace, lcs_trace_device, lcs_semilocal, lcs_path and
 * lcs_dist_view of this plan only until the next lcs_dist_build_noalloc on the
 * same GPU (with any plan) overwrites them.  Everything that must start at
 * zero is cleared by the build itself, with kernels (no memset).
 * Errors: those of lcs_dist_build, and LCS_E_WORKSPACE when
 * lcs_plan_workspace(plan, m, n) exceeds LCS_NOALLOC_WORKSPACE_BYTES (about
 * 1450 x 1450 symbols with 64-row base strips); LCS_E_HIP if the array cannot
 * be found on the current device.
 */
#define LCS_NOALLOC_WORKSPACE_BYTES ((size_t)64 << 20)
int32_t lcs_dist_build_noalloc(lcs_plan_t plan, const uint8_t *a, int32_t m, const uint8_t *b,
                               int32_t n, void *stream);

/*
 * LCS length of the last build: the largest weight j whose breakout from top
 * vertex 0 of the whole grid is reachable (Sections II-B-1 and II-C).
 * Copies it to *length_host and SYNCHRONISES the stream.
 * Errors: LCS_E_STATE (no build), LCS_E_SYMBOL, LCS_E_HIP.
 */
int32_t lcs_length(lcs_plan_t plan, int32_t *length_host, void *stream);

/* Same value written to device memory *length_dev, asynchronously (graph-safe). */
int32_t lcs_length_device(lcs_plan_t plan, int32_t *length_dev, void *stream);

/*
 * One witness of the last build via the recursive midpoint-vertex search
 * (Section II-D): at every split of a strip into upper and lower halves the
 * cross vertex on the boundary row is taken with the smallest upper weight
 * (the tie rule of Alg. 2), which yields the optimal path entering every row
 * as far left as possible; inside a base strip the same rule is applied row by
 * row.  The diagonal (weight 1) edges of that path are the matched pairs
 * (Section II-E): a_idx[t], b_idx[t] (device int32 arrays) receive them in
 * increasing order, t = 0..L-1, with a[a_idx[t]] == b[b_idx[t]].
 * capacity must be >= min(m, n).  *length_host receives L (the stream is
 * SYNCHRONISED).
 * Errors: LCS_E_STATE, LCS_E_CAPACITY, LCS_E_INVAL, LCS_E_SYMBOL, LCS_E_HIP.
 */
int32_t lcs_trace(lcs_plan_t plan, int32_t *a_idx, int32_t *b_idx, int32_t capacity,
                  int32_t *length_host, void *stream);

/*
 * Witness of the last build, enqueued only (no synchronisation; usable inside
 * a captured graph).  Writes L to device memory *length_dev; a_idx and b_idx
 * as for lcs_trace.  Errors are the argument errors of lcs_trace; a device
 * error is reported by the next lcs_length.
 */
int32_t lcs_trace_device(lcs_plan_t plan, int32_t *a_idx, int32_t *b_idx, int32_t capacity,
                         int32_t *length_dev, void *stream);

/*
 * Semi-local LCS queries on the last build: out[q] = LCS(a, b[i_q : k_q]) for
 * count queries with 0 <= i_q <= k_q <= n, read from the top breakout matrix
 * (Section II-B-1: D(i, j) is the smallest end column c with
 * LCS(a, b[i:c]) >= j, so the answer is the largest j with D(i, j) <= k;
 * one binary search over row i).  qi, qk: device int32[count] (column
 * indices, 0-based, half-open substring); out: device int32[count]; a query
 * outside 0 <= i <= k <= n gets -1.  Asynchronous on `stream`, graph-safe.
 * Errors: LCS_E_INVAL (null pointer with count > 0, count < 0),
 * LCS_E_STATE (no build), LCS_E_HIP.
 */
int32_t lcs_semilocal(lcs_plan_t plan, const int32_t *qi, const int32_t *qk, int32_t count,
                      int32_t *out, void *stream);

/*
 * Every vertex of the canonical path, row by row (Section II-E, the vertices
 * between two cross-vertices of a row): the path enters grid row r (the row
 * between the first r and r+1 symbols of a, r = 0..m) at column col_in[r] and
 * leaves it at col_out[r] >= col_in[r]; it then goes down (col_out[r] ==
 * col_in[r + 1]) or along the match a[r] = b[col_out[r]] (col_in[r + 1] =
 * col_out[r] + 1).  The path is the leftmost one, whose matches are the
 * canonical witness: it comes down as early as it can and runs right along the
 * row of its next match (col_out[m] = n).
 *   a_idx, b_idx, length_dev: the device witness of lcs_trace_device for the
 *   last build (pairs sorted, *length_dev of them); col_in, col_out: device
 *   int32[m + 1] each.  Asynchronous, graph-safe.
 * Errors: LCS_E_INVAL (null pointer), LCS_E_STATE (no build), LCS_E_HIP.
 */
int32_t lcs_path(lcs_plan_t plan, const int32_t *a_idx, const int32_t *b_idx,
                 const int32_t *length_dev, int32_t *col_in, int32_t *col_out, void *stream);

/*
 * Per-kernel timing of a plan made with LCS_PLAN_PROFILE: one record per
 * launch of every build and trace since the records were last read, in launch
 * order, measured with HIP events recorded on the caller's stream right
 * before and after the launch (at most 32768 records are kept).
 * `bytes` is the launch's algorithmic traffic: the breakout-matrix cells (and
 * tables) it must read and write once, 4 bytes each.  For a combine level
 * each parent row i costs row i of D_U, row i of D_L and row i of D_G; the
 * anchor kernel owns the anchor rows and the bracket kernel the others.
 * Waits for the recorded events.  Returns at most max records; *count
 * receives the number available.  When all of them fit (max >= *count) the
 * records are cleared, so the next read starts with the next launch.
 */
#define LCS_PHASE_NEXTMATCH 0
#define LCS_PHASE_BASE 1
#define LCS_PHASE_ANCHOR 2
#define LCS_PHASE_BRACKET 3
#define LCS_PHASE_LENGTH 4
#define LCS_PHASE_TRACE_SPLIT 5
#define LCS_PHASE_TRACE_LEAF 6
typedef struct lcs_phase_time {
    int32_t kind;  /* LCS_PHASE_* */
    int32_t level; /* recursion level of the launch (0 = base strips) */
    float ms;      /* elapsed time between the two events */
    int64_t bytes; /* algorithmic bytes of the launch */
} lcs_phase_time;
int32_t lcs_plan_profile(lcs_plan_t plan, lcs_phase_time *out, int32_t max, int32_t *count);

/*
 * Inspection of the last build (for tests and debugging).
 * lcs_plan_levels: number of levels (level 0 = base strips, the last level is
 * the whole grid) and, if strips_per_level is not NULL, the strip count of
 * each level (the array must hold *levels entries; pass NULL first to size it).
 * lcs_dist_view: device pointer to the breakout matrix of strip `strip` at
 * level `level`, row-major with (*rows) = n + 2 rows (vertices 0..n and one
 * all-unreachable sentinel row) and (*cols) = h + 1 columns (weights 0..h);
 * *row0 is the first grid row of the strip (rows row0 .. row0 + h - 1 of a).
 */
int32_t lcs_plan_levels(lcs_plan_t plan, int32_t *levels, int32_t *strips_per_level);
int32_t lcs_dist_view(lcs_plan_t plan, int32_t level, int32_t strip, const int32_t **matrix,
                      int32_t *rows, int32_t *cols, int32_t *row0);

/* ============================================================== batches */

typedef struct lcs_batch_s *lcs_batch_t;

/* One pair of a batch: offsets (in symbols) into the shared symbol buffer. */
typedef struct lcs_pair_desc {
    int64_t a_off;
    int64_t b_off;
    int32_t m;
    int32_t n;
} lcs_pair_desc;

#define LCS_BATCH_PERSISTENT 0u /* one persistent launch drains a device work queue of
                                   the staged mode's items, step by step across the
                                   pairs that hold the slots, in chunks of one stage */
#define LCS_BATCH_PER_PAIR 1u   /* same kernels, launched pair after pair */
#define LCS_BATCH_GRAPH 2u      /* OR-able: replay the launch as a captured hipGraph */
#define LCS_BATCH_STAGED 4u     /* one launch per step of the method across all pairs
                                   (work-groups over every pair's items); pairs are
                                   packed into the slot area in waves */
#define LCS_BATCH_PAIR_QUEUE 8u /* one persistent launch whose work-groups take whole
                                   pairs from a device queue (largest first) and run
                                   every step of a pair in order, separated by
                                   work-group barriers, in the work-group's own slot:
                                   no waits between work-groups */

typedef struct lcs_batch_desc {
    int32_t max_pairs; /* most pairs per submit */
    int32_t max_len;   /* largest m and largest n of any pair */
    int32_t alphabet;  /* 1..256 */
    int32_t base_rows; /* 16, 32 or 64 (0 selects 64); 128 to 1024 with
                          LCS_BATCH_STAGED or LCS_BATCH_PER_PAIR only
                          (lcs_batch_submit returns LCS_E_INVAL otherwise) */
    int32_t tile;      /* as in lcs_plan_desc */
    int32_t slots;     /* pairs whose matrices may be resident at once (0 = all);
                          pair p reuses slot p mod slots after pair p - slots
                          has been traced */
    uint32_t flags;    /* reserved, must be 0 */
} lcs_batch_desc;

/*
 * Plan a batch.  *workspace_bytes receives the device workspace needed by
 * lcs_batch_submit: `slots` pair-sized regions for the largest allowed pair
 * plus the task queue and its dependency counters.
 */
int32_t lcs_batch_plan(const lcs_batch_desc *desc, lcs_batch_t *out, size_t *workspace_bytes);
int32_t lcs_batch_destroy(lcs_batch_t batch);

/*
 * Length and witness of every pair (Sections II-B to II-E, per pair).
 *   pairs      HOST array of `count` descriptors; m, n in 0..max_len.
 *   symbols    device buffer holding all strings (symbols_len bytes).
 *   lengths    device int32[count] <- LCS lengths.
 *   a_idx/b_idx device int32 arrays <- witnesses; pair p's L pairs start at
 *              wit_off[p] = sum over q < p of min(m_q, n_q); witness_capacity
 *              must be >= that sum over all pairs.  May be NULL (lengths only)
 *              when witness_capacity is 0.
 *   mode       LCS_BATCH_PERSISTENT, LCS_BATCH_PAIR_QUEUE, LCS_BATCH_STAGED or
 *              LCS_BATCH_PER_PAIR, optionally OR LCS_BATCH_GRAPH (not with
 *              PER_PAIR).
 * Asynchronous on `stream`.  Submits of one batch handle must not overlap:
 * the call waits until the previous submit has consumed its staged pair
 * records.  Errors: LCS_E_INVAL, LCS_E_TOO_BIG,
 * LCS_E_WORKSPACE, LCS_E_CAPACITY, LCS_E_NOMEM, LCS_E_HIP.  A bad symbol sets
 * the length of its pair to LCS_E_SYMBOL.
 */
int32_t lcs_batch_submit(lcs_batch_t batch, const lcs_pair_desc *pairs, int32_t count,
                         const uint8_t *symbols, int64_t symbols_len, int32_t *lengths,
                         int32_t *a_idx, int32_t *b_idx, int64_t witness_capacity,
                         void *workspace, size_t workspace_bytes, uint32_t mode, void *stream);

/*
 * Outcome of the last persistent submit on `workspace`: LCS_OK, or LCS_E_HIP
 * if a work-group gave up waiting for a task it depends on (a bounded wait
 * that only a library defect can exhaust).  Synchronises the stream.
 */
int32_t lcs_batch_status(lcs_batch_t batch, void *workspace, void *stream);

/*
 * Host simulation of the persistent schedule for `count` pairs (no device
 * work; for tests): builds the task records and the task order as
 * lcs_batch_submit does and checks that the order covers every stage of every
 * pair once, that, running the order one stage at a time, every wait of a
 * stage's tasks is already met by earlier stages (so a chunk of one stage can
 * wait for all of its inputs first), that every wait target equals the number
 * of producers of its counter, that every task of a pair leads to the pair's
 * finish (so reuse of a workspace slot is ordered after all work of its
 * previous pair) and that each pair's layout fits its slot.  LCS_OK, or
 * LCS_E_STATE on a defect.
 */
int32_t lcs_batch_selftest(const lcs_batch_desc *desc, const lcs_pair_desc *pairs, int32_t count);

/* ============================================================== serving */

typedef struct lcs_server_s *lcs_server_t;

typedef struct lcs_server_desc {
    int32_t max_len;   /* largest m and n of a request */
    int32_t alphabet;  /* largest alphabet of a request, 1..256 */
    int32_t base_rows; /* 16, 32 or 64; 0 selects 64 */
    int32_t tile;      /* as in lcs_plan_desc */
    int32_t slots;     /* requests that may run on the device at once (1..64) */
    int32_t max_queue; /* waiting requests held on the host */
    uint32_t flags;    /* reserved, must be 0 */
} lcs_server_desc;

typedef struct lcs_result {
    int64_t tag;      /* caller's tag from lcs_server_submit */
    int32_t status;   /* LCS_OK or an error code (LCS_E_SYMBOL, LCS_E_HIP) */
    int32_t length;   /* LCS length */
    double t_submit;  /* host clock, seconds since lcs_server_open */
    double t_admit;   /* when its device work was enqueued */
    double t_done;    /* when poll observed its completion */
} lcs_result;

/*
 * Open a continuous-batching server over a caller-owned device arena of
 * arena_bytes: the memory budget for the inputs and breakout matrices of the
 * requests in flight.  Requests wait on the host in arrival order; the head of
 * the queue is admitted as soon as a slot is free AND a block of its footprint
 * can be carved out of the arena (first fit), so requests that arrive while
 * others run join them on the device, each on its own stream.  The arena and
 * the outputs stay the caller's; the server holds streams, events, pinned
 * staging buffers and one plan per slot.
 */
int32_t lcs_server_open(const lcs_server_desc *desc, void *arena, size_t arena_bytes,
                        lcs_server_t *out);

/* Arena bytes a request of sizes (m, n) occupies while it runs, at most (the
   next-match tables are sized for the server's largest alphabet here; a request
   of a smaller alphabet takes a little less). */
int32_t lcs_server_footprint(lcs_server_t server, int32_t m, int32_t n, size_t *bytes);

/*
 * Queue one request.  a and b are HOST strings (copied at submit) over the
 * request's own alphabet (1..the server's alphabet): its build uses that many
 * next-match tables, and a symbol >= alphabet ends the request with status
 * LCS_E_SYMBOL.  a_idx and
 * b_idx are device int32 arrays of at least min(m, n) entries that receive the
 * witness (both NULL: length only).  The request runs on a stream of the
 * server, so the caller must have no pending device work on a_idx / b_idx
 * when it submits (e.g. synchronise the stream that allocated or cleared them).  Returns LCS_E_BUDGET if the request can
 * never fit the arena, LCS_E_AGAIN if the host queue is full, LCS_E_INVAL /
 * LCS_E_TOO_BIG on bad arguments.
 */
int32_t lcs_server_submit(lcs_server_t server, int64_t tag, const uint8_t *a, int32_t m,
                          const uint8_t *b, int32_t n, int32_t alphabet, int32_t *a_idx,
                          int32_t *b_idx);

/*
 * Make progress without blocking on the device: collect finished requests
 * (their witnesses are then complete in the caller's arrays), then admit
 * waiting requests in arrival order while a slot and arena memory are free.
 * Up to max_results finished requests are written to results; *count
 * receives how many (the others are returned by later polls).
 */
int32_t lcs_server_poll(lcs_server_t server, lcs_result *results, int32_t max_results,
                        int32_t *count);

/* Requests on the device, requests waiting, arena bytes in use and peak use. */
int32_t lcs_server_pending(lcs_server_t server, int32_t *running, int32_t *waiting,
                           size_t *arena_used, size_t *arena_peak);

/* Wait for every running request, then release the server (not the arena). */
int32_t lcs_server_close(lcs_server_t server);

/*
 * The admission policy alone, under a virtual clock (no device; for tests):
 * `count` requests with arrival times, footprints and service times (seconds)
 * go through the same FIFO queue and first-fit arena as the server, with
 * `slots` concurrent executions whose completions are simulated.  Writes each
 * request's admission and completion time and the peak arena use.
 */
int32_t lcs_server_simulate(size_t arena_bytes, int32_t slots, int32_t count,
                            const double *arrival, const size_t *footprint,
                            const double *service, double *t_admit, double *t_done,
                            size_t *peak);

#ifdef __cplusplus
}
#endif

#endif /* LCS_H_ */
