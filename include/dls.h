/*
 * dls.h -- C ABI of the MI355X (gfx950) library that counts diagonal Latin
 * squares (DLS) exactly.
 *
 * Method: Kochemazov, Vatutin, Zaikin, "Fast Algorithm for Enumerating
 * Diagonal Latin Squares of Small Order" (arXiv:1709.02599).
 *
 * Conventions shared by every entry point
 *  - A square of order n (1 <= n <= 16) is n*n uint8 cells, row-major; a cell
 *    holds a value 0..n-1 or DLS_EMPTY.  A "prefix" is such a square with some
 *    cells assigned; its count is the exact number of DLS that agree with it
 *    (definition: Sec. 1).  A prefix that breaks a constraint is not an error:
 *    its count is 0.
 *  - All buffers are owned by the caller.  The library keeps no pointer to a
 *    caller buffer after the call returns (the *_async calls: after the work
 *    enqueued on the stream completes).
 *  - Every entry point returns DLS_OK (0) or a negative DLS_E* code; nothing
 *    is thrown across the ABI.  dls_strerror() names a code.
 *  - Host planning calls (dls_order, dls_split*, dls_group_order) need no GPU.
 *    Counting calls run on the current HIP device.
 */
#ifndef DLS_H
#define DLS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DLS_EMPTY 0xFFu
#define DLS_MAXN 16

/* flags */
enum {
    /* vertical symmetry a[i][j] + a[i][n-1-j] = n-1 (Sec. 1; Sec. 5.4).
     * Only the left half is searched; each value also fixes its mirror. */
    DLS_VSYM = 1u << 0,
    /* dls_split only: symmetry breaking on hourglass designs (Sec. 4.2-4.3,
     * Alg. 5-6).  Emits only prefixes whose hourglass is canonical, each with
     * the power of its class in mult_out. */
    DLS_SYMBREAK = 1u << 1,
    /* counting: use the plain one-prefix-per-lane kernel instead of the
     * persistent work-stealing kernel (both give identical counts). */
    DLS_PLAIN = 1u << 2
};

/* error codes */
enum {
    DLS_OK = 0,
    DLS_EINVAL = -1,   /* bad n, depth, flags, cell value or pointer          */
    DLS_ERANGE = -2,   /* output capacity too small (required size reported)  */
    DLS_ENOMEM = -3,   /* host or device allocation failed                    */
    DLS_EDEVICE = -4,  /* HIP runtime error, no device, or kernel fault flag  */
    DLS_EPATTERN = -5, /* a prefix's assigned cells differ from the pattern   */
    DLS_ECAPTURE = -6, /* the stream is under HIP graph capture and the call
                          would allocate (first call on the stream, or a
                          larger batch than any before) or asked for
                          kernel timing                                     */
    DLS_EBUSY = -7     /* serving: no ring slot or task-pool room free now   */
};

const char *dls_strerror(int err);

/* Library version string, e.g. "dls-mi355x 1.0 (gfx950)". */
const char *dls_version(void);

/* Name and text of the last HIP runtime error that made a call on this
 * thread return DLS_EDEVICE ("" if none).  Diagnostics only. */
const char *dls_last_hip_error(void);

/*
 * Fill order of the empty cells (Sec. 2.3, Fig. 1).  Starting from the
 * assigned cells (assigned[c] != 0 for c in 0..n*n-1), repeatedly: if a row,
 * column, main diagonal or antidiagonal has exactly n-1 assigned cells, its
 * last cell is next (row-major-first if several); otherwise the cell with the
 * largest V = r_i + c_j + md + ad (Sec. 2.3), ties broken row-major.
 * DLS_VSYM: only left-half cells (j < n/2, or j <= n/2 for odd n) are listed;
 * each also assigns its mirror.  DLS_SYMBREAK: the hourglass cells (rows 0 and
 * n-1, both diagonals; Sec. 4.2) come before all others.
 * order_out: capacity n*n; receives flat cell indices i*n+j; *len_out gets the
 * number written.
 */
int dls_order(int n, uint32_t flags, const uint8_t *assigned, uint8_t *order_out,
              int *len_out);

/* Variants of the fill order for tuning (counts never depend on the order):
 * 0 = the Sec. 2.3 rule as in dls_order; 1 ties broken column-major; 2 row
 * counts weigh double in V; 3 column counts weigh double; 4 no forced-cell
 * rule; 5 ties broken towards the last cell; 6 diagonal counts weigh double;
 * 7 diagonals ignored in V.  Arguments as dls_order; DLS_EINVAL for an
 * unknown variant. */
int dls_order_variant(int n, uint32_t flags, const uint8_t *assigned, int variant,
                      uint8_t *order_out, int *len_out);

/*
 * Split into independent workunits (Sec. 5.2).  Starts from row 0 = 0..n-1
 * and assigns the next `depth` cells of the dls_order() sequence in every way
 * that keeps all constraints among assigned cells, in depth-first order with
 * values increasing.  Two-call pattern: with prefixes_out == NULL only
 * *num_out = P (the number of prefixes) is set.  Otherwise prefixes_out is
 * [cap][n*n] uint8 and mult_out [cap] uint32 or NULL; returns DLS_ERANGE with
 * *num_out = P if cap < P.
 * DLS_SYMBREAK: depth must cover the hourglass (>= 3n-3 plain, fewer left-half
 * cells with DLS_VSYM); only prefixes whose hourglass is its class's
 * lexicographically least member are emitted, with mult_out = class power,
 * so that sum(mult * count) is the fixed-first-row total (Corollary 1).
 * Without it mult_out is all 1.
 */
int dls_split(int n, uint32_t flags, int depth, uint8_t *prefixes_out, uint32_t *mult_out,
              int64_t cap, int64_t *num_out);

/* As dls_split, but starting from an arbitrary prefix `base` (n*n cells)
 * instead of the bare first row; DLS_SYMBREAK is not accepted.  With
 * DLS_VSYM, `base` is first completed by mirror pairs (an inconsistent pair
 * yields P = 0). */
int dls_split_from(int n, uint32_t flags, const uint8_t *base, int depth,
                   uint8_t *prefixes_out, int64_t cap, int64_t *num_out);

/* Workunits on a given cell list: every consistent assignment of exactly
 * cells[0..ncells) (flat indices, empty in base, no repeats; with DLS_VSYM
 * left-half cells, mirrors implied) on top of base, in depth-first order with
 * values increasing.  Two-call pattern and errors as dls_split_from. */
int dls_split_cells(int n, uint32_t flags, const uint8_t *base, const int *cells, int ncells,
                    uint8_t *prefixes_out, int64_t cap, int64_t *num_out);

/* Workunits to a target count (Sec. 5.2), breadth-first: every consistent
 * assignment of the first d cells of the dls_order() sequence after `base`
 * (with DLS_VSYM left-half cells, each with its mirror), for the smallest d
 * with at least min_tasks of them, or d = max_depth (never deeper than two
 * cells before the end).  The counts of the workunits sum to the count of
 * base.  Two-call pattern (prefixes_out NULL: only *num_out); DLS_ERANGE if
 * cap is too small.  P = 0 for an inconsistent base.  Host only; the serving
 * calls split requests this way. */
int dls_split_target(int n, uint32_t flags, const uint8_t *base, int64_t min_tasks, int max_depth,
                     uint8_t *prefixes_out, int64_t cap, int64_t *num_out);

/* Cost of a fill order (Sec. 2.3: the order decides the speed, never the
 * count): over the host prefixes [num][n*n], the number of downward DFS
 * steps the search kernels take when they fill exactly cells[0..ncells) in
 * that order (*steps_out), and the number of squares reached (*leaves_out).
 * Host only, multithreaded.  DLS_EINVAL for a bad cell list or a cell
 * assigned in some prefix. */
int dls_order_cost(int n, uint32_t flags, const int *cells, int ncells, const uint8_t *prefixes,
                   int64_t num, uint64_t *steps_out, uint64_t *leaves_out);

/* Uniform sampling of workunits (Sec. 5.3 estimates from a random sample):
 * the prefixes that dls_split(n, flags, depth) would emit at the positions
 * listed in `indices` (k strictly increasing 0-based positions) are written to
 * prefixes_out [k][n*n]; *total_out gets P.  Streams the split without
 * storing it.  DLS_SYMBREAK is not accepted.  Returns DLS_ERANGE if an index
 * is >= P. */
int dls_split_sample(int n, uint32_t flags, int depth, const int64_t *indices, int64_t k,
                     uint8_t *prefixes_out, int64_t *total_out);

/* Order of the hourglass transformation group used by DLS_SYMBREAK
 * (2 * 2^(n/2) * (n/2 - 1)!, Sec. 4.3 Alg. 5), or a negative error. */
int64_t dls_group_order(int n);

/* Canonicity test of one hourglass design h (n*n cells; rows 0 and n-1 and
 * both diagonals assigned, row 0 = 0..n-1): 0 if some transformed and
 * renormalised image is lexicographically smaller (row-major), else the class
 * power (Alg. 5).  Written to *mult_out. */
int dls_canon(int n, const uint8_t *h, uint32_t *mult_out);

/*
 * Exact counts on the GPU, host buffers, blocking.  The count of a prefix is
 * the number of squares that satisfy the definition of Sec. 1 (every row,
 * column, the main diagonal and the main antidiagonal a permutation of
 * 0..n-1; with DLS_VSYM also a[i][j] + a[i][n-1-j] = n-1) and agree with the
 * prefix on its assigned cells: the answer to one workunit of Sec. 5.2, whose
 * sum over a split is the count of the parent.
 * prefixes: [num][n*n] uint8 (DLS_EMPTY = unassigned); counts_out: [num]
 * uint64, counts_out[k] = the count of prefixes[k].  Prefixes may differ in
 * which cells are assigned; they are grouped by pattern internally (with
 * DLS_VSYM each prefix is first completed by mirror pairs; an inconsistent
 * pair counts 0).  DLS_PLAIN selects the plain kernel.  With DLS_VSYM and
 * odd n > 1 every count is 0 and nothing is launched.  Errors: DLS_EINVAL
 * (bad n, flags, cell value, NULL buffer with num > 0), DLS_ENOMEM,
 * DLS_EDEVICE (HIP error, or a kernel reported lost work).
 */
int dls_count(int n, uint32_t flags, const uint8_t *prefixes, int64_t num,
              uint64_t *counts_out);

/*
 * The same counts (Sec. 1 definition, one integer per Sec. 5.2 workunit) on
 * device buffers, asynchronous on `stream` (a hipStream_t; NULL = the null
 * stream).  d_prefixes: device [num][n*n] uint8; d_counts: device [num]
 * uint64, overwritten once the stream reaches the work.  Both stay the
 * caller's; the library keeps no pointer to them after the work completes.
 * One fill order serves the batch, so every prefix must assign the same cells
 * as prefix 0 (with DLS_VSYM each assigned cell's mirror assigned too).  The
 * call reads that pattern from d_prefixes[0] with an n*n-byte device-to-host
 * copy on `stream` (which waits for the work already queued there), then
 * enqueues the count and returns.  A prefix that assigns other cells counts
 * 0 and sets bit 0 of the stream's status word; a task lost to an expired
 * bounded wait sets bit 1 (its count is then short), an expansion overflow
 * bit 2: read the word with dls_stream_status after the work.  Under HIP
 * graph capture this call returns DLS_ECAPTURE (the pattern copy cannot be
 * captured): use dls_count_async_ex with an explicit pattern.  Other errors
 * as dls_count, returned before anything is enqueued.
 */
int dls_count_async(int n, uint32_t flags, const uint8_t *d_prefixes, int64_t num,
                    uint64_t *d_counts, void *stream);

/*
 * Status word of the counting calls made on `stream` without a d_status
 * buffer (dls_count_async, and the *_ex forms given d_status = NULL): waits
 * for the stream, writes the OR of the bits those calls set since the last
 * read to *status_out (0 = every count is exact) and clears it.  Bit 0
 * (value 1): a prefix did not match the pattern (counted 0); bit 1 (2): a
 * bounded wait expired (a count is short); bit 2 (4): an expansion buffer
 * overflowed.  DLS_ECAPTURE under capture.
 */
int dls_stream_status(void *stream, uint32_t *status_out);

/* Launch shape for the *_ex calls; zero fields mean "library default". */
typedef struct {
    int block;          /* threads per workgroup (64..1024, multiple of 64);
                           halved while the workgroup's LDS would exceed
                           what the device allows a workgroup (160 KiB on
                           gfx950)                                         */
    int blocks_per_cu;  /* persistent kernel: workgroups per CU in the grid
                           (0 = 2048 / block).  Workgroups beyond those that
                           fit at once start when others leave; they still
                           count in the guided chunk size (remaining tasks /
                           (2 x waves)), so a larger grid means smaller
                           chunks.  The expansion default follows it too.  */
    int steal_depth;    /* persistent kernel: give subtrees to idle waves on
                           other CUs only from levels < (levels - steal_depth);
                           0 = library default (on for batches too small to
                           fill the GPU), negative = off                       */
    int refill_every;   /* persistent kernel: DFS steps between refills
                           (0 = 32; rounded up to an even number)          */
    int order_variant;  /* fill-order variant (see dls_order_variant); 0 =
                           the rule of Sec. 2.3.  Counts never depend on it. */
    int time_kernel;    /* nonzero: record a HIP event pair around the
                           search kernels on the launch stream (not under
                           graph capture); read with dls_kernel_time_ms  */
    int expand_target;  /* persistent kernel: a batch of fewer tasks than
                           this is first deepened on the device, one level
                           per pass, until it has this many tasks (the split
                           of Sec. 5.2 done breadth-first on the GPU).
                           0 = default (the number of lanes launched),
                           negative = off; at most 2^28.  Uses 4x this many
                           task slots of device memory per stream.        */
    int chunk_min;      /* persistent kernel: smallest number of tasks a
                           wave takes from the static queue at once
                           (0 = default 8; at most 65536)                  */
    int lds_masks;      /* persistent kernel: positive = keep the row and
                           column masks of each lane in LDS (one xor per
                           line to mark a value) instead of packed VGPR
                           words; negative = VGPR layout; 0 = library
                           default (LDS from order 9 on)                 */
    int refill_min;     /* persistent kernel: while static tasks remain, a
                           wave refills its idle lanes when at least this
                           many are idle (1..64; 0 = default 8)           */
    int wg_pool;        /* persistent kernel, line masks in VGPRs, no
                           donation across the chip: once the static queue
                           is empty, the waves of a workgroup share subtrees
                           through a pool of at most this many task records
                           in LDS (as many as fit in half the record area);
                           0 = default (on, as many as fit), negative = off
                           (each wave shares only among its own lanes)     */
} dls_launch;

/*
 * Partial squares on a given cell list (the incomplete squares DLS_N^k of
 * Sec. 5.3, formed by the first k cells of a fixed order): counts_out[k] =
 * the number of ways to assign exactly the cells cells[0..ncells) (flat
 * indices, each empty in every prefix, in this order) so that no row,
 * column or diagonal repeats a value among assigned cells.  Other empty
 * cells stay empty.  With DLS_VSYM the cells are left-half cells (column
 * j <= (n-1)/2) and each assignment also sets its mirror to n-1-v.  ncells =
 * 0 counts 1 per consistent prefix.  Errors as dls_count; DLS_EINVAL for a
 * cell out of range, repeated, assigned in a prefix, or (VS) in the right
 * half.  The _async form takes device buffers, the pattern of assigned cells
 * shared by all prefixes, and a launch shape, as dls_count_async_ex.
 */
int dls_count_cells(int n, uint32_t flags, const int *cells, int ncells,
                    const uint8_t *prefixes, int64_t num, uint64_t *counts_out);
int dls_count_cells_async(int n, uint32_t flags, const int *cells, int ncells,
                          const uint8_t *pattern, const uint8_t *d_prefixes,
                          int64_t num, uint64_t *d_counts, uint32_t *d_status,
                          void *stream, const dls_launch *launch);

/*
 * Hourglass designs and their canonical forms on the GPU (Sec. 4.2-4.3,
 * Alg. 5), 4 <= n <= 9.  d_designs: [num][n*n] diagonal designs (row 0,
 * main diagonal and antidiagonal assigned and consistent, every other cell
 * 0xFF), e.g. dls_split_cells over the diagonal cells.  Every consistent
 * filling of the rest of the last row makes an hourglass design; the
 * canonical ones (no transformed and renamed image lexicographically
 * smaller) are written to d_out [cap][n*n] with their class powers in
 * d_mult [cap], in no particular order; *d_count (device uint64) receives
 * their number.  If it exceeds cap, only cap designs are written and bit 3
 * of *d_status is set: call again with a larger buffer.  Device buffers on
 * `stream`; the first call for an order uploads the group table.
 */
int dls_hourglass_classes_async(int n, const uint8_t *d_designs, int64_t num, uint8_t *d_out,
                                uint32_t *d_mult, int64_t cap, uint64_t *d_count,
                                uint32_t *d_status, void *stream);

/* Mean duration in milliseconds of the search kernels launched with
 * time_kernel on `stream` since the previous call (at most 65536 launches),
 * and their number in *launches_out (may be NULL).  Resets the tally.  The
 * caller must have synchronised the stream.  DLS_EINVAL if no timed launch
 * happened on it. */
int dls_kernel_time_ms(void *stream, float *ms_out, int64_t *launches_out);

/*
 * dls_count_async with the batch's pattern and a status buffer given by the
 * caller, and an optional launch shape (NULL = library defaults); nothing is
 * copied back, so these forms can be captured in a HIP graph once the
 * stream's scratch has been sized by an uncaptured call.  pattern: host array
 * of n*n bytes, nonzero = assigned in every prefix (NULL = "row 0 only").
 * d_status: device uint32, OR-ed with the bits listed at dls_stream_status;
 * NULL = the stream's own status word (read with dls_stream_status).
 * Returns after enqueueing (host-side argument errors are returned at once).
 */
int dls_count_async_ex(int n, uint32_t flags, const uint8_t *pattern, const uint8_t *d_prefixes,
                       int64_t num, uint64_t *d_counts, uint32_t *d_status, void *stream,
                       const dls_launch *launch);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * count as dls_count_async_ex, with every scratch buffer (work-queue control
 * block, donated-record slots, task records, expansion buffers) carved out
 * of one static device array of 128 MiB that each GPU the library runs on
 * holds until the process ends.  The call allocates nothing: no hipMalloc,
 * no hipFree, no events.  The caller passes inputs, outputs and d_status
 * (required: NULL gives DLS_EINVAL); launch->time_kernel is refused
 * (DLS_EINVAL).  DLS_ERANGE if the batch's task records do not fit the array
 * next to the fixed parts (about 4 million prefixes up to order 8, 32 bytes
 * each; 80 bytes per prefix at order 16); the breadth-first expansion of
 * small batches gets what is left, its target lowered to fit.  Every call on
 * one GPU shares that GPU's array: calls that overlap on one GPU (on
 * different streams, or from several threads) race and give wrong counts;
 * serialise them.  Each call clears what it needs cleared by kernels.
 */
int dls_count_async_noalloc(int n, uint32_t flags, const uint8_t *pattern, const uint8_t *d_prefixes,
                            int64_t num, uint64_t *d_counts, uint32_t *d_status, void *stream,
                            const dls_launch *launch);

/* As dls_count_async_ex; in addition, when d_steps != NULL (device
 * uint64[2]): d_steps[0] += the number of DFS steps taken by all lanes, and
 * d_steps[1] += the number of steps the lanes executed, including the steps
 * of lanes without work that run along with their wave (so d_steps[0] /
 * d_steps[1] is the share of useful lane-steps).  A DFS step either enters a
 * cell with a candidate value or returns from a cell whose candidates are
 * exhausted; the count is the same for every launch shape and feeds the
 * operation-count model behind the roofline figures. */
int dls_count_async_stats(int n, uint32_t flags, const uint8_t *pattern,
                          const uint8_t *d_prefixes, int64_t num, uint64_t *d_counts,
                          uint32_t *d_status, void *stream, const dls_launch *launch,
                          uint64_t *d_steps);

/* Device-side weighted total, the Corollary 1 sum:  *d_out = sum over k of
 * d_mult[k] * d_counts[k] (d_mult NULL: all 1), uint64 arithmetic, on
 * `stream`.  Launches only kernels (no memset), so it can be captured in a
 * HIP graph with the counting launch. */
int dls_reduce_weighted(const uint64_t *d_counts, const uint32_t *d_mult, int64_t num,
                        uint64_t *d_out, void *stream);

/* Integer-VALU throughput probe: `iters` rounds of independent 32-bit
 * and/or/xor/add chains on every lane of `blocks` x 256 threads; d_sink gets
 * one word per thread.  Used to measure the achievable integer-op peak. */
int dls_valu_probe(int blocks, int iters, uint32_t *d_sink, void *stream);

/*
 * Serving: counting requests that arrive while others run, batched
 * continuously on the device.  A server holds one long-running kernel on its
 * own non-blocking stream, serving requests of every order 4..9 with or
 * without DLS_VSYM, a ring of max_jobs (1..256) job slots and a pool of
 * pool_bytes of workunit cells, both in host-pinned memory.  A request is
 * one prefix; the server splits it on the host into at least min_tasks
 * workunits (Sec. 5.2: the counts of a split sum to the count of the
 * prefix), writes them to the pool (each workunit padded to a multiple of 16
 * bytes: 64 bytes at orders 7 and 8, 96 at order 9) and publishes the job in
 * the ring; no stream operation is involved.  The running kernel takes jobs
 * oldest first as its waves free up: waves of different jobs, and of
 * different orders, run side by side, so a request admitted while others
 * run is served at once.  The kernel keeps each job's outstanding pieces
 * and computes its total (the exact count of the request, the definition of
 * Sec. 1) on the device; the piece that finishes a job writes its result to
 * host-pinned memory, read by dls_server_poll.  A wave takes about the
 * job's workunits over twice the grid's waves at a time, so even a small job
 * spreads over the grid, and its lanes share subtrees among themselves (the
 * split of Sec. 5.2 done on the device).  With steal_depth > 0, a wave with
 * fewer than 8 idle lanes also hands the untried siblings of a shallow level
 * (more than steal_depth levels above the last) to the job's donation queue
 * in device memory while waves that found no work are waiting (a ring of
 * 2048 records per job; while it is full, waves keep their work), and each
 * such wave takes one and shares it among its lanes.  The grid leaves as a
 * whole:
 * once a wave has found no job for 50 ms while no wave is inside a job, every
 * wave leaves, and the next submit or poll launches the kernel again; while
 * any job runs, every wave of the grid stays (none leaves on its own).
 */
typedef struct dls_server dls_server;

/* launch (may be NULL): blocks_per_cu (1 or 2 workgroups of 256 per CU;
 * default 1: the request mix ran twice as fast as with 2), refill_every (default 64), chunk_min = most workunits a wave
 * takes from a job at once (default 64; a wave takes about the job's
 * workunits over twice the grid's waves, at least one), order_variant (fill
 * order), steal_depth
 * (> 0: hand subtrees between waves as above; 0 or negative: off, the
 * default -- measured slower on the serving mix); block 0 or 256; other
 * fields ignored.  The donation rings take
 * 144 KiB of device memory per job slot.  A request is split at most 24
 * cells deep.
 * DLS_EINVAL for bad arguments, DLS_ENOMEM. */
int dls_server_create(int max_jobs, int64_t pool_bytes, const dls_launch *launch, dls_server **out);

/* Admits one request of order n (4..9) and flags (0 or DLS_VSYM): prefix is
 * a host array of n*n cells.  *ticket_out identifies it for dls_server_poll.
 * DLS_EBUSY: no ring slot, or no contiguous pool room for its workunits, is
 * free now (nothing was done; retry once a job has been polled done) --
 * admission follows the server's real allocation.  DLS_ERANGE: its
 * workunits need more than the whole pool.  A request whose count is 0
 * without search (inconsistent prefix; vertical symmetry at odd n) is done
 * at once.  Thread-safe per server. */
int dls_server_submit(dls_server *s, int n, uint32_t flags, const uint8_t *prefix, int64_t min_tasks,
                      int64_t *ticket_out);

/* *done_out = 1 once the request is done; then *count_out (may be NULL) is
 * its exact count, ticks_out[0..1] (may be NULL) the device times
 * (s_memrealtime, 100 MHz) when its job was first taken up and when it
 * finished (0 for requests done without search), and the ticket is retired
 * (its slot and pool room freed).  DLS_EINVAL for an unknown ticket. */
int dls_server_poll(dls_server *s, int64_t ticket, uint64_t *count_out, uint64_t *ticks_out, int *done_out);

/* Bytes the server allocated (device and host-pinned), free pool bytes,
 * free ring slots, launches of the serving kernel so far (any pointer may
 * be NULL). */
int dls_server_info(dls_server *s, int64_t *allocated_bytes, int64_t *pool_free, int *slots_free,
                    int64_t *launches);

/* Waves of the serving kernel running now (*live_out) and waves of its grid
 * (*grid_out: 4 per workgroup, blocks_per_cu workgroups per CU); read from
 * host-pinned flags each wave sets while it runs (either pointer may be
 * NULL).  While the kernel runs, *live_out equals *grid_out except while the
 * grid starts or leaves.  DLS_EINVAL for a NULL server. */
int dls_server_waves(dls_server *s, int *live_out, int *grid_out);

/* Subtrees handed between waves through the jobs' donation queues, summed
 * over the requests retired so far by dls_server_poll.  DLS_EINVAL for a
 * NULL argument. */
int dls_server_shared(dls_server *s, int64_t *subtrees_out);

/* Stops the kernel (bounded wait) and frees everything.  Requests not polled
 * done are dropped.  DLS_EDEVICE if the kernel did not stop (the server's
 * memory is then not freed). */
int dls_server_destroy(dls_server *s);

#ifdef __cplusplus
}
#endif

#endif /* DLS_H */
