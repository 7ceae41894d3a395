/*
 * msp.h -- C ABI of libmsp, an exact GPU solver (AMD Instinct MI355X,
 * gfx950) for the feasibility market split problem.
 *
 * Problem (Section 1, eq. nSSP): given A in N0^{m x n} and d in N0^m, find
 * EVERY x in {0,1}^n with sum_j a_ij x_j = d_i for all i = 1..m.
 *
 * Method (Sections 2-3): the first r rows are folded into one 1-D key by the
 * surrogate constraint of Section 1 (eq. surrogate): with D = max(100,
 * max a_ij + 1) and base B = n*D, key(x) = sum_{i<r} B^i (a_i . x) and
 * K_d = sum_{i<r} B^i d_i; key(x) = K_d holds exactly when rows 1..r hold.
 * msp_opts.key_base = 1 gives row i the mixed radix rowsum_i + 1 instead of
 * B (the same exactness with a smaller key).  Keys up to 96 bits are exact:
 * past 63 bits the sums are carried in 128 bits and the half records keep
 * a second key word (msp_opts.key_words).  A slice selects on the left
 * key modulo slice_mod, exact for any key width.
 * Every solution of that 1-D subset-sum problem (a "1-D hit") is enumerated
 * with a Schroeppel-Shamir style four-list meet in the middle (Algorithm 1,
 * with the heaps replaced by residue classes of the key), and every hit is
 * checked exactly against the remaining m - r rows (Algorithm 2).  All
 * arithmetic is exact integer.
 *
 * Counting conventions:
 *   H    = number of 1-D hits = #{x : rows 1..r hold}, a 128-bit count;
 *   S    = the solution set; |S| is exact even when not all vectors are
 *          stored (see max_solutions).
 *   slice: with slice_mod = 2^s > 0, only x whose left-half key
 *          k_L(x) = key of x restricted to columns 0..ceil(n/2)-1 satisfies
 *          k_L(x) mod slice_mod == slice_res are counted and returned.
 *
 * Column partition (Algorithm 1 leaves it open): contiguous quarters,
 * h_L = ceil(n/2), q_A = ceil(h_L/2), q_B = floor(h_L/2),
 * q_C = ceil((n-h_L)/2), q_D = floor((n-h_L)/2), or unequal ones
 * (msp_opts.log2_outer).
 *
 * Threading: one context is used by one host thread at a time; distinct
 * contexts may be used concurrently.  All calls return MSP_OK (0) or a
 * negative MSP_E_* code; msp_strerror() names it.
 */
#ifndef MSP_H
#define MSP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MSP_OK               0
#define MSP_E_INVALID      (-1)  /* null pointer, m<1, n<1, a_ij<0, d_i<0, bad option */
#define MSP_E_RANGE        (-2)  /* some row sum exceeds 65534 (uint16 row packing)    */
#define MSP_E_KEY_OVERFLOW (-3)  /* largest key >= 2^96, or >= 2^63 with key_words = 1 */
#define MSP_E_UNSUPPORTED  (-4)  /* m > 16, n > 100, m - r > 10, or > 2^29 cells needed*/
#define MSP_E_NOMEM        (-5)  /* workspace does not fit the budget, or a residue
                                    bucket holds 2^32 or more records                  */
#define MSP_E_DEVICE       (-6)  /* HIP runtime error; the context is poisoned          */
#define MSP_E_CANCELLED    (-7)  /* solve cancelled                                     */
#define MSP_E_TRUNCATED    (-8)  /* caller buffer smaller than the result               */
#define MSP_E_STATE        (-9)  /* no result yet (msp_solve not run or failed)         */
#define MSP_E_NOLIB        (-10) /* GPU not present or not usable                       */
#define MSP_E_BUSY         (-11) /* the context is in use by another solve or request   */

typedef struct msp_ctx msp_ctx;

typedef struct {
    int32_t  key_rows;        /* r >= 1 rows folded into the 1-D key; 0 = 1            */
    int32_t  log2_m;          /* residue modulus M = 2^log2_m; 0 = planner's choice     */
    int32_t  log2_cells;      /* residue cells T = 2^log2_cells; 0 = planner's choice   */
    int32_t  parts;           /* work-groups per cell; 0 = planner's choice             */
    int64_t  slice_mod;       /* 0 = full solve; else a power of two (see above)        */
    int64_t  slice_res;       /* residue kept by the slice, 0 <= slice_res < slice_mod  */
    uint64_t max_solutions;   /* solution vectors kept on the device; 0 = 1<<20         */
    uint64_t window_records;  /* half records per side per window, and the least the
                                 record buffers hold (for a class far denser than
                                 the average cell); 0 = planner's choice          */
    void    *workspace;       /* caller-owned device buffer, or NULL (library allocates)*/
    uint64_t workspace_bytes; /* size of `workspace`; with NULL workspace: budget, 0=auto*/
    void    *stream;          /* hipStream_t to run on, or NULL (library's own stream)  */
    int32_t  first_only;      /* 1: stop after the first residue window that yields a
                                 solution (Algorithm 2 returns the first x); H, |S| and
                                 the solutions then cover the windows processed        */
    int32_t  join_variant;    /* bucket join: 0 = planner's choice (from the expected
                                 number of equal-key records per key), 1 = per-slot
                                 chains (groups of ~1), 2 = contiguous key groups
                                 (groups of ~5-250), 3 = one wavefront per bucket
                                 comparing keys directly (buckets of a few dozen
                                 records)                                           */
    int32_t  verify_join;     /* how equal-key run pairs are decided: 1 = an exact
                                 hash join on (key, packed non-key rows) (the sort/
                                 search check of Algorithms 3-4 with an exact key in
                                 place of a hash): a device-wide table for exact
                                 buckets, an LDS table per bucket for hash buckets
                                 (buckets too large for LDS keep the pairwise check);
                                 2 = every one of the |G_L||G_R| pairs compared on its
                                 own (1-D hits verified one by one); 0 = planner's
                                 choice: the hash join when the expected equal-key
                                 group holds >= 32 records per side.  Same H, |S| and
                                 solutions; no effect when every row is a key row   */
    int32_t  key_base;        /* radix of the surrogate key (Section 1, eq. surrogate):
                                 0 = B = n*D for every key row (D = max(100, max a_ij
                                 + 1)); 1 = mixed radix rowsum_i + 1 per key row, the
                                 smallest radix that keeps the key exact, so int64
                                 holds more rows.  Both give the same H, |S| and
                                 solutions on a whole solve; a slice keeps
                                 k_L mod slice_mod of the key in use             */
    int32_t  row_fingerprint; /* what a half record stores of the non-key rows:
                                 1 = one 32-bit fingerprint h(v) = sum_i c_i v_i mod
                                 2^32 (linear, so h(left) = h(a) + h(b) and the right
                                 side stores h(d) - h(c) - h(e)); equal fingerprints
                                 are candidates, each checked exactly on the packed
                                 rows of its four quarter subsets; 2 = the packed
                                 rows themselves (2 rows per word); 0 = planner:
                                 the fingerprint when the rows take 2 or more words.
                                 Same H, |S| and solutions                        */
    int32_t  first_order;     /* with first_only: 0 = residue windows in decreasing
                                 order of candidate pairs (sum over buckets of left x
                                 right records, from one count pass over all windows;
                                 for buckets of one key value, the window's 1-D hits),
                                 so the densest windows come first; 1 = cell order */
    int32_t  log2_outer;      /* q_A, variables of the left outer quarter: 0 = the
                                 planner's choice; ceil(hL / 2) (hL = ceil(n / 2)) =
                                 equal quarters as in Algorithm 1; smaller moves
                                 s = ceil(hL / 2) - q_A variables of each half from
                                 its outer quarter to its inner one (same pairs,
                                 fewer outer elements per residue cell).  Same H,
                                 |S| and solutions                                  */
    int32_t  key_words;       /* what a half record keeps of key >> log2_m (Section 1,
                                 eq. surrogate): 1 = the bits above the two quarter
                                 positions of its 64-bit header (64 - ceil(n/2)),
                                 the modulus raised until they suffice; 2 = a
                                 second key word of 32 more bits (records carry
                                 the row fingerprint and that word, 16 bytes),
                                 needed for keys past int64 (up to 96 bits; more
                                 key rows, e.g. six at n = 90); 0 = the planner's
                                 choice: two words for keys past int64 or when one
                                 word would force the modulus up.  Two words
                                 need row_fingerprint != 2.  Same H, |S| and
                                 solutions                                          */
} msp_opts;

/* Per-solve statistics; phase times are measured with HIP events on the
 * solve's stream and summed over windows. */
typedef struct {
    double   ms_total;        /* host wall time of msp_solve                        */
    double   ms_quarters;     /* quarter-list generation + residue-cell sort         */
    double   ms_count;        /* bucket counting pass                                */
    double   ms_scan;         /* offset scans                                        */
    double   ms_scatter;      /* bucket generation (scatter) pass                    */
    double   ms_join;         /* per-bucket join (and in-join verify)                */
    double   ms_verify;       /* tiled verify of large equal-key runs                */
    uint64_t records_left;    /* half records generated, left side                   */
    uint64_t records_right;   /* half records generated, right side                  */
    uint64_t windows;         /* residue windows processed                           */
    uint64_t verify_launches; /* launches of the tiled verify kernel                  */
    uint64_t verify_pairs;    /* pairs covered by the tiled verify                   */
    uint64_t record_bytes;    /* bytes of one half record                            */
    int32_t  log2_m, log2_cells, parts, key_rows;
    int32_t  exact_buckets;   /* 1: each bucket holds one key value                  */
    int32_t  words;           /* 32-bit words of packed non-key rows                 */
    int32_t  complete;        /* 1: every residue window was processed               */
    int32_t  vector_join;     /* 1: equal-key runs were decided by the vector join   */
    uint64_t windows_total;   /* residue windows of the whole (sliced) solve         */
    int32_t  join_grouped;    /* hash buckets: 0 = chains, 1 = contiguous key groups,
                                 2 = one wavefront per bucket                        */
    int32_t  key_base;        /* the key radix used (msp_opts.key_base)              */
    int32_t  row_fingerprint; /* 1: half records carried a row fingerprint          */
    uint64_t cells_done;      /* residue cells processed; in cell order (window_order
                                 0) they are the cells k_first + i * k_step,
                                 i < cells_done (k_step = 1 and k_first = 0 without a
                                 slice); all of them unless first_only stopped early */
    int32_t  window_order;    /* 1: first_only took windows in density order        */
    int32_t  log2_outer;      /* q_A used (msp_opts.log2_outer)                      */
    uint64_t first_cell;      /* window_order 1: index of the first cell of the first
                                 window processed (the densest)                      */
    int32_t  key_words;       /* 1 or 2 (msp_opts.key_words)                         */
    int32_t  key_bits;        /* bits of K_d + 1: up to 96                           */
} msp_stats_t;

/* Device memory from the caller, e.g. a torch-allocated arena, so that the
 * framework around the library owns all device memory: from this call on,
 * every workspace the library allocates itself (msp_solve without a caller
 * workspace, and the arena of msp_batch_solve and of a server) comes from
 * alloc(bytes, user) and goes back through release(ptr, user) instead of
 * hipMalloc / hipFree.  alloc returns device memory of the current device,
 * aligned to 256 bytes, or NULL (the call that needed it then fails with
 * MSP_E_NOMEM).  Each allocation is released through the pair that made it.
 * Both NULL restores hipMalloc / hipFree; exactly one NULL is MSP_E_INVALID.
 * Process-wide.  The callbacks may run on a server's scheduler thread. */
typedef void *(*msp_alloc_fn)(size_t bytes, void *user);
typedef void (*msp_release_fn)(void *ptr, void *user);
int  msp_set_allocator(msp_alloc_fn alloc, msp_release_fn release, void *user);

/* Copies A (row-major m*n int32) and d (m int32); the caller may free both
 * on return.  Validates the instance (see the error codes). */
int  msp_create(const int32_t *A, const int32_t *d, int32_t m, int32_t n, msp_ctx **out);

/* Fills *o with the defaults (all zero / NULL). */
void msp_default_opts(msp_opts *o);

/* Runs the whole solve on the GPU and keeps H, |S| and up to max_solutions
 * vectors in the context.  Synchronous: returns when results are ready.
 * opts may be NULL (defaults). */
int  msp_solve(msp_ctx *ctx, const msp_opts *opts);

/* msp_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same solve and the same kernels, but the workspace is a fixed device array
 * inside the library (MSP_NOALLOC_SCRATCH_BYTES = 128 MiB per GPU, held by
 * every GPU the library runs on until the process ends), and the call makes
 * no hipMalloc, hipFree, pinned-host or event allocation and creates no
 * stream.  opts->workspace must be NULL (workspace_bytes 0 or the scratch
 * size); opts->stream NULL runs on the null stream.  A plan that does not fit
 * the scratch array fails with MSP_E_NOMEM.  Phase times in msp_stats are 0.
 * Results are read as after msp_solve (they are kept in the context's host
 * memory).  Every call on one GPU shares that GPU's scratch array: calls that
 * overlap on the same GPU race and must be serialised by the caller. */
#define MSP_NOALLOC_SCRATCH_BYTES (128ull << 20)
int  msp_solve_noalloc(msp_ctx *ctx, const msp_opts *opts);

/* Results of the last successful msp_solve. */
int  msp_num_solutions(const msp_ctx *ctx, uint64_t *count);
int  msp_hits(const msp_ctx *ctx, uint64_t *lo, uint64_t *hi);   /* 128-bit H */
/* Writes up to `capacity` solutions as count*n bytes of 0/1 (x_1..x_n),
 * in canonical lexicographic order.  Returns MSP_E_TRUNCATED (with
 * *written = what fit) when capacity, or the stored set, is smaller than
 * |S|. */
int  msp_get_solutions(const msp_ctx *ctx, uint8_t *x, uint64_t capacity, uint64_t *written);
int  msp_stats(const msp_ctx *ctx, msp_stats_t *out);

void msp_destroy(msp_ctx *ctx);
const char *msp_strerror(int code);

/* ------------------------------------------------------------------------
 * Batched and served solves.  Many instances of uneven (m, n) run together:
 * each admitted solve gets a share of one device arena and its own stream,
 * and every scheduler step advances one residue window of every admitted
 * solve, so their kernels overlap on the GPU.  A solve is admitted when a
 * slot is free and its device footprint (planned for hbm_budget/max_slots,
 * or for the whole budget when that is the only way it fits) fits in the
 * free part of the arena; otherwise it waits, in arrival order.  Results
 * land in each context exactly as msp_solve would leave them.
 * ------------------------------------------------------------------------ */
typedef struct {
    uint64_t hbm_budget;      /* arena bytes for all admitted solves; 0 = 60% of free, <=128 GiB */
    int32_t  max_slots;       /* solves admitted at once; 0 = 16                              */
    int32_t  reserved;
} msp_batch_opts;

/* Solves ctxs[0..count) together; opts is NULL or an array of count
 * options (their workspace and stream fields are ignored).  Returns the
 * first error of any solve (each context records its own result). */
int  msp_batch_solve(msp_ctx *const *ctxs, const msp_opts *opts, int32_t count,
                     const msp_batch_opts *bo);

/* A server runs the batched scheduler on its own thread: requests submitted
 * while others are on the GPU join at the next step (continuous batching).
 * A context must stay alive, and unused by anything else, until its request
 * is done (msp_server_poll / msp_server_wait report completion). */
typedef msp_batch_opts msp_server_opts;
typedef struct msp_server msp_server;
int  msp_server_start(const msp_server_opts *o, msp_server **out);
int  msp_server_submit(msp_server *s, msp_ctx *ctx, const msp_opts *o, uint64_t *ticket);
int  msp_server_poll(msp_server *s, uint64_t ticket, int32_t *done, int32_t *status);
int  msp_server_wait(msp_server *s, uint64_t ticket, int32_t *status);
/* Stops a request at its next residue window (status MSP_E_CANCELLED). */
int  msp_server_cancel(msp_server *s, uint64_t ticket);
/* Seconds since server start: t4 = {submit, admit, first step, finish}. */
int  msp_server_times(msp_server *s, uint64_t ticket, double *t4);
/* Finishes every queued request, then frees the server. */
int  msp_server_stop(msp_server *s);

/* The plan msp_solve would run with these options, made on the host only
 * (no GPU needed), with the workspace shrunk to opts->workspace_bytes when
 * that is non-zero.  Returns the planner's code: MSP_E_UNSUPPORTED when a
 * launch of the plan would exceed the device's grid limits (2^32 work-items
 * per dimension) even with one residue cell per window, MSP_E_NOMEM when the
 * workspace cannot fit, MSP_E_INVALID for bad options. */
typedef struct {
    int32_t  key_rows, log2_m, log2_cells, log2_fine;  /* r, M = 2^log2_m, cells, fine buckets */
    int32_t  parts;            /* work-groups per cell in count and scatter              */
    int32_t  exact_buckets;    /* 1: each bucket holds one key value                     */
    int32_t  words;            /* 32-bit words of the packed non-key rows (2 rows each)  */
    int32_t  join_variant;     /* hash buckets: 0 chains, 1 key groups, 2 one wavefront  */
    int32_t  vector_join;      /* 1: equal-key runs decided by the vector join           */
    int32_t  key_base;         /* key radix (msp_opts.key_base)                          */
    int32_t  infeasible;       /* 1: a key row cannot hold; no GPU work is done          */
    int32_t  row_fingerprint;  /* 1: half records carry a row fingerprint               */
    int32_t  log2_outer;       /* q_A: variables of the left outer quarter               */
    int32_t  log2_inner;       /* q_B: variables of the left inner quarter               */
    uint64_t cells;            /* residue cells visited (all, or those of the slice)     */
    uint64_t cells_per_window; /* planned; the count pass may halve it                   */
    uint64_t windows;          /* planned windows                                        */
    uint64_t window_records;   /* half records per side a window's buffers hold          */
    uint64_t record_bytes;     /* bytes of one half record                               */
    uint64_t workspace_bytes;  /* device workspace of the plan                           */
    uint64_t max_grid_items;   /* largest work-item count of the window's launches whose
                                  size the plan fixes (< 2^32)                           */
    int32_t  key_words;        /* 1 or 2: key words per half record (msp_opts.key_words) */
    int32_t  key_bits;         /* bits of K_d + 1                                        */
} msp_plan_t;
int  msp_plan(const msp_ctx *ctx, const msp_opts *opts, msp_plan_t *out);

/* Device workspace bytes msp_solve would use with these options, the
 * plan shrunk to fit opts->workspace_bytes when that is non-zero (0 on
 * error or when it cannot fit).  Size a caller-owned workspace with it. */
uint64_t msp_workspace_bytes(const msp_ctx *ctx, const msp_opts *opts);

#ifdef __cplusplus
}
#endif
#endif /* MSP_H */
