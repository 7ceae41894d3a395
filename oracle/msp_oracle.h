/*
 * msp_oracle.h -- reference (oracle) solver for the feasibility market split
 * problem, used ONLY as test infrastructure: by the tests, by the smoke check
 * and by the benchmark's CPU-baseline leg.  Nothing in the GPU library
 * includes, links or calls this code, and this code includes nothing of the
 * GPU library.
 *
 * Problem (Section 1, eq. nSSP): given A in N0^{m x n} and d in N0^m, find
 * every x in {0,1}^n with sum_j a_ij x_j = d_i for i = 1..m.
 *
 * The 1-D key of Section 1, eq. surrogate: with D = max(100, max a_ij + 1)
 * and base B = n*D, key(x) = sum_{i<r} B^i (a_i . x) over the first r rows
 * (row 1 least significant).  Because every partial row sum is < B, key(x) = K_d
 * (= sum_{i<r} B^i d_i) holds exactly when rows 1..r hold.  key_base = 1
 * (every routine takes it after key_rows) swaps B for the mixed radix
 * rowsum_i + 1 of each key row: the digits a_i . x still stay below their
 * radix, so the key stays exact with a smaller K_d; key_base = 0 is the
 * paper's choice.
 *
 * A key past int64 (six or more rows in radix n*D at n >= 20, say): orc_brute
 * and orc_mitm_residues keep every key value modulo 2^64 (exact for residues
 * modulo 2^k, so slices must be powers of two) and decide k_L + k_R = K_d on
 * what the key encodes, the equality of the key rows' sums; orc_key_setup
 * and orc_ss_heap return -3 for such keys.
 *
 * H ("1-D hits") = #{x : key(x) = K_d} = #{x : rows 1..r hold}.
 * S = the full solution set.  Slice (optional): only x whose left-half key
 * k_L(x) = key of x restricted to columns 0..ceil(n/2)-1 satisfies
 * k_L(x) mod slice_mod == slice_res.
 *
 * Quarter partition (the paper leaves it open, Algorithm 1 "partition S into
 * A,B,C,D of size ~n/4"): contiguous columns, h_L = ceil(n/2),
 * q_A = ceil(h_L/2), q_B = floor(h_L/2), q_C = ceil((n-h_L)/2), q_D the rest.
 *
 * Pins (tests/test_oracle.py, tests/test_oracle_mitm_pins.py): orc_brute,
 * orc_dp_count_row, orc_dp_count_2rows and orc_ss_heap are pinned by closed
 * forms, brute force and the paper's expected number of solutions.
 * orc_mitm_residues is pinned against brute force (n <= 22, r = 1..3), and
 * against orc_ss_heap on whole solves of (4,30) (r = 1), of the (6,50) seed-0
 * instance and its planted twin (r = 1, 2, 3; moduli 2^9..2^12 and a split
 * class range; also r = 1 against the row-1 counting DP), of the (6,50)
 * planted twin with five key rows in the mixed radix, and of the (5,40) pair
 * with r = 2 (two moduli, a split range, and the 2-row counting DP).  With
 * keys past int64 (tests/test_oracle_wide.py) it equals brute force (r = 6, 7
 * at n = 22, two moduli, a split range), the mixed radix on the same rows
 * (where the key fits int64 and keys are compared directly), and its slices
 * partition the solve.  At the sizes of its golden values
 * (tests/test_oracle_mitm_large.py: n = 70, 80, 90, two key rows, a modulus
 * above every left key so that a class is one pair of left row sums) its H
 * equals the product of the two halves' subset counts by row sums (a
 * dynamic programme in the test), up to 7e12 hits per class, and the
 * planted vector is among the class's solutions.  Key rows 3 and 4, which
 * most n >= 70 golden values add, are pinned at the smaller sizes above.
 *
 * Every entry point returns 0 on success or a negative code:
 *   -1 invalid argument, -2 row sum exceeds 65534, -3 key overflows int64,
 *   -4 problem too large for this routine, -5 out of memory.
 */
#ifndef MSP_ORACLE_H
#define MSP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    uint64_t h_lo, h_hi;  /* 128-bit count of 1-D hits H (within the slice) */
    uint64_t nsol;        /* |S| (within the slice); may exceed capacity     */
    uint64_t stored;      /* solution vectors written to the caller's buffer */
} orc_result;

/* Brute force over all 2^n vectors (the definition written out), n <= 30.
 * hr[k] (k = 0..m-1) receives #{x : rows 1..k+1 hold} (inside the slice,
 * which is defined with `key_rows` rows).  sol: capacity*n bytes of 0/1. */
int orc_brute(const int32_t *A, const int32_t *d, int m, int n, int key_rows, int key_base,
              int64_t slice_mod, int64_t slice_res, uint64_t *hr,
              uint8_t *sol, uint64_t capacity, orc_result *res);

/* Number of subsets of a[0..n) summing to target: textbook subset-sum
 * counting dynamic programme, exact 128-bit counts. */
int orc_dp_count_row(const int32_t *a, int n, int64_t target,
                     uint64_t *lo, uint64_t *hi);

/* Number of subsets meeting two rows at once (2-D counting DP), n <= 63. */
int orc_dp_count_2rows(const int32_t *a1, const int32_t *a2, int n,
                       int64_t t1, int64_t t2, uint64_t *count);

/* Schroeppel-Shamir with a min-heap over 2^A x 2^B and a max-heap over
 * 2^C x 2^D (Algorithm 1) on the 1-D key, every equal-key group verified
 * against all m rows by an exact sort-and-search join of the partial vectors
 * (Algorithms 2 and 3; exact vectors instead of hashes). */
int orc_ss_heap(const int32_t *A, const int32_t *d, int m, int n, int key_rows, int key_base,
                int64_t slice_mod, int64_t slice_res,
                uint8_t *sol, uint64_t capacity, orc_result *res);

/* Meet-in-the-middle by residue class of the left key modulo M = 2^log2_m:
 * for each class rho in [rho_lo, rho_hi) (and inside the slice) list every
 * left half with k_L = rho (mod M) and every right half with
 * K_d - k_R = rho (mod M), count equal-key pairs and join the full row
 * vectors.  Summed over all classes this is the whole solve.
 * The slice must satisfy slice_mod | M. */
int orc_mitm_residues(const int32_t *A, const int32_t *d, int m, int n,
                      int key_rows, int key_base, int log2_m, int64_t rho_lo, int64_t rho_hi,
                      int64_t slice_mod, int64_t slice_res,
                      uint8_t *sol, uint64_t capacity, orc_result *res);

/* The key setup shared by the routines above, exposed for tests: the radix
 * of row 1 (*base), K_d and the per-column key weights w_j (n entries).
 * *infeasible is set when some key row has d_i > row sum (then H = 0). */
int orc_key_setup(const int32_t *A, const int32_t *d, int m, int n, int key_rows,
                  int key_base, int64_t *base, int64_t *kd, int64_t *w, int *infeasible);

/* orc_key_setup that also takes a key past int64: then *wide = 1 and K_d
 * and w are the values modulo 2^64 (as int64 bit patterns). */
int orc_key_setup_wide(const int32_t *A, const int32_t *d, int m, int n, int key_rows,
                       int key_base, int64_t *base, int64_t *kd, int64_t *w, int *infeasible,
                       int *wide);

#ifdef __cplusplus
}
#endif
#endif
