// Internal declarations shared by the engine and the kernels of libmsp.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace msp {

constexpr int kMaxWords = 5;        // packed uint16 non-key rows: up to 10 rows
constexpr int kMaxN = 100;          // variables per instance (two halves of <= 50)
constexpr int kMaxFine = 4096;      // fine buckets per residue cell (LDS counters)
constexpr int kJoinCap = 1536;      // left records per bucket held in LDS by the join
constexpr int kJoinSlots = 4096;    // LDS hash slots of the join (power of two)
constexpr int kTileL = 4096;        // left records per verify tile
constexpr int kThreads = 256;
constexpr int kBigPairs = 4096;     // equal-key groups with this many pairs go to the tiled verify
constexpr int kMaxBig = 64;         // such groups exported per chunk pair (the rest verified in place)
constexpr int kLightGroup = 256;    // largest left group the light join verifies per lane
constexpr uint32_t kGroupCap = 1344;   // left records per bucket in the grouped join
constexpr uint32_t kGroupSlots = 2048; // its LDS table (at most two-thirds full)
constexpr uint32_t kGroupCapBig = 4096;    // the same for buckets of a few thousand records
constexpr uint32_t kGroupSlotsBig = 8192;  // (1024-thread work-groups, one-word records)

// Multipliers of the row fingerprint h(v) = sum_i kFpMul[i] * v_i mod 2^32
// over the non-key rows (odd constants).  h is linear, so a half record's
// fingerprint is the sum of its two quarters', and the right side stores
// h(d) - h(v_c) - h(v_e).
constexpr uint32_t kFpMul[2 * kMaxWords] = {0x9E3779B1u, 0x85EBCA77u, 0xC2B2AE3Du, 0x27D4EB2Fu,
                                            0x165667B1u, 0xD3A2646Du, 0xFD7046C5u, 0xB55A4F09u,
                                            0x8F1BBCDBu, 0x6C8E9CF5u};

// Everything the kernels need to know about one solve.
struct Plan {
    int32_t m, n, r, nv, W;          // rows, columns, key rows, non-key rows, words
    int32_t qa, qb, qc, qd, hL;      // quarter widths, left-half width
    int32_t log2M, log2T, log2F;     // modulus M, cells T, fine buckets per cell F
    int32_t parts;                   // work-groups per cell in count/scatter
    int32_t exact;                   // 1: M > K_d, each bucket is one key value
    int32_t hsh;                     // qa + qb: shift of the key in Rec::hdr
    int32_t join_grouped;            // join variant: 0 chains, 1 contiguous groups, 2 pairs
    int32_t gbig;                    // grouped join with 1024-thread groups (big buckets)
    int32_t vjoin;                   // exact runs decided by the vector hash join
    int32_t khb;                     // bits of key >> log2M (every stored key is in [0, K_d])
    int32_t kw;                      // 1: keys past int64 (a high word per quarter subset)
    int32_t wide;                    // 1: half records carry a second key word, vec[Wr - 1]
    int64_t Kd;                      // target key (its low 64 bits when kw)
    int64_t Kdh;                     // kw: high word of the target key
    int64_t slice_mod, slice_res;    // slice on the left key (0 = none)
    int64_t kstep, kfirst;           // cell k = kfirst + idx * kstep
    uint32_t dpk[kMaxWords];         // packed non-key right-hand sides
    uint32_t Q[4];                   // quarter sizes
    int32_t fp;                      // 1: half records carry a row fingerprint, not the rows
    int32_t Wr;                      // 32-bit words per half record and quarter record (1 with fp)
    uint32_t hd;                     // fingerprint of the non-key right-hand sides
    const uint32_t *qv[4];           // with fp: packed rows (W words) of the sorted quarters
    const int64_t *qkh[4];           // kw: high key words of the sorted quarters
};

// A quarter subset: 1-D key (for quarter C: K_d - key), subset mask, packed
// partial sums of the non-key rows.  Records are packed at 4-byte alignment
// (no padding word for odd W): every access is a dword-aligned load or store.
template <int W>
struct __attribute__((packed, aligned(4))) QRec {
    int64_t key;
    uint32_t vec[W > 0 ? W : 1];     // key and rows adjacent: one wide load for both
    uint32_t mask;
};

// A half record in a bucket: left (key k_a + k_b, packed row sums) or right
// (key K_d - k_c - k_d, packed d' - row sums with 0xFFFF for negatives).
// hdr = outer position | inner position << qa | (key >> log2M) << (qa + qb):
// the low log2M key bits are the bucket's residue, and the subset masks are
// read back from the sorted quarter lists only for solutions.  With a second
// key word (Plan::wide), key >> log2M continues in vec[W - 1]: its bits past
// the 64 - (qa + qb) that the header holds.  Packed at 4-byte alignment like
// QRec: 12 + 4W bytes, so odd W costs no padding.
template <int W>
struct __attribute__((packed, aligned(4))) Rec {
    uint64_t hdr;
    uint32_t vec[W > 0 ? W : 1];
};

static_assert(sizeof(Rec<3>) == 20 && sizeof(QRec<3>) == 24, "packed record layout");

struct RunPair {
    uint32_t l0, nl, r0, nr;         // window-relative record ranges
};

// Device pointers of one solve.
struct DevBufs {
    void *qraw[4];                   // unsorted quarter records
    void *qsrt[4];                   // quarter records sorted by residue cell
    uint32_t *qvraw[4];              // with fp: packed rows of the quarter subsets, raw order
    uint32_t *qvsrt[4];              // ... and in sorted order
    uint32_t *qcnt[4];               // per-cell counts, then exclusive offsets (T+1)
    uint32_t *qcur[4];               // scatter cursors (T)
    uint32_t *cnt[2];                // window counts per side (K*F*P + 1)
    uint32_t *off[2];                // bucket starts per side [c][f] (+1: the total)
    uint32_t *pre[2];                // per part, records of earlier parts in the bucket [c][p][f]
    uint32_t *tot[2];                // records per bucket [c][f]
    void *rec[2];                    // window records per side
    RunPair *runs;                   // run pairs for the tiled verify (record ranges)
    uint32_t *tiles;                 // per run pair tile counts -> offsets (+1)
    RunPair *iruns;                  // run pairs given as ranges of `idx`
    uint32_t *itiles;                // tile offsets of iruns (+1)
    uint32_t *idx;                   // record indices of large equal-key groups
    uint32_t *heavy;                 // buckets deferred to the heavy join
    uint32_t *heavy2;                // ... and those the big-bucket pass defers again
    uint64_t iruns_cap, idx_cap;     // capacities of iruns and idx
    uint32_t *vtab;                  // vector join table: left record index or ~0
    uint32_t vtab_mask;              // slots - 1 (a power of two, >= 2x the left records)
    uint64_t *sol;                   // solutions: (maskL, maskR) pairs
    uint64_t *wscore;                // per planned window: candidate pairs (first-solution order)
    uint64_t *scal;                  // scalars (see Scal)
    void *scan_tmp;                  // scratch of the device-wide scan
    size_t scan_tmp_bytes;
    int64_t *colw;                   // per-column key weight (n; its low word when kw)
    int64_t *colwh;                  // kw: high words of the column weights (n)
    int64_t *qkhraw[4];              // kw: high key words of the quarter subsets, raw order
    int64_t *qkhsrt[4];              // ... and in sorted order
    uint16_t *rows;                  // non-key rows, nv x n
};

// Slots of DevBufs::scal.
// S_OVF is set by the count pass when one work-group enumerates 2^32 or more
// pairs (its 32-bit bucket counters would wrap: bit 1), by the offset pass
// when a bucket's parts add up to 2^32 or more records (bit 4), and when a
// run pair needs 2^32 or more verify tiles (bit 2).
// S_NHEAVY2 counts the buckets the second join pass (big-bucket groups)
// defers to the heavy kernels.
enum Scal {
    S_H_LO = 0, S_H_HI, S_NSOL, S_NRUNS, S_TOT_L, S_TOT_R, S_TOT_TILES, S_STORED,
    S_NIRUNS, S_TOT_ITILES, S_IDX, S_NHEAVY, S_NHEAVY2, S_OVF, S_COUNT
};

// Launchers (kernels.hip).  All asynchronous on `st`.
hipError_t launch_quarters(const Plan &p, const DevBufs &b, int log2T_unused, hipStream_t st);
hipError_t launch_count(const Plan &p, const DevBufs &b, int64_t idx0, int32_t K, hipStream_t st);
// Grid checks of the launchers: a launch the device cannot take returns
// hipErrorInvalidConfiguration before anything is enqueued.
hipError_t launch_scatter(const Plan &p, const DevBufs &b, int64_t idx0, int32_t K, hipStream_t st);
hipError_t launch_exact_runs(const Plan &p, const DevBufs &b, int32_t K, hipStream_t st);
hipError_t launch_hash_join(const Plan &p, const DevBufs &b, int32_t K, uint64_t sol_cap,
                            hipStream_t st);
// mode 0: exact run pairs, 1: key-checked run pairs, 2: indexed run pairs.
hipError_t launch_verify(const Plan &p, const DevBufs &b, uint32_t nruns, uint32_t ntiles,
                         uint64_t sol_cap, int mode, hipStream_t st);
// Adds sum over the nbk buckets of tot[0][b] * tot[1][b] (left x right
// records) to *score.
hipError_t launch_window_score(const DevBufs &b, uint64_t nbk, uint64_t *score, hipStream_t st);
// Exact-bucket runs decided by a hash join on the packed non-key rows.
hipError_t launch_vector_join(const Plan &p, const DevBufs &b, uint32_t nruns, uint64_t sol_cap,
                              hipStream_t st);
hipError_t launch_tile_counts(const Plan &p, const DevBufs &b, uint32_t nruns, int mode,
                              hipStream_t st);
// Exclusive scan of n uint32 values (out[n] = total; out may equal in);
// the total is also stored to *total64 when non-null.
hipError_t scan_u32(const uint32_t *in, uint32_t *out, size_t n, uint64_t *total64,
                    void *tmp, size_t tmp_bytes, hipStream_t st);
size_t scan_tmp_bytes(size_t n);
// Offsets of the count pass's part-major counts (nbk = cells x F buckets):
// per-part prefixes within each bucket to `pre`, bucket totals to `tot`, and
// bucket starts to `start` (start[nbk] = total, also to *total64 exactly).
// A bucket total of 2^32 or more sets bit 4 of *ovf (S_OVF).
hipError_t scan_counts(const uint32_t *cnt, uint32_t *pre, uint32_t *tot, uint32_t *start,
                       uint64_t nbk, uint32_t F, uint32_t P, uint64_t *total64, uint64_t *ovf,
                       void *tmp, size_t tmp_bytes, hipStream_t st);

size_t qrec_bytes(int W);
size_t rec_bytes(int W);

}  // namespace msp
