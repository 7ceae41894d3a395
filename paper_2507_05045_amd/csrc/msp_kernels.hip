// HIP kernels of libmsp for gfx950 (wave64).  Integer only; no MFMA: nothing
// on this path is a dense contraction.
//
// Pipeline of one solve (Section 2, Algorithm 1, and Section 3, Algorithm 2):
//   quarter lists  -> residue-cell sort of each quarter
//   per window of residue cells:
//     bucket count -> offset scan -> bucket scatter (half records grouped by
//     residue bucket) -> per-bucket equal-key join (+ verify of small runs)
//     -> tiled verify of large equal-key runs against the non-key rows.
//
// Residue structure.  Left key k_L = k_a + k_b, right target t_R = K_d - k_c
// - k_d; a pair is a 1-D hit iff k_L == t_R.  A bucket is a residue class
// rho = key mod M (M = 2^log2M).  A residue cell is rho mod T (T = 2^log2T,
// low bits), the fine index f = (key mod M) >> log2T.  Because cells use the
// low bits, cell(a + b) = cell(a) + cell(b) mod T exactly, so the left
// records of output cell k are exactly the products A_i x B_{k-i}: every
// enumerated pair lands in the cell being built.
#include <type_traits>

#include "msp_internal.h"

#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cstring>

namespace msp {

// ---------------------------------------------------------------------------
// Small device helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// Sum over a block of NT threads (lds holds NT / 64 words); result valid in
// thread 0.
template <int NT = 256>
__device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, uint64_t *lds) {
    v = wave_sum_u64(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    uint64_t t = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NT / 64; ++w) t += lds[w];
    __syncthreads();
    return t;
}

__device__ __forceinline__ void add_u128(uint64_t *lo, uint64_t *hi, uint64_t v) {
    if (!v) return;
    unsigned long long old = atomicAdd((unsigned long long *)lo, (unsigned long long)v);
    if (old + v < old) atomicAdd((unsigned long long *)hi, 1ull);
}

// Inclusive scan across a wave of 64 lanes.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int lane = threadIdx.x & 63;
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive scan of a[0 .. 256*E) held in LDS, by a 256-thread block.
// Returns the total.  `w4` is 4 words of LDS scratch.
template <int E>
__device__ uint32_t block_excl_scan_lds(uint32_t *a, uint32_t *w4) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    uint32_t loc[E];
    uint32_t s = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) { loc[e] = a[t * E + e]; s += loc[e]; }
    uint32_t inc = wave_incl_scan(s);
    if (lane == 63) w4[wave] = inc;
    __syncthreads();
    uint32_t wbase = 0, total = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        uint32_t x = w4[w];
        if (w < wave) wbase += x;
        total += x;
    }
    uint32_t run = wbase + inc - s;
#pragma unroll
    for (int e = 0; e < E; ++e) { a[t * E + e] = run; run += loc[e]; }
    __syncthreads();
    return total;
}

// Packed right residual: per 16-bit half, d'_i - c_i - e_i, or 0xFFFF when
// negative (a left half-sum never equals 0xFFFF because row sums <= 65534).
__device__ __forceinline__ uint32_t resid_word(uint32_t dp, uint32_t c, uint32_t e) {
    int lo = (int)(dp & 0xFFFFu) - (int)(c & 0xFFFFu) - (int)(e & 0xFFFFu);
    int hi = (int)(dp >> 16) - (int)(c >> 16) - (int)(e >> 16);
    uint32_t l = lo < 0 ? 0xFFFFu : (uint32_t)lo;
    uint32_t h = hi < 0 ? 0xFFFFu : (uint32_t)hi;
    return l | (h << 16);
}

template <int W>
struct QPtrs { QRec<W> *q[4]; };
struct UPtrs { uint32_t *q[4]; };
struct KPtrs { int64_t *q[4]; };

// A record's key above the residue, key >> log2M: the header's high bits
// and, with a second key word (p.wide), their continuation in the record's
// last word.  Equal for two records exactly when their keys are equal.
__device__ __forceinline__ uint64_t hkey(const Plan &p, uint64_t hdr, uint32_t kx) {
    uint64_t k = hdr >> p.hsh;
    if (p.wide) k |= (uint64_t)kx << (64 - p.hsh);
    return k;
}

template <int W>
__device__ __forceinline__ uint32_t kword(const uint32_t *v) {
    return W >= 2 ? v[W - 1] : 0u;
}

template <int W>
__device__ __forceinline__ int64_t rkey(const Plan &p, const Rec<W> &r) {
    return (int64_t)hkey(p, r.hdr, kword<W>(r.vec));
}

// The subset masks of a half record (outer | inner << width of the outer).
template <int W>
__device__ __forceinline__ uint64_t half_mask(const Plan &p, const QPtrs<W> &qs, int side,
                                              uint64_t hdr) {
    const uint32_t o = (uint32_t)(hdr & ((1ull << p.qa) - 1));
    const uint32_t i = (uint32_t)((hdr >> p.qa) & ((1ull << p.qb) - 1));
    const QRec<W> *outer = qs.q[side ? 2 : 0], *inner = qs.q[side ? 3 : 1];
    return (uint64_t)outer[o].mask | ((uint64_t)inner[i].mask << (side ? p.qc : p.qa));
}

// ---------------------------------------------------------------------------
// Quarter lists (Algorithm 1, the power sets 2^A .. 2^D with their sums)
// ---------------------------------------------------------------------------

// One thread per subset u of one quarter: its key weight, its packed partial
// sums of the non-key rows, and its residue cell (counted).
template <int W>
__global__ __launch_bounds__(256) void k_quarter_gen(Plan p, const int64_t *__restrict__ colw,
                                                     const int64_t *__restrict__ colwh,
                                                     const uint16_t *__restrict__ rows,
                                                     QPtrs<W> out, UPtrs cnt, UPtrs qvec,
                                                     KPtrs qkh) {
    __shared__ int64_t s_w[kMaxN];
    __shared__ int64_t s_wh[kMaxN];
    __shared__ uint16_t s_rows[kMaxWords * 2 * kMaxN];
    for (int i = threadIdx.x; i < p.n; i += blockDim.x) {
        s_w[i] = colw[i];
        s_wh[i] = p.kw ? colwh[i] : 0;
    }
    for (int i = threadIdx.x; i < p.nv * p.n; i += blockDim.x) s_rows[i] = rows[i];
    __syncthreads();
    uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int x = 0;
    while (x < 4 && g >= p.Q[x]) { g -= p.Q[x]; ++x; }
    if (x >= 4) return;
    const int col0 = x == 0 ? 0 : x == 1 ? p.qa : x == 2 ? p.hL : p.hL + p.qc;
    const int width = x == 0 ? p.qa : x == 1 ? p.qb : x == 2 ? p.qc : p.qd;
    const uint32_t u = (uint32_t)g;
    // Key in 128 bits (lo, hi) when it does not fit int64 (p.kw), else lo.
    uint64_t klo = 0;
    int64_t khi = 0;
    uint32_t s[kMaxWords * 2];
#pragma unroll
    for (int v = 0; v < kMaxWords * 2; ++v) s[v] = 0;
    for (int b = 0; b < width; ++b) {
        if (!((u >> b) & 1u)) continue;
        const int j = col0 + b;
        const uint64_t wl = (uint64_t)s_w[j];
        klo += wl;
        khi += s_wh[j] + (klo < wl ? 1 : 0);
#pragma unroll
        for (int v = 0; v < kMaxWords * 2; ++v)
            if (v < p.nv) s[v] += s_rows[v * p.n + j];
    }
    if (x == 2) {                        // quarter C carries K_d - k_c
        const uint64_t kl = (uint64_t)p.Kd;
        khi = p.Kdh - khi - (kl < klo ? 1 : 0);
        klo = kl - klo;
    }
    QRec<W> r;
    r.key = (int64_t)klo;
    r.mask = u;
    if (p.kw) qkh.q[x][u] = khi;
    if (p.fp) {
        // Fingerprint: sum_v kFpMul[v] * s_v mod 2^32 (linear, so the halves
        // add up); the packed rows go to their own array for exact checks.
        uint32_t h = 0;
#pragma unroll
        for (int v = 0; v < kMaxWords * 2; ++v) h += kFpMul[v] * s[v];
        r.vec[0] = h;
#pragma unroll
        for (int w = 1; w < (W > 0 ? W : 1); ++w) r.vec[w] = 0;
        for (int w = 0; w < p.W; ++w) qvec.q[x][(size_t)u * p.W + w] = s[2 * w] | (s[2 * w + 1] << 16);
    } else {
#pragma unroll
        for (int w = 0; w < (W > 0 ? W : 1); ++w) r.vec[w] = s[2 * w] | (s[2 * w + 1] << 16);
    }
    out.q[x][u] = r;
    const uint32_t T = 1u << p.log2T;
    atomicAdd(&cnt.q[x][(uint32_t)klo & (T - 1)], 1u);
}

// Counting-sort scatter of each quarter by residue cell.
template <int W>
__global__ __launch_bounds__(256) void k_quarter_sort(Plan p, QPtrs<W> raw, QPtrs<W> srt,
                                                      UPtrs cur, UPtrs vraw, UPtrs vsrt,
                                                      KPtrs khraw, KPtrs khsrt) {
    uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int x = 0;
    while (x < 4 && g >= p.Q[x]) { g -= p.Q[x]; ++x; }
    if (x >= 4) return;
    const QRec<W> r = raw.q[x][g];
    const uint32_t T = 1u << p.log2T;
    const uint32_t pos = atomicAdd(&cur.q[x][(uint32_t)r.key & (T - 1)], 1u);
    srt.q[x][pos] = r;
    if (p.kw) khsrt.q[x][pos] = khraw.q[x][g];
    if (p.fp)
        for (int w = 0; w < p.W; ++w)
            vsrt.q[x][(size_t)pos * p.W + w] = vraw.q[x][(size_t)g * p.W + w];
}

// Work-group -> (cell in window, part).  Work-groups are dealt to the 8 XCDs
// round robin, so with P a multiple of 8 each XCD gets parts x, x + 8, ...
// and takes every cell of one part before the next.  A part is a contiguous
// slice of the (cell-sorted) outer list, whose inner partners are then a
// contiguous slice of the inner list as well: each XCD keeps about 8/P of
// the inner list hot in its own L2 instead of all of it.
__device__ __forceinline__ void cell_part(uint32_t b, uint32_t K, uint32_t P, int &cw, int &part) {
    if ((P & 7u) == 0) {
        const uint32_t x = b & 7u, sq = b >> 3;
        part = (int)(x + 8u * (sq / K));
        cw = (int)(sq % K);
    } else {
        cw = (int)(b / P);
        part = (int)(b % P);
    }
}

// ---------------------------------------------------------------------------
// Bucket count and scatter
// ---------------------------------------------------------------------------
//
// Work-group (cell-in-window c, part p, side s).  Side 0 builds left records
// of cell k from (a in A) x (b in B_{k - cell(a)}); side 1 builds right
// records from (c in C) x (e in D_{cell(c) - k}).  Part p takes a contiguous
// slice of the outer quarter.  Counts are laid out [c][f][p] so that one
// exclusive scan makes every bucket (c, f) contiguous, parts in order.

// Count pass (the enumeration of the scatter without records).  Each thread
// takes PER outer elements at a time, 256 apart so that a wave reads
// consecutive records, and loads KU inner keys together (KU about the inner
// elements per outer element of a cell, so few loads are wasted).  The side
// and the slice filter are compile-time.  Out-of-range lanes load a valid
// record and ignore it, so every step issues the same loads.
// A pair's key in 128 bits (keys past int64, KW): low word `lo` from the two
// quarters' low words, the filter (left key <= K_d, right key >= 0) on the
// full value.  Returns whether the pair can meet the other side.
template <int SIDE>
__device__ __forceinline__ bool key128(const Plan &p, uint64_t a, int64_t ah, uint64_t b,
                                       int64_t bh, uint64_t &lo, int64_t &hi) {
    if (SIDE) {
        lo = a - b;
        hi = ah - bh - (a < b ? 1 : 0);
        return hi >= 0;
    }
    lo = a + b;
    hi = ah + bh + (lo < a ? 1 : 0);
    return hi < p.Kdh || (hi == p.Kdh && lo <= (uint64_t)p.Kd);
}

template <int W, int PER, int KU, bool SLICE, int SIDE, bool KW>
__device__ __forceinline__ void count_body(const Plan &p, const QRec<W> *__restrict__ outer,
                                           const QRec<W> *__restrict__ inner,
                                           const uint32_t *__restrict__ ioff, uint64_t Qo,
                                           uint32_t *cnt, int64_t idx0, uint64_t *scal,
                                           uint32_t *s_f, unsigned long long *s_pairs,
                                           const int64_t *__restrict__ okh,
                                           const int64_t *__restrict__ ikh) {
    const int P = p.parts;
    int cw, part;
    cell_part(blockIdx.x, gridDim.x / P, P, cw, part);
    const int t = threadIdx.x;
    const uint32_t T = 1u << p.log2T;
    const int F = 1 << p.log2F;
    const uint32_t k = (uint32_t)(p.kfirst + (idx0 + cw) * p.kstep) & (T - 1);
    for (int f = t; f < F; f += 256) s_f[f] = 0u;
    if (t == 0) *s_pairs = 0;
    __syncthreads();
    const uint64_t lo = Qo * part / P, hi = Qo * (part + 1) / P;
    const int64_t smod1 = p.slice_mod - 1, sres = p.slice_res, Kd = p.Kd;
    const int lt = p.log2T;
    const uint32_t fmask = (uint32_t)F - 1;
    uint64_t npairs = 0;                 // pairs this thread enumerates
    for (uint64_t c0 = lo; c0 < hi; c0 += (uint64_t)256 * PER) {
        int64_t ak[PER], akh[PER];
        uint32_t b0[PER], b1[PER];
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const uint64_t i = c0 + (uint64_t)e * 256 + t;
            ak[e] = outer[i < hi ? i : lo].key;
            akh[e] = KW ? okh[i < hi ? i : lo] : 0;
        }
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const uint32_t ca = (uint32_t)ak[e] & (T - 1);
            const uint32_t j = SIDE ? ((ca - k) & (T - 1)) : ((k - ca) & (T - 1));
            b0[e] = ioff[j];
            b1[e] = ioff[j + 1];
        }
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            if (c0 + (uint64_t)e * 256 + t >= hi) b1[e] = b0[e];
            npairs += b1[e] - b0[e];
            for (uint32_t q0 = b0[e]; q0 < b1[e]; q0 += KU) {
                int64_t bk[KU], bkh[KU];
#pragma unroll
                for (int u = 0; u < KU; ++u) {
                    bk[u] = inner[min(q0 + u, b1[e] - 1)].key;
                    bkh[u] = KW ? ikh[min(q0 + u, b1[e] - 1)] : 0;
                }
#pragma unroll
                for (int u = 0; u < KU; ++u) {
                    if (q0 + u >= b1[e]) break;
                    int64_t key;
                    bool keep;
                    if (KW) {
                        uint64_t l;
                        int64_t h;
                        keep = key128<SIDE>(p, (uint64_t)ak[e], akh[e], (uint64_t)bk[u], bkh[u], l, h);
                        key = (int64_t)l;
                    } else {
                        key = SIDE ? ak[e] - bk[u] : ak[e] + bk[u];
                        keep = SIDE ? key >= 0 : key <= Kd;   // only these can meet
                    }
                    if (SLICE) keep = keep && ((key & smod1) == sres);
                    if (keep) atomicAdd(&s_f[(uint32_t)((uint64_t)key >> lt) & fmask], 1u);
                }
            }
        }
    }
    if (npairs) atomicAdd(s_pairs, (unsigned long long)npairs);
    __syncthreads();
    // Counts of one work-group are contiguous ([cell][part][fine] layout):
    // whole cache lines, not one word per line.
    const uint64_t cbase = ((uint64_t)cw * P + part) * F;
    for (int f = t; f < F; f += 256) cnt[cbase + f] = s_f[f];
    if (t == 0 && *s_pairs > 0xFFFFFFFFull) atomicOr((unsigned long long *)&scal[S_OVF], 1ull);
}

template <int W, int PER, int KU, bool SLICE, bool KW>
__global__ __launch_bounds__(256) void k_count(Plan p, const QRec<W> *__restrict__ A,
                                               const QRec<W> *__restrict__ B,
                                               const uint32_t *__restrict__ offB,
                                               const QRec<W> *__restrict__ Cq,
                                               const QRec<W> *__restrict__ Dq,
                                               const uint32_t *__restrict__ offD,
                                               uint32_t *cntL, uint32_t *cntR, int64_t idx0,
                                               uint64_t *scal) {
    __shared__ uint32_t s_f[kMaxFine];
    __shared__ unsigned long long s_pairs;
    if (blockIdx.y == 0)
        count_body<W, PER, KU, SLICE, 0, KW>(p, A, B, offB, p.Q[0], cntL, idx0, scal, s_f,
                                             &s_pairs, p.qkh[0], p.qkh[1]);
    else
        count_body<W, PER, KU, SLICE, 1, KW>(p, Cq, Dq, offD, p.Q[2], cntR, idx0, scal, s_f,
                                             &s_pairs, p.qkh[2], p.qkh[3]);
}

// Exclusive scan of a[0 .. n) in LDS by an NT-thread block (n a multiple of
// NT, at most 16 NT); wv holds NT / 64 wave totals.  Returns the total.
template <typename T, int NT = 256>
__device__ uint32_t block_excl_scan_rt(T *a, int n, uint32_t *wv) {
    constexpr int NW = NT / 64;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int E = n / NT;
    uint32_t loc[16];
    uint32_t s = 0;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        loc[e] = e < E ? (uint32_t)a[t * E + e] : 0u;
        s += loc[e];
    }
    const uint32_t inc = wave_incl_scan(s);
    if (lane == 63) wv[wave] = inc;
    __syncthreads();
    uint32_t wbase = 0, total = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const uint32_t x = wv[w];
        if (w < wave) wbase += x;
        total += x;
    }
    uint32_t run = wbase + inc - s;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        if (e < E) { a[t * E + e] = (T)run; run += loc[e]; }
    }
    __syncthreads();
    return total;
}

// Bucket scatter staged through LDS.  The work-group enumerates its pairs in
// batches; each batch is counting-sorted by fine bucket in LDS and written
// out so that consecutive lanes store consecutive records of one bucket
// (whole cache lines instead of one partial line per record).  Only the pair
// (outer element, inner element) and its fine bucket are staged, 8 bytes per
// pair: the record itself is rebuilt from the quarter lists at write-out,
// which costs two cached loads instead of a 16-24 byte LDS round trip.
constexpr int kStageBatch = 3072;          // pairs per LDS batch (index staging, per 256 threads)

// Records of two or more row words: the pair's (outer, inner) indices are
// staged (10 bytes per pair, batches of 12 per thread) and the record is
// rebuilt from the quarter lists at write-out.
template <int W, int PER, int MAXF, int NT>
__global__ __launch_bounds__(NT) void k_scatter_staged(Plan p, const QRec<W> *__restrict__ A,
                                                        const QRec<W> *__restrict__ B,
                                                        const uint32_t *__restrict__ offB,
                                                        const QRec<W> *__restrict__ Cq,
                                                        const QRec<W> *__restrict__ Dq,
                                                        const uint32_t *__restrict__ offD,
                                                        const uint32_t *__restrict__ offL,
                                                        const uint32_t *__restrict__ offR,
                                                        const uint32_t *__restrict__ preL,
                                                        const uint32_t *__restrict__ preR,
                                                        Rec<W> *recL, Rec<W> *recR, int64_t idx0) {
    constexpr int BATCH = kStageBatch * (NT / 256);
    constexpr int NW = NT / 64;
    constexpr int per = PER;                     // outer elements per thread per chunk
    constexpr int WV = W > 0 ? W : 1;
    static_assert(NT * PER <= 65536, "chunk-relative outer index must fit 16 bits");
    static_assert(BATCH <= 65536, "batch slots must fit 16 bits");
    __shared__ uint32_t s_cur[MAXF];
    __shared__ uint32_t s_cnt[MAXF];
    __shared__ uint32_t s_q[BATCH];              // inner element of the pair
    __shared__ uint16_t s_io[BATCH];             // outer element, relative to the chunk
    __shared__ uint16_t s_f[BATCH];              // fine bucket, 0xFFFF = filtered out
    __shared__ uint16_t s_perm[BATCH];
    __shared__ uint32_t s_w4[NW];
    const int side = blockIdx.y;
    const int P = p.parts;
    int cw, part;
    cell_part(blockIdx.x, gridDim.x / P, P, cw, part);
    const int t = threadIdx.x;
    const uint32_t T = 1u << p.log2T;
    const int F = 1 << p.log2F;
    const int Fs = F < NT ? NT : F;              // scan length (multiple of NT)
    const int64_t M1 = ((int64_t)1 << p.log2M) - 1;
    const uint32_t k = (uint32_t)(p.kfirst + (idx0 + cw) * p.kstep) & (T - 1);
    const QRec<W> *outer = side ? Cq : A;
    const QRec<W> *inner = side ? Dq : B;
    const uint32_t *ioff = side ? offD : offB;
    const uint64_t Qo = side ? p.Q[2] : p.Q[0];
    const uint32_t *pre = side ? preR : preL;
    const uint32_t *bst = side ? offR : offL;
    Rec<W> *rec = side ? recR : recL;
    // Where this work-group's records of bucket (cell, f) start: the bucket's
    // start plus the records of the parts before it (both contiguous in f).
    const uint64_t tbase = ((uint64_t)cw * P + part) * F;
    for (int f = t; f < F; f += NT) s_cur[f] = bst[(uint64_t)cw * F + f] + pre[tbase + f];
    const uint64_t lo = Qo * part / P, hi = Qo * (part + 1) / P;
    const int64_t smod1 = p.slice_mod - 1;
    for (uint64_t c0 = lo; c0 < hi; c0 += (uint64_t)NT * per) {
        // This thread's outer elements (per of them, NT apart so that a wave
        // reads consecutive records) and the chunk-relative offsets of their
        // pairs.
        // Every lane issues the same loads (past the end it reads element lo
        // and ignores it), so the keys, then the cell ranges, of all its
        // elements are in flight together.
        int64_t akey[PER];
        uint32_t b0[PER], nn[PER], c1[PER];
        uint32_t mysum = 0;
#pragma unroll
        for (int e = 0; e < per; ++e) {
            const uint64_t i = c0 + (uint64_t)e * NT + t;
            akey[e] = outer[i < hi ? i : lo].key;
        }
#pragma unroll
        for (int e = 0; e < per; ++e) {
            const uint32_t ca = (uint32_t)akey[e] & (T - 1);
            const uint32_t j = side ? ((ca - k) & (T - 1)) : ((k - ca) & (T - 1));
            b0[e] = ioff[j];
            c1[e] = ioff[j + 1];
        }
#pragma unroll
        for (int e = 0; e < per; ++e) {
            nn[e] = (c0 + (uint64_t)e * NT + t < hi) ? c1[e] - b0[e] : 0u;
            mysum += nn[e];
        }
        const uint32_t inc = wave_incl_scan(mysum);
        __syncthreads();                          // previous chunk done with s_w4
        if ((t & 63) == 63) s_w4[t >> 6] = inc;
        __syncthreads();
        uint32_t myoff = inc - mysum, total = 0;
        for (int w = 0; w < NW; ++w) {
            if (w < (t >> 6)) myoff += s_w4[w];
            total += s_w4[w];
        }
        for (uint32_t P0 = 0; P0 < total; P0 += BATCH) {
            const uint32_t nb = min((uint32_t)BATCH, total - P0);
            for (int f = t; f < Fs; f += NT) s_cnt[f] = 0;
            // Stage my pairs whose index falls in [P0, P0 + nb).
            uint32_t off = myoff;
#pragma unroll
            for (int e = 0; e < per; ++e) {
                const uint32_t n = nn[e];
                const uint32_t qa = off >= P0 ? 0u : min(n, P0 - off);
                const uint32_t qb = (off + n <= P0 + nb) ? n : (P0 + nb > off ? P0 + nb - off : 0u);
                // Keys of up to 8 inner elements are loaded together, then used.
                constexpr int kU = 8;
                for (uint32_t q0 = qa; q0 < qb; q0 += kU) {
                    int64_t bk[kU];
#pragma unroll
                    for (int u = 0; u < kU; ++u)
                        if (q0 + u < qb) bk[u] = inner[b0[e] + q0 + u].key;
#pragma unroll
                    for (int u = 0; u < kU; ++u) {
                        if (q0 + u >= qb) break;
                        const int64_t key = side ? akey[e] - bk[u] : akey[e] + bk[u];
                        bool keep = side ? key >= 0 : key <= p.Kd;
                        if (p.slice_mod) keep = keep && ((key & smod1) == p.slice_res);
                        const uint32_t o = off + q0 + u - P0;
                        s_q[o] = b0[e] + q0 + u;
                        s_io[o] = (uint16_t)(e * NT + t);
                        s_f[o] = keep ? (uint16_t)((key & M1) >> p.log2T) : (uint16_t)0xFFFF;
                    }
                }
                off += n;
            }
            __syncthreads();
            for (uint32_t o = t; o < nb; o += NT)
                if (s_f[o] != 0xFFFF) atomicAdd(&s_cnt[s_f[o]], 1u);
            __syncthreads();
            const uint32_t nvalid = block_excl_scan_rt<uint32_t, NT>(s_cnt, Fs, s_w4);
            // Rank within the batch; afterwards s_cnt[f] = end of group f.
            for (uint32_t o = t; o < nb; o += NT) {
                const uint32_t f = s_f[o];
                if (f != 0xFFFF) s_perm[atomicAdd(&s_cnt[f], 1u)] = (uint16_t)o;
            }
            __syncthreads();
            for (uint32_t o = t; o < nvalid; o += NT) {
                const uint32_t slot = s_perm[o];
                const uint32_t f = s_f[slot];
                const uint32_t start = f ? s_cnt[f - 1] : 0u;
                const uint32_t q = s_q[slot];
                const uint64_t ai = c0 + s_io[slot];
                // Key and rows only (adjacent in QRec): the mask is not needed.
                const int64_t ak = outer[ai].key, bk = inner[q].key;
                uint32_t av[WV], bv[WV];
#pragma unroll
                for (int w = 0; w < WV; ++w) {
                    av[w] = outer[ai].vec[w];
                    bv[w] = inner[q].vec[w];
                }
                const int64_t key = side ? ak - bk : ak + bk;
                Rec<W> r;
                r.hdr = ai | ((uint64_t)q << p.qa) | ((uint64_t)(key >> p.log2M) << p.hsh);
#pragma unroll
                for (int w = 0; w < WV; ++w)
                    r.vec[w] = side ? resid_word(p.dpk[w], av[w], bv[w]) : av[w] + bv[w];
                rec[s_cur[f] + (o - start)] = r;
            }
            __syncthreads();
            for (int f = t; f < F; f += NT) s_cur[f] += s_cnt[f] - (f ? s_cnt[f - 1] : 0u);
            __syncthreads();
        }
    }
}

// Scatter of one-word records (a fingerprint, one packed word, or none):
// the same enumeration and batching as k_scatter_staged, with the record
// built whole as its pair is enumerated and staged in LDS as it will be
// stored (8-byte header, 4-byte word, fine bucket, permutation slot: 16 bytes
// per pair, 8 per thread; 7 beside 4096 bucket cursors).  The side (left or
// right), the fingerprint and the slice filter are compile-time, so the pair
// loop carries no selects between them.
constexpr int kRecNT = 1024;

// Records staged per batch: 16 bytes each (20 with a second key word) beside
// the bucket cursors, within one CU's 160 KB of LDS.
template <int W, int MAXF>
constexpr int rec_batch() {
    return (W == 2 ? (MAXF > 2048 ? 6 : 7) : (MAXF > 2048 ? 7 : 8)) * kRecNT;
}

// W = 2: records with a second key word (vec[0] the fingerprint, vec[1] the
// bits of key >> log2M past the header's); KW: keys past int64, whose high
// words come from p.qkh.
template <int W, int PER, int MAXF, bool FP, bool SLICE, int SIDE, bool KW>
__device__ __forceinline__ void scatter_rec_body(
    const Plan &p, const QRec<W> *__restrict__ outer, const QRec<W> *__restrict__ inner,
    const uint32_t *__restrict__ ioff, uint64_t Qo, const uint32_t *__restrict__ bst,
    const uint32_t *__restrict__ pre, Rec<W> *rec, int64_t idx0, uint32_t *s_cur,
    uint32_t *s_cnt, uint64_t *s_hdr, uint32_t *s_wd, uint32_t *s_kx, uint16_t *s_f,
    uint16_t *s_perm, uint32_t *s_w4, const int64_t *__restrict__ okh,
    const int64_t *__restrict__ ikh) {
    constexpr int NT = kRecNT;
    constexpr int BATCH = rec_batch<W, MAXF>();
    constexpr int NW = NT / 64;
    const int P = p.parts;
    int cw, part;
    cell_part(blockIdx.x, gridDim.x / P, P, cw, part);
    const int t = threadIdx.x;
    const uint32_t T = 1u << p.log2T;
    const int F = 1 << p.log2F;
    const int Fs = F < NT ? NT : F;              // scan length (multiple of NT)
    const uint32_t k = (uint32_t)(p.kfirst + (idx0 + cw) * p.kstep) & (T - 1);
    const uint64_t tbase = ((uint64_t)cw * P + part) * F;
    for (int f = t; f < F; f += NT) s_cur[f] = bst[(uint64_t)cw * F + f] + pre[tbase + f];
    const uint64_t lo = Qo * part / P, hi = Qo * (part + 1) / P;
    const int64_t smod1 = p.slice_mod - 1, sres = p.slice_res, Kd = p.Kd;
    const int qa = p.qa, hsh = p.hsh, lm = p.log2M, lt = p.log2T;
    const uint32_t hd = p.hd, dp0 = p.dpk[0];
    // Sort the nb staged records by fine bucket and store each bucket's run
    // at its cursor.  Staged slots past nb are stale and never read.
    auto flush = [&](uint32_t nb) {
        for (int f = t; f < Fs; f += NT) s_cnt[f] = 0;
        __syncthreads();                          // staging and zeroing done
        for (uint32_t o = t; o < nb; o += NT)
            if (s_f[o] != 0xFFFF) atomicAdd(&s_cnt[s_f[o]], 1u);
        __syncthreads();
        const uint32_t nvalid = block_excl_scan_rt<uint32_t, NT>(s_cnt, Fs, s_w4);
        // Rank within the batch; afterwards s_cnt[f] = end of group f.
        for (uint32_t o = t; o < nb; o += NT) {
            const uint32_t f = s_f[o];
            if (f != 0xFFFF) s_perm[atomicAdd(&s_cnt[f], 1u)] = (uint16_t)o;
        }
        __syncthreads();
        for (uint32_t o = t; o < nvalid; o += NT) {
            const uint32_t slot = s_perm[o];
            const uint32_t f = s_f[slot];
            const uint32_t start = f ? s_cnt[f - 1] : 0u;
            Rec<W> r;
            r.hdr = s_hdr[slot];
            r.vec[0] = s_wd[slot];
            if constexpr (W == 2) r.vec[1] = s_kx[slot];
            rec[s_cur[f] + (o - start)] = r;
        }
        __syncthreads();
        for (int f = t; f < F; f += NT) s_cur[f] += s_cnt[f] - (f ? s_cnt[f - 1] : 0u);
        __syncthreads();
    };
    // Records are staged across chunks until a batch is full, so chunks of
    // few pairs (cells that hold about one inner element) share one sort.
    uint32_t fill = 0;
    for (uint64_t c0 = lo; c0 < hi; c0 += (uint64_t)NT * PER) {
        // This thread's outer elements (PER of them, NT apart so that a wave
        // reads consecutive records) and the offsets of their pairs in the
        // chunk.  Past the end a lane reads element lo and ignores it, so all
        // loads of an element are issued together.
        int64_t akey[PER], akh[PER];
        uint32_t aw[PER], b0[PER], nn[PER], c1[PER];
        uint32_t mysum = 0;
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const uint64_t i = c0 + (uint64_t)e * NT + t;
            akey[e] = outer[i < hi ? i : lo].key;
            aw[e] = outer[i < hi ? i : lo].vec[0];
            akh[e] = KW ? okh[i < hi ? i : lo] : 0;
        }
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const uint32_t ca = (uint32_t)akey[e] & (T - 1);
            const uint32_t j = SIDE ? ((ca - k) & (T - 1)) : ((k - ca) & (T - 1));
            b0[e] = ioff[j];
            c1[e] = ioff[j + 1];
        }
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            nn[e] = (c0 + (uint64_t)e * NT + t < hi) ? c1[e] - b0[e] : 0u;
            mysum += nn[e];
        }
        const uint32_t inc = wave_incl_scan(mysum);
        __syncthreads();                          // previous chunk done with s_w4
        if ((t & 63) == 63) s_w4[t >> 6] = inc;
        __syncthreads();
        uint32_t myoff = inc - mysum, total = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            if (w < (t >> 6)) myoff += s_w4[w];
            total += s_w4[w];
        }
        if (fill > 0 && fill + total > (uint32_t)BATCH) {   // block-uniform
            flush(fill);
            fill = 0;
        }
        for (uint32_t P0 = 0; P0 < total;) {
            const uint32_t nb = min((uint32_t)BATCH - fill, total - P0);
            // Stage my pairs whose index falls in [P0, P0 + nb), records
            // whole, at slots fill + (index - P0).
            uint32_t off = myoff;
#pragma unroll
            for (int e = 0; e < PER; ++e) {
                const uint32_t n = nn[e];
                const uint32_t qa0 = off >= P0 ? 0u : min(n, P0 - off);
                const uint32_t qb0 = (off + n <= P0 + nb) ? n : (P0 + nb > off ? P0 + nb - off : 0u);
                const uint64_t ai = c0 + (uint64_t)e * NT + t;
                for (uint32_t q = qa0; q < qb0; ++q) {
                    const uint64_t qi = b0[e] + q;
                    const int64_t bk = inner[qi].key;
                    const uint32_t bw = inner[qi].vec[0];
                    int64_t key;
                    bool keep;
                    uint64_t c;                   // key >> log2M
                    if (KW) {
                        uint64_t l;
                        int64_t h;
                        keep = key128<SIDE>(p, (uint64_t)akey[e], akh[e], (uint64_t)bk, ikh[qi], l, h);
                        key = (int64_t)l;
                        c = (l >> lm) | ((uint64_t)h << (64 - lm));
                    } else {
                        key = SIDE ? akey[e] - bk : akey[e] + bk;
                        keep = SIDE ? key >= 0 : key <= Kd;
                        c = (uint64_t)key >> lm;
                    }
                    if (SLICE) keep = keep && ((key & smod1) == sres);
                    const uint32_t o = fill + off + q - P0;
                    s_hdr[o] = ai | (qi << qa) | (c << hsh);
                    if constexpr (W == 2) s_kx[o] = (uint32_t)(c >> (64 - hsh));
                    uint32_t wd;
                    if (FP) wd = SIDE ? hd - aw[e] - bw : aw[e] + bw;
                    else wd = SIDE ? resid_word(dp0, aw[e], bw) : aw[e] + bw;
                    s_wd[o] = wd;
                    s_f[o] = keep ? (uint16_t)((uint32_t)((uint64_t)key >> lt) & (uint32_t)(F - 1))
                                  : (uint16_t)0xFFFF;
                }
                off += n;
            }
            fill += nb;
            P0 += nb;
            if (fill == (uint32_t)BATCH) {
                flush(fill);
                fill = 0;
            }
        }
    }
    if (fill > 0) flush(fill);
}

template <int W, int PER, int MAXF, bool FP, bool SLICE, bool KW>
__global__ __launch_bounds__(kRecNT) void k_scatter_rec(Plan p, const QRec<W> *__restrict__ A,
                                                       const QRec<W> *__restrict__ B,
                                                       const uint32_t *__restrict__ offB,
                                                       const QRec<W> *__restrict__ Cq,
                                                       const QRec<W> *__restrict__ Dq,
                                                       const uint32_t *__restrict__ offD,
                                                       const uint32_t *__restrict__ offL,
                                                       const uint32_t *__restrict__ offR,
                                                       const uint32_t *__restrict__ preL,
                                                       const uint32_t *__restrict__ preR,
                                                       Rec<W> *recL, Rec<W> *recR, int64_t idx0) {
    static_assert(W <= 2, "one-word records, or two with a second key word");
    constexpr int BATCH = rec_batch<W, MAXF>();
    static_assert(BATCH <= 65536, "batch slots must fit 16 bits");
    __shared__ uint32_t s_cur[MAXF];
    __shared__ uint32_t s_cnt[MAXF > kRecNT ? MAXF : kRecNT];
    __shared__ uint64_t s_hdr[BATCH];
    __shared__ uint32_t s_wd[BATCH];
    __shared__ uint32_t s_kx[W == 2 ? BATCH : 1];
    __shared__ uint16_t s_f[BATCH];
    __shared__ uint16_t s_perm[BATCH];
    __shared__ uint32_t s_w4[kRecNT / 64];
    if (blockIdx.y == 0)
        scatter_rec_body<W, PER, MAXF, FP, SLICE, 0, KW>(p, A, B, offB, p.Q[0], offL, preL, recL,
                                                         idx0, s_cur, s_cnt, s_hdr, s_wd, s_kx,
                                                         s_f, s_perm, s_w4, p.qkh[0], p.qkh[1]);
    else
        scatter_rec_body<W, PER, MAXF, FP, SLICE, 1, KW>(p, Cq, Dq, offD, p.Q[2], offR, preR,
                                                         recR, idx0, s_cur, s_cnt, s_hdr, s_wd,
                                                         s_kx, s_f, s_perm, s_w4, p.qkh[2],
                                                         p.qkh[3]);
}

// ---------------------------------------------------------------------------
// Exact buckets (M > K_d): a bucket is one key value, so the whole bucket pair
// is one equal-key run pair (the E_A x E_C groups of Algorithm 1).
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_exact_runs(Plan p, const uint32_t *__restrict__ offL,
                                                    const uint32_t *__restrict__ offR,
                                                    uint32_t nb, RunPair *runs,
                                                    uint64_t *scal, int w_zero) {
    __shared__ uint64_t s4[4];
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t h = 0;
    if (b < nb) {
        const uint32_t l0 = offL[b], l1 = offL[b + 1];
        const uint32_t r0 = offR[b], r1 = offR[b + 1];
        if (l1 > l0 && r1 > r0) {
            h = (uint64_t)(l1 - l0) * (r1 - r0);
            const uint64_t idx = atomicAdd((unsigned long long *)&scal[S_NRUNS], 1ull);
            runs[idx] = RunPair{l0, l1 - l0, r0, r1 - r0};
        }
    }
    const uint64_t t = block_sum_u64(h, s4);
    if (threadIdx.x == 0) {
        add_u128(&scal[S_H_LO], &scal[S_H_HI], t);
        if (w_zero) atomicAdd((unsigned long long *)&scal[S_NSOL], (unsigned long long)t);
    }
}

// Tiles of each run pair; a run pair of 2^32 or more tiles (far beyond any
// pairwise check that ends) sets bit 2 of S_OVF and counts as 0xFFFFFFFF.
__global__ void k_tile_counts(const RunPair *__restrict__ runs, uint32_t n, uint32_t *tiles,
                              uint32_t tile_r, uint64_t *scal) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const RunPair r = runs[i];
    const uint64_t t = (uint64_t)((r.nl + kTileL - 1) / kTileL) * ((r.nr + tile_r - 1) / tile_r);
    if (t > 0xFFFFFFFFull) atomicOr((unsigned long long *)&scal[S_OVF], 2ull);
    tiles[i] = (uint32_t)std::min<uint64_t>(t, 0xFFFFFFFFull);
}

__device__ __forceinline__ void emit_solution(uint64_t *sol, uint64_t cap, uint64_t *ctr,
                                              uint64_t ml, uint64_t mr) {
    const uint64_t idx = atomicAdd((unsigned long long *)ctr, 1ull);
    if (idx < cap) {
        sol[2 * idx] = ml;
        sol[2 * idx + 1] = mr;
    }
}

// Full check of one 1-D hit against the non-key rows (the key rows hold by
// key equality): every packed word of the left sums equals the right residual.
template <int W>
__device__ __forceinline__ bool rows_match(const Rec<W> &l, const Rec<W> &r) {
    bool ok = true;
#pragma unroll
    for (int w = 0; w < W; ++w) ok = ok && (l.vec[w] == r.vec[w]);
    return ok;
}

// Exact check of the non-key rows of a candidate pair from the quarter lists.
// Half records either carry the packed rows themselves (then equality of the
// stored words already is the exact check) or, with p.fp, one 32-bit
// fingerprint of them; a fingerprint match is only a candidate, decided here
// by the packed rows of the four quarter subsets the headers point to.
__device__ __forceinline__ bool exact_rows(const Plan &p, uint64_t hl, uint64_t hr) {
    if (!p.fp) return true;
    const uint64_t mo = (1ull << p.qa) - 1, mi = (1ull << p.qb) - 1;
    const size_t oL = hl & mo, iL = (hl >> p.qa) & mi, oR = hr & mo, iR = (hr >> p.qa) & mi;
    const int W = p.W;
    bool ok = true;
    for (int w = 0; w < W; ++w) {
        const uint32_t l = p.qv[0][oL * W + w] + p.qv[1][iL * W + w];
        const uint32_t r = resid_word(p.dpk[w], p.qv[2][oR * W + w], p.qv[3][iR * W + w]);
        ok = ok && (l == r);
    }
    return ok;
}

// A pair whose stored words match: a solution once its rows hold exactly.
template <int W>
__device__ __forceinline__ void emit_pair(const Plan &p, const QPtrs<W> &qs, uint64_t *sol,
                                          uint64_t cap, uint64_t *ctr, uint64_t hl, uint64_t hr) {
    if (!exact_rows(p, hl, hr)) return;
    emit_solution(sol, cap, ctr, half_mask(p, qs, 0, hl), half_mask(p, qs, 1, hr));
}

// ---------------------------------------------------------------------------
// Hash join of one bucket (keys of several values): left keys grouped by a
// hash table in LDS, right records probe it; small equal-key groups are
// verified in place.  Buckets with more than kJoinCap left records are sent
// to the key-checking tiled verify instead.
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t key_hash(int64_t k) {
    return (uint32_t)(((uint64_t)k * 0x9E3779B97F4A7C15ull) >> 40);
}

// ---------------------------------------------------------------------------
// Vector join of exact-bucket runs.  Within a run every left and right record
// has the same key, so a pair is a solution exactly when the packed non-key
// rows agree word for word (the right side holds d' - rows, 0xFFFF where
// negative, which no left sum reaches).  Algorithms 3-4 decide such pairs by
// encoding the partial vectors, sorting and searching; here the encoding is
// the exact packed vector and the search a hash table: the left records of
// every run go into one open-addressing table keyed by (run, vector), and
// each right record probes it once.  Cost O(|G_L| + |G_R|) per run instead of
// |G_L| |G_R| compares; H is the sum of |G_L| |G_R| as before.
// ---------------------------------------------------------------------------
constexpr uint32_t kVEmpty = 0xFFFFFFFFu;

template <int W>
__device__ __forceinline__ uint32_t vj_hash(uint32_t run, const uint32_t *v) {
    uint32_t h = run * 0x9E3779B1u + 0x7F4A7C15u;
#pragma unroll
    for (int w = 0; w < (W > 0 ? W : 1); ++w) {
        h = (h ^ v[w]) * 0x85EBCA77u;
        h ^= h >> 13;
    }
    h *= 0xC2B2AE35u;
    return h ^ (h >> 16);
}

template <int W>
__global__ __launch_bounds__(256) void k_vjoin_insert(const RunPair *__restrict__ runs,
                                                      uint32_t nruns,
                                                      const Rec<W> *__restrict__ L,
                                                      uint32_t *tab, uint32_t mask) {
    constexpr int WV = W > 0 ? W : 1;
    for (uint32_t ri = blockIdx.x; ri < nruns; ri += gridDim.x) {
        const RunPair r = runs[ri];
        for (uint32_t i = blockIdx.y * 256 + threadIdx.x; i < r.nl; i += 256 * gridDim.y) {
            const uint32_t li = r.l0 + i;
            uint32_t v[WV];
#pragma unroll
            for (int w = 0; w < WV; ++w) v[w] = L[li].vec[w];
            uint32_t h = vj_hash<W>(ri, v) & mask;
            // The table is at most half full: an empty slot is always reached.
            while (atomicCAS(&tab[h], kVEmpty, li) != kVEmpty) h = (h + 1) & mask;
        }
    }
}

template <int W>
__global__ __launch_bounds__(256) void k_vjoin_probe(Plan p, const RunPair *__restrict__ runs,
                                                     uint32_t nruns,
                                                     const Rec<W> *__restrict__ L,
                                                     const Rec<W> *__restrict__ R,
                                                     const uint32_t *__restrict__ tab,
                                                     uint32_t mask, uint64_t *scal, uint64_t *sol,
                                                     uint64_t cap, QPtrs<W> qs) {
    constexpr int WV = W > 0 ? W : 1;
    for (uint32_t ri = blockIdx.x; ri < nruns; ri += gridDim.x) {
        const RunPair r = runs[ri];
        for (uint32_t j = blockIdx.y * 256 + threadIdx.x; j < r.nr; j += 256 * gridDim.y) {
            const uint32_t rj = r.r0 + j;
            uint32_t v[WV];
#pragma unroll
            for (int w = 0; w < WV; ++w) v[w] = R[rj].vec[w];
            for (uint32_t h = vj_hash<W>(ri, v) & mask;; h = (h + 1) & mask) {
                const uint32_t e = tab[h];
                if (e == kVEmpty) break;
                if (e - r.l0 >= r.nl) continue;          // another run's record
                bool ok = true;
#pragma unroll
                for (int w = 0; w < WV; ++w) ok = ok && (L[e].vec[w] == v[w]);
                if (ok)
                    emit_pair(p, qs, sol, cap, &scal[S_NSOL], L[e].hdr, R[rj].hdr);
            }
        }
    }
}

// Light join of one bucket whose equal-key groups are small: left records
// are pushed onto per-slot chains in LDS (one CAS per record, the slot word
// packs chain head and length); each right record walks its slot's chain.
// Buckets with more than kJoinCap left records, or a chain longer than
// kLightGroup, are handed to k_join_heavy unprocessed.
template <int W, bool K32>
__global__ __launch_bounds__(256) void k_join_light(Plan p, const uint32_t *__restrict__ offL,
                                                   const uint32_t *__restrict__ offR,
                                                   const Rec<W> *__restrict__ L,
                                                   const Rec<W> *__restrict__ R, uint32_t *heavy,
                                                   uint64_t *scal, uint64_t *sol, uint64_t cap,
                                                   QPtrs<W> qs, uint32_t nb) {
    constexpr uint32_t kEnd = 0xFFFFu;
    constexpr uint32_t kEmpty = kEnd << 16;               // head = end of chain, length 0
    constexpr int kPre = 4;                              // right records preloaded per lane
    constexpr int kLU = (kJoinCap + 255) / 256;           // left records per lane
    constexpr int WV = W > 0 ? W : 1;
    // Keys in 32 bits when key >> log2M fits (K32): more work-groups per CU.
    using KT = typename std::conditional<K32, uint32_t, int64_t>::type;
    __shared__ KT s_key[kJoinCap];
    __shared__ uint32_t s_vec[WV][kJoinCap];             // left packed rows, by left index
    constexpr uint32_t kLightSlots = 2048;               // load factor <= 3/4 at kJoinCap
    __shared__ uint32_t s_head[kLightSlots];             // (first left index << 16) | length
    __shared__ uint16_t s_next[kJoinCap];
    __shared__ uint64_t s_s4[4];
    __shared__ uint32_t s_gmax;
    const int t = threadIdx.x;
    // A bucket's ranges and this lane's share of its records, in registers.
    // Headers are kept raw (the key shift is applied where they are used), so
    // no instruction depends on a load inside its guard and all loads of a
    // bucket stay in flight together.
    struct Slot {
        uint32_t l0, nl, r0, nr;
        uint64_t lh[kLU];
        uint32_t lv[kLU][WV];
        uint64_t rh[kPre];
        uint32_t rv[kPre][WV];
    };
    // Every lane issues the same loads for every bucket (lanes past a range
    // read record 0 and ignore it): a fixed number of loads per bucket lets
    // the wait for the current bucket leave the next bucket's loads pending.
    auto fetch = [&](uint32_t bb, Slot &f) {
        f.l0 = offL[bb];
        f.nl = offL[bb + 1] - f.l0;
        f.r0 = offR[bb];
        f.nr = offR[bb + 1] - f.r0;
#pragma unroll
        for (int u = 0; u < kLU; ++u) {
            const uint32_t i = t + 256 * u;
            const uint32_t li = i < f.nl ? f.l0 + i : 0u;
            f.lh[u] = L[li].hdr;
#pragma unroll
            for (int w = 0; w < WV; ++w) f.lv[u][w] = L[li].vec[w];
        }
#pragma unroll
        for (int e = 0; e < kPre; ++e) {
            const uint32_t j = t + 256 * e;
            const uint32_t rj = j < f.nr ? f.r0 + j : 0u;
            f.rh[e] = R[rj].hdr;
#pragma unroll
            for (int w = 0; w < WV; ++w) f.rv[e][w] = R[rj].vec[w];
        }
    };
    uint64_t hits = 0;
    // Work-groups stride over the buckets; the next bucket's records are
    // loaded while the current one is joined, so their latency is hidden.
    Slot cur, nxt;
    uint32_t b = blockIdx.x;
    fetch(min(b, nb - 1), cur);
    while (b < nb) {
        const uint32_t bn = b + gridDim.x;
        fetch(min(bn, nb - 1), nxt);                    // past the end: a repeat, unused
        const uint32_t l0 = cur.l0, nl = cur.nl, r0 = cur.r0, nr = cur.nr;
        __syncthreads();                                // the previous bucket is done with LDS
        const bool run = nl != 0 && nr != 0 && nl <= (uint32_t)kJoinCap;   // uniform
        if (nl > (uint32_t)kJoinCap && nr != 0 && t == 0)           // too big for LDS
            heavy[atomicAdd((unsigned long long *)&scal[S_NHEAVY], 1ull)] = b;
        if (run) {
            uint32_t slots = 256;
            while (3 * slots < 4 * nl) slots <<= 1;
            const uint32_t smask = slots - 1;
            for (uint32_t i = t; i < slots; i += 256) s_head[i] = kEmpty;
            if (t == 0) s_gmax = 0;
#pragma unroll
            for (int u = 0; u < kLU; ++u) {
                const uint32_t i = t + 256 * u;
                if (i < nl) {
                    s_key[i] = (KT)hkey(p, cur.lh[u], kword<W>(cur.lv[u]));
#pragma unroll
                    for (int w = 0; w < WV; ++w) s_vec[w][i] = cur.lv[u][w];
                }
            }
            __syncthreads();
            for (uint32_t i = t; i < nl; i += 256) {
                const uint32_t h = key_hash((int64_t)s_key[i]) & smask;
                uint32_t old = s_head[h];
                for (;;) {
                    const uint32_t got =
                        atomicCAS(&s_head[h], old, (i << 16) | ((old & 0xFFFFu) + 1));
                    if (got == old) break;
                    old = got;
                }
                s_next[i] = (uint16_t)(old >> 16);
                const uint32_t len = (old & 0xFFFFu) + 1;
                if (len > (uint32_t)kLightGroup) atomicMax(&s_gmax, len);   // rare
            }
            __syncthreads();
            if (s_gmax > (uint32_t)kLightGroup) {       // a large group: heavy kernel
                if (t == 0) heavy[atomicAdd((unsigned long long *)&scal[S_NHEAVY], 1ull)] = b;
            } else {
                auto hit = [&](uint32_t i, const uint32_t *v, uint32_t rj) {
                    ++hits;
                    if (W == 0) {
                        atomicAdd((unsigned long long *)&scal[S_NSOL], 1ull);
                        if (scal[S_STORED] < cap)
                            emit_solution(sol, cap, &scal[S_STORED],
                                          half_mask(p, qs, 0, L[l0 + i].hdr),
                                          half_mask(p, qs, 1, R[r0 + rj].hdr));
                    } else {
                        bool ok = true;
#pragma unroll
                        for (int w = 0; w < WV; ++w) ok = ok && (s_vec[w][i] == v[w]);
                        if (ok)
                            emit_pair(p, qs, sol, cap, &scal[S_NSOL], L[l0 + i].hdr, R[r0 + rj].hdr);
                    }
                };
                auto probe = [&](const int64_t key, const uint32_t *v, uint32_t rj) {
                    for (uint32_t i = s_head[key_hash(key) & smask] >> 16; i != kEnd; i = s_next[i])
                        if (s_key[i] == (KT)key) hit(i, v, rj);
                };
#pragma unroll
                for (int e = 0; e < kPre; ++e) {
                    const uint32_t j = t + 256 * e;
                    if (j < nr) probe((int64_t)hkey(p, cur.rh[e], kword<W>(cur.rv[e])), cur.rv[e], j);
                }
                for (uint32_t j = t + 256 * kPre; j < nr; j += 256) {
                    uint32_t v[WV];
#pragma unroll
                    for (int w = 0; w < WV; ++w) v[w] = R[r0 + j].vec[w];
                    probe(rkey(p, R[r0 + j]), v, j);
                }
            }
        }
        cur = nxt;
        b = bn;
    }
    const uint64_t tot = block_sum_u64(hits, s_s4);
    if (t == 0) add_u128(&scal[S_H_LO], &scal[S_H_HI], tot);
}

// Join of buckets that hold a few dozen records per side (a large modulus,
// as many key rows force): one wavefront per bucket and no LDS.  The lanes
// hold 64 left keys at a time; right records follow 64 at a time, one per
// lane, and each left key is broadcast to the wavefront in turn.  A key match
// is a 1-D hit, whose rows are then read and compared.  Buckets with more
// than kPairsCap left records are handed to k_join_heavy.
constexpr uint32_t kPairsCap = 256;

template <typename KT>
__device__ __forceinline__ KT wave_bcast(KT v, uint32_t lane) {
    if constexpr (sizeof(KT) == 4) {
        return (KT)__builtin_amdgcn_readlane((int)v, (int)lane);
    } else {
        const uint64_t u = (uint64_t)v;
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, (int)lane);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), (int)lane);
        return (KT)(((uint64_t)hi << 32) | lo);
    }
}

template <int W, bool K32>
__global__ __launch_bounds__(256) void k_join_pairs(Plan p, const uint32_t *__restrict__ offL,
                                                   const uint32_t *__restrict__ offR,
                                                   const Rec<W> *__restrict__ L,
                                                   const Rec<W> *__restrict__ R, uint32_t *heavy,
                                                   uint64_t *scal, uint64_t *sol, uint64_t cap,
                                                   QPtrs<W> qs, uint32_t nb) {
    constexpr int WV = W > 0 ? W : 1;
    using KT = typename std::conditional<K32, uint32_t, int64_t>::type;
    __shared__ uint64_t s_s4[4];
    const uint32_t lane = threadIdx.x & 63u;
    uint64_t hits = 0;
    // Bucket ranges are read by the whole wavefront, so every branch below
    // is uniform per wavefront.
    for (uint32_t b = blockIdx.x * 4u + (threadIdx.x >> 6); b < nb; b += gridDim.x * 4u) {
        const uint32_t l0 = offL[b], nl = offL[b + 1] - l0;
        const uint32_t r0 = offR[b], nr = offR[b + 1] - r0;
        if (nl == 0 || nr == 0) continue;
        if (nl > kPairsCap) {
            if (lane == 0) heavy[atomicAdd((unsigned long long *)&scal[S_NHEAVY], 1ull)] = b;
            continue;
        }
        for (uint32_t i0 = 0; i0 < nl; i0 += 64) {
            const uint32_t ni = min(64u, nl - i0);
            const KT lk = (KT)rkey(p, L[l0 + i0 + min(lane, ni - 1)]);
            for (uint32_t j0 = 0; j0 < nr; j0 += 64) {
                const bool rin = j0 + lane < nr;
                const uint32_t rj = r0 + j0 + min(lane, nr - j0 - 1);
                const uint64_t rh = R[rj].hdr;
                const KT rk = (KT)rkey(p, R[rj]);
                for (uint32_t i = 0; i < ni; ++i) {
                    const KT k = wave_bcast(lk, i);
                    if (rin && k == rk) {
                        ++hits;
                        const uint32_t li = l0 + i0 + i;
                        if (W == 0) {
                            atomicAdd((unsigned long long *)&scal[S_NSOL], 1ull);
                            if (scal[S_STORED] < cap)
                                emit_solution(sol, cap, &scal[S_STORED],
                                              half_mask(p, qs, 0, L[li].hdr),
                                              half_mask(p, qs, 1, rh));
                        } else {
                            bool ok = true;
#pragma unroll
                            for (int w = 0; w < WV; ++w) ok = ok && (L[li].vec[w] == R[rj].vec[w]);
                            if (ok)
                                emit_pair(p, qs, sol, cap, &scal[S_NSOL], L[li].hdr, rh);
                        }
                    }
                }
            }
        }
    }
    const uint64_t tot = block_sum_u64(hits, s_s4);
    if (threadIdx.x == 0) add_u128(&scal[S_H_LO], &scal[S_H_HI], tot);
}

// Hash of a (key, packed rows) pair for the vector join table.
// Table hashes of the grouped join, in 32-bit arithmetic when the key part
// fits 32 bits (fewer instructions than the 64-bit mixes).
__device__ __forceinline__ uint32_t khash(uint32_t k) {
    const uint32_t h = k * 0x9E3779B1u;
    return h ^ (h >> 16);
}
__device__ __forceinline__ uint32_t khash(int64_t k) { return key_hash(k); }

template <int W>
__device__ __forceinline__ uint32_t kv_hash(int64_t key, const uint32_t *v);

template <int W, typename KT>
__device__ __forceinline__ uint32_t kvhash(KT key, const uint32_t *v) {
    if constexpr (sizeof(KT) == 4 && W <= 1) {
        uint32_t h = key * 0x9E3779B1u ^ v[0] * 0x85EBCA77u;
        h ^= h >> 15;
        h *= 0xC2B2AE3Du;
        return h ^ (h >> 13);
    } else {
        return kv_hash<W>((int64_t)key, v);
    }
}

template <int W>
__device__ __forceinline__ uint32_t kv_hash(int64_t key, const uint32_t *v) {
    uint64_t h = (uint64_t)key * 0x9E3779B97F4A7C15ull;
#pragma unroll
    for (int w = 0; w < (W > 0 ? W : 1); ++w) h = (h ^ v[w]) * 0xC2B2AE3D27D4EB4Full;
    return (uint32_t)(h >> 32);
}

// Light join variant for buckets whose equal-key groups hold a few to a
// few hundred records: linear-probe table with one representative per
// distinct key, counts scanned into contiguous groups, and the left rows laid
// out in group order.  Each right record then walks its group with eight
// independent LDS loads of first words in flight per step; the other words
// are read only where the first matches.  NTJ threads per work-group and
// CAP left records at most (SLOTS table entries): 256 / 1344 for buckets of
// about a thousand records, 1024 / 4096 for buckets of a few thousand.
template <int W, bool K32, bool VJ, int NTJ, uint32_t CAP, uint32_t SLOTS>
__device__ __forceinline__ void grouped_bucket(const Plan &p, const uint32_t *__restrict__ offL,
                                               const uint32_t *__restrict__ offR,
                                               const Rec<W> *__restrict__ L,
                                               const Rec<W> *__restrict__ R, uint32_t *heavy,
                                               int hslot, uint64_t *scal, uint64_t *sol,
                                               uint64_t cap, const QPtrs<W> &qs,
                                               const uint32_t b) {
    // s_tab[h] = (representative left index << 16) | count, then | group end.
    constexpr uint32_t kEmpty = 0xFFFF0000u;
    constexpr int WV = W > 0 ? W : 1;
    constexpr uint32_t kNone = 0xFFFFu;
    // Capacity and table sized for four work-groups per CU: keys held in 32
    // bits when key >> log2M fits (K32), table at most two-thirds full.
    using KT = typename std::conditional<K32, uint32_t, int64_t>::type;
    constexpr uint32_t kCap = CAP;
    constexpr int NW = NTJ / 64;
    static_assert(SLOTS * 2 >= CAP * 3 && SLOTS / NTJ <= 16 && SLOTS >= NTJ, "table size");
    __shared__ KT s_key[kCap];
    __shared__ uint32_t s_vec[WV][kCap + 8];             // left rows: by left index, then by group
    __shared__ uint32_t s_tab[SLOTS];
    __shared__ uint16_t s_slot[kCap];
    __shared__ uint16_t s_grp[VJ ? 1 : kCap];            // group order -> left index
    __shared__ uint32_t s_vt[VJ ? SLOTS : 1];            // VJ: (key, rows) -> left index
    __shared__ uint32_t s_w4[NW];
    __shared__ uint64_t s_s4[NW];
    __shared__ uint32_t s_gmax;
    const uint32_t l0 = offL[b], l1 = offL[b + 1];
    const uint32_t r0 = offR[b], r1 = offR[b + 1];
    const uint32_t nl = l1 - l0, nr = r1 - r0;
    if (nl == 0 || nr == 0) return;                     // uniform across the block
    if (nl > kCap) {                                    // too big for LDS: heavy kernel
        if (threadIdx.x == 0)
            heavy[atomicAdd((unsigned long long *)&scal[hslot], 1ull)] = b;
        return;
    }
    const int t = threadIdx.x;
    // Right records are loaded first and consumed after the build.  Every
    // lane issues the same loads (lanes past a range read record 0 and
    // ignore it) and headers stay raw until used, so no load waits inside
    // its guard and all of them are in flight together.
    constexpr int kPre = 4;                              // right records preloaded per lane
    uint64_t rh[kPre];
    uint32_t rv[kPre][WV];
#pragma unroll
    for (int e = 0; e < kPre; ++e) {
        const uint32_t j = t + NTJ * e;
        const uint32_t rj = j < nr ? r0 + j : 0u;
        rh[e] = R[rj].hdr;
#pragma unroll
        for (int w = 0; w < WV; ++w) rv[e][w] = R[rj].vec[w];
    }
    uint32_t slots = NTJ;
    while (2 * slots < 3 * nl) slots <<= 1;             // <= SLOTS for nl <= kCap
    const uint32_t smask = slots - 1;
    for (uint32_t i = t; i < slots; i += NTJ) {
        s_tab[i] = kEmpty;
        if (VJ) s_vt[i] = 0xFFFFFFFFu;
    }
    if (t == 0) s_gmax = 0;
    {   // all left loads of this lane issued together, then staged into LDS
        constexpr int kLU = (kCap + NTJ - 1) / NTJ;
        uint64_t lh[kLU];
        uint32_t lv[kLU][WV];
#pragma unroll
        for (int u = 0; u < kLU; ++u) {
            const uint32_t i = t + NTJ * u;
            const uint32_t li = i < nl ? l0 + i : 0u;
            lh[u] = L[li].hdr;
#pragma unroll
            for (int w = 0; w < WV; ++w) lv[u][w] = L[li].vec[w];
        }
#pragma unroll
        for (int u = 0; u < kLU; ++u) {
            const uint32_t i = t + NTJ * u;
            if (i < nl) {
                s_key[i] = (KT)hkey(p, lh[u], kword<W>(lv[u]));
#pragma unroll
                for (int w = 0; w < WV; ++w) s_vec[w][i] = lv[u][w];
            }
        }
    }
    __syncthreads();
    // Build: one representative per distinct key, count per slot.
    for (uint32_t i = t; i < nl; i += NTJ) {
        const KT k = s_key[i];
        uint32_t h = khash(k) & smask;
        for (;;) {
            uint32_t w = s_tab[h];
            if (w == kEmpty) {
                const uint32_t old = atomicCAS(&s_tab[h], kEmpty, i << 16);
                if (old == kEmpty) break;
                w = old;
            }
            if (s_key[w >> 16] == k) break;
            h = (h + 1) & smask;
        }
        s_slot[i] = (uint16_t)h;
        atomicAdd(&s_tab[h], 1u);
        if (VJ) {
            uint32_t lvv[WV];
#pragma unroll
            for (int w = 0; w < WV; ++w) lvv[w] = s_vec[w][i];
            // At most two-thirds full: an empty slot is always reached.
            uint32_t g = kvhash<W>(k, lvv) & smask;
            while (atomicCAS(&s_vt[g], 0xFFFFFFFFu, i) != 0xFFFFFFFFu) g = (g + 1) & smask;
        }
    }
    __syncthreads();
    if (VJ) {
        uint64_t hits = 0;
        auto probe_vj = [&](const int64_t key, const uint32_t *v, uint32_t rj) {
            uint32_t h = khash((KT)key) & smask;
            for (;;) {
                const uint32_t w = s_tab[h];
                if (w == kEmpty) return;                 // no left record has this key
                if (s_key[w >> 16] == (KT)key) break;
                h = (h + 1) & smask;
            }
            hits += s_tab[h] & 0xFFFFu;                  // |G_L| pairs for this right record
            for (uint32_t g = kvhash<W>((KT)key, v) & smask;; g = (g + 1) & smask) {
                const uint32_t li = s_vt[g];
                if (li == 0xFFFFFFFFu) break;
                if (s_key[li] != (KT)key) continue;
                bool ok = true;
#pragma unroll
                for (int w = 0; w < WV; ++w) ok = ok && (s_vec[w][li] == v[w]);
                if (ok)
                    emit_pair(p, qs, sol, cap, &scal[S_NSOL], L[l0 + li].hdr, R[r0 + rj].hdr);
            }
        };
#pragma unroll
        for (int q = 0; q < kPre; ++q) {
            const uint32_t j = t + NTJ * q;
            if (j < nr) probe_vj((int64_t)hkey(p, rh[q], kword<W>(rv[q])), rv[q], j);
        }
        for (uint32_t j = t + NTJ * kPre; j < nr; j += NTJ) {
            uint32_t v[WV];
#pragma unroll
            for (int w = 0; w < WV; ++w) v[w] = R[r0 + j].vec[w];
            probe_vj(rkey(p, R[r0 + j]), v, j);
        }
        const uint64_t tot = block_sum_u64<NTJ>(hits, s_s4);
        if (t == 0) add_u128(&scal[S_H_LO], &scal[S_H_HI], tot);
        return;
    }
    {   // exclusive scan of the counts (low halves), heads kept
        const int E = (int)(slots / NTJ), lane = t & 63, wave = t >> 6;
        uint32_t loc[16], sum = 0, gm = 0;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            loc[e] = e < E ? (s_tab[t * E + e] & 0xFFFFu) : 0u;
            sum += loc[e];
            gm = max(gm, loc[e]);
        }
        atomicMax(&s_gmax, gm);
        const uint32_t inc = wave_incl_scan(sum);
        if (lane == 63) s_w4[wave] = inc;
        __syncthreads();
        uint32_t run = inc - sum;
        for (int w = 0; w < wave; ++w) run += s_w4[w];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            if (e < E) {
                s_tab[t * E + e] = (s_tab[t * E + e] & 0xFFFF0000u) | run;
                run += loc[e];
            }
        }
        __syncthreads();
    }
    // A left group larger than kLightGroup makes per-lane loops slow: the
    // whole bucket goes to the heavy kernel (tiled verify of big groups).
    if (s_gmax > (uint32_t)kLightGroup) {
        if (t == 0) heavy[atomicAdd((unsigned long long *)&scal[hslot], 1ull)] = b;
        return;
    }
    // Group left records by slot; afterwards the low half is the group end.
    for (uint32_t i = t; i < nl; i += NTJ) {
        const uint32_t pos = atomicAdd(&s_tab[s_slot[i]], 1u) & 0xFFFFu;
        s_grp[pos] = (uint16_t)i;
    }
    __syncthreads();
    {   // left rows into group order
        constexpr int kLU = (kCap + NTJ - 1) / NTJ;
        uint32_t tmp[kLU][WV];
#pragma unroll
        for (int u = 0; u < kLU; ++u) {
            const uint32_t q = t + NTJ * u;
            if (q < nl) {
                const uint32_t li = s_grp[q];
#pragma unroll
                for (int w = 0; w < WV; ++w) tmp[u][w] = s_vec[w][li];
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kLU; ++u) {
            const uint32_t q = t + NTJ * u;
            if (q < nl) {
#pragma unroll
                for (int w = 0; w < WV; ++w) s_vec[w][q] = tmp[u][w];
            }
        }
    }
    uint64_t hits = 0;
    __syncthreads();                                    // left rows reordered
    auto probe = [&](const int64_t key, const uint32_t *v, uint32_t rj) {
        // After the scan an empty slot keeps head 0xFFFF but its low half
        // holds a running offset, so emptiness is read from the head half.
        uint32_t h = khash((KT)key) & smask;
        uint32_t gs = kNone, ge = 0;
        for (;;) {
            const uint32_t w = s_tab[h];
            if ((w >> 16) == 0xFFFFu) break;
            if (s_key[w >> 16] == (KT)key) {
                ge = w & 0xFFFFu;
                gs = h ? (s_tab[h - 1] & 0xFFFFu) : 0u;
                break;
            }
            h = (h + 1) & smask;
        }
        if (gs == kNone) return;
        hits += ge - gs;
        if (W == 0) {
            atomicAdd((unsigned long long *)&scal[S_NSOL], (unsigned long long)(ge - gs));
            for (uint32_t q = gs; q < ge; ++q) {
                if (scal[S_STORED] >= cap) break;
                emit_solution(sol, cap, &scal[S_STORED], half_mask(p, qs, 0, L[l0 + s_grp[q]].hdr),
                              half_mask(p, qs, 1, R[r0 + rj].hdr));
            }
            return;
        }
        // Eight first words in flight per step; the rest of a word vector is
        // read only where the first word matches.  A first word equal to v[0]
        // is rare (the fingerprint of a probable solution), so each step
        // tests the eight differences for a zero by their minimum and builds
        // the match mask, bounded by the group end, only when one is zero;
        // the words past the group end (a next group, or the padding) can
        // only send a step to that slower test.
        for (uint32_t q0 = gs; q0 < ge; q0 += 8) {
            const uint32_t *sv = &s_vec[0][q0];                   // padded past nl
            uint32_t x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) x[u] = sv[u] ^ v[0];
            const uint32_t mn = min(min(min(x[0], x[1]), min(x[2], x[3])),
                                    min(min(x[4], x[5]), min(x[6], x[7])));
            if (mn != 0u) continue;
            uint32_t m = 0;
#pragma unroll
            for (int u = 0; u < 8; ++u) m |= (uint32_t)(x[u] == 0u && q0 + u < ge) << u;
            while (m) {
                const uint32_t q = q0 + __builtin_ctz(m);
                m &= m - 1;
                bool ok = true;
#pragma unroll
                for (int w = 1; w < WV; ++w) ok = ok && (s_vec[w][q] == v[w]);
                if (ok)
                    emit_pair(p, qs, sol, cap, &scal[S_NSOL], L[l0 + s_grp[q]].hdr, R[r0 + rj].hdr);
            }
        }
    };
#pragma unroll
    for (int e = 0; e < kPre; ++e) {
        const uint32_t j = t + NTJ * e;
        if (j < nr) probe((int64_t)hkey(p, rh[e], kword<W>(rv[e])), rv[e], j);
    }
    for (uint32_t j = t + NTJ * kPre; j < nr; j += NTJ) {
        uint32_t v[WV];
#pragma unroll
        for (int w = 0; w < WV; ++w) v[w] = R[r0 + j].vec[w];
        probe(rkey(p, R[r0 + j]), v, j);
    }
    const uint64_t tot = block_sum_u64<NTJ>(hits, s_s4);
    if (t == 0) add_u128(&scal[S_H_LO], &scal[S_H_HI], tot);
}

// One work-group per bucket of the window.
template <int W, bool K32, bool VJ, int NTJ = 256, uint32_t CAP = kGroupCap,
          uint32_t SLOTS = kGroupSlots>
__global__ __launch_bounds__(NTJ) void k_join_grouped(Plan p, const uint32_t *__restrict__ offL,
                                                   const uint32_t *__restrict__ offR,
                                                   const Rec<W> *__restrict__ L,
                                                   const Rec<W> *__restrict__ R, uint32_t *heavy,
                                                   uint64_t *scal, uint64_t *sol, uint64_t cap,
                                                   QPtrs<W> qs) {
    grouped_bucket<W, K32, VJ, NTJ, CAP, SLOTS>(p, offL, offR, L, R, heavy, S_NHEAVY, scal, sol,
                                                cap, qs, blockIdx.x);
}

// Second pass over the buckets the first deferred (list[0 .. scal[S_NHEAVY])):
// 1024-thread groups for buckets of up to kGroupCapBig left records, which a
// few dense keys make common when equal-key groups hold hundreds of records;
// larger ones go on to the heavy kernels (heavy2, S_NHEAVY2).
template <int W, bool K32, bool VJ>
__global__ __launch_bounds__(1024) void k_join_grouped_list(Plan p,
                                                         const uint32_t *__restrict__ offL,
                                                         const uint32_t *__restrict__ offR,
                                                         const Rec<W> *__restrict__ L,
                                                         const Rec<W> *__restrict__ R,
                                                         const uint32_t *__restrict__ list,
                                                         uint32_t *heavy2, uint64_t *scal,
                                                         uint64_t *sol, uint64_t cap,
                                                         QPtrs<W> qs) {
    const uint64_t n = scal[S_NHEAVY];
    for (uint64_t i = blockIdx.x; i < n; i += gridDim.x) {
        __syncthreads();                                 // the previous bucket is done with LDS
        grouped_bucket<W, K32, VJ, 1024, kGroupCapBig, kGroupSlotsBig>(
            p, offL, offR, L, R, heavy2, S_NHEAVY2, scal, sol, cap, qs, list[i]);
    }
}

// Vector join of the buckets too large for k_join_grouped's LDS: left
// chunks of kGroupCap records, each against the whole right side of the
// bucket, with the same two LDS tables (key -> count for H, (key, rows) ->
// left index for the solutions).  Every (left, right) pair of the bucket is
// met once; nothing is compared pair by pair.
template <int W, bool K32>
__global__ __launch_bounds__(256) void k_join_heavy_vj(Plan p, const uint32_t *__restrict__ offL,
                                                      const uint32_t *__restrict__ offR,
                                                      const Rec<W> *__restrict__ L,
                                                      const Rec<W> *__restrict__ R,
                                                      const uint32_t *__restrict__ heavy,
                                                      uint64_t *scal, uint64_t *sol, uint64_t cap,
                                                      QPtrs<W> qs, int hslot) {
    constexpr uint32_t kEmpty = 0xFFFF0000u;
    constexpr int WV = W > 0 ? W : 1;
    using KT = typename std::conditional<K32, uint32_t, int64_t>::type;
    constexpr uint32_t kCap = kGroupCap;
    constexpr int kLU = (kCap + 255) / 256;
    __shared__ KT s_key[kCap];
    __shared__ uint32_t s_vec[WV][kCap];
    __shared__ uint32_t s_tab[kGroupSlots];              // (representative << 16) | count
    __shared__ uint32_t s_vt[kGroupSlots];               // (key, rows) -> left index
    __shared__ uint64_t s_s4[4];
    const int t = threadIdx.x;
    const uint32_t nheavy = (uint32_t)scal[hslot];
    uint64_t hits = 0;
    for (uint32_t hb = blockIdx.x; hb < nheavy; hb += gridDim.x) {
        const uint32_t b = heavy[hb];
        const uint32_t L0 = offL[b], L1 = offL[b + 1];
        const uint32_t r0 = offR[b], nr = offR[b + 1] - r0;
        for (uint32_t l0 = L0; l0 < L1; l0 += kCap) {
            const uint32_t nl = min(kCap, L1 - l0);
            __syncthreads();                            // previous chunk done with LDS
            uint32_t slots = 256;
            while (2 * slots < 3 * nl) slots <<= 1;     // <= kGroupSlots
            const uint32_t smask = slots - 1;
            for (uint32_t i = t; i < slots; i += 256) {
                s_tab[i] = kEmpty;
                s_vt[i] = 0xFFFFFFFFu;
            }
            uint64_t lh[kLU];
            uint32_t lv[kLU][WV];
#pragma unroll
            for (int u = 0; u < kLU; ++u) {
                const uint32_t i = t + 256 * u;
                const uint32_t li = i < nl ? l0 + i : 0u;
                lh[u] = L[li].hdr;
#pragma unroll
                for (int w = 0; w < WV; ++w) lv[u][w] = L[li].vec[w];
            }
#pragma unroll
            for (int u = 0; u < kLU; ++u) {
                const uint32_t i = t + 256 * u;
                if (i < nl) {
                    s_key[i] = (KT)hkey(p, lh[u], kword<W>(lv[u]));
#pragma unroll
                    for (int w = 0; w < WV; ++w) s_vec[w][i] = lv[u][w];
                }
            }
            __syncthreads();
            for (uint32_t i = t; i < nl; i += 256) {
                const KT k = s_key[i];
                uint32_t h = key_hash((int64_t)k) & smask;
                for (;;) {
                    uint32_t w = s_tab[h];
                    if (w == kEmpty) {
                        const uint32_t old = atomicCAS(&s_tab[h], kEmpty, i << 16);
                        if (old == kEmpty) break;
                        w = old;
                    }
                    if (s_key[w >> 16] == k) break;
                    h = (h + 1) & smask;
                }
                atomicAdd(&s_tab[h], 1u);
                uint32_t lvv[WV];
#pragma unroll
                for (int w = 0; w < WV; ++w) lvv[w] = s_vec[w][i];
                uint32_t g = kv_hash<W>((int64_t)k, lvv) & smask;
                while (atomicCAS(&s_vt[g], 0xFFFFFFFFu, i) != 0xFFFFFFFFu) g = (g + 1) & smask;
            }
            __syncthreads();
            // Right records four per lane at a time (clamped into the bucket),
            // all loads in flight together.
            constexpr int kRU = 4;
            for (uint32_t j0 = t; j0 < nr; j0 += 256 * kRU) {
            uint64_t rhs[kRU];
            uint32_t rvs[kRU][WV];
#pragma unroll
            for (int u = 0; u < kRU; ++u) {
                const uint32_t rj = r0 + min(j0 + 256u * u, nr - 1);
                rhs[u] = R[rj].hdr;
#pragma unroll
                for (int w = 0; w < WV; ++w) rvs[u][w] = R[rj].vec[w];
            }
            for (int u = 0; u < kRU; ++u) {
                if (j0 + 256u * u >= nr) break;
                const uint64_t rhdr = rhs[u];
                const uint32_t *v = rvs[u];
                const int64_t key = (int64_t)hkey(p, rhdr, kword<W>(v));
                uint32_t h = key_hash(key) & smask;
                bool found = false;
                for (;;) {
                    const uint32_t w = s_tab[h];
                    if (w == kEmpty) break;
                    if (s_key[w >> 16] == (KT)key) { found = true; break; }
                    h = (h + 1) & smask;
                }
                if (!found) continue;
                hits += s_tab[h] & 0xFFFFu;
                for (uint32_t g = kv_hash<W>(key, v) & smask;; g = (g + 1) & smask) {
                    const uint32_t li = s_vt[g];
                    if (li == 0xFFFFFFFFu) break;
                    if (s_key[li] != (KT)key) continue;
                    bool ok = true;
#pragma unroll
                    for (int w = 0; w < WV; ++w) ok = ok && (s_vec[w][li] == v[w]);
                    if (ok)
                        emit_pair(p, qs, sol, cap, &scal[S_NSOL], L[l0 + li].hdr, rhdr);
                }
            }
            }   // right steps
        }
    }
    const uint64_t tot = block_sum_u64(hits, s_s4);
    if (t == 0) add_u128(&scal[S_H_LO], &scal[S_H_HI], tot);
}

// Vector join of the buckets over the grouped kernels' LDS capacity (few
// keys with thousands of records each, as at (11,100)): 1024 threads, left
// chunks of kHeavyCap records (not kGroupCap), so the whole right side is
// read once per 5461 left records.  Two LDS tables hold no left records: a
// key table (key -> left count) gives every right record its |G_L| for H,
// and a set of 32-bit tags of (key, words) flags the right records that may
// match a left record exactly; only those scan the chunk's left records (in
// global memory) for the equal ones.  Keys are stored as themselves, so the
// all-ones word marks an empty slot: K32 needs key >> log2M < 2^31, the
// 64-bit form < 2^63.
constexpr uint32_t kHeavySlots = 8192;
constexpr uint32_t kHeavyCap = kHeavySlots * 2 / 3;   // 5461

template <int W>
__device__ __forceinline__ uint32_t rec_tag(uint64_t key, const uint32_t *v) {
    uint64_t h = key * 0x9E3779B97F4A7C15ull;
#pragma unroll
    for (int w = 0; w < (W > 0 ? W : 1); ++w) h = (h ^ v[w]) * 0xC2B2AE3D27D4EB4Full;
    return (uint32_t)(h >> 32) | 1u;                  // 0 marks an empty slot
}

template <int W, bool K32>
__global__ __launch_bounds__(1024) void k_join_heavy_vj2(Plan p,
                                                        const uint32_t *__restrict__ offL,
                                                        const uint32_t *__restrict__ offR,
                                                        const Rec<W> *__restrict__ L,
                                                        const Rec<W> *__restrict__ R,
                                                        const uint32_t *__restrict__ heavy,
                                                        uint64_t *scal, uint64_t *sol,
                                                        uint64_t cap, QPtrs<W> qs, int hslot) {
    using KT = typename std::conditional<K32, uint32_t, unsigned long long>::type;
    constexpr KT kEmptyKey = (KT)~(KT)0;
    constexpr uint32_t kMask = kHeavySlots - 1;
    constexpr int WV = W > 0 ? W : 1;
    __shared__ KT s_kk[kHeavySlots];
    __shared__ uint32_t s_kc[kHeavySlots];
    __shared__ uint32_t s_tag[kHeavySlots];
    __shared__ uint64_t s_s[16];
    const int t = threadIdx.x;
    const uint32_t nheavy = (uint32_t)scal[hslot];
    uint64_t hits = 0;
    for (uint32_t hb = blockIdx.x; hb < nheavy; hb += gridDim.x) {
        const uint32_t b = heavy[hb];
        const uint32_t L0 = offL[b], L1 = offL[b + 1];
        const uint32_t r0 = offR[b], nr = offR[b + 1] - r0;
        for (uint32_t c0 = L0; c0 < L1; c0 += kHeavyCap) {
            const uint32_t c1 = min(L1, c0 + kHeavyCap);
            __syncthreads();                             // previous chunk done with LDS
            for (uint32_t i = t; i < kHeavySlots; i += 1024) {
                s_kk[i] = kEmptyKey;
                s_kc[i] = 0;
                s_tag[i] = 0;
            }
            __syncthreads();
            for (uint32_t i = c0 + t; i < c1; i += 1024) {
                const Rec<W> r = L[i];
                const uint64_t k64 = hkey(p, r.hdr, kword<W>(r.vec));
                const KT k = (KT)k64;
                uint32_t h = khash((uint32_t)k64 ^ (uint32_t)(k64 >> 32)) & kMask;
                for (;;) {                               // at most two-thirds full
                    const KT cur = s_kk[h];
                    if (cur == k) break;
                    if (cur == kEmptyKey) {
                        const KT old = atomicCAS(&s_kk[h], kEmptyKey, k);
                        if (old == kEmptyKey || old == k) break;
                    }
                    h = (h + 1) & kMask;
                }
                atomicAdd(&s_kc[h], 1u);
                const uint32_t tag = rec_tag<W>(k64, r.vec);
                uint32_t g = tag & kMask;
                for (;;) {
                    const uint32_t cur = s_tag[g];
                    if (cur == tag) break;
                    if (cur == 0u) {
                        const uint32_t old = atomicCAS(&s_tag[g], 0u, tag);
                        if (old == 0u || old == tag) break;
                    }
                    g = (g + 1) & kMask;
                }
            }
            __syncthreads();
            for (uint32_t j = t; j < nr; j += 1024) {
                const Rec<W> rr = R[r0 + j];
                const uint64_t k64 = hkey(p, rr.hdr, kword<W>(rr.vec));
                const KT k = (KT)k64;
                uint32_t h = khash((uint32_t)k64 ^ (uint32_t)(k64 >> 32)) & kMask;
                uint32_t cnt = 0;
                for (;;) {
                    const KT cur = s_kk[h];
                    if (cur == k) { cnt = s_kc[h]; break; }
                    if (cur == kEmptyKey) break;
                    h = (h + 1) & kMask;
                }
                if (cnt == 0) continue;
                hits += cnt;
                const uint32_t tag = rec_tag<W>(k64, rr.vec);
                bool cand = false;
                for (uint32_t g = tag & kMask;; g = (g + 1) & kMask) {
                    const uint32_t cur = s_tag[g];
                    if (cur == tag) { cand = true; break; }
                    if (cur == 0u) break;
                }
                if (!cand) continue;
                // A possible exact match: the chunk's left records with the
                // same key and words (rare: solutions and fingerprint ties).
                for (uint32_t i = c0; i < c1; ++i) {
                    const Rec<W> l = L[i];
                    if (hkey(p, l.hdr, kword<W>(l.vec)) != k64) continue;
                    bool ok = true;
#pragma unroll
                    for (int w = 0; w < WV; ++w) ok = ok && (l.vec[w] == rr.vec[w]);
                    if (ok) emit_pair(p, qs, sol, cap, &scal[S_NSOL], l.hdr, rr.hdr);
                }
            }
        }
    }
    const uint64_t tot = block_sum_u64<1024>(hits, s_s);
    if (t == 0 && tot) add_u128(&scal[S_H_LO], &scal[S_H_HI], tot);
}

template <int W>
__global__ __launch_bounds__(256) void k_join_heavy(Plan p, const uint32_t *__restrict__ offL,
                                                   const uint32_t *__restrict__ offR,
                                                   const Rec<W> *__restrict__ L,
                                                   const Rec<W> *__restrict__ R,
                                                   const uint32_t *__restrict__ heavy,
                                                   RunPair *iruns, uint32_t *idx,
                                                   uint64_t *scal, uint64_t *sol, uint64_t cap,
                                                   uint64_t iruns_cap, uint64_t idx_cap,
                                                   QPtrs<W> qs, int hslot) {
    // s_tab[h] = (representative left index << 16) | count, then | group end.
    constexpr uint32_t kEmpty = 0xFFFF0000u;
    constexpr int WV = W > 0 ? W : 1;
    __shared__ int64_t s_key[kJoinCap];
    __shared__ uint32_t s_vec[WV][kJoinCap];             // left packed rows, by left index
    __shared__ uint32_t s_tab[kJoinSlots];
    __shared__ uint32_t s_rcnt[kJoinSlots];              // right records per slot
    __shared__ uint8_t s_bigidx[kJoinSlots];             // slot -> exported group, or 0xFF
    __shared__ uint16_t s_slot[kJoinCap];
    __shared__ uint16_t s_lpos[kJoinCap];                // position of a left record in s_grp
    __shared__ uint16_t s_grp[kJoinCap];
    __shared__ uint32_t s_bbase[kMaxBig], s_bgl[kMaxBig], s_bfill[kMaxBig];
    __shared__ uint32_t s_nbig;
    __shared__ uint32_t s_w4[4];
    __shared__ uint64_t s_s4[4];
    const int t = threadIdx.x;
    const uint32_t nheavy = (uint32_t)scal[hslot];
    uint64_t hits = 0;
    for (uint32_t hb = blockIdx.x; hb < nheavy; hb += gridDim.x) {
    const uint32_t b = heavy[hb];
    const uint32_t L0 = offL[b], L1 = offL[b + 1];
    const uint32_t R0 = offR[b], R1 = offR[b + 1];
    // Left chunks of at most kJoinCap records, each against the whole right
    // side: every (left, right) pair of the bucket is met exactly once.
    for (uint32_t lc0 = L0; lc0 < L1; lc0 += kJoinCap) {
    const uint32_t l0 = lc0, nl = min((uint32_t)kJoinCap, L1 - lc0);
    __syncthreads();                                    // previous chunk done with LDS
    uint32_t slots = 256;
    while (slots < 2 * nl) slots <<= 1;
    const uint32_t smask = slots - 1;
    for (uint32_t i = t; i < slots; i += 256) {
        s_tab[i] = kEmpty;
        s_rcnt[i] = 0;
        s_bigidx[i] = 0xFF;
    }
    {   // all left loads of this lane issued together, then staged into LDS
        constexpr int kLU = (kJoinCap + 255) / 256;
        // Fixed loads per lane (past the chunk: record l0, ignored), raw
        // headers: all in flight together.
        uint64_t lh[kLU];
        uint32_t lv[kLU][WV];
#pragma unroll
        for (int u = 0; u < kLU; ++u) {
            const uint32_t i = t + 256 * u;
            const uint32_t li = l0 + (i < nl ? i : 0u);
            lh[u] = L[li].hdr;
#pragma unroll
            for (int w = 0; w < WV; ++w) lv[u][w] = L[li].vec[w];
        }
#pragma unroll
        for (int u = 0; u < kLU; ++u) {
            const uint32_t i = t + 256 * u;
            if (i < nl) {
                s_key[i] = (int64_t)hkey(p, lh[u], kword<W>(lv[u]));
#pragma unroll
                for (int w = 0; w < WV; ++w) s_vec[w][i] = lv[u][w];
            }
        }
    }
    __syncthreads();
    // Build: one representative per distinct key, count per slot.
    for (uint32_t i = t; i < nl; i += 256) {
        const int64_t k = s_key[i];
        uint32_t h = key_hash(k) & smask;
        for (;;) {
            uint32_t w = s_tab[h];
            if (w == kEmpty) {
                const uint32_t old = atomicCAS(&s_tab[h], kEmpty, i << 16);
                if (old == kEmpty) break;
                w = old;
            }
            if (s_key[w >> 16] == k) break;
            h = (h + 1) & smask;
        }
        s_slot[i] = (uint16_t)h;
        atomicAdd(&s_tab[h], 1u);
    }
    __syncthreads();
    {   // exclusive scan of the counts (low halves), heads kept
        const int E = (int)(slots >> 8), lane = t & 63, wave = t >> 6;
        uint32_t loc[16], sum = 0;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            loc[e] = e < E ? (s_tab[t * E + e] & 0xFFFFu) : 0u;
            sum += loc[e];
        }
        const uint32_t inc = wave_incl_scan(sum);
        if (lane == 63) s_w4[wave] = inc;
        __syncthreads();
        uint32_t run = inc - sum;
        for (int w = 0; w < wave; ++w) run += s_w4[w];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            if (e < E) {
                s_tab[t * E + e] = (s_tab[t * E + e] & 0xFFFF0000u) | run;
                run += loc[e];
            }
        }
        __syncthreads();
    }
    // Group left records by slot; afterwards the low half is the group end.
    for (uint32_t i = t; i < nl; i += 256) {
        const uint32_t pos = atomicAdd(&s_tab[s_slot[i]], 1u) & 0xFFFFu;
        s_grp[pos] = (uint16_t)i;
        s_lpos[i] = (uint16_t)pos;
    }
    __syncthreads();
    // Slot of a key, or 0xFFFF.  After the scan an empty slot keeps head
    // 0xFFFF but its low half holds a running offset, so emptiness is read
    // from the head half.
    auto find = [&](const int64_t key) -> uint32_t {
        uint32_t h = key_hash(key) & smask;
        for (;;) {
            const uint32_t w = s_tab[h];
            if ((w >> 16) == 0xFFFFu) return 0xFFFFu;
            if (s_key[w >> 16] == key) return h;
            h = (h + 1) & smask;
        }
    };
    auto gstart = [&](uint32_t h) { return h ? (s_tab[h - 1] & 0xFFFFu) : 0u; };
    // All right records of the bucket against this left chunk.  Pass 1
    // counts 1-D hits and right records per slot; large groups are then
    // exported as index lists (when the lists have room, else verified here);
    // pass 2 probes again, writes right indices of exported groups and
    // verifies the small groups in place.
    const uint32_t r0 = R0, nr = R1 - R0;
    for (uint32_t i = t; i < slots; i += 256) {
        s_rcnt[i] = 0;
        s_bigidx[i] = 0xFF;
    }
    if (t == 0) s_nbig = 0;
    __syncthreads();
    // Right headers four per lane at a time (clamped into the bucket).
    constexpr int kRU = 4;
    for (uint32_t j0 = t; j0 < nr; j0 += 256 * kRU) {
        uint64_t rh[kRU];
        uint32_t rx[kRU];
#pragma unroll
        for (int u = 0; u < kRU; ++u) {
            const uint32_t rj = r0 + min(j0 + 256u * u, nr - 1);
            rh[u] = R[rj].hdr;
            rx[u] = kword<W>(R[rj].vec);
        }
#pragma unroll
        for (int u = 0; u < kRU; ++u) {
            if (j0 + 256u * u >= nr) break;
            const uint32_t h = find((int64_t)hkey(p, rh[u], rx[u]));
            if (h != 0xFFFFu) {
                const uint32_t g = (s_tab[h] & 0xFFFFu) - gstart(h);
                hits += g;
                atomicAdd(&s_rcnt[h], 1u);
                if (W == 0)
                    atomicAdd((unsigned long long *)&scal[S_NSOL], (unsigned long long)g);
            }
        }
    }
    __syncthreads();
    for (uint32_t h = t; h < slots; h += 256) {
        const uint32_t gr = s_rcnt[h];
        if (!gr) continue;
        const uint32_t gl = (s_tab[h] & 0xFFFFu) - gstart(h);
        if ((uint64_t)gl * gr < (uint64_t)kBigPairs) continue;
        const uint32_t bi = atomicAdd(&s_nbig, 1u);
        if (bi >= (uint32_t)kMaxBig) continue;
        const uint64_t ri = atomicAdd((unsigned long long *)&scal[S_NIRUNS], 1ull);
        if (ri >= iruns_cap) continue;                  // no room: verified in place
        const uint64_t base = atomicAdd((unsigned long long *)&scal[S_IDX],
                                        (unsigned long long)(gl + gr));
        if (base + gl + gr > idx_cap) {                 // no room: empty run, verified in place
            iruns[ri] = RunPair{0, 0, 0, 0};
            continue;
        }
        s_bbase[bi] = (uint32_t)base;
        s_bgl[bi] = gl;
        s_bfill[bi] = 0;
        s_bigidx[h] = (uint8_t)bi;
        iruns[ri] = RunPair{(uint32_t)base, gl, (uint32_t)base + gl, gr};
    }
    __syncthreads();
    for (uint32_t i = t; i < nl; i += 256) {
        const uint32_t h = s_slot[i], bi = s_bigidx[h];
        if (bi != 0xFFu) idx[s_bbase[bi] + (s_lpos[i] - gstart(h))] = l0 + i;
    }
    for (uint32_t j0 = t; j0 < nr; j0 += 256 * kRU) {
    uint64_t rh[kRU];
    uint32_t rx[kRU];
#pragma unroll
    for (int u = 0; u < kRU; ++u) {
        const uint32_t rj = r0 + min(j0 + 256u * u, nr - 1);
        rh[u] = R[rj].hdr;
        rx[u] = kword<W>(R[rj].vec);
    }
    for (int u = 0; u < kRU; ++u) {
        const uint32_t j = j0 + 256u * u;
        if (j >= nr) break;
        const uint32_t h = find((int64_t)hkey(p, rh[u], rx[u]));
        if (h == 0xFFFFu) continue;
        const uint32_t bi = s_bigidx[h];
        if (bi != 0xFFu) {
            const uint32_t rp = atomicAdd(&s_bfill[bi], 1u);
            idx[s_bbase[bi] + s_bgl[bi] + rp] = r0 + j;
            continue;
        }
        const uint32_t ge = s_tab[h] & 0xFFFFu, gs = gstart(h);
        if (W == 0) {
            for (uint32_t q = gs; q < ge; ++q) {
                if (scal[S_STORED] >= cap) break;
                emit_solution(sol, cap, &scal[S_STORED], half_mask(p, qs, 0, L[l0 + s_grp[q]].hdr),
                              half_mask(p, qs, 1, R[r0 + j].hdr));
            }
        } else {
            uint32_t v[WV];
#pragma unroll
            for (int w = 0; w < WV; ++w) v[w] = R[r0 + j].vec[w];
            for (uint32_t q = gs; q < ge; ++q) {
                const uint32_t li = s_grp[q];
                bool ok = true;
#pragma unroll
                for (int w = 0; w < WV; ++w) ok = ok && (s_vec[w][li] == v[w]);
                if (ok)
                    emit_pair(p, qs, sol, cap, &scal[S_NSOL], L[l0 + li].hdr, R[r0 + j].hdr);
            }
        }
    }
    }   // right steps
    }   // left chunks
    }   // heavy buckets
    const uint64_t tot = block_sum_u64(hits, s_s4);
    if (t == 0) add_u128(&scal[S_H_LO], &scal[S_H_HI], tot);
}

// ---------------------------------------------------------------------------
// Tiled verify of equal-key run pairs (exact buckets), or of oversized hash
// buckets with the key compared per pair (CK).  Tile = kTileL left x 256*kKR
// right records.  Each lane holds kKR right records as 32-bit fingerprints of
// their packed non-key rows; left fingerprints are staged in LDS and read
// as broadcasts, 4 at a time.  Equal vectors have equal fingerprints, so a
// wave-wide ballot OR over 4 x 8 compares flags every candidate group; the
// (rare) flagged groups are then checked in full, word by word.
// ---------------------------------------------------------------------------

constexpr int kChunk = 1024;          // left records per LDS stage

// Fingerprint of a packed row vector: the word itself for one word, else a
// multiplicative mix of all words.  Only equality of fingerprints is used,
// as a filter in front of the exact word-by-word compare.
template <int W>
__device__ __forceinline__ uint32_t fingerprint(const uint32_t *v) {
    if (W <= 1) return v[0];
    uint32_t h = v[0] * 0x9E3779B1u;
#pragma unroll
    for (int w = 1; w < W; ++w) {
        h ^= h >> 15;
        h = (h + v[w]) * 0x85EBCA77u;
    }
    h ^= h >> 13;
    return h;
}

// Lanes of this wave whose 8 right fingerprints hold any of the 4 left
// fingerprints q.x..q.w.  Each v_cmpx_ne clears the EXEC bit of a lane that
// saw equality, so the 32 compares need no scalar work; the flagged lanes
// are EXEC before XOR EXEC after, and EXEC is restored inside the block.
#define MSP_CMPX(r, l) "v_cmpx_ne_u32_e32 vcc, %" #r ", %" #l "\n\t"
#define MSP_CMPX8(l) MSP_CMPX(2, l) MSP_CMPX(3, l) MSP_CMPX(4, l) MSP_CMPX(5, l) \
                     MSP_CMPX(6, l) MSP_CMPX(7, l) MSP_CMPX(8, l) MSP_CMPX(9, l)
__device__ __forceinline__ uint64_t match4x8(const uint32_t *rf, uint4 q) {
    uint64_t save, flag;
    asm volatile(
        "s_mov_b64 %0, exec\n\t"
        MSP_CMPX8(10) MSP_CMPX8(11) MSP_CMPX8(12) MSP_CMPX8(13)
        "s_nop 4\n\t"
        "s_xor_b64 %1, exec, %0\n\t"
        "s_mov_b64 exec, %0\n\t"
        : "=&s"(save), "=&s"(flag)
        : "v"(rf[0]), "v"(rf[1]), "v"(rf[2]), "v"(rf[3]), "v"(rf[4]), "v"(rf[5]), "v"(rf[6]),
          "v"(rf[7]), "v"(q.x), "v"(q.y), "v"(q.z), "v"(q.w)
        : "vcc");
    return flag;
}
#undef MSP_CMPX8
#undef MSP_CMPX

template <int W, bool CK, int kKR, bool CMPX = false, bool IDX = false>
__global__ __launch_bounds__(256) void k_verify(Plan p, const Rec<W> *__restrict__ L,
                                                const Rec<W> *__restrict__ R,
                                                const RunPair *__restrict__ runs,
                                                const uint32_t *__restrict__ toff,
                                                uint32_t nruns, uint64_t *scal, uint64_t *sol,
                                                uint64_t cap, const uint32_t *__restrict__ idx,
                                                QPtrs<W> qs, uint32_t tile0) {
    // IDX: run ranges index `idx`, which holds the record positions.
    auto lrec = [&](uint32_t i) -> const Rec<W> & { return IDX ? L[idx[i]] : L[i]; };
    auto rrec = [&](uint32_t i) -> const Rec<W> & { return IDX ? R[idx[i]] : R[i]; };
    __shared__ __attribute__((aligned(16))) uint32_t s_fp[kChunk];
    __shared__ int64_t s_lk[CK ? kChunk : 1];
    __shared__ uint64_t s_s4[4];
    const uint32_t tile = tile0 + blockIdx.x;
    // Run pair of this tile: last ri with toff[ri] <= tile.
    uint32_t lo = 0, hi = nruns;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (toff[mid] <= tile) lo = mid; else hi = mid;
    }
    const RunPair rp = runs[lo];
    const uint32_t loc = tile - toff[lo];
    constexpr uint32_t kTR = 256u * kKR;       // right records per tile
    const uint32_t tr_n = (rp.nr + kTR - 1) / kTR;
    const uint32_t tl = loc / tr_n, tr = loc % tr_n;
    const uint32_t lb = rp.l0 + tl * kTileL;
    const uint32_t le = min(rp.l0 + rp.nl, lb + (uint32_t)kTileL);
    const uint32_t rb = rp.r0 + tr * kTR;
    const uint32_t re = min(rp.r0 + rp.nr, rb + kTR);
    const int t = threadIdx.x;

    if (W == 0 && !CK) {
        // Every pair is a solution: store while there is room.
        for (uint32_t li = lb; li < le; ++li) {
#pragma unroll
            for (int k = 0; k < kKR; ++k) {
                const uint32_t ri = rb + k * 256 + t;
                if (ri < re && scal[S_STORED] < cap)
                    emit_solution(sol, cap, &scal[S_STORED], half_mask(p, qs, 0, lrec(li).hdr),
                                  half_mask(p, qs, 1, rrec(ri).hdr));
            }
        }
        return;
    }

    uint32_t rf[kKR];
    int64_t rk[CK ? kKR : 1];
#pragma unroll
    for (int k = 0; k < kKR; ++k) {
        const uint32_t ri = rb + k * 256 + t;
        rf[k] = 0u;
        if (CK) rk[k] = -1;                       // never equals a left key (>= 0)
        if (ri < re) {
            if (W > 0) rf[k] = fingerprint<W>(rrec(ri).vec);
            if (CK) rk[k] = rkey(p, rrec(ri));
        }
    }
    // Full check of a flagged (left j, right slot k) pair.
    auto check = [&](uint32_t li, int k) {
        const uint32_t ri = rb + k * 256 + t;
        if (ri >= re) return;
        const Rec<W> ll = lrec(li);
        const Rec<W> rr = rrec(ri);
        if (rows_match<W>(ll, rr))
            emit_pair(p, qs, sol, cap, &scal[S_NSOL], ll.hdr, rr.hdr);
    };
    uint64_t hits = 0;
    for (uint32_t c0 = lb; c0 < le; c0 += kChunk) {
        const uint32_t cn = min((uint32_t)kChunk, le - c0);
        __syncthreads();
        for (uint32_t i = t; i < cn; i += 256) {
            s_fp[i] = W > 0 ? fingerprint<W>(lrec(c0 + i).vec) : 0u;
            if (CK) s_lk[i] = rkey(p, lrec(c0 + i));
        }
        __syncthreads();
        if (!CK) {
            uint32_t j = 0;
            for (; j + 4 <= cn; j += 4) {
                const uint4 q = *reinterpret_cast<const uint4 *>(&s_fp[j]);
                uint64_t acc = 0;
                if constexpr (CMPX && kKR == 8) {
                    acc = match4x8(rf, q);
                } else {
#pragma unroll
                    for (int k = 0; k < kKR; ++k) acc |= __builtin_amdgcn_ballot_w64(rf[k] == q.x);
#pragma unroll
                    for (int k = 0; k < kKR; ++k) acc |= __builtin_amdgcn_ballot_w64(rf[k] == q.y);
#pragma unroll
                    for (int k = 0; k < kKR; ++k) acc |= __builtin_amdgcn_ballot_w64(rf[k] == q.z);
#pragma unroll
                    for (int k = 0; k < kKR; ++k) acc |= __builtin_amdgcn_ballot_w64(rf[k] == q.w);
                }
                if (__builtin_expect(acc != 0, 0)) {
#pragma unroll
                    for (int k = 0; k < kKR; ++k) {
                        if (rf[k] == q.x) check(c0 + j, k);
                        if (rf[k] == q.y) check(c0 + j + 1, k);
                        if (rf[k] == q.z) check(c0 + j + 2, k);
                        if (rf[k] == q.w) check(c0 + j + 3, k);
                    }
                }
            }
            for (; j < cn; ++j) {
                const uint32_t x = s_fp[j];
#pragma unroll
                for (int k = 0; k < kKR; ++k)
                    if (rf[k] == x) check(c0 + j, k);
            }
        } else {
            for (uint32_t jj = 0; jj < cn; ++jj) {
                const int64_t lk = s_lk[jj];
                const uint32_t x = s_fp[jj];
#pragma unroll
                for (int k = 0; k < kKR; ++k) {
                    if (rk[k] == lk) {
                        ++hits;
                        if (W == 0) {
                            atomicAdd((unsigned long long *)&scal[S_NSOL], 1ull);
                            if (scal[S_STORED] < cap)
                                emit_solution(sol, cap, &scal[S_STORED],
                                              half_mask(p, qs, 0, lrec(c0 + jj).hdr),
                                              half_mask(p, qs, 1, rrec(rb + k * 256 + t).hdr));
                        } else if (rf[k] == x) {
                            check(c0 + jj, k);
                        }
                    }
                }
            }
        }
    }
    if (CK) {
        const uint64_t tot = block_sum_u64(hits, s_s4);
        if (t == 0) add_u128(&scal[S_H_LO], &scal[S_H_HI], tot);
    }
}

// ---------------------------------------------------------------------------
// Launch limits.  An HSA dispatch holds the grid size in work-items as 32-bit
// numbers, so blocks x threads stays below 2^32 in x; y is the side index or
// a small split.  Launchers check every grid before enqueueing anything and
// return hipErrorInvalidConfiguration for one the device cannot take.
// ---------------------------------------------------------------------------

constexpr uint64_t kMaxGridItems = 0xFFFFFFFFull;
constexpr uint32_t kMaxGridY = 65535;

static bool grid_ok(dim3 g, uint32_t threads) {
    return g.x >= 1 && (uint64_t)g.x * threads <= kMaxGridItems && g.y >= 1 && g.y <= kMaxGridY &&
           g.z == 1;
}

#define MSP_GRID_CHECK(g, threads)                                      \
    do {                                                                \
        if (!grid_ok((g), (threads))) return hipErrorInvalidConfiguration; \
    } while (0)

// ---------------------------------------------------------------------------
// Device-wide exclusive scan of uint32 (reduce -> scan of block sums -> apply)
// ---------------------------------------------------------------------------

constexpr int kScanE = 4;
constexpr int kScanBlock = 256 * kScanE;

// Block sums (uint32, they feed the scan of offsets) and, when total64 is
// given, the exact 64-bit total: offsets wrap once the total passes 2^32, but
// the caller compares the 64-bit total with its capacity before using them.
__global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t *__restrict__ in, size_t n,
                                                     uint32_t *sums, uint64_t *total64) {
    __shared__ uint64_t s4[4];
    const size_t base = (size_t)blockIdx.x * kScanBlock;
    uint64_t s = 0;
    for (int e = 0; e < kScanE; ++e) {
        const size_t i = base + (size_t)e * 256 + threadIdx.x;
        if (i < n) s += in[i];
    }
    s = block_sum_u64(s, s4);
    if (threadIdx.x == 0) {
        sums[blockIdx.x] = (uint32_t)s;
        if (total64) atomicAdd((unsigned long long *)total64, (unsigned long long)s);
    }
}

// total64 (single-block scans only): the exact 64-bit sum of the inputs.
__global__ __launch_bounds__(256) void k_scan_apply(const uint32_t *__restrict__ in, uint32_t *out,
                                                    size_t n, const uint32_t *__restrict__ pref,
                                                    uint64_t *total64, int write_total) {
    __shared__ uint32_t s_a[kScanBlock];
    __shared__ uint32_t s_w4[4];
    __shared__ uint64_t s_t4[4];
    const size_t base = (size_t)blockIdx.x * kScanBlock;
    uint64_t s64 = 0;
    for (int e = 0; e < kScanE; ++e) {
        const size_t i = base + (size_t)e * 256 + threadIdx.x;
        const uint32_t v = i < n ? in[i] : 0u;
        s_a[e * 256 + threadIdx.x] = v;
        s64 += v;
    }
    __syncthreads();
    if (total64) s64 = block_sum_u64(s64, s_t4);
    const uint32_t tot = block_excl_scan_lds<kScanE>(s_a, s_w4);
    const uint32_t add = pref ? pref[blockIdx.x] : 0u;
    for (int e = 0; e < kScanE; ++e) {
        const size_t i = base + (size_t)e * 256 + threadIdx.x;
        if (i < n) out[i] = s_a[e * 256 + threadIdx.x] + add;
    }
    if (write_total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        out[n] = add + tot;
        if (total64) *total64 = s64;
    }
}

// Offsets of the count pass's part-major counts cnt[cell][part][fine]: one
// thread per bucket (cell, fine) walks the parts, writing each part's
// exclusive prefix within the bucket to pre[cell][part][fine] and the
// bucket's total to tot[cell][fine] (lanes take consecutive buckets, so every
// access is coalesced).  A scan of tot then gives each bucket's start.
// A bucket of 2^32 or more records (its parts' counts summed) cannot be
// addressed by the 32-bit offsets: bit 4 of *ovf, and the solve stops.
__global__ __launch_bounds__(256) void k_part_prefix(const uint32_t *__restrict__ cnt,
                                                     uint32_t *pre, uint32_t *tot, uint64_t nbk,
                                                     uint32_t F, uint32_t P, uint64_t *ovf) {
    const uint64_t bk = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (bk >= nbk) return;
    const uint64_t c = bk / F, f = bk - c * F;
    const uint64_t base = c * P * F + f;
    uint64_t run = 0;
    uint32_t p = 0;
    for (; p + 4 <= P; p += 4) {              // four independent loads in flight
        uint32_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = cnt[base + (uint64_t)(p + u) * F];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            pre[base + (uint64_t)(p + u) * F] = (uint32_t)run;
            run += v[u];
        }
    }
    for (; p < P; ++p) {
        const uint32_t v = cnt[base + (uint64_t)p * F];
        pre[base + (uint64_t)p * F] = (uint32_t)run;
        run += v;
    }
    tot[bk] = (uint32_t)run;
    if (run > 0xFFFFFFFFull) atomicOr((unsigned long long *)ovf, 4ull);
}

size_t scan_tmp_bytes(size_t n) {
    size_t bytes = 0;
    while (n > (size_t)kScanBlock) {
        n = (n + kScanBlock - 1) / kScanBlock;
        bytes += (n + 1) * sizeof(uint32_t) * 2 + 256;
    }
    return bytes + 256;
}

hipError_t scan_u32(const uint32_t *in, uint32_t *out, size_t n, uint64_t *total64, void *tmp,
                    size_t tmp_bytes, hipStream_t st) {
    if (n == 0) {
        hipError_t e = hipMemsetAsync(out, 0, sizeof(uint32_t), st);
        if (e == hipSuccess && total64) e = hipMemsetAsync(total64, 0, sizeof(uint64_t), st);
        return e;
    }
    const size_t nb = (n + kScanBlock - 1) / kScanBlock;
    if ((uint64_t)nb * 256 > kMaxGridItems) return hipErrorInvalidConfiguration;
    if (nb == 1) {
        hipLaunchKernelGGL(k_scan_apply, dim3(1), dim3(256), 0, st, in, out, n, nullptr, total64, 1);
        return hipGetLastError();
    }
    const size_t need = (nb + 1) * sizeof(uint32_t) * 2 + 256;
    if (tmp_bytes < need) return hipErrorInvalidValue;
    uint32_t *sums = (uint32_t *)tmp;
    uint32_t *pref = sums + nb + 1;
    if (total64) {
        hipError_t e0 = hipMemsetAsync(total64, 0, sizeof(uint64_t), st);
        if (e0 != hipSuccess) return e0;
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3((uint32_t)nb), dim3(256), 0, st, in, n, sums, total64);
    hipError_t e = scan_u32(sums, pref, nb, nullptr, (char *)tmp + need, tmp_bytes - need, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_apply, dim3((uint32_t)nb), dim3(256), 0, st, in, out, n, pref,
                       nullptr, 1);
    return hipGetLastError();
}

hipError_t scan_counts(const uint32_t *cnt, uint32_t *pre, uint32_t *tot, uint32_t *start,
                       uint64_t nbk, uint32_t F, uint32_t P, uint64_t *total64, uint64_t *ovf,
                       void *tmp, size_t tmp_bytes, hipStream_t st) {
    if (nbk == 0) return scan_u32(tot, start, 0, total64, tmp, tmp_bytes, st);
    const dim3 g((uint32_t)((nbk + 255) / 256));
    MSP_GRID_CHECK(g, 256);
    hipLaunchKernelGGL(k_part_prefix, g, dim3(256), 0, st, cnt, pre, tot, nbk, F, P, ovf);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return scan_u32(tot, start, nbk, total64, tmp, tmp_bytes, st);
}

// Candidate pairs of a window: sum over buckets of left x right records.
__global__ __launch_bounds__(256) void k_window_score(const uint32_t *__restrict__ totL,
                                                      const uint32_t *__restrict__ totR,
                                                      uint64_t nbk, uint64_t *score) {
    __shared__ uint64_t s4[4];
    uint64_t v = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < nbk;
         i += (uint64_t)gridDim.x * 256)
        v += (uint64_t)totL[i] * totR[i];
    v = block_sum_u64(v, s4);
    if (threadIdx.x == 0 && v) atomicAdd((unsigned long long *)score, (unsigned long long)v);
}

hipError_t launch_window_score(const DevBufs &b, uint64_t nbk, uint64_t *score, hipStream_t st) {
    if (nbk == 0) return hipSuccess;
    const dim3 g((uint32_t)std::min<uint64_t>((nbk + 255) / 256, 1024));
    hipLaunchKernelGGL(k_window_score, g, dim3(256), 0, st, b.tot[0], b.tot[1], nbk, score);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

size_t qrec_bytes(int W) {
    switch (W) {
        case 0: return sizeof(QRec<0>);
        case 1: return sizeof(QRec<1>);
        case 2: return sizeof(QRec<2>);
        case 3: return sizeof(QRec<3>);
        case 4: return sizeof(QRec<4>);
        default: return sizeof(QRec<5>);
    }
}

size_t rec_bytes(int W) {
    switch (W) {
        case 0: return sizeof(Rec<0>);
        case 1: return sizeof(Rec<1>);
        case 2: return sizeof(Rec<2>);
        case 3: return sizeof(Rec<3>);
        case 4: return sizeof(Rec<4>);
        default: return sizeof(Rec<5>);
    }
}

template <int W>
static QPtrs<W> sorted_quarters(const DevBufs &b) {
    QPtrs<W> q;
    for (int x = 0; x < 4; ++x) q.q[x] = (QRec<W> *)b.qsrt[x];
    return q;
}

#define MSP_DISPATCH_W(W, CALL)                       \
    switch (W) {                                      \
        case 0: { constexpr int WW = 0; CALL; } break; \
        case 1: { constexpr int WW = 1; CALL; } break; \
        case 2: { constexpr int WW = 2; CALL; } break; \
        case 3: { constexpr int WW = 3; CALL; } break; \
        case 4: { constexpr int WW = 4; CALL; } break; \
        case 5: { constexpr int WW = 5; CALL; } break; \
        default: return hipErrorInvalidValue;         \
    }

template <int W>
static hipError_t quarters_impl(const Plan &p, const DevBufs &b, hipStream_t st) {
    const uint64_t tot = (uint64_t)p.Q[0] + p.Q[1] + p.Q[2] + p.Q[3];
    const uint32_t grid = (uint32_t)((tot + 255) / 256);
    MSP_GRID_CHECK(dim3(grid), 256);
    QPtrs<W> raw, srt;
    UPtrs cnt, cur;
    for (int x = 0; x < 4; ++x) {
        raw.q[x] = (QRec<W> *)b.qraw[x];
        srt.q[x] = (QRec<W> *)b.qsrt[x];
        cnt.q[x] = b.qcnt[x];
        cur.q[x] = b.qcur[x];
    }
    UPtrs vraw, vsrt;
    for (int x = 0; x < 4; ++x) {
        vraw.q[x] = b.qvraw[x];
        vsrt.q[x] = b.qvsrt[x];
    }
    KPtrs khraw, khsrt;
    for (int x = 0; x < 4; ++x) {
        khraw.q[x] = b.qkhraw[x];
        khsrt.q[x] = b.qkhsrt[x];
    }
    hipLaunchKernelGGL(k_quarter_gen<W>, dim3(grid), dim3(256), 0, st, p, b.colw, b.colwh, b.rows,
                       raw, cnt, vraw, khraw);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t T = (size_t)1 << p.log2T;
    for (int x = 0; x < 4; ++x) {
        e = scan_u32(b.qcnt[x], b.qcnt[x], T, nullptr, b.scan_tmp, b.scan_tmp_bytes, st);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(b.qcur[x], b.qcnt[x], T * sizeof(uint32_t), hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_quarter_sort<W>, dim3(grid), dim3(256), 0, st, p, raw, srt, cur, vraw,
                       vsrt, khraw, khsrt);
    return hipGetLastError();
}

hipError_t launch_quarters(const Plan &p, const DevBufs &b, int, hipStream_t st) {
    MSP_DISPATCH_W(p.Wr, return quarters_impl<WW>(p, b, st));
    return hipSuccess;
}

template <int W>
static hipError_t count_impl(const Plan &p, const DevBufs &b, int64_t idx0, int32_t K,
                             hipStream_t st) {
    // Four outer elements per thread while cells hold few inner elements;
    // inner keys loaded about as many at a time as a cell holds per element.
    const uint64_t T = (uint64_t)1 << p.log2T;
    const uint64_t qin = std::min((uint64_t)p.Q[1], (uint64_t)p.Q[3]);
    if ((uint64_t)K * p.parts > 0xFFFFFFFFull) return hipErrorInvalidConfiguration;
    dim3 grid((uint32_t)K * p.parts, 2);
    MSP_GRID_CHECK(grid, 256);
    const bool sl = p.slice_mod != 0;
#define MSP_COUNT_K(PERV, KUV, KWV)                                                             \
    do {                                                                                        \
        if (sl)                                                                                 \
            hipLaunchKernelGGL((k_count<W, PERV, KUV, true, KWV>), grid, dim3(256), 0, st, p,   \
                               (const QRec<W> *)b.qsrt[0], (const QRec<W> *)b.qsrt[1],          \
                               b.qcnt[1], (const QRec<W> *)b.qsrt[2],                           \
                               (const QRec<W> *)b.qsrt[3], b.qcnt[3], b.cnt[0], b.cnt[1], idx0, \
                               b.scal);                                                         \
        else                                                                                    \
            hipLaunchKernelGGL((k_count<W, PERV, KUV, false, KWV>), grid, dim3(256), 0, st, p,  \
                               (const QRec<W> *)b.qsrt[0], (const QRec<W> *)b.qsrt[1],          \
                               b.qcnt[1], (const QRec<W> *)b.qsrt[2],                           \
                               (const QRec<W> *)b.qsrt[3], b.qcnt[3], b.cnt[0], b.cnt[1], idx0, \
                               b.scal);                                                         \
    } while (0)
    // Keys past int64 come with second-key-word records (two words).
    if constexpr (W == 2) {
        if (p.kw) {
            if (qin >= 16 * T) MSP_COUNT_K(1, 8, true);
            else if (qin > 2 * T) MSP_COUNT_K(4, 4, true);
            else MSP_COUNT_K(4, 2, true);
            return hipGetLastError();
        }
    }
#define MSP_COUNT(PERV, KUV) MSP_COUNT_K(PERV, KUV, false)
    if (qin >= 16 * T) MSP_COUNT(1, 8);
    else if (qin > 2 * T) MSP_COUNT(4, 4);
    else MSP_COUNT(4, 2);
#undef MSP_COUNT
#undef MSP_COUNT_K
    return hipGetLastError();
}

hipError_t launch_count(const Plan &p, const DevBufs &b, int64_t idx0, int32_t K, hipStream_t st) {
    MSP_DISPATCH_W(p.Wr, return count_impl<WW>(p, b, idx0, K, st));
    return hipSuccess;
}

template <int W>
static hipError_t staged_impl(const Plan &p, const DevBufs &b, int64_t idx0, int32_t K,
                              hipStream_t st) {
    // Outer elements per thread per chunk: enough pairs (about Q_inner / T
    // per outer element) to fill about one batch.
    const uint64_t T = (uint64_t)1 << p.log2T;
    const uint64_t qin = std::min((uint64_t)p.Q[1], (uint64_t)p.Q[3]);
    int per = 1;
    while (per < 16 && (uint64_t)256 * (2 * per) * qin <= (uint64_t)kStageBatch * T) per *= 2;
    // 1024-thread groups hold 128 registers per lane: at most 4 elements per
    // thread there (more spill).
    const int F = 1 << p.log2F;
    if (F > 1024 && F <= 2048) per = std::min(per, 4);
    // LDS for the per-bucket cursors is sized to F: more work-groups per CU.
    if ((uint64_t)K * p.parts > 0xFFFFFFFFull) return hipErrorInvalidConfiguration;
    dim3 grid((uint32_t)K * p.parts, 2);
    MSP_GRID_CHECK(grid, 1024);
    // Threads per work-group (batch = 12 pairs per thread), by the LDS that
    // the bucket cursors leave: 512 for F <= 1024 (two groups per CU), 1024
    // for F = 2048 (one group of 16 waves), 256 for F = 4096.
#define MSP_NT(MF) ((MF) <= 1024 ? 512 : (MF) <= 2048 ? 1024 : 256)
#define MSP_STAGED(PERV, MF)                                                                    \
    hipLaunchKernelGGL((k_scatter_staged<W, PERV, MF, MSP_NT(MF)>), grid, dim3(MSP_NT(MF)), 0, \
                       st, p,                                                                   \
                       (const QRec<W> *)b.qsrt[0], (const QRec<W> *)b.qsrt[1], b.qcnt[1],       \
                       (const QRec<W> *)b.qsrt[2], (const QRec<W> *)b.qsrt[3], b.qcnt[3],       \
                       b.off[0], b.off[1], b.pre[0], b.pre[1], (Rec<W> *)b.rec[0],         \
                       (Rec<W> *)b.rec[1], idx0)
#define MSP_STAGED_PER(MF)                                                                      \
    switch (per) {                                                                              \
        case 1: MSP_STAGED(1, MF); break;                                                       \
        case 2: MSP_STAGED(2, MF); break;                                                       \
        case 4: MSP_STAGED(4, MF); break;                                                       \
        case 8: MSP_STAGED(8, MF); break;                                                       \
        default: MSP_STAGED(16, MF); break;                                                     \
    }
    if (F <= 1024) {
        MSP_STAGED_PER(1024)
    } else if (F <= 2048) {
        MSP_STAGED_PER(2048)
    } else {
        MSP_STAGED_PER(kMaxFine)
    }
#undef MSP_STAGED_PER
#undef MSP_STAGED
#undef MSP_NT
    return hipGetLastError();
}

template <int W, bool FP, bool SLICE, bool KW = false>
static hipError_t rec_impl(const Plan &p, const DevBufs &b, int64_t idx0, int32_t K,
                           hipStream_t st) {
    // Outer elements per thread per chunk: enough pairs (about Q_inner / T
    // per outer element) to fill one batch, at most 4 (128 registers).
    const uint64_t T = (uint64_t)1 << p.log2T;
    const uint64_t qin = std::min((uint64_t)p.Q[1], (uint64_t)p.Q[3]);
    const int F = 1 << p.log2F;
    const uint64_t batch = F > 2048 ? rec_batch<W, 4096>() : rec_batch<W, 2048>();
    int per = 1;
    while (per < 4 && (uint64_t)kRecNT * (2 * per) * qin <= batch * T) per *= 2;
    if ((uint64_t)K * p.parts > 0xFFFFFFFFull) return hipErrorInvalidConfiguration;
    dim3 grid((uint32_t)K * p.parts, 2);
    MSP_GRID_CHECK(grid, kRecNT);
#define MSP_REC(PERV, MF)                                                                       \
    hipLaunchKernelGGL((k_scatter_rec<W, PERV, MF, FP, SLICE, KW>), grid, dim3(kRecNT), 0, st,  \
                       p,                                                                       \
                       (const QRec<W> *)b.qsrt[0], (const QRec<W> *)b.qsrt[1], b.qcnt[1],       \
                       (const QRec<W> *)b.qsrt[2], (const QRec<W> *)b.qsrt[3], b.qcnt[3],       \
                       b.off[0], b.off[1], b.pre[0], b.pre[1], (Rec<W> *)b.rec[0],              \
                       (Rec<W> *)b.rec[1], idx0)
#define MSP_REC_PER(MF)                                                                         \
    switch (per) {                                                                              \
        case 1: MSP_REC(1, MF); break;                                                          \
        case 2: MSP_REC(2, MF); break;                                                          \
        default: MSP_REC(4, MF); break;                                                         \
    }
    if (F <= 1024) {
        MSP_REC_PER(1024)
    } else if (F <= 2048) {
        MSP_REC_PER(2048)
    } else {
        MSP_REC_PER(kMaxFine)
    }
#undef MSP_REC_PER
#undef MSP_REC
    return hipGetLastError();
}

hipError_t launch_scatter(const Plan &p, const DevBufs &b, int64_t idx0, int32_t K,
                          hipStream_t st) {
    const bool sl = p.slice_mod != 0;
    if (p.wide) {                        // fingerprint + second key word
        if (p.Wr != 2 || !p.fp) return hipErrorInvalidValue;
        if (p.kw)
            return sl ? rec_impl<2, true, true, true>(p, b, idx0, K, st)
                      : rec_impl<2, true, false, true>(p, b, idx0, K, st);
        return sl ? rec_impl<2, true, true, false>(p, b, idx0, K, st)
                  : rec_impl<2, true, false, false>(p, b, idx0, K, st);
    }
    if (p.Wr == 0)
        return sl ? rec_impl<0, false, true>(p, b, idx0, K, st)
                  : rec_impl<0, false, false>(p, b, idx0, K, st);
    if (p.Wr == 1) {
        if (p.fp)
            return sl ? rec_impl<1, true, true>(p, b, idx0, K, st)
                      : rec_impl<1, true, false>(p, b, idx0, K, st);
        return sl ? rec_impl<1, false, true>(p, b, idx0, K, st)
                  : rec_impl<1, false, false>(p, b, idx0, K, st);
    }
    switch (p.Wr) {
        case 2: return staged_impl<2>(p, b, idx0, K, st);
        case 3: return staged_impl<3>(p, b, idx0, K, st);
        case 4: return staged_impl<4>(p, b, idx0, K, st);
        case 5: return staged_impl<5>(p, b, idx0, K, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_exact_runs(const Plan &p, const DevBufs &b, int32_t K, hipStream_t st) {
    if (((uint64_t)K << p.log2F) > 0xFFFFFFFFull) return hipErrorInvalidConfiguration;
    const uint32_t nb = (uint32_t)K << p.log2F;
    MSP_GRID_CHECK(dim3((nb + 255) / 256), 256);
    hipLaunchKernelGGL(k_exact_runs, dim3((nb + 255) / 256), dim3(256), 0, st, p, b.off[0],
                       b.off[1], nb, b.runs, b.scal, p.W == 0 ? 1 : 0);
    return hipGetLastError();
}

template <int W>
static hipError_t join_impl(const Plan &p, const DevBufs &b, int32_t K, uint64_t cap,
                            hipStream_t st) {
    if (((uint64_t)K << p.log2F) > 0xFFFFFFFFull) return hipErrorInvalidConfiguration;
    const uint32_t nb = (uint32_t)K << p.log2F;
    const Rec<W> *L = (const Rec<W> *)b.rec[0], *R = (const Rec<W> *)b.rec[1];
    const dim3 pg(std::min<uint32_t>(nb, 4096));         // persistent chain join
    // The grouped join takes one work-group per bucket: 256 threads for
    // buckets of about a thousand records, 1024 for buckets of a few thousand
    // (p.gbig).
    if (p.vjoin || p.join_grouped == 1) MSP_GRID_CHECK(dim3(nb), p.gbig ? 1024 : 256);
#define MSP_GROUPED(K32V, VJV)                                                                  \
    do {                                                                                        \
        if constexpr (W <= 2) {                                                                 \
            if (p.gbig) {                                                                       \
                hipLaunchKernelGGL((k_join_grouped<W, K32V, VJV, 1024, kGroupCapBig,            \
                                                   kGroupSlotsBig>),                            \
                                   dim3(nb), dim3(1024), 0, st, p, b.off[0], b.off[1], L, R,     \
                                   b.heavy, b.scal, b.sol, cap, sorted_quarters<W>(b));         \
                break;                                                                          \
            }                                                                                   \
        }                                                                                       \
            hipLaunchKernelGGL((k_join_grouped<W, K32V, VJV>), dim3(nb), dim3(256), 0, st, p,   \
                               b.off[0], b.off[1], L, R, b.heavy, b.scal, b.sol, cap,            \
                               sorted_quarters<W>(b));                                          \
    } while (0)
    if (p.vjoin && p.khb <= 32)            // vector join: the grouped kernel decides every run
        MSP_GROUPED(true, true);
    else if (p.vjoin)
        MSP_GROUPED(false, true);
    else if (p.join_grouped == 2 && p.khb <= 32)
        hipLaunchKernelGGL((k_join_pairs<W, true>), dim3(std::min<uint32_t>((nb + 3) / 4, 8192)),
                           dim3(256), 0, st, p, b.off[0], b.off[1], L, R, b.heavy, b.scal, b.sol,
                           cap, sorted_quarters<W>(b), nb);
    else if (p.join_grouped == 2)
        hipLaunchKernelGGL((k_join_pairs<W, false>), dim3(std::min<uint32_t>((nb + 3) / 4, 8192)),
                           dim3(256), 0, st, p, b.off[0], b.off[1], L, R, b.heavy, b.scal, b.sol,
                           cap, sorted_quarters<W>(b), nb);
    else if (p.join_grouped && p.khb <= 32)
        MSP_GROUPED(true, false);
    else if (p.join_grouped)
        MSP_GROUPED(false, false);
    else if (p.khb <= 32)
        hipLaunchKernelGGL((k_join_light<W, true>), pg, dim3(256), 0, st, p, b.off[0], b.off[1], L,
                           R, b.heavy, b.scal, b.sol, cap, sorted_quarters<W>(b), nb);
    else
        hipLaunchKernelGGL((k_join_light<W, false>), pg, dim3(256), 0, st, p, b.off[0], b.off[1],
                           L, R, b.heavy, b.scal, b.sol, cap, sorted_quarters<W>(b), nb);
#undef MSP_GROUPED
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // Second pass over the buckets the 256-thread grouped join deferred:
    // 1024-thread groups for those of up to kGroupCapBig left records.
    bool second = false;
    if constexpr (W <= 2) {
        if ((p.vjoin || p.join_grouped == 1) && !p.gbig) {
            second = true;
            const dim3 g2(std::min<uint32_t>(nb, 512));
#define MSP_LIST(K32V, VJV)                                                                      \
    hipLaunchKernelGGL((k_join_grouped_list<W, K32V, VJV>), g2, dim3(1024), 0, st, p, b.off[0],  \
                       b.off[1], L, R, b.heavy, b.heavy2, b.scal, b.sol, cap, sorted_quarters<W>(b))
            if (p.vjoin && p.khb <= 32) MSP_LIST(true, true);
            else if (p.vjoin) MSP_LIST(false, true);
            else if (p.khb <= 32) MSP_LIST(true, false);
            else MSP_LIST(false, false);
#undef MSP_LIST
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    // Buckets deferred once more go to the heavy kernels (count read on the
    // device).
    uint32_t *hl = second ? b.heavy2 : b.heavy;
    const int hs = second ? (int)S_NHEAVY2 : (int)S_NHEAVY;
    if (p.vjoin && p.khb <= 31)
        hipLaunchKernelGGL((k_join_heavy_vj2<W, true>), dim3(std::min<uint32_t>(nb, 1024)),
                           dim3(1024), 0, st, p, b.off[0], b.off[1], L, R, hl, b.scal, b.sol, cap,
                           sorted_quarters<W>(b), hs);
    else if (p.vjoin && p.khb <= 63)
        hipLaunchKernelGGL((k_join_heavy_vj2<W, false>), dim3(std::min<uint32_t>(nb, 1024)),
                           dim3(1024), 0, st, p, b.off[0], b.off[1], L, R, hl, b.scal, b.sol, cap,
                           sorted_quarters<W>(b), hs);
    else if (p.vjoin && p.khb <= 32)
        hipLaunchKernelGGL((k_join_heavy_vj<W, true>), dim3(std::min<uint32_t>(nb, 2048)), dim3(256),
                           0, st, p, b.off[0], b.off[1], L, R, hl, b.scal, b.sol, cap,
                           sorted_quarters<W>(b), hs);
    else if (p.vjoin)
        hipLaunchKernelGGL((k_join_heavy_vj<W, false>), dim3(std::min<uint32_t>(nb, 2048)),
                           dim3(256), 0, st, p, b.off[0], b.off[1], L, R, hl, b.scal, b.sol,
                           cap, sorted_quarters<W>(b), hs);
    else
        hipLaunchKernelGGL(k_join_heavy<W>, dim3(std::min<uint32_t>(nb, 2048)), dim3(256), 0, st,
                           p, b.off[0], b.off[1], L, R, hl, b.iruns, b.idx, b.scal, b.sol, cap,
                           b.iruns_cap, b.idx_cap, sorted_quarters<W>(b), hs);
    return hipGetLastError();
}

hipError_t launch_hash_join(const Plan &p, const DevBufs &b, int32_t K, uint64_t cap,
                            hipStream_t st) {
    MSP_DISPATCH_W(p.Wr, return join_impl<WW>(p, b, K, cap, st));
    return hipSuccess;
}

template <int W>
static hipError_t vjoin_impl(const Plan &p, const DevBufs &b, uint32_t nruns, uint64_t cap,
                             hipStream_t st) {
    const uint64_t slots = (uint64_t)b.vtab_mask + 1;
    MSP_GRID_CHECK(dim3(std::min<uint32_t>(nruns, 4096), 16), 256);
    hipError_t e = hipMemsetAsync(b.vtab, 0xFF, slots * 4, st);
    if (e != hipSuccess) return e;
    // Blocks stride over runs; the second grid dimension splits long runs.
    const dim3 grid(std::min<uint32_t>(nruns, 4096), 16);
    MSP_GRID_CHECK(grid, 256);
    hipLaunchKernelGGL(k_vjoin_insert<W>, grid, dim3(256), 0, st, b.runs, nruns,
                       (const Rec<W> *)b.rec[0], b.vtab, b.vtab_mask);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_vjoin_probe<W>, grid, dim3(256), 0, st, p, b.runs, nruns,
                       (const Rec<W> *)b.rec[0], (const Rec<W> *)b.rec[1], b.vtab, b.vtab_mask,
                       b.scal, b.sol, cap, sorted_quarters<W>(b));
    return hipGetLastError();
}

hipError_t launch_vector_join(const Plan &p, const DevBufs &b, uint32_t nruns, uint64_t cap,
                              hipStream_t st) {
    if (nruns == 0) return hipSuccess;
    MSP_DISPATCH_W(p.Wr, return vjoin_impl<WW>(p, b, nruns, cap, st));
    return hipSuccess;
}

hipError_t launch_tile_counts(const Plan &, const DevBufs &b, uint32_t nruns, int mode,
                              hipStream_t st) {
    if (nruns == 0) return hipSuccess;
    const uint32_t tile_r = 256u * 8;        // right records per verify tile
    MSP_GRID_CHECK(dim3((nruns + 255) / 256), 256);
    if (mode == 2)
        hipLaunchKernelGGL(k_tile_counts, dim3((nruns + 255) / 256), dim3(256), 0, st, b.iruns,
                           nruns, b.itiles, tile_r, b.scal);
    else
        hipLaunchKernelGGL(k_tile_counts, dim3((nruns + 255) / 256), dim3(256), 0, st, b.runs,
                           nruns, b.tiles, tile_r, b.scal);
    return hipGetLastError();
}

template <int W>
static hipError_t verify_impl(const Plan &p, const DevBufs &b, uint32_t nruns, uint32_t ntiles,
                              uint64_t cap, int mode, hipStream_t st) {
    const Rec<W> *L = (const Rec<W> *)b.rec[0], *R = (const Rec<W> *)b.rec[1];
    // One work-group per tile, in launches of at most 2^23 tiles.
    constexpr uint32_t kTilesPerLaunch = 1u << 23;
    for (uint32_t t0 = 0; t0 < ntiles; t0 += kTilesPerLaunch) {
        const dim3 g(std::min(kTilesPerLaunch, ntiles - t0));
        MSP_GRID_CHECK(g, 256);
        if (mode == 2)
            hipLaunchKernelGGL((k_verify<W, false, 8, true, true>), g, dim3(256), 0, st, p, L, R,
                               b.iruns, b.itiles, nruns, b.scal, b.sol, cap, b.idx,
                               sorted_quarters<W>(b), t0);
        else if (mode == 1)
            hipLaunchKernelGGL((k_verify<W, true, 8>), g, dim3(256), 0, st, p, L, R, b.runs,
                               b.tiles, nruns, b.scal, b.sol, cap, b.idx, sorted_quarters<W>(b),
                               t0);
        else
            hipLaunchKernelGGL((k_verify<W, false, 8, true>), g, dim3(256), 0, st, p, L, R,
                               b.runs, b.tiles, nruns, b.scal, b.sol, cap, b.idx,
                               sorted_quarters<W>(b), t0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_verify(const Plan &p, const DevBufs &b, uint32_t nruns, uint32_t ntiles,
                         uint64_t cap, int mode, hipStream_t st) {
    if (ntiles == 0) return hipSuccess;
    MSP_DISPATCH_W(p.Wr, return verify_impl<WW>(p, b, nruns, ntiles, cap, mode, st));
    return hipSuccess;
}

}  // namespace msp
