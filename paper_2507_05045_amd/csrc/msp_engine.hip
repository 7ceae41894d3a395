// Host side of libmsp: instance validation, the solve plan, workspace
// layout, the per-window launch sequence and the C ABI of include/msp.h.
#include "msp.h"
#include "msp_internal.h"

#include <algorithm>
#include <cmath>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <thread>
#include <vector>

using namespace msp;

struct msp_ctx {
    int m = 0, n = 0;
    std::vector<int32_t> A, d;
    bool have_result = false;
    uint64_t h_lo = 0, h_hi = 0, nsol = 0;
    std::vector<uint8_t> sol;          // stored solutions, canonical order, n bytes each
    uint64_t stored = 0;
    msp_stats_t stats{};
    void *ws = nullptr;                // library-owned workspace (cached)
    size_t ws_bytes = 0;
    msp_alloc_fn ws_alloc = nullptr;   // allocator that made ws (null: hipMalloc)
    msp_release_fn ws_release = nullptr;
    void *ws_user = nullptr;
    hipStream_t own_stream = nullptr;
    bool poisoned = false;
    std::atomic<int> busy{0};          // a solve or request is using this context
    uint64_t hs_fixed[msp::S_COUNT] = {};   // scalar copies of msp_solve_noalloc
};

namespace {

int lg2ceil(uint64_t x) {
    int k = 0;
    while (k < 63 && ((uint64_t)1 << k) < x) ++k;
    return k;
}

uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// Device memory for workspaces the library owns: hipMalloc/hipFree, or the
// caller's allocator (msp_set_allocator).  Each allocation keeps the pair
// that made it, so a later change of allocator still frees it correctly.
struct DevAllocator {
    msp_alloc_fn alloc = nullptr;
    msp_release_fn release = nullptr;
    void *user = nullptr;
};
std::mutex g_alloc_mu;
DevAllocator g_alloc;

struct DevMem {
    void *ptr = nullptr;
    DevAllocator by;
};

DevMem dev_alloc(uint64_t bytes) {
    DevMem m;
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        m.by = g_alloc;
    }
    if (m.by.alloc) {
        m.ptr = m.by.alloc((size_t)bytes, m.by.user);
        if (m.ptr && ((uintptr_t)m.ptr & 255u)) {     // the workspace layout needs 256-byte alignment
            if (m.by.release) m.by.release(m.ptr, m.by.user);
            m.ptr = nullptr;
        }
    } else if (hipMalloc(&m.ptr, bytes) != hipSuccess) {
        (void)hipGetLastError();
        m.ptr = nullptr;
    }
    return m;
}

void dev_free(DevMem &m) {
    if (!m.ptr) return;
    if (m.by.alloc) {
        if (m.by.release) m.by.release(m.ptr, m.by.user);
    } else {
        (void)hipFree(m.ptr);
    }
    m.ptr = nullptr;
}

struct Sizes {
    uint64_t ncells = 0;     // cells to visit (all, or those of the slice)
    uint64_t kwin = 0;       // cells per window (planned)
    uint64_t cap_rec = 0;    // half records per side per window
    uint64_t sol_cap = 0;
    uint64_t total = 0;      // workspace bytes
    // offsets into the workspace
    uint64_t o_qraw[4], o_qsrt[4], o_qcnt[4], o_qcur[4], o_cnt[2], o_off[2], o_rec[2];
    uint64_t o_qvraw[4], o_qvsrt[4], o_pre[2], o_tot[2], o_wscore = 0;
    uint64_t o_runs, o_tiles, o_sol, o_scal, o_scan, scan_bytes, o_colw, o_rows;
    uint64_t o_colwh = 0, o_qkhraw[4] = {}, o_qkhsrt[4] = {};
    uint64_t o_iruns, o_itiles, o_idx, n_iruns, o_heavy, o_heavy2, idx_n;
    uint64_t o_vtab, vtab_slots;
    uint64_t max_items = 0;  // largest launch of a window, work-items
};

struct Prepared {
    Plan p{};
    std::vector<int64_t> colw, colwh;       // column weights: low and high words
    std::vector<uint16_t> rows;
    bool infeasible = false;
    int key_bits = 0;                       // bits of K_d + 1
    Sizes z;
};

// Instance-level checks shared by msp_create and the plan.
int validate(const int32_t *A, const int32_t *d, int m, int n) {
    if (!A || !d || m < 1 || n < 1) return MSP_E_INVALID;
    if (m > 16 || n > kMaxN) return MSP_E_UNSUPPORTED;
    for (int i = 0; i < m; ++i) {
        if (d[i] < 0) return MSP_E_INVALID;
        int64_t s = 0;
        for (int j = 0; j < n; ++j) {
            const int32_t a = A[(size_t)i * n + j];
            if (a < 0) return MSP_E_INVALID;
            s += a;
        }
        if (s > 65534) return MSP_E_RANGE;
    }
    return MSP_OK;
}

constexpr uint64_t kMaxLaunchItems = 0xFFFFFFFFull;

// Largest work-item count among the launches of one window of kw cells
// (the tiled verify's grid depends on the data and is split at launch).
uint64_t plan_max_items(const Plan &p, uint64_t kw) {
    uint64_t items = 0;
    auto mx = [&](uint64_t v) { items = std::max(items, v); };
    const uint64_t F = (uint64_t)1 << p.log2F;
    mx(((uint64_t)p.Q[0] + p.Q[1] + p.Q[2] + p.Q[3] + 255) / 256 * 256);   // quarter lists
    mx(kw * (uint64_t)p.parts * 256);                                          // count
    const uint64_t nt = F <= 1024 ? 512 : F <= 2048 ? 1024 : 256;           // scatter threads
    mx(kw * (uint64_t)p.parts * nt);
    const uint64_t nb = kw * F;                                                // buckets
    mx((nb + 255) / 256 * 256);                                                // exact runs
    if (!p.exact && (p.vjoin || p.join_grouped == 1)) mx(nb * 256);            // one group per bucket
    return items;
}

// log2 of the expected number of equal-key records per side near K_d: the
// 2^h_L left halves spread over the key rows' half sums, each about normal
// with variance sum a_ij^2 / 4 over the left columns (a planning estimate).
double expected_group_lg2(const msp_ctx *c, const Plan &p) {
    double lg = p.hL;
    for (int i = 0; i < p.r; ++i) {
        double s2 = 0.0;
        for (int j = 0; j < p.hL; ++j) {
            const double a = c->A[(size_t)i * c->n + j];
            s2 += a * a / 4.0;
        }
        if (s2 > 0.0) lg -= 0.5 * std::log2(2.0 * 3.141592653589793 * s2);
    }
    return lg;
}

// The plan: surrogate key (Section 1, eq. surrogate), quarter widths
// (Algorithm 1's partition, contiguous), residue modulus, cells, windows.
// Widest inner quarter: 2^28 subsets (4 GiB of quarter records at most);
// at most 2^29 residue cells (cell tables of 2 GiB per quarter and copy).
constexpr int kMaxQuarterBits = 28;
constexpr int kMaxCellBits = 29;

int prepare(const msp_ctx *c, const msp_opts &o, uint64_t budget, Prepared &P) {
    Plan &p = P.p;
    const int m = c->m, n = c->n;
    const int r = o.key_rows ? o.key_rows : 1;
    if (r < 1 || r > m) return MSP_E_INVALID;
    if (m - r > 2 * kMaxWords) return MSP_E_UNSUPPORTED;
    if (o.slice_mod < 0 || (o.slice_mod > 0 && ((o.slice_mod & (o.slice_mod - 1)) != 0 ||
                                                o.slice_res < 0 || o.slice_res >= o.slice_mod)))
        return MSP_E_INVALID;
    if (o.log2_m < 0 || o.log2_m > 62 || o.log2_cells < 0 || o.log2_cells > kMaxCellBits ||
        o.parts < 0)
        return MSP_E_INVALID;
    p.m = m; p.n = n; p.r = r; p.nv = m - r; p.W = (p.nv + 1) / 2;
    p.hL = (n + 1) / 2;
    // Quarters: Algorithm 1 splits each half into two lists of equal size.
    // log2_outer = q_A < ceil(hL / 2) moves s = ceil(hL / 2) - q_A variables
    // of each half from its outer quarter (A, C) to its inner one (B, D):
    // the same pairs, fewer outer elements per residue cell, so more cells
    // (and fewer fine buckets per cell) cost the same outer re-reads.
    {
        const int qa0 = (p.hL + 1) / 2;
        if (o.log2_outer < 0 || o.log2_outer > qa0) return MSP_E_INVALID;
        const int s = o.log2_outer ? qa0 - o.log2_outer : 0;
        p.qa = qa0 - s; p.qb = p.hL - p.qa;
        p.qc = (n - p.hL + 1) / 2 - s; p.qd = (n - p.hL) - p.qc;
        if (p.qa < 0 || p.qc < 0) return MSP_E_INVALID;
        if (p.qb > kMaxQuarterBits || p.qd > kMaxQuarterBits) return MSP_E_UNSUPPORTED;
    }
    p.Q[0] = 1u << p.qa; p.Q[1] = 1u << p.qb; p.Q[2] = 1u << p.qc; p.Q[3] = 1u << p.qd;

    // Key (Section 1, eq. surrogate): digit i is the row sum a_i.x, radix
    // rad_i.  key_base 0 takes the paper's B = n*D for every row (D > every
    // a_ij, D = 100 for the [0,99] family); key_base 1 the mixed radix
    // rowsum_i + 1, the smallest that still bounds every digit, so the same
    // int64 holds more rows.  Either way 0 <= a_i.x <= rowsum_i < rad_i, so
    // key(x) = K_d exactly when rows 1..r hold.
    if (o.key_base < 0 || o.key_base > 1) return MSP_E_INVALID;
    if (o.key_words < 0 || o.key_words > 2) return MSP_E_INVALID;
    int32_t amax = 0;
    for (int32_t a : c->A) amax = std::max(amax, a);
    const int64_t D = std::max<int64_t>(100, (int64_t)amax + 1);
    // The key in 128 bits: past int64 the quarters carry a high word (kw)
    // and the records a second key word.  Keys stay below 2^96.
    using u128 = unsigned __int128;
    const u128 kKeyLimit = (u128)1 << 96;
    std::vector<u128> pw(r, 1);                     // place value of digit i
    u128 kmax = 0, place = 1;
    P.infeasible = false;
    for (int i = 0; i < r; ++i) {
        int64_t rs = 0;
        for (int j = 0; j < n; ++j) rs += c->A[(size_t)i * n + j];
        if (c->d[i] > rs) P.infeasible = true;      // row i can never hold: H = 0
        pw[i] = place;
        kmax += place * (u128)rs;
        if (kmax >= kKeyLimit) return MSP_E_KEY_OVERFLOW;
        place *= (u128)(o.key_base ? rs + 1 : (int64_t)n * D);
        if (i + 1 < r && place >= kKeyLimit) return MSP_E_KEY_OVERFLOW;
    }
    p.kw = kmax >= ((u128)1 << 63) ? 1 : 0;
    // d_i <= rowsum_i on every key row keeps K_d below the largest key.
    u128 kd = 0;
    if (!P.infeasible)
        for (int i = 0; i < r; ++i) kd += pw[i] * (u128)c->d[i];
    p.Kd = (int64_t)(uint64_t)kd;
    p.Kdh = (int64_t)(uint64_t)(kd >> 64);
    P.colw.assign(n, 0);
    P.colwh.assign(n, 0);
    for (int j = 0; j < n; ++j) {
        u128 sw = 0;
        for (int i = 0; i < r; ++i) sw += pw[i] * (u128)c->A[(size_t)i * n + j];
        P.colw[j] = (int64_t)(uint64_t)sw;
        P.colwh[j] = (int64_t)(uint64_t)(sw >> 64);
    }
    P.rows.assign((size_t)std::max(p.nv, 1) * n, 0);
    for (int v = 0; v < p.nv; ++v)
        for (int j = 0; j < n; ++j) P.rows[(size_t)v * n + j] = (uint16_t)c->A[(size_t)(r + v) * n + j];
    for (int w = 0; w < kMaxWords; ++w) {
        uint32_t lo = 0, hi = 0;
        if (2 * w < p.nv) lo = (uint32_t)std::min<int32_t>(c->d[r + 2 * w], 65535);
        if (2 * w + 1 < p.nv) hi = (uint32_t)std::min<int32_t>(c->d[r + 2 * w + 1], 65535);
        p.dpk[w] = lo | (hi << 16);
    }
    // Half records carry the packed rows (W words) or one fingerprint word;
    // fingerprint matches are candidates that the joins check exactly.
    if (o.row_fingerprint < 0 || o.row_fingerprint > 2) return MSP_E_INVALID;
    p.fp = o.row_fingerprint == 2 ? 0 : o.row_fingerprint == 1 ? (p.W >= 1) : (p.W >= 2);
    p.Wr = p.fp ? 1 : p.W;
    p.hd = 0;
    for (int v = 0; v < p.nv; ++v) p.hd += kFpMul[v] * (uint32_t)c->d[r + v];
    for (int x = 0; x < 4; ++x) {
        p.qv[x] = nullptr;
        p.qkh[x] = nullptr;
    }

    // Residue modulus M and cells T.  Exact buckets when M can exceed K_d
    // cheaply (small keys, e.g. one key row); else buckets of ~1K records.
    int lgKd = 0;                                   // bits of K_d + 1
    while (lgKd < 127 && ((u128)1 << lgKd) < kd + 1) ++lgKd;
    P.key_bits = lgKd;
    int log2M, log2T;
    if (o.log2_m) {
        log2M = o.log2_m;
    } else if (lgKd <= 16) {
        log2M = std::max(lgKd, 1);
    } else {
        log2M = std::max(p.qa + p.qb - 10, 1);
    }
    // Records keep key >> log2M in the bits above the two quarter positions,
    // and with a second key word (p.wide) in 32 more bits of the record.
    // The planner takes the second word for keys past int64, and when the
    // header alone would force the modulus up (more cells than the quarters
    // have inner elements, each outer element yielding a record or two):
    // 4 more bytes per record against a much slower enumeration.
    p.hsh = p.qa + p.qb;
    {
        const int room1 = 64 - p.hsh;
        const int room2 = std::min(64, room1 + 32);
        int words = o.key_words;
        if (!words)
            words = (p.kw || lgKd - log2M > room1) && o.row_fingerprint != 2 ? 2 : 1;
        if (words == 1 && p.kw) return MSP_E_KEY_OVERFLOW;
        if (words == 2 && o.row_fingerprint == 2) return MSP_E_UNSUPPORTED;
        p.wide = words == 2 ? 1 : 0;
        const int need = lgKd - (p.wide ? room2 : room1);   // smallest log2M that fits
        if (log2M < need) {
            if (o.log2_m) return MSP_E_INVALID;
            log2M = need;
        }
    }
    if (p.wide) {                                   // fingerprint + second key word
        p.fp = 1;
        p.Wr = 2;
    }
    p.exact = (!p.kw && ((uint64_t)1 << std::min(log2M, 62)) > (uint64_t)p.Kd) ? 1 : 0;
    if (o.log2_cells) {
        log2T = o.log2_cells;
    } else {
        // |B_j| ~ 8 pairs per outer element, and at most 1024 fine buckets
        // per cell (the staged scatter's LDS budget).
        log2T = std::max(p.qb - 3, 0);
        log2T = std::max(log2T, log2M - 10);
        // A large M forced by the key room (many key rows) would give more
        // cells than inner elements; every cell re-reads the outer quarter,
        // so take the most fine buckets per cell instead (measured at
        // (8,70) with five key rows: 2^18 cells 4.7 s, 2^20 cells 8.8 s).
        if (log2T > p.qb + 1) log2T = std::max(p.qb + 1, log2M - 12);
        if (log2T > 23) log2T = std::max(23, log2M - 12);   // cell tables <= 2^23
    }
    log2T = std::min(log2T, log2M);
    if (log2M - log2T > 12) return MSP_E_INVALID;       // fine buckets per cell <= 4096
    if (log2T > kMaxCellBits) return MSP_E_UNSUPPORTED;
    // More cells than the equal quarters have inner elements (a modulus
    // forced up by the key room: n near 100, five key rows at n = 90): the
    // planner moves variables to the inner quarters until a cell holds about
    // one inner element, so the outer quarter is not re-read for every one or
    // two records (measured at (10,90), four key rows: 2^23 cells, q_B 22 ->
    // 23, count and scatter 3.2 -> 2.2 s per 1/512 slice).
    if (!o.log2_outer && log2T > p.qb) {
        const int s = std::min({log2T - p.qb, kMaxQuarterBits - p.qb, p.qc - 1, p.qa - 1});
        if (s > 0) {
            p.qa -= s; p.qb += s; p.qc -= s; p.qd += s;
            p.Q[0] = 1u << p.qa; p.Q[1] = 1u << p.qb; p.Q[2] = 1u << p.qc; p.Q[3] = 1u << p.qd;
        }
    }
    p.log2M = log2M; p.log2T = log2T; p.log2F = log2M - log2T;
    p.khb = std::max(0, lgKd - log2M);
    p.slice_mod = o.slice_mod;
    p.slice_res = o.slice_res;
    if (o.join_variant < 0 || o.join_variant > 3) return MSP_E_INVALID;
    if (o.join_variant) {
        p.join_grouped = o.join_variant == 3 ? 2 : o.join_variant == 2 ? 1 : 0;
    } else {
        // From groups of about six the grouped join is faster than the
        // chains (measured: ~1 chains, >= 17 groups).
        p.join_grouped = expected_group_lg2(c, p) >= std::log2(6.0) ? 1 : 0;
        // A few dozen records per bucket and side (a modulus forced up by the
        // key room): one wavefront per bucket.
        const uint64_t per_bucket =
            std::max((uint64_t)p.Q[0] * p.Q[1], (uint64_t)p.Q[2] * p.Q[3]) >> std::min(log2M, 62);
        if (!p.exact && per_bucket <= 48) p.join_grouped = 2;
    }
    // Deciding equal-key runs: the vector join (Algorithms 3-4: one table
    // probe per record) against the pairwise check (|G_L| |G_R| compares).
    // The planner takes the vector join when the expected equal-key group
    // holds 16 or more records per side (hundreds of pairs per run).
    // Buckets of more than about a thousand records per side (a smaller
    // modulus): the grouped join's 1024-thread variant, up to 4096 records.
    {
        const uint64_t per_bucket =
            std::max((uint64_t)p.Q[0] * p.Q[1], (uint64_t)p.Q[2] * p.Q[3]) >> std::min(log2M, 62);
        p.gbig = 0;
        if (!p.exact && per_bucket > 1100) p.gbig = 1;
    }
    if (o.verify_join < 0 || o.verify_join > 2) return MSP_E_INVALID;
    if (o.first_order < 0 || o.first_order > 1) return MSP_E_INVALID;
    if (o.verify_join == 1) p.vjoin = 1;
    else if (o.verify_join == 2) p.vjoin = 0;
    // Planner's choice: the pairwise walk of a group costs about one compare
    // per left record against the vector join's fixed probe, and is still
    // the faster at groups of ~23 records ((9,80) with four key rows); from
    // 32 records per group the vector join decides the runs.
    else p.vjoin = expected_group_lg2(c, p) >= 5.0 ? 1 : 0;
    if (p.W == 0) p.vjoin = 0;
    const uint64_t T = (uint64_t)1 << log2T;
    if (o.slice_mod > 0) {
        p.kstep = (int64_t)std::min<uint64_t>((uint64_t)o.slice_mod, T);
        p.kfirst = o.slice_res & (p.kstep - 1);
    } else {
        p.kstep = 1;
        p.kfirst = 0;
    }
    Sizes &z = P.z;
    z.ncells = T / (uint64_t)p.kstep;

    // Window: enough cells that one launch fills the chip, bounded by memory.
    // Records per cell: at most Q_A*Q_B over all T cells; a slice finer
    // than the cells keeps only 1/(slice_mod/T) of a cell.
    const uint64_t all_rec = std::max((uint64_t)p.Q[0] * p.Q[1], (uint64_t)p.Q[2] * p.Q[3]);
    const uint64_t thin = (o.slice_mod > 0 && (uint64_t)o.slice_mod > T) ? (uint64_t)o.slice_mod / T : 1;
    const uint64_t est_cell = std::max<uint64_t>(1, all_rec / T / thin);
    const uint64_t rb = rec_bytes(p.Wr), qb = qrec_bytes(p.Wr);
    const uint64_t qvb = p.fp ? 4ull * p.W : 0;     // packed rows per quarter subset (fp)
    const int F = 1 << p.log2F;
    z.sol_cap = o.max_solutions ? o.max_solutions : ((uint64_t)1 << 20);
    // A window that covers every cell needs at most Q_A*Q_B records per
    // side (each pair lands in exactly one cell); smaller windows get a 25%
    // margin per cell, and the count pass checks the real totals anyway.
    const uint64_t hard_cap = ((uint64_t)1 << 31) - 1;
    const uint64_t per_cell = est_cell + est_cell / 4 + 1;
    uint64_t want = o.window_records ? o.window_records : ((uint64_t)1 << 30);
    want = std::min(std::max<uint64_t>(want, per_cell + 1024), hard_cap);
    uint64_t kwin;
    if (std::min(all_rec, z.ncells * per_cell) <= want && !o.window_records) {
        kwin = z.ncells;
    } else {
        kwin = std::max<uint64_t>(1, std::min<uint64_t>(z.ncells, want / per_cell));
    }
    // At most 2^23 buckets per window: the grouped join launches one
    // work-group of 256 lanes per bucket, and a HIP grid holds fewer than
    // 2^32 lanes.  Only a large modulus (many key rows) reaches this.
    kwin = std::min<uint64_t>(kwin, std::max<uint64_t>(1, ((uint64_t)1 << 23) >> p.log2F));
    int parts = o.parts;
    if (!parts) {
        const uint64_t target = 8192;            // work-groups per launch (tuned: 4x fill)
        parts = (int)std::min<uint64_t>(64, std::max<uint64_t>(1, (target + kwin - 1) / kwin));
        parts = (int)std::min<uint64_t>(parts, std::max<uint64_t>(1, p.Q[0] / 256));
        parts = (int)std::min<uint64_t>(parts, std::max<uint64_t>(1, p.Q[2] / 256));
    }
    // When the inner quarter lists outgrow one XCD's L2 (4 MB), parts come in
    // multiples of 8: the count and scatter kernels then give each XCD whole
    // parts, whose inner partners are a contiguous slice of the list.
    if (!o.parts && (uint64_t)std::max(p.Q[1], p.Q[3]) * qb > ((uint64_t)4 << 20))
        parts = std::max(8, (parts + 7) & ~7);
    p.parts = parts;
    // Launch limits: every grid whose size the plan fixes stays below 2^32
    // work-items (the launchers check again before each launch).
    while (kwin > 1 && plan_max_items(p, kwin) > kMaxLaunchItems) kwin = (kwin + 1) / 2;
    if (plan_max_items(p, kwin) > kMaxLaunchItems) return MSP_E_UNSUPPORTED;
    auto layout = [&](uint64_t cap_rec, uint64_t kw) -> uint64_t {
        uint64_t off = 0;
        auto take = [&](uint64_t bytes) { uint64_t o2 = off; off += align_up(bytes, 256); return o2; };
        for (int x = 0; x < 4; ++x) z.o_qraw[x] = take((uint64_t)p.Q[x] * qb);
        for (int x = 0; x < 4; ++x) z.o_qsrt[x] = take((uint64_t)p.Q[x] * qb);
        for (int x = 0; x < 4; ++x) z.o_qvraw[x] = take((uint64_t)p.Q[x] * qvb + 4);
        for (int x = 0; x < 4; ++x) z.o_qvsrt[x] = take((uint64_t)p.Q[x] * qvb + 4);
        for (int x = 0; x < 4; ++x) z.o_qkhraw[x] = take(p.kw ? (uint64_t)p.Q[x] * 8 : 8);
        for (int x = 0; x < 4; ++x) z.o_qkhsrt[x] = take(p.kw ? (uint64_t)p.Q[x] * 8 : 8);
        for (int x = 0; x < 4; ++x) z.o_qcnt[x] = take((T + 1) * 4);
        for (int x = 0; x < 4; ++x) z.o_qcur[x] = take((T + 1) * 4);
        const uint64_t ncnt = kw * F * (uint64_t)parts + 1;
        for (int s = 0; s < 2; ++s) z.o_cnt[s] = take(ncnt * 4);
        for (int s = 0; s < 2; ++s) z.o_off[s] = take((kw * F + 1) * 4);
        for (int s = 0; s < 2; ++s) z.o_pre[s] = take(ncnt * 4);
        for (int s = 0; s < 2; ++s) z.o_tot[s] = take((kw * F + 1) * 4);
        for (int s = 0; s < 2; ++s) z.o_rec[s] = take(cap_rec * rb);
        z.o_runs = take(kw * F * sizeof(RunPair));
        z.o_tiles = take((kw * F + 1) * 4);
        // Large equal-key groups exported by the hash join as index lists.
        // A left chunk exports each record at most once and each right
        // record once per left chunk; sized for three records' worth per
        // record (buckets of up to two left chunks).  The join checks both
        // capacities on the device and verifies in place what does not fit.
        // Each group has >= kBigPairs pairs, hence >= 128 records.
        const uint64_t idx_n = p.exact ? 1 : 3 * cap_rec;
        const uint64_t nI = p.exact ? 1 : idx_n / 128 + 1024;
        z.n_iruns = nI;
        z.idx_n = idx_n;
        z.o_iruns = take(nI * sizeof(RunPair));
        z.o_itiles = take((nI + 1) * 4);
        z.o_idx = take(idx_n * 4);
        z.o_heavy = take(p.exact ? 4 : kw * F * 4);
        z.o_heavy2 = take(p.exact ? 4 : kw * F * 4);
        // Vector join table: at most half full, so every probe ends.
        z.vtab_slots = 1;
        if (p.vjoin && p.exact)
            while (z.vtab_slots < 2 * cap_rec) z.vtab_slots <<= 1;
        z.o_vtab = take(z.vtab_slots * 4);
        z.o_wscore = take(((z.ncells + kw - 1) / kw) * 8 + 8);
        z.o_sol = take(z.sol_cap * 16);
        z.o_scal = take(S_COUNT * 8);
        z.scan_bytes = scan_tmp_bytes(std::max<uint64_t>(std::max<uint64_t>(T + 1, ncnt),
                                                         std::max<uint64_t>(kw * F + 1, nI + 1)));
        z.o_scan = take(z.scan_bytes);
        z.o_colw = take((uint64_t)n * 8);
        z.o_colwh = take((uint64_t)n * 8);
        z.o_rows = take(P.rows.size() * 2);
        return off;
    };
    // The caller's window_records is also a floor on the buffers: a window
    // of one cell can still hold a class far denser than the average cell.
    auto cap_for = [&](uint64_t kw) {
        return std::min<uint64_t>(
            hard_cap, std::min<uint64_t>(all_rec, std::max<uint64_t>(kw * per_cell + 1024,
                                                                     o.window_records)));
    };
    uint64_t cap_rec = cap_for(kwin);
    uint64_t total = layout(cap_rec, kwin);
    if (budget) {
        while (total > budget && kwin > 1) {
            kwin = (kwin + 1) / 2;
            cap_rec = cap_for(kwin);
            total = layout(cap_rec, kwin);
        }
        if (total > budget) return MSP_E_NOMEM;
    }
    z.kwin = kwin;
    z.cap_rec = cap_rec;
    z.total = total;
    z.max_items = plan_max_items(p, kwin);
    return MSP_OK;
}

double ev_ms(hipEvent_t a, hipEvent_t b) {
    if (!a || !b) return 0.0;                 // a solve without timing events
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
    return (double)ms;
}

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------------------
// Device memory arena for batched / served solves: one allocation, first-fit
// ranges, adjacent free ranges merged.  Host-side bookkeeping only.
// ---------------------------------------------------------------------------
struct Arena {
    char *base = nullptr;
    DevMem mem;
    uint64_t size = 0;
    std::map<uint64_t, uint64_t> free_;      // offset -> length
    bool init(uint64_t bytes) {
        mem = dev_alloc(bytes);
        base = (char *)mem.ptr;
        if (!base) return false;
        size = bytes;
        free_.clear();
        free_[0] = bytes;
        return true;
    }
    void release_all() {
        dev_free(mem);
        base = nullptr;
        free_.clear();
    }
    char *alloc(uint64_t bytes) {
        bytes = (bytes + 4095) & ~(uint64_t)4095;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const uint64_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > bytes) free_[off + bytes] = len - bytes;
                return base + off;
            }
        }
        return nullptr;
    }
    void free(char *p, uint64_t bytes) {
        bytes = (bytes + 4095) & ~(uint64_t)4095;
        uint64_t off = (uint64_t)(p - base);
        auto nx = free_.lower_bound(off);
        if (nx != free_.end() && off + bytes == nx->first) {
            bytes += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) {
                pv->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }
};

// ---------------------------------------------------------------------------
// A solve in progress.  Each call of step() enqueues the next group of
// kernels on the job's stream; the runner synchronises all jobs between
// calls, so concurrent jobs overlap on the device.
// ---------------------------------------------------------------------------
enum Action { A_BEGIN, A_ORDER, A_COUNTED, A_JOINED, A_TILED, A_FINAL1, A_FINAL2, A_DONE };
enum Ev { E_Q0, E_Q1, E_C0, E_C1, E_C2, E_S0, E_S1, E_S2, E_V0, E_V1, E_COUNT };

struct Job {
    msp_ctx *c = nullptr;
    msp_opts o{};
    Prepared P;
    DevBufs b{};
    char *ws = nullptr;
    uint64_t ws_bytes = 0;
    bool arena_ws = false;
    hipStream_t s = nullptr;
    hipEvent_t ev[E_COUNT] = {};
    uint64_t *hs = nullptr;              // host copy of the device scalars (pinned, or
                                         // the context's own array without events)
    bool hs_pinned = false;
    Action next = A_BEGIN;
    uint64_t idx = 0, kw = 0, K = 0;
    // First-solution mode in density order: planned windows (start cells)
    // in processing order, the current one's cell range, and cells done.
    bool ordered = false;
    std::vector<uint64_t> order;
    std::vector<uint64_t> scores;
    size_t oi = 0;
    uint64_t win_hi = 0, cells_done = 0;
    bool verify_pending = false;
    std::vector<uint64_t> solbuf;
    msp_stats_t st{};
    int rc = MSP_OK;
    // Server stamps, seconds since server start.  t_finish is published
    // under the server mutex (last, once the context is free again); the
    // scheduler thread keeps its own end time in t_retired.
    double t_submit = 0, t_admit = 0, t_start = 0, t_finish = 0, t_wall0 = 0, t_retired = 0;
    uint64_t ticket = 0;
    bool cancel = false;
    bool inflight = false;               // work enqueued by the last job_step not yet checked
    int slot = -1;                       // runner stream slot
};

// Phase events are recorded only when the job has them (the no-allocation
// entry point runs without).
hipError_t ev_rec(Job &j, int e) { return j.ev[e] ? hipEventRecord(j.ev[e], j.s) : hipSuccess; }

int job_setup_events(Job &j) {
    for (auto &e : j.ev)
        if (!e && hipEventCreate(&e) != hipSuccess) return MSP_E_DEVICE;
    if (!j.hs) {
        if (hipHostMalloc((void **)&j.hs, S_COUNT * 8, hipHostMallocDefault) != hipSuccess) {
            j.hs = nullptr;
            return MSP_E_DEVICE;
        }
        j.hs_pinned = true;
    }
    return MSP_OK;
}

void job_release_events(Job &j) {
    for (auto &e : j.ev)
        if (e) (void)hipEventDestroy(e), e = nullptr;
    if (j.hs && j.hs_pinned) (void)hipHostFree(j.hs);
    j.hs = nullptr;
    j.hs_pinned = false;
}

void job_carve(Job &j) {
    const Sizes &z = j.P.z;
    char *ws = j.ws;
    for (int x = 0; x < 4; ++x) {
        j.b.qraw[x] = ws + z.o_qraw[x];
        j.b.qsrt[x] = ws + z.o_qsrt[x];
        j.b.qcnt[x] = (uint32_t *)(ws + z.o_qcnt[x]);
        j.b.qcur[x] = (uint32_t *)(ws + z.o_qcur[x]);
        j.b.qvraw[x] = (uint32_t *)(ws + z.o_qvraw[x]);
        j.b.qvsrt[x] = (uint32_t *)(ws + z.o_qvsrt[x]);
        j.P.p.qv[x] = j.P.p.fp ? j.b.qvsrt[x] : nullptr;
        j.b.qkhraw[x] = (int64_t *)(ws + z.o_qkhraw[x]);
        j.b.qkhsrt[x] = (int64_t *)(ws + z.o_qkhsrt[x]);
        j.P.p.qkh[x] = j.P.p.kw ? j.b.qkhsrt[x] : nullptr;
    }
    for (int sd = 0; sd < 2; ++sd) {
        j.b.cnt[sd] = (uint32_t *)(ws + z.o_cnt[sd]);
        j.b.off[sd] = (uint32_t *)(ws + z.o_off[sd]);
        j.b.pre[sd] = (uint32_t *)(ws + z.o_pre[sd]);
        j.b.tot[sd] = (uint32_t *)(ws + z.o_tot[sd]);
        j.b.rec[sd] = ws + z.o_rec[sd];
    }
    j.b.runs = (RunPair *)(ws + z.o_runs);
    j.b.tiles = (uint32_t *)(ws + z.o_tiles);
    j.b.iruns = (RunPair *)(ws + z.o_iruns);
    j.b.itiles = (uint32_t *)(ws + z.o_itiles);
    j.b.idx = (uint32_t *)(ws + z.o_idx);
    j.b.heavy = (uint32_t *)(ws + z.o_heavy);
    j.b.heavy2 = (uint32_t *)(ws + z.o_heavy2);
    j.b.vtab = (uint32_t *)(ws + z.o_vtab);
    j.b.vtab_mask = (uint32_t)(z.vtab_slots - 1);
    j.b.iruns_cap = z.n_iruns;
    j.b.idx_cap = z.idx_n;
    j.b.sol = (uint64_t *)(ws + z.o_sol);
    j.b.wscore = (uint64_t *)(ws + z.o_wscore);
    j.b.scal = (uint64_t *)(ws + z.o_scal);
    j.b.scan_tmp = ws + z.o_scan;
    j.b.scan_tmp_bytes = z.scan_bytes;
    j.b.colw = (int64_t *)(ws + z.o_colw);
    j.b.colwh = (int64_t *)(ws + z.o_colwh);
    j.b.rows = (uint16_t *)(ws + z.o_rows);
}

// A HIP error poisons the solve (MSP_E_DEVICE), except a grid the launchers
// refused before enqueueing it: that plan is beyond the device's launch
// limits (MSP_E_UNSUPPORTED) and nothing ran.
#define JCHK(x)                                                                       \
    do {                                                                              \
        const hipError_t e_ = (x);                                                    \
        if (e_ != hipSuccess) {                                                       \
            (void)hipGetLastError();                                                  \
            return e_ == hipErrorInvalidConfiguration ? MSP_E_UNSUPPORTED : MSP_E_DEVICE; \
        }                                                                             \
    } while (0)

int enqueue_count(Job &j) {
    const Plan &p = j.P.p;
    JCHK(ev_rec(j, E_C0));
    JCHK(launch_count(p, j.b, (int64_t)j.idx, (int32_t)j.K, j.s));
    JCHK(ev_rec(j, E_C1));
    const uint32_t F = 1u << p.log2F, P = (uint32_t)p.parts;
    const uint64_t nbk = (uint64_t)j.K << p.log2F;
    for (int sd = 0; sd < 2; ++sd)
        JCHK(scan_counts(j.b.cnt[sd], j.b.pre[sd], j.b.tot[sd], j.b.off[sd], nbk, F, P,
                         &j.b.scal[sd ? S_TOT_R : S_TOT_L], &j.b.scal[S_OVF], j.b.scan_tmp,
                         j.b.scan_tmp_bytes, j.s));
    JCHK(ev_rec(j, E_C2));
    JCHK(hipMemcpyAsync(j.hs, j.b.scal, S_COUNT * 8, hipMemcpyDeviceToHost, j.s));
    return MSP_OK;
}

// Run the job's next action.  Everything it enqueues is complete when the
// runner calls step() again.
int job_step(Job &j) {
    const Plan &p = j.P.p;
    const Sizes &z = j.P.z;
    switch (j.next) {
        case A_BEGIN: {
            const uint64_t T = (uint64_t)1 << p.log2T;
            JCHK(hipMemcpyAsync(j.b.colw, j.P.colw.data(), j.P.colw.size() * 8, hipMemcpyHostToDevice, j.s));
            JCHK(hipMemcpyAsync(j.b.colwh, j.P.colwh.data(), j.P.colwh.size() * 8, hipMemcpyHostToDevice, j.s));
            JCHK(hipMemcpyAsync(j.b.rows, j.P.rows.data(), j.P.rows.size() * 2, hipMemcpyHostToDevice, j.s));
            JCHK(hipMemsetAsync(j.b.scal, 0, S_COUNT * 8, j.s));
            for (int x = 0; x < 4; ++x) JCHK(hipMemsetAsync(j.b.qcnt[x], 0, (T + 1) * 4, j.s));
            JCHK(ev_rec(j, E_Q0));
            JCHK(launch_quarters(p, j.b, 0, j.s));
            JCHK(ev_rec(j, E_Q1));
            j.kw = z.kwin;
            j.cells_done = 0;
            const uint64_t nwin = (z.ncells + z.kwin - 1) / z.kwin;
            if (j.o.first_only && j.o.first_order == 0 && nwin > 1) {
                // Algorithm 2 stops at the first solution; windows are taken
                // in order of their count of candidate pairs (sum over
                // buckets of left x right records; for buckets of one key
                // value that is the window's number of 1-D hits), so the
                // densest windows come first.  One count pass over every
                // window gives the scores.
                j.ordered = true;
                JCHK(hipMemsetAsync(j.b.wscore, 0, nwin * 8, j.s));
                for (uint64_t w = 0; w < nwin; ++w) {
                    j.idx = w * z.kwin;
                    j.K = std::min<uint64_t>(z.kwin, z.ncells - j.idx);
                    JCHK(launch_count(p, j.b, (int64_t)j.idx, (int32_t)j.K, j.s));
                    const uint64_t nbk = j.K << p.log2F;
                    for (int sd = 0; sd < 2; ++sd)
                        JCHK(scan_counts(j.b.cnt[sd], j.b.pre[sd], j.b.tot[sd], j.b.off[sd], nbk,
                                         1u << p.log2F, (uint32_t)p.parts, nullptr,
                                         &j.b.scal[S_OVF], j.b.scan_tmp, j.b.scan_tmp_bytes, j.s));
                    JCHK(launch_window_score(j.b, nbk, j.b.wscore + w, j.s));
                }
                j.scores.assign(nwin, 0);
                JCHK(hipMemcpyAsync(j.scores.data(), j.b.wscore, nwin * 8, hipMemcpyDeviceToHost,
                                    j.s));
                j.next = A_ORDER;
                return MSP_OK;
            }
            j.idx = 0;
            j.win_hi = z.ncells;
            j.K = std::min<uint64_t>(j.kw, z.ncells - j.idx);
            int rc = enqueue_count(j);
            if (rc) return rc;
            j.next = A_COUNTED;
            return MSP_OK;
        }
        case A_ORDER: {
            const uint64_t nwin = j.scores.size();
            j.order.resize(nwin);
            std::iota(j.order.begin(), j.order.end(), (uint64_t)0);
            std::stable_sort(j.order.begin(), j.order.end(),
                             [&](uint64_t a, uint64_t bb) { return j.scores[a] > j.scores[bb]; });
            j.oi = 0;
            j.idx = j.order[0] * z.kwin;
            j.win_hi = std::min<uint64_t>(j.idx + z.kwin, z.ncells);
            j.K = j.win_hi - j.idx;
            int rc = enqueue_count(j);
            if (rc) return rc;
            j.next = A_COUNTED;
            return MSP_OK;
        }
        case A_COUNTED: {
            if (j.st.ms_quarters == 0.0) j.st.ms_quarters = ev_ms(j.ev[E_Q0], j.ev[E_Q1]);
            if (j.verify_pending) {
                j.st.ms_verify += ev_ms(j.ev[E_V0], j.ev[E_V1]);
                j.verify_pending = false;
            }
            j.st.ms_count += ev_ms(j.ev[E_C0], j.ev[E_C1]);
            j.st.ms_scan += ev_ms(j.ev[E_C1], j.ev[E_C2]);
            // First-solution mode: the scalars copied with this count already
            // include every earlier window's verify.
            if (j.o.first_only && j.hs[S_NSOL] > 0) {
                JCHK(hipMemcpyAsync(j.hs, j.b.scal, S_COUNT * 8, hipMemcpyDeviceToHost, j.s));
                j.next = A_FINAL1;
                return MSP_OK;
            }
            // A work-group whose 32-bit bucket counters could wrap, or a
            // bucket of 2^32 or more records: no window split helps (one
            // bucket cannot be divided), so the solve does not fit.
            if (j.hs[S_OVF] & 5) return MSP_E_NOMEM;
            // Window totals are exact 64-bit sums; the scatter runs only when
            // both fit the record buffers (offsets are 32-bit below cap_rec).
            const uint64_t totL = j.hs[S_TOT_L], totR = j.hs[S_TOT_R];
            if (totL > z.cap_rec || totR > z.cap_rec) {
                if (j.K == 1) return MSP_E_NOMEM;
                j.K = (j.K + 1) / 2;
                j.kw = j.K;
                int rc = enqueue_count(j);
                if (rc) return rc;
                return MSP_OK;                  // next stays A_COUNTED
            }
            j.st.records_left += totL;
            j.st.records_right += totR;
            JCHK(hipMemsetAsync(&j.b.scal[S_NRUNS], 0, 8, j.s));
            JCHK(hipMemsetAsync(&j.b.scal[S_NIRUNS], 0, 5 * 8, j.s));   // NIRUNS .. NHEAVY2
            JCHK(ev_rec(j, E_S0));
            JCHK(launch_scatter(p, j.b, (int64_t)j.idx, (int32_t)j.K, j.s));
            JCHK(ev_rec(j, E_S1));
            if (p.exact)
                JCHK(launch_exact_runs(p, j.b, (int32_t)j.K, j.s));
            else
                JCHK(launch_hash_join(p, j.b, (int32_t)j.K, z.sol_cap, j.s));
            JCHK(ev_rec(j, E_S2));
            JCHK(hipMemcpyAsync(j.hs, j.b.scal, S_COUNT * 8, hipMemcpyDeviceToHost, j.s));
            j.next = A_JOINED;
            return MSP_OK;
        }
        case A_JOINED:
        case A_TILED: {
            const uint32_t nruns = (uint32_t)j.hs[S_NRUNS];
            // Reservations past the capacity were not written (see k_join_heavy).
            const uint32_t niruns = (uint32_t)std::min<uint64_t>(j.hs[S_NIRUNS], z.n_iruns);
            if (j.next == A_JOINED) {
                j.st.ms_scatter += ev_ms(j.ev[E_S0], j.ev[E_S1]);
                j.st.ms_join += ev_ms(j.ev[E_S1], j.ev[E_S2]);
                if (p.vjoin && p.exact && nruns) {
                    // Exact runs: one hash join on the packed rows decides them all.
                    JCHK(ev_rec(j, E_V0));
                    JCHK(launch_vector_join(p, j.b, nruns, z.sol_cap, j.s));
                    JCHK(ev_rec(j, E_V1));
                    j.verify_pending = true;
                    j.st.verify_launches += 1;
                } else if (nruns || niruns) {
                    if (nruns) {
                        JCHK(launch_tile_counts(p, j.b, nruns, p.exact ? 0 : 1, j.s));
                        JCHK(scan_u32(j.b.tiles, j.b.tiles, nruns, &j.b.scal[S_TOT_TILES],
                                      j.b.scan_tmp, j.b.scan_tmp_bytes, j.s));
                    }
                    if (niruns) {
                        JCHK(launch_tile_counts(p, j.b, niruns, 2, j.s));
                        JCHK(scan_u32(j.b.itiles, j.b.itiles, niruns, &j.b.scal[S_TOT_ITILES],
                                      j.b.scan_tmp, j.b.scan_tmp_bytes, j.s));
                    }
                    JCHK(hipMemcpyAsync(j.hs, j.b.scal, S_COUNT * 8, hipMemcpyDeviceToHost, j.s));
                    j.next = A_TILED;
                    return MSP_OK;
                }
            } else {
                // Tile totals are exact 64-bit sums; offsets are 32-bit.
                if ((j.hs[S_OVF] & 2) || j.hs[S_TOT_TILES] > 0xFFFFFFFFull ||
                    j.hs[S_TOT_ITILES] > 0xFFFFFFFFull)
                    return MSP_E_UNSUPPORTED;
                JCHK(ev_rec(j, E_V0));
                if (nruns)
                    JCHK(launch_verify(p, j.b, nruns, (uint32_t)j.hs[S_TOT_TILES], z.sol_cap,
                                       p.exact ? 0 : 1, j.s));
                if (niruns)
                    JCHK(launch_verify(p, j.b, niruns, (uint32_t)j.hs[S_TOT_ITILES], z.sol_cap, 2,
                                       j.s));
                JCHK(ev_rec(j, E_V1));
                j.verify_pending = true;
                j.st.verify_launches += (nruns ? 1 : 0) + (niruns ? 1 : 0);
            }
            // Window done; move to the next one or finish.
            j.st.windows++;
            j.cells_done += j.K;
            j.idx += j.K;
            bool more;
            if (j.ordered) {
                if (j.idx >= j.win_hi && ++j.oi < j.order.size()) {   // next planned window
                    j.idx = j.order[j.oi] * z.kwin;
                    j.win_hi = std::min<uint64_t>(j.idx + z.kwin, z.ncells);
                    j.kw = z.kwin;
                }
                more = j.oi < j.order.size();
            } else {
                more = j.idx < z.ncells;
            }
            if (more && !j.cancel) {
                j.K = std::min<uint64_t>(j.kw, j.win_hi - j.idx);
                int rc = enqueue_count(j);
                if (rc) return rc;
                j.next = A_COUNTED;
            } else {
                JCHK(hipMemcpyAsync(j.hs, j.b.scal, S_COUNT * 8, hipMemcpyDeviceToHost, j.s));
                j.next = A_FINAL1;
            }
            return MSP_OK;
        }
        case A_FINAL1: {
            if (j.verify_pending) {
                j.st.ms_verify += ev_ms(j.ev[E_V0], j.ev[E_V1]);
                j.verify_pending = false;
            }
            if (j.cancel) return MSP_E_CANCELLED;
            const uint64_t stored =
                std::min<uint64_t>(z.sol_cap, p.Wr == 0 ? j.hs[S_STORED] : j.hs[S_NSOL]);
            j.solbuf.resize(stored * 2);
            if (stored)
                JCHK(hipMemcpyAsync(j.solbuf.data(), j.b.sol, stored * 16, hipMemcpyDeviceToHost, j.s));
            j.next = A_FINAL2;
            return MSP_OK;
        }
        case A_FINAL2: {
            // Expand half masks to x (left-half columns first) and sort
            // canonically (lexicographic on x_1..x_n, 0 < 1).
            msp_ctx *c = j.c;
            const int n = c->n;
            const uint64_t stored = j.solbuf.size() / 2;
            std::vector<uint8_t> xs(stored * n);
            for (uint64_t k = 0; k < stored; ++k) {
                const uint64_t ml = j.solbuf[2 * k], mr = j.solbuf[2 * k + 1];
                for (int jj = 0; jj < n; ++jj)
                    xs[k * n + jj] = (uint8_t)(jj < p.hL ? (ml >> jj) & 1u : (mr >> (jj - p.hL)) & 1u);
            }
            std::vector<uint64_t> ord(stored);
            std::iota(ord.begin(), ord.end(), 0);
            std::sort(ord.begin(), ord.end(), [&](uint64_t a, uint64_t bb) {
                return std::memcmp(&xs[a * n], &xs[bb * n], n) < 0;
            });
            c->sol.resize(stored * n);
            for (uint64_t k = 0; k < stored; ++k) std::memcpy(&c->sol[k * n], &xs[ord[k] * n], n);
            c->stored = stored;
            c->h_lo = j.hs[S_H_LO];
            c->h_hi = j.hs[S_H_HI];
            c->nsol = j.hs[S_NSOL];
            j.st.complete = j.cells_done >= z.ncells ? 1 : 0;
            j.st.cells_done = j.cells_done;
            j.st.window_order = j.ordered ? 1 : 0;
            j.st.first_cell = j.ordered && !j.order.empty() ? j.order[0] * z.kwin : 0;
            j.st.ms_total = (now_s() - j.t_wall0) * 1e3;
            c->stats = j.st;
            c->have_result = true;
            j.next = A_DONE;
            return MSP_OK;
        }
        case A_DONE:
            return MSP_OK;
    }
    return MSP_OK;
}

// Results of a solve that needs no GPU work (a key row can never hold).
void job_trivial(Job &j) {
    msp_ctx *c = j.c;
    c->h_lo = c->h_hi = c->nsol = 0;
    c->sol.clear();
    c->stored = 0;
    j.st.ms_total = (now_s() - j.t_wall0) * 1e3;
    c->stats = j.st;
    c->have_result = true;
    j.next = A_DONE;
}

void job_init_stats(Job &j) {
    const Plan &p = j.P.p;
    j.st = msp_stats_t{};
    j.st.key_rows = p.r;
    j.st.log2_m = p.log2M;
    j.st.log2_cells = p.log2T;
    j.st.parts = p.parts;
    j.st.exact_buckets = p.exact;
    j.st.words = p.W;
    j.st.record_bytes = rec_bytes(p.Wr);
    j.st.row_fingerprint = p.fp;
    j.st.log2_outer = p.qa;
    j.st.key_words = p.wide ? 2 : 1;
    j.st.key_bits = j.P.key_bits;
    j.st.vector_join = p.vjoin;
    j.st.join_grouped = p.exact ? 0 : p.join_grouped;
    j.st.key_base = j.o.key_base;
    j.st.complete = 1;
    j.st.cells_done = j.P.z.ncells;
    j.st.windows_total = (j.P.z.ncells + j.P.z.kwin - 1) / std::max<uint64_t>(j.P.z.kwin, 1);
}

// ---------------------------------------------------------------------------
// Runner: drives a set of jobs; admission by device-memory footprint.
// ---------------------------------------------------------------------------
struct Runner {
    Arena arena;
    uint64_t budget = 0;            // bytes for all admitted jobs together
    int max_slots = 16;
    std::vector<hipStream_t> streams;
    std::vector<int> stream_free;
    std::deque<Job *> pending;
    std::vector<Job *> active;
    double t0 = 0;

    int init(uint64_t hbm_budget, int slots) {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return MSP_E_NOLIB;
        max_slots = slots > 0 ? slots : 16;
        budget = hbm_budget;
        if (!budget) {
            size_t fr = 0, tot = 0;
            if (hipMemGetInfo(&fr, &tot) != hipSuccess) return MSP_E_NOLIB;
            budget = std::min<uint64_t>((uint64_t)(fr * 0.6), (uint64_t)128 << 30);
        }
        if (!arena.init(budget)) return MSP_E_NOMEM;
        streams.resize(max_slots);
        for (int i = 0; i < max_slots; ++i) {
            if (hipStreamCreateWithFlags(&streams[i], hipStreamNonBlocking) != hipSuccess)
                return MSP_E_DEVICE;
            stream_free.push_back(i);
        }
        t0 = now_s();
        return MSP_OK;
    }
    void shutdown() {
        for (auto s : streams)
            if (s) (void)hipStreamSynchronize(s), (void)hipStreamDestroy(s);
        streams.clear();
        arena.release_all();
    }
    // Per-job planning budget: an equal share of the arena per slot.
    uint64_t job_budget() const { return budget / (uint64_t)max_slots; }

    // Plan a job (host only).  Sets j.rc on failure.
    void plan(Job &j) {
        j.t_wall0 = now_s();
        uint64_t jb = job_budget();
        j.rc = prepare(j.c, j.o, jb, j.P);
        if (j.rc == MSP_E_NOMEM) j.rc = prepare(j.c, j.o, budget, j.P);   // alone, it may fit
        if (j.rc == MSP_OK) {
            job_init_stats(j);
            j.ws_bytes = j.P.z.total;
        }
    }

    // Admit pending jobs while a slot and memory are free (FIFO order).
    void admit(std::vector<Job *> &failed) {
        while (!pending.empty() && (int)active.size() < max_slots) {
            Job *j = pending.front();
            if (j->rc == MSP_OK && j->c->busy.load() == 2) j->rc = MSP_E_CANCELLED;
            if (j->rc != MSP_OK) { pending.pop_front(); failed.push_back(j); continue; }
            if (j->P.infeasible) {
                pending.pop_front();
                j->t_admit = j->t_start = now_s() - t0;
                job_trivial(*j);
                j->t_retired = now_s() - t0;
                failed.push_back(j);               // reported as finished (rc OK)
                continue;
            }
            if (j->ws_bytes > budget) { j->rc = MSP_E_NOMEM; pending.pop_front(); failed.push_back(j); continue; }
            char *ws = arena.alloc(j->ws_bytes);
            if (!ws) break;                        // wait for memory to free up
            pending.pop_front();
            j->ws = ws;
            j->arena_ws = true;
            const int si = stream_free.back();
            stream_free.pop_back();
            j->s = streams[si];
            j->slot = si;
            job_carve(*j);
            if (job_setup_events(*j) != MSP_OK) { j->rc = MSP_E_DEVICE; retire(j); failed.push_back(j); continue; }
            j->t_admit = now_s() - t0;
            active.push_back(j);
        }
    }

    void retire(Job *j) {
        if (j->arena_ws && j->ws) arena.free(j->ws, j->ws_bytes);
        j->ws = nullptr;
        if (j->s) {
            (void)hipStreamSynchronize(j->s);
            if (j->slot >= 0) stream_free.push_back(j->slot);
            j->slot = -1;
            j->s = nullptr;
        }
        job_release_events(*j);
        j->t_retired = now_s() - t0;
    }

    // One pass over the active jobs: every job whose stream has drained the
    // work of its last action runs its next action; jobs still busy on the
    // device are skipped, so no job waits for another's kernels.  Finished or
    // failed jobs are returned in `done`.  Returns false when no job could
    // advance (the caller then backs off briefly).
    bool step(std::vector<Job *> &done) {
        bool advanced = false;
        for (Job *j : active) {
            if (j->rc != MSP_OK || j->next == A_DONE) continue;
            if (j->inflight) {
                const hipError_t q = hipStreamQuery(j->s);
                if (q == hipErrorNotReady) continue;
                if (q != hipSuccess) {
                    (void)hipGetLastError();
                    j->rc = MSP_E_DEVICE;
                    continue;
                }
                j->inflight = false;
            }
            if (j->t_start == 0) j->t_start = now_s() - t0;
            const int rc = job_step(*j);
            advanced = true;
            if (rc != MSP_OK) j->rc = rc;
            else if (j->next != A_DONE) j->inflight = true;
        }
        std::vector<Job *> keep;
        for (Job *j : active) {
            if (j->rc != MSP_OK || j->next == A_DONE) {
                retire(j);
                done.push_back(j);
                advanced = true;
            } else {
                keep.push_back(j);
            }
        }
        active.swap(keep);
        return advanced;
    }
};

// Back-off of a scheduler pass in which no job could advance.
void idle_wait() { std::this_thread::sleep_for(std::chrono::microseconds(20)); }

}  // namespace

// ---------------------------------------------------------------------------
// Server: the runner on its own thread; requests join while others run.
// ---------------------------------------------------------------------------
struct msp_server {
    Runner run;
    std::mutex mu;
    std::condition_variable cv, cv_done;
    std::deque<Job *> inbox;
    std::map<uint64_t, Job *> jobs;        // ticket -> job (kept until stop)
    uint64_t next_ticket = 1;
    bool stopping = false;
    std::thread th;
};

static void server_loop(msp_server *sv) {
    std::vector<Job *> done;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv.wait(lk, [&] {
                return sv->stopping || !sv->inbox.empty() || !sv->run.active.empty() ||
                       !sv->run.pending.empty();
            });
            if (sv->stopping && sv->run.active.empty() && sv->inbox.empty() && sv->run.pending.empty())
                break;
            while (!sv->inbox.empty()) {
                sv->run.pending.push_back(sv->inbox.front());
                sv->inbox.pop_front();
            }
            for (Job *j : sv->run.active)
                if (j->c->busy.load() == 2) j->cancel = true;   // cancellation request
        }
        done.clear();
        sv->run.admit(done);
        bool advanced = false;
        if (!sv->run.active.empty()) advanced = sv->run.step(done);
        if (!done.empty()) {
            // Publish: free the context first, then the finish stamp that
            // waiters and pollers read (all under the mutex).
            std::lock_guard<std::mutex> lk(sv->mu);
            for (Job *j : done) {
                j->c->busy.store(0);
                j->t_finish = j->t_retired > 0 ? j->t_retired : now_s() - sv->run.t0;
            }
            sv->cv_done.notify_all();
        }
        if (sv->run.active.empty() && !sv->run.pending.empty() && done.empty()) {
            // The queue head does not fit even with nothing running.
            std::lock_guard<std::mutex> lk(sv->mu);
            Job *j = sv->run.pending.front();
            sv->run.pending.pop_front();
            j->rc = MSP_E_NOMEM;
            j->c->busy.store(0);
            j->t_finish = now_s() - sv->run.t0;
            sv->cv_done.notify_all();
        } else if (!advanced && done.empty() && !sv->run.active.empty()) {
            idle_wait();
        }
    }
}

// ---------------------------------------------------------------------------
// The no-allocation entry point's workspace: one file-scope device array per
// GPU (every device that loads this library holds it until the process
// ends).  Host code never passes the array's name to a kernel or a copy: it
// is a host-side stand-in.  The device address comes from
// hipGetSymbolAddress, once per device with that device current, and only
// that address is used.
// ---------------------------------------------------------------------------
constexpr uint64_t kScratchBytes = MSP_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on each device).
static int scratch_address(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return MSP_E_NOLIB;
    }
    if (dev < 0 || dev >= kMaxDevices) return MSP_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return MSP_E_DEVICE;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return MSP_OK;
}

extern "C" {

const char *msp_strerror(int code) {
    switch (code) {
        case MSP_OK: return "ok";
        case MSP_E_INVALID: return "invalid argument";
        case MSP_E_RANGE: return "a row sum exceeds 65534";
        case MSP_E_KEY_OVERFLOW: return "the 1-D key overflows int64";
        case MSP_E_UNSUPPORTED: return "instance size not supported";
        case MSP_E_NOMEM: return "device workspace does not fit";
        case MSP_E_DEVICE: return "HIP runtime error";
        case MSP_E_CANCELLED: return "cancelled";
        case MSP_E_TRUNCATED: return "buffer smaller than the result";
        case MSP_E_STATE: return "no result available";
        case MSP_E_NOLIB: return "no usable GPU";
        case MSP_E_BUSY: return "context is in use by another solve";
        default: return "unknown error";
    }
}

void msp_default_opts(msp_opts *o) {
    if (o) std::memset(o, 0, sizeof *o);
}

int msp_create(const int32_t *A, const int32_t *d, int32_t m, int32_t n, msp_ctx **out) {
    if (!out) return MSP_E_INVALID;
    *out = nullptr;
    const int rc = validate(A, d, m, n);
    if (rc) return rc;
    msp_ctx *c = new (std::nothrow) msp_ctx();
    if (!c) return MSP_E_NOMEM;
    c->m = m;
    c->n = n;
    c->A.assign(A, A + (size_t)m * n);
    c->d.assign(d, d + m);
    *out = c;
    return MSP_OK;
}

// Frees the context's library-owned workspace with the allocator that made it.
static void ctx_free_ws(msp_ctx *c) {
    DevMem m;
    m.ptr = c->ws;
    m.by.alloc = c->ws_alloc;
    m.by.release = c->ws_release;
    m.by.user = c->ws_user;
    dev_free(m);
    c->ws = nullptr;
    c->ws_bytes = 0;
}

int msp_set_allocator(msp_alloc_fn alloc, msp_release_fn release, void *user) {
    if ((alloc == nullptr) != (release == nullptr)) return MSP_E_INVALID;
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_alloc.alloc = alloc;
    g_alloc.release = release;
    g_alloc.user = user;
    return MSP_OK;
}

void msp_destroy(msp_ctx *c) {
    if (!c) return;
    if (c->ws) ctx_free_ws(c);
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
    delete c;
}

uint64_t msp_workspace_bytes(const msp_ctx *c, const msp_opts *opts) {
    if (!c) return 0;
    msp_opts o;
    msp_default_opts(&o);
    if (opts) o = *opts;
    Prepared P;
    if (prepare(c, o, o.workspace_bytes, P) != MSP_OK) return 0;
    return P.z.total;
}

int msp_plan(const msp_ctx *c, const msp_opts *opts, msp_plan_t *out) {
    if (!c || !out) return MSP_E_INVALID;
    msp_opts o;
    msp_default_opts(&o);
    if (opts) o = *opts;
    Prepared P;
    const int rc = prepare(c, o, o.workspace_bytes, P);
    if (rc) return rc;
    const Plan &p = P.p;
    const Sizes &z = P.z;
    msp_plan_t t{};
    t.key_rows = p.r;
    t.log2_m = p.log2M;
    t.log2_cells = p.log2T;
    t.log2_fine = p.log2F;
    t.parts = p.parts;
    t.exact_buckets = p.exact;
    t.words = p.W;
    t.join_variant = p.exact ? 0 : p.join_grouped;
    t.vector_join = p.vjoin;
    t.key_base = o.key_base;
    t.infeasible = P.infeasible ? 1 : 0;
    t.cells = z.ncells;
    t.cells_per_window = z.kwin;
    t.windows = (z.ncells + z.kwin - 1) / std::max<uint64_t>(z.kwin, 1);
    t.window_records = z.cap_rec;
    t.record_bytes = rec_bytes(p.Wr);
    t.row_fingerprint = p.fp;
    t.log2_outer = p.qa;
    t.log2_inner = p.qb;
    t.key_words = p.wide ? 2 : 1;
    t.key_bits = P.key_bits;
    t.workspace_bytes = z.total;
    t.max_grid_items = z.max_items;
    *out = t;
    return MSP_OK;
}

int msp_solve(msp_ctx *c, const msp_opts *opts) {
    if (!c) return MSP_E_INVALID;
    if (c->poisoned) return MSP_E_DEVICE;
    int expect = 0;
    if (!c->busy.compare_exchange_strong(expect, 1)) return MSP_E_BUSY;
    struct Unbusy { msp_ctx *c; ~Unbusy() { c->busy.store(0); } } unbusy{c};
    Job j;
    j.c = c;
    msp_default_opts(&j.o);
    if (opts) j.o = *opts;
    j.t_wall0 = now_s();
    c->have_result = false;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return MSP_E_NOLIB;
    if (j.o.workspace && !j.o.workspace_bytes) return MSP_E_INVALID;
    uint64_t budget = j.o.workspace_bytes;
    if (!j.o.workspace && !budget) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) return MSP_E_NOLIB;
        budget = std::min<uint64_t>((uint64_t)(fr * 0.6), (uint64_t)64 << 30);
    }
    int rc = prepare(c, j.o, budget, j.P);
    if (rc) return rc;
    job_init_stats(j);
    if (j.P.infeasible) {
        job_trivial(j);
        return MSP_OK;
    }
    j.s = (hipStream_t)j.o.stream;
    if (!j.s) {
        if (!c->own_stream && hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking) != hipSuccess)
            return MSP_E_DEVICE;
        j.s = c->own_stream;
    }
    if (j.o.workspace) {
        j.ws = (char *)j.o.workspace;
    } else {
        if (c->ws_bytes < j.P.z.total) {
            if (c->ws) ctx_free_ws(c);
            DevMem m = dev_alloc(j.P.z.total);
            if (!m.ptr) return MSP_E_NOMEM;
            c->ws = m.ptr;
            c->ws_alloc = m.by.alloc;
            c->ws_release = m.by.release;
            c->ws_user = m.by.user;
            c->ws_bytes = j.P.z.total;
        }
        j.ws = (char *)c->ws;
    }
    job_carve(j);
    rc = job_setup_events(j);
    while (rc == MSP_OK && j.next != A_DONE) {
        rc = job_step(j);
        if (rc == MSP_OK && j.next != A_DONE && hipStreamSynchronize(j.s) != hipSuccess) {
            (void)hipGetLastError();
            rc = MSP_E_DEVICE;
        }
    }
    job_release_events(j);
    if (rc == MSP_E_DEVICE) c->poisoned = true;
    return rc;
}

int msp_solve_noalloc(msp_ctx *c, const msp_opts *opts) {
    if (!c) return MSP_E_INVALID;
    if (c->poisoned) return MSP_E_DEVICE;
    msp_opts o;
    msp_default_opts(&o);
    if (opts) o = *opts;
    if (o.workspace || (o.workspace_bytes && o.workspace_bytes != kScratchBytes))
        return MSP_E_INVALID;            // the workspace is the library's scratch array
    int expect = 0;
    if (!c->busy.compare_exchange_strong(expect, 1)) return MSP_E_BUSY;
    struct Unbusy { msp_ctx *c; ~Unbusy() { c->busy.store(0); } } unbusy{c};
    Job j;
    j.c = c;
    j.o = o;
    j.t_wall0 = now_s();
    c->have_result = false;
    void *ws = nullptr;
    int rc = scratch_address(&ws);
    if (rc) return rc;
    // The plan must fit the scratch array: MSP_E_NOMEM otherwise.
    rc = prepare(c, j.o, kScratchBytes, j.P);
    if (rc) return rc;
    job_init_stats(j);
    if (j.P.infeasible) {
        job_trivial(j);
        return MSP_OK;
    }
    j.s = (hipStream_t)j.o.stream;       // NULL: the null stream (no stream is created)
    j.ws = (char *)ws;
    job_carve(j);
    j.hs = c->hs_fixed;                  // no pinned buffer, no timing events
    j.hs_pinned = false;
    while (rc == MSP_OK && j.next != A_DONE) {
        rc = job_step(j);
        if (rc == MSP_OK && j.next != A_DONE && hipStreamSynchronize(j.s) != hipSuccess) {
            (void)hipGetLastError();
            rc = MSP_E_DEVICE;
        }
    }
    j.hs = nullptr;
    if (rc == MSP_E_DEVICE) c->poisoned = true;
    return rc;
}

int msp_batch_solve(msp_ctx *const *ctxs, const msp_opts *opts, int32_t count,
                    const msp_batch_opts *bo) {
    if (!ctxs || count < 0) return MSP_E_INVALID;
    for (int32_t i = 0; i < count; ++i)
        if (!ctxs[i]) return MSP_E_INVALID;
    Runner run;
    int rc = run.init(bo ? bo->hbm_budget : 0, bo ? bo->max_slots : 0);
    if (rc) { run.shutdown(); return rc; }
    std::vector<Job> jobs(count);
    for (int32_t i = 0; i < count; ++i) {
        Job &j = jobs[i];
        j.c = ctxs[i];
        msp_default_opts(&j.o);
        if (opts) j.o = opts[i];
        j.o.workspace = nullptr;
        j.o.stream = nullptr;
        j.c->have_result = false;
        run.plan(j);
        run.pending.push_back(&j);
    }
    std::vector<Job *> done;
    while (!run.pending.empty() || !run.active.empty()) {
        run.admit(done);
        if (run.active.empty()) {
            if (!run.pending.empty()) {      // head cannot fit even alone
                run.pending.front()->rc = MSP_E_NOMEM;
                done.push_back(run.pending.front());
                run.pending.pop_front();
            }
            continue;
        }
        if (!run.step(done)) idle_wait();
    }
    run.shutdown();
    int first = MSP_OK;
    for (auto &j : jobs)
        if (j.rc != MSP_OK && first == MSP_OK) first = j.rc;
    return first;
}

int msp_server_start(const msp_server_opts *o, msp_server **out) {
    if (!out) return MSP_E_INVALID;
    *out = nullptr;
    msp_server *sv = new (std::nothrow) msp_server();
    if (!sv) return MSP_E_NOMEM;
    int rc = sv->run.init(o ? o->hbm_budget : 0, o ? o->max_slots : 0);
    if (rc) {
        sv->run.shutdown();
        delete sv;
        return rc;
    }
    sv->th = std::thread(server_loop, sv);
    *out = sv;
    return MSP_OK;
}

int msp_server_submit(msp_server *sv, msp_ctx *c, const msp_opts *o, uint64_t *ticket) {
    if (!sv || !c || !ticket) return MSP_E_INVALID;
    int expect = 0;
    if (!c->busy.compare_exchange_strong(expect, 1)) return MSP_E_BUSY;
    Job *j = new (std::nothrow) Job();
    if (!j) { c->busy.store(0); return MSP_E_NOMEM; }
    j->c = c;
    msp_default_opts(&j->o);
    if (o) j->o = *o;
    j->o.workspace = nullptr;
    j->o.stream = nullptr;
    c->have_result = false;
    sv->run.plan(*j);                       // host-only planning, before queueing
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stopping) { c->busy.store(0); delete j; return MSP_E_STATE; }
    j->ticket = sv->next_ticket++;
    j->t_submit = now_s() - sv->run.t0;
    sv->jobs[j->ticket] = j;
    sv->inbox.push_back(j);
    *ticket = j->ticket;
    sv->cv.notify_all();
    return MSP_OK;
}

int msp_server_poll(msp_server *sv, uint64_t ticket, int32_t *done, int32_t *status) {
    if (!sv || !done) return MSP_E_INVALID;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->jobs.find(ticket);
    if (it == sv->jobs.end()) return MSP_E_INVALID;
    Job *j = it->second;
    *done = j->t_finish > 0 ? 1 : 0;
    if (status) *status = *done ? j->rc : MSP_OK;
    return MSP_OK;
}

int msp_server_wait(msp_server *sv, uint64_t ticket, int32_t *status) {
    if (!sv) return MSP_E_INVALID;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->jobs.find(ticket);
    if (it == sv->jobs.end()) return MSP_E_INVALID;
    Job *j = it->second;
    sv->cv_done.wait(lk, [&] { return j->t_finish > 0; });
    if (status) *status = j->rc;
    return MSP_OK;
}

int msp_server_cancel(msp_server *sv, uint64_t ticket) {
    if (!sv) return MSP_E_INVALID;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->jobs.find(ticket);
    if (it == sv->jobs.end()) return MSP_E_INVALID;
    Job *j = it->second;
    if (j->t_finish > 0) return MSP_OK;
    for (auto p = sv->inbox.begin(); p != sv->inbox.end(); ++p) {
        if (*p == j) {                       // not yet seen by the scheduler
            sv->inbox.erase(p);
            j->rc = MSP_E_CANCELLED;
            j->c->busy.store(0);
            j->t_finish = now_s() - sv->run.t0;
            sv->cv_done.notify_all();
            return MSP_OK;
        }
    }
    j->c->busy.store(2);                    // the scheduler stops it at the next window
    sv->cv.notify_all();
    return MSP_OK;
}

int msp_server_times(msp_server *sv, uint64_t ticket, double *t4) {
    if (!sv || !t4) return MSP_E_INVALID;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->jobs.find(ticket);
    if (it == sv->jobs.end()) return MSP_E_INVALID;
    const Job *j = it->second;
    t4[0] = j->t_submit;
    t4[1] = j->t_admit;
    t4[2] = j->t_start;
    t4[3] = j->t_finish;
    return MSP_OK;
}

int msp_server_stop(msp_server *sv) {
    if (!sv) return MSP_E_INVALID;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stopping = true;
        sv->cv.notify_all();
    }
    if (sv->th.joinable()) sv->th.join();
    sv->run.shutdown();
    for (auto &kv : sv->jobs) delete kv.second;
    delete sv;
    return MSP_OK;
}

int msp_num_solutions(const msp_ctx *c, uint64_t *count) {
    if (!c || !count) return MSP_E_INVALID;
    if (!c->have_result) return MSP_E_STATE;
    *count = c->nsol;
    return MSP_OK;
}

int msp_hits(const msp_ctx *c, uint64_t *lo, uint64_t *hi) {
    if (!c || !lo || !hi) return MSP_E_INVALID;
    if (!c->have_result) return MSP_E_STATE;
    *lo = c->h_lo;
    *hi = c->h_hi;
    return MSP_OK;
}

int msp_get_solutions(const msp_ctx *c, uint8_t *x, uint64_t capacity, uint64_t *written) {
    if (!c || !written || (capacity && !x)) return MSP_E_INVALID;
    if (!c->have_result) return MSP_E_STATE;
    const uint64_t k = std::min<uint64_t>(capacity, c->stored);
    if (k) std::memcpy(x, c->sol.data(), k * (uint64_t)c->n);
    *written = k;
    return (k < c->nsol) ? MSP_E_TRUNCATED : MSP_OK;
}

int msp_stats(const msp_ctx *c, msp_stats_t *out) {
    if (!c || !out) return MSP_E_INVALID;
    if (!c->have_result) return MSP_E_STATE;
    *out = c->stats;
    return MSP_OK;
}

}  // extern "C"
