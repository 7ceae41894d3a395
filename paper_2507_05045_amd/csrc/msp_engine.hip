// Host side of libmsp: instance validation, the solve plan, workspace
// layout, the per-window launch sequence and the C ABI of include/msp.h.
#include "msp.h"
#include "msp_internal.h"

#include <algorithm>
#include <chrono>
#include <cstring>
#include <new>
#include <numeric>
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
    hipStream_t own_stream = nullptr;
    hipEvent_t ev[8] = {};
    bool poisoned = false;
};

namespace {

int lg2ceil(uint64_t x) {
    int k = 0;
    while (k < 63 && ((uint64_t)1 << k) < x) ++k;
    return k;
}

uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

struct Sizes {
    uint64_t ncells = 0;     // cells to visit (all, or those of the slice)
    uint64_t kwin = 0;       // cells per window (planned)
    uint64_t cap_rec = 0;    // half records per side per window
    uint64_t sol_cap = 0;
    uint64_t total = 0;      // workspace bytes
    // offsets into the workspace
    uint64_t o_qraw[4], o_qsrt[4], o_qcnt[4], o_qcur[4], o_cnt[2], o_off[2], o_rec[2];
    uint64_t o_runs, o_tiles, o_sol, o_scal, o_scan, scan_bytes, o_colw, o_rows;
};

struct Prepared {
    Plan p{};
    std::vector<int64_t> colw;
    std::vector<uint16_t> rows;
    bool infeasible = false;
    Sizes z;
};

// Instance-level checks shared by msp_create and the plan.
int validate(const int32_t *A, const int32_t *d, int m, int n) {
    if (!A || !d || m < 1 || n < 1) return MSP_E_INVALID;
    if (m > 16 || n > 92) return MSP_E_UNSUPPORTED;
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

// The plan: surrogate key (Section 1, eq. surrogate), quarter widths
// (Algorithm 1's partition, contiguous), residue modulus, cells, windows.
int prepare(const msp_ctx *c, const msp_opts &o, uint64_t budget, Prepared &P) {
    Plan &p = P.p;
    const int m = c->m, n = c->n;
    const int r = o.key_rows ? o.key_rows : 1;
    if (r < 1 || r > m) return MSP_E_INVALID;
    if (m - r > 2 * kMaxWords) return MSP_E_UNSUPPORTED;
    if (o.slice_mod < 0 || (o.slice_mod > 0 && ((o.slice_mod & (o.slice_mod - 1)) != 0 ||
                                                o.slice_res < 0 || o.slice_res >= o.slice_mod)))
        return MSP_E_INVALID;
    if (o.log2_m < 0 || o.log2_m > 62 || o.log2_cells < 0 || o.log2_cells > 24 || o.parts < 0)
        return MSP_E_INVALID;
    p.m = m; p.n = n; p.r = r; p.nv = m - r; p.W = (p.nv + 1) / 2;
    p.hL = (n + 1) / 2;
    p.qa = (p.hL + 1) / 2; p.qb = p.hL / 2;
    p.qc = (n - p.hL + 1) / 2; p.qd = (n - p.hL) / 2;
    p.Q[0] = 1u << p.qa; p.Q[1] = 1u << p.qb; p.Q[2] = 1u << p.qc; p.Q[3] = 1u << p.qd;

    // Key: D > every a_ij (D = 100 for the [0,99] family), base B = n*D.
    int32_t amax = 0;
    for (int32_t a : c->A) amax = std::max(amax, a);
    const int64_t D = std::max<int64_t>(100, (int64_t)amax + 1);
    const int64_t B = (int64_t)n * D;
    __int128 kmax = 0, pw = 1;
    P.infeasible = false;
    for (int i = 0; i < r; ++i) {
        int64_t rs = 0;
        for (int j = 0; j < n; ++j) rs += c->A[(size_t)i * n + j];
        if (c->d[i] > rs) P.infeasible = true;      // row i can never hold: H = 0
        kmax += pw * rs;
        if (kmax >= ((__int128)1 << 63)) return MSP_E_KEY_OVERFLOW;
        pw *= B;
        if (i + 1 < r && pw >= ((__int128)1 << 63)) return MSP_E_KEY_OVERFLOW;
    }
    int64_t kd = 0, q = 1;
    for (int i = 0; i < r; ++i) {
        kd += q * (int64_t)c->d[i];
        if (i + 1 < r) q *= B;
    }
    p.Kd = P.infeasible ? 0 : kd;
    P.colw.assign(n, 0);
    for (int j = 0; j < n; ++j) {
        int64_t s = 0, qq = 1;
        for (int i = 0; i < r; ++i) {
            s += qq * (int64_t)c->A[(size_t)i * n + j];
            if (i + 1 < r) qq *= B;
        }
        P.colw[j] = s;
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

    // Residue modulus M and cells T.  Exact buckets when M can exceed K_d
    // cheaply (small keys, e.g. one key row); else buckets of ~1K records.
    const int lgKd = lg2ceil((uint64_t)p.Kd + 1);
    int log2M, log2T;
    if (o.log2_m) {
        log2M = o.log2_m;
    } else if (lgKd <= 16) {
        log2M = std::max(lgKd, 1);
    } else {
        log2M = std::max(p.qa + p.qb - 10, 1);
    }
    p.exact = (((uint64_t)1 << std::min(log2M, 62)) > (uint64_t)p.Kd) ? 1 : 0;
    if (o.log2_cells) {
        log2T = o.log2_cells;
    } else {
        // |B_j| ~ 8 pairs per outer element, and at most 1024 fine buckets
        // per cell (the staged scatter's LDS budget).
        log2T = std::max(p.qb - 3, 0);
        log2T = std::max(log2T, log2M - 10);
        if (log2T > 23) log2T = std::max(23, log2M - 12);   // cell tables <= 2^23
    }
    log2T = std::min(log2T, log2M);
    if (log2M - log2T > 12) return MSP_E_INVALID;       // fine buckets per cell <= 4096
    if (log2T > 24) return MSP_E_UNSUPPORTED;
    p.log2M = log2M; p.log2T = log2T; p.log2F = log2M - log2T;
    p.slice_mod = o.slice_mod;
    p.slice_res = o.slice_res;
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
    const uint64_t rb = rec_bytes(p.W), qb = qrec_bytes(p.W);
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
    int parts = o.parts;
    if (!parts) {
        const uint64_t target = 2048;
        parts = (int)std::min<uint64_t>(64, std::max<uint64_t>(1, (target + kwin - 1) / kwin));
        parts = (int)std::min<uint64_t>(parts, std::max<uint64_t>(1, p.Q[0] / 256));
        parts = (int)std::min<uint64_t>(parts, std::max<uint64_t>(1, p.Q[2] / 256));
    }
    p.parts = parts;
    auto layout = [&](uint64_t cap_rec, uint64_t kw) -> uint64_t {
        uint64_t off = 0;
        auto take = [&](uint64_t bytes) { uint64_t o2 = off; off += align_up(bytes, 256); return o2; };
        for (int x = 0; x < 4; ++x) z.o_qraw[x] = take((uint64_t)p.Q[x] * qb);
        for (int x = 0; x < 4; ++x) z.o_qsrt[x] = take((uint64_t)p.Q[x] * qb);
        for (int x = 0; x < 4; ++x) z.o_qcnt[x] = take((T + 1) * 4);
        for (int x = 0; x < 4; ++x) z.o_qcur[x] = take((T + 1) * 4);
        const uint64_t ncnt = kw * F * (uint64_t)parts + 1;
        for (int s = 0; s < 2; ++s) z.o_cnt[s] = take(ncnt * 4);
        for (int s = 0; s < 2; ++s) z.o_off[s] = take(ncnt * 4);
        for (int s = 0; s < 2; ++s) z.o_rec[s] = take(cap_rec * rb);
        z.o_runs = take(kw * F * sizeof(RunPair));
        z.o_tiles = take((kw * F + 1) * 4);
        z.o_sol = take(z.sol_cap * 16);
        z.o_scal = take(S_COUNT * 8);
        z.scan_bytes = scan_tmp_bytes(std::max<uint64_t>(std::max<uint64_t>(T + 1, ncnt), kw * F + 1));
        z.o_scan = take(z.scan_bytes);
        z.o_colw = take((uint64_t)n * 8);
        z.o_rows = take(P.rows.size() * 2);
        return off;
    };
    auto cap_for = [&](uint64_t kw) {
        return std::min<uint64_t>(hard_cap, std::min<uint64_t>(all_rec, kw * per_cell + 1024));
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
    return MSP_OK;
}

double ev_ms(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0;
    return (double)ms;
}

#define HIPCHK(x)                                      \
    do {                                               \
        hipError_t e_ = (x);                           \
        if (e_ != hipSuccess) { rc = MSP_E_DEVICE; goto fail; } \
    } while (0)

}  // namespace

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

void msp_destroy(msp_ctx *c) {
    if (!c) return;
    if (c->ws) (void)hipFree(c->ws);
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
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

int msp_solve(msp_ctx *c, const msp_opts *opts) {
    if (!c) return MSP_E_INVALID;
    if (c->poisoned) return MSP_E_DEVICE;
    const auto t0 = std::chrono::steady_clock::now();
    msp_opts o;
    msp_default_opts(&o);
    if (opts) o = *opts;
    c->have_result = false;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return MSP_E_NOLIB;

    if (o.workspace && !o.workspace_bytes) return MSP_E_INVALID;
    uint64_t budget = o.workspace_bytes;
    if (!o.workspace && !budget) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) return MSP_E_NOLIB;
        budget = std::min<uint64_t>((uint64_t)(fr * 0.6), (uint64_t)64 << 30);
    }
    Prepared P;
    int rc = prepare(c, o, budget, P);
    if (rc) return rc;
    const Plan &p = P.p;
    const Sizes &z = P.z;
    msp_stats_t st{};
    st.key_rows = p.r;
    st.log2_m = p.log2M;
    st.log2_cells = p.log2T;
    st.parts = p.parts;
    st.exact_buckets = p.exact;
    st.words = p.W;
    st.record_bytes = rec_bytes(p.W);
    c->sol.clear();
    c->stored = 0;
    if (P.infeasible) {
        c->h_lo = c->h_hi = c->nsol = 0;
        st.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        c->stats = st;
        c->have_result = true;
        return MSP_OK;
    }

    hipStream_t s = (hipStream_t)o.stream;
    char *ws = nullptr;
    DevBufs b{};
    uint64_t scal[S_COUNT] = {0};
    std::vector<uint64_t> solbuf;
    if (!s) {
        if (!c->own_stream && hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking) != hipSuccess)
            return MSP_E_DEVICE;
        s = c->own_stream;
    }
    for (auto &e : c->ev)
        if (!e && hipEventCreate(&e) != hipSuccess) return MSP_E_DEVICE;
    if (o.workspace) {
        ws = (char *)o.workspace;
    } else {
        if (c->ws_bytes < z.total) {
            if (c->ws) (void)hipFree(c->ws);
            c->ws = nullptr;
            c->ws_bytes = 0;
            if (hipMalloc(&c->ws, z.total) != hipSuccess) {
                (void)hipGetLastError();
                return MSP_E_NOMEM;
            }
            c->ws_bytes = z.total;
        }
        ws = (char *)c->ws;
    }
    for (int x = 0; x < 4; ++x) {
        b.qraw[x] = ws + z.o_qraw[x];
        b.qsrt[x] = ws + z.o_qsrt[x];
        b.qcnt[x] = (uint32_t *)(ws + z.o_qcnt[x]);
        b.qcur[x] = (uint32_t *)(ws + z.o_qcur[x]);
    }
    for (int sd = 0; sd < 2; ++sd) {
        b.cnt[sd] = (uint32_t *)(ws + z.o_cnt[sd]);
        b.off[sd] = (uint32_t *)(ws + z.o_off[sd]);
        b.rec[sd] = ws + z.o_rec[sd];
    }
    b.runs = (RunPair *)(ws + z.o_runs);
    b.tiles = (uint32_t *)(ws + z.o_tiles);
    b.sol = (uint64_t *)(ws + z.o_sol);
    b.scal = (uint64_t *)(ws + z.o_scal);
    b.scan_tmp = ws + z.o_scan;
    b.scan_tmp_bytes = z.scan_bytes;
    b.colw = (int64_t *)(ws + z.o_colw);
    b.rows = (uint16_t *)(ws + z.o_rows);

    {
        const uint64_t T = (uint64_t)1 << p.log2T;
        const int F = 1 << p.log2F;
        HIPCHK(hipMemcpyAsync(b.colw, P.colw.data(), P.colw.size() * 8, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(b.rows, P.rows.data(), P.rows.size() * 2, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemsetAsync(b.scal, 0, S_COUNT * 8, s));
        for (int x = 0; x < 4; ++x) HIPCHK(hipMemsetAsync(b.qcnt[x], 0, (T + 1) * 4, s));
        HIPCHK(hipEventRecord(c->ev[0], s));
        HIPCHK(launch_quarters(p, b, 0, s));
        HIPCHK(hipEventRecord(c->ev[1], s));

        uint64_t idx = 0;
        uint64_t kw = z.kwin;
        const uint64_t rb = rec_bytes(p.W);
        (void)rb;
        while (idx < z.ncells) {
            uint64_t K = std::min<uint64_t>(kw, z.ncells - idx);
            uint64_t totL = 0, totR = 0;
            for (;;) {
                const size_t ncnt = (size_t)K * F * p.parts;
                HIPCHK(hipEventRecord(c->ev[2], s));
                HIPCHK(launch_count(p, b, (int64_t)idx, (int32_t)K, s));
                HIPCHK(hipEventRecord(c->ev[3], s));
                HIPCHK(scan_u32(b.cnt[0], b.off[0], ncnt, &b.scal[S_TOT_L], b.scan_tmp, b.scan_tmp_bytes, s));
                HIPCHK(scan_u32(b.cnt[1], b.off[1], ncnt, &b.scal[S_TOT_R], b.scan_tmp, b.scan_tmp_bytes, s));
                HIPCHK(hipEventRecord(c->ev[4], s));
                HIPCHK(hipMemcpyAsync(scal, b.scal, S_COUNT * 8, hipMemcpyDeviceToHost, s));
                HIPCHK(hipStreamSynchronize(s));
                st.ms_count += ev_ms(c->ev[2], c->ev[3]);
                st.ms_scan += ev_ms(c->ev[3], c->ev[4]);
                totL = scal[S_TOT_L];
                totR = scal[S_TOT_R];
                if (totL <= z.cap_rec && totR <= z.cap_rec) break;
                if (K == 1) { rc = MSP_E_NOMEM; goto fail; }
                K = (K + 1) / 2;
                kw = K;
            }
            st.records_left += totL;
            st.records_right += totR;
            HIPCHK(hipMemsetAsync(&b.scal[S_NRUNS], 0, 8, s));
            HIPCHK(hipEventRecord(c->ev[2], s));
            HIPCHK(launch_scatter(p, b, (int64_t)idx, (int32_t)K, s));
            HIPCHK(hipEventRecord(c->ev[3], s));
            if (p.exact)
                HIPCHK(launch_exact_runs(p, b, (int32_t)K, s));
            else
                HIPCHK(launch_hash_join(p, b, (int32_t)K, z.sol_cap, s));
            HIPCHK(hipEventRecord(c->ev[4], s));
            HIPCHK(hipMemcpyAsync(scal, b.scal, S_COUNT * 8, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            st.ms_scatter += ev_ms(c->ev[2], c->ev[3]);
            st.ms_join += ev_ms(c->ev[3], c->ev[4]);
            const uint32_t nruns = (uint32_t)scal[S_NRUNS];
            if (nruns) {
                HIPCHK(launch_tile_counts(p, b, nruns, !p.exact, s));
                HIPCHK(scan_u32(b.tiles, b.tiles, nruns, &b.scal[S_TOT_TILES], b.scan_tmp, b.scan_tmp_bytes, s));
                HIPCHK(hipMemcpyAsync(&scal[S_TOT_TILES], &b.scal[S_TOT_TILES], 8, hipMemcpyDeviceToHost, s));
                HIPCHK(hipStreamSynchronize(s));
                const uint32_t ntiles = (uint32_t)scal[S_TOT_TILES];
                HIPCHK(hipEventRecord(c->ev[5], s));
                HIPCHK(launch_verify(p, b, nruns, ntiles, z.sol_cap, !p.exact, s));
                HIPCHK(hipEventRecord(c->ev[6], s));
                HIPCHK(hipEventSynchronize(c->ev[6]));
                st.ms_verify += ev_ms(c->ev[5], c->ev[6]);
                st.verify_launches++;
            }
            st.windows++;
            idx += K;
        }
        HIPCHK(hipMemcpyAsync(scal, b.scal, S_COUNT * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        st.ms_quarters = ev_ms(c->ev[0], c->ev[1]);
        c->h_lo = scal[S_H_LO];
        c->h_hi = scal[S_H_HI];
        c->nsol = scal[S_NSOL];
        const uint64_t stored = std::min<uint64_t>(z.sol_cap, p.W == 0 ? scal[S_STORED] : scal[S_NSOL]);
        solbuf.resize(stored * 2);
        if (stored) {
            HIPCHK(hipMemcpyAsync(solbuf.data(), b.sol, stored * 16, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
        }
        // Expand half masks to x (columns of the left half first) and sort
        // canonically (lexicographic on x_1..x_n, 0 < 1).
        const int n = c->n;
        std::vector<uint8_t> xs(stored * n);
        for (uint64_t k = 0; k < stored; ++k) {
            const uint64_t ml = solbuf[2 * k], mr = solbuf[2 * k + 1];
            for (int j = 0; j < n; ++j)
                xs[k * n + j] = (uint8_t)(j < p.hL ? (ml >> j) & 1u : (mr >> (j - p.hL)) & 1u);
        }
        std::vector<uint64_t> ord(stored);
        std::iota(ord.begin(), ord.end(), 0);
        std::sort(ord.begin(), ord.end(), [&](uint64_t a, uint64_t bb) {
            return std::memcmp(&xs[a * n], &xs[bb * n], n) < 0;
        });
        c->sol.resize(stored * n);
        for (uint64_t k = 0; k < stored; ++k) std::memcpy(&c->sol[k * n], &xs[ord[k] * n], n);
        c->stored = stored;
    }
    st.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    c->stats = st;
    c->have_result = true;
    return MSP_OK;
fail:
    (void)hipGetLastError();
    if (rc == MSP_E_DEVICE) c->poisoned = true;
    return rc;
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
