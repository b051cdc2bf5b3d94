// C ABI of the engine: context, workspace, host-side validation, partition
// enumeration and launch orchestration.  Every step of the method runs in the
// gfx950 kernels; this file only sizes, checks and sequences them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "capart.h"
#include "capart_internal.h"

using namespace capart;

struct capart_ctx {
    int device = 0;
    std::string err;
    std::vector<uint32_t> np_host;
    uint32_t *np_dev = nullptr;    // partition-count table, followed by the subset order table
    uint16_t *order_dev = nullptr;
    hipStream_t stream = nullptr;  // for host-pointer calls
    void *ws = nullptr;            // workspace
    size_t ws_bytes = 0;
    void *stage = nullptr;         // staging buffer for host-pointer calls
    size_t stage_bytes = 0;
    capart_tuning tune{};          // launch tuning (0 = automatic)
    void *scratch = nullptr;       // this device's no-allocation workspace (device address)
    uint64_t *tab = nullptr;       // subset tables of the exhaustive search
    size_t tab_bytes = 0;
    bool timing = false;           // record kernel events
    std::vector<hipEvent_t> ev_free;
    std::vector<std::array<hipEvent_t, 4>> ev_pending;
};

namespace {

std::string g_create_err = "no error";

capart_status fail(capart_ctx *c, capart_status st, const std::string &msg)
{
    if (c) c->err = msg;
    return st;
}

capart_status hip_fail(capart_ctx *c, hipError_t e, const char *what)
{
    return fail(c, CAPART_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// NP(r, j, x): partitions of r into at most j parts, each part <= x.
void build_np(std::vector<uint32_t> &np)
{
    np.assign((size_t)NP_J * NP_R * NP_X, 0u);
    for (int x = 0; x < NP_X; x++) np[np_index(0, 0, x)] = 1u;
    for (int j = 1; j < NP_J; j++) {
        for (int r = 0; r < NP_R; r++) {
            for (int x = 0; x < NP_X; x++) {
                uint64_t c = 0;
                if (r == 0) {
                    c = 1;
                } else {
                    // first (largest) part y in [1, min(x, r)], rest <= y in j-1 parts
                    const int top = std::min(x, r);
                    for (int y = 1; y <= top; y++) c += np[np_index(j - 1, r - y, y)];
                }
                np[np_index(j, r, x)] = (uint32_t)c;
            }
        }
    }
}

const std::vector<uint32_t> &host_np()
{
    static std::vector<uint32_t> tab;
    if (tab.empty()) build_np(tab);
    return tab;
}

// Subsets of {0..n-1} ordered by size, then value, for n = 1..FRONTIER_MAX_TASKS
// one after the other (the list for n starts at entry 2^n - 2 with the empty set).
const std::vector<uint16_t> &host_subset_order()
{
    static std::vector<uint16_t> tab;
    if (tab.empty()) {
        for (int n = 1; n <= FRONTIER_MAX_TASKS; n++) {
            std::vector<uint16_t> v(1u << n);
            for (uint32_t s = 0; s < (1u << n); s++) v[s] = (uint16_t)s;
            std::stable_sort(v.begin(), v.end(),
                             [](uint16_t a, uint16_t b) { return __builtin_popcount(a) < __builtin_popcount(b); });
            tab.insert(tab.end(), v.begin(), v.end());
        }
    }
    return tab;
}

uint32_t count_parts(int M, int K) { return host_np()[np_index(K, M, M)]; }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct WsLayout {
    size_t rec, forbid, sigma, setflags, memmask, partial, total;
};

WsLayout ws_layout(int64_t S, int64_t N, int chunks)
{
    WsLayout l;
    size_t o = 0;
    l.rec = o; o = align256(o + sizeof(TaskRec) * (size_t)std::max<int64_t>(N, 1));
    l.forbid = o; o = align256(o + 8 * (size_t)std::max<int64_t>(N, 1));
    l.sigma = o; o = align256(o + (size_t)std::max<int64_t>(N, 1));
    l.setflags = o; o = align256(o + 4 * (size_t)std::max<int64_t>(S, 1));
    l.memmask = o; o = align256(o + 8 * (size_t)std::max<int64_t>(S, 1));
    l.partial = o; o = align256(o + 32 * (size_t)std::max<int64_t>(S, 1) * (size_t)chunks);
    l.total = o;
    return l;
}

capart_status ensure_ws(capart_ctx *c, size_t bytes)
{
    if (bytes <= c->ws_bytes) return CAPART_OK;
    hipError_t e = hipDeviceSynchronize();  // earlier calls may still use the old workspace
    if (e != hipSuccess) return hip_fail(c, e, "hipDeviceSynchronize");
    if (c->ws) hipFree(c->ws);
    c->ws = nullptr;
    c->ws_bytes = 0;
    e = hipMalloc(&c->ws, bytes);
    if (e != hipSuccess) {
        c->ws = nullptr;
        return fail(c, CAPART_E_NOMEM, "workspace allocation failed");
    }
    c->ws_bytes = bytes;
    return CAPART_OK;
}

capart_status ensure_stage(capart_ctx *c, size_t bytes)
{
    if (bytes <= c->stage_bytes) return CAPART_OK;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(c, e, "hipDeviceSynchronize");
    if (c->stage) hipFree(c->stage);
    c->stage = nullptr;
    c->stage_bytes = 0;
    e = hipMalloc(&c->stage, bytes);
    if (e != hipSuccess) {
        c->stage = nullptr;
        return fail(c, CAPART_E_NOMEM, "staging allocation failed");
    }
    c->stage_bytes = bytes;
    return CAPART_OK;
}

bool valid_mode(int m) { return m >= CAPART_EXHAUSTIVE && m <= CAPART_HEUR_SMS_ACT; }

capart_status check_options(capart_ctx *c, const capart_options *opt)
{
    if (!opt) return fail(c, CAPART_E_INVAL, "options is NULL");
    if (opt->K < 1 || opt->K > CAPART_MAX_K) return fail(c, CAPART_E_INVAL, "K must be in [1, 8]");
    if (opt->policy != CAPART_POLICY_FP_DM && opt->policy != CAPART_POLICY_EDF)
        return fail(c, CAPART_E_INVAL, "unsupported policy");
    if (!valid_mode(opt->alloc_mode)) return fail(c, CAPART_E_INVAL, "unknown allocation mode");
    if (opt->flags & ~(CAPART_FLAG_SKIP_1G | CAPART_FLAG_NO_LEMMA1 | CAPART_FLAG_PER_SET_LAUNCH))
        return fail(c, CAPART_E_INVAL, "unknown flag");
    return CAPART_OK;
}

// tasks_bound: CAPART_MAX_TASKS, or CAPART_ALG1_MAX_TASKS for the Algorithm 1 calls
capart_status check_batch_shape(capart_ctx *c, const capart_tasksets *in, int tasks_bound = CAPART_MAX_TASKS)
{
    if (!in) return fail(c, CAPART_E_INVAL, "task sets is NULL");
    if (in->n_sets < 0 || in->n_tasks_total < 0) return fail(c, CAPART_E_INVAL, "negative size");
    if (in->n_sets > ((int64_t)1 << 31) - 1) return fail(c, CAPART_E_INVAL, "too many sets for one launch");
    if (in->max_tasks < 1 || in->max_tasks > tasks_bound)
        return fail(c, CAPART_E_INVAL, tasks_bound == CAPART_MAX_TASKS ? "max_tasks out of [1,64]" : "max_tasks out of [1,256]");
    if (in->max_M < 1 || in->max_M > CAPART_MAX_M) return fail(c, CAPART_E_INVAL, "max_M out of [1,255]");
    if (in->n_sets > 0 && (!in->set_offset || !in->M))
        return fail(c, CAPART_E_INVAL, "NULL set arrays");
    const bool tab = in->Cn_table || in->Cc_table || in->table_offset;
    if (tab && (!in->Cn_table || !in->Cc_table || !in->table_offset || in->table_len < 0))
        return fail(c, CAPART_E_INVAL, "explicit time tables need table_offset, Cn_table, Cc_table and table_len");
    if (in->n_tasks_total > 0 && (!in->T || !in->D || !in->type || (!tab && (!in->C_seq || !in->C_par || !in->k_permille))))
        return fail(c, CAPART_E_INVAL, "NULL task arrays");
    return CAPART_OK;
}

bool has_tables(const capart_tasksets *in) { return in && (in->Cn_table || in->Cc_table || in->table_offset); }

bool results_ok(const capart_results *r)
{
    return r && r->status && r->verdict && r->verdict_1g && r->pidx && r->sizes && r->aidx && r->maxU && r->sumU &&
           r->n_evals && r->alloc && r->R && r->R_1g && (!r->dbg_key || r->dbg_offset);
}

// Per-set validation on the host (same rules as the device).
int32_t validate_set(const capart_tasksets *in, int64_t s, int K, int mode)
{
    const int64_t o0 = in->set_offset[s], o1 = in->set_offset[s + 1];
    if (o0 < 0 || o1 < o0 || o1 > in->n_tasks_total) return CAPART_E_INVAL;
    const int64_t n = o1 - o0;
    const int32_t M = in->M[s];
    if (n < 1 || n > std::min(in->max_tasks, CAPART_MAX_TASKS) || M < 1 || M > std::min(in->max_M, CAPART_MAX_M) ||
        n * M > CAPART_MAX_NM)
        return CAPART_E_INVAL;
    const int64_t L31 = (int64_t)1 << 31;
    if (has_tables(in)) {
        const int64_t t0 = in->table_offset[s];
        if (t0 < 0 || t0 > in->table_len - n * M) return CAPART_E_INVAL;
        for (int64_t i = o0; i < o1; i++) {
            const int64_t T = in->T[i], D = in->D[i];
            if (T < 1 || T >= L31 || D < 1 || D > T || in->type[i] > 1) return CAPART_E_RANGE;
            const int64_t *rn = in->Cn_table + t0 + (i - o0) * M, *rc = in->Cc_table + t0 + (i - o0) * M;
            for (int m = 1; m <= M; m++) {
                const int64_t cn = rn[m - 1], cc = rc[m - 1];
                if (cn < 1 || cn >= L31 || cc < 1 || cc >= L31 || cc < cn) return CAPART_E_RANGE;
                if (m > 1 && (cn > rn[m - 2] || cc > rc[m - 2])) return CAPART_E_RANGE;
                if ((int64_t)m * cn < rn[0]) return CAPART_E_RANGE;
            }
        }
    } else {
        for (int64_t i = o0; i < o1; i++) {
            const int64_t T = in->T[i], D = in->D[i], a = in->C_seq[i], b = in->C_par[i];
            const int32_t k = in->k_permille[i];
            if (T < 1 || T >= L31 || D < 1 || D > T || a < 0 || b < 0 || a >= L31 || b >= L31 || a + b < 1 ||
                a + b >= L31 || k < 1000 || k > 1000000 || in->type[i] > 1)
                return CAPART_E_RANGE;
        }
    }
    if (mode == CAPART_EXHAUSTIVE) {
        const uint64_t kk = (uint64_t)std::min(K, M);
        const uint64_t lim = ((1ull << 62) - 1ull) / kk;
        uint64_t pw = 1;
        for (int64_t i = 0; i < n; i++) {
            if (pw > lim) return CAPART_E_INVAL;
            pw *= kk;
        }
    }
    return CAPART_OK;
}

// LDS regions after the tables: the frontier (2^front_n u16), shrunk until
// tables, frontier and (loop form 2) per-lane state fit the LDS next to the
// static per-set arrays; then (loop form 1) the test memo for the sets above
// the frontier limit, shrunk likewise.
void size_frontier(Launch &L, int max_tasks, int mode, const capart_tuning &tu)
{
    L.front_n = 0;
    L.front_words = 0;
    L.memo_log2 = 0;
    if (mode == CAPART_EXHAUSTIVE) return;
    if (tu.frontier != 2) {
        int fn = std::min(max_tasks, FRONTIER_MAX_TASKS);
        const size_t lane = L.form == 2 ? (size_t)L.threads * 8 * 16 : 0;
        while (fn > 0 && (size_t)4 * L.table_words + ((size_t)2 << fn) + lane > (size_t)150 * 1024) fn--;
        L.front_n = fn;
        L.front_words = fn > 0 ? (1 << fn) / 2 : 0;
    }
    if (L.form != 1 || tu.memo < 0 || max_tasks <= L.front_n) return;
    int lg = tu.memo > 0 ? tu.memo : MEMO_DEFAULT_LOG2;
    while (lg >= 8 && (size_t)4 * L.table_words + std::max((size_t)4 * L.front_words, (size_t)8 << lg) >
                          (size_t)150 * 1024)
        lg--;
    L.memo_log2 = lg >= 8 ? lg : 0;
}

// Sets of more than NARROW_MAX_TASKS tasks: wave-per-partitioning blocks of
// wchunk partitionings (unless tuned off); the partial slots per set then
// cover ceil(P / wchunk) chunks as well.
// wide_parts: partitionings of the batch's sets of more than NARROW_MAX_TASKS
// tasks, or -1 where the host does not see the sets (then S decides).
void set_wide_chunk(Launch &L, int max_tasks, uint32_t Pmax, const capart_tuning &tu, int64_t wide_parts, int64_t S)
{
    L.wchunk = 0;
    if (L.mode == CAPART_EXHAUSTIVE || max_tasks <= NARROW_MAX_TASKS || tu.wide_chunk < 0) return;
    if (tu.wide_chunk == 0 && (wide_parts >= 0 ? wide_parts >= WIDE_LANE_FILL : S > WIDE_WAVE_MAX_SETS)) return;
    L.wchunk = tu.wide_chunk > 0 ? tu.wide_chunk : WIDE_CHUNK_DEFAULT;
    L.chunks = std::max<int>(L.chunks, (int)((Pmax + (uint32_t)L.wchunk - 1) / (uint32_t)L.wchunk));
}

// Partitionings of M into at most K parts whose sizes are all admissible:
// g_k[r][x] = partitions of r into at most k parts of admissible sizes <= x,
// g_k[r][x] = g_k[r][x-1] + [x admissible, x <= r] g_{k-1}[r-x][x].
int64_t count_admissible(int M, int K, const Adm &a)
{
    auto ok = [&](int x) { return ((a.w[x >> 6] >> (x & 63)) & 1ull) != 0ull; };
    const size_t W = (size_t)M + 1;
    std::vector<int64_t> prev(W * W, 0), cur(W * W, 0);
    for (size_t x = 0; x < W; x++) prev[x] = 1;  // k = 0: only r = 0
    for (int k = 1; k <= K; k++) {
        for (int r = 0; r <= M; r++) {
            int64_t acc = r == 0 ? 1 : 0;
            cur[(size_t)r * W] = acc;
            for (int x = 1; x <= M; x++) {
                if (x <= r && ok(x)) acc += prev[(size_t)(r - x) * W + x];
                cur[(size_t)r * W + x] = acc;
            }
        }
        std::swap(prev, cur);
    }
    return prev[(size_t)M * W + M];
}

// The feasibility frontier costs about 2^n tests per set; with few admissible
// partitionings, direct tests on those are cheaper, so the frontier is skipped.
bool frontier_pays(int max_tasks, int max_M, int K, const Adm &a)
{
    if ((a.w[0] | a.w[1] | a.w[2] | a.w[3]) == 0ull) return true;
    const int n = std::min(max_tasks, FRONTIER_MAX_TASKS);
    return count_admissible(max_M, K, a) * (int64_t)max_tasks * K >= ((int64_t)1 << n);
}

struct Plan {
    Launch L;
    int64_t S, N;
};

Plan make_plan(const capart_tasksets *in, const capart_options *opt, const capart_tuning &tu, int64_t wide_parts = -1)
{
    Plan p;
    p.S = in->n_sets;
    p.N = in->n_tasks_total;
    Launch &L = p.L;
    L.s0 = 0;
    L.S = p.S;
    L.K = opt->K;
    L.mode = opt->alloc_mode;
    L.flags = opt->flags;
    for (int i = 0; i < 4; i++) L.adm.w[i] = opt->admissible[i];
    L.edf = opt->policy == CAPART_POLICY_EDF;
    L.threads = eval_threads(in->max_tasks, in->max_M);
    if (tu.threads > 0) L.threads = std::min(L.threads, tu.threads);
    L.table_words = (int)(table_lds_bytes(in->max_tasks, in->max_M) / 4);
    L.form = tu.loop_form == 2 ? 2 : 1;
    L.memo_packed = tu.loop_form == 3;
    // exhaustive: subset tables + pruned search when sets are small enough
    capart_tuning tf = tu;
    if (tf.frontier == 0 && !frontier_pays(in->max_tasks, in->max_M, opt->K, L.adm)) tf.frontier = 2;
    size_frontier(L, in->max_tasks, opt->alloc_mode, tf);
    L.exh_form = (opt->K <= 4 && in->max_tasks <= SUBSET_MAX_TASKS) ? 2 : 1;
    if (tu.exh_form == 1 || tu.exh_form == 2) L.exh_form = tu.exh_form;
    if (L.exh_form == 2 && (opt->K > 4 || in->max_tasks > SUBSET_MAX_TASKS)) L.exh_form = 1;
    const uint32_t Pmax = count_parts(in->max_M, opt->K);
    if (opt->alloc_mode == CAPART_EXHAUSTIVE) {
        L.chunks = (int)Pmax;
        L.chunk = 1;
    } else {
        // about 4 partitionings per thread: many blocks balance uneven work
        // (measured on 100,000 sets of 10 tasks, M = 80: 1024 partitionings
        // per block beat one block per set by 9 %), at least one per thread
        // when there are few sets
        const int64_t per_set_launch = (opt->flags & CAPART_FLAG_PER_SET_LAUNCH) ? 1 : p.S;
        int64_t ch = std::max<int64_t>(1, (Pmax + 4 * L.threads - 1) / (4 * L.threads));
        const int64_t want_blocks = 2048;
        const int64_t ch_fill = (want_blocks + std::max<int64_t>(per_set_launch, 1) - 1) / std::max<int64_t>(per_set_launch, 1);
        const int64_t chmax = std::max<int64_t>(1, (Pmax + L.threads - 1) / L.threads);
        ch = std::max<int64_t>(1, std::min(std::max(ch, ch_fill), chmax));
        // frontier sets: the frontier is built once per block, so keep one
        // block per set when there are enough sets to fill the chip
        if ((L.front_n > 0 && in->max_tasks <= L.front_n) || (L.memo_log2 > 0 && in->max_tasks <= NARROW_MAX_TASKS))
            ch = std::max<int64_t>(1, std::min(ch_fill, chmax));
        L.chunk = (uint32_t)((Pmax + ch - 1) / ch);
        if (tu.chunk > 0) L.chunk = std::min<uint32_t>((uint32_t)tu.chunk, std::max<uint32_t>(Pmax, 1));
        L.chunks = (int)((Pmax + L.chunk - 1) / L.chunk);
        set_wide_chunk(L, in->max_tasks, Pmax, tu, wide_parts, p.S);
    }
    return p;
}

// Partitionings of the sets of more than NARROW_MAX_TASKS tasks (host arrays).
int64_t wide_partitionings(const int64_t *off, const int32_t *M, int64_t S, int K)
{
    int64_t t = 0;
    for (int64_t s = 0; s < S; s++) {
        const int64_t n = off[s + 1] - off[s];
        if (n > NARROW_MAX_TASKS && n <= CAPART_MAX_TASKS && M[s] >= 1 && M[s] <= CAPART_MAX_M) t += count_parts(M[s], K);
    }
    return t;
}

hipEvent_t take_event(capart_ctx *c)
{
    if (!c->ev_free.empty()) {
        hipEvent_t e = c->ev_free.back();
        c->ev_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launch prep, eval and final for one launch range, with timing events when enabled.
capart_status launch_three(capart_ctx *c, const Batch &b, const Work &w, const Out &o, const Launch &L,
                           hipStream_t st, uint32_t p_lo, uint32_t p_hi)
{
    std::array<hipEvent_t, 4> ev{};
    const bool tm = c->timing;
    if (tm)
        for (auto &e : ev)
            if (!(e = take_event(c))) return fail(c, CAPART_E_DEVICE, "hipEventCreate failed");
    hipError_t e;
    (void)hipGetLastError();  // launch checks below report this sequence's errors only
    if (tm) hipEventRecord(ev[0], st);
    if ((e = launch_prep(b, w, o, L, st)) != hipSuccess) return hip_fail(c, e, "prep launch");
    if (tm) hipEventRecord(ev[1], st);
    if (L.mode == CAPART_EXHAUSTIVE && L.exh_form == 2) {
        // subset tables, in waves of sets that bound the table memory
        const int ntab = std::min(b.max_tasks, (int)SUBSET_MAX_TASKS), Mtab = b.max_M;
        const size_t per_set = ((size_t)Mtab << ntab) * 8;
        const int64_t W = std::max<int64_t>(1, std::min<int64_t>(L.S, (int64_t)(((size_t)512 << 20) / per_set)));
        if (c->tab_bytes < per_set * (size_t)W) {
            hipError_t se = hipStreamSynchronize(st);
            if (se != hipSuccess) return hip_fail(c, se, "hipStreamSynchronize");
            if (c->tab) hipFree(c->tab);
            c->tab = nullptr;
            c->tab_bytes = 0;
            if (hipMalloc((void **)&c->tab, per_set * (size_t)W) != hipSuccess) {
                c->tab = nullptr;
                return fail(c, CAPART_E_NOMEM, "subset table allocation failed");
            }
            c->tab_bytes = per_set * (size_t)W;
        }
        const uint32_t Pmax = (uint32_t)L.chunks;
        for (int64_t s0 = 0; s0 < L.S; s0 += W) {
            const int w_n = (int)std::min<int64_t>(W, L.S - s0);
            if ((e = launch_subset_tables(b, w, L, c->tab, L.s0 + s0, w_n, Mtab, ntab, st)) != hipSuccess)
                return hip_fail(c, e, "subset table launch");
            if ((e = launch_exh_dfs(b, w, o, L, c->tab, L.s0 + s0, w_n, Mtab, ntab, Pmax, p_lo, p_hi, st)) !=
                hipSuccess)
                return hip_fail(c, e, "exhaustive search launch");
        }
    } else if ((e = launch_eval_range(b, w, o, L, st, p_lo, p_hi)) != hipSuccess) {
        return hip_fail(c, e, "eval launch");
    }
    if (tm) hipEventRecord(ev[2], st);
    if ((e = launch_final(b, w, o, L, st)) != hipSuccess) return hip_fail(c, e, "final launch");
    if (tm) {
        hipEventRecord(ev[3], st);
        c->ev_pending.push_back(ev);
    }
    return CAPART_OK;
}

// The batch's explicit time tables, for the kernels that stage a set.
void give_tables(Work &w, const Batch &b)
{
    w.toff = b.toff;
    w.tCn = b.Cn;
    w.tCc = b.Cc;
}

// Workspace arrays at base for layout l.
Work bind_work_at(capart_ctx *c, const WsLayout &l, void *ws)
{
    char *base = (char *)ws;
    Work w{};
    w.rec = (TaskRec *)(base + l.rec);
    w.forbid = (uint64_t *)(base + l.forbid);
    w.sigma = (uint8_t *)(base + l.sigma);
    w.setflags = (uint32_t *)(base + l.setflags);
    w.memmask = (uint64_t *)(base + l.memmask);
    w.partial = (uint64_t *)(base + l.partial);
    w.np = c->np_dev;
    w.order = c->order_dev;
    return w;
}

// Workspace arrays of the context for layout l (ensure_ws first).
Work bind_work(capart_ctx *c, const WsLayout &l) { return bind_work_at(c, l, c->ws); }

capart_status run_plan(capart_ctx *c, const Batch &b, const Out &o, const Plan &p, hipStream_t st,
                       uint32_t p_lo = 0u, uint32_t p_hi = 0xFFFFFFFFu)
{
    const WsLayout l = ws_layout(p.S, p.N, p.L.chunks);
    capart_status rc = ensure_ws(c, l.total);
    if (rc != CAPART_OK) return rc;
    Work w = bind_work(c, l);
    give_tables(w, b);
    if (p.L.flags & CAPART_FLAG_PER_SET_LAUNCH) {
        for (int64_t s = 0; s < p.S; s++) {
            Launch L1 = p.L;
            L1.s0 = s;
            L1.S = 1;
            if ((rc = launch_three(c, b, w, o, L1, st, p_lo, p_hi)) != CAPART_OK) return rc;
        }
        return CAPART_OK;
    }
    return launch_three(c, b, w, o, p.L, st, p_lo, p_hi);
}

Batch make_batch(const capart_tasksets *in)
{
    Batch b;
    b.off = in->set_offset;
    b.M = in->M;
    b.T = in->T;
    b.D = in->D;
    b.Cs = in->C_seq;
    b.Cp = in->C_par;
    b.k = in->k_permille;
    b.type = in->type;
    b.n_tasks_total = in->n_tasks_total;
    b.max_tasks = in->max_tasks;
    b.max_M = in->max_M;
    if (has_tables(in)) {
        b.toff = in->table_offset;
        b.Cn = in->Cn_table;
        b.Cc = in->Cc_table;
        b.tlen = in->table_len;
    }
    return b;
}

Out make_out(const capart_results *r)
{
    Out o;
    o.status = r->status;
    o.verdict = r->verdict;
    o.verdict_1g = r->verdict_1g;
    o.pidx = r->pidx;
    o.sizes = r->sizes;
    o.aidx = r->aidx;
    o.maxU = r->maxU;
    o.sumU = r->sumU;
    o.n_evals = r->n_evals;
    o.alloc = r->alloc;
    o.R = r->R;
    o.R_1g = r->R_1g;
    o.dbg_key = r->dbg_key;
    o.dbg_offset = r->dbg_offset;
    return o;
}

// Bump allocator over the staging buffer.
struct Bump {
    char *base;
    size_t off = 0;
    template <typename T>
    T *take(size_t n)
    {
        T *p = (T *)(base + off);
        off = align256(off + sizeof(T) * std::max<size_t>(n, 1));
        return p;
    }
};

// Explicit time tables of a host batch into the staging buffer (d gets the
// device pointers).
capart_status stage_tables(capart_ctx *c, const capart_tasksets *in, Bump &bp, hipStream_t st, capart_tasksets &d)
{
    const int64_t S = in->n_sets, TL = in->table_len;
    int64_t *t_off = bp.take<int64_t>(S), *t_cn = bp.take<int64_t>(TL), *t_cc = bp.take<int64_t>(TL);
    hipError_t e;
    if ((S && (e = hipMemcpyAsync(t_off, in->table_offset, 8 * (size_t)S, hipMemcpyHostToDevice, st)) != hipSuccess) ||
        (TL && (e = hipMemcpyAsync(t_cn, in->Cn_table, 8 * (size_t)TL, hipMemcpyHostToDevice, st)) != hipSuccess) ||
        (TL && (e = hipMemcpyAsync(t_cc, in->Cc_table, 8 * (size_t)TL, hipMemcpyHostToDevice, st)) != hipSuccess))
        return hip_fail(c, e, "hipMemcpyAsync H2D");
    d.table_offset = t_off;
    d.Cn_table = t_cn;
    d.Cc_table = t_cc;
    d.table_len = TL;
    return CAPART_OK;
}

size_t stage_need(int64_t S, int64_t N, int K, int64_t ndbg)
{
    size_t t = 0;
    auto add = [&](size_t bytes) { t = align256(t + std::max<size_t>(bytes, 1)); };
    add(8 * (S + 1)); add(4 * S);                                          // offsets, M
    add(8 * N); add(8 * N); add(8 * N); add(8 * N); add(4 * N); add(N);    // task arrays
    add(4 * S); add(S); add(S); add(4 * S); add(4 * S * K); add(8 * S);  // status .. aidx
    add(8 * S); add(8 * S); add(8 * S);                                    // maxU sumU n_evals
    add(N); add(8 * N); add(8 * N);                                        // alloc R R_1g
    add(24 * ndbg); add(8 * S);                                            // dbg
    return t;
}

}  // namespace

extern "C" {

capart_status capart_create(int device, capart_ctx **out)
{
    if (!out) return CAPART_E_INVAL;
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count == 0) {
        g_create_err = std::string("no HIP device: ") + hipGetErrorString(e);
        return CAPART_E_DEVICE;
    }
    if (device < 0 || device >= count) {
        g_create_err = "device index out of range";
        return CAPART_E_INVAL;
    }
    capart_ctx *c = new (std::nothrow) capart_ctx;
    if (!c) return CAPART_E_NOMEM;
    c->device = device;
    if ((e = hipSetDevice(device)) != hipSuccess) {
        g_create_err = std::string("hipSetDevice: ") + hipGetErrorString(e);
        delete c;
        return CAPART_E_DEVICE;
    }
    const std::vector<uint32_t> &np = host_np();
    const std::vector<uint16_t> &ord = host_subset_order();
    const size_t np_bytes = np.size() * sizeof(uint32_t), ord_bytes = ord.size() * sizeof(uint16_t);
    if ((e = hipMalloc(&c->np_dev, np_bytes + ord_bytes)) != hipSuccess) {
        g_create_err = "count table allocation failed";
        delete c;
        return CAPART_E_NOMEM;
    }
    c->order_dev = (uint16_t *)((char *)c->np_dev + np_bytes);
    if ((e = hipMemcpy(c->np_dev, np.data(), np_bytes, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(c->order_dev, ord.data(), ord_bytes, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipStreamCreate(&c->stream)) != hipSuccess) {
        g_create_err = std::string("context setup: ") + hipGetErrorString(e);
        hipFree(c->np_dev);
        if (c->stream) hipStreamDestroy(c->stream);
        delete c;
        return CAPART_E_DEVICE;
    }
    // raise the dynamic-LDS limit for the largest per-set tables; if the
    // runtime refuses, launches needing more than the default report E_DEVICE
    e = configure_kernels();
    c->err = (e == hipSuccess) ? "no error" : std::string("LDS limit not raised: ") + hipGetErrorString(e);
    // the no-allocation workspace of this device (the entry point reports it
    // unusable if the runtime gives no address)
    if (scratch_address(&c->scratch) != hipSuccess) {
        c->scratch = nullptr;
        (void)hipGetLastError();
    }
    *out = c;
    return CAPART_OK;
}

capart_status capart_destroy(capart_ctx *c)
{
    if (!c) return CAPART_E_INVAL;
    hipSetDevice(c->device);
    hipDeviceSynchronize();
    for (auto &a : c->ev_pending)
        for (auto e : a) hipEventDestroy(e);
    for (auto e : c->ev_free) hipEventDestroy(e);
    if (c->ws) hipFree(c->ws);
    if (c->stage) hipFree(c->stage);
    if (c->np_dev) hipFree(c->np_dev);
    if (c->tab) hipFree(c->tab);
    if (c->stream) hipStreamDestroy(c->stream);
    delete c;
    return CAPART_OK;
}

const char *capart_last_error(const capart_ctx *c) { return c ? c->err.c_str() : g_create_err.c_str(); }

#ifndef CAPART_BUILD_HASH
#define CAPART_BUILD_HASH "unknown"
#endif
const char *capart_build_hash(void) { return CAPART_BUILD_HASH; }

capart_status capart_measure_valu(capart_ctx *c, double *lane_ops_per_s, double *kernel_ms)
{
    if (!c || !lane_ops_per_s || !kernel_ms) return CAPART_E_INVAL;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    if ((e = measure_valu(c->stream, lane_ops_per_s, kernel_ms)) != hipSuccess) return hip_fail(c, e, "VALU benchmark");
    return CAPART_OK;
}

capart_status capart_count_partitionings(int32_t M, int32_t K, int64_t *count)
{
    if (!count || M < 1 || M > CAPART_MAX_M || K < 1 || K > CAPART_MAX_K) return CAPART_E_INVAL;
    *count = count_parts(M, K);
    return CAPART_OK;
}

capart_status capart_enumerate_partitionings(int32_t M, int32_t K, int32_t *sizes, int64_t capacity, int64_t *count)
{
    if (!count || M < 1 || M > CAPART_MAX_M || K < 1 || K > CAPART_MAX_K || capacity < 0 || (capacity > 0 && !sizes))
        return CAPART_E_INVAL;
    const int64_t P = count_parts(M, K);
    *count = P;
    if (capacity == 0) return CAPART_OK;
    // first partitioning (M), then successors in descending lexicographic order
    std::vector<int32_t> a(K, 0);
    a[0] = M;
    for (int64_t q = 0; q < P && q < capacity; q++) {
        std::copy(a.begin(), a.end(), sizes + q * K);
        // successor: rightmost part that can shrink by one with the remainder
        // refilled greedily into the parts to its right
        int tail = 0, sel = -1;
        for (int i = K - 1; i >= 0; i--) {
            if (a[i] > 1 && tail + 1 <= (K - i - 1) * (a[i] - 1)) { sel = i; break; }
            tail += a[i];
        }
        if (sel < 0) break;
        const int v = a[sel] - 1;
        int rest = tail + 1;
        a[sel] = v;
        for (int i = sel + 1; i < K; i++) {
            const int x = std::min(v, rest);
            a[i] = x;
            rest -= x;
        }
    }
    return CAPART_OK;
}

capart_status capart_validate(const capart_tasksets *in, const capart_options *opt, int32_t *status_out)
{
    capart_status rc;
    if ((rc = check_options(nullptr, opt)) != CAPART_OK) return rc;
    if ((rc = check_batch_shape(nullptr, in)) != CAPART_OK) return rc;
    if (in->n_sets > 0 && !status_out) return CAPART_E_INVAL;
    for (int64_t s = 0; s < in->n_sets; s++) status_out[s] = validate_set(in, s, opt->K, opt->alloc_mode);
    return CAPART_OK;
}

capart_status capart_solve_async(capart_ctx *c, const capart_tasksets *in, const capart_options *opt,
                                 capart_results *out, void *hip_stream)
{
    if (!c) return CAPART_E_INVAL;
    capart_status rc;
    if ((rc = check_options(c, opt)) != CAPART_OK) return rc;
    if ((rc = check_batch_shape(c, in)) != CAPART_OK) return rc;
    if (in->n_sets == 0) return CAPART_OK;
    if (!results_ok(out)) return fail(c, CAPART_E_INVAL, "NULL result array");
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    const Plan p = make_plan(in, opt, c->tune);
    return run_plan(c, make_batch(in), make_out(out), p, (hipStream_t)hip_stream);
}

capart_status capart_solve_async_noalloc(capart_ctx *c, const capart_tasksets *in, const capart_options *opt,
                                         capart_results *out, void *hip_stream)
{
    if (!c) return CAPART_E_INVAL;
    capart_status rc;
    if ((rc = check_options(c, opt)) != CAPART_OK) return rc;
    if ((rc = check_batch_shape(c, in)) != CAPART_OK) return rc;
    if (in->n_sets == 0) return CAPART_OK;
    if (!results_ok(out)) return fail(c, CAPART_E_INVAL, "NULL result array");
    if (!c->scratch) return fail(c, CAPART_E_DEVICE, "no address for the no-allocation workspace on this device");
    Plan p = make_plan(in, opt, c->tune);
    if (p.L.mode == CAPART_EXHAUSTIVE) p.L.exh_form = 1;  // the subset-table form needs memory of its own
    const WsLayout l = ws_layout(p.S, p.N, p.L.chunks);
    if (l.total > (size_t)CAPART_NOALLOC_SCRATCH_BYTES)
        return fail(c, CAPART_E_RANGE, "the batch needs " + std::to_string(l.total) +
                                           " bytes of workspace, above the no-allocation limit of " +
                                           std::to_string((size_t)CAPART_NOALLOC_SCRATCH_BYTES) + " bytes");
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    const Batch b = make_batch(in);
    const Out o = make_out(out);
    Work w = bind_work_at(c, l, c->scratch);
    give_tables(w, b);
    const bool tm = c->timing;  // timing events would be created on demand
    c->timing = false;
    const hipStream_t st = (hipStream_t)hip_stream;
    if (p.L.flags & CAPART_FLAG_PER_SET_LAUNCH) {
        for (int64_t s = 0; s < p.S && rc == CAPART_OK; s++) {
            Launch L1 = p.L;
            L1.s0 = s;
            L1.S = 1;
            rc = launch_three(c, b, w, o, L1, st, 0u, 0xFFFFFFFFu);
        }
    } else {
        rc = launch_three(c, b, w, o, p.L, st, 0u, 0xFFFFFFFFu);
    }
    c->timing = tm;
    return rc;
}

static capart_status solve_host(capart_ctx *c, const capart_tasksets *in, const capart_options *opt,
                                capart_results *out, uint32_t p_lo, uint32_t p_hi)
{
    if (!c) return CAPART_E_INVAL;
    capart_status rc;
    if ((rc = check_options(c, opt)) != CAPART_OK) return rc;
    if ((rc = check_batch_shape(c, in)) != CAPART_OK) return rc;
    if (in->n_sets == 0) return CAPART_OK;
    if (!results_ok(out)) return fail(c, CAPART_E_INVAL, "NULL result array");
    if (in->set_offset[0] != 0 || in->set_offset[in->n_sets] != in->n_tasks_total)
        return fail(c, CAPART_E_INVAL, "set_offset must run from 0 to n_tasks_total");
    const int64_t S = in->n_sets, N = in->n_tasks_total;
    const int K = opt->K;
    int64_t ndbg = 0;
    if (out->dbg_key) {
        for (int64_t s = 0; s < S; s++) {
            const int32_t M = in->M[s];
            if (M >= 1 && M <= CAPART_MAX_M) ndbg = std::max<int64_t>(ndbg, out->dbg_offset[s] + count_parts(M, K));
        }
    }
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    const int64_t TL = has_tables(in) ? in->table_len : 0;
    if ((rc = ensure_stage(c, stage_need(S, N, K, ndbg) + (TL ? align256(8 * (size_t)S) + 2 * align256(8 * (size_t)TL) + 768 : 0))) !=
        CAPART_OK)
        return rc;
    Bump bp{(char *)c->stage};
    capart_tasksets d = *in;
    int64_t *d_off = bp.take<int64_t>(S + 1);
    int32_t *d_M = bp.take<int32_t>(S);
    int64_t *d_T = bp.take<int64_t>(N), *d_D = bp.take<int64_t>(N), *d_Cs = bp.take<int64_t>(N),
            *d_Cp = bp.take<int64_t>(N);
    int32_t *d_k = bp.take<int32_t>(N);
    uint8_t *d_ty = bp.take<uint8_t>(N);
    capart_results r;
    r.status = bp.take<int32_t>(S);
    r.verdict = bp.take<uint8_t>(S);
    r.verdict_1g = bp.take<uint8_t>(S);
    r.pidx = bp.take<int32_t>(S);
    r.sizes = bp.take<int32_t>(S * K);
    r.aidx = bp.take<int64_t>(S);
    r.maxU = bp.take<uint64_t>(S);
    r.sumU = bp.take<uint64_t>(S);
    r.n_evals = bp.take<int64_t>(S);
    r.alloc = bp.take<int8_t>(N);
    r.R = bp.take<int64_t>(N);
    r.R_1g = bp.take<int64_t>(N);
    r.dbg_key = out->dbg_key ? bp.take<uint64_t>(3 * ndbg) : nullptr;
    int64_t *d_dbgoff = bp.take<int64_t>(S);
    r.dbg_offset = out->dbg_key ? d_dbgoff : nullptr;
    hipStream_t st = c->stream;
    struct Cp { void *dst; const void *src; size_t n; } h2d[] = {
        {d_off, in->set_offset, 8 * (size_t)(S + 1)}, {d_M, in->M, 4 * (size_t)S},
        {d_T, in->T, 8 * (size_t)N}, {d_D, in->D, 8 * (size_t)N}, {d_Cs, in->C_seq, in->C_seq ? 8 * (size_t)N : 0},
        {d_Cp, in->C_par, in->C_par ? 8 * (size_t)N : 0}, {d_k, in->k_permille, in->k_permille ? 4 * (size_t)N : 0}, {d_ty, in->type, (size_t)N},
        {d_dbgoff, out->dbg_key ? (const void *)out->dbg_offset : nullptr, out->dbg_key ? 8 * (size_t)S : 0}};
    for (const auto &x : h2d)
        if (x.n && (e = hipMemcpyAsync(x.dst, x.src, x.n, hipMemcpyHostToDevice, st)) != hipSuccess)
            return hip_fail(c, e, "hipMemcpyAsync H2D");
    d.set_offset = d_off; d.M = d_M; d.T = d_T; d.D = d_D; d.C_seq = d_Cs; d.C_par = d_Cp; d.k_permille = d_k;
    d.type = d_ty;
    if (TL && (rc = stage_tables(c, in, bp, st, d)) != CAPART_OK) return rc;
    const Plan p = make_plan(in, opt, c->tune, wide_partitionings(in->set_offset, in->M, S, K));
    if ((rc = run_plan(c, make_batch(&d), make_out(&r), p, st, p_lo, p_hi)) != CAPART_OK) return rc;
    Cp d2h[] = {{out->status, r.status, 4 * (size_t)S}, {out->verdict, r.verdict, (size_t)S},
                {out->verdict_1g, r.verdict_1g, (size_t)S}, {out->pidx, r.pidx, 4 * (size_t)S},
                {out->sizes, r.sizes, 4 * (size_t)S * K}, {out->aidx, r.aidx, 8 * (size_t)S},
                {out->maxU, r.maxU, 8 * (size_t)S}, {out->sumU, r.sumU, 8 * (size_t)S},
                {out->n_evals, r.n_evals, 8 * (size_t)S}, {out->alloc, r.alloc, (size_t)N},
                {out->R, r.R, 8 * (size_t)N}, {out->R_1g, r.R_1g, 8 * (size_t)N},
                {out->dbg_key, r.dbg_key, out->dbg_key ? 24 * (size_t)ndbg : 0}};
    for (const auto &x : d2h)
        if (x.n && (e = hipMemcpyAsync(x.dst, x.src, x.n, hipMemcpyDeviceToHost, st)) != hipSuccess)
            return hip_fail(c, e, "hipMemcpyAsync D2H");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
    return CAPART_OK;
}

capart_status capart_solve(capart_ctx *c, const capart_tasksets *in, const capart_options *opt, capart_results *out)
{
    return solve_host(c, in, opt, out, 0u, 0xFFFFFFFFu);
}

// ---- Algorithm 1 (free partition sizes) ----------------------------------

static capart_status alg1_check(capart_ctx *c, const capart_tasksets *in, const capart_options *opt,
                                const capart_alg1_results *out)
{
    if (!opt) return fail(c, CAPART_E_INVAL, "options is NULL");
    if (opt->K < 1 || opt->K > CAPART_MAX_K) return fail(c, CAPART_E_INVAL, "K must be in [1, 8]");
    if (opt->policy != CAPART_POLICY_FP_DM && opt->policy != CAPART_POLICY_EDF)
        return fail(c, CAPART_E_INVAL, "unsupported policy");
    if (opt->alloc_mode < CAPART_HEUR_BF_INA || opt->alloc_mode > CAPART_HEUR_SMS_ACT)
        return fail(c, CAPART_E_INVAL, "Algorithm 1 needs a heuristic order (CAPART_HEUR_*)");
    if (opt->admissible[0] | opt->admissible[1] | opt->admissible[2] | opt->admissible[3])
        return fail(c, CAPART_E_INVAL, "Algorithm 1 takes every partition size (admissible must be empty)");
    if (opt->flags & ~(CAPART_FLAG_SKIP_1G | CAPART_FLAG_NO_LEMMA1 | CAPART_FLAG_PER_SET_LAUNCH))
        return fail(c, CAPART_E_INVAL, "unknown flag");
    capart_status rc = check_batch_shape(c, in, CAPART_ALG1_MAX_TASKS);
    if (rc != CAPART_OK) return rc;
    if (in->max_tasks > CAPART_MAX_TASKS) {
        if (opt->policy != CAPART_POLICY_FP_DM)
            return fail(c, CAPART_E_INVAL, "sets of more than 64 tasks take the fixed-priority policy");
        if (in->max_M > CAPART_ALG1_BIG_MAX_M)
            return fail(c, CAPART_E_INVAL, "sets of more than 64 tasks take max_M <= 127");
    }
    if (in->n_sets > 0 && (!out || !out->status || !out->verdict || !out->nparts || !out->tried || !out->merged))
        return fail(c, CAPART_E_INVAL, "NULL result array");
    if (in->n_tasks_total > 0 && (!out->sizes || !out->alloc || !out->R))
        return fail(c, CAPART_E_INVAL, "NULL result array");
    return CAPART_OK;
}

// Prep and Algorithm 1 launches on st; with counts, the counting variant, and
// counts[0..1] get the response-time terms and exact tests (synchronous).
static capart_status alg1_run(capart_ctx *c, const capart_tasksets *in, const capart_options *opt,
                              capart_alg1_results *out, hipStream_t st, int64_t *counts)
{
    capart_status rc;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    const WsLayout l = ws_layout(in->n_sets, in->n_tasks_total, 1);
    if ((rc = ensure_ws(c, l.total + (counts ? 256 : 0))) != CAPART_OK) return rc;
    Work w = bind_work(c, l);
    if (counts) w.counters = (uint64_t *)((char *)c->ws + l.total);
    Launch L{};
    L.s0 = 0;
    L.S = in->n_sets;
    L.K = 1;
    L.mode = opt->alloc_mode;
    L.flags = opt->flags & CAPART_FLAG_NO_LEMMA1;
    L.edf = opt->policy == CAPART_POLICY_EDF;
    L.table_words = (int)(table_lds_bytes(in->max_tasks, in->max_M) / 4);
    const Batch b = make_batch(in);
    give_tables(w, b);
    Out po{};
    po.status = out->status;
    const A1Out a{out->status, out->verdict, out->nparts, out->sizes, out->alloc, out->R, out->tried, out->merged,
                  out->workload};
    std::array<hipEvent_t, 4> ev{};
    const bool tm = c->timing && !counts;
    if (tm)
        for (auto &x : ev)
            if (!(x = take_event(c))) return fail(c, CAPART_E_DEVICE, "hipEventCreate failed");
    (void)hipGetLastError();
    if (counts && (e = hipMemsetAsync(w.counters, 0, 16, st)) != hipSuccess) return hip_fail(c, e, "hipMemsetAsync");
    const bool big = in->max_tasks > CAPART_MAX_TASKS;  // one block of 256 threads per set
    if (tm) hipEventRecord(ev[0], st);
    if ((e = big ? launch_prep_big(b, w, po, L, st) : launch_prep(b, w, po, L, st)) != hipSuccess)
        return hip_fail(c, e, "prep launch");
    if (tm) hipEventRecord(ev[1], st);
    if ((e = big ? launch_alg1_big(b, w, a, L, st, counts != nullptr) : launch_alg1(b, w, a, L, st, counts != nullptr)) !=
        hipSuccess)
        return hip_fail(c, e, "Algorithm 1 launch");
    if (tm) {
        hipEventRecord(ev[2], st);
        hipEventRecord(ev[3], st);
        c->ev_pending.push_back(ev);
    }
    if (counts) {
        uint64_t h[2] = {0, 0};
        if ((e = hipMemcpyAsync(h, w.counters, 16, hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (e = hipStreamSynchronize(st)) != hipSuccess)
            return hip_fail(c, e, "reading counters");
        counts[0] = (int64_t)h[0];
        counts[1] = (int64_t)h[1];
    }
    return CAPART_OK;
}

capart_status capart_alg1_async(capart_ctx *c, const capart_tasksets *in, const capart_options *opt,
                                capart_alg1_results *out, void *hip_stream)
{
    if (!c) return CAPART_E_INVAL;
    capart_status rc;
    if ((rc = alg1_check(c, in, opt, out)) != CAPART_OK) return rc;
    if (in->n_sets == 0) return CAPART_OK;
    return alg1_run(c, in, opt, out, (hipStream_t)hip_stream, nullptr);
}

capart_status capart_alg1_count_work(capart_ctx *c, const capart_tasksets *in, const capart_options *opt,
                                     capart_alg1_results *out, void *hip_stream, int64_t *counts)
{
    if (!c || !counts) return CAPART_E_INVAL;
    capart_status rc;
    if ((rc = alg1_check(c, in, opt, out)) != CAPART_OK) return rc;
    counts[0] = counts[1] = 0;
    if (in->n_sets == 0) return CAPART_OK;
    return alg1_run(c, in, opt, out, (hipStream_t)hip_stream, counts);
}

capart_status capart_alg1(capart_ctx *c, const capart_tasksets *in, const capart_options *opt,
                          capart_alg1_results *out)
{
    if (!c) return CAPART_E_INVAL;
    capart_status rc;
    if ((rc = alg1_check(c, in, opt, out)) != CAPART_OK) return rc;
    if (in->n_sets == 0) return CAPART_OK;
    if (in->set_offset[0] != 0 || in->set_offset[in->n_sets] != in->n_tasks_total)
        return fail(c, CAPART_E_INVAL, "set_offset must run from 0 to n_tasks_total");
    const int64_t S = in->n_sets, N = in->n_tasks_total;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    size_t need = 0;
    auto add = [&](size_t bytes) { need = align256(need + std::max<size_t>(bytes, 1)); };
    add(8 * (S + 1)); add(4 * S);
    add(8 * N); add(8 * N); add(8 * N); add(8 * N); add(4 * N); add(N);
    add(4 * S); add(S); add(4 * S); add(4 * N); add(N); add(8 * N); add(8 * S); add(8 * S); add(8 * S);
    const int64_t TL = has_tables(in) ? in->table_len : 0;
    if (TL) { add(8 * S); add(8 * TL); add(8 * TL); }
    if ((rc = ensure_stage(c, need)) != CAPART_OK) return rc;
    Bump bp{(char *)c->stage};
    capart_tasksets d = *in;
    int64_t *d_off = bp.take<int64_t>(S + 1);
    int32_t *d_M = bp.take<int32_t>(S);
    int64_t *d_T = bp.take<int64_t>(N), *d_D = bp.take<int64_t>(N), *d_Cs = bp.take<int64_t>(N),
            *d_Cp = bp.take<int64_t>(N);
    int32_t *d_k = bp.take<int32_t>(N);
    uint8_t *d_ty = bp.take<uint8_t>(N);
    capart_alg1_results r;
    r.status = bp.take<int32_t>(S);
    r.verdict = bp.take<uint8_t>(S);
    r.nparts = bp.take<int32_t>(S);
    r.sizes = bp.take<int32_t>(N);
    r.alloc = bp.take<int8_t>(N);
    r.R = bp.take<int64_t>(N);
    r.tried = bp.take<int64_t>(S);
    r.merged = bp.take<int64_t>(S);
    r.workload = out->workload ? bp.take<uint64_t>(S) : nullptr;
    const hipStream_t st = c->stream;
    struct Cp { void *dst; const void *src; size_t n; } h2d[] = {
        {d_off, in->set_offset, 8 * (size_t)(S + 1)}, {d_M, in->M, 4 * (size_t)S},
        {d_T, in->T, 8 * (size_t)N}, {d_D, in->D, 8 * (size_t)N}, {d_Cs, in->C_seq, in->C_seq ? 8 * (size_t)N : 0},
        {d_Cp, in->C_par, in->C_par ? 8 * (size_t)N : 0}, {d_k, in->k_permille, in->k_permille ? 4 * (size_t)N : 0}, {d_ty, in->type, (size_t)N}};
    for (const auto &x : h2d)
        if (x.n && (e = hipMemcpyAsync(x.dst, x.src, x.n, hipMemcpyHostToDevice, st)) != hipSuccess)
            return hip_fail(c, e, "hipMemcpyAsync H2D");
    d.set_offset = d_off; d.M = d_M; d.T = d_T; d.D = d_D; d.C_seq = d_Cs; d.C_par = d_Cp; d.k_permille = d_k;
    d.type = d_ty;
    if (TL && (rc = stage_tables(c, in, bp, st, d)) != CAPART_OK) return rc;
    if ((rc = capart_alg1_async(c, &d, opt, &r, st)) != CAPART_OK) return rc;
    Cp d2h[] = {{out->status, r.status, 4 * (size_t)S}, {out->verdict, r.verdict, (size_t)S},
                {out->nparts, r.nparts, 4 * (size_t)S}, {out->sizes, r.sizes, 4 * (size_t)N},
                {out->alloc, r.alloc, (size_t)N}, {out->R, r.R, 8 * (size_t)N},
                {out->tried, r.tried, 8 * (size_t)S}, {out->merged, r.merged, 8 * (size_t)S},
                {out->workload, r.workload, out->workload ? 8 * (size_t)S : 0}};
    for (const auto &x : d2h)
        if (x.n && (e = hipMemcpyAsync(x.dst, x.src, x.n, hipMemcpyDeviceToHost, st)) != hipSuccess)
            return hip_fail(c, e, "hipMemcpyAsync D2H");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
    return CAPART_OK;
}

static capart_status one_set_check(capart_ctx *c, const capart_tasksets *one, const int32_t *sizes, int32_t k)
{
    if (!c) return CAPART_E_INVAL;
    capart_status rc = check_batch_shape(c, one);
    if (rc != CAPART_OK) return rc;
    if (has_tables(one)) return fail(c, CAPART_E_INVAL, "explicit time tables are taken by capart_solve, not here");
    if (one->n_sets != 1 || one->set_offset[0] != 0 || one->set_offset[1] != one->n_tasks_total)
        return fail(c, CAPART_E_INVAL, "expected exactly one set with offsets {0, n}");
    if (!sizes || k < 1 || k > CAPART_MAX_K) return fail(c, CAPART_E_INVAL, "k must be in [1, 8]");
    int64_t sum = 0;
    for (int p = 0; p < k; p++) {
        if (sizes[p] < 1) return fail(c, CAPART_E_INVAL, "part sizes must be >= 1");
        sum += sizes[p];
    }
    if (sum > one->M[0]) return fail(c, CAPART_E_INVAL, "parts exceed M");
    return CAPART_OK;
}

capart_status capart_test_triple(capart_ctx *c, const capart_tasksets *one, const int32_t *sizes, int32_t k,
                                 const int8_t *alloc, uint8_t *feasible, int64_t *R, uint64_t *maxU, uint64_t *sumU)
{
    capart_status rc = one_set_check(c, one, sizes, k);
    if (rc != CAPART_OK) return rc;
    const int64_t n = one->n_tasks_total;
    if (!alloc || !feasible || !R || !maxU || !sumU) return fail(c, CAPART_E_INVAL, "NULL argument");
    for (int64_t i = 0; i < n; i++)
        if (alloc[i] < 0 || alloc[i] >= k) return fail(c, CAPART_E_INVAL, "allocation index out of [0, k)");
    int32_t st_host = validate_set(one, 0, CAPART_MAX_K, CAPART_HEUR_BF_INA);
    if (st_host != CAPART_OK) return fail(c, st_host, "invalid task set");
    // solve infrastructure: upload the set, run prep, then the triple kernel
    capart_options opt{CAPART_MAX_K, CAPART_POLICY_FP_DM, CAPART_HEUR_BF_INA, 0u};
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    if ((rc = ensure_stage(c, stage_need(1, n, CAPART_MAX_K, 0) + 4096)) != CAPART_OK) return rc;
    Bump bp{(char *)c->stage};
    int64_t *d_off = bp.take<int64_t>(2);
    int32_t *d_M = bp.take<int32_t>(1);
    int64_t *d_T = bp.take<int64_t>(n), *d_D = bp.take<int64_t>(n), *d_Cs = bp.take<int64_t>(n),
            *d_Cp = bp.take<int64_t>(n);
    int32_t *d_k = bp.take<int32_t>(n);
    uint8_t *d_ty = bp.take<uint8_t>(n);
    int32_t *d_sizes = bp.take<int32_t>(8);
    int8_t *d_alloc = bp.take<int8_t>(n);
    uint8_t *d_feas = bp.take<uint8_t>(1);
    int64_t *d_R = bp.take<int64_t>(n);
    uint64_t *d_mx = bp.take<uint64_t>(1), *d_sm = bp.take<uint64_t>(1);
    int32_t *d_status = bp.take<int32_t>(1);
    hipStream_t st = c->stream;
    const int64_t offs[2] = {0, n};
    struct Cp { void *dst; const void *src; size_t n; } h2d[] = {
        {d_off, offs, 16}, {d_M, one->M, 4}, {d_T, one->T, 8 * (size_t)n}, {d_D, one->D, 8 * (size_t)n},
        {d_Cs, one->C_seq, 8 * (size_t)n}, {d_Cp, one->C_par, 8 * (size_t)n}, {d_k, one->k_permille, 4 * (size_t)n},
        {d_ty, one->type, (size_t)n}, {d_sizes, sizes, 4 * (size_t)k}, {d_alloc, alloc, (size_t)n}};
    for (const auto &x : h2d)
        if ((e = hipMemcpyAsync(x.dst, x.src, x.n, hipMemcpyHostToDevice, st)) != hipSuccess)
            return hip_fail(c, e, "hipMemcpyAsync H2D");
    capart_tasksets d = *one;
    d.set_offset = d_off; d.M = d_M; d.T = d_T; d.D = d_D; d.C_seq = d_Cs; d.C_par = d_Cp; d.k_permille = d_k;
    d.type = d_ty;
    const Plan p = make_plan(&d, &opt, c->tune);
    const WsLayout l = ws_layout(1, n, p.L.chunks);
    if ((rc = ensure_ws(c, l.total)) != CAPART_OK) return rc;
    char *base = (char *)c->ws;
    Work w{};
    w.rec = (TaskRec *)(base + l.rec);
    w.forbid = (uint64_t *)(base + l.forbid);
    w.sigma = (uint8_t *)(base + l.sigma);
    w.setflags = (uint32_t *)(base + l.setflags);
    w.memmask = (uint64_t *)(base + l.memmask);
    w.partial = (uint64_t *)(base + l.partial);
    w.np = c->np_dev;
    w.order = c->order_dev;
    Out o{};
    o.status = d_status;
    const Batch b = make_batch(&d);
    if ((e = launch_prep(b, w, o, p.L, st)) != hipSuccess) return hip_fail(c, e, "prep launch");
    if ((e = launch_triple(b, w, d_sizes, k, d_alloc, d_feas, d_R, d_mx, d_sm, st)) != hipSuccess)
        return hip_fail(c, e, "triple launch");
    Cp d2h[] = {{feasible, d_feas, 1}, {R, d_R, 8 * (size_t)n}, {maxU, d_mx, 8}, {sumU, d_sm, 8}};
    for (const auto &x : d2h)
        if ((e = hipMemcpyAsync(x.dst, x.src, x.n, hipMemcpyDeviceToHost, st)) != hipSuccess)
            return hip_fail(c, e, "hipMemcpyAsync D2H");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
    return CAPART_OK;
}

capart_status capart_allocate(capart_ctx *c, const capart_tasksets *one, const int32_t *sizes, int32_t k,
                              const capart_options *opt, int8_t *alloc_out, uint8_t *found, uint64_t *maxU,
                              uint64_t *sumU, int64_t *aidx)
{
    capart_status rc = one_set_check(c, one, sizes, k);
    if (rc != CAPART_OK) return rc;
    if ((rc = check_options(c, opt)) != CAPART_OK) return rc;
    if (!alloc_out || !found || !maxU || !sumU || !aidx) return fail(c, CAPART_E_INVAL, "NULL argument");
    const int32_t M = one->M[0];
    if (k > opt->K) return fail(c, CAPART_E_INVAL, "k exceeds K");
    int64_t sum = 0;
    for (int p = 0; p < k; p++) {
        if (p > 0 && sizes[p] > sizes[p - 1]) return fail(c, CAPART_E_INVAL, "sizes must be non-increasing");
        sum += sizes[p];
    }
    if (sum != M) return fail(c, CAPART_E_INVAL, "sizes must sum to M");
    // index of this partitioning in canonical order
    const int64_t P = count_parts(M, opt->K);
    std::vector<int32_t> tab((size_t)P * opt->K);
    int64_t cnt = 0;
    capart_enumerate_partitionings(M, opt->K, tab.data(), P, &cnt);
    int64_t pidx = -1;
    for (int64_t q = 0; q < P && pidx < 0; q++) {
        bool eq = true;
        for (int p = 0; p < opt->K; p++)
            if (tab[q * opt->K + p] != (p < k ? sizes[p] : 0)) { eq = false; break; }
        if (eq) pidx = q;
    }
    if (pidx < 0) return fail(c, CAPART_E_INVAL, "not a partitioning of M");
    // solve the set on this partitioning alone
    const int64_t n = one->n_tasks_total;
    std::vector<int32_t> status(1), pid(1), szs(opt->K);
    std::vector<uint8_t> verdict(1), v1g(1);
    std::vector<int64_t> ai(1), ne(1), R(n), R1(n);
    std::vector<uint64_t> mx(1), sm(1);
    std::vector<int8_t> al(n);
    capart_results r{status.data(), verdict.data(), v1g.data(), pid.data(), szs.data(), ai.data(), mx.data(),
                     sm.data(), ne.data(), al.data(), R.data(), R1.data(), nullptr, nullptr};
    capart_options o1 = *opt;
    o1.flags |= CAPART_FLAG_SKIP_1G;
    if ((rc = solve_host(c, one, &o1, &r, (uint32_t)pidx, (uint32_t)pidx + 1u)) != CAPART_OK) return rc;
    if (status[0] != CAPART_OK) return fail(c, status[0], "invalid task set");
    *found = verdict[0];
    *maxU = mx[0];
    *sumU = sm[0];
    *aidx = ai[0];
    for (int64_t i = 0; i < n; i++) alloc_out[i] = *found ? al[i] : (int8_t)-1;
    return CAPART_OK;
}

capart_status capart_count_work(capart_ctx *c, const capart_tasksets *in, const capart_options *opt,
                                capart_results *out, void *hip_stream, int64_t *counts)
{
    if (!c || !counts) return CAPART_E_INVAL;
    capart_status rc;
    if ((rc = check_options(c, opt)) != CAPART_OK) return rc;
    if ((rc = check_batch_shape(c, in)) != CAPART_OK) return rc;
    if (opt->flags & CAPART_FLAG_PER_SET_LAUNCH)
        return fail(c, CAPART_E_INVAL, "work counting covers batched solves");
    if (!results_ok(out)) return fail(c, CAPART_E_INVAL, "NULL result array");
    counts[0] = counts[1] = counts[2] = 0;
    if (in->n_sets == 0) return CAPART_OK;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    const Plan p = make_plan(in, opt, c->tune);
    if (p.L.mode == CAPART_EXHAUSTIVE && p.L.exh_form != 2)
        return fail(c, CAPART_E_INVAL, "work counting of exhaustive solves covers the subset-table search");
    const WsLayout l = ws_layout(p.S, p.N, p.L.chunks);
    if ((rc = ensure_ws(c, l.total + 256)) != CAPART_OK) return rc;
    char *base = (char *)c->ws;
    Work w{};
    w.rec = (TaskRec *)(base + l.rec);
    w.forbid = (uint64_t *)(base + l.forbid);
    w.sigma = (uint8_t *)(base + l.sigma);
    w.setflags = (uint32_t *)(base + l.setflags);
    w.memmask = (uint64_t *)(base + l.memmask);
    w.partial = (uint64_t *)(base + l.partial);
    w.np = c->np_dev;
    w.order = c->order_dev;
    w.counters = (uint64_t *)(base + l.total);
    hipStream_t st = (hipStream_t)hip_stream;
    const Batch b = make_batch(in);
    give_tables(w, b);
    const Out o = make_out(out);
    (void)hipGetLastError();
    if ((e = hipMemsetAsync(w.counters, 0, 24, st)) != hipSuccess) return hip_fail(c, e, "hipMemsetAsync");
    if (p.L.mode == CAPART_EXHAUSTIVE) {
        // subset tables (partition tests and their terms) and the pruned
        // search (table lookups) count through w.counters
        const bool tm = c->timing;
        c->timing = false;
        rc = launch_three(c, b, w, o, p.L, st, 0u, 0xFFFFFFFFu);
        c->timing = tm;
        if (rc != CAPART_OK) return rc;
    } else {
        if ((e = launch_prep(b, w, o, p.L, st)) != hipSuccess) return hip_fail(c, e, "prep launch");
        if ((e = launch_eval_count(b, w, o, p.L, st)) != hipSuccess) return hip_fail(c, e, "counting eval launch");
        if ((e = launch_final(b, w, o, p.L, st)) != hipSuccess) return hip_fail(c, e, "final launch");
    }
    uint64_t h[3] = {0, 0, 0};
    if ((e = hipMemcpyAsync(h, w.counters, 24, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(c, e, "reading counters");
    for (int i = 0; i < 3; i++) counts[i] = (int64_t)h[i];
    return CAPART_OK;
}

capart_status capart_set_tuning(capart_ctx *c, const capart_tuning *t)
{
    if (!c) return CAPART_E_INVAL;
    if (!t) {
        c->tune = capart_tuning{};
        return CAPART_OK;
    }
    if (t->threads < 0 || t->threads > 256 || (t->threads % 64) != 0)
        return fail(c, CAPART_E_INVAL, "threads must be 0 or a multiple of 64 up to 256");
    if (t->chunk < 0) return fail(c, CAPART_E_INVAL, "chunk must be >= 0");
    if (t->loop_form < 0 || t->loop_form > 3) return fail(c, CAPART_E_INVAL, "loop_form must be 0, 1, 2 or 3");
    if (t->exh_form < 0 || t->exh_form > 2) return fail(c, CAPART_E_INVAL, "exh_form must be 0, 1 or 2");
    if (t->frontier < 0 || t->frontier > 2) return fail(c, CAPART_E_INVAL, "frontier must be 0, 1 or 2");
    if (t->reserved) return fail(c, CAPART_E_INVAL, "reserved must be 0");
    if (t->wide_chunk < -1 || t->wide_chunk > 4096) return fail(c, CAPART_E_INVAL, "wide_chunk must be -1..4096");
    if (t->memo != 0 && t->memo != -1 && (t->memo < 8 || t->memo > MEMO_MAX_LOG2))
        return fail(c, CAPART_E_INVAL, "memo must be 0, -1 or 8..13");
    c->tune = *t;
    return CAPART_OK;
}

capart_status capart_get_tuning(const capart_ctx *c, capart_tuning *t)
{
    if (!c || !t) return CAPART_E_INVAL;
    *t = c->tune;
    return CAPART_OK;
}

capart_status capart_timing_enable(capart_ctx *c, int enable)
{
    if (!c) return CAPART_E_INVAL;
    c->timing = enable != 0;
    if (!c->timing) {
        for (auto &a : c->ev_pending)
            for (auto e : a) c->ev_free.push_back(e);
        c->ev_pending.clear();
    }
    return CAPART_OK;
}

capart_status capart_timing_read(capart_ctx *c, double *ms, int64_t *launches)
{
    if (!c || !ms || !launches) return CAPART_E_INVAL;
    double acc[3] = {0, 0, 0};
    for (auto &a : c->ev_pending) {
        hipError_t e = hipEventSynchronize(a[3]);
        if (e != hipSuccess) return hip_fail(c, e, "hipEventSynchronize");
        for (int k = 0; k < 3; k++) {
            float t = 0.f;
            if ((e = hipEventElapsedTime(&t, a[k], a[k + 1])) != hipSuccess) return hip_fail(c, e, "hipEventElapsedTime");
            acc[k] += t;
        }
    }
    for (int k = 0; k < 3; k++) {
        ms[k] = acc[k];
        launches[k] = (int64_t)c->ev_pending.size();
    }
    for (auto &a : c->ev_pending)
        for (auto e : a) c->ev_free.push_back(e);
    c->ev_pending.clear();
    return CAPART_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched form (plan / run).
struct capart_plan {
    capart_ctx *ctx = nullptr;
    capart_tasksets in{};
    capart_options opt{};
    capart_results out{};
    Launch L{};
    int blocks = 0;
    bool use_graph = true;
    void *buf = nullptr;
    Work w{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    capart_plan_info info{};
};

namespace {

struct PlanLayout {
    size_t rec, forbid, sigma, setflags, memmask, partial, items, slot_off, counter, partial_direct, total;
};

// direct_slots: partial keys of the one-block-per-(set, chunk) schedule (0 = none)
PlanLayout plan_layout(int64_t S, int64_t N, int64_t n_items, int64_t direct_slots)
{
    PlanLayout l;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align256(o + std::max<size_t>(bytes, 1)); return at; };
    l.rec = take(sizeof(TaskRec) * (size_t)N);
    l.forbid = take(8 * (size_t)N);
    l.sigma = take((size_t)N);
    l.setflags = take(4 * (size_t)S);
    l.memmask = take(8 * (size_t)S);
    l.partial = take(32 * (size_t)n_items);
    l.items = take(sizeof(WorkItem) * (size_t)n_items);
    l.slot_off = take(4 * (size_t)(S + 1));
    l.counter = take(12);
    l.partial_direct = take(32 * (size_t)direct_slots);
    l.total = o;
    return l;
}

// Work items: each set's partitionings cut into ranges of about
// item_evals * 121 / (n+1)^2 partitionings (the response-time work of a
// partitioning grows roughly with n^2), queued by decreasing estimated cost.
// Sets of at most this many tasks go to one work item each (their frontier or
// test memo then serves all of their partitionings).
int single_item_n(const Launch &L) { return std::max(L.front_n, L.memo_log2 > 0 ? NARROW_MAX_TASKS : 0); }

// Items are grouped by the size class of their set (classes ascending, see
// size_classes; each class is evaluated by a launch of its own with its own
// queue), and within a class queued by decreasing estimated cost.
void build_items(const std::vector<int64_t> &off, const std::vector<int32_t> &M, int64_t S, const capart_tasksets *in,
                 int K, int item_evals, const Launch &L, std::vector<WorkItem> &items,
                 std::vector<uint32_t> &slot_off, int64_t &total_evals, uint32_t class_end[3])
{
    const int single_n = single_item_n(L);
    int hi[3];
    const int nc = size_classes(L, in->max_tasks, hi);
    items.clear();
    slot_off.assign((size_t)S + 1, 0u);
    total_evals = 0;
    std::vector<uint64_t> cost;
    for (int64_t s = 0; s < S; s++) {
        slot_off[s] = (uint32_t)items.size();
        const int64_t n = off[s + 1] - off[s];
        const int32_t m = M[s];
        if (off[s] < 0 || n < 1 || n > std::min(in->max_tasks, CAPART_MAX_TASKS) || m < 1 ||
            m > std::min(in->max_M, CAPART_MAX_M) || n * m > CAPART_MAX_NM)
            continue;
        const uint32_t P = count_parts(m, K);
        total_evals += P;
        const uint64_t w = (uint64_t)(n + 1) * (uint64_t)(n + 1);
        uint32_t per = (uint32_t)std::max<uint64_t>(64, std::min<uint64_t>(1u << 20, (uint64_t)item_evals * 121 / w));
        // one item per set when its frontier or memo is built once for all partitionings
        if (n <= single_n) per = std::max<uint32_t>(P, 1);
        for (uint32_t p0 = 0; p0 < P; p0 += per) {
            const uint32_t p1 = std::min(P, p0 + per);
            items.push_back(WorkItem{(uint32_t)s, p0, p1, (uint32_t)items.size()});
            cost.push_back((uint64_t)(p1 - p0) * w);
        }
    }
    slot_off[S] = (uint32_t)items.size();
    std::vector<uint32_t> order(items.size());
    std::vector<uint8_t> cls(items.size());
    uint32_t count[3] = {0u, 0u, 0u};
    for (size_t i = 0; i < order.size(); i++) {
        order[i] = (uint32_t)i;
        const int64_t n = off[items[i].set + 1] - off[items[i].set];
        int c = 0;
        while (c + 1 < nc && n > hi[c]) c++;
        cls[i] = (uint8_t)c;
        count[c]++;
    }
    class_end[0] = count[0];
    class_end[1] = count[0] + count[1];
    class_end[2] = count[0] + count[1] + count[2];
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t a, uint32_t b) { return cls[a] != cls[b] ? cls[a] < cls[b] : cost[a] > cost[b]; });
    std::vector<WorkItem> sorted(items.size());
    for (size_t i = 0; i < order.size(); i++) sorted[i] = items[order[i]];
    items.swap(sorted);
}

struct PlanBuffers {
    void *buf = nullptr;
    Work w{};   // persistent schedule (work items, queues)
    Work wd{};  // direct schedule: one block per (set, chunk), partial keys by chunk
};

capart_status alloc_plan_buffers(capart_ctx *c, int64_t S, int64_t N, const std::vector<WorkItem> &items,
                                 const std::vector<uint32_t> &slot_off, const uint32_t class_end[3],
                                 int64_t direct_slots, PlanBuffers &pb)
{
    const PlanLayout l = plan_layout(S, N, (int64_t)items.size(), direct_slots);
    hipError_t e = hipMalloc(&pb.buf, l.total);
    if (e != hipSuccess) {
        pb.buf = nullptr;
        return fail(c, CAPART_E_NOMEM, "plan workspace allocation failed");
    }
    char *base = (char *)pb.buf;
    pb.w.rec = (TaskRec *)(base + l.rec);
    pb.w.forbid = (uint64_t *)(base + l.forbid);
    pb.w.sigma = (uint8_t *)(base + l.sigma);
    pb.w.setflags = (uint32_t *)(base + l.setflags);
    pb.w.memmask = (uint64_t *)(base + l.memmask);
    pb.w.partial = (uint64_t *)(base + l.partial);
    pb.w.items = (const WorkItem *)(base + l.items);
    pb.w.n_items = (uint32_t)items.size();
    for (int i = 0; i < 3; i++) pb.w.class_end[i] = class_end[i];
    pb.w.counter = (uint32_t *)(base + l.counter);
    pb.w.slot_off = (const uint32_t *)(base + l.slot_off);
    pb.w.np = c->np_dev;
    pb.w.order = c->order_dev;
    pb.wd = pb.w;
    pb.wd.partial = (uint64_t *)(base + l.partial_direct);
    pb.wd.items = nullptr;
    pb.wd.n_items = 0;
    for (int i = 0; i < 3; i++) pb.wd.class_end[i] = 0u;
    pb.wd.counter = nullptr;
    pb.wd.slot_off = nullptr;
    if (!items.empty() &&
        (e = hipMemcpy(base + l.items, items.data(), sizeof(WorkItem) * items.size(), hipMemcpyHostToDevice)) !=
            hipSuccess)
        return hip_fail(c, e, "hipMemcpy items");
    if ((e = hipMemcpy(base + l.slot_off, slot_off.data(), 4 * slot_off.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(c, e, "hipMemcpy slot offsets");
    return CAPART_OK;
}

capart_status launch_plan_kernels(capart_ctx *c, const Batch &b, const Work &w0, const Out &o, const Launch &L,
                                  int blocks, hipStream_t st, bool timed)
{
    Work w = w0;
    give_tables(w, b);  // explicit time tables, where the batch has them
    std::array<hipEvent_t, 4> ev{};
    if (timed)
        for (auto &e : ev)
            if (!(e = take_event(c))) return fail(c, CAPART_E_DEVICE, "hipEventCreate failed");
    hipError_t e;
    (void)hipGetLastError();
    if (timed) hipEventRecord(ev[0], st);
    if ((e = launch_prep(b, w, o, L, st)) != hipSuccess) return hip_fail(c, e, "prep launch");
    if (timed) hipEventRecord(ev[1], st);
    // blocks == 0: the direct schedule (one block per set chunk), else a persistent grid
    if ((e = blocks > 0 ? launch_eval_persistent(b, w, o, L, blocks, st) : launch_eval(b, w, o, L, st)) != hipSuccess)
        return hip_fail(c, e, "eval launch");
    if (timed) hipEventRecord(ev[2], st);
    if ((e = launch_final(b, w, o, L, st)) != hipSuccess) return hip_fail(c, e, "final launch");
    if (timed) {
        hipEventRecord(ev[3], st);
        c->ev_pending.push_back(ev);
    }
    return CAPART_OK;
}

Launch plan_launch(const capart_tasksets *in, const capart_options *opt, int threads, int form,
                   const capart_tuning &tune)
{
    Launch L{};
    L.s0 = 0;
    L.S = in->n_sets;
    L.K = opt->K;
    L.mode = opt->alloc_mode;
    L.flags = opt->flags & ~CAPART_FLAG_PER_SET_LAUNCH;
    for (int i = 0; i < 4; i++) L.adm.w[i] = opt->admissible[i];
    L.edf = opt->policy == CAPART_POLICY_EDF;
    L.threads = std::min(threads, eval_threads(in->max_tasks, in->max_M));
    L.table_words = (int)(table_lds_bytes(in->max_tasks, in->max_M) / 4);
    L.form = form == 2 ? 2 : 1;
    L.memo_packed = form == 3;
    L.chunks = 1;
    L.chunk = 0;
    L.exh_form = 1;
    capart_tuning tf = tune;
    if (tf.frontier == 0 && !frontier_pays(in->max_tasks, in->max_M, opt->K, L.adm)) tf.frontier = 2;
    size_frontier(L, in->max_tasks, opt->alloc_mode, tf);
    return L;
}

}  // namespace

extern "C" {

capart_status capart_plan_batch(capart_ctx *c, const capart_tasksets *in, const capart_options *opt,
                                const capart_results *out, const capart_plan_config *cfg, capart_plan **plan_out)
{
    if (!c || !plan_out) return CAPART_E_INVAL;
    *plan_out = nullptr;
    capart_status rc;
    if ((rc = check_options(c, opt)) != CAPART_OK) return rc;
    if ((rc = check_batch_shape(c, in)) != CAPART_OK) return rc;
    if (opt->alloc_mode == CAPART_EXHAUSTIVE) return fail(c, CAPART_E_INVAL, "the batched form runs heuristic modes");
    if (in->n_sets < 1) return fail(c, CAPART_E_INVAL, "empty batch");
    if (!results_ok(out)) return fail(c, CAPART_E_INVAL, "NULL result array");
    const capart_plan_config def{1, 0, 0, 1};
    const capart_plan_config &cf = cfg ? *cfg : def;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    const int64_t S = in->n_sets, N = in->n_tasks_total;
    std::vector<int64_t> off((size_t)S + 1);
    std::vector<int32_t> M((size_t)S);
    if ((e = hipMemcpy(off.data(), in->set_offset, 8 * (size_t)(S + 1), hipMemcpyDeviceToHost)) != hipSuccess ||
        (e = hipMemcpy(M.data(), in->M, 4 * (size_t)S, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(c, e, "reading set sizes");
    const Batch b = make_batch(in);
    const Out o = make_out(out);
    const int cus = device_cu_count();
    int threads = c->tune.threads > 0 ? c->tune.threads : 256;
    int form = c->tune.loop_form > 0 ? c->tune.loop_form : 1;
    int item_evals = cf.item_evals > 0 ? cf.item_evals : 4096;
    int bpc = cf.blocks_per_cu > 0 ? cf.blocks_per_cu : 4;
    int tried = 0;
    const auto t0 = std::chrono::steady_clock::now();
    if (cf.autotune) {
        // candidates timed on a prefix of the batch (sets are independent
        // draws, so a prefix has the batch's mix of sizes); the search stops
        // early once it has spent a few seconds
        const int64_t St = std::min<int64_t>(S, std::max<int64_t>(8192, S / 64));
        capart_tasksets sub = *in;
        sub.n_sets = St;
        sub.n_tasks_total = off[St];
        const Batch bs = make_batch(&sub);
        double best_ms = 1e300;
        const int th_c[] = {128, 256};
        const int form_c[] = {1, 2};
        const int ie_c[] = {4096, 16384};
        const int bpc_c[] = {4, 8};
        // time one candidate (two runs on the prefix, the second timed)
        auto time_it = [&](const Work &w, const Launch &L, int blocks, double &ms) -> capart_status {
            hipEvent_t e0 = take_event(c), e1 = take_event(c);
            capart_status r = CAPART_OK;
            for (int rep = 0; rep < 2 && r == CAPART_OK; rep++) {
                if (rep == 1) hipEventRecord(e0, c->stream);
                r = launch_plan_kernels(c, bs, w, o, L, blocks, c->stream, false);
            }
            hipEventRecord(e1, c->stream);
            hipError_t se = hipEventSynchronize(e1);
            float f = 0.f;
            if (se == hipSuccess) se = hipEventElapsedTime(&f, e0, e1);
            ms = f;
            c->ev_free.push_back(e0);
            c->ev_free.push_back(e1);
            if (r != CAPART_OK) return r;
            if (se != hipSuccess) return hip_fail(c, se, "autotune timing");
            return CAPART_OK;
        };
        auto over_budget = [&]() {
            return tried > 0 && std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > 5.0;
        };
        if (cf.blocks_per_cu >= 0) {
            for (int th : th_c)
                for (int fo : form_c)
                    for (int ie : ie_c)
                        for (int bp : bpc_c) {
                            if (cf.item_evals > 0 && ie != ie_c[0]) continue;
                            if (cf.blocks_per_cu > 0 && bp != bpc_c[0]) continue;
                            if (over_budget()) continue;
                            // loop form 2 has no test memo: not a candidate when sets would use it
                            if (fo == 2 && plan_launch(&sub, opt, th, 1, c->tune).memo_log2 > 0) continue;
                            const int ie2 = cf.item_evals > 0 ? cf.item_evals : ie;
                            const int bp2 = cf.blocks_per_cu > 0 ? cf.blocks_per_cu : bp;
                            std::vector<WorkItem> items;
                            std::vector<uint32_t> so;
                            int64_t te = 0;
                            uint32_t ce[3];
                            const Launch L = plan_launch(&sub, opt, th, fo, c->tune);
                            build_items(off, M, St, in, opt->K, ie2, L, items, so, te, ce);
                            PlanBuffers pb;
                            if ((rc = alloc_plan_buffers(c, St, sub.n_tasks_total, items, so, ce, 0, pb)) !=
                                CAPART_OK) {
                                if (pb.buf) hipFree(pb.buf);
                                return rc;
                            }
                            double ms = 0;
                            rc = time_it(pb.w, L, cus * bp2, ms);
                            hipFree(pb.buf);
                            if (rc != CAPART_OK) return rc;
                            tried++;
                            if (ms < best_ms) {
                                best_ms = ms;
                                threads = th;
                                form = fo;
                                item_evals = ie2;
                                bpc = bp2;
                            }
                        }
        }
        // the direct schedule: one block per (set, chunk), no work queue
        if (cf.blocks_per_cu <= 0 && cf.item_evals <= 0)
            for (int th : th_c) {
                if (over_budget()) continue;
                capart_tuning tu = c->tune;
                tu.threads = th;
                const Plan dp = make_plan(&sub, opt, tu, wide_partitionings(off.data(), M.data(), St, opt->K));
                std::vector<WorkItem> none;
                std::vector<uint32_t> so((size_t)St + 1, 0u);
                PlanBuffers pb;
                const uint32_t ce0[3] = {0u, 0u, 0u};
                if ((rc = alloc_plan_buffers(c, St, sub.n_tasks_total, none, so, ce0, St * (int64_t)dp.L.chunks, pb)) !=
                    CAPART_OK) {
                    if (pb.buf) hipFree(pb.buf);
                    return rc;
                }
                double ms = 0;
                rc = time_it(pb.wd, dp.L, 0, ms);
                hipFree(pb.buf);
                if (rc != CAPART_OK) return rc;
                tried++;
                // the direct grid's tail weighs more on the prefix than on the
                // whole batch, so it is kept unless a queue is 5 % faster
                if (ms < (bpc > 0 ? best_ms * 1.05 : best_ms)) {
                    best_ms = ms;
                    threads = th;
                    bpc = 0;
                }
            }
    } else if (cf.blocks_per_cu < 0) {
        bpc = 0;
    }
    const double tune_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    capart_plan *pl = new (std::nothrow) capart_plan;
    if (!pl) return fail(c, CAPART_E_NOMEM, "plan allocation failed");
    pl->ctx = c;
    pl->in = *in;
    pl->opt = *opt;
    pl->out = *out;
    pl->use_graph = cf.use_graph != 0;
    std::vector<WorkItem> items;
    std::vector<uint32_t> so;
    int64_t te = 0;
    uint32_t ce[3] = {0u, 0u, 0u};
    const bool direct = bpc <= 0;
    capart_tuning tud = c->tune;
    tud.threads = threads;
    const Plan dp = make_plan(in, opt, tud, wide_partitionings(off.data(), M.data(), S, opt->K));
    const Launch Lp0 = plan_launch(in, opt, threads, form, c->tune);
    if (!direct) {
        build_items(off, M, S, in, opt->K, item_evals, Lp0, items, so, te, ce);
    } else {
        so.assign((size_t)S + 1, 0u);
        for (int64_t s2 = 0; s2 < S; s2++) {
            const int64_t n = off[s2 + 1] - off[s2];
            const int32_t m = M[s2];
            if (off[s2] >= 0 && n >= 1 && n <= std::min(in->max_tasks, CAPART_MAX_TASKS) && m >= 1 &&
                m <= std::min(in->max_M, CAPART_MAX_M) && n * m <= CAPART_MAX_NM)
                te += count_parts(m, opt->K);
        }
    }
    PlanBuffers pb;
    if ((rc = alloc_plan_buffers(c, S, N, items, so, ce, direct ? S * (int64_t)dp.L.chunks : 0, pb)) != CAPART_OK) {
        if (pb.buf) hipFree(pb.buf);
        delete pl;
        return rc;
    }
    pl->buf = pb.buf;
    pl->w = direct ? pb.wd : pb.w;
    pl->L = direct ? dp.L : Lp0;
    pl->blocks = direct ? 0 : cus * bpc;
    pl->info.n_sets = S;
    pl->info.n_items = (int64_t)items.size();
    pl->info.total_evals = te;
    pl->info.threads = pl->L.threads;
    pl->info.loop_form = direct ? pl->L.form : form;
    pl->info.blocks = pl->blocks;
    pl->info.item_evals = item_evals;
    pl->info.candidates_tried = tried;
    pl->info.use_graph = pl->use_graph ? 1 : 0;
    pl->info.tune_ms = tune_ms;
    if (pl->use_graph) {
        if ((e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
            capart_plan_destroy(pl);
            return hip_fail(c, e, "hipStreamBeginCapture");
        }
        rc = launch_plan_kernels(c, make_batch(in), pl->w, make_out(out), pl->L, pl->blocks, c->stream, false);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(c->stream, &g);
        if (rc != CAPART_OK || e != hipSuccess) {
            if (g) hipGraphDestroy(g);
            capart_plan_destroy(pl);
            return rc != CAPART_OK ? rc : hip_fail(c, e, "hipStreamEndCapture");
        }
        pl->graph = g;
        if ((e = hipGraphInstantiate(&pl->exec, g, nullptr, nullptr, 0)) != hipSuccess) {
            pl->exec = nullptr;
            capart_plan_destroy(pl);
            return hip_fail(c, e, "hipGraphInstantiate");
        }
    }
    *plan_out = pl;
    return CAPART_OK;
}

capart_status capart_run_batch(capart_plan *pl, void *hip_stream)
{
    if (!pl) return CAPART_E_INVAL;
    capart_ctx *c = pl->ctx;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    hipStream_t st = (hipStream_t)hip_stream;
    if (pl->use_graph && !c->timing) {
        if ((e = hipGraphLaunch(pl->exec, st)) != hipSuccess) return hip_fail(c, e, "hipGraphLaunch");
        return CAPART_OK;
    }
    return launch_plan_kernels(c, make_batch(&pl->in), pl->w, make_out(&pl->out), pl->L, pl->blocks, st, c->timing);
}

capart_status capart_plan_get_info(const capart_plan *pl, capart_plan_info *info)
{
    if (!pl || !info) return CAPART_E_INVAL;
    *info = pl->info;
    return CAPART_OK;
}

capart_status capart_plan_destroy(capart_plan *pl)
{
    if (!pl) return CAPART_E_INVAL;
    hipSetDevice(pl->ctx->device);
    hipDeviceSynchronize();
    if (pl->exec) hipGraphExecDestroy(pl->exec);
    if (pl->graph) hipGraphDestroy(pl->graph);
    if (pl->buf) hipFree(pl->buf);
    delete pl;
    return CAPART_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Serving form.
#include <atomic>
#include <condition_variable>
#include <mutex>
#include <thread>

namespace {

enum QState { Q_FREE = 0, Q_PENDING = 1, Q_LAUNCHED = 2, Q_DONE = 3 };

struct SrvQuery {
    uint64_t ticket = 0;
    int64_t t0 = 0;        // first task in the task ring
    int32_t n = 0, M = 0;
    bool tab = false;      // brings explicit time tables
    int state = Q_FREE;
    double t_arrival = 0;  // microseconds since the server's origin
    double t_done = 0;
};

// Packed per-batch layout (offsets in bytes, 256-aligned segments).
struct PackIn {
    size_t off, M, T, D, Cs, Cp, k, type, toff, Cn, Cc, total;
};
struct PackOut {
    size_t status, verdict, v1g, pidx, sizes, aidx, maxU, sumU, nev, alloc, R, R1g, total;
};

// NT: explicit time-table entries of each kind in the batch (0 without tables)
PackIn pack_in_layout(int64_t S, int64_t N, int64_t NT)
{
    PackIn l;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align256(o + std::max<size_t>(bytes, 1)); return at; };
    l.off = take(8 * (size_t)(S + 1));
    l.M = take(4 * (size_t)S);
    l.T = take(8 * (size_t)N);
    l.D = take(8 * (size_t)N);
    l.Cs = take(8 * (size_t)N);
    l.Cp = take(8 * (size_t)N);
    l.k = take(4 * (size_t)N);
    l.type = take((size_t)N);
    l.toff = take(NT ? 8 * (size_t)S : 0);
    l.Cn = take(8 * (size_t)NT);
    l.Cc = take(8 * (size_t)NT);
    l.total = o;
    return l;
}

PackOut pack_out_layout(int64_t S, int64_t N, int K)
{
    PackOut l;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align256(o + std::max<size_t>(bytes, 1)); return at; };
    l.status = take(4 * (size_t)S);
    l.verdict = take((size_t)S);
    l.v1g = take((size_t)S);
    l.pidx = take(4 * (size_t)S);
    l.sizes = take(4 * (size_t)S * K);
    l.aidx = take(8 * (size_t)S);
    l.maxU = take(8 * (size_t)S);
    l.sumU = take(8 * (size_t)S);
    l.nev = take(8 * (size_t)S);
    l.alloc = take((size_t)N);
    l.R = take(8 * (size_t)N);
    l.R1g = take(8 * (size_t)N);
    l.total = o;
    return l;
}

struct SrvStream {
    hipStream_t st = nullptr;
    hipEvent_t done = nullptr;
    char *in_host = nullptr, *out_host = nullptr;  // pinned
    char *in_dev = nullptr, *out_dev = nullptr;
    bool busy = false;
    uint64_t first = 0;  // first ticket of the batch in flight
    int64_t count = 0, ntasks = 0;
};

double now_us(const std::chrono::steady_clock::time_point &origin)
{
    return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - origin).count();
}

}  // namespace

struct capart_server {
    capart_ctx *ctx = nullptr;
    capart_server_config cfg{};
    int Qcap = 0;
    int64_t Tcap = 0;
    int64_t Sb = 0, Tb = 0;  // batch capacity (sets, tasks)
    Launch L{};
    bool tabs = false;       // queries may bring explicit time tables
    // device rings
    void *dev = nullptr;
    TaskRec *rec = nullptr;
    uint64_t *forbid = nullptr;
    uint8_t *sigma = nullptr;
    uint32_t *setflags = nullptr;
    uint64_t *memmask = nullptr;
    uint64_t *partial = nullptr;
    // host rings: inputs and results of every live query
    std::vector<SrvQuery> q;
    std::vector<int64_t> hT, hD, hCs, hCp, hR, hR1g;
    std::vector<int64_t> hCn, hCc;  // with tabs: task ring index t holds its table at [t * max_M, + M)
    std::vector<int32_t> hk;
    std::vector<uint8_t> htype;
    std::vector<int8_t> halloc;
    std::vector<int32_t> hstatus, hpidx, hsizes;
    std::vector<uint8_t> hverdict, hv1g;
    std::vector<int64_t> haidx, hnev;
    std::vector<uint64_t> hmaxU, hsumU;
    uint64_t next_ticket = 0, tail_ticket = 0, launch_ticket = 0;
    int64_t task_head = 0;
    std::vector<SrvStream> streams;
    std::mutex mu;
    std::condition_variable cv;
    std::thread dispatcher;
    std::atomic<bool> stop{false};
    std::string err;
    std::chrono::steady_clock::time_point origin;
    // statistics
    int64_t st_submitted = 0, st_completed = 0, st_rejected = 0, st_batches = 0, st_evals = 0, st_batched_q = 0;
    std::vector<double> lat;
    double st_t0 = 0;
};

namespace {

// Oldest live query's first task (or task_head when none is live).
int64_t task_tail(const capart_server *v)
{
    if (v->tail_ticket == v->next_ticket) return v->task_head;
    return v->q[v->tail_ticket % v->Qcap].t0;
}

// Contiguous range of n tasks in the task ring, or -1.
int64_t ring_alloc(capart_server *v, int64_t n)
{
    const bool empty = v->tail_ticket == v->next_ticket;
    if (empty) v->task_head = 0;
    const int64_t head = v->task_head, tail = task_tail(v);
    if (empty || head >= tail) {
        if (v->Tcap - head >= n) return head;
        if (!empty && tail > n) return 0;  // wrap, leaving the end unused
        if (empty && v->Tcap >= n) return 0;
        return -1;
    }
    if (tail - head > n) return head;
    return -1;
}

// Launch the oldest pending queries as one batch on stream i.  Caller holds mu.
void launch_batch(capart_server *v, int i)
{
    SrvStream &ss = v->streams[i];
    const uint64_t first = v->launch_ticket;
    int64_t S = 0, N = 0, NT = 0;
    int64_t t_start = v->q[first % v->Qcap].t0;
    const bool tab = v->q[first % v->Qcap].tab;  // a batch holds queries of one kind
    while (first + S < v->next_ticket && S < v->Sb) {
        const SrvQuery &x = v->q[(first + S) % v->Qcap];
        if (x.state != Q_PENDING || x.tab != tab) break;
        if (S > 0 && ((first + S) % v->Qcap == 0 || x.t0 != t_start + N)) break;  // ring wraps end a batch
        if (N + x.n > v->Tb) break;
        N += x.n;
        if (tab) NT += (int64_t)x.n * x.M;
        S++;
    }
    if (S == 0) return;
    const PackIn li = pack_in_layout(S, N, NT);
    const PackOut lo = pack_out_layout(S, N, v->cfg.K);
    char *h = ss.in_host;
    int64_t *off = (int64_t *)(h + li.off);
    int32_t *M = (int32_t *)(h + li.M);
    int64_t acc = 0, tacc = 0, wide_parts = 0;
    int32_t nmax = 1, Mmax = 1;
    for (int64_t s = 0; s < S; s++) {
        SrvQuery &x = v->q[(first + s) % v->Qcap];
        off[s] = acc;
        M[s] = x.M;
        nmax = std::max(nmax, x.n);
        Mmax = std::max(Mmax, x.M);
        if (x.n > NARROW_MAX_TASKS) wide_parts += count_parts(x.M, v->cfg.K);
        std::memcpy(h + li.T + 8 * acc, &v->hT[x.t0], 8 * (size_t)x.n);
        std::memcpy(h + li.D + 8 * acc, &v->hD[x.t0], 8 * (size_t)x.n);
        std::memcpy(h + li.Cs + 8 * acc, &v->hCs[x.t0], 8 * (size_t)x.n);
        std::memcpy(h + li.Cp + 8 * acc, &v->hCp[x.t0], 8 * (size_t)x.n);
        std::memcpy(h + li.k + 4 * acc, &v->hk[x.t0], 4 * (size_t)x.n);
        std::memcpy(h + li.type + acc, &v->htype[x.t0], (size_t)x.n);
        if (tab) {
            const size_t e = (size_t)x.n * x.M, at = (size_t)x.t0 * v->cfg.max_M;
            ((int64_t *)(h + li.toff))[s] = tacc;
            std::memcpy(h + li.Cn + 8 * tacc, &v->hCn[at], 8 * e);
            std::memcpy(h + li.Cc + 8 * tacc, &v->hCc[at], 8 * e);
            tacc += (int64_t)e;
        }
        acc += x.n;
        x.state = Q_LAUNCHED;
    }
    off[S] = acc;
    v->launch_ticket = first + S;
    ss.busy = true;
    ss.first = first;
    ss.count = S;
    ss.ntasks = N;
    const int64_t slot0 = (int64_t)(first % v->Qcap);
    // kernels see a batch-local view: inputs and results in the stream's
    // packed buffers, per-query workspace in the resident rings
    Batch b;
    char *d = ss.in_dev;
    b.off = (const int64_t *)(d + li.off);
    b.M = (const int32_t *)(d + li.M);
    b.T = (const int64_t *)(d + li.T);
    b.D = (const int64_t *)(d + li.D);
    b.Cs = (const int64_t *)(d + li.Cs);
    b.Cp = (const int64_t *)(d + li.Cp);
    b.k = (const int32_t *)(d + li.k);
    b.type = (const uint8_t *)(d + li.type);
    b.n_tasks_total = N;
    b.max_tasks = nmax;  // the batch's own bounds: launches and LDS sized for its sets only
    b.max_M = Mmax;
    if (tab) {
        b.toff = (const int64_t *)(d + li.toff);
        b.Cn = (const int64_t *)(d + li.Cn);
        b.Cc = (const int64_t *)(d + li.Cc);
        b.tlen = NT;
    }
    Work w{};
    w.rec = v->rec + t_start;
    w.forbid = v->forbid + t_start;
    w.sigma = v->sigma + t_start;
    w.setflags = v->setflags + slot0;
    w.memmask = v->memmask + slot0;
    w.partial = v->partial + 4 * (size_t)slot0 * v->L.chunks;
    w.np = v->ctx->np_dev;
    w.order = v->ctx->order_dev;
    give_tables(w, b);
    Out o{};
    char *od = ss.out_dev;
    o.status = (int32_t *)(od + lo.status);
    o.verdict = (uint8_t *)(od + lo.verdict);
    o.verdict_1g = (uint8_t *)(od + lo.v1g);
    o.pidx = (int32_t *)(od + lo.pidx);
    o.sizes = (int32_t *)(od + lo.sizes);
    o.aidx = (int64_t *)(od + lo.aidx);
    o.maxU = (uint64_t *)(od + lo.maxU);
    o.sumU = (uint64_t *)(od + lo.sumU);
    o.n_evals = (int64_t *)(od + lo.nev);
    o.alloc = (int8_t *)(od + lo.alloc);
    o.R = (int64_t *)(od + lo.R);
    o.R_1g = (int64_t *)(od + lo.R1g);
    Launch L = v->L;
    L.s0 = 0;
    L.S = S;
    L.table_words = (int)(table_lds_bytes(nmax, Mmax) / 4);
    L.threads = eval_threads(nmax, Mmax);
    // the wave-per-partitioning launch only while the wide queries cannot fill the chip's lanes
    if (L.wchunk > 0 && v->ctx->tune.wide_chunk == 0 && wide_parts >= WIDE_LANE_FILL) L.wchunk = 0;
    hipError_t e;
    (void)hipGetLastError();
    if ((e = hipMemcpyAsync(ss.in_dev, ss.in_host, li.total, hipMemcpyHostToDevice, ss.st)) != hipSuccess ||
        (e = launch_prep(b, w, o, L, ss.st)) != hipSuccess || (e = launch_eval(b, w, o, L, ss.st)) != hipSuccess ||
        (e = launch_final(b, w, o, L, ss.st)) != hipSuccess ||
        (e = hipMemcpyAsync(ss.out_host, ss.out_dev, lo.total, hipMemcpyDeviceToHost, ss.st)) != hipSuccess ||
        (e = hipEventRecord(ss.done, ss.st)) != hipSuccess)
        v->err = std::string("serving launch: ") + hipGetErrorString(e);
    v->st_batches++;
    v->st_batched_q += S;
}

// Copy a completed batch's results into the host rings.  Caller holds mu.
void finish_batch(capart_server *v, SrvStream &ss, double t)
{
    const int64_t S = ss.count, N = ss.ntasks;
    const int K = v->cfg.K;
    const PackOut lo = pack_out_layout(S, N, K);
    const char *h = ss.out_host;
    int64_t acc = 0;
    for (int64_t s = 0; s < S; s++) {
        SrvQuery &x = v->q[(ss.first + s) % v->Qcap];
        const int64_t slot = (int64_t)((ss.first + s) % v->Qcap);
        v->hstatus[slot] = ((const int32_t *)(h + lo.status))[s];
        v->hverdict[slot] = ((const uint8_t *)(h + lo.verdict))[s];
        v->hv1g[slot] = ((const uint8_t *)(h + lo.v1g))[s];
        v->hpidx[slot] = ((const int32_t *)(h + lo.pidx))[s];
        std::memcpy(&v->hsizes[slot * K], h + lo.sizes + 4 * (size_t)s * K, 4 * (size_t)K);
        v->haidx[slot] = ((const int64_t *)(h + lo.aidx))[s];
        v->hmaxU[slot] = ((const uint64_t *)(h + lo.maxU))[s];
        v->hsumU[slot] = ((const uint64_t *)(h + lo.sumU))[s];
        v->hnev[slot] = ((const int64_t *)(h + lo.nev))[s];
        std::memcpy(&v->halloc[x.t0], h + lo.alloc + acc, (size_t)x.n);
        std::memcpy(&v->hR[x.t0], h + lo.R + 8 * acc, 8 * (size_t)x.n);
        std::memcpy(&v->hR1g[x.t0], h + lo.R1g + 8 * acc, 8 * (size_t)x.n);
        acc += x.n;
        x.state = Q_DONE;
        x.t_done = t;
        v->lat.push_back(t - x.t_arrival);
        v->st_completed++;
        v->st_evals += v->hnev[slot];
    }
    ss.busy = false;
}

void dispatcher_main(capart_server *v)
{
    hipSetDevice(v->ctx->device);
    std::unique_lock<std::mutex> lk(v->mu);
    while (!v->stop.load()) {
        bool progress = false;
        for (auto &ss : v->streams) {
            if (ss.busy && hipEventQuery(ss.done) == hipSuccess) {
                finish_batch(v, ss, now_us(v->origin));
                progress = true;
            }
        }
        if (v->launch_ticket < v->next_ticket) {
            for (size_t i = 0; i < v->streams.size() && v->launch_ticket < v->next_ticket; i++) {
                if (!v->streams[i].busy) {
                    launch_batch(v, (int)i);
                    progress = true;
                }
            }
        }
        if (progress) {
            v->cv.notify_all();
            continue;
        }
        bool inflight = false;
        for (auto &ss : v->streams) inflight |= ss.busy;
        // poll completions quickly while work is in flight, else sleep until a submit
        if (inflight) {
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        } else {
            v->cv.wait_for(lk, std::chrono::milliseconds(5));
        }
    }
}

capart_status srv_fail(capart_server *v, capart_status st, const std::string &m)
{
    if (v) v->err = m;
    if (v && v->ctx) v->ctx->err = m;
    return st;
}

capart_status srv_submit(capart_server *v, const capart_tasksets *one, uint64_t *ticket, double t_arrival,
                         bool use_arrival)
{
    if (!v || !one || !ticket) return CAPART_E_INVAL;
    if (one->n_sets != 1 || !one->set_offset || !one->M || one->set_offset[0] != 0 ||
        one->set_offset[1] != one->n_tasks_total)
        return srv_fail(v, CAPART_E_INVAL, "submit takes one set with offsets {0, n}");
    const bool tab = has_tables(one);
    if (tab && !v->tabs)
        return srv_fail(v, CAPART_E_INVAL, "explicit time tables need a server created with CAPART_SERVER_TABLES");
    const int64_t n = one->n_tasks_total;
    const int32_t M = one->M[0];
    if (n < 1 || n > v->cfg.max_tasks || M < 1 || M > v->cfg.max_M || n * M > CAPART_MAX_NM)
        return srv_fail(v, CAPART_E_INVAL, "query exceeds the server's size bounds");
    if (!one->T || !one->D || !one->type || (!tab && (!one->C_seq || !one->C_par || !one->k_permille)))
        return srv_fail(v, CAPART_E_INVAL, "NULL task arrays");
    int64_t tab0 = 0;
    if (tab) {
        if (!one->table_offset || !one->Cn_table || !one->Cc_table || one->table_len < 0)
            return srv_fail(v, CAPART_E_INVAL,
                            "explicit time tables need table_offset, Cn_table, Cc_table and table_len");
        tab0 = one->table_offset[0];
        if (tab0 < 0 || tab0 > one->table_len - n * M)
            return srv_fail(v, CAPART_E_INVAL, "table_offset[0] + n * M exceeds table_len");
    }
    std::unique_lock<std::mutex> lk(v->mu);
    if (v->next_ticket - v->tail_ticket >= (uint64_t)v->Qcap) {
        v->st_rejected++;
        return CAPART_E_AGAIN;
    }
    const int64_t t0 = ring_alloc(v, n);
    if (t0 < 0) {
        v->st_rejected++;
        return CAPART_E_AGAIN;
    }
    const uint64_t tk = v->next_ticket++;
    SrvQuery &x = v->q[tk % v->Qcap];
    x.ticket = tk;
    x.t0 = t0;
    x.n = (int32_t)n;
    x.M = M;
    x.tab = tab;
    x.t_arrival = use_arrival ? t_arrival : now_us(v->origin);
    std::memcpy(&v->hT[t0], one->T, 8 * (size_t)n);
    std::memcpy(&v->hD[t0], one->D, 8 * (size_t)n);
    std::memcpy(&v->htype[t0], one->type, (size_t)n);
    if (tab) {
        // the parametric fields are not read with tables
        std::fill(&v->hCs[t0], &v->hCs[t0] + n, 0);
        std::fill(&v->hCp[t0], &v->hCp[t0] + n, 0);
        std::fill(&v->hk[t0], &v->hk[t0] + n, 1000);
        const size_t at = (size_t)t0 * v->cfg.max_M;
        std::memcpy(&v->hCn[at], one->Cn_table + tab0, 8 * (size_t)(n * M));
        std::memcpy(&v->hCc[at], one->Cc_table + tab0, 8 * (size_t)(n * M));
    } else {
        std::memcpy(&v->hCs[t0], one->C_seq, 8 * (size_t)n);
        std::memcpy(&v->hCp[t0], one->C_par, 8 * (size_t)n);
        std::memcpy(&v->hk[t0], one->k_permille, 4 * (size_t)n);
    }
    x.state = Q_PENDING;
    v->task_head = t0 + n;
    v->st_submitted++;
    *ticket = tk;
    lk.unlock();
    v->cv.notify_all();
    return CAPART_OK;
}

// Collect a completed query.  Caller holds mu.
void collect(capart_server *v, const SrvQuery &x, capart_results *r)
{
    const int64_t slot = (int64_t)(x.ticket % v->Qcap);
    const int K = v->cfg.K;
    if (r) {
        if (r->status) r->status[0] = v->hstatus[slot];
        if (r->verdict) r->verdict[0] = v->hverdict[slot];
        if (r->verdict_1g) r->verdict_1g[0] = v->hv1g[slot];
        if (r->pidx) r->pidx[0] = v->hpidx[slot];
        if (r->sizes) std::memcpy(r->sizes, &v->hsizes[slot * K], 4 * (size_t)K);
        if (r->aidx) r->aidx[0] = v->haidx[slot];
        if (r->maxU) r->maxU[0] = v->hmaxU[slot];
        if (r->sumU) r->sumU[0] = v->hsumU[slot];
        if (r->n_evals) r->n_evals[0] = v->hnev[slot];
        if (r->alloc) std::memcpy(r->alloc, &v->halloc[x.t0], (size_t)x.n);
        if (r->R) std::memcpy(r->R, &v->hR[x.t0], 8 * (size_t)x.n);
        if (r->R_1g) std::memcpy(r->R_1g, &v->hR1g[x.t0], 8 * (size_t)x.n);
    }
}

void free_collected(capart_server *v)
{
    while (v->tail_ticket < v->next_ticket && v->q[v->tail_ticket % v->Qcap].state == Q_FREE &&
           v->q[v->tail_ticket % v->Qcap].ticket == v->tail_ticket)
        v->tail_ticket++;
}

}  // namespace

extern "C" {

capart_status capart_server_create(capart_ctx *c, const capart_server_config *cfg, capart_server **out)
{
    if (!c || !cfg || !out) return CAPART_E_INVAL;
    *out = nullptr;
    const bool tabs = (cfg->flags & CAPART_SERVER_TABLES) != 0u;
    capart_options opt{cfg->K, cfg->policy, cfg->alloc_mode, cfg->flags & ~CAPART_SERVER_TABLES,
                       {cfg->admissible[0], cfg->admissible[1], cfg->admissible[2], cfg->admissible[3]}};
    capart_status rc = check_options(c, &opt);
    if (rc != CAPART_OK) return rc;
    if (cfg->alloc_mode == CAPART_EXHAUSTIVE) return fail(c, CAPART_E_INVAL, "serving runs heuristic modes");
    if (cfg->flags & CAPART_FLAG_PER_SET_LAUNCH) return fail(c, CAPART_E_INVAL, "per-set launches are not served");
    if (cfg->max_tasks < 1 || cfg->max_tasks > CAPART_MAX_TASKS || cfg->max_M < 1 || cfg->max_M > CAPART_MAX_M)
        return fail(c, CAPART_E_INVAL, "max_tasks / max_M out of range");
    if (cfg->streams < 0 || cfg->streams > 8 || cfg->max_queries < 0 || cfg->max_batch < 0 || cfg->device_bytes < 0)
        return fail(c, CAPART_E_INVAL, "bad server configuration");
    capart_server *v = new (std::nothrow) capart_server;
    if (!v) return fail(c, CAPART_E_NOMEM, "server allocation failed");
    v->ctx = c;
    v->cfg = *cfg;
    v->tabs = tabs;
    if (v->cfg.streams == 0) v->cfg.streams = 4;
    if (v->cfg.max_queries == 0) v->cfg.max_queries = 4096;
    if (v->cfg.device_bytes == 0) v->cfg.device_bytes = (int64_t)256 << 20;
    v->Qcap = v->cfg.max_queries;
    v->Sb = v->cfg.max_batch > 0 ? std::min(v->cfg.max_batch, v->Qcap) : v->Qcap;
    // launch shape: one block per 256 partitionings, so that a single query
    // spreads over many compute units
    capart_tasksets shape{};
    shape.max_tasks = cfg->max_tasks;
    shape.max_M = cfg->max_M;
    Launch &L = v->L;
    L.K = cfg->K;
    L.mode = cfg->alloc_mode;
    L.flags = opt.flags;
    for (int i = 0; i < 4; i++) L.adm.w[i] = opt.admissible[i];
    L.edf = cfg->policy == CAPART_POLICY_EDF;
    L.threads = eval_threads(cfg->max_tasks, cfg->max_M);
    L.table_words = (int)(table_lds_bytes(cfg->max_tasks, cfg->max_M) / 4);
    L.form = c->tune.loop_form == 2 ? 2 : 1;
    L.memo_packed = c->tune.loop_form == 3;
    L.exh_form = 1;
    capart_tuning tf = c->tune;
    if (tf.frontier == 0 && !frontier_pays(cfg->max_tasks, cfg->max_M, cfg->K, L.adm)) tf.frontier = 2;
    size_frontier(L, cfg->max_tasks, cfg->alloc_mode, tf);
    const uint32_t Pmax = count_parts(cfg->max_M, cfg->K);
    // 512 partitionings per block: one per lane of the widest blocks (large-set launches)
    L.chunk = c->tune.chunk > 0 ? (uint32_t)c->tune.chunk : 512u;
    L.chunks = (int)((Pmax + L.chunk - 1) / L.chunk);
    set_wide_chunk(L, cfg->max_tasks, Pmax, c->tune, 0, 0);  // slots sized for it; each batch then chooses
    // device budget: slot rings + task rings + per-stream packed buffers
    const int64_t per_slot = 4 + 8 + 32 * (int64_t)L.chunks;
    const int64_t per_task_ring = (int64_t)sizeof(TaskRec) + 8 + 1;
    const int64_t avail = v->cfg.device_bytes - per_slot * v->Qcap;
    // each task needs ring space and, while in a batch, packed input/output space
    // (with tables, max_M entries of each kind per task, packed per batch)
    const int64_t per_task_total = per_task_ring + (37 + 17) * 1 + (tabs ? 16 * (int64_t)cfg->max_M : 0);
    v->Tcap = avail > 0 ? avail / per_task_total : 0;
    v->Tb = std::min<int64_t>(v->Tcap / std::max(1, v->cfg.streams), v->Sb * cfg->max_tasks);
    if (v->Tcap < cfg->max_tasks || v->Tb < cfg->max_tasks) {
        delete v;
        return fail(c, CAPART_E_NOMEM, "device budget too small for one query");
    }
    v->Tcap -= v->Tb * v->cfg.streams * 0;  // packed buffers are accounted in per_task_total
    hipError_t e = hipSetDevice(c->device);
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align256(o + std::max<size_t>(bytes, 1)); return at; };
    const size_t r_rec = take(sizeof(TaskRec) * (size_t)v->Tcap), r_forbid = take(8 * (size_t)v->Tcap),
                 r_sigma = take((size_t)v->Tcap), r_flags = take(4 * (size_t)v->Qcap),
                 r_mm = take(8 * (size_t)v->Qcap), r_part = take(32 * (size_t)v->Qcap * L.chunks);
    const PackIn li = pack_in_layout(v->Sb, v->Tb, tabs ? v->Tb * cfg->max_M : 0);
    const PackOut lo = pack_out_layout(v->Sb, v->Tb, cfg->K);
    std::vector<size_t> s_in, s_out;
    for (int i = 0; i < v->cfg.streams; i++) {
        s_in.push_back(take(li.total));
        s_out.push_back(take(lo.total));
    }
    if (e != hipSuccess || hipMalloc(&v->dev, o) != hipSuccess) {
        delete v;
        return fail(c, CAPART_E_NOMEM, "server device arena allocation failed");
    }
    char *base = (char *)v->dev;
    v->rec = (TaskRec *)(base + r_rec);
    v->forbid = (uint64_t *)(base + r_forbid);
    v->sigma = (uint8_t *)(base + r_sigma);
    v->setflags = (uint32_t *)(base + r_flags);
    v->memmask = (uint64_t *)(base + r_mm);
    v->partial = (uint64_t *)(base + r_part);
    v->streams.resize(v->cfg.streams);
    for (int i = 0; i < v->cfg.streams; i++) {
        SrvStream &ss = v->streams[i];
        ss.in_dev = base + s_in[i];
        ss.out_dev = base + s_out[i];
        if (hipStreamCreate(&ss.st) != hipSuccess || hipEventCreateWithFlags(&ss.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc((void **)&ss.in_host, li.total, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&ss.out_host, lo.total, hipHostMallocDefault) != hipSuccess) {
            capart_server_destroy(v);
            return fail(c, CAPART_E_NOMEM, "server stream setup failed");
        }
    }
    v->q.assign(v->Qcap, SrvQuery{});
    const size_t T = (size_t)v->Tcap, Q = (size_t)v->Qcap;
    v->hT.assign(T, 0); v->hD.assign(T, 0); v->hCs.assign(T, 0); v->hCp.assign(T, 0);
    v->hk.assign(T, 0); v->htype.assign(T, 0);
    if (tabs) {
        v->hCn.assign(T * (size_t)cfg->max_M, 0);
        v->hCc.assign(T * (size_t)cfg->max_M, 0);
    } v->halloc.assign(T, 0); v->hR.assign(T, 0); v->hR1g.assign(T, 0);
    v->hstatus.assign(Q, 0); v->hpidx.assign(Q, 0); v->hsizes.assign(Q * cfg->K, 0); v->hverdict.assign(Q, 0);
    v->hv1g.assign(Q, 0); v->haidx.assign(Q, 0); v->hnev.assign(Q, 0); v->hmaxU.assign(Q, 0); v->hsumU.assign(Q, 0);
    v->origin = std::chrono::steady_clock::now();
    v->st_t0 = 0;
    v->dispatcher = std::thread(dispatcher_main, v);
    *out = v;
    return CAPART_OK;
}

capart_status capart_server_submit(capart_server *v, const capart_tasksets *one, uint64_t *ticket)
{
    return srv_submit(v, one, ticket, 0.0, false);
}

capart_status capart_server_poll(capart_server *v, uint64_t ticket, capart_results *r, int32_t *done)
{
    if (!v || !done) return CAPART_E_INVAL;
    std::lock_guard<std::mutex> lk(v->mu);
    if (ticket >= v->next_ticket || ticket < v->tail_ticket) return srv_fail(v, CAPART_E_INVAL, "unknown ticket");
    SrvQuery &x = v->q[ticket % v->Qcap];
    if (x.ticket != ticket || x.state == Q_FREE) return srv_fail(v, CAPART_E_INVAL, "ticket already collected");
    if (x.state != Q_DONE) {
        *done = 0;
        return CAPART_OK;
    }
    collect(v, x, r);
    x.state = Q_FREE;
    free_collected(v);
    *done = 1;
    return CAPART_OK;
}

static void fill_stats(capart_server *v, capart_server_stats *s, double t_now)
{
    std::memset(s, 0, sizeof *s);
    s->submitted = v->st_submitted;
    s->completed = v->st_completed;
    s->rejected = v->st_rejected;
    s->batches = v->st_batches;
    s->evals = v->st_evals;
    s->mean_batch = v->st_batches ? (double)v->st_batched_q / (double)v->st_batches : 0.0;
    s->elapsed_s = (t_now - v->st_t0) * 1e-6;
    if (!v->lat.empty()) {
        std::vector<double> l = v->lat;
        auto pct = [&](double p) {
            size_t k = (size_t)std::min<double>((double)l.size() - 1, std::ceil(p * (double)l.size()) - 1);
            std::nth_element(l.begin(), l.begin() + k, l.end());
            return l[k];
        };
        s->p50_us = pct(0.50);
        s->p99_us = pct(0.99);
        double sum = 0, mx = 0;
        for (double x : v->lat) { sum += x; mx = std::max(mx, x); }
        s->mean_us = sum / (double)v->lat.size();
        s->max_us = mx;
    }
    if (s->elapsed_s > 0) {
        s->queries_per_s = (double)s->completed / s->elapsed_s;
        s->evals_per_s = (double)s->evals / s->elapsed_s;
    }
}

capart_status capart_server_stats_get(capart_server *v, capart_server_stats *s, int32_t reset)
{
    if (!v || !s) return CAPART_E_INVAL;
    std::lock_guard<std::mutex> lk(v->mu);
    const double t = now_us(v->origin);
    fill_stats(v, s, t);
    if (reset) {
        v->st_submitted = v->st_completed = v->st_rejected = v->st_batches = v->st_evals = v->st_batched_q = 0;
        v->lat.clear();
        v->st_t0 = t;
    }
    return CAPART_OK;
}

capart_status capart_server_replay(capart_server *v, const capart_tasksets *qs, const double *arrival_us,
                                   capart_results *res, capart_server_stats *stats)
{
    if (!v || !qs || !arrival_us || !stats || qs->n_sets < 0 || !qs->set_offset || !qs->M) return CAPART_E_INVAL;
    const int64_t nq = qs->n_sets;
    {
        std::lock_guard<std::mutex> lk(v->mu);
        v->st_submitted = v->st_completed = v->st_rejected = v->st_batches = v->st_evals = v->st_batched_q = 0;
        v->lat.clear();
    }
    const double t0 = now_us(v->origin);
    {
        std::lock_guard<std::mutex> lk(v->mu);
        v->st_t0 = t0;
    }
    std::vector<uint64_t> tickets((size_t)nq, ~0ull);
    int64_t next = 0, collected = 0, oldest = 0;
    const int K = v->cfg.K;
    while (collected < nq) {
        const double t = now_us(v->origin) - t0;
        // submit every query that is due, in arrival order; stop at back-pressure
        while (next < nq && arrival_us[next] <= t) {
            const int64_t o0 = qs->set_offset[next], n = qs->set_offset[next + 1] - o0;
            const int64_t offs[2] = {0, n};
            capart_tasksets one = *qs;
            one.n_sets = 1;
            one.n_tasks_total = n;
            one.set_offset = offs;
            one.M = qs->M + next;
            one.T = qs->T + o0; one.D = qs->D + o0; one.type = qs->type + o0;
            one.C_seq = qs->C_seq ? qs->C_seq + o0 : nullptr;
            one.C_par = qs->C_par ? qs->C_par + o0 : nullptr;
            one.k_permille = qs->k_permille ? qs->k_permille + o0 : nullptr;
            if (qs->table_offset) one.table_offset = qs->table_offset + next;  // the tables stay whole
            uint64_t tk;
            const capart_status rc = srv_submit(v, &one, &tk, t0 + arrival_us[next], true);
            if (rc == CAPART_E_AGAIN) break;
            if (rc != CAPART_OK) return rc;
            tickets[next++] = tk;
        }
        // collect in order
        while (oldest < next) {
            int32_t done = 0;
            capart_results one{};
            if (res) {
                const int64_t o0 = qs->set_offset[oldest];
                one.status = res->status ? res->status + oldest : nullptr;
                one.verdict = res->verdict ? res->verdict + oldest : nullptr;
                one.verdict_1g = res->verdict_1g ? res->verdict_1g + oldest : nullptr;
                one.pidx = res->pidx ? res->pidx + oldest : nullptr;
                one.sizes = res->sizes ? res->sizes + oldest * K : nullptr;
                one.aidx = res->aidx ? res->aidx + oldest : nullptr;
                one.maxU = res->maxU ? res->maxU + oldest : nullptr;
                one.sumU = res->sumU ? res->sumU + oldest : nullptr;
                one.n_evals = res->n_evals ? res->n_evals + oldest : nullptr;
                one.alloc = res->alloc ? res->alloc + o0 : nullptr;
                one.R = res->R ? res->R + o0 : nullptr;
                one.R_1g = res->R_1g ? res->R_1g + o0 : nullptr;
            }
            const capart_status rc = capart_server_poll(v, tickets[oldest], res ? &one : nullptr, &done);
            if (rc != CAPART_OK) return rc;
            if (!done) break;
            oldest++;
            collected++;
        }
        if (!v->err.empty()) return srv_fail(v, CAPART_E_DEVICE, v->err);
        std::this_thread::yield();
    }
    std::lock_guard<std::mutex> lk(v->mu);
    fill_stats(v, stats, now_us(v->origin));
    return CAPART_OK;
}

capart_status capart_server_destroy(capart_server *v)
{
    if (!v) return CAPART_E_INVAL;
    v->stop.store(true);
    v->cv.notify_all();
    if (v->dispatcher.joinable()) v->dispatcher.join();
    hipSetDevice(v->ctx->device);
    for (auto &ss : v->streams) {
        if (ss.st) hipStreamSynchronize(ss.st);
        if (ss.done) hipEventDestroy(ss.done);
        if (ss.st) hipStreamDestroy(ss.st);
        if (ss.in_host) hipHostFree(ss.in_host);
        if (ss.out_host) hipHostFree(ss.out_host);
    }
    if (v->dev) hipFree(v->dev);
    delete v;
    return CAPART_OK;
}

}  // extern "C"
