// gfx950 kernels of the contention-aware partitioning engine.
//
// Work decomposition (one HIP stream, three launches per batch):
//   prep  : one wave per task set -- validation, deadline-monotonic ranks,
//           Lemma 1 and Lemma 2, heuristic order, exact-division constants,
//           ACT forbidden pairs; writes a packed per-task record.
//   eval  : one block per (set, chunk of partitionings).  The block stages the
//           set's records and a per-(m, conflict, task) table of execution
//           times and Q32 utilisations in LDS, then every lane walks a
//           contiguous run of partitionings (unranked once, then stepped in
//           descending lexicographic order), allocates tasks (heuristic) or
//           scans allocations (exhaustive), and keeps its best key; the block
//           reduces keys with cross-lane shuffles and writes one partial.
//   final : one wave per set -- reduces the partials, rebuilds the chosen
//           allocation, computes response times of the chosen triple and of
//           the whole-GPU baseline (one lane per task) and writes the results.
//
// All arithmetic is integer.  Response-time iterations use 32-bit operands
// with 64-bit accumulation: every hp task that has passed satisfies
// C_j <= D_j <= T_j, so each term ceil(R/T_j)*C_j < 2^32 and the sum of at
// most 64 terms stays far below 2^64; a task whose time reaches its period
// (utilisation >= 1) makes every lower-priority task miss, which is decided
// without iterating.
#include "capart_internal.h"
#include "capart_arith.h"

#include <type_traits>

namespace capart {

constexpr int MAXN = CAPART_MAX_TASKS;

struct Key {
    uint64_t a, b, c, d;  // (maxU, sumU, pidx, aidx); "none" = all ones
};

__device__ __forceinline__ Key key_none() { return Key{~0ull, ~0ull, ~0ull, ~0ull}; }

__device__ __forceinline__ bool key_less(const Key &x, const Key &y)
{
    if (x.a != y.a) return x.a < y.a;
    if (x.b != y.b) return x.b < y.b;
    if (x.c != y.c) return x.c < y.c;
    return x.d < y.d;
}

__device__ __forceinline__ Key key_shfl_xor(const Key &k, int mask)
{
    Key o;
    o.a = __shfl_xor(k.a, mask, 64);
    o.b = __shfl_xor(k.b, mask, 64);
    o.c = __shfl_xor(k.c, mask, 64);
    o.d = __shfl_xor(k.d, mask, 64);
    return o;
}

__device__ __forceinline__ Key wave_min(Key k)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        Key t = key_shfl_xor(k, o);
        if (key_less(t, k)) k = t;
    }
    return k;
}

// Block-wide minimum; result valid in thread 0.  `scratch` holds >= 16 keys.
__device__ Key block_min(Key k, Key *scratch)
{
    k = wave_min(k);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    if (nw == 1) return k;
    if (lane == 0) scratch[wid] = k;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < nw; i++)
            if (key_less(scratch[i], k)) k = scratch[i];
    }
    return k;
}

__device__ __forceinline__ int ctz64(uint64_t x) { return __builtin_ctzll(x); }

// Work tallies: the evaluation kernel is also built in a counting variant that
// totals the work its algorithm performs (response-time terms: one per
// iteration plus one per higher-priority term; exact partition tests; frontier
// lookups).  NoTally compiles to nothing.
struct NoTally {
    __device__ __forceinline__ void term(uint32_t) {}
    __device__ __forceinline__ void test() {}
    __device__ __forceinline__ void look() {}
};
struct Tally {
    uint64_t terms = 0, tests = 0, looks = 0;
    __device__ __forceinline__ void term(uint32_t k) { terms += k; }
    __device__ __forceinline__ void test() { tests++; }
    __device__ __forceinline__ void look() { looks++; }
};

// ---------------------------------------------------------------------------
// Per-set data in LDS (ranks are deadline-monotonic priority positions).
struct SetLDS {
    uint32_t T[MAXN], D[MAXN], clo[MAXN], chi[MAXN];
    uint32_t Cs[MAXN], Cp[MAXN], k[MAXN];
    uint32_t mmin[MAXN];
    uint64_t forbid[MAXN];
    uint64_t intf[MAXN];  // ranks j with T_j < D_r: the only ones that can add a second job
    uint8_t sigma[MAXN];
    uint8_t orig[MAXN];
    uint8_t rank_of[MAXN];
    uint64_t memmask;
};

// Execution-time and utilisation tables, [m-1][conflict][rank], u32:
//   tabC: time on m units; tabU: ceil(C*2^32/T) - 1.
struct Tables {
    const uint32_t *C;
    const uint32_t *U;
    int n;
};

extern __shared__ uint32_t capart_dyn_lds[];

__device__ void stage_set(SetLDS &L, const Work &w, int64_t off, int n, int M, int64_t s, bool act, Tables &tb)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int i = tid; i < n; i += nt) {
        TaskRec t = w.rec[off + i];
        L.T[i] = t.T; L.D[i] = t.D; L.clo[i] = t.clo; L.chi[i] = t.chi;
        L.Cs[i] = t.Cs; L.Cp[i] = t.Cp; L.k[i] = t.k;
        L.mmin[i] = t.mmin;
        L.orig[i] = t.orig;
        L.rank_of[t.orig] = (uint8_t)i;
        L.sigma[i] = w.sigma[off + i];
        L.forbid[i] = act ? w.forbid[off + i] : 0ull;
    }
    if (tid == 0) L.memmask = w.memmask[s];
    __syncthreads();
    for (int r = tid; r < n; r += nt) {
        uint64_t f = 0ull;
        for (int j = 0; j < n; j++) f |= (uint64_t)(L.T[j] < L.D[r]) << j;
        L.intf[r] = f;
    }
    uint32_t *tc = capart_dyn_lds;
    uint32_t *tu = capart_dyn_lds + 2 * n * M;
    for (int e = tid; e < n * M; e += nt) {
        const int m = e / n + 1, r = e - (m - 1) * n;
        const uint32_t cn = time_n(L.Cs[r], L.Cp[r], (uint32_t)m);
        const uint32_t cc = time_c(L.k[r], cn);
        const int base = (m - 1) * 2 * n + r;
        tc[base] = cn;
        tc[base + n] = cc;
        tu[base] = util_q32_m1(cn, L.T[r]);
        tu[base + n] = util_q32_m1(cc, L.T[r]);
    }
    __syncthreads();
    tb.C = tc;
    tb.U = tu;
    tb.n = n;
}

// Rank masks: 32-bit when every set of the launch has at most 32 tasks.
__device__ __forceinline__ int mctz(uint32_t x) { return __builtin_ctz(x); }
__device__ __forceinline__ int mctz(uint64_t x) { return __builtin_ctzll(x); }
__device__ __forceinline__ int mpopc(uint32_t x) { return __popc(x); }
__device__ __forceinline__ int mpopc(uint64_t x) { return __popcll(x); }
template <typename MT>
__device__ __forceinline__ MT below(int r) { return (MT(1) << r) - MT(1); }
template <typename MT>
__device__ __forceinline__ uint32_t mbit(MT m, int j) { return (uint32_t)(m >> j) & 1u; }

// Conflict mask of a partition holding rank set S: bit r set iff task r has
// another task of its type in S (Section "Task Model").
template <typename MT>
__device__ __forceinline__ MT conflict_mask(MT S, MT memmask)
{
    const MT mem = S & memmask, cmp = S & ~memmask;
    return (mpopc(mem) >= 2 ? memmask : MT(0)) | (mpopc(cmp) >= 2 ? ~memmask : MT(0));
}

// Fixed point of R = base + sum_{j in hp} floor((R-1)/T_j) C_j from R = base,
// where base = C_r + sum_{j in hp} C_j is the demand with one job of every
// higher-priority task (so the sum equals C_r + sum ceil(R/T_j) C_j), and hp
// holds only tasks with T_j < D_r (the others never release a second job
// before D_r).  Returns R, or 0 once R exceeds D.
template <typename MT, typename TY>
__device__ __forceinline__ uint32_t rta_fp(const SetLDS &L, const uint32_t *row, int n, uint64_t base, uint32_t D,
                                           MT hp, MT cm, TY &ty)
{
    if (base > D) return 0u;
    uint64_t R = base;
    while (hp) {
        ty.term(1u + (uint32_t)mpopc(hp));
        const uint32_t x = (uint32_t)R - 1u;
        uint64_t W = base;
        for (MT h = hp; h; h &= h - MT(1)) {
            const int j = mctz(h);
            const uint32_t Cj = row[(int)mbit(cm, j) * n + j];
            W += (uint64_t)floordiv_magic(x, L.clo[j], L.chi[j]) * Cj;
        }
        if (W > D) return 0u;
        if (W == R) break;
        R = W;
    }
    return (uint32_t)R;
}

// Test the members of S with rank >= first on one partition of m units,
// taking the members below `first` as already schedulable (their response
// times cannot change).  cm = conflict mask of S.
template <typename MT, typename TY>
__device__ bool test_from(const SetLDS &L, const Tables &tb, MT S, int first, int m, MT cm, TY &ty)
{
    ty.test();
    const int n = tb.n;
    const uint32_t *row = tb.C + (m - 1) * 2 * n;
    uint64_t sumC = 0;
    bool sat = false;  // some higher-priority task has utilisation >= 1
    for (MT h = S & below<MT>(first); h; h &= h - MT(1)) {
        const int j = mctz(h);
        const uint32_t Cj = row[(int)mbit(cm, j) * n + j];
        sumC += Cj;
        sat |= (Cj >= L.T[j]);
    }
    for (MT rem = S & ~below<MT>(first); rem; rem &= rem - MT(1)) {
        const int r = mctz(rem);
        const uint32_t Cr = row[(int)mbit(cm, r) * n + r];
        if (sat) return false;
        const MT hp = S & below<MT>(r) & (MT)L.intf[r];
        if (!rta_fp<MT>(L, row, n, sumC + Cr, L.D[r], hp, cm, ty)) return false;
        sumC += Cr;
        sat |= (Cr >= L.T[r]);
    }
    return true;
}

// Whole-partition test with its Q32 utilisation.
template <typename MT, typename TY>
__device__ bool part_test(const SetLDS &L, const Tables &tb, MT S, int m, uint64_t *U, TY &ty)
{
    const int n = tb.n;
    const MT cm = conflict_mask<MT>(S, (MT)L.memmask);
    if (!test_from<MT>(L, tb, S, 0, m, cm, ty)) return false;
    const uint32_t *urow = tb.U + (m - 1) * 2 * n;
    uint64_t u = 0;
    for (MT h = S; h; h &= h - MT(1)) {
        const int r = mctz(h);
        u += (uint64_t)urow[(int)mbit(cm, r) * n + r] + 1ull;
    }
    *U = u;
    return true;
}

// Test of S_old + {tau} on m units when S_old is known schedulable there with
// utilisation U_old.  Only tau, the lower-priority members and (if tau makes
// the single same-type member conflict) that member and those below it can
// change; U is updated by the same differences.
template <typename MT, typename TY>
__device__ bool part_test_add(const SetLDS &L, const Tables &tb, MT Sold, int tau, int m, uint64_t Uold,
                              uint64_t *U, TY &ty)
{
    const int n = tb.n;
    const MT memm = (MT)L.memmask;
    const MT S = Sold | (MT(1) << tau);
    const MT same = Sold & (mbit(memm, tau) ? memm : ~memm);
    const int ns = mpopc(same);
    const MT cm = conflict_mask<MT>(S, memm);
    int first = tau, flip = -1;
    if (ns == 1) {
        flip = mctz(same);
        first = min(first, flip);
    }
    if (!test_from<MT>(L, tb, S, first, m, cm, ty)) return false;
    const uint32_t *urow = tb.U + (m - 1) * 2 * n;
    uint64_t u = Uold + (uint64_t)urow[(ns >= 1 ? n : 0) + tau] + 1ull;
    if (flip >= 0) u += (uint64_t)urow[n + flip] - (uint64_t)urow[flip];
    *U = u;
    return true;
}

// Fewest units (<= mp, where S is known schedulable) that schedule S: binary
// search, valid because schedulability is monotone in m (no timing anomalies).
template <typename MT, typename TY>
__device__ int min_units(const SetLDS &L, const Tables &tb, MT S, int mp, TY &ty)
{
    int lo = 1;
    for (MT h = S; h; h &= h - MT(1)) lo = max(lo, (int)L.mmin[mctz(h)]);
    int hi = mp;
    const MT cm = conflict_mask<MT>(S, (MT)L.memmask);
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (test_from<MT>(L, tb, S, 0, mid, cm, ty))
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// Response time of rank r on m units with higher-priority members hp (every
// task of hp is evaluated whether or not it meets its own deadline); 0 on a miss.
template <typename MT>
__device__ uint32_t rta_one(const SetLDS &L, const Tables &tb, int m, int r, MT hp, MT cm)
{
    const int n = tb.n;
    const uint32_t *row = tb.C + (m - 1) * 2 * n;
    uint64_t base = row[(int)mbit(cm, r) * n + r];
    bool sat = false;
    for (MT h = hp; h; h &= h - MT(1)) {
        const int j = mctz(h);
        const uint32_t Cj = row[(int)mbit(cm, j) * n + j];
        base += Cj;
        sat |= (Cj >= L.T[j]);
    }
    if (sat) return 0u;
    NoTally nt;
    return rta_fp<MT>(L, row, n, base, L.D[r], hp & (MT)L.intf[r], cm, nt);
}

template <int KMAX, typename V>
__device__ __forceinline__ V pick(const V (&a)[KMAX], int p)
{
    V v = a[0];
#pragma unroll
    for (int i = 1; i < KMAX; i++) v = (p == i) ? a[i] : v;
    return v;
}

// Heuristic allocation on a fixed partitioning m[0..k) (non-increasing):
// tasks in decreasing one-unit utilisation, each to the best-ranked part that
// stays schedulable.  S[p] = rank masks, U[p] = Q32 utilisations.
template <int KMAX, bool ACT, bool SMS, typename MT, typename TY>
__device__ __forceinline__ bool heuristic(const SetLDS &L, const Tables &tb, int n, const int (&m)[KMAX], int k,
                                          MT (&S)[KMAX], uint64_t (&U)[KMAX], TY &ty)
{
#pragma unroll
    for (int p = 0; p < KMAX; p++) { S[p] = MT(0); U[p] = 0ull; }
    for (int t = 0; t < n; t++) {
        const int r = L.sigma[t];
        const int mm = (int)L.mmin[r];
        const MT fb = ACT ? (MT)L.forbid[r] : MT(0);
        int best = -1, bestReq = 0;
        uint64_t bestU = 0;
        // parts are visited with compile-time indices so that S, U and m stay in registers
#pragma unroll
        for (int p = 0; p < KMAX; p++) {
            const int mp = m[p];
            const MT Sp = S[p];
            if (p >= k || mm > mp) continue;
            if (ACT && (fb & Sp)) continue;
            uint64_t Un;
            if (!part_test_add<MT>(L, tb, Sp, r, mp, U[p], &Un, ty)) continue;
            int req = 0;
            if (SMS) req = min_units<MT>(L, tb, Sp | (MT(1) << r), mp, ty);
            const bool better = (best < 0) || (SMS ? (req < bestReq || (req == bestReq && Un < bestU)) : (Un < bestU));
            if (better) { best = p; bestU = Un; bestReq = req; }
        }
        if (best < 0) return false;
#pragma unroll
        for (int p = 0; p < KMAX; p++)
            if (p == best) { S[p] |= MT(1) << r; U[p] = bestU; }
    }
    return true;
}

// ---------------------------------------------------------------------------
// Feasibility frontier of a set of at most FRONT_MAX_N tasks: ms[S] = fewest
// units that schedule rank subset S on one partition (FRONT_NONE if even M
// units do not).  Schedulability is monotone in m (no timing anomalies) and
// in S (a task added to a partition never helps), so ms[S] is at least the
// largest ms of its subsets with one task less; subsets are filled level by
// level (by size) with a binary search above that bound.  Every candidate test
// of the heuristic on any partitioning is then one lookup:
// S + {tau} fits a part of m units iff ms[S + {tau}] <= m, and the fewest
// units the merged part needs (order >>) is ms[S + {tau}] itself.
constexpr int FRONT_MAX_N = 14;
constexpr uint16_t FRONT_NONE = 0xFFFFu;

// Lanes that search one subset's fewest units together (k-ary search).
constexpr int FRONT_GROUP = 16;

// Fill ms[] level by level (subsets of equal size, taken in the order of the
// host-built list `order`: subsets of {0..n-1} by size, then value).
// For S with lowest-priority member r (largest rank) and S' = S - {r}:
// lo = max(ms of the subsets with one member less, m_min of r) bounds ms[S]
// from below, and S is schedulable on m >= lo units iff the members whose
// response times can differ from those in S' pass: r alone, or, when r makes
// the single member j of its type in S' conflict, j and every member below j.
// Phase 1 gives each lane one subset and tests it at lo; the subsets that
// fail there are searched in phase 2 by groups of FRONT_GROUP lanes, each
// round testing FRONT_GROUP evenly spaced sizes of the open interval (a, b)
// with a failing and b passing (b = M + 1 stands for "none").
template <typename MT, typename TY>
__device__ void build_frontier(const SetLDS &L, const Tables &tb, int n, int M, uint16_t *ms,
                               const uint16_t *order, TY &ty)
{
    __shared__ uint32_t fails[256];
    __shared__ uint32_t nfail[2];  // alternate chunks: one is cleared while the other is read
    const uint16_t *ord = order + ((1u << n) - 2u);
    const MT memm = (MT)L.memmask;
    if (threadIdx.x == 0) { ms[0] = 0; nfail[0] = 0u; nfail[1] = 0u; }
    uint32_t cur = 0;
    uint32_t lvl_off = 1, lvl_cnt = (uint32_t)n;  // level 1 follows the empty set
    for (int c = 1; c <= n; c++) {
        for (uint32_t base = 0; base < lvl_cnt; base += blockDim.x, cur ^= 1u) {
            __syncthreads();  // orders the previous chunk's ms[] writes and counter reads before what follows
            if (threadIdx.x == 0) nfail[cur ^ 1u] = 0u;
            const uint32_t i = base + threadIdx.x;
            if (i < lvl_cnt) {
                const uint32_t S = ord[lvl_off + i];
                const int r = 31 - __clz(S);
                int lo = max(1, (int)L.mmin[r]);
                bool none = lo > M;
                for (uint32_t h = S; h; h &= h - 1u) {
                    const uint16_t v = ms[S & ~(h & (0u - h))];
                    none |= (v == FRONT_NONE);
                    lo = max(lo, (int)v);
                }
                uint16_t res = FRONT_NONE;
                if (!none) {
                    const MT SM = (MT)S;
                    const MT Sp = SM & ~(MT(1) << r);
                    const MT same = Sp & (mbit(memm, r) ? memm : ~memm);
                    const int first = (mpopc(same) == 1) ? mctz(same) : r;
                    const MT cm = conflict_mask<MT>(SM, memm);
                    if (test_from<MT>(L, tb, SM, first, lo, cm, ty)) {
                        res = (uint16_t)lo;
                    } else if (lo < M) {
                        res = 0u;  // searched in phase 2
                        fails[atomicAdd(&nfail[cur], 1u)] = S | ((uint32_t)first << 16) | ((uint32_t)lo << 20);
                    }
                }
                if (res) ms[S] = res;
            }
            __syncthreads();
            const uint32_t F = nfail[cur];
            const int groups = blockDim.x / FRONT_GROUP;
            const int g = threadIdx.x / FRONT_GROUP, li = threadIdx.x % FRONT_GROUP;
            const int shift = (threadIdx.x & 63) & ~(FRONT_GROUP - 1);
            for (uint32_t f = g; f < F; f += groups) {
                const uint32_t e = fails[f];
                const uint32_t S = e & 0xFFFFu;
                const int first = (int)((e >> 16) & 0xFu);
                const MT SM = (MT)S;
                const MT cm = conflict_mask<MT>(SM, memm);
                int a = (int)(e >> 20), b = M + 1;  // fails at a; passes at b (or none if b = M + 1)
                while (b - a > 1) {
                    const int span = b - a;
                    const bool dense = span - 1 <= FRONT_GROUP;
                    const int x = dense ? a + 1 + li : a + ((li + 1) * span) / (FRONT_GROUP + 1);
                    const bool pass = x < b && test_from<MT>(L, tb, SM, first, x, cm, ty);
                    const uint32_t gm = (uint32_t)(__ballot(pass) >> shift) & ((1u << FRONT_GROUP) - 1u);
                    if (gm) {
                        const int fl = __ffs(gm) - 1;
                        const int xf = dense ? a + 1 + fl : a + ((fl + 1) * span) / (FRONT_GROUP + 1);
                        const int xp = fl == 0 ? a : (dense ? a + fl : a + (fl * span) / (FRONT_GROUP + 1));
                        a = xp;
                        b = xf;
                    } else {
                        a = dense ? b - 1 : a + (FRONT_GROUP * span) / (FRONT_GROUP + 1);
                    }
                }
                if (li == 0) ms[S] = (b > M) ? FRONT_NONE : (uint16_t)b;
            }
        }
        lvl_off += lvl_cnt;
        lvl_cnt = lvl_cnt * (uint32_t)(n - c) / (uint32_t)(c + 1);
    }
    __syncthreads();
}

// Q32 utilisation of S_old + {tau} on m units from that of S_old (the new
// task's term and, when it makes the lone same-type member conflict, that
// member's change).
template <typename MT>
__device__ __forceinline__ uint64_t util_add(const SetLDS &L, const Tables &tb, MT Sold, int tau, int m, uint64_t Uold)
{
    const int n = tb.n;
    const MT memm = (MT)L.memmask;
    const MT same = Sold & (mbit(memm, tau) ? memm : ~memm);
    const int ns = mpopc(same);
    const uint32_t *urow = tb.U + (m - 1) * 2 * n;
    uint64_t u = Uold + (uint64_t)urow[(ns >= 1 ? n : 0) + tau] + 1ull;
    if (ns == 1) {
        const int flip = mctz(same);
        u += (uint64_t)urow[n + flip] - (uint64_t)urow[flip];
    }
    return u;
}

// The heuristic on one fixed partitioning with every candidate test answered
// by the frontier (same decisions as `heuristic`, which tests directly).
template <int KMAX, bool ACT, bool SMS, typename MT, typename TY>
__device__ __forceinline__ bool heuristic_front(const SetLDS &L, const Tables &tb, const uint16_t *ms, int n,
                                                const int (&m)[KMAX], int k, MT (&S)[KMAX], uint64_t (&U)[KMAX],
                                                TY &ty)
{
#pragma unroll
    for (int p = 0; p < KMAX; p++) { S[p] = MT(0); U[p] = 0ull; }
    for (int t = 0; t < n; t++) {
        const int r = L.sigma[t];
        const MT bit = MT(1) << r;
        const MT fb = ACT ? (MT)L.forbid[r] : MT(0);
        int best = -1, bestReq = 0;
        uint64_t bestU = 0;
#pragma unroll
        for (int p = 0; p < KMAX; p++) {
            if (p >= k) continue;
            ty.look();
            const MT Sp = S[p];
            const int req = (int)ms[(uint32_t)(Sp | bit)];
            if (req > m[p]) continue;
            if (ACT && (fb & Sp)) continue;
            const uint64_t Un = util_add<MT>(L, tb, Sp, r, m[p], U[p]);
            const bool better = (best < 0) || (SMS ? (req < bestReq || (req == bestReq && Un < bestU)) : (Un < bestU));
            if (better) { best = p; bestU = Un; bestReq = req; }
        }
        if (best < 0) return false;
#pragma unroll
        for (int p = 0; p < KMAX; p++)
            if (p == best) { S[p] |= bit; U[p] = bestU; }
    }
    return true;
}

// ---------------------------------------------------------------------------
// Partitionings of M into at most K parts in descending lexicographic order.
template <int KMAX>
__device__ __forceinline__ int unrank(const uint32_t *np, int M, int K, uint32_t rank, int (&a)[KMAX])
{
    int rem = M, maxp = M, k = 0;
#pragma unroll
    for (int j = 0; j < KMAX; j++) {
        int y = 0;
        if (j < K && rem > 0) {
            const int left = K - j - 1;
            y = min(rem, maxp);
            for (; y > 1; y--) {
                const uint32_t c = np[np_index(left, rem - y, y)];
                if (rank < c) break;
                rank -= c;
            }
            rem -= y;
            maxp = y;
            k++;
        }
        a[j] = y;
    }
    return k;
}

// Next partitioning in descending lexicographic order; returns the new number
// of parts (0 if `a` was the last one).
template <int KMAX>
__device__ __forceinline__ int next_partition(int (&a)[KMAX], int K)
{
    int tail = 0, sel = -1, v = 0;
#pragma unroll
    for (int i = KMAX - 1; i >= 0; i--) {
        if (sel < 0 && i < K) {
            const int vi = a[i] - 1;
            if (a[i] > 1 && tail + 1 <= (K - i - 1) * vi) {
                sel = i;
                v = vi;
            } else {
                tail += a[i];
            }
        }
    }
    if (sel < 0) return 0;
    int rest = tail + 1, k = 0;
#pragma unroll
    for (int i = 0; i < KMAX; i++) {
        if (i == sel) {
            a[i] = v;
        } else if (i > sel) {
            const int x = min(v, rest);
            a[i] = x;
            rest -= x;
        }
        k += (a[i] > 0);
    }
    return k;
}

// ---------------------------------------------------------------------------
// prep: one wave per set.
__global__ __launch_bounds__(64) void prep_kernel(Batch b, Work w, Out o, Launch Lp)
{
    __shared__ uint32_t sD[MAXN], sT[MAXN];
    __shared__ uint64_t su1[MAXN];
    __shared__ TaskRec srec[MAXN];
    __shared__ uint64_t sforbid[MAXN];
    const int64_t s = Lp.s0 + blockIdx.x;
    const int lane = threadIdx.x;
    if (w.counter != nullptr && blockIdx.x == 0 && lane == 0) *w.counter = 0u;  // batched form: restart the queue
    const int64_t off0 = b.off[s], off1 = b.off[s + 1];
    const int M = b.M[s];
    int status = CAPART_OK;
    const int nmax = min(b.max_tasks, MAXN), Mmax = min(b.max_M, CAPART_MAX_M);
    if (off0 < 0 || off1 < off0 || off1 > b.n_tasks_total) status = CAPART_E_INVAL;
    const int64_t n64 = off1 - off0;
    if (status == CAPART_OK && (n64 < 1 || n64 > nmax || M < 1 || M > Mmax || n64 * M > CAPART_MAX_NM))
        status = CAPART_E_INVAL;
    if (status != CAPART_OK) {
        if (lane == 0) { o.status[s] = status; w.setflags[s] = 0u; }
        return;
    }
    const int n = (int)n64;
    int64_t T = 1, D = 1, Cs = 0, Cp = 1;
    int32_t kk = 1000;
    int ty = 0;
    bool bad = false;
    if (lane < n) {
        T = b.T[off0 + lane]; D = b.D[off0 + lane];
        Cs = b.Cs[off0 + lane]; Cp = b.Cp[off0 + lane];
        kk = b.k[off0 + lane]; ty = b.type[off0 + lane];
        const int64_t L31 = (int64_t)1 << 31;
        bad = (T < 1 || T >= L31 || D < 1 || D > T || Cs < 0 || Cp < 0 || Cs >= L31 || Cp >= L31 ||
               Cs + Cp < 1 || Cs + Cp >= L31 || kk < 1000 || kk > 1000000 || ty > 1);
    }
    if (__ballot(bad)) status = CAPART_E_RANGE;
    if (status == CAPART_OK && Lp.mode == CAPART_EXHAUSTIVE) {
        // k^n < 2^62 for the largest k = min(K, M)
        const uint64_t kk2 = (uint64_t)min(Lp.K, M);
        const uint64_t lim = ((1ull << 62) - 1ull) / kk2;
        uint64_t pw = 1;
        for (int i = 0; i < n; i++) {
            if (pw > lim) { status = CAPART_E_INVAL; break; }
            pw *= kk2;
        }
    }
    if (lane == 0) o.status[s] = status;
    if (status != CAPART_OK) {
        if (lane == 0) w.setflags[s] = 0u;
        return;
    }
    // deadline-monotonic rank and heuristic order
    const uint32_t c1 = (uint32_t)(Cs + Cp);
    uint64_t u1 = 0, l1 = 0;
    if (lane < n) {
        const uint64_t num = (uint64_t)c1 << 32;
        u1 = (num + (uint64_t)T - 1) / (uint64_t)T;  // ceil(Cn(1) 2^32 / T)
        l1 = num / (uint64_t)T;                      // floor, for Lemma 1
        sD[lane] = (uint32_t)D;
        sT[lane] = (uint32_t)T;
        su1[lane] = u1;
    }
    __syncthreads();
    int rank = 0, pos = 0;
    if (lane < n) {
        for (int j = 0; j < n; j++) {
            const bool before = (sD[j] < (uint32_t)D) || (sD[j] == (uint32_t)D && (sT[j] < (uint32_t)T ||
                                                                                   (sT[j] == (uint32_t)T && j < lane)));
            rank += before;
            pos += (su1[j] > u1) || (su1[j] == u1 && j < lane);
        }
    }
    // Lemma 1: saturating wave sum of floor-Q32 utilisations
    uint64_t acc = (lane < n) ? l1 : 0ull;
    const uint64_t cap = (uint64_t)M << 32;
#pragma unroll
    for (int o2 = 32; o2 >= 1; o2 >>= 1) {
        const uint64_t t = __shfl_xor(acc, o2, 64);
        acc = (acc > cap || t > cap) ? cap + 1 : acc + t;
    }
    const bool reject = (acc > cap) && !(Lp.flags & CAPART_FLAG_NO_LEMMA1);
    // memory-intensive ranks
    uint64_t mm = (lane < n && ty == 1) ? (1ull << rank) : 0ull;
#pragma unroll
    for (int o2 = 32; o2 >= 1; o2 >>= 1) mm |= __shfl_xor(mm, o2, 64);
    if (lane < n) {
        TaskRec r;
        r.T = (uint32_t)T; r.D = (uint32_t)D; r.Cs = (uint32_t)Cs; r.Cp = (uint32_t)Cp; r.k = (uint32_t)kk;
        magic_u32((uint32_t)T, &r.clo, &r.chi);
        r.mmin = m_min((uint32_t)Cs, (uint32_t)Cp, (uint32_t)D, (uint32_t)M);
        r.orig = (uint8_t)lane;
        r.mem = (uint8_t)ty;
        w.rec[off0 + rank] = r;
        w.sigma[off0 + pos] = (uint8_t)rank;
        srec[rank] = r;
        sforbid[rank] = 0ull;
    }
    if (lane == 0) {
        w.memmask[s] = mm;
        w.setflags[s] = SETF_VALID | (reject ? SETF_LEMMA1 : 0u);
    }
    const bool act = (Lp.mode == CAPART_HEUR_BF_ACT || Lp.mode == CAPART_HEUR_SMS_ACT);
    if (!act) return;
    __syncthreads();
    // ACT: pair (a, b), a < b in rank order, is forbidden iff no size in
    // [max(mmin), min(mmin_a + mmin_b - 1, M)] schedules both together; by
    // monotonicity in m it suffices to test the top of that range.
    if (lane < n) {
        const int bb = lane;
        const TaskRec tb = srec[bb];
        uint64_t fb = 0ull;
        for (int a = 0; a < bb; a++) {
            const TaskRec ta = srec[a];
            bool forb = true;
            if (ta.mmin != MMIN_NONE && tb.mmin != MMIN_NONE) {
                const uint32_t m = min((uint32_t)ta.mmin + tb.mmin - 1u, (uint32_t)M);
                const bool conf = ta.mem == tb.mem;
                uint32_t Ca = time_n(ta.Cs, ta.Cp, m), Cb = time_n(tb.Cs, tb.Cp, m);
                if (conf) { Ca = time_c(ta.k, Ca); Cb = time_c(tb.k, Cb); }
                if (Ca <= ta.D && Ca < ta.T) {
                    uint64_t R = (uint64_t)Cb + Ca;
                    for (;;) {
                        if (R > tb.D) break;
                        const uint64_t W = (uint64_t)Cb + ((R + ta.T - 1) / ta.T) * (uint64_t)Ca;
                        if (W > tb.D) break;
                        if (W == R) { forb = false; break; }
                        R = W;
                    }
                }
            }
            if (forb) {
                fb |= 1ull << a;
                atomicOr((unsigned long long *)&sforbid[a], (unsigned long long)(1ull << bb));
            }
        }
        atomicOr((unsigned long long *)&sforbid[bb], (unsigned long long)fb);
    }
    __syncthreads();
    if (lane < n) w.forbid[off0 + lane] = sforbid[lane];
}

// ---------------------------------------------------------------------------
// eval, heuristic allocation: one block per (set, chunk of partitionings).
// Every lane walks a contiguous run of partitionings.  The heuristic is run as
// a per-lane state machine whose loop step is ONE candidate test (task sigma_t
// on part p): a lane that finishes a partitioning starts the next one at the
// next step instead of idling until the slowest lane of its wave has finished.
template <int KMAX>
__device__ __forceinline__ uint64_t pack_sizes(const int (&m)[KMAX])
{
    uint64_t v = 0;
#pragma unroll
    for (int i = 0; i < KMAX; i++) v |= (uint64_t)(uint32_t)m[i] << (8 * i);
    return v;
}

__device__ __forceinline__ int size_of(uint64_t mpack, int p) { return (int)((mpack >> (8 * p)) & 0xFFu); }

// Per-lane part state (rank masks and utilisations) lives in LDS, lane-
// interleaved (entry p of lane l at p * blockDim + l), so that the
// data-dependent part index costs one conflict-free LDS access.
template <int KMAX, bool ACT, bool SMS, typename MT, typename TY>
__device__ void heur_run(const SetLDS &L, const Tables &tb, const uint32_t *np, int n, int M, int K, uint32_t q0,
                         uint32_t q1, Key &best, uint64_t *dbg, MT *lS, uint64_t *lU, TY &ty)
{
    const int stride = blockDim.x;
    MT *myS = lS + threadIdx.x;
    uint64_t *myU = lU + threadIdx.x;
    int m[KMAX];
    int k = unrank<KMAX>(np, M, K, q0, m);
    uint64_t mpack = pack_sizes<KMAX>(m);
#pragma unroll
    for (int i = 0; i < KMAX; i++) { myS[i * stride] = MT(0); myU[i * stride] = 0ull; }
    uint32_t q = q0;
    int t = 0, p = 0, bp = -1, breq = 0;
    uint64_t bu = 0;
    for (;;) {
        const int tau = L.sigma[t];
        const int mm = (int)L.mmin[tau];
        const MT fb = ACT ? (MT)L.forbid[tau] : MT(0);
        // next candidate part that can hold tau (Lemma 2 size, ACT pairs)
        while (p < k && (mm > size_of(mpack, p) || (ACT && (fb & myS[p * stride])))) p++;
        if (p < k) {
            const int mp = size_of(mpack, p);
            const MT Sp = myS[p * stride];
            uint64_t Un;
            if (part_test_add<MT>(L, tb, Sp, tau, mp, myU[p * stride], &Un, ty)) {
                int req = 0;
                if (SMS) req = min_units<MT>(L, tb, Sp | (MT(1) << tau), mp, ty);
                const bool better = (bp < 0) || (SMS ? (req < breq || (req == breq && Un < bu)) : (Un < bu));
                if (better) { bp = p; bu = Un; breq = req; }
            }
            p++;
        }
        bool done = false, ok = false;
        if (p >= k) {
            if (bp < 0) {
                done = true;
            } else {
                myS[bp * stride] |= MT(1) << tau;
                myU[bp * stride] = bu;
                bp = -1;
                p = 0;
                if (++t >= n) done = ok = true;
            }
        }
        if (done) {
            uint64_t mx = 0, sm = 0;
            if (ok) {
                for (int i = 0; i < k; i++) {
                    const uint64_t u = myU[i * stride];
                    mx = max(mx, u);
                    sm += u;
                }
                const Key kk{mx, sm, q, 0ull};
                if (key_less(kk, best)) best = kk;
            }
            if (dbg) {
                uint64_t *d = dbg + 3 * (uint64_t)q;
                d[0] = ok ? mx : ~0ull;
                d[1] = ok ? sm : ~0ull;
                d[2] = ok ? 0ull : ~0ull;
            }
            if (++q >= q1) break;
            k = next_partition<KMAX>(m, K);
            mpack = pack_sizes<KMAX>(m);
#pragma unroll
            for (int i = 0; i < KMAX; i++) { myS[i * stride] = MT(0); myU[i * stride] = 0ull; }
            t = 0;
            p = 0;
            bp = -1;
        }
    }
}

// Loop form 1: one loop step per partitioning (the heuristic of one
// partitioning runs to completion, parts unrolled over registers).
template <int KMAX, bool ACT, bool SMS, typename MT, typename TY>
__device__ void heur_run_nested(const SetLDS &L, const Tables &tb, const uint32_t *np, int n, int M, int K,
                                uint32_t q0, uint32_t q1, Key &best, uint64_t *dbg, TY &ty)
{
    int m[KMAX];
    int k = unrank<KMAX>(np, M, K, q0, m);
    for (uint32_t q = q0;;) {
        MT S[KMAX];
        uint64_t U[KMAX];
        const bool ok = heuristic<KMAX, ACT, SMS, MT>(L, tb, n, m, k, S, U, ty);
        uint64_t mx = 0, sm = 0;
        if (ok) {
#pragma unroll
            for (int i = 0; i < KMAX; i++) { mx = max(mx, U[i]); sm += U[i]; }
            const Key kk{mx, sm, q, 0ull};
            if (key_less(kk, best)) best = kk;
        }
        if (dbg) {
            uint64_t *d = dbg + 3 * (uint64_t)q;
            d[0] = ok ? mx : ~0ull;
            d[1] = ok ? sm : ~0ull;
            d[2] = ok ? 0ull : ~0ull;
        }
        if (++q >= q1) break;
        k = next_partition<KMAX>(m, K);
    }
}

template <int KMAX, bool ACT, bool SMS, typename MT, typename TY>
__device__ void heur_run_front(const SetLDS &L, const Tables &tb, const uint16_t *ms, const uint32_t *np, int n, int M,
                               int K, uint32_t q0, uint32_t q1, Key &best, uint64_t *dbg, TY &ty)
{
    int m[KMAX];
    int k = unrank<KMAX>(np, M, K, q0, m);
    for (uint32_t q = q0;;) {
        MT S[KMAX];
        uint64_t U[KMAX];
        const bool ok = heuristic_front<KMAX, ACT, SMS, MT>(L, tb, ms, n, m, k, S, U, ty);
        uint64_t mx = 0, sm = 0;
        if (ok) {
#pragma unroll
            for (int i = 0; i < KMAX; i++) { mx = max(mx, U[i]); sm += U[i]; }
            const Key kk{mx, sm, q, 0ull};
            if (key_less(kk, best)) best = kk;
        }
        if (dbg) {
            uint64_t *d = dbg + 3 * (uint64_t)q;
            d[0] = ok ? mx : ~0ull;
            d[1] = ok ? sm : ~0ull;
            d[2] = ok ? 0ull : ~0ull;
        }
        if (++q >= q1) break;
        k = next_partition<KMAX>(m, K);
    }
}

// Evaluate partitionings [p0, p1) of one staged set in this block (all
// lanes): through the frontier when the set is small enough, else with
// direct incremental tests.
template <int KMAX, bool ACT, bool SMS, typename MT, int FORM, typename TY>
__device__ void eval_range(const SetLDS &L, const Tables &tb, const Launch &Lp, const uint32_t *np,
                           const uint16_t *order, int n, int M,
                           uint32_t p0, uint32_t p1, uint32_t p_lo, uint32_t p_hi, Key &best, uint64_t *dbg, TY &ty)
{
    const uint32_t cnt = p1 - p0;
    const uint32_t per = (cnt + blockDim.x - 1) / blockDim.x;
    uint32_t q0 = p0 + threadIdx.x * per, q1 = min(p1, q0 + per);
    q0 = max(q0, p_lo);
    q1 = min(q1, p_hi);
    if (Lp.front_n > 0 && n <= Lp.front_n) {
        uint16_t *ms = (uint16_t *)(capart_dyn_lds + Lp.table_words);
        build_frontier<MT>(L, tb, n, M, ms, order, ty);
        if (q0 < q1) heur_run_front<KMAX, ACT, SMS, MT>(L, tb, ms, np, n, M, Lp.K, q0, q1, best, dbg, ty);
        return;
    }
    if (q0 >= q1) return;
    if (FORM == 2) {
        uint64_t *lU = (uint64_t *)(capart_dyn_lds + Lp.table_words + Lp.front_words);
        MT *lS = (MT *)(lU + KMAX * blockDim.x);
        heur_run<KMAX, ACT, SMS, MT>(L, tb, np, n, M, Lp.K, q0, q1, best, dbg, lS, lU, ty);
    } else {
        heur_run_nested<KMAX, ACT, SMS, MT>(L, tb, np, n, M, Lp.K, q0, q1, best, dbg, ty);
    }
}

template <int KMAX, bool ACT, bool SMS, typename MT, int FORM, bool COUNT = false>
__global__ __launch_bounds__(256) void eval_heur_kernel(Batch b, Work w, Out o, Launch Lp, uint32_t p_lo,
                                                        uint32_t p_hi)
{
    __shared__ SetLDS L;
    __shared__ Key red[16];
    typename std::conditional<COUNT, Tally, NoTally>::type ty;
    const int64_t s = Lp.s0 + blockIdx.x / Lp.chunks;
    const int c = blockIdx.x % Lp.chunks;
    const uint32_t f = w.setflags[s];
    if (!(f & SETF_VALID)) return;
    const int64_t off = b.off[s];
    const int n = (int)(b.off[s + 1] - off);
    const int M = b.M[s];
    const uint32_t P = w.np[np_index(Lp.K, M, M)];
    const uint32_t p0 = (uint32_t)c * Lp.chunk;
    if (p0 >= P) return;
    const uint32_t p1 = min(P, p0 + Lp.chunk);
    uint64_t *dbg = o.dbg_key ? o.dbg_key + 3 * o.dbg_offset[s] : nullptr;
    Key best = key_none();
    if (!(f & SETF_LEMMA1)) {
        Tables tb;
        stage_set(L, w, off, n, M, s, ACT, tb);
        eval_range<KMAX, ACT, SMS, MT, FORM>(L, tb, Lp, w.np, w.order, n, M, p0, p1, p_lo, p_hi, best, dbg, ty);
    } else if (dbg) {
        for (uint32_t q = p0 + threadIdx.x; q < p1; q += blockDim.x) {
            if (q < p_lo || q >= p_hi) continue;
            uint64_t *d = dbg + 3 * (uint64_t)q;
            d[0] = d[1] = d[2] = ~0ull;
        }
    }
    best = block_min(best, red);
    if (threadIdx.x == 0) {
        uint64_t *dst = w.partial + 4 * ((s) * (int64_t)Lp.chunks + c);
        dst[0] = best.a; dst[1] = best.b; dst[2] = best.c; dst[3] = best.d;
    }
    if constexpr (COUNT) {
        uint64_t a = ty.terms, bb = ty.tests, cc = ty.looks;
#pragma unroll
        for (int o2 = 32; o2 >= 1; o2 >>= 1) {
            a += __shfl_xor(a, o2, 64);
            bb += __shfl_xor(bb, o2, 64);
            cc += __shfl_xor(cc, o2, 64);
        }
        if ((threadIdx.x & 63) == 0 && w.counters) {
            atomicAdd((unsigned long long *)&w.counters[0], (unsigned long long)a);
            atomicAdd((unsigned long long *)&w.counters[1], (unsigned long long)bb);
            atomicAdd((unsigned long long *)&w.counters[2], (unsigned long long)cc);
        }
    }
}

// eval, batched form: a persistent grid; each block repeatedly takes the next
// work item (set, partitioning range) from a global counter, restages the
// set's LDS tables only when the set changes, and writes the item's best key
// to its partial slot.  Items come largest first, so the tail is short.
template <int KMAX, bool ACT, bool SMS, typename MT, int FORM>
__global__ __launch_bounds__(256) void eval_persistent_kernel(Batch b, Work w, Out o, Launch Lp)
{
    __shared__ SetLDS L;
    __shared__ Key red[16];
    __shared__ uint32_t s_item;
    int64_t staged = -1;
    Tables tb;
    tb.C = tb.U = nullptr;
    tb.n = 0;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(w.counter, 1u);
        __syncthreads();
        const uint32_t it = s_item;
        __syncthreads();
        if (it >= w.n_items) break;
        const WorkItem wi = w.items[it];
        const int64_t s = wi.set;
        const uint32_t f = w.setflags[s];
        Key best = key_none();
        uint64_t *dbg = o.dbg_key ? o.dbg_key + 3 * o.dbg_offset[s] : nullptr;
        if ((f & SETF_VALID) && !(f & SETF_LEMMA1)) {
            const int64_t off = b.off[s];
            const int n = (int)(b.off[s + 1] - off);
            const int M = b.M[s];
            if (s != staged) {
                stage_set(L, w, off, n, M, s, ACT, tb);
                staged = s;
            }
            NoTally nt;
            eval_range<KMAX, ACT, SMS, MT, FORM>(L, tb, Lp, w.np, w.order, n, M, wi.p0, wi.p1, 0u, 0xFFFFFFFFu, best, dbg, nt);
        } else if (dbg && (f & SETF_VALID)) {
            for (uint32_t q = wi.p0 + threadIdx.x; q < wi.p1; q += blockDim.x) {
                uint64_t *d = dbg + 3 * (uint64_t)q;
                d[0] = d[1] = d[2] = ~0ull;
            }
        }
        best = block_min(best, red);
        if (threadIdx.x == 0) {
            uint64_t *dst = w.partial + 4 * (uint64_t)wi.slot;
            dst[0] = best.a; dst[1] = best.b; dst[2] = best.c; dst[3] = best.d;
        }
        __syncthreads();
    }
}

// eval, exhaustive allocation: one block per (set, partitioning); lanes stride
// over allocation indices (base-k digits, task 0 most significant).
template <int KMAX>
__global__ __launch_bounds__(256) void eval_exh_kernel(Batch b, Work w, Out o, Launch Lp, uint32_t p_lo,
                                                       uint32_t p_hi)
{
    __shared__ SetLDS L;
    __shared__ Key red[16];
    const int64_t s = Lp.s0 + blockIdx.x / Lp.chunks;
    const uint32_t q = blockIdx.x % Lp.chunks;
    const uint32_t f = w.setflags[s];
    if (!(f & SETF_VALID)) return;
    const int64_t off = b.off[s];
    const int n = (int)(b.off[s + 1] - off);
    const int M = b.M[s];
    const uint32_t P = w.np[np_index(Lp.K, M, M)];
    if (q >= P) return;
    Key best = key_none();
    if (!(f & SETF_LEMMA1) && q >= p_lo && q < p_hi) {
        Tables tb;
        stage_set(L, w, off, n, M, s, false, tb);
        int m[KMAX];
        const int k = unrank<KMAX>(w.np, M, Lp.K, q, m);
        uint64_t A = 1;
        for (int i = 0; i < n; i++) A *= (uint64_t)k;
        for (uint64_t a = threadIdx.x; a < A; a += blockDim.x) {
            uint64_t S[KMAX];
#pragma unroll
            for (int p = 0; p < KMAX; p++) S[p] = 0ull;
            uint64_t x = a;
            for (int i = n - 1; i >= 0; i--) {
                const int d = (int)(x % (uint64_t)k);
                x /= (uint64_t)k;
                const uint64_t bit = 1ull << L.rank_of[i];
#pragma unroll
                for (int p = 0; p < KMAX; p++)
                    if (p == d) S[p] |= bit;
            }
            bool ok = true;
            uint64_t mx = 0, sm = 0;
#pragma unroll
            for (int p = 0; p < KMAX; p++) {
                if (ok && p < k && S[p]) {
                    uint64_t u;
                    NoTally nt;
                    if (!part_test<uint64_t>(L, tb, S[p], m[p], &u, nt)) {
                        ok = false;
                    } else {
                        mx = max(mx, u);
                        sm += u;
                    }
                }
            }
            if (ok) {
                const Key kk{mx, sm, q, a};
                if (key_less(kk, best)) best = kk;
            }
        }
    }
    best = block_min(best, red);
    if (threadIdx.x == 0) {
        uint64_t *dst = w.partial + 4 * ((s) * (int64_t)Lp.chunks + q);
        dst[0] = best.a; dst[1] = best.b; dst[2] = best.c; dst[3] = best.d;
        if (o.dbg_key != nullptr && q >= p_lo && q < p_hi) {
            uint64_t *d = o.dbg_key + 3 * (o.dbg_offset[s] + q);
            d[0] = best.a; d[1] = best.b; d[2] = best.d;
        }
    }
}

// ---------------------------------------------------------------------------
// final: one wave per set.
template <int KMAX>
__global__ __launch_bounds__(64) void final_kernel(Batch b, Work w, Out o, Launch Lp)
{
    __shared__ SetLDS L;
    __shared__ uint64_t sS[KMAX];
    __shared__ int sm_[KMAX];
    __shared__ int sk;
    const int64_t s = Lp.s0 + blockIdx.x;
    const int lane = threadIdx.x;
    const uint32_t f = w.setflags[s];
    const int K = Lp.K;
    if (!(f & SETF_VALID)) {
        const int64_t off0 = b.off[s], off1 = b.off[s + 1];
        if (lane == 0) {
            o.verdict[s] = 0; o.verdict_1g[s] = 0; o.pidx[s] = -1; o.aidx[s] = -1;
            o.maxU[s] = 0; o.sumU[s] = 0; o.n_evals[s] = 0;
        }
        for (int p = lane; p < K; p += 64) o.sizes[s * K + p] = 0;
        if (off0 >= 0 && off1 >= off0 && off1 <= b.n_tasks_total) {
            for (int64_t i = off0 + lane; i < off1; i += 64) { o.alloc[i] = -1; o.R[i] = -1; o.R_1g[i] = -1; }
        }
        return;
    }
    const int64_t off = b.off[s];
    const int n = (int)(b.off[s + 1] - off);
    const int M = b.M[s];
    const uint32_t P = w.np[np_index(K, M, M)];
    // reduce the partials of this set's live chunks
    Key best = key_none();
    const bool exh = (Lp.mode == CAPART_EXHAUSTIVE);
    if (w.slot_off != nullptr) {  // batched form: the set's item slots
        for (uint32_t c = w.slot_off[s] + lane; c < w.slot_off[s + 1]; c += 64) {
            const uint64_t *src = w.partial + 4 * (uint64_t)c;
            const Key kk{src[0], src[1], src[2], src[3]};
            if (key_less(kk, best)) best = kk;
        }
    } else {
        for (int c = lane; c < Lp.chunks; c += 64) {
            const bool live = exh ? ((uint32_t)c < P) : ((uint64_t)c * Lp.chunk < P);
            if (!live) continue;
            const uint64_t *src = w.partial + 4 * (s * (int64_t)Lp.chunks + c);
            const Key kk{src[0], src[1], src[2], src[3]};
            if (key_less(kk, best)) best = kk;
        }
    }
    best = wave_min(best);
    const bool found = best.a != ~0ull;
    const bool act = (Lp.mode == CAPART_HEUR_BF_ACT || Lp.mode == CAPART_HEUR_SMS_ACT);
    Tables tb;
    stage_set(L, w, off, n, M, s, act, tb);
    if (found && lane == 0) {
        int m[KMAX];
        int k = unrank<KMAX>(w.np, M, K, (uint32_t)best.c, m);
        uint64_t S[KMAX], U[KMAX];
#pragma unroll
        for (int p = 0; p < KMAX; p++) S[p] = 0ull;
        if (exh) {
            uint64_t x = best.d;
            for (int i = n - 1; i >= 0; i--) {
                const int d = (int)(x % (uint64_t)k);
                x /= (uint64_t)k;
#pragma unroll
                for (int p = 0; p < KMAX; p++)
                    if (p == d) S[p] |= 1ull << L.rank_of[i];
            }
        } else {
            NoTally nt;
            switch (Lp.mode) {
            case CAPART_HEUR_BF_INA: heuristic<KMAX, false, false, uint64_t>(L, tb, n, m, k, S, U, nt); break;
            case CAPART_HEUR_BF_ACT: heuristic<KMAX, true, false, uint64_t>(L, tb, n, m, k, S, U, nt); break;
            case CAPART_HEUR_SMS_INA: heuristic<KMAX, false, true, uint64_t>(L, tb, n, m, k, S, U, nt); break;
            default: heuristic<KMAX, true, true, uint64_t>(L, tb, n, m, k, S, U, nt); break;
            }
        }
#pragma unroll
        for (int p = 0; p < KMAX; p++) { sS[p] = S[p]; sm_[p] = m[p]; }
        sk = k;
    }
    __syncthreads();
    // response times of the chosen triple
    if (lane < n) {
        const int64_t gi = off + L.orig[lane];
        if (found) {
            int part = 0, mp = 0;
            uint64_t Sp = 0;
            for (int p = 0; p < sk; p++)
                if ((sS[p] >> lane) & 1ull) { part = p; mp = sm_[p]; Sp = sS[p]; }
            const uint32_t R = rta_one<uint64_t>(L, tb, mp, lane, Sp & ((1ull << lane) - 1ull),
                                                 conflict_mask<uint64_t>(Sp, L.memmask));
            o.alloc[gi] = (int8_t)part;
            o.R[gi] = R ? (int64_t)R : -1;
        } else {
            o.alloc[gi] = -1;
            o.R[gi] = -1;
        }
    }
    // whole-GPU baseline: every task on one partition of M units
    bool ok1 = true;
    if (!(Lp.flags & CAPART_FLAG_SKIP_1G)) {
        const uint64_t all = (n == 64) ? ~0ull : ((1ull << n) - 1ull);
        uint32_t R1 = 0;
        if (lane < n) {
            R1 = rta_one<uint64_t>(L, tb, M, lane, all & ((1ull << lane) - 1ull), conflict_mask<uint64_t>(all, L.memmask));
            o.R_1g[off + L.orig[lane]] = R1 ? (int64_t)R1 : -1;
        }
        ok1 = !__ballot(lane < n && R1 == 0u);
    } else {
        if (lane < n) o.R_1g[off + L.orig[lane]] = -1;
        ok1 = false;
    }
    if (lane == 0) {
        o.verdict[s] = found ? 1 : 0;
        o.verdict_1g[s] = ok1 ? 1 : 0;
        o.pidx[s] = found ? (int32_t)best.c : -1;
        o.aidx[s] = found ? (int64_t)best.d : -1;
        o.maxU[s] = found ? best.a : 0ull;
        o.sumU[s] = found ? best.b : 0ull;
        o.n_evals[s] = (int64_t)P;
    }
    for (int p = lane; p < K; p += 64) o.sizes[s * K + p] = (found && p < KMAX) ? sm_[p] : 0;
}

// ---------------------------------------------------------------------------
// Exhaustive allocation through subset tables (sets of at most 14 tasks, at
// most 4 parts).  tab[set][m-1][A] = Q32 utilisation of task subset A (bits
// = task indices within the set) on one partition of m units, or all ones if
// A is not schedulable there.  One block per (set, m) fills it.
__global__ __launch_bounds__(256) void subset_table_kernel(Batch b, Work w, Launch Lp, uint64_t *tab, int64_t s_begin,
                                                           int W, int Mtab, int ntab)
{
    __shared__ SetLDS L;
    const int s_local = blockIdx.x / Mtab;
    const int m = blockIdx.x % Mtab + 1;
    if (s_local >= W) return;
    const int64_t s = s_begin + s_local;
    const uint32_t f = w.setflags[s];
    if (!(f & SETF_VALID) || (f & SETF_LEMMA1)) return;
    const int64_t off = b.off[s];
    const int n = (int)(b.off[s + 1] - off);
    const int M = b.M[s];
    if (m > M || n > ntab) return;
    Tables tb;
    stage_set(L, w, off, n, M, s, false, tb);
    uint64_t *dst = tab + (((size_t)s_local * Mtab + (size_t)(m - 1)) << ntab);
    const uint32_t NA = 1u << n;
    for (uint32_t A = threadIdx.x; A < NA; A += blockDim.x) {
        uint32_t RA = 0;
        for (uint32_t a = A; a; a &= a - 1u) RA |= 1u << L.rank_of[__builtin_ctz(a)];
        uint64_t u = 0;
        NoTally nt;
        dst[A] = part_test<uint32_t>(L, tb, RA, m, &u, nt) ? u : ~0ull;
    }
}

// Depth-first search over allocations of one (set, partitioning), in
// allocation-index order (task 0 most significant).  Lane l owns the digits
// of the first tasks (prefix l of k^Lpre <= blockDim) and searches the rest.
// Exact pruning: a part that is not schedulable stays so when tasks are added;
// part utilisations only grow, so a partial (maxU, sumU) at or above the
// lane's best cannot lead to a better or equal key with a smaller index; among
// parts of equal size only the labelling whose first tasks come in part order
// is visited (it is the smallest index among the relabellings, which share
// their key).  Blocks are dealt to XCDs by set (block b runs on XCD b mod 8),
// so all partitionings of a set read its table from one L2.
__global__ __launch_bounds__(256) void exh_dfs_kernel(Batch b, Work w, Out o, Launch Lp, const uint64_t *tab,
                                                      int64_t s_begin, int W, int Mtab, int ntab, uint32_t Pmax,
                                                      uint32_t p_lo, uint32_t p_hi)
{
    __shared__ Key red[16];
    __shared__ uint64_t pw[16];
    __shared__ unsigned long long shared_mx;  // smallest maxU of any complete allocation found in the block
    const uint32_t xcd = blockIdx.x & 7u, j = blockIdx.x >> 3;
    const int s_local = (int)(xcd + 8u * (j / Pmax));
    const uint32_t q = j % Pmax;
    if (s_local >= W) return;
    const int64_t s = s_begin + s_local;
    const uint32_t f = w.setflags[s];
    if (!(f & SETF_VALID)) return;
    const int64_t off = b.off[s];
    const int n = (int)(b.off[s + 1] - off);
    const int M = b.M[s];
    const uint32_t P = w.np[np_index(Lp.K, M, M)];
    if (q >= P) return;
    Key best = key_none();
    int m[4];
    const int k = unrank<4>(w.np, M, Lp.K, q, m);
    if (threadIdx.x == 0) {
        uint64_t v = 1;
        for (int i = n - 1; i >= 0; i--) { pw[i] = v; v *= (uint64_t)k; }
        shared_mx = ~0ull;
    }
    __syncthreads();
    int Lpre = 0;
    uint32_t npre = 1;
    while (Lpre < n && npre * (uint32_t)k <= blockDim.x) { npre *= (uint32_t)k; Lpre++; }
    const uint64_t msz = (uint64_t)(uint32_t)m[0] | ((uint64_t)(uint32_t)m[1] << 8) | ((uint64_t)(uint32_t)m[2] << 16) |
                         ((uint64_t)(uint32_t)m[3] << 24);
    if (!(f & SETF_LEMMA1) && threadIdx.x < npre && q >= p_lo && q < p_hi) {
        const uint64_t *t = tab + (((size_t)s_local * Mtab) << ntab);
        // prefix digits: task Lpre-1 least significant
        uint64_t Apack = 0, aidx = 0;
        uint32_t x = threadIdx.x;
        for (int i = Lpre - 1; i >= 0; i--) {
            const int d = (int)(x % (uint32_t)k);
            x /= (uint32_t)k;
            Apack |= (uint64_t)(1u << i) << (16 * d);
            aidx += (uint64_t)d * pw[i];
        }
        uint64_t U[4];
        bool ok = true;
#pragma unroll
        for (int p = 0; p < 4; p++) {
            const uint32_t Ap = (uint32_t)(Apack >> (16 * p)) & 0xFFFFu;
            U[p] = 0ull;
            if (p < k) {
                U[p] = t[((size_t)(m[p] - 1) << ntab) | Ap];
                if (U[p] == ~0ull) ok = false;
                if (p > 0 && m[p - 1] == m[p] && Ap) {
                    const uint32_t Aq = (uint32_t)(Apack >> (16 * (p - 1))) & 0xFFFFu;
                    if (!Aq || __builtin_ctz(Aq) > __builtin_ctz(Ap)) ok = false;
                }
            }
        }
        if (ok) {
            uint64_t mx = 0, sm = 0;
#pragma unroll
            for (int p = 0; p < 4; p++) { mx = max(mx, U[p]); sm += U[p]; }
            if (Lpre == n) {
                best = Key{mx, sm, q, aidx};
            } else {
                // other lanes' complete allocations bound maxU strictly: a
                // partial maxU above one can never win, whatever its index
                uint64_t dig = 0;
                int i = Lpre, p = 0;
                for (;;) {
                    bool placed = false;
                    for (; p < k; p++) {
                        const int mp = (int)((msz >> (8 * p)) & 0xFFu);
                        if (p > 0 && (int)((msz >> (8 * (p - 1))) & 0xFFu) == mp &&
                            ((Apack >> (16 * (p - 1))) & 0xFFFFull) == 0ull)
                            continue;
                        const uint32_t An = ((uint32_t)(Apack >> (16 * p)) & 0xFFFFu) | (1u << i);
                        const uint64_t u = t[((size_t)(mp - 1) << ntab) | An];
                        if (u == ~0ull) continue;
                        uint64_t nmx = 0, nsm = 0;
#pragma unroll
                        for (int r = 0; r < 4; r++) {
                            const uint64_t v = (r == p) ? u : U[r];
                            nmx = max(nmx, v);
                            nsm += v;
                        }
                        if (nmx > best.a || (nmx == best.a && nsm >= best.b)) continue;
                        if (nmx > (uint64_t)*(volatile unsigned long long *)&shared_mx) continue;
                        if (i == n - 1) {
                            best = Key{nmx, nsm, q, aidx + (uint64_t)p * pw[i]};
                            atomicMin(&shared_mx, (unsigned long long)nmx);
                            continue;
                        }
                        Apack |= (uint64_t)(1u << i) << (16 * p);
#pragma unroll
                        for (int r = 0; r < 4; r++)
                            if (r == p) U[r] = u;
                        aidx += (uint64_t)p * pw[i];
                        dig = (dig & ~(0xFull << (4 * i))) | ((uint64_t)p << (4 * i));
                        placed = true;
                        break;
                    }
                    if (placed) {
                        i++;
                        p = 0;
                        continue;
                    }
                    if (i == Lpre) break;
                    i--;
                    const int pd = (int)((dig >> (4 * i)) & 0xFull);
                    Apack &= ~((uint64_t)(1u << i) << (16 * pd));
                    const int mpd = (int)((msz >> (8 * pd)) & 0xFFu);
                    const uint64_t ur = t[((size_t)(mpd - 1) << ntab) | ((uint32_t)(Apack >> (16 * pd)) & 0xFFFFu)];
#pragma unroll
                    for (int r = 0; r < 4; r++)
                        if (r == pd) U[r] = ur;
                    aidx -= (uint64_t)pd * pw[i];
                    p = pd + 1;
                }
            }
        }
    }
    best = block_min(best, red);
    if (threadIdx.x == 0) {
        uint64_t *dst = w.partial + 4 * (s * (int64_t)Lp.chunks + q);
        dst[0] = best.a; dst[1] = best.b; dst[2] = best.c; dst[3] = best.d;
        if (o.dbg_key != nullptr && q >= p_lo && q < p_hi) {
            uint64_t *d = o.dbg_key + 3 * (o.dbg_offset[s] + q);
            d[0] = best.a; d[1] = best.b; d[2] = best.d;
        }
    }
}

// ---------------------------------------------------------------------------
// One triple of one set (set 0 of the batch): every task tested, one lane each.
template <int KMAX>
__global__ __launch_bounds__(64) void triple_kernel(Batch b, Work w, const int32_t *sizes, int k, const int8_t *alloc,
                                                    uint8_t *feasible, int64_t *Rout, uint64_t *maxU, uint64_t *sumU)
{
    __shared__ SetLDS L;
    __shared__ uint64_t sS[KMAX];
    __shared__ unsigned long long sU[KMAX];
    const int lane = threadIdx.x;
    if (!(w.setflags[0] & SETF_VALID)) return;
    const int n = (int)(b.off[1] - b.off[0]);
    const int M = b.M[0];  // every part size is in [1, M] (checked by the host)
    Tables tb;
    stage_set(L, w, 0, n, M, 0, false, tb);
    if (lane < KMAX) { sS[lane] = 0ull; sU[lane] = 0ull; }
    __syncthreads();
    if (lane < n) {
        const int p = alloc[L.orig[lane]];
        atomicOr((unsigned long long *)&sS[p], (unsigned long long)(1ull << lane));
    }
    __syncthreads();
    uint32_t R = 0;
    if (lane < n) {
        const int p = alloc[L.orig[lane]];
        const uint64_t Sp = sS[p];
        const uint64_t cm = conflict_mask<uint64_t>(Sp, L.memmask);
        R = rta_one<uint64_t>(L, tb, sizes[p], lane, Sp & ((1ull << lane) - 1ull), cm);
        Rout[L.orig[lane]] = R ? (int64_t)R : -1;
        if (R) {
            const uint32_t u = tb.U[(sizes[p] - 1) * 2 * n + (int)((cm >> lane) & 1ull) * n + lane];
            atomicAdd(&sU[p], (unsigned long long)u + 1ull);
        }
    }
    const bool ok = !__ballot(lane < n && R == 0u);
    __syncthreads();
    if (lane == 0) {
        uint64_t mx = 0, sm = 0;
        for (int p = 0; p < k; p++) { mx = max(mx, (uint64_t)sU[p]); sm += sU[p]; }
        *feasible = ok ? 1 : 0;
        *maxU = ok ? mx : 0ull;
        *sumU = ok ? sm : 0ull;
    }
}

// ---------------------------------------------------------------------------
// Per-set tables: 4 u32 per (m, task) pair; every valid set has n * M <= CAPART_MAX_NM.
size_t table_lds_bytes(int max_tasks, int max_M)
{
    const long nm = (long)max_tasks * max_M;
    return (size_t)16 * (size_t)(nm < CAPART_MAX_NM ? nm : CAPART_MAX_NM);
}

// Blocks of 256 threads, or 128 when the tables are large, so that tables,
// per-lane part state (at most 8 parts x 16 bytes per lane) and the static
// per-set arrays fit the 160 KB of LDS.
int eval_threads(int max_tasks, int max_M) { return table_lds_bytes(max_tasks, max_M) > 96 * 1024 ? 128 : 256; }

static size_t dyn_bytes(const Batch &b) { return table_lds_bytes(min(b.max_tasks, MAXN), min(b.max_M, 255)); }

template <int KMAX, typename MT>
static size_t heur_dyn_bytes(const Launch &L, int form)
{
    return (size_t)4 * (L.table_words + L.front_words) +
           (form == 2 ? (size_t)L.threads * KMAX * (sizeof(MT) + sizeof(uint64_t)) : 0);
}

hipError_t launch_prep(const Batch &b, const Work &w, const Out &o, const Launch &L, hipStream_t st)
{
    if (L.S <= 0) return hipSuccess;
    hipLaunchKernelGGL(prep_kernel, dim3((unsigned)L.S), dim3(64), 0, st, b, w, o, L);
    return hipGetLastError();
}

template <int KMAX, typename MT, int FORM>
static hipError_t launch_heur(const Launch &L, const Batch &b, const Work &w, const Out &o, hipStream_t st,
                              uint32_t p_lo, uint32_t p_hi)
{
    const dim3 grid((unsigned)(L.S * L.chunks)), block((unsigned)L.threads);
    const size_t lds = heur_dyn_bytes<KMAX, MT>(L, FORM);
    switch (L.mode) {
    case CAPART_HEUR_BF_INA:
        hipLaunchKernelGGL((eval_heur_kernel<KMAX, false, false, MT, FORM>), grid, block, lds, st, b, w, o, L, p_lo,
                           p_hi);
        break;
    case CAPART_HEUR_BF_ACT:
        hipLaunchKernelGGL((eval_heur_kernel<KMAX, true, false, MT, FORM>), grid, block, lds, st, b, w, o, L, p_lo,
                           p_hi);
        break;
    case CAPART_HEUR_SMS_INA:
        hipLaunchKernelGGL((eval_heur_kernel<KMAX, false, true, MT, FORM>), grid, block, lds, st, b, w, o, L, p_lo,
                           p_hi);
        break;
    default:
        hipLaunchKernelGGL((eval_heur_kernel<KMAX, true, true, MT, FORM>), grid, block, lds, st, b, w, o, L, p_lo,
                           p_hi);
        break;
    }
    return hipGetLastError();
}

template <int KMAX, typename MT>
static hipError_t launch_eval_k(const Batch &b, const Work &w, const Out &o, const Launch &L, hipStream_t st,
                                uint32_t p_lo, uint32_t p_hi)
{
    if (L.mode == CAPART_EXHAUSTIVE) {
        const dim3 grid((unsigned)(L.S * L.chunks)), block((unsigned)L.threads);
        hipLaunchKernelGGL((eval_exh_kernel<KMAX>), grid, block, dyn_bytes(b), st, b, w, o, L, p_lo, p_hi);
        return hipGetLastError();
    }
    return L.form == 2 ? launch_heur<KMAX, MT, 2>(L, b, w, o, st, p_lo, p_hi)
                       : launch_heur<KMAX, MT, 1>(L, b, w, o, st, p_lo, p_hi);
}

template <int KMAX, typename MT, int FORM>
static hipError_t launch_persistent_k(const Batch &b, const Work &w, const Out &o, const Launch &L, int blocks,
                                      hipStream_t st)
{
    const dim3 grid((unsigned)blocks), block((unsigned)L.threads);
    const size_t lds = heur_dyn_bytes<KMAX, MT>(L, FORM);
    switch (L.mode) {
    case CAPART_HEUR_BF_INA:
        hipLaunchKernelGGL((eval_persistent_kernel<KMAX, false, false, MT, FORM>), grid, block, lds, st, b, w, o, L);
        break;
    case CAPART_HEUR_BF_ACT:
        hipLaunchKernelGGL((eval_persistent_kernel<KMAX, true, false, MT, FORM>), grid, block, lds, st, b, w, o, L);
        break;
    case CAPART_HEUR_SMS_INA:
        hipLaunchKernelGGL((eval_persistent_kernel<KMAX, false, true, MT, FORM>), grid, block, lds, st, b, w, o, L);
        break;
    default:
        hipLaunchKernelGGL((eval_persistent_kernel<KMAX, true, true, MT, FORM>), grid, block, lds, st, b, w, o, L);
        break;
    }
    return hipGetLastError();
}

template <int KMAX, typename MT>
static hipError_t launch_persistent_f(const Batch &b, const Work &w, const Out &o, const Launch &L, int blocks,
                                      hipStream_t st)
{
    return L.form == 2 ? launch_persistent_k<KMAX, MT, 2>(b, w, o, L, blocks, st)
                       : launch_persistent_k<KMAX, MT, 1>(b, w, o, L, blocks, st);
}

hipError_t launch_eval_persistent(const Batch &b, const Work &w, const Out &o, const Launch &L, int blocks,
                                  hipStream_t st)
{
    if (b.max_tasks <= 32)
        return L.K <= 4 ? launch_persistent_f<4, uint32_t>(b, w, o, L, blocks, st)
                        : launch_persistent_f<8, uint32_t>(b, w, o, L, blocks, st);
    return L.K <= 4 ? launch_persistent_f<4, uint64_t>(b, w, o, L, blocks, st)
                    : launch_persistent_f<8, uint64_t>(b, w, o, L, blocks, st);
}

int device_cu_count()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 256;
    return cus;
}

template <int KMAX, typename MT>
static hipError_t launch_count_k(const Batch &b, const Work &w, const Out &o, const Launch &L, hipStream_t st)
{
    const dim3 grid((unsigned)(L.S * L.chunks)), block((unsigned)L.threads);
    const size_t lds = heur_dyn_bytes<KMAX, MT>(L, 1);
    const uint32_t lo = 0u, hi = 0xFFFFFFFFu;
    switch (L.mode) {
    case CAPART_HEUR_BF_INA:
        hipLaunchKernelGGL((eval_heur_kernel<KMAX, false, false, MT, 1, true>), grid, block, lds, st, b, w, o, L, lo, hi);
        break;
    case CAPART_HEUR_BF_ACT:
        hipLaunchKernelGGL((eval_heur_kernel<KMAX, true, false, MT, 1, true>), grid, block, lds, st, b, w, o, L, lo, hi);
        break;
    case CAPART_HEUR_SMS_INA:
        hipLaunchKernelGGL((eval_heur_kernel<KMAX, false, true, MT, 1, true>), grid, block, lds, st, b, w, o, L, lo, hi);
        break;
    default:
        hipLaunchKernelGGL((eval_heur_kernel<KMAX, true, true, MT, 1, true>), grid, block, lds, st, b, w, o, L, lo, hi);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_eval_count(const Batch &b, const Work &w, const Out &o, const Launch &L, hipStream_t st)
{
    if (L.S <= 0 || L.mode == CAPART_EXHAUSTIVE) return hipSuccess;
    if (b.max_tasks <= 32)
        return L.K <= 4 ? launch_count_k<4, uint32_t>(b, w, o, L, st) : launch_count_k<8, uint32_t>(b, w, o, L, st);
    return L.K <= 4 ? launch_count_k<4, uint64_t>(b, w, o, L, st) : launch_count_k<8, uint64_t>(b, w, o, L, st);
}

hipError_t launch_eval_range(const Batch &b, const Work &w, const Out &o, const Launch &L, hipStream_t st,
                             uint32_t p_lo, uint32_t p_hi)
{
    if (L.S <= 0) return hipSuccess;
    // 32-bit rank masks when every set of the launch has at most 32 tasks
    if (b.max_tasks <= 32)
        return L.K <= 4 ? launch_eval_k<4, uint32_t>(b, w, o, L, st, p_lo, p_hi)
                        : launch_eval_k<8, uint32_t>(b, w, o, L, st, p_lo, p_hi);
    return L.K <= 4 ? launch_eval_k<4, uint64_t>(b, w, o, L, st, p_lo, p_hi)
                    : launch_eval_k<8, uint64_t>(b, w, o, L, st, p_lo, p_hi);
}

hipError_t launch_eval(const Batch &b, const Work &w, const Out &o, const Launch &L, hipStream_t st)
{
    return launch_eval_range(b, w, o, L, st, 0u, 0xFFFFFFFFu);
}

hipError_t launch_subset_tables(const Batch &b, const Work &w, const Launch &L, uint64_t *tab, int64_t s_begin, int W,
                                int Mtab, int ntab, hipStream_t st)
{
    hipLaunchKernelGGL(subset_table_kernel, dim3((unsigned)(W * Mtab)), dim3(256), dyn_bytes(b), st, b, w, L, tab,
                       s_begin, W, Mtab, ntab);
    return hipGetLastError();
}

hipError_t launch_exh_dfs(const Batch &b, const Work &w, const Out &o, const Launch &L, const uint64_t *tab,
                          int64_t s_begin, int W, int Mtab, int ntab, uint32_t Pmax, uint32_t p_lo, uint32_t p_hi,
                          hipStream_t st)
{
    const unsigned blocks = 8u * (unsigned)((W + 7) / 8) * Pmax;
    hipLaunchKernelGGL(exh_dfs_kernel, dim3(blocks), dim3(256), 0, st, b, w, o, L, tab, s_begin, W, Mtab, ntab, Pmax,
                       p_lo, p_hi);
    return hipGetLastError();
}

hipError_t launch_final(const Batch &b, const Work &w, const Out &o, const Launch &L, hipStream_t st)
{
    if (L.S <= 0) return hipSuccess;
    const size_t lds = dyn_bytes(b);
    if (L.K <= 4)
        hipLaunchKernelGGL((final_kernel<4>), dim3((unsigned)L.S), dim3(64), lds, st, b, w, o, L);
    else
        hipLaunchKernelGGL((final_kernel<8>), dim3((unsigned)L.S), dim3(64), lds, st, b, w, o, L);
    return hipGetLastError();
}

hipError_t launch_triple(const Batch &b, const Work &w, const int32_t *sizes, int k, const int8_t *alloc,
                         uint8_t *feasible, int64_t *R, uint64_t *maxU, uint64_t *sumU, hipStream_t st)
{
    const size_t lds = dyn_bytes(b);
    hipLaunchKernelGGL((triple_kernel<8>), dim3(1), dim3(64), lds, st, b, w, sizes, k, alloc, feasible, R, maxU,
                       sumU);
    return hipGetLastError();
}

// Let a kernel use all of the 160 KB LDS beyond its static arrays.
template <typename F>
static hipError_t allow_lds(F *fn)
{
    hipFuncAttributes a;
    hipError_t e = hipFuncGetAttributes(&a, reinterpret_cast<const void *>(fn));
    if (e != hipSuccess) return e;
    const int dyn = 160 * 1024 - (int)a.sharedSizeBytes;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(fn), hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
}

hipError_t configure_kernels()
{
    hipError_t e = hipSuccess, t;
#define CAPART_ALLOW(fn) do { t = allow_lds(fn); if (t != hipSuccess) e = t; } while (0)
    CAPART_ALLOW((eval_exh_kernel<4>));
    CAPART_ALLOW((eval_exh_kernel<8>));
    CAPART_ALLOW((eval_heur_kernel<4, false, false, uint32_t, 1>));
    CAPART_ALLOW((eval_heur_kernel<4, true, false, uint32_t, 1>));
    CAPART_ALLOW((eval_heur_kernel<4, false, true, uint32_t, 1>));
    CAPART_ALLOW((eval_heur_kernel<4, true, true, uint32_t, 1>));
    CAPART_ALLOW((eval_heur_kernel<4, false, false, uint32_t, 2>));
    CAPART_ALLOW((eval_heur_kernel<4, true, false, uint32_t, 2>));
    CAPART_ALLOW((eval_heur_kernel<4, false, true, uint32_t, 2>));
    CAPART_ALLOW((eval_heur_kernel<4, true, true, uint32_t, 2>));
    CAPART_ALLOW((eval_heur_kernel<4, false, false, uint64_t, 1>));
    CAPART_ALLOW((eval_heur_kernel<4, true, false, uint64_t, 1>));
    CAPART_ALLOW((eval_heur_kernel<4, false, true, uint64_t, 1>));
    CAPART_ALLOW((eval_heur_kernel<4, true, true, uint64_t, 1>));
    CAPART_ALLOW((eval_heur_kernel<4, false, false, uint64_t, 2>));
    CAPART_ALLOW((eval_heur_kernel<4, true, false, uint64_t, 2>));
    CAPART_ALLOW((eval_heur_kernel<4, false, true, uint64_t, 2>));
    CAPART_ALLOW((eval_heur_kernel<4, true, true, uint64_t, 2>));
    CAPART_ALLOW((eval_heur_kernel<8, false, false, uint32_t, 1>));
    CAPART_ALLOW((eval_heur_kernel<8, true, false, uint32_t, 1>));
    CAPART_ALLOW((eval_heur_kernel<8, false, true, uint32_t, 1>));
    CAPART_ALLOW((eval_heur_kernel<8, true, true, uint32_t, 1>));
    CAPART_ALLOW((eval_heur_kernel<8, false, false, uint32_t, 2>));
    CAPART_ALLOW((eval_heur_kernel<8, true, false, uint32_t, 2>));
    CAPART_ALLOW((eval_heur_kernel<8, false, true, uint32_t, 2>));
    CAPART_ALLOW((eval_heur_kernel<8, true, true, uint32_t, 2>));
    CAPART_ALLOW((eval_heur_kernel<8, false, false, uint64_t, 1>));
    CAPART_ALLOW((eval_heur_kernel<8, true, false, uint64_t, 1>));
    CAPART_ALLOW((eval_heur_kernel<8, false, true, uint64_t, 1>));
    CAPART_ALLOW((eval_heur_kernel<8, true, true, uint64_t, 1>));
    CAPART_ALLOW((eval_heur_kernel<8, false, false, uint64_t, 2>));
    CAPART_ALLOW((eval_heur_kernel<8, true, false, uint64_t, 2>));
    CAPART_ALLOW((eval_heur_kernel<8, false, true, uint64_t, 2>));
    CAPART_ALLOW((eval_heur_kernel<8, true, true, uint64_t, 2>));
    CAPART_ALLOW((eval_persistent_kernel<4, false, false, uint32_t, 1>));
    CAPART_ALLOW((eval_persistent_kernel<4, true, false, uint32_t, 1>));
    CAPART_ALLOW((eval_persistent_kernel<4, false, true, uint32_t, 1>));
    CAPART_ALLOW((eval_persistent_kernel<4, true, true, uint32_t, 1>));
    CAPART_ALLOW((eval_persistent_kernel<4, false, false, uint32_t, 2>));
    CAPART_ALLOW((eval_persistent_kernel<4, true, false, uint32_t, 2>));
    CAPART_ALLOW((eval_persistent_kernel<4, false, true, uint32_t, 2>));
    CAPART_ALLOW((eval_persistent_kernel<4, true, true, uint32_t, 2>));
    CAPART_ALLOW((eval_persistent_kernel<4, false, false, uint64_t, 1>));
    CAPART_ALLOW((eval_persistent_kernel<4, true, false, uint64_t, 1>));
    CAPART_ALLOW((eval_persistent_kernel<4, false, true, uint64_t, 1>));
    CAPART_ALLOW((eval_persistent_kernel<4, true, true, uint64_t, 1>));
    CAPART_ALLOW((eval_persistent_kernel<4, false, false, uint64_t, 2>));
    CAPART_ALLOW((eval_persistent_kernel<4, true, false, uint64_t, 2>));
    CAPART_ALLOW((eval_persistent_kernel<4, false, true, uint64_t, 2>));
    CAPART_ALLOW((eval_persistent_kernel<4, true, true, uint64_t, 2>));
    CAPART_ALLOW((eval_persistent_kernel<8, false, false, uint32_t, 1>));
    CAPART_ALLOW((eval_persistent_kernel<8, true, false, uint32_t, 1>));
    CAPART_ALLOW((eval_persistent_kernel<8, false, true, uint32_t, 1>));
    CAPART_ALLOW((eval_persistent_kernel<8, true, true, uint32_t, 1>));
    CAPART_ALLOW((eval_persistent_kernel<8, false, false, uint32_t, 2>));
    CAPART_ALLOW((eval_persistent_kernel<8, true, false, uint32_t, 2>));
    CAPART_ALLOW((eval_persistent_kernel<8, false, true, uint32_t, 2>));
    CAPART_ALLOW((eval_persistent_kernel<8, true, true, uint32_t, 2>));
    CAPART_ALLOW((eval_persistent_kernel<8, false, false, uint64_t, 1>));
    CAPART_ALLOW((eval_persistent_kernel<8, true, false, uint64_t, 1>));
    CAPART_ALLOW((eval_persistent_kernel<8, false, true, uint64_t, 1>));
    CAPART_ALLOW((eval_persistent_kernel<8, true, true, uint64_t, 1>));
    CAPART_ALLOW((eval_persistent_kernel<8, false, false, uint64_t, 2>));
    CAPART_ALLOW((eval_persistent_kernel<8, true, false, uint64_t, 2>));
    CAPART_ALLOW((eval_persistent_kernel<8, false, true, uint64_t, 2>));
    CAPART_ALLOW((eval_persistent_kernel<8, true, true, uint64_t, 2>));
    CAPART_ALLOW((eval_heur_kernel<4, false, false, uint32_t, 1, true>));
    CAPART_ALLOW((eval_heur_kernel<4, true, false, uint32_t, 1, true>));
    CAPART_ALLOW((eval_heur_kernel<4, false, true, uint32_t, 1, true>));
    CAPART_ALLOW((eval_heur_kernel<4, true, true, uint32_t, 1, true>));
    CAPART_ALLOW((eval_heur_kernel<4, false, false, uint64_t, 1, true>));
    CAPART_ALLOW((eval_heur_kernel<4, true, false, uint64_t, 1, true>));
    CAPART_ALLOW((eval_heur_kernel<4, false, true, uint64_t, 1, true>));
    CAPART_ALLOW((eval_heur_kernel<4, true, true, uint64_t, 1, true>));
    CAPART_ALLOW((eval_heur_kernel<8, false, false, uint32_t, 1, true>));
    CAPART_ALLOW((eval_heur_kernel<8, true, false, uint32_t, 1, true>));
    CAPART_ALLOW((eval_heur_kernel<8, false, true, uint32_t, 1, true>));
    CAPART_ALLOW((eval_heur_kernel<8, true, true, uint32_t, 1, true>));
    CAPART_ALLOW((eval_heur_kernel<8, false, false, uint64_t, 1, true>));
    CAPART_ALLOW((eval_heur_kernel<8, true, false, uint64_t, 1, true>));
    CAPART_ALLOW((eval_heur_kernel<8, false, true, uint64_t, 1, true>));
    CAPART_ALLOW((eval_heur_kernel<8, true, true, uint64_t, 1, true>));
    CAPART_ALLOW((subset_table_kernel));
    CAPART_ALLOW((final_kernel<4>));
    CAPART_ALLOW((final_kernel<8>));
    CAPART_ALLOW((triple_kernel<8>));
#undef CAPART_ALLOW
    (void)hipGetLastError();  // leave no sticky error behind for the next launch check
    return e;
}

}  // namespace capart
