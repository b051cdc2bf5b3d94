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
#pragma once
// Device code shared by the kernel translation units: every kernel template
// and device function is defined here; the host launchers that instantiate
// them live in capart_launch_*.hip (one object per policy, rank-mask width
// and part count, compiled in parallel) and capart_kernels.hip (the
// non-template kernels and the dispatch).
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

// A heuristic result's allocation rides in the key's last word: the
// allocation index of every heuristic result is 0 and each partitioning is
// evaluated once, so that word never decides a comparison.  The part of
// priority rank r sits in bits [ALLOC_BITS*r, ALLOC_BITS*r + ALLOC_BITS);
// sets with more ranks than fit replay the heuristic in the final kernel.
template <int KMAX>
struct AllocPack {
    static constexpr int BITS = KMAX <= 4 ? 2 : 3;
    static constexpr int MAX_N = 64 / BITS;
};

template <int KMAX, typename MT>
__device__ __forceinline__ uint64_t pack_alloc(int n, const MT (&S)[KMAX])
{
    if (n > AllocPack<KMAX>::MAX_N) return 0ull;
    uint64_t w = 0ull;
#pragma unroll
    for (int p = 1; p < KMAX; p++)
        for (MT h = S[p]; h; h &= h - MT(1))
            w |= (uint64_t)p << (AllocPack<KMAX>::BITS * __builtin_ctzll((uint64_t)h));
    return w;
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
// lookups).  NoTally compiles to nothing.  A tally also carries the
// per-partition policy its kernel is compiled for: POL_FP and POL_EDF fix it
// (the other policy's test is not compiled into the kernel), POL_ANY reads
// the staged set's flag.
enum : int { POL_ANY = 0, POL_FP = 1, POL_EDF = 2 };
template <int P>
struct NoTallyP {
    static constexpr int kPol = P;
    __device__ __forceinline__ void term(uint32_t) {}
    __device__ __forceinline__ void test() {}
    __device__ __forceinline__ void look() {}
};
template <int P>
struct TallyP {
    static constexpr int kPol = P;
    uint64_t terms = 0, tests = 0, looks = 0;
    __device__ __forceinline__ void term(uint32_t k) { terms += k; }
    __device__ __forceinline__ void test() { tests++; }
    __device__ __forceinline__ void look() { looks++; }
};
using NoTally = NoTallyP<POL_ANY>;
using Tally = TallyP<POL_ANY>;

// ---------------------------------------------------------------------------
// Per-set data in LDS (ranks are deadline-monotonic priority positions).
struct SetLDS {
    uint32_t T[MAXN], D[MAXN], clo[MAXN], chi[MAXN];
    uint32_t rm[MAXN], rs[MAXN];    // 32-bit multiplier and shift of T (floordiv31, response times)
    uint32_t dlo[MAXN], dhi[MAXN];  // 2^64 reciprocal of D (EDF density and demand)
    uint32_t Cs[MAXN], Cp[MAXN], k[MAXN];
    uint32_t mmin[MAXN];
    uint64_t forbid[MAXN];
    uint64_t intf[MAXN];  // ranks j with T_j < D_r: the only ones that can add a second job
    uint8_t sigma[MAXN];
    uint8_t orig[MAXN];
    uint8_t rank_of[MAXN];
    uint64_t memmask;
    uint32_t edf;  // 1: partitions are scheduled by EDF, 0: fixed-priority DM
    // bit m of lbad[k-1]: no allocation schedules a k-part partitioning whose
    // largest part has m units (stage_bounds)
    uint64_t lbad[CAPART_MAX_K][4];
};

// Whether a test compiled with tally type TY uses EDF on the staged set.
template <typename TY>
__device__ __forceinline__ bool use_edf(const SetLDS &L)
{
    if constexpr (TY::kPol == POL_FP) return false;
    else if constexpr (TY::kPol == POL_EDF) return true;
    else return L.edf != 0u;
}

// Execution-time and utilisation tables, [m-1][conflict][rank], u32:
//   tabC: time on m units; tabU: ceil(C*2^32/T) - 1.
struct Tables {
    const uint32_t *C;
    const uint32_t *U;
    int n;
};

extern __shared__ uint32_t capart_dyn_lds[];

// Per-set records (by priority rank) and interference masks into LDS.
__device__ void stage_records(SetLDS &L, const Work &w, int64_t off, int n, int64_t s, bool act)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int i = tid; i < n; i += nt) {
        TaskRec t = w.rec[off + i];
        L.T[i] = t.T; L.D[i] = t.D; L.clo[i] = t.clo; L.chi[i] = t.chi;
        uint32_t rm, rs;
        magic31_of(t.T, t.clo, t.chi, &rm, &rs);
        L.rm[i] = rm; L.rs[i] = rs;
        L.Cs[i] = t.Cs; L.Cp[i] = t.Cp; L.k[i] = t.k;
        L.mmin[i] = t.mmin;
        L.orig[i] = t.orig;
        L.rank_of[t.orig] = (uint8_t)i;
        L.sigma[i] = w.sigma[off + i];
        L.forbid[i] = act ? w.forbid[off + i] : 0ull;
    }
    if (tid == 0) {
        L.memmask = w.memmask[s];
        L.edf = (w.setflags[s] & SETF_EDF) ? 1u : 0u;
    }
    __syncthreads();
    for (int r = tid; r < n; r += nt) {
        uint64_t f = 0ull;
        for (int j = 0; j < n; j++) f |= (uint64_t)(L.T[j] < L.D[r]) << j;
        L.intf[r] = f;
        if (L.edf) magic_u32(L.D[r], &L.dlo[r], &L.dhi[r]);  // the EDF test divides by D
    }
}

// Times of rank r on m units, without and in conflict: the batch's explicit
// tables (read by the task's index in its set), or the parametric model.
__device__ __forceinline__ void exec_times(const SetLDS &L, const Work &w, int64_t s, int M, int r, int m,
                                           uint32_t &cn, uint32_t &cc)
{
    if (w.tCn) {
        const int64_t at = w.toff[s] + (int64_t)L.orig[r] * M + (m - 1);
        cn = (uint32_t)w.tCn[at];
        cc = (uint32_t)w.tCc[at];
    } else {
        cn = time_n(L.Cs[r], L.Cp[r], (uint32_t)m);
        cc = time_c(L.k[r], cn);
    }
}

// Records plus the whole [m][conflict][rank] tables of execution times and
// Q32 utilisations (m = 1..M).
__device__ void stage_set(SetLDS &L, const Work &w, int64_t off, int n, int M, int64_t s, bool act, Tables &tb)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    stage_records(L, w, off, n, s, act);
    uint32_t *tc = capart_dyn_lds;
    uint32_t *tu = capart_dyn_lds + 2 * n * M;
    for (int e = tid; e < n * M; e += nt) {
        const int m = e / n + 1, r = e - (m - 1) * n;
        uint32_t cn, cc;
        exec_times(L, w, s, M, r, m, cn, cc);
        const int base = (m - 1) * 2 * n + r;
        tc[base] = cn;
        tc[base + n] = cc;
        tu[base] = util_q32_m1_magic(cn, L.T[r], L.clo[r], L.chi[r]);
        tu[base + n] = util_q32_m1_magic(cc, L.T[r], L.clo[r], L.chi[r]);
    }
    __syncthreads();
    tb.C = tc;
    tb.U = tu;
    tb.n = n;
}

// Records plus the execution-time table [m-1][conflict][rank] (u32, m = 1..M)
__device__ void stage_set_times(SetLDS &L, const Work &w, int64_t off, int n, int M, int64_t s, bool act,
                                Tables &tb)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    stage_records(L, w, off, n, s, act);
    uint32_t *tc = capart_dyn_lds;
    for (int e = tid; e < n * M; e += nt) {
        const int m = e / n + 1, r = e - (m - 1) * n;
        uint32_t cn, cc;
        exec_times(L, w, s, M, r, m, cn, cc);
        const int base = (m - 1) * 2 * n + r;
        tc[base] = cn;
        tc[base + n] = cc;
    }
    __syncthreads();
    tb.C = tc;
    tb.U = nullptr;
    tb.n = n;
}

// ceil(C 2^32 / T) of rank r on m units where C <= T, else 2^32 + 1 (any
// C > T has C 2^32 / T above 2^32): at least the exact Q32 utilisation minus 1.
__device__ __forceinline__ uint64_t util_ceil_bound(const SetLDS &L, const Tables &tb, int r, int m, uint32_t conf)
{
    const int at = (m - 1) * 2 * tb.n + (int)conf * tb.n + r;
    const uint32_t C = tb.C[at], T = L.T[r];
    if (C > T) return (1ull << 32) + 1ull;
    const uint32_t u = tb.U ? tb.U[at] : util_q32_m1_magic(C, T, L.clo[r], L.chi[r]);
    return (uint64_t)u + 1ull;
}

// Partitionings that no allocation can schedule, from a necessary condition
// (so skipping them changes no result): a schedulable partition has
// utilisation at most 1, so the k parts together carry at most k; a task on a
// part of m_p <= m_1 units needs at least its utilisation on m_1 units (times
// never grow with more units); and at most one task of each type per part is
// free of conflict (a conflict needs two of a type), so at most k of each
// type take their time without conflict.  Hence a k-part partitioning whose
// largest part has m_1 units is infeasible when
//   sum_i uc_i(m_1) - (k largest uc_i - un_i of memory tasks)
//                   - (k largest uc_i - un_i of compute tasks)  >  k,
// with uc, un the utilisations in and out of conflict, taken as Q32 ceilings
// (each at most 1 above 2^32 times the exact value, hence the n below).
// One thread per m fills bit m of lbad[k-1] for k = 1..KMAX.
template <int KMAX>
__device__ void stage_bounds(SetLDS &L, const Tables &tb, int n, int M)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int i = tid; i < KMAX * 4; i += nt) L.lbad[i >> 2][i & 3] = 0ull;
    __syncthreads();
    for (int m = tid + 1; m <= M; m += nt) {
        uint64_t sum = 0, tm[KMAX], tcp[KMAX];
#pragma unroll
        for (int i = 0; i < KMAX; i++) { tm[i] = 0ull; tcp[i] = 0ull; }
        for (int r = 0; r < n; r++) {
            const uint64_t un = util_ceil_bound(L, tb, r, m, 0u), uc = util_ceil_bound(L, tb, r, m, 1u);
            sum += uc;
            uint64_t v = uc > un ? uc - un : 0ull;
            if ((L.memmask >> r) & 1ull) {
#pragma unroll
                for (int i = 0; i < KMAX; i++)
                    if (v > tm[i]) { const uint64_t t = tm[i]; tm[i] = v; v = t; }
            } else {
#pragma unroll
                for (int i = 0; i < KMAX; i++)
                    if (v > tcp[i]) { const uint64_t t = tcp[i]; tcp[i] = v; v = t; }
            }
        }
        uint64_t cut = 0;
#pragma unroll
        for (int k = 1; k <= KMAX; k++) {
            cut += tm[k - 1] + tcp[k - 1];
            if (sum - cut >= (uint64_t)n + ((uint64_t)k << 32))
                atomicOr((unsigned long long *)&L.lbad[k - 1][m >> 6], (unsigned long long)(1ull << (m & 63)));
        }
    }
    __syncthreads();
}

// Q32 utilisation ceil(C 2^32 / T) of rank r on m units, exact modulo 2^64
// also where C > T (an unschedulable group): only a table entry saturated at
// C_SAT (a parametric conflict time of 2^31 or more) is recomputed in 64 bits.
__device__ __forceinline__ uint64_t util_term(const SetLDS &L, const Tables &tb, int r, int m, uint32_t conf)
{
    const uint32_t C = tb.C[(m - 1) * 2 * tb.n + (int)conf * tb.n + r];
    const uint32_t T = L.T[r];
    if (C <= T) return (uint64_t)util_q32_m1_magic(C, T, L.clo[r], L.chi[r]) + 1ull;
    const uint64_t T64 = T;
    uint64_t C64 = C;
    if (C >= C_SAT) {
        const uint64_t cn = (uint64_t)L.Cs[r] + ((uint64_t)L.Cp[r] + (uint64_t)m - 1ull) / (uint64_t)m;
        C64 = conf ? ((uint64_t)L.k[r] * cn + 999ull) / 1000ull : cn;
    }
    return ((C64 / T64) << 32) + ((((C64 % T64) << 32) + T64 - 1ull) / T64);
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

// Least fixed point of R = base + sum_{j in hp} floor((R-1)/T_j) C_j, where
// base = C_r + sum C_j over every higher-priority member is the demand with
// one job of each (so the sum equals C_r + sum ceil(R/T_j) C_j), and hp holds
// only members with T_j < D_r (the others never release a second job before
// D_r).  The iteration starts at `start`, a lower bound of the fixed point
// that is at least base (base itself, or the response time of the next
// higher-priority member plus C_r: the level-r demand exceeds every t below
// that bound, since the higher level's demand exceeds every t below its own
// response time).  Returns R, or 0 once R exceeds D.
template <typename MT, typename TY>
__device__ __forceinline__ uint32_t rta_fp(const SetLDS &L, const uint32_t *row, int n, uint64_t base,
                                           uint64_t start, uint32_t D, MT hp, MT cm, TY &ty)
{
    if (base > D) return 0u;
    if (!hp) return (uint32_t)base;
    if (start > D) return 0u;
    uint64_t R = start;
    // members out of conflict read the first row, the others the second
    const MT hpn = hp & ~cm, hpc = hp & cm;
    const uint32_t *rowc = row + n;
    while (hp) {
        ty.term(1u + (uint32_t)mpopc(hp));
        const uint32_t x2 = ((uint32_t)R - 1u) << 1;  // R <= D < 2^31
        uint64_t W = base;
        for (MT h = hpn; h; h &= h - MT(1)) {
            const int j = mctz(h);
            W += (uint64_t)floordiv31(x2, L.rm[j], L.rs[j]) * row[j];
        }
        for (MT h = hpc; h; h &= h - MT(1)) {
            const int j = mctz(h);
            W += (uint64_t)floordiv31(x2, L.rm[j], L.rs[j]) * rowc[j];
        }
        if (W > D) return 0u;
        if (W == R) break;
        R = W;
    }
    return (uint32_t)R;
}

// EDF on one partition (Section "Schedulability test" admits any policy with
// an exact test): the processor-demand criterion (Baruah, Rosier and Howell
// 1990) for constrained deadlines, walked with Zhang and Burns' quick
// processor-demand analysis (QPA, 2009).  Integer definition, in order:
//   1. floor-Q32 utilisation above 2^32: unschedulable (U > 1);
//   2. ceil-Q32 density sum ceil(C 2^32 / D) at most 2^32: schedulable
//      (density at most 1 is sufficient for EDF);
//   3. horizon H = the synchronous busy period L (least fixed point of
//      w = sum ceil(w/T_j) C_j, iterated from sum C_j) if the iteration settles
//      within EDF_BP_STEPS steps, else the bound ceil(sum C 2^32 / (2^32 - Uq))
//      >= L with the ceil-Q32 utilisation Uq, else (Uq >= 2^32) undetermined;
//   4. H determined with at most EDF_ND_CAP absolute deadlines below it:
//      schedulable iff h(d) <= d at every absolute deadline d < H, with
//      h(t) = sum_{D_j <= t} (floor((t - D_j)/T_j) + 1) C_j;
//   5. otherwise (a work limit reached): schedulable iff every member passes
//      the fixed-priority deadline-monotonic response-time test, which is
//      sufficient for EDF (members are walked in rank order, which is DM order).
// Step 4 walks t down from the last deadline below H: to h(t) while h(t) < t,
// else to the previous deadline, until h(t) <= min D (schedulable) or h(t) > t
// (a miss).  h is a non-decreasing step function that changes only at
// deadlines, so every skipped deadline d has h(d) <= d, and the walk moves
// below at least one deadline every two points: at most 2 ND + 1 points.
// get(j, C, T, D) reads member j.  Returns ok, H (0 where undetermined or not
// wanted; when ok every job of the partition completes by min(D_i, H); where
// step 2 decided, a value at or above the largest D stands for any H that
// large, since only min(D_i, H) is reported) and
// the terms evaluated (members x busy-period steps, demand points and DM
// fixed-point steps).  64-bit bounds: C < 2^31 and T, D < 2^31; w < 2^50 over
// the busy-period steps (U < 1 + 2^-26); H < 2^57 (a larger bound puts more
// than 2^25 deadlines below it, so H is not needed: step 5 decides).
// Kept out of line (one call on the EDF side of each test) so that the
// runtime-policy kernels keep most of their registers.
constexpr int EDF_BP_STEPS = 4096;
constexpr uint64_t EDF_ND_CAP = 65536;

struct EdfRes {
    uint64_t H;
    uint32_t terms;
    bool ok;
};

// Member j's record as an EDF test reads it: C, T, D and the 2^64
// reciprocals of T and D (magic_u32), which replace 64-bit divisions by
// multiplies wherever the dividend fits 32 bits.
struct EdfTask {
    uint32_t C, T, D, tlo, thi, dlo, dhi;
};

// ceil(w / T) for w < 2^32 by the reciprocal, else by a 64-bit division.
__device__ __forceinline__ uint64_t ceil_div_t(uint64_t w, const EdfTask &e)
{
    if (w == 0ull) return 0ull;
    if (w <= 0xFFFFFFFFull) return (uint64_t)udiv_magic((uint32_t)(w - 1ull), e.T, e.tlo, e.thi) + 1ull;
    return (w + e.T - 1ull) / e.T;
}

// floor(x / T) likewise.
__device__ __forceinline__ uint64_t floor_div_t(uint64_t x, const EdfTask &e)
{
    if (x <= 0xFFFFFFFFull) return (uint64_t)udiv_magic((uint32_t)x, e.T, e.tlo, e.thi);
    return x / e.T;
}

template <typename MT, typename GET>
__device__ __noinline__ EdfRes edf_demand(MT S, GET get, bool need_h)
{
    constexpr uint64_t ONE = 1ull << 32;
    const uint32_t cnt = (uint32_t)mpopc(S);
    EdfRes res{0ull, 0u, false};
    uint64_t uf = 0, uc = 0, dc = 0, sumC = 0;
    bool dense = false;  // some C_j / D_j above 1
    uint32_t dmin = 0xFFFFFFFFu, dmax = 0u;
    for (MT h = S; h; h &= h - MT(1)) {
        const EdfTask e = get(mctz(h));
        if (e.C > e.T) return res;  // C/T > 1: U > 1
        uint64_t fl, cl;
        q32_floor_ceil(e.C, e.T, e.tlo, e.thi, &fl, &cl);
        uf += fl;
        if (uf > ONE) return res;
        uc += cl;
        if (e.C > e.D) {
            dense = true;
        } else if (e.D == e.T) {
            dc += cl;
        } else {
            uint64_t dfl, dcl;
            q32_floor_ceil(e.C, e.D, e.dlo, e.dhi, &dfl, &dcl);
            dc += dcl;
        }
        sumC += e.C;
        dmin = min(dmin, e.D);
        dmax = max(dmax, e.D);
    }
    res.terms += cnt;
    const bool density_ok = !dense && dc <= ONE;
    if (density_ok && !need_h) {
        res.ok = true;
        return res;
    }
    uint64_t w = sumC, H = 0;
    bool settled = false;
    // with the verdict decided by the density bound, H is wanted only for the
    // members' min(D_i, H): the iterates rise to H, so once one reaches the
    // largest D it stands in for H (every min is then D_i)
    const uint64_t wcap = density_ok ? (uint64_t)dmax : ~0ull;
    for (int step = 0; step < EDF_BP_STEPS; step++) {
        if (w >= wcap) { settled = true; break; }
        uint64_t W = 0;
        for (MT h = S; h; h &= h - MT(1)) {
            const EdfTask e = get(mctz(h));
            W += ceil_div_t(w, e) * e.C;
        }
        res.terms += cnt;
        if (W == w) { settled = true; break; }
        w = W;
    }
    if (settled) {
        H = w;
    } else if (uc < ONE) {
        const uint64_t den = ONE - uc, a = sumC / den, r = sumC % den;
        if (a < (1ull << 24)) H = (a << 32) + (((r << 32) + den - 1ull) / den);
    }
    res.H = H;
    if (density_ok) {
        res.ok = true;
        return res;
    }
    uint64_t nd = EDF_ND_CAP + 1ull;
    if (H != 0ull) {
        nd = 0;
        for (MT h = S; h; h &= h - MT(1)) {
            const EdfTask e = get(mctz(h));
            if (e.D < H) nd += floor_div_t(H - 1ull - e.D, e) + 1ull;
        }
    }
    if (nd > EDF_ND_CAP) {
        // step 5: deadline-monotonic response times, members in rank order
        for (MT rem = S; rem; rem &= rem - MT(1)) {
            const int r = mctz(rem);
            const EdfTask er = get(r);
            const MT hp = S & below<MT>(r);
            uint64_t R = er.C;
            for (MT h = hp; h; h &= h - MT(1)) R += get(mctz(h)).C;
            if (R > er.D) return res;
            for (;;) {
                uint64_t W = er.C;
                for (MT h = hp; h; h &= h - MT(1)) {
                    const EdfTask e = get(mctz(h));
                    W += ceil_div_t(R, e) * e.C;  // R <= D < 2^31
                    if (W > er.D) return res;
                }
                res.terms += 1u + (uint32_t)mpopc(hp);
                if (W == R) break;
                R = W;
            }
        }
        res.ok = true;
        return res;
    }
    if (H <= dmin) {
        res.ok = true;
        return res;
    }
    auto demand = [&](uint64_t t) {
        uint64_t d = 0;
        for (MT h = S; h; h &= h - MT(1)) {
            const EdfTask e = get(mctz(h));
            if (e.D <= t) d += (floor_div_t(t - e.D, e) + 1ull) * e.C;
        }
        return d;
    };
    auto last_before = [&](uint64_t t) {  // largest absolute deadline < t (t > min D)
        uint64_t d = 0;
        for (MT h = S; h; h &= h - MT(1)) {
            const EdfTask e = get(mctz(h));
            if (e.D < t) d = max(d, (uint64_t)e.D + floor_div_t(t - 1ull - e.D, e) * e.T);
        }
        return d;
    };
    uint64_t t = last_before(H);
    for (uint64_t it = 0; it < 2 * EDF_ND_CAP + 4; it++) {
        const uint64_t hd = demand(t);
        res.terms += cnt;
        if (hd > t) return res;
        if (hd <= dmin) {
            res.ok = true;
            return res;
        }
        t = hd < t ? hd : last_before(t);
    }
    return res;  // not reached (at most 2 ND + 1 points)
}

// EDF test of rank set S on m units (conflict mask cm) from the staged tables.
template <typename MT, typename TY>
__device__ __forceinline__ bool edf_part(const SetLDS &L, const Tables &tb, MT S, int m, MT cm, TY &ty,
                                         uint64_t *Hout)
{
    const int n = tb.n;
    const uint32_t *row = tb.C + (m - 1) * 2 * n;
    const SetLDS *Ls = &L;
    auto get = [=](int j) {
        return EdfTask{row[(int)mbit(cm, j) * n + j], Ls->T[j], Ls->D[j], Ls->clo[j], Ls->chi[j], Ls->dlo[j],
                       Ls->dhi[j]};
    };
    const EdfRes r = edf_demand<MT>(S, get, Hout != nullptr);
    ty.term(r.terms);
    if (Hout) *Hout = r.H;
    return r.ok;
}

// Test the members of S with rank >= first on one partition of m units,
// taking the members below `first` as already schedulable (their response
// times cannot change).  cm = conflict mask of S.
template <typename MT, typename TY>
__device__ bool test_from(const SetLDS &L, const Tables &tb, MT S, int first, int m, MT cm, TY &ty)
{
    ty.test();
    if (use_edf<TY>(L)) return edf_part<MT>(L, tb, S, m, cm, ty, nullptr);  // whole-set test
    const int n = tb.n;
    const uint32_t *row = tb.C + (m - 1) * 2 * n;
    uint64_t sumC = 0;
    bool sat = false;  // some higher-priority task has utilisation >= 1
    const MT above = S & below<MT>(first);
    for (MT h = above & ~cm; h; h &= h - MT(1)) {  // out of conflict: first row
        const int j = mctz(h);
        const uint32_t Cj = row[j];
        sumC += Cj;
        sat |= (Cj >= L.T[j]);
    }
    for (MT h = above & cm; h; h &= h - MT(1)) {  // in conflict: second row
        const int j = mctz(h);
        const uint32_t Cj = row[n + j];
        sumC += Cj;
        sat |= (Cj >= L.T[j]);
    }
    uint64_t Rprev = 0;  // response time of the member tested before (0: none yet)
    for (MT rem = S & ~below<MT>(first); rem; rem &= rem - MT(1)) {
        const int r = mctz(rem);
        const uint32_t Cr = row[(int)mbit(cm, r) * n + r];
        if (sat) return false;
        const MT hp = S & below<MT>(r) & (MT)L.intf[r];
        const uint64_t base = sumC + Cr;
        const uint32_t R = rta_fp<MT>(L, row, n, base, max(base, Rprev + Cr), L.D[r], hp, cm, ty);
        if (!R) return false;
        Rprev = R;
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
    return rta_fp<MT>(L, row, n, base, base, L.D[r], hp & (MT)L.intf[r], cm, nt);
}

// Reported response time of rank r in partition Sp (m units, conflict mask
// cm), 0 on a miss: the response-time fixed point under fixed priority; under
// EDF min(D_r, H) for a schedulable partition (H bounds every busy period),
// D_r where H is undetermined.
template <typename MT, typename TY = NoTally>
__device__ uint32_t resp_one(const SetLDS &L, const Tables &tb, int m, int r, MT Sp, MT cm)
{
    if (use_edf<TY>(L)) {
        NoTally nt;
        uint64_t H = 0;
        if (!edf_part<MT>(L, tb, Sp, m, cm, nt, &H)) return 0u;
        return H ? (uint32_t)min(H, (uint64_t)L.D[r]) : L.D[r];
    }
    return rta_one<MT>(L, tb, m, r, Sp & below<MT>(r), cm);
}

template <int KMAX, typename V>
__device__ __forceinline__ V pick(const V (&a)[KMAX], int p)
{
    V v = a[0];
#pragma unroll
    for (int i = 1; i < KMAX; i++) v = (p == i) ? a[i] : v;
    return v;
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

// ---------------------------------------------------------------------------
// Test memo of one staged set (sets between the frontier limit and 32
// tasks): an open-addressing hash table in LDS whose entry for a rank subset S
// records the largest size known to fail (f, 0 = none) and the smallest size
// known to pass (p, 256 = none); by monotonicity in m, S passes on m >= p and
// fails on m <= f.  Across the partitionings of a set the heuristic repeats
// the same subsets many times.  Entries only ever gain exact facts (f grows,
// p shrinks, by compare-and-swap), so lanes that race at worst repeat a test.
// Entry: S in bits 0..31, f in 32..40, p in 41..49 (0 = empty; S is never
// empty).  Larger sets are left to direct tests: the costly ones (schedulable
// on many partitionings) meet so many distinct subsets that a table in LDS
// answers few of their tests.
constexpr int MEMO_PROBES = 8;

struct Memo {
    unsigned long long *tab;
    uint32_t mask;  // entries - 1 (0 = no memo)
};

__device__ __forceinline__ uint32_t memo_hash(uint32_t S, uint32_t mask) { return (S * 0x9E3779B1u >> 7) & mask; }

// f and p of S (0 and 256 when unknown)
__device__ __forceinline__ void memo_get(const Memo &mo, uint32_t S, int &f, int &p)
{
    f = 0;
    p = 256;
    uint32_t h = memo_hash(S, mo.mask);
    for (int i = 0; i < MEMO_PROBES; i++, h = (h + 1u) & mo.mask) {
        const unsigned long long v = mo.tab[h];
        if (v == 0ull) return;
        if ((uint32_t)v == S) {
            f = (int)((v >> 32) & 0x1FFu);
            p = (int)((v >> 41) & 0x1FFu);
            return;
        }
    }
}

// record that S passes (ok) or fails on m units
__device__ __forceinline__ void memo_put(const Memo &mo, uint32_t S, int m, bool ok)
{
    uint32_t h = memo_hash(S, mo.mask);
    for (int i = 0; i < MEMO_PROBES; i++, h = (h + 1u) & mo.mask) {
        unsigned long long v = mo.tab[h];
        if (v == 0ull) {
            const unsigned long long nv = (unsigned long long)S | ((unsigned long long)(ok ? 0 : m) << 32) |
                                          ((unsigned long long)(ok ? m : 256) << 41);
            const unsigned long long old = atomicCAS(&mo.tab[h], 0ull, nv);
            if (old == 0ull) return;
            v = old;
        }
        if ((uint32_t)v != S) continue;
        for (;;) {
            int f = (int)((v >> 32) & 0x1FFu), p = (int)((v >> 41) & 0x1FFu);
            if (ok) p = min(p, m); else f = max(f, m);
            const unsigned long long nv = (unsigned long long)S | ((unsigned long long)f << 32) |
                                          ((unsigned long long)p << 41);
            if (nv == v) return;
            const unsigned long long old = atomicCAS(&mo.tab[h], v, nv);
            if (old == v) return;
            v = old;
        }
    }
}

// min_units with the test memo: the search starts above the largest size
// known to fail (f) and below the smallest known to pass (hi), and records
// every size it tests.
template <typename MT, typename TY>
__device__ int min_units_memo(const SetLDS &L, const Tables &tb, MT S, int f, int hi, const Memo &mo, TY &ty)
{
    int lo = f + 1;
    for (MT h = S; h; h &= h - MT(1)) lo = max(lo, (int)L.mmin[mctz(h)]);
    const MT cm = conflict_mask<MT>(S, (MT)L.memmask);
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const bool ok = test_from<MT>(L, tb, S, 0, mid, cm, ty);
        memo_put(mo, (uint32_t)S, mid, ok);
        if (ok)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// Heuristic allocation on a fixed partitioning m[0..k) (non-increasing):
// tasks in decreasing one-unit utilisation, each to the best-ranked part that
// stays schedulable.  S[p] = rank masks, U[p] = Q32 utilisations.
template <int KMAX, bool ACT, bool SMS, typename MT, typename TY>
__device__ __forceinline__ bool heuristic(const SetLDS &L, const Tables &tb, int n, const int (&m)[KMAX], int k,
                                          MT (&S)[KMAX], uint64_t (&U)[KMAX], TY &ty, const Memo &mo = Memo{nullptr, 0u})
{
    int lbm[KMAX];  // per part, the largest Lemma 2 size of its members (SMS: a floor on the fewest units)
#pragma unroll
    for (int p = 0; p < KMAX; p++) { S[p] = MT(0); U[p] = 0ull; lbm[p] = 0; }
    // Capacity stop: every part of a schedulable partitioning has utilisation at
    // most 1, a placed task never gets cheaper (members only gain conflicts),
    // and an unplaced task needs at least its conflict-free utilisation on the
    // largest part.  Once that need exceeds the room the parts can still have,
    // no placement of the rest can succeed, so the heuristic, which only makes
    // schedulable placements, must fail: it stops there (same outcome).
    // Q32: table terms are ceil(u 2^32) - 1 <= u 2^32 for the need, and the
    // parts' sums exceed the exact utilisation by less than one per member.
    const uint32_t *urow1 = tb.U + (m[0] - 1) * 2 * n;
    uint64_t need = 0;
    for (int i = 0; i < n; i++) need += (uint64_t)urow1[i];
    uint64_t room = (uint64_t)k << 32;  // k 2^32 - sum U + (members placed)
    for (int t = 0; t < n; t++) {
        if (need > room) return false;
        const int r = L.sigma[t];
        const int mm = (int)L.mmin[r];
        const MT fb = ACT ? (MT)L.forbid[r] : MT(0);
        int best = -1, bestReq = 0;
        uint64_t bestU = 0;
        // the candidate test of part (Sp, mp): through the memo where the set has
        // one (a recorded fact, else the incremental test, recorded), else direct
        auto passes = [&](MT Sp, int mp, uint64_t Up, int &f, int &pz) -> bool {
            uint64_t Un;
            f = 0;
            pz = 256;
            if (sizeof(MT) == 4 && mo.mask) {
                const MT Sn = Sp | (MT(1) << r);
                ty.look();
                memo_get(mo, (uint32_t)Sn, f, pz);
                bool ok = mp >= pz;
                if (!ok && mp > f) {
                    ok = part_test_add<MT>(L, tb, Sp, r, mp, Up, &Un, ty);
                    memo_put(mo, (uint32_t)Sn, mp, ok);
                    if (ok) pz = mp;
                }
                return ok;
            }
            return part_test_add<MT>(L, tb, Sp, r, mp, Up, &Un, ty);
        };
        if (!SMS) {
            // ">": the part taken is the passing one of least (utilisation with the
            // task, index).  The utilisations are known from the tables before any
            // test, so the candidates are tested in that order and the first that
            // passes is taken; the others need no test.  (Parts are selected with
            // compile-time indices so that S, U and m stay in registers.)
            uint64_t un[KMAX];
            uint32_t cand = 0u;
#pragma unroll
            for (int p = 0; p < KMAX; p++) {
                un[p] = 0ull;
                if (p >= k || mm > m[p] || (ACT && (fb & S[p]))) continue;
                un[p] = util_add<MT>(L, tb, S[p], r, m[p], U[p]);
                cand |= 1u << p;
            }
            while (cand) {
                int q = -1, mq = 0;
                uint64_t uq = 0ull, Uq = 0ull;
                MT Sq = MT(0);
#pragma unroll
                for (int p = 0; p < KMAX; p++)
                    if (((cand >> p) & 1u) && (q < 0 || un[p] < uq)) { q = p; uq = un[p]; Sq = S[p]; mq = m[p]; Uq = U[p]; }
                cand &= ~(1u << q);
                // utilisation above 1 (the Q32 terms less one each bound it from
                // below) cannot be scheduled: no test
                if (uq - (uint64_t)(mpopc(Sq) + 1) > (1ull << 32)) continue;
                int f, pz;
                if (passes(Sq, mq, Uq, f, pz)) { best = q; bestU = uq; break; }
            }
        } else {
            // ">>": the part taken is the passing one of least (fewest units,
            // utilisation with the task, index).  The fewest units are at least
            // lb, the largest Lemma 2 size of the part's members and the task, so
            // the candidates are visited in order of (lb, utilisation, index) and
            // the visit stops at the first that cannot beat the best found; once
            // there is a best, a candidate's fewest units only matter up to the
            // best's, so its test is at that size and its search below it.
            uint64_t un[KMAX];
            int lbp[KMAX];
            uint32_t cand = 0u;
#pragma unroll
            for (int p = 0; p < KMAX; p++) {
                un[p] = 0ull;
                lbp[p] = 0;
                if (p >= k || mm > m[p] || (ACT && (fb & S[p]))) continue;
                un[p] = util_add<MT>(L, tb, S[p], r, m[p], U[p]);
                lbp[p] = max(lbm[p], mm);
                cand |= 1u << p;
            }
            while (cand) {
                int q = -1, mq = 0, lq = 0;
                uint64_t uq = 0ull, Uq = 0ull;
                MT Sq = MT(0);
#pragma unroll
                for (int p = 0; p < KMAX; p++)
                    if (((cand >> p) & 1u) && (q < 0 || lbp[p] < lq || (lbp[p] == lq && un[p] < uq))) {
                        q = p; lq = lbp[p]; uq = un[p]; Sq = S[p]; mq = m[p]; Uq = U[p];
                    }
                cand &= ~(1u << q);
                if (best >= 0 && (lq > bestReq || (lq == bestReq && (uq > bestU || (uq == bestU && q > best))))) break;
                if (uq - (uint64_t)(mpopc(Sq) + 1) > (1ull << 32)) continue;  // utilisation above 1 on m[q]
                const MT Sn = Sq | (MT(1) << r);
                const MT cm = conflict_mask<MT>(Sn, (MT)L.memmask);
                int f = 0, pz = 256;  // largest size known to fail, smallest known to pass
                if (sizeof(MT) == 4 && mo.mask) {
                    ty.look();
                    memo_get(mo, (uint32_t)Sn, f, pz);
                }
                auto test_at = [&](int msz) -> bool {  // the whole union at msz units
                    if (msz <= f) return false;
                    if (msz >= pz) return true;
                    const bool ok = test_from<MT>(L, tb, Sn, 0, msz, cm, ty);
                    if (sizeof(MT) == 4 && mo.mask) memo_put(mo, (uint32_t)Sn, msz, ok);
                    if (ok) pz = msz; else f = msz;
                    return ok;
                };
                int hi = mq;
                if (best >= 0 && bestReq < mq) {
                    if (!test_at(bestReq)) continue;  // needs more units than the best (or does not fit)
                    hi = bestReq;
                } else {
                    // the part's own test at its size: the incremental test
                    bool ok = mq >= pz;
                    if (!ok && mq > f) {
                        uint64_t Un2;
                        ok = part_test_add<MT>(L, tb, Sq, r, mq, Uq, &Un2, ty);
                        if (sizeof(MT) == 4 && mo.mask) memo_put(mo, (uint32_t)Sn, mq, ok);
                        if (ok) pz = mq; else f = mq;
                    }
                    if (!ok) continue;
                }
                // the fewest units: the least passing size in [max(lb, f + 1), hi]
                int lo = max(lq, f + 1);
                hi = min(hi, pz);
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (test_at(mid))
                        hi = mid;
                    else
                        lo = mid + 1;
                }
                const int req = lo;
                if (best < 0 || req < bestReq || (req == bestReq && (uq < bestU || (uq == bestU && q < best)))) {
                    best = q;
                    bestU = uq;
                    bestReq = req;
                }
            }
        }
        if (best < 0) return false;
        uint64_t Uold = 0;
#pragma unroll
        for (int p = 0; p < KMAX; p++)
            if (p == best) { Uold = U[p]; S[p] |= MT(1) << r; U[p] = bestU; lbm[p] = max(lbm[p], mm); }
        need -= (uint64_t)urow1[r];
        room = room + 1ull - (bestU - Uold);
    }
    return true;
}

// The same test as test_from with one lane per member (lane j tests rank j;
// all 64 lanes call it with the same arguments): the critical path is one
// response-time fixed point instead of all of them.  Wave-uniform result.
template <typename TY>
__device__ bool wave_test_from(const SetLDS &L, const Tables &tb, uint64_t S, int first, int m, uint64_t cm, TY &ty)
{
    const int lane = threadIdx.x & 63;
    const int n = tb.n;
    if (use_edf<TY>(L)) {  // whole-set test, the same in every lane, tallied once
        Tally one;
        const bool ok = edf_part<uint64_t>(L, tb, S, m, cm, one, nullptr);
        if (lane == 0) {
            ty.test();
            ty.term((uint32_t)one.terms);
        }
        return ok;
    }
    bool fail = false;
    if (((S >> lane) & 1ull) && lane >= first) {
        const uint32_t *row = tb.C + (m - 1) * 2 * n;
        const uint64_t hp = S & ((1ull << lane) - 1ull);
        uint64_t base = row[(int)((cm >> lane) & 1ull) * n + lane];
        bool sat = false;  // some higher-priority member has utilisation >= 1
        for (uint64_t h = hp; h; h &= h - 1ull) {
            const int j = __builtin_ctzll(h);
            const uint32_t Cj = row[(int)((cm >> j) & 1ull) * n + j];
            base += Cj;
            sat |= (Cj >= L.T[j]);
        }
        fail = sat || rta_fp<uint64_t>(L, row, n, base, base, L.D[lane], hp & L.intf[lane], cm, ty) == 0u;
    }
    if (lane == 0) ty.test();
    return !__any(fail);
}

// heuristic() for one partitioning with the whole wave: the same decisions
// (tasks in the heuristic order, parts in index order, the same ranks and
// tie-breaks), each candidate test spread over the part's members.  S, U, m
// and k are wave-uniform.
template <int KMAX, bool ACT, bool SMS, typename TY>
__device__ bool wave_heuristic(const SetLDS &L, const Tables &tb, int n, const int (&m)[KMAX], int k,
                               uint64_t (&S)[KMAX], uint64_t (&U)[KMAX], TY &ty)
{
    const uint64_t memm = L.memmask;
    int lbm[KMAX];  // per part, the largest Lemma 2 size of its members
#pragma unroll
    for (int p = 0; p < KMAX; p++) { S[p] = 0ull; U[p] = 0ull; lbm[p] = 0; }
    // the capacity stop of heuristic(): lane i holds task i's conflict-free
    // utilisation on the largest part, less one (a lower bound in Q32)
    const int lane = threadIdx.x & 63;
    const uint64_t li = lane < n ? util_term(L, tb, lane, m[0], 0u) - 1ull : 0ull;
    uint64_t need = li;
#pragma unroll
    for (int o2 = 32; o2 >= 1; o2 >>= 1) need += __shfl_xor(need, o2, 64);
    uint64_t room = (uint64_t)k << 32;
    for (int t = 0; t < n; t++) {
        if (need > room) return false;
        const int r = L.sigma[t];
        const int mm = (int)L.mmin[r];
        const uint64_t fb = ACT ? L.forbid[r] : 0ull;
        const uint64_t typ = ((memm >> r) & 1ull) ? memm : ~memm;
        int best = -1, bestReq = 0;
        uint64_t bestU = 0;
        // part p's union with the task: its mask, conflict mask, first member
        // whose response time can change, and utilisation
        auto cand_of = [&](uint64_t Sp, int mp, uint64_t Up, uint64_t &Sn, uint64_t &cm, int &first) -> uint64_t {
            Sn = Sp | (1ull << r);
            const uint64_t same = Sp & typ;
            const int ns = __popcll(same);
            cm = conflict_mask<uint64_t>(Sn, memm);
            first = r;
            uint64_t Un = Up + util_term(L, tb, r, mp, ns >= 1 ? 1u : 0u);
            if (ns == 1) {
                const int flip = __builtin_ctzll(same);
                first = min(first, flip);
                Un += util_term(L, tb, flip, mp, 1u) - util_term(L, tb, flip, mp, 0u);
            }
            return Un;
        };
        if (!SMS) {
            // ">": candidates tested in order of (utilisation with the task,
            // index), the first that passes taken (as in heuristic())
            uint64_t un[KMAX];
            uint32_t cand = 0u;
#pragma unroll
            for (int p = 0; p < KMAX; p++) {
                un[p] = 0ull;
                if (p >= k || mm > m[p] || (ACT && (fb & S[p]))) continue;
                uint64_t Sn, cm;
                int first;
                un[p] = cand_of(S[p], m[p], U[p], Sn, cm, first);
                cand |= 1u << p;
            }
            while (cand) {
                int q = -1, mq = 0;
                uint64_t uq = 0ull, Sq = 0ull, Uq = 0ull;
#pragma unroll
                for (int p = 0; p < KMAX; p++)
                    if (((cand >> p) & 1u) && (q < 0 || un[p] < uq)) { q = p; uq = un[p]; Sq = S[p]; mq = m[p]; Uq = U[p]; }
                cand &= ~(1u << q);
                uint64_t Sn, cm;
                int first;
                cand_of(Sq, mq, Uq, Sn, cm, first);
                if (wave_test_from(L, tb, Sn, first, mq, cm, ty)) { best = q; bestU = uq; break; }
            }
        } else {
#pragma unroll
            for (int p = 0; p < KMAX; p++) {
                const int mp = m[p];
                if (p >= k || mm > mp) continue;
                if (ACT && (fb & S[p])) continue;
                uint64_t Sn, cm;
                int first;
                const uint64_t Un = cand_of(S[p], mp, U[p], Sn, cm, first);
                // cannot be taken whatever its test says (as in heuristic()): no test
                if (best >= 0) {
                    const int lb = max(lbm[p], mm);
                    if (lb > bestReq || (lb == bestReq && Un >= bestU)) continue;
                }
                if (!wave_test_from(L, tb, Sn, first, mp, cm, ty)) continue;
                // fewest units for Sn (binary search, as min_units)
                int lo = 1;
                for (uint64_t h = Sn; h; h &= h - 1ull) lo = max(lo, (int)L.mmin[__builtin_ctzll(h)]);
                int hi = mp;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (wave_test_from(L, tb, Sn, 0, mid, cm, ty))
                        hi = mid;
                    else
                        lo = mid + 1;
                }
                const int req = lo;
                if (best < 0 || req < bestReq || (req == bestReq && Un < bestU)) { best = p; bestU = Un; bestReq = req; }
            }
        }
        if (best < 0) return false;
        uint64_t Uold = 0;
#pragma unroll
        for (int p = 0; p < KMAX; p++)
            if (p == best) { Uold = U[p]; S[p] |= 1ull << r; U[p] = bestU; lbm[p] = max(lbm[p], mm); }
        need -= __shfl(li, r, 64);
        room = room + 1ull - (bestU - Uold);
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

// Offsets above the failing bound tried in the first round of a subset's
// search by a group of 16, 8 or 4 lanes (a 0 stands for the largest size
// still open, which also settles "none"): on random sets most subsets that
// fail at their lower bound need one to three more units.  Wide groups end
// most searches in one round (short dependency chains when few subsets are
// searched), narrow ones test fewer sizes per subset (less work when many are).
static __constant__ uint8_t FRONT_STEP16[16] = {1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 20, 24, 32, 0};
static __constant__ uint8_t FRONT_STEP8[8] = {1, 2, 3, 4, 6, 8, 16, 0};
static __constant__ uint8_t FRONT_STEP4[4] = {1, 2, 3, 0};

// Fill ms[] level by level (subsets of equal size, taken in the order of the
// host-built list `order`: subsets of {0..n-1} by size, then value).
// For S with lowest-priority member r (largest rank) and S' = S - {r}:
// lo = max(ms of the subsets with one member less, m_min of r) bounds ms[S]
// from below, and S is schedulable on m >= lo units iff the members whose
// response times can differ from those in S' pass: r alone, or, when r makes
// the single member j of its type in S' conflict, j and every member below j.
// Per chunk of at most blockDim subsets of a level:
//  A. one lane per subset: bounds; "none" is inherited without a test, the
//     others are queued (so that the tests of B run on packed lanes);
//  B. one lane per queued subset tests it at lo; failures with lo < M are
//     queued again;
//  C. groups of G = 16, 8 or 4 lanes (the widest that covers the queue in one
//     pass) search those: each round tests G sizes of the open interval (a, b)
//     with a failing and b passing (b = M + 1 stands for "none"), at the
//     first-round offsets above a, then evenly spaced; monotonicity in m makes
//     the first passing size of a round bracket the answer.
template <typename MT, typename TY>
__device__ void build_frontier(const SetLDS &L, const Tables &tb, int n, int M, uint16_t *ms,
                               const uint16_t *order, TY &ty)
{
    __shared__ uint32_t q1[256], q2[256];  // queued subsets: S | first << 16 | lo << 20
    __shared__ uint32_t cnt[2][2];         // queue lengths; chunks alternate rows (one is cleared while the other is read)
    const uint16_t *ord = order + ((1u << n) - 2u);
    const MT memm = (MT)L.memmask;
    // the utilisation screen below pays where utilisation is what limits a
    // fixed-priority partition, i.e. with implicit deadlines; with shorter
    // deadlines it rarely moves a bound, and under EDF the test itself starts
    // with the same utilisation check, so there it only costs its reads (the
    // block has >= n threads)
    const bool screen = __syncthreads_and((int)threadIdx.x >= n || L.D[threadIdx.x] == L.T[threadIdx.x]) != 0 &&
                        !use_edf<TY>(L);
    if (threadIdx.x == 0) { ms[0] = 0; cnt[0][0] = cnt[0][1] = cnt[1][0] = cnt[1][1] = 0u; }
    uint32_t cur = 0;
    uint32_t lvl_off = 1, lvl_cnt = (uint32_t)n;  // level 1 follows the empty set
    for (int c = 1; c <= n; c++) {
        for (uint32_t base = 0; base < lvl_cnt; base += blockDim.x, cur ^= 1u) {
            __syncthreads();  // the previous chunk's ms[] writes and queue reads are done
            if (threadIdx.x == 0) { cnt[cur ^ 1u][0] = 0u; cnt[cur ^ 1u][1] = 0u; }
            // A
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
                if (!none && screen) {
                    // utilisation screen: a partition whose utilisation exceeds 1
                    // on m units is unschedulable there, and utilisations never
                    // grow with m, so ms[S] lies above every m where the Q32 lower
                    // bound of the sum (table terms ceil(u 2^32) - 1 <= u 2^32)
                    // exceeds 2^32; no test is spent on those sizes
                    const MT cmS = conflict_mask<MT>((MT)S, memm);
                    while (lo <= M) {
                        const uint32_t *urow = tb.U + (lo - 1) * 2 * n;
                        uint64_t u = 0;
                        for (uint32_t h = S; h; h &= h - 1u) {
                            const int j = __ffs(h) - 1;
                            u += urow[(int)mbit(cmS, j) * n + j];
                        }
                        if (u <= (1ull << 32)) break;
                        lo++;
                    }
                    none = lo > M;
                }
                if (none) {
                    ms[S] = FRONT_NONE;
                } else {
                    const MT Sp = (MT)S & ~(MT(1) << r);
                    const MT same = Sp & (mbit(memm, r) ? memm : ~memm);
                    const int first = (mpopc(same) == 1) ? mctz(same) : r;
                    q1[atomicAdd(&cnt[cur][0], 1u)] = S | ((uint32_t)first << 16) | ((uint32_t)lo << 20);
                }
            }
            __syncthreads();
            // B
            const uint32_t N1 = cnt[cur][0];
            if (threadIdx.x < N1) {
                const uint32_t e = q1[threadIdx.x];
                const uint32_t S = e & 0xFFFFu;
                const int lo = (int)(e >> 20);
                const MT SM = (MT)S;
                if (test_from<MT>(L, tb, SM, (int)((e >> 16) & 0xFu), lo, conflict_mask<MT>(SM, memm), ty))
                    ms[S] = (uint16_t)lo;
                else if (lo < M)
                    q2[atomicAdd(&cnt[cur][1], 1u)] = e;
                else
                    ms[S] = FRONT_NONE;
            }
            __syncthreads();
            // C
            const uint32_t N2 = cnt[cur][1];
            const int G = N2 * 16u <= blockDim.x ? 16 : (N2 * 8u <= blockDim.x ? 8 : 4);
            const uint8_t *step = G == 16 ? FRONT_STEP16 : (G == 8 ? FRONT_STEP8 : FRONT_STEP4);
            const int groups = blockDim.x / G;
            const int g = threadIdx.x / G, li = threadIdx.x % G;
            const int shift = (threadIdx.x & 63) & ~(G - 1);
            const uint32_t gmask = (1u << G) - 1u;
            for (uint32_t f = g; f < N2; f += groups) {
                const uint32_t e = q2[f];
                const uint32_t S = e & 0xFFFFu;
                const int first = (int)((e >> 16) & 0xFu);
                const MT SM = (MT)S;
                const MT cm = conflict_mask<MT>(SM, memm);
                int a = (int)(e >> 20), b = M + 1;  // fails at a; passes at b (or none if b = M + 1)
                bool round1 = true;
                while (b - a > 1) {
                    // size tried by group lane i in this round: non-decreasing in i, within (a, b)
                    const int span = b - a;
                    const bool dense = span - 1 <= G;
                    auto point = [&](int i) {
                        if (round1) return step[i] ? min(a + (int)step[i], b - 1) : b - 1;
                        return dense ? min(a + 1 + i, b - 1) : a + ((i + 1) * span) / (G + 1);
                    };
                    const int x = point(li);
                    const bool pass = test_from<MT>(L, tb, SM, first, x, cm, ty);
                    const uint32_t gm = (uint32_t)(__ballot(pass) >> shift) & gmask;
                    if (gm) {
                        const int fl = __ffs(gm) - 1;
                        const int xf = point(fl);
                        a = fl == 0 ? a : point(fl - 1);
                        b = xf;
                    } else {
                        a = point(G - 1);
                    }
                    round1 = false;
                }
                if (li == 0) ms[S] = (b > M) ? FRONT_NONE : (uint16_t)b;
            }
        }
        lvl_off += lvl_cnt;
        lvl_cnt = lvl_cnt * (uint32_t)(n - c) / (uint32_t)(c + 1);
    }
    __syncthreads();
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

// k, or 0 when a part of m[0..k) has a size outside the admissible set: such
// a partitioning then has no part to place a task on, and is infeasible.
template <int KMAX>
__device__ __forceinline__ int admit(const Adm &a, const int (&m)[KMAX], int k)
{
    if ((a.w[0] | a.w[1] | a.w[2] | a.w[3]) == 0ull) return k;
    bool ok = true;
#pragma unroll
    for (int i = 0; i < KMAX; i++) {
        if (i < k) {
            const int x = m[i];
            const uint64_t wd = x < 64 ? a.w[0] : (x < 128 ? a.w[1] : (x < 192 ? a.w[2] : a.w[3]));
            ok &= ((wd >> (x & 63)) & 1ull) != 0ull;
        }
    }
    return ok ? k : 0;
}

// k, or 0 for a partitioning (sizes m, non-increasing, k parts) that
// stage_bounds found infeasible for every allocation: like an inadmissible
// size, it then gets no parts and fails at its first task.
template <int KMAX>
__device__ __forceinline__ int bound_k(const SetLDS &L, const int (&m)[KMAX], int k)
{
    if (k <= 0) return k;
    const int m1 = m[0];
    return ((L.lbad[k - 1][m1 >> 6] >> (m1 & 63)) & 1ull) ? 0 : k;
}

#ifdef CAPART_MAIN_TU  // non-template kernels: compiled in the main translation unit only
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
    if (w.counter != nullptr && blockIdx.x == 0 && lane == 0) {  // batched form: restart the queues
        w.counter[0] = 0u;
        w.counter[1] = 0u;
        w.counter[2] = 0u;
    }
    const int64_t off0 = b.off[s], off1 = b.off[s + 1];
    const int M = b.M[s];
    int status = CAPART_OK;
    const int nmax = min(b.max_tasks, MAXN), Mmax = min(b.max_M, CAPART_MAX_M);
    if (off0 < 0 || off1 < off0 || off1 > b.n_tasks_total) status = CAPART_E_INVAL;
    const int64_t n64 = off1 - off0;
    if (status == CAPART_OK && (n64 < 1 || n64 > nmax || M < 1 || M > Mmax || n64 * M > CAPART_MAX_NM))
        status = CAPART_E_INVAL;
    const bool tab = b.Cn != nullptr;  // explicit time tables
    int64_t toff = 0;
    if (status == CAPART_OK && tab) {
        toff = b.toff[s];
        if (toff < 0 || toff > b.tlen - n64 * M) status = CAPART_E_INVAL;
        if (w.tCn == nullptr) status = CAPART_E_INVAL;  // a path that does not stage tables
    }
    if (status != CAPART_OK) {
        if (lane == 0) { o.status[s] = status; w.setflags[s] = 0u; }
        return;
    }
    const int n = (int)n64;
    int64_t T = 1, D = 1, Cs = 0, Cp = 1;
    int32_t kk = 1000;
    int ty = 0;
    uint16_t tmmin = MMIN_NONE;
    bool bad = false;
    if (lane < n) {
        T = b.T[off0 + lane]; D = b.D[off0 + lane];
        ty = b.type[off0 + lane];
        const int64_t L31 = (int64_t)1 << 31;
        bad = (T < 1 || T >= L31 || D < 1 || D > T || ty > 1);
        if (tab) {
            // entries in [1, 2^31), non-increasing in m, Cc >= Cn, m Cn(m) >= Cn(1);
            // Cn(1) stands in for C_seq + C_par, Lemma 2 is the first m with Cn(m) <= D
            const int64_t *rn = b.Cn + toff + (int64_t)lane * M, *rc = b.Cc + toff + (int64_t)lane * M;
            const int64_t c1v = rn[0];
            int64_t pn = rn[0], pc = rc[0];
            for (int m = 1; m <= M; m++) {
                const int64_t cn = rn[m - 1], cc = rc[m - 1];
                bad |= cn < 1 || cn >= L31 || cc < 1 || cc >= L31 || cc < cn || cn > pn || cc > pc ||
                       (int64_t)m * cn < c1v;
                if (tmmin == MMIN_NONE && cn <= D) tmmin = (uint16_t)m;
                pn = cn;
                pc = cc;
            }
            Cs = 0;
            Cp = (c1v >= 1 && c1v < L31) ? c1v : 1;
        } else {
            Cs = b.Cs[off0 + lane]; Cp = b.Cp[off0 + lane];
            kk = b.k[off0 + lane];
            bad |= (Cs < 0 || Cp < 0 || Cs >= L31 || Cp >= L31 || Cs + Cp < 1 || Cs + Cp >= L31 || kk < 1000 ||
                    kk > 1000000);
        }
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
    // the bound of stage_bounds at the largest part a k-part partitioning can
    // have (M - k + 1 units; the bound only weakens as the largest part grows
    // and as k grows): when it rules out every k <= K, no partitioning of the
    // fixed-partitioning search can be schedulable and the set is not evaluated
    bool nofit = true;
    for (int k = 1; k <= min(Lp.K, M) && nofit; k++) {
        const int m1 = M - k + 1;
        uint64_t un = 0, uc = 0;
        if (lane < n) {
            uint64_t cn, cc;
            if (tab) {
                cn = (uint64_t)b.Cn[toff + (int64_t)lane * M + (m1 - 1)];
                cc = (uint64_t)b.Cc[toff + (int64_t)lane * M + (m1 - 1)];
            } else {
                cn = (uint64_t)Cs + ((uint64_t)Cp + (uint64_t)m1 - 1ull) / (uint64_t)m1;
                cc = ((uint64_t)kk * cn + 999ull) / 1000ull;
            }
            const uint64_t T64 = (uint64_t)T;
            un = cn > T64 ? (1ull << 32) + 1ull : ((cn << 32) + T64 - 1ull) / T64;
            uc = cc > T64 ? (1ull << 32) + 1ull : ((cc << 32) + T64 - 1ull) / T64;
        }
        uint64_t sum = uc;
#pragma unroll
        for (int o2 = 32; o2 >= 1; o2 >>= 1) sum += __shfl_xor(sum, o2, 64);
        // the k largest savings uc - un of each type, taken one by one
        uint64_t sv = (lane < n && uc > un) ? uc - un : 0ull, cut = 0;
        for (int t2 = 0; t2 < 2; t2++) {
            uint64_t mine = (lane < n && ty == t2) ? sv : 0ull;
            for (int j = 0; j < k; j++) {
                uint64_t mx = mine;
#pragma unroll
                for (int o2 = 32; o2 >= 1; o2 >>= 1) mx = max(mx, (uint64_t)__shfl_xor(mx, o2, 64));
                cut += mx;
                const uint64_t who = __ballot(mine == mx && mx != 0ull);
                if (who && lane == __ffsll((long long)who) - 1) mine = 0ull;
            }
        }
        nofit = sum - cut >= (uint64_t)n + ((uint64_t)k << 32);
    }
    // memory-intensive ranks
    uint64_t mm = (lane < n && ty == 1) ? (1ull << rank) : 0ull;
#pragma unroll
    for (int o2 = 32; o2 >= 1; o2 >>= 1) mm |= __shfl_xor(mm, o2, 64);
    if (lane < n) {
        TaskRec r;
        r.T = (uint32_t)T; r.D = (uint32_t)D; r.Cs = (uint32_t)Cs; r.Cp = (uint32_t)Cp; r.k = (uint32_t)kk;
        magic_u32((uint32_t)T, &r.clo, &r.chi);
        r.mmin = tab ? tmmin : m_min((uint32_t)Cs, (uint32_t)Cp, (uint32_t)D, (uint32_t)M);
        r.orig = (uint8_t)lane;
        r.mem = (uint8_t)ty;
        w.rec[off0 + rank] = r;
        w.sigma[off0 + pos] = (uint8_t)rank;
        srec[rank] = r;
        sforbid[rank] = 0ull;
    }
    if (lane == 0) {
        w.memmask[s] = mm;
        w.setflags[s] = SETF_VALID | (reject ? SETF_LEMMA1 : 0u) | (nofit ? SETF_NOFIT : 0u) | (Lp.edf ? SETF_EDF : 0u);
    }
    const bool act = (Lp.mode == CAPART_HEUR_BF_ACT || Lp.mode == CAPART_HEUR_SMS_ACT);
    if (!act) return;
    __syncthreads();
    // ACT: pair (a, b), a < b in rank order, is forbidden iff no size in
    // [max(mmin), min(mmin_a + mmin_b - 1, M)] schedules both together; by
    // monotonicity in m it suffices to test the top of that range.  The
    // n(n-1)/2 pairs are spread evenly over the lanes: pair q = b(b-1)/2 + a.
    const int npairs = n * (n - 1) / 2;
    for (int q = lane; q < npairs; q += 64) {
        int bb = (int)((1.0f + sqrtf(1.0f + 8.0f * (float)q)) * 0.5f);
        while (bb * (bb - 1) / 2 > q) bb--;
        while ((bb + 1) * bb / 2 <= q) bb++;
        const int a = q - bb * (bb - 1) / 2;
        const TaskRec ta = srec[a], tb = srec[bb];
        bool forb = true;
        if (ta.mmin != MMIN_NONE && tb.mmin != MMIN_NONE) {
            const uint32_t m = min((uint32_t)ta.mmin + tb.mmin - 1u, (uint32_t)M);
            const bool conf = ta.mem == tb.mem;
            uint32_t Ca, Cb;
            if (tab) {
                const int64_t *tt = conf ? b.Cc : b.Cn;
                Ca = (uint32_t)tt[toff + (int64_t)ta.orig * M + (m - 1)];
                Cb = (uint32_t)tt[toff + (int64_t)tb.orig * M + (m - 1)];
            } else {
                Ca = time_n(ta.Cs, ta.Cp, m);
                Cb = time_n(tb.Cs, tb.Cp, m);
                if (conf) { Ca = time_c(ta.k, Ca); Cb = time_c(tb.k, Cb); }
            }
            if (Lp.edf) {
                uint32_t dla, dha, dlb, dhb;
                magic_u32(ta.D, &dla, &dha);
                magic_u32(tb.D, &dlb, &dhb);
                const EdfTask ea{Ca, ta.T, ta.D, ta.clo, ta.chi, dla, dha}, eb{Cb, tb.T, tb.D, tb.clo, tb.chi, dlb, dhb};
                auto get = [=](int j) { return j ? eb : ea; };
                forb = !edf_demand<uint32_t>(3u, get, false).ok;
            } else if (Ca <= ta.D && Ca < ta.T) {
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
            atomicOr((unsigned long long *)&sforbid[a], (unsigned long long)(1ull << bb));
            atomicOr((unsigned long long *)&sforbid[bb], (unsigned long long)(1ull << a));
        }
    }
    __syncthreads();
    if (lane < n) w.forbid[off0 + lane] = sforbid[lane];
}

#endif  // CAPART_MAIN_TU
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
__device__ void heur_run(const SetLDS &L, const Tables &tb, const uint32_t *np, int n, int M, int K, const Adm &adm,
                         uint32_t q0, uint32_t q1, Key &best, uint64_t *dbg, MT *lS, uint64_t *lU, TY &ty)
{
    const int stride = blockDim.x;
    MT *myS = lS + threadIdx.x;
    uint64_t *myU = lU + threadIdx.x;
    int m[KMAX];
    int k = bound_k<KMAX>(L, m, admit<KMAX>(adm, m, unrank<KMAX>(np, M, K, q0, m)));
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
                if (key_less(kk, best)) {
                    best = kk;
                    MT Sl[KMAX];
#pragma unroll
                    for (int i = 0; i < KMAX; i++) Sl[i] = i < k ? myS[i * stride] : MT(0);
                    best.d = pack_alloc<KMAX, MT>(n, Sl);
                }
            }
            if (dbg) {
                uint64_t *d = dbg + 3 * (uint64_t)q;
                d[0] = ok ? mx : ~0ull;
                d[1] = ok ? sm : ~0ull;
                d[2] = ok ? 0ull : ~0ull;
            }
            if (++q >= q1) break;
            k = bound_k<KMAX>(L, m, admit<KMAX>(adm, m, next_partition<KMAX>(m, K)));
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
                                const Adm &adm, uint32_t q0, uint32_t q1, Key &best, uint64_t *dbg, TY &ty,
                                const Memo &mo)
{
    int m[KMAX];
    int k = bound_k<KMAX>(L, m, admit<KMAX>(adm, m, unrank<KMAX>(np, M, K, q0, m)));
    for (uint32_t q = q0;;) {
        MT S[KMAX];
        uint64_t U[KMAX];
        const bool ok = heuristic<KMAX, ACT, SMS, MT>(L, tb, n, m, k, S, U, ty, mo);
        uint64_t mx = 0, sm = 0;
        if (ok) {
#pragma unroll
            for (int i = 0; i < KMAX; i++) { mx = max(mx, U[i]); sm += U[i]; }
            const Key kk{mx, sm, q, 0ull};
            if (key_less(kk, best)) {
                best = kk;
                best.d = pack_alloc<KMAX, MT>(n, S);
            }
        }
        if (dbg) {
            uint64_t *d = dbg + 3 * (uint64_t)q;
            d[0] = ok ? mx : ~0ull;
            d[1] = ok ? sm : ~0ull;
            d[2] = ok ? 0ull : ~0ull;
        }
        if (++q >= q1) break;
        k = bound_k<KMAX>(L, m, admit<KMAX>(adm, m, next_partition<KMAX>(m, K)));
    }
}

template <int KMAX, bool ACT, bool SMS, typename MT, typename TY>
__device__ void heur_run_front(const SetLDS &L, const Tables &tb, const uint16_t *ms, const uint32_t *np, int n, int M,
                               int K, const Adm &adm, uint32_t q0, uint32_t q1, Key &best, uint64_t *dbg, TY &ty)
{
    int m[KMAX];
    int k = bound_k<KMAX>(L, m, admit<KMAX>(adm, m, unrank<KMAX>(np, M, K, q0, m)));
    for (uint32_t q = q0;;) {
        MT S[KMAX];
        uint64_t U[KMAX];
        const bool ok = heuristic_front<KMAX, ACT, SMS, MT>(L, tb, ms, n, m, k, S, U, ty);
        uint64_t mx = 0, sm = 0;
        if (ok) {
#pragma unroll
            for (int i = 0; i < KMAX; i++) { mx = max(mx, U[i]); sm += U[i]; }
            const Key kk{mx, sm, q, 0ull};
            if (key_less(kk, best)) {
                best = kk;
                best.d = pack_alloc<KMAX, MT>(n, S);
            }
        }
        if (dbg) {
            uint64_t *d = dbg + 3 * (uint64_t)q;
            d[0] = ok ? mx : ~0ull;
            d[1] = ok ? sm : ~0ull;
            d[2] = ok ? 0ull : ~0ull;
        }
        if (++q >= q1) break;
        k = bound_k<KMAX>(L, m, admit<KMAX>(adm, m, next_partition<KMAX>(m, K)));
    }
}

// Loop form 1 for sets with a test memo: every lane runs the heuristic on
// its partitionings as a state machine whose step places one task, answering
// its candidate tests from the memo; a lane that meets a test the memo cannot
// answer parks on it, and once every lane of the wave is parked or finished,
// the parked lanes run their tests together (packed, instead of one lane
// testing while the others idle).  Each result is recorded in the memo and
// kept by its lane, which resumes at the same candidate.  Candidates already
// settled for the current task are kept in registers (bit masks), and for SMS
// the fewest-units search of one candidate at a time keeps its bounds there,
// so progress never depends on the memo having room.  Parts are only ever
// indexed by compile-time constants (unrolled loops), which keeps them in
// registers.
template <int KMAX, bool ACT, bool SMS, typename TY>
__device__ void heur_run_memo(const SetLDS &L, const Tables &tb, const uint32_t *np, int n, int M, int K,
                              const Adm &adm, uint32_t q0, uint32_t q1, Key &best, uint64_t *dbg, TY &ty,
                              const Memo &mo)
{
    typedef uint32_t MT;
    int m[KMAX];
    MT S[KMAX];
    uint64_t U[KMAX];
#pragma unroll
    for (int i = 0; i < KMAX; i++) { m[i] = 0; S[i] = 0u; U[i] = 0ull; }
    bool active = q0 < q1;
    int k = active ? bound_k<KMAX>(L, m, admit<KMAX>(adm, m, unrank<KMAX>(np, M, K, q0, m))) : 0;
    uint32_t q = q0;
    int t = 0;
    uint32_t known = 0u, passm = 0u;  // candidates of the current task settled / schedulable
    uint64_t reqs = 0ull;             // SMS: fewest units of each schedulable candidate (8 bits each)
    int sp = -1, slo = 0, shi = 0;    // SMS: candidate being searched, sizes below slo fail, shi passes
    bool parked = false;              // a test of (tS, tfirst, tm) is due
    MT tS = 0u;
    int tfirst = 0, tm = 0;
    bool own = false, own_ok = false;  // result of this lane's last test, about (tS, tm)
    const MT memm = (MT)L.memmask;
    for (;;) {
        if (!__any(active)) break;
        while (active && !parked) {
            const int tau = L.sigma[t];
            const int mm = (int)L.mmin[tau];
            const MT bit = MT(1) << tau;
            const MT fb = ACT ? (MT)L.forbid[tau] : 0u;
#pragma unroll
            for (int p = 0; p < KMAX; p++) {
                if (parked || p >= k || ((known >> p) & 1u)) continue;
                const int mp = m[p];
                const MT Sp = S[p];
                if (mm > mp || (ACT && (fb & Sp))) { known |= 1u << p; continue; }
                const MT Sn = Sp | bit;
                int f, pz;
                ty.look();
                memo_get(mo, Sn, f, pz);
                if (own && tS == Sn) {
                    if (own_ok) pz = min(pz, tm); else f = max(f, tm);
                }
                if (sp != p) {
                    if (mp > f && mp < pz) {
                        // the incremental test: tau, the members below it and
                        // the lone same-type member it makes conflict (and below)
                        const MT same = Sp & (mbit(memm, tau) ? memm : ~memm);
                        tS = Sn;
                        tfirst = mpopc(same) == 1 ? min(tau, mctz(same)) : tau;
                        tm = mp;
                        parked = true;
                        continue;
                    }
                    if (mp <= f) { known |= 1u << p; continue; }
                    if (!SMS) { known |= 1u << p; passm |= 1u << p; continue; }
                    sp = p;
                    slo = 1;
                    for (MT h = Sn; h; h &= h - 1u) slo = max(slo, (int)L.mmin[mctz(h)]);
                    shi = mp;
                }
                slo = max(slo, f + 1);
                shi = min(shi, pz);
                if (slo < shi) {
                    tS = Sn;
                    tfirst = 0;
                    tm = (slo + shi) >> 1;
                    parked = true;
                    continue;
                }
                reqs |= (uint64_t)slo << (8 * p);
                known |= 1u << p;
                passm |= 1u << p;
                sp = -1;
            }
            if (parked) break;
            // every candidate settled: place tau on the best one, or the partitioning fails
            int bp = -1, breq = 0;
            uint64_t bu = 0;
#pragma unroll
            for (int p = 0; p < KMAX; p++) {
                if (!((passm >> p) & 1u)) continue;
                const uint64_t Un = util_add<MT>(L, tb, S[p], tau, m[p], U[p]);
                const int req = SMS ? (int)((reqs >> (8 * p)) & 0xFFu) : 0;
                if (bp < 0 || (SMS ? (req < breq || (req == breq && Un < bu)) : (Un < bu))) {
                    bp = p;
                    bu = Un;
                    breq = req;
                }
            }
            known = passm = 0u;
            reqs = 0ull;
            bool done = false, ok = false;
            if (bp < 0) {
                done = true;
            } else {
#pragma unroll
                for (int i = 0; i < KMAX; i++)
                    if (i == bp) { S[i] |= bit; U[i] = bu; }
                if (++t >= n) done = ok = true;
            }
            if (done) {
                uint64_t mx = 0, sm = 0;
                if (ok) {
#pragma unroll
                    for (int i = 0; i < KMAX; i++) { mx = max(mx, U[i]); sm += U[i]; }
                    const Key kk{mx, sm, q, 0ull};
                    if (key_less(kk, best)) {
                        best = kk;
                        best.d = pack_alloc<KMAX, MT>(n, S);
                    }
                }
                if (dbg) {
                    uint64_t *d = dbg + 3 * (uint64_t)q;
                    d[0] = ok ? mx : ~0ull;
                    d[1] = ok ? sm : ~0ull;
                    d[2] = ok ? 0ull : ~0ull;
                }
                if (++q >= q1) {
                    active = false;
                } else {
                    k = bound_k<KMAX>(L, m, admit<KMAX>(adm, m, next_partition<KMAX>(m, K)));
#pragma unroll
                    for (int i = 0; i < KMAX; i++) { S[i] = 0u; U[i] = 0ull; }
                    t = 0;
                }
            }
        }
        if (parked) {
            own_ok = test_from<MT>(L, tb, tS, tfirst, tm, conflict_mask<MT>(tS, memm), ty);
            memo_put(mo, tS, tm, own_ok);
            own = true;
            parked = false;
        }
    }
}

// The staged set's test memo (loop form 1, sets between the frontier limit
// and 32 tasks), placed after the tables, where frontier sets keep their
// frontier.
template <typename MT>
__device__ __forceinline__ Memo set_memo(const Launch &Lp, int n)
{
    if (sizeof(MT) != 4 || Lp.memo_log2 == 0 || n <= Lp.front_n || n > NARROW_MAX_TASKS) return Memo{nullptr, 0u};
    return Memo{(unsigned long long *)(capart_dyn_lds + Lp.table_words), (1u << Lp.memo_log2) - 1u};
}

// Empty the memo for a newly staged set (all threads; ends with a barrier).
template <typename MT, int FORM>
__device__ __forceinline__ void memo_clear(const Launch &Lp, int n)
{
    const Memo mo = set_memo<MT>(Lp, n);
    if (FORM != 1 || mo.mask == 0u) return;
    for (uint32_t i = threadIdx.x; i <= mo.mask; i += blockDim.x) mo.tab[i] = 0ull;
    __syncthreads();
}

// Evaluate partitionings [p0, p1) of one staged set in this block (all
// lanes).  FORM 0: every set of the launch is answered through its
// frontier; FORM 1 (nested loops, or the memo state machine) and FORM 2 (one
// candidate test per loop step): sets above the frontier limit, with direct
// incremental tests or the test memo.  Each launch compiles only its own path.
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
    if constexpr (FORM == 0) {
        uint16_t *ms = (uint16_t *)(capart_dyn_lds + Lp.table_words);
        build_frontier<MT>(L, tb, n, M, ms, order, ty);
        if (q0 < q1) heur_run_front<KMAX, ACT, SMS, MT>(L, tb, ms, np, n, M, Lp.K, Lp.adm, q0, q1, best, dbg, ty);
        return;
    } else {
    if (q0 >= q1) return;
    if constexpr (FORM == 2) {
        uint64_t *lU = (uint64_t *)(capart_dyn_lds + Lp.table_words + Lp.front_words);
        MT *lS = (MT *)(lU + KMAX * blockDim.x);
        heur_run<KMAX, ACT, SMS, MT>(L, tb, np, n, M, Lp.K, Lp.adm, q0, q1, best, dbg, lS, lU, ty);
    } else {
        const Memo mo = set_memo<MT>(Lp, n);
        if constexpr (sizeof(MT) == 4 && KMAX <= 4) {  // (K = 8 keeps the nested form: fewer registers)
            if (mo.mask && Lp.memo_packed) {
                heur_run_memo<KMAX, ACT, SMS>(L, tb, np, n, M, Lp.K, Lp.adm, q0, q1, best, dbg, ty, mo);
                return;
            }
        }
        heur_run_nested<KMAX, ACT, SMS, MT>(L, tb, np, n, M, Lp.K, Lp.adm, q0, q1, best, dbg, ty, mo);
    }
    }
}

template <int KMAX, bool ACT, bool SMS, typename MT, int FORM, bool COUNT = false, int POL = POL_ANY>
__global__ __launch_bounds__(512) void eval_heur_kernel(Batch b, Work w, Out o, Launch Lp, uint32_t p_lo,
                                                        uint32_t p_hi)
{
    __shared__ SetLDS L;
    __shared__ Key red[16];
    typename std::conditional<COUNT, TallyP<POL>, NoTallyP<POL>>::type ty;
    const int64_t s = Lp.s0 + blockIdx.x / Lp.chunks;
    const int c = blockIdx.x % Lp.chunks;
    const uint32_t f = w.setflags[s];
    if (!(f & SETF_VALID)) return;
    const int64_t off = b.off[s];
    const int n = (int)(b.off[s + 1] - off);
    if (n < Lp.n_lo || (Lp.n_hi > 0 && n > Lp.n_hi)) return;  // evaluated by the launch for its size
    const int M = b.M[s];
    const uint32_t P = w.np[np_index(Lp.K, M, M)];
    const uint32_t p0 = (uint32_t)c * Lp.chunk;
    if (p0 >= P) return;
    const uint32_t p1 = min(P, p0 + Lp.chunk);
    uint64_t *dbg = o.dbg_key ? o.dbg_key + 3 * o.dbg_offset[s] : nullptr;
    Key best = key_none();
    if (!(f & (SETF_LEMMA1 | SETF_NOFIT))) {
        Tables tb;
        stage_set(L, w, off, n, M, s, ACT, tb);
        stage_bounds<KMAX>(L, tb, n, M);
        memo_clear<MT, FORM>(Lp, n);
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

// eval, wide sets (launches of sets above NARROW_MAX_TASKS tasks with
// Lp.wchunk > 0): one block per (set, chunk of Lp.wchunk partitionings), each
// wave takes every nw-th partitioning of the chunk and runs wave_heuristic on
// it, so a partitioning costs one test's critical path per candidate instead
// of all of its members' fixed points in one lane.  Only the execution-time
// table is staged (utilisations through the reciprocal of T).
template <int KMAX, bool ACT, bool SMS, bool COUNT = false, int POL = POL_ANY>
__global__ __launch_bounds__(512) void eval_wide_kernel(Batch b, Work w, Out o, Launch Lp, uint32_t p_lo,
                                                        uint32_t p_hi)
{
    __shared__ SetLDS L;
    __shared__ Key red[16];
    typename std::conditional<COUNT, TallyP<POL>, NoTallyP<POL>>::type ty;
    const int64_t s = Lp.s0 + blockIdx.x / Lp.chunks;
    const int c = blockIdx.x % Lp.chunks;
    const uint32_t f = w.setflags[s];
    if (!(f & SETF_VALID)) return;
    const int64_t off = b.off[s];
    const int n = (int)(b.off[s + 1] - off);
    if (n < Lp.n_lo || (Lp.n_hi > 0 && n > Lp.n_hi)) return;  // evaluated by the launch for its size
    const int M = b.M[s];
    const uint32_t P = w.np[np_index(Lp.K, M, M)];
    const uint32_t p0 = (uint32_t)c * (uint32_t)Lp.wchunk;
    if (p0 >= P) return;
    const uint32_t p1 = min(P, p0 + (uint32_t)Lp.wchunk);
    uint64_t *dbg = o.dbg_key ? o.dbg_key + 3 * o.dbg_offset[s] : nullptr;
    const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    Key best = key_none();
    if (!(f & (SETF_LEMMA1 | SETF_NOFIT))) {
        Tables tb;
        stage_set_times(L, w, off, n, M, s, ACT, tb);
        stage_bounds<KMAX>(L, tb, n, M);
        const uint32_t q0 = p0 + (uint32_t)wv;
        if (q0 < p1) {
            int m[KMAX];
            int k = bound_k<KMAX>(L, m, admit<KMAX>(Lp.adm, m, unrank<KMAX>(w.np, M, Lp.K, q0, m)));
            for (uint32_t q = q0;;) {
                if (q >= p_lo && q < p_hi) {
                    uint64_t S[KMAX], U[KMAX];
                    const bool ok = wave_heuristic<KMAX, ACT, SMS>(L, tb, n, m, k, S, U, ty);
                    uint64_t mx = 0, sm = 0;
                    if (ok) {
#pragma unroll
                        for (int i = 0; i < KMAX; i++) { mx = max(mx, U[i]); sm += U[i]; }
                        const Key kk{mx, sm, q, 0ull};
                        if (key_less(kk, best)) {
                            best = kk;
                            best.d = pack_alloc<KMAX, uint64_t>(n, S);
                        }
                    }
                    if (dbg && (threadIdx.x & 63) == 0) {
                        uint64_t *d = dbg + 3 * (uint64_t)q;
                        d[0] = ok ? mx : ~0ull;
                        d[1] = ok ? sm : ~0ull;
                        d[2] = ok ? 0ull : ~0ull;
                    }
                }
                q += (uint32_t)nw;
                if (q >= p1) break;
                for (int i = 0; i < nw; i++) k = next_partition<KMAX>(m, Lp.K);
                k = bound_k<KMAX>(L, m, admit<KMAX>(Lp.adm, m, k));
            }
        }
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
        uint64_t a = ty.terms, bb = ty.tests;
#pragma unroll
        for (int o2 = 32; o2 >= 1; o2 >>= 1) {
            a += __shfl_xor(a, o2, 64);
            bb += __shfl_xor(bb, o2, 64);
        }
        if ((threadIdx.x & 63) == 0 && w.counters) {
            atomicAdd((unsigned long long *)&w.counters[0], (unsigned long long)a);
            atomicAdd((unsigned long long *)&w.counters[1], (unsigned long long)bb);
        }
    }
}

// eval, batched form: a persistent grid; each block repeatedly takes the next
// work item (set, partitioning range) from a global counter, restages the
// set's LDS tables only when the set changes, and writes the item's best key
// to its partial slot.  Items come largest first, so the tail is short.
template <int KMAX, bool ACT, bool SMS, typename MT, int FORM, int POL = POL_ANY>
__global__ __launch_bounds__(512) void eval_persistent_kernel(Batch b, Work w, Out o, Launch Lp)
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
        if ((f & SETF_VALID) && !(f & (SETF_LEMMA1 | SETF_NOFIT))) {
            const int64_t off = b.off[s];
            const int n = (int)(b.off[s + 1] - off);
            const int M = b.M[s];
            if (s != staged) {
                stage_set(L, w, off, n, M, s, ACT, tb);
                stage_bounds<KMAX>(L, tb, n, M);
                memo_clear<MT, FORM>(Lp, n);
                staged = s;
            }
            NoTallyP<POL> nt;
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
    if (!(f & (SETF_LEMMA1 | SETF_NOFIT)) && q >= p_lo && q < p_hi) {
        Tables tb;
        stage_set(L, w, off, n, M, s, false, tb);
        stage_bounds<KMAX>(L, tb, n, M);
        int m[KMAX];
        const int k = bound_k<KMAX>(L, m, admit<KMAX>(Lp.adm, m, unrank<KMAX>(w.np, M, Lp.K, q, m)));
        uint64_t A = k > 0 ? 1 : 0;  // an inadmissible partitioning has no allocation
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
        // partitionings per chunk: the wide-set launch uses its own chunk size
        const uint64_t ch = (!exh && Lp.wchunk > 0 && n > NARROW_MAX_TASKS) ? (uint64_t)Lp.wchunk : (uint64_t)Lp.chunk;
        for (int c = lane; c < Lp.chunks; c += 64) {
            const bool live = exh ? ((uint32_t)c < P) : ((uint64_t)c * ch < P);
            if (!live) continue;
            const uint64_t *src = w.partial + 4 * (s * (int64_t)Lp.chunks + c);
            const Key kk{src[0], src[1], src[2], src[3]};
            if (key_less(kk, best)) best = kk;
        }
    }
    best = wave_min(best);
    const bool found = best.a != ~0ull;
    const bool act = (Lp.mode == CAPART_HEUR_BF_ACT || Lp.mode == CAPART_HEUR_SMS_ACT);
    // the chosen allocation comes from the allocation index (exhaustive), from
    // the allocation packed in the key (heuristic), or, for sets too large to
    // pack, from replaying the heuristic on the chosen partitioning, which
    // needs the whole tables; otherwise only the rows of the chosen sizes and
    // of M are filled
    const bool replay = found && !exh && n > AllocPack<KMAX>::MAX_N;
    Tables tb;
    if (replay) {
        stage_set(L, w, off, n, M, s, act, tb);
    } else {
        stage_records(L, w, off, n, s, act);
        tb.C = capart_dyn_lds;
        tb.U = capart_dyn_lds + 2 * n * M;
        tb.n = n;
        __syncthreads();
    }
    if (found) {
        int m[KMAX];
        int k = unrank<KMAX>(w.np, M, K, (uint32_t)best.c, m);
        uint64_t S[KMAX], U[KMAX];
#pragma unroll
        for (int p = 0; p < KMAX; p++) S[p] = 0ull;
        if (replay) {  // the whole wave replays the heuristic on the chosen partitioning
            NoTally nt;
            switch (Lp.mode) {
            case CAPART_HEUR_BF_INA: wave_heuristic<KMAX, false, false>(L, tb, n, m, k, S, U, nt); break;
            case CAPART_HEUR_BF_ACT: wave_heuristic<KMAX, true, false>(L, tb, n, m, k, S, U, nt); break;
            case CAPART_HEUR_SMS_INA: wave_heuristic<KMAX, false, true>(L, tb, n, m, k, S, U, nt); break;
            default: wave_heuristic<KMAX, true, true>(L, tb, n, m, k, S, U, nt); break;
            }
        } else if (lane == 0 && exh) {
            uint64_t x = best.d;
            for (int i = n - 1; i >= 0; i--) {
                const int d = (int)(x % (uint64_t)k);
                x /= (uint64_t)k;
#pragma unroll
                for (int p = 0; p < KMAX; p++)
                    if (p == d) S[p] |= 1ull << L.rank_of[i];
            }
        } else if (lane == 0) {
            constexpr int B = AllocPack<KMAX>::BITS;
            for (int r = 0; r < n; r++) {
                const int d = (int)((best.d >> (B * r)) & ((1u << B) - 1u));
#pragma unroll
                for (int p = 0; p < KMAX; p++)
                    if (p == d) S[p] |= 1ull << r;
            }
        }
        if (lane == 0) {
#pragma unroll
            for (int p = 0; p < KMAX; p++) { sS[p] = S[p]; sm_[p] = m[p]; }
            sk = k;
        }
    }
    __syncthreads();
    if (!replay) {
        // execution-time rows of the chosen part sizes and of M (the whole GPU)
        const int rows = found ? sk + 1 : 1;
        uint32_t *tc = capart_dyn_lds;
        for (int e = lane; e < rows * n; e += 64) {
            const int i = e / n, r = e - i * n;
            const int m = (i + 1 < rows) ? sm_[i] : M;
            uint32_t cn, cc;
            exec_times(L, w, s, M, r, m, cn, cc);
            const int base = (m - 1) * 2 * n + r;
            tc[base] = cn;
            tc[base + n] = cc;
        }
        __syncthreads();
    }
    // response times of the chosen triple
    if (lane < n) {
        const int64_t gi = off + L.orig[lane];
        if (found) {
            int part = 0, mp = 0;
            uint64_t Sp = 0;
            for (int p = 0; p < sk; p++)
                if ((sS[p] >> lane) & 1ull) { part = p; mp = sm_[p]; Sp = sS[p]; }
            const uint32_t R = resp_one<uint64_t>(L, tb, mp, lane, Sp, conflict_mask<uint64_t>(Sp, L.memmask));
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
            R1 = resp_one<uint64_t>(L, tb, M, lane, all, conflict_mask<uint64_t>(all, L.memmask));
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
        o.aidx[s] = found ? (exh ? (int64_t)best.d : 0) : -1;
        o.maxU[s] = found ? best.a : 0ull;
        o.sumU[s] = found ? best.b : 0ull;
        o.n_evals[s] = (int64_t)P;
    }
    for (int p = lane; p < K; p += 64) o.sizes[s * K + p] = (found && p < KMAX) ? sm_[p] : 0;
}

// ---------------------------------------------------------------------------
// Algorithm 1 with free partition sizes (Section "Heuristics"), one wave per
// set.  Lane p holds par_list position p in registers: the partition's rank
// mask, units, Q32 utilisation, lowest task index and the set of partitions
// it may not merge with, as a mask of partition ids (a partition's id is its
// lowest rank; a forbidden task pair puts each partition's id in the other's
// mask, a merge keeps the smaller id and relabels the other one everywhere).
// par_list is kept in decreasing utilisation (ties: lowest task index).
// While the partitions need more than M units, the first partition with an
// eligible partner (Algorithm 3) is found with one ballot, and every eligible
// partner's merge (Algorithm 2) is computed at once, one lane per partner: the
// fewest units in [max(m1, m2), min(m1 + m2 - 1, M)], by binary search
// (schedulability is monotone in m, so this is the first size of the paper's
// upward scan).  Order ">": partners ranked by the union's utilisation at
// max(m1, m2); the first valid merge in that order is taken and the merges
// ranked before it (all failed) forbid their task pairs.  Order ">>": the
// valid merge with the fewest units (then utilisation, then par_list
// position) is taken and every failed merge forbids its pairs.  With ACT the
// forbidden pairs start from Definition 3's pair test (prep kernel).  A merge
// replaces the two partitions by their union at its place in the order: every
// lane's new position follows from one ballot, and a forward permute moves it.

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

// value of the lane CTRL-shifted within its row of 16 (DPP row_shr), or `id`
// where that lane lies outside the row
template <int CTRL>
__device__ __forceinline__ uint64_t dpp_row_shr64(uint64_t v, uint64_t id)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)id, (int)(uint32_t)v, CTRL, 0xF, 0xF, false);
    const uint32_t hi =
        (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(id >> 32), (int)(uint32_t)(v >> 32), CTRL, 0xF, 0xF, false);
    return ((uint64_t)hi << 32) | lo;
}

// wave reductions (all 64 lanes active): row scans by DPP shifts of 1, 2, 4
// and 8 lanes, then the four row results combined from lanes 15, 31, 47, 63
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v)
{
    v = min(v, dpp_row_shr64<0x111>(v, ~0ull));
    v = min(v, dpp_row_shr64<0x112>(v, ~0ull));
    v = min(v, dpp_row_shr64<0x114>(v, ~0ull));
    v = min(v, dpp_row_shr64<0x118>(v, ~0ull));
    return min(min(readlane64(v, 15), readlane64(v, 31)), min(readlane64(v, 47), readlane64(v, 63)));
}

__device__ __forceinline__ uint64_t wave_or(uint64_t v)
{
    v |= dpp_row_shr64<0x111>(v, 0ull);
    v |= dpp_row_shr64<0x112>(v, 0ull);
    v |= dpp_row_shr64<0x114>(v, 0ull);
    v |= dpp_row_shr64<0x118>(v, 0ull);
    return readlane64(v, 15) | readlane64(v, 31) | readlane64(v, 47) | readlane64(v, 63);
}

__device__ __forceinline__ int readlane32(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

// forward permute: the value of this lane goes to lane dst (a permutation of the wave)
__device__ __forceinline__ uint64_t permute64(uint64_t v, int dst)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_permute(dst << 2, (int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_permute(dst << 2, (int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ int permute32(int v, int dst) { return __builtin_amdgcn_ds_permute(dst << 2, v); }


// Q32 utilisation of rank set S on m units (schedulable or not), mod 2^64
__device__ __forceinline__ uint64_t group_util(const SetLDS &L, const Tables &tb, uint64_t S, int m, uint64_t cm)
{
    uint64_t u = 0;
    for (uint64_t h = S; h; h &= h - 1ull) {
        const int r = __builtin_ctzll(h);
        u += util_term(L, tb, r, m, (uint32_t)((cm >> r) & 1ull));
    }
    return u;
}

template <bool ACT, bool SMS, typename TY>
__global__ __launch_bounds__(64) void alg1_kernel(Batch b, Work w, A1Out o, Launch Lp)
{
    __shared__ SetLDS L;
    const int64_t s = Lp.s0 + blockIdx.x;
    const int lane = threadIdx.x;
    const uint32_t f = w.setflags[s];
    const int64_t off0 = b.off[s], off1 = b.off[s + 1];
    auto write_failure = [&](int64_t tried, int64_t merged) {
        if (lane == 0) {
            o.verdict[s] = 0;
            o.nparts[s] = 0;
            o.tried[s] = tried;
            o.merged[s] = merged;
            if (o.workload) o.workload[s] = 0ull;
        }
        if (off0 >= 0 && off1 >= off0 && off1 <= b.n_tasks_total)
            for (int64_t i = off0 + lane; i < off1; i += 64) { o.sizes[i] = 0; o.alloc[i] = -1; o.R[i] = -1; }
    };
    if (!(f & SETF_VALID)) { write_failure(0, 0); return; }
    const int n = (int)(off1 - off0);
    const int M = b.M[s];
    Tables tb;
    stage_set_times(L, w, off0, n, M, s, ACT, tb);
    if (f & SETF_LEMMA1) { write_failure(0, 0); return; }
    const uint64_t memm = L.memmask;
    // init partitions: one per task, of its Lemma 2 size (partition id = rank)
    uint64_t Pm = 0, PX = 0, PU = 0;
    int Pmu = 0, Pl = lane;
    bool bad = false;
    if (lane < n) {
        const int m = (int)L.mmin[lane];
        bad = m > M;
        Pm = 1ull << lane;
        PX = ACT ? L.forbid[lane] : 0ull;
        Pmu = bad ? 1 : m;
        PU = bad ? 0ull : util_term(L, tb, lane, m, 0u);
        Pl = L.orig[lane];
    }
    if (__any(bad)) { write_failure(0, 0); return; }
    {
        int pos = 0;
        for (int j = 0; j < n; j++) {
            const uint64_t uj = readlane64(PU, j);
            const int lj = readlane32(Pl, j);
            pos += (uj > PU || (uj == PU && lj < Pl)) ? 1 : 0;
        }
        if (lane >= n) pos = lane;
        Pm = permute64(Pm, pos); PX = permute64(PX, pos); PU = permute64(PU, pos);
        Pmu = permute32(Pmu, pos); Pl = permute32(Pl, pos);
    }
    uint64_t live = n == 64 ? ~0ull : (1ull << n) - 1ull;  // ids of the partitions
    int np = n;
    int Pi = 0;
    for (int j = 0; j < n; j++) Pi += readlane32(Pmu, j);
    int64_t tried = 0, merged = 0;
    TY ty;
    bool ok = false;
    for (;;) {
        if (Pi <= M) { ok = true; break; }
        // partitions with an eligible partner; the first one is the operand
        const uint64_t idb = Pm & (0ull - Pm);  // this partition's id bit
        const uint64_t cand = __ballot(lane < np && (live & ~PX & ~idb) != 0ull);
        if (!cand) break;  // no partition has an eligible partner: fail
        const int c = __builtin_ctzll(cand);
        const uint64_t Sc = readlane64(Pm, c), Xc = readlane64(PX, c);
        const uint64_t idc = Sc & (0ull - Sc);
        const int mc = readlane32(Pmu, c);
        const bool elig = lane < np && lane != c && (Xc & idb) == 0ull;
        // every eligible partner's merge, one lane each; rank key (ka, lane):
        // ">" the union's utilisation at max(m1, m2), ">>" (units, U) of the
        // merge (valid merges only)
        bool mok = false;
        int m3 = 0;
        uint64_t U3 = 0, ka = ~0ull, S3 = 0;
        if (elig) {
            S3 = Sc | Pm;
            const uint64_t cm = conflict_mask<uint64_t>(S3, memm);
            const int mlo = max(mc, Pmu), mhi = min(mc + Pmu - 1, M);
            if (!SMS) ka = group_util(L, tb, S3, mlo, cm);
            if (test_from<uint64_t>(L, tb, S3, 0, mhi, cm, ty)) {
                int lo = mlo, hi = mhi;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (test_from<uint64_t>(L, tb, S3, 0, mid, cm, ty))
                        hi = mid;
                    else
                        lo = mid + 1;
                }
                mok = true;
                m3 = lo;
                U3 = group_util(L, tb, S3, lo, cm);
            }
            if (SMS && mok) ka = ((uint64_t)m3 << 44) | U3;  // U3 <= 64 * 2^32: every member meets D <= T
        }
        // the merge taken: the valid one of least (ka, lane); for ">" that is
        // the first valid merge in rank order, for ">>" the best one
        const uint64_t best_a = wave_min_u64(mok ? ka : ~0ull);
        const int best_l = (int)wave_min_u64(mok && ka == best_a ? (uint64_t)lane : 64ull);
        const bool before = ka < best_a || (ka == best_a && lane < best_l);
        // failed merges that forbid their pairs: for ">" those ranked before
        // the merge taken (all of them if none is valid), for ">>" all
        const bool forbid = elig && !mok && (SMS || before);
        tried += (int64_t)__popcll(__ballot(elig && (SMS || before || lane == best_l)));
        if (forbid) PX |= idc;
        const uint64_t Xfail = wave_or(forbid ? idb : 0ull);
        if (lane == c) PX |= Xfail;
        if (best_l == 64) continue;  // P_c has no valid merge; its partners are now forbidden
        // merge P_c with partner j: par_list minus both, plus the union (which
        // keeps the smaller id; the other id is relabelled in every mask)
        const int j = best_l;
        const uint64_t Sj3 = readlane64(S3, j), Uj3 = readlane64(U3, j);
        const uint64_t X3 = readlane64(PX, c) | readlane64(PX, j);
        const uint64_t idj = readlane64(idb, j);
        const uint64_t keep = min(idc, idj), gone = max(idc, idj);
        const int mj3 = readlane32(m3, j), mj = readlane32(Pmu, j);
        const int lead = min(readlane32(Pl, c), readlane32(Pl, j));
        const bool rem = lane < np && lane != c && lane != j;
        const bool bnew = rem && (PU > Uj3 || (PU == Uj3 && Pl < lead));
        const int pos_new = __popcll(__ballot(bnew));
        const int r = lane - (lane > c ? 1 : 0) - (lane > j ? 1 : 0);
        int dst = lane;
        if (rem) {
            dst = r + (r >= pos_new ? 1 : 0);
        } else if (lane == c) {
            dst = pos_new;
            Pm = Sj3; PX = X3; PU = Uj3; Pmu = mj3; Pl = lead;
        } else if (lane == j) {
            dst = np - 1;
        }
        if (PX & gone) PX = (PX & ~gone) | keep;
        Pm = permute64(Pm, dst); PX = permute64(PX, dst); PU = permute64(PU, dst);
        Pmu = permute32(Pmu, dst); Pl = permute32(Pl, dst);
        live &= ~gone;
        np -= 1;
        Pi += mj3 - mc - mj;
        merged += 1;
    }
    if constexpr (std::is_same<TY, TallyP<TY::kPol>>::value) {
        uint64_t a = ty.terms, bb = ty.tests;
#pragma unroll
        for (int o2 = 32; o2 >= 1; o2 >>= 1) {
            a += __shfl_xor(a, o2, 64);
            bb += __shfl_xor(bb, o2, 64);
        }
        if (lane == 0 && w.counters) {
            atomicAdd((unsigned long long *)&w.counters[0], (unsigned long long)a);
            atomicAdd((unsigned long long *)&w.counters[1], (unsigned long long)bb);
        }
    }
    if (!ok) { write_failure(tried, merged); return; }
    if (lane == 0) {
        o.verdict[s] = 1;
        o.nparts[s] = np;
        o.tried[s] = tried;
        o.merged[s] = merged;
    }
    if (lane < n) o.sizes[off0 + lane] = lane < np ? Pmu : 0;
    // each task's partition, then its response time there
    int part = 0, mp = 1;
    uint64_t Sp = 0;
    for (int p = 0; p < np; p++) {
        const uint64_t mk = readlane64(Pm, p);
        const int mm = readlane32(Pmu, p);
        if ((mk >> lane) & 1ull) { part = p; Sp = mk; mp = mm; }
    }
    uint64_t wl = 0ull;  // the scheduled workload: one-unit utilisations in the final conflict states
    if (lane < n) {
        const uint64_t cm = conflict_mask<uint64_t>(Sp, memm);
        const uint32_t R = resp_one<uint64_t, TY>(L, tb, mp, lane, Sp, cm);
        const int64_t gi = off0 + L.orig[lane];
        o.alloc[gi] = (int8_t)part;
        o.R[gi] = R ? (int64_t)R : -1;
        wl = util_term(L, tb, lane, 1, (uint32_t)((cm >> lane) & 1ull));
    }
#pragma unroll
    for (int o2 = 32; o2 >= 1; o2 >>= 1) wl += __shfl_xor(wl, o2, 64);
    if (lane == 0 && o.workload) o.workload[s] = wl;
}

#ifdef CAPART_MAIN_TU
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
    if (!(f & SETF_VALID) || (f & (SETF_LEMMA1 | SETF_NOFIT))) return;
    const int64_t off = b.off[s];
    const int n = (int)(b.off[s + 1] - off);
    const int M = b.M[s];
    if (m > M || n > ntab) return;
    Tables tb;
    stage_set(L, w, off, n, M, s, false, tb);
    uint64_t *dst = tab + (((size_t)s_local * Mtab + (size_t)(m - 1)) << ntab);
    const uint32_t NA = 1u << n;
    Tally ty;  // kept only when the launch counts work (w.counters)
    for (uint32_t A = threadIdx.x; A < NA; A += blockDim.x) {
        uint32_t RA = 0;
        for (uint32_t a = A; a; a &= a - 1u) RA |= 1u << L.rank_of[__builtin_ctz(a)];
        uint64_t u = 0;
        if (w.counters) {
            dst[A] = part_test<uint32_t>(L, tb, RA, m, &u, ty) ? u : ~0ull;
        } else {
            NoTally nt;
            dst[A] = part_test<uint32_t>(L, tb, RA, m, &u, nt) ? u : ~0ull;
        }
    }
    if (w.counters) {
        uint64_t a = ty.terms, bb = ty.tests;
#pragma unroll
        for (int o2 = 32; o2 >= 1; o2 >>= 1) {
            a += __shfl_xor(a, o2, 64);
            bb += __shfl_xor(bb, o2, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            atomicAdd((unsigned long long *)&w.counters[0], (unsigned long long)a);
            atomicAdd((unsigned long long *)&w.counters[1], (unsigned long long)bb);
        }
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
    uint64_t combines = 0;  // subset-table lookups of candidate parts (counted when w.counters is set)
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
    const bool admitted = admit<4>(Lp.adm, m, k) > 0;
    if (!(f & (SETF_LEMMA1 | SETF_NOFIT)) && admitted && threadIdx.x < npre && q >= p_lo && q < p_hi) {
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
                        combines++;
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
    if (w.counters) {
        uint64_t c2 = combines;
#pragma unroll
        for (int o2 = 32; o2 >= 1; o2 >>= 1) c2 += __shfl_xor(c2, o2, 64);
        if ((threadIdx.x & 63) == 0 && c2) atomicAdd((unsigned long long *)&w.counters[2], (unsigned long long)c2);
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

#endif  // CAPART_MAIN_TU
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
        R = resp_one<uint64_t>(L, tb, sizes[p], lane, Sp, cm);
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
// Launch groups.  Each group's members are defined in a launcher translation
// unit of its own and explicitly instantiated there; the dispatch in
// capart_kernels.hip sees these declarations only.
//
// form: 0 = every set answered through its feasibility frontier, 1 = nested
// loops (direct tests or the test memo), 2 = one candidate test per loop step.
template <int KMAX, typename MT, int POL>
struct HeurLaunch {
    static hipError_t eval(const Batch &b, const Work &w, const Out &o, const Launch &L, hipStream_t st, uint32_t p_lo,
                           uint32_t p_hi, int form);
    static hipError_t persistent(const Batch &b, const Work &w, const Out &o, const Launch &L, int blocks,
                                 hipStream_t st, int form);
    static hipError_t count(const Batch &b, const Work &w, const Out &o, const Launch &L, hipStream_t st, int form);
    static hipError_t allow();
};

template <int POL>
struct WideLaunch {
    static hipError_t eval(int kmax, bool count, const Batch &b, const Work &w, const Out &o, const Launch &L,
                           hipStream_t st, uint32_t p_lo, uint32_t p_hi);
    static hipError_t allow();
};

template <int POL>
struct Alg1Launch {
    static hipError_t run(bool count, const Batch &b, const Work &w, const A1Out &o, const Launch &L, hipStream_t st);
    static hipError_t allow();
};

// Dynamic LDS of the kernels that stage a whole set's tables.
static inline size_t dyn_bytes(const Batch &b) { return table_lds_bytes(min(b.max_tasks, MAXN), min(b.max_M, 255)); }

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

}  // namespace capart
