// Algorithm 1 (free partition sizes, Section "Heuristics") for batches with
// sets of up to 256 tasks (the paper's 200-task experiments, Figs. 6-8): one
// block of 256 threads per set, thread p holding par_list position p.  The
// same steps, orders, readings and outputs as alg1_kernel (one wave per set,
// at most 64 tasks), with 256-bit rank and partition-id sets and block-wide
// reductions through LDS atomics in place of wave ballots and DPP, and the
// ACT pairs (Definition 3) computed in the kernel.  Fixed-priority DM per
// partition.  Included by its launch translation unit only.
#pragma once
#include "capart_device.h"

namespace capart {

constexpr int BIGN = 256;  // tasks (and partitions) per set

// A set of ranks (or partition ids) 0..255.
struct M256 {
    uint64_t w[4];
};

__device__ __forceinline__ M256 m_zero() { return M256{{0ull, 0ull, 0ull, 0ull}}; }
__device__ __forceinline__ M256 m_bit(int i)
{
    M256 r = m_zero();
#pragma unroll
    for (int k = 0; k < 4; k++) r.w[k] = (i >> 6) == k ? (1ull << (i & 63)) : 0ull;
    return r;
}
__device__ __forceinline__ M256 m_or(const M256 &a, const M256 &b)
{
    return M256{{a.w[0] | b.w[0], a.w[1] | b.w[1], a.w[2] | b.w[2], a.w[3] | b.w[3]}};
}
__device__ __forceinline__ M256 m_and(const M256 &a, const M256 &b)
{
    return M256{{a.w[0] & b.w[0], a.w[1] & b.w[1], a.w[2] & b.w[2], a.w[3] & b.w[3]}};
}
__device__ __forceinline__ M256 m_andn(const M256 &a, const M256 &b)
{
    return M256{{a.w[0] & ~b.w[0], a.w[1] & ~b.w[1], a.w[2] & ~b.w[2], a.w[3] & ~b.w[3]}};
}
__device__ __forceinline__ bool m_any(const M256 &a) { return (a.w[0] | a.w[1] | a.w[2] | a.w[3]) != 0ull; }
// word of member i, combined through masks so that the register array is
// never indexed (an indexed one would live in scratch memory)
__device__ __forceinline__ uint64_t m_word(const M256 &a, int i)
{
    const int k = i >> 6;
    return (a.w[0] & (0ull - (uint64_t)(k == 0))) | (a.w[1] & (0ull - (uint64_t)(k == 1))) |
           (a.w[2] & (0ull - (uint64_t)(k == 2))) | (a.w[3] & (0ull - (uint64_t)(k == 3)));
}
__device__ __forceinline__ bool m_has(const M256 &a, int i) { return ((m_word(a, i) >> (i & 63)) & 1ull) != 0ull; }
// ranks 0..n-1
__device__ __forceinline__ M256 m_prefix(int n)
{
    M256 r;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int c = n - 64 * k;
        r.w[k] = c >= 64 ? ~0ull : c <= 0 ? 0ull : (1ull << c) - 1ull;
    }
    return r;
}
__device__ __forceinline__ int m_popc(const M256 &a)
{
    return __popcll(a.w[0]) + __popcll(a.w[1]) + __popcll(a.w[2]) + __popcll(a.w[3]);
}
// lowest member (a must be non-empty)
__device__ __forceinline__ int m_low(const M256 &a)
{
#pragma unroll
    for (int k = 0; k < 4; k++)
        if (a.w[k]) return 64 * k + __builtin_ctzll(a.w[k]);
    return BIGN;
}
// members in increasing order: for (int r = m_first(S); r < BIGN; r = m_next(S, r))
__device__ __forceinline__ int m_next(const M256 &a, int r)
{
    const int q = r + 1;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int lo = 64 * k;
        if (q >= lo + 64) continue;
        const uint64_t v = q > lo ? a.w[k] & (~0ull << (q - lo)) : a.w[k];
        if (v) return lo + __builtin_ctzll(v);
    }
    return BIGN;
}
__device__ __forceinline__ int m_first(const M256 &a) { return m_any(a) ? m_low(a) : BIGN; }

// Per-set records (by deadline-monotonic rank) of a set of up to 256 tasks.
struct BigLDS {
    uint32_t T[BIGN], D[BIGN], clo[BIGN], chi[BIGN];
    uint32_t rm[BIGN], rs[BIGN];  // 32-bit multiplier and shift of T (floordiv31, response times)
    uint32_t Cs[BIGN], Cp[BIGN], k[BIGN];
    uint16_t mmin[BIGN];
    uint8_t orig[BIGN];
    M256 memmask;
    M256 forbid[BIGN];  // ACT: ranks whose two-task merge with this rank is invalid (Definition 3)
};

// Time of rank r on m units (conflict state conf) from the staged table.
__device__ __forceinline__ uint32_t big_time(const uint32_t *tc, int n, int r, int m, int conf)
{
    return tc[(m - 1) * 2 * n + conf * n + r];
}

__device__ __forceinline__ M256 big_conflicts(const M256 &S, const M256 &memm)
{
    const M256 mem = m_and(S, memm), cmp = m_andn(S, memm);
    M256 r = m_zero();
    if (m_popc(mem) >= 2) r = m_or(r, memm);
    if (m_popc(cmp) >= 2) r = m_or(r, M256{{~memm.w[0], ~memm.w[1], ~memm.w[2], ~memm.w[3]}});
    return r;
}

// Q32 utilisation of rank r on m units, exact modulo 2^64 also where C > T.
__device__ __forceinline__ uint64_t big_util(const BigLDS &L, const uint32_t *tc, int n, int r, int m, int conf)
{
    const uint32_t C = big_time(tc, n, r, m, conf), T = L.T[r];
    if (C <= T) return (uint64_t)util_q32_m1_magic(C, T, L.clo[r], L.chi[r]) + 1ull;
    uint64_t C64 = C;
    if (C >= C_SAT) {
        const uint64_t cn = (uint64_t)L.Cs[r] + ((uint64_t)L.Cp[r] + (uint64_t)m - 1ull) / (uint64_t)m;
        C64 = conf ? ((uint64_t)L.k[r] * cn + 999ull) / 1000ull : cn;
    }
    return ((C64 / T) << 32) + ((((C64 % T) << 32) + T - 1ull) / T);
}

__device__ __forceinline__ uint64_t big_group_util(const BigLDS &L, const uint32_t *tc, int n, const M256 &S, int m,
                                                   const M256 &cm)
{
    uint64_t u = 0;
    for (int r = m_first(S); r < BIGN; r = m_next(S, r)) u += big_util(L, tc, n, r, m, m_has(cm, r) ? 1 : 0);
    return u;
}

// Response time of rank r on m units under the members hp (all of higher DM
// priority), exact fixed point, 0 on a miss.  start: a lower bound of the
// fixed point (0, or the response time of the next higher-priority member
// plus C_r, below which the level-r demand exceeds the time).
template <typename TY>
__device__ __forceinline__ uint32_t big_rta(const BigLDS &L, const uint32_t *tc, int n, int r, const M256 &hp, int m, const M256 &cm,
                            TY &ty, uint64_t start = 0)
{
    const uint32_t Cr = big_time(tc, n, r, m, m_has(cm, r) ? 1 : 0), D = L.D[r];
    uint64_t R = Cr;
    for (int j = m_first(hp); j < BIGN; j = m_next(hp, j)) {
        const uint32_t Cj = big_time(tc, n, j, m, m_has(cm, j) ? 1 : 0);
        if (Cj >= L.T[j]) return 0u;  // a higher-priority utilisation of 1 or more leaves no time
        R += Cj;
    }
    if (R > D) return 0u;
    if (!m_any(hp)) return (uint32_t)R;
    if (start > R) R = start;
    if (R > D) return 0u;
    for (;;) {
        uint64_t W = Cr;
        uint32_t terms = 1u;
        const uint32_t x2 = ((uint32_t)R - 1u) << 1;  // R <= D < 2^31
        for (int j = m_first(hp); j < BIGN; j = m_next(hp, j)) {
            const uint32_t Cj = big_time(tc, n, j, m, m_has(cm, j) ? 1 : 0);
            W += ((uint64_t)floordiv31(x2, L.rm[j], L.rs[j]) + 1ull) * Cj;
            terms++;
        }
        ty.term(terms);
        if (W > D) return 0u;
        if (W == R) return (uint32_t)R;
        R = W;
    }
}

// Every member of S meets its deadline on m units (fixed priority, DM).
template <typename TY>
__device__ __forceinline__ bool big_test(const BigLDS &L, const uint32_t *tc, int n, const M256 &S, int m, const M256 &cm, TY &ty)
{
    ty.test();
    M256 hp = m_zero();
    uint64_t Rprev = 0;  // response time of the member before (0: none yet)
    for (int r = m_first(S); r < BIGN; r = m_next(S, r)) {
        const uint32_t R = big_rta(L, tc, n, r, hp, m, cm, ty,
                                   Rprev ? Rprev + big_time(tc, n, r, m, m_has(cm, r) ? 1 : 0) : 0);
        if (!R) return false;
        Rprev = R;
        hp = m_or(hp, m_bit(r));
    }
    return true;
}

// The same test with the whole block (all threads call it): thread r tests
// member r against the members above it, and the partition passes when every
// member does.  okf[par] collects the result; okf[par ^ 1] is made ready for
// the next call once every thread has read the previous call's result.
template <typename TY>
__device__ __forceinline__ bool coop_test(const BigLDS &L, const uint32_t *tc, int n, const M256 &S, int m,
                                          const M256 &cm, int *okf, int &par, TY &ty)
{
    const int t = threadIdx.x;
    __syncthreads();
    if (t == 0) {
        okf[par ^ 1] = 1;
        ty.test();
    }
    if (t < n && m_has(S, t) && !big_rta(L, tc, n, t, m_and(S, m_prefix(t)), m, cm, ty)) okf[par] = 0;
    __syncthreads();
    const bool r = okf[par] != 0;
    par ^= 1;
    return r;
}

// Operands of at least this many members take the block-wide tests under ">".
constexpr int LAZY_MIN = 32;

// ---------------------------------------------------------------------------
// prep for batches with sets of up to 256 tasks: validation, DM ranks, Lemma 1,
// Lemma 2; one block of 256 threads per set (thread i reads task i), records
// into w.rec by rank, as prep_kernel does for sets of at most 64 tasks.
__global__ __launch_bounds__(256) void prep_big_kernel(Batch b, Work w, Out o, Launch Lp)
{
    __shared__ uint32_t sD[BIGN], sT[BIGN];
    __shared__ int s_bad;
    __shared__ unsigned long long s_acc;
    const int64_t s = Lp.s0 + blockIdx.x;
    const int i = threadIdx.x;
    const int64_t off0 = b.off[s], off1 = b.off[s + 1];
    const int M = b.M[s];
    int status = CAPART_OK;
    if (off0 < 0 || off1 < off0 || off1 > b.n_tasks_total) status = CAPART_E_INVAL;
    const int64_t n64 = off1 - off0;
    if (status == CAPART_OK && (n64 < 1 || n64 > min(b.max_tasks, BIGN) || M < 1 || M > min(b.max_M, 127) ||
                                n64 * M > CAPART_ALG1_BIG_MAX_NM))
        status = CAPART_E_INVAL;
    const bool tab = b.Cn != nullptr;
    int64_t toff = 0;
    if (status == CAPART_OK && tab) {
        toff = b.toff[s];
        if (toff < 0 || toff > b.tlen - n64 * M || w.tCn == nullptr) status = CAPART_E_INVAL;
    }
    if (status != CAPART_OK) {
        if (i == 0) { o.status[s] = status; w.setflags[s] = 0u; }
        return;
    }
    const int n = (int)n64;
    if (i == 0) { s_bad = 0; s_acc = 0ull; }
    __syncthreads();
    int64_t T = 1, D = 1, Cs = 0, Cp = 1;
    int32_t kk = 1000;
    int ty = 0;
    uint16_t tmmin = MMIN_NONE;
    const int64_t L31 = (int64_t)1 << 31;
    if (i < n) {
        T = b.T[off0 + i];
        D = b.D[off0 + i];
        ty = b.type[off0 + i];
        bool bad = (T < 1 || T >= L31 || D < 1 || D > T || ty > 1);
        if (tab) {
            const int64_t *rn = b.Cn + toff + (int64_t)i * M, *rc = b.Cc + toff + (int64_t)i * M;
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
            Cs = b.Cs[off0 + i];
            Cp = b.Cp[off0 + i];
            kk = b.k[off0 + i];
            bad |= (Cs < 0 || Cp < 0 || Cs >= L31 || Cp >= L31 || Cs + Cp < 1 || Cs + Cp >= L31 || kk < 1000 ||
                    kk > 1000000);
        }
        if (bad) atomicOr(&s_bad, 1);
        sD[i] = (uint32_t)D;
        sT[i] = (uint32_t)T;
    }
    __syncthreads();
    if (s_bad) {
        if (i == 0) { o.status[s] = CAPART_E_RANGE; w.setflags[s] = 0u; }
        return;
    }
    if (i == 0) o.status[s] = CAPART_OK;
    int rank = 0;
    uint64_t l1 = 0;
    if (i < n) {
        for (int j = 0; j < n; j++)
            rank += (sD[j] < (uint32_t)D) || (sD[j] == (uint32_t)D && (sT[j] < (uint32_t)T ||
                                                                     (sT[j] == (uint32_t)T && j < i)));
        l1 = ((uint64_t)(Cs + Cp) << 32) / (uint64_t)T;  // floor-Q32 one-unit utilisation (Lemma 1)
        const uint64_t cap = ((uint64_t)M + 1ull) << 32;
        atomicAdd(&s_acc, (unsigned long long)min(l1, cap));
        TaskRec r;
        r.T = (uint32_t)T; r.D = (uint32_t)D; r.Cs = (uint32_t)Cs; r.Cp = (uint32_t)Cp; r.k = (uint32_t)kk;
        magic_u32((uint32_t)T, &r.clo, &r.chi);
        r.mmin = tab ? tmmin : m_min((uint32_t)Cs, (uint32_t)Cp, (uint32_t)D, (uint32_t)M);
        r.orig = (uint8_t)i;
        r.mem = (uint8_t)ty;
        w.rec[off0 + rank] = r;
    }
    __syncthreads();
    if (i == 0) {
        const bool reject = (s_acc > ((uint64_t)M << 32)) && !(Lp.flags & CAPART_FLAG_NO_LEMMA1);
        w.setflags[s] = SETF_VALID | (reject ? SETF_LEMMA1 : 0u);
    }
}

// ---------------------------------------------------------------------------
// The tables hold one block per compute unit (one wave per SIMD), so the
// kernel may take the whole register file rather than spill.
template <bool ACT, bool SMS, typename TY>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void alg1_big_kernel(Batch b, Work w, A1Out o, Launch Lp)
{
    __shared__ BigLDS L;
    // block communication
    __shared__ M256 s_Sc, s_Xc, s_X3, s_S3, s_fail, s_Pm[BIGN];
    __shared__ int s_c, s_bestl, s_cnt, s_mc, s_m3, s_mj, s_lead, s_ok, s_idj, s_lo, s_hi;
    __shared__ int s_okf[2];  // results of the block-wide tests, alternating
    __shared__ M256 s_cm3;
    __shared__ unsigned long long s_besta, s_U3, s_wl, s_tried;
    __shared__ uint64_t s_PU[BIGN];
    __shared__ M256 s_PX[BIGN];
    __shared__ int s_Pmu[BIGN], s_Pl[BIGN];
    const int64_t s = Lp.s0 + blockIdx.x;
    const int t = threadIdx.x;
    const uint32_t f = w.setflags[s];
    const int64_t off0 = b.off[s], off1 = b.off[s + 1];
    auto write_failure = [&](int64_t tried, int64_t merged) {
        if (t == 0) {
            o.verdict[s] = 0;
            o.nparts[s] = 0;
            o.tried[s] = tried;
            o.merged[s] = merged;
            if (o.workload) o.workload[s] = 0ull;
        }
        if (off0 >= 0 && off1 >= off0 && off1 <= b.n_tasks_total)
            for (int64_t i = off0 + t; i < off1; i += blockDim.x) { o.sizes[i] = 0; o.alloc[i] = -1; o.R[i] = -1; }
    };
    if (!(f & SETF_VALID)) { write_failure(0, 0); return; }
    const int n = (int)(off1 - off0);
    const int M = b.M[s];
    // records by rank and the [m][conflict][rank] execution-time table
    uint32_t *tc = capart_dyn_lds;
    if (t == 0) L.memmask = m_zero();
    __syncthreads();
    if (t < n) {
        const TaskRec r = w.rec[off0 + t];
        L.T[t] = r.T; L.D[t] = r.D; L.clo[t] = r.clo; L.chi[t] = r.chi;
        uint32_t rm, rs;
        magic31_of(r.T, r.clo, r.chi, &rm, &rs);
        L.rm[t] = rm; L.rs[t] = rs;
        L.Cs[t] = r.Cs; L.Cp[t] = r.Cp; L.k[t] = r.k;
        L.mmin[t] = r.mmin;
        L.orig[t] = r.orig;
        L.forbid[t] = m_zero();
        if (r.mem) atomicOr((unsigned long long *)&L.memmask.w[t >> 6], (unsigned long long)(1ull << (t & 63)));
    }
    __syncthreads();
    for (int e = t; e < n * M; e += blockDim.x) {
        const int m = e / n + 1, r = e - (m - 1) * n;
        uint32_t cn, cc;
        if (w.tCn) {
            const int64_t at = w.toff[s] + (int64_t)L.orig[r] * M + (m - 1);
            cn = (uint32_t)w.tCn[at];
            cc = (uint32_t)w.tCc[at];
        } else {
            cn = time_n(L.Cs[r], L.Cp[r], (uint32_t)m);
            cc = time_c(L.k[r], cn);
        }
        tc[(m - 1) * 2 * n + r] = cn;
        tc[(m - 1) * 2 * n + n + r] = cc;
    }
    __syncthreads();
    if (f & SETF_LEMMA1) { write_failure(0, 0); return; }
    const M256 memm = L.memmask;
    TY ty;
    // ACT: the pairs whose two-task merge is invalid (Definition 3): no size in
    // [max(mmin), min(mmin_a + mmin_b - 1, M)] schedules them; by monotonicity in
    // m the top of that range decides
    if (ACT) {
        const int npairs = n * (n - 1) / 2;
        NoTallyP<POL_FP> nt;
        for (int q = t; q < npairs; q += blockDim.x) {
            int bb = (int)((1.0f + sqrtf(1.0f + 8.0f * (float)q)) * 0.5f);
            while (bb * (bb - 1) / 2 > q) bb--;
            while ((bb + 1) * bb / 2 <= q) bb++;
            const int a = q - bb * (bb - 1) / 2;
            bool forb = true;
            if (L.mmin[a] != MMIN_NONE && L.mmin[bb] != MMIN_NONE) {
                const int m = min((int)L.mmin[a] + (int)L.mmin[bb] - 1, M);
                const M256 S2 = m_or(m_bit(a), m_bit(bb));
                forb = !big_test(L, tc, n, S2, m, big_conflicts(S2, memm), nt);
            }
            if (forb) {
                atomicOr((unsigned long long *)&L.forbid[a].w[bb >> 6], (unsigned long long)(1ull << (bb & 63)));
                atomicOr((unsigned long long *)&L.forbid[bb].w[a >> 6], (unsigned long long)(1ull << (a & 63)));
            }
        }
        __syncthreads();
    }
    // init partitions: one per task (partition id = rank), Lemma 2 size
    M256 Pm = m_zero(), PX = m_zero();
    uint64_t PU = 0;
    int Pmu = 0, Pl = t;
    if (t == 0) { s_ok = 1; s_cnt = 0; }
    __syncthreads();
    if (t < n) {
        const int m = (int)L.mmin[t];
        if (m > M) atomicAnd(&s_ok, 0);
        Pm = m_bit(t);
        PX = ACT ? L.forbid[t] : m_zero();
        Pmu = m > M ? 1 : m;
        PU = m > M ? 0ull : big_util(L, tc, n, t, m, 0);
        Pl = L.orig[t];
        atomicAdd(&s_cnt, Pmu);
    }
    __syncthreads();
    if (!s_ok) { write_failure(0, 0); return; }
    int Pi = s_cnt;
    // par_list order: decreasing U, ties by lowest task index
    {
        s_PU[t] = PU;
        s_Pl[t] = Pl;
        __syncthreads();
        int pos = t;
        if (t < n) {
            pos = 0;
            for (int j = 0; j < n; j++) pos += (s_PU[j] > PU || (s_PU[j] == PU && s_Pl[j] < Pl)) ? 1 : 0;
        }
        __syncthreads();
        s_Pm[pos] = Pm; s_PX[pos] = PX; s_PU[pos] = PU; s_Pmu[pos] = Pmu; s_Pl[pos] = Pl;
        __syncthreads();
        Pm = s_Pm[t]; PX = s_PX[t]; PU = s_PU[t]; Pmu = s_Pmu[t]; Pl = s_Pl[t];
        __syncthreads();
    }
    if (t == 0) s_okf[0] = 1;  // the first block-wide test's flag (others are set one test ahead)
    int par = 0;
    M256 live = m_prefix(n);  // ids of the partitions
    int np = n;
    int64_t tried = 0, merged = 0;
    bool ok = false;
    for (;;) {
        if (Pi <= M) { ok = true; break; }
        __syncthreads();  // every read of the previous iteration's block values is done
        const int idb_i = t < np ? m_low(Pm) : BIGN;  // this partition's id
        const M256 idb = t < np ? m_bit(idb_i) : m_zero();
        // the operand: the first partition in par_list order with an eligible partner
        if (t == 0) { s_c = BIGN; s_besta = ~0ull; s_bestl = BIGN; s_cnt = 0; s_tried = 0ull; s_fail = m_zero(); }
        __syncthreads();
        if (t < np && m_any(m_andn(m_andn(live, PX), idb))) atomicMin(&s_c, t);
        __syncthreads();
        const int c = s_c;
        if (c >= BIGN) break;  // no partition has an eligible partner: fail
        if (t == c) { s_Sc = Pm; s_Xc = PX; s_mc = Pmu; }
        __syncthreads();
        const M256 Sc = s_Sc, Xc = s_Xc;
        const int mc = s_mc;
        const int idc_i = m_low(Sc);
        const bool elig = t < np && t != c && !m_has(Xc, idb_i);
        bool mok = false;
        int m3 = 0;
        uint64_t U3 = 0, ka = ~0ull;
        M256 S3 = m_zero();
        bool counted = false, forbid = false;
        int best_l = BIGN;
        if (SMS || m_popc(Sc) < LAZY_MIN) {
            // every eligible partner's merge, one thread each; rank key (ka, t)
            if (elig) {
                S3 = m_or(Sc, Pm);
                const M256 cm = big_conflicts(S3, memm);
                const int mlo = max(mc, Pmu), mhi = min(mc + Pmu - 1, M);
                if (!SMS) ka = big_group_util(L, tc, n, S3, mlo, cm);
                if (mlo <= mhi && big_test(L, tc, n, S3, mhi, cm, ty)) {
                    int lo = mlo, hi = mhi;
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (big_test(L, tc, n, S3, mid, cm, ty))
                            hi = mid;
                        else
                            lo = mid + 1;
                    }
                    mok = true;
                    m3 = lo;
                    U3 = big_group_util(L, tc, n, S3, lo, cm);
                }
                if (SMS && mok) ka = ((uint64_t)m3 << 44) | U3;  // U3 <= 256 * 2^32: every member meets D <= T
            }
            if (mok) atomicMin(&s_besta, (unsigned long long)ka);
            __syncthreads();
            const uint64_t best_a = s_besta;
            if (mok && ka == best_a) atomicMin(&s_bestl, t);
            __syncthreads();
            best_l = s_bestl;
            const bool before = ka < best_a || (ka == best_a && t < best_l);
            // failed merges that forbid their pairs: for ">" those ranked before the
            // merge taken (all of them if none is valid), for ">>" all of them
            forbid = elig && !mok && (SMS || before);
            counted = elig && (SMS || before || t == best_l);
        } else {
            // ">" with a large operand: the partners are ranked by (ka, t) as
            // above, then tried in that order, each merge's tests spread over
            // the union's members (a thread per member), until one is valid;
            // the same merges are tried, taken and forbidden as above
            M256 cm = m_zero();
            int mlo = 0, mhi = 0;
            if (elig) {
                S3 = m_or(Sc, Pm);
                cm = big_conflicts(S3, memm);
                mlo = max(mc, Pmu);
                mhi = min(mc + Pmu - 1, M);
                ka = big_group_util(L, tc, n, S3, mlo, cm);
            }
            bool pend = elig;
            for (;;) {
                if (t == 0) { s_besta = ~0ull; s_bestl = BIGN; }
                __syncthreads();
                if (pend) atomicMin(&s_besta, (unsigned long long)ka);
                __syncthreads();
                if (pend && ka == s_besta) atomicMin(&s_bestl, t);
                __syncthreads();
                const int x = s_bestl;
                if (x >= BIGN) break;  // every eligible merge failed
                if (t == x) { s_S3 = S3; s_cm3 = cm; s_lo = mlo; s_hi = mhi; pend = false; counted = true; }
                __syncthreads();
                const M256 Sx = s_S3, cx = s_cm3;
                int lo = s_lo, hi = s_hi;
                const bool okx = lo <= hi && coop_test(L, tc, n, Sx, hi, cx, s_okf, par, ty);
                if (okx) {
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (coop_test(L, tc, n, Sx, mid, cx, s_okf, par, ty))
                            hi = mid;
                        else
                            lo = mid + 1;
                    }
                }
                if (t == x) {
                    if (okx) {
                        mok = true;
                        m3 = lo;
                        U3 = big_group_util(L, tc, n, S3, lo, cm);
                    } else {
                        forbid = true;
                    }
                }
                if (okx) { best_l = x; break; }
            }
        }
        if (counted) atomicAdd(&s_tried, 1ull);
        if (forbid) {
            PX = m_or(PX, m_bit(idc_i));
            atomicOr((unsigned long long *)&s_fail.w[idb_i >> 6], (unsigned long long)(1ull << (idb_i & 63)));
        }
        __syncthreads();
        tried += (int64_t)s_tried;
        if (t == c) PX = m_or(PX, s_fail);
        if (best_l >= BIGN) continue;  // P_c has no valid merge; its partners are now forbidden
        // merge P_c with partner j: par_list minus both, plus the union (which
        // keeps the smaller id; the other id is relabelled in every set)
        const int j = best_l;
        if (t == j) { s_S3 = S3; s_U3 = U3; s_m3 = m3; s_mj = Pmu; s_X3 = PX; s_lead = Pl; s_idj = idb_i; }
        __syncthreads();
        if (t == c) { s_X3 = m_or(s_X3, PX); s_lead = min(s_lead, Pl); }
        __syncthreads();
        const M256 Sj3 = s_S3;
        const uint64_t Uj3 = s_U3;
        const int mj3 = s_m3, mj = s_mj, lead = s_lead;
        const int idj_i = s_idj;
        const int keep = min(idc_i, idj_i), gone = max(idc_i, idj_i);
        const bool rem = t < np && t != c && t != j;
        const bool bnew = rem && (PU > Uj3 || (PU == Uj3 && Pl < lead));
        if (t == 0) s_cnt = 0;
        __syncthreads();
        if (bnew) atomicAdd(&s_cnt, 1);
        __syncthreads();
        const int pos_new = s_cnt;
        const int r = t - (t > c ? 1 : 0) - (t > j ? 1 : 0);
        int dst = t;
        if (rem) {
            dst = r + (r >= pos_new ? 1 : 0);
        } else if (t == c) {
            dst = pos_new;
            Pm = Sj3; PX = s_X3; PU = Uj3; Pmu = mj3; Pl = lead;
        } else if (t == j) {
            dst = np - 1;
        }
        if (m_has(PX, gone)) PX = m_or(m_andn(PX, m_bit(gone)), m_bit(keep));
        __syncthreads();
        s_Pm[dst] = Pm; s_PX[dst] = PX; s_PU[dst] = PU; s_Pmu[dst] = Pmu; s_Pl[dst] = Pl;
        __syncthreads();
        Pm = s_Pm[t]; PX = s_PX[t]; PU = s_PU[t]; Pmu = s_Pmu[t]; Pl = s_Pl[t];
        live = m_andn(live, m_bit(gone));
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
        if ((t & 63) == 0 && w.counters) {
            atomicAdd((unsigned long long *)&w.counters[0], (unsigned long long)a);
            atomicAdd((unsigned long long *)&w.counters[1], (unsigned long long)bb);
        }
    }
    if (!ok) { write_failure(tried, merged); return; }
    if (t == 0) {
        o.verdict[s] = 1;
        o.nparts[s] = np;
        o.tried[s] = tried;
        o.merged[s] = merged;
        s_wl = 0ull;
    }
    if (t < n) o.sizes[off0 + t] = t < np ? Pmu : 0;
    s_Pm[t] = Pm;
    s_Pmu[t] = Pmu;
    __syncthreads();
    // each task's partition, then its response time there and its workload term
    if (t < n) {
        int part = 0;
        for (int p = 0; p < np; p++)
            if (m_has(s_Pm[p], t)) part = p;
        const M256 Sp = s_Pm[part];
        const M256 cm = big_conflicts(Sp, memm);
        M256 hp = m_zero();
        for (int q = m_first(Sp); q < t; q = m_next(Sp, q)) hp = m_or(hp, m_bit(q));
        NoTallyP<POL_FP> nt;
        const uint32_t R = big_rta(L, tc, n, t, hp, s_Pmu[part], cm, nt);
        const int64_t gi = off0 + L.orig[t];
        o.alloc[gi] = (int8_t)part;
        o.R[gi] = R ? (int64_t)R : -1;
        atomicAdd(&s_wl, (unsigned long long)big_util(L, tc, n, t, 1, m_has(cm, t) ? 1 : 0));
    }
    __syncthreads();
    if (t == 0 && o.workload) o.workload[s] = s_wl;
}

}  // namespace capart
