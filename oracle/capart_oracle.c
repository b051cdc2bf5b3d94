/*
 * capart_oracle.c -- plain, slow, obviously-correct CPU oracle for
 * contention-aware GPU partitioning and task-to-partition allocation
 * (Zahaf et al., arXiv 2105.10312).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the HIP engine; it is written directly
 * from the paper's definitions, in the paper's order, with no blocking,
 * fusion or reordering.  All arithmetic is integer; intermediate products
 * are carried in 128 bits so that no overflow argument is needed here.
 *
 * What is computed, per task set (n tasks, M compute units, at most K parts):
 *   1. execution times (Section "Modeling kernel execution times" and the
 *      scaling function of Section "Task set generation"):
 *        Cn(m) = C_seq + ceil(C_par / m)          no conflict
 *        Cc(m) = ceil(k * Cn(m) / 1000)            conflict (k per-mille)
 *   2. conflict (Section "Task Model"): a task is in conflict iff at least one
 *      OTHER task of the same type (memory / compute) shares its partition;
 *      its execution time is Cc then, Cn otherwise;
 *   3. per-partition test (Section "Schedulability test": any policy with an
 *      exact test; interference folded into the execution times): each
 *      partition is one server running its tasks one at a time on all its
 *      compute units, preemptive fixed priority, deadline-monotonic order by
 *      (D, T, index), exact response-time fixed point
 *        R = C_i + sum_{j in hp(i)} ceil(R / T_j) * C_j ,  R <= D_i;
 *      or, with OR_FLAG_EDF, preemptive EDF on the same server: the
 *      processor-demand criterion below the synchronous busy period, with
 *      the density bound and the work limits stated at or_edf_part;
 *   4. Lemma 1 (necessary test): sum_i Cn_i(1)/T_i > M => unschedulable,
 *      evaluated as floor-Q32 utilisations so the rejection is sound;
 *   5. Lemma 2: smallest partition for one task, m_min = min{m : Cn(m) <= D};
 *   6. partitionings: integer partitions of M into at most K positive parts,
 *      non-increasing, listed in descending lexicographic order;
 *   7. allocation: exhaustive (all k^n maps, index = base-k digits with task
 *      0 most significant) or the heuristic H(pi) below;
 *   8. partition utilisation U(P) = sum ceil(C_i * 2^32 / T_i) (Q32, the
 *      order relation ">" of Definition 5); the best feasible triple minimises
 *      (max_p U_p, sum_p U_p, partitioning index, allocation index);
 *   9. the whole-GPU baseline ("1G"): every task on one partition of M.
 *
 * H(pi), the paper's heuristic ingredients applied to fixed partition sizes:
 * tasks in decreasing one-unit utilisation (Algorithm 1's ordered list),
 * each placed on the candidate partition that stays schedulable and ranks
 * best, by ">" (lower merged utilisation, Definition 5, "BF") or by ">>"
 * (fewer compute units needed by the merged partition, Definition 4 with the
 * search of Algorithm 2, "SMS"); with ACT, task pairs whose two-task merge is
 * invalid (Definition 3 / Algorithm 2) are forbidden to share a partition
 * (Section "Forbidden list").  Ties fall to the lower partition index.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

typedef __int128 i128;
typedef unsigned __int128 u128;

enum { OR_EXH = 0, OR_BF_INA = 1, OR_BF_ACT = 2, OR_SMS_INA = 3, OR_SMS_ACT = 4 };
enum { OR_OK = 0, OR_E_INVAL = -1, OR_E_RANGE = -2 };
#define OR_FLAG_NO_LEMMA1 1
#define OR_FLAG_EDF 2     /* per-partition policy: EDF instead of fixed-priority DM */
#define OR_FLAG_EXH_FAST 4 /* exhaustive mode through the memo of partition tests (or_exh_memo) */
/* EDF work limits (part of the test's definition, identical in the engine):
 * busy-period iterations before the utilisation bound is used instead, and
 * absolute deadlines below the horizon beyond which the exact demand check
 * gives way to the sufficient fixed-priority test */
#define OR_EDF_BP_STEPS 4096
#define OR_EDF_ND_CAP 65536
#define OR_MAXN 256       /* task capacity of the arrays (Algorithm 1 takes up to 256 tasks) */
#define OR_MAXN_FIXED 64  /* largest set of the fixed-partitioning search */
#define OR_MINF 1000000 /* "no such m" for Lemma 2 */

typedef struct {
    int64_t terms;   /* response-time terms: seed + each ceil(R/T_j)*C_j */
    int64_t tests;   /* partition schedulability tests                   */
    int64_t combines;/* exhaustive allocations examined                  */
} or_counters;

typedef struct {
    int n, M;
    const int64_t *T, *D, *Cs, *Cp;
    const int32_t *k;
    const uint8_t *type;
    /* explicit time tables (NULL: the parametric model from Cs, Cp, k):
     * task i's time on m units at [i*M + m-1], without and in conflict */
    const int64_t *Cn_tab, *Cc_tab;
    /* admissible partition sizes: bit m of the 256-bit mask (NULL: every size) */
    const uint64_t *adm;
    int edf;         /* 1: every partition is scheduled by EDF, 0: fixed-priority DM */
    or_counters *cnt;
} or_set;

/* ---- 1. execution times ------------------------------------------------ */
static int64_t or_cn(const or_set *s, int i, int m)
{
    if (s->Cn_tab) return s->Cn_tab[(int64_t)i * s->M + m - 1];
    return s->Cs[i] + (s->Cp[i] + m - 1) / m;
}

static int64_t or_cc(const or_set *s, int i, int m)
{
    i128 x;
    if (s->Cc_tab) return s->Cc_tab[(int64_t)i * s->M + m - 1];
    x = (i128)s->k[i] * (i128)or_cn(s, i, m);
    return (int64_t)((x + 999) / 1000);
}

int64_t or_time(const int64_t *Cs, const int64_t *Cp, const int32_t *k, int i, int m, int conflict)
{
    or_set s = {0};
    s.Cs = Cs; s.Cp = Cp; s.k = k;
    return conflict ? or_cc(&s, i, m) : or_cn(&s, i, m);
}

/* ---- 3. fixed priority: exact response times in DM order ------------- */
/* order[0..cnt) lists positions in mem[] by deadline-monotonic priority.
 * R_out (indexed by task) gets the response time or -1; with early_exit the
 * test stops at the first miss (the rest of R_out is left untouched).
 * Returns 1 iff every task meets its deadline. */
static int or_fp_part(const or_set *s, const int *mem, int cnt, const int64_t *C, const int *order, int early_exit,
                      int64_t *R_out)
{
    int t, u, feasible = 1;
    for (t = 0; t < cnt; t++) {
        int pi = order[t], i = mem[pi];
        i128 R = C[pi], W;
        int ok = 0;
        for (;;) {
            W = C[pi];
            if (s->cnt) s->cnt->terms++;
            for (u = 0; u < t; u++) {
                int pj = order[u], j = mem[pj];
                i128 q = (R + s->T[j] - 1) / s->T[j];
                W += q * C[pj];
                if (s->cnt) s->cnt->terms++;
            }
            if (W > s->D[i]) { ok = 0; break; }
            if (W == R) { ok = 1; break; }
            R = W;
        }
        if (R_out) R_out[i] = ok ? (int64_t)R : -1;
        if (!ok) {
            feasible = 0;
            if (early_exit) return 0;
        }
    }
    return feasible;
}

/* ---- 3'. one partition under preemptive EDF ---------------------------- */
/* Processor-demand criterion for constrained-deadline sporadic tasks on one
 * server (Baruah, Rosier and Howell 1990): with total utilisation U <= 1, the
 * partition is schedulable iff at every absolute deadline d below the
 * synchronous busy period L the demand
 *     h(d) = sum_{j : D_j <= d} (floor((d - D_j) / T_j) + 1) * C_j
 * is at most d.  Checking deadlines beyond L changes nothing, so any horizon
 * H >= L gives the same answer.  Integer definition used here, in order:
 *   1. floor-Q32 sum of C_j 2^32 / T_j above 2^32: U > 1, unschedulable;
 *   2. ceil-Q32 density sum of C_j 2^32 / D_j at most 2^32: density at most 1,
 *      which is sufficient for EDF (h(t) <= t at every t), schedulable;
 *   3. the horizon: L = least fixed point of w = sum ceil(w / T_j) C_j,
 *      iterated from sum C_j; if it has not settled after OR_EDF_BP_STEPS
 *      iterations, H is the bound L <= sum C / (1 - U) taken with the ceil-Q32
 *      utilisation Uq (H = ceil(sum C 2^32 / (2^32 - Uq)), needs Uq < 2^32),
 *      else H is undetermined;
 *   4. H determined and at most OR_EDF_ND_CAP absolute deadlines below it:
 *      schedulable iff h(d) <= d at every absolute deadline d < H (exact);
 *   5. otherwise (a work limit reached): schedulable iff every member passes
 *      the fixed-priority deadline-monotonic response-time test.  That is
 *      sufficient for EDF (EDF is optimal on one preemptive server, so a set
 *      that DM schedules, EDF schedules), so the answer is never optimistic
 *      and EDF verdicts always dominate fixed-priority ones.
 * Every job of a schedulable partition completes within its deadline and
 * within the longest (synchronous) busy period, so the response time reported
 * for each member is min(D_i, H) where H is determined, D_i where it is not;
 * -1 for every member of an unschedulable partition.  *U = the ceil-Q32 sum. */
static int or_cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

static int or_edf_part(const or_set *s, const int *mem, int cnt, const int64_t *C, const int *order,
                       int64_t *R_out, uint64_t *U)
{
    const u128 one = (u128)1 << 32;
    u128 uf = 0, uc = 0, dc = 0;
    i128 sumC = 0, w, H = 0;
    int64_t nd = 0, *dl = NULL;
    int a, j, step, settled = 0, have_h = 0, feasible = 0, decided = 0;
    for (a = 0; a < cnt; a++) {
        u128 num = ((u128)C[a]) << 32, den = (u128)s->T[mem[a]], dd = (u128)s->D[mem[a]];
        uf += num / den;
        uc += (num + den - 1) / den;
        dc += (num + dd - 1) / dd;
        sumC += C[a];
    }
    if (uf > one) goto done; /* 1 */
    if (dc <= one) { feasible = 1; decided = 1; } /* 2 */
    /* 3: the synchronous busy period */
    w = sumC;
    for (step = 0; step < OR_EDF_BP_STEPS; step++) {
        i128 W = 0;
        for (a = 0; a < cnt; a++) {
            W += ((w + s->T[mem[a]] - 1) / s->T[mem[a]]) * C[a];
            if (s->cnt) s->cnt->terms++;
        }
        if (W == w) { settled = 1; break; }
        w = W;
    }
    if (settled) {
        H = w;
        have_h = 1;
    } else if (uc < one) {
        u128 den = one - uc;
        H = (i128)((((u128)sumC << 32) + den - 1) / den);
        have_h = 1;
    }
    if (decided) goto done;
    /* 4: the absolute deadlines below H, if there are not too many */
    if (have_h) {
        i128 cntd = 0;
        for (a = 0; a < cnt && cntd <= OR_EDF_ND_CAP; a++) {
            i128 D = s->D[mem[a]];
            if (D < H) cntd += (H - 1 - D) / s->T[mem[a]] + 1;
        }
        nd = cntd > OR_EDF_ND_CAP ? OR_EDF_ND_CAP + 1 : (int64_t)cntd;
    }
    if (!have_h || nd > OR_EDF_ND_CAP) {
        feasible = or_fp_part(s, mem, cnt, C, order, 1, NULL); /* 5 */
        goto done;
    }
    dl = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nd > 0 ? nd : 1));
    nd = 0;
    for (a = 0; a < cnt; a++)
        for (w = s->D[mem[a]]; w < H; w += s->T[mem[a]]) dl[nd++] = (int64_t)w;
    qsort(dl, (size_t)nd, sizeof(int64_t), or_cmp_i64);
    /* the demand at each of them, in increasing order */
    feasible = 1;
    for (j = 0; j < nd && feasible; j++) {
        i128 d = dl[j], h = 0;
        for (a = 0; a < cnt; a++) {
            int64_t D = s->D[mem[a]];
            if (D <= d) h += ((d - D) / s->T[mem[a]] + 1) * C[a];
            if (s->cnt) s->cnt->terms++;
        }
        if (h > d) feasible = 0;
    }
    free(dl);
done:
    if (R_out)
        for (a = 0; a < cnt; a++) {
            int64_t D = s->D[mem[a]];
            R_out[mem[a]] = feasible ? ((have_h && H < D) ? (int64_t)H : D) : -1;
        }
    if (feasible && U) *U = (uint64_t)uc;
    return feasible;
}

/* ---- 2+3. one partition: conflicts, DM order, the policy's test -------- */
/* mem[0..cnt) are task indices.  R_out (indexed by task) gets the response
 * time or -1; with early_exit a fixed-priority test stops at the first miss
 * (the rest of R_out is left untouched).  Returns 1 iff every task meets its
 * deadline and then *U = sum ceil(C_i 2^32 / T_i). */
static int or_eval_part(const or_set *s, const int *mem, int cnt, int m, int early_exit,
                        int64_t *R_out, uint64_t *U)
{
    int order[OR_MAXN];
    int64_t C[OR_MAXN];
    int a, b;
    int feasible;
    if (s->cnt) s->cnt->tests++;
    for (a = 0; a < cnt; a++) {
        int same = 0;
        for (b = 0; b < cnt; b++)
            if (s->type[mem[b]] == s->type[mem[a]]) same++;
        /* "same" counts the task itself: a conflict needs one other task */
        C[a] = (same >= 2) ? or_cc(s, mem[a], m) : or_cn(s, mem[a], m);
        order[a] = a;
    }
    /* deadline-monotonic priority: (D, T, index) ascending; insertion sort */
    for (a = 1; a < cnt; a++) {
        int x = order[a];
        b = a - 1;
        while (b >= 0) {
            int y = order[b];
            int64_t dx = s->D[mem[x]], dy = s->D[mem[y]];
            int64_t tx = s->T[mem[x]], ty = s->T[mem[y]];
            int later = (dy > dx) || (dy == dx && (ty > tx || (ty == tx && mem[y] > mem[x])));
            if (!later) break;
            order[b + 1] = y;
            b--;
        }
        order[b + 1] = x;
    }
    if (s->edf) return or_edf_part(s, mem, cnt, C, order, R_out, U);
    feasible = or_fp_part(s, mem, cnt, C, order, early_exit, R_out);
    if (feasible && U) {
        u128 acc = 0;
        for (a = 0; a < cnt; a++) {
            u128 num = ((u128)C[a]) << 32;
            u128 den = (u128)s->T[mem[a]];
            acc += (num + den - 1) / den;
        }
        *U = (uint64_t)acc;
    }
    return feasible;
}

/* ---- a whole triple (partitioning, allocation) -------------------------- */
static int or_eval_triple(const or_set *s, const int *sizes, int k, const int8_t *alloc,
                          int early_exit, int64_t *R_out, uint64_t *maxU, uint64_t *sumU)
{
    int mem[OR_MAXN];
    int p, i, feasible = 1;
    uint64_t mx = 0, sm = 0;
    for (p = 0; p < k; p++) {
        int cnt = 0;
        uint64_t U = 0;
        for (i = 0; i < s->n; i++)
            if (alloc[i] == p) mem[cnt++] = i;
        if (cnt == 0) continue; /* an empty partition is trivially schedulable, U = 0 */
        if (!or_eval_part(s, mem, cnt, sizes[p], early_exit, R_out, &U)) {
            feasible = 0;
            if (early_exit) return 0;
            continue;
        }
        if (U > mx) mx = U;
        sm += U;
    }
    if (feasible) {
        if (maxU) *maxU = mx;
        if (sumU) *sumU = sm;
    }
    return feasible;
}

/* ---- 4. Lemma 1 ---------------------------------------------------------- */
static int or_lemma1_reject(const or_set *s)
{
    u128 acc = 0;
    int i;
    for (i = 0; i < s->n; i++)
        acc += (((u128)or_cn(s, i, 1)) << 32) / (u128)s->T[i];
    return acc > (((u128)s->M) << 32);
}

/* ---- 5. Lemma 2 (linear scan, as stated) ------------------------------- */
static int or_m_min(const or_set *s, int i)
{
    int m;
    for (m = 1; m <= s->M; m++)
        if (or_cn(s, i, m) - s->D[i] <= 0) return m;
    return OR_MINF;
}

/* ---- 6. integer partitions of M into <= K parts, descending lex ------- */
typedef struct {
    int64_t count, want;
    int *out;      /* if non-NULL: write K sizes per partitioning (0-padded) */
    int64_t cap;
    int K;
    int cur[16];
} or_enum_ctx;

static void or_enum_rec(or_enum_ctx *c, int rem, int maxpart, int depth)
{
    int x, j;
    if (rem == 0) {
        if (c->out && c->count < c->cap) {
            for (j = 0; j < c->K; j++) c->out[c->count * c->K + j] = j < depth ? c->cur[j] : 0;
        }
        c->count++;
        return;
    }
    if (depth == c->K) return;
    for (x = (rem < maxpart ? rem : maxpart); x >= 1; x--) {
        if ((int64_t)x * (c->K - depth) < rem) break; /* cannot fill with parts <= x */
        c->cur[depth] = x;
        or_enum_rec(c, rem - x, x, depth + 1);
    }
}

int64_t or_count_partitionings(int M, int K)
{
    or_enum_ctx c;
    memset(&c, 0, sizeof c);
    if (M < 1 || K < 1 || K > 16) return 0;
    c.K = K;
    or_enum_rec(&c, M, M, 0);
    return c.count;
}

int64_t or_enumerate_partitionings(int M, int K, int *out, int64_t cap)
{
    or_enum_ctx c;
    memset(&c, 0, sizeof c);
    if (M < 1 || K < 1 || K > 16) return 0;
    c.K = K; c.out = out; c.cap = cap;
    or_enum_rec(&c, M, M, 0);
    return c.count;
}

/* ---- 7b. the heuristic H(pi) -------------------------------------------- */
static uint64_t or_u1(const or_set *s, int i)
{
    u128 num = ((u128)or_cn(s, i, 1)) << 32, den = (u128)s->T[i];
    return (uint64_t)((num + den - 1) / den);
}

/* forbidden pair (ACT): no valid two-task merge (Definition 3, Algorithm 2) */
static int or_forbidden(const or_set *s, int i, int j, const int *mm)
{
    int mem[2], m, lo, hi;
    if (mm[i] >= OR_MINF || mm[j] >= OR_MINF) return 1;
    mem[0] = i; mem[1] = j;
    lo = mm[i] > mm[j] ? mm[i] : mm[j];
    hi = mm[i] + mm[j] - 1;
    if (hi > s->M) hi = s->M;
    for (m = lo; m <= hi; m++)
        if (or_eval_part(s, mem, 2, m, 1, NULL, NULL)) return 0;
    return 1;
}

static int or_heuristic(const or_set *s, const int *sizes, int k, int variant, int8_t *alloc)
{
    int n = s->n, i, t, p, a, b;
    int mm[OR_MAXN], sigma[OR_MAXN];
    uint64_t u1[OR_MAXN];
    int members[8][OR_MAXN];
    int nmem[8];
    int act = (variant == OR_BF_ACT || variant == OR_SMS_ACT);
    int sms = (variant == OR_SMS_INA || variant == OR_SMS_ACT);
    static const int none = -1;
    (void)none;

    for (i = 0; i < n; i++) {
        mm[i] = or_m_min(s, i);
        u1[i] = or_u1(s, i);
        sigma[i] = i;
        alloc[i] = -1;
    }
    /* decreasing one-unit utilisation, ties by index */
    for (a = 1; a < n; a++) {
        int x = sigma[a];
        b = a - 1;
        while (b >= 0 && (u1[sigma[b]] < u1[x] || (u1[sigma[b]] == u1[x] && sigma[b] > x))) {
            sigma[b + 1] = sigma[b];
            b--;
        }
        sigma[b + 1] = x;
    }
    for (p = 0; p < k; p++) nmem[p] = 0;
    for (t = 0; t < n; t++) {
        int tau = sigma[t];
        int best_p = -1;
        uint64_t best_U = 0;
        int best_req = 0;
        for (p = 0; p < k; p++) {
            int cand[OR_MAXN], c = nmem[p], q, feas, req = 0;
            uint64_t U = 0;
            if (mm[tau] > sizes[p]) continue;
            if (act) {
                int bad = 0;
                for (q = 0; q < nmem[p]; q++)
                    if (or_forbidden(s, tau, members[p][q], mm)) { bad = 1; break; }
                if (bad) continue;
            }
            memcpy(cand, members[p], sizeof(int) * (size_t)c);
            cand[c++] = tau;
            feas = or_eval_part(s, cand, c, sizes[p], 1, NULL, &U);
            if (!feas) continue;
            if (sms) {
                int m;
                for (m = 1; m <= sizes[p]; m++)
                    if (or_eval_part(s, cand, c, m, 1, NULL, NULL)) { req = m; break; }
            }
            if (best_p < 0) {
                best_p = p; best_U = U; best_req = req;
            } else if (sms) {
                if (req < best_req || (req == best_req && U < best_U)) {
                    best_p = p; best_U = U; best_req = req;
                }
            } else if (U < best_U) {
                best_p = p; best_U = U;
            }
        }
        if (best_p < 0) {
            for (i = 0; i < n; i++) alloc[i] = -1;
            return 0;
        }
        members[best_p][nmem[best_p]++] = tau;
        alloc[tau] = (int8_t)best_p;
    }
    return 1;
}

/* ---- validation (the boundary's input contract) ------------------------- */
static int or_validate(const or_set *s, int K, int mode)
{
    int i;
    if (s->n < 1 || s->n > OR_MAXN_FIXED || s->M < 1 || s->M > 255) return OR_E_INVAL;
    if (s->n * s->M > 8192) return OR_E_INVAL; /* the boundary's per-set size limit */
    for (i = 0; i < s->n; i++) {
        int64_t T = s->T[i], D = s->D[i];
        if (T < 1 || T >= ((int64_t)1 << 31)) return OR_E_RANGE;
        if (D < 1 || D > T) return OR_E_RANGE;
        if (s->type[i] > 1) return OR_E_RANGE;
        if (s->Cn_tab) {
            /* explicit tables: times in [1, 2^31), never rising with m, a
             * conflict never faster, and no super-linear speed-up
             * (m Cn(m) >= Cn(1), which keeps Lemma 1 sound) */
            int m;
            for (m = 1; m <= s->M; m++) {
                int64_t cn = or_cn(s, i, m), cc = or_cc(s, i, m);
                if (cn < 1 || cn >= ((int64_t)1 << 31) || cc < 1 || cc >= ((int64_t)1 << 31)) return OR_E_RANGE;
                if (cc < cn) return OR_E_RANGE;
                if (m > 1 && (cn > or_cn(s, i, m - 1) || cc > or_cc(s, i, m - 1))) return OR_E_RANGE;
                if ((i128)m * cn < (i128)or_cn(s, i, 1)) return OR_E_RANGE;
            }
        } else {
            int64_t a = s->Cs[i], b = s->Cp[i];
            if (a < 0 || b < 0 || a >= ((int64_t)1 << 31) || b >= ((int64_t)1 << 31)) return OR_E_RANGE;
            if (a + b < 1 || a + b >= ((int64_t)1 << 31)) return OR_E_RANGE;
            if (s->k[i] < 1000 || s->k[i] > 1000000) return OR_E_RANGE;
        }
    }
    if (mode == OR_EXH) {
        int kk = K < s->M ? K : s->M;
        u128 pw = 1;
        for (i = 0; i < s->n; i++) {
            pw *= (u128)kk;
            if (pw >= ((u128)1 << 62)) return OR_E_INVAL;
        }
    }
    return OR_OK;
}

/* ---- one set ----------------------------------------------------------- */
/* ---- 7'. exhaustive allocation through a memo of partition tests ------- */
/* The same search as step 7 over every allocation, with each partition's
 * test memoised: U[m-1][A] for every task subset A (bit i = task i) and size
 * m = 1..M, filled by or_eval_part (an empty part is schedulable with U = 0;
 * an unschedulable subset holds OR_MEMO_NONE, above any schedulable U, which
 * is at most 2^32 + n).  Every allocation index of every partitioning is
 * then scored from the memo in increasing index order, so the result (best
 * key (maxU, sumU, partitioning index, allocation index)) is the plain
 * search's by construction; tests/test_oracle_fast.py checks it against the
 * plain search.  Sets of at most OR_FAST_MAXN tasks. */
#define OR_FAST_MAXN 16

#define OR_MEMO_NONE (~(uint64_t)0)

typedef struct {
    int n, M;
    uint64_t *U;  /* [M][2^n] */
} or_memo;

static int or_memo_build(const or_set *s, or_memo *mo)
{
    const int64_t W = (int64_t)1 << s->n;
    int64_t A;
    int m, i;
    mo->n = s->n; mo->M = s->M;
    mo->U = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(W * s->M));
    if (!mo->U) return 0;
    for (m = 1; m <= s->M; m++)
        for (A = 0; A < W; A++) {
            int mem[OR_MAXN], cnt = 0;
            uint64_t U = 0;
            for (i = 0; i < s->n; i++)
                if ((A >> i) & 1) mem[cnt++] = i;
            if (cnt > 0 && !or_eval_part(s, mem, cnt, m, 1, NULL, &U)) U = OR_MEMO_NONE;
            mo->U[(m - 1) * W + A] = U;
        }
    return 1;
}

/* Score every allocation of partitioning sz[0..k) (task 0 the most
 * significant base-k digit); keeps the best (maxU, sumU) seen so far, which
 * a later index replaces only when strictly smaller.  The indices are taken
 * in runs of k that differ only in the last task's part d: the other parts'
 * memo entries are read once per run. */
static void or_memo_scan(const or_set *s, const or_memo *mo, const int *sz, int k, int64_t pidx, int *found,
                         uint64_t *best_max, uint64_t *best_sum, int64_t *best_pidx, int64_t *best_aidx,
                         int8_t *best_alloc)
{
    const int n = s->n, last = n - 1;
    const int64_t W = (int64_t)1 << n;
    const uint32_t lbit = 1u << last;
    int digit[OR_MAXN];
    uint32_t mask[8];
    uint64_t u0[8], u1[8];
    int64_t r, runs = 1;
    int i, p, d;
    for (i = 0; i < last; i++) { digit[i] = 0; runs *= k; }
    for (p = 0; p < k; p++) mask[p] = 0;
    mask[0] = (uint32_t)(W - 1) & ~lbit;
    for (r = 0; r < runs; r++) {
        int bad = 0, badp = -1;
        for (p = 0; p < k; p++) {
            const uint64_t *row = mo->U + (int64_t)(sz[p] - 1) * W;
            u0[p] = row[mask[p]];          /* part p without the last task */
            u1[p] = row[mask[p] | lbit];   /* part p with it */
            if (u0[p] == OR_MEMO_NONE) { bad++; badp = p; }
        }
        for (d = 0; d < k; d++) {
            uint64_t mx = 0, sm = 0;
            if (s->cnt) s->cnt->combines++;
            /* parts other than d must be schedulable as they are, part d with the last task */
            if (bad > 1 || (bad == 1 && badp != d) || u1[d] == OR_MEMO_NONE) continue;
            for (p = 0; p < k; p++) {
                const uint64_t u = p == d ? u1[p] : u0[p];
                if (u > mx) mx = u;
                sm += u;
            }
            if (!*found || mx < *best_max || (mx == *best_max && sm < *best_sum)) {
                *found = 1; *best_max = mx; *best_sum = sm; *best_pidx = pidx; *best_aidx = r * k + d;
                for (i = 0; i < last; i++) best_alloc[i] = (int8_t)digit[i];
                best_alloc[last] = (int8_t)d;
            }
        }
        /* next run: increment the base-k number of tasks 0..n-2, task n-2 least significant */
        for (i = last - 1; i >= 0; i--) {
            mask[digit[i]] &= ~(1u << i);
            if (++digit[i] < k) { mask[digit[i]] |= 1u << i; break; }
            digit[i] = 0;
            mask[0] |= 1u << i;
        }
    }
}

typedef struct {
    int32_t status;
    uint8_t verdict, verdict_1g;
    int32_t pidx;
    int64_t aidx;
    uint64_t maxU, sumU;
    int64_t n_evals;
} or_set_result;

/* solve one set; sizes_out[K], alloc_out[n], R_out[n], R1g_out[n] */
static void or_solve_one(const or_set *s, int K, int mode, int flags, or_set_result *res,
                         int32_t *sizes_out, int8_t *alloc_out, int64_t *R_out, int64_t *R1g_out)
{
    int n = s->n, i, p, k;
    int64_t P, pi;
    int *table;
    int8_t cur[OR_MAXN], best_alloc[OR_MAXN];
    int best_found = 0;
    int64_t best_pidx = -1, best_aidx = -1;
    uint64_t best_max = 0, best_sum = 0;
    int reject, use_memo;
    or_memo memo = {0, 0, NULL};
    int one[1];
    int8_t zeros[OR_MAXN];

    memset(res, 0, sizeof *res);
    res->pidx = -1; res->aidx = -1;
    for (p = 0; p < K; p++) sizes_out[p] = 0;
    for (i = 0; i < n && i < OR_MAXN; i++) { alloc_out[i] = -1; R_out[i] = -1; R1g_out[i] = -1; }
    res->status = or_validate(s, K, mode);
    if (res->status != OR_OK) {
        if (n > 0 && n <= OR_MAXN) for (i = 0; i < n; i++) { alloc_out[i] = -1; R_out[i] = -1; R1g_out[i] = -1; }
        return;
    }
    P = or_count_partitionings(s->M, K);
    res->n_evals = P;
    table = (int *)malloc(sizeof(int) * (size_t)(P * K));
    or_enumerate_partitionings(s->M, K, table, P);
    reject = (flags & OR_FLAG_NO_LEMMA1) ? 0 : or_lemma1_reject(s);
    use_memo = !reject && mode == OR_EXH && (flags & OR_FLAG_EXH_FAST) && n <= OR_FAST_MAXN &&
               or_memo_build(s, &memo);
    if (!reject) {
        for (pi = 0; pi < P; pi++) {
            const int *sz = table + pi * K;
            int allowed = 1;
            for (k = 0; k < K && sz[k] > 0; k++)
                if (s->adm && !((s->adm[sz[k] / 64] >> (sz[k] % 64)) & 1u)) allowed = 0;
            if (!allowed) continue; /* a part size outside the admissible set */
            if (use_memo) {
                or_memo_scan(s, &memo, sz, k, pi, &best_found, &best_max, &best_sum, &best_pidx, &best_aidx,
                             best_alloc);
            } else if (mode == OR_EXH) {
                int64_t a, A = 1;
                for (i = 0; i < n; i++) A *= k;
                for (a = 0; a < A; a++) {
                    int64_t x = a;
                    uint64_t mx, sm;
                    for (i = n - 1; i >= 0; i--) { cur[i] = (int8_t)(x % k); x /= k; }
                    if (s->cnt) s->cnt->combines++;
                    if (!or_eval_triple(s, sz, k, cur, 1, NULL, &mx, &sm)) continue;
                    if (!best_found || mx < best_max || (mx == best_max && sm < best_sum)) {
                        best_found = 1; best_max = mx; best_sum = sm;
                        best_pidx = pi; best_aidx = a;
                        memcpy(best_alloc, cur, (size_t)n);
                    }
                }
            } else {
                uint64_t mx, sm;
                if (!or_heuristic(s, sz, k, mode, cur)) continue;
                if (!or_eval_triple(s, sz, k, cur, 1, NULL, &mx, &sm)) abort(); /* H builds feasible maps */
                if (!best_found || mx < best_max || (mx == best_max && sm < best_sum)) {
                    best_found = 1; best_max = mx; best_sum = sm;
                    best_pidx = pi; best_aidx = 0;
                    memcpy(best_alloc, cur, (size_t)n);
                }
            }
        }
    }
    if (best_found) {
        const int *sz = table + best_pidx * K;
        for (k = 0; k < K && sz[k] > 0; k++) sizes_out[k] = sz[k];
        res->verdict = 1;
        res->pidx = (int32_t)best_pidx;
        res->aidx = best_aidx;
        res->maxU = best_max;
        res->sumU = best_sum;
        memcpy(alloc_out, best_alloc, (size_t)n);
        or_eval_triple(s, sz, k, best_alloc, 0, R_out, NULL, NULL);
    }
    /* whole-GPU baseline: one partition of M units, every task evaluated */
    one[0] = s->M;
    memset(zeros, 0, sizeof zeros);
    res->verdict_1g = (uint8_t)or_eval_triple(s, one, 1, zeros, 0, R1g_out, NULL, NULL);
    free(table);
    free(memo.U);
}

/* ---- exported entry points ----------------------------------------------- */
static void or_make_set(or_set *s, int64_t off0, int64_t off1, int32_t M, const int64_t *T, const int64_t *D,
                        const int64_t *Cs, const int64_t *Cp, const int32_t *k, const uint8_t *type,
                        or_counters *cnt)
{
    s->n = (int)(off1 - off0);
    s->M = M;
    s->T = T + off0; s->D = D + off0;
    s->Cs = Cs ? Cs + off0 : NULL; s->Cp = Cp ? Cp + off0 : NULL; s->k = k ? k + off0 : NULL;
    s->type = type + off0;
    s->Cn_tab = s->Cc_tab = NULL;
    s->adm = NULL;
    s->edf = 0;
    s->cnt = cnt;
}

typedef struct {
    int64_t n_sets;
    const int64_t *off; const int32_t *M;
    const int64_t *T, *D, *Cs, *Cp; const int32_t *k; const uint8_t *type;
    const int64_t *tab_off, *Cn_tab, *Cc_tab; /* explicit tables (NULL: parametric) */
    const uint64_t *adm;                      /* admissible sizes (NULL: every size) */
    int K, mode, flags;
    int32_t *status; uint8_t *verdict, *verdict_1g; int32_t *pidx, *sizes;
    int64_t *aidx; uint64_t *maxU, *sumU; int64_t *n_evals;
    int8_t *alloc; int64_t *R, *R1g; int64_t *counters;
    int64_t next;
    pthread_mutex_t lock;
} or_batch;

static void or_batch_set(or_batch *b, int64_t si)
{
    or_set s;
    or_counters cnt = {0, 0, 0};
    or_set_result r;
    int64_t o0 = b->off[si], o1 = b->off[si + 1];
    int n = (int)(o1 - o0), i;
    int8_t al[OR_MAXN]; int64_t R[OR_MAXN], R1[OR_MAXN];
    or_make_set(&s, o0, o1, b->M[si], b->T, b->D, b->Cs, b->Cp, b->k, b->type, &cnt);
    if (b->Cn_tab) {
        s.Cn_tab = b->Cn_tab + b->tab_off[si];
        s.Cc_tab = b->Cc_tab + b->tab_off[si];
    }
    s.adm = b->adm;
    s.edf = (b->flags & OR_FLAG_EDF) != 0;
    if (n < 0) n = 0;
    or_solve_one(&s, b->K, b->mode, b->flags, &r, b->sizes + si * b->K, al, R, R1);
    b->status[si] = r.status; b->verdict[si] = r.verdict; b->verdict_1g[si] = r.verdict_1g;
    b->pidx[si] = r.pidx; b->aidx[si] = r.aidx; b->maxU[si] = r.maxU; b->sumU[si] = r.sumU;
    b->n_evals[si] = r.n_evals;
    for (i = 0; i < n; i++) {
        if (i < OR_MAXN && r.status == OR_OK) {
            b->alloc[o0 + i] = al[i]; b->R[o0 + i] = R[i]; b->R1g[o0 + i] = R1[i];
        } else {
            b->alloc[o0 + i] = -1; b->R[o0 + i] = -1; b->R1g[o0 + i] = -1;
        }
    }
    if (b->counters) {
        b->counters[si * 3 + 0] = cnt.terms;
        b->counters[si * 3 + 1] = cnt.tests;
        b->counters[si * 3 + 2] = cnt.combines;
    }
}

static void *or_worker(void *arg)
{
    or_batch *b = (or_batch *)arg;
    for (;;) {
        int64_t si;
        pthread_mutex_lock(&b->lock);
        si = b->next++;
        pthread_mutex_unlock(&b->lock);
        if (si >= b->n_sets) break;
        or_batch_set(b, si);
    }
    return NULL;
}

/* Solve a batch of task sets (SoA, offsets[n_sets+1]) with nthreads workers.
 * Explicit time tables (optional, all three or none): set s's task i has its
 * time on m units at Cn_tab/Cc_tab[tab_off[s] + i*M[s] + m-1]; Cs, Cp and k
 * may then be NULL.  adm (optional, 4 words): only partitionings whose part
 * sizes all have their bit set are considered (NULL: every partitioning).
 * Outputs: per set status, verdict, verdict_1g, pidx, sizes[K], aidx, maxU,
 * sumU, n_evals; per task alloc, R, R1g; counters[3] per set (optional). */
int or_solve_batch(int64_t n_sets, const int64_t *off, const int32_t *M,
                   const int64_t *T, const int64_t *D, const int64_t *Cs, const int64_t *Cp,
                   const int32_t *k, const uint8_t *type, const int64_t *tab_off, const int64_t *Cn_tab,
                   const int64_t *Cc_tab, const uint64_t *adm, int K, int mode, int flags, int nthreads,
                   int32_t *status, uint8_t *verdict, uint8_t *verdict_1g, int32_t *pidx, int32_t *sizes,
                   int64_t *aidx, uint64_t *maxU, uint64_t *sumU, int64_t *n_evals,
                   int8_t *alloc, int64_t *R, int64_t *R1g, int64_t *counters)
{
    or_batch b;
    pthread_t th[256];
    int t;
    if (K < 1 || K > 8 || mode < OR_EXH || mode > OR_SMS_ACT) return OR_E_INVAL;
    b.n_sets = n_sets; b.off = off; b.M = M; b.T = T; b.D = D; b.Cs = Cs; b.Cp = Cp; b.k = k;
    b.tab_off = tab_off; b.Cn_tab = tab_off ? Cn_tab : NULL; b.Cc_tab = tab_off ? Cc_tab : NULL;
    b.adm = adm;
    b.type = type; b.K = K; b.mode = mode; b.flags = flags; b.status = status; b.verdict = verdict;
    b.verdict_1g = verdict_1g; b.pidx = pidx; b.sizes = sizes; b.aidx = aidx; b.maxU = maxU;
    b.sumU = sumU; b.n_evals = n_evals; b.alloc = alloc; b.R = R; b.R1g = R1g; b.counters = counters;
    b.next = 0;
    pthread_mutex_init(&b.lock, NULL);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if (nthreads == 1) {
        or_worker(&b);
    } else {
        for (t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, or_worker, &b);
        for (t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    }
    pthread_mutex_destroy(&b.lock);
    return OR_OK;
}

/* ---- single-function entry points used by the pins ---------------------- */
#define OR_SET_ARGS int n, int M, const int64_t *T, const int64_t *D, const int64_t *Cs, \
                    const int64_t *Cp, const int32_t *k, const uint8_t *type
#define OR_SET_INIT(s) do { (s).n = n; (s).M = M; (s).T = T; (s).D = D; (s).Cs = Cs; (s).Cp = Cp; \
                            (s).k = k; (s).type = type; (s).Cn_tab = NULL; (s).Cc_tab = NULL; \
                            (s).adm = NULL; (s).edf = 0; (s).cnt = NULL; } while (0)

/* evaluate one triple; returns feasible; R_out[n] (-1 for misses or, with
 * early_exit, for tasks never reached) */
int or_eval_triple_ex(OR_SET_ARGS, const int32_t *sizes, int nparts, const int8_t *alloc,
                      int early_exit, int64_t *R_out, uint64_t *maxU, uint64_t *sumU, int64_t *counters)
{
    or_set s;
    or_counters cnt = {0, 0, 0};
    int sz[16], i, f;
    OR_SET_INIT(s);
    s.cnt = &cnt;
    for (i = 0; i < nparts && i < 16; i++) sz[i] = sizes[i];
    for (i = 0; i < n; i++) R_out[i] = -1;
    *maxU = 0; *sumU = 0;
    f = or_eval_triple(&s, sz, nparts, alloc, early_exit, R_out, maxU, sumU);
    if (counters) { counters[0] = cnt.terms; counters[1] = cnt.tests; counters[2] = cnt.combines; }
    return f;
}

int or_heuristic_ex(OR_SET_ARGS, const int32_t *sizes, int nparts, int variant, int8_t *alloc)
{
    or_set s;
    int sz[16], i;
    OR_SET_INIT(s);
    for (i = 0; i < nparts && i < 16; i++) sz[i] = sizes[i];
    return or_heuristic(&s, sz, nparts, variant, alloc);
}

/* best allocation on one fixed partitioning (exhaustive or heuristic):
 * returns found; writes alloc[n], maxU, sumU, aidx */
int or_best_on_partitioning(OR_SET_ARGS, const int32_t *sizes, int nparts, int mode,
                            int8_t *alloc, uint64_t *maxU, uint64_t *sumU, int64_t *aidx)
{
    or_set s;
    int sz[16], i, found = 0;
    int8_t cur[OR_MAXN];
    OR_SET_INIT(s);
    if (n < 1 || n > OR_MAXN_FIXED) return -1;
    for (i = 0; i < nparts && i < 16; i++) sz[i] = sizes[i];
    if (mode == OR_EXH) {
        int64_t a, A = 1;
        for (i = 0; i < n; i++) A *= nparts;
        for (a = 0; a < A; a++) {
            int64_t x = a;
            uint64_t mx, sm;
            for (i = n - 1; i >= 0; i--) { cur[i] = (int8_t)(x % nparts); x /= nparts; }
            if (!or_eval_triple(&s, sz, nparts, cur, 1, NULL, &mx, &sm)) continue;
            if (!found || mx < *maxU || (mx == *maxU && sm < *sumU)) {
                found = 1; *maxU = mx; *sumU = sm; *aidx = a;
                memcpy(alloc, cur, (size_t)n);
            }
        }
    } else {
        if (or_heuristic(&s, sz, nparts, mode, cur)) {
            found = or_eval_triple(&s, sz, nparts, cur, 1, NULL, maxU, sumU);
            *aidx = 0;
            memcpy(alloc, cur, (size_t)n);
        }
    }
    if (!found) for (i = 0; i < n; i++) alloc[i] = -1;
    return found;
}

int or_m_min_ex(OR_SET_ARGS, int i)
{
    or_set s;
    OR_SET_INIT(s);
    return or_m_min(&s, i);
}

int or_forbidden_ex(OR_SET_ARGS, int i, int j)
{
    or_set s;
    int mm[OR_MAXN], t;
    OR_SET_INIT(s);
    if (n < 1 || n > OR_MAXN || i < 0 || j < 0 || i >= n || j >= n) return -1;
    for (t = 0; t < n; t++) mm[t] = or_m_min(&s, t);
    return or_forbidden(&s, i, j, mm);
}

int or_lemma1_reject_ex(OR_SET_ARGS)
{
    or_set s;
    OR_SET_INIT(s);
    return or_lemma1_reject(&s);
}

uint64_t or_u1_ex(OR_SET_ARGS, int i)
{
    or_set s;
    OR_SET_INIT(s);
    return or_u1(&s, i);
}

/* ==== Algorithm 1 with free partition sizes (Section "Heuristics") ==========
 *
 * The paper's own heuristic: start from one partition per task, each of the
 * Lemma 2 size (Section "Init partitions"), and while the partitions need
 * more than M compute units in total (Pi > M; Lemma 3: Pi <= M means every
 * partition schedulable on its own units, so the set is), pick a first
 * operand and merge it with an eligible partner (Algorithm 3,
 * select_partitions); a merge (Algorithm 2) is valid when the union is
 * schedulable on fewer units than the two partitions apart (Definition 3),
 * tried from max(m1, m2) upwards one unit at a time; a failed merge forbids
 * its task pairs (Section "Forbidden list"), which ACT fills beforehand for
 * every task pair.  Readings taken where the paper is silent or garbled:
 *   - par_list is kept in decreasing partition utilisation U(P) (Q32, as for
 *     H(pi)), ties by the partition's lowest task index; choose_from and
 *     choose take the first element;
 *   - order ">" (Definition 5, "BF") ranks the partners by U of the union at
 *     the merge's starting size max(m1, m2), which needs no merge, ties by
 *     par_list order; order ">>" (Definition 4, "SMS") computes every
 *     eligible merge and ranks the valid ones by merged size, then U, then
 *     par_list order;
 *   - a merged partition never exceeds M units;
 *   - every failed merge, also one computed while ranking for ">>", forbids
 *     all of its cross task pairs;
 *   - the algorithm fails when no partition has an eligible partner left.
 * Output: the final partitions in par_list order (sizes, task -> partition),
 * response times, and counters of merges tried and accepted.
 */
typedef struct {
    int mem[OR_MAXN];
    int cnt, m, lead; /* members, units, lowest task index */
    uint64_t U;       /* Q32 utilisation on m units */
} or_part;

/* Q32 utilisation of a task group on m units, schedulable or not */
static uint64_t or_group_util(const or_set *s, const int *mem, int cnt, int m)
{
    u128 acc = 0;
    int a, b;
    for (a = 0; a < cnt; a++) {
        int same = 0;
        int64_t C;
        for (b = 0; b < cnt; b++)
            if (s->type[mem[b]] == s->type[mem[a]]) same++;
        C = (same >= 2) ? or_cc(s, mem[a], m) : or_cn(s, mem[a], m);
        acc += ((((u128)C) << 32) + (u128)s->T[mem[a]] - 1) / (u128)s->T[mem[a]];
    }
    return (uint64_t)acc;
}

static int or_part_before(const or_part *a, const or_part *b)
{
    if (a->U != b->U) return a->U > b->U;
    return a->lead < b->lead;
}

static void or_sort_parts(or_part *p, int np)
{
    int a, b;
    for (a = 1; a < np; a++) {
        or_part x = p[a];
        b = a - 1;
        while (b >= 0 && or_part_before(&x, &p[b])) {
            p[b + 1] = p[b];
            b--;
        }
        p[b + 1] = x;
    }
}

/* Algorithm 2: the union of a and b on the first m in [max(m1, m2), m1 + m2)
 * (and <= M) that schedules it */
static int or_merge(const or_set *s, const or_part *a, const or_part *b, or_part *out)
{
    int m, t;
    out->cnt = 0;
    for (t = 0; t < a->cnt; t++) out->mem[out->cnt++] = a->mem[t];
    for (t = 0; t < b->cnt; t++) out->mem[out->cnt++] = b->mem[t];
    out->lead = a->lead < b->lead ? a->lead : b->lead;
    m = a->m > b->m ? a->m : b->m;
    while (m < a->m + b->m && m <= s->M) {
        uint64_t U = 0;
        if (or_eval_part(s, out->mem, out->cnt, m, 1, NULL, &U)) {
            out->m = m;
            out->U = U;
            return 1;
        }
        m++;
    }
    return 0;
}

static void or_forbid_cross(unsigned char *forb, int n, const or_part *a, const or_part *b)
{
    int x, y;
    for (x = 0; x < a->cnt; x++)
        for (y = 0; y < b->cnt; y++) {
            forb[a->mem[x] * n + b->mem[y]] = 1;
            forb[b->mem[y] * n + a->mem[x]] = 1;
        }
}

static int or_pair_forbidden(const unsigned char *forb, int n, const or_part *a, const or_part *b)
{
    int x, y;
    for (x = 0; x < a->cnt; x++)
        for (y = 0; y < b->cnt; y++)
            if (forb[a->mem[x] * n + b->mem[y]]) return 1;
    return 0;
}

/* returns 1 (schedulable, Pi <= M) or 0; variant: OR_BF_* (">") or OR_SMS_* (">>") */
static int or_alg1(const or_set *s, int variant, int flags, int *nparts, int32_t *sizes, int8_t *alloc,
                   int64_t *R, int64_t *stats)
{
    const int n = s->n;
    const int act = (variant == OR_BF_ACT || variant == OR_SMS_ACT);
    const int sms = (variant == OR_SMS_INA || variant == OR_SMS_ACT);
    or_part *parts = (or_part *)malloc(sizeof(or_part) * (size_t)n);
    or_part *cand = (or_part *)malloc(sizeof(or_part) * (size_t)n);
    unsigned char *forb = (unsigned char *)calloc((size_t)n * (size_t)n, 1);
    int mm[OR_MAXN], okc[OR_MAXN], order[OR_MAXN];
    uint64_t key[OR_MAXN];
    int np = 0, i, j, c, Pi = 0, ok = 0;
    stats[0] = stats[1] = stats[2] = 0;
    *nparts = 0;
    for (i = 0; i < n; i++) { alloc[i] = -1; R[i] = -1; }
    if (!(flags & OR_FLAG_NO_LEMMA1) && or_lemma1_reject(s)) goto done;
    /* init partitions (Lemma 2 sizes) */
    for (i = 0; i < n; i++) {
        mm[i] = or_m_min(s, i);
        if (mm[i] >= OR_MINF) goto done;
        parts[np].mem[0] = i;
        parts[np].cnt = 1;
        parts[np].m = mm[i];
        parts[np].lead = i;
        parts[np].U = or_group_util(s, &i, 1, mm[i]);
        np++;
    }
    or_sort_parts(parts, np);
    if (act)
        for (i = 0; i < n; i++)
            for (j = i + 1; j < n; j++)
                if (or_forbidden(s, i, j, mm)) forb[i * n + j] = forb[j * n + i] = 1;
    for (;;) {
        int merged = 0;
        Pi = 0;
        for (c = 0; c < np; c++) Pi += parts[c].m;
        if (Pi <= s->M) { ok = 1; break; }
        /* Algorithm 3: first operand in par_list order with an eligible partner */
        for (c = 0; c < np && !merged; c++) {
            int ne = 0, a, b;
            for (j = 0; j < np; j++)
                if (j != c && !or_pair_forbidden(forb, n, &parts[c], &parts[j])) order[ne++] = j;
            if (ne == 0) continue;
            /* rank the eligible partners */
            for (a = 0; a < ne; a++) {
                j = order[a];
                if (sms) {
                    stats[0]++;
                    okc[a] = or_merge(s, &parts[c], &parts[j], &cand[a]);
                    if (!okc[a]) or_forbid_cross(forb, n, &parts[c], &parts[j]);
                    key[a] = okc[a] ? (((uint64_t)cand[a].m) << 40) : ~0ull;
                } else {
                    or_part u;
                    int m0 = parts[c].m > parts[j].m ? parts[c].m : parts[j].m, t;
                    u.cnt = 0;
                    for (t = 0; t < parts[c].cnt; t++) u.mem[u.cnt++] = parts[c].mem[t];
                    for (t = 0; t < parts[j].cnt; t++) u.mem[u.cnt++] = parts[j].mem[t];
                    key[a] = or_group_util(s, u.mem, u.cnt, m0);
                    okc[a] = -1; /* not merged yet */
                }
            }
            /* stable insertion sort of (order, key, okc, cand) by key; for ">>"
               ties by U of the merge */
            for (a = 1; a < ne; a++) {
                int xo = order[a], xk2 = okc[a];
                uint64_t xk = key[a];
                or_part xc = cand[a];
                b = a - 1;
                while (b >= 0) {
                    int later = key[b] > xk;
                    if (sms && key[b] == xk && okc[b] == 1 && xk2 == 1) later = cand[b].U > xc.U;
                    if (!later) break;
                    order[b + 1] = order[b]; key[b + 1] = key[b]; okc[b + 1] = okc[b]; cand[b + 1] = cand[b];
                    b--;
                }
                order[b + 1] = xo; key[b + 1] = xk; okc[b + 1] = xk2; cand[b + 1] = xc;
            }
            /* Algorithm 1's repeat loop: merge with the partners in order */
            for (a = 0; a < ne && !merged; a++) {
                or_part m3;
                j = order[a];
                if (sms) {
                    if (okc[a] != 1) break; /* only failed merges remain (already forbidden) */
                    m3 = cand[a];
                } else {
                    stats[0]++;
                    if (!or_merge(s, &parts[c], &parts[j], &m3)) {
                        or_forbid_cross(forb, n, &parts[c], &parts[j]);
                        continue;
                    }
                }
                stats[1]++;
                /* par_list minus the two operands, plus the merge, in order */
                {
                    int lo = c < j ? c : j, hi = c < j ? j : c, t, w = 0;
                    for (t = 0; t < np; t++)
                        if (t != lo && t != hi) parts[w++] = parts[t];
                    parts[w++] = m3;
                    np = w;
                    or_sort_parts(parts, np);
                }
                merged = 1;
            }
        }
        if (!merged) break; /* no partition has an eligible partner: fail */
    }
done:
    if (ok) {
        *nparts = np;
        for (c = 0; c < np; c++) {
            int t;
            sizes[c] = parts[c].m;
            for (t = 0; t < parts[c].cnt; t++) alloc[parts[c].mem[t]] = (int8_t)c;
            or_eval_part(s, parts[c].mem, parts[c].cnt, parts[c].m, 0, R, NULL);
        }
        /* the scheduled workload (Figs. 5 and 7): every task's one-unit
         * utilisation in the conflict state its partition gives it, Q32 ceil */
        for (c = 0; c < np; c++) {
            int t, u;
            for (t = 0; t < parts[c].cnt; t++) {
                int i = parts[c].mem[t], same = 0;
                for (u = 0; u < parts[c].cnt; u++)
                    if (s->type[parts[c].mem[u]] == s->type[i]) same++;
                const int64_t C1 = same >= 2 ? or_cc(s, i, 1) : or_cn(s, i, 1);
                stats[2] += (int64_t)(uint64_t)(((((u128)C1) << 32) + (u128)s->T[i] - 1) / (u128)s->T[i]);
            }
        }
    }
    free(parts);
    free(cand);
    free(forb);
    return ok;
}

/* Cn_tab/Cc_tab: explicit time tables of the set ([i*M + m-1]) or NULL */
int or_alg1_ex(OR_SET_ARGS, const int64_t *Cn_tab, const int64_t *Cc_tab, int variant, int flags, int32_t *nparts,
               int32_t *sizes, int8_t *alloc, int64_t *R, int64_t *stats)
{
    or_set s;
    int np = 0, ok;
    OR_SET_INIT(s);
    s.Cn_tab = Cn_tab;
    s.Cc_tab = Cn_tab ? Cc_tab : NULL;
    s.edf = (flags & OR_FLAG_EDF) != 0;
    /* partition indices are int8: beyond 64 tasks the final partitions (at
     * most M of them) must number at most 127 */
    if (n < 1 || n > OR_MAXN || M < 1 || (n > OR_MAXN_FIXED && M > 127)) return -1;
    ok = or_alg1(&s, variant, flags, &np, sizes, alloc, R, stats);
    *nparts = np;
    return ok;
}
