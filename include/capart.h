/*
 * capart.h -- C ABI of the contention-aware GPU partitioning engine for
 * MI355X (gfx950).  Method: Zahaf et al., "Contention-Aware GPU Partitioning
 * and Task-to-Partition Allocation for Real-Time Workloads", arXiv 2105.10312.
 *
 * Problem (paper, Section "Heuristics", problem statement and Algorithm 1's
 * inputs/outputs): given a set of real-time GPU kernels (tasks) and an integer
 * number M of compute units, choose partition sizes and a task-to-partition
 * allocation so that every task meets its deadline, and say whether the set is
 * schedulable.  This library evaluates, for many task sets at once, every
 * partitioning of M compute units into at most K partitions, allocates tasks to
 * the partitions of each partitioning (exhaustively, or with the paper's greedy
 * heuristic ingredients), tests each partition and keeps the best feasible
 * (partitioning, allocation); the whole-GPU baseline ("1G", every task on one
 * partition of M units) is evaluated alongside.
 *
 * Model (all integers; times in microseconds):
 *   Cn_i(m) = C_seq_i + ceil(C_par_i / m)          time on m units, no conflict
 *   Cc_i(m) = ceil(k_i * Cn_i(m) / 1000)            time on m units, in conflict
 *     (Section "Modeling kernel execution times": a/m + b per interference
 *      state; Section "Task set generation": conflict inflation factor k)
 *   task i is in conflict iff another task of the same type (memory/compute)
 *   shares its partition (Section "Task Model");
 *   each partition runs its tasks one at a time on all its units, preemptive
 *   fixed priority in deadline-monotonic order (D, T, index), exact
 *   response-time test R_i = C_i + sum_{hp} ceil(R_i/T_j) C_j <= D_i
 *   (Section "Schedulability test": any policy with an exact test, interference
 *   folded into the execution times);
 *   U(P) = sum_{i in P} ceil(C_i * 2^32 / T_i)  (Q32 utilisation, Definition 5);
 *   best triple = min over feasible triples of (max_p U_p, sum_p U_p,
 *   partitioning index, allocation index).
 *   Lemma 1 (sum Cn_i(1)/T_i > M => unschedulable) prunes sets; Lemma 2 gives
 *   the smallest partition for one task.
 *
 * Partitionings of M into at most K parts are integer partitions (parts >= 1,
 * sum M) written non-increasing and numbered in descending lexicographic order
 * from 0: M=8, K=3 gives (8),(7,1),(6,2),(6,1,1),(5,3),(5,2,1),(4,4),(4,3,1),
 * (4,2,2),(3,3,2).  An allocation maps task i to part a_i in [0, k); the
 * exhaustive mode numbers allocations by the base-k digits of (a_0 .. a_{n-1}),
 * task 0 most significant; a part may stay empty.
 *
 * Heuristic allocation on a fixed partitioning (modes HEUR_*): tasks are taken
 * in decreasing Cn_i(1)/T_i (ties: lower index); each is placed on the part
 * that stays schedulable with it and ranks best: BF ranks by (U of the merged
 * part, part index) -- the order ">" of Definition 5; SMS ranks by (fewest units
 * the merged part needs, U, part index) -- the order ">>" of Definition 4 with
 * the search of Algorithm 2; ACT additionally never co-locates a task pair whose
 * two-task merge is invalid (Definition 3, Section "Forbidden list"); INA does
 * not.  A task with no candidate part makes the partitioning fail.
 *
 * Ownership: callers own every input and output buffer.  Host-pointer calls are
 * synchronous and borrow buffers for the call only.  *_async calls take device
 * pointers and are ordered on the given HIP stream; the caller keeps buffers
 * alive until the stream has passed the operation.  A context owns only its
 * device workspace and is not thread-safe; use one context per host thread.
 * No C++ exception crosses this interface.
 *
 * Errors: every call returns a capart_status.  Problems with one task set
 * (invalid sizes or values) are reported in results.status[s] and the batch
 * continues; an infeasible set is not an error (verdict 0, pidx -1, alloc -1,
 * R -1).  capart_last_error() gives a message for the last failing call.
 */
#ifndef CAPART_H
#define CAPART_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t capart_status;
#define CAPART_OK        0
#define CAPART_E_INVAL  (-1) /* null/inconsistent arguments, sizes out of the supported range */
#define CAPART_E_RANGE  (-2) /* a task value outside its domain (see capart_tasksets)         */
#define CAPART_E_NOMEM  (-3) /* device or host allocation failed                              */
#define CAPART_E_DEVICE (-4) /* HIP runtime error                                             */
#define CAPART_E_AGAIN  (-5) /* serving back-pressure: no slot or memory free, retry later    */
#define CAPART_E_STATE  (-6) /* call not valid in the object's current state                  */

/* allocation modes */
#define CAPART_EXHAUSTIVE    0
#define CAPART_HEUR_BF_INA   1
#define CAPART_HEUR_BF_ACT   2
#define CAPART_HEUR_SMS_INA  3
#define CAPART_HEUR_SMS_ACT  4

/* per-partition scheduling policy (Section "Schedulability test": any
 * policy with an exact test; each partition is one server running its tasks
 * one at a time on all its units) */
#define CAPART_POLICY_FP_DM  0 /* preemptive fixed priority, deadline monotonic, exact RTA */
#define CAPART_POLICY_EDF    1 /* preemptive EDF, processor-demand test (below)          */
/*
 * CAPART_POLICY_EDF: a partition is schedulable iff (1) its floor-Q32
 * utilisation sum floor(C_i 2^32 / T_i) is at most 2^32, and (2) the demand
 * h(d) = sum_{D_j <= d} (floor((d - D_j)/T_j) + 1) C_j is at most d at every
 * absolute deadline d below the horizon H (processor-demand criterion for
 * constrained deadlines, Baruah, Rosier and Howell 1990).  H is the
 * synchronous busy period (least fixed point of w = sum ceil(w/T_j) C_j from
 * sum C_j) when that iteration settles within 4096 steps, else the bound
 * ceil(sum C 2^32 / (2^32 - Uq)) with the ceil-Q32 utilisation Uq; a
 * partition whose utilisation is within n 2^-32 of 1 without a settled busy
 * period, or with more than 65536 absolute deadlines below H, is declared
 * unschedulable (a pessimistic limit that bounds the work of one test).
 * Reported response times: min(D_i, H) for every task of a schedulable
 * partition (each job completes by its deadline and within the busy period),
 * -1 for every task of an unschedulable one (1G included).  Lemma 2 sizes,
 * the Lemma 1 filter, utilisations and keys are policy-independent; ACT's
 * pair test uses the policy.  Honoured by capart_solve, capart_solve_async,
 * capart_count_work, capart_allocate, the batched plans, Algorithm 1 and
 * the server (capart_server_config.policy); capart_test_triple schedules by
 * CAPART_POLICY_FP_DM (its arguments carry no policy).
 */

/* option flags */
#define CAPART_FLAG_SKIP_1G         1u /* do not evaluate the whole-GPU baseline (R_1g = -1)    */
#define CAPART_FLAG_NO_LEMMA1       2u /* disable the Lemma 1 pre-filter (results identical)     */
#define CAPART_FLAG_PER_SET_LAUNCH  4u /* plain path: one launch sequence per task set           */
/* capart_server_config.flags only: reserve room for explicit time tables
 * (max_M entries of each kind per task) so that queries may carry them. */
#define CAPART_SERVER_TABLES        8u

/* limits */
#define CAPART_MAX_TASKS   64   /* tasks per set                                          */
#define CAPART_MAX_M       255  /* compute units per set                                  */
#define CAPART_MAX_K       8    /* parts per partitioning                                  */
#define CAPART_MAX_NM      8192 /* n * M per set (the per-set time table lives in LDS)    */
/* Algorithm 1 (capart_alg1 calls) also takes sets of up to 256 tasks under
 * fixed priority, with M <= 127 and n * M <= CAPART_ALG1_BIG_MAX_NM per set */
#define CAPART_ALG1_MAX_TASKS  256
#define CAPART_ALG1_BIG_MAX_M  127
#define CAPART_ALG1_BIG_MAX_NM 14336

/*
 * Task sets, structure of arrays.  Set s holds tasks set_offset[s] ..
 * set_offset[s+1]-1 and has M[s] compute units.  Domains (else per-set status
 * E_RANGE): 1 <= T < 2^31; 1 <= D <= T; C_seq >= 0, C_par >= 0,
 * 1 <= C_seq + C_par < 2^31; 1000 <= k_permille <= 1000000; type in {0, 1}
 * (0 = compute-intensive, 1 = memory-intensive).  Sizes (else per-set status
 * E_INVAL): 1 <= n <= min(max_tasks, 64); 1 <= M <= min(max_M, 255);
 * n * M <= 8192; exhaustive mode needs min(K, M)^n < 2^62.  max_tasks and
 * max_M are caller-declared bounds over the batch (the launch is sized from
 * them without reading device memory).
 *
 * Explicit time tables (optional; all three pointers set, or all NULL for the
 * parametric model above): task i (0-based within set s) takes
 * Cn_table[table_offset[s] + i*M[s] + m-1] on m units without conflict and
 * Cc_table[same] in conflict, m = 1..M[s] (Section "Modeling kernel execution
 * times": one time function per interference state, here given pointwise, as
 * measured kernels give it).  C_seq, C_par and k_permille are then not read
 * and may be NULL.  Domain (else per-set status E_RANGE): every entry in
 * [1, 2^31), non-increasing in m, Cc >= Cn at every m, and m * Cn(m) >= Cn(1)
 * (no super-linear speed-up, which Lemma 1 needs).  table_offset[s] >= 0 and
 * table_offset[s] + n * M[s] <= table_len (else E_INVAL).  Tables are taken by
 * capart_validate, capart_solve, capart_solve_async,
 * capart_solve_async_noalloc, capart_count_work, the batched plans, the
 * capart_alg1 calls and a server created with CAPART_SERVER_TABLES; other
 * servers and the one-set calls (capart_test_triple, capart_allocate) return
 * E_INVAL for them.
 */
typedef struct capart_tasksets {
    int64_t n_sets;
    int64_t n_tasks_total;       /* = set_offset[n_sets]                    */
    int32_t max_tasks;           /* bound on tasks per set, 1..64 (1..256
                                    for the capart_alg1 calls)             */
    int32_t max_M;               /* bound on M, 1..255                      */
    const int64_t *set_offset;   /* [n_sets + 1], non-decreasing, from 0    */
    const int32_t *M;            /* [n_sets]                                */
    const int64_t *T;            /* [n_tasks_total] period                  */
    const int64_t *D;            /* [n_tasks_total] relative deadline       */
    const int64_t *C_seq;        /* [n_tasks_total] part not sped up by m   */
    const int64_t *C_par;        /* [n_tasks_total] part divided over m     */
    const int32_t *k_permille;   /* [n_tasks_total] conflict inflation      */
    const uint8_t *type;         /* [n_tasks_total] 0 compute, 1 memory     */
    const int64_t *table_offset; /* [n_sets] or NULL: explicit time tables  */
    const int64_t *Cn_table;     /* [table_len] or NULL                     */
    const int64_t *Cc_table;     /* [table_len] or NULL                     */
    int64_t table_len;
} capart_tasksets;

/*
 * Admissible partition sizes (MIG-like restrictions of the sizes a partition
 * may take; Section "Conclusion" names such partitioning mechanisms):
 * admissible[m >> 6] bit (m & 63) set allows size m (1..255); all four words
 * 0 allows every size.  A partitioning with a part of another size is still
 * numbered and counted in n_evals but is infeasible (its debug key is
 * "none"); the whole-GPU baseline is unaffected.  Honoured by capart_solve,
 * capart_solve_async, capart_count_work, the batched plans and the server
 * (capart_server_config.admissible, for every query); capart_alg1
 * and capart_alg1_async return E_INVAL for a non-empty mask; the one-set calls
 * evaluate the partitioning they are given.
 */
typedef struct capart_options {
    int32_t K;           /* maximum number of parts, 1..8      */
    int32_t policy;      /* CAPART_POLICY_FP_DM or _EDF        */
    int32_t alloc_mode;  /* CAPART_EXHAUSTIVE or CAPART_HEUR_* */
    uint32_t flags;      /* CAPART_FLAG_*                      */
    uint64_t admissible[4];  /* allowed part sizes, all 0 = every size */
} capart_options;

/*
 * Results.  Per set: status (CAPART_OK or the set's error), verdict (1 iff a
 * feasible triple exists), verdict_1g, pidx (index of the chosen partitioning
 * of M[s] into <= K parts, -1 if none), sizes[s*K .. s*K+K) (its parts,
 * 0-padded), aidx (allocation index: base-k digits in exhaustive mode, 0 for the
 * heuristic, -1 if none), maxU and sumU (Q32 utilisation key of the chosen
 * triple), n_evals (number of partitionings resolved: P(M, K), including sets
 * rejected by Lemma 1; 0 for invalid sets).  Per task: alloc (part index or -1),
 * R (response time in the chosen triple or -1), R_1g (response time on the
 * whole GPU, -1 on a miss or with CAPART_FLAG_SKIP_1G).
 * Optional debug output, per (set, partitioning): if dbg_key is non-NULL,
 * dbg_key[3*(dbg_offset[s] + p) + {0,1,2}] = {maxU, sumU, found ? aidx : ~0}
 * for partitioning p of set s (maxU = sumU = ~0 when nothing is feasible);
 * dbg_offset[s] is supplied by the caller (e.g. prefix sums of P(M_s, K)).
 */
typedef struct capart_results {
    int32_t *status;
    uint8_t *verdict;
    uint8_t *verdict_1g;
    int32_t *pidx;
    int32_t *sizes;
    int64_t *aidx;
    uint64_t *maxU;
    uint64_t *sumU;
    int64_t *n_evals;
    int8_t *alloc;
    int64_t *R;
    int64_t *R_1g;
    uint64_t *dbg_key;           /* optional, may be NULL */
    const int64_t *dbg_offset;   /* required iff dbg_key  */
} capart_results;

typedef struct capart_ctx capart_ctx;

/* Create a context on HIP device `device` (uploads the partition-count table).
 * E_DEVICE if the device cannot be used, E_NOMEM on allocation failure. */
capart_status capart_create(int device, capart_ctx **out);
capart_status capart_destroy(capart_ctx *ctx);
/* Message for the last failing call on ctx (or for capart_create when ctx is
 * NULL); never NULL; valid until the next call on ctx. */
const char *capart_last_error(const capart_ctx *ctx);
/* Hash (16 hex digits) of the kernel and host sources this library was built
 * from; never NULL, static storage.  A caller that ships sources beside the
 * library compares it with the sources' hash to refuse a stale build. */
const char *capart_build_hash(void);

/* Measure the full-rate 32-bit VALU throughput of the context's device: a
 * kernel of independent integer-add chains (eight per lane, eight waves per
 * SIMD), best of three timed launches.  *lane_ops_per_s gets lane-operations
 * per second (for the integer roofline beside the nominal 256 CUs x 64 lanes
 * x clock), *kernel_ms the best launch's time.  Synchronous; E_DEVICE on a
 * HIP error. */
capart_status capart_measure_valu(capart_ctx *ctx, double *lane_ops_per_s, double *kernel_ms);

/* Number of partitionings of M into at most K positive parts (host only). */
capart_status capart_count_partitionings(int32_t M, int32_t K, int64_t *count);
/* Write them in canonical order into sizes[count*K] (0-padded); at most
 * `capacity` partitionings are written; *count gets the total (host only). */
capart_status capart_enumerate_partitionings(int32_t M, int32_t K, int32_t *sizes, int64_t capacity,
                                             int64_t *count);
/* Host-side validation of a host-pointer batch: status_out[n_sets] gets each
 * set's status (the same rules the device applies).  Returns E_INVAL for
 * batch-level problems (NULL pointers, bad offsets, K or mode out of range). */
capart_status capart_validate(const capart_tasksets *host_in, const capart_options *opt, int32_t *status_out);

/* Evaluate one triple of one set (host pointers, set_offset = {0, n}):
 * sizes[k] (parts, any order), alloc[n] in [0, k).  Every task is tested (no
 * early exit): R[n] gets response times or -1; *feasible = all met; *maxU and
 * *sumU are valid when feasible.  Runs on the device. */
capart_status capart_test_triple(capart_ctx *ctx, const capart_tasksets *one_set, const int32_t *sizes, int32_t k,
                                 const int8_t *alloc, uint8_t *feasible, int64_t *R, uint64_t *maxU,
                                 uint64_t *sumU);
/* Best allocation of one set on one fixed partitioning sizes[k] (non-increasing,
 * sum M, k <= opt->K) under opt->alloc_mode: *found, alloc_out[n] (-1 if not
 * found), *maxU, *sumU, *aidx.  Runs on the device. */
capart_status capart_allocate(capart_ctx *ctx, const capart_tasksets *one_set, const int32_t *sizes, int32_t k,
                              const capart_options *opt, int8_t *alloc_out, uint8_t *found, uint64_t *maxU,
                              uint64_t *sumU, int64_t *aidx);

/* Solve a batch held in host memory; results in host memory (synchronous). */
capart_status capart_solve(capart_ctx *ctx, const capart_tasksets *host_in, const capart_options *opt,
                           capart_results *host_out);
/* Solve a batch held in device memory; results written to device memory,
 * ordered on hip_stream (a hipStream_t, NULL = default stream).  This is the
 * plain GPU path: one launch sequence over the whole batch, or one per set
 * with CAPART_FLAG_PER_SET_LAUNCH. */
capart_status capart_solve_async(capart_ctx *ctx, const capart_tasksets *dev_in, const capart_options *opt,
                                 capart_results *dev_out, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and results as capart_solve_async, bit for bit, with no
 * allocation at all (no hipMalloc, hipFree or allocating library routine;
 * the context, created beforehand, keeps the device tables it allocated at
 * set-up).  Its workspace (per-task records, forbidden-pair masks, heuristic
 * order, per-set flags and masks, one 32-byte key per set chunk) lives in one
 * file-scope device array of CAPART_NOALLOC_SCRATCH_BYTES per GPU, which the
 * library holds until the process ends.  A batch whose workspace exceeds it
 * returns CAPART_E_RANGE (message from capart_last_error) before anything is
 * launched; roughly 41 bytes per task plus 44 bytes per set plus 32 bytes per
 * set chunk, so 100,000 sets of 10 tasks fit.  Exhaustive allocation runs by
 * plain enumeration (the subset-table form needs its own memory); timing
 * events are not recorded.  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (on different streams, or from different
 * threads or contexts) race and give undefined results; calls ordered on one
 * stream do not.  Nothing in the array needs clearing between calls (every
 * word a launch reads is written earlier in the same launch sequence). */
#define CAPART_NOALLOC_SCRATCH_BYTES (64u << 20)
capart_status capart_solve_async_noalloc(capart_ctx *ctx, const capart_tasksets *dev_in, const capart_options *opt,
                                         capart_results *dev_out, void *hip_stream);

/*
 * Algorithm 1 with free partition sizes (Section "Heuristics": Algorithms 1,
 * 2 and 3, Definitions 3-5, Lemma 3).  Each task starts alone on a partition
 * of its Lemma 2 size; while the partitions need more than M units in total,
 * the first partition in par_list order that has an eligible partner (no
 * forbidden task pair between the two) is merged with one of them.  A merge
 * (Algorithm 2) is valid when the union is schedulable on some m in
 * [max(m1, m2), m1 + m2 - 1], m <= M, and takes the least such m.  par_list is
 * kept in decreasing Q32 utilisation U(P), ties by the partition's lowest task
 * index.  opt->alloc_mode picks the order and the forbidden list:
 *   CAPART_HEUR_BF_*  order ">" (Definition 5): partners ranked by U of the
 *                     union at max(m1, m2), ties by par_list position; the
 *                     first valid merge in that order is taken;
 *   CAPART_HEUR_SMS_* order ">>" (Definition 4): every eligible merge is
 *                     computed and the valid one with the fewest units, then
 *                     least U, then par_list position, is taken;
 *   *_INA             forbidden pairs only from failed merges: a failed merge
 *                     (for ">" one tried before the merge taken, for ">>" any)
 *                     forbids every task pair across its two partitions;
 *   *_ACT             in addition every pair whose two-task merge is invalid
 *                     (Definition 3) is forbidden from the start.
 * The set is schedulable (verdict 1) once the units fit M (Lemma 3), and not
 * schedulable (verdict 0) when Lemma 1 rejects it (unless
 * CAPART_FLAG_NO_LEMMA1), a task has no Lemma 2 size within M, or no partition
 * has an eligible partner left.  opt->K is not used (any value 1..8);
 * CAPART_EXHAUSTIVE is E_INVAL; flags other than NO_LEMMA1 have no effect.
 * Per-set validation as for capart_solve (status[s], the set's outputs then
 * hold the failure values).
 *
 * Set sizes: a batch with max_tasks <= 64 runs one wave of 64 lanes per set
 * under either policy.  A batch with max_tasks in 65..CAPART_ALG1_MAX_TASKS
 * (the paper's 200-task experiments) runs one block of 256 threads per set:
 * it takes CAPART_POLICY_FP_DM only and max_M <= CAPART_ALG1_BIG_MAX_M (else
 * E_INVAL for the call), and a set with n * M > CAPART_ALG1_BIG_MAX_NM gets
 * status E_INVAL.  Results are the same whichever path runs a set.
 *
 * Results (caller-owned; device pointers for the async call, host pointers for
 * capart_alg1):
 *   status[S], verdict[S];
 *   nparts[S]   number of partitions (0 when not schedulable);
 *   sizes[N]    set s's partition sizes in par_list order at
 *               sizes[set_offset[s] .. set_offset[s] + nparts[s]), the rest of
 *               the set's slots 0 (a set of n tasks has at most n partitions);
 *   alloc[N]    each task's partition (index into that set's sizes), -1 if none;
 *   R[N]        response time on its partition, -1 if none;
 *   tried[S], merged[S]  merges attempted (Algorithm 2 runs the algorithm
 *               asks for) and accepted; both 0 for sets rejected before any.
 * Every set of the batch runs in one launch (after the prep kernel) ordered
 * on hip_stream.
 */
typedef struct capart_alg1_results {
    int32_t *status;
    uint8_t *verdict;
    int32_t *nparts;
    int32_t *sizes;
    int8_t *alloc;
    int64_t *R;
    int64_t *tried;
    int64_t *merged;
    /* [n_sets], may be NULL: on success the scheduled workload of the result
     * (Section "Results and discussions", the efficiency of Figs. 5 and 7):
     * sum over the tasks of ceil(C_i(1) 2^32 / T_i) with C_i(1) the one-unit
     * time in the conflict state the task's final partition gives it (Q32,
     * modulo 2^64); 0 for an unschedulable set.  Between the same sum without
     * any conflict and with every task in conflict. */
    uint64_t *workload;
} capart_alg1_results;

/* Algorithm 1 over a batch in device memory; results in device memory. */
capart_status capart_alg1_async(capart_ctx *ctx, const capart_tasksets *dev_in, const capart_options *opt,
                                capart_alg1_results *dev_out, void *hip_stream);
/* Algorithm 1 over a batch in host memory; results in host memory (synchronous). */
capart_status capart_alg1(capart_ctx *ctx, const capart_tasksets *host_in, const capart_options *opt,
                          capart_alg1_results *host_out);

/*
 * Batched form.  A plan binds one device-resident batch (capart_tasksets with
 * device pointers) and its device result buffers, and prepares one persistent
 * launch over all of it: the per-set sizes are read back once (set_offset and
 * M), every set's partitionings are cut into work items of similar estimated
 * cost (number of partitionings x (n+1)^2), items are queued largest first,
 * and a persistent evaluation grid pulls them from a device counter, so sets of
 * uneven size and budget share one launch without idle blocks.  With
 * use_graph the prep, evaluation and final kernels are captured into a HIP
 * graph; capart_run_batch then costs one graph launch.  With autotune the plan
 * times candidate tunings (threads per block, loop form, item size, blocks per
 * compute unit) on a prefix of the batch (1/64 of it, at least 8192 sets) and
 * keeps the fastest, spending at most about 5 s; every candidate computes
 * identical results.  The candidates include the direct schedule (one block
 * per set chunk, as capart_solve_async, no work queue), which wins when every
 * set is one item and the persistent loop only costs registers.  Sets whose
 * frontier or test memo serves all of their partitionings form one item each.  Autotuning runs the path on that prefix
 * and so writes into the result buffers.  The plan owns its workspace; the caller
 * keeps the bound buffers alive and unchanged in size while the plan exists.
 * Results are those of capart_solve_async on the same batch, bit for bit.
 * Exhaustive mode is not batched this way (E_INVAL).
 */
typedef struct capart_plan capart_plan;

typedef struct capart_plan_config {
    int32_t autotune;       /* 1: time candidates on a prefix of the batch; 0: use the context's tuning */
    int32_t blocks_per_cu;  /* persistent blocks per compute unit, 0 = automatic, -1 = direct schedule   */
    int32_t item_evals;     /* partitionings per work item for a 10-task set, 0 = automatic             */
    int32_t use_graph;      /* 1: capture the launch sequence into a HIP graph                          */
} capart_plan_config;

typedef struct capart_plan_info {
    int64_t n_sets, n_items, total_evals;
    int32_t threads, loop_form, blocks, item_evals;  /* blocks 0: direct schedule */
    int32_t candidates_tried, use_graph;
    double tune_ms;         /* host wall time spent autotuning */
} capart_plan_info;

capart_status capart_plan_batch(capart_ctx *ctx, const capart_tasksets *dev_in, const capart_options *opt,
                                const capart_results *dev_out, const capart_plan_config *cfg, capart_plan **out);
/* Run the plan on hip_stream (NULL = default stream): one graph launch, or the
 * three kernels when kernel timing is enabled on the plan's context (same
 * kernels and arguments, bracketed by timing events). */
capart_status capart_run_batch(capart_plan *plan, void *hip_stream);
capart_status capart_plan_get_info(const capart_plan *plan, capart_plan_info *info);
capart_status capart_plan_destroy(capart_plan *plan);

/*
 * Serving form.  A server keeps admitted queries (one task set each) resident
 * in a device arena of a fixed memory budget: per-query inputs, workspace and
 * results live in ring buffers indexed by query slot and task index.
 * capart_server_submit admits a query if a slot and a contiguous range of the
 * task ring are free, else returns E_AGAIN (back-pressure); it copies the
 * query into pinned host staging and returns a ticket.  A dispatcher thread
 * launches every admitted, not yet launched query as one batch on the next
 * free stream (up to `streams` batches in flight), so queries that arrive while
 * others are on the GPU start at once and their work overlaps on the device
 * (continuous batching).  capart_server_poll returns a query's results once
 * its batch has completed and frees its ring space.  A query's results do not
 * depend on the other queries of its batch.  submit and poll are thread-safe.
 * With CAPART_SERVER_TABLES in cfg.flags a query may bring explicit time
 * tables (its table_offset[0] .. + n * M entries of Cn_table and Cc_table are
 * copied at submit; their domain is checked on the device, as for
 * capart_solve, giving the query status E_RANGE); a batch then holds queries
 * of one kind only, with tables or without.  The device budget counts
 * 16 * max_M more bytes per task for them.
 * Latency is measured from submit (or the replayed arrival time) to the moment
 * the dispatcher sees the batch complete.
 */
typedef struct capart_server capart_server;

typedef struct capart_server_config {
    int32_t K, alloc_mode;  /* options applied to every query (heuristic modes) */
    uint32_t flags;         /* CAPART_FLAG_SKIP_1G, _NO_LEMMA1, CAPART_SERVER_TABLES */
    int32_t max_tasks;      /* bound on tasks per query, 1..64        */
    int32_t max_M;          /* bound on M per query, 1..255           */
    int32_t max_queries;    /* query slots (0 = 4096)                 */
    int64_t device_bytes;   /* device budget for resident queries (0 = 256 MiB) */
    int32_t streams;        /* batches in flight, 1..8 (0 = 4)        */
    int32_t max_batch;      /* queries per launch (0 = no limit)      */
    int32_t policy;         /* CAPART_POLICY_FP_DM (0) or CAPART_POLICY_EDF, every query */
    uint64_t admissible[4]; /* allowed part sizes for every query (as capart_options), all 0 = every size */
} capart_server_config;

typedef struct capart_server_stats {
    int64_t submitted, completed, rejected, batches, evals;
    double p50_us, p99_us, mean_us, max_us;  /* latency over completed queries   */
    double elapsed_s, queries_per_s, evals_per_s, mean_batch;
} capart_server_stats;

capart_status capart_server_create(capart_ctx *ctx, const capart_server_config *cfg, capart_server **out);
/* one_set: host pointers, one set with offsets {0, n}. */
capart_status capart_server_submit(capart_server *srv, const capart_tasksets *one_set, uint64_t *ticket);
/* one_out: host pointers sized for one set (sizes[K], per-task arrays[n]);
 * *done = 1 and one_out filled when complete, else *done = 0. E_INVAL for an
 * unknown or already collected ticket. */
capart_status capart_server_poll(capart_server *srv, uint64_t ticket, capart_results *one_out, int32_t *done);
/* Statistics since creation or the last reset (reset != 0 clears them). */
capart_status capart_server_stats_get(capart_server *srv, capart_server_stats *out, int32_t reset);
/* Open-loop replay: submits the sets of `queries` (host pointers) at their
 * arrival times (microseconds from the start of the call), retrying rejected
 * queries as soon as space frees, collects every result into `results` (host,
 * sized for the whole batch, may be NULL) and returns the statistics of the
 * replay in *stats. */
capart_status capart_server_replay(capart_server *srv, const capart_tasksets *queries, const double *arrival_us,
                                   capart_results *results, capart_server_stats *stats);
capart_status capart_server_destroy(capart_server *srv);

/* Launch tuning of a context (applies to later calls on it).  Every choice
 * computes identical results; they trade divergence, occupancy and block
 * count.  threads: threads per evaluation block, 0 = automatic, else 64, 128,
 * 192 or 256 (reduced automatically when a set's LDS tables need it); chunk:
 * partitionings per evaluation block, 0 = automatic (enough blocks to fill the
 * chip); loop_form: 0 = automatic, 1 = each lane runs the heuristic of one
 * partitioning per loop step, 2 = each loop step is one candidate test (a lane
 * that finishes a partitioning continues with its next one at the next step),
 * 3 = as 1, but sets served by the test memo run a state machine in which
 * lanes advance through memo answers and run the tests the memo cannot answer
 * together (K <= 4; otherwise as 1).
 * exh_form (exhaustive mode): 0 = automatic, 1 = every block enumerates all
 * k^n allocations of one partitioning, 2 = per-set subset tables of partition
 * utilisation (every task subset on every size) and a depth-first search in
 * allocation-index order with exact pruning (sets of at most 14 tasks, K <= 4;
 * otherwise form 1 is used).  frontier (heuristic modes): 0 = automatic (on),
 * 1 = on, 2 = off; when on, a set of at most 14 tasks first gets its
 * feasibility frontier (for every task subset, the fewest units that schedule
 * it, by exact tests) and every candidate test of the heuristic on every
 * partitioning becomes a lookup in it.  memo (heuristic modes, loop form 1,
 * sets of more tasks than the frontier takes and at most 32): 0 = automatic
 * (2^11 entries, fewer if the LDS is short), -1 = off, 8..13 = log2 of the
 * entries of a per-set table in LDS that records, for each task subset met,
 * the largest size known to fail and the smallest known to pass, so that
 * repeated candidate tests across partitionings become lookups.
 * wide_chunk (heuristic modes, sets of more than 32 tasks): 0 = automatic
 * (16), -1 = off, else 1..4096: partitionings per block of a launch in which
 * each wave runs the heuristic of one partitioning at a time with the exact
 * tests of a candidate part spread over the wave, one lane per member; off:
 * such sets run one partitioning per lane like the others (more throughput
 * on large batches of wide sets, much longer latency per set).  NULL
 * restores the automatic choices.
 * E_INVAL for values out of range. */
typedef struct capart_tuning {
    int32_t threads;
    int32_t chunk;
    int32_t loop_form;
    int32_t exh_form;
    int32_t frontier;
    int32_t memo;
    int32_t wide_chunk;
    int32_t reserved;  /* must be 0 */
} capart_tuning;
capart_status capart_set_tuning(capart_ctx *ctx, const capart_tuning *tuning);
capart_status capart_get_tuning(const capart_ctx *ctx, capart_tuning *tuning);

/* Algorithmic work of a solve, counted exactly (for roofline accounting; not
 * for timing).  Heuristic modes, by a counting variant of the evaluation
 * kernel: counts[0] = response-time terms (per fixed-point iteration, one plus
 * one per higher-priority term), counts[1] = exact partition tests, counts[2]
 * = candidate tests answered from a feasibility frontier.  Exhaustive mode,
 * in its subset-table form (sets of at most 14 tasks, K <= 4): counts[0] and
 * counts[1] = the terms and tests of filling the subset tables, counts[2] =
 * table lookups of the pruned search.  Same arguments as capart_solve_async
 * (device pointers); results are written as by it.  Synchronous.  E_INVAL
 * for per-set launches and for exhaustive batches outside the table form. */
capart_status capart_count_work(capart_ctx *ctx, const capart_tasksets *dev_in, const capart_options *opt,
                                capart_results *dev_out, void *hip_stream, int64_t *counts);
/* Algorithmic work of Algorithm 1 (capart_alg1_async), counted by a counting
 * variant of its kernel: counts[0] = response-time terms, counts[1] = exact
 * partition tests (each Algorithm 2 size tried by its binary search).  Same
 * arguments as capart_alg1_async; results are written as by it.  Synchronous. */
capart_status capart_alg1_count_work(capart_ctx *ctx, const capart_tasksets *dev_in, const capart_options *opt,
                                     capart_alg1_results *dev_out, void *hip_stream, int64_t *counts);

/* Kernel timing.  While enabled on a context, every launch sequence of
 * capart_solve / capart_solve_async records HIP events on its own stream
 * before and after the prep, eval and final kernels (one sequence per batch,
 * or per set with CAPART_FLAG_PER_SET_LAUNCH); capart_alg1 / capart_alg1_async
 * record the same way, with the Algorithm 1 kernel as "eval" and no final.  capart_timing_read waits for
 * the recorded events, returns the summed durations in milliseconds
 * (ms[0] prep, ms[1] eval, ms[2] final) and the number of launches of each
 * (launches[3]), and clears them.  Disabling drops unread records. */
capart_status capart_timing_enable(capart_ctx *ctx, int enable);
capart_status capart_timing_read(capart_ctx *ctx, double *ms, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* CAPART_H */
