// Internal interface between the C-ABI host code and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "capart.h"

namespace capart {

// Per-task record in deadline-monotonic rank order (32 bytes).  clo/chi hold
// c = ceil(2^64 / T) so that floor(x / T) = (c * x) >> 64 for every 32-bit x
// (T >= 2; Lemire, Kaser & Kurz, "Faster remainder by direct computation").
struct TaskRec {
    uint32_t T, D, Cs, Cp;
    uint32_t k, clo, chi;
    uint16_t mmin;  // Lemma 2: least m with Cn(m) <= D, 0xFFFF if none <= M
    uint8_t orig;   // index of the task inside its set
    uint8_t mem;    // 1 = memory-intensive
};
static_assert(sizeof(TaskRec) == 32, "TaskRec layout");

constexpr uint32_t SETF_VALID = 1u;
constexpr uint32_t SETF_LEMMA1 = 2u;  // Lemma 1 rejects the set
constexpr uint32_t SETF_EDF = 4u;     // the set's partitions are scheduled by EDF (else fixed-priority DM)
constexpr uint32_t SETF_NOFIT = 8u;   // no partitioning into at most K parts can be schedulable (prep's bound)

// Partition-count table: NP(r, j, x) = number of partitions of r into at most
// j parts, each part <= x (parts >= 1); r, x in [0, 255], j in [0, 8].
constexpr int NP_R = 256, NP_J = 9, NP_X = 256;
__host__ __device__ inline int np_index(int j, int r, int x) { return (j * NP_R + r) * NP_X + x; }

struct Batch {           // device pointers of the caller's batch (set range [s0, s0+S))
    const int64_t *off;
    const int32_t *M;
    const int64_t *T, *D, *Cs, *Cp;
    const int32_t *k;
    const uint8_t *type;
    int64_t n_tasks_total;
    int32_t max_tasks, max_M;
    // explicit time tables (nullptr: the parametric model): set s's task i on m
    // units at Cn/Cc[toff[s] + i*M + m-1]
    const int64_t *toff = nullptr, *Cn = nullptr, *Cc = nullptr;
    int64_t tlen = 0;
};

// One unit of batched (persistent-kernel) work: partitionings [p0, p1) of a
// set; its best key goes to partial slot `slot`.
struct WorkItem {
    uint32_t set, p0, p1, slot;
};

struct Work {            // device workspace owned by the context
    TaskRec *rec;        // [N]
    uint64_t *forbid;    // [N] ACT forbidden-pair masks, by rank
    uint8_t *sigma;      // [N] ranks in decreasing one-unit utilisation
    uint32_t *setflags;  // [S]
    uint64_t *memmask;   // [S] memory-intensive ranks
    uint64_t *partial;   // [S * CH * 4] best key per (set, chunk), or per item slot
    const uint32_t *np;  // partition-count table
    const uint16_t *order;  // subsets of {0..n-1} by size then value, n = 1..FRONTIER_MAX_TASKS,
                            // the list for n at entry 2^n - 2 (frontier build)
    // batched form only
    const WorkItem *items;     // [n_items], largest first
    uint32_t n_items;
    uint32_t *counter;         // [3] next item to take, per queue (reset by the prep kernel)
    uint32_t class_end[3];     // items of size class i are [class_end[i-1], class_end[i]) (one queue each)
    const uint32_t *slot_off;  // [S + 1] partial slots of each set
    // counting variant of the evaluation kernel only
    uint64_t *counters;        // [3]: response-time terms, exact tests, frontier lookups
    // explicit time tables of the batch (as in Batch; read when staging a set)
    const int64_t *toff = nullptr, *tCn = nullptr, *tCc = nullptr;
};

struct Out {             // device pointers of the caller's results
    int32_t *status;
    uint8_t *verdict, *verdict_1g;
    int32_t *pidx, *sizes;
    int64_t *aidx;
    uint64_t *maxU, *sumU;
    int64_t *n_evals;
    int8_t *alloc;
    int64_t *R, *R_1g;
    uint64_t *dbg_key;
    const int64_t *dbg_offset;
};

// Admissible partition sizes: size m is allowed iff bit m of the 256-bit mask
// w[0..3] is set; an all-zero mask allows every size.
struct Adm {
    uint64_t w[4] = {0, 0, 0, 0};
};

struct Launch {
    int64_t s0, S;       // set range
    int K, mode;
    uint32_t flags;
    int chunks;          // CH: chunks per set
    uint32_t chunk;      // partitionings per chunk (heuristic) / 1 (exhaustive)
    int threads;         // threads per evaluation block
    int table_words;     // u32 words of dynamic LDS reserved for the per-set tables
    int form;            // heuristic loop form: 1 = one step per partitioning, 2 = one step per candidate test
    int exh_form;        // exhaustive: 1 = enumerate every allocation, 2 = subset tables + pruned search
    int front_n;         // heuristic: sets of at most front_n tasks use the feasibility frontier (0 = never)
    int front_words;     // u32 words of dynamic LDS reserved for the frontier (2^front_n u16)
    int memo_log2 = 0;   // heuristic, sets of front_n < n <= 32 tasks: 2^memo_log2 memo entries (0 = no memo);
                         // the memo shares the frontier's LDS region (a set uses one or the other)
    int memo_packed = 0; // 1: memo sets run the packed-test state machine instead of the nested loops
    int n_lo = 0;        // this evaluation launch takes the sets of n_lo <= n (<= n_hi if n_hi > 0) tasks
    int n_hi = 0;
    Adm adm;             // admissible part sizes (a partitioning with another size is infeasible)
    int edf = 0;         // 1: per-partition EDF (processor demand) instead of fixed-priority DM
    int wchunk = 0;      // heuristic, sets above NARROW_MAX_TASKS tasks: partitionings per block of the
                         // wave-per-partitioning launch (0 = one lane per partitioning, chunk per block);
                         // chunks then covers ceil(P / wchunk) as well
};

// Host-side sizing helpers shared by the launchers.
size_t table_lds_bytes(int max_tasks, int max_M);
int eval_threads(int max_tasks, int max_M);
// largest set size answered through the feasibility frontier
constexpr int FRONTIER_MAX_TASKS = 14;
// A heuristic launch is split by set size into up to three launches, each
// compiled for its own path and reserving only the LDS its sets use: sets of
// at most front_n tasks (frontier), of at most NARROW_MAX_TASKS (32-bit rank
// masks, test memo) and larger ones (64-bit masks).  Fills the classes' upper
// task counts (ascending) and returns how many there are (0: no split).
int size_classes(const Launch &L, int max_tasks, int hi[3]);
// largest set size with 32-bit rank masks
constexpr int NARROW_MAX_TASKS = 32;
// partitionings per block of the wide-set (wave-per-partitioning) launch by default
constexpr int WIDE_CHUNK_DEFAULT = 8;
// automatic choice of that launch: while a batch's wide sets have fewer
// partitionings than this (one lane each would leave the chip idle, so one
// partitioning's whole heuristic in one lane sets the latency), or, where the
// host does not see the sets, while the batch has at most WIDE_WAVE_MAX_SETS sets
constexpr int64_t WIDE_LANE_FILL = 65536;
constexpr int64_t WIDE_WAVE_MAX_SETS = 64;
// test memo (sets between the frontier limit and 32 tasks): default and
// largest log2 of its entries (8 bytes each)
constexpr int MEMO_DEFAULT_LOG2 = 11;
constexpr int MEMO_MAX_LOG2 = 13;

hipError_t launch_prep(const Batch &b, const Work &w, const Out &o, const Launch &L, hipStream_t st);
// Algorithm 1 (free partition sizes): device pointers of the results
struct A1Out {
    int32_t *status;
    uint8_t *verdict;
    int32_t *nparts;
    int32_t *sizes;   // [N]: set s's part sizes from set_offset[s], par_list order, 0-padded
    int8_t *alloc;    // [N]
    int64_t *R;       // [N]
    int64_t *tried, *merged;
    uint64_t *workload;  // [S] or nullptr
};
// count: the counting variant (adds response-time terms and exact tests to w.counters[0..1])
hipError_t launch_alg1(const Batch &b, const Work &w, const A1Out &o, const Launch &L, hipStream_t st,
                       bool count = false);
// Algorithm 1 for batches with sets of more than 64 tasks (fixed priority): its
// own prep kernel, then one block of 256 threads per set.
hipError_t launch_prep_big(const Batch &b, const Work &w, const Out &o, const Launch &L, hipStream_t st);
hipError_t launch_alg1_big(const Batch &b, const Work &w, const A1Out &o, const Launch &L, hipStream_t st,
                           bool count);
hipError_t allow_alg1_big();
hipError_t launch_eval(const Batch &b, const Work &w, const Out &o, const Launch &L, hipStream_t st);
// evaluation restricted to partitioning indices [p_lo, p_hi)
hipError_t launch_eval_range(const Batch &b, const Work &w, const Out &o, const Launch &L, hipStream_t st,
                             uint32_t p_lo, uint32_t p_hi);
hipError_t launch_final(const Batch &b, const Work &w, const Out &o, const Launch &L, hipStream_t st);
// batched form: persistent evaluation over the work items with `blocks` blocks
hipError_t launch_eval_persistent(const Batch &b, const Work &w, const Out &o, const Launch &L, int blocks,
                                  hipStream_t st);
int device_cu_count();
// exhaustive allocation through subset tables (<= 14 tasks per set, <= 4 parts)
constexpr int SUBSET_MAX_TASKS = 14;
hipError_t launch_subset_tables(const Batch &b, const Work &w, const Launch &L, uint64_t *tab, int64_t s_begin, int W,
                                int Mtab, int ntab, hipStream_t st);
hipError_t launch_exh_dfs(const Batch &b, const Work &w, const Out &o, const Launch &L, const uint64_t *tab,
                          int64_t s_begin, int W, int Mtab, int ntab, uint32_t Pmax, uint32_t p_lo, uint32_t p_hi,
                          hipStream_t st);
hipError_t launch_triple(const Batch &b, const Work &w, const int32_t *sizes, int k, const int8_t *alloc,
                         uint8_t *feasible, int64_t *R, uint64_t *maxU, uint64_t *sumU, hipStream_t st);
hipError_t configure_kernels();
// Device address of this GPU's no-allocation workspace (current device).
hipError_t scratch_address(void **ptr);
// Full-rate 32-bit VALU lane-operations per second, measured.
hipError_t measure_valu(hipStream_t st, double *lane_ops_per_s, double *best_ms);
// counting variant of the heuristic evaluation (w.counters must be set)
hipError_t launch_eval_count(const Batch &b, const Work &w, const Out &o, const Launch &L, hipStream_t st);

}  // namespace capart
