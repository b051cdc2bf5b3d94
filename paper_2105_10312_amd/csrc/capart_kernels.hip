// gfx950 kernels of the contention-aware partitioning engine: the
// non-template kernels (prep, exhaustive subset tables and search), the
// exhaustive, final and one-triple kernels, and the host dispatch that picks
// each launch's compiled path (size class, rank-mask width, part count,
// policy, loop form).  Device code lives in capart_device.h.
//
// Work decomposition (one HIP stream, three launches per batch):
//   prep  : one wave per task set -- validation, deadline-monotonic ranks,
//           Lemma 1 and Lemma 2, heuristic order, exact-division constants,
//           ACT forbidden pairs; writes a packed per-task record.
//   eval  : one block per (set, chunk of partitionings), or a persistent grid
//           over work items; heuristic or exhaustive allocation per
//           partitioning; one partial key per block or item.
//   final : one wave per set -- reduces the partials, rebuilds the chosen
//           allocation, computes response times of the chosen triple and of
//           the whole-GPU baseline and writes the results.
#define CAPART_MAIN_TU
#include "capart_device.h"

namespace capart {

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

hipError_t launch_prep(const Batch &b, const Work &w, const Out &o, const Launch &L, hipStream_t st)
{
    if (L.S <= 0) return hipSuccess;
    hipLaunchKernelGGL(prep_kernel, dim3((unsigned)L.S), dim3(64), 0, st, b, w, o, L);
    return hipGetLastError();
}

// largest set size of a launch
static int launch_max_n(const Launch &L, const Batch &b) { return L.n_hi > 0 ? min(L.n_hi, b.max_tasks) : b.max_tasks; }

// Threads per block of a loop-form-1 launch whose LDS per block leaves room
// for only a few blocks on a compute unit (large per-set tables): wider
// blocks keep 16 or more waves per compute unit.  Frontier and form-2 launches
// keep their width (the frontier build and form 2's lane state assume at
// most 256 threads).
static Launch fit_block(const Launch &L, const Batch &b)
{
    Launch C = L;
    if (L.mode == CAPART_EXHAUSTIVE || L.form != 1) return C;
    const bool narrow = launch_max_n(L, b) <= NARROW_MAX_TASKS;
    const size_t dyn = (size_t)4 * L.table_words + (narrow && L.memo_log2 > 0 ? (size_t)8 << L.memo_log2 : 0);
    const size_t per_block = dyn + 8 * 1024;  // with the static per-set arrays
    const int fit = (int)((size_t)160 * 1024 / per_block);
    if (fit <= 2) C.threads = 512;
    else if (fit <= 4) C.threads = max(C.threads, 256);
    return C;
}

// Every set of the launch is at most front_n tasks (a frontier launch).
static bool frontier_launch(const Launch &L, const Batch &b)
{
    return L.mode != CAPART_EXHAUSTIVE && L.front_n > 0 && launch_max_n(L, b) <= L.front_n;
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
    const int form = frontier_launch(L, b) ? 0 : (L.form == 2 ? 2 : 1);
    return L.edf ? HeurLaunch<KMAX, MT, POL_EDF>::eval(b, w, o, L, st, p_lo, p_hi, form)
                 : HeurLaunch<KMAX, MT, POL_FP>::eval(b, w, o, L, st, p_lo, p_hi, form);
}

template <int KMAX, typename MT>
static hipError_t launch_persistent_f(const Batch &b, const Work &w, const Out &o, const Launch &L, int blocks,
                                      hipStream_t st)
{
    const int form = frontier_launch(L, b) ? 0 : (L.form == 2 ? 2 : 1);
    return L.edf ? HeurLaunch<KMAX, MT, POL_EDF>::persistent(b, w, o, L, blocks, st, form)
                 : HeurLaunch<KMAX, MT, POL_FP>::persistent(b, w, o, L, blocks, st, form);
}

int size_classes(const Launch &L, int max_tasks, int hi[3])
{
    if (L.mode == CAPART_EXHAUSTIVE || L.n_lo > 0 || L.n_hi > 0) return 0;
    int c = 0;
    if (L.front_n > 0) hi[c++] = min(L.front_n, max_tasks);
    const int prev = c ? hi[c - 1] : 0;
    if (max_tasks > prev && prev < NARROW_MAX_TASKS) hi[c++] = min(max_tasks, NARROW_MAX_TASKS);
    if (max_tasks > NARROW_MAX_TASKS) hi[c++] = max_tasks;
    return c;
}

// The launch of size class i: its task range, tables for its largest set,
// and the frontier region (frontier class) or the memo (others).
static Launch class_launch(const Launch &L, const Batch &b, const int hi[3], int i)
{
    Launch C = L;
    C.n_lo = i > 0 ? hi[i - 1] + 1 : 0;
    C.n_hi = hi[i];
    C.table_words = (int)(table_lds_bytes(hi[i], min(b.max_M, 255)) / 4);
    const bool front = L.front_n > 0 && hi[i] <= L.front_n;
    if (front) C.memo_log2 = 0; else C.front_words = 0;
    return C;
}

static hipError_t launch_eval_persistent_one(const Batch &b, const Work &w, const Out &o, const Launch &L0, int blocks,
                                             hipStream_t st)
{
    const Launch L = frontier_launch(L0, b) ? L0 : fit_block(L0, b);
    if (launch_max_n(L, b) <= 32)
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

// The wide-set launch (sets above NARROW_MAX_TASKS tasks) in its wave-per-
// partitioning form: 512-thread blocks (eight waves share one staged table),
// the execution-time table only.
static bool wide_launch(const Launch &L) { return L.mode != CAPART_EXHAUSTIVE && L.wchunk > 0 && L.n_lo > NARROW_MAX_TASKS; }

static hipError_t launch_wide(const Batch &b, const Work &w, const Out &o, const Launch &L, hipStream_t st,
                              bool count, uint32_t p_lo, uint32_t p_hi)
{
    return L.edf ? WideLaunch<POL_EDF>::eval(L.K, count, b, w, o, L, st, p_lo, p_hi)
                 : WideLaunch<POL_FP>::eval(L.K, count, b, w, o, L, st, p_lo, p_hi);
}

template <int KMAX, typename MT>
static hipError_t launch_count_pol(const Batch &b, const Work &w, const Out &o, const Launch &L, hipStream_t st,
                                   int form)
{
    return L.edf ? HeurLaunch<KMAX, MT, POL_EDF>::count(b, w, o, L, st, form)
                 : HeurLaunch<KMAX, MT, POL_FP>::count(b, w, o, L, st, form);
}

static hipError_t launch_eval_count_one(const Batch &b, const Work &w, const Out &o, const Launch &L0, hipStream_t st)
{
    if (wide_launch(L0)) return launch_wide(b, w, o, L0, st, true, 0u, 0xFFFFFFFFu);
    const Launch L = frontier_launch(L0, b) ? L0 : fit_block(L0, b);
    const int form = frontier_launch(L, b) ? 0 : 1;
    if (launch_max_n(L, b) <= 32)
        return L.K <= 4 ? launch_count_pol<4, uint32_t>(b, w, o, L, st, form)
                        : launch_count_pol<8, uint32_t>(b, w, o, L, st, form);
    return L.K <= 4 ? launch_count_pol<4, uint64_t>(b, w, o, L, st, form)
                    : launch_count_pol<8, uint64_t>(b, w, o, L, st, form);
}

static hipError_t launch_eval_range_one(const Batch &b, const Work &w, const Out &o, const Launch &L0, hipStream_t st,
                                        uint32_t p_lo, uint32_t p_hi)
{
    if (wide_launch(L0)) return launch_wide(b, w, o, L0, st, false, p_lo, p_hi);
    const Launch L = (L0.mode == CAPART_EXHAUSTIVE || frontier_launch(L0, b)) ? L0 : fit_block(L0, b);
    // 32-bit rank masks when every set of the launch has at most 32 tasks
    if (launch_max_n(L, b) <= 32)
        return L.K <= 4 ? launch_eval_k<4, uint32_t>(b, w, o, L, st, p_lo, p_hi)
                        : launch_eval_k<8, uint32_t>(b, w, o, L, st, p_lo, p_hi);
    return L.K <= 4 ? launch_eval_k<4, uint64_t>(b, w, o, L, st, p_lo, p_hi)
                    : launch_eval_k<8, uint64_t>(b, w, o, L, st, p_lo, p_hi);
}

hipError_t launch_eval_range(const Batch &b, const Work &w, const Out &o, const Launch &L, hipStream_t st,
                             uint32_t p_lo, uint32_t p_hi)
{
    if (L.S <= 0) return hipSuccess;
    int hi[3];
    const int nc = size_classes(L, b.max_tasks, hi);
    if (nc <= 1) return launch_eval_range_one(b, w, o, L, st, p_lo, p_hi);
    for (int i = 0; i < nc; i++) {
        const hipError_t e = launch_eval_range_one(b, w, o, class_launch(L, b, hi, i), st, p_lo, p_hi);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_eval(const Batch &b, const Work &w, const Out &o, const Launch &L, hipStream_t st)
{
    return launch_eval_range(b, w, o, L, st, 0u, 0xFFFFFFFFu);
}

hipError_t launch_eval_count(const Batch &b, const Work &w, const Out &o, const Launch &L, hipStream_t st)
{
    if (L.S <= 0 || L.mode == CAPART_EXHAUSTIVE) return hipSuccess;
    int hi[3];
    const int nc = size_classes(L, b.max_tasks, hi);
    if (nc <= 1) return launch_eval_count_one(b, w, o, L, st);
    for (int i = 0; i < nc; i++) {
        const hipError_t e = launch_eval_count_one(b, w, o, class_launch(L, b, hi, i), st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Batched form: the items of each size class are contiguous in the item list
// (classes ascending) and form a queue of their own (counter[i]).
hipError_t launch_eval_persistent(const Batch &b, const Work &w, const Out &o, const Launch &L, int blocks,
                                  hipStream_t st)
{
    int hi[3];
    const int nc = size_classes(L, b.max_tasks, hi);
    if (nc <= 1) return launch_eval_persistent_one(b, w, o, L, blocks, st);
    for (int i = 0; i < nc; i++) {
        const uint32_t begin = i > 0 ? w.class_end[i - 1] : 0u, end = w.class_end[i];
        if (end <= begin) continue;
        Work wc = w;
        wc.items = w.items + begin;
        wc.n_items = end - begin;
        wc.counter = w.counter + i;
        const hipError_t e = launch_eval_persistent_one(b, wc, o, class_launch(L, b, hi, i), blocks, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_alg1(const Batch &b, const Work &w, const A1Out &o, const Launch &L, hipStream_t st, bool count)
{
    if (L.S <= 0) return hipSuccess;
    return L.edf ? Alg1Launch<POL_EDF>::run(count, b, w, o, L, st) : Alg1Launch<POL_FP>::run(count, b, w, o, L, st);
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

// ---------------------------------------------------------------------------
// Workspace of the no-allocation entry point (capart_solve_async_noalloc): a
// file-scope device array, one copy per GPU, held until the process ends.
// Host code never names it in a launch: it takes the device address that
// hipGetSymbolAddress returns for the current device (scratch_address).
static __device__ __align__(256) uint8_t scratch[CAPART_NOALLOC_SCRATCH_BYTES];

hipError_t scratch_address(void **ptr)
{
    *ptr = nullptr;
    return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch));
}

// ---------------------------------------------------------------------------
// Integer VALU throughput: every lane runs eight independent chains of
// full-rate 32-bit adds (v_add_u32), 32 per loop step, written as inline asm
// so that the compiler can neither fold the chains nor change the operation.
// Lane-operations = blocks x threads x iters x 32.
__global__ __launch_bounds__(256) void valu_peak_kernel(uint32_t *sink, uint32_t iters)
{
    uint32_t a0 = threadIdx.x, a1 = a0 + 1u, a2 = a0 + 2u, a3 = a0 + 3u, a4 = a0 + 4u, a5 = a0 + 5u, a6 = a0 + 6u,
             a7 = a0 + 7u;
    const uint32_t k = blockIdx.x | 1u;
    for (uint32_t i = 0; i < iters; i++) {
#pragma unroll
        for (int r = 0; r < 4; r++)
            asm volatile(
                "v_add_u32 %0, %0, %8\n\t"
                "v_add_u32 %1, %1, %8\n\t"
                "v_add_u32 %2, %2, %8\n\t"
                "v_add_u32 %3, %3, %8\n\t"
                "v_add_u32 %4, %4, %8\n\t"
                "v_add_u32 %5, %5, %8\n\t"
                "v_add_u32 %6, %6, %8\n\t"
                "v_add_u32 %7, %7, %8"
                : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)
                : "v"(k));
    }
    const uint32_t x = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;
    if (x == 0x9E3779B9u) sink[blockIdx.x] = x;  // keeps the chains live; the store is almost never taken
}

// Best of three timed launches of valu_peak_kernel over 8 blocks of 256
// threads per compute unit (eight waves per SIMD).
hipError_t measure_valu(hipStream_t st, double *lane_ops_per_s, double *best_ms)
{
    const int blocks = device_cu_count() * 8;
    const uint32_t iters = 20000;
    uint32_t *sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc((void **)&sink, sizeof(uint32_t) * (size_t)blocks);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float best = 0.0f;
    for (int rep = 0; rep < 4 && e == hipSuccess; rep++) {
        (void)hipEventRecord(e0, st);
        hipLaunchKernelGGL(valu_peak_kernel, dim3((unsigned)blocks), dim3(256), 0, st, sink, iters);
        if ((e = hipGetLastError()) != hipSuccess) break;
        (void)hipEventRecord(e1, st);
        if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
        float ms = 0.0f;
        if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
        if (rep > 0 && (best == 0.0f || ms < best)) best = ms;  // the first launch warms up
    }
    if (e == hipSuccess) {
        *best_ms = best;
        *lane_ops_per_s = (double)blocks * 256.0 * iters * 32.0 / (best * 1e-3);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (sink) (void)hipFree(sink);
    return e;
}

// Let every kernel use all of the 160 KB LDS beyond its static arrays.
hipError_t configure_kernels()
{
    hipError_t e = hipSuccess, t;
#define CAPART_ALLOW(call) do { t = (call); if (t != hipSuccess) e = t; } while (0)
    CAPART_ALLOW(allow_lds(eval_exh_kernel<4>));
    CAPART_ALLOW(allow_lds(eval_exh_kernel<8>));
    CAPART_ALLOW((HeurLaunch<4, uint32_t, POL_FP>::allow()));
    CAPART_ALLOW((HeurLaunch<4, uint64_t, POL_FP>::allow()));
    CAPART_ALLOW((HeurLaunch<8, uint32_t, POL_FP>::allow()));
    CAPART_ALLOW((HeurLaunch<8, uint64_t, POL_FP>::allow()));
    CAPART_ALLOW((HeurLaunch<4, uint32_t, POL_EDF>::allow()));
    CAPART_ALLOW((HeurLaunch<4, uint64_t, POL_EDF>::allow()));
    CAPART_ALLOW((HeurLaunch<8, uint32_t, POL_EDF>::allow()));
    CAPART_ALLOW((HeurLaunch<8, uint64_t, POL_EDF>::allow()));
    CAPART_ALLOW(WideLaunch<POL_FP>::allow());
    CAPART_ALLOW(WideLaunch<POL_EDF>::allow());
    CAPART_ALLOW(Alg1Launch<POL_FP>::allow());
    CAPART_ALLOW(Alg1Launch<POL_EDF>::allow());
    CAPART_ALLOW(allow_alg1_big());
    CAPART_ALLOW(allow_lds(subset_table_kernel));
    CAPART_ALLOW(allow_lds(final_kernel<4>));
    CAPART_ALLOW(allow_lds(final_kernel<8>));
    CAPART_ALLOW(allow_lds(triple_kernel<8>));
#undef CAPART_ALLOW
    (void)hipGetLastError();  // leave no sticky error behind for the next launch check
    return e;
}

}  // namespace capart
