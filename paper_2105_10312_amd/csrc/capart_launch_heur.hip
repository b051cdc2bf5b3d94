// Launchers of the heuristic evaluation kernels for one (part count, rank-mask
// width, policy): the direct, persistent and counting grids in every loop form
// and order.  Built once per combination (CAPART_I_K, CAPART_I_MT,
// CAPART_I_POL), so the kernel instantiations compile in parallel.
#include "capart_device.h"

#if !defined(CAPART_I_K) || !defined(CAPART_I_MT) || !defined(CAPART_I_POL)
#error "build with -DCAPART_I_K=<4|8> -DCAPART_I_MT=<uint32_t|uint64_t> -DCAPART_I_POL=<POL_FP|POL_EDF>"
#endif

namespace capart {

template <int KMAX, typename MT>
static size_t heur_dyn_bytes(const Launch &L, int form)
{
    const size_t front = (size_t)4 * L.front_words;
    const size_t memo = (form == 1 && sizeof(MT) == 4 && L.memo_log2 > 0) ? (size_t)8 << L.memo_log2 : 0;
    if (form == 0) return (size_t)4 * L.table_words + front;
    return (size_t)4 * L.table_words + (front > memo ? front : memo) +
           (form == 2 ? (size_t)L.threads * KMAX * (sizeof(MT) + sizeof(uint64_t)) : 0);
}

template <int KMAX, typename MT, int FORM, bool COUNT, int POL>
static hipError_t launch_heur(const Launch &L, const Batch &b, const Work &w, const Out &o, hipStream_t st,
                              uint32_t p_lo, uint32_t p_hi)
{
    const dim3 grid((unsigned)(L.S * L.chunks)), block((unsigned)L.threads);
    const size_t lds = heur_dyn_bytes<KMAX, MT>(L, FORM);
    switch (L.mode) {
    case CAPART_HEUR_BF_INA:
        hipLaunchKernelGGL((eval_heur_kernel<KMAX, false, false, MT, FORM, COUNT, POL>), grid, block, lds, st, b, w, o,
                           L, p_lo, p_hi);
        break;
    case CAPART_HEUR_BF_ACT:
        hipLaunchKernelGGL((eval_heur_kernel<KMAX, true, false, MT, FORM, COUNT, POL>), grid, block, lds, st, b, w, o, L,
                           p_lo, p_hi);
        break;
    case CAPART_HEUR_SMS_INA:
        hipLaunchKernelGGL((eval_heur_kernel<KMAX, false, true, MT, FORM, COUNT, POL>), grid, block, lds, st, b, w, o, L,
                           p_lo, p_hi);
        break;
    default:
        hipLaunchKernelGGL((eval_heur_kernel<KMAX, true, true, MT, FORM, COUNT, POL>), grid, block, lds, st, b, w, o, L,
                           p_lo, p_hi);
        break;
    }
    return hipGetLastError();
}

template <int KMAX, typename MT, int FORM, int POL>
static hipError_t launch_persistent(const Batch &b, const Work &w, const Out &o, const Launch &L, int blocks,
                                    hipStream_t st)
{
    const dim3 grid((unsigned)blocks), block((unsigned)L.threads);
    const size_t lds = heur_dyn_bytes<KMAX, MT>(L, FORM);
    switch (L.mode) {
    case CAPART_HEUR_BF_INA:
        hipLaunchKernelGGL((eval_persistent_kernel<KMAX, false, false, MT, FORM, POL>), grid, block, lds, st, b, w, o, L);
        break;
    case CAPART_HEUR_BF_ACT:
        hipLaunchKernelGGL((eval_persistent_kernel<KMAX, true, false, MT, FORM, POL>), grid, block, lds, st, b, w, o, L);
        break;
    case CAPART_HEUR_SMS_INA:
        hipLaunchKernelGGL((eval_persistent_kernel<KMAX, false, true, MT, FORM, POL>), grid, block, lds, st, b, w, o, L);
        break;
    default:
        hipLaunchKernelGGL((eval_persistent_kernel<KMAX, true, true, MT, FORM, POL>), grid, block, lds, st, b, w, o, L);
        break;
    }
    return hipGetLastError();
}

template <int KMAX, typename MT, int POL>
hipError_t HeurLaunch<KMAX, MT, POL>::eval(const Batch &b, const Work &w, const Out &o, const Launch &L,
                                           hipStream_t st, uint32_t p_lo, uint32_t p_hi, int form)
{
    if (form == 0) return launch_heur<KMAX, MT, 0, false, POL>(L, b, w, o, st, p_lo, p_hi);
    if (form == 2) return launch_heur<KMAX, MT, 2, false, POL>(L, b, w, o, st, p_lo, p_hi);
    return launch_heur<KMAX, MT, 1, false, POL>(L, b, w, o, st, p_lo, p_hi);
}

template <int KMAX, typename MT, int POL>
hipError_t HeurLaunch<KMAX, MT, POL>::persistent(const Batch &b, const Work &w, const Out &o, const Launch &L,
                                                 int blocks, hipStream_t st, int form)
{
    if (form == 0) return launch_persistent<KMAX, MT, 0, POL>(b, w, o, L, blocks, st);
    if (form == 2) return launch_persistent<KMAX, MT, 2, POL>(b, w, o, L, blocks, st);
    return launch_persistent<KMAX, MT, 1, POL>(b, w, o, L, blocks, st);
}

// The counting variant (algorithmic work tallies) over every partitioning.
template <int KMAX, typename MT, int POL>
hipError_t HeurLaunch<KMAX, MT, POL>::count(const Batch &b, const Work &w, const Out &o, const Launch &L,
                                            hipStream_t st, int form)
{
    if (form == 0) return launch_heur<KMAX, MT, 0, true, POL>(L, b, w, o, st, 0u, 0xFFFFFFFFu);
    return launch_heur<KMAX, MT, 1, true, POL>(L, b, w, o, st, 0u, 0xFFFFFFFFu);
}

template <int KMAX, typename MT, int FORM, bool COUNT, int POL>
static hipError_t allow_heur()
{
    hipError_t e = hipSuccess, t;
    if ((t = allow_lds(eval_heur_kernel<KMAX, false, false, MT, FORM, COUNT, POL>)) != hipSuccess) e = t;
    if ((t = allow_lds(eval_heur_kernel<KMAX, true, false, MT, FORM, COUNT, POL>)) != hipSuccess) e = t;
    if ((t = allow_lds(eval_heur_kernel<KMAX, false, true, MT, FORM, COUNT, POL>)) != hipSuccess) e = t;
    if ((t = allow_lds(eval_heur_kernel<KMAX, true, true, MT, FORM, COUNT, POL>)) != hipSuccess) e = t;
    if constexpr (!COUNT) {
        if ((t = allow_lds(eval_persistent_kernel<KMAX, false, false, MT, FORM, POL>)) != hipSuccess) e = t;
        if ((t = allow_lds(eval_persistent_kernel<KMAX, true, false, MT, FORM, POL>)) != hipSuccess) e = t;
        if ((t = allow_lds(eval_persistent_kernel<KMAX, false, true, MT, FORM, POL>)) != hipSuccess) e = t;
        if ((t = allow_lds(eval_persistent_kernel<KMAX, true, true, MT, FORM, POL>)) != hipSuccess) e = t;
    }
    return e;
}

// Raise the dynamic-LDS limit of every instantiation of this group (order
// variants, loop forms, counting variant).
template <int KMAX, typename MT, int POL>
hipError_t HeurLaunch<KMAX, MT, POL>::allow()
{
    hipError_t e = hipSuccess, t;
    if ((t = allow_heur<KMAX, MT, 0, false, POL>()) != hipSuccess) e = t;
    if ((t = allow_heur<KMAX, MT, 1, false, POL>()) != hipSuccess) e = t;
    if ((t = allow_heur<KMAX, MT, 2, false, POL>()) != hipSuccess) e = t;
    if ((t = allow_heur<KMAX, MT, 0, true, POL>()) != hipSuccess) e = t;
    if ((t = allow_heur<KMAX, MT, 1, true, POL>()) != hipSuccess) e = t;
    return e;
}

template struct HeurLaunch<CAPART_I_K, CAPART_I_MT, CAPART_I_POL>;

}  // namespace capart
