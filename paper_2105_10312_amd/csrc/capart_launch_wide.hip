// Launchers of the wave-per-partitioning kernels for sets above
// NARROW_MAX_TASKS tasks, for one policy (CAPART_I_POL): 512-thread blocks
// (eight waves share one staged execution-time table).
#include "capart_device.h"

#if !defined(CAPART_I_POL)
#error "build with -DCAPART_I_POL=<POL_FP|POL_EDF>"
#endif

namespace capart {

template <int KMAX, bool COUNT, int POL>
static hipError_t launch_wide(const Batch &b, const Work &w, const Out &o, const Launch &L, hipStream_t st,
                              uint32_t p_lo, uint32_t p_hi)
{
    const dim3 grid((unsigned)(L.S * L.chunks)), block(512);
    const size_t lds = (size_t)2 * L.table_words;  // half of the [m][conflict][rank] time + utilisation tables
    switch (L.mode) {
    case CAPART_HEUR_BF_INA:
        hipLaunchKernelGGL((eval_wide_kernel<KMAX, false, false, COUNT, POL>), grid, block, lds, st, b, w, o, L, p_lo, p_hi);
        break;
    case CAPART_HEUR_BF_ACT:
        hipLaunchKernelGGL((eval_wide_kernel<KMAX, true, false, COUNT, POL>), grid, block, lds, st, b, w, o, L, p_lo, p_hi);
        break;
    case CAPART_HEUR_SMS_INA:
        hipLaunchKernelGGL((eval_wide_kernel<KMAX, false, true, COUNT, POL>), grid, block, lds, st, b, w, o, L, p_lo, p_hi);
        break;
    default:
        hipLaunchKernelGGL((eval_wide_kernel<KMAX, true, true, COUNT, POL>), grid, block, lds, st, b, w, o, L, p_lo, p_hi);
        break;
    }
    return hipGetLastError();
}

template <int POL>
hipError_t WideLaunch<POL>::eval(int kmax, bool count, const Batch &b, const Work &w, const Out &o, const Launch &L,
                                 hipStream_t st, uint32_t p_lo, uint32_t p_hi)
{
    if (kmax <= 4)
        return count ? launch_wide<4, true, POL>(b, w, o, L, st, p_lo, p_hi)
                     : launch_wide<4, false, POL>(b, w, o, L, st, p_lo, p_hi);
    return count ? launch_wide<8, true, POL>(b, w, o, L, st, p_lo, p_hi)
                 : launch_wide<8, false, POL>(b, w, o, L, st, p_lo, p_hi);
}

template <int KMAX, bool COUNT, int POL>
static hipError_t allow_wide()
{
    hipError_t e = hipSuccess, t;
    if ((t = allow_lds(eval_wide_kernel<KMAX, false, false, COUNT, POL>)) != hipSuccess) e = t;
    if ((t = allow_lds(eval_wide_kernel<KMAX, true, false, COUNT, POL>)) != hipSuccess) e = t;
    if ((t = allow_lds(eval_wide_kernel<KMAX, false, true, COUNT, POL>)) != hipSuccess) e = t;
    if ((t = allow_lds(eval_wide_kernel<KMAX, true, true, COUNT, POL>)) != hipSuccess) e = t;
    return e;
}

template <int POL>
hipError_t WideLaunch<POL>::allow()
{
    hipError_t e = hipSuccess, t;
    if ((t = allow_wide<4, false, POL>()) != hipSuccess) e = t;
    if ((t = allow_wide<8, false, POL>()) != hipSuccess) e = t;
    if ((t = allow_wide<4, true, POL>()) != hipSuccess) e = t;
    if ((t = allow_wide<8, true, POL>()) != hipSuccess) e = t;
    return e;
}

template struct WideLaunch<CAPART_I_POL>;

}  // namespace capart
