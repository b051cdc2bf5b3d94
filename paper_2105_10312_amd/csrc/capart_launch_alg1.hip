// Launchers of the Algorithm 1 kernel (free partition sizes, one wave per
// set) for one policy (CAPART_I_POL), plain and counting variants.
#include "capart_device.h"

#if !defined(CAPART_I_POL)
#error "build with -DCAPART_I_POL=<POL_FP|POL_EDF>"
#endif

namespace capart {

template <typename TY>
static void launch_alg1_ty(const Batch &b, const Work &w, const A1Out &o, const Launch &L, hipStream_t st)
{
    const dim3 grid((unsigned)L.S), block(64);
    const size_t lds = dyn_bytes(b) / 2;  // the execution-time half of the per-set tables
    switch (L.mode) {
    case CAPART_HEUR_BF_INA: hipLaunchKernelGGL((alg1_kernel<false, false, TY>), grid, block, lds, st, b, w, o, L); break;
    case CAPART_HEUR_BF_ACT: hipLaunchKernelGGL((alg1_kernel<true, false, TY>), grid, block, lds, st, b, w, o, L); break;
    case CAPART_HEUR_SMS_INA: hipLaunchKernelGGL((alg1_kernel<false, true, TY>), grid, block, lds, st, b, w, o, L); break;
    default: hipLaunchKernelGGL((alg1_kernel<true, true, TY>), grid, block, lds, st, b, w, o, L); break;
    }
}

template <int POL>
hipError_t Alg1Launch<POL>::run(bool count, const Batch &b, const Work &w, const A1Out &o, const Launch &L,
                                hipStream_t st)
{
    if (count)
        launch_alg1_ty<TallyP<POL>>(b, w, o, L, st);
    else
        launch_alg1_ty<NoTallyP<POL>>(b, w, o, L, st);
    return hipGetLastError();
}

template <typename TY>
static hipError_t allow_alg1()
{
    hipError_t e = hipSuccess, t;
    if ((t = allow_lds(alg1_kernel<false, false, TY>)) != hipSuccess) e = t;
    if ((t = allow_lds(alg1_kernel<true, false, TY>)) != hipSuccess) e = t;
    if ((t = allow_lds(alg1_kernel<false, true, TY>)) != hipSuccess) e = t;
    if ((t = allow_lds(alg1_kernel<true, true, TY>)) != hipSuccess) e = t;
    return e;
}

template <int POL>
hipError_t Alg1Launch<POL>::allow()
{
    hipError_t e = allow_alg1<NoTallyP<POL>>(), t;
    if ((t = allow_alg1<TallyP<POL>>()) != hipSuccess) e = t;
    return e;
}

template struct Alg1Launch<CAPART_I_POL>;

}  // namespace capart
