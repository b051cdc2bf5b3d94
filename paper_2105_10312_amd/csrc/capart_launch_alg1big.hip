// Launchers of Algorithm 1 for batches with sets of more than 64 tasks (one
// block of 256 threads per set, fixed priority): the prep kernel of such sets,
// then the Algorithm 1 kernel, plain and counting variants.
#include <algorithm>

#include "capart_alg1_big.h"

namespace capart {

// Dynamic LDS of the execution-time table of the batch's largest set.
static size_t big_table_bytes(const Batch &b)
{
    const int64_t nm = (int64_t)std::min(b.max_tasks, BIGN) * (int64_t)std::min(b.max_M, CAPART_ALG1_BIG_MAX_M);
    return (size_t)8 * (size_t)std::min<int64_t>(nm, CAPART_ALG1_BIG_MAX_NM);
}

hipError_t launch_prep_big(const Batch &b, const Work &w, const Out &o, const Launch &L, hipStream_t st)
{
    hipLaunchKernelGGL(prep_big_kernel, dim3((unsigned)L.S), dim3(256), 0, st, b, w, o, L);
    return hipGetLastError();
}

template <typename TY>
static void launch_big_ty(const Batch &b, const Work &w, const A1Out &o, const Launch &L, hipStream_t st)
{
    const dim3 grid((unsigned)L.S), block(256);
    const size_t lds = big_table_bytes(b);
    switch (L.mode) {
    case CAPART_HEUR_BF_INA: hipLaunchKernelGGL((alg1_big_kernel<false, false, TY>), grid, block, lds, st, b, w, o, L); break;
    case CAPART_HEUR_BF_ACT: hipLaunchKernelGGL((alg1_big_kernel<true, false, TY>), grid, block, lds, st, b, w, o, L); break;
    case CAPART_HEUR_SMS_INA: hipLaunchKernelGGL((alg1_big_kernel<false, true, TY>), grid, block, lds, st, b, w, o, L); break;
    default: hipLaunchKernelGGL((alg1_big_kernel<true, true, TY>), grid, block, lds, st, b, w, o, L); break;
    }
}

hipError_t launch_alg1_big(const Batch &b, const Work &w, const A1Out &o, const Launch &L, hipStream_t st, bool count)
{
    if (count)
        launch_big_ty<TallyP<POL_FP>>(b, w, o, L, st);
    else
        launch_big_ty<NoTallyP<POL_FP>>(b, w, o, L, st);
    return hipGetLastError();
}

template <typename TY>
static hipError_t allow_big_ty()
{
    hipError_t e = hipSuccess, t;
    if ((t = allow_lds(alg1_big_kernel<false, false, TY>)) != hipSuccess) e = t;
    if ((t = allow_lds(alg1_big_kernel<true, false, TY>)) != hipSuccess) e = t;
    if ((t = allow_lds(alg1_big_kernel<false, true, TY>)) != hipSuccess) e = t;
    if ((t = allow_lds(alg1_big_kernel<true, true, TY>)) != hipSuccess) e = t;
    return e;
}

hipError_t allow_alg1_big()
{
    hipError_t e = allow_big_ty<NoTallyP<POL_FP>>(), t;
    if ((t = allow_big_ty<TallyP<POL_FP>>()) != hipSuccess) e = t;
    return e;
}

}  // namespace capart
