// kbc_step_inst.hip -- the step, pool and stabilizer-statistics kernels of one
// storage form and stabilizer mode.  The build compiles this file once per
// pair (KBC_INST_STORAGE in {0, 1, 2, 3}, KBC_INST_EXACT in {0, 1}); the
// launchers in kbc_kernels.hip reach the kernels through the tables below.
#include "kbc_step.h"

#if !defined(KBC_INST_STORAGE) || !defined(KBC_INST_EXACT)
#error "compile with -DKBC_INST_STORAGE=<storage form> -DKBC_INST_EXACT=<0|1>"
#endif

namespace kbc {

namespace {

constexpr int kS = KBC_INST_STORAGE;
constexpr bool kGX = KBC_INST_EXACT != 0;

// The pull sweep on 64-node chunks with the chunk geometry compiled in is
// instantiated where it removes scalar-register spills of the per-direction
// bases: FP16 storage (4.7-5.9% faster at 256^3) and the exact stabilizer
// (53 spilled scalars down to 4; 0.5-2% faster).  The other forms measured
// the same either way.
constexpr bool kC64 = kS == ST_F16 || kGX;

template <int V>
StepFn step_of_sweep(int sw, bool c64)
{
    if (sw == SW_PULL) {
        if constexpr (kC64) {
            if (c64) return k_step<kS, V, SW_PULL, kGX, true>;
        }
        return k_step<kS, V, SW_PULL, kGX>;
    }
    return sw == SW_AA_EVEN ? k_step<kS, V, SW_AA_EVEN, kGX> : k_step<kS, V, SW_AA_ODD, kGX>;
}

template <int V>
PoolFn pool_of_sweep(int sw, bool one)
{
    if (one) return sw == SW_AA_EVEN ? k_pool_step<kS, V, SW_AA_EVEN, true> : k_pool_step<kS, V, SW_AA_ODD, true>;
    return sw == SW_AA_EVEN ? k_pool_step<kS, V, SW_AA_EVEN> : k_pool_step<kS, V, SW_AA_ODD>;
}

}  // namespace

template <int S, bool GX>
StepFn step_kernel(int v, int sw, bool c64)
{
    static_assert(S == kS && GX == kGX, "instantiated for one storage form and mode only");
    switch (v) {
    case V_D: return step_of_sweep<V_D>(sw, c64);
    case V_DT: return step_of_sweep<V_DT>(sw, c64);
    case V_DQ: return step_of_sweep<V_DQ>(sw, c64);
    case V_CD: return step_of_sweep<V_CD>(sw, c64);
    case V_CDT: return step_of_sweep<V_CDT>(sw, c64);
    case V_CDQ: return step_of_sweep<V_CDQ>(sw, c64);
    case V_CDTQ: return step_of_sweep<V_CDTQ>(sw, c64);
    default: return step_of_sweep<V_DTQ>(sw, c64);
    }
}

template <int S, bool GX>
GammaFn gamma_kernel(int v)
{
    static_assert(S == kS && GX == kGX, "instantiated for one storage form and mode only");
    switch (v) {
    case V_D: return k_gamma_stats<kS, V_D, kGX>;
    case V_DT: return k_gamma_stats<kS, V_DT, kGX>;
    case V_DQ: return k_gamma_stats<kS, V_DQ, kGX>;
    case V_CD: return k_gamma_stats<kS, V_CD, kGX>;
    case V_CDT: return k_gamma_stats<kS, V_CDT, kGX>;
    case V_CDQ: return k_gamma_stats<kS, V_CDQ, kGX>;
    case V_CDTQ: return k_gamma_stats<kS, V_CDTQ, kGX>;
    default: return k_gamma_stats<kS, V_DTQ, kGX>;
    }
}

template StepFn step_kernel<kS, kGX>(int, int, bool);
template GammaFn gamma_kernel<kS, kGX>(int);

#if !KBC_INST_EXACT
// the pool runs the estimate gamma* only
template <int S>
PoolFn pool_kernel(int v, int sw, bool one)
{
    static_assert(S == kS, "instantiated for one storage form only");
    switch (v) {
    case V_D: return pool_of_sweep<V_D>(sw, one);
    case V_DT: return pool_of_sweep<V_DT>(sw, one);
    case V_DQ: return pool_of_sweep<V_DQ>(sw, one);
    case V_CD: return pool_of_sweep<V_CD>(sw, one);
    case V_CDT: return pool_of_sweep<V_CDT>(sw, one);
    case V_CDQ: return pool_of_sweep<V_CDQ>(sw, one);
    case V_CDTQ: return pool_of_sweep<V_CDTQ>(sw, one);
    default: return pool_of_sweep<V_DTQ>(sw, one);
    }
}

template PoolFn pool_kernel<kS>(int, int, bool);
#endif

}  // namespace kbc
