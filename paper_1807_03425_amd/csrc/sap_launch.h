// Typed launchers of the kernels templated on the projection width K.
//
// The host runtime (sap_api.hip) calls these; their definitions, and the
// kernels they launch, are compiled once per K in sap_kinst.hip (one
// translation unit per K, built in parallel) and linked into libsap.so.
// Every launcher enqueues one kernel with hipExtLaunchKernelGGL on
// c.stream (with the dispatch timestamps c.ea / c.eb when non-null) and
// returns hipGetLastError().
#pragma once

#include "sap_common.h"

namespace sap {

template <typename TX> struct SweepArgs;
struct SmArgs;
struct BatchArgs;

template <int K, typename TX>
struct KLaunch {
    // the iteration (sap_iter.hip)
    static hipError_t prep(const LaunchCfg &c, const SweepArgs<TX> &a, const double *mu, float *Y,
                           int64_t Npad);
    static hipError_t pass(const LaunchCfg &c, bool fused, const SweepArgs<TX> &a, int nshort);
    static hipError_t select(const LaunchCfg &c, bool fused, const SweepArgs<TX> &a, int nshort,
                             double *P64t, void *Pr, int pr_kind, double alpha, int rule, int do_step);
    static hipError_t selprep(const LaunchCfg &c, const SweepArgs<TX> &a, int nshort, double *Pn,
                              double alpha, int rule, const double *mu, float *Y, int64_t Npad);
    // dynamic LDS limit of the selection kernels and of k_prep (bytes)
    static hipError_t set_select_lds(int bytes);
    // the soft-min (sap_softmin.hip)
    static hipError_t sm_prep(const LaunchCfg &c, const SmArgs &a, const TX *X, int64_t ldx, int64_t N,
                              const double *mu, float *Y, int64_t Npad, int gemm_blocks, int bwd);
    static hipError_t sm_fwd(const LaunchCfg &c, const SmArgs &a);
    static hipError_t sm_bwd(const LaunchCfg &c, const SmArgs &a);
    static hipError_t sm_zred(const LaunchCfg &c, const SmArgs &a, int64_t nb, int64_t N,
                              const int32_t *rp_i, const int32_t *rp_j, const int32_t *permj, double *Z);
};

}  // namespace sap
