// The kernels templated on the projection width K, and their typed
// launchers, for one K (SAP_K, set on the compiler line).  The build compiles
// this unit once per K = 1..16, in parallel; sap_api.hip holds the host
// runtime and the K-independent kernels.
#ifndef SAP_K
#error "compile with -DSAP_K=<projection width>"
#endif
#define SAP_KINST 1

#include <hip/hip_ext.h>

#include "sap_iter.hip"
#include "sap_softmin.hip"
#include "sap_launch.h"

namespace sap {

template <int K, typename TX>
hipError_t KLaunch<K, TX>::prep(const LaunchCfg &c, const SweepArgs<TX> &a, const double *mu, float *Y,
                                int64_t Npad) {
    hipExtLaunchKernelGGL(k_prep<K, TX>, c.grid, c.block, c.shmem, c.stream, c.ea, c.eb, 0, a, mu, Y, Npad);
    return hipGetLastError();
}

template <int K, typename TX>
hipError_t KLaunch<K, TX>::pass(const LaunchCfg &c, bool fused, const SweepArgs<TX> &a, int nshort) {
    if (fused)
        hipExtLaunchKernelGGL(k_pass<K, TX, true>, c.grid, c.block, c.shmem, c.stream, c.ea, c.eb, 0, a, nshort);
    else
        hipExtLaunchKernelGGL(k_pass<K, TX, false>, c.grid, c.block, c.shmem, c.stream, c.ea, c.eb, 0, a, nshort);
    return hipGetLastError();
}

template <int K, typename TX>
hipError_t KLaunch<K, TX>::select(const LaunchCfg &c, bool fused, const SweepArgs<TX> &a, int nshort,
                                  double *P64t, void *Pr, int pr_kind, double alpha, int rule, int do_step) {
    if (fused)
        hipExtLaunchKernelGGL(k_select<K, TX, true>, c.grid, c.block, c.shmem, c.stream, c.ea, c.eb, 0, a,
                              nshort, P64t, Pr, pr_kind, alpha, rule, do_step);
    else
        hipExtLaunchKernelGGL(k_select<K, TX, false>, c.grid, c.block, c.shmem, c.stream, c.ea, c.eb, 0, a,
                              nshort, P64t, Pr, pr_kind, alpha, rule, do_step);
    return hipGetLastError();
}

template <int K, typename TX>
hipError_t KLaunch<K, TX>::selprep(const LaunchCfg &c, const SweepArgs<TX> &a, int nshort, double *Pn,
                                   double alpha, int rule, const double *mu, float *Y, int64_t Npad) {
    if (a.gtiles == 2)
        hipExtLaunchKernelGGL(k_selprep<K, TX, 2>, c.grid, c.block, c.shmem, c.stream, c.ea, c.eb, 0, a, nshort,
                              Pn, alpha, rule, mu, Y, Npad);
    else
        hipExtLaunchKernelGGL(k_selprep<K, TX, 1>, c.grid, c.block, c.shmem, c.stream, c.ea, c.eb, 0, a, nshort,
                              Pn, alpha, rule, mu, Y, Npad);
    return hipGetLastError();
}

template <int K, typename TX>
hipError_t KLaunch<K, TX>::set_select_lds(int bytes) {
    const void *fns[5] = {reinterpret_cast<const void *>(&k_select<K, TX, true>),
                          reinterpret_cast<const void *>(&k_select<K, TX, false>),
                          reinterpret_cast<const void *>(&k_selprep<K, TX, 1>),
                          reinterpret_cast<const void *>(&k_selprep<K, TX, 2>),
                          reinterpret_cast<const void *>(&k_prep<K, TX>)};
    for (const void *f : fns) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int K, typename TX>
hipError_t KLaunch<K, TX>::sm_prep(const LaunchCfg &c, const SmArgs &a, const TX *X, int64_t ldx, int64_t N,
                                   const double *mu, float *Y, int64_t Npad, int gemm_blocks, int bwd) {
    hipExtLaunchKernelGGL(k_sm_prep<K, TX>, c.grid, c.block, c.shmem, c.stream, c.ea, c.eb, 0, a, X, ldx, N, mu,
                          Y, Npad, gemm_blocks, bwd);
    return hipGetLastError();
}

template <int K, typename TX>
hipError_t KLaunch<K, TX>::sm_fwd(const LaunchCfg &c, const SmArgs &a) {
    hipExtLaunchKernelGGL(k_sm_fwd<K>, c.grid, c.block, c.shmem, c.stream, c.ea, c.eb, 0, a);
    return hipGetLastError();
}

template <int K, typename TX>
hipError_t KLaunch<K, TX>::sm_bwd(const LaunchCfg &c, const SmArgs &a) {
    hipExtLaunchKernelGGL(k_sm_bwd<K>, c.grid, c.block, c.shmem, c.stream, c.ea, c.eb, 0, a);
    return hipGetLastError();
}

template <int K, typename TX>
hipError_t KLaunch<K, TX>::sm_zred(const LaunchCfg &c, const SmArgs &a, int64_t nb, int64_t N,
                                   const int32_t *rp_i, const int32_t *rp_j, const int32_t *permj, double *Z) {
    hipExtLaunchKernelGGL(k_sm_zred<K>, c.grid, c.block, c.shmem, c.stream, c.ea, c.eb, 0, a, nb, N, rp_i, rp_j,
                          permj, Z);
    return hipGetLastError();
}

template struct KLaunch<SAP_K, float>;
template struct KLaunch<SAP_K, double>;

}  // namespace sap
