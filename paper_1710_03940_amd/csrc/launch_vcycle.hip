// Launchers of the V-cycle matrix kernels for one value type, chosen at
// compile time with -DDFAMG_VT_DOUBLE (FP64 hierarchy) or without it (FP32
// hierarchy of the mixed-precision path).
#include "devmat.hpp"

namespace dfamg {

template <class VT, class FT>
void launch_pre_res(const DevMat<VT> &A, const VT *m, const FT *f, VT *res, const SysState *st,
                    const int32_t *sub_sys, hipStream_t s) {
    with_mat(A, [&](auto v) {
        hipLaunchKernelGGL((k_pre_res<VT, FT, decltype(v)>), dim3(grid_for_tiles(v.ntiles)), dim3(kBlock),
                           A.stage_bytes(), s, v, m, f, res, st, sub_sys);
    });
}

// The two launches of a column-tiled operator: partial sums per segment, then
// their sum per row.
template <class VT, class FT>
void launch_seg(const DevMat<VT> &M, const FT *x, VT *y, const SysState *st, const int32_t *sub_sys,
                hipStream_t s) {
    switch (M.seg_nt) {
        case 1024:
            hipLaunchKernelGGL((k_seg_partial<VT, FT, 1024>), dim3(grid_for_tiles(M.ntiles)), dim3(1024),
                               M.stage_bytes(), s, seg_view(M), x, M.seg_part, st, sub_sys);
            break;
        case 512:
            hipLaunchKernelGGL((k_seg_partial<VT, FT, 512>), dim3(grid_for_tiles(M.ntiles)), dim3(512),
                               M.stage_bytes(), s, seg_view(M), x, M.seg_part, st, sub_sys);
            break;
        default:
            hipLaunchKernelGGL((k_seg_partial<VT, FT, 256>), dim3(grid_for_tiles(M.ntiles)), dim3(256),
                               M.stage_bytes(), s, seg_view(M), x, M.seg_part, st, sub_sys);
    }
    hipLaunchKernelGGL((k_seg_combine<VT>), dim3(grid_for_tiles(M.seg_nrt)), dim3(kBlock), 0, s, M.seg_rtiles,
                       M.seg_nrt, M.seg_pp, M.seg_part, y, M.rowmap, st, sub_sys);
}

template <class VT>
void launch_spmv(const DevMat<VT> &M, const VT *x, VT *y, const SysState *st, const int32_t *sub_sys,
                 hipStream_t s) {
    if (M.fmt == kFormatSeg) {
        launch_seg<VT, VT>(M, x, y, st, sub_sys, s);
        return;
    }
    with_mat(M, [&](auto v) {
        hipLaunchKernelGGL((k_spmv<VT, decltype(v)>), dim3(grid_for_tiles(v.ntiles)), dim3(kBlock), M.stage_bytes(),
                           s, v, x, y, st, sub_sys);
    });
}

template <class VT, class FT>
void launch_restrict(const DevMat<VT> &B, const FT *f, VT *fc, const SysState *st, const int32_t *sub_sys,
                     hipStream_t s) {
    if (B.fmt == kFormatSeg) {
        launch_seg<VT, FT>(B, f, fc, st, sub_sys, s);
        return;
    }
    with_mat(B, [&](auto v) {
        hipLaunchKernelGGL((k_restrict<VT, FT, decltype(v)>), dim3(grid_for_tiles(v.ntiles)), dim3(kBlock),
                           B.stage_bytes(), s, v, f, fc, B.rowmap, st, sub_sys);
    });
}

template <class VT, class FT>
void launch_prolong(const DevMat<VT> &P, const VT *m, const FT *f, const VT *xc, VT *z, const SysState *st,
                    const int32_t *sub_sys, hipStream_t s) {
    with_mat(P, [&](auto v) {
        hipLaunchKernelGGL((k_prolong<VT, FT, decltype(v)>), dim3(grid_for_tiles(v.ntiles)), dim3(kBlock),
                           P.stage_bytes(), s, v, m, f, xc, z, st, sub_sys);
    });
}

template <class VT, class FT, class OT, bool DOT>
void launch_post(const DevMat<VT> &A, const VT *m, const FT *f, const VT *z, OT *x, double *part,
                 const SysState *st, const int32_t *sub_sys, hipStream_t s) {
    with_mat(A, [&](auto v) {
        hipLaunchKernelGGL((k_post<VT, FT, OT, DOT, decltype(v)>), dim3(grid_for_tiles(v.ntiles)), dim3(kBlock),
                           A.stage_bytes(), s, v, m, f, z, x, part, st, sub_sys);
    });
}

template <class VT, class FT>
void launch_resid(const DevMat<VT> &A, const FT *f, const VT *x, VT *res, const SysState *st,
                  const int32_t *sub_sys, hipStream_t s) {
    with_mat(A, [&](auto v) {
        hipLaunchKernelGGL((k_resid<VT, FT, decltype(v)>), dim3(grid_for_tiles(v.ntiles)), dim3(kBlock),
                           A.stage_bytes(), s, v, f, x, res, st, sub_sys);
    });
}

template <class VT>
void launch_prolong_add(const DevMat<VT> &P, const VT *x, const VT *xc, VT *z, const SysState *st,
                        const int32_t *sub_sys, hipStream_t s) {
    with_mat(P, [&](auto v) {
        hipLaunchKernelGGL((k_prolong_add<VT, decltype(v)>), dim3(grid_for_tiles(v.ntiles)), dim3(kBlock),
                           P.stage_bytes(), s, v, x, xc, z, st, sub_sys);
    });
}

#ifdef DFAMG_VT_DOUBLE
template void launch_resid<double, double>(const DevMat<double> &, const double *, const double *, double *,
                                           const SysState *, const int32_t *, hipStream_t);
template void launch_prolong_add<double>(const DevMat<double> &, const double *, const double *, double *,
                                         const SysState *, const int32_t *, hipStream_t);
template void launch_pre_res<double, double>(const DevMat<double> &, const double *, const double *, double *,
                                             const SysState *, const int32_t *, hipStream_t);
template void launch_restrict<double, double>(const DevMat<double> &, const double *, double *, const SysState *,
                                              const int32_t *, hipStream_t);
template void launch_spmv<double>(const DevMat<double> &, const double *, double *, const SysState *,
                                  const int32_t *, hipStream_t);
template void launch_prolong<double, double>(const DevMat<double> &, const double *, const double *, const double *,
                                             double *, const SysState *, const int32_t *, hipStream_t);
template void launch_post<double, double, double, true>(const DevMat<double> &, const double *, const double *,
                                                        const double *, double *, double *, const SysState *,
                                                        const int32_t *, hipStream_t);
template void launch_post<double, double, double, false>(const DevMat<double> &, const double *, const double *,
                                                         const double *, double *, double *, const SysState *,
                                                         const int32_t *, hipStream_t);
#else
template void launch_resid<float, float>(const DevMat<float> &, const float *, const float *, float *,
                                         const SysState *, const int32_t *, hipStream_t);
template void launch_resid<float, double>(const DevMat<float> &, const double *, const float *, float *,
                                          const SysState *, const int32_t *, hipStream_t);
template void launch_prolong_add<float>(const DevMat<float> &, const float *, const float *, float *,
                                        const SysState *, const int32_t *, hipStream_t);
template void launch_post<float, double, float, false>(const DevMat<float> &, const float *, const double *,
                                                       const float *, float *, double *, const SysState *,
                                                       const int32_t *, hipStream_t);
template void launch_pre_res<float, float>(const DevMat<float> &, const float *, const float *, float *,
                                           const SysState *, const int32_t *, hipStream_t);
template void launch_pre_res<float, double>(const DevMat<float> &, const float *, const double *, float *,
                                            const SysState *, const int32_t *, hipStream_t);
template void launch_spmv<float>(const DevMat<float> &, const float *, float *, const SysState *, const int32_t *,
                                 hipStream_t);
template void launch_restrict<float, float>(const DevMat<float> &, const float *, float *, const SysState *,
                                            const int32_t *, hipStream_t);
template void launch_restrict<float, double>(const DevMat<float> &, const double *, float *, const SysState *,
                                             const int32_t *, hipStream_t);
template void launch_prolong<float, float>(const DevMat<float> &, const float *, const float *, const float *, float *,
                                           const SysState *, const int32_t *, hipStream_t);
template void launch_prolong<float, double>(const DevMat<float> &, const float *, const double *, const float *,
                                            float *, const SysState *, const int32_t *, hipStream_t);
template void launch_post<float, float, float, false>(const DevMat<float> &, const float *, const float *,
                                                      const float *, float *, double *, const SysState *,
                                                      const int32_t *, hipStream_t);
template void launch_post<float, double, double, true>(const DevMat<float> &, const float *, const double *,
                                                       const float *, double *, double *, const SysState *,
                                                       const int32_t *, hipStream_t);
#endif

}  // namespace dfamg
