// Launchers of the outer-operator kernels (FP64 global matrix: block-diagonal
// part in a tuned layout plus the couplings between subdomains, with the
// deflation epilogues).
#include "devmat.hpp"

namespace dfamg {

namespace {

template <int N>
struct NdvC {
    static constexpr int value = N;
};

// Compile-time bound on the deflation vectors per subdomain: the epilogues
// unroll their Z loops to the bound (0, 1, 4 or 8) and skip the terms beyond
// the run-time count.
template <class Fn>
void with_ndv(int ndv, Fn &&fn) {
    if (ndv == 0) fn(NdvC<0>{});
    else if (ndv == 1) fn(NdvC<1>{});
    else if (ndv <= 4) fn(NdvC<4>{});
    else if (ndv <= kMaxNdv) fn(NdvC<kMaxNdv>{});
    else throw std::runtime_error("ndv out of range");
}

}  // namespace

void launch_outer(int mode, int ndv, const DevMat<double> &A, const OffM &off, const double *x, const double *b,
                  double *out, const ZView &Z, double *part, const SysState *st, const int32_t *sub_sys,
                  hipStream_t s) {
    with_mat(A, [&](auto v) {
        with_ndv(ndv, [&](auto nd_c) {
            constexpr int ND = decltype(nd_c)::value;
            using MT = decltype(v);
            const dim3 g(grid_for_tiles(v.ntiles)), bl(kBlock);
            switch (mode) {
                case 0: hipLaunchKernelGGL((k_outer<0, ND, MT>), g, bl, A.stage_bytes(), s, v, off, x, b, out, Z, ndv, part, A.ntiles, st, sub_sys); break;
                case 1: hipLaunchKernelGGL((k_outer<1, ND, MT>), g, bl, A.stage_bytes(), s, v, off, x, b, out, Z, ndv, part, A.ntiles, st, sub_sys); break;
                case 2: hipLaunchKernelGGL((k_outer<2, ND, MT>), g, bl, A.stage_bytes(), s, v, off, x, b, out, Z, ndv, part, A.ntiles, st, sub_sys); break;
                case 3: hipLaunchKernelGGL((k_outer<3, ND, MT>), g, bl, A.stage_bytes(), s, v, off, x, b, out, Z, ndv, part, A.ntiles, st, sub_sys); break;
                default: hipLaunchKernelGGL((k_outer<4, ND, MT>), g, bl, A.stage_bytes(), s, v, off, x, b, out, Z, ndv, part, A.ntiles, st, sub_sys); break;
            }
        });
    });
}

void launch_outer_spmv_plain(const DevMat<double> &A, const double *x, double *y, hipStream_t s) {
    with_mat(A, [&](auto v) {
        hipLaunchKernelGGL((k_spmv<double, decltype(v)>), dim3(grid_for_tiles(v.ntiles)), dim3(kBlock), A.stage_bytes(), s, v, x, y,
                           (const SysState *)nullptr, (const int32_t *)nullptr);
    });
}

}  // namespace dfamg
