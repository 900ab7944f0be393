// Kernels of the Schur pressure-correction preconditioner (section
// "Navier-Stokes problem"): the local SPAI-0 preconditioner of the velocity
// solves, the block products with D and G, and the moves between the whole
// system's vectors and its velocity and pressure parts.
#pragma once

#include "kernels.hpp"

namespace dfamg {

// s = m o r (SPAI-0, m_i = a_ii / sum_j a_ij^2) with the partial (r, s) per
// tile, the preconditioner of the velocity solves
static __global__ void __launch_bounds__(kBlock) k_diag_scale(const DevTile *__restrict__ tiles, int32_t ntiles,
                                                              const double *__restrict__ m,
                                                              const double *__restrict__ r, double *__restrict__ s,
                                                              double *__restrict__ part,
                                                              const SysState *__restrict__ st,
                                                              const int32_t *__restrict__ sub_sys) {
    __shared__ double lds[4];
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    if (st[sub_sys[T.sub]].done) return;
    double d = 0.0;
    for_tile_rows(T, [&](int row) {
        const double v = r[row];
        const double w = m[row] * v;
        s[row] = w;
        d += v * w;
    });
    const double sum = block_sum(d, lds, kBlock);
    if (threadIdx.x == 0) part[T.slot] = sum;
}

// y = b - M x for a CSR block: kCsrLanes lanes per row stride over the
// row's entries (consecutive lanes read consecutive entries), then a
// shuffle reduction inside the lane group
constexpr int kCsrLanes = 16;

static __global__ void __launch_bounds__(kBlock) k_csr_resid(int64_t nrows, const int64_t *__restrict__ ptr,
                                                             const int32_t *__restrict__ col,
                                                             const double *__restrict__ val,
                                                             const double *__restrict__ x,
                                                             const double *__restrict__ b, double *__restrict__ y) {
    const int64_t row = (int64_t)blockIdx.x * (kBlock / kCsrLanes) + threadIdx.x / kCsrLanes;
    const int lane = threadIdx.x % kCsrLanes;
    double a = 0.0;
    if (row < nrows)
        for (int64_t e = ptr[row] + lane; e < ptr[row + 1]; e += kCsrLanes) a += stream_load(val + e) * x[col[e]];
#pragma unroll
    for (int o = kCsrLanes / 2; o > 0; o >>= 1) a += __shfl_xor(a, o, kCsrLanes);
    if (row < nrows && lane == 0) y[row] = b[row] - a;
}

// dst[i] = src[idx[i]]
static __global__ void k_gather_idx(int64_t n, const int64_t *__restrict__ idx, const double *__restrict__ src,
                                    double *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[idx[i]];
}

// dst[idx[i]] = src[i]
static __global__ void k_scatter_idx(int64_t n, const int64_t *__restrict__ idx, const double *__restrict__ src,
                                     double *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[idx[i]] = src[i];
}

// acc[0] += iterations of the system (the inner solves of the Schur step run
// one system per handle)
static __global__ void k_add_iters(const SysState *__restrict__ st, int nsys, int64_t *__restrict__ acc) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int64_t a = 0;
        for (int i = 0; i < nsys; ++i) a += st[i].iter;
        acc[0] += a;
    }
}

}  // namespace dfamg
