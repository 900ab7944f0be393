// Device assembly of the coarse operator E = Z^T A Z (setup): one column per
// outer-operator product, with the operator's Z^T epilogue doing the
// projection onto the deflation space.
#pragma once

#include "kernels.hpp"

namespace dfamg {

// v = Z e_c: column k of the local deflation block of subdomain `sub` on that
// subdomain's rows, zero on every other row
static __global__ void __launch_bounds__(kBlock) k_zcol(const DevTile *__restrict__ tiles, int32_t ntiles,
                                                        const double *__restrict__ Z, int ndv, int sub, int k,
                                                        double *__restrict__ v) {
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    const bool own = T.sub == sub;
    for_tile_rows(T, [&](int row) { v[row] = own ? Z[(int64_t)row * ndv + k] : 0.0; });
}

// column `col` of the row-major m x m block E (system coarse indices c0 ..
// c0 + m - 1) from the per-subdomain sums t1 = Z^T A v
static __global__ void k_ecol(const double *__restrict__ t1, int64_t c0, int m, int col, double *__restrict__ E) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < m) E[(int64_t)r * m + col] = t1[c0 + r];
}

}  // namespace dfamg
