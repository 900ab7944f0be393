// Level kernels of the block SPAI-0 smoother (point-block hierarchies): the
// smoother couples the bs rows of a node, so its steps run as separate
// row-wise passes around the plain SpMV of the level matrix instead of being
// folded into the SpMV's gathers like the diagonal smoother.  Packed level
// rows are node-aligned (every subdomain block holds whole nodes), so the
// node of row i starts at bs * (i / bs); mb holds, for row i, the bs entries
// of row i % bs of its node's block.
#pragma once

#include "kernels.hpp"

namespace dfamg {

// x = M f (pre-smoothing from a zero guess)
template <class VT, class FT>
__global__ void __launch_bounds__(kBlock) k_bsm_pre(const DevTile *__restrict__ tiles, int32_t ntiles, int bs,
                                                    const VT *__restrict__ mb, const FT *__restrict__ f,
                                                    VT *__restrict__ x, const SysState *__restrict__ st,
                                                    const int32_t *__restrict__ sub_sys) {
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    if (st[sub_sys[T.sub]].done) return;
    for_tile_rows(T, [&](int row) {
        const int64_t nb = (int64_t)(row / bs) * bs;
        VT a = 0;
        for (int k = 0; k < bs; ++k) a += mb[(int64_t)row * bs + k] * (VT)f[nb + k];
        x[row] = a;
    });
}

// y = f - y (the residual of the pre-smoothed iterate, y = A x on entry)
template <class VT, class FT>
__global__ void __launch_bounds__(kBlock) k_bsm_res(const DevTile *__restrict__ tiles, int32_t ntiles,
                                                    const FT *__restrict__ f, VT *__restrict__ y,
                                                    const SysState *__restrict__ st,
                                                    const int32_t *__restrict__ sub_sys) {
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    if (st[sub_sys[T.sub]].done) return;
    for_tile_rows(T, [&](int row) { y[row] = (VT)f[row] - y[row]; });
}

// z += x (the coarse correction added to the pre-smoothed iterate)
template <class VT>
__global__ void __launch_bounds__(kBlock) k_bsm_add(const DevTile *__restrict__ tiles, int32_t ntiles,
                                                    const VT *__restrict__ x, VT *__restrict__ z,
                                                    const SysState *__restrict__ st,
                                                    const int32_t *__restrict__ sub_sys) {
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    if (st[sub_sys[T.sub]].done) return;
    for_tile_rows(T, [&](int row) { z[row] += x[row]; });
}

// out = z + M (f - y) with y = A z (post-smoothing); DOT: partial (f, out)
template <class VT, class FT, class OT, bool DOT>
__global__ void __launch_bounds__(kBlock) k_bsm_post(const DevTile *__restrict__ tiles, int32_t ntiles, int bs,
                                                     const VT *__restrict__ mb, const FT *__restrict__ f,
                                                     const VT *__restrict__ z, const VT *__restrict__ y,
                                                     OT *__restrict__ out, double *__restrict__ part,
                                                     const SysState *__restrict__ st,
                                                     const int32_t *__restrict__ sub_sys) {
    __shared__ double lds[4];
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    if (st[sub_sys[T.sub]].done) return;
    double d = 0.0;
    for_tile_rows(T, [&](int row) {
        const int64_t nb = (int64_t)(row / bs) * bs;
        VT a = z[row];
        for (int k = 0; k < bs; ++k) a += mb[(int64_t)row * bs + k] * ((VT)f[nb + k] - y[nb + k]);
        out[row] = (OT)a;
        if (DOT) d += (double)f[row] * (double)(OT)a;
    });
    if (!DOT) return;
    const double s = block_sum(d, lds, kBlock);
    if (threadIdx.x == 0) part[T.slot] = s;
}

}  // namespace dfamg
