// Device sparse matrices in the layouts of kernels.hpp and the launchers of
// the matrix kernels.  The launchers are instantiated in their own
// translation units (launch_vcycle.hip for FP32 and FP64, launch_outer.hip);
// the driver only calls them.
#pragma once

#include <hip/hip_runtime.h>

#include <stdexcept>
#include <vector>

#include "dfamg.h"
#include "host_plan.hpp"
#include "kernels.hpp"

namespace dfamg {

// Internal layout of the restrictions, chosen by the tuner only: the
// operator split by column tiles of `par` columns (see SegM), 256 * rpg
// threads per block.
constexpr int kFormatSeg = 16;

// A layout candidate: SELL (par = rows per lane), CSR (par = lanes per row),
// BSR4, or column-tiled segments (par = columns per tile)
struct Layout {
    int fmt, par;
    bool sorted, idx16, stage;
    int rpg = 0;   // CSR: rows per lane group in a tile (tile = rpg * 256 / lanes rows); 0 = 256-row tiles
    bool glist = false;   // staged CSR: stage the tile's distinct columns (gather list), not a window
};

template <class VT>
struct DevMat {
    int fmt = DFAMG_FORMAT_SELL;  // DFAMG_FORMAT_SELL, _CSR or _BSR4 (ptr, col: block rows / columns)
    int par = 1;                  // rows per lane (SELL) or lanes per row (CSR)
    bool idx16 = false, sorted = false, stage = false;
    DevTile *tiles = nullptr;
    int32_t ntiles = 0;
    int64_t *soff = nullptr;
    int32_t *sw = nullptr;
    int32_t *ptr = nullptr;
    int32_t *col = nullptr;
    uint16_t *col16 = nullptr;
    int32_t *cbase = nullptr, *cspan = nullptr;
    int16_t *ridx = nullptr;
    int32_t *uoff = nullptr, *ucol = nullptr;   // gather list of the staged CSR form (null: window)
    VT *val = nullptr;
    int32_t *rowmap = nullptr;    // restriction B: output position of each stored row (null: the row itself)
    // kFormatSeg: tiles are the column tiles; slices of each tile, per-lane
    // partial slots, the row -> partials pointer, the row tiles of the
    // combine step and its partial sums
    int32_t *seg_slices = nullptr, *seg_slot = nullptr, *seg_pp = nullptr;
    DevTile *seg_rtiles = nullptr;
    int32_t seg_nrt = 0;
    int32_t seg_nt = 256;         // threads per block of the partial-sum kernel
    VT *seg_part = nullptr;
    int32_t max_span = 0;         // LDS entries of the staged layouts (window or gather list)
    int64_t nnz = 0, stored = 0;
    double tuned_us = 0.0;
    std::vector<int32_t> sys_tile_off;  // host: tiles of each system
    std::vector<int32_t> sub_tile_off;  // host: tiles of each subdomain
    std::vector<DevTile> host_tiles;    // host copy of `tiles`
    size_t stage_bytes() const { return stage ? (size_t)max_span * sizeof(VT) : 0; }
};

// Largest LDS window (bytes) a staged layout may use per block.
constexpr size_t kMaxStageBytes = 65536;

// Calls fn(view) with the kernel view type of M.
template <class VT>
SegM<VT> seg_view(const DevMat<VT> &M) {
    return SegM<VT>{M.tiles, M.seg_slices, M.soff, M.sw, M.col16, M.val, M.seg_slot, M.ntiles};
}

template <class VT, class Fn>
void with_mat(const DevMat<VT> &M, Fn &&fn) {
#define DFAMG_SELL(R, I, S) \
    fn(SellM<VT, R, I, S>{M.tiles, M.soff, M.sw, M.col, M.col16, M.cbase, M.cspan, M.ridx, M.val, M.ntiles})
#define DFAMG_CSR(L, S) \
    fn(CsrM<VT, L, S>{M.tiles, M.ptr, M.col, M.cbase, M.cspan, M.val, M.ntiles, M.uoff, M.ucol, M.col16})
    if (M.fmt == DFAMG_FORMAT_BSR4) {
        fn(BsrM<VT>{M.tiles, M.ptr, M.col, M.val, M.ntiles});
        return;
    }
    if (M.fmt == DFAMG_FORMAT_SELL) {
        if (!M.stage) {
            if (M.idx16) {
                switch (M.par) {
                    case 1: DFAMG_SELL(1, true, false); return;
                    case 2: DFAMG_SELL(2, true, false); return;
                    case 4: DFAMG_SELL(4, true, false); return;
                }
            } else {
                switch (M.par) {
                    case 1: DFAMG_SELL(1, false, false); return;
                    case 2: DFAMG_SELL(2, false, false); return;
                    case 4: DFAMG_SELL(4, false, false); return;
                }
            }
        } else {
            switch (M.par) {
                case 1: DFAMG_SELL(1, true, true); return;
                case 2: DFAMG_SELL(2, true, true); return;
            }
        }
    } else {
        if (M.stage) {
            switch (M.par) {
                case 1: DFAMG_CSR(1, true); return;
                case 2: DFAMG_CSR(2, true); return;
                case 4: DFAMG_CSR(4, true); return;
                case 8: DFAMG_CSR(8, true); return;
                case 16: DFAMG_CSR(16, true); return;
                case 32: DFAMG_CSR(32, true); return;
                case 64: DFAMG_CSR(64, true); return;
            }
        } else {
            switch (M.par) {
                case 1: DFAMG_CSR(1, false); return;
                case 2: DFAMG_CSR(2, false); return;
                case 4: DFAMG_CSR(4, false); return;
                case 8: DFAMG_CSR(8, false); return;
                case 16: DFAMG_CSR(16, false); return;
                case 32: DFAMG_CSR(32, false); return;
                case 64: DFAMG_CSR(64, false); return;
            }
        }
    }
#undef DFAMG_SELL
#undef DFAMG_CSR
    throw std::runtime_error("unsupported matrix layout");
}

// ---- V-cycle launchers (launch_vcycle.hip) -------------------------------
// FT is the type of the level's right-hand side (double on level 0).
template <class VT, class FT>
void launch_pre_res(const DevMat<VT> &A, const VT *m, const FT *f, VT *res, const SysState *st,
                    const int32_t *sub_sys, hipStream_t s);
template <class VT>
void launch_spmv(const DevMat<VT> &M, const VT *x, VT *y, const SysState *st, const int32_t *sub_sys,
                 hipStream_t s);
// fc = B f (see k_restrict)
template <class VT, class FT>
void launch_restrict(const DevMat<VT> &B, const FT *f, VT *fc, const SysState *st, const int32_t *sub_sys,
                     hipStream_t s);
template <class VT, class FT>
void launch_prolong(const DevMat<VT> &P, const VT *m, const FT *f, const VT *xc, VT *z, const SysState *st,
                    const int32_t *sub_sys, hipStream_t s);
template <class VT, class FT, class OT, bool DOT>
void launch_post(const DevMat<VT> &A, const VT *m, const FT *f, const VT *z, OT *x, double *part,
                 const SysState *st, const int32_t *sub_sys, hipStream_t s);
// res = f - A x and z = x + P xc (x may be null) for V-cycles with other
// than one pre-smoothing sweep
template <class VT, class FT>
void launch_resid(const DevMat<VT> &A, const FT *f, const VT *x, VT *res, const SysState *st,
                  const int32_t *sub_sys, hipStream_t s);
template <class VT>
void launch_prolong_add(const DevMat<VT> &P, const VT *x, const VT *xc, VT *z, const SysState *st,
                        const int32_t *sub_sys, hipStream_t s);

// ---- outer operator (launch_outer.hip) -----------------------------------
// A: block-diagonal part, off: couplings between subdomains (see OffM).
void launch_outer(int mode, int ndv, const DevMat<double> &A, const OffM &off, const double *x, const double *b,
                  double *out, const ZView &Z, double *part, const SysState *st, const int32_t *sub_sys,
                  hipStream_t s);
void launch_outer_spmv_plain(const DevMat<double> &A, const double *x, double *y, hipStream_t s);

}  // namespace dfamg
