// CDNA4 (gfx950) kernels of the deflated block-AMG Krylov solve.
//
// Layout conventions
//   * every row-parallel kernel works on a list of row tiles; a tile lies
//     inside one subdomain (hence one system), so per-tile partial sums are
//     segmented by construction and every reduction is deterministic (fixed
//     tile order, fixed wavefront/LDS reduction tree, no atomics);
//   * block b is mapped to tile (b % 8) * per + b / 8: workgroups are
//     dispatched round-robin over the 8 XCDs, so each XCD walks a contiguous
//     range of tiles and its L2 holds the neighbouring rows of its tiles;
//   * sparse matrices come in two layouts, chosen per matrix by the setup
//     autotuner: sliced ELLPACK (64-row slices, one row per lane, RPL rows per
//     lane, slice-major storage so a wavefront streams consecutive addresses)
//     or CSR with L lanes per row (for the long rows of Galerkin operators and
//     of the restriction);
//   * matrix entries are streamed with non-temporal loads so that the
//     gathered vectors keep the caches;
//   * Krylov scalars live on the device (SysState, one per system) and every
//     in-loop kernel returns early once its system has stopped, so a fixed
//     launch sequence (or a captured graph) can run past convergence.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dfamg {

constexpr int kWave = 64;
constexpr int kBlock = 256;          // 4 wavefronts
constexpr int kWideBlock = 1024;     // per-system reductions
constexpr int kMaxNdv = 8;
constexpr int kGemvRows = 4;         // rows of E^{-1} per GEMV block (one per wavefront)

struct DevTile {
    int32_t row0, nrows, sub, slot;
};

// Per-system Krylov state.
struct SysState {
    double rho, alpha, beta, omega;  // CG / BiCGStab scalars
    double pq;                       // (p, P A p) of the last CG step
    double bb;                       // ||b||^2
    double rr;                       // ||r||^2
    double relres;                   // ||r|| / ||b|| of the last test
    double tt, ts;                   // BiCGStab (t,t), (t,s)
    double rho_old, pad0;
    double bl[8];                    // BiCGStab(2): see the kBl* slots below
    int32_t iter;
    int32_t done;                    // 0 running, 1 converged, 2 maxiter, 3 nan, 4 breakdown
    int32_t half;                    // BiCGStab: stopped on the half step
    int32_t pad;
};

enum { kRunning = 0, kConverged = 1, kMaxIter = 2, kNaN = 3, kBreakdown = 4 };

// BiCGStab(2) scalars in SysState::bl (rho0 lives in rho, alpha, beta, omega
// in their fields)
enum { kBlRhoNext = 0, kBlTau = 1, kBlSigma1 = 2, kBlG1p = 3, kBlG2p = 4, kBlG1 = 5, kBlG2 = 6 };

// ---------------------------------------------------------------------------
// matrix views
// ---------------------------------------------------------------------------

// SELL: I16 selects 16-bit column offsets from a per-tile base (cbase);
// ridx (may be null) gives the tile-local row of each slot when the rows of
// the tile are stored sorted by length.  STAGE (requires I16) first copies
// the tile's column window [cbase, cbase + cspan) of the gathered vector into
// LDS, so the irregular gathers of Galerkin operators and transfer matrices
// hit LDS instead of fetching a cache line per lane from L2.
template <class VT, int RPL, bool I16, bool STAGE>
struct SellM {
    const DevTile *tiles;
    const int64_t *soff;
    const int32_t *sw;
    const int32_t *col;
    const uint16_t *col16;
    const int32_t *cbase;
    const int32_t *cspan;
    const int16_t *ridx;
    const VT *val;
    int32_t ntiles;
};

// CSR with L lanes per row; STAGE as above (cbase/cspan per tile), or, when
// ucol is set, from a gather list: the tile's distinct columns
// ucol[uoff[tile] .. uoff[tile+1]) in ascending order are copied into LDS and
// col16 (16 bits: a list never exceeds the LDS budget) holds each entry's
// position in that list, so a column that several rows of the tile read is
// fetched once per tile however far apart the columns lie.
template <class VT, int L, bool STAGE>
struct CsrM {
    const DevTile *tiles;
    const int32_t *ptr;
    const int32_t *col;
    const int32_t *cbase;
    const int32_t *cspan;
    const VT *val;
    int32_t ntiles;
    const int32_t *uoff;
    const int32_t *ucol;
    const uint16_t *col16;
};

// BSR with 4 x 4 blocks: one column index per block (the block's first
// scalar column / 4), 16 values per block, row-major within the block;
// bptr over the block rows of the whole matrix.  Tiles hold 256 rows (64
// block rows) of one subdomain.
template <class VT>
struct BsrM {
    const DevTile *tiles;
    const int32_t *bptr;
    const int32_t *bcol;
    const VT *val;
    int32_t ntiles;
};

// A restriction (or any operator whose rows are long and whose columns are
// a contiguous range per subdomain) split by column tiles: every row's
// entries in one column tile form a segment; a column tile's segments are
// stored as SELL-64 slices (segments sorted by length, entry e of lane l at
// soff[slice] + 64 e + l, 16-bit columns relative to the tile's first
// column).  One block stages the tile's part of the input vector in LDS once
// and writes one partial sum per segment to part[slot]; the partials of a
// row are then added in column-tile order (k_seg_combine).
template <class VT>
struct SegM {
    const DevTile *tiles;      // column tiles: row0 = first column, nrows = width, sub
    const int32_t *slices;     // [ntiles + 1]: slices of each column tile
    const int64_t *soff;
    const int32_t *sw;
    const uint16_t *col16;
    const VT *val;
    const int32_t *slot;       // [64 * slices]: partial of each lane, -1 = padding
    int32_t ntiles;
};

__device__ __forceinline__ int tile_of_block(int ntiles) {
    const int per = (ntiles + 7) >> 3;
    return (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
}

inline int grid_for_tiles(int ntiles) { return ((ntiles + 7) >> 3) * 8; }

typedef double f64x2 __attribute__((ext_vector_type(2)));

template <class T>
__device__ __forceinline__ T stream_load(const T *p) {
    return __builtin_nontemporal_load(p);
}

// Dynamic LDS of the staged layouts.
extern __shared__ double dfamg_stage_lds[];

// Copies src(cb + k), k < span, into LDS; every thread of the block calls it.
// Four loads per thread are issued before the first store, so a thread waits
// for one memory latency per four entries rather than per entry.
template <class VT, int NT = kBlock, class SRC>
__device__ __forceinline__ VT *stage_window(int cb, int span, SRC src) {
    VT *lds = reinterpret_cast<VT *>(dfamg_stage_lds);
    int k = threadIdx.x;
    for (; k + 3 * NT < span; k += 4 * NT) {
        VT v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = (VT)src(cb + k + u * NT);
#pragma unroll
        for (int u = 0; u < 4; ++u) lds[k + u * NT] = v[u];
    }
    for (; k < span; k += NT) lds[k] = (VT)src(cb + k);
    __syncthreads();
    return lds;
}

// Copies src(ucol[u0 + k]), k < u1 - u0, into LDS; every thread of the block
// calls it.  The list indices of four entries are loaded first, then their
// four values, then the four stores.
template <class VT, class SRC>
__device__ __forceinline__ VT *stage_list(int u0, int u1, const int32_t *__restrict__ ucol, SRC src) {
    VT *lds = reinterpret_cast<VT *>(dfamg_stage_lds);
    const int n = u1 - u0;
    const int32_t *__restrict__ uc = ucol + u0;
    int k = threadIdx.x;
    for (; k + 3 * kBlock < n; k += 4 * kBlock) {
        int c[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) c[u] = uc[k + u * kBlock];
        VT v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = (VT)src(c[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u) lds[k + u * kBlock] = v[u];
    }
    for (; k < n; k += kBlock) lds[k] = (VT)src(uc[k]);
    __syncthreads();
    return lds;
}

// sum_j val_j * x(cadd + col_j) over one SELL row (w entries, stride 64; w
// is the same for the whole wavefront).  Per chunk of eight entries the
// column and value loads are issued first, then the eight gathers (entries
// past w gather x(cadd), a valid position, and are not added), then the
// sums in entry order: the gathers of a chunk are in flight together
// instead of one memory round trip each.
template <class VT, class ACC, class CT, class XF>
__device__ __forceinline__ ACC sell_dot(const CT *__restrict__ col, int cadd, const VT *__restrict__ val,
                                        int64_t off, int w, XF x) {
    ACC acc = 0;
    for (int j0 = 0; j0 < w; j0 += 8) {
        int c[8];
        VT v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            c[u] = cadd;
            v[u] = 0;
            if (j0 + u < w) {
                c[u] = cadd + (int)stream_load(col + off + (int64_t)(j0 + u) * 64);
                v[u] = stream_load(val + off + (int64_t)(j0 + u) * 64);
            }
        }
        ACC xv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) xv[u] = (ACC)x(c[u]);
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (j0 + u < w) acc += (ACC)v[u] * xv[u];
    }
    return acc;
}

// Two SELL rows of one lane at once (slices with widths w0 and w1, both
// wave-uniform): per chunk of eight entries, the loads of both rows, then
// both rows' gathers, then the sums in entry order (each row summed as by
// sell_dot, so the results are the same to the bit); twice the loads in
// flight per wavefront.
template <class VT, class ACC, class CT, class XF>
__device__ __forceinline__ void sell_dot2(const CT *__restrict__ col, int cadd, const VT *__restrict__ val,
                                          int64_t off0, int w0, int64_t off1, int w1, XF x, ACC &acc0, ACC &acc1) {
    acc0 = 0;
    acc1 = 0;
    const int wm = w0 > w1 ? w0 : w1;
    for (int j0 = 0; j0 < wm; j0 += 8) {
        int c0[8], c1[8];
        VT v0[8], v1[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            c0[u] = cadd;
            v0[u] = 0;
            c1[u] = cadd;
            v1[u] = 0;
            if (j0 + u < w0) {
                c0[u] = cadd + (int)stream_load(col + off0 + (int64_t)(j0 + u) * 64);
                v0[u] = stream_load(val + off0 + (int64_t)(j0 + u) * 64);
            }
            if (j0 + u < w1) {
                c1[u] = cadd + (int)stream_load(col + off1 + (int64_t)(j0 + u) * 64);
                v1[u] = stream_load(val + off1 + (int64_t)(j0 + u) * 64);
            }
        }
        ACC x0[8], x1[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            x0[u] = (ACC)x(c0[u]);
            x1[u] = (ACC)x(c1[u]);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (j0 + u < w0) acc0 += (ACC)v0[u] * x0[u];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (j0 + u < w1) acc1 += (ACC)v1[u] * x1[u];
    }
}

// Calls f(row, sum_j a_rj src(c_j)) for every row of the tile owned by this
// thread (exactly once per row over the block).  Every thread of the block
// must call it (the staged layouts synchronise the block).
template <class ACC, class VT, int RPL, bool I16, bool STAGE, class SRC, class F>
__device__ __forceinline__ void for_rows(const SellM<VT, RPL, I16, STAGE> &M, int tile, const DevTile &T, SRC src,
                                         F f) {
    static_assert(!STAGE || I16, "staged SELL needs 16-bit column offsets");
    // the wavefront index is uniform: slice offsets and widths become scalar loads
    const int t = threadIdx.x, w = __builtin_amdgcn_readfirstlane(t >> 6), lane = t & 63;
    const int cb = I16 ? M.cbase[tile] : 0;
    const VT *lds = nullptr;
    if (STAGE) lds = stage_window<VT>(cb, M.cspan[tile], src);
    if constexpr (RPL % 2 == 0) {
        // slices in pairs (their padding lanes load zero values at valid
        // positions; only rows of the tile are passed to f)
#pragma unroll
        for (int r = 0; r < RPL; r += 2) {
            const int sl = w * RPL + r;
            const int64_t si = (int64_t)tile * 4 * RPL + sl;
            ACC acc[2];
            if (STAGE)
                sell_dot2<VT, ACC>(M.col16, 0, M.val, M.soff[si] + lane, M.sw[si], M.soff[si + 1] + lane, M.sw[si + 1],
                                   [&](int c) { return lds[c]; }, acc[0], acc[1]);
            else if (I16)
                sell_dot2<VT, ACC>(M.col16, cb, M.val, M.soff[si] + lane, M.sw[si], M.soff[si + 1] + lane,
                                   M.sw[si + 1], src, acc[0], acc[1]);
            else
                sell_dot2<VT, ACC>(M.col, 0, M.val, M.soff[si] + lane, M.sw[si], M.soff[si + 1] + lane, M.sw[si + 1],
                                   src, acc[0], acc[1]);
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int lr = (sl + q) * 64 + lane;
                if (lr < T.nrows) {
                    const int lrow = M.ridx ? (int)M.ridx[(int64_t)tile * 256 * RPL + lr] : lr;
                    f(T.row0 + lrow, acc[q]);
                }
            }
        }
        return;
    }
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int sl = w * RPL + r;
        const int lr = sl * 64 + lane;
        if (lr < T.nrows) {
            const int64_t si = (int64_t)tile * 4 * RPL + sl;
            ACC acc;
            if (STAGE) acc = sell_dot<VT, ACC>(M.col16, 0, M.val, M.soff[si] + lane, M.sw[si], [&](int c) { return lds[c]; });
            else if (I16) acc = sell_dot<VT, ACC>(M.col16, cb, M.val, M.soff[si] + lane, M.sw[si], src);
            else acc = sell_dot<VT, ACC>(M.col, 0, M.val, M.soff[si] + lane, M.sw[si], src);
            const int lrow = M.ridx ? (int)M.ridx[(int64_t)tile * 256 * RPL + lr] : lr;
            f(T.row0 + lrow, acc);
        }
    }
}

// CSR: groups of L lanes share a row; the kBlock/L groups of the block walk
// the tile's rows with stride kBlock/L (the trip count is uniform inside a
// group, so the group's shuffles always see all of its lanes).
template <class ACC, class VT, int L, bool STAGE, class SRC, class F>
__device__ __forceinline__ void for_rows(const CsrM<VT, L, STAGE> &M, int tile, const DevTile &T, SRC src, F f) {
    constexpr int G = kBlock / L;
    const int t = threadIdx.x, g = t / L, lane = t % L;
    int cb = 0;
    const VT *lds = nullptr;
    if (STAGE) {
        if (M.ucol) {
            lds = stage_list<VT>(M.uoff[tile], M.uoff[tile + 1], M.ucol, src);
        } else {
            cb = M.cbase[tile];
            lds = stage_window<VT>(cb, M.cspan[tile], src);
        }
    }
    auto x = [&](int c) -> VT {
        if (STAGE) return lds[c - cb];
        return (VT)src(c);
    };
    // A row is read in chunks of 8 L entries: per chunk every lane issues
    // its (up to) eight column and value loads, then the eight gathers
    // (entries past the row's end gather x at the window base, a valid
    // position, and are not added), then sums them in entry order, so a
    // row of up to 8 L entries costs one load round trip and one gather
    // round trip.  The next row's pointers are loaded before the current
    // row is summed.
    auto rows = [&](const auto *__restrict__ colp) {
        int lr = g;
        int n0 = 0, n1 = 0;
        if (lr < T.nrows) {
            n0 = M.ptr[T.row0 + lr];
            n1 = M.ptr[T.row0 + lr + 1];
        }
        for (; lr < T.nrows; lr += G) {
            const int row = T.row0 + lr;
            const int k0 = n0, k1 = n1;
            if (lr + G < T.nrows) {
                n0 = M.ptr[row + G];
                n1 = M.ptr[row + G + 1];
            }
            ACC acc = 0;
            for (int kc = k0 + lane; kc - lane < k1; kc += 8 * L) {
                int c[8];
                VT v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    c[u] = cb;
                    v[u] = 0;
                    if (kc + u * L < k1) {
                        c[u] = (int)stream_load(colp + kc + u * L);
                        v[u] = stream_load(M.val + kc + u * L);
                    }
                }
                ACC xv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) xv[u] = (ACC)x(c[u]);
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (kc + u * L < k1) acc += (ACC)v[u] * xv[u];
            }
#pragma unroll
            for (int o = L / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, L);
            if (lane == 0) f(row, acc);
        }
    };
    if (STAGE && M.ucol) rows(M.col16);
    else rows(M.col);
}

// BSR4: thread t takes row t of the tile; the four threads of a block row
// read the block's column once and their own row of each block (16 bytes
// of FP32 or 32 of FP64, one 64- or 128-byte segment per block row), and the
// four gathered entries the block row shares.
template <class ACC, class VT, class SRC, class F>
__device__ __forceinline__ void for_rows(const BsrM<VT> &M, int tile, const DevTile &T, SRC src, F f) {
    (void)tile;
    const int lr = threadIdx.x;
    if (lr >= T.nrows) return;
    const int row = T.row0 + lr, br = row >> 2, r = row & 3;
    const int k0 = M.bptr[br], k1 = M.bptr[br + 1];
    ACC acc = 0;
    for (int k = k0; k < k1; ++k) {
        const int c = 4 * stream_load(M.bcol + k);
        const VT *v = M.val + (int64_t)k * 16 + r * 4;
        VT a[4];
        if constexpr (sizeof(VT) == 8) {
            const f64x2 p0 = stream_load(reinterpret_cast<const f64x2 *>(v));
            const f64x2 p1 = stream_load(reinterpret_cast<const f64x2 *>(v) + 1);
            a[0] = p0.x;
            a[1] = p0.y;
            a[2] = p1.x;
            a[3] = p1.y;
        } else {
            typedef float f32x4 __attribute__((ext_vector_type(4)));
            const f32x4 p = stream_load(reinterpret_cast<const f32x4 *>(v));
            a[0] = p.x;
            a[1] = p.y;
            a[2] = p.z;
            a[3] = p.w;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) acc += (ACC)a[q] * (ACC)src(c + q);
    }
    f(row, acc);
}

// Rows of a tile for kernels without a matrix: thread t takes rows t, t+256, ..
template <class F>
__device__ __forceinline__ void for_tile_rows(const DevTile &T, F f) {
#pragma unroll 4
    for (int lr = threadIdx.x; lr < T.nrows; lr += kBlock) f(T.row0 + lr);
}

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Sum over a block of `nthreads` (multiple of 64); result valid in every thread.
__device__ __forceinline__ double block_sum(double v, double *lds, int nthreads) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    double r = 0.0;
    const int nw = nthreads >> 6;
    for (int i = 0; i < nw; ++i) r += lds[i];
    __syncthreads();
    return r;
}

// Deterministic sum of a[lo..hi) by one wavefront (all lanes get the result).
__device__ __forceinline__ double wave_range_sum(const double *__restrict__ a, int lo, int hi) {
    const int lane = threadIdx.x & 63;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int i = lo + lane;
    for (; i + 192 < hi; i += 256) {
        s0 += a[i];
        s1 += a[i + 64];
        s2 += a[i + 128];
        s3 += a[i + 192];
    }
    for (; i < hi; i += 64) s0 += a[i];
    return wave_sum((s0 + s1) + (s2 + s3));
}

// ---------------------------------------------------------------------------
// outer operator and deflation
// ---------------------------------------------------------------------------

// The global operator is stored as its block-diagonal part (columns inside
// the row's subdomain, held in one of the layouts above, which can then use
// 16-bit column offsets and LDS staging) plus the couplings between
// subdomains in CSR over all rows (ptr has n + 1 entries); any[t] is nonzero
// when tile t of the block-diagonal layout has a coupled row, so the other
// tiles skip the pointer reads.
struct OffM {
    const int32_t *any;
    const int32_t *ptr;
    const int32_t *col;
    const double *val;
};

// Epilogue partials per tile, slot-major: part[q * nslots + slot]
//   MODE 0: q = A p;     partials (p,q), Z^T q              (CG operator product)
//   MODE 1: w = b - A y; partials (b,b), Z^T w              (initial / final residual)
//   MODE 2: w = b - A x; partial (w,w)                      (true residual)
//   MODE 3: q = A p;     partials Z^T q, skip when stopped  (BiCGStab operator product)
//   MODE 4: q = A p;     no partials, no stop check         (plain product)
// The thread that forms a row's block-diagonal sum adds the row's couplings.
// Deflation vectors as the operator epilogue reads them: row-major FP64 (z),
// or, when every column of every subdomain block takes at most 256 distinct
// values (constant, linear and indicator vectors on structured grids), one
// byte per entry that indexes the block's table of those values -- the same
// FP64 numbers in an eighth of the bytes.
struct ZView {
    const double *z;
    const uint8_t *code;      // null: read z
    const double *tab;
    const int32_t *tab_off;   // per (subdomain, column): first table entry
};

template <int MODE, int NDV, class MAT>
__global__ void __launch_bounds__(kBlock) k_outer(MAT A, OffM off, const double *__restrict__ x,
                                                  const double *__restrict__ b, double *__restrict__ out,
                                                  ZView Zv, int ndv_rt, double *__restrict__ part,
                                                  int32_t nslots, const SysState *__restrict__ st,
                                                  const int32_t *__restrict__ sub_sys) {
    __shared__ double lds[(kMaxNdv + 1) * 4];
    const int ndv = ndv_rt;   // <= NDV, the unroll bound
    const int tile = tile_of_block(A.ntiles);
    if (tile >= A.ntiles) return;
    const DevTile T = A.tiles[tile];
    if ((MODE == 0 || MODE == 3) && st[sub_sys[T.sub]].done) return;
    double d0 = 0.0;
    double zq[NDV > 0 ? NDV : 1];
    const double *ztab[NDV > 0 ? NDV : 1];
    const bool coded = Zv.code != nullptr;
#pragma unroll
    for (int k = 0; k < NDV; ++k) {
        zq[k] = 0.0;
        ztab[k] = (coded && k < ndv) ? Zv.tab + Zv.tab_off[T.sub * ndv + k] : nullptr;
    }
    const bool coupled = off.any[tile] != 0;
    auto finish_row = [&](int row, double ax) {
        if (coupled) {
            int e = off.ptr[row];
            const int e1 = off.ptr[row + 1];
            for (; e + 4 <= e1; e += 4) {   // four independent gathers in flight
                int c[4];
                double v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    c[u] = off.col[e + u];
                    v[u] = off.val[e + u];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) ax += v[u] * x[c[u]];
            }
            for (; e < e1; ++e) ax += off.val[e] * x[off.col[e]];
        }
        double v;
        if (MODE == 0 || MODE == 3 || MODE == 4) {
            v = ax;
            if (MODE == 0) d0 += x[row] * v;
        } else {
            const double bi = b[row];
            v = bi - ax;
            d0 += MODE == 1 ? bi * bi : v * v;
        }
        out[row] = v;
        if (MODE == 0 || MODE == 1 || MODE == 3) {
            if (coded && NDV == 4 && ndv == 4) {
                const uint32_t c4 = *reinterpret_cast<const uint32_t *>(Zv.code + (int64_t)row * 4);
#pragma unroll
                for (int k = 0; k < NDV; ++k) zq[k] += ztab[k][(c4 >> (8 * k)) & 0xff] * v;
            } else if (coded) {
#pragma unroll
                for (int k = 0; k < NDV; ++k)
                    if (k < ndv) zq[k] += ztab[k][Zv.code[(int64_t)row * ndv + k]] * v;
            } else {
#pragma unroll
                for (int k = 0; k < NDV; ++k)
                    if (k < ndv) zq[k] += Zv.z[(int64_t)row * ndv + k] * v;
            }
        }
    };
    for_rows<double>(A, tile, T, [&](int c) { return x[c]; }, finish_row);
    if (MODE == 4) return;
    const int t = threadIdx.x, w = t >> 6;
    const int nq = (MODE == 2) ? 1 : ndv + 1;
    d0 = wave_sum(d0);
    if ((t & 63) == 0) lds[w] = d0;
    auto zq_one_by_one = [&] {
#pragma unroll
        for (int k = 0; k < NDV; ++k) {
            if (k < ndv && MODE != 2) {
                const double s = wave_sum(zq[k]);
                if ((t & 63) == 0) lds[4 * (k + 1) + w] = s;
            }
        }
    };
    if constexpr (NDV == 4) {
        if (ndv == 4 && MODE != 2) {
            // the four Z^T q sums of the wavefront together: seven exchanges
            // instead of four times six.  Across lane halves each lane keeps
            // two of the four values and adds its partner's, then one of the
            // two across quarters, then the usual butterfly over the 16-lane
            // group; lane 16 q ends with the sum of value q (the same sums,
            // in the same order, as the butterfly of each value alone).
            const int lane = t & 63;
            const bool hi = (lane & 32) != 0, mid = (lane & 16) != 0;
            double k0 = hi ? zq[2] : zq[0], k1 = hi ? zq[3] : zq[1];
            const double g0 = hi ? zq[0] : zq[2], g1 = hi ? zq[1] : zq[3];
            k0 += __shfl_xor(g0, 32, kWave);
            k1 += __shfl_xor(g1, 32, kWave);
            double v = mid ? k1 : k0;
            v += __shfl_xor(mid ? k0 : k1, 16, kWave);
#pragma unroll
            for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
            if ((lane & 15) == 0) lds[4 * (1 + (lane >> 4)) + w] = v;
        } else {
            zq_one_by_one();
        }
    } else {
        zq_one_by_one();
    }
    __syncthreads();
    if (t < nq && (MODE != 3 || t > 0)) {
        const double s = ((lds[4 * t] + lds[4 * t + 1]) + lds[4 * t + 2]) + lds[4 * t + 3];
        part[(int64_t)t * nslots + T.slot] = s;
    }
}

// One block per subdomain: sums of the subdomain's tile partials.
//   t1[sub*ndv + k] = sum of partial k+1;  psub[sub] = sum of partial 0
template <bool CHECK_DONE>
__global__ void __launch_bounds__(kBlock) k_t1(const double *__restrict__ part, int32_t nslots,
                                               const int32_t *__restrict__ sub_tile_off, int ndv,
                                               double *__restrict__ t1, double *__restrict__ psub,
                                               const SysState *__restrict__ st, const int32_t *__restrict__ sub_sys,
                                               int with_p0) {
    const int sub = blockIdx.x;
    if (CHECK_DONE && st[sub_sys[sub]].done) return;
    const int w = threadIdx.x >> 6;
    const int lo = sub_tile_off[sub], hi = sub_tile_off[sub + 1];
    for (int q = w; q <= ndv; q += 4) {
        if (q == 0 && !with_p0) continue;
        const double s = wave_range_sum(part + (int64_t)q * nslots, lo, hi);
        if ((threadIdx.x & 63) == 0) {
            if (q == 0) psub[sub] = s;
            else t1[(int64_t)sub * ndv + q - 1] = s;
        }
    }
}

// t2 = E^{-1} t1: one wavefront per row of E^{-1} (row-major, lanes stride
// the columns so every load is a contiguous 512-byte access), kGemvRows rows
// per block; each block also leaves the partial sum_i t1_i t2_i of its rows.
struct GemvJob {
    int32_t sys, row0, m, coarse0;   // coarse0 = first coarse index of the system
    int64_t e_off;
};

template <bool CHECK_DONE>
__global__ void __launch_bounds__(kBlock) k_egemv(const GemvJob *__restrict__ jobs, const double *__restrict__ Einv,
                                                  const double *__restrict__ t1, double *__restrict__ t2,
                                                  double *__restrict__ tt_part, const SysState *__restrict__ st) {
    __shared__ double red[kGemvRows];
    const GemvJob J = jobs[blockIdx.x];
    if (CHECK_DONE && st[J.sys].done) return;
    const int m = J.m;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const double *tl = t1 + J.coarse0;
    double tt = 0.0;
    const int i = J.row0 + w;
    if (i < m) {
        const double *row = Einv + J.e_off + (int64_t)i * m;
        double a0 = 0.0, a1 = 0.0;
        int j = lane;
        for (; j + 64 < m; j += 128) {
            a0 += row[j] * tl[j];
            a1 += row[j + 64] * tl[j + 64];
        }
        if (j < m) a0 += row[j] * tl[j];
        const double v = wave_sum(a0 + a1);
        if (lane == 0) {
            t2[J.coarse0 + i] = v;
            tt = v * tl[i];
        }
    }
    if (lane == 0) red[w] = tt;
    __syncthreads();
    if (threadIdx.x == 0) tt_part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// Per-system offsets used by the fused scalar computations.
struct SysRanges {
    const int32_t *sub_off;   // subdomains of each system
    const int32_t *job_off;   // GEMV jobs of each system
};

// (p, P A p) = (p, A p) - t1 . t2 for symmetric A, summed in a fixed order
// by one wavefront.
__device__ __forceinline__ double cg_curvature(const double *__restrict__ psub, const double *__restrict__ tt_part,
                                               const SysRanges &R, int sys) {
    const double pq = wave_range_sum(psub, R.sub_off[sys], R.sub_off[sys + 1]);
    const double tt = wave_range_sum(tt_part, R.job_off[sys], R.job_off[sys + 1]);
    return pq - tt;
}

// MODE 0 (CG): alpha = rho / (p,PAp); w = q - AZ t2; y += alpha p; r -= alpha w; partial (r,r)
// MODE 1 (init): r = w - AZ t2; partial (r,r)
// MODE 2 (projection only): out = v - AZ t2
// MODE 3 (flexible CG): MODE 0 and the partial (r, s) of the new residual with
//         the previous preconditioned residual s, in part[ntiles + slot]
template <int MODE, int NDV>
__global__ void __launch_bounds__(kBlock) k_update(
    const DevTile *__restrict__ tiles, int32_t ntiles, const double *__restrict__ p, const double *__restrict__ q,
    double *__restrict__ y, double *__restrict__ r, const double *__restrict__ AZown, int ndv_rt,
    const int32_t *__restrict__ offp, const int32_t *__restrict__ offc, const double *__restrict__ offv,
    const double *__restrict__ t2, double *__restrict__ part, SysState *__restrict__ st,
    const int32_t *__restrict__ sub_sys, const double *__restrict__ psub, const double *__restrict__ tt_part,
    SysRanges R, const double *__restrict__ s_prev) {
    constexpr bool CG = MODE == 0 || MODE == 3;
    __shared__ double lds[4];
    __shared__ double alpha_s;
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    const int ndv = ndv_rt;   // <= NDV, the unroll bound
    // A row's operands do not depend on alpha, so they are loaded before it
    // (row tiles hold at most kBlock rows: one row per thread) and their
    // memory round trip overlaps the curvature reads and the block's
    // synchronisation instead of following them; a stopped system's rows are
    // not read at all (batched systems stop at different iterations).
    struct RowIn {
        double q, p, y, r, s;
        int e, e1;
        f64x2 a01, a23;   // the row of the own AZ block (ndv == 4)
    };
    auto load_row = [&](int row) {
        RowIn o{};
        o.q = stream_load(q + row);
        if (CG) {
            o.p = stream_load(p + row);
            o.y = y[row];
            o.r = r[row];
        }
        if (MODE == 3) o.s = stream_load(s_prev + row);
        if (ndv > 0) {
            o.e = offp[row];
            o.e1 = offp[row + 1];
        }
        if (NDV == 4 && ndv == 4) {
            // one row of the own AZ block is 32 contiguous bytes
            const f64x2 *az = reinterpret_cast<const f64x2 *>(AZown + (int64_t)row * 4);
            o.a01 = stream_load(az);
            o.a23 = stream_load(az + 1);
        }
        return o;
    };
    const int sys = sub_sys[T.sub];
    SysState &S = st[sys];
    if (CG && S.done) return;
    const bool own = (int)threadIdx.x < T.nrows;
    RowIn first{};
    if (own) first = load_row(T.row0 + (int)threadIdx.x);
    if (CG) {
        if (threadIdx.x < 64) {
            const double pq = cg_curvature(psub, tt_part, R, sys);
            if (threadIdx.x == 0) alpha_s = S.rho / pq;
        }
        __syncthreads();
    }
    const double a = CG ? alpha_s : 0.0;
    double rr = 0.0, rs = 0.0;
    double t2s[NDV > 0 ? NDV : 1];
#pragma unroll
    for (int k = 0; k < NDV; ++k) t2s[k] = k < ndv ? t2[(int64_t)T.sub * ndv + k] : 0.0;
    auto finish_row = [&](int row, const RowIn &o) {
        double corr = 0.0;
        if (NDV == 4 && ndv == 4) {
            corr = ((o.a01.x * t2s[0] + o.a01.y * t2s[1]) + o.a23.x * t2s[2]) + o.a23.y * t2s[3];
        } else {
#pragma unroll
            for (int k = 0; k < NDV; ++k)
                if (k < ndv) corr += stream_load(AZown + (int64_t)row * ndv + k) * t2s[k];
        }
        // couplings to other subdomains: groups of four independent gathers
        int e = o.e;
        for (; e + 4 <= o.e1; e += 4) {
            int c[4];
            double v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                c[u] = offc[e + u];
                v[u] = offv[e + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) corr += v[u] * t2[c[u]];
        }
        for (; e < o.e1; ++e) corr += offv[e] * t2[offc[e]];
        const double wv = o.q - corr;
        if (CG) {
            y[row] = o.y + a * o.p;
            const double rn = o.r - a * wv;
            r[row] = rn;
            rr += rn * rn;
            if (MODE == 3) rs += rn * o.s;
        } else if (MODE == 1) {
            r[row] = wv;
            rr += wv * wv;
        } else {
            r[row] = wv;
        }
    };
    if (own) finish_row(T.row0 + (int)threadIdx.x, first);
    for (int lr = (int)threadIdx.x + kBlock; lr < T.nrows; lr += kBlock) finish_row(T.row0 + lr, load_row(T.row0 + lr));
    if (MODE == 2) return;
    const double s = block_sum(rr, lds, kBlock);
    if (threadIdx.x == 0) part[T.slot] = s;
    if (MODE == 3) {
        __syncthreads();
        const double s2 = block_sum(rs, lds, kBlock);
        if (threadIdx.x == 0) part[ntiles + T.slot] = s2;
    }
}

// x = y + Z t2 (solution recovery, x = y + Z lambda)
template <int NDV>
__global__ void __launch_bounds__(kBlock) k_expand(const DevTile *__restrict__ tiles, int32_t ntiles,
                                                   const double *__restrict__ y, const double *__restrict__ Z, int ndv_rt,
                                                   const double *__restrict__ t2, double *__restrict__ x) {
    const int ndv = ndv_rt;   // <= NDV, the unroll bound
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    const double *t2s = t2 + (int64_t)T.sub * ndv;
    for_tile_rows(T, [&](int row) {
        double v = y[row];
#pragma unroll
        for (int k = 0; k < NDV; ++k)
            if (k < ndv) v += Z[(int64_t)row * ndv + k] * t2s[k];
        x[row] = v;
    });
}

// Per-system sum of tile partials and the stopping test (1024 threads).
//   MODE 0 (loop): rr, iter++, history, stop test; records alpha and (p,PAp)
//   MODE 1 (initial residual): bb from the per-subdomain (b,b) sums, rr,
//           iter = 0, history[0], stop test
//   MODE 2 (true residual): out[sys] = sqrt(sum / bb)
template <int MODE>
__global__ void __launch_bounds__(kWideBlock) k_residual_test(const double *__restrict__ part,
                                                              const int32_t *__restrict__ sys_tile_off,
                                                              SysState *__restrict__ st, double *__restrict__ hist,
                                                              int32_t hist_stride, double rtol, int32_t maxiter,
                                                              double *__restrict__ out,
                                                              const double *__restrict__ psub, SysRanges R) {
    __shared__ double lds[16];
    const int sys = blockIdx.x;
    SysState &S = st[sys];
    if (MODE == 0 && S.done) return;
    double a = 0.0;
    for (int tl = sys_tile_off[sys] + threadIdx.x; tl < sys_tile_off[sys + 1]; tl += kWideBlock) a += part[tl];
    const double rr = block_sum(a, lds, kWideBlock);
    double bb = 0.0;
    if (MODE == 1) {
        if (threadIdx.x < 64) bb = wave_range_sum(psub, R.sub_off[sys], R.sub_off[sys + 1]);
    }
    if (threadIdx.x != 0) return;
    if (MODE == 1) S.bb = bb;
    // A non-finite ||b||^2 or ||r||^2 must not take the b = 0 shortcut below
    // (NaN > 0 is false): the relative residual is then NaN itself.
    const bool finite = isfinite(S.bb) && isfinite(rr);
    const double h = !finite ? (double)NAN : (S.bb > 0.0 ? sqrt(rr / S.bb) : 0.0);
    if (MODE == 2) {
        out[sys] = h;
        return;
    }
    S.rr = rr;
    S.relres = h;
    if (MODE == 1) {
        S.iter = 0;
        S.done = kRunning;
        S.half = 0;
        hist[(int64_t)sys * hist_stride] = h;
        if (!finite) S.done = kNaN;
        else if (S.bb == 0.0 || h <= rtol) S.done = kConverged;
        else if (maxiter == 0) S.done = kMaxIter;
        return;
    }
    const int it = S.iter + 1;
    S.iter = it;
    if (it < hist_stride) hist[(int64_t)sys * hist_stride + it] = h;
    if (!isfinite(h)) S.done = kNaN;
    else if (h <= rtol) S.done = kConverged;
    else if (it >= maxiter) S.done = kMaxIter;
}

// rho' = (r, s) from the tile partials of the preconditioner's last kernel
// (and the per-block partials of level-0 direct solves); CG beta.
//   MODE 0: beta = rho'/rho, rho = rho'      MODE 1 (init): rho = rho', beta = 0
template <int MODE>
__global__ void __launch_bounds__(kWideBlock) k_rho(const double *__restrict__ part,
                                                    const int32_t *__restrict__ sys_tile_off,
                                                    const double *__restrict__ part_job,
                                                    const int32_t *__restrict__ sys_job_off, SysState *__restrict__ st) {
    __shared__ double lds[16];
    const int sys = blockIdx.x;
    SysState &S = st[sys];
    if (S.done) return;
    double a = 0.0;
    for (int tl = sys_tile_off[sys] + threadIdx.x; tl < sys_tile_off[sys + 1]; tl += kWideBlock) a += part[tl];
    for (int j = sys_job_off[sys] + threadIdx.x; j < sys_job_off[sys + 1]; j += kWideBlock) a += part_job[j];
    const double rs = block_sum(a, lds, kWideBlock);
    if (threadIdx.x == 0) {
        S.beta = MODE == 0 ? rs / S.rho : 0.0;
        S.rho = rs;
    }
}

// Flexible CG: rho' = (r, s) as in k_rho, and with (r, s_prev) from the
// update's second partials beta = (rho' - (r, s_prev)) / rho (Polak-Ribiere)
static __global__ void __launch_bounds__(kWideBlock) k_rho_flexible(
    const double *__restrict__ part, const int32_t *__restrict__ sys_tile_off, const double *__restrict__ part_job,
    const int32_t *__restrict__ sys_job_off, const double *__restrict__ part_prev,
    const int32_t *__restrict__ sys_row_tile_off, SysState *__restrict__ st) {
    __shared__ double lds[16];
    const int sys = blockIdx.x;
    SysState &S = st[sys];
    if (S.done) return;
    double a = 0.0, b = 0.0;
    for (int tl = sys_tile_off[sys] + threadIdx.x; tl < sys_tile_off[sys + 1]; tl += kWideBlock) a += part[tl];
    for (int j = sys_job_off[sys] + threadIdx.x; j < sys_job_off[sys + 1]; j += kWideBlock) a += part_job[j];
    for (int tl = sys_row_tile_off[sys] + threadIdx.x; tl < sys_row_tile_off[sys + 1]; tl += kWideBlock)
        b += part_prev[tl];
    const double rs = block_sum(a, lds, kWideBlock);
    __syncthreads();
    const double rsp = block_sum(b, lds, kWideBlock);
    if (threadIdx.x == 0) {
        S.beta = (rs - rsp) / S.rho;
        S.rho = rs;
    }
}

// p = s + beta p   (INIT: p = s)
template <bool INIT>
__global__ void __launch_bounds__(kBlock) k_cg_direction(const DevTile *__restrict__ tiles, int32_t ntiles,
                                                         const double *__restrict__ s, double *__restrict__ p,
                                                         const SysState *__restrict__ st,
                                                         const int32_t *__restrict__ sub_sys) {
    // two row tiles per block (launched on grid_for_tiles((ntiles + 1) / 2)):
    // both tiles' descriptors and states are read first and then both rows'
    // s and p, so each block pays its chain of dependent reads (tile,
    // system, state, data) once per two tiles
    const int pairs = (ntiles + 1) >> 1;
    const int pair = tile_of_block(pairs);
    if (pair >= pairs) return;
    const int t0 = 2 * pair;
    const bool has1 = t0 + 1 < ntiles;
    const DevTile T0 = tiles[t0];
    const DevTile T1 = tiles[has1 ? t0 + 1 : t0];
    const SysState &S0 = st[sub_sys[T0.sub]];
    const SysState &S1 = st[sub_sys[T1.sub]];
    const bool go0 = INIT || !S0.done, go1 = has1 && (INIT || !S1.done);
    const double b0 = S0.beta, b1 = S1.beta;
    // row tiles hold at most kBlock rows: one row of each tile per thread
    const int lr = (int)threadIdx.x;
    const bool own0 = go0 && lr < T0.nrows, own1 = go1 && lr < T1.nrows;
    const int r0 = T0.row0 + lr, r1 = T1.row0 + lr;
    double s0 = 0.0, p0 = 0.0, s1 = 0.0, p1 = 0.0;
    if (own0) {
        s0 = s[r0];
        if (!INIT) p0 = p[r0];
    }
    if (own1) {
        s1 = s[r1];
        if (!INIT) p1 = p[r1];
    }
    if (own0) p[r0] = INIT ? s0 : s0 + b0 * p0;
    if (own1) p[r1] = INIT ? s1 : s1 + b1 * p1;
    for (int l = lr + kBlock; l < T0.nrows; l += kBlock)
        if (go0) p[T0.row0 + l] = INIT ? s[T0.row0 + l] : s[T0.row0 + l] + b0 * p[T0.row0 + l];
    for (int l = lr + kBlock; l < T1.nrows; l += kBlock)
        if (go1) p[T1.row0 + l] = INIT ? s[T1.row0 + l] : s[T1.row0 + l] + b1 * p[T1.row0 + l];
}

// ---------------------------------------------------------------------------
// BiCGStab (right-preconditioned, Templates form) on the deflated operator
// ---------------------------------------------------------------------------

// p = r + beta (p - omega v), beta = (rho / rho_old) (alpha / omega)
static __global__ void __launch_bounds__(kBlock) k_bicg_p(const DevTile *__restrict__ tiles, int32_t ntiles,
                                                          const double *__restrict__ r, const double *__restrict__ v,
                                                          double *__restrict__ p, const SysState *__restrict__ st,
                                                          const int32_t *__restrict__ sub_sys) {
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    const SysState &S = st[sub_sys[T.sub]];
    if (S.done) return;
    const double beta = (S.rho / S.rho_old) * (S.alpha / S.omega), om = S.omega;
    for_tile_rows(T, [&](int row) { p[row] = r[row] + beta * (p[row] - om * v[row]); });
}

// out = q - AZ t2 (the projected operator product) with partials
//   MODE 0: (rt, out)              -> v and (r~, v)
//   MODE 1: (out, s), (out, out)   -> t and (t, s), (t, t)
template <int MODE, int NDV>
__global__ void __launch_bounds__(kBlock) k_bicg_proj(
    const DevTile *__restrict__ tiles, int32_t ntiles, const double *__restrict__ q, double *__restrict__ out,
    const double *__restrict__ other, int ndv, const double *__restrict__ AZown, const int32_t *__restrict__ offp,
    const int32_t *__restrict__ offc, const double *__restrict__ offv, const double *__restrict__ t2,
    double *__restrict__ part, int32_t nslots, const SysState *__restrict__ st, const int32_t *__restrict__ sub_sys) {
    __shared__ double lds[4];
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    if (st[sub_sys[T.sub]].done) return;
    double d0 = 0.0, d1 = 0.0;
    double t2s[NDV > 0 ? NDV : 1];
#pragma unroll
    for (int k = 0; k < NDV; ++k) t2s[k] = k < ndv ? t2[(int64_t)T.sub * ndv + k] : 0.0;
    for_tile_rows(T, [&](int row) {
        // independent loads first, then the couplings in groups of four gathers
        const double qv = q[row], ov = other[row];
        int e = 0, e1 = 0;
        if (ndv > 0) {
            e = offp[row];
            e1 = offp[row + 1];
        }
        double corr = 0.0;
        if (NDV == 4 && ndv == 4) {
            const f64x2 *az = reinterpret_cast<const f64x2 *>(AZown + (int64_t)row * 4);
            const f64x2 a01 = stream_load(az), a23 = stream_load(az + 1);
            corr = ((a01.x * t2s[0] + a01.y * t2s[1]) + a23.x * t2s[2]) + a23.y * t2s[3];
        } else {
#pragma unroll
            for (int k = 0; k < NDV; ++k)
                if (k < ndv) corr += stream_load(AZown + (int64_t)row * ndv + k) * t2s[k];
        }
        for (; e + 4 <= e1; e += 4) {
            int c[4];
            double w[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                c[u] = offc[e + u];
                w[u] = offv[e + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) corr += w[u] * t2[c[u]];
        }
        for (; e < e1; ++e) corr += offv[e] * t2[offc[e]];
        const double v = qv - corr;
        out[row] = v;
        d0 += ov * v;
        if (MODE == 1) d1 += v * v;
    });
    const double s0 = block_sum(d0, lds, kBlock);
    if (threadIdx.x == 0) part[T.slot] = s0;
    if (MODE == 1) {
        const double s1 = block_sum(d1, lds, kBlock);
        if (threadIdx.x == 0) part[(int64_t)nslots + T.slot] = s1;
    }
}

// s = r - alpha v, partial (s, s)
static __global__ void __launch_bounds__(kBlock) k_bicg_s(const DevTile *__restrict__ tiles, int32_t ntiles,
                                                          const double *__restrict__ r, const double *__restrict__ v,
                                                          double *__restrict__ s, double *__restrict__ part,
                                                          const SysState *__restrict__ st,
                                                          const int32_t *__restrict__ sub_sys) {
    __shared__ double lds[4];
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    const SysState &S = st[sub_sys[T.sub]];
    if (S.done) return;
    const double a = S.alpha;
    double d = 0.0;
    for_tile_rows(T, [&](int row) {
        const double sv = r[row] - a * v[row];
        s[row] = sv;
        d += sv * sv;
    });
    const double sum = block_sum(d, lds, kBlock);
    if (threadIdx.x == 0) part[T.slot] = sum;
}

// y += alpha p^ + omega s^; r = s - omega t; partials (r, r), (r~, r)
static __global__ void __launch_bounds__(kBlock) k_bicg_update(
    const DevTile *__restrict__ tiles, int32_t ntiles, double *__restrict__ y, double *__restrict__ r,
    const double *__restrict__ ph, const double *__restrict__ sh, const double *__restrict__ s,
    const double *__restrict__ t, const double *__restrict__ rt, double *__restrict__ part, int32_t nslots,
    const SysState *__restrict__ st, const int32_t *__restrict__ sub_sys) {
    __shared__ double lds[4];
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    const SysState &S = st[sub_sys[T.sub]];
    if (S.done) return;
    const double a = S.alpha, om = S.omega;
    double d0 = 0.0, d1 = 0.0;
    for_tile_rows(T, [&](int row) {
        y[row] += a * ph[row] + om * sh[row];
        const double rn = s[row] - om * t[row];
        r[row] = rn;
        d0 += rn * rn;
        d1 += rt[row] * rn;
    });
    const double s0 = block_sum(d0, lds, kBlock);
    if (threadIdx.x == 0) part[T.slot] = s0;
    const double s1 = block_sum(d1, lds, kBlock);
    if (threadIdx.x == 0) part[(int64_t)nslots + T.slot] = s1;
}

// Per-system scalar steps of BiCGStab (1024 threads, sums of tile partials)
//   STEP 0 (alpha): alpha = rho / (r~, v)
//   STEP 1 (half test): ||s|| / ||b|| <= rtol stops with the half step
//   STEP 2 (omega): omega = (t, s) / (t, t)
//   STEP 3 (test): ||r|| / ||b||, iteration count, history, stop test,
//                  rho_old = rho, rho = (r~, r)
//   STEP 4 (init): rho = (r~, r) = ||r0||^2, rho_old = alpha = omega = 1
template <int STEP>
__global__ void __launch_bounds__(kWideBlock) k_bicg_scalar(const double *__restrict__ part, int32_t nslots,
                                                            const int32_t *__restrict__ sys_tile_off,
                                                            SysState *__restrict__ st, double *__restrict__ hist,
                                                            int32_t hist_stride, double rtol, int32_t maxiter) {
    __shared__ double lds[16];
    const int sys = blockIdx.x;
    SysState &S = st[sys];
    if (STEP != 4 && S.done) return;
    double a0 = 0.0, a1 = 0.0;
    for (int tl = sys_tile_off[sys] + threadIdx.x; tl < sys_tile_off[sys + 1]; tl += kWideBlock) {
        a0 += part[tl];
        if (STEP == 2 || STEP == 3) a1 += part[(int64_t)nslots + tl];
    }
    const double s0 = block_sum(a0, lds, kWideBlock);
    double s1 = 0.0;
    if (STEP == 2 || STEP == 3) s1 = block_sum(a1, lds, kWideBlock);
    if (threadIdx.x != 0) return;
    if (STEP == 4) {
        S.rho = S.rr;
        S.rho_old = S.alpha = S.omega = 1.0;
        return;
    }
    if (STEP == 0) {
        if (s0 == 0.0) {
            S.done = kBreakdown;
            return;
        }
        S.alpha = S.rho / s0;
        return;
    }
    if (STEP == 1) {
        const double h = sqrt(s0 / S.bb);
        if (!isfinite(h)) {
            S.done = kNaN;
        } else if (h <= rtol) {
            const int it = S.iter + 1;
            S.iter = it;
            S.relres = h;
            S.half = 1;
            if (it < hist_stride) hist[(int64_t)sys * hist_stride + it] = h;
            S.done = kConverged;
        }
        return;
    }
    if (STEP == 2) {
        const double om = s1 != 0.0 ? s0 / s1 : 0.0;
        S.tt = s1;
        S.ts = s0;
        if (om == 0.0) {   // counted as a (failed) iteration, y keeps its value
            S.iter = S.iter + 1;
            S.done = kBreakdown;
        }
        S.omega = om;
        return;
    }
    // STEP 3
    const double h = sqrt(s0 / S.bb);
    const int it = S.iter + 1;
    S.iter = it;
    S.rr = s0;
    S.relres = h;
    if (it < hist_stride) hist[(int64_t)sys * hist_stride + it] = h;
    S.rho_old = S.rho;
    S.rho = s1;
    if (!isfinite(h)) S.done = kNaN;
    else if (h <= rtol) S.done = kConverged;
    else if (it >= maxiter) S.done = kMaxIter;
    else if (s1 == 0.0) S.done = kBreakdown;
}

// After a half-step stop: y += alpha p^ for the systems that stopped there.
static __global__ void __launch_bounds__(kBlock) k_bicg_halffix(const DevTile *__restrict__ tiles, int32_t ntiles,
                                                                double *__restrict__ y, const double *__restrict__ ph,
                                                                const SysState *__restrict__ st,
                                                                const int32_t *__restrict__ sub_sys) {
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    const SysState &S = st[sub_sys[T.sub]];
    if (!S.half) return;
    const double a = S.alpha;
    for_tile_rows(T, [&](int row) { y[row] += a * ph[row]; });
}

// ---------------------------------------------------------------------------
// BiCGStab(2) (Sleijpen & Fokkema) on K = P A M^{-1}.  One cycle: two BiCG
// steps (u^ and r^ sequences, four products with K), then the
// minimal-residual step over r^_1, r^_2 (modified Gram-Schmidt).  The iterate
// y is updated with the preconditioned vectors whose products the residual
// recurrence used: pu0, pu1 (u^_1 = P A pu0, u^_2 = P A pu1) and pr0, pr1
// (r^_1 = P A pr0, r^_2 = P A pr1), kept by the same recurrences as u^ and r^,
// so the recurrence residual stays the true one with an inexact (FP32)
// preconditioner too.  The vector kernels carry the updates between the
// products, each with the dot products the next scalar step needs.
// ---------------------------------------------------------------------------

// u0 = r0 - beta u0; second step (r1 non-null) also u1 = r1 - beta u1 and
// pu0 = pr0 - beta pu0
static __global__ void __launch_bounds__(kBlock) k_bl_u(const DevTile *__restrict__ tiles, int32_t ntiles,
                                                        const double *__restrict__ r0, double *__restrict__ u0,
                                                        const double *__restrict__ r1, double *__restrict__ u1,
                                                        const double *__restrict__ pr0, double *__restrict__ pu0,
                                                        const SysState *__restrict__ st,
                                                        const int32_t *__restrict__ sub_sys) {
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    const SysState &S = st[sub_sys[T.sub]];
    if (S.done) return;
    const double beta = S.beta;
    for_tile_rows(T, [&](int row) {
        u0[row] = r0[row] - beta * u0[row];
        if (r1) {
            u1[row] = r1[row] - beta * u1[row];
            pu0[row] = pr0[row] - beta * pu0[row];
        }
    });
}

// r0 -= alpha u1, y += alpha pu0; second step (r1 non-null) also
// r1 -= alpha u2, pr0 -= alpha pu1, with partials (r1, r1), (r0, r1)
static __global__ void __launch_bounds__(kBlock) k_bl_r(const DevTile *__restrict__ tiles, int32_t ntiles,
                                                        double *__restrict__ r0, const double *__restrict__ u1,
                                                        double *__restrict__ r1, const double *__restrict__ u2,
                                                        double *__restrict__ pr0, const double *__restrict__ pu1,
                                                        double *__restrict__ y, const double *__restrict__ pu0,
                                                        double *__restrict__ part, int32_t nslots,
                                                        const SysState *__restrict__ st,
                                                        const int32_t *__restrict__ sub_sys) {
    __shared__ double lds[4];
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    const SysState &S = st[sub_sys[T.sub]];
    if (S.done) return;
    const double a = S.alpha;
    double d0 = 0.0, d1 = 0.0;
    for_tile_rows(T, [&](int row) {
        const double r0n = r0[row] - a * u1[row];
        r0[row] = r0n;
        y[row] += a * pu0[row];
        if (r1) {
            const double r1n = r1[row] - a * u2[row];
            r1[row] = r1n;
            pr0[row] -= a * pu1[row];
            d0 += r1n * r1n;
            d1 += r0n * r1n;
        }
    });
    if (!r1) return;
    const double s0 = block_sum(d0, lds, kBlock);
    if (threadIdx.x == 0) part[T.slot] = s0;
    const double s1 = block_sum(d1, lds, kBlock);
    if (threadIdx.x == 0) part[(int64_t)nslots + T.slot] = s1;
}

// r2 -= tau r1 (Gram-Schmidt) with partials (r2, r2), (r0, r2)
static __global__ void __launch_bounds__(kBlock) k_bl_mgs(const DevTile *__restrict__ tiles, int32_t ntiles,
                                                          const double *__restrict__ r0, const double *__restrict__ r1,
                                                          double *__restrict__ r2, double *__restrict__ part,
                                                          int32_t nslots, const SysState *__restrict__ st,
                                                          const int32_t *__restrict__ sub_sys) {
    __shared__ double lds[4];
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    const SysState &S = st[sub_sys[T.sub]];
    if (S.done) return;
    const double tau = S.bl[kBlTau];
    double d0 = 0.0, d1 = 0.0;
    for_tile_rows(T, [&](int row) {
        const double v = r2[row] - tau * r1[row];
        r2[row] = v;
        d0 += v * v;
        d1 += r0[row] * v;
    });
    const double s0 = block_sum(d0, lds, kBlock);
    if (threadIdx.x == 0) part[T.slot] = s0;
    const double s1 = block_sum(d1, lds, kBlock);
    if (threadIdx.x == 0) part[(int64_t)nslots + T.slot] = s1;
}

// end of a cycle: y += g1 pr0 + g2 pr1 (the iterate steps g1 r0 + g2 r1 of
// K d = r_0, gamma''_1 = gamma_2 for ell = 2); r0 -= g2' r2, then -= g1' r1;
// u0 -= g2 u2, then -= g1 u1; partials (r0, r0), (r0, r~)
static __global__ void __launch_bounds__(kBlock) k_bl_final(
    const DevTile *__restrict__ tiles, int32_t ntiles, double *__restrict__ y, const double *__restrict__ pr0,
    const double *__restrict__ pr1, double *__restrict__ r0, const double *__restrict__ r1,
    const double *__restrict__ r2, double *__restrict__ u0, const double *__restrict__ u1,
    const double *__restrict__ u2, const double *__restrict__ rt, double *__restrict__ part, int32_t nslots,
    const SysState *__restrict__ st, const int32_t *__restrict__ sub_sys) {
    __shared__ double lds[4];
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    const SysState &S = st[sub_sys[T.sub]];
    if (S.done) return;
    const double g1 = S.bl[kBlG1], g2 = S.bl[kBlG2], g1p = S.bl[kBlG1p], g2p = S.bl[kBlG2p];
    double d0 = 0.0, d1 = 0.0;
    for_tile_rows(T, [&](int row) {
        double yn = y[row] + g1 * pr0[row];
        yn += g2 * pr1[row];
        y[row] = yn;
        double rn = r0[row] - g2p * r2[row];
        rn -= g1p * r1[row];
        r0[row] = rn;
        double un = u0[row] - g2 * u2[row];
        un -= g1 * u1[row];
        u0[row] = un;
        d0 += rn * rn;
        d1 += rt[row] * rn;
    });
    const double s0 = block_sum(d0, lds, kBlock);
    if (threadIdx.x == 0) part[T.slot] = s0;
    const double s1 = block_sum(d1, lds, kBlock);
    if (threadIdx.x == 0) part[(int64_t)nslots + T.slot] = s1;
}

// Per-system scalar steps of BiCGStab(2) (1024 threads, sums of partials):
//   STEP 0 (cycle start): rho0 = -omega rho0, rho1 = (r0, r~) kept from the
//                         last test, beta = alpha rho1 / rho0, rho0 = rho1
//   STEP 1 (second step): rho1 = (r1, r~) from partials, beta and rho0 as above
//   STEP 2 (alpha):       alpha = rho0 / (u_{j+1}, r~)
//   STEP 3 (MR, first):   sigma1 = (r1, r1), tau = (r2, r1) / sigma1,
//                         g1' = (r0, r1) / sigma1 (three partial regions)
//   STEP 4 (MR, second):  sigma2 = (r2, r2), g2' = (r0, r2) / sigma2, g2 = g2',
//                         omega = g2, g1 = g1' - tau g2
//   STEP 5 (test):        ||r0|| / ||b||, iteration, history, stop test,
//                         (r0, r~) kept for the next cycle
//   STEP 6 (init):        rho0 = omega = 1, alpha = 0, (r0, r~) = ||r0||^2
// A zero rho, (u, r~) or sigma is a breakdown; one in the BiCG part leaves the
// cycle uncounted, one in the MR part counts it.
template <int STEP>
__global__ void __launch_bounds__(kWideBlock) k_bl_scalar(const double *__restrict__ part, int32_t nslots,
                                                          const int32_t *__restrict__ sys_tile_off,
                                                          SysState *__restrict__ st, double *__restrict__ hist,
                                                          int32_t hist_stride, double rtol, int32_t maxiter) {
    __shared__ double lds[16];
    const int sys = blockIdx.x;
    SysState &S = st[sys];
    if (STEP != 6 && S.done) return;
    constexpr bool two = STEP == 3 || STEP == 4 || STEP == 5;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    if (STEP == 1 || STEP == 2 || two) {
        for (int tl = sys_tile_off[sys] + threadIdx.x; tl < sys_tile_off[sys + 1]; tl += kWideBlock) {
            a0 += part[tl];
            if (two) a1 += part[(int64_t)nslots + tl];
            if (STEP == 3) a2 += part[2 * (int64_t)nslots + tl];
        }
    }
    const double s0 = (STEP == 1 || STEP == 2 || two) ? block_sum(a0, lds, kWideBlock) : 0.0;
    const double s1 = two ? block_sum(a1, lds, kWideBlock) : 0.0;
    const double s2 = STEP == 3 ? block_sum(a2, lds, kWideBlock) : 0.0;
    if (threadIdx.x != 0) return;
    if (STEP == 6) {
        S.rho = 1.0;
        S.omega = 1.0;
        S.alpha = 0.0;
        S.bl[kBlRhoNext] = S.rr;
        return;
    }
    if (STEP == 0 || STEP == 1) {
        double rho0 = S.rho;
        if (STEP == 0) rho0 = -S.omega * rho0;
        const double rho1 = STEP == 0 ? S.bl[kBlRhoNext] : s0;
        if (rho0 == 0.0 || rho1 == 0.0) {
            S.done = kBreakdown;
            return;
        }
        S.beta = S.alpha * rho1 / rho0;
        S.rho = rho1;
        return;
    }
    if (STEP == 2) {
        if (s0 == 0.0) {
            S.done = kBreakdown;
            return;
        }
        S.alpha = S.rho / s0;
        return;
    }
    if (STEP == 3) {
        // s0 = (r1, r1), s1 = (r0, r1), s2 = (r2, r1)
        const double sig = s0;
        if (sig == 0.0) {
            S.iter = S.iter + 1;
            S.done = kBreakdown;
            return;
        }
        S.bl[kBlSigma1] = sig;
        S.bl[kBlG1p] = s1 / sig;
        S.bl[kBlTau] = s2 / sig;
        return;
    }
    if (STEP == 4) {
        if (s0 == 0.0) {
            S.iter = S.iter + 1;
            S.done = kBreakdown;
            return;
        }
        const double g2p = s1 / s0;
        S.bl[kBlG2p] = g2p;
        S.bl[kBlG2] = g2p;
        S.omega = g2p;
        S.bl[kBlG1] = S.bl[kBlG1p] - S.bl[kBlTau] * g2p;
        return;
    }
    // STEP 5
    const double h = sqrt(s0 / S.bb);
    const int it = S.iter + 1;
    S.iter = it;
    S.rr = s0;
    S.relres = h;
    S.bl[kBlRhoNext] = s1;
    if (it < hist_stride) hist[(int64_t)sys * hist_stride + it] = h;
    if (!isfinite(h)) S.done = kNaN;
    else if (h <= rtol) S.done = kConverged;
    else if (it >= maxiter) S.done = kMaxIter;
    else if (S.omega == 0.0) S.done = kBreakdown;
}

// dst = src (used for r~ = r0 and zero-filled vectors)
static __global__ void __launch_bounds__(kBlock) k_copy(const DevTile *__restrict__ tiles, int32_t ntiles,
                                                        const double *__restrict__ src, double *__restrict__ dst) {
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    for_tile_rows(T, [&](int row) { dst[row] = src ? src[row] : 0.0; });
}

// y = 0 for systems with b = 0
static __global__ void k_zero_null_rhs(const DevTile *__restrict__ tiles, int32_t ntiles, double *__restrict__ y,
                                const SysState *__restrict__ st, const int32_t *__restrict__ sub_sys) {
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    if (st[sub_sys[T.sub]].bb != 0.0) return;
    for_tile_rows(T, [&](int row) { y[row] = 0.0; });
}

// ---------------------------------------------------------------------------
// V-cycle level kernels (VT = value type of the hierarchy, FT = type of the
// level's right-hand side: double on level 0, VT below)
// ---------------------------------------------------------------------------

// res = f - A (m o f)        (pre-smoothing from a zero guess + residual)
template <class VT, class FT, class MAT>
__global__ void __launch_bounds__(kBlock) k_pre_res(MAT A, const VT *__restrict__ m, const FT *__restrict__ f,
                                                    VT *__restrict__ res, const SysState *__restrict__ st,
                                                    const int32_t *__restrict__ sub_sys) {
    const int tile = tile_of_block(A.ntiles);
    if (tile >= A.ntiles) return;
    const DevTile T = A.tiles[tile];
    if (st && st[sub_sys[T.sub]].done) return;
    for_rows<VT>(A, tile, T, [&](int c) { return m[c] * (VT)f[c]; },
                 [&](int row, VT ax) { res[row] = (VT)f[row] - ax; });
}

// y = M x (restriction, or a plain product)
template <class VT, class MAT>
__global__ void __launch_bounds__(kBlock) k_spmv(MAT M, const VT *__restrict__ x, VT *__restrict__ y,
                                                 const SysState *__restrict__ st, const int32_t *__restrict__ sub_sys) {
    const int tile = tile_of_block(M.ntiles);
    if (tile >= M.ntiles) return;
    const DevTile T = M.tiles[tile];
    if (st && st[sub_sys[T.sub]].done) return;
    for_rows<VT>(M, tile, T, [&](int c) { return x[c]; }, [&](int row, VT v) { y[row] = v; });
}

// f_c = B f with B = R (I - A diag(m)): pre-smoothing from a zero guess,
// residual and restriction of one level in a single operator; stored row k
// of B is coarse row rowmap[k] (rows kept in a clustered order), or k
template <class VT, class FT, class MAT>
__global__ void __launch_bounds__(kBlock) k_restrict(MAT B, const FT *__restrict__ f, VT *__restrict__ fc,
                                                     const int32_t *__restrict__ rowmap,
                                                     const SysState *__restrict__ st,
                                                     const int32_t *__restrict__ sub_sys) {
    const int tile = tile_of_block(B.ntiles);
    if (tile >= B.ntiles) return;
    const DevTile T = B.tiles[tile];
    if (st && st[sub_sys[T.sub]].done) return;
    for_rows<VT>(B, tile, T, [&](int c) { return (VT)f[c]; },
                 [&](int row, VT v) { fc[rowmap ? rowmap[row] : row] = v; });
}

// Partial sums of the segments of a column-tiled operator (see SegM); NT
// threads per block, one column tile per block, wavefront w taking slices
// w, w + NT/64, ...
template <class VT, class FT, int NT>
__global__ void __launch_bounds__(NT) k_seg_partial(SegM<VT> M, const FT *__restrict__ f, VT *__restrict__ part,
                                                    const SysState *__restrict__ st,
                                                    const int32_t *__restrict__ sub_sys) {
    const int tile = tile_of_block(M.ntiles);
    if (tile >= M.ntiles) return;
    const DevTile T = M.tiles[tile];
    if (st && st[sub_sys[T.sub]].done) return;
    const VT *lds = stage_window<VT, NT>(T.row0, T.nrows, [&](int c) { return (VT)f[c]; });
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int s1 = M.slices[tile + 1];
    for (int sl = M.slices[tile] + w; sl < s1; sl += NT / 64) {
        const VT acc = sell_dot<VT, VT>(M.col16, 0, M.val, M.soff[sl] + lane, M.sw[sl], [&](int c) { return lds[c]; });
        const int q = M.slot[(int64_t)sl * 64 + lane];
        if (q >= 0) part[q] = acc;
    }
}

// y[rowmap ? rowmap[row] : row] = sum of the row's partials part[pp[row] ..
// pp[row + 1]) in column-tile order; `rt` tiles the rows.
template <class VT>
__global__ void __launch_bounds__(kBlock) k_seg_combine(const DevTile *__restrict__ rt, int32_t nrt,
                                                        const int32_t *__restrict__ pp, const VT *__restrict__ part,
                                                        VT *__restrict__ y, const int32_t *__restrict__ rowmap,
                                                        const SysState *__restrict__ st,
                                                        const int32_t *__restrict__ sub_sys) {
    const int tile = tile_of_block(nrt);
    if (tile >= nrt) return;
    const DevTile T = rt[tile];
    if (st && st[sub_sys[T.sub]].done) return;
    for_tile_rows(T, [&](int row) {
        VT acc = 0;
        for (int q = pp[row]; q < pp[row + 1]; ++q) acc += part[q];
        y[rowmap ? rowmap[row] : row] = acc;
    });
}

// z = m o f + P xc   (pre-smoothed iterate plus the coarse correction)
template <class VT, class FT, class MAT>
__global__ void __launch_bounds__(kBlock) k_prolong(MAT P, const VT *__restrict__ m, const FT *__restrict__ f,
                                                    const VT *__restrict__ xc, VT *__restrict__ z,
                                                    const SysState *__restrict__ st, const int32_t *__restrict__ sub_sys) {
    const int tile = tile_of_block(P.ntiles);
    if (tile >= P.ntiles) return;
    const DevTile T = P.tiles[tile];
    if (st && st[sub_sys[T.sub]].done) return;
    for_rows<VT>(P, tile, T, [&](int c) { return xc[c]; },
                 [&](int row, VT px) { z[row] = m[row] * (VT)f[row] + px; });
}

// Kernels of V-cycles with other than one pre-smoothing sweep: the first
// sweep from the zero guess x = m o f, the residual of an explicit iterate
// res = f - A x, and the coarse correction of an explicit iterate z = x + P xc
// (x == nullptr: z = P xc, no pre-smoothing).
template <class VT, class FT>
__global__ void __launch_bounds__(kBlock) k_vscale(int64_t n, const VT *__restrict__ m, const FT *__restrict__ f,
                                                   VT *__restrict__ x) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        x[i] = m[i] * (VT)f[i];
}

template <class VT, class FT, class MAT>
__global__ void __launch_bounds__(kBlock) k_resid(MAT A, const FT *__restrict__ f, const VT *__restrict__ x,
                                                  VT *__restrict__ res, const SysState *__restrict__ st,
                                                  const int32_t *__restrict__ sub_sys) {
    const int tile = tile_of_block(A.ntiles);
    if (tile >= A.ntiles) return;
    const DevTile T = A.tiles[tile];
    if (st && st[sub_sys[T.sub]].done) return;
    for_rows<VT>(A, tile, T, [&](int c) { return x[c]; }, [&](int row, VT ax) { res[row] = (VT)f[row] - ax; });
}

template <class VT, class MAT>
__global__ void __launch_bounds__(kBlock) k_prolong_add(MAT P, const VT *__restrict__ x, const VT *__restrict__ xc,
                                                        VT *__restrict__ z, const SysState *__restrict__ st,
                                                        const int32_t *__restrict__ sub_sys) {
    const int tile = tile_of_block(P.ntiles);
    if (tile >= P.ntiles) return;
    const DevTile T = P.tiles[tile];
    if (st && st[sub_sys[T.sub]].done) return;
    for_rows<VT>(P, tile, T, [&](int c) { return xc[c]; },
                 [&](int row, VT px) { z[row] = (x ? x[row] : (VT)0) + px; });
}

// x = z + m o (f - A z)   (post-smoothing); DOT: partial (f, x) per tile
template <class VT, class FT, class OT, bool DOT, class MAT>
__global__ void __launch_bounds__(kBlock) k_post(MAT A, const VT *__restrict__ m, const FT *__restrict__ f,
                                                 const VT *__restrict__ z, OT *__restrict__ x,
                                                 double *__restrict__ part, const SysState *__restrict__ st,
                                                 const int32_t *__restrict__ sub_sys) {
    __shared__ double lds[4];
    const int tile = tile_of_block(A.ntiles);
    if (tile >= A.ntiles) return;
    const DevTile T = A.tiles[tile];
    if (st && st[sub_sys[T.sub]].done) return;
    double d = 0.0;
    for_rows<VT>(A, tile, T, [&](int c) { return z[c]; }, [&](int row, VT az) {
        const VT fr = (VT)f[row];
        const VT xv = z[row] + m[row] * (fr - az);
        x[row] = (OT)xv;
        if (DOT) d += (double)f[row] * (double)(OT)xv;
    });
    if (!DOT) return;
    const double s = block_sum(d, lds, kBlock);
    if (threadIdx.x == 0) part[T.slot] = s;
}

// Dense direct solve on the coarsest level of each listed subdomain:
// x = A_L^{-1} f with the inverse stored row-major, one wavefront per row
// (lanes stride the columns), 4 rows per block.  DOT: partial (f, x) per
// block, summed per subdomain by the (r, s) reduction.
struct CoarseEntry {
    int32_t sub, n;
    int64_t off;      // first row in the level's packed vectors
    int64_t inv_off;  // offset of the row-major inverse (n rows of ld entries)
    int32_t ld;       // row stride: n rounded up to a 16-byte multiple, zero padded
    int32_t pad;
};

constexpr int kCoarseRowsPerWave = 4;
constexpr int kCoarseRows = kCoarseRowsPerWave * (kBlock / kWave);   // rows per block

struct CoarseJob {
    int32_t entry;    // index into the CoarseEntry table
    int32_t row0;     // first of the block's kCoarseRows rows
};

template <class VT>
struct Vec16;   // 16-byte vector of VT
template <>
struct Vec16<float> {
    typedef float type __attribute__((ext_vector_type(4)));
    static constexpr int N = 4;
};
template <>
struct Vec16<double> {
    typedef double type __attribute__((ext_vector_type(2)));
    static constexpr int N = 2;
};

// x = A_c^{-1} f on the coarsest level of every listed subdomain: each
// wavefront takes kCoarseRowsPerWave rows of the inverse and reads them as
// 16-byte vectors (the lanes of a wavefront cover 1 KB of a row per step),
// the right-hand side chunk being shared by the rows; DOT leaves the
// partial (f, x) of the block's rows.
template <class VT, class FT, class OT, bool DOT>
__global__ void __launch_bounds__(kBlock) k_coarse(const CoarseJob *__restrict__ jobs, const CoarseEntry *__restrict__ ent,
                                                   const VT *__restrict__ inv, const FT *__restrict__ f,
                                                   OT *__restrict__ x, double *__restrict__ part_job,
                                                   const SysState *__restrict__ st, const int32_t *__restrict__ sub_sys) {
    using V = typename Vec16<VT>::type;
    constexpr int NV = Vec16<VT>::N;
    constexpr int R = kCoarseRowsPerWave;
    __shared__ double red[4];
    const CoarseJob J = jobs[blockIdx.x];
    const CoarseEntry E = ent[J.entry];
    if (st[sub_sys[E.sub]].done) return;
    const int n = E.n, ld = E.ld, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i0 = J.row0 + w * R;
    const FT *fl = f + E.off;
    const V *rows[R];
#pragma unroll
    for (int r = 0; r < R; ++r)
        rows[r] = reinterpret_cast<const V *>(inv + E.inv_off + (int64_t)min(i0 + r, n - 1) * ld);
    VT acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0;
    for (int j = lane * NV; j < n; j += 64 * NV) {
        VT fv[NV];
#pragma unroll
        for (int u = 0; u < NV; ++u) fv[u] = j + u < n ? (VT)fl[j + u] : (VT)0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const V a = __builtin_nontemporal_load(rows[r] + j / NV);
#pragma unroll
            for (int u = 0; u < NV; ++u) acc[r] += a[u] * fv[u];
        }
    }
    double d = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        VT a = acc[r];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, kWave);
        const int i = i0 + r;
        if (lane == 0 && i < n) {
            x[E.off + i] = (OT)a;
            if (DOT) d += (double)fl[i] * (double)(OT)a;
        }
    }
    if (!DOT) return;
    if (lane == 0) red[w] = d;
    __syncthreads();
    if (threadIdx.x == 0) part_job[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// s = r (no preconditioner) with partial (r, s)
static __global__ void __launch_bounds__(kBlock) k_identity(const DevTile *__restrict__ tiles, int32_t ntiles,
                                                     const double *__restrict__ r, double *__restrict__ s,
                                                     double *__restrict__ part, const SysState *__restrict__ st,
                                                     const int32_t *__restrict__ sub_sys) {
    __shared__ double lds[4];
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    if (st[sub_sys[T.sub]].done) return;
    double d = 0.0;
    for_tile_rows(T, [&](int row) {
        const double v = r[row];
        s[row] = v;
        d += v * v;
    });
    const double sum = block_sum(d, lds, kBlock);
    if (threadIdx.x == 0) part[T.slot] = sum;
}

// Partials Z^T v per tile (for a stand-alone projection).
static __global__ void __launch_bounds__(kBlock) k_zt_partial(const DevTile *__restrict__ tiles, int32_t ntiles,
                                                       const double *__restrict__ v, const double *__restrict__ Z,
                                                       int ndv, double *__restrict__ part, int32_t nslots) {
    __shared__ double lds[4];
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    for (int k = 0; k < ndv; ++k) {
        double a = 0.0;
        for_tile_rows(T, [&](int row) { a += Z[(int64_t)row * ndv + k] * v[row]; });
        const double sum = block_sum(a, lds, kBlock);
        if (threadIdx.x == 0) part[(int64_t)(k + 1) * nslots + T.slot] = sum;
    }
}

// ---------------------------------------------------------------------------
// permutation
// ---------------------------------------------------------------------------

static __global__ void k_gather(int64_t n, const int64_t *__restrict__ perm, const double *__restrict__ src,
                         double *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[perm[i]];
}

static __global__ void k_scatter(int64_t n, const int64_t *__restrict__ perm, const double *__restrict__ src,
                          double *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[perm[i]] = src[i];
}

// ---------------------------------------------------------------------------
// batched Gauss-Jordan inversion with partial pivoting (FP64), used for E of
// every system and for the coarsest-level blocks.  Matrix b is stored
// augmented [A | I] (n x 2n, row-major) at aug + aug_off[b].
// ---------------------------------------------------------------------------

struct InvJob {
    int32_t n;
    int32_t singular;   // set by the pivot kernel
    int64_t aug_off;
};

// Step k, part 1 (one block per matrix): pivot search, row swap, pivot row
// scaling and a copy of column k for the elimination.
static __global__ void __launch_bounds__(kBlock) k_gj_pivot(InvJob *__restrict__ jobs, double *__restrict__ aug,
                                                     double *__restrict__ colk, const int64_t *__restrict__ col_off,
                                                     int k) {
    __shared__ double bv[kBlock];
    __shared__ int bi[kBlock];
    InvJob &J = jobs[blockIdx.x];
    const int n = J.n;
    if (k >= n || J.singular) return;
    double *A = aug + J.aug_off;
    const int w2 = 2 * n;
    double best = -1.0;
    int bidx = n;
    for (int i = k + threadIdx.x; i < n; i += kBlock) {
        const double v = fabs(A[(int64_t)i * w2 + k]);
        if (v > best) {
            best = v;
            bidx = i;
        }
    }
    bv[threadIdx.x] = best;
    bi[threadIdx.x] = bidx;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double o = bv[threadIdx.x + s];
            const int oi = bi[threadIdx.x + s];
            if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
                bv[threadIdx.x] = o;
                bi[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    const int p = bi[0];
    if (!(bv[0] > 0.0) || p >= n) {
        if (threadIdx.x == 0) J.singular = 1;
        return;
    }
    if (p != k)
        for (int j = threadIdx.x; j < w2; j += kBlock) {
            const double a = A[(int64_t)k * w2 + j];
            A[(int64_t)k * w2 + j] = A[(int64_t)p * w2 + j];
            A[(int64_t)p * w2 + j] = a;
        }
    __syncthreads();
    const double inv = 1.0 / A[(int64_t)k * w2 + k];
    __syncthreads();
    for (int j = threadIdx.x; j < w2; j += kBlock) A[(int64_t)k * w2 + j] *= inv;
    double *ck = colk + col_off[blockIdx.x];
    for (int i = threadIdx.x; i < n; i += kBlock) ck[i] = (i == k) ? 0.0 : A[(int64_t)i * w2 + k];
}

// Step k, part 2: row_i -= a_ik row_k for every i != k; grid (row blocks, matrices)
static __global__ void __launch_bounds__(kBlock) k_gj_eliminate(const InvJob *__restrict__ jobs, double *__restrict__ aug,
                                                         const double *__restrict__ colk,
                                                         const int64_t *__restrict__ col_off, int k) {
    const InvJob J = jobs[blockIdx.y];
    const int n = J.n;
    if (k >= n || J.singular) return;
    double *A = aug + J.aug_off;
    const double *ck = colk + col_off[blockIdx.y];
    const int w2 = 2 * n;
    const int64_t total = (int64_t)n * w2;
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < total; e += (int64_t)gridDim.x * kBlock) {
        const int i = (int)(e / w2), j = (int)(e % w2);
        if (i == k || j < k) continue;
        const double f = ck[i];
        if (f != 0.0) A[e] = (j == k) ? 0.0 : A[e] - f * A[(int64_t)k * w2 + j];
    }
}

// Copy the inverse (right half) out in type VT, transposed or row-major.
template <class VT>
__global__ void k_gj_extract(const InvJob *__restrict__ jobs, const double *__restrict__ aug,
                             const int64_t *__restrict__ out_off, const int32_t *__restrict__ out_ld,
                             VT *__restrict__ out) {
    const InvJob J = jobs[blockIdx.y];
    const int n = J.n, ld = out_ld[blockIdx.y];
    const double *A = aug + J.aug_off;
    VT *O = out + out_off[blockIdx.y];
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < (int64_t)n * ld; e += (int64_t)gridDim.x * kBlock) {
        const int i = (int)(e / ld), j = (int)(e % ld);
        O[e] = j < n ? (VT)A[(int64_t)i * 2 * n + n + j] : (VT)0;
    }
}

}  // namespace dfamg
