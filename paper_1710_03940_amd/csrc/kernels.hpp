// CDNA4 (gfx950) kernels of the deflated block-AMG Krylov solve.
//
// Layout conventions
//   * every row-parallel kernel works on a list of row tiles; a tile lies
//     inside one subdomain (hence one system), so per-tile partial sums are
//     segmented by construction and the reductions are deterministic
//     (fixed tile order, fixed wavefront/LDS reduction tree, no atomics);
//   * block b is mapped to tile (b % 8) * per + b / 8 so that each of the 8
//     XCDs (workgroups are dispatched round-robin over them) walks a
//     contiguous range of tiles and its L2 sees the neighbouring rows;
//   * sparse matrices are sliced ELLPACK with 64-row slices (one wavefront per
//     slice, one row per lane, column-major inside the slice) or CSR with
//     several lanes per row;
//   * Krylov scalars live on the device (SysState, one per system) and every
//     in-loop kernel returns early once its system has stopped, so a fixed
//     sequence of launches (or a captured graph) can run past convergence.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dfamg {

constexpr int kWave = 64;
constexpr int kBlock = 256;          // 4 wavefronts
constexpr int kReduceBlock = 1024;   // one block per system for reductions

struct DevTile {
    int32_t row0, nrows, sub, slot;
};

// Per-system Krylov state.
struct SysState {
    double rho, alpha, beta, omega;  // CG / BiCGStab scalars
    double pq;                       // (p, A p) or (r~, v)
    double bb;                       // ||b||^2
    double rr;                       // ||r||^2
    double relres;                   // ||r|| / ||b|| of the last test
    double tt, ts;                   // BiCGStab (t,t), (t,s)
    int32_t iter;
    int32_t done;                    // 0 running, 1 converged, 2 maxiter, 3 nan, 4 breakdown
    int32_t half;                    // BiCGStab: stopped on the half step
    int32_t pad;
};

enum { kRunning = 0, kConverged = 1, kMaxIter = 2, kNaN = 3, kBreakdown = 4 };

template <class VT>
struct SellView {
    const DevTile *tiles;
    const int64_t *soff;
    const int32_t *sw;
    const int32_t *col;
    const VT *val;
    int32_t ntiles;
};

template <class VT>
struct CsrView {
    const DevTile *tiles;
    const int32_t *ptr;
    const int32_t *col;
    const VT *val;
    int32_t ntiles;
    int32_t lanes;
};

__device__ __forceinline__ int tile_of_block(int ntiles) {
    const int per = (ntiles + 7) >> 3;
    return (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
}

inline int grid_for_tiles(int ntiles) { return ((ntiles + 7) >> 3) * 8; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Sum over a 256-thread block; the result is valid in thread 0.
__device__ __forceinline__ double block_sum256(double v, double *lds4) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) lds4[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = ((lds4[0] + lds4[1]) + lds4[2]) + lds4[3];
    __syncthreads();
    return r;
}

// Sum over a block of `nthreads` (multiple of 64, <= 1024); result valid in
// every thread.
__device__ __forceinline__ double block_sum_all(double v, double *lds, int nthreads) {
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

// Row-dot of one SELL row: sum_j a_j * x(c_j).
template <class VT, class ACC, class XF>
__device__ __forceinline__ ACC sell_row(const SellView<VT> &M, int tile, int t, XF x) {
    const int k = t >> 6, lane = t & 63;
    const int64_t off = M.soff[tile * 4 + k] + lane;
    const int w = M.sw[tile * 4 + k];
    ACC acc = 0;
    int j = 0;
    for (; j + 1 < w; j += 2) {
        const int c0 = M.col[off + (int64_t)j * 64];
        const int c1 = M.col[off + (int64_t)(j + 1) * 64];
        const ACC a0 = (ACC)M.val[off + (int64_t)j * 64];
        const ACC a1 = (ACC)M.val[off + (int64_t)(j + 1) * 64];
        acc += a0 * x(c0);
        acc += a1 * x(c1);
    }
    if (j < w) acc += (ACC)M.val[off + (int64_t)j * 64] * x(M.col[off + (int64_t)j * 64]);
    return acc;
}

// ---------------------------------------------------------------------------
// outer operator and deflation
// ---------------------------------------------------------------------------

// MODE 0: q = A p, partials (p,q), Z^T q           (CG operator product)
// MODE 1: w = b - A y, partials (b,b), Z^T w       (initial / final residual)
// MODE 2: w = b - A x, partial (w,w)               (true residual)
// MODE 3: q = A p, partials Z^T q only             (BiCGStab operator product)
template <int NDV, int MODE>
__global__ void __launch_bounds__(kBlock) k_outer(SellView<double> A, const double *__restrict__ x,
                                                  const double *__restrict__ b, double *__restrict__ out,
                                                  const double *__restrict__ Z, double *__restrict__ part,
                                                  int32_t nslots, const SysState *__restrict__ st,
                                                  const int32_t *__restrict__ sub_sys) {
    __shared__ double lds[4 * (NDV + 1)];
    const int tile = tile_of_block(A.ntiles);
    if (tile >= A.ntiles) return;
    const DevTile T = A.tiles[tile];
    if ((MODE == 0 || MODE == 3) && st[sub_sys[T.sub]].done) return;
    const int t = threadIdx.x;
    const bool valid = t < T.nrows;
    const int row = T.row0 + t;
    double v = 0.0, d0 = 0.0;
    double zq[NDV > 0 ? NDV : 1];
    if (valid) {
        const double ax = sell_row<double, double>(A, tile, t, [&](int c) { return x[c]; });
        if (MODE == 0 || MODE == 3) {
            v = ax;
            if (MODE == 0) d0 = x[row] * v;
        } else {
            const double bi = b[row];
            v = bi - ax;
            d0 = MODE == 1 ? bi * bi : v * v;
        }
        out[row] = v;
    }
#pragma unroll
    for (int k = 0; k < NDV; ++k) zq[k] = (valid && MODE != 2) ? Z[(int64_t)row * NDV + k] * v : 0.0;
    // reduce d0 and zq over the block
    const int w = t >> 6;
    d0 = wave_sum(d0);
#pragma unroll
    for (int k = 0; k < NDV; ++k) zq[k] = wave_sum(zq[k]);
    if ((t & 63) == 0) {
        lds[w] = d0;
#pragma unroll
        for (int k = 0; k < NDV; ++k) lds[4 * (k + 1) + w] = zq[k];
    }
    __syncthreads();
    if (t <= NDV && (MODE != 2 || t == 0)) {
        const double s = ((lds[4 * t] + lds[4 * t + 1]) + lds[4 * t + 2]) + lds[4 * t + 3];
        part[(int64_t)t * nslots + T.slot] = s;
    }
}

// One block per system: t1 = Z^T v per subdomain (sum of tile partials),
// t2 = E^{-1} t1 (explicit FP64 inverse, stored transposed), then
//   MODE 0 (CG):   alpha = rho / ((p,q) - t1.t2)        [(p, P A p) for symmetric A]
//   MODE 1 (init): bb = sum of partial 0                 [(b,b)]
//   MODE 2 (plain projection / recovery): t2 only
//   MODE 3 (BiCGStab): t2 only, skipped when stopped
template <int NDV, int MODE>
__global__ void __launch_bounds__(kReduceBlock) k_project_reduce(
    const double *__restrict__ part, int32_t nslots, const int32_t *__restrict__ sys_tile_off,
    const int32_t *__restrict__ sub_tile_off, const int32_t *__restrict__ sys_sub_off,
    const double *__restrict__ EinvT, const int64_t *__restrict__ sys_E_off,
    double *__restrict__ t2, SysState *__restrict__ st) {
    extern __shared__ double sh[];
    double *t1 = sh;                 // m values
    double *red = sh + 4096;         // 16 wave partials
    const int sys = blockIdx.x;
    SysState &S = st[sys];
    if ((MODE == 0 || MODE == 3) && S.done) return;
    const int s0 = sys_sub_off[sys], s1 = sys_sub_off[sys + 1];
    const int m = (s1 - s0) * NDV;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int nw = kReduceBlock / 64;
    // t1 per subdomain: one wavefront per (subdomain, vector)
    for (int item = w; item < (s1 - s0) * NDV; item += nw) {
        const int s = s0 + item / (NDV > 0 ? NDV : 1), k = item % (NDV > 0 ? NDV : 1);
        double a = 0.0;
        for (int tl = sub_tile_off[s] + lane; tl < sub_tile_off[s + 1]; tl += 64)
            a += part[(int64_t)(k + 1) * nslots + tl];
        a = wave_sum(a);
        if (lane == 0) t1[item] = a;
    }
    double d0 = 0.0;
    if (MODE == 0 || MODE == 1)
        for (int tl = sys_tile_off[sys] + t; tl < sys_tile_off[sys + 1]; tl += kReduceBlock) d0 += part[tl];
    __syncthreads();
    const double D0 = block_sum_all(d0, red, kReduceBlock);
    // t2 = E^{-1} t1
    const double *Ei = EinvT + sys_E_off[sys];
    double tt = 0.0;
    for (int i = t; i < m; i += kReduceBlock) {
        double a = 0.0;
        for (int j = 0; j < m; ++j) a += Ei[(int64_t)j * m + i] * t1[j];
        t2[(int64_t)s0 * NDV + i] = a;
        tt += a * t1[i];
    }
    const double T12 = block_sum_all(tt, red, kReduceBlock);
    if (t == 0) {
        if (MODE == 0) {
            S.pq = D0 - T12;
            S.alpha = S.rho / S.pq;
        } else if (MODE == 1) {
            S.bb = D0;
        }
    }
}

// MODE 0 (CG): w = q - AZ t2; y += alpha p; r -= alpha w; partial (r,r)
// MODE 1 (init): r = w - AZ t2; partial (r,r)
// MODE 2 (project only): out = v - AZ t2
template <int NDV, int MODE>
__global__ void __launch_bounds__(kBlock) k_update(
    const DevTile *__restrict__ tiles, int32_t ntiles, const double *__restrict__ p,
    const double *__restrict__ q, double *__restrict__ y, double *__restrict__ r,
    const double *__restrict__ AZown, const int32_t *__restrict__ offp, const int32_t *__restrict__ offc,
    const double *__restrict__ offv, const double *__restrict__ t2, double *__restrict__ part,
    const SysState *__restrict__ st, const int32_t *__restrict__ sub_sys) {
    __shared__ double lds[4];
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    const SysState &S = st[sub_sys[T.sub]];
    if (MODE == 0 && S.done) return;
    const int t = threadIdx.x;
    double rr = 0.0;
    if (t < T.nrows) {
        const int row = T.row0 + t;
        double corr = 0.0;
#pragma unroll
        for (int k = 0; k < NDV; ++k) corr += AZown[(int64_t)row * NDV + k] * t2[(int64_t)T.sub * NDV + k];
        if (NDV > 0)
            for (int e = offp[row]; e < offp[row + 1]; ++e) corr += offv[e] * t2[offc[e]];
        const double wv = q[row] - corr;
        if (MODE == 0) {
            const double a = S.alpha;
            y[row] += a * p[row];
            const double rn = r[row] - a * wv;
            r[row] = rn;
            rr = rn * rn;
        } else if (MODE == 1) {
            r[row] = wv;
            rr = wv * wv;
        } else {
            r[row] = wv;
        }
    }
    if (MODE == 2) return;
    const double s = block_sum256(rr, lds);
    if (t == 0) part[T.slot] = s;
}

// x = y + Z t2 (solution recovery, x = y + Z lambda)
template <int NDV>
__global__ void __launch_bounds__(kBlock) k_expand(const DevTile *__restrict__ tiles, int32_t ntiles,
                                                   const double *__restrict__ y, const double *__restrict__ Z,
                                                   const double *__restrict__ t2, double *__restrict__ x) {
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    const int t = threadIdx.x;
    if (t >= T.nrows) return;
    const int row = T.row0 + t;
    double v = y[row];
#pragma unroll
    for (int k = 0; k < NDV; ++k) v += Z[(int64_t)row * NDV + k] * t2[(int64_t)T.sub * NDV + k];
    x[row] = v;
}

// Per-system sum of tile partials into a SysState field and the stopping test.
//   MODE 0 (CG loop): rr, iter++, history, stop test
//   MODE 1 (initial residual): rr, iter = 0, history[0], stop test
//   MODE 2 (true residual): relres = sqrt(sum / bb) written to out[sys]
template <int MODE>
__global__ void __launch_bounds__(kBlock) k_residual_test(const double *__restrict__ part,
                                                          const int32_t *__restrict__ sys_tile_off,
                                                          SysState *__restrict__ st, double *__restrict__ hist,
                                                          int32_t hist_stride, double rtol, int32_t maxiter,
                                                          double *__restrict__ out) {
    __shared__ double lds[4];
    const int sys = blockIdx.x;
    SysState &S = st[sys];
    if (MODE == 0 && S.done) return;
    double a = 0.0;
    for (int tl = sys_tile_off[sys] + threadIdx.x; tl < sys_tile_off[sys + 1]; tl += kBlock) a += part[tl];
    const double rr = block_sum256(a, lds);
    if (threadIdx.x != 0) return;
    if (MODE == 2) {
        out[sys] = S.bb > 0.0 ? sqrt(rr / S.bb) : 0.0;
        return;
    }
    S.rr = rr;
    const double h = S.bb > 0.0 ? sqrt(rr / S.bb) : 0.0;
    S.relres = h;
    if (MODE == 1) {
        S.iter = 0;
        S.done = kRunning;
        S.half = 0;
        hist[(int64_t)sys * hist_stride] = h;
        if (S.bb == 0.0 || h <= rtol) S.done = kConverged;
        else if (!isfinite(h)) S.done = kNaN;
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
// (and the per-subdomain partials of level-0 direct solves); CG beta.
//   MODE 0: beta = rho'/rho, rho = rho'      MODE 1 (init): rho = rho', beta = 0
template <int MODE>
__global__ void __launch_bounds__(kBlock) k_rho(const double *__restrict__ part, const int32_t *__restrict__ sys_tile_off,
                                                const double *__restrict__ part_sub,
                                                const int32_t *__restrict__ sys_sub_off, SysState *__restrict__ st) {
    __shared__ double lds[4];
    const int sys = blockIdx.x;
    SysState &S = st[sys];
    if (S.done) return;
    double a = 0.0;
    for (int tl = sys_tile_off[sys] + threadIdx.x; tl < sys_tile_off[sys + 1]; tl += kBlock) a += part[tl];
    for (int s = sys_sub_off[sys] + threadIdx.x; s < sys_sub_off[sys + 1]; s += kBlock) a += part_sub[s];
    const double rs = block_sum256(a, lds);
    if (threadIdx.x == 0) {
        if (MODE == 0) {
            S.beta = rs / S.rho;
        } else {
            S.beta = 0.0;
        }
        S.rho = rs;
    }
}

// p = s + beta p
__global__ void __launch_bounds__(kBlock) k_cg_direction(const DevTile *__restrict__ tiles, int32_t ntiles,
                                                         const double *__restrict__ s, double *__restrict__ p,
                                                         const SysState *__restrict__ st,
                                                         const int32_t *__restrict__ sub_sys) {
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    const SysState &S = st[sub_sys[T.sub]];
    if (S.done) return;
    const int t = threadIdx.x;
    if (t >= T.nrows) return;
    const int row = T.row0 + t;
    p[row] = s[row] + S.beta * p[row];
}

// ---------------------------------------------------------------------------
// V-cycle level kernels (VT = value type of the hierarchy, FT = type of the
// level's right-hand side: double on level 0, VT below)
// ---------------------------------------------------------------------------

// res = f - A (m o f)        (pre-smoothing from a zero guess + residual)
template <class VT, class FT>
__global__ void __launch_bounds__(kBlock) k_pre_res(SellView<VT> A, const VT *__restrict__ m,
                                                    const FT *__restrict__ f, VT *__restrict__ res,
                                                    const SysState *__restrict__ st, const int32_t *__restrict__ sub_sys) {
    const int tile = tile_of_block(A.ntiles);
    if (tile >= A.ntiles) return;
    const DevTile T = A.tiles[tile];
    if (st[sub_sys[T.sub]].done) return;
    const int t = threadIdx.x;
    if (t >= T.nrows) return;
    const int row = T.row0 + t;
    const VT ax = sell_row<VT, VT>(A, tile, t, [&](int c) { return m[c] * (VT)f[c]; });
    res[row] = (VT)f[row] - ax;
}

// y = M x (restriction)
template <class VT>
__global__ void __launch_bounds__(kBlock) k_spmv(SellView<VT> M, const VT *__restrict__ x, VT *__restrict__ y,
                                                 const SysState *__restrict__ st, const int32_t *__restrict__ sub_sys) {
    const int tile = tile_of_block(M.ntiles);
    if (tile >= M.ntiles) return;
    const DevTile T = M.tiles[tile];
    if (st[sub_sys[T.sub]].done) return;
    const int t = threadIdx.x;
    if (t >= T.nrows) return;
    y[T.row0 + t] = sell_row<VT, VT>(M, tile, t, [&](int c) { return x[c]; });
}

// z = m o f + P xc   (pre-smoothed iterate plus the coarse correction)
template <class VT, class FT>
__global__ void __launch_bounds__(kBlock) k_prolong(SellView<VT> P, const VT *__restrict__ m,
                                                    const FT *__restrict__ f, const VT *__restrict__ xc,
                                                    VT *__restrict__ z, const SysState *__restrict__ st,
                                                    const int32_t *__restrict__ sub_sys) {
    const int tile = tile_of_block(P.ntiles);
    if (tile >= P.ntiles) return;
    const DevTile T = P.tiles[tile];
    if (st[sub_sys[T.sub]].done) return;
    const int t = threadIdx.x;
    if (t >= T.nrows) return;
    const int row = T.row0 + t;
    z[row] = m[row] * (VT)f[row] + sell_row<VT, VT>(P, tile, t, [&](int c) { return xc[c]; });
}

// x = z + m o (f - A z)   (post-smoothing); DOT: partial (f, x) per tile
template <class VT, class FT, class OT, bool DOT>
__global__ void __launch_bounds__(kBlock) k_post(SellView<VT> A, const VT *__restrict__ m,
                                                 const FT *__restrict__ f, const VT *__restrict__ z,
                                                 OT *__restrict__ x, double *__restrict__ part,
                                                 const SysState *__restrict__ st, const int32_t *__restrict__ sub_sys) {
    __shared__ double lds[4];
    const int tile = tile_of_block(A.ntiles);
    if (tile >= A.ntiles) return;
    const DevTile T = A.tiles[tile];
    if (st[sub_sys[T.sub]].done) return;
    const int t = threadIdx.x;
    double d = 0.0;
    if (t < T.nrows) {
        const int row = T.row0 + t;
        const VT az = sell_row<VT, VT>(A, tile, t, [&](int c) { return z[c]; });
        const VT fr = (VT)f[row];
        const VT xv = z[row] + m[row] * (fr - az);
        x[row] = (OT)xv;
        if (DOT) d = (double)f[row] * (double)(OT)xv;
    }
    if (!DOT) return;
    const double s = block_sum256(d, lds);
    if (t == 0) part[T.slot] = s;
}

// Dense direct solve on the coarsest level of each listed subdomain:
// x = A_L^{-1} f with the inverse stored transposed.  DOT: partial (f, x)
// per subdomain (level-0 coarsest subdomains only).
struct CoarseEntry {
    int32_t sub, n;
    int64_t off;      // first row in the level's packed vectors
    int64_t inv_off;  // offset of the n x n transposed inverse
};

template <class VT, class FT, class OT, bool DOT>
__global__ void __launch_bounds__(kBlock) k_coarse(const CoarseEntry *__restrict__ ent, const VT *__restrict__ invT,
                                                   const FT *__restrict__ f, OT *__restrict__ x,
                                                   double *__restrict__ part_sub, const SysState *__restrict__ st,
                                                   const int32_t *__restrict__ sub_sys) {
    extern __shared__ char smem[];
    VT *fl = reinterpret_cast<VT *>(smem);
    __shared__ double lds[4];
    const CoarseEntry E = ent[blockIdx.x];
    if (st[sub_sys[E.sub]].done) return;
    const int n = E.n;
    for (int i = threadIdx.x; i < n; i += kBlock) fl[i] = (VT)f[E.off + i];
    __syncthreads();
    const VT *Ai = invT + E.inv_off;
    double d = 0.0;
    for (int i = threadIdx.x; i < n; i += kBlock) {
        VT a = 0;
        for (int j = 0; j < n; ++j) a += Ai[(int64_t)j * n + i] * fl[j];
        x[E.off + i] = (OT)a;
        if (DOT) d += (double)f[E.off + i] * (double)(OT)a;
    }
    if (!DOT) return;
    const double s = block_sum256(d, lds);
    if (threadIdx.x == 0) part_sub[E.sub] = s;
}

// s = r (no preconditioner) with partial (r, s)
__global__ void __launch_bounds__(kBlock) k_identity(const DevTile *__restrict__ tiles, int32_t ntiles,
                                                     const double *__restrict__ r, double *__restrict__ s,
                                                     double *__restrict__ part, const SysState *__restrict__ st,
                                                     const int32_t *__restrict__ sub_sys) {
    __shared__ double lds[4];
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    if (st[sub_sys[T.sub]].done) return;
    const int t = threadIdx.x;
    double d = 0.0;
    if (t < T.nrows) {
        const double v = r[T.row0 + t];
        s[T.row0 + t] = v;
        d = v * v;
    }
    const double sum = block_sum256(d, lds);
    if (t == 0) part[T.slot] = sum;
}

// ---------------------------------------------------------------------------
// permutation
// ---------------------------------------------------------------------------

__global__ void k_gather(int64_t n, const int64_t *__restrict__ perm, const double *__restrict__ src,
                         double *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[perm[i]];
}

__global__ void k_scatter(int64_t n, const int64_t *__restrict__ perm, const double *__restrict__ src,
                          double *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[perm[i]] = src[i];
}

__global__ void k_fill(int64_t n, double v, double *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = v;
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
__global__ void __launch_bounds__(kBlock) k_gj_pivot(InvJob *__restrict__ jobs, double *__restrict__ aug,
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
__global__ void __launch_bounds__(kBlock) k_gj_eliminate(const InvJob *__restrict__ jobs, double *__restrict__ aug,
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
        if (f != 0.0) A[e] -= f * A[(int64_t)k * w2 + j];
    }
}

// Copy the inverse (right half) out, transposed, in type VT.
template <class VT>
__global__ void k_gj_extract(const InvJob *__restrict__ jobs, const double *__restrict__ aug,
                             const int64_t *__restrict__ out_off, VT *__restrict__ outT) {
    const InvJob J = jobs[blockIdx.y];
    const int n = J.n;
    const double *A = aug + J.aug_off;
    VT *O = outT + out_off[blockIdx.y];
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < (int64_t)n * n; e += (int64_t)gridDim.x * kBlock) {
        const int i = (int)(e / n), j = (int)(e % n);
        O[(int64_t)j * n + i] = (VT)A[(int64_t)i * 2 * n + n + j];
    }
}

}  // namespace dfamg
