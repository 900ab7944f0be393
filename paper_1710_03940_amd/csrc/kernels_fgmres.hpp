// Kernels of restarted flexible GMRES on A x = b, preconditioned by the
// deflation combined multiplicatively with the block AMG (section "On
// precision of the coarse system solution": with an inexact coarse solve the
// projector becomes part of a variable preconditioner of the original system,
// which needs a flexible Krylov method):
//
//   B(v) = Z t2 + M^{-1}(v - (AZ) t2),   t2 = E_hat Z^T v.
//
// One Arnoldi step j of a cycle, per system:
//   t1 = Z^T v_j (partials left by the kernel that wrote v_j), t2_j = E_hat t1
//   f = v_j - (AZ) t2_j                                  k_fg_rhs
//   s_j = M^{-1} f                                       V-cycle kernels
//   q = A s_j                                            k_outer
//   w = q + (AZ) t2_j = A z_j,  z_j = s_j + Z t2_j       k_fg_dots
//   two classical Gram-Schmidt passes against v_0..v_j   k_fg_dots, k_fg_sum, k_fg_axpy_dots,
//                                                        k_fg_axpy
//   h_{j+1,j} = ||w||, Givens rotation, residual test    k_fg_givens
// and at the end of a cycle
//   y = R^{-1} g (back substitution)                     k_fg_solve
//   x += sum_i y_i s_i + Z sum_i y_i t2_i                k_fg_update_x.
//
// The Arnoldi vectors are stored unnormalised (V_i = v_i / sc_i with
// sc_i = 1 / ||V_i|| kept per system), which saves a normalisation pass: every
// consumer multiplies by sc_i.  z_j is never formed: its two parts s_j and
// t2_j are kept, A z_j is formed as A s_j + (AZ) t2_j, and the final update
// expands Z sum_i y_i t2_i once per cycle.  Gram-Schmidt is classical with
// one full reorthogonalisation (two passes: dots, then one update of all
// vectors), equal in exact arithmetic to the modified Gram-Schmidt of the
// textbook algorithm and one grid-wide reduction per pass instead of one per
// vector.
#pragma once

#include "kernels.hpp"

namespace dfamg {

constexpr int kFgMax = 64;   // largest restart length

// Per-system FGMRES state (device).  H is the (restart+1) x restart upper
// Hessenberg matrix, column-major with leading dimension kFgMax + 1; after
// the rotations its leading k x k block is the triangular R.
struct FgState {
    double H[(kFgMax + 1) * kFgMax];
    double cs[kFgMax], sn[kFgMax];
    double g[kFgMax + 1];      // rotated right-hand side beta e_1
    double sc[kFgMax + 1];     // 1 / ||V_i||
    double coef[kFgMax + 1];   // Gram-Schmidt coefficients of the current pass (times sc_i)
    double y[kFgMax];          // least-squares solution of the cycle
    double yt[kFgMax];         // y_i sc_i: weights of the stored t2_i
    int32_t k;                 // Arnoldi steps of the current cycle
    int32_t pad[3];
};

// (AZ t2)_row: the own-subdomain AZ block (ndv contiguous values per row,
// read as two 16-byte loads when ndv = 4) plus the row's couplings to other
// subdomains, four independent gathers at a time
template <int NDV>
__device__ __forceinline__ double az_times_t2(int64_t row, const double *__restrict__ AZown, int ndv,
                                              const double *t2s, const int32_t *__restrict__ offp,
                                              const int32_t *__restrict__ offc, const double *__restrict__ offv,
                                              const double *__restrict__ t2) {
    double corr = 0.0;
    if (NDV == 4 && ndv == 4) {
        const f64x2 *az = reinterpret_cast<const f64x2 *>(AZown + row * 4);
        const f64x2 a01 = stream_load(az), a23 = stream_load(az + 1);
        corr = ((a01.x * t2s[0] + a01.y * t2s[1]) + a23.x * t2s[2]) + a23.y * t2s[3];
    } else {
#pragma unroll
        for (int k = 0; k < NDV; ++k)
            if (k < ndv) corr += stream_load(AZown + row * ndv + k) * t2s[k];
    }
    if (ndv > 0) {
        int e = offp[row];
        const int e1 = offp[row + 1];
        for (; e + 4 <= e1; e += 4) {
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
        for (; e < e1; ++e) corr += offv[e] * t2[offc[e]];
    }
    return corr;
}

// f = sc_j (V_j - (AZ) t2_j): the residual the coarse correction leaves,
// handed to the V-cycle
template <int NDV>
__global__ void __launch_bounds__(kBlock) k_fg_rhs(const DevTile *__restrict__ tiles, int32_t ntiles,
                                                   const double *__restrict__ Vj, const double *__restrict__ AZown,
                                                   int ndv_rt, const int32_t *__restrict__ offp,
                                                   const int32_t *__restrict__ offc, const double *__restrict__ offv,
                                                   const double *__restrict__ t2, const FgState *__restrict__ fg, int j,
                                                   double *__restrict__ f, const SysState *__restrict__ st,
                                                   const int32_t *__restrict__ sub_sys) {
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    const int sys = sub_sys[T.sub];
    if (st[sys].done) return;
    const double sc = fg[sys].sc[j];
    const int ndv = ndv_rt;
    double t2s[NDV > 0 ? NDV : 1];
#pragma unroll
    for (int k = 0; k < NDV; ++k) t2s[k] = k < ndv ? t2[(int64_t)T.sub * ndv + k] : 0.0;
    for_tile_rows(T, [&](int row) {
        const double vj = stream_load(Vj + row);
        const double corr = az_times_t2<NDV>(row, AZown, ndv, t2s, offp, offc, offv, t2);
        f[row] = sc * (vj - corr);
    });
}

// w = q + sc_j (AZ) t2_j (the product A z_j, stored) and its dots with
// V_0 .. V_{J-1}: one partial per tile and vector, part[i * nslots + slot].
// One row per thread (row tiles hold at most kBlock rows).
template <int NDV>
__global__ void __launch_bounds__(kBlock) k_fg_dots(
    const DevTile *__restrict__ tiles, int32_t ntiles, const double *__restrict__ q, double *__restrict__ w,
    const double *__restrict__ AZown, int ndv_rt, const int32_t *__restrict__ offp, const int32_t *__restrict__ offc,
    const double *__restrict__ offv, const double *__restrict__ t2, const double *__restrict__ V, int64_t ld, int J,
    const FgState *__restrict__ fg, int j, double *__restrict__ part, int32_t nslots,
    const SysState *__restrict__ st, const int32_t *__restrict__ sub_sys) {
    __shared__ double red[(kFgMax + 1) * 4];
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    const int sys = sub_sys[T.sub];
    if (st[sys].done) return;
    const int lr = threadIdx.x;
    const bool has = lr < T.nrows;
    const int64_t row = (int64_t)T.row0 + lr;
    double wv = 0.0;
    if (has) {
        const int ndv = ndv_rt;
        double t2s[NDV > 0 ? NDV : 1];
#pragma unroll
        for (int k = 0; k < NDV; ++k) t2s[k] = k < ndv ? t2[(int64_t)T.sub * ndv + k] : 0.0;
        const double qv = stream_load(q + row);
        const double corr = az_times_t2<NDV>(row, AZown, ndv, t2s, offp, offc, offv, t2);
        wv = qv + fg[sys].sc[j] * corr;
        w[row] = wv;
    }
    const int wave = threadIdx.x >> 6;
    for (int i = 0; i < J; ++i) {
        const double d = has ? wv * V[(int64_t)i * ld + row] : 0.0;
        const double s = wave_sum(d);
        if ((threadIdx.x & 63) == 0) red[i * 4 + wave] = s;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < J; i += kBlock)
        part[(int64_t)i * nslots + T.slot] = ((red[i * 4] + red[i * 4 + 1]) + red[i * 4 + 2]) + red[i * 4 + 3];
}

// Per-system sums of the J dot partials (block (i, sys) sums vector i in a
// fixed order); PASS 1 sets column j of H to h_i = sc_i (w, V_i), PASS 2
// adds the reorthogonalisation's h_i; both leave coef_i = h_i sc_i, the
// weight of the stored V_i in the update.
template <int PASS>
__global__ void __launch_bounds__(kWideBlock) k_fg_sum(const double *__restrict__ part, int32_t nslots,
                                                       const int32_t *__restrict__ sys_tile_off,
                                                       FgState *__restrict__ fg, int j,
                                                       const SysState *__restrict__ st) {
    __shared__ double lds[16];
    const int i = blockIdx.x, sys = blockIdx.y;
    if (st[sys].done) return;
    double a = 0.0;
    const double *p = part + (int64_t)i * nslots;
    for (int tl = sys_tile_off[sys] + threadIdx.x; tl < sys_tile_off[sys + 1]; tl += kWideBlock) a += p[tl];
    const double s = block_sum(a, lds, kWideBlock);
    if (threadIdx.x != 0) return;
    FgState &F = fg[sys];
    const double h = F.sc[i] * s;
    double &Hij = F.H[(int64_t)j * (kFgMax + 1) + i];
    Hij = PASS == 1 ? h : Hij + h;
    F.coef[i] = h * F.sc[i];
}

// Second Gram-Schmidt update: V_{j+1} = w - sum_i coef_i V_i, with the
// partials ||V_{j+1}||^2 (part row 0) and Z^T V_{j+1} (rows 1..ndv) for the
// next step.
template <int NDV>
__global__ void __launch_bounds__(kBlock) k_fg_axpy(const DevTile *__restrict__ tiles, int32_t ntiles,
                                                    const double *__restrict__ w, double *__restrict__ out,
                                                    const double *__restrict__ V, int64_t ld, int J,
                                                    const FgState *__restrict__ fg, const double *__restrict__ Z,
                                                    int ndv_rt, double *__restrict__ part, int32_t nslots,
                                                    const SysState *__restrict__ st,
                                                    const int32_t *__restrict__ sub_sys) {
    __shared__ double cf[kFgMax + 1];
    __shared__ double red[(kMaxNdv + 1) * 4];
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    const int sys = sub_sys[T.sub];
    if (st[sys].done) return;
    for (int i = threadIdx.x; i < J; i += kBlock) cf[i] = fg[sys].coef[i];
    __syncthreads();
    const int lr = threadIdx.x;
    const bool has = lr < T.nrows;
    const int64_t row = (int64_t)T.row0 + lr;
    double v = 0.0;
    if (has) {
        double a0 = w[row], a1 = 0.0;
        int i = 0;
        for (; i + 1 < J; i += 2) {
            a0 -= cf[i] * V[(int64_t)i * ld + row];
            a1 -= cf[i + 1] * V[(int64_t)(i + 1) * ld + row];
        }
        if (i < J) a0 -= cf[i] * V[(int64_t)i * ld + row];
        v = a0 + a1;
        out[row] = v;
    }
    const int ndv = ndv_rt;
    const int wave = threadIdx.x >> 6;
    const double s0 = wave_sum(v * v);
    if ((threadIdx.x & 63) == 0) red[wave] = s0;
#pragma unroll
    for (int k = 0; k < NDV; ++k) {
        if (k < ndv) {
            const double s = wave_sum(has ? Z[row * ndv + k] * v : 0.0);
            if ((threadIdx.x & 63) == 0) red[4 * (k + 1) + wave] = s;
        }
    }
    __syncthreads();
    if (threadIdx.x <= ndv)
        part[(int64_t)threadIdx.x * nslots + T.slot] =
            ((red[4 * threadIdx.x] + red[4 * threadIdx.x + 1]) + red[4 * threadIdx.x + 2]) + red[4 * threadIdx.x + 3];
}

// First Gram-Schmidt update fused with the dots of the second pass:
// w' = w - sum_i coef_i V_i (stored in place), then the partials (w', V_i).
// The second read of a row of V_i follows the first closely, so it is
// mostly served by the caches: the pass costs one read of the basis from HBM
// instead of two.
static __global__ void __launch_bounds__(kBlock) k_fg_axpy_dots(const DevTile *__restrict__ tiles, int32_t ntiles,
                                                                double *__restrict__ w, const double *__restrict__ V,
                                                                int64_t ld, int J, const FgState *__restrict__ fg,
                                                                double *__restrict__ part, int32_t nslots,
                                                                const SysState *__restrict__ st,
                                                                const int32_t *__restrict__ sub_sys) {
    __shared__ double cf[kFgMax + 1];
    __shared__ double red[(kFgMax + 1) * 4];
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    const int sys = sub_sys[T.sub];
    if (st[sys].done) return;
    for (int i = threadIdx.x; i < J; i += kBlock) cf[i] = fg[sys].coef[i];
    __syncthreads();
    const int lr = threadIdx.x;
    const bool has = lr < T.nrows;
    const int64_t row = (int64_t)T.row0 + lr;
    double v = 0.0;
    if (has) {
        double a0 = w[row], a1 = 0.0;
        int i = 0;
        for (; i + 1 < J; i += 2) {
            a0 -= cf[i] * V[(int64_t)i * ld + row];
            a1 -= cf[i + 1] * V[(int64_t)(i + 1) * ld + row];
        }
        if (i < J) a0 -= cf[i] * V[(int64_t)i * ld + row];
        v = a0 + a1;
        w[row] = v;
    }
    const int wave = threadIdx.x >> 6;
    for (int i = 0; i < J; ++i) {
        const double d = has ? v * V[(int64_t)i * ld + row] : 0.0;
        const double s = wave_sum(d);
        if ((threadIdx.x & 63) == 0) red[i * 4 + wave] = s;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < J; i += kBlock)
        part[(int64_t)i * nslots + T.slot] = ((red[i * 4] + red[i * 4 + 1]) + red[i * 4 + 2]) + red[i * 4 + 3];
}

// Partial ||v||^2 per tile (part row 0): the norm of a cycle's first vector.
template <bool CHECK_DONE>
__global__ void __launch_bounds__(kBlock) k_fg_norm(const DevTile *__restrict__ tiles, int32_t ntiles,
                                                    const double *__restrict__ v, double *__restrict__ part,
                                                    const SysState *__restrict__ st,
                                                    const int32_t *__restrict__ sub_sys) {
    __shared__ double lds[4];
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    if (CHECK_DONE && st[sub_sys[T.sub]].done) return;
    double d = 0.0;
    for_tile_rows(T, [&](int row) {
        const double a = v[row];
        d += a * a;
    });
    const double s = block_sum(d, lds, kBlock);
    if (threadIdx.x == 0) part[T.slot] = s;
}

// Start of a cycle from the partials of ||V_0||^2: beta = ||V_0||,
// g = beta e_1, sc_0 = 1 / beta, k = 0 (also for stopped systems, so that
// the end-of-cycle kernels leave them alone).
static __global__ void __launch_bounds__(kWideBlock) k_fg_restart(const double *__restrict__ part,
                                                                  const int32_t *__restrict__ sys_tile_off,
                                                                  FgState *__restrict__ fg,
                                                                  SysState *__restrict__ st) {
    __shared__ double lds[16];
    const int sys = blockIdx.x;
    SysState &S = st[sys];
    FgState &F = fg[sys];
    const bool run = S.done == kRunning;
    double a = 0.0;
    if (run)
        for (int tl = sys_tile_off[sys] + threadIdx.x; tl < sys_tile_off[sys + 1]; tl += kWideBlock) a += part[tl];
    const double bb = block_sum(a, lds, kWideBlock);
    for (int i = threadIdx.x; i <= kFgMax; i += kWideBlock) F.g[i] = 0.0;
    __syncthreads();
    if (threadIdx.x != 0) return;
    F.k = 0;
    if (!run) return;
    const double beta = sqrt(bb);
    if (beta == 0.0) {   // x is exact
        S.done = kConverged;
        return;
    }
    if (!isfinite(beta)) {
        S.done = kNaN;
        return;
    }
    F.g[0] = beta;
    F.sc[0] = 1.0 / beta;
}

// Arnoldi step j, second half, per system: h_{j+1,j} = ||V_{j+1}|| from the
// partials, the earlier rotations applied to column j, a new rotation that
// zeroes h_{j+1,j}, the residual estimate |g_{j+1}|, the iteration count,
// the history and the stopping test.  A zero diagonal after the rotations
// (singular Hessenberg matrix) is a breakdown: the step counts but its column
// is not used.  h_{j+1,j} = 0 gives |g_{j+1}| = 0 (an invariant Krylov
// space: converged).
static __global__ void __launch_bounds__(kWideBlock) k_fg_givens(const double *__restrict__ part,
                                                                 const int32_t *__restrict__ sys_tile_off,
                                                                 FgState *__restrict__ fg, SysState *__restrict__ st,
                                                                 double *__restrict__ hist, int32_t hist_stride,
                                                                 double rtol, int32_t maxiter, int j) {
    __shared__ double lds[16];
    const int sys = blockIdx.x;
    SysState &S = st[sys];
    if (S.done) return;
    double a = 0.0;
    for (int tl = sys_tile_off[sys] + threadIdx.x; tl < sys_tile_off[sys + 1]; tl += kWideBlock) a += part[tl];
    const double nn = block_sum(a, lds, kWideBlock);
    if (threadIdx.x != 0) return;
    FgState &F = fg[sys];
    double *h = F.H + (int64_t)j * (kFgMax + 1);
    const double hn = sqrt(nn);
    h[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
        const double x0 = h[i], x1 = h[i + 1];
        h[i] = F.cs[i] * x0 + F.sn[i] * x1;
        h[i + 1] = -F.sn[i] * x0 + F.cs[i] * x1;
    }
    const int it = S.iter + 1;
    S.iter = it;
    const double d = hypot(h[j], h[j + 1]);
    if (d == 0.0 || !isfinite(d)) {
        if (it < hist_stride) hist[(int64_t)sys * hist_stride + it] = S.relres;
        S.done = d == 0.0 ? kBreakdown : kNaN;
        F.k = j;
        return;
    }
    const double c = h[j] / d, s = h[j + 1] / d;
    F.cs[j] = c;
    F.sn[j] = s;
    h[j] = d;
    h[j + 1] = 0.0;
    const double gj = F.g[j];
    F.g[j + 1] = -s * gj;
    F.g[j] = c * gj;
    F.k = j + 1;
    F.sc[j + 1] = hn > 0.0 ? 1.0 / hn : 0.0;
    const double rel = fabs(F.g[j + 1]) / sqrt(S.bb);
    S.relres = rel;
    S.rr = F.g[j + 1] * F.g[j + 1];
    if (it < hist_stride) hist[(int64_t)sys * hist_stride + it] = rel;
    if (!isfinite(rel)) S.done = kNaN;
    else if (rel <= rtol || hn == 0.0) S.done = kConverged;
    else if (it >= maxiter) S.done = kMaxIter;
}

// End of a cycle: y = R^{-1} g over the k steps taken (back substitution by
// one thread per system), yt_i = y_i sc_i.  Runs for every system with
// k > 0, including those that stopped during the cycle.
static __global__ void k_fg_solve(FgState *__restrict__ fg, int nsys) {
    const int sys = blockIdx.x * blockDim.x + threadIdx.x;
    if (sys >= nsys) return;
    FgState &F = fg[sys];
    const int k = F.k;
    for (int i = k - 1; i >= 0; --i) {
        double a = F.g[i];
        for (int l = i + 1; l < k; ++l) a -= F.H[(int64_t)l * (kFgMax + 1) + i] * F.y[l];
        F.y[i] = a / F.H[(int64_t)i * (kFgMax + 1) + i];
        F.yt[i] = F.y[i] * F.sc[i];
    }
}

// x += sum_i y_i s_i + Z c with c = sum_i yt_i t2_i of the row's subdomain.
template <int NDV>
__global__ void __launch_bounds__(kBlock) k_fg_update_x(const DevTile *__restrict__ tiles, int32_t ntiles,
                                                        double *__restrict__ x, const double *__restrict__ S,
                                                        int64_t ld, const double *__restrict__ Z, int ndv_rt,
                                                        const double *__restrict__ t2h, int64_t mtot,
                                                        const FgState *__restrict__ fg,
                                                        const int32_t *__restrict__ sub_sys) {
    __shared__ double yv[kFgMax];
    __shared__ double cz[kMaxNdv];
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    const FgState &F = fg[sub_sys[T.sub]];
    const int k = F.k;
    if (k == 0) return;
    const int ndv = ndv_rt;
    for (int i = threadIdx.x; i < k; i += kBlock) yv[i] = F.y[i];
    if (threadIdx.x < ndv) {
        double c = 0.0;
        for (int i = 0; i < k; ++i) c += F.yt[i] * t2h[(int64_t)i * mtot + (int64_t)T.sub * ndv + threadIdx.x];
        cz[threadIdx.x] = c;
    }
    __syncthreads();
    for_tile_rows(T, [&](int row) {
        double a0 = x[row], a1 = 0.0;
        int i = 0;
        for (; i + 1 < k; i += 2) {
            a0 += yv[i] * S[(int64_t)i * ld + row];
            a1 += yv[i + 1] * S[(int64_t)(i + 1) * ld + row];
        }
        if (i < k) a0 += yv[i] * S[(int64_t)i * ld + row];
#pragma unroll
        for (int kk = 0; kk < NDV; ++kk)
            if (kk < ndv) a1 += Z[(int64_t)row * ndv + kk] * cz[kk];
        x[row] = a0 + a1;
    });
}

// t2 = E_hat t1 with E_hat = E^{-1} rounded to single precision, applied in
// single precision (the inexact coarse solve): one wavefront per row as in
// the FP64 GEMV.
template <bool CHECK_DONE>
__global__ void __launch_bounds__(kBlock) k_egemv32(const GemvJob *__restrict__ jobs, const float *__restrict__ Einv,
                                                    const double *__restrict__ t1, double *__restrict__ t2,
                                                    const SysState *__restrict__ st) {
    const GemvJob J = jobs[blockIdx.x];
    if (CHECK_DONE && st[J.sys].done) return;
    const int m = J.m;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const double *tl = t1 + J.coarse0;
    const int i = J.row0 + w;
    if (i >= m) return;
    const float *row = Einv + J.e_off + (int64_t)i * m;
    float a0 = 0.f, a1 = 0.f;
    int jj = lane;
    for (; jj + 64 < m; jj += 128) {
        a0 += row[jj] * (float)tl[jj];
        a1 += row[jj + 64] * (float)tl[jj + 64];
    }
    if (jj < m) a0 += row[jj] * (float)tl[jj];
    float v = a0 + a1;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    if (lane == 0) t2[J.coarse0 + i] = (double)v;
}

// t2 = E_hat t1 by an iterative solve (the inexact coarse solve that varies
// from call to call): Jacobi-preconditioned CG on E t2 = t1 from t2 = 0,
// stopped at the first step with ||t1 - E t2|| <= rtol ||t1|| or after
// maxiter steps.  One 1024-thread block per system; E in CSR over the global
// coarse numbering (block diagonal by system, exact zeros dropped), dinv its
// inverse diagonal.  LDS: r, p, q of the system in dynamic shared memory
// (systems of at most kEcgLdsRows unknowns); else in work (3 x mtot).  Every
// sum is a fixed-order block reduction whose result every thread holds, so
// the loop test is uniform over the block; (r, z) and (r, r) share one.
// iters[sys] accumulates the steps taken.
constexpr int kEcgLdsRows = 2048;

__device__ __forceinline__ void block_sum2(double &a, double &b, double *lds) {
    a = wave_sum(a);
    b = wave_sum(b);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        lds[w] = a;
        lds[16 + w] = b;
    }
    __syncthreads();
    double ra = 0.0, rb = 0.0;
    for (int i = 0; i < kWideBlock / 64; ++i) {
        ra += lds[i];
        rb += lds[16 + i];
    }
    __syncthreads();
    a = ra;
    b = rb;
}

template <bool LDS>
__global__ void __launch_bounds__(kWideBlock) k_ecg(
    const int64_t *__restrict__ ptr, const int32_t *__restrict__ col, const double *__restrict__ val,
    const double *__restrict__ dinv, const int32_t *__restrict__ sys_coarse_off, const double *__restrict__ t1,
    double *__restrict__ t2, double *__restrict__ work, int64_t mtot, double rtol, int32_t maxiter,
    const SysState *__restrict__ st, int64_t *__restrict__ iters) {
    __shared__ double lds[32];
    extern __shared__ double ecg_lds[];
    const int sys = blockIdx.x;
    if (st[sys].done) return;
    const int c0 = sys_coarse_off[sys], c1 = sys_coarse_off[sys + 1];
    // vectors indexed by c - base
    const int base = LDS ? c0 : 0;
    const int64_t len = LDS ? (c1 - c0) : mtot;
    double *r = LDS ? ecg_lds : work;
    double *p = r + len, *q = p + len;
    double a = 0.0, b = 0.0;
    for (int c = c0 + threadIdx.x; c < c1; c += kWideBlock) {
        const double tc = t1[c];
        const double zc = dinv[c] * tc;
        r[c - base] = tc;
        p[c - base] = zc;
        t2[c] = 0.0;
        a += tc * zc;
        b += tc * tc;
    }
    block_sum2(a, b, lds);   // synchronises: p is visible
    double rho = a, rr = b;
    const double lim = rtol * rtol * rr;
    int k = 0;
    while (k < maxiter && rr > lim) {
        double pq = 0.0;
        for (int c = c0 + threadIdx.x; c < c1; c += kWideBlock) {
            double sacc = 0.0;
            for (int64_t e = ptr[c]; e < ptr[c + 1]; ++e) sacc += val[e] * p[col[e] - base];
            q[c - base] = sacc;
            pq += p[c - base] * sacc;
        }
        const double alpha = rho / block_sum(pq, lds, kWideBlock);
        double rz = 0.0, r2 = 0.0;
        for (int c = c0 + threadIdx.x; c < c1; c += kWideBlock) {
            t2[c] += alpha * p[c - base];
            const double rn = r[c - base] - alpha * q[c - base];
            r[c - base] = rn;
            rz += rn * (dinv[c] * rn);
            r2 += rn * rn;
        }
        block_sum2(rz, r2, lds);
        const double beta = rz / rho;
        rho = rz;
        rr = r2;
        for (int c = c0 + threadIdx.x; c < c1; c += kWideBlock) p[c - base] = dinv[c] * r[c - base] + beta * p[c - base];
        __syncthreads();   // p complete before the next product
        ++k;
    }
    if (threadIdx.x == 0) iters[sys] += k;
}

// dst = (float) src: E^{-1} rounded to single precision for the FP32 coarse
// solve
static __global__ void k_to_f32(int64_t n, const double *__restrict__ src, float *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (float)src[i];
}

}  // namespace dfamg
