// Device side of the solver: uploads of the host plan, FP64 inversion of E
// and of the coarsest blocks on the GPU, the Krylov driver (direct launches
// or captured HIP graphs) and the C ABI.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "dfamg.h"
#include "host_plan.hpp"
#include "kernels.hpp"

namespace dfamg {

namespace {

thread_local std::string g_last_error;

struct HipError {
    hipError_t e;
    std::string where;
};

#define HIP_CHECK(call)                                                      \
    do {                                                                     \
        hipError_t e_ = (call);                                              \
        if (e_ != hipSuccess) throw HipError{e_, #call};                     \
    } while (0)

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Owns every device allocation of a handle.
struct DevArena {
    std::vector<void *> ptrs;
    int64_t bytes = 0;
    template <class T>
    T *alloc(size_t count) {
        if (count == 0) count = 1;
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, count * sizeof(T));
        if (e != hipSuccess) {
            if (e == hipErrorOutOfMemory) throw Error{DFAMG_ENOMEM, "device allocation failed"};
            throw HipError{e, "hipMalloc"};
        }
        ptrs.push_back(p);
        bytes += (int64_t)(count * sizeof(T));
        return static_cast<T *>(p);
    }
    template <class T>
    T *upload(const std::vector<T> &v, hipStream_t s) {
        T *p = alloc<T>(v.size());
        if (!v.empty()) HIP_CHECK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
        return p;
    }
    ~DevArena() {
        for (void *p : ptrs) (void)hipFree(p);
    }
};

template <class VT>
struct DevSell {
    DevTile *tiles = nullptr;
    int64_t *soff = nullptr;
    int32_t *sw = nullptr;
    int32_t *col = nullptr;
    VT *val = nullptr;
    int32_t ntiles = 0;
    int64_t nnz = 0, stored = 0;
    std::vector<int32_t> sys_tile_off;  // host copy: tiles per system
    SellView<VT> view() const { return SellView<VT>{tiles, soff, sw, col, val, ntiles}; }
};

std::vector<DevTile> to_dev_tiles(const std::vector<Tile> &t) {
    std::vector<DevTile> d(t.size());
    for (size_t i = 0; i < t.size(); ++i) d[i] = DevTile{t[i].row0, t[i].nrows, t[i].sub, t[i].slot};
    return d;
}

template <class VT>
DevSell<VT> upload_sell(DevArena &ar, const HostSell &S, hipStream_t s, const std::vector<int32_t> &sub_sys,
                        int nsys) {
    DevSell<VT> D;
    D.tiles = ar.upload(to_dev_tiles(S.tiles), s);
    D.soff = ar.upload(S.slice_off, s);
    D.sw = ar.upload(S.slice_w, s);
    D.col = ar.upload(S.col, s);
    std::vector<VT> v(S.val.size());
    for (size_t i = 0; i < v.size(); ++i) v[i] = (VT)S.val[i];
    D.val = ar.upload(v, s);
    D.ntiles = (int32_t)S.tiles.size();
    D.nnz = S.nnz;
    D.stored = (int64_t)S.val.size();
    D.sys_tile_off.assign(nsys + 1, 0);
    for (const Tile &t : S.tiles) D.sys_tile_off[sub_sys[t.sub] + 1]++;
    for (int i = 0; i < nsys; ++i) D.sys_tile_off[i + 1] += D.sys_tile_off[i];
    return D;
}

// Ranges of the packed rows of `subs` at a level.
std::vector<RowRange> ranges_of(const PackedLevel &L, const std::vector<int32_t> &subs) {
    std::vector<RowRange> r;
    for (int32_t s : subs) r.push_back(RowRange{L.sub_off[s], L.sub_len[s], s, 0});
    return r;
}

void assign_slots(std::vector<RowRange> &r, int rows_per_tile) {
    int32_t slot = 0;
    for (auto &x : r) {
        x.slot0 = slot;
        slot += (x.nrows + rows_per_tile - 1) / rows_per_tile;
    }
}

// Batched FP64 Gauss-Jordan inversion on the device of the dense matrices
// `mats` (row-major, sizes `ns`); returns the transposed inverses in type VT
// concatenated at `out` (offsets `out_off`), and the index of the first
// singular matrix or -1.
template <class VT>
int invert_on_device(DevArena &ar, hipStream_t s, const std::vector<const double *> &mats,
                     const std::vector<int32_t> &ns, VT *out, const std::vector<int64_t> &out_off) {
    const int nb = (int)mats.size();
    if (nb == 0) return -1;
    std::vector<InvJob> jobs(nb);
    std::vector<int64_t> col_off(nb + 1, 0);
    int64_t aug_total = 0;
    int nmax = 0;
    for (int b = 0; b < nb; ++b) {
        jobs[b] = InvJob{ns[b], 0, aug_total};
        aug_total += (int64_t)ns[b] * 2 * ns[b];
        col_off[b + 1] = col_off[b] + ns[b];
        nmax = std::max(nmax, ns[b]);
    }
    std::vector<double> aug(aug_total, 0.0);
    for (int b = 0; b < nb; ++b) {
        const int n = ns[b];
        double *A = &aug[jobs[b].aug_off];
        for (int i = 0; i < n; ++i) {
            for (int j = 0; j < n; ++j) A[(int64_t)i * 2 * n + j] = mats[b][(int64_t)i * n + j];
            A[(int64_t)i * 2 * n + n + i] = 1.0;
        }
    }
    // scratch of this call only
    DevArena tmp;
    double *d_aug = tmp.upload(aug, s);
    InvJob *d_jobs = tmp.upload(jobs, s);
    int64_t *d_coff = tmp.upload(col_off, s);
    double *d_colk = tmp.alloc<double>(col_off[nb]);
    int64_t *d_oof = tmp.upload(out_off, s);
    int64_t maxel = (int64_t)nmax * 2 * nmax;
    const int gx = (int)std::min<int64_t>(1024, (maxel + kBlock - 1) / kBlock);
    for (int k = 0; k < nmax; ++k) {
        hipLaunchKernelGGL(k_gj_pivot, dim3(nb), dim3(kBlock), 0, s, d_jobs, d_aug, d_colk, d_coff, k);
        hipLaunchKernelGGL(k_gj_eliminate, dim3(gx, nb), dim3(kBlock), 0, s, d_jobs, d_aug, d_colk, d_coff, k);
    }
    hipLaunchKernelGGL(k_gj_extract<VT>, dim3(gx, nb), dim3(kBlock), 0, s, d_jobs, d_aug, d_oof, out);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipMemcpyAsync(jobs.data(), d_jobs, nb * sizeof(InvJob), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    for (int b = 0; b < nb; ++b)
        if (jobs[b].singular) return b;
    return -1;
}

}  // namespace

// Event pairs around the hot kernels of each Krylov iteration (one set per
// iteration slot of a chunk / captured graph).
enum KernelId {
    KID_SPMV = DFAMG_KERNEL_SPMV, KID_PROJECT = DFAMG_KERNEL_PROJECT, KID_UPDATE = DFAMG_KERNEL_UPDATE,
    KID_TEST = DFAMG_KERNEL_TEST, KID_PRE0 = DFAMG_KERNEL_PRESMOOTH0, KID_RESTRICT0 = DFAMG_KERNEL_RESTRICT0,
    KID_COARSER = DFAMG_KERNEL_COARSER, KID_PROLONG0 = DFAMG_KERNEL_PROLONG0, KID_POST0 = DFAMG_KERNEL_POSTSMOOTH0,
    KID_DIR = DFAMG_KERNEL_DIRECTION, KID_N = DFAMG_KERNEL_COUNT
};

struct Prof {
    bool on = false, capturing = false;
    int slot = 0, nslots = 0;
    std::vector<hipEvent_t> ev;          // [slot][kid][2]
    std::vector<char> used;              // [slot][kid] recorded in this chunk / graph
    double ms[KID_N] = {};
    int64_t calls[KID_N] = {};
    double bytes[KID_N] = {};
    void init(int n) {
        on = true;
        nslots = n;
        ev.resize((size_t)n * KID_N * 2);
        used.assign((size_t)n * KID_N, 0);
        for (auto &e : ev) HIP_CHECK(hipEventCreate(&e));
    }
    void mark(int kid, int which, hipStream_t st) {
        if (!on) return;
        hipEvent_t e = ev[((size_t)slot * KID_N + kid) * 2 + which];
        if (capturing) HIP_CHECK(record_in_capture(e, st));
        else HIP_CHECK(hipEventRecord(e, st));
        used[(size_t)slot * KID_N + kid] = 1;
    }
    // Append an event-record node to the graph being captured on `st` and
    // make it the capture's only dependency, so it sits between the kernels
    // launched before and after it.
    static hipError_t record_in_capture(hipEvent_t e, hipStream_t st) {
        hipStreamCaptureStatus cs;
        unsigned long long id = 0;
        hipGraph_t g = nullptr;
        const hipGraphNode_t *deps = nullptr;
        size_t nd = 0;
        hipError_t r = hipStreamGetCaptureInfo_v2(st, &cs, &id, &g, &deps, &nd);
        if (r != hipSuccess) return r;
        if (cs != hipStreamCaptureStatusActive) return hipErrorInvalidValue;
        hipGraphNode_t node;
        r = hipGraphAddEventRecordNode(&node, g, deps, nd, e);
        if (r != hipSuccess) return r;
        return hipStreamUpdateCaptureDependencies(st, &node, 1, hipStreamSetCaptureDependencies);
    }
    // Add the spans of the first `full` slots (all kernels) and of `partial`
    // further slots (only kernels up to the stopping test, the rest of such an
    // iteration exits early).
    void collect(int full, int partial) {
        if (!on) return;
        for (int sl = 0; sl < std::min(nslots, full + partial); ++sl)
            for (int k = 0; k < KID_N; ++k) {
                if (!used[(size_t)sl * KID_N + k]) continue;
                if (sl >= full && k > KID_TEST) continue;
                float t = 0.f;
                if (hipEventElapsedTime(&t, ev[((size_t)sl * KID_N + k) * 2], ev[((size_t)sl * KID_N + k) * 2 + 1]) ==
                    hipSuccess) {
                    ms[k] += t;
                    calls[k] += 1;
                }
            }
    }
    void clear_used() {
        if (!capturing) std::fill(used.begin(), used.end(), 0);
    }
    ~Prof() {
        for (auto &e : ev) (void)hipEventDestroy(e);
    }
};

// ---------------------------------------------------------------------------
// preconditioner: packed hierarchy of every subdomain, one launch per step
// ---------------------------------------------------------------------------

struct PrecondBase {
    virtual ~PrecondBase() = default;
    // s = M^{-1} r with partial (r, s) per level-0 tile (part) and per
    // level-0 direct-solved subdomain (part_sub)
    virtual void apply(hipStream_t st, const double *r, double *s, double *part, double *part_sub,
                       const SysState *states, const int32_t *sub_sys, Prof *prof) = 0;
    double kbytes[KID_N] = {};
    virtual const std::vector<int32_t> &sys_tile_off0() const = 0;
    virtual int32_t nslots0() const = 0;
    virtual double bytes_per_apply() const = 0;
};

template <class VT>
struct Hierarchy_dev : PrecondBase {
    struct Lvl {
        int64_t nrows = 0;
        bool active = false;
        DevSell<VT> A, P, R;
        VT *m = nullptr;
        VT *f = nullptr, *res = nullptr, *z = nullptr, *x = nullptr;
        CoarseEntry *coarse = nullptr;
        int32_t ncoarse = 0, coarse_nmax = 0;
        VT *coarse_inv = nullptr;
        int64_t coarse_elems = 0;
    };
    std::vector<Lvl> lv;
    std::vector<int32_t> sto0;
    int32_t slots0 = 0;
    double bytes = 0.0;

    const std::vector<int32_t> &sys_tile_off0() const override { return sto0; }
    int32_t nslots0() const override { return slots0; }
    double bytes_per_apply() const override { return bytes; }

    void build(DevArena &ar, const Plan &plan, hipStream_t s) {
        const int L = plan.nlevels_max;
        lv.resize(L);
        const double sv = sizeof(VT);
        for (int l = 0; l < L; ++l) {
            const PackedLevel &PL = plan.levels[l];
            Lvl &D = lv[l];
            D.nrows = PL.nrows;
            D.active = !PL.active_subs.empty();
            if (l > 0) {
                D.f = ar.alloc<VT>(PL.nrows);
                D.x = ar.alloc<VT>(PL.nrows);
            }
            if (D.active) {
                D.res = ar.alloc<VT>(PL.nrows);
                D.z = ar.alloc<VT>(PL.nrows);
                auto rr = ranges_of(PL, PL.active_subs);
                assign_slots(rr, kSellTileRows);
                D.A = upload_sell<VT>(ar, make_sell(PL.A, rr), s, plan.sub_sys, plan.nsys);
                D.P = upload_sell<VT>(ar, make_sell(PL.P, rr), s, plan.sub_sys, plan.nsys);
                const PackedLevel &PN = plan.levels[l + 1];
                std::vector<int32_t> next_subs;
                for (int sub = 0; sub < plan.nsub; ++sub)
                    if (PN.sub_off[sub] >= 0) next_subs.push_back(sub);
                auto rn = ranges_of(PN, next_subs);
                assign_slots(rn, kSellTileRows);
                D.R = upload_sell<VT>(ar, make_sell(PL.R, rn), s, plan.sub_sys, plan.nsys);
                std::vector<VT> m(PL.m.size());
                for (size_t i = 0; i < m.size(); ++i) m[i] = (VT)PL.m[i];
                D.m = ar.upload(m, s);
                if (l == 0) {
                    sto0 = D.A.sys_tile_off;
                    slots0 = D.A.ntiles;
                    const double n0 = (double)PL.nrows, n1 = (double)plan.levels[1].nrows;
                    const double ib = 4.0;
                    // f = r is FP64 on level 0; m, res, z in VT; s written FP64
                    kbytes[KID_PRE0] = D.A.nnz * (sv + ib) + n0 * (8.0 + 2.0 * sv);
                    kbytes[KID_RESTRICT0] = D.R.nnz * (sv + ib) + n0 * sv + n1 * sv;
                    kbytes[KID_PROLONG0] = D.P.nnz * (sv + ib) + n0 * (2.0 * sv + 8.0) + n1 * sv;
                    kbytes[KID_POST0] = D.A.nnz * (sv + ib) + n0 * (2.0 * sv + 16.0);
                }
                // algorithmic bytes: A twice (pre/res and post), P, R, vectors
                const double ib = 4.0;
                bytes += 2.0 * (D.A.nnz * (sv + ib)) + (D.P.nnz + D.R.nnz) * (sv + ib) +
                         (double)PL.nrows * sv * 10.0;
            }
            if (!PL.coarse_subs.empty()) {
                std::vector<CoarseEntry> ce;
                std::vector<const double *> mats;
                std::vector<std::vector<double>> dense;
                std::vector<int32_t> ns;
                std::vector<int64_t> off;
                int64_t total = 0;
                for (int32_t sub : PL.coarse_subs) {
                    const Csr &M = plan.hier[sub].lv.back().A;
                    const int n = (int)M.nrows;
                    std::vector<double> d((size_t)n * n, 0.0);
                    for (int i = 0; i < n; ++i)
                        for (int64_t k = M.ptr[i]; k < M.ptr[i + 1]; ++k) d[(size_t)i * n + M.col[k]] = M.val[k];
                    dense.push_back(std::move(d));
                    ns.push_back(n);
                    off.push_back(total);
                    ce.push_back(CoarseEntry{sub, n, PL.sub_off[sub], total});
                    total += (int64_t)n * n;
                    D.coarse_nmax = std::max(D.coarse_nmax, n);
                }
                for (auto &d : dense) mats.push_back(d.data());
                D.coarse_inv = ar.alloc<VT>(total);
                D.coarse_elems = total;
                const int bad = invert_on_device<VT>(ar, s, mats, ns, D.coarse_inv, off);
                if (bad >= 0)
                    throw Error{DFAMG_ESINGULAR, "coarsest-level matrix of subdomain " +
                                                     std::to_string(plan.sub_user[PL.coarse_subs[bad]]) +
                                                     " is singular"};
                D.coarse = ar.upload(ce, s);
                D.ncoarse = (int32_t)ce.size();
                bytes += total * sv + 2.0 * PL.nrows * sv;
            }
        }
        if (L > 0 && !lv[0].active) {
            sto0.assign(plan.nsys + 1, 0);
            slots0 = 0;
        }
    }

    void apply(hipStream_t st, const double *r, double *s, double *part, double *part_sub,
               const SysState *states, const int32_t *sub_sys, Prof *prof) override {
        const int L = (int)lv.size();
        auto mark = [&](int kid, int which) {
            if (prof) prof->mark(kid, which, st);
        };
        // downward: pre-smoothing residuals and restriction
        for (int l = 0; l + 1 < L; ++l) {
            Lvl &D = lv[l];
            if (!D.active) continue;
            const dim3 g(grid_for_tiles(D.A.ntiles)), b(kBlock);
            if (l == 0) {
                mark(KID_PRE0, 0);
                hipLaunchKernelGGL((k_pre_res<VT, double>), g, b, 0, st, D.A.view(), D.m, r, D.res, states, sub_sys);
                mark(KID_PRE0, 1);
                mark(KID_RESTRICT0, 0);
            } else {
                hipLaunchKernelGGL((k_pre_res<VT, VT>), g, b, 0, st, D.A.view(), D.m, D.f, D.res, states, sub_sys);
            }
            hipLaunchKernelGGL((k_spmv<VT>), dim3(grid_for_tiles(D.R.ntiles)), b, 0, st, D.R.view(), D.res,
                               lv[l + 1].f, states, sub_sys);
            if (l == 0) {
                mark(KID_RESTRICT0, 1);
                mark(KID_COARSER, 0);
            }
        }
        // direct solves on every subdomain's coarsest level
        for (int l = 0; l < L; ++l) {
            Lvl &D = lv[l];
            if (!D.ncoarse) continue;
            const size_t shm = (size_t)D.coarse_nmax * sizeof(VT);
            if (l == 0)
                hipLaunchKernelGGL((k_coarse<VT, double, double, true>), dim3(D.ncoarse), dim3(kBlock), shm, st,
                                   D.coarse, D.coarse_inv, r, s, part_sub, states, sub_sys);
            else
                hipLaunchKernelGGL((k_coarse<VT, VT, VT, false>), dim3(D.ncoarse), dim3(kBlock), shm, st, D.coarse,
                                   D.coarse_inv, D.f, D.x, part_sub, states, sub_sys);
        }
        // upward: coarse correction and post-smoothing
        for (int l = L - 2; l >= 0; --l) {
            Lvl &D = lv[l];
            if (!D.active) continue;
            const dim3 g(grid_for_tiles(D.A.ntiles)), b(kBlock);
            if (l == 0) {
                mark(KID_COARSER, 1);
                mark(KID_PROLONG0, 0);
                hipLaunchKernelGGL((k_prolong<VT, double>), g, b, 0, st, D.P.view(), D.m, r, lv[1].x, D.z, states,
                                   sub_sys);
                mark(KID_PROLONG0, 1);
                mark(KID_POST0, 0);
                hipLaunchKernelGGL((k_post<VT, double, double, true>), g, b, 0, st, D.A.view(), D.m, r, D.z, s, part,
                                   states, sub_sys);
                mark(KID_POST0, 1);
            } else {
                hipLaunchKernelGGL((k_prolong<VT, VT>), g, b, 0, st, D.P.view(), D.m, D.f, lv[l + 1].x, D.z, states,
                                   sub_sys);
                hipLaunchKernelGGL((k_post<VT, VT, VT, false>), g, b, 0, st, D.A.view(), D.m, D.f, D.z, D.x, part,
                                   states, sub_sys);
            }
        }
    }
};

// ---------------------------------------------------------------------------
// the handle
// ---------------------------------------------------------------------------

struct Handle {
    Plan plan;
    dfamg_params prm{};
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    int device = 0;
    DevArena ar;
    std::string err;
    // outer operator and deflation
    DevSell<double> A;
    std::vector<int32_t> sto_outer;        // tiles per system (outer tiling)
    int32_t *d_sto_outer = nullptr;
    int32_t *d_sub_tile_off = nullptr;     // outer tiles per subdomain
    int32_t *d_sub_sys = nullptr;
    int32_t *d_sys_sub_off = nullptr;
    int64_t *d_perm = nullptr;
    double *Z = nullptr, *AZown = nullptr, *AZoffv = nullptr, *EinvT = nullptr, *t2 = nullptr;
    int32_t *AZoffp = nullptr, *AZoffc = nullptr;
    int64_t *d_sys_E_off = nullptr;
    // vectors
    double *b = nullptr, *y = nullptr, *r = nullptr, *p = nullptr, *q = nullptr, *s = nullptr, *w = nullptr,
           *x = nullptr;
    // partials and state
    double *part_outer = nullptr, *part_rr = nullptr, *part_rs = nullptr, *part_rs_sub = nullptr;
    int32_t *d_sto0 = nullptr;
    SysState *states = nullptr;
    SysState *h_states = nullptr;          // pinned
    double *hist = nullptr;
    int32_t hist_stride = 0;
    double *relres_true = nullptr;
    std::unique_ptr<PrecondBase> M;
    // graph of `graph_iters` iterations
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int32_t graph_k = 0;
    bool have_rhs = false;
    double setup_device_s = 0.0, solve_s = 0.0;
    double bytes_iter = 0.0;
    Prof prof;
    bool graph_profile_fallback = false;
    bool probe_graph_events();

    ~Handle() {
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (h_states) (void)hipHostFree(h_states);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }

    int nsys() const { return plan.nsys; }
    int ndv() const { return plan.ndv; }

    void setup_device();
    void iteration(hipStream_t st);
    void initial(hipStream_t st);
    void finish(hipStream_t st);
    void precond(hipStream_t st, const double *rin, double *sout, bool profiled = false);
    void launch_iterations(int k);
    dfamg_status run_solve(const double *rhs, double *xio);
    void apply_op(int op, const double *in, double *out);
};

#define DISPATCH_NDV(NDV_VALUE, FN)                                         \
    switch (NDV_VALUE) {                                                    \
        case 0: FN(0); break;                                               \
        case 1: FN(1); break;                                               \
        case 2: FN(2); break;                                               \
        case 3: FN(3); break;                                               \
        case 4: FN(4); break;                                               \
        case 5: FN(5); break;                                               \
        case 6: FN(6); break;                                               \
        case 7: FN(7); break;                                               \
        case 8: FN(8); break;                                               \
        default: throw Error{DFAMG_EINVAL, "ndv out of range"};            \
    }

void Handle::setup_device() {
    const double t0 = now_s();
    hipStream_t sm = stream;
    const Plan &P = plan;
    const int nsys = P.nsys, nsub = P.nsub, ndv = P.ndv;
    const int64_t n = P.n;
    for (int sy = 0; sy < nsys; ++sy)
        if (P.sys_m[sy] > 4096)
            throw Error{DFAMG_EINVAL, "coarse operator of a system exceeds 4096 unknowns (subdomains x vectors)"};
    // outer matrix over all subdomains
    std::vector<RowRange> rr;
    for (int sub = 0; sub < nsub; ++sub)
        rr.push_back(RowRange{P.sub_row_off[sub], (int32_t)(P.sub_row_off[sub + 1] - P.sub_row_off[sub]), sub, 0});
    assign_slots(rr, kSellTileRows);
    HostSell outer = make_sell(P.A, rr);
    A = upload_sell<double>(ar, outer, sm, P.sub_sys, nsys);
    sto_outer = A.sys_tile_off;
    d_sto_outer = ar.upload(sto_outer, sm);
    std::vector<int32_t> sub_tile_off(nsub + 1, 0);
    for (const Tile &t : outer.tiles) sub_tile_off[t.sub + 1]++;
    for (int i = 0; i < nsub; ++i) sub_tile_off[i + 1] += sub_tile_off[i];
    d_sub_tile_off = ar.upload(sub_tile_off, sm);
    d_sub_sys = ar.upload(P.sub_sys, sm);
    d_sys_sub_off = ar.upload(P.sys_sub_off, sm);
    d_perm = ar.upload(P.perm, sm);
    Z = ar.upload(P.Z, sm);
    AZown = ar.upload(P.AZown, sm);
    std::vector<int32_t> offp(P.AZoff.ptr.begin(), P.AZoff.ptr.end());
    AZoffp = ar.upload(offp, sm);
    AZoffc = ar.upload(P.AZoff.col, sm);
    AZoffv = ar.upload(P.AZoff.val, sm);
    t2 = ar.alloc<double>((size_t)nsub * std::max(ndv, 1));
    // E^{-1} per system (FP64, Gauss-Jordan on the device)
    std::vector<int64_t> eoff(P.sys_E_off.begin(), P.sys_E_off.end());
    d_sys_E_off = ar.upload(eoff, sm);
    EinvT = ar.alloc<double>(std::max<int64_t>(1, P.sys_E_off[nsys]));
    if (ndv > 0) {
        std::vector<const double *> mats;
        std::vector<int32_t> ns;
        std::vector<int64_t> off;
        for (int sy = 0; sy < nsys; ++sy) {
            mats.push_back(&P.E[P.sys_E_off[sy]]);
            ns.push_back(P.sys_m[sy]);
            off.push_back(P.sys_E_off[sy]);
        }
        const int bad = invert_on_device<double>(ar, sm, mats, ns, EinvT, off);
        if (bad >= 0)
            throw Error{DFAMG_ESINGULAR, "E = Z^T A Z of system " + std::to_string(bad) + " is singular"};
    }
    // vectors
    b = ar.alloc<double>(n);
    y = ar.alloc<double>(n);
    r = ar.alloc<double>(n);
    p = ar.alloc<double>(n);
    q = ar.alloc<double>(n);
    s = ar.alloc<double>(n);
    w = ar.alloc<double>(n);
    x = ar.alloc<double>(n);
    const int nt = A.ntiles;
    part_outer = ar.alloc<double>((size_t)nt * (ndv + 1));
    part_rr = ar.alloc<double>(nt);
    part_rs_sub = ar.alloc<double>(nsub);
    HIP_CHECK(hipMemsetAsync(part_rs_sub, 0, sizeof(double) * nsub, sm));
    states = ar.alloc<SysState>(nsys);
    HIP_CHECK(hipMemsetAsync(states, 0, sizeof(SysState) * nsys, sm));
    HIP_CHECK(hipHostMalloc((void **)&h_states, sizeof(SysState) * nsys, hipHostMallocDefault));
    hist_stride = prm.maxiter + 1;
    hist = ar.alloc<double>((size_t)nsys * hist_stride);
    relres_true = ar.alloc<double>(nsys);
    // preconditioner
    if (prm.precond == DFAMG_PRECOND_AMG) {
        if (prm.precision == DFAMG_PREC_MIXED) {
            auto H = std::make_unique<Hierarchy_dev<float>>();
            H->build(ar, P, sm);
            M = std::move(H);
        } else {
            auto H = std::make_unique<Hierarchy_dev<double>>();
            H->build(ar, P, sm);
            M = std::move(H);
        }
        part_rs = ar.alloc<double>(std::max(1, M->nslots0()));
        HIP_CHECK(hipMemsetAsync(part_rs, 0, sizeof(double) * std::max(1, M->nslots0()), sm));
        d_sto0 = ar.upload(M->sys_tile_off0(), sm);
    } else {
        part_rs = ar.alloc<double>(nt);
        d_sto0 = d_sto_outer;
    }
    if (prm.profile) {
        prof.init(std::max(prm.graph_iters, 8));
        if (prm.graph_iters > 0 && !probe_graph_events()) {
            // event nodes cannot be captured here: profile with direct launches
            prm.graph_iters = 0;
            graph_profile_fallback = true;
        }
    }
    {
        const double nd = (double)n, nnzA = (double)P.nnz;
        prof.bytes[KID_SPMV] = nnzA * 12.0 + 16.0 * nd + 8.0 * ndv * nd;
        prof.bytes[KID_UPDATE] = 48.0 * nd + 8.0 * ndv * nd + (ndv ? 12.0 * (double)P.AZoff.nnz() + 4.0 * nd : 0.0);
        prof.bytes[KID_PROJECT] = 8.0 * (double)P.sys_E_off[nsys] + 8.0 * (ndv + 1) * A.ntiles;
        if (M)
            for (int k = 0; k < KID_N; ++k)
                if (M->kbytes[k] > 0) prof.bytes[k] = M->kbytes[k];
    }
    // algorithmic bytes of one CG iteration
    {
        const double nnz = (double)P.nnz;
        bytes_iter = nnz * 12.0 + 4.0 * (n + 1) + 16.0 * n;                  // SpMV: A, x, q
        bytes_iter += 8.0 * ndv * n * 2.0 + 12.0 * (double)P.AZoff.nnz();   // Z, AZ
        bytes_iter += 8.0 * (double)P.sys_E_off[nsys];                      // E^{-1}
        bytes_iter += 8.0 * n * 8.0;                                        // y,r (rw), p,q read; s,p read, p write
        if (M) bytes_iter += M->bytes_per_apply();
    }
    HIP_CHECK(hipStreamSynchronize(sm));
    setup_device_s = now_s() - t0;
}

__global__ void k_probe(double *p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) p[0] += 1.0;
}

// True when event-record nodes can be placed inside a captured graph.
bool Handle::probe_graph_events() {
    double *buf = ar.alloc<double>(1);
    HIP_CHECK(hipMemsetAsync(buf, 0, sizeof(double), stream));
    HIP_CHECK(hipStreamSynchronize(stream));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_CHECK(hipEventCreate(&e0));
    HIP_CHECK(hipEventCreate(&e1));
    bool ok = false;
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    if (hipStreamBeginCapture(cap_stream, hipStreamCaptureModeRelaxed) == hipSuccess) {
        bool rec = Prof::record_in_capture(e0, cap_stream) == hipSuccess;
        hipLaunchKernelGGL(k_probe, dim3(1), dim3(64), 0, cap_stream, buf);
        rec = rec && Prof::record_in_capture(e1, cap_stream) == hipSuccess;
        const bool ended = hipStreamEndCapture(cap_stream, &g) == hipSuccess;
        if (rec && ended && hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) == hipSuccess &&
            hipGraphLaunch(ge, stream) == hipSuccess && hipStreamSynchronize(stream) == hipSuccess) {
            float t = -1.f;
            ok = hipEventElapsedTime(&t, e0, e1) == hipSuccess && t >= 0.f;
        }
    }
    (void)hipGetLastError();
    if (ge) (void)hipGraphExecDestroy(ge);
    if (g) (void)hipGraphDestroy(g);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ok;
}

void Handle::precond(hipStream_t st, const double *rin, double *sout, bool profiled) {
    if (M) {
        M->apply(st, rin, sout, part_rs, part_rs_sub, states, d_sub_sys, (profiled && prof.on) ? &prof : nullptr);
    } else {
        hipLaunchKernelGGL(k_identity, dim3(grid_for_tiles(A.ntiles)), dim3(kBlock), 0, st, A.tiles, A.ntiles, rin,
                           sout, part_rs, states, d_sub_sys);
    }
}

// One CG iteration on the deflated system (all systems at once).
void Handle::iteration(hipStream_t st) {
    const dim3 gt(grid_for_tiles(A.ntiles)), b(kBlock);
    const int nt = A.ntiles;
    const size_t red_shm = sizeof(double) * (4096 + 16);
#define ITER_NDV(K)                                                                                             \
    prof.mark(KID_SPMV, 0, st);                                                                                 \
    hipLaunchKernelGGL((k_outer<K, 0>), gt, b, 0, st, A.view(), p, nullptr, q, Z, part_outer, nt, states,        \
                       d_sub_sys);                                                                              \
    prof.mark(KID_SPMV, 1, st);                                                                                 \
    prof.mark(KID_PROJECT, 0, st);                                                                              \
    hipLaunchKernelGGL((k_project_reduce<K, 0>), dim3(nsys()), dim3(kReduceBlock), red_shm, st, part_outer, nt,  \
                       d_sto_outer, d_sub_tile_off, d_sys_sub_off, EinvT, d_sys_E_off, t2, states);             \
    prof.mark(KID_PROJECT, 1, st);                                                                              \
    prof.mark(KID_UPDATE, 0, st);                                                                               \
    hipLaunchKernelGGL((k_update<K, 0>), gt, b, 0, st, A.tiles, nt, p, q, y, r, AZown, AZoffp, AZoffc, AZoffv,  \
                       t2, part_rr, states, d_sub_sys);                                                         \
    prof.mark(KID_UPDATE, 1, st);
    DISPATCH_NDV(ndv(), ITER_NDV)
#undef ITER_NDV
    prof.mark(KID_TEST, 0, st);
    hipLaunchKernelGGL(k_residual_test<0>, dim3(nsys()), b, 0, st, part_rr, d_sto_outer, states, hist, hist_stride,
                       prm.rtol, prm.maxiter, nullptr);
    prof.mark(KID_TEST, 1, st);
    precond(st, r, s, true);
    prof.mark(KID_DIR, 0, st);
    hipLaunchKernelGGL(k_rho<0>, dim3(nsys()), b, 0, st, part_rs, d_sto0, part_rs_sub, d_sys_sub_off, states);
    hipLaunchKernelGGL(k_cg_direction, gt, b, 0, st, A.tiles, nt, s, p, states, d_sub_sys);
    prof.mark(KID_DIR, 1, st);
}

__global__ void k_zero_null_rhs(const DevTile *__restrict__ tiles, int32_t ntiles, double *__restrict__ y,
                                const SysState *__restrict__ st, const int32_t *__restrict__ sub_sys) {
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    if (st[sub_sys[T.sub]].bb != 0.0) return;
    if ((int)threadIdx.x < T.nrows) y[T.row0 + threadIdx.x] = 0.0;
}

__global__ void k_copy_dir(const DevTile *__restrict__ tiles, int32_t ntiles, const double *__restrict__ s,
                           double *__restrict__ p) {
    const int tile = tile_of_block(ntiles);
    if (tile >= ntiles) return;
    const DevTile T = tiles[tile];
    if ((int)threadIdx.x < T.nrows) p[T.row0 + threadIdx.x] = s[T.row0 + threadIdx.x];
}

// r0 = P(b - A y0), stopping test, s0 = M^{-1} r0, rho0, p0 = s0
void Handle::initial(hipStream_t st) {
    const dim3 gt(grid_for_tiles(A.ntiles)), b(kBlock);
    const int nt = A.ntiles;
    const size_t red_shm = sizeof(double) * (4096 + 16);
#define INIT_NDV(K)                                                                                             \
    hipLaunchKernelGGL((k_outer<K, 1>), gt, b, 0, st, A.view(), y, this->b, w, Z, part_outer, nt, states,       \
                       d_sub_sys);                                                                              \
    hipLaunchKernelGGL((k_project_reduce<K, 1>), dim3(nsys()), dim3(kReduceBlock), red_shm, st, part_outer, nt,  \
                       d_sto_outer, d_sub_tile_off, d_sys_sub_off, EinvT, d_sys_E_off, t2, states);             \
    hipLaunchKernelGGL((k_update<K, 1>), gt, b, 0, st, A.tiles, nt, nullptr, w, nullptr, r, AZown, AZoffp,       \
                       AZoffc, AZoffv, t2, part_rr, states, d_sub_sys);
    DISPATCH_NDV(ndv(), INIT_NDV)
#undef INIT_NDV
    hipLaunchKernelGGL(k_residual_test<1>, dim3(nsys()), b, 0, st, part_rr, d_sto_outer, states, hist, hist_stride,
                       prm.rtol, prm.maxiter, nullptr);
    hipLaunchKernelGGL(k_zero_null_rhs, gt, b, 0, st, A.tiles, nt, y, states, d_sub_sys);
    precond(st, r, s);
    hipLaunchKernelGGL(k_rho<1>, dim3(nsys()), b, 0, st, part_rs, d_sto0, part_rs_sub, d_sys_sub_off, states);
    hipLaunchKernelGGL(k_copy_dir, gt, b, 0, st, A.tiles, nt, s, p);
}

// x = y + Z E^{-1} Z^T (b - A y), then ||b - A x|| / ||b||
void Handle::finish(hipStream_t st) {
    const dim3 gt(grid_for_tiles(A.ntiles)), b(kBlock);
    const int nt = A.ntiles;
    const size_t red_shm = sizeof(double) * (4096 + 16);
#define FIN_NDV(K)                                                                                              \
    hipLaunchKernelGGL((k_outer<K, 1>), gt, b, 0, st, A.view(), y, this->b, w, Z, part_outer, nt, states,       \
                       d_sub_sys);                                                                              \
    hipLaunchKernelGGL((k_project_reduce<K, 2>), dim3(nsys()), dim3(kReduceBlock), red_shm, st, part_outer, nt,  \
                       d_sto_outer, d_sub_tile_off, d_sys_sub_off, EinvT, d_sys_E_off, t2, states);             \
    hipLaunchKernelGGL((k_expand<K>), gt, b, 0, st, A.tiles, nt, y, Z, t2, x);                                   \
    hipLaunchKernelGGL((k_outer<K, 2>), gt, b, 0, st, A.view(), x, this->b, w, Z, part_outer, nt, states,       \
                       d_sub_sys);
    DISPATCH_NDV(ndv(), FIN_NDV)
#undef FIN_NDV
    hipLaunchKernelGGL(k_residual_test<2>, dim3(nsys()), b, 0, st, part_outer, d_sto_outer, states, hist,
                       hist_stride, prm.rtol, prm.maxiter, relres_true);
}

void Handle::launch_iterations(int k) {
    if (prm.graph_iters <= 0) {
        prof.clear_used();
        for (int i = 0; i < k; ++i) {
            prof.slot = i;
            iteration(stream);
        }
        return;
    }
    if (!graph_exec) {
        prof.capturing = prof.on;
        HIP_CHECK(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeRelaxed));
        for (int i = 0; i < prm.graph_iters; ++i) {
            prof.slot = i;
            iteration(cap_stream);
        }
        HIP_CHECK(hipStreamEndCapture(cap_stream, &graph));
        HIP_CHECK(hipGraphInstantiate(&graph_exec, graph, nullptr, nullptr, 0));
        graph_k = prm.graph_iters;
        prof.capturing = false;
    }
    for (int i = 0; i < k; i += graph_k) HIP_CHECK(hipGraphLaunch(graph_exec, stream));
}

dfamg_status Handle::run_solve(const double *rhs, double *xio) {
    const double t0 = now_s();
    const int64_t n = plan.n;
    const int nsys = plan.nsys;
    const int nb = (int)((n + 255) / 256);
    hipLaunchKernelGGL(k_gather, dim3(nb), dim3(256), 0, stream, n, d_perm, rhs, b);
    hipLaunchKernelGGL(k_gather, dim3(nb), dim3(256), 0, stream, n, d_perm, xio, y);
    have_rhs = true;
    initial(stream);
    HIP_CHECK(hipGetLastError());
    const int chunk = prm.graph_iters > 0 ? prm.graph_iters : 8;
    int done_iters = 0;
    std::vector<int32_t> it_before(nsys, 0);
    bool first = true;
    for (;;) {
        HIP_CHECK(hipMemcpyAsync(h_states, states, sizeof(SysState) * nsys, hipMemcpyDeviceToHost, stream));
        HIP_CHECK(hipStreamSynchronize(stream));
        if (!first && prof.on) {
            // iterations of this chunk that ran to the end, and the one that
            // stopped at the test
            int full = 0, partial = 0;
            for (int i = 0; i < nsys; ++i) {
                const int ran = h_states[i].iter - it_before[i];
                const int f = h_states[i].done == kRunning ? ran : std::max(0, ran - 1);
                full = std::max(full, f);
                partial = std::max(partial, ran - f);
            }
            if (full > 0) partial = 0;
            prof.collect(full, partial);
        }
        first = false;
        bool all = true;
        for (int i = 0; i < nsys; ++i) {
            if (h_states[i].done == kRunning) all = false;
            it_before[i] = h_states[i].iter;
        }
        if (all || done_iters > prm.maxiter + chunk) break;
        launch_iterations(chunk);
        HIP_CHECK(hipGetLastError());
        done_iters += chunk;
    }
    finish(stream);
    hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(256), 0, stream, n, d_perm, x, xio);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipMemcpyAsync(h_states, states, sizeof(SysState) * nsys, hipMemcpyDeviceToHost, stream));
    HIP_CHECK(hipStreamSynchronize(stream));
    solve_s = now_s() - t0;
    dfamg_status st = DFAMG_OK;
    for (int i = 0; i < nsys && st == DFAMG_OK; ++i) {
        switch (h_states[i].done) {
            case kConverged: break;
            case kMaxIter: st = DFAMG_ENOCONV; break;
            case kNaN: st = DFAMG_ENAN; break;
            case kBreakdown: st = DFAMG_EBREAKDOWN; break;
            default: st = DFAMG_ENOCONV; break;
        }
    }
    return st;
}

__global__ void k_zt_partial(SellView<double> A, const double *__restrict__ v, const double *__restrict__ Z,
                             double *__restrict__ part, int32_t nslots, int ndv) {
    __shared__ double lds[4];
    const int tile = tile_of_block(A.ntiles);
    if (tile >= A.ntiles) return;
    const DevTile T = A.tiles[tile];
    for (int k = 0; k < ndv; ++k) {
        double a = 0.0;
        if ((int)threadIdx.x < T.nrows) {
            const int row = T.row0 + threadIdx.x;
            a = Z[(int64_t)row * ndv + k] * v[row];
        }
        const double sum = block_sum256(a, lds);
        if (threadIdx.x == 0) part[(int64_t)(k + 1) * nslots + T.slot] = sum;
    }
}

__global__ void k_plain_spmv(SellView<double> A, const double *__restrict__ x, double *__restrict__ y) {
    const int tile = tile_of_block(A.ntiles);
    if (tile >= A.ntiles) return;
    const DevTile T = A.tiles[tile];
    if ((int)threadIdx.x >= T.nrows) return;
    y[T.row0 + threadIdx.x] = sell_row<double, double>(A, tile, threadIdx.x, [&](int c) { return x[c]; });
}

void Handle::apply_op(int op, const double *in, double *out) {
    const int64_t n = plan.n;
    const int nb = (int)((n + 255) / 256);
    const dim3 gt(grid_for_tiles(A.ntiles)), b(kBlock);
    const int nt = A.ntiles;
    const size_t red_shm = sizeof(double) * (4096 + 16);
    hipStream_t st = stream;
    hipLaunchKernelGGL(k_gather, dim3(nb), dim3(256), 0, st, n, d_perm, in, w);
    HIP_CHECK(hipMemsetAsync(states, 0, sizeof(SysState) * plan.nsys, st));
    switch (op) {
        case DFAMG_OP_SPMV:
            hipLaunchKernelGGL(k_plain_spmv, gt, b, 0, st, A.view(), w, x);
            break;
        case DFAMG_OP_PROJECT:
            hipLaunchKernelGGL(k_zt_partial, gt, b, 0, st, A.view(), w, Z, part_outer, nt, ndv());
#define PROJ_NDV(K)                                                                                             \
    hipLaunchKernelGGL((k_project_reduce<K, 2>), dim3(nsys()), dim3(kReduceBlock), red_shm, st, part_outer, nt,  \
                       d_sto_outer, d_sub_tile_off, d_sys_sub_off, EinvT, d_sys_E_off, t2, states);             \
    hipLaunchKernelGGL((k_update<K, 2>), gt, b, 0, st, A.tiles, nt, nullptr, w, nullptr, x, AZown, AZoffp,       \
                       AZoffc, AZoffv, t2, part_rr, states, d_sub_sys);
            DISPATCH_NDV(ndv(), PROJ_NDV)
#undef PROJ_NDV
            break;
        case DFAMG_OP_PRECOND:
            precond(st, w, x);
            break;
        case DFAMG_OP_RECOVER:
            if (!have_rhs) throw Error{DFAMG_EINVAL, "RECOVER needs a previous solve (for b)"};
#define REC_NDV(K)                                                                                              \
    hipLaunchKernelGGL((k_outer<K, 1>), gt, b, 0, st, A.view(), w, this->b, q, Z, part_outer, nt, states,       \
                       d_sub_sys);                                                                              \
    hipLaunchKernelGGL((k_project_reduce<K, 2>), dim3(nsys()), dim3(kReduceBlock), red_shm, st, part_outer, nt,  \
                       d_sto_outer, d_sub_tile_off, d_sys_sub_off, EinvT, d_sys_E_off, t2, states);             \
    hipLaunchKernelGGL((k_expand<K>), gt, b, 0, st, A.tiles, nt, w, Z, t2, x);
            DISPATCH_NDV(ndv(), REC_NDV)
#undef REC_NDV
            break;
        default:
            throw Error{DFAMG_EINVAL, "unknown operator"};
    }
    hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(256), 0, st, n, d_perm, x, out);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(st));
}

}  // namespace dfamg

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

using namespace dfamg;

struct dfamg_handle_s {
    Handle h;
};

struct dfamg_plan_s {
    Plan plan;
    std::string err;
};

namespace {

template <class F>
dfamg_status guarded(std::string *err, F &&fn) {
    try {
        return fn();
    } catch (const Error &e) {
        if (err) *err = e.msg;
        g_last_error = e.msg;
        return e.status;
    } catch (const HipError &e) {
        std::string m = std::string("HIP error ") + hipGetErrorString(e.e) + " in " + e.where;
        if (err) *err = m;
        g_last_error = m;
        return DFAMG_EHIP;
    } catch (const std::bad_alloc &) {
        if (err) *err = "host allocation failed";
        g_last_error = "host allocation failed";
        return DFAMG_ENOMEM;
    }
}

void check_device() {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count == 0) throw Error{DFAMG_ENOGPU, "no HIP device"};
    int dev = 0;
    HIP_CHECK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_CHECK(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        throw Error{DFAMG_ENOGPU, std::string("this build targets gfx950, device is ") + prop.gcnArchName};
}

dfamg_status do_setup(const dfamg_params *prm, int32_t nsys, const int64_t *sys_row_off, int64_t n,
                      const int64_t *row_ptr, const int32_t *col, const double *val, const int32_t *part,
                      int32_t nsub, int32_t ndv, const double *Z, void *stream, dfamg_handle *out) {
    if (!out) {
        g_last_error = "out is NULL";
        return DFAMG_EINVAL;
    }
    *out = nullptr;
    return guarded(nullptr, [&]() -> dfamg_status {
        dfamg_params p;
        if (prm) p = *prm;
        else dfamg_params_default(&p);
        auto H = std::make_unique<dfamg_handle_s>();
        build_plan(H->h.plan, p, nsys, sys_row_off, n, row_ptr, col, val, part, nsub, ndv, Z);
        check_device();
        H->h.prm = p;
        H->h.stream = static_cast<hipStream_t>(stream);
        HIP_CHECK(hipGetDevice(&H->h.device));
        HIP_CHECK(hipStreamCreateWithFlags(&H->h.cap_stream, hipStreamNonBlocking));
        H->h.setup_device();
        if (p.verbose)
            std::fprintf(stderr, "[dfamg] setup host %.3f s, device %.3f s, levels %d, device memory %.1f MB\n",
                         H->h.plan.host_seconds, H->h.setup_device_s, H->h.plan.nlevels_max,
                         H->h.ar.bytes / 1048576.0);
        *out = H.release();
        return DFAMG_OK;
    });
}

}  // namespace

extern "C" {

void dfamg_params_default(dfamg_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->solver = DFAMG_SOLVER_CG;
    p->maxiter = 1000;
    p->rtol = 1e-8;
    p->precision = DFAMG_PREC_FP64;
    p->smoother = DFAMG_SMOOTHER_SPAI0;
    p->jacobi_omega = 0.8;
    p->coarse_enough = 500;
    p->eps_strong = 0.08;
    p->max_levels = 20;
    p->block_size = 1;
    p->precond = DFAMG_PRECOND_AMG;
    p->spmv_format = DFAMG_FORMAT_AUTO;
    p->graph_iters = 16;
    p->host_threads = 0;
    p->verbose = 0;
}

dfamg_status dfamg_setup(const dfamg_params *prm, int64_t n, const int64_t *row_ptr, const int32_t *col,
                         const double *val, const int32_t *part, int32_t nsub, int32_t ndv, const double *Z,
                         void *stream, dfamg_handle *out) {
    return do_setup(prm, 1, nullptr, n, row_ptr, col, val, part, nsub, ndv, Z, stream, out);
}

dfamg_status dfamg_setup_batched(const dfamg_params *prm, int32_t nsys, const int64_t *sys_row_off, int64_t n,
                                 const int64_t *row_ptr, const int32_t *col, const double *val, const int32_t *part,
                                 int32_t nsub, int32_t ndv, const double *Z, void *stream, dfamg_handle *out) {
    if (!sys_row_off) {
        g_last_error = "sys_row_off is NULL";
        return DFAMG_EINVAL;
    }
    return do_setup(prm, nsys, sys_row_off, n, row_ptr, col, val, part, nsub, ndv, Z, stream, out);
}

dfamg_status dfamg_solve(dfamg_handle h, const double *rhs, double *x, int32_t *iters, double *relres,
                         double *relres_true, double *history, int32_t history_cap) {
    if (!h || !rhs || !x) {
        g_last_error = "null argument";
        return DFAMG_EINVAL;
    }
    Handle &H = h->h;
    if (H.plan.nsys != 1) {
        H.err = "dfamg_solve needs a single-system handle (use dfamg_solve_batched)";
        return DFAMG_EINVAL;
    }
    return guarded(&H.err, [&]() -> dfamg_status {
        HIP_CHECK(hipSetDevice(H.device));
        const dfamg_status st = H.run_solve(rhs, x);
        const SysState &S = H.h_states[0];
        if (iters) *iters = S.iter;
        if (relres) *relres = S.relres;
        double rt = 0.0;
        HIP_CHECK(hipMemcpy(&rt, H.relres_true, sizeof(double), hipMemcpyDeviceToHost));
        if (relres_true) *relres_true = rt;
        if (history && history_cap > 0) {
            const int cnt = std::min(history_cap, std::min(S.iter + 1, H.hist_stride));
            HIP_CHECK(hipMemcpy(history, H.hist, sizeof(double) * cnt, hipMemcpyDeviceToHost));
        }
        if (H.prm.verbose)
            std::fprintf(stderr, "[dfamg] solve %.3f ms, %d iterations, relres %.3e\n", H.solve_s * 1e3, S.iter,
                         rt);
        return st;
    });
}

dfamg_status dfamg_solve_batched(dfamg_handle h, const double *rhs, double *x, int32_t *iters,
                                 double *relres_true, int32_t *status) {
    if (!h || !rhs || !x) {
        g_last_error = "null argument";
        return DFAMG_EINVAL;
    }
    Handle &H = h->h;
    return guarded(&H.err, [&]() -> dfamg_status {
        HIP_CHECK(hipSetDevice(H.device));
        const dfamg_status st = H.run_solve(rhs, x);
        const int ns = H.plan.nsys;
        std::vector<double> rt(ns);
        HIP_CHECK(hipMemcpy(rt.data(), H.relres_true, sizeof(double) * ns, hipMemcpyDeviceToHost));
        for (int i = 0; i < ns; ++i) {
            const SysState &S = H.h_states[i];
            if (iters) iters[i] = S.iter;
            if (relres_true) relres_true[i] = rt[i];
            if (status) {
                int32_t v = DFAMG_OK;
                if (S.done == kMaxIter) v = DFAMG_ENOCONV;
                else if (S.done == kNaN) v = DFAMG_ENAN;
                else if (S.done == kBreakdown) v = DFAMG_EBREAKDOWN;
                status[i] = v;
            }
        }
        return st;
    });
}

dfamg_status dfamg_apply(dfamg_handle h, int32_t op, const double *in, double *out) {
    if (!h || !in || !out) {
        g_last_error = "null argument";
        return DFAMG_EINVAL;
    }
    Handle &H = h->h;
    return guarded(&H.err, [&]() -> dfamg_status {
        HIP_CHECK(hipSetDevice(H.device));
        H.apply_op(op, in, out);
        return DFAMG_OK;
    });
}

dfamg_status dfamg_get_stats(dfamg_handle h, dfamg_stats *o) {
    if (!h || !o) {
        g_last_error = "null argument";
        return DFAMG_EINVAL;
    }
    Handle &H = h->h;
    std::memset(o, 0, sizeof(*o));
    const Plan &P = H.plan;
    o->n = P.n;
    o->nnz = P.nnz;
    o->nsys = P.nsys;
    o->nsub = P.nsub;
    o->ndv = P.ndv;
    o->m_total = P.nsub * P.ndv;
    o->nlevels_max = P.nlevels_max;
    for (int l = 0; l < P.nlevels_max && l < 20; ++l) {
        o->level_rows[l] = P.levels[l].nrows;
        o->level_nnz[l] = P.levels[l].A.nnz();
        o->level_p_nnz[l] = P.levels[l].P.nnz();
        o->format_level[l] = DFAMG_FORMAT_SELL;
        o->lanes_level[l] = 1;
    }
    o->format_outer = DFAMG_FORMAT_SELL;
    o->setup_host_s = P.host_seconds;
    o->setup_device_s = H.setup_device_s;
    o->solve_s = H.solve_s;
    o->device_bytes = H.ar.bytes;
    o->bytes_per_iter = H.bytes_iter;
    for (int k = 0; k < KID_N; ++k) {
        o->kernel_calls[k] = H.prof.calls[k];
        o->kernel_ms[k] = H.prof.ms[k];
        o->kernel_bytes[k] = H.prof.bytes[k];
    }
    o->profile_in_graph = H.prof.on && H.prm.graph_iters > 0;
    return DFAMG_OK;
}

dfamg_status dfamg_destroy(dfamg_handle h) {
    if (!h) return DFAMG_OK;
    (void)hipSetDevice(h->h.device);
    (void)hipStreamSynchronize(h->h.stream);
    delete h;
    return DFAMG_OK;
}

const char *dfamg_last_error(dfamg_handle h) {
    if (h) return h->h.err.c_str();
    return g_last_error.c_str();
}

// ---------------------------------------------------------------------------
// host-only plan inspection
// ---------------------------------------------------------------------------

dfamg_status dfamg_plan_create(const dfamg_params *prm, int32_t nsys, const int64_t *sys_row_off, int64_t n,
                               const int64_t *row_ptr, const int32_t *col, const double *val, const int32_t *part,
                               int32_t nsub, int32_t ndv, const double *Z, dfamg_plan *out) {
    if (!out) {
        g_last_error = "out is NULL";
        return DFAMG_EINVAL;
    }
    *out = nullptr;
    return guarded(nullptr, [&]() -> dfamg_status {
        dfamg_params p;
        if (prm) p = *prm;
        else dfamg_params_default(&p);
        auto P = std::make_unique<dfamg_plan_s>();
        build_plan(P->plan, p, nsys, sys_row_off, n, row_ptr, col, val, part, nsub, ndv, Z);
        *out = P.release();
        return DFAMG_OK;
    });
}

static const Hierarchy *plan_hier(dfamg_plan p, int32_t sub) {
    if (!p || sub < 0 || sub >= p->plan.nsub) return nullptr;
    return &p->plan.hier[p->plan.user_to_sub[sub]];
}

dfamg_status dfamg_plan_levels(dfamg_plan p, int32_t sub, int32_t cap, int32_t *nlevels, int64_t *rows,
                               int64_t *nnz, int64_t *p_nnz, double *omega) {
    const Hierarchy *H = plan_hier(p, sub);
    if (!H) {
        g_last_error = "bad plan or subdomain";
        return DFAMG_EINVAL;
    }
    if (nlevels) *nlevels = H->nlevels();
    for (int l = 0; l < H->nlevels() && l < cap; ++l) {
        const Level &L = H->lv[l];
        if (rows) rows[l] = L.A.nrows;
        if (nnz) nnz[l] = L.A.nnz();
        if (p_nnz) p_nnz[l] = (l + 1 < H->nlevels()) ? L.P.nnz() : 0;
        if (omega) omega[l] = (l + 1 < H->nlevels()) ? L.omega : 0.0;
    }
    return DFAMG_OK;
}

dfamg_status dfamg_plan_aggregates(dfamg_plan p, int32_t sub, int32_t level, int64_t cap, int32_t *agg,
                                   int64_t *count) {
    const Hierarchy *H = plan_hier(p, sub);
    if (!H || level < 0 || level + 1 >= H->nlevels()) {
        g_last_error = "bad plan, subdomain or level";
        return DFAMG_EINVAL;
    }
    const auto &a = H->lv[level].agg;
    if (count) *count = (int64_t)a.size();
    if (agg)
        for (int64_t i = 0; i < (int64_t)a.size() && i < cap; ++i) agg[i] = a[i];
    return DFAMG_OK;
}

dfamg_status dfamg_plan_level_matrix(dfamg_plan p, int32_t sub, int32_t level, int32_t which, int64_t *nrows,
                                     int64_t *ncols, int64_t *nnz, int64_t *row_ptr, int32_t *col, double *val) {
    const Hierarchy *H = plan_hier(p, sub);
    if (!H || level < 0 || level >= H->nlevels() || (which == 1 && level + 1 >= H->nlevels()) || which < 0 ||
        which > 1) {
        g_last_error = "bad plan, subdomain, level or matrix";
        return DFAMG_EINVAL;
    }
    const Csr &M = which == 0 ? H->lv[level].A : H->lv[level].P;
    if (nrows) *nrows = M.nrows;
    if (ncols) *ncols = M.ncols;
    if (nnz) *nnz = M.nnz();
    if (row_ptr) std::memcpy(row_ptr, M.ptr.data(), sizeof(int64_t) * (M.nrows + 1));
    if (col) std::memcpy(col, M.col.data(), sizeof(int32_t) * M.nnz());
    if (val) std::memcpy(val, M.val.data(), sizeof(double) * M.nnz());
    return DFAMG_OK;
}

dfamg_status dfamg_plan_coarse_operator(dfamg_plan p, int32_t sys, int32_t *m, double *E, int64_t cap) {
    if (!p || sys < 0 || sys >= p->plan.nsys) {
        g_last_error = "bad plan or system";
        return DFAMG_EINVAL;
    }
    const Plan &P = p->plan;
    const int32_t mm = P.sys_m[sys];
    if (m) *m = mm;
    if (E && cap >= (int64_t)mm * mm) std::memcpy(E, &P.E[P.sys_E_off[sys]], sizeof(double) * mm * mm);
    return DFAMG_OK;
}

dfamg_status dfamg_plan_destroy(dfamg_plan p) {
    delete p;
    return DFAMG_OK;
}

}  // extern "C"
