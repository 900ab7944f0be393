// Setup on the GPU: the per-subdomain smoothed-aggregation hierarchies of
// the block-local AMG (section "Implementation": one AMG per subdomain, built
// on the square diagonal block of A) constructed with device kernels, level
// by level for all subdomains at once, in the packed (block-diagonal)
// numbering.  The paper builds them on the CPU and then moves them to the GPU,
// which it names as what erodes the GPU's solve-phase advantage (section
// "Benchmarks", weak scaling discussion).
//
// Every step computes what the host construction (build_hierarchy in
// host_plan.cpp) computes, in the same order of floating-point operations,
// so that the two hierarchies agree bit for bit (this unit is compiled with
// -ffp-contract=off: no product may be fused into a following sum):
//   1. strength: a_ij^2 >= eps^2 |a_ii| |a_jj| (|a_ii| as sqrt(a_ii^2)),
//      eps halved per level;
//   2. plain aggregation in three passes in ascending node order.  Pass 1
//      (a node all of whose strong neighbours are free seeds an aggregate of
//      itself and them) is sequential on the host; here it is computed in
//      rounds: a node is decided as soon as every node before it that could
//      claim it or one of its strong neighbours is decided, and it is a seed
//      exactly when none of those became a seed -- the same seeds as the
//      ascending sweep, found in about as many rounds as the longest chain of
//      such dependences (142 on a 55k-node subdomain of the 150^3 problem).
//      Pass 2 (attach to the heaviest pass-1 neighbour) is parallel as it
//      stands.  Pass 3 never finds a node: a node with strong neighbours that
//      pass 1 left free had one of them claimed, so pass 2 attached it; the
//      kernel checks this and reports any such node as an internal error;
//   3. the filtered matrix A_F (weak off-diagonal entries added to the
//      diagonal), omega = (4/3) / max_i sum_j |a_F,ij / a_F,ii| per
//      subdomain, the smoothed prolongator P = P_tent - omega D^-1 A_F P_tent
//      and R = P^T;
//   4. the smoother diagonal m, the Galerkin product A_c = (R A) P and the
//      restriction operator B = R - (R A) diag(m), the products formed row
//      by row as merges of sorted rows that add each new term to the running
//      sum in the order of the left operand's entries, as the host's dense
//      accumulator does.
// Scalar matrices only (block size 1) and diagonal smoothers (SPAI-0,
// damped Jacobi).
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <functional>
#include <thread>
#include <memory>
#include <type_traits>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "host_plan.hpp"

namespace dfamg {

namespace {

#define SU_CHECK(call)                                                                               \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess)                                                                        \
            throw Error{DFAMG_EHIP, std::string("device setup: ") + #call + ": " + hipGetErrorString(e_)}; \
    } while (0)

constexpr int kSuBlock = 256;
constexpr int kAggBlock = 1024;
constexpr int kRowCap = 160;      // aggregates one row of A_F P_tent may touch (per thread)
constexpr int kMergeCap = 2048;   // entries of one product row held in LDS
constexpr int kYCap = 512;        // entries of one row of the right operand of a product
constexpr int kStatusLds = 150 * 1024;   // subdomains up to this many nodes keep pass 1 in LDS

// error codes of the setup kernels (first one wins)
enum { kSuOk = 0, kSuPass3 = 1, kSuRowCap = 2, kSuMergeCap = 3, kSuRounds = 4 };
enum { kUnd = 0, kRoot = 1, kNot = 2 };

// Owning device allocations of one setup call.
struct Arena {
    std::vector<void *> ptrs;
    template <class T>
    T *alloc(size_t n) {
        void *p = nullptr;
        const hipError_t e = hipMalloc(&p, std::max<size_t>(1, n) * sizeof(T));
        if (e == hipErrorOutOfMemory) throw Error{DFAMG_ENOMEM, "device setup: out of device memory"};
        SU_CHECK(e);
        ptrs.push_back(p);
        return static_cast<T *>(p);
    }
    template <class T>
    T *upload(const std::vector<T> &v, hipStream_t s) {
        T *p = alloc<T>(v.size());
        if (!v.empty()) SU_CHECK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
        return p;
    }
    ~Arena() {
        for (void *p : ptrs) (void)hipFree(p);
    }
};

template <class T>
std::vector<T> download(const T *d, size_t n, hipStream_t s) {
    std::vector<T> h(n);
    if (n) SU_CHECK(hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, s));
    SU_CHECK(hipStreamSynchronize(s));
    return h;
}

// fn(i) for i in [0, count) on up to 16 host threads
void host_parallel(int64_t count, const std::function<void(int64_t)> &fn) {
    const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(count, std::min(16u, std::max(1u, std::thread::hardware_concurrency()))));
    std::atomic<int64_t> next{0};
    auto work = [&] {
        for (int64_t i; (i = next.fetch_add(1)) < count;) fn(i);
    };
    std::vector<std::thread> th;
    for (int t = 1; t < nt; ++t) th.emplace_back(work);
    work();
    for (auto &t : th) t.join();
}

inline unsigned grid_of(int64_t n, int b = kSuBlock) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + b - 1) / b, 1 << 20));
}

__device__ inline void set_err(int32_t *err, int code) { atomicCAS(err, 0, code); }

// ---------------------------------------------------------------------------
// kernels (rows of a packed level; row_sub maps a row to its subdomain, and
// only rows of subdomains with coarsen[s] != 0 are worked on)
// ---------------------------------------------------------------------------

// |a_ii| as sqrt(a_ii^2) (0 without a diagonal entry), and the smoother
// diagonal m_i: SPAI-0 a_ii / sum_j a_ij^2, or damped Jacobi omega / a_ii
__global__ void k_su_diag(int64_t n, const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                          const double *__restrict__ val, double *__restrict__ dn, double *__restrict__ m,
                          int jacobi, double jomega) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double d = 0.0, s = 0.0, sq = 0.0;
        for (int32_t k = ptr[i]; k < ptr[i + 1]; ++k) {
            const double v = val[k];
            if (col[k] == i) {
                d = v;
                sq = v * v;
            }
            s += v * v;
        }
        dn[i] = std::sqrt(sq);
        m[i] = jacobi ? jomega / d : d / s;
    }
}

// strong flags per entry, rows with a strong entry, and the in-degree of
// every node in the strong graph
__global__ void k_su_strong(int64_t n, const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                            const double *__restrict__ val, const double *__restrict__ dn,
                            const int32_t *__restrict__ row_sub, const int32_t *__restrict__ coarsen, double e2,
                            uint8_t *__restrict__ strong, int32_t *__restrict__ has, int32_t *__restrict__ indeg) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t h = 0;
        const bool work = coarsen[row_sub[i]] != 0;
        for (int32_t k = ptr[i]; k < ptr[i + 1]; ++k) {
            const int32_t j = col[k];
            const double f = val[k] * val[k];
            const bool s = work && j != i && f >= e2 * dn[i] * dn[j];
            strong[k] = s ? 1 : 0;
            if (s) {
                h = 1;
                atomicAdd(&indeg[j], 1);
            }
        }
        has[i] = h;
    }
}

// in-neighbour lists of the strong graph (order within a list arbitrary:
// only membership is used)
__global__ void k_su_tfill(int64_t n, const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                           const uint8_t *__restrict__ strong, const int32_t *__restrict__ tptr,
                           int32_t *__restrict__ tfill, int32_t *__restrict__ tcol) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        for (int32_t k = ptr[i]; k < ptr[i + 1]; ++k)
            if (strong[k]) {
                const int32_t j = col[k];
                tcol[tptr[j] + atomicAdd(&tfill[j], 1)] = (int32_t)i;
            }
}

// Status of a node during pass 1: in LDS (one byte per node of the
// workgroup's subdomain) when it fits, else in global memory, read and
// written with workgroup-scope atomics (every reader and writer of a
// subdomain's entries is in its workgroup).
struct StatusLds {
    uint8_t *st;
    __device__ int32_t ld(int64_t local) const { return st[local]; }
    __device__ void put(int64_t local, int32_t v) const { st[local] = (uint8_t)v; }
};
struct StatusGlobal {
    int32_t *st;
    __device__ int32_t ld(int64_t local) const {
        return __hip_atomic_load(st + local, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __device__ void put(int64_t local, int32_t v) const {
        __hip_atomic_store(st + local, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
};

// The nodes j < i whose seeding would block node i in pass 1: j = k and the
// in-neighbours j of k, for k in {i} u N(i) (duplicates kept).  FILL = 0
// counts them.
template <bool FILL>
__global__ void k_su_conflicts(int64_t n, const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                               const uint8_t *__restrict__ strong, const int32_t *__restrict__ tptr,
                               const int32_t *__restrict__ tcol, const int32_t *__restrict__ has,
                               int32_t *__restrict__ cnt, const int64_t *__restrict__ cptr,
                               int32_t *__restrict__ clist) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t c = 0;
        const int64_t base = FILL ? cptr[i] : 0;
        if (has[i])
            for (int32_t e = ptr[i] - 1; e < ptr[i + 1]; ++e) {
                int64_t k;
                if (e < ptr[i]) {
                    k = i;
                } else {
                    if (!strong[e]) continue;
                    k = col[e];
                    if (k < i) {
                        if (FILL) clist[base + c] = (int32_t)k;
                        ++c;
                    }
                }
                for (int32_t q = tptr[k]; q < tptr[k + 1]; ++q) {
                    const int32_t j = tcol[q];
                    if (j >= i) continue;
                    if (FILL) clist[base + c] = j;
                    ++c;
                }
            }
        if (!FILL) cnt[i] = (int32_t)c;
    }
}

// Pass 1 of one subdomain per workgroup, in rounds.  The seeds of the
// ascending sweep are the nodes i with a strong neighbour such that none of
// its conflicts (k_su_conflicts) became a seed; a node is decided once
// every conflict is.  The smallest undecided node is decided in every
// round, so the rounds end; the bound below is never reached.  The final
// status goes to `status`.
template <bool LDS>
__global__ void __launch_bounds__(kAggBlock) k_su_pass1(const int32_t *__restrict__ subs,
                                                        const int64_t *__restrict__ sub_row0,
                                                        const int32_t *__restrict__ sub_n,
                                                        const int64_t *__restrict__ cptr,
                                                        const int32_t *__restrict__ clist,
                                                        const int32_t *__restrict__ has, int32_t *status,
                                                        int32_t *__restrict__ err) {
    extern __shared__ uint8_t lds_status[];
    const int s = subs[blockIdx.x];
    const int64_t r0 = sub_row0[s];
    const int32_t n = sub_n[s];
    typename std::conditional<LDS, StatusLds, StatusGlobal>::type S;
    if constexpr (LDS) S.st = lds_status;
    else S.st = status + r0;
    for (int32_t t = threadIdx.x; t < n; t += kAggBlock) S.put(t, has[r0 + t] ? kUnd : kNot);
    __syncthreads();
    bool done = false;
    for (int32_t round = 0; round <= n && !done; ++round) {
        int open = 0;
        for (int32_t t = threadIdx.x; t < n; t += kAggBlock) {
            if (S.ld(t) != kUnd) continue;
            const int64_t i = r0 + t;
            bool root_conf = false, und_conf = false;
            for (int64_t q = cptr[i]; q < cptr[i + 1]; ++q) {
                const int32_t sj = S.ld(clist[q] - r0);
                root_conf |= sj == kRoot;
                und_conf |= sj == kUnd;
            }
            if (root_conf) S.put(t, kNot);
            else if (!und_conf) S.put(t, kRoot);
            else open = 1;
        }
        done = !__syncthreads_or(open);
    }
    if (!done && threadIdx.x == 0) set_err(err, kSuRounds);
    if constexpr (LDS)
        for (int32_t t = threadIdx.x; t < n; t += kAggBlock) status[r0 + t] = S.ld(t);
}

// Seed numbers in ascending order per subdomain (one workgroup each):
// agg1 = seed number for seeds, nagg[s] = number of seeds.
__global__ void __launch_bounds__(kAggBlock) k_su_seed_ids(const int32_t *__restrict__ subs,
                                                           const int64_t *__restrict__ sub_row0,
                                                           const int32_t *__restrict__ sub_n,
                                                           const int32_t *__restrict__ status,
                                                           int32_t *__restrict__ agg1, int32_t *__restrict__ nagg) {
    typedef hipcub::BlockScan<int32_t, kAggBlock> Scan;
    __shared__ typename Scan::TempStorage tmp;
    __shared__ int32_t base;
    const int s = subs[blockIdx.x];
    const int64_t r0 = sub_row0[s];
    const int32_t n = sub_n[s];
    if (threadIdx.x == 0) base = 0;
    __syncthreads();
    for (int32_t c0 = 0; c0 < n; c0 += kAggBlock) {
        const int32_t t = c0 + threadIdx.x;
        const int32_t flag = (t < n && status[r0 + t] == kRoot) ? 1 : 0;
        int32_t pre = 0, tot = 0;
        Scan(tmp).ExclusiveSum(flag, pre, tot);
        if (flag) agg1[r0 + t] = base + pre;
        __syncthreads();
        if (threadIdx.x == 0) base += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) nagg[s] = base;
}

__global__ void k_su_fill_i32(int64_t n, int32_t *__restrict__ p, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// every seed claims its strong neighbours (each node is claimed by at most
// one seed: two seeds sharing a neighbour would conflict)
__global__ void k_su_claim(int64_t n, const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                           const uint8_t *__restrict__ strong, const int32_t *__restrict__ status,
                           const int32_t *__restrict__ seed_id, int32_t *__restrict__ agg1) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (status[i] != kRoot) continue;
        const int32_t id = seed_id[i];
        agg1[i] = id;
        for (int32_t k = ptr[i]; k < ptr[i + 1]; ++k)
            if (strong[k]) agg1[col[k]] = id;
    }
}

// pass 2 against the pass-1 result, and the check that pass 3 has no work
__global__ void k_su_pass2(int64_t n, const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                           const double *__restrict__ val, const uint8_t *__restrict__ strong,
                           const int32_t *__restrict__ has, const int32_t *__restrict__ row_sub,
                           const int32_t *__restrict__ coarsen, const int32_t *__restrict__ agg1,
                           int32_t *__restrict__ agg, int32_t *__restrict__ err) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (!coarsen[row_sub[i]]) {
            agg[i] = -1;
            continue;
        }
        int32_t a = agg1[i];
        if (a < 0 && has[i]) {
            int32_t target = -1;
            double wbest = 0.0;
            for (int32_t k = ptr[i]; k < ptr[i + 1]; ++k) {
                if (!strong[k]) continue;
                const int32_t g = agg1[col[k]];
                const double w = std::sqrt(val[k] * val[k]);
                if (g >= 0 && (target < 0 || w > wbest)) {
                    target = g;
                    wbest = w;
                }
            }
            a = target;
            if (a < 0) set_err(err, kSuPass3);
        }
        agg[i] = a;
    }
}

// Diagonal of the filtered matrix: the diagonal entry and every weak
// off-diagonal entry of the row, summed in column order; hasd = 0 when the
// row of A_F has no diagonal entry at all.
__global__ void k_su_filtdiag(int64_t n, const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                              const double *__restrict__ val, const uint8_t *__restrict__ strong,
                              const int32_t *__restrict__ row_sub, const int32_t *__restrict__ cont,
                              double *__restrict__ D, int32_t *__restrict__ hasd) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (!cont[row_sub[i]]) continue;
        double d = 0.0;
        int32_t got = 0;
        for (int32_t k = ptr[i]; k < ptr[i + 1]; ++k)
            if (col[k] == i || !strong[k]) {
                d = got ? d + val[k] : val[k];
                got = 1;
            }
        D[i] = d;
        hasd[i] = got;
    }
}

// Row sums of |D^-1 A_F| in column order (the diagonal term at its column)
// and their maximum over the rows of one subdomain per workgroup (rows with
// a zero filtered diagonal are left out; any[s] = 0 when no row is left).
__global__ void __launch_bounds__(kSuBlock) k_su_rho(const int32_t *__restrict__ subs,
                                                     const int64_t *__restrict__ sub_row0,
                                                     const int32_t *__restrict__ sub_n,
                                                     const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                                                     const double *__restrict__ val,
                                                     const uint8_t *__restrict__ strong,
                                                     const double *__restrict__ D, const int32_t *__restrict__ hasd,
                                                     double *__restrict__ rho, int32_t *__restrict__ any) {
    __shared__ double red[kSuBlock];
    __shared__ int32_t got[kSuBlock];
    const int s = subs[blockIdx.x];
    const int64_t r0 = sub_row0[s];
    double best = 0.0;
    int32_t g = 0;
    for (int64_t i = r0 + threadIdx.x; i < r0 + sub_n[s]; i += kSuBlock) {
        if (D[i] == 0.0) continue;
        const double dinv = 1.0 / D[i];
        double r = 0.0;
        bool placed = !hasd[i];
        for (int32_t k = ptr[i]; k < ptr[i + 1]; ++k) {
            const int32_t j = col[k];
            if (!placed && j > i) {
                r = r + std::fabs(dinv * D[i]);
                placed = true;
            }
            if (j != i && strong[k]) r = r + std::fabs(dinv * val[k]);
        }
        if (!placed) r = r + std::fabs(dinv * D[i]);
        best = (g == 0 || r > best) ? r : best;
        g = 1;
    }
    red[threadIdx.x] = best;
    got[threadIdx.x] = g;
    __syncthreads();
    for (int w = kSuBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const double o = red[threadIdx.x + w];
            if (got[threadIdx.x + w] && (!got[threadIdx.x] || o > red[threadIdx.x])) red[threadIdx.x] = o;
            got[threadIdx.x] |= got[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        rho[s] = red[0];
        any[s] = got[0];
    }
}

// One row of P = P_tent - omega D^-1 (A_F P_tent): the A_F entries (strong
// off-diagonals and the filtered diagonal, in column order) with an
// aggregated column, summed per aggregate in that order; entries in
// ascending aggregate order, exact zeros dropped.  Returns the count
// (fills cols / vals when FILL) or -1 when the row exceeds kRowCap.
template <bool FILL>
__device__ int32_t su_prow(int64_t i, const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                           const double *__restrict__ val, const uint8_t *__restrict__ strong,
                           const int32_t *__restrict__ agg, double Dv, int32_t hasd, double omega,
                           int32_t coff, int32_t *__restrict__ ocol, double *__restrict__ oval) {
    int32_t cs[kRowCap];
    double acc[kRowCap];
    int32_t nc = 0;
    auto add = [&](int32_t g, double v) -> bool {
        for (int32_t q = 0; q < nc; ++q)
            if (cs[q] == g) {
                acc[q] = acc[q] + v;
                return true;
            }
        if (nc == kRowCap) return false;
        cs[nc] = g;
        acc[nc] = 0.0 + v;
        ++nc;
        return true;
    };
    bool placed = !hasd;
    for (int32_t k = ptr[i]; k < ptr[i + 1]; ++k) {
        const int32_t j = col[k];
        if (!placed && j > i) {
            placed = true;
            if (agg[i] >= 0 && !add(agg[i], Dv)) return -1;
        }
        if (j != i && strong[k]) {
            const int32_t g = agg[j];
            if (g >= 0 && !add(g, val[k])) return -1;
        }
    }
    if (!placed && agg[i] >= 0 && !add(agg[i], Dv)) return -1;
    // ascending aggregate order (insertion sort; rows are short)
    for (int32_t a = 1; a < nc; ++a) {
        const int32_t c = cs[a];
        const double x = acc[a];
        int32_t b = a - 1;
        while (b >= 0 && cs[b] > c) {
            cs[b + 1] = cs[b];
            acc[b + 1] = acc[b];
            --b;
        }
        cs[b + 1] = c;
        acc[b + 1] = x;
    }
    const double d = Dv != 0.0 ? 1.0 / Dv : 0.0;
    const int32_t own = agg[i];
    bool own_seen = false;
    int32_t cnt = 0;
    auto emit = [&](int32_t c, double v) {
        if (v == 0.0) return;
        if (FILL) {
            ocol[cnt] = coff + c;
            oval[cnt] = v;
        }
        ++cnt;
    };
    for (int32_t q = 0; q < nc; ++q) {
        const int32_t c = cs[q];
        const double x = acc[q];
        if (own >= 0 && !own_seen && c > own) {
            // the tentative entry of the own aggregate, not reached by A_F
            emit(own, 1.0);
            own_seen = true;
        }
        const bool have = !(d == 0.0 || x == 0.0);
        const double y = d * x;
        if (c == own) own_seen = true;
        if (have && y != 0.0) emit(c, (c == own ? 1.0 : 0.0) - omega * y);
        else if (c == own) emit(c, 1.0);
    }
    if (own >= 0 && !own_seen) emit(own, 1.0);
    return cnt;
}

__global__ void k_su_prow(int64_t n, int fill, const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                          const double *__restrict__ val, const uint8_t *__restrict__ strong,
                          const int32_t *__restrict__ agg, const double *__restrict__ D,
                          const int32_t *__restrict__ hasd, const int32_t *__restrict__ row_sub,
                          const int32_t *__restrict__ cont, const double *__restrict__ omega,
                          const int32_t *__restrict__ coarse_off, int32_t *__restrict__ pcount,
                          const int32_t *__restrict__ pptr, int32_t *__restrict__ pcol, double *__restrict__ pval,
                          int32_t *__restrict__ err) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int s = row_sub[i];
        if (!cont[s]) {
            if (!fill) pcount[i] = 0;
            continue;
        }
        int32_t c;
        if (fill)
            c = su_prow<true>(i, ptr, col, val, strong, agg, D[i], hasd[i], omega[s], coarse_off[s], pcol + pptr[i],
                              pval + pptr[i]);
        else
            c = su_prow<false>(i, ptr, col, val, strong, agg, D[i], hasd[i], omega[s], 0, nullptr, nullptr);
        if (c < 0) {
            set_err(err, kSuRowCap);
            c = 0;
        }
        if (!fill) pcount[i] = c;
    }
}

// transpose: column counts, scatter, then each row sorted by column
__global__ void k_su_colcount(int64_t nnz, const int32_t *__restrict__ col, int32_t *__restrict__ cnt) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&cnt[col[k]], 1);
}

__global__ void k_su_scatter_t(int64_t n, const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                               const double *__restrict__ val, const int32_t *__restrict__ tptr,
                               int32_t *__restrict__ tfill, int32_t *__restrict__ tcol, double *__restrict__ tval) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        for (int32_t k = ptr[i]; k < ptr[i + 1]; ++k) {
            const int32_t c = col[k];
            const int32_t d = tptr[c] + atomicAdd(&tfill[c], 1);
            tcol[d] = (int32_t)i;
            tval[d] = val[k];
        }
}

__global__ void k_su_sort_rows(int64_t n, const int32_t *__restrict__ ptr, int32_t *__restrict__ col,
                               double *__restrict__ val) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        for (int32_t a = ptr[i] + 1; a < ptr[i + 1]; ++a) {
            const int32_t c = col[a];
            const double v = val[a];
            int32_t b = a - 1;
            while (b >= ptr[i] && col[b] > c) {
                col[b + 1] = col[b];
                val[b + 1] = val[b];
                --b;
            }
            col[b + 1] = c;
            val[b + 1] = v;
        }
}

// Per row of L: the longest row of M it reaches and the sum of their
// lengths (a bound on the product row's length), as maxima over all rows.
__global__ void k_su_bound(int64_t nrows, const int32_t *__restrict__ Lp, const int32_t *__restrict__ Lj,
                           const int32_t *__restrict__ Mp, int32_t *__restrict__ maxes) {
    int32_t my = 0, mb = 0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nrows; r += (int64_t)gridDim.x * blockDim.x) {
        int64_t b = 0;
        for (int32_t k = Lp[r]; k < Lp[r + 1]; ++k) {
            const int32_t ny = Mp[Lj[k] + 1] - Mp[Lj[k]];
            my = max(my, ny);
            b += ny;
        }
        mb = max(mb, (int32_t)min<int64_t>(b, INT32_MAX));
    }
    atomicMax(&maxes[0], my);
    atomicMax(&maxes[1], mb);
}

// C = L * M, one wavefront per row of C.  The row is kept in LDS as a
// sorted list; for every entry (j, a) of L's row, in order, row j of M
// scaled by a is merged in: a column already present gets the product added
// to its running sum, a new column enters with the product itself -- the
// order in which the host's dense accumulator forms each entry.  Exact
// zeros are dropped at the end.  FILL = 0 writes the row lengths.
template <bool FILL>
__global__ void __launch_bounds__(64) k_su_spgemm(int64_t nrows, const int32_t *__restrict__ Lp,
                                                  const int32_t *__restrict__ Lj, const double *__restrict__ Lx,
                                                  const int32_t *__restrict__ Mp, const int32_t *__restrict__ Mj,
                                                  const double *__restrict__ Mx, int32_t *__restrict__ Ccount,
                                                  const int32_t *__restrict__ Cp, int32_t *__restrict__ Cj,
                                                  double *__restrict__ Cx, int32_t cap, int32_t ycap,
                                                  int32_t *__restrict__ err) {
    // LDS: two lists of cap (column, value) entries and three arrays of ycap
    extern __shared__ double lds_merge[];
    double *vbuf[2] = {lds_merge, lds_merge + cap};
    int32_t *cbuf[2] = {reinterpret_cast<int32_t *>(lds_merge + 2 * cap),
                        reinterpret_cast<int32_t *>(lds_merge + 2 * cap) + cap};
    int32_t *tpos = cbuf[1] + cap;      // per entry of M's row: insert position, -1 when the column exists
    int32_t *newpos = tpos + ycap;      // per new column, in ascending order: insert position
    int32_t *newsrc = newpos + ycap;    // per new column: its entry in M's row
    const int lane = threadIdx.x;
    for (int64_t row = blockIdx.x; row < nrows; row += gridDim.x) {
        int cur = 0;
        int32_t len = 0;
        bool over = false;
        for (int32_t ka = Lp[row]; ka < Lp[row + 1]; ++ka) {
            const int32_t j = Lj[ka];
            const double a = Lx[ka];
            const int32_t y0 = Mp[j], ny = Mp[j + 1] - y0;
            if (ny > ycap || len + ny > cap) {
                over = true;
                break;
            }
            const int32_t *xc = cbuf[cur];
            double *xv = vbuf[cur];
            // 1. positions of M's entries in the current list; an existing
            //    column takes the product into its running sum
            for (int32_t t = lane; t < ny; t += 64) {
                const int32_t c = Mj[y0 + t];
                int32_t lo = 0, hi = len;
                while (lo < hi) {
                    const int32_t mid = (lo + hi) >> 1;
                    if (xc[mid] < c) lo = mid + 1;
                    else hi = mid;
                }
                if (lo < len && xc[lo] == c) {
                    const double p = a * Mx[y0 + t];
                    xv[lo] = xv[lo] + p;
                    tpos[t] = -1;
                } else {
                    tpos[t] = lo;
                }
            }
            __syncthreads();
            // 2. the new columns, ranked in M's row order (ascending)
            int32_t nnew = 0;
            for (int32_t t0 = 0; t0 < ny; t0 += 64) {
                const int32_t t = t0 + lane;
                const bool isnew = t < ny && tpos[t] >= 0;
                const unsigned long long msk = __ballot(isnew);
                if (isnew) {
                    const int32_t r = nnew + __popcll(msk & ((1ull << lane) - 1ull));
                    newpos[r] = tpos[t];
                    newsrc[r] = t;
                }
                nnew += __popcll(msk);
            }
            __syncthreads();
            if (nnew == 0) continue;   // the list keeps its place
            const int nxt = cur ^ 1;
            // 3. an existing entry moves right by the number of new columns
            //    inserted at or before its position; new column r lands at
            //    its insert position plus r
            for (int32_t x = lane; x < len; x += 64) {
                int32_t lo = 0, hi = nnew;
                while (lo < hi) {
                    const int32_t mid = (lo + hi) >> 1;
                    if (newpos[mid] <= x) lo = mid + 1;
                    else hi = mid;
                }
                cbuf[nxt][x + lo] = xc[x];
                vbuf[nxt][x + lo] = xv[x];
            }
            for (int32_t r = lane; r < nnew; r += 64) {
                const int32_t t = newsrc[r];
                cbuf[nxt][newpos[r] + r] = Mj[y0 + t];
                vbuf[nxt][newpos[r] + r] = a * Mx[y0 + t];
            }
            __syncthreads();
            len += nnew;
            cur = nxt;
        }
        if (over) {
            if (lane == 0) {
                set_err(err, kSuMergeCap);
                if (!FILL) Ccount[row] = 0;
            }
            __syncthreads();
            continue;
        }
        // drop exact zeros and write out
        int32_t out = 0;
        for (int32_t x0 = 0; x0 < len; x0 += 64) {
            const int32_t x = x0 + lane;
            const bool keep = x < len && vbuf[cur][x] != 0.0;
            const unsigned long long msk = __ballot(keep);
            if (FILL && keep) {
                const int32_t d = Cp[row] + out + __popcll(msk & ((1ull << lane) - 1ull));
                Cj[d] = cbuf[cur][x];
                Cx[d] = vbuf[cur][x];
            }
            out += __popcll(msk);
        }
        if (!FILL && lane == 0) Ccount[row] = out;
        __syncthreads();
    }
}

// B = R - (R A) diag(m), rows merged column by column, exact zeros dropped
__global__ void k_su_bmap(int64_t nrows, int fill, const int32_t *__restrict__ Rp, const int32_t *__restrict__ Rj,
                          const double *__restrict__ Rx, const int32_t *__restrict__ Qp,
                          const int32_t *__restrict__ Qj, const double *__restrict__ Qx,
                          const double *__restrict__ m, int32_t *__restrict__ Bcount,
                          const int32_t *__restrict__ Bp, int32_t *__restrict__ Bj, double *__restrict__ Bx) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nrows;
         k += (int64_t)gridDim.x * blockDim.x) {
        int32_t a = Rp[k], b = Qp[k];
        const int32_t ae = Rp[k + 1], be = Qp[k + 1];
        int32_t cnt = 0;
        while (a < ae || b < be) {
            int32_t c;
            double v;
            if (b >= be || (a < ae && Rj[a] < Qj[b])) {
                c = Rj[a];
                v = Rx[a++];
            } else if (a >= ae || Qj[b] < Rj[a]) {
                c = Qj[b];
                v = -Qx[b++] * m[c];
            } else {
                c = Rj[a];
                v = Rx[a++] - Qx[b++] * m[c];
            }
            if (v != 0.0) {
                if (fill) {
                    Bj[Bp[k] + cnt] = c;
                    Bx[Bp[k] + cnt] = v;
                }
                ++cnt;
            }
        }
        if (!fill) Bcount[k] = cnt;
    }
}

// AZ of one row i of the permuted operator: the own-subdomain columns
// (row_sub[j] == own) summed into AZown[i][q] in the row's order, the others
// as (t * ndv + q, a_ij z_jq) pairs ordered by column (stable) with equal
// columns summed in that order.  FILL = 0 counts the row's coupling entries.
constexpr int kAzCap = 256;
template <bool FILL>
__global__ void k_su_az(int64_t n, const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                        const double *__restrict__ val, const int32_t *__restrict__ row_sub,
                        const double *__restrict__ Z, int ndv, double *__restrict__ AZown,
                        int32_t *__restrict__ cnt, const int64_t *__restrict__ optr, int32_t *__restrict__ ocol,
                        double *__restrict__ oval, int32_t *__restrict__ err) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t own = row_sub[i];
        int32_t key[kAzCap];
        double v[kAzCap];
        int32_t ne = 0;
        double acc[8];
        for (int q = 0; q < ndv; ++q) acc[q] = 0.0;
        bool over = false;
        for (int32_t k = ptr[i]; k < ptr[i + 1]; ++k) {
            const int32_t j = col[k];
            const int32_t t = row_sub[j];
            for (int q = 0; q < ndv; ++q) {
                const double p = val[k] * Z[(int64_t)j * ndv + q];
                if (t == own) {
                    acc[q] += p;
                } else if (ne < kAzCap) {
                    // stable insertion by column
                    const int32_t c = t * ndv + q;
                    int32_t b = ne - 1;
                    while (b >= 0 && key[b] > c) {
                        key[b + 1] = key[b];
                        v[b + 1] = v[b];
                        --b;
                    }
                    key[b + 1] = c;
                    v[b + 1] = p;
                    ++ne;
                } else {
                    over = true;
                }
            }
        }
        if (over) {
            set_err(err, kSuRowCap);
            if (!FILL) cnt[i] = 0;
            continue;
        }
        if (FILL)
            for (int q = 0; q < ndv; ++q) AZown[i * ndv + q] = acc[q];
        int32_t out = 0;
        for (int32_t a = 0; a < ne;) {
            int32_t e = a + 1;
            double sum = v[a];
            while (e < ne && key[e] == key[a]) sum += v[e++];
            if (FILL) {
                ocol[optr[i] + out] = key[a];
                oval[optr[i] + out] = sum;
            }
            ++out;
            a = e;
        }
        if (!FILL) cnt[i] = out;
    }
}

// ---------------------------------------------------------------------------
// host orchestration
// ---------------------------------------------------------------------------

// Exclusive prefix sum of n counts into ptr (n + 1 entries, ptr[n] = total).
int64_t scan_counts(Arena &ar, const int32_t *cnt, int32_t *ptr, int64_t n, hipStream_t s) {
    size_t bytes = 0;
    SU_CHECK(hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, cnt, ptr, (int)n, s));
    void *tmp = ar.alloc<char>(bytes);
    SU_CHECK(hipcub::DeviceScan::ExclusiveSum(tmp, bytes, cnt, ptr, (int)n, s));
    int32_t last_ptr = 0, last_cnt = 0;
    if (n > 0) {
        SU_CHECK(hipMemcpyAsync(&last_ptr, ptr + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        SU_CHECK(hipMemcpyAsync(&last_cnt, cnt + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    }
    SU_CHECK(hipStreamSynchronize(s));
    const int64_t total = (int64_t)last_ptr + last_cnt;
    if (total > INT32_MAX) throw Error{DFAMG_EINVAL, "device setup: a level exceeds 2^31 entries"};
    const int32_t t32 = (int32_t)total;
    SU_CHECK(hipMemcpyAsync(ptr + n, &t32, sizeof(int32_t), hipMemcpyHostToDevice, s));
    SU_CHECK(hipStreamSynchronize(s));
    return total;
}

struct DCsr {
    int64_t nrows = 0, ncols = 0, nnz = 0;
    int32_t *ptr = nullptr, *col = nullptr;
    double *val = nullptr;
};

DCsr upload_csr(Arena &ar, const Csr &A, hipStream_t s) {
    DCsr D;
    D.nrows = A.nrows;
    D.ncols = A.ncols;
    D.nnz = A.nnz();
    std::vector<int32_t> p(A.ptr.begin(), A.ptr.end());
    D.ptr = ar.upload(p, s);
    D.col = ar.upload(A.col, s);
    D.val = ar.upload(A.val, s);
    return D;
}

// C = L * M (both sorted CSR) on the device
DCsr spgemm(Arena &ar, const DCsr &L, const DCsr &M, int32_t *err, hipStream_t s) {
    DCsr C;
    C.nrows = L.nrows;
    C.ncols = M.ncols;
    int32_t *cnt = ar.alloc<int32_t>(C.nrows + 1);
    // LDS sized for the longest rows this product meets
    int32_t *maxes = ar.alloc<int32_t>(2);
    SU_CHECK(hipMemsetAsync(maxes, 0, 2 * sizeof(int32_t), s));
    hipLaunchKernelGGL(k_su_bound, dim3(grid_of(C.nrows)), dim3(kSuBlock), 0, s, C.nrows, L.ptr, L.col, M.ptr, maxes);
    const std::vector<int32_t> mx = download(maxes, 2, s);
    const int32_t ycap = std::min<int32_t>(std::max(mx[0], 1), kYCap);
    const int32_t cap = std::min<int32_t>(std::max<int32_t>(std::min<int64_t>(mx[1], M.ncols), 1), kMergeCap);
    const size_t lds = (size_t)cap * 2 * (sizeof(double) + sizeof(int32_t)) + (size_t)ycap * 3 * sizeof(int32_t);
    const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(C.nrows, 65536));
    hipLaunchKernelGGL(k_su_spgemm<false>, dim3(g), dim3(64), lds, s, C.nrows, L.ptr, L.col, L.val, M.ptr, M.col,
                       M.val, cnt, nullptr, nullptr, nullptr, cap, ycap, err);
    SU_CHECK(hipGetLastError());
    C.ptr = ar.alloc<int32_t>(C.nrows + 1);
    C.nnz = scan_counts(ar, cnt, C.ptr, C.nrows, s);
    C.col = ar.alloc<int32_t>(C.nnz);
    C.val = ar.alloc<double>(C.nnz);
    hipLaunchKernelGGL(k_su_spgemm<true>, dim3(g), dim3(64), lds, s, C.nrows, L.ptr, L.col, L.val, M.ptr, M.col,
                       M.val, nullptr, C.ptr, C.col, C.val, cap, ycap, err);
    SU_CHECK(hipGetLastError());
    return C;
}

// Rows [r0, r0 + nr) of a packed device CSR, columns shifted by -c0, as a
// host Csr with ncols columns.
Csr local_block(const std::vector<int32_t> &p, const std::vector<int32_t> &c, const std::vector<double> &v,
                int64_t r0, int64_t nr, int64_t c0, int64_t ncols) {
    Csr L;
    L.nrows = nr;
    L.ncols = ncols;
    L.ptr.assign(nr + 1, 0);
    const int64_t k0 = p[r0], k1 = p[r0 + nr];
    L.col.resize(k1 - k0);
    L.val.assign(v.begin() + k0, v.begin() + k1);
    for (int64_t k = k0; k < k1; ++k) L.col[k - k0] = (int32_t)(c[k] - c0);
    for (int64_t i = 0; i <= nr; ++i) L.ptr[i] = p[r0 + i] - k0;
    return L;
}

void check_err(const int32_t *err, hipStream_t s) {
    int32_t e = 0;
    SU_CHECK(hipMemcpyAsync(&e, err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    SU_CHECK(hipStreamSynchronize(s));
    if (e == kSuOk) return;
    const char *why = e == kSuPass3   ? "a node left by the first two aggregation passes (internal error)"
                      : e == kSuRowCap ? "a row of the smoothed prolongator touches more than 160 aggregates "
                                         "(or a row of AZ more than 256 coupling entries)"
                      : e == kSuMergeCap ? "a row of a Galerkin product exceeds 2048 entries (or a row of "
                                           "its right operand 512)"
                                         : "the aggregation rounds did not end (internal error)";
    throw Error{DFAMG_EINVAL, std::string("device setup: ") + why};
}

}  // namespace

void build_hierarchies_device(std::vector<Csr> &local, const SaParams &sp, std::vector<Hierarchy> &out,
                              void *stream) {
    const hipStream_t s = static_cast<hipStream_t>(stream);
    if (sp.bs != 1) throw Error{DFAMG_EINVAL, "device setup supports scalar matrices (block_size 1) only"};
    if (sp.smoother != DFAMG_SMOOTHER_SPAI0 && sp.smoother != DFAMG_SMOOTHER_JACOBI)
        throw Error{DFAMG_EINVAL, "device setup supports the SPAI-0 and damped Jacobi smoothers only"};
    const int nsub = (int)local.size();
    out.assign(nsub, Hierarchy{});
    Arena ar;
    int32_t *err = ar.alloc<int32_t>(1);
    SU_CHECK(hipMemsetAsync(err, 0, sizeof(int32_t), s));

    // level 0: the subdomains' diagonal blocks, packed (block diagonal); the
    // packed operator of every later level is the previous level's Galerkin
    // product, which the kernels leave in exactly that layout
    std::vector<int32_t> alive(nsub, 1);
    std::unique_ptr<Arena> a_mem(new Arena);   // device memory of the current level's operator
    DCsr A;
    {
        int64_t n = 0, nnz = 0;
        for (const Csr &M : local) {
            n += M.nrows;
            nnz += M.nnz();
        }
        if (nnz > INT32_MAX) throw Error{DFAMG_EINVAL, "device setup: a level exceeds 2^31 entries"};
        std::vector<int32_t> p(n + 1, 0), c(nnz);
        std::vector<double> v(nnz);
        std::vector<int64_t> r0(nsub + 1, 0), k0(nsub + 1, 0);
        for (int sb = 0; sb < nsub; ++sb) {
            r0[sb + 1] = r0[sb] + local[sb].nrows;
            k0[sb + 1] = k0[sb] + local[sb].nnz();
        }
        host_parallel(nsub, [&](int64_t sb) {
            const Csr &M = local[sb];
            for (int64_t i = 0; i < M.nrows; ++i) {
                for (int64_t e = M.ptr[i]; e < M.ptr[i + 1]; ++e) {
                    c[k0[sb] + e] = (int32_t)(M.col[e] + r0[sb]);
                    v[k0[sb] + e] = M.val[e];
                }
                p[r0[sb] + i + 1] = (int32_t)(k0[sb] + M.ptr[i + 1]);
            }
        });
        A.nrows = A.ncols = n;
        A.nnz = nnz;
        A.ptr = a_mem->upload(p, s);
        A.col = a_mem->upload(c, s);
        A.val = a_mem->upload(v, s);
    }
    std::vector<Csr> &curA = local;   // host copy of every alive subdomain's current level
    double eps = sp.eps_strong;
    for (int lvl = 0;; ++lvl) {
        // layout of the alive subdomains (in subdomain order)
        std::vector<int64_t> row0(nsub, 0);
        std::vector<int32_t> nrow(nsub, 0), coarsen(nsub, 0);
        int64_t n = 0;
        int32_t nmax = 0;
        for (int sb = 0; sb < nsub; ++sb) {
            if (!alive[sb]) continue;
            row0[sb] = n;
            nrow[sb] = (int32_t)curA[sb].nrows;
            n += curA[sb].nrows;
            Level L;
            L.A = std::move(curA[sb]);
            L.eps = eps;
            out[sb].lv.push_back(std::move(L));
            coarsen[sb] = nrow[sb] > sp.coarse_enough && (int)out[sb].lv.size() < sp.max_levels;
        }
        std::vector<int32_t> subs;
        for (int sb = 0; sb < nsub; ++sb)
            if (alive[sb] && coarsen[sb]) {
                subs.push_back(sb);
                nmax = std::max(nmax, nrow[sb]);
            }
        if (subs.empty()) break;
        if (n != A.nrows) throw Error{DFAMG_EINVAL, "device setup: internal error (level layout)"};
        std::vector<int32_t> row_sub(n);
        for (int sb = 0; sb < nsub; ++sb)
            if (alive[sb])
                for (int64_t i = 0; i < nrow[sb]; ++i) row_sub[row0[sb] + i] = sb;
        Arena lv;   // device memory of this level's steps
        int32_t *d_row_sub = lv.upload(row_sub, s);
        int32_t *d_coarsen = lv.upload(coarsen, s);
        int32_t *d_nrow = lv.upload(nrow, s);
        int64_t *d_row0 = lv.upload(row0, s);
        int32_t *d_subs = lv.upload(subs, s);
        const unsigned g = grid_of(n);
        // 1. |a_ii|, m, strength, in-neighbour lists
        double *dn = lv.alloc<double>(n), *m = lv.alloc<double>(n);
        hipLaunchKernelGGL(k_su_diag, dim3(g), dim3(kSuBlock), 0, s, n, A.ptr, A.col, A.val, dn, m,
                           sp.smoother == DFAMG_SMOOTHER_JACOBI ? 1 : 0, sp.jacobi_omega);
        uint8_t *strong = lv.alloc<uint8_t>(A.nnz);
        int32_t *has = lv.alloc<int32_t>(n), *indeg = lv.alloc<int32_t>(n + 1);
        SU_CHECK(hipMemsetAsync(indeg, 0, sizeof(int32_t) * (n + 1), s));
        hipLaunchKernelGGL(k_su_strong, dim3(g), dim3(kSuBlock), 0, s, n, A.ptr, A.col, A.val, dn, d_row_sub,
                           d_coarsen, eps * eps, strong, has, indeg);
        int32_t *tptr = lv.alloc<int32_t>(n + 1);
        const int64_t tnnz = scan_counts(lv, indeg, tptr, n, s);
        int32_t *tcol = lv.alloc<int32_t>(tnnz), *tfill = lv.alloc<int32_t>(n);
        SU_CHECK(hipMemsetAsync(tfill, 0, sizeof(int32_t) * n, s));
        hipLaunchKernelGGL(k_su_tfill, dim3(g), dim3(kSuBlock), 0, s, n, A.ptr, A.col, strong, tptr, tfill, tcol);
        // 2. aggregation
        int32_t *status = lv.alloc<int32_t>(n), *agg1 = lv.alloc<int32_t>(n), *seed = lv.alloc<int32_t>(n);
        int32_t *agg = lv.alloc<int32_t>(n), *d_nagg = lv.alloc<int32_t>(nsub);
        SU_CHECK(hipMemsetAsync(d_nagg, 0, sizeof(int32_t) * nsub, s));
        hipLaunchKernelGGL(k_su_fill_i32, dim3(g), dim3(kSuBlock), 0, s, n, status, (int32_t)kNot);
        {
            // conflict lists, then the rounds
            int32_t *ccnt = lv.alloc<int32_t>(n);
            hipLaunchKernelGGL(k_su_conflicts<false>, dim3(g), dim3(kSuBlock), 0, s, n, A.ptr, A.col, strong, tptr,
                               tcol, has, ccnt, nullptr, nullptr);
            const std::vector<int32_t> cc = download(ccnt, n, s);
            std::vector<int64_t> cp(n + 1, 0);
            for (int64_t i = 0; i < n; ++i) cp[i + 1] = cp[i] + cc[i];
            int64_t *d_cptr = lv.upload(cp, s);
            int32_t *clist = lv.alloc<int32_t>(cp[n]);
            hipLaunchKernelGGL(k_su_conflicts<true>, dim3(g), dim3(kSuBlock), 0, s, n, A.ptr, A.col, strong, tptr,
                               tcol, has, nullptr, d_cptr, clist);
            if (nmax <= kStatusLds)
                hipLaunchKernelGGL(k_su_pass1<true>, dim3((unsigned)subs.size()), dim3(kAggBlock), (size_t)nmax, s,
                                   d_subs, d_row0, d_nrow, d_cptr, clist, has, status, err);
            else
                hipLaunchKernelGGL(k_su_pass1<false>, dim3((unsigned)subs.size()), dim3(kAggBlock), 0, s, d_subs,
                                   d_row0, d_nrow, d_cptr, clist, has, status, err);
        }
        hipLaunchKernelGGL(k_su_fill_i32, dim3(g), dim3(kSuBlock), 0, s, n, seed, (int32_t)-1);
        hipLaunchKernelGGL(k_su_seed_ids, dim3((unsigned)subs.size()), dim3(kAggBlock), 0, s, d_subs, d_row0,
                           d_nrow, status, seed, d_nagg);
        hipLaunchKernelGGL(k_su_fill_i32, dim3(g), dim3(kSuBlock), 0, s, n, agg1, (int32_t)-1);
        hipLaunchKernelGGL(k_su_claim, dim3(g), dim3(kSuBlock), 0, s, n, A.ptr, A.col, strong, status, seed, agg1);
        hipLaunchKernelGGL(k_su_pass2, dim3(g), dim3(kSuBlock), 0, s, n, A.ptr, A.col, A.val, strong, has,
                           d_row_sub, d_coarsen, agg1, agg, err);
        SU_CHECK(hipGetLastError());
        check_err(err, s);
        const std::vector<int32_t> nagg = download(d_nagg, nsub, s);
        // subdomains whose level stays the coarsest: no aggregate, or no reduction
        std::vector<int32_t> cont(nsub, 0), coarse_off(nsub, 0), csubs;
        int64_t nc = 0;
        for (int sb : subs)
            if (nagg[sb] > 0 && nagg[sb] < nrow[sb]) {
                cont[sb] = 1;
                coarse_off[sb] = (int32_t)nc;
                nc += nagg[sb];
                csubs.push_back(sb);
            }
        if (csubs.empty()) break;
        int32_t *d_cont = lv.upload(cont, s);
        int32_t *d_coff = lv.upload(coarse_off, s);
        int32_t *d_csubs = lv.upload(csubs, s);
        // 3. filtered diagonal, omega, smoothed prolongator
        double *D = lv.alloc<double>(n);
        int32_t *hasd = lv.alloc<int32_t>(n);
        hipLaunchKernelGGL(k_su_filtdiag, dim3(g), dim3(kSuBlock), 0, s, n, A.ptr, A.col, A.val, strong, d_row_sub,
                           d_cont, D, hasd);
        double *d_rho = lv.alloc<double>(nsub);
        int32_t *any = lv.alloc<int32_t>(nsub);
        SU_CHECK(hipMemsetAsync(any, 0, sizeof(int32_t) * nsub, s));
        hipLaunchKernelGGL(k_su_rho, dim3((unsigned)csubs.size()), dim3(kSuBlock), 0, s, d_csubs, d_row0, d_nrow,
                           A.ptr, A.col, A.val, strong, D, hasd, d_rho, any);
        const std::vector<double> rh = download(d_rho, nsub, s);
        const std::vector<int32_t> anyh = download(any, nsub, s);
        std::vector<double> omega(nsub, 0.0);
        for (int sb = 0; sb < nsub; ++sb) omega[sb] = (4.0 / 3.0) / (anyh[sb] ? rh[sb] : 1.0);
        double *d_omega = lv.upload(omega, s);
        DCsr Pm;
        Pm.nrows = n;
        Pm.ncols = nc;
        int32_t *pcnt = lv.alloc<int32_t>(n + 1);
        hipLaunchKernelGGL(k_su_prow, dim3(g), dim3(kSuBlock), 0, s, n, 0, A.ptr, A.col, A.val, strong, agg, D, hasd,
                           d_row_sub, d_cont, d_omega, d_coff, pcnt, nullptr, nullptr, nullptr, err);
        Pm.ptr = lv.alloc<int32_t>(n + 1);
        Pm.nnz = scan_counts(lv, pcnt, Pm.ptr, n, s);
        Pm.col = lv.alloc<int32_t>(Pm.nnz);
        Pm.val = lv.alloc<double>(Pm.nnz);
        hipLaunchKernelGGL(k_su_prow, dim3(g), dim3(kSuBlock), 0, s, n, 1, A.ptr, A.col, A.val, strong, agg, D, hasd,
                           d_row_sub, d_cont, d_omega, d_coff, nullptr, Pm.ptr, Pm.col, Pm.val, err);
        SU_CHECK(hipGetLastError());
        check_err(err, s);
        // R = P^T
        DCsr R;
        R.nrows = nc;
        R.ncols = n;
        int32_t *rcnt = lv.alloc<int32_t>(nc + 1), *rfill = lv.alloc<int32_t>(nc);
        SU_CHECK(hipMemsetAsync(rcnt, 0, sizeof(int32_t) * (nc + 1), s));
        SU_CHECK(hipMemsetAsync(rfill, 0, sizeof(int32_t) * nc, s));
        hipLaunchKernelGGL(k_su_colcount, dim3(grid_of(Pm.nnz)), dim3(kSuBlock), 0, s, Pm.nnz, Pm.col, rcnt);
        R.ptr = lv.alloc<int32_t>(nc + 1);
        R.nnz = scan_counts(lv, rcnt, R.ptr, nc, s);
        R.col = lv.alloc<int32_t>(R.nnz);
        R.val = lv.alloc<double>(R.nnz);
        hipLaunchKernelGGL(k_su_scatter_t, dim3(g), dim3(kSuBlock), 0, s, n, Pm.ptr, Pm.col, Pm.val, R.ptr, rfill,
                           R.col, R.val);
        hipLaunchKernelGGL(k_su_sort_rows, dim3(grid_of(nc)), dim3(kSuBlock), 0, s, nc, R.ptr, R.col, R.val);
        // 4. R A, the Galerkin product (the next level's operator, kept on the
        //    device) and the restriction operator
        const DCsr RA = spgemm(lv, R, A, err, s);
        std::unique_ptr<Arena> next_mem(new Arena);
        const DCsr Ac = spgemm(*next_mem, RA, Pm, err, s);
        DCsr Bm;
        Bm.nrows = nc;
        Bm.ncols = n;
        int32_t *bcnt = lv.alloc<int32_t>(nc + 1);
        hipLaunchKernelGGL(k_su_bmap, dim3(grid_of(nc)), dim3(kSuBlock), 0, s, nc, 0, R.ptr, R.col, R.val, RA.ptr,
                           RA.col, RA.val, m, bcnt, nullptr, nullptr, nullptr);
        Bm.ptr = lv.alloc<int32_t>(nc + 1);
        Bm.nnz = scan_counts(lv, bcnt, Bm.ptr, nc, s);
        Bm.col = lv.alloc<int32_t>(Bm.nnz);
        Bm.val = lv.alloc<double>(Bm.nnz);
        hipLaunchKernelGGL(k_su_bmap, dim3(grid_of(nc)), dim3(kSuBlock), 0, s, nc, 1, R.ptr, R.col, R.val, RA.ptr,
                           RA.col, RA.val, m, nullptr, Bm.ptr, Bm.col, Bm.val);
        SU_CHECK(hipGetLastError());
        check_err(err, s);
        // back to the per-subdomain host hierarchies
        const std::vector<int32_t> aggh = download(agg, n, s);
        const std::vector<double> mh = download(m, n, s);
        const std::vector<int32_t> pp = download(Pm.ptr, n + 1, s), pc = download(Pm.col, Pm.nnz, s);
        const std::vector<double> pv = download(Pm.val, Pm.nnz, s);
        const std::vector<int32_t> rp = download(R.ptr, nc + 1, s), rc = download(R.col, R.nnz, s);
        const std::vector<double> rv = download(R.val, R.nnz, s);
        const std::vector<int32_t> bp = download(Bm.ptr, nc + 1, s), bc = download(Bm.col, Bm.nnz, s);
        const std::vector<double> bv = download(Bm.val, Bm.nnz, s);
        const std::vector<int32_t> ap = download(Ac.ptr, nc + 1, s), ac = download(Ac.col, Ac.nnz, s);
        const std::vector<double> av = download(Ac.val, Ac.nnz, s);
        host_parallel(nsub, [&](int64_t sb) {
            if (!alive[sb] || !cont[sb]) return;
            Level &L = out[sb].lv.back();
            const int64_t r0 = row0[sb], nr = nrow[sb], c0 = coarse_off[sb], ncs = nagg[sb];
            L.agg.assign(aggh.begin() + r0, aggh.begin() + r0 + nr);
            L.nagg = (int32_t)ncs;
            L.omega = omega[sb];
            L.m.assign(mh.begin() + r0, mh.begin() + r0 + nr);
            L.P = local_block(pp, pc, pv, r0, nr, c0, ncs);
            L.R = local_block(rp, rc, rv, c0, ncs, r0, nr);
            L.B = local_block(bp, bc, bv, c0, ncs, r0, nr);
            curA[sb] = local_block(ap, ac, av, c0, ncs, c0, ncs);
        });
        for (int sb = 0; sb < nsub; ++sb)
            if (!cont[sb]) alive[sb] = 0;   // this level is the subdomain's coarsest
        A = Ac;
        a_mem = std::move(next_mem);
        eps *= 0.5;
    }
}

void build_az_device(const Csr &A, const std::vector<int32_t> &row_sub, const std::vector<double> &Z, int ndv,
                     std::vector<double> &AZown, Csr &AZoff, void *stream) {
    const hipStream_t s = static_cast<hipStream_t>(stream);
    if (ndv > 8) throw Error{DFAMG_EINVAL, "device setup: at most 8 deflation vectors"};
    const int64_t n = A.nrows;
    if (A.nnz() > INT32_MAX) throw Error{DFAMG_EINVAL, "device setup: the operator exceeds 2^31 entries"};
    Arena ar;
    int32_t *err = ar.alloc<int32_t>(1);
    SU_CHECK(hipMemsetAsync(err, 0, sizeof(int32_t), s));
    const DCsr D = upload_csr(ar, A, s);
    int32_t *d_sub = ar.upload(row_sub, s);
    double *d_Z = ar.upload(Z, s);
    double *d_own = ar.alloc<double>((size_t)n * ndv);
    int32_t *cnt = ar.alloc<int32_t>(n);
    const unsigned g = grid_of(n);
    hipLaunchKernelGGL(k_su_az<false>, dim3(g), dim3(kSuBlock), 0, s, n, D.ptr, D.col, D.val, d_sub, d_Z, ndv, d_own,
                       cnt, nullptr, nullptr, nullptr, err);
    SU_CHECK(hipGetLastError());
    check_err(err, s);
    const std::vector<int32_t> c = download(cnt, n, s);
    AZoff.nrows = n;
    AZoff.ptr.assign(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) AZoff.ptr[i + 1] = AZoff.ptr[i] + c[i];
    const int64_t nz = AZoff.ptr[n];
    int64_t *d_optr = ar.upload(AZoff.ptr, s);
    int32_t *d_ocol = ar.alloc<int32_t>(nz);
    double *d_oval = ar.alloc<double>(nz);
    hipLaunchKernelGGL(k_su_az<true>, dim3(g), dim3(kSuBlock), 0, s, n, D.ptr, D.col, D.val, d_sub, d_Z, ndv, d_own,
                       nullptr, d_optr, d_ocol, d_oval, err);
    SU_CHECK(hipGetLastError());
    check_err(err, s);
    AZown = download(d_own, (size_t)n * ndv, s);
    AZoff.col = download(d_ocol, nz, s);
    AZoff.val = download(d_oval, nz, s);
}

}  // namespace dfamg
