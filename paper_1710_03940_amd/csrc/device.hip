// Device side of the solver: uploads of the host plan with per-matrix layout
// autotuning, FP64 inversion of E and of the coarsest blocks on the GPU, the
// Krylov driver (direct launches or captured HIP graphs) and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "dfamg.h"
#include "dense_inverse.hpp"
#include "devmat.hpp"
#include "host_plan.hpp"
#include "kernels.hpp"
#include "kernels_fgmres.hpp"
#include "kernels_schur.hpp"
#include "kernels_bsmooth.hpp"
#include "kernels_coarse_setup.hpp"

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

// Owns device allocations.
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
        if (!v.empty()) {
            // sources are often temporaries: complete the copy before returning
            HIP_CHECK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
            HIP_CHECK(hipStreamSynchronize(s));
        }
        return p;
    }
    void adopt(DevArena &o) {
        ptrs.insert(ptrs.end(), o.ptrs.begin(), o.ptrs.end());
        bytes += o.bytes;
        o.ptrs.clear();
        o.bytes = 0;
    }
    ~DevArena() {
        for (void *p : ptrs) (void)hipFree(p);
    }
};

}  // namespace

// Compile-time bound on the deflation vectors per subdomain: kernels unroll
// their Z / AZ loops to the bound (0, 1, 4 or 8) and skip the terms beyond
// the run-time count.
template <int N>
struct NdvC {
    static constexpr int value = N;
};

template <class Fn>
void with_ndv(int ndv, Fn &&fn) {
    if (ndv == 0) fn(NdvC<0>{});
    else if (ndv == 1) fn(NdvC<1>{});
    else if (ndv <= 4) fn(NdvC<4>{});
    else if (ndv <= kMaxNdv) fn(NdvC<kMaxNdv>{});
    else throw Error{DFAMG_EINVAL, "ndv out of range"};
}

namespace {

std::vector<DevTile> to_dev_tiles(const std::vector<Tile> &t) {
    std::vector<DevTile> d(t.size());
    for (size_t i = 0; i < t.size(); ++i) d[i] = DevTile{t[i].row0, t[i].nrows, t[i].sub, (int32_t)i};
    return d;
}

void tile_offsets(const std::vector<Tile> &tiles, const std::vector<int32_t> &sub_sys, int nsys, int nsub,
                  std::vector<int32_t> &sys_off, std::vector<int32_t> &sub_off) {
    sys_off.assign(nsys + 1, 0);
    sub_off.assign(nsub + 1, 0);
    for (const Tile &t : tiles) {
        sys_off[sub_sys[t.sub] + 1]++;
        sub_off[t.sub + 1]++;
    }
    for (int i = 0; i < nsys; ++i) sys_off[i + 1] += sys_off[i];
    for (int i = 0; i < nsub; ++i) sub_off[i + 1] += sub_off[i];
}

// Host form of a layout: SELL (rows per lane, row order, column width) or
// CSR (lanes per row, rows per tile).  A staged and an unstaged candidate of
// the same structure share one host form.
// BSR4 host form: tiles of 256 rows, block-row pointers over the whole
// matrix, block columns (ascending in a block row), 16 values per block.
struct HostBsr {
    std::vector<Tile> tiles;
    std::vector<int32_t> bptr, bcol;
    std::vector<double> val;
    int64_t nnz = 0;
};

// The matrix in 4 x 4 blocks; false when its rows, columns or row ranges do
// not fall on multiples of 4, or the blocks exceed 32-bit offsets.
bool make_bsr4(const Csr &M, const std::vector<RowRange> &ranges, HostBsr &B) {
    if (M.nrows % 4 || M.ncols % 4) return false;
    for (const RowRange &rg : ranges)
        if (rg.row0 % 4 || rg.nrows % 4) return false;
    const int64_t nbr = M.nrows / 4;
    std::vector<int32_t> cnt(nbr, 0);
    parallel_for(nbr, 8, [&](int64_t I) {
        std::vector<int32_t> js;
        for (int64_t i = 4 * I; i < 4 * I + 4; ++i)
            for (int64_t k = M.ptr[i]; k < M.ptr[i + 1]; ++k) js.push_back(M.col[k] / 4);
        std::sort(js.begin(), js.end());
        cnt[I] = (int32_t)(std::unique(js.begin(), js.end()) - js.begin());
    });
    B.bptr.assign(nbr + 1, 0);
    for (int64_t I = 0; I < nbr; ++I) {
        if ((int64_t)B.bptr[I] + cnt[I] > INT32_MAX / 16) return false;
        B.bptr[I + 1] = B.bptr[I] + cnt[I];
    }
    B.bcol.assign(B.bptr[nbr], 0);
    B.val.assign((size_t)B.bptr[nbr] * 16, 0.0);
    parallel_for(nbr, 8, [&](int64_t I) {
        std::vector<int32_t> js;
        for (int64_t i = 4 * I; i < 4 * I + 4; ++i)
            for (int64_t k = M.ptr[i]; k < M.ptr[i + 1]; ++k) js.push_back(M.col[k] / 4);
        std::sort(js.begin(), js.end());
        js.erase(std::unique(js.begin(), js.end()), js.end());
        const int32_t b0 = B.bptr[I];
        for (size_t q = 0; q < js.size(); ++q) B.bcol[b0 + q] = js[q];
        for (int64_t i = 4 * I; i < 4 * I + 4; ++i)
            for (int64_t k = M.ptr[i]; k < M.ptr[i + 1]; ++k) {
                const int32_t J = M.col[k] / 4;
                const int64_t b = b0 + (std::lower_bound(js.begin(), js.end(), J) - js.begin());
                B.val[(size_t)b * 16 + (i % 4) * 4 + M.col[k] % 4] = M.val[k];
            }
    });
    for (const RowRange &rg : ranges) {
        int32_t slot = rg.slot0;
        for (int32_t r0 = 0; r0 < rg.nrows; r0 += kBlock)
            B.tiles.push_back(Tile{(int32_t)(rg.row0 + r0), std::min(kBlock, rg.nrows - r0), rg.sub, slot++});
    }
    B.nnz = M.nnz();
    return true;
}

// Host form of the column-tiled layout (SegM): every range's columns (the
// columns its rows touch) cut into tiles of `ct` columns; a row's entries in
// one tile form a segment (a new segment starts wherever the tile of the next
// entry differs, so the split holds for rows in any column order).
struct HostSeg {
    std::vector<Tile> ctiles;       // column tiles (row0 = first column, nrows = width)
    std::vector<int32_t> slices;    // [ctiles + 1]
    std::vector<int64_t> soff;      // per slice
    std::vector<int32_t> sw;        // per slice
    std::vector<uint16_t> col16;
    std::vector<double> val;
    std::vector<int32_t> slot;      // 64 per slice
    std::vector<int32_t> pp;        // [nrows + 1]: partials of each row
    std::vector<Tile> rtiles;       // 256-row tiles of the ranges, for the combine step
    int64_t nnz = 0;
    int32_t widest = 1;             // widest column tile
};

bool make_seg(const Csr &M, const std::vector<RowRange> &ranges, int ct, HostSeg &S) {
    if (ct < 64 || ct > 65536 || M.nrows > INT32_MAX) return false;
    const int nr = (int)ranges.size();
    // pass 1: segments per row
    std::vector<int32_t> cnt(M.nrows, 0);
    std::vector<int32_t> fmin(nr, 0), ntile(nr, 0);
    parallel_for(nr, 8, [&](int64_t r) {
        const RowRange &rg = ranges[r];
        int32_t lo = INT32_MAX, hi = -1;
        for (int64_t k = M.ptr[rg.row0]; k < M.ptr[rg.row0 + rg.nrows]; ++k) {
            lo = std::min(lo, M.col[k]);
            hi = std::max(hi, M.col[k]);
        }
        if (hi < 0) return;
        fmin[r] = lo;
        ntile[r] = (hi - lo) / ct + 1;
        for (int64_t i = rg.row0; i < rg.row0 + rg.nrows; ++i) {
            int last = -1;
            for (int64_t k = M.ptr[i]; k < M.ptr[i + 1]; ++k) {
                const int t = (M.col[k] - lo) / ct;
                if (t != last) ++cnt[i];
                last = t;
            }
        }
    });
    S.pp.assign(M.nrows + 1, 0);
    for (int64_t i = 0; i < M.nrows; ++i) {
        if ((int64_t)S.pp[i] + cnt[i] > INT32_MAX) return false;
        S.pp[i + 1] = S.pp[i] + cnt[i];
    }
    // pass 2: every range's tiles and slices (offsets local to the range)
    struct Part {
        std::vector<Tile> ct;
        std::vector<int32_t> first_slice;
        std::vector<int64_t> soff;
        std::vector<int32_t> sw, slot;
        std::vector<uint16_t> col16;
        std::vector<double> val;
    };
    std::vector<Part> parts(nr);
    parallel_for(nr, 8, [&](int64_t r) {
        const RowRange &rg = ranges[r];
        Part &P = parts[r];
        const int nt = ntile[r];
        struct Segm {
            int32_t len, row;
            int64_t k0;
            int32_t slot;
        };
        std::vector<std::vector<Segm>> per(nt);
        for (int64_t i = rg.row0; i < rg.row0 + rg.nrows; ++i) {
            int32_t rank = 0;
            int64_t k = M.ptr[i];
            while (k < M.ptr[i + 1]) {
                const int t = (M.col[k] - fmin[r]) / ct;
                int64_t e = k;
                while (e < M.ptr[i + 1] && (M.col[e] - fmin[r]) / ct == t) ++e;
                per[t].push_back(Segm{(int32_t)(e - k), (int32_t)i, k, S.pp[i] + rank++});
                k = e;
            }
        }
        int64_t stored = 0;
        for (int t = 0; t < nt; ++t) {
            auto &sg = per[t];
            std::stable_sort(sg.begin(), sg.end(), [](const Segm &a, const Segm &b) { return a.len > b.len; });
            const int32_t c0 = fmin[r] + t * ct;
            P.ct.push_back(Tile{c0, 0, rg.sub, 0});
            P.first_slice.push_back((int32_t)P.sw.size());
            int32_t cmax = c0;
            for (size_t s0 = 0; s0 < sg.size(); s0 += 64) {
                const int32_t w = sg[s0].len;
                P.soff.push_back(stored);
                P.sw.push_back(w);
                P.val.resize((size_t)(stored + (int64_t)w * 64), 0.0);
                P.col16.resize((size_t)(stored + (int64_t)w * 64), 0);
                for (int l = 0; l < 64; ++l) {
                    if (s0 + l >= sg.size()) {
                        P.slot.push_back(-1);
                        continue;
                    }
                    const Segm &q = sg[s0 + l];
                    P.slot.push_back(q.slot);
                    for (int32_t e = 0; e < q.len; ++e) {
                        const int32_t c = M.col[q.k0 + e];
                        P.val[(size_t)(stored + (int64_t)e * 64 + l)] = M.val[q.k0 + e];
                        P.col16[(size_t)(stored + (int64_t)e * 64 + l)] = (uint16_t)(c - c0);
                        cmax = std::max(cmax, c);
                    }
                }
                stored += (int64_t)w * 64;
            }
            P.ct.back().nrows = cmax - c0 + 1;
        }
    });
    // pass 3: concatenation
    int64_t stored = 0;
    for (int r = 0; r < nr; ++r) {
        Part &P = parts[r];
        const int32_t sbase = (int32_t)S.sw.size();
        for (size_t t = 0; t < P.ct.size(); ++t) {
            S.ctiles.push_back(P.ct[t]);
            S.slices.push_back(sbase + P.first_slice[t]);
            S.widest = std::max(S.widest, P.ct[t].nrows);
        }
        for (int64_t o : P.soff) S.soff.push_back(stored + o);
        S.sw.insert(S.sw.end(), P.sw.begin(), P.sw.end());
        S.slot.insert(S.slot.end(), P.slot.begin(), P.slot.end());
        S.col16.insert(S.col16.end(), P.col16.begin(), P.col16.end());
        S.val.insert(S.val.end(), P.val.begin(), P.val.end());
        stored += (int64_t)P.val.size();
        const RowRange &rg = ranges[r];
        for (int32_t r0 = 0; r0 < rg.nrows; r0 += kBlock)
            S.rtiles.push_back(Tile{(int32_t)(rg.row0 + r0), std::min(kBlock, rg.nrows - r0), rg.sub, 0});
        P = Part{};
    }
    S.slices.push_back((int32_t)S.sw.size());
    S.nnz = M.nnz();
    return !S.ctiles.empty();
}

struct HostLayout {
    int fmt = DFAMG_FORMAT_SELL;
    bool ok = false;          // false: 16-bit columns requested but do not fit, or no 4 x 4 blocks
    HostSell S;
    HostCsrv C;
    HostBsr Bs;
    HostSeg G;
};

struct HostKey {
    int fmt, par, sorted, idx16, tile_rows;
    bool operator<(const HostKey &o) const {
        return std::tie(fmt, par, sorted, idx16, tile_rows) < std::tie(o.fmt, o.par, o.sorted, o.idx16, o.tile_rows);
    }
};

inline int csr_tile_rows_of(const Layout &L) { return L.rpg > 0 ? L.rpg * (kBlock / L.par) : kBlock; }

HostKey host_key(const Layout &L) {
    if (L.fmt == DFAMG_FORMAT_BSR4) return HostKey{L.fmt, 4, 0, 0, kBlock};
    if (L.fmt == kFormatSeg) return HostKey{L.fmt, L.par, 0, 0, 0};
    if (L.fmt == DFAMG_FORMAT_SELL) return HostKey{L.fmt, L.par, L.sorted ? 1 : 0, (L.idx16 || L.stage) ? 1 : 0, 0};
    return HostKey{L.fmt, L.par, 0, 0, csr_tile_rows_of(L)};
}

void build_host_layout(const Csr &M, const std::vector<RowRange> &ranges, const HostKey &k, HostLayout &H) {
    H.fmt = k.fmt;
    if (k.fmt == DFAMG_FORMAT_BSR4) {
        H.ok = make_bsr4(M, ranges, H.Bs);
    } else if (k.fmt == kFormatSeg) {
        H.ok = make_seg(M, ranges, k.par, H.G);
    } else if (k.fmt == DFAMG_FORMAT_SELL) {
        H.ok = make_sell(M, ranges, k.par, k.sorted != 0, k.idx16 != 0, H.S);
    } else {
        H.C = make_csrv(M, ranges, k.par, k.tile_rows);
        H.ok = true;
    }
}

// Gather lists of a CSR host form (see CsrM): per tile its distinct columns
// in ascending order, and every entry's position among them.  They depend
// only on the tiles, so CSR forms with the same tile height share them.
struct GatherLists {
    std::vector<int32_t> uoff, ucol, lcol;
    size_t longest = 0;
};

GatherLists make_gather_lists(const HostCsrv &C) {
    const size_t nt = C.tiles.size();
    std::vector<std::vector<int32_t>> lists(nt);
    GatherLists G;
    G.lcol.resize(C.col.size());
    parallel_for((int64_t)nt, 8, [&](int64_t ti) {
        const Tile &t = C.tiles[ti];
        const int32_t k0 = C.ptr[t.row0], k1 = C.ptr[t.row0 + t.nrows];
        std::vector<int32_t> &u = lists[ti];
        u.assign(C.col.begin() + k0, C.col.begin() + k1);
        std::sort(u.begin(), u.end());
        u.erase(std::unique(u.begin(), u.end()), u.end());
        for (int32_t k = k0; k < k1; ++k)
            G.lcol[k] = (int32_t)(std::lower_bound(u.begin(), u.end(), C.col[k]) - u.begin());
    });
    G.uoff.assign(nt + 1, 0);
    G.longest = 1;
    for (size_t ti = 0; ti < nt; ++ti) {
        G.uoff[ti + 1] = G.uoff[ti] + (int32_t)lists[ti].size();
        G.longest = std::max(G.longest, lists[ti].size());
    }
    G.ucol.reserve((size_t)G.uoff[nt]);
    for (auto &u : lists) G.ucol.insert(G.ucol.end(), u.begin(), u.end());
    return G;
}

// Uploads the host form H as layout L; returns false (nothing kept) when the
// layout cannot hold the matrix: 16-bit offsets that do not fit, or a staged
// column window or gather list larger than the LDS budget.  gl_cache (may be
// null) keeps the gather lists by tile height for the other candidates of
// the same matrix.
template <class VT>
bool upload_built(DevArena &ar, const HostLayout &H, const Layout &L, hipStream_t s,
                  const std::vector<int32_t> &sub_sys, int nsys, int nsub, DevMat<VT> &D,
                  size_t stage_limit = kMaxStageBytes, std::map<int, GatherLists> *gl_cache = nullptr) {
    if (!H.ok) return false;
    D = DevMat<VT>{};
    D.fmt = L.fmt;
    D.par = L.par;
    std::vector<Tile> tiles;
    if (L.fmt == kFormatSeg) {
        const HostSeg &G = H.G;
        if ((size_t)G.widest * sizeof(VT) > stage_limit) return false;
        tiles = G.ctiles;
        D.stage = true;
        D.max_span = G.widest;
        D.seg_slices = ar.upload(G.slices, s);
        D.soff = ar.upload(G.soff, s);
        D.sw = ar.upload(G.sw, s);
        D.col16 = ar.upload(G.col16, s);
        std::vector<VT> v(G.val.size());
        for (size_t i = 0; i < v.size(); ++i) v[i] = (VT)G.val[i];
        D.val = ar.upload(v, s);
        D.seg_slot = ar.upload(G.slot, s);
        D.seg_pp = ar.upload(G.pp, s);
        D.seg_rtiles = ar.upload(to_dev_tiles(G.rtiles), s);
        D.seg_nrt = (int32_t)G.rtiles.size();
        D.seg_part = ar.alloc<VT>(std::max<int64_t>(1, G.pp.back()));
        D.seg_nt = L.rpg == 4 ? 1024 : L.rpg == 2 ? 512 : 256;
        D.nnz = G.nnz;
        D.stored = (int64_t)G.val.size();
    } else if (L.fmt == DFAMG_FORMAT_BSR4) {
        const HostBsr &B = H.Bs;
        tiles = B.tiles;
        D.ptr = ar.upload(B.bptr, s);
        D.col = ar.upload(B.bcol, s);
        std::vector<VT> v(B.val.size());
        for (size_t i = 0; i < v.size(); ++i) v[i] = (VT)B.val[i];
        D.val = ar.upload(v, s);
        D.nnz = B.nnz;
        D.stored = (int64_t)B.val.size();
    } else if (L.fmt == DFAMG_FORMAT_SELL) {
        const HostSell &S = H.S;
        if (L.stage) {
            const int32_t mx = S.cspan.empty() ? 1 : *std::max_element(S.cspan.begin(), S.cspan.end());
            if ((size_t)mx * sizeof(VT) > stage_limit) return false;
            D.max_span = mx;
        }
        D.sorted = L.sorted;
        D.idx16 = L.idx16 || L.stage;
        D.stage = L.stage;
        tiles = S.tiles;
        D.soff = ar.upload(S.slice_off, s);
        D.sw = ar.upload(S.slice_w, s);
        if (D.idx16) {
            D.col16 = ar.upload(S.col16, s);
            D.cbase = ar.upload(S.cbase, s);
            D.cspan = ar.upload(S.cspan, s);
        } else {
            D.col = ar.upload(S.col, s);
        }
        if (L.sorted) D.ridx = ar.upload(S.ridx, s);
        std::vector<VT> v(S.val.size());
        for (size_t i = 0; i < v.size(); ++i) v[i] = (VT)S.val[i];
        D.val = ar.upload(v, s);
        D.nnz = S.nnz;
        D.stored = (int64_t)S.val.size();
    } else {
        const HostCsrv &C = H.C;
        if (L.stage && L.glist) {
            GatherLists own;
            const GatherLists *G = nullptr;
            if (gl_cache) {
                // keyed by the nominal tile height (equal heights give equal tiles)
                const int th = csr_tile_rows_of(L);
                auto it = gl_cache->find(th);
                if (it == gl_cache->end()) it = gl_cache->emplace(th, make_gather_lists(C)).first;
                G = &it->second;
            }
            if (!G || G->uoff.size() != C.tiles.size() + 1 || G->lcol.size() != C.col.size()) {
                own = make_gather_lists(C);
                G = &own;
            }
            // positions within a list are 16-bit: the LDS budget keeps every
            // list far below 65536 entries
            if (G->longest * sizeof(VT) > stage_limit || G->longest > 65536) return false;
            D.max_span = (int32_t)G->longest;
            D.stage = true;
            tiles = C.tiles;
            D.ptr = ar.upload(C.ptr, s);
            std::vector<uint16_t> l16(G->lcol.begin(), G->lcol.end());
            D.col16 = ar.upload(l16, s);
            D.uoff = ar.upload(G->uoff, s);
            D.ucol = ar.upload(G->ucol, s);
            std::vector<VT> v(C.val.size());
            for (size_t i = 0; i < v.size(); ++i) v[i] = (VT)C.val[i];
            D.val = ar.upload(v, s);
            D.nnz = C.nnz;
            D.stored = C.nnz;
            D.host_tiles = to_dev_tiles(tiles);
            D.tiles = ar.upload(D.host_tiles, s);
            D.ntiles = (int32_t)tiles.size();
            tile_offsets(tiles, sub_sys, nsys, nsub, D.sys_tile_off, D.sub_tile_off);
            return true;
        }
        if (L.stage) {
            const int32_t mx = C.cspan.empty() ? 1 : *std::max_element(C.cspan.begin(), C.cspan.end());
            if ((size_t)mx * sizeof(VT) > stage_limit) return false;
            D.max_span = mx;
            D.stage = true;
        }
        tiles = C.tiles;
        D.ptr = ar.upload(C.ptr, s);
        D.col = ar.upload(C.col, s);
        D.cbase = ar.upload(C.cbase, s);
        D.cspan = ar.upload(C.cspan, s);
        std::vector<VT> v(C.val.size());
        for (size_t i = 0; i < v.size(); ++i) v[i] = (VT)C.val[i];
        D.val = ar.upload(v, s);
        D.nnz = C.nnz;
        D.stored = C.nnz;
    }
    D.host_tiles = to_dev_tiles(tiles);
    D.tiles = ar.upload(D.host_tiles, s);
    D.ntiles = (int32_t)tiles.size();
    tile_offsets(tiles, sub_sys, nsys, nsub, D.sys_tile_off, D.sub_tile_off);
    return true;
}

template <class VT>
std::string describe(const DevMat<VT> &D);

// What a matrix is used for, and so which kernel times its candidates.
enum TuneKind { TUNE_OUTER, TUNE_SMOOTH, TUNE_RESTRICT, TUNE_PROLONG };

template <class VT>
void launch_for_tuning(TuneKind kind, const DevMat<VT> &M, const VT *x, VT *y, hipStream_t s);

template <>
void launch_for_tuning<double>(TuneKind kind, const DevMat<double> &M, const double *x, double *y, hipStream_t s) {
    switch (kind) {
        case TUNE_OUTER: launch_outer_spmv_plain(M, x, y, s); break;
        case TUNE_SMOOTH: launch_pre_res<double, double>(M, x, x, y, nullptr, nullptr, s); break;
        case TUNE_RESTRICT: launch_spmv<double>(M, x, y, nullptr, nullptr, s); break;
        case TUNE_PROLONG: launch_prolong<double, double>(M, x, y, x, y, nullptr, nullptr, s); break;
    }
}

template <>
void launch_for_tuning<float>(TuneKind kind, const DevMat<float> &M, const float *x, float *y, hipStream_t s) {
    switch (kind) {
        case TUNE_OUTER:
        case TUNE_RESTRICT: launch_spmv<float>(M, x, y, nullptr, nullptr, s); break;
        case TUNE_SMOOTH: launch_pre_res<float, float>(M, x, x, y, nullptr, nullptr, s); break;
        case TUNE_PROLONG: launch_prolong<float, float>(M, x, y, x, y, nullptr, nullptr, s); break;
    }
}

// Microseconds per call of `launch` (2 untimed calls, then 8 timed).
template <class F>
double time_launches(F &&launch, hipStream_t s) {
    hipEvent_t e0, e1;
    HIP_CHECK(hipEventCreate(&e0));
    HIP_CHECK(hipEventCreate(&e1));
    for (int i = 0; i < 2; ++i) launch();
    // a launch the runtime refuses never wins the comparison
    if (hipGetLastError() != hipSuccess) {
        HIP_CHECK(hipStreamSynchronize(s));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return 1e30;
    }
    const int reps = 8;
    HIP_CHECK(hipEventRecord(e0, s));
    for (int i = 0; i < reps; ++i) launch();
    HIP_CHECK(hipEventRecord(e1, s));
    HIP_CHECK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms * 1e3 / reps;
}

// Microseconds per launch of the kernel that will use M.
template <class VT>
double time_layout(TuneKind kind, const DevMat<VT> &M, const VT *x, VT *y, hipStream_t s) {
    return time_launches([&] { launch_for_tuning(kind, M, x, y, s); }, s);
}

// Layout of one matrix: the fastest candidate of the family `format` (SELL,
// CSR, or both with DFAMG_FORMAT_AUTO), timed on the device with the kernel
// that will use the matrix.  SELL candidates: 1 or 2 rows per lane (2 only
// while the tiles still fill the chip), natural or length-sorted rows,
// 16-bit column offsets (32-bit when they do not fit), with or without an LDS
// stage of the gathered vector; CSR: 4, 8 or 16 lanes per row, staged or
// not, for rows of 10+ entries.  The block-diagonal part of the global
// operator also tries 4 rows per lane and only 256-row CSR tiles.
// Process-wide record of tuned layouts.  When the environment variable
// DFAMG_TUNE_CACHE names a file, the record also persists across processes:
// it is read from that file on first use and every newly tuned matrix is
// appended to it, one line per matrix:
//   kind value-bytes format structure-hash  fmt par sorted idx16 stage rpg glist  microseconds
// A matrix found there takes the stored layout without timing, so that the
// choice (and hence every dispatch) is the same from one process to the next.
struct TuneKey {
    int kind, vt, format;
    uint64_t hash;
    bool operator<(const TuneKey &o) const {
        return std::tie(kind, vt, format, hash) < std::tie(o.kind, o.vt, o.format, o.hash);
    }
};
constexpr const char *kTuneFileTag = "# dfamg tuned layouts v1";

const char *tune_file() {
    const char *f = std::getenv("DFAMG_TUNE_CACHE");
    return (f && *f) ? f : nullptr;
}

// Callers hold tune_cache_mutex().
std::map<TuneKey, std::pair<Layout, double>> &tune_cache() {
    static std::map<TuneKey, std::pair<Layout, double>> c;
    static bool loaded = false;
    if (!loaded) {
        loaded = true;
        if (const char *path = tune_file())
            if (FILE *fp = std::fopen(path, "r")) {
                char line[512];
                while (std::fgets(line, sizeof line, fp)) {
                    if (line[0] == '#') continue;
                    TuneKey k{};
                    Layout L{};
                    unsigned long long h = 0;
                    int so = 0, i16 = 0, st = 0, gl = 0;
                    double us = 0.0;
                    if (std::sscanf(line, "%d %d %d %llx %d %d %d %d %d %d %d %lf", &k.kind, &k.vt, &k.format, &h,
                                    &L.fmt, &L.par, &so, &i16, &st, &L.rpg, &gl, &us) != 12)
                        continue;
                    k.hash = h;
                    L.sorted = so != 0;
                    L.idx16 = i16 != 0;
                    L.stage = st != 0;
                    L.glist = gl != 0;
                    c[k] = {L, us};
                }
                std::fclose(fp);
            }
    }
    return c;
}
std::mutex &tune_cache_mutex() {
    static std::mutex m;
    return m;
}

// Callers hold tune_cache_mutex().
void tune_cache_store(const TuneKey &k, const Layout &L, double us) {
    tune_cache()[k] = {L, us};
    const char *path = tune_file();
    if (!path) return;
    FILE *fp = std::fopen(path, "a+");
    if (!fp) return;   // an unwritable record only costs the timing next time
    std::fseek(fp, 0, SEEK_END);
    if (std::ftell(fp) == 0) std::fprintf(fp, "%s\n", kTuneFileTag);
    std::fprintf(fp, "%d %d %d %llx %d %d %d %d %d %d %d %.3f\n", k.kind, k.vt, k.format, (unsigned long long)k.hash,
                 L.fmt, L.par, (int)L.sorted, (int)L.idx16, (int)L.stage, L.rpg, (int)L.glist, us);
    std::fclose(fp);
}

// Hash of the row ranges, row lengths and columns of the rows covered
// (64-bit multiply-xorshift per word).
// Hash of a matrix's structure over the row ranges: each range hashed on
// its own (in parallel), the range hashes then combined in order.
uint64_t structure_hash(const Csr &M, const std::vector<RowRange> &ranges) {
    auto mix = [](uint64_t &h, uint64_t v) {
        h = (h ^ v) * 0x9e3779b97f4a7c15ull;
        h ^= h >> 29;
    };
    std::vector<uint64_t> rh(ranges.size());
    parallel_for((int64_t)ranges.size(), 8, [&](int64_t j) {
        const RowRange &r = ranges[j];
        uint64_t h = 1469598103934665603ull;
        mix(h, (uint64_t)r.row0);
        mix(h, (uint64_t)r.nrows);
        for (int64_t i = r.row0; i < r.row0 + r.nrows; ++i) {
            mix(h, (uint64_t)(M.ptr[i + 1] - M.ptr[i]));
            for (int64_t k = M.ptr[i]; k < M.ptr[i + 1]; ++k) mix(h, (uint64_t)(uint32_t)M.col[k]);
        }
        rh[j] = h;
    });
    uint64_t h = 1469598103934665603ull;
    mix(h, (uint64_t)M.nrows);
    mix(h, (uint64_t)M.ncols);
    for (uint64_t v : rh) mix(h, v);
    return h;
}

// The time recorded for a matrix of this kind, value type, family and
// structure (tuned before in this process, or read from the layout record),
// or -1.
template <class VT>
double recorded_us(int kind, int format, uint64_t hash) {
    std::lock_guard<std::mutex> g(tune_cache_mutex());
    auto it = tune_cache().find(TuneKey{kind, (int)sizeof(VT), format, hash});
    return it == tune_cache().end() ? -1.0 : it->second.second;
}

// `timer` (optional) replaces the default timing of a candidate; `verbose`
// above 1 prints every candidate's time.
template <class VT>
DevMat<VT> upload_tuned(DevArena &ar, const Csr &M, const std::vector<RowRange> &ranges, int format,
                        bool autotune, TuneKind kind, hipStream_t s, const std::vector<int32_t> &sub_sys, int nsys,
                        int nsub, const std::function<double(const DevMat<VT> &)> &timer = {}, int verbose = 0,
                        bool bsr4 = false, uint64_t hash = 0) {
    int64_t rows = 0;
    for (auto &r : ranges) rows += r.nrows;
    const double avg_len = rows ? (double)M.nnz() / (double)rows : 0.0;
    std::vector<Layout> cand;
    const bool outer = kind == TUNE_OUTER;
    // CSR_GATHER: the CSR family, with the multigrid operators staged from
    // gather lists only (the outer operator as plain CSR)
    const bool gather = format == DFAMG_FORMAT_CSR_GATHER;
    const int family = gather ? DFAMG_FORMAT_CSR : format;
    if (family == DFAMG_FORMAT_BSR4) {
        cand.push_back(Layout{DFAMG_FORMAT_BSR4, 4, false, false, false, 0});
    } else if (family == DFAMG_FORMAT_COLUMN_TILED) {
        // restrictions in column tiles of 512 unknowns (256 threads), the
        // other operators in SELL; nothing timed
        cand.push_back(kind == TUNE_RESTRICT ? Layout{kFormatSeg, 512, false, false, true, 1}
                                             : Layout{DFAMG_FORMAT_SELL, 1, false, false, false, 0});
    } else if (!autotune) {
        if (gather && !outer) {
            Layout c{DFAMG_FORMAT_CSR, 8, false, false, true, 0};
            c.glist = true;
            cand.push_back(c);
        } else {
            cand.push_back(family == DFAMG_FORMAT_CSR ? Layout{DFAMG_FORMAT_CSR, 8, false, false, false, 0}
                                                      : Layout{DFAMG_FORMAT_SELL, 1, false, false, false, 0});
        }
    } else {
        if (family == DFAMG_FORMAT_SELL || family == DFAMG_FORMAT_AUTO) {
            for (int r : outer ? std::vector<int>{1, 2, 4} : std::vector<int>{1, 2}) {
                if (r > 1 && rows / (256 * r) < 512) continue;
                for (bool sorted : {false, true}) {
                    cand.push_back(Layout{DFAMG_FORMAT_SELL, r, sorted, true, false, 0});
                    if (r <= 2) cand.push_back(Layout{DFAMG_FORMAT_SELL, r, sorted, true, true, 0});
                }
            }
        }
        // 4 x 4 blocks for point-block operators
        if (family == DFAMG_FORMAT_AUTO && bsr4) cand.push_back(Layout{DFAMG_FORMAT_BSR4, 4, false, false, false, 0});
        // restrictions split by column tiles of 4 to 64 KB of the input
        // vector (rows of 16+ entries)
        if (family == DFAMG_FORMAT_AUTO && kind == TUNE_RESTRICT && avg_len >= 16.0)
            for (int kb : {4, 8, 16, 32, 64})
                for (int nt : {1, 2, 4})
                    cand.push_back(Layout{kFormatSeg, kb * 1024 / (int)sizeof(VT), false, false, true, nt});
        // lanes per row: 32 and 64 for the long rows of the restrictions
        // (tens to hundreds of entries) and of the denser coarse operators,
        // 1, 2 and 4 for rows of fewer than ten
        const bool short_rows = avg_len < 10.0;
        const std::vector<int> lane_set = short_rows              ? std::vector<int>{1, 2, 4}
                                          : outer                 ? std::vector<int>{8, 16}
                                          : kind == TUNE_RESTRICT ? std::vector<int>{8, 16, 32, 64}
                                          : avg_len >= 24.0       ? std::vector<int>{4, 8, 16, 32}
                                                                  : std::vector<int>{4, 8, 16};
        if (family == DFAMG_FORMAT_CSR || family == DFAMG_FORMAT_AUTO)
            for (int l : lane_set)
                // 256-row tiles, and tiles of 4/16/64 rows (64 lanes), 8/16/64
                // rows (32 lanes) or of kBlock/l and 4 kBlock/l rows (fewer lanes)
                for (int rpg : l == 64 ? std::vector<int>{0, 1, 4, 16} : l == 32 ? std::vector<int>{0, 1, 2, 8}
                                                                                   : std::vector<int>{0, 1, 4}) {
                    // smaller tiles where 256-row tiles leave the chip idle, and
                    // for restrictions (long rows gathering from a wide window)
                    if (rpg > 0 && (outer || (rows / 256 >= 2048 && kind != TUNE_RESTRICT))) continue;
                    // unstaged, staged window, staged gather list (for the
                    // restrictions, whose rows read the most scattered
                    // columns; every multigrid operator with CSR_GATHER)
                    const int nsv = outer ? 2 : (gather || kind == TUNE_RESTRICT) ? 3 : 2;
                    for (int sv = 0; sv < nsv; ++sv) {
                        if (gather && !outer && sv != 2) continue;
                        Layout c{DFAMG_FORMAT_CSR, l, false, false, sv > 0, rpg};
                        c.glist = sv == 2;
                        // rpg values that give the same tile are one candidate
                        bool dup = false;
                        for (const Layout &o : cand)
                            dup |= o.fmt == c.fmt && o.par == c.par && o.stage == c.stage && o.glist == c.glist &&
                                   csr_tile_rows_of(o) == csr_tile_rows_of(c);
                        if (!dup) cand.push_back(c);
                    }
                }
    }
    // a matrix tuned before in this process (same kind, value type, family and
    // structure) gets the layout chosen then, without timing
    const TuneKey key{(int)kind, (int)sizeof(VT), format, hash ? hash : structure_hash(M, ranges)};
    double cached_us = -1.0;
    // (DFAMG_TUNE_VERIFY, below, times and checks every candidate anew)
    if (cand.size() > 1 && std::getenv("DFAMG_TUNE_VERIFY") == nullptr) {
        std::lock_guard<std::mutex> g(tune_cache_mutex());
        auto it = tune_cache().find(key);
        if (it != tune_cache().end()) {
            cand.assign(1, it->second.first);
            cached_us = it->second.second;
        }
    }
    DevArena scratch;
    VT *x = scratch.alloc<VT>(std::max<int64_t>(1, std::max(M.ncols, M.nrows)));
    VT *y = scratch.alloc<VT>(std::max<int64_t>(1, std::max(M.ncols, M.nrows)));
    // With the environment variable DFAMG_TUNE_VERIFY set, every candidate
    // is first applied once to the same varied input (entries in [1, 2)) and
    // its output compared with the first candidate's: a layout that differs
    // by more than rounding is an error, not a slower choice.  The bound is
    // relative to the largest row sum of |entries| times the input's bound.
    const bool verify = cand.size() > 1 && cached_us < 0.0 && std::getenv("DFAMG_TUNE_VERIFY") != nullptr;
    std::vector<VT> yref;
    std::string ref_name;
    double vbound = 0.0;
    if (cand.size() > 1) {
        std::vector<VT> xin(std::max<int64_t>(1, std::max(M.ncols, M.nrows)), (VT)1);
        if (verify) {
            for (size_t i = 0; i < xin.size(); ++i) xin[i] = (VT)(1.0 + (double)((i * 7919) % 1013) / 1013.0);
            // smoothing: f - A (m o f) with m = f = x, so |entries| x 4 plus 2
            for (int64_t r = 0; r < M.nrows; ++r) {
                double a = 0.0;
                for (int64_t k = M.ptr[r]; k < M.ptr[r + 1]; ++k) a += std::fabs(M.val[k]);
                vbound = std::max(vbound, 4.0 * a + 2.0);
            }
        }
        HIP_CHECK(hipMemcpyAsync(x, xin.data(), xin.size() * sizeof(VT), hipMemcpyHostToDevice, s));
        HIP_CHECK(hipStreamSynchronize(s));
    }
    auto check_candidate = [&](const DevMat<VT> &D) {
        const int64_t ny = std::max<int64_t>(1, M.nrows);
        // the prolongation kernel adds to its output: start from zero
        HIP_CHECK(hipMemsetAsync(y, 0, (size_t)ny * sizeof(VT), s));
        launch_for_tuning(kind, D, x, y, s);
        HIP_CHECK(hipGetLastError());
        std::vector<VT> yh(ny);
        HIP_CHECK(hipMemcpyAsync(yh.data(), y, (size_t)ny * sizeof(VT), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        if (yref.empty()) {
            yref = std::move(yh);
            ref_name = describe(D);
            return;
        }
        const double tol = (sizeof(VT) == 8 ? 1e-12 : 1e-4) * vbound;
        double dmax = 0.0;
        for (int64_t i = 0; i < ny; ++i) {
            const double d = std::fabs((double)yh[i] - (double)yref[i]);
            if (!(d <= tol)) {   // also catches NaN
                char msg[256];
                std::snprintf(msg, sizeof msg, "layout check: %s differs from %s by %.3g at row %lld (bound %.3g)",
                              describe(D).c_str(), ref_name.c_str(), d, (long long)i, tol);
                throw Error{DFAMG_EINVAL, msg};
            }
            dmax = std::max(dmax, d);
        }
        if (verbose > 1)
            std::fprintf(stderr, "[dfamg] layout check %s against %s: max difference %.3g (bound %.3g)\n",
                         describe(D).c_str(), ref_name.c_str(), dmax, tol);
    };
    double best = 1e30;
    DevMat<VT> bestM;
    Layout bestL{};
    std::unique_ptr<DevArena> bestA;
    // the outer kernel also keeps its reduction slots in static LDS
    const size_t stage_limit = outer ? kMaxStageBytes - 512 : kMaxStageBytes;
    // host forms of all candidates, built in parallel (one per distinct
    // structure); 32-bit SELL forms for the unstaged candidates whose 16-bit
    // offsets may not fit (the whole outer operator)
    std::map<HostKey, HostLayout> built;
    for (const Layout &c : cand) {
        built[host_key(c)];
        if (outer && c.fmt == DFAMG_FORMAT_SELL && !c.stage && c.idx16) {
            Layout c32 = c;
            c32.idx16 = false;
            built[host_key(c32)];
        }
    }
    {
        std::vector<std::pair<const HostKey, HostLayout> *> jobs;
        for (auto &kv : built) jobs.push_back(&kv);
        parallel_for((int64_t)jobs.size(), std::min<int>(8, (int)jobs.size()),
                     [&](int64_t j) { build_host_layout(M, ranges, jobs[j]->first, jobs[j]->second); });
    }
    auto form_of = [&](const Layout &c) -> const HostLayout * {
        auto it = built.find(host_key(c));
        if (it == built.end()) {   // a fallback not built above
            HostLayout &H = built[host_key(c)];
            build_host_layout(M, ranges, host_key(c), H);
            return &H;
        }
        return &it->second;
    };
    std::map<int, GatherLists> gl_cache;
    for (Layout c : cand) {
        auto A = std::make_unique<DevArena>();
        DevMat<VT> D;
        if (!upload_built<VT>(*A, *form_of(c), c, s, sub_sys, nsys, nsub, D, stage_limit, &gl_cache)) {
            // 16-bit offsets that do not fit: fall back to 32-bit columns
            // once; a gather list above the LDS budget (CSR_GATHER): to the
            // unstaged form
            if (c.fmt == DFAMG_FORMAT_SELL && !c.stage && c.idx16) {
                c.idx16 = false;
            } else if (c.fmt == kFormatSeg && family == DFAMG_FORMAT_COLUMN_TILED) {
                // an operator with no entries to tile: SELL
                c = Layout{DFAMG_FORMAT_SELL, 1, false, false, false, 0};
            } else if (gather && c.glist) {
                c.stage = false;
                c.glist = false;
            } else {
                continue;
            }
            A = std::make_unique<DevArena>();
            if (!upload_built<VT>(*A, *form_of(c), c, s, sub_sys, nsys, nsub, D, stage_limit, &gl_cache)) continue;
        }
        if (verify) check_candidate(D);
        const double t = cached_us >= 0.0 ? cached_us
                         : cand.size() > 1 ? (timer ? timer(D) : time_layout(kind, D, x, y, s))
                                           : 0.0;
        if (verbose > 1)
            std::fprintf(stderr, "[dfamg] tune kind %d rows %lld nnz %lld: %s %.2f us\n", (int)kind, (long long)rows,
                         (long long)M.nnz(), describe(D).c_str(), t);
        if (t < best) {
            best = t;
            bestM = D;
            bestA = std::move(A);
            bestL = c;
        }
    }
    if (bestA && cand.size() > 1) {
        std::lock_guard<std::mutex> g(tune_cache_mutex());
        tune_cache_store(key, bestL, best);
    }
    if (!bestA) throw Error{DFAMG_EINVAL, "no sparse layout can hold a matrix"};
    bestM.tuned_us = best;
    ar.adopt(*bestA);
    return bestM;
}

// Couplings between subdomains of the permuted global operator (host side of
// OffM): CSR over all rows.
struct HostOff {
    std::vector<int32_t> ptr, col;
    std::vector<double> val;
};

// Splits the permuted operator into its block-diagonal part (columns inside
// the row's subdomain; same row and column numbering) and the couplings.
void split_operator(const Plan &P, Csr &loc, HostOff &off) {
    loc.nrows = loc.ncols = P.n;
    loc.ptr.assign(P.n + 1, 0);
    loc.col.clear();
    loc.val.clear();
    loc.col.reserve(P.A.col.size());
    loc.val.reserve(P.A.val.size());
    off.ptr.assign(P.n + 1, 0);
    for (int sub = 0; sub < P.nsub; ++sub) {
        const int64_t lo = P.sub_row_off[sub], hi = P.sub_row_off[sub + 1];
        for (int64_t i = lo; i < hi; ++i) {
            for (int64_t k = P.A.ptr[i]; k < P.A.ptr[i + 1]; ++k) {
                const int32_t c = P.A.col[k];
                if (c >= lo && c < hi) {
                    loc.col.push_back(c);
                    loc.val.push_back(P.A.val[k]);
                } else {
                    off.col.push_back(c);
                    off.val.push_back(P.A.val[k]);
                }
            }
            loc.ptr[i + 1] = (int64_t)loc.col.size();
            if (off.col.size() > (size_t)INT32_MAX) throw Error{DFAMG_EINVAL, "too many couplings"};
            off.ptr[i + 1] = (int32_t)off.col.size();
        }
    }
}

// Dictionary coding of the deflation blocks (see ZView): per subdomain and
// column the distinct values in first-appearance order and a byte per entry.
struct ZCodes {
    std::vector<uint8_t> code;
    std::vector<double> tab;
    std::vector<int32_t> tab_off;
};

bool code_deflation(const Plan &P, ZCodes &zc) {
    const int ndv = P.ndv;
    zc.code.assign((size_t)P.n * ndv, 0);
    zc.tab_off.assign((size_t)P.nsub * ndv, 0);
    for (int s = 0; s < P.nsub; ++s)
        for (int k = 0; k < ndv; ++k) {
            zc.tab_off[(size_t)s * ndv + k] = (int32_t)zc.tab.size();
            std::vector<double> vals;
            std::unordered_map<uint64_t, int> seen;   // keyed by the bit pattern (-0.0 != 0.0)
            for (int64_t i = P.sub_row_off[s]; i < P.sub_row_off[s + 1]; ++i) {
                const double v = P.Z[(size_t)i * ndv + k];
                uint64_t bits;
                std::memcpy(&bits, &v, sizeof bits);
                auto it = seen.find(bits);
                int c;
                if (it == seen.end()) {
                    if (vals.size() == 256) return false;
                    c = (int)vals.size();
                    seen.emplace(bits, c);
                    vals.push_back(v);
                } else {
                    c = it->second;
                }
                zc.code[(size_t)i * ndv + k] = (uint8_t)c;
            }
            zc.tab.insert(zc.tab.end(), vals.begin(), vals.end());
            if (zc.tab.size() > (size_t)INT32_MAX) return false;
        }
    return true;
}

// Device OffM for the tiles of the block-diagonal layout D.
OffM upload_off(DevArena &ar, const HostOff &off, const DevMat<double> &D, hipStream_t s) {
    std::vector<int32_t> any(std::max<size_t>(1, D.host_tiles.size()), 0);
    for (size_t t = 0; t < D.host_tiles.size(); ++t) {
        const DevTile &T = D.host_tiles[t];
        any[t] = off.ptr[T.row0 + T.nrows] > off.ptr[T.row0] ? 1 : 0;
    }
    OffM o{};
    o.any = ar.upload(any, s);
    o.ptr = ar.upload(off.ptr, s);
    o.col = ar.upload(off.col.empty() ? std::vector<int32_t>{0} : off.col, s);
    o.val = ar.upload(off.val.empty() ? std::vector<double>{0.0} : off.val, s);
    return o;
}

// Short text of a chosen layout, e.g. "sell2/i16/stage" or "csr8/t64".
template <class VT>
std::string describe(const DevMat<VT> &D) {
    if (D.fmt == DFAMG_FORMAT_BSR4) return "bsr4";
    if (D.fmt == kFormatSeg) return "seg" + std::to_string(D.par) + "/b" + std::to_string(D.seg_nt);
    std::string t = D.fmt == DFAMG_FORMAT_SELL ? "sell" + std::to_string(D.par) : "csr" + std::to_string(D.par);
    if (D.fmt == DFAMG_FORMAT_SELL) {
        t += D.idx16 ? "/i16" : "/i32";
        if (D.sorted) t += "/sorted";
    } else if (!D.host_tiles.empty()) {
        t += "/t" + std::to_string(D.host_tiles[0].nrows);
    }
    if (D.stage) t += D.ucol ? "/glist" : "/stage";
    return t;
}

// Ranges of the packed rows of `subs` at a level.
std::vector<RowRange> ranges_of(const PackedLevel &L, const std::vector<int32_t> &subs) {
    std::vector<RowRange> r;
    for (int32_t s : subs) r.push_back(RowRange{L.sub_off[s], L.sub_len[s], s, 0});
    return r;
}

// Batched FP64 Gauss-Jordan inversion on the device of the dense matrices
// `mats` (row-major, sizes `ns`); writes the transposed inverses in type VT
// at `out` (offsets `out_off`) and returns the index of the first singular
// matrix or -1.
// Coarse operators of at least this size are inverted one at a time by the
// blocked elimination (dense_inverse.hip); smaller ones, and the coarsest
// AMG blocks, together by the unblocked one below (measured on the MI355X,
// host copies included: 8 against 20 ms at 1024 unknowns, 62 against 622 ms
// at 4096, equal at 256, where the unblocked form also serves many systems
// in one pass).
constexpr int kBlockedInverseMin = 1024;

template <class VT>
int invert_on_device(hipStream_t s, const std::vector<const double *> &mats, const std::vector<int32_t> &ns,
                     VT *out, const std::vector<int64_t> &out_off, const std::vector<int32_t> &out_ld) {
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
    DevArena tmp;
    double *d_aug = tmp.upload(aug, s);
    InvJob *d_jobs = tmp.upload(jobs, s);
    int64_t *d_coff = tmp.upload(col_off, s);
    double *d_colk = tmp.alloc<double>(col_off[nb]);
    int64_t *d_oof = tmp.upload(out_off, s);
    int32_t *d_old = tmp.upload(out_ld, s);
    const int64_t maxel = (int64_t)nmax * 2 * nmax;
    const int gx = (int)std::min<int64_t>(1024, (maxel + kBlock - 1) / kBlock);
    for (int k = 0; k < nmax; ++k) {
        hipLaunchKernelGGL(k_gj_pivot, dim3(nb), dim3(kBlock), 0, s, d_jobs, d_aug, d_colk, d_coff, k);
        hipLaunchKernelGGL(k_gj_eliminate, dim3(gx, nb), dim3(kBlock), 0, s, d_jobs, d_aug, d_colk, d_coff, k);
    }
    hipLaunchKernelGGL(k_gj_extract<VT>, dim3(gx, nb), dim3(kBlock), 0, s, d_jobs, d_aug, d_oof, d_old, out);
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
    KID_DIR = DFAMG_KERNEL_DIRECTION, KID_RESTRICT1 = DFAMG_KERNEL_RESTRICT1, KID_DEEP = DFAMG_KERNEL_DEEP,
    KID_UP1 = DFAMG_KERNEL_UP1, KID_N = DFAMG_KERNEL_COUNT
};

struct Prof {
    bool on = false, capturing = false;
    bool suppress = false;               // capturing the graph without event nodes
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
    int level = 1;                        // 1: outer SpMV and level-0 restriction, 2: every span
    void mark(int kid, int which, hipStream_t st) {
        if (!on || suppress || (level < 2 && kid != KID_SPMV && kid != KID_PRE0)) return;
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
    // further slots (only kernels up to the stopping test: the rest of such an
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
    // block of the level-0 direct solves (part_job)
    virtual void apply(hipStream_t st, const double *r, double *s, double *part, double *part_job,
                       const SysState *states, const int32_t *sub_sys, Prof *prof) = 0;
    virtual const std::vector<int32_t> &sys_tile_off0() const = 0;
    virtual int32_t nslots0() const = 0;
    std::vector<int32_t> sys_cjob_off0;  // level-0 direct-solve blocks per system
    int32_t ncjobs0 = 0;
    double bytes = 0.0;                 // algorithmic bytes per application
    double kbytes[KID_N] = {};          // per profiled kernel
    int fmt[20] = {}, par[20] = {};     // chosen layout of A_l
    std::string layouts;                // chosen layouts, as text
};

template <class VT>
struct Hierarchy_dev : PrecondBase {
    struct Lvl {
        int64_t nrows = 0;
        bool active = false;
        DevMat<VT> A, P, R, B;   // B = R (I - A diag(m)), see k_restrict
        bool fused = false;      // restrict with B, else pre-smoothing residual then R
        VT *m = nullptr;
        VT *mb = nullptr, *xpre = nullptr;   // block SPAI-0 rows and the pre-smoothed iterate
        VT *f = nullptr, *res = nullptr, *z = nullptr, *x = nullptr;
        VT *w = nullptr;          // second iterate buffer of repeated smoothing sweeps
        VT *xcur = nullptr;       // the pre-smoothed iterate (xpre or w) when npre >= 2
        CoarseEntry *coarse = nullptr;
        CoarseJob *cjobs = nullptr;
        int32_t ncoarse = 0, ncjobs = 0;
        VT *coarse_inv = nullptr;
    };
    std::vector<Lvl> lv;
    int bs = 1;
    int npre = 1, npost = 1;             // smoothing sweeps of the V-cycle
    bool block = false;                  // block SPAI-0 smoother
    std::vector<int32_t> sto0;
    int32_t slots0 = 0;

    const std::vector<int32_t> &sys_tile_off0() const override { return sto0; }
    int32_t nslots0() const override { return slots0; }

    void build(DevArena &ar, const Plan &plan, hipStream_t s, int format, bool autotune, int verbose) {
        const int L = plan.nlevels_max;
        lv.resize(L);
        block = plan.prm.smoother == DFAMG_SMOOTHER_BLOCK_SPAI0;
        bs = plan.bs;
        npre = plan.prm.npre;
        npost = plan.prm.npost;
        const double sv = sizeof(VT), ib = 4.0;
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
                D.z = ar.alloc<VT>(PL.nrows);
                const auto rr = ranges_of(PL, PL.active_subs);
                D.A = upload_tuned<VT>(ar, PL.A, rr, format, autotune, TUNE_SMOOTH, s, plan.sub_sys, plan.nsys,
                                       plan.nsub, {}, verbose, plan.bs == 4);
                D.P = upload_tuned<VT>(ar, PL.P, rr, format, autotune, TUNE_PROLONG, s, plan.sub_sys, plan.nsys,
                                       plan.nsub, {}, verbose, plan.bs == 4);
                const PackedLevel &PN = plan.levels[l + 1];
                std::vector<int32_t> next_subs;
                for (int sub = 0; sub < plan.nsub; ++sub)
                    if (PN.sub_off[sub] >= 0) next_subs.push_back(sub);
                // the level's restricted residual either through B in one launch or
                // as pre-smoothing residual (A) plus restriction (R): the faster by
                // the tuner's timings (R without tuning)
                {
                    const auto rn = ranges_of(PN, next_subs);
                    const bool column_tiled = format == DFAMG_FORMAT_COLUMN_TILED;
                    const bool can_fuse = (autotune || column_tiled) && !block && npre == 1;
                    const bool has_bc = can_fuse && PL.Bc.nnz() > 0;
                    const uint64_t hR = structure_hash(PL.R, rn);
                    const uint64_t hB = can_fuse ? structure_hash(PL.B, rn) : 0;
                    const uint64_t hBc = has_bc ? structure_hash(PL.Bc, rn) : 0;
                    const double uR = autotune ? recorded_us<VT>(TUNE_RESTRICT, format, hR) : -1.0;
                    const double uB = can_fuse ? recorded_us<VT>(TUNE_RESTRICT, format, hB) : -1.0;
                    const double uBc = has_bc ? recorded_us<VT>(TUNE_RESTRICT, format, hBc) : -1.0;
                    if (uR >= 0.0 && (!can_fuse || (uB >= 0.0 && (!has_bc || uBc >= 0.0)))) {
                        // every candidate's time is recorded: build only the
                        // operators the comparison below keeps
                        const bool clustered = has_bc && uBc < uB;
                        D.fused = can_fuse && (clustered ? uBc : uB) < D.A.tuned_us + uR;
                        if (D.fused) {
                            D.B = upload_tuned<VT>(ar, clustered ? PL.Bc : PL.B, rn, format, autotune, TUNE_RESTRICT, s,
                                                   plan.sub_sys, plan.nsys, plan.nsub, {}, verbose, plan.bs == 4,
                                                   clustered ? hBc : hB);
                            if (clustered) D.B.rowmap = ar.upload(PL.B_rowmap, s);
                        } else {
                            D.R = upload_tuned<VT>(ar, PL.R, rn, format, autotune, TUNE_RESTRICT, s, plan.sub_sys,
                                                   plan.nsys, plan.nsub, {}, verbose, plan.bs == 4, hR);
                            D.res = ar.alloc<VT>(PL.nrows);
                        }
                    } else {
                        // the level's restricted residual either through B in one
                        // launch or as pre-smoothing residual (A) plus restriction
                        // (R): the faster by the tuner's timings (R without tuning)
                        DevArena arR, arB;
                        D.R = upload_tuned<VT>(arR, PL.R, rn, format, autotune, TUNE_RESTRICT, s, plan.sub_sys,
                                               plan.nsys, plan.nsub, {}, verbose, plan.bs == 4, hR);
                        // B holds exactly one pre-smoothing sweep from the zero guess
                        bool clustered = false;
                        DevArena arBc;
                        if (can_fuse) {
                            D.B = upload_tuned<VT>(arB, PL.B, rn, format, autotune, TUNE_RESTRICT, s, plan.sub_sys,
                                                   plan.nsys, plan.nsub, {}, verbose, plan.bs == 4, hB);
                            // the rows in the clustered order: fewer distinct
                            // columns per tile, but wider column windows
                            if (has_bc) {
                                DevMat<VT> Bc = upload_tuned<VT>(arBc, PL.Bc, rn, format, autotune, TUNE_RESTRICT, s,
                                                                 plan.sub_sys, plan.nsys, plan.nsub, {}, verbose,
                                                                 plan.bs == 4, hBc);
                                if (Bc.tuned_us < D.B.tuned_us) {
                                    D.B = Bc;
                                    clustered = true;
                                }
                            }
                            D.fused = column_tiled || D.B.tuned_us < D.A.tuned_us + D.R.tuned_us;
                        }
                        if (D.fused) {
                            ar.adopt(clustered ? arBc : arB);
                            if (clustered) D.B.rowmap = ar.upload(PL.B_rowmap, s);
                            D.R = DevMat<VT>{};
                        } else {
                            ar.adopt(arR);
                            D.B = DevMat<VT>{};
                            D.res = ar.alloc<VT>(PL.nrows);
                        }
                    }
                }
                if (l < 20) {
                    fmt[l] = D.A.fmt;
                    par[l] = D.A.par;
                }
                layouts += " L" + std::to_string(l) + "{A " + describe(D.A) +
                           (D.fused ? ", B " + describe(D.B) + (D.B.rowmap ? "/clustered" : "") : ", R " + describe(D.R)) +
                           ", P " + describe(D.P) + "}";
                std::vector<VT> m(PL.m.size());
                for (size_t i = 0; i < m.size(); ++i) m[i] = (VT)PL.m[i];
                D.m = ar.upload(m, s);
                if (npre >= 2 || npost >= 2) {
                    D.xpre = ar.alloc<VT>(PL.nrows);
                    D.w = ar.alloc<VT>(PL.nrows);
                }
                if (block) {
                    std::vector<VT> mb(PL.mb.size());
                    for (size_t i = 0; i < mb.size(); ++i) mb[i] = (VT)PL.mb[i];
                    D.mb = ar.upload(mb, s);
                    D.xpre = ar.alloc<VT>(PL.nrows);
                }
                HIP_CHECK(hipStreamSynchronize(s));
                const double n0 = (double)PL.nrows, n1 = (double)PN.nrows;
                // the level's right-hand side is FP64 on level 0
                const double fb = l == 0 ? 8.0 : sv;
                // pre-smoothing residual and restriction, or both as one operator B
                // (one sweep); a sweep x + m (f - A x) reads A, m, f, x and
                // writes x; the first sweep from zero is x = m o f
                const double sweep = D.A.nnz * (sv + ib) + n0 * (fb + 3.0 * sv);
                double kb_pre = D.fused ? D.B.nnz * (sv + ib) + n0 * fb + n1 * sv
                                        : D.A.nnz * (sv + ib) + n0 * (fb + 2.0 * sv);
                double kb_res = D.fused ? 0.0 : D.R.nnz * (sv + ib) + n0 * sv + n1 * sv;
                double kb_pro = D.P.nnz * (sv + ib) + n0 * (2.0 * sv + fb) + n1 * sv;
                if (npre == 0) {
                    kb_pre = D.R.nnz * (sv + ib) + n0 * fb + n1 * sv;
                    kb_res = 0.0;
                    kb_pro = D.P.nnz * (sv + ib) + n0 * sv + n1 * sv;
                } else if (npre >= 2) {
                    kb_pre = n0 * (fb + 2.0 * sv) + (npre - 1) * sweep + D.A.nnz * (sv + ib) + n0 * (fb + 2.0 * sv);
                    kb_pro = D.P.nnz * (sv + ib) + n0 * 2.0 * sv + n1 * sv;
                }
                const double kb_post = (npost - 1) * sweep +
                                       D.A.nnz * (sv + ib) + n0 * (2.0 * sv + fb + (l == 0 ? 8.0 : sv));
                if (l == 0) {
                    sto0 = D.A.sys_tile_off;
                    slots0 = D.A.ntiles;
                    kbytes[KID_PRE0] = kb_pre;
                    kbytes[KID_RESTRICT0] = kb_res;
                    kbytes[KID_PROLONG0] = kb_pro;
                    kbytes[KID_POST0] = kb_post;
                } else {
                    kbytes[KID_COARSER] += kb_pre + kb_res + kb_pro + kb_post;
                    if (l == 1) {
                        kbytes[KID_RESTRICT1] = kb_pre + kb_res;
                        kbytes[KID_UP1] = kb_pro + kb_post;
                    } else {
                        kbytes[KID_DEEP] += kb_pre + kb_res + kb_pro + kb_post;
                    }
                }
                bytes += kb_pre + kb_res + kb_pro + kb_post;
            }
            if (!PL.coarse_subs.empty()) {
                std::vector<CoarseEntry> ce;
                std::vector<std::vector<double>> dense;
                std::vector<int32_t> ns, lds;
                std::vector<int64_t> off;
                int64_t total = 0;
                constexpr int nv = 16 / (int)sizeof(VT);
                for (int32_t sub : PL.coarse_subs) {
                    const Csr &M = plan.hier[sub].lv.back().A;
                    const int n = (int)M.nrows, ld = (n + nv - 1) / nv * nv;
                    std::vector<double> d((size_t)n * n, 0.0);
                    for (int i = 0; i < n; ++i)
                        for (int64_t k = M.ptr[i]; k < M.ptr[i + 1]; ++k) d[(size_t)i * n + M.col[k]] = M.val[k];
                    dense.push_back(std::move(d));
                    ns.push_back(n);
                    lds.push_back(ld);
                    off.push_back(total);
                    ce.push_back(CoarseEntry{sub, n, PL.sub_off[sub], total, ld, 0});
                    total += (int64_t)n * ld;
                }
                // one block per kCoarseRows rows of every coarsest matrix, in
                // subdomain (hence system) order
                std::vector<CoarseJob> cj;
                std::vector<int32_t> sjo(plan.nsys + 1, 0);
                for (size_t e = 0; e < ce.size(); ++e)
                    for (int r0 = 0; r0 < ce[e].n; r0 += kCoarseRows) {
                        cj.push_back(CoarseJob{(int32_t)e, r0});
                        sjo[plan.sub_sys[ce[e].sub] + 1]++;
                    }
                for (int i = 0; i < plan.nsys; ++i) sjo[i + 1] += sjo[i];
                D.cjobs = ar.upload(cj, s);
                D.ncjobs = (int32_t)cj.size();
                if (l == 0) {
                    sys_cjob_off0 = sjo;
                    ncjobs0 = D.ncjobs;
                }
                std::vector<const double *> mats;
                for (auto &d : dense) mats.push_back(d.data());
                D.coarse_inv = ar.alloc<VT>(total);
                const int bad = invert_on_device<VT>(s, mats, ns, D.coarse_inv, off, lds);
                if (bad >= 0)
                    throw Error{DFAMG_ESINGULAR, "coarsest-level matrix of subdomain " +
                                                     std::to_string(plan.sub_user[PL.coarse_subs[bad]]) +
                                                     " is singular"};
                D.coarse = ar.upload(ce, s);
                D.ncoarse = (int32_t)ce.size();
                HIP_CHECK(hipStreamSynchronize(s));
                double nsq = 0.0;
                for (int nn : ns) nsq += (double)nn * nn;
                const double cb = nsq * sv + 2.0 * PL.nrows * sv;
                bytes += cb;
                if (l > 0) {
                    kbytes[KID_COARSER] += cb;
                    kbytes[KID_DEEP] += cb;
                }
            }
        }
        if (L > 0 && !lv[0].active) {
            sto0.assign(plan.nsys + 1, 0);
            slots0 = 0;
        }
        if (sys_cjob_off0.empty()) sys_cjob_off0.assign(plan.nsys + 1, 0);
    }

    // V(1,1) with the block SPAI-0 smoother: per level x = M f, y = A x,
    // f_c = R (f - y); after the coarse solves z = x + P x_c, y = A z,
    // out = z + M (f - y).  The same steps as the diagonal smoother's, as
    // separate passes (the node's rows share one block of M).
    void apply_block(hipStream_t st, const double *r, double *s, double *part, double *part_job,
                     const SysState *states, const int32_t *sub_sys) {
        const int L = (int)lv.size();
        const dim3 b(kBlock);
        for (int l = 0; l + 1 < L; ++l) {
            Lvl &D = lv[l];
            if (!D.active) continue;
            const dim3 g(grid_for_tiles(D.A.ntiles));
            if (l == 0) {
                hipLaunchKernelGGL((k_bsm_pre<VT, double>), g, b, 0, st, D.A.tiles, D.A.ntiles, bs, D.mb, r, D.xpre,
                                   states, sub_sys);
                launch_spmv<VT>(D.A, D.xpre, D.res, states, sub_sys, st);
                hipLaunchKernelGGL((k_bsm_res<VT, double>), g, b, 0, st, D.A.tiles, D.A.ntiles, r, D.res, states,
                                   sub_sys);
            } else {
                hipLaunchKernelGGL((k_bsm_pre<VT, VT>), g, b, 0, st, D.A.tiles, D.A.ntiles, bs, D.mb, D.f, D.xpre,
                                   states, sub_sys);
                launch_spmv<VT>(D.A, D.xpre, D.res, states, sub_sys, st);
                hipLaunchKernelGGL((k_bsm_res<VT, VT>), g, b, 0, st, D.A.tiles, D.A.ntiles, D.f, D.res, states,
                                   sub_sys);
            }
            launch_spmv<VT>(D.R, D.res, lv[l + 1].f, states, sub_sys, st);
        }
        for (int l = 0; l < L; ++l) {
            Lvl &D = lv[l];
            if (!D.ncoarse) continue;
            if (l == 0)
                hipLaunchKernelGGL((k_coarse<VT, double, double, true>), dim3(D.ncjobs), b, 0, st, D.cjobs, D.coarse,
                                   D.coarse_inv, r, s, part_job, states, sub_sys);
            else
                hipLaunchKernelGGL((k_coarse<VT, VT, VT, false>), dim3(D.ncjobs), b, 0, st, D.cjobs, D.coarse,
                                   D.coarse_inv, D.f, D.x, part_job, states, sub_sys);
        }
        for (int l = L - 2; l >= 0; --l) {
            Lvl &D = lv[l];
            if (!D.active) continue;
            const dim3 g(grid_for_tiles(D.A.ntiles));
            launch_spmv<VT>(D.P, lv[l + 1].x, D.z, states, sub_sys, st);
            hipLaunchKernelGGL((k_bsm_add<VT>), g, b, 0, st, D.A.tiles, D.A.ntiles, D.xpre, D.z, states, sub_sys);
            launch_spmv<VT>(D.A, D.z, D.res, states, sub_sys, st);
            if (l == 0)
                hipLaunchKernelGGL((k_bsm_post<VT, double, double, true>), g, b, 0, st, D.A.tiles, D.A.ntiles, bs,
                                   D.mb, r, D.z, D.res, s, part, states, sub_sys);
            else
                hipLaunchKernelGGL((k_bsm_post<VT, VT, VT, false>), g, b, 0, st, D.A.tiles, D.A.ntiles, bs, D.mb,
                                   D.f, D.z, D.res, D.x, part, states, sub_sys);
        }
    }

    // Downward step of a level with npre != 1 sweeps: fc = R (f - A x) with x
    // the pre-smoothed iterate (x = 0 when npre = 0, else x = m o f followed
    // by npre - 1 sweeps x + m o (f - A x)), kept in D.xcur for the upward step.
    template <class FT>
    void down_sweeps(Lvl &D, const FT *f, VT *fc, const SysState *states, const int32_t *sub_sys, hipStream_t st) {
        if (npre == 0) {
            launch_restrict<VT, FT>(D.R, f, fc, states, sub_sys, st);
            D.xcur = nullptr;
            return;
        }
        VT *x = D.xpre, *o = D.w;
        const int g = (int)std::min<int64_t>(4096, (D.nrows + kBlock - 1) / kBlock);
        hipLaunchKernelGGL((k_vscale<VT, FT>), dim3(std::max(g, 1)), dim3(kBlock), 0, st, D.nrows, D.m, f, x);
        for (int k = 1; k < npre; ++k) {
            launch_post<VT, FT, VT, false>(D.A, D.m, f, x, o, nullptr, states, sub_sys, st);
            std::swap(x, o);
        }
        D.xcur = x;
        launch_resid<VT, FT>(D.A, f, x, D.res, states, sub_sys, st);
        launch_spmv<VT>(D.R, D.res, fc, states, sub_sys, st);
    }

    // Upward step: z = x_pre + P xc, then npost sweeps; the last one writes
    // `out` (with the (f, out) partials when DOT).
    template <class FT, class OT, bool DOT>
    void up_sweeps(Lvl &D, const FT *f, const VT *xc, OT *out, double *part, const SysState *states,
                   const int32_t *sub_sys, hipStream_t st) {
        if (npre == 1) launch_prolong<VT, FT>(D.P, D.m, f, xc, D.z, states, sub_sys, st);
        else launch_prolong_add<VT>(D.P, D.xcur, xc, D.z, states, sub_sys, st);
        VT *z = D.z, *o = D.w;
        for (int k = 1; k < npost; ++k) {
            launch_post<VT, FT, VT, false>(D.A, D.m, f, z, o, nullptr, states, sub_sys, st);
            std::swap(z, o);
        }
        launch_post<VT, FT, OT, DOT>(D.A, D.m, f, z, out, part, states, sub_sys, st);
    }

    void apply(hipStream_t st, const double *r, double *s, double *part, double *part_job,
               const SysState *states, const int32_t *sub_sys, Prof *prof) override {
        if (block) {
            apply_block(st, r, s, part, part_job, states, sub_sys);
            return;
        }
        const int L = (int)lv.size();
        auto mark = [&](int kid, int which) {
            if (prof) prof->mark(kid, which, st);
        };
        const dim3 b(kBlock);
        // spans of the profile: level 0 step by step, level 1 down and up,
        // and everything deeper (levels >= 2 and the coarsest solves) as one
        bool deep_open = false;
        auto open_deep = [&] {
            if (!deep_open) mark(KID_DEEP, 0);
            deep_open = true;
        };
        auto close_deep = [&] {
            if (deep_open) mark(KID_DEEP, 1);
            deep_open = false;
        };
        // downward: pre-smoothing residuals and restriction
        for (int l = 0; l + 1 < L; ++l) {
            Lvl &D = lv[l];
            if (!D.active) continue;
            if (l >= 2) open_deep();
            if (l == 1) mark(KID_RESTRICT1, 0);
            if (l == 0) {
                mark(KID_PRE0, 0);
                if (npre != 1) {
                    down_sweeps<double>(D, r, lv[1].f, states, sub_sys, st);
                    mark(KID_PRE0, 1);
                } else if (D.fused) {
                    launch_restrict<VT, double>(D.B, r, lv[1].f, states, sub_sys, st);
                    mark(KID_PRE0, 1);
                } else {
                    launch_pre_res<VT, double>(D.A, D.m, r, D.res, states, sub_sys, st);
                    mark(KID_PRE0, 1);
                    mark(KID_RESTRICT0, 0);
                    launch_spmv<VT>(D.R, D.res, lv[1].f, states, sub_sys, st);
                    mark(KID_RESTRICT0, 1);
                }
                mark(KID_COARSER, 0);
            } else if (npre != 1) {
                down_sweeps<VT>(D, D.f, lv[l + 1].f, states, sub_sys, st);
            } else if (D.fused) {
                launch_restrict<VT, VT>(D.B, D.f, lv[l + 1].f, states, sub_sys, st);
            } else {
                launch_pre_res<VT, VT>(D.A, D.m, D.f, D.res, states, sub_sys, st);
                launch_spmv<VT>(D.R, D.res, lv[l + 1].f, states, sub_sys, st);
            }
            if (l == 1) mark(KID_RESTRICT1, 1);
        }
        open_deep();
        // direct solves on every subdomain's coarsest level
        for (int l = 0; l < L; ++l) {
            Lvl &D = lv[l];
            if (!D.ncoarse) continue;
            if (l == 0)
                hipLaunchKernelGGL((k_coarse<VT, double, double, true>), dim3(D.ncjobs), b, 0, st, D.cjobs, D.coarse,
                                   D.coarse_inv, r, s, part_job, states, sub_sys);
            else
                hipLaunchKernelGGL((k_coarse<VT, VT, VT, false>), dim3(D.ncjobs), b, 0, st, D.cjobs, D.coarse,
                                   D.coarse_inv, D.f, D.x, part_job, states, sub_sys);
        }
        // upward: coarse correction and post-smoothing
        for (int l = L - 2; l >= 0; --l) {
            Lvl &D = lv[l];
            if (!D.active) continue;
            if (l <= 1) close_deep();
            if (l == 0) {
                mark(KID_COARSER, 1);
                if (npre == 1 && npost == 1) {
                    mark(KID_PROLONG0, 0);
                    launch_prolong<VT, double>(D.P, D.m, r, lv[1].x, D.z, states, sub_sys, st);
                    mark(KID_PROLONG0, 1);
                    mark(KID_POST0, 0);
                    launch_post<VT, double, double, true>(D.A, D.m, r, D.z, s, part, states, sub_sys, st);
                    mark(KID_POST0, 1);
                } else {
                    mark(KID_POST0, 0);
                    up_sweeps<double, double, true>(D, r, lv[1].x, s, part, states, sub_sys, st);
                    mark(KID_POST0, 1);
                }
            } else {
                if (l == 1) mark(KID_UP1, 0);
                if (npre == 1 && npost == 1) {
                    launch_prolong<VT, VT>(D.P, D.m, D.f, lv[l + 1].x, D.z, states, sub_sys, st);
                    launch_post<VT, VT, VT, false>(D.A, D.m, D.f, D.z, D.x, part, states, sub_sys, st);
                } else {
                    up_sweeps<VT, VT, false>(D, D.f, lv[l + 1].x, D.x, part, states, sub_sys, st);
                }
                if (l == 1) mark(KID_UP1, 1);
            }
        }
        close_deep();
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
    // outer operator: block-diagonal part (its tiles carry the SpMV partials)
    // and the couplings between subdomains
    DevMat<double> A;
    OffM offA{};
    ZView zview{};                          // Z as the operator epilogue reads it
    double zview_bytes = 0.0;               // bytes of Z in that form (0: read at FP64)
    bool outer_split = false;
    int64_t outer_off_nnz = 0;              // couplings stored apart (split form)
    double outer_layout_bytes = 0.0;
    int32_t *d_sto_A = nullptr, *d_subto_A = nullptr;
    // row tiles for the vector kernels (update, direction, expansion)
    DevTile *rows = nullptr;
    int32_t nrow_tiles = 0;
    int32_t *d_sto_rows = nullptr, *d_subto_rows = nullptr;
    int32_t *d_sub_sys = nullptr, *d_sys_sub_off = nullptr, *d_sys_job_off = nullptr;
    int64_t *d_perm = nullptr;
    double *Z = nullptr, *AZown = nullptr, *AZoffv = nullptr, *t1 = nullptr, *t2 = nullptr;
    double *EinvT = nullptr;               // row-major E^{-1} of every system
    int32_t *AZoffp = nullptr, *AZoffc = nullptr;
    GemvJob *d_jobs = nullptr;
    int32_t njobs = 0;
    // vectors
    double *b = nullptr, *y = nullptr, *r = nullptr, *p = nullptr, *q = nullptr, *s = nullptr, *w = nullptr,
           *x = nullptr;
    // BiCGStab: r~, v, p^, s^, s, t
    double *rt = nullptr, *v = nullptr, *ph = nullptr, *sh = nullptr, *sv = nullptr, *tv = nullptr;
    bool bicg() const { return prm.solver == DFAMG_SOLVER_BICGSTAB; }
    // BiCGStab(2): r^_1, r^_2, u^_0 .. u^_2 and the preconditioned vectors
    // pr0, pr1, pu0, pu1 (r^_0 is r, r~ is rt)
    double *b2r1 = nullptr, *b2r2 = nullptr, *b2u0 = nullptr, *b2u1 = nullptr, *b2u2 = nullptr, *b2pr0 = nullptr,
           *b2pr1 = nullptr, *b2pu0 = nullptr, *b2pu1 = nullptr;
    bool bicg2() const { return prm.solver == DFAMG_SOLVER_BICGSTAB2; }
    // FGMRES: Arnoldi vectors V_0..V_m (unnormalised), V-cycle outputs
    // s_0..s_{m-1} and coarse solutions t2_0..t2_{m-1} of one cycle, the
    // per-system state and the dot partials of the Gram-Schmidt passes
    double *fgV = nullptr, *fgS = nullptr, *fgT2 = nullptr, *part_fg = nullptr;
    float *Einv32 = nullptr;                // E^{-1} in single precision (FP32 coarse solve)
    // CG coarse solve: E in CSR (global coarse numbering), inverse diagonal,
    // work vectors, per-system coarse-system offsets and step counters
    int64_t *ecg_ptr = nullptr, *ecg_iters = nullptr;
    int32_t *ecg_col = nullptr, *d_sys_coarse_off = nullptr;
    double *ecg_val = nullptr, *ecg_dinv = nullptr, *ecg_work = nullptr;
    int64_t coarse_iters_last = 0;
    int ecg_mmax = 0;                       // largest coarse system (LDS form of k_ecg)
    FgState *fg = nullptr;
    int64_t fg_ld = 0, fg_mtot = 0;
    bool fgmres() const { return prm.solver == DFAMG_SOLVER_FGMRES; }
    // partials and state
    double *part_A = nullptr, *part_rows = nullptr, *part_rs = nullptr, *part_rs_job = nullptr;
    int32_t *d_sys_cjob_off0 = nullptr;
    double *psub = nullptr, *tt_part = nullptr;
    int32_t *d_sto0 = nullptr;
    SysState *states = nullptr;
    SysState *h_states = nullptr;          // pinned
    double *hist = nullptr;
    int32_t hist_stride = 0;
    double *relres_true = nullptr;
    std::unique_ptr<PrecondBase> M;
    double *d_spai = nullptr;              // SPAI-0 diagonal (precond SPAI0)
    // a preconditioner supplied by a composite solver (the Schur pressure
    // correction); it may synchronise the stream, so it runs with direct
    // launches only
    std::function<void(hipStream_t, const double *, double *)> ext_precond;
    // graph of `graph_iters` iterations; with profile = 1 a second graph of the
    // same iterations without the event nodes, replayed after the first chunk
    // of every solve (each event node costs a few microseconds in the graph)
    hipGraph_t graph = nullptr, graph_plain = nullptr;
    hipGraphExec_t graph_exec = nullptr, graph_exec_plain = nullptr;
    int32_t graph_k = 0;
    bool want_events = true;     // the next chunk records the profile's events
    bool chunk_events = false;   // the chunk just launched recorded them
    bool have_rhs = false;
    double setup_device_s = 0.0, solve_s = 0.0;
    double bytes_iter = 0.0;
    Prof prof;
    bool graph_profile_fallback = false;

    ~Handle() {
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (graph_exec_plain) (void)hipGraphExecDestroy(graph_exec_plain);
        if (graph_plain) (void)hipGraphDestroy(graph_plain);
        if (h_states) (void)hipHostFree(h_states);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }

    int nsys() const { return plan.nsys; }
    int ndv() const { return plan.ndv; }
    SysRanges ranges() const { return SysRanges{d_sys_sub_off, d_sys_job_off}; }

    void setup_device();
    bool probe_graph_events();
    void outer(int mode, hipStream_t st, const double *xin, const double *bin, double *out, bool profiled = false);
    void project_solve(hipStream_t st, bool in_loop, const int32_t *subto, double *part, int32_t nslots,
                       int with_p0);
    void iteration(hipStream_t st);
    void iteration_bicg(hipStream_t st);
    void iteration_bicg2(hipStream_t st);
    void cycle_fgmres(hipStream_t st);
    void initial(hipStream_t st);
    void finish(hipStream_t st);
    void precond(hipStream_t st, const double *rin, double *sout, bool profiled = false);
    void launch_iterations(int k);
    void solve_one_cycle(const double *rhs, double *xio, int64_t *iter_acc);
    void assemble_E(double *Eout);
    dfamg_status run_solve(const double *rhs, double *xio);
    void apply_op(int op, const double *in, double *out);
};

void Handle::setup_device() {
    const double t0 = now_s();
    // phase times, printed with verbose >= 1
    double tmark = t0;
    std::string phases;
    auto phase = [&](const char *name) {
        HIP_CHECK(hipStreamSynchronize(stream));
        const double t = now_s();
        phases += std::string(phases.empty() ? "" : ", ") + name + " " + std::to_string((int)((t - tmark) * 1e3)) + " ms";
        tmark = t;
    };
    hipStream_t sm = stream;
    const Plan &P = plan;
    const int nsys = P.nsys, nsub = P.nsub, ndv = P.ndv;
    const int64_t n = P.n;
    for (int sy = 0; sy < nsys; ++sy)
        if (P.sys_m[sy] > 4096)
            throw Error{DFAMG_EINVAL, "coarse operator of a system exceeds 4096 unknowns (subdomains x vectors)"};
    std::vector<RowRange> rr;
    for (int sub = 0; sub < nsub; ++sub)
        rr.push_back(RowRange{P.sub_row_off[sub], (int32_t)(P.sub_row_off[sub + 1] - P.sub_row_off[sub]), sub, 0});
    d_sub_sys = ar.upload(P.sub_sys, sm);
    Z = ar.upload(P.Z, sm);
    zview = ZView{Z, nullptr, nullptr, nullptr};
    {
        ZCodes zc;
        if (ndv > 0 && code_deflation(P, zc)) {
            zview.code = ar.upload(zc.code, sm);
            zview.tab = ar.upload(zc.tab, sm);
            zview.tab_off = ar.upload(zc.tab_off, sm);
            zview_bytes = (double)zc.code.size() + 8.0 * (double)zc.tab.size() + 4.0 * (double)zc.tab_off.size();
        }
    }
    states = ar.alloc<SysState>(nsys);
    HIP_CHECK(hipMemsetAsync(states, 0, sizeof(SysState) * nsys, sm));
    // outer matrix over all subdomains, either whole or as block-diagonal part
    // plus couplings (which lets the layouts use 16-bit columns and LDS
    // staging); every candidate is timed with the in-loop kernel (couplings
    // and deflation epilogue included) and the faster form is kept
    {
        Csr loc;
        HostOff off, none;
        split_operator(P, loc, off);
        none.ptr.assign(n + 1, 0);
        DevArena vecs;
        double *tx = vecs.alloc<double>(n), *ty = vecs.alloc<double>(n);
        HIP_CHECK(hipMemsetAsync(tx, 0, sizeof(double) * n, sm));
        auto make_timer = [&](const HostOff &o_) {
            return std::function<double(const DevMat<double> &)>([&, po = &o_](const DevMat<double> &D) {
                DevArena tmp;
                const OffM o = upload_off(tmp, *po, D, sm);
                double *tp = tmp.alloc<double>((size_t)D.ntiles * (ndv + 1));
                const double t = time_launches(
                    [&] { launch_outer(0, ndv, D, o, tx, nullptr, ty, zview, tp, states, d_sub_sys, sm); }, sm);
                HIP_CHECK(hipStreamSynchronize(sm));
                return t;
            });
        };
        const bool tune = prm.autotune != 0;
        const bool try_split = tune && !off.col.empty();
        const uint64_t hF = structure_hash(P.A, rr), hS = try_split ? structure_hash(loc, rr) : 0;
        const double uF = tune ? recorded_us<double>(TUNE_OUTER, prm.spmv_format, hF) : -1.0;
        const double uS = try_split ? recorded_us<double>(TUNE_OUTER, prm.spmv_format, hS) : -1.0;
        bool split = false;
        if (uF >= 0.0 && (!try_split || uS >= 0.0)) {
            // both forms' times recorded: build only the faster one
            split = try_split && uS < uF;
            A = upload_tuned<double>(ar, split ? loc : P.A, rr, prm.spmv_format, tune, TUNE_OUTER, sm, P.sub_sys, nsys,
                                     nsub, make_timer(split ? off : none), prm.verbose, P.bs == 4, split ? hS : hF);
        } else {
            DevArena arF, arS;
            const DevMat<double> AF = upload_tuned<double>(arF, P.A, rr, prm.spmv_format, tune, TUNE_OUTER, sm,
                                                           P.sub_sys, nsys, nsub, make_timer(none), prm.verbose,
                                                           P.bs == 4, hF);
            DevMat<double> AS;
            if (try_split) {
                AS = upload_tuned<double>(arS, loc, rr, prm.spmv_format, tune, TUNE_OUTER, sm, P.sub_sys, nsys, nsub,
                                          make_timer(off), prm.verbose, P.bs == 4, hS);
                split = AS.tuned_us < AF.tuned_us;
            }
            ar.adopt(split ? arS : arF);
            A = split ? AS : AF;
        }
        offA = upload_off(ar, split ? off : none, A, sm);
        outer_split = split;
        outer_off_nnz = split ? (int64_t)off.col.size() : 0;
        HIP_CHECK(hipStreamSynchronize(sm));
    }
    phase("outer operator");
    d_sto_A = ar.upload(A.sys_tile_off, sm);
    d_subto_A = ar.upload(A.sub_tile_off, sm);
    // row tiles of 256 rows: one row per thread in the vector kernels
    {
        const int tr = kBlock;
        std::vector<Tile> tiles;
        for (auto &g : rr)
            for (int32_t r0 = 0; r0 < g.nrows; r0 += tr)
                tiles.push_back(Tile{(int32_t)(g.row0 + r0), std::min(tr, g.nrows - r0), g.sub, 0});
        rows = ar.upload(to_dev_tiles(tiles), sm);
        nrow_tiles = (int32_t)tiles.size();
        std::vector<int32_t> so, su;
        tile_offsets(tiles, P.sub_sys, nsys, nsub, so, su);
        d_sto_rows = ar.upload(so, sm);
        d_subto_rows = ar.upload(su, sm);
        HIP_CHECK(hipStreamSynchronize(sm));
    }
    d_sys_sub_off = ar.upload(P.sys_sub_off, sm);
    d_perm = ar.upload(P.perm, sm);
    AZown = ar.upload(P.AZown, sm);
    std::vector<int32_t> offp(P.AZoff.ptr.begin(), P.AZoff.ptr.end());
    AZoffp = ar.upload(offp, sm);
    AZoffc = ar.upload(P.AZoff.col, sm);
    AZoffv = ar.upload(P.AZoff.val, sm);
    t1 = ar.alloc<double>((size_t)nsub * std::max(ndv, 1));
    t2 = ar.alloc<double>((size_t)nsub * std::max(ndv, 1));
    psub = ar.alloc<double>(nsub);
    // GEMV jobs of t2 = E^{-1} t1
    std::vector<GemvJob> jobs;
    std::vector<int32_t> joff(nsys + 1, 0);
    for (int sy = 0; sy < nsys; ++sy) {
        const int m = P.sys_m[sy];
        for (int r0 = 0; r0 < m; r0 += kGemvRows)
            jobs.push_back(GemvJob{sy, r0, m, P.sys_sub_off[sy] * ndv, P.sys_E_off[sy]});
        joff[sy + 1] = (int32_t)jobs.size();
    }
    njobs = (int32_t)jobs.size();
    d_jobs = ar.upload(jobs, sm);
    d_sys_job_off = ar.upload(joff, sm);
    tt_part = ar.alloc<double>(std::max(1, njobs));
    HIP_CHECK(hipStreamSynchronize(sm));
    EinvT = ar.alloc<double>(std::max<int64_t>(1, P.sys_E_off[nsys]));
    b = ar.alloc<double>(n);
    y = ar.alloc<double>(n);
    r = ar.alloc<double>(n);
    p = ar.alloc<double>(n);
    q = ar.alloc<double>(n);
    s = ar.alloc<double>(n);
    w = ar.alloc<double>(n);
    x = ar.alloc<double>(n);
    if (prm.solver == DFAMG_SOLVER_BICGSTAB) {
        rt = ar.alloc<double>(n);
        v = ar.alloc<double>(n);
        ph = ar.alloc<double>(n);
        sh = ar.alloc<double>(n);
        sv = ar.alloc<double>(n);
        tv = ar.alloc<double>(n);
    }
    if (bicg2()) {
        rt = ar.alloc<double>(n);
        b2r1 = ar.alloc<double>(n);
        b2r2 = ar.alloc<double>(n);
        b2u0 = ar.alloc<double>(n);
        b2u1 = ar.alloc<double>(n);
        b2u2 = ar.alloc<double>(n);
        b2pr0 = ar.alloc<double>(n);
        b2pr1 = ar.alloc<double>(n);
        b2pu0 = ar.alloc<double>(n);
        b2pu1 = ar.alloc<double>(n);
    }
    if (fgmres()) {
        const int m = prm.restart;
        fg_ld = (n + 63) / 64 * 64;   // every vector starts on a 512-byte boundary
        fg_mtot = (int64_t)nsub * std::max(ndv, 1);
        fgV = ar.alloc<double>((size_t)(m + 1) * fg_ld);
        fgS = ar.alloc<double>((size_t)m * fg_ld);
        fgT2 = ar.alloc<double>((size_t)m * fg_mtot);
        fg = ar.alloc<FgState>(nsys);
        HIP_CHECK(hipMemsetAsync(fg, 0, sizeof(FgState) * nsys, sm));
        part_fg = ar.alloc<double>((size_t)(m + 1) * nrow_tiles);
        if (prm.coarse_solve == DFAMG_COARSE_CG && ndv > 0) {
            // E of every system in CSR (exact zeros dropped); CG needs it
            // symmetric with a positive diagonal
            std::vector<int64_t> ep(1, 0);
            std::vector<int32_t> ec, co(nsys + 1, 0);
            std::vector<double> ev, dv;
            for (int sy = 0; sy < nsys; ++sy) {
                const int m = P.sys_m[sy];
                const int64_t c0 = (int64_t)P.sys_sub_off[sy] * ndv;
                const double *E = &P.E[P.sys_E_off[sy]];
                double emax = 0.0;
                for (int64_t i = 0; i < (int64_t)m * m; ++i) emax = std::max(emax, std::fabs(E[i]));
                for (int i = 0; i < m; ++i) {
                    if (!(E[(int64_t)i * m + i] > 0.0))
                        throw Error{DFAMG_EINVAL, "the CG coarse solve needs E with a positive diagonal (system " +
                                                      std::to_string(sy) + ")"};
                    for (int j = 0; j < m; ++j) {
                        const double e = E[(int64_t)i * m + j];
                        if (std::fabs(e - E[(int64_t)j * m + i]) > 1e-10 * emax)
                            throw Error{DFAMG_EINVAL, "the CG coarse solve needs a symmetric E (system " +
                                                          std::to_string(sy) + ")"};
                        if (e != 0.0) {
                            ec.push_back((int32_t)(c0 + j));
                            ev.push_back(e);
                        }
                    }
                    ep.push_back((int64_t)ec.size());
                    dv.push_back(1.0 / E[(int64_t)i * m + i]);
                }
                co[sy + 1] = (int32_t)(c0 + m);
            }
            ecg_ptr = ar.upload(ep, sm);
            ecg_col = ar.upload(ec, sm);
            ecg_val = ar.upload(ev, sm);
            ecg_dinv = ar.upload(dv, sm);
            d_sys_coarse_off = ar.upload(co, sm);
            ecg_work = ar.alloc<double>((size_t)3 * fg_mtot);
            for (int sy = 0; sy < nsys; ++sy) ecg_mmax = std::max(ecg_mmax, P.sys_m[sy]);
            ecg_iters = ar.alloc<int64_t>(nsys);
            HIP_CHECK(hipMemsetAsync(ecg_iters, 0, sizeof(int64_t) * nsys, sm));
        }

    }
    part_A = ar.alloc<double>((size_t)A.ntiles * (ndv + 1));
    part_rows = ar.alloc<double>((size_t)nrow_tiles * std::max(ndv + 1, 3));
    // E^{-1} per system (FP64 Gauss-Jordan with partial pivoting on the
    // device): large systems one at a time in column panels with GEMM
    // updates, small ones together with the unblocked elimination
    if (ndv > 0) {
        // large coarse operators are assembled on the device (one operator
        // product per column) and inverted in place there
        bool any_large = false;
        for (int sy = 0; sy < nsys; ++sy) any_large = any_large || P.sys_m[sy] >= kBlockedInverseMin;
        if (any_large) assemble_E(EinvT);
        std::vector<const double *> mats;
        std::vector<int32_t> ns, which;
        std::vector<int64_t> off;
        for (int sy = 0; sy < nsys; ++sy) {
            const int m = P.sys_m[sy];
            if (m >= kBlockedInverseMin) {
                double *Ed = EinvT + P.sys_E_off[sy];   // E assembled on the device above
                bool ok = false;
                try {
                    ok = invert_dense_inplace(sm, Ed, m);
                } catch (const DenseInverseError &e) {
                    throw Error{DFAMG_EHIP, e.msg};
                }
                if (!ok) throw Error{DFAMG_ESINGULAR, "E = Z^T A Z of system " + std::to_string(sy) + " is singular"};
                continue;
            }
            mats.push_back(&P.E[P.sys_E_off[sy]]);
            ns.push_back(m);
            off.push_back(P.sys_E_off[sy]);
            which.push_back(sy);
        }
        if (!mats.empty()) {
            const int bad = invert_on_device<double>(sm, mats, ns, EinvT, off, ns);
            if (bad >= 0)
                throw Error{DFAMG_ESINGULAR,
                            "E = Z^T A Z of system " + std::to_string(which[bad]) + " is singular"};
        }
    }
    phase("vectors, AZ and E^-1");
    // the single-precision copy of E^{-1} for the inexact coarse solve
    if (fgmres() && prm.coarse_solve == DFAMG_COARSE_FP32 && ndv > 0) {
        const int64_t ne = P.sys_E_off[nsys];
        Einv32 = ar.alloc<float>(ne);
        hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, sm, ne, EinvT, Einv32);
        HIP_CHECK(hipGetLastError());
    }

    HIP_CHECK(hipHostMalloc((void **)&h_states, sizeof(SysState) * nsys, hipHostMallocDefault));
    hist_stride = prm.maxiter + 1;
    hist = ar.alloc<double>((size_t)nsys * hist_stride);
    relres_true = ar.alloc<double>(nsys);
    if (prm.precond == DFAMG_PRECOND_AMG) {
        if (prm.precision == DFAMG_PREC_MIXED) {
            auto H = std::make_unique<Hierarchy_dev<float>>();
            H->build(ar, P, sm, prm.spmv_format, prm.autotune != 0, prm.verbose);
            M = std::move(H);
        } else {
            auto H = std::make_unique<Hierarchy_dev<double>>();
            H->build(ar, P, sm, prm.spmv_format, prm.autotune != 0, prm.verbose);
            M = std::move(H);
        }
        part_rs = ar.alloc<double>(std::max(1, M->nslots0()));
        HIP_CHECK(hipMemsetAsync(part_rs, 0, sizeof(double) * std::max(1, M->nslots0()), sm));
        d_sto0 = ar.upload(M->sys_tile_off0(), sm);
        part_rs_job = ar.alloc<double>(std::max(1, M->ncjobs0));
        HIP_CHECK(hipMemsetAsync(part_rs_job, 0, sizeof(double) * std::max(1, M->ncjobs0), sm));
        d_sys_cjob_off0 = ar.upload(M->sys_cjob_off0, sm);
        phase("hierarchy layouts and coarsest inverses");
    } else {
        if (prm.precond == DFAMG_PRECOND_SPAI0) {
            // m_i = a_ii / sum_j a_ij^2 over the rows of the permuted matrix
            std::vector<double> m(n);
            for (int64_t i = 0; i < n; ++i) {
                double d = 0.0, ss = 0.0;
                for (int64_t e = P.A.ptr[i]; e < P.A.ptr[i + 1]; ++e) {
                    ss += P.A.val[e] * P.A.val[e];
                    if (P.A.col[e] == i) d = P.A.val[e];
                }
                if (d == 0.0) throw Error{DFAMG_EINVAL, "SPAI-0 needs a nonzero diagonal"};
                m[i] = d / ss;
            }
            d_spai = ar.upload(m, sm);
        }
        part_rs = ar.alloc<double>(nrow_tiles);
        d_sto0 = d_sto_rows;
        part_rs_job = ar.alloc<double>(1);
        d_sys_cjob_off0 = ar.upload(std::vector<int32_t>(nsys + 1, 0), sm);
    }
    if (prm.profile) {
        prof.init(std::max({prm.graph_iters, 8, fgmres() ? prm.restart : 0}));
        prof.level = prm.profile;
        if (prm.graph_iters > 0 && !probe_graph_events()) {
            // event nodes cannot be captured here: profile with direct launches
            prm.graph_iters = 0;
            graph_profile_fallback = true;
        }
    }
    // algorithmic bytes per launch of the profiled kernels and per iteration
    {
        const double nd = (double)n, nnzA = (double)P.nnz;
        // CSR of A (values, columns, row pointers), v read, q written, and Z
        // at the size it is stored in (one-byte codes and per-subdomain
        // tables when the deflation vectors take few distinct values)
        const double zbytes = zview.code ? zview_bytes : 8.0 * ndv * nd;
        prof.bytes[KID_SPMV] = nnzA * 12.0 + 4.0 * (nd + 1.0) + 16.0 * nd + zbytes;
        {
            const double ib = A.fmt == DFAMG_FORMAT_SELL ? (A.idx16 ? 2.0 : 4.0) : 4.0;
            double b = A.fmt == DFAMG_FORMAT_BSR4
                           ? (double)A.stored * 8.0 + (double)A.stored / 16.0 * 4.0 + 4.0 * (nd / 4.0 + 1.0) + 16.0 * nd
                           : (double)A.stored * (8.0 + ib) + 16.0 * nd;
            if (A.fmt == DFAMG_FORMAT_CSR) b += 4.0 * nd;
            if (A.sorted) b += 2.0 * nd;
            if (outer_split) b += 12.0 * (double)outer_off_nnz + 4.0 * nd;
            b += zbytes;
            outer_layout_bytes = b;
        }
        prof.bytes[KID_UPDATE] = 48.0 * nd + 8.0 * ndv * nd + (ndv ? 12.0 * (double)P.AZoff.nnz() + 4.0 * nd : 0.0);
        prof.bytes[KID_PROJECT] = 8.0 * (double)P.sys_E_off[nsys] + 8.0 * (ndv + 1) * A.ntiles;
        prof.bytes[KID_DIR] = 24.0 * nd;
        if (M)
            for (int k = 0; k < KID_N; ++k)
                if (M->kbytes[k] > 0) prof.bytes[k] = M->kbytes[k];
        bytes_iter = prof.bytes[KID_SPMV] + prof.bytes[KID_UPDATE] + prof.bytes[KID_PROJECT] + prof.bytes[KID_DIR];
        bytes_iter += M ? M->bytes : 16.0 * nd;
        if (prm.solver == DFAMG_SOLVER_BICGSTAB) {
            // two operator products, each followed by the projection and the
            // AZ correction (q, other vector and AZ read, result written), two
            // preconditioner applications, and the vector kernels: p = r +
            // beta (p - omega v) (r, v, p read, p written), s = r - alpha v
            // (r, v read, s written), y += alpha p^ + omega s^ and
            // r = s - omega t with its dots (y, p^, s^, s, t, r~ read; y, r
            // written)
            const double azb = 8.0 * ndv * nd + (ndv ? 12.0 * (double)P.AZoff.nnz() + 4.0 * nd : 0.0);
            prof.bytes[KID_UPDATE] = 64.0 * nd;
            bytes_iter = 2.0 * (prof.bytes[KID_SPMV] + prof.bytes[KID_PROJECT] + (M ? M->bytes : 16.0 * nd) +
                                24.0 * nd + azb) +
                         32.0 * nd + 24.0 * nd + prof.bytes[KID_UPDATE];
        } else if (prm.solver == DFAMG_SOLVER_BICGSTAB2) {
            bytes_iter = 0.0;   // not modelled
        }
        if (fgmres()) {
            // one Arnoldi step at the cycle's mean basis size J = (m + 1) / 2:
            // f = sc (V_j - AZ t2) reads V_j, AZ and writes f; the Gram-Schmidt
            // span forms w = q + AZ t2 (q, AZ read, w written), reads the J
            // basis vectors in each of its three kernels (the fused update +
            // dots kernel reads them twice, counted once: the second read
            // comes from the caches), reads w in the two later kernels, writes
            // w and V_{j+1}, and reads Z for the Z^T V_{j+1} partials
            const double J = 0.5 * (prm.restart + 1);
            const double azb = 8.0 * ndv * nd + (ndv ? 12.0 * (double)P.AZoff.nnz() + 4.0 * nd : 0.0);
            prof.bytes[KID_UPDATE] = 48.0 * nd + azb + 24.0 * J * nd + 8.0 * ndv * nd;
            bytes_iter = prof.bytes[KID_SPMV] + prof.bytes[KID_PROJECT] + (M ? M->bytes : 16.0 * nd) +
                         (16.0 * nd + azb) + prof.bytes[KID_UPDATE];
        }
    }
    HIP_CHECK(hipStreamSynchronize(sm));
    phase("rest");
    setup_device_s = now_s() - t0;
    if (prm.verbose >= 1) std::fprintf(stderr, "[dfamg] device setup %.3f s: %s\n", setup_device_s, phases.c_str());
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

// Outer SpMV launch with the epilogue of `mode` (see k_outer).
void Handle::outer(int mode, hipStream_t st, const double *xin, const double *bin, double *out, bool profiled) {
    if (profiled) prof.mark(KID_SPMV, 0, st);
    launch_outer(mode, ndv(), A, offA, xin, bin, out, zview, part_A, states, d_sub_sys, st);
    if (profiled) prof.mark(KID_SPMV, 1, st);
}

// t1 per subdomain from tile partials, then t2 = E^{-1} t1 per system.
void Handle::project_solve(hipStream_t st, bool in_loop, const int32_t *subto, double *part, int32_t nslots,
                           int with_p0) {
    const int nsub = plan.nsub;
    if (in_loop)
        hipLaunchKernelGGL(k_t1<true>, dim3(nsub), dim3(kBlock), 0, st, part, nslots, subto, ndv(), t1, psub, states,
                           d_sub_sys, with_p0);
    else
        hipLaunchKernelGGL(k_t1<false>, dim3(nsub), dim3(kBlock), 0, st, part, nslots, subto, ndv(), t1, psub, states,
                           d_sub_sys, with_p0);
    if (ndv() > 0) {
        if (in_loop)
            hipLaunchKernelGGL(k_egemv<true>, dim3(njobs), dim3(kBlock), 0, st, d_jobs, EinvT, t1, t2, tt_part, states);
        else
            hipLaunchKernelGGL(k_egemv<false>, dim3(njobs), dim3(kBlock), 0, st, d_jobs, EinvT, t1, t2, tt_part,
                               states);
    }
}

void Handle::precond(hipStream_t st, const double *rin, double *sout, bool profiled) {
    if (ext_precond) {
        ext_precond(st, rin, sout);
    } else if (d_spai) {
        hipLaunchKernelGGL(k_diag_scale, dim3(grid_for_tiles(nrow_tiles)), dim3(kBlock), 0, st, rows, nrow_tiles,
                           d_spai, rin, sout, part_rs, states, d_sub_sys);
    } else if (M) {
        M->apply(st, rin, sout, part_rs, part_rs_job, states, d_sub_sys, (profiled && prof.on) ? &prof : nullptr);
    } else {
        hipLaunchKernelGGL(k_identity, dim3(grid_for_tiles(nrow_tiles)), dim3(kBlock), 0, st, rows, nrow_tiles, rin,
                           sout, part_rs, states, d_sub_sys);
    }
}

// One CG iteration on the deflated system (all systems at once).
void Handle::iteration(hipStream_t st) {
    const dim3 gr(grid_for_tiles(nrow_tiles)), bl(kBlock);
    outer(0, st, p, nullptr, q, true);
    prof.mark(KID_PROJECT, 0, st);
    project_solve(st, true, d_subto_A, part_A, A.ntiles, 1);
    prof.mark(KID_PROJECT, 1, st);
    prof.mark(KID_UPDATE, 0, st);
    with_ndv(ndv(), [&](auto c) {
        if (prm.flexible_cg)
            hipLaunchKernelGGL((k_update<3, decltype(c)::value>), gr, bl, 0, st, rows, nrow_tiles, p, q, y, r, AZown,
                               ndv(), AZoffp, AZoffc, AZoffv, t2, part_rows, states, d_sub_sys, psub, tt_part,
                               ranges(), s);
        else
            hipLaunchKernelGGL((k_update<0, decltype(c)::value>), gr, bl, 0, st, rows, nrow_tiles, p, q, y, r, AZown,
                               ndv(), AZoffp, AZoffc, AZoffv, t2, part_rows, states, d_sub_sys, psub, tt_part,
                               ranges(), nullptr);
    });
    prof.mark(KID_UPDATE, 1, st);
    prof.mark(KID_TEST, 0, st);
    hipLaunchKernelGGL(k_residual_test<0>, dim3(nsys()), dim3(kWideBlock), 0, st, part_rows, d_sto_rows, states, hist,
                       hist_stride, prm.rtol, prm.maxiter, nullptr, psub, ranges());
    prof.mark(KID_TEST, 1, st);
    precond(st, r, s, true);
    prof.mark(KID_DIR, 0, st);
    if (prm.flexible_cg)
        hipLaunchKernelGGL(k_rho_flexible, dim3(nsys()), dim3(kWideBlock), 0, st, part_rs, d_sto0, part_rs_job,
                           d_sys_cjob_off0, part_rows + nrow_tiles, d_sto_rows, states);
    else
        hipLaunchKernelGGL(k_rho<0>, dim3(nsys()), dim3(kWideBlock), 0, st, part_rs, d_sto0, part_rs_job,
                           d_sys_cjob_off0, states);
    hipLaunchKernelGGL(k_cg_direction<false>, dim3(grid_for_tiles((nrow_tiles + 1) / 2)), bl, 0, st, rows, nrow_tiles, s,
                       p, states, d_sub_sys);
    prof.mark(KID_DIR, 1, st);
}

// One BiCGStab iteration on the deflated operator P A (all systems at once).
void Handle::iteration_bicg(hipStream_t st) {
    const dim3 gr(grid_for_tiles(nrow_tiles)), bl(kBlock), gs(nsys()), wb(kWideBlock);
    const int nt = nrow_tiles;
    hipLaunchKernelGGL(k_bicg_p, gr, bl, 0, st, rows, nt, r, v, p, states, d_sub_sys);
    precond(st, p, ph, true);
    // v = P A p^, alpha = rho / (r~, v)
    outer(3, st, ph, nullptr, q, true);
    prof.mark(KID_PROJECT, 0, st);
    project_solve(st, true, d_subto_A, part_A, A.ntiles, 0);
    prof.mark(KID_PROJECT, 1, st);
    with_ndv(ndv(), [&](auto c) {
        hipLaunchKernelGGL((k_bicg_proj<0, decltype(c)::value>), gr, bl, 0, st, rows, nt, q, v, rt, ndv(), AZown,
                           AZoffp, AZoffc, AZoffv, t2, part_rows, nt, states, d_sub_sys);
    });
    hipLaunchKernelGGL(k_bicg_scalar<0>, gs, wb, 0, st, part_rows, nt, d_sto_rows, states, hist, hist_stride,
                       prm.rtol, prm.maxiter);
    // s = r - alpha v and the half-step test
    hipLaunchKernelGGL(k_bicg_s, gr, bl, 0, st, rows, nt, r, v, sv, part_rows, states, d_sub_sys);
    hipLaunchKernelGGL(k_bicg_scalar<1>, gs, wb, 0, st, part_rows, nt, d_sto_rows, states, hist, hist_stride,
                       prm.rtol, prm.maxiter);
    precond(st, sv, sh);
    // t = P A s^, omega = (t, s) / (t, t)
    outer(3, st, sh, nullptr, q);
    project_solve(st, true, d_subto_A, part_A, A.ntiles, 0);
    with_ndv(ndv(), [&](auto c) {
        hipLaunchKernelGGL((k_bicg_proj<1, decltype(c)::value>), gr, bl, 0, st, rows, nt, q, tv, sv, ndv(), AZown,
                           AZoffp, AZoffc, AZoffv, t2, part_rows, nt, states, d_sub_sys);
    });
    hipLaunchKernelGGL(k_bicg_scalar<2>, gs, wb, 0, st, part_rows, nt, d_sto_rows, states, hist, hist_stride,
                       prm.rtol, prm.maxiter);
    // y += alpha p^ + omega s^, r = s - omega t, test, rho
    prof.mark(KID_UPDATE, 0, st);
    hipLaunchKernelGGL(k_bicg_update, gr, bl, 0, st, rows, nt, y, r, ph, sh, sv, tv, rt, part_rows, nt, states,
                       d_sub_sys);
    prof.mark(KID_UPDATE, 1, st);
    prof.mark(KID_TEST, 0, st);
    hipLaunchKernelGGL(k_bicg_scalar<3>, gs, wb, 0, st, part_rows, nt, d_sto_rows, states, hist, hist_stride,
                       prm.rtol, prm.maxiter);
    prof.mark(KID_TEST, 1, st);
}

// One BiCGStab(2) cycle on K = P A M^{-1} (see the kernels' comments)
void Handle::iteration_bicg2(hipStream_t st) {
    const dim3 gr(grid_for_tiles(nrow_tiles)), bl(kBlock), gs(nsys()), wb(kWideBlock);
    const int nt = nrow_tiles;
    double *r0 = r, *r1 = b2r1, *r2 = b2r2, *u0 = b2u0, *u1 = b2u1, *u2 = b2u2;
    // out = P A pre with pre = M^{-1} in, and the partial (other, out) in
    // partial region `region`
    auto K = [&](const double *in, double *pre, double *out, const double *other, int region, bool profiled) {
        precond(st, in, pre, profiled);
        outer(3, st, pre, nullptr, q, profiled);
        if (profiled) prof.mark(KID_PROJECT, 0, st);
        project_solve(st, true, d_subto_A, part_A, A.ntiles, 0);
        if (profiled) prof.mark(KID_PROJECT, 1, st);
        with_ndv(ndv(), [&](auto c) {
            hipLaunchKernelGGL((k_bicg_proj<0, decltype(c)::value>), gr, bl, 0, st, rows, nt, q, out, other, ndv(),
                               AZown, AZoffp, AZoffc, AZoffv, t2, part_rows + (int64_t)region * nt, nt, states,
                               d_sub_sys);
        });
    };
    auto scalar = [&](auto kern) {
        hipLaunchKernelGGL(kern, gs, wb, 0, st, part_rows, nt, d_sto_rows, states, hist, hist_stride, prm.rtol,
                           prm.maxiter);
    };
    const double *cnull = nullptr;
    double *null = nullptr;
    // first BiCG step
    scalar(k_bl_scalar<0>);
    hipLaunchKernelGGL(k_bl_u, gr, bl, 0, st, rows, nt, r0, u0, cnull, null, cnull, null, states, d_sub_sys);
    K(u0, b2pu0, u1, rt, 0, true);
    scalar(k_bl_scalar<2>);
    hipLaunchKernelGGL(k_bl_r, gr, bl, 0, st, rows, nt, r0, u1, null, cnull, null, cnull, y, b2pu0, part_rows, nt,
                       states, d_sub_sys);
    K(r0, b2pr0, r1, rt, 0, false);
    // second BiCG step
    scalar(k_bl_scalar<1>);
    hipLaunchKernelGGL(k_bl_u, gr, bl, 0, st, rows, nt, r0, u0, r1, u1, b2pr0, b2pu0, states, d_sub_sys);
    K(u1, b2pu1, u2, rt, 0, false);
    scalar(k_bl_scalar<2>);
    hipLaunchKernelGGL(k_bl_r, gr, bl, 0, st, rows, nt, r0, u1, r1, u2, b2pr0, b2pu1, y, b2pu0, part_rows, nt,
                       states, d_sub_sys);
    K(r1, b2pr1, r2, r1, 2, false);
    // minimal-residual step
    scalar(k_bl_scalar<3>);
    hipLaunchKernelGGL(k_bl_mgs, gr, bl, 0, st, rows, nt, r0, r1, r2, part_rows, nt, states, d_sub_sys);
    scalar(k_bl_scalar<4>);
    prof.mark(KID_UPDATE, 0, st);
    hipLaunchKernelGGL(k_bl_final, gr, bl, 0, st, rows, nt, y, b2pr0, b2pr1, r0, r1, r2, u0, u1, u2, rt, part_rows,
                       nt, states, d_sub_sys);
    prof.mark(KID_UPDATE, 1, st);
    prof.mark(KID_TEST, 0, st);
    scalar(k_bl_scalar<5>);
    prof.mark(KID_TEST, 1, st);
}

// One restart cycle of flexible GMRES on A x = b (all systems at once; see
// the kernels' comments): `restart` Arnoldi steps, then the update of the
// iterate (held in y) and the first vector of the next cycle.
void Handle::cycle_fgmres(hipStream_t st) {
    const dim3 gr(grid_for_tiles(nrow_tiles)), bl(kBlock), gs(nsys()), wb(kWideBlock);
    const int nt = nrow_tiles, m = prm.restart, nd = ndv();
    for (int j = 0; j < m; ++j) {
        prof.slot = j;
        const double *Vj = fgV + (int64_t)j * fg_ld;
        double *Sj = fgS + (int64_t)j * fg_ld, *t2j = fgT2 + (int64_t)j * fg_mtot;
        double *Vn = fgV + (int64_t)(j + 1) * fg_ld;
        const int J = j + 1;
        // t2_j = E_hat Z^T V_j (the partials of Z^T V_0 come from the outer
        // operator's epilogue, the later ones from the Gram-Schmidt update)
        if (nd > 0) {
            prof.mark(KID_PROJECT, 0, st);
            const bool first = j == 0;
            hipLaunchKernelGGL(k_t1<true>, dim3(plan.nsub), bl, 0, st, first ? part_A : part_rows,
                               first ? A.ntiles : nt, first ? d_subto_A : d_subto_rows, nd, t1, psub, states,
                               d_sub_sys, 0);
            if (ecg_ptr && ecg_mmax <= kEcgLdsRows)
                hipLaunchKernelGGL(k_ecg<true>, gs, wb, sizeof(double) * 3 * ecg_mmax, st, ecg_ptr, ecg_col, ecg_val,
                                   ecg_dinv, d_sys_coarse_off, t1, t2j, ecg_work, fg_mtot, prm.coarse_rtol,
                                   prm.coarse_maxiter, states, ecg_iters);
            else if (ecg_ptr)
                hipLaunchKernelGGL(k_ecg<false>, gs, wb, 0, st, ecg_ptr, ecg_col, ecg_val, ecg_dinv,
                                   d_sys_coarse_off, t1, t2j, ecg_work, fg_mtot, prm.coarse_rtol, prm.coarse_maxiter,
                                   states, ecg_iters);
            else if (Einv32)
                hipLaunchKernelGGL(k_egemv32<true>, dim3(njobs), bl, 0, st, d_jobs, Einv32, t1, t2j, states);
            else
                hipLaunchKernelGGL(k_egemv<true>, dim3(njobs), bl, 0, st, d_jobs, EinvT, t1, t2j, tt_part, states);
            prof.mark(KID_PROJECT, 1, st);
        }
        with_ndv(nd, [&](auto c) {
            hipLaunchKernelGGL((k_fg_rhs<decltype(c)::value>), gr, bl, 0, st, rows, nt, Vj, AZown, nd, AZoffp, AZoffc,
                               AZoffv, t2j, fg, j, r, states, d_sub_sys);
        });
        precond(st, r, Sj, true);
        outer(3, st, Sj, nullptr, q, true);
        prof.mark(KID_UPDATE, 0, st);
        with_ndv(nd, [&](auto c) {
            constexpr int N = decltype(c)::value;
            hipLaunchKernelGGL((k_fg_dots<N>), gr, bl, 0, st, rows, nt, q, w, AZown, nd, AZoffp, AZoffc,
                               AZoffv, t2j, fgV, fg_ld, J, fg, j, part_fg, nt, states, d_sub_sys);
            hipLaunchKernelGGL(k_fg_sum<1>, dim3(J, nsys()), wb, 0, st, part_fg, nt, d_sto_rows, fg, j, states);
            hipLaunchKernelGGL(k_fg_axpy_dots, gr, bl, 0, st, rows, nt, w, fgV, fg_ld, J, fg, part_fg, nt, states,
                               d_sub_sys);
            hipLaunchKernelGGL(k_fg_sum<2>, dim3(J, nsys()), wb, 0, st, part_fg, nt, d_sto_rows, fg, j, states);
            hipLaunchKernelGGL((k_fg_axpy<N>), gr, bl, 0, st, rows, nt, w, Vn, fgV, fg_ld, J, fg, Z, nd,
                               part_rows, nt, states, d_sub_sys);
        });
        prof.mark(KID_UPDATE, 1, st);
        prof.mark(KID_TEST, 0, st);
        hipLaunchKernelGGL(k_fg_givens, gs, wb, 0, st, part_rows, d_sto_rows, fg, states, hist, hist_stride, prm.rtol,
                           prm.maxiter, j);
        prof.mark(KID_TEST, 1, st);
        if (ext_precond) {
            // an external preconditioner does real work even for stopped
            // systems: leave the cycle as soon as every system has stopped
            HIP_CHECK(hipMemcpyAsync(h_states, states, sizeof(SysState) * nsys(), hipMemcpyDeviceToHost, st));
            HIP_CHECK(hipStreamSynchronize(st));
            bool all = true;
            for (int i = 0; i < nsys(); ++i) all = all && h_states[i].done != kRunning;
            if (all) break;
        }
    }
    // x += sum_i y_i z_i, then V_0 = b - A x, its Z^T partials and norm
    hipLaunchKernelGGL(k_fg_solve, dim3((nsys() + 63) / 64), dim3(64), 0, st, fg, nsys());
    with_ndv(nd, [&](auto c) {
        hipLaunchKernelGGL((k_fg_update_x<decltype(c)::value>), gr, bl, 0, st, rows, nt, y, fgS, fg_ld, Z, nd, fgT2,
                           fg_mtot, fg, d_sub_sys);
    });
    outer(1, st, y, b, fgV);
    hipLaunchKernelGGL(k_fg_norm<true>, gr, bl, 0, st, rows, nt, fgV, part_rows, states, d_sub_sys);
    hipLaunchKernelGGL(k_fg_restart, gs, wb, 0, st, part_rows, d_sto_rows, fg, states);
}

// r0 = P(b - A y0), stopping test, s0 = M^{-1} r0, rho0, p0 = s0
void Handle::initial(hipStream_t st) {
    const dim3 gr(grid_for_tiles(nrow_tiles)), bl(kBlock);
    if (fgmres()) {
        // V_0 = b - A x0 with the Z^T V_0 partials, (b, b) per subdomain,
        // ||V_0||, the initial test, then beta, g and sc_0 of the first cycle
        outer(1, st, y, b, fgV);
        hipLaunchKernelGGL(k_t1<false>, dim3(plan.nsub), bl, 0, st, part_A, A.ntiles, d_subto_A, ndv(), t1, psub,
                           states, d_sub_sys, 1);
        hipLaunchKernelGGL(k_fg_norm<false>, gr, bl, 0, st, rows, nrow_tiles, fgV, part_rows, states, d_sub_sys);
        hipLaunchKernelGGL(k_residual_test<1>, dim3(nsys()), dim3(kWideBlock), 0, st, part_rows, d_sto_rows, states,
                           hist, hist_stride, prm.rtol, prm.maxiter, nullptr, psub, ranges());
        hipLaunchKernelGGL(k_zero_null_rhs, gr, bl, 0, st, rows, nrow_tiles, y, states, d_sub_sys);
        hipLaunchKernelGGL(k_fg_restart, dim3(nsys()), dim3(kWideBlock), 0, st, part_rows, d_sto_rows, fg, states);
        return;
    }
    outer(1, st, y, b, w);
    project_solve(st, false, d_subto_A, part_A, A.ntiles, 1);
    with_ndv(ndv(), [&](auto c) {
        hipLaunchKernelGGL((k_update<1, decltype(c)::value>), gr, bl, 0, st, rows, nrow_tiles, nullptr, w, nullptr, r,
                           AZown, ndv(), AZoffp, AZoffc, AZoffv, t2, part_rows, states, d_sub_sys, psub, tt_part,
                           ranges(), nullptr);
    });
    hipLaunchKernelGGL(k_residual_test<1>, dim3(nsys()), dim3(kWideBlock), 0, st, part_rows, d_sto_rows, states, hist,
                       hist_stride, prm.rtol, prm.maxiter, nullptr, psub, ranges());
    hipLaunchKernelGGL(k_zero_null_rhs, gr, bl, 0, st, rows, nrow_tiles, y, states, d_sub_sys);
    if (bicg()) {
        // r~ = r0, v = p = 0, rho = (r~, r0), rho_old = alpha = omega = 1
        hipLaunchKernelGGL(k_copy, gr, bl, 0, st, rows, nrow_tiles, r, rt);
        hipLaunchKernelGGL(k_copy, gr, bl, 0, st, rows, nrow_tiles, (const double *)nullptr, v);
        hipLaunchKernelGGL(k_copy, gr, bl, 0, st, rows, nrow_tiles, (const double *)nullptr, p);
        hipLaunchKernelGGL(k_bicg_scalar<4>, dim3(nsys()), dim3(kWideBlock), 0, st, part_rows, nrow_tiles,
                           d_sto_rows, states, hist, hist_stride, prm.rtol, prm.maxiter);
        return;
    }
    if (bicg2()) {
        // r~ = r0, u0 = 0, rho0 = omega = 1, alpha = 0, (r0, r~) = ||r0||^2
        hipLaunchKernelGGL(k_copy, gr, bl, 0, st, rows, nrow_tiles, r, rt);
        hipLaunchKernelGGL(k_copy, gr, bl, 0, st, rows, nrow_tiles, (const double *)nullptr, b2u0);
        hipLaunchKernelGGL(k_bl_scalar<6>, dim3(nsys()), dim3(kWideBlock), 0, st, part_rows, nrow_tiles, d_sto_rows,
                           states, hist, hist_stride, prm.rtol, prm.maxiter);
        return;
    }
    precond(st, r, s);
    hipLaunchKernelGGL(k_rho<1>, dim3(nsys()), dim3(kWideBlock), 0, st, part_rs, d_sto0, part_rs_job,
                       d_sys_cjob_off0, states);
    hipLaunchKernelGGL(k_cg_direction<true>, dim3(grid_for_tiles((nrow_tiles + 1) / 2)), bl, 0, st, rows, nrow_tiles, s,
                       p, states, d_sub_sys);
}

// x = y + Z E^{-1} Z^T (b - A y), then ||b - A x|| / ||b||
void Handle::finish(hipStream_t st) {
    const dim3 gr(grid_for_tiles(nrow_tiles)), bl(kBlock);
    if (fgmres()) {
        // the iterate solves A x = b itself: no recovery step
        hipLaunchKernelGGL(k_copy, gr, bl, 0, st, rows, nrow_tiles, (const double *)y, x);
        outer(2, st, x, b, w);
        hipLaunchKernelGGL(k_residual_test<2>, dim3(nsys()), dim3(kWideBlock), 0, st, part_A, d_sto_A, states, hist,
                           hist_stride, prm.rtol, prm.maxiter, relres_true, psub, ranges());
        return;
    }
    if (bicg()) hipLaunchKernelGGL(k_bicg_halffix, gr, bl, 0, st, rows, nrow_tiles, y, ph, states, d_sub_sys);
    outer(1, st, y, b, w);
    project_solve(st, false, d_subto_A, part_A, A.ntiles, 0);
    with_ndv(ndv(), [&](auto c) {
        hipLaunchKernelGGL((k_expand<decltype(c)::value>), gr, bl, 0, st, rows, nrow_tiles, y, Z, ndv(), t2, x);
    });
    outer(2, st, x, b, w);
    hipLaunchKernelGGL(k_residual_test<2>, dim3(nsys()), dim3(kWideBlock), 0, st, part_A, d_sto_A, states, hist,
                       hist_stride, prm.rtol, prm.maxiter, relres_true, psub, ranges());
}

void Handle::launch_iterations(int k) {
    if (fgmres()) {
        // one restart cycle per call (one captured graph per cycle)
        chunk_events = prof.on;
        if (prm.graph_iters <= 0) {
            prof.clear_used();
            cycle_fgmres(stream);
            return;
        }
        if (!graph_exec) {
            prof.capturing = prof.on;
            HIP_CHECK(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeRelaxed));
            cycle_fgmres(cap_stream);
            HIP_CHECK(hipStreamEndCapture(cap_stream, &graph));
            HIP_CHECK(hipGraphInstantiate(&graph_exec, graph, nullptr, nullptr, 0));
            graph_k = prm.restart;
            prof.capturing = false;
        }
        HIP_CHECK(hipGraphLaunch(graph_exec, stream));
        return;
    }
    if (prm.graph_iters <= 0) {
        prof.clear_used();
        for (int i = 0; i < k; ++i) {
            prof.slot = i;
            if (bicg()) iteration_bicg(stream);
            else if (bicg2()) iteration_bicg2(stream);
            else iteration(stream);
        }
        chunk_events = prof.on;
        return;
    }
    auto capture = [&](bool events, hipGraph_t &g, hipGraphExec_t &ge) {
        prof.capturing = prof.on && events;
        prof.suppress = !events;
        HIP_CHECK(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeRelaxed));
        for (int i = 0; i < prm.graph_iters; ++i) {
            prof.slot = i;
            if (bicg()) iteration_bicg(cap_stream);
            else if (bicg2()) iteration_bicg2(cap_stream);
            else iteration(cap_stream);
        }
        HIP_CHECK(hipStreamEndCapture(cap_stream, &g));
        HIP_CHECK(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
        prof.capturing = false;
        prof.suppress = false;
    };
    if (!graph_exec) {
        capture(true, graph, graph_exec);
        graph_k = prm.graph_iters;
        if (prof.on && prof.level < 2) capture(false, graph_plain, graph_exec_plain);
    }
    // profile = 1: events in the first chunk of a solve only
    const bool events = !graph_exec_plain || want_events;
    for (int i = 0; i < k; i += graph_k) HIP_CHECK(hipGraphLaunch(events ? graph_exec : graph_exec_plain, stream));
    chunk_events = prof.on && events;
    want_events = false;
}

// E = Z^T A Z of every system assembled on the device into Eout (row-major
// blocks at the systems' E offsets): for each coarse column c (subdomain s,
// vector k) v = Z e_c goes through the outer operator (mode 3, whose
// epilogue leaves the Z^T (A v) partials of every tile) and the per-subdomain
// sums are column c of its system's block.  Uses the vectors x and q and
// resets the Krylov state.
void Handle::assemble_E(double *Eout) {
    const int nd = ndv();
    if (nd == 0) return;
    const Plan &P = plan;
    const dim3 gr(grid_for_tiles(nrow_tiles)), bl(kBlock);
    HIP_CHECK(hipMemsetAsync(states, 0, sizeof(SysState) * P.nsys, stream));
    for (int sy = 0; sy < P.nsys; ++sy) {
        const int m = P.sys_m[sy];
        const int64_t c0 = (int64_t)P.sys_sub_off[sy] * nd;
        for (int sub = P.sys_sub_off[sy]; sub < P.sys_sub_off[sy + 1]; ++sub)
            for (int k = 0; k < nd; ++k) {
                const int col = (int)((int64_t)sub * nd + k - c0);
                hipLaunchKernelGGL(k_zcol, gr, bl, 0, stream, rows, nrow_tiles, Z, nd, sub, k, x);
                outer(3, stream, x, nullptr, q);
                hipLaunchKernelGGL(k_t1<false>, dim3(P.nsub), bl, 0, stream, part_A, A.ntiles, d_subto_A, nd, t1, psub,
                                   states, d_sub_sys, 0);
                hipLaunchKernelGGL(k_ecol, dim3((m + 255) / 256), dim3(256), 0, stream, t1, c0, m, col,
                                   Eout + P.sys_E_off[sy]);
            }
    }
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(stream));
}

// A solve that fits in one FGMRES cycle (maxiter <= restart), issued on the
// handle's stream without any host synchronisation: the inner solves of a
// composite preconditioner.  The iterations taken are added to *iter_acc on
// the device.
void Handle::solve_one_cycle(const double *rhs, double *xio, int64_t *iter_acc) {
    if (!fgmres() || prm.maxiter > prm.restart)
        throw Error{DFAMG_EINVAL, "a single-cycle solve needs FGMRES with maxiter <= restart"};
    const int64_t n = plan.n;
    const int nb = (int)((n + 255) / 256);
    hipLaunchKernelGGL(k_gather, dim3(nb), dim3(256), 0, stream, n, d_perm, rhs, b);
    hipLaunchKernelGGL(k_gather, dim3(nb), dim3(256), 0, stream, n, d_perm, xio, y);
    have_rhs = true;
    initial(stream);
    launch_iterations(prm.restart);
    finish(stream);
    hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(256), 0, stream, n, d_perm, x, xio);
    hipLaunchKernelGGL(k_add_iters, dim3(1), dim3(64), 0, stream, states, nsys(), iter_acc);
    HIP_CHECK(hipGetLastError());
}

dfamg_status Handle::run_solve(const double *rhs, double *xio) {
    const double t0 = now_s();
    const int64_t n = plan.n;
    const int nsys = plan.nsys;
    const int nb = (int)((n + 255) / 256);
    hipLaunchKernelGGL(k_gather, dim3(nb), dim3(256), 0, stream, n, d_perm, rhs, b);
    hipLaunchKernelGGL(k_gather, dim3(nb), dim3(256), 0, stream, n, d_perm, xio, y);
    if (ecg_iters) HIP_CHECK(hipMemsetAsync(ecg_iters, 0, sizeof(int64_t) * nsys, stream));
    have_rhs = true;
    initial(stream);
    HIP_CHECK(hipGetLastError());
    const int chunk = fgmres() ? prm.restart : (prm.graph_iters > 0 ? prm.graph_iters : 8);
    int done_iters = 0;
    want_events = true;
    chunk_events = false;
    std::vector<int32_t> it_before(nsys, 0);
    bool first = true;
    for (;;) {
        HIP_CHECK(hipMemcpyAsync(h_states, states, sizeof(SysState) * nsys, hipMemcpyDeviceToHost, stream));
        HIP_CHECK(hipStreamSynchronize(stream));
        if (!first && prof.on && chunk_events) {
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
    std::vector<int64_t> cit(ecg_iters ? nsys : 0);
    if (ecg_iters) HIP_CHECK(hipMemcpyAsync(cit.data(), ecg_iters, sizeof(int64_t) * nsys, hipMemcpyDeviceToHost, stream));
    HIP_CHECK(hipStreamSynchronize(stream));
    coarse_iters_last = 0;
    for (int64_t c : cit) coarse_iters_last += c;
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

void Handle::apply_op(int op, const double *in, double *out) {
    const int64_t n = plan.n;
    const int nb = (int)((n + 255) / 256);
    const dim3 gr(grid_for_tiles(nrow_tiles)), bl(kBlock);
    hipStream_t st = stream;
    hipLaunchKernelGGL(k_gather, dim3(nb), dim3(256), 0, st, n, d_perm, in, w);
    HIP_CHECK(hipMemsetAsync(states, 0, sizeof(SysState) * plan.nsys, st));
    switch (op) {
        case DFAMG_OP_SPMV:
            outer(4, st, w, nullptr, x);
            break;
        case DFAMG_OP_PROJECT:
            hipLaunchKernelGGL(k_zt_partial, gr, bl, 0, st, rows, nrow_tiles, w, Z, ndv(), part_rows, nrow_tiles);
            project_solve(st, false, d_subto_rows, part_rows, nrow_tiles, 0);
            with_ndv(ndv(), [&](auto c) {
                hipLaunchKernelGGL((k_update<2, decltype(c)::value>), gr, bl, 0, st, rows, nrow_tiles, nullptr, w,
                                   nullptr, x, AZown, ndv(), AZoffp, AZoffc, AZoffv, t2, part_rows, states, d_sub_sys,
                                   psub, tt_part, ranges(), nullptr);
            });
            break;
        case DFAMG_OP_PRECOND:
            precond(st, w, x);
            break;
        case DFAMG_OP_RECOVER:
            if (!have_rhs) throw Error{DFAMG_EINVAL, "RECOVER needs a previous solve (for b)"};
            outer(1, st, w, b, q);
            project_solve(st, false, d_subto_A, part_A, A.ntiles, 0);
            with_ndv(ndv(), [&](auto c) {
                hipLaunchKernelGGL((k_expand<decltype(c)::value>), gr, bl, 0, st, rows, nrow_tiles, w, Z, ndv(), t2, x);
            });
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

namespace dfamg {

// Schur pressure correction (section "Navier-Stokes problem"): the velocity
// and pressure blocks, the two inner solvers and the preconditioner step
// that the outer FGMRES handle calls.
struct SchurParts {
    std::unique_ptr<Handle> K, P;        // velocity solves, pressure solves
    DevArena ar;
    hipStream_t stream = nullptr;
    int64_t nu = 0, np = 0;
    int64_t *uidx = nullptr, *pidx = nullptr;
    int64_t *Dp = nullptr, *Gp = nullptr;
    int32_t *Dc = nullptr, *Gc = nullptr;
    double *Dv = nullptr, *Gv = nullptr;
    double *ru = nullptr, *rp = nullptr, *uh = nullptr, *t = nullptr, *p = nullptr, *t2 = nullptr, *u = nullptr;
    int64_t *d_iters = nullptr;          // device: velocity, pressure inner iterations

    static dim3 grid(int64_t m) { return dim3((unsigned)((m + 255) / 256)); }
    static dim3 rgrid(int64_t rows) {   // k_csr_resid: kBlock / kCsrLanes rows per block
        const int64_t per = kBlock / kCsrLanes;
        return dim3((unsigned)((rows + per - 1) / per));
    }

    // x = approximate H^{-1} rhs from x = 0 in one FGMRES cycle (maxiter =
    // restart), without host synchronisation; a solve that reaches its step
    // limit (or breaks down) returns its last iterate
    void inner(Handle &H, const double *rhs, double *x, int64_t m, int64_t *acc) {
        HIP_CHECK(hipMemsetAsync(x, 0, sizeof(double) * m, stream));
        H.solve_one_cycle(rhs, x, acc);
    }

    // (u, p) for the residual r, both in the whole system's numbering
    void apply(hipStream_t st, const double *rin, double *sout) {
        hipLaunchKernelGGL(k_gather_idx, grid(nu), dim3(256), 0, st, nu, uidx, rin, ru);
        hipLaunchKernelGGL(k_gather_idx, grid(np), dim3(256), 0, st, np, pidx, rin, rp);
        inner(*K, ru, uh, nu, d_iters);
        hipLaunchKernelGGL(k_csr_resid, rgrid(np), dim3(kBlock), 0, st, np, Dp, Dc, Dv, uh, rp, t);
        inner(*P, t, p, np, d_iters + 1);
        hipLaunchKernelGGL(k_csr_resid, rgrid(nu), dim3(kBlock), 0, st, nu, Gp, Gc, Gv, p, ru, t2);
        inner(*K, t2, u, nu, d_iters);
        hipLaunchKernelGGL(k_scatter_idx, grid(nu), dim3(256), 0, st, nu, uidx, u, sout);
        hipLaunchKernelGGL(k_scatter_idx, grid(np), dim3(256), 0, st, np, pidx, p, sout);
        HIP_CHECK(hipGetLastError());
    }
};

}  // namespace dfamg

struct dfamg_handle_s {
    Handle h;
    std::unique_ptr<SchurParts> schur;   // set for a Schur pressure-correction handle
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
        throw Error{DFAMG_ENOGPU, std::string("the library is compiled for gfx950, device is ") + prop.gcnArchName};
}

// Builds a handle in place (validation, host plan, device setup).
void init_handle(Handle &H, const dfamg_params &p, int64_t n, const int64_t *row_ptr, const int32_t *col,
                 const double *val, const int32_t *part, int32_t nsub, int32_t ndv, const double *Z, void *stream) {
    if (p.setup_device) {
        validate_params(p);
        check_device();
    }
    build_plan(H.plan, p, 1, nullptr, n, row_ptr, col, val, part, nsub, ndv, Z, stream);
    check_device();
    H.prm = p;
    H.stream = static_cast<hipStream_t>(stream);
    HIP_CHECK(hipGetDevice(&H.device));
    HIP_CHECK(hipStreamCreateWithFlags(&H.cap_stream, hipStreamNonBlocking));
    H.setup_device();
}

// CSR block of the given rows restricted to the columns that have a position
// in pos (-1: column outside the block), columns renumbered by pos, sorted.
struct HostCsr {
    std::vector<int64_t> ptr{0};
    std::vector<int32_t> col;
    std::vector<double> val;
};

HostCsr extract_block(const int64_t *row_ptr, const int32_t *col, const double *val, const std::vector<int64_t> &rows,
                      const std::vector<int64_t> &pos) {
    HostCsr B;
    for (int64_t i : rows) {
        std::vector<std::pair<int32_t, double>> e;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            if (pos[col[k]] >= 0) e.emplace_back((int32_t)pos[col[k]], val[k]);
        std::sort(e.begin(), e.end());
        for (auto &x : e) {
            B.col.push_back(x.first);
            B.val.push_back(x.second);
        }
        B.ptr.push_back((int64_t)B.col.size());
    }
    return B;
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
        if (p.setup_device) {
        validate_params(p);
        check_device();
    }
        build_plan(H->h.plan, p, nsys, sys_row_off, n, row_ptr, col, val, part, nsub, ndv, Z, stream);
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


// ---------------------------------------------------------------------------
// Workspace of dfamg_dense_inverse_noalloc: one static array per device,
// holding the job record, the offsets, the pivot column and the augmented
// matrix [A | I] of the unblocked Gauss-Jordan elimination.  Host code never
// passes `scratch` itself to a kernel (in host code the name is a host-side
// stand-in, not a device address): it uses the address that
// hipGetSymbolAddress returns on each device, looked up once per device.
// ---------------------------------------------------------------------------
constexpr int kNoAllocMaxN = DFAMG_NOALLOC_MAX_N;
constexpr int64_t kNoAllocHeader = 64;                      // doubles: job, col_off, out_off, out_ld
constexpr int64_t kNoAllocColk = kNoAllocHeader;            // n doubles (pivot column)
constexpr int64_t kNoAllocAug = kNoAllocColk + kNoAllocMaxN; // n x 2n doubles
constexpr int64_t kNoAllocDoubles = kNoAllocAug + (int64_t)kNoAllocMaxN * 2 * kNoAllocMaxN;
static_assert(kNoAllocAug * 8 % 256 == 0, "augmented matrix 256-byte aligned");

static __device__ __align__(256) double scratch[kNoAllocDoubles];

// Fills the job record and offsets of one n x n matrix and its augmented
// copy [a | I] (row-major n x 2n) from the device matrix a.
__global__ void k_noalloc_init(double *__restrict__ ws, const double *__restrict__ a, int n) {
    const int64_t w2 = 2 * (int64_t)n;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        InvJob *job = reinterpret_cast<InvJob *>(ws);
        job->n = n;
        job->singular = 0;
        job->aug_off = 0;
        int64_t *col_off = reinterpret_cast<int64_t *>(ws + 8);
        col_off[0] = 0;
        col_off[1] = n;
        *reinterpret_cast<int64_t *>(ws + 12) = 0;   // out_off
        *reinterpret_cast<int32_t *>(ws + 14) = n;   // out_ld
    }
    double *aug = ws + kNoAllocAug;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)n * w2;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / w2, j = e % w2;
        aug[e] = j < n ? a[i * n + j] : (j - n == i ? 1.0 : 0.0);
    }
}

// Device address of `scratch` on the current device, looked up on the first
// call on that device.
double *noalloc_workspace() {
    static std::mutex mu;
    static std::map<int, double *> ptrs;
    int dev = 0;
    HIP_CHECK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto it = ptrs.find(dev);
    if (it != ptrs.end()) return it->second;
    double *p = nullptr;
    HIP_CHECK(hipGetSymbolAddress(reinterpret_cast<void **>(&p), HIP_SYMBOL(scratch)));
    if (!p) throw Error{DFAMG_EHIP, "hipGetSymbolAddress returned no address for the workspace"};
    ptrs[dev] = p;
    return p;
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
    p->autotune = 1;
    p->graph_iters = 16;
    p->host_threads = 0;
    p->verbose = 0;
    p->profile = 0;
    p->restart = 30;
    p->coarse_solve = DFAMG_COARSE_EXACT;
    p->coarse_rtol = 1e-2;
    p->coarse_maxiter = 100;
    p->flexible_cg = 0;
    p->npre = 1;
    p->npost = 1;
    p->setup_device = 0;
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
        if (h->schur) HIP_CHECK(hipMemsetAsync(h->schur->d_iters, 0, sizeof(int64_t) * 2, H.stream));
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
    if (h->schur) {
        H.err = "dfamg_apply does not take a Schur pressure-correction handle";
        return DFAMG_EINVAL;
    }
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
        if (H.M) {
            o->format_level[l] = H.M->fmt[l];
            o->lanes_level[l] = H.M->par[l];
        }
    }
    o->format_outer = H.A.fmt;
    o->outer_layout_bytes = H.outer_layout_bytes;
    o->coarse_iters = H.coarse_iters_last;
    if (h->schur) {
        int64_t it[2] = {0, 0};
        if (hipMemcpy(it, h->schur->d_iters, sizeof(it), hipMemcpyDeviceToHost) == hipSuccess) {
            o->schur_inner_iters[0] = it[0];
            o->schur_inner_iters[1] = it[1];
        }
    }
    {
        const std::string t = "outer " + describe(H.A) + (H.outer_split ? "+couplings" : "") +
                              (H.M ? ";" + H.M->layouts : std::string());
        std::snprintf(o->layouts, sizeof(o->layouts), "%s", t.c_str());
    }
    o->setup_host_s = P.host_seconds;
    o->setup_device_s = H.setup_device_s;
    o->solve_s = H.solve_s;
    o->device_bytes = H.ar.bytes;
    o->bytes_per_iter = H.bytes_iter;
    o->setup_hierarchy_s = P.hier_seconds;
    o->setup_hierarchy_device = P.hier_on_device;
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
        if (p.setup_device) {
        validate_params(p);
        check_device();
    }
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
    if (!H || level < 0 || level >= H->nlevels() || (which >= 1 && level + 1 >= H->nlevels()) || which < 0 ||
        which > 3) {
        g_last_error = "bad plan, subdomain, level or matrix";
        return DFAMG_EINVAL;
    }
    Csr Msm;   // which 3: the smoother as a matrix
    if (which == 3) {
        const Level &Lv = H->lv[level];
        const int64_t n = Lv.A.nrows;
        const int bs = Lv.mb.empty() ? 1 : (int)(Lv.mb.size() / std::max<int64_t>(n, 1));
        Msm.nrows = Msm.ncols = n;
        Msm.ptr.assign(1, 0);
        for (int64_t i = 0; i < n; ++i) {
            if (Lv.mb.empty()) {
                Msm.col.push_back((int32_t)i);
                Msm.val.push_back(Lv.m[i]);
            } else {
                const int64_t nb = i / bs * bs;
                for (int k = 0; k < bs; ++k) {
                    Msm.col.push_back((int32_t)(nb + k));
                    Msm.val.push_back(Lv.mb[(size_t)i * bs + k]);
                }
            }
            Msm.ptr.push_back((int64_t)Msm.col.size());
        }
    }
    const Csr &M = which == 0 ? H->lv[level].A : which == 1 ? H->lv[level].P : which == 2 ? H->lv[level].B : Msm;
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

dfamg_status dfamg_setup_schur(const dfamg_params *prm, int64_t n, const int64_t *row_ptr, const int32_t *col,
                               const double *val, const int32_t *pmask, const int32_t *part, int32_t nsub,
                               int32_t ndv, const double *Z, void *stream, dfamg_handle *out) {
    if (!out) {
        g_last_error = "out is NULL";
        return DFAMG_EINVAL;
    }
    *out = nullptr;
    return guarded(nullptr, [&]() -> dfamg_status {
        dfamg_params p;
        if (prm) p = *prm;
        else dfamg_params_default(&p);
        if (p.solver != DFAMG_SOLVER_FGMRES) throw Error{DFAMG_EINVAL, "the Schur solver runs FGMRES (solver = FGMRES)"};
        if (n < 2 || !row_ptr || !col || !val || !pmask) throw Error{DFAMG_EINVAL, "bad system arrays"};
        for (int64_t i = 0; i < n; ++i)
            if (row_ptr[i + 1] < row_ptr[i]) throw Error{DFAMG_EINVAL, "row_ptr not monotone"};
        for (int64_t k = 0; k < row_ptr[n]; ++k)
            if (col[k] < 0 || col[k] >= n) throw Error{DFAMG_EINVAL, "column index out of range"};
        std::vector<int64_t> urows, prows, pos(n, -1);
        for (int64_t i = 0; i < n; ++i) {
            if (pmask[i]) {
                pos[i] = (int64_t)prows.size();
                prows.push_back(i);
            } else {
                pos[i] = (int64_t)urows.size();
                urows.push_back(i);
            }
        }
        if (urows.empty() || prows.empty()) throw Error{DFAMG_EINVAL, "the velocity or the pressure block is empty"};
        std::vector<int64_t> upos(n, -1), ppos(n, -1);
        for (int64_t i = 0; i < n; ++i) (pmask[i] ? ppos : upos)[i] = pos[i];
        HostCsr K = extract_block(row_ptr, col, val, urows, upos);
        HostCsr G = extract_block(row_ptr, col, val, urows, ppos);
        HostCsr D = extract_block(row_ptr, col, val, prows, upos);
        HostCsr S = extract_block(row_ptr, col, val, prows, ppos);
        const int64_t nu = (int64_t)urows.size(), np = (int64_t)prows.size();
        // S^ = S - D diag(K)^{-1} G, rows accumulated densely over a marker
        std::vector<double> kinv(nu);
        for (int64_t i = 0; i < nu; ++i) {
            double d = 0.0;
            for (int64_t e = K.ptr[i]; e < K.ptr[i + 1]; ++e)
                if (K.col[e] == i) d = K.val[e];
            if (d == 0.0) throw Error{DFAMG_EINVAL, "zero diagonal entry in the velocity block"};
            kinv[i] = 1.0 / d;
        }
        HostCsr Sh;
        {
            std::vector<double> acc(np, 0.0);
            std::vector<int64_t> mark(np, -1);
            std::vector<int32_t> cols;
            for (int64_t r = 0; r < np; ++r) {
                cols.clear();
                auto add = [&](int32_t c, double v) {
                    if (mark[c] != r) {
                        mark[c] = r;
                        acc[c] = 0.0;
                        cols.push_back(c);
                    }
                    acc[c] += v;
                };
                for (int64_t e = S.ptr[r]; e < S.ptr[r + 1]; ++e) add(S.col[e], S.val[e]);
                for (int64_t e = D.ptr[r]; e < D.ptr[r + 1]; ++e) {
                    const int32_t k = D.col[e];
                    const double f = D.val[e] * kinv[k];
                    for (int64_t g = G.ptr[k]; g < G.ptr[k + 1]; ++g) add(G.col[g], -f * G.val[g]);
                }
                std::sort(cols.begin(), cols.end());
                for (int32_t c : cols) {
                    Sh.col.push_back(c);
                    Sh.val.push_back(acc[c]);
                }
                Sh.ptr.push_back((int64_t)Sh.col.size());
            }
        }
        auto H = std::make_unique<dfamg_handle_s>();
        auto parts = std::make_unique<SchurParts>();
        parts->stream = static_cast<hipStream_t>(stream);
        parts->nu = nu;
        parts->np = np;
        // velocity solves: FGMRES(5) to 1e-3 with the local SPAI-0
        {
            dfamg_params q = p;
            q.solver = DFAMG_SOLVER_FGMRES;
            q.restart = 5;
            q.maxiter = 5;
            q.rtol = 1e-3;
            q.precond = DFAMG_PRECOND_SPAI0;
            q.coarse_solve = DFAMG_COARSE_EXACT;
            q.block_size = 1;
            q.profile = 0;
            q.graph_iters = 16;
            std::vector<int32_t> part0(nu, 0);
            parts->K = std::make_unique<Handle>();
            init_handle(*parts->K, q, nu, K.ptr.data(), K.col.data(), K.val.data(), part0.data(), 1, 0, nullptr,
                        stream);
        }
        // pressure solves: FGMRES(20) to 1e-2, deflation + block-local AMG of S^
        {
            dfamg_params q = p;
            q.solver = DFAMG_SOLVER_FGMRES;
            q.restart = 20;
            q.maxiter = 20;
            q.rtol = 1e-2;
            q.precond = DFAMG_PRECOND_AMG;
            q.coarse_solve = DFAMG_COARSE_EXACT;
            q.block_size = 1;
            q.profile = 0;
            q.graph_iters = 16;
            parts->P = std::make_unique<Handle>();
            init_handle(*parts->P, q, np, Sh.ptr.data(), Sh.col.data(), Sh.val.data(), part, nsub, ndv, Z, stream);
        }
        // the outer FGMRES on the whole system, direct launches (the
        // preconditioner synchronises)
        {
            dfamg_params q = p;
            q.precond = DFAMG_PRECOND_NONE;
            q.coarse_solve = DFAMG_COARSE_EXACT;
            q.graph_iters = 0;
            q.profile = 0;
            std::vector<int32_t> part0(n, 0);
            init_handle(H->h, q, n, row_ptr, col, val, part0.data(), 1, 0, nullptr, stream);
        }
        hipStream_t sm = parts->stream;
        DevArena &ar = parts->ar;
        parts->uidx = ar.upload(urows, sm);
        parts->pidx = ar.upload(prows, sm);
        parts->Dp = ar.upload(D.ptr, sm);
        parts->Dc = ar.upload(D.col, sm);
        parts->Dv = ar.upload(D.val, sm);
        parts->Gp = ar.upload(G.ptr, sm);
        parts->Gc = ar.upload(G.col, sm);
        parts->Gv = ar.upload(G.val, sm);
        parts->ru = ar.alloc<double>(nu);
        parts->uh = ar.alloc<double>(nu);
        parts->t2 = ar.alloc<double>(nu);
        parts->u = ar.alloc<double>(nu);
        parts->rp = ar.alloc<double>(np);
        parts->t = ar.alloc<double>(np);
        parts->p = ar.alloc<double>(np);
        parts->d_iters = ar.alloc<int64_t>(2);
        HIP_CHECK(hipMemsetAsync(parts->d_iters, 0, sizeof(int64_t) * 2, sm));
        SchurParts *sp = parts.get();
        H->h.ext_precond = [sp](hipStream_t st, const double *rin, double *sout) { sp->apply(st, rin, sout); };
        H->schur = std::move(parts);
        *out = H.release();
        return DFAMG_OK;
    });
}

dfamg_status dfamg_coarse_inverse(dfamg_handle h, int32_t sys, int32_t *m, double *Einv, int64_t cap) {
    if (!h) {
        g_last_error = "null handle";
        return DFAMG_EINVAL;
    }
    Handle &H = h->h;
    return guarded(&H.err, [&]() -> dfamg_status {
        const Plan &P = H.plan;
        if (sys < 0 || sys >= P.nsys) throw Error{DFAMG_EINVAL, "system out of range"};
        const int32_t mm = P.ndv > 0 ? P.sys_m[sys] : 0;
        if (m) *m = mm;
        if (!Einv) return DFAMG_OK;
        if (cap < (int64_t)mm * mm) throw Error{DFAMG_EINVAL, "buffer too small for E^{-1}"};
        if (mm == 0) return DFAMG_OK;
        HIP_CHECK(hipSetDevice(H.device));
        HIP_CHECK(hipMemcpyAsync(Einv, H.EinvT + P.sys_E_off[sys], sizeof(double) * (size_t)mm * mm,
                                 hipMemcpyDeviceToHost, H.stream));
        HIP_CHECK(hipStreamSynchronize(H.stream));
        return DFAMG_OK;
    });
}

dfamg_status dfamg_coarse_operator(dfamg_handle h, int32_t sys, int32_t *m, double *E, int64_t cap) {
    if (!h) {
        g_last_error = "null handle";
        return DFAMG_EINVAL;
    }
    Handle &H = h->h;
    return guarded(&H.err, [&]() -> dfamg_status {
        const Plan &P = H.plan;
        if (sys < 0 || sys >= P.nsys) throw Error{DFAMG_EINVAL, "system out of range"};
        const int32_t mm = P.ndv > 0 ? P.sys_m[sys] : 0;
        if (m) *m = mm;
        if (!E) return DFAMG_OK;
        if (cap < (int64_t)mm * mm) throw Error{DFAMG_EINVAL, "buffer too small for E"};
        if (mm == 0) return DFAMG_OK;
        HIP_CHECK(hipSetDevice(H.device));
        DevArena tmp;
        double *d = tmp.alloc<double>(std::max<int64_t>(1, P.sys_E_off[P.nsys]));
        H.assemble_E(d);
        HIP_CHECK(hipMemcpy(E, d + P.sys_E_off[sys], sizeof(double) * (size_t)mm * mm, hipMemcpyDeviceToHost));
        return DFAMG_OK;
    });
}

dfamg_status dfamg_dense_inverse(const double *a, int32_t n, int32_t method, double *out) {
    return guarded(nullptr, [&]() -> dfamg_status {
        if (!a || !out || n < 1 || n > 4096 || (method != 0 && method != 1))
            throw Error{DFAMG_EINVAL, "dfamg_dense_inverse: need a, out, 1 <= n <= 4096, method 0 or 1"};
        check_device();
        hipStream_t s = nullptr;
        const size_t nn = (size_t)n * n;
        if (method == 0) {
            DevArena tmp;
            double *d = tmp.alloc<double>(nn);
            HIP_CHECK(hipMemcpy(d, a, sizeof(double) * nn, hipMemcpyHostToDevice));
            bool ok = false;
            try {
                ok = invert_dense_inplace(s, d, n);
            } catch (const DenseInverseError &e) {
                throw Error{DFAMG_EHIP, e.msg};
            }
            if (!ok) throw Error{DFAMG_ESINGULAR, "matrix is singular"};
            HIP_CHECK(hipMemcpy(out, d, sizeof(double) * nn, hipMemcpyDeviceToHost));
            return DFAMG_OK;
        }
        DevArena tmp;
        double *d = tmp.alloc<double>(nn);
        const int bad = invert_on_device<double>(s, {a}, {n}, d, {0}, {n});
        if (bad >= 0) throw Error{DFAMG_ESINGULAR, "matrix is singular"};
        HIP_CHECK(hipMemcpy(out, d, sizeof(double) * nn, hipMemcpyDeviceToHost));
        return DFAMG_OK;
    });
}


dfamg_status dfamg_dense_inverse_noalloc(const double *a, int32_t n, double *out, void *stream) {
    return guarded(nullptr, [&]() -> dfamg_status {
        if (!a || !out || n < 1)
            throw Error{DFAMG_EINVAL, "dfamg_dense_inverse_noalloc: need device pointers a, out and n >= 1"};
        if (n > kNoAllocMaxN)
            throw Error{DFAMG_EINVAL, "dfamg_dense_inverse_noalloc: n = " + std::to_string(n) +
                                          " exceeds the workspace limit of " + std::to_string(kNoAllocMaxN)};
        check_device();
        hipStream_t s = static_cast<hipStream_t>(stream);
        double *ws = noalloc_workspace();
        InvJob *d_job = reinterpret_cast<InvJob *>(ws);
        const int64_t *d_coff = reinterpret_cast<const int64_t *>(ws + 8);
        const int64_t *d_oof = reinterpret_cast<const int64_t *>(ws + 12);
        const int32_t *d_old = reinterpret_cast<const int32_t *>(ws + 14);
        double *d_colk = ws + kNoAllocColk;
        double *d_aug = ws + kNoAllocAug;
        const int64_t maxel = (int64_t)n * 2 * n;
        const int gx = (int)std::min<int64_t>(1024, (maxel + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(k_noalloc_init, dim3(gx), dim3(kBlock), 0, s, ws, a, n);
        for (int k = 0; k < n; ++k) {
            hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(kBlock), 0, s, d_job, d_aug, d_colk, d_coff, k);
            hipLaunchKernelGGL(k_gj_eliminate, dim3(gx, 1), dim3(kBlock), 0, s, d_job, d_aug, d_colk, d_coff, k);
        }
        hipLaunchKernelGGL(k_gj_extract<double>, dim3(gx, 1), dim3(kBlock), 0, s, d_job, d_aug, d_oof, d_old, out);
        HIP_CHECK(hipGetLastError());
        InvJob job{};
        HIP_CHECK(hipMemcpyAsync(&job, d_job, sizeof(InvJob), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        if (job.singular) throw Error{DFAMG_ESINGULAR, "matrix is singular"};
        return DFAMG_OK;
    });
}

}  // extern "C"
