// Host-only driver of the setup planner (host_plan.cpp), built by
// tests/test_host_sanitize.py with AddressSanitizer and
// UndefinedBehaviorSanitizer and g++, without the HIP parts of the library.
//
// Usage: host_plan_driver <dir>
//   <dir>/params.bin   the raw bytes of a dfamg_params
//   <dir>/meta.txt     "n nsub ndv nsys"
//   <dir>/row_ptr.bin  int64[n+1]; col.bin int32[nnz]; val.bin float64[nnz]
//   <dir>/part.bin     int32[n];   Z.bin float64[n*ndv] (may be empty)
//   <dir>/sys_off.bin  int64[nsys+1] (only read when nsys > 1)
//
// Output (stdout): "ERR <status>" when build_plan rejects the input;
// otherwise, per user subdomain, "S <user> <nlevels>" followed by the rows,
// nnz(A), nnz(P) and omega of each level; per system "E <sys> <m> <sum of E>";
// per packed level the sparse layouts built from it (SELL with every row
// order and column width, CSR with lane counts 1 to 64 and tile heights 4 to
// 1024 rows, with the rows the tiles cover) as
// "L <level> <rows> <nnz A> <nnz B> <layout entries ...>", which exercises the
// layout builders on every operator of the hierarchy.
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <string>
#include <utility>
#include <vector>

#include "host_plan.hpp"

namespace dfamg {
// The GPU construction is not part of this build: a request for it is an
// error, as on a machine without a GPU.
void build_hierarchies_device(std::vector<Csr> &, const SaParams &, std::vector<Hierarchy> &, void *) {
    throw Error{DFAMG_ENOGPU, "host-only build"};
}
void build_az_device(const Csr &, const std::vector<int32_t> &, const std::vector<double> &, int,
                     std::vector<double> &, Csr &, void *) {
    throw Error{DFAMG_ENOGPU, "host-only build"};
}
}  // namespace dfamg

template <class T>
static std::vector<T> read_all(const std::string &path) {
    std::ifstream f(path, std::ios::binary | std::ios::ate);
    if (!f) return {};
    const std::streamsize bytes = f.tellg();
    f.seekg(0);
    std::vector<T> v((size_t)bytes / sizeof(T));
    if (!v.empty()) f.read(reinterpret_cast<char *>(v.data()), (std::streamsize)(v.size() * sizeof(T)));
    return v;
}

using namespace dfamg;

static std::vector<RowRange> ranges_of(const PackedLevel &L) {
    std::vector<RowRange> r;
    int32_t slot = 0;
    for (size_t s = 0; s < L.sub_len.size(); ++s) {
        if (L.sub_off[s] < 0 || L.sub_len[s] == 0) continue;
        r.push_back(RowRange{L.sub_off[s], L.sub_len[s], (int32_t)s, slot});
        slot += (L.sub_len[s] + 255) / 256;
    }
    return r;
}

// Ranges of a rectangular operator whose rows are the next level's
// unknowns (B, R): the next level's subdomain offsets.
static std::vector<RowRange> coarse_ranges(const Plan &P, size_t l) {
    return l + 1 < P.levels.size() ? ranges_of(P.levels[l + 1]) : std::vector<RowRange>{};
}

static void layouts(const Csr &M, const std::vector<RowRange> &rg, std::string &out) {
    if (M.nrows == 0 || rg.empty()) return;
    for (int rpl : {1, 2})
        for (bool sorted : {false, true})
            for (bool i16 : {false, true}) {
                HostSell S;
                const bool ok = make_sell(M, rg, rpl, sorted, i16, S);
                out += " sell" + std::to_string(rpl) + (sorted ? "s" : "") + (i16 ? "i" : "") + "=" +
                       (ok ? std::to_string(S.nnz) : std::string("no"));
            }
    // lane counts with their tile heights: one row per 64- or 32-lane group
    // (4 and 8 rows), the usual 64- and 256-row tiles, 1024 rows of 1 lane
    const std::pair<int, int> forms[] = {{4, 64}, {4, 256}, {16, 64}, {16, 256}, {64, 4}, {32, 8}, {1, 1024}};
    for (const auto &fr : forms) {
        HostCsrv C = make_csrv(M, rg, fr.first, fr.second);
        int64_t rows = 0;
        for (const Tile &t : C.tiles) rows += t.nrows;
        out += " csr" + std::to_string(fr.first) + "t" + std::to_string(fr.second) + "=" + std::to_string(C.nnz) + "/" +
               std::to_string(rows);
    }
}

int main(int argc, char **argv) {
    if (argc != 2) {
        std::fprintf(stderr, "usage: %s <dir>\n", argv[0]);
        return 2;
    }
    const std::string dir = argv[1];
    auto pbytes = read_all<char>(dir + "/params.bin");
    if (pbytes.size() != sizeof(dfamg_params)) {
        std::fprintf(stderr, "params.bin holds %zu bytes, dfamg_params %zu\n", pbytes.size(), sizeof(dfamg_params));
        return 2;
    }
    dfamg_params prm;
    std::copy(pbytes.begin(), pbytes.end(), reinterpret_cast<char *>(&prm));
    long long n = 0;
    int nsub = 0, ndv = 0, nsys = 1;
    {
        std::ifstream m(dir + "/meta.txt");
        if (!(m >> n >> nsub >> ndv >> nsys)) {
            std::fprintf(stderr, "bad meta.txt\n");
            return 2;
        }
    }
    auto ptr = read_all<int64_t>(dir + "/row_ptr.bin");
    auto col = read_all<int32_t>(dir + "/col.bin");
    auto val = read_all<double>(dir + "/val.bin");
    auto part = read_all<int32_t>(dir + "/part.bin");
    auto Z = read_all<double>(dir + "/Z.bin");
    auto soff = read_all<int64_t>(dir + "/sys_off.bin");
    if ((long long)ptr.size() != n + 1 || (long long)part.size() != n || col.size() != val.size() ||
        (int64_t)col.size() != ptr.back() || (long long)Z.size() != n * ndv) {
        std::fprintf(stderr, "inconsistent input arrays\n");
        return 2;
    }
    Plan P;
    try {
        build_plan(P, prm, nsys, nsys > 1 ? soff.data() : nullptr, n, ptr.data(), col.data(), val.data(),
                   part.data(), nsub, ndv, ndv ? Z.data() : nullptr);
    } catch (const Error &e) {
        std::printf("ERR %d %s\n", (int)e.status, e.msg.c_str());
        return 0;
    }
    for (int u = 0; u < nsub; ++u) {
        const Hierarchy &H = P.hier[P.user_to_sub[u]];
        std::printf("S %d %d", u, H.nlevels());
        for (int l = 0; l < H.nlevels(); ++l) {
            const Level &L = H.lv[l];
            const bool last = l + 1 == H.nlevels();
            std::printf(" %lld %lld %lld %.17g", (long long)L.A.nrows, (long long)L.A.nnz(),
                        (long long)(last ? 0 : L.P.nnz()), last ? 0.0 : L.omega);
        }
        std::printf("\n");
    }
    for (int s = 0; s < P.nsys; ++s) {
        const int32_t m = P.sys_m[s];
        double sum = 0.0;
        for (int64_t k = 0; k < (int64_t)m * m; ++k) sum += P.E[P.sys_E_off[s] + k];
        std::printf("E %d %d %.17g\n", s, m, sum);
    }
    for (size_t l = 0; l < P.levels.size(); ++l) {
        const PackedLevel &L = P.levels[l];
        std::string out;
        const auto rg = ranges_of(L);
        layouts(L.A, rg, out);
        if (L.B.nrows) layouts(L.B, coarse_ranges(P, l), out);
        if (L.P.nrows) layouts(L.P, rg, out);
        std::printf("L %zu %lld %lld %lld%s\n", l, (long long)L.nrows, (long long)L.A.nnz(), (long long)L.B.nnz(),
                    out.c_str());
    }
    return 0;
}
