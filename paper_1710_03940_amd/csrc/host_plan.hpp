// Host-side setup of the deflated block-AMG solver: validation, subdomain
// permutation, per-subdomain smoothed-aggregation hierarchies, AZ and E, and
// the packed per-level layout that the device code consumes.  Nothing here
// touches the GPU except the hierarchy construction with setup_device = 1
// (build_hierarchies_device).
#pragma once

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "dfamg.h"

namespace dfamg {

struct Error {
    dfamg_status status;
    std::string msg;
};

// Compressed sparse rows, 0-based, sorted column indices.
struct Csr {
    int64_t nrows = 0, ncols = 0;
    std::vector<int64_t> ptr{0};
    std::vector<int32_t> col;
    std::vector<double> val;
    int64_t nnz() const { return ptr.empty() ? 0 : ptr.back(); }
};

Csr transpose(const Csr &A);
// C = A * B with exact-zero results dropped; rows of C sorted.
Csr multiply(const Csr &A, const Csr &B);

// One level of a subdomain hierarchy (local numbering).
struct Level {
    Csr A;                   // level operator
    Csr P, R;                // prolongation (n_l x n_{l+1}) and R = P^T
    Csr B;                   // R (I - A diag(m)): the restricted residual of the
                             // pre-smoothed iterate (zero initial guess) as one map
    std::vector<double> m;   // smoother diagonal
    std::vector<double> mb;  // block SPAI-0: row i holds row i % bs of its node's block
    double eps = 0.0, omega = 0.0;
    std::vector<int32_t> agg;  // node -> aggregate (-1: none)
    int32_t nagg = 0;
};

struct Hierarchy {
    std::vector<Level> lv;   // lv.back() is the coarsest level
    int nlevels() const { return (int)lv.size(); }
};

struct SaParams {
    double eps_strong = 0.08;
    int coarse_enough = 500;
    int max_levels = 20;
    int smoother = DFAMG_SMOOTHER_SPAI0;
    double jacobi_omega = 0.8;
    int bs = 1;
};

Hierarchy build_hierarchy(Csr A, const SaParams &prm);

// Throws Error{EINVAL} for parameters the library does not accept.
void validate_params(const dfamg_params &p);

// The hierarchies of all subdomains (local diagonal blocks `local`, moved
// from) built on the current HIP device (setup_device.hip), equal to
// build_hierarchy's; scalar matrices and diagonal smoothers only.  `stream`
// is a hipStream_t.
void build_hierarchies_device(std::vector<Csr> &local, const SaParams &sp, std::vector<Hierarchy> &out,
                              void *stream);
// AZ of the permuted operator on the current device (own-subdomain block
// n x ndv and the couplings to other subdomains), equal to the host's.
void build_az_device(const Csr &A, const std::vector<int32_t> &row_sub, const std::vector<double> &Z, int ndv,
                     std::vector<double> &AZown, Csr &AZoff, void *stream);

// A row-tile of a packed level: up to `rows per tile` consecutive rows of one
// subdomain.
struct Tile {
    int32_t row0;    // first packed row
    int32_t nrows;
    int32_t sub;     // internal subdomain index
    int32_t slot;    // index of the tile's partial-sum slot
};

// Sliced ELLPACK with 64-row slices (one wavefront per slice, one row per
// lane), entries stored slice-major so that a wavefront reads consecutive
// addresses: entry j of lane l of slice s sits at off[s] + j*64 + l.  A tile
// of 256*rpl rows holds 4*rpl slices; wavefront w of the block walks slices
// w*rpl .. w*rpl+rpl-1.
struct HostSell {
    int rpl = 1;                     // rows per lane
    bool sorted = false;             // rows of each tile ordered by length (SELL-sigma)
    bool idx16 = false;              // columns stored as 16-bit offsets from a tile base
    std::vector<int16_t> ridx;       // sorted: tile-local row of each slot
    std::vector<uint16_t> col16;     // idx16: col - cbase[tile]
    std::vector<int32_t> cbase;      // idx16: smallest column of each tile
    std::vector<int32_t> cspan;      // idx16: largest - smallest column + 1
    std::vector<Tile> tiles;         // tile t covers slices 4*rpl*t ..
    std::vector<int64_t> slice_off;  // 4*rpl per tile
    std::vector<int32_t> slice_w;
    std::vector<int32_t> col;
    std::vector<double> val;
    int64_t nnz = 0;                 // structural nonzeros (without padding)
    int64_t nrows_covered = 0;
};

// CSR rows handled by `lanes` lanes each; a 256-thread block covers a tile of
// 256 rows, its 256/lanes lane groups striding over them.
struct HostCsrv {
    std::vector<Tile> tiles;
    std::vector<int32_t> cbase, cspan;   // column window of every tile
    std::vector<int32_t> ptr;        // packed CSR over all rows of the level
    std::vector<int32_t> col;
    std::vector<double> val;
    int lanes = 8;
    int64_t nnz = 0;
};

struct HostMat {
    int format = DFAMG_FORMAT_SELL;  // DFAMG_FORMAT_SELL or _CSR
    int lanes = 1;
    HostSell sell;
    HostCsrv csr;
    int64_t nrows = 0, ncols = 0;    // packed row / column spaces
};

// All subdomains at one level, packed in internal subdomain order.
struct PackedLevel {
    int64_t nrows = 0;                   // unknowns of all subdomains present
    std::vector<int64_t> sub_off;        // nsub+1 style: offset or -1 when absent
    std::vector<int32_t> sub_len;
    Csr A, P, R, B;                      // packed (block-diagonal) matrices
    Csr Bc;                              // B with each subdomain's rows in the next
                                         // level's clustered order
    std::vector<int32_t> B_rowmap;       // packed row of Bc -> natural packed row
    std::vector<double> m;               // smoother diagonal (0 when inactive)
    std::vector<double> mb;              // block smoother rows (bs per row), block SPAI-0 only
    std::vector<int32_t> active_subs;    // subdomains smoothing on this level
    std::vector<int32_t> coarse_subs;    // subdomains whose coarsest level is this
};

struct Plan {
    dfamg_params prm{};
    int64_t n = 0, nnz = 0;
    int32_t nsys = 1, nsub = 0, ndv = 0, bs = 1;
    // internal ordering
    std::vector<int64_t> perm;          // internal row -> original row
    std::vector<int64_t> sub_row_off;   // nsub+1
    std::vector<int32_t> sub_sys;       // internal subdomain -> system
    std::vector<int32_t> sub_user;      // internal subdomain -> user id
    std::vector<int32_t> user_to_sub;   // user id -> internal subdomain
    std::vector<int64_t> sys_row_off;   // nsys+1 (internal rows)
    std::vector<int32_t> sys_sub_off;   // nsys+1 (internal subdomains)
    Csr A;                              // permuted matrix
    std::vector<double> Z;              // permuted n x ndv
    std::vector<double> AZown;          // n x ndv, own-subdomain columns
    Csr AZoff;                          // n rows; columns = global coarse index
    std::vector<int32_t> sys_m;         // coarse size per system
    std::vector<int64_t> sys_E_off;     // offset of each system's E block
    std::vector<double> E;              // concatenated dense row-major blocks
    std::vector<Hierarchy> hier;        // per internal subdomain
    std::vector<PackedLevel> levels;
    int nlevels_max = 0;
    double host_seconds = 0.0;
    double hier_seconds = 0.0;          // hierarchy construction (part of host_seconds)
    int hier_on_device = 0;             // 1: built on the GPU
};

// Validates, permutes and builds everything; throws Error.
void build_plan(Plan &plan, const dfamg_params &prm, int32_t nsys,
                const int64_t *sys_row_off, int64_t n, const int64_t *row_ptr,
                const int32_t *col, const double *val, const int32_t *part,
                int32_t nsub, int32_t ndv, const double *Z, void *stream = nullptr);

// Device-ready layouts.  `ranges` lists, per subdomain covered by the
// matrix, its first packed row and row count; tiles never straddle two
// subdomains.  `slots` (optional) gives the partial-sum slot of the first tile
// of each range; consecutive tiles of a range take consecutive slots.
struct RowRange {
    int64_t row0;
    int32_t nrows;
    int32_t sub;
    int32_t slot0;
};
// `sorted` orders the rows of every tile by decreasing length (SELL-sigma
// with sigma = tile); `idx16` stores columns as unsigned 16-bit offsets from
// the smallest column of the tile and fails (returns false) when a tile's
// columns span more than 65536 values.
bool make_sell(const Csr &M, const std::vector<RowRange> &ranges, int rpl, bool sorted, bool idx16,
               HostSell &S);
// tile_rows: rows per 256-thread block (the block's 256/lanes groups stride
// over them)
HostCsrv make_csrv(const Csr &M, const std::vector<RowRange> &ranges, int lanes, int tile_rows = 256);
// rows per block-sized tile of each layout
inline int sell_tile_rows(int rpl) { return 256 * rpl; }
inline int csr_tile_rows(int lanes) { return lanes > 0 ? 256 : 256; }

// Runs fn(i) for i in [0, count) on `threads` host threads.
void parallel_for(int64_t count, int threads, const std::function<void(int64_t)> &fn);

}  // namespace dfamg
