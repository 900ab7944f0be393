// Host-side setup: validation, subdomain permutation, smoothed-aggregation
// hierarchies, AZ / E assembly and the packed level layout.  See host_plan.hpp.
//
// The subdomain deflation method of Demidov & Rossi (arXiv:1710.03940):
//   * one AMG per subdomain, built on the square diagonal block of A with the
//     non-local columns dropped (section "Implementation");
//   * Z holds one local block per subdomain (sections "Constant deflation",
//     "Linear deflation"); AZ and E = Z^T A Z are formed explicitly
//     (section "Implementation", after the projector equation).
// The smoothed-aggregation internals are not spelled out in the paper; this
// file implements the following choices (Vanek, Mandel & Brezina 1996 style):
//   strength   |A_IJ|_F^2 >= eps^2 |A_II|_F |A_JJ|_F on the node graph,
//              eps = eps_strong on level 0, halved per level;
//   aggregates three greedy passes in ascending node order (new aggregate
//              from a node whose strong neighbourhood is free; attach the
//              rest to the aggregate of the heaviest strong neighbour found
//              aggregated after pass 1, first one on ties; new aggregates
//              from what is left); nodes without strong neighbours stay out;
//   P          (I - omega D_F^{-1} A_F) P_tent with unnormalised P_tent,
//              A_F = A with weak off-diagonal blocks added to the diagonal
//              block, omega = (4/3) / max_I sum_J ||D_I^{-1} A_F,IJ||_inf;
//   coarse     Galerkin R A P with R = P^T, until <= coarse_enough unknowns;
//   smoother   SPAI-0 m_i = a_ii / sum_j a_ij^2 (Broeker & Grote 2002) or
//              damped Jacobi m_i = omega_J / a_ii.
#include "host_plan.hpp"

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <numeric>
#include <thread>

namespace dfamg {

namespace {

[[noreturn]] void fail(dfamg_status st, const std::string &msg) { throw Error{st, msg}; }

}  // namespace

void parallel_for(int64_t count, int threads, const std::function<void(int64_t)> &fn) {
    if (count <= 0) return;
    if (threads <= 0) threads = (int)std::max(1u, std::thread::hardware_concurrency());
    threads = (int)std::min<int64_t>(threads, count);
    if (threads <= 1) {
        for (int64_t i = 0; i < count; ++i) fn(i);
        return;
    }
    std::atomic<int64_t> next{0};
    std::vector<Error> errs;
    std::vector<char> failed(threads, 0);
    errs.resize(threads);
    std::vector<std::thread> pool;
    for (int t = 0; t < threads; ++t) {
        pool.emplace_back([&, t] {
            try {
                for (int64_t i = next++; i < count; i = next++) fn(i);
            } catch (const Error &e) {
                errs[t] = e;
                failed[t] = 1;
                next = count;
            } catch (const std::bad_alloc &) {
                errs[t] = Error{DFAMG_ENOMEM, "host allocation failed"};
                failed[t] = 1;
                next = count;
            }
        });
    }
    for (auto &th : pool) th.join();
    for (int t = 0; t < threads; ++t)
        if (failed[t]) throw errs[t];
}

// ---------------------------------------------------------------------------
// sparse kernels
// ---------------------------------------------------------------------------

Csr transpose(const Csr &A) {
    Csr T;
    T.nrows = A.ncols;
    T.ncols = A.nrows;
    T.ptr.assign(T.nrows + 1, 0);
    for (int64_t k = 0; k < A.nnz(); ++k) T.ptr[A.col[k] + 1]++;
    for (int64_t i = 0; i < T.nrows; ++i) T.ptr[i + 1] += T.ptr[i];
    T.col.resize(A.nnz());
    T.val.resize(A.nnz());
    std::vector<int64_t> pos(T.ptr.begin(), T.ptr.end() - 1);
    for (int64_t i = 0; i < A.nrows; ++i)
        for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
            int64_t d = pos[A.col[k]]++;
            T.col[d] = (int32_t)i;
            T.val[d] = A.val[k];
        }
    return T;
}

Csr multiply(const Csr &A, const Csr &B) {
    Csr C;
    C.nrows = A.nrows;
    C.ncols = B.ncols;
    C.ptr.assign(C.nrows + 1, 0);
    std::vector<int64_t> mark(B.ncols, -1);
    std::vector<double> acc(B.ncols, 0.0);
    std::vector<int32_t> cols;
    for (int64_t i = 0; i < A.nrows; ++i) {
        cols.clear();
        for (int64_t ka = A.ptr[i]; ka < A.ptr[i + 1]; ++ka) {
            const int32_t j = A.col[ka];
            const double a = A.val[ka];
            for (int64_t kb = B.ptr[j]; kb < B.ptr[j + 1]; ++kb) {
                const int32_t c = B.col[kb];
                if (mark[c] != i) {
                    mark[c] = i;
                    acc[c] = a * B.val[kb];
                    cols.push_back(c);
                } else {
                    acc[c] += a * B.val[kb];
                }
            }
        }
        std::sort(cols.begin(), cols.end());
        for (int32_t c : cols)
            if (acc[c] != 0.0) {
                C.col.push_back(c);
                C.val.push_back(acc[c]);
            }
        C.ptr[i + 1] = (int64_t)C.col.size();
    }
    return C;
}

// ---------------------------------------------------------------------------
// smoothed aggregation for one subdomain block
// ---------------------------------------------------------------------------

namespace {

// Node graph with the squared Frobenius norm of every stored block.
Csr node_norms(const Csr &A, int bs) {
    if (bs == 1) {
        Csr F = A;
        for (auto &v : F.val) v = v * v;
        return F;
    }
    const int64_t nn = A.nrows / bs;
    Csr F;
    F.nrows = F.ncols = nn;
    F.ptr.assign(nn + 1, 0);
    std::vector<int64_t> mark(nn, -1);
    std::vector<double> acc(nn, 0.0);
    std::vector<int32_t> cols;
    for (int64_t I = 0; I < nn; ++I) {
        cols.clear();
        for (int c = 0; c < bs; ++c) {
            const int64_t i = I * bs + c;
            for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
                const int32_t J = A.col[k] / bs;
                const double sq = A.val[k] * A.val[k];
                if (mark[J] != I) {
                    mark[J] = I;
                    acc[J] = sq;
                    cols.push_back(J);
                } else {
                    acc[J] += sq;
                }
            }
        }
        std::sort(cols.begin(), cols.end());
        for (int32_t J : cols) {
            F.col.push_back(J);
            F.val.push_back(acc[J]);
        }
        F.ptr[I + 1] = (int64_t)F.col.size();
    }
    return F;
}

std::vector<char> strength(const Csr &F, double eps) {
    const int64_t nn = F.nrows;
    std::vector<double> dn(nn, 0.0);
    for (int64_t I = 0; I < nn; ++I)
        for (int64_t k = F.ptr[I]; k < F.ptr[I + 1]; ++k)
            if (F.col[k] == I) dn[I] = std::sqrt(F.val[k]);
    std::vector<char> s(F.nnz(), 0);
    const double e2 = eps * eps;
    for (int64_t I = 0; I < nn; ++I)
        for (int64_t k = F.ptr[I]; k < F.ptr[I + 1]; ++k) {
            const int32_t J = F.col[k];
            s[k] = (J != I) && (F.val[k] >= e2 * dn[I] * dn[J]);
        }
    return s;
}

int32_t aggregate(const Csr &F, const std::vector<char> &strong, std::vector<int32_t> &agg) {
    const int64_t nn = F.nrows;
    agg.assign(nn, -1);
    int32_t count = 0;
    auto has_strong = [&](int64_t I) {
        for (int64_t k = F.ptr[I]; k < F.ptr[I + 1]; ++k)
            if (strong[k]) return true;
        return false;
    };
    // first pass: seeds whose whole strong neighbourhood is still free
    for (int64_t I = 0; I < nn; ++I) {
        if (agg[I] >= 0 || !has_strong(I)) continue;
        bool free_nbhd = true;
        for (int64_t k = F.ptr[I]; k < F.ptr[I + 1] && free_nbhd; ++k)
            if (strong[k] && agg[F.col[k]] >= 0) free_nbhd = false;
        if (!free_nbhd) continue;
        agg[I] = count;
        for (int64_t k = F.ptr[I]; k < F.ptr[I + 1]; ++k)
            if (strong[k]) agg[F.col[k]] = count;
        ++count;
    }
    // second pass: attach to the heaviest neighbour aggregated by pass one
    const std::vector<int32_t> first(agg);
    for (int64_t I = 0; I < nn; ++I) {
        if (first[I] >= 0) continue;
        int32_t target = -1;
        double wbest = 0.0;
        for (int64_t k = F.ptr[I]; k < F.ptr[I + 1]; ++k) {
            if (!strong[k]) continue;
            const int32_t J = F.col[k];
            const double w = std::sqrt(F.val[k]);
            if (first[J] >= 0 && (target < 0 || w > wbest)) {
                target = first[J];
                wbest = w;
            }
        }
        if (target >= 0) agg[I] = target;
    }
    // third pass: whatever still has strong neighbours seeds a new aggregate
    for (int64_t I = 0; I < nn; ++I) {
        if (agg[I] >= 0 || !has_strong(I)) continue;
        agg[I] = count;
        for (int64_t k = F.ptr[I]; k < F.ptr[I + 1]; ++k)
            if (strong[k] && agg[F.col[k]] < 0) agg[F.col[k]] = count;
        ++count;
    }
    return count;
}

// Filtered matrix: weak off-diagonal blocks are added into the diagonal block.
Csr filtered(const Csr &A, const Csr &F, const std::vector<char> &strong, int bs) {
    const int64_t n = A.nrows, nn = F.nrows;
    std::vector<int64_t> mark(nn, -1);    // node column -> strong flag row stamp
    std::vector<char> is_strong(nn, 0);
    Csr R;
    R.nrows = R.ncols = n;
    R.ptr.assign(n + 1, 0);
    std::vector<std::pair<int32_t, double>> row;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t I = i / bs;
        for (int64_t k = F.ptr[I]; k < F.ptr[I + 1]; ++k) {
            mark[F.col[k]] = i;
            is_strong[F.col[k]] = strong[k];
        }
        row.clear();
        for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
            const int32_t j = A.col[k];
            const int64_t J = j / bs;
            const bool weak = (J != I) && !(mark[J] == i && is_strong[J]);
            row.emplace_back(weak ? (int32_t)(I * bs + j % bs) : j, A.val[k]);
        }
        std::stable_sort(row.begin(), row.end(),
                         [](const auto &a, const auto &b) { return a.first < b.first; });
        for (size_t q = 0; q < row.size();) {
            size_t e = q + 1;
            double s = row[q].second;
            while (e < row.size() && row[e].first == row[q].first) s += row[e++].second;
            R.col.push_back(row[q].first);
            R.val.push_back(s);
            q = e;
        }
        R.ptr[i + 1] = (int64_t)R.col.size();
    }
    return R;
}

// Inverse of a small dense block (row-major, b x b) by Gauss-Jordan with
// partial pivoting; false when a pivot is exactly zero.
bool invert_small(const double *in, double *out, int b) {
    double a[8][16];
    for (int r = 0; r < b; ++r)
        for (int c = 0; c < 2 * b; ++c) a[r][c] = c < b ? in[r * b + c] : (c - b == r ? 1.0 : 0.0);
    for (int k = 0; k < b; ++k) {
        int p = k;
        for (int r = k + 1; r < b; ++r)
            if (std::fabs(a[r][k]) > std::fabs(a[p][k])) p = r;
        if (a[p][k] == 0.0) return false;
        if (p != k)
            for (int c = 0; c < 2 * b; ++c) std::swap(a[p][c], a[k][c]);
        const double inv = 1.0 / a[k][k];
        for (int c = 0; c < 2 * b; ++c) a[k][c] *= inv;
        for (int r = 0; r < b; ++r) {
            if (r == k || a[r][k] == 0.0) continue;
            const double f = a[r][k];
            for (int c = 0; c < 2 * b; ++c) a[r][c] -= f * a[k][c];
        }
    }
    for (int r = 0; r < b; ++r)
        for (int c = 0; c < b; ++c) out[r * b + c] = a[r][b + c];
    return true;
}

void smoothed_prolongation(const Csr &AF, const std::vector<int32_t> &agg, int32_t nagg, int bs,
                           Level &lvl) {
    const int64_t n = AF.nrows, nn = n / bs, nc = (int64_t)nagg * bs;
    // block diagonal of A_F and its inverse
    std::vector<double> D(nn * bs * bs, 0.0), Dinv(nn * bs * bs, 0.0);
    std::vector<char> ok(nn, 0);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t I = i / bs;
        for (int64_t k = AF.ptr[i]; k < AF.ptr[i + 1]; ++k)
            if (AF.col[k] / bs == I) D[I * bs * bs + (i % bs) * bs + AF.col[k] % bs] = AF.val[k];
    }
    for (int64_t I = 0; I < nn; ++I) {
        if (bs == 1) {
            if (D[I] != 0.0) {
                Dinv[I] = 1.0 / D[I];
                ok[I] = 1;
            }
        } else {
            ok[I] = invert_small(&D[I * bs * bs], &Dinv[I * bs * bs], bs);
            if (!ok[I]) std::fill(&Dinv[I * bs * bs], &Dinv[(I + 1) * bs * bs], 0.0);
        }
    }
    // Gershgorin-type bound of D^{-1} A_F: per node I, the sum over node
    // columns J of the inf-norm of block (D^{-1} A_F)_IJ
    double rho = 0.0;
    bool any = false;
    {
        std::vector<int32_t> slot(nn, -1);           // node column -> local index
        std::vector<int32_t> cols;
        std::vector<double> rs;                      // [local J][c] abs row sums
        std::vector<std::pair<int32_t, double>> brow;
        for (int64_t I = 0; I < nn; ++I) {
            if (!ok[I]) continue;
            cols.clear();
            rs.clear();
            for (int c = 0; c < bs; ++c) {
                // scalar row I*bs+c of B = D^{-1} A_F
                brow.clear();
                for (int cp = 0; cp < bs; ++cp) {
                    const double d = Dinv[I * bs * bs + c * bs + cp];
                    if (d == 0.0) continue;
                    const int64_t r = I * bs + cp;
                    for (int64_t k = AF.ptr[r]; k < AF.ptr[r + 1]; ++k)
                        brow.emplace_back(AF.col[k], d * AF.val[k]);
                }
                std::stable_sort(brow.begin(), brow.end(),
                                 [](const auto &a, const auto &b) { return a.first < b.first; });
                for (size_t q = 0; q < brow.size();) {
                    size_t e = q + 1;
                    double v = brow[q].second;
                    while (e < brow.size() && brow[e].first == brow[q].first) v += brow[e++].second;
                    const int32_t J = brow[q].first / bs;
                    if (slot[J] < 0) {
                        slot[J] = (int32_t)cols.size();
                        cols.push_back(J);
                        rs.resize(rs.size() + bs, 0.0);
                    }
                    rs[(size_t)slot[J] * bs + c] += std::fabs(v);
                    q = e;
                }
            }
            std::vector<int32_t> order(cols);
            std::sort(order.begin(), order.end());
            double r = 0.0;
            for (int32_t J : order) {
                double inf = 0.0;
                for (int c = 0; c < bs; ++c) inf = std::max(inf, rs[(size_t)slot[J] * bs + c]);
                r += inf;
            }
            for (int32_t J : cols) slot[J] = -1;
            if (!any || r > rho) rho = r;
            any = true;
        }
    }
    if (!any) rho = 1.0;
    const double omega = (4.0 / 3.0) / rho;
    lvl.omega = omega;

    // P = P_tent - omega * D^{-1} (A_F P_tent)
    Csr &P = lvl.P;
    P.nrows = n;
    P.ncols = nc;
    P.ptr.assign(n + 1, 0);
    std::vector<int64_t> mark(nc, -1);
    std::vector<double> acc(nc * (size_t)bs, 0.0);  // X rows of the node
    std::vector<int32_t> cols;
    for (int64_t I = 0; I < nn; ++I) {
        cols.clear();
        // X[c'][col] = (A_F P_tent)[I*bs + c', col]
        for (int cp = 0; cp < bs; ++cp) {
            const int64_t r = I * bs + cp;
            for (int64_t k = AF.ptr[r]; k < AF.ptr[r + 1]; ++k) {
                const int32_t j = AF.col[k];
                const int32_t g = agg[j / bs];
                if (g < 0) continue;
                const int32_t c = g * bs + j % bs;
                if (mark[c] != I) {
                    mark[c] = I;
                    for (int q = 0; q < bs; ++q) acc[(size_t)c * bs + q] = 0.0;
                    cols.push_back(c);
                }
                acc[(size_t)c * bs + cp] += AF.val[k];
            }
        }
        std::sort(cols.begin(), cols.end());
        for (int c = 0; c < bs; ++c) {
            const int64_t i = I * bs + c;
            const int32_t own = agg[I] >= 0 ? agg[I] * bs + c : -1;
            // row i of D^{-1} X, then P_tent - omega * (that)
            std::vector<std::pair<int32_t, double>> row;
            bool own_seen = false;
            for (int32_t col : cols) {
                double y = 0.0;
                bool have = false;
                for (int cp = 0; cp < bs; ++cp) {
                    const double d = Dinv[I * bs * bs + c * bs + cp];
                    const double x = acc[(size_t)col * bs + cp];
                    if (d == 0.0 || x == 0.0) continue;
                    y = have ? y + d * x : d * x;
                    have = true;
                }
                if (col == own) own_seen = true;
                if (have && y != 0.0) row.emplace_back(col, (col == own ? 1.0 : 0.0) - omega * y);
                else if (col == own) row.emplace_back(col, 1.0);
            }
            if (own >= 0 && !own_seen) row.emplace_back(own, 1.0);
            std::sort(row.begin(), row.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
            for (auto &e : row)
                if (e.second != 0.0) {
                    P.col.push_back(e.first);
                    P.val.push_back(e.second);
                }
            P.ptr[i + 1] = (int64_t)P.col.size();
        }
    }
}

}  // namespace

// B = R - (R A) diag(m), rows merged column by column; exact zeros dropped.
// With one pre-smoothing sweep from a zero guess, x = m o f and the level's
// restricted residual is R (f - A x) = B f.
// Block SPAI-0 of a point-block matrix: per node i the bs x bs block
// M_i = A_ii^T G_i^{-1}, G_i = A_(i,:) A_(i,:)^T (the Gram matrix of the node's
// rows), the minimiser of ||I - M A||_F over block-diagonal M.  Row r of the
// result holds row r % bs of its node's block.
void block_spai0(const Csr &A, int bs, std::vector<double> &mb) {
    const int64_t n = A.nrows, nb = n / bs;
    mb.assign((size_t)n * bs, 0.0);
    std::vector<double> G((size_t)bs * bs), Aii((size_t)bs * bs), dense;
    std::vector<int64_t> where(A.ncols, -1);
    for (int64_t b = 0; b < nb; ++b) {
        const int64_t r0 = b * bs;
        // the node's rows as a dense block over the union of their columns
        std::vector<int32_t> cols;
        for (int r = 0; r < bs; ++r)
            for (int64_t k = A.ptr[r0 + r]; k < A.ptr[r0 + r + 1]; ++k)
                if (where[A.col[k]] < 0) {
                    where[A.col[k]] = (int64_t)cols.size();
                    cols.push_back(A.col[k]);
                }
        const size_t nc = cols.size();
        dense.assign((size_t)bs * nc, 0.0);
        for (int r = 0; r < bs; ++r)
            for (int64_t k = A.ptr[r0 + r]; k < A.ptr[r0 + r + 1]; ++k) dense[r * nc + where[A.col[k]]] = A.val[k];
        for (int r = 0; r < bs; ++r)
            for (int c = 0; c < bs; ++c) {
                double g = 0.0;
                for (size_t j = 0; j < nc; ++j) g += dense[r * nc + j] * dense[c * nc + j];
                G[r * bs + c] = g;
                const int64_t w = where[r0 + c];
                Aii[r * bs + c] = w >= 0 ? dense[r * nc + w] : 0.0;
            }
        for (int32_t c : cols) where[c] = -1;
        // M_i = A_ii^T G^{-1}: solve G^T M_i^T = A_ii (G is symmetric), by
        // Gauss-Jordan with partial pivoting on [G | A_ii]
        std::vector<double> aug((size_t)bs * 2 * bs);
        for (int r = 0; r < bs; ++r)
            for (int c = 0; c < bs; ++c) {
                aug[r * 2 * bs + c] = G[c * bs + r];
                aug[r * 2 * bs + bs + c] = Aii[r * bs + c];
            }
        for (int k = 0; k < bs; ++k) {
            int p = k;
            for (int r = k + 1; r < bs; ++r)
                if (std::fabs(aug[r * 2 * bs + k]) > std::fabs(aug[p * 2 * bs + k])) p = r;
            if (aug[p * 2 * bs + k] == 0.0)
                fail(DFAMG_ESINGULAR, "block SPAI-0: rows of node " + std::to_string(b) + " are linearly dependent");
            if (p != k)
                for (int c = 0; c < 2 * bs; ++c) std::swap(aug[k * 2 * bs + c], aug[p * 2 * bs + c]);
            const double d = aug[k * 2 * bs + k];
            for (int c = 0; c < 2 * bs; ++c) aug[k * 2 * bs + c] /= d;
            for (int r = 0; r < bs; ++r) {
                if (r == k) continue;
                const double f = aug[r * 2 * bs + k];
                if (f != 0.0)
                    for (int c = 0; c < 2 * bs; ++c) aug[r * 2 * bs + c] -= f * aug[k * 2 * bs + c];
            }
        }
        // aug's right half is X = G^{-T} A_ii = M_i^T: M_i[r][c] = X[c][r]
        for (int r = 0; r < bs; ++r)
            for (int c = 0; c < bs; ++c) mb[(size_t)(r0 + r) * bs + c] = aug[c * 2 * bs + bs + r];
    }
}

Csr restricted_residual_map(const Csr &R, const Csr &RA, const std::vector<double> &m) {
    Csr B;
    B.nrows = R.nrows;
    B.ncols = R.ncols;
    B.ptr.assign(R.nrows + 1, 0);
    for (int64_t k = 0; k < R.nrows; ++k) {
        int64_t a = R.ptr[k], b = RA.ptr[k];
        const int64_t ae = R.ptr[k + 1], be = RA.ptr[k + 1];
        while (a < ae || b < be) {
            int32_t c;
            double v;
            if (b >= be || (a < ae && R.col[a] < RA.col[b])) {
                c = R.col[a];
                v = R.val[a++];
            } else if (a >= ae || RA.col[b] < R.col[a]) {
                c = RA.col[b];
                v = -RA.val[b++] * m[c];
            } else {
                c = R.col[a];
                v = R.val[a++] - RA.val[b++] * m[c];
            }
            if (v != 0.0) {
                B.col.push_back(c);
                B.val.push_back(v);
            }
        }
        B.ptr[k + 1] = (int64_t)B.col.size();
    }
    return B;
}

Hierarchy build_hierarchy(Csr A, const SaParams &prm) {
    Hierarchy H;
    double eps = prm.eps_strong;
    const int bs = prm.bs;
    for (;;) {
        H.lv.emplace_back();
        Level &L = H.lv.back();
        L.A = std::move(A);
        L.eps = eps;
        const int64_t n = L.A.nrows;
        if (n <= prm.coarse_enough || (int)H.lv.size() >= prm.max_levels) break;
        const Csr F = node_norms(L.A, bs);
        const std::vector<char> strong = strength(F, eps);
        const int32_t nagg = aggregate(F, strong, L.agg);
        if (nagg == 0 || (int64_t)nagg * bs >= n) {
            L.agg.clear();
            break;
        }
        L.nagg = nagg;
        const Csr AF = filtered(L.A, F, strong, bs);
        smoothed_prolongation(AF, L.agg, nagg, bs, L);
        L.R = transpose(L.P);
        // smoother diagonal of this level
        L.m.assign(n, 0.0);
        for (int64_t i = 0; i < n; ++i) {
            double d = 0.0, s = 0.0;
            for (int64_t k = L.A.ptr[i]; k < L.A.ptr[i + 1]; ++k) {
                if (L.A.col[k] == i) d = L.A.val[k];
                s += L.A.val[k] * L.A.val[k];
            }
            L.m[i] = prm.smoother == DFAMG_SMOOTHER_JACOBI ? prm.jacobi_omega / d : d / s;
        }
        if (prm.smoother == DFAMG_SMOOTHER_BLOCK_SPAI0) block_spai0(L.A, bs, L.mb);
        const Csr RA = multiply(L.R, L.A);
        // the fused restriction operator assumes a diagonal smoother
        if (prm.smoother != DFAMG_SMOOTHER_BLOCK_SPAI0) L.B = restricted_residual_map(L.R, RA, L.m);
        A = multiply(RA, L.P);
        eps *= 0.5;
    }
    return H;
}

// ---------------------------------------------------------------------------
// device layouts
// ---------------------------------------------------------------------------

bool make_sell(const Csr &M, const std::vector<RowRange> &ranges, int rpl, bool sorted, bool idx16,
               HostSell &S) {
    S = HostSell{};
    S.rpl = rpl;
    S.sorted = sorted;
    S.idx16 = idx16;
    const int tile_rows = sell_tile_rows(rpl), nsl = 4 * rpl;
    for (const RowRange &rg : ranges) {
        int32_t slot = rg.slot0;
        for (int32_t r0 = 0; r0 < rg.nrows; r0 += tile_rows) {
            Tile t{(int32_t)(rg.row0 + r0), std::min(tile_rows, rg.nrows - r0), rg.sub, slot++};
            S.tiles.push_back(t);
        }
    }
    auto len = [&](int64_t r) { return (int)(M.ptr[r + 1] - M.ptr[r]); };
    // tile-local order of the rows (identity unless sorted)
    std::vector<int16_t> order((size_t)S.tiles.size() * tile_rows, 0);
    const int64_t ntiles = (int64_t)S.tiles.size();
    // every tile's rows, slices and entries are independent of the others'
    parallel_for(ntiles, 8, [&](int64_t ti) {
        const Tile &t = S.tiles[ti];
        int16_t *o = &order[ti * tile_rows];
        for (int k = 0; k < t.nrows; ++k) o[k] = (int16_t)k;
        if (sorted)
            std::stable_sort(o, o + t.nrows, [&](int16_t a, int16_t b) { return len(t.row0 + a) > len(t.row0 + b); });
    });
    if (sorted) S.ridx = order;
    int64_t off = 0;
    S.slice_off.reserve(S.tiles.size() * nsl);
    for (size_t ti = 0; ti < S.tiles.size(); ++ti) {
        const Tile &t = S.tiles[ti];
        for (int k = 0; k < nsl; ++k) {
            int w = 0;
            for (int l = 0; l < 64; ++l) {
                const int32_t lr = k * 64 + l;
                if (lr >= t.nrows) break;
                w = std::max(w, len(t.row0 + order[ti * tile_rows + lr]));
            }
            S.slice_off.push_back(off);
            S.slice_w.push_back(w);
            off += (int64_t)w * 64;
        }
        S.nrows_covered += t.nrows;
    }
    if (idx16) {
        S.col16.assign(off, 0);
        S.cbase.assign(S.tiles.size(), 0);
        S.cspan.assign(S.tiles.size(), 1);
        std::atomic<bool> fits{true};
        parallel_for(ntiles, 8, [&](int64_t ti) {
            const Tile &t = S.tiles[ti];
            int64_t lo = INT64_MAX, hi = -1;
            for (int64_t r = t.row0; r < t.row0 + t.nrows; ++r)
                for (int64_t k = M.ptr[r]; k < M.ptr[r + 1]; ++k) {
                    lo = std::min<int64_t>(lo, M.col[k]);
                    hi = std::max<int64_t>(hi, M.col[k]);
                }
            if (hi < 0) lo = hi = std::min<int64_t>(t.row0, M.ncols - 1);
            // padding of empty rows uses the base itself
            if (hi - lo > 65535) fits = false;
            S.cbase[ti] = (int32_t)lo;
            S.cspan[ti] = (int32_t)(hi - lo + 1);
        });
        if (!fits) return false;
    } else {
        S.col.assign(off, 0);
    }
    S.val.assign(off, 0.0);
    std::vector<int64_t> tile_nnz(ntiles, 0);
    parallel_for(ntiles, 8, [&](int64_t ti) {
        const Tile &t = S.tiles[ti];
        for (int k = 0; k < nsl; ++k) {
            const int64_t base = S.slice_off[ti * nsl + k];
            const int w = S.slice_w[ti * nsl + k];
            for (int l = 0; l < 64; ++l) {
                const int32_t lr = k * 64 + l;
                if (lr >= t.nrows) break;
                const int64_t r = t.row0 + order[ti * tile_rows + lr];
                const int64_t n = len(r);
                const int32_t padc = n > 0 ? M.col[M.ptr[r + 1] - 1]
                                           : (idx16 ? S.cbase[ti] : (int32_t)std::min<int64_t>(r, M.ncols - 1));
                for (int j = 0; j < w; ++j) {
                    const int64_t d = base + (int64_t)j * 64 + l;
                    const int32_t c = j < n ? M.col[M.ptr[r] + j] : padc;
                    if (idx16) S.col16[d] = (uint16_t)(c - S.cbase[ti]);
                    else S.col[d] = c;
                    S.val[d] = j < n ? M.val[M.ptr[r] + j] : 0.0;
                }
                tile_nnz[ti] += n;
            }
        }
    });
    for (int64_t v : tile_nnz) S.nnz += v;
    return true;
}

HostCsrv make_csrv(const Csr &M, const std::vector<RowRange> &ranges, int lanes, int tile_rows) {
    HostCsrv C;
    C.lanes = lanes;
    const int rows_per_tile = tile_rows;
    for (const RowRange &rg : ranges) {
        int32_t slot = rg.slot0;
        for (int32_t r0 = 0; r0 < rg.nrows; r0 += rows_per_tile)
            C.tiles.push_back(Tile{(int32_t)(rg.row0 + r0), std::min(rows_per_tile, rg.nrows - r0),
                                   rg.sub, slot++});
    }
    C.cbase.assign(C.tiles.size(), 0);
    C.cspan.assign(C.tiles.size(), 1);
    for (size_t ti = 0; ti < C.tiles.size(); ++ti) {
        const Tile &t = C.tiles[ti];
        int64_t lo = INT64_MAX, hi = -1;
        for (int64_t r = t.row0; r < t.row0 + t.nrows; ++r)
            for (int64_t k = M.ptr[r]; k < M.ptr[r + 1]; ++k) {
                lo = std::min<int64_t>(lo, M.col[k]);
                hi = std::max<int64_t>(hi, M.col[k]);
            }
        if (hi >= 0) {
            C.cbase[ti] = (int32_t)lo;
            C.cspan[ti] = (int32_t)(hi - lo + 1);
        }
    }
    C.ptr.resize(M.nrows + 1);
    for (int64_t i = 0; i <= M.nrows; ++i) C.ptr[i] = (int32_t)M.ptr[i];
    C.col = M.col;
    C.val = M.val;
    C.nnz = M.nnz();
    return C;
}

// ---------------------------------------------------------------------------
// the plan
// ---------------------------------------------------------------------------

namespace {

// Clustered order of the levels of one subdomain's hierarchy:
// ord[l][k] = the k-th row of level l in that order, pos[l] its inverse.
// Level 0 and the coarsest level keep their numbering; on every level in
// between the nodes are grouped by their aggregate on the next level, the
// aggregates taken in that level's clustered order (recursively), the nodes
// of one aggregate in ascending index and nodes in no aggregate last; the
// rows of a point-block node stay together.  The restriction operators B_l
// store their rows (the nodes of level l+1) in this order: a tile of
// consecutive rows then covers a compact cluster of level l, so the entries
// of the finer vector that the tile gathers overlap far more than along the
// natural (aggregate formation) order, while every vector keeps its natural
// numbering (the kernel writes each row's result through a row map).
void level_orders(const Hierarchy &H, int bs, std::vector<std::vector<int64_t>> &ord,
                  std::vector<std::vector<int64_t>> &pos) {
    const int L = H.nlevels();
    std::vector<std::vector<int64_t>> node(L);   // node order per level
    for (int l = L - 1; l >= 0; --l) {
        const int64_t nn = H.lv[l].A.nrows / bs;
        std::vector<int64_t> &o = node[l];
        if (l == 0 || l == L - 1) {
            o.resize(nn);
            std::iota(o.begin(), o.end(), 0);
            continue;
        }
        const std::vector<int32_t> &agg = H.lv[l].agg;
        const int64_t nc = (int64_t)node[l + 1].size();
        std::vector<int64_t> start(nc + 1, 0);
        for (int64_t i = 0; i < nn; ++i)
            if (agg[i] >= 0) start[agg[i] + 1]++;
        for (int64_t c = 0; c < nc; ++c) start[c + 1] += start[c];
        std::vector<int64_t> kids(start[nc]), fill(start.begin(), start.end() - 1);
        for (int64_t i = 0; i < nn; ++i)
            if (agg[i] >= 0) kids[fill[agg[i]]++] = i;   // ascending within an aggregate
        o.reserve(nn);
        for (int64_t c : node[l + 1])
            for (int64_t k = start[c]; k < start[c + 1]; ++k) o.push_back(kids[k]);
        for (int64_t i = 0; i < nn; ++i)
            if (agg[i] < 0) o.push_back(i);
    }
    ord.assign(L, {});
    pos.assign(L, {});
    for (int l = 0; l < L; ++l) {
        const int64_t nr = H.lv[l].A.nrows;
        ord[l].resize(nr);
        pos[l].resize(nr);
        for (int64_t k = 0; k < (int64_t)node[l].size(); ++k)
            for (int b = 0; b < bs; ++b) ord[l][k * bs + b] = node[l][k] * bs + b;
        for (int64_t r = 0; r < nr; ++r) pos[l][ord[l][r]] = r;
    }
}


// Rank of the local block of one subdomain (rows x ndv, row-major) by
// Gram-Schmidt with reorthogonalisation; columns whose remaining norm is
// below 1e-12 times the largest column norm count as dependent.
int local_rank(const double *Z, int64_t rows, int ndv) {
    std::vector<double> Q((size_t)rows * ndv);
    for (int64_t i = 0; i < rows * ndv; ++i) Q[i] = Z[i];
    double maxnorm = 0.0;
    for (int k = 0; k < ndv; ++k) {
        double s = 0.0;
        for (int64_t i = 0; i < rows; ++i) s += Q[i * ndv + k] * Q[i * ndv + k];
        maxnorm = std::max(maxnorm, std::sqrt(s));
    }
    if (maxnorm == 0.0) return 0;
    int rank = 0;
    std::vector<char> keep(ndv, 0);
    for (int k = 0; k < ndv; ++k) {
        for (int pass = 0; pass < 2; ++pass)
            for (int q = 0; q < k; ++q) {
                if (!keep[q]) continue;
                double d = 0.0;
                for (int64_t i = 0; i < rows; ++i) d += Q[i * ndv + q] * Q[i * ndv + k];
                for (int64_t i = 0; i < rows; ++i) Q[i * ndv + k] -= d * Q[i * ndv + q];
            }
        double s = 0.0;
        for (int64_t i = 0; i < rows; ++i) s += Q[i * ndv + k] * Q[i * ndv + k];
        s = std::sqrt(s);
        if (s > 1e-12 * maxnorm) {
            keep[k] = 1;
            ++rank;
            for (int64_t i = 0; i < rows; ++i) Q[i * ndv + k] /= s;
        }
    }
    return rank;
}

}  // namespace

void validate_params(const dfamg_params &p) {
    if (p.solver != DFAMG_SOLVER_CG && p.solver != DFAMG_SOLVER_BICGSTAB && p.solver != DFAMG_SOLVER_BICGSTAB2 &&
        p.solver != DFAMG_SOLVER_FGMRES)
        fail(DFAMG_EINVAL, "unknown solver");
    if (p.solver == DFAMG_SOLVER_FGMRES && (p.restart < 1 || p.restart > 64))
        fail(DFAMG_EINVAL, "restart must be in [1, 64]");
    if (p.coarse_solve != DFAMG_COARSE_EXACT && p.coarse_solve != DFAMG_COARSE_FP32 &&
        p.coarse_solve != DFAMG_COARSE_CG)
        fail(DFAMG_EINVAL, "unknown coarse_solve");
    if (p.coarse_solve != DFAMG_COARSE_EXACT && p.solver != DFAMG_SOLVER_FGMRES)
        fail(DFAMG_EINVAL, "an inexact coarse solve needs solver = FGMRES (the projected solvers need the exact E)");
    if (p.coarse_solve == DFAMG_COARSE_CG) {
        if (!(p.coarse_rtol >= 0.0) || !std::isfinite(p.coarse_rtol)) fail(DFAMG_EINVAL, "coarse_rtol must be >= 0");
        if (p.coarse_maxiter < 1) fail(DFAMG_EINVAL, "coarse_maxiter must be >= 1");
    }
    if (p.maxiter < 0) fail(DFAMG_EINVAL, "maxiter must be >= 0");
    if (!(p.rtol >= 0.0) || !std::isfinite(p.rtol)) fail(DFAMG_EINVAL, "rtol must be finite and >= 0");
    if (p.precision != DFAMG_PREC_FP64 && p.precision != DFAMG_PREC_MIXED) fail(DFAMG_EINVAL, "unknown precision");
    if (p.smoother != DFAMG_SMOOTHER_SPAI0 && p.smoother != DFAMG_SMOOTHER_JACOBI &&
        p.smoother != DFAMG_SMOOTHER_BLOCK_SPAI0)
        fail(DFAMG_EINVAL, "unknown smoother");
    if (!std::isfinite(p.jacobi_omega)) fail(DFAMG_EINVAL, "jacobi_omega must be finite");
    if (p.coarse_enough < 1) fail(DFAMG_EINVAL, "coarse_enough must be >= 1");
    if (p.coarse_enough > 4096) fail(DFAMG_EINVAL, "coarse_enough must be <= 4096 (dense coarsest blocks)");
    if (!(p.eps_strong >= 0.0) || !std::isfinite(p.eps_strong)) fail(DFAMG_EINVAL, "eps_strong must be >= 0");
    if (p.max_levels < 1 || p.max_levels > 20) fail(DFAMG_EINVAL, "max_levels must be in [1, 20]");
    if (p.block_size < 1 || p.block_size > 8) fail(DFAMG_EINVAL, "block_size must be in [1, 8]");
    if (p.precond != DFAMG_PRECOND_AMG && p.precond != DFAMG_PRECOND_NONE && p.precond != DFAMG_PRECOND_SPAI0)
        fail(DFAMG_EINVAL, "unknown precond");
    if (p.spmv_format < DFAMG_FORMAT_AUTO || p.spmv_format > DFAMG_FORMAT_COLUMN_TILED)
        fail(DFAMG_EINVAL, "unknown spmv_format");
    if (p.spmv_format == DFAMG_FORMAT_BSR4 && p.block_size != 4)
        fail(DFAMG_EINVAL, "spmv_format BSR4 needs block_size 4");
    if (p.graph_iters < 0) fail(DFAMG_EINVAL, "graph_iters must be >= 0");
    if (p.flexible_cg != 0 && p.flexible_cg != 1) fail(DFAMG_EINVAL, "flexible_cg must be 0 or 1");
    if (p.flexible_cg && p.solver != DFAMG_SOLVER_CG) fail(DFAMG_EINVAL, "flexible_cg needs solver = CG");
    if (p.setup_device != 0 && p.setup_device != 1) fail(DFAMG_EINVAL, "setup_device must be 0 or 1");
    if (p.setup_device && p.precond == DFAMG_PRECOND_AMG &&
        (p.block_size != 1 || p.smoother == DFAMG_SMOOTHER_BLOCK_SPAI0))
        fail(DFAMG_EINVAL, "setup_device = 1 builds scalar hierarchies with a diagonal smoother only "
                           "(block_size 1, SPAI-0 or damped Jacobi)");
    if (p.npre < 0 || p.npre > 4) fail(DFAMG_EINVAL, "npre must be in [0, 4]");
    if (p.npost < 1 || p.npost > 4) fail(DFAMG_EINVAL, "npost must be in [1, 4]");
    if ((p.npre != 1 || p.npost != 1) && p.smoother == DFAMG_SMOOTHER_BLOCK_SPAI0)
        fail(DFAMG_EINVAL, "the block SPAI-0 smoother supports npre = npost = 1 only");
}

void build_plan(Plan &plan, const dfamg_params &prm, int32_t nsys, const int64_t *sys_row_off,
                int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                const int32_t *part, int32_t nsub, int32_t ndv, const double *Z, void *stream) {
    const auto t0 = std::chrono::steady_clock::now();
    validate_params(prm);
    plan.prm = prm;
    const int bs = prm.block_size;
    const int threads = prm.host_threads;
    if (n < 1) fail(DFAMG_EINVAL, "n must be >= 1");
    if (n >= (int64_t)std::numeric_limits<int32_t>::max() / 2) fail(DFAMG_EINVAL, "n too large for 32-bit row indices");
    if (!row_ptr || !col || !val || !part) fail(DFAMG_EINVAL, "null input array");
    if (nsub < 1) fail(DFAMG_EINVAL, "nsub must be >= 1");
    if (ndv < 0 || ndv > 8) fail(DFAMG_EINVAL, "ndv must be in [0, 8]");
    if (ndv > 0 && !Z) fail(DFAMG_EINVAL, "Z is NULL");
    if (nsys < 1) fail(DFAMG_EINVAL, "nsys must be >= 1");
    if (n % bs != 0) fail(DFAMG_EINVAL, "n is not a multiple of block_size");
    if (row_ptr[0] != 0) fail(DFAMG_EINVAL, "row_ptr[0] must be 0");
    for (int64_t i = 0; i < n; ++i)
        if (row_ptr[i + 1] < row_ptr[i]) fail(DFAMG_EINVAL, "row_ptr is not monotone at row " + std::to_string(i));
    const int64_t nnz = row_ptr[n];
    if (nnz >= (int64_t)std::numeric_limits<int32_t>::max()) fail(DFAMG_EINVAL, "too many nonzeros for 32-bit offsets");
    std::vector<int64_t> soff(nsys + 1);
    if (sys_row_off) {
        for (int s = 0; s <= nsys; ++s) soff[s] = sys_row_off[s];
        if (soff[0] != 0 || soff[nsys] != n) fail(DFAMG_EINVAL, "sys_row_off must start at 0 and end at n");
        for (int s = 0; s < nsys; ++s) {
            if (soff[s + 1] <= soff[s]) fail(DFAMG_EINVAL, "every system needs at least one row");
            if (soff[s] % bs) fail(DFAMG_EINVAL, "system boundaries must align with blocks");
        }
    } else {
        if (nsys != 1) fail(DFAMG_EINVAL, "sys_row_off required for nsys > 1");
        soff[0] = 0;
        soff[1] = n;
    }
    std::vector<int32_t> row_sys(n);
    for (int s = 0; s < nsys; ++s)
        for (int64_t i = soff[s]; i < soff[s + 1]; ++i) row_sys[i] = s;
    // partition
    std::vector<int32_t> user_sys(nsub, -1);
    std::vector<int64_t> cnt(nsub, 0);
    for (int64_t i = 0; i < n; ++i) {
        const int32_t p = part[i];
        if (p < 0 || p >= nsub) fail(DFAMG_EINVAL, "part[" + std::to_string(i) + "] out of range");
        if (user_sys[p] < 0) user_sys[p] = row_sys[i];
        else if (user_sys[p] != row_sys[i]) fail(DFAMG_EINVAL, "subdomain " + std::to_string(p) + " spans two systems");
        if (bs > 1 && part[i - i % bs] != p) fail(DFAMG_EINVAL, "a node's unknowns lie in different subdomains");
        cnt[p]++;
    }
    for (int p = 0; p < nsub; ++p)
        if (cnt[p] == 0) fail(DFAMG_EINVAL, "subdomain " + std::to_string(p) + " is empty");
    for (int64_t k = 0; k < nnz; ++k) {
        if (col[k] < 0 || col[k] >= n) fail(DFAMG_EINVAL, "column index out of range at entry " + std::to_string(k));
        if (!std::isfinite(val[k])) fail(DFAMG_EINVAL, "non-finite matrix value at entry " + std::to_string(k));
    }
    if (ndv > 0)
        for (int64_t k = 0; k < n * ndv; ++k)
            if (!std::isfinite(Z[k])) fail(DFAMG_EINVAL, "non-finite deflation vector entry");

    plan.n = n;
    plan.nnz = nnz;
    plan.nsys = nsys;
    plan.nsub = nsub;
    plan.ndv = ndv;
    plan.bs = bs;

    // internal subdomain order: by system, then user id
    plan.sub_user.resize(nsub);
    std::iota(plan.sub_user.begin(), plan.sub_user.end(), 0);
    std::stable_sort(plan.sub_user.begin(), plan.sub_user.end(),
                     [&](int32_t a, int32_t b) { return user_sys[a] < user_sys[b]; });
    plan.user_to_sub.resize(nsub);
    plan.sub_sys.resize(nsub);
    for (int s = 0; s < nsub; ++s) {
        plan.user_to_sub[plan.sub_user[s]] = s;
        plan.sub_sys[s] = user_sys[plan.sub_user[s]];
    }
    plan.sys_sub_off.assign(nsys + 1, 0);
    for (int s = 0; s < nsub; ++s) plan.sys_sub_off[plan.sub_sys[s] + 1]++;
    for (int s = 0; s < nsys; ++s) {
        if (plan.sys_sub_off[s + 1] == 0) fail(DFAMG_EINVAL, "system " + std::to_string(s) + " has no subdomain");
        plan.sys_sub_off[s + 1] += plan.sys_sub_off[s];
    }
    plan.sub_row_off.assign(nsub + 1, 0);
    for (int s = 0; s < nsub; ++s) {
        plan.sub_row_off[s + 1] = plan.sub_row_off[s] + cnt[plan.sub_user[s]];
        if (cnt[plan.sub_user[s]] % bs) fail(DFAMG_EINVAL, "subdomain size not a multiple of block_size");
    }
    plan.sys_row_off.assign(nsys + 1, 0);
    for (int s = 0; s < nsys; ++s) plan.sys_row_off[s + 1] = plan.sub_row_off[plan.sys_sub_off[s + 1]];
    // stable counting sort of rows by internal subdomain
    plan.perm.resize(n);
    std::vector<int64_t> iperm(n);
    {
        std::vector<int64_t> pos(plan.sub_row_off.begin(), plan.sub_row_off.end() - 1);
        for (int64_t i = 0; i < n; ++i) {
            const int64_t d = pos[plan.user_to_sub[part[i]]]++;
            plan.perm[d] = i;
            iperm[i] = d;
        }
    }
    std::vector<int32_t> row_sub(n);
    for (int s = 0; s < nsub; ++s)
        for (int64_t i = plan.sub_row_off[s]; i < plan.sub_row_off[s + 1]; ++i) row_sub[i] = s;

    // permuted matrix, rows sorted, duplicates and cross-system entries rejected
    Csr &A = plan.A;
    A.nrows = A.ncols = n;
    A.ptr.assign(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) A.ptr[i + 1] = A.ptr[i] + (row_ptr[plan.perm[i] + 1] - row_ptr[plan.perm[i]]);
    A.col.resize(nnz);
    A.val.resize(nnz);
    parallel_for((n + 4095) / 4096, threads, [&](int64_t chunk) {
        std::vector<std::pair<int32_t, double>> row;
        const int64_t e = std::min<int64_t>(n, (chunk + 1) * 4096);
        for (int64_t i = chunk * 4096; i < e; ++i) {
            const int64_t o = plan.perm[i];
            row.clear();
            for (int64_t k = row_ptr[o]; k < row_ptr[o + 1]; ++k) row.emplace_back((int32_t)iperm[col[k]], val[k]);
            std::sort(row.begin(), row.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
            bool diag = false;
            for (size_t q = 0; q < row.size(); ++q) {
                if (q && row[q].first == row[q - 1].first)
                    fail(DFAMG_EINVAL, "duplicate column in row " + std::to_string(o));
                if (plan.sub_sys[row_sub[row[q].first]] != plan.sub_sys[row_sub[i]])
                    fail(DFAMG_EINVAL, "row " + std::to_string(o) + " couples two systems");
                if (row[q].first == i && row[q].second != 0.0) diag = true;
                A.col[A.ptr[i] + q] = row[q].first;
                A.val[A.ptr[i] + q] = row[q].second;
            }
            if (!diag) fail(DFAMG_EINVAL, "row " + std::to_string(o) + " has a zero or missing diagonal");
        }
    });
    // permuted deflation blocks
    plan.Z.assign((size_t)n * ndv, 0.0);
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < ndv; ++k) plan.Z[i * ndv + k] = Z[plan.perm[i] * ndv + k];
    if (ndv > 0) {
        std::vector<int32_t> bad(nsub, 0);
        parallel_for(nsub, threads, [&](int64_t s) {
            const int64_t r0 = plan.sub_row_off[s], rows = plan.sub_row_off[s + 1] - r0;
            bad[s] = rows < ndv || local_rank(&plan.Z[r0 * ndv], rows, ndv) < ndv;
        });
        for (int s = 0; s < nsub; ++s)
            if (bad[s]) fail(DFAMG_ESINGULAR, "deflation block of subdomain " + std::to_string(plan.sub_user[s]) +
                                                  " is rank deficient");
    }

    // AZ split into the own-subdomain part and the rest, then E per system
    plan.AZown.assign((size_t)n * ndv, 0.0);
    plan.AZoff.nrows = n;
    plan.AZoff.ncols = (int64_t)nsub * ndv;
    plan.AZoff.ptr.assign(n + 1, 0);
    if (ndv > 0 && prm.setup_device) {
        build_az_device(A, row_sub, plan.Z, ndv, plan.AZown, plan.AZoff, stream);
        plan.AZoff.ncols = (int64_t)nsub * ndv;
    } else if (ndv > 0) {
        std::vector<std::vector<std::pair<int32_t, double>>> off_rows(nsub);
        std::vector<std::vector<int64_t>> off_cnt(nsub);
        parallel_for(nsub, threads, [&](int64_t s) {
            const int64_t r0 = plan.sub_row_off[s], r1 = plan.sub_row_off[s + 1];
            auto &ent = off_rows[s];
            auto &rc = off_cnt[s];
            rc.assign(r1 - r0, 0);
            std::vector<std::pair<int32_t, double>> row;
            for (int64_t i = r0; i < r1; ++i) {
                row.clear();
                for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
                    const int64_t j = A.col[k];
                    const int32_t t = row_sub[j];
                    for (int q = 0; q < ndv; ++q) {
                        const double v = A.val[k] * plan.Z[j * ndv + q];
                        if (t == s) plan.AZown[i * ndv + q] += v;
                        else row.emplace_back(t * ndv + q, v);
                    }
                }
                std::stable_sort(row.begin(), row.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
                for (size_t q = 0; q < row.size();) {
                    size_t e = q + 1;
                    double v = row[q].second;
                    while (e < row.size() && row[e].first == row[q].first) v += row[e++].second;
                    ent.emplace_back(row[q].first, v);
                    rc[i - r0]++;
                    q = e;
                }
            }
        });
        for (int s = 0; s < nsub; ++s) {
            const int64_t r0 = plan.sub_row_off[s];
            for (size_t q = 0; q < off_cnt[s].size(); ++q) plan.AZoff.ptr[r0 + q + 1] = off_cnt[s][q];
        }
        for (int64_t i = 0; i < n; ++i) plan.AZoff.ptr[i + 1] += plan.AZoff.ptr[i];
        for (int s = 0; s < nsub; ++s)
            for (auto &e : off_rows[s]) {
                plan.AZoff.col.push_back(e.first);
                plan.AZoff.val.push_back(e.second);
            }
    }
    plan.sys_m.resize(nsys);
    plan.sys_E_off.assign(nsys + 1, 0);
    for (int s = 0; s < nsys; ++s) {
        plan.sys_m[s] = (plan.sys_sub_off[s + 1] - plan.sys_sub_off[s]) * ndv;
        plan.sys_E_off[s + 1] = plan.sys_E_off[s] + (int64_t)plan.sys_m[s] * plan.sys_m[s];
    }
    plan.E.assign(plan.sys_E_off[nsys], 0.0);
    if (ndv > 0)
        parallel_for(nsub, threads, [&](int64_t s) {
            const int sy = plan.sub_sys[s];
            const int64_t m = plan.sys_m[sy];
            const int32_t s0 = plan.sys_sub_off[sy];
            double *E = &plan.E[plan.sys_E_off[sy]];
            for (int64_t i = plan.sub_row_off[s]; i < plan.sub_row_off[s + 1]; ++i)
                for (int k = 0; k < ndv; ++k) {
                    const double z = plan.Z[i * ndv + k];
                    double *Erow = E + ((s - s0) * ndv + k) * m;
                    for (int q = 0; q < ndv; ++q) Erow[(s - s0) * ndv + q] += z * plan.AZown[i * ndv + q];
                    for (int64_t e = plan.AZoff.ptr[i]; e < plan.AZoff.ptr[i + 1]; ++e)
                        Erow[plan.AZoff.col[e] - (int64_t)s0 * ndv] += z * plan.AZoff.val[e];
                }
        });

    // per-subdomain hierarchies
    plan.hier.assign(nsub, Hierarchy{});
    SaParams sp;
    sp.eps_strong = prm.eps_strong;
    sp.coarse_enough = prm.coarse_enough;
    sp.max_levels = prm.precond == DFAMG_PRECOND_AMG ? prm.max_levels : 1;
    sp.smoother = prm.smoother;
    sp.jacobi_omega = prm.jacobi_omega;
    sp.bs = bs;
    const auto th = std::chrono::steady_clock::now();
    if (prm.precond == DFAMG_PRECOND_AMG) {
        // the square diagonal block of every subdomain
        std::vector<Csr> local(nsub);
        parallel_for(nsub, threads, [&](int64_t s) {
            const int64_t r0 = plan.sub_row_off[s], r1 = plan.sub_row_off[s + 1];
            Csr &L = local[s];
            L.nrows = L.ncols = r1 - r0;
            L.ptr.assign(r1 - r0 + 1, 0);
            for (int64_t i = r0; i < r1; ++i) {
                for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
                    if (A.col[k] >= r0 && A.col[k] < r1) {
                        L.col.push_back((int32_t)(A.col[k] - r0));
                        L.val.push_back(A.val[k]);
                    }
                L.ptr[i - r0 + 1] = (int64_t)L.col.size();
            }
        });
        if (prm.setup_device) {
            build_hierarchies_device(local, sp, plan.hier, stream);
            plan.hier_on_device = 1;
        } else {
            parallel_for(nsub, threads, [&](int64_t s) { plan.hier[s] = build_hierarchy(std::move(local[s]), sp); });
        }
    }
    plan.hier_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - th).count();

    // storage order of every subdomain's levels (identity on level 0 and on
    // the coarsest level)
    std::vector<std::vector<std::vector<int64_t>>> ord(nsub), pos(nsub);
    parallel_for(nsub, threads, [&](int64_t s) { level_orders(plan.hier[s], bs, ord[s], pos[s]); });

    // packed levels
    plan.nlevels_max = 0;
    for (auto &H : plan.hier) plan.nlevels_max = std::max(plan.nlevels_max, H.nlevels());
    plan.levels.assign(plan.nlevels_max, PackedLevel{});
    for (int l = 0; l < plan.nlevels_max; ++l) {
        PackedLevel &PL = plan.levels[l];
        PL.sub_off.assign(nsub, -1);
        PL.sub_len.assign(nsub, 0);
        int64_t off = 0;
        for (int s = 0; s < nsub; ++s) {
            const Hierarchy &H = plan.hier[s];
            if (H.nlevels() > l) {
                PL.sub_off[s] = off;
                PL.sub_len[s] = (int32_t)H.lv[l].A.nrows;
                off += H.lv[l].A.nrows;
                if (H.nlevels() - 1 > l) PL.active_subs.push_back(s);
                else PL.coarse_subs.push_back(s);
            }
        }
        PL.nrows = off;
    }
    for (int l = 0; l < plan.nlevels_max; ++l) {
        PackedLevel &PL = plan.levels[l];
        const bool has_next = l + 1 < plan.nlevels_max;
        const int64_t ncoarse = has_next ? plan.levels[l + 1].nrows : 0;
        PL.A.nrows = PL.A.ncols = PL.nrows;
        PL.A.ptr.assign(PL.nrows + 1, 0);
        PL.P.nrows = PL.nrows;
        PL.P.ncols = ncoarse;
        PL.P.ptr.assign(PL.nrows + 1, 0);
        PL.m.assign(PL.nrows, 0.0);
        if (prm.smoother == DFAMG_SMOOTHER_BLOCK_SPAI0) PL.mb.assign((size_t)PL.nrows * bs, 0.0);
        for (int s = 0; s < nsub; ++s) {
            if (PL.sub_off[s] < 0) continue;
            const Hierarchy &H = plan.hier[s];
            const bool active = H.nlevels() - 1 > l;
            const int64_t o = PL.sub_off[s];
            for (int64_t i = 0; i < PL.sub_len[s]; ++i) {
                if (active) {
                    const Csr &M = H.lv[l].A;
                    for (int64_t k = M.ptr[i]; k < M.ptr[i + 1]; ++k) {
                        PL.A.col.push_back((int32_t)(M.col[k] + o));
                        PL.A.val.push_back(M.val[k]);
                    }
                    const Csr &P = H.lv[l].P;
                    const int64_t oc = plan.levels[l + 1].sub_off[s];
                    for (int64_t k = P.ptr[i]; k < P.ptr[i + 1]; ++k) {
                        PL.P.col.push_back((int32_t)(P.col[k] + oc));
                        PL.P.val.push_back(P.val[k]);
                    }
                    PL.m[o + i] = H.lv[l].m[i];
                    if (!H.lv[l].mb.empty())
                        for (int k = 0; k < bs; ++k) PL.mb[(size_t)(o + i) * bs + k] = H.lv[l].mb[(size_t)i * bs + k];
                }
                PL.A.ptr[o + i + 1] = (int64_t)PL.A.col.size();
                PL.P.ptr[o + i + 1] = (int64_t)PL.P.col.size();
            }
        }
        PL.R = transpose(PL.P);
        // B packed like R: rows of the next level's packed order, this level's columns
        // B in the natural row order, and again with the rows of every
        // subdomain in the next level's clustered order (Bc, with the map
        // from its rows to the natural packed rows); the device keeps the
        // faster of the two
        auto pack_b = [&](Csr &B, bool clustered, std::vector<int32_t> *rowmap) {
            B.nrows = ncoarse;
            B.ncols = PL.nrows;
            B.ptr.assign(ncoarse + 1, 0);
            if (!has_next) return;
            if (rowmap) {
                rowmap->resize(ncoarse);
                for (int64_t k = 0; k < ncoarse; ++k) (*rowmap)[k] = (int32_t)k;
            }
            auto src = [&](int s, int64_t k) { return clustered ? ord[s][l + 1][k] : k; };
            for (int s = 0; s < nsub; ++s) {
                if (PL.sub_off[s] < 0 || plan.hier[s].nlevels() - 1 <= l) continue;
                const Csr &Bs = plan.hier[s].lv[l].B;
                const int64_t oc = plan.levels[l + 1].sub_off[s];
                for (int64_t k = 0; k < Bs.nrows; ++k) B.ptr[oc + k + 1] = Bs.ptr[src(s, k) + 1] - Bs.ptr[src(s, k)];
            }
            for (int64_t k = 0; k < ncoarse; ++k) B.ptr[k + 1] += B.ptr[k];
            B.col.resize(B.ptr[ncoarse]);
            B.val.resize(B.ptr[ncoarse]);
            for (int s = 0; s < nsub; ++s) {
                if (PL.sub_off[s] < 0 || plan.hier[s].nlevels() - 1 <= l) continue;
                const Csr &Bs = plan.hier[s].lv[l].B;
                const int64_t o = PL.sub_off[s], oc = plan.levels[l + 1].sub_off[s];
                for (int64_t k = 0; k < Bs.nrows; ++k) {
                    const int64_t r = src(s, k);
                    int64_t d = B.ptr[oc + k];
                    for (int64_t e = Bs.ptr[r]; e < Bs.ptr[r + 1]; ++e, ++d) {
                        B.col[d] = (int32_t)(Bs.col[e] + o);
                        B.val[d] = Bs.val[e];
                    }
                    if (rowmap) (*rowmap)[oc + k] = (int32_t)(oc + r);
                }
            }
        };
        pack_b(PL.B, false, nullptr);
        pack_b(PL.Bc, true, &PL.B_rowmap);
    }
    plan.host_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace dfamg
