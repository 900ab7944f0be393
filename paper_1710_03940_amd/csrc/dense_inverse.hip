// Dense FP64 inverse of the coarse operator E on the GPU, blocked for size.
//
// E = Z^T A Z has nsub x ndv rows per system; the paper observes that its
// factorisation dominates the setup at scale (section "Benchmarks", the
// profiling tables).  The inverse is formed in place by Gauss-Jordan
// elimination with partial pivoting in column panels of width kPanel
// (the blocked in-place variant of Quintana-Orti, Quintana-Orti, Sun and van
// de Geijn, "A note on parallel matrix inversion", SIAM J. Sci. Comput. 22,
// 2001): per panel, the unblocked in-place steps are applied to the n x b
// panel (pivot search over the rows not yet used as pivots, whole-row swaps;
// one workgroup for the pivot row, one wavefront per other row), which leaves
// [-A01 A11^{-1}; A11^{-1}; -A21 A11^{-1}] in it; the
// rest of the matrix is then updated with six GEMMs (rocBLAS, which runs them
// on the FP64 matrix cores):
//   [A00 A02; A20 A22] += [A01; A21] [A10 A12],   [A10 A12] := A11 [A10 A12].
// After the last panel the matrix holds (P A)^{-1}; the column swaps undo P.
// The work is 2 n^3 flops with the n^2 b-sized panel work outside the GEMMs,
// against an unblocked elimination that streams the whole matrix once per
// pivot.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "dense_inverse.hpp"

namespace dfamg {

namespace {

constexpr int kPanel = 64;
constexpr int kPanelThreads = 1024;

void hip_ok(hipError_t e, const char *what) {
    if (e != hipSuccess) throw DenseInverseError{std::string(what) + ": " + hipGetErrorString(e)};
}

void rb_ok(rocblas_status s, const char *what) {
    if (s != rocblas_status_success) throw DenseInverseError{std::string(what) + ": rocBLAS status " +
                                                             std::to_string((int)s)};
}

// Unblocked in-place Gauss-Jordan step k on the panel columns [K, K+b) of
// the row-major n x n matrix A, in two launches.  Step k: pivot p = first row
// of largest |a_ik| among i >= k, rows k and p swapped over all n columns;
// then with d = a_kk: a_kj /= d (panel j != k), a_kk = 1 / d (this kernel,
// one workgroup), and a_ij -= a_ik a_kj (i != k, panel j != k), a_ik = -a_ik / d
// (k_gjb_step, one wavefront per row).  rowk receives the scaled pivot row's
// panel entries and dk[0] = d.
__global__ void __launch_bounds__(kPanelThreads) k_gjb_pivot(double *__restrict__ A, int n, int K, int b, int k,
                                                             int32_t *__restrict__ piv, int32_t *__restrict__ singular,
                                                             double *__restrict__ rowk, double *__restrict__ dk) {
    __shared__ double bv[kPanelThreads];
    __shared__ int bi[kPanelThreads];
    if (*singular) return;
    const int t = threadIdx.x;
    double best = -1.0;
    int bidx = n;
    for (int i = k + t; i < n; i += kPanelThreads) {
        const double v = fabs(A[(int64_t)i * n + k]);
        if (v > best) {
            best = v;
            bidx = i;
        }
    }
    bv[t] = best;
    bi[t] = bidx;
    __syncthreads();
    for (int s = kPanelThreads / 2; s > 0; s >>= 1) {
        if (t < s) {
            const double o = bv[t + s];
            const int oi = bi[t + s];
            if (o > bv[t] || (o == bv[t] && oi < bi[t])) {
                bv[t] = o;
                bi[t] = oi;
            }
        }
        __syncthreads();
    }
    const int p = bi[0];
    if (!(bv[0] > 0.0) || p >= n) {   // uniform: every thread read the same LDS values
        if (t == 0) *singular = 1;
        return;
    }
    if (t == 0) piv[k] = p;
    if (p != k)
        for (int j = t; j < n; j += kPanelThreads) {
            const double a = A[(int64_t)k * n + j];
            A[(int64_t)k * n + j] = A[(int64_t)p * n + j];
            A[(int64_t)p * n + j] = a;
        }
    __syncthreads();
    const double d = A[(int64_t)k * n + k];
    __syncthreads();
    if (t < b) {
        const int j = K + t;
        const double v = j != k ? A[(int64_t)k * n + j] / d : 0.0;
        if (j != k) A[(int64_t)k * n + j] = v;
        else A[(int64_t)k * n + j] = 1.0 / d;
        rowk[t] = v;
    }
    if (t == 0) dk[0] = d;
}

// Rows i != k of step k (see k_gjb_pivot): lane jj of the row's wavefront
// owns panel column K + jj; a_ik is loaded by every lane before the lane of
// column k overwrites it.
__global__ void __launch_bounds__(256) k_gjb_step(double *__restrict__ A, int n, int K, int b, int k,
                                                  const int32_t *__restrict__ singular,
                                                  const double *__restrict__ rowk, const double *__restrict__ dk) {
    if (*singular) return;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int jj = threadIdx.x & 63;
    if (i >= n || i == k) return;
    double *r = A + (int64_t)i * n;
    const double aik = r[k];
    if (jj >= b) return;
    const int j = K + jj;
    if (j == k) r[k] = -aik / dk[0];
    else r[j] -= aik * rowk[jj];
}

// W (b x n) = rows [K, K+b) of A
__global__ void k_gjb_copy_rows(const double *__restrict__ A, int n, int K, int b, double *__restrict__ W) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < (int64_t)b * n) W[e] = A[(int64_t)K * n + e];
}

// piv[k] = k: the interchanges of a matrix found singular part-way stay
// within bounds
__global__ void k_gjb_piv_init(int32_t *__restrict__ piv, int n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) piv[k] = k;
}

// Undo the row interchanges: swap columns k and piv[k] for k = n-1 .. 0 (one
// thread per row).
__global__ void k_gjb_colswap(double *__restrict__ A, int n, const int32_t *__restrict__ piv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double *r = A + (int64_t)i * n;
    for (int k = n - 1; k >= 0; --k) {
        const int p = piv[k];
        if (p != k) {
            const double a = r[k];
            r[k] = r[p];
            r[p] = a;
        }
    }
}

// Row-major C (rows x cols, ldc) = beta C + A (rows x kk, lda) B (kk x cols, ldb),
// issued as the column-major product C^T = B^T A^T.
void gemm_rm(rocblas_handle h, int rows, int cols, int kk, const double *Ap, int lda, const double *Bp, int ldb,
             double beta, double *Cp, int ldc) {
    if (rows <= 0 || cols <= 0 || kk <= 0) return;
    const double one = 1.0;
    rb_ok(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, cols, rows, kk, &one, Bp, ldb, Ap, lda,
                        &beta, Cp, ldc),
          "rocblas_dgemm");
}

// One rocBLAS handle per device for the life of the process (creating one
// costs milliseconds); the caller holds the returned lock while using it.
rocblas_handle device_handle(std::unique_lock<std::mutex> &lk) {
    static std::mutex mu;
    static std::map<int, rocblas_handle> handles;
    lk = std::unique_lock<std::mutex>(mu);
    int dev = 0;
    hip_ok(hipGetDevice(&dev), "hipGetDevice");
    auto it = handles.find(dev);
    if (it != handles.end()) return it->second;
    rocblas_handle h = nullptr;
    rb_ok(rocblas_create_handle(&h), "rocblas_create_handle");
    handles[dev] = h;
    return h;
}

}  // namespace

bool invert_dense_inplace(hipStream_t s, double *A, int n) {
    if (n <= 0) return true;
    int32_t *piv = nullptr, *sing = nullptr;
    double *W = nullptr, *rowk = nullptr, *dk = nullptr;
    std::unique_lock<std::mutex> lk;
    auto release = [&] {
        if (W) (void)hipFree(W);
        if (rowk) (void)hipFree(rowk);
        if (dk) (void)hipFree(dk);
        if (piv) (void)hipFree(piv);
        if (sing) (void)hipFree(sing);
    };
    try {
        hip_ok(hipMalloc(&piv, sizeof(int32_t) * n), "hipMalloc");
        hip_ok(hipMalloc(&sing, sizeof(int32_t)), "hipMalloc");
        hip_ok(hipMalloc(&W, sizeof(double) * (size_t)kPanel * n), "hipMalloc");
        hip_ok(hipMalloc(&rowk, sizeof(double) * kPanel), "hipMalloc");
        hip_ok(hipMalloc(&dk, sizeof(double)), "hipMalloc");
        hip_ok(hipMemsetAsync(sing, 0, sizeof(int32_t), s), "hipMemsetAsync");
        hipLaunchKernelGGL(k_gjb_piv_init, dim3((n + 255) / 256), dim3(256), 0, s, piv, n);
        rocblas_handle h = device_handle(lk);
        rb_ok(rocblas_set_stream(h, s), "rocblas_set_stream");
        rb_ok(rocblas_set_pointer_mode(h, rocblas_pointer_mode_host), "rocblas_set_pointer_mode");
        for (int K = 0; K < n; K += kPanel) {
            const int b = std::min(kPanel, n - K);
            const int R = K + b;   // first row / column after the panel
            for (int k = K; k < R; ++k) {
                hipLaunchKernelGGL(k_gjb_pivot, dim3(1), dim3(kPanelThreads), 0, s, A, n, K, b, k, piv, sing, rowk,
                                   dk);
                hipLaunchKernelGGL(k_gjb_step, dim3((n + 3) / 4), dim3(256), 0, s, A, n, K, b, k, sing, rowk, dk);
            }
            const int64_t nw = (int64_t)b * n;
            hipLaunchKernelGGL(k_gjb_copy_rows, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, A, n, K, b, W);
            hip_ok(hipGetLastError(), "panel launch");
            const double *P_top = A + K;                        // rows [0, K), panel columns
            const double *P_bot = A + (int64_t)R * n + K;       // rows [R, n), panel columns
            // [A00 A02; A20 A22] += [A01; A21] [A10 A12]   (W holds [A10 A11 A12])
            gemm_rm(h, K, K, b, P_top, n, W, n, 1.0, A, n);
            gemm_rm(h, K, n - R, b, P_top, n, W + R, n, 1.0, A + R, n);
            gemm_rm(h, n - R, K, b, P_bot, n, W, n, 1.0, A + (int64_t)R * n, n);
            gemm_rm(h, n - R, n - R, b, P_bot, n, W + R, n, 1.0, A + (int64_t)R * n + R, n);
            // [A10 A12] := A11 [A10 A12]
            const double *A11 = A + (int64_t)K * n + K;
            gemm_rm(h, b, K, b, A11, n, W, n, 0.0, A + (int64_t)K * n, n);
            gemm_rm(h, b, n - R, b, A11, n, W + R, n, 0.0, A + (int64_t)K * n + R, n);
        }
        hipLaunchKernelGGL(k_gjb_colswap, dim3((n + 255) / 256), dim3(256), 0, s, A, n, piv);
        hip_ok(hipGetLastError(), "colswap launch");
        int32_t hs = 0;
        hip_ok(hipMemcpyAsync(&hs, sing, sizeof(int32_t), hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
        hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize");
        release();
        return hs == 0;
    } catch (...) {
        (void)hipStreamSynchronize(s);
        release();
        throw;
    }
}

}  // namespace dfamg
