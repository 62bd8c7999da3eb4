// Test-only C entry points that run single kernels of the library on host
// buffers (GEMM, permute, Jacobi SVD), so that kernel-level numerics can be
// checked in isolation.  Built into libctm_selftest.so, not into libctm.so.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace {
template <class T>
T* dev_copy(const T* h, size_t n)
{
    T* d = nullptr;
    if (hipMalloc(&d, n * sizeof(T) + 8) != hipSuccess) return nullptr;
    if (h && hipMemcpy(d, h, n * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
    return d;
}
}  // namespace

extern "C" {

// C[batch][M][N] = op(A) op(B), all row-major, host buffers
int ctm_selftest_gemm(int ta, int tb, int M, int N, int K, int batch, const double* A,
                      const double* B, double* C)
{
    const size_t na = (size_t)M * K * batch, nb = (size_t)K * N * batch, nc = (size_t)M * N * batch;
    double *dA = dev_copy(A, na), *dB = dev_copy(B, nb), *dC = dev_copy<double>(nullptr, nc);
    if (!dA || !dB || !dC) return 1;
    ctmk::gemm_f64(nullptr, ta != 0, tb != 0, M, N, K, 1.0, dA, ta ? M : K, (int64_t)M * K, dB,
                   tb ? K : N, (int64_t)K * N, 0.0, dC, N, (int64_t)M * N, batch);
    int rc = hipMemcpy(C, dC, nc * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess;
    rc |= hipDeviceSynchronize() != hipSuccess;
    (void)hipFree(dA);
    (void)hipFree(dB);
    (void)hipFree(dC);
    return rc;
}

// X (m x n column-major) = U S V^T
int ctm_selftest_jacobi(int m, int n, const double* X, double* U, double* S, double* V)
{
    double *dX = dev_copy(X, (size_t)m * n), *dW = dev_copy<double>(nullptr, (size_t)n * n);
    double *dU = dev_copy<double>(nullptr, (size_t)m * n), *dV = dev_copy<double>(nullptr, (size_t)n * n);
    double* dS = dev_copy<double>(nullptr, n);
    if (!dX || !dW || !dU || !dV || !dS) return 1;
    ctmk::JacobiBatch jb{};
    jb.n = 1;
    jb.job[0] = ctmk::JacobiJob{dX, dW, dU, dV, dS, m, n, 1};
    ctmk::jacobi_svd(nullptr, jb, 40);
    int rc = hipDeviceSynchronize() != hipSuccess;
    rc |= hipMemcpy(U, dU, (size_t)m * n * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess;
    rc |= hipMemcpy(V, dV, (size_t)n * n * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess;
    rc |= hipMemcpy(S, dS, (size_t)n * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess;
    (void)hipFree(dX);
    (void)hipFree(dW);
    (void)hipFree(dU);
    (void)hipFree(dV);
    (void)hipFree(dS);
    return rc;
}

}  // extern "C"
