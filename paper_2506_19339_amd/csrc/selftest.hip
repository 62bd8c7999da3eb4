// Test-only C entry points that run single kernels of the library on host
// buffers (GEMM, Jacobi SVD, Cholesky QR factor), so that kernel-level numerics can be
// checked in isolation.  Built into libctm_selftest.so, not into libctm.so.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "kernels.h"
#include "perm_plan.h"

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

// C[batch][M][N] = op(A) op(B), all row-major, host buffers.  ws_cap > 0
// gives the GEMM a split-K workspace of that many doubles.
int ctm_selftest_gemm(int ta, int tb, int M, int N, int K, int batch, const double* A,
                      const double* B, double* C, long long ws_cap)
{
    const size_t na = (size_t)M * K * batch, nb = (size_t)K * N * batch, nc = (size_t)M * N * batch;
    double *dA = dev_copy(A, na), *dB = dev_copy(B, nb), *dC = dev_copy<double>(nullptr, nc);
    double* dW = ws_cap > 0 ? dev_copy<double>(nullptr, (size_t)ws_cap) : nullptr;
    if (!dA || !dB || !dC || (ws_cap > 0 && !dW)) return 1;
    ctmk::gemm_f64(nullptr, ta != 0, tb != 0, M, N, K, 1.0, dA, ta ? M : K, (int64_t)M * K, dB,
                   tb ? K : N, (int64_t)K * N, 0.0, dC, N, (int64_t)M * N, batch, dW, ws_cap);
    int rc = hipMemcpy(C, dC, nc * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess;
    rc |= hipDeviceSynchronize() != hipSuccess;
    (void)hipFree(dA);
    (void)hipFree(dB);
    (void)hipFree(dC);
    if (dW) (void)hipFree(dW);
    return rc;
}

// grouped GEMM of n problems (shapes M[i], N[i], K[i]; dense operands packed
// one after the other in A, B and C as for ctm_selftest_gemm with batch 1);
// returns the number of problems whose K range was split through *n_split
int ctm_selftest_gemm_group(int ta, int tb, int n, const int* M, const int* N, const int* K, const double* A,
                            const double* B, double* C, long long ws_cap, int* n_split)
{
    if (n < 1 || n > ctmk::kMaxGemmGroup) return 1;
    size_t na = 0, nb = 0, nc = 0;
    for (int i = 0; i < n; ++i) {
        na += (size_t)M[i] * K[i];
        nb += (size_t)K[i] * N[i];
        nc += (size_t)M[i] * N[i];
    }
    double *dA = dev_copy(A, na), *dB = dev_copy(B, nb), *dC = dev_copy<double>(nullptr, nc);
    double* dW = ws_cap > 0 ? dev_copy<double>(nullptr, (size_t)ws_cap) : nullptr;
    if (!dA || !dB || !dC || (ws_cap > 0 && !dW)) return 1;
    ctmk::GemmProb pr[ctmk::kMaxGemmGroup];
    size_t oa = 0, ob = 0, oc = 0;
    for (int i = 0; i < n; ++i) {
        pr[i] = ctmk::GemmProb{dA + oa, dB + ob, dC + oc, M[i], N[i], K[i], ta ? M[i] : K[i], tb ? K[i] : N[i], N[i]};
        oa += (size_t)M[i] * K[i];
        ob += (size_t)K[i] * N[i];
        oc += (size_t)M[i] * N[i];
    }
    if (n_split) *n_split = ctmk::gemm_group_splits(pr, n, ws_cap);
    ctmk::gemm_f64_group(nullptr, ta != 0, tb != 0, pr, n, 1.0, dW, ws_cap, nullptr);
    int rc = hipMemcpy(C, dC, nc * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess;
    rc |= hipDeviceSynchronize() != hipSuccess;
    (void)hipFree(dA);
    (void)hipFree(dB);
    (void)hipFree(dC);
    if (dW) (void)hipFree(dW);
    return rc;
}

// sign convention of singular-vector pairs, in place on host copies
int ctm_selftest_sign_fix(int rows, int m, int n, double* UT, double* VT)
{
    double *dU = dev_copy(UT, (size_t)rows * m), *dV = dev_copy(VT, (size_t)rows * n);
    if (!dU || !dV) return 1;
    ctmk::sign_fix(nullptr, dU, dV, rows, m, n);
    int rc = hipMemcpy(UT, dU, (size_t)rows * m * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess;
    rc |= hipMemcpy(VT, dV, (size_t)rows * n * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess;
    rc |= hipDeviceSynchronize() != hipSuccess;
    (void)hipFree(dU);
    (void)hipFree(dV);
    return rc;
}

// the same with FP32 (prec 1) or BF16 (prec 2) products and FP32 accumulation
int ctm_selftest_gemm_lp(int prec, int ta, int tb, int M, int N, int K, int batch, const double* A,
                         const double* B, double* C, long long ws_cap)
{
    const size_t na = (size_t)M * K * batch, nb = (size_t)K * N * batch, nc = (size_t)M * N * batch;
    double *dA = dev_copy(A, na), *dB = dev_copy(B, nb), *dC = dev_copy<double>(nullptr, nc);
    double* dW = ws_cap > 0 ? dev_copy<double>(nullptr, (size_t)ws_cap) : nullptr;
    if (!dA || !dB || !dC || (ws_cap > 0 && !dW)) return 1;
    ctmk::gemm_lp(nullptr, prec, ta != 0, tb != 0, M, N, K, 1.0, dA, ta ? M : K, (int64_t)M * K, dB,
                  tb ? K : N, (int64_t)K * N, 0.0, dC, N, (int64_t)M * N, batch, dW, ws_cap);
    int rc = hipMemcpy(C, dC, nc * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess;
    rc |= hipDeviceSynchronize() != hipSuccess;
    (void)hipFree(dA);
    (void)hipFree(dB);
    (void)hipFree(dC);
    if (dW) (void)hipFree(dW);
    return rc;
}

// 1 when ctmk::permute takes the LDS-tiled form for transpose(dims, axes)
// (same arguments as ctm_selftest_permute), 0 otherwise
int ctm_selftest_permute_tiled(int rank, const long long* dims, const int* axes)
{
    int64_t n = 1, stride[12], od[12], is[12];
    for (int k = rank - 1; k >= 0; --k) {
        stride[k] = n;
        n *= dims[k];
    }
    for (int k = 0; k < rank; ++k) {
        od[k] = dims[axes[k]];
        is[k] = stride[axes[k]];
    }
    ctmk::PermTile t{};
    return ctmk::plan_perm_tile(rank, od, is, t) ? 1 : 0;
}

// Host check of the tiled permute's plan and index arithmetic (no device
// work): the tile loop of permute_tile_kernel replayed on the host for
// transpose(dims, axes) of in[i] = i, against the element-wise definition.
// Returns 1 when the plan takes the tiled form and every output element is
// written once with the right value, 0 when the plan keeps the element-wise
// form, -1 on a mismatch, -2 when a tile exceeds the kernel's LDS buffer.
int ctm_selftest_permute_tile_check(int rank, const long long* dims, const int* axes)
{
    int64_t n = 1, stride[12], od[12], is[12];
    for (int k = rank - 1; k >= 0; --k) {
        stride[k] = n;
        n *= dims[k];
    }
    for (int k = 0; k < rank; ++k) {
        od[k] = dims[axes[k]];
        is[k] = stride[axes[k]];
    }
    ctmk::PermTile t{};
    if (!ctmk::plan_perm_tile(rank, od, is, t)) return 0;
    auto fdiv = [](uint32_t x, const ctmk::FastDiv& f) {
        return (uint32_t)(((((uint64_t)x * f.mul) >> 32) + x) >> f.shr);
    };
    std::vector<double> out((size_t)n, -1.0), buf(ctmk::kPermTileElems + ctmk::kPermTileSide + 1);
    std::vector<uint32_t> itab(ctmk::kPermTileSide), otab(ctmk::kPermTileSide);
    const int U = t.U, P = (t.TI * t.U) | 1;
    for (uint32_t tile = 0; tile < (uint32_t)t.tiles; ++tile) {
        uint32_t r = fdiv(tile, t.fco);
        const int co = (int)(tile - r * t.fco.d);
        const uint32_t r2 = fdiv(r, t.fci);
        const int ci = (int)(r - r2 * t.fci.d);
        r = r2;
        uint32_t ib = 0, ob = 0;
        for (int k = 0; k < t.nrest; ++k) {
            const uint32_t q = fdiv(r, t.rest_d[k]);
            const uint32_t c = r - q * t.rest_d[k].d;
            r = q;
            ib += c * (uint32_t)t.rest_is[k];
            ob += c * (uint32_t)t.rest_os[k];
        }
        const int i0 = ci * t.TI, o0 = co * t.TO;
        const int ti = std::min(t.TI, t.Lin - i0), to = std::min(t.TO, t.Lout - o0);
        const ctmk::FastDiv& fr = t.frun[ci == t.nci - 1 ? 1 : 0];
        const ctmk::FastDiv& fo = t.fruno[co == t.nco - 1 ? 1 : 0];
        if ((int)fr.d != ti * U || (int)fo.d != to * U || to * P > (int)buf.size()) return -2;
        for (int o = 0; o < to; ++o) {
            uint32_t x = (uint32_t)(o0 + o), off = 0;
            for (int k = 0; k < t.nout; ++k) {
                const uint32_t q = x / (uint32_t)t.out_d[k];
                off += (x - q * (uint32_t)t.out_d[k]) * (uint32_t)t.out_is[k];
                x = q;
            }
            itab[o] = off;
        }
        for (int i = 0; i < ti; ++i) {
            uint32_t x = (uint32_t)(i0 + i), off = 0;
            for (int k = 0; k < t.nin; ++k) {
                const uint32_t q = x / (uint32_t)t.in_d[k];
                off += (x - q * (uint32_t)t.in_d[k]) * (uint32_t)t.in_os[k];
                x = q;
            }
            otab[i] = off;
        }
        const int run = (int)fr.d;
        const uint32_t ibase = ib + (uint32_t)i0 * (uint32_t)U;
        for (int e = 0; e < to * run; ++e) {
            const int o = (int)fdiv((uint32_t)e, fr);
            buf[o * P + (e - o * run)] = (double)(ibase + itab[o] + (uint32_t)(e - o * run));
        }
        const int runo = (int)fo.d;
        const uint32_t obase = ob + (uint32_t)o0 * (uint32_t)U;
        for (int e = 0; e < ti * runo; ++e) {
            const int i = (int)fdiv((uint32_t)e, fo);
            const int w = e - i * runo;
            const int o = (int)fdiv((uint32_t)w, t.fU);
            const uint32_t dst = obase + otab[i] + (uint32_t)w;
            if ((int64_t)dst >= n || out[dst] != -1.0) return -1;
            out[dst] = buf[o * P + i * U + (w - o * U)];
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        int64_t rem = i, off = 0;
        for (int k = rank - 1; k >= 0; --k) {
            off += (rem % od[k]) * is[k];
            rem /= od[k];
        }
        if (out[i] != (double)off) return -1;
    }
    return 1;
}

// out = transpose(in, axes): in has dims[0..rank-1] (row-major), out axis k is
// input axis axes[k]
int ctm_selftest_permute(int rank, const long long* dims, const int* axes, const double* in, double* out)
{
    int64_t n = 1, stride[12];
    for (int k = rank - 1; k >= 0; --k) {
        stride[k] = n;
        n *= dims[k];
    }
    ctmk::PermDesc pd{};
    pd.rank = rank;
    for (int k = 0; k < rank; ++k) {
        pd.od[k] = dims[axes[k]];
        pd.is[k] = stride[axes[k]];
    }
    double *di = dev_copy(in, (size_t)n), *dout = dev_copy<double>(nullptr, (size_t)n);
    if (!di || !dout) return 1;
    ctmk::permute(nullptr, di, dout, pd, n);
    int rc = hipMemcpy(out, dout, (size_t)n * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess;
    rc |= hipDeviceSynchronize() != hipSuccess;
    (void)hipFree(di);
    (void)hipFree(dout);
    return rc;
}

// number of K slices gemm_f64 uses for this shape and workspace
int ctm_selftest_gemm_splits(int M, int N, int K, int batch, long long ws_cap)
{
    return ctmk::gemm_split_plan(M, N, K, batch, ws_cap);
}

// T = L^-1 D for G (k x k, row-major Gram matrix): D = diag(G)^-1/2,
// L L^T = D G D + shift I
int ctm_selftest_cholqr(int k, const double* G, double shift, double* T)
{
    double *dG = dev_copy(G, (size_t)k * k), *dT = dev_copy<double>(nullptr, (size_t)k * k);
    double* dw = dev_copy<double>(nullptr, (size_t)2 * k);
    if (!dG || !dT || !dw) return 1;
    ctmk::CholBatch cb{};
    cb.n = 1;
    cb.job[0] = ctmk::CholJob{dG, dw, dT, k};
    ctmk::cholqr(nullptr, cb, shift);
    int rc = hipDeviceSynchronize() != hipSuccess;
    rc |= hipMemcpy(T, dT, (size_t)k * k * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess;
    (void)hipFree(dG);
    (void)hipFree(dT);
    (void)hipFree(dw);
    return rc;
}

// X (m x n column-major) = U S V^T; *sweeps (may be NULL) receives the sweeps done
int ctm_selftest_jacobi(int m, int n, const double* X, double* U, double* S, double* V, int* sweeps)
{
    int* dsw = dev_copy<int>(nullptr, 1);
    if (!dsw) return 1;
    double *dX = dev_copy(X, (size_t)m * n), *dW = dev_copy<double>(nullptr, (size_t)n * n);
    double *dU = dev_copy<double>(nullptr, (size_t)m * n), *dV = dev_copy<double>(nullptr, (size_t)n * n);
    double* dS = dev_copy<double>(nullptr, n);
    if (!dX || !dW || !dU || !dV || !dS) return 1;
    ctmk::JacobiBatch jb{};
    jb.n = 1;
    jb.job[0] = ctmk::JacobiJob{dX, dW, dU, dV, dS, m, n, 1, dsw};
    ctmk::jacobi_svd(nullptr, jb, 40);
    int rc = hipDeviceSynchronize() != hipSuccess;
    int sw = 0;
    rc |= hipMemcpy(&sw, dsw, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess;
    if (sweeps) *sweeps = sw;
    (void)hipFree(dsw);
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

// Timing of the factorisation kernels alone (device buffers, the same launch
// shapes as in a move): which = 0, the register Cholesky-QR factor of nprob
// k x k Gram matrices (k <= 128); which = 1 and 2, the register one-sided
// Jacobi of nprob k x k matrices with and without V, stopped after exactly
// `sweeps` sweeps (random input does not converge earlier).  *us receives the
// average time per launch over `reps` launches after a few untimed ones.
int ctm_selftest_time_factor(int which, int k, int nprob, int sweeps, int reps, double* us)
{
    if (k < 1 || k > 128 || nprob < 1 || nprob > ctmk::kMaxJacobiBatch || reps < 1 || !us) return 2;
    std::vector<double> h((size_t)k * k);
    uint64_t z = 0x9e3779b97f4a7c15ull;
    auto uni = [&]() {   // splitmix64 -> [-1, 1)
        z += 0x9e3779b97f4a7c15ull;
        uint64_t x = z;
        x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
        x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
        x ^= x >> 31;
        return (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    };
    if (which == 0) {
        // Gram matrix of k graded random rows of length 4k
        std::vector<double> y((size_t)k * 4 * k);
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < 4 * k; ++j) y[(size_t)i * 4 * k + j] = uni() * std::pow(10.0, -6.0 * i / k);
        for (int i = 0; i < k; ++i)
            for (int j = 0; j <= i; ++j) {
                double v = 0.0;
                for (int t = 0; t < 4 * k; ++t) v += y[(size_t)i * 4 * k + t] * y[(size_t)j * 4 * k + t];
                h[(size_t)i * k + j] = h[(size_t)j * k + i] = v;
            }
    } else {
        for (double& v : h) v = uni();
    }
    std::vector<double*> bufs;
    auto dev = [&](size_t n) {
        double* d = dev_copy<double>(nullptr, n);
        bufs.push_back(d);
        return d;
    };
    int rc = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return 1;
    }
    const size_t kk = (size_t)k * k;
    if (which == 0) {
        ctmk::CholBatch cb{};
        cb.n = nprob;
        for (int j = 0; j < nprob; ++j) {
            double *G = dev(kk), *w = dev(2 * (size_t)k), *T = dev(kk);
            if (!G || !w || !T || hipMemcpy(G, h.data(), kk * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) rc = 1;
            cb.job[j] = ctmk::CholJob{G, w, T, k};
        }
        if (!rc) {
            for (int r = 0; r < 3; ++r) ctmk::cholqr(nullptr, cb, 1e-14);
            rc |= hipDeviceSynchronize() != hipSuccess;
            rc |= hipEventRecord(e0, nullptr) != hipSuccess;
            for (int r = 0; r < reps; ++r) ctmk::cholqr(nullptr, cb, 1e-14);
            rc |= hipEventRecord(e1, nullptr) != hipSuccess;
        }
    } else {
        ctmk::JacobiBatch jb{};
        jb.n = nprob;
        for (int j = 0; j < nprob; ++j) {
            double *X = dev(kk), *W = dev(kk), *U = dev(kk), *V = dev(kk), *S = dev((size_t)k);
            if (!X || !W || !U || !V || !S || hipMemcpy(X, h.data(), kk * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
                rc = 1;
            jb.job[j] = ctmk::JacobiJob{X, W, U, V, S, k, k, which == 1 ? 1 : 0, nullptr};
        }
        if (!rc && !ctmk::jacobi_reads_only(jb)) rc = 2;   // the register kernel reads X only
        if (!rc) {
            ctmk::jacobi_svd(nullptr, jb, sweeps);
            rc |= hipDeviceSynchronize() != hipSuccess;
            rc |= hipEventRecord(e0, nullptr) != hipSuccess;
            for (int r = 0; r < reps; ++r) ctmk::jacobi_svd(nullptr, jb, sweeps);
            rc |= hipEventRecord(e1, nullptr) != hipSuccess;
        }
    }
    float ms = 0.0f;
    if (!rc) {
        rc |= hipEventSynchronize(e1) != hipSuccess;
        rc |= hipEventElapsedTime(&ms, e0, e1) != hipSuccess;
        *us = 1000.0 * ms / reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (double* d : bufs) (void)hipFree(d);
    return rc;
}

// Time per launch of the FP64 GEMM C = A B (row-major, M x K times K x N,
// zero operands) with the split-K plan of the library (split = 1: a 32 MiB
// workspace as in a move) or without split-K (split = 0).
int ctm_selftest_time_gemm(int M, int N, int K, int split, int reps, double* us)
{
    if (M < 1 || N < 1 || K < 1 || reps < 1 || !us) return 2;
    const int64_t ws_cap = (int64_t)1 << 22;
    double *A = dev_copy<double>(nullptr, (size_t)M * K), *B = dev_copy<double>(nullptr, (size_t)K * N);
    double *C = dev_copy<double>(nullptr, (size_t)M * N), *W = split ? dev_copy<double>(nullptr, (size_t)ws_cap) : nullptr;
    int rc = (!A || !B || !C || (split && !W)) ? 1 : 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!rc) {
        rc |= hipMemset(A, 0, (size_t)M * K * sizeof(double)) != hipSuccess;
        rc |= hipMemset(B, 0, (size_t)K * N * sizeof(double)) != hipSuccess;
        rc |= hipEventCreate(&e0) != hipSuccess;
        rc |= hipEventCreate(&e1) != hipSuccess;
    }
    if (!rc) {
        auto run = [&]() {
            ctmk::gemm_f64(nullptr, false, false, M, N, K, 1.0, A, K, 0, B, N, 0, 0.0, C, N, 0, 1, W,
                           split ? ws_cap : 0, nullptr);
        };
        for (int r = 0; r < 3; ++r) run();
        rc |= hipDeviceSynchronize() != hipSuccess;
        rc |= hipEventRecord(e0, nullptr) != hipSuccess;
        for (int r = 0; r < reps; ++r) run();
        rc |= hipEventRecord(e1, nullptr) != hipSuccess;
        float ms = 0.0f;
        rc |= hipEventSynchronize(e1) != hipSuccess;
        rc |= hipEventElapsedTime(&ms, e0, e1) != hipSuccess;
        if (!rc) *us = 1000.0 * ms / reps;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(A);
    (void)hipFree(B);
    (void)hipFree(C);
    if (W) (void)hipFree(W);
    return rc;
}

}  // extern "C"
