// Device kernels of the split-CTMRG library (gfx950 / CDNA4).
//
//   gemm_f64      batched C = alpha op(A) op(B) + beta C on the FP64 matrix cores
//                 (v_mfma_f64_16x16x4_f64): 64x64 block tile, four 64-wide
//                 waves of 32x32, K staged through LDS 16 at a time.
//   permute       dense tensor transposition (generic rank <= 8).
//   dot / norms   deterministic two-pass reductions to device scalars.
//   jacobi_svd    one-sided (Hestenes) Jacobi SVD, one workgroup per matrix,
//                 round-robin pair ordering, columns sorted by singular value.
//   small kernels fill / scale / symmetrise / identity / counter-based normals /
//                 D4 projection of the PEPS tensor / Ising PEPO / scalar algebra.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace ctmk {

typedef double dbl4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// GEMM (FP64 MFMA)
// ---------------------------------------------------------------------------
// A(m,k) = TA ? A[k*lda + m] : A[m*lda + k];  B(k,n) = TB ? B[n*ldb + k] : B[k*ldb + n]
// C(m,n) = C[m*ldc + n].  blockIdx.z selects the batch entry.
// MFMA 16x16x4 f64 operand layout (lane l of a 64-wide wave):
//   a = A[row = l%16][k = l/16],  b = B[k = l/16][col = l%16],
//   acc[r] = C[row = l/16 + 4*r][col = l%16].
constexpr int GT = 64;   // block tile (M and N)
constexpr int GK = 16;   // K step held in LDS

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm_f64_kernel(
    int M, int N, int K, double alpha,
    const double* __restrict__ A, int64_t lda, int64_t sA,
    const double* __restrict__ B, int64_t ldb, int64_t sB,
    double beta, double* __restrict__ C, int64_t ldc, int64_t sC)
{
    __shared__ double As[GK][GT + 1];
    __shared__ double Bs[GK][GT + 1];
    const int bz = blockIdx.z;
    A += bz * sA;
    B += bz * sB;
    C += bz * sC;
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    dbl4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};

    for (int k0 = 0; k0 < K; k0 += GK) {
#pragma unroll
        for (int t = 0; t < (GT * GK) / 256; ++t) {
            const int e = tid + t * 256;
            int mm, kk;
            if (!TA) { kk = e % GK; mm = e / GK; } else { mm = e % GT; kk = e / GT; }
            const int gm = m0 + mm, gk = k0 + kk;
            double v = 0.0;
            if (gm < M && gk < K) v = TA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk];
            As[kk][mm] = v;
        }
#pragma unroll
        for (int t = 0; t < (GT * GK) / 256; ++t) {
            const int e = tid + t * 256;
            int nn, kk;
            if (!TB) { nn = e % GT; kk = e / GT; } else { kk = e % GK; nn = e / GK; }
            const int gn = n0 + nn, gk = k0 + kk;
            double v = 0.0;
            if (gn < N && gk < K) v = TB ? B[(int64_t)gn * ldb + gk] : B[(int64_t)gk * ldb + gn];
            Bs[kk][nn] = v;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GK; kk += 4) {
            const int kq = kk + (lane >> 4);
            double a0 = As[kq][wm * 32 + (lane & 15)];
            double a1 = As[kq][wm * 32 + 16 + (lane & 15)];
            double b0 = Bs[kq][wn * 32 + (lane & 15)];
            double b1 = Bs[kq][wn * 32 + 16 + (lane & 15)];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wm * 32 + i * 16 + (lane >> 4) + 4 * r;
                const int gn = n0 + wn * 32 + j * 16 + (lane & 15);
                if (gm < M && gn < N) {
                    double* c = C + (int64_t)gm * ldc + gn;
                    const double v = alpha * acc[i][j][r];
                    *c = (beta == 0.0) ? v : v + beta * (*c);
                }
            }
}

void gemm_f64(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha,
              const double* A, int64_t lda, int64_t sA, const double* B, int64_t ldb, int64_t sB,
              double beta, double* C, int64_t ldc, int64_t sC, int batch)
{
    if (M <= 0 || N <= 0 || batch <= 0) return;
    dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT, batch);
    dim3 block(256);
    if (!ta && !tb)
        hipLaunchKernelGGL((gemm_f64_kernel<false, false>), grid, block, 0, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC);
    else if (ta && !tb)
        hipLaunchKernelGGL((gemm_f64_kernel<true, false>), grid, block, 0, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC);
    else if (!ta && tb)
        hipLaunchKernelGGL((gemm_f64_kernel<false, true>), grid, block, 0, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC);
    else
        hipLaunchKernelGGL((gemm_f64_kernel<true, true>), grid, block, 0, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC);
}

// ---------------------------------------------------------------------------
// permute: out (dims od[0..r-1], row-major) gathers in[sum_k c_k * is[k]]
// ---------------------------------------------------------------------------
__global__ void permute_kernel(const double* __restrict__ in, double* __restrict__ out, int64_t n,
                               PermDesc pd)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t rem = i, off = 0;
        for (int k = pd.rank - 1; k >= 0; --k) {
            const int64_t c = rem % pd.od[k];
            rem /= pd.od[k];
            off += c * pd.is[k];
        }
        out[i] = in[off];
    }
}

static int grid_for(int64_t n, int block = 256, int cap = 8192)
{
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

void permute(hipStream_t s, const double* in, double* out, const PermDesc& pd, int64_t n)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(permute_kernel, dim3(grid_for(n)), dim3(256), 0, s, in, out, n, pd);
}

// ---------------------------------------------------------------------------
// reductions (deterministic: fixed grid, fixed tree)
// ---------------------------------------------------------------------------
constexpr int RED_BLOCKS = 256;

__device__ inline double block_sum(double v, double* sh)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x < (blockDim.x >> 6)) t = sh[threadIdx.x];
    if (w == 0) {
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    }
    __syncthreads();
    return t;  // valid in thread 0
}

__global__ void dot_partial_kernel(const double* __restrict__ x, const double* __restrict__ y,
                                   int64_t n, double* __restrict__ part)
{
    __shared__ double sh[16];
    double v = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        v += x[i] * y[i];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// mode 0: out = sum, 1: out = sqrt(sum)
__global__ void reduce_final_kernel(const double* __restrict__ part, int n, double* out, int mode)
{
    __shared__ double sh[16];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v += part[i];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) *out = (mode == 1) ? sqrt(v) : v;
}

void dot(hipStream_t s, const double* x, const double* y, int64_t n, double* out, double* part, int mode)
{
    hipLaunchKernelGGL(dot_partial_kernel, dim3(RED_BLOCKS), dim3(256), 0, s, x, y, n, part);
    hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(256), 0, s, part, RED_BLOCKS, out, mode);
}

// ---------------------------------------------------------------------------
// elementwise
// ---------------------------------------------------------------------------
__global__ void scale_inv_kernel(double* x, int64_t n, const double* __restrict__ s)
{
    const double inv = 1.0 / *s;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] *= inv;
}

void scale_inv(hipStream_t s, double* x, int64_t n, const double* dev_scalar)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(scale_inv_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, n, dev_scalar);
}

__global__ void fill_kernel(double* x, int64_t n, double v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = v;
}

void fill(hipStream_t s, double* x, int64_t n, double v)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, n, v);
}

__global__ void copy_kernel(const double* __restrict__ a, double* __restrict__ b, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

void copy(hipStream_t s, const double* a, double* b, int64_t n)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n)), dim3(256), 0, s, a, b, n);
}

__global__ void eye_kernel(double* x, int n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)n * n;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = ((i / n) == (i % n)) ? 1.0 : 0.0;
}

void eye(hipStream_t s, double* x, int n)
{
    hipLaunchKernelGGL(eye_kernel, dim3(grid_for((int64_t)n * n)), dim3(256), 0, s, x, n);
}

// in-place (X + X^T)/2 of an n x n matrix
__global__ void symmetrize_kernel(double* x, int n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)n * n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(i / n), c = (int)(i % n);
        if (r < c) {
            const double v = 0.5 * (x[(int64_t)r * n + c] + x[(int64_t)c * n + r]);
            x[(int64_t)r * n + c] = v;
            x[(int64_t)c * n + r] = v;
        }
    }
}

void symmetrize(hipStream_t s, double* x, int n)
{
    hipLaunchKernelGGL(symmetrize_kernel, dim3(grid_for((int64_t)n * n)), dim3(256), 0, s, x, n);
}

// rows (mode 0) or columns (mode 1) of a row-major R x C matrix scaled by f[i]
__global__ void scale_lines_kernel(double* x, int R, int Cc, const double* __restrict__ f, int mode)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)R * Cc;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(i / Cc), c = (int)(i % Cc);
        x[i] *= f[mode == 0 ? r : c];
    }
}

void scale_lines(hipStream_t s, double* x, int R, int Cc, const double* f, int mode)
{
    hipLaunchKernelGGL(scale_lines_kernel, dim3(grid_for((int64_t)R * Cc)), dim3(256), 0, s, x, R, Cc, f, mode);
}

// f[i] = S[i] > cutoff * S[0] ? S[i]^(-1/2) : 0  (pseudo-inverse of S^(1/2))
__global__ void inv_sqrt_cut_kernel(const double* __restrict__ S, double* f, int n, double cutoff)
{
    const double s0 = S[0];
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double v = S[i];
        f[i] = (s0 > 0.0 && v > cutoff * s0) ? 1.0 / sqrt(v) : 0.0;
    }
}

void inv_sqrt_cut(hipStream_t s, const double* S, double* f, int n, double cutoff)
{
    hipLaunchKernelGGL(inv_sqrt_cut_kernel, dim3(1), dim3(256), 0, s, S, f, n, cutoff);
}

// d[i] = G[i][i]^-1/2 (0 for a zero diagonal)
__global__ void diag_inv_sqrt_kernel(const double* __restrict__ G, int n, double* d)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double v = G[(int64_t)i * n + i];
        d[i] = v > 0.0 ? 1.0 / sqrt(v) : 0.0;
    }
}

void diag_inv_sqrt(hipStream_t s, const double* G, int n, double* d)
{
    hipLaunchKernelGGL(diag_inv_sqrt_kernel, dim3(1), dim3(256), 0, s, G, n, d);
}

// out = #{i < n : S[i] > cutoff * S[0]}  (S descending)
__global__ void count_above_kernel(const double* __restrict__ S, int n, double cutoff, int* out)
{
    if (threadIdx.x == 0) {
        const double s0 = S[0];
        int c = 0;
        for (int i = 0; i < n; ++i) c += (s0 > 0.0 && S[i] > cutoff * s0);
        *out = c;
    }
}

void count_above(hipStream_t s, const double* S, int n, double cutoff, int* out)
{
    hipLaunchKernelGGL(count_above_kernel, dim3(1), dim3(1), 0, s, S, n, cutoff, out);
}

// counter-based standard normals (splitmix64 + Box-Muller)
__device__ inline uint64_t splitmix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void randn_kernel(double* x, int64_t n, uint64_t seed)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t a = splitmix64(seed * 0x632BE59BD9B4E019ull + 2 * (uint64_t)i);
        const uint64_t b = splitmix64(seed * 0x632BE59BD9B4E019ull + 2 * (uint64_t)i + 1);
        const double u1 = ((a >> 11) + 1.0) * (1.0 / 9007199254740993.0);
        const double u2 = (b >> 11) * (1.0 / 9007199254740992.0);
        x[i] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    }
}

void randn(hipStream_t s, double* x, int64_t n, uint64_t seed)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(randn_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, n, seed);
}

// ---------------------------------------------------------------------------
// model: D4 projection of A[p][l][u][r][d], Ising PEPO, identity PEPO
// ---------------------------------------------------------------------------
__global__ void d4_project_kernel(const double* __restrict__ A, double* __restrict__ out, int D)
{
    const int n = 2 * D * D * D * D;
    const int perms[8][4] = {{0, 1, 2, 3}, {1, 2, 3, 0}, {2, 3, 0, 1}, {3, 0, 1, 2},
                             {0, 3, 2, 1}, {2, 1, 0, 3}, {1, 0, 3, 2}, {3, 2, 1, 0}};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int idx[4];
        int rem = i;
        for (int k = 3; k >= 0; --k) { idx[k] = rem % D; rem /= D; }
        const int p = rem;
        double acc = 0.0;
        for (int g = 0; g < 8; ++g) {
            // out[p, x0..x3] += A[p, x_perm[0], ..]: the transpose of A by perm
            int src = p;
            int j[4];
            for (int k = 0; k < 4; ++k) j[perms[g][k]] = idx[k];
            for (int k = 0; k < 4; ++k) src = src * D + j[k];
            acc += A[src];
        }
        out[i] = acc * 0.125;
    }
}

void d4_project(hipStream_t s, const double* A, double* out, int D)
{
    const int n = 2 * D * D * D * D;
    hipLaunchKernelGGL(d4_project_kernel, dim3((n + 255) / 256), dim3(256), 0, s, A, out, D);
}

// O[p,q,l,u,r,d] = sum_s w[s,p] w[s,q] w[s,l] w[s,u] w[s,r] w[s,d], w = sqrt(W),
// W = [[e^b, e^-b], [e^-b, e^b]]: eigenvalues 2cosh b (vector (1,1)/sqrt2) and
// 2sinh b (vector (1,-1)/sqrt2), so w = (sqrt(2cosh b) P+ + sqrt(2sinh b) P-).
__global__ void ising_pepo_kernel(double* O, double beta)
{
    const int i = threadIdx.x;
    if (i >= 64) return;
    const double a = sqrt(2.0 * cosh(beta)), b = sqrt(2.0 * sinh(beta));
    const double w[2][2] = {{0.5 * (a + b), 0.5 * (a - b)}, {0.5 * (a - b), 0.5 * (a + b)}};
    int idx[6];
    int rem = i;
    for (int k = 5; k >= 0; --k) { idx[k] = rem & 1; rem >>= 1; }
    double acc = 0.0;
    for (int s = 0; s < 2; ++s) {
        double t = 1.0;
        for (int k = 0; k < 6; ++k) t *= w[s][idx[k]];
        acc += t;
    }
    O[i] = acc;
}

void ising_pepo(hipStream_t s, double* O, double beta)
{
    hipLaunchKernelGGL(ising_pepo_kernel, dim3(1), dim3(64), 0, s, O, beta);
}

__global__ void identity_pepo_kernel(double* O)
{
    const int i = threadIdx.x;
    if (i < 4) O[i] = ((i >> 1) == (i & 1)) ? 1.0 : 0.0;
}

void identity_pepo(hipStream_t s, double* O)
{
    hipLaunchKernelGGL(identity_pepo_kernel, dim3(1), dim3(4), 0, s, O);
}

// ---------------------------------------------------------------------------
// scalar algebra on device
// ---------------------------------------------------------------------------
// sc[0..3] = n1, n2h, n2v, n0 -> out[0] = ln kappa, out[1] = flag (1 if any <= 0 / nan)
__global__ void log_kappa_kernel(const double* sc, double* out)
{
    if (threadIdx.x == 0) {
        const double kap = sc[0] * sc[3] / (sc[1] * sc[2]);
        const bool bad = !(kap > 0.0) || !isfinite(kap);
        out[0] = bad ? 0.0 : log(kap);
        out[1] = bad ? 1.0 : 0.0;
    }
}

void log_kappa(hipStream_t s, const double* sc, double* out)
{
    hipLaunchKernelGGL(log_kappa_kernel, dim3(1), dim3(1), 0, s, sc, out);
}

// f = -(lk3 - lk2)/beta
__global__ void free_energy_kernel(const double* lk3, const double* lk2, double beta, double* f)
{
    if (threadIdx.x == 0) *f = -(lk3[0] - lk2[0]) / beta;
}

void free_energy(hipStream_t s, const double* lk3, const double* lk2, double beta, double* f)
{
    hipLaunchKernelGGL(free_energy_kernel, dim3(1), dim3(1), 0, s, lk3, lk2, beta, f);
}

// g = -(2/beta) (E3 / n13 - E2 / n12)
__global__ void grad_combine_kernel(const double* __restrict__ E3, const double* n13,
                                    const double* __restrict__ E2, const double* n12,
                                    double beta, double* __restrict__ g, int n)
{
    const double a = 1.0 / n13[0], b = 1.0 / n12[0];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        g[i] = -(2.0 / beta) * (E3[i] * a - E2[i] * b);
}

void grad_combine(hipStream_t s, const double* E3, const double* n13, const double* E2,
                  const double* n12, double beta, double* g, int n)
{
    hipLaunchKernelGGL(grad_combine_kernel, dim3((n + 255) / 256), dim3(256), 0, s, E3, n13, E2, n12, beta, g, n);
}

// spectrum post-processing: s[i] /= |trace|, then delta = ||s - s_old||_2 with
// zero padding; s_old <- s.  One block.
__global__ void spectrum_delta_kernel(double* s, int n, const double* trace, double* s_old,
                                      int* n_old, double* delta)
{
    __shared__ double sh[16];
    const double t = fabs(*trace);
    const double inv = (t > 0.0) ? 1.0 / t : 0.0;
    const int no = *n_old;
    const int nm = n > no ? n : no;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nm; i += blockDim.x) {
        const double a = (i < n) ? s[i] * inv : 0.0;
        const double b = (i < no) ? s_old[i] : 0.0;
        acc += (a - b) * (a - b);
    }
    acc = block_sum(acc, sh);
    __syncthreads();
    for (int i = threadIdx.x; i < nm; i += blockDim.x) {
        const double a = (i < n) ? s[i] * inv : 0.0;
        if (i < n) s[i] = a;
        s_old[i] = a;
    }
    if (threadIdx.x == 0) {
        *delta = sqrt(acc);
        *n_old = n;
    }
}

void spectrum_delta(hipStream_t s, double* sv, int n, const double* trace, double* s_old,
                    int* n_old, double* delta)
{
    hipLaunchKernelGGL(spectrum_delta_kernel, dim3(1), dim3(256), 0, s, sv, n, trace, s_old, n_old, delta);
}

__global__ void trace_kernel(const double* __restrict__ X, int n, double* out)
{
    __shared__ double sh[16];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v += X[(int64_t)i * n + i];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) *out = v;
}

void trace(hipStream_t s, const double* X, int n, double* out)
{
    hipLaunchKernelGGL(trace_kernel, dim3(1), dim3(256), 0, s, X, n, out);
}

// NaN / Inf scan: flag[0] = 1 if any non-finite entry
__global__ void finite_check_kernel(const double* __restrict__ x, int64_t n, int* flag)
{
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        bad |= !isfinite(x[i]);
    if (bad) atomicOr(flag, 1);
}

void finite_check(hipStream_t s, const double* x, int64_t n, int* flag)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(finite_check_kernel, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, x, n, flag);
}

// ---------------------------------------------------------------------------
// one-sided Jacobi SVD, one workgroup per problem
// ---------------------------------------------------------------------------
// Input  X: m x n, column-major (column j at X + j*m), destroyed.
// Output U: m x n column-major (unit columns, 0 where sigma = 0), V: n x n
//        column-major, S: n, sorted descending (ties by column index):
//        X = U diag(S) V^T.
// Work:  W (n x n) holds V during the sweeps.  When m * n doubles fit in LDS
//        the columns of X are rotated there.
// A pair (p, q) is rotated while |x_p . x_q| > tol * |x_p| |x_q| with
// tol = 2 sqrt(m) eps (the rounding level of the dot product itself).
constexpr int kJacobiLdsDoubles = 18432;   // 144 KiB of the 160 KiB LDS

__global__ __launch_bounds__(1024) void jacobi_svd_kernel(JacobiBatch jobs, int max_sweeps)
{
    extern __shared__ double lds[];
    const JacobiJob jb = jobs.job[blockIdx.x];
    const int m = jb.m, n = jb.n;
    const bool acc_v = jb.want_v != 0;
    const bool x_lds = (int64_t)m * n <= kJacobiLdsDoubles;
    const bool w_lds = acc_v && (int64_t)m * n + (int64_t)n * n <= kJacobiLdsDoubles;
    double* X = x_lds ? lds : jb.X;
    double* W = w_lds ? lds + (int64_t)m * n : jb.W;
    const int ne = n + (n & 1);
    const int npairs = ne / 2;
    const int nthr = blockDim.x;
    int G = 64;
    while (G > 1 && G * npairs > nthr) G >>= 1;
    const int ngroups = nthr / G;
    const int gid = threadIdx.x / G, gl = threadIdx.x % G;
    __shared__ int rotated;
    __shared__ double sig[1024];
    __shared__ int rnk[1024];

    __shared__ double fro2;
    if (x_lds)
        for (int64_t i = threadIdx.x; i < (int64_t)m * n; i += nthr) X[i] = jb.X[i];
    if (acc_v)
        for (int64_t i = threadIdx.x; i < (int64_t)n * n; i += nthr)
            W[i] = ((i / n) == (i % n)) ? 1.0 : 0.0;
    __syncthreads();
    // ||X||_F^2 (invariant under the rotations): columns below ~eps ||X||_F are
    // rounding noise and are left alone (they would never test orthogonal)
    for (int j = gid; j < n; j += ngroups) {
        const double* xj = X + (int64_t)j * m;
        double v = 0.0;
        for (int r = gl; r < m; r += G) v += xj[r] * xj[r];
        for (int o = G >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
        if (gl == 0) sig[j] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int j = 0; j < n; ++j) t += sig[j];
        fro2 = t;
    }
    __syncthreads();
    const double noise2 = 1e-30 * fro2;

    const double tol = 2.0 * sqrt((double)m) * 2.220446049250313e-16;
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        if (threadIdx.x == 0) rotated = 0;
        __syncthreads();
        for (int step = 0; step < ne - 1; ++step) {
            for (int pi = gid; pi < npairs; pi += ngroups) {
                int p, q;
                if (pi == 0) { p = ne - 1; q = step; }
                else { p = (step + pi) % (ne - 1); q = (step - pi + (ne - 1)) % (ne - 1); }
                if (p >= n || q >= n) continue;       // virtual zero column
                if (p > q) { int t = p; p = q; q = t; }
                double* xp = X + (int64_t)p * m;
                double* xq = X + (int64_t)q * m;
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int r = gl; r < m; r += G) {
                    const double a = xp[r], b = xq[r];
                    al += a * a;
                    be += b * b;
                    ga += a * b;
                }
                for (int o = G >> 1; o > 0; o >>= 1) {
                    al += __shfl_xor(al, o, G);
                    be += __shfl_xor(be, o, G);
                    ga += __shfl_xor(ga, o, G);
                }
                if (ga != 0.0 && al > noise2 && be > noise2 && fabs(ga) > tol * sqrt(al * be)) {
                    const double zeta = (be - al) / (2.0 * ga);
                    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
                    for (int r = gl; r < m; r += G) {
                        const double a = xp[r], b = xq[r];
                        xp[r] = c * a - sn * b;
                        xq[r] = sn * a + c * b;
                    }
                    if (acc_v) {
                        double* wp = W + (int64_t)p * n;
                        double* wq = W + (int64_t)q * n;
                        for (int r = gl; r < n; r += G) {
                            const double a = wp[r], b = wq[r];
                            wp[r] = c * a - sn * b;
                            wq[r] = sn * a + c * b;
                        }
                    }
                    if (gl == 0) rotated = 1;
                }
            }
            __syncthreads();
        }
        if (rotated == 0) break;
        __syncthreads();
    }
    // singular values = column norms
    for (int j = gid; j < n; j += ngroups) {
        const double* xj = X + (int64_t)j * m;
        double v = 0.0;
        for (int r = gl; r < m; r += G) v += xj[r] * xj[r];
        for (int o = G >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
        if (gl == 0) sig[j] = sqrt(v);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += nthr) {
        int r = 0;
        const double sj = sig[j];
        for (int i = 0; i < n; ++i) {
            const double si = sig[i];
            r += (si > sj) || (si == sj && i < j);
        }
        rnk[j] = r;
    }
    __syncthreads();
    for (int j = gid; j < n; j += ngroups) {
        const int dst = rnk[j];
        const double sj = sig[j];
        const double inv = sj > 0.0 ? 1.0 / sj : 0.0;
        const double* xj = X + (int64_t)j * m;
        double* uo = jb.U + (int64_t)dst * m;
        for (int r = gl; r < m; r += G) uo[r] = xj[r] * inv;
        if (acc_v) {
            const double* wj = W + (int64_t)j * n;
            double* vo = jb.V + (int64_t)dst * n;
            for (int r = gl; r < n; r += G) vo[r] = wj[r];
        }
        if (gl == 0) jb.S[dst] = sj;
    }
}

void jacobi_svd(hipStream_t s, const JacobiBatch& jobs, int max_sweeps)
{
    if (jobs.n <= 0) return;
    int64_t need = 0;
    for (int i = 0; i < jobs.n; ++i) {
        const int64_t mn = (int64_t)jobs.job[i].m * jobs.job[i].n;
        const int64_t nn = jobs.job[i].want_v ? (int64_t)jobs.job[i].n * jobs.job[i].n : 0;
        int64_t use = 0;
        if (mn + nn <= kJacobiLdsDoubles) use = mn + nn;
        else if (mn <= kJacobiLdsDoubles) use = mn;
        if (use > need) need = use;
    }
    hipLaunchKernelGGL(jacobi_svd_kernel, dim3(jobs.n), dim3(1024), need * sizeof(double), s, jobs, max_sweeps);
}

// ---------------------------------------------------------------------------
// shifted Cholesky QR factor, one workgroup per problem
// ---------------------------------------------------------------------------
// Input  G: k x k Gram matrix Y Y^T of the k rows of Y (row-major, global).
// Output T: k x k lower-triangular, T = L^-1 D with D = diag(G)^-1/2 and
//        L L^T = D G D + shift I, so that the rows of T Y are orthonormal
//        (up to the shift).  G lives in LDS when k*k (+k) doubles fit.
__global__ __launch_bounds__(1024) void cholqr_kernel(CholBatch jobs, double shift)
{
    extern __shared__ double lds[];
    const CholJob jb = jobs.job[blockIdx.x];
    const int k = jb.k;
    const bool in_lds = (int64_t)k * k + 2 * k <= kJacobiLdsDoubles;
    double* A = in_lds ? lds : jb.G;                 // working copy (lower = L)
    double* dsc = in_lds ? lds + (int64_t)k * k : jb.work;
    double* dinv = dsc + k;
    const int nthr = blockDim.x, tid = threadIdx.x;
    for (int i = tid; i < k; i += nthr) {
        const double v = jb.G[(int64_t)i * k + i];
        dsc[i] = v > 0.0 ? 1.0 / sqrt(v) : 0.0;
    }
    __syncthreads();
    // A = D G D + shift I (lower triangle incl. diagonal)
    for (int64_t e = tid; e < (int64_t)k * k; e += nthr) {
        const int i = (int)(e / k), l = (int)(e % k);
        if (l <= i) A[e] = jb.G[e] * dsc[i] * dsc[l] + (i == l ? shift : 0.0);
    }
    __syncthreads();
    // right-looking Cholesky, one barrier per column: step j updates the
    // trailing lower triangle with the unscaled column j and scales column j-1
    for (int j = 0; j < k; ++j) {
        const double ajj = A[(int64_t)j * k + j];
        const double inv = ajj > 0.0 ? 1.0 / ajj : 0.0;   // 1 / L_jj^2
        const int nt = k - 1 - j;
        const int64_t ntri = (int64_t)nt * (nt + 1) / 2;
        for (int64_t e = tid; e < ntri; e += nthr) {
            // e -> (i, l) with j < l <= i < k
            const int ii = (int)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
            int i0 = ii, l0 = (int)(e - (int64_t)ii * (ii + 1) / 2);
            if (l0 > i0) { ++i0; l0 = (int)(e - (int64_t)i0 * (i0 + 1) / 2); }
            if (l0 < 0) { --i0; l0 = (int)(e - (int64_t)i0 * (i0 + 1) / 2); }
            const int i = j + 1 + i0, l = j + 1 + l0;
            A[(int64_t)i * k + l] -= A[(int64_t)i * k + j] * A[(int64_t)l * k + j] * inv;
        }
        if (j > 0) {
            const int jm = j - 1;
            const double lj = sqrt(fmax(A[(int64_t)jm * k + jm], 0.0));
            const double li = lj > 0.0 ? 1.0 / lj : 0.0;
            for (int i = jm + 1 + tid; i < k; i += nthr) A[(int64_t)i * k + jm] *= li;
        }
        __syncthreads();
        if (tid == 0 && j > 0) A[(int64_t)(j - 1) * k + (j - 1)] = sqrt(fmax(A[(int64_t)(j - 1) * k + (j - 1)], 0.0));
        __syncthreads();
    }
    {
        const int jm = k - 1;
        if (tid == 0) A[(int64_t)jm * k + jm] = sqrt(fmax(A[(int64_t)jm * k + jm], 0.0));
        __syncthreads();
    }
    // L^-1 by columns: thread c solves L x = e_c, x_i stored at A[c][i] (i > c)
    for (int c = tid; c < k; c += nthr) {
        const double lcc = A[(int64_t)c * k + c];
        const double xc = lcc > 0.0 ? 1.0 / lcc : 0.0;
        dinv[c] = xc;
        for (int i = c + 1; i < k; ++i) {
            double sacc = A[(int64_t)i * k + c] * xc;
            for (int jj = c + 1; jj < i; ++jj) sacc += A[(int64_t)i * k + jj] * A[(int64_t)c * k + jj];
            const double lii = A[(int64_t)i * k + i];
            A[(int64_t)c * k + i] = lii > 0.0 ? -sacc / lii : 0.0;
        }
    }
    __syncthreads();
    // T[i][c] = (L^-1)[i][c] d_c
    for (int64_t e = tid; e < (int64_t)k * k; e += nthr) {
        const int i = (int)(e / k), c = (int)(e % k);
        double v = 0.0;
        if (i == c) v = dinv[c];
        else if (i > c) v = A[(int64_t)c * k + i];
        jb.T[e] = v * dsc[c];
    }
}

void cholqr(hipStream_t s, const CholBatch& jobs, double shift)
{
    if (jobs.n <= 0) return;
    int64_t need = 0;
    for (int i = 0; i < jobs.n; ++i) {
        const int64_t kk = jobs.job[i].k;
        if (kk * kk + 2 * kk <= kJacobiLdsDoubles && kk * kk + 2 * kk > need) need = kk * kk + 2 * kk;
    }
    hipLaunchKernelGGL(cholqr_kernel, dim3(jobs.n), dim3(1024), need * sizeof(double), s, jobs, shift);
}

}  // namespace ctmk

