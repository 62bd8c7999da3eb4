// Device kernels of the split-CTMRG library (gfx950 / CDNA4).
//
//   gemm_f64      batched C = alpha op(A) op(B) + beta C on the FP64 matrix cores
//                 (v_mfma_f64_16x16x4_f64): 64x64 block tile, four 64-wide
//                 waves of 32x32, K staged through LDS 32 at a time, split-K
//                 with a deterministic reduction when the tile grid is small.
//   permute       dense tensor transposition (generic rank <= 8).
//   dot / norms   deterministic two-pass reductions to device scalars.
//   jacobi_svd    one-sided (Hestenes) Jacobi SVD, one workgroup per matrix,
//                 round-robin pair ordering, columns sorted by singular value.
//   small kernels fill / scale / symmetrise / identity / counter-based normals /
//                 D4 projection of the PEPS tensor / Ising PEPO / scalar algebra.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "kernels.h"
#include "perm_plan.h"

namespace ctmk {

typedef double dbl4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// GEMM (FP64 MFMA)
// ---------------------------------------------------------------------------
// A(m,k) = TA ? A[k*lda + m] : A[m*lda + k];  B(k,n) = TB ? B[n*ldb + k] : B[k*ldb + n]
// C(m,n) = C[m*ldc + n].  blockIdx.z = batch entry * ksplit + K slice.
// MFMA 16x16x4 f64 operand layout (lane l of a 64-wide wave):
//   a = A[row = l%16][k = l/16],  b = B[k = l/16][col = l%16],
//   acc[r] = C[row = l/16 + 4*r][col = l%16].
// The next K step is fetched into registers while the matrix cores work on
// the current one (one LDS stage, register double buffer).  With ksplit > 1
// each K slice writes alpha * (its partial product) to P[z][M][N] and
// gemm_reduce_kernel sums the slices into C (beta must be 0 then).
constexpr int GT = 64;   // block tile (M and N)
constexpr int GK = 32;   // K step held in LDS
constexpr int GL = (GT * GK) / 256;   // elements of each operand a thread stages per step

// One 64x64 tile of out = alpha op(A) op(B) (+ beta out when accumulate),
// over the K range [kbeg, kend).
template <bool TA, bool TB>
__device__ __forceinline__ void gemm_tile(int M, int N, int kbeg, int kend, double alpha,
                                          const double* __restrict__ A, int64_t lda,
                                          const double* __restrict__ B, int64_t ldb, double beta,
                                          bool accumulate, double* __restrict__ out, int64_t ldo, int m0, int n0,
                                          double (&As)[GK][GT + 1], double (&Bs)[GK][GT + 1])
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    dbl4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};

    double ra[GL], rb[GL];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int t = 0; t < GL; ++t) {
            const int e = tid + t * 256;
            int mm, kk;
            if (!TA) { kk = e % GK; mm = e / GK; } else { mm = e % GT; kk = e / GT; }
            const int gm = m0 + mm, gk = k0 + kk;
            ra[t] = (gm < M && gk < kend) ? (TA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk]) : 0.0;
        }
#pragma unroll
        for (int t = 0; t < GL; ++t) {
            const int e = tid + t * 256;
            int nn, kk;
            if (!TB) { nn = e % GT; kk = e / GT; } else { kk = e % GK; nn = e / GK; }
            const int gn = n0 + nn, gk = k0 + kk;
            rb[t] = (gn < N && gk < kend) ? (TB ? B[(int64_t)gn * ldb + gk] : B[(int64_t)gk * ldb + gn]) : 0.0;
        }
    };
    auto stage = [&]() {
#pragma unroll
        for (int t = 0; t < GL; ++t) {
            const int e = tid + t * 256;
            int mm, kk;
            if (!TA) { kk = e % GK; mm = e / GK; } else { mm = e % GT; kk = e / GT; }
            As[kk][mm] = ra[t];
        }
#pragma unroll
        for (int t = 0; t < GL; ++t) {
            const int e = tid + t * 256;
            int nn, kk;
            if (!TB) { nn = e % GT; kk = e / GT; } else { kk = e % GK; nn = e / GK; }
            Bs[kk][nn] = rb[t];
        }
    };

    if (kbeg < kend) fetch(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += GK) {
        stage();
        __syncthreads();
        if (k0 + GK < kend) fetch(k0 + GK);
#pragma unroll
        for (int kk = 0; kk < GK; kk += 4) {
            const int kq = kk + (lane >> 4);
            const double a0 = As[kq][wm * 32 + (lane & 15)];
            const double a1 = As[kq][wm * 32 + 16 + (lane & 15)];
            const double b0 = Bs[kq][wn * 32 + (lane & 15)];
            const double b1 = Bs[kq][wn * 32 + 16 + (lane & 15)];
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
                    double* c = out + (int64_t)gm * ldo + gn;
                    const double v = alpha * acc[i][j][r];
                    *c = accumulate ? v + beta * (*c) : v;
                }
            }
}

// Workgroups go to the 8 XCDs round-robin (linear id mod 8), and each XCD
// has its own L2.  xcd_remap(b, n) gives XCD k the contiguous range of tile
// ids [k q + min(k, r), (k + 1) q + min(k + 1, r)) in order (q = n / 8,
// r = n % 8): neighbouring tiles, which share an operand panel, run on one
// XCD and read it from that XCD's L2.  It is a bijection of [0, n).
__device__ inline int xcd_remap(int b, int n)
{
    const int q = n >> 3, r = n & 7, k = b & 7, j = b >> 3;
    return k * q + min(k, r) + j;
}

template <bool TA, bool TB>
__global__ __launch_bounds__(256, 4) void gemm_f64_kernel(
    int M, int N, int K, double alpha,
    const double* __restrict__ A, int64_t lda, int64_t sA,
    const double* __restrict__ B, int64_t ldb, int64_t sB,
    double beta, double* __restrict__ C, int64_t ldc, int64_t sC,
    int ksplit, int kchunk, double* __restrict__ P)
{
    __shared__ double As[GK][GT + 1];
    __shared__ double Bs[GK][GT + 1];
    const int gx = gridDim.x, gy = gridDim.y;
    const int t = xcd_remap(blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z), gx * gy * gridDim.z);
    const int tx = t % gx, ty = (t / gx) % gy, z = t / (gx * gy);
    const int bz = z / ksplit, sp = z % ksplit;
    const int kbeg = sp * kchunk;
    const int kend = min(K, kbeg + kchunk);
    double* out;
    int64_t ldo;
    if (ksplit > 1) { out = P + (int64_t)z * M * N; ldo = N; }
    else { out = C + bz * sC; ldo = ldc; }
    gemm_tile<TA, TB>(M, N, kbeg, kend, alpha, A + bz * sA, lda, B + bz * sB, ldb, beta,
                      !(beta == 0.0 || ksplit > 1), out, ldo, ty * GT, tx * GT, As, Bs);
}

// Grouped form: problem i owns the blocks [start[i], start[i + 1]) of a 1-D
// grid, ks[i] K slices per output tile (slice-major within a tile).  Slices
// of split problems write to P + poff[i] + slice * M * N.
struct GemmGroupDev {
    GemmProb p[kMaxGemmGroup];
    int start[kMaxGemmGroup + 1];
    int tn[kMaxGemmGroup];       // tiles along N
    int ks[kMaxGemmGroup];       // K slices
    int kc[kMaxGemmGroup];       // K per slice
    int64_t poff[kMaxGemmGroup]; // partial-product offset (split problems)
    int n;
};

template <bool TA, bool TB>
__global__ __launch_bounds__(256, 4) void gemm_f64_group_kernel(GemmGroupDev g, double alpha, double* __restrict__ P)
{
    __shared__ double As[GK][GT + 1];
    __shared__ double Bs[GK][GT + 1];
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    int i = 0;
    while (i + 1 < g.n && b >= g.start[i + 1]) ++i;
    const GemmProb q = g.p[i];
    const int local = b - g.start[i], ks = g.ks[i];
    const int sp = local % ks, tile = local / ks;
    const int m0 = (tile / g.tn[i]) * GT, n0 = (tile % g.tn[i]) * GT;
    const int kbeg = sp * g.kc[i], kend = min(q.K, kbeg + g.kc[i]);
    double* out = ks > 1 ? P + g.poff[i] + (int64_t)sp * q.M * q.N : q.C;
    const int64_t ldo = ks > 1 ? q.N : q.ldc;
    gemm_tile<TA, TB>(q.M, q.N, kbeg, kend, alpha, q.A, q.lda, q.B, q.ldb, 0.0, false, out, ldo, m0, n0, As, Bs);
}

// C_i = sum of the ks[i] slices, for every split problem i (blockIdx.y)
__global__ void gemm_group_reduce_kernel(GemmGroupDev g, const double* __restrict__ P)
{
    const int i = blockIdx.y;
    if (i >= g.n || g.ks[i] <= 1) return;
    const GemmProb q = g.p[i];
    const int64_t mn = (int64_t)q.M * q.N;
    const double* p = P + g.poff[i];
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < mn; e += (int64_t)gridDim.x * blockDim.x) {
        double v = 0.0;
        for (int s = 0; s < g.ks[i]; ++s) v += p[s * mn + e];
        q.C[(e / q.N) * q.ldc + (e % q.N)] = v;
    }
}

// C[b][m][n] = sum over the ksplit slices of P[b * ksplit + s][m][n]
__global__ void gemm_reduce_kernel(const double* __restrict__ P, int M, int N, int ksplit,
                                   double* __restrict__ C, int64_t ldc, int64_t sC, int64_t total)
{
    const int64_t mn = (int64_t)M * N;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = i / mn, e = i % mn;
        const double* p = P + b * ksplit * mn + e;
        double v = 0.0;
        for (int s = 0; s < ksplit; ++s) v += p[s * mn];
        C[b * sC + (e / N) * ldc + (e % N)] = v;
    }
}

int gemm_split_plan(int M, int N, int K, int batch, int64_t ws_cap)
{
    const int64_t tiles = (int64_t)((N + GT - 1) / GT) * ((M + GT - 1) / GT) * batch;
    int s = 1;
    if (tiles < 160 && K >= 4 * GK)
        s = (int)std::min<int64_t>((320 + tiles - 1) / tiles, K / (2 * GK));   // few tiles: ~320 blocks
    else if (tiles < 1024 && K >= 16 * GK)
        s = (int)std::min<int64_t>((1024 + tiles - 1) / tiles, K / (4 * GK));  // long K: ~4 blocks per CU
    if (s <= 1) return 1;
    while (s > 1 && (int64_t)s * M * N * batch > ws_cap) --s;
    return std::max(s, 1);
}

// Long, skinny products with a short contraction (A M x K and B K x N, both
// untransposed, N at most 8, K at most kSkinnyMax): the absorption of the
// PEPO into an environment tensor (M up to ~1e6, N = K = 2 ... 8).  The
// 64-wide MFMA tiles would be mostly padding here and the product is
// HBM-bound (8 (M K + M N) bytes for 2 M N K flops).  One thread per row (the
// kernel also takes wider N in groups of 8 columns, but from N = 25 on the
// MFMA tile kernel is faster: its output tiles are written coalesced); B is
// staged in LDS and read by broadcast.  M = 1.25e6, N = K = 8: 57 us against
// 236 us in the tile kernel.
constexpr int kSkinnyMax = 64;
constexpr int kSkinnyCols = 8;

__global__ __launch_bounds__(256) void gemm_skinny_kernel(int M, int N, int K, double alpha,
                                                          const double* __restrict__ A, int64_t lda,
                                                          const double* __restrict__ B, int64_t ldb, double beta,
                                                          double* __restrict__ C, int64_t ldc)
{
    __shared__ double Bs[kSkinnyMax * kSkinnyMax];
    for (int e = threadIdx.x; e < K * N; e += blockDim.x) Bs[e] = B[(int64_t)(e / N) * ldb + (e % N)];
    __syncthreads();
    const int nch = (N + kSkinnyCols - 1) / kSkinnyCols;
    const int rows = (int)blockDim.x / nch;
    const int r = (int)threadIdx.x / nch, ch = (int)threadIdx.x % nch;
    const int64_t m = (int64_t)blockIdx.x * rows + r;
    if (r >= rows || m >= M) return;
    const int n0 = ch * kSkinnyCols;
    double acc[kSkinnyCols];
#pragma unroll
    for (int j = 0; j < kSkinnyCols; ++j) acc[j] = 0.0;
    const double* a = A + m * lda;
    for (int k = 0; k < K; ++k) {
        const double av = a[k];
        const double* b = Bs + k * N + n0;
#pragma unroll
        for (int j = 0; j < kSkinnyCols; ++j)
            if (n0 + j < N) acc[j] += av * b[j];
    }
    double* c = C + m * ldc + n0;
#pragma unroll
    for (int j = 0; j < kSkinnyCols; ++j)
        if (n0 + j < N) c[j] = beta == 0.0 ? alpha * acc[j] : alpha * acc[j] + beta * c[j];
}

void gemm_f64(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha,
              const double* A, int64_t lda, int64_t sA, const double* B, int64_t ldb, int64_t sB,
              double beta, double* C, int64_t ldc, int64_t sC, int batch, double* ws, int64_t ws_cap,
              hipEvent_t mid)
{
    if (M <= 0 || N <= 0 || batch <= 0) return;
    if (!ta && !tb && batch == 1 && K >= 1 && N <= kSkinnyCols && K <= kSkinnyMax && (int64_t)M * N >= (1 << 16)) {
        const int rows = 256 / ((N + kSkinnyCols - 1) / kSkinnyCols);
        hipLaunchKernelGGL(gemm_skinny_kernel, dim3((unsigned)((M + rows - 1) / rows)), dim3(256), 0, s, M, N, K,
                           alpha, A, lda, B, ldb, beta, C, ldc);
        if (mid) (void)hipEventRecord(mid, s);
        return;
    }
    int ksplit = (beta == 0.0 && ws) ? gemm_split_plan(M, N, K, batch, ws_cap) : 1;
    int kchunk = K;
    if (ksplit > 1) {
        kchunk = (((K + ksplit - 1) / ksplit) + GK - 1) / GK * GK;
        ksplit = (K + kchunk - 1) / kchunk;
    }
    dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT, batch * ksplit);
    dim3 block(256);
    double* P = ksplit > 1 ? ws : nullptr;
    if (!ta && !tb)
        hipLaunchKernelGGL((gemm_f64_kernel<false, false>), grid, block, 0, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, ksplit, kchunk, P);
    else if (ta && !tb)
        hipLaunchKernelGGL((gemm_f64_kernel<true, false>), grid, block, 0, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, ksplit, kchunk, P);
    else if (!ta && tb)
        hipLaunchKernelGGL((gemm_f64_kernel<false, true>), grid, block, 0, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, ksplit, kchunk, P);
    else
        hipLaunchKernelGGL((gemm_f64_kernel<true, true>), grid, block, 0, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, ksplit, kchunk, P);
    if (mid) (void)hipEventRecord(mid, s);
    if (ksplit > 1) {
        const int64_t total = (int64_t)batch * M * N;
        const int g = (int)std::min<int64_t>((total + 255) / 256, 4096);
        hipLaunchKernelGGL(gemm_reduce_kernel, dim3(g), dim3(256), 0, s, P, M, N, ksplit, C, ldc, sC, total);
    }
}

// K slices of every problem of a group: none when the group's tiles fill the
// chip, else up to ~320 blocks in all, within the workspace
static void gemm_group_plan(const GemmProb* p, int n, int64_t ws_cap, GemmGroupDev& g)
{
    int64_t tiles = 0;
    for (int i = 0; i < n; ++i) tiles += (int64_t)((p[i].N + GT - 1) / GT) * ((p[i].M + GT - 1) / GT);
    const int want = tiles >= 160 ? 1 : (int)((320 + tiles - 1) / std::max<int64_t>(tiles, 1));
    for (int cap = want;; cap = std::max(1, cap / 2)) {
        int64_t need = 0;
        for (int i = 0; i < n; ++i) {
            int s = std::max(1, std::min(cap, p[i].K / (2 * GK)));
            if (p[i].K < 4 * GK) s = 1;
            int kc = p[i].K;
            if (s > 1) {
                kc = (((p[i].K + s - 1) / s) + GK - 1) / GK * GK;
                s = (p[i].K + kc - 1) / kc;
            }
            g.ks[i] = s;
            g.kc[i] = std::max(kc, 1);
            g.poff[i] = need;
            if (s > 1) need += (int64_t)s * p[i].M * p[i].N;
        }
        if (need <= ws_cap || cap == 1) {
            if (need > ws_cap)
                for (int i = 0; i < n; ++i) g.ks[i] = 1, g.kc[i] = std::max(p[i].K, 1);
            return;
        }
    }
}

int gemm_group_splits(const GemmProb* p, int n, int64_t ws_cap)
{
    GemmGroupDev g{};
    gemm_group_plan(p, n, ws_cap, g);
    int any = 0;
    for (int i = 0; i < n; ++i) any += g.ks[i] > 1;
    return any;
}

void gemm_f64_group(hipStream_t s, bool ta, bool tb, const GemmProb* p, int n, double alpha, double* ws,
                    int64_t ws_cap, hipEvent_t mid)
{
    GemmGroupDev g{};
    int nz = 0;
    for (int i = 0; i < n && i < kMaxGemmGroup; ++i)
        if (p[i].M > 0 && p[i].N > 0) g.p[nz++] = p[i];
    g.n = nz;
    if (nz == 0) {
        if (mid) (void)hipEventRecord(mid, s);
        return;
    }
    gemm_group_plan(g.p, nz, ws ? ws_cap : 0, g);
    int total = 0, split = 0;
    int64_t maxmn = 0;
    for (int i = 0; i < nz; ++i) {
        const int tm = (g.p[i].M + GT - 1) / GT;
        g.tn[i] = (g.p[i].N + GT - 1) / GT;
        g.start[i] = total;
        total += tm * g.tn[i] * g.ks[i];
        if (g.ks[i] > 1) {
            split = 1;
            maxmn = std::max<int64_t>(maxmn, (int64_t)g.p[i].M * g.p[i].N);
        }
    }
    g.start[nz] = total;
    if (!ta && !tb)
        hipLaunchKernelGGL((gemm_f64_group_kernel<false, false>), dim3(total), dim3(256), 0, s, g, alpha, ws);
    else if (ta && !tb)
        hipLaunchKernelGGL((gemm_f64_group_kernel<true, false>), dim3(total), dim3(256), 0, s, g, alpha, ws);
    else if (!ta && tb)
        hipLaunchKernelGGL((gemm_f64_group_kernel<false, true>), dim3(total), dim3(256), 0, s, g, alpha, ws);
    else
        hipLaunchKernelGGL((gemm_f64_group_kernel<true, true>), dim3(total), dim3(256), 0, s, g, alpha, ws);
    if (mid) (void)hipEventRecord(mid, s);
    if (split) {
        const int gx = (int)std::min<int64_t>((maxmn + 255) / 256, 1024);
        hipLaunchKernelGGL(gemm_group_reduce_kernel, dim3(gx, nz), dim3(256), 0, s, g, ws);
    }
}

// ---------------------------------------------------------------------------
// GEMM with FP32 or BF16 products and FP32 accumulation (reduced-precision
// forms of the bulk contractions).  Operands and result stay FP64 in memory:
// the operands are rounded (to nearest even) when staged into LDS, the
// matrix cores multiply in the reduced precision and accumulate in FP32, and
// alpha * acc is written back as FP64.  Tiles as in gemm_f64_kernel; the LDS
// tiles keep k contiguous ([row][k]) so that a lane's k-run is one load.
//   FP32: v_mfma_f32_16x16x4_f32   a = A[l%16][l/16], b = B[l/16][l%16]
//   BF16: v_mfma_f32_16x16x32_bf16 a = A[l%16][8(l/16) .. +7], b likewise
//   result: acc[r] = C[4(l/16) + r][l%16]
// ---------------------------------------------------------------------------
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int LK = 32;             // K step held in LDS
constexpr int LGL = (GT * LK) / 256;

__device__ inline unsigned short to_bf16_bits(double x)
{
    const float f = (float)x;
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even (finite inputs)
    return (unsigned short)(u >> 16);
}

template <bool TA, bool TB, int P>   // P = 1: FP32, P = 2: BF16
__global__ __launch_bounds__(256) void gemm_lp_kernel(
    int M, int N, int K, double alpha,
    const double* __restrict__ A, int64_t lda, int64_t sA,
    const double* __restrict__ B, int64_t ldb, int64_t sB,
    double beta, double* __restrict__ C, int64_t ldc, int64_t sC,
    int ksplit, int kchunk, double* __restrict__ Pp)
{
    typedef typename std::conditional<P == 1, float, unsigned short>::type elem;
    constexpr int PAD = (P == 1) ? 1 : 8;        // keeps 16-byte alignment of bf16 k-runs
    __shared__ __attribute__((aligned(16))) elem As[GT][LK + PAD];
    __shared__ __attribute__((aligned(16))) elem Bs[GT][LK + PAD];
    const int gx = gridDim.x, gy = gridDim.y;
    const int t = xcd_remap(blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z), gx * gy * gridDim.z);
    const int z = t / (gx * gy);
    const int bz = z / ksplit, sp = z % ksplit;
    A += bz * sA;
    B += bz * sB;
    const int kbeg = sp * kchunk;
    const int kend = min(K, kbeg + kchunk);
    const int m0 = ((t / gx) % gy) * GT, n0 = (t % gx) * GT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    flt4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = flt4{0.f, 0.f, 0.f, 0.f};

    double ra[LGL], rb[LGL];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int t = 0; t < LGL; ++t) {
            const int e = tid + t * 256;
            int mm, kk;
            if (!TA) { kk = e % LK; mm = e / LK; } else { mm = e % GT; kk = e / GT; }
            const int gm = m0 + mm, gk = k0 + kk;
            ra[t] = (gm < M && gk < kend) ? (TA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk]) : 0.0;
        }
#pragma unroll
        for (int t = 0; t < LGL; ++t) {
            const int e = tid + t * 256;
            int nn, kk;
            if (!TB) { nn = e % GT; kk = e / GT; } else { kk = e % LK; nn = e / LK; }
            const int gn = n0 + nn, gk = k0 + kk;
            rb[t] = (gn < N && gk < kend) ? (TB ? B[(int64_t)gn * ldb + gk] : B[(int64_t)gk * ldb + gn]) : 0.0;
        }
    };
    auto cvt = [](double x) -> elem {
        if constexpr (P == 1) return (float)x;
        else return to_bf16_bits(x);
    };
    auto stage = [&]() {
#pragma unroll
        for (int t = 0; t < LGL; ++t) {
            const int e = tid + t * 256;
            int mm, kk;
            if (!TA) { kk = e % LK; mm = e / LK; } else { mm = e % GT; kk = e / GT; }
            As[mm][kk] = cvt(ra[t]);
        }
#pragma unroll
        for (int t = 0; t < LGL; ++t) {
            const int e = tid + t * 256;
            int nn, kk;
            if (!TB) { nn = e % GT; kk = e / GT; } else { kk = e % LK; nn = e / LK; }
            Bs[nn][kk] = cvt(rb[t]);
        }
    };

    if (kbeg < kend) fetch(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += LK) {
        stage();
        __syncthreads();
        if (k0 + LK < kend) fetch(k0 + LK);
        const int r16 = lane & 15, q = lane >> 4;
        if constexpr (P == 1) {
#pragma unroll
            for (int kk = 0; kk < LK; kk += 4) {
                const float a0 = As[wm * 32 + r16][kk + q], a1 = As[wm * 32 + 16 + r16][kk + q];
                const float b0 = Bs[wn * 32 + r16][kk + q], b1 = Bs[wn * 32 + 16 + r16][kk + q];
                acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
                acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
                acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
                acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
            }
        } else {
            const bf16x8 a0 = *(const bf16x8*)&As[wm * 32 + r16][8 * q];
            const bf16x8 a1 = *(const bf16x8*)&As[wm * 32 + 16 + r16][8 * q];
            const bf16x8 b0 = *(const bf16x8*)&Bs[wn * 32 + r16][8 * q];
            const bf16x8 b1 = *(const bf16x8*)&Bs[wn * 32 + 16 + r16][8 * q];
            acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc[1][1], 0, 0, 0);
        }
        __syncthreads();
    }
    double* out;
    int64_t ldo;
    if (ksplit > 1) { out = Pp + (int64_t)z * M * N; ldo = N; }
    else { out = C + bz * sC; ldo = ldc; }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
                const int gn = n0 + wn * 32 + j * 16 + (lane & 15);
                if (gm < M && gn < N) {
                    double* c = out + (int64_t)gm * ldo + gn;
                    const double v = alpha * (double)acc[i][j][r];
                    *c = (beta == 0.0 || ksplit > 1) ? v : v + beta * (*c);
                }
            }
}

void gemm_lp(hipStream_t s, int prec, bool ta, bool tb, int M, int N, int K, double alpha,
             const double* A, int64_t lda, int64_t sA, const double* B, int64_t ldb, int64_t sB,
             double beta, double* C, int64_t ldc, int64_t sC, int batch, double* ws, int64_t ws_cap,
             hipEvent_t mid)
{
    if (M <= 0 || N <= 0 || batch <= 0) return;
    if (!ta && !tb && batch == 1 && K >= 1 && N <= kSkinnyCols && K <= kSkinnyMax && (int64_t)M * N >= (1 << 16)) {
        // HBM-bound: the FP64 skinny kernel moves the same bytes as an FP32
        // product would (operands and result are FP64 in memory)
        const int rows = 256 / ((N + kSkinnyCols - 1) / kSkinnyCols);
        hipLaunchKernelGGL(gemm_skinny_kernel, dim3((unsigned)((M + rows - 1) / rows)), dim3(256), 0, s, M, N, K,
                           alpha, A, lda, B, ldb, beta, C, ldc);
        if (mid) (void)hipEventRecord(mid, s);
        return;
    }
    int ksplit = (beta == 0.0 && ws) ? gemm_split_plan(M, N, K, batch, ws_cap) : 1;
    int kchunk = K;
    if (ksplit > 1) {
        kchunk = (((K + ksplit - 1) / ksplit) + LK - 1) / LK * LK;
        ksplit = (K + kchunk - 1) / kchunk;
    }
    dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT, batch * ksplit);
    dim3 block(256);
    double* P = ksplit > 1 ? ws : nullptr;
#define CTM_LP_LAUNCH(TA_, TB_, P_) \
    hipLaunchKernelGGL((gemm_lp_kernel<TA_, TB_, P_>), grid, block, 0, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, ksplit, kchunk, P)
    if (prec == 1) {
        if (!ta && !tb) CTM_LP_LAUNCH(false, false, 1);
        else if (ta && !tb) CTM_LP_LAUNCH(true, false, 1);
        else if (!ta && tb) CTM_LP_LAUNCH(false, true, 1);
        else CTM_LP_LAUNCH(true, true, 1);
    } else {
        if (!ta && !tb) CTM_LP_LAUNCH(false, false, 2);
        else if (ta && !tb) CTM_LP_LAUNCH(true, false, 2);
        else if (!ta && tb) CTM_LP_LAUNCH(false, true, 2);
        else CTM_LP_LAUNCH(true, true, 2);
    }
#undef CTM_LP_LAUNCH
    if (mid) (void)hipEventRecord(mid, s);
    if (ksplit > 1) {
        const int64_t total = (int64_t)batch * M * N;
        const int g = (int)std::min<int64_t>((total + 255) / 256, 4096);
        hipLaunchKernelGGL(gemm_reduce_kernel, dim3(g), dim3(256), 0, s, P, M, N, ksplit, C, ldc, sC, total);
    }
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

// 32-bit form (fewer than 2^31 elements): the mixed-radix digits of the output
// index come from division by invariant integers, q = (umulhi(x, mul) + x) >> s
// with s = ceil(log2 d) and mul = floor(2^32 (2^s - d) / d) + 1, exact for
// x < 2^31.
struct PermDesc32 {
    int rank;
    uint32_t od[12], is[12], mul[12], shr[12];
};

__global__ void permute32_kernel(const double* __restrict__ in, double* __restrict__ out, uint32_t n,
                                 PermDesc32 pd)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        uint32_t rem = i, off = 0;
        for (int k = pd.rank - 1; k >= 0; --k) {
            const uint32_t q = (__umulhi(rem, pd.mul[k]) + rem) >> pd.shr[k];
            off += (rem - q * pd.od[k]) * pd.is[k];
            rem = q;
        }
        out[i] = in[off];
    }
}

// testing aid: CTM_NO_TILED_PERMUTE=1 keeps every permute element-wise
static bool no_tiled_permute()
{
    static const bool off = std::getenv("CTM_NO_TILED_PERMUTE") != nullptr;
    return off;
}

// LDS-tiled form (plan in perm_plan.h): one tile per iteration of a
// grid-stride loop.  Per tile the 32-bit offsets of the out-block chunk in the
// input (itab) and of the in-block chunk in the output (otab) are decoded once.
// Load: one wave per LDS row (one out-block element), lanes along the in-block
// chunk x unit, contiguous in the input; store: one wave per in-block element,
// lanes along the out-block chunk x unit, contiguous in the output.  The LDS
// rows have an odd pitch.  Divisions by runtime values use multiply-shift.
__device__ inline uint32_t fdiv(uint32_t x, const FastDiv& f)
{
    return (__umulhi(x, f.mul) + x) >> f.shr;
}

constexpr int kPermPerThread = kPermTileElems / 256;

__global__ __launch_bounds__(256) void permute_tile_kernel(const double* __restrict__ in, double* __restrict__ out,
                                                           PermTile t)
{
    __shared__ double buf[kPermTileElems + kPermTileSide + 1];
    __shared__ uint32_t itab[kPermTileSide], otab[kPermTileSide];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nwv = blockDim.x >> 6;
    const int U = t.U, P = (t.TI * t.U) | 1;
    for (uint32_t tile = blockIdx.x; tile < (uint32_t)t.tiles; tile += gridDim.x) {
        uint32_t r = fdiv(tile, t.fco);
        const int co = (int)(tile - r * t.fco.d);
        uint32_t r2 = fdiv(r, t.fci);
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
        const int ti = min(t.TI, t.Lin - i0), to = min(t.TO, t.Lout - o0);
        for (int o = tid; o < to; o += blockDim.x) {
            uint32_t x = (uint32_t)(o0 + o), off = 0;
            for (int k = 0; k < t.nout; ++k) {
                const uint32_t q = x / (uint32_t)t.out_d[k];
                off += (x - q * (uint32_t)t.out_d[k]) * (uint32_t)t.out_is[k];
                x = q;
            }
            itab[o] = off;
        }
        for (int i = tid; i < ti; i += blockDim.x) {
            uint32_t x = (uint32_t)(i0 + i), off = 0;
            for (int k = 0; k < t.nin; ++k) {
                const uint32_t q = x / (uint32_t)t.in_d[k];
                off += (x - q * (uint32_t)t.in_d[k]) * (uint32_t)t.in_os[k];
                x = q;
            }
            otab[i] = off;
        }
        __syncthreads();
        // load: every thread issues its (up to kPermPerThread) reads before
        // writing any of them to LDS, so that they are in flight together
        const FastDiv& fr = t.frun[ci == t.nci - 1 ? 1 : 0];
        const int run = (int)fr.d, tot = to * run;
        const uint32_t ibase = ib + (uint32_t)i0 * (uint32_t)U;
        double v[kPermPerThread];
#pragma unroll
        for (int k = 0; k < kPermPerThread; ++k) {
            const int e = tid + k * 256;
            if (e < tot) {
                const int o = (int)fdiv((uint32_t)e, fr);
                v[k] = in[ibase + itab[o] + (uint32_t)(e - o * run)];
            }
        }
#pragma unroll
        for (int k = 0; k < kPermPerThread; ++k) {
            const int e = tid + k * 256;
            if (e < tot) {
                const int o = (int)fdiv((uint32_t)e, fr);
                buf[o * P + (e - o * run)] = v[k];
            }
        }
        __syncthreads();
        // store: row i of the output tile (one in-block element) is contiguous
        const FastDiv& fo = t.fruno[co == t.nco - 1 ? 1 : 0];
        const int runo = (int)fo.d, toto = ti * runo;
        const uint32_t obase = ob + (uint32_t)o0 * (uint32_t)U;
#pragma unroll
        for (int k = 0; k < kPermPerThread; ++k) {
            const int e = tid + k * 256;
            if (e < toto) {
                const int i = (int)fdiv((uint32_t)e, fo);
                const int w = e - i * runo;
                const int o = (int)fdiv((uint32_t)w, t.fU);
                out[obase + otab[i] + (uint32_t)w] = buf[o * P + i * U + (w - o * U)];
            }
        }
        __syncthreads();
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
    const int64_t lim = (int64_t)1 << 31;
    bool small = n < lim;
    int64_t span = 1;   // largest input offset + 1
    for (int k = 0; k < pd.rank; ++k) span += (pd.od[k] - 1) * pd.is[k];
    small = small && span < lim;
    PermTile pt{};
    if (small && !no_tiled_permute() && plan_perm_tile(pd.rank, pd.od, pd.is, pt)) {
        const int g = (int)std::min<int64_t>(pt.tiles, 4096);
        hipLaunchKernelGGL(permute_tile_kernel, dim3(g), dim3(256), 0, s, in, out, pt);
    } else if (small) {
        PermDesc32 p32{};
        p32.rank = pd.rank;
        for (int k = 0; k < pd.rank; ++k) {
            const uint64_t d = (uint64_t)pd.od[k];
            uint32_t sh = 0;
            while (((uint64_t)1 << sh) < d) ++sh;
            p32.od[k] = (uint32_t)d;
            p32.is[k] = (uint32_t)pd.is[k];
            p32.shr[k] = sh;
            p32.mul[k] = (uint32_t)((((uint64_t)1 << 32) * (((uint64_t)1 << sh) - d)) / d + 1);
        }
        hipLaunchKernelGGL(permute32_kernel, dim3(grid_for(n)), dim3(256), 0, s, in, out, (uint32_t)n, p32);
    } else {
        hipLaunchKernelGGL(permute_kernel, dim3(grid_for(n)), dim3(256), 0, s, in, out, n, pd);
    }
}

// ---------------------------------------------------------------------------
// sign convention of singular vectors: row i of UT (kk x m) and VT (kk x n)
// are negated when the entry of UT's row with the largest magnitude (first
// one on ties) is negative.  One block per row.
// ---------------------------------------------------------------------------
__global__ void sign_fix_kernel(double* __restrict__ UT, double* __restrict__ VT, int m, int n)
{
    __shared__ double bv[256];
    __shared__ int bi[256];
    const int row = blockIdx.x, tid = threadIdx.x;
    double* u = UT + (int64_t)row * m;
    double best = -1.0;
    int idx = m;
    for (int j = tid; j < m; j += blockDim.x) {
        const double a = fabs(u[j]);
        if (a > best) { best = a; idx = j; }
    }
    bv[tid] = best;
    bi[tid] = idx;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (tid < o) {
            const double b2 = bv[tid + o];
            const int i2 = bi[tid + o];
            if (b2 > bv[tid] || (b2 == bv[tid] && i2 < bi[tid])) { bv[tid] = b2; bi[tid] = i2; }
        }
        __syncthreads();
    }
    // every thread takes the decision before any thread negates u[jm]
    const int jm = bi[0];
    const bool neg = jm < m && u[jm] < 0.0;
    __syncthreads();
    if (neg) {
        double* v = VT + (int64_t)row * n;
        for (int j = tid; j < m; j += blockDim.x) u[j] = -u[j];
        for (int j = tid; j < n; j += blockDim.x) v[j] = -v[j];
    }
}

void sign_fix(hipStream_t s, double* UT, double* VT, int rows, int m, int n)
{
    if (rows <= 0) return;
    hipLaunchKernelGGL(sign_fix_kernel, dim3(rows), dim3(256), 0, s, UT, VT, m, n);
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

// copy j of the batch is served by the blocks with blockIdx.y == j
__global__ void copy_batch_kernel(CopyBatch cb)
{
    const int j = blockIdx.y;
    if (j >= cb.cnt) return;
    const double* __restrict__ a = cb.src[j];
    double* __restrict__ b = cb.dst[j];
    const int64_t n = cb.n[j];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

void copy_batch(hipStream_t s, const CopyBatch& cb)
{
    int64_t mx = 0;
    for (int j = 0; j < cb.cnt; ++j) mx = std::max(mx, cb.n[j]);
    if (cb.cnt <= 0 || mx <= 0) return;
    hipLaunchKernelGGL(copy_batch_kernel, dim3(grid_for(mx), cb.cnt), dim3(256), 0, s, cb);
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

// T[a][m][b] and T[b][m][a] replaced by their mean (edge tensor of the
// reduced method, symmetric in its two chi legs)
__global__ void symmetrize_edge_kernel(double* T, int x, int Df)
{
    const int64_t n = (int64_t)x * x * Df;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(i % x), m = (int)((i / x) % Df), a = (int)(i / ((int64_t)x * Df));
        if (a < b) {
            const int64_t j = ((int64_t)b * Df + m) * x + a;
            const double v = 0.5 * (T[i] + T[j]);
            T[i] = v;
            T[j] = v;
        }
    }
}

void symmetrize_edge(hipStream_t s, double* T, int x, int Df)
{
    hipLaunchKernelGGL(symmetrize_edge_kernel, dim3(grid_for((int64_t)x * x * Df)), dim3(256), 0, s, T, x, Df);
}

// Fused site tensor of the reduced method (Sec. II):
// a[(lk,li,lb),(uk,ui,ub),(rk,ri,rb),(dk,di,db)] = sum_{p,q} A[p,lk,uk,rk,dk]
// O[p,q,li,ui,ri,di] A[q,lb,ub,rb,db]; fused leg (ket, PEPO, bra) with the
// bra index fastest.  With the identity PEPO (dd = 1) this is the norm
// network's sum_p A[p] A[p].
__global__ void fuse_site_kernel(const double* __restrict__ A, const double* __restrict__ O, int D, int dd,
                                 double* __restrict__ a)
{
    const int Df = D * dd * D;
    const int64_t n = (int64_t)Df * Df * Df * Df;
    const int64_t D4 = (int64_t)D * D * D * D;
    const int d4 = dd * dd * dd * dd;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        int64_t t = e;
        int k[4], o[4], b[4];
        for (int leg = 3; leg >= 0; --leg) {
            int f = (int)(t % Df);
            t /= Df;
            b[leg] = f % D;
            f /= D;
            o[leg] = f % dd;
            k[leg] = f / dd;
        }
        const int64_t ik = (((int64_t)k[0] * D + k[1]) * D + k[2]) * D + k[3];
        const int64_t ib = (((int64_t)b[0] * D + b[1]) * D + b[2]) * D + b[3];
        const int io = ((o[0] * dd + o[1]) * dd + o[2]) * dd + o[3];
        double v = 0.0;
        for (int p = 0; p < 2; ++p)
            for (int q = 0; q < 2; ++q) v += A[p * D4 + ik] * O[(p * 2 + q) * d4 + io] * A[q * D4 + ib];
        a[e] = v;
    }
}

void fuse_site(hipStream_t s, const double* A, const double* O, int D, int dd, double* a)
{
    const int64_t Df = (int64_t)D * dd * D;
    hipLaunchKernelGGL(fuse_site_kernel, dim3(grid_for(Df * Df * Df * Df)), dim3(256), 0, s, A, O, D, dd, a);
}

// Environment of the bra tensor from the environment env of the fused site
// (legs as in fuse_site):
// E[q,lb,ub,rb,db] = sum env[...] A[p,lk,uk,rk,dk] O[p,q,li,ui,ri,di] over
// p and the ket and PEPO indices.  One workgroup per output entry, fixed
// reduction tree.
__global__ void unfuse_env_kernel(const double* __restrict__ env, const double* __restrict__ A,
                                  const double* __restrict__ O, int D, int dd, double* __restrict__ E)
{
    __shared__ double sh[16];
    const int64_t D4 = (int64_t)D * D * D * D;
    const int d4 = dd * dd * dd * dd;
    const int Df = D * dd * D;
    const int64_t out = blockIdx.x;                 // q * D4 + ib
    const int q = (int)(out / D4);
    int64_t ib = out % D4;
    int b[4];
    for (int leg = 3; leg >= 0; --leg) {
        b[leg] = (int)(ib % D);
        ib /= D;
    }
    const int64_t terms = 2 * D4 * d4;
    double v = 0.0;
    for (int64_t t = threadIdx.x; t < terms; t += blockDim.x) {
        const int io = (int)(t % d4);
        const int64_t ik = (t / d4) % D4;
        const int p = (int)(t / (d4 * D4));
        int64_t r = ik;
        int k[4], o[4];
        int rr = io;
        for (int leg = 3; leg >= 0; --leg) {
            k[leg] = (int)(r % D);
            r /= D;
            o[leg] = rr % dd;
            rr /= dd;
        }
        int64_t fe = 0;
        for (int leg = 0; leg < 4; ++leg) fe = fe * Df + ((int64_t)k[leg] * dd + o[leg]) * D + b[leg];
        v += env[fe] * A[p * D4 + ik] * O[(p * 2 + q) * d4 + io];
    }
    v = block_sum(v, sh);
    if (threadIdx.x == 0) E[out] = v;
}

void unfuse_env(hipStream_t s, const double* env, const double* A, const double* O, int D, int dd, double* E)
{
    const int64_t n = 2 * (int64_t)D * D * D * D;
    hipLaunchKernelGGL(unfuse_env_kernel, dim3((unsigned)n), dim3(256), 0, s, env, A, O, D, dd, E);
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
// kind PEPO_SPIN: the spin's value sigma(s) = +1 (s = 0), -1 (s = 1) under the
// sum (impurity tensor of the local magnetisation).  kind PEPO_DBETA: dO/dbeta,
// the product rule over the six legs with dw = (sinh b / sqrt(2cosh b)) P+ +
// (cosh b / sqrt(2sinh b)) P- (impurity tensor of the internal energy).
__global__ void ising_pepo_kernel(double* O, double beta, int kind)
{
    const int i = threadIdx.x;
    if (i >= 64) return;
    const double a = sqrt(2.0 * cosh(beta)), b = sqrt(2.0 * sinh(beta));
    const double w[2][2] = {{0.5 * (a + b), 0.5 * (a - b)}, {0.5 * (a - b), 0.5 * (a + b)}};
    const double da = sinh(beta) / a, db = cosh(beta) / b;
    const double dw[2][2] = {{0.5 * (da + db), 0.5 * (da - db)}, {0.5 * (da - db), 0.5 * (da + db)}};
    int idx[6];
    int rem = i;
    for (int k = 5; k >= 0; --k) { idx[k] = rem & 1; rem >>= 1; }
    double acc = 0.0;
    for (int s = 0; s < 2; ++s) {
        if (kind == PEPO_DBETA) {
            for (int k = 0; k < 6; ++k) {
                double t = dw[s][idx[k]];
                for (int j = 0; j < 6; ++j)
                    if (j != k) t *= w[s][idx[j]];
                acc += t;
            }
        } else {
            double t = (kind == PEPO_SPIN && s == 1) ? -1.0 : 1.0;
            for (int k = 0; k < 6; ++k) t *= w[s][idx[k]];
            acc += t;
        }
    }
    O[i] = acc;
}

void ising_pepo(hipStream_t s, double* O, double beta, int kind)
{
    hipLaunchKernelGGL(ising_pepo_kernel, dim3(1), dim3(64), 0, s, O, beta, kind);
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
constexpr int kCholLdsDoubles = 20224;     // 158 KiB

// (x_p, x_q) <- (c x_p - s x_q, s x_p + c x_q) over len entries, the G lanes of
// a group striding by G.  Loads are batched ahead of the stores (the columns
// are distinct) so that their latency is paid once per batch.
__device__ inline void rotate_pair(double* __restrict__ xp, double* __restrict__ xq, int len,
                                   int gl, int G, double c, double sn)
{
    constexpr int RB = 12;
    for (int r0 = gl; r0 < len; r0 += RB * G) {
        double a[RB], b[RB];
#pragma unroll
        for (int u = 0; u < RB; ++u) {
            const int r = r0 + u * G;
            a[u] = r < len ? xp[r] : 0.0;
            b[u] = r < len ? xq[r] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < RB; ++u) {
            const int r = r0 + u * G;
            if (r < len) {
                xp[r] = c * a[u] - sn * b[u];
                xq[r] = sn * a[u] + c * b[u];
            }
        }
    }
}

// A sweep whose rotations all had gamma^2 / (alpha beta) below this (cosines
// below 1e-8) is the last: cyclic Jacobi converges quadratically, so the
// columns are then orthogonal to ~1e-16 relative, and the sweep that would
// follow only confirms it.  (1e-20, the earlier bound, ran that sweep.)
constexpr float kJacobiDone = 1e-16f;

// XL / WL: X / W live in LDS (decided per batch on the host, so that every
// access compiles to LDS or global instructions instead of flat ones).
template <bool XL, bool WL>
__global__ __launch_bounds__(1024) void jacobi_svd_kernel(JacobiBatch jobs, int max_sweeps)
{
    extern __shared__ double lds[];
    const JacobiJob jb = jobs.job[blockIdx.x];
    const int m = jb.m, n = jb.n;
    const bool acc_v = jb.want_v != 0;
    double* X = XL ? lds : jb.X;
    double* W = WL ? lds + (int64_t)m * n : jb.W;
    const int ne = n + (n & 1);
    const int npairs = ne / 2;
    const int nthr = blockDim.x;
    int G = 64;
    while (G > 1 && G * npairs > nthr) G >>= 1;
    const int ngroups = nthr / G;
    const int gid = threadIdx.x / G, gl = threadIdx.x % G;
    __shared__ int rotated;
    __shared__ unsigned int maxr;                  // largest (gamma^2 / alpha beta) of the sweep, float bits
    __shared__ double sig[1024];
    __shared__ int rnk[1024];

    __shared__ double fro2;
    if (XL)
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
        if (threadIdx.x == 0) {
            rotated = 0;
            maxr = 0u;
        }
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
                    rotate_pair(xp, xq, m, gl, G, c, sn);
                    if (acc_v) rotate_pair(W + (int64_t)p * n, W + (int64_t)q * n, n, gl, G, c, sn);
                    if (gl == 0) {
                        rotated = 1;
                        atomicMax(&maxr, __float_as_uint((float)(ga * ga / (al * be))));
                    }
                }
            }
            __syncthreads();
        }
        if (rotated == 0 || __uint_as_float(maxr) < kJacobiDone) {
            if (jb.sweeps && threadIdx.x == 0) jb.sweeps[0] = sweep + 1;
            break;
        }
        __syncthreads();
        if (sweep + 1 == max_sweeps && jb.sweeps && threadIdx.x == 0) jb.sweeps[0] = max_sweeps;
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

// Small problems (m, n <= 128, X in LDS): every column pair of a round is
// served by 16 lanes; lanes 0-7 hold 16 rows each of the two columns of X,
// lanes 8-15 16 rows each of the two columns of V.  All loads of a round are
// issued together and V's (global) loads overlap the dot products and their
// reduction; the rotation is applied from registers.
typedef __attribute__((address_space(1))) double gdouble;
constexpr int kSmallJacobi = 128;

// v from the lane that the DPP control CTRL names (all 64 lanes active; the
// patterns used here read within a row of 16 lanes, so every lane is written
// and no old value is needed), FP64
template <int CTRL>
__device__ inline double dpp_f64(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
// sum over each aligned group of 16 lanes, result in every lane of the group:
// quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror
__device__ inline double sum16(double v)
{
    v += dpp_f64<0xB1>(v);
    v += dpp_f64<0x4E>(v);
    v += dpp_f64<0x141>(v);
    v += dpp_f64<0x140>(v);
    return v;
}
// the same over aligned groups of 8 lanes (the first three stages)
__device__ inline double sum8(double v)
{
    v += dpp_f64<0xB1>(v);
    v += dpp_f64<0x4E>(v);
    v += dpp_f64<0x141>(v);
    return v;
}

template <bool WL>
__global__ __launch_bounds__(1024) void jacobi_small_kernel(JacobiBatch jobs, int max_sweeps)
{
    extern __shared__ double lds[];
    const JacobiJob jb = jobs.job[blockIdx.x];
    const int m = jb.m, n = jb.n;
    const bool acc_v = jb.want_v != 0;
    double* X = lds;
    double* Wl = lds + (int64_t)m * n;              // WL: V in LDS
    gdouble* Wg = (gdouble*)jb.W;                    // !WL: V in global memory
    const int ne = n + (n & 1);
    const int npairs = ne / 2;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int grp = tid >> 4, l16 = tid & 15, half = l16 >> 3, sub = l16 & 7;
    __shared__ int rotated;
    __shared__ double sig[kSmallJacobi];
    __shared__ int rnk[kSmallJacobi];
    __shared__ double fro2;

    for (int i = tid; i < m * n; i += nthr) X[i] = jb.X[i];
    if (acc_v) {
        for (int i = tid; i < n * n; i += nthr) {
            const double v = ((i / n) == (i % n)) ? 1.0 : 0.0;
            if (WL) Wl[i] = v;
            else Wg[i] = v;
        }
    }
    __syncthreads();
    for (int j = tid; j < n; j += nthr) {
        double v = 0.0;
        for (int r = 0; r < m; ++r) v += X[j * m + r] * X[j * m + r];
        sig[j] = v;
    }
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int j = 0; j < n; ++j) t += sig[j];
        fro2 = t;
    }
    __syncthreads();
    const double noise2 = 1e-30 * fro2;
    const double tol = 2.0 * sqrt((double)m) * 2.220446049250313e-16;

    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        if (tid == 0) rotated = 0;
        __syncthreads();
        for (int step = 0; step < ne - 1; ++step) {
            int p = 0, q = 0;
            bool active = grp < npairs;
            if (active) {
                if (grp == 0) { p = ne - 1; q = step; }
                else { p = (step + grp) % (ne - 1); q = (step - grp + (ne - 1)) % (ne - 1); }
                if (p >= n || q >= n) active = false;
                if (p > q) { const int t = p; p = q; q = t; }
            }
            double a[16], b[16];
            double al = 0.0, be = 0.0, ga = 0.0;
            if (active && half == 1 && acc_v) {
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int r = sub + 8 * u;
                    a[u] = r < n ? (WL ? Wl[p * n + r] : Wg[p * n + r]) : 0.0;
                    b[u] = r < n ? (WL ? Wl[q * n + r] : Wg[q * n + r]) : 0.0;
                }
            }
            if (active && half == 0) {
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int r = sub + 8 * u;
                    a[u] = r < m ? X[p * m + r] : 0.0;
                    b[u] = r < m ? X[q * m + r] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    al += a[u] * a[u];
                    be += b[u] * b[u];
                    ga += a[u] * b[u];
                }
            }
            al = sum16(al);
            be = sum16(be);
            ga = sum16(ga);
            if (active && ga != 0.0 && al > noise2 && be > noise2 && ga * ga > tol * tol * (al * be)) {
                const double zeta = (be - al) / (2.0 * ga);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
                if (half == 0) {
#pragma unroll
                    for (int u = 0; u < 16; ++u) {
                        const int r = sub + 8 * u;
                        if (r < m) {
                            X[p * m + r] = c * a[u] - sn * b[u];
                            X[q * m + r] = sn * a[u] + c * b[u];
                        }
                    }
                    if (l16 == 0) rotated = 1;
                } else if (acc_v) {
#pragma unroll
                    for (int u = 0; u < 16; ++u) {
                        const int r = sub + 8 * u;
                        if (r < n) {
                            const double va = c * a[u] - sn * b[u], vb = sn * a[u] + c * b[u];
                            if (WL) { Wl[p * n + r] = va; Wl[q * n + r] = vb; }
                            else { Wg[p * n + r] = va; Wg[q * n + r] = vb; }
                        }
                    }
                }
            }
            __syncthreads();
        }
        if (rotated == 0) {
            if (jb.sweeps && tid == 0) jb.sweeps[0] = sweep + 1;
            break;
        }
        __syncthreads();
        if (sweep + 1 == max_sweeps && jb.sweeps && tid == 0) jb.sweeps[0] = max_sweeps;
    }
    // singular values = column norms; outputs sorted by descending value
    for (int j = tid; j < n; j += nthr) {
        double v = 0.0;
        for (int r = 0; r < m; ++r) v += X[j * m + r] * X[j * m + r];
        sig[j] = sqrt(v);
    }
    __syncthreads();
    for (int j = tid; j < n; j += nthr) {
        int r = 0;
        const double sj = sig[j];
        for (int i = 0; i < n; ++i) {
            const double si = sig[i];
            r += (si > sj) || (si == sj && i < j);
        }
        rnk[j] = r;
    }
    __syncthreads();
    for (int e = tid; e < n * m; e += nthr) {
        const int j = e / m, r = e % m;
        const double sj = sig[j];
        jb.U[(int64_t)rnk[j] * m + r] = X[e] * (sj > 0.0 ? 1.0 / sj : 0.0);
    }
    if (acc_v) {
        for (int e = tid; e < n * n; e += nthr) {
            const int j = e / n, r = e % n;
            jb.V[(int64_t)rnk[j] * n + r] = WL ? Wl[e] : Wg[e];
        }
    }
    for (int j = tid; j < n; j += nthr) jb.S[rnk[j]] = sig[j];
}

// Register-resident one-sided Jacobi for m, n <= 128 with the odd-even
// (transposition) ordering.  The n columns (a zero column is added when n is
// odd) sit at positions 0 .. ne-1; step s pairs positions (2p, 2p+1) when s is
// even and (2p+1, 2p+2) when s is odd, rotates each pair and swaps the two
// columns' positions.  After ne steps the order is reversed and every pair has
// met once (odd-even transposition sort of a reversed sequence), so a sweep is
// ne steps.  Pair p is held in registers by the 8 lanes of group p of a
// 512-thread workgroup: lane l holds rows l, l + 8, ..., l + 120 of both
// columns of X and of V (64 doubles).  Every wave computes the rotation of its
// eight pairs once, so the per-pair scalar work (the lane sums and the
// rotation parameters) is issued by two waves per SIMD; with 16 lanes per pair
// it took four and set the step time.  Between steps each pair hands one
// column to a neighbour through LDS: per step half of the columns move and
// nothing else touches memory.
constexpr int kRegJacobi = 128;
constexpr int kRegLanes = 8;                       // lanes per column pair
constexpr int kRegThreads = kRegJacobi / 2 * kRegLanes;

template <bool WANT_V>
__global__ __launch_bounds__(kRegThreads) void jacobi_reg_kernel(JacobiBatch jobs, int max_sweeps)
{
    constexpr int NP = kRegJacobi / 2;             // pairs = 8-lane groups
    constexpr int RL = kRegJacobi / kRegLanes;     // rows per lane
    // LDS column slot: X rows, V rows, and a pad that puts the groups of a
    // wave on different banks (slot stride = 64 bytes modulo 256)
    constexpr int XS = 2 * kRegJacobi + kRegLanes;
    static_assert(NP * kRegLanes == kRegThreads && kRegLanes == 8, "one pair per 8-lane group");
    __shared__ __attribute__((aligned(16))) double xfer[NP][XS];
    __shared__ __attribute__((aligned(16))) double park[XS];
    __shared__ int xid[NP];
    __shared__ int park_id;
    __shared__ double sig[kRegJacobi + 1];
    __shared__ int rnk[kRegJacobi + 1];
    __shared__ double gsum[NP];
    __shared__ int rotated;
    __shared__ unsigned int maxr;                  // largest (gamma^2 / alpha beta) of the sweep, float bits
    __shared__ double fro2;
    const JacobiJob jb = jobs.job[blockIdx.x];
    const int m = jb.m, n = jb.n;
    const int ne = n + (n & 1);
    const int P = ne / 2;
    const int tid = threadIdx.x, p = tid >> 3, l8 = tid & 7;

    // columns at positions 2p (a) and 2p+1 (b): X rows in ax/bx, V rows in av/bv
    double ax[RL], bx[RL], av[RL], bv[RL];
    int ia = 2 * p, ib = 2 * p + 1;
#pragma unroll
    for (int u = 0; u < RL; ++u) {
        const int r = l8 + 8 * u;
        const bool live = p < P;
        ax[u] = (live && r < m && ia < n) ? jb.X[(int64_t)ia * m + r] : 0.0;
        bx[u] = (live && r < m && ib < n) ? jb.X[(int64_t)ib * m + r] : 0.0;
        av[u] = (WANT_V && live && r < n && r == ia) ? 1.0 : 0.0;
        bv[u] = (WANT_V && live && r < n && r == ib) ? 1.0 : 0.0;
    }
    {
        double t = 0.0;
#pragma unroll
        for (int u = 0; u < RL; ++u) t += ax[u] * ax[u] + bx[u] * bx[u];
        t = sum8(t);
        if (l8 == 0) gsum[p] = t;
        __syncthreads();
        if (tid == 0) {
            double f = 0.0;
            for (int i = 0; i < NP; ++i) f += gsum[i];
            fro2 = f;
        }
        __syncthreads();
    }
    const double noise2 = 1e-30 * fro2;
    const double tol = 2.0 * sqrt((double)m) * 2.220446049250313e-16;
    const double tol2 = tol * tol;

    // largest (gamma^2 / alpha beta) and whether any rotation happened, of
    // this thread's pairs in the current sweep (published once per sweep)
    float my_max = 0.0f;
    bool my_rot = false;
    // rotation of the pair held in (L, R), then swap of their positions:
    // L <- s L + c R, R <- c L - s R; lid / rid follow the columns
    auto rotate = [&](double (&Lx)[RL], double (&Rx)[RL], double (&Lv)[RL], double (&Rv)[RL], int& lid, int& rid,
                      bool odd) {
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
        for (int u = 0; u < RL; ++u) {
            al += Lx[u] * Lx[u];
            be += Rx[u] * Rx[u];
            ga += Lx[u] * Rx[u];
        }
        al = sum8(al);
        be = sum8(be);
        ga = sum8(ga);
        if (!(p < P && (!odd || p < P - 1))) return;
        double c = 1.0, sn = 0.0;
        if (ga != 0.0 && al > noise2 && be > noise2 && ga * ga > tol2 * (al * be)) {
            // t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)) with zeta = d / g2,
            // numerator and denominator scaled by |g2|: one division fewer
            // (the quotient and 1 / sqrt(1 + t^2) from the hardware reciprocal
            // and reciprocal square root, each refined by two Newton steps to
            // full FP64 accuracy; the denominator is at least |g2| > 0 and
            // 1 + t^2 lies in [1, 2])
            const double d = be - al, g2 = 2.0 * ga;
            const double sg = (d == 0.0 || ((d > 0.0) == (g2 > 0.0))) ? 1.0 : -1.0;
            const double den = fabs(d) + sqrt(d * d + g2 * g2);
            double q = __builtin_amdgcn_rcp(den);
            q = fma(q, fma(-den, q, 1.0), q);
            q = fma(q, fma(-den, q, 1.0), q);
            const double t = sg * fabs(g2) * q;
            const double h = fma(t, t, 1.0);
            double y = __builtin_amdgcn_rsq(h);
            y = y * fma(-0.5 * h * y, y, 1.5);
            y = y * fma(-0.5 * h * y, y, 1.5);
            c = y;
            sn = c * t;
            my_rot = true;
            // only compared with kJacobiDone: the unrefined reciprocal suffices
            my_max = fmaxf(my_max, (float)(ga * ga * __builtin_amdgcn_rcp(al * be)));
        }
#pragma unroll
        for (int u = 0; u < RL; ++u) {
            const double x = Lx[u], y = Rx[u];
            Lx[u] = sn * x + c * y;
            Rx[u] = c * x - sn * y;
        }
        if (WANT_V) {
#pragma unroll
            for (int u = 0; u < RL; ++u) {
                const double x = Lv[u], y = Rv[u];
                Lv[u] = sn * x + c * y;
                Rv[u] = c * x - sn * y;
            }
        }
        const int t = lid;
        lid = rid;
        rid = t;
    };
    auto put = [&](double* dst, const double (&x)[RL], const double (&v)[RL]) {
#pragma unroll
        for (int u = 0; u < RL; ++u) dst[l8 + 8 * u] = x[u];
        if (WANT_V)
#pragma unroll
            for (int u = 0; u < RL; ++u) dst[kRegJacobi + l8 + 8 * u] = v[u];
    };
    auto get = [&](const double* src, double (&x)[RL], double (&v)[RL]) {
#pragma unroll
        for (int u = 0; u < RL; ++u) x[u] = src[l8 + 8 * u];
        if (WANT_V)
#pragma unroll
            for (int u = 0; u < RL; ++u) v[u] = src[kRegJacobi + l8 + 8 * u];
    };

    // Registers a and b trade roles between the two halves of a double step:
    // even step: left = a (position 2p), right = b (2p+1); the column at 2p
    // leaves and the one at 2p+2 arrives into a, so the odd step has left = b
    // (2p+1), right = a (2p+2); then the column at 2p+2 leaves and the one at
    // 2p arrives into a, restoring the even-step roles.
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        if (tid == 0) {
            rotated = 0;
            maxr = 0u;
        }
        my_max = 0.0f;
        my_rot = false;
        __syncthreads();
        for (int step = 0; step < ne; step += 2) {
            rotate(ax, bx, av, bv, ia, ib, false);
            // even -> odd: send position 2p (a) to p-1 (p = 0: park), receive 2p+2 into a
            if (p < P) {
                put(p == 0 ? park : xfer[p], ax, av);
                if (l8 == 0) {
                    if (p == 0) park_id = ia;
                    else xid[p] = ia;
                }
            }
            __syncthreads();
            if (p < P) {
                if (p + 1 < P) {
                    get(xfer[p + 1], ax, av);
                    ia = xid[p + 1];
                } else {
#pragma unroll
                    for (int u = 0; u < RL; ++u) ax[u] = av[u] = 0.0;
                    ia = -1;
                }
            }
            __syncthreads();
            rotate(bx, ax, bv, av, ib, ia, true);
            // odd -> even: send position 2p+2 (a) to p+1, receive 2p into a (p = 0: park)
            if (p + 1 < P) {
                put(xfer[p], ax, av);
                if (l8 == 0) xid[p] = ia;
            }
            __syncthreads();
            if (p < P) {
                get(p == 0 ? park : xfer[p - 1], ax, av);
                ia = p == 0 ? park_id : xid[p - 1];
            }
            __syncthreads();
        }
        if (l8 == 0 && my_rot) {
            rotated = 1;
            atomicMax(&maxr, __float_as_uint(my_max));
        }
        __syncthreads();
        // done when no pair rotated, or when every rotation of this sweep was
        // below kJacobiDone (see there)
        if (rotated == 0 || __uint_as_float(maxr) < kJacobiDone) {
            if (jb.sweeps && tid == 0) jb.sweeps[0] = sweep + 1;
            break;
        }
        __syncthreads();
        if (sweep + 1 == max_sweeps && jb.sweeps && tid == 0) jb.sweeps[0] = max_sweeps;
    }
    // singular values = column norms, by original column id (the padding column has id n)
    {
        double na = 0.0, nb = 0.0;
#pragma unroll
        for (int u = 0; u < RL; ++u) {
            na += ax[u] * ax[u];
            nb += bx[u] * bx[u];
        }
        na = sum8(na);
        nb = sum8(nb);
        if (p < P && l8 == 0) {
            if (ia >= 0 && ia < n) sig[ia] = sqrt(na);
            if (ib >= 0 && ib < n) sig[ib] = sqrt(nb);
        }
    }
    __syncthreads();
    for (int j = tid; j < n; j += blockDim.x) {
        int r = 0;
        const double sj = sig[j];
        for (int i = 0; i < n; ++i) {
            const double si = sig[i];
            r += (si > sj) || (si == sj && i < j);
        }
        rnk[j] = r;
    }
    __syncthreads();
    if (p >= P) return;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const int id = side == 0 ? ia : ib;
        if (id < 0 || id >= n) continue;
        const int dst = rnk[id];
        const double sj = sig[id];
        const double inv = sj > 0.0 ? 1.0 / sj : 0.0;
#pragma unroll
        for (int u = 0; u < RL; ++u) {
            const int r = l8 + 8 * u;
            if (r < m) jb.U[(int64_t)dst * m + r] = (side == 0 ? ax[u] : bx[u]) * inv;
            if (WANT_V && r < n) jb.V[(int64_t)dst * n + r] = side == 0 ? av[u] : bv[u];
        }
        if (l8 == 0) jb.S[dst] = sj;
    }
}

// the register kernel takes every job of the batch (m, n <= kSmallJacobi and
// one want_v for all); it reads X and never writes it
bool jacobi_reads_only(const JacobiBatch& jobs)
{
    bool small = jobs.n > 0, any_v = false, all_v = true;
    for (int i = 0; i < jobs.n; ++i) {
        const JacobiJob& j = jobs.job[i];
        small = small && j.m <= kSmallJacobi && j.n <= kSmallJacobi;
        any_v = any_v || j.want_v;
        all_v = all_v && j.want_v;
    }
    return small && (all_v || !any_v);
}

void jacobi_svd(hipStream_t s, const JacobiBatch& jobs, int max_sweeps)
{
    if (jobs.n <= 0) return;
    bool xl = true, wl = true, small = true;
    int64_t need_x = 0, need_w = 0;
    for (int i = 0; i < jobs.n; ++i) {
        const JacobiJob& j = jobs.job[i];
        const int64_t mn = (int64_t)j.m * j.n;
        const int64_t nn = j.want_v ? (int64_t)j.n * j.n : 0;
        xl = xl && mn <= kJacobiLdsDoubles;
        wl = wl && mn + nn <= kJacobiLdsDoubles;
        small = small && j.m <= kSmallJacobi && j.n <= kSmallJacobi;
        need_x = std::max(need_x, mn);
        need_w = std::max(need_w, mn + nn);
    }
    bool any_v = false, all_v = true;
    for (int i = 0; i < jobs.n; ++i) {
        any_v = any_v || jobs.job[i].want_v;
        all_v = all_v && jobs.job[i].want_v;
    }
    if (jacobi_reads_only(jobs)) {
        if (all_v)
            hipLaunchKernelGGL((jacobi_reg_kernel<true>), dim3(jobs.n), dim3(kRegThreads), 0, s, jobs, max_sweeps);
        else
            hipLaunchKernelGGL((jacobi_reg_kernel<false>), dim3(jobs.n), dim3(kRegThreads), 0, s, jobs, max_sweeps);
    } else if (small && wl)
        hipLaunchKernelGGL((jacobi_small_kernel<true>), dim3(jobs.n), dim3(1024), need_w * sizeof(double), s, jobs, max_sweeps);
    else if (small)
        hipLaunchKernelGGL((jacobi_small_kernel<false>), dim3(jobs.n), dim3(1024), need_x * sizeof(double), s, jobs, max_sweeps);
    else if (xl && wl)
        hipLaunchKernelGGL((jacobi_svd_kernel<true, true>), dim3(jobs.n), dim3(1024), need_w * sizeof(double), s, jobs, max_sweeps);
    else if (xl)
        hipLaunchKernelGGL((jacobi_svd_kernel<true, false>), dim3(jobs.n), dim3(1024), need_x * sizeof(double), s, jobs, max_sweeps);
    else
        hipLaunchKernelGGL((jacobi_svd_kernel<false, false>), dim3(jobs.n), dim3(1024), 0, s, jobs, max_sweeps);
}

// ---------------------------------------------------------------------------
// shifted Cholesky QR factor, one workgroup per problem
// ---------------------------------------------------------------------------
// Input  G: k x k Gram matrix Y Y^T of the k rows of Y (row-major, global).
// Output T: k x k lower-triangular, T = L^-1 D with D = diag(G)^-1/2 and
//        L L^T = D G D + shift I, so that the rows of T Y are orthonormal
//        (up to the shift).  The work lives in LDS when k*k + 2k doubles fit.
//        Non-positive pivots (rank deficiency beyond the shift) give zero rows.
template <bool IN_LDS>
__global__ __launch_bounds__(1024) void cholqr_kernel(CholBatch jobs, double shift)
{
    extern __shared__ double lds[];
    const CholJob jb = jobs.job[blockIdx.x];
    const int k = jb.k;
    double* A = IN_LDS ? lds : jb.G;                 // working matrix
    double* dsc = IN_LDS ? lds + (int64_t)k * k : jb.work;
    double* dinv = dsc + k;
    const int nthr = blockDim.x, tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6, nw = nthr >> 6;
    for (int i = tid; i < k; i += nthr) {
        const double v = jb.G[(int64_t)i * k + i];
        dsc[i] = v > 0.0 ? 1.0 / sqrt(v) : 0.0;
    }
    __syncthreads();
    // lower triangle: D G D + shift I; strict upper triangle: 0 (X = identity)
    for (int64_t e = tid; e < (int64_t)k * k; e += nthr) {
        const int i = (int)(e / k), l = (int)(e % k);
        A[e] = (l <= i) ? jb.G[e] * dsc[i] * dsc[l] + (i == l ? shift : 0.0) : 0.0;
    }
    __syncthreads();
    // Gaussian elimination without pivoting (LDL^T): the lower triangle holds
    // the Schur complement, the strict upper triangle the unit lower-triangular
    // elimination matrix X transposed (X_ic at A[c][i]), so that X A0 X^T =
    // diag(p) with the pivots p on the diagonal, and L^-1 = diag(p)^-1/2 X.
    // Step j, row i > j, with f = A_ij / A_jj, touches in one sweep over e <= i:
    //   e <  j : X_ie -= f X_je     (A[e][i] -= f A[e][j])
    //   e == j : X_ij  = -f         (A[j][i]  = -f)
    //   e >  j : S_ie -= f S_ej     (A[i][e] -= f A[e][j])
    // Column j is read and never written in step j: one barrier per step.
    for (int j = 0; j < k; ++j) {
        const double pj = A[(int64_t)j * k + j];
        const double inv = pj > 0.0 ? 1.0 / pj : 0.0;
        for (int i = j + 1 + wave; i < k; i += nw) {
            const double f = A[(int64_t)i * k + j] * inv;
            for (int e = lane; e <= i; e += 64) {
                if (e == j) { A[(int64_t)j * k + i] = -f; continue; }
                const double v = f * A[(int64_t)e * k + j];
                if (e < j) A[(int64_t)e * k + i] -= v;
                else A[(int64_t)i * k + e] -= v;
            }
        }
        __syncthreads();
    }
    for (int i = tid; i < k; i += nthr) {
        const double p = A[(int64_t)i * k + i];
        dinv[i] = p > 0.0 ? 1.0 / sqrt(p) : 0.0;
    }
    __syncthreads();
    // T[i][c] = p_i^-1/2 X_ic d_c  (X_ii = 1)
    for (int64_t e = tid; e < (int64_t)k * k; e += nthr) {
        const int i = (int)(e / k), c = (int)(e % k);
        double v = 0.0;
        if (i == c) v = dinv[i] * dsc[c];
        else if (i > c) v = dinv[i] * A[(int64_t)c * k + i] * dsc[c];
        jb.T[e] = v;
    }
}

// k <= 128: the same elimination, blocked, with the rows in registers.
// Waves 1-15 own the rows (row i in wave 1 + i % 15, slot i / 15; each lane
// holds the entries e = lane and lane + 64 of its rows of the Schur
// complement S and of the elimination matrix X).  Per block of kCholB columns
// j0 .. j0+nb-1: wave 0 (the panel wave) eliminates within the block in
// registers, broadcasting the factors with readlane, and writes back the
// block rows as they stand at their own pivot step together with the
// reciprocal pivots; every row below the block then applies the nb
// eliminations S_i -= f S_t, X_i -= f X_t with f = S_t[i] / p_t (S_t[i] =
// S_i[t] by symmetry of the Schur complement).  Look-ahead: after a block's
// panel step the owners first bring the next block's rows up to date and
// publish them, so that the panel wave eliminates the next block while the
// owners apply the current one to the remaining rows.  Every row receives
// the blocks in order, with the same factors, as without the look-ahead.  Two
// barriers per block instead of one per column; the block buffers are
// double-buffered.
constexpr int kCholReg = 128;
constexpr int kCholB = 8;
constexpr int kCholOwners = 15;
constexpr int kCholSlots = (kCholReg + kCholOwners - 1) / kCholOwners;

__device__ inline double readlane_f64(double v, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// The eliminations of one block (pivot rows bSb / bXb [0, nbb) as they stand
// at their own pivot steps, reciprocal pivots binvb, first column jb0)
// applied to the owner's rows i in [lo, hi): S_i -= f S_t, X_i -= f X_t with
// f = S_t[i] / p_t, pivots in order.  s0 = 0 once entry 64 is passed and
// x1 = 0 until it is reached, so all four updates run unconditionally (exact
// no-ops then; the conditional form compiled to selects).
__device__ __forceinline__ void chol_apply_block(double (&S)[kCholSlots][2], double (&Xr)[kCholSlots][2],
                                                 const double (&bSb)[kCholB][kCholReg],
                                                 const double (&bXb)[kCholB][kCholReg], const double* binvb,
                                                 int jb0, int nbb, int ow, int lane, int lo, int hi)
{
    const bool s_lo = jb0 < 64;                   // S entries 0-63 still live
    const bool x_hi = jb0 + nbb > 64;             // X_t entries 64-127 can be nonzero
#pragma unroll
    for (int t = 0; t < kCholB; ++t) {
        if (t >= nbb) break;
        const double s0 = s_lo ? bSb[t][lane] : 0.0, s1 = bSb[t][lane + 64];
        const double x0 = bXb[t][lane], x1 = x_hi ? bXb[t][lane + 64] : 0.0;
        const double inv = binvb[t];
#pragma unroll
        for (int s = 0; s < kCholSlots; ++s) {
            const int i = ow + kCholOwners * s;
            if (i >= lo && i < hi) {
                const double f = bSb[t][i] * inv;
                S[s][0] -= f * s0;
                S[s][1] -= f * s1;
                Xr[s][0] -= f * x0;
                Xr[s][1] -= f * x1;
            }
        }
    }
}

__global__ __launch_bounds__(1024) void cholqr_reg_kernel(CholBatch jobs, double shift)
{
    __shared__ double dsc[kCholReg];
    __shared__ double bS[2][kCholB][kCholReg];
    __shared__ double bX[2][kCholB][kCholReg];
    __shared__ double binv[2][kCholB];
    const CholJob jb = jobs.job[blockIdx.x];
    const int k = jb.k;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ow = wave - 1;                       // owner index; -1: the panel wave
    for (int i = tid; i < k; i += blockDim.x) {
        const double v = jb.G[(int64_t)i * k + i];
        dsc[i] = v > 0.0 ? 1.0 / sqrt(v) : 0.0;
    }
    __syncthreads();
    double S[kCholSlots][2], Xr[kCholSlots][2];
#pragma unroll
    for (int s = 0; s < kCholSlots; ++s) {
        const int i = ow + kCholOwners * s;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int e = lane + 64 * u;
            const bool ok = ow >= 0 && i < k && e < k;
            S[s][u] = ok ? jb.G[(int64_t)i * k + e] * dsc[i] * dsc[e] + (i == e ? shift : 0.0) : 0.0;
            Xr[s][u] = (ok && i == e) ? 1.0 : 0.0;
        }
    }
    // the owners publish the rows of the first block
    if (ow >= 0) {
#pragma unroll
        for (int s = 0; s < kCholSlots; ++s) {
            const int i = ow + kCholOwners * s;
            if (i < min(kCholB, k)) {
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    bS[0][i][lane + 64 * u] = S[s][u];
                    bX[0][i][lane + 64 * u] = Xr[s][u];
                }
            }
        }
    }
    __syncthreads();
    int buf = 0;
    for (int j0 = 0; j0 < k; j0 += kCholB, buf ^= 1) {
        const int nb = min(kCholB, k - j0);
        const int j1 = j0 + nb, nb1 = min(kCholB, k - j1);   // the next block (nb1 <= 0: none)
        if (ow < 0) {
            // panel wave: elimination within the block, in the registers that
            // hold rows in the owner waves (the panel wave owns none)
            static_assert(kCholB <= kCholSlots, "block rows fit the row registers");
            double (&rs)[kCholSlots][2] = S;
            double (&rx)[kCholSlots][2] = Xr;
#pragma unroll
            for (int t = 0; t < kCholB; ++t)
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    rs[t][u] = t < nb ? bS[buf][t][lane + 64 * u] : 0.0;
                    rx[t][u] = t < nb ? bX[buf][t][lane + 64 * u] : 0.0;
                }
            const bool hi = j0 >= 64;                 // a block never straddles entry 64
            const int el = j0 & 63;
#pragma unroll
            for (int t = 0; t < kCholB; ++t) {
                if (t >= nb) break;
                const double piv = readlane_f64(hi ? rs[t][1] : rs[t][0], el + t);
                // reciprocal pivot: hardware reciprocal and two Newton steps
                // (full FP64 accuracy; the serial chain of the panel is shorter
                // than with the IEEE division sequence)
                double q = __builtin_amdgcn_rcp(piv);
                q = fma(q, fma(-piv, q, 1.0), q);
                q = fma(q, fma(-piv, q, 1.0), q);
                const double inv = piv > 0.0 ? q : 0.0;
                if (lane == 0) binv[buf][t] = inv;
#pragma unroll
                for (int t2 = t + 1; t2 < kCholB; ++t2) {
                    if (t2 >= nb) break;
                    const double f = readlane_f64(hi ? rs[t2][1] : rs[t2][0], el + t) * inv;
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        rs[t2][u] -= f * rs[t][u];
                        rx[t2][u] -= f * rx[t][u];
                    }
                }
            }
#pragma unroll
            for (int t = 0; t < kCholB; ++t)
                if (t < nb)
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        bS[buf][t][lane + 64 * u] = rs[t][u];
                        bX[buf][t][lane + 64 * u] = rx[t][u];
                    }
        } else if (j0 > 0) {
            // look-ahead: while the panel wave works on this block, the
            // previous block's eliminations reach the rows below this block
            // (the rows of this block took them before it was published)
            chol_apply_block(S, Xr, bS[buf ^ 1], bX[buf ^ 1], binv[buf ^ 1], j0 - kCholB, kCholB, ow, lane, j1, k);
        }
        __syncthreads();
        if (ow >= 0) {
            // the block's own rows take their eliminated values
#pragma unroll
            for (int s = 0; s < kCholSlots; ++s) {
                const int i = ow + kCholOwners * s;
                if (i >= j0 && i < j1) {
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        S[s][u] = bS[buf][i - j0][lane + 64 * u];
                        Xr[s][u] = bX[buf][i - j0][lane + 64 * u];
                    }
                }
            }
            // the next block's rows (at most one per owner: 8 consecutive
            // rows fall on 8 different owners) take this block's
            // eliminations first and are published for the panel wave
            if (nb1 > 0) {
                chol_apply_block(S, Xr, bS[buf], bX[buf], binv[buf], j0, nb, ow, lane, j1, j1 + nb1);
#pragma unroll
                for (int s = 0; s < kCholSlots; ++s) {
                    const int i = ow + kCholOwners * s;
                    if (i >= j1 && i < j1 + nb1) {
#pragma unroll
                        for (int u = 0; u < 2; ++u) {
                            bS[buf ^ 1][i - j1][lane + 64 * u] = S[s][u];
                            bX[buf ^ 1][i - j1][lane + 64 * u] = Xr[s][u];
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    // pivots p_i = S_ii; T[i][c] = p_i^-1/2 X_ic d_c
    if (ow < 0) return;
#pragma unroll
    for (int s = 0; s < kCholSlots; ++s) {
        const int i = ow + kCholOwners * s;
        if (i >= k) continue;
        const double pii = readlane_f64((i >> 6) ? S[s][1] : S[s][0], i & 63);
        const double di = pii > 0.0 ? 1.0 / sqrt(pii) : 0.0;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int c = lane + 64 * u;
            if (c < k) jb.T[(int64_t)i * k + c] = c <= i ? di * Xr[s][u] * dsc[c] : 0.0;
        }
    }
}

void cholqr(hipStream_t s, const CholBatch& jobs, double shift)
{
    if (jobs.n <= 0) return;
    int64_t need = 0;
    bool fits = true, reg = true;
    for (int i = 0; i < jobs.n; ++i) {
        const int64_t kk = jobs.job[i].k;
        fits = fits && kk * kk + 2 * kk <= kCholLdsDoubles;
        reg = reg && kk <= kCholReg;
        need = std::max(need, kk * kk + 2 * kk);
    }
    if (reg)
        hipLaunchKernelGGL(cholqr_reg_kernel, dim3(jobs.n), dim3(1024), 0, s, jobs, shift);
    else if (fits)
        hipLaunchKernelGGL((cholqr_kernel<true>), dim3(jobs.n), dim3(1024), need * sizeof(double), s, jobs, shift);
    else
        hipLaunchKernelGGL((cholqr_kernel<false>), dim3(jobs.n), dim3(1024), 0, s, jobs, shift);
}

}  // namespace ctmk

