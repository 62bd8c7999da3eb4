// Internal launcher declarations of the split-CTMRG device kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ctmk {

struct PermDesc {
    int rank;
    int64_t od[12];  // output dims (row-major)
    int64_t is[12];  // input stride of each output dim
};

struct JacobiJob {
    double* X;  // m x n column-major input (destroyed, unless jacobi_reads_only)
    double* W;  // n x n workspace
    double* U;  // m x n column-major output
    double* V;  // n x n column-major output
    double* S;  // n singular values, descending
    int m, n;
    int want_v; // 0: do not accumulate V (V output left untouched)
    int* sweeps; // optional (may be NULL): sweeps done
};

constexpr int kMaxJacobiBatch = 16;
struct JacobiBatch {            // passed by value as a kernel argument
    JacobiJob job[kMaxJacobiBatch];
    int n;
};

struct CholJob {
    double* G;     // k x k Gram (input; used as workspace when it does not fit in LDS)
    double* work;  // 2k doubles of workspace (global fallback)
    double* T;     // k x k output, T = L^-1 D
    int k;
};
struct CholBatch {
    CholJob job[kMaxJacobiBatch];
    int n;
};

// ws (may be NULL): workspace of ws_cap doubles for split-K partial products;
// mid (may be NULL): event recorded between the product and the split-K
// reduction (profiling)
void gemm_f64(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha,
              const double* A, int64_t lda, int64_t sA, const double* B, int64_t ldb, int64_t sB,
              double beta, double* C, int64_t ldc, int64_t sC, int batch,
              double* ws = nullptr, int64_t ws_cap = 0, hipEvent_t mid = nullptr);
int gemm_split_plan(int M, int N, int K, int batch, int64_t ws_cap);

// Grouped FP64 GEMM: C_i = alpha op(A_i) op(B_i) for up to kMaxGemmGroup
// problems of different shapes (same transposes) in one launch, plus one
// reduction launch when some problem's K range is split (deterministic).
constexpr int kMaxGemmGroup = 16;
struct GemmProb {
    const double* A;
    const double* B;
    double* C;
    int M, N, K;
    int64_t lda, ldb, ldc;
};
void gemm_f64_group(hipStream_t s, bool ta, bool tb, const GemmProb* p, int n, double alpha, double* ws,
                    int64_t ws_cap, hipEvent_t mid);
int gemm_group_splits(const GemmProb* p, int n, int64_t ws_cap);   // problems whose K range is split
// the same product with FP32 (prec 1) or BF16 (prec 2) operands and FP32
// accumulation; operands and result FP64 in memory
void gemm_lp(hipStream_t s, int prec, bool ta, bool tb, int M, int N, int K, double alpha,
             const double* A, int64_t lda, int64_t sA, const double* B, int64_t ldb, int64_t sB,
             double beta, double* C, int64_t ldc, int64_t sC, int batch, double* ws, int64_t ws_cap,
             hipEvent_t mid = nullptr);
void permute(hipStream_t s, const double* in, double* out, const PermDesc& pd, int64_t n);
void dot(hipStream_t s, const double* x, const double* y, int64_t n, double* out, double* part, int mode);
void scale_inv(hipStream_t s, double* x, int64_t n, const double* dev_scalar);
void fill(hipStream_t s, double* x, int64_t n, double v);
void copy(hipStream_t s, const double* a, double* b, int64_t n);
// up to kMaxCopyBatch copies in one launch; no destination may overlap any
// source or other destination of the batch
constexpr int kMaxCopyBatch = 8;
struct CopyBatch {
    const double* src[kMaxCopyBatch];
    double* dst[kMaxCopyBatch];
    int64_t n[kMaxCopyBatch];
    int cnt;
};
void copy_batch(hipStream_t s, const CopyBatch& cb);
void eye(hipStream_t s, double* x, int n);
void symmetrize(hipStream_t s, double* x, int n);
void scale_lines(hipStream_t s, double* x, int R, int C, const double* f, int mode);
void inv_sqrt_cut(hipStream_t s, const double* S, double* f, int n, double cutoff);
void diag_inv_sqrt(hipStream_t s, const double* G, int n, double* d);
void count_above(hipStream_t s, const double* S, int n, double cutoff, int* out);
void randn(hipStream_t s, double* x, int64_t n, uint64_t seed);
void d4_project(hipStream_t s, const double* A, double* out, int D);
enum { PEPO_PLAIN = 0, PEPO_SPIN = 1, PEPO_DBETA = 2 };
void ising_pepo(hipStream_t s, double* O, double beta, int kind = PEPO_PLAIN);
void identity_pepo(hipStream_t s, double* O);
// reduced method: fused site tensor (Df = D dd D per leg), bra environment
// from the fused-site environment, chi-leg symmetrisation of an edge tensor
void fuse_site(hipStream_t s, const double* A, const double* O, int D, int dd, double* a);
void unfuse_env(hipStream_t s, const double* env, const double* A, const double* O, int D, int dd, double* E);
void symmetrize_edge(hipStream_t s, double* T, int x, int Df);
void log_kappa(hipStream_t s, const double* sc, double* out);
void free_energy(hipStream_t s, const double* lk3, const double* lk2, double beta, double* f);
void grad_combine(hipStream_t s, const double* E3, const double* n13, const double* E2,
                  const double* n12, double beta, double* g, int n);
void spectrum_delta(hipStream_t s, double* sv, int n, const double* trace, double* s_old,
                    int* n_old, double* delta);
void trace(hipStream_t s, const double* X, int n, double* out);
void finite_check(hipStream_t s, const double* x, int64_t n, int* flag);
void jacobi_svd(hipStream_t s, const JacobiBatch& jobs, int max_sweeps);
// true when jacobi_svd leaves every job's X unchanged (register kernel)
bool jacobi_reads_only(const JacobiBatch& jobs);
void cholqr(hipStream_t s, const CholBatch& jobs, double shift);
// negate row i of UT (rows x m) and VT (rows x n) when UT's largest-magnitude
// entry in that row is negative
void sign_fix(hipStream_t s, double* UT, double* VT, int rows, int m, int n);

constexpr int kRedBlocks = 256;  // partial-sum slots needed by dot()

}  // namespace ctmk
