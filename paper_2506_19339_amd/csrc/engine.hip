// Host side of the split-CTMRG library: context state, a small contraction
// engine (labelled pairwise contractions -> permute + batched MFMA GEMM), the
// projector construction, one symmetric split-CTMRG iteration, the free-energy
// and gradient contractions, and the C ABI declared in include/ctm.h.
//
// Method (paper passages):
//   * split environment and its D2 relations        Sec. III A, Eq. (Symmetry constraints)
//   * left move: insert, absorb, truncate with six
//     projector pairs, bra-related stage first        Sec. III B
//   * projector pair from rho_B rho_T = U S V:
//     P_B = rho_T V^+ S^-1/2, P_T = S^-1/2 U^+ rho_B  Sec. III C, Eqs. (projector construction)
//   * P1 (one column, two rows), P2 / P3 (1x1 cell),
//     half P4 (two enlarged corners renormalised by
//     P1 and its up/down images), P5 / P6 (two
//     columns, renormalised by P2, P2^R / P3, P3^R)  Appendix, six-projector scheme
//   * convergence on the spectrum of C1C2C3C4/Tr      Sec. III D
//   * f and g from the 3x3 patch                      Eqs. (free energy / gradient expression)
//
// Layout of the stored state (row-major, float64, device):
//   C1[x][y]   (x -> top edge, y -> left edge)      C4[x][y] (x -> left edge, y -> bottom edge)
//   Tk[a][m][b], Ti[a][m][b], Tb[a][m][b]           left-edge chain, a up, m into the bulk, b down
//   the right / bottom edges are the transposes Tb^T, Ti^T, Tk^T (D2 relations), C2 = C4, C3 = C1.
// The bond between Tb and the next Tk (and every corner leg) is "bk", between Tk
// and Ti "ki", between Ti and Tb "ib".
//
// The lower halves of the projector environments are never contracted: the
// 180-degree rotation about the PEPO site (ket <-> bra, left <-> right, up <->
// down) maps each upper half onto the matching lower half, so they are index
// permutations of the upper ones.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <stdexcept>
#include <exception>
#include <string>
#include <mutex>
#include <thread>
#include <vector>

#include "ctm.h"
#include "kernels.h"

namespace {

struct CtmError : std::runtime_error {
    int code;
    CtmError(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(x)                                                                              \
    do {                                                                                       \
        hipError_t e_ = (x);                                                                   \
        if (e_ != hipSuccess)                                                                  \
            throw CtmError(e_ == hipErrorOutOfMemory ? CTM_ENOMEM : CTM_EDEVICE,               \
                           std::string(#x) + ": " + hipGetErrorString(e_));                    \
    } while (0)

#define REQUIRE(cond, msg)                                                                     \
    do {                                                                                       \
        if (!(cond)) throw CtmError(CTM_EINVAL, std::string("internal: ") + (msg));           \
    } while (0)

// ---------------------------------------------------------------------------
// device memory: a chunked bump arena (stack discipline via mark / release)
// ---------------------------------------------------------------------------
class Arena {
    struct Chunk { char* p; size_t cap; };
    std::vector<Chunk> ch_;
    size_t cur_ = 0, off_ = 0;
    bool fixed_ = false;
    std::vector<Chunk> saved_;
    size_t saved_cur_ = 0, saved_off_ = 0;

public:
    struct Mark { size_t cur, off; };
    size_t bytes_held = 0;

    Mark mark() const { return {cur_, off_}; }
    void release(Mark m) { cur_ = m.cur; off_ = m.off; }
    // order of an address inside the arena (chunk, offset), -1 outside it
    int64_t key_of(const void* p) const
    {
        for (size_t c = 0; c < ch_.size(); ++c) {
            const char* b = ch_[c].p;
            if ((const char*)p >= b && (const char*)p < b + ch_[c].cap)
                return ((int64_t)c << 40) + (int64_t)((const char*)p - b);
        }
        return -1;
    }

    // fixed-buffer mode (the allocation-free entry point): every allocation
    // comes from [p, p + cap); running out raises CTM_ENOMEM instead of
    // growing the arena with hipMalloc
    void begin_fixed(char* p, size_t cap)
    {
        saved_.swap(ch_);
        saved_cur_ = cur_;
        saved_off_ = off_;
        ch_.assign(1, Chunk{p, cap});
        cur_ = off_ = 0;
        fixed_ = true;
    }
    void end_fixed()
    {
        if (!fixed_) return;
        saved_.swap(ch_);
        saved_.clear();
        cur_ = saved_cur_;
        off_ = saved_off_;
        fixed_ = false;
    }

    double* alloc(int64_t count)
    {
        size_t bytes = (size_t)std::max<int64_t>(count, 1) * sizeof(double);
        bytes = (bytes + 255) & ~(size_t)255;
        for (;;) {
            if (cur_ < ch_.size()) {
                if (off_ + bytes <= ch_[cur_].cap) {
                    char* r = ch_[cur_].p + off_;
                    off_ += bytes;
                    return (double*)r;
                }
                if (cur_ + 1 < ch_.size()) { ++cur_; off_ = 0; continue; }
            }
            if (fixed_)
                throw CtmError(CTM_ENOMEM, "the temporaries exceed the fixed scratch of the allocation-free "
                                           "call (64 MiB per network)");
            size_t sz = std::max(bytes, (size_t)128 << 20);
            void* p = nullptr;
            hipError_t e = hipMalloc(&p, sz);
            if (e != hipSuccess) throw CtmError(CTM_ENOMEM, "workspace allocation failed");
            ch_.push_back({(char*)p, sz});
            bytes_held += sz;
            cur_ = ch_.size() - 1;
            off_ = 0;
        }
    }

    void free_all()
    {
        for (auto& c : ch_) (void)hipFree(c.p);
        ch_.clear();
        cur_ = off_ = 0;
        bytes_held = 0;
    }
};

// ---------------------------------------------------------------------------
// dense tensor handle (device buffer + row-major dims)
// ---------------------------------------------------------------------------
constexpr int kMaxRank = 12;

// d[] are the logical dimensions (the order the caller's labels refer to).
// A contraction result whose requested label order differs from the GEMM's
// natural output order is kept in the natural order (lazy): storage axis s
// holds logical axis sp[s].  The next contraction folds that order into its
// own operand permutation, so the two permutes become one; view(), mm() and
// raw-pointer consumers materialise first.
struct Tn {
    double* p = nullptr;
    int r = 0;
    int64_t d[kMaxRank] = {0};
    bool lazy = false;
    int8_t sp[kMaxRank] = {0};
    int64_t n() const
    {
        int64_t s = 1;
        for (int i = 0; i < r; ++i) s *= d[i];
        return s;
    }
};

static Tn make_tn(double* p, std::initializer_list<int64_t> dims)
{
    Tn t;
    t.p = p;
    for (int64_t v : dims) t.d[t.r++] = v;
    return t;
}

struct Projector {
    Tn PT;   // k x trunc
    Tn PB;   // trunc x k
    int k = 0;
};

// one network (triple layer: PEPO d = 2; double layer: delta PEPO, d = 1)
struct Net {
    int d = 2;
    double* O = nullptr;             // [2][2][d][d][d][d]
    double *C1 = nullptr, *C4 = nullptr, *Tk = nullptr, *Ti = nullptr, *Tb = nullptr;
    int64_t xbk = 1, xki = 1, xib = 1;
    // the corner bond has reached chi since the product boundary; before that
    // (growth phase) rank-deficient projector environments are not trusted
    bool grown = false;
    double* s_old = nullptr;         // previous normalised spectrum
    int* n_old = nullptr;
    double* delta = nullptr;         // last spectrum change
    double* sc = nullptr;            // scalars: n1 n2h n2v n0 | lk flag | tr
    double* E = nullptr;             // bra environment, 2 D^4
    double* sv = nullptr;            // spectrum buffer
    // reduced method (CTM_FLAG_REDUCED): corner in C1, edge T [chi][Df][chi],
    // fused site tensor a [Df]^4 with Df = D d D
    int64_t Df = 0;
    double* a = nullptr;
    double* Tf = nullptr;
};

// per-kernel-class launch statistics (CTM_FLAG_PROFILE): HIP events on the
// context stream around every launch, algorithmic flops per launch
struct KStat {
    int64_t launches = 0;
    double flops = 0.0;
    double bytes = 0.0;              // algorithmic operand + result bytes
    double ms = 0.0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    bool owns_events = true;         // false: the events belong to another class
};

constexpr int kJacobiExact = 64;    // exact Jacobi SVD when min(m, n) <= this
constexpr int64_t kJacobiExactArea = 18432;  // ... and m * n <= this (LDS-resident)
constexpr int kOversample = 16;
constexpr int kWarmPowerIters = 4;  // power steps when every subspace starts from last move's basis
                                    // (the iteration continues across moves).  At D = 5, chi = 100
                                    // the converged f is 2.7e-10 from the oracle's with 2 steps,
                                    // 7e-12 with 4 (6 % more time), 3e-13 with 8 (19 %)
constexpr int kWarmPowerItersEarly = 2;  // ... while the spectrum still moves by more than
constexpr double kWarmTight = 1e-6;      // kWarmTight per move (the state is not final yet)
constexpr int kColdPowerIters = 4;  // power steps from random normals (the moves before the
                                    // spectrum change drops below kWarmGate; ten made D = 5,
                                    // chi = 100 7 % slower at the same converged f)
constexpr int kColdPowerItersReduced = 10;  // the reduced method starts every move cold
// the same when the Rayleigh-Ritz core is less than 1.25 kk wide (kk > 112):
// at D = 6, chi = 144 (core 160) ten cold steps resolve the early moves'
// projectors to ~1e-6 only (f 2e-5 off the oracle after six moves), forty to
// rounding
constexpr int kColdPowerItersThin = 40;
constexpr int kWarmPowerItersThin = 8;
constexpr double kWarmGate = 1e-3;  // spectrum change per move below which the last bases are reused
constexpr int64_t kCoreMax = 128;   // largest Rayleigh-Ritz core (register-resident Jacobi)
// relative pseudo-inverse cutoff of S^1/2: singular values of rho_B rho_T below
// 1e-8 of the largest are dropped.  The subspace factorisation squares the
// spectrum in its Gram steps, so 1e-8 is the smallest relative singular value
// it resolves in FP64.
constexpr double kDefaultCutoff = 1e-8;
constexpr int kJacobiSweeps = 40;
constexpr int kWarmJacobiSweeps = 3;   // Rayleigh-Ritz core sweeps of a settling warm move
constexpr int64_t kCholRegRows = 128;  // rows of the register-resident Cholesky-QR kernel
constexpr int kFillPowerIters = 40; // power steps of the growth-phase Gram factorisations
constexpr int kMaxBatch = 16;       // projectors factorised together
constexpr int kMaxIterateBatch = 64; // contexts advanced by one ctm_iterate_batch call
// spectrum-change floors of the reduced-precision phases (rounding noise of
// the FP32 / BF16 products keeps the change of the normalised spectrum above
// roughly these values)
constexpr double kLpTolFp32 = 1e-6;
constexpr double kLpTolBf16 = 1e-2;
// pseudo-inverse cutoffs of the reduced-precision phases (above the relative
// rounding level of rho_B rho_T formed from FP32 / BF16 products)
constexpr double kLpCutFp32 = 1e-7;
constexpr double kLpCutBf16 = 1e-3;

}  // namespace

// ---------------------------------------------------------------------------
// one worker per network: its own stream, workspace arena, scratch and launch
// statistics, so that the triple- and double-layer networks (independent until
// f is formed) run concurrently, each from its own host thread.
// ---------------------------------------------------------------------------
struct Worker {
    ctm_config cfg{};
    int D = 0;
    const double* A = nullptr;       // D4-projected A, owned by the context
    hipStream_t st = nullptr;        // created by the context (default priority)
    hipStream_t st_side = nullptr;   // side work (convergence spectrum): the caller's stream
    hipEvent_t ev_side_fork = nullptr, ev_side_done = nullptr;
    bool on_side = false, side_pending = false;
    bool side_ok = true;             // side work allowed in this call (one context at a time)
    Arena ws;
    std::vector<void*> owned;        // persistent allocations of this worker
    double* part = nullptr;          // reduction partials
    double* scal = nullptr;          // scratch scalars
    int* icount = nullptr;           // device ints for rank read-back
    double* gws = nullptr;           // split-K partial products of the GEMMs
    int64_t gws_cap = 0;
    uint64_t svd_calls = 0;
    int64_t exact_min = kJacobiExact, exact_area = kJacobiExactArea;
    int64_t trace_perm = 0;          // testing aid: log permutes of at least this many elements
    bool trace_gemm = false;         // testing aid: log GEMM shapes
    bool no_group = false;           // testing aid: one launch per product in mm_group
    bool trace_ranks = false;        // testing aid: log the kept rank of every projector
    bool trace_sweeps = false;       // testing aid: log the sweeps of every Jacobi job (profile mode)
    bool warm_starts = true;         // keep each slot's Ritz basis for the next move
    bool reduced = false;            // reduced (unsplit) C4v CTMRG on the fused site tensor
    bool full_p4 = false;            // projector 4 from the 2x2 block (default: the half construction)
    double last_delta = 1.0;         // spectrum change of this network's last move (host copy)
    bool final_phase = false;        // the change has been below kWarmTight: every move runs the
                                     // factorisations to convergence from then on (no switching
                                     // back and forth at the threshold)
    void note_delta(double d)
    {
        last_delta = d;
        if (d < kWarmTight) final_phase = true;
    }
    void restart()
    {
        last_delta = 1.0;
        final_phase = false;
    }
    int bulk = CTM_FP64;             // precision of the bulk contractions in the current phase
    double lp_cut = 0.0;             // testing aid: cutoff of the reduced-precision phase
    int cur = CTM_FP64;              // precision of the GEMMs issued now
    bool profiling = false;
    KStat kstat[6];                  // [0] FP64 GEMM, [1] Jacobi SVD, [2] Cholesky QR, [3] FP32/BF16 GEMM,
                                     // [4] split-K reduction, [5] the part of [0] issued by the
                                     // factorisations (subspace iteration, Cholesky QR, Rayleigh-Ritz,
                                     // projector assembly; shares [0]'s events)
    int factor_depth = 0;            // > 0 while a factorisation issues GEMMs
    struct FactorScope {
        Worker& w;
        explicit FactorScope(Worker& x) : w(x) { ++w.factor_depth; }
        ~FactorScope() { --w.factor_depth; }
    };
    std::vector<hipEvent_t> ev_pool;
    // profile mode: sweeps of every Jacobi job, for its algorithmic flop count
    static constexpr int kSweepSlots = 4096;
    int* sweeps_dev = nullptr;
    struct JobShape { int64_t m, n; bool v; };
    std::vector<JobShape> sweep_jobs;

    void setup(const ctm_config& c, int d_bond, const double* a)
    {
        cfg = c;
        D = d_bond;
        A = a;
        profiling = (c.flags & CTM_FLAG_PROFILE) != 0;
        kstat[5].owns_events = false;
        reduced = (c.flags & CTM_FLAG_REDUCED) != 0;
        full_p4 = (c.flags & CTM_FLAG_FULL_P4) != 0;
        // the reduced method's enlarged corner (chi D^2 d wide, cut in a flat
        // part of its spectrum) needs the full power iteration every move: with
        // two warm steps its spectrum change stalls near 1e-7 (D = 5, chi = 100)
        if (reduced) warm_starts = false;
        HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&ev_side_fork, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&ev_side_done, hipEventDisableTiming));
        part = keep(ctmk::kRedBlocks);
        scal = keep(16);
        icount = (int*)keep(kMaxBatch);
        gws_cap = (int64_t)1 << 22;   // 32 MiB
        gws = keep(gws_cap);
        if (profiling) sweeps_dev = (int*)keep(kSweepSlots / 2);
    }
    void release()
    {
        if (st) (void)hipStreamSynchronize(st);
        ws.free_all();
        for (void* p : owned) (void)hipFree(p);
        owned.clear();
        for (auto& k : kstat) {
            if (k.owns_events)
                for (auto& pr : k.pending) {
                    (void)hipEventDestroy(pr.first);
                    (void)hipEventDestroy(pr.second);
                }
            k.pending.clear();
        }
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
        ev_pool.clear();
        if (ev_side_fork) (void)hipEventDestroy(ev_side_fork);
        if (ev_side_done) (void)hipEventDestroy(ev_side_done);
        st_side = nullptr;
        ev_side_fork = ev_side_done = nullptr;
        if (st) (void)hipStreamDestroy(st);
        st = nullptr;
    }

    // Work enqueued between side_begin and side_end goes to the side stream
    // (after everything enqueued on the worker stream so far) and runs
    // concurrently with what the worker stream does next, until side_wait.
    // The side stream is the caller's stream, idle between the fork and the
    // join of a call, so that a context uses three streams in all (a process
    // gets four hardware queues by default; two more streams would share
    // queues with the worker streams and serialise with them).  The side work
    // must not use the split-K workspace or the reduction scratch of the
    // worker stream.  In profile mode everything stays on the worker stream.
    void side_begin()
    {
        if (profiling || !side_ok) return;
        HIPCHK(hipEventRecord(ev_side_fork, st));
        HIPCHK(hipStreamWaitEvent(st_side, ev_side_fork, 0));
        std::swap(st, st_side);
        on_side = true;
    }
    void side_end()
    {
        if (!on_side) return;
        HIPCHK(hipEventRecord(ev_side_done, st));
        std::swap(st, st_side);
        on_side = false;
        side_pending = true;
    }
    void side_wait()
    {
        if (!side_pending) return;
        HIPCHK(hipStreamWaitEvent(st, ev_side_done, 0));
        side_pending = false;
    }

    hipEvent_t ev_get()
    {
        if (ev_pool.empty()) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            return e;
        }
        hipEvent_t e = ev_pool.back();
        ev_pool.pop_back();
        return e;
    }
    hipEvent_t prof_begin()
    {
        if (!profiling) return nullptr;
        hipEvent_t a = ev_get();
        HIPCHK(hipEventRecord(a, st));
        return a;
    }
    void prof_end(int cls, hipEvent_t a, double flops)
    {
        if (!profiling) return;
        hipEvent_t b = ev_get();
        HIPCHK(hipEventRecord(b, st));
        kstat[cls].launches += 1;
        kstat[cls].flops += flops;
        kstat[cls].pending.push_back({a, b});
    }
    // one-sided Jacobi, per sweep and column pair: three dot products (6m
    // flops) and the rotation of the two columns of X (6m) and of V (6n)
    void collect_sweeps()
    {
        if (sweep_jobs.empty()) return;
        std::vector<int> sw(sweep_jobs.size());
        HIPCHK(hipMemcpyAsync(sw.data(), sweeps_dev, sw.size() * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (size_t i = 0; i < sw.size(); ++i) {
            const JobShape& j = sweep_jobs[i];
            if (trace_sweeps)
                std::fprintf(stderr, "sweeps %lld %lld %d %d\n", (long long)j.m, (long long)j.n, (int)j.v, sw[i]);
            kstat[1].flops += (double)sw[i] * 0.5 * (double)j.n * (double)(j.n - 1) *
                              (12.0 * (double)j.m + (j.v ? 6.0 * (double)j.n : 0.0));
        }
        sweep_jobs.clear();
    }
    void prof_collect()
    {
        HIPCHK(hipStreamSynchronize(st));
        collect_sweeps();
        for (auto& k : kstat) {
            for (auto& pr : k.pending) {
                float t = 0.f;
                HIPCHK(hipEventElapsedTime(&t, pr.first, pr.second));
                k.ms += t;
                if (!k.owns_events) continue;
                ev_pool.push_back(pr.first);
                ev_pool.push_back(pr.second);
            }
            k.pending.clear();
        }
    }
    void gemm(bool ta, bool tb, int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
              int64_t sA, const double* B, int64_t ldb, int64_t sB, double* C, int64_t ldc,
              int64_t sC, int64_t nb, double alpha = 1.0, double beta = 0.0)
    {
        if (trace_gemm)
            std::fprintf(stderr, "gemm %lld %lld %lld %lld %d %d %d\n", (long long)M, (long long)N, (long long)K,
                         (long long)nb, (int)ta, (int)tb, cur);
        hipEvent_t e = prof_begin();
        hipEvent_t mid = profiling ? ev_get() : nullptr;
        if (cur == CTM_FP64)
            ctmk::gemm_f64(st, ta, tb, (int)M, (int)N, (int)K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC,
                           (int)nb, gws, gws_cap, mid);
        else
            ctmk::gemm_lp(st, cur, ta, tb, (int)M, (int)N, (int)K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC,
                          (int)nb, gws, gws_cap, mid);
        if (profiling)
            prof_gemm(e, mid, 2.0 * (double)M * (double)N * (double)K * (double)nb,
                      8.0 * ((double)M * K + (double)K * N + (double)M * N) * (double)nb,
                      beta == 0.0 && ctmk::gemm_split_plan((int)M, (int)N, (int)K, (int)nb, gws_cap) > 1);
    }
    // profile mode: product kernel [e, mid], split-K reduction [mid, end]
    void prof_gemm(hipEvent_t e, hipEvent_t mid, double flops, double bytes, bool split)
    {
        const int cls = cur == CTM_FP64 ? 0 : 3;
        kstat[cls].launches += 1;
        kstat[cls].flops += flops;
        kstat[cls].bytes += bytes;
        kstat[cls].pending.push_back({e, mid});
        if (cls == 0 && factor_depth > 0) {
            kstat[5].launches += 1;
            kstat[5].flops += flops;
            kstat[5].bytes += bytes;
            kstat[5].pending.push_back({e, mid});
        }
        hipEvent_t end = ev_get();
        HIPCHK(hipEventRecord(end, st));
        if (split) kstat[4].launches += 1;
        kstat[4].pending.push_back({mid, end});
    }

    // GEMM precision for the lifetime of the guard
    struct Prec {
        Worker& w;
        int old;
        Prec(Worker& w_, int p) : w(w_), old(w_.cur) { w.cur = p; }
        ~Prec() { w.cur = old; }
    };

    // ---------------- allocation helpers
    double* keep(int64_t count)
    {
        void* p = nullptr;
        HIPCHK(hipMalloc(&p, (size_t)std::max<int64_t>(count, 1) * sizeof(double)));
        owned.push_back(p);
        return (double*)p;
    }
    Tn tmp(std::initializer_list<int64_t> dims)
    {
        Tn t;
        for (int64_t v : dims) t.d[t.r++] = v;
        t.p = ws.alloc(t.n());
        return t;
    }
    Tn tmp_dims(const int64_t* dims, int r)
    {
        Tn t;
        t.r = r;
        for (int i = 0; i < r; ++i) t.d[i] = dims[i];
        t.p = ws.alloc(t.n());
        return t;
    }

    // ---------------- contraction engine
    // permute(A, "abc->cab")
    Tn perm(const Tn& A, const char* spec)
    {
        std::string s(spec);
        const size_t ar = s.find("->");
        REQUIRE(ar != std::string::npos, spec);
        const std::string li = s.substr(0, ar), lo = s.substr(ar + 2);
        REQUIRE((int)li.size() == A.r && lo.size() == li.size(), spec);
        std::string sl;
        const Tn As = storage(A, li, sl);
        return permute_labels(As, sl, lo);
    }

    // the stored array of A with its dims in storage order, and the caller's
    // labels li rearranged to that order
    static Tn storage(const Tn& A, const std::string& li, std::string& sl)
    {
        Tn S = A;
        S.lazy = false;
        sl = li;
        if (!A.lazy) return S;
        for (int k = 0; k < A.r; ++k) {
            S.d[k] = A.d[A.sp[k]];
            sl[k] = li[A.sp[k]];
        }
        return S;
    }

    // A in its logical order (a permute if A is lazy)
    Tn mat(const Tn& A)
    {
        if (!A.lazy) return A;
        std::string li;
        for (int k = 0; k < A.r; ++k) li += (char)('a' + k);
        std::string sl;
        const Tn As = storage(A, li, sl);
        return permute_labels(As, sl, li);
    }

    Tn permute_labels(const Tn& A, const std::string& li, const std::string& lo)
    {
        if (li == lo) return A;
        REQUIRE(A.r <= kMaxRank, "rank too large");
        int64_t istride[kMaxRank];
        int64_t acc = 1;
        for (int k = A.r - 1; k >= 0; --k) { istride[k] = acc; acc *= A.d[k]; }
        ctmk::PermDesc pd{};
        pd.rank = A.r;
        int64_t od[kMaxRank];
        for (int k = 0; k < A.r; ++k) {
            const size_t pos = li.find(lo[k]);
            REQUIRE(pos != std::string::npos, "permute label");
            od[k] = A.d[pos];
            pd.od[k] = od[k];
            pd.is[k] = istride[pos];
        }
        Tn out = tmp_dims(od, A.r);
        if (trace_perm && out.n() >= trace_perm) {
            std::fprintf(stderr, "permute %s->%s %lld [", li.c_str(), lo.c_str(), (long long)out.n());
            for (int k = 0; k < A.r; ++k) std::fprintf(stderr, k ? " %lld" : "%lld", (long long)A.d[k]);
            std::fprintf(stderr, "]\n");
        }
        ctmk::permute(st, A.p, out.p, pd, out.n());
        return out;
    }

    Tn view(const Tn& A0, std::initializer_list<int64_t> dims)
    {
        const Tn A = mat(A0);
        Tn t;
        t.p = A.p;
        for (int64_t v : dims) t.d[t.r++] = v;
        if (t.n() != A.n()) throw CtmError(CTM_EINVAL, "internal: view size mismatch");
        return t;
    }

    // Keeps the listed tensors and returns everything else allocated since m
    // to the arena, so that a chain of contractions holds its intermediates
    // only while it runs.  The distinct buffers of the kept tensors are copied
    // above the arena's top, in arena order, and then down from m: a bump
    // allocator places a subset of its earlier allocations, taken in order,
    // no higher than they were, so no copy overlaps its source.  Should a
    // placement still reach a copy above the top (chunk boundaries), the
    // tensors stay in their copies above the top instead.  Not used while
    // work is on the side stream.
    void settle(Arena::Mark m, std::initializer_list<Tn*> keep)
    {
        REQUIRE(!on_side, "settle during side work");
        REQUIRE(keep.size() <= 8, "settle: too many tensors");
        struct Buf {
            double* src;
            int64_t n, key;
            double *up, *q;
        };
        Buf b[8];
        int nb = 0;
        for (Tn* t : keep) {
            int j = 0;
            while (j < nb && b[j].src != t->p) ++j;
            if (j == nb) b[nb++] = Buf{t->p, t->n(), ws.key_of(t->p), nullptr, nullptr};
            else b[j].n = std::max(b[j].n, t->n());
        }
        std::sort(b, b + nb, [](const Buf& x, const Buf& y) { return x.key < y.key; });
        // all bounces up in one launch (the copies land above everything live)
        static_assert(ctmk::kMaxCopyBatch >= 8, "one copy batch per settle");
        ctmk::CopyBatch up{};
        for (int j = 0; j < nb; ++j) {
            b[j].up = ws.alloc(b[j].n);
            up.src[up.cnt] = b[j].src;
            up.dst[up.cnt] = b[j].up;
            up.n[up.cnt++] = b[j].n;
        }
        ctmk::copy_batch(st, up);
        const Arena::Mark above = ws.mark();
        ws.release(m);
        // ... and all copies down in one launch, provided no final place
        // overlaps a bounce (else the bounces stay where they are)
        bool ok = true;
        ctmk::CopyBatch down{};
        for (int j = 0; j < nb && ok; ++j) {
            double* q = ws.alloc(b[j].n);
            for (int i = 0; i < nb; ++i)
                if (q < b[i].up + b[i].n && b[i].up < q + b[j].n) ok = false;
            if (ok) {
                down.src[down.cnt] = b[j].up;
                down.dst[down.cnt] = q;
                down.n[down.cnt++] = b[j].n;
                b[j].q = q;
            }
        }
        if (ok) {
            ctmk::copy_batch(st, down);
        } else {
            ws.release(above);
            for (int j = 0; j < nb; ++j) b[j].q = b[j].up;
        }
        for (Tn* t : keep)
            for (int j = 0; j < nb; ++j)
                if (b[j].src == t->p) {
                    t->p = b[j].q;
                    break;
                }
    }

    // ctr("ab,bc->ac", A, B): labelled pairwise contraction.  Labels shared by
    // A, B and the output are batch labels; shared by A and B only are summed.
    Tn ctr(const char* spec, const Tn& A0, const Tn& B0)
    {
        std::string s(spec);
        const size_t cm = s.find(','), ar = s.find("->");
        REQUIRE(cm != std::string::npos && ar != std::string::npos, spec);
        const std::string la0 = s.substr(0, cm), lb0 = s.substr(cm + 1, ar - cm - 1), lo = s.substr(ar + 2);
        REQUIRE((int)la0.size() == A0.r && (int)lb0.size() == B0.r, spec);
        std::string la, lb;
        const Tn A = storage(A0, la0, la), B = storage(B0, lb0, lb);
        int64_t dim[128];
        for (int i = 0; i < 128; ++i) dim[i] = -1;
        for (int i = 0; i < A.r; ++i) dim[(int)la[i]] = A.d[i];
        for (int i = 0; i < B.r; ++i) {
            const int c = (int)lb[i];
            REQUIRE(dim[c] < 0 || dim[c] == B.d[i], std::string("dimension mismatch in ") + spec);
            dim[c] = B.d[i];
        }
        std::string bt, con, fa, fb;
        for (char c : la) {
            const bool inB = lb.find(c) != std::string::npos, inO = lo.find(c) != std::string::npos;
            if (inB && inO) bt += c;
            else if (inB) con += c;
            else if (inO) fa += c;
            else REQUIRE(false, std::string("label summed out of one operand in ") + spec);
        }
        for (char c : lb)
            if (la.find(c) == std::string::npos) {
                REQUIRE(lo.find(c) != std::string::npos, spec);
                fb += c;
            }
        REQUIRE(lo.size() == bt.size() + fa.size() + fb.size(), spec);
        // contracted order: A's if A needs no permute, else B's if B needs none
        auto in_order = [](const std::string& lab, const std::string& sub) {
            std::string r;
            for (char c : lab)
                if (sub.find(c) != std::string::npos) r += c;
            return r;
        };
        std::string conA = in_order(la, con), conB = in_order(lb, con);
        std::string fbB = in_order(lb, fb);
        const std::string faA = in_order(la, fa);
        bool tA = false, tB = false, okA = false, okB = false;
        std::string cord = conA;
        if (la == bt + faA + conA) { okA = true; tA = false; }
        else if (la == bt + conA + faA) { okA = true; tA = true; }
        if (!okA) {
            const std::string btB = in_order(lb, bt);
            if (btB == bt && (lb == bt + conB + fbB || lb == bt + fbB + conB)) cord = conB;
        }
        if (lb == bt + cord + fbB) { okB = true; tB = false; }
        else if (lb == bt + fbB + cord) { okB = true; tB = true; }
        int64_t M = 1, N = 1, K = 1, nb = 1;
        for (char c : faA) M *= dim[(int)c];
        for (char c : fbB) N *= dim[(int)c];
        for (char c : cord) K *= dim[(int)c];
        for (char c : bt) nb *= dim[(int)c];
        const std::string nat = bt + faA + fbB;
        REQUIRE((int)nat.size() <= kMaxRank, "rank too large");
        int64_t od[kMaxRank];
        int orank = 0;
        for (char c : nat) od[orank++] = dim[(int)c];
        // the result first, then the transposed operands above it, which are
        // returned to the arena once the product is enqueued (later work on
        // this stream reuses them in stream order; side work keeps them)
        Tn C = tmp_dims(od, orank);
        const Arena::Mark opm = ws.mark();
        Tn Ao = A, Bo = B;
        if (!okA) { Ao = permute_labels(A, la, bt + faA + cord); tA = false; }
        if (!okB) { Bo = permute_labels(B, lb, bt + cord + fbB); tB = false; }
        if (M == 1 && N == 1 && nb == 1) {
            ctmk::dot(st, Ao.p, Bo.p, K, C.p, part, 0);
        } else {
            REQUIRE(M < INT_MAX && N < INT_MAX && K < INT_MAX, "GEMM too large");
            gemm(tA, tB, M, N, K, Ao.p, tA ? M : K, M * K, Bo.p, tB ? K : N, K * N,
                 C.p, N, M * N, nb);
        }
        if (!on_side) ws.release(opm);
        if (lo == nat) return C;
        // keep the natural order; record where each logical axis is stored
        Tn L = C;
        L.lazy = true;
        for (int i = 0; i < orank; ++i) L.d[i] = dim[(int)lo[i]];
        for (int k = 0; k < orank; ++k) L.sp[k] = (int8_t)lo.find(nat[k]);
        return L;
    }

    // ---------------- dense linear algebra on row-major matrices
    // C[M][N] = op(A) op(B)
    Tn mm(const Tn& A0, bool ta, const Tn& B0, bool tb)
    {
        const Tn A = mat(A0), B = mat(B0);
        const int64_t M = ta ? A.d[1] : A.d[0], K = ta ? A.d[0] : A.d[1];
        const int64_t K2 = tb ? B.d[1] : B.d[0], N = tb ? B.d[0] : B.d[1];
        REQUIRE(A.r == 2 && B.r == 2 && K == K2, "mm shapes");
        Tn C = tmp({M, N});
        gemm(ta, tb, M, N, K, A.p, A.d[1], 0, B.p, B.d[1], 0, C.p, N, 0, 1);
        return C;
    }

    // C_i = op(A_i) op(B_i) for every i of the lists, the products of up to
    // kMaxGemmGroup problems in one launch (FP64 GEMMs; in a reduced-precision
    // phase one launch per problem)
    std::vector<Tn> mm_group(const std::vector<Tn>& A0, bool ta, const std::vector<Tn>& B0, bool tb)
    {
        REQUIRE(A0.size() == B0.size(), "mm_group: list sizes");
        std::vector<Tn> C(A0.size());
        if (cur != CTM_FP64 || A0.size() == 1 || no_group) {
            for (size_t i = 0; i < A0.size(); ++i) C[i] = mm(A0[i], ta, B0[i], tb);
            return C;
        }
        for (size_t b0 = 0; b0 < A0.size(); b0 += ctmk::kMaxGemmGroup) {
            const size_t b1 = std::min(A0.size(), b0 + (size_t)ctmk::kMaxGemmGroup);
            ctmk::GemmProb pr[ctmk::kMaxGemmGroup];
            int np = 0;
            double fl = 0.0, by = 0.0;
            for (size_t i = b0; i < b1; ++i) {
                const Tn A = mat(A0[i]), B = mat(B0[i]);
                const int64_t M = ta ? A.d[1] : A.d[0], K = ta ? A.d[0] : A.d[1];
                const int64_t K2 = tb ? B.d[1] : B.d[0], N = tb ? B.d[0] : B.d[1];
                REQUIRE(A.r == 2 && B.r == 2 && K == K2, "mm shapes");
                C[i] = tmp({M, N});
                pr[np++] = ctmk::GemmProb{A.p, B.p, C[i].p, (int)M, (int)N, (int)K, A.d[1], B.d[1], N};
                fl += 2.0 * (double)M * (double)N * (double)K;
                by += 8.0 * ((double)M * K + (double)K * N + (double)M * N);
                if (trace_gemm)
                    std::fprintf(stderr, "gemm %lld %lld %lld group %d %d\n", (long long)M, (long long)N,
                                 (long long)K, (int)ta, (int)tb);
            }
            hipEvent_t e = prof_begin();
            hipEvent_t mid = profiling ? ev_get() : nullptr;
            ctmk::gemm_f64_group(st, ta, tb, pr, np, 1.0, gws, gws_cap, mid);
            if (profiling) prof_gemm(e, mid, fl, by, ctmk::gemm_group_splits(pr, np, gws_cap) > 0);
        }
        return C;
    }

    // ---------------- batched factorisations
    // One-sided Jacobi SVDs of matrices given column-major (m rows, n columns),
    // all problems of the list in one launch per group of kMaxJacobiBatch:
    // X = U S V^T with U (n x m: row j = column j), V (n x n), S (n, descending).
    struct JReq {
        const double* X;
        int64_t m, n;
        bool want_v;
        Tn U, V, S;
    };
    void jacobi_batch(std::vector<JReq>& rq, int max_sweeps = kJacobiSweeps)
    {
        for (size_t b0 = 0; b0 < rq.size(); b0 += ctmk::kMaxJacobiBatch) {
            ctmk::JacobiBatch jb{};
            const size_t b1 = std::min(rq.size(), b0 + (size_t)ctmk::kMaxJacobiBatch);
            for (size_t i = b0; i < b1; ++i) {
                JReq& r = rq[i];
                REQUIRE(r.n <= 1024, "Jacobi: too many columns");
                Tn W = tmp({r.n, r.n});
                r.U = tmp({r.n, r.m});
                r.V = tmp({r.n, r.n});
                r.S = tmp({r.n});
                int* sw = nullptr;
                if (profiling) {
                    if ((int)sweep_jobs.size() == kSweepSlots) collect_sweeps();
                    sw = sweeps_dev + sweep_jobs.size();
                    sweep_jobs.push_back({r.m, r.n, r.want_v});
                }
                jb.job[jb.n++] = ctmk::JacobiJob{const_cast<double*>(r.X), W.p, r.U.p, r.V.p, r.S.p, (int)r.m,
                                                 (int)r.n, r.want_v ? 1 : 0, sw};
            }
            // the kernels for larger problems rotate X in place: they get copies
            if (!ctmk::jacobi_reads_only(jb))
                for (int t = 0; t < jb.n; ++t) {
                    ctmk::JacobiJob& j = jb.job[t];
                    Tn X = tmp({(int64_t)j.n, (int64_t)j.m});
                    ctmk::copy(st, j.X, X.p, (int64_t)j.m * j.n);
                    j.X = X.p;
                }
            hipEvent_t e = prof_begin();
            ctmk::jacobi_svd(st, jb, max_sweeps);
            prof_end(1, e, 0.0);
        }
    }

    // one shifted Cholesky QR pass on the rows of every Y (k x L) of the list:
    // G = Y Y^T, T = L^-1 D with L L^T = D G D + shift I, D = diag(G)^-1/2;
    // Y <- T Y.  The factors of all problems are built in one launch.
    void cholqr_pass(std::vector<Tn>& Ys)
    {
        for (const Tn& y : Ys)
            if (y.d[0] > kCholRegRows) {
                cholqr_pass_blocked(Ys);
                return;
            }
        std::vector<Tn> Ts(Ys.size());
        for (size_t b0 = 0; b0 < Ys.size(); b0 += ctmk::kMaxJacobiBatch) {
            const size_t b1 = std::min(Ys.size(), b0 + (size_t)ctmk::kMaxJacobiBatch);
            ctmk::CholBatch cb{};
            double fl = 0.0;
            const std::vector<Tn> Yb(Ys.begin() + b0, Ys.begin() + b1);
            const std::vector<Tn> Gs = mm_group(Yb, false, Yb, true);   // Gram matrices
            for (size_t i = b0; i < b1; ++i) {
                const int64_t k = Ys[i].d[0];
                fl += 2.0 / 3.0 * (double)k * (double)k * (double)k;   // elimination: 2 sum_i i^2
                Ts[i] = tmp({k, k});
                Tn work = tmp({2 * k});
                cb.job[cb.n++] = ctmk::CholJob{Gs[i - b0].p, work.p, Ts[i].p, (int)k};
            }
            hipEvent_t e = prof_begin();
            ctmk::cholqr(st, cb, 1e-14);
            prof_end(2, e, fl);
        }
        Ys = mm_group(Ts, false, Ys, false);
    }

    // Y with more than kCholRegRows rows: the head H (first kCholRegRows
    // rows) by one Cholesky-QR pass (-> Q1), the tail R projected off it,
    // R <- R - (R Q1^T) Q1, and then given a pass of its own (recursively):
    // block classical Gram-Schmidt whose factorisations all fit the
    // register-resident kernel.  Two passes (orth) re-project the tail, which
    // restores the orthogonality between the blocks.
    void cholqr_pass_blocked(std::vector<Tn>& Ys)
    {
        const size_t nb = Ys.size();
        std::vector<Tn> H(nb), R;
        std::vector<size_t> r_of;
        for (size_t i = 0; i < nb; ++i) {
            const Tn Y = mat(Ys[i]);
            const int64_t k = Y.d[0], n = Y.d[1], k1 = std::min<int64_t>(k, kCholRegRows);
            H[i] = make_tn(Y.p, {k1, n});
            if (k > k1) {
                R.push_back(make_tn(Y.p + k1 * n, {k - k1, n}));
                r_of.push_back(i);
            }
        }
        cholqr_pass(H);
        std::vector<Tn> Hr(R.size());
        for (size_t j = 0; j < R.size(); ++j) Hr[j] = H[r_of[j]];
        const std::vector<Tn> C = mm_group(R, false, Hr, true);        // R Q1^T
        for (size_t j = 0; j < R.size(); ++j) {
            const int64_t k2 = R[j].d[0], n = R[j].d[1], k1 = Hr[j].d[0];
            gemm(false, false, k2, n, k1, C[j].p, k1, 0, Hr[j].p, n, 0, R[j].p, n, 0, 1, -1.0, 1.0);
        }
        cholqr_pass(R);
        for (size_t i = 0; i < nb; ++i) Ys[i] = H[i];
        for (size_t j = 0; j < R.size(); ++j) {
            const size_t i = r_of[j];
            const int64_t k1 = H[i].d[0], k2 = R[j].d[0], n = H[i].d[1];
            Tn Q = tmp({k1 + k2, n});
            ctmk::copy(st, H[i].p, Q.p, k1 * n);
            ctmk::copy(st, R[j].p, Q.p + k1 * n, k2 * n);
            Ys[i] = Q;
        }
    }

    // rows of every Y -> orthonormal rows spanning the same space (shifted
    // Cholesky QR, twice).  Small directions are kept (the shift bounds their
    // amplification) so that the power steps can refine them.
    void orth(std::vector<Tn>& Ys)
    {
        cholqr_pass(Ys);
        cholqr_pass(Ys);
    }

    // top-kk singular triplets of each M (m x n row-major): UT (kk x m), S (kk),
    // VT (kk x n).  min(m, n) <= exact_min or m n <= exact_area: exact one-sided
    // Jacobi SVD.  Otherwise block subspace iteration on M^T M (k vectors,
    // k >= kk + oversampling) from counter-based normals, and a Rayleigh-Ritz
    // step whose small core Q^T M P is factorised by Jacobi.  All problems of
    // the list advance together so that every factorisation kernel serves all
    // of them in one launch.
    struct SvdReq {
        Tn M;
        int64_t kk;
        int slot = -1;               // projector slot (warm start), -1: none
        Tn UT, S, VT;
    };

    // right singular vectors kept by each projector slot in the last move, the
    // start of the next subspace iteration of that slot (with a fixed sign
    // convention the bond gauge, and with it rho_B rho_T, settles as the
    // environment converges)
    struct Warm {
        double* V = nullptr;
        int64_t cap = 0, kk = 0, n = 0;
        bool valid = false;
    };
    Warm warm[6];
    // power: power steps of the subspace iteration (0: the schedule below)
    void svd_batch(std::vector<SvdReq>& rq, int power = 0)
    {
        FactorScope fs(*this);
        Prec fp64(*this, CTM_FP64);   // factorisations stay FP64 in every precision form
        std::vector<JReq> ex;
        std::vector<size_t> ex_of, rnd;
        std::vector<bool> ex_t;
        for (size_t i = 0; i < rq.size(); ++i) {
            const Tn& M = rq[i].M;
            const int64_t m = M.d[0], n = M.d[1], mn = std::min(m, n);
            if (mn <= exact_min || m * n <= exact_area) {
                if (m <= n) {
                    // M row-major == M^T column-major (n rows, m columns)
                    ex.push_back(JReq{M.p, n, m, true, {}, {}, {}});
                    ex_t.push_back(false);
                } else {
                    Tn Mt = perm(M, "ab->ba");   // M column-major: m rows, n columns
                    ex.push_back(JReq{Mt.p, m, n, true, {}, {}, {}});
                    ex_t.push_back(true);
                }
                ex_of.push_back(i);
            } else {
                rnd.push_back(i);
            }
        }
        jacobi_batch(ex);
        for (size_t e = 0; e < ex.size(); ++e) {
            SvdReq& r = rq[ex_of[e]];
            const int64_t m = r.M.d[0], n = r.M.d[1];
            if (!ex_t[e]) {
                // M^T = U S V^T -> M = V S U^T: left vectors = rows of V, right = rows of U
                r.UT = make_tn(ex[e].V.p, {r.kk, m});
                r.VT = make_tn(ex[e].U.p, {r.kk, n});
            } else {
                r.UT = make_tn(ex[e].U.p, {r.kk, m});
                r.VT = make_tn(ex[e].V.p, {r.kk, n});
            }
            r.S = make_tn(ex[e].S.p, {r.kk});
        }
        if (rnd.empty()) return;
        // oversampling: near the cut the spectra of these environments are
        // flat (sigma_{1.28 chi} / sigma_chi ~ 0.3-0.5), so the subspace extends
        // to min(2 kk, 128) vectors (at least kk + 16) and ten power steps
        // resolve the kept singular values to ~1e-11.  With the sign
        // convention of sign_fix the bond gauge settles as the environment
        // converges, and the last move's Ritz basis of a slot is then a far
        // better start than random normals (fewer power steps).
        const size_t nr = rnd.size();
        std::vector<Tn> Pt(nr), Qt(nr);
        bool all_warm = true, all_full = true;
        for (size_t j = 0; j < nr; ++j) {
            const SvdReq& r = rq[rnd[j]];
            const int64_t m = r.M.d[0], n = r.M.d[1], mn = std::min(m, n);
            const int64_t k = std::min<int64_t>(
                std::max<int64_t>(std::min<int64_t>(2 * r.kk, kCoreMax), r.kk + kOversample), mn);
            Pt[j] = tmp({k, n});
            ++svd_calls;
            // a slot starts from its last basis once the network's spectrum
            // moves by less than kWarmGate per move; earlier, while the
            // environment still changes a lot, it starts from fresh normals
            const bool use = warm_starts && r.slot >= 0 && last_delta < kWarmGate;
            const Warm* w = use ? &warm[r.slot] : nullptr;
            const bool warm_ok = w && w->valid && w->n == n && w->kk <= k;
            const bool full = warm_ok && w->kk == k;
            if (!full) ctmk::randn(st, Pt[j].p, k * n, 0x5eedull + 7919ull * svd_calls);
            if (warm_ok)
                ctmk::copy(st, w->V, Pt[j].p, w->kk * n);   // last move's Ritz vectors first
            all_warm = all_warm && warm_ok;
            all_full = all_full && full;
        }
        // inside the power steps one Cholesky-QR pass keeps the basis well
        // conditioned; the bases that enter the Rayleigh-Ritz core (last P, Q)
        // get the second pass that makes them orthonormal
        // with little oversampling (core narrower than 1.25 kk: the core is
        // capped at 128 + the 16 oversampling vectors only when kk > 112) the
        // kept space converges as (sigma_k / sigma_kk)^q over a flat spectrum
        // near the cut, so such batches get more steps
        bool thin = false;
        for (size_t j = 0; j < nr; ++j) thin = thin || 4 * Pt[j].d[0] < 5 * rq[rnd[j]].kk;
        const int q = power > 0 ? power
                    : (cfg.power_iters > 0 ? cfg.power_iters
                                           : (all_warm ? (!final_phase ? kWarmPowerItersEarly
                                                               : (thin ? kWarmPowerItersThin : kWarmPowerIters))
                                                       : (thin ? kColdPowerItersThin
                                                               : (reduced ? kColdPowerItersReduced
                                                                          : kColdPowerIters))));
        std::vector<Tn> Ms(nr);
        for (size_t j = 0; j < nr; ++j) Ms[j] = rq[rnd[j]].M;
        // a whole last-move Ritz basis has orthonormal rows already
        if (!all_full) cholqr_pass(Pt);
        // a settling warm move (spectrum change above kWarmTight) gives its
        // last bases one Cholesky-QR pass instead of two: the next move
        // continues from them, and the final moves make them orthonormal
        const bool loose = all_warm && !final_phase && !thin;
        for (int it = 0; it < q; ++it) {
            Qt = mm_group(Pt, false, Ms, true);    // (M P)^T
            cholqr_pass(Qt);
            Pt = mm_group(Qt, false, Ms, false);   // (M^T Q)^T
            if (it + 1 < q || loose) cholqr_pass(Pt);
            else orth(Pt);
        }
        Qt = mm_group(Pt, false, Ms, true);
        if (loose) cholqr_pass(Qt);
        else orth(Qt);
        const std::vector<Tn> X1 = mm_group(Qt, false, Ms, false);   // Q^T M   (k x n)
        const std::vector<Tn> Bs = mm_group(X1, false, Pt, true);    // Q^T M P (k x k)
        std::vector<JReq> core(nr);
        for (size_t j = 0; j < nr; ++j) {
            const int64_t k = Bs[j].d[0];
            // Bs row-major == Bs^T col-major: Bs^T = Uj S Vj^T -> Bs = Vj S Uj^T
            core[j] = JReq{Bs[j].p, k, k, true, {}, {}, {}};
        }
        // while a warm iteration is still settling (spectrum change above
        // kWarmTight) three sweeps of the core suffice: the next move continues
        // from these Ritz vectors; the final moves converge it fully
        jacobi_batch(core, (all_warm && !final_phase) ? kWarmJacobiSweeps : kJacobiSweeps);
        std::vector<Tn> Vjt(nr), Ujt(nr);
        for (size_t j = 0; j < nr; ++j) {
            const int64_t k = core[j].S.d[0];
            Vjt[j] = make_tn(core[j].V.p, {k, k});   // rows = left vectors of Bs
            Ujt[j] = make_tn(core[j].U.p, {k, k});   // rows = right vectors of Bs
        }
        const std::vector<Tn> UTs = mm_group(Vjt, false, Qt, false);   // (Q Us)^T
        const std::vector<Tn> VTs = mm_group(Ujt, false, Pt, false);   // (P Vs)^T
        for (size_t j = 0; j < nr; ++j) {
            SvdReq& r = rq[rnd[j]];
            const int64_t m = r.M.d[0], n = r.M.d[1], k = core[j].S.d[0];
            const Tn &UTf = UTs[j], &VTf = VTs[j];
            ctmk::sign_fix(st, UTf.p, VTf.p, (int)r.kk, (int)m, (int)n);
            if (warm_starts && r.slot >= 0) {
                // the whole Ritz basis (kept and oversampling vectors) starts
                // the next move's iteration of this slot
                Warm& w = warm[r.slot];
                if (w.cap < k * n) {
                    w.V = keep(k * n);
                    w.cap = k * n;
                }
                ctmk::copy(st, VTf.p, w.V, k * n);
                w.kk = k;
                w.n = n;
                w.valid = true;
            }
            r.UT = make_tn(UTf.p, {r.kk, m});
            r.VT = make_tn(VTf.p, {r.kk, n});
            r.S = make_tn(core[j].S.p, {r.kk});
        }
    }

    // projector pairs from (rhoT (t x rT), rhoB (rB x t)) for every entry of
    // the list; the factorisations of all entries share their launches and one
    // read-back of the kept ranks.
    // fill (growth phase, environment-selection principle): an entry whose
    // rho_B rho_T has fewer than min(chi, t) singular values above the cutoff
    // gets the orthogonal pair PT = Q^T, PB = Q instead, Q the min(chi, t)
    // leading eigenvectors of G = rhoT rhoT^T / |rhoT|^2 + rhoB^T rhoB / |rhoB|^2
    std::vector<Projector> projectors(const std::vector<std::pair<Tn, Tn>>& prs, int64_t chi, int slot0,
                                      bool fill = false)
    {
        FactorScope fs(*this);
        REQUIRE(prs.size() <= (size_t)kMaxBatch, "too many projectors in one batch");
        std::vector<Projector> out(prs.size());
        std::vector<SvdReq> rq;
        std::vector<size_t> of;
        for (size_t i = 0; i < prs.size(); ++i) {
            const Tn &rT = prs[i].first, &rB = prs[i].second;
            const int64_t t = rT.d[0], remT = rT.d[1], remB = rB.d[0];
            REQUIRE(rT.r == 2 && rB.r == 2 && rB.d[1] == t, "projector shapes");
            if (t <= chi) {
                Tn I = tmp({t, t});
                ctmk::eye(st, I.p, (int)t);
                out[i].PT = I;
                out[i].PB = I;
                out[i].k = (int)t;
                continue;
            }
            SvdReq r;
            {
                // rho_B rho_T in FP64 in every form: its small singular values
                // (down to ~1e-7 of the largest) decide the projectors
                Prec fp64(*this, CTM_FP64);
                r.M = mm(rB, false, rT, false);      // remB x remT
            }
            r.kk = std::min<int64_t>(chi, std::min(remB, remT));
            r.slot = slot0 + (int)i;
            rq.push_back(r);
            of.push_back(i);
        }
        if (rq.empty()) return out;
        svd_batch(rq);
        // each bond keeps the chi largest singular values that are above the
        // relative cutoff (its numerical rank): one small read-back for all
        double cut = cfg.svd_cutoff > 0 ? cfg.svd_cutoff : kDefaultCutoff;
        // rho_B rho_T built from FP32 / BF16 products carries a relative error of
        // order the unit roundoff; singular values below that level are noise
        if (bulk == CTM_FP32) cut = std::max(cut, lp_cut > 0 ? lp_cut : kLpCutFp32);
        if (bulk == CTM_BF16) cut = std::max(cut, lp_cut > 0 ? lp_cut : kLpCutBf16);
        for (size_t j = 0; j < rq.size(); ++j) ctmk::count_above(st, rq[j].S.p, (int)rq[j].kk, cut, icount + j);
        int rank[kMaxBatch] = {0};
        HIPCHK(hipMemcpyAsync(rank, icount, rq.size() * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (trace_ranks) {
            for (size_t j = 0; j < rq.size(); ++j) {
                std::vector<double> sv((size_t)rq[j].kk);
                HIPCHK(hipMemcpy(sv.data(), rq[j].S.p, sv.size() * sizeof(double), hipMemcpyDeviceToHost));
                const int r = rank[j];
                std::fprintf(stderr, "rank P%d %d/%lld last %.3e next %.3e\n", slot0 + (int)j + 1, r,
                             (long long)rq[j].kk, r > 0 ? sv[r - 1] / sv[0] : 0.0,
                             r < (int)sv.size() ? sv[r] / sv[0] : 0.0);
            }
        }
        // P_B = rho_T V S^-1/2 and P_T = S^-1/2 U^T rho_B amplify the directions
        // of small singular values: FP64 in every form
        Prec fp64(*this, CTM_FP64);
        std::vector<SvdReq> fq;
        std::vector<int> fill_of(rq.size(), -1);
        int frank[kMaxBatch] = {0};
        if (fill) {
            for (size_t j = 0; j < rq.size(); ++j) {
                const Tn &rT = prs[of[j]].first, &rB = prs[of[j]].second;
                const int64_t t = rT.d[0], remT = rT.d[1], remB = rB.d[0], k = std::min<int64_t>(chi, t);
                if (rank[j] >= k) continue;
                // Z^T = [rhoT^T / |rhoT| ; rhoB / |rhoB|]  ((remT + remB) x t): its right
                // singular vectors are the leading eigenvectors of the Gram matrix
                Tn Zt = tmp({remT + remB, t});
                Tn rTt = perm(rT, "ab->ba");
                ctmk::copy(st, rTt.p, Zt.p, remT * t);
                ctmk::copy(st, rB.p, Zt.p + remT * t, remB * t);
                Tn nrm = tmp({2});
                ctmk::dot(st, rT.p, rT.p, rT.n(), nrm.p, part, 1);
                ctmk::dot(st, rB.p, rB.p, rB.n(), nrm.p + 1, part, 1);
                ctmk::scale_inv(st, Zt.p, remT * t, nrm.p);
                ctmk::scale_inv(st, Zt.p + remT * t, remB * t, nrm.p + 1);
                SvdReq r;
                r.M = Zt;
                r.kk = std::min<int64_t>(k, remT + remB);
                r.slot = -1;
                fill_of[j] = (int)fq.size();
                fq.push_back(r);
            }
            if (!fq.empty()) {
                // growth-phase moves only: resolve the kept vectors to rounding
                svd_batch(fq, kFillPowerIters);
                for (size_t f = 0; f < fq.size(); ++f)
                    ctmk::count_above(st, fq[f].S.p, (int)fq[f].kk, cut, icount + f);
                HIPCHK(hipMemcpyAsync(frank, icount, fq.size() * sizeof(int), hipMemcpyDeviceToHost, st));
                HIPCHK(hipStreamSynchronize(st));
            }
        }
        for (size_t j = 0; j < rq.size(); ++j) {
            const size_t i = of[j];
            const Tn &rT = prs[i].first, &rB = prs[i].second;
            const int64_t t = rT.d[0];
            if (fill_of[j] >= 0) {
                // orthogonal pair on the right singular vectors of Z^T whose
                // singular value is above the cutoff
                const SvdReq& f = fq[fill_of[j]];
                const int64_t kf = std::max<int64_t>(1, std::min<int64_t>(f.kk, frank[fill_of[j]]));
                Tn Q = f.VT;
                Q.d[0] = kf;                                   // kf x t
                out[i].PT = Q;
                out[i].PB = perm(Q, "ab->ba");                // t x kf
                out[i].k = (int)kf;
                continue;
            }
            const int64_t kk = std::max<int64_t>(1, std::min<int64_t>(rq[j].kk, rank[j]));
            Tn UT = rq[j].UT, VT = rq[j].VT;
            UT.d[0] = kk;
            VT.d[0] = kk;
            Tn f = tmp({kk});
            ctmk::inv_sqrt_cut(st, rq[j].S.p, f.p, (int)kk, cut);
            out[i].PB = mm(rT, false, VT, true);           // t x kk
            ctmk::scale_lines(st, out[i].PB.p, (int)t, (int)kk, f.p, 1);
            out[i].PT = mm(UT, false, rB, false);          // kk x t
            ctmk::scale_lines(st, out[i].PT.p, (int)kk, (int)t, f.p, 0);
            out[i].k = (int)kk;
        }
        return out;
    }

    void normalize(Tn& X)
    {
        ctmk::dot(st, X.p, X.p, X.n(), scal, part, 1);
        ctmk::scale_inv(st, X.p, X.n(), scal);
    }

    // ---------------- one symmetric split-CTMRG iteration of one network
    void step(Net& N, int64_t chi);
    void values(Net& N, bool with_env);
    // the corner spectrum of the current environment with converged Jacobi
    // sweeps into N.s_old / N.n_old (a settling move may have capped them)
    void exact_spectrum(Net& N);
    // ---------------- the same for the reduced method
    void step_reduced(Net& N, int64_t chi);
    void values_reduced(Net& N, bool with_env);
    // n1 of the 3x3 patch with the PEPO Oc at its centre (the rest of the
    // network as in N) into *out (device scalar)
    void centre_value(Net& N, const double* Oc, double* out);
    // the 3x4 patch around two horizontally adjacent sites, both with the
    // PEPO Oc, into *out (device scalar)
    void pair_value(Net& N, const double* Oc, double* out);
    void pair_value_split(Net& N, const double* Oc, double* out);
};

// --------------------------------------------------------------------------
// the iteration
// --------------------------------------------------------------------------
void Worker::step(Net& N, int64_t chi)
{
    if (reduced) {
        step_reduced(N, chi);
        return;
    }
    Prec bulk_prec(*this, bulk);   // absorption, environments, projector application
    const int64_t D = this->D, d = N.d, P = 2;
    const Arena::Mark mk = ws.mark();
    // growth phase: the corner bond is still below chi (Sec. III C: the
    // projector environments cannot have rank chi yet)
    const bool growing = !N.grown && N.xbk < chi;
    Tn C1 = make_tn(N.C1, {N.xbk, N.xbk}), C4 = make_tn(N.C4, {N.xbk, N.xbk});
    Tn K = make_tn(N.Tk, {N.xbk, D, N.xki});
    Tn I = make_tn(N.Ti, {N.xki, d, N.xib});
    Tn Bt = make_tn(N.Tb, {N.xib, D, N.xbk});
    Tn A = make_tn(const_cast<double*>(this->A), {P, D, D, D, D});
    Tn O = make_tn(N.O, {P, P, d, d, d, d});
    // right / bottom edge chain (D2 relations)
    Tn Rk = perm(Bt, "bma->amb"), Ri = perm(I, "bma->amb"), Rb = perm(K, "bma->amb");
    // Each section below ends by settling its results (settle), so that the
    // step holds the intermediates of one chain at a time: the largest is
    // chi^2 D^3 d^2 P doubles (Sec. III C, memory cost of the split scheme).
    const Arena::Mark m_s1 = ws.mark();

    // ---- top row C1 T1(k,i,b) C2 and the upper halves at ki, ib, bk
    Tn H = ctr("xy,xkc->ykc", C1, K);
    H = ctr("ykc,cie->ykie", H, I);
    Tn TRpre = ctr("ykie,ebf->ykibf", H, Bt);          // [y1, Au, Ou, Bu, s3]
    Tn TR = ctr("ykibf,fz->ykibz", TRpre, C4);          // [y1, Au, Ou, Bu, y2]
    Tn U = ctr("ykibz,ylg->glkibz", TR, K);
    U = ctr("glkibz,plkrn->gpnribz", U, A);
    Tn upki = ctr("gpnribz,zrh->gpnibh", U, Rk);        // [tkb, p, Ad, Ou, Bu, rkb]
    U = ctr("gpnibh,gmj->jmpnibh", upki, I);
    U = ctr("jmpnibh,pqmist->jqtsnbh", U, O);
    Tn upib = ctr("jqtsnbh,hsk->jqtnbk", U, Ri);        // [tib, q, Od, Ad, Bu, rib]
    U = ctr("jqtnbk,jwv->vwqtnbk", upib, Bt);
    U = ctr("vwqtnbk,qwbse->vsetnk", U, A);
    Tn upbk = ctr("vsetnk,ksz->vetnz", U, Rb);          // [tbb, Bd, Od, Ad, rbb]

    // ---- stage 1: P1 (bk, trunc (chi, B)), P2 (ki, (chi, O, B)), P3 (ib, (chi, B, q))
    const int64_t xbk = N.xbk, xki = N.xki, xib = N.xib;
    Tn rT1 = perm(upbk, "vetnz->ventz");
    Tn rB1 = perm(upbk, "fbcea->bcfae");
    Tn rT2 = perm(upki, "gpnibh->gibnph");
    Tn rB2 = perm(upib, "jqtnbk->bqjktn");
    Tn rT3 = perm(upib, "jqtnbk->jbqntk");
    Tn rB3 = perm(upki, "gpnibh->bighnp");
    std::vector<Projector> S1 = projectors(
        {{view(rT1, {xbk * D, D * d * xbk}), view(rB1, {D * d * xbk, xbk * D})},
         {view(rT2, {xki * d * D, D * P * xib}), view(rB2, {D * P * xib, xki * d * D})},
         {view(rT3, {xib * D * P, D * d * xki}), view(rB3, {D * d * xki, xib * D * P})}},
        chi, 0, growing);
    settle(m_s1, {&TRpre, &S1[0].PT, &S1[0].PB, &S1[1].PT, &S1[1].PB, &S1[2].PT, &S1[2].PB});
    const Projector &P1 = S1[0], &P2 = S1[1], &P3 = S1[2];
    const int64_t c1 = P1.k, c2 = P2.k, c3 = P3.k;
    Tn P1T = view(P1.PT, {c1, xbk, D}), P1B = view(P1.PB, {xbk, D, c1});
    Tn P2T = view(P2.PT, {c2, xki, d, D}), P2B = view(P2.PB, {xki, d, D, c2});
    Tn P3T = view(P3.PT, {c3, xib, D, P}), P3B = view(P3.PB, {xib, D, P, c3});

    // ---- enlarged corners with the stage-1 bra projections on both legs.
    // The bra site and the projector that cuts its leg are joined into a
    // small piece before they meet the ket and PEPO layers, so that no
    // intermediate carries D^4 (chi^2 D^3 d^2 P at most).
    const Arena::Mark m_e = ws.mark();
    Tn Etop = ctr("xy,xkc->ykc", C1, K);
    Tn E = ctr("ykc,ylg->kclg", Etop, K);
    E = ctr("kclg,plkrn->cgprn", E, A);
    E = ctr("cgprn,cie->egiprn", E, I);
    E = ctr("egiprn,gmj->eijmprn", E, I);
    E = ctr("eijmprn,pqmist->ejqrnst", E, O);
    E = ctr("ejqrnst,ebf->fbjqrnst", E, Bt);
    Tn G = ctr("jwv,cve->jwce", Bt, P1T);                 // bra edge cut by P1
    G = ctr("jwce,qwbhe->jcqbh", G, A);                   // [tib, c_d, q, Bu, Br]
    E = ctr("fbjqrnst,jcqbh->fcrnsth", E, G);            // [s3, c_d, Ar, Ad, Or, Od, Br]
    Tn C1p = ctr("fcrnsth,Xfh->cntXrs", E, P1T);       // [c_d, Ad, Od, c_r, Ar, Or]
    if (full_p4) settle(m_e, {&C1p, &E});
    else settle(m_e, {&C1p});
    const Arena::Mark m_f = ws.mark();
    Tn F = ctr("xy,wvx->wvy", C4, Bt);
    F = ctr("wvy,yac->wvac", F, Rk);
    F = ctr("wvac,jmw->jmvac", F, I);
    F = ctr("jmvac,cod->jmvaod", F, Ri);
    F = ctr("jmvaod,pqmuro->jvadpqur", F, O);
    Tn F0;
    if (full_p4) {
        // the full P4 also needs the enlarged corner before P1 (F0)
        F = ctr("jvadpqur,klj->klvadpqur", F, K);
        F = ctr("klvadpqur,plzsa->kvdqurzs", F, A);
        F = ctr("kvdqurzs,dbe->kvbequrzs", F, Rb);
        F0 = ctr("kvbequrzs,qvtwb->keurzstw", F, A);     // [a0, s3, Ou, Or, Au, Ar, Bu, Br]
        F = ctr("keurzstw,ktc->ceurzsw", F0, P1B);        // [c_u, s3, Ou, Or, Au, Ar, Br]
    } else {
        Tn Z = ctr("dbe,qvtwb->deqvtw", Rb, A);            // bra site on the bottom edge
        F = ctr("jvadpqur,deqvtw->japuretw", F, Z);
        Tn Y = ctr("klj,ktc->ljtc", K, P1B);               // left edge cut by P1
        F = ctr("japuretw,ljtc->apurewlc", F, Y);
        F = ctr("apurewlc,plzsa->ceurzsw", F, A);         // [c_u, s3, Ou, Or, Au, Ar, Br]
    }
    Tn C4p = ctr("ceurzsw,esX->czuXwr", F, P1B);       // [c_u, Au, Ou, c_r', Br, Or]

    // ---- stage 2: P4 from the enlarged corners
    const int64_t n4 = c1 * D * d;
    Tn rT4 = C1p, rB4;
    if (full_p4) {
        // full P4 (Appendix, Fig. Projector4(a)): the 2x2 block of enlarged
        // corners, vertical legs after P1 (left bond) and its right-move image
        // P1^R = (P1B, P1T) (right bond), horizontal legs whole.  Upper right:
        // the diagonal-reflection image of the enlarged C4 (legs a0, s3, Au, Ar,
        // Ou, Or, Bu, Br -> left chi, down chi, A.l, A.d, O.l, O.d, B.l, B.d)
        // with P1^R_T = P1B on its down leg's (chi, A.d)
        Tn C2e = ctr("keurzstw,esX->kzutXrw", F0, P1B);      // [chi, Al, Ol, Bl, X, Od, Bd]
        rT4 = ctr("fcrnsth,frshXiy->cntXiy", E, C2e);       // [c, Ad, Od | X, Od2, Bd2]
        // lower right: the 180-degree image of the enlarged C1 with
        // P1^R_B = P1T on its up leg's (chi, A.u): the arrays of E with legs
        // [chi left, c', B.l, B.u, O.l, O.u, A.l]
        Tn Q = ctr("ceurzsw,eCwBrOs->czuCBO", F, E);          // [c, Au, Ou | C, Bu2, Ou2]
        rB4 = perm(Q, "cauCBO->CBOcau");
    } else {
        // half P4 (Fig. Projector4(b)): the two left enlarged corners, their
        // horizontal legs renormalised by the up / down images of P1
        rB4 = perm(C4p, "cauXbo->Xbocau");
    }
    if (full_p4) settle(m_f, {&C4p, &rT4, &rB4});
    else settle(m_f, {&C4p, &rB4});

    // ---- stage 2: P5 (ki) and P6 (ib) from the two-column block
    const Arena::Mark m_s3 = ws.mark();
    Tn L = ctr("ykibf,ylg->kibflg", TRpre, K);
    Tn ULraw = ctr("kibflg,plkrn->ibfgpnr", L, A);      // [Ou, Bu, s3, tkb, p, Ad, Ar]
    Tn UL5 = ctr("ibfgpnr,cgib->cfpnr", ULraw, P2T);   // [c2L, s3, p, Ad, Ar]
    Tn J = ctr("fkc,cie->fkie", K, I);
    J = ctr("fkie,ebh->fkibh", J, Bt);
    J = ctr("fkibh,hz->fkibz", J, C4);
    J = ctr("fkibz,zrg->fkibrg", J, Rk);
    Tn URraw = ctr("fkibrg,plkrn->fibgpln", J, A);      // [s3, Ou, Bu, rkb, p, Al, Ad]
    Tn UR5 = ctr("fibgpln,gnpc->fiblc", URraw, P3B);   // P2^R_T = P3_B: [s3, Ou2, Bu2, Al2, c2R]
    Tn rT5 = ctr("cfpnr,fibrd->cnpibd", UL5, UR5);      // [c2L, Ad1, p1, Ou2, Bu2, c2R]
    const Arena::Mark m_h = ws.mark();
    Tn H6 = ctr("ibfgpnr,gmj->ibfjmpnr", ULraw, I);
    H6 = ctr("ibfjmpnr,pqmist->bfjqnrst", H6, O);
    Tn UL6 = ctr("bfjqnrst,cjbq->cfnrst", H6, P3T);    // [c3L, s3, Ad1, Ar1, Or1, Od1]
    settle(m_h, {&UL6});
    const Arena::Mark m_k = ws.mark();
    Tn K6 = ctr("fibgpln,gsh->fibpslnh", URraw, Ri);
    K6 = ctr("fibpslnh,pqmist->fblnhqmt", K6, O);
    Tn UR6 = ctr("fblnhqmt,htnc->fblqmc", K6, P2B);    // P3^R_T = P2_B: [s3, Bu2, Al2, q2, Ol2, c3R]
    settle(m_k, {&UR6});
    Tn rT6 = ctr("cfnrst,fbrqsd->cntbqd", UL6, UR6);    // [c3L, Ad1, Od1, Bu2, q2, c3R]
    Tn rB5 = perm(rT6, "gfebca->efgabc");               // rotation image of rho_T6
    Tn rB6 = perm(rT5, "gefcba->efgabc");               // rotation image of rho_T5
    std::vector<Projector> S2 = projectors(
        {{view(rT4, {n4, n4}), view(rB4, {n4, n4})},
         {view(rT5, {c2 * D * P, d * D * c3}), view(rB5, {d * D * c3, c2 * D * P})},
         {view(rT6, {c3 * D * d, D * P * c2}), view(rB6, {D * P * c2, c3 * D * d})}},
        chi, 3, growing);
    settle(m_s3, {&S2[0].PT, &S2[0].PB, &S2[1].PT, &S2[1].PB, &S2[2].PT, &S2[2].PB});
    const Projector &P4 = S2[0], &P5 = S2[1], &P6 = S2[2];
    const int64_t k4 = P4.k, k5 = P5.k, k6 = P6.k;
    Tn P4T = view(P4.PT, {k4, c1, D, d}), P4B = view(P4.PB, {c1, D, d, k4});
    Tn P5T = view(P5.PT, {k5, c2, D, P}), P5B = view(P5.PB, {c2, D, P, k5});
    Tn P6T = view(P6.PT, {k6, c3, D, d}), P6B = view(P6.PB, {c3, D, d, k6});

    // ---- two-stage projectors of the three bonds
    Tn PbkT = ctr("ncao,cxb->nxaob", P4T, P1T);         // [n, chi, A, O, B]
    Tn PbkB = ctr("xbc,caon->xaobn", P1B, P4B);         // [chi, A, O, B, n]
    Tn PkiT = ctr("ncap,cxob->nxapob", P5T, P2T);       // [n, chi, A, p, O, B]
    Tn PkiB = ctr("xobc,capn->xapobn", P2B, P5B);       // [chi, A, p, O, B, n]
    Tn PibT = ctr("ncao,cxbq->nxaoqb", P6T, P3T);       // [n, chi, A, O, q, B]
    Tn PibB = ctr("xbqc,caon->xaoqbn", P3B, P6B);       // [chi, A, O, q, B, n]

    // ---- corners: second-stage projectors on the stage-1 renormalised corners
    Tn W1 = ctr("cdfqre,Xqre->cdfX", C1p, P4T);
    Tn C1_n = mat(ctr("cdfX,Ycdf->XY", W1, P4T));
    Tn W4 = ctr("cwhXyi,cwhx->xXyi", C4p, P4B);
    Tn C4_n = mat(ctr("xXyi,Xyiz->xz", W4, P4B));
    ctmk::symmetrize(st, C1_n.p, (int)k4);
    ctmk::symmetrize(st, C4_n.p, (int)k4);
    normalize(C1_n);
    normalize(C4_n);

    // ---- convergence spectrum of C1 C2 C3 C4 = (C1 C4)^2 (FP64 in every form).
    // The two products run on this stream; the Jacobi SVD and the spectrum
    // change run on the side stream while this stream renormalises the edges.
    {
        Prec spec64(*this, CTM_FP64);
        Tn R1 = ctr("ab,bc->ac", C1_n, C4_n);
        Tn R = mat(ctr("ab,bc->ac", R1, R1));
        ctmk::trace(st, R.p, (int)k4, N.sc + 7);
        side_begin();
        std::vector<JReq> sp{JReq{R.p, k4, k4, false, {}, {}, {}}};
        // far from convergence the change only has to be known roughly (it
        // gates warm starts at 1e-3 and 1e-6): a few sweeps; near it, all
        // (ctm_corner_spectrum recomputes the spectrum it returns)
        jacobi_batch(sp, !final_phase ? kWarmJacobiSweeps : kJacobiSweeps);
        ctmk::spectrum_delta(st, sp[0].S.p, (int)k4, N.sc + 7, N.s_old, N.n_old, N.delta);
        side_end();
    }

    // ---- renormalised left edge (row-wise absorption, both neighbouring bonds)
    Tn X = ctr("xuosn,xlb->nuoslb", PbkB, K);
    X = ctr("nuoslb,plumd->nosbpmd", X, A);
    Tn Tk_n = ctr("nosbpmd,kbdpos->nmk", X, PkiT);
    X = ctr("xapusn,xlb->napuslb", PkiB, I);
    X = ctr("napuslb,pqlumt->nasbmtq", X, O);
    Tn Ti_n = ctr("nasbmtq,kbatqs->nmk", X, PibT);
    X = ctr("xaoqun,xlb->naoqulb", PibB, Bt);
    X = ctr("naoqulb,qlumt->naobmt", X, A);
    Tn Tb_n = ctr("naobmt,kbaot->nmk", X, PbkT);
    Tk_n = mat(Tk_n);
    Ti_n = mat(Ti_n);
    Tb_n = mat(Tb_n);
    normalize(Tk_n);
    normalize(Ti_n);
    normalize(Tb_n);
    side_wait();

    // ---- store
    N.xbk = k4;
    N.xki = k5;
    N.xib = k6;
    if (N.xbk >= chi) N.grown = true;
    ctmk::copy(st, C1_n.p, N.C1, C1_n.n());
    ctmk::copy(st, C4_n.p, N.C4, C4_n.n());
    ctmk::copy(st, Tk_n.p, N.Tk, Tk_n.n());
    ctmk::copy(st, Ti_n.p, N.Ti, Ti_n.n());
    ctmk::copy(st, Tb_n.p, N.Tb, Tb_n.n());
    ws.release(mk);
}

void Worker::exact_spectrum(Net& N)
{
    Prec fp64(*this, CTM_FP64);
    const Arena::Mark mk = ws.mark();
    const int64_t k = N.xbk;
    Tn C1 = make_tn(N.C1, {k, k});
    Tn C4 = reduced ? C1 : make_tn(N.C4, {k, k});   // reduced method: one corner, C^4
    Tn R1 = ctr("ab,bc->ac", C1, C4);
    Tn R = mat(ctr("ab,bc->ac", R1, R1));
    ctmk::trace(st, R.p, (int)k, N.sc + 7);
    std::vector<JReq> sp{JReq{R.p, k, k, false, {}, {}, {}}};
    jacobi_batch(sp, kJacobiSweeps);
    ctmk::spectrum_delta(st, sp[0].S.p, (int)k, N.sc + 7, N.s_old, N.n_old, scal);   // change not kept
    ws.release(mk);
}

// n1, n2h, n2v, n0 into N.sc[0..3], ln kappa into N.sc[4], flag N.sc[5];
// with_env: also the bra environment into N.E and its overlap with A in N.sc[6]
void Worker::values(Net& N, bool with_env)
{
    if (reduced) {
        values_reduced(N, with_env);
        return;
    }
    Prec fp64(*this, CTM_FP64);   // f and g are evaluated in FP64 in every form
    const int64_t D = this->D, d = N.d, P = 2;
    const Arena::Mark mk = ws.mark();
    Tn C1 = make_tn(N.C1, {N.xbk, N.xbk}), C4 = make_tn(N.C4, {N.xbk, N.xbk});
    Tn K = make_tn(N.Tk, {N.xbk, D, N.xki});
    Tn I = make_tn(N.Ti, {N.xki, d, N.xib});
    Tn Bt = make_tn(N.Tb, {N.xib, D, N.xbk});
    Tn A = make_tn(const_cast<double*>(this->A), {P, D, D, D, D});
    Tn O = make_tn(N.O, {P, P, d, d, d, d});
    Tn Rk = perm(Bt, "bma->amb"), Ri = perm(I, "bma->amb"), Rb = perm(K, "bma->amb");
    Tn H = ctr("xy,xkc->ykc", C1, K);
    H = ctr("ykc,cie->ykie", H, I);
    H = ctr("ykie,ebf->ykibf", H, Bt);
    Tn TR = ctr("ykibf,fz->ykibz", H, C4);              // [y1, Au, Ou, Bu, y2]
    Tn BR = perm(TR, "fecba->abcef");                   // [x4, Ad, Od, Bd, x3] (rotation image)
    Tn U = ctr("ykibz,ylg->glkibz", TR, K);
    U = ctr("glkibz,plkrn->gpnribz", U, A);
    U = ctr("gpnribz,zrh->gpnibh", U, Rk);
    U = ctr("gpnibh,gmj->jmpnibh", U, I);
    U = ctr("jmpnibh,pqmist->jqtsnbh", U, O);
    Tn upib = ctr("jqtsnbh,hsk->jqtnbk", U, Ri);
    U = ctr("jqtnbk,jwv->vwqtnbk", upib, Bt);
    U = ctr("vwqtnbk,qwbse->vsetnk", U, A);
    Tn upbk = ctr("vsetnk,ksz->vetnz", U, Rb);
    Tn s1 = ctr("vetnz,vntez->", upbk, BR);
    Tn s2h = ctr("yaobz,yaobz->", TR, BR);
    Tn X = ctr("xy,xz->yz", C1, C4);
    X = ctr("yz,yma->zma", X, K);
    X = ctr("zma,zmb->ab", X, Rk);
    X = ctr("ab,amc->bmc", X, I);
    X = ctr("bmc,bme->ce", X, Ri);
    X = ctr("ce,cmf->emf", X, Bt);
    X = ctr("emf,emg->fg", X, Rb);
    X = ctr("fg,fh->gh", X, C4);
    Tn s2v = ctr("gh,gh->", X, C1);
    Tn R1 = ctr("ab,bc->ac", C1, C4);
    Tn s0 = ctr("ab,ba->", R1, R1);
    ctmk::copy(st, s1.p, N.sc + 0, 1);
    ctmk::copy(st, s2h.p, N.sc + 1, 1);
    ctmk::copy(st, s2v.p, N.sc + 2, 1);
    ctmk::copy(st, s0.p, N.sc + 3, 1);
    ctmk::log_kappa(st, N.sc, N.sc + 4);
    if (with_env) {
        // the bottom edge joins the lower half first, so that no intermediate
        // carries D^4
        Tn G = ctr("jqtnbk,jwv->qtnbwvk", upib, Bt);
        Tn RB = ctr("ksz,vntez->ksvnte", Rb, BR);
        Tn Env = mat(ctr("qtnbwvk,ksvnte->qwbse", G, RB));   // [q, Bl, Bu, Br, Bd]
        ctmk::copy(st, Env.p, N.E, Env.n());
        ctmk::dot(st, Env.p, this->A, Env.n(), N.sc + 6, part, 0);
    }
    ws.release(mk);
}

// ---------------------------------------------------------------------------
// reduced method (Sec. II): C4v-symmetric CTMRG on the fused site tensor a,
// one corner C (chi x chi, symmetric) and one edge T [chi][Df][chi]
// (symmetric in its chi legs) for all four directions
// ---------------------------------------------------------------------------
void Worker::step_reduced(Net& N, int64_t chi)
{
    Prec fp64(*this, CTM_FP64);
    const Arena::Mark mk = ws.mark();
    const int64_t x = N.xbk, Df = N.Df, n = x * Df;
    Tn C = make_tn(N.C1, {x, x});
    Tn T = make_tn(N.Tf, {x, Df, x});
    Tn a = make_tn(N.a, {Df, Df, Df, Df});
    // enlarged corner M[(b,d),(c,r)] = C[x,y] T[x,m,b] T[y,n,c] a[m,n,r,d]
    Tn X = ctr("xy,xmb->ymb", C, T);
    X = ctr("ymb,ync->mbnc", X, T);
    Tn M = view(mat(ctr("mbnc,mnrd->bdcr", X, a)), {n, n});
    ctmk::symmetrize(st, M.p, (int)n);
    // the chi eigenvectors of largest |lambda|: for the symmetric M these are
    // its leading right singular vectors (singular values = |lambda|)
    std::vector<SvdReq> rq(1);
    rq[0].M = M;
    rq[0].kk = std::min<int64_t>(chi, n);
    rq[0].slot = 0;
    svd_batch(rq);
    const double cut = cfg.svd_cutoff > 0 ? cfg.svd_cutoff : kDefaultCutoff;
    ctmk::count_above(st, rq[0].S.p, (int)rq[0].kk, cut, icount);
    int rank = 0;
    HIPCHK(hipMemcpyAsync(&rank, icount, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const int64_t k = std::max<int64_t>(1, std::min<int64_t>(rq[0].kk, rank));
    Tn VT = rq[0].VT;                          // rows: the kept eigenvectors
    VT.d[0] = k;
    // C' = V^T M V
    Tn Cn = mm(VT, false, mm(M, false, VT, true), false);
    // T'[z,r,w] = V[(a,u),z] T[a,m,b] a[m,u,r,d] V[(b,d),w], the projector
    // taken into the edge before the site (never forms T a)
    Tn P3 = view(VT, {k, x, Df});
    Tn Y = ctr("zau,amb->zumb", P3, T);
    Y = ctr("zumb,murd->zbrd", Y, a);
    Tn Tn_ = mat(ctr("zbrd,wbd->zrw", Y, P3));
    ctmk::symmetrize(st, Cn.p, (int)k);
    ctmk::symmetrize_edge(st, Tn_.p, (int)k, (int)Df);
    normalize(Cn);
    normalize(Tn_);
    // convergence spectrum: singular values of C^4 / Tr C^4 (= lambda^4, normalised)
    Tn R1 = ctr("ab,bc->ac", Cn, Cn);
    Tn R = mat(ctr("ab,bc->ac", R1, R1));
    ctmk::trace(st, R.p, (int)k, N.sc + 7);
    std::vector<JReq> sp{JReq{R.p, k, k, false, {}, {}, {}}};
    jacobi_batch(sp);
    ctmk::spectrum_delta(st, sp[0].S.p, (int)k, N.sc + 7, N.s_old, N.n_old, N.delta);
    N.xbk = k;
    ctmk::copy(st, Cn.p, N.C1, Cn.n());
    ctmk::copy(st, Tn_.p, N.Tf, Tn_.n());
    ws.release(mk);
}

// n1 (3x3 patch), n2 (3x2 strip), n0 = Tr C^4; with_env: the bra environment
// E[q,l,u,r,d] (the fused-site environment with the ket and PEPO contracted)
// and its overlap with A
void Worker::values_reduced(Net& N, bool with_env)
{
    Prec fp64(*this, CTM_FP64);
    const Arena::Mark mk = ws.mark();
    const int64_t x = N.xbk, Df = N.Df;
    Tn C = make_tn(N.C1, {x, x});
    Tn T = make_tn(N.Tf, {x, Df, x});
    Tn a = make_tn(N.a, {Df, Df, Df, Df});
    Tn CTC = ctr("xa,amb->xmb", C, T);
    CTC = mat(ctr("xmb,by->xmy", CTC, C));              // corner-edge-corner row
    Tn s2 = ctr("xmy,xmy->", CTC, CTC);
    Tn R1 = ctr("ab,bc->ac", C, C);
    Tn s0 = ctr("ab,ba->", R1, R1);
    // environment of the centre site: top row with the left edge, bottom row
    // with the right edge, joined over the two corner-edge bonds
    Tn X1 = ctr("xuy,xlc->uylc", CTC, T);
    Tn X2 = ctr("cde,yre->cdyr", CTC, T);
    Tn env = mat(ctr("uylc,cdyr->lurd", X1, X2));
    Tn s1 = ctr("lurd,lurd->", env, a);
    ctmk::copy(st, s1.p, N.sc + 0, 1);
    ctmk::copy(st, s2.p, N.sc + 1, 1);
    ctmk::copy(st, s2.p, N.sc + 2, 1);
    ctmk::copy(st, s0.p, N.sc + 3, 1);
    ctmk::log_kappa(st, N.sc, N.sc + 4);
    if (with_env) {
        ctmk::unfuse_env(st, env.p, this->A, N.O, (int)D, (int)N.d, N.E);
        ctmk::dot(st, N.E, this->A, 2 * D * D * D * D, N.sc + 6, part, 0);
    }
    ws.release(mk);
}

void Worker::centre_value(Net& N, const double* Oc, double* out)
{
    Prec fp64(*this, CTM_FP64);
    const Arena::Mark mk = ws.mark();
    const int64_t D = this->D, d = N.d, P = 2;
    Tn A = make_tn(const_cast<double*>(this->A), {P, D, D, D, D});
    Tn O = make_tn(const_cast<double*>(Oc), {P, P, d, d, d, d});
    if (reduced) {
        const int64_t x = N.xbk, Df = N.Df;
        Tn C = make_tn(N.C1, {x, x});
        Tn T = make_tn(N.Tf, {x, Df, x});
        Tn a = tmp({Df, Df, Df, Df});
        ctmk::fuse_site(st, this->A, Oc, (int)D, (int)d, a.p);
        Tn CTC = ctr("xa,amb->xmb", C, T);
        CTC = mat(ctr("xmb,by->xmy", CTC, C));
        Tn X1 = ctr("xuy,xlc->uylc", CTC, T);
        Tn X2 = ctr("cde,yre->cdyr", CTC, T);
        Tn env = mat(ctr("uylc,cdyr->lurd", X1, X2));
        Tn s1 = ctr("lurd,lurd->", env, a);
        ctmk::copy(st, s1.p, out, 1);
        ws.release(mk);
        return;
    }
    // split: the upper two rows with the centre site, closed by the bottom
    // row (the n1 contraction of values() with the centre PEPO replaced)
    Tn C1 = make_tn(N.C1, {N.xbk, N.xbk}), C4 = make_tn(N.C4, {N.xbk, N.xbk});
    Tn K = make_tn(N.Tk, {N.xbk, D, N.xki});
    Tn I = make_tn(N.Ti, {N.xki, d, N.xib});
    Tn Bt = make_tn(N.Tb, {N.xib, D, N.xbk});
    Tn Rk = perm(Bt, "bma->amb"), Ri = perm(I, "bma->amb"), Rb = perm(K, "bma->amb");
    Tn H = ctr("xy,xkc->ykc", C1, K);
    H = ctr("ykc,cie->ykie", H, I);
    H = ctr("ykie,ebf->ykibf", H, Bt);
    Tn TR = ctr("ykibf,fz->ykibz", H, C4);
    Tn BR = perm(TR, "fecba->abcef");
    Tn U = ctr("ykibz,ylg->glkibz", TR, K);
    U = ctr("glkibz,plkrn->gpnribz", U, A);
    U = ctr("gpnribz,zrh->gpnibh", U, Rk);
    U = ctr("gpnibh,gmj->jmpnibh", U, I);
    U = ctr("jmpnibh,pqmist->jqtsnbh", U, O);
    U = ctr("jqtsnbh,hsk->jqtnbk", U, Ri);
    U = ctr("jqtnbk,jwv->vwqtnbk", U, Bt);
    U = ctr("vwqtnbk,qwbse->vsetnk", U, A);
    Tn upbk = ctr("vsetnk,ksz->vetnz", U, Rb);
    Tn s1 = ctr("vetnz,vntez->", upbk, BR);
    ctmk::copy(st, s1.p, out, 1);
    ws.release(mk);
}

void Worker::pair_value(Net& N, const double* Oc, double* out)
{
    Prec fp64(*this, CTM_FP64);
    if (!reduced) {
        pair_value_split(N, Oc, out);
        return;
    }
    const Arena::Mark mk = ws.mark();
    const int64_t x = N.xbk, Df = N.Df;
    Tn C = make_tn(N.C1, {x, x});
    Tn T = make_tn(N.Tf, {x, Df, x});
    Tn a = tmp({Df, Df, Df, Df});
    ctmk::fuse_site(st, this->A, Oc, (int)D, (int)N.d, a.p);
    // left half L[b,k,g]: top-left corner and edge, left edge, site 1,
    // bottom-left corner and edge; right half R[b,k,g] likewise
    Tn L = ctr("xa,amb->xmb", C, T);
    L = ctr("xmb,xlp->mblp", L, T);
    L = ctr("mblp,lmkd->bpkd", L, a);
    L = ctr("bpkd,pz->bkdz", L, C);
    L = mat(ctr("bkdz,zdg->bkg", L, T));
    Tn R = ctr("bnc,cy->bny", T, C);
    R = ctr("bny,yrq->bnrq", R, T);
    R = ctr("bnrq,knre->bkqe", R, a);
    R = ctr("bkqe,hq->bkeh", R, C);
    R = mat(ctr("bkeh,geh->bkg", R, T));
    Tn v = ctr("bkg,bkg->", L, R);
    ctmk::copy(st, v.p, out, 1);
    ws.release(mk);
}

// split environment: two-column top row, then the ket, PEPO and bra layers of
// both sites absorbed layer by layer between the left edge chain and its D2
// image, closed by the two-column bottom row
void Worker::pair_value_split(Net& N, const double* Oc, double* out)
{
    const Arena::Mark mk = ws.mark();
    const int64_t D = this->D, d = N.d, P = 2;
    Tn C1 = make_tn(N.C1, {N.xbk, N.xbk}), C4 = make_tn(N.C4, {N.xbk, N.xbk});
    Tn K = make_tn(N.Tk, {N.xbk, D, N.xki});
    Tn I = make_tn(N.Ti, {N.xki, d, N.xib});
    Tn Bt = make_tn(N.Tb, {N.xib, D, N.xbk});
    Tn A = make_tn(const_cast<double*>(this->A), {P, D, D, D, D});
    Tn O = make_tn(const_cast<double*>(Oc), {P, P, d, d, d, d});
    Tn Rk = perm(Bt, "bma->amb"), Ri = perm(I, "bma->amb"), Rb = perm(K, "bma->amb");
    // top row: [y, a o b (site 1 up), c p d (site 2 up), z]
    Tn X = ctr("xy,xas->yas", C1, K);
    X = ctr("yas,sot->yaot", X, I);
    X = ctr("yaot,tbu->yaobu", X, Bt);
    X = ctr("yaobu,ucv->yaobcv", X, K);
    X = ctr("yaobcv,vpw->yaobcpw", X, I);
    X = ctr("yaobcpw,wdz->yaobcpdz", X, Bt);
    X = ctr("yaobcpdz,zq->yaobcpdq", X, C4);
    // ket layer
    X = ctr("yaobcpdz,ylg->glaobcpdz", X, K);
    X = ctr("glaobcpdz,slare->gserobcpdz", X, A);
    X = ctr("gserobcpdz,trcvf->gseobtfvpdz", X, A);
    X = ctr("gseobtfvpdz,zvh->gseobtfpdh", X, Rk);
    // PEPO layer
    X = ctr("gseobtfpdh,gmj->jmseobtfpdh", X, I);
    X = ctr("jmseobtfpdh,sqmonk->jqknebtfpdh", X, O);
    X = ctr("jqknebtfpdh,twnpxu->jqkebwuxfdh", X, O);
    X = ctr("jqkebwuxfdh,hxi->jqkebwufdi", X, Ri);
    // bra layer
    X = ctr("jqkebwufdi,jLJ->JLqkebwufdi", X, Bt);
    X = ctr("JLqkebwufdi,qLbRE->JERkewufdi", X, A);
    X = ctr("JERkewufdi,wRdVF->JEkeFVufi", X, A);
    Tn up2 = ctr("JEkeFVufi,iVH->JEkeFufH", X, Rb);
    // bottom row: [x4, Ad1 Od1 Bd1, Ad2 Od2 Bd2, x3]
    Tn Y = ctr("xy,yas->xas", C4, Rk);
    Y = ctr("xas,sot->xaot", Y, Ri);
    Y = ctr("xaot,tbu->xaobu", Y, Rb);
    Y = ctr("xaobu,ucv->xaobcv", Y, Rk);
    Y = ctr("xaobcv,vpw->xaobcpw", Y, Ri);
    Y = ctr("xaobcpw,wdz->xaobcpdz", Y, Rb);
    Tn bot2 = ctr("xaobcpdz,qz->xaobcpdq", Y, C1);
    Tn v = ctr("JEkeFufH,JekEfuFH->", up2, bot2);
    ctmk::copy(st, v.p, out, 1);
    ws.release(mk);
}

// ---------------------------------------------------------------------------
// context: the shared state (A, configuration) and one worker per network
// ---------------------------------------------------------------------------
struct ctm_ctx {
    ctm_config cfg{};
    double beta = 0.0;
    int D = 0, chi = 0, xmax = 0;
    hipStream_t ust = nullptr;       // the caller's stream
    int device = 0;
    std::vector<void*> owned;        // persistent allocations
    double* A = nullptr;             // D4-projected A, [2][D][D][D][D]
    Net net[2];                      // [0] triple, [1] double
    Worker w[2];                     // one per network
    hipEvent_t ev_fork = nullptr, ev_join[2] = {nullptr, nullptr};
    int iters = 0;
    int base_iters = 0;              // iters at the last ctm_reset_tensor (max_iter counts from here)
    bool lp_done = false;            // reduced-precision phase over (FP64 refinement runs)
    std::string err;

    // spectrum change that ends the reduced-precision phase
    double lp_tol() const
    {
        if (cfg.lp_tol > 0.0) return cfg.lp_tol;
        return cfg.precision == CTM_FP32 ? kLpTolFp32 : kLpTolBf16;
    }

    double* keep(int64_t count)
    {
        void* p = nullptr;
        HIPCHK(hipMalloc(&p, (size_t)std::max<int64_t>(count, 1) * sizeof(double)));
        owned.push_back(p);
        return (double*)p;
    }
    // work on the worker streams starts after everything enqueued so far on
    // the caller's stream ...
    void fork()
    {
        HIPCHK(hipEventRecord(ev_fork, ust));
        for (auto& x : w) HIPCHK(hipStreamWaitEvent(x.st, ev_fork, 0));
    }
    // ... and the caller's stream continues after the worker streams
    void join()
    {
        for (int i = 0; i < 2; ++i) {
            HIPCHK(hipEventRecord(ev_join[i], w[i].st));
            HIPCHK(hipStreamWaitEvent(ust, ev_join[i], 0));
        }
    }
    // worker b continues after what worker a has enqueued so far
    void order(int a, int b)
    {
        HIPCHK(hipEventRecord(ev_join[a], w[a].st));
        HIPCHK(hipStreamWaitEvent(w[b].st, ev_join[a], 0));
    }
    // f(w[0], net[0]) and f(w[1], net[1]) from two host threads
    template <class F>
    void both(F&& f)
    {
        std::exception_ptr e1;
        std::thread t([&] {
            try {
                f(w[1], net[1]);
            } catch (...) {
                e1 = std::current_exception();
            }
        });
        std::exception_ptr e0;
        try {
            f(w[0], net[0]);
        } catch (...) {
            e0 = std::current_exception();
        }
        t.join();
        if (e0) std::rethrow_exception(e0);
        if (e1) std::rethrow_exception(e1);
    }
};

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
static std::string g_init_err = "no error";

template <class F>
static ctm_status guarded(ctm_ctx* c, F&& f)
{
    try {
        f();
        return CTM_OK;
    } catch (const CtmError& e) {
        if (c) c->err = e.what();
        return (ctm_status)e.code;
    } catch (const std::exception& e) {
        if (c) c->err = e.what();
        return CTM_EDEVICE;
    }
}

static void init_net(ctm_ctx* c, Net& N, int d)
{
    N.d = d;
    const int64_t x = c->xmax, D = c->D;
    N.O = c->keep(4 * (int64_t)d * d * d * d);
    N.C1 = c->keep(x * x);
    N.C4 = c->keep(x * x);
    N.Tk = c->keep(x * x * D);
    N.Ti = c->keep(x * x * d);
    N.Tb = c->keep(x * x * D);
    N.s_old = c->keep(x);
    N.n_old = (int*)c->keep(1);
    N.delta = c->keep(1);
    N.sc = c->keep(16);
    N.E = c->keep(2 * D * D * D * D);
    N.sv = c->keep(x);
    if (c->cfg.flags & CTM_FLAG_REDUCED) {
        N.Df = D * d * D;
        N.a = c->keep(N.Df * N.Df * N.Df * N.Df);
        N.Tf = c->keep(x * x * N.Df);
    }
}

static void reset_env(Worker& W, Net& N, int D)
{
    const int64_t d = N.d;
    N.xbk = N.xki = N.xib = 1;
    N.grown = false;
    W.restart();
    if (W.reduced)   // product boundary of the fused legs: T[0, m, 0] = 1/sqrt(Df)
        ctmk::fill(W.st, N.Tf, N.Df, 1.0 / std::sqrt((double)N.Df));
    ctmk::fill(W.st, N.C1, 1, 1.0);
    ctmk::fill(W.st, N.C4, 1, 1.0);
    ctmk::fill(W.st, N.Tk, D, 1.0 / std::sqrt((double)D));
    ctmk::fill(W.st, N.Ti, d, 1.0 / std::sqrt((double)d));
    ctmk::fill(W.st, N.Tb, D, 1.0 / std::sqrt((double)D));
    ctmk::fill(W.st, N.s_old, 1, 1.0);
    int one = 1;
    HIPCHK(hipMemcpyAsync(N.n_old, &one, sizeof(int), hipMemcpyHostToDevice, W.st));
    HIPCHK(hipStreamSynchronize(W.st));
}

// A (host or device) -> D4-projected c->A and the two PEPOs; enqueued on
// worker 0 (worker 1 is ordered after it).  The caller has made sure that no
// earlier work still reads c->A.
static void load_tensor(ctm_ctx* c, double beta, const double* A)
{
    Worker& W = c->w[0];
    const int64_t n = 2 * (int64_t)c->D * c->D * c->D * c->D;
    const Arena::Mark mk = W.ws.mark();
    double* raw = W.ws.alloc(n);
    const bool dev = (c->cfg.flags & CTM_FLAG_DEVICE_PTRS) != 0;
    HIPCHK(hipMemcpyAsync(raw, A, n * sizeof(double), dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, W.st));
    ctmk::d4_project(W.st, raw, c->A, c->D);
    int* flag = (int*)W.ws.alloc(1);
    HIPCHK(hipMemsetAsync(flag, 0, sizeof(int), W.st));
    ctmk::finite_check(W.st, c->A, n, flag);
    int hflag = 0;
    HIPCHK(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, W.st));
    ctmk::ising_pepo(W.st, c->net[0].O, beta);
    ctmk::identity_pepo(W.st, c->net[1].O);
    if (c->cfg.flags & CTM_FLAG_REDUCED)
        for (Net& N : c->net) ctmk::fuse_site(W.st, c->A, N.O, c->D, N.d, N.a);
    HIPCHK(hipStreamSynchronize(W.st));
    W.ws.release(mk);
    c->order(0, 1);
    if (hflag) throw CtmError(CTM_ENUMERIC, "A contains NaN or Inf");
    c->beta = beta;
}

static void sync_workers(ctm_ctx* c)
{
    for (auto& x : c->w) HIPCHK(hipStreamSynchronize(x.st));
}

// Moves of several contexts at once: in every move the two networks of every
// active context step concurrently (one host thread each), then each context
// checks its spectrum change.  n_iter <= 0: each context runs until its
// spectrum change is below tol (with the reduced-precision phase logic) or
// max_iter; n_iter < 0: the same rule for at most -n_iter moves (a slice of
// the run, for schedulers); n_iter > 0: exactly n_iter moves.  Per-context
// results in the arrays (may be NULL); the return value is the first non-OK
// status.
static ctm_status iterate_many(ctm_ctx** cs, int n, int n_iter, int* iters_done, double* last_delta,
                               int* converged, int* status)
{
    const bool until = n_iter <= 0;
    std::vector<int> budget(n), done(n, 0);
    std::vector<double> dl(n, 0.0);
    std::vector<char> active(n, 0), conv(n, 0), capped(n, 0);
    std::vector<int> st(n, CTM_OK);
    for (int i = 0; i < n; ++i) {
        ctm_ctx* c = cs[i];
        // contexts advanced together may share the caller's stream: their side
        // work would queue up behind each other there, so it stays inline
        for (auto& x : c->w) x.side_ok = (n == 1);
        const int left = std::max(0, c->cfg.max_iter - (c->iters - c->base_iters));
        budget[i] = n_iter > 0 ? n_iter : (n_iter == 0 ? left : std::min(left, -n_iter));
        capped[i] = until && budget[i] == left;   // the budget ends at max_iter
        st[i] = guarded(c, [&] { c->fork(); });
        active[i] = st[i] == CTM_OK && budget[i] > 0;
    }
    for (;;) {
        std::vector<int> act;
        for (int i = 0; i < n; ++i)
            if (active[i]) act.push_back(i);
        if (act.empty()) break;
        // one move of every active context
        std::vector<std::exception_ptr> ep(2 * act.size());
        std::vector<std::thread> th;
        auto task = [&](size_t a, int wi) {
            ctm_ctx* c = cs[act[a]];
            try {
                const int64_t chi = (c->iters == 0) ? (int64_t)INT_MAX : (int64_t)c->chi;
                // the reduced-precision forms apply to the triple-layer network;
                // the norm network stays FP64 (it is cheaper, and its
                // environment can be far more sensitive to rounding)
                const int prec = (c->lp_done || wi == 1) ? CTM_FP64 : c->cfg.precision;
                Worker& W = c->w[wi];
                W.bulk = prec;
                W.step(c->net[wi], chi);
                HIPCHK(hipGetLastError());
            } catch (...) {
                ep[2 * a + wi] = std::current_exception();
            }
        };
        for (size_t a = 0; a < act.size(); ++a)
            for (int wi = 0; wi < 2; ++wi)
                if (a + wi > 0) th.emplace_back(task, a, wi);
        task(0, 0);
        for (auto& t : th) t.join();
        for (size_t a = 0; a < act.size(); ++a) {
            const int i = act[a];
            ctm_ctx* c = cs[i];
            st[i] = guarded(c, [&] {
                for (int wi = 0; wi < 2; ++wi)
                    if (ep[2 * a + wi]) std::rethrow_exception(ep[2 * a + wi]);
                const int prec = c->lp_done ? CTM_FP64 : c->cfg.precision;   // of the triple layer
                ++c->iters;
                ++done[i];
                {
                    // every move: the spectrum changes decide convergence and
                    // whether the next move's subspace iterations start warm
                    double h[2];
                    for (int wi = 0; wi < 2; ++wi)
                        HIPCHK(hipMemcpyAsync(&h[wi], c->net[wi].delta, sizeof(double), hipMemcpyDeviceToHost,
                                              c->w[wi].st));
                    sync_workers(c);
                    for (int wi = 0; wi < 2; ++wi) c->w[wi].note_delta(std::isfinite(h[wi]) ? h[wi] : 1.0);
                    dl[i] = std::max(h[0], h[1]);
                    if (!std::isfinite(dl[i])) throw CtmError(CTM_ENUMERIC, "non-finite spectrum");
                    if (until && c->iters > 1) {
                        if (prec == CTM_FP64) {
                            if (dl[i] < c->cfg.tol) conv[i] = 1;
                        } else if (dl[i] < std::max(c->cfg.tol, c->lp_tol())) {
                            // end of the reduced-precision phase: stop, or refine in FP64
                            if (!c->cfg.refine) conv[i] = 1;
                            else c->lp_done = true;
                        } else if (c->cfg.refine && 4 * (c->iters - c->base_iters) >= c->cfg.max_iter) {
                            // the reduced-precision phase gets at most a quarter of max_iter
                            c->lp_done = true;
                        }
                    }
                }
            });
            if (st[i] != CTM_OK || conv[i] || done[i] >= budget[i]) active[i] = 0;
        }
    }
    ctm_status first = CTM_OK;
    for (int i = 0; i < n; ++i) {
        ctm_ctx* c = cs[i];
        const int s2 = guarded(c, [&] {
            c->join();
            HIPCHK(hipStreamSynchronize(c->ust));
        });
        if (st[i] == CTM_OK) st[i] = s2;
        if (st[i] == CTM_OK && capped[i] && !conv[i]) {
            c->err = "max_iter reached before tol";
            st[i] = CTM_ENOCONV;
        }
        if (iters_done) iters_done[i] = done[i];
        if (last_delta) last_delta[i] = dl[i];
        if (converged) converged[i] = conv[i];
        if (status) status[i] = st[i];
        if (first == CTM_OK && st[i] != CTM_OK) first = (ctm_status)st[i];
    }
    return first;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free entry point (ctm_free_energy_noalloc): the
// contraction temporaries of both networks' values (one half each) come from
// this file-scope device array instead of the context's workspace arena,
// which grows by hipMalloc.  Each GPU the library runs on holds its own copy
// until the process ends.  In host code the array's name is a host-side
// stand-in: every host use goes through the per-device address returned by
// hipGetSymbolAddress.  Every call on a GPU shares that GPU's array (calls
// that overlap on one GPU race); nothing in it has to start at zero (every
// temporary is written before it is read).
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static char* g_scratch[kMaxDevices] = {};

// the address of `scratch` on device `device` (looked up once per device,
// with that device current)
static char* scratch_on(int device)
{
    REQUIRE(device >= 0 && device < kMaxDevices, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[device]) {
        int cur = 0;
        HIPCHK(hipGetDevice(&cur));
        HIPCHK(hipSetDevice(device));
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        HIPCHK(hipSetDevice(cur));
        if (e != hipSuccess || p == nullptr)
            throw CtmError(CTM_EDEVICE, "hipGetSymbolAddress of the scratch array failed");
        g_scratch[device] = (char*)p;
    }
    return g_scratch[device];
}

extern "C" {

int ctm_abi_version(void) { return CTM_ABI_VERSION; }

const char* ctm_status_string(int s)
{
    switch (s) {
    case CTM_OK: return "ok";
    case CTM_EINVAL: return "invalid argument";
    case CTM_ENOMEM: return "out of device memory";
    case CTM_EDEVICE: return "HIP device error";
    case CTM_ENOCONV: return "not converged";
    case CTM_ENUMERIC: return "numerical failure";
    case CTM_ESTATE: return "call out of order";
    default: return "unknown status";
    }
}

const char* ctm_last_error(const ctm_ctx* c)
{
    if (!c) return g_init_err.c_str();
    return c->err.c_str();
}

ctm_status ctm_init(const ctm_config* cfg, double beta, const double* A, void* hip_stream, ctm_ctx** out)
{
    if (out) *out = nullptr;
    if (!cfg || !A || !out) { g_init_err = "NULL argument"; return CTM_EINVAL; }
    if (!(beta > 0.0) || !std::isfinite(beta)) { g_init_err = "beta must be > 0"; return CTM_EINVAL; }
    if (cfg->D < 1 || cfg->D > 8) { g_init_err = "D must be in [1, 8]"; return CTM_EINVAL; }
    if (cfg->chi < 1 || cfg->chi > 512) { g_init_err = "chi must be in [1, 512]"; return CTM_EINVAL; }
    if (cfg->tol < 0.0 || cfg->max_iter < 0) { g_init_err = "tol and max_iter must be >= 0"; return CTM_EINVAL; }
    if (cfg->precision != CTM_FP64 && cfg->precision != CTM_FP32 && cfg->precision != CTM_BF16) {
        g_init_err = "precision must be CTM_FP64, CTM_FP32 or CTM_BF16";
        return CTM_EINVAL;
    }
    if (cfg->lp_tol < 0.0) { g_init_err = "lp_tol must be >= 0"; return CTM_EINVAL; }
    if ((cfg->flags & CTM_FLAG_REDUCED) && cfg->precision != CTM_FP64) {
        g_init_err = "the reduced method runs in CTM_FP64 only";
        return CTM_EINVAL;
    }
    ctm_ctx* c = new (std::nothrow) ctm_ctx();
    if (!c) { g_init_err = "host allocation failed"; return CTM_ENOMEM; }
    ctm_status s = guarded(c, [&] {
        c->cfg = *cfg;
        c->D = cfg->D;
        c->chi = cfg->chi;
        c->xmax = std::max(cfg->chi, 2 * 2 * cfg->D * cfg->D);
        c->ust = (hipStream_t)hip_stream;
        HIPCHK(hipGetDevice(&c->device));
        c->A = c->keep(2 * (int64_t)c->D * c->D * c->D * c->D);
        for (auto& x : c->w) {
            x.setup(*cfg, c->D, c->A);
            x.st_side = c->ust;
            if (const char* e = std::getenv("CTM_JACOBI_EXACT_MAX")) {   // testing aid
                x.exact_min = std::atoll(e);
                x.exact_area = x.exact_min * x.exact_min * 4;
            }
            if (const char* e = std::getenv("CTM_TRACE_PERMUTE")) x.trace_perm = std::atoll(e);   // testing aid
            if (const char* e = std::getenv("CTM_LP_CUTOFF")) x.lp_cut = std::atof(e);            // testing aid
            if (std::getenv("CTM_TRACE_GEMM")) x.trace_gemm = true;                                // testing aid
            if (std::getenv("CTM_TRACE_RANKS")) x.trace_ranks = true;                              // testing aid
            if (std::getenv("CTM_NO_WARM_SVD")) x.warm_starts = false;                             // testing aid
            if (std::getenv("CTM_NO_GEMM_GROUP")) x.no_group = true;                               // testing aid
            if (std::getenv("CTM_TRACE_SWEEPS")) x.trace_sweeps = true;                            // testing aid
        }
        HIPCHK(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
        for (auto& e : c->ev_join) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        init_net(c, c->net[0], 2);
        init_net(c, c->net[1], 1);
        c->fork();
        load_tensor(c, beta, A);
        reset_env(c->w[0], c->net[0], c->D);
        reset_env(c->w[1], c->net[1], c->D);
        c->join();
    });
    if (s != CTM_OK) {
        g_init_err = c->err;
        ctm_destroy(c);
        return s;
    }
    *out = c;
    return CTM_OK;
}

ctm_status ctm_iterate(ctm_ctx* c, int n_iter, int* iters_done, double* last_delta)
{
    if (!c) return CTM_EINVAL;
    int st = CTM_OK;
    return iterate_many(&c, 1, n_iter, iters_done, last_delta, nullptr, &st);
}

ctm_status ctm_iterate_batch(ctm_ctx** cs, int n, int n_iter, int* iters_done, double* last_delta,
                             int* converged, int* status)
{
    if (!cs || n < 1 || n > kMaxIterateBatch) return CTM_EINVAL;
    for (int i = 0; i < n; ++i) {
        if (!cs[i]) return CTM_EINVAL;
        for (int j = 0; j < i; ++j)
            if (cs[j] == cs[i]) return CTM_EINVAL;
    }
    std::vector<int> st(n, CTM_OK);
    const ctm_status s = iterate_many(cs, n, n_iter, iters_done, last_delta, converged, st.data());
    if (status)
        for (int i = 0; i < n; ++i) status[i] = st[i];
    return s;
}

ctm_status ctm_free_energy(ctm_ctx* c, double* f, double* lk3, double* lk2)
{
    if (!c) return CTM_EINVAL;
    if (c->iters == 0) { c->err = "no iteration done yet"; return CTM_ESTATE; }
    double h[6] = {0, 0, 0, 0, 0, 0};
    ctm_status s = guarded(c, [&] {
        c->fork();
        c->both([&](Worker& W, Net& N) { W.values(N, false); });
        c->order(1, 0);
        Worker& W = c->w[0];
        ctmk::free_energy(W.st, c->net[0].sc + 4, c->net[1].sc + 4, c->beta, W.scal);
        HIPCHK(hipMemcpyAsync(&h[0], W.scal, sizeof(double), hipMemcpyDeviceToHost, W.st));
        HIPCHK(hipMemcpyAsync(&h[1], c->net[0].sc + 4, 2 * sizeof(double), hipMemcpyDeviceToHost, W.st));
        HIPCHK(hipMemcpyAsync(&h[3], c->net[1].sc + 4, 2 * sizeof(double), hipMemcpyDeviceToHost, W.st));
        HIPCHK(hipStreamSynchronize(W.st));
        c->join();
        if (h[2] != 0.0 || h[4] != 0.0 || !std::isfinite(h[0]))
            throw CtmError(CTM_ENUMERIC, "non-positive or non-finite network value");
    });
    if (s == CTM_OK) {
        if (f) *f = h[0];
        if (lk3) *lk3 = h[1];
        if (lk2) *lk2 = h[3];
    }
    return s;
}

ctm_status ctm_free_energy_noalloc(ctm_ctx* c, double* f, double* lk3, double* lk2)
{
    if (!c) return CTM_EINVAL;
    if (c->iters == 0) { c->err = "no iteration done yet"; return CTM_ESTATE; }
    double h[6] = {0, 0, 0, 0, 0, 0};
    ctm_status s = guarded(c, [&] {
        char* base = scratch_on(c->device);
        const size_t half = kScratchBytes / 2;
        c->w[0].ws.begin_fixed(base, half);
        c->w[1].ws.begin_fixed(base + half, half);
        try {
            c->fork();
            c->both([&](Worker& W, Net& N) { W.values(N, false); });
            c->order(1, 0);
            Worker& W = c->w[0];
            ctmk::free_energy(W.st, c->net[0].sc + 4, c->net[1].sc + 4, c->beta, W.scal);
            HIPCHK(hipMemcpyAsync(&h[0], W.scal, sizeof(double), hipMemcpyDeviceToHost, W.st));
            HIPCHK(hipMemcpyAsync(&h[1], c->net[0].sc + 4, 2 * sizeof(double), hipMemcpyDeviceToHost, W.st));
            HIPCHK(hipMemcpyAsync(&h[3], c->net[1].sc + 4, 2 * sizeof(double), hipMemcpyDeviceToHost, W.st));
            HIPCHK(hipStreamSynchronize(W.st));
            c->join();
        } catch (...) {
            // work already enqueued may still read the scratch: drain it
            for (auto& x : c->w) (void)hipStreamSynchronize(x.st);
            for (auto& x : c->w) x.ws.end_fixed();
            throw;
        }
        for (auto& x : c->w) x.ws.end_fixed();
        if (h[2] != 0.0 || h[4] != 0.0 || !std::isfinite(h[0]))
            throw CtmError(CTM_ENUMERIC, "non-positive or non-finite network value");
    });
    if (s == CTM_OK) {
        if (f) *f = h[0];
        if (lk3) *lk3 = h[1];
        if (lk2) *lk2 = h[3];
    }
    return s;
}

ctm_status ctm_grad(ctm_ctx* c, double* g)
{
    if (!c || !g) return CTM_EINVAL;
    if (c->iters == 0) { c->err = "no iteration done yet"; return CTM_ESTATE; }
    return guarded(c, [&] {
        c->fork();
        c->both([&](Worker& W, Net& N) { W.values(N, true); });
        c->order(1, 0);
        Worker& W = c->w[0];
        const int n = 2 * c->D * c->D * c->D * c->D;
        const Arena::Mark mk = W.ws.mark();
        double* graw = W.ws.alloc(n);
        double* gsym = W.ws.alloc(n);
        ctmk::grad_combine(W.st, c->net[0].E, c->net[0].sc + 6, c->net[1].E, c->net[1].sc + 6,
                           c->beta, graw, n);
        ctmk::d4_project(W.st, graw, gsym, c->D);
        const bool dev = (c->cfg.flags & CTM_FLAG_DEVICE_PTRS) != 0;
        HIPCHK(hipMemcpyAsync(g, gsym, n * sizeof(double), dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, W.st));
        HIPCHK(hipStreamSynchronize(W.st));
        W.ws.release(mk);
        c->join();
    });
}

ctm_status ctm_magnetization(ctm_ctx* c, double* m)
{
    if (!c || !m) return CTM_EINVAL;
    if (c->iters == 0) { c->err = "no iteration done yet"; return CTM_ESTATE; }
    double h[2] = {0.0, 0.0};
    ctm_status s = guarded(c, [&] {
        c->fork();
        Worker& W = c->w[0];
        const Arena::Mark mk = W.ws.mark();
        double* Oz = W.ws.alloc(64);
        double* val = W.ws.alloc(2);
        ctmk::ising_pepo(W.st, Oz, c->beta, ctmk::PEPO_SPIN);
        W.centre_value(c->net[0], Oz, val + 0);
        W.centre_value(c->net[0], c->net[0].O, val + 1);
        HIPCHK(hipMemcpyAsync(h, val, 2 * sizeof(double), hipMemcpyDeviceToHost, W.st));
        HIPCHK(hipStreamSynchronize(W.st));
        W.ws.release(mk);
        c->join();
        if (!(h[1] != 0.0) || !std::isfinite(h[0] / h[1]))
            throw CtmError(CTM_ENUMERIC, "zero or non-finite network value");
    });
    if (s == CTM_OK) *m = h[0] / h[1];
    return s;
}

ctm_status ctm_energy(ctm_ctx* c, double* u)
{
    if (!c || !u) return CTM_EINVAL;
    if (c->iters == 0) { c->err = "no iteration done yet"; return CTM_ESTATE; }
    double h[2] = {0.0, 0.0};
    ctm_status s = guarded(c, [&] {
        c->fork();
        Worker& W = c->w[0];
        const Arena::Mark mk = W.ws.mark();
        double* dO = W.ws.alloc(64);
        double* val = W.ws.alloc(2);
        ctmk::ising_pepo(W.st, dO, c->beta, ctmk::PEPO_DBETA);
        W.centre_value(c->net[0], dO, val + 0);
        W.centre_value(c->net[0], c->net[0].O, val + 1);
        HIPCHK(hipMemcpyAsync(h, val, 2 * sizeof(double), hipMemcpyDeviceToHost, W.st));
        HIPCHK(hipStreamSynchronize(W.st));
        W.ws.release(mk);
        c->join();
        if (!(h[1] != 0.0) || !std::isfinite(h[0] / h[1]))
            throw CtmError(CTM_ENUMERIC, "zero or non-finite network value");
    });
    if (s == CTM_OK) *u = -h[0] / h[1];
    return s;
}

ctm_status ctm_bond_correlation(ctm_ctx* c, double* zz)
{
    if (!c || !zz) return CTM_EINVAL;
    if (c->iters == 0) { c->err = "no iteration done yet"; return CTM_ESTATE; }
    double h[2] = {0.0, 0.0};
    ctm_status s = guarded(c, [&] {
        c->fork();
        Worker& W = c->w[0];
        const Arena::Mark mk = W.ws.mark();
        double* Oz = W.ws.alloc(64);
        double* val = W.ws.alloc(2);
        ctmk::ising_pepo(W.st, Oz, c->beta, ctmk::PEPO_SPIN);
        W.pair_value(c->net[0], Oz, val + 0);
        W.pair_value(c->net[0], c->net[0].O, val + 1);
        HIPCHK(hipMemcpyAsync(h, val, 2 * sizeof(double), hipMemcpyDeviceToHost, W.st));
        HIPCHK(hipStreamSynchronize(W.st));
        W.ws.release(mk);
        c->join();
        if (!(h[1] != 0.0) || !std::isfinite(h[0] / h[1]))
            throw CtmError(CTM_ENUMERIC, "zero or non-finite network value");
    });
    if (s == CTM_OK) *zz = h[0] / h[1];
    return s;
}

ctm_status ctm_corner_spectrum(ctm_ctx* c, int which, double* s, int cap, int* n)
{
    if (!c || !s || !n || (which != 2 && which != 3)) return CTM_EINVAL;
    if (c->iters == 0) { c->err = "no iteration done yet"; return CTM_ESTATE; }
    return guarded(c, [&] {
        const int i = which == 3 ? 0 : 1;
        Net& N = c->net[i];
        hipStream_t st = c->w[i].st;
        c->w[i].exact_spectrum(N);
        int cnt = 0;
        HIPCHK(hipMemcpyAsync(&cnt, N.n_old, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        cnt = std::min(cnt, cap);
        HIPCHK(hipMemcpyAsync(s, N.s_old, cnt * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        *n = cnt;
    });
}

ctm_status ctm_reset_tensor(ctm_ctx* c, double beta, const double* A)
{
    if (!c || !A) return CTM_EINVAL;
    if (!(beta > 0.0)) { c->err = "beta must be > 0"; return CTM_EINVAL; }
    return guarded(c, [&] {
        sync_workers(c);
        c->fork();
        load_tensor(c, beta, A);
        c->join();
        c->lp_done = false;
        c->base_iters = c->iters;
        for (auto& x : c->w) x.restart();   // the first move on the new tensor starts cold
    });
}

ctm_status ctm_query(const ctm_ctx* c, int* total_iters, long long* device_bytes)
{
    if (!c) return CTM_EINVAL;
    if (total_iters) *total_iters = c->iters;
    if (device_bytes) {
        long long b = 0;
        for (const auto& x : c->w) b += (long long)x.ws.bytes_held + (long long)sizeof(double) * x.gws_cap;
        const int64_t xm = c->xmax, D = c->D;
        b += (long long)sizeof(double) * (2 * (2 * xm * xm + 2 * xm * xm * D + xm * xm * 2) + 2 * D * D * D * D);
        *device_bytes = b;
    }
    return CTM_OK;
}

ctm_status ctm_kernel_stats(ctm_ctx* c, int which, long long* launches, double* ms, double* flops,
                            double* bytes)
{
    if (!c || which < 0 || which > 5) return CTM_EINVAL;
    if (!(c->cfg.flags & CTM_FLAG_PROFILE)) { c->err = "context not built with CTM_FLAG_PROFILE"; return CTM_ESTATE; }
    return guarded(c, [&] {
        long long l = 0;
        double t = 0.0, fl = 0.0, by = 0.0;
        for (auto& x : c->w) {
            x.prof_collect();
            l += x.kstat[which].launches;
            t += x.kstat[which].ms;
            fl += x.kstat[which].flops;
            by += x.kstat[which].bytes;
        }
        if (launches) *launches = l;
        if (ms) *ms = t;
        if (flops) *flops = fl;
        if (bytes) *bytes = by;
    });
}

void ctm_destroy(ctm_ctx* c)
{
    if (!c) return;
    for (auto& x : c->w) x.release();
    if (c->ust) (void)hipStreamSynchronize(c->ust);
    for (void* p : c->owned) (void)hipFree(p);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    for (auto& e : c->ev_join)
        if (e) (void)hipEventDestroy(e);
    delete c;
}

}  // extern "C"
