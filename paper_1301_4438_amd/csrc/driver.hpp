// Internal state of one decomposition call (host side).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <condition_variable>
#include <functional>
#include <memory>
#include <mutex>
#include <thread>
#include <utility>
#include <vector>

#include "kernels.hpp"

namespace pluq {

struct DeviceError {
    hipError_t e;
};
// A speculative decomposition found a base-case tile that is not full rank
// in the identity order (the caller restores the matrix and starts again).
struct SpecFail {};

struct Stats {
    int64_t nodes = 0, basecases = 0, launches = 0, syncs = 0;
};
extern thread_local Stats g_last_stats;

// Per-kernel-class device timing (HIP events), per host thread.
constexpr int KCLASSES = 10;
enum KClass {
    K_MODMM = 0, K_TRSM = 1, K_PERM = 2, K_BASE = 3, K_SCAN = 4, K_LIMB = 5, K_MODMM_I8 = 6, K_TRSM_DIAG = 7,
    K_BASE_RPM = 8, K_LINCOMB = 9
};
struct KStat {
    int64_t launches = 0;
    double ms = 0, flops = 0, bytes = 0;
};
struct Profiler {
    int32_t mask = 0;
    KStat k[KCLASSES];
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    struct Pending {
        int cls;
        size_t e0;
        double flops, bytes;
    };
    std::vector<Pending> pending;
    hipError_t begin(hipStream_t st, size_t *idx);
    hipError_t end(hipStream_t st, size_t idx, int cls, double flops, double bytes);
    void resolve();  // after the stream has been synchronised
    void discard();
};
extern thread_local Profiler g_prof;

// INT8-limb form: updates with fewer multiply-adds than this stay in the FP64
// kernel (a split launch costs more than it saves on small updates).
constexpr double I8_MIN_WORK = 64.0 * 1024 * 1024;

// FP64 / FP32 forms: MM updates whose three dimensions are all at least this
// take one level of Winograd's 7-product scheme (default; tuned).
constexpr int64_t STRASSEN_MIN = 4096;
// Elements of the Winograd buffers for one M x N x K product: two block sums
// of each operand and two block products.
inline int64_t winograd_elems(int64_t M, int64_t N, int64_t K) {
    const int64_t m2 = M / 2, n2 = N / 2, k2 = K / 2;
    return 2 * (m2 * k2 + k2 * n2 + m2 * n2);
}

enum Zero { Z_UNKNOWN = 0, Z_ZERO = 1, Z_NONZERO = 2 };

struct Blk {
    int64_t i, j, m, n;
};

// One permutation of a node's block: the nr x nc block at (gi, gj) gets new
// row t = old row (*rmap)[t] and new column t = old column (*cmap)[t]
// (either map may be null).
struct PermJob {
    int64_t gi, gj, nr, nc;
    const std::vector<int32_t> *rmap, *cmap;
};

// Layout of the int32 status area in device workspace.
constexpr int64_t STAT_FLAG = 0;     // 8 zero-flag slots
constexpr int64_t STAT_SPEC = 8;     // sticky flag: a speculated base case failed
constexpr int64_t STAT_ERR = 9;      // sticky flag: an ordered base case failed its self-check
constexpr int64_t STAT_MARK = 10;    // completion marker of a read-back (generation)
constexpr int64_t STAT_BC = 64;      // base-case status: r, ok / rpm columns
constexpr int64_t STAT_WORDS = 64 + 2 + 16384 + 64;

// Device regions of one recursion branch: every branch (the caller's and
// each helper that runs a PLUQ(G) beside a PLUQ(F)) has its own.
struct Branch {
    char *scratch = nullptr;
    size_t scratch_bytes = 0;
    int32_t *d_idx = nullptr;
    size_t idx_cap = 0;
    int32_t *d_stat = nullptr;    // status words in the workspace (when host memory cannot be mapped)
    char *trsm_w = nullptr, *trsm_w2 = nullptr;
    char *limb = nullptr;
    size_t limb_bytes = 0;
};

struct Ctx;

// A persistent helper thread that runs one posted job at a time (its
// thread-local pinned status words and event pool are set up once and kept).
struct Worker {
    std::thread th;
    std::mutex mu;
    std::condition_variable cv;
    std::function<void()> job;
    bool busy = false, quit = false;
    Worker();
    ~Worker();
    void post(std::function<void()> j);
    void wait();
};

// Helper branches of one decomposition: the independent calls PLUQ(F) and
// PLUQ(G) of a node (Section 9's perspective) run concurrently when a slot
// is free -- G on a helper host thread with the slot's stream and regions.
struct ForkPool {
    std::mutex mu;
    std::vector<Branch> slot;
    std::vector<hipStream_t> stream;
    std::vector<hipEvent_t> ev_start, ev_done;
    std::vector<Worker *> worker;
    std::vector<char> busy;
    int dev = 0;
    int64_t min_dim = 256;   // F and G must both be at least this in each dimension
    // sets up the calling (helper) thread's pinned status words in c
    std::function<bool(Ctx &)> bind_thread;
    int acquire();
    void release(int s);
};

struct Ctx {
    // problem
    int dt = 0;
    size_t esz = 8;
    uint64_t p = 0;
    int form = 0;
    int kchunk = 16;
    int64_t cap = 16384;
    char *A = nullptr;
    int64_t lda = 0;
    hipStream_t st = nullptr;
    // device workspace
    char *scratch = nullptr;
    size_t scratch_bytes = 0;
    int32_t *d_idx = nullptr;
    size_t idx_cap = 0, idx_used = 0;
    int32_t *d_stat = nullptr;
    uint16_t *inv_table = nullptr;   // inverses mod p for the base case (or null)
    char *trsm_w = nullptr;          // I - T_qq^{-1} blocks of the current (or lower) solve
    char *trsm_w2 = nullptr;         // the same for the upper solve of a node's pair
    char *limb = nullptr;            // digit planes of the INT8-limb form (or null)
    size_t limb_bytes = 0;
    char *wino = nullptr;            // Winograd block sums and products (or null)
    size_t wino_bytes = 0;
    int64_t strassen_min = STRASSEN_MIN;
    int kchunk32 = 0;                // FP32 form: products between reductions
    // tuned parameters (performance only)
    int mm_t128 = 240, mm_t64 = 192;    // MM tile choice thresholds
    double i8_min_work = I8_MIN_WORK;  // INT8 form: smaller updates stay in FP64
    // pinned host mirrors
    int32_t *h_idx = nullptr;
    int32_t *h_stat = nullptr;
    bool stat_mapped = false;        // d_stat is h_stat's device address (no copies)
    Stats stats;
    // Speculative mode: every base-case tile is taken to be full rank in the
    // identity order without reading its result back; the tiles record a
    // failed assumption in d_stat[STAT_SPEC], which is read with every zero
    // test and at the end (SpecFail is thrown when it is set).
    bool spec = false;
    // Exact mode: after two tiles in a row failed the identity-order attempt,
    // the next tiles go straight to the rank-profile search, until one comes
    // out in the identity order (inputs far from generic stay so; a single
    // failure, as with a small p where tiles fail at random, does not switch).
    int opt_fails = 0;
    // No per-launch event timing (the entry point that allocates nothing).
    bool noprof = false;
    // Helper branches for PLUQ(F) || PLUQ(G) (null: none).
    ForkPool *pool = nullptr;

    void check(hipError_t e);
    // Issue one kernel launch (f returns its hipError_t), timed when the
    // profiler is on.
    template <class F> void launch(int cls, double flops, double bytes, F f) {
        size_t idx = 0;
        const bool timed = !noprof && ((g_prof.mask >> cls) & 1);
        if (timed) check(g_prof.begin(st, &idx));
        check(f());
        if (timed) check(g_prof.end(st, idx, cls, flops, bytes));
        stats.launches++;
    }
    char *at(int64_t i, int64_t j) const;
    void sync();
    const int32_t *upload(const int32_t *v, int64_t n);
    int32_t next_gen();
    void read_status(int64_t offset, int64_t count);
    void perm_rows(int64_t gi, int64_t gj, int64_t nr, int64_t nc, const std::vector<int32_t> &map);
    void perm_cols(int64_t gi, int64_t gj, int64_t nr, int64_t nc, const std::vector<int32_t> &map);
    // Permutations of disjoint blocks applied together: one map upload, one
    // gather launch into the scratch and one copy back per group of jobs.
    void perm_batch(PermJob *jobs, int nj);
    void mm(MMProblem *probs, int n);
    void mm_launch(MMProblem *probs, int n);   // the classical kernel of the form, no splitting
    bool mm_i8(const MMProblem &pb);
    // C (M x N) <- C - A B by one level of Winograd's scheme (pair s of pb);
    // nzflag / nzgen of pb are set by the writers of C's final values.
    void mm_winograd(const MMProblem &pb, int s);
    void trsm_pair(int64_t ti, int64_t tj, int64_t r, int64_t di, int64_t dj, int64_t ncols, int64_t ei, int64_t ej,
                   int64_t nrows);
    void trsm_pair_rec(const char *T, int64_t r, char *BD, char *BE, int64_t ncols, int64_t nrows, int64_t off);
    void trsm_llu(int64_t li, int64_t lj, int64_t r, int64_t bi, int64_t bj, int64_t ncols);
    void trsm_run(int64_t bi, int64_t bj, int64_t nrows, int64_t ui, int64_t uj, int64_t r);
    void trsm_llu_p(const char *L, int64_t ldl, int64_t r, char *B, int64_t ldb, int64_t ncols);
    void trsm_run_p(char *B, int64_t ldb, int64_t nrows, const char *U, int64_t ldu, int64_t r);
    void trsm_llu_rec(const char *L, int64_t ldl, int64_t r, char *B, int64_t ldb, int64_t ncols, int64_t off);
    void trsm_run_rec(char *B, int64_t ldb, int64_t nrows, const char *U, int64_t ldu, int64_t r, int64_t off);
    int64_t basecase(int64_t gi, int64_t gj, int64_t m, int64_t n, std::vector<int32_t> &prow,
                     std::vector<int32_t> &pcol);
    void resolve_zero(int nb, const Blk *blk, Zero *z, const int32_t *gens);
    void check_spec();   // synchronising read of the speculation flag
    void check_err();    // the error flag among the words just read back
    int64_t node(int64_t gi, int64_t gj, int64_t m, int64_t n, Zero z, std::vector<int32_t> &prow,
                 std::vector<int32_t> &pcol);
    // PLUQ(F) and PLUQ(G) of a node, concurrently when a helper slot is free
    void node_pair(const Blk &bF, Zero zF, const Blk &bG, Zero zG, int64_t &r2, int64_t &r3,
                   std::vector<int32_t> &P2, std::vector<int32_t> &Q2, std::vector<int32_t> &P3,
                   std::vector<int32_t> &Q3);
    void use_branch(const Branch &b);
};

void zorder_from_rpm(int64_t m, int64_t n, const int32_t *rpm_col, std::vector<int32_t> &prow,
                     std::vector<int32_t> &pcol);

}  // namespace pluq
