// Host driver of the quad recursion (Algorithm 1, Section 2).
//
// node() follows the algorithm's block steps on the device-resident matrix:
//   PLUQ(A1); PermR(A2, P1^T); PermC(A3, Q1^T);
//   D <- L1^{-1} B1; E <- C1 U1^{-1}  (together: every launch of the two
//                                      solves carries both, one stream);
//   F <- B2 - M1 D; G <- C2 - E V1; H <- A4 - E D        (one grouped MM launch)
//   PLUQ(F); PLUQ(G);
//   H <- P3^T H Q2^T; E <- P3^T E; M1 <- P2^T M1; D <- D Q2^T; V1 <- V1 Q3^T;
//   [I; K] <- [H1; H3] U2^{-1};
//   O <- L3^{-1} (H2 - I V2)   (= N - J V2 with J = L3^{-1} I, N = L3^{-1} H2,
//                               exact over the field, so no copy of I needed);
//   R <- H4 - K V2 - M3 O                                (one MM launch, 2 pairs)
//   PLUQ(R); P4^T [E2 M3 0 K]; [D2; V2; 0; O] Q4^T;
//   A <- S^T A T^T (block rotations of rows and columns).
// A block known to be zero (from the zero flags the MM epilogues raise, or a
// scan) returns rank 0 with identity permutations.  Tiles small enough for
// the LDS go to the base case.  The driver needs the ranks r_i, so it reads
// them back after each base case; permutation vectors are composed on the
// host (they are index bookkeeping) and uploaded only when a permutation is
// not the identity.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <exception>
#include <numeric>
#include <thread>
#include <vector>

#include "driver.hpp"
#include "pluq.h"

namespace pluq {

thread_local Stats g_last_stats;
thread_local Profiler g_prof;
thread_local LaunchEvents g_launch_events;

hipError_t Profiler::begin(hipStream_t st, size_t *idx) {
    while (pool.size() < used + 2) {
        hipEvent_t e;
        hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess) return err;
        pool.push_back(e);
    }
    (void)st;
    *idx = used;
    used += 2;
    g_launch_events.start = pool[*idx];
    g_launch_events.stop = pool[*idx + 1];
    return hipSuccess;
}

hipError_t Profiler::end(hipStream_t st, size_t idx, int cls, double flops, double bytes) {
    (void)st;
    g_launch_events = LaunchEvents();
    pending.push_back({cls, idx, flops, bytes});
    return hipSuccess;
}

void Profiler::resolve() {
    for (const Pending &q : pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, pool[q.e0], pool[q.e0 + 1]) == hipSuccess) {
            k[q.cls].launches++;
            k[q.cls].ms += ms;
            k[q.cls].flops += q.flops;
            k[q.cls].bytes += q.bytes;
        }
    }
    discard();
}

void Profiler::discard() {
    pending.clear();
    used = 0;
}

// ---------------------------------------------------------------- helpers --

static bool is_identity(const std::vector<int32_t> &v) {
    for (size_t i = 0; i < v.size(); ++i)
        if (v[i] != (int32_t)i) return false;
    return true;
}

// A gather map must be a permutation of [0, n): checked before any upload
// so that no kernel can index outside its block.
static void require_permutation(const std::vector<int32_t> &v) {
    std::vector<char> seen(v.size(), 0);
    for (int32_t x : v) {
        if (x < 0 || (size_t)x >= v.size() || seen[(size_t)x]) throw DeviceError{hipErrorInvalidValue};
        seen[(size_t)x] = 1;
    }
}

static void iota(std::vector<int32_t> &v, int64_t n) {
    v.resize((size_t)n);
    std::iota(v.begin(), v.end(), 0);
}

void Ctx::check(hipError_t e) {
    if (e != hipSuccess) throw DeviceError{e};
}

char *Ctx::at(int64_t i, int64_t j) const { return A + ((size_t)i * (size_t)lda + (size_t)j) * esz; }

void Ctx::sync() {
    check(hipStreamSynchronize(st));
    idx_used = 0;
    stats.syncs++;
}

const int32_t *Ctx::upload(const int32_t *v, int64_t n) {
    const size_t need = ((size_t)n + 63) & ~(size_t)63;
    if (idx_used + need > idx_cap) sync();
    if (need > idx_cap) throw DeviceError{hipErrorOutOfMemory};
    std::memcpy(h_idx + idx_used, v, (size_t)n * sizeof(int32_t));
    check(hipMemcpyAsync(d_idx + idx_used, h_idx + idx_used, (size_t)n * sizeof(int32_t),
                         hipMemcpyHostToDevice, st));
    const int32_t *d = d_idx + idx_used;
    idx_used += need;
    return d;
}

// Flag generations never repeat within a thread (the status words it uses
// outlive a call), so a flag left by an earlier call cannot match.
thread_local int32_t g_gen = 0;

int32_t Ctx::next_gen() {
    g_gen = (g_gen % 2000000000) + 1;
    return g_gen;
}

// Completion marker: written after every earlier command of the stream has
// finished (stream order), so the host that sees it sees their results too.
__global__ void mark_kernel(int32_t *w, int32_t gen) {
    if (threadIdx.x == 0) *(volatile int32_t *)w = gen;
}

// Read `count` int32 status words back.  When the kernels write them into
// mapped host memory, a one-thread marker kernel follows them on the stream
// and the host waits for its generation in that memory, which ends sooner
// than a stream synchronisation; past a bounded wait (a device that stopped
// making progress, or a failed launch) it synchronises, which also reports
// any error.  Otherwise the words are copied back and the stream is
// synchronised.
void Ctx::read_status(int64_t offset, int64_t count) {
    if (!stat_mapped) {
        check(hipMemcpyAsync(h_stat + offset, d_stat + offset, (size_t)count * sizeof(int32_t),
                             hipMemcpyDeviceToHost, st));
        sync();
        return;
    }
    const int32_t gen = next_gen();
    hipLaunchKernelGGL(mark_kernel, dim3(1), dim3(64), 0, st, d_stat + STAT_MARK, gen);
    check(hipGetLastError());
    const int32_t *h = h_stat + STAT_MARK;
    const auto t0 = std::chrono::steady_clock::now();
    for (int spin = 0; __atomic_load_n(h, __ATOMIC_ACQUIRE) != gen; ++spin) {
        __builtin_ia32_pause();
        if ((spin & 1023) == 1023 && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(200)) {
            sync();
            if (__atomic_load_n(h, __ATOMIC_ACQUIRE) != gen) throw DeviceError{hipErrorUnknown};
            return;
        }
    }
    idx_used = 0;
    stats.syncs++;
}

// ------------------------------------------------------------ permutations --

// Rows of the nr x nc block at (gi, gj): new row t = old row map[t].
void Ctx::perm_rows(int64_t gi, int64_t gj, int64_t nr, int64_t nc, const std::vector<int32_t> &map) {
    if (nr <= 1 || nc <= 0 || is_identity(map)) return;
    if ((int64_t)map.size() != nr) throw DeviceError{hipErrorInvalidValue};
    require_permutation(map);
    const int32_t *dmap = upload(map.data(), nr);
    const int64_t w = std::max<int64_t>(1, std::min<int64_t>(nc, (int64_t)(scratch_bytes / esz) / nr));
    for (int64_t c0 = 0; c0 < nc; c0 += w) {
        const int64_t cw = std::min(w, nc - c0);
        const double bytes = 2.0 * (double)nr * (double)cw * (double)esz;
        launch(K_PERM, 0, bytes, [&] { return launch_gather2d(dt, at(gi, gj + c0), lda, scratch, cw, nr, cw, dmap, nullptr, st); });
        launch(K_PERM, 0, bytes, [&] { return launch_gather2d(dt, scratch, cw, at(gi, gj + c0), lda, nr, cw, nullptr, nullptr, st); });
    }
}

// Columns of the nr x nc block at (gi, gj): new column t = old column map[t].
void Ctx::perm_cols(int64_t gi, int64_t gj, int64_t nr, int64_t nc, const std::vector<int32_t> &map) {
    if (nc <= 1 || nr <= 0 || is_identity(map)) return;
    if ((int64_t)map.size() != nc) throw DeviceError{hipErrorInvalidValue};
    require_permutation(map);
    const int32_t *dmap = upload(map.data(), nc);
    const int64_t h = std::max<int64_t>(1, std::min<int64_t>(nr, (int64_t)(scratch_bytes / esz) / nc));
    for (int64_t r0 = 0; r0 < nr; r0 += h) {
        const int64_t rh = std::min(h, nr - r0);
        const double bytes = 2.0 * (double)rh * (double)nc * (double)esz;
        launch(K_PERM, 0, bytes, [&] { return launch_gather2d(dt, at(gi + r0, gj), lda, scratch, nc, rh, nc, nullptr, dmap, st); });
        launch(K_PERM, 0, bytes, [&] { return launch_gather2d(dt, scratch, nc, at(gi + r0, gj), lda, rh, nc, nullptr, nullptr, st); });
    }
}

void Ctx::perm_batch(PermJob *jobs, int nj) {
    struct Live {
        PermJob j;
        bool rows, cols;
        size_t bytes;
    };
    std::vector<Live> live;
    live.reserve((size_t)nj);
    for (int q = 0; q < nj; ++q) {
        const PermJob &J = jobs[q];
        const bool r = J.rmap && J.nr > 1 && J.nc > 0 && !is_identity(*J.rmap);
        const bool c = J.cmap && J.nc > 1 && J.nr > 0 && !is_identity(*J.cmap);
        if (!r && !c) continue;
        if ((r && (int64_t)J.rmap->size() != J.nr) || (c && (int64_t)J.cmap->size() != J.nc))
            throw DeviceError{hipErrorInvalidValue};
        if (r) require_permutation(*J.rmap);
        if (c) require_permutation(*J.cmap);
        const size_t bytes = ((size_t)J.nr * (size_t)J.nc * esz + 255) & ~(size_t)255;
        if (bytes > scratch_bytes) {
            // larger than the scratch: strip-mined, one map at a time
            if (r) perm_rows(J.gi, J.gj, J.nr, J.nc, *J.rmap);
            if (c) perm_cols(J.gi, J.gj, J.nr, J.nc, *J.cmap);
            continue;
        }
        live.push_back(Live{J, r, c, bytes});
    }
    std::vector<int32_t> maps;
    size_t q0 = 0;
    while (q0 < live.size()) {
        size_t q1 = q0, used = 0;
        while (q1 < live.size() && q1 - q0 < (size_t)GATHER_MAX_JOBS && used + live[q1].bytes <= scratch_bytes)
            used += live[q1++].bytes;
        // the group's maps in one upload
        maps.clear();
        size_t off[GATHER_MAX_JOBS][2];
        for (size_t q = q0; q < q1; ++q) {
            const Live &L = live[q];
            off[q - q0][0] = maps.size();
            if (L.rows) maps.insert(maps.end(), L.j.rmap->begin(), L.j.rmap->end());
            off[q - q0][1] = maps.size();
            if (L.cols) maps.insert(maps.end(), L.j.cmap->begin(), L.j.cmap->end());
        }
        const int32_t *dmap = upload(maps.data(), (int64_t)maps.size());
        GatherJob to[GATHER_MAX_JOBS], back[GATHER_MAX_JOBS];
        char *sp = scratch;
        double bytes = 0;
        for (size_t q = q0; q < q1; ++q) {
            const Live &L = live[q];
            const int t = (int)(q - q0);
            to[t] = GatherJob{at(L.j.gi, L.j.gj), lda, sp, L.j.nc, L.j.nr, L.j.nc,
                              L.rows ? dmap + off[t][0] : nullptr, L.cols ? dmap + off[t][1] : nullptr, 0, 0, 0};
            back[t] = GatherJob{sp, L.j.nc, at(L.j.gi, L.j.gj), lda, L.j.nr, L.j.nc, nullptr, nullptr, 0, 0, 0};
            sp += L.bytes;
            bytes += 2.0 * (double)L.j.nr * (double)L.j.nc * (double)esz;
        }
        const int n = (int)(q1 - q0);
        launch(K_PERM, 0, bytes, [&] { return launch_gather_jobs(dt, to, n, st); });
        launch(K_PERM, 0, bytes, [&] { return launch_gather_jobs(dt, back, n, st); });
        q0 = q1;
    }
}

// -------------------------------------------------------------------- MM --

void Ctx::mm(MMProblem *probs, int n) {
    int live = 0;
    for (int q = 0; q < n; ++q)
        if (probs[q].M > 0 && probs[q].N > 0 && (probs[q].K[0] > 0 || probs[q].K[1] > 0)) probs[live++] = probs[q];
    if (!live) return;
    if (form != PLUQ_FORM_INT8 && wino && strassen_min > 0) {
        // Large updates take one level of Winograd's scheme (7 block
        // products instead of 8), pair by pair; what stays classical runs
        // afterwards in the grouped launch and then reports non-zero
        // outputs, else the last Winograd pair does.
        int rest = 0;
        for (int q = 0; q < live; ++q) {
            MMProblem pb = probs[q];
            bool w[2] = {false, false};
            for (int s = 0; s < 2; ++s)
                w[s] = pb.K[s] > 0 && pb.inplace == 0 &&
                       std::min<int64_t>(std::min(pb.M, pb.N), pb.K[s]) >= strassen_min &&
                       (size_t)winograd_elems(pb.M, pb.N, pb.K[s]) * esz <= wino_bytes;
            if (!w[0] && !w[1]) {
                probs[rest++] = pb;
                continue;
            }
            const bool classical_left = (pb.K[0] > 0 && !w[0]) || (pb.K[1] > 0 && !w[1]);
            const int last = w[1] ? 1 : 0;
            for (int s = 0; s < 2; ++s) {
                if (!w[s]) continue;
                MMProblem one = pb;
                if (classical_left || s != last) one.nzflag = nullptr;
                mm_winograd(one, s);
                pb.K[s] = 0;
            }
            if (classical_left) probs[rest++] = pb;
        }
        live = rest;
        if (!live) return;
    }
    if (form == PLUQ_FORM_INT8 && limb) {
        // Large updates go to the int8 matrix cores; small ones (latency
        // bound either way) stay in the FP64 kernel, grouped.
        int rest = 0;
        for (int q = 0; q < live; ++q) {
            const MMProblem &pb = probs[q];
            const int64_t K = (int64_t)std::max(pb.K[0], 0) + std::max(pb.K[1], 0);
            const bool big = pb.M >= 128 && pb.N >= 128 && K >= 128 && (double)pb.M * pb.N * K >= i8_min_work;
            if (!(big && mm_i8(pb))) probs[rest++] = pb;
        }
        live = rest;
        if (!live) return;
    }
    mm_launch(probs, live);
}

void Ctx::mm_launch(MMProblem *probs, int live) {
    double flops = 0, bytes = 0;
    for (int q = 0; q < live; ++q) {
        const double M = probs[q].M, N = probs[q].N;
        bytes += 2.0 * M * N;
        for (int s = 0; s < 2; ++s) {
            const double K = probs[q].K[s] > 0 ? probs[q].K[s] : 0;
            flops += 2.0 * M * N * K;
            bytes += M * K + K * N;
        }
    }
    if (form == PLUQ_FORM_FP32)
        launch(K_MODMM, flops, bytes * (double)esz,
               [&] { return launch_modmm_f32(dt, probs, live, (double)p, kchunk32, mm_t128, mm_t64, st); });
    else
        launch(K_MODMM, flops, bytes * (double)esz,
               [&] { return launch_modmm_f64(dt, probs, live, (double)p, kchunk, mm_t128, mm_t64, st); });
}

// One update in the INT8-limb form: the inner dimension (both operand pairs)
// is cut into pieces of at most KMAX_I8 positions (and what the digit-plane
// workspace holds); each piece is split into digit planes and multiplied,
// updating C in place.  Only the last piece reports non-zero outputs.
// Returns false (nothing launched) when the workspace cannot hold one
// 64-deep piece.
bool Ctx::mm_i8(const MMProblem &pb) {
    const int nl = i8_limbs((double)p);
    const int64_t M = pb.M, N = pb.N;
    int64_t ks = (nl > 0) ? (int64_t)(limb_bytes / ((size_t)nl * (size_t)(M + N))) / 64 * 64 : 0;
    ks = std::min<int64_t>(ks, KMAX_I8);
    if (nl == 0 || ks < 64) return false;
    // Pieces of at most ks positions, operand pair 0 then pair 1, taken in
    // order (no list is built: the next piece is formed on demand).
    struct Seg { int pair; int64_t k0, len; };
    int cur_pair = 0;
    int64_t cur_k = 0;
    auto next = [&](Seg &sg) -> bool {
        while (cur_pair < 2 && cur_k >= (int64_t)pb.K[cur_pair]) {
            ++cur_pair;
            cur_k = 0;
        }
        if (cur_pair >= 2) return false;
        sg.pair = cur_pair;
        sg.k0 = cur_k;
        sg.len = std::min<int64_t>(ks, (int64_t)pb.K[cur_pair] - cur_k);
        cur_k += sg.len;
        return true;
    };
    int8_t *a0 = (int8_t *)limb;
    Seg pend;
    bool have = next(pend);
    while (have) {
        // up to two consecutive pieces share a launch while their padded
        // widths fit in ks
        Seg grp[2];
        int ng = 0;
        int64_t kp = 0;
        while (have && ng < 2 && kp + (pend.len + 63) / 64 * 64 <= ks) {
            kp += (pend.len + 63) / 64 * 64;
            grp[ng++] = pend;
            have = next(pend);
        }
        int8_t *a1 = a0 + M * kp, *b0 = a0 + (size_t)nl * M * kp, *b1 = b0 + N * kp;
        SplitJob jobs[SPLIT_MAX_JOBS];
        int nj = 0;
        int64_t koff = 0, klen = 0;
        for (int q = 0; q < ng; ++q) {
            const Seg &sg = grp[q];
            const int64_t w = (sg.len + 63) / 64 * 64;
            SplitJob ja;
            ja.src = (const char *)pb.A[sg.pair] + sg.k0 * (int64_t)esz;
            ja.ld = pb.lda[sg.pair];
            ja.rows = (int32_t)M;
            ja.K = (int32_t)sg.len;
            ja.Kp = (int32_t)w;
            ja.trans = 0;
            ja.dst0 = a0 + koff;
            ja.dst1 = a1 + koff;
            ja.ldd = kp;
            jobs[nj++] = ja;
            SplitJob jb;
            jb.src = (const char *)pb.B[sg.pair] + sg.k0 * pb.ldb[sg.pair] * (int64_t)esz;
            jb.ld = pb.ldb[sg.pair];
            jb.rows = (int32_t)N;
            jb.K = (int32_t)sg.len;
            jb.Kp = (int32_t)w;
            jb.trans = 1;
            jb.dst0 = b0 + koff;
            jb.dst1 = b1 + koff;
            jb.ldd = kp;
            jobs[nj++] = jb;
            koff += w;
            klen += sg.len;
        }
        const double split_bytes = (double)(M + N) * (double)kp * ((double)esz + nl);
        launch(K_LIMB, 0, split_bytes, [&] { return launch_limb_split(dt, jobs, nj, (double)p, st); });
        const bool last = !have;   // only the last piece reports non-zero outputs
        const int8_t *pa[2] = {a0, a1}, *pbp[2] = {b0, b1};
        const double flops = 2.0 * (double)M * (double)N * (double)klen;
        const double bytes = 2.0 * M * N * (double)esz + (double)(M + N) * (double)kp * nl;
        launch(K_MODMM_I8, flops * nl * nl, bytes, [&] {
            return launch_modmm_i8(dt, pb.C, pb.ldc, (int)M, (int)N, (int)kp, pa, pbp, kp, kp, (double)p,
                                   last ? pb.nzflag : nullptr, pb.nzgen, st);
        });
    }
    return true;
}

static MMProblem mmprob(void *C, int64_t ldc, int64_t M, int64_t N) {
    MMProblem pb;
    std::memset(&pb, 0, sizeof(pb));
    pb.C = C;
    pb.ldc = ldc;
    pb.M = (int32_t)M;
    pb.N = (int32_t)N;
    return pb;
}

static void mmpair(MMProblem &pb, int s, const void *A, int64_t lda, const void *B, int64_t ldb, int64_t K) {
    pb.A[s] = A;
    pb.lda[s] = lda;
    pb.B[s] = B;
    pb.ldb[s] = ldb;
    pb.K[s] = (int32_t)K;
}

// ------------------------------------------------------------- Winograd --

// One level of Winograd's form of Strassen's product for C <- C - A B
// (pair s): with the 2 x 2 blocks of floor(M/2) x floor(K/2),
// floor(K/2) x floor(N/2) and floor(M/2) x floor(N/2),
//   S1 = A21 + A22, S2 = S1 - A11, S3 = A11 - A21, S4 = A12 - S2,
//   T1 = B12 - B11, T2 = B22 - T1, T3 = B22 - B12, T4 = T2 - B21,
//   M1 = A11 B11, M2 = A12 B21, M3 = S4 B22, M4 = A22 T4,
//   M5 = S1 T1, M6 = S2 T2, M7 = S3 T3,
//   C11 -= M1 + M2,            C12 -= M1 + M6 + M5 + M3,
//   C21 -= M1 + M6 + M7 - M4,  C22 -= M1 + M6 + M7 + M5.
// Two block products are kept negated (X1 accumulates -(M1 + M6 + M7),
// X3 = -M5); the sums go to two A-shaped and two B-shaped buffers that are
// reused as soon as their last product has run, and M4 is added by
// subtracting A22 (-T4).  Every sum and product is reduced to a canonical
// residue, so the MM kernel's bounds hold as for the inputs and the result
// is exactly the classical one.  A last inner index, row or column left by
// odd sizes is updated classically at the end.
void Ctx::mm_winograd(const MMProblem &pb, int s) {
    const int64_t M = pb.M, N = pb.N, K = pb.K[s];
    const int64_t m2 = M / 2, n2 = N / 2, k2 = K / 2;
    if (m2 < 1 || n2 < 1 || k2 < 1 || (size_t)winograd_elems(M, N, K) * esz > wino_bytes)
        throw DeviceError{hipErrorInvalidValue};
    const int64_t e = (int64_t)esz;
    const char *A = (const char *)pb.A[s], *B = (const char *)pb.B[s];
    char *C = (char *)pb.C;
    const int64_t lda = pb.lda[s], ldb = pb.ldb[s], ldc = pb.ldc;
    auto cblk = [&](const char *base, int64_t ld, int64_t i, int64_t j) { return base + (i * ld + j) * e; };
    auto blk = [&](char *base, int64_t ld, int64_t i, int64_t j) { return base + (i * ld + j) * e; };
    char *Sa = wino, *Sb = Sa + m2 * k2 * e, *Ta = Sb + m2 * k2 * e, *Tb = Ta + k2 * n2 * e;
    char *X1 = Tb + k2 * n2 * e, *X3 = X1 + m2 * n2 * e;
    const char *A11 = cblk(A, lda, 0, 0), *A12 = cblk(A, lda, 0, k2), *A21 = cblk(A, lda, m2, 0),
               *A22 = cblk(A, lda, m2, k2);
    const char *B11 = cblk(B, ldb, 0, 0), *B12 = cblk(B, ldb, 0, n2), *B21 = cblk(B, ldb, k2, 0),
               *B22 = cblk(B, ldb, k2, n2);
    char *C11 = blk(C, ldc, 0, 0), *C12 = blk(C, ldc, 0, n2), *C21 = blk(C, ldc, m2, 0), *C22 = blk(C, ldc, m2, n2);
    // the final values of the even block come from these writers unless a
    // last inner index is still to be added
    int32_t *fin = (K & 1) ? nullptr : pb.nzflag;
    struct Op {
        const char *x;
        int64_t ld;
        int c;
    };
    auto lin = [&](char *out, int64_t ldo, int64_t rows, int64_t cols, Op a, Op b, Op c, int32_t *flag) {
        LinComb l;
        l.out = out;
        l.ldo = ldo;
        const Op ops[3] = {a, b, c};
        int nops = 0;
        for (int t = 0; t < 3; ++t) {
            l.X[t] = ops[t].x;
            l.ld[t] = ops[t].ld;
            l.c[t] = ops[t].c;
            nops += (ops[t].x && ops[t].c) ? 1 : 0;
        }
        l.rows = rows;
        l.cols = cols;
        l.nzflag = flag;
        l.nzgen = pb.nzgen;
        launch(K_LINCOMB, 0, (double)(nops + 1) * (double)rows * (double)cols * (double)esz,
               [&] { return launch_lincomb(dt, l, (double)p, st); });
    };
    const Op none{nullptr, 0, 0};
    auto prod = [&](char *Cb, int64_t ldcb, const char *Ab, int64_t ldab, const char *Bb, int64_t ldbb, int32_t *flag) {
        MMProblem q = mmprob(Cb, ldcb, m2, n2);
        mmpair(q, 0, Ab, ldab, Bb, ldbb, k2);
        q.nzflag = flag;
        q.nzgen = pb.nzgen;
        mm_launch(&q, 1);
    };
    lin(X1, n2, m2, n2, none, none, none, nullptr);                                  // X1 = 0
    prod(X1, n2, A11, lda, B11, ldb, nullptr);                                       // X1 = -M1
    lin(C11, ldc, m2, n2, {C11, ldc, 1}, {X1, n2, 1}, none, nullptr);                // C11 -= M1
    prod(C11, ldc, A12, lda, B21, ldb, fin);                                         // C11 -= M2
    lin(Sa, k2, m2, k2, {A21, lda, 1}, {A22, lda, 1}, none, nullptr);                // S1
    lin(Ta, n2, k2, n2, {B12, ldb, 1}, {B11, ldb, -1}, none, nullptr);               // T1
    lin(X3, n2, m2, n2, none, none, none, nullptr);
    prod(X3, n2, Sa, k2, Ta, n2, nullptr);                                           // X3 = -M5
    lin(Sb, k2, m2, k2, {Sa, k2, 1}, {A11, lda, -1}, none, nullptr);                 // S2
    lin(Tb, n2, k2, n2, {B22, ldb, 1}, {Ta, n2, -1}, none, nullptr);                 // T2
    prod(X1, n2, Sb, k2, Tb, n2, nullptr);                                           // X1 = -(M1 + M6)
    lin(Sa, k2, m2, k2, {A12, lda, 1}, {Sb, k2, -1}, none, nullptr);                 // S4
    lin(C12, ldc, m2, n2, {C12, ldc, 1}, {X1, n2, 1}, {X3, n2, 1}, nullptr);         // C12 -= M1 + M6 + M5
    prod(C12, ldc, Sa, k2, B22, ldb, fin);                                           // C12 -= M3
    lin(Sa, k2, m2, k2, {A11, lda, 1}, {A21, lda, -1}, none, nullptr);               // S3
    lin(Ta, n2, k2, n2, {B22, ldb, 1}, {B12, ldb, -1}, none, nullptr);               // T3
    prod(X1, n2, Sa, k2, Ta, n2, nullptr);                                           // X1 = -(M1 + M6 + M7)
    lin(C22, ldc, m2, n2, {C22, ldc, 1}, {X1, n2, 1}, {X3, n2, 1}, fin);             // C22 -= M1 + M6 + M7 + M5
    lin(Ta, n2, k2, n2, {B21, ldb, 1}, {Tb, n2, -1}, none, nullptr);                 // -T4
    lin(C21, ldc, m2, n2, {C21, ldc, 1}, {X1, n2, 1}, none, nullptr);                // C21 -= M1 + M6 + M7
    prod(C21, ldc, A22, lda, Ta, n2, fin);                                           // C21 += M4
    // leftovers of odd sizes (disjoint parts of C, one grouped launch): the
    // last inner index over the even block, the last row and the last
    // column over the whole inner dimension
    MMProblem rest[3];
    int nr = 0;
    if (K & 1) {
        rest[nr] = mmprob(C, ldc, 2 * m2, 2 * n2);
        mmpair(rest[nr], 0, cblk(A, lda, 0, 2 * k2), lda, cblk(B, ldb, 2 * k2, 0), ldb, 1);
        ++nr;
    }
    if (M & 1) {
        rest[nr] = mmprob(blk(C, ldc, 2 * m2, 0), ldc, 1, N);
        mmpair(rest[nr], 0, cblk(A, lda, 2 * m2, 0), lda, B, ldb, K);
        ++nr;
    }
    if (N & 1) {
        rest[nr] = mmprob(blk(C, ldc, 0, 2 * n2), ldc, 2 * m2, 1);
        mmpair(rest[nr], 0, A, lda, cblk(B, ldb, 0, 2 * n2), ldb, K);
        ++nr;
    }
    for (int q = 0; q < nr; ++q) {
        rest[q].nzflag = pb.nzflag;
        rest[q].nzgen = pb.nzgen;
    }
    if (nr) mm_launch(rest, nr);
}

// ------------------------------------------------------------------ TRSM --

// Split of a triangle of order r > 256: a multiple of 64 near r/2, so that
// every leaf starts on a 64 x 64 diagonal block inverted up front.
static int64_t trsm_split(int64_t r) {
    const int64_t h = (r / 2) - (r / 2) % TRSM_NB;
    return h < TRSM_NB ? TRSM_NB : h;
}

// TRSM(L, B) of Section 2: B (r x ncols, ldb) <- L^{-1} B, L unit lower r x r.
// The diagonal blocks are inverted in one launch; the recursion then runs on
// the matrix cores only: two half solves around an MM update, down to leaves
// of order <= 256 solved in one launch each (block forward substitution with
// the inverted diagonal blocks, one work-group per strip of right-hand sides).
void Ctx::trsm_llu_p(const char *L, int64_t ldl, int64_t r, char *B, int64_t ldb, int64_t ncols) {
    if (r <= 0 || ncols <= 0) return;
    launch(K_TRSM_DIAG, (double)r * TRSM_NB * TRSM_NB / 3.0, (double)r * TRSM_NB * esz * 2,
           [&] { return launch_trsm_diag_inv(dt, 0, L, ldl, r, trsm_w, (double)p, kchunk, st); });
    trsm_llu_rec(L, ldl, r, B, ldb, ncols, 0);
}

void Ctx::trsm_llu_rec(const char *L, int64_t ldl, int64_t r, char *B, int64_t ldb, int64_t ncols, int64_t off) {
    if (r <= TRSM_FUSE_MAX) {
        const char *W = trsm_w + (size_t)(off / TRSM_NB) * TRSM_NB * TRSM_NB * esz;
        launch(K_TRSM, (double)r * r * ncols + 2.0 * TRSM_NB * r * ncols, (0.5 * r * r + 2.0 * r * ncols) * esz,
               [&] { return launch_trsm_leaf(dt, 0, L, ldl, r, B, ldb, ncols, W, (double)p, kchunk, st); });
        return;
    }
    const int64_t r1 = trsm_split(r);
    trsm_llu_rec(L, ldl, r1, B, ldb, ncols, off);
    MMProblem pb = mmprob(B + (size_t)r1 * ldb * esz, ldb, r - r1, ncols);
    mmpair(pb, 0, L + (size_t)r1 * ldl * esz, ldl, B, ldb, r1);
    mm(&pb, 1);
    trsm_llu_rec(L + ((size_t)r1 * ldl + r1) * esz, ldl, r - r1, B + (size_t)r1 * ldb * esz, ldb, ncols, off + r1);
}

// TRSM(B, U) of Section 2: B (nrows x r, ldb) <- B U^{-1}, U upper r x r
// with non-zero diagonal; same scheme, the leaf solving the transposed system.
void Ctx::trsm_run_p(char *B, int64_t ldb, int64_t nrows, const char *U, int64_t ldu, int64_t r) {
    if (r <= 0 || nrows <= 0) return;
    launch(K_TRSM_DIAG, (double)r * TRSM_NB * TRSM_NB / 3.0, (double)r * TRSM_NB * esz * 2,
           [&] { return launch_trsm_diag_inv(dt, 1, U, ldu, r, trsm_w, (double)p, kchunk, st); });
    trsm_run_rec(B, ldb, nrows, U, ldu, r, 0);
}

void Ctx::trsm_run_rec(char *B, int64_t ldb, int64_t nrows, const char *U, int64_t ldu, int64_t r, int64_t off) {
    if (r <= TRSM_FUSE_MAX) {
        const char *W = trsm_w + (size_t)(off / TRSM_NB) * TRSM_NB * TRSM_NB * esz;
        launch(K_TRSM, (double)r * r * nrows + 2.0 * TRSM_NB * r * nrows, (0.5 * r * r + 2.0 * r * nrows) * esz,
               [&] { return launch_trsm_leaf(dt, 1, U, ldu, r, B, ldb, nrows, W, (double)p, kchunk, st); });
        return;
    }
    const int64_t r1 = trsm_split(r);
    trsm_run_rec(B, ldb, nrows, U, ldu, r1, off);
    MMProblem pb = mmprob(B + (size_t)r1 * esz, ldb, nrows, r - r1);
    mmpair(pb, 0, B, ldb, U + (size_t)r1 * esz, ldu, r1);
    mm(&pb, 1);
    trsm_run_rec(B + (size_t)r1 * esz, ldb, nrows, U + ((size_t)r1 * ldu + r1) * esz, ldu, r - r1, off + r1);
}

// The two solves of a node, D <- L^{-1} D (r x ncols at (di, dj)) and
// E <- E U^{-1} (nrows x r at (ei, ej)), with L\U the r x r block at
// (ti, tj): they read and write disjoint blocks and recurse at the same
// split points, so each launch carries both, the diagonal inverses, every
// leaf and every MM update (two problems), on the one stream.
void Ctx::trsm_pair(int64_t ti, int64_t tj, int64_t r, int64_t di, int64_t dj, int64_t ncols, int64_t ei, int64_t ej,
                    int64_t nrows) {
    if (r <= 0) return;
    if (ncols <= 0 || nrows <= 0) {
        if (ncols > 0) trsm_llu(ti, tj, r, di, dj, ncols);
        if (nrows > 0) trsm_run(ei, ej, nrows, ti, tj, r);
        return;
    }
    const char *T = at(ti, tj);
    launch(K_TRSM_DIAG, 2.0 * r * TRSM_NB * TRSM_NB / 3.0, (double)r * TRSM_NB * esz * 4, [&] {
        return launch_trsm_diag_inv_pair(dt, T, lda, T, lda, r, trsm_w, trsm_w2, (double)p, kchunk, st);
    });
    trsm_pair_rec(T, r, at(di, dj), at(ei, ej), ncols, nrows, 0);
}

void Ctx::trsm_pair_rec(const char *T, int64_t r, char *BD, char *BE, int64_t ncols, int64_t nrows, int64_t off) {
    if (r <= TRSM_FUSE_MAX) {
        const size_t wo = (size_t)(off / TRSM_NB) * TRSM_NB * TRSM_NB * esz;
        const double nst = (double)(ncols + nrows);
        launch(K_TRSM, (double)r * r * nst + 2.0 * TRSM_NB * r * nst, (r * r + 2.0 * r * nst) * esz, [&] {
            return launch_trsm_leaf_pair(dt, T, lda, T, lda, r, BD, lda, ncols, BE, lda, nrows, trsm_w + wo,
                                         trsm_w2 + wo, (double)p, kchunk, st);
        });
        return;
    }
    const int64_t r1 = trsm_split(r);
    trsm_pair_rec(T, r1, BD, BE, ncols, nrows, off);
    MMProblem pb[2];
    pb[0] = mmprob(BD + (size_t)r1 * lda * esz, lda, r - r1, ncols);   // D2 -= L21 X1
    mmpair(pb[0], 0, T + (size_t)r1 * lda * esz, lda, BD, lda, r1);
    pb[1] = mmprob(BE + (size_t)r1 * esz, lda, nrows, r - r1);         // E2 -= Y1 U12
    mmpair(pb[1], 0, BE, lda, T + (size_t)r1 * esz, lda, r1);
    mm(pb, 2);
    trsm_pair_rec(T + ((size_t)r1 * lda + r1) * esz, r - r1, BD + (size_t)r1 * lda * esz, BE + (size_t)r1 * esz,
                  ncols, nrows, off + r1);
}

void Ctx::trsm_llu(int64_t li, int64_t lj, int64_t r, int64_t bi, int64_t bj, int64_t ncols) {
    trsm_llu_p(at(li, lj), lda, r, at(bi, bj), lda, ncols);
}

void Ctx::trsm_run(int64_t bi, int64_t bj, int64_t nrows, int64_t ui, int64_t uj, int64_t r) {
    trsm_run_p(at(bi, bj), lda, nrows, at(ui, uj), lda, r);
}

// ------------------------------------------------------------- base case --

// Pivot order of Algorithm 1 for the RPM given by rpm_col (row -> column or
// -1): the recursion visits A1, F, G, R on floor(|rows|/2) x floor(|cols|/2)
// splits of the remaining index sets; a single row or column holds at most
// one pivot.  Appends pivots to (pr, pc).
static void zorder_rec(const std::vector<int32_t> &rows, const std::vector<int32_t> &cols,
                       const std::vector<int32_t> &rpm_col, const std::vector<int32_t> &colpos,
                       std::vector<int32_t> &pr, std::vector<int32_t> &pc, std::vector<int32_t> &mark,
                       int32_t &stamp) {
    if (rows.empty() || cols.empty()) return;
    // mark the columns of this call
    const int32_t my = ++stamp;
    for (int32_t c : cols) mark[c] = my;
    int npiv = 0, last = -1;
    for (int32_t i : rows) {
        const int32_t c = rpm_col[i];
        if (c >= 0 && mark[c] == my) { ++npiv; last = i; }
    }
    if (npiv == 0) return;
    if (rows.size() == 1 || cols.size() == 1) {
        pr.push_back(last);
        pc.push_back(rpm_col[last]);
        return;
    }
    const size_t k = rows.size() / 2, h = cols.size() / 2;
    std::vector<int32_t> r_top(rows.begin(), rows.begin() + k), r_bot(rows.begin() + k, rows.end());
    std::vector<int32_t> c_left(cols.begin(), cols.begin() + h), c_right(cols.begin() + h, cols.end());
    auto minus = [&](const std::vector<int32_t> &src, const std::vector<int32_t> &rem) {
        const int32_t s2 = ++stamp;
        for (int32_t x : rem) mark[x] = s2;
        std::vector<int32_t> out;
        out.reserve(src.size());
        for (int32_t x : src)
            if (mark[x] != s2) out.push_back(x);
        return out;
    };
    (void)colpos;
    const size_t s1 = pr.size();
    zorder_rec(r_top, c_left, rpm_col, colpos, pr, pc, mark, stamp);                 // A1
    const size_t e1 = pr.size();
    std::vector<int32_t> rows1(pr.begin() + s1, pr.begin() + e1), cols1(pc.begin() + s1, pc.begin() + e1);
    zorder_rec(minus(r_top, rows1), c_right, rpm_col, colpos, pr, pc, mark, stamp);  // F
    const size_t e2 = pr.size();
    std::vector<int32_t> cols2(pc.begin() + e1, pc.begin() + e2);
    zorder_rec(r_bot, minus(c_left, cols1), rpm_col, colpos, pr, pc, mark, stamp);   // G
    const size_t e3 = pr.size();
    std::vector<int32_t> rows3(pr.begin() + e2, pr.begin() + e3);
    zorder_rec(minus(r_bot, rows3), minus(c_right, cols2), rpm_col, colpos, pr, pc, mark, stamp);  // R
}

// The same recursion for tiles of at most 128 rows and columns, on 128-bit
// row and column sets (ascending index order is bit order) and fixed arrays:
// no allocation per call.
struct Set128 {
    uint64_t lo = 0, hi = 0;
};
static inline int count128(const Set128 &a) { return __builtin_popcountll(a.lo) + __builtin_popcountll(a.hi); }
static inline bool has128(const Set128 &a, int i) { return i < 64 ? (a.lo >> i) & 1u : (a.hi >> (i - 64)) & 1u; }
static inline void add128(Set128 &a, int i) {
    if (i < 64) a.lo |= 1ull << i;
    else a.hi |= 1ull << (i - 64);
}
static inline Set128 minus128(const Set128 &a, const Set128 &b) { return Set128{a.lo & ~b.lo, a.hi & ~b.hi}; }
// the k lowest members of a
static inline uint64_t lowest64(uint64_t x, int k) {
    if (k >= __builtin_popcountll(x)) return x;
    // b: index of the (k+1)-th lowest member (it exists), found by halving the window
    uint64_t y = x;
    int b = 0;
    for (int w = 32; w >= 1; w >>= 1) {
        const int c = __builtin_popcountll(y & ((1ull << w) - 1));
        if (c <= k) {
            k -= c;
            y >>= w;
            b += w;
        }
    }
    return x & ((1ull << b) - 1);
}
static inline Set128 lowest128(const Set128 &a, int k) {
    const int nlo = __builtin_popcountll(a.lo);
    if (k <= nlo) return Set128{lowest64(a.lo, k), 0};
    return Set128{a.lo, lowest64(a.hi, k - nlo)};
}
struct ZTile {
    const int32_t *rpm_col;
    int32_t pr[128], pc[128];
    int np = 0;
};
static inline Set128 and128(const Set128 &a, const Set128 &b) { return Set128{a.lo & b.lo, a.hi & b.hi}; }
static inline Set128 or128(const Set128 &a, const Set128 &b) { return Set128{a.lo | b.lo, a.hi | b.hi}; }
static inline int top128(const Set128 &a) { return a.hi ? 127 - __builtin_clzll(a.hi) : 63 - __builtin_clzll(a.lo); }
// Emits the pivots of R x C in the recursion's order and returns the sets of
// their rows (rows) and columns (cols).  pc: the rows whose pivot column lies
// in C, so the call's pivots are R & pc and the children's masks follow from
// the pivots alone.
static void zorder_tile(ZTile &z, const Set128 &R, const Set128 &C, const Set128 &pc, Set128 &rows, Set128 &cols) {
    rows = Set128{};
    cols = Set128{};
    const Set128 piv = and128(R, pc);
    if (!piv.lo && !piv.hi) return;
    const int nr = count128(R), nc = count128(C);
    if (nr == 1 || nc == 1 || count128(piv) == 1) {
        // a single row or column holds one pivot; a block with one pivot
        // emits it wherever the splits put it
        const int last = top128(piv);
        z.pr[z.np] = last;
        z.pc[z.np] = z.rpm_col[last];
        ++z.np;
        add128(rows, last);
        add128(cols, z.rpm_col[last]);
        return;
    }
    const Set128 rt = lowest128(R, nr / 2), rb = minus128(R, rt);
    const Set128 cl = lowest128(C, nc / 2), cr = minus128(C, cl);
    Set128 pl;   // pivots of this call whose column lies in cl
    for (int w = 0; w < 2; ++w)
        for (uint64_t x = w ? piv.hi : piv.lo; x; x &= x - 1) {
            const int i = 64 * w + __builtin_ctzll(x);
            if (has128(cl, z.rpm_col[i])) add128(pl, i);
        }
    const Set128 pr = minus128(piv, pl);
    Set128 r1, c1, r2, c2, r3, c3, r4, c4;
    zorder_tile(z, rt, cl, pl, r1, c1);                                               // A1
    zorder_tile(z, minus128(rt, r1), cr, pr, r2, c2);                                 // F
    // the rows paired with a set of pivot columns are the rows emitted with them
    zorder_tile(z, rb, minus128(cl, c1), minus128(pl, r1), r3, c3);                   // G
    zorder_tile(z, minus128(rb, r3), minus128(cr, c2), minus128(pr, r2), r4, c4);     // R
    rows = or128(or128(r1, r2), or128(r3, r4));
    cols = or128(or128(c1, c2), or128(c3, c4));
}

void zorder_from_rpm(int64_t m, int64_t n, const int32_t *rpm_col_in, std::vector<int32_t> &prow,
                     std::vector<int32_t> &pcol) {
    if (m <= 128 && n <= 128) {
        ZTile z;
        z.rpm_col = rpm_col_in;
        Set128 R, C, pc;
        for (int i = 0; i < m; ++i) {
            add128(R, i);
            if (rpm_col_in[i] >= 0 && rpm_col_in[i] < n) add128(pc, i);
        }
        for (int j = 0; j < n; ++j) add128(C, j);
        Set128 rp, cp;
        zorder_tile(z, R, C, pc, rp, cp);
        prow.assign(z.pr, z.pr + z.np);
        pcol.assign(z.pc, z.pc + z.np);
        for (int i = 0; i < m; ++i)
            if (!has128(rp, i)) prow.push_back(i);
        for (int j = 0; j < n; ++j)
            if (!has128(cp, j)) pcol.push_back(j);
        return;
    }
    std::vector<int32_t> rows((size_t)m), cols((size_t)n), rpm(rpm_col_in, rpm_col_in + m), colpos;
    std::iota(rows.begin(), rows.end(), 0);
    std::iota(cols.begin(), cols.end(), 0);
    std::vector<int32_t> pr, pc, mark((size_t)std::max(m, n), 0);
    int32_t stamp = 0;
    // the marks are shared by rows and columns; use separate stamps via one array
    // sized max(m, n): rows and columns are never marked in the same pass.
    zorder_rec(rows, cols, rpm, colpos, pr, pc, mark, stamp);
    std::vector<char> rowp((size_t)m, 0), colp((size_t)n, 0);
    prow = pr;
    pcol = pc;
    for (int32_t x : pr) rowp[x] = 1;
    for (int32_t x : pc) colp[x] = 1;
    for (int64_t i = 0; i < m; ++i)
        if (!rowp[i]) prow.push_back((int32_t)i);
    for (int64_t j = 0; j < n; ++j)
        if (!colp[j]) pcol.push_back((int32_t)j);
}

// Algorithmic flops of eliminating an m x n tile through all min(m, n)
// steps: per step k, the (m-k-1)(n-k-1) multiply-adds of the update and the
// m-k-1 multipliers.
static double bc_flops(int64_t m, int64_t n) {
    double f = 0;
    for (int64_t k = 0; k < std::min(m, n); ++k) f += 2.0 * (double)(m - k - 1) * (double)(n - k - 1) + (double)(m - k - 1);
    return f;
}

int64_t Ctx::basecase(int64_t gi, int64_t gj, int64_t m, int64_t n, std::vector<int32_t> &prow,
                      std::vector<int32_t> &pcol) {
    stats.basecases++;
    const double bflops = bc_flops(m, n);
    if (spec) {
        // full rank in the identity order assumed; checked later
        launch(K_BASE, bflops, 2.0 * m * n * esz, [&] {
            return launch_bc_lu(dt, at(gi, gj), lda, (int)m, (int)n, nullptr, nullptr, -1, (double)p, kchunk, inv_table,
                                d_stat + STAT_BC, d_stat + STAT_SPEC, nullptr, st);
        });
        iota(prow, m);
        iota(pcol, n);
        return std::min(m, n);
    }
    // optimistic: the identity order (generic rank profile)
    const double tbytes = 2.0 * m * n * esz;
    if (opt_fails < 2) {
        launch(K_BASE, bflops, tbytes, [&] {
            return launch_bc_lu(dt, at(gi, gj), lda, (int)m, (int)n, nullptr, nullptr, -1, (double)p, kchunk, inv_table,
                                d_stat + STAT_BC, nullptr, nullptr, st);
        });
        read_status(STAT_BC, 2);
        if (h_stat[STAT_BC + 1] == 1) {
            opt_fails = 0;
            iota(prow, m);
            iota(pcol, n);
            return h_stat[STAT_BC];
        }
        ++opt_fails;
    }
    // general: rank profile matrix, then the pivot order, then the ordered LU
    launch(K_BASE_RPM, bflops, 1.0 * m * n * esz,
           [&] { return launch_bc_rpm(dt, at(gi, gj), lda, (int)m, (int)n, (double)p, kchunk, inv_table, d_stat + STAT_BC, st); });
    read_status(STAT_BC, 1 + m);
    const int64_t r = h_stat[STAT_BC];
    for (int64_t i = 0; i < m; ++i)
        if (h_stat[STAT_BC + 1 + i] < -1 || h_stat[STAT_BC + 1 + i] >= n) throw DeviceError{hipErrorInvalidValue};
    zorder_from_rpm(m, n, h_stat + STAT_BC + 1, prow, pcol);
    if ((int64_t)prow.size() != m || (int64_t)pcol.size() != n) throw DeviceError{hipErrorInvalidValue};
    require_permutation(prow);
    require_permutation(pcol);
    // the identity order again: try the optimistic attempt on the next tile
    bool ident = true;
    for (int64_t i = 0; i < m && ident; ++i) ident = prow[(size_t)i] == i;
    for (int64_t j = 0; j < n && ident; ++j) ident = pcol[(size_t)j] == j;
    if (ident) opt_fails = 0;
    const int32_t *drow = upload(prow.data(), m);
    const int32_t *dcol = upload(pcol.data(), n);
    // The ordered elimination checks itself (r non-zero pivots, zero
    // remainder) into the sticky error flag, which the host reads with the
    // next read-back and at the end instead of waiting for it here.
    launch(K_BASE, bflops, tbytes, [&] {
        return launch_bc_lu(dt, at(gi, gj), lda, (int)m, (int)n, drow, dcol, (int)r, (double)p, kchunk, inv_table,
                            d_stat + STAT_BC, nullptr, d_stat + STAT_ERR, st);
    });
    return r;
}

// ------------------------------------------------------------ zero flags --

// Resolve the zero status of up to 4 blocks with one synchronisation.
void Ctx::resolve_zero(int nb, const Blk *blk, Zero *z, const int32_t *gens) {
    bool need = false;
    int32_t g[8];
    for (int b = 0; b < nb; ++b) {
        g[b] = gens ? gens[b] : 0;
        if (z[b] != Z_UNKNOWN) continue;
        if (blk[b].m <= 0 || blk[b].n <= 0) { z[b] = Z_ZERO; continue; }
        if (!g[b]) {
            g[b] = next_gen();
            launch(K_SCAN, 0, (double)blk[b].m * blk[b].n * esz, [&] {
                return launch_zscan(dt, at(blk[b].i, blk[b].j), lda, blk[b].m, blk[b].n, d_stat + STAT_FLAG + b, g[b], st);
            });
        }
        need = true;
    }
    if (!need) return;
    // in speculative mode the flags may rest on a failed assumption: the
    // speculation flag is read with them and checked first
    read_status(STAT_FLAG, STAT_ERR + 1);
    check_err();
    if (spec && h_stat[STAT_SPEC] != 0) throw SpecFail{};
    for (int b = 0; b < nb; ++b)
        if (z[b] == Z_UNKNOWN) z[b] = (h_stat[STAT_FLAG + b] == g[b]) ? Z_NONZERO : Z_ZERO;
}

void Ctx::check_spec() {
    read_status(STAT_SPEC, 1);
    if (h_stat[STAT_SPEC] != 0) throw SpecFail{};
}

void Ctx::check_err() {
    if (h_stat[STAT_ERR] != 0) throw DeviceError{hipErrorUnknown};
}

// ------------------------------------------------------------------ node --

int64_t Ctx::node(int64_t gi, int64_t gj, int64_t m, int64_t n, Zero z, std::vector<int32_t> &prow,
                  std::vector<int32_t> &pcol) {
    stats.nodes++;
    if (m <= 0 || n <= 0 || z == Z_ZERO) {
        iota(prow, m);
        iota(pcol, n);
        return 0;
    }
    if (m <= cap && n <= cap) return basecase(gi, gj, m, n, prow, pcol);
    if (z == Z_UNKNOWN) {
        Blk b{gi, gj, m, n};
        resolve_zero(1, &b, &z, nullptr);
        if (z == Z_ZERO) {
            iota(prow, m);
            iota(pcol, n);
            return 0;
        }
    }
    const int64_t k = m / 2, h = n / 2;

    // PLUQ(A1)
    std::vector<int32_t> P1, Q1;
    // (a speculative attempt does not test the leading quadrant for zero: a
    // generic rank profile has none, and a zero quadrant fails its tiles)
    const int64_t r1 = node(gi, gj, k, h, spec ? Z_NONZERO : Z_UNKNOWN, P1, Q1);
    {
        PermJob pj[2] = {{gi, gj + h, k, n - h, &P1, nullptr},    // [B1; B2] <- P1^T A2
                         {gi + k, gj, m - k, h, nullptr, &Q1}};   // [C1 C2] <- A3 Q1^T
        perm_batch(pj, 2);
    }

    // F = B2 - M1 D, G = C2 - E V1, H = A4 - E D
    Blk bF{gi + r1, gj + h, k - r1, n - h}, bG{gi + k, gj + r1, m - k, h - r1}, bH{gi + k, gj + h, m - k, n - h};
    Zero zFGH[3] = {Z_UNKNOWN, Z_UNKNOWN, Z_UNKNOWN};
    int32_t gFGH[3] = {0, 0, 0};
    if (r1 > 0) {
        // D <- L1^{-1} B1 and E <- C1 U1^{-1}: independent, solved together
        trsm_pair(gi, gj, r1, gi, gj + h, n - h, gi + k, gj, m - k);
        MMProblem pb[3];
        pb[0] = mmprob(at(bF.i, bF.j), lda, bF.m, bF.n);
        mmpair(pb[0], 0, at(gi + r1, gj), lda, at(gi, gj + h), lda, r1);
        pb[1] = mmprob(at(bG.i, bG.j), lda, bG.m, bG.n);
        mmpair(pb[1], 0, at(gi + k, gj), lda, at(gi, gj + r1), lda, r1);
        pb[2] = mmprob(at(bH.i, bH.j), lda, bH.m, bH.n);
        mmpair(pb[2], 0, at(gi + k, gj), lda, at(gi, gj + h), lda, r1);
        for (int q = 0; q < 3; ++q) {
            gFGH[q] = next_gen();
            pb[q].nzflag = d_stat + STAT_FLAG + q;
            pb[q].nzgen = gFGH[q];
        }
        mm(pb, 3);
    }
    {
        // A non-empty block that fits a base-case tile needs no zero test
        // first: the base case handles a zero tile itself (rank 0, identity
        // order), so only larger blocks are resolved, and a node whose
        // blocks are all small skips the synchronisation.
        Blk bl[3] = {bF, bG, bH};
        Zero zt[3];
        for (int q = 0; q < 3; ++q) {
            const bool small = bl[q].m > 0 && bl[q].n > 0 && bl[q].m <= cap && bl[q].n <= cap;
            zt[q] = small ? Z_NONZERO : zFGH[q];   // Z_NONZERO here only means "not tested"
        }
        resolve_zero(3, bl, zt, r1 > 0 ? gFGH : nullptr);
        for (int q = 0; q < 3; ++q)
            if (!(bl[q].m > 0 && bl[q].n > 0 && bl[q].m <= cap && bl[q].n <= cap)) zFGH[q] = zt[q];
    }

    std::vector<int32_t> P2, Q2, P3, Q3;
    int64_t r2 = 0, r3 = 0;
    node_pair(bF, zFGH[0], bG, zFGH[1], r2, r3, P2, Q2, P3, Q3);      // PLUQ(F), PLUQ(G)

    {
        // five disjoint blocks: rows [r1, k) and [k, m) of columns [0, r1),
        // rows [0, r1) of columns [h, n) and [r1, h), and H
        PermJob pj[5] = {{gi + r1, gj, k - r1, r1, &P2, nullptr},      // M1 <- P2^T M1
                         {gi + k, gj, m - k, r1, &P3, nullptr},        // E  <- P3^T E
                         {gi, gj + h, r1, n - h, nullptr, &Q2},        // D  <- D Q2^T
                         {gi, gj + r1, r1, h - r1, nullptr, &Q3},      // V1 <- V1 Q3^T
                         {gi + k, gj + h, m - k, n - h, &P3, &Q2}};    // H  <- P3^T H Q2^T
        perm_batch(pj, zFGH[2] != Z_ZERO ? 5 : 4);
    }

    // R = H4 - K V2 - M3 O after the solves
    Blk bR{gi + k + r3, gj + h + r2, m - k - r3, n - h - r2};
    Zero zR = (zFGH[2] == Z_ZERO) ? Z_ZERO : Z_UNKNOWN;
    if (zFGH[2] != Z_ZERO) {
        if (r2 > 0) trsm_run(gi + k, gj + h, m - k, gi + r1, gj + h, r2);   // [I; K] <- [H1; H3] U2^{-1}
        if (r3 > 0) {
            if (r2 > 0) {                                                   // H2 <- H2 - I V2
                MMProblem pb = mmprob(at(gi + k, gj + h + r2), lda, r3, n - h - r2);
                mmpair(pb, 0, at(gi + k, gj + h), lda, at(gi + r1, gj + h + r2), lda, r2);
                mm(&pb, 1);
            }
            trsm_llu(gi + k, gj + r1, r3, gi + k, gj + h + r2, n - h - r2);  // O <- L3^{-1} H2
        }
        if (r2 > 0 || r3 > 0) {
            MMProblem pb = mmprob(at(bR.i, bR.j), lda, bR.m, bR.n);
            int s = 0;
            if (r2 > 0) mmpair(pb, s++, at(gi + k + r3, gj + h), lda, at(gi + r1, gj + h + r2), lda, r2);   // K V2
            if (r3 > 0) mmpair(pb, s++, at(gi + k + r3, gj + r1), lda, at(gi + k, gj + h + r2), lda, r3);   // M3 O
            const int32_t gR = next_gen();
            pb.nzflag = d_stat + STAT_FLAG;
            pb.nzgen = gR;
            mm(&pb, 1);
            if (bR.m > cap || bR.n > cap) resolve_zero(1, &bR, &zR, &gR);   // a small R goes to the base case as is
        } else {
            zR = zFGH[2];   // R is H itself
        }
    }

    std::vector<int32_t> P4, Q4;
    const int64_t r4 = node(bR.i, bR.j, bR.m, bR.n, zR, P4, Q4);       // PLUQ(R)
    {
        // disjoint: r1 + r3 <= h and r1 + r2 <= k
        PermJob pj[4] = {{gi + k + r3, gj, m - k - r3, r1 + r3, &P4, nullptr},       // P4^T [E2 M3]
                         {gi + k + r3, gj + h, m - k - r3, r2, &P4, nullptr},        // P4^T K
                         {gi, gj + h + r2, r1 + r2, n - h - r2, nullptr, &Q4},       // [D2; V2] Q4^T
                         {gi + k, gj + h + r2, r3, n - h - r2, nullptr, &Q4}};       // O Q4^T
        perm_batch(pj, 4);
    }

    // S^T A T^T
    {
        const int64_t a = r1 + r2, b = k + r3 + r4;      // row band [a, b)
        if (k > a && b > k) {
            std::vector<int32_t> map;
            map.reserve((size_t)(b - a));
            for (int64_t t = k; t < b; ++t) map.push_back((int32_t)(t - a));
            for (int64_t t = a; t < k; ++t) map.push_back((int32_t)(t - a));
            perm_rows(gi + a, gj, b - a, n, map);
        }
        // columns: c0 [0,r1) c1 [r1,r1+r3) c2 [r1+r3,h) c3 [h,h+r2) c4 [h+r2,h+r2+r4) c5 rest
        // new order c0 c3 c1 c4 c2 c5 over the band [r1, h+r2+r4)
        const int64_t ca = r1, cb = h + r2 + r4;
        std::vector<int32_t> map;
        map.reserve((size_t)(cb - ca));
        for (int64_t t = h; t < h + r2; ++t) map.push_back((int32_t)(t - ca));
        for (int64_t t = r1; t < r1 + r3; ++t) map.push_back((int32_t)(t - ca));
        for (int64_t t = h + r2; t < h + r2 + r4; ++t) map.push_back((int32_t)(t - ca));
        for (int64_t t = r1 + r3; t < h; ++t) map.push_back((int32_t)(t - ca));
        perm_cols(gi, gj + ca, m, cb - ca, map);
    }

    // P = Diag(P1 [I; P2], P3 [I; P4]) S ;  Q = T Diag([I; Q3] Q1, [I; Q4] Q2)
    prow.clear();
    prow.reserve((size_t)m);
    for (int64_t t = 0; t < r1; ++t) prow.push_back(P1[t]);
    for (int64_t t = 0; t < r2; ++t) prow.push_back(P1[r1 + P2[t]]);
    for (int64_t t = 0; t < r3; ++t) prow.push_back((int32_t)(k + P3[t]));
    for (int64_t t = 0; t < r4; ++t) prow.push_back((int32_t)(k + P3[r3 + P4[t]]));
    for (int64_t t = r2; t < k - r1; ++t) prow.push_back(P1[r1 + P2[t]]);
    for (int64_t t = r4; t < m - k - r3; ++t) prow.push_back((int32_t)(k + P3[r3 + P4[t]]));
    pcol.clear();
    pcol.reserve((size_t)n);
    for (int64_t t = 0; t < r1; ++t) pcol.push_back(Q1[t]);
    for (int64_t t = 0; t < r2; ++t) pcol.push_back((int32_t)(h + Q2[t]));
    for (int64_t t = 0; t < r3; ++t) pcol.push_back(Q1[r1 + Q3[t]]);
    for (int64_t t = 0; t < r4; ++t) pcol.push_back((int32_t)(h + Q2[r2 + Q4[t]]));
    for (int64_t t = r3; t < h - r1; ++t) pcol.push_back(Q1[r1 + Q3[t]]);
    for (int64_t t = r4; t < n - h - r2; ++t) pcol.push_back((int32_t)(h + Q2[r2 + Q4[t]]));
    return r1 + r2 + r3 + r4;
}

// ----------------------------------------------------------- branches --

Worker::Worker() {
    th = std::thread([this] {
        std::unique_lock<std::mutex> lock(mu);
        for (;;) {
            cv.wait(lock, [&] { return quit || static_cast<bool>(job); });
            if (!job) return;   // asked to quit with nothing pending
            std::function<void()> j = std::move(job);
            job = nullptr;
            lock.unlock();
            j();
            lock.lock();
            busy = false;
            cv.notify_all();
        }
    });
}

Worker::~Worker() {
    {
        std::lock_guard<std::mutex> lock(mu);
        quit = true;
    }
    cv.notify_all();
    th.join();
}

void Worker::post(std::function<void()> j) {
    {
        std::lock_guard<std::mutex> lock(mu);
        job = std::move(j);
        busy = true;
    }
    cv.notify_all();
}

void Worker::wait() {
    std::unique_lock<std::mutex> lock(mu);
    cv.wait(lock, [&] { return !busy; });
}

int ForkPool::acquire() {
    std::lock_guard<std::mutex> lock(mu);
    for (size_t s = 0; s < busy.size(); ++s)
        if (!busy[s]) {
            busy[s] = 1;
            return (int)s;
        }
    return -1;
}

void ForkPool::release(int s) {
    std::lock_guard<std::mutex> lock(mu);
    busy[(size_t)s] = 0;
}

void Ctx::use_branch(const Branch &b) {
    scratch = b.scratch;
    scratch_bytes = b.scratch_bytes;
    d_idx = b.d_idx;
    idx_cap = b.idx_cap;
    idx_used = 0;
    trsm_w = b.trsm_w;
    trsm_w2 = b.trsm_w2;
    limb = b.limb;
    limb_bytes = b.limb_bytes;
    wino = nullptr;   // the Winograd buffers belong to the caller's branch
    wino_bytes = 0;
    if (!stat_mapped) d_stat = b.d_stat;
}

// F = (k - r1) x (n - h) and G = (m - k) x (h - r1) are disjoint blocks and
// their decompositions independent, so when both are large and a helper
// slot is free, G runs on the slot's helper thread (its own stream, device
// regions and pinned status words; its stream waits for the caller's work
// so far, and the caller's stream waits for G's end) while F runs here.
void Ctx::node_pair(const Blk &bF, Zero zF, const Blk &bG, Zero zG, int64_t &r2, int64_t &r3,
                    std::vector<int32_t> &P2, std::vector<int32_t> &Q2, std::vector<int32_t> &P3,
                    std::vector<int32_t> &Q3) {
    const bool big = pool && zF != Z_ZERO && zG != Z_ZERO && std::min(bF.m, bF.n) >= pool->min_dim &&
                     std::min(bG.m, bG.n) >= pool->min_dim;
    const int s = big ? pool->acquire() : -1;
    if (s < 0) {
        r2 = node(bF.i, bF.j, bF.m, bF.n, zF, P2, Q2);
        r3 = node(bG.i, bG.j, bG.m, bG.n, zG, P3, Q3);
        return;
    }
    Ctx sub = *this;
    sub.st = pool->stream[(size_t)s];
    sub.stats = Stats();
    sub.use_branch(pool->slot[(size_t)s]);
    check(hipEventRecord(pool->ev_start[(size_t)s], st));
    check(hipStreamWaitEvent(sub.st, pool->ev_start[(size_t)s], 0));
    const int32_t mask = g_prof.mask;
    KStat kst[KCLASSES];
    std::exception_ptr sub_err;
    Worker *helper = pool->worker[(size_t)s];
    helper->post([&] {
        try {
            check(hipSetDevice(pool->dev));
            if (!pool->bind_thread(sub)) throw DeviceError{hipErrorOutOfMemory};
            sub.use_branch(pool->slot[(size_t)s]);
            // this branch's sticky flags (failed speculation, base-case
            // self-check) start cleared and are checked at its end
            sub.h_stat[STAT_SPEC] = 0;
            sub.h_stat[STAT_ERR] = 0;
            if (!sub.stat_mapped)
                check(hipMemcpyAsync(sub.d_stat + STAT_SPEC, sub.h_stat + STAT_SPEC, 2 * sizeof(int32_t),
                                     hipMemcpyHostToDevice, sub.st));
            g_prof.discard();
            g_prof.mask = mask;
            for (int c = 0; c < KCLASSES; ++c) g_prof.k[c] = KStat();
            r3 = sub.node(bG.i, bG.j, bG.m, bG.n, zG, P3, Q3);
            sub.read_status(STAT_SPEC, 2);
            sub.check_err();
            if (sub.spec && sub.h_stat[STAT_SPEC] != 0) throw SpecFail{};
            check(hipEventRecord(pool->ev_done[(size_t)s], sub.st));
            if (mask) {
                check(hipStreamSynchronize(sub.st));
                g_prof.resolve();
            }
            for (int c = 0; c < KCLASSES; ++c) kst[c] = g_prof.k[c];
            g_prof.mask = 0;
        } catch (...) {
            sub_err = std::current_exception();
            g_prof.discard();
            (void)hipStreamSynchronize(sub.st);
        }
    });
    try {
        r2 = node(bF.i, bF.j, bF.m, bF.n, zF, P2, Q2);
    } catch (...) {
        helper->wait();
        (void)hipStreamSynchronize(sub.st);
        pool->release(s);
        throw;
    }
    helper->wait();
    pool->release(s);
    if (sub_err) std::rethrow_exception(sub_err);
    check(hipStreamWaitEvent(st, pool->ev_done[(size_t)s], 0));
    stats.nodes += sub.stats.nodes;
    stats.basecases += sub.stats.basecases;
    stats.launches += sub.stats.launches;
    stats.syncs += sub.stats.syncs;
    opt_fails = std::max(opt_fails, sub.opt_fails);
    for (int c = 0; c < KCLASSES; ++c) {
        g_prof.k[c].launches += kst[c].launches;
        g_prof.k[c].ms += kst[c].ms;
        g_prof.k[c].flops += kst[c].flops;
        g_prof.k[c].bytes += kst[c].bytes;
    }
}

}  // namespace pluq
