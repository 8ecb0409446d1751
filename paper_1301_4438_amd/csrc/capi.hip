// extern "C" entry points (declared in include/pluq.h): argument checks,
// workspace carving, pinned host staging, and the top-level call of the
// recursion driver.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "driver.hpp"
#include "pluq.h"

using namespace pluq;

// Scratch of pluq_modmm_noalloc: the INT8 form's digit planes, in a static
// device array (each device holds its own copy for the life of the
// process).  Host code uses only the device address from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) int8_t scratch[NOALLOC_SCRATCH_BYTES];

namespace {

constexpr uint64_t P_MAX = 1ull << 26;
constexpr size_t ALIGN = 256;

size_t align_up(size_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

size_t esize(pluq_dtype dt) {
    switch (dt) {
    case PLUQ_I64: return 8;
    case PLUQ_F64: return 8;
    case PLUQ_I32: return 4;
    }
    return 0;
}

// Largest multiple of 16 such that kchunk * (p/2)^2 + 4p < 2^52.
int64_t fp64_kchunk(uint64_t p) {
    const double half = (double)(p / 2);
    const double lim = 4503599627370496.0 - 4.0 * (double)p;  // 2^52 - 4p
    double k = half > 0 ? lim / (half * half) : 1e18;
    if (k > (double)(1 << 30)) k = (double)(1 << 30);
    int64_t kc = (int64_t)k;
    kc -= kc % 16;
    return kc;
}

// FP32 form: largest multiple of 16 such that kchunk * (p/2)^2 + p < 2^24
// (0 when below 16: the form cannot be exact for this modulus).
int64_t fp32_kchunk(uint64_t p) {
    const double half = (double)(p / 2);
    const double lim = 16777216.0 - (double)p;
    double k = half > 0 ? lim / (half * half) : 1e9;
    if (k > (double)(1 << 30)) k = (double)(1 << 30);
    int64_t kc = (int64_t)k;
    kc -= kc % 16;
    return kc >= 16 ? kc : 0;
}

// Bytes of digit planes for the INT8-limb form of an m x n decomposition:
// enough for one KMAX_I8-deep piece of any update (rows + columns <= m + n).
size_t limb_bytes_for(int64_t m, int64_t n, uint64_t p, int64_t depth = KMAX_I8) {
    const int nl = i8_limbs((double)p);
    const int64_t kmax = std::min<int64_t>((std::min(m, n) + 63) / 64 * 64 + 128, depth);
    return (size_t)nl * (size_t)(m + n) * (size_t)kmax;
}

struct Pinned {
    int32_t *idx = nullptr;
    size_t idx_cap = 0;
    int32_t *stat = nullptr;
    int32_t *stat_dev = nullptr;   // the device's address of `stat`, or null
    int64_t *pq = nullptr;
    size_t pq_cap = 0;
};

thread_local Pinned g_pin;

// Detail of the last failure on this thread (pluq_last_error).
thread_local char g_err[256] = "";

void set_err(const char *where, hipError_t e) {
    std::snprintf(g_err, sizeof(g_err), "%s: %s", where, e == hipSuccess ? "failed" : hipGetErrorString(e));
}

bool ensure_pinned(size_t idx_elems, size_t pq_elems) {
    if (!g_pin.stat) {
        const hipError_t e = hipHostMalloc((void **)&g_pin.stat, STAT_WORDS * sizeof(int32_t), hipHostMallocDefault);
        if (e != hipSuccess) {
            set_err("hipHostMalloc (status words)", e);
            g_pin.stat = nullptr;
            return false;
        }
        // The status words are written by the kernels straight into this
        // (coherent) host memory when the device can address it, so that a
        // read-back is a stream synchronisation with no copy launched.
        void *dp = nullptr;
        if (hipHostGetDevicePointer(&dp, g_pin.stat, 0) == hipSuccess) g_pin.stat_dev = (int32_t *)dp;
        else (void)hipGetLastError();
    }
    if (g_pin.idx_cap < idx_elems) {
        if (g_pin.idx) (void)hipHostFree(g_pin.idx);
        g_pin.idx = nullptr;
        g_pin.idx_cap = 0;
        const hipError_t e = hipHostMalloc((void **)&g_pin.idx, idx_elems * sizeof(int32_t), hipHostMallocDefault);
        if (e != hipSuccess) {
            set_err("hipHostMalloc (index staging)", e);
            return false;
        }
        g_pin.idx_cap = idx_elems;
    }
    if (g_pin.pq_cap < pq_elems) {
        if (g_pin.pq) (void)hipHostFree(g_pin.pq);
        g_pin.pq = nullptr;
        g_pin.pq_cap = 0;
        const hipError_t e = hipHostMalloc((void **)&g_pin.pq, pq_elems * sizeof(int64_t), hipHostMallocDefault);
        if (e != hipSuccess) {
            set_err("hipHostMalloc (permutation staging)", e);
            return false;
        }
        g_pin.pq_cap = pq_elems;
    }
    return true;
}

std::once_flag g_bc_once;
int g_bc_cap = 0;

// Base-case tile dimension (rows and columns at most this).
int bc_cap() {
    std::call_once(g_bc_once, [] { g_bc_cap = (bc_init() == hipSuccess) ? bc_capacity() : 0; });
    return g_bc_cap;
}

struct Layout {
    // branch 0 (the caller's) at offset 0; branch b at b * branch_bytes
    size_t stat_off, idx_off, w_off, w2_off, scratch_off, limb_off, branch_bytes;
    int nbranch;
    size_t tab_off, spec_off, wino_off, total;
    size_t idx_elems, scratch_bytes, tab_bytes, w_bytes, limb_bytes, spec_bytes, wino_bytes;
};

// Largest matrix (bytes) for which the workspace holds a copy of A, taken
// before a speculative decomposition so that a failed one can start again.
constexpr size_t SPEC_MAX_BYTES = (size_t)1 << 30;

// Concurrent recursion branches (PLUQ(F) || PLUQ(G)) by default, and the
// smallest F and G (in each dimension) that are run side by side.
constexpr int DEFAULT_BRANCHES = 8;
constexpr int64_t FORK_MIN_DIM = 128;

// Diagonal-block inverses of a triangle of order r (TRSM).
size_t trsm_w_bytes(int64_t r, size_t esz) {
    return (size_t)((r + TRSM_NB - 1) / TRSM_NB) * TRSM_NB * TRSM_NB * esz;
}

// The in-place variant: permutation strips and digit-plane depth.
constexpr int64_t IN_PLACE_STRIP = 64;
constexpr int64_t IN_PLACE_DEPTH = 512;

bool in_place(const pluq_opts *o) { return o && o->in_place; }

int branches_for(int64_t m, int64_t n, const pluq_opts *o) {
    if (std::min(m, n) < 2 * FORK_MIN_DIM || in_place(o)) return 1;
    const int b = (o && o->branches > 0) ? o->branches : DEFAULT_BRANCHES;
    return std::min(b, 16);
}

// Winograd buffers of the caller's branch: room for the largest update of
// the recursion (at most ceil(m/2) x ceil(n/2), inner dimension at most the
// smaller of the two) when it can reach the tuned threshold smin.
size_t wino_bytes_for(int64_t m, int64_t n, size_t esz, int form, bool inplace, int64_t smin) {
    if (form == PLUQ_FORM_INT8 || inplace || smin <= 0 || std::min(m, n) < 2 * smin) return 0;
    const int64_t mh = (m + 1) / 2, nh = (n + 1) / 2;
    return (size_t)winograd_elems(mh, nh, std::min(mh, nh)) * esz;
}

Layout layout(int64_t m, int64_t n, size_t esz, uint64_t p, int form, bool spec, int nbranch, bool inplace,
              int64_t smin) {
    Layout L;
    L.idx_elems = (size_t)(4 * (m + n) + 65536);
    const size_t full = (size_t)m * (size_t)n * esz;
    const size_t strip = (size_t)IN_PLACE_STRIP * (size_t)std::max<int64_t>(std::max<int64_t>(m, n), 1) * esz;
    // permutations go through strips of this scratch (at least one 64-wide
    // strip of the largest block; 256 MiB unless in place)
    L.scratch_bytes = inplace ? std::min(full, strip) : std::max(std::min(full, (size_t)256 << 20), std::min(full, strip));
    if (L.scratch_bytes == 0) L.scratch_bytes = ALIGN;
    L.w_bytes = trsm_w_bytes(std::min(m, n), esz);
    L.limb_bytes = (form == PLUQ_FORM_INT8 && m > 0 && n > 0)
                       ? limb_bytes_for(m, n, p, inplace ? IN_PLACE_DEPTH : KMAX_I8) : 0;
    if (inplace) spec = false;
    L.stat_off = 0;
    L.idx_off = align_up(STAT_WORDS * sizeof(int32_t));
    L.w_off = L.idx_off + align_up(L.idx_elems * sizeof(int32_t));
    L.w2_off = L.w_off + align_up(L.w_bytes);   // the upper solve of a node's pair
    L.scratch_off = L.w2_off + align_up(L.w_bytes);
    L.limb_off = L.scratch_off + align_up(L.scratch_bytes);
    L.branch_bytes = L.limb_off + align_up(L.limb_bytes);
    L.nbranch = nbranch;
    L.tab_bytes = (p <= 65536) ? BC_TABLE_RESERVE : 0;
    L.tab_off = (size_t)nbranch * L.branch_bytes;
    L.spec_bytes = (spec && full <= SPEC_MAX_BYTES) ? full : 0;
    L.spec_off = L.tab_off + align_up(L.tab_bytes);
    L.wino_bytes = wino_bytes_for(m, n, esz, form, inplace, smin);
    L.wino_off = L.spec_off + align_up(L.spec_bytes);
    L.total = L.wino_off + align_up(L.wino_bytes);
    return L;
}

Branch branch_at(char *w, const Layout &L, int b) {
    char *base = w + (size_t)b * L.branch_bytes;
    Branch br;
    br.d_stat = (int32_t *)(base + L.stat_off);
    br.d_idx = (int32_t *)(base + L.idx_off);
    br.idx_cap = L.idx_elems;
    br.trsm_w = base + L.w_off;
    br.trsm_w2 = base + L.w2_off;
    br.scratch = base + L.scratch_off;
    br.scratch_bytes = L.scratch_bytes;
    if (L.limb_bytes) {
        br.limb = base + L.limb_off;
        br.limb_bytes = L.limb_bytes;
    }
    return br;
}

// Streams and events of the helper branches, created once per calling
// thread and device (default priority) and kept.
struct HelperCache {
    int dev = -1;
    std::vector<hipStream_t> stream;
    std::vector<hipEvent_t> ev;
    std::vector<std::unique_ptr<Worker>> worker;
};
thread_local HelperCache g_help;

bool helpers_ready(int dev, size_t count) {
    if (g_help.dev != dev) {
        g_help = HelperCache();
        g_help.dev = dev;
    }
    while (g_help.stream.size() < count) {
        hipStream_t s = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e != hipSuccess) {
            set_err("hipStreamCreateWithFlags (helper branch)", e);
            return false;
        }
        g_help.stream.push_back(s);
    }
    while (g_help.worker.size() < count) g_help.worker.push_back(std::unique_ptr<Worker>(new Worker()));
    while (g_help.ev.size() < 2 * count) {
        hipEvent_t ev = nullptr;
        hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            set_err("hipEventCreateWithFlags (helper branch)", e);
            return false;
        }
        g_help.ev.push_back(ev);
    }
    return true;
}

pluq_status check_common(int64_t m, int64_t n, int64_t lda, pluq_dtype dt, uint64_t p, const pluq_opts *o) {
    if (m < 0 || n < 0 || m > (1ll << 31) - 2 || n > (1ll << 31) - 2) return PLUQ_ERR_ARG;
    if (esize(dt) == 0) return PLUQ_ERR_ARG;
    if (lda < std::max<int64_t>(1, n)) return PLUQ_ERR_ARG;
    if (p < 2 || p >= P_MAX) return PLUQ_ERR_MODULUS;
    if (o) {
        if (o->form != PLUQ_FORM_FP64 && o->form != PLUQ_FORM_INT8 && o->form != PLUQ_FORM_FP32) return PLUQ_ERR_ARG;
        if (o->cutoff_override < 0 || o->branches < 0) return PLUQ_ERR_ARG;
    }
    return PLUQ_OK;
}

// Every form keeps the FP64 kernels for the triangular-solve inverses and the
// base case, so all of them need the FP64 bound as well.
pluq_status form_check(int form, uint64_t p) {
    if (fp64_kchunk(p) < 16) return PLUQ_ERR_UNSUPPORTED;
    if (form == PLUQ_FORM_FP64) return PLUQ_OK;
    if (form == PLUQ_FORM_INT8) return i8_limbs((double)p) > 0 ? PLUQ_OK : PLUQ_ERR_UNSUPPORTED;
    if (form == PLUQ_FORM_FP32) return fp32_kchunk(p) >= 16 ? PLUQ_OK : PLUQ_ERR_UNSUPPORTED;
    return PLUQ_ERR_ARG;
}



// --------------------------------------------------------------- tuning --

struct TuneEntry {
    int32_t form, pclass, dtype, bucket;
    pluq_tune t;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;

int pclass_of(uint64_t p) { return p <= 256 ? 0 : (p <= 65536 ? 1 : 2); }

constexpr int32_t TUNE_FORM_BATCHED = 3;   // tuning key of the batched form

int bucket_of(int64_t m, int64_t n) {
    int64_t d = std::max<int64_t>(std::min(m, n), 1);
    int b = 0;
    while (d > 1 && b < 31) {
        d >>= 1;
        ++b;
    }
    return b;
}

// The effective parameters: the most specific matching entry, defaults for
// its zero fields.
pluq_tune tune_for(int32_t form, uint64_t p, int32_t dtype, int64_t m, int64_t n, bool *hit) {
    pluq_tune t;
    std::memset(&t, 0, sizeof(t));
    const int pc = pclass_of(p), b = bucket_of(m, n);
    int best = -1;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        for (const TuneEntry &e : g_tune) {
            if ((e.form >= 0 && e.form != form) || (e.pclass >= 0 && e.pclass != pc) ||
                (e.dtype >= 0 && e.dtype != dtype) || (e.bucket >= 0 && e.bucket != b))
                continue;
            const int spec = (e.form >= 0) + (e.pclass >= 0) + (e.dtype >= 0) + (e.bucket >= 0);
            if (spec > best) {
                best = spec;
                t = e.t;
            }
        }
    }
    if (hit) *hit = best >= 0;
    if (t.mm_tiles128 <= 0) t.mm_tiles128 = 240;
    if (t.mm_tiles64 <= 0) t.mm_tiles64 = 192;
    if (t.cutoff <= 0) t.cutoff = 128;
    if (t.fork_min_dim <= 0) t.fork_min_dim = (int32_t)FORK_MIN_DIM;
    if (t.i8_min_work <= 0) t.i8_min_work = (int64_t)I8_MIN_WORK;
    if (t.batch_panel != 8 && t.batch_panel != 16) t.batch_panel = 8;
    if (t.batch_groups <= 0 || t.batch_groups > 8) t.batch_groups = t.batch_panel == 8 ? 4 : 2;
    if (t.strassen_min <= 0) t.strassen_min = (int32_t)STRASSEN_MIN;
    return t;
}

// ---------------------------------------------------- MM building block --

pluq_status modmm_check(int64_t m, int64_t n, int64_t k, const void *dC, int64_t ldc, const void *dA, int64_t lda,
                        const void *dB, int64_t ldb, pluq_dtype dt, uint64_t p, int32_t form) {
    if (m < 0 || n < 0 || k < 0 || m > INT32_MAX || n > INT32_MAX || k > INT32_MAX) return PLUQ_ERR_ARG;
    if (esize(dt) == 0) return PLUQ_ERR_ARG;
    if (p < 2 || p >= P_MAX) return PLUQ_ERR_MODULUS;
    pluq_status s = form_check(form, p);
    if (s != PLUQ_OK) return s;
    if (m == 0 || n == 0) return PLUQ_OK;
    if (!dC || (k > 0 && (!dA || !dB))) return PLUQ_ERR_ARG;
    if (ldc < n || (k > 0 && (lda < k || ldb < n))) return PLUQ_ERR_ARG;
    return PLUQ_OK;
}

// C <- C - A B on the caller's stream; `limb` / `limb_bytes` hold the INT8
// form's digit planes.  noprof: no event timing (nothing is allocated).
// wino / wino_bytes: when given (FP64 / FP32 forms), one level of
// Winograd's scheme with these buffers.
pluq_status modmm_run(int64_t m, int64_t n, int64_t k, void *dC, int64_t ldc, const void *dA, int64_t lda,
                      const void *dB, int64_t ldb, pluq_dtype dt, uint64_t p, int32_t form, char *limb,
                      size_t limb_bytes, bool noprof, void *stream, char *wino = nullptr, size_t wino_bytes = 0) {
    MMProblem pb;
    std::memset(&pb, 0, sizeof(pb));
    pb.C = dC;
    pb.ldc = ldc;
    pb.M = (int32_t)m;
    pb.N = (int32_t)n;
    pb.A[0] = dA;
    pb.lda[0] = lda;
    pb.B[0] = dB;
    pb.ldb[0] = ldb;
    pb.K[0] = (int32_t)k;
    try {
        Ctx c;
        c.dt = (int)dt;
        c.esz = esize(dt);
        c.p = p;
        c.form = form;
        c.kchunk = (int)fp64_kchunk(p);
        c.kchunk32 = (int)fp32_kchunk(p);
        c.st = (hipStream_t)stream;
        c.noprof = noprof;
        const pluq_tune tp = tune_for(form, p, (int32_t)dt, m, n, nullptr);
        c.mm_t128 = tp.mm_tiles128;
        c.mm_t64 = tp.mm_tiles64;
        if (form == PLUQ_FORM_INT8) {
            // the kernel-level entry always takes the int8 path
            c.limb = limb;
            c.limb_bytes = limb_bytes;
            if (!c.mm_i8(pb)) return PLUQ_ERR_WORKSPACE;
        } else if (wino) {
            c.wino = wino;
            c.wino_bytes = wino_bytes;
            c.mm_winograd(pb, 0);
        } else {
            c.mm_launch(&pb, 1);
        }
    } catch (const DeviceError &e) {
        set_err("pluq_modmm: HIP call", e.e);
        return PLUQ_ERR_DEVICE;
    }
    return PLUQ_OK;
}

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

pluq_status scratch_address(char **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
        set_err("pluq_modmm_noalloc: hipGetDevice", e);
        return PLUQ_ERR_DEVICE;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_err("pluq_modmm_noalloc: hipGetSymbolAddress", e);
            return PLUQ_ERR_DEVICE;
        }
        g_scratch_ptr[dev] = (char *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return PLUQ_OK;
}

}  // namespace

extern "C" {

const char *pluq_status_string(pluq_status s) {
    switch (s) {
    case PLUQ_OK: return "ok";
    case PLUQ_ERR_ARG: return "invalid argument";
    case PLUQ_ERR_MODULUS: return "modulus outside [2, 2^26)";
    case PLUQ_ERR_RANGE: return "entry outside [0, p)";
    case PLUQ_ERR_UNSUPPORTED: return "form cannot be exact for this modulus";
    case PLUQ_ERR_NOMEM: return "host allocation failed";
    case PLUQ_ERR_DEVICE: return "device (HIP) error";
    case PLUQ_ERR_WORKSPACE: return "workspace too small";
    }
    return "unknown status";
}

const char *pluq_version(void) { return "pluq-mi355x 0.2 (gfx950)"; }

const char *pluq_last_error(void) { return g_err; }

size_t pluq_workspace_size(int64_t m, int64_t n, pluq_dtype dt, uint64_t p, const pluq_opts *opts) {
    if (check_common(m, n, std::max<int64_t>(1, n), dt, p, opts) != PLUQ_OK) return 0;
    const int form = opts ? opts->form : PLUQ_FORM_FP64;
    const pluq_tune tp = tune_for(form, p, (int32_t)dt, m, n, nullptr);
    return layout(m, n, esize(dt), p, form, !(opts && opts->no_speculation), branches_for(m, n, opts),
                  in_place(opts), tp.strassen_min).total;
}

pluq_status pluq_modp(int64_t m, int64_t n, void *dA, int64_t lda, pluq_dtype dt, uint64_t p, int64_t *dP,
                      int64_t *dQ, int64_t *r_out, const pluq_opts *opts, void *dWork, size_t work_bytes,
                      void *stream) {
    pluq_status s = check_common(m, n, lda, dt, p, opts);
    if (s != PLUQ_OK) return s;
    if (!r_out) return PLUQ_ERR_ARG;
    if (m > 0 && n > 0 && !dA) return PLUQ_ERR_ARG;
    if ((m > 0 && !dP) || (n > 0 && !dQ)) return PLUQ_ERR_ARG;
    const int form = opts ? opts->form : PLUQ_FORM_FP64;
    if ((s = form_check(form, p)) != PLUQ_OK) return s;
    const size_t esz = esize(dt);
    const pluq_tune tp = tune_for(form, p, (int32_t)dt, m, n, nullptr);
    const Layout L = layout(m, n, esz, p, form, !(opts && opts->no_speculation), branches_for(m, n, opts),
                            in_place(opts), tp.strassen_min);
    if (work_bytes < L.total || (m > 0 && n > 0 && !dWork)) return PLUQ_ERR_WORKSPACE;
    if (dWork && ((uintptr_t)dWork % ALIGN)) return PLUQ_ERR_ARG;

    Stats stats;
    try {
        if (!ensure_pinned(L.idx_elems, (size_t)(m + n))) return PLUQ_ERR_NOMEM;
        Ctx c;
        c.dt = (int)dt;
        c.esz = esz;
        c.p = p;
        c.form = form;
        c.kchunk = (int)std::min<int64_t>(fp64_kchunk(p), 1 << 30);
        c.kchunk32 = (int)fp32_kchunk(p);
        c.cap = bc_cap();
        if (c.cap <= 0) return PLUQ_ERR_DEVICE;
        c.mm_t128 = tp.mm_tiles128;
        c.mm_t64 = tp.mm_tiles64;
        c.i8_min_work = (double)tp.i8_min_work;
        c.cap = std::min<int64_t>(c.cap, (opts && opts->cutoff_override > 0) ? opts->cutoff_override : tp.cutoff);
        c.A = (char *)dA;
        c.lda = lda;
        c.st = (hipStream_t)stream;
        char *w = (char *)dWork;
        c.d_stat = (int32_t *)(w + L.stat_off);
        if (g_pin.stat_dev) {
            c.d_stat = g_pin.stat_dev;
            c.stat_mapped = true;
        }
        c.use_branch(branch_at(w, L, 0));
        if (L.wino_bytes) {
            c.wino = w + L.wino_off;
            c.wino_bytes = L.wino_bytes;
            c.strassen_min = tp.strassen_min;
        }
        c.h_idx = g_pin.idx;
        c.h_stat = g_pin.stat;
        // helper branches for PLUQ(F) || PLUQ(G)
        ForkPool pool;
        if (L.nbranch > 1 && m > 0 && n > 0) {
            int dev = 0;
            c.check(hipGetDevice(&dev));
            if (!helpers_ready(dev, (size_t)L.nbranch - 1)) return PLUQ_ERR_DEVICE;
            pool.dev = dev;
            pool.min_dim = tp.fork_min_dim;
            for (int b = 1; b < L.nbranch; ++b) {
                pool.slot.push_back(branch_at(w, L, b));
                pool.stream.push_back(g_help.stream[(size_t)b - 1]);
                pool.ev_start.push_back(g_help.ev[2 * ((size_t)b - 1)]);
                pool.ev_done.push_back(g_help.ev[2 * ((size_t)b - 1) + 1]);
                pool.worker.push_back(g_help.worker[(size_t)b - 1].get());
                pool.busy.push_back(0);
            }
            const size_t idx_elems = L.idx_elems;
            pool.bind_thread = [idx_elems](Ctx &h) {
                if (!ensure_pinned(idx_elems, 0)) return false;
                h.h_idx = g_pin.idx;
                h.h_stat = g_pin.stat;
                h.stat_mapped = g_pin.stat_dev != nullptr;
                if (h.stat_mapped) h.d_stat = g_pin.stat_dev;
                return true;
            };
            c.pool = &pool;
        }
        if (L.tab_bytes && bc_table_bytes((double)p) && m > 0 && n > 0) {
            c.inv_table = (uint16_t *)(w + L.tab_off);
            c.cap = std::min<int64_t>(c.cap, bc_tile_limit((double)p));
            c.launch(K_SCAN, 0, (double)L.tab_bytes, [&] { return launch_build_inv_table(c.inv_table, (double)p, c.st); });
        }

        std::vector<int32_t> prow, pcol;
        int64_t r = 0;
        if (m > 0 && n > 0) {
            if (opts && opts->validate_entries) {
                const int32_t g = c.next_gen();
                c.check(launch_rangescan(c.dt, dA, lda, m, n, (double)p, c.d_stat + STAT_FLAG, g, c.st));
                c.read_status(STAT_FLAG, 1);
                if (c.h_stat[STAT_FLAG] == g) {
                    g_last_stats = c.stats;
                    return PLUQ_ERR_RANGE;
                }
            }
            // Speculative first attempt when the workspace holds a copy of A
            // and there is more than one base-case tile: every tile is taken
            // to be full rank in the identity order (a generic rank profile,
            // Section 5) without reading its result back.  The assumption is
            // checked at every zero test and at the end; if it failed, A is
            // restored and the exact recursion runs from the start.
            // the sticky flags start cleared
            c.h_stat[STAT_SPEC] = 0;
            c.h_stat[STAT_ERR] = 0;
            if (!c.stat_mapped)
                c.check(hipMemcpyAsync(c.d_stat + STAT_SPEC, c.h_stat + STAT_SPEC, 2 * sizeof(int32_t),
                                       hipMemcpyHostToDevice, c.st));
            bool done = false;
            if (L.spec_bytes && (m > c.cap || n > c.cap)) {
                char *backup = w + L.spec_off;
                const double bytes = 2.0 * (double)m * (double)n * (double)esz;
                c.launch(K_PERM, 0, bytes, [&] { return launch_gather2d(c.dt, dA, lda, backup, n, m, n, nullptr, nullptr, c.st); });
                c.spec = true;
                try {
                    // nor is A itself tested for zero first: an all-zero A
                    // fails its first tile and goes to the exact recursion
                    r = c.node(0, 0, m, n, Z_NONZERO, prow, pcol);
                    c.check_spec();
                    done = true;
                } catch (const SpecFail &) {
                    c.launch(K_PERM, 0, bytes, [&] { return launch_gather2d(c.dt, backup, n, dA, lda, m, n, nullptr, nullptr, c.st); });
                    prow.clear();
                    pcol.clear();
                }
                c.spec = false;
            }
            if (!done) r = c.node(0, 0, m, n, Z_UNKNOWN, prow, pcol);
        } else {
            prow.resize((size_t)m);
            pcol.resize((size_t)n);
            for (int64_t i = 0; i < m; ++i) prow[(size_t)i] = (int32_t)i;
            for (int64_t j = 0; j < n; ++j) pcol[(size_t)j] = (int32_t)j;
        }
        // P and Q to the device (int64), one synchronisation for both
        for (int64_t i = 0; i < m; ++i) g_pin.pq[i] = prow[(size_t)i];
        for (int64_t j = 0; j < n; ++j) g_pin.pq[m + j] = pcol[(size_t)j];
        if (m > 0) c.check(hipMemcpyAsync(dP, g_pin.pq, (size_t)m * sizeof(int64_t), hipMemcpyHostToDevice, c.st));
        if (n > 0) c.check(hipMemcpyAsync(dQ, g_pin.pq + m, (size_t)n * sizeof(int64_t), hipMemcpyHostToDevice, c.st));
        if (m > 0 && n > 0) {
            // with the last read-back: the base cases' error flag
            c.read_status(STAT_ERR, 1);
            c.check_err();
            c.sync();   // the stream is idle on return
        } else if (m > 0 || n > 0) {
            c.sync();
        }
        *r_out = r;
        stats = c.stats;
        g_prof.resolve();
    } catch (const DeviceError &e) {
        set_err("pluq_modp: HIP call", e.e);
        g_prof.discard();
        return PLUQ_ERR_DEVICE;
    } catch (const std::bad_alloc &) {
        set_err("pluq_modp: host allocation (std::bad_alloc)", hipSuccess);
        g_prof.discard();
        return PLUQ_ERR_NOMEM;
    }
    g_last_stats = stats;
    return PLUQ_OK;
}

pluq_status pluq_rank_profiles(int64_t m, int64_t n, int64_t r, const int64_t *P, const int64_t *Q,
                               int64_t *row_rp, int64_t *col_rp) {
    if (m < 0 || n < 0 || r < 0 || r > std::min(m, n)) return PLUQ_ERR_ARG;
    if (r > 0 && (!P || !Q || !row_rp || !col_rp)) return PLUQ_ERR_ARG;
    std::copy(P, P + r, row_rp);
    std::copy(Q, Q + r, col_rp);
    std::sort(row_rp, row_rp + r);
    std::sort(col_rp, col_rp + r);
    return PLUQ_OK;
}

pluq_status pluq_leading_rank_profiles(int64_t m, int64_t n, int64_t r, const int64_t *P, const int64_t *Q,
                                       int64_t k, int64_t t, int64_t *rows, int64_t *cols, int64_t *count) {
    if (m < 0 || n < 0 || r < 0 || r > std::min(m, n) || k < 0 || t < 0 || k > m || t > n || !count)
        return PLUQ_ERR_ARG;
    if (r > 0 && (!P || !Q || !rows || !cols)) return PLUQ_ERR_ARG;
    int64_t c = 0;
    for (int64_t s = 0; s < r; ++s)
        if (P[s] < k && Q[s] < t) {
            rows[c] = P[s];
            cols[c] = Q[s];
            ++c;
        }
    std::sort(rows, rows + c);
    std::sort(cols, cols + c);
    *count = c;
    return PLUQ_OK;
}

// Batched workspace: descriptor table, then one backup copy per matrix.
static size_t batched_layout(int64_t batch, const int64_t *m, const int64_t *n, size_t esz,
                             std::vector<int64_t> *woff) {
    size_t off = align_up((size_t)batch * sizeof(BatchDesc));
    const size_t base = off;
    if (woff) woff->resize((size_t)batch);
    for (int64_t b = 0; b < batch; ++b) {
        if (woff) (*woff)[(size_t)b] = (int64_t)(off - base);
        off += align_up((size_t)std::max<int64_t>(m[b], 0) * (size_t)std::max<int64_t>(n[b], 0) * esz);
    }
    return off;
}

static pluq_status batched_check(int64_t batch, const int64_t *m, const int64_t *n, pluq_dtype dt, uint64_t p,
                                 const pluq_opts *opts) {
    if (batch < 0 || batch > INT32_MAX || esize(dt) == 0) return PLUQ_ERR_ARG;
    if (batch > 0 && (!m || !n)) return PLUQ_ERR_ARG;
    if (p < 2 || p >= P_MAX) return PLUQ_ERR_MODULUS;
    if (fp64_kchunk(p) < 16) return PLUQ_ERR_UNSUPPORTED;
    if (opts) {
        if (opts->batch_panel != 0 && opts->batch_panel != 8 && opts->batch_panel != 16) return PLUQ_ERR_ARG;
        if (opts->batch_groups < 0 || opts->batch_groups > 8) return PLUQ_ERR_ARG;
    }
    for (int64_t b = 0; b < batch; ++b) {
        if (m[b] < 0 || n[b] < 0) return PLUQ_ERR_ARG;
        if (m[b] > BATCH_MAX_DIM || n[b] > BATCH_MAX_DIM) return PLUQ_ERR_UNSUPPORTED;
    }
    return PLUQ_OK;
}

size_t pluq_batched_workspace_size(int64_t batch, const int64_t *m, const int64_t *n, pluq_dtype dt, uint64_t p,
                                   const pluq_opts *opts) {
    if (batched_check(batch, m, n, dt, p, opts) != PLUQ_OK) return 0;
    return std::max<size_t>(ALIGN, batched_layout(batch, m, n, esize(dt), nullptr));
}

pluq_status pluq_batched_prepare(int64_t batch, const int64_t *m, const int64_t *n, void *const *dA,
                                 const int64_t *lda, pluq_dtype dt, uint64_t p, int64_t *const *dP,
                                 int64_t *const *dQ, int64_t *d_r, const pluq_opts *opts, void *dWork,
                                 size_t work_bytes) {
    pluq_status s = batched_check(batch, m, n, dt, p, opts);
    if (s != PLUQ_OK) return s;
    if (batch == 0) return PLUQ_OK;
    if (!dA || !lda || !dP || !dQ || !d_r || !dWork) return PLUQ_ERR_ARG;
    if ((uintptr_t)dWork % ALIGN) return PLUQ_ERR_ARG;
    std::vector<int64_t> woff;
    const size_t need = batched_layout(batch, m, n, esize(dt), &woff);
    if (work_bytes < need) return PLUQ_ERR_WORKSPACE;
    for (int64_t b = 0; b < batch; ++b) {
        if (m[b] > 0 && n[b] > 0 && (!dA[b] || lda[b] < n[b])) return PLUQ_ERR_ARG;
        if ((m[b] > 0 && !dP[b]) || (n[b] > 0 && !dQ[b])) return PLUQ_ERR_ARG;
    }
    // largest work first: the persistent work-groups take them round-robin
    std::vector<int64_t> order((size_t)batch);
    for (int64_t b = 0; b < batch; ++b) order[(size_t)b] = b;
    auto cost = [&](int64_t b) { return (double)m[b] * (double)n[b] * (double)std::min(m[b], n[b]); };
    std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return cost(x) > cost(y); });
    std::vector<BatchDesc> desc((size_t)batch);
    for (int64_t q = 0; q < batch; ++q) {
        const int64_t b = order[(size_t)q];
        BatchDesc &d = desc[(size_t)q];
        d.A = dA[b];
        d.lda = std::max<int64_t>(lda[b], 1);
        d.P = dP[b];
        d.Q = dQ[b];
        d.R = d_r + b;
        d.woff = woff[(size_t)b];
        d.m = (int32_t)m[b];
        d.n = (int32_t)n[b];
    }
    if (hipMemcpy(dWork, desc.data(), desc.size() * sizeof(BatchDesc), hipMemcpyHostToDevice) != hipSuccess)
        return PLUQ_ERR_DEVICE;
    return PLUQ_OK;
}

pluq_status pluq_batched_run(int64_t batch, pluq_dtype dt, uint64_t p, const pluq_opts *opts, void *dWork,
                             size_t work_bytes, void *stream) {
    if (batch < 0 || batch > INT32_MAX || esize(dt) == 0) return PLUQ_ERR_ARG;
    if (p < 2 || p >= P_MAX) return PLUQ_ERR_MODULUS;
    if (fp64_kchunk(p) < 16) return PLUQ_ERR_UNSUPPORTED;
    if (batch == 0) return PLUQ_OK;
    if (!dWork || (uintptr_t)dWork % ALIGN || work_bytes < align_up((size_t)batch * sizeof(BatchDesc)))
        return PLUQ_ERR_ARG;
    // explicit options, else the tuned entry of the batched form (key form 3)
    const pluq_tune tb = tune_for(TUNE_FORM_BATCHED, p, (int32_t)dt, 0, 0, nullptr);
    const int kb = (opts && opts->batch_panel) ? opts->batch_panel : tb.batch_panel;
    const int per_cu = (opts && opts->batch_groups) ? opts->batch_groups
                                                     : ((opts && opts->batch_panel && opts->batch_panel != tb.batch_panel)
                                                            ? (kb == 8 ? 4 : 2) : tb.batch_groups);
    if ((kb != 8 && kb != 16) || per_cu < 1 || per_cu > 8) return PLUQ_ERR_ARG;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return PLUQ_ERR_DEVICE;
    const int grid = (int)std::min<int64_t>(batch, (int64_t)cus * per_cu);
    char *w = (char *)dWork;
    const hipError_t e = launch_batched_pluq((int)dt, kb, (const BatchDesc *)w, (int32_t)batch,
                                             w + align_up((size_t)batch * sizeof(BatchDesc)), (double)p, grid,
                                             (hipStream_t)stream);
    return e == hipSuccess ? PLUQ_OK : PLUQ_ERR_DEVICE;
}

pluq_status pluq_modp_batched(int64_t batch, const int64_t *m, const int64_t *n, void *const *dA,
                              const int64_t *lda, pluq_dtype dt, uint64_t p, int64_t *const *dP,
                              int64_t *const *dQ, int64_t *d_r, const pluq_opts *opts, void *dWork,
                              size_t work_bytes, void *stream) {
    pluq_status s = pluq_batched_prepare(batch, m, n, dA, lda, dt, p, dP, dQ, d_r, opts, dWork, work_bytes);
    if (s != PLUQ_OK) return s;
    return pluq_batched_run(batch, dt, p, opts, dWork, work_bytes, stream);
}

size_t pluq_modmm_workspace_size(int64_t m, int64_t n, int64_t k, int32_t form) {
    if (m < 0 || n < 0 || k < 0) return 0;
    if (form != PLUQ_FORM_INT8 || m == 0 || n == 0 || k == 0) return 0;
    // two digit planes of one KMAX_I8-deep piece of A and B
    return align_up((size_t)2 * (size_t)(m + n) * (size_t)std::min<int64_t>((k + 63) / 64 * 64, KMAX_I8));
}

pluq_status pluq_modmm(int64_t m, int64_t n, int64_t k, void *dC, int64_t ldc, const void *dA, int64_t lda,
                       const void *dB, int64_t ldb, pluq_dtype dt, uint64_t p, int32_t form, void *dWork,
                       size_t work_bytes, void *stream) {
    pluq_status s = modmm_check(m, n, k, dC, ldc, dA, lda, dB, ldb, dt, p, form);
    if (s != PLUQ_OK || m == 0 || n == 0 || k == 0) return s;
    const size_t need = pluq_modmm_workspace_size(m, n, k, form);
    if (need && (!dWork || work_bytes < need)) return PLUQ_ERR_WORKSPACE;
    if (need && ((uintptr_t)dWork % ALIGN)) return PLUQ_ERR_ARG;
    return modmm_run(m, n, k, dC, ldc, dA, lda, dB, ldb, dt, p, form, (char *)dWork, work_bytes, false, stream);
}

size_t pluq_modmm_winograd_workspace_size(int64_t m, int64_t n, int64_t k, pluq_dtype dt) {
    if (m < 2 || n < 2 || k < 2 || esize(dt) == 0) return 0;
    return align_up((size_t)winograd_elems(m, n, k) * esize(dt));
}

pluq_status pluq_modmm_winograd(int64_t m, int64_t n, int64_t k, void *dC, int64_t ldc, const void *dA,
                                int64_t lda, const void *dB, int64_t ldb, pluq_dtype dt, uint64_t p, int32_t form,
                                void *dWork, size_t work_bytes, void *stream) {
    pluq_status s = modmm_check(m, n, k, dC, ldc, dA, lda, dB, ldb, dt, p, form);
    if (s != PLUQ_OK) return s;
    if (form == PLUQ_FORM_INT8) return PLUQ_ERR_UNSUPPORTED;
    if (m < 2 || n < 2 || k < 2) return PLUQ_ERR_ARG;
    const size_t need = pluq_modmm_winograd_workspace_size(m, n, k, dt);
    if (!dWork || work_bytes < need) return PLUQ_ERR_WORKSPACE;
    if ((uintptr_t)dWork % ALIGN) return PLUQ_ERR_ARG;
    return modmm_run(m, n, k, dC, ldc, dA, lda, dB, ldb, dt, p, form, nullptr, 0, false, stream, (char *)dWork,
                     work_bytes);
}

pluq_status pluq_modmm_noalloc(int64_t m, int64_t n, int64_t k, void *dC, int64_t ldc, const void *dA, int64_t lda,
                               const void *dB, int64_t ldb, pluq_dtype dt, uint64_t p, int32_t form,
                               void *stream) {
    pluq_status s = modmm_check(m, n, k, dC, ldc, dA, lda, dB, ldb, dt, p, form);
    if (s != PLUQ_OK || m == 0 || n == 0 || k == 0) return s;
    if (form != PLUQ_FORM_INT8)
        return modmm_run(m, n, k, dC, ldc, dA, lda, dB, ldb, dt, p, form, nullptr, 0, true, stream);
    // the digit planes of one 64-deep piece must fit in the static scratch
    const size_t nl = (size_t)i8_limbs((double)p);
    if (nl * (size_t)(m + n) * 64 > NOALLOC_SCRATCH_BYTES) {
        std::snprintf(g_err, sizeof(g_err),
                      "pluq_modmm_noalloc: m + n = %lld above %lld, the most its static scratch serves",
                      (long long)(m + n), (long long)(NOALLOC_SCRATCH_BYTES / (nl * 64)));
        return PLUQ_ERR_WORKSPACE;
    }
    char *ptr = nullptr;
    if ((s = scratch_address(&ptr)) != PLUQ_OK) return s;
    return modmm_run(m, n, k, dC, ldc, dA, lda, dB, ldb, dt, p, form, ptr, NOALLOC_SCRATCH_BYTES, true, stream);
}

size_t pluq_trsm_workspace_size(int64_t r, pluq_dtype dt) {
    if (r < 0 || esize(dt) == 0) return 0;
    return std::max<size_t>(ALIGN, trsm_w_bytes(r, esize(dt)));
}

pluq_status pluq_trsm(int32_t side, int64_t r, int64_t other, const void *dT, int64_t ldt, void *dB, int64_t ldb,
                      pluq_dtype dt, uint64_t p, int32_t form, void *dWork, size_t work_bytes, void *stream) {
    if ((side != 0 && side != 1) || r < 0 || other < 0 || r > INT32_MAX || other > INT32_MAX) return PLUQ_ERR_ARG;
    if (esize(dt) == 0) return PLUQ_ERR_ARG;
    if (p < 2 || p >= P_MAX) return PLUQ_ERR_MODULUS;
    pluq_status s = form_check(form, p);
    if (s != PLUQ_OK) return s;
    if (r == 0 || other == 0) return PLUQ_OK;
    if (!dT || !dB || ldt < r) return PLUQ_ERR_ARG;
    if (side == 0 && ldb < other) return PLUQ_ERR_ARG;
    if (side == 1 && ldb < r) return PLUQ_ERR_ARG;
    if (!dWork || work_bytes < trsm_w_bytes(r, esize(dt))) return PLUQ_ERR_WORKSPACE;
    if ((uintptr_t)dWork % ALIGN) return PLUQ_ERR_ARG;
    try {
        Ctx c;
        c.dt = (int)dt;
        c.esz = esize(dt);
        c.p = p;
        c.form = form;
        c.kchunk = (int)fp64_kchunk(p);
        c.kchunk32 = (int)fp32_kchunk(p);
        c.st = (hipStream_t)stream;
        c.trsm_w = (char *)dWork;
        if (side == 0)
            c.trsm_llu_p((const char *)dT, ldt, r, (char *)dB, ldb, other);
        else
            c.trsm_run_p((char *)dB, ldb, other, (const char *)dT, ldt, r);
    } catch (const DeviceError &) {
        return PLUQ_ERR_DEVICE;
    }
    return PLUQ_OK;
}

void pluq_profile_enable(int32_t mask) {
    for (int c = 0; c < KCLASSES; ++c) g_prof.k[c] = KStat();
    g_prof.discard();
    g_prof.mask = mask;
}

void pluq_profile_read(pluq_kernel_stat *out) {
    if (!out) return;
    // launches of the asynchronous entry points (MM, TRSM) still pending:
    // wait for their events, which were recorded in issue order
    if (!g_prof.pending.empty()) {
        const Profiler::Pending &last = g_prof.pending.back();
        if (hipEventSynchronize(g_prof.pool[last.e0 + 1]) == hipSuccess) g_prof.resolve();
        else g_prof.discard();
    }
    for (int c = 0; c < KCLASSES; ++c) {
        out[c].launches = g_prof.k[c].launches;
        out[c].ms = g_prof.k[c].ms;
        out[c].flops = g_prof.k[c].flops;
        out[c].bytes = g_prof.k[c].bytes;
    }
}

void pluq_last_stats(int64_t *nodes, int64_t *basecases, int64_t *launches, int64_t *syncs) {
    if (nodes) *nodes = g_last_stats.nodes;
    if (basecases) *basecases = g_last_stats.basecases;
    if (launches) *launches = g_last_stats.launches;
    if (syncs) *syncs = g_last_stats.syncs;
}

}  // extern "C"

// ------------------------------------------- outputs derived by permutation --

size_t pluq_post_workspace_size(int64_t m, int64_t n) {
    if (m < 0 || n < 0) return 0;
    const size_t mm = (size_t)std::max<int64_t>(m, 1), nn = (size_t)std::max<int64_t>(n, 1);
    // inverse maps, pairings, a sorted profile and two composed maps (int32)
    return align_up(4 * mm) * 2 + align_up(4 * nn) * 2 + align_up(4 * std::max(mm, nn)) * 3;
}

namespace {

struct PostWs {
    int32_t *pinv, *qinv, *rowpair, *colpair, *sel, *map1, *map2;
};

PostWs post_layout(int64_t m, int64_t n, void *dWork) {
    const size_t mm = (size_t)std::max<int64_t>(m, 1), nn = (size_t)std::max<int64_t>(n, 1);
    const size_t mx = std::max(mm, nn);
    char *w = (char *)dWork;
    PostWs ws;
    ws.pinv = (int32_t *)w;
    w += align_up(4 * mm);
    ws.rowpair = (int32_t *)w;
    w += align_up(4 * mm);
    ws.qinv = (int32_t *)w;
    w += align_up(4 * nn);
    ws.colpair = (int32_t *)w;
    w += align_up(4 * nn);
    ws.sel = (int32_t *)w;
    w += align_up(4 * mx);
    ws.map1 = (int32_t *)w;
    w += align_up(4 * mx);
    ws.map2 = (int32_t *)w;
    return ws;
}

pluq_status post_check(int64_t m, int64_t n, int64_t r, const int64_t *dP, const int64_t *dQ, void *dWork,
                       size_t work_bytes) {
    if (m < 0 || n < 0 || r < 0 || r > std::min(m, n) || m > INT32_MAX || n > INT32_MAX) return PLUQ_ERR_ARG;
    if ((m > 0 && !dP) || (n > 0 && !dQ)) return PLUQ_ERR_ARG;
    if (!dWork || work_bytes < pluq_post_workspace_size(m, n)) return PLUQ_ERR_WORKSPACE;
    if ((uintptr_t)dWork % ALIGN) return PLUQ_ERR_ARG;
    return PLUQ_OK;
}

// Inverse permutations and the rank profile matrix's row <-> column pairing.
void post_maps(int64_t m, int64_t n, int64_t r, const int64_t *dP, const int64_t *dQ, const PostWs &ws,
               hipStream_t st) {
    auto ck = [](hipError_t e) { if (e != hipSuccess) throw DeviceError{e}; };
    ck(launch_fill_i32(ws.pinv, m, 0, st));
    ck(launch_fill_i32(ws.qinv, n, 0, st));
    ck(launch_fill_i32(ws.rowpair, m, -1, st));
    ck(launch_fill_i32(ws.colpair, n, -1, st));
    ck(launch_inverse_map(dP, m, ws.pinv, st));
    ck(launch_inverse_map(dQ, n, ws.qinv, st));
    ck(launch_pair(dP, dQ, m, n, r, ws.rowpair, ws.colpair, st));
}

}  // namespace

extern "C" {

pluq_status pluq_leu(int64_t m, int64_t n, int64_t r, const void *dX, int64_t ldx, pluq_dtype dt, const int64_t *dP,
                     const int64_t *dQ, void *dLbar, int64_t ldl, void *dUbar, int64_t ldu, int64_t *dErow,
                     void *dWork, size_t work_bytes, void *stream) {
    pluq_status s = post_check(m, n, r, dP, dQ, dWork, work_bytes);
    if (s != PLUQ_OK) return s;
    if (esize(dt) == 0) return PLUQ_ERR_ARG;
    if ((m > 0 && n > 0 && (!dX || ldx < n)) || (m > 0 && (!dLbar || ldl < m)) || (n > 0 && (!dUbar || ldu < n)))
        return PLUQ_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    const PostWs ws = post_layout(m, n, dWork);
    try {
        post_maps(m, n, r, dP, dQ, ws, st);
        auto ck = [](hipError_t e) { if (e != hipSuccess) throw DeviceError{e}; };
        ck(launch_post_gather((int)dt, false, dX, ldx, r, dLbar, ldl, m, m, ws.pinv, ws.pinv, st));
        ck(launch_post_gather((int)dt, true, dX, ldx, r, dUbar, ldu, n, n, ws.qinv, ws.qinv, st));
        if (dErow) ck(launch_widen(ws.rowpair, m, dErow, st));
    } catch (const DeviceError &e) {
        set_err("pluq_leu: HIP call", e.e);
        return PLUQ_ERR_DEVICE;
    }
    return PLUQ_OK;
}

pluq_status pluq_echelon(int32_t kind, int64_t m, int64_t n, int64_t r, const void *dX, int64_t ldx, pluq_dtype dt,
                         const int64_t *dP, const int64_t *dQ, void *dF, int64_t ldf, void *dG, int64_t ldg,
                         int64_t *dProf, void *dWork, size_t work_bytes, void *stream) {
    pluq_status s = post_check(m, n, r, dP, dQ, dWork, work_bytes);
    if (s != PLUQ_OK) return s;
    if ((kind != PLUQ_ECHELON_COLUMN && kind != PLUQ_ECHELON_ROW) || esize(dt) == 0) return PLUQ_ERR_ARG;
    if (m > 0 && n > 0 && (!dX || ldx < n)) return PLUQ_ERR_ARG;
    if (r > 0) {
        // F: m x r (column echelon) or r x n (row echelon); G the other factor
        const int64_t fcols = kind == PLUQ_ECHELON_COLUMN ? r : n, gcols = kind == PLUQ_ECHELON_COLUMN ? n : r;
        if (!dF || !dG || ldf < fcols || ldg < gcols) return PLUQ_ERR_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    const PostWs ws = post_layout(m, n, dWork);
    try {
        post_maps(m, n, r, dP, dQ, ws, st);
        if (r == 0) return PLUQ_OK;
        auto ck = [](hipError_t e) { if (e != hipSuccess) throw DeviceError{e}; };
        ck(launch_fill_i32(ws.sel, std::max(m, n), 0, st));
        if (kind == PLUQ_ECHELON_COLUMN) {
            // pivot rows ascending (the row rank profile); C = Lbar[:, rows],
            // R = Ubar[paired columns, :]
            ck(launch_compact(ws.rowpair, m, n, r, ws.sel, dProf, nullptr, st));
            ck(launch_compose(ws.pinv, ws.sel, nullptr, r, ws.map1, st));
            ck(launch_compose(ws.qinv, ws.sel, ws.rowpair, r, ws.map2, st));
            ck(launch_post_gather((int)dt, false, dX, ldx, r, dF, ldf, m, r, ws.pinv, ws.map1, st));
            ck(launch_post_gather((int)dt, true, dX, ldx, r, dG, ldg, r, n, ws.map2, ws.qinv, st));
        } else {
            // pivot columns ascending (the column rank profile);
            // E = Ubar[columns, :], L_E = Lbar[:, paired rows]
            ck(launch_compact(ws.colpair, n, m, r, ws.sel, dProf, nullptr, st));
            ck(launch_compose(ws.qinv, ws.sel, nullptr, r, ws.map1, st));
            ck(launch_compose(ws.pinv, ws.sel, ws.colpair, r, ws.map2, st));
            ck(launch_post_gather((int)dt, true, dX, ldx, r, dF, ldf, r, n, ws.map1, ws.qinv, st));
            ck(launch_post_gather((int)dt, false, dX, ldx, r, dG, ldg, m, r, ws.pinv, ws.map2, st));
        }
    } catch (const DeviceError &e) {
        set_err("pluq_echelon: HIP call", e.e);
        return PLUQ_ERR_DEVICE;
    }
    return PLUQ_OK;
}

pluq_status pluq_leading_ranks(int64_t m, int64_t n, int64_t r, const int64_t *dP, const int64_t *dQ, int64_t nq,
                               const int64_t *dk, const int64_t *dt_, int64_t *dranks, void *dWork,
                               size_t work_bytes, void *stream) {
    pluq_status s = post_check(m, n, r, dP, dQ, dWork, work_bytes);
    if (s != PLUQ_OK) return s;
    if (nq < 0 || (nq > 0 && (!dk || !dt_ || !dranks))) return PLUQ_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    const PostWs ws = post_layout(m, n, dWork);
    try {
        post_maps(m, n, r, dP, dQ, ws, st);
        const hipError_t e = launch_leading_ranks(ws.rowpair, m, dk, dt_, nq, dranks, st);
        if (e != hipSuccess) throw DeviceError{e};
    } catch (const DeviceError &e) {
        set_err("pluq_leading_ranks: HIP call", e.e);
        return PLUQ_ERR_DEVICE;
    }
    return PLUQ_OK;
}

pluq_status pluq_leading_rank_profiles_device(int64_t m, int64_t n, int64_t r, const int64_t *dP, const int64_t *dQ,
                                              int64_t k, int64_t t, int64_t *drows, int64_t *dcols,
                                              int64_t *dcount, void *dWork, size_t work_bytes, void *stream) {
    pluq_status s = post_check(m, n, r, dP, dQ, dWork, work_bytes);
    if (s != PLUQ_OK) return s;
    if (k < 0 || t < 0 || !dcount || (r > 0 && (!drows || !dcols))) return PLUQ_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    const PostWs ws = post_layout(m, n, dWork);
    try {
        post_maps(m, n, r, dP, dQ, ws, st);
        auto ck = [](hipError_t e) { if (e != hipSuccess) throw DeviceError{e}; };
        // rows i < k whose pivot column is < t, and columns j < t whose pivot
        // row is < k, both ascending
        ck(launch_compact(ws.rowpair, std::min(k, m), t, r, nullptr, drows, dcount, st));
        ck(launch_compact(ws.colpair, std::min(t, n), k, r, nullptr, dcols, dcount + 1, st));
    } catch (const DeviceError &e) {
        set_err("pluq_leading_rank_profiles_device: HIP call", e.e);
        return PLUQ_ERR_DEVICE;
    }
    return PLUQ_OK;
}

pluq_status pluq_tune_set(int32_t form, int32_t pclass, int32_t dtype, int32_t bucket, const pluq_tune *t) {
    if (!t || form < -1 || form > TUNE_FORM_BATCHED || pclass < -1 || pclass > 2 || dtype < -1 || dtype > 2 ||
        bucket < -1 ||
        bucket > 31)
        return PLUQ_ERR_ARG;
    if (t->cutoff < 0 || t->cutoff > 128 || (t->cutoff > 0 && t->cutoff < 16) || t->mm_tiles128 < 0 ||
        t->mm_tiles64 < 0 || t->fork_min_dim < 0 || t->i8_min_work < 0 ||
        (t->batch_panel != 0 && t->batch_panel != 8 && t->batch_panel != 16) || t->batch_groups < 0 ||
        t->batch_groups > 8 || t->strassen_min < 0 || (t->strassen_min > 0 && t->strassen_min < 128))
        return PLUQ_ERR_ARG;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    for (TuneEntry &e : g_tune)
        if (e.form == form && e.pclass == pclass && e.dtype == dtype && e.bucket == bucket) {
            e.t = *t;
            return PLUQ_OK;
        }
    g_tune.push_back(TuneEntry{form, pclass, dtype, bucket, *t});
    return PLUQ_OK;
}

void pluq_tune_clear(void) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune.clear();
}

pluq_status pluq_tune_get(int32_t form, uint64_t p, int32_t dtype, int64_t m, int64_t n, pluq_tune *out,
                          int32_t *from_table) {
    if (!out || m < 0 || n < 0) return PLUQ_ERR_ARG;
    bool hit = false;
    *out = tune_for(form, p, dtype, m, n, &hit);
    if (from_table) *from_table = hit ? 1 : 0;
    return PLUQ_OK;
}

}  // extern "C"
