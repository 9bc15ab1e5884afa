// Host driver and C ABI of libwenott (see include/wenott.h).
//
// One SSP-RK3 step of WENO-TT (Sec. 4): for each stage, the Lax-Friedrichs alpha of the
// stage input; for each direction, one rank-adaptive cross of the fused LF + WENO5-JS flux
// (the LF-cross and WENO-cross of Algorithms lf-cross / weno-cross fused into a single
// function of the state, with one slice per conserved variable on the last core as in
// Sec. 4.2); the shift difference (T - 1)/h on that direction's core; the stage's linear
// combination as a TT sum; one TT-rounding (Sec. 3.2) at eps_TT, which follows eq.
// eps-tt-formula in dynamic mode.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

#include "common.h"

using namespace wtt;

namespace {

// splitmix64: the library's own counter-based generator (pivot enrichment and probe points).
struct Rng {
    uint64_t s;
    explicit Rng(uint64_t seed) : s(seed) {}
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        return z ^ (z >> 31);
    }
    int below(int n) { return (int)(next() % (uint64_t)n); }
};

// Stream-ordered device allocation with a per-stream cache of freed blocks. The work of one
// stream runs in order, so a block freed on a stream can be handed out again on that stream at
// once: whatever is enqueued later runs after everything that used the block before. Sizes are
// rounded up to eight classes per power of two; up to kCacheBytes per stream stay cached, beyond
// that a freed block goes back to the runtime. The TT cores of every cross and rounding come and
// go through here, so a step makes no runtime allocation once the ranks have settled.
constexpr size_t kCacheBytes = size_t(2) << 30;

struct AllocCache {
    std::mutex mu;
    std::unordered_map<void *, std::pair<hipStream_t, size_t>> live;  // pointer -> (stream, bytes)
    std::map<hipStream_t, std::multimap<size_t, void *>> idle;
    std::map<hipStream_t, size_t> idle_bytes;
};

AllocCache &alloc_cache() {
    static AllocCache *ac = new AllocCache;  // never destroyed: blocks outlive static destructors
    return *ac;
}

size_t size_class(size_t bytes) {
    bytes = std::max<size_t>(bytes, 256);
    const int p = 63 - __builtin_clzll((unsigned long long)bytes);
    const size_t step = size_t(1) << (p - 3);
    return (bytes + step - 1) / step * step;
}

// Returns the idle blocks of stream s to the runtime.
void release_stream_cache(hipStream_t s) {
    AllocCache &ac = alloc_cache();
    std::multimap<size_t, void *> blocks;
    {
        std::lock_guard<std::mutex> g(ac.mu);
        auto it = ac.idle.find(s);
        if (it == ac.idle.end()) return;
        blocks.swap(it->second);
        ac.idle.erase(it);
        ac.idle_bytes.erase(s);
    }
    for (auto &b : blocks) (void)hipFreeAsync(b.second, s);
}

// Returns the idle blocks of every stream to the runtime (blocks still in use stay tracked).
void release_all_caches() {
    std::vector<hipStream_t> streams;
    {
        AllocCache &ac = alloc_cache();
        std::lock_guard<std::mutex> g(ac.mu);
        for (auto &kv : ac.idle) streams.push_back(kv.first);
    }
    for (hipStream_t s : streams) release_stream_cache(s);
}

// Drops p from the bookkeeping (for teardown paths that free it themselves).
void forget_block(void *p) {
    AllocCache &ac = alloc_cache();
    std::lock_guard<std::mutex> g(ac.mu);
    ac.live.erase(p);
}

template <typename T>
T *dalloc(hipStream_t s, size_t count) {
    const size_t bytes = size_class(std::max<size_t>(count, 1) * sizeof(T));
    AllocCache &ac = alloc_cache();
    {
        std::lock_guard<std::mutex> g(ac.mu);
        auto it = ac.idle.find(s);
        if (it != ac.idle.end()) {
            auto f = it->second.find(bytes);
            if (f != it->second.end()) {
                void *p = f->second;
                it->second.erase(f);
                ac.idle_bytes[s] -= bytes;
                ac.live[p] = {s, bytes};
                return (T *)p;
            }
        }
    }
    void *p = nullptr;
    hipError_t e = hipMallocAsync(&p, bytes, s);
    if (e == hipErrorOutOfMemory) {  // give the idle blocks back and try once more
        (void)hipGetLastError();
        release_stream_cache(s);
        e = hipMallocAsync(&p, bytes, s);
    }
    if (e == hipErrorOutOfMemory) throw StatusError(WENOTT_ENOMEM, "device allocation failed");
    WTT_HIP(e);
    std::lock_guard<std::mutex> g(ac.mu);
    ac.live[p] = {s, bytes};
    return (T *)p;
}

inline void dfree(hipStream_t s, void *p) {
    if (!p) return;
    AllocCache &ac = alloc_cache();
    {
        std::lock_guard<std::mutex> g(ac.mu);
        auto it = ac.live.find(p);
        if (it != ac.live.end()) {
            const hipStream_t owner = it->second.first;
            const size_t bytes = it->second.second;
            ac.live.erase(it);
            if (owner == s && ac.idle_bytes[s] + bytes <= kCacheBytes) {
                ac.idle[s].emplace(bytes, p);
                ac.idle_bytes[s] += bytes;
                return;
            }
        }
    }
    WTT_HIP(hipFreeAsync(p, s));
}

enum Slot {
    S_P, S_Q, S_T, S_W, S_PTS, S_BLOCK, S_L, S_PIV, S_ROWBUF, S_TSQR, S_R, S_SIG, S_V, S_JAC, S_W1, S_W2,
    S_RANKS, S_PART, S_UST, S_LM, S_NORMS, S_TMP, S_DENSE,
    S_PD0, S_PD1, S_QD0, S_QD1, S_TD0, S_TD1, S_WD0, S_WD1, S_PN, S_QN, S_TN, S_WN, S_SPLIT,
    S_F_G, S_F_P, S_F_Q, S_F_T, S_F_W0, S_F_WD0, S_F_WD1, S_MLPY, S_MLPW, S_AL_I, S_AL_D, S_NSLOTS
};

struct Scratch {
    hipStream_t s = nullptr;
    void *p[S_NSLOTS] = {};
    size_t cap[S_NSLOTS] = {};
    template <typename T>
    T *get(int slot, size_t count) {
        size_t bytes = std::max<size_t>(count * sizeof(T), 256);
        if (cap[slot] < bytes) {
            dfree(s, p[slot]);
            p[slot] = nullptr;
            size_t nb = std::max(bytes, cap[slot] + cap[slot] / 2);
            p[slot] = dalloc<char>(s, nb);
            cap[slot] = nb;
        }
        return (T *)p[slot];
    }
    void release() {
        for (int i = 0; i < S_NSLOTS; ++i) {
            if (p[i]) {
                forget_block(p[i]);
                (void)hipFreeAsync(p[i], s);
            }
            p[i] = nullptr;
            cap[i] = 0;
        }
    }
};

// Upload ring: pinned host staging + device mirror, reused in stream order.
struct Ring {
    hipStream_t s = nullptr;
    char *h = nullptr, *dv = nullptr;
    size_t cap = 0, off = 0;
    void init(hipStream_t st, size_t bytes) {
        s = st;
        cap = bytes;
        WTT_HIP(hipHostMalloc((void **)&h, cap, hipHostMallocDefault));
        WTT_HIP(hipMalloc((void **)&dv, cap));
    }
    void destroy() {
        if (h) (void)hipHostFree(h);
        if (dv) (void)hipFree(dv);
        h = dv = nullptr;
    }
    template <typename T>
    T *put(const T *src, size_t count) {
        size_t bytes = std::max<size_t>(count * sizeof(T), 8);
        bytes = (bytes + 255) / 256 * 256;
        WTT_REQUIRE(bytes <= cap, WENOTT_EINVAL, "upload larger than the staging ring");
        if (off + bytes > cap) {
            WTT_HIP(hipStreamSynchronize(s));
            off = 0;
        }
        std::memcpy(h + off, src, count * sizeof(T));
        WTT_HIP(hipMemcpyAsync(dv + off, h + off, count * sizeof(T), hipMemcpyHostToDevice, s));
        T *r = (T *)(dv + off);
        off += bytes;
        return r;
    }
};

// A list of ncomp TTs with common (padded) bond ranks; core k is [c][R_k][N_k][R_{k+1}].
struct TT {
    int d = 0, nc = 0;
    int N[kMaxDim] = {};
    int R[kMaxDim + 1] = {};
    double *core[kMaxDim] = {};
    long long cstride(int k) const { return (long long)R[k] * N[k] * R[k + 1]; }
    int maxrank() const {
        int r = 1;
        for (int k = 1; k < d; ++k) r = std::max(r, R[k]);
        return r;
    }
    void alloc(hipStream_t s) {
        for (int k = 0; k < d; ++k) core[k] = dalloc<double>(s, (size_t)cstride(k) * nc);
    }
    void release(hipStream_t s) {
        for (int k = 0; k < d; ++k) {
            dfree(s, core[k]);
            core[k] = nullptr;
        }
    }
};

// Output of one cross: shared cores [R_k][M_k][R_{k+1}] for k < d-1 and the last core
// [R_{d-1}][M_{d-1}][ncomp] carrying one slice per conserved variable.
struct FluxTT {
    int d = 0, nc = 0;
    int M[kMaxDim] = {};
    int R[kMaxDim + 1] = {};
    double *core[kMaxDim] = {};
    void release(hipStream_t s) {
        for (int k = 0; k < d; ++k) {
            dfree(s, core[k]);
            core[k] = nullptr;
        }
    }
};

// Warm-start slots of the crosses (their last right index sets and pivot ranks): the flux cross
// of each direction (scheme 1), the stage cross (scheme 0), and per direction the LF-cross and the
// WENO-crosses of its 2 ncomp split-flux slices (scheme 2).
constexpr int kSlotStage = kMaxDim;
constexpr int kSlotLf = kMaxDim + 1;
constexpr int kSlotWeno = 2 * kMaxDim + 1;
constexpr int kMaxSlices = 10;
constexpr int kWarmSlots = kSlotWeno + kMaxDim * kMaxSlices;

struct ISet {  // a set of multi-indices of a fixed length
    int len = 0, count = 0;
    std::vector<int> v;
};

}  // namespace

// Device workspace of wenott_max_wavespeed_noalloc: a file-scope array, one copy per GPU, held
// until the process ends. Its device address is taken once per device (at the first wenott_init
// on that device) with hipGetSymbolAddress; host code only ever uses that address.
constexpr size_t kNoAllocBytes = size_t(1) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[kMaxDevices] = {};

// The address of this device's copy of scratch (obtained on the first call per device).
void *noalloc_scratch_of(int dev) {
    WTT_REQUIRE(dev >= 0 && dev < kMaxDevices, WENOTT_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> g(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *p = nullptr;
        WTT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_noalloc_ptr[dev] = p;
    }
    return g_noalloc_ptr[dev];
}

struct wenott_ctx {
    int d = 0, nc = 0;
    int law = 0;                 // wenott_law
    void *noalloc_ws = nullptr;  // this device's copy of scratch
    int N[kMaxDim] = {};
    double lo[kMaxDim] = {}, hi[kMaxDim] = {}, h[kMaxDim] = {};
    double gamma = 1.4;
    int bc[kMaxDim] = {};         // bc_code(low, high) per dimension
    double qin[kMaxDim][2][5] = {};  // conserved inflow state per inflow side
    bool qin_set[kMaxDim][2] = {};
    wenott_opts o{};
    hipStream_t s = nullptr;
    hipEvent_t ev_wait = nullptr;  // host_wait's marker on s
    unsigned long long waits = 0;  // host_wait calls so far
    TT U;
    TT rhs;
    bool have_rhs = false;
    std::vector<int64_t> view_ranks;
    std::vector<const void *> view_ptrs;
    Scratch sc;
    Ring ring;
    int *d_flags = nullptr;  // first word of d_status
    // Status block: [0] flag word, [1..4] alpha slots, [8..) residual partials; copied to the
    // pinned mirror h_status in one transfer per readback.
    double *d_status = nullptr, *h_status = nullptr;
    int *h_pinned_int = nullptr;
    double *h_pinned_dbl = nullptr;
    std::vector<ISet> warm[kWarmSlots];  // right index sets of the last cross of each slot
    bool warm_valid[kWarmSlots] = {};
    uint64_t counter = 0;        // random streams of the crosses
    uint64_t alpha_counter = 0;  // random start cells of the alpha searches
    double c_eps = 0.0, max_norm = 0.0;
    bool profiling = false;
    std::vector<hipEvent_t> ev;
    std::vector<int> ev_class;
    int ev_used = 0;
    wenott_info info{};
    std::string last_error;
    // learned proposal and pivot logs of stage crosses (one history per TT bond)
    struct BondHist {
        bool valid = false;
        int rank = 0;
        float hist[WENOTT_MLP_BINS] = {};
        float sig[16] = {};
        std::vector<int> useful;  // right multi-indices whose columns were pivots (len d-1-k each)
    };
    BondHist bond[kMaxDim];
    int piv_hist[kWarmSlots * 2 * kMaxDim];  // last pivot rank per (cross slot, sweep direction, core)
    int *d_best = nullptr;              // best cell of the last alpha search (device int[kMaxDim])
    const double *alpha_dev = nullptr;  // stage alpha on the device (read by the fiber kernels) when set
    double alpha_cache = 0.0;           // alpha of the current state (alpha_mode rule), if alpha_cache_valid
    bool alpha_cache_valid = false;
    float last_sig[16] = {};
    int prev_sweeps = 1;
    double prev_resid = 0.0;
    const float *proposal = nullptr;
    bool logging = false;
    std::vector<float> log_x, log_hist;
    std::vector<int> log_cls;
};

// Waits on the host for the work queued on c->s by recording an event and polling it. A
// blocking stream synchronisation may put the host thread to sleep until an interrupt once
// its short spin runs out; the wake-up then delays the next launch at each of the
// data-dependent readbacks of a step (pivot ranks, residuals, truncation ranks).
void host_wait(wenott_ctx *c) {
    ++c->waits;
    WTT_HIP(hipEventRecord(c->ev_wait, c->s));
    hipError_t e;
    while ((e = hipEventQuery(c->ev_wait)) == hipErrorNotReady) {
    }
    WTT_HIP(e);
}

namespace {

inline double seconds_now() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------------------ helpers
// Raise the status recorded in a flag word already copied to the host.
void raise_flags(wenott_ctx *c, int f) {
    if (f) {
        WTT_HIP(hipMemsetAsync(c->d_flags, 0, sizeof(int), c->s));
        if (f & kFlagNaN) throw StatusError(WENOTT_ENAN, "NaN or Inf in a flux evaluation");
        throw StatusError(WENOTT_ENONPHYS, "rho <= 0 or p <= 0 at an evaluated point");
    }
}

constexpr int kStatusAlpha = 1, kStatusAcc = 8, kMaxResidualBlocks = 256;
constexpr int kStatusDoubles = kStatusAcc + 2 * kMaxResidualBlocks;

int status_flags(const wenott_ctx *c) { return *(const int *)c->h_status; }

// Copy the first `doubles` entries of the status block to its pinned mirror.
void status_readback(wenott_ctx *c, int doubles) {
    WTT_HIP(hipMemcpyAsync(c->h_status, c->d_status, sizeof(double) * doubles, hipMemcpyDeviceToHost, c->s));
}

// Kernel classes timed with HIP events when profiling is on (wenott_info.class_*).
enum KClass { KC_FIBER = 0, KC_PIVOT = 1, KC_TSQR = 2, KC_SVD = 3 };

void ev_record(wenott_ctx *c, int cls = KC_FIBER) {
    if (!c->profiling) return;
    if (c->ev_used == (int)c->ev.size()) {
        hipEvent_t e;
        WTT_HIP(hipEventCreate(&e));
        c->ev.push_back(e);
        c->ev_class.push_back(0);
    }
    c->ev_class[c->ev_used] = cls;
    WTT_HIP(hipEventRecord(c->ev[c->ev_used++], c->s));
}

void add_work(wenott_ctx *c, int cls, double flops, double bytes) {
    c->info.class_flops[cls] += flops;
    c->info.class_bytes[cls] += bytes;
    c->info.class_launches[cls] += 1;
}

TT copy_tt(wenott_ctx *c, const TT &a) {
    TT b = a;
    b.alloc(c->s);
    for (int k = 0; k < a.d; ++k)
        WTT_HIP(hipMemcpyAsync(b.core[k], a.core[k], sizeof(double) * a.cstride(k) * a.nc, hipMemcpyDeviceToDevice,
                               c->s));
    return b;
}

// ------------------------------------------------------------------- exact alpha
// Left part of every cell's chain product: (N_0 ... N_{d-2}) x R_{d-1} per component.
const double *left_part(wenott_ctx *c, const TT &U, long long *stride) {
    if (U.d == 2) {
        *stride = U.cstride(0);
        return U.core[0];
    }
    long long rows = (long long)U.N[0] * U.N[1];
    double *Lm = c->sc.get<double>(S_LM, (size_t)rows * U.R[2] * U.nc);
    GemmBatch bt;
    bt.nb1 = U.nc;
    bt.sA1 = U.cstride(0);
    bt.sB1 = U.cstride(1);
    bt.sC1 = rows * U.R[2];
    gemm_f64(c->s, false, false, U.N[0], U.N[1] * U.R[2], U.R[1], 1.0, U.core[0], U.R[1], U.core[1],
             U.N[1] * U.R[2], 0.0, Lm, U.N[1] * U.R[2], bt);
    *stride = rows * U.R[2];
    return Lm;
}

// Pinned host slots read after a later synchronisation: the component norms of the last rounding.
constexpr int kPinNorms = 4080;

// Enqueue the alpha of U (alpha_mode 0: exact, every cell; 1: the line-search estimate) into
// alpha slot `slot` of the status block and, with readback,
// a copy of the block head (flag word and alpha slots) to its pinned mirror. Returns the device
// address. Without readback the head reaches the host with the next status readback (every
// stage cross makes one: its sampled residual).
double *alpha_launch(wenott_ctx *c, const TT &U, int slot, bool readback = true) {
    double *dst = c->d_status + kStatusAlpha + slot;
    if (c->law == WENOTT_LAW_LINADV) {  // f'(u) = 1 along every axis
        fill(c->s, dst, 1, 1.0);
        if (readback) status_readback(c, kStatusAlpha + 4);
        return dst;
    }
    if (c->o.alpha_mode == 1) {  // line search (the tt_max_abs estimate of eq. cfl-other)
        int ranks[kMaxDim + 1];
        const double *cores[kMaxDim];
        for (int k = 0; k <= U.d; ++k) ranks[k] = U.R[k];
        for (int k = 0; k < U.d; ++k) cores[k] = U.core[k];
        // its own counter: the cross's random sets follow the same sequence whether or not the
        // caller asked for alpha in between
        const unsigned long long seed = c->o.seed * 0x9E3779B97F4A7C15ULL + 0xA5A5ULL * (++c->alpha_counter);
        alpha_search(c->s, U.d, c->law, U.N, cores, ranks, c->gamma, seed, c->d_best,
                     c->sc.get<int>(S_AL_I, alpha_search_ints(U.d, U.N[1])),
                     c->sc.get<double>(S_AL_D, alpha_search_doubles(U.d, U.N[1])),
                     dst, c->d_flags);
        if (readback) status_readback(c, kStatusAlpha + 4);
        return dst;
    }
    long long lms = 0;
    const double *Lm = left_part(c, U, &lms);
    long long nrows = 1;
    for (int k = 0; k < U.d - 1; ++k) nrows *= U.N[k];
    int nlast = U.N[U.d - 1];
    const int nblocks = dense_eval_blocks(1, nrows, U.R[U.d - 1], nlast);
    double *part = c->sc.get<double>(S_PART, nblocks);
    dense_eval(c->s, 1, U.d, c->law, nrows, U.R[U.d - 1], nlast, Lm, lms, U.core[U.d - 1], U.cstride(U.d - 1),
               c->gamma, nullptr, part, nblocks, c->d_flags);
    reduce_max_dev(c->s, part, nblocks, dst);
    if (readback) status_readback(c, kStatusAlpha + 4);
    return dst;
}

double status_alpha(const wenott_ctx *c, int slot) { return c->h_status[kStatusAlpha + slot]; }

double alpha_now(wenott_ctx *c, const TT &U) {
    alpha_launch(c, U, 3);
    host_wait(c);
    raise_flags(c, status_flags(c));
    return status_alpha(c, 3);
}

void to_dense_dev(wenott_ctx *c, const TT &U, double *out) {
    long long lms = 0;
    const double *Lm = left_part(c, U, &lms);
    long long nrows = 1;
    for (int k = 0; k < U.d - 1; ++k) nrows *= U.N[k];
    int nlast = U.N[U.d - 1];
    const int nblocks = dense_eval_blocks(0, nrows, U.R[U.d - 1], nlast);
    dense_eval(c->s, 0, U.d, c->law, nrows, U.R[U.d - 1], nlast, Lm, lms, U.core[U.d - 1], U.cstride(U.d - 1),
               c->gamma, out, nullptr, nblocks, c->d_flags);
}

// ---------------------------------------------------------------- boundary sides
void require_inflow_states(const wenott_ctx *c) {
    for (int k = 0; k < c->d; ++k)
        for (int side = 0; side < 2; ++side)
            WTT_REQUIRE(bc_side(c->bc[k], side) != WENOTT_BC_INFLOW || c->qin_set[k][side], WENOTT_EINVAL,
                        "an inflow side has no state (wenott_set_inflow)");
}

bool has_inflow(const wenott_ctx *c, int m) {
    return bc_side(c->bc[m], 0) == WENOTT_BC_INFLOW || bc_side(c->bc[m], 1) == WENOTT_BC_INFLOW;
}

// (shift, pivot, side) triples of the index tuples of `set` (mode m at tuple position pos) whose
// shifted cell v - 3 + s (s < S) along m lies on an inflow side of m.
std::vector<int> inflow_pairs(const wenott_ctx *c, const std::vector<int> &v, int len, int count, int pos, int m,
                              int S) {
    std::vector<int> out;
    const int n = c->N[m];
    for (int t = 0; t < count; ++t)
        for (int sh = 0; sh < S; ++sh) {
            const int raw = v[(size_t)t * len + pos] - 3 + sh;
            if (ghost_kind(raw, n, c->bc[m]) != kGhostInflow) continue;
            out.push_back(sh);
            out.push_back(t);
            out.push_back(raw >= n ? 1 : 0);
        }
    return out;
}

// The inflow state into a gathered block W ([c][S][p][Nk][q]) shifted along mode m != k, after
// its interface rows of the inflow cells were zeroed.
template <typename T>
void fill_inflow_block(wenott_ctx *c, const FiberGeom &g, int m, int k, const ISet &L, const ISet &Rs, int S, int Nk,
                       T *W) {
    if (m < 0 || m == k || !has_inflow(c, m)) return;
    const bool right = m > k;
    const ISet &set = right ? Rs : L;
    const std::vector<int> pr = inflow_pairs(c, set.v, set.len, set.count, right ? m - k - 1 : m, m, S);
    if (pr.empty()) return;
    const int p = L.count, q = Rs.count;
    const long long blk = (long long)p * Nk * q;
    inflow_fill<T>(c->s, g, m, (int)pr.size() / 3, c->ring.put(pr.data(), pr.size()), right, p, Nk, q, S * blk, blk,
                   W);
}

// ---------------------------------------------------------------- block evaluation
// Flux block Fhat_dir(I_<k[a], i, J_>k[b], c) written with strides (L->R or R->L unfolding).
// law: the conservation law whose split fluxes are reconstructed (the context's; the WENO-crosses
// of scheme 2 pass linear advection with alpha = +1 or -1, whose split fluxes are the input slice
// and zero, so that the kernel forms the one-sided WENO5 reconstruction of the slice).
void eval_block(wenott_ctx *c, const TT &U, int dir, int k, const ISet &L, const ISet &Rs, double alpha, bool lr,
                double *out, int law) {
    const int d = U.d, nc = U.nc;
    FiberGeom g{};
    g.d = d; g.ncomp = nc; g.dir = dir; g.k = k;
    for (int j = 0; j < d; ++j) { g.n[j] = U.N[j]; g.bc[j] = c->bc[j]; }
    g.law = law; std::memcpy(g.qin, c->qin, sizeof g.qin); g.gamma = c->gamma; g.alpha = alpha; g.eps_w = c->h[dir] * c->h[dir];
    const int p = L.count, q = Rs.count;
    const int SL = dir < k ? 6 : 1, SR = dir > k ? 6 : 1, S = std::max(SL, SR);
    const int Rk = U.R[k], Rk1 = U.R[k + 1], Nk = U.N[k];
    int ranks[kMaxDim + 1];
    for (int j = 0; j <= d; ++j) ranks[j] = U.R[j];
    const double *cores[kMaxDim];
    for (int j = 0; j < d; ++j) cores[j] = U.core[j];

    double *P = c->sc.get<double>(S_P, (size_t)nc * SL * p * Rk);
    if (k == 0) fill(c->s, P, (long long)nc * SL * p * Rk, 1.0);
    else iface(c->s, g, 0, cores, ranks, p, c->ring.put(L.v.data(), L.v.size()), SL, SL == 6 ? dir : -1, P);
    double *Q = c->sc.get<double>(S_Q, (size_t)nc * SR * Rk1 * q);
    if (k == d - 1) fill(c->s, Q, (long long)nc * SR * Rk1 * q, 1.0);
    else iface(c->s, g, 1, cores, ranks, q, c->ring.put(Rs.v.data(), Rs.v.size()), SR, SR == 6 ? dir : -1, Q);

    const long long tsz = (long long)p * Nk * Rk1;
    double *T = c->sc.get<double>(S_T, (size_t)nc * SL * tsz);
    GemmBatch b1;
    b1.nb1 = nc; b1.nb2 = SL;
    b1.sA1 = (long long)SL * p * Rk; b1.sA2 = (long long)p * Rk;
    b1.sB1 = U.cstride(k); b1.sB2 = 0;
    b1.sC1 = SL * tsz; b1.sC2 = tsz;
    gemm_f64(c->s, false, false, p, Nk * Rk1, Rk, 1.0, P, Rk, U.core[k], Nk * Rk1, 0.0, T, Nk * Rk1, b1);
    const long long wsz = (long long)p * Nk * q;
    double *W = c->sc.get<double>(S_W, (size_t)nc * S * wsz);
    GemmBatch b2;
    b2.nb1 = nc; b2.nb2 = S;
    b2.sA1 = SL * tsz; b2.sA2 = SL == 6 ? tsz : 0;
    b2.sB1 = (long long)SR * Rk1 * q; b2.sB2 = SR == 6 ? (long long)Rk1 * q : 0;
    b2.sC1 = S * wsz; b2.sC2 = wsz;
    gemm_f64(c->s, false, false, p * Nk, q, Rk1, 1.0, T, Rk1, Q, q, 0.0, W, q, b2);
    if (dir != k) fill_inflow_block<double>(c, g, dir, k, L, Rs, 6, Nk, W);

    const int M = k == dir ? Nk + 1 : Nk;
    long long sa, si, sb, sc;
    if (lr) { sa = (long long)M * q * nc; si = (long long)q * nc; sb = nc; sc = 1; }
    else { sa = nc; si = (long long)q * p * nc; sb = (long long)p * nc; sc = 1; }
    ev_record(c, KC_FIBER);
    weno_block<double>(c->s, g, p, q, W, out, sa, si, sb, sc, c->d_flags);
    ev_record(c, KC_FIBER);
    c->info.fiber_points += (long long)p * M * q;
    c->info.fiber_launches += 1;
    {  // one face flux per point: 6 cells x (primitives, flux, split) + 2 nc WENO5 + nc adds
        const double pts = (double)p * M * q;
        const double per = d == 2 ? 814.0 : 1013.0;
        const double reads = (k == dir ? 1.0 : 6.0) * nc * 8.0;  // distinct gathered values per point
        add_work(c, KC_FIBER, pts * per, pts * (reads + nc * 8.0));
    }
}

ISet random_set(Rng &rng, int count, int first_mode, int len, const int *M) {
    ISet s;
    s.len = len;
    s.count = count;
    s.v.resize((size_t)count * len);
    for (int a = 0; a < count; ++a)
        for (int j = 0; j < len; ++j) s.v[(size_t)a * len + j] = rng.below(M[first_mode + j]);
    return s;
}

ISet with_kick(const ISet &base, Rng &rng, int kick, int first_mode, const int *M) {
    ISet s = base;
    if (base.len == 0 || kick <= 0) return s;
    ISet extra = random_set(rng, kick, first_mode, base.len, M);
    s.v.insert(s.v.end(), extra.v.begin(), extra.v.end());
    s.count += kick;
    return s;
}

struct PivotResult {
    int rank;
    bool capped = false;  // stopped at the rank limit with the residual above the tolerance
    std::vector<int> rows, cols;
};

inline int hist_index(int slot, int dir, int k) { return (slot * 2 + dir) * kMaxDim + k; }

// First number of pivot steps to launch for a block: the rank this bond had the last time,
// with a margin, else the number of index tuples on the block's column side.
int pivot_guess(const wenott_ctx *c, int hist_slot, int n, int rmax) {
    const int h = hist_slot >= 0 ? c->piv_hist[hist_slot] : -1;
    const int g = h > 0 ? h + std::max(2, h / 4) : n / std::max(c->U.nc, 1);
    return std::max(1, std::min(g, rmax));
}

// Pivot indices (2 rmax + 2 ints) and the {rank, residual, threshold} triple share one device
// buffer, so that one transfer brings both back: byte offset of the triple.
size_t pivot_info_offset(int rmax) { return ((2 * (size_t)rmax + 2) * sizeof(int) + 7) / 8 * 8; }

int *pivot_buffer(wenott_ctx *c, int rmax, double **info) {
    const size_t off = pivot_info_offset(rmax);
    int *piv = c->sc.get<int>(S_PIV, off / sizeof(int) + 6);
    *info = (double *)((char *)piv + off);
    return piv;
}

double pinned_pivot_info(const wenott_ctx *c, int rmax, int which) {
    return ((const double *)((const char *)c->h_pinned_int + pivot_info_offset(rmax)))[which];
}

// Full-pivot rank-revealing LU of the block B (m x n). When the single-launch persistent form
// gives up waiting for workgroups that are not all resident (info -2), the block is partly
// eliminated: reeval() writes it again and the search is redone one launch per step.
PivotResult pivots(wenott_ctx *c, double *B, int m, int n, double rel_tol2, double **Lout, int hist_slot,
                   const std::function<void()> &reeval) {
    int rmax = std::min(std::min(c->o.rank_cap, kMaxRankLds), std::min(m, n));
    double *info = nullptr;
    int *piv = pivot_buffer(c, rmax, &info);
    double *L = c->sc.get<double>(S_L, (size_t)m * rmax);
    double *ws = c->sc.get<double>(S_ROWBUF, prrlu_ws_doubles(m, n));
    bool persistent = true;
    ev_record(c, KC_PIVOT);
    int next = prrlu(c->s, m, n, B, rmax, rel_tol2, piv, piv + rmax, L, info, ws, 0,
                     pivot_guess(c, hist_slot, n, rmax) + 1);
    ev_record(c, KC_PIVOT);
    for (;;) {
        WTT_HIP(hipMemcpyAsync(c->h_pinned_int, piv, pivot_info_offset(rmax) + 3 * sizeof(double),
                               hipMemcpyDeviceToHost, c->s));
        host_wait(c);
        const double state = pinned_pivot_info(c, rmax, 0);
        if (state >= 0.0) break;
        if (state == -2.0) {
            WTT_REQUIRE(persistent, WENOTT_EHIP, "pivot search: the stepped form reported a persistent failure");
            persistent = false;
            c->info.pivot_fallbacks += 1;
            reeval();
            ev_record(c, KC_PIVOT);
            next = prrlu(c->s, m, n, B, rmax, rel_tol2, piv, piv + rmax, L, info, ws, 0,
                         pivot_guess(c, hist_slot, n, rmax) + 1, false);
            ev_record(c, KC_PIVOT);
            continue;
        }
        WTT_REQUIRE(next <= rmax + 1, WENOTT_EHIP, "pivot search did not stop");
        ev_record(c, KC_PIVOT);
        next = prrlu(c->s, m, n, B, rmax, rel_tol2, piv, piv + rmax, L, info, ws, next, next + std::max(8, next / 2),
                     persistent);
        ev_record(c, KC_PIVOT);
    }
    PivotResult r;
    r.rank = (int)pinned_pivot_info(c, rmax, 0);
    // stopped at the rank limit with the residual above the tolerance
    r.capped = r.rank >= rmax && rmax < std::min(m, n) && pinned_pivot_info(c, rmax, 1) > pinned_pivot_info(c, rmax, 2);
    if (r.capped) c->info.rank_capped += 1;
    if (hist_slot >= 0) c->piv_hist[hist_slot] = r.rank;
    r.cols.assign(c->h_pinned_int + rmax, c->h_pinned_int + rmax + r.rank);
    c->info.pivots_total += r.rank;
    {  // full-pivot elimination to rank r: sum_t 2 (m - t)(n - t) flops; the block is read once, L written
        double fl = 0.0;
        for (int t = 0; t < r.rank; ++t) fl += 2.0 * (double)(m - t) * (double)(n - t);
        add_work(c, KC_PIVOT, fl, 8.0 * ((double)m * n + (double)m * r.rank));
    }
    r.rows.assign(c->h_pinned_int, c->h_pinned_int + r.rank);
    *Lout = L;
    return r;
}

double sampled_residual(wenott_ctx *c, const TT &U, const FluxTT &F, int dir, double alpha, Rng &rng, int law,
                        bool lf = false) {
    const int d = U.d, npts = std::max(c->o.probe_points, 16);
    FiberGeom g{};
    g.d = d; g.ncomp = U.nc; g.dir = dir; g.k = 0;
    for (int j = 0; j < d; ++j) { g.n[j] = U.N[j]; g.bc[j] = c->bc[j]; }
    g.law = law; std::memcpy(g.qin, c->qin, sizeof g.qin); g.gamma = c->gamma; g.alpha = alpha; g.eps_w = c->h[dir] * c->h[dir];
    int *dp = c->sc.get<int>(S_PTS, (size_t)npts * d);
    sample_points(c->s, npts, d, F.M, rng.next(), dp);
    double *ust = c->sc.get<double>(S_UST, (size_t)npts * 6 * U.nc);
    int nb = (npts + 255) / 256;
    WTT_REQUIRE(nb <= kMaxResidualBlocks, WENOTT_EINVAL, "too many probe points");
    double *acc = c->d_status + kStatusAcc;
    int ranks[kMaxDim + 1], franks[kMaxDim + 1];
    for (int j = 0; j <= d; ++j) { ranks[j] = U.R[j]; franks[j] = F.R[j]; }
    const double *uc[kMaxDim], *fc[kMaxDim];
    for (int j = 0; j < d; ++j) { uc[j] = U.core[j]; fc[j] = F.core[j]; }
    if (lf) sample_lf_residual(c->s, g, uc, ranks, npts, dp, fc, franks, ust, acc, c->d_flags);
    else sample_residual(c->s, g, uc, ranks, npts, dp, fc, franks, ust, acc, c->d_flags);
    WTT_REQUIRE(2 * (size_t)nb <= 3000, WENOTT_EINVAL, "too many probe points");
    status_readback(c, kStatusAcc + 2 * nb);
    host_wait(c);
    raise_flags(c, status_flags(c));
    const double *h = c->h_status + kStatusAcc;
    double d2 = 0.0, n2 = 0.0;
    for (int b = 0; b < nb; ++b) { d2 += h[2 * b]; n2 += h[2 * b + 1]; }
    return n2 > 0.0 ? std::sqrt(d2 / n2) : std::sqrt(d2);
}

// ---------------------------------------------------------------------- the cross
struct CrossStat {
    int sweeps = 0;
    double residual = 0.0;
    int maxrank = 0;
};

// ------------------------------------------------------------- learned proposal hooks
// Per-bond features of the proposal (see include/wenott.h): the previous cross's useful-right-
// index histogram, the last rounding's singular-value tail, log rank, eps, CFL, sweeps,
// residual, stage and dimension.
std::vector<float> proposal_features(wenott_ctx *c, int d, double eps, double lambda, int stage) {
    const int IN = WENOTT_MLP_IN, NB = WENOTT_MLP_BINS;
    std::vector<float> x((size_t)(d - 1) * IN, 0.f);
    for (int k = 0; k < d - 1; ++k) {
        float *f = x.data() + (size_t)k * IN;
        const auto &b = c->bond[k];
        for (int j = 0; j < NB; ++j) f[j] = b.hist[j];
        for (int j = 0; j < 16; ++j) f[NB + j] = b.sig[j];
        f[80] = (float)(std::log2((double)b.rank + 1.0) / 8.0);
        f[81] = (float)(std::log10(eps) / 16.0 + 1.0);
        f[82] = (float)lambda;
        f[83] = (float)(c->prev_sweeps / 4.0);
        f[84] = (float)(std::min(4.0, std::max(-4.0, std::log10(std::max(c->prev_resid, 1e-300) / eps))) / 4.0);
        if (stage >= 0 && stage < 3) f[85 + stage] = 1.f;
        f[88] = (float)(d - 2);
    }
    return x;
}

// Right index sets from the proposal: the previous useful multi-indices, then new ones whose
// first mode is drawn from the predicted bin distribution, up to the predicted rank + 2.
void apply_proposal(wenott_ctx *c, int d, const int *M, const std::vector<float> &x, std::vector<ISet> &Rset,
                    Rng &rng) {
    const int OUT = WENOTT_MLP_OUT, NR = WENOTT_MLP_RANK_CLASSES, NB = WENOTT_MLP_BINS;
    const int nb = d - 1;
    const float *dx = c->ring.put(x.data(), x.size());
    float *y = c->sc.get<float>(S_MLPY, (size_t)nb * OUT);
    float *work = c->sc.get<float>(S_MLPW, (size_t)wenott_mlp_workspace(nb));
    WTT_REQUIRE(wenott_mlp_forward(c->proposal, dx, nb, y, 1, work, c->s) == WENOTT_OK, WENOTT_EHIP,
                "proposal forward failed");
    std::vector<float> hy((size_t)nb * OUT);
    WTT_HIP(hipMemcpyAsync(hy.data(), y, hy.size() * sizeof(float), hipMemcpyDeviceToHost, c->s));
    host_wait(c);
    for (int k = 0; k < nb; ++k) {
        const float *yk = hy.data() + (size_t)k * OUT;
        int cls = 0;
        for (int j = 1; j < NR; ++j)
            if (yk[j] > yk[cls]) cls = j;
        const auto &b = c->bond[k];
        const int rhat = std::max(1, b.rank + cls - NR / 2);
        const int want = rhat + 2;
        const int len = d - 1 - k;
        ISet s;
        s.len = len;
        const int nuse = std::min<int>((int)b.useful.size() / len, want);
        s.v.assign(b.useful.begin(), b.useful.begin() + (size_t)nuse * len);
        s.count = nuse;
        // bin distribution
        float mx = yk[NR];
        for (int j = 1; j < NB; ++j) mx = std::max(mx, yk[NR + j]);
        std::vector<double> p(NB);
        double tot = 0.0;
        for (int j = 0; j < NB; ++j) tot += (p[j] = std::exp((double)yk[NR + j] - mx));
        while (s.count < want) {
            double u = (rng.next() >> 11) * (1.0 / 9007199254740992.0) * tot, acc = 0.0;
            int bin = NB - 1;
            for (int j = 0; j < NB; ++j) {
                acc += p[j];
                if (u < acc) { bin = j; break; }
            }
            const int m = M[k + 1];
            const int lo = (int)((long long)bin * m / NB), hi = std::max(lo + 1, (int)((long long)(bin + 1) * m / NB));
            s.v.push_back(std::min(m - 1, lo + rng.below(hi - lo)));
            for (int j = 1; j < len; ++j) {
                if (nuse > 0) s.v.push_back(b.useful[(size_t)rng.below(nuse) * len + j]);
                else s.v.push_back(rng.below(M[k + 1 + j]));
            }
            ++s.count;
        }
        Rset[k] = std::move(s);
    }
}

// After a stage cross: log (features, rank class, useful-index histogram) and update the bond
// histories. usedR[k] is the right set of core k in the accepted sweep, usedC[k] its pivot columns.
void learn_update(wenott_ctx *c, int d, int nc, const int *M, const FluxTT &F, const std::vector<ISet> &usedR,
                  const std::vector<std::vector<int>> &usedC, const std::vector<float> &feats, bool have_feats,
                  int sweeps, double resid) {
    const int IN = WENOTT_MLP_IN, NB = WENOTT_MLP_BINS, NR = WENOTT_MLP_RANK_CLASSES;
    for (int k = 0; k < d - 1; ++k) {
        auto &b = c->bond[k];
        const ISet &R = usedR[k];
        float hist[WENOTT_MLP_BINS] = {};
        std::vector<int> useful;
        std::vector<char> seen(R.count, 0);
        for (int col : usedC[k]) {
            const int bi = col / nc;
            if (bi < 0 || bi >= R.count || seen[bi]) continue;
            seen[bi] = 1;
            const int pos = R.v[(size_t)bi * R.len];
            hist[std::min(NB - 1, (int)((long long)pos * NB / M[k + 1]))] += 1.f;
            useful.insert(useful.end(), R.v.begin() + (size_t)bi * R.len, R.v.begin() + (size_t)(bi + 1) * R.len);
        }
        float tot = 0.f;
        for (float h : hist) tot += h;
        if (tot > 0.f)
            for (float &h : hist) h /= tot;
        const int rnew = F.R[k + 1];
        if (c->logging && have_feats && b.valid) {
            const int cls = std::min(NR - 1, std::max(0, rnew - b.rank + NR / 2));
            c->log_x.insert(c->log_x.end(), feats.begin() + (size_t)k * IN, feats.begin() + (size_t)(k + 1) * IN);
            c->log_cls.push_back(cls);
            c->log_hist.insert(c->log_hist.end(), hist, hist + NB);
        }
        b.valid = true;
        b.rank = rnew;
        std::memcpy(b.hist, hist, sizeof(hist));
        b.useful = std::move(useful);
    }
    c->prev_sweeps = sweeps;
    c->prev_resid = resid;
}

// A cross target: mode sizes, a block evaluator and the sampled residual of a candidate TT.
struct CrossTarget {
    int d = 0, nc = 0, q0 = 2;
    int M[kMaxDim] = {};
    std::function<void(int k, const ISet &L, const ISet &R, bool lr, double *out)> eval;
    std::function<double(const FluxTT &F, Rng &rng)> residual;
    // Optional speculation: residual_launch queues the residual check without waiting,
    // speculate queues the consumer of an accepted F (and synchronises at its own readbacks),
    // residual_finish then reads the residual, and discard drops the speculative result when
    // the sweep is not accepted.
    std::function<int(const FluxTT &F, Rng &rng)> residual_launch;
    std::function<double(int nb)> residual_finish;
    std::function<void(const FluxTT &F)> speculate;
    std::function<void()> discard;
    int warm_slot = 0;
    bool learn = false;  // stage cross: keep bond histories, log samples, use the proposal
    double lambda = 0.0;
    int stage = -1;
};

// Rank-adaptive cross (Sec. 3.3): left-to-right sweeps build interpolative cores
// B(:, J) B(I, J)^{-1} from full-pivot rank-revealing LU pivots on the unfolding
// (rows: left index x mode, columns: right index x component); a sweep is accepted when the
// relative residual at random points is <= eps, otherwise a right-to-left sweep refreshes the
// right index sets and the next sweep starts with a tighter pivot tolerance. Every sampled
// index set is enriched by kick_rank random indices.
FluxTT cross_generic(wenott_ctx *c, const CrossTarget &t, double eps, CrossStat &st) {
    eps *= c->o.cross_ratio;  // eps_cross
    const int d = t.d, nc = t.nc;
    const int *M = t.M;
    Rng rng(c->o.seed ^ (0x5851F42D4C957F2DULL * (++c->counter)));
    std::vector<ISet> Rset(d);
    Rset[d - 1].len = 0;
    Rset[d - 1].count = 1;
    // Without the previous cross's index sets the right sets start random, and a feature that
    // is localised in every mode (the first update of a discontinuity crossing, say) can fall
    // between them and between the sampled points alike; such a cold start always takes the
    // refresh sweep, whose right sets come from the pivot rows of the first sweep.
    const bool cold = !c->warm_valid[t.warm_slot];
    if (!cold) {
        Rset = c->warm[t.warm_slot];
    } else {
        for (int k = 0; k < d - 1; ++k) Rset[k] = random_set(rng, t.q0, k + 1, d - 1 - k, M);
    }
    std::vector<ISet> Lset(d);
    FluxTT F;
    F.d = d; F.nc = nc;
    for (int j = 0; j < d; ++j) F.M[j] = M[j];
    double rel2 = eps * eps / (4.0 * d);
    int kick = c->o.kick_rank;
    double resid = 1e300;
    int sweep = 0;
    bool have_feats = t.learn;
    for (int k = 0; k < d - 1; ++k) have_feats = have_feats && c->bond[k].valid;
    std::vector<float> feats;
    if (have_feats) feats = proposal_features(c, d, eps, t.lambda, t.stage);
    bool proposed = false;
    if (have_feats && c->proposal && c->o.use_proposal) {
        apply_proposal(c, d, M, feats, Rset, rng);
        proposed = true;
        c->info.proposals_tried += 1;
    }
    std::vector<ISet> usedR(d);
    std::vector<std::vector<int>> usedC(d);
    bool capped = false;  // a pivot search of the last left-to-right sweep stopped at its rank limit
    for (; sweep < c->o.max_sweeps; ++sweep) {
        capped = false;
        bool saturated = false;  // a pivot search used every column of its block
        F.release(c->s);
        Lset[0].len = 0;
        Lset[0].count = 1;
        Lset[0].v.clear();
        F.R[0] = 1;
        F.R[d] = 1;
        for (int k = 0; k < d; ++k) {
            const int kick_now = (proposed && sweep == 0) ? 0 : kick;  // the proposal replaces the random kick
            ISet Rk = k < d - 1 ? with_kick(Rset[k], rng, kick_now, k + 1, M) : Rset[k];
            const int p = Lset[k].count, q = Rk.count;
            const long long rows = (long long)p * M[k], cols = (long long)q * nc;
            // the last core is the block itself: evaluated straight into its allocation
            double *B = k < d - 1 ? c->sc.get<double>(S_BLOCK, (size_t)(rows * cols))
                                  : (F.core[k] = dalloc<double>(c->s, (size_t)(rows * cols)));
            t.eval(k, Lset[k], Rk, true, B);
            if (k < d - 1) {
                double *L = nullptr;
                PivotResult pr = pivots(c, B, (int)rows, (int)cols, rel2, &L, hist_index(t.warm_slot, 0, k),
                                        [&] { t.eval(k, Lset[k], Rk, true, B); });
                capped = capped || pr.capped;
                saturated = saturated || (pr.rank >= cols && cols < rows);
                if (t.learn) {
                    usedR[k] = Rk;
                    usedC[k] = pr.cols;
                }
                const int r = pr.rank;
                int rmax = std::min(std::min(c->o.rank_cap, kMaxRankLds), (int)std::min(rows, cols));
                F.core[k] = dalloc<double>(c->s, (size_t)rows * r);
                interp_solve(c->s, (int)rows, r, L, rmax, c->sc.get<int>(S_PIV, 1), F.core[k]);
                F.R[k + 1] = r;
                ISet nl;
                nl.len = k + 1;
                nl.count = r;
                nl.v.resize((size_t)r * (k + 1));
                for (int tt = 0; tt < r; ++tt) {
                    int row = pr.rows[tt], a = row / M[k], i = row % M[k];
                    for (int j = 0; j < k; ++j) nl.v[(size_t)tt * (k + 1) + j] = Lset[k].v[(size_t)a * k + j];
                    nl.v[(size_t)tt * (k + 1) + k] = i;
                }
                Lset[k + 1] = std::move(nl);
                st.maxrank = std::max(st.maxrank, r);
            }
        }
        if (t.speculate && !(cold && sweep == 0)) {
            // the sweep is usually accepted: its consumer runs behind the residual check, and one
            // synchronisation (the consumer's first readback) serves both
            const int nb = t.residual_launch(F, rng);
            const unsigned long long w0 = c->waits;
            try {
                t.speculate(F);
            } catch (...) {
                host_wait(c);
                raise_flags(c, status_flags(c));  // a flux failure outranks its consequences
                throw;
            }
            if (c->waits == w0) host_wait(c);
            resid = t.residual_finish(nb);
            if (resid <= eps || sweep + 1 == c->o.max_sweeps) { ++sweep; break; }
            t.discard();
        } else {
            resid = t.residual(F, rng);
            if ((resid <= eps && !(cold && sweep == 0)) || sweep + 1 == c->o.max_sweeps) { ++sweep; break; }
        }
        // right-to-left sweep: refresh the right index sets from the new left ones
        for (int k = d - 1; k >= 1; --k) {
            ISet Lk = with_kick(Lset[k], rng, kick, 0, M);
            const ISet &Rk = Rset[k];
            const int p = Lk.count, q = Rk.count;
            const long long rows = (long long)M[k] * q, cols = (long long)p * nc;
            double *B = c->sc.get<double>(S_BLOCK, (size_t)(rows * cols));
            t.eval(k, Lk, Rk, false, B);
            double *L = nullptr;
            PivotResult pr = pivots(c, B, (int)rows, (int)cols, rel2, &L, hist_index(t.warm_slot, 1, k),
                                    [&] { t.eval(k, Lk, Rk, false, B); });
            saturated = saturated || (pr.rank >= cols && cols < rows);
            ISet nr;
            nr.len = d - k;
            nr.count = pr.rank;
            nr.v.resize((size_t)pr.rank * nr.len);
            for (int tt = 0; tt < pr.rank; ++tt) {
                int row = pr.rows[tt], i = row / q, b = row % q;
                nr.v[(size_t)tt * nr.len] = i;
                for (int j = 0; j < Rk.len; ++j) nr.v[(size_t)tt * nr.len + 1 + j] = Rk.v[(size_t)b * Rk.len + j];
            }
            Rset[k - 1] = std::move(nr);
        }
        rel2 *= 0.25;
        // A search that used every column found as many pivots as the index sets allowed: the rank
        // is limited by the sets (one column per index tuple and component, so a single-component
        // law adds at most kick pivots per sweep), not by the tolerance. Such a cross doubles its
        // enrichment for the next sweep.
        if (saturated) kick = std::min(2 * std::max(kick, 2), 128);
    }
    c->warm[t.warm_slot] = Rset;
    c->warm_valid[t.warm_slot] = true;
    st.sweeps = sweep;
    st.residual = resid;
    if (proposed && sweep == 1 && resid <= eps) c->info.proposals_accepted += 1;
    if (t.learn) learn_update(c, d, nc, M, F, usedR, usedC, feats, have_feats, sweep, resid);
    if (!(resid <= c->o.conv_slack * eps) && !(resid <= 1e-12)) {
        F.release(c->s);
        char msg[192];
        std::snprintf(msg, sizeof(msg), "%s (sampled residual %.3e, eps_cross %.3e, %d sweeps, rank %d)",
                      capped ? "cross did not converge: a pivot search stopped at the rank limit"
                             : "cross did not converge within max_sweeps sweeps",
                      resid, eps, sweep, st.maxrank);
        throw StatusError(WENOTT_ENOCONV, msg);
    }
    return F;
}

// Cross of the numerical flux Fhat_dir on the faces (scheme 1; with law and slot given, a
// WENO-cross of scheme 2).
FluxTT cross_flux(wenott_ctx *c, const TT &U, int dir, double alpha, double eps, CrossStat &st, int slot = -1,
                  int law = -1) {
    if (law < 0) law = c->law;
    CrossTarget t;
    t.d = U.d;
    t.nc = U.nc;
    t.q0 = std::max(2, U.maxrank());
    for (int j = 0; j < U.d; ++j) t.M[j] = U.N[j] + (j == dir ? 1 : 0);
    t.eval = [&](int k, const ISet &L, const ISet &R, bool lr, double *out) {
        eval_block(c, U, dir, k, L, R, alpha, lr, out, law);
    };
    t.residual = [&](const FluxTT &F, Rng &rng) { return sampled_residual(c, U, F, dir, alpha, rng, law); };
    t.warm_slot = slot >= 0 ? slot : dir;
    return cross_generic(c, t, eps, st);
}

// LF-cross block (Sec. 4.2): the state at the block's cells, gathered as P G_k Q, then the split
// fluxes f^+ and f^- of every component (2 ncomp outputs per point).
void eval_lf_block(wenott_ctx *c, const TT &U, int dir, int k, const ISet &L, const ISet &Rs, double alpha, bool lr,
                   double *out) {
    const int d = U.d, nc = U.nc;
    FiberGeom g{};
    g.d = d; g.ncomp = nc; g.dir = dir; g.k = k;
    for (int j = 0; j < d; ++j) { g.n[j] = U.N[j]; g.bc[j] = c->bc[j]; }
    g.law = c->law; g.gamma = c->gamma; g.alpha = alpha;
    const int p = L.count, q = Rs.count, Rk = U.R[k], Rk1 = U.R[k + 1], Nk = U.N[k];
    int ranks[kMaxDim + 1];
    for (int j = 0; j <= d; ++j) ranks[j] = U.R[j];
    const double *cores[kMaxDim];
    for (int j = 0; j < d; ++j) cores[j] = U.core[j];
    double *P = c->sc.get<double>(S_P, (size_t)nc * p * Rk);
    if (k == 0) fill(c->s, P, (long long)nc * p * Rk, 1.0);
    else iface(c->s, g, 0, cores, ranks, p, c->ring.put(L.v.data(), L.v.size()), 1, -1, P);
    double *Q = c->sc.get<double>(S_Q, (size_t)nc * Rk1 * q);
    if (k == d - 1) fill(c->s, Q, (long long)nc * Rk1 * q, 1.0);
    else iface(c->s, g, 1, cores, ranks, q, c->ring.put(Rs.v.data(), Rs.v.size()), 1, -1, Q);
    const long long tsz = (long long)p * Nk * Rk1, wsz = (long long)p * Nk * q;
    double *T = c->sc.get<double>(S_T, (size_t)nc * tsz);
    GemmBatch b1;
    b1.nb1 = nc;
    b1.sA1 = (long long)p * Rk; b1.sB1 = U.cstride(k); b1.sC1 = tsz;
    gemm_f64(c->s, false, false, p, Nk * Rk1, Rk, 1.0, P, Rk, U.core[k], Nk * Rk1, 0.0, T, Nk * Rk1, b1);
    double *W = c->sc.get<double>(S_W, (size_t)nc * wsz);
    GemmBatch b2;
    b2.nb1 = nc;
    b2.sA1 = tsz; b2.sB1 = (long long)Rk1 * q; b2.sC1 = wsz;
    gemm_f64(c->s, false, false, p * Nk, q, Rk1, 1.0, T, Rk1, Q, q, 0.0, W, q, b2);
    const int no = 2 * nc;
    long long sa, si, sb, sc;
    if (lr) { sa = (long long)Nk * q * no; si = (long long)q * no; sb = no; sc = 1; }
    else { sa = no; si = (long long)q * p * no; sb = (long long)p * no; sc = 1; }
    ev_record(c, KC_FIBER);
    lf_block(c->s, g, p, q, W, wsz, out, sa, si, sb, sc, c->d_flags);
    ev_record(c, KC_FIBER);
    c->info.fiber_points += (long long)p * Nk * q;
    c->info.fiber_launches += 1;
}

// LF-cross (Sec. 4.2, Algorithm lf-cross): one cross of the 2 ncomp split fluxes at the cells,
// a TT whose last core carries the 2 ncomp slices.
FluxTT cross_lf(wenott_ctx *c, const TT &U, int dir, double alpha, double eps, CrossStat &st) {
    CrossTarget t;
    t.d = U.d;
    t.nc = 2 * U.nc;
    t.q0 = std::max(2, U.maxrank());
    for (int j = 0; j < U.d; ++j) t.M[j] = U.N[j];
    t.eval = [&](int k, const ISet &L, const ISet &R, bool lr, double *out) {
        eval_lf_block(c, U, dir, k, L, R, alpha, lr, out);
    };
    t.residual = [&](const FluxTT &F, Rng &rng) { return sampled_residual(c, U, F, dir, alpha, rng, c->law, true); };
    t.warm_slot = kSlotLf + dir;
    return cross_generic(c, t, eps, st);
}

// ------------------------------------------------------------------- stage value
struct StageWeights {
    double wn, wx, wl;  // Y = wn Un + wx X + wl L(X)
};

// Interface matrices + gathered stencil blocks of X (and Un) for core k, then the fused stage kernel.
void eval_stage_block(wenott_ctx *c, const TT &X, const TT *Un, StageWeights w, double alpha, int k, const ISet &L,
                      const ISet &Rs, bool lr, double *out) {
    const int d = X.d, nc = X.nc;
    hipStream_t s = c->s;
    FiberGeom g{};
    g.d = d; g.ncomp = nc; g.dir = 0; g.k = k;
    for (int j = 0; j < d; ++j) { g.n[j] = X.N[j]; g.bc[j] = c->bc[j]; }
    g.law = c->law; std::memcpy(g.qin, c->qin, sizeof g.qin); g.gamma = c->gamma; g.alpha = alpha; g.eps_w = 0.0; g.alpha_dev = c->alpha_dev;
    const int p = L.count, q = Rs.count, Nk = X.N[k];
    const int *didxL = k > 0 ? c->ring.put(L.v.data(), L.v.size()) : nullptr;
    const int *didxR = k < d - 1 ? c->ring.put(Rs.v.data(), Rs.v.size()) : nullptr;

    // W = P G_k Q for a TT (X or Un); S shifts on P (left) or Q (right) of mode `shift`. In two
    // parts, so that the interface matrices of all the gathers of a block go in one launch: gplan
    // takes P and Q from their slots and queues their requests, gfinish forms T = P G_k and
    // W = T Q. A GatherJob stays in place until its requests have been launched.
    struct GatherJob {
        const TT *Y = nullptr;
        int shift = -1, slotP = 0, slotQ = 0, slotT = 0, slotW = 0, SL = 1, SR = 1;
        int ranks[kMaxDim + 1] = {};
        const double *cores[kMaxDim] = {};
        double *P = nullptr, *Q = nullptr;
    };
    auto gplan = [&](GatherJob &G, std::vector<IfaceReq> &rq) {
        const TT &Y = *G.Y;
        for (int j = 0; j <= d; ++j) G.ranks[j] = Y.R[j];
        for (int j = 0; j < d; ++j) G.cores[j] = Y.core[j];
        G.SL = (G.shift >= 0 && G.shift < k) ? 7 : 1;
        G.SR = (G.shift > k) ? 7 : 1;
        if (k > 0) {  // at the first core the left part is the scalar 1 (p = 1, R_0 = 1)
            G.P = c->sc.get<double>(G.slotP, (size_t)nc * G.SL * p * Y.R[k]);
            rq.push_back(IfaceReq{G.cores, G.ranks, 0, p, G.SL, G.SL == 7 ? G.shift : -1, didxL, G.P});
        }
        if (k < d - 1) {  // at the last core the right part is the scalar 1 (q = 1, R_d = 1)
            G.Q = c->sc.get<double>(G.slotQ, (size_t)nc * G.SR * Y.R[k + 1] * q);
            rq.push_back(IfaceReq{G.cores, G.ranks, 1, q, G.SR, G.SR == 7 ? G.shift : -1, didxR, G.Q});
        }
    };
    auto gfinish = [&](GatherJob &G) -> double * {
        const TT &Y = *G.Y;
        const int Rk = Y.R[k], Rk1 = Y.R[k + 1], SL = G.SL, SR = G.SR, S = std::max(SL, SR);
        const long long tsz = (long long)p * Nk * Rk1;
        // Shifts on the left with a right part: W_s = P_s (G_k Q) forms G_k Q once instead of
        // P_s G_k for every shift, when that is fewer multiply-adds
        // (Rk Nk Rk1 q + SL p Rk Nk q against SL p Nk Rk1 (Rk + q)).
        if (SL > 1 && k < d - 1 &&
            (double)Rk * Rk1 * q + (double)SL * p * Rk * q < (double)SL * p * Rk1 * (Rk + q)) {
            const long long zsz = (long long)Rk * Nk * q, wsz = (long long)p * Nk * q;
            double *Z = c->sc.get<double>(G.slotT, (size_t)nc * zsz);
            GemmBatch bz;
            bz.nb1 = nc;
            bz.sA1 = Y.cstride(k); bz.sB1 = (long long)Rk1 * q; bz.sC1 = zsz;
            gemm_f64(s, false, false, Rk * Nk, q, Rk1, 1.0, Y.core[k], Rk1, G.Q, q, 0.0, Z, q, bz);
            double *W = c->sc.get<double>(G.slotW, (size_t)nc * SL * wsz);
            GemmBatch bw;
            bw.nb1 = nc; bw.nb2 = SL;
            bw.sA1 = (long long)SL * p * Rk; bw.sA2 = (long long)p * Rk;
            bw.sB1 = zsz; bw.sB2 = 0;
            bw.sC1 = SL * wsz; bw.sC2 = wsz;
            gemm_f64(s, false, false, p, Nk * q, Rk, 1.0, G.P, Rk, Z, Nk * q, 0.0, W, Nk * q, bw);
            return W;
        }
        // T = P G_k; at the first core T is the core itself
        const double *T;
        long long tA1;
        if (k == 0) {
            T = Y.core[k];
            tA1 = Y.cstride(k);
        } else {
            double *Tm = c->sc.get<double>(G.slotT, (size_t)nc * SL * tsz);
            GemmBatch b1;
            b1.nb1 = nc; b1.nb2 = SL;
            b1.sA1 = (long long)SL * p * Rk; b1.sA2 = (long long)p * Rk;
            b1.sB1 = Y.cstride(k); b1.sB2 = 0;
            b1.sC1 = SL * tsz; b1.sC2 = tsz;
            gemm_f64(s, false, false, p, Nk * Rk1, Rk, 1.0, G.P, Rk, Y.core[k], Nk * Rk1, 0.0, Tm, Nk * Rk1, b1);
            T = Tm;
            tA1 = SL * tsz;
        }
        // W = T Q; at the last core W = T
        if (k == d - 1) return const_cast<double *>(T);
        const long long wsz = (long long)p * Nk * q;
        double *W = c->sc.get<double>(G.slotW, (size_t)nc * S * wsz);
        GemmBatch b2;
        b2.nb1 = nc; b2.nb2 = S;
        b2.sA1 = tA1; b2.sA2 = SL == 7 ? tsz : 0;
        b2.sB1 = (long long)SR * Rk1 * q; b2.sB2 = SR == 7 ? (long long)Rk1 * q : 0;
        b2.sC1 = S * wsz; b2.sC2 = wsz;
        gemm_f64(s, false, false, p * Nk, q, Rk1, 1.0, T, Rk1, G.Q, q, 0.0, W, q, b2);
        return W;
    };
    auto gather = [&](const TT &Y, int shift, int slotP, int slotQ, int slotT, int slotW) -> double * {
        GatherJob G;
        G.Y = &Y; G.shift = shift; G.slotP = slotP; G.slotQ = slotQ; G.slotT = slotT; G.slotW = slotW;
        std::vector<IfaceReq> rq;
        gplan(G, rq);
        iface_batch(s, g, (int)rq.size(), rq.data());
        return gfinish(G);
    };
    // FP32 gather: interface matrices formed in FP64 and rounded, the block contractions
    // P G_k Q in FP32 on the matrix cores.
    auto gather32 = [&](const TT &Y, int shift, int slotW) -> float * {
        const int Rk = Y.R[k], Rk1 = Y.R[k + 1];
        int ranks[kMaxDim + 1];
        for (int j = 0; j <= d; ++j) ranks[j] = Y.R[j];
        const double *cores[kMaxDim];
        for (int j = 0; j < d; ++j) cores[j] = Y.core[j];
        const int SL = (shift >= 0 && shift < k) ? 7 : 1, SR = (shift > k) ? 7 : 1, S = std::max(SL, SR);
        double *P = c->sc.get<double>(S_P, (size_t)nc * SL * p * Rk);
        if (k == 0) fill(s, P, (long long)nc * SL * p * Rk, 1.0);
        else iface(s, g, 0, cores, ranks, p, didxL, SL, SL == 7 ? shift : -1, P);
        double *Q = c->sc.get<double>(S_Q, (size_t)nc * SR * Rk1 * q);
        if (k == d - 1) fill(s, Q, (long long)nc * SR * Rk1 * q, 1.0);
        else iface(s, g, 1, cores, ranks, q, didxR, SR, SR == 7 ? shift : -1, Q);
        float *P32 = c->sc.get<float>(S_F_P, (size_t)nc * SL * p * Rk);
        float *Q32 = c->sc.get<float>(S_F_Q, (size_t)nc * SR * Rk1 * q);
        float *G32 = c->sc.get<float>(S_F_G, (size_t)Y.cstride(k) * nc);
        to_f32(s, (long long)nc * SL * p * Rk, P, P32);
        to_f32(s, (long long)nc * SR * Rk1 * q, Q, Q32);
        to_f32(s, Y.cstride(k) * nc, Y.core[k], G32);
        const long long tsz = (long long)p * Nk * Rk1;
        float *T = c->sc.get<float>(S_F_T, (size_t)nc * SL * tsz);
        GemmBatch b1;
        b1.nb1 = nc; b1.nb2 = SL;
        b1.sA1 = (long long)SL * p * Rk; b1.sA2 = (long long)p * Rk;
        b1.sB1 = Y.cstride(k); b1.sB2 = 0;
        b1.sC1 = SL * tsz; b1.sC2 = tsz;
        gemm_f32(s, p, Nk * Rk1, Rk, P32, Rk, G32, Nk * Rk1, T, Nk * Rk1, b1);
        const long long wsz = (long long)p * Nk * q;
        float *W = c->sc.get<float>(slotW, (size_t)nc * S * wsz);
        GemmBatch b2;
        b2.nb1 = nc; b2.nb2 = S;
        b2.sA1 = SL * tsz; b2.sA2 = SL == 7 ? tsz : 0;
        b2.sB1 = (long long)SR * Rk1 * q; b2.sB2 = SR == 7 ? (long long)Rk1 * q : 0;
        b2.sC1 = S * wsz; b2.sC2 = wsz;
        gemm_f32(s, p * Nk, q, Rk1, T, Rk1, Q32, q, W, q, b2);
        return W;
    };
    StageArgsT<double> a{};
    StageArgsT<float> a32{};
    const bool fp32 = c->o.precision == 1;
    const long long blk = (long long)p * Nk * q;
    a.w0_cs = a32.w0_cs = blk;
    if (fp32) {  // the FP64 values of X at the block points for the combination, FP32 for the fluxes
        a.W0 = gather(X, -1, S_P, S_Q, S_T, S_W);
        a.X0 = a.W0;
        a32.W0 = gather32(X, -1, S_F_W0);
        a32.X0 = a.W0;
    }
    // FP64: the gathers of X along the other directions and of Un, their interface matrices in
    // one launch
    GatherJob gj[kMaxDim + 1];
    int gdir[kMaxDim + 1], ng = 0;
    int od = 0;
    for (int dd = 0; dd < d; ++dd) {
        a.inv_h[dd] = a32.inv_h[dd] = 1.0 / c->h[dd];
        a.eps_w[dd] = a32.eps_w[dd] = c->h[dd] * c->h[dd];
        if (dd == k) continue;
        if (fp32) {
            float *W32 = gather32(X, dd, od == 0 ? S_F_WD0 : S_F_WD1);
            fill_inflow_block<float>(c, g, dd, k, L, Rs, 7, Nk, W32);
            a32.Wd[dd] = W32;
        } else {
            GatherJob &G = gj[ng];
            G.Y = &X; G.shift = dd;
            G.slotP = od == 0 ? S_PD0 : S_PD1; G.slotQ = od == 0 ? S_QD0 : S_QD1;
            G.slotT = od == 0 ? S_TD0 : S_TD1; G.slotW = od == 0 ? S_WD0 : S_WD1;
            gdir[ng++] = dd;
        }
        ++od;
    }
    a.WN = nullptr;
    const bool want_un = Un && w.wn != 0.0;
    if (fp32) {
        if (want_un) a.WN = gather(*Un, -1, S_PN, S_QN, S_TN, S_WN);
    } else {
        if (want_un) {
            GatherJob &G = gj[ng];
            G.Y = Un; G.shift = -1; G.slotP = S_PN; G.slotQ = S_QN; G.slotT = S_TN; G.slotW = S_WN;
            gdir[ng++] = -1;
        }
        std::vector<IfaceReq> rq;
        for (int i = 0; i < ng; ++i) gplan(gj[i], rq);
        iface_batch(s, g, (int)rq.size(), rq.data());
        bool first = true;
        for (int i = 0; i < ng; ++i) {
            double *W = gfinish(gj[i]);
            if (gdir[i] < 0) {
                a.WN = W;
            } else {
                fill_inflow_block<double>(c, g, gdir[i], k, L, Rs, 7, Nk, W);
                a.Wd[gdir[i]] = W;
                if (first) {  // X at the block points is the unshifted (centre) slice of this gather
                    a.W0 = W + 3 * blk;
                    a.X0 = a.W0;
                    a.w0_cs = 7 * blk;
                    first = false;
                }
            }
        }
    }
    a.wn = a32.wn = w.wn; a.wx = a32.wx = w.wx; a.wl = a32.wl = w.wl;
    a32.WN = a.WN;
    long long sa, si, sb, sc;
    if (lr) { sa = (long long)Nk * q * nc; si = (long long)q * nc; sb = nc; sc = 1; }
    else { sa = nc; si = (long long)q * p * nc; sb = (long long)p * nc; sc = 1; }
    ev_record(c, KC_FIBER);
    if (fp32) stage_block<float>(s, g, p, q, a32, out, sa, si, sb, sc, c->d_flags);
    else stage_block<double>(s, g, p, q, a, out, sa, si, sb, sc, c->d_flags);
    ev_record(c, KC_FIBER);
    c->info.fiber_points += (long long)p * Nk * q;
    c->info.fiber_launches += 1;
    {  // per point and direction: 7 cells x (primitives, flux, split) + 4 nc WENO5 + difference;
       // distinct gathered values: the point itself, 6 shifted cells per other direction, Un
        const double pts = (double)p * Nk * q;
        const double per = d == 2 ? 2894.0 : 5398.0;
        const double reads = (1.0 + 6.0 * (d - 1) + (a.WN ? 1.0 : 0.0)) * nc * 8.0;
        add_work(c, KC_FIBER, pts * per, pts * (reads + nc * 8.0));
    }
}

int sampled_stage_residual_launch(wenott_ctx *c, const TT &X, const TT *Un, StageWeights w, double alpha,
                                  const FluxTT &F, Rng &rng) {
    const int d = X.d, npts = std::max(c->o.probe_points, 16);
    FiberGeom g{};
    g.d = d; g.ncomp = X.nc; g.dir = 0; g.k = 0;
    for (int j = 0; j < d; ++j) { g.n[j] = X.N[j]; g.bc[j] = c->bc[j]; }
    g.law = c->law; std::memcpy(g.qin, c->qin, sizeof g.qin); g.gamma = c->gamma; g.alpha = alpha; g.alpha_dev = c->alpha_dev;
    const unsigned long long seed = rng.next();
    const int SL = 7 * d + 1;
    double *ust = c->sc.get<double>(S_UST, (size_t)npts * SL * X.nc);
    const int nb = sample_stage_blocks(d, npts);
    WTT_REQUIRE(nb <= kMaxResidualBlocks, WENOTT_EINVAL, "too many probe points");
    double *acc = c->d_status + kStatusAcc;
    int xr[kMaxDim + 1], nr[kMaxDim + 1], fr[kMaxDim + 1];
    const double *xc[kMaxDim], *ncs[kMaxDim], *fc[kMaxDim];
    for (int j = 0; j <= d; ++j) { xr[j] = X.R[j]; fr[j] = F.R[j]; nr[j] = Un ? Un->R[j] : 1; }
    for (int j = 0; j < d; ++j) { xc[j] = X.core[j]; fc[j] = F.core[j]; ncs[j] = Un ? Un->core[j] : nullptr; }
    double inv_h[kMaxDim], eps_w[kMaxDim];
    for (int j = 0; j < d; ++j) { inv_h[j] = 1.0 / c->h[j]; eps_w[j] = c->h[j] * c->h[j]; }
    const bool use_un = Un && w.wn != 0.0;
    sample_stage(c->s, g, xc, xr, use_un ? ncs : nullptr, nr, npts, seed, fc, fr, use_un ? w.wn : 0.0, w.wx, w.wl,
                 inv_h, eps_w, ust, acc, c->d_flags);
    status_readback(c, kStatusAcc + 2 * nb);
    return nb;
}

// Residual from the pinned copies of a launched sampled residual (after a synchronisation).
double sampled_residual_finish(wenott_ctx *c, int nb) {
    raise_flags(c, status_flags(c));
    const double *h = c->h_status + kStatusAcc;
    double d2 = 0.0, n2 = 0.0;
    for (int b = 0; b < nb; ++b) { d2 += h[2 * b]; n2 += h[2 * b + 1]; }
    return n2 > 0.0 ? std::sqrt(d2 / n2) : std::sqrt(d2);
}

double sampled_stage_residual(wenott_ctx *c, const TT &X, const TT *Un, StageWeights w, double alpha,
                              const FluxTT &F, Rng &rng) {
    const int nb = sampled_stage_residual_launch(c, X, Un, w, alpha, F, rng);
    host_wait(c);
    return sampled_residual_finish(c, nb);
}

FluxTT cross_stage(wenott_ctx *c, const TT &X, const TT *Un, StageWeights w, double alpha, double eps,
                   CrossStat &st, const std::function<void(const FluxTT &)> *speculate = nullptr,
                   const std::function<void()> *discard = nullptr) {
    // FP32 flux evaluation: the face-flux differences (Fhat(+1/2) - Fhat(-1/2)) / h cancel, so
    // the dt L part of the stage value carries relative noise up to ~1e-6 of the stage value;
    // the cross tolerance is floored there (pivots chasing FP32 noise would run to the cap).
    if (c->o.precision == 1) eps = std::max(eps, 1e-6);
    CrossTarget t;
    t.d = X.d;
    t.nc = X.nc;
    t.q0 = std::max(2, X.maxrank());
    for (int j = 0; j < X.d; ++j) t.M[j] = X.N[j];
    t.eval = [&](int k, const ISet &L, const ISet &R, bool lr, double *out) {
        eval_stage_block(c, X, Un, w, alpha, k, L, R, lr, out);
    };
    t.residual = [&](const FluxTT &F, Rng &rng) { return sampled_stage_residual(c, X, Un, w, alpha, F, rng); };
    if (speculate && discard) {
        t.residual_launch = [&](const FluxTT &F, Rng &rng) {
            return sampled_stage_residual_launch(c, X, Un, w, alpha, F, rng);
        };
        t.residual_finish = [&](int nb) { return sampled_residual_finish(c, nb); };
        t.speculate = *speculate;
        t.discard = *discard;
    }
    t.warm_slot = kMaxDim;
    t.learn = w.wx != 0.0;  // stage crosses of rk3_step
    double hmin = c->h[0];
    for (int j = 1; j < X.d; ++j) hmin = std::min(hmin, c->h[j]);
    t.lambda = w.wx != 0.0 ? w.wl / w.wx * alpha / hmin : 0.0;
    t.stage = w.wx == 0.0 ? -1 : (w.wn == 0.0 ? 0 : (w.wn > 0.5 ? 1 : 2));
    return cross_generic(c, t, eps, st);
}

// Per-component TT of a cross result: shared cores copied to every component, the last
// core split into its component slices. With dir >= 0 the result is the flux term
// L_dir = -(T^dir - 1) Fhat_dir / h_dir: the shift difference acts on core dir only
// (eqs. shifted-fluxes and euler-system-TT) and maps its N + 1 faces to N cells.
TT cross_to_tt(wenott_ctx *c, const FluxTT &F, int dir) {
    const int d = F.d, nc = F.nc;
    TT L;
    L.d = d; L.nc = nc;
    for (int j = 0; j < d; ++j) L.N[j] = c->N[j];
    for (int j = 0; j <= d; ++j) L.R[j] = F.R[j];
    L.alloc(c->s);
    const double scale = dir >= 0 ? -1.0 / c->h[dir] : 1.0;
    for (int k = 0; k < d - 1; ++k) {
        long long len = L.cstride(k);
        if (k == dir) {
            double *tmp = c->sc.get<double>(S_TMP, (size_t)len);
            face_diff(c->s, 1, F.R[k], L.N[k], F.R[k + 1], F.core[k], 0, scale, tmp, 0);
            broadcast_core(c->s, nc, len, tmp, L.core[k], len);
        } else {
            broadcast_core(c->s, nc, len, F.core[k], L.core[k], len);
        }
    }
    const int k = d - 1;
    if (k == dir) {
        long long per = (long long)F.R[k] * F.M[k];
        double *tmp = c->sc.get<double>(S_TMP, (size_t)per * nc);
        split_last(c->s, F.R[k], F.M[k], nc, F.core[k], tmp, per);
        face_diff(c->s, nc, F.R[k], L.N[k], 1, tmp, per, scale, L.core[k], L.cstride(k));
    } else {
        split_last(c->s, F.R[k], F.M[k], nc, F.core[k], L.core[k], L.cstride(k));
    }
    return L;
}

// sum_t w_t X_t by core concatenation (first cores side by side, middle block-diagonal,
// last stacked); the weights go on the first cores.
TT tt_sum(wenott_ctx *c, const std::vector<std::pair<double, const TT *>> &terms) {
    const TT &a = *terms[0].second;
    TT S;
    S.d = a.d; S.nc = a.nc;
    for (int j = 0; j < a.d; ++j) S.N[j] = a.N[j];
    S.R[0] = S.R[a.d] = 1;
    for (int k = 1; k < a.d; ++k) {
        S.R[k] = 0;
        for (auto &t : terms) S.R[k] += t.second->R[k];
    }
    S.alloc(c->s);
    for (int k = 0; k < S.d; ++k) fill(c->s, S.core[k], S.cstride(k) * S.nc, 0.0);
    std::vector<int> off(S.d + 1, 0);
    for (auto &t : terms) {
        const TT &X = *t.second;
        for (int k = 0; k < S.d; ++k) {
            int orow = (k == 0) ? 0 : off[k];
            int ocol = (k == S.d - 1) ? 0 : off[k + 1];
            place_block(c->s, S.nc, X.R[k], S.N[k], X.R[k + 1], X.core[k], X.cstride(k), k == 0 ? t.first : 1.0,
                        S.core[k], S.R[k], S.R[k + 1], S.cstride(k), orow, ocol);
        }
        for (int k = 1; k < S.d; ++k) off[k] += X.R[k];
    }
    return S;
}

// SVD pieces of a batch of tall matrices: sigma (sorted) and V, then per-component ranks.
int svd_ranks(wenott_ctx *c, int m, int n, const double *A, long long sz, long long rs, long long cs,
              const double *delta_abs, double rel, int rcap, double **sig, double **V, int **rk) {
    const int nc = c->U.nc;
    double *scr = c->sc.get<double>(S_TSQR, tsqr_scratch_doubles(m, n, nc));
    double *R = c->sc.get<double>(S_R, (size_t)nc * n * n);
    ev_record(c, KC_TSQR);
    tsqr_r(c->s, m, n, nc, A, sz, rs, cs, R, scr);
    ev_record(c, KC_TSQR);
    add_work(c, KC_TSQR, nc * (2.0 * m * (double)n * n - 2.0 / 3.0 * (double)n * n * n), 8.0 * nc * (double)m * n);
    *sig = c->sc.get<double>(S_SIG, (size_t)nc * n);
    *V = c->sc.get<double>(S_V, (size_t)nc * n * n);
    double *jac = c->sc.get<double>(S_JAC, jacobi_scratch_doubles(n, nc));
    *rk = c->sc.get<int>(S_RANKS, nc);
    TruncArgs ta;
    ta.delta_abs = delta_abs; ta.rel = rel; ta.rcap = rcap; ta.ranks = *rk;
    ev_record(c, KC_SVD);
    const bool fused = jacobi_svd(c->s, n, nc, R, *sig, *V, jac, rel == 0.0 ? delta_abs : nullptr, &ta);
    ev_record(c, KC_SVD);
    add_work(c, KC_SVD, 0.0, 8.0 * nc * 3.0 * (double)n * n);
    if (!fused) trunc_ranks(c->s, n, nc, *sig, delta_abs, rel, rcap, *rk);
    WTT_HIP(hipMemcpyAsync(c->h_pinned_int, *rk, nc * sizeof(int), hipMemcpyDeviceToHost, c->s));
    const bool tail = (size_t)nc * n <= 3000 && (c->o.use_proposal || c->logging);
    if (tail) WTT_HIP(hipMemcpyAsync(c->h_pinned_dbl + 1024, *sig, (size_t)nc * n * sizeof(double), hipMemcpyDeviceToHost, c->s));
    host_wait(c);
    int r = 1;
    for (int z = 0; z < nc; ++z) r = std::max(r, c->h_pinned_int[z]);
    // normalised log singular-value tail (largest over components), a feature of the proposal
    for (int j = 0; j < 16; ++j) {
        double v = 0.0;
        if (tail && j < n)
            for (int z = 0; z < nc; ++z) {
                const double *sg = c->h_pinned_dbl + 1024 + (size_t)z * n;
                if (sg[0] > 0.0) v = std::max(v, 1.0 + std::log10(std::max(sg[j] / sg[0], 1e-16)) / 16.0);
            }
        c->last_sig[j] = (float)v;
    }
    return r;
}

// TT-rounding (Sec. 3.2) with one SVD per bond. Right-to-left, only R factors are formed:
// with T_k the R factor of (G_k x_3 T_{k+1}^T) unfolded as R_{k-1} x (N_k r_k) and transposed,
// the right part X_{>=k} equals T_k^T times a matrix with orthonormal rows. Left-to-right,
// C_k = G'_k x_3 T_{k+1}^T has the singular values of the k-th unfolding; its truncated SVD
// gives the new left-orthonormal core U_r = G'_k (T_{k+1}^T V_r Sigma_r^{-1}), and the next
// core becomes (U_r^T G'_k) G_{k+1}. Each truncation keeps the smallest rank whose discarded
// tail is at most eps ||X_c||_F / sqrt(d-1), so ||X - Y||_F <= eps ||X||_F per component.
// Returns the Frobenius norms of the components in norms.
// norms (out): the component norms ||X_c||_F, when want_norms (one transfer; a caller that only
// needs them at its last rounding skips it for the others).
void round_tt(wenott_ctx *c, TT &X, double eps, bool truncate, std::vector<double> &norms, bool want_norms = true) {
    const int d = X.d, nc = X.nc;
    hipStream_t s = c->s;
    std::vector<double *> T(d + 1, nullptr);
    // right-to-left: R factors only
    for (int k = d - 1; k >= 1; --k) {
        const int Rk = X.R[k], Nk = X.N[k], Rk1 = X.R[k + 1];
        const long long m = (long long)Nk * Rk1;
        const double *C = X.core[k];
        if (k < d - 1) {
            double *Cb = c->sc.get<double>(S_TMP, (size_t)nc * Rk * m);
            GemmBatch b;
            b.nb1 = nc; b.sA1 = X.cstride(k); b.sB1 = (long long)Rk1 * Rk1; b.sC1 = (long long)Rk * m;
            gemm_f64(s, false, true, Rk * Nk, Rk1, Rk1, 1.0, X.core[k], Rk1, T[k + 1], Rk1, 0.0, Cb, Rk1, b);
            C = Cb;
        }
        double *scr = c->sc.get<double>(S_TSQR, tsqr_scratch_doubles((int)m, Rk, nc));
        T[k] = dalloc<double>(s, (size_t)nc * Rk * Rk);
        ev_record(c, KC_TSQR);
        tsqr_r(s, (int)m, Rk, nc, C, (long long)Rk * m, 1, m, T[k], scr);
        ev_record(c, KC_TSQR);
        add_work(c, KC_TSQR, nc * (2.0 * m * (double)Rk * Rk - 2.0 / 3.0 * (double)Rk * Rk * Rk),
                 8.0 * nc * (double)m * Rk);
    }
    // norms: ||X_c|| = ||G_0 T_1^T||_F
    {
        const int N0 = X.N[0], R1 = X.R[1];
        double *C0 = c->sc.get<double>(S_TMP, (size_t)nc * N0 * R1);
        GemmBatch b;
        b.nb1 = nc; b.sA1 = X.cstride(0); b.sB1 = (long long)R1 * R1; b.sC1 = (long long)N0 * R1;
        gemm_f64(s, false, true, N0, R1, R1, 1.0, X.core[0], R1, T[1], R1, 0.0, C0, R1, b);
        // the truncation thresholds delta_c = eps ||X_c|| / sqrt(d - 1) stay on the device; the
        // norms reach the host through a pinned copy read after the next synchronisation
        double *dn = c->sc.get<double>(S_NORMS, 2 * (size_t)nc);
        frob_norms(s, nc, (long long)N0 * R1, C0, (long long)N0 * R1, dn, dn + nc,
                   eps / std::sqrt((double)std::max(d - 1, 1)));
        if (want_norms || !truncate || d < 2)
            WTT_HIP(hipMemcpyAsync(c->h_pinned_dbl + kPinNorms, dn, nc * sizeof(double), hipMemcpyDeviceToHost, s));
        norms.assign(nc, 0.0);
    }
    const double *ddelta = c->sc.get<double>(S_NORMS, 2 * (size_t)nc) + nc;
    if (!truncate || d < 2) {
        host_wait(c);
        norms.assign(c->h_pinned_dbl + kPinNorms, c->h_pinned_dbl + kPinNorms + nc);
        for (int k = 1; k < d; ++k) dfree(s, T[k]);
        return;
    }
    for (int k = 0; k < d - 1; ++k) {
        const int Rk = X.R[k], Nk = X.N[k], n = X.R[k + 1];
        const int m = Rk * Nk;
        double *C = c->sc.get<double>(S_TMP, (size_t)nc * m * n);
        if (k > 0) {  // for k = 0 the buffer still holds G_0 T_1^T from the norms
            GemmBatch b0;
            b0.nb1 = nc; b0.sA1 = X.cstride(k); b0.sB1 = (long long)n * n; b0.sC1 = (long long)m * n;
            gemm_f64(s, false, true, m, n, n, 1.0, X.core[k], n, T[k + 1], n, 0.0, C, n, b0);
        }
        double *sig, *V;
        int *rk;
        int r = svd_ranks(c, m, n, C, (long long)m * n, n, 1, ddelta, 0.0, c->o.rank_cap, &sig, &V, &rk);
        std::memcpy(c->bond[k].sig, c->last_sig, sizeof(c->last_sig));
        double *W1 = c->sc.get<double>(S_W1, (size_t)nc * n * r);
        double *W2 = c->sc.get<double>(S_W2, (size_t)nc * n * r);
        build_projectors(s, n, nc, r, sig, V, rk, W1, W2);
        // P = T_{k+1}^T W1 (n x r)
        double *P = c->sc.get<double>(S_P, (size_t)nc * n * r);
        GemmBatch b1;
        b1.nb1 = nc; b1.sA1 = (long long)n * n; b1.sB1 = (long long)n * r; b1.sC1 = (long long)n * r;
        gemm_f64(s, true, false, n, r, n, 1.0, T[k + 1], n, W1, r, 0.0, P, r, b1);
        // new core k = G'_k P (m x r)
        double *nk = dalloc<double>(s, (size_t)nc * m * r);
        GemmBatch b2;
        b2.nb1 = nc; b2.sA1 = X.cstride(k); b2.sB1 = (long long)n * r; b2.sC1 = (long long)m * r;
        gemm_f64(s, false, false, m, r, n, 1.0, X.core[k], n, P, r, 0.0, nk, r, b2);
        // Columns of G'_k P belonging to small kept singular values carry rounding noise along
        // the dominant directions (relative size u ||G'_k|| ||T|| / sigma_j); re-orthonormalise
        // them in descending sigma order (two CholeskyQR passes) before projecting.
        {  // two passes ping-pong between nk and a scratch copy, ending in nk
            double *nk2 = c->sc.get<double>(S_TD1, (size_t)nc * m * r);
            for (int pass = 0; pass < 2; ++pass) {
                double *src = pass == 0 ? nk : nk2, *dst = pass == 0 ? nk2 : nk;
                double *Xi = c->sc.get<double>(S_PD1, (size_t)nc * r * r);
                if (!gram_chol_inv(s, m, r, nc, src, (long long)m * r, Xi)) {
                    double *Gm = c->sc.get<double>(S_PD0, (size_t)nc * r * r);
                    double *ws = c->sc.get<double>(S_TD0, (size_t)nc * r * r);
                    size_t pc = gemm_tn_splitk_part(r, r, m, nc);
                    gemm_tn_splitk(s, r, r, m, src, r, src, r, Gm, r, nc, (long long)m * r, (long long)m * r,
                                   (long long)r * r, c->sc.get<double>(S_SPLIT, pc), pc);
                    chol_upper_inv(s, r, nc, Gm, Xi, ws);
                }
                GemmBatch bx;
                bx.nb1 = nc; bx.sA1 = (long long)m * r; bx.sB1 = (long long)r * r; bx.sC1 = (long long)m * r;
                gemm_f64(s, false, false, m, r, r, 1.0, src, r, Xi, r, 0.0, dst, r, bx);
            }
        }
        // S = new^T G'_k (r x n); next core = S G_{k+1}
        double *Sm = c->sc.get<double>(S_Q, (size_t)nc * r * n);
        {
            size_t pc = gemm_tn_splitk_part(r, n, m, nc);
            gemm_tn_splitk(s, r, n, m, nk, r, X.core[k], n, Sm, n, nc, (long long)m * r, X.cstride(k), (long long)r * n,
                           c->sc.get<double>(S_SPLIT, pc), pc);
        }
        const int mn = X.N[k + 1] * X.R[k + 2];
        double *nk1 = dalloc<double>(s, (size_t)nc * r * mn);
        GemmBatch b4;
        b4.nb1 = nc; b4.sA1 = (long long)r * n; b4.sB1 = X.cstride(k + 1); b4.sC1 = (long long)r * mn;
        gemm_f64(s, false, false, r, mn, n, 1.0, Sm, n, X.core[k + 1], mn, 0.0, nk1, mn, b4);
        dfree(s, X.core[k]);
        dfree(s, X.core[k + 1]);
        X.core[k] = nk;
        X.core[k + 1] = nk1;
        X.R[k + 1] = r;
    }
    for (int k = 1; k < d; ++k) dfree(s, T[k]);
    // the truncation ranks were read after the norms were copied
    if (want_norms) norms.assign(c->h_pinned_dbl + kPinNorms, c->h_pinned_dbl + kPinNorms + nc);
}

// ===================================================================== batched stepping
// Many independent states advance in lock-step through the phases of a stage: every state's
// block evaluations are enqueued, then one batched pivot launch (one workgroup per state) and
// one host synchronisation serve the whole batch; likewise the sampled residuals, the norms,
// the Jacobi SVDs and the truncation ranks of the rounding. Per-state kernels (gathers, stage
// kernel, GEMMs, TSQR) are enqueued back to back on the shared stream.
struct BState {
    wenott_ctx *c = nullptr;
    TT X;
    bool x_owned = false;
    double alpha = 0.0, eps = 0.0, ceps = 0.0, dt = 0.0;
    int M[kMaxDim] = {};
    std::vector<ISet> Rset, Lset;
    FluxTT F;
    Rng rng{0};
    double rel2 = 0.0, resid = 1e300;
    int sweep = 0;
    bool active = true, cold = false;
    int kick = 0;            // enrichment of this sweep's index sets
    bool saturated = false;  // a pivot search of this sweep used every column of its block
    // per-core pivots of the batched pivot phase
    double *B = nullptr, *L = nullptr;
    int *piv = nullptr;
    double *info = nullptr;
    int m = 0, n = 0, rmax = 0;
    std::vector<double> norms;
    int nb_acc = 0;
};

// One batched pivot phase over the given states: prrLU of each state's block. The register
// jobs finish in the first launch; the multi-workgroup jobs run in chunks of pivot steps, each
// chunk followed by one synchronisation, until every job has stopped.
// A job whose single-launch (persistent) form gave up waiting for workgroups that were not all
// resident left its block partly eliminated: reeval(b) writes the block again and the job is redone
// in the one-launch-per-step layout.
void batch_pivots(std::vector<BState *> &act, int dir, int k, const std::function<void(BState *)> &reeval) {
    if (act.empty()) return;
    wenott_ctx *c0 = act[0]->c;
    std::vector<PrrluJob> jobs;
    int t_end = 0;
    for (BState *b : act) {
        wenott_ctx *c = b->c;
        b->rmax = std::min(std::min(c->o.rank_cap, kMaxRankLds), std::min(b->m, b->n));
        b->piv = pivot_buffer(c, b->rmax, &b->info);
        b->L = c->sc.get<double>(S_L, (size_t)b->m * b->rmax);
        PrrluJob j{};
        j.A = b->B; j.m = b->m; j.n = b->n; j.rmax = b->rmax; j.rel_tol2 = b->rel2;
        j.rowpiv = b->piv; j.colpiv = b->piv + b->rmax; j.L = b->L; j.info = b->info;
        j.ws = c->sc.get<double>(S_ROWBUF, prrlu_ws_doubles(b->m, b->n));
        prrlu_prepare(j);
        if (j.mode >= 1) t_end = std::max(t_end, pivot_guess(c, hist_index(kMaxDim, dir, k), b->n, b->rmax) + 1);
        jobs.push_back(j);
    }
    int t_begin = 0;
    std::vector<size_t> open(act.size()), redo;
    for (size_t z = 0; z < act.size(); ++z) open[z] = z;
    for (;;) {
        std::vector<PrrluJob> hj;
        for (size_t z : open) hj.push_back(jobs[z]);
        const PrrluJob *dj = c0->ring.put(hj.data(), hj.size());
        ev_record(c0, KC_PIVOT);
        prrlu_batch(c0->s, (int)hj.size(), hj.data(), dj, t_begin, t_end);
        ev_record(c0, KC_PIVOT);
        for (size_t z : open) {
            BState *b = act[z];
            WTT_HIP(hipMemcpyAsync(b->c->h_pinned_int, b->piv, pivot_info_offset(b->rmax) + 3 * sizeof(double),
                                   hipMemcpyDeviceToHost, b->c->s));
        }
        host_wait(c0);
        std::vector<size_t> still;
        int rmax_open = 0;
        for (size_t z : open) {
            const double state = pinned_pivot_info(act[z]->c, act[z]->rmax, 0);
            if (state == -2.0) {
                WTT_REQUIRE(jobs[z].mode == 2, WENOTT_EHIP, "pivot search: the stepped form reported a persistent failure");
                redo.push_back(z);
            } else if (state < 0.0) {
                still.push_back(z);
                rmax_open = std::max(rmax_open, act[z]->rmax);
            }
        }
        if (still.empty() && !redo.empty()) {
            // the jobs whose persistent launch gave up: one launch per step, from a freshly evaluated block
            for (size_t z : redo) {
                reeval(act[z]);
                jobs[z].mode = 1;
                act[z]->c->info.pivot_fallbacks += 1;
            }
            open = std::move(redo);
            redo.clear();
            t_begin = 0;
            t_end = 0;
            for (size_t z : open)
                t_end = std::max(t_end, pivot_guess(act[z]->c, hist_index(kMaxDim, dir, k), act[z]->n, act[z]->rmax) + 1);
            continue;
        }
        if (still.empty()) break;
        t_begin = t_end + 1;
        WTT_REQUIRE(t_begin <= rmax_open + 1, WENOTT_EHIP, "pivot search did not stop");
        t_end = std::min(rmax_open + 1, t_begin + std::max(8, t_begin / 2));
        open = std::move(still);
    }
    for (BState *b : act) {
        const int r = (int)pinned_pivot_info(b->c, b->rmax, 0);
        b->c->piv_hist[hist_index(kMaxDim, dir, k)] = r;
        double fl = 0.0;
        for (int t = 0; t < r; ++t) fl += 2.0 * (double)(b->m - t) * (double)(b->n - t);
        add_work(b->c, KC_PIVOT, fl, 8.0 * ((double)b->m * b->n + (double)b->m * r));
        b->c->info.pivots_total += r;
    }
}

void batch_cross(std::vector<BState> &bs, const double *aw, const double *bw, int st) {
    const int d = bs[0].X.d, nc = bs[0].X.nc;
    for (auto &b : bs) {
        wenott_ctx *c = b.c;
        for (int j = 0; j < d; ++j) b.M[j] = b.X.N[j];
        b.rng = Rng(c->o.seed ^ (0x5851F42D4C957F2DULL * (++c->counter)));
        b.Rset.assign(d, ISet());
        b.Rset[d - 1].len = 0;
        b.Rset[d - 1].count = 1;
        b.cold = !c->warm_valid[kMaxDim];  // as in the single-state cross: a cold start takes the refresh sweep
        if (!b.cold) b.Rset = c->warm[kMaxDim];
        else
            for (int k = 0; k < d - 1; ++k) b.Rset[k] = random_set(b.rng, std::max(2, b.X.maxrank()), k + 1, d - 1 - k, b.M);
        b.Lset.assign(d, ISet());
        b.F = FluxTT();
        b.F.d = d; b.F.nc = nc;
        for (int j = 0; j < d; ++j) b.F.M[j] = b.M[j];
        // the FP32 fiber path floors the cross tolerance as in the single-state cross
        b.ceps = (c->o.precision == 1 ? std::max(b.eps, 1e-6) : b.eps) * c->o.cross_ratio;
        b.rel2 = b.ceps * b.ceps / (4.0 * d);
        b.resid = 1e300;
        b.sweep = 0;
        b.active = true;
        b.kick = c->o.kick_rank;
        b.saturated = false;
    }
    const int max_sweeps = bs[0].c->o.max_sweeps;
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        std::vector<BState *> act;
        for (auto &b : bs)
            if (b.active) act.push_back(&b);
        if (act.empty()) break;
        for (BState *b : act) {
            b->saturated = false;
            b->F.release(b->c->s);
            b->Lset[0].len = 0; b->Lset[0].count = 1; b->Lset[0].v.clear();
            b->F.R[0] = 1; b->F.R[d] = 1;
        }
        std::vector<ISet> Rk(bs.size());
        for (int k = 0; k < d; ++k) {
            for (BState *b : act) {
                const size_t z = b - bs.data();
                Rk[z] = k < d - 1 ? with_kick(b->Rset[k], b->rng, b->kick, k + 1, b->M) : b->Rset[k];
                const int p = b->Lset[k].count, q = Rk[z].count;
                b->m = p * b->M[k];
                b->n = q * nc;
                const StageWeights w{aw[st], bw[st], bw[st] * b->dt};
                if (k < d - 1) {
                    b->B = b->c->sc.get<double>(S_BLOCK, (size_t)b->m * b->n);
                    eval_stage_block(b->c, b->X, &b->c->U, w, b->alpha, k, b->Lset[k], Rk[z], true, b->B);
                } else {
                    b->F.core[k] = dalloc<double>(b->c->s, (size_t)b->m * b->n);
                    eval_stage_block(b->c, b->X, &b->c->U, w, b->alpha, k, b->Lset[k], Rk[z], true, b->F.core[k]);
                }
            }
            if (k == d - 1) break;
            batch_pivots(act, 0, k, [&](BState *b) {
                const size_t z = b - bs.data();
                const StageWeights w{aw[st], bw[st], bw[st] * b->dt};
                eval_stage_block(b->c, b->X, &b->c->U, w, b->alpha, k, b->Lset[k], Rk[z], true, b->B);
            });
            for (BState *b : act) {
                const int r = (int)pinned_pivot_info(b->c, b->rmax, 0);
                b->saturated = b->saturated || (r >= b->n && b->n < b->m);
                std::vector<int> rows(b->c->h_pinned_int, b->c->h_pinned_int + r);
                b->F.core[k] = dalloc<double>(b->c->s, (size_t)b->m * r);
                interp_solve(b->c->s, b->m, r, b->L, b->rmax, b->piv, b->F.core[k]);
                b->F.R[k + 1] = r;
                ISet nl;
                nl.len = k + 1;
                nl.count = r;
                nl.v.resize((size_t)r * (k + 1));
                for (int tt = 0; tt < r; ++tt) {
                    const int row = rows[tt], a = row / b->M[k], i = row % b->M[k];
                    for (int j = 0; j < k; ++j) nl.v[(size_t)tt * (k + 1) + j] = b->Lset[k].v[(size_t)a * k + j];
                    nl.v[(size_t)tt * (k + 1) + k] = i;
                }
                b->Lset[k + 1] = std::move(nl);
            }
        }
        // sampled residuals of every active state, one synchronisation
        for (BState *b : act) {
            const StageWeights w{aw[st], bw[st], bw[st] * b->dt};
            b->nb_acc = sampled_stage_residual_launch(b->c, b->X, &b->c->U, w, b->alpha, b->F, b->rng);
        }
        host_wait(act[0]->c);
        std::vector<BState *> refresh;
        for (BState *b : act) {
            b->resid = sampled_residual_finish(b->c, b->nb_acc);
            b->sweep = sweep + 1;
            if ((b->resid <= b->ceps && !(b->cold && sweep == 0)) || sweep + 1 == max_sweeps) b->active = false;
            else refresh.push_back(b);
        }
        // right-to-left refresh of the states that missed eps
        for (int k = d - 1; k >= 1 && !refresh.empty(); --k) {
            std::vector<ISet> Lk(bs.size());
            for (BState *b : refresh) {
                const size_t z = b - bs.data();
                Lk[z] = with_kick(b->Lset[k], b->rng, b->kick, 0, b->M);
                const ISet &R = b->Rset[k];
                b->m = b->M[k] * R.count;
                b->n = Lk[z].count * nc;
                b->B = b->c->sc.get<double>(S_BLOCK, (size_t)b->m * b->n);
                const StageWeights w{aw[st], bw[st], bw[st] * b->dt};
                eval_stage_block(b->c, b->X, &b->c->U, w, b->alpha, k, Lk[z], R, false, b->B);
            }
            batch_pivots(refresh, 1, k, [&](BState *b) {
                const size_t z = b - bs.data();
                const StageWeights w{aw[st], bw[st], bw[st] * b->dt};
                eval_stage_block(b->c, b->X, &b->c->U, w, b->alpha, k, Lk[z], b->Rset[k], false, b->B);
            });
            for (BState *b : refresh) {
                const ISet &R = b->Rset[k];
                const int r = (int)pinned_pivot_info(b->c, b->rmax, 0), q = R.count;
                b->saturated = b->saturated || (r >= b->n && b->n < b->m);
                ISet nr;
                nr.len = d - k;
                nr.count = r;
                nr.v.resize((size_t)r * nr.len);
                for (int tt = 0; tt < r; ++tt) {
                    const int row = b->c->h_pinned_int[tt], i = row / q, bb = row % q;
                    nr.v[(size_t)tt * nr.len] = i;
                    for (int j = 0; j < R.len; ++j) nr.v[(size_t)tt * nr.len + 1 + j] = R.v[(size_t)bb * R.len + j];
                }
                b->Rset[k - 1] = std::move(nr);
            }
        }
        for (BState *b : refresh) {
            b->rel2 *= 0.25;
            if (b->saturated) b->kick = std::min(2 * std::max(b->kick, 2), 128);  // as in the single-state cross
        }
    }
    for (auto &b : bs) {
        b.c->warm[kMaxDim] = b.Rset;
        b.c->warm_valid[kMaxDim] = true;
        b.c->info.sweeps[st][0] = b.sweep;
        b.c->info.residual[st][0] = b.resid;
        int fr = 1;
        for (int k = 1; k < d; ++k) fr = std::max(fr, b.F.R[k]);
        b.c->info.flux_rank[st][0] = fr;
        if (!(b.resid <= b.c->o.conv_slack * b.ceps) && !(b.resid <= 1e-12))
            throw StatusError(WENOTT_ENOCONV, "cross did not converge within max_sweeps sweeps");
    }
}

// Lock-step TT-rounding of every state's stage TT (same algorithm as round_tt).
void batch_round(std::vector<BState> &bs, std::vector<TT> &Xs) {
    const int d = Xs[0].d, nc = Xs[0].nc;
    const size_t ns = bs.size();
    std::vector<std::vector<double *>> T(ns, std::vector<double *>(d + 1, nullptr));
    for (size_t z = 0; z < ns; ++z) {
        wenott_ctx *c = bs[z].c;
        TT &X = Xs[z];
        for (int k = d - 1; k >= 1; --k) {
            const int Rk = X.R[k], Nk = X.N[k], Rk1 = X.R[k + 1];
            const long long m = (long long)Nk * Rk1;
            const double *C = X.core[k];
            if (k < d - 1) {
                double *Cb = c->sc.get<double>(S_TMP, (size_t)nc * Rk * m);
                GemmBatch b;
                b.nb1 = nc; b.sA1 = X.cstride(k); b.sB1 = (long long)Rk1 * Rk1; b.sC1 = (long long)Rk * m;
                gemm_f64(c->s, false, true, Rk * Nk, Rk1, Rk1, 1.0, X.core[k], Rk1, T[z][k + 1], Rk1, 0.0, Cb, Rk1, b);
                C = Cb;
            }
            double *scr = c->sc.get<double>(S_TSQR, tsqr_scratch_doubles((int)m, Rk, nc));
            T[z][k] = dalloc<double>(c->s, (size_t)nc * Rk * Rk);
            ev_record(c, KC_TSQR);
            tsqr_r(c->s, (int)m, Rk, nc, C, (long long)Rk * m, 1, m, T[z][k], scr);
            ev_record(c, KC_TSQR);
            add_work(c, KC_TSQR, nc * (2.0 * m * (double)Rk * Rk - 2.0 / 3.0 * (double)Rk * Rk * Rk),
                     8.0 * nc * (double)m * Rk);

        }
        const int N0 = X.N[0], R1 = X.R[1];
        double *C0 = c->sc.get<double>(S_TMP, (size_t)nc * N0 * R1);
        GemmBatch b;
        b.nb1 = nc; b.sA1 = X.cstride(0); b.sB1 = (long long)R1 * R1; b.sC1 = (long long)N0 * R1;
        gemm_f64(c->s, false, true, N0, R1, R1, 1.0, X.core[0], R1, T[z][1], R1, 0.0, C0, R1, b);
        double *dn = c->sc.get<double>(S_NORMS, nc);
        frob_norms(c->s, nc, (long long)N0 * R1, C0, (long long)N0 * R1, dn);
        WTT_HIP(hipMemcpyAsync(c->h_pinned_dbl + 64, dn, nc * sizeof(double), hipMemcpyDeviceToHost, c->s));
    }
    host_wait(bs[0].c);
    std::vector<const double *> ddelta(ns);
    for (size_t z = 0; z < ns; ++z) {
        wenott_ctx *c = bs[z].c;
        bs[z].norms.assign(c->h_pinned_dbl + 64, c->h_pinned_dbl + 64 + nc);
        std::vector<double> delta(nc);
        for (int q = 0; q < nc; ++q) delta[q] = bs[z].eps * bs[z].norms[q] / std::sqrt((double)std::max(d - 1, 1));
        ddelta[z] = c->ring.put(delta.data(), delta.size());
    }
    for (int k = 0; k < d - 1; ++k) {
        std::vector<SvdJob> jobs(ns);
        std::vector<double *> sig(ns), V(ns);
        std::vector<int *> rk(ns);
        int nmax = 1;
        for (size_t z = 0; z < ns; ++z) nmax = std::max(nmax, Xs[z].R[k + 1]);
        const bool fits = jacobi_batch_fits(nmax);
        for (size_t z = 0; z < ns; ++z) {
            wenott_ctx *c = bs[z].c;
            TT &X = Xs[z];
            const int m = X.R[k] * X.N[k], n = X.R[k + 1];
            double *C = c->sc.get<double>(S_TMP, (size_t)nc * m * n);
            if (k > 0) {  // for k = 0 the buffer still holds G_0 T_1^T from the norms
                GemmBatch b0;
                b0.nb1 = nc; b0.sA1 = X.cstride(k); b0.sB1 = (long long)n * n; b0.sC1 = (long long)m * n;
                gemm_f64(c->s, false, true, m, n, n, 1.0, X.core[k], n, T[z][k + 1], n, 0.0, C, n, b0);
            }
            double *scr = c->sc.get<double>(S_TSQR, tsqr_scratch_doubles(m, n, nc));
            double *R = c->sc.get<double>(S_R, (size_t)nc * n * n);
            ev_record(c, KC_TSQR);
            tsqr_r(c->s, m, n, nc, C, (long long)m * n, n, 1, R, scr);
            ev_record(c, KC_TSQR);
            add_work(c, KC_TSQR, nc * (2.0 * m * (double)n * n - 2.0 / 3.0 * (double)n * n * n), 8.0 * nc * (double)m * n);
            add_work(c, KC_SVD, 0.0, 8.0 * nc * 3.0 * (double)n * n);
            sig[z] = c->sc.get<double>(S_SIG, (size_t)nc * n);
            V[z] = c->sc.get<double>(S_V, (size_t)nc * n * n);
            jobs[z] = SvdJob{R, sig[z], V[z], n, nc, ddelta[z]};
            if (!fits) {
                double *jac = c->sc.get<double>(S_JAC, jacobi_scratch_doubles(n, nc));
                ev_record(c, KC_SVD);
                jacobi_svd(c->s, n, nc, R, sig[z], V[z], jac, ddelta[z]);
                ev_record(c, KC_SVD);
            }
        }
        if (fits) {
            SvdJob *dj = bs[0].c->ring.put(jobs.data(), jobs.size());
            ev_record(bs[0].c, KC_SVD);
            jacobi_svd_batch(bs[0].c->s, (int)ns, nc, nmax, dj);
            ev_record(bs[0].c, KC_SVD);
        }
        for (size_t z = 0; z < ns; ++z) {
            wenott_ctx *c = bs[z].c;
            const int n = Xs[z].R[k + 1];
            rk[z] = c->sc.get<int>(S_RANKS, nc);
            trunc_ranks(c->s, n, nc, sig[z], ddelta[z], 0.0, c->o.rank_cap, rk[z]);
            WTT_HIP(hipMemcpyAsync(c->h_pinned_int, rk[z], nc * sizeof(int), hipMemcpyDeviceToHost, c->s));
        }
        host_wait(bs[0].c);
        std::vector<CholJob> cj(ns);
        std::vector<double *> nk(ns), nk2(ns);
        std::vector<int> rr(ns);
        for (size_t z = 0; z < ns; ++z) {
            wenott_ctx *c = bs[z].c;
            TT &X = Xs[z];
            const int m = X.R[k] * X.N[k], n = X.R[k + 1];
            int r = 1;
            for (int q = 0; q < nc; ++q) r = std::max(r, c->h_pinned_int[q]);
            rr[z] = r;
            double *W1 = c->sc.get<double>(S_W1, (size_t)nc * n * r);
            double *W2 = c->sc.get<double>(S_W2, (size_t)nc * n * r);
            build_projectors(c->s, n, nc, r, sig[z], V[z], rk[z], W1, W2);
            double *P = c->sc.get<double>(S_P, (size_t)nc * n * r);
            GemmBatch b1;
            b1.nb1 = nc; b1.sA1 = (long long)n * n; b1.sB1 = (long long)n * r; b1.sC1 = (long long)n * r;
            gemm_f64(c->s, true, false, n, r, n, 1.0, T[z][k + 1], n, W1, r, 0.0, P, r, b1);
            nk[z] = dalloc<double>(c->s, (size_t)nc * m * r);
            GemmBatch b2;
            b2.nb1 = nc; b2.sA1 = X.cstride(k); b2.sB1 = (long long)n * r; b2.sC1 = (long long)m * r;
            gemm_f64(c->s, false, false, m, r, n, 1.0, X.core[k], n, P, r, 0.0, nk[z], r, b2);
        }
        for (size_t z = 0; z < ns; ++z)
            nk2[z] = bs[z].c->sc.get<double>(S_TD1, (size_t)nc * Xs[z].R[k] * Xs[z].N[k] * rr[z]);
        for (int pass = 0; pass < 2; ++pass) {  // ping-pong between nk and nk2, ending in nk
            int rmax_sep = 0;  // largest rank of the states that take the separate Gram path
            for (size_t z = 0; z < ns; ++z) {
                wenott_ctx *c = bs[z].c;
                const int m = Xs[z].R[k] * Xs[z].N[k], r = rr[z];
                double *src = pass == 0 ? nk[z] : nk2[z];
                double *Xi = c->sc.get<double>(S_PD1, (size_t)nc * r * r);
                if (gram_chol_inv(c->s, m, r, nc, src, (long long)m * r, Xi)) {  // as the single-state path
                    cj[z] = CholJob{nullptr, Xi, nullptr, r, 0};
                    continue;
                }
                double *Gm = c->sc.get<double>(S_PD0, (size_t)nc * r * r);
                double *ws = c->sc.get<double>(S_TD0, (size_t)nc * r * r);
                size_t pc = gemm_tn_splitk_part(r, r, m, nc);
                gemm_tn_splitk(c->s, r, r, m, src, r, src, r, Gm, r, nc, (long long)m * r, (long long)m * r,
                               (long long)r * r, c->sc.get<double>(S_SPLIT, pc), pc);
                cj[z] = CholJob{Gm, Xi, ws, r, nc};
                rmax_sep = std::max(rmax_sep, r);
            }
            if (rmax_sep > 0) {
                CholJob *dc = bs[0].c->ring.put(cj.data(), cj.size());
                chol_upper_inv_batch(bs[0].c->s, (int)ns, nc, rmax_sep, dc);
            }
            for (size_t z = 0; z < ns; ++z) {
                wenott_ctx *c = bs[z].c;
                const int m = Xs[z].R[k] * Xs[z].N[k], r = rr[z];
                double *src = pass == 0 ? nk[z] : nk2[z], *dst = pass == 0 ? nk2[z] : nk[z];
                GemmBatch bx;
                bx.nb1 = nc; bx.sA1 = (long long)m * r; bx.sB1 = (long long)r * r; bx.sC1 = (long long)m * r;
                gemm_f64(c->s, false, false, m, r, r, 1.0, src, r, cj[z].X, r, 0.0, dst, r, bx);
            }
        }
        for (size_t z = 0; z < ns; ++z) {
            wenott_ctx *c = bs[z].c;
            TT &X = Xs[z];
            const int m = X.R[k] * X.N[k], n = X.R[k + 1], r = rr[z];
            double *Sm = c->sc.get<double>(S_Q, (size_t)nc * r * n);
            size_t pc = gemm_tn_splitk_part(r, n, m, nc);
            gemm_tn_splitk(c->s, r, n, m, nk[z], r, X.core[k], n, Sm, n, nc, (long long)m * r, X.cstride(k),
                           (long long)r * n, c->sc.get<double>(S_SPLIT, pc), pc);
            const int mn = X.N[k + 1] * X.R[k + 2];
            double *nk1 = dalloc<double>(c->s, (size_t)nc * r * mn);
            GemmBatch b4;
            b4.nb1 = nc; b4.sA1 = (long long)r * n; b4.sB1 = X.cstride(k + 1); b4.sC1 = (long long)r * mn;
            gemm_f64(c->s, false, false, r, mn, n, 1.0, Sm, n, X.core[k + 1], mn, 0.0, nk1, mn, b4);
            dfree(c->s, X.core[k]);
            dfree(c->s, X.core[k + 1]);
            X.core[k] = nk[z];
            X.core[k + 1] = nk1;
            X.R[k + 1] = r;
        }
    }
    for (size_t z = 0; z < ns; ++z)
        for (int k = 1; k < d; ++k) dfree(bs[z].c->s, T[z][k]);
}

double geometric_h(const wenott_ctx *c) {
    double p = 1.0;
    for (int k = 0; k < c->d; ++k) p *= c->h[k];
    return std::pow(p, 1.0 / c->d);
}
double volume(const wenott_ctx *c) {
    double v = 1.0;
    for (int k = 0; k < c->d; ++k) v *= c->hi[k] - c->lo[k];
    return v;
}
// eq. eps-tt-formula generalised to d dimensions: eps = C_eps V^{1/2} h^{5 - d/2} / max_q ||q||_F
double dynamic_eps(const wenott_ctx *c, double max_norm) {
    return c->c_eps * std::sqrt(volume(c)) * std::pow(geometric_h(c), 5.0 - 0.5 * c->d) / max_norm;
}
double current_eps(const wenott_ctx *c) {
    if (c->o.eps_mode == 0) return c->o.eps0;
    return dynamic_eps(c, c->max_norm);
}

// L(U) as a TT: cross per direction, shift difference, sum over directions.
// One TT of nc components from nc single-component TTs of the same grid: ranks padded to the
// largest, each component's cores in the leading block of its slot.
TT pack_components(wenott_ctx *c, const std::vector<TT> &parts) {
    const TT &a = parts[0];
    TT S;
    S.d = a.d; S.nc = (int)parts.size();
    for (int j = 0; j < a.d; ++j) S.N[j] = a.N[j];
    for (int k = 0; k <= a.d; ++k) {
        S.R[k] = 1;
        for (const TT &X : parts) S.R[k] = std::max(S.R[k], X.R[k]);
    }
    S.alloc(c->s);
    for (int k = 0; k < S.d; ++k) {
        fill(c->s, S.core[k], S.cstride(k) * S.nc, 0.0);
        for (int i = 0; i < S.nc; ++i) {
            const TT &X = parts[i];
            place_block(c->s, 1, X.R[k], S.N[k], X.R[k + 1], X.core[k], X.cstride(k), 1.0,
                        S.core[k] + i * S.cstride(k), S.R[k], S.R[k + 1], S.cstride(k), 0, 0);
        }
    }
    return S;
}

// Scheme 2, per direction (Sec. 4.2-4.3): the LF-cross of the 2 ncomp split fluxes at the cells,
// its slices as single-component TTs (the shared cores and one slice of the last core), then per
// slice one WENO-cross of the one-sided reconstruction on the faces (f^+ slices left-biased, f^-
// slices mirrored), each warm-started from its own previous cross. Returns the two terms
// -(T^d - 1)/h_d F^+ and -(T^d - 1)/h_d F^- (their sum is L_d), each packed over components.
void lf_weno_terms(wenott_ctx *c, const TT &U, int dir, double alpha, double eps, int stage, std::vector<TT> &terms) {
    const int d = U.d, nc = U.nc;
    CrossStat lst;
    FluxTT F = cross_lf(c, U, dir, alpha, eps, lst);
    int sweeps = lst.sweeps, rmax = lst.maxrank;
    double resid = lst.residual;
    const int k = d - 1;
    const long long per = (long long)F.R[k] * F.M[k];
    double *slices = dalloc<double>(c->s, (size_t)per * 2 * nc);
    std::vector<TT> plus, minus;
    auto release_all = [&]() {
        for (auto &t : plus) t.release(c->s);
        for (auto &t : minus) t.release(c->s);
        dfree(c->s, slices);
        F.release(c->s);
    };
    try {
        split_last(c->s, F.R[k], F.M[k], 2 * nc, F.core[k], slices, per);
        for (int j = 0; j < 2 * nc; ++j) {
            TT V;  // a view: the LF-cross's shared cores and slice j of its last core
            V.d = d; V.nc = 1;
            for (int m = 0; m < d; ++m) V.N[m] = F.M[m];
            for (int m = 0; m <= d; ++m) V.R[m] = F.R[m];
            for (int m = 0; m < d - 1; ++m) V.core[m] = F.core[m];
            V.core[k] = slices + j * per;
            CrossStat wst;
            FluxTT Wf = cross_flux(c, V, dir, j < nc ? 1.0 : -1.0, eps, wst, kSlotWeno + dir * kMaxSlices + j,
                                   kLawLinAdv);
            sweeps = std::max(sweeps, wst.sweeps);
            rmax = std::max(rmax, wst.maxrank);
            resid = std::max(resid, wst.residual);
            (j < nc ? plus : minus).push_back(cross_to_tt(c, Wf, dir));
            Wf.release(c->s);
        }
        terms.push_back(pack_components(c, plus));
        terms.push_back(pack_components(c, minus));
    } catch (...) {
        release_all();
        throw;
    }
    release_all();
    if (stage >= 0 && stage < 3) {
        c->info.sweeps[stage][dir] = sweeps;
        c->info.residual[stage][dir] = resid;
        c->info.flux_rank[stage][dir] = rmax;
    }
}

std::vector<TT> rhs_terms(wenott_ctx *c, const TT &U, double alpha, double eps, int stage) {
    std::vector<TT> terms;
    if (c->o.scheme == 2) {
        try {
            for (int dir = 0; dir < U.d; ++dir) lf_weno_terms(c, U, dir, alpha, eps, stage, terms);
        } catch (...) {
            for (auto &t : terms) t.release(c->s);
            throw;
        }
        return terms;
    }
    for (int dir = 0; dir < U.d; ++dir) {
        CrossStat st;
        FluxTT F = cross_flux(c, U, dir, alpha, eps, st);
        if (stage >= 0 && stage < 3) {
            c->info.sweeps[stage][dir] = st.sweeps;
            c->info.residual[stage][dir] = st.residual;
            c->info.flux_rank[stage][dir] = st.maxrank;
        }
        terms.push_back(cross_to_tt(c, F, dir));
        F.release(c->s);
    }
    return terms;
}

void reset_call_info(wenott_ctx *c) {
    c->info.proposals_tried = 0;
    c->info.proposals_accepted = 0;
    c->info.pivots_total = 0;
    c->info.rank_capped = 0;
    c->info.pivot_fallbacks = 0;
    c->info.fiber_points = 0;
    c->info.fiber_launches = 0;
    c->info.fiber_ms = 0.0;
    for (int i = 0; i < 4; ++i) {
        c->info.class_ms[i] = 0.0;
        c->info.class_flops[i] = 0.0;
        c->info.class_bytes[i] = 0.0;
        c->info.class_launches[i] = 0;
    }
    c->ev_used = 0;
}

void finish_call_info(wenott_ctx *c, double t0) {
    if (c->profiling && c->ev_used >= 2) {
        host_wait(c);
        for (int i = 0; i + 1 < c->ev_used; i += 2) {
            float e = 0.f;
            WTT_HIP(hipEventElapsedTime(&e, c->ev[i], c->ev[i + 1]));
            c->info.class_ms[c->ev_class[i]] += e;
        }
        c->info.fiber_ms = c->info.class_ms[KC_FIBER];
    }
    c->info.step_ms = (seconds_now() - t0) * 1e3;
}

wenott_status run_guarded(wenott_ctx *c, const std::function<void()> &f);

}  // namespace

// ================================================================== C ABI

namespace {
thread_local std::string g_last_error;

void note_error(wenott_ctx *c, const char *what) {
    g_last_error = what;
    if (c) c->last_error = what;
}

wenott_status run_guarded(wenott_ctx *c, const std::function<void()> &f) {
    try {
        f();
        return WENOTT_OK;
    } catch (const StatusError &e) {
        note_error(c, e.what());
        return e.status;
    } catch (const HipError &e) {
        note_error(c, e.what());
        return e.code == hipErrorOutOfMemory ? WENOTT_ENOMEM : WENOTT_EHIP;
    } catch (const std::bad_alloc &) {
        note_error(c, "host allocation failed");
        return WENOTT_ENOMEM;
    } catch (const std::exception &e) {
        note_error(c, e.what());
        return WENOTT_EINVAL;
    }
}
}  // namespace

extern "C" {

void wenott_default_opts(wenott_opts *o) {
    std::memset(o, 0, sizeof(*o));
    o->c_eps = 0.0;
    o->eps0 = 1e-10;
    o->eps_mode = 0;
    o->precision = 0;
    o->max_sweeps = 4;
    o->kick_rank = 4;
    o->rank_cap = 256;
    o->probe_points = 4096;
    o->seed = 12345;
    o->alpha_mode = 1;
    o->use_proposal = 0;
    o->alpha_given = 0.0;
    o->rounds_per_stage = 1;
    o->graph_mode = 0;
    o->scheme = 0;
    o->conv_slack = 1.0;
    o->law = WENOTT_LAW_EULER;
    o->cross_ratio = 1.0;
}

const char *wenott_strerror(wenott_status s) {
    switch (s) {
    case WENOTT_OK: return "ok";
    case WENOTT_EINVAL: return "invalid argument";
    case WENOTT_ENOMEM: return "out of memory";
    case WENOTT_EHIP: return "HIP runtime error";
    case WENOTT_ENOCONV: return "cross did not converge";
    case WENOTT_ENONPHYS: return "non-physical state (rho <= 0 or p <= 0)";
    case WENOTT_ENAN: return "NaN or Inf";
    case WENOTT_ENOTBUILT: return "not available in this library";
    }
    return "unknown status";
}

wenott_status wenott_init(wenott_ctx **out, const wenott_tt *state, const wenott_grid *grid, double gamma,
                          const int32_t *bc, const wenott_opts *opts, void *hip_stream) {
    if (!out || !state || !grid || !bc) return WENOTT_EINVAL;
    *out = nullptr;
    wenott_ctx *c = new (std::nothrow) wenott_ctx();
    if (!c) return WENOTT_ENOMEM;
    wenott_status st = run_guarded(c, [&] {
        const int d = grid->ndim;
        WTT_REQUIRE(d == 2 || d == 3, WENOTT_EINVAL, "ndim must be 2 or 3");
        if (opts) c->o = *opts; else wenott_default_opts(&c->o);
        const int law = c->o.law;
        WTT_REQUIRE(law == WENOTT_LAW_EULER || law == WENOTT_LAW_LINADV || law == WENOTT_LAW_BURGERS, WENOTT_EINVAL,
                    "unknown conservation law");
        const int nc = law == WENOTT_LAW_EULER ? d + 2 : 1;
        WTT_REQUIRE(state->ndim == d && state->ncomp == nc, WENOTT_EINVAL,
                    "state must hold ndim + 2 TTs (Euler) or one TT (scalar law)");
        WTT_REQUIRE(state->dtype == 0, WENOTT_EINVAL, "only FP64 cores are accepted");
        WTT_REQUIRE(state->ranks && state->cores, WENOTT_EINVAL, "null ranks or cores");
        WTT_REQUIRE(law != WENOTT_LAW_EULER || gamma > 1.0, WENOTT_EINVAL, "gamma must exceed 1");
        WTT_REQUIRE(law == WENOTT_LAW_EULER || c->o.use_proposal == 0, WENOTT_EINVAL,
                    "the scalar laws run without the proposal");
        c->d = d;
        c->law = law;
        c->nc = nc;
        c->gamma = gamma;
        std::fill(std::begin(c->piv_hist), std::end(c->piv_hist), -1);
        WTT_REQUIRE(c->o.graph_mode == 0, WENOTT_ENOTBUILT, "option not available");
        WTT_REQUIRE(c->o.use_proposal == 0 || c->o.use_proposal == 1, WENOTT_EINVAL, "use_proposal must be 0 or 1");
        WTT_REQUIRE(c->o.precision == 0 || c->o.precision == 1, WENOTT_EINVAL, "precision must be 0 or 1");
        WTT_REQUIRE(c->o.max_sweeps >= 1 && c->o.rank_cap >= 1 && c->o.kick_rank >= 0, WENOTT_EINVAL, "bad options");
        WTT_REQUIRE(c->o.eps_mode == 0 || c->o.eps_mode == 1, WENOTT_EINVAL, "eps_mode must be 0 or 1");
        WTT_REQUIRE(c->o.alpha_mode >= 0 && c->o.alpha_mode <= 2, WENOTT_EINVAL, "alpha_mode must be 0, 1 or 2");
        WTT_REQUIRE(c->o.scheme >= 0 && c->o.scheme <= 2, WENOTT_EINVAL, "scheme must be 0, 1 or 2");
        WTT_REQUIRE(c->o.scheme != 2 || c->o.use_proposal == 0, WENOTT_EINVAL, "the proposal serves the stage cross");
        WTT_REQUIRE(c->o.precision == 0 || c->o.scheme == 0, WENOTT_EINVAL, "the FP32 path runs in scheme 0");
        WTT_REQUIRE(c->o.rounds_per_stage == 1 || c->o.rounds_per_stage == 2, WENOTT_EINVAL,
                    "rounds_per_stage must be 1 or 2");
        WTT_REQUIRE(c->o.conv_slack >= 1.0, WENOTT_EINVAL, "conv_slack must be >= 1");
        WTT_REQUIRE(c->o.cross_ratio > 0.0 && c->o.cross_ratio <= 1.0, WENOTT_EINVAL, "cross_ratio must be in (0, 1]");
        WTT_REQUIRE(c->o.probe_points >= 16 && c->o.probe_points <= 65536, WENOTT_EINVAL,
                    "probe_points must be in [16, 65536]");
        for (int k = 0; k < d; ++k) {
            WTT_REQUIRE(grid->n[k] >= 3 && grid->n[k] <= (1 << 20), WENOTT_EINVAL, "grid size out of range");
            WTT_REQUIRE(grid->hi[k] > grid->lo[k], WENOTT_EINVAL, "empty box");
            for (int side = 0; side < 2; ++side)
                WTT_REQUIRE(bc[2 * k + side] >= WENOTT_BC_PERIODIC && bc[2 * k + side] <= WENOTT_BC_INFLOW,
                            WENOTT_EINVAL, "unknown boundary type");
            WTT_REQUIRE((bc[2 * k] == WENOTT_BC_PERIODIC) == (bc[2 * k + 1] == WENOTT_BC_PERIODIC), WENOTT_EINVAL,
                        "a periodic side needs a periodic opposite side");
            // scheme 2 reconstructs the split fluxes' slices, whose ghost values are index maps of
            // their own only for periodic and transmissive sides
            for (int side = 0; side < 2; ++side)
                WTT_REQUIRE(c->o.scheme != 2 || bc[2 * k + side] <= WENOTT_BC_TRANSMISSIVE, WENOTT_EINVAL,
                            "scheme 2 takes periodic and transmissive sides");
            c->N[k] = (int)grid->n[k];
            c->lo[k] = grid->lo[k];
            c->hi[k] = grid->hi[k];
            c->h[k] = (grid->hi[k] - grid->lo[k]) / grid->n[k];
            c->bc[k] = bc_code(bc[2 * k], bc[2 * k + 1]);
        }
        c->s = (hipStream_t)hip_stream;
        {
            int dev = 0;
            WTT_HIP(hipGetDevice(&dev));
            c->noalloc_ws = noalloc_scratch_of(dev);
        }
        c->sc.s = c->s;
        WTT_HIP(hipEventCreateWithFlags(&c->ev_wait, hipEventDisableTiming));
        c->ring.init(c->s, 8u << 20);
        WTT_HIP(hipMalloc((void **)&c->d_status, sizeof(double) * kStatusDoubles));
        WTT_HIP(hipMemsetAsync(c->d_status, 0, sizeof(double) * kStatusDoubles, c->s));
        c->d_flags = (int *)c->d_status;
        WTT_HIP(hipHostMalloc((void **)&c->h_status, sizeof(double) * kStatusDoubles, hipHostMallocDefault));
        WTT_HIP(hipHostMalloc((void **)&c->h_pinned_int, 4096 * sizeof(int), hipHostMallocDefault));
        WTT_HIP(hipHostMalloc((void **)&c->h_pinned_dbl, 4096 * sizeof(double), hipHostMallocDefault));
        WTT_HIP(hipMalloc((void **)&c->d_best, sizeof(int) * kMaxDim));
        WTT_HIP(hipMemsetAsync(c->d_best, 0xff, sizeof(int) * kMaxDim, c->s));  // -1: no best cell yet
        // common padded ranks
        TT U;
        U.d = d; U.nc = nc;
        for (int k = 0; k < d; ++k) U.N[k] = c->N[k];
        U.R[0] = U.R[d] = 1;
        for (int k = 1; k < d; ++k) {
            int r = 1;
            for (int q = 0; q < nc; ++q) {
                int64_t v = state->ranks[q * (d + 1) + k];
                WTT_REQUIRE(v >= 1 && v <= 4096, WENOTT_EINVAL, "rank out of range");
                r = std::max<int>(r, (int)v);
            }
            U.R[k] = r;
        }
        for (int q = 0; q < nc; ++q)
            WTT_REQUIRE(state->ranks[q * (d + 1)] == 1 && state->ranks[q * (d + 1) + d] == 1, WENOTT_EINVAL,
                        "boundary ranks must be 1");
        U.alloc(c->s);
        const hipMemcpyKind kind = state->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        for (int k = 0; k < d; ++k) {
            fill(c->s, U.core[k], U.cstride(k) * nc, 0.0);
            for (int q = 0; q < nc; ++q) {
                const double *src = (const double *)state->cores[q * d + k];
                WTT_REQUIRE(src != nullptr, WENOTT_EINVAL, "null core pointer");
                const int ra = (int)state->ranks[q * (d + 1) + k], rb = (int)state->ranks[q * (d + 1) + k + 1];
                // place the (ra, N, rb) core in the padded (R_k, N, R_{k+1}) slot
                WTT_HIP(hipMemcpy2DAsync(U.core[k] + q * U.cstride(k), sizeof(double) * U.R[k + 1], src,
                                         sizeof(double) * rb, sizeof(double) * rb, (size_t)ra * U.N[k], kind, c->s));
            }
        }
        host_wait(c);
        c->U = U;
        // norms for the dynamic eps
        TT tmp = copy_tt(c, c->U);
        std::vector<double> norms;
        round_tt(c, tmp, 0.0, false, norms);
        tmp.release(c->s);
        c->max_norm = *std::max_element(norms.begin(), norms.end());
        if (c->o.eps_mode == 1) {
            if (c->o.eps0 > 0.0) {
                c->c_eps = 1.0;
                c->c_eps = c->o.eps0 / dynamic_eps(c, c->max_norm);
            } else {
                c->c_eps = c->o.c_eps;
            }
            WTT_REQUIRE(c->c_eps > 0.0, WENOTT_EINVAL, "dynamic eps needs eps0 > 0 or c_eps > 0");
        }
        c->info.ndim = d;
        c->info.ncomp = nc;
    });
    if (st != WENOTT_OK) {
        wenott_destroy(c);
        return st;
    }
    *out = c;
    return WENOTT_OK;
}

void wenott_destroy(wenott_ctx *c) {
    if (!c) return;
    {  // teardown: errors are not reportable here, the context goes away regardless
        (void)hipStreamSynchronize(c->s);
        c->U.release(c->s);
        if (c->have_rhs) c->rhs.release(c->s);
        c->sc.release();
        release_stream_cache(c->s);
        (void)hipStreamSynchronize(c->s);
        c->ring.destroy();
        if (c->d_status) (void)hipFree(c->d_status);
        if (c->d_best) (void)hipFree(c->d_best);
        if (c->h_status) (void)hipHostFree(c->h_status);
        if (c->h_pinned_int) (void)hipHostFree(c->h_pinned_int);
        if (c->h_pinned_dbl) (void)hipHostFree(c->h_pinned_dbl);
        for (auto e : c->ev) (void)hipEventDestroy(e);
        if (c->ev_wait) (void)hipEventDestroy(c->ev_wait);
    }
    delete c;
}

static void fill_view(wenott_ctx *c, const TT &X, wenott_tt *view) {
    c->view_ranks.assign((size_t)X.nc * (X.d + 1), 0);
    c->view_ptrs.assign((size_t)X.nc * X.d, nullptr);
    for (int q = 0; q < X.nc; ++q) {
        for (int k = 0; k <= X.d; ++k) c->view_ranks[q * (X.d + 1) + k] = X.R[k];
        for (int k = 0; k < X.d; ++k) c->view_ptrs[q * X.d + k] = X.core[k] + q * X.cstride(k);
    }
    view->ndim = X.d;
    view->ncomp = X.nc;
    view->ranks = c->view_ranks.data();
    view->cores = c->view_ptrs.data();
    view->dtype = 0;
    view->on_device = 1;
}

wenott_status wenott_rhs(wenott_ctx *c, double alpha, wenott_tt *view) {
    if (!c || !view) return WENOTT_EINVAL;
    return run_guarded(c, [&] {
        require_inflow_states(c);
        double t0 = seconds_now();
        reset_call_info(c);
        double a = alpha > 0.0 ? alpha : (c->o.alpha_mode == 2 ? c->o.alpha_given : alpha_now(c, c->U));
        WTT_REQUIRE(a > 0.0, WENOTT_EINVAL, "alpha must be positive");
        c->info.alpha[0] = a;
        double eps = current_eps(c);
        TT S;
        if (c->o.scheme == 0) {
            // one cross of L(U) itself (stage value with weights 0, 0, 1)
            CrossStat st;
            FluxTT F = cross_stage(c, c->U, nullptr, StageWeights{0.0, 0.0, 1.0}, a, eps, st);
            c->info.sweeps[0][0] = st.sweeps;
            c->info.residual[0][0] = st.residual;
            c->info.flux_rank[0][0] = st.maxrank;
            S = cross_to_tt(c, F, -1);
            F.release(c->s);
        } else {
            std::vector<TT> terms = rhs_terms(c, c->U, a, eps, 0);
            std::vector<std::pair<double, const TT *>> w;
            for (auto &t : terms) w.push_back({1.0, &t});
            S = tt_sum(c, w);
            for (auto &t : terms) t.release(c->s);
        }
        std::vector<double> norms;
        round_tt(c, S, eps, true, norms);
        if (c->have_rhs) c->rhs.release(c->s);
        c->rhs = S;
        c->have_rhs = true;
        fill_view(c, c->rhs, view);
        c->info.eps = eps;
        finish_call_info(c, t0);
    });
}

wenott_status wenott_rk3_step(wenott_ctx *c, double dt, double eps_in, const double *alphas) {
    if (!c || !(dt > 0.0)) return WENOTT_EINVAL;
    return run_guarded(c, [&] {
        require_inflow_states(c);
        double t0 = seconds_now();
        reset_call_info(c);
        const double eps = eps_in > 0.0 ? eps_in : current_eps(c);
        // Shu-Osher SSP-RK3 (eq. tt-ssprk3): stage s input X_s, output
        // a_s U^n + b_s (X_s + dt L(X_s)), rounded once.
        const double aw[3] = {0.0, 0.75, 1.0 / 3.0}, bw[3] = {1.0, 0.25, 2.0 / 3.0};
        TT X = c->U;  // stage input (aliases U for stage 0)
        bool x_owned = false;
        std::vector<double> norms;
        try {
            for (int st = 0; st < 3; ++st) {
                double a = 0.0;
                // Deferred alpha: the exact alpha stays on the device for the fiber kernels and is
                // read back after the stage's next synchronisation (the proposal's features and
                // the per-direction scheme need it on the host at once).
                const bool deferred = !alphas && c->o.alpha_mode != 2 && !(st == 0 && c->alpha_cache_valid) &&
                                      c->o.scheme == 0 && !c->o.use_proposal && !c->logging;
                if (alphas) a = alphas[st];
                else if (c->o.alpha_mode == 2) a = c->o.alpha_given;
                else if (st == 0 && c->alpha_cache_valid) a = c->alpha_cache;
                else if (deferred) {
                    // its value reaches the host with the stage cross's residual readback
                    c->alpha_dev = alpha_launch(c, X, st, false);
                    a = 1.0;  // not used by the kernels while alpha_dev is set
                } else a = alpha_now(c, X);
                if (!deferred) {
                    WTT_REQUIRE(a > 0.0, WENOTT_EINVAL, "alpha must be positive");
                    c->info.alpha[st] = a;
                }
                // rounds_per_stage = 2 (eq. tt-ssprk3 literally): the forward Euler value
                // Z = X + dt L(X) is rounded, then a_s U^n + b_s Z is formed and rounded again
                const bool two = c->o.rounds_per_stage == 2 && aw[st] != 0.0;
                const double wa = two ? 0.0 : aw[st], wb = two ? 1.0 : bw[st];
                TT S;
                bool rounded = false;
                if (c->o.scheme == 0) {
                    // stage-cross: one cross of a_s U^n + b_s (X + dt L(X)) itself; the rounding of
                    // a sweep's result is queued behind that sweep's residual check and dropped
                    // if the sweep is not accepted
                    CrossStat cs;
                    const std::function<void(const FluxTT &)> spec = [&](const FluxTT &F) {
                        S = cross_to_tt(c, F, -1);
                        c->info.sum_rank[st] = S.maxrank();
                        rounded = true;
                        round_tt(c, S, eps, true, norms, st == 2 && !two);
                    };
                    const std::function<void()> drop = [&]() {
                        S.release(c->s);
                        rounded = false;
                    };
                    FluxTT F;
                    try {
                        F = cross_stage(c, X, &c->U, StageWeights{wa, wb, wb * dt}, a, eps, cs, &spec, &drop);
                    } catch (...) {
                        if (rounded) S.release(c->s);
                        throw;
                    }
                    c->info.sweeps[st][0] = cs.sweeps;
                    c->info.residual[st][0] = cs.residual;
                    c->info.flux_rank[st][0] = cs.maxrank;
                    if (!rounded) S = cross_to_tt(c, F, -1);
                    F.release(c->s);
                } else {
                    std::vector<TT> terms = rhs_terms(c, X, a, eps, st);
                    std::vector<std::pair<double, const TT *>> w;
                    if (wa != 0.0) w.push_back({wa, &c->U});
                    w.push_back({wb, &X});
                    for (auto &t : terms) w.push_back({wb * dt, &t});
                    S = tt_sum(c, w);
                    for (auto &t : terms) t.release(c->s);
                }
                if (!rounded) {
                    c->info.sum_rank[st] = S.maxrank();
                    // synchronises (the deferred alpha has arrived); the norms are needed after the last stage
                    round_tt(c, S, eps, true, norms, st == 2 && !two);
                }
                if (two) {  // round(a_s U^n + b_s round(X + dt L(X)))
                    TT Y = tt_sum(c, {{aw[st], &c->U}, {bw[st], &S}});
                    S.release(c->s);
                    S = Y;
                    round_tt(c, S, eps, true, norms, st == 2);
                }
                if (x_owned) X.release(c->s);
                X = S;
                x_owned = true;
                if (deferred) {
                    c->alpha_dev = nullptr;
                    raise_flags(c, status_flags(c));
                    a = status_alpha(c, st);
                    WTT_REQUIRE(a > 0.0, WENOTT_EINVAL, "alpha must be positive");
                    c->info.alpha[st] = a;
                }
            }
        } catch (...) {
            c->alpha_dev = nullptr;
            if (x_owned) X.release(c->s);
            throw;
        }
        c->U.release(c->s);
        c->U = X;
        c->alpha_cache_valid = false;
        c->max_norm = *std::max_element(norms.begin(), norms.end());
        c->info.max_norm = c->max_norm;
        c->info.eps = eps;
        c->info.c_eps = c->c_eps;
        finish_call_info(c, t0);
    });
}

wenott_status wenott_batch_rk3_step(wenott_ctx **ctxs, int32_t n, const double *dt, const double *eps_in) {
    if (!ctxs || n <= 0 || !dt) return WENOTT_EINVAL;
    for (int i = 0; i < n; ++i)
        if (!ctxs[i] || !(dt[i] > 0.0)) return WENOTT_EINVAL;
    return run_guarded(ctxs[0], [&] {
        const int d = ctxs[0]->d;
        for (int i = 0; i < n; ++i) {
            wenott_ctx *c = ctxs[i];
            WTT_REQUIRE(c->d == d && c->s == ctxs[0]->s, WENOTT_EINVAL,
                        "batched states need the same dimension and the same stream");
            WTT_REQUIRE(c->o.scheme == 0 && c->o.use_proposal == 0 && !c->logging && c->o.rounds_per_stage == 1,
                        WENOTT_EINVAL,
                        "batched stepping runs the stage-cross scheme with one rounding per stage, without the "
                        "proposal or cross logging");
            for (int j = 0; j < i; ++j) WTT_REQUIRE(ctxs[j] != c, WENOTT_EINVAL, "a context appears twice");
            require_inflow_states(c);
        }
        double t0 = seconds_now();
        std::vector<BState> bs(n);
        for (int i = 0; i < n; ++i) {
            reset_call_info(ctxs[i]);
            bs[i].c = ctxs[i];
            bs[i].X = ctxs[i]->U;
            bs[i].dt = dt[i];
            bs[i].eps = (eps_in && eps_in[i] > 0.0) ? eps_in[i] : current_eps(ctxs[i]);
        }
        const double aw[3] = {0.0, 0.75, 1.0 / 3.0}, bw[3] = {1.0, 0.25, 2.0 / 3.0};
        std::vector<TT> Ys;
        try {
            for (int st = 0; st < 3; ++st) {
                bool any = false;
                // the first stage reuses an alpha the caller had computed for this state, as the
                // single-state step does
                auto cached = [&](const BState &b) { return st == 0 && b.c->alpha_cache_valid; };
                for (auto &b : bs)
                    if (b.c->o.alpha_mode != 2 && !cached(b)) {
                        alpha_launch(b.c, b.X, 3);
                        any = true;
                    }
                if (any) host_wait(ctxs[0]);
                for (auto &b : bs) {
                    if (b.c->o.alpha_mode == 2) {
                        b.alpha = b.c->o.alpha_given;
                    } else if (cached(b)) {
                        b.alpha = b.c->alpha_cache;
                    } else {
                        raise_flags(b.c, status_flags(b.c));
                        b.alpha = status_alpha(b.c, 3);
                    }
                    WTT_REQUIRE(b.alpha > 0.0, WENOTT_EINVAL, "alpha must be positive");
                    b.c->info.alpha[st] = b.alpha;
                }
                batch_cross(bs, aw, bw, st);
                Ys.assign(n, TT());
                for (int i = 0; i < n; ++i) {
                    Ys[i] = cross_to_tt(bs[i].c, bs[i].F, -1);
                    bs[i].F.release(bs[i].c->s);
                    bs[i].c->info.sum_rank[st] = Ys[i].maxrank();
                }
                batch_round(bs, Ys);
                for (int i = 0; i < n; ++i) {
                    if (bs[i].x_owned) bs[i].X.release(bs[i].c->s);
                    bs[i].X = Ys[i];
                    bs[i].x_owned = true;
                }
                Ys.clear();
            }
        } catch (...) {
            for (auto &y : Ys) y.release(ctxs[0]->s);
            for (auto &b : bs) {
                if (b.x_owned) b.X.release(b.c->s);
                b.F.release(b.c->s);
            }
            throw;
        }
        for (auto &b : bs) {
            wenott_ctx *c = b.c;
            c->U.release(c->s);
            c->U = b.X;
            c->alpha_cache_valid = false;
            c->max_norm = *std::max_element(b.norms.begin(), b.norms.end());
            c->info.max_norm = c->max_norm;
            c->info.eps = b.eps;
            c->info.c_eps = c->c_eps;
        }
        for (int i = 0; i < n; ++i) finish_call_info(ctxs[i], t0);
    });
}

wenott_status wenott_finalize(void) {
    try {
        WTT_HIP(hipDeviceSynchronize());
        release_all_caches();
        gemm_tune_release();
        WTT_HIP(hipDeviceSynchronize());
        return WENOTT_OK;
    } catch (const HipError &e) {
        note_error(nullptr, e.what());
        return WENOTT_EHIP;
    }
}

wenott_status wenott_gemm_autotune(int32_t mode) {
    if (mode < 0 || mode > 9) return WENOTT_EINVAL;  // 2 + k forces shape k = 0..7
    gemm_tune_enable(mode);
    return WENOTT_OK;
}

wenott_status wenott_gemm_autotune_table(int32_t *out, int32_t max, int32_t *count) {
    if (!count || max < 0) return WENOTT_EINVAL;
    *count = gemm_tune_table(out, out ? max : 0);
    return WENOTT_OK;
}

wenott_status wenott_round(wenott_ctx *c, double eps) {
    if (!c || !(eps > 0.0)) return WENOTT_EINVAL;
    return run_guarded(c, [&] {
        std::vector<double> norms;
        round_tt(c, c->U, eps, true, norms);
        c->alpha_cache_valid = false;
        c->max_norm = *std::max_element(norms.begin(), norms.end());
    });
}

wenott_status wenott_to_dense(wenott_ctx *c, double *out, int32_t on_device) {
    if (!c || !out) return WENOTT_EINVAL;
    return run_guarded(c, [&] {
        if (on_device) {
            to_dense_dev(c, c->U, out);
        } else {
            long long n = (long long)c->nc;
            for (int k = 0; k < c->d; ++k) n *= c->N[k];
            double *tmp = c->sc.get<double>(S_DENSE, (size_t)n);
            to_dense_dev(c, c->U, tmp);
            WTT_HIP(hipMemcpyAsync(out, tmp, sizeof(double) * n, hipMemcpyDeviceToHost, c->s));
            host_wait(c);
        }
    });
}

wenott_status wenott_get_state(wenott_ctx *c, wenott_tt *view) {
    if (!c || !view) return WENOTT_EINVAL;
    return run_guarded(c, [&] { fill_view(c, c->U, view); });
}

wenott_status wenott_get_info(wenott_ctx *c, wenott_info *info) {
    if (!c || !info) return WENOTT_EINVAL;
    return run_guarded(c, [&] {
        host_wait(c);
        for (int k = 0; k < 4; ++k) c->info.ranks[k] = k <= c->d ? c->U.R[k] : 0;
        *info = c->info;
    });
}

wenott_status wenott_max_wavespeed(wenott_ctx *c, double *alpha) {
    if (!c || !alpha) return WENOTT_EINVAL;
    return run_guarded(c, [&] {
        *alpha = alpha_now(c, c->U);
        c->alpha_cache = *alpha;  // the first stage of the next step reuses it
        c->alpha_cache_valid = *alpha > 0.0;
    });
}

wenott_status wenott_max_wavespeed_noalloc(wenott_ctx *c, double *alpha) {
    if (!c || !alpha) return WENOTT_EINVAL;
    return run_guarded(c, [&] {
        const TT &U = c->U;
        char *ws = (char *)c->noalloc_ws;
        WTT_REQUIRE(ws != nullptr, WENOTT_EHIP, "no device workspace");
        double *dst = c->d_status + kStatusAlpha + 3;
        if (c->law == WENOTT_LAW_LINADV) {
            fill(c->s, dst, 1, 1.0);
        } else if (c->o.alpha_mode == 1) {
            const size_t ni = alpha_search_ints(U.d, U.N[1]), nd = alpha_search_doubles(U.d, U.N[1]);
            const size_t off = (ni * sizeof(int) + 255) / 256 * 256;
            WTT_REQUIRE(off + nd * sizeof(double) <= kNoAllocBytes, WENOTT_EINVAL, "alpha search workspace too large");
            int ranks[kMaxDim + 1];
            const double *cores[kMaxDim];
            for (int k = 0; k <= U.d; ++k) ranks[k] = U.R[k];
            for (int k = 0; k < U.d; ++k) cores[k] = U.core[k];
            const unsigned long long seed = c->o.seed * 0x9E3779B97F4A7C15ULL + 0xA5A5ULL * (++c->alpha_counter);
            alpha_search(c->s, U.d, c->law, U.N, cores, ranks, c->gamma, seed, c->d_best, (int *)ws,
                         (double *)(ws + off), dst, c->d_flags);
        } else {
            // the exact maximum over every cell: in 2D the left part of a cell is its first core, so
            // the only workspace is one partial maximum per workgroup
            WTT_REQUIRE(U.d == 2, WENOTT_EINVAL,
                        "the exact alpha of a 3D state needs a left-part workspace beyond the static limit; use "
                        "alpha_mode 1 or wenott_max_wavespeed");
            const long long nrows = U.N[0];
            const int nblocks = dense_eval_blocks(1, nrows, U.R[1], U.N[1]);
            WTT_REQUIRE((size_t)nblocks * sizeof(double) <= kNoAllocBytes, WENOTT_EINVAL,
                        "grid too large for the static workspace of the exact alpha");
            dense_eval(c->s, 1, U.d, c->law, nrows, U.R[1], U.N[1], U.core[0], U.cstride(0), U.core[1],
                       U.cstride(1), c->gamma, nullptr, (double *)ws, nblocks, c->d_flags);
            reduce_max_dev(c->s, (double *)ws, nblocks, dst);
        }
        status_readback(c, kStatusAlpha + 4);
        host_wait(c);
        raise_flags(c, status_flags(c));
        *alpha = status_alpha(c, 3);
        c->alpha_cache = *alpha;
        c->alpha_cache_valid = *alpha > 0.0;
    });
}

wenott_status wenott_set_inflow(wenott_ctx *c, int32_t dim, int32_t side, const double *prim) {
    if (!c || !prim) return WENOTT_EINVAL;
    return run_guarded(c, [&] {
        WTT_REQUIRE(dim >= 0 && dim < c->d && (side == 0 || side == 1), WENOTT_EINVAL, "no such side");
        WTT_REQUIRE(bc_side(c->bc[dim], side) == WENOTT_BC_INFLOW, WENOTT_EINVAL, "the side is not an inflow side");
        double q[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        if (c->law == WENOTT_LAW_EULER) {
            // Sec. 4.5.2: rho, rho u_d = rho_in u_d,in, rho E = p_in / (gamma - 1) + rho_in |u_in|^2 / 2
            const double rho = prim[0], p = prim[c->d + 1];
            WTT_REQUIRE(rho > 0.0 && p > 0.0 && std::isfinite(rho) && std::isfinite(p), WENOTT_EINVAL,
                        "non-physical inflow state");
            double ke = 0.0;
            q[0] = rho;
            for (int j = 0; j < c->d; ++j) {
                WTT_REQUIRE(std::isfinite(prim[1 + j]), WENOTT_EINVAL, "non-finite inflow velocity");
                q[1 + j] = rho * prim[1 + j];
                ke += rho * prim[1 + j] * prim[1 + j];
            }
            q[c->d + 1] = p / (c->gamma - 1.0) + 0.5 * ke;
        } else {
            WTT_REQUIRE(std::isfinite(prim[0]), WENOTT_EINVAL, "non-finite inflow value");
            q[0] = prim[0];
        }
        for (int j = 0; j < 5; ++j) c->qin[dim][side][j] = q[j];
        c->qin_set[dim][side] = true;
    });
}

wenott_status wenott_current_eps(wenott_ctx *c, double *eps) {
    if (!c || !eps) return WENOTT_EINVAL;
    return run_guarded(c, [&] { *eps = current_eps(c); });
}

wenott_status wenott_pivot_search(const double *A, int32_t m, int32_t n, int32_t rmax, double rel_tol2,
                                  int32_t allow_persistent, int32_t *rowpiv, int32_t *colpiv, double *L, double *info,
                                  void *hip_stream) {
    if (!A || m < 1 || n < 1 || rmax < 1 || rmax > std::min(m, n) || !(rel_tol2 >= 0.0) || !rowpiv || !colpiv || !L ||
        !info)
        return WENOTT_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    double *B = nullptr, *ws = nullptr, *dinfo = nullptr;
    int *piv = nullptr;
    const wenott_status st = run_guarded(nullptr, [&] {
        WTT_HIP(hipMallocAsync((void **)&B, sizeof(double) * (size_t)m * n, s));
        WTT_HIP(hipMallocAsync((void **)&ws, sizeof(double) * prrlu_ws_doubles(m, n), s));
        WTT_HIP(hipMallocAsync((void **)&dinfo, sizeof(double) * 4, s));
        WTT_HIP(hipMallocAsync((void **)&piv, sizeof(int) * 2 * (size_t)rmax, s));
        WTT_HIP(hipMemcpyAsync(B, A, sizeof(double) * (size_t)m * n, hipMemcpyDeviceToDevice, s));
        bool persistent = allow_persistent != 0;
        int next = prrlu(s, m, n, B, rmax, rel_tol2, piv, piv + rmax, L, dinfo, ws, 0, 8, persistent);
        double h[3];
        for (;;) {
            WTT_HIP(hipMemcpyAsync(h, dinfo, sizeof(double) * 3, hipMemcpyDeviceToHost, s));
            WTT_HIP(hipStreamSynchronize(s));
            if (h[0] >= 0.0) break;
            WTT_REQUIRE(h[0] != -2.0, WENOTT_EHIP, "pivot search: the wait for the other workgroups ran out");
            WTT_REQUIRE(next <= rmax + 1, WENOTT_EHIP, "pivot search did not stop");
            next = prrlu(s, m, n, B, rmax, rel_tol2, piv, piv + rmax, L, dinfo, ws, next, next + std::max(8, next / 2),
                         persistent);
        }
        WTT_HIP(hipMemcpyAsync(rowpiv, piv, sizeof(int) * rmax, hipMemcpyDeviceToDevice, s));
        WTT_HIP(hipMemcpyAsync(colpiv, piv + rmax, sizeof(int) * rmax, hipMemcpyDeviceToDevice, s));
        WTT_HIP(hipStreamSynchronize(s));
        info[0] = h[0];
        info[1] = h[1];
        info[2] = h[2];
    });
    if (B) (void)hipFreeAsync(B, s);
    if (ws) (void)hipFreeAsync(ws, s);
    if (dinfo) (void)hipFreeAsync(dinfo, s);
    if (piv) (void)hipFreeAsync(piv, s);
    (void)hipStreamSynchronize(s);
    return st;
}

wenott_status wenott_pivot_layout(int32_t m, int32_t n, int32_t *out) {
    if (m < 1 || n < 1 || !out) return WENOTT_EINVAL;
    return run_guarded(nullptr, [&] { prrlu_layout(m, n, true, out); });
}

wenott_status wenott_set_pivot_wait_limit(int32_t polls) {
    set_coop_spin(polls);
    return WENOTT_OK;
}

wenott_status wenott_set_profiling(wenott_ctx *c, int32_t on) {
    if (!c) return WENOTT_EINVAL;
    c->profiling = on != 0;
    return WENOTT_OK;
}

wenott_status wenott_set_proposal(wenott_ctx *c, const float *params) {
    if (!c) return WENOTT_EINVAL;
    c->proposal = params;
    return WENOTT_OK;
}

wenott_status wenott_set_cross_logging(wenott_ctx *c, int32_t on) {
    if (!c) return WENOTT_EINVAL;
    c->logging = on != 0;
    return WENOTT_OK;
}

wenott_status wenott_get_cross_log(wenott_ctx *c, float *x, int32_t *rank_class, float *hist, int32_t max, int32_t *n) {
    if (!c || !n || max < 0 || (max > 0 && (!x || !rank_class || !hist))) return WENOTT_EINVAL;
    const int cnt = std::min<int>(max, (int)c->log_cls.size());
    std::memcpy(x, c->log_x.data(), sizeof(float) * (size_t)cnt * WENOTT_MLP_IN);
    std::memcpy(rank_class, c->log_cls.data(), sizeof(int32_t) * (size_t)cnt);
    std::memcpy(hist, c->log_hist.data(), sizeof(float) * (size_t)cnt * WENOTT_MLP_BINS);
    *n = cnt;
    c->log_x.clear();
    c->log_cls.clear();
    c->log_hist.clear();
    return WENOTT_OK;
}

const char *wenott_last_error(wenott_ctx *c) { return c ? c->last_error.c_str() : g_last_error.c_str(); }

}  // extern "C"
