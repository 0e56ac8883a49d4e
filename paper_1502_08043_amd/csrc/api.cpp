// C ABI of libpwcoul: argument checks, table set-up and ownership, launches.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

#include "pwc_internal.h"

using pwc::Table;

namespace {

pwc_status from_hip(hipError_t e) {
    if (e == hipSuccess) return PWC_OK;
    if (e == hipErrorOutOfMemory) return PWC_ERR_NOMEM;
    return PWC_ERR_DEVICE;
}

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

// Choose the node chunking of a table whose entries take `row_bytes` bytes per
// node in LDS (plus 8 bytes of weight per node): the fewest padded nodes
// nchunk * c, c even, with the chunk inside the LDS budget.
bool plan_chunks(int Q, size_t row_bytes, int *c_out, int *nchunk_out) {
    int best_c = 0, best_n = 0;
    long best_total = -1;
    for (int n = 1; n <= Q; ++n) {
        int c = (Q + n - 1) / n;
        c += c & 1;
        if (static_cast<size_t>(c) * (row_bytes + 8) > static_cast<size_t>(pwc::kLdsBudget)) continue;
        const long total = static_cast<long>(c) * n;
        if (best_total < 0 || total < best_total) {
            best_total = total;
            best_c = c;
            best_n = n;
        }
        if (total == Q) break;
    }
    if (best_total < 0) return false;
    *c_out = best_c;
    *nchunk_out = best_n;
    return true;
}

}  // namespace

namespace pwc {

// Node passes of the reconstruction kernels: G lanes per quadruple, W words
// per lane, c = 2 G W nodes per pass, P = ceil(Q / c) passes.  A layout's cost
// is P times the larger of its compute time per pass and the pass's HBM
// stream (packed entries in, partial sums in and out).  Compute times per
// 16 nodes of 1e8 quadruples, in ms, measured on MI355X for each arithmetic
// (the 4x1 layout estimated); the 16-node layouts on the 9171-planewave
// table and the 32-node ones on the 5575-planewave table, both Q = 96.
// The first pass decodes the stream as well, about kDecodeExtra more.  The
// one-lane layout runs fused (one launch, no stream between passes) when
// its slab and the decode maps fit in LDS together: its cost is then P
// times the fused figures, measured the same way for the whole call (1e8
// quadruples of the lookup stream: 2.65, 4.5 and 1.6 ms).  On uniform
// streams of 1045 to 7153 planewaves the fused FP64 call beats the 8x2
// passes by 11-16% from Q = 96 on and trails them by 4% at Q = 64.
// lanes = words = 0 takes the cheapest layout whose slab fits; otherwise
// the given one.
bool plan_fold(int Q, int E, int lanes, int words, pwc_precision p, size_t maps_bytes, FoldLayout &fl) {
    // fp32: ms per 16 nodes of 1e8 quadruples with four nodes per word.
    static const struct { int G, W; double fp64, mixed, fp32; } kLayouts[] = {
        {8, 2, 0.49, 0.83, 0.32}, {16, 1, 0.61, 0.97, 0.40}, {1, 8, 0.575, 0.835, 0.33},
        {4, 2, 0.58, 0.86, 0.34}, {2, 4, 0.58, 0.79, 0.33}, {8, 1, 0.66, 1.02, 0.42},
        {4, 1, 0.80, 1.10, 0.50}};
    static const struct { double fp64, mixed, fp32; } kFused = {0.44, 0.75, 0.27};
    constexpr double kPassStream = 0.30;   // ms per pass of 1e8 quadruples
    constexpr double kDecodeExtra = 0.25;  // ms per call of 1e8 quadruples
    const int npw = nodes_per_word(p);
    const int Qp = (Q + 31) / 32 * 32;
    double best = -1.0;
    for (const auto &l : kLayouts) {
        if (lanes && (l.G != lanes || l.W != words)) continue;
        const int c = npw * l.G * l.W;
        // the slab row is G W 16-byte words whatever the precision
        if (static_cast<size_t>(E) * l.G * l.W * 16 > static_cast<size_t>(kLdsMax)) continue;
        const int P = (Q + c - 1) / c;
        if (P * c > Qp) continue;   // the passes read nodes up to P c of each padded row
        FoldLayout cand;
        cand.G = l.G;
        cand.W = l.W;
        cand.E = E;
        cand.nchunk = P;
        const bool fused = fused_layout(cand, maps_bytes);
        const double per16 = fused ? (p == PWC_MIXED ? kFused.mixed : p == PWC_FP32 ? kFused.fp32 : kFused.fp64)
                                   : (p == PWC_MIXED ? l.mixed : p == PWC_FP32 ? l.fp32 : l.fp64);
        const double cost = fused ? P * per16 * c / 16.0
                                  : P * std::max(per16 * c / 16.0, kPassStream) + kDecodeExtra;
        if (best < 0.0 || cost < best) {
            best = cost;
            fl.G = l.G;
            fl.W = l.W;
            fl.c = c;
            fl.nchunk = P;
        }
    }
    fl.E = E;
    fl.Qp = Qp;
    return best >= 0.0;
}

}  // namespace pwc

namespace {

float2 split_hilo(double v) {
    const float hi = static_cast<float>(v);
    return make_float2(hi, static_cast<float>(v - static_cast<double>(hi)));
}

}  // namespace

namespace pwc {

// Device blocks of released tables and value tables are kept for later
// tables of the same device: allocating and releasing a 0.5 GB value table
// costs about 0.1 ms each way.  At most kCacheBytes are kept; a block is
// reused for a request at most 1/8 smaller than it, so a table never holds
// much more memory than it needs.  A released table's blocks carry the
// events of the streams that used it (EventSet) and are reused only after
// all of them have completed, so releasing a table never waits for work on
// other tables; a block released without events waited for the device.
struct EventSet {
    int refs = 0;                    // blocks that hold the set (g_cache_mu)
    std::vector<hipEvent_t> ev;
};

namespace {
std::mutex g_cache_mu;
struct CachedBlock {
    int device;
    void *p;
    size_t bytes;
    EventSet *es;    // nullptr: idle
};
std::vector<CachedBlock> g_cache;   // oldest first
size_t g_cache_total = 0;
constexpr size_t kCacheBytes = size_t(4) << 30;

void unref(EventSet *es) {   // caller holds g_cache_mu
    if (es && --es->refs == 0) {
        for (hipEvent_t e : es->ev) (void)hipEventDestroy(e);
        delete es;
    }
}

// True once every event of the block's set has completed (the set is then
// dropped).  hipErrorNotReady is not a sticky error; clear it all the same.
bool block_idle(CachedBlock &b) {
    if (!b.es) return true;
    for (hipEvent_t e : b.es->ev) {
        const hipError_t q = hipEventQuery(e);
        if (q == hipErrorNotReady) {
            (void)hipGetLastError();
            return false;
        }
    }
    unref(b.es);
    b.es = nullptr;
    return true;
}

void free_block(CachedBlock &b) {   // caller holds g_cache_mu
    if (b.es)
        for (hipEvent_t e : b.es->ev) (void)hipEventSynchronize(e);
    unref(b.es);
    b.es = nullptr;
    (void)hipFree(b.p);
}

void release_cached(int device) {   // device < 0: every device; caller holds the lock
    for (auto it = g_cache.begin(); it != g_cache.end();) {
        if (device >= 0 && it->device != device) {
            ++it;
            continue;
        }
        free_block(*it);
        g_cache_total -= it->bytes;
        it = g_cache.erase(it);
    }
}
}  // namespace

hipError_t dev_alloc(size_t bytes, void **p, size_t *got) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto best = g_cache.end();
        for (auto it = g_cache.begin(); it != g_cache.end(); ++it)
            if (it->device == dev && it->bytes >= bytes && it->bytes - bytes <= bytes / 8 &&
                (best == g_cache.end() || it->bytes < best->bytes) && block_idle(*it))
                best = it;
        if (best != g_cache.end()) {
            *p = best->p;
            *got = best->bytes;
            g_cache_total -= best->bytes;
            g_cache.erase(best);
            return hipSuccess;
        }
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {   // give the cached blocks back and try once more
        (void)hipGetLastError();
        {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            release_cached(dev);
        }
        e = hipMalloc(p, bytes);
    }
    *got = bytes;
    return e;
}

void dev_release(void *p, size_t bytes, EventSet *es) {
    if (!p) return;
    // Work in flight may still read the block: without the events of its
    // users, wait for the device first, as hipFree would.
    if (!es) (void)hipDeviceSynchronize();
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_cache_mu);
    if (es) ++es->refs;
    g_cache.push_back({dev, p, bytes, es});
    g_cache_total += bytes;
    while (g_cache_total > kCacheBytes && !g_cache.empty()) {
        free_block(g_cache.front());
        g_cache_total -= g_cache.front().bytes;
        g_cache.erase(g_cache.begin());
    }
}

void note_use(const Table &t, hipStream_t s, bool may_create) {
    if (!t.uses) return;
    UseLog &u = *t.uses;
    std::lock_guard<std::mutex> lk(u.mu);
    if (u.overflow) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
        (void)hipGetLastError();
        u.overflow = true;   // a captured record cannot be queried: wait for the device instead
        return;
    }
    hipEvent_t ev = nullptr;
    for (auto &x : u.ev)
        if (x.first == s) ev = x.second;
    if (!ev) {
        if (!may_create || u.ev.size() >= static_cast<size_t>(kMaxUseStreams) ||
            hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            u.overflow = true;
            return;
        }
        u.ev.emplace_back(s, ev);
    }
    if (hipEventRecord(ev, s) != hipSuccess) {
        (void)hipGetLastError();
        u.overflow = true;
    }
}

// Pinned staging buffers for the table uploads.  A copy from pageable
// memory keeps the host until the runtime has staged it (about 20 us for the
// 58 KB of a 9171-planewave table); from pinned memory it is a DMA the host
// only queues.  A buffer is reused once the event recorded after its copy
// has completed; at most kMaxStages exist, and a creation that finds none
// free uploads from pageable memory instead.
namespace {
struct Stage {
    int device = -1;
    void *p = nullptr;        // nullptr: an empty slot
    size_t bytes = 0;
    hipEvent_t done = nullptr;
    bool in_use = false;
};
constexpr int kMaxStages = 16;
std::mutex g_stage_mu;
Stage g_stage[kMaxStages];

// A free pinned buffer of at least `bytes` on the current device: its slot,
// and its address in *p; -1 if none can be had.
int stage_acquire(size_t bytes, char **p) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_stage_mu);
    int empty = -1;
    for (int i = 0; i < kMaxStages; ++i) {
        Stage &st = g_stage[i];
        if (!st.p) {
            if (empty < 0) empty = i;
            continue;
        }
        if (st.device == dev && !st.in_use && st.bytes >= bytes) {
            const hipError_t q = hipEventQuery(st.done);
            if (q == hipSuccess) {
                st.in_use = true;
                *p = static_cast<char *>(st.p);
                return i;
            }
            (void)hipGetLastError();   // hipErrorNotReady: its copy is still in flight
        }
    }
    if (empty < 0) return -1;
    Stage st;
    st.device = dev;
    st.bytes = (bytes + 65535) / 65536 * 65536;
    if (hipHostMalloc(&st.p, st.bytes) != hipSuccess) {
        (void)hipGetLastError();
        return -1;
    }
    if (hipEventCreateWithFlags(&st.done, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipHostFree(st.p);
        return -1;
    }
    st.in_use = true;
    g_stage[empty] = st;
    *p = static_cast<char *>(st.p);
    return empty;
}

// Mark the buffer's copy (queued on s); the buffer is reused after it.
void stage_release(int i, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_stage_mu);
    (void)hipEventRecord(g_stage[i].done, s);
    g_stage[i].in_use = false;
}

void release_stages() {   // buffers whose copies have completed
    std::lock_guard<std::mutex> lk(g_stage_mu);
    for (Stage &st : g_stage) {
        if (!st.p || st.in_use) continue;
        if (hipEventQuery(st.done) != hipSuccess) {
            (void)hipGetLastError();
            continue;
        }
        (void)hipEventDestroy(st.done);
        (void)hipHostFree(st.p);
        st = Stage{};
    }
}
}  // namespace

void free_table(Table &t) {
    // The blocks wait for the table's construction (ready) and for the last
    // work of every stream that used it; if that record is incomplete, the
    // release waits for the device.
    EventSet *es = nullptr;
    if (t.uses && (t.d_block || t.d_val)) {
        std::lock_guard<std::mutex> lk(t.uses->mu);
        if (!t.uses->overflow) {
            es = new (std::nothrow) EventSet;
            if (es) {
                for (auto &x : t.uses->ev) es->ev.push_back(x.second);
                t.uses->ev.clear();
                if (t.ready) es->ev.push_back(t.ready);
                t.ready = nullptr;
            }
        }
    }
    if (es) {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        ++es->refs;   // held across the two releases below
    }
    dev_release(t.d_block, t.block_bytes, es);
    t.d_block = nullptr;
    dev_release(t.d_val, t.val_alloc, es);
    t.d_val = nullptr;
    t.val_bytes = t.val_alloc = 0;
    if (es) {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        unref(es);
    }
    if (t.uses) {   // events of streams the blocks no longer wait for
        std::lock_guard<std::mutex> lk(t.uses->mu);
        for (auto &x : t.uses->ev) (void)hipEventDestroy(x.second);
        t.uses->ev.clear();
    }
    if (t.ready) (void)hipEventDestroy(t.ready);
    t.ready = nullptr;
    t.h_img.reset();
}

// Carve the table's single device allocation.  With base == nullptr only the
// size is computed (used for admission before anything is allocated).
size_t carve(Table &t, size_t n_reps, char *base) {
    const int Q = t.Q, K = t.K, nd = t.nd, E = t.fl.E, D = t.ndir;
    const size_t Qp = static_cast<size_t>(t.fl.Qp);
    const size_t Qd = static_cast<size_t>(t.dl.c) * t.dl.nchunk;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
    // Host-formed inputs first (one upload covers them and the error words),
    // then the kernel-written layouts; tauF .. diagHL hold zero padding.
    const size_t o_basis = take(sizeof(int32_t) * t.N);
    const size_t o_fold = take(sizeof(int32_t) * nd * nd);
    const size_t o_reps = take(sizeof(int32_t) * n_reps);
    const size_t o_beta = take(sizeof(double) * D * Q);
    const size_t o_W = take(sizeof(double) * Q);
    const size_t o_gl = take(sizeof(double) * 2 * kGlPanelPoints);
    const size_t o_Wcbrt = take(sizeof(double) * Q);
    const size_t o_Wdiag = take(sizeof(double) * Qd);
    const size_t o_WdiagHL = take(sizeof(float2) * Qd);
    const size_t o_err = take(sizeof(int) * 64);
    const size_t o_prim = take(sizeof(double) * D * Q * 2 * (K + 1));
    const size_t o_tau = take(sizeof(double) * D * Q * nd * nd);
    const size_t o_tauF = take(sizeof(double) * Qp * E);
    const size_t o_tauHL = take(sizeof(float2) * Qp * E);
    const size_t o_tau32 = take(sizeof(float) * Qp * E);
    const size_t o_diag = take(sizeof(double) * Qd * D * (K + 1));
    const size_t o_diagHL = take(sizeof(float2) * Qd * D * (K + 1));
    const size_t o_kt64 = take(sizeof(double) * static_cast<size_t>(t.kt_n));
    const size_t o_ktMX = take(sizeof(double) * static_cast<size_t>(t.kt_n));
    if (base) {
        t.d_basis = reinterpret_cast<int32_t *>(base + o_basis);
        t.d_fold = reinterpret_cast<int32_t *>(base + o_fold);
        t.d_reps = reinterpret_cast<int32_t *>(base + o_reps);
        t.d_beta = reinterpret_cast<double *>(base + o_beta);
        t.d_W = reinterpret_cast<double *>(base + o_W);
        t.d_gl = reinterpret_cast<double *>(base + o_gl);
        t.d_prim = reinterpret_cast<double *>(base + o_prim);
        t.d_tau = reinterpret_cast<double *>(base + o_tau);
        t.d_tauF = reinterpret_cast<double *>(base + o_tauF);
        t.d_tauHL = reinterpret_cast<float2 *>(base + o_tauHL);
        t.d_tau32 = reinterpret_cast<float *>(base + o_tau32);
        t.d_Wcbrt = reinterpret_cast<double *>(base + o_Wcbrt);
        t.d_diag = reinterpret_cast<double *>(base + o_diag);
        t.d_diagHL = reinterpret_cast<float2 *>(base + o_diagHL);
        t.d_Wdiag = reinterpret_cast<double *>(base + o_Wdiag);
        t.d_WdiagHL = reinterpret_cast<float2 *>(base + o_WdiagHL);
        t.d_ktab64 = t.kt_n ? reinterpret_cast<double *>(base + o_kt64) : nullptr;
        t.d_ktabMX = t.kt_n ? reinterpret_cast<double *>(base + o_ktMX) : nullptr;
        t.d_err = reinterpret_cast<int *>(base + o_err);
    }
    return off;
}

pwc_status plan_table(const double sides[3], int n2max, const pwc_mesh &m, Table &t, TableSetup &su) {
    for (int d = 0; d < 3; ++d)
        if (!(sides[d] > 0.0) || !std::isfinite(sides[d])) return PWC_ERR_ARG;
    if (n2max < 1 || n2max > PWC_MAX_N2MAX) return PWC_ERR_ARG;
    const bool cube = sides[0] == sides[1] && sides[1] == sides[2];
    t.ndir = cube ? 1 : 3;
    // Reference length: the side of a cube; the geometric mean of a box's sides,
    // which makes rho_x rho_y rho_z = 1 and keeps the cube's prefactor.
    t.L = cube ? sides[0]
               : static_cast<double>(std::cbrt(static_cast<long double>(sides[0]) * sides[1] * sides[2]));
    for (int d = 0; d < 3; ++d) {
        t.Ld[d] = sides[d];
        t.rho[d] = cube ? 1.0 : sides[d] / t.L;
    }
    const double L = t.L;
    t.n2max = n2max;
    t.nmax = static_cast<int>(std::floor(std::sqrt(static_cast<double>(n2max)) + 1e-9));
    t.K = 2 * t.nmax;
    t.nd = 2 * t.K + 1;
    t.mesh = m;
    t.h_basis = enumerate_basis(n2max);
    t.N = static_cast<int64_t>(t.h_basis->packed.size());
    if (!build_mesh(m, L, t.h_beta, t.h_W, &t.n_interval1)) return PWC_ERR_ARG;
    t.Q = static_cast<int>(t.h_beta.size());
    build_fold(t.K, su.fold, su.reps);
    t.E1 = static_cast<int>(su.reps.size() / 2);
    t.fl.E = t.ndir * t.E1;                 // slab rows: the direction tables stacked
    (void)hipGetDevice(&t.device);
    if (hipDeviceGetAttribute(&t.n_cu, hipDeviceAttributeMultiprocessorCount, t.device) != hipSuccess ||
        t.n_cu <= 0)
        t.n_cu = 256;
    t.flm.E = t.fls.E = t.fl.E;
    const size_t maps = fold_maps_bytes(t.N, t.nd);
    if (!plan_fold(t.Q, t.fl.E, 0, 0, PWC_FP64, maps, t.fl) || !plan_fold(t.Q, t.fl.E, 0, 0, PWC_MIXED, maps, t.flm) ||
        !plan_fold(t.Q, t.fl.E, 0, 0, PWC_FP32, maps, t.fls) ||
        !plan_chunks(t.Q, static_cast<size_t>(t.ndir) * (t.K + 1) * 8, &t.dl.c, &t.dl.nchunk))
        return PWC_ERR_ARG;
    // The direct kernel beats the fused node sums up to about 2^19
    // quadruples, and the separate node passes (each restaging a slab) up to
    // the largest list it takes.
    t.direct_max = fused_layout(t.fl, maps) ? kDirectDefault : kDirectMaxN;
    // Exchange kernel table when it fits in one workgroup's LDS: K(a <= b <= c)
    // for a cube (the three directions share one table), K(a, b, c) for a box.
    const int64_t n1 = t.K + 1;
    const int64_t kt_n = cube ? n1 * (n1 + 1) * (n1 + 2) / 6 : n1 * n1 * n1;
    t.kt_n = (kt_n * 8 <= kLdsMax - 4096) ? static_cast<int>(kt_n) : 0;
    t.bytes = carve(t, su.reps.size(), nullptr);
    return PWC_OK;
}

pwc_status build_table(Table &t, const TableSetup &su, hipStream_t s, const double *h_tau) {
    hipError_t e = dev_alloc(t.bytes, &t.d_block, &t.block_bytes);
    if (e != hipSuccess) {
        t.d_block = nullptr;
        return from_hip(e);
    }
    carve(t, su.reps.size(), static_cast<char *>(t.d_block));
    t.uses = std::make_shared<UseLog>();
    const int Q = t.Q;
    const size_t Qd = static_cast<size_t>(t.dl.c) * t.dl.nchunk;
    // Host-side inputs of the table kernels.
    const std::vector<int32_t> &packed = t.h_basis->packed;
    std::vector<double> glx, glw, gl;
    gauss_legendre(kGlPanelPoints, 0.0, 1.0, glx, glw);
    gl = glx;
    gl.insert(gl.end(), glw.begin(), glw.end());
    std::vector<double> Wcbrt(Q), Wdiag(Qd, 0.0);
    std::vector<float2> WdiagHL(Qd, make_float2(0.f, 0.f));
    // Node q sits at flat slot q of every node-chunked layout; padded slots
    // carry zero weight.
    for (int q = 0; q < Q; ++q) {
        // W_q^(1/3) multiplies each of the three factors of a node term in
        // the folded tables (mesh weights are positive).
        Wcbrt[q] = static_cast<double>(std::cbrt(static_cast<long double>(t.h_W[q])));
        Wdiag[q] = t.h_W[q];
        WdiagHL[q] = split_hilo(t.h_W[q]);
    }
    std::vector<double> beta_d(static_cast<size_t>(t.ndir) * Q);   // node of each direction
    for (int d = 0; d < t.ndir; ++d)
        for (int q = 0; q < Q; ++q) beta_d[static_cast<size_t>(d) * Q + q] = t.h_beta[q] / (t.rho[d] * t.rho[d]);
    // One host image of the input region (basis .. error words, zeros in the
    // alignment gaps and the error words) and one upload, from a pinned
    // staging buffer when one is free.
    char *dev0 = static_cast<char *>(t.d_block);
    const size_t in_bytes = static_cast<size_t>(reinterpret_cast<char *>(t.d_prim) - dev0);
    char *img = nullptr;
    const int stage = stage_acquire(in_bytes, &img);
    std::shared_ptr<std::vector<char>> img_p;
    if (stage >= 0) {
        std::memset(img, 0, in_bytes);
    } else {
        img_p = std::make_shared<std::vector<char>>(in_bytes, 0);
        img = img_p->data();
    }
    auto put = [&](const void *dst, const void *src, size_t bytes) {
        std::memcpy(img + (static_cast<const char *>(dst) - dev0), src, bytes);
    };
    put(t.d_basis, packed.data(), sizeof(int32_t) * t.N);
    put(t.d_fold, su.fold.data(), sizeof(int32_t) * su.fold.size());
    put(t.d_reps, su.reps.data(), sizeof(int32_t) * su.reps.size());
    put(t.d_beta, beta_d.data(), sizeof(double) * beta_d.size());
    put(t.d_W, t.h_W.data(), sizeof(double) * Q);
    put(t.d_gl, gl.data(), sizeof(double) * gl.size());
    put(t.d_Wcbrt, Wcbrt.data(), sizeof(double) * Q);
    put(t.d_Wdiag, Wdiag.data(), sizeof(double) * Qd);
    put(t.d_WdiagHL, WdiagHL.data(), sizeof(float2) * Qd);
    // A pageable image stays with the table until pwc_table_destroy, which
    // waits for the device; a pinned one goes back to the pool behind its copy.
    pwc_status st = from_hip(hipMemcpyAsync(dev0, img, in_bytes, hipMemcpyHostToDevice, s));
    if (stage >= 0) stage_release(stage, s);
    else t.h_img = img_p;
    // Padding slots of the node-chunked layouts (tauF .. diagHL) must read
    // as zero; the exchange kernel tables after them are written whole.
    char *pad_end = t.d_ktab64 ? reinterpret_cast<char *>(t.d_ktab64) : dev0 + t.bytes;
    if (st == PWC_OK)
        st = from_hip(hipMemsetAsync(t.d_tauF, 0, static_cast<size_t>(pad_end - reinterpret_cast<char *>(t.d_tauF)), s));
    if (h_tau && st == PWC_OK)
        st = from_hip(hipMemcpyAsync(t.d_tau, h_tau, sizeof(double) * static_cast<size_t>(t.ndir) * Q * t.nd * t.nd,
                                     hipMemcpyHostToDevice, s));
    if (st == PWC_OK) st = from_hip(launch_table_build(t, s, h_tau != nullptr));
    if (st == PWC_OK) st = from_hip(launch_ktab_build(t, s));
    if (st == PWC_OK) st = from_hip(hipEventCreateWithFlags(&t.ready, hipEventDisableTiming));
    if (st == PWC_OK) st = from_hip(hipEventRecord(t.ready, s));
    // h_tau is the caller's buffer: a loaded table waits for its copy.
    if (st == PWC_OK && h_tau) st = from_hip(hipStreamSynchronize(s));
    if (st != PWC_OK) {
        (void)hipStreamSynchronize(s);
        free_table(t);
    }
    return st;
}

// Separable Gaussian basis.  Host set-up: the kept pairs u <= v with
// exp(-(a_u a_v / p)(A_u - A_v)^2) >= eps, numbered by u then v, their product
// parameters (c, p, P) and the pair map; then one allocation holding the map,
// the pair parameters, mesh, weights, error words, the full tables and the
// folded rows (the last folded row stays zero).
pwc_status plan_gauss(const double *a, const double *A, int n1, double L, double eps,
                      const pwc_mesh &m, Table &t) {
    if (n1 < 1 || n1 > kGaussMaxN1 || !(L > 0.0) || !std::isfinite(L) || !(eps >= 0.0) || !(eps < 1.0))
        return PWC_ERR_ARG;
    for (int u = 0; u < n1; ++u)
        if (!(a[u] > 0.0) || !std::isfinite(a[u]) || !std::isfinite(A[u])) return PWC_ERR_ARG;
    t.gauss = true;
    t.n1 = n1;
    t.eps = eps;
    t.L = L;
    for (int d = 0; d < 3; ++d) {
        t.Ld[d] = L;
        t.rho[d] = 1.0;
    }
    t.ndir = 1;
    t.mesh = m;
    t.N = static_cast<int64_t>(n1) * n1 * n1;
    t.h_pmap.assign(static_cast<size_t>(n1) * n1, -1);
    t.h_pair.clear();
    int P1 = 0;
    for (int u = 0; u < n1; ++u)
        for (int v = u; v < n1; ++v) {
            const double p = a[u] + a[v];
            const double dA = A[u] - A[v];
            const double K = std::exp(-(a[u] * a[v] / p) * (dA * dA));
            if (!(K >= eps)) continue;
            if (P1 >= kGaussMaxPairs) return PWC_ERR_RANGE;
            t.h_pmap[static_cast<size_t>(u) * n1 + v] = t.h_pmap[static_cast<size_t>(v) * n1 + u] = P1++;
            const double c = std::pow(2.0 * a[u] / M_PI, 0.25) * std::pow(2.0 * a[v] / M_PI, 0.25) * K;
            t.h_pair.push_back(c);
            t.h_pair.push_back(p);
            t.h_pair.push_back((a[u] * A[u] + a[v] * A[v]) / p);
        }
    t.P1 = P1;
    if (!build_mesh(m, L, t.h_beta, t.h_W, &t.n_interval1)) return PWC_ERR_ARG;
    t.Q = static_cast<int>(t.h_beta.size());
    t.E1 = P1 * (P1 + 1) / 2 + 1;    // folded pairs of pairs, then the zero row
    t.fl.E = t.flm.E = t.E1;
    t.fl.Qp = t.flm.Qp = (t.Q + 31) / 32 * 32;
    t.nd = P1;
    (void)hipGetDevice(&t.device);
    if (hipDeviceGetAttribute(&t.n_cu, hipDeviceAttributeMultiprocessorCount, t.device) != hipSuccess ||
        t.n_cu <= 0)
        t.n_cu = 256;
    const size_t Q = static_cast<size_t>(t.Q), Qp = static_cast<size_t>(t.fl.Qp);
    t.bytes = align256(sizeof(int32_t) * t.h_pmap.size()) + align256(sizeof(double) * t.h_pair.size() + 8) +
              3 * align256(sizeof(double) * Q) + align256(sizeof(int) * 64) +
              align256(sizeof(double) * Q * P1 * P1) + align256(sizeof(double) * Qp * t.E1) +
              align256(sizeof(float2) * Qp * t.E1);
    return PWC_OK;
}

pwc_status build_gauss(Table &t, hipStream_t s) {
    hipError_t e = dev_alloc(t.bytes, &t.d_block, &t.block_bytes);
    if (e != hipSuccess) {
        t.d_block = nullptr;
        return from_hip(e);
    }
    t.uses = std::make_shared<UseLog>();
    const size_t Q = static_cast<size_t>(t.Q), Qp = static_cast<size_t>(t.fl.Qp), P1 = static_cast<size_t>(t.P1);
    char *base = static_cast<char *>(t.d_block);
    size_t off = 0;
    auto take = [&](size_t bytes) { char *p = base + off; off += align256(bytes); return p; };
    t.d_pmap = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * t.h_pmap.size()));
    t.d_pair = reinterpret_cast<double *>(take(sizeof(double) * t.h_pair.size() + 8));
    t.d_beta = reinterpret_cast<double *>(take(sizeof(double) * Q));
    t.d_W = reinterpret_cast<double *>(take(sizeof(double) * Q));
    t.d_Wcbrt = reinterpret_cast<double *>(take(sizeof(double) * Q));
    t.d_err = reinterpret_cast<int *>(take(sizeof(int) * 64));
    t.d_tau = reinterpret_cast<double *>(take(sizeof(double) * Q * P1 * P1));
    t.d_tauF = reinterpret_cast<double *>(take(sizeof(double) * Qp * t.E1));
    t.d_tauHL = reinterpret_cast<float2 *>(take(sizeof(float2) * Qp * t.E1));
    // Host image of the inputs (map .. error words), one upload; the folded
    // rows start as zero (node padding and the zero row).
    const size_t in_bytes = static_cast<size_t>(reinterpret_cast<char *>(t.d_tau) - base);
    auto img = std::make_shared<std::vector<char>>(in_bytes, 0);
    auto put = [&](const void *dst, const void *src, size_t bytes) {
        std::memcpy(img->data() + (static_cast<const char *>(dst) - base), src, bytes);
    };
    std::vector<double> Wcbrt(Q);
    for (size_t q = 0; q < Q; ++q) Wcbrt[q] = static_cast<double>(std::cbrt(static_cast<long double>(t.h_W[q])));
    put(t.d_pmap, t.h_pmap.data(), sizeof(int32_t) * t.h_pmap.size());
    put(t.d_pair, t.h_pair.data(), sizeof(double) * t.h_pair.size());
    put(t.d_beta, t.h_beta.data(), sizeof(double) * Q);
    put(t.d_W, t.h_W.data(), sizeof(double) * Q);
    put(t.d_Wcbrt, Wcbrt.data(), sizeof(double) * Q);
    t.h_img = img;   // kept until destroy: the copy may still read it
    pwc_status st = from_hip(hipMemcpyAsync(base, img->data(), in_bytes, hipMemcpyHostToDevice, s));
    if (st == PWC_OK)
        st = from_hip(hipMemsetAsync(t.d_tauF, 0, static_cast<size_t>(base + t.bytes - reinterpret_cast<char *>(t.d_tauF)), s));
    if (st == PWC_OK && t.P1 > 0) st = from_hip(launch_gauss_tables(t, s));
    if (st == PWC_OK) st = from_hip(hipEventCreateWithFlags(&t.ready, hipEventDisableTiming));
    if (st == PWC_OK) st = from_hip(hipEventRecord(t.ready, s));
    if (st != PWC_OK) {
        (void)hipStreamSynchronize(s);
        free_table(t);
    }
    return st;
}

}  // namespace pwc

extern "C" {

const char *pwc_version(void) { return "pwcoul 0.1.0 (gfx950)"; }

const char *pwc_status_str(pwc_status s) {
    switch (s) {
        case PWC_OK: return "ok";
        case PWC_ERR_ARG: return "invalid argument";
        case PWC_ERR_RANGE: return "index out of range";
        case PWC_ERR_NOMEM: return "out of memory";
        case PWC_ERR_DEVICE: return "HIP device error";
        case PWC_ERR_BUSY: return "busy";
        case PWC_ERR_STATE: return "invalid state";
        case PWC_ERR_IO: return "table file error";
        case PWC_ERR_LIMIT: return "size beyond the call's fixed limit";
    }
    return "unknown status";
}

pwc_status pwc_mesh_default(int n_nodes, pwc_mesh *out) {
    if (!out || n_nodes < 16 || n_nodes % 8 != 0 || n_nodes > PWC_MAX_NODES) return PWC_ERR_ARG;
    out->kind = PWC_MESH_GEOMETRIC;
    out->n_sub = 8;
    out->ratio = 5.0;
    out->q_sub = (n_nodes - 8) / 8;
    out->q_tail = 8;
    out->alpha_c = 0.0;
    return PWC_OK;
}

pwc_status pwc_mesh_count(const pwc_mesh *mesh, int *n_nodes) {
    if (!mesh || !n_nodes) return PWC_ERR_ARG;
    return pwc::mesh_valid(*mesh, n_nodes) ? PWC_OK : PWC_ERR_ARG;
}

pwc_status pwc_table_create(double L, int n2max, int n_nodes, const pwc_mesh *mesh, void *stream,
                            pwc_table **out) {
    return pwc_table_create_box(L, L, L, n2max, n_nodes, mesh, stream, out);
}

pwc_status pwc_table_create_box(double Lx, double Ly, double Lz, int n2max, int n_nodes,
                                const pwc_mesh *mesh, void *stream, pwc_table **out) {
    if (!out) return PWC_ERR_ARG;
    *out = nullptr;
    pwc_mesh m{};
    if (mesh) {
        int q = 0;
        if (!pwc::mesh_valid(*mesh, &q)) return PWC_ERR_ARG;
        if (n_nodes != 0 && n_nodes != q) return PWC_ERR_ARG;
        m = *mesh;
    } else if (pwc_mesh_default(n_nodes, &m) != PWC_OK) {
        return PWC_ERR_ARG;
    }
    pwc_table *h = new (std::nothrow) pwc_table;
    if (!h) return PWC_ERR_NOMEM;
    pwc::TableSetup su;
    const double sides[3] = {Lx, Ly, Lz};
    pwc_status st = pwc::plan_table(sides, n2max, m, h->t, su);
    if (st == PWC_OK) st = pwc::build_table(h->t, su, static_cast<hipStream_t>(stream));
    if (st != PWC_OK) {
        delete h;
        return st;
    }
    *out = h;
    return PWC_OK;
}

pwc_status pwc_table_create_gauss(const double *h_exp, const double *h_center, int n1, double L,
                                  double eps, int n_nodes, const pwc_mesh *mesh, void *stream,
                                  pwc_table **out) {
    if (!out) return PWC_ERR_ARG;
    *out = nullptr;
    if (!h_exp || !h_center) return PWC_ERR_ARG;
    pwc_mesh m{};
    if (mesh) {
        int q = 0;
        if (!pwc::mesh_valid(*mesh, &q)) return PWC_ERR_ARG;
        if (n_nodes != 0 && n_nodes != q) return PWC_ERR_ARG;
        m = *mesh;
    } else if (pwc_mesh_default(n_nodes, &m) != PWC_OK) {
        return PWC_ERR_ARG;
    }
    pwc_table *h = new (std::nothrow) pwc_table;
    if (!h) return PWC_ERR_NOMEM;
    pwc_status st = pwc::plan_gauss(h_exp, h_center, n1, L, eps, m, h->t);
    if (st == PWC_OK) st = pwc::build_gauss(h->t, static_cast<hipStream_t>(stream));
    if (st != PWC_OK) {
        delete h;
        return st;
    }
    *out = h;
    return PWC_OK;
}

pwc_status pwc_gauss_info(const pwc_table *t, int *n1, int *n_pairs, double *eps) {
    if (!t || !t->t.gauss) return PWC_ERR_ARG;
    if (n1) *n1 = t->t.n1;
    if (n_pairs) *n_pairs = t->t.P1;
    if (eps) *eps = t->t.eps;
    return PWC_OK;
}

namespace {

// Table file: a fixed header, then beta[Q], W[Q], the folded FP64 tables
// tau[ndir][Q][E1] (one value per orbit of (m, m') under (m, m') -> (m', m)
// and (m, m') -> (-m, -m'), about a quarter of the nd^2 entries) and the
// orbit representatives (m, m') as int8 pairs [E1][2], in native byte order;
// the payload is covered by an FNV-1a checksum.  The representatives are
// those of build_fold; a load checks them and expands the full table.
constexpr char kTableMagic[8] = {'P', 'W', 'C', 'T', 'A', 'B', 'L', '1'};
constexpr uint32_t kTableVersion = 2;

struct TableFileHeader {
    char magic[8];
    uint32_t version, header_bytes;
    double Lx, Ly, Lz;
    int32_t n2max, Q, nd, mesh_kind;
    int64_t N;
    int32_t n_sub, q_sub, q_tail, ndir;
    double ratio, alpha_c;
    uint64_t payload_bytes, checksum;
};

uint64_t fnv1a(const void *data, size_t n, uint64_t h = 1469598103934665603ull) {
    const unsigned char *p = static_cast<const unsigned char *>(data);
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

// Payload size of a file with these fields, or 0 if they are out of the
// library's limits (checked before anything is allocated).
uint64_t table_payload_bytes(int n2max, int Q, int nd, int ndir) {
    if (n2max < 1 || n2max > PWC_MAX_N2MAX || Q < 1 || Q > PWC_MAX_NODES) return 0;
    if (ndir != 1 && ndir != 3) return 0;
    const int nmax = static_cast<int>(std::floor(std::sqrt(static_cast<double>(n2max)) + 1e-9));
    if (nd != 4 * nmax + 1) return 0;
    const uint64_t E1 = static_cast<uint64_t>(2 * nmax + 1) * (2 * nmax + 1);   // orbits of the fold
    return sizeof(double) * (2 * static_cast<uint64_t>(Q) + static_cast<uint64_t>(ndir) * Q * E1) +
           2 * E1;
}

pwc_status table_save(const pwc::Table &tb, const char *path) {
    std::vector<int32_t> fold, reps;
    pwc::build_fold(tb.K, fold, reps);
    const size_t E1 = reps.size() / 2, nd = static_cast<size_t>(tb.nd);
    const size_t nfull = static_cast<size_t>(tb.ndir) * tb.Q * nd * nd;
    std::vector<double> full(nfull);
    hipError_t e = tb.ready ? hipEventSynchronize(tb.ready) : hipSuccess;
    if (e == hipSuccess) e = hipMemcpy(full.data(), tb.d_tau, sizeof(double) * nfull, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return from_hip(e);
    const uint64_t bytes = table_payload_bytes(tb.n2max, tb.Q, tb.nd, tb.ndir);
    std::vector<char> payload(bytes);
    char *w = payload.data();
    std::memcpy(w, tb.h_beta.data(), sizeof(double) * tb.Q);
    std::memcpy(w + sizeof(double) * tb.Q, tb.h_W.data(), sizeof(double) * tb.Q);
    double *folded = reinterpret_cast<double *>(w + 2 * sizeof(double) * tb.Q);
    for (size_t dq = 0; dq < static_cast<size_t>(tb.ndir) * tb.Q; ++dq)
        for (size_t f = 0; f < E1; ++f) {
            const size_t row = static_cast<size_t>(reps[2 * f] + tb.K), col = static_cast<size_t>(reps[2 * f + 1] + tb.K);
            folded[dq * E1 + f] = full[(dq * nd + row) * nd + col];
        }
    int8_t *r8 = reinterpret_cast<int8_t *>(folded + static_cast<size_t>(tb.ndir) * tb.Q * E1);
    for (size_t i = 0; i < 2 * E1; ++i) r8[i] = static_cast<int8_t>(reps[i]);
    TableFileHeader h{};
    std::memcpy(h.magic, kTableMagic, sizeof(h.magic));
    h.version = kTableVersion;
    h.header_bytes = sizeof(h);
    h.Lx = tb.Ld[0];
    h.Ly = tb.Ld[1];
    h.Lz = tb.Ld[2];
    h.ndir = tb.ndir;
    h.n2max = tb.n2max;
    h.Q = tb.Q;
    h.nd = tb.nd;
    h.mesh_kind = tb.mesh.kind;
    h.N = tb.N;
    h.n_sub = tb.mesh.n_sub;
    h.q_sub = tb.mesh.q_sub;
    h.q_tail = tb.mesh.q_tail;
    h.ratio = tb.mesh.ratio;
    h.alpha_c = tb.mesh.alpha_c;
    h.payload_bytes = bytes;
    h.checksum = fnv1a(payload.data(), bytes);
    FILE *f = std::fopen(path, "wb");
    if (!f) return PWC_ERR_IO;
    const bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1 &&
                    std::fwrite(payload.data(), 1, bytes, f) == bytes;
    const bool closed = std::fclose(f) == 0;
    return ok && closed ? PWC_OK : PWC_ERR_IO;
}

pwc_status table_load(const char *path, void *stream, pwc_table **out) {
    FILE *f = std::fopen(path, "rb");
    if (!f) return PWC_ERR_IO;
    TableFileHeader h{};
    // Every header field that sizes an allocation is checked first.
    bool ok = std::fread(&h, sizeof(h), 1, f) == 1 &&
              std::memcmp(h.magic, kTableMagic, sizeof(h.magic)) == 0 &&
              h.version == kTableVersion && h.header_bytes == sizeof(h) &&
              h.payload_bytes != 0 && h.payload_bytes == table_payload_bytes(h.n2max, h.Q, h.nd, h.ndir);
    std::vector<char> payload;
    if (ok) {
        payload.resize(h.payload_bytes);
        ok = std::fread(payload.data(), 1, h.payload_bytes, f) == h.payload_bytes &&
             std::fgetc(f) == EOF && fnv1a(payload.data(), h.payload_bytes) == h.checksum;
    }
    std::fclose(f);
    if (!ok) return PWC_ERR_IO;
    pwc_mesh m{};
    m.kind = static_cast<pwc_mesh_kind>(h.mesh_kind);
    m.n_sub = h.n_sub;
    m.q_sub = h.q_sub;
    m.q_tail = h.q_tail;
    m.ratio = h.ratio;
    m.alpha_c = h.alpha_c;
    int q = 0;
    if (!pwc::mesh_valid(m, &q) || q != h.Q) return PWC_ERR_IO;
    std::unique_ptr<pwc_table> t(new pwc_table);
    pwc::TableSetup su;
    const double sides[3] = {h.Lx, h.Ly, h.Lz};
    pwc_status st = pwc::plan_table(sides, h.n2max, m, t->t, su);
    if (st == PWC_ERR_ARG) st = PWC_ERR_IO;
    if (st == PWC_OK && (t->t.Q != h.Q || t->t.nd != h.nd || t->t.N != h.N || t->t.ndir != h.ndir))
        st = PWC_ERR_IO;
    if (st != PWC_OK) return st;
    const size_t E1 = su.reps.size() / 2, nd = static_cast<size_t>(h.nd);
    const double *beta = reinterpret_cast<const double *>(payload.data());
    const double *folded = beta + 2 * static_cast<size_t>(h.Q);
    const int8_t *r8 = reinterpret_cast<const int8_t *>(folded + static_cast<size_t>(h.ndir) * h.Q * E1);
    for (size_t i = 0; i < 2 * E1; ++i)
        if (r8[i] != su.reps[i]) return PWC_ERR_IO;   // another orbit numbering
    // The stored mesh is the table's mesh; the full tables follow from the
    // folded ones (each entry is its orbit representative's value).
    t->t.h_beta.assign(beta, beta + h.Q);
    t->t.h_W.assign(beta + h.Q, beta + 2 * h.Q);
    std::vector<double> full(static_cast<size_t>(h.ndir) * h.Q * nd * nd);
    for (size_t dq = 0; dq < static_cast<size_t>(h.ndir) * h.Q; ++dq)
        for (size_t e = 0; e < nd * nd; ++e) full[dq * nd * nd + e] = folded[dq * E1 + su.fold[e]];
    st = pwc::build_table(t->t, su, static_cast<hipStream_t>(stream), full.data());
    if (st != PWC_OK) return st;
    *out = t.release();
    return PWC_OK;
}

}  // namespace

pwc_status pwc_table_save(const pwc_table *t, const char *path) {
    if (!t || !path || t->t.gauss) return PWC_ERR_ARG;
    try {
        return table_save(t->t, path);
    } catch (const std::bad_alloc &) {
        return PWC_ERR_NOMEM;
    } catch (...) {
        return PWC_ERR_IO;
    }
}

pwc_status pwc_table_load(const char *path, void *stream, pwc_table **out) {
    if (!out) return PWC_ERR_ARG;
    *out = nullptr;
    if (!path) return PWC_ERR_ARG;
    try {
        return table_load(path, stream, out);
    } catch (const std::bad_alloc &) {
        return PWC_ERR_NOMEM;
    } catch (...) {
        return PWC_ERR_IO;
    }
}

pwc_status pwc_table_destroy(pwc_table *t) {
    if (!t) return PWC_OK;
    pwc::free_table(t->t);
    delete t;
    return PWC_OK;
}

pwc_status pwc_table_info(const pwc_table *t, int64_t *N, int *nmax, int *n_nodes,
                          size_t *device_bytes) {
    if (!t) return PWC_ERR_ARG;
    if (N) *N = t->t.N;
    if (nmax) *nmax = t->t.nmax;
    if (n_nodes) *n_nodes = t->t.Q;
    if (device_bytes) *device_bytes = t->t.bytes + t->t.val_bytes;
    return PWC_OK;
}

pwc_status pwc_mesh_build(const pwc_mesh *mesh, double L, double *h_beta, double *h_W) {
    if (!mesh || !(L > 0.0) || !std::isfinite(L) || !h_beta || !h_W) return PWC_ERR_ARG;
    std::vector<double> beta, W;
    int n1 = 0;
    if (!pwc::build_mesh(*mesh, L, beta, W, &n1)) return PWC_ERR_ARG;
    std::copy(beta.begin(), beta.end(), h_beta);
    std::copy(W.begin(), W.end(), h_W);
    return PWC_OK;
}

pwc_status pwc_basis_enumerate(int n2max, int32_t *h_n, int64_t *N) {
    if (n2max < 1 || n2max > PWC_MAX_N2MAX || !N) return PWC_ERR_ARG;
    const auto b = pwc::enumerate_basis(n2max);
    *N = static_cast<int64_t>(b->packed.size());
    if (h_n) std::copy(b->n.begin(), b->n.end(), h_n);
    return PWC_OK;
}

pwc_status pwc_table_build_values(pwc_table *t, void *stream) {
    if (!t || t->t.gauss) return PWC_ERR_ARG;
    pwc::Table &tb = t->t;
    if (tb.d_val) return PWC_OK;
    const size_t bytes = sizeof(double) * static_cast<size_t>(pwc::value_count(tb));
    void *d = nullptr;
    size_t got = 0;
    if (pwc::dev_alloc(bytes, &d, &got) != hipSuccess) {
        (void)hipGetLastError();
        return PWC_ERR_NOMEM;
    }
    const hipStream_t s = static_cast<hipStream_t>(stream);
    // Stream-ordered: work queued after this call on `stream` sees the values.
    hipError_t err = pwc::wait_ready(tb, s);
    // Test-only switch: start from a block of NaN (all bits set), so that a
    // value the build fails to write cannot pass for one an earlier table
    // left in a recycled block.
    const char *poison = std::getenv("PWC_TEST_POISON_VALUES");
    if (err == hipSuccess && poison && poison[0] && std::strcmp(poison, "0") != 0)
        err = hipMemsetAsync(d, 0xff, bytes, s);
    if (err == hipSuccess) err = pwc::launch_values_build(tb, static_cast<double *>(d), s);
    if (err != hipSuccess) {
        (void)hipStreamSynchronize(s);
        pwc::dev_release(d, got);
        return from_hip(err);
    }
    pwc::note_use(tb, s);
    tb.d_val = static_cast<double *>(d);
    tb.val_bytes = bytes;
    tb.val_alloc = got;
    return PWC_OK;
}

pwc_status pwc_table_values_info(const pwc_table *t, int *built, size_t *bytes) {
    if (!t) return PWC_ERR_ARG;
    if (built) *built = t->t.d_val != nullptr;
    if (bytes) *bytes = t->t.gauss ? 0 : sizeof(double) * static_cast<size_t>(pwc::value_count(t->t));
    return PWC_OK;
}

pwc_status pwc_table_free_values(pwc_table *t) {
    if (!t) return PWC_ERR_ARG;
    pwc::dev_release(t->t.d_val, t->t.val_alloc);
    t->t.d_val = nullptr;
    t->t.val_bytes = t->t.val_alloc = 0;
    return PWC_OK;
}

pwc_status pwc_release_cached_memory(void) {
    (void)hipDeviceSynchronize();
    {
        std::lock_guard<std::mutex> lk(pwc::g_cache_mu);
        pwc::release_cached(-1);
    }
    pwc::release_stages();
    pwc::release_value_plans();
    return PWC_OK;
}

pwc_status pwc_table_layout(const pwc_table *t, pwc_precision p, int *lanes, int *words,
                            int *nodes_per_pass, int *passes, int *entry_bytes) {
    if (!t || t->t.gauss || !pwc::valid_precision(p)) return PWC_ERR_ARG;
    const pwc::FoldLayout &fl = p == PWC_MIXED ? t->t.flm : p == PWC_FP32 ? t->t.fls : t->t.fl;
    if (lanes) *lanes = fl.G;
    if (words) *words = fl.W;
    if (nodes_per_pass) *nodes_per_pass = fl.c;
    if (passes) *passes = fl.nchunk;
    if (entry_bytes) *entry_bytes = pwc::packed_entry_bytes(fl.E);
    return PWC_OK;
}

pwc_status pwc_table_fused(const pwc_table *t, pwc_precision p, int *fused) {
    if (!t || t->t.gauss || !fused || !pwc::valid_precision(p)) return PWC_ERR_ARG;
    const pwc::FoldLayout &fl = p == PWC_MIXED ? t->t.flm : p == PWC_FP32 ? t->t.fls : t->t.fl;
    *fused = pwc::fused_layout(fl, pwc::fold_maps_bytes(t->t.N, t->t.nd)) ? 1 : 0;
    return PWC_OK;
}

pwc_status pwc_table_set_layout(pwc_table *t, int lanes, int words) {
    if (!t || t->t.gauss) return PWC_ERR_ARG;
    if (lanes == 0 && words != 0) return PWC_ERR_ARG;
    if (lanes != 0) {
        const bool ok = (lanes == 16 && words == 1) || ((lanes == 8 || lanes == 4) && (words == 1 || words == 2)) ||
                        (lanes == 2 && words == 4) || (lanes == 1 && words == 8);
        if (!ok) return PWC_ERR_ARG;
    }
    pwc::FoldLayout fl = t->t.fl, flm = t->t.flm, fls = t->t.fls;
    const size_t maps = pwc::fold_maps_bytes(t->t.N, t->t.nd);
    if (!pwc::plan_fold(t->t.Q, t->t.fl.E, lanes, words, PWC_FP64, maps, fl) ||
        !pwc::plan_fold(t->t.Q, t->t.fl.E, lanes, words, PWC_MIXED, maps, flm))
        return PWC_ERR_RANGE;
    // FP32 passes cover twice the nodes; a layout whose passes would run past
    // the padded rows leaves FP32 on its default choice.
    if (!pwc::plan_fold(t->t.Q, t->t.fl.E, lanes, words, PWC_FP32, maps, fls) &&
        !pwc::plan_fold(t->t.Q, t->t.fl.E, 0, 0, PWC_FP32, maps, fls))
        return PWC_ERR_RANGE;
    t->t.fl = fl;
    t->t.flm = flm;
    t->t.fls = fls;
    return PWC_OK;
}

pwc_status pwc_table_params(const pwc_table *t, double *L, int *n2max, pwc_mesh *mesh) {
    if (!t) return PWC_ERR_ARG;
    if (L) *L = t->t.L;
    if (n2max) *n2max = t->t.n2max;
    if (mesh) *mesh = t->t.mesh;
    return PWC_OK;
}

pwc_status pwc_table_box(const pwc_table *t, double *sides) {
    if (!t || !sides) return PWC_ERR_ARG;
    for (int d = 0; d < 3; ++d) sides[d] = t->t.Ld[d];
    return PWC_OK;
}

pwc_status pwc_basis(const pwc_table *t, int32_t *h_n) {
    if (!t || !h_n || t->t.gauss) return PWC_ERR_ARG;
    std::memcpy(h_n, t->t.h_basis->n.data(), sizeof(int32_t) * t->t.h_basis->n.size());
    return PWC_OK;
}

pwc_status pwc_mesh_nodes(const pwc_table *t, double *h_beta, double *h_W) {
    if (!t || !h_beta || !h_W) return PWC_ERR_ARG;
    std::memcpy(h_beta, t->t.h_beta.data(), sizeof(double) * t->t.Q);
    std::memcpy(h_W, t->t.h_W.data(), sizeof(double) * t->t.Q);
    return PWC_OK;
}

pwc_status pwc_table_copy(const pwc_table *t, double *d_dst, void *stream) {
    if (!t || !d_dst) return PWC_ERR_ARG;
    // [ndir][Q][nd][nd]; a Gaussian table: [Q][P1][P1] (nd = P1, ndir = 1)
    const size_t bytes = sizeof(double) * t->t.ndir * t->t.Q * t->t.nd * t->t.nd;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = pwc::wait_ready(t->t, s);
    if (e != hipSuccess) return from_hip(e);
    e = hipMemcpyAsync(d_dst, t->t.d_tau, bytes, hipMemcpyDeviceToDevice, s);
    pwc::note_use(t->t, s);
    return from_hip(e);
}

pwc_status pwc_reconstruct(const pwc_table *t, const int32_t *d_quads, int64_t n, double *d_out,
                           pwc_precision p, void *stream) {
    if (!t || n < 0 || !pwc::valid_precision(p) || (p == PWC_FP32 && t->t.gauss)) return PWC_ERR_ARG;
    if (n == 0) return PWC_OK;
    if (!d_quads || !d_out) return PWC_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(d_quads) & 15) || (reinterpret_cast<uintptr_t>(d_out) & 7))
        return PWC_ERR_ARG;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = pwc::wait_ready(t->t, s);
    if (e != hipSuccess) return from_hip(e);
    if (t->t.gauss) {                    // separable Gaussians: rows from global memory
        e = pwc::launch_rec_gauss(t->t, d_quads, n, d_out, p, s);
    } else if (t->t.d_val && p == PWC_FP64) {   // every distinct value is at hand: one read each
        e = pwc::launch_rec_values(t->t, d_quads, n, d_out, s);
    } else if (n <= t->t.direct_max) {   // small list: four lanes per quadruple, no node passes
        pwc::DirectBatch b{};
        b.job[0] = pwc::direct_job(t->t, d_quads, n, d_out, p, nullptr);
        b.njobs = 1;
        e = pwc::launch_direct(b, s);
    } else {
        e = pwc::launch_reconstruct(t->t, d_quads, n, d_out, p, s);
    }
    pwc::note_use(t->t, s);
    return from_hip(e);
}

pwc_status pwc_reconstruct_noalloc(const pwc_table *t, const int32_t *d_quads, int64_t n,
                                   double *d_out, pwc_precision p, void *stream) {
    if (!t || t->t.gauss || n < 0 || !pwc::valid_precision(p)) return PWC_ERR_ARG;
    if (n > PWC_NOALLOC_MAX_QUADS) return PWC_ERR_LIMIT;
    if (n == 0) return PWC_OK;
    if (!d_quads || !d_out) return PWC_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(d_quads) & 15) || (reinterpret_cast<uintptr_t>(d_out) & 7))
        return PWC_ERR_ARG;
    if (pwc::reconstruct_scratch_bytes(t->t, n, p) > pwc::kNoAllocScratchBytes) return PWC_ERR_LIMIT;
    void *scratch = nullptr;
    hipError_t e = pwc::noalloc_scratch(&scratch);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    if (e == hipSuccess) e = pwc::wait_ready(t->t, s);
    if (e == hipSuccess) e = pwc::launch_reconstruct(t->t, d_quads, n, d_out, p, s, nullptr, nullptr, scratch);
    pwc::note_use(t->t, s, false);   // re-records an existing event, creates none
    return from_hip(e);
}

pwc_status pwc_table_set_direct_max(pwc_table *t, int64_t n) {
    if (!t || n < 0 || n > pwc::kDirectMaxN) return PWC_ERR_ARG;
    t->t.direct_max = n;
    return PWC_OK;
}

pwc_status pwc_reconstruct_profile(const pwc_table *t, const int32_t *d_quads, int64_t n,
                                   double *d_out, pwc_precision p, void *stream, double *h_ms,
                                   int max_stages, int *n_stages) {
    if (!t || t->t.gauss || !h_ms || !n_stages || n <= 0 || !pwc::valid_precision(p)) return PWC_ERR_ARG;
    if (!d_quads || !d_out) return PWC_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(d_quads) & 15) || (reinterpret_cast<uintptr_t>(d_out) & 7))
        return PWC_ERR_ARG;
    const int stages = 1 + (p == PWC_MIXED ? t->t.flm : p == PWC_FP32 ? t->t.fls : t->t.fl).nchunk;
    *n_stages = stages;
    if (max_stages < stages) return PWC_ERR_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<hipEvent_t> ev(stages + 1, nullptr);
    hipError_t e = pwc::wait_ready(t->t, s);
    for (auto &x : ev)
        if (e == hipSuccess) e = hipEventCreate(&x);
    if (e == hipSuccess) e = pwc::launch_reconstruct(t->t, d_quads, n, d_out, p, s, ev.data());
    pwc::note_use(t->t, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    for (int k = 0; k < stages && e == hipSuccess; ++k) {
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
        h_ms[k] = ms;
    }
    for (auto &x : ev)
        if (x) (void)hipEventDestroy(x);
    return from_hip(e);
}

pwc_status pwc_energies_ex(const pwc_table *t, const int32_t *d_occ, const double *d_f,
                           int64_t M, pwc_precision p, pwc_pair_algo algo, double *d_out,
                           void *stream) {
    if (!t || t->t.gauss || !d_out || M < 0 || (p != PWC_FP64 && p != PWC_MIXED)) return PWC_ERR_ARG;
    if (algo != PWC_PAIR_AUTO && algo != PWC_PAIR_NODESUM && algo != PWC_PAIR_KTABLE)
        return PWC_ERR_ARG;
    if (algo == PWC_PAIR_KTABLE && t->t.kt_n == 0) return PWC_ERR_ARG;
    if (M > 0 && !d_occ) return PWC_ERR_ARG;
    if (M > (1 << 17)) return PWC_ERR_ARG;   // pair-tile grid (M/32)^2 workgroups
    if ((reinterpret_cast<uintptr_t>(d_out) & 7) || (d_f && (reinterpret_cast<uintptr_t>(d_f) & 7)))
        return PWC_ERR_ARG;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = pwc::wait_ready(t->t, s);
    if (e != hipSuccess) return from_hip(e);
    e = pwc::launch_energies(t->t, d_occ, d_f, M, p, algo, d_out, s);
    pwc::note_use(t->t, s);
    return from_hip(e);
}

pwc_status pwc_energies_async(const pwc_table *t, const int32_t *d_occ, const double *d_f,
                              int64_t M, pwc_precision p, double *d_out, void *stream) {
    return pwc_energies_ex(t, d_occ, d_f, M, p, PWC_PAIR_AUTO, d_out, stream);
}

pwc_status pwc_energies(const pwc_table *t, const int32_t *d_occ, const double *d_f, int64_t M,
                        pwc_precision p, double *h_out, void *stream) {
    if (!t || !h_out) return PWC_ERR_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    double *d_out = nullptr;
    hipError_t e = hipMallocAsync(reinterpret_cast<void **>(&d_out), 2 * sizeof(double), s);
    if (e != hipSuccess) return from_hip(e);
    pwc_status st = pwc_energies_async(t, d_occ, d_f, M, p, d_out, stream);
    if (st == PWC_OK) st = from_hip(hipMemcpyAsync(h_out, d_out, 2 * sizeof(double),
                                                   hipMemcpyDeviceToHost, s));
    (void)hipFreeAsync(d_out, s);
    const pwc_status st2 = from_hip(hipStreamSynchronize(s));
    if (st != PWC_OK) return st;
    if (st2 != PWC_OK) return st2;
    return pwc_sync(t, stream);
}

pwc_status pwc_sync(const pwc_table *t, void *stream) {
    if (!t) return PWC_ERR_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int flag = 0;
    hipError_t e = pwc::wait_ready(t->t, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&flag, t->t.d_err, sizeof(int), hipMemcpyDeviceToHost, s);
    pwc::note_use(t->t, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return from_hip(e);
    if (flag) {
        const int zero = 0;
        e = hipMemcpyAsync(t->t.d_err, &zero, sizeof(int), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return from_hip(e);
        return PWC_ERR_RANGE;
    }
    return PWC_OK;
}

}  // extern "C"
