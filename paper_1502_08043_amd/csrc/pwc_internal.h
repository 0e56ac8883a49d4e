// Internal declarations shared by the host API and the HIP kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <memory>
#include <mutex>
#include <utility>
#include <vector>

#include "pwcoul.h"

namespace pwc {

// ---------------------------------------------------------------- host ----

// Canonical planewave basis |n|^2 <= n2max, ascending (|n|^2, nx, ny, nz):
// n [N][3], and each vector packed into one int32 (x, y, z in bytes 0..2, as
// the kernels read it).  Formed once per cutoff and shared.
struct Basis {
    std::vector<int32_t> n;
    std::vector<int32_t> packed;
};
std::shared_ptr<const Basis> enumerate_basis(int n2max);

// q-point Gauss-Legendre rule on [a, b] (Newton iteration on the Legendre
// three-term recurrence), nodes ascending.
void gauss_legendre(int q, double a, double b, std::vector<double> &x, std::vector<double> &w);

// Quadrature nodes and weights in beta = 4 alpha / L^2 for a mesh; also
// returns how many leading nodes lie in interval 1.  false if invalid.
bool build_mesh(const pwc_mesh &m, double L, std::vector<double> &beta,
                std::vector<double> &W, int *n_interval1);

bool mesh_valid(const pwc_mesh &m, int *n_nodes);

// Symmetry fold of the (m, m') plane: tau(m, m') = tau(m', m) = tau(-m, -m').
// fold[(m + K) * nd + (m' + K)] = index of the orbit representative, and
// reps[2 * e], reps[2 * e + 1] = (m, m') of representative e.
void build_fold(int K, std::vector<int32_t> &fold, std::vector<int32_t> &reps);

// ------------------------------------------------------------- kernels ----

// LDS budget of one pair-sum workgroup (diagonal-table chunk).
constexpr int kLdsBudget = 80 * 1024;
constexpr int kGlPanelPoints = 16;    // Gauss-Legendre points per panel
constexpr int kGlPanels = 128;        // panels over the Gaussian's support

// Folded-table layout of the reconstruction kernels (see reconstruct_kernels.hip):
// P node passes of c = 2 G W nodes each, G lanes per quadruple with W
// 16-byte words each; the [E][c] FP64 slab of one pass must fit in one
// workgroup's LDS.
struct FoldLayout {
    int E = 0;          // folded entries per node
    int Qp = 0;         // nodes padded to a multiple of 32 (zero weight, zero tau)
    int G = 0;          // lanes per quadruple: 1 .. 16
    int W = 0;          // 16-byte words per lane and row: 1 .. 8
    int c = 0;          // nodes per pass, npw G W (npw = 2 nodes per word, 4 for FP32)
    int nchunk = 0;     // passes P = ceil(Q / c)
};
// A kernel that meets a bad index sets its error word to 1 and never reads
// it: a plain store at system scope, since the word may be mapped host
// memory (the server's), where read-modify-write atomics would need PCIe
// atomics.
__device__ __forceinline__ void raise_error(int *err) {
    __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
// Nodes in one 16-byte word of the folded table of precision p.
inline int nodes_per_word(pwc_precision p) { return p == PWC_FP32 ? 4 : 2; }
inline bool valid_precision(int p) { return p == PWC_FP64 || p == PWC_MIXED || p == PWC_FP32; }
constexpr int kLdsMax = 160 * 1024;          // LDS per workgroup on gfx950
// LDS bytes of the decode's basis (int32 per planewave) and fold map (int16
// per (m, m') pair).
inline size_t fold_maps_bytes(int64_t N, int nd) {
    return sizeof(int32_t) * static_cast<size_t>(N) + sizeof(int16_t) * static_cast<size_t>(nd) * nd;
}
// Quadruples per lane in a chunk of the fused launch (1024 lanes): as many as
// fit in registers beside the staged slab words, 8 beside 6 words per lane,
// 6 beside 8.
inline int fused_chunk_quads(int E) { return E * 8 <= 6 * 1024 ? 8 : 6; }
// LDS area in front of the decode maps in the fused launch: the slab, and
// with several node ranges at least the exchange area of the wave-wide
// pairing (8 bytes per quadruple of a chunk), which reuses it.
inline size_t fused_area_bytes(const FoldLayout &fl) {
    const size_t slab = static_cast<size_t>(fl.E) * 128;
    const size_t xchg = static_cast<size_t>(1024) * fused_chunk_quads(fl.E) * 8;
    return fl.nchunk > 1 ? std::max(slab, xchg) : slab;
}
// True when a reconstruction with layout fl runs as one fused launch: the
// one-lane layout (1 lane, 8 words of 16 bytes per row), its slab (or the
// exchange area) and the decode maps together in one workgroup's LDS, at
// most 8 slab words staged per lane.  It keeps no decoded stream.
inline bool fused_layout(const FoldLayout &fl, size_t maps_bytes) {
    return fl.G == 1 && fl.W == 8 && fl.E <= 1024 &&
           fused_area_bytes(fl) + maps_bytes <= static_cast<size_t>(kLdsMax);
}
constexpr int kGaussMaxN1 = PWC_GAUSS_MAX_N1;
constexpr int kGaussMaxPairs = PWC_GAUSS_MAX_PAIRS;
constexpr int64_t kRecSlab = int64_t(1) << 27;   // quadruples per scratch slab

struct DiagLayout {
    int c = 0;        // nodes per LDS chunk of the diagonal table
    int nchunk = 0;
};

// The streams that queued work reading or writing a table's device memory:
// one event per stream, recorded again after each use.  When the table is
// released, its blocks wait for these events (not for the whole device)
// before another table may reuse them.  A stream under graph capture, or
// more than kMaxUseStreams streams, sets `overflow` and the release waits
// for the device instead.
struct UseLog {
    std::mutex mu;
    std::vector<std::pair<hipStream_t, hipEvent_t>> ev;
    bool overflow = false;
};
constexpr int kMaxUseStreams = 32;

struct Table {
    // Box sides (a cube has three equal sides).  L is the reference length:
    // the side of a cube, (Lx Ly Lz)^(1/3) for a box; direction d of a box
    // uses the node beta / rho_d^2, rho_d = L_d / L, and its own tables.
    double L = 0.0;
    double Ld[3] = {0.0, 0.0, 0.0};
    double rho[3] = {1.0, 1.0, 1.0};
    int ndir = 1;                   // direction tables: 1 (cube) or 3 (box)
    int E1 = 0;                     // folded entries per direction and node
    int n2max = 0, nmax = 0, K = 0, nd = 0, Q = 0;
    int64_t N = 0;
    int n_interval1 = 0;
    pwc_mesh mesh{};
    std::shared_ptr<const Basis> h_basis;
    std::vector<double> h_beta, h_W;
    FoldLayout fl;       // reconstruction layout of the FP64 path
    FoldLayout flm;      // and of the split-FP32 path (same E, Qp)
    FoldLayout fls;      // and of the single-FP32 path (4 nodes per 16-byte word)
    DiagLayout dl;
    int device = 0;
    int n_cu = 0;

    // device memory (one allocation, carved)
    void *d_block = nullptr;
    size_t bytes = 0;
    int32_t *d_basis = nullptr;     // [N] packed (x, y, z) as int8 lanes of an int32
    int32_t *d_fold = nullptr;      // [nd * nd]
    int32_t *d_reps = nullptr;      // [E][2]
    double *d_beta = nullptr;       // [ndir][Q] node of each direction
    double *d_W = nullptr;          // [Q]
    double *d_gl = nullptr;         // [2][kGlPanelPoints] panel rule on [0, 1]
    double *d_prim = nullptr;       // [ndir][Q][2][K + 1]  (S, D)
    double *d_tau = nullptr;        // [ndir][Q][nd][nd]
    double *d_tauF = nullptr;       // [ndir * E1][Qp]  folded W_q^(1/3) tau_q, FP64
    float2 *d_tauHL = nullptr;      // [ndir * E1][Qp]  same, (hi, lo)
    float *d_tau32 = nullptr;       // [ndir * E1][Qp]  same, rounded to FP32
    double *d_Wcbrt = nullptr;      // [Q]      W_q^(1/3)
    double *d_diag = nullptr;       // [dl.nchunk][ndir][K + 1][dl.c]  tau_q(m, -m), m >= 0
    float2 *d_diagHL = nullptr;     // same, (hi, lo)
    double *d_Wdiag = nullptr;      // [dl.nchunk * dl.c]
    float2 *d_WdiagHL = nullptr;
    int64_t direct_max = 0;         // pwc_reconstruct takes the direct kernel for n <= this
    int kt_n = 0;                   // exchange kernel table size: C(K+3, 3) for a cube
                                    // (a <= b <= c), (K+1)^3 for a box; 0 if not kept
    double *d_ktab64 = nullptr;     // [kt_n] K(a, b, c), FP64 node sums
    double *d_ktabMX = nullptr;     // [kt_n] same, split-FP32 node sums
    int *d_err = nullptr;           // kernel error word
    // Value table (pwc_table_build_values): every distinct integral, FP64,
    // its own allocation; nullptr until built.
    double *d_val = nullptr;
    size_t val_bytes = 0;
    size_t val_alloc = 0;           // bytes of the block holding the values (may be larger)
    size_t block_bytes = 0;         // bytes of the block holding d_block
    // Recorded on the creating stream after the table kernels; every call
    // that queues work on a stream waits for it first (wait_ready), so a
    // table may be used on any stream as soon as pwc_table_create returns.
    hipEvent_t ready = nullptr;
    std::shared_ptr<const std::vector<char>> h_img;   // upload source, alive until destroy
    std::shared_ptr<UseLog> uses;   // created by build_table
    // Separable Gaussian basis (pwc_table_create_gauss): the same node sums
    // over a table of kept one-dimensional pair products.  Fields of the
    // planewave layout that a Gaussian table does not use stay empty.
    bool gauss = false;
    int n1 = 0, P1 = 0;             // functions per direction, kept pairs
    double eps = 0.0;               // pair screening threshold
    std::vector<int32_t> h_pmap;    // [n1][n1] pair index or -1
    std::vector<double> h_pair;     // [P1][3] (c, p, P)
    int32_t *d_pmap = nullptr;
    double *d_pair = nullptr;
};

// Record that work on the table's memory was queued on stream s (after the
// launches): the table's release then waits for it.  With may_create false
// no event is created: a stream without one marks the log incomplete (the
// release then waits for the device) -- for callers that cannot allocate.
void note_use(const Table &t, hipStream_t s, bool may_create = true);

// Order work queued next on stream s after the table's construction.
inline hipError_t wait_ready(const Table &t, hipStream_t s) {
    return t.ready ? hipStreamWaitEvent(s, t.ready, 0) : hipSuccess;
}

// api.cpp: table set-up in two phases.  plan_table forms the basis, mesh,
// fold map and layouts on the host and sets t.bytes; build_table allocates,
// uploads and queues the table kernels on the stream and records t.ready
// (a loaded table, whose FP64 tables come from the caller's buffer, also
// waits for the stream).
struct TableSetup {
    std::vector<int32_t> fold, reps;
};
// maps_bytes: fold_maps_bytes of the table (the one-lane layout is priced
// as the fused schedule when it qualifies).
bool plan_fold(int Q, int E, int lanes, int words, pwc_precision p, size_t maps_bytes, FoldLayout &fl);
pwc_status plan_table(const double sides[3], int n2max, const pwc_mesh &m, Table &t, TableSetup &su);
// h_tau: the FP64 tables [Q][nd][nd] of a loaded table (the 1-D integrals are
// then not recomputed), or nullptr.
pwc_status build_table(Table &t, const TableSetup &su, hipStream_t s, const double *h_tau = nullptr);
void free_table(Table &t);
// Device blocks of tables and value tables, through a small per-device cache
// of released blocks.  A block released with an event set is reused only
// once every event of the set has completed; without one, dev_release waits
// for the device first.
struct EventSet;
hipError_t dev_alloc(size_t bytes, void **p, size_t *got);
void dev_release(void *p, size_t bytes, EventSet *es = nullptr);

// table_kernels.hip
hipError_t launch_table_build(Table &t, hipStream_t s, bool from_tau);
// gauss_kernels.hip: the Gaussian tables (full [Q][P1][P1], folded rows with
// W^(1/3), split FP32) and the reconstruction from them.
hipError_t launch_gauss_tables(const Table &t, hipStream_t s);
hipError_t launch_rec_gauss(const Table &t, const int32_t *d_quads, int64_t n, double *d_out,
                            pwc_precision p, hipStream_t s, int *d_err = nullptr);
// reconstruct_kernels.hip
// Bytes of one decoded quadruple in the scratch stream (4 when E <= 1024).
int packed_entry_bytes(int E);
// stage_ev: optional array of nchunk + 2 events (decode start, decode end,
// end of every node pass), recorded for the first slab.
// Every launch_* that checks indices raises d_err when given, else the
// table's own error word.
// d_scratch: a caller-owned buffer for the decoded stream of at least
// reconstruct_scratch_bytes(t, n, p) bytes, or nullptr (a stream-ordered
// allocation per call, none for the fused schedule).
hipError_t launch_reconstruct(const Table &t, const int32_t *d_quads, int64_t n,
                              double *d_out, pwc_precision p, hipStream_t s,
                              hipEvent_t *stage_ev = nullptr, int *d_err = nullptr,
                              void *d_scratch = nullptr);
// Device bytes of the decoded stream of one node-pass call of n quadruples
// in precision p (0 when it runs fused).
size_t reconstruct_scratch_bytes(const Table &t, int64_t n, pwc_precision p);
// pwc_reconstruct_noalloc's fixed scratch: kNoAllocScratchBytes of static
// device memory per device; *p is its address on the current device (looked
// up once per device).  Holds the padded decoded stream of
// PWC_NOALLOC_MAX_QUADS quadruples at 8 bytes each.
constexpr size_t kNoAllocScratchBytes = size_t(8) * PWC_NOALLOC_MAX_QUADS;
hipError_t noalloc_scratch(void **p);
// direct_kernels.hip: small quadruple lists, up to kDirectMaxJobs requests
// (any tables and precisions) per launch, jobs passed by value.
struct DirectJob {
    const int32_t *quads;     // [n][4]
    double *out;              // [n]
    int64_t n;
    const void *tab;          // folded W^(1/3) tau [E][Qp], double or float2
    const int32_t *basis;
    const int32_t *fold;
    int *err;                 // error word of this job
    double pref;
    int N, K, nd, Qp, Q, mixed;  // mixed: 0 FP64, 1 split FP32, 2 single FP32
    int ystride;              // rows between direction tables (E1 for a box, 0 for a cube)
    uint32_t block0;          // first block of the job (set by launch_direct)
};
constexpr int kDirectMaxJobs = 24;
constexpr int64_t kDirectDefault = int64_t(1) << 19;  // direct-kernel threshold of tables with fused node sums
constexpr int64_t kDirectMaxN = int64_t(1) << 20;   // quadruples per job
struct DirectBatch {
    DirectJob job[kDirectMaxJobs];
    int njobs;
};
DirectJob direct_job(const Table &t, const int32_t *d_quads, int64_t n, double *d_out,
                     pwc_precision p, int *d_err);
hipError_t launch_direct(DirectBatch b, hipStream_t s);
// value_kernels.hip: the value table (E (E + 1) (E + 2) / 6 sorted entry
// triples of a cube, E1^3 triples of a box) and the reconstruction that reads it.
int64_t value_count(const Table &t);
hipError_t launch_values_build(const Table &t, double *d_val, hipStream_t s);
void release_value_plans();   // the build's cached block lists (after a device wait)
// The c tiles of the build's pair tile pt (so[f] = m^2 + m'^2 of orbit f,
// ascending): n tiles of 64 c from c_lo, covering every value of its pairs
// that a quadruple can reach.
void value_tile_c_range(const int *so, int E1, bool box, int smax, int64_t pt, int *c_lo, int *n);
hipError_t launch_rec_values(const Table &t, const int32_t *d_quads, int64_t n, double *d_out,
                             hipStream_t s);
// pairsum_kernels.hip
hipError_t launch_ktab_build(Table &t, hipStream_t s);
// Device bytes launch_energies allocates for its partial sums.
size_t energies_scratch_bytes(const Table &t, int64_t M, pwc_pair_algo algo);
hipError_t launch_energies(const Table &t, const int32_t *d_occ, const double *d_f,
                           int64_t M, pwc_precision p, pwc_pair_algo algo, double *d_out,
                           hipStream_t s, int *d_err = nullptr);

}  // namespace pwc

struct pwc_table {
    pwc::Table t;
};
