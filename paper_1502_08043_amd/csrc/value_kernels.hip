// Value table: every distinct integral of a table, each evaluated once.
//
// <ij|kl> depends on the quadruple only through the three folded entries
// (one per direction) that the decode finds (Sec. III: planewave products
// are planewaves, so only index differences matter, and tau is symmetric
// under (m, m') -> (m', m) and (m, m') -> (-m, -m')).  For a cube the three
// entries are interchangeable, so the integral is a function of the sorted
// triple a <= b <= c of entry numbers:
//   V(a, b, c) = (1/(sqrt(pi) L)) sum_q T_q(a) T_q(b) T_q(c),
// T_q = W_q^(1/3) tau_q, which is Eq. 14 for any quadruple with those
// entries.  There are E (E + 1) (E + 2) / 6 such triples: 6.5e7 (0.52 GB in
// FP64) for the 9171-planewave basis, against N^4 = 7e15 integrals.  A box
// reads one table per direction and keeps every (x, y, z) triple, E1^3
// values.
//
// Layout.  Pairs (a, b) are numbered p = b (b + 1) / 2 + a (a <= b; a box
// uses p = a E1 + b), and V(a, b, c) sits at c (c + 1) (c + 2) / 6 + p (a box:
// c E1^2 + p): for each c the pairs are contiguous.
//
// Build.  For fixed c the values are a matrix product: V[p][c] =
// sum_q P_q(p) T_q(c) with P_q(p) = T_q(a) T_q(b).  A workgroup takes 128
// pairs and 64 values of c, stages 8 nodes of P and T at a time in LDS and
// runs the node sums on the FP64 matrix cores, four nodes per step in node
// order; the next chunk's rows are read into registers while they work.
// Short chunks keep the registers at four waves per SIMD, which the
// matrix cores need to stay busy across the barriers.  Only the values a
// quadruple of the basis can read are computed: a cube keeps c >= b, and
// with m = n_k - n_i and m' = n_l - n_j, |m|^2 + |m'|^2 <= 8 n2max, which is
// the total of the three orbits' m^2 + m'^2.  Each tile of 128 pairs takes
// the 64-wide c tiles from its smallest b up to the largest c one of its
// pairs can reach; the list of (pair tile, c tile) blocks depends only on
// the cutoff and the shape and is formed once.  Other entries of the table
// are left unwritten.
//
// Reconstruction.  Decode each quadruple (basis and fold map in LDS), sort
// the cube's entries, read one value.  HBM traffic per quadruple: 16 bytes
// of indices, 8 of the value, 8 out.  Orbits are numbered by ascending
// m^2 + m'^2, so the values a stream reads most sit in the table's first
// megabytes and mostly hit in L2; the quadruple and output streams are
// loaded and stored non-temporally so that they do not evict them.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>

#include "pwc_internal.h"

namespace pwc {
namespace {

constexpr int kVbThreads = 256;
constexpr int kVbTile = 64;      // values of c per block
constexpr int kVbTileP = 128;    // pairs per block
constexpr int kVbChunk = 8;      // nodes per LDS stage

struct ValBuildArgs {
    const double *tab;    // [rows][Qp] folded W^(1/3) tau (a box: x, y, z tables stacked)
    int Qp;
    int E1;
    int box;
    int64_t npairs;
    // Block i takes pair tile pt = desc[i] & 0xffffff (pairs 128 pt ..
    // 128 pt + 127) and its c tile k = desc[i] >> 24, the 64 values of c from
    // c_lo + 64 k, c_lo the smallest b of its pairs (0 for a box); only the
    // tiles value_tile_c_range keeps have a block.
    const uint32_t *desc;
    double pref;
    double *val;
};

__host__ __device__ inline int64_t tri2(int64_t b) { return b * (b + 1) / 2; }
__device__ __forceinline__ int64_t tri3(int64_t c) { return c * (c + 1) * (c + 2) / 6; }

// The b of pair p (cube numbering p = b (b + 1) / 2 + a, 0 <= a <= b).
__host__ __device__ inline int pair_b(int64_t p) {
    int b = static_cast<int>((sqrt(8.0 * static_cast<double>(p) + 1.0) - 1.0) * 0.5);
    while (tri2(b + 1) <= p) ++b;       // guard the rounding of the square root
    while (tri2(b) > p) --b;
    return b;
}

using f64x4 = double __attribute__((ext_vector_type(4)));


// Each of the block's four waves computes 32 values of c by 64 pairs as
// 2 x 4 tiles of v_mfma_f64_16x16x4f64, D[i][j] += sum_k A[i][k] B[k][j]
// over 4 nodes k per step: A = T rows of c (i), B = pair products of p (j).
// Lane l feeds A[l % 16][l / 16] and B[l / 16][l % 16] and receives
// D[4 r + l / 16][l % 16] in register r = 0..3: each output register of a
// 16-lane group covers 16 consecutive pairs of one c, contiguous in the
// table.
__global__ __launch_bounds__(kVbThreads, 4) void k_values_build(ValBuildArgs a) {
    __shared__ double Ps[kVbChunk][kVbTileP];
    __shared__ double Cs[kVbChunk][kVbTile];
    const uint32_t d = a.desc[blockIdx.x];
    const int64_t p0 = static_cast<int64_t>(d & 0xffffffu) * kVbTileP;
    const int c0 = (a.box ? 0 : pair_b(p0)) + static_cast<int>(d >> 24) * kVbTile;
    const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    const int wp = (wave & 1) * 64, wc = (wave >> 1) * 32;
    const int li = lane % 16, lk = lane / 16;

    // Staging roles for each chunk: lane tid forms the products of pair
    // sp = tid / 2 at nodes sq .. sq + 3, sq = (tid % 2) * 4, and copies row
    // sc = tid / 4 of the c tile at nodes scq, scq + 1, scq = (tid % 4) * 2.
    const int sp = tid / 2, sq = (tid % 2) * 4;
    const int sc = tid / 4, scq = (tid % 4) * 2;
    const int64_t myp = p0 + sp;
    const double *ra = nullptr, *rb = nullptr, *rc = nullptr;
    if (myp < a.npairs) {
        int pa, pb;
        if (a.box) {
            pa = static_cast<int>(myp / a.E1);
            pb = a.E1 + static_cast<int>(myp % a.E1);
        } else {
            pb = pair_b(myp);
            pa = static_cast<int>(myp - tri2(pb));
        }
        ra = a.tab + static_cast<size_t>(pa) * a.Qp;
        rb = a.tab + static_cast<size_t>(pb) * a.Qp;
    }
    if (c0 + sc >= 0 && c0 + sc < a.E1) rc = a.tab + static_cast<size_t>((a.box ? 2 * a.E1 : 0) + c0 + sc) * a.Qp;

    f64x4 acc[2][4];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = f64x4{0.0, 0.0, 0.0, 0.0};

    // The next chunk's rows are loaded into registers (16-byte reads) while
    // the matrix cores work on the current one.
    double2 xa[2], xb[2], xc;
    auto fetch = [&](int q0) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int q = q0 + sq + 2 * k;
            xa[k] = ra ? *reinterpret_cast<const double2 *>(ra + q) : double2{0.0, 0.0};
            xb[k] = ra ? *reinterpret_cast<const double2 *>(rb + q) : double2{0.0, 0.0};
        }
        xc = rc ? *reinterpret_cast<const double2 *>(rc + q0 + scq) : double2{0.0, 0.0};
    };
    fetch(0);
    for (int q0 = 0; q0 < a.Qp; q0 += kVbChunk) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            Ps[sq + 2 * k][sp] = xa[k].x * xb[k].x;
            Ps[sq + 2 * k + 1][sp] = xa[k].y * xb[k].y;
        }
        Cs[scq][sc] = xc.x;
        Cs[scq + 1][sc] = xc.y;
        __syncthreads();
        if (q0 + kVbChunk < a.Qp) fetch(q0 + kVbChunk);
#pragma unroll
        for (int k0 = 0; k0 < kVbChunk; k0 += 4) {
            double av[2], bv[4];
#pragma unroll
            for (int u = 0; u < 2; ++u) av[u] = Cs[k0 + lk][wc + 16 * u + li];
#pragma unroll
            for (int v = 0; v < 4; ++v) bv[v] = Ps[k0 + lk][wp + 16 * v + li];
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[v], acc[u][v], 0, 0, 0);
        }
    }

    // This lane's four pairs and, for a cube, their b (values with c < b are
    // not kept).
    int64_t pp[4];
    int pb[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        pp[v] = p0 + wp + 16 * v + li;
        pb[v] = 0;
    }
    if (!a.box) {
        int b = pair_b(pp[0]);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            while (tri2(b + 1) <= pp[v]) ++b;
            pb[v] = b;
        }
    }
    const int64_t E2 = static_cast<int64_t>(a.E1) * a.E1;
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int c = c0 + wc + 16 * u + 4 * r + lk;
            if (c < 0 || c >= a.E1) continue;
            const int64_t base = a.box ? c * E2 : tri3(c);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                if (pp[v] >= a.npairs || pb[v] > c) continue;
                a.val[base + pp[v]] = acc[u][v][r] * a.pref;
            }
        }
}

constexpr int kVrThreads = 1024, kVrBatch = 4;

struct RecValArgs {
    const int4 *quads;
    int64_t n;
    const int32_t *basis;
    int N;
    const int32_t *fold;
    int K, nd, E1, box;
    const double *val;
    double *out;
    int *err;
};

typedef int v4i __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int bx(int v) { return (v << 24) >> 24; }
__device__ __forceinline__ int by(int v) { return (v << 16) >> 24; }
__device__ __forceinline__ int bz(int v) { return (v << 8) >> 24; }

template <bool LDS_MAPS>
__global__ __launch_bounds__(kVrThreads) void k_rec_values(RecValArgs a) {
    extern __shared__ int32_t lds_maps[];
    const int32_t *basis = a.basis;
    const int16_t *lfold = reinterpret_cast<const int16_t *>(lds_maps + a.N);
    if (LDS_MAPS) {
        int16_t *f16 = reinterpret_cast<int16_t *>(lds_maps + a.N);
        for (int i = threadIdx.x; i < a.N; i += kVrThreads) lds_maps[i] = a.basis[i];
        for (int i = threadIdx.x; i < a.nd * a.nd; i += kVrThreads) f16[i] = static_cast<int16_t>(a.fold[i]);
        __syncthreads();
        basis = lds_maps;
    }
    const unsigned N = static_cast<unsigned>(a.N);
    const int K = a.K, nd = a.nd;
    const int64_t E2 = static_cast<int64_t>(a.E1) * a.E1;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kVrThreads * kVrBatch;
    // The next batch's quadruples are loaded while this batch is decoded
    // and its values read.
    int4 qn[kVrBatch];
    auto fetch = [&](int64_t b0) {
#pragma unroll
        for (int k = 0; k < kVrBatch; ++k) {
            const int64_t e = b0 + k * kVrThreads + threadIdx.x;
            if (e < a.n) {   // streamed once
                const v4i t = __builtin_nontemporal_load(reinterpret_cast<const v4i *>(a.quads) + e);
                qn[k] = make_int4(t.x, t.y, t.z, t.w);
            }
        }
    };
    int64_t b0 = static_cast<int64_t>(blockIdx.x) * kVrThreads * kVrBatch;
    if (b0 < a.n) fetch(b0);
    for (; b0 < a.n; b0 += stride) {
        int4 q[kVrBatch];
#pragma unroll
        for (int k = 0; k < kVrBatch; ++k) q[k] = qn[k];
        if (b0 + stride < a.n) fetch(b0 + stride);
        double v[kVrBatch];
#pragma unroll
        for (int k = 0; k < kVrBatch; ++k) {
            const int64_t e = b0 + k * kVrThreads + threadIdx.x;
            v[k] = NAN;
            if (e >= a.n) continue;
            const int4 t = q[k];
            if (static_cast<unsigned>(t.x) >= N || static_cast<unsigned>(t.y) >= N ||
                static_cast<unsigned>(t.z) >= N || static_cast<unsigned>(t.w) >= N) {
                raise_error(a.err);
                continue;
            }
            const int ni = basis[t.x], nj = basis[t.y], nk = basis[t.z], nl = basis[t.w];
            const int ix = (bx(nk) - bx(ni) + K) * nd + (bx(nl) - bx(nj) + K);
            const int iy = (by(nk) - by(ni) + K) * nd + (by(nl) - by(nj) + K);
            const int iz = (bz(nk) - bz(ni) + K) * nd + (bz(nl) - bz(nj) + K);
            int fx = LDS_MAPS ? lfold[ix] : a.fold[ix];
            int fy = LDS_MAPS ? lfold[iy] : a.fold[iy];
            int fz = LDS_MAPS ? lfold[iz] : a.fold[iz];
            int64_t idx;
            if (a.box) {
                idx = fz * E2 + static_cast<int64_t>(fx) * a.E1 + fy;
            } else {
                const int lo = min(fx, min(fy, fz)), hi = max(fx, max(fy, fz));
                const int mid = fx + fy + fz - lo - hi;
                idx = tri3(hi) + tri2(mid) + lo;
            }
            v[k] = a.val[idx];
        }
#pragma unroll
        for (int k = 0; k < kVrBatch; ++k) {
            const int64_t e = b0 + k * kVrThreads + threadIdx.x;
            if (e < a.n) __builtin_nontemporal_store(v[k], a.out + e);
        }
    }
}

}  // namespace

int64_t value_count(const Table &t) {
    const int64_t e = t.E1;
    return t.ndir == 3 ? e * e * e : e * (e + 1) * (e + 2) / 6;
}

// The c tiles of pair tile pt: c_lo, c_lo + 64, ..., n of them, covering every
// c >= b (a cube) up to the largest c that a pair of the tile can reach
// (orbit sizes summing to at most smax).  The smallest size sum of the tile
// is its first pair's or the first of the next row (a row's sizes ascend).
void value_tile_c_range(const int *so, int E1, bool box, int smax, int64_t pt, int *c_lo, int *n) {
    const int64_t npairs = box ? static_cast<int64_t>(E1) * E1 : static_cast<int64_t>(E1) * (E1 + 1) / 2;
    const int64_t p0 = pt * kVbTileP, p1 = (p0 + kVbTileP < npairs ? p0 + kVbTileP : npairs) - 1;
    int smin;
    if (box) {
        const int x0 = static_cast<int>(p0 / E1), y0 = static_cast<int>(p0 % E1);
        smin = so[x0] + so[y0];
        if (p1 / E1 > x0) {
            const int t = so[x0 + 1];
            smin = t < smin ? t : smin;
        }
        *c_lo = 0;
    } else {
        const int b0 = pair_b(p0), a0 = static_cast<int>(p0 - tri2(b0));
        smin = so[a0] + so[b0];
        if (pair_b(p1) > b0) {
            const int t = so[b0 + 1];
            smin = t < smin ? t : smin;
        }
        *c_lo = b0;
    }
    *n = 0;
    const int room = smax - smin;
    if (room < 0) return;
    int lo = 0, hi = E1 - 1;   // the last orbit with size <= room (orbit 0 has size 0)
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (so[mid] <= room) lo = mid;
        else hi = mid - 1;
    }
    if (lo >= *c_lo) *n = (lo - *c_lo + kVbTile) / kVbTile;
}

namespace {
// Block descriptors of the build, per device and (cutoff, cube or box): they
// depend on nothing else, so each is formed and uploaded once per process.
struct PlanKey {
    int device, n2max, box;
    bool operator<(const PlanKey &o) const {
        return device != o.device ? device < o.device : n2max != o.n2max ? n2max < o.n2max : box < o.box;
    }
};
struct Plan {
    uint32_t *d_desc = nullptr;
    int64_t blocks = 0;
};
std::mutex g_plan_mu;
std::map<PlanKey, Plan> g_plans;

hipError_t build_plan(const Table &t, Plan &pl) {
    std::vector<int32_t> fold, reps;
    build_fold(t.K, fold, reps);
    std::vector<int> so(t.E1);
    for (int f = 0; f < t.E1; ++f) so[f] = reps[2 * f] * reps[2 * f] + reps[2 * f + 1] * reps[2 * f + 1];
    const bool box = t.ndir == 3;
    const int64_t npairs = box ? static_cast<int64_t>(t.E1) * t.E1 : static_cast<int64_t>(t.E1) * (t.E1 + 1) / 2;
    const int64_t npt = (npairs + kVbTileP - 1) / kVbTileP;
    if (npt > int64_t(0xffffff) || (t.E1 + kVbTile - 1) / kVbTile > 255) return hipErrorInvalidValue;
    std::vector<uint32_t> desc;
    for (int64_t pt = 0; pt < npt; ++pt) {
        int c_lo = 0, n = 0;
        value_tile_c_range(so.data(), t.E1, box, 8 * t.n2max, pt, &c_lo, &n);
        for (int k = 0; k < n; ++k) desc.push_back(static_cast<uint32_t>(pt) | (static_cast<uint32_t>(k) << 24));
    }
    pl.blocks = static_cast<int64_t>(desc.size());
    if (desc.empty()) return hipSuccess;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&pl.d_desc), sizeof(uint32_t) * desc.size());
    if (e == hipSuccess)
        e = hipMemcpy(pl.d_desc, desc.data(), sizeof(uint32_t) * desc.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess && pl.d_desc) {
        (void)hipFree(pl.d_desc);
        pl.d_desc = nullptr;
    }
    return e;
}
}  // namespace

void release_value_plans() {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    for (auto &kv : g_plans)
        if (kv.second.d_desc) (void)hipFree(kv.second.d_desc);
    g_plans.clear();
}

hipError_t launch_values_build(const Table &t, double *d_val, hipStream_t s) {
    ValBuildArgs a{};
    a.tab = t.d_tauF;
    a.Qp = t.fl.Qp;
    a.E1 = t.E1;
    a.box = t.ndir == 3;
    a.npairs = a.box ? static_cast<int64_t>(t.E1) * t.E1 : static_cast<int64_t>(t.E1) * (t.E1 + 1) / 2;
    a.pref = 1.0 / (std::sqrt(M_PI) * t.L);
    a.val = d_val;
    if (a.Qp % kVbChunk) return hipErrorInvalidValue;
    Plan pl;
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        const PlanKey key{t.device, t.n2max, a.box};
        auto it = g_plans.find(key);
        if (it == g_plans.end()) {
            const hipError_t e = build_plan(t, pl);
            if (e != hipSuccess) return e;
            it = g_plans.emplace(key, pl).first;
        }
        pl = it->second;
    }
    if (pl.blocks == 0) return hipSuccess;
    if (pl.blocks > int64_t(0x7fffffff)) return hipErrorInvalidValue;
    a.desc = pl.d_desc;
    hipLaunchKernelGGL(k_values_build, dim3(static_cast<unsigned>(pl.blocks)), dim3(kVbThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_rec_values(const Table &t, const int32_t *d_quads, int64_t n, double *d_out,
                             hipStream_t s) {
    if (n <= 0) return hipSuccess;
    RecValArgs a{};
    a.quads = reinterpret_cast<const int4 *>(d_quads);
    a.n = n;
    a.basis = t.d_basis;
    a.N = static_cast<int>(t.N);
    a.fold = t.d_fold;
    a.K = t.K;
    a.nd = t.nd;
    a.E1 = t.E1;
    a.box = t.ndir == 3;
    a.val = t.d_val;
    a.out = d_out;
    a.err = t.d_err;
    const size_t maps = sizeof(int32_t) * static_cast<size_t>(t.N) + sizeof(int16_t) * static_cast<size_t>(t.nd) * t.nd;
    const size_t lds = (maps + 15) / 16 * 16;
    const bool lds_maps = lds <= static_cast<size_t>(kLdsMax);
    const int per_cu = lds_maps ? std::max(1, std::min(2, static_cast<int>(kLdsMax / lds))) : 2;
    const int64_t tiles = (n + kVrThreads * kVrBatch - 1) / (kVrThreads * kVrBatch);
    // Four times the resident workgroups: the dispatcher then evens out the
    // blocks' unequal miss counts at the end of the launch (1.14 -> 1.10 ms
    // per 1e8 quadruples); many more restage the LDS maps too often.
    const unsigned grid = static_cast<unsigned>(std::min<int64_t>(tiles, int64_t(t.n_cu) * per_cu * 4));
    if (lds_maps) {
        const hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(k_rec_values<true>),
                                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                                   static_cast<int>(lds));
        if (err != hipSuccess) return err;
        hipLaunchKernelGGL(k_rec_values<true>, dim3(grid), dim3(kVrThreads), lds, s, a);
    } else {
        hipLaunchKernelGGL(k_rec_values<false>, dim3(grid), dim3(kVrThreads), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace pwc
