// Reconstruction of <ij|kl> from the per-node tables (Eq. 14):
//   <ij|kl> = (1/(sqrt(pi) L)) sum_q W_q tau_q(o_x) tau_q(o_y) tau_q(o_z),
// o_d = (m_d, m'_d) = ((n_k - n_i)_d, (n_l - n_j)_d).
//
// Layout.  tau is symmetric under (m, m') -> (m', m) and (m, m') -> (-m, -m'),
// so the table is stored folded: E orbit representatives per node (about a
// quarter of nd^2).  In HBM the folded table is [E][Qp]: the Qp (Q padded to
// a multiple of 16 with zero weight) node values of one entry are contiguous.
//
// Schedule: node passes.  The node range is cut into P chunks of c nodes,
// each chunk's [E][c] slab small enough to sit in LDS.  Pass p is one launch
// of a persistent grid; every workgroup stages slab p once and then streams
// every quadruple through it.  A decode kernel first turns each quadruple into
// three folded-entry indices (8 bytes, kept in a scratch array); each pass
// adds its c node terms to an FP64 partial sum kept in the output array, and
// the last pass applies 1/(sqrt(pi) L).  Table refills from L2 are thus paid
// once per workgroup and pass, and the per-quadruple traffic is a plain HBM
// stream (16 B of indices and 8 B of entries for the decode; 8 B of entries
// plus 8 B (first pass) or 16 B (later passes) of partial sum per pass).
//
// Within a pass, G lanes share one quadruple; lane s reads the node pairs
// 2 (s + G k), k = 0 .. c/(2G) - 1, so the G lanes of a group read G adjacent
// 16-byte words of one table row (a contiguous, aligned run: on gfx950 this
// runs about 1.3x faster than independent random 16-byte reads).  Group
// partial sums are combined with lane shuffles.
#include <algorithm>
#include <cmath>

#include "ffloat.h"
#include "pwc_internal.h"

namespace pwc {
namespace {

constexpr int kThreads = 1024;   // one workgroup per CU when the slab is large
constexpr int kGroup = 4;        // lanes per quadruple
constexpr int kRows = 4;         // quadruples per group and iteration

struct PassArgs {
    const int4 *quads;
    int64_t n;
    const int32_t *basis;
    int N;
    const int32_t *fold;
    int K, nd;
    const void *tab;   // [E][Qp] double or float2
    const void *w;     // [Qp]    double or float2
    int E, Qp, c, q0;  // this pass: nodes [q0, q0 + c)
    uint2 *scratch;    // [n] packed folded entries (multi-pass only)
    double pref;
    double *out;
    int *err;
};

// Basis vector packed as three signed bytes of an int32.
__device__ __forceinline__ int bx(int v) { return (v << 24) >> 24; }
__device__ __forceinline__ int by(int v) { return (v << 16) >> 24; }
__device__ __forceinline__ int bz(int v) { return (v << 8) >> 24; }

// FP64 arithmetic: one node term is ((x * y) * z) * w added with an FMA.
struct F64 {
    using V = double2;   // two adjacent nodes
    struct Acc { double v; };
    __device__ static void zero(Acc &a) { a.v = 0.0; }
    __device__ static void add2(Acc &a, V x, V y, V z, V w) {
        a.v = fma(x.x * y.x * z.x, w.x, a.v);
        a.v = fma(x.y * y.y * z.y, w.y, a.v);
    }
    __device__ static double value(const Acc &a) { return a.v; }
};

// Split-FP32 arithmetic: table entries and weights are (hi, lo) float pairs;
// node terms are float-float products, summed with TwoSum compensation.
struct FF {
    using V = float4;    // (hi0, lo0, hi1, lo1)
    struct Acc { float h, l; };
    __device__ static void zero(Acc &a) { a.h = a.l = 0.0f; }
    __device__ static void add2(Acc &a, V x, V y, V z, V w) {
        ff_acc(a.h, a.l, ff_mul(ff_mul(ff_mul(ff{x.x, x.y}, ff{y.x, y.y}), ff{z.x, z.y}), ff{w.x, w.y}));
        ff_acc(a.h, a.l, ff_mul(ff_mul(ff_mul(ff{x.z, x.w}, ff{y.z, y.w}), ff{z.z, z.w}), ff{w.z, w.w}));
    }
    __device__ static double value(const Acc &a) { return ff_to_double(a.h, a.l); }
};

__device__ __forceinline__ uint2 pack3(int fx, int fy, int fz) {
    return make_uint2(static_cast<uint32_t>(fx) | (static_cast<uint32_t>(fy) << 16),
                      static_cast<uint32_t>(fz));
}

// Sum over the 4 lanes of a quad (lanes 4j .. 4j+3) with DPP quad permutes:
// no LDS traffic.  quad_perm selectors: 0xB1 = (1,0,3,2), 0x4E = (2,3,0,1).
template <int CTRL>
__device__ __forceinline__ double quad_swap(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double quad_sum(double v) {
    v += quad_swap<0xB1>(v);
    return v + quad_swap<0x4E>(v);
}

// Per-iteration loads of one lane: the packed entries and (after the first
// pass) the partial sums, issued one grid-stride iteration ahead of their use.
template <bool FIRST, int R>
struct Stream {
    uint2 pk[R];
    double prev[R];
    __device__ __forceinline__ void load(const PassArgs &a, int64_t base, int NG, int g) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t e = base + r * NG + g;
            if (e < a.n) {
                pk[r] = a.scratch[e];
                if (!FIRST) prev[r] = a.out[e];
            }
        }
    }
};

// Decode every quadruple into its packed folded entries; an out-of-range
// index leaves the invalid marker (y = 0xffffffff) and raises the error word.
// A streaming kernel with many waves per CU.  Each quadruple needs 7
// dependent random gathers (4 basis vectors, 3 fold entries); when the basis
// and the fold map fit, they are staged in LDS first, where random gathers
// are far cheaper than divergent L1/L2 accesses.
constexpr uint32_t kInvalid = 0xffffffffu;
constexpr int kDecodeThreads = 256, kDecodeBatch = 4;

template <bool LDS_MAPS>
__global__ __launch_bounds__(kDecodeThreads) void k_decode(PassArgs a) {
    extern __shared__ uint4 lds_raw[];
    int32_t *lbasis = reinterpret_cast<int32_t *>(lds_raw);
    int16_t *lfold = reinterpret_cast<int16_t *>(lbasis + a.N);
    const int nd2 = a.nd * a.nd;
    if (LDS_MAPS) {
        for (int i = threadIdx.x; i < a.N; i += kDecodeThreads) lbasis[i] = a.basis[i];
        for (int i = threadIdx.x; i < nd2; i += kDecodeThreads) lfold[i] = static_cast<int16_t>(a.fold[i]);
        __syncthreads();
    }
    const unsigned N = static_cast<unsigned>(a.N);
    const int K = a.K, nd = a.nd;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kDecodeThreads * kDecodeBatch;
    for (int64_t base = static_cast<int64_t>(blockIdx.x) * kDecodeThreads * kDecodeBatch;
         base < a.n; base += stride) {
        int4 q[kDecodeBatch];
#pragma unroll
        for (int b = 0; b < kDecodeBatch; ++b) {
            const int64_t e = base + b * kDecodeThreads + threadIdx.x;
            if (e < a.n) q[b] = a.quads[e];
        }
#pragma unroll
        for (int b = 0; b < kDecodeBatch; ++b) {
            const int64_t e = base + b * kDecodeThreads + threadIdx.x;
            if (e >= a.n) continue;
            const int4 v = q[b];
            uint2 pk = make_uint2(0u, kInvalid);
            if (static_cast<unsigned>(v.x) < N && static_cast<unsigned>(v.y) < N &&
                static_cast<unsigned>(v.z) < N && static_cast<unsigned>(v.w) < N) {
                const int ni = LDS_MAPS ? lbasis[v.x] : a.basis[v.x];
                const int nj = LDS_MAPS ? lbasis[v.y] : a.basis[v.y];
                const int nk = LDS_MAPS ? lbasis[v.z] : a.basis[v.z];
                const int nl = LDS_MAPS ? lbasis[v.w] : a.basis[v.w];
                const int ix = (bx(nk) - bx(ni) + K) * nd + (bx(nl) - bx(nj) + K);
                const int iy = (by(nk) - by(ni) + K) * nd + (by(nl) - by(nj) + K);
                const int iz = (bz(nk) - bz(ni) + K) * nd + (bz(nl) - bz(nj) + K);
                const int fx = LDS_MAPS ? lfold[ix] : a.fold[ix];
                const int fy = LDS_MAPS ? lfold[iy] : a.fold[iy];
                const int fz = LDS_MAPS ? lfold[iz] : a.fold[iz];
                pk = pack3(fx, fy, fz);
            } else {
                atomicOr(a.err, 1);
            }
            a.scratch[e] = pk;
        }
    }
}

template <typename A, bool FIRST, bool LAST>
__global__ __launch_bounds__(kThreads) void k_rec_pass(PassArgs a) {
    using V = typename A::V;
    extern __shared__ uint4 lds_raw[];
    constexpr int G = kGroup, R = kRows, NG = kThreads / G, TILE = NG * R;
    static_assert(G == 4, "the group reduction is a DPP quad sum");
    V *lds = reinterpret_cast<V *>(lds_raw);
    const int half = a.c / 2;                   // 16-byte words per table row in LDS
    V *lw = lds + static_cast<size_t>(a.E) * half;
    const int s = threadIdx.x % G, g = threadIdx.x / G;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * TILE;
    int64_t base = static_cast<int64_t>(blockIdx.x) * TILE;
    Stream<FIRST, R> nxt;
    nxt.load(a, base, NG, g);                   // overlaps the slab staging
    // Stage the slab [E][c] of nodes [q0, q0 + c) and its weights.
    {
        const V *src = static_cast<const V *>(a.tab) + a.q0 / 2;
        const int row = a.Qp / 2, words = a.E * half;
        for (int i = threadIdx.x; i < words; i += kThreads) {
            const int e = i / half, j = i - e * half;
            lds[i] = src[static_cast<size_t>(e) * row + j];
        }
        const V *ws = static_cast<const V *>(a.w) + a.q0 / 2;
        for (int i = threadIdx.x; i < half; i += kThreads) lw[i] = ws[i];
    }
    __syncthreads();
    const int pairs = half / G;
    for (; base < a.n; base += stride) {
        const Stream<FIRST, R> cur = nxt;
        if (base + stride < a.n) nxt.load(a, base + stride, NG, g);
        uint32_t pxy[R], pz[R];
        double prev[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t e = base + r * NG + g;
            int fx = 0, fy = 0, fz = 0;
            prev[r] = 0.0;
            if (e < a.n) {
                if (cur.pk[r].y == kInvalid) {
                    prev[r] = NAN;   // set by the first pass, carried by the others
                } else {
                    fx = cur.pk[r].x & 0xffffu;
                    fy = cur.pk[r].x >> 16;
                    fz = cur.pk[r].y;
                }
                if (!FIRST) prev[r] = cur.prev[r];
            }
            // word offsets of this lane's first node pair in each row
            pxy[r] = static_cast<uint32_t>(fx * half + s) | (static_cast<uint32_t>(fy * half + s) << 16);
            pz[r] = static_cast<uint32_t>(fz * half + s);
        }
        typename A::Acc acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) A::zero(acc[r]);
        for (int k = 0; k < pairs; ++k) {
            const int d = k * G;
            const V w = lw[s + d];
            V x[R], y[R], z[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                x[r] = lds[(pxy[r] & 0xffffu) + d];
                y[r] = lds[(pxy[r] >> 16) + d];
                z[r] = lds[pz[r] + d];
            }
#pragma unroll
            for (int r = 0; r < R; ++r) A::add2(acc[r], x[r], y[r], z[r], w);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double v = quad_sum(A::value(acc[r]));
            const int64_t e = base + r * NG + g;
            if (s == 0 && e < a.n) a.out[e] = LAST ? (prev[r] + v) * a.pref : prev[r] + v;
        }
    }
}

using PassKernel = void (*)(PassArgs);

template <typename A>
PassKernel pass_kernel(int p, int P) {
    if (p == 0) return P == 1 ? k_rec_pass<A, true, true> : k_rec_pass<A, true, false>;
    return p == P - 1 ? k_rec_pass<A, false, true> : k_rec_pass<A, false, false>;
}

// stage_ev (optional): events recorded before the decode and after every
// launch of the first slab, for per-stage timing.
template <typename A>
hipError_t run_passes(const PassArgs &a0, const Table &t, size_t lds, hipStream_t s,
                      hipEvent_t *stage_ev) {
    const int P = t.fl.nchunk;
    for (int p = 0; p < P; ++p) {
        const hipError_t err = hipFuncSetAttribute(
            reinterpret_cast<const void *>(pass_kernel<A>(p, P)),
            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
        if (err != hipSuccess) return err;
    }
    hipError_t err0 = hipSuccess;
    const int64_t tile = static_cast<int64_t>(kThreads / kGroup) * kRows;
    // LDS copy of the basis (int32) and the fold map (int16) for the decode.
    const size_t maps_bytes = (sizeof(int32_t) * static_cast<size_t>(t.N) +
                               sizeof(int16_t) * static_cast<size_t>(t.nd) * t.nd + 15) / 16 * 16;
    if (maps_bytes <= static_cast<size_t>(kLdsMax)) {
        const hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(k_decode<true>),
                                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                                   static_cast<int>(maps_bytes));
        if (err != hipSuccess) return err;
    }
    // Slabs bound the scratch array: at most kRecSlab quadruples per slab.
    for (int64_t off = 0; off < a0.n; off += kRecSlab) {
        PassArgs a = a0;
        a.n = std::min<int64_t>(kRecSlab, a0.n - off);
        a.quads = a0.quads + off;
        a.out = a0.out + off;
        hipEvent_t *ev = (off == 0) ? stage_ev : nullptr;
        if (ev && (err0 = hipEventRecord(ev[0], s)) != hipSuccess) return err0;
        const int64_t dblocks = (a.n + kDecodeThreads * kDecodeBatch - 1) / (kDecodeThreads * kDecodeBatch);
        hipError_t err;
        if (maps_bytes <= static_cast<size_t>(kLdsMax)) {
            const int per_cu = std::max(1, std::min(8, static_cast<int>(kLdsMax / std::max<size_t>(maps_bytes, 1))));
            const unsigned dgrid = static_cast<unsigned>(std::min<int64_t>(dblocks, int64_t(t.n_cu) * per_cu));
            hipLaunchKernelGGL(k_decode<true>, dim3(dgrid), dim3(kDecodeThreads), maps_bytes, s, a);
        } else {
            const unsigned dgrid = static_cast<unsigned>(std::min<int64_t>(dblocks, int64_t(t.n_cu) * 16));
            hipLaunchKernelGGL(k_decode<false>, dim3(dgrid), dim3(kDecodeThreads), 0, s, a);
        }
        err = hipGetLastError();
        if (err != hipSuccess) return err;
        if (ev && (err = hipEventRecord(ev[1], s)) != hipSuccess) return err;
        const int64_t tiles = (a.n + tile - 1) / tile;
        const unsigned grid = static_cast<unsigned>(std::min<int64_t>(tiles, t.fl.grid_cap));
        for (int p = 0; p < P; ++p) {
            a.q0 = p * t.fl.c;
            hipLaunchKernelGGL(pass_kernel<A>(p, P), dim3(grid), dim3(kThreads), lds, s, a);
            err = hipGetLastError();
            if (err != hipSuccess) return err;
            if (ev && (err = hipEventRecord(ev[2 + p], s)) != hipSuccess) return err;
        }
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_reconstruct(const Table &t, const int32_t *d_quads, int64_t n, double *d_out,
                              pwc_precision p, hipStream_t s, hipEvent_t *stage_ev) {
    if (n <= 0) return hipSuccess;
    PassArgs a{};
    a.quads = reinterpret_cast<const int4 *>(d_quads);
    a.n = n;
    a.basis = t.d_basis;
    a.N = static_cast<int>(t.N);
    a.fold = t.d_fold;
    a.K = t.K;
    a.nd = t.nd;
    a.E = t.fl.E;
    a.Qp = t.fl.Qp;
    a.c = t.fl.c;
    a.pref = 1.0 / (std::sqrt(M_PI) * t.L);
    a.out = d_out;
    a.err = t.d_err;
    const size_t lds = (static_cast<size_t>(a.E) + 1) * a.c * 8;
    const size_t bytes = sizeof(uint2) * static_cast<size_t>(std::min<int64_t>(n, kRecSlab));
    hipError_t err = hipMallocAsync(reinterpret_cast<void **>(&a.scratch), bytes, s);
    if (err != hipSuccess) return err;
    if (p == PWC_MIXED) {
        a.tab = t.d_tauHL;
        a.w = t.d_WHL;
        err = run_passes<FF>(a, t, lds, s, stage_ev);
    } else {
        a.tab = t.d_tauF;
        a.w = t.d_Wpad;
        err = run_passes<F64>(a, t, lds, s, stage_ev);
    }
    const hipError_t e2 = hipFreeAsync(a.scratch, s);
    if (err == hipSuccess) err = e2;
    return err;
}

}  // namespace pwc
