// Reconstruction of <ij|kl> from the per-node tables (Eq. 14):
//   <ij|kl> = (1/(sqrt(pi) L)) sum_q W_q tau_q(o_x) tau_q(o_y) tau_q(o_z),
// o_d = (m_d, m'_d) = ((n_k - n_i)_d, (n_l - n_j)_d).
//
// Layout.  tau is symmetric under (m, m') -> (m', m) and (m, m') -> (-m, -m'),
// so the table is stored folded: E orbit representatives per node (about a
// quarter of nd^2).  Nodes are grouped in chunks of c; chunk k is a
// contiguous [E][c] block whose c node values per entry sit side by side, so
// one 16-byte LDS read returns two nodes of one entry.
//
// Schedule.  A workgroup owns a tile of R * 256 quadruples; every lane decodes
// R of them once into three LDS offsets and keeps R accumulators in
// registers.  For each chunk the workgroup stages the chunk (at most
// kLdsBudget bytes, two workgroups per CU) from L2 into LDS and every lane
// runs the node loop for its R integrals.  Quadruple loads and result stores
// are coalesced; the table is read from HBM once per tile and otherwise
// served by L2.
#include <cmath>

#include "ffloat.h"
#include "pwc_internal.h"

namespace pwc {
namespace {

constexpr int kThreads = 256;
constexpr int kRows = 8;   // quadruples per lane

struct RecArgs {
    const int4 *quads;
    int64_t n;
    const int32_t *basis;
    int N;
    const int32_t *fold;
    int K, nd;
    const void *tab;   // [nchunk][E][c] double or float2
    const void *w;     // [nchunk * c]   double or float2
    int E, c, nchunk;
    double pref;
    double *out;
    int *err;
};

// Basis vector packed as three signed bytes of an int32.
__device__ __forceinline__ int bx(int v) { return (v << 24) >> 24; }
__device__ __forceinline__ int by(int v) { return (v << 16) >> 24; }
__device__ __forceinline__ int bz(int v) { return (v << 8) >> 24; }

// Decode one quadruple into the three folded-entry offsets (in units of one
// node value, i.e. entry * c).  Returns false if an index is out of range.
__device__ __forceinline__ bool decode(const RecArgs &a, int4 q, int &ox, int &oy, int &oz) {
    const unsigned N = static_cast<unsigned>(a.N);
    if (static_cast<unsigned>(q.x) >= N || static_cast<unsigned>(q.y) >= N ||
        static_cast<unsigned>(q.z) >= N || static_cast<unsigned>(q.w) >= N)
        return false;
    const int ni = a.basis[q.x], nj = a.basis[q.y], nk = a.basis[q.z], nl = a.basis[q.w];
    const int K = a.K, nd = a.nd;
    ox = a.fold[(bx(nk) - bx(ni) + K) * nd + (bx(nl) - bx(nj) + K)] * a.c;
    oy = a.fold[(by(nk) - by(ni) + K) * nd + (by(nl) - by(nj) + K)] * a.c;
    oz = a.fold[(bz(nk) - bz(ni) + K) * nd + (bz(nl) - bz(nj) + K)] * a.c;
    return true;
}

template <typename T>
__device__ __forceinline__ void stage_chunk(const RecArgs &a, int ch, T *lt, T *lw) {
    // E * c is even (c is even), so the chunk copies as 16-byte words.
    const size_t words = static_cast<size_t>(a.E) * a.c * sizeof(T) / 16;
    const uint4 *src = reinterpret_cast<const uint4 *>(static_cast<const T *>(a.tab) +
                                                       static_cast<size_t>(ch) * a.E * a.c);
    uint4 *dst = reinterpret_cast<uint4 *>(lt);
    for (size_t i = threadIdx.x; i < words; i += kThreads) dst[i] = src[i];
    const T *ws = static_cast<const T *>(a.w) + static_cast<size_t>(ch) * a.c;
    for (int i = threadIdx.x; i < a.c; i += kThreads) lw[i] = ws[i];
}

__global__ __launch_bounds__(kThreads, 2) void k_rec_f64(RecArgs a) {
    extern __shared__ uint4 lds_raw[];
    double *lt = reinterpret_cast<double *>(lds_raw);
    double *lw = lt + static_cast<size_t>(a.E) * a.c;
    const int64_t base = static_cast<int64_t>(blockIdx.x) * (kRows * kThreads);
    int ox[kRows], oy[kRows], oz[kRows];
    double acc[kRows];
    bool ok[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const int64_t e = base + r * kThreads + threadIdx.x;
        ox[r] = oy[r] = oz[r] = 0;
        acc[r] = 0.0;
        ok[r] = false;
        if (e < a.n) {
            ok[r] = decode(a, a.quads[e], ox[r], oy[r], oz[r]);
            if (!ok[r]) {
                ox[r] = oy[r] = oz[r] = 0;
                atomicOr(a.err, 1);
            }
        }
    }
    for (int ch = 0; ch < a.nchunk; ++ch) {
        __syncthreads();
        stage_chunk<double>(a, ch, lt, lw);
        __syncthreads();
        for (int q = 0; q < a.c; q += 2) {
            const double2 w = *reinterpret_cast<const double2 *>(lw + q);
#pragma unroll
            for (int r = 0; r < kRows; ++r) {
                const double2 x = *reinterpret_cast<const double2 *>(lt + ox[r] + q);
                const double2 y = *reinterpret_cast<const double2 *>(lt + oy[r] + q);
                const double2 z = *reinterpret_cast<const double2 *>(lt + oz[r] + q);
                acc[r] = fma(x.x * y.x * z.x, w.x, acc[r]);
                acc[r] = fma(x.y * y.y * z.y, w.y, acc[r]);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const int64_t e = base + r * kThreads + threadIdx.x;
        if (e < a.n) a.out[e] = ok[r] ? acc[r] * a.pref : NAN;
    }
}

__global__ __launch_bounds__(kThreads, 2) void k_rec_mixed(RecArgs a) {
    extern __shared__ uint4 lds_raw[];
    float2 *lt = reinterpret_cast<float2 *>(lds_raw);
    float2 *lw = lt + static_cast<size_t>(a.E) * a.c;
    const int64_t base = static_cast<int64_t>(blockIdx.x) * (kRows * kThreads);
    int ox[kRows], oy[kRows], oz[kRows];
    float sh[kRows], sl[kRows];
    bool ok[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const int64_t e = base + r * kThreads + threadIdx.x;
        ox[r] = oy[r] = oz[r] = 0;
        sh[r] = sl[r] = 0.0f;
        ok[r] = false;
        if (e < a.n) {
            ok[r] = decode(a, a.quads[e], ox[r], oy[r], oz[r]);
            if (!ok[r]) {
                ox[r] = oy[r] = oz[r] = 0;
                atomicOr(a.err, 1);
            }
        }
    }
    for (int ch = 0; ch < a.nchunk; ++ch) {
        __syncthreads();
        stage_chunk<float2>(a, ch, lt, lw);
        __syncthreads();
        for (int q = 0; q < a.c; q += 2) {
            const float4 w = *reinterpret_cast<const float4 *>(lw + q);
#pragma unroll
            for (int r = 0; r < kRows; ++r) {
                const float4 x = *reinterpret_cast<const float4 *>(lt + ox[r] + q);
                const float4 y = *reinterpret_cast<const float4 *>(lt + oy[r] + q);
                const float4 z = *reinterpret_cast<const float4 *>(lt + oz[r] + q);
                ff p0 = ff_mul(ff_mul(ff_mul(ff{x.x, x.y}, ff{y.x, y.y}), ff{z.x, z.y}), ff{w.x, w.y});
                ff_acc(sh[r], sl[r], p0);
                ff p1 = ff_mul(ff_mul(ff_mul(ff{x.z, x.w}, ff{y.z, y.w}), ff{z.z, z.w}), ff{w.z, w.w});
                ff_acc(sh[r], sl[r], p1);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const int64_t e = base + r * kThreads + threadIdx.x;
        if (e < a.n) a.out[e] = ok[r] ? ff_to_double(sh[r], sl[r]) * a.pref : NAN;
    }
}

template <typename Kern>
hipError_t set_lds(Kern k, size_t bytes) {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                               hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
}

}  // namespace

hipError_t launch_reconstruct(const Table &t, const int32_t *d_quads, int64_t n, double *d_out,
                              pwc_precision p, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    RecArgs a{};
    a.quads = reinterpret_cast<const int4 *>(d_quads);
    a.n = n;
    a.basis = t.d_basis;
    a.N = static_cast<int>(t.N);
    a.fold = t.d_fold;
    a.K = t.K;
    a.nd = t.nd;
    a.E = t.fl.E;
    a.c = t.fl.c;
    a.nchunk = t.fl.nchunk;
    a.pref = 1.0 / (std::sqrt(M_PI) * t.L);
    a.out = d_out;
    a.err = t.d_err;
    const size_t lds = (static_cast<size_t>(a.E) * a.c + a.c) * 8;
    const int64_t tile = static_cast<int64_t>(kRows) * kThreads;
    const dim3 grid(static_cast<unsigned>((n + tile - 1) / tile));
    hipError_t err;
    if (p == PWC_MIXED) {
        a.tab = t.d_tauHL;
        a.w = t.d_WHL;
        if ((err = set_lds(k_rec_mixed, lds)) != hipSuccess) return err;
        hipLaunchKernelGGL(k_rec_mixed, grid, dim3(kThreads), lds, s, a);
    } else {
        a.tab = t.d_tauF;
        a.w = t.d_Wpad;
        if ((err = set_lds(k_rec_f64, lds)) != hipSuccess) return err;
        hipLaunchKernelGGL(k_rec_f64, grid, dim3(kThreads), lds, s, a);
    }
    return hipGetLastError();
}

}  // namespace pwc
