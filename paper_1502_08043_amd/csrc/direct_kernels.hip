// Direct reconstruction of <ij|kl> (Eq. 14) for small quadruple lists, many
// requests per launch.
//
// The node-pass kernels stage an [E][c] slab per workgroup and pass, which
// costs a fixed few tens of microseconds per call: right for streams of
// millions of quadruples, wasteful for a request of ten thousand.  Here four
// lanes evaluate one quadruple over all Q nodes, reading its three folded
// rows (W_q^(1/3) tau_q, Q contiguous values each) from global memory, where
// a table of a few hundred KB stays in L2 for the whole launch.  Jobs - one
// per request, each with its own table, precision, quadruples and outputs -
// travel by value in the kernel arguments, so requests on different boxes,
// cutoffs and meshes share one launch: block b works for the job whose block
// range holds b.
#include <cmath>

#include "ffloat.h"
#include "pwc_internal.h"

namespace pwc {
namespace {

constexpr int kDirectThreads = 256;
constexpr int kDirectLanes = 4;                          // lanes per quadruple
constexpr int kDirectQuads = kDirectThreads / kDirectLanes;

__device__ __forceinline__ int sx(int v) { return (v << 24) >> 24; }
__device__ __forceinline__ int sy(int v) { return (v << 16) >> 24; }
__device__ __forceinline__ int sz(int v) { return (v << 8) >> 24; }

// Sum over the 4 lanes of a DPP quad: quad_perm (1,0,3,2), then (2,3,0,1).
template <int CTRL>
__device__ __forceinline__ double quad_take(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// Four lanes share a quadruple: lane s takes node pairs s, s + 4, ..., so the
// quad reads 64 contiguous bytes of each row per step.
__global__ __launch_bounds__(kDirectThreads) void k_rec_direct(DirectBatch b) {
    int j = 0;
    for (int i = 1; i < b.njobs; ++i)
        if (b.job[i].block0 <= blockIdx.x) j = i;
    const DirectJob &J = b.job[j];
    const int s = threadIdx.x % kDirectLanes;
    const int64_t e = static_cast<int64_t>(blockIdx.x - J.block0) * kDirectQuads + threadIdx.x / kDirectLanes;
    if (e >= J.n) return;                                // whole quads leave together
    const int4 v = reinterpret_cast<const int4 *>(J.quads)[e];
    const unsigned N = static_cast<unsigned>(J.N);
    if (static_cast<unsigned>(v.x) >= N || static_cast<unsigned>(v.y) >= N ||
        static_cast<unsigned>(v.z) >= N || static_cast<unsigned>(v.w) >= N) {
        if (s == 0) {
            raise_error(J.err);
            J.out[e] = NAN;
        }
        return;
    }
    const int ni = J.basis[v.x], nj = J.basis[v.y], nk = J.basis[v.z], nl = J.basis[v.w];
    const int K = J.K, nd = J.nd;
    // A box stacks its direction tables: y at rows E1.., z at rows 2 E1...
    const int f0 = J.fold[(sx(nk) - sx(ni) + K) * nd + (sx(nl) - sx(nj) + K)];
    const int f1 = J.fold[(sy(nk) - sy(ni) + K) * nd + (sy(nl) - sy(nj) + K)] + J.ystride;
    const int f2 = J.fold[(sz(nk) - sz(ni) + K) * nd + (sz(nl) - sz(nj) + K)] + 2 * J.ystride;
    double r;
    if (J.mixed == 2) {   // single FP32 table: four nodes per word, word sums in FP32
        const int words = (J.Q + 3) / 4;
        const size_t row = static_cast<size_t>(J.Qp / 4);
        const float4 *x = static_cast<const float4 *>(J.tab) + f0 * row;
        const float4 *y = static_cast<const float4 *>(J.tab) + f1 * row;
        const float4 *z = static_cast<const float4 *>(J.tab) + f2 * row;
        double acc = 0.0;
#pragma unroll 2
        for (int w = s; w < words; w += kDirectLanes) {
            const float4 a = x[w], c = y[w], d = z[w];
            // the node passes' word sum: two pairs, each a rounded triple
            // product added into the other by a fused multiply-add
            const float s01 = fmaf(a.x * c.x, d.x, (a.y * c.y) * d.y);
            const float s23 = fmaf(a.z * c.z, d.z, (a.w * c.w) * d.w);
            acc += static_cast<double>(s01 + s23);
        }
        r = acc;
    } else if (!J.mixed) {
        const int words = (J.Q + 1) / 2;            // node pairs; entries past Q are zero
        const size_t row = static_cast<size_t>(J.Qp / 2);
        const double2 *x = static_cast<const double2 *>(J.tab) + f0 * row;
        const double2 *y = static_cast<const double2 *>(J.tab) + f1 * row;
        const double2 *z = static_cast<const double2 *>(J.tab) + f2 * row;
        double acc = 0.0;
#pragma unroll 4
        for (int w = s; w < words; w += kDirectLanes) {
            const double2 a = x[w], c = y[w], d = z[w];
            acc = fma(a.x * c.x, d.x, acc);
            acc = fma(a.y * c.y, d.y, acc);
        }
        r = acc;
    } else {
        const int words = (J.Q + 1) / 2;
        const size_t row = static_cast<size_t>(J.Qp / 2);
        const float4 *x = static_cast<const float4 *>(J.tab) + f0 * row;
        const float4 *y = static_cast<const float4 *>(J.tab) + f1 * row;
        const float4 *z = static_cast<const float4 *>(J.tab) + f2 * row;
        float h = 0.0f, l = 0.0f;
#pragma unroll 2
        for (int w = s; w < words; w += kDirectLanes) {
            const float4 a = x[w], c = y[w], d = z[w];
            ff_acc(h, l, ff_mul(ff_mul(ff{a.x, a.y}, ff{c.x, c.y}), ff{d.x, d.y}));
            ff_acc(h, l, ff_mul(ff_mul(ff{a.z, a.w}, ff{c.z, c.w}), ff{d.z, d.w}));
        }
        r = ff_to_double(h, l);
    }
    r += quad_take<0xB1>(r);
    r += quad_take<0x4E>(r);
    if (s == 0) J.out[e] = r * J.pref;
}

}  // namespace

DirectJob direct_job(const Table &t, const int32_t *d_quads, int64_t n, double *d_out,
                     pwc_precision p, int *d_err) {
    DirectJob j{};
    j.quads = d_quads;
    j.out = d_out;
    j.n = n;
    j.mixed = p == PWC_MIXED ? 1 : p == PWC_FP32 ? 2 : 0;
    j.tab = p == PWC_MIXED ? static_cast<const void *>(t.d_tauHL)
            : p == PWC_FP32 ? static_cast<const void *>(t.d_tau32) : static_cast<const void *>(t.d_tauF);
    j.basis = t.d_basis;
    j.fold = t.d_fold;
    j.err = d_err ? d_err : t.d_err;
    j.pref = 1.0 / (std::sqrt(M_PI) * t.L);
    j.N = static_cast<int>(t.N);
    j.K = t.K;
    j.nd = t.nd;
    j.Qp = t.fl.Qp;
    j.Q = t.Q;
    j.ystride = t.ndir == 3 ? t.E1 : 0;
    return j;
}

hipError_t launch_direct(DirectBatch b, hipStream_t s) {
    if (b.njobs < 1 || b.njobs > kDirectMaxJobs) return hipErrorInvalidValue;
    uint32_t blocks = 0;
    for (int i = 0; i < b.njobs; ++i) {
        if (b.job[i].n < 0 || b.job[i].n > kDirectMaxN) return hipErrorInvalidValue;
        b.job[i].block0 = blocks;
        blocks += static_cast<uint32_t>((b.job[i].n + kDirectQuads - 1) / kDirectQuads);
    }
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rec_direct, dim3(blocks), dim3(kDirectThreads), 0, s, b);
    return hipGetLastError();
}

}  // namespace pwc
