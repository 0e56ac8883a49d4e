// Uniform-electron-gas pair sums (Sec. III), one spin channel:
//   E_x = -1/2 sum_{i,j} f_i f_j <ij|ji>,  E_H = 1/2 sum_{i,j} f_i f_j <ij|ij>.
// For planewaves <ij|ji> depends on Delta = n_j - n_i only through the
// diagonal entries tau_q(Delta_d, -Delta_d), which are even in Delta_d, so the
// exchange kernel K(Delta) = sum_q W_q D_q(|Dx|) D_q(|Dy|) D_q(|Dz|) reads a
// (K+1) x Q table that fits in LDS.  <ij|ij> has m = m' = 0 in every
// direction and equals the single integral <00|00> for every pair; its pair
// sum is carried as sum f_i f_j and multiplied by <00|00> at the end.
//
// The summand is symmetric in (i, j), so each workgroup takes one 32 x 32
// tile of the upper triangle of the pair matrix (diagonal tiles drop i > j;
// off-diagonal pairs count twice).  Lanes hold 4 pairs each; per-pair node
// sums run out of LDS; the two per-tile sums are reduced by wavefront
// shuffles and LDS in a fixed order and written to a per-tile partial.  A
// single workgroup then adds the partials in a fixed order in FP64, so the
// energies are bitwise reproducible for a given input.
#include <cmath>

#include "ffloat.h"
#include "pwc_internal.h"

namespace pwc {
namespace {

constexpr int kThreads = 256;
constexpr int kTile = 32;
constexpr int kPairs = kTile * kTile / kThreads;   // 4

struct PairArgs {
    const int32_t *occ;
    const double *f;
    int M;
    const int32_t *basis;
    int N;
    const void *diag;   // [nchunk][K+1][dc] double or float2
    const void *w;      // [nchunk * dc]     double or float2
    int K, dc, nchunk, nT;
    double *partial;    // [nT * nT][2]
    int *err;           // table error word
};

__device__ __forceinline__ int bx(int v) { return (v << 24) >> 24; }
__device__ __forceinline__ int by(int v) { return (v << 16) >> 24; }
__device__ __forceinline__ int bz(int v) { return (v << 8) >> 24; }
__device__ __forceinline__ int iabs(int v) { return v < 0 ? -v : v; }

// Fixed-order block sum; the result is valid in thread 0.
__device__ double block_sum(double v, double *red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < kThreads / 64; ++k) s += red[k];
    return s;
}

// Per-lane pair set-up shared by both precisions.  Offsets are |Delta_d| * dc.
__device__ __forceinline__ bool pair_setup(const PairArgs &a, int ti, int tj, int p, int &ax,
                                           int &ay, int &az, double &wf) {
    const int idx = threadIdx.x + p * kThreads;
    const int i = ti * kTile + idx / kTile, j = tj * kTile + idx % kTile;
    ax = ay = az = 0;
    wf = 0.0;
    if (i >= a.M || j >= a.M || i > j) return true;
    const int oi = a.occ[i], oj = a.occ[j];
    if (static_cast<unsigned>(oi) >= static_cast<unsigned>(a.N) ||
        static_cast<unsigned>(oj) >= static_cast<unsigned>(a.N)) {
        atomicOr(a.err, 1);
        return false;
    }
    const int vi = a.basis[oi], vj = a.basis[oj];
    ax = iabs(bx(vj) - bx(vi)) * a.dc;
    ay = iabs(by(vj) - by(vi)) * a.dc;
    az = iabs(bz(vj) - bz(vi)) * a.dc;
    const double fi = a.f ? a.f[i] : 1.0, fj = a.f ? a.f[j] : 1.0;
    wf = (i == j ? 1.0 : 2.0) * fi * fj;
    return true;
}

template <typename T>
__device__ __forceinline__ void stage_diag(const PairArgs &a, int ch, T *ld, T *lw) {
    const int n = (a.K + 1) * a.dc;
    const T *src = static_cast<const T *>(a.diag) + static_cast<size_t>(ch) * n;
    for (int i = threadIdx.x; i < n; i += kThreads) ld[i] = src[i];
    const T *ws = static_cast<const T *>(a.w) + static_cast<size_t>(ch) * a.dc;
    for (int i = threadIdx.x; i < a.dc; i += kThreads) lw[i] = ws[i];
}

__global__ __launch_bounds__(kThreads) void k_pair_f64(PairArgs a) {
    extern __shared__ uint4 lds_raw[];
    __shared__ double red[kThreads / 64];
    double *ld = reinterpret_cast<double *>(lds_raw);
    double *lw = ld + (a.K + 1) * a.dc;
    const int ti = blockIdx.y, tj = blockIdx.x;
    const int bid = ti * a.nT + tj;
    if (ti > tj) {   // whole workgroup leaves together
        if (threadIdx.x == 0) {
            a.partial[2 * bid] = 0.0;
            a.partial[2 * bid + 1] = 0.0;
        }
        return;
    }
    int ax[kPairs], ay[kPairs], az[kPairs];
    double wf[kPairs], kq[kPairs];
    bool good = true;
#pragma unroll
    for (int p = 0; p < kPairs; ++p) {
        good &= pair_setup(a, ti, tj, p, ax[p], ay[p], az[p], wf[p]);
        kq[p] = 0.0;
    }
    for (int ch = 0; ch < a.nchunk; ++ch) {
        __syncthreads();
        stage_diag<double>(a, ch, ld, lw);
        __syncthreads();
        for (int q = 0; q < a.dc; q += 2) {
            const double2 w = *reinterpret_cast<const double2 *>(lw + q);
#pragma unroll
            for (int p = 0; p < kPairs; ++p) {
                const double2 x = *reinterpret_cast<const double2 *>(ld + ax[p] + q);
                const double2 y = *reinterpret_cast<const double2 *>(ld + ay[p] + q);
                const double2 z = *reinterpret_cast<const double2 *>(ld + az[p] + q);
                kq[p] = fma(x.x * y.x * z.x, w.x, kq[p]);
                kq[p] = fma(x.y * y.y * z.y, w.y, kq[p]);
            }
        }
    }
    double sx = 0.0, sh = 0.0;
#pragma unroll
    for (int p = 0; p < kPairs; ++p) {
        sx = fma(wf[p], kq[p], sx);
        sh += wf[p];
    }
    if (!good) sx = NAN;
    sx = block_sum(sx, red);
    sh = block_sum(sh, red);
    if (threadIdx.x == 0) {
        a.partial[2 * bid] = sx;
        a.partial[2 * bid + 1] = sh;
    }
}

__global__ __launch_bounds__(kThreads) void k_pair_mixed(PairArgs a) {
    extern __shared__ uint4 lds_raw[];
    __shared__ double red[kThreads / 64];
    float2 *ld = reinterpret_cast<float2 *>(lds_raw);
    float2 *lw = ld + (a.K + 1) * a.dc;
    const int ti = blockIdx.y, tj = blockIdx.x;
    const int bid = ti * a.nT + tj;
    if (ti > tj) {
        if (threadIdx.x == 0) {
            a.partial[2 * bid] = 0.0;
            a.partial[2 * bid + 1] = 0.0;
        }
        return;
    }
    int ax[kPairs], ay[kPairs], az[kPairs];
    double wf[kPairs];
    float kh[kPairs], kl[kPairs];
    bool good = true;
#pragma unroll
    for (int p = 0; p < kPairs; ++p) {
        good &= pair_setup(a, ti, tj, p, ax[p], ay[p], az[p], wf[p]);
        kh[p] = kl[p] = 0.0f;
    }
    for (int ch = 0; ch < a.nchunk; ++ch) {
        __syncthreads();
        stage_diag<float2>(a, ch, ld, lw);
        __syncthreads();
        for (int q = 0; q < a.dc; q += 2) {
            const float4 w = *reinterpret_cast<const float4 *>(lw + q);
#pragma unroll
            for (int p = 0; p < kPairs; ++p) {
                const float4 x = *reinterpret_cast<const float4 *>(ld + ax[p] + q);
                const float4 y = *reinterpret_cast<const float4 *>(ld + ay[p] + q);
                const float4 z = *reinterpret_cast<const float4 *>(ld + az[p] + q);
                ff_acc(kh[p], kl[p],
                       ff_mul(ff_mul(ff_mul(ff{x.x, x.y}, ff{y.x, y.y}), ff{z.x, z.y}), ff{w.x, w.y}));
                ff_acc(kh[p], kl[p],
                       ff_mul(ff_mul(ff_mul(ff{x.z, x.w}, ff{y.z, y.w}), ff{z.z, z.w}), ff{w.z, w.w}));
            }
        }
    }
    double sx = 0.0, sh = 0.0;
#pragma unroll
    for (int p = 0; p < kPairs; ++p) {
        sx = fma(wf[p], ff_to_double(kh[p], kl[p]), sx);
        sh += wf[p];
    }
    if (!good) sx = NAN;
    sx = block_sum(sx, red);
    sh = block_sum(sh, red);
    if (threadIdx.x == 0) {
        a.partial[2 * bid] = sx;
        a.partial[2 * bid + 1] = sh;
    }
}

// Fixed-order FP64 sum of the tile partials, then the energies:
// E_x = -1/2 pref S_x, E_H = 1/2 pref <00|00>_raw S_h, with
// <00|00>_raw = sum_q W_q tau_q(0,0)^3 from the FP64 diagonal table.
__global__ __launch_bounds__(kThreads) void k_pair_final(const double *__restrict__ partial,
                                                        int nblk, const double *__restrict__ diag,
                                                        const double *__restrict__ wd, int K,
                                                        int dc, int nchunk, double pref,
                                                        double *__restrict__ out) {
    __shared__ double red[kThreads / 64];
    double sx = 0.0, sh = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kThreads) {
        sx += partial[2 * b];
        sh += partial[2 * b + 1];
    }
    sx = block_sum(sx, red);
    sh = block_sum(sh, red);
    if (threadIdx.x == 0) {
        double c0 = 0.0;
        for (int ch = 0; ch < nchunk; ++ch)
            for (int q = 0; q < dc; ++q) {
                const double d0 = diag[(static_cast<size_t>(ch) * (K + 1)) * dc + q];
                c0 = fma(d0 * d0 * d0, wd[ch * dc + q], c0);
            }
        out[0] = 0.5 * pref * c0 * sh;
        out[1] = -0.5 * pref * sx;
    }
}

__global__ void k_zero2(double *out) {
    if (threadIdx.x < 2) out[threadIdx.x] = 0.0;
}

template <typename Kern>
hipError_t set_lds(Kern k, size_t bytes) {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                               hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
}

}  // namespace

hipError_t launch_energies(const Table &t, const int32_t *d_occ, const double *d_f, int64_t M,
                           pwc_precision p, double *d_out, hipStream_t s) {
    if (M <= 0) {
        hipLaunchKernelGGL(k_zero2, dim3(1), dim3(64), 0, s, d_out);
        return hipGetLastError();
    }
    PairArgs a{};
    a.occ = d_occ;
    a.f = d_f;
    a.M = static_cast<int>(M);
    a.basis = t.d_basis;
    a.N = static_cast<int>(t.N);
    a.K = t.K;
    a.dc = t.dl.c;
    a.nchunk = t.dl.nchunk;
    a.nT = static_cast<int>((M + kTile - 1) / kTile);
    a.err = t.d_err;
    const int nblk = a.nT * a.nT;
    double *partial = nullptr;
    hipError_t err = hipMallocAsync(reinterpret_cast<void **>(&partial),
                                    sizeof(double) * 2 * static_cast<size_t>(nblk), s);
    if (err != hipSuccess) return err;
    a.partial = partial;
    const size_t lds = (static_cast<size_t>(a.K + 1) * a.dc + a.dc) * 8;
    const dim3 grid(a.nT, a.nT);
    if (p == PWC_MIXED) {
        a.diag = t.d_diagHL;
        a.w = t.d_WdiagHL;
        if ((err = set_lds(k_pair_mixed, lds)) != hipSuccess) return err;
        hipLaunchKernelGGL(k_pair_mixed, grid, dim3(kThreads), lds, s, a);
    } else {
        a.diag = t.d_diag;
        a.w = t.d_Wdiag;
        if ((err = set_lds(k_pair_f64, lds)) != hipSuccess) return err;
        hipLaunchKernelGGL(k_pair_f64, grid, dim3(kThreads), lds, s, a);
    }
    if ((err = hipGetLastError()) != hipSuccess) return err;
    const double pref = 1.0 / (std::sqrt(M_PI) * t.L);
    hipLaunchKernelGGL(k_pair_final, dim3(1), dim3(kThreads), 0, s, partial, nblk, t.d_diag,
                       t.d_Wdiag, t.K, t.dl.c, t.dl.nchunk, pref, d_out);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    return hipFreeAsync(partial, s);
}

}  // namespace pwc
