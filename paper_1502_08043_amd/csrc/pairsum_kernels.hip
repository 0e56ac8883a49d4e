// Uniform-electron-gas pair sums (Sec. III), one spin channel:
//   E_x = -1/2 sum_{i,j} f_i f_j <ij|ji>,  E_H = 1/2 sum_{i,j} f_i f_j <ij|ij>.
// For planewaves <ij|ji> depends on Delta = n_j - n_i only through the
// diagonal entries tau_q(Delta_d, -Delta_d), which are even in Delta_d, so the
// exchange kernel K(Delta) = sum_q W_q D_q(|Dx|) D_q(|Dy|) D_q(|Dz|) reads a
// (K+1) x Q table that fits in LDS (three of them for a box, one per
// direction).  <ij|ij> has m = m' = 0 in every
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
#include <algorithm>
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
    const void *diag;   // [nchunk][ndir][K+1][dc] double or float2
    const void *w;      // [nchunk * dc]     double or float2
    int K, dc, nchunk, nT;
    int ndir;           // 3 for a box (one diagonal table per direction), else 1
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
        raise_error(a.err);
        return false;
    }
    const int vi = a.basis[oi], vj = a.basis[oj];
    const int dstride = a.ndir == 3 ? (a.K + 1) * a.dc : 0;   // a box: per-direction tables
    ax = iabs(bx(vj) - bx(vi)) * a.dc;
    ay = iabs(by(vj) - by(vi)) * a.dc + dstride;
    az = iabs(bz(vj) - bz(vi)) * a.dc + 2 * dstride;
    const double fi = a.f ? a.f[i] : 1.0, fj = a.f ? a.f[j] : 1.0;
    wf = (i == j ? 1.0 : 2.0) * fi * fj;
    return true;
}

template <typename T>
__device__ __forceinline__ void stage_diag(const PairArgs &a, int ch, T *ld, T *lw) {
    const int n = a.ndir * (a.K + 1) * a.dc;
    const T *src = static_cast<const T *>(a.diag) + static_cast<size_t>(ch) * n;
    for (int i = threadIdx.x; i < n; i += kThreads) ld[i] = src[i];
    const T *ws = static_cast<const T *>(a.w) + static_cast<size_t>(ch) * a.dc;
    for (int i = threadIdx.x; i < a.dc; i += kThreads) lw[i] = ws[i];
}

__global__ __launch_bounds__(kThreads) void k_pair_f64(PairArgs a) {
    extern __shared__ uint4 lds_raw[];
    __shared__ double red[kThreads / 64];
    double *ld = reinterpret_cast<double *>(lds_raw);
    double *lw = ld + a.ndir * (a.K + 1) * a.dc;
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
    float2 *lw = ld + a.ndir * (a.K + 1) * a.dc;
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

// Fixed-order FP64 sum of the workgroup partials, then the energies:
// E_x = -1/2 pref S_x, E_H = 1/2 pref <00|00>_raw S_h, with
// <00|00>_raw = sum_q W_q tau^x_q(0,0) tau^y_q(0,0) tau^z_q(0,0) read from c0
// when given, else summed here from the FP64 diagonal tables.
__global__ __launch_bounds__(kThreads) void k_pair_final(const double *__restrict__ partial,
                                                        int nblk, const double *__restrict__ c0p,
                                                        const double *__restrict__ diag,
                                                        const double *__restrict__ wd, int K,
                                                        int dc, int nchunk, int ndir, double pref,
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
        if (c0p) {
            c0 = *c0p;
        } else {
            for (int ch = 0; ch < nchunk; ++ch)
                for (int q = 0; q < dc; ++q) {
                    const size_t base = static_cast<size_t>(ch) * ndir * (K + 1) * dc + q;
                    const size_t step = ndir == 3 ? static_cast<size_t>(K + 1) * dc : 0;
                    const double dx = diag[base], dy = diag[base + step], dz = diag[base + 2 * step];
                    c0 = fma(dx * dy * dz, wd[ch * dc + q], c0);
                }
        }
        out[0] = 0.5 * pref * c0 * sh;
        out[1] = -0.5 * pref * sx;
    }
}

// ---------------------------------------------------------------------------
// Exchange through the kernel table K(a, b, c) = sum_q W_q D_q(a) D_q(b) D_q(c),
// a <= b <= c = the sorted |Delta_d| (the summand is symmetric in the three
// directions and even in each Delta_d).  The same sum as the node-sum kernel,
// reassociated: the Q node terms of each distinct Delta are added once, at
// table creation, and each pair costs one LDS gather and one FMA.

// Position of the sorted triple a <= b <= c: C(c+2,3) + C(b+1,2) + a.
__device__ __forceinline__ int ktab_index(int a, int b, int c) {
    return c * (c + 1) * (c + 2) / 6 + b * (b + 1) / 2 + a;
}

// kKtLanes lanes per kernel-table entry (a, b, c): lane j sums the node
// slots j * per .. (j + 1) * per - 1 in node order, and a fixed butterfly
// over the 16 lanes adds the partial sums; lane 0 writes.  A cube's
// directions share one diagonal table, so only sorted triples are kept
// (entry tri3(c) + tri2(b) + a); a box keeps every triple, a from the x
// table, b from y and c from z, at (a (K+1) + b) (K+1) + c.
constexpr int kKtLanes = 16;

__global__ __launch_bounds__(kThreads) void k_ktab_build(const double *__restrict__ diag,
                                                        const float2 *__restrict__ diagHL,
                                                        const double *__restrict__ wd,
                                                        const float2 *__restrict__ wdHL, int K,
                                                        int dc, int nchunk, int ndir, int kt_n,
                                                        double *__restrict__ k64,
                                                        double *__restrict__ kmx) {
    const int n1 = K + 1;
    const int gid = blockIdx.x * kThreads + threadIdx.x;
    const int e = gid / kKtLanes, j = gid % kKtLanes;
    if (e >= kt_n) return;                    // whole 16-lane groups leave together
    const bool box = ndir == 3;
    int a, b, c;
    if (box) {
        a = e / (n1 * n1);
        b = (e / n1) % n1;
        c = e % n1;
    } else {
        c = 0;
        while (ktab_index(0, 0, c + 1) <= e) ++c;
        const int r = e - ktab_index(0, 0, c);
        b = 0;
        while ((b + 1) * (b + 2) / 2 <= r) ++b;
        a = r - b * (b + 1) / 2;
    }
    const int ry = box ? n1 : 0, rz = box ? 2 * n1 : 0;   // direction rows in a chunk
    const int slots = dc * nchunk;
    const int per = (slots + kKtLanes - 1) / kKtLanes;
    const int g1 = min(slots, (j + 1) * per);
    double s64 = 0.0;
    float sh = 0.0f, sl = 0.0f;
    for (int g = j * per; g < g1; ++g) {
        const int ch = g / dc, q = g % dc;
        const size_t row = static_cast<size_t>(ch) * ndir * n1;
        const double da = diag[(row + a) * dc + q], db = diag[(row + ry + b) * dc + q];
        const double dcv = diag[(row + rz + c) * dc + q];
        s64 = fma(da * db * dcv, wd[g], s64);
        const float2 ha = diagHL[(row + a) * dc + q], hb = diagHL[(row + ry + b) * dc + q];
        const float2 hc = diagHL[(row + rz + c) * dc + q], hw = wdHL[g];
        ff_acc(sh, sl, ff_mul(ff_mul(ff_mul(ff{ha.x, ha.y}, ff{hb.x, hb.y}), ff{hc.x, hc.y}),
                              ff{hw.x, hw.y}));
    }
#pragma unroll
    for (int off = kKtLanes / 2; off > 0; off >>= 1) {
        s64 += __shfl_xor(s64, off, kKtLanes);
        const float oh = __shfl_xor(sh, off, kKtLanes), ol = __shfl_xor(sl, off, kKtLanes);
        ff_acc(sh, sl, ff{oh, ol});
    }
    if (j == 0) {
        k64[e] = s64;
        kmx[e] = ff_to_double(sh, sl);
    }
}

constexpr int kKtTile = 64;                      // 64 x 64 pairs per tile
constexpr int kKtRows = kKtTile * kKtTile / kThreads;   // 16 pairs per lane

struct KtArgs {
    const int32_t *occ;
    const double *f;
    int M;
    const int32_t *basis;
    int N;
    const double *ktab;
    int kt_n;
    int nT;
    int box;           // unsorted (K+1)^3 table of a box
    int n1;            // K + 1
    double *partial;   // [gridDim.x][2]
    int *err;
};

__device__ __forceinline__ void sort3(int &a, int &b, int &c) {
    int t;
    if (a > b) { t = a; a = b; b = t; }
    if (b > c) { t = b; b = c; c = t; }
    if (a > b) { t = a; a = b; b = t; }
}

// Persistent workgroups walk the upper-triangle tiles of the pair matrix in
// a fixed order; the kernel table is staged in LDS once per workgroup.  The
// 128 row and column vectors of a tile come through a two-stage pipeline:
// while tile t is summed, the basis vectors of the next tile (whose
// occupied indices are at hand) and the occupied indices of the one after
// are in flight.
__global__ __launch_bounds__(kThreads) void k_pair_ktab(KtArgs a) {
    extern __shared__ uint4 lds_raw[];
    double *lk = reinterpret_cast<double *>(lds_raw);
    __shared__ int vi_s[kKtTile], vj_s[kKtTile];
    __shared__ double fi_s[kKtTile], fj_s[kKtTile];
    __shared__ double red[kThreads / 64];
    for (int i = threadIdx.x; i < a.kt_n; i += kThreads) lk[i] = a.ktab[i];
    double sx = 0.0, sh = 0.0;   // diagonal and partial tiles, coefficients applied
    double so = 0.0, ho = 0.0;   // full tiles above the diagonal, coefficient 2 pending
    const int jl = threadIdx.x % kKtTile, i0 = (threadIdx.x / kKtTile) * kKtRows;
    const int ntile = a.nT * a.nT, G = gridDim.x;
    // The first tile at or after t on this workgroup's stride with ti <= tj.
    auto valid_from = [&](int t) {
        while (t < ntile && t / a.nT > t % a.nT) t += G;
        return t;
    };
    // Lanes 0..63 stage the tile's rows, 64..127 its columns.
    const bool stager = threadIdx.x < 2 * kKtTile, row = threadIdx.x < kKtTile;
    const int l = row ? threadIdx.x : threadIdx.x - kKtTile;
    // Stage 2: this lane's occupied index and weight in tile t.
    auto load_occ = [&](int t, bool &have, int &o, double &w) {
        have = false;
        o = 0;
        w = 0.0;
        if (!stager || t >= ntile) return;
        const int ti = t / a.nT, tj = t - ti * a.nT;
        const int idx = (row ? ti : tj) * kKtTile + l;
        if (idx >= a.M) return;
        have = true;
        o = a.occ[idx];
        w = a.f ? a.f[idx] : 1.0;
    };
    // Stage 1: its basis vector (a bad index poisons the energies).
    auto load_vec = [&](bool have, int o, double w, int &v, double &wv) {
        v = 0;
        wv = 0.0;
        if (!have) return;
        if (static_cast<unsigned>(o) < static_cast<unsigned>(a.N)) {
            v = a.basis[o];
            wv = w;
        } else {
            raise_error(a.err);
            wv = NAN;
        }
    };
    int t = valid_from(blockIdx.x);
    bool h1;
    int o1, cv;
    double w1, cw;
    load_occ(t, h1, o1, w1);
    load_vec(h1, o1, w1, cv, cw);
    int t1 = valid_from(t + G);
    load_occ(t1, h1, o1, w1);
    while (t < ntile) {
        const int ti = t / a.nT, tj = t - ti * a.nT;
        __syncthreads();                              // previous tile's vectors consumed
        if (stager) {
            if (row) {
                vi_s[l] = cv;
                fi_s[l] = cw;
            } else {
                vj_s[l] = cv;
                fj_s[l] = cw;
            }
        }
        // (a tile holding a bad index takes the weighted path, whose NaN
        // weight poisons the energies)
        const bool poisoned = __syncthreads_or(stager && isnan(cw));
        int nv;
        double nw;
        load_vec(h1, o1, w1, nv, nw);                 // tile t1's vectors
        const int t2 = valid_from(t1 + G);
        load_occ(t2, h1, o1, w1);                     // tile t2's indices
        const int vj = vj_s[jl];
        const double fj = fj_s[jl];
        const int j = tj * kKtTile + jl;
        const int jx = (vj << 24) >> 24, jy = (vj << 16) >> 24, jz = (vj << 8) >> 24;
        if (ti < tj && (tj + 1) * kKtTile <= a.M && !poisoned) {
            // A full tile above the diagonal: every pair has i < j, so its
            // coefficient 2 is applied once at the end.  Row il is the same
            // for all lanes of a wave.
#pragma unroll 4
            for (int k = 0; k < kKtRows; ++k) {
                const int il = i0 + k;
                const int vi = __builtin_amdgcn_readfirstlane(vi_s[il]);
                const int dx = abs(jx - ((vi << 24) >> 24));
                const int dy = abs(jy - ((vi << 16) >> 24));
                const int dz = abs(jz - ((vi << 8) >> 24));
                int kidx;
                if (a.box) {
                    kidx = (dx * a.n1 + dy) * a.n1 + dz;
                } else {
                    const int lo = min(min(dx, dy), dz), hi = max(max(dx, dy), dz);
                    kidx = ktab_index(lo, dx + dy + dz - lo - hi, hi);
                }
                if (a.f) {
                    const double fi = fi_s[il];
                    so = fma(fi * fj, lk[kidx], so);
                    ho = fma(fi, fj, ho);
                } else {
                    so += lk[kidx];
                }
            }
            if (!a.f) ho += static_cast<double>(kKtRows);
        } else {
#pragma unroll 4
            for (int k = 0; k < kKtRows; ++k) {
                const int il = i0 + k, i = ti * kKtTile + il;
                const int vi = vi_s[il];
                int dx = jx - ((vi << 24) >> 24), dy = jy - ((vi << 16) >> 24), dz = jz - ((vi << 8) >> 24);
                dx = dx < 0 ? -dx : dx;
                dy = dy < 0 ? -dy : dy;
                dz = dz < 0 ? -dz : dz;
                int kidx;
                if (a.box) {
                    kidx = (dx * a.n1 + dy) * a.n1 + dz;
                } else {
                    sort3(dx, dy, dz);
                    kidx = ktab_index(dx, dy, dz);
                }
                const double wf = (i < j ? 2.0 : (i == j ? 1.0 : 0.0)) * fi_s[il] * fj;
                sx = fma(wf, lk[kidx], sx);
                sh += wf;
            }
        }
        t = t1;
        t1 = t2;
        cv = nv;
        cw = nw;
    }
    sx = block_sum(fma(2.0, so, sx), red);
    sh = block_sum(fma(2.0, ho, sh), red);
    if (threadIdx.x == 0) {
        a.partial[2 * blockIdx.x] = sx;
        a.partial[2 * blockIdx.x + 1] = sh;
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

hipError_t launch_ktab_build(Table &t, hipStream_t s) {
    if (t.kt_n == 0) return hipSuccess;
    const int64_t threads = static_cast<int64_t>(t.kt_n) * kKtLanes;
    const int blocks = static_cast<int>((threads + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_ktab_build, dim3(blocks), dim3(kThreads), 0, s, t.d_diag, t.d_diagHL,
                       t.d_Wdiag, t.d_WdiagHL, t.K, t.dl.c, t.dl.nchunk, t.ndir, t.kt_n,
                       t.d_ktab64, t.d_ktabMX);
    return hipGetLastError();
}

// Grid of the kernel-table pair sum for M occupied orbitals (its partials
// take 2 doubles per workgroup).
static int ktab_grid(const Table &t, int64_t M) {
    const size_t lds = sizeof(double) * static_cast<size_t>(t.kt_n);
    const int per_cu = std::max(1, std::min(8, static_cast<int>((kLdsMax - 4096) / std::max<size_t>(lds, 1))));
    const int64_t nT = (M + kKtTile - 1) / kKtTile;
    return static_cast<int>(std::min<int64_t>(nT * (nT + 1) / 2, int64_t(t.n_cu) * per_cu));
}

size_t energies_scratch_bytes(const Table &t, int64_t M, pwc_pair_algo algo) {
    if (M <= 0) return 0;
    if (algo != PWC_PAIR_NODESUM && t.kt_n > 0) return sizeof(double) * 2 * static_cast<size_t>(ktab_grid(t, M));
    const size_t nT = static_cast<size_t>((M + kTile - 1) / kTile);
    return sizeof(double) * 2 * nT * nT;
}

hipError_t launch_energies(const Table &t, const int32_t *d_occ, const double *d_f, int64_t M,
                           pwc_precision p, pwc_pair_algo algo, double *d_out, hipStream_t s,
                           int *d_err) {
    if (M <= 0) {
        hipLaunchKernelGGL(k_zero2, dim3(1), dim3(64), 0, s, d_out);
        return hipGetLastError();
    }
    const double pref = 1.0 / (std::sqrt(M_PI) * t.L);
    int *const err_word = d_err ? d_err : t.d_err;
    hipError_t err;
    // The partials are freed on every path once the kernels are enqueued.
    auto finish = [&](double *partial, hipError_t e) {
        const hipError_t ef = hipFreeAsync(partial, s);
        return e != hipSuccess ? e : ef;
    };
    if (algo != PWC_PAIR_NODESUM && t.kt_n > 0) {
        KtArgs a{};
        a.occ = d_occ;
        a.f = d_f;
        a.M = static_cast<int>(M);
        a.basis = t.d_basis;
        a.N = static_cast<int>(t.N);
        a.ktab = (p == PWC_MIXED) ? t.d_ktabMX : t.d_ktab64;
        a.kt_n = t.kt_n;
        a.box = t.ndir == 3;
        a.n1 = t.K + 1;
        a.nT = static_cast<int>((M + kKtTile - 1) / kKtTile);
        a.err = err_word;
        const size_t lds = sizeof(double) * static_cast<size_t>(t.kt_n);
        const int grid = ktab_grid(t, M);
        double *partial = nullptr;
        err = hipMallocAsync(reinterpret_cast<void **>(&partial), sizeof(double) * 2 * grid, s);
        if (err != hipSuccess) return err;
        a.partial = partial;
        err = set_lds(k_pair_ktab, lds);
        if (err == hipSuccess) {
            hipLaunchKernelGGL(k_pair_ktab, dim3(grid), dim3(kThreads), lds, s, a);
            err = hipGetLastError();
        }
        if (err == hipSuccess) {
            hipLaunchKernelGGL(k_pair_final, dim3(1), dim3(kThreads), 0, s, partial, grid, a.ktab,
                               t.d_diag, t.d_Wdiag, t.K, t.dl.c, t.dl.nchunk, t.ndir, pref, d_out);
            err = hipGetLastError();
        }
        return finish(partial, err);
    }
    if (algo == PWC_PAIR_KTABLE) return hipErrorInvalidValue;   // table too large for LDS
    PairArgs a{};
    a.occ = d_occ;
    a.f = d_f;
    a.M = static_cast<int>(M);
    a.basis = t.d_basis;
    a.N = static_cast<int>(t.N);
    a.K = t.K;
    a.dc = t.dl.c;
    a.nchunk = t.dl.nchunk;
    a.ndir = t.ndir;
    a.nT = static_cast<int>((M + kTile - 1) / kTile);
    a.err = err_word;
    const int nblk = a.nT * a.nT;
    double *partial = nullptr;
    err = hipMallocAsync(reinterpret_cast<void **>(&partial),
                         sizeof(double) * 2 * static_cast<size_t>(nblk), s);
    if (err != hipSuccess) return err;
    a.partial = partial;
    const size_t lds = (static_cast<size_t>(a.ndir) * (a.K + 1) * a.dc + a.dc) * 8;
    const dim3 grid(a.nT, a.nT);
    if (p == PWC_MIXED) {
        a.diag = t.d_diagHL;
        a.w = t.d_WdiagHL;
        err = set_lds(k_pair_mixed, lds);
        if (err == hipSuccess) hipLaunchKernelGGL(k_pair_mixed, grid, dim3(kThreads), lds, s, a);
    } else {
        a.diag = t.d_diag;
        a.w = t.d_Wdiag;
        err = set_lds(k_pair_f64, lds);
        if (err == hipSuccess) hipLaunchKernelGGL(k_pair_f64, grid, dim3(kThreads), lds, s, a);
    }
    if (err == hipSuccess) err = hipGetLastError();
    if (err == hipSuccess) {
        hipLaunchKernelGGL(k_pair_final, dim3(1), dim3(kThreads), 0, s, partial, nblk,
                           static_cast<const double *>(nullptr), t.d_diag, t.d_Wdiag, t.K, t.dl.c,
                           t.dl.nchunk, t.ndir, pref, d_out);
        err = hipGetLastError();
    }
    return finish(partial, err);
}

}  // namespace pwc
