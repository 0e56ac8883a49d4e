// Separable s-type Gaussian basis (Sec. II): tables and reconstruction.
//
// One-dimensional functions f_u(x) = (2 a_u / pi)^{1/4} exp(-a_u (x - A_u)^2),
// the same set along x, y and z; basis function I = (l n1 + m) n1 + n is
// f_l(x) f_m(y) f_n(z).  A kept pair (u, v) (u <= v, see the host set-up in
// api.cpp) has the product c exp(-p (x - P)^2).  With s = 1/(beta L^2) in
// 1/r = pi^{-1/2} Int s^{-1/2} exp(-s r^2) ds, each direction contributes the
// table entry
//   tau_q(x, y) = c_x c_y pi / sqrt(p_x p_y beta_q + (p_x + p_y)/L^2)
//                 * exp(-p_x p_y (P_x - P_y)^2 / (p_x p_y beta_q L^2 + p_x + p_y))
// (two Gaussian integrals after the Gaussian product theorem), and
//   <ij|kl> = (1/(sqrt(pi) L)) sum_q W_q tau_q(x_x, y_x) tau_q(x_y, y_y) tau_q(x_z, y_z)
// (Eq. 14), x_d the pair of (i, k) and y_d that of (j, l) along d.  The
// entry is symmetric in (x, y), so the folded table keeps x <= y:
// P1 (P1 + 1)/2 rows of Qp node values, W_q^(1/3) folded in as for
// planewaves.  An integral that needs a dropped pair is zero.
//
// Reconstruction reads the three folded rows from global memory (a table of
// a few MB stays in L2 and the last-level cache): four lanes per quadruple,
// each taking every fourth node pair, summed by DPP inside the quad, as the
// planewave direct kernel does; a persistent grid strides over the list.
// The pair map (n1^2 entries) sits in LDS when it fits.
#include <algorithm>
#include <cmath>

#include "ffloat.h"
#include "pwc_internal.h"

namespace pwc {
namespace {

constexpr int kGtThreads = 256;

struct GaussTabArgs {
    const double *pair;   // [P1][3] (c, p, P)
    const double *beta;   // [Q]
    const double *wcbrt;  // [Q]
    int P1, Q, Qp;
    double L2;            // L^2
    double *tau;          // [Q][P1][P1]
    double *tauF;         // [E][Qp]
    float2 *tauHL;        // [E][Qp]
};

__device__ __forceinline__ float2 split_hl(double v) {
    const float hi = static_cast<float>(v);
    return make_float2(hi, static_cast<float>(v - static_cast<double>(hi)));
}

// Grid (ceil(P1^2 / 256), Q): one (x, y) entry of node q per lane.
__global__ __launch_bounds__(kGtThreads) void k_gauss_tables(GaussTabArgs a) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * kGtThreads + threadIdx.x;
    const int q = blockIdx.y;
    const int64_t n2 = static_cast<int64_t>(a.P1) * a.P1;
    if (e >= n2) return;
    const int x = static_cast<int>(e / a.P1), y = static_cast<int>(e % a.P1);
    const double cx = a.pair[3 * x], px = a.pair[3 * x + 1], Px = a.pair[3 * x + 2];
    const double cy = a.pair[3 * y], py = a.pair[3 * y + 1], Py = a.pair[3 * y + 2];
    // Written so that (x, y) and (y, x) round alike.
    const double pq = px * py, ps = px + py, d = Px - Py;
    const double b = a.beta[q];
    const double v = (cx * cy) * M_PI / sqrt(pq * b + ps / a.L2) * exp(-pq * (d * d) / (pq * b * a.L2 + ps));
    a.tau[(static_cast<size_t>(q) * a.P1 + x) * a.P1 + y] = v;
    if (x <= y) {
        const size_t f = static_cast<size_t>(y) * (y + 1) / 2 + x;
        const double vw = v * a.wcbrt[q];
        a.tauF[f * a.Qp + q] = vw;
        a.tauHL[f * a.Qp + q] = split_hl(vw);
    }
}

struct GaussRecArgs {
    const int4 *quads;
    int64_t n;
    const int32_t *pmap;   // [n1][n1]
    int n1, P1;
    int lds_map;           // the pair map is copied to LDS
    const void *tab;       // [E][Qp] double or float2
    int Q, Qp, mixed;
    double pref;
    double *out;
    int *err;
};

constexpr int kGrLanes = 4;
constexpr int kGrQuads = kGtThreads / kGrLanes;

template <int CTRL>
__device__ __forceinline__ double quad_take(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ int fold_pair(int x, int y) {
    const int lo = min(x, y), hi = max(x, y);
    return hi * (hi + 1) / 2 + lo;
}

__global__ __launch_bounds__(kGtThreads) void k_rec_gauss(GaussRecArgs a) {
    extern __shared__ int32_t lmap[];
    const int32_t *pmap = a.pmap;
    if (a.lds_map) {
        for (int i = threadIdx.x; i < a.n1 * a.n1; i += kGtThreads) lmap[i] = a.pmap[i];
        __syncthreads();
        pmap = lmap;
    }
    const int s = threadIdx.x % kGrLanes;
    const unsigned n1 = static_cast<unsigned>(a.n1);
    const unsigned N = n1 * n1 * n1;
    const int words = (a.Q + 1) / 2;                 // node pairs; entries past Q are zero
    const size_t row = static_cast<size_t>(a.Qp / 2);
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kGrQuads;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * kGrQuads + threadIdx.x / kGrLanes; e < a.n;
         e += stride) {
        const int4 v = a.quads[e];
        if (static_cast<unsigned>(v.x) >= N || static_cast<unsigned>(v.y) >= N ||
            static_cast<unsigned>(v.z) >= N || static_cast<unsigned>(v.w) >= N) {
            if (s == 0) {
                raise_error(a.err);
                a.out[e] = NAN;
            }
            continue;
        }
        // One-dimensional indices of i, j, k, l along z (fastest), y, x.
        unsigned ii = v.x, jj = v.y, kk = v.z, ll = v.w;
        int f[3];
        bool kept = true;
#pragma unroll
        for (int d = 2; d >= 0; --d) {
            const unsigned li = ii % n1, lj = jj % n1, lk = kk % n1, lq = ll % n1;
            ii /= n1;
            jj /= n1;
            kk /= n1;
            ll /= n1;
            const int x = pmap[li * n1 + lk], y = pmap[lj * n1 + lq];   // (i, k) at r, (j, l) at r'
            kept = kept && x >= 0 && y >= 0;
            f[d] = kept ? fold_pair(x, y) : 0;
        }
        double r = 0.0;
        if (kept) {   // uniform across the quad: its four lanes share e
            if (!a.mixed) {
                const double2 *X = static_cast<const double2 *>(a.tab) + f[0] * row;
                const double2 *Y = static_cast<const double2 *>(a.tab) + f[1] * row;
                const double2 *Z = static_cast<const double2 *>(a.tab) + f[2] * row;
                double acc = 0.0;
                for (int w = s; w < words; w += kGrLanes) {
                    const double2 p = X[w], q = Y[w], t = Z[w];
                    acc = fma(p.x * q.x, t.x, acc);
                    acc = fma(p.y * q.y, t.y, acc);
                }
                r = acc;
            } else {
                const float4 *X = static_cast<const float4 *>(a.tab) + f[0] * row;
                const float4 *Y = static_cast<const float4 *>(a.tab) + f[1] * row;
                const float4 *Z = static_cast<const float4 *>(a.tab) + f[2] * row;
                float h = 0.0f, l = 0.0f;
                for (int w = s; w < words; w += kGrLanes) {
                    const float4 p = X[w], q = Y[w], t = Z[w];
                    ff_acc(h, l, ff_mul(ff_mul(ff{p.x, p.y}, ff{q.x, q.y}), ff{t.x, t.y}));
                    ff_acc(h, l, ff_mul(ff_mul(ff{p.z, p.w}, ff{q.z, q.w}), ff{t.z, t.w}));
                }
                r = ff_to_double(h, l);
            }
        }
        r += quad_take<0xB1>(r);
        r += quad_take<0x4E>(r);
        if (s == 0) a.out[e] = kept ? r * a.pref : 0.0;
    }
}

}  // namespace

hipError_t launch_gauss_tables(const Table &t, hipStream_t s) {
    GaussTabArgs a{};
    a.pair = t.d_pair;
    a.beta = t.d_beta;
    a.wcbrt = t.d_Wcbrt;
    a.P1 = t.P1;
    a.Q = t.Q;
    a.Qp = t.fl.Qp;
    a.L2 = t.L * t.L;
    a.tau = t.d_tau;
    a.tauF = t.d_tauF;
    a.tauHL = t.d_tauHL;
    const int64_t n2 = static_cast<int64_t>(t.P1) * t.P1;
    const int64_t bx = (n2 + kGtThreads - 1) / kGtThreads;
    if (bx > int64_t(0x7fffffff) || t.Q > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gauss_tables, dim3(static_cast<unsigned>(bx), t.Q), dim3(kGtThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_rec_gauss(const Table &t, const int32_t *d_quads, int64_t n, double *d_out,
                            pwc_precision p, hipStream_t s, int *d_err) {
    if (n <= 0) return hipSuccess;
    GaussRecArgs a{};
    a.quads = reinterpret_cast<const int4 *>(d_quads);
    a.n = n;
    a.pmap = t.d_pmap;
    a.n1 = t.n1;
    a.P1 = t.P1;
    a.mixed = p == PWC_MIXED;
    a.tab = a.mixed ? static_cast<const void *>(t.d_tauHL) : static_cast<const void *>(t.d_tauF);
    a.Q = t.Q;
    a.Qp = t.fl.Qp;
    a.pref = 1.0 / (std::sqrt(M_PI) * t.L);
    a.out = d_out;
    a.err = d_err ? d_err : t.d_err;
    const size_t map_bytes = sizeof(int32_t) * static_cast<size_t>(t.n1) * t.n1;
    a.lds_map = map_bytes <= size_t(64) << 10;
    const size_t lds = a.lds_map ? map_bytes : 0;
    const int64_t blocks = std::min<int64_t>((n + kGrQuads - 1) / kGrQuads, int64_t(t.n_cu) * 8);
    hipLaunchKernelGGL(k_rec_gauss, dim3(static_cast<unsigned>(blocks)), dim3(kGtThreads), lds, s, a);
    return hipGetLastError();
}

}  // namespace pwc
