// Table construction on the GPU (FP64): the 1-D integrals of Eq. 8 for
// planewave factors at every quadrature node, and the layouts the hot
// kernels read.  A rectangular box has one table per direction, built at
// that direction's node beta_q / rho_d^2 (see pwc_table_create_box).
//
// For one direction, with m = n_k - n_i, m' = n_l - n_j and s = m + m',
//   tau_q(m, m') = 2 beta^{-1/2} D(m)                          if s = 0,
//                = -(S(m) + S(m')) / (pi s beta^{1/2})          otherwise,
//   S(m) = Int_0^1 exp(-u^2/beta) sin(2 pi m u) du   (odd in m),
//   D(m) = Int_0^1 (1 - u) exp(-u^2/beta) cos(2 pi m u) du   (even in m),
// which follows from substituting u = xi - xi' in the double integral
// beta^{-1/2} Int Int exp(-(xi-xi')^2/beta) exp(2 pi i (m xi + m' xi')).
// S and D are integrated by composite Gauss-Legendre (kGlPanels panels of
// kGlPanelPoints points) over [0, min(1, 8 beta^{1/2})]; past that point the
// Gaussian is below e^{-64}.  D is integrated directly: the integration-by-
// parts shortcut through S cancels catastrophically at large beta.
#include <cmath>

#include "pwc_internal.h"

namespace pwc {
namespace {

constexpr int kThreads = 256;

// sin(2 pi m u) and cos(2 pi m u) with the product 2 m u carried to double
// the working precision, so the phase is exact to rounding at large m.
__device__ inline void sincos_2pi_mu(int m, double u, double *s, double *c) {
    const double a = 2.0 * m * u;
    const double da = fma(2.0 * m, u, -a);   // exact remainder of the product
    double sa, ca;
    sincospi(a, &sa, &ca);
    const double pda = M_PI * da;
    *s = fma(pda, ca, sa);
    *c = fma(-pda, sa, ca);
}

// kPrimM values of m per block share the Gaussian factor of each point.
// Grid (ceil((K + 1) / kPrimM), Q, ndir): direction d of a box has its own
// node beta[d][q].  For every m each lane sums its points in order and a
// fixed tree combines the lanes.
constexpr int kPrimM = 3;

__global__ __launch_bounds__(kThreads) void k_prim(const double *__restrict__ beta,
                                                  const double *__restrict__ gl, int K,
                                                  double *__restrict__ prim) {
    const int m0 = blockIdx.x * kPrimM;
    const int q = blockIdx.y + blockIdx.z * gridDim.y;   // (direction, node) flat
    const int nm = min(kPrimM, K + 1 - m0);
    const double b = beta[q];
    const double up = fmin(1.0, 8.0 * sqrt(b));
    const double h = up / kGlPanels;
    double s[kPrimM], d[kPrimM];
#pragma unroll
    for (int j = 0; j < kPrimM; ++j) s[j] = d[j] = 0.0;
    for (int p = threadIdx.x; p < kGlPanels * kGlPanelPoints; p += kThreads) {
        const int panel = p / kGlPanelPoints, k = p % kGlPanelPoints;
        const double u = (panel + gl[k]) * h;
        const double wt = gl[kGlPanelPoints + k] * h;
        const double g = exp(-(u * u) / b);
        const double ws = wt * g, wd = wt * (1.0 - u) * g;
#pragma unroll
        for (int j = 0; j < kPrimM; ++j) {
            if (j >= nm) break;
            double sn, cs;
            sincos_2pi_mu(m0 + j, u, &sn, &cs);
            s[j] = fma(ws, sn, s[j]);
            d[j] = fma(wd, cs, d[j]);
        }
    }
    __shared__ double rs[kPrimM][kThreads], rd[kPrimM][kThreads];
#pragma unroll
    for (int j = 0; j < kPrimM; ++j) {
        rs[j][threadIdx.x] = s[j];
        rd[j][threadIdx.x] = d[j];
    }
    __syncthreads();
    const int tid = threadIdx.x;
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (tid < w) {
#pragma unroll
            for (int j = 0; j < kPrimM; ++j) {
                rs[j][threadIdx.x] += rs[j][threadIdx.x + w];
                rd[j][threadIdx.x] += rd[j][threadIdx.x + w];
            }
        }
        __syncthreads();
    }
    if (tid < nm) {
        const int j = tid, m = m0 + j;
        prim[(static_cast<size_t>(q) * 2 + 0) * (K + 1) + m] = (m == 0) ? 0.0 : rs[j][0];
        prim[(static_cast<size_t>(q) * 2 + 1) * (K + 1) + m] = rd[j][0];
    }
}

__device__ inline float2 split_hilo(double v) {
    const float hi = static_cast<float>(v);
    const float lo = static_cast<float>(v - static_cast<double>(hi));
    return make_float2(hi, lo);
}

struct AsmArgs {
    const double *beta;     // [ndir][Q]
    const double *wcbrt;    // [Q]
    const double *prim;     // [ndir][Q][2][K + 1]
    const int32_t *fold;
    const int32_t *reps;
    int K, nd, E1, Qp, dc, Q, ndir;
    int from_tau;      // 1: tau is given (a loaded table), derive the layouts only
    double *tau;
    double *tauF;
    float2 *tauHL;
    float *tau32;
    double *diag;
    float2 *diagHL;
};

// Grid (nd^2 / kThreads, Q, ndir).
__global__ __launch_bounds__(kThreads) void k_assemble(AsmArgs a) {
    const int e = blockIdx.x * kThreads + threadIdx.x;
    const int q = blockIdx.y, d = blockIdx.z;
    const int dq = d * a.Q + q;                          // (direction, node) flat
    if (e >= a.nd * a.nd) return;
    const int row = e / a.nd, col = e % a.nd;
    const int m = row - a.K, mp = col - a.K;
    const int s = m + mp;
    const size_t ti = (static_cast<size_t>(dq) * a.nd + row) * a.nd + col;
    double v;
    if (a.from_tau) {
        v = a.tau[ti];
    } else {
        const double *S = a.prim + static_cast<size_t>(dq) * 2 * (a.K + 1);
        const double *D = S + (a.K + 1);
        const double rb = sqrt(a.beta[dq]);
        if (s == 0) {
            v = 2.0 / rb * D[m < 0 ? -m : m];
        } else {
            const double sm = m < 0 ? -S[-m] : S[m];
            const double smp = mp < 0 ? -S[-mp] : S[mp];
            v = -(sm + smp) / (M_PI * s * rb);
        }
        a.tau[ti] = v;
    }
    // Folded layout: only the orbit representative writes its slot, scaled
    // by W_q^(1/3) so that a node term of Eq. 14 is the plain product of
    // three folded entries.
    const int f = a.fold[e];
    if (a.reps[2 * f] == m && a.reps[2 * f + 1] == mp) {
        const size_t idx = static_cast<size_t>(d * a.E1 + f) * a.Qp + q;   // direction d's rows
        const double vw = v * a.wcbrt[q];
        a.tauF[idx] = vw;
        a.tauHL[idx] = split_hilo(vw);
        a.tau32[idx] = static_cast<float>(vw);
    }
    // Diagonal tau(m, -m) for m >= 0 (the exchange entries; even in m).
    if (s == 0 && m >= 0) {
        const size_t idx = ((static_cast<size_t>(q / a.dc) * a.ndir + d) * (a.K + 1) + m) * a.dc + (q % a.dc);
        a.diag[idx] = v;
        a.diagHL[idx] = split_hilo(v);
    }
}

}  // namespace

hipError_t launch_table_build(Table &t, hipStream_t s, bool from_tau) {
    if (!from_tau) {
        dim3 gp((t.K + 1 + kPrimM - 1) / kPrimM, t.Q, t.ndir);
        hipLaunchKernelGGL(k_prim, gp, dim3(kThreads), 0, s, t.d_beta, t.d_gl, t.K, t.d_prim);
        const hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    AsmArgs a{t.d_beta, t.d_Wcbrt, t.d_prim, t.d_fold, t.d_reps, t.K, t.nd, t.E1, t.fl.Qp, t.dl.c,
              t.Q, t.ndir, from_tau ? 1 : 0, t.d_tau, t.d_tauF, t.d_tauHL, t.d_tau32, t.d_diag, t.d_diagHL};
    dim3 ga((t.nd * t.nd + kThreads - 1) / kThreads, t.Q, t.ndir);
    hipLaunchKernelGGL(k_assemble, ga, dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace pwc
