/*
 * Oracle node sums and pair sums, plain C, FP64.
 *
 * TEST INFRASTRUCTURE ONLY: linked by nothing in the product path.
 *
 * Inputs are the oracle's own tables (tables.py), mesh (mesh.py) and basis
 * (basis.py).  Table layout: tau[d][q][m + K][m' + K], m, m' in [-K, K],
 * nd = 2K + 1, with ndir = 1 (a cube: one table serves every direction) or
 * ndir = 3 (a rectangular box: table d for direction d).
 *
 * reconstruct: Eq. 14 -- <ij|kl> = (1/(sqrt(pi) L)) sum_q W_q
 *              tau^x_q(m_x, m'_x) tau^y_q(m_y, m'_y) tau^z_q(m_z, m'_z),
 *              with m = n_k - n_i and m' = n_l - n_j per direction (L the
 *              cube side, or the reference length of a box).
 * energies:    Sec. III uniform electron gas, one spin channel:
 *              E_H =  1/2 sum_{i,j} f_i f_j <ij|ij>,
 *              E_x = -1/2 sum_{i,j} f_i f_j <ij|ji>   (i = j included),
 *              both as literal double loops over ordered pairs.
 *
 * Every sum is accumulated with Neumaier's compensated summation, in natural
 * order; the node product is formed left to right with no fused multiply-add
 * (the file is built with -ffp-contract=off).  Per-row partial sums of the
 * pair loops are combined in row order, so results do not depend on the
 * thread count.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double s, c; } nsum;

static inline void nadd(nsum *a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static inline double nval(const nsum *a) { return a->s + a->c; }

static void set_threads(int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* Node sum for one integral given the three flat table offsets; direction
 * d reads table tau + d * dstride (dstride = 0 for a cube). */
static double node_sum(const double *tau, int64_t dstride, const double *W, int Q,
                       int64_t slice, int64_t ox, int64_t oy, int64_t oz) {
    nsum acc = {0.0, 0.0};
    for (int q = 0; q < Q; ++q) {
        const double *t = tau + (int64_t)q * slice;
        double term = W[q] * t[ox] * t[dstride + oy] * t[2 * dstride + oz];
        nadd(&acc, term);
    }
    return nval(&acc);
}

/* Flat offset of tau(m, m') for one direction. */
static inline int64_t offset(int64_t m, int64_t mp, int K) {
    return (m + K) * (int64_t)(2 * K + 1) + (mp + K);
}

int oracle_reconstruct(const double *tau, int ndir, const double *W, int Q, int K,
                       const int64_t *basis, int64_t N, const int32_t *quads,
                       int64_t n, double L, double *out, int nthreads) {
    const int64_t nd = 2 * K + 1, slice = nd * nd;
    const int64_t dstride = ndir == 3 ? (int64_t)Q * slice : 0;
    if (ndir != 1 && ndir != 3) return 1;
    const double pref = 1.0 / (sqrt(M_PI) * L);
    int bad = 0;
    for (int64_t e = 0; e < 4 * n; ++e)
        if (quads[e] < 0 || quads[e] >= N) bad = 1;
    if (bad) return 2;
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < n; ++e) {
        const int64_t *ni = basis + 3 * (int64_t)quads[4 * e + 0];
        const int64_t *nj = basis + 3 * (int64_t)quads[4 * e + 1];
        const int64_t *nk = basis + 3 * (int64_t)quads[4 * e + 2];
        const int64_t *nl = basis + 3 * (int64_t)quads[4 * e + 3];
        int64_t o[3];
        for (int d = 0; d < 3; ++d) {
            int64_t m = nk[d] - ni[d], mp = nl[d] - nj[d];
            if (m < -K || m > K || mp < -K || mp > K) { o[d] = -1; continue; }
            o[d] = offset(m, mp, K);
        }
        if (o[0] < 0 || o[1] < 0 || o[2] < 0) { out[e] = NAN; continue; }
        out[e] = pref * node_sum(tau, dstride, W, Q, slice, o[0], o[1], o[2]);
    }
    return 0;
}

int oracle_energies(const double *tau, int ndir, const double *W, int Q, int K,
                    const int64_t *basis, int64_t N, const int32_t *occ,
                    const double *f, int64_t M, double L, double *eh, double *ex,
                    int nthreads) {
    const int64_t nd = 2 * K + 1, slice = nd * nd;
    const int64_t dstride = ndir == 3 ? (int64_t)Q * slice : 0;
    if (ndir != 1 && ndir != 3) return 1;
    const double pref = 1.0 / (sqrt(M_PI) * L);
    for (int64_t i = 0; i < M; ++i)
        if (occ[i] < 0 || occ[i] >= N) return 2;
    double *rowh = (double *)malloc(sizeof(double) * (size_t)(M > 0 ? M : 1));
    double *rowx = (double *)malloc(sizeof(double) * (size_t)(M > 0 ? M : 1));
    if (!rowh || !rowx) { free(rowh); free(rowx); return 3; }
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < M; ++i) {
        const int64_t *ni = basis + 3 * (int64_t)occ[i];
        const double fi = f ? f[i] : 1.0;
        nsum h = {0.0, 0.0}, x = {0.0, 0.0};
        for (int64_t j = 0; j < M; ++j) {
            const int64_t *nj = basis + 3 * (int64_t)occ[j];
            const double fij = fi * (f ? f[j] : 1.0);
            /* <ij|ij>: k = i, l = j -> m = m' = 0 in every direction. */
            int64_t oh = offset(0, 0, K);
            nadd(&h, fij * node_sum(tau, dstride, W, Q, slice, oh, oh, oh));
            /* <ij|ji>: k = j, l = i -> m = n_j - n_i, m' = n_i - n_j. */
            int64_t o[3];
            for (int d = 0; d < 3; ++d) o[d] = offset(nj[d] - ni[d], ni[d] - nj[d], K);
            nadd(&x, fij * node_sum(tau, dstride, W, Q, slice, o[0], o[1], o[2]));
        }
        rowh[i] = nval(&h);
        rowx[i] = nval(&x);
    }
    nsum H = {0.0, 0.0}, X = {0.0, 0.0};
    for (int64_t i = 0; i < M; ++i) { nadd(&H, rowh[i]); nadd(&X, rowx[i]); }
    *eh = 0.5 * pref * nval(&H);
    *ex = -0.5 * pref * nval(&X);
    free(rowh);
    free(rowx);
    return 0;
}
