// Host-side FP64 set-up: basis enumeration, Gauss-Legendre rules, the Laplace
// meshes of Eqs. 11-14 / Table I, and the symmetry fold of the table plane.
#include <algorithm>
#include <array>
#include <cmath>

#include "pwc_internal.h"

namespace pwc {

std::vector<int32_t> enumerate_basis(int n2max) {
    // Sec. II: keep every product planewave below the cutoff, |n|^2 <= n2max.
    const int r = static_cast<int>(std::floor(std::sqrt(static_cast<double>(n2max)) + 1e-9));
    std::vector<std::array<int32_t, 4>> pts;
    for (int x = -r; x <= r; ++x)
        for (int y = -r; y <= r; ++y)
            for (int z = -r; z <= r; ++z) {
                const int n2 = x * x + y * y + z * z;
                if (n2 <= n2max) pts.push_back({n2, x, y, z});
            }
    std::sort(pts.begin(), pts.end());
    std::vector<int32_t> out;
    out.reserve(pts.size() * 3);
    for (const auto &p : pts) {
        out.push_back(p[1]);
        out.push_back(p[2]);
        out.push_back(p[3]);
    }
    return out;
}

// Legendre P_q(z) and P_q'(z) by the three-term recurrence
// (k + 1) P_{k+1} = (2k + 1) z P_k - k P_{k-1}.
static void legendre(int q, double z, double *p, double *dp) {
    double pk = 1.0, pkm1 = 0.0;
    for (int k = 0; k < q; ++k) {
        const double pk1 = ((2.0 * k + 1.0) * z * pk - k * pkm1) / (k + 1.0);
        pkm1 = pk;
        pk = pk1;
    }
    *p = pk;
    *dp = q * (z * pk - pkm1) / (z * z - 1.0);   // from (z^2 - 1) P' = q (z P_q - P_{q-1})
}

void gauss_legendre(int q, double a, double b, std::vector<double> &x, std::vector<double> &w) {
    x.assign(q, 0.0);
    w.assign(q, 0.0);
    const double half = 0.5 * (b - a), mid = 0.5 * (b + a);
    for (int i = 0; i < (q + 1) / 2; ++i) {
        // Root i of P_q counted from z = 1, started from the Tricomi estimate
        // cos(pi (i + 3/4) / (q + 1/2)) and refined by Newton's method.
        double z = std::cos(M_PI * (i + 0.75) / (q + 0.5));
        double p = 0.0, dp = 1.0;
        for (int it = 0; it < 64; ++it) {
            legendre(q, z, &p, &dp);
            const double step = p / dp;
            z -= step;
            if (std::fabs(step) <= 1e-17 * std::fabs(z) + 1e-300) break;
        }
        legendre(q, z, &p, &dp);
        const double wi = 2.0 / ((1.0 - z * z) * dp * dp);
        // ascending order: the largest root goes last
        x[q - 1 - i] = mid + half * z;
        x[i] = mid - half * z;
        w[q - 1 - i] = half * wi;
        w[i] = half * wi;
    }
    if (q % 2 == 1) x[q / 2] = mid;   // the middle root is exactly 0
}

bool mesh_valid(const pwc_mesh &m, int *n_nodes) {
    int Q = 0;
    if (m.q_sub < 1 || m.q_sub > 256 || m.q_tail < 1 || m.q_tail > 256) return false;
    if (!(std::isfinite(m.alpha_c))) return false;
    if (m.kind == PWC_MESH_GEOMETRIC) {
        if (m.n_sub < 1 || m.n_sub > 32 || !(m.ratio > 1.0) || !std::isfinite(m.ratio)) return false;
        Q = m.n_sub * m.q_sub + m.q_tail;
    } else if (m.kind == PWC_MESH_TWO_INTERVAL) {
        Q = m.q_sub + m.q_tail;
    } else {
        return false;
    }
    if (Q > PWC_MAX_NODES) return false;
    if (n_nodes) *n_nodes = Q;
    return true;
}

bool build_mesh(const pwc_mesh &m, double L, std::vector<double> &beta, std::vector<double> &W,
                int *n_interval1) {
    int Q = 0;
    if (!mesh_valid(m, &Q)) return false;
    // beta = 4 alpha / L^2; the default split is beta_c = 1.
    const double beta_c = m.alpha_c > 0.0 ? 4.0 * m.alpha_c / (L * L) : 1.0;
    beta.clear();
    W.clear();
    std::vector<double> x, w;
    if (m.kind == PWC_MESH_GEOMETRIC) {
        // Interval 1 cut geometrically: edges 0, beta_c r^{-(n-1)}, ..., beta_c r^{-1}, beta_c.
        double lo = 0.0;
        for (int k = 0; k < m.n_sub; ++k) {
            const double hi = beta_c * std::pow(m.ratio, -(m.n_sub - 1 - k));
            gauss_legendre(m.q_sub, lo, hi, x, w);
            beta.insert(beta.end(), x.begin(), x.end());
            W.insert(W.end(), w.begin(), w.end());
            lo = hi;
        }
    } else {
        gauss_legendre(m.q_sub, 0.0, beta_c, x, w);
        beta.insert(beta.end(), x.begin(), x.end());
        W.insert(W.end(), w.begin(), w.end());
    }
    *n_interval1 = static_cast<int>(beta.size());
    // Tail (Eqs. 11-13): Gauss-Legendre in t = beta^{-1/2} on (0, beta_c^{-1/2}];
    // d beta = -2 t^{-3} dt, so node t maps to beta = 1/t^2 with weight 2 w / t^3.
    gauss_legendre(m.q_tail, 0.0, 1.0 / std::sqrt(beta_c), x, w);
    for (int i = 0; i < m.q_tail; ++i) {
        const double t = x[i];
        beta.push_back(1.0 / (t * t));
        W.push_back(2.0 * w[i] / (t * t * t));
    }
    return static_cast<int>(beta.size()) == Q;
}

void build_fold(int K, std::vector<int32_t> &fold, std::vector<int32_t> &reps) {
    const int nd = 2 * K + 1;
    fold.assign(static_cast<size_t>(nd) * nd, -1);
    reps.clear();
    // Representative of the orbit {(m,m'), (m',m), (-m,-m'), (-m',-m)}: the
    // lexicographically smallest (m + K, m' + K) pair of the orbit.  Entries
    // are numbered in the order their representative is met, row by row.
    for (int a = 0; a < nd; ++a)
        for (int b = 0; b < nd; ++b) {
            const int m = a - K, mp = b - K;
            const int orbit[4][2] = {{m, mp}, {mp, m}, {-m, -mp}, {-mp, -m}};
            int best = a * nd + b;
            for (const auto &o : orbit) best = std::min(best, (o[0] + K) * nd + (o[1] + K));
            if (best == a * nd + b) {
                fold[best] = static_cast<int32_t>(reps.size() / 2);
                reps.push_back(m);
                reps.push_back(mp);
            }
        }
    for (int a = 0; a < nd; ++a)
        for (int b = 0; b < nd; ++b) {
            const int m = a - K, mp = b - K;
            const int orbit[4][2] = {{m, mp}, {mp, m}, {-m, -mp}, {-mp, -m}};
            int best = a * nd + b;
            for (const auto &o : orbit) best = std::min(best, (o[0] + K) * nd + (o[1] + K));
            fold[a * nd + b] = fold[best];
        }
}

}  // namespace pwc
