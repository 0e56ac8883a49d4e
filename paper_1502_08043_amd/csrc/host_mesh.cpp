// Host-side FP64 set-up: basis enumeration, Gauss-Legendre rules, the Laplace
// meshes of Eqs. 11-14 / Table I, and the symmetry fold of the table plane.
#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <mutex>

#include "pwc_internal.h"

namespace pwc {

namespace {
// The basis, the fold map and the Gauss-Legendre unit rules are pure
// functions of n2max, K and q; tables of one process mostly share them, so
// each is formed once (the basis is then shared, the others copied out).
std::mutex g_memo_mu;
std::map<int, std::shared_ptr<const Basis>> g_basis_memo;
}  // namespace

static std::vector<int32_t> enumerate_basis_uncached(int n2max);

std::shared_ptr<const Basis> enumerate_basis(int n2max) {
    std::lock_guard<std::mutex> lk(g_memo_mu);
    auto it = g_basis_memo.find(n2max);
    if (it == g_basis_memo.end()) {
        auto b = std::make_shared<Basis>();
        b->n = enumerate_basis_uncached(n2max);
        b->packed.resize(b->n.size() / 3);
        for (size_t i = 0; i < b->packed.size(); ++i)
            b->packed[i] = static_cast<int32_t>((static_cast<uint32_t>(b->n[3 * i]) & 0xffu) |
                                                ((static_cast<uint32_t>(b->n[3 * i + 1]) & 0xffu) << 8) |
                                                ((static_cast<uint32_t>(b->n[3 * i + 2]) & 0xffu) << 16));
        it = g_basis_memo.emplace(n2max, std::move(b)).first;
    }
    return it->second;
}

static std::vector<int32_t> enumerate_basis_uncached(int n2max) {
    // Sec. II: keep every product planewave below the cutoff, |n|^2 <= n2max.
    // The loops meet the vectors in ascending (x, y, z); a stable counting
    // sort by |n|^2 then gives the canonical order (|n|^2, x, y, z).
    const int r = static_cast<int>(std::floor(std::sqrt(static_cast<double>(n2max)) + 1e-9));
    std::vector<int32_t> shell_start(static_cast<size_t>(n2max) + 2, 0);
    for (int x = -r; x <= r; ++x)
        for (int y = -r; y <= r; ++y)
            for (int z = -r; z <= r; ++z) {
                const int n2 = x * x + y * y + z * z;
                if (n2 <= n2max) ++shell_start[n2 + 1];
            }
    for (int k = 0; k <= n2max; ++k) shell_start[k + 1] += shell_start[k];
    std::vector<int32_t> out(static_cast<size_t>(shell_start[n2max + 1]) * 3);
    for (int x = -r; x <= r; ++x)
        for (int y = -r; y <= r; ++y)
            for (int z = -r; z <= r; ++z) {
                const int n2 = x * x + y * y + z * z;
                if (n2 > n2max) continue;
                int32_t *o = &out[static_cast<size_t>(shell_start[n2]++) * 3];
                o[0] = x;
                o[1] = y;
                o[2] = z;
            }
    return out;
}

// Gauss-Legendre rules are formed in x87 extended precision (64-bit
// significand) and rounded to FP64 once, after the map to [a, b] and, for the
// tail, after beta = 1/t^2 and W = 2 w / t^3.  In plain FP64 the node nearest
// an endpoint, a + h (1 - z) with z close to 1, loses about log10(1/(1 - z))
// digits; the tail's smallest t then carries a relative error near 3e-14.
using ext = long double;

// Legendre P_q(z) and P_q'(z) by the three-term recurrence
// (k + 1) P_{k+1} = (2k + 1) z P_k - k P_{k-1}.
static void legendre(int q, ext z, ext *p, ext *dp) {
    ext pk = 1.0L, pkm1 = 0.0L;
    for (int k = 0; k < q; ++k) {
        const ext pk1 = ((2.0L * k + 1.0L) * z * pk - k * pkm1) / (k + 1.0L);
        pkm1 = pk;
        pk = pk1;
    }
    *p = pk;
    *dp = q * (z * pk - pkm1) / ((z - 1.0L) * (z + 1.0L));   // (z^2 - 1) P' = q (z P_q - P_{q-1})
}

// Roots z_i of P_q counted from z = 1 (i < (q + 1) / 2) and the weights
// 2 / ((1 - z^2) P_q'(z)^2), extended precision.
struct UnitRule {
    std::vector<ext> z, w;
};
static UnitRule unit_rule(int q) {
    UnitRule r;
    for (int i = 0; i < (q + 1) / 2; ++i) {
        // Root i of P_q counted from z = 1, started from the Tricomi estimate
        // cos(pi (i + 3/4) / (q + 1/2)) and refined by Newton's method.
        ext z = std::cos(static_cast<ext>(M_PI) * (i + 0.75L) / (q + 0.5L));
        ext p = 0.0L, dp = 1.0L;
        // Newton converges quadratically: two more steps after the step has
        // dropped below 1e-12 |z| reach the extended-precision root.
        for (int it = 0, extra = -1; it < 100 && extra != 0; ++it) {
            legendre(q, z, &p, &dp);
            const ext step = p / dp;
            z -= step;
            if (extra > 0) --extra;
            else if (extra < 0 && std::fabs(step) <= 1e-12L * std::fabs(z) + 1e-300L) extra = 2;
        }
        if (q % 2 == 1 && i == q / 2) z = 0.0L;   // the middle root is exactly 0
        legendre(q, z, &p, &dp);
        r.z.push_back(z);
        r.w.push_back(2.0L / ((1.0L - z) * (1.0L + z) * dp * dp));
    }
    return r;
}

// q-point rule on [a, b] in extended precision, ascending nodes.
static void gauss_legendre_ext(int q, ext a, ext b, std::vector<ext> &x, std::vector<ext> &w) {
    static std::map<int, UnitRule> memo;   // guarded by g_memo_mu
    UnitRule r;
    {
        std::lock_guard<std::mutex> lk(g_memo_mu);
        auto it = memo.find(q);
        if (it == memo.end()) it = memo.emplace(q, unit_rule(q)).first;
        r = it->second;
    }
    x.assign(q, 0.0L);
    w.assign(q, 0.0L);
    const ext half = 0.5L * (b - a);
    for (int i = 0; i < (q + 1) / 2; ++i) {
        const ext z = r.z[i], wi = r.w[i];
        // Each node measured from its nearer end: a + h (1 - z) and b - h (1 - z).
        x[i] = a + half * (1.0L - z);
        x[q - 1 - i] = b - half * (1.0L - z);
        w[q - 1 - i] = half * wi;
        w[i] = half * wi;
    }
}

void gauss_legendre(int q, double a, double b, std::vector<double> &x, std::vector<double> &w) {
    std::vector<ext> xe, we;
    gauss_legendre_ext(q, a, b, xe, we);
    x.assign(xe.begin(), xe.end());
    w.assign(we.begin(), we.end());
}

bool mesh_valid(const pwc_mesh &m, int *n_nodes) {
    int Q = 0;
    if (m.q_sub < 1 || m.q_sub > 256 || m.q_tail < 1 || m.q_tail > 256) return false;
    if (!(std::isfinite(m.alpha_c))) return false;
    if (m.kind == PWC_MESH_GEOMETRIC || m.kind == PWC_MESH_GEOMETRIC_ROOT) {
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
    std::vector<ext> se, we;
    if (m.kind == PWC_MESH_GEOMETRIC || m.kind == PWC_MESH_GEOMETRIC_ROOT) {
        // Interval 1 cut geometrically: edges 0, beta_c r^{-(n-1)}, ..., beta_c r^{-1}, beta_c.
        double lo = 0.0;
        for (int k = 0; k < m.n_sub; ++k) {
            const double hi = beta_c * std::pow(m.ratio, -(m.n_sub - 1 - k));
            if (m.kind == PWC_MESH_GEOMETRIC) {
                gauss_legendre(m.q_sub, lo, hi, x, w);
                beta.insert(beta.end(), x.begin(), x.end());
                W.insert(W.end(), w.begin(), w.end());
            } else {
                // Gauss-Legendre in s = beta^{1/2} on [lo^{1/2}, hi^{1/2}]:
                // beta = s^2, d beta = 2 s ds.  Near beta = 0 the integrand is
                // a series in beta^{1/2}, smooth in s.
                gauss_legendre_ext(m.q_sub, std::sqrt(static_cast<ext>(lo)), std::sqrt(static_cast<ext>(hi)), se, we);
                for (int i = 0; i < m.q_sub; ++i) {
                    beta.push_back(static_cast<double>(se[i] * se[i]));
                    W.push_back(static_cast<double>(2.0L * se[i] * we[i]));
                }
            }
            lo = hi;
        }
    } else {
        gauss_legendre(m.q_sub, 0.0, beta_c, x, w);
        beta.insert(beta.end(), x.begin(), x.end());
        W.insert(W.end(), w.begin(), w.end());
    }
    *n_interval1 = static_cast<int>(beta.size());
    // Tail (Eqs. 11-13): t = beta^{-1/2} on (0, t_c], t_c = beta_c^{-1/2};
    // d beta = -2 t^{-3} dt, so node t maps to beta = 1/t^2 with weight 2 w / t^3.
    // Gauss-Legendre in t, or (GEOMETRIC_ROOT) the rule exact for
    // polynomials in t^2 up to degree 4 q_tail - 2 -- the tail integrand is a
    // series in t^2 (Eqs. 10-11) -- which is the positive half of the
    // 2 q_tail-point Gauss-Legendre rule on [-t_c, t_c].
    const ext tc = 1.0L / std::sqrt(static_cast<ext>(beta_c));
    std::vector<ext> te, wt;
    if (m.kind == PWC_MESH_GEOMETRIC_ROOT) {
        gauss_legendre_ext(2 * m.q_tail, -tc, tc, te, wt);
        te.erase(te.begin(), te.begin() + m.q_tail);   // ascending: the positive half
        wt.erase(wt.begin(), wt.begin() + m.q_tail);
    } else {
        gauss_legendre_ext(m.q_tail, 0.0L, tc, te, wt);
    }
    for (int i = 0; i < m.q_tail; ++i) {
        const ext t = te[i];
        beta.push_back(static_cast<double>(1.0L / (t * t)));
        W.push_back(static_cast<double>(2.0L * wt[i] / (t * t * t)));
    }
    return static_cast<int>(beta.size()) == Q;
}

static void build_fold_uncached(int K, std::vector<int32_t> &fold, std::vector<int32_t> &reps);

void build_fold(int K, std::vector<int32_t> &fold, std::vector<int32_t> &reps) {
    static std::map<int, std::pair<std::vector<int32_t>, std::vector<int32_t>>> memo;   // g_memo_mu
    std::lock_guard<std::mutex> lk(g_memo_mu);
    auto it = memo.find(K);
    if (it == memo.end()) {
        std::vector<int32_t> f, r;
        build_fold_uncached(K, f, r);
        it = memo.emplace(K, std::make_pair(std::move(f), std::move(r))).first;
    }
    fold = it->second.first;
    reps = it->second.second;
}

static void build_fold_uncached(int K, std::vector<int32_t> &fold, std::vector<int32_t> &reps) {
    const int nd = 2 * K + 1;
    fold.assign(static_cast<size_t>(nd) * nd, -1);
    reps.clear();
    // Representative of the orbit {(m,m'), (m',m), (-m,-m'), (-m',-m)}: the
    // lexicographically smallest (m + K, m' + K) pair of the orbit.
    auto rep_of = [&](int a, int b) {
        const int m = a - K, mp = b - K;
        const int orbit[4][2] = {{m, mp}, {mp, m}, {-m, -mp}, {-mp, -m}};
        int best = a * nd + b;
        for (const auto &o : orbit) best = std::min(best, (o[0] + K) * nd + (o[1] + K));
        return best;
    };
    // Orbits are numbered by ascending m^2 + m'^2 (ties in row order): index
    // differences of a planewave basis are small far more often than large,
    // so the entries a quadruple stream reads most get the smallest numbers
    // and the value table's most used part is its first few megabytes.
    std::vector<int> order;
    for (int a = 0; a < nd; ++a)
        for (int b = 0; b < nd; ++b)
            if (rep_of(a, b) == a * nd + b) order.push_back(a * nd + b);
    auto r2 = [&](int v) {
        const int m = v / nd - K, mp = v % nd - K;
        return m * m + mp * mp;
    };
    std::stable_sort(order.begin(), order.end(), [&](int u, int v) { return r2(u) < r2(v); });
    for (size_t e = 0; e < order.size(); ++e) {
        fold[order[e]] = static_cast<int32_t>(e);
        reps.push_back(order[e] / nd - K);
        reps.push_back(order[e] % nd - K);
    }
    for (int a = 0; a < nd; ++a)
        for (int b = 0; b < nd; ++b) fold[a * nd + b] = fold[rep_of(a, b)];
}

}  // namespace pwc
