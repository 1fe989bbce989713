// Host-side setup of the CQ solver: weights, Gauss-Jacobi rules, the fast
// sum-of-geometric-sequences rules and their node-count scan, and the 2x2
// coupling eigen-decomposition. Plain fp64 C++; runs once per solver.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <map>
#include <vector>

#include "internal.h"
#include "kernels.h"

namespace cqfp {

static thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

void clear_error() { g_err.clear(); }

const char* last_error() { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// Weights (eqs. (3.4) and (3.12)).
// BE: (1-z)^beta = sum g_i z^i with g_i = g_{i-1} (1 - (1+beta)/i).
// BDF2: p(z) = 3/2 - 2z + z^2/2 and f = p^beta satisfy p f' = beta p' f;
// comparing coefficients of z^(i-1) gives, with p0 = 3/2, p1 = -2, p2 = 1/2,
//   c_i = [ (beta - (i-1)) p1 c_{i-1} + (2 beta - (i-2)) p2 c_{i-2} ] / (p0 i).
// Both recurrences only shrink errors (the parasitic solution of the
// second decays like 3^-i), so they stay at rounding level for i ~ 1e5.
void weights(int scheme, double beta, double tau, int64_t n, double* d) {
    const double s = std::pow(tau, -beta);
    if (scheme == 1) {
        double g = 1.0;
        d[0] = s;
        for (int64_t i = 1; i <= n; ++i) {
            g *= 1.0 - (1.0 + beta) / double(i);
            d[i] = s * g;
        }
        return;
    }
    const double p0 = 1.5, p1 = -2.0, p2 = 0.5;
    double cm2 = 0.0, cm1 = std::pow(p0, beta);
    d[0] = s * cm1;
    for (int64_t i = 1; i <= n; ++i) {
        const double di = double(i);
        double c = (beta - (di - 1.0)) * p1 * cm1;
        if (i >= 2) c += (2.0 * beta - (di - 2.0)) * p2 * cm2;
        c /= p0 * di;
        d[i] = s * c;
        cm2 = cm1;
        cm1 = c;
    }
}

// d/dbeta of the weights above, by differentiating the same recurrences:
// with s = tau^-beta (s' = -ln(tau) s), BE g_i = g_{i-1} (1 - (1+beta)/i)
// gives g'_i = g'_{i-1} (1 - (1+beta)/i) - g_{i-1}/i; the BDF2 recurrence
// c_i = [(beta-(i-1)) p1 c_{i-1} + (2 beta-(i-2)) p2 c_{i-2}] / (p0 i) gives
// c'_i = [p1 c_{i-1} + (beta-(i-1)) p1 c'_{i-1} + 2 p2 c_{i-2}
//         + (2 beta-(i-2)) p2 c'_{i-2}] / (p0 i), c'_0 = ln(p0) c_0.
void weights_dbeta(int scheme, double beta, double tau, int64_t n, double* dd) {
    const double s = std::pow(tau, -beta), ds = -std::log(tau) * s;
    if (scheme == 1) {
        double g = 1.0, dg = 0.0;
        dd[0] = ds;
        for (int64_t i = 1; i <= n; ++i) {
            const double f = 1.0 - (1.0 + beta) / double(i);
            dg = dg * f - g / double(i);
            g *= f;
            dd[i] = ds * g + s * dg;
        }
        return;
    }
    const double p0 = 1.5, p1 = -2.0, p2 = 0.5;
    double cm2 = 0.0, cm1 = std::pow(p0, beta);
    double dm2 = 0.0, dm1 = std::log(p0) * cm1;
    dd[0] = ds * cm1 + s * dm1;
    for (int64_t i = 1; i <= n; ++i) {
        const double di = double(i);
        double c = (beta - (di - 1.0)) * p1 * cm1;
        double dc = p1 * cm1 + (beta - (di - 1.0)) * p1 * dm1;
        if (i >= 2) {
            c += (2.0 * beta - (di - 2.0)) * p2 * cm2;
            dc += 2.0 * p2 * cm2 + (2.0 * beta - (di - 2.0)) * p2 * dm2;
        }
        c /= p0 * di;
        dc /= p0 * di;
        dd[i] = ds * c + s * dc;
        cm2 = cm1;
        cm1 = c;
        dm2 = dm1;
        dm1 = dc;
    }
}

// ---------------------------------------------------------------------------
// Gauss-Jacobi rule for (1-s)^a (1+s)^b.
// Monic recurrence p_{k+1} = (s - al_k) p_k - be_k p_{k-1} with
//   al_k = (b^2 - a^2) / ((2k+a+b)(2k+a+b+2))   (al_0 = (b-a)/(a+b+2)),
//   be_k = 4k(k+a)(k+b)(k+a+b) / ((2k+a+b)^2 (2k+a+b+1)(2k+a+b-1)),  k >= 1,
//   mu_0 = 2^(a+b+1) Gamma(a+1) Gamma(b+1) / Gamma(a+b+2).
// The nodes are the eigenvalues of the symmetric tridiagonal Jacobi matrix
// (diagonal al_k, off-diagonal sqrt(be_k)); each is isolated by bisection on
// the Sturm count and refined by Newton on the orthonormal polynomial. The
// weights are the Christoffel numbers 1 / sum_{k<n} q_k(s_j)^2 with q_k the
// orthonormal polynomials (q_0 = 1/sqrt(mu_0)). From the third node on,
// Newton starts from an angle extrapolated from the previous two nodes and
// the result is kept when the Sturm counts confirm it; otherwise bisection.
namespace {

struct JacobiRec {
    std::vector<double> al, sq;  // al[k], sq[k] = sqrt(be_k) (sq[0] unused)
    double mu0;
};

JacobiRec jacobi_rec(int n, double a, double b) {
    JacobiRec r;
    r.al.resize(n + 1);
    r.sq.assign(n + 1, 0.0);
    for (int k = 0; k <= n; ++k) {
        const double t = 2.0 * k + a + b;
        if (k == 0)
            r.al[k] = (b - a) / (a + b + 2.0);
        else
            r.al[k] = (b * b - a * a) / (t * (t + 2.0));
        if (k >= 1) {
            const double be = 4.0 * k * (k + a) * (k + b) * (k + a + b) / (t * t * (t + 1.0) * (t - 1.0));
            r.sq[k] = std::sqrt(be);
        }
    }
    r.mu0 = std::exp((a + b + 1.0) * std::log(2.0) + std::lgamma(a + 1.0) + std::lgamma(b + 1.0) -
                     std::lgamma(a + b + 2.0));
    return r;
}

// number of eigenvalues of the leading n x n Jacobi matrix below x
int sturm_count(const JacobiRec& r, int n, double x) {
    int cnt = 0;
    double q = r.al[0] - x;
    if (q < 0) ++cnt;
    for (int k = 1; k < n; ++k) {
        const double qq = (q != 0.0) ? q : 1e-300;
        q = (r.al[k] - x) - r.sq[k] * r.sq[k] / qq;
        if (q < 0) ++cnt;
    }
    return cnt;
}

// orthonormal q_n(x) and its derivative
void ortho_eval(const JacobiRec& r, int n, double x, double& qn, double& dqn, double& sumsq) {
    double qm1 = 0.0, q = 1.0 / std::sqrt(r.mu0);
    double dqm1 = 0.0, dq = 0.0;
    sumsq = q * q;
    for (int k = 0; k < n; ++k) {
        const double sn = r.sq[k + 1];
        const double skm = (k >= 1) ? r.sq[k] : 0.0;
        const double qn1 = ((x - r.al[k]) * q - skm * qm1) / sn;
        const double dqn1 = (q + (x - r.al[k]) * dq - skm * dqm1) / sn;
        qm1 = q;
        q = qn1;
        dqm1 = dq;
        dq = dqn1;
        if (k + 1 < n) sumsq += q * q;
    }
    qn = q;
    dqn = dq;
}

}  // namespace

void gauss_jacobi(int n, double a, double b, std::vector<double>& s, std::vector<double>& lam) {
    const JacobiRec r = jacobi_rec(n, a, b);
    s.assign(n, 0.0);
    lam.assign(n, 0.0);
    for (int j = 0; j < n; ++j) {
        const double lo0 = j > 0 ? s[j - 1] : -1.0;
        double x = 0.0;
        bool ok = false;
        if (j >= 2) {
            // the nodes are nearly evenly spaced in theta (s = -cos theta):
            // Newton from the extrapolated angle, accepted only if the Sturm
            // counts just below and above it show the (j+1)-th eigenvalue
            const double t1 = std::acos(-s[j - 1]), t2 = std::acos(-s[j - 2]);
            const double t = 2.0 * t1 - t2;
            if (t > t1 && t < M_PI) {
                x = -std::cos(t);
                const double spacing = x - lo0;
                bool conv = false;
                for (int it = 0; it < 16 && x > lo0 && x < 1.0; ++it) {
                    double qn, dqn, ss;
                    ortho_eval(r, n, x, qn, dqn, ss);
                    if (dqn == 0.0) break;
                    const double dx = qn / dqn;
                    x -= dx;
                    if (std::fabs(dx) <= 1e-13 * spacing) {  // one more step after this one
                        ortho_eval(r, n, x, qn, dqn, ss);
                        if (dqn != 0.0) x -= qn / dqn;
                        conv = true;
                        break;
                    }
                }
                if (conv && x > lo0 && x < 1.0) {
                    const double e = 1e-9 * (x - lo0);
                    ok = sturm_count(r, n, x - e) == j && sturm_count(r, n, x + e) == j + 1;
                }
            }
        }
        if (!ok) {
            // the (j+1)-th smallest eigenvalue lies where the count passes j,
            // above the previous node. Bisection isolates it to a bracket far
            // narrower than the node spacing (~(pi/n)^2 near the ends), and
            // Newton, which converges quadratically from there, finishes it.
            double lo = lo0, hi = 1.0;
            for (int it = 0; it < 200 && hi - lo > 1e-10; ++it) {
                const double mid = 0.5 * (lo + hi);
                if (mid <= lo || mid >= hi) break;
                if (sturm_count(r, n, mid) > j)
                    hi = mid;
                else
                    lo = mid;
            }
            x = 0.5 * (lo + hi);
            for (int it = 0; it < 4; ++it) {
                double qn, dqn, ss;
                ortho_eval(r, n, x, qn, dqn, ss);
                if (dqn == 0.0) break;
                const double xn = x - qn / dqn;
                if (!(xn > lo - 1e-12 && xn < hi + 1e-12)) break;  // keep the bracketed root
                x = xn;
            }
        }
        double qn, dqn, ss;
        ortho_eval(r, n, x, qn, dqn, ss);
        s[j] = x;
        lam[j] = 1.0 / ss;
    }
}

// ---------------------------------------------------------------------------
// Fast rules. With Gamma(beta) Gamma(1-beta) = pi / sin(pi beta):
// BE (3.6)-(3.7): d_i ~ sum_j w_j ((s_j+1)/2)^(i-2), i >= 2,
//   w_j = -lam_j sin(pi beta) / (4 pi tau^beta), nodes for (1-s)^beta (1+s)^(1-beta).
// BDF2 (3.14)-(3.16), real parts as in the remark after (3.16), i >= 3:
//   family 1: ratio (s+1)/(s+5), w = -2^(2+2beta) cos(pi beta) sin(pi beta)/pi
//             tau^-beta lam_j, dbar_i = (s+5)^-4 ratio^(i-3);
//   family 2: ratio (s+1)/2, w = -2^(-beta-3) sin(pi beta)/pi tau^-beta lam_j,
//             dbar_i = Re(1+3s)^beta ratio^(i-3);
//   both with nodes for (1-s)^beta (1+s)^(2-2beta). Only lags i >= ns use the
//   rule, so coef_j = w_j dbar_ns(s_j) multiplies ratio^(i-ns).
void build_rule(int scheme, double beta, double tau, int np, int np1, int ns, FastRule& out) {
    out.ratio.clear();
    out.coef.clear();
    const double sb = std::sin(M_PI * beta) / M_PI;
    const double tb = std::pow(tau, -beta);
    std::vector<double> s, lam;
    if (scheme == 1) {
        out.lag = 2;
        gauss_jacobi(np, beta, 1.0 - beta, s, lam);
        for (int j = 0; j < np; ++j) {
            out.ratio.push_back(0.5 * (s[j] + 1.0));
            out.coef.push_back(-lam[j] * sb * tb / 4.0);
        }
        return;
    }
    std::vector<double> s2, lam2;
    gauss_jacobi(np1, beta, 2.0 - 2.0 * beta, s, lam);
    gauss_jacobi(np, beta, 2.0 - 2.0 * beta, s2, lam2);
    bdf2_rule_from_nodes(beta, tau, ns, s, lam, s2, lam2, out);
}

void bdf2_rule_from_nodes(double beta, double tau, int ns, const std::vector<double>& s1,
                          const std::vector<double>& lam1, const std::vector<double>& s2,
                          const std::vector<double>& lam2, FastRule& out) {
    out.ratio.clear();
    out.coef.clear();
    out.lag = ns;
    const double sb = std::sin(M_PI * beta) / M_PI;
    const double tb = std::pow(tau, -beta);
    const double c1 = -std::pow(2.0, 2.0 + 2.0 * beta) * std::cos(M_PI * beta) * sb * tb;
    for (size_t j = 0; j < s1.size(); ++j) {
        const double r = (s1[j] + 1.0) / (s1[j] + 5.0);
        const double dbar = std::pow(s1[j] + 5.0, -4.0) * std::pow(r, double(ns - 3));
        out.ratio.push_back(r);
        out.coef.push_back(c1 * lam1[j] * dbar);
    }
    const double c2 = -std::pow(2.0, -beta - 3.0) * sb * tb;
    for (size_t j = 0; j < s2.size(); ++j) {
        const double r = 0.5 * (s2[j] + 1.0);
        const double u = 1.0 + 3.0 * s2[j];
        const double re = std::pow(std::fabs(u), beta) * (u >= 0.0 ? 1.0 : std::cos(M_PI * beta));
        const double dbar = re * std::pow(r, double(ns - 3));
        out.ratio.push_back(r);
        out.coef.push_back(c2 * lam2[j] * dbar);
    }
}

void shift_lag(FastRule& r, int lag) {
    for (size_t j = 0; j < r.ratio.size(); ++j) r.coef[j] *= std::pow(r.ratio[j], double(lag - r.lag));
    r.lag = lag;
}

double rule_error(const FastRule& r, const std::vector<double>& d, int64_t N) {
    const int64_t L = r.lag;
    if (N < L) return 0.0;
    std::vector<double> acc(size_t(N - L + 1), 0.0);
    // a term below 1e-30 |d_0| cannot move the error measured here (the
    // targets are above 1e-16 |d_0|); stopping there also keeps the loop out
    // of subnormal arithmetic for the small ratios
    const double tiny = 1e-30 * std::fabs(d[0]);
    for (size_t j = 0; j < r.ratio.size(); ++j) {
        double p = r.coef[j];
        const double q = r.ratio[j];
        for (int64_t i = L; i <= N && std::fabs(p) >= tiny; ++i) {
            acc[size_t(i - L)] += p;
            p *= q;
        }
    }
    double m = 0.0;
    for (int64_t i = L; i <= N; ++i) m = std::max(m, std::fabs(d[size_t(i)] - acc[size_t(i - L)]));
    return m / std::fabs(d[0]);
}

// d/dbeta of the fast weights sum_j coef_j r_j^(i - lag), i = lag..N, for a
// rule of np nodes (BDF2: np1 + np) started at `lag`. Every coefficient
// carries tau^-beta (3.6)/(3.14): with q_i the sums at tau = 1, the weights
// are tau^-beta q_i and their derivative tau^-beta (q'_i - ln(tau) q_i),
// where q'_i is a five-point central difference in beta of the rule rebuilt
// at beta +- h, +- 2h (nodes and weights move smoothly with beta).
void rule_weights_dbeta(int scheme, double beta, double tau, int np, int np1, int ns, int lag, int64_t N,
                        double h, double* dw) {
    if (N < lag) return;
    const double off[5] = {-2.0 * h, -h, h, 2.0 * h, 0.0};
    const double cf[5] = {1.0 / (12.0 * h), -8.0 / (12.0 * h), 8.0 / (12.0 * h), -1.0 / (12.0 * h), 0.0};
    const size_t len = size_t(N - lag + 1);
    std::vector<double> dq(len, 0.0), q(len, 0.0);
    for (int e = 0; e < 5; ++e) {
        FastRule r;
        build_rule(scheme, beta + off[e], 1.0, np, np1, ns, r);
        shift_lag(r, lag);
        std::vector<double>& acc = (e < 4) ? dq : q;
        const double f = (e < 4) ? cf[e] : 1.0;
        for (size_t j = 0; j < r.ratio.size(); ++j) {
            double pw = r.coef[j] * f;
            const double rr = r.ratio[j];
            for (size_t i = 0; i < len; ++i) {
                acc[i] += pw;
                pw *= rr;
            }
        }
    }
    const double tb = std::pow(tau, -beta), lt = std::log(tau);
    for (size_t i = 0; i < len; ++i) dw[int64_t(i) + lag] = tb * (dq[i] - lt * q[i]);
}

int choose_rule(int scheme, double beta, double tau, int64_t N, double tol, int np_max, int np1,
                int ns, FastRule& out) {
    static const int ladder[] = {8,   12,  16,  24,  32,  48,  64,  96,  128, 160, 192,
                                 256, 320, 384, 448, 512, 576, 640, 768, 896, 1024, 1280, 1536, 2048};
    std::vector<double> d(size_t(N) + 1);
    weights(scheme, beta, tau, N, d.data());
    // fast-vs-direct error grows at most like C n max eps (Section 4); the
    // factor 10 N keeps the measured solution error below tol
    const double target = tol / (10.0 * double(std::max<int64_t>(N, 1)));
    const int lag = (scheme == 1) ? 2 : ns;
    if (N < lag) {  // the window covers every lag: no quadrature needed
        build_rule(scheme, beta, tau, 1, scheme == 2 ? 1 : 0, ns, out);
        out.max_eps = 0.0;
        return CQ_OK;
    }
    for (int np : ladder) {
        if (np > np_max) break;
        build_rule(scheme, beta, tau, np, np1, ns, out);
        out.max_eps = rule_error(out, d, N);
        if (out.max_eps <= target) return CQ_OK;
    }
    return fail(CQ_ETOL, "fast rule: max|eps_i|/d_0 = %.3e > %.3e with np <= %d (beta=%g, N=%lld)", out.max_eps,
                target, np_max, beta, (long long)N);
}

// BDF2 window and first family chosen from the weight errors (Section 5
// picks N_s from the decay of |eps_{2,i}|). Candidates N_s in {12, 16, 20,
// 24, 28, 32} (every lag the time-blocked kernels take) and N_{p,1} in {8,
// 12, 16, 24} (or the caller's); for each, the smallest N_{p,2} on the ladder
// whose rule meets the target for every order beta_k; the pair with the
// least modelled cost per mode, component and step wins:
//   max((4 n + 2 N_s) flops / 78.6, 16 n / min(N_s, 32) bytes / 8),
// n = N_{p,1} + N_{p,2} (the state update and weighting, the exact window;
// the state streamed once per block of min(N_s, 32) steps; FP64 TFLOP/s
// and HBM TB/s of the GPU). The search measures eps_i at every i up to
// 4096 and at ~1% steps beyond (the errors vary slowly there); the winner
// is then checked at every i and moved up the ladder if it falls short.
namespace {
const int kLadder[] = {8,   12,  16,  24,  32,  48,  64,  96,  128, 160, 192,
                       256, 320, 384, 448, 512, 576, 640, 768, 896, 1024, 1280, 1536, 2048};

double rule_error_at(const FastRule& r, const std::vector<double>& d, const std::vector<int64_t>& idx) {
    const int64_t L = r.lag;
    std::vector<double> acc(idx.size(), 0.0);
    const double tiny = 1e-30 * std::fabs(d[0]);
    for (size_t j = 0; j < r.ratio.size(); ++j) {
        const double q = r.ratio[j];
        double p = r.coef[j];
        int64_t at = L;
        for (size_t t = 0; t < idx.size() && std::fabs(p) >= tiny; ++t) {
            const int64_t gap = idx[t] - at;
            if (gap == 1) p *= q;
            else if (gap > 1) p *= std::pow(q, double(gap));
            at = idx[t];
            acc[t] += p;
        }
    }
    double m = 0.0;
    for (size_t t = 0; t < idx.size(); ++t) m = std::max(m, std::fabs(d[size_t(idx[t])] - acc[t]));
    return m / std::fabs(d[0]);
}
}  // namespace

int choose_bdf2_window(const double* betas, int nb, double tau, int64_t N, double tol, int np_max, int np1_fixed,
                       int& ns_out, int& np1_out) {
    static const int ns_c[] = {12, 16, 20, 24, 28, 32};
    static const int np1_c[] = {8, 12, 16, 24};
    const double target = tol / (10.0 * double(std::max<int64_t>(N, 1)));
    std::vector<std::vector<double>> d(static_cast<size_t>(nb));
    for (int k = 0; k < nb; ++k) {
        d[size_t(k)].assign(size_t(N) + 1, 0.0);
        weights(2, betas[k], tau, N, d[size_t(k)].data());
    }
    double best = -1.0;
    int bns = 30, bnp1 = np1_fixed ? np1_fixed : 16, bnp2 = -1;
    FastRule r;
    // Gauss-Jacobi nodes for (1-s)^beta (1+s)^(2-2 beta), both families,
    // computed once per order and size
    std::vector<std::map<int, std::pair<std::vector<double>, std::vector<double>>>> gj(static_cast<size_t>(nb));
    auto nodes = [&](int k, int n) -> const std::pair<std::vector<double>, std::vector<double>>& {
        auto& m = gj[size_t(k)];
        auto it = m.find(n);
        if (it == m.end()) {
            std::pair<std::vector<double>, std::vector<double>> v;
            gauss_jacobi(n, betas[k], 2.0 - 2.0 * betas[k], v.first, v.second);
            it = m.emplace(n, std::move(v)).first;
        }
        return it->second;
    };
    auto make = [&](int k, int np2, int np1, int ns) {
        const auto& a = nodes(k, np1);
        const auto& b = nodes(k, np2);
        bdf2_rule_from_nodes(betas[k], tau, ns, a.first, a.second, b.first, b.second, r);
    };
    for (int ns : ns_c) {
        if (ns > N) break;
        std::vector<int64_t> idx;
        for (int64_t i = ns; i <= N; ++i) {
            if (i <= 4096 || i == N) idx.push_back(i);
            else if (double(i) >= double(idx.back()) * 1.01) idx.push_back(i);
        }
        for (int np1 : np1_c) {
            if (np1_fixed && np1 != np1_fixed) continue;
            int need = 0;  // ladder index meeting the target for every order
            bool ok = true;
            for (int k = 0; k < nb && ok; ++k) {
                int lo = need, hi = int(sizeof(kLadder) / sizeof(int)) - 1;
                while (hi >= lo && kLadder[hi] > np_max) --hi;
                if (hi < lo) { ok = false; break; }
                make(k, kLadder[hi], np1, ns);
                if (rule_error_at(r, d[size_t(k)], idx) > target) { ok = false; break; }
                while (lo < hi) {  // smallest ladder entry that meets the target
                    const int mid = (lo + hi) / 2;
                    make(k, kLadder[mid], np1, ns);
                    if (rule_error_at(r, d[size_t(k)], idx) <= target) hi = mid; else lo = mid + 1;
                }
                need = lo;
            }
            if (!ok) continue;
            const double n = double(np1 + kLadder[need]);
            const double cost = std::max((4.0 * n + 2.0 * ns) / 78.6, 16.0 * n / double(std::min(ns, 32)) / 8.0);
            if (best < 0 || cost < best) {
                best = cost;
                bns = ns;
                bnp1 = np1;
                bnp2 = need;
            }
        }
    }
    if (bnp2 < 0) {  // no candidate: the default window, and the ordinary scan reports any shortfall
        ns_out = 30;
        np1_out = np1_fixed ? np1_fixed : 16;
        return CQ_OK;
    }
    // the winner at every i; up the ladder while it falls short
    const int nl = int(sizeof(kLadder) / sizeof(int));
    for (int k = 0; k < nb; ++k) {
        while (bnp2 < nl && kLadder[bnp2] <= np_max) {
            make(k, kLadder[bnp2], bnp1, bns);
            if (rule_error(r, d[size_t(k)], N) <= target) break;
            ++bnp2;
        }
    }
    ns_out = bns;
    np1_out = bnp1;
    return CQ_OK;
}

// ---------------------------------------------------------------------------
void eig2(const double K[2][2], double theta[2], double V[2][2], double Vinv[2][2]) {
    const double tr2 = 0.5 * (K[0][0] + K[1][1]);
    const double df2 = 0.5 * (K[0][0] - K[1][1]);
    const double off = K[0][1] * K[1][0];  // >= 0 here (= a^2)
    const double rad = std::sqrt(std::max(0.0, df2 * df2 + off));
    if (off == 0.0) {
        theta[0] = K[0][0];
        theta[1] = K[1][1];
        V[0][0] = 1; V[0][1] = 0; V[1][0] = 0; V[1][1] = 1;
        Vinv[0][0] = 1; Vinv[0][1] = 0; Vinv[1][0] = 0; Vinv[1][1] = 1;
        return;
    }
    // theta0 pairs with component 1 when K11 <= K22 (keeps V near identity)
    const double sgn = (df2 >= 0.0) ? 1.0 : -1.0;
    theta[0] = tr2 + sgn * rad;  // closest to K11
    theta[1] = tr2 - sgn * rad;  // closest to K22
    // eigenvector for theta0: (theta0 - K22, K21); for theta1: (K12, theta1 - K11)
    double v0x = theta[0] - K[1][1], v0y = K[1][0];
    double v1x = K[0][1], v1y = theta[1] - K[0][0];
    const double n0 = std::hypot(v0x, v0y), n1 = std::hypot(v1x, v1y);
    v0x /= n0; v0y /= n0; v1x /= n1; v1y /= n1;
    V[0][0] = v0x; V[1][0] = v0y;  // columns are eigenvectors
    V[0][1] = v1x; V[1][1] = v1y;
    const double det = V[0][0] * V[1][1] - V[0][1] * V[1][0];
    Vinv[0][0] = V[1][1] / det;
    Vinv[0][1] = -V[0][1] / det;
    Vinv[1][0] = -V[1][0] / det;
    Vinv[1][1] = V[0][0] / det;
}


// ---------------------------------------------------------------------------
// Tables of the 16-mode MFMA kernel (k_modal_batch_mx) for one problem: the
// fragments of the step-by-node table w_j r_j^{t+1}, the node-by-step table
// r_j^{B-1-s}, r_j^B, the in-block Toeplitz table of c_e = sum_j w_j r_j^e
// and the exact-window table of the earlier levels, in the fragment order of
// the kernel's MFMA operands (layout at the kernel).
bool mx_applies(int L, int np) { return L >= kMxMinLag && L <= kMxMaxLag && (np + 15) / 16 <= 2 * kMxMaxNtw; }

int mx_template(int ntw) {
    for (int t : {4, 5, 6, 7, 8, 9, 10, 12, 13, 14, 16, 18, 19})
        if (ntw <= t) return t;
    return 19;
}

void build_mx_tables(int np, int L, const double* const ratio[2], const double* const coef[2],
                     const double* const d[2], double* out) {
    const int nt = (np + 15) / 16, B = kMxB;
    const int64_t t1 = int64_t(nt + 1) * 256;  // a component's W or R: nt tiles and a zero tile
    double* W = out;
    double* R = out + 2 * t1;
    double* rB = out + 4 * t1;
    double* Cf = rB + int64_t(32) * nt;
    double* Df = Cf + 512;
    std::fill(out, out + mx_table_size(nt), 0.0);
    for (int k = 0; k < 2; ++k) {
        // pw[j][e] = r_j^e, e <= B
        std::vector<double> pw(size_t(nt) * 16 * (B + 1), 0.0);
        for (int j = 0; j < np; ++j) {
            double v = 1.0;
            for (int e = 0; e <= B; ++e) {
                pw[size_t(j) * (B + 1) + e] = v;
                v *= ratio[k][j];
            }
        }
        auto P = [&](int j, int e) { return j < np ? pw[size_t(j) * (B + 1) + e] : 0.0; };
        auto wj = [&](int j) { return j < np ? coef[k][j] : 0.0; };
        for (int jt = 0; jt < nt; ++jt)
            for (int i = 0; i < 4; ++i)
                for (int ln = 0; ln < 64; ++ln) {
                    const size_t o = size_t(k) * size_t(t1) + (size_t(jt) * 4 + i) * 64 + ln;
                    const int t = ln % 16, lk = ln / 16;
                    const int jw = 16 * jt + 4 * i + lk;
                    W[o] = wj(jw) * P(jw, t + 1);
                    const int jr = 16 * jt + t, sidx = 4 * i + lk;
                    R[o] = P(jr, B - 1 - sidx);
                }
        for (int j = 0; j < 16 * nt; ++j) rB[size_t(k) * 16 * nt + j] = P(j, B);
        long double c[B];
        for (int e = 0; e < B; ++e) {
            long double acc = 0.0L;
            for (int j = 0; j < np; ++j) acc += (long double)coef[k][j] * (long double)P(j, e);
            c[e] = acc;
        }
        for (int i = 0; i < 4; ++i)
            for (int ln = 0; ln < 64; ++ln) {
                const int t = ln % 16, sidx = 4 * i + ln / 16;
                Cf[size_t(k) * 256 + i * 64 + ln] = sidx <= t ? double(c[t - sidx]) : 0.0;
            }
        for (int i = 0; i < 8; ++i)
            for (int ln = 0; ln < 64; ++ln) {
                const int t = ln % 16, u = 4 * i + ln / 16, lag = t + 1 + u;
                Df[size_t(k) * 512 + i * 64 + ln] = lag <= L - 1 ? d[k][lag] : 0.0;
            }
    }
}

}  // namespace cqfp
