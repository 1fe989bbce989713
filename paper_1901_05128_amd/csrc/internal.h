// Internal declarations shared by the host setup, the kernels and the C ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/cqfp.h"

namespace cqfp {

// ---- error reporting (thread-local message behind cq_last_error) ----
int fail(int code, const char* fmt, ...);
void clear_error();

// ---- host setup (setup.cpp) ----

// Weights d_i, i = 0..n, of ((1-z)/tau)^beta (scheme 1) or
// (((1-z)+(1-z)^2/2)/tau)^beta (scheme 2), by first-order recurrences.
void weights(int scheme, double beta, double tau, int64_t n, double* d);
// d/dbeta of those weights, i = 0..n (the recurrences differentiated).
void weights_dbeta(int scheme, double beta, double tau, int64_t n, double* dd);

// Gauss-Jacobi nodes s_j (ascending) and weights lam_j for the weight
// (1-s)^a (1+s)^b on [-1,1]: eigenvalues of the Jacobi matrix by Sturm
// bisection, Newton polish, Christoffel weights 1/sum_k p_k(s_j)^2.
void gauss_jacobi(int n, double a, double b, std::vector<double>& s, std::vector<double>& lam);

struct FastRule {
    std::vector<double> ratio;  // r_j
    std::vector<double> coef;   // coefficient of r_j^(i - lag)
    int lag = 2;
    double max_eps = 0.0;       // max |eps_i| / |d_0| over lag <= i <= N
};

// Build the rule for a given node count (np for BE, np1 + np2 for BDF2).
void build_rule(int scheme, double beta, double tau, int np, int np1, int ns, FastRule& out);
// BDF2 rule (3.14)-(3.16) from the Gauss-Jacobi nodes and weights of its two
// families (np1 = s1.size(), np2 = s2.size()).
void bdf2_rule_from_nodes(double beta, double tau, int ns, const std::vector<double>& s1,
                          const std::vector<double>& lam1, const std::vector<double>& s2,
                          const std::vector<double>& lam2, FastRule& out);
// Start the geometric families at a later lag (coef_j *= r_j^(lag - old lag)).
void shift_lag(FastRule& r, int lag);
// max_{lag <= i <= N} |d_i - sum_j coef_j r_j^(i-lag)| / |d_0|
double rule_error(const FastRule& r, const std::vector<double>& d, int64_t N);
// Node-count scan; returns CQ_OK or CQ_ETOL.
int choose_rule(int scheme, double beta, double tau, int64_t N, double tol, int np_max, int np1,
                int ns, FastRule& out);

// BDF2: N_s and N_{p,1} chosen from the weight errors for the orders betas[0..nb)
// (candidates and cost model in setup.cpp); np1_fixed > 0 keeps N_{p,1}.
int choose_bdf2_window(const double* betas, int nb, double tau, int64_t N, double tol, int np_max, int np1_fixed,
                       int& ns_out, int& np1_out);

// d/dbeta of the fast weights of an np-node rule (BDF2: np1 + np) started at
// lag, for lag <= i <= N (five-point difference in beta, step h).
void rule_weights_dbeta(int scheme, double beta, double tau, int np, int np1, int ns, int lag, int64_t N,
                        double h, double* dw);

// Eigen-decomposition of the 2x2 coupling K (real eigenvalues, since
// K12*K21 >= 0): K = V diag(theta) V^{-1}.
void eig2(const double K[2][2], double theta[2], double V[2][2], double Vinv[2][2]);

// 16-mode MFMA kernel (batch_mx.hip): whether a problem's lag and node count
// fit it, the node-tile template for ntw tiles per wave, and its tables for
// one problem (np nodes per component, lag L; d[k] readable up to lag L - 1;
// out holds mx_table_size((np + 15) / 16) doubles).
bool mx_applies(int L, int np);
int mx_template(int ntw);
void build_mx_tables(int np, int L, const double* const ratio[2], const double* const coef[2],
                     const double* const d[2], double* out);

// ---- kernel launchers (kernels.hip) ----
struct DevSolver;  // defined in runtime.cpp

}  // namespace cqfp
