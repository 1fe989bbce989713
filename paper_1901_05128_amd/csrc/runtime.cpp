// C ABI of the CQ solver: argument checks, solver set-up, device buffers and
// the per-step launch sequence (see include/cqfp.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <new>
#include <vector>

#include "internal.h"
#include "kernels.h"

namespace cqfp {
const char* last_error();
}

using namespace cqfp;

#define HIPCHK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) return fail(CQ_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

namespace {

constexpr uint64_t kStateMagic = 0x43514650u;  // "CQFP"
constexpr int64_t kModalBlockedMin = 8192;      // modes
constexpr int64_t kDwPad = 256;                 // zero lags in front of the d/dbeta weights (>= pass rows)
// modal direct: rows of one far-field pass. Measured: 192 and 256 are 4%
// faster than 128 on the 1D 1023-node workload (the levels split over the
// waves of a workgroup); 256 is 2.5% faster than 128 on 2D 255^2.
int modal_far_pass(int64_t M) { return M >= 8192 ? 256 : 192; }

// device arrays of a gradient handle (trajectory, history sums, adjoint)
struct AdjBufs {
    double *traj = nullptr, *Sx = nullptr, *psi = nullptr, *mu = nullptr, *gc = nullptr, *gG0c = nullptr,
           *acc = nullptr, *dw = nullptr, *dd = nullptr, *part = nullptr, *part2 = nullptr;
    int nblk_da = 0, nblk_rows = 0, nchunk = 1;
    // d/dbeta in blocks of spec_bk steps (0: Toeplitz passes over all
    // levels): exact near field over the previous and the current block, and
    // for nb > 2 blocks the farther block pairs through block DFTs of P =
    // 2 spec_bk points (twiddles, window spectra of dw, partial spectra per
    // workgroup, per-block dot products)
    double *tw = nullptr, *W = nullptr, *spec = nullptr, *bpart = nullptr;
    int spec_bk = 0, specP = 0, specLog = 0, spec_nb = 0, spec_nwg = 0, spec_cols = 0, nblk_dot = 0;
    int64_t per = 1;  // steps per chunk of the time-chunked reductions
    // Checkpointed form (fast method): the forward trajectory is not kept.
    // The steps are cut into nseg segments of seg steps; the forward state at
    // a segment start (the fast state H and the last L levels) can be saved
    // in `slots` places, and a binomial schedule (split) decides where the
    // forward is advanced to and saved. Each segment is recomputed once more
    // with its levels and history sums in segLev / segS, the adjoint sweep
    // (own state Ha, Sfa; psi kept whole, mu in segMu) takes the segment's
    // steps, and the segment's share of the gradient sums is added.
    bool ckpt = false;
    int64_t seg = 0, ck_stride = 0, fwd_steps = 0;
    int nseg = 0, slots = 0;
    double *ck = nullptr, *segLev = nullptr, *segS = nullptr, *segMu = nullptr, *ringA = nullptr, *Ha = nullptr,
           *Sfa = nullptr;
    double *Hf = nullptr, *Sff = nullptr;  // the forward's fast state and block sums
    bool mxfwd = false;  // kept-whole fast sweeps on the 16-mode MFMA kernel (Solver::mx)
    // with mxfwd and the block DFTs, where the budget holds them: the columns
    // b_t = g^{t+1} and a_t = psi^{t+1} ([2M][N]) as the sweeps write them
    // (else transposed into Sx and mu after the sweeps)
    double *colG = nullptr, *colPsi = nullptr;
    std::vector<int> split;  // [nseg + 1][slots]: first advance (segments) of an optimal schedule
    std::vector<int64_t> cost;
};

// One problem on the 16-mode MFMA kernel (k_modal_batch_mx): its tables, the
// problem entry, the one-problem list and tile counts (device), the template
struct MxRun {
    bool on = false;
    double* tab = nullptr;
    BatchInst* inst = nullptr;
    int* list = nullptr;
    int64_t* cum = nullptr;
    int64_t tiles = 0;
    int ntw = 0;
};

struct Solver {
    cq_grid g{};
    cq_params p{};
    MxRun mx;  // fast form on the 16-mode MFMA kernel (whole runs, gradient sweeps)
    int dim = 1, nx = 1, ny = 1, nz = 1;
    int64_t M = 0, N = 0, n = 0;
    double tau = 0, a = 0, beta[2] = {0, 0}, c = 0, hx = 0, hy = 0, hz = 0;
    hipStream_t st = nullptr;
    // fast
    int L = 2, np = 0, hlanes = 1, chunk = 0, Bt = 1, BTt = 8;
    int ns_used = 30, np1_used = 16;  // BDF2: N_s and N_{p,1} of the fast rule
    // fast form, blocked: the first state block is blk_off steps long (0: a
    // full block), the rest Bt; the adjoint sweep takes blk_off = N mod Bt so
    // that its block ends fall on the forward's block starts in reversed time
    int64_t blk_off = 0;
    int64_t hstride = 0;  // DOFs between nodes of the state H[2][np][hstride]
    double max_eps = 0;
    // direct
    int B = 0, ks = 1;
    int64_t n0 = 0;
    // modal direct: one pass over the history serves Bf/B blocks. The pass
    // of the block n0 starts at far_base = (n0/Bf)*Bf and covers the levels
    // 1..far_base for the rows far_base+1 .. far_base+Bf (in F); F2 holds the
    // levels far_base+1..n0 for the block mid_n0. Both depend on n0 alone,
    // so a resumed run repeats the arithmetic of an uninterrupted one.
    // -1: not computed.
    int Bf = 64;
    int64_t far_base = -1, mid_n0 = -1;
    double* F2 = nullptr;
    int64_t Lr = 0;
    int64_t dstride = 0;
    std::vector<double> dh[2];
    FastRule rule[2];
    double theta[2] = {0, 0}, V[2][2] = {{1, 0}, {0, 1}}, Vinv[2][2] = {{1, 0}, {0, 1}};
    // device buffers
    double *d_d = nullptr, *d_ratio = nullptr, *d_coef = nullptr, *G0 = nullptr, *levels = nullptr,
           *H = nullptr, *Spart = nullptr, *F = nullptr, *rhs = nullptr, *T1 = nullptr, *T2 = nullptr,
           *Sx = nullptr, *Sy = nullptr, *lamx = nullptr, *lamy = nullptr, *qbuf = nullptr, *Sf = nullptr, *PF = nullptr, *PG = nullptr, *PRB = nullptr, *lam = nullptr,
           *g0c = nullptr, *ring = nullptr;
    // 3D: sine matrix and eigenvalues along z; the eigenvalues of the (y, x)
    // modes of one z-plane (the nodal solve's epilogue adds lamz[r])
    double *Sz = nullptr, *lamz = nullptr, *lamxy = nullptr;
    int levels_pcr = 0;
    bool modal_blocked = false;  // modal fast form with the state streamed in time blocks
    // gradient runs (modal): forward history sums, adjoint sweep
    bool adj = false;
    double *Sout = nullptr, *mu = nullptr;
    const double* gc = nullptr;
    double* Sscratch = nullptr;  // [2][M] row the modal kernels write S to when Sout is not kept
    int kind = 0;                // 0 stepping solver (fp_create), 1 gradient handle (fp_adjoint_create)
    AdjBufs ab;
    size_t lds = 0;
    size_t dev_bytes = 0;
    std::vector<void*> allocs;

    ~Solver() {
        for (void* q : allocs) (void)hipFree(q);
    }
};

// K-split of the far field: about 512 workgroups, at most 32 slices. More
// slices add partial sums that are written and read back once per pass;
// measured, 512 beat 768..3072 (and tied 256) on the 1D workload and
// tied on the 2D one.
#ifndef CQFP_FAR_WORKGROUPS
#define CQFP_FAR_WORKGROUPS 512
#endif
int far_ksplit(int64_t M) {
    const int64_t tiles = 2 * ((M + 63) / 64);
    const int64_t wg = CQFP_FAR_WORKGROUPS;
    return int(std::min<int64_t>(32, std::max<int64_t>(1, (wg + tiles / 2) / tiles)));  // nearest
}

// slices for one launch: at least 64 levels per slice
int far_ks_for(int ks, int64_t nl) { return int(std::max<int64_t>(1, std::min<int64_t>(ks, (nl + 63) / 64))); }

// values of the fast-history state H
size_t hcount(const Solver& s) { return size_t(2) * size_t(s.np) * size_t(s.hstride); }

// slots of the modal few-mode level ring (the time-blocked kernel keeps 2L)
int ring_slots(const Solver& s) { return modal_fast_blocked(s.L, s.np) ? 2 * s.L : s.L; }

int dev_alloc(Solver& s, double** ptr, size_t count) {
    void* q = nullptr;
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(double);
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? CQ_ENOMEM : CQ_EHIP, "hipMalloc(%zu bytes): %s", bytes,
                    hipGetErrorString(e));
    }
    s.allocs.push_back(q);
    s.dev_bytes += bytes;
    *ptr = static_cast<double*>(q);
    return CQ_OK;
}

double lambda_1d(int n, double len, int p) {  // p = 1..n
    const double h = len / (n + 1);
    const double sn = std::sin(p * M_PI / (2.0 * (n + 1)));
    return 4.0 / (h * h) * sn * sn;
}

int validate(const cq_grid* g, const cq_params* p) {
    if (!g || !p) return fail(CQ_EINVAL, "grid and params must not be NULL");
    if (g->dim < 1 || g->dim > 3) return fail(CQ_EINVAL, "dim must be 1, 2 or 3 (got %d)", g->dim);
    if (g->nx < 1 || g->ny < 1) return fail(CQ_EINVAL, "nx, ny must be >= 1");
    if (g->dim == 1 && g->ny != 1) return fail(CQ_EINVAL, "dim 1 needs ny = 1");
    if (g->dim < 3 && g->nz != 0 && g->nz != 1) return fail(CQ_EINVAL, "dim %d needs nz = 0 or 1", g->dim);
    if (g->dim == 3 && g->nz < 1) return fail(CQ_EINVAL, "nz must be >= 1");
    if (g->dim == 1 && g->nx > 4096) return fail(CQ_EINVAL, "1D grids are limited to 4096 nodes (got %d)", g->nx);
    if (g->dim == 3 && int64_t(g->ny) * g->nz > (int64_t(1) << 20))
        return fail(CQ_EINVAL, "3D grids are limited to ny * nz <= 2^20 (got %d x %d)", g->ny, g->nz);
    if (!(g->lx > 0) || (g->dim >= 2 && !(g->ly > 0)) || (g->dim == 3 && !(g->lz > 0)))
        return fail(CQ_EINVAL, "domain lengths must be > 0");
    if (!(p->alpha1 > 0 && p->alpha1 < 1 && p->alpha2 > 0 && p->alpha2 < 1))
        return fail(CQ_EINVAL, "alpha1, alpha2 must lie in (0,1)");
    if (!(p->m >= 0 && p->m <= 1) || p->m == 0.5) return fail(CQ_EINVAL, "m must lie in [0,1] without 1/2");
    if (!(p->T > 0) || !std::isfinite(p->T)) return fail(CQ_EINVAL, "T must be > 0");
    if (p->N < 1) return fail(CQ_EINVAL, "N must be >= 1");
    if (p->scheme != 1 && p->scheme != 2) return fail(CQ_EINVAL, "scheme must be 1 (BE) or 2 (BDF2)");
    if (p->method != 0 && p->method != 1) return fail(CQ_EINVAL, "method must be 0 (direct) or 1 (fast)");
    if (p->np < 0 || p->np1 < 0 || p->ns < 0 || p->np_max < 0 || p->block_B < 0 || p->fast_tol < 0)
        return fail(CQ_EINVAL, "node counts, window, block and tolerance must be >= 0");
    if (p->scheme == 2 && p->ns != 0 && p->ns < 3) return fail(CQ_EINVAL, "ns must be >= 3 (got %d)", p->ns);
    if (p->block_B != 0 && (p->block_B % 64 != 0 || p->block_B > 256))
        return fail(CQ_EINVAL, "block_B must be 64, 128, 192 or 256 (got %d)", p->block_B);
    if (p->np > 4096 || p->np1 > 4096) return fail(CQ_EINVAL, "np, np1 must be <= 4096");
    if (p->solver != 0 && p->solver != 1) return fail(CQ_EINVAL, "solver must be 0 (nodal) or 1 (modal)");
    if (p->fast_kernel != 0 && p->fast_kernel != 1) return fail(CQ_EINVAL, "fast_kernel must be 0 or 1");
    return CQ_OK;
}

// PCR eliminations of T_k = tridiag(-1, fl(2 + theta_k h^2), -1), k = 0, 1:
// per level l (stride 2^l) and row i the multipliers f = a_i/b_{i-s},
// g = c_i/b_{i+s}; after the last level 1/b_i. Layout [levels][2][M], [2][M].
void pcr_multipliers(int64_t M, int levels, const double theta[2], double h, std::vector<double>& pf,
                     std::vector<double>& pg, std::vector<double>& prb) {
    const size_t nl = size_t(std::max(1, levels));
    pf.assign(nl * 2 * size_t(M), 0.0);
    pg.assign(nl * 2 * size_t(M), 0.0);
    prb.assign(2 * size_t(M), 0.0);
    for (int k = 0; k < 2; ++k) {
        const size_t Mz = static_cast<size_t>(M);
        std::vector<double> a(Mz), b(Mz), c(Mz), na(Mz), nb(Mz), nc(Mz);
        for (int64_t i = 0; i < M; ++i) {
            a[size_t(i)] = i > 0 ? -1.0 : 0.0;
            c[size_t(i)] = i + 1 < M ? -1.0 : 0.0;
            b[size_t(i)] = 2.0 + theta[k] * h * h;
        }
        int64_t s = 1;
        for (int l = 0; l < levels; ++l, s <<= 1) {
            for (int64_t i = 0; i < M; ++i) {
                double a2 = 0.0, c2 = 0.0, bb = b[size_t(i)], f = 0.0, g = 0.0;
                if (i - s >= 0) {
                    f = a[size_t(i)] / b[size_t(i - s)];
                    a2 = -a[size_t(i - s)] * f;
                    bb -= c[size_t(i - s)] * f;
                }
                if (i + s < M) {
                    g = c[size_t(i)] / b[size_t(i + s)];
                    c2 = -c[size_t(i + s)] * g;
                    bb -= a[size_t(i + s)] * g;
                }
                pf[(size_t(l) * 2 + k) * size_t(M) + size_t(i)] = f;
                pg[(size_t(l) * 2 + k) * size_t(M) + size_t(i)] = g;
                na[size_t(i)] = a2;
                nb[size_t(i)] = bb;
                nc[size_t(i)] = c2;
            }
            a.swap(na);
            b.swap(nb);
            c.swap(nc);
        }
        for (int64_t i = 0; i < M; ++i) prb[size_t(k) * size_t(M) + size_t(i)] = 1.0 / b[size_t(i)];
    }
}

int setup_host(Solver& s, const cq_grid* g, const cq_params* p, hipStream_t st) {
    s.g = *g;
    s.p = *p;
    s.dim = g->dim;
    s.nx = g->nx;
    s.ny = g->dim >= 2 ? g->ny : 1;
    s.nz = g->dim == 3 ? g->nz : 1;
    s.M = int64_t(s.nx) * s.ny * s.nz;
    s.N = p->N;
    s.st = st;
    s.tau = p->T / double(p->N);
    s.a = (1.0 - p->m) / (2.0 * p->m - 1.0);
    s.beta[0] = 1.0 - p->alpha1;
    s.beta[1] = 1.0 - p->alpha2;
    s.c = (p->scheme == 1 ? 1.0 : 1.5) / s.tau;
    s.hx = g->lx / (s.nx + 1);
    s.hy = s.dim >= 2 ? g->ly / (s.ny + 1) : 1.0;
    s.hz = s.dim == 3 ? g->lz / (s.nz + 1) : 1.0;
    int ns = p->ns ? p->ns : 30;
    int np1 = p->np1 ? p->np1 : 16;
    const int np_max = p->np_max ? p->np_max : 1024;
    const double tol = p->fast_tol > 0 ? p->fast_tol : 1e-8;
    // BDF2 with the node count left to the scan: N_s (and N_{p,1} unless
    // given) from the weight errors too
    if (p->method == 1 && p->scheme == 2 && p->ns == 0 && p->np == 0)
        choose_bdf2_window(s.beta, 2, s.tau, s.N, tol, np_max, p->np1, ns, np1);
    s.ns_used = ns;
    s.np1_used = np1;

    // direct block length and K-split (enough workgroups to fill 256 CUs)
    if (p->method == 0) {
        s.B = p->block_B ? p->block_B : (s.dim == 1 ? 64 : 128);
        if (p->solver == 1) {  // the modal near field keeps a 64-step block in registers
            s.B = 64;
            s.Bf = p->block_B ? p->block_B : modal_far_pass(s.M);
        }
        s.ks = far_ksplit(s.M);
    }
    s.dstride = s.N + 257 + 1;
    for (int k = 0; k < 2; ++k) {
        s.dh[k].assign(size_t(s.dstride), 0.0);
        weights(p->scheme, s.beta[k], s.tau, s.dstride - 1, s.dh[k].data());
    }

    // step operator: diag(d0) (I x A + K x I), K as below; must be positive definite
    const double d10 = s.dh[0][0], d20 = s.dh[1][0];
    const double K[2][2] = {{s.c / d10 + s.a, -s.a * d20 / d10}, {-s.a * d10 / d20, s.c / d20 + s.a}};
    eig2(K, s.theta, s.V, s.Vinv);
    double lam_min = lambda_1d(s.nx, g->lx, 1);
    if (s.dim >= 2) lam_min += lambda_1d(s.ny, g->ly, 1);
    if (s.dim == 3) lam_min += lambda_1d(s.nz, g->lz, 1);
    for (int k = 0; k < 2; ++k)
        if (!(s.theta[k] + lam_min > 0))
            return fail(CQ_ESINGULAR,
                        "step operator not positive definite: theta_%d = %.6g <= -lambda_min = %.6g "
                        "(take a smaller tau or m further from 1/2)",
                        k + 1, s.theta[k], -lam_min);

    // fast rule: one node count for both components
    FastRule rule[2];
    if (p->method == 1) {
        int npk[2];
        for (int k = 0; k < 2; ++k) {
            if (p->np > 0) {
                build_rule(p->scheme, s.beta[k], s.tau, p->np, np1, ns, rule[k]);
                std::vector<double> dk(s.dh[k].begin(), s.dh[k].begin() + s.N + 1);
                rule[k].max_eps = rule_error(rule[k], dk, s.N);
            } else {
                int rc = choose_rule(p->scheme, s.beta[k], s.tau, s.N, tol, np_max, np1, ns, rule[k]);
                if (rc != CQ_OK) return rc;
            }
            npk[k] = int(rule[k].ratio.size());
        }
        if (npk[0] != npk[1]) {  // rebuild the smaller one at the common size
            const int k = npk[0] < npk[1] ? 0 : 1;
            const int target = std::max(npk[0], npk[1]) - (p->scheme == 2 ? np1 : 0);
            build_rule(p->scheme, s.beta[k], s.tau, target, np1, ns, rule[k]);
            std::vector<double> dk(s.dh[k].begin(), s.dh[k].begin() + s.N + 1);
            rule[k].max_eps = rule_error(rule[k], dk, s.N);
        }
        // BE: the Gauss-Jacobi rule is exact for lags 2..2np+1, so summing lags
        // below L' with the exact weights and the rest with the rule is the
        // same fast scheme; a window of up to 32 lets the state advance in
        // blocks of up to 32 steps
        if (p->scheme == 1) {
            const int Lw = std::min(32, 2 * int(rule[0].ratio.size()) + 2);
            shift_lag(rule[0], Lw);
            shift_lag(rule[1], Lw);
        }
        s.np = int(rule[0].ratio.size());
        s.L = rule[0].lag;
        if (s.np > 1024)
            return fail(CQ_EINVAL, "the fast form keeps at most 1024 nodes per component (got %d)", s.np);
        if (p->solver == 1 && s.L > 64)
            return fail(CQ_EINVAL, "modal fast solver needs lag <= 64 (lag %d)", s.L);
        s.Bt = std::min(s.L, 32);
        s.BTt = s.Bt <= 8 ? 8 : (s.Bt <= 16 ? 16 : (s.Bt <= 24 ? 24 : (s.Bt <= 30 ? 30 : 32)));
        s.max_eps = std::max(rule[0].max_eps, rule[1].max_eps);
        // waves per 64-DOF tile in the state pass (node slices): enough for
        // ~1536 waves (1.5 per SIMD; the pass holds ~165 registers per lane,
        // three waves per SIMD), at least 8 nodes per slice, 1, 2 or 4
        const int64_t waves = (2 * s.M + 63) / 64;
        int want = int(std::max<int64_t>(1, (1536 + waves - 1) / waves));
        want = std::min(want, std::max(1, s.np / 8));
        s.hlanes = 1;
        while (s.hlanes < want && s.hlanes < 4) s.hlanes *= 2;
        s.chunk = (s.np + s.hlanes - 1) / s.hlanes;
        s.Lr = s.L;
    } else {
        s.Lr = s.N + 1;
    }
    s.rule[0] = rule[0];
    s.rule[1] = rule[1];
    return CQ_OK;
}

// sine tables: S[i][j] = sin(pi (i+1)(j+1)/(n+1)) (symmetric, S S = (n+1)/2 I)
// and eigenvalues lambda_q of the 3-point Dirichlet Laplacian
std::vector<double> sine_matrix(int n) {
    std::vector<double> S(size_t(n) * size_t(n));
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            // reduce the integer argument first: sin(pi k/(n+1)), k mod 2(n+1)
            const int64_t kk = (int64_t(i + 1) * (j + 1)) % (2 * int64_t(n + 1));
            S[size_t(i) * size_t(n) + size_t(j)] = std::sin(M_PI * double(kk) / double(n + 1));
        }
    return S;
}

int upload(double* dst, const std::vector<double>& v) {
    HIPCHK(hipMemcpy(dst, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice));
    return CQ_OK;
}

int setup_tables(Solver& s) {
    int rc;
    const cq_grid* g = &s.g;
    if ((rc = dev_alloc(s, &s.Sx, size_t(s.nx) * s.nx))) return rc;
    if ((rc = dev_alloc(s, &s.lamx, size_t(s.nx)))) return rc;
    std::vector<double> lx(size_t(s.nx));
    for (int q = 0; q < s.nx; ++q) lx[size_t(q)] = lambda_1d(s.nx, g->lx, q + 1);
    if ((rc = upload(s.Sx, sine_matrix(s.nx)))) return rc;
    if ((rc = upload(s.lamx, lx))) return rc;
    std::vector<double> ly(1, 0.0), lz(1, 0.0);
    if (s.dim >= 2) {
        if ((rc = dev_alloc(s, &s.Sy, size_t(s.ny) * s.ny))) return rc;
        if ((rc = dev_alloc(s, &s.lamy, size_t(s.ny)))) return rc;
        ly.assign(size_t(s.ny), 0.0);
        for (int q = 0; q < s.ny; ++q) ly[size_t(q)] = lambda_1d(s.ny, g->ly, q + 1);
        if ((rc = upload(s.Sy, sine_matrix(s.ny)))) return rc;
        if ((rc = upload(s.lamy, ly))) return rc;
    }
    if (s.dim == 3) {
        if ((rc = dev_alloc(s, &s.Sz, size_t(s.nz) * s.nz))) return rc;
        if ((rc = dev_alloc(s, &s.lamz, size_t(s.nz)))) return rc;
        lz.assign(size_t(s.nz), 0.0);
        for (int r = 0; r < s.nz; ++r) lz[size_t(r)] = lambda_1d(s.nz, g->lz, r + 1);
        if ((rc = upload(s.Sz, sine_matrix(s.nz)))) return rc;
        if ((rc = upload(s.lamz, lz))) return rc;
        std::vector<double> lxy(size_t(s.ny) * size_t(s.nx));
        for (int j = 0; j < s.ny; ++j)
            for (int i = 0; i < s.nx; ++i) lxy[size_t(j) * size_t(s.nx) + size_t(i)] = ly[size_t(j)] + lx[size_t(i)];
        if ((rc = dev_alloc(s, &s.lamxy, lxy.size()))) return rc;
        if ((rc = upload(s.lamxy, lxy))) return rc;
    }
    if (s.p.solver == 1) {  // eigenvalue of every mode, layout [nz][ny][nx] (x-mode fastest)
        if ((rc = dev_alloc(s, &s.lam, size_t(s.M)))) return rc;
        std::vector<double> lm(size_t(s.M));
        for (int r = 0; r < s.nz; ++r)
            for (int j = 0; j < s.ny; ++j)
                for (int i = 0; i < s.nx; ++i)
                    lm[(size_t(r) * size_t(s.ny) + size_t(j)) * size_t(s.nx) + size_t(i)] =
                        lz[s.dim == 3 ? size_t(r) : 0] + ly[s.dim >= 2 ? size_t(j) : 0] + lx[size_t(i)];
        if ((rc = upload(s.lam, lm))) return rc;
    }
    return CQ_OK;
}

// sine coefficients of both components: out = S G (1D, scaled 2/(n+1)),
// S_y G S_x (2D, scaled 4/((nx+1)(ny+1))) or the same along z as well (3D,
// scaled 8/((nx+1)(ny+1)(nz+1))); the inverse is unscaled. tmp: s.T1.
void transform(Solver& s, const double* G, double* out, bool forward) {
    double scale = 1.0;
    if (forward) {
        scale = 2.0 / double(s.nx + 1);
        if (s.dim >= 2) scale *= 2.0 / double(s.ny + 1);
        if (s.dim == 3) scale *= 2.0 / double(s.nz + 1);
    }
    launch_sine_transform(s.dim, s.nx, s.ny, s.nz, s.Sx, s.Sy, s.Sz, G, s.T1, out, scale, s.st);
}

// (re)start a modal solver from G0 (already in s.G0): coefficients of G0,
// zero state, level 0 (and the BDF2 level -1 := 0) in place
int modal_start(Solver& s) {
    const int64_t twoM = 2 * s.M;
    transform(s, s.G0, s.g0c, true);
    if (s.p.method == 1 && s.modal_blocked) {
        HIPCHK(hipMemsetAsync(s.H, 0, hcount(s) * sizeof(double), s.st));
        HIPCHK(hipMemsetAsync(s.levels, 0, size_t(s.Lr) * size_t(twoM) * sizeof(double), s.st));
        HIPCHK(hipMemcpyAsync(s.levels, s.g0c, size_t(twoM) * sizeof(double), hipMemcpyDeviceToDevice, s.st));
    } else if (s.p.method == 1) {
        HIPCHK(hipMemsetAsync(s.H, 0, hcount(s) * sizeof(double), s.st));
        HIPCHK(hipMemsetAsync(s.ring, 0, size_t(ring_slots(s)) * size_t(twoM) * sizeof(double), s.st));
        HIPCHK(hipMemcpyAsync(s.ring, s.g0c, size_t(twoM) * sizeof(double), hipMemcpyDeviceToDevice, s.st));
        if (!modal_fast_blocked(s.L, s.np))  // per-step ring: level -1 := level 0
            HIPCHK(hipMemcpyAsync(s.ring + twoM, s.g0c, size_t(twoM) * sizeof(double), hipMemcpyDeviceToDevice,
                                  s.st));
    } else {
        HIPCHK(hipMemcpyAsync(s.levels, s.g0c, size_t(twoM) * sizeof(double), hipMemcpyDeviceToDevice, s.st));
    }
    HIPCHK(hipGetLastError());
    return CQ_OK;
}

// Tables and the one-problem launch data of the 16-mode MFMA kernel
// (fast method, modal solver; the caller checks mx_applies).
static int setup_mx(Solver& s) {
    int rc;
    const int nt = (s.np + 15) / 16;
    std::vector<double> tab(size_t(mx_table_size(nt)));
    const double* ratio[2] = {s.rule[0].ratio.data(), s.rule[1].ratio.data()};
    const double* coef[2] = {s.rule[0].coef.data(), s.rule[1].coef.data()};
    const double* dk[2] = {s.dh[0].data(), s.dh[1].data()};
    build_mx_tables(s.np, s.L, ratio, coef, dk, tab.data());
    BatchInst I{};
    I.mode_off = 0;
    I.M = s.M;
    I.N = s.N;
    I.np = s.np;
    I.L = s.L;
    I.scheme = s.p.scheme;
    I.d_off = 0;
    I.dstride = s.dstride;
    I.inv_tau = 1.0 / s.tau;
    I.c = s.c;
    I.a = s.a;
    I.d00 = s.dh[0][0];
    I.d01 = s.dh[1][0];
    I.mx_off = 0;
    I.nt = nt;
    MxRun& x = s.mx;
    x.tiles = (s.M + 15) / 16;
    const int list0 = 0;
    const int64_t cum[2] = {0, x.tiles};
    if ((rc = dev_alloc(s, &x.tab, tab.size()))) return rc;
    if ((rc = upload(x.tab, tab))) return rc;
    // the problem entry, the list and the tile counts in one small buffer
    const size_t ninst = (sizeof(BatchInst) + sizeof(double) - 1) / sizeof(double);
    double* small = nullptr;
    if ((rc = dev_alloc(s, &small, ninst + 3))) return rc;
    x.inst = reinterpret_cast<BatchInst*>(small);
    x.cum = reinterpret_cast<int64_t*>(small + ninst);
    x.list = reinterpret_cast<int*>(small + ninst + 2);
    HIPCHK(hipMemcpy(x.inst, &I, sizeof(BatchInst), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(x.list, &list0, sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(x.cum, cum, sizeof(cum), hipMemcpyHostToDevice));
    x.ntw = mx_template((nt + 1) / 2);
    x.on = true;
    return CQ_OK;
}

// Launch arguments of the MFMA kernel for this solver's problem.
static BatchArgs mx_args(const Solver& s) {
    BatchArgs a{};
    a.inst = s.mx.inst;
    a.list = s.mx.list;
    a.cumt = s.mx.cum;
    a.count = 1;
    a.total = s.M;
    a.tiles = s.mx.tiles;
    a.d = s.d_d;
    a.lam = s.lam;
    a.mx = s.mx.tab;
    return a;
}

int setup_device(Solver& s, const double* G0dev, hipStream_t st) {
    const cq_params* p = &s.p;
    int rc;
    const int64_t twoM = 2 * s.M;
    const bool modal = p->solver == 1;
    if ((rc = dev_alloc(s, &s.d_d, size_t(2 * s.dstride)))) return rc;
    if ((rc = dev_alloc(s, &s.G0, size_t(twoM)))) return rc;
    HIPCHK(hipMemcpyAsync(s.d_d, s.dh[0].data(), s.dstride * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(s.d_d + s.dstride, s.dh[1].data(), s.dstride * sizeof(double), hipMemcpyHostToDevice,
                          st));
    HIPCHK(hipMemcpyAsync(s.G0, G0dev, twoM * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (p->method == 1) {
        // the state pass (k_hist_block) runs whole 256-DOF workgroups: its
        // node rows are padded to a multiple of 256; the wave-per-mode
        // kernel (modal, few modes) keeps them at M
        const bool wave_per_mode = modal && !(s.M >= kModalBlockedMin && s.L <= 32);
        s.hstride = wave_per_mode ? s.M : ((s.M + 255) / 256) * 256;
        if ((rc = dev_alloc(s, &s.H, hcount(s)))) return rc;
        if ((rc = dev_alloc(s, &s.d_ratio, size_t(2 * s.np)))) return rc;
        if ((rc = dev_alloc(s, &s.d_coef, size_t(2 * s.np)))) return rc;
        HIPCHK(hipMemsetAsync(s.H, 0, hcount(s) * sizeof(double), st));
        std::vector<double> rr(size_t(2 * s.np)), cc(size_t(2 * s.np));
        for (int k = 0; k < 2; ++k)
            for (int j = 0; j < s.np; ++j) {
                rr[size_t(k * s.np + j)] = s.rule[k].ratio[size_t(j)];
                cc[size_t(k * s.np + j)] = s.rule[k].coef[size_t(j)];
            }
        if ((rc = upload(s.d_ratio, rr))) return rc;
        if ((rc = upload(s.d_coef, cc))) return rc;
    }
    if (p->method == 0) {
        if ((rc = dev_alloc(s, &s.F, size_t(int64_t(s.ks) * std::max(s.B, s.Bf) * twoM)))) return rc;
        if (modal && (rc = dev_alloc(s, &s.F2, size_t(64 * twoM)))) return rc;
    }
    if (modal) {
        if ((rc = setup_tables(s))) return rc;
        if ((rc = dev_alloc(s, &s.g0c, size_t(twoM)))) return rc;
        if ((rc = dev_alloc(s, &s.Sscratch, size_t(twoM)))) return rc;
        if (s.dim >= 2 && (rc = dev_alloc(s, &s.T1, size_t(twoM)))) return rc;
        if (p->method == 1) {
            // many modes: stream the state in time blocks (thread per mode);
            // few modes: keep each mode's state in the registers of one wave
            s.modal_blocked = s.M >= kModalBlockedMin && s.L <= 32;
            if (s.modal_blocked) {
                s.Lr = s.L;
                if ((rc = dev_alloc(s, &s.levels, size_t(s.Lr) * size_t(twoM)))) return rc;
                if ((rc = dev_alloc(s, &s.Sf, size_t(int64_t(s.BTt) * twoM)))) return rc;
            } else {
                if ((rc = dev_alloc(s, &s.ring, size_t(ring_slots(s)) * size_t(twoM)))) return rc;
            }
        } else {
            if ((rc = dev_alloc(s, &s.levels, size_t(s.Lr * twoM)))) return rc;
        }
        if ((rc = modal_start(s))) return rc;
        HIPCHK(hipStreamSynchronize(st));
        return CQ_OK;
    }
    // nodal
    if ((rc = dev_alloc(s, &s.levels, size_t(s.Lr * twoM)))) return rc;
    HIPCHK(hipMemcpyAsync(s.levels, G0dev, twoM * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (p->method == 0 && (rc = dev_alloc(s, &s.Spart, size_t(twoM)))) return rc;
    if (p->method == 1 && (rc = dev_alloc(s, &s.Sf, size_t(int64_t(s.BTt) * twoM)))) return rc;
    if (s.dim == 1) {
        s.levels_pcr = 0;
        while ((int64_t(1) << s.levels_pcr) < s.M) ++s.levels_pcr;
        const size_t nl = size_t(std::max(1, s.levels_pcr));
        if ((rc = dev_alloc(s, &s.PF, nl * size_t(twoM)))) return rc;
        if ((rc = dev_alloc(s, &s.PG, nl * size_t(twoM)))) return rc;
        if ((rc = dev_alloc(s, &s.PRB, size_t(twoM)))) return rc;
        s.lds = size_t(2) * size_t(s.M) * sizeof(double);
        int dev = 0, maxlds = 0;
        HIPCHK(hipGetDevice(&dev));
        HIPCHK(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        if (s.lds > size_t(maxlds))
            return fail(CQ_EINVAL, "1D grid of %lld nodes needs %zu B of LDS, device allows %d", (long long)s.M,
                        s.lds, maxlds);
        std::vector<double> pf, pg, prb;
        pcr_multipliers(s.M, s.levels_pcr, s.theta, s.hx, pf, pg, prb);
        if ((rc = upload(s.PF, pf))) return rc;
        if ((rc = upload(s.PG, pg))) return rc;
        if ((rc = upload(s.PRB, prb))) return rc;
    } else {
        if ((rc = dev_alloc(s, &s.rhs, size_t(twoM)))) return rc;
        if ((rc = dev_alloc(s, &s.qbuf, size_t(twoM)))) return rc;
        if ((rc = dev_alloc(s, &s.T1, size_t(twoM)))) return rc;
        if ((rc = dev_alloc(s, &s.T2, size_t(twoM)))) return rc;
        if ((rc = setup_tables(s))) return rc;
    }
    HIPCHK(hipStreamSynchronize(st));
    return CQ_OK;
}

int check_finite_g0(const double* G0dev, int64_t count, hipStream_t st, const char* what = "G0") {
    std::vector<double> h(static_cast<size_t>(count));
    HIPCHK(hipMemcpyAsync(h.data(), G0dev, size_t(count) * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (double v : h)
        if (!std::isfinite(v)) return fail(CQ_ENONFINITE, "%s holds a non-finite value", what);
    return CQ_OK;
}

void launch_far_block(Solver& s, int rows) {
    FarArgs fa{};
    fa.n0 = s.n0;
    fa.nl = s.n0;
    fa.M = s.M;
    fa.dstride = s.dstride;
    fa.lstride = 2 * s.M;
    fa.B = rows;
    fa.ks = far_ks_for(s.ks, s.n0);
    fa.ncomp = 2;
    int64_t mc = (s.n0 + fa.ks - 1) / fa.ks;
    fa.mchunk = ((mc + 3) / 4) * 4;
    fa.levels = s.levels;
    fa.d = s.d_d;
    fa.F = s.F;
    fa.reduce = 1;
    launch_far(fa, s.st);
}

// modal solver: advance by nsteps
void modal_steps(Solver& s, int64_t nsteps) {
    if (s.p.method == 1 && s.modal_blocked) {
        while (nsteps > 0) {
            // the block of the next step: steps nblk .. nblk + blen - 1
            int64_t nblk, blen;
            if (s.n < s.blk_off) {
                nblk = 1;
                blen = s.blk_off;
            } else {
                nblk = s.blk_off + ((s.n - s.blk_off) / s.Bt) * s.Bt + 1;
                blen = s.Bt;
            }
            if (s.n + 1 == nblk) {
                HistBlockArgs hb{};
                hb.n = nblk;
                hb.L = s.L;
                hb.Lr = s.Lr;
                hb.M = s.M;
                hb.np = s.np;
                hb.chunk = s.chunk;
                hb.BT = s.BTt;
                hb.bt = int(std::min<int64_t>(blen, s.N - nblk + 1));
                hb.slot0 = ((nblk - s.L) % s.Lr + s.Lr) % s.Lr;
                hb.levels = s.levels;
                hb.H = s.H;
                hb.hstride = s.hstride;
                hb.ratio = s.d_ratio;
                hb.coef = s.d_coef;
                hb.Sf = s.Sf;
                launch_hist_block(hb, s.hlanes, s.st);
            }
            const int bt = int(std::min<int64_t>(nblk + blen - 1 - s.n, nsteps));
            ModalWinArgs a{};
            a.M = s.M;
            a.nfirst = s.n + 1;
            a.nblk = nblk;
            a.bt = bt;
            a.L = s.L;
            a.Lr = s.Lr;
            a.BT = s.BTt;
            a.scheme = s.p.scheme;
            a.dstride = s.dstride;
            a.inv_tau = 1.0 / s.tau;
            a.c = s.c;
            a.a = s.a;
            a.d0[0] = s.dh[0][0];
            a.d0[1] = s.dh[1][0];
            a.lam = s.lam;
            a.d = s.d_d;
            a.g0 = s.g0c;
            a.Sf = s.Sf;
            a.levels = s.levels;
            a.Sout = s.Sout ? s.Sout : s.Sscratch;
            a.sstride = s.Sout ? 2 * s.M : 0;
            a.mu = s.mu;
            a.gc = s.gc;
            launch_modal_win(a, s.adj, s.st);
            s.n += bt;
            nsteps -= bt;
        }
        return;
    }
    if (s.p.method == 1) {
        while (nsteps > 0) {
            const int chunk = int(std::min<int64_t>(nsteps, 8192));
            ModalFastArgs a{};
            a.M = s.M;
            a.n0 = s.n;
            a.N = s.N;
            a.nsteps = chunk;
            a.np = s.np;
            a.L = s.L;
            a.scheme = s.p.scheme;
            a.dstride = s.dstride;
            a.inv_tau = 1.0 / s.tau;
            a.c = s.c;
            a.a = s.a;
            a.d0[0] = s.dh[0][0];
            a.d0[1] = s.dh[1][0];
            a.lam = s.lam;
            a.ratio = s.d_ratio;
            a.coef = s.d_coef;
            a.d = s.d_d;
            a.g0 = s.g0c;
            a.H = s.H;
            a.hstride = s.hstride;
            a.ring = s.ring;
            launch_modal_fast(a, s.st);
            s.n += chunk;
            nsteps -= chunk;
        }
        return;
    }
    const int64_t twoM = 2 * s.M;
    while (nsteps > 0) {
        const int64_t n0 = (s.n / s.B) * s.B;  // block of the next step
        const int64_t base = (n0 / s.Bf) * s.Bf;
        if (s.far_base != base) {
            // a pass over levels 1..base for the rows base+1 .. base+Bf
            s.far_base = base;
            s.n0 = base;
            if (base >= 1) launch_far_block(s, s.Bf);
        }
        if (n0 > base && s.mid_n0 != n0) {
            // the levels since the pass, base+1 .. n0, for this block
            s.mid_n0 = n0;
            FarArgs fa{};
            fa.n0 = n0;
            fa.l0 = s.far_base + 1;
            fa.nl = n0;
            fa.M = s.M;
            fa.dstride = s.dstride;
            fa.lstride = twoM;
            fa.B = s.B;
            fa.ks = 1;
            fa.ncomp = 2;
            fa.mchunk = ((n0 - s.far_base + 3) / 4) * 4;
            fa.levels = s.levels;
            fa.d = s.d_d;
            fa.F = s.F2;
            fa.reduce = 0;
            launch_far(fa, s.st);
        }
        const int bt = int(std::min<int64_t>(n0 + s.B - s.n, nsteps));
        ModalNearArgs a{};
        a.M = s.M;
        a.n0 = n0;
        a.nfirst = s.n + 1;
        a.bt = bt;
        a.scheme = s.p.scheme;
        a.dstride = s.dstride;
        a.inv_tau = 1.0 / s.tau;
        a.c = s.c;
        a.a = s.a;
        a.d0[0] = s.dh[0][0];
        a.d0[1] = s.dh[1][0];
        a.lam = s.lam;
        a.d = s.d_d;
        a.g0 = s.g0c;
        a.F = s.far_base >= 1 ? s.F + (n0 - s.far_base) * twoM : nullptr;
        a.F2 = n0 > s.far_base ? s.F2 : nullptr;
        a.levels = s.levels;
        a.Sout = s.Sout ? s.Sout : s.Sscratch;
        a.sstride = s.Sout ? 2 * s.M : 0;
        a.mu = s.mu;
        a.gc = s.gc;
        launch_modal_near(a, s.B, s.adj, s.st);
        s.n += bt;
        nsteps -= bt;
    }
}

// 3D nodal solve of one step: sine transform of w along x, y and z, the
// per-mode 2x2 solve in the z-pass's epilogue (eigenvalue lamz[r] +
// lamxy[(y, x) mode]), inverse transform, minus q.
void step_solve_3d(Solver& s, double* out) {
    const int64_t M = s.M;
    const int nx = s.nx, ny = s.ny, nz = s.nz;
    const int64_t plane = int64_t(ny) * nx;
    // along x: rows of nx values, ny*nz rows
    GemmArgs gx{};
    gx.R = ny * nz; gx.C = nx; gx.K = nx; gx.lda = nx; gx.ldb = nx; gx.ldc = nx;
    gx.A_shared = 0; gx.B_shared = 1;
    gx.B0 = s.Sx; gx.B1 = s.Sx;
    // along y: S_y times each z-plane
    GemmArgs gy{};
    gy.R = ny; gy.C = nx; gy.K = ny; gy.lda = ny; gy.ldb = nx; gy.ldc = nx;
    gy.A_shared = 1; gy.B_shared = 0;
    gy.A0 = s.Sy; gy.A1 = s.Sy;
    gy.batch = nz;
    gy.sB = gy.sC = plane;
    // along z: S_z times the nz x (ny nx) matrix
    GemmArgs gz{};
    gz.R = nz; gz.C = int(plane); gz.K = nz; gz.lda = nz; gz.ldb = int(plane); gz.ldc = int(plane);
    gz.A_shared = 1; gz.B_shared = 0;
    gz.A0 = s.Sz; gz.A1 = s.Sz;
    // forward: rhs -> T1 -> T2 -> T1 (solved coefficients)
    gx.A0 = s.rhs; gx.A1 = s.rhs + M; gx.C0 = s.T1; gx.C1 = s.T1 + M;
    launch_gemm(gx, 0, s.st);
    gy.B0 = s.T1; gy.B1 = s.T1 + M; gy.C0 = s.T2; gy.C1 = s.T2 + M;
    launch_gemm(gy, 0, s.st);
    GemmArgs gs = gz;
    gs.B0 = s.T2; gs.B1 = s.T2 + M; gs.C0 = s.T1; gs.C1 = s.T1 + M;
    gs.lamy = s.lamz; gs.lamx = s.lamxy; gs.cdiag = s.c; gs.a = s.a;
    gs.scale = 8.0 / (double(nx + 1) * double(ny + 1) * double(nz + 1));
    gs.dd0[0] = s.dh[0][0]; gs.dd0[1] = s.dh[1][0];
    launch_gemm(gs, 1, s.st);
    // inverse: T1 -> T2 -> T1 -> out - q
    gx.A0 = s.T1; gx.A1 = s.T1 + M; gx.C0 = s.T2; gx.C1 = s.T2 + M;
    launch_gemm(gx, 0, s.st);
    gy.B0 = s.T2; gy.B1 = s.T2 + M; gy.C0 = s.T1; gy.C1 = s.T1 + M;
    launch_gemm(gy, 0, s.st);
    GemmArgs gi = gz;
    gi.B0 = s.T1; gi.B1 = s.T1 + M; gi.C0 = out; gi.C1 = out + M;
    gi.sub0 = s.qbuf; gi.sub1 = s.qbuf + M;
    launch_gemm(gi, 2, s.st);
}

// one time step n = s.n + 1
void step_once(Solver& s) {
    const int64_t n = ++s.n;
    const int64_t twoM = 2 * s.M;
    StepArgs sa{};
    sa.n = n;
    sa.M = s.M;
    sa.Lr = s.Lr;
    sa.slot1 = (n - 1) % s.Lr;
    sa.slot2 = (n >= 2 ? n - 2 : 0) % s.Lr;
    sa.slot_out = n % s.Lr;
    sa.scheme = s.p.scheme;
    sa.d = s.d_d;
    sa.dstride = s.dstride;
    sa.G0 = s.G0;
    sa.levels = s.levels;
    sa.inv_tau = 1.0 / s.tau;
    sa.cdiag = s.c;
    for (int k = 0; k < 2; ++k) {
        sa.inv_d0[k] = 1.0 / s.dh[k][0];
        sa.corr[k] = s.p.scheme == 2 ? 0.5 * s.dh[k][size_t(n - 1)] : 0.0;
    }
    if (s.p.method == 0) {
        if ((n - 1) % s.B == 0) {
            s.n0 = n - 1;
            if (s.n0 >= 1) launch_far_block(s, s.B);
        }
        HistDirectArgs ha{};
        ha.n = n;
        ha.n0 = s.n0;
        ha.M = s.M;
        ha.dstride = s.dstride;
        ha.B = s.B;
        ha.ks = s.ks;
        ha.levels = s.levels;
        ha.d = s.d_d;
        ha.F = s.F;
        ha.Spart = s.Spart;
        launch_hist_direct(ha, s.st);
        sa.Sp = s.Spart;
        sa.boff = 0;
        sa.win = 0;
    } else {
        if ((n - 1) % s.Bt == 0) {
            HistBlockArgs hb{};
            hb.n = n;
            hb.L = s.L;
            hb.Lr = s.Lr;
            hb.M = s.M;
            hb.np = s.np;
            hb.chunk = s.chunk;
            hb.BT = s.BTt;
            hb.bt = int(std::min<int64_t>(s.Bt, s.N - n + 1));
            hb.slot0 = ((n - s.L) % s.Lr + s.Lr) % s.Lr;
            hb.levels = s.levels;
            hb.H = s.H;
            hb.hstride = s.hstride;
            hb.ratio = s.d_ratio;
            hb.coef = s.d_coef;
            hb.Sf = s.Sf;
            launch_hist_block(hb, s.hlanes, s.st);
        }
        sa.Sp = s.Sf;
        sa.boff = ((n - 1) % s.Bt) * twoM;
        sa.win = int(std::min<int64_t>(s.L - 1, n - 1));
    }
    if (s.dim == 1) {
        sa.h2 = s.hx * s.hx;
        for (int k = 0; k < 2; ++k) sa.delta[k] = s.theta[k] * s.hx * s.hx;
        sa.levels_pcr = s.levels_pcr;
        sa.PF = s.PF;
        sa.PG = s.PG;
        sa.PRB = s.PRB;
        sa.V[0] = s.V[0][0]; sa.V[1] = s.V[0][1]; sa.V[2] = s.V[1][0]; sa.V[3] = s.V[1][1];
        sa.Vinv[0] = s.Vinv[0][0]; sa.Vinv[1] = s.Vinv[0][1]; sa.Vinv[2] = s.Vinv[1][0]; sa.Vinv[3] = s.Vinv[1][1];
        launch_step_1d(sa, s.lds, s.st);
        return;
    }
    const int64_t M = s.M;
    sa.w = s.rhs;
    sa.q = s.qbuf;
    launch_prep_2d(sa, s.st);
    if (s.dim == 3) {
        step_solve_3d(s, s.levels + (n % s.Lr) * 2 * M);
        return;
    }
    GemmArgs ga{};
    // forward: T1 = w Sx ; T2 = solve(Sy T1)
    ga.R = s.ny; ga.C = s.nx; ga.K = s.nx; ga.lda = s.nx; ga.ldb = s.nx; ga.ldc = s.nx;
    ga.A_shared = 0; ga.B_shared = 1;
    ga.A0 = s.rhs; ga.A1 = s.rhs + M; ga.B0 = s.Sx; ga.B1 = s.Sx; ga.C0 = s.T1; ga.C1 = s.T1 + M;
    launch_gemm(ga, 0, s.st);
    GemmArgs gb{};
    gb.R = s.ny; gb.C = s.nx; gb.K = s.ny; gb.lda = s.ny; gb.ldb = s.nx; gb.ldc = s.nx;
    gb.A_shared = 1; gb.B_shared = 0;
    gb.A0 = s.Sy; gb.A1 = s.Sy; gb.B0 = s.T1; gb.B1 = s.T1 + M; gb.C0 = s.T2; gb.C1 = s.T2 + M;
    gb.lamx = s.lamx; gb.lamy = s.lamy; gb.cdiag = s.c; gb.a = s.a;
    gb.scale = 4.0 / (double(s.nx + 1) * double(s.ny + 1));
    gb.dd0[0] = s.dh[0][0]; gb.dd0[1] = s.dh[1][0];
    launch_gemm(gb, 1, s.st);
    // inverse: T1 = T2 Sx ; G^n = Sy T1 - q
    GemmArgs gc = ga;
    gc.A0 = s.T2; gc.A1 = s.T2 + M; gc.C0 = s.T1; gc.C1 = s.T1 + M;
    launch_gemm(gc, 0, s.st);
    GemmArgs gd{};
    gd.R = s.ny; gd.C = s.nx; gd.K = s.ny; gd.lda = s.ny; gd.ldb = s.nx; gd.ldc = s.nx;
    gd.A_shared = 1; gd.B_shared = 0;
    double* out = s.levels + (n % s.Lr) * 2 * M;
    gd.A0 = s.Sy; gd.A1 = s.Sy; gd.B0 = s.T1; gd.B1 = s.T1 + M; gd.C0 = out; gd.C1 = out + M;
    gd.sub0 = s.qbuf; gd.sub1 = s.qbuf + M;
    launch_gemm(gd, 2, s.st);
}

// device buffers that make up the state after step n, in order
struct Seg {
    double* p;
    size_t bytes;
};
std::vector<Seg> state_segments(const Solver& s, int64_t n) {
    const size_t twoM = size_t(2 * s.M) * sizeof(double);
    std::vector<Seg> v;
    v.push_back({s.G0, twoM});
    if (s.p.solver == 1) v.push_back({s.g0c, twoM});
    if (s.p.method == 0) {
        v.push_back({s.levels, size_t(n + 1) * twoM});
    } else {
        const size_t hb = hcount(s) * sizeof(double);
        if (s.p.solver == 1 && !s.modal_blocked) {
            v.push_back({s.H, hb});
            v.push_back({s.ring, size_t(ring_slots(s)) * twoM});
        } else {
            v.push_back({s.levels, size_t(s.Lr) * twoM});
            v.push_back({s.H, hb});
            v.push_back({s.Sf, size_t(s.BTt) * twoM});
        }
    }
    return v;
}

size_t state_bytes(const Solver& s) {
    size_t b = 4 * sizeof(uint64_t);
    for (const Seg& g : state_segments(s, s.n)) b += g.bytes;
    return b;
}

}  // namespace

// ---- kernel timing ----
namespace {
constexpr int kProfKinds = 13;
struct ProfRec {
    hipEvent_t a, b;
};
bool g_prof_on = false;
std::vector<ProfRec> g_prof_open[kProfKinds];
std::vector<ProfRec> g_prof_done[kProfKinds];
}  // namespace

namespace cqfp {
void prof_begin(int kind, hipStream_t st) {
    if (!g_prof_on) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    ProfRec r{};
    if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return;
    (void)hipEventRecord(r.a, st);
    g_prof_open[kind].push_back(r);
}
void prof_end(int kind, hipStream_t st) {
    if (!g_prof_on || g_prof_open[kind].empty()) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    ProfRec r = g_prof_open[kind].back();
    g_prof_open[kind].pop_back();
    (void)hipEventRecord(r.b, st);
    g_prof_done[kind].push_back(r);
}
}  // namespace cqfp

static void prof_clear() {
    for (int k = 0; k < kProfKinds; ++k) {
        for (auto& r : g_prof_done[k]) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        g_prof_done[k].clear();
        g_prof_open[k].clear();
    }
}

extern "C" {

int cq_prof_enable(int32_t on) {
    clear_error();
    prof_clear();
    g_prof_on = on != 0;
    return CQ_OK;
}

int cq_prof_read(int32_t kind, int64_t* launches, double* total_ms) {
    clear_error();
    if (kind < 0 || kind >= kProfKinds || !launches || !total_ms) return fail(CQ_EINVAL, "bad kind or NULL output");
    double tot = 0.0;
    for (auto& r : g_prof_done[kind]) {
        HIPCHK(hipEventSynchronize(r.b));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
        tot += ms;
    }
    *launches = int64_t(g_prof_done[kind].size());
    *total_ms = tot;
    return CQ_OK;
}

int cq_weights(int32_t scheme, double beta, double tau, int64_t n, double* d_out) {
    clear_error();
    if (scheme != 1 && scheme != 2) return fail(CQ_EINVAL, "scheme must be 1 or 2");
    if (!(beta > 0 && beta < 1)) return fail(CQ_EINVAL, "beta must lie in (0,1)");
    if (!(tau > 0) || !std::isfinite(tau)) return fail(CQ_EINVAL, "tau must be > 0");
    if (n < 0) return fail(CQ_EINVAL, "n must be >= 0");
    if (!d_out) return fail(CQ_EINVAL, "d_out is NULL");
    weights(scheme, beta, tau, n, d_out);
    return CQ_OK;
}

int cq_fast_rule(int32_t scheme, double beta, double tau, int64_t N, double tol, int32_t np, int32_t np1, int32_t ns,
                 int32_t np_max, int32_t cap, double* ratio_out, double* coef_out, int32_t* count_out,
                 int32_t* lag_out, double* max_eps_out) {
    clear_error();
    if (scheme != 1 && scheme != 2) return fail(CQ_EINVAL, "scheme must be 1 or 2");
    if (!(beta > 0 && beta < 1)) return fail(CQ_EINVAL, "beta must lie in (0,1)");
    if (!(tau > 0)) return fail(CQ_EINVAL, "tau must be > 0");
    if (N < 1) return fail(CQ_EINVAL, "N must be >= 1");
    if (np < 0 || np1 < 0 || ns < 0 || np_max < 0 || cap < 0 || tol < 0)
        return fail(CQ_EINVAL, "negative count or tolerance");
    if (scheme == 2 && ns != 0 && ns < 3) return fail(CQ_EINVAL, "ns must be >= 3");
    if (!ratio_out || !coef_out || !count_out || !lag_out || !max_eps_out)
        return fail(CQ_EINVAL, "output pointer is NULL");
    if (np > 4096 || np1 > 4096) return fail(CQ_EINVAL, "np, np1 must be <= 4096");
    const int ns_ = ns ? ns : 30, np1_ = np1 ? np1 : 16, npmax = np_max ? np_max : 1024;
    const double tol_ = tol > 0 ? tol : 1e-8;
    FastRule r;
    try {
        if (np > 0) {
            build_rule(scheme, beta, tau, np, np1_, ns_, r);
            std::vector<double> d(size_t(N) + 1);
            weights(scheme, beta, tau, N, d.data());
            r.max_eps = rule_error(r, d, N);
        } else {
            int rc = choose_rule(scheme, beta, tau, N, tol_, npmax, np1_, ns_, r);
            if (rc != CQ_OK) return rc;
        }
    } catch (const std::bad_alloc&) {
        return fail(CQ_ENOMEM, "host allocation failed");
    }
    if (int(r.ratio.size()) > cap) return fail(CQ_EINVAL, "cap %d < %zu terms", cap, r.ratio.size());
    for (size_t j = 0; j < r.ratio.size(); ++j) {
        ratio_out[j] = r.ratio[j];
        coef_out[j] = r.coef[j];
    }
    *count_out = int32_t(r.ratio.size());
    *lag_out = r.lag;
    *max_eps_out = r.max_eps;
    return CQ_OK;
}

int cq_history(int32_t scheme, double beta, double tau, const double* G_hist, int64_t n, int64_t M, double* S_out,
               void* hip_stream) {
    clear_error();
    if (scheme != 1 && scheme != 2) return fail(CQ_EINVAL, "scheme must be 1 or 2");
    if (!(beta > 0 && beta < 1)) return fail(CQ_EINVAL, "beta must lie in (0,1)");
    if (!(tau > 0)) return fail(CQ_EINVAL, "tau must be > 0");
    if (n < 1 || M < 1) return fail(CQ_EINVAL, "n and M must be >= 1");
    if (!G_hist || !S_out) return fail(CQ_EINVAL, "NULL array");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const int ks = hist_row_slices(n, M, -1);
    std::vector<double> dh(static_cast<size_t>(n));  // d_0 .. d_{n-1}
    weights(scheme, beta, tau, n - 1, dh.data());
    // workspace of this call: the weights and the slices' partial sums
    const size_t nd = size_t(n), npart = ks > 1 ? size_t(ks) * size_t(M) : 0;
    double* ws = nullptr;
    hipError_t e = hipMalloc(&ws, (nd + npart) * sizeof(double));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? CQ_ENOMEM : CQ_EHIP, "hipMalloc for the history workspace: %s",
                    hipGetErrorString(e));
    }
    int rc = CQ_OK;
    do {
        e = hipMemcpyAsync(ws, dh.data(), nd * sizeof(double), hipMemcpyHostToDevice, st);
        if (e != hipSuccess) { rc = fail(CQ_EHIP, "copy weights: %s", hipGetErrorString(e)); break; }
        launch_hist_row(G_hist, n, M, ws, ks, ws + nd, S_out, st);
        e = hipGetLastError();
        if (e != hipSuccess) { rc = fail(CQ_EHIP, "launch: %s", hipGetErrorString(e)); break; }
        e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = fail(CQ_EHIP, "sync: %s", hipGetErrorString(e));
    } while (0);
    (void)hipFree(ws);
    return rc;
}

int fp_create(const cq_grid* grid, const cq_params* prm, const double* G0, void* hip_stream, void** handle) {
    clear_error();
    if (!handle) return fail(CQ_EINVAL, "handle is NULL");
    *handle = nullptr;
    int rc = validate(grid, prm);
    if (rc) return rc;
    if (!G0) return fail(CQ_EINVAL, "G0 is NULL");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const int64_t M = int64_t(grid->nx) * (grid->dim >= 2 ? grid->ny : 1) * (grid->dim == 3 ? grid->nz : 1);
    Solver* s = new (std::nothrow) Solver();
    if (!s) return fail(CQ_ENOMEM, "host allocation failed");
    try {
        // host checks (operator definiteness, fast-rule tolerance) come first,
        // so they are reported without touching the device
        rc = setup_host(*s, grid, prm, st);
        if (!rc) rc = check_finite_g0(G0, 2 * M, st);
        if (!rc) rc = setup_device(*s, G0, st);
        if (!rc && prm->solver == 1 && prm->method == 1 && prm->fast_kernel == 1 && mx_applies(s->L, s->np))
            rc = setup_mx(*s);
    } catch (const std::bad_alloc&) {
        rc = fail(CQ_ENOMEM, "host allocation failed");
    }
    if (rc) {
        delete s;
        return rc;
    }
    *handle = s;
    return CQ_OK;
}

int fp_step(void* handle, int64_t nsteps) {
    clear_error();
    if (!handle) return fail(CQ_EINVAL, "handle is NULL");
    Solver& s = *static_cast<Solver*>(handle);
    if (s.kind != 0) return fail(CQ_EINVAL, "not a stepping solver handle (use fp_adjoint_run)");
    if (nsteps < 0 || s.n + nsteps > s.N)
        return fail(CQ_EINVAL, "cannot take %lld steps from n = %lld (N = %lld)", (long long)nsteps, (long long)s.n,
                    (long long)s.N);
    if (s.p.solver == 1 && s.mx.on && s.n == 0 && nsteps == s.N && nsteps > 0) {
        // the whole run in one launch of the 16-mode MFMA kernel (fast_kernel
        // 1): only the final level is kept, where fp_current reads it
        BatchArgs a = mx_args(s);
        a.g0 = s.g0c;
        a.gN = s.modal_blocked ? s.levels + (s.N % s.Lr) * 2 * s.M : s.ring;
        if (launch_modal_batch_mx(a, s.mx.ntw, s.st))
            return fail(CQ_EINVAL, "no template for %d node tiles per wave", s.mx.ntw);
        s.n = s.N;
    } else if (s.p.solver == 1) {
        modal_steps(s, nsteps);
    } else {
        for (int64_t i = 0; i < nsteps; ++i) step_once(s);
    }
    HIPCHK(hipGetLastError());
    return CQ_OK;
}

int fp_current(void* handle, double* G_out, int64_t* n_out) {
    clear_error();
    if (!handle || !G_out) return fail(CQ_EINVAL, "NULL argument");
    Solver& s = *static_cast<Solver*>(handle);
    if (s.kind != 0) return fail(CQ_EINVAL, "not a stepping solver handle (use fp_adjoint_run)");
    if (s.p.solver == 1) {
        const double* c = s.p.method == 1 ? (s.modal_blocked ? s.levels + (s.n % s.Lr) * 2 * s.M : s.ring)
                                           : s.levels + s.n * 2 * s.M;
        transform(s, c, G_out, false);
        HIPCHK(hipGetLastError());
        if (n_out) *n_out = s.n;
        return CQ_OK;
    }
    const double* src = s.levels + (s.n % s.Lr) * 2 * s.M;
    HIPCHK(hipMemcpyAsync(G_out, src, size_t(2 * s.M) * sizeof(double), hipMemcpyDeviceToDevice, s.st));
    if (n_out) *n_out = s.n;
    return CQ_OK;
}

int fp_info(void* handle, cq_info* info) {
    clear_error();
    if (!handle || !info) return fail(CQ_EINVAL, "NULL argument");
    const Solver& s = *static_cast<const Solver*>(handle);
    if (s.kind != 0) return fail(CQ_EINVAL, "not a stepping solver handle (use fp_adjoint_run)");
    info->n = s.n;
    info->N = s.N;
    info->np_total = s.np;
    info->lag = s.p.method == 1 ? s.L : 0;
    info->max_eps = s.max_eps;
    info->theta[0] = s.theta[0];
    info->theta[1] = s.theta[1];
    info->block_B = s.p.method == 1 ? s.Bt : (s.p.solver == 1 ? s.Bf : s.B);
    info->ksplit = s.ks;
    info->device_bytes = s.dev_bytes;
    info->state_bytes = state_bytes(s);
    info->np1 = (s.p.method == 1 && s.p.scheme == 2) ? s.np1_used : 0;
    info->whole_run_kernel = s.mx.on ? 1 : 0;
    return CQ_OK;
}

int fp_get_state(void* handle, void* dst, size_t* bytes) {
    clear_error();
    if (!handle || !bytes) return fail(CQ_EINVAL, "NULL argument");
    Solver& s = *static_cast<Solver*>(handle);
    if (s.kind != 0) return fail(CQ_EINVAL, "not a stepping solver handle (use fp_adjoint_run)");
    const size_t need = state_bytes(s);
    if (!dst) {
        *bytes = need;
        return CQ_OK;
    }
    if (*bytes < need) return fail(CQ_EINVAL, "state buffer of %zu bytes < %zu", *bytes, need);
    HIPCHK(hipStreamSynchronize(s.st));
    uint64_t* hdr = static_cast<uint64_t*>(dst);
    hdr[0] = kStateMagic;
    hdr[1] = uint64_t(s.n);
    hdr[2] = uint64_t(s.M);
    hdr[3] = uint64_t(s.np);
    char* q = static_cast<char*>(dst) + 4 * sizeof(uint64_t);
    for (const Seg& g : state_segments(s, s.n)) {
        HIPCHK(hipMemcpy(q, g.p, g.bytes, hipMemcpyDeviceToHost));
        q += g.bytes;
    }
    *bytes = need;
    return CQ_OK;
}

int fp_set_state(void* handle, const void* src, size_t bytes) {
    clear_error();
    if (!handle || !src) return fail(CQ_EINVAL, "NULL argument");
    Solver& s = *static_cast<Solver*>(handle);
    if (s.kind != 0) return fail(CQ_EINVAL, "not a stepping solver handle (use fp_adjoint_run)");
    if (bytes < 4 * sizeof(uint64_t)) return fail(CQ_EINVAL, "state too short");
    const uint64_t* hdr = static_cast<const uint64_t*>(src);
    if (hdr[0] != kStateMagic || hdr[2] != uint64_t(s.M) || hdr[3] != uint64_t(s.np))
        return fail(CQ_EINVAL, "state does not belong to a solver of this shape");
    const int64_t n = int64_t(hdr[1]);
    if (n < 0 || n > s.N) return fail(CQ_EINVAL, "state step %lld out of range", (long long)n);
    const int64_t save_n = s.n;
    s.n = n;
    const size_t need = state_bytes(s);
    if (bytes < need) {
        s.n = save_n;
        return fail(CQ_EINVAL, "state of %zu bytes < %zu", bytes, need);
    }
    HIPCHK(hipStreamSynchronize(s.st));
    const char* q = static_cast<const char*>(src) + 4 * sizeof(uint64_t);
    for (const Seg& g : state_segments(s, n)) {
        HIPCHK(hipMemcpy(g.p, q, g.bytes, hipMemcpyHostToDevice));
        q += g.bytes;
    }
    if (s.p.method == 0) {  // far field of the block that contains step n+1
        s.n0 = (n / s.B) * s.B;
        s.far_base = -1;  // modal: the next step recomputes its block's far field
        s.mid_n0 = -1;
        if (s.p.solver == 0 && n % s.B != 0 && s.n0 >= 1) launch_far_block(s, s.B);
    }
    HIPCHK(hipGetLastError());
    return CQ_OK;
}

int fp_reset(void* handle, const double* G0) {
    clear_error();
    if (!handle || !G0) return fail(CQ_EINVAL, "NULL argument");
    Solver& s = *static_cast<Solver*>(handle);
    if (s.kind != 0) return fail(CQ_EINVAL, "not a stepping solver handle (use fp_adjoint_run)");
    const int64_t twoM = 2 * s.M;
    int rc = check_finite_g0(G0, twoM, s.st);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(s.G0, G0, size_t(twoM) * sizeof(double), hipMemcpyDeviceToDevice, s.st));
    s.n = 0;
    s.far_base = -1;
    s.mid_n0 = -1;
    s.n0 = 0;
    if (s.p.solver == 1) return modal_start(s);
    HIPCHK(hipMemcpyAsync(s.levels, G0, size_t(twoM) * sizeof(double), hipMemcpyDeviceToDevice, s.st));
    if (s.H) HIPCHK(hipMemsetAsync(s.H, 0, hcount(s) * sizeof(double), s.st));
    return CQ_OK;
}

int fp_destroy(void* handle) {
    clear_error();
    if (!handle) return CQ_OK;
    Solver* s = static_cast<Solver*>(handle);
    (void)hipStreamSynchronize(s->st);
    delete s;
    return CQ_OK;
}

int fp_solve(const cq_grid* grid, const cq_params* prm, const double* G0, double* GN, void* hip_stream) {
    void* h = nullptr;
    int rc = fp_create(grid, prm, G0, hip_stream, &h);
    if (rc) return rc;
    if (!GN) {
        fp_destroy(h);
        return fail(CQ_EINVAL, "GN is NULL");
    }
    rc = fp_step(h, prm->N);
    if (!rc) rc = fp_current(h, GN, nullptr);
    if (!rc) {
        hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(hip_stream));
        if (e != hipSuccess) rc = fail(CQ_EHIP, "sync: %s", hipGetErrorString(e));
    }
    fp_destroy(h);
    return rc;
}

// Gradient of a loss of G^N (forward solve, adjoint sweep in reversed time
// with the same kernels, gradient passes). Two forms: the whole forward
// trajectory, its history sums and the adjoint kept in HBM, or (fast method)
// checkpointed: the forward recomputed segment by segment from saved states
// on a binomial schedule.

// chunk length of the time-chunked gradient reductions: for the fast form a
// multiple of its state block, so that segments of whole chunks start where
// the forward can be resumed
static int64_t adj_chunk_len(const Solver& s) {
    const int64_t base = (s.N + 63) / 64;
    if (s.p.method != 1) return base;
    return ((base + s.Bt - 1) / s.Bt) * s.Bt;
}

// Binomial (revolve) schedule over n segments: with the state at the first
// segment saved and c more states that can be saved, T(n, c) is the fewest
// segment advances of the forward that reverse all n segments:
//   T(1, c) = 0,  T(n, 0) = n (n - 1) / 2  (advance from the start to each),
//   T(n, c) = min_{1 <= m < n} m + T(n - m, c - 1) + T(m, c)
// (advance m segments and save, reverse the last n - m with one state fewer,
// then the first m). split[n][c] holds an optimal m.
static void plan_schedule(int nseg, int slots, std::vector<int64_t>& T, std::vector<int>& split) {
    const int C = std::max(1, slots);  // c = 0 .. C-1 free states
    T.assign(size_t(nseg + 1) * size_t(C), 0);
    split.assign(size_t(nseg + 1) * size_t(C), 0);
    for (int n = 2; n <= nseg; ++n)
        for (int c = 0; c < C; ++c) {
            int64_t best = int64_t(n) * (n - 1) / 2;
            int bm = 0;
            if (c > 0)
                for (int m = 1; m < n; ++m) {
                    const int64_t v = m + T[size_t(n - m) * C + (c - 1)] + T[size_t(m) * C + c];
                    if (v < best) {
                        best = v;
                        bm = m;
                    }
                }
            T[size_t(n) * C + c] = best;
            split[size_t(n) * C + c] = bm;
        }
}

// bytes of the arrays every gradient handle holds (besides the forward /
// adjoint storage of its form)
static size_t adj_common_bytes(const Solver& s, size_t frows) {
    const size_t twoM = size_t(2 * s.M);
    size_t v = 2 * size_t(s.dstride) + 10 * twoM + frows + 64 * twoM + 2 * (size_t(s.dstride) + kDwPad) +
               2 * size_t(s.dstride) + size_t(s.nx) * s.nx + size_t(s.ny) * s.ny + size_t(s.nz) * s.nz +
               size_t(s.M) + size_t(s.nx + s.ny + s.nz) + 8192;
    if (s.p.method == 1) v += 2 * size_t(s.np) * size_t(((s.M + 255) / 256) * 256) + 4 * size_t(s.np) +
                              size_t(s.BTt) * twoM;
    return v * sizeof(double);
}

static int adjoint_setup(Solver& s, const cq_adjoint_opts* opt) {
    int rc;
    const cq_params* p = &s.p;
    const int64_t M = s.M, N = s.N, twoM = 2 * M;
    const size_t lev = size_t(N + 1) * size_t(twoM);
    hipStream_t st = s.st;
    const int mode = opt ? opt->mode : 0;
    if (mode < 0 || mode > 2) return fail(CQ_EINVAL, "adjoint mode must be 0, 1 or 2 (got %d)", mode);
    if (opt && (opt->segment_steps < 0 || opt->slots < 0)) return fail(CQ_EINVAL, "negative segment or slot count");
    const int fwdk = opt ? opt->forward_kernel : 0;
    if (fwdk < 0 || fwdk > 2) return fail(CQ_EINVAL, "forward_kernel must be 0, 1 or 2 (got %d)", fwdk);
    if (mode == 2 && p->method != 1)
        return fail(CQ_EINVAL, "the checkpointed adjoint needs the fast method (the direct form's state at a step "
                               "is its whole history)");
    if (p->method == 1 && s.L > 32)
        return fail(CQ_EINVAL, "the adjoint's fast form needs a window of <= 32 levels (ns = %d)", s.L);
    // the far field of the d/dbeta pass (and of the direct history): blocks of
    // 64, direct history passes of Bf rows
    s.B = 64;
    s.Bf = p->block_B ? p->block_B : modal_far_pass(M);
    s.ks = far_ksplit(M);
    AdjBufs& A = s.ab;
    A.per = adj_chunk_len(s);
    A.nchunk = int((N + A.per - 1) / A.per);
    // d/dbeta: blocks of Bk steps while their P-point transforms fit in LDS
    // (N <= 4096), unless CQFP_BETA_TOEPLITZ is set; else Toeplitz passes
    // over all levels. The exact near field costs about N Bk per mode, the
    // block pairs N^2 / Bk: Bk is the power of two nearest 2.25 sqrt(N)
    // (8..256), the balance measured at N = 4096 (Bk 64, 128, 256)
    const char* force_toeplitz = std::getenv("CQFP_BETA_TOEPLITZ");
    int spec_bk = 0, spec_nb = 0, spec_log = 0;
    {
        const int lb = int(std::min<long>(8, std::max<long>(3, std::lround(std::log2(2.25 * std::sqrt(double(N)))))));
        const int Bk = 1 << lb;
        const int64_t nb = (N + Bk - 1) / Bk;
        const int64_t items = (nb - 2 + kSpecSD - 1) / kSpecSD * (Bk + 1);  // k_beta_spec's thread items
        if (nb * 2 * Bk <= kSpecMaxLds && items <= kSpecItems &&
            !(force_toeplitz && force_toeplitz[0] && force_toeplitz[0] != '0')) {
            spec_bk = Bk;
            spec_log = lb + 1;
            spec_nb = int(nb);
        }
    }
    const size_t frows = size_t(s.ks) * size_t(std::max({s.B, s.Bf, spec_bk})) * size_t(twoM);
    if (p->method == 1) s.hstride = ((M + 255) / 256) * 256;  // the state pass runs whole 256-DOF workgroups
    size_t budget = opt ? opt->max_device_bytes : 0;
    {
        size_t fr = 0, tot = 0;
        HIPCHK(hipMemGetInfo(&fr, &tot));
        const size_t margin = std::min<size_t>(size_t(1) << 30, fr / 50);
        const size_t avail = fr > margin ? fr - margin : 0;
        if (budget == 0 || budget > avail) budget = avail;
    }
    const size_t common = adj_common_bytes(s, frows);
    const size_t storeall = common + 4 * lev * sizeof(double);
    if (mode == 1 || (mode == 0 && (p->method != 1 || storeall <= budget))) {
        if (storeall > budget)
            return fail(CQ_ENOMEM, "the adjoint keeping its whole trajectory needs %zu bytes (4 x (N+1) x 2M values "
                                   "and work arrays); the budget is %zu", storeall, budget);
        A.ckpt = false;
    } else {
        // checkpointed: psi whole, a segment's levels, history sums and mu,
        // the adjoint's own state, a level ring for advancing, saved states
        A.ckpt = true;
        const size_t hc = hcount(s);
        A.ck_stride = int64_t(hc) + int64_t(s.L) * twoM;
        const size_t fixed = common + (lev + hc + size_t(s.BTt) * twoM + size_t(s.L) * twoM) * sizeof(double);
        const int64_t unit = A.per;  // a segment is whole chunks (a multiple of the state block)
        const int64_t want_seg = opt && opt->segment_steps > 0 ? opt->segment_steps : 0;
        const int want_slots = opt ? opt->slots : 0;
        int64_t best_cost = -1;
        size_t best_bytes = 0;
        std::vector<int64_t> T;
        std::vector<int> sp;
        for (int64_t j = 1; j * unit < N + unit; ++j) {
            const int64_t seg = std::min<int64_t>(j * unit, ((N + unit - 1) / unit) * unit);
            if (want_seg && seg != ((want_seg + unit - 1) / unit) * unit) continue;
            const int nseg = int((N + seg - 1) / seg);
            if (nseg > 256) continue;
            const size_t segb = size_t(3 * seg + s.L + 2) * size_t(twoM) * sizeof(double);
            if (fixed + segb + size_t(A.ck_stride) * sizeof(double) > budget) continue;
            const int64_t cmax = int64_t((budget - fixed - segb) / (size_t(A.ck_stride) * sizeof(double)));
            int slots = int(std::min<int64_t>(cmax, nseg));
            if (want_slots > 0) {
                if (want_slots > slots) continue;
                slots = want_slots;
            }
            plan_schedule(nseg, slots, T, sp);
            const int64_t cost = N + seg * T[size_t(nseg) * size_t(slots) + size_t(slots - 1)];
            const size_t bytes = fixed + segb + size_t(slots) * size_t(A.ck_stride) * sizeof(double);
            if (best_cost < 0 || cost < best_cost || (cost == best_cost && bytes < best_bytes)) {
                best_cost = cost;
                best_bytes = bytes;
                A.seg = seg;
                A.nseg = nseg;
                A.slots = slots;
                A.split = sp;
                A.cost = T;
            }
        }
        if (best_cost < 0)
            return fail(CQ_ENOMEM, "no checkpoint schedule fits the budget of %zu bytes (the adjoint keeps "
                                   "(N+1) x 2M values of psi and at least one saved state)", budget);
        A.fwd_steps = best_cost;
        spec_bk = 0;  // the d/dbeta contraction runs as Toeplitz products, segment by segment
        spec_nb = 0;
    }
    A.spec_bk = spec_bk;
    A.specP = 2 * spec_bk;
    A.specLog = spec_log;
    A.spec_nb = spec_nb;
    if ((rc = dev_alloc(s, &s.d_d, size_t(2 * s.dstride)))) return rc;
    if ((rc = dev_alloc(s, &s.G0, size_t(twoM)))) return rc;
    if ((rc = dev_alloc(s, &s.g0c, size_t(twoM)))) return rc;
    if ((rc = dev_alloc(s, &s.Sscratch, size_t(twoM)))) return rc;
    if (s.dim >= 2 && (rc = dev_alloc(s, &s.T1, size_t(twoM)))) return rc;
    if ((rc = setup_tables(s))) return rc;
    if ((rc = dev_alloc(s, &A.psi, lev))) return rc;
    if (!A.ckpt) {
        if ((rc = dev_alloc(s, &A.traj, lev))) return rc;
        if ((rc = dev_alloc(s, &A.Sx, lev))) return rc;
        if ((rc = dev_alloc(s, &A.mu, lev))) return rc;
    }
    if ((rc = dev_alloc(s, &s.F, frows))) return rc;
    if ((rc = dev_alloc(s, &s.F2, size_t(64) * size_t(twoM)))) return rc;
    if ((rc = dev_alloc(s, &A.gc, size_t(twoM)))) return rc;
    if ((rc = dev_alloc(s, &A.gG0c, size_t(twoM)))) return rc;
    if ((rc = dev_alloc(s, &A.acc, size_t(twoM)))) return rc;
    if ((rc = dev_alloc(s, &A.dw, size_t(2 * (s.dstride + kDwPad))))) return rc;
    if ((rc = dev_alloc(s, &A.dd, size_t(2 * s.dstride)))) return rc;
    A.nblk_da = int((M + 255) / 256) * A.nchunk;
    A.nblk_rows = int((M + 4095) / 4096);
    if ((rc = dev_alloc(s, &A.part, size_t(A.nblk_da)))) return rc;
    if ((rc = dev_alloc(s, &A.part2, size_t(2 * A.nblk_rows)))) return rc;
    HIPCHK(hipMemcpyAsync(s.d_d, s.dh[0].data(), s.dstride * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(s.d_d + s.dstride, s.dh[1].data(), s.dstride * sizeof(double), hipMemcpyHostToDevice,
                          st));
    if (p->method == 1) {
        if ((rc = dev_alloc(s, &s.H, hcount(s)))) return rc;
        if ((rc = dev_alloc(s, &s.d_ratio, size_t(2 * s.np)))) return rc;
        if ((rc = dev_alloc(s, &s.d_coef, size_t(2 * s.np)))) return rc;
        if ((rc = dev_alloc(s, &s.Sf, size_t(int64_t(s.BTt) * twoM)))) return rc;
        std::vector<double> rr(size_t(2 * s.np)), cc(size_t(2 * s.np));
        for (int k = 0; k < 2; ++k)
            for (int j = 0; j < s.np; ++j) {
                rr[size_t(k * s.np + j)] = s.rule[k].ratio[size_t(j)];
                cc[size_t(k * s.np + j)] = s.rule[k].coef[size_t(j)];
            }
        if ((rc = upload(s.d_ratio, rr))) return rc;
        if ((rc = upload(s.d_coef, cc))) return rc;
        s.modal_blocked = true;  // thread per mode, level store of all N+1 levels
        A.Hf = s.H;
        A.Sff = s.Sf;
        // the kept-whole sweeps on the 16-mode MFMA kernel (<= 16 node tiles
        // per wave: its per-step output variants keep two waves per SIMD there)
        const int nt = (s.np + 15) / 16;
        // automatic from kModalBlockedMin modes (fewer give the kernel too few
        // workgroups to beat the streamed sweeps); forward_kernel 2 always
        if (!A.ckpt && (fwdk == 2 || (fwdk == 0 && M >= kModalBlockedMin)) && mx_applies(s.L, s.np) && nt <= 32) {
            if ((rc = setup_mx(s))) return rc;
            A.mxfwd = true;
            const size_t colb = 2 * size_t(N) * size_t(twoM) * sizeof(double);
            if (A.spec_nb > 2 && s.mx.ntw < kMxColsNtw && storeall + colb <= budget) {
                if ((rc = dev_alloc(s, &A.colG, size_t(N) * size_t(twoM)))) return rc;
                if ((rc = dev_alloc(s, &A.colPsi, size_t(N) * size_t(twoM)))) return rc;
            }
        }
        if (A.ckpt) {
            if ((rc = dev_alloc(s, &A.Ha, hcount(s)))) return rc;
            if ((rc = dev_alloc(s, &A.Sfa, size_t(int64_t(s.BTt) * twoM)))) return rc;
            if ((rc = dev_alloc(s, &A.ringA, size_t(s.L) * size_t(twoM)))) return rc;
            if ((rc = dev_alloc(s, &A.segLev, size_t(A.seg + s.L) * size_t(twoM)))) return rc;
            if ((rc = dev_alloc(s, &A.segS, size_t(A.seg) * size_t(twoM)))) return rc;
            if ((rc = dev_alloc(s, &A.segMu, size_t(A.seg + 2) * size_t(twoM)))) return rc;
            if ((rc = dev_alloc(s, &A.ck, size_t(A.slots) * size_t(A.ck_stride)))) return rc;
        }
    }
    // weight derivatives: exact (recurrences differentiated); the fast
    // scheme's beyond its lag from the rule
    // dw rows: kDwPad zeros (negative lags), then the derivatives
    std::vector<double> hdw(size_t(2 * (s.dstride + kDwPad)), 0.0), hdd(size_t(2 * s.dstride));
    for (int k = 0; k < 2; ++k) {
        double* ddk = hdd.data() + size_t(k) * size_t(s.dstride);
        double* dwk = hdw.data() + size_t(k) * size_t(s.dstride + kDwPad) + kDwPad;
        weights_dbeta(p->scheme, s.beta[k], s.tau, s.dstride - 1, ddk);
        std::copy(ddk, ddk + s.dstride, dwk);
        if (p->method == 1) {
            const int np1 = p->scheme == 2 ? s.np1_used : 0;
            rule_weights_dbeta(p->scheme, s.beta[k], s.tau, s.np - np1, np1, s.ns_used, s.L, N, 1e-3, dwk);
        }
    }
    if ((rc = upload(A.dw, hdw))) return rc;
    if ((rc = upload(A.dd, hdd))) return rc;
    if (A.spec_nb > 2) {
        const int Bk = A.spec_bk, P = A.specP, nb = A.spec_nb;
        const int Q = (nb - 2) * (Bk + 1);
        const int64_t nwg = std::min<int64_t>(128, M);  // 2 x 128 workgroups: one per CU
        A.spec_cols = int((M + nwg - 1) / nwg);
        A.spec_nwg = int((M + A.spec_cols - 1) / A.spec_cols);
        A.nblk_dot = (Q + 63) / 64;
        std::vector<double> htw(static_cast<size_t>(P));
        for (int j = 0; j < Bk; ++j) {
            const double ang = 2.0 * std::acos(-1.0) * double(j) / double(P);
            htw[size_t(2 * j)] = std::cos(ang);
            htw[size_t(2 * j + 1)] = -std::sin(ang);
        }
        if ((rc = dev_alloc(s, &A.tw, size_t(P)))) return rc;
        if ((rc = upload(A.tw, htw))) return rc;
        if ((rc = dev_alloc(s, &A.W, size_t(4) * size_t(nb) * size_t(Bk + 1)))) return rc;
        if ((rc = dev_alloc(s, &A.spec, size_t(4) * size_t(A.spec_nwg) * size_t(Q)))) return rc;
        if ((rc = dev_alloc(s, &A.bpart, size_t(2 * A.nblk_dot)))) return rc;
        launch_fft_w(A.dw + kDwPad, s.dstride + kDwPad, N, nb, P, A.specLog, A.tw, A.W, st);
        HIPCHK(hipGetLastError());
    }
    if (!A.ckpt) A.fwd_steps = N;
    HIPCHK(hipStreamSynchronize(st));
    s.kind = 1;
    return CQ_OK;
}

// fields of the solver that one sweep of modal_steps uses
struct Sweep {
    double *levels, *H, *Sf, *Sout, *mu;
    const double* gc;
    int64_t Lr, n;
    bool adj;
    int64_t blk_off;
};
static void set_sweep(Solver& s, const Sweep& w) {
    s.levels = w.levels;
    s.H = w.H;
    s.Sf = w.Sf;
    s.Sout = w.Sout;
    s.mu = w.mu;
    s.gc = w.gc;
    s.Lr = w.Lr;
    s.n = w.n;
    s.adj = w.adj;
    s.blk_off = w.blk_off;
    s.far_base = -1;
    s.mid_n0 = -1;
    s.n0 = 0;
}

// one row block of the d/dbeta contraction: rows n0+1 .. n0+bt against the
// levels l0..nl (at levels[l * 2M]), contracted with psi into acc
static void beta_rows(Solver& s, const double* levels, int64_t n0, int bt, int rows, int64_t l0, int64_t nl,
                      bool g0term) {
    AdjBufs& A = s.ab;
    const int64_t M = s.M, twoM = 2 * M;
    FarArgs fa{};
    fa.n0 = n0;
    fa.l0 = l0;
    fa.nl = nl;
    fa.M = M;
    fa.dstride = s.dstride + kDwPad;
    fa.lstride = twoM;
    fa.B = rows;
    const int64_t nlev = nl - l0 + 1;
    fa.ks = far_ks_for(s.ks, nlev);
    fa.ncomp = 2;
    const int64_t mc = (nlev + fa.ks - 1) / fa.ks;
    fa.mchunk = ((mc + 3) / 4) * 4;
    fa.levels = levels;
    fa.d = A.dw + kDwPad;
    fa.F = s.F;
    fa.reduce = 1;
    launch_far(fa, s.st);
    AdjBetaArgs ab{};
    ab.M = M;
    ab.N = s.N;
    ab.n0 = n0;
    ab.bt = bt;
    ab.scheme = s.p.scheme;
    ab.dstride = s.dstride;
    ab.dd = A.dd;
    ab.F = s.F;
    ab.g0 = s.g0c;
    ab.g0term = g0term ? 1 : 0;
    ab.psi = A.psi;
    ab.acc = A.acc;
    launch_adj_beta(ab, s.st);
}

static AdjGradArgs grad_args(Solver& s, const double* traj, const double* Sx, const double* mu) {
    AdjBufs& A = s.ab;
    AdjGradArgs ga{};
    ga.M = s.M;
    ga.N = s.N;
    ga.scheme = s.p.scheme;
    ga.dstride = s.dstride;
    ga.inv_tau = 1.0 / s.tau;
    ga.d0[0] = s.dh[0][0];
    ga.d0[1] = s.dh[1][0];
    ga.d = s.d_d;
    ga.traj = traj;
    ga.Sx = Sx;
    ga.mu = mu;
    ga.psi = A.psi;
    ga.gG0c = A.gG0c;
    ga.part = A.part;
    ga.gpart = s.F;  // free outside the d/dbeta passes: ks*64 >= nchunk rows of 2M
    ga.nchunk = A.nchunk;
    ga.per = A.per;
    return ga;
}

// the scalar gradients from the partial sums on the device
static int adjoint_finish(Solver& s, double* grad) {
    AdjBufs& A = s.ab;
    const cq_params* p = &s.p;
    hipStream_t st = s.st;
    std::vector<double> hp(static_cast<size_t>(A.nblk_da)), hp2(static_cast<size_t>(2 * A.nblk_rows)),
        hb(static_cast<size_t>(2 * A.nblk_dot));
    HIPCHK(hipMemcpyAsync(hp.data(), A.part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hp2.data(), A.part2, hp2.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    if (A.spec_nb > 2)
        HIPCHK(hipMemcpyAsync(hb.data(), A.bpart, hb.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double sa = 0.0, sb0 = 0.0, sb1 = 0.0;
    for (double v : hp) sa += v;
    for (int i = 0; i < A.nblk_rows; ++i) {
        sb0 += hp2[size_t(i)];
        sb1 += hp2[size_t(A.nblk_rows + i)];
    }
    for (int i = 0; i < A.nblk_dot; ++i) {
        sb0 += hb[size_t(i)];
        sb1 += hb[size_t(A.nblk_dot + i)];
    }
    const double da_dm = -1.0 / ((2.0 * p->m - 1.0) * (2.0 * p->m - 1.0));
    grad[0] = sb0;            // dl/dalpha_1 = -dl/dbeta_1
    grad[1] = sb1;
    grad[2] = -sa * da_dm;    // dl/dm = dl/da da/dm, dl/da = -sum
    return CQ_OK;
}

// checkpointed gradient: see AdjBufs
static int adjoint_exec_ckpt(Solver& s, const double* gN, double* gG0, double* grad, double* GN) {
    AdjBufs& A = s.ab;
    const int64_t M = s.M, N = s.N, twoM = 2 * M, L = s.L, seg = A.seg;
    const size_t hc = hcount(s);
    const size_t row = size_t(twoM) * sizeof(double);
    hipStream_t st = s.st;
    double* const Hf = A.Hf;
    double* const Sff = A.Sff;
    int64_t adj_n = 0;  // reversed steps the adjoint has taken
    auto seg_a = [&](int k) { return int64_t(k) * seg; };
    auto seg_b = [&](int k) { return std::min<int64_t>(N, int64_t(k + 1) * seg); };
    // the advancing forward: state Hf, levels in the ring ringA (level l at
    // slot l mod L), at step `cur`
    int64_t cur = 0;
    auto advance_to = [&](int64_t a) {
        Sweep w{A.ringA, Hf, Sff, nullptr, nullptr, nullptr, L, cur, false, 0};
        set_sweep(s, w);
        modal_steps(s, a - cur);
        cur = a;
    };
    auto save = [&](int slot) -> int {
        double* c = A.ck + size_t(slot) * size_t(A.ck_stride);
        HIPCHK(hipMemcpyAsync(c, Hf, hc * sizeof(double), hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(c + hc, A.ringA, size_t(L) * row, hipMemcpyDeviceToDevice, st));
        return CQ_OK;
    };
    auto load = [&](int slot, int64_t a) -> int {
        const double* c = A.ck + size_t(slot) * size_t(A.ck_stride);
        HIPCHK(hipMemcpyAsync(Hf, c, hc * sizeof(double), hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(A.ringA, c + hc, size_t(L) * row, hipMemcpyDeviceToDevice, st));
        cur = a;
        return CQ_OK;
    };
    // reverse segment k, the forward being at its start
    auto reverse_segment = [&](int k) -> int {
        const int64_t a = seg_a(k), b = seg_b(k);
        // forward over the segment, levels a-L+1 .. b linear in segLev
        for (int64_t l = a - L + 1; l <= a; ++l) {
            const int64_t slot = ((l % L) + L) % L;
            HIPCHK(hipMemcpyAsync(A.segLev + (l - (a - L + 1)) * twoM, A.ringA + slot * twoM, row,
                                  hipMemcpyDeviceToDevice, st));
        }
        double* lvb = A.segLev - (a - L + 1) * twoM;  // level l at lvb + l*2M for a-L+1 <= l <= b
        double* sb = A.segS - (a + 1) * twoM;         // S^n at sb + n*2M for a < n <= b
        Sweep wf{lvb, Hf, Sff, sb, nullptr, nullptr, N + 1, a, false, 0};
        set_sweep(s, wf);
        modal_steps(s, b - a);
        if (b == N && GN) transform(s, lvb + N * twoM, GN, false);
        // the adjoint over the reversed steps N-b+1 .. N-a; mu rows for the
        // reversed steps N-b-1 .. N-a (the two before the piece carried over)
        const int64_t r0 = N - b - 1;
        double* mub = A.segMu - r0 * twoM;
        if (b == N) {
            HIPCHK(hipMemsetAsync(A.segMu, 0, 2 * row, st));
        } else {
            // the previous piece's rows r0, r0+1 sit at rows r0 - r0p, r0 - r0p + 1 of segMu,
            // r0p = N - b' - 1, b' = min(N, b + seg)
            // (one row at a time: the two ranges overlap when that piece was one step long)
            const int64_t r0p = N - std::min<int64_t>(N, b + seg) - 1;
            for (int64_t q = 0; q < 2; ++q)
                HIPCHK(hipMemcpyAsync(A.segMu + q * twoM, A.segMu + (r0 - r0p + q) * twoM, row,
                                      hipMemcpyDeviceToDevice, st));
        }
        Sweep wa{A.psi, A.Ha, A.Sfa, nullptr, mub, A.gc, N + 1, adj_n, true, N % s.Bt};
        set_sweep(s, wa);
        modal_steps(s, b - a);
        adj_n += b - a;
        // this segment's share of dl/da (its chunks) and of d/dbeta (the
        // levels a+1..b against every later step)
        AdjGradArgs ga = grad_args(s, lvb, sb, mub);
        ga.chunk0 = int(a / A.per);
        ga.nchunk_da = int((b - a + A.per - 1) / A.per);
        launch_adj_da(ga, st);
        const int rows = s.Bf;
        for (int64_t n0 = (a / rows) * rows; n0 < N; n0 += rows) {
            const int bt = int(std::min<int64_t>(rows, N - n0));
            beta_rows(s, lvb, n0, bt, rows, a + 1, std::min<int64_t>(b, n0 + bt), k == 0);
        }
        if (k == 0) {  // dl/dG0 from psi (whole) and mu^1, mu^2 (this piece)
            launch_adj_g0(grad_args(s, lvb, sb, mub), st);
            transform(s, A.gG0c, gG0, true);
        }
        HIPCHK(hipGetLastError());
        return CQ_OK;
    };
    // revolve over segments i .. j-1 with the state at segment i saved in
    // `slot` and the states in `free` available
    std::vector<int> freeslots;
    for (int c = A.slots - 1; c >= 1; --c) freeslots.push_back(c);
    const int C = std::max(1, A.slots);
    int rc_all = CQ_OK;
    std::function<void(int, int, int)> rev = [&](int i, int j, int slot) {
        if (rc_all) return;
        const int n = j - i;
        if (n == 1) {
            rc_all = load(slot, seg_a(i));
            if (!rc_all) rc_all = reverse_segment(i);
            return;
        }
        const int c = int(freeslots.size());
        const int m = c > 0 ? A.split[size_t(n) * C + size_t(std::min(c, C - 1))] : 0;
        if (c == 0 || m == 0) {
            for (int k = j - 1; k >= i && !rc_all; --k) {
                rc_all = load(slot, seg_a(i));
                if (rc_all) return;
                advance_to(seg_a(k));
                rc_all = reverse_segment(k);
            }
            return;
        }
        rc_all = load(slot, seg_a(i));
        if (rc_all) return;
        advance_to(seg_a(i + m));
        const int s2 = freeslots.back();
        freeslots.pop_back();
        rc_all = save(s2);
        if (rc_all) return;
        rev(i + m, j, s2);
        freeslots.push_back(s2);
        rev(i, i + m, slot);
    };
    // start: state at step 0 (H = 0, level 0 = g^0, earlier levels zero) in slot 0
    HIPCHK(hipMemsetAsync(Hf, 0, hc * sizeof(double), st));
    HIPCHK(hipMemsetAsync(A.ringA, 0, size_t(L) * row, st));
    HIPCHK(hipMemcpyAsync(A.ringA, s.g0c, row, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemsetAsync(A.Ha, 0, hc * sizeof(double), st));
    HIPCHK(hipMemsetAsync(A.psi, 0, row, st));
    HIPCHK(hipMemsetAsync(A.acc, 0, row, st));
    int rc = save(0);
    if (rc) return rc;
    rev(0, A.nseg, 0);
    if (rc_all) return rc_all;
    launch_sum_rows(A.acc, M, A.part2, st);
    HIPCHK(hipGetLastError());
    return adjoint_finish(s, grad);
}

static int adjoint_exec(Solver& s, const double* G0, const double* gN, double* gG0, double* grad, double* GN) {
    const cq_params* p = &s.p;
    AdjBufs& A = s.ab;
    const int64_t M = s.M, N = s.N, twoM = 2 * M;
    hipStream_t st = s.st;
    HIPCHK(hipMemcpyAsync(s.G0, G0, size_t(twoM) * sizeof(double), hipMemcpyDeviceToDevice, st));
    transform(s, s.G0, s.g0c, true);
    transform(s, gN, A.gc, false);  // dl/dg^N = S^T dl/dG^N, S symmetric
    if (A.ckpt) return adjoint_exec_ckpt(s, gN, gG0, grad, GN);
    double *traj = A.traj, *Sx = A.Sx, *psi = A.psi, *mu = A.mu;
    // forward, keeping every level and history sum
    HIPCHK(hipMemcpyAsync(traj, s.g0c, size_t(twoM) * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemsetAsync(Sx, 0, size_t(twoM) * sizeof(double), st));
    if (p->method == 1) HIPCHK(hipMemsetAsync(A.Hf, 0, hcount(s) * sizeof(double), st));
    if (A.mxfwd) {
        // all N steps on the 16-mode MFMA kernel, levels and history sums
        // written per step (the adjoint sweep below on it too)
        BatchArgs a = mx_args(s);
        a.g0 = s.g0c;
        a.gN = s.Sscratch;
        a.traj = traj;
        a.sx = Sx;
        a.tstride = twoM;
        a.tcols = A.colG;  // b_t = g^{t+1}
        a.tcn = N;
        a.tcb = -1;
        a.tcd = 1;
        if (launch_modal_batch_mx(a, s.mx.ntw, st))
            return fail(CQ_EINVAL, "no per-step template for %d node tiles per wave", s.mx.ntw);
        HIPCHK(hipGetLastError());
    } else {
        set_sweep(s, Sweep{traj, A.Hf, A.Sff, Sx, nullptr, nullptr, N + 1, 0, false, 0});
        modal_steps(s, N);
    }
    if (GN) transform(s, traj + N * twoM, GN, false);

    // adjoint sweep: levels psi, multipliers mu, both in reversed time
    HIPCHK(hipMemsetAsync(psi, 0, size_t(twoM) * sizeof(double), st));
    HIPCHK(hipMemsetAsync(mu, 0, size_t(twoM) * sizeof(double), st));
    if (A.mxfwd) {
        // all N steps on the 16-mode MFMA kernel's adjoint variant: psi^n and
        // mu^n written per step, the cotangent entering step 1
        BatchArgs a = mx_args(s);
        a.g0 = A.gc;
        a.gN = s.Sscratch;
        a.traj = psi;
        a.sx = mu;
        a.tstride = twoM;
        a.adj = 1;
        a.tcols = A.colPsi;  // a_t = psi^{t+1}, kept at row N - t
        a.tcn = N;
        a.tcb = N;
        a.tcd = -1;
        if (launch_modal_batch_mx(a, s.mx.ntw, st))
            return fail(CQ_EINVAL, "no per-step template for %d node tiles per wave", s.mx.ntw);
        HIPCHK(hipGetLastError());
    } else {
        if (p->method == 1) HIPCHK(hipMemsetAsync(A.Hf, 0, hcount(s) * sizeof(double), st));
        set_sweep(s, Sweep{psi, A.Hf, A.Sff, nullptr, mu, A.gc, N + 1, 0, true, p->method == 1 ? N % s.Bt : 0});
        modal_steps(s, N);
    }

    // gradients
    AdjGradArgs ga = grad_args(s, traj, Sx, mu);
    launch_adj_g0(ga, st);
    transform(s, A.gG0c, gG0, true);  // dl/dG0 = P^T dl/dg^0, P = scaled S, symmetric
    launch_adj_da(ga, st);
    // d/dbeta: Toeplitz products of the weight derivatives, over all levels
    // in passes of Bf steps, or in blocks of spec_bk steps over the levels of
    // the previous and the current block only (the farther block pairs
    // follow through block DFTs); BDF2's g^0 term enters with the contraction
    HIPCHK(hipMemsetAsync(A.acc, 0, size_t(twoM) * sizeof(double), st));
    const int rows = A.spec_bk ? A.spec_bk : s.Bf;
    for (int64_t n0 = 0; n0 < N; n0 += rows) {
        const int bt = int(std::min<int64_t>(rows, N - n0));
        const int64_t l0 = A.spec_bk ? std::max<int64_t>(1, n0 - rows + 1) : 1;
        beta_rows(s, traj, n0, bt, rows, l0, n0 + bt, true);
    }
    launch_sum_rows(A.acc, M, A.part2, st);
    HIPCHK(hipGetLastError());
    if (A.spec_nb > 2) {
        // columns a_t = psi^{t+1} (stored in reversed time, row N - t) and
        // b_t = g^{t+1}: written by the sweeps, or transposed here into mu and
        // Sx, which the passes above were the last to read
        if (!A.colG) {
            launch_cols_transpose(psi, N, -1, twoM, N, mu, st);
            launch_cols_transpose(traj, 1, 1, twoM, N, Sx, st);
        }
        BetaSpecArgs bs{};
        bs.N = N;
        bs.M = M;
        bs.nb = A.spec_nb;
        bs.P = A.specP;
        bs.logP = A.specLog;
        bs.cols = A.spec_cols;
        bs.psiT = A.colG ? A.colPsi : mu;
        bs.gT = A.colG ? A.colG : Sx;
        bs.tw = A.tw;
        bs.spec = A.spec;
        launch_beta_spec(bs, A.spec_nwg, st);
        BetaDotArgs bd{};
        bd.nb = A.spec_nb;
        bd.P = A.specP;
        bd.nwg = A.spec_nwg;
        bd.spec = A.spec;
        bd.W = A.W;
        bd.part = A.bpart;
        launch_beta_dot(bd, st);
        HIPCHK(hipGetLastError());
    }
    return adjoint_finish(s, grad);
}

int fp_adjoint_create_opts(const cq_grid* grid, const cq_params* prm, const cq_adjoint_opts* opts, void* hip_stream,
                           void** handle) {
    clear_error();
    if (!handle) return fail(CQ_EINVAL, "handle is NULL");
    *handle = nullptr;
    int rc = validate(grid, prm);
    if (rc) return rc;
    if (prm->solver != 1) return fail(CQ_EINVAL, "the adjoint runs on the modal solver (solver = 1)");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    Solver* s = new (std::nothrow) Solver();
    if (!s) return fail(CQ_ENOMEM, "host allocation failed");
    try {
        rc = setup_host(*s, grid, prm, st);
        if (!rc) rc = adjoint_setup(*s, opts);
    } catch (const std::bad_alloc&) {
        rc = fail(CQ_ENOMEM, "host allocation failed");
    }
    if (rc) {
        (void)hipStreamSynchronize(st);
        delete s;
        return rc;
    }
    *handle = s;
    return CQ_OK;
}

int fp_adjoint_create(const cq_grid* grid, const cq_params* prm, void* hip_stream, void** handle) {
    return fp_adjoint_create_opts(grid, prm, nullptr, hip_stream, handle);
}

int fp_adjoint_info(void* handle, cq_adjoint_info* info) {
    clear_error();
    if (!handle || !info) return fail(CQ_EINVAL, "NULL argument");
    const Solver& s = *static_cast<const Solver*>(handle);
    if (s.kind != 1) return fail(CQ_EINVAL, "handle was not made by fp_adjoint_create");
    const AdjBufs& A = s.ab;
    info->mode = A.ckpt ? 2 : 1;
    info->segment_steps = A.ckpt ? A.seg : s.N;
    info->segments = A.ckpt ? A.nseg : 1;
    info->slots = A.ckpt ? A.slots : 0;
    info->forward_steps = A.fwd_steps;
    info->device_bytes = s.dev_bytes;
    info->forward_kernel = A.mxfwd ? 2 : 1;
    return CQ_OK;
}

int fp_adjoint_run(void* handle, const double* G0, const double* gN, double* gG0, double* grad, double* GN) {
    clear_error();
    if (!handle) return fail(CQ_EINVAL, "handle is NULL");
    Solver& s = *static_cast<Solver*>(handle);
    if (s.kind != 1) return fail(CQ_EINVAL, "handle was not made by fp_adjoint_create");
    if (!G0 || !gN || !gG0 || !grad) return fail(CQ_EINVAL, "G0, gN, gG0 and grad must not be NULL");
    int rc = check_finite_g0(G0, 2 * s.M, s.st);
    if (!rc) rc = check_finite_g0(gN, 2 * s.M, s.st, "gN");
    if (!rc) rc = adjoint_exec(s, G0, gN, gG0, grad, GN);
    if (rc) (void)hipStreamSynchronize(s.st);
    return rc;
}

int fp_adjoint(const cq_grid* grid, const cq_params* prm, const double* G0, const double* gN, double* gG0,
               double* grad, double* GN, void* hip_stream) {
    void* h = nullptr;
    int rc = fp_adjoint_create(grid, prm, hip_stream, &h);
    if (rc) return rc;
    rc = fp_adjoint_run(h, G0, gN, gG0, grad, GN);
    fp_destroy(h);
    return rc;
}

const char* cq_last_error(void) { return cqfp::last_error(); }

}  // extern "C"
