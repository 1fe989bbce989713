// Batched fast solves: many independent problems of uneven size in one
// captured HIP graph (the batched modal fast kernels, one branch per register
// class, and the inverse transforms), with the lanes-per-mode tile of every
// register class chosen by timing (autotuner, cached per process). The set-up
// and the instantiated graph of the last batch are kept: a call with the same
// problems and arrays runs the forward transforms and relaunches the graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.h"
#include "kernels.h"

using namespace cqfp;

#define BHIP(expr)                                                                          \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) return fail(CQ_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

namespace {

struct HostProblem {
    int dim = 1, nx = 1, ny = 1, nz = 1;
    int64_t M = 0, N = 0;
    int np = 0, L = 0, scheme = 2;
    double tau = 0, a = 0, c = 0;
    double lx = 1, ly = 1, lz = 1;
    std::vector<double> d[2];  // weights 0..N
    FastRule rule[2];
    int rc = CQ_OK;
    std::string err;
};

double lam1d(int n, double len, int p) {
    const double h = len / (n + 1);
    const double s = std::sin(p * M_PI / (2.0 * (n + 1)));
    return 4.0 / (h * h) * s * s;
}

std::vector<double> sine_tab(int n) {
    std::vector<double> S(size_t(n) * size_t(n));
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const int64_t kk = (int64_t(i + 1) * (j + 1)) % (2 * int64_t(n + 1));
            S[size_t(i) * size_t(n) + size_t(j)] = std::sin(M_PI * double(kk) / double(n + 1));
        }
    return S;
}

// host set-up of one problem: weights, fast rule (lag <= 64, <= 1024 nodes)
void prepare(const cq_grid& g, const cq_params& p, HostProblem& h) {
    h.dim = g.dim;
    h.nx = g.nx;
    h.ny = g.dim >= 2 ? g.ny : 1;
    h.nz = g.dim == 3 ? g.nz : 1;
    h.lx = g.lx;
    h.ly = g.ly;
    h.lz = g.lz;
    h.M = int64_t(h.nx) * h.ny * h.nz;
    h.N = p.N;
    h.scheme = p.scheme;
    h.tau = p.T / double(p.N);
    h.a = (1.0 - p.m) / (2.0 * p.m - 1.0);
    h.c = (p.scheme == 1 ? 1.0 : 1.5) / h.tau;
    const double beta[2] = {1.0 - p.alpha1, 1.0 - p.alpha2};
    const int ns = p.ns ? p.ns : 30, np1 = p.np1 ? p.np1 : 16;
    const int np_max = p.np_max ? p.np_max : 1024;
    const double tol = p.fast_tol > 0 ? p.fast_tol : 1e-8;
    // weights d_0..d_max(N,64): the kernels read the exact-weight window
    // (lags < L <= 64) whatever N is
    const int64_t nd = std::max<int64_t>(h.N, 64);
    for (int k = 0; k < 2; ++k) {
        h.d[k].assign(size_t(nd) + 1, 0.0);
        weights(p.scheme, beta[k], h.tau, nd, h.d[k].data());
    }
    int npk[2];
    for (int k = 0; k < 2; ++k) {
        if (p.np > 0) {
            build_rule(p.scheme, beta[k], h.tau, p.np, np1, ns, h.rule[k]);
        } else {
            const int rc = choose_rule(p.scheme, beta[k], h.tau, h.N, tol, np_max, np1, ns, h.rule[k]);
            if (rc != CQ_OK) {
                h.rc = rc;
                return;
            }
        }
        npk[k] = int(h.rule[k].ratio.size());
    }
    if (npk[0] != npk[1]) {
        const int k = npk[0] < npk[1] ? 0 : 1;
        build_rule(p.scheme, beta[k], h.tau, std::max(npk[0], npk[1]) - (p.scheme == 2 ? np1 : 0), np1, ns,
                   h.rule[k]);
    }
    if (p.scheme == 1) {  // exact window below 2np+2 (the rule is exact there)
        const int Lw = std::min(32, 2 * int(h.rule[0].ratio.size()) + 2);
        shift_lag(h.rule[0], Lw);
        shift_lag(h.rule[1], Lw);
    }
    h.np = int(h.rule[0].ratio.size());
    h.L = h.rule[0].lag;
    if (h.L > 64 || h.np > 1024) h.rc = CQ_EINVAL;
}

struct DevBuf {
    std::vector<void*> p;
    ~DevBuf() {
        for (void* q : p) (void)hipFree(q);
    }
    template <class T>
    int alloc(T** out, size_t count) {
        void* q = nullptr;
        if (hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(CQ_ENOMEM, "batched solve: device allocation of %zu bytes failed", count * sizeof(T));
        }
        p.push_back(q);
        *out = static_cast<T*>(q);
        return CQ_OK;
    }
};

// the last batch's set-up, device tables and instantiated graph
struct BatchCache {
    std::vector<double> key;          // problem fields and array addresses
    DevBuf buf;
    hipStream_t st = nullptr;
    std::vector<hipStream_t> branch;  // class branches of the graph
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    struct Xf {
        const double* in;
        double* out;
        int dim, nx, ny, nz;
        double scale;
        const double *Sx, *Sy, *Sz;
    };
    std::vector<Xf> fwd;  // forward transforms: G0[i] -> its coefficients in the batch arrays
    double* d_tmp = nullptr;
    cq_batch_report rep{};
    ~BatchCache() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (hipStream_t b : branch) (void)hipStreamDestroy(b);
        if (st) (void)hipStreamDestroy(st);
    }
};
std::mutex g_batch_mu;
std::unique_ptr<BatchCache> g_batch;

std::vector<double> batch_key(int count, const cq_grid* grids, const cq_params* params, const double* const* G0,
                              double* const* GN, int autotune) {
    std::vector<double> k;
    k.reserve(size_t(count) * 24 + 2);
    k.push_back(double(count));
    k.push_back(double(autotune));
    int dev = 0;
    (void)hipGetDevice(&dev);
    k.push_back(double(dev));
    for (int i = 0; i < count; ++i) {
        const cq_grid& g = grids[i];
        const cq_params& p = params[i];
        for (double v : {double(g.dim), double(g.nx), double(g.ny), g.lx, g.ly, double(g.dim == 3 ? g.nz : 1),
                         g.dim == 3 ? g.lz : 1.0, p.alpha1, p.alpha2, p.m, p.T, double(p.N), double(p.scheme),
                         double(p.method), p.fast_tol, double(p.np), double(p.np1), double(p.ns), double(p.np_max)})
            k.push_back(v);
        uint64_t a = uint64_t(reinterpret_cast<uintptr_t>(G0[i])), b = uint64_t(reinterpret_cast<uintptr_t>(GN[i]));
        double da, db;
        std::memcpy(&da, &a, 8);
        std::memcpy(&db, &b, 8);
        k.push_back(da);
        k.push_back(db);
    }
    return k;
}

bool same_key(const std::vector<double>& a, const std::vector<double>& b) {
    return a.size() == b.size() && std::memcmp(a.data(), b.data(), a.size() * sizeof(double)) == 0;
}

std::mutex g_tune_mu;
std::map<std::pair<int, int>, int> g_tune;  // (npl at 64 lanes, lag class) -> lanes per mode

int npl_for(int np, int lpm) { return (np + lpm - 1) / lpm; }
// nodes per lane of the time-blocked kernel's templates (32 lanes per component)
int tb_tmpl(int npl32) {
    for (int t : {4, 6, 8, 10, 12, 14, 16, 18, 20, 24})
        if (npl32 <= t) return t;
    return 24;
}
int npl_tmpl(int npl, int lpm) {
    if (lpm == 64 && npl <= 1) return 1;
    if (npl <= 2) return 2;
    if (npl <= 4) return 4;
    if (npl <= 8) return 8;
    if (npl <= 12) return 12;
    return 16;
}

bool mx_ok(const HostProblem& h) { return mx_applies(h.L, h.np); }

void mx_tables(const HostProblem& h, double* out) {
    const double* ratio[2] = {h.rule[0].ratio.data(), h.rule[1].ratio.data()};
    const double* coef[2] = {h.rule[0].coef.data(), h.rule[1].coef.data()};
    const double* d[2] = {h.d[0].data(), h.d[1].data()};
    build_mx_tables(h.np, h.L, ratio, coef, d, out);
}

}  // namespace

extern "C" int fp_solve_batched(int32_t count, const cq_grid* grids, const cq_params* params,
                                const double* const* G0, double* const* GN, void* hip_stream,
                                int32_t autotune, cq_batch_report* report) {
    clear_error();
    if (count < 1 || !grids || !params || !G0 || !GN || autotune < 0 || autotune > 4)
        return fail(CQ_EINVAL, "batched solve: bad arguments");
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<HostProblem> hp(static_cast<size_t>(count));
    for (int i = 0; i < count; ++i) {
        const cq_grid& g = grids[i];
        const cq_params& p = params[i];
        if (g.dim < 1 || g.dim > 3 || g.nx < 1 || g.ny < 1 || (g.dim == 1 && g.ny != 1) || !(g.lx > 0) ||
            (g.dim >= 2 && !(g.ly > 0)) || (g.dim < 3 && g.nz != 0 && g.nz != 1) ||
            (g.dim == 3 && (g.nz < 1 || !(g.lz > 0) || int64_t(g.ny) * g.nz > (int64_t(1) << 20))))
            return fail(CQ_EINVAL, "batched solve: problem %d has a bad grid", i);
        if (!(p.alpha1 > 0 && p.alpha1 < 1 && p.alpha2 > 0 && p.alpha2 < 1) || !(p.m >= 0 && p.m <= 1) ||
            p.m == 0.5 || !(p.T > 0) || p.N < 1 || (p.scheme != 1 && p.scheme != 2) || p.method != 1 ||
            p.np < 0 || p.np > 1024 || (p.scheme == 2 && p.ns != 0 && (p.ns < 3 || p.ns > 64)))
            return fail(CQ_EINVAL, "batched solve: problem %d has bad parameters (fast method only)", i);
        if (!G0[i] || !GN[i]) return fail(CQ_EINVAL, "batched solve: NULL array for problem %d", i);
    }
    hipStream_t user = static_cast<hipStream_t>(hip_stream);
    std::lock_guard<std::mutex> batch_lock(g_batch_mu);  // calls are serialised: they share the cache
    std::vector<double> key = batch_key(count, grids, params, G0, GN, autotune);
    if (g_batch && same_key(g_batch->key, key)) {
        BatchCache& c = *g_batch;
        hipEvent_t ev_in;
        BHIP(hipEventCreateWithFlags(&ev_in, hipEventDisableTiming));
        BHIP(hipEventRecord(ev_in, user));
        BHIP(hipStreamWaitEvent(c.st, ev_in, 0));
        (void)hipEventDestroy(ev_in);
        for (const auto& x : c.fwd)
            launch_sine_transform(x.dim, x.nx, x.ny, x.nz, x.Sx, x.Sy, x.Sz, x.in, c.d_tmp, x.out, x.scale, c.st);
        BHIP(hipGetLastError());
        const auto t1 = std::chrono::steady_clock::now();
        hipError_t ce = hipGraphLaunch(c.exec, c.st);
        if (ce == hipSuccess) ce = hipStreamSynchronize(c.st);
        if (ce != hipSuccess) return fail(CQ_EHIP, "batched graph: %s", hipGetErrorString(ce));
        const auto t2 = std::chrono::steady_clock::now();
        if (report) {
            *report = c.rep;
            report->setup_s = std::chrono::duration<double>(t1 - t0).count();
            report->autotune_s = 0.0;
            report->run_s = std::chrono::duration<double>(t2 - t1).count();
        }
        return CQ_OK;
    }
    g_batch.reset();  // a new batch: release the previous one's device memory first
    // host set-up in parallel
    {
        const int nt = std::max(1u, std::min(8u, std::thread::hardware_concurrency()));
        std::vector<std::thread> th;
        for (int t = 0; t < nt; ++t)
            th.emplace_back([&, t] {
                for (int i = t; i < count; i += nt) prepare(grids[i], params[i], hp[size_t(i)]);
            });
        for (auto& x : th) x.join();
    }
    for (int i = 0; i < count; ++i) {
        const HostProblem& h = hp[size_t(i)];
        if (h.rc == CQ_ETOL) return fail(CQ_ETOL, "batched solve: problem %d: fast rule cannot meet the tolerance", i);
        if (h.rc != CQ_OK)
            return fail(CQ_EINVAL, "batched solve: problem %d needs lag %d <= 64 and %d <= 1024 nodes", i, h.L, h.np);
        // step operator check, as for a single solve
        const double d10 = h.d[0][0], d20 = h.d[1][0];
        const double K[2][2] = {{h.c / d10 + h.a, -h.a * d20 / d10}, {-h.a * d10 / d20, h.c / d20 + h.a}};
        double th[2], V[2][2], Vi[2][2];
        eig2(K, th, V, Vi);
        double lmin = lam1d(h.nx, h.lx, 1) + (h.dim >= 2 ? lam1d(h.ny, h.ly, 1) : 0.0) +
                      (h.dim == 3 ? lam1d(h.nz, h.lz, 1) : 0.0);
        if (!(th[0] + lmin > 0 && th[1] + lmin > 0))
            return fail(CQ_ESINGULAR, "batched solve: problem %d: step operator not positive definite", i);
    }
    // concatenated tables
    std::vector<BatchInst> inst(static_cast<size_t>(count));
    std::vector<double> ratio, coef, dd, lam;
    int64_t modes = 0;
    for (int i = 0; i < count; ++i) {
        HostProblem& h = hp[size_t(i)];
        BatchInst& I = inst[size_t(i)];
        I.mode_off = modes;
        I.M = h.M;
        I.N = h.N;
        I.np = h.np;
        I.L = h.L;
        I.scheme = h.scheme;
        I.rule_off = int64_t(ratio.size());
        for (int k = 0; k < 2; ++k) {
            ratio.insert(ratio.end(), h.rule[k].ratio.begin(), h.rule[k].ratio.end());
            coef.insert(coef.end(), h.rule[k].coef.begin(), h.rule[k].coef.end());
        }
        I.d_off = int64_t(dd.size());
        I.dstride = int64_t(h.d[0].size());
        dd.insert(dd.end(), h.d[0].begin(), h.d[0].end());
        dd.insert(dd.end(), h.d[1].begin(), h.d[1].end());
        I.inv_tau = 1.0 / h.tau;
        I.c = h.c;
        I.a = h.a;
        I.d00 = h.d[0][0];
        I.d01 = h.d[1][0];
        I.mx_off = -1;
        I.nt = (h.np + 15) / 16;
        for (int r = 0; r < h.nz; ++r)
            for (int j = 0; j < h.ny; ++j)
                for (int q = 0; q < h.nx; ++q)
                    lam.push_back(lam1d(h.nx, h.lx, q + 1) + (h.dim >= 2 ? lam1d(h.ny, h.ly, j + 1) : 0.0) +
                                  (h.dim == 3 ? lam1d(h.nz, h.lz, r + 1) : 0.0));
        modes += h.M;
    }
    DevBuf buf;
    BatchInst* d_inst;
    double *d_ratio, *d_coef, *d_d, *d_lam, *d_g0, *d_gN, *d_tmp;
    int rc;
    int64_t maxM = 0;
    for (auto& h : hp) maxM = std::max(maxM, h.M);
    if ((rc = buf.alloc(&d_inst, inst.size())) || (rc = buf.alloc(&d_ratio, ratio.size())) ||
        (rc = buf.alloc(&d_coef, coef.size())) || (rc = buf.alloc(&d_d, dd.size())) ||
        (rc = buf.alloc(&d_lam, lam.size())) || (rc = buf.alloc(&d_g0, size_t(2 * modes))) ||
        (rc = buf.alloc(&d_gN, size_t(2 * modes))) || (rc = buf.alloc(&d_tmp, size_t(2 * maxM))))
        return rc;
    BHIP(hipMemcpy(d_inst, inst.data(), inst.size() * sizeof(BatchInst), hipMemcpyHostToDevice));
    BHIP(hipMemcpy(d_ratio, ratio.data(), ratio.size() * sizeof(double), hipMemcpyHostToDevice));
    BHIP(hipMemcpy(d_coef, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice));
    BHIP(hipMemcpy(d_d, dd.data(), dd.size() * sizeof(double), hipMemcpyHostToDevice));
    BHIP(hipMemcpy(d_lam, lam.data(), lam.size() * sizeof(double), hipMemcpyHostToDevice));
    // sine tables per distinct size
    std::map<int, double*> sines;
    for (auto& h : hp)
        for (int n : {h.nx, h.dim >= 2 ? h.ny : 0, h.dim == 3 ? h.nz : 0}) {
            if (n <= 0 || sines.count(n)) continue;
            double* q;
            if ((rc = buf.alloc(&q, size_t(n) * size_t(n)))) return rc;
            const std::vector<double> S = sine_tab(n);
            BHIP(hipMemcpy(q, S.data(), S.size() * sizeof(double), hipMemcpyHostToDevice));
            sines[n] = q;
        }
    // register classes (nodes per lane at 64 lanes) and the problems in each
    // Problems the time-blocked kernel takes (lags 8..32, <= 768 nodes) are
    // grouped by its nodes per lane at 32 lanes (the template the class runs
    // with), the others by nodes per lane at 64 lanes; a class runs with its
    // largest problem's node count, so tight classes waste fewer lanes.
    std::map<int, std::vector<int>> cls;
    for (int i = 0; i < count; ++i) {
        const HostProblem& h = hp[size_t(i)];
        const int n32 = npl_for(h.np, 32);
        const bool tb = h.L >= 8 && h.L <= 32 && n32 <= 24;
        cls[tb ? 1000 + tb_tmpl(n32) : npl_tmpl(npl_for(h.np, 64), 64)].push_back(i);
    }
    // longest time loops first: workgroups start in index order, so the
    // short modes fill the GPU at the end instead of a long tail
    for (auto& kv : cls)
        std::stable_sort(kv.second.begin(), kv.second.end(), [&](int x, int y) {
            const HostProblem &a = hp[size_t(x)], &b = hp[size_t(y)];
            return a.N * (a.np + a.L) > b.N * (b.np + b.L);
        });
    std::vector<int> lists;
    std::vector<int64_t> cums, cumts;
    // lpm: lanes per mode of the per-step kernel (64 or 32), 0 for the
    // time-blocked kernel (one wave per mode, needs lags <= 32 and <= 768
    // nodes), kLpmMx for the 16-mode MFMA kernel (mx_ok problems)
    struct Launch {
        int npl64, lpm, count, maxnp, minlag;
        int64_t total, tiles;
        size_t list_off, cum_off;
        bool lag32, canmx;
    };
    constexpr int kLpmMx = 16;
    constexpr bool kDefaultMx = true;  // the default (autotune 0) prefers the MFMA kernel
    std::vector<Launch> launches;
    for (auto& kv : cls) {
        Launch l{};
        l.count = int(kv.second.size());
        l.list_off = lists.size();
        l.cum_off = cums.size();
        l.lag32 = true;
        l.canmx = true;
        int64_t c = 0, ct = 0;
        int maxnp = 0, minlag = 64;
        for (int i : kv.second) {
            lists.push_back(i);
            cums.push_back(c);
            cumts.push_back(ct);
            c += hp[size_t(i)].M;
            ct += (hp[size_t(i)].M + 15) / 16;
            l.lag32 = l.lag32 && hp[size_t(i)].L <= 32;
            l.canmx = l.canmx && mx_ok(hp[size_t(i)]);
            maxnp = std::max(maxnp, hp[size_t(i)].np);
            minlag = std::min(minlag, hp[size_t(i)].L);
        }
        cums.push_back(c);
        cumts.push_back(ct);
        l.total = c;
        l.tiles = ct;
        l.maxnp = maxnp;
        l.npl64 = npl_tmpl(npl_for(maxnp, 64), 64);
        l.minlag = minlag;
        // without timing: the MFMA kernel where it applies, else time-blocked
        // where every lag allows blocks of >= 8 steps; a forced kernel
        // (autotune 2..4) where it applies
        const bool cantb = l.lag32 && minlag >= 8 && npl_for(maxnp, 32) <= 24;
        l.lpm = cantb ? 0 : 64;
        if ((autotune == 3 || (autotune == 0 && kDefaultMx)) && l.canmx) l.lpm = kLpmMx;
        if (autotune == 4) l.lpm = 64;
        launches.push_back(l);
    }
    // tables of the MFMA kernel for the problems of the classes that may take it
    double* d_mx = nullptr;
    {
        std::vector<int64_t> mxoff(size_t(count), -1);
        int64_t mxsize = 0;
        for (const Launch& l : launches) {
            if (!l.canmx || !(l.lpm == kLpmMx || autotune == 1)) continue;
            for (int c = 0; c < l.count; ++c) {
                const int i = lists[l.list_off + size_t(c)];
                mxoff[size_t(i)] = mxsize;
                mxsize += mx_table_size((hp[size_t(i)].np + 15) / 16);
            }
        }
        if (mxsize > 0) {
            std::vector<double> mx(size_t(mxsize), 0.0);
            const int nt = std::max(1u, std::min(8u, std::thread::hardware_concurrency()));
            std::vector<std::thread> th;
            for (int t = 0; t < nt; ++t)
                th.emplace_back([&, t] {
                    for (int i = t; i < count; i += nt)
                        if (mxoff[size_t(i)] >= 0) mx_tables(hp[size_t(i)], mx.data() + mxoff[size_t(i)]);
                });
            for (auto& x : th) x.join();
            if ((rc = buf.alloc(&d_mx, mx.size()))) return rc;
            BHIP(hipMemcpy(d_mx, mx.data(), mx.size() * sizeof(double), hipMemcpyHostToDevice));
            for (int i = 0; i < count; ++i) inst[size_t(i)].mx_off = mxoff[size_t(i)];
            BHIP(hipMemcpy(d_inst, inst.data(), inst.size() * sizeof(BatchInst), hipMemcpyHostToDevice));
        }
    }
    int* d_list;
    int64_t *d_cum, *d_cumt;
    if ((rc = buf.alloc(&d_list, lists.size())) || (rc = buf.alloc(&d_cum, cums.size())) ||
        (rc = buf.alloc(&d_cumt, cumts.size())))
        return rc;
    BHIP(hipMemcpy(d_list, lists.data(), lists.size() * sizeof(int), hipMemcpyHostToDevice));
    BHIP(hipMemcpy(d_cum, cums.data(), cums.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    BHIP(hipMemcpy(d_cumt, cumts.data(), cumts.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    std::unique_ptr<BatchCache> cache(new BatchCache());
    BHIP(hipStreamCreateWithFlags(&cache->st, hipStreamNonBlocking));
    hipStream_t st = cache->st;
    // the caller's stream may still be producing G0
    hipEvent_t ev_in;
    BHIP(hipEventCreateWithFlags(&ev_in, hipEventDisableTiming));
    BHIP(hipEventRecord(ev_in, user));
    BHIP(hipStreamWaitEvent(st, ev_in, 0));
    (void)hipEventDestroy(ev_in);

    auto make_args = [&](const Launch& l) {
        BatchArgs a{};
        a.inst = d_inst;
        a.list = d_list + l.list_off;
        a.cum = d_cum + l.cum_off;
        a.count = l.count;
        a.total = l.total;
        a.ratio = d_ratio;
        a.coef = d_coef;
        a.d = d_d;
        a.lam = d_lam;
        a.g0 = d_g0;
        a.gN = d_gN;
        a.cumt = d_cumt + l.cum_off;
        a.tiles = l.tiles;
        a.mx = d_mx;
        return a;
    };
    // one class's kernel
    auto launch_class = [&](const BatchArgs& a, const Launch& l, int lpm, int npl, hipStream_t s) {
        if (lpm == kLpmMx)
            launch_modal_batch_mx(a, mx_template(((l.maxnp + 15) / 16 + 1) / 2), s);
        else
            launch_modal_batch(a, npl, lpm, s);
    };
    // forward transforms of every G0 into the concatenated coefficient array
    auto transforms = [&](bool forward) {
        for (int i = 0; i < count; ++i) {
            const HostProblem& h = hp[size_t(i)];
            const int64_t off = 2 * inst[size_t(i)].mode_off;
            const double* in = forward ? G0[i] : d_gN + off;
            double* out = forward ? d_g0 + off : GN[i];
            double scale = 1.0;
            if (forward) {
                scale = 2.0 / double(h.nx + 1);
                if (h.dim >= 2) scale *= 2.0 / double(h.ny + 1);
                if (h.dim == 3) scale *= 2.0 / double(h.nz + 1);
            }
            const BatchCache::Xf x{in, out, h.dim, h.nx, h.ny, h.nz, scale, sines[h.nx],
                                   h.dim >= 2 ? sines[h.ny] : nullptr, h.dim == 3 ? sines[h.nz] : nullptr};
            if (forward) cache->fwd.push_back(x);
            launch_sine_transform(x.dim, x.nx, x.ny, x.nz, x.Sx, x.Sy, x.Sz, x.in, d_tmp, x.out, x.scale, st);
        }
    };
    transforms(true);
    BHIP(hipGetLastError());
    const auto t1 = std::chrono::steady_clock::now();
    // nodes per lane of a class's kernel
    auto npl_of = [](const Launch& l, int lpm) {
        return lpm == 0 ? npl_for(l.maxnp, 32) : npl_tmpl(npl_for(l.npl64 * 64, lpm), lpm);
    };
    // autotune per class: the time-blocked kernel, 64 and 32 lanes per mode
    // and the 16-mode MFMA kernel (each where it applies), timed on the
    // class's problems truncated to a few steps
    double tune_s = 0.0;
    for (Launch& l : launches) {
        if (autotune != 1) continue;
        const int npl32 = npl_for(l.npl64 * 64, 32);
        const bool can32 = l.lag32 && npl32 <= 16;
        const bool cantb = l.lag32 && npl_for(l.maxnp, 32) <= 24;
        const std::pair<int, int> key{(l.npl64 * 2048 + l.maxnp) * 2 + (l.canmx ? 1 : 0),
                                      l.lag32 ? l.minlag : 64};
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tune.find(key);
            if (it != g_tune.end()) {
                l.lpm = it->second;
                continue;
            }
        }
        if (!can32 && !cantb && !l.canmx) continue;
        const auto ta = std::chrono::steady_clock::now();
        // short copies of the class's problems (at most 256 steps: long enough
        // for the time-blocked kernel to pass its first blocks)
        std::vector<BatchInst> shortI(inst);
        for (auto& I : shortI) I.N = std::min<int64_t>(I.N, 256);
        BatchInst* d_short;
        if ((rc = buf.alloc(&d_short, shortI.size()))) return rc;
        BHIP(hipMemcpy(d_short, shortI.data(), shortI.size() * sizeof(BatchInst), hipMemcpyHostToDevice));
        BatchArgs a = make_args(l);
        a.inst = d_short;
        double* scratch;  // the timing runs write here, not into the results
        if ((rc = buf.alloc(&scratch, size_t(2 * modes)))) return rc;
        a.gN = scratch;
        float best_ms = 1e30f;
        int best = l.lpm;
        hipEvent_t e0, e1;
        BHIP(hipEventCreate(&e0));
        BHIP(hipEventCreate(&e1));
        for (int lpm : {0, 64, 32, kLpmMx}) {
            if ((lpm == 0 && !cantb) || (lpm == 32 && !can32) || (lpm == kLpmMx && !l.canmx)) continue;
            const int npl = npl_of(l, lpm);
            launch_class(a, l, lpm, npl, st);  // warm
            BHIP(hipEventRecord(e0, st));
            launch_class(a, l, lpm, npl, st);
            BHIP(hipEventRecord(e1, st));
            BHIP(hipEventSynchronize(e1));
            float ms = 0.f;
            BHIP(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best_ms) {
                best_ms = ms;
                best = lpm;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        l.lpm = best;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune[key] = best;
        }
        tune_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - ta).count();
    }
    // the batched run (one graph branch per register class, so that the
    // classes' tails overlap) and the inverse transforms, captured as one graph
    cache->branch.assign(launches.size(), nullptr);
    for (auto& b : cache->branch) BHIP(hipStreamCreateWithFlags(&b, hipStreamNonBlocking));
    std::vector<hipEvent_t> evs(launches.size() + 1, nullptr);
    for (auto& e : evs) BHIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    struct EvGuard {
        std::vector<hipEvent_t>& v;
        ~EvGuard() {
            for (hipEvent_t e : v)
                if (e) (void)hipEventDestroy(e);
        }
    } evg{evs};
    BHIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    hipError_t ce = hipEventRecord(evs[0], st);
    for (size_t c = 0; c < launches.size() && ce == hipSuccess; ++c) {
        ce = hipStreamWaitEvent(cache->branch[c], evs[0], 0);
        if (ce != hipSuccess) break;
        launch_class(make_args(launches[c]), launches[c], launches[c].lpm, npl_of(launches[c], launches[c].lpm),
                     cache->branch[c]);
        ce = hipEventRecord(evs[c + 1], cache->branch[c]);
        if (ce == hipSuccess) ce = hipStreamWaitEvent(st, evs[c + 1], 0);
    }
    if (ce == hipSuccess) transforms(false);
    hipGraph_t graph = nullptr;
    hipError_t ce2 = hipStreamEndCapture(st, &graph);
    if (ce != hipSuccess || ce2 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(CQ_EHIP, "graph capture: %s", hipGetErrorString(ce != hipSuccess ? ce : ce2));
    }
    cache->graph = graph;
    ce = hipGraphInstantiate(&cache->exec, graph, nullptr, nullptr, 0);
    if (ce != hipSuccess) return fail(CQ_EHIP, "graph instantiate: %s", hipGetErrorString(ce));
    const auto t2 = std::chrono::steady_clock::now();
    ce = hipGraphLaunch(cache->exec, st);
    if (ce == hipSuccess) ce = hipStreamSynchronize(st);
    const auto t3 = std::chrono::steady_clock::now();
    if (ce != hipSuccess) return fail(CQ_EHIP, "batched graph: %s", hipGetErrorString(ce));
    cq_batch_report r{};
    r.problems = count;
    r.modes = modes;
    r.classes = int32_t(std::min<size_t>(launches.size(), 8));
    for (int c = 0; c < r.classes; ++c) {
        r.class_npl64[c] = launches[size_t(c)].npl64;
        const int lpm = launches[size_t(c)].lpm;
        r.class_lanes[c] = (lpm == 0 || lpm == kLpmMx) ? 64 : lpm;
        r.class_blocked[c] = lpm == 0 ? 1 : lpm == kLpmMx ? 2 : 0;
        r.class_problems[c] = launches[size_t(c)].count;
    }
    r.setup_s = std::chrono::duration<double>(t1 - t0).count();
    r.autotune_s = tune_s;
    r.run_s = std::chrono::duration<double>(t3 - t2).count();
    if (report) *report = r;
    cache->rep = r;
    // keep the set-up, tables and graph for a call with the same batch
    cache->key.swap(key);
    cache->buf.p.swap(buf.p);
    cache->d_tmp = d_tmp;
    g_batch = std::move(cache);
    return CQ_OK;
}
