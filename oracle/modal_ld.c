/*
 * Direct BE and BDF2 CQ schemes for selected sine modes, in long double.
 *
 * ORACLE (test infrastructure only). Plain C written from the paper; shares
 * nothing with the GPU library.
 *
 * The uniform-grid Dirichlet Laplacian has the sine modes as eigenvectors
 * (lambda_p = 4/h^2 sin^2(p pi h/2), h = 1/(n+1); lambda_pq = lambda_p +
 * lambda_q in 2D), and the schemes apply A only as a multiplication, so the
 * coefficient of G^n on one mode follows the scheme with A -> lambda: a 2x2
 * recurrence (3D: lambda_pqr = lambda_p + lambda_q + lambda_r). This file
 * runs that recurrence for full-length runs (N up to
 * 2^16 and beyond) in x87 extended precision (64-bit significand, unit
 * roundoff 2^-64), so that an fp64 result can be measured against the
 * scheme's exact value to well below 1e-12 over N steps.
 *
 * Weights (Section 3):
 *   BE, (3.3)-(3.4):  ((1-z)/tau)^beta = tau^-beta sum_i b_i z^i,
 *                     b_0 = 1, b_i = b_{i-1} (1 - (1+beta)/i).
 *   BDF2, (3.11)-(3.12): ((1-z) + (1-z)^2/2)^beta / tau^beta
 *                     = tau^-beta (3/2)^beta (1-z)^beta (1-z/3)^beta,
 *                     the Cauchy product of the b-series and b_k 3^-k; terms
 *                     with k > 80 are below 3^-80 < 1e-38 of the sum and are
 *                     left out.
 * Schemes, with a = (1-m)/(2m-1), S_k = sum_{i=1}^{n-1} d_{k,i} g_k^{n-i}
 * (the CQ sum without G^0, remark after (4.3)):
 *   BE (4.1), n >= 1:
 *     [[1/tau + d_{1,0}(a+lam), -a d_{2,0}], [-a d_{1,0}, 1/tau + d_{2,0}(a+lam)]] g^n
 *       = g^{n-1}/tau - [(a+lam) S_1 - a S_2; (a+lam) S_2 - a S_1].
 *   BDF2 (4.7), n = 1 (weights 2/3 on g^1 and 1/3 on g^0):
 *     [[1/tau + 2/3 d_{1,0}(a+lam), -2/3 a d_{2,0}], [sym.]] g^1
 *       = g^0/tau - 1/3 [d_{1,0}(a+lam) g_1^0 - a d_{2,0} g_2^0; sym.];
 *   n >= 2, T_k = S_k + 1/2 d_{k,n-1} g_k^0:
 *     [[3/(2tau) + d_{1,0}(a+lam), -a d_{2,0}], [sym.]] g^n
 *       = (2 g^{n-1} - 1/2 g^{n-2})/tau - [(a+lam) T_1 - a T_2; sym.].
 * Each 2x2 system is solved by Cramer's rule.
 *
 * Entry point (fp64 in and out):
 *   modal_direct_ld(dim, nx, ny, nz, K, mp, mq, mr, alpha1, alpha2, m, T, N,
 *                   G0, scheme, out)
 *   G0: [2][nx*ny*nz] nodal values (x fastest, then y, then z); mode j is
 *   (mp[j], mq[j], mr[j]) (mq ignored in 1D, mr below 3D); out: [2][K]
 *   coefficients of G^N on those modes, with G = sum_p c_p phi_p and
 *   phi_p(i) = sin(p pi i/(n+1)) (products over the directions).
 *   The modes run in parallel (OpenMP) when the library is built with it.
 *   Returns 0, or -1 on bad arguments, -3 if memory runs out.
 */
#include <math.h>
#include <stdlib.h>

typedef long double ld;

static ld pi_ld(void) { return acosl(-1.0L); }

static void binomial_series(ld beta, long n, ld* b) {
    b[0] = 1.0L;
    for (long i = 1; i <= n; ++i) b[i] = b[i - 1] * (1.0L - (1.0L + beta) / (ld)i);
}

/* d_0 .. d_n of the scheme, order beta, step tau */
static int cq_weights_ld(int scheme, ld beta, ld tau, long n, ld* d) {
    ld* b = (ld*)malloc(sizeof(ld) * (size_t)(n + 1));
    if (!b) return -3;
    binomial_series(beta, n, b);
    const ld s = powl(tau, -beta);
    if (scheme == 1) {
        for (long i = 0; i <= n; ++i) d[i] = s * b[i];
    } else {
        ld h[81];
        ld p3 = 1.0L;
        for (int k = 0; k <= 80; ++k) {
            h[k] = (k <= n ? b[k] : 0.0L) * p3;
            p3 /= 3.0L;
        }
        const ld f = s * powl(1.5L, beta);
        for (long i = 0; i <= n; ++i) {
            ld acc = 0.0L;
            const long kmax = i < 80 ? i : 80;
            for (long k = 0; k <= kmax; ++k) acc += b[i - k] * h[k];
            d[i] = f * acc;
        }
    }
    free(b);
    return 0;
}

static ld lambda_1d(int n, int p) {
    const ld sn = sinl((ld)p * pi_ld() / (2.0L * (ld)(n + 1)));
    return 4.0L * (ld)(n + 1) * (ld)(n + 1) * sn * sn;
}

/* coefficient of component k of G0 on mode (p, q, r) */
static ld project(int dim, int nx, int ny, int nz, const double* G0k, int p, int q, int r) {
    const ld pi = pi_ld();
    ld* sx = (ld*)malloc(sizeof(ld) * (size_t)nx);
    if (!sx) return NAN;
    for (int i = 0; i < nx; ++i) sx[i] = sinl((ld)p * pi * (ld)(i + 1) / (ld)(nx + 1));
    ld acc = 0.0L;
    const int nyy = dim >= 2 ? ny : 1, nzz = dim == 3 ? nz : 1;
    for (int k = 0; k < nzz; ++k) {
        ld plane = 0.0L;
        for (int j = 0; j < nyy; ++j) {
            ld row = 0.0L;
            const double* g = G0k + ((long)k * nyy + j) * nx;
            for (int i = 0; i < nx; ++i) row += (ld)g[i] * sx[i];
            plane += dim >= 2 ? row * sinl((ld)q * pi * (ld)(j + 1) / (ld)(ny + 1)) : row;
        }
        acc += dim == 3 ? plane * sinl((ld)r * pi * (ld)(k + 1) / (ld)(nz + 1)) : plane;
    }
    free(sx);
    ld scale = 2.0L / (ld)(nx + 1);
    if (dim >= 2) scale *= 2.0L / (ld)(ny + 1);
    if (dim == 3) scale *= 2.0L / (ld)(nz + 1);
    return scale * acc;
}

/* S = sum_{i=1}^{n-1} d_i g^{n-i} (g: one component's levels, g[l]) */
static ld history(const ld* d, const ld* g, long n) {
    ld s0 = 0.0L, s1 = 0.0L, s2 = 0.0L, s3 = 0.0L;
    long i = 1;
    for (; i + 3 <= n - 1; i += 4) {
        s0 += d[i] * g[n - i];
        s1 += d[i + 1] * g[n - i - 1];
        s2 += d[i + 2] * g[n - i - 2];
        s3 += d[i + 3] * g[n - i - 3];
    }
    for (; i <= n - 1; ++i) s0 += d[i] * g[n - i];
    return (s0 + s1) + (s2 + s3);
}

static void solve2(ld a11, ld a12, ld a21, ld a22, ld r1, ld r2, ld* x1, ld* x2) {
    const ld det = a11 * a22 - a12 * a21;
    *x1 = (a22 * r1 - a12 * r2) / det;
    *x2 = (a11 * r2 - a21 * r1) / det;
}

/* one mode: eigenvalue lam, start (c1, c2); writes g^N */
static int run_mode(int scheme, ld lam, ld a, ld tau, long N, const ld* d1, const ld* d2, ld c1, ld c2, ld* o1,
                    ld* o2) {
    ld* g1 = (ld*)malloc(sizeof(ld) * (size_t)(N + 1));
    ld* g2 = (ld*)malloc(sizeof(ld) * (size_t)(N + 1));
    if (!g1 || !g2) {
        free(g1);
        free(g2);
        return -3;
    }
    g1[0] = c1;
    g2[0] = c2;
    const ld al = a + lam;
    for (long n = 1; n <= N; ++n) {
        const ld S1 = history(d1, g1, n), S2 = history(d2, g2, n);
        ld r1, r2, a11, a12, a21, a22;
        if (scheme == 1) {
            const ld c = 1.0L / tau;
            r1 = g1[n - 1] / tau - (al * S1 - a * S2);
            r2 = g2[n - 1] / tau - (al * S2 - a * S1);
            a11 = c + d1[0] * al;
            a12 = -a * d2[0];
            a21 = -a * d1[0];
            a22 = c + d2[0] * al;
        } else if (n == 1) {
            const ld t2 = 2.0L / 3.0L, t1 = 1.0L / 3.0L;
            r1 = g1[0] / tau - t1 * (d1[0] * al * g1[0] - a * d2[0] * g2[0]);
            r2 = g2[0] / tau - t1 * (d2[0] * al * g2[0] - a * d1[0] * g1[0]);
            a11 = 1.0L / tau + t2 * d1[0] * al;
            a12 = -t2 * a * d2[0];
            a21 = -t2 * a * d1[0];
            a22 = 1.0L / tau + t2 * d2[0] * al;
        } else {
            const ld c = 1.5L / tau;
            const ld T1 = S1 + 0.5L * d1[n - 1] * g1[0];
            const ld T2 = S2 + 0.5L * d2[n - 1] * g2[0];
            r1 = (2.0L * g1[n - 1] - 0.5L * g1[n - 2]) / tau - (al * T1 - a * T2);
            r2 = (2.0L * g2[n - 1] - 0.5L * g2[n - 2]) / tau - (al * T2 - a * T1);
            a11 = c + d1[0] * al;
            a12 = -a * d2[0];
            a21 = -a * d1[0];
            a22 = c + d2[0] * al;
        }
        solve2(a11, a12, a21, a22, r1, r2, &g1[n], &g2[n]);
    }
    *o1 = g1[N];
    *o2 = g2[N];
    free(g1);
    free(g2);
    return 0;
}

int modal_direct_ld(int dim, int nx, int ny, int nz, int K, const int* mp, const int* mq, const int* mr,
                    double alpha1, double alpha2, double m, double T, long N, const double* G0, int scheme,
                    double* out) {
    if (dim < 1 || dim > 3 || nx < 1 || (dim >= 2 && ny < 1) || (dim == 3 && nz < 1) || K < 1 || N < 1 || !mp ||
        !G0 || !out || (scheme != 1 && scheme != 2) || (dim >= 2 && !mq) || (dim == 3 && !mr))
        return -1;
    if (dim == 1) ny = 1;
    if (dim < 3) nz = 1;
    const long M = (long)nx * ny * nz;
    const ld tau = (ld)T / (ld)N;
    const ld a = (1.0L - (ld)m) / (2.0L * (ld)m - 1.0L);
    ld* d1 = (ld*)malloc(sizeof(ld) * (size_t)(N + 1));
    ld* d2 = (ld*)malloc(sizeof(ld) * (size_t)(N + 1));
    if (!d1 || !d2) {
        free(d1);
        free(d2);
        return -3;
    }
    int rc = cq_weights_ld(scheme, 1.0L - (ld)alpha1, tau, N, d1);
    if (!rc) rc = cq_weights_ld(scheme, 1.0L - (ld)alpha2, tau, N, d2);
    int bad = rc;
#pragma omp parallel for schedule(dynamic, 1) reduction(min : bad)
    for (int j = 0; j < K; ++j) {
        if (rc) continue;
        const int p = mp[j], q = dim >= 2 ? mq[j] : 1, r = dim == 3 ? mr[j] : 1;
        if (p < 1 || p > nx || q < 1 || q > ny || r < 1 || r > nz) {
            bad = -1;
            continue;
        }
        const ld lam = lambda_1d(nx, p) + (dim >= 2 ? lambda_1d(ny, q) : 0.0L) + (dim == 3 ? lambda_1d(nz, r) : 0.0L);
        const ld c1 = project(dim, nx, ny, nz, G0, p, q, r);
        const ld c2 = project(dim, nx, ny, nz, G0 + M, p, q, r);
        ld o1 = 0.0L, o2 = 0.0L;
        const int st = run_mode(scheme, lam, a, tau, N, d1, d2, c1, c2, &o1, &o2);
        if (st) {
            bad = st;
            continue;
        }
        out[j] = (double)o1;
        out[K + j] = (double)o2;
    }
    free(d1);
    free(d2);
    return bad;
}
