// HIP kernels (gfx950) of the CQ solver's per-step hot path.
//
// Every kernel here is one stage of a time step n of scheme (4.1) or (4.7):
//   history  S_k = sum_{i=1}^{n-1} d_k,i G_k^{n-i}      (direct or fast form)
//   rhs      r_k = E_k - (a + A) S'_k + a S'_k'        (E: time-difference part,
//            S' = S + d_k,n-1 G_k^0 / 2 for BDF2)
//   solve    [[c + d_1,0 (a+A), -a d_2,0], [-a d_1,0, c + d_2,0 (a+A)]] G^n = r
//            (evaluated as G^n = K^-1 (E + c Delta^-1 S') - Delta^-1 S', below)
// Field layout: [2][M] component-major, x fastest. Time levels live in a
// "level store": level l at slot (l mod Lr) of a [Lr][2][M] array (Lr = N+1
// keeps the whole history for the direct form; Lr = window length for the
// fast form).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include <cstdint>

#include "device_util.h"
#include "kernels.h"

namespace cqfp {

// ---------------------------------------------------------------------------
// Fast history (3.10)/(3.18), time-blocked. For lag L the state
//   H_j(m) = sum_{l=1}^{m-L} r_j^(m-L-l) G^l,   H_j(m) = r_j H_j(m-1) + G^{m-L},
// and the fast part of the history sum is S_f(m) = sum_j coef_j H_j(m).
// H_j(m) only involves levels up to m-L, so for the BT steps m = n..n+BT-1
// (BT <= L) every level it needs is known before step n is solved. One pass
// over the state therefore advances it by BT steps and emits S_f for all of
// them: the state (the bulk of the bytes) is read and written once per BT
// steps instead of once per step. blockIdx.z = component. When the DOFs
// alone cannot fill the GPU, S waves of a workgroup share one 64-DOF tile,
// wave s taking the node slice [s*chunk, (s+1)*chunk); their partial sums
// meet in LDS and the slice-0 wave adds them in slice order and stores.
// One DOF per lane; H is [2][np][M], so a wave streams 64 consecutive DOFs
// of one node, and r_j and coef_j are wave-uniform. Output Sf[b][k][x].
// State loads and stores of the pass: non-temporal (streamed past the caches)
// when the state is larger than the Infinity Cache can hold across passes,
// ordinary when it fits (it then stays in the cache from one pass to the
// next: 5% faster per pass for a 54 MB state; non-temporal 3% faster for a
// 1.2 GB one).
template <bool NT>
__device__ __forceinline__ double hb_load(const double* a) {
    if constexpr (NT) return __builtin_nontemporal_load(a);
    else return *a;
}
template <bool NT>
__device__ __forceinline__ void hb_store(double v, double* a) {
    if constexpr (NT) __builtin_nontemporal_store(v, a);
    else *a = v;
}

template <int BT, int S, bool NT>
__global__ __launch_bounds__(256) void k_hist_block(HistBlockArgs p) {
    constexpr int TILES = 4 / S;  // 64-DOF tiles per workgroup
    __shared__ double red[S > 1 ? (S - 1) * TILES * BT * 64 : 1];
    const int k = blockIdx.z;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int sl = wave % S, tile = wave / S;
    const int64_t x = (int64_t(blockIdx.x) * TILES + tile) * 64 + lane;
    const bool xin = x < p.M;
    const int64_t xc = xin ? x : p.M - 1;  // levels of a valid DOF for the padding lanes
    const int64_t twoM = 2 * p.M;
    const double* __restrict__ lv = p.levels + int64_t(k) * p.M + xc;
    double g[BT], acc[BT];
#pragma unroll
    for (int b = 0; b < BT; ++b) {
        const int64_t l = p.n + b - p.L;  // level entering the state at step n+b
        int64_t slot = p.slot0 + b;       // its slot: (n - L + b) mod Lr
        if (slot >= p.Lr) slot -= p.Lr;
        g[b] = (b < p.bt && l >= 1) ? lv[slot * twoM] : 0.0;
        acc[b] = 0.0;
    }
    const int j0 = __builtin_amdgcn_readfirstlane(sl * p.chunk);  // wave-uniform
    const int j1 = (j0 + p.chunk < p.np) ? j0 + p.chunk : p.np;
    // state rows are hstride (a multiple of 256) long: every lane owns a slot
    const int64_t hs = p.hstride;
    double* __restrict__ h = p.H + (int64_t(k) * p.np) * hs + x;
    // ratios and coefficients are wave-uniform: read through the constant
    // address space they become scalar loads, which the wait for a group's
    // state (vector memory counter) does not include, so the next group's
    // state loads stay in flight while this group is advanced
    const cdouble* r = (const cdouble*)(p.ratio + k * p.np);
    const cdouble* w = (const cdouble*)(p.coef + k * p.np);
    // four nodes per group (independent recurrences interleave); the states
    // of the next group are loaded before this group is advanced, so a load
    // is in flight while the previous one is used. A full block (bt == BT)
    // runs without per-step guards.
    auto nodes = [&](auto full_t) {
        constexpr bool FULLB = decltype(full_t)::value;
        int j = j0;
        double hn0 = 0.0, hn1 = 0.0, hn2 = 0.0, hn3 = 0.0;
        if (j + 4 <= j1) {
            hn0 = hb_load<NT>(h + int64_t(j) * hs);
            hn1 = hb_load<NT>(h + int64_t(j + 1) * hs);
            hn2 = hb_load<NT>(h + int64_t(j + 2) * hs);
            hn3 = hb_load<NT>(h + int64_t(j + 3) * hs);
        }
#pragma unroll 1
        for (; j + 4 <= j1; j += 4) {
            double h0 = hn0, h1 = hn1, h2 = hn2, h3 = hn3;
            if (j + 8 <= j1) {
                hn0 = hb_load<NT>(h + int64_t(j + 4) * hs);
                hn1 = hb_load<NT>(h + int64_t(j + 5) * hs);
                hn2 = hb_load<NT>(h + int64_t(j + 6) * hs);
                hn3 = hb_load<NT>(h + int64_t(j + 7) * hs);
            }
            const double r0 = r[j], r1 = r[j + 1], r2 = r[j + 2], r3 = r[j + 3];
            const double w0 = w[j], w1 = w[j + 1], w2 = w[j + 2], w3 = w[j + 3];
#pragma unroll
            for (int b = 0; b < BT; ++b) {
                if (FULLB || b < p.bt) {
                    h0 = fma(r0, h0, g[b]);
                    h1 = fma(r1, h1, g[b]);
                    h2 = fma(r2, h2, g[b]);
                    h3 = fma(r3, h3, g[b]);
                    acc[b] = fma(w0, h0, acc[b]);
                    acc[b] = fma(w1, h1, acc[b]);
                    acc[b] = fma(w2, h2, acc[b]);
                    acc[b] = fma(w3, h3, acc[b]);
                }
            }
            hb_store<NT>(h0, h + int64_t(j) * hs);
            hb_store<NT>(h1, h + int64_t(j + 1) * hs);
            hb_store<NT>(h2, h + int64_t(j + 2) * hs);
            hb_store<NT>(h3, h + int64_t(j + 3) * hs);
        }
        for (; j < j1; ++j) {
            double h0 = h[int64_t(j) * hs];
            const double r0 = r[j], w0 = w[j];
#pragma unroll
            for (int b = 0; b < BT; ++b) {
                if (FULLB || b < p.bt) {
                    h0 = fma(r0, h0, g[b]);
                    acc[b] = fma(w0, h0, acc[b]);
                }
            }
            h[int64_t(j) * hs] = h0;
        }
    };
    if (BT <= 30 && p.bt == BT)  // (at BT = 32 the unguarded copy costs a wave per SIMD in registers)
        nodes(std::true_type{});
    else
        nodes(std::false_type{});
    if (S > 1) {
        double* __restrict__ mine = red + int64_t(tile * (S - 1)) * BT * 64 + lane;
        if (sl > 0) {
#pragma unroll
            for (int b = 0; b < BT; ++b) mine[((sl - 1) * BT + b) * 64] = acc[b];
        }
        __syncthreads();
        if (sl > 0) return;
#pragma unroll 1
        for (int q = 0; q < S - 1; ++q)
#pragma unroll
            for (int b = 0; b < BT; ++b) acc[b] += mine[(q * BT + b) * 64];
    }
    if (!xin) return;
#pragma unroll
    for (int b = 0; b < BT; ++b)
        if (b < p.bt) p.Sf[(int64_t(b) * 2 + k) * p.M + x] = acc[b];
}

// ---------------------------------------------------------------------------
// Direct history, near field: the far part for steps n0+1..n0+B was summed by
// k_far_toeplitz into F[ks][B][2][M]; here the lags inside the block are added
//   S = sum_q F[q][n-n0-1] + sum_{l=n0+1}^{n-1} d_{n-l} G^l.
__global__ __launch_bounds__(256) void k_hist_direct(HistDirectArgs p) {
    const int k = blockIdx.z;
    const int64_t x = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (x >= p.M) return;
    const int64_t twoM = 2 * p.M;
    double S = 0.0;
    if (p.n0 >= 1) S = p.F[(int64_t(p.n - p.n0 - 1) * 2 + k) * p.M + x];  // reduced far field
    const double* __restrict__ dk = p.d + int64_t(k) * p.dstride;
    const double* __restrict__ lv = p.levels + int64_t(k) * p.M + x;
    double S2 = 0.0;
    int64_t l = p.n0 + 1;
    // eight levels per round: the loads are independent, the sum is not
    for (; l + 8 <= p.n; l += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = lv[(l + u) * twoM];
#pragma unroll
        for (int u = 0; u < 8; ++u) S2 = fma(dk[p.n - l - u], v[u], S2);
    }
    for (; l <= p.n - 1; ++l) S2 = fma(dk[p.n - l], lv[l * twoM], S2);
    p.Spart[int64_t(k) * p.M + x] = S + S2;
}

// ---------------------------------------------------------------------------
// Step solve. With L = a + A, D = [[L, -a], [-a, L]] and Delta = diag(d_1,0, d_2,0),
// the step operator is K = c I + D Delta and the right-hand side is E - D S'.
// Since K^-1 D = (I - c K^-1) Delta^-1, the new level is
//   G^n = K^-1 (E + c Delta^-1 S') - Delta^-1 S',
// so the stencil never acts on the (rough) history: every right-hand side
// below is pointwise, and the only spatial coupling is inside K^-1.
// error-free transforms for the double-double residual
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}
__device__ __forceinline__ void dd_add(double& hi, double& lo, double x) {
    double s, e;
    two_sum(hi, x, s, e);
    hi = s;
    lo += e;
}

// History sum of step n at node x of component k, from the partial sum
// (fast: Sf of this step's block; direct: the near/far kernel's output) plus
// the exact-weight window sum_{i=1}^{win} d_i G^{n-i} (win <= 31; the loads
// are issued before the sum) plus the BDF2 correction d_{n-1}/2 G^0.
// Returns S'. Level n-i sits at slot s1 - (i-1) (mod Lr).
__device__ __forceinline__ double history_at(const StepArgs& p, int k, int64_t x) {
    const int64_t M = p.M;
    double s = p.Sp[p.boff + k * M + x];
    if (p.win > 0) {
        const double* __restrict__ dk = p.d + int64_t(k) * p.dstride;
        const double* __restrict__ lv = p.levels + int64_t(k) * M + x;
        const int64_t twoM = 2 * M;
        double v[32];
#pragma unroll
        for (int i = 1; i <= 31; ++i) {
            int64_t sl = p.slot1 - (i - 1);
            if (sl < 0) sl += p.Lr;
            v[i] = (i <= p.win) ? lv[sl * twoM] : 0.0;
        }
        double s2 = 0.0;
#pragma unroll
        for (int i = 1; i <= 31; ++i)
            if (i <= p.win) s2 = fma(dk[i], v[i], s2);
        s += s2;
    }
    return fma(p.corr[k], p.G0[k * M + x], s);
}

// Time-difference part E_k of the right-hand side (BE: G^{n-1}/tau; BDF2:
// (2 G^{n-1} - G^{n-2}/2)/tau with G^{-1} = G^0 at n = 1).
__device__ __forceinline__ double time_part(const StepArgs& p, int k, int64_t x) {
    const int64_t twoM = 2 * p.M;
    const double* lv = p.levels + int64_t(k) * p.M + x;
    const double g1 = lv[p.slot1 * twoM];
    if (p.scheme == 1) return g1 * p.inv_tau;
    return (2.0 * g1 - 0.5 * lv[p.slot2 * twoM]) * p.inv_tau;
}


// 1D: K = Delta (I (x) A + Kc (x) I) with the 2x2 coupling Kc = V diag(theta) V^-1,
// so K^-1 w = V z with (A + theta_k I) z_k = (V^-1 Delta^-1 w)_k: two constant
// tridiagonal systems T_k z = h^2 y, T_k = tridiag(-1, 2 + delta_k, -1),
// delta_k = theta_k h^2, solved by parallel cyclic reduction (PCR) in LDS
// (stride s: every row eliminates rows i-s and i+s; ceil(log2 M) levels),
// with the eliminations precomputed once per run (k_pcr_setup). One
// refinement step follows: the residual h^2 y - T z is summed in
// double-double with the diagonal kept as 2 and delta apart (2 + delta is not
// representable to the accuracy the smallest eigenvalue needs), and PCR
// solves for the correction. One workgroup of 1024 threads, R rows each.
constexpr int kNT1D = 1024;

// The matrices T_k never change within a run, so the PCR eliminations do not
// either: the set-up (host, once per run) runs PCR on (a, b, c) and stores,
// per level l and row i, the multipliers f = a_i / b_{i-s} and g = c_i / b_{i+s}
// and finally 1/b_i. A solve is then the right-hand-side recurrence alone,
//   d_i <- d_i - f d_{i-s} - g d_{i+s},   x_i = d_i / b_i,
// (two FMAs and two LDS reads per row and level). Multipliers: PF, PG
// [levels][2][M]; PRB [2][M]. Rows per thread: at most 4 (M <= 4096).
// Right-hand-side recurrence of PCR with the stored multipliers; sd holds d
// on entry and x on exit. The next level's multipliers are loaded before the
// barrier of the current one.

template <int R>
__device__ void pcr_apply(double* sd, int64_t M, int levels, const double* __restrict__ PF,
                          const double* __restrict__ PG, const double* __restrict__ PRB) {
    const int tid = threadIdx.x;
    double fc[R][2], gc[R][2];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t x = tid + int64_t(r) * kNT1D;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            fc[r][k] = (x < M && levels > 0) ? PF[k * M + x] : 0.0;
            gc[r][k] = (x < M && levels > 0) ? PG[k * M + x] : 0.0;
        }
    }
    int64_t s = 1;
    for (int lvl = 0; lvl < levels; ++lvl, s <<= 1) {
        double nd[R][2], fn[R][2], gn[R][2];
        const bool more = lvl + 1 < levels;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t x = tid + int64_t(r) * kNT1D;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int64_t o = k * M;
                double dd = 0.0;
                if (x < M) {
                    dd = sd[o + x];
                    if (x - s >= 0) dd = fma(-fc[r][k], sd[o + x - s], dd);
                    if (x + s < M) dd = fma(-gc[r][k], sd[o + x + s], dd);
                }
                nd[r][k] = dd;
                fn[r][k] = (more && x < M) ? PF[(int64_t(lvl + 1) * 2 + k) * M + x] : 0.0;
                gn[r][k] = (more && x < M) ? PG[(int64_t(lvl + 1) * 2 + k) * M + x] : 0.0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t x = tid + int64_t(r) * kNT1D;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                if (x < M) sd[k * M + x] = nd[r][k];
                fc[r][k] = fn[r][k];
                gc[r][k] = gn[r][k];
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t x = tid + int64_t(r) * kNT1D;
        if (x < M) {
#pragma unroll
            for (int k = 0; k < 2; ++k) sd[k * M + x] *= PRB[k * M + x];
        }
    }
    __syncthreads();
}

template <int R>
__global__ __launch_bounds__(1024) void k_step_1d(StepArgs p) {
    extern __shared__ double sm[];
    const int64_t M = p.M;
    double* sd = sm;  // [2][M]
    const int64_t twoM = 2 * M;
    const int tid = threadIdx.x;
    // 1. w = E + c S'/d0, q = S'/d0, y = h^2 V^-1 Delta^-1 w
    double ry[R][2], qv[R][2];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t x = tid + int64_t(r) * kNT1D;
        if (x < M) {
            double u[2];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const double qk = history_at(p, k, x) * p.inv_d0[k];
                qv[r][k] = qk;
                u[k] = (time_part(p, k, x) + p.cdiag * qk) * p.inv_d0[k];
            }
            ry[r][0] = (p.Vinv[0] * u[0] + p.Vinv[1] * u[1]) * p.h2;
            ry[r][1] = (p.Vinv[2] * u[0] + p.Vinv[3] * u[1]) * p.h2;
            sd[x] = ry[r][0];
            sd[M + x] = ry[r][1];
        }
    }
    __syncthreads();
    pcr_apply<R>(sd, M, p.levels_pcr, p.PF, p.PG, p.PRB);
    // 2. residual in double-double
    double rr[R][2], zown[R][2];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t x = tid + int64_t(r) * kNT1D;
        if (x < M) {
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int64_t o = k * M;
                const double z = sd[o + x];
                zown[r][k] = z;
                const double zl = (x > 0) ? sd[o + x - 1] : 0.0;
                const double zr = (x + 1 < M) ? sd[o + x + 1] : 0.0;
                double hi = ry[r][k], lo = 0.0;
                dd_add(hi, lo, zl);
                dd_add(hi, lo, zr);
                dd_add(hi, lo, -2.0 * z);
                const double pz = p.delta[k] * z;
                const double pe = fma(p.delta[k], z, -pz);
                dd_add(hi, lo, -pz);
                lo -= pe;
                rr[r][k] = hi + lo;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t x = tid + int64_t(r) * kNT1D;
        if (x < M) {
            sd[x] = rr[r][0];
            sd[M + x] = rr[r][1];
        }
    }
    __syncthreads();
    pcr_apply<R>(sd, M, p.levels_pcr, p.PF, p.PG, p.PRB);
    // 3. G^n = V (z + dz) - Delta^-1 S'
    double* out = p.levels + p.slot_out * twoM;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t x = tid + int64_t(r) * kNT1D;
        if (x < M) {
            const double z0 = zown[r][0] + sd[x];
            const double z1 = zown[r][1] + sd[M + x];
            out[x] = p.V[0] * z0 + p.V[1] * z1 - qv[r][0];
            out[M + x] = p.V[2] * z0 + p.V[3] * z1 - qv[r][1];
        }
    }
}

// The same step for M <= 1024 (one row per thread), with the PCR multipliers
// of every level held in registers (loaded once, all in flight, and used by
// both solves) and the reduction ping-ponging between two LDS buffers (one
// barrier per level). 32-bit indices. The arithmetic, and its order, is that
// of k_step_1d: the results are the same bit for bit.
constexpr int kPcrMaxLevels = 10;  // ceil(log2 1024)

__device__ __forceinline__ void pcr_regs(double*& cur, double*& nxt, int M, int levels, int x,
                                         const double (&f)[kPcrMaxLevels][2], const double (&g)[kPcrMaxLevels][2],
                                         const double (&rb)[2], double (&out)[2]) {
#pragma unroll
    for (int lvl = 0; lvl < kPcrMaxLevels; ++lvl) {
        if (lvl < levels) {  // uniform
            const int st = 1 << lvl;
            if (x < M) {
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const int o = k * M;
                    double dd = cur[o + x];
                    if (x - st >= 0) dd = fma(-f[lvl][k], cur[o + x - st], dd);
                    if (x + st < M) dd = fma(-g[lvl][k], cur[o + x + st], dd);
                    nxt[o + x] = dd;
                }
            }
            __syncthreads();
            double* t = cur;
            cur = nxt;
            nxt = t;
        }
    }
    if (x < M) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            out[k] = cur[k * M + x] * rb[k];
            nxt[k * M + x] = out[k];
        }
    }
    __syncthreads();
    // the solution now also sits in nxt, for the neighbours' reads
    double* t = cur;
    cur = nxt;
    nxt = t;
}

__global__ __launch_bounds__(1024) void k_step_1d_reg(StepArgs p) {
    extern __shared__ double sm[];
    const int M = int(p.M);
    const int x = threadIdx.x;
    const int levels = p.levels_pcr;
    double* cur = sm;          // [2][M]
    double* nxt = sm + 2 * M;  // [2][M]
    // 1. w = E + c S'/d0, q = S'/d0, y = h^2 V^-1 Delta^-1 w
    double ry[2] = {0.0, 0.0}, qv[2] = {0.0, 0.0};
    if (x < M) {
        double u[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const double qk = history_at(p, k, x) * p.inv_d0[k];
            qv[k] = qk;
            u[k] = (time_part(p, k, x) + p.cdiag * qk) * p.inv_d0[k];
        }
        ry[0] = (p.Vinv[0] * u[0] + p.Vinv[1] * u[1]) * p.h2;
        ry[1] = (p.Vinv[2] * u[0] + p.Vinv[3] * u[1]) * p.h2;
        cur[x] = ry[0];
        cur[M + x] = ry[1];
    }
    // multipliers of every level, all loads issued together (after the
    // history window's registers are free)
    double f[kPcrMaxLevels][2], g[kPcrMaxLevels][2], rb[2];
#pragma unroll
    for (int lvl = 0; lvl < kPcrMaxLevels; ++lvl)
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const bool ok = lvl < levels && x < M;
            f[lvl][k] = ok ? p.PF[(lvl * 2 + k) * M + x] : 0.0;
            g[lvl][k] = ok ? p.PG[(lvl * 2 + k) * M + x] : 0.0;
        }
#pragma unroll
    for (int k = 0; k < 2; ++k) rb[k] = x < M ? p.PRB[k * M + x] : 0.0;
    __syncthreads();
    double z[2] = {0.0, 0.0};
    pcr_regs(cur, nxt, M, levels, x, f, g, rb, z);
    // 2. residual h^2 y - T z in double-double (z of the neighbours from cur)
    double rr[2] = {0.0, 0.0};
    if (x < M) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int o = k * M;
            const double zl = (x > 0) ? cur[o + x - 1] : 0.0;
            const double zr = (x + 1 < M) ? cur[o + x + 1] : 0.0;
            double hi = ry[k], lo = 0.0;
            dd_add(hi, lo, zl);
            dd_add(hi, lo, zr);
            dd_add(hi, lo, -2.0 * z[k]);
            const double pz = p.delta[k] * z[k];
            const double pe = fma(p.delta[k], z[k], -pz);
            dd_add(hi, lo, -pz);
            lo -= pe;
            rr[k] = hi + lo;
        }
        nxt[x] = rr[0];
        nxt[M + x] = rr[1];
    }
    __syncthreads();
    {
        double* t = cur;
        cur = nxt;
        nxt = t;
    }
    double dz[2] = {0.0, 0.0};
    pcr_regs(cur, nxt, M, levels, x, f, g, rb, dz);
    // 3. G^n = V (z + dz) - Delta^-1 S'
    if (x < M) {
        double* out = p.levels + p.slot_out * 2 * p.M;
        const double z0 = z[0] + dz[0];
        const double z1 = z[1] + dz[1];
        out[x] = p.V[0] * z0 + p.V[1] * z1 - qv[0];
        out[M + x] = p.V[2] * z0 + p.V[3] * z1 - qv[1];
    }
}

// ---------------------------------------------------------------------------
// 2D: pointwise right-hand side w = E + c Delta^-1 S' and q = Delta^-1 S'
// (the forward DST, per-mode solve and inverse DST follow; the last GEMM
// subtracts q).
__global__ __launch_bounds__(256) void k_prep_2d(StepArgs p) {
    const int64_t M = p.M;
    const int64_t x = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (x >= M) return;
    const int k = blockIdx.y;
    const double qk = history_at(p, k, x) * p.inv_d0[k];
    p.q[k * M + x] = qk;
    p.w[k * M + x] = time_part(p, k, x) + p.cdiag * qk;
}

// ---------------------------------------------------------------------------
// Modal solver. The uniform-grid Dirichlet Laplacian is diagonalised by the
// sine transform, A_h = S diag(lambda) S^-1, and every stage of the schemes
// applies A only as a multiplication, so the sine coefficients of G^n obey
// the same scheme with A -> lambda_p, independently for every mode p:
//   [[c + d_1,0 (a+l), -a d_2,0], [-a d_1,0, c + d_2,0 (a+l)]] g^n
//       = E - [(a+l) S'_1 - a S'_2 ; (a+l) S'_2 - a S'_1].
// With no coupling between modes there is no per-step global dependency:
// the transform runs once at the start and once per read-out.

// sum over each group of G lanes (G = 2, 4, 8, 16), in every lane of the group
template <int G>
__device__ __forceinline__ double row_group_sum(double v) {
    if (G >= 2) v += dpp_move<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
    if (G >= 4) v += dpp_move<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
    if (G >= 8) v += dpp_move<0x141, 0xF>(v);  // row_half_mirror
    if (G >= 16) v += dpp_move<0x140, 0xF>(v); // row_mirror
    return v;
}

// sum over the 64 lanes, in every lane: rows of 16, then row_bcast15 (row r
// += lane 15 of row r-1, rows 1 and 3) and row_bcast31 (rows 2 and 3 += lane
// 31), which leaves the total in lane 63
__device__ __forceinline__ double wave_sum(double v) {
    v = row_group_sum<16>(v);
    v += dpp_move<0x142, 0xA>(v);
    v += dpp_move<0x143, 0xC>(v);
    return lane_value(v, 63);
}

// Fast form, persistent: one wave per mode runs `nsteps` steps. Lane l holds
// nodes j = l + 64 q (q < NPL) of both components (ratio, coefficient and
// state H_j in registers) and the window level g^{n-1-l} (lane l < L): the
// state input g^{n-L} is lane L-1, the exact-weight window is lanes
// 0..min(L-1,n-1)-1 with weights d_1.., and after each step the levels move
// up one lane. One wave reduction per component gives S; every lane then
// solves the 2x2 system. State H[2][np][M] and window ring[L][2][M]
// (ring[i] = g^{n-1-i}) are loaded at entry and stored at exit.
template <int NPL>
__global__ __launch_bounds__(256) void k_modal_fast(ModalFastArgs p) {
    const int lane = threadIdx.x & 63;
    const int64_t mode = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (mode >= p.M) return;  // uniform per wave
    const int64_t M = p.M;
    double r[2][NPL], w[2][NPL], h[2][NPL];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int q = 0; q < NPL; ++q) {
            const int j = lane + 64 * q;
            const bool ok = j < p.np;
            r[k][q] = ok ? p.ratio[k * p.np + j] : 0.0;
            w[k][q] = ok ? p.coef[k * p.np + j] : 0.0;
            h[k][q] = ok ? p.H[(int64_t(k) * p.np + j) * M + mode] : 0.0;
        }
    double dw[2], ring[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        dw[k] = (lane < p.L - 1) ? p.d[k * p.dstride + lane + 1] : 0.0;
        ring[k] = (lane < p.L) ? p.ring[(int64_t(lane) * 2 + k) * M + mode] : 0.0;
    }
    const double lam = p.lam[mode];
    const double g00 = p.g0[mode], g01 = p.g0[M + mode];
    const double L1 = p.a + lam;
    const double m11 = p.c + p.d0[0] * L1, m22 = p.c + p.d0[1] * L1;
    const double m12 = -p.a * p.d0[1], m21 = -p.a * p.d0[0];
    const double idet = 1.0 / (m11 * m22 - m12 * m21);
    for (int t = 0; t < p.nsteps; ++t) {
        const int64_t n = p.n0 + 1 + t;
        double part[2] = {0.0, 0.0};
        if (n >= p.L + 1) {
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const double gin = lane_value(ring[k], p.L - 1);
                double pa = 0.0, pb = 0.0;
#pragma unroll
                for (int q = 0; q < NPL; ++q) {
                    h[k][q] = fma(r[k][q], h[k][q], gin);
                    if (q & 1)
                        pb = fma(w[k][q], h[k][q], pb);
                    else
                        pa = fma(w[k][q], h[k][q], pa);
                }
                part[k] = pa + pb;
            }
        }
        const int64_t wn = (n - 1 < p.L - 1) ? n - 1 : p.L - 1;
        if (lane < wn) {
            part[0] = fma(dw[0], ring[0], part[0]);
            part[1] = fma(dw[1], ring[1], part[1]);
        }
        double S0 = wave_sum(part[0]);
        double S1 = wave_sum(part[1]);
        const double gm10 = lane_value(ring[0], 0), gm11 = lane_value(ring[1], 0);
        double E0, E1;
        if (p.scheme == 1) {
            E0 = gm10 * p.inv_tau;
            E1 = gm11 * p.inv_tau;
        } else {
            const double gm20 = lane_value(ring[0], 1), gm21 = lane_value(ring[1], 1);
            E0 = (2.0 * gm10 - 0.5 * gm20) * p.inv_tau;
            E1 = (2.0 * gm11 - 0.5 * gm21) * p.inv_tau;
            S0 = fma(0.5 * p.d[n - 1], g00, S0);
            S1 = fma(0.5 * p.d[p.dstride + n - 1], g01, S1);
        }
        const double r0 = E0 - (L1 * S0 - p.a * S1);
        const double r1 = E1 - (L1 * S1 - p.a * S0);
        const double gn0 = (m22 * r0 - m12 * r1) * idet;
        const double gn1 = (m11 * r1 - m21 * r0) * idet;
        // levels move up one lane (DPP wave_shr:1)
        const double up0 = dpp_move<0x138, 0xF>(ring[0]), up1 = dpp_move<0x138, 0xF>(ring[1]);
        ring[0] = (lane == 0) ? gn0 : up0;
        ring[1] = (lane == 0) ? gn1 : up1;
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
#pragma unroll
        for (int q = 0; q < NPL; ++q) {
            const int j = lane + 64 * q;
            if (j < p.np) p.H[(int64_t(k) * p.np + j) * M + mode] = h[k][q];
        }
        if (lane < p.L) p.ring[(int64_t(lane) * 2 + k) * M + mode] = ring[k];
    }
}

// Batched fast form: many independent problems (grids, orders, m, N and
// node counts differ) in one launch. Every group of LPM lanes owns one mode
// of one problem and runs that problem's whole time loop, as k_modal_fast
// does for a single problem (state in registers, window in lanes, reduction
// over the group, 2x2 solve); the problem of a group is found by binary
// search over the cumulative mode counts of the launch's problem list. All
// problems of a launch share the register tile NPL (nodes per lane) and the
// group width LPM (32 or 64 lanes; the lag must fit: L <= LPM). Starts from
// zero state and G^0, writes the coefficients of G^N.
template <int LPM>
__device__ __forceinline__ double group_sum(double v) {
    if (LPM == 64) return wave_sum(v);
    if (LPM == 32) {  // rows 0+1 and 2+3: totals in lanes 31 and 63
        v = row_group_sum<16>(v);
        v += dpp_move<0x142, 0xA>(v);
        const double s0 = lane_value(v, 31), s1 = lane_value(v, 63);
        return (threadIdx.x & 32) ? s1 : s0;
    }
    return row_group_sum<LPM>(v);
}

template <int NPL, int LPM>
__global__ __launch_bounds__(256) void k_modal_batch(BatchArgs p) {
    const int lane = threadIdx.x & (LPM - 1);
    const int64_t group = (int64_t(blockIdx.x) * 256 + threadIdx.x) / LPM;
    if (group >= p.total) return;  // uniform per group
    // problem of this group
    int lo = 0, hi = p.count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (p.cum[mid] <= group) lo = mid; else hi = mid - 1;
    }
    const BatchInst& I = p.inst[p.list[lo]];
    const int64_t mode = group - p.cum[lo];
    const int64_t M = I.M;
    const int np = I.np, L = I.L;
    const double* __restrict__ ratio = p.ratio + I.rule_off;
    const double* __restrict__ coef = p.coef + I.rule_off;
    const double* __restrict__ d0p = p.d + I.d_off;
    const double* __restrict__ d1p = d0p + I.dstride;
    double r[2][NPL], w[2][NPL], h[2][NPL];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int q = 0; q < NPL; ++q) {
            const int j = lane + LPM * q;
            const bool ok = j < np;
            r[k][q] = ok ? ratio[k * np + j] : 0.0;
            w[k][q] = ok ? coef[k * np + j] : 0.0;
            h[k][q] = 0.0;
        }
    const double dw0 = (lane < L - 1) ? d0p[lane + 1] : 0.0;
    const double dw1 = (lane < L - 1) ? d1p[lane + 1] : 0.0;
    const double* __restrict__ g0 = p.g0 + 2 * I.mode_off;
    const double g00 = g0[mode], g01 = g0[M + mode];
    // the problem's constants in registers (the loop reads no table entry)
    const int64_t N = I.N;
    const bool bdf2 = I.scheme == 2;
    const double inv_tau = I.inv_tau, ca = I.a;
    // ring[i] = g^{n-1-i} (lane i of the group) at the start of step n
    double ring0 = (lane == 0) ? g00 : 0.0, ring1 = (lane == 0) ? g01 : 0.0;
    // g^{n-1} and g^{n-2} (g^{-1} := g^0), the same in every lane of a group
    double gm10 = g00, gm11 = g01, gm20 = g00, gm21 = g01;
    const double lam = p.lam[I.mode_off + mode];
    const double L1 = ca + lam;
    const double m11 = I.c + I.d00 * L1, m22 = I.c + I.d01 * L1;
    const double m12 = -ca * I.d01, m21 = -ca * I.d00;
    const double idet = 1.0 / (m11 * m22 - m12 * m21);
    const int src_in = (threadIdx.x & ~(LPM - 1) & 63) + L - 2;  // lane of g^{n+1-L} at step n (L >= 2)
    // BDF2 starting correction of step n, 1/2 d_{k,n-1} g_k^0; the weight of
    // the next step is loaded one step ahead
    double cr0 = bdf2 ? 0.5 * d0p[0] * g00 : 0.0, cr1 = bdf2 ? 0.5 * d1p[0] * g01 : 0.0;
    double gin0 = 0.0, gin1 = 0.0;  // g^{n-L} (zero while n < L + 1)
    for (int64_t n = 1; n <= N; ++n) {
        const int64_t nx = n < N ? n : N;
        const double dn0 = d0p[nx], dn1 = d1p[nx];
        // the level entering the state at step n+1 (taken before the shift)
        const double gnext0 = __shfl(ring0, src_in, 64), gnext1 = __shfl(ring1, src_in, 64);
        double p0 = 0.0, p1 = 0.0;
#pragma unroll
        for (int q = 0; q < NPL; ++q) {
            h[0][q] = fma(r[0][q], h[0][q], gin0);
            h[1][q] = fma(r[1][q], h[1][q], gin1);
            p0 = fma(w[0][q], h[0][q], p0);
            p1 = fma(w[1][q], h[1][q], p1);
        }
        // exact-weight window: lags 1..min(L-1, n-1)
        const bool win = lane < ((n - 1 < L - 1) ? n - 1 : L - 1);
        p0 = fma(win ? dw0 : 0.0, ring0, p0);
        p1 = fma(win ? dw1 : 0.0, ring1, p1);
        const double S0 = group_sum<LPM>(p0) + cr0;
        const double S1 = group_sum<LPM>(p1) + cr1;
        const double E0 = (bdf2 ? 2.0 * gm10 - 0.5 * gm20 : gm10) * inv_tau;
        const double E1 = (bdf2 ? 2.0 * gm11 - 0.5 * gm21 : gm11) * inv_tau;
        const double r0 = E0 - (L1 * S0 - ca * S1);
        const double r1 = E1 - (L1 * S1 - ca * S0);
        const double gn0 = (m22 * r0 - m12 * r1) * idet;
        const double gn1 = (m11 * r1 - m21 * r0) * idet;
        // levels move up one lane (DPP wave_shr:1; a group's lane 0 takes the new level)
        const double up0 = dpp_move<0x138, 0xF>(ring0), up1 = dpp_move<0x138, 0xF>(ring1);
        ring0 = (lane == 0) ? gn0 : up0;
        ring1 = (lane == 0) ? gn1 : up1;
        gm20 = gm10;
        gm21 = gm11;
        gm10 = gn0;
        gm11 = gn1;
        const bool enter = n + 1 >= L + 1;
        gin0 = enter ? gnext0 : 0.0;
        gin1 = enter ? gnext1 : 0.0;
        cr0 = bdf2 ? 0.5 * dn0 * g00 : 0.0;
        cr1 = bdf2 ? 0.5 * dn1 * g01 : 0.0;
    }
    if (lane == 0) {
        double* gN = p.gN + 2 * I.mode_off;
        gN[mode] = ring0;
        gN[M + mode] = ring1;
    }
}

// Batched fast solve, time-blocked: one wave per mode, lanes 0..31 hold
// component 0 and lanes 32..63 component 1 (lane l: component k = l/32,
// position t = l%32). The steps go in blocks of bt <= L (the lag): the
// levels entering the compressed state at steps n0+1..n0+bt are
// g^{n0+1-L}..g^{n0+bt-L}, all known when the block starts, so
//  (A) the state advances over the whole block first: each lane owns the
//      nodes t + 32q of its component (NP nodes), and per step it adds its
//      part of sum_j w_j h_j into a[] (no cross-lane work per step);
//  (B) the partial sums of 8 steps are summed over the 32 lanes of a
//      component by recursive halving (pairs by DPP row_half_mirror and
//      quad_perm; each stage keeps half of the values and adds the
//      partner's copy of that half; then the lanes t^8 and t^16, which hold
//      the same step, are added in), which leaves step t's fast part in
//      lane t of its component;
//  (C) the window (exact weights, lags 1..L-1) and the 2x2 solve then run
//      step by step in push form with lane t owning step n0+1+t: the levels
//      before the block are pushed first, and each new level is pushed into
//      the later steps' sums, so a step reads its sum (readlane), solves, and
//      adds one FMA per lane.
// lv: lane 32k+t holds g_k^{n0-t} (zero for levels < 1); wc: lane 32k+t holds
// d_{k,t-b} at step b (zero outside lags 1..L-1); lvnew: lane 32k+b holds
// the block's level of step b. Needs 2 <= L <= 32 and np <= 32*NP.
// Window weight tables of tb_steps in LDS: per wave and component kWinTab
// entries, tab[m] = d_{k,m-32} for 1 <= m-32 <= L-1 and 0 elsewhere, so that
// the push weight d_{k,t-b} of step b and the weight d_{k,t+1+u} of a level
// before the block are plain reads at offsets from a per-lane base. Each wave
// writes and reads only its own table (a wave's LDS operations complete in
// order: wave-scope fences order the writes before the reads).
constexpr int kWinTab = 128;
__device__ __forceinline__ const double* tb_window_table(double* tab, const double* dk, int L, int lane) {
    const int t = lane & 31;
    double* tk = tab + (lane >> 5) * kWinTab;
#pragma unroll
    for (int q = 0; q < kWinTab / 32; ++q) {
        const int lag = t + 32 * q - 32;
        tk[t + 32 * q] = (lag >= 1 && lag <= L - 1) ? dk[lag] : 0.0;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    return tk;
}

// The time-blocked steps nbeg+1..nend of one mode (one wave; lanes 0..31
// component 0, 32..63 component 1, lane l: component k = l/32, position
// t = l%32). The steps go in blocks of bt <= L (the lag): the levels
// entering the compressed state at steps n0+1..n0+bt are g^{n0+1-L}..
// g^{n0+bt-L}, all known when the block starts, so
//  (A) the state advances over the whole block first: each lane owns the
//      nodes t + 32q of its component (NP nodes), and per step it adds its
//      part of sum_j w_j h_j into a[] (no cross-lane work per step);
//  (B) the partial sums of 8 steps are summed over the 32 lanes of a
//      component by recursive halving, which leaves step t's fast part in
//      lane t of its component;
//  (C) the window (exact weights, lags 1..L-1) and the 2x2 solve then run
//      step by step in push form with lane t owning step n0+1+t: the levels
//      before the block are pushed first, and each new level is pushed into
//      the later steps' sums, so a step reads its sum (readlane), solves, and
//      adds one FMA per lane. When the next block is full too, its (A) runs
//      inside these steps.
// Blocks start at nbeg + jL and take min(L, ntot - start) steps; a call may
// end inside a block (nend), after whose steps the rest of the block is not
// taken. The fast part of a block is always formed for its whole length, so
// the arithmetic of every step depends on the block alone, not on where the
// calls end. State in and out: h (this lane's nodes, at the start of the
// block that holds step nend+1: when nend falls inside a block, h as it was
// before that block's state pass is written to hsave (row stride hrow, nodes
// j < np) and e_end receives the steps taken of it, else e_end = 0); lv
// (lane 32k+t: g_k^{s-t}, zero for levels < 1, s the start of that block);
// lvnew_out (lane 32k+j: the block's level of step j < e_end); P = Minv g^n,
// R = Minv g^{n-1}, gl = g^n. dk: this component's exact weights, readable up
// to dlast; wt: this wave's table of them for this lane's component in LDS,
// wt[m] = d_{k,m-32} for 1 <= m-32 <= L-1 and 0 elsewhere, m < kWinTab
// (tb_window_table). Needs 2 <= L <= 32, np <= 32*NP.
template <int NP>
__device__ __forceinline__ void tb_steps(const int lane, const int L, const bool bdf2, const int64_t nbeg,
                                         const int64_t nend, const int64_t ntot, double* __restrict__ hsave,
                                         const int64_t hrow, const int np, int& e_end, double& lvnew_out,
                                         const double (&r_)[NP], const double (&w_)[NP],
                                         double (&h_)[NP], const double* __restrict__ dk, const int64_t dlast,
                                         const double* wt, const double g0k, const double e1, const double e2,
                                         const double s00, const double s01, const double s10, const double s11,
                                         const double i00, const double i01, const double i10, const double i11,
                                         double& P0_, double& P1_, double& R0_, double& R1_, double& gl0_,
                                         double& gl1_, double& lv_) {
    double P0 = P0_, P1 = P1_, R0 = R0_, R1 = R1_, gl0 = gl0_, gl1 = gl1_, lv = lv_;
    double r[NP], w[NP], h[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        r[q] = r_[q];
        w[q] = w_[q];
        h[q] = h_[q];
    }
    const int t = lane & 31;
    const bool hi_half = (lane & 32) != 0;
    const int src0 = (lane & 32) + L - 1;  // lane of g_k^{n0+1-L} in lv
    // (B) sum of 8 steps' partial sums over a component's 32 lanes:
    // a[pos(j)] holds step b0+j (pos swaps bits 0 and 1 of j); halving by
    // row_half_mirror (side bit 2), quad_perm [1,0,3,2] (bit 0) and
    // quad_perm [2,3,0,1] (bit 1) leaves step b0 + t%8 in lane t, and the
    // lanes t^8 and t^16, which hold the same step, are added in; lanes of
    // those eight steps take the total.
    auto reduce8 = [&](double (&a)[8], int b0, double& dst) {
        {
            const bool sd = (lane >> 2) & 1;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const double keep = sd ? a[4 + i] : a[i], send = sd ? a[i] : a[4 + i];
                a[i] = keep + dpp_move<0x141, 0xF>(send);
            }
        }
        {
            const bool sd = lane & 1;
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const double keep = sd ? a[2 + i] : a[i], send = sd ? a[i] : a[2 + i];
                a[i] = keep + dpp_move<0xB1, 0xF>(send);
            }
        }
        double v;
        {
            const bool sd = (lane >> 1) & 1;
            const double keep = sd ? a[1] : a[0], send = sd ? a[0] : a[1];
            v = keep + dpp_move<0x4E, 0xF>(send);
        }
        v += __shfl_xor(v, 8, 64);
        v += __shfl_xor(v, 16, 64);
        if ((t >> 3) == (b0 >> 3)) dst = v;
    };
    constexpr int POS[8] = {0, 2, 1, 3, 4, 6, 5, 7};
    // (C) one step of the block (lane t holds the pending sum of step
    // n0+1+t): with Minv the inverse of the step matrix, g^n = Minv (E - D S):
    // the E part is e1 P + e2 R with P = Minv g^{n-1} and R = Minv g^{n-2},
    // the S part s.S, so a step waits on its sum and two FMAs. Each lane
    // evaluates its own component (the coefficients of its row of Minv and
    // of s) and reads the other component's new value from its half
    // (readlane), which takes fewer instructions than both rows in every
    // lane and gives the same values. wc: the push weight of step b for this
    // lane's step, d_{k,t-b}, read from the LDS table. Returns this lane's
    // component of the new level.
    const double sk0 = hi_half ? s10 : s00, sk1 = hi_half ? s11 : s01;
    const double ik0 = hi_half ? i10 : i00, ik1 = hi_half ? i11 : i01;
    double Pk = hi_half ? P1 : P0, Rk = hi_half ? R1 : R0;
    double acc = 0.0, lvnew = 0.0;
    auto cstep = [&](int b, double wc) {
        const double S0 = lane_value(acc, b), S1 = lane_value(acc, 32 + b);
        const double Ek = fma(e1, Pk, e2 * Rk);
        const double gk = fma(sk1, S1, fma(sk0, S0, Ek));
        acc = fma(wc, gk, acc);
        lvnew = (t == b) ? gk : lvnew;
        const double gn0 = lane_value(gk, 0), gn1 = lane_value(gk, 32);
        Rk = Pk;
        Pk = fma(ik1, gn1, ik0 * gn0);
        gl0 = gn0;
        gl1 = gn1;
        return gk;
    };
    // (A) the state advanced by one step with input gin, this lane's part of
    // sum_j w_j h_j
    auto astep = [&](double gin) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            h[q] = fma(r[q], h[q], gin);
            s = fma(w[q], h[q], s);
        }
        return s;
    };
    bool have_fast = false;  // acc holds the block's fast part already
    e_end = 0;
    for (int64_t n0 = nbeg; n0 < nend; n0 += L) {
        const int bt = int((ntot - n0 < L) ? ntot - n0 : L);     // the block's length
        const int bc = int((nend - n0 < bt) ? nend - n0 : bt);   // its steps taken here
        if (bc < bt && hsave) {
            // the call ends inside this block: keep the state of its start
#pragma unroll
            for (int q = 0; q < NP; ++q)
                if ((lane & 31) + 32 * q < np) hsave[int64_t((lane & 31) + 32 * q) * hrow] = h[q];
        }
        if (!have_fast) {
            // (A) + (B) from the level store, 8 steps at a time; a full pass
            // has no per-step branch, so its eight level loads are all in
            // flight first
            acc = 0.0;
            auto pass = [&](auto full_t, int b0) {
                constexpr bool FULLP = decltype(full_t)::value;
                double gin[8], a[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int b = b0 + j;
                    gin[j] = __shfl(lv, b < L ? src0 - b : 0, 64);
                }
#pragma unroll
                for (int j = 0; j < 8; ++j) a[POS[j]] = (FULLP || b0 + j < bt) ? astep(gin[j]) : 0.0;
                reduce8(a, b0, acc);
            };
#pragma unroll 1
            for (int b0 = 0; b0 < bt; b0 += 8) {
                if (b0 + 8 <= bt)
                    pass(std::true_type{}, b0);
                else
                    pass(std::false_type{}, b0);
            }
        }
        // BDF2 starting correction 1/2 d_{k,n-1} g_k^0 of step n = n0+1+t
        if (bdf2) {
            const int64_t ix = (n0 + t <= dlast) ? n0 + t : dlast;
            acc = fma(0.5 * dk[ix], g0k, acc);
        }
        // (C) window part of the levels before the block: level n0-u reaches
        // step n0+1+t at lag t+1+u (groups of 8 levels; the weights of lags
        // >= L are zero, so the last group may run past L-1)
        {
            for (int u0 = 0; u0 + 1 < L; u0 += 8) {
                const double* wu = wt + 33 + t + u0;  // lane t, level n0-u: d_{k,t+1+u}
                double g[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) g[u] = __shfl(lv, (lane & 32) + ((u0 + u) & 31), 64);
#pragma unroll
                for (int u = 0; u < 8; ++u) acc = fma(wu[u], g[u], acc);
            }
        }
        // (C) the steps. When this block and the next are full, the next
        // block's state pass rides along: its step b takes the level just
        // solved at step b (lag L), so its FMAs fill the solve's dependency
        // chain, 8 steps per group (the group count fixed at compile time,
        // a remainder group of 1..7 steps).
        lvnew = 0.0;
        const bool pipe = bc == L && ntot - (n0 + L) >= L && nend - (n0 + L) >= L;
        if (pipe) {
            double accn = 0.0;
            auto group = [&](auto rc, int c0) {
                constexpr int RC = decltype(rc)::value;
                const double* wg = wt + 25 + t - c0;  // step c0+j: d_{k,t-c0-j} at wg[7-j]
                double a[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) a[POS[j]] = (j < RC) ? astep(cstep(c0 + j, wg[7 - j])) : 0.0;
                reduce8(a, c0, accn);
            };
            int c0 = 0;
#pragma unroll 1
            for (; c0 + 8 <= bt; c0 += 8) group(std::integral_constant<int, 8>{}, c0);
            switch (bt - c0) {
                case 1: group(std::integral_constant<int, 1>{}, c0); break;
                case 2: group(std::integral_constant<int, 2>{}, c0); break;
                case 3: group(std::integral_constant<int, 3>{}, c0); break;
                case 4: group(std::integral_constant<int, 4>{}, c0); break;
                case 5: group(std::integral_constant<int, 5>{}, c0); break;
                case 6: group(std::integral_constant<int, 6>{}, c0); break;
                case 7: group(std::integral_constant<int, 7>{}, c0); break;
                default: break;
            }
            acc = accn;
        } else {
            for (int b = 0; b < bc; ++b) cstep(b, wt[32 + t - b]);
        }
        have_fast = pipe;
        if (bc < bt) {  // the call ends inside this block (the last of the loop)
            e_end = bc;
            lvnew_out = lvnew;
            break;
        }
        // level store for the next block: lane 32k+t <- g_k^{n0+bt-t}
        {
            const double fresh = __shfl(lvnew, (lane & 32) + ((bt - 1 - t) & 31), 64);
            const double older = __shfl(lv, (lane & 32) + ((t - bt) & 31), 64);
            lv = (t < bt) ? fresh : older;
        }
    }
#pragma unroll
    for (int q = 0; q < NP; ++q) h_[q] = h[q];
    P0_ = lane_value(Pk, 0);
    P1_ = lane_value(Pk, 32);
    R0_ = lane_value(Rk, 0);
    R1_ = lane_value(Rk, 32);
    gl0_ = gl0;
    gl1_ = gl1;
    lv_ = lv;
}

// Batched fast solve, time-blocked (tb_steps): one wave per mode, from the
// zero state over all N steps of the mode's problem.
template <int NP>
__global__ __launch_bounds__(256) void k_modal_batch_tb(BatchArgs p) {
    const int lane = threadIdx.x & 63;
    const int64_t group = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (group >= p.total) return;  // uniform per wave
    int lo = 0, hi = p.count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (p.cum[mid] <= group) lo = mid; else hi = mid - 1;
    }
    const BatchInst& I = p.inst[p.list[lo]];
    const int64_t mode = group - p.cum[lo];
    const int64_t M = I.M, N = I.N;
    const int np = I.np, L = I.L;
    const int k = lane >> 5, t = lane & 31;
    const bool hi_half = k != 0;
    const double* __restrict__ ratio = p.ratio + I.rule_off + k * np;
    const double* __restrict__ coef = p.coef + I.rule_off + k * np;
    const double* __restrict__ dk = p.d + I.d_off + k * I.dstride;
    double r[NP], w[NP], h[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        const int j = t + 32 * q;
        const bool ok = j < np;
        r[q] = ok ? ratio[j] : 0.0;
        w[q] = ok ? coef[j] : 0.0;
        h[q] = 0.0;
    }
    // window weights of this wave, d_{k,1..L-1}, in its LDS table
    __shared__ double wtab[4][2 * kWinTab];
    const double* wt = tb_window_table(wtab[threadIdx.x >> 6], dk, L, lane);
    const double* __restrict__ g0 = p.g0 + 2 * I.mode_off;
    const double g00 = g0[mode], g01 = g0[M + mode];
    const double g0k = hi_half ? g01 : g00;
    const bool bdf2 = I.scheme == 2;
    const double inv_tau = I.inv_tau, ca = I.a;
    const double lam = p.lam[I.mode_off + mode];
    const double L1 = ca + lam;
    const double m11 = I.c + I.d00 * L1, m22 = I.c + I.d01 * L1;
    const double m12 = -ca * I.d01, m21 = -ca * I.d00;
    const double idet = 1.0 / (m11 * m22 - m12 * m21);
    const double i00 = m22 * idet, i01 = -m12 * idet, i10 = -m21 * idet, i11 = m11 * idet;
    // g = Minv (E - D S), D = [[L1, -a], [-a, L1]]: coefficients of S
    const double s00 = ca * i01 - L1 * i00, s01 = ca * i00 - L1 * i01;
    const double s10 = ca * i11 - L1 * i10, s11 = ca * i10 - L1 * i11;
    // E = e1 g^{n-1} + e2 g^{n-2} (BE: g^{n-1}/tau; BDF2: (2 g^{n-1} - g^{n-2}/2)/tau)
    const double e1 = (bdf2 ? 2.0 : 1.0) * inv_tau, e2 = (bdf2 ? -0.5 : 0.0) * inv_tau;
    double P0 = fma(i01, g01, i00 * g00), P1 = fma(i11, g01, i10 * g00);  // Minv g^{n-1}
    double R0 = P0, R1 = P1;                                              // Minv g^{n-2}, g^{-1} := g^0
    double gl0 = g00, gl1 = g01;                                          // newest level
    double lv = 0.0;                                                      // no level >= 1 yet
    int e_end;
    double lvnew;
    tb_steps<NP>(lane, L, bdf2, 0, N, N, nullptr, 0, np, e_end, lvnew, r, w, h, dk, N, wt, g0k, e1, e2, s00, s01,
                 s10, s11, i00, i01, i10, i11, P0, P1, R0, R1, gl0, gl1, lv);
    if (lane == 0) {
        double* gN = p.gN + 2 * I.mode_off;
        gN[mode] = gl0;
        gN[M + mode] = gl1;
    }
}

// Fast form for few modes, time-blocked (tb_steps): one wave per mode runs
// the steps n0+1..n0+nsteps. Its blocks are [jL, jL+L) of the whole run, so
// a call that starts inside a block takes that block again from its start
// (the same arithmetic, so the same levels) and the results do not depend
// on how the run is cut into calls. State between calls: H = the state at
// the start of the block that holds step n+1; ring2[i] = g^{n-i} for
// n-i >= 0 (g^0 included), i < 2L.
template <int NP>
__global__ __launch_bounds__(256) void k_modal_fast_tb(ModalFastArgs p) {
    const int lane = threadIdx.x & 63;
    const int64_t mode = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (mode >= p.M) return;  // uniform per wave
    const int64_t M = p.M, twoM = 2 * M;
    const int np = p.np, L = p.L;
    const int k = lane >> 5, t = lane & 31;
    const double* __restrict__ ratio = p.ratio + k * np;
    const double* __restrict__ coef = p.coef + k * np;
    const double* __restrict__ dk = p.d + int64_t(k) * p.dstride;
    double* __restrict__ H = p.H + int64_t(k) * np * p.hstride + mode;
    double r[NP], w[NP], h[NP];
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        const int j = t + 32 * q;
        const bool ok = j < np;
        r[q] = ok ? ratio[j] : 0.0;
        w[q] = ok ? coef[j] : 0.0;
        h[q] = ok ? H[int64_t(j) * p.hstride] : 0.0;
    }
    __shared__ double wtab[4][2 * kWinTab];
    const double* wt = tb_window_table(wtab[threadIdx.x >> 6], dk, L, lane);
    const double g00 = p.g0[mode], g01 = p.g0[M + mode];
    const double g0k = k ? g01 : g00;
    const bool bdf2 = p.scheme == 2;
    const double ca = p.a, lam = p.lam[mode];
    const double L1 = ca + lam;
    const double m11 = p.c + p.d0[0] * L1, m22 = p.c + p.d0[1] * L1;
    const double m12 = -ca * p.d0[1], m21 = -ca * p.d0[0];
    const double idet = 1.0 / (m11 * m22 - m12 * m21);
    const double i00 = m22 * idet, i01 = -m12 * idet, i10 = -m21 * idet, i11 = m11 * idet;
    const double s00 = ca * i01 - L1 * i00, s01 = ca * i00 - L1 * i01;
    const double s10 = ca * i11 - L1 * i10, s11 = ca * i10 - L1 * i11;
    const double e1 = (bdf2 ? 2.0 : 1.0) * p.inv_tau, e2 = (bdf2 ? -0.5 : 0.0) * p.inv_tau;
    // the start of the block that holds step n+1, its levels before it
    const int64_t n = p.n0, ks = (n / L) * L, b = n - ks;
    double* __restrict__ ring = p.ring + mode;
    double lv = (t < L && ks - t >= 1) ? ring[(b + t) * twoM + k * M] : 0.0;
    const double gm10 = ring[b * twoM], gm11 = ring[b * twoM + M];  // g^{ks} (g^0 at ks = 0)
    const double gm20 = ks >= 1 ? ring[(b + 1) * twoM] : g00, gm21 = ks >= 1 ? ring[(b + 1) * twoM + M] : g01;
    double P0 = fma(i01, gm11, i00 * gm10), P1 = fma(i11, gm11, i10 * gm10);
    double R0 = fma(i01, gm21, i00 * gm20), R1 = fma(i11, gm21, i10 * gm20);
    double gl0 = gm10, gl1 = gm11;
    const int64_t nend = n + p.nsteps;
    int e_end;
    double lvnew = 0.0;
    tb_steps<NP>(lane, L, bdf2, ks, nend, p.N, H, p.hstride, np, e_end, lvnew, r, w, h, dk, p.dstride - 1, wt,
                 g0k, e1, e2, s00, s01, s10, s11, i00, i01, i10, i11, P0, P1, R0, R1, gl0, gl1, lv);
    if (e_end == 0) {  // ended on a block boundary: h is the next block's starting state
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const int j = t + 32 * q;
            if (j < np) H[int64_t(j) * p.hstride] = h[q];
        }
    }
    // ring2[i] = g^{nend-i}: the block's levels taken so far (lvnew, newest
    // first), then the levels before the block (lv); g^0 itself at level 0
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        const int i = t + 32 * half;
        const int inew = e_end - 1 - i, iold = i - e_end;
        const double vnew = __shfl(lvnew, (lane & 32) + (inew & 31), 64);
        const double vold = __shfl(lv, (lane & 32) + (iold & 31), 64);
        const int64_t l = nend - i;
        const double v = l == 0 ? g0k : (l < 0 ? 0.0 : (inew >= 0 ? vnew : (iold < 32 ? vold : 0.0)));
        if (i < 2 * L) ring[int64_t(i) * twoM + k * M] = v;
    }
}

// Exchange of a double between the two lanes of a pair (lane ^ 1) with a
// DPP quad permutation [1,0,3,2] on each 32-bit half.
__device__ __forceinline__ double pair_swap(double x) {
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, int(v & 0xffffffffll), 0xB1, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, int(v >> 32), 0xB1, 0xF, 0xF, false);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// Fast form for many modes: the compressed state streams through
// k_hist_block (time-blocked, exactly as for the nodal solver, here on the
// sine coefficients), and this kernel takes the bt <= 32 steps of the block.
// A lane pair owns one mode, lane k of the pair component k. The history
// sum of step n is
//   S_k^n = Sf[n - nblk][k]                         (lags >= L, fast part)
//         + sum_{i=1}^{min(L-1, n-1)} d_{k,i} g_k^{n-i}   (exact window),
// accumulated in push form as in the direct near field: the window part of
// the levels before this launch is added first (from the level store, slot
// l mod Lr), and each new level is pushed into the later steps of the
// launch, so a step waits on one FMA and the loop makes no global loads.
// The 2x2 solve and the adjoint variant (ADJ) are those of k_modal_near.
template <bool ADJ>
__global__ __launch_bounds__(64) void k_modal_win(ModalWinArgs p) {
    constexpr int BB = 32;
    __shared__ double wd[2 * (BB + 1)];  // window weights d_{k,1..L-1}, zero beyond
    for (int e = threadIdx.x; e < 2 * BB; e += 64) {
        const int kk = e / BB, i = e % BB;
        wd[kk * (BB + 1) + i] = (i >= 1 && i < p.L) ? p.d[int64_t(kk) * p.dstride + i] : 0.0;
    }
    __syncthreads();
    const int64_t gid = int64_t(blockIdx.x) * 64 + threadIdx.x;
    const int64_t mode = gid >> 1;
    const int k = int(gid & 1);
    if (mode >= p.M) return;  // both lanes of a pair leave together
    const double* __restrict__ w = wd + k * (BB + 1);
    const int64_t M = p.M, twoM = 2 * M;
    const double lam = p.lam[mode];
    const double g0k = p.g0[k * M + mode];
    const double L1 = p.a + lam;
    const double m11 = p.c + p.d0[0] * L1, m22 = p.c + p.d0[1] * L1;
    const double m12 = -p.a * p.d0[1], m21 = -p.a * p.d0[0];
    const double idet = 1.0 / (m11 * m22 - m12 * m21);
    const double i00 = m22 * idet, i01 = -m12 * idet, i10 = -m21 * idet, i11 = m11 * idet;
    const double c_own = k ? i11 : i00;
    const double c_part = k ? i01 : i10;
    const double u = p.a * (k ? i10 : i01) - L1 * c_own;
    const double x = c_part;
    const double y = p.a * (k ? i00 : i11) - L1 * c_part;
    const double t_part = k ? i10 : i01;
    const double et = p.inv_tau;
    double* __restrict__ lv = p.levels + k * M + mode;
    const double* __restrict__ dk = p.d + int64_t(k) * p.dstride;
    const int64_t b0 = p.nfirst - p.nblk;
    const int bt = p.bt;
    // Prologue loads are unconditional (clamped, valid addresses; at most one
    // uniform branch around a group) so that they are all in flight at once.
    double acc[BB];
#pragma unroll
    for (int b = 0; b < BB; ++b) {
        const int64_t r = (b0 + b < p.BT) ? b0 + b : p.BT - 1;  // rows past the block are not used
        acc[b] = p.Sf[(r * 2 + k) * M + mode];
    }
    if (!ADJ && p.scheme == 2) {
#pragma unroll
        for (int b = 0; b < BB; ++b) acc[b] = fma(0.5 * dk[p.nfirst + b - 1], g0k, acc[b]);
    }
    if (ADJ && p.nfirst == 1) acc[0] -= p.gc[k * M + mode];  // cotangent enters step 1
    // window part of the levels l = nfirst-j (j < L, l >= 1) already taken:
    // all loads first (an absent level reads level nfirst-1, which every
    // level store holds and is finite, times 0), then the sums
    {
        double old[BB];
        const int64_t sl1 = (p.nfirst - 1) % p.Lr;  // slot of level nfirst-1
        int64_t sl = sl1;
#pragma unroll
        for (int j = 1; j < BB; ++j) {
            const bool ok = j < p.L && p.nfirst - j >= 1;
            old[j] = lv[(ok ? sl : sl1) * twoM] * (ok ? 1.0 : 0.0);
            sl = (sl == 0) ? p.Lr - 1 : sl - 1;
        }
#pragma unroll
        for (int j = 1; j < BB; ++j)
#pragma unroll
            for (int b = 0; b + j < BB; ++b) acc[b] = fma(w[b + j], old[j], acc[b]);  // b >= bt unused
    }
    // variables of the time difference: levels (forward; level -1 reads as
    // level 0) or mu (adjoint; row 0 of mu is zero and stands for mu^0 and
    // mu^{-1}); unconditional loads, like those above
    double gm1, gm2;
    const int64_t nm2 = (p.nfirst >= 2) ? p.nfirst - 2 : 0;
    if (ADJ) {
        const double* __restrict__ mv = p.mu + k * M + mode;
        gm1 = mv[(p.nfirst - 1) * twoM];
        gm2 = mv[nm2 * twoM];
    } else {
        gm1 = lv[((p.nfirst - 1) % p.Lr) * twoM];
        gm2 = lv[(nm2 % p.Lr) * twoM];
    }
    const bool bdf2 = p.scheme == 2;
    const double w1 = w[1];
    double wr[BB - 2];
#pragma unroll
    for (int i = 0; i < BB - 2; ++i) wr[i] = w[i + 2];
    int64_t slot = p.nfirst % p.Lr;
    double gprev = 0.0;
    // every prologue load has landed: the steps below are separate blocks
    // (b < bt), and without this wait the compiler waits for all memory
    // operations, the previous step's stores included, at each step
    __builtin_amdgcn_s_waitcnt(0);
#pragma unroll
    for (int b = 0; b < BB; ++b) {
        if (b < bt) {
            __builtin_amdgcn_sched_barrier(0);
            const int64_t n = p.nfirst + b;
            double S = acc[b];
            if (b > 0) S = fma(w1, gprev, S);
            const double E = bdf2 ? (2.0 * gm1 - 0.5 * gm2) * et : gm1 * et;
            double lev, e_new;
            if (ADJ) {
                const double r = E - S;
                const double P = c_own * r, Q = t_part * r;
                const double A = L1 * P - p.a * Q, Bv = L1 * Q - p.a * P;
                e_new = P + pair_swap(Q);
                lev = A + pair_swap(Bv);
                p.mu[n * twoM + k * M + mode] = e_new;
            } else {
                const double Q = fma(y, S, x * E);
                const double P = fma(u, S, c_own * E);
                lev = P + pair_swap(Q);
                e_new = lev;
                p.Sout[n * p.sstride + k * M + mode] = S;
            }
            lv[slot * twoM] = lev;
            slot = (slot + 1 == p.Lr) ? 0 : slot + 1;
            if (b > 0) {
#pragma unroll
                for (int bb = b + 1; bb < BB; ++bb) acc[bb] = fma(wr[bb - b - 1], gprev, acc[bb]);
            }
            gprev = lev;
            gm2 = gm1;
            gm1 = e_new;
        }
    }
}

// Direct form, part of one time block: the steps n = nfirst .. nfirst+bt-1
// (inside the block n0+1 .. n0+B) in order. A lane pair owns one mode, lane
// k of the pair component k. The history sum of step n0+1+b is
//   S_k[b] = F[b][k] (far field of the block, summed over the K-split by
//            k_reduce_far) + sum_{j<b} d_{k,b-j} g_k^{n0+1+j},
// accumulated in push form: acc[b] starts as the far field (plus BDF2's
// starting correction 1/2 d_{k,n-1} g_k^0) and each level is added into the
// pending sums of all later steps of the block, so a step waits on one FMA
// only and the loop makes no global loads. Steps are
// unrolled so that acc[] stays in registers. The 2x2 solve is split by
// lanes: g_k = P_k + Q_{k'}, where P_k = c_own E_k + u S_k is the lane's own
// part and Q_k = x E_k + y S_k its part of the partner's value, so a step
// exchanges one double. FULL is the whole-block case without per-step
// guards; otherwise a run that resumes inside a block first pushes the
// block's earlier levels from memory.
template <int BB, bool FULL, bool ADJ>
__global__ __launch_bounds__(64) void k_modal_near(ModalNearArgs p) {
    // weights d_{k,0..BB-1} in LDS; the component rows are BB+1 apart so
    // that the two components of a lane pair read different banks
    __shared__ double wd[2 * (BB + 1)];
    for (int e = threadIdx.x; e < 2 * BB; e += 64) {
        const int kk = e / BB, i = e % BB;
        wd[kk * (BB + 1) + i] = (i >= 1 && i < p.dstride) ? p.d[int64_t(kk) * p.dstride + i] : 0.0;
    }
    __syncthreads();
    const int64_t gid = int64_t(blockIdx.x) * 64 + threadIdx.x;
    const int64_t mode = gid >> 1;
    const int k = int(gid & 1);
    if (mode >= p.M) return;  // both lanes of a pair leave together
    const double* __restrict__ w = wd + k * (BB + 1);
    const int64_t M = p.M, twoM = 2 * M;
    const double lam = p.lam[mode];
    const double g0k = p.g0[k * M + mode];
    const double L1 = p.a + lam;
    const double m11 = p.c + p.d0[0] * L1, m22 = p.c + p.d0[1] * L1;
    const double m12 = -p.a * p.d0[1], m21 = -p.a * p.d0[0];
    const double idet = 1.0 / (m11 * m22 - m12 * m21);
    const double i00 = m22 * idet, i01 = -m12 * idet, i10 = -m21 * idet, i11 = m11 * idet;
    const double c_own = k ? i11 : i00;  // Minv[k][k]
    // forward: g = Minv r with r_k = E_k - L1 S_k + a S_k'
    const double c_part = k ? i01 : i10;                   // Minv[k'][k]: weight of r_k in g_k'
    const double u = p.a * (k ? i10 : i01) - L1 * c_own;   // S_k in g_k (through r_k and r_k')
    const double x = c_part;
    const double y = p.a * (k ? i00 : i11) - L1 * c_part;  // S_k in g_k'
    // adjoint: mu = Minv^T r with r_k = E_k - S_k; r_k enters mu_k' with Minv[k][k']
    const double t_part = k ? i10 : i01;
    const double et = p.inv_tau;
    double* __restrict__ lv = p.levels + k * M + mode;
    const double* __restrict__ dk = p.d + int64_t(k) * p.dstride;
    const int b0 = int(p.nfirst - p.n0 - 1);  // first block offset taken here
    const int bend = b0 + p.bt;               // one past the last
    // Prologue loads are unconditional within one uniform branch per group
    // (all BB rows of F and F2 exist; the weights reach index n0+B-1 <
    // dstride), so they are all in flight at once; rows outside the launch
    // are not used.
    double acc[BB];
#pragma unroll
    for (int b = 0; b < BB; ++b) acc[b] = 0.0;
    if (p.F) {
#pragma unroll
        for (int b = 0; b < BB; ++b) acc[b] = p.F[(int64_t(b) * 2 + k) * M + mode];
    }
    if (p.F2) {
#pragma unroll
        for (int b = 0; b < BB; ++b) acc[b] += p.F2[(int64_t(b) * 2 + k) * M + mode];
    }
    if (!ADJ && p.scheme == 2) {
#pragma unroll
        for (int b = 0; b < BB; ++b) acc[b] = fma(0.5 * dk[p.n0 + b], g0k, acc[b]);
    }
    if (ADJ && p.n0 == 0 && b0 == 0) acc[0] -= p.gc[k * M + mode];  // cotangent enters step 1
    if (!FULL) {
        for (int j = 0; j < b0; ++j) {
            const double g = lv[(p.n0 + 1 + j) * twoM];
#pragma unroll
            for (int b = 1; b < BB; ++b)
                if (b >= b0 && b > j) acc[b] = fma(w[b - j], g, acc[b]);
        }
    }
    // variables of the time difference: levels (forward; level -1 reads as
    // level 0) or mu (adjoint; row 0 of mu is zero and stands for mu^0 and
    // mu^{-1})
    const double* __restrict__ ev = ADJ ? p.mu + k * M + mode : lv;
    double gm1 = ev[(p.nfirst - 1) * twoM];
    double gm2 = ev[((p.nfirst >= 2) ? p.nfirst - 2 : 0) * twoM];
    const bool bdf2 = p.scheme == 2;
    const double w1 = w[1];
    // the most used weights stay in registers, the rest are read from LDS
    constexpr int WR = 32;
    double wr[WR];
#pragma unroll
    for (int i = 0; i < WR; ++i) wr[i] = w[i + 2];
    // Step b adds the previous level with one FMA (the critical path) and
    // then pushes that level into the later sums; the barrier keeps each
    // step's instructions together so that the pushes overlap the solve
    // instead of being sunk into a serial chain before their use.
    double gprev = 0.0;
    __builtin_amdgcn_s_waitcnt(0);  // prologue loads landed (see k_modal_win)
#pragma unroll
    for (int b = 0; b < BB; ++b) {
        if (FULL || (b >= b0 && b < bend)) {
            __builtin_amdgcn_sched_barrier(0);
            const bool has_prev = FULL ? (b > 0) : (b > b0);
            double S = acc[b];
            if (has_prev) S = fma(w1, gprev, S);
            const double E = bdf2 ? (2.0 * gm1 - 0.5 * gm2) * et : gm1 * et;
            double lev, e_new;
            if (ADJ) {
                const double r = E - S;
                const double P = c_own * r, Q = t_part * r;
                const double A = L1 * P - p.a * Q, Bv = L1 * Q - p.a * P;
                e_new = P + pair_swap(Q);    // mu_k
                lev = A + pair_swap(Bv);     // psi_k = L1 mu_k - a mu_k'
                p.mu[(p.n0 + 1 + b) * twoM + k * M + mode] = e_new;
            } else {
                const double Q = fma(y, S, x * E);
                const double P = fma(u, S, c_own * E);
                lev = P + pair_swap(Q);
                e_new = lev;
                p.Sout[(p.n0 + 1 + b) * p.sstride + k * M + mode] = S;
            }
            lv[(p.n0 + 1 + b) * twoM] = lev;
            if (has_prev) {
#pragma unroll
                for (int bb = b + 1; bb < BB; ++bb) {
                    const int i = bb - b + 1;
                    acc[bb] = fma(i - 2 < WR ? wr[i - 2] : w[i], gprev, acc[bb]);
                }
            }
            gprev = lev;
            gm2 = gm1;
            gm1 = e_new;
        }
    }
}

// ---------------------------------------------------------------------------
// Gradient passes of the adjoint (modal coefficients). With the forward
// levels g^n, history sums S^n (with BDF2's starting correction), and the
// adjoint's mu^n, psi^n = Dm mu^n stored in reversed time (index N+1-n):
//   dl/dg^0 = mu^1/tau (BE),
//           = (3 mu^1 - mu^2)/(2 tau) - 1/2 sum_n d_{k,n-1} psi_k^n (BDF2),
//   dl/da   = -sum_n (mu_1^n - mu_2^n)(X_1^n - X_2^n),  X^n = d_0 g^n + S^n,
//   dl/dalpha_k = sum_n psi_k^n Y_k^n,
//   Y_k^n = sum_{l=1}^{n} dw_{k,n-l} g_k^l + [BDF2] 1/2 dd_{k,n-1} g_k^0,
// with dw, dd the beta-derivatives of the scheme's and the exact weights.

// 256-thread block sum in a fixed order (deterministic)
__device__ __forceinline__ double block_sum256(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int s = 128; s > 0; s >>= 1) {
        if (int(threadIdx.x) < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    return red[0];
}

// dl/dg^0, BDF2 part: partial sums over time chunks, one thread per
// (component, mode) and chunk: gpart[c][e] = sum_{n in chunk c} d_{k,n-1} psi_k^n
__global__ __launch_bounds__(256) void k_adj_g0_part(AdjGradArgs p) {
    const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (e >= 2 * p.M) return;
    const int64_t twoM = 2 * p.M, N = p.N;
    const int k = int(e / p.M);
    const int64_t per = p.per;
    const int64_t lo = 1 + int64_t(blockIdx.y) * per;
    const int64_t hi = (lo + per - 1 < N) ? lo + per - 1 : N;
    const double* __restrict__ dk = p.d + int64_t(k) * p.dstride;
    double s0 = 0.0, s1 = 0.0;
    int64_t n = lo;
    for (; n + 1 <= hi; n += 2) {
        s0 = fma(dk[n - 1], p.psi[(N + 1 - n) * twoM + e], s0);
        s1 = fma(dk[n], p.psi[(N - n) * twoM + e], s1);
    }
    if (n <= hi) s0 = fma(dk[n - 1], p.psi[(N + 1 - n) * twoM + e], s0);
    p.gpart[int64_t(blockIdx.y) * twoM + e] = s0 + s1;
}

// dl/dg^0 = mu^1/tau (BE) or (3 mu^1 - mu^2)/(2 tau) - 1/2 sum_c gpart[c] (BDF2)
__global__ __launch_bounds__(256) void k_adj_g0(AdjGradArgs p) {
    const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (e >= 2 * p.M) return;
    const int64_t twoM = 2 * p.M, N = p.N;
    const double mu1 = p.mu[N * twoM + e];
    if (p.scheme == 1) {
        p.gG0c[e] = mu1 * p.inv_tau;
        return;
    }
    const double mu2 = N >= 2 ? p.mu[(N - 1) * twoM + e] : 0.0;
    double sum = 0.0;
    for (int c = 0; c < p.nchunk; ++c) sum += p.gpart[int64_t(c) * twoM + e];
    p.gG0c[e] = (3.0 * mu1 - mu2) * (0.5 * p.inv_tau) - 0.5 * sum;
}

// sum_n (mu_1^n - mu_2^n)(X_1^n - X_2^n) over a time chunk: one thread per
// mode, a partial sum per block and chunk at part[chunk][block]
__global__ __launch_bounds__(256) void k_adj_da(AdjGradArgs p) {
    __shared__ double red[256];
    const int64_t mode = int64_t(blockIdx.x) * 256 + threadIdx.x;
    double acc0 = 0.0, acc1 = 0.0;
    if (mode < p.M) {
        const int64_t M = p.M, twoM = 2 * M, N = p.N;
        const int64_t per = p.per;
        const int64_t lo = 1 + int64_t(p.chunk0 + blockIdx.y) * per;
        const int64_t hi = (lo + per - 1 < N) ? lo + per - 1 : N;
        for (int64_t n = lo; n <= hi; ++n) {
            const int64_t t = n * twoM + mode, r = (N + 1 - n) * twoM + mode;
            const double X0 = fma(p.d0[0], p.traj[t], p.Sx[t]);
            const double X1 = fma(p.d0[1], p.traj[t + M], p.Sx[t + M]);
            if (n & 1)
                acc1 = fma(p.mu[r] - p.mu[r + M], X0 - X1, acc1);
            else
                acc0 = fma(p.mu[r] - p.mu[r + M], X0 - X1, acc0);
        }
    }
    const double tot = block_sum256(acc0 + acc1, red);
    if (threadIdx.x == 0) p.part[int64_t(p.chunk0 + blockIdx.y) * gridDim.x + blockIdx.x] = tot;
}

// d/dbeta over one time block: F holds the CQ sum of the weight derivatives
// over the levels l0..n of k_far_toeplitz (all levels, or those of the
// previous and the current block); add BDF2's starting correction and
// contract with psi. A
// workgroup covers 64 (component, mode) pairs; its kAdjBetaWaves waves take
// a slice of the block's steps each (a row of 64 F and psi values per wave
// and step, read coalesced; many waves keep enough loads in flight), and the
// partial sums meet in LDS in a fixed order.
__global__ __launch_bounds__(64 * kAdjBetaWaves) void k_adj_beta(AdjBetaArgs p) {
    __shared__ double red[kAdjBetaWaves - 1][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t M = p.M, twoM = 2 * M, N = p.N;
    const int64_t e = int64_t(blockIdx.x) * 64 + lane;
    const bool ein = e < twoM;
    const int64_t ec = ein ? e : twoM - 1;  // idle lanes read a valid column
    const int k = int(ec / M);
    const int64_t mode = ec - int64_t(k) * M;
    const double g0 = p.g0[ec];
    const double* __restrict__ ddk = p.dd + int64_t(k) * p.dstride;
    const int per = (p.bt + kAdjBetaWaves - 1) / kAdjBetaWaves;
    const int b0 = w * per, b1 = min(p.bt, b0 + per);
    double acc0 = 0.0, acc1 = 0.0;
#pragma unroll 4
    for (int b = b0; b < b1; ++b) {
        const int64_t n = p.n0 + 1 + b;
        double Y = p.F[(int64_t(b) * 2 + k) * M + mode];
        if (p.scheme == 2 && p.g0term) Y = fma(0.5 * ddk[n - 1], g0, Y);
        if (b & 1)
            acc1 = fma(p.psi[(N + 1 - n) * twoM + ec], Y, acc1);
        else
            acc0 = fma(p.psi[(N + 1 - n) * twoM + ec], Y, acc0);
    }
    const double v = acc0 + acc1;
    if (w) red[w - 1][lane] = v;
    __syncthreads();
    if (w == 0 && ein) {
        double t = v;
#pragma unroll
        for (int i = 0; i < kAdjBetaWaves - 1; ++i) t += red[i][lane];
        p.acc[e] += t;
    }
}

// ---------------------------------------------------------------------------
// d/dbeta in the frequency domain, block by block. With a_t = psi^{t+1},
// b_t = g^{t+1} and c = dw * b (c_t = Y^{t+1} without BDF2's g^0 term), cut
// the steps into nb blocks of Bk; block i of a and block j of b (i >= j)
// meet only through the lags (i-j) Bk + r, |r| < Bk, i.e. through the window
// w_d[r] = dw_{d Bk + r}, d = i - j. Zero-padded to P = 2 Bk points the
// circular correlation of the pair is the linear one, and Parseval gives
//   sum_t a_t c_t = (1/P) sum_d sum_f W_{d,f} sum_j conj(A^(j+d)_f) B^(j)_f,
// with A^(i), B^(j) the P-point DFTs of the blocks and W_d that of the
// window. Rounding of a block pair scales with |a| |b| over the pair times
// the weights of its window, not with the products that occur (for a fast-
// decaying mode a is large where b is negligible), so the pairs d = 0, 1,
// whose windows hold the largest weights, are summed exactly (Toeplitz
// products over the levels of the previous and the current block) and only
// d >= 2 (lags above Bk) here: (1/P) sum_{d>=2,f} W_{d,f} X_{d,f}, X summed
// over the modes, nb FFTs and (nb-2)(nb-1)/2 block products of Bk+1
// frequencies per mode. Both real blocks share one complex FFT, z = a + i b:
//   A_f = (Z_f + conj Z_{P-f}) / 2,   B_f = (Z_f - conj Z_{P-f}) / (2i).

// dst[c][t] = src[(row0 + dir * t) * ncols + c] for c < ncols, t < nt: time
// series of the time-major [rows][ncols] arrays as contiguous columns
// (64 x 64 tiles through LDS, both sides coalesced)
__global__ __launch_bounds__(256) void k_cols_transpose(const double* __restrict__ src, int64_t row0, int dir,
                                                        int64_t ncols, int64_t nt, double* __restrict__ dst) {
    __shared__ double tile[64][65];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int64_t c0 = int64_t(blockIdx.x) * 64, t0 = int64_t(blockIdx.y) * 64;
    for (int r = ty; r < 64; r += 4) {
        const int64_t t = t0 + r, c = c0 + tx;
        if (t < nt && c < ncols) tile[r][tx] = src[(row0 + dir * t) * ncols + c];
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int64_t c = c0 + r, t = t0 + tx;
        if (t < nt && c < ncols) dst[c * nt + t] = tile[tx][r];
    }
}

// nb in-place FFTs (decimation in time) of P = 2^logP complex values each,
// side by side in LDS (block i at z + i P): input in bit-reversed order,
// output X_f = sum_t x_t exp(-2 pi i f t / P) in natural order; tw[j] =
// exp(-2 pi i j / P), j < P/2 (in LDS). The radix-2 stages go in pairs: a
// thread takes four values i, i+h, i+2h, i+3h (h = 2^s) through stage s
// (pairs (i, i+h), (i+2h, i+3h), twiddle W_2h^pos) and stage s+1 (pairs
// (i, i+2h) with W_4h^pos, (i+h, i+3h) with W_4h^(pos+h)) in registers, so
// the values cross LDS once per two stages; an odd last stage is radix 2.
// Ends synchronised.
__device__ __forceinline__ double2 cmul(double2 a, double2 w) {
    return make_double2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x);
}

// LDS slot of complex point i of the transforms (and of twiddle i): one pad
// slot after every 16, so that the early passes' strided accesses (points 4
// or 16 apart), the bit-reversed stores and the later passes' strided
// twiddle reads spread over all banks
__device__ __forceinline__ int zp(int i) { return i + (i >> 4); }

__device__ __forceinline__ void lds_fft_batch(double2* z, int nb, int P, int logP, const double2* tw) {
    int s = 0;
    for (; s + 1 < logP; s += 2) {
        const int h = 1 << s, qP = P >> 2;
        for (int t = threadIdx.x; t < nb * qP; t += blockDim.x) {
            const int blk = t >> (logP - 2), tt = t & (qP - 1);
            const int pos = tt & (h - 1);
            const int i = blk * P + ((tt >> s) << (s + 2)) + pos;
            double2 a = z[zp(i)], b = z[zp(i + h)], c = z[zp(i + 2 * h)], d = z[zp(i + 3 * h)];
            const double2 w1 = tw[zp(pos << (logP - 1 - s))];
            const double2 w2 = tw[zp(pos << (logP - 2 - s))];
            const double2 w3 = tw[zp((pos + h) << (logP - 2 - s))];
            double2 u = cmul(b, w1);
            b = make_double2(a.x - u.x, a.y - u.y);
            a = make_double2(a.x + u.x, a.y + u.y);
            u = cmul(d, w1);
            d = make_double2(c.x - u.x, c.y - u.y);
            c = make_double2(c.x + u.x, c.y + u.y);
            u = cmul(c, w2);
            z[zp(i + 2 * h)] = make_double2(a.x - u.x, a.y - u.y);
            z[zp(i)] = make_double2(a.x + u.x, a.y + u.y);
            u = cmul(d, w3);
            z[zp(i + 3 * h)] = make_double2(b.x - u.x, b.y - u.y);
            z[zp(i + h)] = make_double2(b.x + u.x, b.y + u.y);
        }
        __syncthreads();
    }
    if (s < logP) {  // last stage, radix 2 (s = logP - 1)
        const int h = 1 << s, hP = P >> 1;
        for (int t = threadIdx.x; t < nb * hP; t += blockDim.x) {
            const int blk = t >> (logP - 1), pos = t & (hP - 1);
            const int i = blk * P + pos;
            const double2 u = cmul(z[zp(i + h)], tw[zp(pos)]);
            const double2 a = z[zp(i)];
            z[zp(i)] = make_double2(a.x + u.x, a.y + u.y);
            z[zp(i + h)] = make_double2(a.x - u.x, a.y - u.y);
        }
        __syncthreads();
    }
}

__device__ __forceinline__ int bit_reverse(int t, int logP) {
    return logP ? int(__builtin_bitreverse32(unsigned(t)) >> (32 - logP)) : 0;
}

// X_{d,f} over the modes [blockIdx.x * cols, +cols) of component blockIdx.y:
// per mode, load the nb blocks (a, b) into LDS in bit-reversed order, FFT
// them, split each block's spectrum in place (A_f into slot f, B_f into slot
// P-f for 0 < f < Bk; at f = 0 and Bk both are real and share the slot as
// (A, B)), and add sum_j conj(A^(j+d)_f) B^(j)_f for d >= 2, f <= Bk into
// registers. A thread item is one frequency f and kSpecSD consecutive
// distances d0 .. d0+kSpecSD-1 (item = (d0-2)/kSpecSD (Bk+1) + f, tid + 1024 r):
// it walks j upwards with B^(j) and a window of the kSpecSD values
// A^(j+d0..), so that a step reads two LDS values for kSpecSD products
// (blocks from nb on read as zero). Partial spectra per workgroup at
// q = (d-2)(Bk+1) + f, summed in k_beta_dot in a fixed order.
__global__ __launch_bounds__(1024) void k_beta_spec(BetaSpecArgs p) {
    __shared__ double2 z[kSpecMaxLds + kSpecMaxLds / 16];
    __shared__ double2 tws[kSpecMaxP / 2 + kSpecMaxP / 32];
    constexpr int SD = kSpecSD, IR = kSpecItems / 1024;
    const int k = blockIdx.y, tid = threadIdx.x;
    const int P = p.P, logP = p.logP, Bk = P >> 1, nb = p.nb, F1 = Bk + 1;
    const int Q = (nb - 2) * F1, NI = nb * F1, NIT = (nb - 2 + SD - 1) / SD * F1;
    for (int j = tid; j < Bk; j += 1024) tws[zp(j)] = reinterpret_cast<const double2*>(p.tw)[j];
    double xr[IR][SD], xi[IR][SD];
#pragma unroll
    for (int r = 0; r < IR; ++r)
#pragma unroll
        for (int dd = 0; dd < SD; ++dd) xr[r][dd] = xi[r][dd] = 0.0;
    const int64_t m0 = int64_t(blockIdx.x) * p.cols;
    const int64_t m1 = (m0 + p.cols < p.M) ? m0 + p.cols : p.M;
    // a mode's steps t = blk Bk + u < nb Bk <= kSpecMaxLds / 2, LV per thread;
    // the next mode's are loaded into registers while this one is transformed
    constexpr int LV = kSpecMaxLds / 2 / 1024;
    double pa[LV], pb[LV];
    auto fetch = [&](int64_t mode) {
        const int64_t e = int64_t(k) * p.M + mode;
        const double* __restrict__ a = p.psiT + e * p.N;
        const double* __restrict__ b = p.gT + e * p.N;
#pragma unroll
        for (int v = 0; v < LV; ++v) {
            const int t = tid + 1024 * v;
            pa[v] = (t < p.N) ? a[t] : 0.0;
            pb[v] = (t < p.N) ? b[t] : 0.0;
        }
    };
    if (m0 < m1) fetch(m0);
    for (int64_t mode = m0; mode < m1; ++mode) {
        // block blk, step u to slot bit_reverse(u), its zero padding u + Bk to
        // bit_reverse(u + Bk): every slot of the nb blocks is written
#pragma unroll
        for (int v = 0; v < LV; ++v) {
            const int t = tid + 1024 * v;
            if (t < nb * Bk) {
                const int blk = t >> (logP - 1), u = t & (Bk - 1);
                z[zp(blk * P + bit_reverse(u, logP))] = make_double2(pa[v], pb[v]);
                z[zp(blk * P + bit_reverse(u + Bk, logP))] = make_double2(0.0, 0.0);
            }
        }
        __syncthreads();
        if (mode + 1 < m1) fetch(mode + 1);
        lds_fft_batch(z, nb, P, logP, tws);
        // A_f = (Z_f + conj Z_{P-f}) / 2, B_f = (Z_f - conj Z_{P-f}) / (2i); the
        // slot pair (f, P-f) belongs to one thread
        for (int it = tid; it < NI; it += 1024) {
            const int blk = it / F1, f = it - blk * F1;
            const int i0 = blk * P + f, i1 = blk * P + ((P - f) & (P - 1));
            const double2 zf = z[zp(i0)], zc = z[zp(i1)];
            const double2 A = make_double2(0.5 * (zf.x + zc.x), 0.5 * (zf.y - zc.y));
            const double2 B = make_double2(0.5 * (zf.y + zc.y), -0.5 * (zf.x - zc.x));
            if (f == 0 || f == Bk) {
                z[zp(i0)] = make_double2(A.x, B.x);
            } else {
                z[zp(i0)] = A;
                z[zp(i1)] = B;
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < IR; ++r) {
            const int item = tid + 1024 * r;
            if (item < NIT) {
                const int d0 = 2 + SD * (item / F1), f = item % F1;
                const bool edge = f == 0 || f == Bk;
                const int fb = edge ? f : P - f;
                // A at f (real part only at the edges), B at P - f (the
                // imaginary part of slot f at the edges)
                auto ldA = [&](int blk) {
                    const double2 za = blk < nb ? z[zp(blk * P + f)] : make_double2(0.0, 0.0);
                    return edge ? make_double2(za.x, 0.0) : za;
                };
                double2 win[SD];
#pragma unroll
                for (int dd = 0; dd < SD; ++dd) win[dd] = ldA(d0 + dd);
                double sr[SD], si[SD];
#pragma unroll
                for (int dd = 0; dd < SD; ++dd) sr[dd] = si[dd] = 0.0;
                for (int j = 0; j + d0 < nb; ++j) {
                    const double2 zb = z[zp(j * P + fb)];
                    const double2 B = edge ? make_double2(zb.y, 0.0) : zb;
#pragma unroll
                    for (int dd = 0; dd < SD; ++dd) {
                        sr[dd] += win[dd].x * B.x + win[dd].y * B.y;  // conj(A) B
                        si[dd] += win[dd].x * B.y - win[dd].y * B.x;
                    }
#pragma unroll
                    for (int dd = 0; dd + 1 < SD; ++dd) win[dd] = win[dd + 1];
                    win[SD - 1] = ldA(j + 1 + d0 + SD - 1);
                }
#pragma unroll
                for (int dd = 0; dd < SD; ++dd) {
                    xr[r][dd] += sr[dd];
                    xi[r][dd] += si[dd];
                }
            }
        }
        __syncthreads();  // z is reloaded by the next mode
    }
    double* __restrict__ out = p.spec + (int64_t(k) * gridDim.x + blockIdx.x) * int64_t(Q) * 2;
#pragma unroll
    for (int r = 0; r < IR; ++r) {
        const int item = tid + 1024 * r;
        if (item < NIT) {
            const int d0 = 2 + SD * (item / F1), f = item % F1;
#pragma unroll
            for (int dd = 0; dd < SD; ++dd) {
                if (d0 + dd < nb) {
                    const int q = (d0 + dd - 2) * F1 + f;
                    out[2 * q] = xr[r][dd];
                    out[2 * q + 1] = xi[r][dd];
                }
            }
        }
    }
}

// W_{d,f}^(k): P-point DFTs of the windows w_d[r] = dw_{k, d Bk + r} (r in
// (-Bk, Bk) at index r mod P; lags below 0 or from N on are 0), both
// components from one complex FFT (z = w^(0) + i w^(1)): W[k][d][f][re, im],
// f <= Bk. One workgroup.
__global__ __launch_bounds__(1024) void k_fft_w(const double* __restrict__ dw, int64_t dwstride, int64_t N,
                                                int nb, int P, int logP, const double* __restrict__ twp,
                                                double* __restrict__ W) {
    __shared__ double2 z[kSpecMaxLds + kSpecMaxLds / 16];
    __shared__ double2 tws[kSpecMaxP / 2 + kSpecMaxP / 32];
    const int Bk = P >> 1, Q = nb * (Bk + 1);
    for (int j = threadIdx.x; j < Bk; j += 1024) tws[zp(j)] = reinterpret_cast<const double2*>(twp)[j];
    for (int t = threadIdx.x; t < nb * P; t += 1024) {
        const int d = t >> logP, r = t & (P - 1);
        const int64_t lag = int64_t(d) * Bk + (r < Bk ? r : r - P);
        const bool ok = r != Bk && lag >= 0 && lag < N;
        z[zp(d * P + bit_reverse(r, logP))] =
            ok ? make_double2(dw[lag], dw[dwstride + lag]) : make_double2(0.0, 0.0);
    }
    __syncthreads();
    lds_fft_batch(z, nb, P, logP, tws);
    for (int q = threadIdx.x; q < Q; q += 1024) {
        const int d = q / (Bk + 1), f = q - d * (Bk + 1);
        const double2 zf = z[zp(d * P + f)], zc = z[zp(d * P + ((P - f) & (P - 1)))];
        W[2 * q] = 0.5 * (zf.x + zc.x);
        W[2 * q + 1] = 0.5 * (zf.y - zc.y);
        W[2 * (Q + q)] = 0.5 * (zf.y + zc.y);
        W[2 * (Q + q) + 1] = -0.5 * (zf.x - zc.x);
    }
}

// part[k][block] = (1/P) sum over the block's q = (d-2)(Bk+1) + f, d >= 2,
// of w_f Re(W_{d,f} X_q), X_q the sum of the nwg partial spectra (in order),
// w_f = 1 at f = 0 and Bk, else 2 (the conjugate half). grid (blocks, 2),
// 64 threads.
__global__ __launch_bounds__(64) void k_beta_dot(BetaDotArgs p) {
    const int Bk = p.P >> 1, Q = (p.nb - 2) * (Bk + 1), QW = p.nb * (Bk + 1), k = blockIdx.y;
    const int q = blockIdx.x * 64 + threadIdx.x;
    double v = 0.0;
    if (q < Q) {
        const int f = q % (Bk + 1);
        double xr = 0.0, xi = 0.0;
        const double* __restrict__ sp = p.spec + (int64_t(k) * p.nwg * Q + q) * 2;
        for (int g = 0; g < p.nwg; ++g) {
            xr += sp[int64_t(g) * Q * 2];
            xi += sp[int64_t(g) * Q * 2 + 1];
        }
        const double* __restrict__ w = p.W + (int64_t(k) * QW + 2 * (Bk + 1) + q) * 2;
        v = ((f == 0 || f == Bk) ? 1.0 : 2.0) * (w[0] * xr - w[1] * xi);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (threadIdx.x == 0) p.part[int64_t(k) * gridDim.x + blockIdx.x] = v / double(p.P);
}

// per-component sums of acc[2][M]: partials part[k][block]
__global__ __launch_bounds__(256) void k_sum_rows(const double* __restrict__ acc, int64_t M, int64_t per,
                                                  double* __restrict__ part) {
    __shared__ double red[256];
    const int k = blockIdx.y;
    const int64_t lo = int64_t(blockIdx.x) * per;
    double v = 0.0;
    for (int64_t x = lo + threadIdx.x; x < lo + per && x < M; x += 256) v += acc[int64_t(k) * M + x];
    const double tot = block_sum256(v, red);
    if (threadIdx.x == 0) part[int64_t(k) * gridDim.x + blockIdx.x] = tot;
}

// ---------------------------------------------------------------------------
// Small dense GEMM pair for the 2D DST-I: C_k = A_k B_k, k = 0, 1, with
// FP64 MFMA 16x16x4. One workgroup = one 16x16 output tile of both
// components; its 4 waves split the K loop and reduce through LDS.
// Epilogues: 0 plain store; 1 per-mode 2x2 solve (forward transform
// finished); 2 store minus a field (inverse transform finished: G^n = K^-1 w - q);
// 3 scaled store (sine coefficients of a field).
template <int EPI>
__global__ __launch_bounds__(256) void k_dst_gemm(GemmArgs p) {
    __shared__ double red[4][2][16][17];
    if (blockIdx.z) {  // operand set of this GEMM of the batch
        const int64_t b = blockIdx.z;
        if (!p.A_shared) {
            p.A0 += b * p.sA;
            p.A1 += b * p.sA;
        }
        if (!p.B_shared) {
            p.B0 += b * p.sB;
            p.B1 += b * p.sB;
        }
        p.C0 += b * p.sC;
        p.C1 += b * p.sC;
        if (EPI == 2) {
            p.sub0 += b * p.sC;
            p.sub1 += b * p.sC;
        }
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int r0 = blockIdx.y * 16, c0 = blockIdx.x * 16;
    const int row = r0 + li, col = c0 + li;
    d4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
    // wave w takes the K-steps kk = 4w, 4w + 16, ...; the operands of KB of
    // them are loaded together before their products, so a wave waits for
    // memory once per KB K-steps rather than at every one
    constexpr int KB = 8;
    for (int kb = wave * 4; kb < p.K; kb += 16 * KB) {
        double a0[KB], a1[KB], b0[KB], b1[KB];
#pragma unroll
        for (int u = 0; u < KB; ++u) {
            const int kx = kb + 16 * u + lk;
            const bool kin = kx < p.K;
            a0[u] = a1[u] = b0[u] = b1[u] = 0.0;
            if (kin && row < p.R) {
                // A is either a per-component field (row-major, lda) or a shared
                // symmetric sine matrix (read transposed for coalescing)
                if (p.A_shared) {
                    a0[u] = a1[u] = p.A0[int64_t(kx) * p.lda + row];
                } else {
                    a0[u] = p.A0[int64_t(row) * p.lda + kx];
                    a1[u] = p.A1[int64_t(row) * p.lda + kx];
                }
            }
            if (kin && col < p.C) {
                if (p.B_shared) {
                    b0[u] = b1[u] = p.B0[int64_t(kx) * p.ldb + col];
                } else {
                    b0[u] = p.B0[int64_t(kx) * p.ldb + col];
                    b1[u] = p.B1[int64_t(kx) * p.ldb + col];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < KB; ++u) {
            if (kb + 16 * u < p.K) {  // the K-steps of this wave, as one after another
                acc0 = mfma16x16x4(a0[u], b0[u], acc0);
                acc1 = mfma16x16x4(a1[u], b1[u], acc1);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        red[wave][0][lk + 4 * i][li] = acc0[i];
        red[wave][1][lk + 4 * i][li] = acc1[i];
    }
    __syncthreads();
    // 256 threads, one output element (i, j) of the 16x16 tile each
    const int ti = threadIdx.x >> 4, tj = threadIdx.x & 15;
    const int orow = r0 + ti, ocol = c0 + tj;
    if (orow >= p.R || ocol >= p.C) return;
    double v0 = red[0][0][ti][tj] + red[1][0][ti][tj] + red[2][0][ti][tj] + red[3][0][ti][tj];
    double v1 = red[0][1][ti][tj] + red[1][1][ti][tj] + red[2][1][ti][tj] + red[3][1][ti][tj];
    const int64_t o = int64_t(orow) * p.ldc + ocol;
    if (EPI == 1) {
        // per-mode solve: row = y-mode p, col = x-mode q
        const double lam = p.lamy[orow] + p.lamx[ocol];
        const double m11 = p.cdiag + p.dd0[0] * (p.a + lam);
        const double m22 = p.cdiag + p.dd0[1] * (p.a + lam);
        const double m12 = -p.a * p.dd0[1], m21 = -p.a * p.dd0[0];
        const double det = m11 * m22 - m12 * m21;
        const double s = p.scale / det;
        const double g0 = (m22 * v0 - m12 * v1) * s;
        const double g1 = (m11 * v1 - m21 * v0) * s;
        v0 = g0;
        v1 = g1;
    } else if (EPI == 2) {
        v0 -= p.sub0[o];
        v1 -= p.sub1[o];
    } else if (EPI == 3) {
        v0 *= p.scale;
        v1 *= p.scale;
    }
    p.C0[o] = v0;
    p.C1[o] = v1;
}

// ---------------------------------------------------------------------------
// launchers (optionally bracketed by timing events, see prof_begin/prof_end)
// state sizes up to this many bytes stay cached between passes (the 256 MB
// Infinity Cache, with room for the level window and the sums)
constexpr int64_t kHistCachedBytes = int64_t(128) << 20;

void launch_hist_block(const HistBlockArgs& a, int lanes, hipStream_t st) {
    dim3 grid(unsigned((a.M * lanes + 255) / 256), 1, 2);
    const bool nt = int64_t(2) * a.np * a.hstride * int64_t(sizeof(double)) > kHistCachedBytes;
#define CQ_HB(BT, S)                                                                                    \
    if (nt)                                                                                             \
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_hist_block<BT, S, true>), grid, dim3(256), 0, st, a);      \
    else                                                                                                \
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_hist_block<BT, S, false>), grid, dim3(256), 0, st, a)
#define CQ_HB_S(BT)               \
    switch (lanes) {              \
        case 1: CQ_HB(BT, 1); break; \
        case 2: CQ_HB(BT, 2); break; \
        default: CQ_HB(BT, 4); break; \
    }
    prof_begin(0, st);
    if (a.BT <= 8) {
        CQ_HB_S(8)
    } else if (a.BT <= 16) {
        CQ_HB_S(16)
    } else if (a.BT <= 24) {
        CQ_HB_S(24)
    } else if (a.BT <= 30) {  // the BDF2 lag 30: two fewer rows of registers than 32
        CQ_HB_S(30)
    } else {
        CQ_HB_S(32)
    }
    prof_end(0, st);
#undef CQ_HB_S
#undef CQ_HB
}

void launch_hist_direct(const HistDirectArgs& a, hipStream_t st) {
    dim3 grid(unsigned((a.M + 255) / 256), 1, 2);
    prof_begin(1, st);
    hipLaunchKernelGGL(k_hist_direct, grid, dim3(256), 0, st, a);
    prof_end(1, st);
}

// ---------------------------------------------------------------------------
// One direct history row (cq_history and its allocation-free variant), the
// convolution of (3.8)/(3.17) at a single step n:
//   S[x] = sum_{l=1}^{n-1} d[n-l] G^l[x],   G^l[x] at G[l*M + x].
// A weighted sum over stored levels: every level is read once, so the kernel
// streams HBM (8 bytes per DOF and level). One DOF per lane (a wave reads 64
// consecutive doubles of a level); blockIdx.y = slice q of the levels
// 1 + q*lchunk .. min(n-1, (q+1)*lchunk), so that a short row still fills the
// GPU. The weights are wave-uniform scalar loads. A single slice writes
// out[x]; several write part[q][x] and k_row_sum adds them in slice order.
__global__ __launch_bounds__(256) void k_hist_row(const double* __restrict__ G, int64_t n, int64_t M,
                                                  const double* __restrict__ d, int64_t lchunk,
                                                  double* __restrict__ out) {
    const int64_t x = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (x >= M) return;
    const int64_t lb = 1 + int64_t(blockIdx.y) * lchunk;
    const int64_t le = (lb + lchunk - 1 < n - 1) ? lb + lchunk - 1 : n - 1;  // inclusive
    const cdouble* dd = (const cdouble*)(d);
    const double* __restrict__ g = G + x;
    double acc = 0.0;
    int64_t l = lb;
    // eight levels per round: the loads are independent, the sum is not
    for (; l + 8 <= le + 1; l += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = g[(l + u) * M];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = fma(dd[n - l - u], v[u], acc);
    }
    for (; l <= le; ++l) acc = fma(dd[n - l], g[l * M], acc);
    out[int64_t(blockIdx.y) * M + x] = acc;
}

// out[x] = sum_{q < ks} part[q*M + x], q ascending
__global__ __launch_bounds__(256) void k_row_sum(const double* __restrict__ part, int ks, int64_t M,
                                                 double* __restrict__ out) {
    const int64_t x = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (x >= M) return;
    double s = part[x];
    for (int q = 1; q < ks; ++q) s += part[int64_t(q) * M + x];
    out[x] = s;
}

// out[x] = 0 (a kernel, not a memset, so that the call can sit in a captured graph)
__global__ __launch_bounds__(256) void k_fill_zero(double* __restrict__ out, int64_t M) {
    const int64_t x = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (x < M) out[x] = 0.0;
}

int hist_row_slices(int64_t n, int64_t M, int64_t part_cap) {
    if (n <= 2) return 1;
    // about 8192 waves (32 per CU) so that enough level loads are in flight
    const int64_t wg = (M + 255) / 256;
    int64_t ks = (2048 + wg - 1) / wg;
    ks = std::min<int64_t>(ks, std::min<int64_t>(1024, (n - 1 + 15) / 16));  // >= 16 levels per slice
    if (part_cap >= 0) ks = std::min<int64_t>(ks, part_cap / M);
    return int(std::max<int64_t>(1, ks));
}

void launch_hist_row(const double* G, int64_t n, int64_t M, const double* d, int ks, double* part, double* out,
                     hipStream_t st) {
    const unsigned gx = unsigned((M + 255) / 256);
    prof_begin(6, st);
    if (n <= 1) {
        hipLaunchKernelGGL(k_fill_zero, dim3(gx), dim3(256), 0, st, out, M);
    } else {
        const int64_t lchunk = (n - 1 + ks - 1) / ks;
        const int64_t slices = (n - 1 + lchunk - 1) / lchunk;
        if (slices == 1) {
            hipLaunchKernelGGL(k_hist_row, dim3(gx, 1), dim3(256), 0, st, G, n, M, d, lchunk, out);
        } else {
            hipLaunchKernelGGL(k_hist_row, dim3(gx, unsigned(slices)), dim3(256), 0, st, G, n, M, d, lchunk, part);
            hipLaunchKernelGGL(k_row_sum, dim3(gx), dim3(256), 0, st, part, int(slices), M, out);
        }
    }
    prof_end(6, st);
}

void launch_step_1d(const StepArgs& a, size_t lds, hipStream_t st) {
    prof_begin(3, st);
    const int R = int((a.M + kNT1D - 1) / kNT1D);
    switch (R) {
        // (two LDS buffers: twice the single buffer the caller sized)
        case 1: hipLaunchKernelGGL(k_step_1d_reg, dim3(1), dim3(kNT1D), 2 * lds, st, a); break;
        case 2: hipLaunchKernelGGL(k_step_1d<2>, dim3(1), dim3(kNT1D), lds, st, a); break;
        case 3: hipLaunchKernelGGL(k_step_1d<3>, dim3(1), dim3(kNT1D), lds, st, a); break;
        default: hipLaunchKernelGGL(k_step_1d<4>, dim3(1), dim3(kNT1D), lds, st, a); break;
    }
    prof_end(3, st);
}

void launch_prep_2d(const StepArgs& a, hipStream_t st) {
    dim3 grid(unsigned((a.M + 255) / 256), 2);
    prof_begin(4, st);
    hipLaunchKernelGGL(k_prep_2d, grid, dim3(256), 0, st, a);
    prof_end(4, st);
}

void launch_gemm(const GemmArgs& a, int epi, hipStream_t st) {
    dim3 grid(unsigned((a.C + 15) / 16), unsigned((a.R + 15) / 16), unsigned(a.batch > 1 ? a.batch : 1));
    prof_begin(5, st);
    if (epi == 1)
        hipLaunchKernelGGL(k_dst_gemm<1>, grid, dim3(256), 0, st, a);
    else if (epi == 2)
        hipLaunchKernelGGL(k_dst_gemm<2>, grid, dim3(256), 0, st, a);
    else if (epi == 3)
        hipLaunchKernelGGL(k_dst_gemm<3>, grid, dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(k_dst_gemm<0>, grid, dim3(256), 0, st, a);
    prof_end(5, st);
}

void launch_sine_transform(int dim, int nx, int ny, int nz, const double* Sx, const double* Sy, const double* Sz,
                           const double* G, double* tmp, double* out, double scale, hipStream_t st) {
    const int64_t M = int64_t(nx) * (dim >= 2 ? ny : 1) * (dim == 3 ? nz : 1);
    if (dim == 1) {
        GemmArgs ga{};
        ga.R = 1; ga.C = nx; ga.K = nx; ga.lda = nx; ga.ldb = nx; ga.ldc = nx;
        ga.A_shared = 0; ga.B_shared = 1;
        ga.A0 = G; ga.A1 = G + M; ga.B0 = Sx; ga.B1 = Sx; ga.C0 = out; ga.C1 = out + M;
        ga.scale = scale;
        launch_gemm(ga, 3, st);
        return;
    }
    const int planes = dim == 3 ? nz : 1;
    // along x: every row of nx values (ny * planes rows) times S_x
    // (2D: into tmp, then y into out; 3D: into out, y into tmp, z into out)
    double* xo = dim == 2 ? tmp : out;
    double* yo = dim == 2 ? out : tmp;
    GemmArgs ga{};
    ga.R = ny * planes; ga.C = nx; ga.K = nx; ga.lda = nx; ga.ldb = nx; ga.ldc = nx;
    ga.A_shared = 0; ga.B_shared = 1;
    ga.A0 = G; ga.A1 = G + M; ga.B0 = Sx; ga.B1 = Sx; ga.C0 = xo; ga.C1 = xo + M;
    launch_gemm(ga, 0, st);
    // along y: S_y times each z-plane (ny x nx)
    GemmArgs gb{};
    gb.R = ny; gb.C = nx; gb.K = ny; gb.lda = ny; gb.ldb = nx; gb.ldc = nx;
    gb.A_shared = 1; gb.B_shared = 0;
    gb.A0 = Sy; gb.A1 = Sy; gb.B0 = xo; gb.B1 = xo + M; gb.C0 = yo; gb.C1 = yo + M;
    gb.batch = planes;
    gb.sB = gb.sC = int64_t(ny) * nx;
    gb.scale = scale;
    if (dim == 2) {
        launch_gemm(gb, 3, st);
        return;
    }
    launch_gemm(gb, 0, st);
    // along z: S_z times the (nz) x (ny nx) matrix
    GemmArgs gc{};
    gc.R = nz; gc.C = ny * nx; gc.K = nz; gc.lda = nz; gc.ldb = ny * nx; gc.ldc = ny * nx;
    gc.A_shared = 1; gc.B_shared = 0;
    gc.A0 = Sz; gc.A1 = Sz; gc.B0 = yo; gc.B1 = yo + M; gc.C0 = out; gc.C1 = out + M;
    gc.scale = scale;
    launch_gemm(gc, 3, st);
}

// time-blocked where the lag allows blocks of 8..32 steps and the nodes fit
// 24 per lane over 32 lanes; otherwise a reduction per step
bool modal_fast_blocked(int L, int np) { return L >= 8 && L <= 32 && (np + 31) / 32 <= 24; }

void launch_modal_fast(const ModalFastArgs& a, hipStream_t st) {
    dim3 grid(unsigned((a.M + 3) / 4));
    prof_begin(7, st);
    const int np32 = (a.np + 31) / 32;
    if (modal_fast_blocked(a.L, a.np)) {
        if (np32 <= 4)
            hipLaunchKernelGGL(k_modal_fast_tb<4>, grid, dim3(256), 0, st, a);
        else if (np32 <= 8)
            hipLaunchKernelGGL(k_modal_fast_tb<8>, grid, dim3(256), 0, st, a);
        else if (np32 <= 12)
            hipLaunchKernelGGL(k_modal_fast_tb<12>, grid, dim3(256), 0, st, a);
        else if (np32 <= 16)
            hipLaunchKernelGGL(k_modal_fast_tb<16>, grid, dim3(256), 0, st, a);
        else if (np32 <= 20)
            hipLaunchKernelGGL(k_modal_fast_tb<20>, grid, dim3(256), 0, st, a);
        else
            hipLaunchKernelGGL(k_modal_fast_tb<24>, grid, dim3(256), 0, st, a);
        prof_end(7, st);
        return;
    }
    const int npl = (a.np + 63) / 64;
    if (npl <= 1)
        hipLaunchKernelGGL(k_modal_fast<1>, grid, dim3(256), 0, st, a);
    else if (npl <= 2)
        hipLaunchKernelGGL(k_modal_fast<2>, grid, dim3(256), 0, st, a);
    else if (npl <= 4)
        hipLaunchKernelGGL(k_modal_fast<4>, grid, dim3(256), 0, st, a);
    else if (npl <= 8)
        hipLaunchKernelGGL(k_modal_fast<8>, grid, dim3(256), 0, st, a);
    else if (npl <= 12)
        hipLaunchKernelGGL(k_modal_fast<12>, grid, dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(k_modal_fast<16>, grid, dim3(256), 0, st, a);
    prof_end(7, st);
}

void launch_modal_batch(const BatchArgs& a, int npl, int lpm, hipStream_t st) {
    if (lpm == 0) {  // time-blocked, one wave per mode; npl = nodes per lane over 32 lanes
        const dim3 grid(unsigned((a.total + 3) / 4));
#define CQ_BATCH_TB(NP) hipLaunchKernelGGL((k_modal_batch_tb<NP>), grid, dim3(256), 0, st, a)
        prof_begin(9, st);
        if (npl <= 4) CQ_BATCH_TB(4);
        else if (npl <= 6) CQ_BATCH_TB(6);
        else if (npl <= 8) CQ_BATCH_TB(8);
        else if (npl <= 10) CQ_BATCH_TB(10);
        else if (npl <= 12) CQ_BATCH_TB(12);
        else if (npl <= 14) CQ_BATCH_TB(14);
        else if (npl <= 16) CQ_BATCH_TB(16);
        else if (npl <= 18) CQ_BATCH_TB(18);
        else if (npl <= 20) CQ_BATCH_TB(20);
        else CQ_BATCH_TB(24);
        prof_end(9, st);
#undef CQ_BATCH_TB
        return;
    }
    const int64_t threads = a.total * lpm;
    const dim3 grid(unsigned((threads + 255) / 256));
#define CQ_BATCH(NP, LP) hipLaunchKernelGGL((k_modal_batch<NP, LP>), grid, dim3(256), 0, st, a)
    prof_begin(9, st);
    if (lpm == 32) {
        if (npl <= 2) CQ_BATCH(2, 32);
        else if (npl <= 4) CQ_BATCH(4, 32);
        else if (npl <= 8) CQ_BATCH(8, 32);
        else if (npl <= 12) CQ_BATCH(12, 32);
        else CQ_BATCH(16, 32);
    } else {
        if (npl <= 1) CQ_BATCH(1, 64);
        else if (npl <= 2) CQ_BATCH(2, 64);
        else if (npl <= 4) CQ_BATCH(4, 64);
        else if (npl <= 8) CQ_BATCH(8, 64);
        else if (npl <= 12) CQ_BATCH(12, 64);
        else CQ_BATCH(16, 64);
    }
    prof_end(9, st);
#undef CQ_BATCH
}

void launch_modal_win(const ModalWinArgs& a, bool adj, hipStream_t st) {
    prof_begin(7, st);
    const dim3 grid(unsigned((2 * a.M + 63) / 64));
    if (adj)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_modal_win<true>), grid, dim3(64), 0, st, a);
    else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_modal_win<false>), grid, dim3(64), 0, st, a);
    prof_end(7, st);
}

void launch_modal_near(const ModalNearArgs& a, int B, bool adj, hipStream_t st) {
    // the modal direct solver always uses blocks of 64 steps
    (void)B;
    const dim3 grid(unsigned((2 * a.M + 63) / 64));
    const bool full = a.nfirst == a.n0 + 1 && a.bt == 64;
    prof_begin(8, st);
    if (adj) {
        if (full)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_modal_near<64, true, true>), grid, dim3(64), 0, st, a);
        else
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_modal_near<64, false, true>), grid, dim3(64), 0, st, a);
    } else {
        if (full)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_modal_near<64, true, false>), grid, dim3(64), 0, st, a);
        else
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_modal_near<64, false, false>), grid, dim3(64), 0, st, a);
    }
    prof_end(8, st);
}

void launch_adj_g0(const AdjGradArgs& a, hipStream_t st) {
    const unsigned bx = unsigned((2 * a.M + 255) / 256);
    if (a.scheme == 2) hipLaunchKernelGGL(k_adj_g0_part, dim3(bx, unsigned(a.nchunk)), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_adj_g0, dim3(bx), dim3(256), 0, st, a);
}

int launch_adj_da(const AdjGradArgs& a, hipStream_t st) {
    const int blocks = int((a.M + 255) / 256);
    const int nc = a.nchunk_da > 0 ? a.nchunk_da : a.nchunk;
    hipLaunchKernelGGL(k_adj_da, dim3(unsigned(blocks), unsigned(nc)), dim3(256), 0, st, a);
    return blocks * a.nchunk;
}

void launch_adj_beta(const AdjBetaArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_beta, dim3(unsigned((2 * a.M + 63) / 64)), dim3(64 * kAdjBetaWaves), 0, st, a);
}

void launch_cols_transpose(const double* src, int64_t row0, int dir, int64_t ncols, int64_t nt, double* dst,
                           hipStream_t st) {
    prof_begin(11, st);
    hipLaunchKernelGGL(k_cols_transpose, dim3(unsigned((ncols + 63) / 64), unsigned((nt + 63) / 64)), dim3(256), 0,
                       st, src, row0, dir, ncols, nt, dst);
    prof_end(11, st);
}

void launch_beta_spec(const BetaSpecArgs& a, int nwg, hipStream_t st) {
    prof_begin(12, st);
    hipLaunchKernelGGL(k_beta_spec, dim3(unsigned(nwg), 2), dim3(1024), 0, st, a);
    prof_end(12, st);
}

void launch_fft_w(const double* dw, int64_t dwstride, int64_t N, int nb, int P, int logP, const double* tw,
                  double* W, hipStream_t st) {
    hipLaunchKernelGGL(k_fft_w, dim3(1), dim3(1024), 0, st, dw, dwstride, N, nb, P, logP, tw, W);
}

int launch_beta_dot(const BetaDotArgs& a, hipStream_t st) {
    const int blocks = ((a.nb - 2) * ((a.P >> 1) + 1) + 63) / 64;
    prof_begin(12, st);
    hipLaunchKernelGGL(k_beta_dot, dim3(unsigned(blocks), 2), dim3(64), 0, st, a);
    prof_end(12, st);
    return blocks;
}

int launch_sum_rows(const double* acc, int64_t M, double* part, hipStream_t st) {
    const int64_t per = 4096;
    const int blocks = int((M + per - 1) / per);
    hipLaunchKernelGGL(k_sum_rows, dim3(unsigned(blocks), 2), dim3(256), 0, st, acc, M, per, part);
    return blocks;
}

const void* kernel_step_1d(int R) {
    switch (R) {
        case 1: return reinterpret_cast<const void*>(&k_step_1d<1>);
        case 2: return reinterpret_cast<const void*>(&k_step_1d<2>);
        case 3: return reinterpret_cast<const void*>(&k_step_1d<3>);
        default: return reinterpret_cast<const void*>(&k_step_1d<4>);
    }
}

}  // namespace cqfp
