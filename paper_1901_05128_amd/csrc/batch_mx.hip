// Fast CQ on the FP64 matrix cores: the compressed history state of 16 modes
// of one problem advanced and summed as small GEMMs (fast sum of geometric
// sequences, (3.9)-(3.10) and (3.18); the per-mode form of schemes
// (4.1)-(4.3) and (4.7)-(4.8)), for batched solves, whole runs of one
// problem and the two sweeps of a gradient.
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "kernels.h"

namespace cqfp {

// One workgroup (4 waves) runs the whole time loop of 16 modes of one
// problem, in blocks of B = 16 steps (B <= L, the lag of the exact window).
// The state of node j of component k after the levels up to n - L is
// h_j^n = r_j h_j^{n-1} + g_k^{n-L}, and step n's fast part is sum_j w_j h_j^n.
// Over a block of steps n0+1..n0+B every level the state takes in is at most
// n0, so with H = h^{n0} ([nodes][modes]) and the block's inputs
// Gin[s] = g^{n0+1+s-L}, s < B:
//   fast part of step n0+1+t = sum_j w_j r_j^{t+1} H_j
//                              + sum_{s<=t} c_{t-s} Gin[s],  c_e = sum_j w_j r_j^e
//   h^{n0+B} = r^B H + sum_s r^{B-1-s} Gin[s]
// Both are GEMMs over the 16 modes of the tile (the node and step tables
// are the same for every mode). The exact window (lags 1..L-1) splits into
// the levels before the block (a Toeplitz-by-levels GEMM as well) and the
// block's own levels, which the serial steps push into their later steps.
//
// Phase A (all waves, matrix cores): wave w holds the node tiles
// jt = h, h+2, ... (h = w & 1) of component k = w >> 1 as MFMA accumulators
// ([16 nodes][16 modes] per tile). It advances each tile over the block
// (h^{n0+B}) and then forms from the new state its part of the next block's
// W H sums (a double-buffered LDS slot); of each component, wave h = 0 adds
// this block's in-block Toeplitz term and BDF2's starting correction
// 1/2 d_{k,n-1} g_k^0, wave h = 1 the window of the earlier levels (another
// LDS slot). Phase B (wave 0): the block's steps one by one, lane 4p + 2k + e
// for mode p, component k, steps of parity e (the lane keeps their pending
// sums, which start as the two slots' partial sums); each new level is
// pushed into the later steps of the block and written to the LDS level ring
// that phase A of the next block reads.
//
// MFMA 16x16x4 f64 operands: A(16x4) lane L -> (row L%16, k L/16);
// B(4x16) lane L -> (k L/16, col L%16); C: item i of lane L is row
// L/16 + 4i, col L%16.
//
// Tables (host-built, per problem, nt node tiles per component and a zero
// tile jt = nt, at mx_off):
//   W[k][jt][i][L] = w_j r_j^{t+1}, t = L%16, j = 16 jt + 4i + L/16
//   R[k][jt][i][L] = r_j^{B-1-s},   j = 16 jt + L%16, s = 4i + L/16
//   rB[k][j]       = r_j^B
//   C[k][i][L]     = c_{t-s} (s <= t, else 0), t = L%16, s = 4i + L/16
//   D[k][i][L]     = d_{k,t+1+u} (t+1+u <= L-1, else 0), u = 4i + L/16, i < 8
// (zero for nodes j >= np). Needs kMxMinLag <= L <= kMxMaxLag and
// nt <= 2 NTW.
//
// MODE 0: the final level only (batched solves, whole runs); 1: every step's
// level and history sum also go to p.traj / p.sx (the forward of a
// gradient); 2: the adjoint sweep of a gradient in reversed time, the same
// recurrence on the levels psi = Dm mu with the transposed step
// mu^n = Minv^T (E^n - S^n), E^n from mu^{n-1}, mu^{n-2}, the cotangent
// (p.g0) subtracted from S^1, no starting correction; psi^n and mu^n go to
// p.traj / p.sx. With p.tcols (modes 1, 2, NTW < kMxColsNtw) each finished
// block's levels are also written from the ring as time series, 16 steps of
// a place at a time.

// a global-memory double (keeps global loads after an asm statement)
typedef __attribute__((address_space(1))) const double gdouble;

template <int NTW, int MODE>
__global__ __launch_bounds__(256, 2) void k_modal_batch_mx(BatchArgs p) {
    constexpr bool TRAJ = MODE != 0, ADJ = MODE == 2;
    constexpr bool COLS = TRAJ && NTW < kMxColsNtw;  // p.tcols taken (the widest variant has no registers left)
    constexpr int B = kMxB;
    __shared__ double fW[2][4][B][16];             // state part of the fast sums [block & 1][wave][step][mode]
    __shared__ double fT[4][B][16];                // in-block Toeplitz, earlier-level window, correction
    __shared__ double ring[64][2][16];             // level g_k^m of the tile's modes at [m & 63][k]
    __shared__ double rbt[2][32 * NTW];            // r_j^B [k][j] (j < 32 NTW: tiles jt <= 2 NTW - 1)
    __shared__ double dtab[2][B];                  // push weights d_{k,lag}, lag 1..B-1 (0 at lag 0)
    __shared__ double cst[7][64];                  // phase B: per-lane constants and state
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    const int64_t tile = blockIdx.x;
    int lo = 0, hi = p.count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (p.cumt[mid] <= tile) lo = mid; else hi = mid - 1;
    }
    const BatchInst& I = p.inst[p.list[lo]];
    const int64_t mode0 = (tile - p.cumt[lo]) * 16;
    const int64_t M = I.M, N = I.N;
    const int L = I.L, NT = I.nt;
    const bool bdf2 = I.scheme == 2;
    const double* __restrict__ tab = p.mx + I.mx_off;
    for (int e = threadIdx.x; e < 64 * 2 * 16; e += 256) (&ring[0][0][0])[e] = 0.0;
    for (int e = threadIdx.x; e < 4 * B * 16; e += 256) (&fW[0][0][0][0])[e] = 0.0;  // h^0 = 0
    const int64_t t1 = int64_t(NT + 1) * 256;  // doubles of one component's W or R table
    for (int e = threadIdx.x; e < 2 * 32 * NTW; e += 256) {
        const int kk = e / (32 * NTW), j = e - kk * 32 * NTW;
        rbt[kk][j] = j < 16 * NT ? tab[4 * t1 + kk * 16 * NT + j] : 0.0;
    }
    if (threadIdx.x < 2 * B) {
        const int kk = threadIdx.x / B, lag = threadIdx.x % B;
        dtab[kk][lag] = lag >= 1 ? p.d[I.d_off + kk * I.dstride + lag] : 0.0;
    }

    // ---- phase A roles
    const int k = wave >> 1, h = wave & 1;
    const int li = lane & 15, lk = lane >> 4;
    const double* __restrict__ Wb = tab + k * t1;
    const double* __restrict__ Rb = tab + (2 + k) * t1;
    const double* __restrict__ Ck = tab + 4 * t1 + int64_t(32) * NT + k * 256;
    const double* __restrict__ Dk = tab + 4 * t1 + int64_t(32) * NT + 512 + k * 512;
    const unsigned ul = unsigned(lane);
    const double* __restrict__ dkA = p.d + I.d_off + k * I.dstride;
    const int64_t dlast = I.dstride - 1;

    // ---- phase B (wave 0): lane 4p + 2k + e, per-mode constants kept in LDS
    const int cp = lane >> 2, ck = (lane >> 1) & 1, ce = lane & 1;
    const double inv_tau = I.inv_tau;
    // E = e1 g^{n-1} + e2 g^{n-2} (BE: g^{n-1}/tau; BDF2: (2 g^{n-1} - g^{n-2}/2)/tau)
    const double e1 = (bdf2 ? 2.0 : 1.0) * inv_tau, e2 = (bdf2 ? -0.5 : 0.0) * inv_tau;
    if (wave == 0 && ADJ) {
        // mu^n = Minv^T r: the own and the other row's entry of column k;
        // psi = Dm mu = L1 mu_k - a mu_k'
        const int64_t mB = (mode0 + cp < M) ? mode0 + cp : M - 1;
        const double ca = I.a;
        const double L1 = ca + p.lam[I.mode_off + mB];
        const double m11 = I.c + I.d00 * L1, m22 = I.c + I.d01 * L1;
        const double m12 = -ca * I.d01, m21 = -ca * I.d00;
        const double idet = 1.0 / (m11 * m22 - m12 * m21);
        const double i00 = m22 * idet, i01 = -m12 * idet, i10 = -m21 * idet, i11 = m11 * idet;
        cst[0][lane] = ck ? i11 : i00;
        cst[1][lane] = ck ? i01 : i10;
        cst[2][lane] = L1;
        cst[3][lane] = -ca;
        cst[4][lane] = 0.0;  // mu^{n-1}
        cst[5][lane] = 0.0;  // mu^{n-2}
        cst[6][lane] = 0.0;  // newest level
    } else if (wave == 0) {
        const int64_t mB = (mode0 + cp < M) ? mode0 + cp : M - 1;
        const double* __restrict__ g0 = p.g0 + 2 * I.mode_off;
        const double g00 = g0[mB], g01 = g0[M + mB];
        const double ca = I.a;
        const double lam = p.lam[I.mode_off + mB];
        const double L1 = ca + lam;
        const double m11 = I.c + I.d00 * L1, m22 = I.c + I.d01 * L1;
        const double m12 = -ca * I.d01, m21 = -ca * I.d00;
        const double idet = 1.0 / (m11 * m22 - m12 * m21);
        const double i00 = m22 * idet, i01 = -m12 * idet, i10 = -m21 * idet, i11 = m11 * idet;
        // g = Minv (E - D S), D = [[L1, -a], [-a, L1]]: coefficients of S
        const double s00 = ca * i01 - L1 * i00, s01 = ca * i00 - L1 * i01;
        const double s10 = ca * i11 - L1 * i10, s11 = ca * i10 - L1 * i11;
        const double i_own = ck ? i11 : i00, i_oth = ck ? i10 : i01;
        const double g0own = ck ? g01 : g00, g0oth = ck ? g00 : g01;
        const double P = fma(i_oth, g0oth, i_own * g0own);  // own row of Minv g^{n-1}
        cst[0][lane] = ck ? s11 : s00;  // own and other coefficient of S
        cst[1][lane] = ck ? s10 : s01;
        cst[2][lane] = i_own;
        cst[3][lane] = i_oth;
        cst[4][lane] = P;               // Minv g^{n-1}
        cst[5][lane] = P;               // Minv g^{n-2}, g^{-1} := g^0
        cst[6][lane] = g0own;           // newest level
    }

    d4 H[NTW];
#pragma unroll
    for (int q = 0; q < NTW; ++q) H[q] = d4{0.0, 0.0, 0.0, 0.0};
    // the first tile's table fragments (then always one tile ahead)
    double w0[4], r0[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        w0[i] = Wb[unsigned(i * 64) + ul];
        r0[i] = Rb[unsigned(i * 64) + ul];
    }
    __syncthreads();

    // the levels of steps n0c+1..n0c+btc (ring slots that the next three
    // blocks leave alone) to p.tcols: wave w writes modes 4w..4w+3 of both
    // components, lane 16u + b step b of mode 4w + u (a wave-uniform base and
    // a small lane offset keep the addresses out of the loop's registers)
    auto put_cols = [&](int64_t n0c, int btc) {
        const int u = lane >> 4, b = lane & 15;
        if (b < btc && mode0 + 4 * wave + u < M) {
#pragma unroll
            for (int kk = 0; kk < 2; ++kk) {
                double* base = p.tcols + (2 * I.mode_off + kk * M + mode0 + 4 * wave) * p.tcn + p.tcb +
                               p.tcd * (n0c + 1);
                base[int64_t(u) * p.tcn + p.tcd * b] = ring[(n0c + 1 + b) & 63][kk][4 * wave + u];
            }
        }
    };

    for (int64_t n0 = 0; n0 < N; n0 += B) {
        const int bt = (N - n0 < B) ? int(N - n0) : B;  // steps of this block
        if constexpr (COLS) {
            if (p.tcols && n0 > 0) put_cols(n0 - B, B);
        }
        // ---- phase A: the state advanced over this block (its inputs are
        // levels <= n0) and its part of the next block's fast sums; this
        // block's in-block Toeplitz term, window of the earlier levels and
        // starting correction
        {
            double gin[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) gin[i] = ring[(n0 + 1 + 4 * i + lk - L) & 63][k][li];
            // table fragments of tile q at a wave-uniform address (a tile past
            // the problem's nodes reads the zero tile NT, so it stays zero and
            // adds nothing); the bases pass through an empty asm statement
            // each block, so that no per-tile address is kept live across the
            // time loop
            const gdouble* Wq = (const gdouble*)(Wb);
            const gdouble* Rq = (const gdouble*)(Rb);
            asm volatile("" : "+s"(Wq), "+s"(Rq));
            auto ld = [&](int q, double (&aw)[4], double (&ar)[4]) {
                const int jt = (h + 2 * q < NT) ? h + 2 * q : NT;
                const gdouble* __restrict__ wt = Wq + jt * 256;
                const gdouble* __restrict__ rt = Rq + jt * 256;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    aw[i] = wt[unsigned(i * 64) + ul];
                    ar[i] = rt[unsigned(i * 64) + ul];
                }
            };
            d4 S = d4{0.0, 0.0, 0.0, 0.0};
            // The tiles in order, the table fragments of the next tile loaded
            // while a tile computes (after the last tile, the first tile of
            // the next block: the tables are the same for every block); the
            // compiler barriers keep later loads from moving earlier. Tile q's
            // advance is interleaved with the sums of tile q-1, whose advance
            // has completed.
            if constexpr (NTW > 18) {
                // fewer registers for the largest template: the R fragments
                // one tile ahead, the W fragments of tile q-1 loaded again
                // (a cache hit) for its sums after the advance of tile q
                auto ldw = [&](int q, double (&aw)[4]) {
                    const int jt = (h + 2 * q < NT) ? h + 2 * q : NT;
                    const gdouble* __restrict__ wt = Wq + jt * 256;
#pragma unroll
                    for (int i = 0; i < 4; ++i) aw[i] = wt[unsigned(i * 64) + ul];
                };
                auto ldr = [&](int q, double (&ar)[4]) {
                    const int jt = (h + 2 * q < NT) ? h + 2 * q : NT;
                    const gdouble* __restrict__ rt = Rq + jt * 256;
#pragma unroll
                    for (int i = 0; i < 4; ++i) ar[i] = rt[unsigned(i * 64) + ul];
                };
#pragma unroll
                for (int q = 0; q < NTW; ++q) {
                    asm volatile("" ::: "memory");
                    double r1[4], wq[4];
                    ldr(q + 1 < NTW ? q + 1 : 0, r1);
                    if (q > 0) ldw(q - 1, wq);
                    const int jt = h + 2 * q;
#pragma unroll
                    for (int i = 0; i < 4; ++i) H[q][i] *= rbt[k][jt * 16 + 4 * i + lk];
#pragma unroll
                    for (int i = 0; i < 4; ++i) H[q] = mfma16x16x4(r0[i], gin[i], H[q]);
                    if (q > 0) {
#pragma unroll
                        for (int i = 0; i < 4; ++i) S = mfma16x16x4(wq[i], H[q - 1][i], S);
                    }
#pragma unroll
                    for (int i = 0; i < 4; ++i) r0[i] = r1[i];
                }
                double wq[4];
                ldw(NTW - 1, wq);
#pragma unroll
                for (int i = 0; i < 4; ++i) S = mfma16x16x4(wq[i], H[NTW - 1][i], S);
            } else {
                double wp[4];
    #pragma unroll
                for (int q = 0; q < NTW; ++q) {
                    asm volatile("" ::: "memory");
                    double w1[4], r1[4];
                    ld(q + 1 < NTW ? q + 1 : 0, w1, r1);
                    const int jt = h + 2 * q;
                    // advanced in place: h^{n0+B} = r^B h^{n0} + R Gin; the next
                    // block's sums read the new state
    #pragma unroll
                    for (int i = 0; i < 4; ++i) H[q][i] *= rbt[k][jt * 16 + 4 * i + lk];
    #pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        H[q] = mfma16x16x4(r0[i], gin[i], H[q]);
                        if (q > 0) S = mfma16x16x4(wp[i], H[q - 1][i], S);
                    }
    #pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        wp[i] = w0[i];
                        w0[i] = w1[i];
                        r0[i] = r1[i];
                    }
                }
    #pragma unroll
                for (int i = 0; i < 4; ++i) S = mfma16x16x4(wp[i], H[NTW - 1][i], S);
            }
            const int nb = int((n0 / B + 1) & 1);  // the next block's slot
#pragma unroll
            for (int i = 0; i < 4; ++i) fW[nb][wave][lk + 4 * i][li] = S[i];
            asm volatile("" ::: "memory");
            d4 T = d4{0.0, 0.0, 0.0, 0.0};
            if (h == 1) {
                double df[8], gp[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    df[i] = Dk[unsigned(i * 64) + ul];
                    gp[i] = ring[(n0 - 4 * i - lk) & 63][k][li];
                }
#pragma unroll
                for (int i = 0; i < 8; ++i) T = mfma16x16x4(df[i], gp[i], T);
            } else {
                double cf[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) cf[i] = Ck[unsigned(i * 64) + ul];
#pragma unroll
                for (int i = 0; i < 4; ++i) T = mfma16x16x4(cf[i], gin[i], T);
                if (bdf2 && !ADJ) {
                    const int64_t mA = (mode0 + li < M) ? mode0 + li : M - 1;
                    const double g0A = p.g0[2 * I.mode_off + k * M + mA];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int64_t ix = (n0 + 4 * i + lk <= dlast) ? n0 + 4 * i + lk : dlast;
                        T[i] = fma(0.5 * dkA[ix], g0A, T[i]);
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) fT[wave][lk + 4 * i][li] = T[i];
        }
        __syncthreads();
        // ---- phase B: the block's steps (wave 0)
        if (wave == 0) {
            const double s_own = cst[0][lane], s_oth = cst[1][lane];
            const double i_own = cst[2][lane], i_oth = cst[3][lane];
            double Pk = cst[4][lane], Qk = cst[5][lane], glast = cst[6][lane];
            const int cb = int((n0 / B) & 1);  // this block's slot
            double pend[B / 2];
#pragma unroll
            for (int m = 0; m < B / 2; ++m) {
                const int b = 2 * m + ce;
                pend[m] = (fW[cb][2 * ck][b][cp] + fW[cb][2 * ck + 1][b][cp]) +
                          (fT[2 * ck][b][cp] + fT[2 * ck + 1][b][cp]);
            }
            if (ADJ && n0 == 0 && ce == 0 && mode0 + cp < M)
                pend[0] -= p.g0[2 * I.mode_off + ck * M + mode0 + cp];  // the cotangent enters step 1
            const double* dl = dtab[ck] + ce;  // dl[j]: weight of lag j + e
            const uint32_t toff = uint32_t(2 * I.mode_off + ck * M + mode0 + cp);  // trajectory place
#pragma unroll
            for (int b = 0; b < B; ++b) {
                if (b < bt) {
                    // the step's sum sits in the lane of its parity; quad_perm
                    // [0,0,2,2] / [1,1,3,3] give it to both lanes of the component
                    const double Sk = (b & 1) ? dpp_zero<0xF5>(pend[b >> 1]) : dpp_zero<0xA0>(pend[b >> 1]);
                    const double Ek = fma(e1, Pk, e2 * Qk);
                    double gk, go, ok;  // the new level, the other component's value, this lane's output
                    if constexpr (ADJ) {
                        // r = E - S, mu = Minv^T r, psi = Dm mu (s_own, s_oth:
                        // column k of Minv; i_own, i_oth: L1 and -a)
                        const double rk = Ek - Sk;
                        const double ro = dpp_zero<0x4E>(rk);
                        ok = fma(s_oth, ro, s_own * rk);
                        go = dpp_zero<0x4E>(ok);
                        gk = fma(i_oth, go, i_own * ok);
                    } else {
                        const double So = dpp_zero<0x4E>(Sk);  // the other component's
                        gk = fma(s_oth, So, fma(s_own, Sk, Ek));
                        go = dpp_zero<0x4E>(gk);
                        ok = Sk;
                    }
                    if (ce == 0) ring[(n0 + 1 + b) & 63][ck][cp] = gk;
                    if (TRAJ && ce == 0 && mode0 + cp < M) {
                        // the step's rows at wave-uniform addresses, the lane's
                        // place as a 32-bit offset
                        const int64_t row = (n0 + 1 + b) * p.tstride;
                        p.traj[row + toff] = gk;
                        p.sx[row + toff] = ok;
                    }
                    Qk = Pk;
                    Pk = ADJ ? ok : fma(i_oth, go, i_own * gk);
                    glast = gk;
                    // push into the later steps b' = 2m + e > b, lag b' - b
#pragma unroll
                    for (int m = (b + 1) / 2; m < B / 2; ++m) {
                        const int j = 2 * m - b;  // lag j + e <= B - 1
                        pend[m] = fma(dl[j], gk, pend[m]);
                    }
                }
            }
            cst[4][lane] = Pk;
            cst[5][lane] = Qk;
            cst[6][lane] = glast;
        }
        __syncthreads();
    }
    if constexpr (COLS) {
        if (p.tcols) {
            const int64_t nl = ((N - 1) / B) * B;  // the last block
            put_cols(nl, int(N - nl));
        }
    }
    if (wave == 0 && ce == 0 && mode0 + cp < M) p.gN[2 * I.mode_off + ck * M + mode0 + cp] = cst[6][lane];
}

template <int MODE>
static void launch_mx(const BatchArgs& a, int ntw, hipStream_t st) {
    const dim3 grid(unsigned(a.tiles));
#define CQ_BATCH_MX(T) hipLaunchKernelGGL((k_modal_batch_mx<T, MODE>), grid, dim3(256), 0, st, a)
    switch (ntw) {
        case 4: CQ_BATCH_MX(4); break;
        case 5: CQ_BATCH_MX(5); break;
        case 6: CQ_BATCH_MX(6); break;
        case 7: CQ_BATCH_MX(7); break;
        case 8: CQ_BATCH_MX(8); break;
        case 9: CQ_BATCH_MX(9); break;
        case 10: CQ_BATCH_MX(10); break;
        case 12: CQ_BATCH_MX(12); break;
        case 13: CQ_BATCH_MX(13); break;
        case 14: CQ_BATCH_MX(14); break;
        case 16: CQ_BATCH_MX(16); break;
        case 18:
            if constexpr (MODE == 0) CQ_BATCH_MX(18);
            break;
        default:
            if constexpr (MODE == 0) CQ_BATCH_MX(19);
            break;
    }
#undef CQ_BATCH_MX
}

int launch_modal_batch_mx(const BatchArgs& a, int ntw, hipStream_t st) {
    if (a.traj && ntw > 16) return -1;
    if (a.tcols && (!a.traj || ntw >= kMxColsNtw)) return -1;  // no per-step output template beyond 16 tiles per wave
    prof_begin(9, st);
    if (!a.traj)
        launch_mx<0>(a, ntw, st);
    else if (!a.adj)
        launch_mx<1>(a, ntw, st);
    else
        launch_mx<2>(a, ntw, st);
    prof_end(9, st);
    return 0;
}

}  // namespace cqfp
