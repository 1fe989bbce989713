// HIP kernels (gfx950) of the direct CQ history's far field, (3.8) and
// (3.17): the lags beyond a time block, summed as lower-triangular Toeplitz
// products of the weights with the stored levels on the FP64 matrix cores.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "device_util.h"
#include "kernels.h"

namespace cqfp {

// Workgroups are dispatched to the 8 XCDs in turn (linear id mod 8), each XCD
// with its own L2. Neighbouring DOF tiles share the cache lines at their
// edges (a level row of M doubles is not 128-byte aligned), so the tiles are
// renumbered to give each XCD a contiguous range: the index that XCD x's
// i-th workgroup takes is x*(n/8) + min(x, n mod 8) + i, a bijection of
// [0, n). Returns the tile, slice and component of this workgroup, tile
// fastest.
// (32-bit arithmetic: a launch holds far fewer than 2^31 workgroups; the
// results are wave-uniform and kept in scalar registers.)
__device__ __forceinline__ void far_tile(int64_t& tile, int& q, int& k) {
    const uint32_t nx = gridDim.x, ny = gridDim.y;
    const uint32_t n = nx * ny * gridDim.z;
    const uint32_t lin = blockIdx.x + nx * (blockIdx.y + ny * blockIdx.z);
    const uint32_t x = lin & 7u, i = lin >> 3;
    const uint32_t g = x * (n >> 3) + (x < (n & 7u) ? x : (n & 7u)) + i;
    const uint32_t rest = g / nx;
    tile = int64_t(__builtin_amdgcn_readfirstlane(g - rest * nx));
    const uint32_t qq = rest % ny;
    q = __builtin_amdgcn_readfirstlane(int(qq));
    k = __builtin_amdgcn_readfirstlane(int((rest - qq) / ny));
}

// Sum the K-split partials of the far field once per block, into slice 0:
// F[0][b][k][x] = sum_q F[q][b][k][x].
__global__ __launch_bounds__(256) void k_reduce_far(double* __restrict__ F, int ks, int64_t per) {
    const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (e >= per) return;
    double s = F[e];
    for (int q = 1; q < ks; ++q) s += F[int64_t(q) * per + e];
    F[e] = s;
}

// ---------------------------------------------------------------------------
// Direct history, far field of one time block (FP64 MFMA):
//   F[q][b][k][x] = sum_{l in chunk q} d_k[n0+1+b-l] G_k^l[x],  b < B, l0 <= l <= nl
// (l0 = 1 and nl = n0 for the history; larger nl reaches into the block,
// where the caller's weights read as zero at negative lags). A lower-triangular
// Toeplitz block T[b][l] = d[n0+1+b-l] times the stored levels.
//
// Workgroup: 4 waves on one 64-wide DOF tile; wave w owns the 16 columns
// x0+16w.. and all B rows (NR = B/16 row fragments), so one level operand
// (B fragment, a single 8-byte load per lane) feeds NR MFMAs. The Toeplitz
// A fragments come from LDS: per stage of up to TL levels the weights
// d[n0+1+b-l] of the stage are staged once per workgroup (B + TL values),
// which keeps the vector-memory address unit (the limit of a layout that
// reloads both operands per product) for the levels alone.
// MFMA 16x16x4 f64 operands: A(16x4) lane L -> (row L%16, k L/16);
// B(4x16) lane L -> (k L/16, col L%16); C: item i of lane L is row
// L/16 + 4i, col L%16 (checked on gfx950).
// row fragments from which far_stage reads the next K-step's A fragments
// ahead (measured: 256 rows 84.2% -> 89.5% of the FP64 peak; 128 rows a few
// per cent faster at three waves per SIMD instead of four)
#ifndef CQFP_FAR_APIPE_MIN_NR
#define CQFP_FAR_APIPE_MIN_NR 8
#endif

// One weight stage of the far-field product: the levels s0 .. s1-1 (s0 < s1)
// of the strip G (16 columns per wave) against the weights wt staged for
// them, wt[j] = d[n0+1 - (s1-1) + j], with 16*NR zeros from wt[zero], added
// into acc.
template <int NR>
__device__ __forceinline__ void far_stage(const double* __restrict__ G, int64_t ls, const double* wt, int zero,
                                          int64_t s0, int64_t s1, int li, int lk, d4 (&acc)[NR]) {
    constexpr int U = 4;  // K-steps of 4 levels per batch
    // level operands (the B fragments): one 8-byte load per lane and K-step
    auto loadb = [&](int64_t l0, double (&b_)[U]) {
#pragma unroll
        for (int uu = 0; uu < U; ++uu) {
            const int64_t l = l0 + 4 * uu + lk;
            b_[uu] = G[(l < s1 ? l : s0) * ls];
        }
    };
    // A fragment of row fragment r at level l: wt[(16r + li) + (s1 - 1 - l)],
    // or, for a level past the stage, wt[zero + 16r] in the zero tail (so
    // the row offsets 16r are constants: paired LDS reads); read from LDS
    // just before its products, so no register buffer holds them (four
    // waves fit on a SIMD)
    auto mma = [&](int64_t l0, const double (&b_)[U]) {
#pragma unroll
        for (int uu = 0; uu < U; ++uu) {
            const int64_t l = l0 + 4 * uu + lk;
            const int base_i = l < s1 ? li + int(s1 - 1 - l) : zero;
            double a_[NR];
#pragma unroll
            for (int r = 0; r < NR; ++r) a_[r] = wt[base_i + 16 * r];
#pragma unroll
            for (int r = 0; r < NR; ++r) acc[r] = mfma16x16x4(a_[r], b_[uu], acc[r]);
        }
    };
    // two level buffers in turn: the loads of one batch are in flight
    // while the other's products run
    double bv[U], bw[U];
    loadb(s0, bv);
    if constexpr (NR >= CQFP_FAR_APIPE_MIN_NR) {
        // the A fragments of the next K-step are read while this K-step's
        // products run (two register buffers), so no product waits on the LDS
        double a0[NR], a1[NR];
        auto loada = [&](int64_t l, double (&a_)[NR]) {
            const int base_i = l < s1 ? li + int(s1 - 1 - l) : zero;
#pragma unroll
            for (int r = 0; r < NR; ++r) a_[r] = wt[base_i + 16 * r];
        };
        auto mm = [&](const double (&a_)[NR], double b) {
#pragma unroll
            for (int r = 0; r < NR; ++r) acc[r] = mfma16x16x4(a_[r], b, acc[r]);
        };
        // entering, a0 holds the A fragments of level l0's K-step; leaving,
        // those of level l0 + 16's
        auto mma_p = [&](int64_t l0, const double (&b_)[U]) {
            loada(l0 + 4 + lk, a1);
            mm(a0, b_[0]);
            loada(l0 + 8 + lk, a0);
            mm(a1, b_[1]);
            loada(l0 + 12 + lk, a1);
            mm(a0, b_[2]);
            loada(l0 + 16 + lk, a0);
            mm(a1, b_[3]);
        };
        loada(s0 + lk, a0);
        for (int64_t l0 = s0; l0 < s1; l0 += 8 * U) {
            loadb(l0 + 4 * U, bw);
            __builtin_amdgcn_sched_barrier(0);
            mma_p(l0, bv);
            __builtin_amdgcn_sched_barrier(0);
            loadb(l0 + 8 * U, bv);
            __builtin_amdgcn_sched_barrier(0);
            mma_p(l0 + 4 * U, bw);
            __builtin_amdgcn_sched_barrier(0);
        }
        return;
    }
    for (int64_t l0 = s0; l0 < s1; l0 += 8 * U) {
        loadb(l0 + 4 * U, bw);
        __builtin_amdgcn_sched_barrier(0);
        mma(l0, bv);
        __builtin_amdgcn_sched_barrier(0);
        loadb(l0 + 8 * U, bv);
        __builtin_amdgcn_sched_barrier(0);
        mma(l0 + 4 * U, bw);
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <int NR>
__global__ __launch_bounds__(256) void k_far_toeplitz(FarArgs p) {
    constexpr int TL = 1024;           // levels per weight stage
    constexpr int B = NR * 16;
    constexpr int WS = B + TL + B;     // [B + TL] weights of a stage, then B zeros
    __shared__ double wt[WS];
    int64_t tile;
    int q, k;
    far_tile(tile, q, k);
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t xcol = tile * 64 + wave * 16 + li;
    const bool xin = xcol < p.M;
    const int64_t xc = xin ? xcol : 0;
    const int64_t l_lo = p.l0 + int64_t(q) * p.mchunk;
    const int64_t l_hi = (l_lo + p.mchunk < p.nl + 1) ? l_lo + p.mchunk : p.nl + 1;
    const double* __restrict__ dk = p.d + int64_t(k) * p.dstride;
    const double* __restrict__ G = p.levels + int64_t(k) * p.M + xc;
    d4 acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = d4{0.0, 0.0, 0.0, 0.0};
    for (int64_t s0 = l_lo; s0 < l_hi; s0 += TL) {
        const int64_t s1 = (s0 + TL < l_hi) ? s0 + TL : l_hi;
        // stage: wt[j] = d[n0+1 - (s1-1) + j], j < B + (s1 - s0) - 1; zero after
        const int64_t base = p.n0 + 1 - (s1 - 1);
        const int len = int(B + (s1 - s0) - 1);
        // every load in flight at once (index clamped into the stage's
        // weights; entries past them become zero after the load)
        constexpr int WL = B + TL;  // entries that may hold weights
        double v[(WL + 255) / 256];
#pragma unroll
        for (int t = 0; t < (WL + 255) / 256; ++t) {
            const int j = int(threadIdx.x) + 256 * t;
            v[t] = dk[base + (j < len ? j : len - 1)];
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < (WS + 255) / 256; ++t) {
            const int j = int(threadIdx.x) + 256 * t;
            if (j < WS) wt[j] = (t < (WL + 255) / 256 && j < len) ? v[t < (WL + 255) / 256 ? t : 0] : 0.0;
        }
        __syncthreads();
        far_stage<NR>(G, p.lstride, wt, B + TL, s0, s1, li, lk, acc);
    }
    if (!xin) return;
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int b = 16 * r + lk + 4 * i;
            if (b < p.B) p.F[((int64_t(q) * p.B + b) * p.ncomp + k) * p.M + xcol] = acc[r][i];
        }
}

// The same product for few DOFs, where the 64-column tiles alone cannot fill
// the chip and the levels must be split: KW waves of a workgroup share one
// 16-column strip, each summing its own contiguous part of the workgroup's
// levels (its own weight stages), and the parts are added in LDS, pairwise
// (waves h..2h-1 into waves 0..h-1, h = KW/2, ..., 1), before one store. The
// split therefore costs no HBM traffic inside a workgroup; only the
// workgroup slices along the levels (usually a few) leave
// partial sums for k_reduce_far.
template <int NR, int KW>
__global__ __launch_bounds__(64 * KW) void k_far_toeplitz_kw(FarArgs p) {
    constexpr int TL = NR >= 12 ? 256 : 512;  // levels per weight stage of a wave (registers)
    constexpr int B = NR * 16;
    constexpr int WS = B + TL + B;     // a wave's stage weights, then B zeros
    constexpr int PART = NR * 4 * 64;  // one wave's sums
    constexpr int LDSN = (KW * WS > (KW / 2) * PART) ? KW * WS : (KW / 2) * PART;
    __shared__ double sm[LDSN];
    int64_t tile;
    int q, k;
    far_tile(tile, q, k);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: the level range is scalar
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t xcol = tile * 16 + li;
    const bool xin = xcol < p.M;
    const int64_t xc = xin ? xcol : 0;
    const int64_t g_lo = p.l0 + int64_t(q) * p.mchunk;
    const int64_t g_hi = (g_lo + p.mchunk < p.nl + 1) ? g_lo + p.mchunk : p.nl + 1;
    // this wave's levels: wchunk (a multiple of 4) from g_lo + wave * wchunk
    // (none for a wave past g_hi); the waves meet only for the sums below
    const int64_t wchunk = ((p.mchunk + KW - 1) / KW + 3) / 4 * 4;
    const int64_t l_lo = g_lo + wave * wchunk;
    const int64_t l_hi = (l_lo + wchunk < g_hi) ? l_lo + wchunk : g_hi;
    const double* __restrict__ dk = p.d + int64_t(k) * p.dstride;
    const double* __restrict__ G = p.levels + int64_t(k) * p.M + xc;
    double* wt = sm + wave * WS;
    d4 acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = d4{0.0, 0.0, 0.0, 0.0};
    for (int64_t s0 = l_lo; s0 < l_hi; s0 += TL) {
        const int64_t s1 = (s0 + TL < l_hi) ? s0 + TL : l_hi;
        // stage: wt[j] = d[n0+1 - (s1-1) + j], j < B + (s1 - s0) - 1; zero after.
        // The region is this wave's alone and a wave's LDS operations complete
        // in order, so wave-scope fences (compiler barriers) order the last
        // stage's reads before these writes and these writes before the reads.
        const int64_t base = p.n0 + 1 - (s1 - 1);
        const int len = int(B + (s1 - s0) - 1);
        // (every load in flight at once: the index is clamped into the stage's
        // weights, and entries past them are set to zero after the load)
        constexpr int WL = B + TL;  // entries that may hold weights
        double v[(WL + 63) / 64];
#pragma unroll
        for (int t = 0; t < (WL + 63) / 64; ++t) {
            const int j = lane + 64 * t;
            v[t] = dk[base + (j < len ? j : len - 1)];
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int t = 0; t < (WS + 63) / 64; ++t) {
            const int j = lane + 64 * t;
            if (j < WS) wt[j] = (t < (WL + 63) / 64 && j < len) ? v[t < (WL + 63) / 64 ? t : 0] : 0.0;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        far_stage<NR>(G, p.lstride, wt, B + TL, s0, s1, li, lk, acc);
    }
#pragma unroll
    for (int h = KW / 2; h >= 1; h /= 2) {
        __syncthreads();  // the stage weights (or the last step's sums) are read
        // (one fragment at a time, so that few registers hold the sums in flight)
        if (wave >= h && wave < 2 * h) {
            double* dst = sm + (wave - h) * PART + lane;
#pragma unroll
            for (int r = 0; r < NR; ++r) {
#pragma unroll
                for (int i = 0; i < 4; ++i) dst[(r * 4 + i) * 64] = acc[r][i];
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        __syncthreads();
        if (wave < h) {
            const double* src = sm + wave * PART + lane;
#pragma unroll
            for (int r = 0; r < NR; ++r) {
#pragma unroll
                for (int i = 0; i < 4; ++i) acc[r][i] += src[(r * 4 + i) * 64];
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    if (wave != 0 || !xin) return;
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int b = 16 * r + lk + 4 * i;
            if (b < p.B) p.F[((int64_t(q) * p.B + b) * p.ncomp + k) * p.M + xcol] = acc[r][i];
        }
}

// waves per workgroup of k_far_toeplitz_kw, and its level slices per strip
// relative to the slices ks the caller asked of the 64-column kernel (the
// strips are a quarter as wide, so ks * CQFP_FAR_KW_OVERSUB / KW workgroup
// slices keep ks * CQFP_FAR_KW_OVERSUB waves on each 64 columns)
#ifndef CQFP_FAR_KW
#define CQFP_FAR_KW 4
#endif
#ifndef CQFP_FAR_KW_OVERSUB
#define CQFP_FAR_KW_OVERSUB 1
#endif

void launch_far(const FarArgs& a0, hipStream_t st) {
    FarArgs a = a0;
    prof_begin(2, st);
    if (a.ks > 1 && a.B <= 192) {
        // the levels were to be split over ks workgroup slices: split them over
        // the waves of a workgroup instead, and over fewer workgroup slices
        // (up to 192 rows: the 256-row variant's sums, copied out of the
        // accumulation registers for the LDS step, would leave one wave per SIMD)
        constexpr int KW = CQFP_FAR_KW;
        const int64_t nlev = a.nl - a.l0 + 1;
        const int ksw = std::max(1, std::min(a.ks, (a.ks * CQFP_FAR_KW_OVERSUB + KW / 2) / KW));
        a.ks = ksw;
        a.mchunk = ((nlev + ksw - 1) / ksw + 3) / 4 * 4;
        dim3 grid(unsigned((a.M + 15) / 16), unsigned(ksw), unsigned(a.ncomp));
        switch ((a.B + 63) / 64) {
            case 1: hipLaunchKernelGGL((k_far_toeplitz_kw<4, KW>), grid, dim3(64 * KW), 0, st, a); break;
            case 2: hipLaunchKernelGGL((k_far_toeplitz_kw<8, KW>), grid, dim3(64 * KW), 0, st, a); break;
            default: hipLaunchKernelGGL((k_far_toeplitz_kw<12, KW>), grid, dim3(64 * KW), 0, st, a); break;
        }
    } else {
        dim3 grid(unsigned((a.M + 63) / 64), unsigned(a.ks), unsigned(a.ncomp));
        switch ((a.B + 63) / 64) {
            case 1: hipLaunchKernelGGL(k_far_toeplitz<4>, grid, dim3(256), 0, st, a); break;
            case 2: hipLaunchKernelGGL(k_far_toeplitz<8>, grid, dim3(256), 0, st, a); break;
            case 3: hipLaunchKernelGGL(k_far_toeplitz<12>, grid, dim3(256), 0, st, a); break;
            default: hipLaunchKernelGGL(k_far_toeplitz<16>, grid, dim3(256), 0, st, a); break;
        }
    }
    prof_end(2, st);
    if (a.ks > 1 && a.reduce) {
        const int64_t per = int64_t(a.B) * a.ncomp * a.M;
        prof_begin(10, st);
        hipLaunchKernelGGL(k_reduce_far, dim3(unsigned((per + 255) / 256)), dim3(256), 0, st, a.F, a.ks, per);
        prof_end(10, st);
    }
}

}  // namespace cqfp
