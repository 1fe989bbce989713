// Argument blocks and launchers of the per-step kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cqfp {

struct HistFastArgs {
    int64_t n;            // step being computed (>= 1)
    int64_t L;            // lag of the first quadrature term (2 or N_s)
    int64_t Lr;           // slots in the level store
    int64_t M;            // nodes per component
    int np;               // fast nodes per component
    int chunk;            // nodes per blockIdx.y slice
    int64_t dstride;      // stride between the two components' weights
    const double* levels; // [Lr][2][M]
    double* H;            // [2][np][M]
    const double* ratio;  // [2][np]
    const double* coef;   // [2][np]
    const double* d;      // [2][dstride]
    double* Spart;        // [nsplit][2][M]
};

struct HistDirectArgs {
    int64_t n, n0, M;
    int64_t dstride;
    int B, ks;
    const double* levels;  // [N+1][2][M]
    const double* d;       // [2][dstride]
    const double* F;       // [ks][B][2][M]
    double* Spart;         // [1][2][M]
};

struct FarArgs {
    int64_t n0, M, mchunk, dstride;
    int64_t lstride;       // elements between time levels (2M for a solver)
    int B, ks, ncomp;      // ncomp components (blockIdx.z), offset M apart
    const double* levels;  // level l of component k at levels[l*lstride + k*M]
    const double* d;       // [ncomp][dstride], dstride >= n0 + B + 1
    double* F;             // [ks][B][ncomp][M]
};

struct Solve1DArgs {
    int64_t n, M, Mpad, Lr;
    int nsplit, scheme;
    double inv_tau, cdiag, h2;
    double inv_d0[2];     // 1/d_k,0
    double corr[2];       // BDF2: d_k,n-1 / 2; BE: 0
    double diag[2];       // fl(2 + delta_k)
    double delta[2];      // delta_k = theta_k h^2
    double V[4], Vinv[4]; // row-major 2x2
    const double* Spart;  // [nsplit][2][M]
    const double* G0;     // [2][M]
    double* levels;       // [Lr][2][M]
};

struct Prep2DArgs {
    int64_t n, Lr, M;
    int nsplit, scheme;
    double inv_tau, cdiag;
    double inv_d0[2];
    double corr[2];
    const double* Spart;
    const double* G0;
    const double* levels;
    double* w;  // [2][M]  E + c S'/d0
    double* q;  // [2][M]  S'/d0
};

struct GemmArgs {
    int R, C, K;
    int lda, ldb, ldc;
    int A_shared, B_shared;
    const double *A0, *A1, *B0, *B1;
    double *C0, *C1;
    // per-mode solve epilogue
    const double *lamx, *lamy;
    double cdiag, a, scale;
    double dd0[2];
    // epilogue 2: C_k = A_k B_k - sub_k
    const double *sub0, *sub1;
};

void launch_hist_fast(const HistFastArgs& a, int nsplit, hipStream_t st);
void launch_hist_direct(const HistDirectArgs& a, hipStream_t st);
void launch_far(const FarArgs& a, hipStream_t st);
// out[x] = sum_q F[q][0][0][x] (one history row of a single component)
void launch_reduce_row(const double* F, int ks, int B, int64_t M, double* out, hipStream_t st);
void launch_solve_1d(const Solve1DArgs& a, size_t lds, hipStream_t st);
void launch_prep_2d(const Prep2DArgs& a, hipStream_t st);
void launch_gemm(const GemmArgs& a, int epi, hipStream_t st);
const void* kernel_solve_1d();

// kernel timing (runtime.cpp): no-ops unless cq_prof_enable(1)
void prof_begin(int kind, hipStream_t st);
void prof_end(int kind, hipStream_t st);

}  // namespace cqfp
