// Argument blocks and launchers of the per-step kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cqfp {

struct HistBlockArgs {
    int64_t n;            // first step of the block (>= 1)
    int64_t L;            // lag of the first quadrature term
    int64_t Lr;           // slots in the level store (>= L)
    int64_t M;            // nodes per component
    int np;               // fast nodes per component
    int chunk;            // nodes per lane of a DOF's lane group
    int BT;               // template block length (>= bt)
    int bt;               // steps in this block (<= L)
    int64_t slot0;        // slot of level n - L: (n - L) mod Lr, in [0, Lr)
    const double* levels; // [Lr][2][M]
    double* H;            // [2][np][hstride]
    int64_t hstride;      // >= M rounded up to 256 (every lane of the pass has a slot)
    const double* ratio;  // [2][np]
    const double* coef;   // [2][np]
    double* Sf;           // [BT][2][M]
};

struct HistDirectArgs {
    int64_t n, n0, M;
    int64_t dstride;
    int B, ks;
    const double* levels;  // [N+1][2][M]
    const double* d;       // [2][dstride]
    const double* F;       // [B][2][M] (slice 0 of the reduced far field)
    double* Spart;         // [1][2][M]
};

struct FarArgs {
    int64_t n0, M, mchunk, dstride;
    int64_t nl;            // levels l0..nl enter (nl = n0 for a history; up to n0 + B, with
                           // d readable, and zero, down to index n0 + 1 - nl)
    int64_t l0 = 1;        // first level (slice q covers l0 + q*mchunk ..)
    int64_t lstride;       // elements between time levels (2M for a solver)
    int B, ks, ncomp;      // ncomp components (blockIdx.z), offset M apart
    int reduce;            // also sum the ks partials into slice 0
    const double* levels;  // level l of component k at levels[l*lstride + k*M]
    const double* d;       // [ncomp][dstride], dstride >= n0 + B + 1
    double* F;             // [ks][B][ncomp][M]
};

// Per-step right-hand side (and, in 1D, the step solve).
struct StepArgs {
    int64_t n, M, Lr;
    int64_t slot1, slot2, slot_out;  // slots of levels n-1, max(n-2,0) and n
    int scheme;
    // history: S' = Sp[boff + k*M + x] + sum_{i<=win} d_i G^{n-i} + corr_k G0
    const double* Sp;
    int64_t boff;
    int win;
    const double* d;      // [2][dstride]
    int64_t dstride;
    double corr[2];       // BDF2: d_k,n-1 / 2; BE: 0
    const double* G0;     // [2][M]
    double* levels;       // [Lr][2][M]
    double inv_tau, cdiag;
    double inv_d0[2];     // 1/d_k,0
    // 1D solve
    double h2;
    double delta[2];      // delta_k = theta_k h^2
    int levels_pcr;       // ceil(log2 M)
    const double *PF, *PG, *PRB;  // PCR multipliers (k_pcr_setup)
    double V[4], Vinv[4]; // row-major 2x2
    // 2D outputs
    double* w;            // [2][M]  E + c S'/d0
    double* q;            // [2][M]  S'/d0
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
    // batch of GEMMs (blockIdx.z): operand b of a per-component A, B or C
    // (and sub) starts sA, sB or sC elements after operand 0; shared
    // operands are not offset
    int batch = 1;
    int64_t sA = 0, sB = 0, sC = 0;
};

struct ModalFastArgs {
    int64_t M;            // modes (nodes per component)
    int64_t n0;           // steps already taken
    int64_t N;            // steps of the whole run (time-blocked kernel: block lengths)
    int nsteps;
    int np, L;            // nodes per component (<= 1024), lag (<= 64)
    int scheme;
    int64_t dstride;
    double inv_tau, c, a;
    double d0[2];
    const double* lam;    // [M]
    const double* ratio;  // [2][np]
    const double* coef;   // [2][np]
    const double* d;      // [2][dstride]
    const double* g0;     // [2][M] sine coefficients of G^0
    double* H;            // [2][np][hstride]
    int64_t hstride;      // DOFs between nodes of H (M here)
    // per-step kernel: [L][2][M], ring[i] = g^{n-1-i} before step n (g^{-1} := g^0);
    // time-blocked kernel (modal_fast_blocked): [2L][2][M], ring[i] = g^{n-i}
    // after n steps (g^0 included, zero below), and H is the state at the
    // start of the L-block that holds step n+1
    double* ring;
};

struct ModalNearArgs {
    int64_t M, n0;        // time block of the far field: steps n0+1 .. n0+B
    int64_t nfirst;       // first step taken here (n0 < nfirst <= n0 + B)
    int bt, scheme;
    int64_t dstride;
    double inv_tau, c, a;
    double d0[2];
    const double* lam;
    const double* d;
    const double* g0;
    // far field of the block, the sum of two parts (either may be NULL =
    // zero): F, rows of a reduced pass over levels 1..n0' (n0' <= n0), and
    // F2, the levels n0'+1..n0 that pass did not see
    const double* F;      // [64][2][M] (row stride 2M)
    const double* F2;     // [64][2][M]
    double* levels;       // [N+1][2][M] coefficients
    // forward: history sums S^n (with BDF2's starting correction) at
    // Sout[n * sstride]; sstride = 0 points every step at one [2][M] scratch row
    double* Sout;         // [N+1][2][M] (or [2][M] with sstride 0)
    int64_t sstride;
    // adjoint sweep (template ADJ): levels hold psi = Dm mu, mu^n goes to mu[n]
    // (mu[0] = 0), and the cotangent gc enters the first step
    double* mu;           // [N+1][2][M]
    const double* gc;     // [2][M]
};

struct ModalWinArgs {
    int64_t M;
    int64_t nfirst;       // first step taken here
    int64_t nblk;         // first step of the block whose Sf is in the buffer
    int bt;               // steps taken here (within that block)
    int L;                // lag (<= 32)
    int64_t Lr;           // slots of the level store (= L)
    int BT;               // Sf[BT][2][M]
    int scheme;
    int64_t dstride;
    double inv_tau, c, a;
    double d0[2];
    const double* lam;
    const double* d;
    const double* g0;
    const double* Sf;
    double* levels;       // [Lr][2][M] coefficients, level l at slot l mod Lr
    double* Sout;         // as in ModalNearArgs
    int64_t sstride;
    double* mu;           // adjoint: [N+1][2][M]
    const double* gc;     // adjoint: [2][M]
};

// Gradient passes of the adjoint (modal coefficients, time-major arrays
// [N+1][2][M]; the adjoint's arrays are in reversed time, index N+1-n).
struct AdjGradArgs {
    int64_t M, N;
    int scheme;
    int64_t dstride;
    double inv_tau;
    double d0[2];          // d_{1,0}, d_{2,0}
    const double* d;       // [2][dstride] exact weights
    const double* traj;    // forward levels g^n
    const double* Sx;      // forward history sums S^n
    const double* mu;      // adjoint mu (reversed)
    const double* psi;     // adjoint psi = Dm mu (reversed)
    double* gG0c;          // [2][M] out: dl/dg^0
    double* part;          // [nchunk][blocks] out: partial sums of sum_n (mu_0 - mu_1).(X_0 - X_1)
    double* gpart;         // [nchunk][2][M] scratch: time-chunk partial sums for dl/dg^0
    int nchunk;            // time chunks (<= N): chunk c covers steps 1 + c per .. min(N, (c+1) per)
    int64_t per;           // steps per chunk
    // k_adj_da: chunks chunk0 .. chunk0 + nchunk_da - 1 only (0: all), so
    // that a run that has one time segment at a time in memory fills the
    // same partial sums as a run over all steps
    int chunk0 = 0, nchunk_da = 0;
};

// d/dbeta pass over one time block n0+1..n0+bt: for each component and mode
//   acc += sum_b psi^n (F[b] + [BDF2] 1/2 dd_{n-1} g^0),
// F[b] = sum_{l=l0}^{n} dw_{n-l} g^l from k_far_toeplitz over levels
// l0..n0+bt (l0 = 1, or the first level of the previous block when the
// farther levels go through block DFTs)
constexpr int kAdjBetaWaves = 16;  // k_adj_beta: waves per 64 columns (slices of a block's steps)
struct AdjBetaArgs {
    int64_t M, N, n0;
    int bt, scheme;
    int64_t dstride;
    const double* dd;      // [2][dstride] d/dbeta of the exact weights
    const double* F;       // [B][2][M] reduced far field of the block
    const double* g0;      // [2][M] g^0 (BDF2's starting-correction term)
    int g0term;            // add that term (once per step n over all calls)
    const double* psi;
    double* acc;           // [2][M]
};

// d/dbeta through block DFTs, block pairs d >= 2: per column e of [2][M]
// (component k = e / M), a_t = psi^{t+1}, b_t = g^{t+1} for t < N, in nb > 2
// blocks of Bk = P/2 steps
constexpr int kSpecMaxLds = 8192;  // nb * P complex doubles (136 KB of LDS with one pad slot per 16)
constexpr int kSpecMaxP = 512;     // blocks of at most 256 steps
// k_beta_spec: distances per thread item, items per workgroup (1024 threads);
// ceil((nb - 2) / kSpecSD) (Bk + 1) <= kSpecItems for every nb, Bk >= 8 with
// nb P <= kSpecMaxLds (at most 1152)
constexpr int kSpecSD = 4, kSpecItems = 2048;
struct BetaSpecArgs {
    int64_t N, M;
    int nb, P, logP;      // P = 2^logP = 2 Bk, nb = ceil(N / Bk), nb P <= kSpecMaxLds
    int cols;             // modes per workgroup (blockIdx.x), component blockIdx.y
    const double* psiT;   // [2M][N] columns a
    const double* gT;     // [2M][N] columns b
    const double* tw;     // [P/2][2] exp(-2 pi i j / P)
    double* spec;         // [2][nwg][(nb-2)(Bk+1)][2] partial block spectra X_{d,f}, d >= 2
};

struct BetaDotArgs {
    int nb, P, nwg;
    const double* spec;   // as in BetaSpecArgs
    const double* W;      // [2][nb (Bk+1)][2] window spectra, every d
    double* part;         // [2][blocks]
};

// one problem of a batch (device table entry)
struct BatchInst {
    int64_t mode_off;     // first mode of the problem in the concatenated arrays
    int64_t M, N;         // modes, steps
    int np, L, scheme, pad;
    int64_t rule_off;     // ratio/coef [2][np] at rule_off
    int64_t d_off;        // weights [2][dstride] at d_off
    int64_t dstride;
    double inv_tau, c, a, d00, d01;
    int64_t mx_off;       // tables of the 16-mode MFMA kernel at mx_off (-1: none)
    int nt, pad2;         // node tiles of 16 per component in those tables
};

struct BatchArgs {
    const BatchInst* inst;
    const int* list;      // problems of this launch
    const int64_t* cum;   // cumulative mode counts over list (cum[0] = 0)
    int count;            // problems in this launch
    int64_t total;        // their modes
    const double *ratio, *coef, *d, *lam, *g0;
    double* gN;
    // 16-mode MFMA kernel: cumulative 16-mode tile counts over list
    // (cumt[0] = 0), their total, and the tables (k_modal_batch_mx)
    const int64_t* cumt;
    int64_t tiles;
    const double* mx;
    // optional per-step output of the MFMA kernel (NULL: none), at
    // [n * tstride + 2 mode_off + k M + mode]: the forward's level g^n (traj)
    // and history sum S^n (sx), or with adj the adjoint's level psi^n (traj)
    // and multiplier mu^n (sx); then g0 holds the cotangent, not G^0
    double* traj;
    double* sx;
    int64_t tstride;
    int adj;
    // optional (with traj; NULL: none): the same levels as time series by
    // place, tcols[place * tcn + tcb + tcd * n] = traj's value of step n
    double* tcols;
    int64_t tcn, tcb;
    int tcd;
};

void launch_modal_fast(const ModalFastArgs& a, hipStream_t st);
void launch_modal_batch(const BatchArgs& a, int npl, int lpm, hipStream_t st);
// 16-mode MFMA kernel: steps per block, lags it takes, node tiles per wave
constexpr int kMxB = 16, kMxMinLag = 16, kMxMaxLag = 33, kMxMaxNtw = 19;
// node tiles per wave from which the per-step variants take no tcols
constexpr int kMxColsNtw = 16;
// doubles of one problem's tables with nt node tiles per component
inline int64_t mx_table_size(int nt) { return int64_t(nt + 1) * 4 * 256 + int64_t(nt) * 32 + 2 * 256 + 2 * 512; }
// ntw: one of 4, 5, 6, 7, 8, 9, 10, 12, 13, 14, 16, 18, 19 (others take 19);
// with per-step output (a.traj) at most 16 and with a.tcols below
// kMxColsNtw, else nothing is launched and -1 returned (0 on a launch)
int launch_modal_batch_mx(const BatchArgs& a, int ntw, hipStream_t st);
bool modal_fast_blocked(int L, int np);  // launch_modal_fast takes the time-blocked kernel
void launch_modal_win(const ModalWinArgs& a, bool adj, hipStream_t st);
void launch_modal_near(const ModalNearArgs& a, int B, bool adj, hipStream_t st);
void launch_adj_g0(const AdjGradArgs& a, hipStream_t st);
// returns the number of partial sums written to a.part (blocks x chunks)
int launch_adj_da(const AdjGradArgs& a, hipStream_t st);
void launch_adj_beta(const AdjBetaArgs& a, hipStream_t st);
// out[k] = sum_x acc[k][x] over blocks: partials [2][blocks]; returns blocks
int launch_sum_rows(const double* acc, int64_t M, double* part, hipStream_t st);
void launch_cols_transpose(const double* src, int64_t row0, int dir, int64_t ncols, int64_t nt, double* dst,
                           hipStream_t st);
void launch_beta_spec(const BetaSpecArgs& a, int nwg, hipStream_t st);
void launch_fft_w(const double* dw, int64_t dwstride, int64_t N, int nb, int P, int logP, const double* tw,
                  double* W, hipStream_t st);
int launch_beta_dot(const BetaDotArgs& a, hipStream_t st);  // returns blocks per component
void launch_hist_block(const HistBlockArgs& a, int lanes, hipStream_t st);
void launch_hist_direct(const HistDirectArgs& a, hipStream_t st);
void launch_far(const FarArgs& a, hipStream_t st);
// One direct history row S[x] = sum_{l=1}^{n-1} d[n-l] G[l*M + x] (x < M),
// the levels split into ks slices (hist_row_slices); with more than one slice
// part holds [ks][M] partial sums (summed in slice order into out). n <= 1
// writes zeros. part_cap: most doubles part may hold (-1: no limit).
int hist_row_slices(int64_t n, int64_t M, int64_t part_cap);
void launch_hist_row(const double* G, int64_t n, int64_t M, const double* d, int ks, double* part, double* out,
                     hipStream_t st);
void launch_step_1d(const StepArgs& a, size_t lds, hipStream_t st);
void launch_prep_2d(const StepArgs& a, hipStream_t st);
void launch_gemm(const GemmArgs& a, int epi, hipStream_t st);
// Separable sine transform of both components of G ([2][M], M = nx ny nz, x
// fastest) on a grid of dim 1, 2 or 3: out = scale * (S_z (x) S_y (x) S_x) G,
// as GEMMs along x (one), y (one per z-plane, batched) and z (one). tmp:
// [2][M] scratch (dim >= 2). S_k: the n_k x n_k sine matrices.
void launch_sine_transform(int dim, int nx, int ny, int nz, const double* Sx, const double* Sy, const double* Sz,
                           const double* G, double* tmp, double* out, double scale, hipStream_t st);
const void* kernel_step_1d(int R);

// kernel timing (runtime.cpp): no-ops unless cq_prof_enable(1)
void prof_begin(int kind, hipStream_t st);
void prof_end(int kind, hipStream_t st);

}  // namespace cqfp
