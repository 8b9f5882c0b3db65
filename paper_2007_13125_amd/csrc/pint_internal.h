// Internal declarations shared by the host runtime (pint_host.cpp) and the
// gfx950 kernels (pint_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <string>

#include "../../include/pint.h"

namespace pint {

// Spectrum layout: every frequency plane stores the grid with its x-rows
// padded to mxp = mx rounded up to a multiple of 16 slots (so rows start on a
// 128-byte boundary); slot P of a plane holds dof (P / mxp) * mx + P % mxp when
// P % mxp < mx, and zero otherwise.  Planes are ldS >= Mp = mxp * my * mz apart.

// Everything the first kernel of a sweep (right-hand side / residual, kappa
// scaling, forward time FFT) needs.  All pointers are device pointers.
struct FwdArgs {
    const double* U;        // [N][M] current iterate U_{m-1} (t_1..t_N)
    const double* f;        // [N+1][M] or nullptr (f == 0)
    const double* v;        // [M]
    const double* corr;     // [k-1][M] starting-step corrections, or nullptr
    void* S;                // [N/2+1][ldS] complex spectrum (double2 or float2)
    const double* scale;    // [N] kappa^{q/N}
    const double* s;        // [N] s_n = sum_{j<n} omega_j, n = 1..N
    const void* tw;         // [N] twiddles e^{-2 pi i j/N} in the spectrum precision
    const double* w;        // [N] time weights omega_0..omega_{N-1} (CQ)
    const double2* what;    // [2N] DFT of omega zero-padded to 2N (CQ), FP64
    const double2* tw2;     // [2N] FP64 twiddles for the CQ convolution
    double wk[8];           // omega_0..omega_k, zero beyond k (heat)
    int M, N, k, ldS;
    int mxp, Mp;            // spectrum layout: rows of mxp >= mx slots, Mp slots per plane
    int mx, my, mz;         // grid (my = mz = 1 in lower dimensions)
    double ihx2, ihy2, ihz2;  // 1/h^2 per direction (0 for absent directions)
    double ta;              // tau^{-alpha}
    double kappa;
    int form;               // 0 residual, 1 direct, 2 the source part G alone (U not read)
    int ncorr;              // number of correction rows (k-1, or 0)
    int var;                // forward kernel variant (kFwdVariants; 0 = built-in choice)
    void* Rb;               // [N][Mp] kappa-scaled residual in spectrum-slot layout, in the
                            // spectrum's real type (split forward variant), or nullptr
};

// Inverse time FFT + unscale + update + norm partials.
struct InvArgs {
    double* U;              // [N][M] in/out
    const void* S;          // [N/2+1][ldS] complex spectrum
    const double* unscale;  // [N] kappa^{-q/N} / N
    const void* tw;         // [N] twiddles in the spectrum precision
    double* partial;        // [nblocks][2] (max |delta|, sum delta^2 at q = N-1)
    int M, N, ldS;
    int mx, mxp, Mp;        // grid row length and the padded spectrum layout
    int form;               // 0 residual (U += delta), 1 direct (U = delta)
};

// Sweeps whose time axis is not a power of two (pint_gentime.hip): residual /
// right-hand side into an FP64 buffer, then length-N Bluestein DFTs.
struct GenArgs {
    const double* U;        // [N][M] current iterate (residual kernel)
    double* Uw;             // [N][M] iterate updated in place (inverse kernel)
    const double* f;        // [N+1][M] or nullptr
    const double* v;        // [M]
    const double* corr;     // [k-1][M] starting-step corrections, or nullptr
    double* Rb;             // [N][M] kappa^{q/N}-scaled residual / right-hand side (FP64)
    void* S;                // [N/2+1][ldS] complex spectrum (double2 or float2)
    const double* scale;    // [N] kappa^{q/N}
    const double* unscale;  // [N] kappa^{-q/N} / N
    const double* s;        // [N] s_n
    const double* w;        // [N] time weights omega_0..omega_{N-1} (zero beyond k for BDF-k)
    const void* chirp;      // [N] e^{-pi i t^2/N}, spectrum precision
    const void* bh;         // [P] FFT_P of the conjugate chirp wrapped around 0, divided by P
    const void* twP;        // [P] e^{-2 pi i j/P}
    double* partial;        // [max_partials][2] norm partials of the inverse kernel
    int logP;               // P = 2^logP >= 2N - 1
    int max_partials;
    int M, N, k, ldS, mxp, Mp, mx, my, mz;
    int jmax;               // last nonzero weight index (k for BDF-k, N-1 for CQ)
    double ihx2, ihy2, ihz2, ta, kappa;
    int form;               // 0 residual, 1 direct
    int ncorr;
    // semilinear problems (Algorithm 3): residual of d^alpha u + A u + g(u) = f
    // with g(u) = c3 u^3 + c1 u when nl = 1 (the Table 1 rows then also carry
    // -a_n g(v), a_n from an); dvar, when set, adds diag(dvar) to A_h (the
    // time-averaged Jacobian of the linearised system); raw = 1 writes the
    // residual unscaled (no kappa^{q/N}).
    int nl, raw;
    double c3, c1;
    const double* an;       // [5] a_n of Table 1
    const double* dvar;     // [M] or nullptr
    // residual form with the full CQ history: the causal sums by a zero-padded
    // length-P convolution (nullptr: direct sums)
    const double2* wh;      // [P] FFT_P(omega_0..omega_{N-1}, 0, ..., 0) / P
    const double2* twh;     // [P] e^{-2 pi i j/P} in FP64
    // 1D P1 elements: the scaled mass matrix tridiag(1, 4, 1)/6 multiplies the
    // time-derivative terms (history sums and the s_n v term)
    int fem;
    // N a power of two >= 16 (then P = 2N): the time DFTs are plain length-N
    // FFTs with the twiddles twN = e^{-2 pi i j/N} (spectrum precision)
    int pow2;
    const void* twN;
};

// One 1D problem of a batched sweep (every pass one launch over all active
// problems of a class): its sweep arguments and the Thomas solve's tables.
struct Batch1D {
    GenArgs ga;             // the problem's sweep arguments (U, data, tables, workspace)
    const double2* sigma;   // [N/2+1] tau^{-alpha} d_p
    void* thomas;           // [N/2+1][m] complex scratch in the spectrum precision
    const void* twN;        // [N] e^{-2 pi i j/N}, spectrum precision (power-of-two N)
    double ih2, hd;
};

// One batched sweep over the n active problems of a class (same spectrum
// precision and time Bluestein length 2^logP, and either all of power-of-two
// time length N = 2^(logP-1) >= 16 (pow2: plain FFTs of length N) or none;
// N the largest time length of the class).  Device arrays: descs [n]; res_start / dft_start [n+1] prefix
// sums of each problem's residual tiles / DFT tiles; part [dft_start[n]][2]
// scratch; norms [n][2] out.
struct BatchLaunch {
    const Batch1D* descs;
    const int *res_start, *dft_start;
    double* part;
    double* norms;
    int n, N, logP, nres, ndft;
    bool mixed, pow2;
};

// Spatial shifted solves on the spectrum.
struct SpaceArgs {
    void* S;                // [nP][ldS] complex, in place
    int nP, ldS;
    int mxp;                // slots per spectrum row (grid rows padded to a multiple of 16)
    int dim, mx, my, mz;
    const double2* sigma;   // [nP] tau^{-alpha} d_p
    const double* mu[3];    // sine eigenvalues per axis (FP64)
    const void* twL[3];     // twiddles of length 2(m_a+1) per axis, spectrum precision
    // axes with 2(m_a+1) not a power of two (Bluestein), spectrum precision; logP[a] = 0 otherwise
    int logP[3];            // P_a = 2^logP[a] >= 4(m_a+1) - 1
    const void* chirp[3];   // [2(m_a+1)] e^{-pi i t^2/(2(m_a+1))}
    const void* bh[3];      // [P_a] FFT_P of the conjugate chirp wrapped around 0, divided by P_a
    const void* twP[3];     // [P_a] twiddles e^{-2 pi i j/P_a}
    double ih2[3];          // 1/h^2 per axis
    double inv_factor;      // 1 / prod_a (-2 (m_a + 1)) for the raw DST pair
    int var_rows;           // x-pass variant: 0 = built-in rows per workgroup, 1 = half as many
    int var_cols;           // y/z-pass variant: 0 = built-in column tile, 1 = the other width
    int var_tri;            // 1D with 2(m+1) not a power of two: 0 = Bluestein sine solve,
                            // 1 = PCR/Thomas (built-in split), 2 = PCR/Thomas with more PCR lanes
    const double* dvar;     // 1D only: [m] extra diagonal of the shifted operator (sigma_p + A_h +
                            // diag(dvar)), solved by PCR/Thomas whatever var_tri; or nullptr
    const double* mass;     // 1D P1 elements only: [m] sine eigenvalues of the scaled mass
                            // matrix; the divide is by sigma_p mass_j + mu_j (Bluestein pass); or nullptr
};

// Kernel variants the autotuner chooses between (index 0 is the built-in choice).
//   forward, BDF-k residual 2D/3D: 0 split: a residual kernel that marches along
//     time (one pass over U, the time stencil in registers) into a slot-layout
//     buffer, then a time-FFT kernel (else as 4); 1 march with the time-FFT tile,
//     2 one workgroup per tile, 3 half-width wide-tile march, two workgroups per
//     CU (N in 64..512), 4 wide-tile march along the outer axis when eligible
//     (else 1);
//   forward, CQ: 0 y-march with radix <= 8 transforms when eligible (else 2),
//     1 y-march with radix <= 16, 2 persistent one-tile-at-a-time kernel.
constexpr int kFwdVariants = 5;

// Host-side launchers (defined in pint_kernels.hip).  Each returns the
// hipError_t of the launch; shapes are validated by the caller.
hipError_t launch_prep(const double* v, const double* f, const double* fder, double* corr,
                       const double* a_n, const double* b_ln_tau, int k, int M,
                       int mx, int my, int mz, double ihx2, double ihy2, double ihz2,
                       hipStream_t st);
hipError_t launch_fill(double* U, const double* v, long long N, int M, int zero, hipStream_t st);
hipError_t launch_forward(const FwdArgs& a, bool mixed, bool cq, int* nblocks_out, hipStream_t st);
hipError_t launch_inverse(const InvArgs& a, bool mixed, int* nblocks_out, hipStream_t st);
// Direct form, BDF-k: spectrum of the right-hand side from the stored source
// spectrum Sg and the last k rows of U (replaces launch_forward).
hipError_t launch_inject(const FwdArgs& a, const void* Sg, bool mixed, hipStream_t st);
hipError_t launch_space(const SpaceArgs& a, bool mixed, hipStream_t st);
// General-N sweeps (time axis not a power of two).
hipError_t launch_gn_resid(const GenArgs& a, hipStream_t st);
hipError_t launch_gn_forward(const GenArgs& a, bool mixed, hipStream_t st);
hipError_t launch_gn_inverse(const GenArgs& a, bool mixed, int* nblocks_out, hipStream_t st);
// Batched sweep in three steps: launch_batch_forward (residual, forward time
// DFT) per class, launch_batch_thomas (a Thomas solve per retained frequency)
// over all problems of one precision, whatever their class (bstart [n+1]
// prefix sums of each problem's waves ceil((N_i/2+1)/64), one workgroup of 64
// lanes each), launch_batch_inverse (inverse DFT + update, norms) per class.
// Tiles per problem: residual tiles of batch_hist_width(logP) dofs when its
// history is convolved (ga.wh set), else of batch_resid_width(N) dofs; DFT
// tiles of batch_dft_slots(mixed, pow2 ? logP - 1 : logP) slots.
hipError_t launch_batch_forward(const BatchLaunch& L, hipStream_t st);
hipError_t launch_batch_thomas(const Batch1D* descs, const int* bstart, int n, int nwaves, bool mixed,
                               hipStream_t st);
hipError_t launch_batch_inverse(const BatchLaunch& L, hipStream_t st);
int batch_dft_slots(bool mixed, int logP);
int batch_resid_width(int N);
int batch_hist_width(int logP);
// Sequential-in-time solver: right-hand side of step n into one complex plane
// (slot order), and U^n back from the solved plane.
hipError_t launch_seq_rhs(const GenArgs& a, int n, void* plane, hipStream_t st);
hipError_t launch_seq_store(const GenArgs& a, int n, const void* plane, hipStream_t st);
// Semilinear solves: dg[x] = g'(mean over the N levels of U[.][x]); U += W with
// per-workgroup (max |W|, sum of W^2 at the last level) partials.
hipError_t launch_nl_mean_dg(const double* U, double* dg, int N, int M, double c3, double c1, hipStream_t st);
hipError_t launch_nl_axpy(double* U, const double* W, double* partial, int N, int M, int max_partials, int* nb,
                          hipStream_t st);
int space_pass_count(const SpaceArgs& a);
const char* space_pass_name(const SpaceArgs& a, int pass);
hipError_t launch_space_pass(const SpaceArgs& a, bool mixed, int pass, hipStream_t st);
hipError_t launch_norm_reduce(const double* partial, int nblocks, double hd, double* out,
                              hipStream_t st);
// Whether a variant differs from the built-in choice for this problem (the
// autotuner skips the ones that would launch the same kernel).
bool forward_variant_distinct(const FwdArgs& a, bool mixed, bool cq, int var);
bool rows_variant_distinct(const SpaceArgs& a, bool mixed);
bool cols_variant_distinct(const SpaceArgs& a, bool mixed);

// Largest time-FFT length and DST length the kernels are compiled for.
constexpr int kMaxLogN = 11;      // N <= 2048 (any even N; powers of two >= 8 take the FFT kernels)
constexpr int kMinLogN = 3;       // smallest power of two the FFT kernels take
constexpr int kMaxLogL = 12;      // DST via odd extension of length 2(m+1) <= 4096
constexpr int kMinLogL = 2;
constexpr int kMaxTri1D = 2048;   // 1D tridiagonal systems up to this size

// The sweep loop of pint_solve (host stop test after every sweep); allocates nothing.
pint_status solve_loop(pint_plan* P, double* U, double* upd, double* upd_l2T, int* sweeps);
// Record an error message for pint_last_error and return s.
pint_status set_error(pint_status s, const std::string& msg);
// pint_solve on a workspace lent for this call only (ws_cap bytes at ws); the
// plan's own workspace is restored afterwards and the plan left unbound.
pint_status solve_in_workspace(pint_plan* P, void* ws, size_t ws_cap, const double* v, const double* f,
                               const double* fder, double* U, double* upd, double* upd_l2T, int* sweeps);

}  // namespace pint
