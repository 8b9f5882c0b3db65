// gfx950 kernels of a diagonalized waveform-relaxation sweep whose time axis
// is not a power of two (any even N up to 2048; also N = 2, 4): the residual
// (or direct-form right-hand side) in FP64, and the forward / inverse time DFTs
// of length N by Bluestein's chirp-z identity on power-of-two LDS FFTs.  The
// spatial passes between them are the ones of every other sweep: they work on
// the N/2+1 retained frequency planes whatever N is.
#include "pint_device.h"

namespace pint {
namespace {

constexpr int kGenNT = 256;

// ---------------------------------------------------------------------------
// Residual / right-hand side, kappa-scaled (Step 1 before the transform):
//   residual  r_q = G_q - tau^{-alpha} sum_{j=0..q} w_j U_{q-j} - A_h U_q
//   direct    F_q = G_q + kappa tau^{-alpha} sum_{j=q+1..N-1} w_j U_{N+q-j}
// with G_q = f(t_{q+1}) + Table 1 corrections (q < k-1) + tau^{-alpha} s_q v,
// rows q = 0..N-1 holding t_1..t_N, and the result kappa^{q/N} r_q written to
// Rb [N][M] (FP64).  A workgroup owns W consecutive dofs: their N time levels
// and the weights w_0..w_{N-1} are staged in LDS, so the history sums read LDS
// only; stencil neighbours come from global memory (L2).
// The residual of dof d at row q from its level u = U_q[d] and the history sum
// h = sum_{j<=q} w_j U_{q-j}[d] (residual form), or the direct-form
// right-hand side with c = sum_{j>q} w_j U_{N+q-j}[d] in h; written to Rb.
// 1D P1 elements: (Mt x)_d with Mt = tridiag(1, 4, 1)/6 and zero Dirichlet values.
__device__ __forceinline__ double mass_row(const double* x, int d, int m) {
    return (4.0 * x[d] + (d > 0 ? x[d - 1] : 0.0) + (d + 1 < m ? x[d + 1] : 0.0)) * (1.0 / 6.0);
}

// A value at (row q, dof d) of the history sums' input: U, or Mt U for P1 elements.
__device__ __forceinline__ double hist_input(const GenArgs& a, int q, int d) {
    const double* Uq = a.U + (size_t)q * a.M;
    return a.fem ? mass_row(Uq, d, a.mx) : Uq[d];
}

__device__ __forceinline__ void gn_resid_point(const GenArgs& a, int q, int d, double u, double h) {
    const size_t M = a.M;
    double r = a.v ? a.ta * a.s[q] * (a.fem ? mass_row(a.v, d, a.mx) : a.v[d]) : 0.0;
    if (a.f) r += a.f[(size_t)(q + 1) * M + d];
    if (q < a.ncorr) r += a.corr[(size_t)q * M + d];
    if (a.nl) {
        const double vd = a.v ? a.v[d] : 0.0;
        r -= a.c3 * u * u * u + a.c1 * u;
        if (q < a.ncorr) r -= a.an[q] * (a.c3 * vd * vd * vd + a.c1 * vd);
    }
    if (a.dvar) r -= a.dvar[d] * u;
    if (a.form == 0) {
        const int x = d % a.mx, rr = d / a.mx, y = rr % a.my, z = rr / a.my;
        const double* Uq = a.U + (size_t)q * M;
        const size_t sy = (size_t)a.mx, sz = (size_t)a.mx * a.my;
        double nb = a.ihx2 * ((x > 0 ? Uq[d - 1] : 0.0) + (x < a.mx - 1 ? Uq[d + 1] : 0.0));
        if (a.my > 1) nb += a.ihy2 * ((y > 0 ? Uq[d - sy] : 0.0) + (y < a.my - 1 ? Uq[d + sy] : 0.0));
        if (a.mz > 1) nb += a.ihz2 * ((z > 0 ? Uq[d - sz] : 0.0) + (z < a.mz - 1 ? Uq[d + sz] : 0.0));
        r += nb - 2.0 * (a.ihx2 + a.ihy2 + a.ihz2) * u - a.ta * h;
    } else {
        r += a.kappa * a.ta * h;
    }
    a.Rb[(size_t)q * M + d] = a.raw ? r : r * a.scale[q];
}

// Short histories (BDF-k) and the direct form: a workgroup owns W consecutive
// dofs; their N time levels and the weights w_0..w_{N-1} are staged in LDS and
// the sums read LDS only; stencil neighbours come from global memory (L2).
// For P1 elements the staged levels are Mt U (the history carries the mass).
// Tiles t0, t0 + tstride, ... of the problem (every workgroup of a grid, or one
// workgroup per tile); gl: N (W + 1) doubles of LDS.
__device__ __forceinline__ void gn_resid_body(const GenArgs& a, int W, int t0, int tstride, double* gl) {
    const int N = a.N;
    const size_t M = a.M;
    double* om = gl;            // [N]
    double* tl = gl + N;        // [N][W]
    const int tid = threadIdx.x;
    const int ntiles = (a.M + W - 1) / W;
    for (int j = tid; j < N; j += kGenNT) om[j] = j <= a.jmax ? a.w[j] : 0.0;
    for (int tile = t0; tile < ntiles; tile += tstride) {
        const int d0 = tile * W;
        __syncthreads();   // the previous tile's sums are done with tl
        for (int idx = tid; idx < N * W; idx += kGenNT) {
            const int q = idx / W, d = d0 + idx % W;
            tl[idx] = d < a.M ? hist_input(a, q, d) : 0.0;
        }
        __syncthreads();
        for (int idx = tid; idx < N * W; idx += kGenNT) {
            const int q = idx / W, wl = idx % W, d = d0 + wl;
            if (d >= a.M) continue;
            double h = 0.0;
            if (a.form == 0) {
                const int top = q < a.jmax ? q : a.jmax;
                for (int j = 0; j <= top; ++j) h += om[j] * tl[(q - j) * W + wl];
            } else {
                const int top = a.jmax < N - 1 ? a.jmax : N - 1;
                for (int j = q + 1; j <= top; ++j) h += om[j] * tl[(N + q - j) * W + wl];
            }
            gn_resid_point(a, q, d, a.fem ? a.U[(size_t)q * M + d] : tl[q * W + wl], h);
        }
    }
}

__global__ __launch_bounds__(kGenNT) void k_gn_resid(GenArgs a, int W) {
    extern __shared__ double gl[];
    gn_resid_body(a, W, blockIdx.x, gridDim.x, gl);
}

// Residual form with a short history (BDF-k: w_j = 0 beyond j = k <= 6): one lane
// per dof and a chunk of kGnQC rows, the k levels before the chunk and then each
// row's level held in registers (no LDS; consecutive lanes read consecutive
// dofs).  Same sums, in the same order, as the tile kernel below.
constexpr int kGnQC = 32;
__global__ __launch_bounds__(kGenNT) void k_gn_resid_short(GenArgs a) {
    const int d = blockIdx.x * kGenNT + threadIdx.x;
    if (d >= a.M) return;
    const int q0 = blockIdx.y * kGnQC, q1 = min(a.N, q0 + kGnQC);
    double w[7], hist[7];   // hist[j]: the history input at row q - j (zero before row 0)
#pragma unroll
    for (int j = 0; j < 7; ++j) w[j] = j <= a.jmax ? a.w[j] : 0.0;
    hist[0] = 0.0;
#pragma unroll
    for (int j = 1; j < 7; ++j) hist[j] = (j <= a.jmax && q0 - j >= 0) ? hist_input(a, q0 - j, d) : 0.0;
    for (int q = q0; q < q1; ++q) {
        hist[0] = hist_input(a, q, d);
        double h = 0.0;
#pragma unroll
        for (int j = 0; j < 7; ++j) h += w[j] * hist[j];
        gn_resid_point(a, q, d, a.fem ? a.U[(size_t)q * a.M + d] : hist[0], h);
#pragma unroll
        for (int j = 6; j > 0; --j) hist[j] = hist[j - 1];
    }
}

// Dofs per tile of the direct-sum residual: the N weights and the N x W tile of
// levels within 64 KB of LDS.
__host__ __device__ inline int gn_resid_width(int N) {
    int W = 16;
    while (W > 1 && (size_t)N * (W + 1) * sizeof(double) > 65536) W /= 2;
    return W;
}

// Residual form with the full CQ history (a.wh set): the causal sums of a tile
// of 2B dofs by one linear convolution per pair of dofs (dof d0 + 2j in the real
// part, d0 + 2j + 1 in the imaginary part; the weights are real), zero-padded
// to P = 2^LOGP >= 2N - 1 points so that no wrap-around reaches rows q < N:
// h = IFFT_P(Wh . FFT_P(u)), Wh = FFT_P(omega, 0)/P.  This is the circulant
// embedding of the lower-triangular Toeplitz history product (Sec. 3, cost of
// Step 1), O(N log N) per dof instead of O(N^2).  For P1 elements the
// convolved levels are Mt U.  sm: P B complex of LDS.
template <int LOGP, int B>
__device__ __forceinline__ void gn_resid_fft_body(const GenArgs& a, int t0, int tstride, double2* sm) {
    constexpr int P = 1 << LOGP;
    constexpr int W = 2 * B;
    const int N = a.N;
    const size_t M = a.M;
    const int tid = threadIdx.x;
    const int ntiles = (a.M + W - 1) / W;
    for (int tile = t0; tile < ntiles; tile += tstride) {
        const int d0 = tile * W;
        for (int idx = tid; idx < P * B; idx += kGenNT) {
            const int t = idx / B, d = d0 + 2 * (idx % B);
            double2 z = mk<double2>(0.0, 0.0);
            if (t < N) {
                if (d < a.M) z.x = hist_input(a, t, d);
                if (d + 1 < a.M) z.y = hist_input(a, t, d + 1);
            }
            sm[idx] = z;
        }
        __syncthreads();
        lds_fft<double, LOGP, B, kGenNT, false, true, 0>(sm, a.twh);
        for (int idx = tid; idx < P * B; idx += kGenNT) sm[idx] = cmul(sm[idx], a.wh[idx / B]);
        __syncthreads();
        lds_fft<double, LOGP, B, kGenNT, true, true, 0>(sm, a.twh);
        for (int idx = tid; idx < N * W; idx += kGenNT) {
            const int q = idx / W, wl = idx % W, d = d0 + wl;
            if (d >= a.M) continue;
            const double2 hz = sm[q * B + (wl >> 1)];
            gn_resid_point(a, q, d, a.U[(size_t)q * M + d], (wl & 1) ? hz.y : hz.x);
        }
        __syncthreads();   // the next tile overwrites sm
    }
}

// Dof pairs per tile of the convolution residual: the [P][B] tile within 64 KB.
template <int LOGP> constexpr int gn_hist_pairs() {
    const int b = 65536 / ((1 << LOGP) * (int)sizeof(double2));
    return b > 16 ? 16 : (b < 1 ? 1 : b);
}

template <int LOGP>
__global__ __launch_bounds__(kGenNT) void k_gn_resid_fft(GenArgs a) {
    __shared__ double2 sm[(1 << LOGP) * gn_hist_pairs<LOGP>()];
    gn_resid_fft_body<LOGP, gn_hist_pairs<LOGP>()>(a, blockIdx.x, gridDim.x, sm);
}

template <int LOGP>
hipError_t gn_resid_fft_one(const GenArgs& a, hipStream_t st) {
    constexpr int W = 2 * gn_hist_pairs<LOGP>();
    const void* fn = reinterpret_cast<const void*>(&k_gn_resid_fft<LOGP>);
    const long long ntiles = ((long long)a.M + W - 1) / W;
    const long long grid = std::max<long long>(1, std::min<long long>(ntiles, persistent_blocks(fn, kGenNT)));
    PINT_LAUNCH(k_gn_resid_fft<LOGP>, dim3((unsigned)grid), dim3(kGenNT), 0, st, a);
    return hipGetLastError();
}

hipError_t gn_resid_fft_dispatch(const GenArgs& a, hipStream_t st) {
    switch (a.logP) {
        case 2: return gn_resid_fft_one<2>(a, st);
        case 3: return gn_resid_fft_one<3>(a, st);
        case 4: return gn_resid_fft_one<4>(a, st);
        case 5: return gn_resid_fft_one<5>(a, st);
        case 6: return gn_resid_fft_one<6>(a, st);
        case 7: return gn_resid_fft_one<7>(a, st);
        case 8: return gn_resid_fft_one<8>(a, st);
        case 9: return gn_resid_fft_one<9>(a, st);
        case 10: return gn_resid_fft_one<10>(a, st);
        case 11: return gn_resid_fft_one<11>(a, st);
        case 12: return gn_resid_fft_one<12>(a, st);
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// Length-N DFT by Bluestein: with c_t = e^{-pi i t^2/N},
//   X_p = sum_q x_q e^{-2 pi i p q/N} = c_p sum_q (x_q c_q) conj(c_{p-q}),
// the linear convolution evaluated by power-of-two FFTs of length P >= 2N-1 in
// LDS against Bh = FFT_P(conj c wrapped around 0)/P (a host table).
// B spectrum slots per workgroup, layout [P][B].
//   forward (!INV): x_q = Rb[q][dof] (real); X_p, p = 0..N/2, goes to the
//                   spectrum (padding slots receive zeros).
//   inverse (INV):  the full spectrum Q_p = conj(Q_{N-p}) is rebuilt from the
//                   retained half (imaginary parts of Q_0, Q_{N/2} dropped);
//                   y_q = sum_p Q_p e^{+2 pi i p q/N} = Re DFT(conj Q)_q, then
//                   delta_q = y_q kappa^{-q/N}/N updates U (residual: U += delta;
//                   direct: U = delta), and each workgroup leaves its
//                   (max |U_m - U_{m-1}|, sum at q = N-1 of the update squared).
// Tiles g0, g0 + gstride, ... of B slots; sm: P B values of LDS, red: 2 x 4
// doubles of LDS.  INV: on return every lane holds the workgroup's (max |U_m -
// U_{m-1}|, sum over q = N-1 of the update squared) in mx_out, s2_out.
// BLUE = false (N = 2^LOGP itself, twx its twiddles): the same transforms by
// one power-of-two FFT of length N, no chirp.
template <typename R, int LOGP, int B, bool INV, bool BLUE = true>
__device__ __forceinline__ void gn_dft_body(const GenArgs& a, int g0, int gstride, cx<R>* sm, double (*red)[kGenNT / 64],
                                            double& mx_out, double& s2_out, const cx<R>* twx = nullptr) {
    using T = cx<R>;
    constexpr int P = 1 << LOGP;
    const int tid = threadIdx.x;
    const int N = a.N;
    const size_t M = a.M;
    const T* cw = reinterpret_cast<const T*>(a.chirp);
    const T* bh = reinterpret_cast<const T*>(a.bh);
    const T* tw = reinterpret_cast<const T*>(a.twP);
    T* S = reinterpret_cast<T*>(a.S);
    const T zero = mk<T>((R)0, (R)0);
    const int ntiles = (a.Mp + B - 1) / B;
    double mx = 0.0, s2 = 0.0;
    bool bad = false;
    for (int g = g0; g < ntiles; g += gstride) {
        const int s0 = g * B;
        for (int idx = tid; idx < P * B; idx += kGenNT) {
            const int t = idx / B, slot = s0 + idx % B;
            T val = zero;
            if (t < N && slot < a.Mp) {
                if constexpr (!INV) {
                    const int d = slot_dof(slot, a.mx, a.mxp, a.Mp);
                    if (d >= 0) val = mk<T>((R)a.Rb[(size_t)t * M + d], (R)0);
                } else {
                    const int p = t <= N / 2 ? t : N - t;
                    T qv = S[(size_t)p * a.ldS + slot];
                    if (p == 0 || 2 * p == N) qv.y = 0;
                    if (t > N / 2) qv.y = -qv.y;     // Q_t = conj(Q_{N-t})
                    val = mk<T>(qv.x, -qv.y);        // DFT input conj(Q_t)
                }
                if (BLUE) val = cmul(val, cw[t]);
            }
            sm[idx] = val;
        }
        __syncthreads();
        if constexpr (BLUE) {
            lds_fft<R, LOGP, B, kGenNT, false, true, 0>(sm, tw);
            for (int idx = tid; idx < P * B; idx += kGenNT) sm[idx] = cmul(sm[idx], bh[idx / B]);
            __syncthreads();
            lds_fft<R, LOGP, B, kGenNT, true, true, 0>(sm, tw);
        } else {
            lds_fft<R, LOGP, B, kGenNT, false, true, 0>(sm, twx);
        }
        if constexpr (!INV) {
            for (int idx = tid; idx < (N / 2 + 1) * B; idx += kGenNT) {
                const int p = idx / B, slot = s0 + idx % B;
                if (slot < a.Mp) S[(size_t)p * a.ldS + slot] = BLUE ? cmul(sm[idx], cw[p]) : sm[idx];
            }
        } else {
            for (int idx = tid; idx < N * B; idx += kGenNT) {
                const int q = idx / B, slot = s0 + idx % B;
                const int d = slot < a.Mp ? slot_dof(slot, a.mx, a.mxp, a.Mp) : -1;
                if (d < 0) continue;
                const T xq = BLUE ? cmul(sm[idx], cw[q]) : sm[idx];
                const double delta = (double)xq.x * a.unscale[q];
                double* up = a.Uw + (size_t)q * M + d;
                const double u = *up;
                const double un = a.form == 0 ? u + delta : delta;
                const double upd = un - u;
                *up = un;
                const double au = fabs(upd);
                bad |= !(au <= 1.0e300);
                mx = au > mx ? au : mx;
                if (q == N - 1) s2 += upd * upd;
            }
        }
        __syncthreads();   // the next tile overwrites sm
    }
    if constexpr (INV) {
        if (bad) mx = __builtin_nan("");
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            mx = nanmax(mx, __shfl_xor(mx, off, 64));
            s2 += __shfl_xor(s2, off, 64);
        }
        if ((tid & 63) == 0) {
            red[0][tid >> 6] = mx;
            red[1][tid >> 6] = s2;
        }
        __syncthreads();
        double m0 = red[0][0], t0 = red[1][0];
        for (int i = 1; i < kGenNT / 64; ++i) {
            m0 = nanmax(m0, red[0][i]);
            t0 += red[1][i];
        }
        mx_out = m0;
        s2_out = t0;
        __syncthreads();   // red is free again
    }
}

template <typename R, int LOGP, int B, bool INV, bool BLUE>
__global__ __launch_bounds__(kGenNT) void k_gn_dft(GenArgs a) {
    __shared__ cx<R> sm[(1 << LOGP) * B];
    __shared__ double red[2][kGenNT / 64];
    double mx = 0.0, s2 = 0.0;
    gn_dft_body<R, LOGP, B, INV, BLUE>(a, blockIdx.x, gridDim.x, sm, red, mx, s2,
                                       reinterpret_cast<const cx<R>*>(a.twN));
    if (INV && threadIdx.x == 0) {
        a.partial[2 * blockIdx.x] = mx;
        a.partial[2 * blockIdx.x + 1] = s2;
    }
}

// Slots per workgroup: the [P][B] tile fits 64 KB of LDS, at most 16 slots.
template <typename R, int LOGP> constexpr int gn_slots() {
    const int b = 65536 / ((1 << LOGP) * (int)sizeof(cx<R>));
    return b > 16 ? 16 : (b < 1 ? 1 : b);
}

// LOGP: log2 of the transform length (Bluestein's P, or N itself when !BLUE).
template <typename R, int LOGP, bool INV, bool BLUE = true>
hipError_t gn_dft_one(const GenArgs& a, int* nb, hipStream_t st) {
    constexpr int B = gn_slots<R, LOGP>();
    const void* fn = reinterpret_cast<const void*>(&k_gn_dft<R, LOGP, B, INV, BLUE>);
    const long long ntiles = ((long long)a.Mp + B - 1) / B;
    long long grid = std::min<long long>(ntiles, persistent_blocks(fn, kGenNT));
    if (INV) grid = std::min<long long>(grid, a.max_partials);
    if (grid < 1) grid = 1;
    PINT_LAUNCH((k_gn_dft<R, LOGP, B, INV, BLUE>), dim3((unsigned)grid), dim3(kGenNT), 0, st, a);
    if (nb) *nb = (int)grid;
    return hipGetLastError();
}

template <typename R, bool INV>
hipError_t gn_dft_dispatch(const GenArgs& a, int* nb, hipStream_t st) {
    if (a.pow2) {
        switch (a.logP - 1) {   // N = P/2
            case 4: return gn_dft_one<R, 4, INV, false>(a, nb, st);
            case 5: return gn_dft_one<R, 5, INV, false>(a, nb, st);
            case 6: return gn_dft_one<R, 6, INV, false>(a, nb, st);
            case 7: return gn_dft_one<R, 7, INV, false>(a, nb, st);
            case 8: return gn_dft_one<R, 8, INV, false>(a, nb, st);
            case 9: return gn_dft_one<R, 9, INV, false>(a, nb, st);
            case 10: return gn_dft_one<R, 10, INV, false>(a, nb, st);
            case 11: return gn_dft_one<R, 11, INV, false>(a, nb, st);
            default: return hipErrorInvalidValue;
        }
    }
    switch (a.logP) {
        case 2: return gn_dft_one<R, 2, INV>(a, nb, st);
        case 3: return gn_dft_one<R, 3, INV>(a, nb, st);
        case 4: return gn_dft_one<R, 4, INV>(a, nb, st);
        case 5: return gn_dft_one<R, 5, INV>(a, nb, st);
        case 6: return gn_dft_one<R, 6, INV>(a, nb, st);
        case 7: return gn_dft_one<R, 7, INV>(a, nb, st);
        case 8: return gn_dft_one<R, 8, INV>(a, nb, st);
        case 9: return gn_dft_one<R, 9, INV>(a, nb, st);
        case 10: return gn_dft_one<R, 10, INV>(a, nb, st);
        case 11: return gn_dft_one<R, 11, INV>(a, nb, st);
        case 12: return gn_dft_one<R, 12, INV>(a, nb, st);
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// Batched sweeps over many 1D problems that share the spectrum precision R and
// the time Bluestein length 2^LOGP: every pass of a sweep is one launch over
// all active problems (their tiles or frequency rows laid end to end), so each
// pass fills the device however small the problems are.  tstart[i] .. tstart[i+1]
// are problem i's blocks (residual and DFT tiles) or lanes (Thomas rows).
__device__ __forceinline__ int batch_owner(const int* __restrict__ start, int n, int x) {
    int lo = 0, hi = n;   // start[lo] <= x < start[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (start[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <int LOGP>
__global__ __launch_bounds__(kGenNT) void k_batch_resid(const Batch1D* __restrict__ descs,
                                                       const int* __restrict__ tstart, int n, int W) {
    extern __shared__ double gl[];
    const int i = batch_owner(tstart, n, blockIdx.x);
    const GenArgs& a = descs[i].ga;
    if (a.wh) {
        gn_resid_fft_body<LOGP, gn_hist_pairs<LOGP>()>(a, blockIdx.x - tstart[i], 1 << 30,
                                                       reinterpret_cast<double2*>(gl));
    } else {
        gn_resid_body(a, W, blockIdx.x - tstart[i], 1 << 30, gl);
    }
}

// Time DFTs of a class: Bluestein on 2^LOGX points (BLUE), or, for a class of
// power-of-two time lengths N = 2^LOGX, one FFT of length N.
template <typename R, int LOGX, int B, bool INV, bool BLUE>
__global__ __launch_bounds__(kGenNT) void k_batch_dft(const Batch1D* __restrict__ descs,
                                                     const int* __restrict__ tstart, int n,
                                                     double* __restrict__ part) {
    __shared__ cx<R> sm[(1 << LOGX) * B];
    __shared__ double red[2][kGenNT / 64];
    const int i = batch_owner(tstart, n, blockIdx.x);
    double mx = 0.0, s2 = 0.0;
    gn_dft_body<R, LOGX, B, INV, BLUE>(descs[i].ga, blockIdx.x - tstart[i], 1 << 30, sm, red, mx, s2,
                                       reinterpret_cast<const cx<R>*>(descs[i].twN));
    if (INV && threadIdx.x == 0) {
        part[2 * blockIdx.x] = mx;
        part[2 * blockIdx.x + 1] = s2;
    }
}

// The Thomas solves of (sigma_p + A_h) Q_p = H_p (diagonal sigma_p + 2/h^2,
// off-diagonals -1/h^2) for the retained frequencies of one problem, without
// pivoting (stable on these diagonally dominant shifted systems), on the
// spectrum rows in place with the modified super-diagonals in the scratch.
// One wave per 64 frequencies, one frequency per lane: chunks of TC equations
// of the 64 rows pass through LDS by coalesced loads and stores (consecutive
// lanes take consecutive equations of a row), each lane runs its row's
// recurrence on registers, and the next chunk's loads are in flight meanwhile
// (issued unconditionally, from a clamped address, so that they overlap).
// Problems of any time length share a launch; bstart[i] .. bstart[i+1] are
// problem i's waves.
template <typename R>
__global__ __launch_bounds__(64) void k_batch_thomas(const Batch1D* __restrict__ descs,
                                                    const int* __restrict__ bstart, int n) {
    using T = cx<R>;
    constexpr int TC = 16;        // equations per chunk
    constexpr int RS = 64 / TC;   // rows per load instruction
    constexpr int LDW = TC + 1;   // row pitch: the lanes' row reads fall on distinct banks
    __shared__ T xs[64 * LDW];
    __shared__ T cs[64 * LDW];
    const int i = batch_owner(bstart, n, blockIdx.x);
    const Batch1D& d = descs[i];
    const int m = d.ga.mx, nP = d.ga.N / 2 + 1;
    const int p0 = (blockIdx.x - bstart[i]) * 64;
    const int lane = threadIdx.x;
    const int rows = nP - p0 < 64 ? nP - p0 : 64;
    const bool live = lane < rows;
    T* S = reinterpret_cast<T*>(d.ga.S) + (size_t)p0 * d.ga.ldS;
    T* C = reinterpret_cast<T*>(d.thomas) + (size_t)p0 * m;
    const size_t ld = d.ga.ldS;
    const R off = (R)(-d.ih2);
    const T zero = mk<T>((R)0, (R)0);
    const double2 sg = d.sigma[live ? p0 + lane : p0];
    const T b = mk<T>((R)(sg.x + 2.0 * d.ih2), (R)sg.y);
    // the lane's share of a chunk: element k is (row lane/TC + k RS, equation
    // i0 + lane%TC).  Raw buffer accesses over the wave's rows (32-bit lane
    // offsets; a lane without an element gets the offset kNoLane, whose load
    // returns 0 and whose store is dropped), so the loads of a chunk issue
    // back to back and only the vector-memory counter tracks them.  The chunk
    // buffers are real and imaginary arrays, which the compiler keeps in
    // registers.
    const int e = lane % TC, r0 = lane / TC;
    const __amdgpu_buffer_rsrc_t rs_S = buf_rsrc(S, (unsigned long long)rows * ld * sizeof(T));
    const __amdgpu_buffer_rsrc_t rs_C = buf_rsrc(C, (unsigned long long)rows * m * sizeof(T));
    auto offs = [&](size_t pitch, int i0, int len, int k) -> unsigned {
        const int r = r0 + k * RS;
        return (r < rows && e < len) ? (unsigned)(((size_t)r * pitch + i0 + e) * sizeof(T)) : kNoLane;
    };
    auto gload = [&](__amdgpu_buffer_rsrc_t rsrc, size_t pitch, int i0, int len, R (&re)[TC], R (&im)[TC]) {
#pragma unroll
        for (int k = 0; k < TC; ++k) {
            const T t = buf_ld(rsrc, offs(pitch, i0, len, k), T{});
            re[k] = t.x;
            im[k] = t.y;
        }
    };
    auto to_lds = [&](T* dst, const R (&re)[TC], const R (&im)[TC]) {
#pragma unroll
        for (int k = 0; k < TC; ++k) dst[(r0 + k * RS) * LDW + e] = mk<T>(re[k], im[k]);
    };
    auto from_lds = [&](__amdgpu_buffer_rsrc_t rsrc, size_t pitch, int i0, int len, const T* src) {
#pragma unroll
        for (int k = 0; k < TC; ++k) buf_st(rsrc, offs(pitch, i0, len, k), src[(r0 + k * RS) * LDW + e]);
    };
    // forward elimination: c_i = off / den_i, x_i = (r_i - off x_{i-1}) / den_i,
    // den_i = b - off c_{i-1} (c_{-1} = x_{-1} = 0)
    T cprev = zero, xprev = zero;
    R bxr[TC], bxi[TC], bcr[TC], bci[TC];
    gload(rs_S, ld, 0, m < TC ? m : TC, bxr, bxi);
    for (int i0 = 0; i0 < m; i0 += TC) {
        const int len = m - i0 < TC ? m - i0 : TC;
        to_lds(xs, bxr, bxi);
        if (i0 + TC < m) gload(rs_S, ld, i0 + TC, m - i0 - TC < TC ? m - i0 - TC : TC, bxr, bxi);
        __syncthreads();
        if (live) {
            T v[TC];
#pragma unroll
            for (int j = 0; j < TC; ++j) v[j] = xs[lane * LDW + j];
#pragma unroll
            for (int j = 0; j < TC; ++j) {
                if (j < len) {
                    const T den = mk<T>(b.x - off * cprev.x, b.y - off * cprev.y);
                    cprev = cdiv(mk<T>(off, (R)0), den);
                    xprev = cdiv(mk<T>(v[j].x - off * xprev.x, v[j].y - off * xprev.y), den);
                    cs[lane * LDW + j] = cprev;
                    xs[lane * LDW + j] = xprev;
                }
            }
        }
        __syncthreads();
        from_lds(rs_S, ld, i0, len, xs);
        from_lds(rs_C, (size_t)m, i0, len, cs);
        __syncthreads();
    }
    // back substitution x_i -= c_i x_{i+1}, chunks from the last one down
    // (x_{m-1} is final: it is the carry xprev)
    int i0 = ((m - 1) / TC) * TC;
    gload(rs_S, ld, i0, m - i0, bxr, bxi);
    gload(rs_C, (size_t)m, i0, m - i0, bcr, bci);
    for (; i0 >= 0; i0 -= TC) {
        const int len = m - i0 < TC ? m - i0 : TC;
        to_lds(xs, bxr, bxi);
        to_lds(cs, bcr, bci);
        if (i0 >= TC) {
            gload(rs_S, ld, i0 - TC, TC, bxr, bxi);
            gload(rs_C, (size_t)m, i0 - TC, TC, bcr, bci);
        }
        __syncthreads();
        if (live) {
#pragma unroll
            for (int j = TC - 1; j >= 0; --j) {
                if (j < len && i0 + j < m - 1) {
                    const T x = xs[lane * LDW + j], c = cs[lane * LDW + j];
                    xprev = mk<T>(x.x - (c.x * xprev.x - c.y * xprev.y), x.y - (c.x * xprev.y + c.y * xprev.x));
                    xs[lane * LDW + j] = xprev;
                }
            }
        }
        __syncthreads();
        from_lds(rs_S, ld, i0, len, xs);
        __syncthreads();
    }
}

// Norms of each problem's update from its inverse-DFT blocks' partials, in a
// fixed order: norms[i] = (max |U_m - U_{m-1}|, (h sum_x (U_m^N - U_{m-1}^N)^2)^{1/2}).
__global__ __launch_bounds__(64) void k_batch_norms(const Batch1D* __restrict__ descs, const int* __restrict__ tstart,
                                                    const double* __restrict__ part, double* __restrict__ norms) {
    const int i = blockIdx.x;
    double mx = 0.0, s2 = 0.0;
    for (int b = tstart[i] + (int)threadIdx.x; b < tstart[i + 1]; b += 64) {
        mx = nanmax(mx, part[2 * b]);
        s2 += part[2 * b + 1];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        mx = nanmax(mx, __shfl_xor(mx, off, 64));
        s2 += __shfl_xor(s2, off, 64);
    }
    if (threadIdx.x == 0) {
        norms[2 * i] = mx;
        norms[2 * i + 1] = sqrt(descs[i].hd * s2);
    }
}

template <typename R, int LOGP, bool INV, bool POW2>
hipError_t batch_pass_one(const BatchLaunch& L, hipStream_t st) {
    constexpr int LOGX = POW2 ? LOGP - 1 : LOGP;   // power-of-two N: P = 2N
    constexpr int B = gn_slots<R, LOGX>();
    if (!INV) {
        const int W = gn_resid_width(L.N);
        const size_t lds = std::max((size_t)L.N * (W + 1) * sizeof(double),
                                    (size_t)(1 << LOGP) * gn_hist_pairs<LOGP>() * sizeof(double2));
        PINT_LAUNCH(k_batch_resid<LOGP>, dim3(L.nres), dim3(kGenNT), lds, st, L.descs, L.res_start, L.n, W);
        PINT_LAUNCH((k_batch_dft<R, LOGX, B, false, !POW2>), dim3(L.ndft), dim3(kGenNT), 0, st, L.descs,
                    L.dft_start, L.n, L.part);
    } else {
        PINT_LAUNCH((k_batch_dft<R, LOGX, B, true, !POW2>), dim3(L.ndft), dim3(kGenNT), 0, st, L.descs,
                    L.dft_start, L.n, L.part);
        PINT_LAUNCH(k_batch_norms, dim3(L.n), dim3(64), 0, st, L.descs, L.dft_start, L.part, L.norms);
    }
    return hipGetLastError();
}

template <typename R, bool INV>
hipError_t batch_pass_dispatch(const BatchLaunch& L, hipStream_t st) {
    if (L.pow2) {
        switch (L.logP) {
            case 5: return batch_pass_one<R, 5, INV, true>(L, st);
            case 6: return batch_pass_one<R, 6, INV, true>(L, st);
            case 7: return batch_pass_one<R, 7, INV, true>(L, st);
            case 8: return batch_pass_one<R, 8, INV, true>(L, st);
            case 9: return batch_pass_one<R, 9, INV, true>(L, st);
            case 10: return batch_pass_one<R, 10, INV, true>(L, st);
            case 11: return batch_pass_one<R, 11, INV, true>(L, st);
            case 12: return batch_pass_one<R, 12, INV, true>(L, st);
            default: return hipErrorInvalidValue;
        }
    }
    switch (L.logP) {
        case 2: return batch_pass_one<R, 2, INV, false>(L, st);
        case 3: return batch_pass_one<R, 3, INV, false>(L, st);
        case 4: return batch_pass_one<R, 4, INV, false>(L, st);
        case 5: return batch_pass_one<R, 5, INV, false>(L, st);
        case 6: return batch_pass_one<R, 6, INV, false>(L, st);
        case 7: return batch_pass_one<R, 7, INV, false>(L, st);
        case 8: return batch_pass_one<R, 8, INV, false>(L, st);
        case 9: return batch_pass_one<R, 9, INV, false>(L, st);
        case 10: return batch_pass_one<R, 10, INV, false>(L, st);
        case 11: return batch_pass_one<R, 11, INV, false>(L, st);
        case 12: return batch_pass_one<R, 12, INV, false>(L, st);
        default: return hipErrorInvalidValue;
    }
}

// g'(Ubar) with Ubar[x] the mean of U over the N time levels (fixed order).
// A workgroup of 16 waves per 64 dofs: wave w sums rows w, w + 16, ... (eight
// loads in flight per lane), then the 16 partial sums combine in wave order.
constexpr int kMeanWaves = 16;
__global__ __launch_bounds__(64 * kMeanWaves) void k_nl_mean_dg(const double* __restrict__ U, double* __restrict__ dg,
                                                               int N, int M, double c3, double c1) {
    __shared__ double part[kMeanWaves][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int d = blockIdx.x * 64 + lane;
    double s = 0.0;
    if (d < M) {
        int n = wv;
        for (; n + 7 * kMeanWaves < N; n += 8 * kMeanWaves) {
            double v[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) v[i] = U[(size_t)(n + i * kMeanWaves) * M + d];
#pragma unroll
            for (int i = 0; i < 8; ++i) s += v[i];
        }
        for (; n < N; n += kMeanWaves) s += U[(size_t)n * M + d];
    }
    part[wv][lane] = s;
    __syncthreads();
    if (wv == 0 && d < M) {
        double t = part[0][lane];
        for (int i = 1; i < kMeanWaves; ++i) t += part[i][lane];
        const double ub = t / N;
        dg[d] = 3.0 * c3 * ub * ub + c1;
    }
}

// U += W over [N][M], with per-workgroup partials (max |W|, sum of W^2 on the
// last time level) for the fixed-order norm reduction.
__global__ __launch_bounds__(kGenNT) void k_nl_axpy(double* __restrict__ U, const double* __restrict__ W,
                                                    double* __restrict__ partial, int N, int M) {
    __shared__ double red[2][kGenNT / 64];
    const long long total = (long long)N * M;
    double mx = 0.0, s2 = 0.0;
    bool bad = false;
    for (long long i = (long long)blockIdx.x * kGenNT + threadIdx.x; i < total; i += (long long)gridDim.x * kGenNT) {
        const double w = W[i];
        U[i] += w;
        const double aw = fabs(w);
        bad |= !(aw <= 1.0e300);
        mx = aw > mx ? aw : mx;
        if (i >= total - M) s2 += w * w;
    }
    if (bad) mx = __builtin_nan("");
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        mx = nanmax(mx, __shfl_xor(mx, off, 64));
        s2 += __shfl_xor(s2, off, 64);
    }
    const int tid = threadIdx.x;
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = mx;
        red[1][tid >> 6] = s2;
    }
    __syncthreads();
    if (tid == 0) {
        double m0 = red[0][0], t0 = red[1][0];
        for (int i = 1; i < kGenNT / 64; ++i) {
            m0 = nanmax(m0, red[0][i]);
            t0 += red[1][i];
        }
        partial[2 * blockIdx.x] = m0;
        partial[2 * blockIdx.x + 1] = t0;
    }
}

}  // namespace

int batch_dft_slots(bool mixed, int logP) {
    const int cb = mixed ? 8 : 16;
    const int b = 65536 / ((1 << logP) * cb);
    return b > 16 ? 16 : (b < 1 ? 1 : b);
}

int batch_resid_width(int N) { return gn_resid_width(N); }

int batch_hist_width(int logP) {
    const int b = 65536 / ((1 << logP) * (int)sizeof(double2));
    return 2 * (b > 16 ? 16 : (b < 1 ? 1 : b));
}

hipError_t launch_batch_forward(const BatchLaunch& L, hipStream_t st) {
    if (L.n < 1) return hipSuccess;
    return L.mixed ? batch_pass_dispatch<float, false>(L, st) : batch_pass_dispatch<double, false>(L, st);
}

hipError_t launch_batch_inverse(const BatchLaunch& L, hipStream_t st) {
    if (L.n < 1) return hipSuccess;
    return L.mixed ? batch_pass_dispatch<float, true>(L, st) : batch_pass_dispatch<double, true>(L, st);
}

hipError_t launch_batch_thomas(const Batch1D* descs, const int* bstart, int n, int nwaves, bool mixed,
                               hipStream_t st) {
    if (n < 1) return hipSuccess;
    if (mixed)
        PINT_LAUNCH((k_batch_thomas<float>), dim3(nwaves), dim3(64), 0, st, descs, bstart, n);
    else
        PINT_LAUNCH((k_batch_thomas<double>), dim3(nwaves), dim3(64), 0, st, descs, bstart, n);
    return hipGetLastError();
}

hipError_t launch_nl_mean_dg(const double* U, double* dg, int N, int M, double c3, double c1, hipStream_t st) {
    PINT_LAUNCH(k_nl_mean_dg, dim3((M + 63) / 64), dim3(64 * kMeanWaves), 0, st, U, dg, N, M, c3, c1);
    return hipGetLastError();
}

hipError_t launch_nl_axpy(double* U, const double* W, double* partial, int N, int M, int max_partials, int* nb,
                          hipStream_t st) {
    const long long total = (long long)N * M;
    const long long want = (total + kGenNT - 1) / kGenNT;
    const int grid = (int)std::max<long long>(1, std::min<long long>(want, std::min(max_partials, 1024)));
    PINT_LAUNCH(k_nl_axpy, dim3(grid), dim3(kGenNT), 0, st, U, W, partial, N, M);
    if (nb) *nb = grid;
    return hipGetLastError();
}

hipError_t launch_gn_resid(const GenArgs& a, hipStream_t st) {
    if (a.wh && a.form == 0) return gn_resid_fft_dispatch(a, st);
    // short histories on grids of >= 128 such workgroups (fewer: the tile kernel,
    // whose lanes share the rows of a tile, is faster; the paper's 999 x 100 runs 16)
    const dim3 sgrid((unsigned)((a.M + kGenNT - 1) / kGenNT), (unsigned)((a.N + kGnQC - 1) / kGnQC));
    if (a.form == 0 && a.jmax <= 6 && (long long)sgrid.x * sgrid.y >= 128) {
        PINT_LAUNCH(k_gn_resid_short, sgrid, dim3(kGenNT), 0, st, a);
        return hipGetLastError();
    }
    // dofs per workgroup: the N x W tile and the N weights within 64 KB of LDS
    const int W = gn_resid_width(a.N);
    const size_t lds = (size_t)a.N * (W + 1) * sizeof(double);
    const void* fn = reinterpret_cast<const void*>(&k_gn_resid);
    const long long ntiles = ((long long)a.M + W - 1) / W;
    const long long grid = std::max<long long>(1, std::min<long long>(ntiles, persistent_blocks(fn, kGenNT)));
    PINT_LAUNCH(k_gn_resid, dim3((unsigned)grid), dim3(kGenNT), lds, st, a, W);
    return hipGetLastError();
}

hipError_t launch_gn_forward(const GenArgs& a, bool mixed, hipStream_t st) {
    return mixed ? gn_dft_dispatch<float, false>(a, nullptr, st) : gn_dft_dispatch<double, false>(a, nullptr, st);
}

hipError_t launch_gn_inverse(const GenArgs& a, bool mixed, int* nb, hipStream_t st) {
    return mixed ? gn_dft_dispatch<float, true>(a, nb, st) : gn_dft_dispatch<double, true>(a, nb, st);
}

}  // namespace pint
