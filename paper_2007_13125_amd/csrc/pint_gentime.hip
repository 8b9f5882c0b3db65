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
// Tiles t0, t0 + tstride, ... of the problem (every workgroup of a grid, or one
// workgroup walking all tiles of its problem); gl: N (W + 1) doubles of LDS.
__device__ __forceinline__ void gn_resid_body(const GenArgs& a, int W, int t0, int tstride, double* gl) {
    const int N = a.N;
    const size_t M = a.M;
    double* om = gl;            // [N]
    double* tl = gl + N;        // [N][W]
    double* hs = tl + (size_t)N * W;   // [N][W] history sums (long histories only)
    const int tid = threadIdx.x;
    const int ntiles = (a.M + W - 1) / W;
    const double diag = 2.0 * (a.ihx2 + a.ihy2 + a.ihz2);
    for (int j = tid; j < N; j += kGenNT) om[j] = j <= a.jmax ? a.w[j] : 0.0;
    for (int tile = t0; tile < ntiles; tile += tstride) {
        const int d0 = tile * W;
        __syncthreads();   // the previous tile's sums are done with tl
        for (int idx = tid; idx < N * W; idx += kGenNT) {
            const int q = idx / W, d = d0 + idx % W;
            tl[idx] = d < a.M ? a.U[(size_t)q * M + d] : 0.0;
        }
        __syncthreads();
        // Long histories (CQ): the time-stencil sums of QB consecutive rows of one
        // dof are formed together, QB independent accumulators, the weights in a
        // sliding register window; they go to the LDS row of the dof's sums hs.
        constexpr int QB = 8;
        const bool blocked = a.form == 0 && a.jmax >= 16;
        if (blocked) {
            const int nb = (N + QB - 1) / QB;
            for (int it = tid; it < nb * W; it += kGenNT) {
                const int q0 = (it / W) * QB, wl = it % W;
                double acc[QB], win[QB];
#pragma unroll
                for (int r = 0; r < QB; ++r) {
                    acc[r] = 0.0;
                    win[r] = (q0 + r < N && q0 + r <= a.jmax) ? om[q0 + r] : 0.0;   // w_{q0+r-i} at i = 0
                }
                const int iend = q0 + QB < N ? q0 + QB : N;
                for (int i = 0; i < iend; ++i) {
                    const double ui = tl[i * W + wl];
#pragma unroll
                    for (int r = 0; r < QB; ++r)
                        if (i <= q0 + r) acc[r] += win[r] * ui;
                    // next i: w_{q0+r-i-1}: shift the window down, the new low entry
#pragma unroll
                    for (int r = QB - 1; r > 0; --r) win[r] = win[r - 1];
                    const int jn = q0 - i - 1;
                    win[0] = (jn >= 0 && jn <= a.jmax) ? om[jn] : 0.0;
                }
#pragma unroll
                for (int r = 0; r < QB; ++r)
                    if (q0 + r < N) hs[(q0 + r) * W + wl] = acc[r];
            }
            __syncthreads();
        }
        for (int idx = tid; idx < N * W; idx += kGenNT) {
            const int q = idx / W, wl = idx % W, d = d0 + wl;
            if (d >= a.M) continue;
            double r = a.v ? a.ta * a.s[q] * a.v[d] : 0.0;
            if (a.f) r += a.f[(size_t)(q + 1) * M + d];
            if (q < a.ncorr) r += a.corr[(size_t)q * M + d];
            if (a.nl) {
                const double u = tl[q * W + wl], vd = a.v ? a.v[d] : 0.0;
                r -= a.c3 * u * u * u + a.c1 * u;
                if (q < a.ncorr) r -= a.an[q] * (a.c3 * vd * vd * vd + a.c1 * vd);
            }
            if (a.dvar) r -= a.dvar[d] * tl[q * W + wl];
            if (a.form == 0) {
                const int x = d % a.mx, rr = d / a.mx, y = rr % a.my, z = rr / a.my;
                const double* Uq = a.U + (size_t)q * M;
                const size_t sy = (size_t)a.mx, sz = (size_t)a.mx * a.my;
                double nb = a.ihx2 * ((x > 0 ? Uq[d - 1] : 0.0) + (x < a.mx - 1 ? Uq[d + 1] : 0.0));
                if (a.my > 1) nb += a.ihy2 * ((y > 0 ? Uq[d - sy] : 0.0) + (y < a.my - 1 ? Uq[d + sy] : 0.0));
                if (a.mz > 1) nb += a.ihz2 * ((z > 0 ? Uq[d - sz] : 0.0) + (z < a.mz - 1 ? Uq[d + sz] : 0.0));
                double h = 0.0;
                if (blocked) {
                    h = hs[q * W + wl];
                } else {
                    const int top = q < a.jmax ? q : a.jmax;
                    for (int j = 0; j <= top; ++j) h += om[j] * tl[(q - j) * W + wl];
                }
                r += nb - diag * tl[q * W + wl] - a.ta * h;
            } else {
                double c = 0.0;
                const int top = a.jmax < N - 1 ? a.jmax : N - 1;
                for (int j = q + 1; j <= top; ++j) c += om[j] * tl[(N + q - j) * W + wl];
                r += a.kappa * a.ta * c;
            }
            a.Rb[(size_t)q * M + d] = a.raw ? r : r * a.scale[q];
        }
    }
}

__global__ __launch_bounds__(kGenNT) void k_gn_resid(GenArgs a, int W) {
    extern __shared__ double gl[];
    gn_resid_body(a, W, blockIdx.x, gridDim.x, gl);
}

// Dofs per tile of the residual: the N weights and two N x W tiles (levels,
// history sums) within 64 KB of LDS.
__host__ __device__ inline int gn_resid_width(int N) {
    int W = 16;
    while (W > 1 && (size_t)N * (2 * W + 1) * sizeof(double) > 65536) W /= 2;
    return W;
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
template <typename R, int LOGP, int B, bool INV>
__device__ __forceinline__ void gn_dft_body(const GenArgs& a, int g0, int gstride, cx<R>* sm, double (*red)[kGenNT / 64],
                                            double& mx_out, double& s2_out) {
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
                val = cmul(val, cw[t]);
            }
            sm[idx] = val;
        }
        __syncthreads();
        lds_fft<R, LOGP, B, kGenNT, false, true, 0>(sm, tw);
        for (int idx = tid; idx < P * B; idx += kGenNT) sm[idx] = cmul(sm[idx], bh[idx / B]);
        __syncthreads();
        lds_fft<R, LOGP, B, kGenNT, true, true, 0>(sm, tw);
        if constexpr (!INV) {
            for (int idx = tid; idx < (N / 2 + 1) * B; idx += kGenNT) {
                const int p = idx / B, slot = s0 + idx % B;
                if (slot < a.Mp) S[(size_t)p * a.ldS + slot] = cmul(sm[idx], cw[p]);
            }
        } else {
            for (int idx = tid; idx < N * B; idx += kGenNT) {
                const int q = idx / B, slot = s0 + idx % B;
                const int d = slot < a.Mp ? slot_dof(slot, a.mx, a.mxp, a.Mp) : -1;
                if (d < 0) continue;
                const T xq = cmul(sm[idx], cw[q]);
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

template <typename R, int LOGP, int B, bool INV>
__global__ __launch_bounds__(kGenNT) void k_gn_dft(GenArgs a) {
    __shared__ cx<R> sm[(1 << LOGP) * B];
    __shared__ double red[2][kGenNT / 64];
    double mx = 0.0, s2 = 0.0;
    gn_dft_body<R, LOGP, B, INV>(a, blockIdx.x, gridDim.x, sm, red, mx, s2);
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

template <typename R, int LOGP, bool INV>
hipError_t gn_dft_one(const GenArgs& a, int* nb, hipStream_t st) {
    constexpr int B = gn_slots<R, LOGP>();
    const void* fn = reinterpret_cast<const void*>(&k_gn_dft<R, LOGP, B, INV>);
    const long long ntiles = ((long long)a.Mp + B - 1) / B;
    long long grid = std::min<long long>(ntiles, persistent_blocks(fn, kGenNT));
    if (INV) grid = std::min<long long>(grid, a.max_partials);
    if (grid < 1) grid = 1;
    PINT_LAUNCH((k_gn_dft<R, LOGP, B, INV>), dim3((unsigned)grid), dim3(kGenNT), 0, st, a);
    if (nb) *nb = (int)grid;
    return hipGetLastError();
}

template <typename R, bool INV>
hipError_t gn_dft_dispatch(const GenArgs& a, int* nb, hipStream_t st) {
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
// Persistent batch of 1D problems: workgroup i runs the whole solve of problem
// i, sweep after sweep (residual, forward time DFT, one Thomas solve per
// retained frequency, inverse time DFT + update + norms), and stops on its own
// update norm with the rules of the single-problem solve (tolerance, non-finite
// update, growth in two consecutive sweeps beyond the first).  Problems of one
// launch share the spectrum precision R and the time Bluestein length 2^LOGP.
// The Thomas solve of (sigma_p + A_h) Q_p = H_p (diagonal sigma_p + 2/h^2,
// off-diagonals -1/h^2) runs one frequency per lane, without pivoting (stable
// on these diagonally dominant shifted systems), on the spectrum row in place
// with the modified super-diagonal in the scratch.
template <typename R>
__device__ __forceinline__ void thomas_rows(const Batch1D& d) {
    using T = cx<R>;
    const int m = d.ga.mx, nP = d.ga.N / 2 + 1;
    T* S = reinterpret_cast<T*>(d.ga.S);
    T* C = reinterpret_cast<T*>(d.thomas);
    const R off = (R)(-d.ih2);
    for (int p = threadIdx.x; p < nP; p += kGenNT) {
        const double2 sg = d.sigma[p];
        const T b = mk<T>((R)(sg.x + 2.0 * d.ih2), (R)sg.y);
        T* X = S + (size_t)p * d.ga.ldS;
        T* Cp = C + (size_t)p * m;
        T den = b;
        T cprev = cdiv(mk<T>(off, (R)0), den);
        Cp[0] = cprev;
        T xprev = cdiv(X[0], den);
        X[0] = xprev;
        // chunks of CH equations: the chunk's loads are issued together, then the
        // recurrence runs on registers (no memory latency per step)
        constexpr int CH = 16;
        for (int i0 = 1; i0 < m; i0 += CH) {
            T xs[CH];
#pragma unroll
            for (int r = 0; r < CH; ++r) xs[r] = i0 + r < m ? X[i0 + r] : mk<T>((R)0, (R)0);
#pragma unroll
            for (int r = 0; r < CH; ++r) {
                if (i0 + r < m) {
                    den = mk<T>(b.x - off * cprev.x, b.y - off * cprev.y);
                    cprev = cdiv(mk<T>(off, (R)0), den);
                    Cp[i0 + r] = cprev;
                    xprev = cdiv(mk<T>(xs[r].x - off * xprev.x, xs[r].y - off * xprev.y), den);
                    xs[r] = xprev;
                }
            }
#pragma unroll
            for (int r = 0; r < CH; ++r)
                if (i0 + r < m) X[i0 + r] = xs[r];
        }
        // back substitution, chunks from the end (x_{m-1} = xprev already)
        for (int i1 = m - 2; i1 >= 0; i1 -= CH) {
            T xs[CH], cs[CH];
#pragma unroll
            for (int r = 0; r < CH; ++r) {
                const int i = i1 - r;
                xs[r] = i >= 0 ? X[i] : mk<T>((R)0, (R)0);
                cs[r] = i >= 0 ? Cp[i] : mk<T>((R)0, (R)0);
            }
#pragma unroll
            for (int r = 0; r < CH; ++r) {
                if (i1 - r >= 0) {
                    xprev = mk<T>(xs[r].x - (cs[r].x * xprev.x - cs[r].y * xprev.y),
                                  xs[r].y - (cs[r].x * xprev.y + cs[r].y * xprev.x));
                    xs[r] = xprev;
                }
            }
#pragma unroll
            for (int r = 0; r < CH; ++r)
                if (i1 - r >= 0) X[i1 - r] = xs[r];
        }
    }
}

template <typename R, int LOGP>
__global__ __launch_bounds__(kGenNT) void k_batch1d(const Batch1D* __restrict__ descs, int count) {
    constexpr int B = gn_slots<R, LOGP>();
    __shared__ __align__(16) double lds[8192];        // 64 KB: residual tile, then DFT tile
    __shared__ double red[2][kGenNT / 64];
    const int i = blockIdx.x;
    if (i >= count) return;
    const Batch1D& d = descs[i];
    const int W = gn_resid_width(d.ga.N);
    double first = 0.0, prev1 = 0.0, prev2 = 0.0, mx = 0.0, s2 = 0.0;
    int status = 1, m = 0;
    while (m < d.max_sweeps) {
        gn_resid_body(d.ga, W, 0, 1, lds);
        __syncthreads();
        gn_dft_body<R, LOGP, B, false>(d.ga, 0, 1, reinterpret_cast<cx<R>*>(lds), red, mx, s2);
        __syncthreads();
        thomas_rows<R>(d);
        __syncthreads();
        gn_dft_body<R, LOGP, B, true>(d.ga, 0, 1, reinterpret_cast<cx<R>*>(lds), red, mx, s2);
        const double l2 = sqrt(d.hd * s2);
        if (threadIdx.x == 0) {
            d.upd[m] = mx;
            d.upd_l2[m] = l2;
        }
        ++m;
        const double crit = d.norm == 0 ? mx : l2;
        if (!(mx <= 1.0e300) || !(l2 <= 1.0e300)) {
            status = -5;
            break;
        }
        if (m == 1) first = crit;
        if (crit <= d.tol) {
            status = 0;
            break;
        }
        if (m >= 3 && crit > prev1 && prev1 > prev2 && crit > first) {
            status = -5;
            break;
        }
        prev2 = prev1;
        prev1 = crit;
    }
    if (threadIdx.x == 0) {
        d.result[0] = m;
        d.result[1] = status;
    }
}

template <typename R>
hipError_t batch1d_dispatch(const Batch1D* descs, int count, int logP, hipStream_t st) {
    const dim3 g((unsigned)count), b(kGenNT);
    switch (logP) {
        case 2: PINT_LAUNCH((k_batch1d<R, 2>), g, b, 0, st, descs, count); break;
        case 3: PINT_LAUNCH((k_batch1d<R, 3>), g, b, 0, st, descs, count); break;
        case 4: PINT_LAUNCH((k_batch1d<R, 4>), g, b, 0, st, descs, count); break;
        case 5: PINT_LAUNCH((k_batch1d<R, 5>), g, b, 0, st, descs, count); break;
        case 6: PINT_LAUNCH((k_batch1d<R, 6>), g, b, 0, st, descs, count); break;
        case 7: PINT_LAUNCH((k_batch1d<R, 7>), g, b, 0, st, descs, count); break;
        case 8: PINT_LAUNCH((k_batch1d<R, 8>), g, b, 0, st, descs, count); break;
        case 9: PINT_LAUNCH((k_batch1d<R, 9>), g, b, 0, st, descs, count); break;
        case 10: PINT_LAUNCH((k_batch1d<R, 10>), g, b, 0, st, descs, count); break;
        case 11: PINT_LAUNCH((k_batch1d<R, 11>), g, b, 0, st, descs, count); break;
        case 12: PINT_LAUNCH((k_batch1d<R, 12>), g, b, 0, st, descs, count); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// g'(Ubar) with Ubar[x] the mean of U over the N time levels (fixed order).
__global__ __launch_bounds__(kGenNT) void k_nl_mean_dg(const double* __restrict__ U, double* __restrict__ dg, int N,
                                                       int M, double c3, double c1) {
    const int d = blockIdx.x * kGenNT + threadIdx.x;
    if (d >= M) return;
    double s = 0.0;
    for (int n = 0; n < N; ++n) s += U[(size_t)n * M + d];
    const double ub = s / N;
    dg[d] = 3.0 * c3 * ub * ub + c1;
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

hipError_t launch_batch1d(const Batch1D* descs, int count, bool mixed, int logP, hipStream_t st) {
    if (count < 1) return hipSuccess;
    return mixed ? batch1d_dispatch<float>(descs, count, logP, st) : batch1d_dispatch<double>(descs, count, logP, st);
}

hipError_t launch_nl_mean_dg(const double* U, double* dg, int N, int M, double c3, double c1, hipStream_t st) {
    PINT_LAUNCH(k_nl_mean_dg, dim3((M + kGenNT - 1) / kGenNT), dim3(kGenNT), 0, st, U, dg, N, M, c3, c1);
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
    // dofs per workgroup: the N x W tile and the N weights within 64 KB of LDS
    const int W = gn_resid_width(a.N);
    const size_t lds = (size_t)a.N * (2 * W + 1) * sizeof(double);
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
