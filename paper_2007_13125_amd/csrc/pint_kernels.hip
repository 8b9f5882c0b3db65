// gfx950 kernels of one diagonalized waveform-relaxation sweep
// (Algorithm 1 for BDF-k, Algorithm 2 for CQ-BDF-k of Wu & Zhou, arXiv 2007.13125).
//
// A sweep is:  forward kernel   residual / right-hand side (FP64) -> kappa^{q/N}
//                               scaling -> R2C FFT along time, one dof tile per
//                               workgroup staged in LDS        (Alg. 1/2, Step 1)
//              spatial passes   (tau^{-alpha} d_p + A_h) Q_p = H_p for the N/2+1
//                               retained frequencies: PCR/Thomas in 1D, sine
//                               transforms (DST-I) + pointwise divide in 2D/3D
//                                                              (Step 2)
//              inverse kernel   C2R FFT along time -> kappa^{-q/N}/N -> update
//                               of U (FP64) -> per-workgroup norm partials (Step 3)
//              norm reduction   fixed-order reduction of the partials.
// Spectra are [N/2+1][ldS] complex in FP64 or (mixed mode) FP32, dof fastest.
#include "pint_internal.h"

#include <cstdint>

namespace pint {
namespace {

template <typename R> struct CT;
template <> struct CT<double> { using T = double2; };
template <> struct CT<float> { using T = float2; };
template <typename R> using cx = typename CT<R>::T;

template <typename T> __device__ __forceinline__ T mk(decltype(T::x) re, decltype(T::x) im) {
    T r;
    r.x = re;
    r.y = im;
    return r;
}
template <typename T> __device__ __forceinline__ T cadd(T a, T b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ T csub(T a, T b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T> __device__ __forceinline__ T cmul(T a, T b) {
    return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename T> __device__ __forceinline__ T cmulc(T a, T b) {
    return mk<T>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename T> __device__ __forceinline__ T cdiv(T a, T b) {
    const auto inv = decltype(T::x)(1) / (b.x * b.x + b.y * b.y);
    return mk<T>((a.x * b.x + a.y * b.y) * inv, (a.y * b.x - a.x * b.y) * inv);
}
template <bool INV, typename T> __device__ __forceinline__ T twmul(T a, T w) {
    return INV ? cmulc(a, w) : cmul(a, w);
}

// Natural-order 4-point DFT in place; forward uses e^{-2 pi i rs/4}.
template <bool INV, typename T> __device__ __forceinline__ void dft4(T& v0, T& v1, T& v2, T& v3) {
    const T t0 = cadd(v0, v2), t1 = csub(v0, v2), t2 = cadd(v1, v3), t3 = csub(v1, v3);
    const T mit3 = mk<T>(t3.y, -t3.x);  // -i * t3
    v0 = cadd(t0, t2);
    v2 = csub(t0, t2);
    if (!INV) {
        v1 = cadd(t1, mit3);
        v3 = csub(t1, mit3);
    } else {
        v1 = csub(t1, mit3);
        v3 = cadd(t1, mit3);
    }
}

// Batched in-place complex FFT of length L = 2^LOGL on B sequences held in LDS.
// Element t of sequence b sits at s[t*B + b] when BFAST, else at s[b*BSTR + t].
// Stockham auto-sort formulation: radix-4 stages with span Ns = 1, 4, 16, ...,
// then one radix-2 stage when LOGL is odd; each radix-4 stage reads its
// butterfly inputs into registers, synchronises, and writes the outputs to
// their sorted positions, so no second buffer is needed.
// Forward: X_k = sum_t x_t e^{-2 pi i t k/L}; INV uses e^{+...} and no 1/L.
// tw[j] = e^{-2 pi i j/L}, j < L (global, read through the caches).
// Every thread of the block must call it; it ends with a barrier.
template <typename R, int LOGL, int B, int NT, bool INV, bool BFAST, int BSTR>
__device__ void lds_fft(cx<R>* s, const cx<R>* __restrict__ tw) {
    using T = cx<R>;
    constexpr int L = 1 << LOGL;
    constexpr int Q = L / 4;
    constexpr int TOT4 = Q * B;
    constexpr int PER4 = (TOT4 + NT - 1) / NT;
    const int tid = threadIdx.x;
    auto at = [](int t, int b) { return BFAST ? t * B + b : b * BSTR + t; };
    int Ns = 1;
#pragma unroll 1
    for (int st = 0; st < LOGL / 2; ++st) {
        T v[PER4][4];
#pragma unroll
        for (int i = 0; i < PER4; ++i) {
            const int idx = tid + i * NT;
            if ((TOT4 % NT) == 0 || idx < TOT4) {
                const int j = BFAST ? idx / B : idx % Q;
                const int b = BFAST ? idx % B : idx / Q;
#pragma unroll
                for (int r = 0; r < 4; ++r) v[i][r] = s[at(j + r * Q, b)];
                const int k = j & (Ns - 1);
                const int e = k * (Q / Ns);
                v[i][1] = twmul<INV>(v[i][1], tw[e]);
                v[i][2] = twmul<INV>(v[i][2], tw[2 * e]);
                v[i][3] = twmul<INV>(v[i][3], tw[3 * e]);
                dft4<INV>(v[i][0], v[i][1], v[i][2], v[i][3]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < PER4; ++i) {
            const int idx = tid + i * NT;
            if ((TOT4 % NT) == 0 || idx < TOT4) {
                const int j = BFAST ? idx / B : idx % Q;
                const int b = BFAST ? idx % B : idx / Q;
                const int k = j & (Ns - 1);
                const int base = ((j - k) << 2) + k;
#pragma unroll
                for (int r = 0; r < 4; ++r) s[at(base + r * Ns, b)] = v[i][r];
            }
        }
        __syncthreads();
        Ns <<= 2;
    }
    if constexpr ((LOGL & 1) != 0) {
        // Last stage, span L/2: butterfly j reads and writes positions j, j + L/2.
        constexpr int H = L / 2;
        constexpr int TOT2 = H * B;
        for (int idx = tid; idx < TOT2; idx += NT) {
            const int j = BFAST ? idx / B : idx % H;
            const int b = BFAST ? idx % B : idx / H;
            const T v0 = s[at(j, b)];
            const T v1 = twmul<INV>(s[at(j + H, b)], tw[j]);
            s[at(j, b)] = cadd(v0, v1);
            s[at(j + H, b)] = csub(v0, v1);
        }
        __syncthreads();
    }
}

// Workgroups are dispatched round-robin over the 8 XCDs of the chip.  Give
// each XCD a contiguous range of tiles so that neighbouring tiles (shared
// cache lines, stencil neighbours) are served by the same L2.
__device__ __forceinline__ int xcd_tile(int bid, int nblocks) {
    const int per = nblocks >> 3;
    return (bid & 7) * per + (bid >> 3);
}

__device__ __forceinline__ double nanmax(double a, double b) {
    if (a != a) return a;
    if (b != b) return b;
    return a > b ? a : b;
}

// Hermitian split of the packed-pair spectrum Z = FFT(a + i b):
// A_p = (Z_p + conj Z_{N-p})/2,  B_p = (Z_p - conj Z_{N-p})/(2i).
template <typename R, int N, int B, int NT>
__device__ __forceinline__ void store_half_spectrum(const cx<R>* sm, cx<R>* S, int ldS, int d0, int M) {
    constexpr int NP = N / 2 + 1;
    for (int idx = threadIdx.x; idx < NP * B; idx += NT) {
        const int b = idx % B, p = idx / B;
        const cx<R> zp = sm[p * B + b];
        const cx<R> zn = sm[((N - p) & (N - 1)) * B + b];
        const R h = R(0.5);
        const cx<R> A = mk<cx<R>>((zp.x + zn.x) * h, (zp.y - zn.y) * h);
        const cx<R> Bv = mk<cx<R>>((zp.y + zn.y) * h, (zn.x - zp.x) * h);
        const int e = d0 + 2 * b;
        cx<R>* row = S + (size_t)p * ldS;
        if (e < M) row[e] = A;
        if (e + 1 < M) row[e + 1] = Bv;
    }
}

// ---------------------------------------------------------------------------
// Forward kernel, BDF-k (alpha = 1).  One workgroup per tile of W consecutive
// dofs and all N time rows.  Thread (dl, ch) owns dof d0+dl and a contiguous
// chunk of rows, so the k+1-tap time stencil runs on a register window.
//   residual: r_n = f_n + corr_n + tau^{-1} s_n v - tau^{-1} sum_{j<n} w_j U^{n-j} - A_h U^n
//   direct:   F_n = f_n + corr_n + tau^{-1} s_n v + kappa tau^{-1} sum_{j=n..k} w_j U^{N+n-j}
// (eqs. BDF-k-matrix and BDF-k-F with the kappa sum over j = n..k).
template <typename R, int LOGN, int W, int NT>
__global__ __launch_bounds__(NT) void k_fwd_heat(FwdArgs a) {
    constexpr int N = 1 << LOGN;
    constexpr int B = W / 2;
    constexpr int NCH = NT / W;
    constexpr int RPC = N / NCH;
    static_assert(NCH >= 1 && RPC >= 1 && NCH * RPC == N, "tile shape");
    __shared__ cx<R> sm[N * B];
    R* smr = reinterpret_cast<R*>(sm);

    const int ntiles = (a.M + W - 1) / W;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= ntiles) return;
    const int d0 = tile * W;
    const int tid = threadIdx.x;
    const int dl = tid % W, ch = tid / W;
    const int d = d0 + dl;
    const bool valid = d < a.M;
    const int q0 = ch * RPC;
    const size_t M = a.M;

    int x = 0, y = 0, z = 0;
    if (valid) {
        x = d % a.mx;
        const int rr = d / a.mx;
        y = rr % a.my;
        z = rr / a.my;
    }
    const bool hxm = x > 0, hxp = x < a.mx - 1;
    const bool hym = y > 0, hyp = y < a.my - 1;
    const bool hzm = z > 0, hzp = z < a.mz - 1;
    const size_t sy = (size_t)a.mx, sz = (size_t)a.mx * a.my;
    const double diag = 2.0 * (a.ihx2 + a.ihy2 + a.ihz2);
    const double vv = valid ? a.v[d] : 0.0;
    const bool resid = a.form == 0;

    double win[7];
    win[0] = 0.0;
#pragma unroll
    for (int j = 1; j < 7; ++j) {
        const int l = q0 + 1 - j;
        win[j] = (resid && valid && l >= 1 && j <= a.k) ? a.U[(size_t)(l - 1) * M + d] : 0.0;
    }
    for (int q = q0; q < q0 + RPC; ++q) {
        const int n = q + 1;
        double r = 0.0;
        if (valid) {
            const size_t o = (size_t)q * M + d;
            double g = a.ta * a.s[q] * vv;
            if (a.f) g += a.f[o + M];
            if (n - 1 < a.ncorr) g += a.corr[(size_t)(n - 1) * M + d];
            if (resid) {
                const double u = a.U[o];
                win[0] = u;
                double ts = 0.0;
#pragma unroll
                for (int j = 0; j < 7; ++j) ts += a.wk[j] * win[j];
                double au = diag * u;
                if (hxm) au -= a.ihx2 * a.U[o - 1];
                if (hxp) au -= a.ihx2 * a.U[o + 1];
                if (hym) au -= a.ihy2 * a.U[o - sy];
                if (hyp) au -= a.ihy2 * a.U[o + sy];
                if (hzm) au -= a.ihz2 * a.U[o - sz];
                if (hzp) au -= a.ihz2 * a.U[o + sz];
                r = g - a.ta * ts - au;
            } else {
                r = g;
                if (n <= a.k) {
                    double acc = 0.0;
                    for (int j = n; j <= a.k; ++j) acc += a.wk[j] * a.U[(size_t)(a.N + n - j - 1) * M + d];
                    r += a.kappa * a.ta * acc;
                }
            }
            r *= a.scale[q];
        }
        smr[q * W + dl] = (R)r;
#pragma unroll
        for (int j = 6; j > 0; --j) win[j] = win[j - 1];
    }
    __syncthreads();
    lds_fft<R, LOGN, B, NT, false, true, 0>(sm, reinterpret_cast<const cx<R>*>(a.tw));
    store_half_spectrum<R, N, B, NT>(sm, reinterpret_cast<cx<R>*>(a.S), a.ldS, d0, a.M);
}

// ---------------------------------------------------------------------------
// Forward kernel, CQ-BDF-k (alpha < 1).  The history sum over all earlier
// levels is a causal convolution in time; it is evaluated per dof pair as a
// length-2N circular convolution (the circulant embedding of the Toeplitz
// history matrix, Sec. 3.2 cost paragraph) with FP64 FFTs in LDS:
//   c = IFFT_2N( FFT_2N(omega, 0) . FFT_2N(u, 0) ),  u_i = U^{i+1}.
// residual: r_n = G_n - tau^{-alpha} c_{n-1} - A_h U^n;
// direct:   F_n = G_n + kappa tau^{-alpha} c_{N+n-1} (= sum_{j=n..N-1} w_j U^{N+n-j}).
template <typename R, int LOGN, int W, int NT>
__global__ __launch_bounds__(NT) void k_fwd_cq(FwdArgs a) {
    constexpr int N = 1 << LOGN;
    constexpr int N2 = 2 * N;
    constexpr int B = W / 2;
    __shared__ double2 cb[N2 * B];
    double* cbr = reinterpret_cast<double*>(cb);

    const int ntiles = (a.M + W - 1) / W;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= ntiles) return;
    const int d0 = tile * W;
    const int tid = threadIdx.x;
    const size_t M = a.M;

    for (int idx = tid; idx < N * W; idx += NT) {
        const int q = idx / W, dl = idx % W, d = d0 + dl;
        cbr[idx] = d < a.M ? a.U[(size_t)q * M + d] : 0.0;
    }
    for (int idx = N * W + tid; idx < N2 * W; idx += NT) cbr[idx] = 0.0;
    __syncthreads();
    lds_fft<double, LOGN + 1, B, NT, false, true, 0>(cb, a.tw2);
    for (int idx = tid; idx < N2 * B; idx += NT) cb[idx] = cmul(cb[idx], a.what[idx / B]);
    __syncthreads();
    lds_fft<double, LOGN + 1, B, NT, true, true, 0>(cb, a.tw2);

    // The residual form reads convolution rows [0, N), the direct form rows
    // [N, 2N); the time-FFT buffer (N x B values of cx<R>) goes into the other
    // half, so it never overwrites a value still to be read.
    const bool resid = a.form == 0;
    cx<R>* sm = reinterpret_cast<cx<R>*>(cb + (resid ? N * B : 0));
    R* smr = reinterpret_cast<R*>(sm);
    for (int idx = tid; idx < N * W; idx += NT) {
        const int q = idx / W, dl = idx % W, d = d0 + dl;
        const int n = q + 1;
        double r = 0.0;
        if (d < a.M) {
            const size_t o = (size_t)q * M + d;
            double g = a.ta * a.s[q] * a.v[d];
            if (a.f) g += a.f[o + M];
            if (n - 1 < a.ncorr) g += a.corr[(size_t)(n - 1) * M + d];
            if (resid) {
                const int x = d % a.mx, rr = d / a.mx, y = rr % a.my, z = rr / a.my;
                const double u = a.U[o];
                double au = 2.0 * (a.ihx2 + a.ihy2 + a.ihz2) * u;
                if (x > 0) au -= a.ihx2 * a.U[o - 1];
                if (x < a.mx - 1) au -= a.ihx2 * a.U[o + 1];
                if (y > 0) au -= a.ihy2 * a.U[o - a.mx];
                if (y < a.my - 1) au -= a.ihy2 * a.U[o + a.mx];
                if (z > 0) au -= a.ihz2 * a.U[o - (size_t)a.mx * a.my];
                if (z < a.mz - 1) au -= a.ihz2 * a.U[o + (size_t)a.mx * a.my];
                r = g - a.ta * cbr[q * W + dl] - au;
            } else {
                r = g + a.kappa * a.ta * cbr[(N + q) * W + dl];
            }
            r *= a.scale[q];
        }
        smr[idx] = (R)r;
    }
    __syncthreads();
    lds_fft<R, LOGN, B, NT, false, true, 0>(sm, reinterpret_cast<const cx<R>*>(a.tw));
    store_half_spectrum<R, N, B, NT>(sm, reinterpret_cast<cx<R>*>(a.S), a.ldS, d0, a.M);
}

// ---------------------------------------------------------------------------
// Inverse kernel: rebuild the packed-pair spectrum Z_p = A_p + i B_p for all
// p from the retained half (conjugate symmetry), inverse FFT in LDS, scale row
// q by kappa^{-q/N}/N (FP64), update U and accumulate the update norms.
template <typename R, int LOGN, int W, int NT>
__global__ __launch_bounds__(NT) void k_inv(InvArgs a) {
    constexpr int N = 1 << LOGN;
    constexpr int B = W / 2;
    constexpr int NP = N / 2 + 1;
    constexpr int NCH = NT / W;
    constexpr int RPC = N / NCH;
    static_assert(NCH * RPC == N, "tile shape");
    __shared__ cx<R> sm[N * B];
    __shared__ double red[2][NT / 64];
    R* smr = reinterpret_cast<R*>(sm);
    const int tid = threadIdx.x;

    const int ntiles = (a.M + W - 1) / W;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= ntiles) {
        if (tid == 0) {
            a.partial[2 * blockIdx.x] = 0.0;
            a.partial[2 * blockIdx.x + 1] = 0.0;
        }
        return;
    }
    const int d0 = tile * W;
    const cx<R>* S = reinterpret_cast<const cx<R>*>(a.S);
    for (int idx = tid; idx < NP * B; idx += NT) {
        const int b = idx % B, p = idx / B;
        const int e = d0 + 2 * b;
        const cx<R>* row = S + (size_t)p * a.ldS;
        cx<R> A = mk<cx<R>>(0, 0), Bv = mk<cx<R>>(0, 0);
        if (e < a.M) A = row[e];
        if (e + 1 < a.M) Bv = row[e + 1];
        if (p == 0 || p == N / 2) {
            A.y = 0;
            Bv.y = 0;
        }
        sm[p * B + b] = mk<cx<R>>(A.x - Bv.y, A.y + Bv.x);
        if (p > 0 && p < N / 2) sm[(N - p) * B + b] = mk<cx<R>>(A.x + Bv.y, Bv.x - A.y);
    }
    __syncthreads();
    lds_fft<R, LOGN, B, NT, true, true, 0>(sm, reinterpret_cast<const cx<R>*>(a.tw));

    const int dl = tid % W, ch = tid / W;
    const int d = d0 + dl;
    const bool valid = d < a.M;
    const size_t M = a.M;
    double mx = 0.0, s2 = 0.0;
    bool bad = false;
    if (valid) {
        for (int q = ch * RPC; q < (ch + 1) * RPC; ++q) {
            const double delta = (double)smr[q * W + dl] * a.unscale[q];
            const size_t o = (size_t)q * M + d;
            const double old = a.U[o];
            const double un = a.form == 0 ? old + delta : delta;
            const double upd = un - old;
            a.U[o] = un;
            const double au = fabs(upd);
            bad |= !(au <= 1.0e300);
            mx = au > mx ? au : mx;
            if (q == N - 1) s2 += upd * upd;
        }
    }
    if (bad) mx = __builtin_nan("");
    // wave64 butterfly reduction, then across waves in a fixed order
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
    if (tid == 0) {
        double m0 = red[0][0], t0 = red[1][0];
        for (int i = 1; i < NT / 64; ++i) {
            m0 = nanmax(m0, red[0][i]);
            t0 += red[1][i];
        }
        a.partial[2 * blockIdx.x] = m0;
        a.partial[2 * blockIdx.x + 1] = t0;
    }
}

__global__ __launch_bounds__(256) void k_norm_reduce(const double* __restrict__ partial, int nb, double hd,
                                                     double* __restrict__ out) {
    __shared__ double red[2][4];
    const int tid = threadIdx.x;
    double mx = 0.0, s2 = 0.0;
    for (int i = tid; i < nb; i += 256) {
        mx = nanmax(mx, partial[2 * i]);
        s2 += partial[2 * i + 1];
    }
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
    if (tid == 0) {
        double m0 = red[0][0], t0 = red[1][0];
        for (int i = 1; i < 4; ++i) {
            m0 = nanmax(m0, red[0][i]);
            t0 += red[1][i];
        }
        out[0] = m0;
        out[1] = sqrt(hd * t0);
    }
}

// ---------------------------------------------------------------------------
// 1D shifted solve (sigma_p + A_h) Q_p = H_p, one workgroup per frequency.
// A_h = h^{-2} tridiag(-1, 2, -1).  Parallel cyclic reduction with spans
// 1, 2, ..., NT/2 decouples the system into NT interleaved subsystems
// (equation i then couples only to i +- NT); thread t owns equations
// t, t+NT, ... and finishes its subsystem with the Thomas algorithm.
template <typename R, int EPT, int NT>
__global__ __launch_bounds__(NT) void k_tri1d(SpaceArgs a) {
    using T = cx<R>;
    extern __shared__ unsigned char smraw[];
    const int m = a.mx;
    T* la = reinterpret_cast<T*>(smraw);
    T* lb = la + m;
    T* lc = lb + m;
    T* ld = lc + m;
    const int p = blockIdx.x;
    const int tid = threadIdx.x;
    T* X = reinterpret_cast<T*>(a.S) + (size_t)p * a.ldS;
    const double2 sg = a.sigma[p];
    const T diag = mk<T>((R)(sg.x + 2.0 * a.ih2[0]), (R)sg.y);
    const T off = mk<T>((R)(-a.ih2[0]), (R)0);
    const T zero = mk<T>((R)0, (R)0);
    T ea[EPT], eb[EPT], ec[EPT], ed[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int i = tid + e * NT;
        if (i < m) {
            ea[e] = i > 0 ? off : zero;
            ec[e] = i < m - 1 ? off : zero;
            eb[e] = diag;
            ed[e] = X[i];
        } else {
            ea[e] = zero;
            ec[e] = zero;
            eb[e] = mk<T>((R)1, (R)0);
            ed[e] = zero;
        }
    }
    for (int delta = 1; delta < NT && delta < m; delta <<= 1) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int i = tid + e * NT;
            if (i < m) {
                la[i] = ea[e];
                lb[i] = eb[e];
                lc[i] = ec[e];
                ld[i] = ed[e];
            }
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int i = tid + e * NT;
            if (i < m) {
                T na = zero, nc = zero, nb = eb[e], nd = ed[e];
                if (i - delta >= 0) {
                    const T k1 = cdiv(ea[e], lb[i - delta]);
                    na = csub(zero, cmul(la[i - delta], k1));
                    nb = csub(nb, cmul(lc[i - delta], k1));
                    nd = csub(nd, cmul(ld[i - delta], k1));
                }
                if (i + delta < m) {
                    const T k2 = cdiv(ec[e], lb[i + delta]);
                    nc = csub(zero, cmul(lc[i + delta], k2));
                    nb = csub(nb, cmul(la[i + delta], k2));
                    nd = csub(nd, cmul(ld[i + delta], k2));
                }
                ea[e] = na;
                eb[e] = nb;
                ec[e] = nc;
                ed[e] = nd;
            }
        }
        __syncthreads();
    }
    // Thomas on the thread's own subsystem (coupling i <-> i + NT).
    T cp[EPT], dp[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int i = tid + e * NT;
        if (i < m) {
            T den = eb[e];
            T rhs = ed[e];
            if (e > 0) {
                den = csub(den, cmul(ea[e], cp[e - 1]));
                rhs = csub(rhs, cmul(ea[e], dp[e - 1]));
            }
            cp[e] = cdiv(ec[e], den);
            dp[e] = cdiv(rhs, den);
        }
    }
    T xn = zero;
#pragma unroll
    for (int e = EPT - 1; e >= 0; --e) {
        const int i = tid + e * NT;
        if (i < m) {
            xn = csub(dp[e], cmul(cp[e], xn));
            X[i] = xn;
        }
    }
}

// Raw sine transform along x (contiguous rows): Y_k = FFT_L(odd extension of
// x)_k = -2i sum_t x_t sin(pi t k/(m+1)), k = 1..m, L = 2(m+1).  ROWS rows per
// workgroup, layout [ROWS][L] in LDS.  Applying it twice multiplies by
// -2(m+1), which the divide pass folds in.
// With SOLVE (1D problems), the transformed row of frequency p is divided by
// (sigma_p + mu_x) times the raw-transform factor and transformed back.
template <typename R, int LOGL, int ROWS, int NT, bool SOLVE>
__global__ __launch_bounds__(NT) void k_dst_rows(SpaceArgs a, long long nlines) {
    using T = cx<R>;
    constexpr int L = 1 << LOGL;
    __shared__ T sm[ROWS * L];
    const int m = a.mx;
    const int lpp = a.my * a.mz;
    const long long g0 = (long long)blockIdx.x * ROWS;
    T* S = reinterpret_cast<T*>(a.S);
    const T zero = mk<T>((R)0, (R)0);
    for (int idx = threadIdx.x; idx < ROWS * L; idx += NT) {
        const int b = idx / L, t = idx % L;
        const long long g = g0 + b;
        T val = zero;
        if (g < nlines) {
            const long long p = g / lpp, rr = g % lpp;
            const T* row = S + p * a.ldS + rr * m;
            if (t >= 1 && t <= m) {
                val = row[t - 1];
            } else if (t >= m + 2) {
                const T w = row[L - t - 1];
                val = mk<T>(-w.x, -w.y);
            }
        }
        sm[b * L + t] = val;
    }
    __syncthreads();
    lds_fft<R, LOGL, ROWS, NT, false, false, L>(sm, reinterpret_cast<const T*>(a.twL[0]));
    if constexpr (SOLVE) {
        for (int idx = threadIdx.x; idx < ROWS * (m + 2); idx += NT) {
            const int b = idx / (m + 2), t = idx % (m + 2);
            const long long g = g0 + b;
            if (t == 0 || t == m + 1 || g >= nlines) {
                sm[b * L + t] = zero;
                if (t > 0 && t <= m) sm[b * L + L - t] = zero;
                continue;
            }
            const double2 sg = a.sigma[g / lpp];
            const double dre = sg.x + a.mu[0][t - 1];
            const double inv = a.inv_factor / (dre * dre + sg.y * sg.y);
            const T c = mk<T>((R)(dre * inv), (R)(-sg.y * inv));
            const T z = cmul(sm[b * L + t], c);
            sm[b * L + t] = z;
            sm[b * L + L - t] = mk<T>(-z.x, -z.y);
        }
        __syncthreads();
        lds_fft<R, LOGL, ROWS, NT, false, false, L>(sm, reinterpret_cast<const T*>(a.twL[0]));
    }
    for (int idx = threadIdx.x; idx < ROWS * m; idx += NT) {
        const int b = idx / m, t = idx % m + 1;
        const long long g = g0 + b;
        if (g < nlines) {
            const long long p = g / lpp, rr = g % lpp;
            S[p * a.ldS + rr * m + t - 1] = sm[b * L + t];
        }
    }
}

// Raw sine transform along y (axis 1) or z (axis 2) for W adjacent x columns,
// layout [L][W] in LDS.  With SOLVE, the transformed values are divided by
// (sigma_p + mu_x + mu_y (+ mu_z)) times the accumulated raw-transform factor
// and transformed back in the same workgroup (DST, divide, inverse DST).
template <typename R, int LOGL, int W, int NT, bool SOLVE>
__global__ __launch_bounds__(NT) void k_dst_cols(SpaceArgs a, int axis) {
    using T = cx<R>;
    constexpr int L = 1 << LOGL;
    __shared__ T sm[L * W];
    const int m = axis == 1 ? a.my : a.mz;
    const long long st = axis == 1 ? (long long)a.mx : (long long)a.mx * a.my;
    const int other = axis == 1 ? a.mz : a.my;
    const int nxg = (a.mx + W - 1) / W;
    const int gid = blockIdx.x;
    const int xg = gid % nxg;
    const int rest = gid / nxg;
    const int o = rest % other;
    const int p = rest / other;
    const int x0 = xg * W;
    const long long base = (long long)p * a.ldS + x0 + (axis == 1 ? (long long)o * a.mx * a.my : (long long)o * a.mx);
    T* S = reinterpret_cast<T*>(a.S);
    const T zero = mk<T>((R)0, (R)0);
    for (int idx = threadIdx.x; idx < L * W; idx += NT) {
        const int t = idx / W, w = idx % W;
        T val = zero;
        if (x0 + w < a.mx) {
            if (t >= 1 && t <= m) {
                val = S[base + (t - 1) * st + w];
            } else if (t >= m + 2) {
                const T u = S[base + (L - t - 1) * st + w];
                val = mk<T>(-u.x, -u.y);
            }
        }
        sm[t * W + w] = val;
    }
    __syncthreads();
    const T* tw = reinterpret_cast<const T*>(a.twL[axis]);
    lds_fft<R, LOGL, W, NT, false, true, 0>(sm, tw);
    if constexpr (SOLVE) {
        const double2 sg = a.sigma[p];
        for (int idx = threadIdx.x; idx < (m + 2) * W; idx += NT) {
            const int t = idx / W, w = idx % W;
            if (t == 0 || t == m + 1) {
                sm[t * W + w] = zero;
            } else if (x0 + w >= a.mx) {
                sm[t * W + w] = zero;
                sm[(L - t) * W + w] = zero;
            } else {
                double dre = sg.x + a.mu[0][x0 + w] + a.mu[axis][t - 1];
                if (axis == 2) dre += a.mu[1][o];
                const double dim_ = sg.y;
                const double inv = a.inv_factor / (dre * dre + dim_ * dim_);
                const T c = mk<T>((R)(dre * inv), (R)(-dim_ * inv));
                const T z = cmul(sm[t * W + w], c);
                sm[t * W + w] = z;
                sm[(L - t) * W + w] = mk<T>(-z.x, -z.y);
            }
        }
        __syncthreads();
        lds_fft<R, LOGL, W, NT, false, true, 0>(sm, tw);
    }
    for (int idx = threadIdx.x; idx < m * W; idx += NT) {
        const int t = idx / W + 1, w = idx % W;
        if (x0 + w < a.mx) S[base + (t - 1) * st + w] = sm[t * W + w];
    }
}

// Starting-step corrections of Table 1 for rows n = 1..k-1:
//   corr_n = a_n (f(0) - A_h v) + sum_{l=1..k-2} (b_{l,n} tau^l) d^l f/dt^l (0).
__global__ void k_prep(const double* __restrict__ v, const double* __restrict__ f, const double* __restrict__ fder,
                       double* __restrict__ corr, const double* __restrict__ a_n, const double* __restrict__ b_lt,
                       int k, int M, int mx, int my, int mz, double ihx2, double ihy2, double ihz2) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= M) return;
    const int x = d % mx, rr = d / mx, y = rr % my, z = rr / my;
    double av = 2.0 * (ihx2 + ihy2 + ihz2) * v[d];
    if (x > 0) av -= ihx2 * v[d - 1];
    if (x < mx - 1) av -= ihx2 * v[d + 1];
    if (y > 0) av -= ihy2 * v[d - mx];
    if (y < my - 1) av -= ihy2 * v[d + mx];
    if (z > 0) av -= ihz2 * v[d - mx * my];
    if (z < mz - 1) av -= ihz2 * v[d + mx * my];
    const double f0 = f ? f[d] : 0.0;
    for (int n = 1; n <= k - 1; ++n) {
        double c = a_n[n - 1] * (f0 - av);
        if (fder)
            for (int l = 1; l <= k - 2; ++l) c += b_lt[(l - 1) * 6 + (n - 1)] * fder[(size_t)(l - 1) * M + d];
        corr[(size_t)(n - 1) * M + d] = c;
    }
}

__global__ void k_fill(double* __restrict__ U, const double* __restrict__ v, long long total, int M, int zero) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    U[i] = zero ? 0.0 : v[i % M];
}

// ---------------------------------------------------------------------------
// Tile widths: the LDS tile of the time FFT holds N x W values of type R.
template <typename R> constexpr int time_tile(int logn) {
    const int w = 65536 / ((1 << logn) * (int)sizeof(R));
    return w > 64 ? 64 : (w < 2 ? 2 : w);
}
constexpr int cq_tile(int logn) {
    const int w = 8192 >> logn;
    return w > 64 ? 64 : (w < 2 ? 2 : w);
}
template <typename R> constexpr int rows_per_block(int logl) {
    const int r = 65536 / ((1 << logl) * (int)sizeof(cx<R>));
    return r > 16 ? 16 : (r < 1 ? 1 : r);
}
template <typename R> constexpr int cols_per_block(int logl) {
    // at least 8 columns (a 128-byte row segment in FP64) when 128 KB of LDS allows it
    const int w64 = 65536 / ((1 << logl) * (int)sizeof(cx<R>));
    const int w128 = 131072 / ((1 << logl) * (int)sizeof(cx<R>));
    const int w = w64 >= 8 ? w64 : (w128 >= 8 ? 8 : (w128 < 1 ? 1 : w128));
    return w > 32 ? 32 : w;
}

constexpr int kNT = 256;
constexpr int kNTcq = 512;  // the length-2N FP64 convolution FFT needs more lanes per tile

template <typename R, int LOGN>
hipError_t fwd_one(const FwdArgs& a, bool cq, int* nb, hipStream_t st) {
    if (cq) {
        constexpr int W = cq_tile(LOGN);
        const int ntiles = (a.M + W - 1) / W;
        const int grid = ((ntiles + 7) / 8) * 8;
        if (nb) *nb = grid;
        hipLaunchKernelGGL((k_fwd_cq<R, LOGN, W, kNTcq>), dim3(grid), dim3(kNTcq), 0, st, a);
    } else {
        constexpr int W = time_tile<R>(LOGN);
        const int ntiles = (a.M + W - 1) / W;
        const int grid = ((ntiles + 7) / 8) * 8;
        if (nb) *nb = grid;
        hipLaunchKernelGGL((k_fwd_heat<R, LOGN, W, kNT>), dim3(grid), dim3(kNT), 0, st, a);
    }
    return hipGetLastError();
}

template <typename R, int LOGN>
hipError_t inv_one(const InvArgs& a, int* nb, hipStream_t st) {
    constexpr int W = time_tile<R>(LOGN);
    const int ntiles = (a.M + W - 1) / W;
    const int grid = ((ntiles + 7) / 8) * 8;
    if (nb) *nb = grid;
    hipLaunchKernelGGL((k_inv<R, LOGN, W, kNT>), dim3(grid), dim3(kNT), 0, st, a);
    return hipGetLastError();
}

template <typename R>
hipError_t fwd_dispatch(const FwdArgs& a, bool cq, int* nb, hipStream_t st) {
    switch (__builtin_ctz((unsigned)a.N)) {
        case 3: return fwd_one<R, 3>(a, cq, nb, st);
        case 4: return fwd_one<R, 4>(a, cq, nb, st);
        case 5: return fwd_one<R, 5>(a, cq, nb, st);
        case 6: return fwd_one<R, 6>(a, cq, nb, st);
        case 7: return fwd_one<R, 7>(a, cq, nb, st);
        case 8: return fwd_one<R, 8>(a, cq, nb, st);
        case 9: return fwd_one<R, 9>(a, cq, nb, st);
        case 10: return fwd_one<R, 10>(a, cq, nb, st);
        case 11: return fwd_one<R, 11>(a, cq, nb, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename R>
hipError_t inv_dispatch(const InvArgs& a, int* nb, hipStream_t st) {
    switch (__builtin_ctz((unsigned)a.N)) {
        case 3: return inv_one<R, 3>(a, nb, st);
        case 4: return inv_one<R, 4>(a, nb, st);
        case 5: return inv_one<R, 5>(a, nb, st);
        case 6: return inv_one<R, 6>(a, nb, st);
        case 7: return inv_one<R, 7>(a, nb, st);
        case 8: return inv_one<R, 8>(a, nb, st);
        case 9: return inv_one<R, 9>(a, nb, st);
        case 10: return inv_one<R, 10>(a, nb, st);
        case 11: return inv_one<R, 11>(a, nb, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename R, int EPT, int NT>
hipError_t tri1d_one(const SpaceArgs& a, hipStream_t st) {
    const size_t lds = 4 * (size_t)a.mx * sizeof(cx<R>);
    static bool attr_set = false;
    if (!attr_set && lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tri1d<R, EPT, NT>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 163840);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL((k_tri1d<R, EPT, NT>), dim3(a.nP), dim3(NT), lds, st, a);
    return hipGetLastError();
}

template <typename R>
hipError_t tri1d_dispatch(const SpaceArgs& a, hipStream_t st) {
    const int m = a.mx;
    if (m <= 64) return tri1d_one<R, 1, 64>(a, st);
    if (m <= 128) return tri1d_one<R, 2, 64>(a, st);
    if (m <= 256) return tri1d_one<R, 4, 64>(a, st);
    if (m <= 512) return tri1d_one<R, 8, 64>(a, st);
    if (m <= 1024) return tri1d_one<R, 4, 256>(a, st);
    if (m <= 2048) return tri1d_one<R, 8, 256>(a, st);
    return hipErrorInvalidValue;
}

template <typename R, int LOGL, bool SOLVE>
hipError_t rows_one(const SpaceArgs& a, hipStream_t st) {
    constexpr int ROWS = rows_per_block<R>(LOGL);
    const long long nlines = (long long)a.nP * a.my * a.mz;
    const long long grid = (nlines + ROWS - 1) / ROWS;
    hipLaunchKernelGGL((k_dst_rows<R, LOGL, ROWS, kNT, SOLVE>), dim3((unsigned)grid), dim3(kNT), 0, st, a, nlines);
    return hipGetLastError();
}

template <typename R, int LOGL, bool SOLVE>
hipError_t cols_one(const SpaceArgs& a, int axis, hipStream_t st) {
    constexpr int W = cols_per_block<R>(LOGL);
    // tiles above 64 KB of LDS get 512 lanes so the FFT stages stay in registers
    constexpr int NT = ((1 << LOGL) * W * (int)sizeof(cx<R>) > 65536) ? 512 : kNT;
    const int other = axis == 1 ? a.mz : a.my;
    const long long grid = (long long)a.nP * other * ((a.mx + W - 1) / W);
    hipLaunchKernelGGL((k_dst_cols<R, LOGL, W, NT, SOLVE>), dim3((unsigned)grid), dim3(NT), 0, st, a, axis);
    return hipGetLastError();
}

template <typename R, bool SOLVE = false>
hipError_t rows_dispatch(const SpaceArgs& a, hipStream_t st) {
    switch (__builtin_ctz((unsigned)(2 * (a.mx + 1)))) {
        case 2: return rows_one<R, 2, SOLVE>(a, st);
        case 3: return rows_one<R, 3, SOLVE>(a, st);
        case 4: return rows_one<R, 4, SOLVE>(a, st);
        case 5: return rows_one<R, 5, SOLVE>(a, st);
        case 6: return rows_one<R, 6, SOLVE>(a, st);
        case 7: return rows_one<R, 7, SOLVE>(a, st);
        case 8: return rows_one<R, 8, SOLVE>(a, st);
        case 9: return rows_one<R, 9, SOLVE>(a, st);
        case 10: return rows_one<R, 10, SOLVE>(a, st);
        case 11: return rows_one<R, 11, SOLVE>(a, st);
        case 12: return rows_one<R, 12, SOLVE>(a, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename R, bool SOLVE>
hipError_t cols_dispatch(const SpaceArgs& a, int axis, hipStream_t st) {
    const int m = axis == 1 ? a.my : a.mz;
    switch (__builtin_ctz((unsigned)(2 * (m + 1)))) {
        case 3: return cols_one<R, 3, SOLVE>(a, axis, st);
        case 4: return cols_one<R, 4, SOLVE>(a, axis, st);
        case 5: return cols_one<R, 5, SOLVE>(a, axis, st);
        case 6: return cols_one<R, 6, SOLVE>(a, axis, st);
        case 7: return cols_one<R, 7, SOLVE>(a, axis, st);
        case 8: return cols_one<R, 8, SOLVE>(a, axis, st);
        case 9: return cols_one<R, 9, SOLVE>(a, axis, st);
        case 10: return cols_one<R, 10, SOLVE>(a, axis, st);
        case 11: return cols_one<R, 11, SOLVE>(a, axis, st);
        case 12: return cols_one<R, 12, SOLVE>(a, axis, st);
        default: return hipErrorInvalidValue;
    }
}

// The spatial solve is a short sequence of passes over the spectrum:
//   1D: one pass (sine transform + divide + inverse, or PCR/Thomas);
//   2D: DST-x rows, DST-y + divide + inverse DST-y, DST-x rows;
//   3D: DST-x, DST-y, DST-z + divide + inverse, DST-y, DST-x.
int pass_count(const SpaceArgs& a) { return a.dim == 1 ? 1 : (a.dim == 2 ? 3 : 5); }

bool dst1d(const SpaceArgs& a) {
    const unsigned L = 2u * (unsigned)(a.mx + 1);
    return (L & (L - 1)) == 0 && L <= (1u << kMaxLogL);
}

const char* pass_name(const SpaceArgs& a, int i) {
    if (a.dim == 1) return dst1d(a) ? "dst_x_solve" : "tridiag_pcr_thomas";
    if (a.dim == 2) return i == 1 ? "dst_y_solve" : "dst_x";
    static const char* n3[5] = {"dst_x", "dst_y", "dst_z_solve", "dst_y", "dst_x"};
    return n3[i];
}

template <typename R>
hipError_t space_pass(const SpaceArgs& a, int i, hipStream_t st) {
    if (a.dim == 1) return dst1d(a) ? rows_dispatch<R, true>(a, st) : tri1d_dispatch<R>(a, st);
    if (a.dim == 2) return i == 1 ? cols_dispatch<R, true>(a, 1, st) : rows_dispatch<R>(a, st);
    switch (i) {
        case 1: case 3: return cols_dispatch<R, false>(a, 1, st);
        case 2: return cols_dispatch<R, true>(a, 2, st);
        default: return rows_dispatch<R>(a, st);
    }
}

}  // namespace

hipError_t launch_prep(const double* v, const double* f, const double* fder, double* corr, const double* a_n,
                       const double* b_lt, int k, int M, int mx, int my, int mz, double ihx2, double ihy2,
                       double ihz2, hipStream_t st) {
    if (k < 2) return hipSuccess;
    hipLaunchKernelGGL(k_prep, dim3((M + 255) / 256), dim3(256), 0, st, v, f, fder, corr, a_n, b_lt, k, M, mx, my, mz,
                       ihx2, ihy2, ihz2);
    return hipGetLastError();
}

hipError_t launch_fill(double* U, const double* v, long long N, int M, int zero, hipStream_t st) {
    const long long total = N * M;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, U, v, total, M, zero);
    return hipGetLastError();
}

hipError_t launch_forward(const FwdArgs& a, bool mixed, bool cq, int* nb, hipStream_t st) {
    return mixed ? fwd_dispatch<float>(a, cq, nb, st) : fwd_dispatch<double>(a, cq, nb, st);
}

hipError_t launch_inverse(const InvArgs& a, bool mixed, int* nb, hipStream_t st) {
    return mixed ? inv_dispatch<float>(a, nb, st) : inv_dispatch<double>(a, nb, st);
}

int space_pass_count(const SpaceArgs& a) { return pass_count(a); }

const char* space_pass_name(const SpaceArgs& a, int pass) { return pass_name(a, pass); }

hipError_t launch_space_pass(const SpaceArgs& a, bool mixed, int pass, hipStream_t st) {
    return mixed ? space_pass<float>(a, pass, st) : space_pass<double>(a, pass, st);
}

hipError_t launch_space(const SpaceArgs& a, bool mixed, hipStream_t st) {
    for (int i = 0; i < pass_count(a); ++i) {
        const hipError_t e = launch_space_pass(a, mixed, i, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_norm_reduce(const double* partial, int nb, double hd, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_norm_reduce, dim3(1), dim3(256), 0, st, partial, nb, hd, out);
    return hipGetLastError();
}

}  // namespace pint
