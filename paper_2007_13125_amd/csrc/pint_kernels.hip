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

#include <algorithm>
#include <map>
#include <mutex>
#include <utility>
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

// Raw buffer access: a scalar descriptor (base, byte extent) plus a 32-bit
// byte offset per lane.  A load at or beyond the extent returns 0 and a store
// there is dropped by the hardware, so lanes without work are masked by the
// offset kNoLane instead of a branch: the number of memory instructions a
// wave issues stays fixed, and the compiler can count the stores in flight
// when it waits for earlier loads.
constexpr unsigned kNoLane = 0xFFFFFFF0u;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, unsigned long long bytes) {
    const unsigned nrec = bytes >= (unsigned long long)kNoLane ? kNoLane : (unsigned)bytes;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)nrec, 0x00020000);
}
__device__ __forceinline__ double2 buf_ld(__amdgpu_buffer_rsrc_t r, unsigned off, double2) {
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
}
__device__ __forceinline__ double buf_ld(__amdgpu_buffer_rsrc_t r, unsigned off, double) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
__device__ __forceinline__ float2 buf_ld(__amdgpu_buffer_rsrc_t r, unsigned off, float2) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, unsigned off, double2 v) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, (int)off, 0, 0);
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, unsigned off, float2 v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)off, 0, 0);
}

// e^{-2 pi i j/16}, j = 0..15 (real and imaginary parts), for the
// constant twiddles inside the in-register radix-8 and radix-16 DFTs.
__device__ __constant__ double kW16re[16] = {
    1.0, 0.92387953251128674, 0.70710678118654757, 0.38268343236508978,
    0.0, -0.38268343236508978, -0.70710678118654757, -0.92387953251128674,
    -1.0, -0.92387953251128674, -0.70710678118654757, -0.38268343236508978,
    0.0, 0.38268343236508978, 0.70710678118654757, 0.92387953251128674};
__device__ __constant__ double kW16im[16] = {
    0.0, -0.38268343236508978, -0.70710678118654757, -0.92387953251128674,
    -1.0, -0.92387953251128674, -0.70710678118654757, -0.38268343236508978,
    0.0, 0.38268343236508978, 0.70710678118654757, 0.92387953251128674,
    1.0, 0.92387953251128674, 0.70710678118654757, 0.38268343236508978};

// Natural-order R-point DFT of v[0..R) in registers (R = 2, 4, 8, 16), by
// recursive decimation in time; forward uses e^{-2 pi i rs/R}, INV e^{+...}.
template <int R, bool INV, typename T> struct SmallDft {
    __device__ __forceinline__ static void run(T* v) {
        constexpr int H = R / 2;
        T e[H], o[H];
#pragma unroll
        for (int i = 0; i < H; ++i) {
            e[i] = v[2 * i];
            o[i] = v[2 * i + 1];
        }
        SmallDft<H, INV, T>::run(e);
        SmallDft<H, INV, T>::run(o);
#pragma unroll
        for (int k = 0; k < H; ++k) {
            using E = decltype(T::x);
            T t = o[k];
            if (k != 0) {
                const int j = k * (16 / R);
                const E wr = (E)kW16re[j], wi = INV ? -(E)kW16im[j] : (E)kW16im[j];
                if (2 * k == H) {            // +-i
                    t = INV ? mk<T>(-t.y, t.x) : mk<T>(t.y, -t.x);
                } else {
                    t = mk<T>(t.x * wr - t.y * wi, t.x * wi + t.y * wr);
                }
            }
            v[k] = cadd(e[k], t);
            v[k + H] = csub(e[k], t);
        }
    }
};
template <bool INV, typename T> struct SmallDft<1, INV, T> {
    __device__ __forceinline__ static void run(T*) {}
};

// Radix schedule of a 2^LOGL transform: the fewest stages of radix <= 16,
// with the factors of two spread evenly over them (512 = 8 x 8 x 8,
// 1024 = 16 x 8 x 8, 32 = 8 x 4, ...).
// MAXLOG = 3 caps the radix at 8 (one more LDS pass for some lengths, but
// half the registers per butterfly).
constexpr int stage_count(int logl, int maxlog = 4) { return (logl + maxlog - 1) / maxlog; }
constexpr int stage_radix(int logl, int st, int maxlog = 4) {
    return 1 << (logl / stage_count(logl, maxlog) + (st < logl % stage_count(logl, maxlog) ? 1 : 0));
}

// One Stockham stage of radix RAD and span Ns: butterfly j (with k = j mod Ns)
// reads x[j + r L/RAD], multiplies by w^{r k L/(RAD Ns)}, takes the RAD-point
// DFT and writes position (j - k) RAD + k + r Ns.  Inputs of all butterflies
// are read into registers before a barrier, so the stage works in place.
// Twiddles w^r, r = 1..RAD-1, of one butterfly from the table entries for
// w^e, w^{2e}, w^{4e}, w^{8e} (log2 RAD loads instead of RAD - 1); every other
// power is a product of at most three of them.
// TWS > 1 reads every TWS-th entry of a finer table (w of a TWS times longer transform).
template <int RAD, bool INV, typename T, int TWS = 1>
__device__ __forceinline__ void apply_twiddles(T* v, const T* __restrict__ tw, int e) {
    T p[4];
#pragma unroll
    for (int i = 0; (1 << i) < RAD; ++i) p[i] = tw[(1 << i) * e * TWS];
#pragma unroll
    for (int r = 1; r < RAD; ++r) {
        T w = mk<T>(1, 0);
        bool first = true;
#pragma unroll
        for (int i = 0; (1 << i) < RAD; ++i)
            if (r & (1 << i)) {
                w = first ? p[i] : cmul(w, p[i]);
                first = false;
            }
        v[r] = twmul<INV>(v[r], w);
    }
}

// One Stockham stage of radix RAD and span Ns: butterfly j (with k = j mod Ns)
// reads x[j + r L/RAD], multiplies by w^{r k L/(RAD Ns)}, takes the RAD-point
// DFT and writes position (j - k) RAD + k + r Ns.  Inputs of all butterflies
// are read into registers before a barrier, so the stage works in place.
// Sequence layouts: BFAST s[t*B + b]; otherwise s[b*BSTR + t + (t >> PADSH)]
// (one padding slot per 2^PADSH elements keeps the strided writes of the first
// stage off a single LDS bank group; PADSH = 0 means no padding).
template <typename R, int LOGL, int RAD, int B, int NT, bool INV, bool BFAST, int BSTR, int PADSH, int TWS>
__device__ __forceinline__ void fft_stage(cx<R>* s, const cx<R>* __restrict__ tw, int Ns, int tid) {
    using T = cx<R>;
    constexpr int L = 1 << LOGL;
    constexpr int Q = L / RAD;
    constexpr int TOT = Q * B;
    constexpr int PER = (TOT + NT - 1) / NT;
    auto at = [](int t, int b) { return BFAST ? t * B + b : b * BSTR + t + (PADSH ? (t >> PADSH) : 0); };
    T v[PER][RAD];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int idx = tid + i * NT;
        if ((TOT % NT) == 0 || idx < TOT) {
            const int j = BFAST ? idx / B : idx % Q;
            const int b = BFAST ? idx % B : idx / Q;
#pragma unroll
            for (int r = 0; r < RAD; ++r) v[i][r] = s[at(j + r * Q, b)];
            const int k = j & (Ns - 1);
            if (Ns > 1) apply_twiddles<RAD, INV, T, TWS>(v[i], tw, k * (Q / Ns));
            SmallDft<RAD, INV, T>::run(v[i]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int idx = tid + i * NT;
        if ((TOT % NT) == 0 || idx < TOT) {
            const int j = BFAST ? idx / B : idx % Q;
            const int b = BFAST ? idx % B : idx / Q;
            const int k = j & (Ns - 1);
            const int base = (j - k) * RAD + k;
#pragma unroll
            for (int r = 0; r < RAD; ++r) s[at(base + r * Ns, b)] = v[i][r];
        }
    }
    __syncthreads();
}

template <typename R, int LOGL, int ST, int B, int NT, bool INV, bool BFAST, int BSTR, int PADSH, int TWS, int MAXLOG>
__device__ __forceinline__ void fft_stages(cx<R>* s, const cx<R>* __restrict__ tw, int Ns, int tid) {
    if constexpr (ST < stage_count(LOGL, MAXLOG)) {
        constexpr int RAD = stage_radix(LOGL, ST, MAXLOG);
        fft_stage<R, LOGL, RAD, B, NT, INV, BFAST, BSTR, PADSH, TWS>(s, tw, Ns, tid);
        fft_stages<R, LOGL, ST + 1, B, NT, INV, BFAST, BSTR, PADSH, TWS, MAXLOG>(s, tw, Ns * RAD, tid);
    }
}

// Batched in-place complex FFT of length L = 2^LOGL on B sequences held in LDS.
// Element t of sequence b sits at s[t*B + b] when BFAST, else at s[b*BSTR + t].
// Stockham auto-sort formulation with radix-16/8 stages (radix-4/2 for the
// remainder), in-register sub-DFTs, and one LDS round trip per stage.
// Forward: X_k = sum_t x_t e^{-2 pi i t k/L}; INV uses e^{+...} and no 1/L.
// tw[j] = e^{-2 pi i j/L}; the stages only index j < L/2 (in LDS or global memory).
// With TWS > 1, tw is the table of a TWS times longer transform (tw[TWS j] is used).
// Every thread of the block must call it; it ends with a barrier.
// Always inlined: as a call it would make the caller wait for all of its
// outstanding loads (prefetches) at the call and spill around it.  tid is the
// caller's lane index (threadIdx.x, or a copy of it that a persistent loop
// keeps from being treated as loop-invariant).
template <typename R, int LOGL, int B, int NT, bool INV, bool BFAST, int BSTR, int PADSH = 0, int TWS = 1,
          int MAXLOG = 4>
__device__ __forceinline__ void lds_fft(cx<R>* s, const cx<R>* __restrict__ tw, int tid) {
    fft_stages<R, LOGL, 0, B, NT, INV, BFAST, BSTR, PADSH, TWS, MAXLOG>(s, tw, 1, tid);
}
template <typename R, int LOGL, int B, int NT, bool INV, bool BFAST, int BSTR, int PADSH = 0, int TWS = 1,
          int MAXLOG = 4>
__device__ __forceinline__ void lds_fft(cx<R>* s, const cx<R>* __restrict__ tw) {
    fft_stages<R, LOGL, 0, B, NT, INV, BFAST, BSTR, PADSH, TWS, MAXLOG>(s, tw, 1, (int)threadIdx.x);
}

// threadIdx.x through an empty asm statement, called inside a persistent
// loop: the compiler cannot prove the result loop-invariant, so the LDS
// address arithmetic derived from it is recomputed per iteration instead of
// being hoisted out of the loop and held (or spilled) across all of it.
__device__ __forceinline__ int loop_tid() {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// Padding shift for sequences stored element-contiguously: one slot per
// first-stage radix group.
constexpr int pad_shift(int logl) {
    const int r = stage_radix(logl, 0);
    return r == 16 ? 4 : (r == 8 ? 3 : (r == 4 ? 2 : 1));
}

// Workgroups are dispatched round-robin over the 8 XCDs of the chip.  Give
// each XCD a contiguous range of tiles so that neighbouring tiles (shared
// cache lines, stencil neighbours) are served by the same L2.
__device__ __forceinline__ int xcd_tile(int bid, int nblocks) {
    const int per = nblocks >> 3;
    return (bid & 7) * per + (bid >> 3);
}

// Tile order for kernels with a y-stencil: inside each XCD's contiguous range
// of tiles, walk down columns (R tiles per grid row) so that the tiles holding
// a tile's y-neighbours are fetched by workgroups running at the same time on
// the same XCD, and the neighbour loads hit in its L2.
__device__ __forceinline__ int xcd_tile_columns(int bid, int nblocks, int R) {
    const int per = nblocks >> 3;
    const int s = bid >> 3, base = (bid & 7) * per;
    const int rows = R > 0 ? per / R : 0;
    if (rows > 1 && s < rows * R) return base + (s % rows) * R + s / rows;
    return base + s;
}

// dof index of padded spectrum slot P, or -1 for a padding slot
__device__ __forceinline__ int slot_dof(int P, int mx, int mxp, int Mp) {
    if (P >= Mp) return -1;
    const int x = P % mxp;
    return x < mx ? (P / mxp) * mx + x : -1;
}

__device__ __forceinline__ double nanmax(double a, double b) {
    if (a != a) return a;
    if (b != b) return b;
    return a > b ? a : b;
}

// Hermitian split of the packed-pair spectrum Z = FFT(a + i b):
// A_p = (Z_p + conj Z_{N-p})/2,  B_p = (Z_p - conj Z_{N-p})/(2i).
// Lane (p, e) produces dof d0 + e of row p, so consecutive lanes store
// consecutive complex values (one contiguous W-value segment per row).
// The loop has a compile-time trip count (all but the last pass unconditional),
// so the number of stores in flight is known to the compiler and later waits
// for earlier loads need not wait for these stores.  CHECK = false when the
// caller's tile never extends past the last slot.
template <typename R, int N, int B, int NT, bool CHECK = true>
__device__ __forceinline__ void store_half_spectrum(const cx<R>* sm, cx<R>* S, int ldS, int d0, int M,
                                                    int tid = -1) {
    constexpr int NP = N / 2 + 1;
    constexpr int W = 2 * B;
    constexpr int TOT = NP * W;
    constexpr int IT = (TOT + NT - 1) / NT;
    if (tid < 0) tid = threadIdx.x;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int idx = tid + it * NT;
        if ((it + 1) * NT <= TOT || idx < TOT) {
            const int e = idx % W, p = idx / W;
            const int b = e >> 1;
            const cx<R> zp = sm[p * B + b];
            const cx<R> zn = sm[((N - p) & (N - 1)) * B + b];
            const R h = R(0.5);
            const cx<R> out = (e & 1) ? mk<cx<R>>((zp.y + zn.y) * h, (zn.x - zp.x) * h)
                                      : mk<cx<R>>((zp.x + zn.x) * h, (zp.y - zn.y) * h);
            if (!CHECK || d0 + e < M) S[(size_t)p * ldS + d0 + e] = out;
        }
    }
}

// ---------------------------------------------------------------------------
// Forward kernel, BDF-k (alpha = 1).  One workgroup per tile of W consecutive
// dofs and all N time rows.
//   residual: r_n = f_n + corr_n + tau^{-1} s_n v - tau^{-1} sum_{j<n} w_j U^{n-j} - A_h U^n
//   direct:   F_n = f_n + corr_n + tau^{-1} s_n v + kappa tau^{-1} sum_{j=n..k} w_j U^{N+n-j}
// (eqs. BDF-k-matrix and BDF-k-F with the kappa sum over j = n..k).
// Phase A issues every global load of the tile at once: the U tile goes to LDS
// (FP64), while the source terms and the stencil neighbours outside the tile
// (y, z, and x at the tile edges) are folded into one register per element.
// Phase B adds the parts read from LDS (time stencil, centre, x neighbours
// inside the tile) and scales by kappa^{q/N}.  The FFT buffer then reuses the
// LDS of the U tile.
#ifndef PINT_FWD_WAVES
#define PINT_FWD_WAVES 4
#endif
#ifndef PINT_INV_WAVES
#define PINT_INV_WAVES 1
#endif
template <typename R, int LOGN, int W, int NT>
__global__ __launch_bounds__(NT, PINT_FWD_WAVES) void k_fwd_heat(FwdArgs a) {
    constexpr int N = 1 << LOGN;
    constexpr int B = W / 2;
    constexpr int PER = N * W / NT;
    static_assert(PER * NT == N * W, "tile shape");
    __shared__ double su[N * W];
    cx<R>* sm = reinterpret_cast<cx<R>*>(su);
    R* smr = reinterpret_cast<R*>(su);

    const int ntiles = (a.Mp + W - 1) / W;
    const int tile = (a.my > 1 && a.mxp >= W) ? xcd_tile_columns(blockIdx.x, gridDim.x, a.mxp / W)
                                              : xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= ntiles) return;
    const int d0 = tile * W;           // first spectrum slot of the tile
    const int tid = threadIdx.x;
    const int dl = tid % W;            // the slot of every element this thread owns
    const int d = slot_dof(d0 + dl, a.mx, a.mxp, a.Mp);
    const bool valid = d >= 0;
    const size_t M = a.M;
    const bool resid = a.form == 0;
    const bool useU = a.form != 2;     // form 2: the source part G alone (U not read)

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
    const bool exm = hxm && dl == 0, exp_ = hxp && dl == W - 1;   // x neighbours outside the tile
    const size_t sy = (size_t)a.mx, sz = (size_t)a.mx * a.my;
    const double vt = valid ? a.ta * a.v[d] : 0.0;

    // Neighbours outside the tile: branch-free loads (a missing neighbour reads
    // the centre with weight zero), so every load of the tile is in flight at once.
    const bool nbx = resid && valid;
    const double cxm = (nbx && exm) ? a.ihx2 : 0.0, cxp = (nbx && exp_) ? a.ihx2 : 0.0;
    const double cym = (nbx && hym) ? a.ihy2 : 0.0, cyp = (nbx && hyp) ? a.ihy2 : 0.0;
    const double czm = (nbx && hzm) ? a.ihz2 : 0.0, czp = (nbx && hzp) ? a.ihz2 : 0.0;
    const long long oxm = cxm != 0.0 ? -1 : 0, oxp = cxp != 0.0 ? 1 : 0;
    const long long oym = cym != 0.0 ? -(long long)sy : 0, oyp = cyp != 0.0 ? (long long)sy : 0;
    const long long ozm = czm != 0.0 ? -(long long)sz : 0, ozp = czp != 0.0 ? (long long)sz : 0;
    const bool has3 = a.mz > 1;
    const double* Ub = a.U + (valid ? d : 0);
    const double* fb = a.f ? a.f + (valid ? d : 0) + M : nullptr;
    double g[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int q = (tid + i * NT) / W;
        const double* uq = Ub + (size_t)q * M;
        const double u = useU ? uq[0] : 0.0;
        double acc = vt * a.s[q];
        if (fb) acc += fb[(size_t)q * M];
        if (resid) {
            acc += cxm * uq[oxm] + cxp * uq[oxp] + cym * uq[oym] + cyp * uq[oyp];
            if (has3) acc += czm * uq[ozm] + czp * uq[ozp];
        }
        su[q * W + dl] = valid ? u : 0.0;
        g[i] = valid ? acc : 0.0;
    }
    if (valid && a.ncorr > 0) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int q = (tid + i * NT) / W;
            if (q < a.ncorr) g[i] += a.corr[(size_t)q * M + d];
        }
    }
    __syncthreads();

    const double diag = 2.0 * (a.ihx2 + a.ihy2 + a.ihz2);
    const double cim = (hxm && dl > 0) ? a.ihx2 : 0.0, cip = (hxp && dl < W - 1) ? a.ihx2 : 0.0;
    const int lm = dl > 0 ? dl - 1 : dl, lp = dl < W - 1 ? dl + 1 : dl;   // x neighbours inside the tile
    double wk[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) wk[j] = a.wk[j];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int q = (tid + i * NT) / W;
        const int n = q + 1;
        double r = 0.0;
        if (valid) {
            r = g[i];
            if (resid) {
                const double u = su[q * W + dl];
                // time stencil sum_{j<n, j<=k} w_j U^{n-j}; w_j = 0 beyond k
                double ts = wk[0] * u;
#pragma unroll
                for (int j = 1; j < 7; ++j) ts += (q >= j) ? wk[j] * su[(q >= j ? q - j : 0) * W + dl] : 0.0;
                const double au = diag * u - cim * su[q * W + lm] - cip * su[q * W + lp];
                r -= a.ta * ts + au;
            } else if (a.form == 1 && n <= a.k) {
                double acc = 0.0;
                for (int j = n; j <= a.k; ++j) acc += wk[j] * su[(a.N + n - j - 1) * W + dl];
                r += a.kappa * a.ta * acc;
            }
            r *= a.scale[q];
        }
        g[i] = r;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) smr[tid + i * NT] = (R)g[i];
    __syncthreads();
    lds_fft<R, LOGN, B, NT, false, true, 0>(sm, reinterpret_cast<const cx<R>*>(a.tw));
    store_half_spectrum<R, N, B, NT>(sm, reinterpret_cast<cx<R>*>(a.S), a.ldS, d0, a.Mp);
}

// ---------------------------------------------------------------------------
// Forward kernel, BDF-k residual form on 2D and 3D grids, marching along the
// outermost axis (y in 2D, z in 3D).  A workgroup owns the W x slots of one
// line and walks a chunk of consecutive outer indices c.  Each lane keeps its
// time rows of U at c-1, c and c+1 in registers, so the outer-axis stencil
// neighbours are read from memory once (not three times), and every load of
// position c+1 (U at c+2, f, v, x halo, 3D y neighbours) is issued before the
// LDS phases, FFT and spectrum store of position c.  Per position the
// arithmetic is that of k_fwd_heat (same residual, same FFT, same store).
#ifndef PINT_MARCH_WAVES
#define PINT_MARCH_WAVES 1
#endif
#ifndef PINT_MARCH_NT
#define PINT_MARCH_NT 512
#endif
#ifndef PINT_FWD_WIDE
#define PINT_FWD_WIDE 1
#endif
template <typename R, int LOGN, int W, int NT, bool IS3>
__global__ __launch_bounds__(NT, PINT_MARCH_WAVES) void k_fwd_march(FwdArgs a, int ncol, int nchunk, int chunk) {
    using T = cx<R>;
    constexpr int N = 1 << LOGN;
    constexpr int B = W / 2;
    constexpr int PER = N * W / NT;
    static_assert(PER * NT == N * W, "tile shape");
    constexpr int CI = (6 * W + NT - 1) / NT < PER ? (6 * W + NT - 1) / NT : PER;   // i with q_i < 6 possible
    constexpr int Z = 6 * W;            // six zero rows below time row 0: U^{n-j} = 0 for n - j < 1
    __shared__ double sbuf[Z + N * W];
    __shared__ double ssn[N], ssc[N];   // tau^{-1} s_n and kappa^{q/N}
    __shared__ T stw[N / 2];            // FFT twiddles, read from LDS so that the FFT never
                                        // waits on the vector-memory counter of the prefetches
    double* su = sbuf + Z;              // su[q W + l] = U^{q+1} at slot l of the tile
    T* sm = reinterpret_cast<T*>(sbuf); // FFT buffer [N][B], reuses the LDS of the tile
    R* smr = reinterpret_cast<R*>(sbuf);

    const int lin = xcd_tile(blockIdx.x, gridDim.x);
    if (lin >= ncol * nchunk) return;
    const int col = lin % ncol, chk = lin / ncol;
    const int nxt = a.mxp / W;
    // x tile and y line (3D): consecutive workgroups take consecutive y lines of
    // one x tile, so the lines whose U a workgroup reads as y neighbours are
    // marched at the same time by workgroups on the same XCD (shared L2)
    const int xt = IS3 ? col / a.my : col % nxt, yl = IS3 ? col % a.my : col / nxt;
    const int nm = IS3 ? a.mz : a.my;                  // length of the marching axis
    const int c0 = chk * chunk, c1 = min(nm, c0 + chunk);
    const int tid = threadIdx.x;
    const int dl = tid % W;
    const int x = xt * W + dl;
    const bool valid = x < a.mx;
    const size_t M = a.M;
    const long long sdof = IS3 ? (long long)a.mx * a.my : a.mx;      // dof stride along the march
    const long long sslot = IS3 ? (long long)a.mxp * a.my : a.mxp;   // spectrum slot stride
    const long long dbase = (valid ? x : 0) + (IS3 ? (long long)a.mx * yl : 0);
    const long long slot0 = (long long)xt * W + (IS3 ? (long long)a.mxp * yl : 0);

    for (int i = tid; i < N; i += NT) {
        ssn[i] = a.ta * a.s[i];
        ssc[i] = a.scale[i];
        if (i < N / 2) stw[i] = reinterpret_cast<const T*>(a.tw)[i];
    }
    // Coefficients fixed along the march; a missing neighbour reads the centre with weight 0.
    const bool hxm = valid && x > 0 && dl == 0, hxp = valid && x < a.mx - 1 && dl == W - 1;
    const double chx = (hxm || hxp) ? a.ihx2 : 0.0;
    const long long ohx = hxm ? -1 : (hxp ? 1 : 0);
    const double cym = (IS3 && valid && yl > 0) ? a.ihy2 : 0.0;
    const double cyp = (IS3 && valid && yl < a.my - 1) ? a.ihy2 : 0.0;
    const long long oym = cym != 0.0 ? -(long long)a.mx : 0, oyp = cyp != 0.0 ? (long long)a.mx : 0;
    const double co = valid ? (IS3 ? a.ihz2 : a.ihy2) : 0.0;
    const double diag = 2.0 * (a.ihx2 + a.ihy2 + a.ihz2);
    const double cim = (valid && x > 0 && dl > 0) ? a.ihx2 : 0.0;
    const double cip = (valid && x < a.mx - 1 && dl < W - 1) ? a.ihx2 : 0.0;
    const int om = dl > 0 ? -1 : 0, op = dl < W - 1 ? 1 : 0;   // x neighbours inside the tile
    double wk[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) wk[j] = a.wk[j];

    // Addresses: a uniform (scalar) base per row group i and outer index c plus
    // one 32-bit byte offset per lane that is fixed for the whole kernel, so
    // the loads take the scalar-base + vector-offset form and need no 64-bit
    // address arithmetic per element (the host guarantees the offsets fit).
    // Every load is unconditional (rows clamped to the grid, absent terms read
    // a valid array with weight 0), so no loaded register is ever copied or
    // merged before use and the prefetches stay in flight across the FFT.
    constexpr int RS = NT / W;                         // time rows between row groups i and i+1
    const int qb = tid / W;
    const unsigned lo = (unsigned)(((long long)qb * (long long)M + dbase) * 8);
    const unsigned lhx = (unsigned)((long long)lo + ohx * 8);
    const unsigned lym = (unsigned)((long long)lo + oym * 8), lyp = (unsigned)((long long)lo + oyp * 8);
    const unsigned lv = (unsigned)(dbase * 8);
    const double cf = a.f ? 1.0 : 0.0;
    const double* fbase = a.f ? a.f + M : a.U;         // f(t_{q+1}), or U with weight 0
    const double* cbase = a.ncorr > 0 ? a.corr : a.U;  // correction rows, or U with weight 0
    double ccf[CI];
    unsigned lcr[CI];
#pragma unroll
    for (int i = 0; i < CI; ++i) {
        const int q = qb + i * RS;
        ccf[i] = q < a.ncorr ? 1.0 : 0.0;
        lcr[i] = (unsigned)(((long long)(q < a.ncorr ? q : 0) * (long long)M + dbase) * 8);
    }
    const size_t nU = (size_t)a.N * M;
    const size_t nF = a.f ? (size_t)a.N * M : nU;          // f rows 1..N (fbase skips row 0)
    const size_t nC = a.ncorr > 0 ? (size_t)a.ncorr * M : nU;
    // buffer load of arr[e0 + lane offset]: the descriptor spans arr[e0 .. n), so an
    // offset outside the array reads 0 instead of faulting
    auto at = [](const double* arr, size_t n, size_t e0, unsigned off) {
        const unsigned long long avail = (unsigned long long)(n - e0) * 8ull;
        const int nrec = avail > 0xffffffffull ? -1 : (int)(unsigned)avail;
        __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(arr + e0), (short)0, nrec,
                                                                     0x00020000);
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
    };
    double A[PER], Bv[PER], C[PER], fr[PER], hx[PER], ym[PER], yp[PER], cr[CI];
    double vv;
    auto load_row = [&](double (&dst)[PER], int c) {   // U at outer index c (within the grid)
#pragma unroll
        for (int i = 0; i < PER; ++i) dst[i] = at(a.U, nU, (size_t)i * RS * M + (size_t)c * sdof, lo);
    };
    auto load_side = [&](int c) {                      // everything else position c needs
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const size_t e0 = (size_t)i * RS * M + (size_t)c * sdof;
            hx[i] = at(a.U, nU, e0, lhx);
            if (IS3) {
                ym[i] = at(a.U, nU, e0, lym);
                yp[i] = at(a.U, nU, e0, lyp);
            }
            fr[i] = at(fbase, nF, e0, lo);
        }
#pragma unroll
        for (int i = 0; i < CI; ++i) cr[i] = at(cbase, nC, (size_t)c * sdof, lcr[i]);
        vv = at(a.v, M, (size_t)c * sdof, lv);
    };

    // One position c of the march with U at c-1, c, c+1 in Um, Uc, Up; Um is
    // refilled with U at c+2.  The three arrays rotate by renaming (the loop
    // below is unrolled three times), never by register copies.
    auto step = [&](int c, double (&Um)[PER], double (&Uc)[PER], double (&Up)[PER]) {
        const double cm = c > 0 ? co : 0.0, cp = c < nm - 1 ? co : 0.0;
        double g[PER];
        for (int e = tid; e < Z; e += NT) sbuf[e] = 0.0;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            double acc = vv * ssn[qb + i * RS] + cf * fr[i] + chx * hx[i] + cm * Um[i] + cp * Up[i];
            if (IS3) acc += cym * ym[i] + cyp * yp[i];
            if (i < CI) acc += ccf[i] * cr[i];
            su[tid + i * NT] = valid ? Uc[i] : 0.0;
            g[i] = acc;
        }
        // every loaded value of position c is consumed above before new loads are issued
        __builtin_amdgcn_sched_barrier(0);
        load_row(Um, min(c + 2, nm - 1));
        load_side(min(c + 1, nm - 1));
        __syncthreads();
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int q = qb + i * RS;
            const double* sp = su + tid + i * NT;
            const double u = sp[0];
            // time stencil sum_{j<=k} w_j U^{n-j} over the zero-padded tile (w_j = 0 beyond k)
            double ts = wk[0] * u;
#pragma unroll
            for (int j = 1; j < 7; ++j) ts += wk[j] * sp[-j * W];
            const double au = diag * u - cim * sp[om] - cip * sp[op];
            const double r = (g[i] - (a.ta * ts + au)) * ssc[q];
            g[i] = valid ? r : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < PER; ++i) smr[tid + i * NT] = (R)g[i];
        __syncthreads();
        lds_fft<R, LOGN, B, NT, false, true, 0>(sm, stw);
        store_half_spectrum<R, N, B, NT, false>(sm, reinterpret_cast<T*>(a.S), a.ldS, (int)(slot0 + c * sslot), a.Mp);
        __syncthreads();
    };

    load_row(A, max(c0 - 1, 0));
    load_row(Bv, c0);
    load_row(C, min(c0 + 1, nm - 1));
    load_side(c0);
    __syncthreads();   // ssn, ssc, stw
    for (int c = c0; c < c1; c += 3) {
        step(c, A, Bv, C);
        if (c + 1 < c1) step(c + 1, Bv, C, A);
        if (c + 2 < c1) step(c + 2, C, A, Bv);
    }
}

// ---------------------------------------------------------------------------
// Forward kernel, BDF-k residual form on 2D and 3D grids: wide-tile march.
// The same march as k_fwd_march, laid out for wider tiles (W = 16 FP64 slots,
// whole 128-byte row segments per load, for N = 512) within the register file:
//  - U at the previous outer index is read back from the LDS tile of the
//    previous position (each lane reads and rewrites only its own elements),
//    so only U at c and c+1 are held in registers;
//  - the partial sums of Phase A go to a separate LDS buffer, which Phase B
//    overwrites in place with the residual and the FFT then transforms, so no
//    per-element sum stays in registers across the barrier (FP64 spectra);
//  - the x neighbours outside the tile are loaded by the two edge lanes only
//    (every other lane's load is masked off) and written to halo columns of
//    the LDS tile, so Phase B applies one stencil to every slot.
//  - TAB = false (two workgroups per CU): the per-row factors are not staged
//    in LDS; tau^{-1} s_q (nonzero only for q < k, all in row group 0) is read
//    once per lane and kappa^{q/N} follows row group by row group from
//    kappa^{qb/N} times powers of kappa^{RS/N}.
template <typename R, int LOGN, int W, int NT, bool IS3, bool TAB = true>
__global__ __launch_bounds__(NT, TAB ? 1 : 2) void k_fwd_wide(FwdArgs a, int ncol, int nchunk, int chunk) {
    using T = cx<R>;
    constexpr int N = 1 << LOGN;
    constexpr int B = W / 2;
    constexpr int PER = N * W / NT;
    static_assert(PER * NT == N * W, "tile shape");
    constexpr int RS = NT / W;                       // time rows between row groups i and i+1
    static_assert(TAB || (PER >= 2 && RS >= 7), "row group 0 must hold every q < k");
    constexpr int WS = W + 2;                        // LDS row: halo, W slots, halo
    constexpr int Z = 6;                             // zero time rows below row 0
    constexpr int CI = (6 * W + NT - 1) / NT < PER ? (6 * W + NT - 1) / NT : PER;
    __shared__ double su[(Z + N) * WS];
    __shared__ double sg[N * W];
    __shared__ double ssn[TAB ? N : 1], ssc[TAB ? N : 1];   // tau^{-1} s_n and kappa^{q/N}
    __shared__ T stw[N / 2];
    double* u0 = su + Z * WS + 1;                    // u0[q WS + l]: slot l of time row q (l = -1, W: halo)
    T* sm = reinterpret_cast<T*>(sg);                // FFT buffer [N][B]
    R* smr = reinterpret_cast<R*>(sg);

    const int lin = xcd_tile(blockIdx.x, gridDim.x);
    if (lin >= ncol * nchunk) return;
    const int col = lin % ncol, chk = lin / ncol;
    const int nxt = a.mxp / W;
    const int xt = IS3 ? col / a.my : col % nxt, yl = IS3 ? col % a.my : col / nxt;   // 3D: y lines fastest
    const int nm = IS3 ? a.mz : a.my;
    const int c0 = chk * chunk, c1 = min(nm, c0 + chunk);
    const int tid = threadIdx.x;
    const int dl = tid % W, qb = tid / W;
    const int x0 = xt * W, x = x0 + dl;
    const bool valid = x < a.mx;
    const size_t M = a.M;
    const long long sdof = IS3 ? (long long)a.mx * a.my : a.mx;
    const long long sslot = IS3 ? (long long)a.mxp * a.my : a.mxp;
    const long long dbase = (valid ? x : 0) + (IS3 ? (long long)a.mx * yl : 0);
    const long long slot0 = (long long)x0 + (IS3 ? (long long)a.mxp * yl : 0);

    for (int i = tid; i < N; i += NT) {
        if constexpr (TAB) {
            ssn[i] = a.ta * a.s[i];
            ssc[i] = a.scale[i];
        }
        if (i < N / 2) stw[i] = reinterpret_cast<const T*>(a.tw)[i];
    }
    for (int j = tid; j < Z * WS; j += NT) su[j] = 0.0;
    const double sn0 = TAB ? 0.0 : a.ta * a.s[qb];   // tau^{-1} s_q of row group 0
    const double sc0 = TAB ? 0.0 : a.scale[qb];      // kappa^{qb/N}
    const double scs = TAB ? 0.0 : a.scale[RS];      // kappa^{RS/N}

    // halo loads: lane dl = 0 reads x0 - 1, lane dl = W-1 reads x0 + W; all others, and
    // neighbours outside the grid, are masked off (they read 0 without a memory access)
    const bool hl = dl == 0 && x0 > 0, hr = dl == W - 1 && x0 + W < a.mx;
    const long long ohx = hl ? -1 : (hr ? 1 : 0);
    const double cym = (IS3 && valid && yl > 0) ? a.ihy2 : 0.0;
    const double cyp = (IS3 && valid && yl < a.my - 1) ? a.ihy2 : 0.0;
    const long long oym = cym != 0.0 ? -(long long)a.mx : 0, oyp = cyp != 0.0 ? (long long)a.mx : 0;
    const double co = valid ? (IS3 ? a.ihz2 : a.ihy2) : 0.0;
    const double diag = 2.0 * (a.ihx2 + a.ihy2 + a.ihz2);
    const double cx = a.ihx2;
    double wk[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) wk[j] = a.wk[j];

    const unsigned lo = (unsigned)(((long long)qb * (long long)M + dbase) * 8);
    const unsigned lhx = (hl || hr) ? (unsigned)((long long)lo + ohx * 8) : kNoLane;
    const unsigned lym = (unsigned)((long long)lo + oym * 8), lyp = (unsigned)((long long)lo + oyp * 8);
    const unsigned lv = (unsigned)(dbase * 8);
    const double cf = a.f ? 1.0 : 0.0;
    const double* fbase = a.f ? a.f + M : a.U;
    const double* cbase = a.ncorr > 0 ? a.corr : a.U;
    const size_t nU = (size_t)a.N * M;
    const size_t nC = a.ncorr > 0 ? (size_t)a.ncorr * M : nU;
    double ccf[CI];
    unsigned lcr[CI];
#pragma unroll
    for (int i = 0; i < CI; ++i) {
        const int q = qb + i * RS;
        ccf[i] = q < a.ncorr ? 1.0 : 0.0;
        lcr[i] = (unsigned)(((long long)(q < a.ncorr ? q : 0) * (long long)M + dbase) * 8);
    }
    auto at = [](const double* arr, size_t n, size_t e0, unsigned off) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
                                              buf_rsrc(arr + e0, (unsigned long long)(n - e0) * 8ull), (int)off, 0, 0));
    };
    // 3D: with YAHEAD the y-neighbour lines of position c are loaded together
    // with U at c (two positions ahead, in the same step as the workgroups that
    // own those lines load them, so L2 serves them; two sets alternate with the
    // steps); otherwise one position ahead with the other side loads.
    // FP64 needs radix <= 8 time-FFT stages (half the registers per butterfly) to make
    // room for the second set; both precisions fit it only up to 8 rows per lane
    constexpr bool YAHEAD = IS3 && PER <= 8;
    constexpr int FMAXLOG = (YAHEAD && sizeof(R) == 8) ? 3 : 4;
    double A[PER], Bv[PER], fr[PER], hx[PER], ymA[PER], ypA[PER], ymB[YAHEAD ? PER : 1], ypB[YAHEAD ? PER : 1], cr[CI];
    double vv;
    auto load_row = [&](double (&dst)[PER], int c) {
#pragma unroll
        for (int i = 0; i < PER; ++i) dst[i] = at(a.U, nU, (size_t)i * RS * M + (size_t)c * sdof, lo);
    };
    auto load_side = [&](int c) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const size_t e0 = (size_t)i * RS * M + (size_t)c * sdof;
            hx[i] = at(a.U, nU, e0, lhx);
            if constexpr (IS3 && !YAHEAD) {
                ymA[i] = at(a.U, nU, e0, lym);
                ypA[i] = at(a.U, nU, e0, lyp);
            }
            fr[i] = at(fbase, nU, e0, lo);
        }
#pragma unroll
        for (int i = 0; i < CI; ++i) cr[i] = at(cbase, nC, (size_t)c * sdof, lcr[i]);
        vv = at(a.v, M, (size_t)c * sdof, lv);
    };
    auto load_ynb = [&](double (&ym)[PER], double (&yp)[PER], int c) {   // y neighbours at position c
        if constexpr (YAHEAD) {
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const size_t e0 = (size_t)i * RS * M + (size_t)c * sdof;
                ym[i] = at(a.U, nU, e0, lym);
                yp[i] = at(a.U, nU, e0, lyp);
            }
        }
    };
    // LDS index of element i of this lane: (q_i, dl) with q_i = qb + i RS
    const int sb = qb * WS + dl;
    constexpr int SSTEP = RS * WS;

    // One position c with U at c and c+1 in Uc, Up (Uc is refilled with U at c+2)
    // and, in 3D, the y neighbours at c in Ym, Yp (refilled with those at c+2).
    auto step = [&](int c, double (&Uc)[PER], double (&Up)[PER], double (&Ym)[PER], double (&Yp)[PER]) {
        const double cm = c > 0 ? co : 0.0, cp = c < nm - 1 ? co : 0.0;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int q = qb + i * RS;
            double* p = u0 + sb + i * SSTEP;
            const double sn = TAB ? ssn[q] : (i == 0 ? sn0 : 0.0);
            double acc = vv * sn + cf * fr[i] + cm * p[0] + cp * Up[i];   // p[0]: U at c-1
            if (IS3) acc += cym * Ym[i] + cyp * Yp[i];
            if (i < CI) acc += ccf[i] * cr[i];
            p[0] = valid ? Uc[i] : 0.0;
            if (dl == 0) p[-1] = hx[i];
            if (dl == W - 1) p[1] = hx[i];
            sg[tid + i * NT] = acc;
        }
        __builtin_amdgcn_sched_barrier(0);
        load_row(Uc, min(c + 2, nm - 1));
        load_ynb(Ym, Yp, min(c + 2, nm - 1));
        load_side(min(c + 1, nm - 1));
        __syncthreads();
        if constexpr (sizeof(R) == 8) {
            // LDS to LDS: a partial unroll keeps the hoisted stencil reads few
            double sc = sc0;
#pragma unroll 2
            for (int i = 0; i < PER; ++i) {
                const int q = qb + i * RS;
                const double* p = u0 + sb + i * SSTEP;
                const double u = p[0];
                double ts = wk[0] * u;
#pragma unroll
                for (int j = 1; j < 7; ++j) ts += wk[j] * p[-j * WS];
                const double au = diag * u - cx * (p[-1] + p[1]);
                const double r = (sg[tid + i * NT] - (a.ta * ts + au)) * (TAB ? ssc[q] : sc);
                sg[tid + i * NT] = valid ? r : 0.0;
                if (!TAB) sc *= scs;
            }
            __syncthreads();
        } else {
            R rr[PER];
            double sc = sc0;
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const int q = qb + i * RS;
                const double* p = u0 + sb + i * SSTEP;
                const double u = p[0];
                double ts = wk[0] * u;
#pragma unroll
                for (int j = 1; j < 7; ++j) ts += wk[j] * p[-j * WS];
                const double au = diag * u - cx * (p[-1] + p[1]);
                const double r = (sg[tid + i * NT] - (a.ta * ts + au)) * (TAB ? ssc[q] : sc);
                rr[i] = valid ? (R)r : (R)0;
                if (!TAB) sc *= scs;
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < PER; ++i) smr[tid + i * NT] = rr[i];
            __syncthreads();
        }
        lds_fft<R, LOGN, B, NT, false, true, 0, 0, 1, FMAXLOG>(sm, stw);
        store_half_spectrum<R, N, B, NT, false>(sm, reinterpret_cast<T*>(a.S), a.ldS, (int)(slot0 + c * sslot), a.Mp);
        __syncthreads();
    };

    // prologue: U at c0 - 1 into the LDS tile, U at c0 and c0 + 1 and the rest of c0 into registers
    load_row(A, max(c0 - 1, 0));
    __syncthreads();   // tables and zero rows
#pragma unroll
    for (int i = 0; i < PER; ++i) u0[sb + i * SSTEP] = valid ? A[i] : 0.0;
    load_row(A, c0);
    load_row(Bv, min(c0 + 1, nm - 1));
    if constexpr (YAHEAD) {
        load_ynb(ymA, ypA, c0);
        load_ynb(ymB, ypB, min(c0 + 1, nm - 1));
    }
    load_side(c0);
    __syncthreads();
    for (int c = c0; c < c1; c += 2) {
        if constexpr (YAHEAD) {
            step(c, A, Bv, ymA, ypA);
            if (c + 1 < c1) step(c + 1, Bv, A, ymB, ypB);
        } else {
            step(c, A, Bv, ymA, ypA);
            if (c + 1 < c1) step(c + 1, Bv, A, ymA, ypA);
        }
    }
}

// ---------------------------------------------------------------------------
// Direct form, BDF-k (eq. BDF-k-F): the right-hand side is the source part G
// (the same every sweep) plus a relaxation term that is nonzero only in rows
// n = 1..k.  Its spectrum is therefore the stored spectrum of kappa^{q/N} G
// (computed once when the data are bound) plus a k-term DFT per dof:
//   H_p = Sg_p + sum_{n=1..k} kappa^{(n-1)/N} c_n e^{-2 pi i (n-1) p/N},
//   c_n = kappa tau^{-1} sum_{j=n..k} w_j U^{N+n-j},
// which replaces the forward kernel of a direct sweep (no FFT, U read only in
// its last k rows).  One lane per spectrum slot and a chunk of frequencies.
template <typename R>
__global__ __launch_bounds__(256) void k_inject(FwdArgs a, const void* Sg, int pchunk) {
    using T = cx<R>;
    const int P0 = blockIdx.y * pchunk, P1 = min(a.N / 2 + 1, P0 + pchunk);
    const int slot = blockIdx.x * 256 + threadIdx.x;
    if (slot >= a.Mp) return;
    const int d = slot_dof(slot, a.mx, a.mxp, a.Mp);
    double c[6];
#pragma unroll
    for (int n = 1; n <= 6; ++n) {
        double acc = 0.0;
        if (d >= 0 && n <= a.k)
            for (int j = n; j <= a.k; ++j) acc += a.wk[j] * a.U[(size_t)(a.N + n - j - 1) * a.M + d];
        c[n - 1] = n <= a.k ? a.kappa * a.ta * acc * a.scale[n - 1] : 0.0;
    }
    const T* src = reinterpret_cast<const T*>(Sg);
    T* dst = reinterpret_cast<T*>(a.S);
    const T* tw = reinterpret_cast<const T*>(a.tw);
    for (int p = P0; p < P1; ++p) {
        const T g = src[(size_t)p * a.ldS + slot];
        double hr = (double)g.x, hi = (double)g.y;
#pragma unroll
        for (int n = 1; n <= 6; ++n) {
            if (n > a.k) break;
            const T w = tw[((n - 1) * p) & (a.N - 1)];
            hr += c[n - 1] * (double)w.x;
            hi += c[n - 1] * (double)w.y;
        }
        dst[(size_t)p * a.ldS + slot] = mk<T>((R)hr, (R)hi);
    }
}

// ---------------------------------------------------------------------------
// Forward kernel, CQ-BDF-k (alpha < 1).  The history sum over all earlier
// levels is a causal convolution in time; it is evaluated per dof pair as a
// length-2N circular convolution (the circulant embedding of the Toeplitz
// history matrix, Sec. 3.2 cost paragraph) with FP64 FFTs in LDS:
//   c = IFFT_2N( FFT_2N(omega, 0) . FFT_2N(u, 0) ),  u_i = U^{i+1}.
// residual: r_n = G_n - tau^{-alpha} c_{n-1} - A_h U^n;
// direct:   F_n = G_n + kappa tau^{-alpha} c_{N+n-1} (= sum_{j=n..N-1} w_j U^{N+n-j}).
// Persistent: each workgroup (one per CU, the tile and twiddle tables fill the
// LDS) walks tiles of W dofs, reading the twiddles into LDS once.  Per tile,
// Phase A issues every global load at once (U, the stencil neighbours outside
// the tile, v, f, corrections) and folds all but the history term into one
// FP64 register per element (x neighbours inside the tile are read back from
// LDS); the DFT of omega and the scale factors are fetched while the
// transforms run.  In 2D/3D the tiles of a workgroup go down grid columns, so
// the tiles that workgroups of one XCD hold at the same time are y neighbours
// and the neighbour loads hit in that XCD's L2.
template <typename R, int LOGN, int W, int NT>
__global__ __launch_bounds__(NT, 1) void k_fwd_cq(FwdArgs a, int nvirt) {
    using T = cx<R>;
    constexpr int N = 1 << LOGN;
    constexpr int N2 = 2 * N;
    constexpr int B = W / 2;
    constexpr int PER = N * W / NT;     // time rows of the tile per thread; also points per thread of the 2N product
    static_assert(PER * NT == N * W, "tile shape");
    constexpr int RS = NT / W;          // time rows between a thread's consecutive elements
    static_assert(RS >= 8, "correction rows must lie in the first row group");
    // twiddles in LDS when they fit beside the tile (N <= 1024), else read from the global tables
    constexpr bool TWL = (size_t)N2 * B * 16 + (size_t)N * 16 + (size_t)(N / 2) * sizeof(T) <= 163840;
    __shared__ double2 cb[N2 * B];
    __shared__ double2 stw2[TWL ? N : 1];   // e^{-2 pi i j/(2N)}, j < N
    __shared__ T stw1[TWL ? N / 2 : 1];     // e^{-2 pi i j/N}, j < N/2, in the spectrum precision
    double* cbr = reinterpret_cast<double*>(cb);
    const double2* tw2 = TWL ? stw2 : a.tw2;
    const T* tw1 = TWL ? stw1 : reinterpret_cast<const T*>(a.tw);

    if constexpr (TWL) {
        for (int j = threadIdx.x; j < N; j += NT) {
            stw2[j] = a.tw2[j];
            if (j < N / 2) stw1[j] = reinterpret_cast<const T*>(a.tw)[j];
        }
    }
    const int ntiles = (a.Mp + W - 1) / W;
    const bool cols = a.my > 1 && a.mxp >= W;
    const size_t M = a.M;
    const bool resid = a.form == 0;
    const size_t sy = (size_t)a.mx, sz = (size_t)a.mx * a.my;
    const bool has3 = a.mz > 1;
    const double diag = 2.0 * (a.ihx2 + a.ihy2 + a.ihz2);
    // the residual form reads convolution rows [0, N), the direct form rows
    // [N, 2N); the time-FFT buffer (N x B values of cx<R>) goes into the other
    // half, so it never overwrites a value still to be read
    T* sm = reinterpret_cast<T*>(cb + (resid ? N * B : 0));
    R* smr = reinterpret_cast<R*>(sm);
    const int crow = resid ? 0 : N;

    for (int vb = blockIdx.x; vb < nvirt; vb += gridDim.x) {
        const int tile = cols ? xcd_tile_columns(vb, nvirt, a.mxp / W) : xcd_tile(vb, nvirt);
        if (tile >= ntiles) continue;   // uniform over the workgroup
        const int tid = loop_tid();
        const int dl = tid % W;
        const int qb = tid / W;
        const int d0 = tile * W;
        const int d = slot_dof(d0 + dl, a.mx, a.mxp, a.Mp);
        const bool valid = d >= 0;
        int x = 0, y = 0, z = 0;
        if (valid) {
            x = d % a.mx;
            const int rr = d / a.mx;
            y = rr % a.my;
            z = rr / a.my;
        }
        const bool hxm = x > 0, hxp = x < a.mx - 1;
        // Buffer loads: a scalar base per wave and row group (the wave's first
        // time row qb0 + i RS) plus a 32-bit byte offset per lane that is fixed
        // for the tile.  Absent stencil neighbours and padding slots take the
        // offset kNoLane and read 0, so every load is unconditional.
        const int qb0 = __builtin_amdgcn_readfirstlane(qb);
        const bool nb = resid && valid;
        const unsigned lu = valid ? ((unsigned)(qb - qb0) * (unsigned)M + (unsigned)d) * 8u : kNoLane;
        const unsigned lxm = (nb && hxm && dl == 0) ? lu - 8u : kNoLane;
        const unsigned lxp = (nb && hxp && dl == W - 1) ? lu + 8u : kNoLane;
        const unsigned lym = (nb && y > 0) ? lu - 8u * (unsigned)sy : kNoLane;
        const unsigned lyp = (nb && y < a.my - 1) ? lu + 8u * (unsigned)sy : kNoLane;
        const unsigned lzm = (nb && z > 0) ? lu - 8u * (unsigned)sz : kNoLane;
        const unsigned lzp = (nb && z < a.mz - 1) ? lu + 8u * (unsigned)sz : kNoLane;
        const unsigned lq = (unsigned)(qb - qb0) * 8u;   // per-row tables s, scale
        const double vt = a.ta * buf_ld(buf_rsrc(a.v, M * 8), valid ? (unsigned)d * 8u : kNoLane, 0.0);

        double g[PER];
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const size_t r0 = (size_t)(qb0 + i * RS);
            const auto rU = buf_rsrc(a.U + r0 * M, ((size_t)a.N - r0) * M * 8);
            const double u = buf_ld(rU, lu, 0.0);
            double acc = vt * buf_ld(buf_rsrc(a.s + r0, ((size_t)a.N - r0) * 8), lq, 0.0);
            if (a.f) acc += buf_ld(buf_rsrc(a.f + (r0 + 1) * M, ((size_t)a.N - r0) * M * 8), lu, 0.0);
            if (resid) {
                acc += a.ihx2 * (buf_ld(rU, lxm, 0.0) + buf_ld(rU, lxp, 0.0)) +
                       a.ihy2 * (buf_ld(rU, lym, 0.0) + buf_ld(rU, lyp, 0.0));
                if (has3) acc += a.ihz2 * (buf_ld(rU, lzm, 0.0) + buf_ld(rU, lzp, 0.0));
            }
            cbr[tid + i * NT] = u;
            cbr[N * W + tid + i * NT] = 0.0;   // zero padding to length 2N
            g[i] = acc;
        }
        if (a.ncorr > 0) {
            // correction rows q < ncorr <= 5 all lie in row group 0 (RS >= 8)
            const unsigned lc = (valid && qb < a.ncorr) ? ((unsigned)qb * (unsigned)M + (unsigned)d) * 8u : kNoLane;
            g[0] += buf_ld(buf_rsrc(a.corr, (size_t)a.ncorr * M * 8), lc, 0.0);
        }
        __syncthreads();
        if (resid) {
            // A_h U^n: centre and the x neighbours inside the tile
            const double cim = (hxm && dl > 0) ? a.ihx2 : 0.0, cip = (hxp && dl < W - 1) ? a.ihx2 : 0.0;
            const int om = dl > 0 ? -1 : 0, op = dl < W - 1 ? 1 : 0;
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const double* sp = cbr + tid + i * NT;
                g[i] -= diag * sp[0] - cim * sp[om] - cip * sp[op];
            }
        }
        // DFT of omega at the points this thread multiplies (consumed after the forward FFT)
        double2 wv[PER];
        const auto rW = buf_rsrc(a.what, (size_t)N2 * 16);
#pragma unroll
        for (int j = 0; j < PER; ++j) wv[j] = buf_ld(rW, (unsigned)((tid + j * NT) / B) * 16u, double2{});
        lds_fft<double, LOGN + 1, B, NT, false, true, 0>(cb, tw2, tid);
#pragma unroll
        for (int j = 0; j < PER; ++j) cb[tid + j * NT] = cmul(cb[tid + j * NT], wv[j]);
        double sc[PER];
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const size_t r0 = (size_t)(qb0 + i * RS);
            sc[i] = buf_ld(buf_rsrc(a.scale + r0, ((size_t)a.N - r0) * 8), lq, 0.0);
        }
        __syncthreads();
        lds_fft<double, LOGN + 1, B, NT, true, true, 0>(cb, tw2, tid);
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const double c = cbr[crow * W + tid + i * NT];
            const double r = resid ? g[i] - a.ta * c : g[i] + a.kappa * a.ta * c;
            smr[tid + i * NT] = valid ? (R)(r * sc[i]) : (R)0;
        }
        __syncthreads();
        lds_fft<R, LOGN, B, NT, false, true, 0>(sm, tw1, tid);
        store_half_spectrum<R, N, B, NT>(sm, reinterpret_cast<T*>(a.S), a.ldS, d0, a.Mp, tid);
        __syncthreads();   // the next tile overwrites the buffer
    }
}

// ---------------------------------------------------------------------------
// Forward kernel, CQ-BDF-k residual form on 2D grids, marching along y.
// The history convolution of k_fwd_cq is split into two length-N transforms:
// with z the tile's pair sequences, zero-padded to 2N, and t_j = e^{-pi i j/N},
// the even points of FFT_2N(z, 0) are FFT_N(z) and the odd points FFT_N(z t),
// so for j < N
//   c_j = IFFT_N(W_even . FFT_N(z))_j + conj(t_j) IFFT_N(W_odd . FFT_N(z t))_j,
// W the 2N-point DFT of (omega, 0) divided by 2N.  Both halves go through one
// batched length-N transform pair over 2B sequences (z and z t side by side in
// an N x 2B buffer, half the size of the 2N x B one), so the omega DFT, the
// twiddles and the per-row factors all stay in LDS and no partial sum is held
// in registers across a transform.  As in k_fwd_march, a workgroup owns W x
// slots and walks a chunk of y; each lane keeps its time rows of U at y-1, y,
// y+1 in registers (renamed, never copied), x neighbours inside the tile come
// from the adjacent lanes (DPP), and the load of U at y+2 is issued once U at
// y-1 has been used, one whole position (two batched FP64 transforms, the time
// FFT and the spectrum store) before it is needed.
template <int W>
__device__ __forceinline__ double lane_dpp(double v, bool next) {
    if constexpr (W <= 16) {
        // row_shl:1 / row_shr:1 inside 16-lane DPP rows (the W-lane groups never
        // straddle a row); a lane with no source in its row reads 0
        const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
        int lo = (int)(unsigned)b, hi = (int)(unsigned)(b >> 32);
        if (next) {
            lo = __builtin_amdgcn_update_dpp(0, lo, 0x101, 0xF, 0xF, true);
            hi = __builtin_amdgcn_update_dpp(0, hi, 0x101, 0xF, 0xF, true);
        } else {
            lo = __builtin_amdgcn_update_dpp(0, lo, 0x111, 0xF, 0xF, true);
            hi = __builtin_amdgcn_update_dpp(0, hi, 0x111, 0xF, 0xF, true);
        }
        return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
    } else {
        return next ? __shfl_down(v, 1, 64) : __shfl_up(v, 1, 64);
    }
}
// value of the partner lane (lane ^ 1): quad_perm [1, 0, 3, 2]
__device__ __forceinline__ double lane_pair(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, 0xB1, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), 0xB1, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
// x slots per tile of the CQ march: 4096 (time row, slot) elements
constexpr int cqm_tile(int logn) {
    const int w = 4096 >> logn;
    return w > 64 ? 64 : (w < 2 ? 2 : w);
}
template <typename R, int LOGN, int W> constexpr size_t cqm_lds() {
    constexpr size_t N = size_t(1) << LOGN;
    return N * W * 8 * 2 + 3 * N * 16 + (N / 2) * sizeof(cx<R>) + 2 * N * 8;
}
// MAXLOG: log2 of the largest radix of the length-N transforms (3 or 4).
template <typename R, int LOGN, int W, int NT, int MAXLOG>
__global__ __launch_bounds__(NT, 1) void k_fwd_cqm(FwdArgs a, int ncol, int nchunk, int chunk) {
    using T = cx<R>;
    constexpr int N = 1 << LOGN;
    constexpr int B = W / 2;
    constexpr int PER = N * W / NT;     // (time row, slot) elements per thread
    constexpr int PC = 2 * N * B / NT;  // complex points per thread in the pointwise products
    constexpr int RS = NT / W;          // time rows between a thread's consecutive elements
    static_assert(PER * NT == N * W && PC * NT == 2 * N * B && RS >= 8, "tile shape");
    // 2B sequences transformed together: the B pair sequences z (even points)
    // and the B twisted sequences z t (odd points); row q holds 2W doubles
    __shared__ double2 buf[N * 2 * B];  // then the time-FFT buffer (cx<R>, N x B)
    __shared__ double2 swe[N], swo[N];  // W_{2j}, W_{2j+1}
    __shared__ double2 stw[N];          // e^{-pi i j/N}, j < N (twist; FFT_N twiddles at stride 2)
    __shared__ T stw1[N / 2];           // e^{-2 pi i j/N} in the spectrum precision
    __shared__ double ssn[N], ssc[N];   // tau^{-alpha} s_q and kappa^{q/N}
    double* cbr = reinterpret_cast<double*>(buf);
    R* smr = reinterpret_cast<R*>(buf);
    T* sm = reinterpret_cast<T*>(buf);

    const int lin = xcd_tile(blockIdx.x, gridDim.x);
    if (lin >= ncol * nchunk) return;
    const int xt = lin % ncol, chk = lin / ncol;
    const int nm = a.my;
    const int c0 = chk * chunk, c1 = min(nm, c0 + chunk);
    const int tid = threadIdx.x;
    const int dl = tid % W;
    const int qb = tid / W;
    const int x = xt * W + dl;
    const bool valid = x < a.mx;
    const size_t M = a.M;
    const long long sdof = a.mx;                    // dof stride along y
    const long long slot0 = (long long)xt * W;

    for (int j = tid; j < N; j += NT) {
        swe[j] = a.what[2 * j];
        swo[j] = a.what[2 * j + 1];
        stw[j] = a.tw2[j];
        ssn[j] = a.ta * a.s[j];
        ssc[j] = a.scale[j];
        if (j < N / 2) stw1[j] = reinterpret_cast<const T*>(a.tw)[j];
    }
    // Loads: a uniform base per row group i and position c plus a 32-bit byte
    // offset per lane fixed for the whole kernel (the host checks that it
    // fits); padding slots and absent x neighbours read 0 through kNoLane.
    const unsigned lo = valid ? (unsigned)(((long long)qb * (long long)M + x) * 8) : kNoLane;
    const unsigned lhx = (valid && dl == 0 && x > 0) ? lo - 8u : ((valid && dl == W - 1 && x < a.mx - 1) ? lo + 8u : kNoLane);
    const unsigned lv = valid ? (unsigned)x * 8u : kNoLane;
    const size_t nU = (size_t)a.N * M;
    const double diag = 2.0 * (a.ihx2 + a.ihy2);
    const double cxm = dl > 0 ? a.ihx2 : 0.0, cxp = dl < W - 1 ? a.ihx2 : 0.0;   // inside the tile (DPP)
    const double hxc = (dl == 0 || dl == W - 1) ? a.ihx2 : 0.0;                   // the halo value
    const double sgn = (dl & 1) ? 1.0 : -1.0;      // odd lanes hold imaginary parts of the pairs

    double A[PER], Bv[PER], C[PER];
    auto load_row = [&](double (&dst)[PER], int c) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const size_t e0 = (size_t)i * RS * M + (size_t)c * sdof;
            dst[i] = buf_ld(buf_rsrc(a.U + e0, (nU - e0) * 8), lo, 0.0);
        }
    };

    // One position c with U at c-1, c, c+1 in Um, Uc, Up; Um is refilled with U at c+2.
    // The x halo, v, f and the corrections of position c are read at its start
    // and used after the transforms of the convolution.
    auto step = [&](int c, double (&Um)[PER], double (&Uc)[PER], double (&Up)[PER]) {
        const double cm = c > 0 ? a.ihy2 : 0.0, cp = c < nm - 1 ? a.ihy2 : 0.0;
        const int t = loop_tid();   // LDS addressing is recomputed per position, not hoisted
        double hx[PER], fr[PER];
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const size_t e0 = (size_t)i * RS * M + (size_t)c * sdof;
            hx[i] = buf_ld(buf_rsrc(a.U + e0, (nU - e0) * 8), lhx, 0.0);
        }
        const double vv = buf_ld(buf_rsrc(a.v + (size_t)c * sdof, (M - (size_t)c * sdof) * 8), lv, 0.0);
        if (a.f) {
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const size_t e0 = (size_t)(i * RS + 1) * M + (size_t)c * sdof;
                fr[i] = buf_ld(buf_rsrc(a.f + e0, ((size_t)a.N * M + M - e0) * 8), lo, 0.0);
            }
        }
        double cr = 0.0;
        if (a.ncorr > 0) {   // rows q < ncorr <= 5 lie in row group 0
            const size_t e0 = (size_t)c * sdof;
            cr = buf_ld(buf_rsrc(a.corr + e0, ((size_t)a.ncorr * M - e0) * 8), qb < a.ncorr ? lo : kNoLane, 0.0);
        }
        // both halves of the 2N-point transform in one batch: z in the first W
        // doubles of each row, z t_q in the second W (pair partner from the adjacent lane)
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int q = t / W + i * RS;
            const int e = q * 2 * W + t % W;
            const double2 tq = stw[q];
            const double u = Uc[i];
            cbr[e] = u;
            cbr[e + W] = u * tq.x + sgn * lane_pair(u) * tq.y;
        }
        __syncthreads();
        lds_fft<double, LOGN, 2 * B, NT, false, true, 0, 0, 2, MAXLOG>(buf, stw, t);
#pragma unroll
        for (int j = 0; j < PC; ++j) {
            const int idx = t + j * NT, pf = idx / (2 * B);
            buf[idx] = cmul(buf[idx], (idx % (2 * B)) < B ? swe[pf] : swo[pf]);
        }
        __syncthreads();
        lds_fft<double, LOGN, 2 * B, NT, true, true, 0, 0, 2, MAXLOG>(buf, stw, t);
        // r = (G - A_h U^n - tau^{-alpha} c) kappa^{q/N}
        double r[PER];
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int q = t / W + i * RS;
            const int e = q * 2 * W + t % W;
            const double2 tq = stw[q];
            const double p = cbr[e + W];
            const double c2 = p * tq.x - sgn * lane_pair(p) * tq.y;   // conj(t_q) times the pair value
            const double u = Uc[i];
            const double xm = lane_dpp<W>(u, false), xp = lane_dpp<W>(u, true);
            const double au = diag * u - cxm * xm - cxp * xp - hxc * hx[i] - cm * Um[i] - cp * Up[i];
            double g = ssn[q] * vv - au;
            if (a.f) g += fr[i];
            if (i == 0) g += cr;
            r[i] = (g - a.ta * (cbr[e] + c2)) * ssc[q];
        }
        // U at c-1 is consumed: prefetch U at c+2
        __builtin_amdgcn_sched_barrier(0);
        load_row(Um, min(c + 2, nm - 1));
        __syncthreads();   // the R buffer aliases FP64 elements of other lanes
#pragma unroll
        for (int i = 0; i < PER; ++i) smr[t + i * NT] = valid ? (R)r[i] : (R)0;
        __syncthreads();
        lds_fft<R, LOGN, B, NT, false, true, 0, 0, 1, MAXLOG>(sm, stw1, t);
        store_half_spectrum<R, N, B, NT, false>(sm, reinterpret_cast<T*>(a.S), a.ldS, (int)(slot0 + (long long)c * a.mxp),
                                                a.Mp, t);
        __syncthreads();
    };

    load_row(A, max(c0 - 1, 0));
    load_row(Bv, c0);
    load_row(C, min(c0 + 1, nm - 1));
    __syncthreads();   // tables
    for (int c = c0; c < c1; c += 3) {
        step(c, A, Bv, C);
        if (c + 1 < c1) step(c + 1, Bv, C, A);
        if (c + 2 < c1) step(c + 2, C, A, Bv);
    }
}

// ---------------------------------------------------------------------------
// Inverse kernel: rebuild the packed-pair spectrum Z_p = A_p + i B_p for all
// p from the retained half (conjugate symmetry), inverse FFT in LDS, scale row
// q by kappa^{-q/N}/N (FP64), update U and accumulate the update norms.  The
// U tile is fetched into registers together with the spectrum, so both
// streams of loads are in flight at once.
template <typename R, int LOGN, int W, int NT>
__global__ __launch_bounds__(NT, PINT_INV_WAVES) void k_inv(InvArgs a) {
    constexpr int N = 1 << LOGN;
    constexpr int B = W / 2;
    constexpr int NP = N / 2 + 1;
    constexpr int PER = N * W / NT;
    constexpr int PERS = (NP * B + NT - 1) / NT;
    static_assert(PER * NT == N * W, "tile shape");
    __shared__ cx<R> sm[N * B];
    __shared__ cx<R> stw[N / 2];    // twiddles w^j, j < N/2 (the only ones the stages use)
    __shared__ double sun[N];       // kappa^{-q/N}/N
    __shared__ double red[2][NT / 64];
    R* smr = reinterpret_cast<R*>(sm);
    const int tid = threadIdx.x;

    const int ntiles = (a.Mp + W - 1) / W;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= ntiles) {
        if (tid == 0) {
            a.partial[2 * blockIdx.x] = 0.0;
            a.partial[2 * blockIdx.x + 1] = 0.0;
        }
        return;
    }
    const int d0 = tile * W;
    const int dl = tid % W;
    const int d = slot_dof(d0 + dl, a.mx, a.mxp, a.Mp);
    const bool valid = d >= 0;
    const size_t M = a.M;
    const cx<R>* S = reinterpret_cast<const cx<R>*>(a.S);

    cx<R> sa[PERS], sb[PERS];
#pragma unroll
    for (int i = 0; i < PERS; ++i) {
        const int idx = tid + i * NT;
        sa[i] = mk<cx<R>>(0, 0);
        sb[i] = mk<cx<R>>(0, 0);
        if (idx < NP * B) {
            const int b = idx % B, p = idx / B;
            const int e = d0 + 2 * b;
            const cx<R>* row = S + (size_t)p * a.ldS;
            if (e < a.Mp) sa[i] = row[e];
            if (e + 1 < a.Mp) sb[i] = row[e + 1];
        }
    }
    double u[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int q = (tid + i * NT) / W;
        u[i] = valid ? a.U[(size_t)q * M + d] : 0.0;
    }
    // The FFT reads its twiddles from LDS: a global twiddle load there would
    // wait (in-order vector-memory counter) for the U tile loaded above.
    // The scaling table too: a global load between the U stores below would
    // make every store wait for the previous one.
    for (int j = tid; j < N / 2; j += NT) stw[j] = reinterpret_cast<const cx<R>*>(a.tw)[j];
    for (int j = tid; j < N; j += NT) sun[j] = a.unscale[j];
#pragma unroll
    for (int i = 0; i < PERS; ++i) {
        const int idx = tid + i * NT;
        if (idx < NP * B) {
            const int b = idx % B, p = idx / B;
            cx<R> A = sa[i], Bv = sb[i];
            if (p == 0 || p == N / 2) {
                A.y = 0;
                Bv.y = 0;
            }
            sm[p * B + b] = mk<cx<R>>(A.x - Bv.y, A.y + Bv.x);
            if (p > 0 && p < N / 2) sm[(N - p) * B + b] = mk<cx<R>>(A.x + Bv.y, Bv.x - A.y);
        }
    }
    __syncthreads();
    lds_fft<R, LOGN, B, NT, true, true, 0>(sm, stw);

    double mx = 0.0, s2 = 0.0;
    bool bad = false;
    if (valid) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int q = (tid + i * NT) / W;
            const double delta = (double)smr[q * W + dl] * sun[q];
            const double un = a.form == 0 ? u[i] + delta : delta;
            const double upd = un - u[i];
            a.U[(size_t)q * M + d] = un;
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

// One workgroup of 1024 lanes; each lane has eight partial pairs in flight
// before it uses any (a loop of dependent loads made the reduction of the
// 64K partials of a 3D sweep take 0.2 ms).  Fixed order: per lane, then across
// a wave by butterfly, then across waves, so the result is deterministic.
constexpr int kNormNT = 1024;
__global__ __launch_bounds__(kNormNT) void k_norm_reduce(const double* __restrict__ partial, int nb, double hd,
                                                         double* __restrict__ out) {
    __shared__ double red[2][kNormNT / 64];
    const int tid = threadIdx.x;
    const double2* p2 = reinterpret_cast<const double2*>(partial);   // (max |delta|, sum delta^2) pairs
    double mx = 0.0, s2 = 0.0;
    for (int base = 0; base < nb; base += 8 * kNormNT) {
        double vx[8], vy[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int i = base + k * kNormNT + tid;
            vx[k] = 0.0;
            vy[k] = 0.0;
            if (i < nb) {
                const double2 t = p2[i];
                vx[k] = t.x;
                vy[k] = t.y;
            }
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            mx = nanmax(mx, vx[k]);
            s2 += vy[k];
        }
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
        for (int i = 1; i < kNormNT / 64; ++i) {
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
    constexpr int PS = pad_shift(LOGL);
    constexpr int LP = L + (L >> PS);            // padded sequence stride
    __shared__ T sm[ROWS * LP];
    // Twiddles in LDS (when two workgroups per CU still fit), so that the FFT
    // does not wait on the vector-memory counter behind the next group's prefetch.
    constexpr bool TWL = (ROWS * LP + L / 2) * (int)sizeof(T) <= 81920;
    __shared__ T stw[TWL ? L / 2 : 1];
    const T* tw = TWL ? stw : reinterpret_cast<const T*>(a.twL[0]);
    if (TWL)
        for (int j = threadIdx.x; j < L / 2; j += NT) stw[j] = reinterpret_cast<const T*>(a.twL[0])[j];
    auto ix = [](int b, int t) { return b * LP + t + (t >> PS); };
    const int m = a.mx;
    const int lpp = a.my * a.mz;
    T* S = reinterpret_cast<T*>(a.S);
    const T zero = mk<T>((R)0, (R)0);
    const long long ngroups = (nlines + ROWS - 1) / ROWS;
    // Element e of a group is (row b, position t) = (e >> LH, e & (H - 1)) with
    // H = L/2 > m, so no integer division appears per element; the offset of
    // each row of the group is computed once per group into LDS.
    constexpr int H = L / 2;
    constexpr int LH = LOGL - 1;
    constexpr int PER = (ROWS * H + NT - 1) / NT;
    __shared__ long long rowoff[2][ROWS];
    T val[PER];
    auto offsets = [&](long long grp, int slot) {
        if (threadIdx.x < ROWS) {
            const long long g = grp * ROWS + threadIdx.x;
            const unsigned gu = (unsigned)g;
            rowoff[slot][threadIdx.x] =
                g < nlines ? (long long)(gu / (unsigned)lpp) * a.ldS + (long long)(gu % (unsigned)lpp) * a.mxp : -1;
        }
    };
    const unsigned long long sbytes = (unsigned long long)a.nP * a.ldS * sizeof(T);
    // offset of the first row of group grp (uniform, so the descriptor stays scalar)
    auto first_row = [&](long long grp) {
        const unsigned g = (unsigned)(grp * ROWS);
        return (long long)(g / (unsigned)lpp) * a.ldS + (long long)(g % (unsigned)lpp) * a.mxp;
    };
    // byte offset of (row b, position t) from the group's first row o0, or kNoLane
    auto lane_off = [&](int slot, long long o0, int b, int t, bool ok) {
        const long long off = rowoff[slot][b];
        return (ok && off >= 0) ? (unsigned)((off - o0 + t) * (long long)sizeof(T)) : kNoLane;
    };
    // A group past the end gets an empty descriptor: its loads return 0 without
    // touching memory, so every iteration issues the same loads.
    auto fetch = [&](int slot, long long grp) {
        const bool live = grp < ngroups;
        const long long o0 = live ? first_row(grp) : 0;
        const __amdgpu_buffer_rsrc_t rs = buf_rsrc(S + o0, live ? sbytes - (unsigned long long)o0 * sizeof(T) : 0);
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = threadIdx.x + i * NT;
            const bool in = (ROWS * H) % NT == 0 || e < ROWS * H;
            const int b = in ? e >> LH : 0, t = e & (H - 1);
            val[i] = buf_ld(rs, lane_off(slot, o0, b, t, in && t < m), zero);
        }
    };
    long long grp = blockIdx.x;
    int slot = 0;
    if (grp < ngroups) {
        offsets(grp, 0);
        __syncthreads();
        fetch(0, grp);
    }
    for (; grp < ngroups; grp += gridDim.x, slot ^= 1) {
        const long long g0 = grp * ROWS;
        // odd extension: x_t at t and -x_t at L - t, zeros at 0 and m + 1
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = threadIdx.x + i * NT;
            const int b = e >> LH, t = (e & (H - 1)) + 1;
            if (((ROWS * H) % NT == 0 || e < ROWS * H) && t <= m) {
                sm[ix(b, t)] = val[i];
                sm[ix(b, L - t)] = mk<T>(-val[i].x, -val[i].y);
            }
        }
        if (threadIdx.x < 2 * ROWS) {
            const int b = threadIdx.x >> 1;
            sm[ix(b, (threadIdx.x & 1) ? m + 1 : 0)] = zero;
        }
        offsets(grp + gridDim.x, slot ^ 1);
        __syncthreads();
        fetch(slot ^ 1, grp + gridDim.x);
        lds_fft<R, LOGL, ROWS, NT, false, false, LP, PS>(sm, tw);
        if constexpr (SOLVE) {
            for (int idx = threadIdx.x; idx < ROWS * L; idx += NT) {
                const int b = idx >> LOGL, t = idx & (L - 1);
                if (t > m + 1) continue;
                const long long g = g0 + b;
                if (t == 0 || t == m + 1 || g >= nlines) {
                    sm[ix(b, t)] = zero;
                    if (t > 0 && t <= m) sm[ix(b, L - t)] = zero;
                    continue;
                }
                const double2 sg = a.sigma[(unsigned)g / (unsigned)lpp];
                const double dre = sg.x + a.mu[0][t - 1];
                const double inv = a.inv_factor / (dre * dre + sg.y * sg.y);
                const T c = mk<T>((R)(dre * inv), (R)(-sg.y * inv));
                const T z = cmul(sm[ix(b, t)], c);
                sm[ix(b, t)] = z;
                sm[ix(b, L - t)] = mk<T>(-z.x, -z.y);
            }
            __syncthreads();
            lds_fft<R, LOGL, ROWS, NT, false, false, LP, PS>(sm, tw);
        }
        const long long o0 = first_row(grp);
        const __amdgpu_buffer_rsrc_t rs = buf_rsrc(S + o0, sbytes - (unsigned long long)o0 * sizeof(T));
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = threadIdx.x + i * NT;
            const bool in = (ROWS * H) % NT == 0 || e < ROWS * H;
            const int b = in ? e >> LH : 0, t = (e & (H - 1)) + 1;
            buf_st(rs, lane_off(slot, o0, b, t - 1, in && t <= m), sm[ix(b, t)]);
        }
        __syncthreads();
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
    static_assert(NT % W == 0, "a lane keeps one column");
    __shared__ T sm[L * W];
    // Twiddles (when they fit) and the eigenvalues of the transformed axis in
    // LDS, so that neither the FFT nor the divide waits on the vector-memory
    // counter behind the next group's prefetch.
    constexpr bool TWL = (L * W + L / 2) * (int)sizeof(T) + (L / 2) * 8 <= 155648;
    __shared__ T stw[TWL ? L / 2 : 1];
    __shared__ double smu[SOLVE ? L / 2 : 1];
    const int m = axis == 1 ? a.my : a.mz;
    const long long st = axis == 1 ? (long long)a.mxp : (long long)a.mxp * a.my;
    const int other = axis == 1 ? a.mz : a.my;
    const int nxg = (a.mx + W - 1) / W;
    const long long ngroups = (long long)a.nP * other * nxg;
    T* S = reinterpret_cast<T*>(a.S);
    const T zero = mk<T>((R)0, (R)0);
    const T* tw = TWL ? stw : reinterpret_cast<const T*>(a.twL[axis]);
    if (TWL)
        for (int j = threadIdx.x; j < L / 2; j += NT) stw[j] = reinterpret_cast<const T*>(a.twL[axis])[j];
    if (SOLVE)
        for (int j = threadIdx.x; j < m; j += NT) smu[j] = a.mu[axis][j];
    const int wl = threadIdx.x % W;      // the column this lane loads, stores and scales
    struct Grp {
        int p, o, x0;
        long long base;
    };
    auto decode = [&](long long gid) {
        Grp g;
        const int xg = (int)(gid % nxg);
        const long long rest = gid / nxg;
        g.o = (int)(rest % other);
        g.p = (int)(rest / other);
        g.x0 = xg * W;
        g.base = (long long)g.p * a.ldS + g.x0 +
                 (axis == 1 ? (long long)g.o * a.mxp * a.my : (long long)g.o * a.mxp);
        return g;
    };
    // Persistent workgroups with the next group's loads (rows of W contiguous
    // values, and the x eigenvalue of the lane's column) issued before the
    // current group's transforms.
    constexpr int PER = ((L / 2 - 1) * W + NT - 1) / NT;
    T val[PER];
    double mux_next = 0.0, muo_next = 0.0;   // x eigenvalue of the lane's column, eigenvalue of the other axis
    double2 sg_next = double2{};             // sigma_p of the group
    const unsigned long long sbytes = (unsigned long long)a.nP * a.ldS * sizeof(T);
    // byte offset of row t of the lane's column from the group base, or kNoLane
    auto lane_off = [&](int t, bool ok) {
        return ok ? (unsigned)(((long long)t * st + wl) * (long long)sizeof(T)) : kNoLane;
    };
    // A group past the end (live = false) gets an empty descriptor: its loads
    // return 0 without touching memory, so every iteration issues the same loads.
    auto fetch = [&](const Grp& g, bool live) {
        const bool colok = live && g.x0 + wl < a.mx;
        const long long b0 = live ? g.base : 0;
        const __amdgpu_buffer_rsrc_t rs = buf_rsrc(S + b0, live ? sbytes - (unsigned long long)b0 * sizeof(T) : 0);
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int idx = threadIdx.x + i * NT;
            val[i] = buf_ld(rs, lane_off(idx / W, colok && idx < m * W), zero);
        }
        if (SOLVE) {
            mux_next = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
                                                      buf_rsrc(a.mu[0], (unsigned long long)a.mx * 8),
                                                      (int)(colok ? (unsigned)(g.x0 + wl) * 8u : kNoLane), 0, 0));
            sg_next = buf_ld(buf_rsrc(a.sigma, (unsigned long long)a.nP * 16), live ? (unsigned)g.p * 16u : kNoLane,
                             double2{});
            muo_next = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
                                                      buf_rsrc(a.mu[1], (unsigned long long)a.my * 8),
                                                      (int)(live && axis == 2 ? (unsigned)g.o * 8u : kNoLane), 0, 0));
        }
    };
    long long gid = blockIdx.x;
    if (gid < ngroups) fetch(decode(gid), true);
    for (; gid < ngroups; gid += gridDim.x) {
        const Grp g = decode(gid);
        const double mux = mux_next, muo = muo_next;
        const double2 sg = sg_next;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int idx = threadIdx.x + i * NT;
            if (idx < m * W) {
                const int t = idx / W + 1;
                sm[t * W + wl] = val[i];
                sm[(L - t) * W + wl] = mk<T>(-val[i].x, -val[i].y);
            }
        }
        if (threadIdx.x < 2 * W) sm[((threadIdx.x < W) ? 0 : m + 1) * W + wl] = zero;
        __syncthreads();
        fetch(decode(gid + gridDim.x), gid + gridDim.x < ngroups);
        lds_fft<R, LOGL, W, NT, false, true, 0>(sm, tw);
        if constexpr (SOLVE) {
            const double base_re = sg.x + (axis == 2 ? muo : 0.0) + mux;
            const bool colok = g.x0 + wl < a.mx;
            for (int idx = threadIdx.x; idx < (m + 2) * W; idx += NT) {
                const int t = idx / W;
                if (t == 0 || t == m + 1) {
                    sm[t * W + wl] = zero;
                } else if (!colok) {
                    sm[t * W + wl] = zero;
                    sm[(L - t) * W + wl] = zero;
                } else {
                    const double dre = base_re + smu[t - 1];
                    const double dim_ = sg.y;
                    const double inv = a.inv_factor / (dre * dre + dim_ * dim_);
                    const T c = mk<T>((R)(dre * inv), (R)(-dim_ * inv));
                    const T z = cmul(sm[t * W + wl], c);
                    sm[t * W + wl] = z;
                    sm[(L - t) * W + wl] = mk<T>(-z.x, -z.y);
                }
            }
            __syncthreads();
            lds_fft<R, LOGL, W, NT, false, true, 0>(sm, tw);
        }
        {
            const bool colok = g.x0 + wl < a.mx;
            const __amdgpu_buffer_rsrc_t rs = buf_rsrc(S + g.base, sbytes - (unsigned long long)g.base * sizeof(T));
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const int idx = threadIdx.x + i * NT;
                const bool ok = colok && idx < m * W;
                const int t = ok ? idx / W + 1 : 1;
                buf_st(rs, lane_off(t - 1, ok), sm[t * W + wl]);
            }
        }
        __syncthreads();
    }
}

// The same column pass with the odd extension folded into the first and last
// FFT stages (lengths L = 2^8..2^11, with a radix schedule that starts and ends
// with the same radix R0 = L / Q: 16 x 16, 8 x 8 x 8, 16 x 4 x 16, 16 x 8 x 16).
// For an odd sequence of length L (y_0 = y_{L/2} = 0, y_{L-t} = -y_t), butterfly
// j of the first Stockham stage reads y_{j + Q r}; its upper half r >= R0/2 is
// minus the lower half of butterfly Q - j, reversed:
// y_{j + Q r} = -x_{(Q - j) + Q (R0 - 1 - r)}.  So the loaded values x_t,
// t = 1..m, are written once in natural order (positions 0 and L/2 hold zero),
// and butterfly j reads x at j + Q s and at (Q - j) + Q s, s < R0/2: the odd
// extension is never stored, and no full-length read precedes the first stage.
// At the other end the last stage's butterfly j holds Y_{j + Q r}, whose lower
// half is the transform on k = 1..m: it is divided by the shift (SOLVE) and
// written in natural order for the second transform, or (last stage of the last
// transform) stored straight from registers.  That is two LDS passes fewer per
// transform than k_dst_cols (5.5 instead of 7.5 per value for L = 512, 3.5
// instead of 5.5 for L = 256), and one more fewer at the divide.
constexpr int fused_r0(int logl) { return (logl == 8 || logl == 10 || logl == 11) ? 16 : (logl == 9 ? 8 : 0); }

template <typename R, int LOGL, int W, int NT, bool SOLVE>
__global__ __launch_bounds__(NT) void k_dst_colsf(SpaceArgs a, int axis) {
    using T = cx<R>;
    constexpr int L = 1 << LOGL;
    constexpr int R0 = fused_r0(LOGL);
    static_assert(R0 == 8 || R0 == 16, "length without a fused radix schedule");
    constexpr int LR0 = R0 == 16 ? 4 : 3;
    constexpr int H = R0 / 2;
    constexpr int Q = L / R0;                  // butterflies per column in the first and last stage
    constexpr int LMID = LOGL - 2 * LR0;       // one middle stage of radix 2^LMID (0: none)
    static_assert(LMID == 0 || LMID == 2 || LMID == 3, "middle stage radix");
    constexpr int TASKS = Q * W;
    constexpr int TPL = (TASKS + NT - 1) / NT; // butterflies per lane
    static_assert(NT % W == 0, "a lane keeps one column");
    static_assert(TASKS % NT == 0 || TASKS < NT, "whole butterflies per lane");
    __shared__ T sm[L * W];
    constexpr bool TWL = (L * W + L / 2) * (int)sizeof(T) + (L / 2) * 8 <= 155648;
    __shared__ T stw[TWL ? L / 2 : 1];
    __shared__ double smu[SOLVE ? L / 2 : 1];
    const int m = axis == 1 ? a.my : a.mz;     // = L/2 - 1
    const long long st = axis == 1 ? (long long)a.mxp : (long long)a.mxp * a.my;
    const int other = axis == 1 ? a.mz : a.my;
    const int nxg = (a.mx + W - 1) / W;
    const long long ngroups = (long long)a.nP * other * nxg;
    T* S = reinterpret_cast<T*>(a.S);
    const T zero = mk<T>((R)0, (R)0);
    const T* tw = TWL ? stw : reinterpret_cast<const T*>(a.twL[axis]);
    if (TWL)
        for (int j = threadIdx.x; j < L / 2; j += NT) stw[j] = reinterpret_cast<const T*>(a.twL[axis])[j];
    if (SOLVE)
        for (int j = threadIdx.x; j < m; j += NT) smu[j] = a.mu[axis][j];
    const int wl = threadIdx.x % W;
    struct Grp {
        int p, o, x0;
        long long base;
    };
    auto decode = [&](long long gid) {
        Grp g;
        const int xg = (int)(gid % nxg);
        const long long rest = gid / nxg;
        g.o = (int)(rest % other);
        g.p = (int)(rest / other);
        g.x0 = xg * W;
        g.base = (long long)g.p * a.ldS + g.x0 +
                 (axis == 1 ? (long long)g.o * a.mxp * a.my : (long long)g.o * a.mxp);
        return g;
    };
    // butterfly g = 1..Q of task i (g = Q stands for j = 0)
    auto task_g = [&](int i) { return (int)(threadIdx.x + i * NT) / W + 1; };
    auto task_on = [&](int i) { return TASKS % NT == 0 || (int)(threadIdx.x + i * NT) < TASKS; };
    T val[TPL][H];
    double mux_next = 0.0, muo_next = 0.0;
    double2 sg_next = double2{};
    const unsigned long long sbytes = (unsigned long long)a.nP * a.ldS * sizeof(T);
    // byte offset of value t (1..m) of the lane's column from the group base, or kNoLane
    auto lane_off = [&](int t, bool ok) {
        return ok ? (unsigned)(((long long)(t - 1) * st + wl) * (long long)sizeof(T)) : kNoLane;
    };
    auto fetch = [&](const Grp& g, bool live) {
        const bool colok = live && g.x0 + wl < a.mx;
        const long long b0 = live ? g.base : 0;
        const __amdgpu_buffer_rsrc_t rs = buf_rsrc(S + b0, live ? sbytes - (unsigned long long)b0 * sizeof(T) : 0);
#pragma unroll
        for (int i = 0; i < TPL; ++i) {
            const int gg = task_g(i);
#pragma unroll
            for (int s = 0; s < H; ++s) {
                const int t = gg + Q * s;
                val[i][s] = buf_ld(rs, lane_off(t, colok && task_on(i) && t <= m), zero);
            }
        }
        if (SOLVE) {
            mux_next = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
                                                      buf_rsrc(a.mu[0], (unsigned long long)a.mx * 8),
                                                      (int)(colok ? (unsigned)(g.x0 + wl) * 8u : kNoLane), 0, 0));
            sg_next = buf_ld(buf_rsrc(a.sigma, (unsigned long long)a.nP * 16), live ? (unsigned)g.p * 16u : kNoLane,
                             double2{});
            muo_next = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
                                                      buf_rsrc(a.mu[1], (unsigned long long)a.my * 8),
                                                      (int)(live && axis == 2 ? (unsigned)g.o * 8u : kNoLane), 0, 0));
        }
    };
    // Odd sequences in natural layout sm[k W + col], k = 0..L/2 (k = 0 and L/2
    // hold zero): the first stage's butterfly j takes its lower half from
    // k = j + Q s and its upper half from k = (Q - j) + Q s, negated and
    // reversed; it writes position j R0 + r after a barrier.
    auto zero_ends = [&]() {
        if (threadIdx.x < 2 * W) sm[((threadIdx.x < W) ? 0 : L / 2) * W + wl] = zero;
    };
    auto first_stage = [&]() {
        T v[TPL][R0];
#pragma unroll
        for (int i = 0; i < TPL; ++i) {
            if (!task_on(i)) continue;
            const int j = task_g(i) % Q;
#pragma unroll
            for (int s2 = 0; s2 < H; ++s2) {
                v[i][s2] = sm[(j + Q * s2) * W + wl];
                const T p = sm[((Q - j) + Q * s2) * W + wl];
                v[i][R0 - 1 - s2] = mk<T>(-p.x, -p.y);
            }
            SmallDft<R0, false, T>::run(v[i]);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < TPL; ++i) {
            if (!task_on(i)) continue;
            const int j = task_g(i) % Q;
#pragma unroll
            for (int r = 0; r < R0; ++r) sm[(j * R0 + r) * W + wl] = v[i][r];
        }
        __syncthreads();
    };
    // Last stage (span Q): butterfly j = g mod Q reads y_{j + Q r}, twiddles
    // w^{r j}, DFT; returns the lower half (k = j + Q r, r < H) in Y.
    auto last_stage = [&](T (&Y)[TPL][H]) {
#pragma unroll
        for (int i = 0; i < TPL; ++i) {
            if (!task_on(i)) continue;
            const int j = task_g(i) % Q;
            T v[R0];
#pragma unroll
            for (int r = 0; r < R0; ++r) v[r] = sm[(j + Q * r) * W + wl];
            apply_twiddles<R0, false, T>(v, tw, j);
            SmallDft<R0, false, T>::run(v);
#pragma unroll
            for (int r = 0; r < H; ++r) Y[i][r] = v[r];
        }
    };
    auto middle = [&]() {
        if constexpr (LMID > 0) fft_stage<R, LOGL, (1 << LMID), W, NT, false, true, 0, 0, 1>(sm, tw, R0, threadIdx.x);
    };

    long long gid = blockIdx.x;
    if (gid < ngroups) fetch(decode(gid), true);
    for (; gid < ngroups; gid += gridDim.x) {
        const Grp g = decode(gid);
        const double mux = mux_next, muo = muo_next;
        const double2 sg = sg_next;
        const bool colok = g.x0 + wl < a.mx;
        // the loaded values x_t, t = g + Q s <= m, into the natural layout
#pragma unroll
        for (int i = 0; i < TPL; ++i) {
            if (!task_on(i)) continue;
            const int gg = task_g(i);
#pragma unroll
            for (int s2 = 0; s2 < H; ++s2) {
                const int t = gg + Q * s2;
                if (t <= m) sm[t * W + wl] = val[i][s2];
            }
        }
        zero_ends();
        __syncthreads();
        // the next group's loads fly during this group's transforms
        fetch(decode(gid + gridDim.x), gid + gridDim.x < ngroups);
        first_stage();
        middle();
        T Y[TPL][H];
        last_stage(Y);
        if constexpr (SOLVE) {
            const double base_re = sg.x + (axis == 2 ? muo : 0.0) + mux;
            __syncthreads();   // every last-stage read is done before the natural-layout writes
#pragma unroll
            for (int i = 0; i < TPL; ++i) {
                if (!task_on(i)) continue;
                const int j = task_g(i) % Q;
#pragma unroll
                for (int r = 0; r < H; ++r) {
                    const int k = j + Q * r;
                    if (k >= 1 && k <= m) {
                        // columns past the grid get 0 (a scalar factor: a select of the
                        // complex value itself is lowered through scratch memory)
                        const double dre = base_re + smu[k - 1];
                        const double inv = colok ? a.inv_factor / (dre * dre + sg.y * sg.y) : 0.0;
                        sm[k * W + wl] = cmul(Y[i][r], mk<T>((R)(dre * inv), (R)(-sg.y * inv)));
                    }
                }
            }
            zero_ends();
            __syncthreads();
            // the same raw transform again (the sine transform is its own inverse
            // up to the factor folded into inv_factor, sign included)
            first_stage();
            middle();
            last_stage(Y);
        }
        {
            const __amdgpu_buffer_rsrc_t rs = buf_rsrc(S + g.base, sbytes - (unsigned long long)g.base * sizeof(T));
#pragma unroll
            for (int i = 0; i < TPL; ++i) {
                const int j = task_g(i) % Q;
#pragma unroll
                for (int r = 0; r < H; ++r) {
                    const int t = j + Q * r;
                    buf_st(rs, lane_off(t, colok && task_on(i) && t >= 1 && t <= m), Y[i][r]);
                }
            }
        }
        __syncthreads();
    }
}

// The x pass without the divide, with the odd extension folded into the first
// and last FFT stages as in k_dst_colsf (same radix schedules and butterfly
// pairing), on the element-contiguous padded row layout of k_dst_rows: the row
// values are written once in natural order, butterfly j of the first stage reads
// positions j + Q s and (Q - j) + Q s, and the last stage's lower half is stored
// straight from registers.  Butterfly (row b, j) of task i: j fastest, so the
// stores of a wave cover consecutive positions of a row.
template <typename R, int LOGL, int ROWS, int NT>
__global__ __launch_bounds__(NT) void k_dst_rowsf(SpaceArgs a, long long nlines) {
    using T = cx<R>;
    constexpr int L = 1 << LOGL;
    constexpr int PS = pad_shift(LOGL);
    constexpr int LP = L + (L >> PS);            // padded sequence stride
    constexpr int R0 = fused_r0(LOGL);
    static_assert(R0 == 8 || R0 == 16, "length without a fused radix schedule");
    constexpr int LR0 = R0 == 16 ? 4 : 3;
    constexpr int HR = R0 / 2;
    constexpr int Q = L / R0;
    constexpr int LMID = LOGL - 2 * LR0;
    static_assert(LMID == 0 || LMID == 2 || LMID == 3, "middle stage radix");
    constexpr int TASKS = ROWS * Q;
    constexpr int TPL = (TASKS + NT - 1) / NT;
    static_assert(TASKS % NT == 0 || TASKS < NT, "whole butterflies per lane");
    __shared__ T sm[ROWS * LP];
    constexpr bool TWL = (ROWS * LP + L / 2) * (int)sizeof(T) <= 81920;
    __shared__ T stw[TWL ? L / 2 : 1];
    const T* tw = TWL ? stw : reinterpret_cast<const T*>(a.twL[0]);
    if (TWL)
        for (int j = threadIdx.x; j < L / 2; j += NT) stw[j] = reinterpret_cast<const T*>(a.twL[0])[j];
    auto ix = [](int b, int t) { return b * LP + t + (t >> PS); };
    const int m = a.mx;                          // = L/2 - 1
    const int lpp = a.my * a.mz;
    T* S = reinterpret_cast<T*>(a.S);
    const T zero = mk<T>((R)0, (R)0);
    const long long ngroups = (nlines + ROWS - 1) / ROWS;
    constexpr int H = L / 2;
    constexpr int LH = LOGL - 1;
    constexpr int PER = (ROWS * H + NT - 1) / NT;
    __shared__ long long rowoff[2][ROWS];
    T val[PER];
    auto offsets = [&](long long grp, int slot) {
        if (threadIdx.x < ROWS) {
            const long long g = grp * ROWS + threadIdx.x;
            const unsigned gu = (unsigned)g;
            rowoff[slot][threadIdx.x] =
                g < nlines ? (long long)(gu / (unsigned)lpp) * a.ldS + (long long)(gu % (unsigned)lpp) * a.mxp : -1;
        }
    };
    const unsigned long long sbytes = (unsigned long long)a.nP * a.ldS * sizeof(T);
    auto first_row = [&](long long grp) {
        const unsigned g = (unsigned)(grp * ROWS);
        return (long long)(g / (unsigned)lpp) * a.ldS + (long long)(g % (unsigned)lpp) * a.mxp;
    };
    auto lane_off = [&](int slot, long long o0, int b, int t, bool ok) {
        const long long off = rowoff[slot][b];
        return (ok && off >= 0) ? (unsigned)((off - o0 + t) * (long long)sizeof(T)) : kNoLane;
    };
    auto fetch = [&](int slot, long long grp) {
        const bool live = grp < ngroups;
        const long long o0 = live ? first_row(grp) : 0;
        const __amdgpu_buffer_rsrc_t rs = buf_rsrc(S + o0, live ? sbytes - (unsigned long long)o0 * sizeof(T) : 0);
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = threadIdx.x + i * NT;
            const bool in = (ROWS * H) % NT == 0 || e < ROWS * H;
            const int b = in ? e >> LH : 0, t = e & (H - 1);
            val[i] = buf_ld(rs, lane_off(slot, o0, b, t, in && t < m), zero);
        }
    };
    auto task_on = [&](int i) { return TASKS % NT == 0 || (int)(threadIdx.x + i * NT) < TASKS; };
    auto task_b = [&](int i) { return (int)(threadIdx.x + i * NT) / Q; };
    auto task_j = [&](int i) { return (int)(threadIdx.x + i * NT) % Q; };
    long long grp = blockIdx.x;
    int slot = 0;
    if (grp < ngroups) {
        offsets(grp, 0);
        __syncthreads();
        fetch(0, grp);
    }
    for (; grp < ngroups; grp += gridDim.x, slot ^= 1) {
        // natural order: x_t at t = 1..m, zeros at 0 and L/2
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = threadIdx.x + i * NT;
            const int b = e >> LH, t = (e & (H - 1)) + 1;
            if (((ROWS * H) % NT == 0 || e < ROWS * H) && t <= m) sm[ix(b, t)] = val[i];
        }
        if (threadIdx.x < 2 * ROWS) {
            const int b = threadIdx.x >> 1;
            sm[ix(b, (threadIdx.x & 1) ? H : 0)] = zero;
        }
        offsets(grp + gridDim.x, slot ^ 1);
        __syncthreads();
        fetch(slot ^ 1, grp + gridDim.x);
        // first stage (span 1) from the natural-order halves
        {
            T v[TPL][R0];
#pragma unroll
            for (int i = 0; i < TPL; ++i) {
                if (!task_on(i)) continue;
                const int b = task_b(i), j = task_j(i);
#pragma unroll
                for (int s2 = 0; s2 < HR; ++s2) {
                    v[i][s2] = sm[ix(b, j + Q * s2)];
                    const T p = sm[ix(b, (Q - j) + Q * s2)];
                    v[i][R0 - 1 - s2] = mk<T>(-p.x, -p.y);
                }
                SmallDft<R0, false, T>::run(v[i]);
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < TPL; ++i) {
                if (!task_on(i)) continue;
                const int b = task_b(i), j = task_j(i);
#pragma unroll
                for (int r = 0; r < R0; ++r) sm[ix(b, j * R0 + r)] = v[i][r];
            }
            __syncthreads();
        }
        if constexpr (LMID > 0)
            fft_stage<R, LOGL, (1 << LMID), ROWS, NT, false, false, LP, PS, 1>(sm, tw, R0, threadIdx.x);
        // last stage (span Q); its lower half Y_{j + Q r}, r < R0/2, is the transform on k = 1..m
        const long long o0 = first_row(grp);
        const __amdgpu_buffer_rsrc_t rs = buf_rsrc(S + o0, sbytes - (unsigned long long)o0 * sizeof(T));
#pragma unroll
        for (int i = 0; i < TPL; ++i) {
            // lanes without a butterfly read row 0 (in range) and store nothing; the
            // row index is selected, not the loaded value (a select of the complex
            // value itself is lowered through scratch memory)
            const int b = task_on(i) ? task_b(i) : 0, j = task_j(i);
            T v[R0];
#pragma unroll
            for (int r = 0; r < R0; ++r) v[r] = sm[ix(b, j + Q * r)];
            apply_twiddles<R0, false, T>(v, tw, j);
            SmallDft<R0, false, T>::run(v);
#pragma unroll
            for (int r = 0; r < HR; ++r) {
                const int t = j + Q * r;
                buf_st(rs, lane_off(slot, o0, b, t - 1, task_on(i) && t >= 1 && t <= m), v[r]);
            }
        }
        __syncthreads();
    }
}

// Raw sine transform of any length (axes whose 2(m+1) is not a power of two),
// by Bluestein's chirp-z identity jk = (j^2 + k^2 - (k-j)^2)/2:
//   Y_k = sum_{t<L} y_t e^{-2 pi i t k/L} = c_k sum_t (y_t c_t) conj(c_{k-t}),
//   c_t = e^{-pi i t^2/L},  L = 2(m+1),  y = odd extension of the line,
// the linear convolution evaluated with power-of-two FFTs of length P >= 2L-1
// in LDS: Y = c . IFFT_P(FFT_P(a) . Bh), a_t = y_t c_t (t < L, zero beyond),
// Bh = FFT_P(conj c wrapped to -(L-1)..L-1)/P (a host table).  It returns the
// same raw values Y_1..Y_m as the power-of-two path, so the scale factors agree.
// B lines (one grid line of one frequency plane each) per workgroup, layout
// [P][B] in LDS.  With SOLVE the transformed line is divided by sigma_p plus the
// sine eigenvalues and transformed again (the last axis of the spatial solve).
template <typename R, int LOGP, int B, int NT, bool SOLVE>
__global__ __launch_bounds__(NT) void k_dst_blue(SpaceArgs a, int axis, long long nlines) {
    using T = cx<R>;
    constexpr int P = 1 << LOGP;
    constexpr int MAXPER = ((P / 4) * B + NT - 1) / NT;   // m < P/4 values per line
    __shared__ T sm[P * B];
    const int m = axis == 0 ? a.mx : (axis == 1 ? a.my : a.mz);
    const int L = 2 * (m + 1);
    const long long stride = axis == 0 ? 1 : (axis == 1 ? (long long)a.mxp : (long long)a.mxp * a.my);
    const T* cw = reinterpret_cast<const T*>(a.chirp[axis]);
    const T* bh = reinterpret_cast<const T*>(a.bh[axis]);
    const T* tw = reinterpret_cast<const T*>(a.twP[axis]);
    T* S = reinterpret_cast<T*>(a.S);
    const T zero = mk<T>((R)0, (R)0);
    // line l: offset of its first element, frequency p and the other two grid
    // indices (axis 0: y, z; axis 1: x, z; axis 2: x, y)
    struct Line {
        long long off;
        int p, i1, i2;
    };
    auto line = [&](long long l) {
        Line r;
        if (axis == 0) {
            const long long lpp = (long long)a.my * a.mz;
            const long long q = l % lpp;
            r.p = (int)(l / lpp);
            r.i1 = (int)(q % a.my);
            r.i2 = (int)(q / a.my);
            r.off = (long long)r.p * a.ldS + q * a.mxp;
        } else {
            const long long q = l / a.mx;
            const int o = axis == 1 ? a.mz : a.my;
            r.i1 = (int)(l % a.mx);
            r.i2 = (int)(q % o);
            r.p = (int)(q / o);
            r.off = (long long)r.p * a.ldS + r.i1 +
                    (axis == 1 ? (long long)r.i2 * a.mxp * a.my : (long long)r.i2 * a.mxp);
        }
        return r;
    };
    T val[MAXPER];
    // a = chirped odd extension of val (element i of this lane is (b, j) =
    // (idx / m, idx % m), idx = tid + i NT, i.e. v_{j+1} of line b), zero elsewhere
    auto build = [&]() {
#pragma unroll
        for (int i = 0; i < MAXPER; ++i) {
            const int idx = threadIdx.x + i * NT;
            if (idx < m * B) {
                const int b = idx / m, j = idx % m;
                const T v = val[i];
                sm[(j + 1) * B + b] = cmul(v, cw[j + 1]);
                const T u = cmul(v, cw[L - 1 - j]);
                sm[(L - 1 - j) * B + b] = mk<T>(-u.x, -u.y);
            }
        }
        for (int idx = threadIdx.x; idx < (2 + P - L) * B; idx += NT) {
            const int r = idx / B, b = idx % B;
            const int t = r == 0 ? 0 : (r == 1 ? m + 1 : L + r - 2);
            sm[t * B + b] = zero;
        }
        __syncthreads();
    };
    // FFT, multiply by Bh, inverse FFT; afterwards Y_k = c_k sm[k B + b]
    auto convolve = [&]() {
        lds_fft<R, LOGP, B, NT, false, true, 0>(sm, tw);
        for (int idx = threadIdx.x; idx < P * B; idx += NT) sm[idx] = cmul(sm[idx], bh[idx / B]);
        __syncthreads();
        lds_fft<R, LOGP, B, NT, true, true, 0>(sm, tw);
    };
    for (long long g = blockIdx.x; g * B < nlines; g += gridDim.x) {
#pragma unroll
        for (int i = 0; i < MAXPER; ++i) {
            const int idx = threadIdx.x + i * NT;
            val[i] = zero;
            if (idx < m * B) {
                const long long l = g * B + idx / m;
                if (l < nlines) val[i] = S[line(l).off + (long long)(idx % m) * stride];
            }
        }
        build();
        convolve();
        if constexpr (SOLVE) {
#pragma unroll
            for (int i = 0; i < MAXPER; ++i) {
                const int idx = threadIdx.x + i * NT;
                if (idx < m * B) {
                    const int b = idx / m, k = idx % m + 1;
                    const long long l = g * B + b;
                    const Line ln = line(l < nlines ? l : 0);
                    const double2 sg = a.sigma[ln.p];
                    double dre = sg.x + (axis == 0 ? a.mu[0] : (axis == 1 ? a.mu[1] : a.mu[2]))[k - 1];
                    if (axis >= 1) dre += a.mu[0][ln.i1];
                    if (axis == 2) dre += a.mu[1][ln.i2];
                    const double inv = a.inv_factor / (dre * dre + sg.y * sg.y);
                    const T c = mk<T>((R)(dre * inv), (R)(-sg.y * inv));
                    val[i] = cmul(cmul(sm[k * B + b], cw[k]), c);
                }
            }
            __syncthreads();
            build();
            convolve();
        }
#pragma unroll
        for (int i = 0; i < MAXPER; ++i) {
            const int idx = threadIdx.x + i * NT;
            if (idx < m * B) {
                const int b = idx / m, k = idx % m + 1;
                const long long l = g * B + b;
                if (l < nlines) S[line(l).off + (long long)(k - 1) * stride] = cmul(sm[k * B + b], cw[k]);
            }
        }
        __syncthreads();
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
// The forward kernel stages the FP64 U tile (N x W doubles) in LDS.
#ifndef PINT_TIME_TILE_BYTES
#define PINT_TIME_TILE_BYTES 65536
#endif
template <typename R> constexpr int time_tile(int logn) {
    const int w = PINT_TIME_TILE_BYTES / ((1 << logn) * 8);
    return w > 64 ? 64 : (w < 2 ? 2 : w);
}
// The forward kernel's LDS holds the FP64 U tile, later reused as the FFT buffer.
#ifndef PINT_FWD_TILE_BYTES
#define PINT_FWD_TILE_BYTES 32768
#endif
constexpr int fwd_tile(int logn) {
    const int w = PINT_FWD_TILE_BYTES / ((1 << logn) * 8);
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
#ifndef PINT_INV_NT
#define PINT_INV_NT 512
#endif

// Workgroups that fit on the whole device at once for a kernel (persistent
// launches), cached per kernel and lane count: the runtime is asked once, and
// never again for a kernel that has been prepared, so a sweep recorded into a
// graph makes no such query while its stream is capturing.
int persistent_blocks(const void* fn, int nt) {
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, int> cache;
    static int cus = 0;
    std::lock_guard<std::mutex> lock(mu);
    const auto it = cache.find({fn, nt});
    if (it != cache.end()) return it->second;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, nt, 0) != hipSuccess || per <= 0) per = 1;
    cache[{fn, nt}] = cus * per;
    return cus * per;
}

// Prepare-only mode (per host thread): the launchers make every runtime query
// and attribute setting of a launch but launch nothing.  A batch runs one
// prepared sweep of its instances before recording the sweep into a graph.
thread_local bool g_prepare_only = false;
#define PINT_LAUNCH(...)                                        \
    do {                                                        \
        if (!g_prepare_only) hipLaunchKernelGGL(__VA_ARGS__);   \
    } while (0)
#define N_OF(logn) (1 << (logn))
// Lanes of the CQ forward kernel (512: the register budget of two waves per SIMD
// holds a radix-16 FP64 butterfly beside the per-element partial sums).
#ifndef PINT_CQ_NT
#define PINT_CQ_NT 512
#endif
constexpr int cq_nt(int logn) {
    const int e = (1 << logn) * cq_tile(logn);
    return e < PINT_CQ_NT ? e : PINT_CQ_NT;
}

// Marching forward launch: one workgroup per (x tile, line, chunk of the
// outer axis), with the chunk length chosen so that the grid fills the device once.
template <typename R, int LOGN, int W, int NT, bool WIDE, bool TAB = true>
hipError_t fwd_march(const FwdArgs& a, int* nb, hipStream_t st) {
    const bool is3 = a.mz > 1;
    auto kern = [](bool three) {
        if constexpr (WIDE && LOGN <= 8)
            return three ? &k_fwd_wide<R, LOGN, W, NT, true, TAB> : &k_fwd_wide<R, LOGN, W, NT, false, TAB>;
        else if constexpr (WIDE)   // the 3D wide tile is used up to N = 256 only
            return (void)three, &k_fwd_wide<R, LOGN, W, NT, false, TAB>;
        else return three ? &k_fwd_march<R, LOGN, W, NT, true> : &k_fwd_march<R, LOGN, W, NT, false>;
    };
    if constexpr (WIDE && LOGN > 8)
        if (is3) return hipErrorInvalidValue;   // never chosen (fwd_kind)
    const void* fn = reinterpret_cast<const void*>(kern(is3));
    const int ncol = (a.mxp / W) * (is3 ? a.my : 1);
    const int nm = is3 ? a.mz : a.my;
    const int target = persistent_blocks(fn, NT);
    int nchunk = std::max(1, std::min(nm, (target + ncol - 1) / ncol));
    const int chunk = (nm + nchunk - 1) / nchunk;
    nchunk = (nm + chunk - 1) / chunk;
    const int grid = ((ncol * nchunk + 7) / 8) * 8;
    if (nb) *nb = grid;
    PINT_LAUNCH(kern(is3), dim3(grid), dim3(NT), 0, st, a, ncol, nchunk, chunk);
    return hipGetLastError();
}

// Which forward kernel a variant launches for this problem:
//   BDF-k: 0 wide-tile march (kind 0 in 2D, 3 in 3D), 1 march with the
//   time-FFT tile, 2 one workgroup per tile, 3 half-width wide-tile march with
//   two workgroups per CU (kind 4);
//   CQ: 0 y-march (radix <= 8), 1 y-march (radix <= 16), 2 persistent one-tile kernel.
// A variant whose kernel does not apply falls back to the next one that does.
template <typename R, int LOGN>
int fwd_kind(const FwdArgs& a, bool cq) {
    const int var = a.var < 0 || a.var >= kFwdVariants ? 0 : a.var;
    if (cq) {
        constexpr int WM = cqm_tile(LOGN);
        if constexpr (cqm_lds<R, LOGN, WM>() <= 163840 && N_OF(LOGN) * WM >= 2 * PINT_CQ_NT) {
            // 2D residual form: march along y (32-bit lane offsets, whole tiles per grid row)
            if (var < 2 && a.form == 0 && a.my > 1 && a.mz == 1 && a.mxp % WM == 0 &&
                (long long)(PINT_CQ_NT / WM + 2) * a.M * 8 < (1LL << 32))
                return var;
        }
        return 2;
    }
    if (a.form != 0 || a.my == 1 || var == 2) return 2;
    constexpr int W = fwd_tile(LOGN);
    constexpr int NT = (N_OF(LOGN) * W >= kNT) ? kNT : 64;
    constexpr int NTM = (N_OF(LOGN) * W >= PINT_MARCH_NT) ? PINT_MARCH_NT : NT;
    constexpr int WW = 16;
    constexpr int NTW = N_OF(LOGN) * WW < 512 ? N_OF(LOGN) * WW : 512;
    constexpr bool WIDE_OK = LOGN <= 9 && PINT_FWD_WIDE;
    // the marching kernels address with 32-bit byte offsets per lane
    // (3D: up to N = 256, where the wide tile's eight rows per lane leave room
    // for the y-neighbour loads without spilling)
    const bool wide_ok = WIDE_OK && (a.mz == 1 || LOGN <= 8) && WW <= a.mxp &&
                         (long long)(NTW / WW + 2) * a.M * 8 < (1LL << 32);
    if (var == 0 && wide_ok) return a.mz == 1 ? 0 : 3;
    // half-width wide tiles, two workgroups per CU
    if (var == 3 && WIDE_OK && (a.mz == 1 || LOGN <= 8) && N_OF(LOGN) * 8 >= 2 * 256 && 8 <= a.mxp &&
        (256 / 8 + 2) * (long long)a.M * 8 < (1LL << 32))
        return 4;
    if (W <= a.mxp && a.mxp % W == 0 && (long long)(NTM / W + 2) * a.M * 8 < (1LL << 32)) return 1;
    return 2;
}

template <typename R, int LOGN, int MAXLOG>
hipError_t fwd_cqm_launch(const FwdArgs& a, int* nb, hipStream_t st) {
    constexpr int WM = cqm_tile(LOGN);
    constexpr int NTM = PINT_CQ_NT;
    if constexpr (cqm_lds<R, LOGN, WM>() <= 163840 && N_OF(LOGN) * WM >= 2 * PINT_CQ_NT) {
        const void* fn = reinterpret_cast<const void*>(&k_fwd_cqm<R, LOGN, WM, NTM, MAXLOG>);
        const int ncol = a.mxp / WM;
        const int target = persistent_blocks(fn, NTM);
        int nchunk = std::max(1, std::min(a.my, (target + ncol - 1) / ncol));
        const int chunk = (a.my + nchunk - 1) / nchunk;
        nchunk = (a.my + chunk - 1) / chunk;
        const int grid = ((ncol * nchunk + 7) / 8) * 8;
        if (nb) *nb = grid;
        PINT_LAUNCH((k_fwd_cqm<R, LOGN, WM, NTM, MAXLOG>), dim3(grid), dim3(NTM), 0, st, a, ncol, nchunk, chunk);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

template <typename R, int LOGN>
hipError_t fwd_one(const FwdArgs& a, bool cq, int* nb, hipStream_t st) {
    const int kind = fwd_kind<R, LOGN>(a, cq);
    if (cq) {
        if (kind == 0) return fwd_cqm_launch<R, LOGN, 3>(a, nb, st);
        if (kind == 1) return fwd_cqm_launch<R, LOGN, 4>(a, nb, st);
        constexpr int W = cq_tile(LOGN);
        constexpr int NT = cq_nt(LOGN);
        // per-lane byte offsets of the kernel's buffer loads are 32-bit
        if ((long long)(64 / W + 1) * a.M * 8 >= (1LL << 32)) return hipErrorInvalidValue;
        const int ntiles = (a.Mp + W - 1) / W;
        const int nvirt = ((ntiles + 7) / 8) * 8;
        const void* fn = reinterpret_cast<const void*>(&k_fwd_cq<R, LOGN, W, NT>);
        // a multiple of 8 workgroups, so workgroup b stays on XCD b mod 8 for all its tiles
        const int grid = std::min(nvirt, std::max(8, persistent_blocks(fn, NT) / 8 * 8));
        if (nb) *nb = grid;
        PINT_LAUNCH((k_fwd_cq<R, LOGN, W, NT>), dim3(grid), dim3(NT), 0, st, a, nvirt);
        return hipGetLastError();
    }
    constexpr int W = fwd_tile(LOGN);
    constexpr int NT = (N_OF(LOGN) * W >= kNT) ? kNT : 64;
    constexpr int NTM = (N_OF(LOGN) * W >= PINT_MARCH_NT) ? PINT_MARCH_NT : NT;
    constexpr int WW = 16;
    constexpr int NTW = N_OF(LOGN) * WW < 512 ? N_OF(LOGN) * WW : 512;
    if (kind == 0 || kind == 3) {
        if constexpr (LOGN <= 9 && PINT_FWD_WIDE) return fwd_march<R, LOGN, WW, NTW, true>(a, nb, st);
        return hipErrorInvalidValue;
    }
    if (kind == 4) {
        if constexpr (LOGN <= 9 && LOGN >= 6 && PINT_FWD_WIDE) return fwd_march<R, LOGN, 8, 256, true, false>(a, nb, st);
        return hipErrorInvalidValue;
    }
    if (kind == 1) return fwd_march<R, LOGN, W, NTM, false>(a, nb, st);
    const int ntiles = (a.Mp + W - 1) / W;
    const int grid = ((ntiles + 7) / 8) * 8;
    if (nb) *nb = grid;
    PINT_LAUNCH((k_fwd_heat<R, LOGN, W, NT>), dim3(grid), dim3(NT), 0, st, a);
    return hipGetLastError();
}

template <typename R, int LOGN>
hipError_t inv_one(const InvArgs& a, int* nb, hipStream_t st) {
    constexpr int W = time_tile<R>(LOGN);
    const int ntiles = (a.Mp + W - 1) / W;
    const int grid = ((ntiles + 7) / 8) * 8;
    if (nb) *nb = grid;
    constexpr int NT = (N_OF(LOGN) * W >= PINT_INV_NT) ? PINT_INV_NT : kNT;
    PINT_LAUNCH((k_inv<R, LOGN, W, NT>), dim3(grid), dim3(NT), 0, st, a);
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
    PINT_LAUNCH((k_tri1d<R, EPT, NT>), dim3(a.nP), dim3(NT), lds, st, a);
    return hipGetLastError();
}

// Split of a 1D system of size m between PCR (NT lanes) and Thomas (EPT
// equations per lane): the built-in choice, and with var_tri = 1 one with
// more PCR lanes (fewer Thomas equations), where that differs.
template <typename R>
hipError_t tri1d_dispatch(const SpaceArgs& a, hipStream_t st) {
    const int m = a.mx;
    const bool alt = a.var_tri == 1;
    if (m <= 64) return tri1d_one<R, 1, 64>(a, st);
    if (m <= 128) return alt ? tri1d_one<R, 1, 128>(a, st) : tri1d_one<R, 2, 64>(a, st);
    if (m <= 256) return alt ? tri1d_one<R, 1, 256>(a, st) : tri1d_one<R, 4, 64>(a, st);
    if (m <= 512) return alt ? tri1d_one<R, 2, 256>(a, st) : tri1d_one<R, 8, 64>(a, st);
    if (m <= 1024) return alt ? tri1d_one<R, 2, 512>(a, st) : tri1d_one<R, 4, 256>(a, st);
    if (m <= 2048) return alt ? tri1d_one<R, 4, 512>(a, st) : tri1d_one<R, 8, 256>(a, st);
    return hipErrorInvalidValue;
}

#ifndef PINT_ROWS_FUSED
#define PINT_ROWS_FUSED 1
#endif
// Whether the x pass without the divide takes the folded kernel: lengths with a
// folded radix schedule, one butterfly for each of the 256 lanes (two of radix 8);
// with fewer butterflies than lanes the compiler's register use doubles.
constexpr bool rows_fused_ok(int logl, int rows) {
    return PINT_ROWS_FUSED && fused_r0(logl) != 0 && rows * ((1 << logl) / fused_r0(logl)) >= 256 &&
           rows * ((1 << logl) / fused_r0(logl)) <= (fused_r0(logl) == 16 ? 256 : 512);
}
// Rows per workgroup of the x pass: the LDS-sized count, lowered for the
// transform-only pass until the folded kernel takes it (faster than the plain
// kernel with twice the rows on every measured grid).
template <typename R, bool SOLVE> constexpr int rows_default(int logl) {
    const int r = rows_per_block<R>(logl);
    if (SOLVE || fused_r0(logl) == 0) return r;
    for (int c = r; c >= 1; c /= 2)
        if (rows_fused_ok(logl, c)) return c;
    return r;
}
// The built-in count, or half of it (var_rows = 1).
template <typename R, bool SOLVE> constexpr int rows_alt(int logl) {
    const int r = rows_default<R, SOLVE>(logl);
    return r >= 2 ? r / 2 : r;
}
#ifndef PINT_COLS_FUSED
#define PINT_COLS_FUSED 1
#endif
// Butterflies per workgroup in the first stage of the folded y/z kernel (Q W), and
// whether that kernel takes W columns of length 2^logl: at most 512 lanes with one
// butterfly each, or two of radix 8 (more spill registers).
constexpr int fused_tasks(int logl, int w) { return fused_r0(logl) ? ((1 << logl) / fused_r0(logl)) * w : 0; }
constexpr bool fused_ok(int logl, int w) {
    return PINT_COLS_FUSED && fused_r0(logl) != 0 && fused_tasks(logl, w) >= 64 &&
           fused_tasks(logl, w) <= (fused_r0(logl) == 16 ? 512 : 1024);
}
// Columns per workgroup of the y/z pass.  With the folded kernel: 16 columns for
// the solve pass (256-byte FP64 / 128-byte FP32 row segments) and 32 for the
// transform-only pass, or half that, when the tile fits 128 KB of LDS (the
// fastest measured on the 2D and 3D workloads); otherwise the LDS-sized width.
template <typename R, bool SOLVE> constexpr int cols_default(int logl) {
    const int c0 = SOLVE ? 16 : 32;
    for (int c = c0; c >= c0 / 2; c /= 2)
        if ((1 << logl) * c * (int)sizeof(cx<R>) <= 131072 && fused_ok(logl, c)) return c;
    return cols_per_block<R>(logl);
}
// The other width (var_cols = 1): twice the built-in one when the tile still
// fits 128 KB of LDS and 32 columns, else half.
template <typename R, bool SOLVE> constexpr int cols_alt(int logl) {
    const int w = cols_default<R, SOLVE>(logl);
    if (2 * w <= 32 && (1 << logl) * 2 * w * (int)sizeof(cx<R>) <= 131072) return 2 * w;
    return w >= 2 ? w / 2 : w;
}

template <typename R, int LOGL, int ROWS, bool SOLVE>
hipError_t rows_run(const SpaceArgs& a, hipStream_t st) {
    constexpr int NT = kNT;
    const long long nlines = (long long)a.nP * a.my * a.mz;
    const long long groups = (nlines + ROWS - 1) / ROWS;
    auto kern = []() {
        if constexpr (!SOLVE && rows_fused_ok(LOGL, ROWS)) return &k_dst_rowsf<R, LOGL, ROWS, NT>;
        else return &k_dst_rows<R, LOGL, ROWS, NT, SOLVE>;
    };
    const long long grid =
        std::min<long long>(groups, persistent_blocks(reinterpret_cast<const void*>(kern()), NT));
    PINT_LAUNCH(kern(), dim3((unsigned)grid), dim3(NT), 0, st, a, nlines);
    return hipGetLastError();
}


template <typename R, int LOGL, int W, bool SOLVE>
hipError_t cols_run(const SpaceArgs& a, int axis, hipStream_t st) {
    // tiles above 64 KB of LDS get 512 lanes so the FFT stages stay in registers
    // (FP64 tiles of 64 KB as well: measured faster with 8 waves per workgroup)
    // the folded kernel (lengths it covers) runs min(Q W, 512) lanes
    constexpr bool FUSED = fused_ok(LOGL, W);
    constexpr int NT = FUSED ? (fused_tasks(LOGL, W) > 512 ? 512 : fused_tasks(LOGL, W))
                             : (((1 << LOGL) * W * (int)sizeof(cx<R>) > 65536 || sizeof(R) == 8) ? 512 : kNT);
    const int other = axis == 1 ? a.mz : a.my;
    const long long groups = (long long)a.nP * other * ((a.mx + W - 1) / W);
    auto kern = []() {
        if constexpr (FUSED) return &k_dst_colsf<R, LOGL, W, NT, SOLVE>;
        else return &k_dst_cols<R, LOGL, W, NT, SOLVE>;
    };
    const long long grid =
        std::min<long long>(groups, persistent_blocks(reinterpret_cast<const void*>(kern()), NT));
    PINT_LAUNCH(kern(), dim3((unsigned)grid), dim3(NT), 0, st, a, axis);
    return hipGetLastError();
}

template <typename R, int LOGL, bool SOLVE>
hipError_t rows_one(const SpaceArgs& a, hipStream_t st) {
    if (a.var_rows == 1 && rows_alt<R, SOLVE>(LOGL) != rows_default<R, SOLVE>(LOGL))
        return rows_run<R, LOGL, rows_alt<R, SOLVE>(LOGL), SOLVE>(a, st);
    return rows_run<R, LOGL, rows_default<R, SOLVE>(LOGL), SOLVE>(a, st);
}

template <typename R, int LOGL, bool SOLVE>
hipError_t cols_one(const SpaceArgs& a, int axis, hipStream_t st) {
    if (a.var_cols == 1 && cols_alt<R, SOLVE>(LOGL) != cols_default<R, SOLVE>(LOGL))
        return cols_run<R, LOGL, cols_alt<R, SOLVE>(LOGL), SOLVE>(a, axis, st);
    return cols_run<R, LOGL, cols_default<R, SOLVE>(LOGL), SOLVE>(a, axis, st);
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

template <typename R, int LOGP, bool SOLVE>
hipError_t blue_one(const SpaceArgs& a, int axis, hipStream_t st) {
    constexpr int P = 1 << LOGP;
    constexpr int BQ = 65536 / (P * (int)sizeof(cx<R>));
    constexpr int B = BQ > 16 ? 16 : (BQ < 1 ? 1 : BQ);
    constexpr int NT = kNT;
    const long long other = axis == 0 ? (long long)a.my * a.mz : (long long)a.mx * (axis == 1 ? a.mz : a.my);
    const long long nlines = (long long)a.nP * other;
    const long long groups = (nlines + B - 1) / B;
    const long long grid = std::min<long long>(
        groups, persistent_blocks(reinterpret_cast<const void*>(&k_dst_blue<R, LOGP, B, NT, SOLVE>), NT));
    PINT_LAUNCH((k_dst_blue<R, LOGP, B, NT, SOLVE>), dim3((unsigned)grid), dim3(NT), 0, st, a, axis, nlines);
    return hipGetLastError();
}

template <typename R, bool SOLVE>
hipError_t blue_dispatch(const SpaceArgs& a, int axis, hipStream_t st) {
    switch (a.logP[axis]) {
        case 4: return blue_one<R, 4, SOLVE>(a, axis, st);
        case 5: return blue_one<R, 5, SOLVE>(a, axis, st);
        case 6: return blue_one<R, 6, SOLVE>(a, axis, st);
        case 7: return blue_one<R, 7, SOLVE>(a, axis, st);
        case 8: return blue_one<R, 8, SOLVE>(a, axis, st);
        case 9: return blue_one<R, 9, SOLVE>(a, axis, st);
        case 10: return blue_one<R, 10, SOLVE>(a, axis, st);
        case 11: return blue_one<R, 11, SOLVE>(a, axis, st);
        case 12: return blue_one<R, 12, SOLVE>(a, axis, st);
        case 13: return blue_one<R, 13, SOLVE>(a, axis, st);
        default: return hipErrorInvalidValue;
    }
}

// One spatial pass of a 2D/3D solve along `axis`: the power-of-two kernels
// when 2(m+1) is a power of two, Bluestein otherwise.
template <typename R, bool SOLVE>
hipError_t axis_pass(const SpaceArgs& a, int axis, hipStream_t st) {
    if (a.logP[axis] != 0) return blue_dispatch<R, SOLVE>(a, axis, st);
    if (axis == 0) return rows_dispatch<R, SOLVE>(a, st);
    return cols_dispatch<R, SOLVE>(a, axis, st);
}

template <typename R>
hipError_t space_pass(const SpaceArgs& a, int i, hipStream_t st) {
    if (a.dim == 1) return dst1d(a) ? rows_dispatch<R, true>(a, st) : tri1d_dispatch<R>(a, st);
    if (a.dim == 2) return i == 1 ? axis_pass<R, true>(a, 1, st) : axis_pass<R, false>(a, 0, st);
    switch (i) {
        case 1: case 3: return axis_pass<R, false>(a, 1, st);
        case 2: return axis_pass<R, true>(a, 2, st);
        default: return axis_pass<R, false>(a, 0, st);
    }
}

}  // namespace

hipError_t launch_prep(const double* v, const double* f, const double* fder, double* corr, const double* a_n,
                       const double* b_lt, int k, int M, int mx, int my, int mz, double ihx2, double ihy2,
                       double ihz2, hipStream_t st) {
    if (k < 2) return hipSuccess;
    PINT_LAUNCH(k_prep, dim3((M + 255) / 256), dim3(256), 0, st, v, f, fder, corr, a_n, b_lt, k, M, mx, my, mz,
                       ihx2, ihy2, ihz2);
    return hipGetLastError();
}

hipError_t launch_fill(double* U, const double* v, long long N, int M, int zero, hipStream_t st) {
    const long long total = N * M;
    PINT_LAUNCH(k_fill, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, U, v, total, M, zero);
    return hipGetLastError();
}

hipError_t launch_forward(const FwdArgs& a, bool mixed, bool cq, int* nb, hipStream_t st) {
    return mixed ? fwd_dispatch<float>(a, cq, nb, st) : fwd_dispatch<double>(a, cq, nb, st);
}

hipError_t launch_inject(const FwdArgs& a, const void* Sg, bool mixed, hipStream_t st) {
    const int pchunk = 16;
    const dim3 grid((unsigned)((a.Mp + 255) / 256), (unsigned)((a.N / 2 + 1 + pchunk - 1) / pchunk));
    if (mixed)
        PINT_LAUNCH(k_inject<float>, grid, dim3(256), 0, st, a, Sg, pchunk);
    else
        PINT_LAUNCH(k_inject<double>, grid, dim3(256), 0, st, a, Sg, pchunk);
    return hipGetLastError();
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

void set_prepare_only(bool on) { g_prepare_only = on; }

hipError_t launch_norm_reduce(const double* partial, int nb, double hd, double* out, hipStream_t st) {
    PINT_LAUNCH(k_norm_reduce, dim3(1), dim3(kNormNT), 0, st, partial, nb, hd, out);
    return hipGetLastError();
}

namespace {
template <typename R>
int fwd_kind_of(const FwdArgs& a, bool cq) {
    switch (__builtin_ctz((unsigned)a.N)) {
        case 3: return fwd_kind<R, 3>(a, cq);
        case 4: return fwd_kind<R, 4>(a, cq);
        case 5: return fwd_kind<R, 5>(a, cq);
        case 6: return fwd_kind<R, 6>(a, cq);
        case 7: return fwd_kind<R, 7>(a, cq);
        case 8: return fwd_kind<R, 8>(a, cq);
        case 9: return fwd_kind<R, 9>(a, cq);
        case 10: return fwd_kind<R, 10>(a, cq);
        case 11: return fwd_kind<R, 11>(a, cq);
        default: return -1;
    }
}
template <typename R>
bool rows_distinct(int logl, bool solve) {
    if (logl < kMinLogL || logl > kMaxLogL) return false;
    return solve ? rows_alt<R, true>(logl) != rows_default<R, true>(logl)
                 : rows_alt<R, false>(logl) != rows_default<R, false>(logl);
}
template <typename R>
bool cols_distinct(int logl, bool solve) {
    if (logl < kMinLogL || logl > kMaxLogL) return false;
    return solve ? cols_alt<R, true>(logl) != cols_default<R, true>(logl)
                 : cols_alt<R, false>(logl) != cols_default<R, false>(logl);
}
int log2_of_pow2(unsigned v) { return (v & (v - 1)) == 0 ? __builtin_ctz(v) : -1; }
}  // namespace

bool forward_variant_distinct(const FwdArgs& a, bool mixed, bool cq, int var) {
    FwdArgs b = a, c = a;
    b.var = 0;
    c.var = var;
    return mixed ? fwd_kind_of<float>(b, cq) != fwd_kind_of<float>(c, cq)
                 : fwd_kind_of<double>(b, cq) != fwd_kind_of<double>(c, cq);
}

bool rows_variant_distinct(const SpaceArgs& a, bool mixed) {
    const bool has_rows = a.dim == 1 ? dst1d(a) : a.logP[0] == 0;
    if (!has_rows) return false;
    const int logl = log2_of_pow2(2u * (unsigned)(a.mx + 1));
    const bool solve = a.dim == 1;   // the 1D pass carries the divide
    return mixed ? rows_distinct<float>(logl, solve) : rows_distinct<double>(logl, solve);
}

bool cols_variant_distinct(const SpaceArgs& a, bool mixed) {
    for (int axis = 1; axis < a.dim; ++axis) {
        if (a.logP[axis] != 0) continue;
        const int m = axis == 1 ? a.my : a.mz;
        const int logl = log2_of_pow2(2u * (unsigned)(m + 1));
        const bool solve = axis == a.dim - 1;   // the last axis carries the divide
        if (mixed ? cols_distinct<float>(logl, solve) : cols_distinct<double>(logl, solve)) return true;
    }
    return false;
}

bool tri_variant_distinct(const SpaceArgs& a) { return a.dim == 1 && !dst1d(a) && a.mx > 64 && a.mx <= kMaxTri1D; }

}  // namespace pint
