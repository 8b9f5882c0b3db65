// Device-side building blocks shared by the gfx950 kernel translation units
// (pint_forward.hip, pint_space.hip, pint_time.hip): complex helpers, raw
// buffer access, the in-LDS Stockham FFT, XCD-aware tile order, spectrum
// layout helpers, tile widths and the launch macro.  Not part of the ABI.
#pragma once

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


}  // namespace

// Workgroups that fit on the whole device at once for a kernel (cached).
int persistent_blocks(const void* fn, int nt);

}  // namespace pint

#define PINT_LAUNCH(...) hipLaunchKernelGGL(__VA_ARGS__)
#define N_OF(logn) (1 << (logn))
