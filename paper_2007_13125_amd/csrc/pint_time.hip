// gfx950 kernels of one diagonalized waveform-relaxation sweep: the inverse kernel, norm reduction, setup kernels
#include "pint_device.h"

namespace pint {
namespace {

#ifndef PINT_INV_WAVES
#define PINT_INV_WAVES 1
#endif

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

template <typename R, int LOGN>
hipError_t inv_one(const InvArgs& a, int* nb, hipStream_t st) {
    constexpr int W = time_tile<R>(LOGN);
    const int ntiles = (a.Mp + W - 1) / W;
    if constexpr (W >= 8) {
        // small grids: tiles of W/4 slots (4 times as many workgroups)
        constexpr int WS = W / 4;
        constexpr int E = N_OF(LOGN) * WS;
        constexpr int NTS = E >= PINT_INV_NT ? PINT_INV_NT : (E >= kNT ? kNT : 64);
        if (ntiles < 32) {
            const int grid = (((a.Mp + WS - 1) / WS + 7) / 8) * 8;
            if (nb) *nb = grid;
            PINT_LAUNCH((k_inv<R, LOGN, WS, NTS>), dim3(grid), dim3(NTS), 0, st, a);
            return hipGetLastError();
        }
    }
    const int grid = ((ntiles + 7) / 8) * 8;
    if (nb) *nb = grid;
    constexpr int NT = (N_OF(LOGN) * W >= PINT_INV_NT) ? PINT_INV_NT : kNT;
    PINT_LAUNCH((k_inv<R, LOGN, W, NT>), dim3(grid), dim3(NT), 0, st, a);
    return hipGetLastError();
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

}  // namespace

// Workgroups that fit on the whole device at once for a kernel (persistent
// launches), cached per kernel and lane count: the runtime is asked once.
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

hipError_t launch_inverse(const InvArgs& a, bool mixed, int* nb, hipStream_t st) {
    return mixed ? inv_dispatch<float>(a, nb, st) : inv_dispatch<double>(a, nb, st);
}

hipError_t launch_norm_reduce(const double* partial, int nb, double hd, double* out, hipStream_t st) {
    PINT_LAUNCH(k_norm_reduce, dim3(1), dim3(kNormNT), 0, st, partial, nb, hd, out);
    return hipGetLastError();
}

}  // namespace pint

