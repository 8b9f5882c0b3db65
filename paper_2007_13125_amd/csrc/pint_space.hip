// gfx950 kernels of one diagonalized waveform-relaxation sweep: the spatial shifted solves
#include "pint_device.h"

namespace pint {
namespace {

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
            eb[e] = a.dvar ? mk<T>((R)(sg.x + 2.0 * a.ih2[0] + a.dvar[i]), (R)sg.y) : diag;
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
// (sigma_p + mu_x) times the raw-transform factor (sigma_p mass_x + mu_x for P1
// elements) and transformed back.
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
                // P1 elements (1D): sigma_p mass_t + mu_t
                const double mm = a.mass ? a.mass[t - 1] : 1.0;
                const double dre = sg.x * mm + a.mu[0][t - 1], dim = sg.y * mm;
                const double inv = a.inv_factor / (dre * dre + dim * dim);
                const T c = mk<T>((R)(dre * inv), (R)(-dim * inv));
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
                    // P1 elements (1D): sigma_p mass_k + mu_k
                    const double mm = a.mass ? a.mass[k - 1] : 1.0;
                    double dre = sg.x * mm + (axis == 0 ? a.mu[0] : (axis == 1 ? a.mu[1] : a.mu[2]))[k - 1];
                    if (axis >= 1) dre += a.mu[0][ln.i1];
                    if (axis == 2) dre += a.mu[1][ln.i2];
                    const double dim = sg.y * mm;
                    const double inv = a.inv_factor / (dre * dre + dim * dim);
                    const T c = mk<T>((R)(dre * inv), (R)(-dim * inv));
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
// equations per lane): var_tri = 1 the built-in split, var_tri = 2 one with
// more PCR lanes (fewer Thomas equations), where that differs.
template <typename R>
hipError_t tri1d_dispatch(const SpaceArgs& a, hipStream_t st) {
    const int m = a.mx;
    const bool alt = a.var_tri == 2;
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
    constexpr int RD = rows_default<R, SOLVE>(LOGL);
    if constexpr (RD >= 8) {
        // small grids (fewer than 32 row groups): groups of RD/8 rows, so the lines
        // spread over 8 times as many workgroups
        const long long nlines = (long long)a.nP * a.my * a.mz;
        if (a.var_rows == 0 && (nlines + RD - 1) / RD < 32) return rows_run<R, LOGL, RD / 8, SOLVE>(a, st);
    }
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
//   1D: one pass: sine transform + divide + inverse (Bluestein when 2(m+1) is
//       not a power of two), or, when pinned (var_tri >= 1), PCR/Thomas;
//   2D: DST-x rows, DST-y + divide + inverse DST-y, DST-x rows;
//   3D: DST-x, DST-y, DST-z + divide + inverse, DST-y, DST-x.
int pass_count(const SpaceArgs& a) { return a.dim == 1 ? 1 : (a.dim == 2 ? 3 : 5); }

// 1D: the power-of-two sine solve (for P1 elements its divide carries the mass
// eigenvalues).
bool dst1d(const SpaceArgs& a) {
    const unsigned L = 2u * (unsigned)(a.mx + 1);
    return (L & (L - 1)) == 0 && L <= (1u << kMaxLogL);
}

bool tri1d(const SpaceArgs& a) {
    return a.dim == 1 && !a.mass && (a.dvar || (!dst1d(a) && a.var_tri >= 1));
}

const char* pass_name(const SpaceArgs& a, int i) {
    if (a.dim == 1) return tri1d(a) ? "tridiag_pcr_thomas" : "dst_x_solve";
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
    if (a.dim == 1) {
        if (tri1d(a)) return tri1d_dispatch<R>(a, st);
        return dst1d(a) ? rows_dispatch<R, true>(a, st) : blue_dispatch<R, true>(a, 0, st);
    }
    if (a.dim == 2) return i == 1 ? axis_pass<R, true>(a, 1, st) : axis_pass<R, false>(a, 0, st);
    switch (i) {
        case 1: case 3: return axis_pass<R, false>(a, 1, st);
        case 2: return axis_pass<R, true>(a, 2, st);
        default: return axis_pass<R, false>(a, 0, st);
    }
}

}  // namespace

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

namespace {
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

}  // namespace pint

