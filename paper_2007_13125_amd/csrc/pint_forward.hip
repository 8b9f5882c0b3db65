// gfx950 kernels of one diagonalized waveform-relaxation sweep: the forward kernels
#include "pint_device.h"

namespace pint {
namespace {

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
    // x tiles fastest: an XCD's resident workgroups hold whole grid rows of a few
    // consecutive lines, so the x halos and most y-neighbour lines are loaded by
    // workgroups of the same XCD at the same time (its L2 serves them)
    const int xt = col % nxt, yl = col / nxt;
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
// its last k rows).  One lane per spectrum slot and a chunk of frequencies,
// read in batches of 8 so that a lane keeps 8 loads in flight (the next batch
// is issued before the current one is combined and stored).
constexpr int kInjectBatch = 8;
template <typename R>
__global__ __launch_bounds__(256) void k_inject(FwdArgs a, const void* Sg, int pchunk) {
    using T = cx<R>;
    constexpr int PB = kInjectBatch;
    const int P0 = blockIdx.y * pchunk, P1 = min(a.N / 2 + 1, P0 + pchunk);
    const int slot = blockIdx.x * 256 + threadIdx.x;
    if (slot >= a.Mp) return;
    const int d = slot_dof(slot, a.mx, a.mxp, a.Mp);
    // the last k rows of U, then c_n = kappa tau^{-1} kappa^{(n-1)/N} sum_{j=n..k} w_j U^{N+n-j}
    double ul[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) ul[i] = (d >= 0 && i < a.k) ? a.U[(size_t)(a.N - 1 - i) * a.M + d] : 0.0;
    double c[6];
#pragma unroll
    for (int n = 1; n <= 6; ++n) {
        double acc = 0.0;
#pragma unroll
        for (int j = n; j <= 6; ++j)
            if (j <= a.k) acc += a.wk[j] * ul[j - n];   // U^{N+n-j} is row N+n-j-1 = N-1-(j-n)
        c[n - 1] = n <= a.k ? a.kappa * a.ta * acc * a.scale[n - 1] : 0.0;
    }
    const T* src = reinterpret_cast<const T*>(Sg);
    T* dst = reinterpret_cast<T*>(a.S);
    const T* tw = reinterpret_cast<const T*>(a.tw);
    const unsigned so = (unsigned)slot * (unsigned)sizeof(T);   // within one frequency row
    auto load = [&](int p0, T (&g)[PB]) {
#pragma unroll
        for (int i = 0; i < PB; ++i) {
            const int p = p0 + i;   // a row of its own (the spectrum may exceed 4 GB)
            const auto rs = buf_rsrc(src + (size_t)min(p, P1 - 1) * a.ldS, (size_t)a.ldS * sizeof(T));
            g[i] = buf_ld(rs, p < P1 ? so : kNoLane, mk<T>(0, 0));
        }
    };
    T g[PB], gn[PB];
    load(P0, g);
    for (int p0 = P0; p0 < P1; p0 += PB) {
        if (p0 + PB < P1) load(p0 + PB, gn);
#pragma unroll
        for (int i = 0; i < PB; ++i) {
            const int p = p0 + i;
            if (p >= P1) break;
            double hr = (double)g[i].x, hi = (double)g[i].y;
#pragma unroll
            for (int n = 1; n <= 6; ++n) {
                if (n > a.k) break;
                const T w = tw[((n - 1) * p) & (a.N - 1)];
                hr += c[n - 1] * (double)w.x;
                hi += c[n - 1] * (double)w.y;
            }
            dst[(size_t)p * a.ldS + slot] = mk<T>((R)hr, (R)hi);
        }
#pragma unroll
        for (int i = 0; i < PB; ++i) g[i] = gn[i];
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
// Forward pass in two kernels (BDF-k residual form, 2D/3D).
// k_resid: each workgroup owns a block of 64 x slots by 8 x 4 grid lines (3D;
// 64 x 16 lines in 2D) and marches along time, q = 0..N-1, writing the kappa^{q/N}-scaled
// residual
//   r~_q = kappa^{q/N} (f(t_{q+1}) + corrections + tau^{-1} s_q v
//                       - tau^{-1} sum_{j<=min(q,k)} w_j U_{q-j} - A_h U_q)
// to Rb[q][slot] in the spectrum's real type (zero in padding slots).  The
// time stencil's earlier rows stay in registers.  Row q of the block is staged
// in LDS with its halo faces, so every space stencil neighbour is an LDS read:
// the loads per element are U, f (and the correction rows while q < k - 1) plus
// 0.8 halo values in 3D (0.16 in 2D), instead of one per neighbour (the
// kernel is bound by the rate at which the texture addresser takes load
// instructions, and neighbour lines of other workgroups mostly come from HBM).
// The loads of row q+1 are in flight while row q is combined.  Two LDS buffers
// alternate by row, so one barrier per row separates each row's writes from its
// reads.
// k_tfft: the time FFT of Rb, a tile of W slots x N rows in LDS, stored as the
// half spectrum.
constexpr int kBlkX = 64;   // x slots of a block (one wave's lanes)
// Block of a workgroup: 64 x slots by BY grid lines by BZ planes (BY BZ / NW
// lines per lane, NW waves), and the halo values it stages per row: the y and z
// faces (64 values each line) and the x neighbours of its lines.
// 3D: 64 x 8 x 4 points, 512 lanes (measured against 64 x 4 x 4 / 256 lanes, 5%
// slower, 64 x 4 x 8 and 64 x 16 x 2 / 512 lanes, and 64 x 8 x 8 at 512 or 1024
// lanes, which spill); 2D: 64 x 16, 512 lanes (3% faster than 64 x 8 or 64 x 32
// with 512 lanes, 64 x 8 with 256, and 10% faster than 64 x 16 with 256).
template <bool IS3> struct ResidBlock {
    static constexpr int BY = IS3 ? 8 : 16, BZ = IS3 ? 4 : 1;
    static constexpr int NT = 512, NW = NT / 64;   // lanes, waves
    static constexpr int NH = 2 * BZ * kBlkX + (IS3 ? 2 * BY * kBlkX : 0) + 2 * BY * BZ;
    static constexpr int HPL = (NH + NT - 1) / NT;   // halo values per lane
    static constexpr int LZ = IS3 ? BZ + 2 : 1;                  // LDS planes (z halo in 3D)
    static constexpr int LY = BY + 2, LX = kBlkX + 2;
};
// 3D block order: regions of nxb x kRegY x kRegZ blocks (whole x rows, 2 y by 8 z
// blocks: about the workgroups an XCD holds at once) one after another, so the
// y and z halo faces of most blocks are rows that co-resident workgroups of the
// same XCD load, and come from its L2.
constexpr int kRegY = 2, kRegZ = 8;
template <typename RT, bool IS3>
__global__ __launch_bounds__(ResidBlock<IS3>::NT) void k_resid(FwdArgs a, int qc, int nxb, int nyb, int nzb) {
    using BL = ResidBlock<IS3>;
    constexpr int BY = BL::BY, BZ = BL::BZ, LZ = BL::LZ, LY = BL::LY, LX = BL::LX, NW = BL::NW, PT = BY * BZ / NW;
    static_assert(PT * NW == BY * BZ, "whole lines per lane");
    __shared__ double su[2][LZ * LY * LX];   // [buffer][(z + zo) LY + y + 1][x + 1], zo = 1 in 3D
    const int b = xcd_tile(blockIdx.x, gridDim.x);
    int xb, yb, zb;
    if (IS3) {
        // b runs over whole regions (the host rounds nyb, nzb up to them)
        const int per = nxb * kRegY * kRegZ, nry = (nyb + kRegY - 1) / kRegY;
        const int r = b / per, w = b % per;
        xb = w % nxb;
        yb = (r % nry) * kRegY + (w / nxb) % kRegY;
        zb = (r / nry) * kRegZ + w / (nxb * kRegY);
        if (yb >= nyb || zb >= nzb) return;
    } else {
        if (b >= nxb * nyb * nzb) return;
        xb = b % nxb;
        const int rb = b / nxb;
        yb = rb % nyb;
        zb = rb / nyb;
    }
    const int q0 = blockIdx.y * qc, q1 = min(a.N, q0 + qc);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int x0 = xb * kBlkX, y0 = yb * BY, z0 = zb * BZ;
    const int x = x0 + lane;
    const size_t M = a.M;
    const double diag = 2.0 * (a.ihx2 + a.ihy2 + a.ihz2);
    const auto rU = buf_rsrc(a.U, (size_t)a.N * M * 8);
    const auto rF = buf_rsrc(a.f ? a.f + M : a.U, (size_t)a.N * M * 8);
    const auto rC = buf_rsrc(a.ncorr > 0 ? a.corr : a.U, (size_t)(a.ncorr > 0 ? a.ncorr : 1) * M * 8);
    constexpr int zo = IS3 ? 1 : 0;
    auto lidx = [&](int zl, int yl, int xl) { return ((zl + zo) * LY + yl + 1) * LX + xl + 1; };
    auto gofs = [&](int zz, int yy, int xx) -> unsigned {   // byte offset within a row of U, or kNoLane
        const bool in = xx >= 0 && xx < a.mx && yy >= 0 && yy < a.my && zz >= 0 && zz < a.mz;
        return in ? (((unsigned)zz * (unsigned)a.my + (unsigned)yy) * (unsigned)a.mx + (unsigned)xx) * 8u : kNoLane;
    };
    // the lane's lines (line l = wv + NW e of the block: y = l % BY, z = l / BY)
    unsigned lu[PT];
    int li[PT];
    double vt[PT], hist[7][PT];
    bool valid[PT], store[PT];
    long long slot[PT];
#pragma unroll
    for (int e = 0; e < PT; ++e) {
        const int l = wv + NW * e, yl = l % BY, zl = l / BY;
        const int y = y0 + yl, z = z0 + zl;
        lu[e] = gofs(z, y, x);
        valid[e] = lu[e] != kNoLane;
        store[e] = x < a.mxp && y < a.my && z < a.mz;
        li[e] = lidx(zl, yl, lane);
        slot[e] = ((long long)z * a.my + y) * a.mxp + x;
        vt[e] = valid[e] ? a.ta * a.v[lu[e] / 8u] : 0.0;
#pragma unroll
        for (int j = 0; j < 7; ++j) hist[j][e] = 0.0;
    }
    // halo values h = tid + 256 i: the y faces (y0 - 1, y0 + BY) of each plane, in 3D
    // the z faces (z0 - 1, z0 + BZ) of each line, then the x neighbours (x0 - 1,
    // x0 + 64) of the block's lines
    unsigned ho[BL::HPL];
    int hl[BL::HPL];
#pragma unroll
    for (int i = 0; i < BL::HPL; ++i) {
        int h = tid + BL::NT * i;
        ho[i] = kNoLane;
        hl[i] = -1;
        if (h < 2 * BZ * kBlkX) {
            const int xl = h % kBlkX, r = h / kBlkX, zl = r % BZ, side = r / BZ;
            const int yl = side ? BY : -1;
            ho[i] = gofs(z0 + zl, y0 + yl, x0 + xl);
            hl[i] = lidx(zl, yl, xl);
            continue;
        }
        h -= 2 * BZ * kBlkX;
        if (IS3 && h < 2 * BY * kBlkX) {
            const int xl = h % kBlkX, r = h / kBlkX, yl = r % BY, side = r / BY;
            const int zl = side ? BZ : -1;
            ho[i] = gofs(z0 + zl, y0 + yl, x0 + xl);
            hl[i] = lidx(zl, yl, xl);
            continue;
        }
        if (IS3) h -= 2 * BY * kBlkX;
        if (h < 2 * BY * BZ) {
            const int l = h % (BY * BZ), side = h / (BY * BZ), yl = l % BY, zl = l / BY;
            const int xl = side ? kBlkX : -1;
            ho[i] = gofs(z0 + zl, y0 + yl, x0 + xl);
            hl[i] = lidx(zl, yl, xl);
        }
    }
    double wk[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) wk[j] = a.wk[j];
    RT* __restrict__ out = reinterpret_cast<RT*>(a.Rb);
    struct Row {
        double u[PT], f[PT], c[PT], h[BL::HPL];
    };
    auto load_row = [&](int q, Row& r) {
        const unsigned rq = (unsigned)q * (unsigned)M * 8u;   // row offset (the plan bounds N M 8 < 2^32)
        auto off = [&](unsigned l) { return l == kNoLane ? kNoLane : rq + l; };
#pragma unroll
        for (int e = 0; e < PT; ++e) {
            r.u[e] = buf_ld(rU, off(lu[e]), 0.0);
            r.f[e] = a.f ? buf_ld(rF, off(lu[e]), 0.0) : 0.0;
            r.c[e] = q < a.ncorr ? buf_ld(rC, off(lu[e]), 0.0) : 0.0;
        }
#pragma unroll
        for (int i = 0; i < BL::HPL; ++i) r.h[i] = hl[i] >= 0 ? buf_ld(rU, off(ho[i]), 0.0) : 0.0;
    };
    constexpr int SY = LX, SZ = LY * LX;   // LDS strides of the y and z neighbours
    auto emit = [&](int q, const Row& r) {
        double* S = su[q & 1];
#pragma unroll
        for (int e = 0; e < PT; ++e) S[li[e]] = r.u[e];
#pragma unroll
        for (int i = 0; i < BL::HPL; ++i)
            if (hl[i] >= 0) S[hl[i]] = r.h[i];
        __syncthreads();
        const double sq = a.s[q], sc = a.scale[q];
#pragma unroll
        for (int e = 0; e < PT; ++e) {
            const int c = li[e];
#pragma unroll
            for (int j = 6; j > 0; --j) hist[j][e] = hist[j - 1][e];
            hist[0][e] = r.u[e];
            double ts = 0.0;
#pragma unroll
            for (int j = 0; j < 7; ++j) ts += wk[j] * hist[j][e];
            double nb = a.ihx2 * (S[c - 1] + S[c + 1]) + a.ihy2 * (S[c - SY] + S[c + SY]);
            if (IS3) nb += a.ihz2 * (S[c - SZ] + S[c + SZ]);
            const double res = vt[e] * sq + r.f[e] + r.c[e] - a.ta * ts - (diag * r.u[e] - nb);
            if (store[e]) out[(size_t)q * a.Mp + slot[e]] = valid[e] ? (RT)(res * sc) : (RT)0;
        }
    };
    // history rows q0-k..q0-1 (absent rows, and lags beyond k whose weights are
    // zero, stay zero); hist[0] holds the row before q0
#pragma unroll
    for (int j = 6; j >= 1; --j) {
        const int qh = q0 - j;
        if (qh >= 0 && j <= a.k) {
            const unsigned rq = (unsigned)qh * (unsigned)M * 8u;
#pragma unroll
            for (int e = 0; e < PT; ++e) {
#pragma unroll
                for (int i = 6; i > 0; --i) hist[i][e] = hist[i - 1][e];
                hist[0][e] = buf_ld(rU, lu[e] == kNoLane ? kNoLane : rq + lu[e], 0.0);
            }
        }
    }
    Row cur, nxt;
    load_row(q0, cur);
    for (int q = q0; q + 1 < q1; ++q) {
        load_row(q + 1, nxt);
        emit(q, cur);
        cur = nxt;
    }
    emit(q1 - 1, cur);
}

template <typename R, int LOGN, int W, int NT>
__global__ __launch_bounds__(NT) void k_tfft(FwdArgs a) {
    constexpr int N = 1 << LOGN;
    constexpr int B = W / 2;
    constexpr int PER = N * W / NT;
    static_assert(PER * NT == N * W, "tile shape");
    __shared__ cx<R> sm[N * B];
    __shared__ cx<R> stw[N / 2];
    R* smr = reinterpret_cast<R*>(sm);
    const int ntiles = (a.Mp + W - 1) / W;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (tile >= ntiles) return;
    const int tid = threadIdx.x;
    const int s0 = tile * W;
    const R* rb = reinterpret_cast<const R*>(a.Rb);
    R v[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int idx = tid + i * NT;
        const int q = idx / W, l = idx % W;
        v[i] = s0 + l < a.Mp ? rb[(size_t)q * a.Mp + s0 + l] : (R)0;
    }
    for (int j = tid; j < N / 2; j += NT) stw[j] = reinterpret_cast<const cx<R>*>(a.tw)[j];
#pragma unroll
    for (int i = 0; i < PER; ++i) smr[tid + i * NT] = v[i];
    __syncthreads();
    lds_fft<R, LOGN, B, NT, false, true, 0>(sm, stw);
    store_half_spectrum<R, N, B, NT>(sm, reinterpret_cast<cx<R>*>(a.S), a.ldS, s0, a.Mp);
}

template <typename R, int LOGN>
hipError_t fwd_split(const FwdArgs& a, int* nb, hipStream_t st) {
    const bool is3 = a.mz > 1;
    const int by = is3 ? ResidBlock<true>::BY : ResidBlock<false>::BY;
    const int bz = is3 ? ResidBlock<true>::BZ : ResidBlock<false>::BZ;
    const int nxb = (a.mxp + kBlkX - 1) / kBlkX, nyb = (a.my + by - 1) / by, nzb = (a.mz + bz - 1) / bz;
    const int nblk = nxb * nyb * nzb;
    const int nvirt = is3 ? nxb * ((nyb + kRegY - 1) / kRegY * kRegY) * ((nzb + kRegZ - 1) / kRegZ * kRegZ) : nblk;
    const int nres = (nvirt + 7) / 8 * 8;
    // time rows per workgroup: each chunk re-reads the k rows before it,
    // so the longest chunk (up to 256) that still leaves >= 1024 workgroups
    int qc = 32;
    while (qc < 256 && (long long)nblk * ((a.N + 2 * qc - 1) / (2 * qc)) >= 1024) qc *= 2;
    const int nq = (a.N + qc - 1) / qc;
    if (is3)
        PINT_LAUNCH((k_resid<R, true>), dim3(nres, nq), dim3(ResidBlock<true>::NT), 0, st, a, qc, nxb, nyb, nzb);
    else
        PINT_LAUNCH((k_resid<R, false>), dim3(nres, nq), dim3(ResidBlock<false>::NT), 0, st, a, qc, nxb, nyb, nzb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // 128-byte row segments where the N x W tile fits 64 KB of LDS
    constexpr int WL = 65536 / (N_OF(LOGN) * (int)sizeof(R));
    constexpr int W0 = sizeof(R) == 8 ? 16 : 32;
    constexpr int W = WL < W0 ? (WL < 2 ? 2 : WL) : W0;
    // lanes: 256 for N <= 256, else 512 (each measured ~1% ahead of the other there)
    constexpr int NTC = LOGN <= 8 ? 256 : 512;
    constexpr int NT = N_OF(LOGN) * W >= NTC ? NTC : N_OF(LOGN) * W;
    const int ntiles = ((a.Mp + W - 1) / W + 7) / 8 * 8;
    if (nb) *nb = ntiles;
    PINT_LAUNCH((k_tfft<R, LOGN, W, NT>), dim3(ntiles), dim3(NT), 0, st, a);
    return hipGetLastError();
}

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
//   BDF-k: 0 split residual + time FFT (kind 5), 4 wide-tile march (kind 0 in
//   2D, 3 in 3D), 1 march with the time-FFT tile, 2 one workgroup per tile,
//   3 half-width wide-tile march with two workgroups per CU (kind 4);
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
    // split residual + time FFT (needs the slot-layout buffer and 32-bit row offsets)
    if (var == 0 && a.Rb && (long long)a.N * a.M * 8 < (long long)kNoLane) return 5;
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
    if ((var == 0 || var == 4) && wide_ok) return a.mz == 1 ? 0 : 3;
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
    if (kind == 5) return fwd_split<R, LOGN>(a, nb, st);
    const int ntiles = (a.Mp + W - 1) / W;
    if constexpr (W >= 16) {
        // small grids (fewer tiles than a tenth of the CUs' worth): tiles of W/8 slots,
        // so the work spreads over 8 times as many workgroups (each one's chain of
        // loads, barriers and FFT stages is what a launch this small waits for)
        constexpr int WS = W / 8;
        constexpr int NTS = N_OF(LOGN) * WS >= kNT ? kNT : 64;
        if (ntiles < 32) {
            const int grid = (((a.Mp + WS - 1) / WS + 7) / 8) * 8;
            if (nb) *nb = grid;
            PINT_LAUNCH((k_fwd_heat<R, LOGN, WS, NTS>), dim3(grid), dim3(NTS), 0, st, a);
            return hipGetLastError();
        }
    }
    const int grid = ((ntiles + 7) / 8) * 8;
    if (nb) *nb = grid;
    PINT_LAUNCH((k_fwd_heat<R, LOGN, W, NT>), dim3(grid), dim3(NT), 0, st, a);
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

}  // namespace

hipError_t launch_forward(const FwdArgs& a, bool mixed, bool cq, int* nb, hipStream_t st) {
    return mixed ? fwd_dispatch<float>(a, cq, nb, st) : fwd_dispatch<double>(a, cq, nb, st);
}

hipError_t launch_inject(const FwdArgs& a, const void* Sg, bool mixed, hipStream_t st) {
    const int pchunk = 4 * kInjectBatch;
    const dim3 grid((unsigned)((a.Mp + 255) / 256), (unsigned)((a.N / 2 + 1 + pchunk - 1) / pchunk));
    if (mixed)
        PINT_LAUNCH(k_inject<float>, grid, dim3(256), 0, st, a, Sg, pchunk);
    else
        PINT_LAUNCH(k_inject<double>, grid, dim3(256), 0, st, a, Sg, pchunk);
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
}  // namespace

bool forward_variant_distinct(const FwdArgs& a, bool mixed, bool cq, int var) {
    FwdArgs b = a, c = a;
    b.var = 0;
    c.var = var;
    return mixed ? fwd_kind_of<float>(b, cq) != fwd_kind_of<float>(c, cq)
                 : fwd_kind_of<double>(b, cq) != fwd_kind_of<double>(c, cq);
}

}  // namespace pint

