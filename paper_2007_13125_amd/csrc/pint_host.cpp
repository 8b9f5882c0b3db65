// Host runtime of the C ABI declared in include/pint.h: argument validation,
// FP64 setup tables, workspace layout, the sweep loop and the stop test.
#include "../../include/pint.h"
#include "pint_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <new>
#include <utility>
#include <string>
#include <vector>

using pint::FwdArgs;
using pint::GenArgs;
using pint::InvArgs;
using pint::SpaceArgs;

namespace {

thread_local std::string g_err;

pint_status fail(pint_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

#define HIP_TRY(expr)                                                                                 \
    do {                                                                                              \
        hipError_t e_ = (expr);                                                                       \
        if (e_ != hipSuccess)                                                                         \
            return fail(e_ == hipErrorOutOfMemory ? PINT_E_NOMEM : PINT_E_HIP,                        \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                           \
    } while (0)

bool is_pow2(long long x) { return x > 0 && (x & (x - 1)) == 0; }
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

using cld = std::complex<long double>;
const long double kPi = 3.141592653589793238462643383279502884L;

// e^{-2 pi i j / L}, evaluated in extended precision and rounded once.
cld twiddle(long long j, long long L) {
    const long double ang = -2.0L * kPi * (long double)(j % L) / (long double)L;
    return cld(cosl(ang), sinl(ang));
}

// BDF-k weights: coefficients of delta_k(z) = sum_{l=1..k} (1 - z)^l / l
// (Sec. 2.1, eq. bdf-gen), by the binomial expansion of each power.
std::vector<long double> bdf_weights(int k) {
    std::vector<long double> w(k + 1, 0.0L);
    for (int l = 1; l <= k; ++l) {
        long double binom = 1.0L;  // C(l, j)
        for (int j = 0; j <= l; ++j) {
            w[j] += ((j & 1) ? -binom : binom) / (long double)l;
            binom = binom * (long double)(l - j) / (long double)(j + 1);
        }
    }
    return w;
}

// Power-series coefficients of delta_k(xi)^alpha (Sec. 3.1, eq. delta), by
// J.C.P. Miller's recurrence for the power of a series (from P Q' = alpha P' Q).
std::vector<long double> cq_weights(int k, long double alpha, int n) {
    const std::vector<long double> p = bdf_weights(k);
    std::vector<long double> c(n, 0.0L);
    c[0] = powl(p[0], alpha);
    for (int j = 1; j < n; ++j) {
        long double acc = 0.0L;
        const int top = j < k ? j : k;
        for (int i = 1; i <= top; ++i) acc += ((alpha + 1.0L) * i - j) * p[i] * c[j - i];
        c[j] = acc / (j * p[0]);
    }
    return c;
}

// Starting-step corrections of Table 1 (the same table is used by BDF-k and
// CQ-BDF-k): a_n^{(k)}, n = 1..k-1, and b_{l,n}^{(k)}, l = 1..k-2.
struct Table1 {
    double a[5];
    double b[4][5];
};
Table1 table1(int k) {
    Table1 t;
    std::memset(&t, 0, sizeof(t));
    switch (k) {
        case 2:
            t.a[0] = 1.0 / 2;
            break;
        case 3:
            t.a[0] = 11.0 / 12; t.a[1] = -5.0 / 12;
            t.b[0][0] = 1.0 / 12;
            break;
        case 4:
            t.a[0] = 31.0 / 24; t.a[1] = -7.0 / 6; t.a[2] = 3.0 / 8;
            t.b[0][0] = 1.0 / 6; t.b[0][1] = -1.0 / 12;
            break;
        case 5:
            t.a[0] = 1181.0 / 720; t.a[1] = -177.0 / 80; t.a[2] = 341.0 / 240; t.a[3] = -251.0 / 720;
            t.b[0][0] = 59.0 / 240; t.b[0][1] = -29.0 / 120; t.b[0][2] = 19.0 / 240;
            t.b[1][0] = 1.0 / 240; t.b[1][1] = -1.0 / 240;
            t.b[2][0] = 1.0 / 720;
            break;
        case 6:
            t.a[0] = 2837.0 / 1440; t.a[1] = -2543.0 / 720; t.a[2] = 17.0 / 5; t.a[3] = -1201.0 / 720;
            t.a[4] = 95.0 / 288;
            t.b[0][0] = 77.0 / 240; t.b[0][1] = -7.0 / 15; t.b[0][2] = 73.0 / 240; t.b[0][3] = -3.0 / 40;
            t.b[1][0] = 1.0 / 96; t.b[1][1] = -1.0 / 60; t.b[1][2] = 1.0 / 160;
            t.b[2][0] = -1.0 / 360; t.b[2][1] = 1.0 / 720;
            break;
        default:
            break;
    }
    return t;
}

}  // namespace

struct pint_plan {
    pint_grid g{};
    pint_params p{};
    int M = 0, N = 0, nP = 0, ldS = 0, dim = 0, mx = 1, my = 1, mz = 1;
    int mxp = 16, Mp = 16;  // padded spectrum rows (multiple of 16 slots) and slots per plane
    double tau = 0, ta = 0, hd = 1, ih2[3] = {0, 0, 0};
    bool mixed = false, cq = false;
    hipStream_t st = nullptr;
    int device = 0;
    // small device tables (owned)
    std::vector<void*> owned;
    double *d_scale = nullptr, *d_unscale = nullptr, *d_s = nullptr, *d_w = nullptr;
    double *d_an = nullptr, *d_blt = nullptr, *d_mu[3] = {nullptr, nullptr, nullptr};
    double2 *d_sigma = nullptr, *d_what = nullptr, *d_tw2 = nullptr;
    void *d_twN = nullptr, *d_twL[3] = {nullptr, nullptr, nullptr};
    // Bluestein tables of the axes whose 2(m+1) is not a power of two
    int logP[3] = {0, 0, 0};
    void *d_chirp[3] = {nullptr, nullptr, nullptr}, *d_bh[3] = {nullptr, nullptr, nullptr};
    void *d_twP[3] = {nullptr, nullptr, nullptr};
    // time axis that is not a power of two >= 8: residual buffer + Bluestein DFT tables
    bool gn = false;
    int logPt = 0;
    void *d_chirpT = nullptr, *d_bhT = nullptr, *d_twPT = nullptr;
    double2 *d_whT = nullptr, *d_twhT = nullptr;   // CQ history convolution on the Bluestein length
    bool fem = false;                 // P1 elements (1D): mass matrix on the time derivative
    double* d_mass = nullptr;         // [m] eigenvalues of the scaled mass matrix (P1 only)
    double* Rb = nullptr;
    size_t off_r = 0;
    // 1D plans: buffers of the semilinear solve (Newton correction W, Newton
    // residual R, Jacobian diagonal g'(Ubar))
    double *nlW = nullptr, *nlR = nullptr, *nlD = nullptr;
    size_t off_nl = 0;
    int max_partials = 0;
    double2* d_sigma_seq = nullptr;   // {omega_0 tau^{-alpha}, 0}: the shift of the sequential stepper
    double wk[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double inv_factor = 1.0;
    // workspace
    void* ws = nullptr;
    size_t ws_bytes = 0;
    bool ws_owned = false;
    void* S = nullptr;
    double *corr = nullptr, *partial = nullptr, *norm_tmp = nullptr;
    void* Sg = nullptr;   // direct form, BDF-k: spectrum of the source part (set at bind)
    size_t off_corr = 0, off_partial = 0, off_norm = 0, off_sg = 0;
    // bound data
    const double *v = nullptr, *f = nullptr, *fder = nullptr;
    bool bound = false;
    double* h_norms = nullptr;  // pinned host, 2 doubles
    // batch: sub-plans sharing the stream
    std::vector<pint_plan*> inst;
    // batch of 1D instances in batched sweeps: descriptors, prefix tables and
    // norms (device block and its pinned host stage, same layout), DFT partials
    void* d_bblk = nullptr;
    void* h_bblk = nullptr;
    size_t b_int_off = 0, b_norm_off = 0, b_bytes = 0;
    double* d_bpart = nullptr;
    // batch 1D instance: Thomas scratch [N/2+1][M] complex in the workspace
    size_t off_th = 0;
    void* thomas = nullptr;
    // kernel variants in use: forward, x pass, y/z pass, 1D tridiagonal split (0 = built-in)
    int var[4] = {0, 0, 0, 0};
    int tune_reps = 0;                // > 0: the solves time the variants first (autotune)
    bool tuned = false;

    ~pint_plan() {
        for (void* q : owned) (void)hipFree(q);
        if (ws_owned && ws) (void)hipFree(ws);
        if (h_norms) (void)hipHostFree(h_norms);
        if (h_bblk) (void)hipHostFree(h_bblk);
        for (pint_plan* q : inst) delete q;
    }
};

namespace {

template <typename T>
pint_status upload(pint_plan* P, T** dst, const T* src, size_t n) {
    void* q = nullptr;
    HIP_TRY(hipMalloc(&q, n * sizeof(T) > 0 ? n * sizeof(T) : 16));
    P->owned.push_back(q);
    HIP_TRY(hipMemcpy(q, src, n * sizeof(T), hipMemcpyHostToDevice));
    *dst = static_cast<T*>(q);
    return PINT_OK;
}

pint_status upload_tw(pint_plan* P, void** dst, long long L, bool single) {
    if (single) {
        std::vector<float2> t(L);
        for (long long j = 0; j < L; ++j) {
            const cld w = twiddle(j, L);
            t[j].x = (float)w.real();
            t[j].y = (float)w.imag();
        }
        float2* q = nullptr;
        pint_status s = upload(P, &q, t.data(), t.size());
        *dst = q;
        return s;
    }
    std::vector<double2> t(L);
    for (long long j = 0; j < L; ++j) {
        const cld w = twiddle(j, L);
        t[j].x = (double)w.real();
        t[j].y = (double)w.imag();
    }
    double2* q = nullptr;
    pint_status s = upload(P, &q, t.data(), t.size());
    *dst = q;
    return s;
}

// In-place radix-2 FFT, X_k = sum_j x_j e^{-2 pi i jk/n}, n a power of two (host, long double).
void host_fft(std::vector<cld>& x) {
    const size_t n = x.size();
    for (size_t i = 1, j = 0; i < n; ++i) {
        size_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(x[i], x[j]);
    }
    for (size_t len = 2; len <= n; len <<= 1)
        for (size_t i = 0; i < n; i += len)
            for (size_t k = 0; k < len / 2; ++k) {
                const cld w = twiddle((long long)(k * (n / len)), (long long)n);
                const cld u = x[i + k], v = x[i + k + len / 2] * w;
                x[i + k] = u + v;
                x[i + k + len / 2] = u - v;
            }
}

template <typename C>
pint_status upload_cld(pint_plan* P, void** dst, const std::vector<cld>& v) {
    std::vector<C> t(v.size());
    for (size_t j = 0; j < v.size(); ++j) {
        t[j].x = (decltype(t[j].x))v[j].real();
        t[j].y = (decltype(t[j].y))v[j].imag();
    }
    C* q = nullptr;
    pint_status s = upload(P, &q, t.data(), t.size());
    *dst = q;
    return s;
}

// Bluestein tables of a length-L DFT: chirp c_t = e^{-pi i t^2/L} (t < L,
// argument reduced mod 2L), Bh = FFT_P(b)/P with b_l = conj(c_|l|) for |l| < L
// wrapped mod P, P >= max(2L-1, 2^min_logp); twiddles of length P.  Tables in
// the spectrum precision.
pint_status upload_bluestein_tables(pint_plan* P, long long L, int min_logp, void** chirp, void** bh, void** twP,
                                    int* logp_out) {
    int logp = min_logp;
    while ((1LL << logp) < 2 * L - 1) ++logp;
    const long long Pn = 1LL << logp;
    std::vector<cld> c(L), b(Pn, cld(0, 0));
    for (long long t = 0; t < L; ++t) c[t] = twiddle((t * t) % (2 * L), 2 * L);
    for (long long l = 0; l < L; ++l) {
        b[l] = std::conj(c[l]);
        if (l > 0) b[Pn - l] = std::conj(c[l]);
    }
    host_fft(b);
    for (auto& z : b) z /= (long double)Pn;
    pint_status rc;
    if (P->mixed) {
        if ((rc = upload_cld<float2>(P, chirp, c)) != PINT_OK) return rc;
        if ((rc = upload_cld<float2>(P, bh, b)) != PINT_OK) return rc;
    } else {
        if ((rc = upload_cld<double2>(P, chirp, c)) != PINT_OK) return rc;
        if ((rc = upload_cld<double2>(P, bh, b)) != PINT_OK) return rc;
    }
    if ((rc = upload_tw(P, twP, Pn, P->mixed)) != PINT_OK) return rc;
    *logp_out = logp;
    return PINT_OK;
}

// Sine transform of an axis with m interior nodes whose odd extension has
// length L = 2(m+1) not a power of two (P >= 16, the smallest transform the
// Bluestein DST kernels are built for).
pint_status upload_bluestein(pint_plan* P, int axis, int m) {
    return upload_bluestein_tables(P, 2LL * (m + 1), 4, &P->d_chirp[axis], &P->d_bh[axis], &P->d_twP[axis],
                                   &P->logP[axis]);
}

pint_status validate(const pint_grid* g, const pint_params* p) {
    if (!g || !p) return fail(PINT_E_ARG, "grid and params must not be NULL");
    if (g->dim < 1 || g->dim > 3) return fail(PINT_E_ARG, "grid.dim must be 1, 2 or 3");
    long long M = 1;
    for (int i = 0; i < g->dim; ++i) {
        if (g->m[i] < 1) return fail(PINT_E_ARG, "grid.m[i] must be >= 1");
        if (!(g->len[i] > 0.0) || !std::isfinite(g->len[i])) return fail(PINT_E_ARG, "grid.len[i] must be > 0");
        M *= g->m[i];
    }
    if (M > (1LL << 30)) return fail(PINT_E_UNSUPPORTED, "more than 2^30 spatial unknowns");
    if (p->k < 1 || p->k > 6) return fail(PINT_E_ARG, "k must be in 1..6");
    if (!(p->alpha > 0.0 && p->alpha <= 1.0)) return fail(PINT_E_ARG, "alpha must be in (0, 1]");
    if (!(p->T > 0.0) || !std::isfinite(p->T)) return fail(PINT_E_ARG, "T must be > 0");
    if (!(p->kappa > 0.0 && p->kappa < 1.0)) return fail(PINT_E_ARG, "kappa must be in (0, 1)");
    if (!(p->tol > 0.0)) return fail(PINT_E_ARG, "tol must be > 0");
    if (p->max_sweeps < 1) return fail(PINT_E_ARG, "max_sweeps must be >= 1");
    if (p->precision != PINT_FP64 && p->precision != PINT_MIXED) return fail(PINT_E_ARG, "bad precision");
    if (p->form != PINT_RESIDUAL && p->form != PINT_DIRECT) return fail(PINT_E_ARG, "bad form");
    if (p->norm != PINT_NORM_INF && p->norm != PINT_NORM_L2_TERMINAL) return fail(PINT_E_ARG, "bad norm");
    if (p->init < PINT_INIT_V || p->init > PINT_INIT_USER) return fail(PINT_E_ARG, "bad init");
    if (p->space != PINT_SPACE_FD && p->space != PINT_SPACE_FEM_P1) return fail(PINT_E_ARG, "bad space");
    if (p->space == PINT_SPACE_FEM_P1 && g->dim != 1)
        return fail(PINT_E_UNSUPPORTED, "P1 elements are implemented for 1D grids");
    if (p->N <= p->k) return fail(PINT_E_ARG, "N must exceed k");
    if (p->N % 2 != 0) return fail(PINT_E_ARG, "N must be even");
    // The direct form's right-hand side would be assembled from FP32 spectra, so
    // its fixed point would carry FP32 rounding; the FP64 outer correction of
    // the mixed form needs the residual form.
    if (p->precision == PINT_MIXED && p->form == PINT_DIRECT)
        return fail(PINT_E_UNSUPPORTED, "mixed precision runs the residual form only");
    if (p->N > (1 << pint::kMaxLogN)) return fail(PINT_E_UNSUPPORTED, "N must be at most 2048");
    if (g->dim == 1) {
        if (2LL * (g->m[0] + 1) > (1 << pint::kMaxLogL))
            return fail(PINT_E_UNSUPPORTED, "1D grids are limited to m <= 2047");
    } else {
        long long plane = 16;   // complex FP64 slots of one spectrum plane, in bytes
        for (int i = 0; i < g->dim; ++i) {
            if (2LL * (g->m[i] + 1) > (1 << pint::kMaxLogL))
                return fail(PINT_E_UNSUPPORTED, "2D/3D grids are limited to m_i <= 2047");
            plane *= i == 0 ? (g->m[0] + 15) / 16 * 16 : g->m[i];
        }
        // the spatial passes address within a spectrum plane with 32-bit byte offsets
        if (plane >= (1LL << 32) - (1LL << 24))
            return fail(PINT_E_UNSUPPORTED, "2D/3D grids are limited to spectrum planes below 4 GiB");
    }
    return PINT_OK;
}

pint_status build_plan(pint_plan* P, const pint_grid* g, const pint_params* p, hipStream_t st) {
    P->g = *g;
    P->p = *p;
    P->st = st;
    HIP_TRY(hipGetDevice(&P->device));
    P->dim = g->dim;
    P->mx = g->m[0];
    P->my = g->dim >= 2 ? g->m[1] : 1;
    P->mz = g->dim >= 3 ? g->m[2] : 1;
    P->M = P->mx * P->my * P->mz;
    P->N = p->N;
    P->nP = p->N / 2 + 1;
    P->mxp = (P->mx + 15) / 16 * 16;
    P->Mp = P->mxp * P->my * P->mz;
    P->ldS = (int)((P->Mp + 63) / 64 * 64);
    P->mixed = p->precision == PINT_MIXED;
    P->cq = p->alpha < 1.0;
    P->fem = p->space == PINT_SPACE_FEM_P1;
    // P1 elements take the general-length kernels, whose residual applies the mass matrix
    P->gn = P->fem || !(is_pow2(p->N) && p->N >= (1 << pint::kMinLogN));
    const int N = P->N, k = p->k;
    const long double tau = (long double)p->T / N;
    P->tau = (double)tau;
    P->ta = (double)powl(tau, -(long double)p->alpha);
    P->hd = 1.0;
    P->inv_factor = 1.0;
    for (int i = 0; i < g->dim; ++i) {
        const double h = g->len[i] / (g->m[i] + 1);
        P->ih2[i] = 1.0 / (h * h);
        P->hd *= h;
        P->inv_factor *= -2.0 * (g->m[i] + 1);
    }
    P->inv_factor = 1.0 / P->inv_factor;

    // time weights omega_0..omega_{N-1}
    std::vector<long double> w(N, 0.0L);
    const std::vector<long double> wb = bdf_weights(k);
    if (!P->cq) {
        for (int j = 0; j <= k; ++j) w[j] = wb[j];
    } else {
        w = cq_weights(k, p->alpha, N);
    }
    for (int j = 0; j <= k; ++j) P->wk[j] = P->cq ? 0.0 : (double)wb[j];
    // s_n = sum_{j<n} omega_j; zero for n > k in BDF-k (the weights sum to 0)
    std::vector<double> s(N);
    long double acc = 0.0L;
    for (int n = 1; n <= N; ++n) {
        acc += w[n - 1];
        s[n - 1] = (!P->cq && n > k) ? 0.0 : (double)acc;
    }
    // kappa^{+-q/N}; the 1/N of the inverse transform is folded into the unscale table
    std::vector<double> scale(N), unscale(N);
    const long double lk = logl((long double)p->kappa);
    for (int q = 0; q < N; ++q) {
        scale[q] = (double)expl(lk * q / N);
        unscale[q] = (double)(expl(-lk * q / N) / N);
    }
    // eigenvalues d_p of the scaled circulant, p = 0..N/2, and sigma_p = tau^{-alpha} d_p
    std::vector<double2> sigma(P->nP);
    const long double kap1 = expl(lk / N);
    for (int q = 0; q < P->nP; ++q) {
        cld d(0.0L, 0.0L);
        if (!P->cq) {
            // BDF-k: d_p = delta_k(kappa^{1/N} e^{-2 pi i p/N}) (Sec. 2.2, roundoff paragraph)
            const cld zeta = kap1 * twiddle(q, N);
            cld pw(1.0L, 0.0L);
            for (int l = 1; l <= k; ++l) {
                pw *= (cld(1.0L, 0.0L) - zeta);
                d += pw / (long double)l;
            }
        } else {
            // CQ: first column kappa^{j/N} omega_j of the N x N scaled circulant, DFT'd directly
            for (int j = 0; j < N; ++j) d += expl(lk * j / N) * w[j] * twiddle((long long)j * q, N);
        }
        const cld sg = (long double)P->ta * d;
        sigma[q].x = (double)sg.real();
        sigma[q].y = (double)sg.imag();
    }
    pint_status rc;
    if ((rc = upload(P, &P->d_scale, scale.data(), N)) != PINT_OK) return rc;
    if ((rc = upload(P, &P->d_unscale, unscale.data(), N)) != PINT_OK) return rc;
    if ((rc = upload(P, &P->d_s, s.data(), N)) != PINT_OK) return rc;
    if ((rc = upload(P, &P->d_sigma, sigma.data(), P->nP)) != PINT_OK) return rc;
    {
        double2 s0;
        s0.x = (double)((long double)P->ta * w[0]);
        s0.y = 0.0;
        if ((rc = upload(P, &P->d_sigma_seq, &s0, 1)) != PINT_OK) return rc;
    }
    if ((rc = upload_tw(P, &P->d_twN, N, P->mixed)) != PINT_OK) return rc;
    {
        std::vector<double> wd(N);
        for (int j = 0; j < N; ++j) wd[j] = (double)w[j];
        if ((rc = upload(P, &P->d_w, wd.data(), N)) != PINT_OK) return rc;
    }
    // Bluestein time-DFT tables: sweeps whose time axis is not a power of two,
    // and every 1D plan (the semilinear solve runs the general-length kernels)
    if (P->gn || g->dim == 1) {
        if ((rc = upload_bluestein_tables(P, N, 2, &P->d_chirpT, &P->d_bhT, &P->d_twPT, &P->logPt)) != PINT_OK)
            return rc;
        if (P->cq) {
            // the residual's causal history sums as a linear convolution on the
            // same P >= 2N - 1 points: FFT_P(omega, 0)/P and FP64 twiddles
            const long long Pn = 1LL << P->logPt;
            std::vector<cld> wz(Pn, cld(0, 0));
            for (int j = 0; j < N; ++j) wz[j] = (long double)w[j];
            host_fft(wz);
            std::vector<double2> wh(Pn);
            for (long long t = 0; t < Pn; ++t) {
                wh[t].x = (double)(wz[t].real() / (long double)Pn);
                wh[t].y = (double)(wz[t].imag() / (long double)Pn);
            }
            if ((rc = upload(P, &P->d_whT, wh.data(), (size_t)Pn)) != PINT_OK) return rc;
            if (P->mixed) {
                void* t2 = nullptr;
                if ((rc = upload_tw(P, &t2, Pn, false)) != PINT_OK) return rc;
                P->d_twhT = static_cast<double2*>(t2);
            } else {
                P->d_twhT = static_cast<double2*>(P->d_twPT);
            }
        }
    }
    if (!P->gn && P->cq) {
        // spectrum of (omega, 0) on 2N points, divided by 2N (inverse normalisation)
        const int N2 = 2 * N;
        std::vector<double2> what(N2);
        for (int q = 0; q < N2; ++q) {
            cld z(0.0L, 0.0L);
            for (int j = 0; j < N; ++j) z += w[j] * twiddle((long long)j * q, N2);
            z /= (long double)N2;
            what[q].x = (double)z.real();
            what[q].y = (double)z.imag();
        }
        if ((rc = upload(P, &P->d_what, what.data(), N2)) != PINT_OK) return rc;
        void* t2 = nullptr;
        if ((rc = upload_tw(P, &t2, N2, false)) != PINT_OK) return rc;
        P->d_tw2 = static_cast<double2*>(t2);
    }
    // Table 1 rows with tau^l folded into b
    const Table1 t1 = table1(k);
    double an[5], blt[4 * 6];
    std::memset(blt, 0, sizeof(blt));
    for (int n = 0; n < 5; ++n) an[n] = t1.a[n];
    for (int l = 1; l <= 4; ++l)
        for (int n = 1; n <= 5; ++n) blt[(l - 1) * 6 + (n - 1)] = t1.b[l - 1][n - 1] * (double)powl(tau, l);
    if ((rc = upload(P, &P->d_an, an, 5)) != PINT_OK) return rc;
    if ((rc = upload(P, &P->d_blt, blt, 24)) != PINT_OK) return rc;
    // sine eigenvalues of each second-difference factor and DST twiddles
    for (int i = 0; i < g->dim; ++i) {
        const int m = g->m[i];
        std::vector<double> mu(m);
        const double h = g->len[i] / (m + 1);
        for (int j = 0; j < m; ++j) {
            const long double sn = sinl((j + 1) * kPi / (2.0L * (m + 1)));
            mu[j] = (double)(4.0L / ((long double)h * h) * sn * sn);
        }
        if ((rc = upload(P, &P->d_mu[i], mu.data(), m)) != PINT_OK) return rc;
        if (P->fem) {
            // eigenvalues (2 + cos(j pi h))/3 of the scaled P1 mass matrix tridiag(1, 4, 1)/6
            std::vector<double> mt(m);
            for (int j = 0; j < m; ++j) mt[j] = (double)((2.0L + cosl((j + 1) * kPi / (m + 1))) / 3.0L);
            if ((rc = upload(P, &P->d_mass, mt.data(), m)) != PINT_OK) return rc;
        }
        const long long L = 2LL * (m + 1);
        if (is_pow2(L) && L <= (1LL << pint::kMaxLogL) && (g->dim == 1 || L >= 8)) {
            if ((rc = upload_tw(P, &P->d_twL[i], L, P->mixed)) != PINT_OK) return rc;
        } else {
            if ((rc = upload_bluestein(P, i, m)) != PINT_OK) return rc;
        }
    }
    // workspace layout
    const size_t cbytes = P->mixed ? 2 * sizeof(float) : 2 * sizeof(double);
    size_t off = align256((size_t)P->nP * P->ldS * cbytes);
    P->off_corr = off;
    off += align256((size_t)(k > 1 ? k - 1 : 1) * P->M * sizeof(double));
    P->off_partial = off;
    const size_t maxblocks = ((size_t)(P->Mp + 1) / 2 + 8) / 8 * 8 + 8;
    P->max_partials = (int)maxblocks;
    off += align256(maxblocks * 2 * sizeof(double));
    P->off_norm = off;
    off += 256;
    // residual buffer: [N][M] FP64 for a time axis that is not a power of two, or
    // [N][Mp] (spectrum-slot layout, spectrum real type) for the split forward
    // variant of BDF-k residual sweeps on 2D/3D grids
    if (P->gn || g->dim == 1 || (!P->cq && p->form == PINT_RESIDUAL && g->dim >= 2)) {
        P->off_r = off;
        off += align256((size_t)N * P->Mp * sizeof(double));
    }
    if (g->dim == 1) {
        P->off_nl = off;
        off += 2 * align256((size_t)N * P->M * sizeof(double)) + align256((size_t)P->M * sizeof(double));
    }
    if (!P->cq && !P->gn && p->form == PINT_DIRECT) {
        P->off_sg = off;
        off += align256((size_t)P->nP * P->ldS * cbytes);
    }
    P->ws_bytes = off;
    HIP_TRY(hipHostMalloc((void**)&P->h_norms, 2 * sizeof(double), hipHostMallocDefault));
    return PINT_OK;
}

void attach_workspace(pint_plan* P, void* ws) {
    P->ws = ws;
    char* b = static_cast<char*>(ws);
    P->S = b;
    P->corr = reinterpret_cast<double*>(b + P->off_corr);
    P->partial = reinterpret_cast<double*>(b + P->off_partial);
    P->norm_tmp = reinterpret_cast<double*>(b + P->off_norm);
    P->Sg = P->off_sg ? static_cast<void*>(b + P->off_sg) : nullptr;
    P->Rb = P->off_r ? reinterpret_cast<double*>(b + P->off_r) : nullptr;
    P->thomas = P->off_th ? static_cast<void*>(b + P->off_th) : nullptr;
    if (P->off_nl) {
        const size_t nm = align256((size_t)P->N * P->M * sizeof(double));
        P->nlW = reinterpret_cast<double*>(b + P->off_nl);
        P->nlR = reinterpret_cast<double*>(b + P->off_nl + nm);
        P->nlD = reinterpret_cast<double*>(b + P->off_nl + 2 * nm);
    } else {
        P->nlW = P->nlR = P->nlD = nullptr;
    }
}

// Workspace owned by the plan itself (batch instances only; single plans get
// theirs from the caller through pint_plan_set_workspace).
pint_status own_workspace(pint_plan* P) {
    void* q = nullptr;
    HIP_TRY(hipMalloc(&q, P->ws_bytes));
    P->ws_owned = true;
    attach_workspace(P, q);
    return PINT_OK;
}

// Optional per-launch timing: an event pair around every kernel launch of a
// sweep, on the plan's stream.
struct Profiler {
    std::vector<std::string> names;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;   // one pair per launch
    std::vector<int> slot;                               // launch -> slot index
    int cursor = 0;                                      // slot index within the sweep
    hipStream_t st = nullptr;
    hipError_t begin(const char* name) {
        if (cursor >= (int)names.size()) names.push_back(name);
        hipEvent_t a, b;
        hipError_t e = hipEventCreate(&a);
        if (e != hipSuccess) return e;
        if ((e = hipEventCreate(&b)) != hipSuccess) return e;
        ev.push_back({a, b});
        slot.push_back(cursor);
        return hipEventRecord(a, st);
    }
    hipError_t end() {
        ++cursor;
        return hipEventRecord(ev.back().second, st);
    }
    ~Profiler() {
        for (auto& e : ev) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
    }
};

#define PROF_BEGIN(prof, name) \
    if (prof) HIP_TRY((prof)->begin(name))
#define PROF_END(prof) \
    if (prof) HIP_TRY((prof)->end())

FwdArgs fwd_args(const pint_plan* P, const double* U) {
    FwdArgs fa{};
    fa.U = U;
    fa.f = P->f;
    fa.v = P->v;
    fa.corr = P->p.k > 1 ? P->corr : nullptr;
    fa.S = P->S;
    fa.scale = P->d_scale;
    fa.s = P->d_s;
    fa.tw = P->d_twN;
    fa.w = P->d_w;
    fa.what = P->d_what;
    fa.tw2 = P->d_tw2;
    for (int j = 0; j < 8; ++j) fa.wk[j] = P->wk[j];
    fa.M = P->M;
    fa.N = P->N;
    fa.k = P->p.k;
    fa.ldS = P->ldS;
    fa.mxp = P->mxp;
    fa.Mp = P->Mp;
    fa.mx = P->mx;
    fa.my = P->my;
    fa.mz = P->mz;
    fa.ihx2 = P->ih2[0];
    fa.ihy2 = P->ih2[1];
    fa.ihz2 = P->ih2[2];
    fa.ta = P->ta;
    fa.kappa = P->p.kappa;
    fa.form = P->p.form == PINT_DIRECT ? 1 : 0;
    fa.ncorr = P->p.k > 1 ? P->p.k - 1 : 0;
    fa.var = P->var[0];
    fa.Rb = P->Rb;
    return fa;
}

SpaceArgs space_args(const pint_plan* P) {
    SpaceArgs sa{};
    sa.S = P->S;
    sa.nP = P->nP;
    sa.ldS = P->ldS;
    sa.mxp = P->mxp;
    sa.dim = P->dim;
    sa.mx = P->mx;
    sa.my = P->my;
    sa.mz = P->mz;
    sa.sigma = P->d_sigma;
    for (int i = 0; i < 3; ++i) {
        sa.mu[i] = P->d_mu[i];
        sa.twL[i] = P->d_twL[i];
        sa.logP[i] = P->logP[i];
        sa.chirp[i] = P->d_chirp[i];
        sa.bh[i] = P->d_bh[i];
        sa.twP[i] = P->d_twP[i];
        sa.ih2[i] = P->ih2[i];
    }
    sa.inv_factor = P->inv_factor;
    sa.var_rows = P->var[1];
    sa.var_cols = P->var[2];
    sa.var_tri = P->var[3];
    sa.mass = P->d_mass;
    return sa;
}

// A 1D batch instance whose time DFTs take plain FFTs of length N (power of
// two, at least 16; the Bluestein length is then 2N).
bool batch_pow2(const pint_plan* Q) { return is_pow2(Q->N) && Q->N >= 16 && (1 << Q->logPt) == 2 * Q->N; }

GenArgs gen_args(const pint_plan* P, double* U) {
    GenArgs ga{};
    ga.U = U;
    ga.Uw = U;
    ga.f = P->f;
    ga.v = P->v;
    ga.corr = P->p.k > 1 ? P->corr : nullptr;
    ga.Rb = P->Rb;
    ga.S = P->S;
    ga.scale = P->d_scale;
    ga.unscale = P->d_unscale;
    ga.s = P->d_s;
    ga.w = P->d_w;
    ga.chirp = P->d_chirpT;
    ga.bh = P->d_bhT;
    ga.twP = P->d_twPT;
    ga.partial = P->partial;
    ga.logP = P->logPt;
    ga.max_partials = P->max_partials;
    ga.M = P->M;
    ga.N = P->N;
    ga.k = P->p.k;
    ga.ldS = P->ldS;
    ga.mxp = P->mxp;
    ga.Mp = P->Mp;
    ga.mx = P->mx;
    ga.my = P->my;
    ga.mz = P->mz;
    ga.jmax = P->cq ? P->N - 1 : P->p.k;
    ga.ihx2 = P->ih2[0];
    ga.ihy2 = P->ih2[1];
    ga.ihz2 = P->ih2[2];
    ga.ta = P->ta;
    ga.kappa = P->p.kappa;
    ga.form = P->p.form == PINT_DIRECT ? 1 : 0;
    ga.ncorr = P->p.k > 1 ? P->p.k - 1 : 0;
    ga.an = P->d_an;
    ga.fem = P->fem ? 1 : 0;
    ga.pow2 = batch_pow2(P) ? 1 : 0;
    ga.twN = P->d_twN;
    if (ga.form == 0) {
        ga.wh = P->d_whT;
        ga.twh = P->d_twhT;
    }
    return ga;
}

InvArgs inv_args(const pint_plan* P, double* U, int form) {
    InvArgs ia{};
    ia.U = U;
    ia.S = P->S;
    ia.unscale = P->d_unscale;
    ia.tw = P->d_twN;
    ia.partial = P->partial;
    ia.M = P->M;
    ia.N = P->N;
    ia.ldS = P->ldS;
    ia.mx = P->mx;
    ia.mxp = P->mxp;
    ia.Mp = P->Mp;
    ia.form = form;
    return ia;
}

// One sweep of a plan on the general-length kernels (time axis not a power of
// two >= 8, or P1 elements).  With N a power of two >= 16 the inverse is the
// power-of-two kernel (same spectrum layout, same update and norm partials).
pint_status one_sweep_gn(pint_plan* P, double* U, double* norms_out, Profiler* prof) {
    const GenArgs ga = gen_args(P, U);
    PROF_BEGIN(prof, "residual_rhs");
    HIP_TRY(pint::launch_gn_resid(ga, P->st));
    PROF_END(prof);
    PROF_BEGIN(prof, "forward_tdft");
    HIP_TRY(pint::launch_gn_forward(ga, P->mixed, P->st));
    PROF_END(prof);
    const SpaceArgs sa = space_args(P);
    for (int i = 0; i < pint::space_pass_count(sa); ++i) {
        PROF_BEGIN(prof, pint::space_pass_name(sa, i));
        HIP_TRY(pint::launch_space_pass(sa, P->mixed, i, P->st));
        PROF_END(prof);
    }
    int nb = 0;
    PROF_BEGIN(prof, "inverse_tdft_update");
    if (ga.pow2)
        HIP_TRY(pint::launch_inverse(inv_args(P, U, ga.form), P->mixed, &nb, P->st));
    else
        HIP_TRY(pint::launch_gn_inverse(ga, P->mixed, &nb, P->st));
    PROF_END(prof);
    PROF_BEGIN(prof, "norm_reduce");
    HIP_TRY(pint::launch_norm_reduce(P->partial, nb, P->hd, norms_out, P->st));
    PROF_END(prof);
    return PINT_OK;
}

pint_status one_sweep(pint_plan* P, double* U, double* norms_out, Profiler* prof = nullptr) {
    if (prof) prof->cursor = 0;
    if (P->gn) return one_sweep_gn(P, U, norms_out, prof);
    FwdArgs fa = fwd_args(P, U);
    if (P->Sg) {
        // direct form, BDF-k: stored source spectrum + the k relaxation rows
        PROF_BEGIN(prof, "direct_rhs_spectrum");
        HIP_TRY(pint::launch_inject(fa, P->Sg, P->mixed, P->st));
        PROF_END(prof);
    } else {
        PROF_BEGIN(prof, P->cq ? "forward_cq_rhs_tfft" : "forward_rhs_tfft");
        HIP_TRY(pint::launch_forward(fa, P->mixed, P->cq, nullptr, P->st));
        PROF_END(prof);
    }

    const SpaceArgs sa = space_args(P);
    for (int i = 0; i < pint::space_pass_count(sa); ++i) {
        PROF_BEGIN(prof, pint::space_pass_name(sa, i));
        HIP_TRY(pint::launch_space_pass(sa, P->mixed, i, P->st));
        PROF_END(prof);
    }

    int nb = 0;
    PROF_BEGIN(prof, "inverse_tfft_update");
    HIP_TRY(pint::launch_inverse(inv_args(P, U, fa.form), P->mixed, &nb, P->st));
    PROF_END(prof);
    PROF_BEGIN(prof, "norm_reduce");
    HIP_TRY(pint::launch_norm_reduce(P->partial, nb, P->hd, norms_out, P->st));
    PROF_END(prof);
    return PINT_OK;
}

// Autotuner: times each kernel variant that launches a different kernel for
// this problem than the built-in choice, on the plan's own spectrum buffer and
// the caller's U (read only: the forward kernels read U and write the spectrum,
// the spatial passes work on the spectrum in place, so the values they leave
// behind are overwritten by the next sweep's first kernel), and keeps the
// fastest.  Knobs: the forward kernel (not used by direct-form BDF sweeps),
// rows per workgroup of the x sine pass, the column tile of the y/z passes,
// and the PCR/Thomas split of 1D tridiagonal solves.
struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    ~Timer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

template <typename F>
pint_status time_launches(pint_plan* P, Timer& t, int reps, F&& launch, float* ms) {
    HIP_TRY(launch());   // first launch: code object load, caches
    HIP_TRY(hipEventRecord(t.a, P->st));
    for (int r = 0; r < reps; ++r) HIP_TRY(launch());
    HIP_TRY(hipEventRecord(t.b, P->st));
    HIP_TRY(hipEventSynchronize(t.b));
    HIP_TRY(hipEventElapsedTime(ms, t.a, t.b));
    return PINT_OK;
}

pint_status tune_plan(pint_plan* P, const double* U, int reps) {
    Timer t;
    HIP_TRY(hipEventCreate(&t.a));
    HIP_TRY(hipEventCreate(&t.b));
    pint_status rc;
    // Fastest candidate value of knob k (cand[0] = 0, the built-in choice): the
    // candidates are timed in three interleaved rounds (so a clock ramp does not
    // favour the later ones) and each keeps its best round; another value
    // replaces the built-in one only when it is at least 3% faster.
    auto pick = [&](int k, const std::vector<int>& cand, auto&& launch) -> pint_status {
        std::vector<float> best(cand.size(), 0.0f);
        for (int round = 0; round < 3; ++round) {
            for (size_t c = 0; c < cand.size(); ++c) {
                P->var[k] = cand[c];
                float ms = 0.0f;
                pint_status r = time_launches(P, t, reps, launch, &ms);
                if (r != PINT_OK) {
                    P->var[k] = 0;
                    return r;
                }
                if (round == 0 || ms < best[c]) best[c] = ms;
            }
        }
        int arg = 0;
        float bt = best[0];
        for (size_t c = 1; c < cand.size(); ++c)
            if (best[c] < 0.97f * best[0] && best[c] < bt) {
                bt = best[c];
                arg = cand[c];
            }
        P->var[k] = arg;
        return PINT_OK;
    };
    if (!P->Sg && !P->gn) {
        std::vector<int> cand{0};
        const FwdArgs fa0 = fwd_args(P, U);
        for (int v = 1; v < pint::kFwdVariants; ++v)
            if (pint::forward_variant_distinct(fa0, P->mixed, P->cq, v)) cand.push_back(v);
        if (cand.size() > 1) {
            rc = pick(0, cand, [&]() { return pint::launch_forward(fwd_args(P, U), P->mixed, P->cq, nullptr, P->st); });
            if (rc != PINT_OK) return rc;
        }
    }
    const SpaceArgs sa0 = space_args(P);
    // the x pass is pass 0 (1D: the whole solve); the y/z passes are 1 .. count-2
    if (pint::rows_variant_distinct(sa0, P->mixed)) {
        rc = pick(1, {0, 1}, [&]() { return pint::launch_space_pass(space_args(P), P->mixed, 0, P->st); });
        if (rc != PINT_OK) return rc;
    }
    if (pint::cols_variant_distinct(sa0, P->mixed)) {
        rc = pick(2, {0, 1}, [&]() {
            const SpaceArgs sa = space_args(P);
            const int n = pint::space_pass_count(sa);
            for (int i = 1; i < n - 1; ++i) {
                const hipError_t e = pint::launch_space_pass(sa, P->mixed, i, P->st);
                if (e != hipSuccess) return e;
            }
            return hipSuccess;
        });
        if (rc != PINT_OK) return rc;
    }
    // knob 3 (1D: sine solve or PCR/Thomas) is not tuned: the choice changes the
    // accuracy of a sweep, not only its speed; pint_plan_set_variants pins it
    P->tuned = true;
    return PINT_OK;
}

}  // namespace

namespace pint {

// Sweeps until the chosen update norm is <= tol or max_sweeps is reached, with
// the host stop test after every sweep (the stopping rule of Sec. 4): the
// update norms of the sweep are copied to pinned host memory and the stream
// is synchronised.  Divergence guard: a non-finite update, or an update that
// grew in two consecutive sweeps to above the first update.  Allocates
// nothing.
pint_status solve_loop(pint_plan* P, double* U, double* upd, double* upd_l2T, int* sweeps) {
    int done = 0;
    double first = 0.0, prev2 = 0.0, prev1 = 0.0;
    pint_status result = PINT_NOT_CONVERGED;
    for (int m = 0; m < P->p.max_sweeps; ++m) {
        pint_status rc = one_sweep(P, U, P->norm_tmp);
        if (rc != PINT_OK) return rc;
        HIP_TRY(hipMemcpyAsync(P->h_norms, P->norm_tmp, 2 * sizeof(double), hipMemcpyDeviceToHost, P->st));
        HIP_TRY(hipStreamSynchronize(P->st));
        const double ninf = P->h_norms[0], nl2 = P->h_norms[1];
        if (upd) upd[m] = ninf;
        if (upd_l2T) upd_l2T[m] = nl2;
        done = m + 1;
        const double crit = P->p.norm == PINT_NORM_INF ? ninf : nl2;
        if (!std::isfinite(ninf) || !std::isfinite(nl2)) {
            result = fail(PINT_E_DIVERGED, "non-finite update in sweep " + std::to_string(m + 1));
            break;
        }
        if (m == 0) first = crit;
        if (crit <= P->p.tol) {
            result = PINT_OK;
            break;
        }
        if (m >= 2 && crit > prev1 && prev1 > prev2 && crit > first) {
            result = fail(PINT_E_DIVERGED, "update grew in two consecutive sweeps beyond the first update");
            break;
        }
        prev2 = prev1;
        prev1 = crit;
    }
    if (sweeps) *sweeps = done;
    return result;
}

pint_status set_error(pint_status s, const std::string& msg) { return fail(s, msg); }

// One WR sweep of the linearised system of a Newton step (eq. BDF-CQ-m-r-N-w)
// on W, residual form: W += P^{-1} (R - T_D W) with T_D the all-at-once
// operator of the scheme with zero history and the spatial operator
// A_h + diag(D); time DFTs of general length, PCR/Thomas per frequency.
pint_status nl_sweep(pint_plan* P, double* norms_out) {
    GenArgs ga = gen_args(P, P->nlW);
    ga.f = P->nlR - P->M;            // row q + 1 of f is row q of R
    ga.v = nullptr;
    ga.corr = nullptr;
    ga.ncorr = 0;
    ga.form = 0;
    ga.dvar = P->nlD;
    HIP_TRY(pint::launch_gn_resid(ga, P->st));
    HIP_TRY(pint::launch_gn_forward(ga, P->mixed, P->st));
    SpaceArgs sa = space_args(P);
    sa.dvar = P->nlD;
    HIP_TRY(pint::launch_space_pass(sa, P->mixed, 0, P->st));
    int nb = 0;
    HIP_TRY(pint::launch_gn_inverse(ga, P->mixed, &nb, P->st));
    HIP_TRY(pint::launch_norm_reduce(P->partial, nb, P->hd, norms_out, P->st));
    return PINT_OK;
}

pint_status fetch_norms(pint_plan* P) {
    HIP_TRY(hipMemcpyAsync(P->h_norms, P->norm_tmp, 2 * sizeof(double), hipMemcpyDeviceToHost, P->st));
    HIP_TRY(hipStreamSynchronize(P->st));
    return PINT_OK;
}

// Algorithm 3 on a bound 1D plan.
pint_status nonlinear_solve(pint_plan* P, double c3, double c1, double* U, int steps, double newton_tol,
                            int* inner, double* newton_upd, int* done) {
    if (done) *done = 0;
    HIP_TRY(pint::launch_fill(U, P->v, P->N, P->M, 0, P->st));   // U_0^n = v
    for (int l = 0; l < steps; ++l) {
        // time-averaged Jacobian g'(Ubar) and the Newton residual
        HIP_TRY(pint::launch_nl_mean_dg(U, P->nlD, P->N, P->M, c3, c1, P->st));
        GenArgs ga = gen_args(P, U);
        ga.form = 0;
        ga.nl = 1;
        ga.raw = 1;
        ga.c3 = c3;
        ga.c1 = c1;
        ga.Rb = P->nlR;
        HIP_TRY(pint::launch_gn_resid(ga, P->st));
        HIP_TRY(pint::launch_fill(P->nlW, nullptr, P->N, P->M, 1, P->st));   // W_{l,0} = 0
        int m = 0;
        bool ok = false;
        for (m = 1; m <= P->p.max_sweeps; ++m) {
            pint_status rc = nl_sweep(P, P->norm_tmp);
            if (rc != PINT_OK) return rc;
            if ((rc = fetch_norms(P)) != PINT_OK) return rc;
            const double upd = P->h_norms[0];
            if (!std::isfinite(upd)) return fail(PINT_E_DIVERGED, "non-finite inner update");
            if (upd < P->p.tol) {
                ok = true;
                break;
            }
        }
        if (inner) inner[l] = ok ? m : P->p.max_sweeps;
        int nb = 0;
        HIP_TRY(pint::launch_nl_axpy(U, P->nlW, P->partial, P->N, P->M, P->max_partials, &nb, P->st));
        HIP_TRY(pint::launch_norm_reduce(P->partial, nb, P->hd, P->norm_tmp, P->st));
        pint_status rc = fetch_norms(P);
        if (rc != PINT_OK) return rc;
        const double wn = P->h_norms[0];
        if (newton_upd) newton_upd[l] = wn;
        if (done) *done = l + 1;
        if (!std::isfinite(wn)) return fail(PINT_E_DIVERGED, "non-finite Newton update");
        if (!ok) return PINT_NOT_CONVERGED;
        if (wn <= newton_tol) return PINT_OK;
    }
    return PINT_NOT_CONVERGED;
}

// pint_solve on a workspace the caller names for this call only (the static
// scratch of the allocation-free entry point): the plan's own workspace
// attachment is set aside and restored afterwards, and the plan is left
// unbound (its bound tables lived in the borrowed workspace).  No autotuning
// (tuning creates timing events).  Allocates nothing.
pint_status solve_in_workspace(pint_plan* P, void* ws, size_t ws_cap, const double* v, const double* f,
                               const double* fder, double* U, double* upd, double* upd_l2T, int* sweeps) {
    if (!P || !U || !v) return fail(PINT_E_ARG, "plan, v and U must not be NULL");
    if (!P->inst.empty()) return fail(PINT_E_ARG, "batch plans are not supported here");
    if (P->ws_bytes > ws_cap)
        return fail(PINT_E_ARG, "the plan needs " + std::to_string(P->ws_bytes) + " bytes of workspace; the "
                                "static scratch holds " + std::to_string(ws_cap));
    void* keep = P->ws;
    attach_workspace(P, ws);
    pint_status rc = pint_bind(P, v, f, fder);
    if (rc == PINT_OK) rc = pint_init_iterate(P, U);
    if (rc == PINT_OK) rc = solve_loop(P, U, upd, upd_l2T, sweeps);
    if (keep) {
        attach_workspace(P, keep);
    } else {
        P->ws = nullptr;
        P->S = nullptr;
        P->corr = P->partial = P->norm_tmp = nullptr;
        P->Sg = nullptr;
    }
    P->bound = false;
    return rc;
}

}  // namespace pint

extern "C" {

pint_status pint_plan_create(pint_plan** plan, const pint_grid* grid, const pint_params* params, void* hip_stream) {
    if (!plan) return fail(PINT_E_ARG, "plan must not be NULL");
    *plan = nullptr;
    pint_status rc = validate(grid, params);
    if (rc != PINT_OK) return rc;
    pint_plan* P = new (std::nothrow) pint_plan();
    if (!P) return fail(PINT_E_NOMEM, "host allocation failed");
    rc = build_plan(P, grid, params, static_cast<hipStream_t>(hip_stream));
    if (rc != PINT_OK) {
        delete P;
        return rc;
    }
    *plan = P;
    return PINT_OK;
}

size_t pint_plan_workspace_bytes(const pint_plan* plan) {
    if (!plan) return 0;
    if (!plan->inst.empty()) return 0;
    return plan->ws_bytes;
}

pint_status pint_plan_set_workspace(pint_plan* P, void* dev_ptr, size_t bytes) {
    if (!P || !dev_ptr) return fail(PINT_E_ARG, "plan and workspace must not be NULL");
    if (!P->inst.empty()) return fail(PINT_E_ARG, "batch plans manage their own workspace");
    if (bytes < P->ws_bytes) return fail(PINT_E_ARG, "workspace too small");
    if ((reinterpret_cast<uintptr_t>(dev_ptr) & 255) != 0) return fail(PINT_E_ARG, "workspace must be 256-byte aligned");
    if (P->ws_owned && P->ws) {
        HIP_TRY(hipStreamSynchronize(P->st));
        HIP_TRY(hipFree(P->ws));
    }
    P->ws_owned = false;
    attach_workspace(P, dev_ptr);
    return PINT_OK;
}

pint_status pint_bind(pint_plan* P, const double* v, const double* f, const double* fder) {
    if (!P || !v) return fail(PINT_E_ARG, "plan and v must not be NULL");
    if (!P->inst.empty()) return fail(PINT_E_ARG, "batch plans bind their instances in pint_batch_solve");
    if (!P->ws) return fail(PINT_E_ARG, "no workspace: call pint_plan_set_workspace first");
    P->v = v;
    P->f = f;
    P->fder = fder;
    HIP_TRY(pint::launch_prep(v, f, P->p.k > 2 ? fder : nullptr, P->corr, P->d_an, P->d_blt, P->p.k, P->M, P->mx,
                              P->my, P->mz, P->ih2[0], P->ih2[1], P->ih2[2], P->st));
    if (P->Sg) {
        // spectrum of kappa^{q/N} G_q, the part of the direct-form right-hand side
        // that does not change between sweeps
        FwdArgs fa = fwd_args(P, nullptr);
        fa.form = 2;
        fa.S = P->Sg;
        HIP_TRY(pint::launch_forward(fa, P->mixed, false, nullptr, P->st));
    }
    P->bound = true;
    return PINT_OK;
}

pint_status pint_init_iterate(pint_plan* P, double* U) {
    if (!P || !U) return fail(PINT_E_ARG, "plan and U must not be NULL");
    if (!P->bound) return fail(PINT_E_ARG, "pint_bind must be called first");
    if (P->p.init == PINT_INIT_USER) return PINT_OK;
    HIP_TRY(pint::launch_fill(U, P->v, P->N, P->M, P->p.init == PINT_INIT_ZERO, P->st));
    return PINT_OK;
}

pint_status pint_sweeps(pint_plan* P, double* U, int nsweeps, double* dev_norms) {
    if (!P || !U || nsweeps < 0) return fail(PINT_E_ARG, "bad arguments to pint_sweeps");
    if (!P->bound) return fail(PINT_E_ARG, "pint_bind must be called first");
    for (int i = 0; i < nsweeps; ++i) {
        pint_status rc = one_sweep(P, U, dev_norms ? dev_norms + 2 * i : P->norm_tmp);
        if (rc != PINT_OK) return rc;
    }
    return PINT_OK;
}

int pint_profile_sweeps(pint_plan* P, double* U, int nsweeps, double* ms, const char** names, int max_slots) {
    if (!P || !U || nsweeps < 1 || !ms || max_slots < 1) {
        fail(PINT_E_ARG, "bad arguments to pint_profile_sweeps");
        return PINT_E_ARG;
    }
    if (!P->bound) {
        fail(PINT_E_ARG, "pint_bind must be called first");
        return PINT_E_ARG;
    }
    Profiler prof;
    prof.st = P->st;
    for (int i = 0; i < nsweeps; ++i) {
        pint_status rc = one_sweep(P, U, P->norm_tmp, &prof);
        if (rc != PINT_OK) return rc;
    }
    hipError_t e = hipStreamSynchronize(P->st);
    if (e != hipSuccess) {
        fail(PINT_E_HIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
        return PINT_E_HIP;
    }
    const int ns = (int)prof.names.size();
    for (int j = 0; j < max_slots; ++j) ms[j] = 0.0;
    for (size_t i = 0; i < prof.ev.size(); ++i) {
        float t = 0.0f;
        e = hipEventElapsedTime(&t, prof.ev[i].first, prof.ev[i].second);
        if (e != hipSuccess) {
            fail(PINT_E_HIP, std::string("hipEventElapsedTime: ") + hipGetErrorString(e));
            return PINT_E_HIP;
        }
        if (prof.slot[i] < max_slots) ms[prof.slot[i]] += t;
    }
    static thread_local std::vector<std::string> keep;
    keep = prof.names;
    for (int j = 0; j < ns && j < max_slots; ++j) {
        ms[j] /= nsweeps;
        if (names) names[j] = keep[j].c_str();
    }
    return ns;
}

pint_status pint_solve(pint_plan* P, const double* v, const double* f, const double* fder, double* U, double* upd,
                       double* upd_l2T, int* sweeps) {
    if (!P || !U) return fail(PINT_E_ARG, "plan and U must not be NULL");
    if (!P->inst.empty()) return fail(PINT_E_ARG, "use pint_batch_solve for batch plans");
    pint_status rc = pint_bind(P, v, f, fder);
    if (rc != PINT_OK) return rc;
    if ((rc = pint_init_iterate(P, U)) != PINT_OK) return rc;
    if (P->tune_reps > 0 && !P->tuned && (rc = tune_plan(P, U, P->tune_reps)) != PINT_OK) return rc;
    return pint::solve_loop(P, U, upd, upd_l2T, sweeps);
}

pint_status pint_solve_windows(pint_plan* P, int nwin, const double* v, const double* f, const double* fder,
                               double* U, double* upd, int* sweeps) {
    if (!P || !U || !v || nwin < 1) return fail(PINT_E_ARG, "bad arguments to pint_solve_windows");
    if (!P->inst.empty()) return fail(PINT_E_ARG, "batch plans are not supported here");
    const size_t N = P->N, M = P->M, kd = P->p.k > 2 ? P->p.k - 2 : 0;
    pint_status result = PINT_OK;
    for (int w = 0; w < nwin; ++w) {
        // window w starts from the last level of window w-1 (U_w[-1] stays untouched
        // while window w sweeps)
        const double* vw = w == 0 ? v : U + ((size_t)w * N - 1) * M;
        const double* fw = f ? f + (size_t)w * N * M : nullptr;
        const double* dw = (fder && kd > 0) ? fder + (size_t)w * kd * M : nullptr;
        int done = 0;
        const pint_status rc = pint_solve(P, vw, fw, dw, U + (size_t)w * N * M,
                                          upd ? upd + (size_t)w * P->p.max_sweeps : nullptr, nullptr, &done);
        if (sweeps) sweeps[w] = done;
        if (rc < 0) return rc;
        if (rc == PINT_NOT_CONVERGED) result = rc;
    }
    return result;
}

pint_status pint_sequential_solve(pint_plan* P, const double* v, const double* f, const double* fder, double* U) {
    if (!P || !U || !v) return fail(PINT_E_ARG, "plan, v and U must not be NULL");
    if (!P->inst.empty()) return fail(PINT_E_ARG, "batch plans are not supported here");
    if (P->mixed) return fail(PINT_E_UNSUPPORTED, "the sequential solver runs in FP64");
    if (P->fem) return fail(PINT_E_UNSUPPORTED, "the sequential solver is implemented for finite differences");
    pint_status rc = pint_bind(P, v, f, fder);
    if (rc != PINT_OK) return rc;
    GenArgs ga = gen_args(P, U);
    SpaceArgs sa = space_args(P);
    sa.nP = 1;
    sa.sigma = P->d_sigma_seq;
    sa.var_tri = 0;
    const int passes = pint::space_pass_count(sa);
    for (int n = 1; n <= P->N; ++n) {
        HIP_TRY(pint::launch_seq_rhs(ga, n, P->S, P->st));
        for (int i = 0; i < passes; ++i) HIP_TRY(pint::launch_space_pass(sa, false, i, P->st));
        HIP_TRY(pint::launch_seq_store(ga, n, P->S, P->st));
    }
    return PINT_OK;
}

pint_status pint_nonlinear_solve(pint_plan* P, double c3, double c1, const double* v, const double* f,
                                 const double* fder, double* U, int newton_steps, double newton_tol,
                                 int* inner_sweeps, double* newton_upd, int* steps_done) {
    if (!P || !U || !v) return fail(PINT_E_ARG, "plan, v and U must not be NULL");
    if (!P->inst.empty()) return fail(PINT_E_ARG, "batch plans are not supported here");
    if (P->dim != 1 || !P->nlW) return fail(PINT_E_UNSUPPORTED, "the semilinear solve is implemented for 1D grids");
    if (P->fem) return fail(PINT_E_UNSUPPORTED, "the semilinear solve is implemented for finite differences");
    if (newton_steps < 1 || !(newton_tol >= 0.0) || !std::isfinite(c3) || !std::isfinite(c1))
        return fail(PINT_E_ARG, "bad arguments to pint_nonlinear_solve");
    if (P->p.form != PINT_RESIDUAL || P->p.precision != PINT_FP64)
        return fail(PINT_E_UNSUPPORTED, "the semilinear solve runs FP64 residual-form sweeps");
    pint_status rc = pint_bind(P, v, f, fder);
    if (rc != PINT_OK) return rc;
    return pint::nonlinear_solve(P, c3, c1, U, newton_steps, newton_tol, inner_sweeps, newton_upd, steps_done);
}

pint_status pint_plan_set_autotune(pint_plan* P, int reps) {
    if (!P || reps < 0 || reps > 1000) return fail(PINT_E_ARG, "bad arguments to pint_plan_set_autotune");
    P->tune_reps = reps;
    return PINT_OK;
}

pint_status pint_plan_tune(pint_plan* P, const double* U, int reps) {
    if (!P || !U || reps < 1 || reps > 1000) return fail(PINT_E_ARG, "bad arguments to pint_plan_tune");
    if (!P->inst.empty()) return fail(PINT_E_ARG, "batch plans tune their instances in pint_batch_solve");
    if (!P->bound) return fail(PINT_E_ARG, "pint_bind must be called first");
    for (int k = 0; k < 4; ++k) P->var[k] = 0;
    return tune_plan(P, U, reps);
}

pint_status pint_plan_get_variants(const pint_plan* P, int instance, int* choices) {
    if (!P || !choices) return fail(PINT_E_ARG, "plan and choices must not be NULL");
    const pint_plan* Q = P;
    if (!P->inst.empty()) {
        if (instance < 0 || instance >= (int)P->inst.size()) return fail(PINT_E_ARG, "instance out of range");
        Q = P->inst[instance];
    } else if (instance != 0) {
        return fail(PINT_E_ARG, "instance must be 0 for a single plan");
    }
    for (int k = 0; k < 4; ++k) choices[k] = Q->var[k];
    return PINT_OK;
}

pint_status pint_plan_set_variants(pint_plan* P, int instance, const int* choices) {
    if (!P || !choices) return fail(PINT_E_ARG, "plan and choices must not be NULL");
    pint_plan* Q = P;
    if (!P->inst.empty()) {
        if (instance < 0 || instance >= (int)P->inst.size()) return fail(PINT_E_ARG, "instance out of range");
        Q = P->inst[instance];
    } else if (instance != 0) {
        return fail(PINT_E_ARG, "instance must be 0 for a single plan");
    }
    const int hi[4] = {pint::kFwdVariants - 1, 1, 1, 2};
    for (int k = 0; k < 4; ++k)
        if (choices[k] < 0 || choices[k] > hi[k]) return fail(PINT_E_ARG, "variant out of range");
    if (Q->fem && choices[3] != 0)
        return fail(PINT_E_UNSUPPORTED, "P1 elements take the sine solve (knob 3 must be 0)");
    for (int k = 0; k < 4; ++k) Q->var[k] = choices[k];
    Q->tuned = true;   // pinned choices are not re-tuned
    return PINT_OK;
}

pint_status pint_plan_destroy(pint_plan* P) {
    if (!P) return PINT_OK;
    if (P->st || true) (void)hipStreamSynchronize(P->st);
    delete P;
    return PINT_OK;
}

long long pint_plan_unknowns(const pint_plan* P) {
    if (!P) return 0;
    if (!P->inst.empty()) {
        long long s = 0;
        for (const pint_plan* q : P->inst) s += (long long)q->N * q->M;
        return s;
    }
    return (long long)P->N * P->M;
}

const char* pint_status_str(pint_status s) {
    switch (s) {
        case PINT_OK: return "PINT_OK";
        case PINT_NOT_CONVERGED: return "PINT_NOT_CONVERGED";
        case PINT_E_ARG: return "PINT_E_ARG";
        case PINT_E_UNSUPPORTED: return "PINT_E_UNSUPPORTED";
        case PINT_E_NOMEM: return "PINT_E_NOMEM";
        case PINT_E_HIP: return "PINT_E_HIP";
        case PINT_E_DIVERGED: return "PINT_E_DIVERGED";
    }
    return "PINT_UNKNOWN";
}

const char* pint_last_error(void) { return g_err.c_str(); }

pint_status pint_batch_plan_create(pint_plan** plan, int count, const pint_grid* grids, const pint_params* params,
                                   void* hip_stream) {
    if (!plan || count < 1 || !grids || !params) return fail(PINT_E_ARG, "bad arguments to pint_batch_plan_create");
    *plan = nullptr;
    for (int i = 0; i < count; ++i) {
        pint_status rc = validate(&grids[i], &params[i]);
        if (rc != PINT_OK) return fail(rc, "instance " + std::to_string(i) + ": " + g_err);
        if (params[i].space != PINT_SPACE_FD)
            return fail(PINT_E_UNSUPPORTED, "instance " + std::to_string(i) + ": batches take finite differences");
    }
    pint_plan* P = new (std::nothrow) pint_plan();
    if (!P) return fail(PINT_E_NOMEM, "host allocation failed");
    P->st = static_cast<hipStream_t>(hip_stream);
    auto bail = [&](pint_status rc) {
        delete P;
        return rc;
    };
    hipError_t e = hipGetDevice(&P->device);
    if (e != hipSuccess) return bail(fail(PINT_E_HIP, hipGetErrorString(e)));
    for (int i = 0; i < count; ++i) {
        pint_plan* Q = new (std::nothrow) pint_plan();
        if (!Q) return bail(fail(PINT_E_NOMEM, "host allocation failed"));
        P->inst.push_back(Q);
        pint_status rc = build_plan(Q, &grids[i], &params[i], P->st);
        if (rc == PINT_OK && Q->dim == 1) {
            // the batched 1D sweep solves each frequency by Thomas in place,
            // with the modified super-diagonal kept here
            Q->off_th = Q->ws_bytes;
            Q->ws_bytes += align256((size_t)Q->nP * Q->M * (Q->mixed ? 8 : 16));
        }
        if (rc == PINT_OK) rc = own_workspace(Q);
        if (rc != PINT_OK) return bail(fail(rc, "instance " + std::to_string(i) + ": " + g_err));
    }
    // batched 1D sweeps: descriptors [count], prefix tables (two of n+1
    // entries per class, one of n+1 per precision: at most 5 count + 2 in
    // all), norms [count][2]; DFT partials, one pair per DFT tile of every 1D
    // instance
    size_t ntile = 0;
    for (pint_plan* Q : P->inst)
        if (Q->dim == 1) {
            const int B = pint::batch_dft_slots(Q->mixed, batch_pow2(Q) ? Q->logPt - 1 : Q->logPt);
            ntile += ((size_t)Q->Mp + B - 1) / B;
        }
    P->b_int_off = align256((size_t)count * sizeof(pint::Batch1D));
    P->b_norm_off = P->b_int_off + align256((size_t)6 * (count + 1) * sizeof(int));
    P->b_bytes = P->b_norm_off + align256((size_t)count * 2 * sizeof(double));
    void* q = nullptr;
    if ((e = hipMalloc(&q, P->b_bytes)) != hipSuccess) return bail(fail(PINT_E_NOMEM, hipGetErrorString(e)));
    P->owned.push_back(q);
    P->d_bblk = q;
    if ((e = hipMalloc(&q, std::max<size_t>(ntile, 1) * 2 * sizeof(double))) != hipSuccess)
        return bail(fail(PINT_E_NOMEM, hipGetErrorString(e)));
    P->owned.push_back(q);
    P->d_bpart = static_cast<double*>(q);
    if ((e = hipHostMalloc(&P->h_bblk, P->b_bytes, hipHostMallocDefault)) != hipSuccess) {
        P->h_bblk = nullptr;
        return bail(fail(PINT_E_NOMEM, hipGetErrorString(e)));
    }
    *plan = P;
    return PINT_OK;
}

pint_status pint_batch_solve(pint_plan* P, const double* const* v, const double* const* f, const double* const* fder,
                             double* const* U, double* upd, int stride, int* sweeps) {
    if (!P || P->inst.empty() || !v || !U) return fail(PINT_E_ARG, "bad arguments to pint_batch_solve");
    const int count = (int)P->inst.size();
    for (int i = 0; i < count; ++i) {
        if (!v[i] || !U[i]) return fail(PINT_E_ARG, "instance " + std::to_string(i) + ": NULL v or U");
        if (upd && P->inst[i]->p.max_sweeps > stride)
            return fail(PINT_E_ARG, "instance " + std::to_string(i) + ": max_sweeps exceeds the upd stride");
    }
    pint_status result = PINT_OK;
    // 1D instances: bound and started here, then swept together: each sweep is
    // one launch per pass over all active instances of a (precision, time
    // Bluestein length) class, followed by the host stop test of every instance
    // (the rules of the single-problem solve); finished instances drop out
    struct Track {
        int i;
        int key;           // 128 mixed + 64 pow2 + logP: the class (the precisions apart)
        double first, prev1, prev2;
        bool active;
    };
    std::vector<Track> tr;
    for (int i = 0; i < count; ++i) {
        pint_plan* Q = P->inst[i];
        if (Q->dim != 1) continue;
        pint_status rc = pint_bind(Q, v[i], f ? f[i] : nullptr, fder ? fder[i] : nullptr);
        if (rc == PINT_OK) rc = pint_init_iterate(Q, U[i]);
        if (rc != PINT_OK) return fail(rc, "instance " + std::to_string(i) + ": " + g_err);
        if (sweeps) sweeps[i] = 0;
        tr.push_back({i, (Q->mixed ? 128 : 0) + (batch_pow2(Q) ? 64 : 0) + Q->logPt, 0.0, 0.0, 0.0, true});
    }
    std::stable_sort(tr.begin(), tr.end(), [](const Track& x, const Track& y) { return x.key < y.key; });
    char* hb = static_cast<char*>(P->h_bblk);
    char* db = static_cast<char*>(P->d_bblk);
    pint::Batch1D* hdesc = reinterpret_cast<pint::Batch1D*>(hb);
    int* hint = reinterpret_cast<int*>(hb + P->b_int_off);
    const double* hnorm = reinterpret_cast<const double*>(hb + P->b_norm_off);
    std::vector<pint::BatchLaunch> launches;
    std::vector<int> who;   // packed position -> index into tr
    struct ThomasLaunch {
        int d0, n, nwaves, i0;   // descriptors d0 .. d0+n-1, prefix table at int offset i0
        bool mixed;
    };
    std::vector<ThomasLaunch> thomas;
    for (int m = 0;; ++m) {
        // pack the active instances, class by class (all FP64 classes first)
        launches.clear();
        who.clear();
        thomas.clear();
        int nd = 0, ni = 0, npart = 0;
        for (size_t a = 0; a < tr.size();) {
            size_t e2 = a;
            while (e2 < tr.size() && tr[e2].key == tr[a].key) ++e2;
            pint::BatchLaunch L{};
            L.logP = tr[a].key & 63;
            L.pow2 = (tr[a].key & 64) != 0;
            L.mixed = tr[a].key >= 128;
            const int B = pint::batch_dft_slots(L.mixed, L.pow2 ? L.logP - 1 : L.logP);
            for (size_t t = a; t < e2; ++t)
                if (tr[t].active && P->inst[tr[t].i]->p.max_sweeps > m) L.N = std::max(L.N, P->inst[tr[t].i]->N);
            const int W = L.N > 0 ? pint::batch_resid_width(L.N) : 1;
            int* rs = hint + ni;
            int n = 0;
            rs[0] = 0;
            std::vector<int> ds{0};
            for (size_t t = a; t < e2; ++t) {
                pint_plan* Q = P->inst[tr[t].i];
                if (!tr[t].active || Q->p.max_sweeps <= m) continue;
                pint::Batch1D& b = hdesc[nd + n];
                b = pint::Batch1D{};
                b.ga = gen_args(Q, U[tr[t].i]);
                b.sigma = Q->d_sigma;
                b.thomas = Q->thomas;
                b.twN = Q->d_twN;
                b.ih2 = Q->ih2[0];
                b.hd = Q->hd;
                const int Wq = b.ga.wh ? pint::batch_hist_width(L.logP) : W;
                rs[n + 1] = rs[n] + (Q->M + Wq - 1) / Wq;
                ds.push_back(ds.back() + (Q->Mp + B - 1) / B);
                who.push_back((int)t);
                ++n;
            }
            if (n > 0) {
                std::copy(ds.begin(), ds.end(), rs + n + 1);
                L.descs = reinterpret_cast<const pint::Batch1D*>(db) + nd;
                L.res_start = reinterpret_cast<const int*>(db + P->b_int_off) + ni;
                L.dft_start = L.res_start + n + 1;
                L.part = P->d_bpart + 2 * (size_t)npart;
                L.norms = reinterpret_cast<double*>(db + P->b_norm_off) + 2 * nd;
                L.n = n;
                L.nres = rs[n];
                L.ndft = ds.back();
                launches.push_back(L);
                if (thomas.empty() || thomas.back().mixed != L.mixed) thomas.push_back({nd, 0, 0, 0, L.mixed});
                thomas.back().n += n;
                nd += n;
                ni += 2 * (n + 1);
                npart += ds.back();
            }
            a = e2;
        }
        if (nd == 0) break;
        // the Thomas pass: one launch per precision over its instances of every class
        for (ThomasLaunch& T : thomas) {
            T.i0 = ni;
            int* ts = hint + ni;
            ts[0] = 0;
            for (int k = 0; k < T.n; ++k) ts[k + 1] = ts[k] + (hdesc[T.d0 + k].ga.N / 2 + 1 + 63) / 64;
            T.nwaves = ts[T.n];
            ni += T.n + 1;
        }
        HIP_TRY(hipMemcpyAsync(db, hb, (size_t)nd * sizeof(pint::Batch1D), hipMemcpyHostToDevice, P->st));
        HIP_TRY(hipMemcpyAsync(db + P->b_int_off, hint, (size_t)ni * sizeof(int), hipMemcpyHostToDevice, P->st));
        for (const pint::BatchLaunch& L : launches) HIP_TRY(pint::launch_batch_forward(L, P->st));
        for (const ThomasLaunch& T : thomas)
            HIP_TRY(pint::launch_batch_thomas(reinterpret_cast<const pint::Batch1D*>(db) + T.d0,
                                              reinterpret_cast<const int*>(db + P->b_int_off) + T.i0, T.n,
                                              T.nwaves, T.mixed, P->st));
        for (const pint::BatchLaunch& L : launches) HIP_TRY(pint::launch_batch_inverse(L, P->st));
        HIP_TRY(hipMemcpyAsync(hb + P->b_norm_off, db + P->b_norm_off, (size_t)nd * 2 * sizeof(double),
                               hipMemcpyDeviceToHost, P->st));
        HIP_TRY(hipStreamSynchronize(P->st));   // also frees the stage for the next sweep
        for (int k = 0; k < nd; ++k) {
            Track& T = tr[who[k]];
            pint_plan* Q = P->inst[T.i];
            const double ninf = hnorm[2 * k], nl2 = hnorm[2 * k + 1];
            if (upd) upd[(size_t)T.i * stride + m] = ninf;
            if (sweeps) sweeps[T.i] = m + 1;
            const double crit = Q->p.norm == PINT_NORM_INF ? ninf : nl2;
            if (!std::isfinite(ninf) || !std::isfinite(nl2)) {
                result = fail(PINT_E_DIVERGED, "instance " + std::to_string(T.i) + ": non-finite update");
                T.active = false;
                continue;
            }
            if (m == 0) T.first = crit;
            if (crit <= Q->p.tol) {
                T.active = false;
                continue;
            }
            if (m >= 2 && crit > T.prev1 && T.prev1 > T.prev2 && crit > T.first) {
                result = fail(PINT_E_DIVERGED, "instance " + std::to_string(T.i) + ": update grew");
                T.active = false;
                continue;
            }
            T.prev2 = T.prev1;
            T.prev1 = crit;
            if (m + 1 >= Q->p.max_sweeps) {
                T.active = false;
                if (result == PINT_OK) result = PINT_NOT_CONVERGED;
            }
        }
    }
    for (int i = 0; i < count; ++i) {
        pint_plan* Q = P->inst[i];
        if (Q->dim == 1) continue;
        Q->tune_reps = P->tune_reps;
        int done = 0;
        const pint_status rc = pint_solve(Q, v[i], f ? f[i] : nullptr, fder ? fder[i] : nullptr, U[i],
                                          upd ? upd + (size_t)i * stride : nullptr, nullptr, &done);
        if (sweeps) sweeps[i] = done;
        if (rc == PINT_E_DIVERGED) {
            result = rc;
        } else if (rc == PINT_NOT_CONVERGED) {
            if (result == PINT_OK) result = rc;
        } else if (rc != PINT_OK) {
            return fail(rc, "instance " + std::to_string(i) + ": " + g_err);
        }
    }
    return result;
}

}  // extern "C"
