// gfx950 kernels of the sequential-in-time solver: the corrected BDF-k /
// CQ-BDF-k scheme stepped one time level after another (the cost model of
// Sec. 3.2, O(M N^2) history work for CQ and O(k M N) for BDF-k, plus one
// shifted spatial solve per step), the baseline the diagonalized sweep is
// compared with.  Step n solves
//   (omega_0 tau^{-alpha} + A_h) U^n = fbar_n + tau^{-alpha} (omega_0 v - sum_{j=1..n} omega_j (U^{n-j} - v)),
// with U^0 = v, by the same spatial passes as a sweep, on one complex plane
// of the spectrum buffer with zero imaginary part.
#include "pint_device.h"

namespace pint {
namespace {

constexpr int kSeqNT = 256;

// Right-hand side of step n (1-based) into plane slot order; padding slots 0.
__global__ __launch_bounds__(kSeqNT) void k_seq_rhs(GenArgs a, int n, double2* __restrict__ plane) {
    const int slot = blockIdx.x * kSeqNT + threadIdx.x;
    if (slot >= a.Mp) return;
    const int d = slot_dof(slot, a.mx, a.mxp, a.Mp);
    double r = 0.0;
    if (d >= 0) {
        const size_t M = a.M;
        const double vd = a.v[d];
        double h = a.w[0] * vd;
        const int top = n < a.jmax ? n : a.jmax;   // omega_j = 0 beyond jmax; U^0 - v = 0
        for (int j = 1; j <= top && j < n; ++j) h -= a.w[j] * (a.U[(size_t)(n - j - 1) * M + d] - vd);
        r = a.ta * h;
        if (a.f) r += a.f[(size_t)n * M + d];
        if (n - 1 < a.ncorr) r += a.corr[(size_t)(n - 1) * M + d];
    }
    plane[slot] = make_double2(r, 0.0);
}

// U^n (row n-1) from the solved plane.
__global__ __launch_bounds__(kSeqNT) void k_seq_store(GenArgs a, int n, const double2* __restrict__ plane) {
    const int d = blockIdx.x * kSeqNT + threadIdx.x;
    if (d >= a.M) return;
    const int slot = (d / a.mx) * a.mxp + d % a.mx;
    a.Uw[(size_t)(n - 1) * a.M + d] = plane[slot].x;
}

}  // namespace

hipError_t launch_seq_rhs(const GenArgs& a, int n, void* plane, hipStream_t st) {
    PINT_LAUNCH(k_seq_rhs, dim3((a.Mp + kSeqNT - 1) / kSeqNT), dim3(kSeqNT), 0, st, a, n,
                reinterpret_cast<double2*>(plane));
    return hipGetLastError();
}

hipError_t launch_seq_store(const GenArgs& a, int n, const void* plane, hipStream_t st) {
    PINT_LAUNCH(k_seq_store, dim3((a.M + kSeqNT - 1) / kSeqNT), dim3(kSeqNT), 0, st, a, n,
                reinterpret_cast<const double2*>(plane));
    return hipGetLastError();
}

}  // namespace pint
