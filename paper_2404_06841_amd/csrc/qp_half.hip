// Stiffness product on Hermitian half storage (real coefficient, odd N).
//
// For a real coefficient the Fourier coefficients satisfy Ahat_{-m} =
// conj(Ahat_m), and Q_{-k,-j} = conj(Q_{kj}) because W = (Pk).(Pj) is real
// (eq. n-discrete).  A vector with u_{-k} = conj(u_k) (the coefficients of a
// real function, Sec. 2.3) is therefore mapped to one with the same symmetry,
// and only one of each pair {k, -k} needs storing.  At odd N every k in K_N
// has its negative in K_N and k = -k only for k = 0.
//
// Half H: the k != 0 whose first nonzero component (axis order 1..n) is
// positive.  In the C(k) order the entries with zero digits on axes
// 1..t-1 and digit a_t in [1, (N-1)/2] form the contiguous index range
// [S_t, (N+1)/2 * S_t) with S_t = N^(n-t); the half layout stores k = 0 at
// position 0 and then these ranges for t = n, n-1, ..., 1, so index i of
// range t sits at position i - (S_t - 1)/2, and (D+1)/2 positions hold it all.
//
// One thread per stored output; the g neighbours k - m are read from the
// stored half, conjugated when rep(k - m) lies in -H.  Reads and writes (D+1)/2
// entries instead of D: 16 B per stored entry each way in FP64.
#include <algorithm>

#include "qp_device.h"

namespace qp {
namespace {

// DD, NN: d and n (the loops over them unroll); modes satisfy |m_t| < N/2,
// so rep(k_t - m_t) needs one compare-and-shift per axis.  W is
// (Pk).(Pk - Pm) - N sum_t c_t (Pk).p_t for the wrap c_t in {-1, 0, 1}.
template <int DD, int NN>
__global__ __launch_bounds__(kBlock) void k_matvec_half(const Table *__restrict__ tab,
                                                        const double2 *__restrict__ u,
                                                        double2 *__restrict__ y, int half)
{
    const int N = tab->N, g = tab->g;
    const int h = (N - 1) / 2;
    int topS = 1;  // N^(n-1)
    for (int t = 1; t < NN; ++t) topS *= N;
    for (int pos = blockIdx.x * blockDim.x + threadIdx.x; pos < half;
         pos += gridDim.x * blockDim.x) {
        if (pos == 0) {
            y[0] = make_double2(0.0, 0.0);
            continue;
        }
        // the range t holding this position: S = N^(n-t), the largest power
        // of N with 1 + (S - 1)/2 <= pos
        int S = 1;
        while (S < topS && 1 + (S * N - 1) / 2 <= pos) S *= N;
        int i = pos + (S - 1) / 2;
        int k[NN];
#pragma unroll
        for (int t = NN - 1; t >= 0; --t) {
            const int a = i % N;
            i /= N;
            k[t] = (a <= h) ? a : a - N;
        }
        double pk[DD], pkp[NN];  // P k and (P k).p_t
        double pk2 = 0.0;
#pragma unroll
        for (int l = 0; l < DD; ++l) {
            double s = 0.0;
#pragma unroll
            for (int t = 0; t < NN; ++t) s += tab->P[l][t] * (double)k[t];
            pk[l] = s;
            pk2 += s * s;
        }
#pragma unroll
        for (int t = 0; t < NN; ++t) {
            double s = 0.0;
#pragma unroll
            for (int l = 0; l < DD; ++l) s += pk[l] * tab->P[l][t];
            pkp[t] = s;
        }
        double acc_re = 0.0, acc_im = 0.0;
        for (int r = 0; r < g; ++r) {
            int j[NN];
            int first = NN;  // first axis with a nonzero component of rep(k - m)
            double wrap = 0.0;
#pragma unroll
            for (int t = NN - 1; t >= 0; --t) {
                int v = k[t] - tab->modes[r][t];
                if (v > h) {
                    v -= N;
                    wrap += pkp[t];
                } else if (v < -h) {
                    v += N;
                    wrap -= pkp[t];
                }
                j[t] = v;
                if (v != 0) first = t;
            }
            if (first == NN) continue;  // the zero mode: W = 0
            const bool neg = j[first] < 0;
            // stored index of j (or of -j) and its position
            int idx = 0, Sj = 1;
#pragma unroll
            for (int t = 0; t < NN; ++t) {
                int a = neg ? -j[t] : j[t];
                if (a < 0) a += N;
                idx = idx * N + a;
                if (t > first) Sj *= N;
            }
            double2 v = u[idx - (Sj - 1) / 2];
            if (neg) v.y = -v.y;
            double pkpm = 0.0;
#pragma unroll
            for (int l = 0; l < DD; ++l) pkpm += pk[l] * tab->Pm[r][l];
            // rep(k - m) = k - m + N c, c_t = -1 above the range, +1 below
            const double w = pk2 - pkpm - (double)N * wrap;
            const double cr = tab->coef[r][0] * w, ci = tab->coef[r][1] * w;
            acc_re += cr * v.x - ci * v.y;
            acc_im += cr * v.y + ci * v.x;
        }
        y[pos] = make_double2(acc_re, acc_im);
    }
}

}  // namespace

hipError_t launch_matvec_half(const Table *tab, const Table &ht, const void *u, void *y,
                              hipStream_t s)
{
    const int half = (ht.D + 1) / 2;
    const int grid = std::min((half + kBlock - 1) / kBlock, 65536);
    auto U = static_cast<const double2 *>(u);
    auto Y = static_cast<double2 *>(y);
    switch (ht.d * 16 + ht.n) {
#define QP_DN(DD, NN)                                                                         \
    case DD * 16 + NN:                                                                         \
        hipLaunchKernelGGL((k_matvec_half<DD, NN>), dim3(grid), dim3(kBlock), 0, s, tab, U, Y, \
                           half);                                                              \
        break;
#define QP_D(DD) QP_DN(DD, 1) QP_DN(DD, 2) QP_DN(DD, 3) QP_DN(DD, 4) QP_DN(DD, 5) QP_DN(DD, 6) \
        QP_DN(DD, 7) QP_DN(DD, 8)
        QP_D(1) QP_D(2) QP_D(3) QP_D(4)
#undef QP_D
#undef QP_DN
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace qp
