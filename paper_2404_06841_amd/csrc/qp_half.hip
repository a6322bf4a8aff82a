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

__global__ __launch_bounds__(kBlock) void k_matvec_half(const Table *__restrict__ tab,
                                                        const double2 *__restrict__ u,
                                                        double2 *__restrict__ y, int half)
{
    const int n = tab->n, N = tab->N, d = tab->d, g = tab->g;
    const int h = (N - 1) / 2;
    for (int pos = blockIdx.x * blockDim.x + threadIdx.x; pos < half;
         pos += gridDim.x * blockDim.x) {
        if (pos == 0) {
            y[0] = make_double2(0.0, 0.0);
            continue;
        }
        // the range t holding this position: S = N^(n-t), the largest power
        // of N with 1 + (S - 1)/2 <= pos
        int S = 1;
        while (S * N <= tab->D / N && 1 + (S * N - 1) / 2 <= pos) S *= N;
        int i = pos + (S - 1) / 2;
        int k[kMaxN];
        for (int t = n - 1; t >= 0; --t) {
            const int a = i % N;
            i /= N;
            k[t] = (a <= h) ? a : a - N;
        }
        double pk[kMaxD];
        for (int l = 0; l < d; ++l) {
            double s = 0.0;
            for (int t = 0; t < n; ++t) s += tab->P[l][t] * (double)k[t];
            pk[l] = s;
        }
        double acc_re = 0.0, acc_im = 0.0;
        for (int r = 0; r < g; ++r) {
            int j[kMaxN];
            int first = -1;  // first axis with a nonzero component of rep(k - m)
            for (int t = 0; t < n; ++t) {
                const int v = k[t] - tab->modes[r][t];
                const int w = ((v + h) % N + N) % N - h;
                j[t] = w;
                if (first < 0 && w != 0) first = t;
            }
            if (first < 0) continue;  // the zero mode: W = 0
            const bool neg = j[first] < 0;
            // stored index of j (or of -j) and its position
            int idx = 0;
            for (int t = 0; t < n; ++t) {
                int a = neg ? -j[t] : j[t];
                if (a < 0) a += N;
                idx = idx * N + a;
            }
            int Sj = 1;
            for (int t = first + 1; t < n; ++t) Sj *= N;
            double2 v = u[idx - (Sj - 1) / 2];
            if (neg) v.y = -v.y;
            double w = 0.0;
            for (int l = 0; l < d; ++l) {
                double pj = 0.0;
                for (int t = 0; t < n; ++t) pj += tab->P[l][t] * (double)j[t];
                w += pk[l] * pj;
            }
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
    hipLaunchKernelGGL(k_matvec_half, dim3(grid), dim3(kBlock), 0, s, tab,
                       static_cast<const double2 *>(u), static_cast<double2 *>(y), half);
    return hipGetLastError();
}

}  // namespace qp
