// The compressed stiffness matrix of Alg. 1 (the paper's stored format) and
// its product, kept as a comparison for the matrix-free product.
//
// Alg. 1 stores Q = A o W as triples (i, j, Q_ij): for the row k_V (storage
// index i) and each coefficient mode m, the column is k_U = rep(k_V - m)
// (storage index j), A_ij = Ahat_m and W_ij = (P k_V).(P k_U) (for a
// diagonal coefficient, App. D: sum_l Ahat^l_m (P k_V)_l (P k_U)_l).  Here
// the triples are ordered mode-major: the entry of row i for the r-th mode
// (table order) is e = r D + i, so the product's threads (one per row) read
// consecutive entries; an entry whose value is zero (the zero row, the zero
// column, an exactly vanishing weight) keeps its slot with value 0.  Every
// value is computed in FP64 from the integer indices, with no per-unit
// tables.
#include <algorithm>

#include "qp_device.h"

namespace qp {
namespace {

__device__ __forceinline__ int signed_from(int b, int N) { return (2 * b < N) ? b : b - N; }

__global__ __launch_bounds__(kBlock) void k_coo_build(const Table *__restrict__ tab,
                                                      int32_t *__restrict__ rows,
                                                      int32_t *__restrict__ cols,
                                                      double2 *__restrict__ vals)
{
    const int N = tab->N, n = tab->n, d = tab->d, g = tab->g;
    const long long total = (long long)tab->D * g;
    const long long D = tab->D;
    for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < total;
         e += (long long)gridDim.x * kBlock) {
        const int r = (int)(e / D);
        const int i = (int)(e - (long long)r * D);
        int kv[kMaxN], ku[kMaxN];
        int rest = i;
        for (int t = n - 1; t >= 0; --t) {
            const int q = div_n(tab, rest);
            kv[t] = signed_from(rest - q * N, N);
            rest = q;
        }
        int j = 0;
        bool zero_row = true;
        for (int t = 0; t < n; ++t) {
            zero_row = zero_row && kv[t] == 0;
            int b = kv[t] - tab->modes[r][t];  // k_V - m, reduced to [0, N)
            b %= N;
            b += (b < 0) ? N : 0;
            ku[t] = signed_from(b, N);
            j = j * N + b;
        }
        double pv[kMaxD], pu[kMaxD];
        for (int l = 0; l < d; ++l) {
            double a = 0.0, b = 0.0;
            for (int t = 0; t < n; ++t) {
                a += tab->P[l][t] * (double)kv[t];
                b += tab->P[l][t] * (double)ku[t];
            }
            pv[l] = a;
            pu[l] = b;
        }
        double qr = 0.0, qi = 0.0;
        if (!zero_row) {
            if (tab->aniso) {
                for (int l = 0; l < d; ++l) {
                    const double w = pv[l] * pu[l];
                    qr += tab->coefl[r][l][0] * w;
                    qi += tab->coefl[r][l][1] * w;
                }
            } else {
                double w = 0.0;
                for (int l = 0; l < d; ++l) w += pv[l] * pu[l];
                qr = tab->coef[r][0] * w;
                qi = tab->coef[r][1] * w;
            }
        }
        rows[e] = i;
        cols[e] = j;
        vals[e] = make_double2(qr, qi);
    }
}

// y_i = sum over row i's g entries of Q_ij x_j (one thread per row, which
// reads entries i, D + i, 2 D + i, ...; the row index is implicit).
__global__ __launch_bounds__(kBlock) void k_coo_matvec(int D, int g,
                                                       const int32_t *__restrict__ cols,
                                                       const double2 *__restrict__ vals,
                                                       const double2 *__restrict__ x,
                                                       double2 *__restrict__ y)
{
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < D; i += gridDim.x * kBlock) {
        double ar = 0.0, ai = 0.0;
        for (int r = 0; r < g; ++r) {
            const size_t e = (size_t)r * D + i;
            const double2 q = vals[e];
            const double2 u = x[cols[e]];
            ar += q.x * u.x - q.y * u.y;
            ai += q.x * u.y + q.y * u.x;
        }
        y[i] = make_double2(ar, ai);
    }
}

}  // namespace

hipError_t launch_coo_build(const Table *tab, const Table &ht, int32_t *rows, int32_t *cols,
                            double *vals, hipStream_t s)
{
    const long long total = (long long)ht.D * ht.g;
    const int grid = (int)std::min<long long>(8192, (total + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_coo_build, dim3(grid), dim3(kBlock), 0, s, tab, rows, cols,
                       reinterpret_cast<double2 *>(vals));
    return hipGetLastError();
}

hipError_t launch_coo_matvec(const Table &ht, const int32_t *cols, const double *vals,
                             const double *x, double *y, hipStream_t s)
{
    const int grid = (int)std::min<long long>(8192, ((long long)ht.D + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_coo_matvec, dim3(grid), dim3(kBlock), 0, s, ht.D, ht.g, cols,
                       reinterpret_cast<const double2 *>(vals), reinterpret_cast<const double2 *>(x),
                       reinterpret_cast<double2 *>(y));
    return hipGetLastError();
}

}  // namespace qp
