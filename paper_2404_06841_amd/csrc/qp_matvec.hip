// Stiffness product of the projection method on gfx950:
//
//   y_k = sum_{m in S} Ahat_m (P k).(P j) x_j,   j = rep(k - m),   k != 0,
//
// (eq. n-discrete: the column k_U with k_V -_N k_U = m is the representative of
// k - m in K_N^n; W = (P k_V).(P k_U) uses both representatives).  Matrix free:
// only the g modes are read; every W is recomputed.
#include "qp_device.h"

namespace qp {
namespace {

// One thread per output entry.  The neighbour's storage digits wrap mod N and
// its signed representative gives W = sum_t q_t j_t with q_t = (P k).p_t.
template <typename T, int ND, int EPI>
__global__ __launch_bounds__(kBlock) void k_matvec_generic(const Table *__restrict__ tab,
                                                           const cplx_t<T> *__restrict__ x,
                                                           void *__restrict__ yv,
                                                           const double2 *__restrict__ f,
                                                           const float *__restrict__ M32,
                                                           double *__restrict__ part,
                                                           State *__restrict__ st,
                                                           int *__restrict__ exec)
{
    if (EPI == EPI_ALPHA && (st->done || st->pause)) return;
    if (EPI == EPI_RESID && st->done) return;
    const int N = tab->N;
    const int d = tab->d;
    const int g = tab->g;
    const double inv_unit = (EPI == EPI_RESID) ? st->inv_unit : 1.0;
    int begin, end;
    chunk_of_block(tab, begin, end);
    double acc2[2] = {0.0, 0.0};
    for (int i = begin + threadIdx.x; i < end; i += kBlock) {
        int ib[ND];
        T q[ND];
        {
            int rest = i;
#pragma unroll
            for (int t = ND - 1; t >= 0; --t) {
                const int qt = div_n(tab, rest);
                ib[t] = rest - qt * N;
                rest = qt;
            }
            T pk[kMaxD];
#pragma unroll
            for (int l = 0; l < kMaxD; ++l) {
                T s = 0;
                if (l < d) {
#pragma unroll
                    for (int t = 0; t < ND; ++t) {
                        const int kt = (2 * ib[t] < N) ? ib[t] : ib[t] - N;
                        s += (T)tab->P[l][t] * (T)kt;
                    }
                }
                pk[l] = s;
            }
#pragma unroll
            for (int t = 0; t < ND; ++t) {
                T s = 0;
#pragma unroll
                for (int l = 0; l < kMaxD; ++l)
                    if (l < d) s += pk[l] * (T)tab->P[l][t];
                q[t] = s;
            }
        }
        T acc_re = 0, acc_im = 0;
        if (i != 0) {
            for (int r = 0; r < g; ++r) {
                int src = 0;
                T w = 0;
#pragma unroll
                for (int t = 0; t < ND; ++t) {
                    int jb = ib[t] - tab->modes[r][t];
                    jb += (jb < 0) ? N : 0;
                    jb -= (jb >= N) ? N : 0;
                    src = src * N + jb;
                    const int jt = (2 * jb < N) ? jb : jb - N;
                    w += q[t] * (T)jt;
                }
                const T cr = (T)tab->coef[r][0] * w;
                const T ci = (T)tab->coef[r][1] * w;
                const cplx_t<T> u = x[src];
                acc_re += cr * u.x - ci * u.y;
                acc_im += cr * u.y + ci * u.x;
            }
        }
        if (EPI == EPI_RESID) {
            // replaced residual of FP32-IR: (f' - Q x) / ||F'|| stored as float
            const double2 fv = f[i];
            const double rx = (i != 0) ? (fv.x - (double)acc_re) * inv_unit : 0.0;
            const double ry = (i != 0) ? (fv.y - (double)acc_im) * inv_unit : 0.0;
            const float2 o = make_float2((float)rx, (float)ry);
            static_cast<float2 *>(yv)[i] = o;
            acc2[0] += (double)M32[i] * ((double)o.x * (double)o.x + (double)o.y * (double)o.y);
            acc2[1] += rx * rx + ry * ry;
        } else {
            cplx_t<T> o;
            o.x = acc_re;
            o.y = acc_im;
            static_cast<cplx_t<T> *>(yv)[i] = o;
            if (EPI == EPI_ALPHA) {
                const cplx_t<T> xi = x[i];
                acc2[0] += (double)xi.x * (double)acc_re + (double)xi.y * (double)acc_im;
            }
        }
    }
    if (EPI == EPI_ALPHA) {
        double v[1] = {acc2[0]};
        store_partials<1>(v, part);
        if (exec && blockIdx.x == 0 && threadIdx.x == 0) *exec = 1;
    } else if (EPI == EPI_RESID) {
        store_partials<2>(acc2, part);
        if (exec && blockIdx.x == 0 && threadIdx.x == 0) *exec = 1;
    }
}

template <typename T, int EPI>
hipError_t dispatch(const Table *tab, const Table &ht, const void *x, void *y, const double *f,
                    const float *M32, double *part, State *st, int *exec, hipStream_t s)
{
    const dim3 grid(ht.nblocks), block(kBlock);
    auto X = static_cast<const cplx_t<T> *>(x);
    auto Fv = reinterpret_cast<const double2 *>(f);
    switch (ht.n) {
#define QP_CASE(NDIM)                                                                        \
    case NDIM:                                                                                \
        hipLaunchKernelGGL((k_matvec_generic<T, NDIM, EPI>), grid, block, 0, s, tab, X, y, Fv, \
                           M32, part, st, exec);                                              \
        break;
        QP_CASE(1) QP_CASE(2) QP_CASE(3) QP_CASE(4) QP_CASE(5) QP_CASE(6) QP_CASE(7) QP_CASE(8)
#undef QP_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_matvec(int prec, int epi, const Table *tab, const Table &ht, const void *x,
                         void *y, const double *f, const float *M32, const Parts &parts,
                         State *st, int *exec, hipStream_t s)
{
    if (prec == F64) {
        if (epi == EPI_NONE)
            return dispatch<double, EPI_NONE>(tab, ht, x, y, f, M32, parts.a, st, exec, s);
        if (epi == EPI_ALPHA)
            return dispatch<double, EPI_ALPHA>(tab, ht, x, y, f, M32, parts.a, st, exec, s);
        return dispatch<double, EPI_RESID>(tab, ht, x, y, f, M32, parts.b, st, exec, s);
    }
    if (epi == EPI_NONE) return dispatch<float, EPI_NONE>(tab, ht, x, y, f, M32, parts.a, st, exec, s);
    if (epi == EPI_ALPHA) return dispatch<float, EPI_ALPHA>(tab, ht, x, y, f, M32, parts.a, st, exec, s);
    return hipErrorInvalidValue;  // the replaced residual is always computed in FP64
}

}  // namespace qp
