// C-PCG (Alg. 2) vector steps and the FP32 refinement steps, for gfx950.
//
// One PCG iteration j is three launches on one stream:
//   stiffness product   q = Q h, partial sums of Re(h^H q)            (parts.a)
//   update              alpha = rz / (Q h, h); U += alpha h; r -= alpha q;
//                       partial sums of (r, M r) and ||r||^2          (parts.b)
//   direction           beta = (r, M r)_new / rz; h = M r + beta h
// z = M r is never stored; it is recomputed from r and the diagonal M.
// The scalars stay on the device; the host only polls `done`.
//
// FP32-IR runs the same loop with float vectors (entries scaled by 1/||F'||)
// and FP64 scalars and dot products.  Whenever the float residual has dropped
// by delta since the last replacement (or reached the tolerance), the float
// iterations pause; the host then queues a replacement: the float increment
// is folded into the FP64 solution X, the FP64 residual F' - Q X replaces r,
// convergence is decided on that true residual, and the iteration continues
// with the same search direction.
#include "qp_device.h"

namespace qp {
namespace {

template <typename T>
__global__ __launch_bounds__(kBlock) void k_pcg_init(const Table *__restrict__ tab,
                                                     const double2 *__restrict__ f,
                                                     double2 *__restrict__ X64,
                                                     cplx_t<T> *__restrict__ U,
                                                     cplx_t<T> *__restrict__ r,
                                                     cplx_t<T> *__restrict__ h,
                                                     const T *__restrict__ M,
                                                     double *__restrict__ part,
                                                     const State *__restrict__ st)
{
    const double scale = (sizeof(T) == 4) ? st->inv_unit : 1.0;
    int begin, end;
    chunk_of_block(tab, begin, end);
    double acc[2] = {0.0, 0.0};
    for (int i = begin + threadIdx.x; i < end; i += kBlock) {
        const double2 fv = f[i];
        cplx_t<T> rv, hv, zero;
        rv.x = (i != 0) ? (T)(fv.x * scale) : (T)0;
        rv.y = (i != 0) ? (T)(fv.y * scale) : (T)0;
        const T m = M[i];
        hv.x = m * rv.x;
        hv.y = m * rv.y;
        zero.x = 0;
        zero.y = 0;
        U[i] = zero;
        r[i] = rv;
        h[i] = hv;
        if (X64) X64[i] = make_double2(0.0, 0.0);
        const double n2 = (double)rv.x * (double)rv.x + (double)rv.y * (double)rv.y;
        acc[0] += (double)m * n2;
        acc[1] += n2;
    }
    store_partials<2>(acc, part);
}

// One workgroup: start the state from the init partials.
__global__ __launch_bounds__(kBlock) void k_pcg_start(int is_ir, double tol, double delta,
                                                      int maxit, const double *__restrict__ part,
                                                      int nb, State *__restrict__ st)
{
    double v[2];
    load_totals<2>(part, nb, v);
    if (threadIdx.x != 0) return;
    const double rz = v[0], rr = v[1];
    st->rz[0] = rz;
    st->rz[1] = rz;
    st->rr = rr;
    st->iters = 0;
    st->replacements = 0;
    st->maxit = maxit;
    st->pause = 0;
    st->alpha = st->beta = st->hq = 0.0;
    if (is_ir) {
        st->thresh = tol * tol;  // float residual is scaled to ||r_0|| = 1
        st->delta2 = delta * delta;
        st->rr_last = rr;
    } else {
        st->rr0 = rr;
        st->thresh = tol * tol * rr;
        st->delta2 = 0.0;
        st->rr_last = rr;
    }
    if (!finite(rr) || !finite(rz)) {
        st->status = QP_ENONFINITE;
        st->done = 1;
    } else if (rr == 0.0 || (is_ir && st->rr0 == 0.0)) {
        st->status = QP_OK;
        st->done = 1;
    } else {
        st->status = QP_OK;
        st->done = 0;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_pcg_update(int j, const Table *__restrict__ tab,
                                                       cplx_t<T> *__restrict__ U,
                                                       cplx_t<T> *__restrict__ r,
                                                       const cplx_t<T> *__restrict__ h,
                                                       const cplx_t<T> *__restrict__ q,
                                                       const T *__restrict__ M,
                                                       const double *__restrict__ part_in,
                                                       double *__restrict__ part_out,
                                                       State *__restrict__ st)
{
    if (st->done || st->pause) return;
    double hq[1];
    load_totals<1>(part_in, tab->nb_mv, hq);  // partials of the stiffness product
    if (!(hq[0] > 0.0)) {
        // (Q h, h) <= 0: Q is not positive definite on this Krylov space
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->hq = hq[0];
            st->status = finite(hq[0]) ? QP_ENOTSPD : QP_ENONFINITE;
            st->done = 1;
        }
        return;
    }
    const double alpha = st->rz[j & 1] / hq[0];
    const T a = (T)alpha;
    int begin, end;
    chunk_of_block(tab, begin, end);
    double acc[2] = {0.0, 0.0};
    for (int i = begin + threadIdx.x; i < end; i += kBlock) {
        cplx_t<T> u = U[i];
        cplx_t<T> rv = r[i];
        const cplx_t<T> hv = h[i];
        const cplx_t<T> qv = q[i];
        u.x += a * hv.x;
        u.y += a * hv.y;
        rv.x -= a * qv.x;
        rv.y -= a * qv.y;
        U[i] = u;
        r[i] = rv;
        const double n2 = (double)rv.x * (double)rv.x + (double)rv.y * (double)rv.y;
        acc[0] += (double)M[i] * n2;
        acc[1] += n2;
    }
    store_partials<2>(acc, part_out);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->alpha = alpha;
        st->hq = hq[0];
        st->iters = st->iters + 1;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_pcg_direction(int j, int is_ir,
                                                          const Table *__restrict__ tab,
                                                          const cplx_t<T> *__restrict__ r,
                                                          cplx_t<T> *__restrict__ h,
                                                          const T *__restrict__ M,
                                                          const double *__restrict__ part_in,
                                                          State *__restrict__ st)
{
    if (st->done) return;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    const double rz_old = st->rz[j & 1];
    if (st->pause) {
        // carry the last rz forward so iteration j+1 finds it in its slot
        if (lead) st->rz[(j + 1) & 1] = rz_old;
        return;
    }
    double v[2];
    load_totals<2>(part_in, gridDim.x, v);
    const double rz_new = v[0], rr = v[1];
    if (!finite(rr) || !finite(rz_new)) {
        if (lead) {
            st->status = QP_ENONFINITE;
            st->done = 1;
        }
        return;
    }
    if (is_ir) {
        if (rr <= fmax(st->thresh, st->delta2 * st->rr_last)) {
            if (lead) {
                st->rr = rr;
                st->pause = 1;
                st->rz[(j + 1) & 1] = rz_old;
            }
            return;
        }
    } else {
        const bool conv = rr <= st->thresh;
        const bool limit = st->iters >= st->maxit;  // iters counts this update
        if (conv || limit) {
            if (lead) {
                st->rr = rr;
                st->status = conv ? QP_OK : QP_ENOCONV;
                st->done = 1;
            }
            return;
        }
    }
    const double beta = rz_new / rz_old;
    const T b = (T)beta;
    int begin, end;
    chunk_of_block(tab, begin, end);
    for (int i = begin + threadIdx.x; i < end; i += kBlock) {
        const cplx_t<T> rv = r[i];
        const T m = M[i];
        cplx_t<T> hv = h[i];
        hv.x = m * rv.x + b * hv.x;
        hv.y = m * rv.y + b * hv.y;
        h[i] = hv;
    }
    if (lead) {
        st->rr = rr;
        st->beta = beta;
        st->rz[(j + 1) & 1] = rz_new;
    }
}

// ||f'||^2 partials (FP32-IR unit).
__global__ __launch_bounds__(kBlock) void k_norm2(const Table *__restrict__ tab,
                                                  const double2 *__restrict__ f,
                                                  double *__restrict__ part)
{
    int begin, end;
    chunk_of_block(tab, begin, end);
    double acc[1] = {0.0};
    for (int i = begin + threadIdx.x; i < end; i += kBlock) {
        if (i == 0) continue;
        const double2 v = f[i];
        acc[0] += v.x * v.x + v.y * v.y;
    }
    store_partials<1>(acc, part);
}

__global__ __launch_bounds__(kBlock) void k_ir_unit(const double *__restrict__ part, int nb,
                                                    State *__restrict__ st)
{
    double v[1];
    load_totals<1>(part, nb, v);
    if (threadIdx.x != 0) return;
    st->rr0 = v[0];
    st->unit = sqrt(v[0]);
    st->inv_unit = (v[0] > 0.0 && finite(v[0])) ? 1.0 / sqrt(v[0]) : 0.0;
}

__global__ __launch_bounds__(kBlock) void k_ir_fold(const Table *__restrict__ tab,
                                                    double2 *__restrict__ X,
                                                    float2 *__restrict__ x,
                                                    const State *__restrict__ st)
{
    if (st->done) return;
    const double unit = st->unit;
    int begin, end;
    chunk_of_block(tab, begin, end);
    for (int i = begin + threadIdx.x; i < end; i += kBlock) {
        double2 a = X[i];
        const float2 e = x[i];
        a.x += unit * (double)e.x;
        a.y += unit * (double)e.y;
        X[i] = a;
        x[i] = make_float2(0.f, 0.f);
    }
}

__global__ __launch_bounds__(kBlock) void k_ir_direction(int j, const Table *__restrict__ tab,
                                                         const float2 *__restrict__ r,
                                                         float2 *__restrict__ h,
                                                         const float *__restrict__ M,
                                                         const double *__restrict__ part_in,
                                                         State *__restrict__ st)
{
    if (st->done) return;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    double v[2];
    load_totals<2>(part_in, tab->nb_mv, v);  // partials of the FP64 residual product
    const double rz_new = v[0], rr = v[1];  // true residual, scaled by 1/unit
    if (!finite(rr) || !finite(rz_new)) {
        if (lead) {
            st->status = QP_ENONFINITE;
            st->done = 1;
        }
        return;
    }
    if (rr <= st->thresh) {
        if (lead) {
            st->rr = rr;
            st->status = QP_OK;
            st->done = 1;
            st->replacements = st->replacements + 1;
        }
        return;
    }
    const double beta = rz_new / st->rz[j & 1];
    const float b = (float)beta;
    int begin, end;
    chunk_of_block(tab, begin, end);
    for (int i = begin + threadIdx.x; i < end; i += kBlock) {
        const float2 rv = r[i];
        const float m = M[i];
        float2 hv = h[i];
        hv.x = m * rv.x + b * hv.x;
        hv.y = m * rv.y + b * hv.y;
        h[i] = hv;
    }
    if (lead) {
        st->rr = rr;
        st->rr_last = rr;
        st->beta = beta;
        st->rz[(j + 1) & 1] = rz_new;
        st->pause = 0;
        st->replacements = st->replacements + 1;
    }
}

__global__ void k_state_reset(State *st)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->rz[0] = st->rz[1] = 0.0;
        st->alpha = st->beta = st->hq = 0.0;
        st->rr = st->rr0 = st->thresh = st->delta2 = st->rr_last = 0.0;
        st->unit = 1.0;
        st->inv_unit = 1.0;
        st->iters = 0;
        st->replacements = 0;
        st->done = 0;
        st->pause = 0;
        st->status = 0;
        st->maxit = 0;
    }
}

}  // namespace

hipError_t launch_pcg_init(int prec, const Table *tab, const Table &ht, const double *f,
                           double *X64, void *U, void *r, void *h, const void *M,
                           const Parts &parts, State *st, hipStream_t s)
{
    const dim3 grid(ht.nblocks), block(kBlock);
    auto F = reinterpret_cast<const double2 *>(f);
    auto X = reinterpret_cast<double2 *>(X64);
    if (prec == F64)
        hipLaunchKernelGGL(k_pcg_init<double>, grid, block, 0, s, tab, F, X, (double2 *)U,
                           (double2 *)r, (double2 *)h, (const double *)M, parts.b, st);
    else
        hipLaunchKernelGGL(k_pcg_init<float>, grid, block, 0, s, tab, F, X, (float2 *)U,
                           (float2 *)r, (float2 *)h, (const float *)M, parts.b, st);
    return hipGetLastError();
}

hipError_t launch_pcg_start(int prec, const Table &ht, double tol, double delta, int maxit,
                            const Parts &parts, State *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_pcg_start, dim3(1), dim3(kBlock), 0, s, prec == F32 ? 1 : 0, tol, delta,
                       maxit, (const double *)parts.b, ht.nblocks, st);
    return hipGetLastError();
}

hipError_t launch_pcg_update(int prec, int j, const Table *tab, const Table &ht, void *U, void *r,
                             const void *h, const void *q, const void *M, const Parts &parts,
                             State *st, hipStream_t s)
{
    const dim3 grid(ht.nblocks), block(kBlock);
    if (prec == F64)
        hipLaunchKernelGGL(k_pcg_update<double>, grid, block, 0, s, j, tab, (double2 *)U,
                           (double2 *)r, (const double2 *)h, (const double2 *)q, (const double *)M,
                           (const double *)parts.a, parts.b, st);
    else
        hipLaunchKernelGGL(k_pcg_update<float>, grid, block, 0, s, j, tab, (float2 *)U, (float2 *)r,
                           (const float2 *)h, (const float2 *)q, (const float *)M,
                           (const double *)parts.a, parts.b, st);
    return hipGetLastError();
}

hipError_t launch_pcg_direction(int prec, int j, const Table *tab, const Table &ht, const void *r,
                                void *h, const void *M, const Parts &parts, State *st,
                                hipStream_t s)
{
    const dim3 grid(ht.nblocks), block(kBlock);
    if (prec == F64)
        hipLaunchKernelGGL(k_pcg_direction<double>, grid, block, 0, s, j, 0, tab,
                           (const double2 *)r, (double2 *)h, (const double *)M,
                           (const double *)parts.b, st);
    else
        hipLaunchKernelGGL(k_pcg_direction<float>, grid, block, 0, s, j, 1, tab, (const float2 *)r,
                           (float2 *)h, (const float *)M, (const double *)parts.b, st);
    return hipGetLastError();
}

hipError_t launch_ir_unit(const Table *tab, const Table &ht, const double *f, const Parts &parts,
                          State *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_norm2, dim3(ht.nblocks), dim3(kBlock), 0, s, tab,
                       reinterpret_cast<const double2 *>(f), parts.c);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ir_unit, dim3(1), dim3(kBlock), 0, s, (const double *)parts.c, ht.nblocks,
                       st);
    return hipGetLastError();
}

hipError_t launch_ir_fold(const Table *tab, const Table &ht, double *X, float *x, State *st,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_ir_fold, dim3(ht.nblocks), dim3(kBlock), 0, s, tab,
                       reinterpret_cast<double2 *>(X), reinterpret_cast<float2 *>(x),
                       (const State *)st);
    return hipGetLastError();
}

hipError_t launch_ir_direction(int j, const Table *tab, const Table &ht, const float *r, float *h,
                               const float *M, const Parts &parts, State *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_ir_direction, dim3(ht.nblocks), dim3(kBlock), 0, s, j, tab,
                       reinterpret_cast<const float2 *>(r), reinterpret_cast<float2 *>(h), M,
                       (const double *)parts.b, st);
    return hipGetLastError();
}

hipError_t launch_state_reset(State *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(64), 0, s, st);
    return hipGetLastError();
}

}  // namespace qp
