// C-PCG (Alg. 2) vector steps and the FP32 refinement steps, for gfx950.
//
// One PCG iteration j is three launches on one stream:
//   stiffness product   q = Q h, partial sums of Re(h^H q)            (parts.a)
//   update              alpha = rz / (Q h, h); r -= alpha q;
//                       partial sums of (r, M r) and ||r||^2          (parts.b)
//   direction           U += alpha h (the h of this iteration); unless the
//                       residual test stops the iteration:
//                       beta = (r, M r)_new / rz; h = M r + beta h
// The solution update sits in the direction pass, which reads h anyway, so
// h is read once per iteration by the vector steps.
// z = M r is never stored; it is recomputed from r and the diagonal M.
// The scalars stay on the device; the host only polls `done`.
//
// Every kernel serves K right-hand sides at once (K <= d): vector k of a
// family starts at element k * D, its state is st[k], its partial sums start
// at part + k * kPartStride.  A right-hand side that has finished (or, in
// FP32-IR, paused) is skipped by every workgroup alike.
//
// FP32-IR runs the same loop with float vectors (entries scaled by 1/||F'||)
// and FP64 scalars and dot products.  Whenever the float residual has dropped
// by delta since the last replacement (or reached the tolerance), the float
// iterations of that right-hand side pause; the replacement steps queued at
// the end of every batch act on the paused ones only: the float increment is
// folded into the FP64 solution X, the FP64 residual F' - Q X replaces r,
// convergence is decided on that true residual, and the iteration continues
// with the same search direction.
#include "qp_device.h"

// Workgroup loop over its chunk, four elements per thread per pass with every
// load of the pass issued before the first use (the chunk is a multiple of
// kBlock, usually 4 * kBlock).
#define QP_STREAM(i)                                                              \
    for (int i##0 = begin + threadIdx.x; i##0 < end; i##0 += 4 * kBlock)          \
        _Pragma("unroll") for (int i##u = 0; i##u < 4; ++i##u)                    \
            if (const int i = i##0 + i##u * kBlock; i < end)

namespace qp {
namespace {

template <typename T>
__global__ __launch_bounds__(kBlock) void k_pcg_init(int K, const Table *__restrict__ tab,
                                                     const double2 *__restrict__ f,
                                                     double2 *__restrict__ X64,
                                                     cplx_t<T> *__restrict__ U,
                                                     cplx_t<T> *__restrict__ r,
                                                     cplx_t<T> *__restrict__ h,
                                                     const T *__restrict__ M,
                                                     double *__restrict__ part,
                                                     const State *__restrict__ st)
{
    const size_t D = tab->D;
    int begin, end;
    chunk_of_block(tab, begin, end);
    for (int k = 0; k < K; ++k) {
        const double scale = (sizeof(T) == 4) ? st[k].inv_unit : 1.0;
        const double2 *fk = f + k * D;
        double acc[2] = {0.0, 0.0};
        QP_STREAM(i) {
            const double2 fv = fk[i];
            cplx_t<T> rv, hv, zero;
            rv.x = (i != 0) ? (T)(fv.x * scale) : (T)0;
            rv.y = (i != 0) ? (T)(fv.y * scale) : (T)0;
            const T m = M[i];
            hv.x = m * rv.x;
            hv.y = m * rv.y;
            zero.x = 0;
            zero.y = 0;
            U[k * D + i] = zero;
            r[k * D + i] = rv;
            h[k * D + i] = hv;
            if (X64) X64[k * D + i] = make_double2(0.0, 0.0);
            const double n2 = (double)rv.x * (double)rv.x + (double)rv.y * (double)rv.y;
            acc[0] += (double)m * n2;
            acc[1] += n2;
        }
        store_partials<2>(acc, part + k * kPartStride);
    }
}

// One workgroup: start each state from the init partials.
__global__ __launch_bounds__(kBlock) void k_pcg_start(int K, int is_ir, double tol, double delta,
                                                      int maxit, const double *__restrict__ part,
                                                      int nb, State *__restrict__ sts)
{
    for (int k = 0; k < K; ++k) {
        double v[2];
        load_totals<2>(part + k * kPartStride, nb, v);
        if (threadIdx.x != 0) continue;
        State *st = sts + k;
        const double rz = v[0], rr = v[1];
        st->rz[0] = rz;
        st->rz[1] = rz;
        st->rr = rr;
        st->iters = 0;
        st->replacements = 0;
        st->maxit = maxit;
        st->pause = 0;
        st->did_update = 0;
        st->replace = 0;
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
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_pcg_update(int j, int K, const Table *__restrict__ tab,
                                                       cplx_t<T> *__restrict__ r,
                                                       const cplx_t<T> *__restrict__ q,
                                                       const T *__restrict__ M,
                                                       const double *__restrict__ part_in,
                                                       double *__restrict__ part_out,
                                                       State *__restrict__ sts)
{
    const size_t D = tab->D;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    int begin, end;
    chunk_of_block(tab, begin, end);
    for (int k = 0; k < K; ++k) {
        State *st = sts + k;
        if (st->done || st->pause) {
            if (lead) st->did_update = 0;
            continue;
        }
        double hq[1];
        load_totals<1>(part_in + k * kPartStride, tab->nb_mv, hq);  // the product's partials
        if (!(hq[0] > 0.0)) {
            // (Q h, h) <= 0: Q is not positive definite on this Krylov space
            if (lead) {
                st->hq = hq[0];
                st->status = finite(hq[0]) ? QP_ENOTSPD : QP_ENONFINITE;
                st->done = 1;
                st->did_update = 0;
            }
            continue;
        }
        const double alpha = st->rz[j & 1] / hq[0];
        const T a = (T)alpha;
        double acc[2] = {0.0, 0.0};
        QP_STREAM(i) {
            const size_t e = k * D + i;
            cplx_t<T> rv = r[e];
            const cplx_t<T> qv = q[e];
            rv.x -= a * qv.x;
            rv.y -= a * qv.y;
            r[e] = rv;
            const double n2 = (double)rv.x * (double)rv.x + (double)rv.y * (double)rv.y;
            acc[0] += (double)M[i] * n2;
            acc[1] += n2;
        }
        store_partials<2>(acc, part_out + k * kPartStride);
        if (lead) {
            st->alpha = alpha;
            st->hq = hq[0];
            st->iters = st->iters + 1;
            st->did_update = 1;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_pcg_direction(int j, int is_ir, int K,
                                                          const Table *__restrict__ tab,
                                                          cplx_t<T> *__restrict__ U,
                                                          const cplx_t<T> *__restrict__ r,
                                                          cplx_t<T> *__restrict__ h,
                                                          const T *__restrict__ M,
                                                          const double *__restrict__ part_in,
                                                          State *__restrict__ sts)
{
    const size_t D = tab->D;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    int begin, end;
    chunk_of_block(tab, begin, end);
    for (int k = 0; k < K; ++k) {
        State *st = sts + k;
        const double rz_old = st->rz[j & 1];
        if (!st->did_update) {
            // no update this iteration; a paused solve carries rz forward so
            // iteration j+1 finds it in its slot
            if (lead && !st->done && st->pause) st->rz[(j + 1) & 1] = rz_old;
            continue;
        }
        double v[2];
        load_totals<2>(part_in + k * kPartStride, gridDim.x, v);
        const double rz_new = v[0], rr = v[1];
        // the update ran: U += alpha h with this iteration's h, whatever the
        // residual test below decides
        const T a = (T)st->alpha;
        bool stop = false;
        if (!finite(rr) || !finite(rz_new)) {
            if (lead) {
                st->status = QP_ENONFINITE;
                st->done = 1;
            }
            stop = true;
        } else if (is_ir) {
            if (rr <= fmax(st->thresh, st->delta2 * st->rr_last)) {
                if (lead) {
                    st->rr = rr;
                    st->pause = 1;
                    st->rz[(j + 1) & 1] = rz_old;
                }
                stop = true;
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
                stop = true;
            }
        }
        if (stop) {
            QP_STREAM(i) {
                const size_t e = k * D + i;
                const cplx_t<T> hv = h[e];
                cplx_t<T> u = U[e];
                u.x += a * hv.x;
                u.y += a * hv.y;
                U[e] = u;
            }
            continue;
        }
        const double beta = rz_new / rz_old;
        const T b = (T)beta;
        QP_STREAM(i) {
            const size_t e = k * D + i;
            const cplx_t<T> rv = r[e];
            const T m = M[i];
            cplx_t<T> hv = h[e];
            cplx_t<T> u = U[e];
            u.x += a * hv.x;
            u.y += a * hv.y;
            U[e] = u;
            hv.x = m * rv.x + b * hv.x;
            hv.y = m * rv.y + b * hv.y;
            h[e] = hv;
        }
        if (lead) {
            st->rr = rr;
            st->beta = beta;
            st->rz[(j + 1) & 1] = rz_new;
        }
    }
}

// ||f'_k||^2 partials (FP32-IR unit).
__global__ __launch_bounds__(kBlock) void k_norm2(int K, const Table *__restrict__ tab,
                                                  const double2 *__restrict__ f,
                                                  double *__restrict__ part)
{
    const size_t D = tab->D;
    int begin, end;
    chunk_of_block(tab, begin, end);
    for (int k = 0; k < K; ++k) {
        double acc[1] = {0.0};
        QP_STREAM(i) {
            if (i == 0) continue;
            const double2 v = f[k * D + i];
            acc[0] += v.x * v.x + v.y * v.y;
        }
        store_partials<1>(acc, part + k * kPartStride);
    }
}

__global__ __launch_bounds__(kBlock) void k_ir_unit(int K, const double *__restrict__ part, int nb,
                                                    State *__restrict__ sts)
{
    for (int k = 0; k < K; ++k) {
        double v[1];
        load_totals<1>(part + k * kPartStride, nb, v);
        if (threadIdx.x != 0) continue;
        State *st = sts + k;
        st->rr0 = v[0];
        st->unit = sqrt(v[0]);
        st->inv_unit = (v[0] > 0.0 && finite(v[0])) ? 1.0 / sqrt(v[0]) : 0.0;
    }
}

__global__ __launch_bounds__(kBlock) void k_ir_fold(int K, const Table *__restrict__ tab,
                                                    double2 *__restrict__ X,
                                                    float2 *__restrict__ x,
                                                    State *__restrict__ sts)
{
    const size_t D = tab->D;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    int begin, end;
    chunk_of_block(tab, begin, end);
    for (int k = 0; k < K; ++k) {
        // replaced only once paused; the decision is kept for the later
        // replacement steps, which must not read the flags they change
        const bool rep = !sts[k].done && sts[k].pause;
        if (lead) sts[k].replace = rep ? 1 : 0;
        if (!rep) continue;
        const double unit = sts[k].unit;
        QP_STREAM(i) {
            const size_t e = k * D + i;
            double2 a = X[e];
            const float2 v = x[e];
            a.x += unit * (double)v.x;
            a.y += unit * (double)v.y;
            X[e] = a;
            x[e] = make_float2(0.f, 0.f);
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_ir_direction(int j, int K, const Table *__restrict__ tab,
                                                         const float2 *__restrict__ r,
                                                         float2 *__restrict__ h,
                                                         const float *__restrict__ M,
                                                         const double *__restrict__ part_in,
                                                         State *__restrict__ sts)
{
    const size_t D = tab->D;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    int begin, end;
    chunk_of_block(tab, begin, end);
    for (int k = 0; k < K; ++k) {
        State *st = sts + k;
        if (!st->replace) continue;  // decided by the fold
        double v[2];
        load_totals<2>(part_in + k * kPartStride, tab->nb_mv, v);  // FP64 residual product
        const double rz_new = v[0], rr = v[1];  // true residual, scaled by 1/unit
        if (!finite(rr) || !finite(rz_new)) {
            if (lead) {
                st->status = QP_ENONFINITE;
                st->done = 1;
            }
            continue;
        }
        if (rr <= st->thresh) {
            if (lead) {
                st->rr = rr;
                st->status = QP_OK;
                st->done = 1;
                st->replacements = st->replacements + 1;
            }
            continue;
        }
        // Keep the search direction while the float recursion tracked the true
        // residual; restart it (beta = 0) when the true residual is well above
        // the recursive one it replaces (the recursion has drifted).
        const bool restart = rr > 4.0 * st->rr;
        const double beta = restart ? 0.0 : rz_new / st->rz[j & 1];
        const float b = (float)beta;
        QP_STREAM(i) {
            const size_t e = k * D + i;
            const float2 rv = r[e];
            const float m = M[i];
            float2 hv = h[e];
            hv.x = m * rv.x + b * hv.x;
            hv.y = m * rv.y + b * hv.y;
            h[e] = hv;
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
}

// Pause every unfinished right-hand side (the forced final replacement).
__global__ void k_ir_force(int K, State *sts)
{
    if (blockIdx.x == 0 && threadIdx.x < K && !sts[threadIdx.x].done) sts[threadIdx.x].pause = 1;
}

__global__ void k_state_reset(int K, State *sts)
{
    if (blockIdx.x != 0) return;
    const int k = threadIdx.x;
    if (k >= K) return;
    State *st = sts + k;
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
    st->did_update = 0;
    st->replace = 0;
}

}  // namespace

hipError_t launch_pcg_init(int prec, int K, const Table *tab, const Table &ht, const double *f,
                           double *X64, void *U, void *r, void *h, const void *M,
                           const Parts &parts, State *st, hipStream_t s)
{
    const dim3 grid(ht.nblocks), block(kBlock);
    auto F = reinterpret_cast<const double2 *>(f);
    auto X = reinterpret_cast<double2 *>(X64);
    if (prec == F64)
        hipLaunchKernelGGL(k_pcg_init<double>, grid, block, 0, s, K, tab, F, X, (double2 *)U,
                           (double2 *)r, (double2 *)h, (const double *)M, parts.b, st);
    else
        hipLaunchKernelGGL(k_pcg_init<float>, grid, block, 0, s, K, tab, F, X, (float2 *)U,
                           (float2 *)r, (float2 *)h, (const float *)M, parts.b, st);
    return hipGetLastError();
}

hipError_t launch_pcg_start(int prec, int K, const Table &ht, double tol, double delta, int maxit,
                            const Parts &parts, State *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_pcg_start, dim3(1), dim3(kBlock), 0, s, K, prec == F32 ? 1 : 0, tol,
                       delta, maxit, (const double *)parts.b, ht.nblocks, st);
    return hipGetLastError();
}

hipError_t launch_pcg_update(int prec, int j, int K, const Table *tab, const Table &ht, void *r,
                             const void *q, const void *M, const Parts &parts, State *st,
                             hipStream_t s)
{
    const dim3 grid(ht.nblocks), block(kBlock);
    if (prec == F64)
        hipLaunchKernelGGL(k_pcg_update<double>, grid, block, 0, s, j, K, tab, (double2 *)r,
                           (const double2 *)q, (const double *)M, (const double *)parts.a, parts.b,
                           st);
    else
        hipLaunchKernelGGL(k_pcg_update<float>, grid, block, 0, s, j, K, tab, (float2 *)r,
                           (const float2 *)q, (const float *)M, (const double *)parts.a, parts.b,
                           st);
    return hipGetLastError();
}

hipError_t launch_pcg_direction(int prec, int j, int K, const Table *tab, const Table &ht, void *U,
                                const void *r, void *h, const void *M, const Parts &parts,
                                State *st, hipStream_t s)
{
    const dim3 grid(ht.nblocks), block(kBlock);
    if (prec == F64)
        hipLaunchKernelGGL(k_pcg_direction<double>, grid, block, 0, s, j, 0, K, tab, (double2 *)U,
                           (const double2 *)r, (double2 *)h, (const double *)M,
                           (const double *)parts.b, st);
    else
        hipLaunchKernelGGL(k_pcg_direction<float>, grid, block, 0, s, j, 1, K, tab, (float2 *)U,
                           (const float2 *)r, (float2 *)h, (const float *)M,
                           (const double *)parts.b, st);
    return hipGetLastError();
}

hipError_t launch_ir_unit(int K, const Table *tab, const Table &ht, const double *f,
                          const Parts &parts, State *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_norm2, dim3(ht.nblocks), dim3(kBlock), 0, s, K, tab,
                       reinterpret_cast<const double2 *>(f), parts.c);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ir_unit, dim3(1), dim3(kBlock), 0, s, K, (const double *)parts.c,
                       ht.nblocks, st);
    return hipGetLastError();
}

hipError_t launch_ir_fold(int K, const Table *tab, const Table &ht, double *X, float *x, State *st,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_ir_fold, dim3(ht.nblocks), dim3(kBlock), 0, s, K, tab,
                       reinterpret_cast<double2 *>(X), reinterpret_cast<float2 *>(x), st);
    return hipGetLastError();
}

hipError_t launch_ir_direction(int j, int K, const Table *tab, const Table &ht, const float *r,
                               float *h, const float *M, const Parts &parts, State *st,
                               hipStream_t s)
{
    hipLaunchKernelGGL(k_ir_direction, dim3(ht.nblocks), dim3(kBlock), 0, s, j, K, tab,
                       reinterpret_cast<const float2 *>(r), reinterpret_cast<float2 *>(h), M,
                       (const double *)parts.b, st);
    return hipGetLastError();
}

hipError_t launch_ir_force(int K, State *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_ir_force, dim3(1), dim3(64), 0, s, K, st);
    return hipGetLastError();
}

hipError_t launch_state_reset(int K, State *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(64), 0, s, K, st);
    return hipGetLastError();
}

}  // namespace qp
