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
// Every kernel serves K right-hand sides at once (K <= d): entry i of vector
// k of a family is at vec_at<T>(k, K, D, i) (FP64 vectors one after the
// other, float vectors interleaved), its state is st[k], its partial sums
// start at part + k * kPartStride.  A right-hand side that has finished (or, in
// FP32-IR, paused) is skipped by every workgroup alike.  The FP64 kernels
// sweep the vectors one after the other; the float kernels (further down)
// read the K values of an entry with one load.
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
            const size_t e = vec_at<T>(k, K, D, i);
            U[e] = zero;
            r[e] = rv;
            h[e] = hv;
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
    const int nbp = sizeof(T) == 8 ? tab->nb_mv64 : tab->nb_mv;
    // the flags, scalars and product partials of every right-hand side, in
    // one round trip before the first branch
    int skip[kMaxRhs];
    double rz[kMaxRhs], p[kMaxRhs][kPartPer];
#pragma unroll
    for (int k = 0; k < kMaxRhs; ++k) {
        if (k >= K) break;
        skip[k] = sts[k].done | sts[k].pause;
        rz[k] = sts[k].rz[j & 1];
        double pk[1][kPartPer];
        fetch_partials<1>(part_in + k * kPartStride, pk);
#pragma unroll
        for (int t = 0; t < kPartPer; ++t) p[k][t] = pk[0][t];
    }
#pragma unroll
    for (int k = 0; k < kMaxRhs; ++k) {
        if (k >= K) break;
        pin(skip[k]);
        pin(rz[k]);
    }
    pin(begin);
    pin(end);
    pin(nbp);
#pragma unroll
    for (int k = 0; k < kMaxRhs; ++k) {
        if (k >= K) break;
        State *st = sts + k;
        if (skip[k]) {
            if (lead) st->did_update = 0;
            continue;
        }
        double hq[1];
        {
            double pk[1][kPartPer];
#pragma unroll
            for (int t = 0; t < kPartPer; ++t) pk[0][t] = p[k][t];
            sum_partials<1>(pk, nbp, hq);
        }
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
        const double alpha = rz[k] / hq[0];
        const T a = (T)alpha;
        double acc[2] = {0.0, 0.0};
        QP_STREAM(i) {
            const size_t e = vec_at<T>(k, K, D, i);
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
            hist_alpha(st, st->iters, alpha);
            st->alpha = alpha;
            st->hq = hq[0];
            st->iters = st->iters + 1;
            st->did_update = 1;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_pcg_direction(int j, int K,
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
    // the flags, scalars and update partials of every right-hand side, in one
    // round trip before the first branch (this launch's lead writes none of
    // the fields read here)
    int did[kMaxRhs], carry[kMaxRhs], limit_hit[kMaxRhs];
    double rz_old[kMaxRhs], alpha[kMaxRhs], thresh[kMaxRhs], p[kMaxRhs][2][kPartPer];
#pragma unroll
    for (int k = 0; k < kMaxRhs; ++k) {
        if (k >= K) break;
        const State *st = sts + k;
        did[k] = st->did_update;
        carry[k] = !st->done & (st->pause != 0);
        limit_hit[k] = st->iters >= st->maxit;  // iters counts this update
        rz_old[k] = st->rz[j & 1];
        alpha[k] = st->alpha;
        thresh[k] = st->thresh;
        fetch_partials<2>(part_in + k * kPartStride, p[k]);
    }
#pragma unroll
    for (int k = 0; k < kMaxRhs; ++k) {
        if (k >= K) break;
        pin(did[k]);
        pin(carry[k]);
        pin(limit_hit[k]);
        pin(rz_old[k]);
        pin(alpha[k]);
        pin(thresh[k]);
    }
    pin(begin);
    pin(end);
#pragma unroll
    for (int k = 0; k < kMaxRhs; ++k) {
        if (k >= K) break;
        State *st = sts + k;
        if (!did[k]) {
            // no update this iteration; a paused solve carries rz forward so
            // iteration j+1 finds it in its slot
            if (lead && carry[k]) st->rz[(j + 1) & 1] = rz_old[k];
            continue;
        }
        double v[2];
        sum_partials<2>(p[k], gridDim.x, v);
        const double rz_new = v[0], rr = v[1];
        // the update ran: U += alpha h with this iteration's h, whatever the
        // residual test below decides
        const T a = (T)alpha[k];
        bool stop = false;
        if (!finite(rr) || !finite(rz_new)) {
            if (lead) {
                st->status = QP_ENONFINITE;
                st->done = 1;
            }
            stop = true;
        } else {
            const bool conv = rr <= thresh[k];
            const bool limit = limit_hit[k] != 0;
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
                const size_t e = vec_at<T>(k, K, D, i);
                const cplx_t<T> hv = h[e];
                cplx_t<T> u = U[e];
                u.x += a * hv.x;
                u.y += a * hv.y;
                U[e] = u;
            }
            continue;
        }
        const double beta = rz_new / rz_old[k];
        const T b = (T)beta;
        QP_STREAM(i) {
            const size_t e = vec_at<T>(k, K, D, i);
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
            hist_beta(st, st->iters - 1, beta);
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

// Pause every unfinished right-hand side (the forced final replacement).
__global__ void k_ir_force(int K, State *sts)
{
    if (blockIdx.x == 0 && (int)threadIdx.x < K && !sts[threadIdx.x].done) sts[threadIdx.x].pause = 1;
}

__global__ void k_state_hist(State *sts, double *hist)
{
    if (blockIdx.x == 0 && (int)threadIdx.x < kMaxRhs)
        sts[threadIdx.x].hist = hist + (size_t)2 * kHist * threadIdx.x;
}

__global__ void k_state_reset(int K, State *sts)
{
    if (blockIdx.x != 0) return;
    const int k = threadIdx.x;
    if (k >= K) return;
    State *st = sts + k;
    st->rz[0] = st->rz[1] = 0.0;
    st->alpha = st->beta = st->hq = 0.0;
    st->rr = st->rr0 = st->thresh = st->delta2 = st->rr_last = st->rr_pause = 0.0;
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

// ---------------------------------------------------------------- float families
//
// The float vectors of the FP32-IR inner solve interleave their KK
// right-hand sides (entry i of all of them at i KK .. i KK + KK - 1), so the
// stiffness product gathers them with one load; these kernels walk entries
// once and treat the KK right-hand sides of an entry together, each with its
// own state, scalars and partial sums.  The arithmetic per (entry,
// right-hand side) is that of the FP64 kernels above, with the FP32-IR
// rules for pausing and replacing.

template <int KK>
__device__ __forceinline__ void ld_row(const float2 *__restrict__ p, size_t i, float2 (&v)[KK])
{
    const float2 *q = p + i * KK;
    if constexpr (KK == 2) {
        const float4 a = *reinterpret_cast<const float4 *>(q);
        v[0] = make_float2(a.x, a.y);
        v[1] = make_float2(a.z, a.w);
    } else if constexpr (KK == 4) {
        const float4 a = *reinterpret_cast<const float4 *>(q);
        const float4 b = *reinterpret_cast<const float4 *>(q + 2);
        v[0] = make_float2(a.x, a.y);
        v[1] = make_float2(a.z, a.w);
        v[2] = make_float2(b.x, b.y);
        v[3] = make_float2(b.z, b.w);
    } else {
#pragma unroll
        for (int k = 0; k < KK; ++k) v[k] = q[k];
    }
}

template <int KK>
__device__ __forceinline__ void st_row(float2 *__restrict__ p, size_t i, const float2 (&v)[KK])
{
    float2 *q = p + i * KK;
    if constexpr (KK == 2) {
        *reinterpret_cast<float4 *>(q) = make_float4(v[0].x, v[0].y, v[1].x, v[1].y);
    } else if constexpr (KK == 4) {
        *reinterpret_cast<float4 *>(q) = make_float4(v[0].x, v[0].y, v[1].x, v[1].y);
        *reinterpret_cast<float4 *>(q + 2) = make_float4(v[2].x, v[2].y, v[3].x, v[3].y);
    } else {
#pragma unroll
        for (int k = 0; k < KK; ++k) q[k] = v[k];
    }
}

template <int KK>
__global__ __launch_bounds__(kBlock) void k_init_f(const Table *__restrict__ tab,
                                                   const double2 *__restrict__ f,
                                                   double2 *__restrict__ X64, float2 *__restrict__ U,
                                                   float2 *__restrict__ r, float2 *__restrict__ h,
                                                   const float *__restrict__ M,
                                                   double *__restrict__ part,
                                                   const State *__restrict__ st)
{
    const size_t D = tab->D;
    int begin, end;
    chunk_of_block(tab, begin, end);
    double scale[KK], acc[KK][2];
#pragma unroll
    for (int k = 0; k < KK; ++k) {
        scale[k] = st[k].inv_unit;
        acc[k][0] = acc[k][1] = 0.0;
    }
    QP_STREAM(i) {
        const float m = M[i];
        float2 rv[KK], hv[KK], zero[KK];
#pragma unroll
        for (int k = 0; k < KK; ++k) {
            const double2 fv = f[k * D + i];
            rv[k].x = (i != 0) ? (float)(fv.x * scale[k]) : 0.f;
            rv[k].y = (i != 0) ? (float)(fv.y * scale[k]) : 0.f;
            hv[k].x = m * rv[k].x;
            hv[k].y = m * rv[k].y;
            zero[k] = make_float2(0.f, 0.f);
            if (X64) X64[k * D + i] = make_double2(0.0, 0.0);
            const double n2 = (double)rv[k].x * (double)rv[k].x + (double)rv[k].y * (double)rv[k].y;
            acc[k][0] += (double)m * n2;
            acc[k][1] += n2;
        }
        st_row<KK>(U, i, zero);
        st_row<KK>(r, i, rv);
        st_row<KK>(h, i, hv);
    }
#pragma unroll
    for (int k = 0; k < KK; ++k) store_partials<2>(acc[k], part + k * kPartStride);
}

// The first pass's rows of the update and the direction are requested before
// the previous launch's partial sums are reduced, so the reduction's latency
// overlaps the loads.  A pass loads ROWS entries per thread.  A later pass's
// loads of r cannot move above the earlier pass's stores to r, so each pass
// costs a wave a round trip to memory: chunks longer than 4 * kBlock take the
// 8-row instance (one pass up to 2048 entries), shorter ones the 4-row
// instance, whose smaller register count keeps more waves resident when many
// problems share the device.

template <int KK, int ROWS>
__device__ __forceinline__ void update_f(const int vb, const int vnb, int j,
                                         const Table *__restrict__ tab,
                                                     float2 *__restrict__ r,
                                                     const float2 *__restrict__ q,
                                                     const float *__restrict__ M,
                                                     const double *__restrict__ part_in,
                                                     double *__restrict__ part_out,
                                                     State *__restrict__ sts)
{
    const bool lead = vb == 0 && threadIdx.x == 0;
    int begin, end;
    chunk_of_block_at(tab, vb, vnb, begin, end);
    const int nbp = tab->nb_mv;
    // every flag and scalar of the right-hand sides, with the table fields,
    // in one round trip before the first branch
    int done[KK], pause[KK];
    double rz[KK];
#pragma unroll
    for (int k = 0; k < KK; ++k) {
        done[k] = sts[k].done;
        pause[k] = sts[k].pause;
        rz[k] = sts[k].rz[j & 1];
    }
#pragma unroll
    for (int k = 0; k < KK; ++k) pin(rz[k]);
    pin(begin);
    pin(end);
    pin(nbp);
    bool act[KK];
    bool any = false;
#pragma unroll
    for (int k = 0; k < KK; ++k) {
        act[k] = !(done[k] | pause[k]);
        if (!act[k] && lead) sts[k].did_update = 0;
        any = any || act[k];
    }
    if (!any) return;
    const int i0 = begin + threadIdx.x;
    // rows past the chunk load its last entry (and are never stored), so the
    // loads of every row are issued back to back without branches
    const int last = max(end - 1, 0);
    float2 rv[ROWS][KK], qv[ROWS][KK];
    float mv[ROWS];
#pragma unroll
    for (int u = 0; u < ROWS; ++u) {
        const int i = min(i0 + u * kBlock, last);
        ld_row<KK>(r, i, rv[u]);
        ld_row<KK>(q, i, qv[u]);
        mv[u] = M[i];
    }
    // the product's partials of every right-hand side, fetched together and
    // reduced in one pass (each value as load_totals reduces it)
    double hq_all[KK];
    {
        double p[KK][kPartPer];
#pragma unroll
        for (int k = 0; k < KK; ++k) {
            double pk[1][kPartPer];
            fetch_partials<1>(part_in + k * kPartStride, pk);
#pragma unroll
            for (int t = 0; t < kPartPer; ++t) p[k][t] = pk[0][t];
        }
        sum_partials<KK>(p, nbp, hq_all);
    }
    float a[KK];
    double alpha[KK], hqv[KK], acc[KK][2];
    any = false;
#pragma unroll
    for (int k = 0; k < KK; ++k) {
        State *st = sts + k;
        a[k] = 0.f;
        alpha[k] = hqv[k] = 0.0;
        acc[k][0] = acc[k][1] = 0.0;
        if (!act[k]) continue;
        const double hq[1] = {hq_all[k]};
        if (!(hq[0] > 0.0)) {
            // (Q h, h) <= 0: Q is not positive definite on this Krylov space
            if (lead) {
                st->hq = hq[0];
                st->status = finite(hq[0]) ? QP_ENOTSPD : QP_ENONFINITE;
                st->done = 1;
                st->did_update = 0;
            }
            act[k] = false;
            continue;
        }
        hqv[k] = hq[0];
        alpha[k] = rz[k] / hq[0];
        a[k] = (float)alpha[k];
        any = true;
    }
    if (!any) return;
    auto step = [&](int i, float2(&rw)[KK], const float2(&qw)[KK], float m) {
        const double md = (double)m;
#pragma unroll
        for (int k = 0; k < KK; ++k) {
            if (!act[k]) continue;
            rw[k].x -= a[k] * qw[k].x;
            rw[k].y -= a[k] * qw[k].y;
            const double n2 = (double)rw[k].x * (double)rw[k].x + (double)rw[k].y * (double)rw[k].y;
            acc[k][0] += md * n2;
            acc[k][1] += n2;
        }
        st_row<KK>(r, i, rw);
    };
#pragma unroll
    for (int u = 0; u < ROWS; ++u) {
        const int i = i0 + u * kBlock;
        if (i < end) step(i, rv[u], qv[u], mv[u]);
    }
    for (int ib = i0 + ROWS * kBlock; ib < end; ib += ROWS * kBlock) {
#pragma unroll
        for (int u = 0; u < ROWS; ++u) {
            const int i = min(ib + u * kBlock, last);
            ld_row<KK>(r, i, rv[u]);
            ld_row<KK>(q, i, qv[u]);
            mv[u] = M[i];
        }
#pragma unroll
        for (int u = 0; u < ROWS; ++u) {
            const int i = ib + u * kBlock;
            if (i < end) step(i, rv[u], qv[u], mv[u]);
        }
    }
    // this launch's partials of every right-hand side in one reduction pass
    {
        double v[2 * KK];
#pragma unroll
        for (int k = 0; k < KK; ++k) {
            v[2 * k] = acc[k][0];
            v[2 * k + 1] = acc[k][1];
        }
        block_reduce<2 * KK>(v);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < KK; ++k) {
                if (!act[k]) continue;
                part_out[k * kPartStride + vb] = v[2 * k];
                part_out[k * kPartStride + kMaxBlocks + vb] = v[2 * k + 1];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < KK; ++k) {
        if (!act[k]) continue;
        if (lead) {
            State *st = sts + k;
            hist_alpha(st, st->iters, alpha[k]);
            st->alpha = alpha[k];
            st->hq = hqv[k];
            st->iters = st->iters + 1;
            st->did_update = 1;
        }
    }
}

// FP32-IR direction (the FP32-IR rules of k_pcg_direction): U += alpha h for
// every right-hand side whose update ran; h = M r + beta h unless it pauses.
template <int KK, int ROWS>
__device__ __forceinline__ void direction_f(const int vb, const int vnb, int j,
                                         const Table *__restrict__ tab,
                                                        float2 *__restrict__ U,
                                                        const float2 *__restrict__ r,
                                                        float2 *__restrict__ h,
                                                        const float *__restrict__ M,
                                                        const double *__restrict__ part_in,
                                                        State *__restrict__ sts)
{
    const bool lead = vb == 0 && threadIdx.x == 0;
    int begin, end;
    chunk_of_block_at(tab, vb, vnb, begin, end);
    // every flag and scalar of the right-hand sides in one round trip before
    // the first branch (this launch's lead writes none of them)
    int did_up[KK], done[KK], pause[KK];
    double rz_old[KK], alpha[KK], thresh[KK], delta2[KK], rr_last[KK];
#pragma unroll
    for (int k = 0; k < KK; ++k) {
        const State *st = sts + k;
        did_up[k] = st->did_update;
        done[k] = st->done;
        pause[k] = st->pause;
        rz_old[k] = st->rz[j & 1];
        alpha[k] = st->alpha;
        thresh[k] = st->thresh;
        delta2[k] = st->delta2;
        rr_last[k] = st->rr_last;
    }
#pragma unroll
    for (int k = 0; k < KK; ++k) {
        pin(rz_old[k]);
        pin(alpha[k]);
        pin(thresh[k]);
        pin(delta2[k]);
        pin(rr_last[k]);
    }
    pin(begin);
    pin(end);
    bool did[KK];
    bool any_did = false;
#pragma unroll
    for (int k = 0; k < KK; ++k) {
        did[k] = did_up[k] != 0;
        // no update this iteration; a paused solve carries rz forward so
        // iteration j+1 finds it in its slot
        if (!did[k] && lead && !done[k] && pause[k]) sts[k].rz[(j + 1) & 1] = rz_old[k];
        any_did = any_did || did[k];
    }
    if (!any_did) return;
    const int i0 = begin + threadIdx.x;
    // rows past the chunk load its last entry (and are never stored)
    const int last = max(end - 1, 0);
    float2 uv[ROWS][KK], hv[ROWS][KK], rv[ROWS][KK];
    float mv[ROWS];
#pragma unroll
    for (int u = 0; u < ROWS; ++u) {
        const int i = min(i0 + u * kBlock, last);
        ld_row<KK>(U, i, uv[u]);
        ld_row<KK>(h, i, hv[u]);
        ld_row<KK>(r, i, rv[u]);
        mv[u] = M[i];
    }
    // the update's partials (r, M r) and (r, r) of every right-hand side,
    // fetched together and reduced in one pass
    double tot[2 * KK];
    {
        double p[2 * KK][kPartPer];
#pragma unroll
        for (int k = 0; k < KK; ++k) {
            double pk[2][kPartPer];
            fetch_partials<2>(part_in + k * kPartStride, pk);
#pragma unroll
            for (int t = 0; t < kPartPer; ++t) {
                p[2 * k][t] = pk[0][t];
                p[2 * k + 1][t] = pk[1][t];
            }
        }
        sum_partials<2 * KK>(p, vnb, tot);
    }
    bool go[KK];
    float a[KK], b[KK];
    double rzn[KK], rrv[KK], betav[KK];
    bool any_go = false;
#pragma unroll
    for (int k = 0; k < KK; ++k) {
        State *st = sts + k;
        go[k] = false;
        a[k] = b[k] = 0.f;
        rzn[k] = rrv[k] = betav[k] = 0.0;
        if (!did[k]) continue;
        a[k] = (float)alpha[k];
        const double rz_new = tot[2 * k], rr = tot[2 * k + 1];
        if (!finite(rr) || !finite(rz_new)) {
            if (lead) {
                st->status = QP_ENONFINITE;
                st->done = 1;
            }
            continue;
        }
        if (rr <= fmax(thresh[k], delta2[k] * rr_last[k])) {
            if (lead) {
                st->rr = rr;
                st->pause = 1;
                st->rz[(j + 1) & 1] = rz_old[k];
            }
            continue;
        }
        go[k] = true;
        any_go = true;
        rzn[k] = rz_new;
        rrv[k] = rr;
        betav[k] = rz_new / rz_old[k];
        b[k] = (float)betav[k];
    }
    auto step = [&](int i, float2(&uw)[KK], float2(&hw)[KK], const float2(&rw)[KK], float m) {
#pragma unroll
        for (int k = 0; k < KK; ++k) {
            if (!did[k]) continue;
            uw[k].x += a[k] * hw[k].x;
            uw[k].y += a[k] * hw[k].y;
            if (go[k]) {
                hw[k].x = m * rw[k].x + b[k] * hw[k].x;
                hw[k].y = m * rw[k].y + b[k] * hw[k].y;
            }
        }
        st_row<KK>(U, i, uw);
        if (any_go) st_row<KK>(h, i, hw);
    };
#pragma unroll
    for (int u = 0; u < ROWS; ++u) {
        const int i = i0 + u * kBlock;
        if (i < end) step(i, uv[u], hv[u], rv[u], mv[u]);
    }
    for (int ib = i0 + ROWS * kBlock; ib < end; ib += ROWS * kBlock) {
#pragma unroll
        for (int u = 0; u < ROWS; ++u) {
            const int i = min(ib + u * kBlock, last);
            ld_row<KK>(U, i, uv[u]);
            ld_row<KK>(h, i, hv[u]);
            ld_row<KK>(r, i, rv[u]);
            mv[u] = M[i];
        }
#pragma unroll
        for (int u = 0; u < ROWS; ++u) {
            const int i = ib + u * kBlock;
            if (i < end) step(i, uv[u], hv[u], rv[u], mv[u]);
        }
    }
    if (lead) {
#pragma unroll
        for (int k = 0; k < KK; ++k) {
            if (!go[k]) continue;
            State *st = sts + k;
            hist_beta(st, st->iters - 1, betav[k]);
            st->rr = rrv[k];
            st->beta = betav[k];
            st->rz[(j + 1) & 1] = rzn[k];
        }
    }
}

template <int KK>
__device__ __forceinline__ void fold_f(const int vb, const int vnb, const Table *__restrict__ tab,
                                                   double2 *__restrict__ X,
                                                   float2 *__restrict__ x,
                                                   State *__restrict__ sts)
{
    const size_t D = tab->D;
    const bool lead = vb == 0 && threadIdx.x == 0;
    int begin, end;
    chunk_of_block_at(tab, vb, vnb, begin, end);
    bool rep[KK];
    int done[KK], pause[KK];
    double unit[KK], rr[KK];
#pragma unroll
    for (int k = 0; k < KK; ++k) {  // one round trip before the first branch
        done[k] = sts[k].done;
        pause[k] = sts[k].pause;
        unit[k] = sts[k].unit;
        rr[k] = sts[k].rr;
    }
#pragma unroll
    for (int k = 0; k < KK; ++k) {
        pin(unit[k]);
        pin(rr[k]);
    }
    pin(begin);
    pin(end);
    bool any = false;
#pragma unroll
    for (int k = 0; k < KK; ++k) {
        // replaced only once paused; the decision is kept for the later
        // replacement steps, which must not read the flags they change
        rep[k] = !done[k] && pause[k];
        if (lead) {
            sts[k].replace = rep[k] ? 1 : 0;
            sts[k].rr_pause = rr[k];
        }
        any = any || rep[k];
    }
    if (!any) return;
    QP_STREAM(i) {
        float2 v[KK];
        ld_row<KK>(x, i, v);
#pragma unroll
        for (int k = 0; k < KK; ++k) {
            if (!rep[k]) continue;
            const size_t e = (size_t)k * D + i;
            double2 s = X[e];
            s.x += unit[k] * (double)v[k].x;
            s.y += unit[k] * (double)v[k].y;
            X[e] = s;
            v[k] = make_float2(0.f, 0.f);
        }
        st_row<KK>(x, i, v);
    }
}

template <int KK>
__device__ __forceinline__ void irdir_f(const int vb, const int vnb, int j,
                                         const Table *__restrict__ tab,
                                                    const float2 *__restrict__ r,
                                                    float2 *__restrict__ h,
                                                    const float *__restrict__ M,
                                                    const double *__restrict__ part_in,
                                                    State *__restrict__ sts)
{
    const bool lead = vb == 0 && threadIdx.x == 0;
    int begin, end;
    chunk_of_block_at(tab, vb, vnb, begin, end);
    bool go[KK];
    float b[KK];
    double rzn[KK], rrv[KK], betav[KK];
    int replace[KK];
    double thresh[KK], rr_pause[KK], rz_old[KK];
    const int nbp = tab->nb_mv64;
#pragma unroll
    for (int k = 0; k < KK; ++k) {  // one round trip before the first branch
        const State *st = sts + k;
        replace[k] = st->replace;
        thresh[k] = st->thresh;
        rr_pause[k] = st->rr_pause;
        rz_old[k] = st->rz[j & 1];
    }
#pragma unroll
    for (int k = 0; k < KK; ++k) {
        pin(thresh[k]);
        pin(rr_pause[k]);
        pin(rz_old[k]);
    }
    pin(begin);
    pin(end);
    pin(nbp);
    // the FP64 residual product's partials of every right-hand side, fetched
    // together and reduced in one pass
    double tot[2 * KK];
    {
        double p[2 * KK][kPartPer];
#pragma unroll
        for (int k = 0; k < KK; ++k) {
            double pk[2][kPartPer];
            fetch_partials<2>(part_in + k * kPartStride, pk);
#pragma unroll
            for (int t = 0; t < kPartPer; ++t) {
                p[2 * k][t] = pk[0][t];
                p[2 * k + 1][t] = pk[1][t];
            }
        }
        sum_partials<2 * KK>(p, nbp, tot);
    }
    bool any = false;
#pragma unroll
    for (int k = 0; k < KK; ++k) {
        State *st = sts + k;
        go[k] = false;
        b[k] = 0.f;
        rzn[k] = rrv[k] = betav[k] = 0.0;
        if (!replace[k]) continue;  // decided by the fold
        const double rz_new = tot[2 * k], rr = tot[2 * k + 1];  // true residual, scaled by 1/unit
        if (!finite(rr) || !finite(rz_new)) {
            if (lead) {
                st->status = QP_ENONFINITE;
                st->done = 1;
            }
            continue;
        }
        if (rr <= thresh[k]) {
            if (lead) {
                st->rr = rr;
                st->status = QP_OK;
                st->done = 1;
                st->replacements = st->replacements + 1;
            }
            continue;
        }
        // keep the search direction while the float recursion tracked the
        // true residual; restart it (beta = 0) when the true residual is well
        // above the recursive one it replaces (the recursion has drifted)
        // (rr_pause is the snapshot the fold took: st->rr itself is rewritten
        // by this kernel's lead while other workgroups may still read it)
        const bool restart = rr > 4.0 * rr_pause[k];
        go[k] = true;
        any = true;
        rzn[k] = rz_new;
        rrv[k] = rr;
        betav[k] = restart ? 0.0 : rz_new / rz_old[k];
        b[k] = (float)betav[k];
    }
    if (!any) return;
    QP_STREAM(i) {
        float2 rv[KK], hv[KK];
        ld_row<KK>(r, i, rv);
        ld_row<KK>(h, i, hv);
        const float m = M[i];
#pragma unroll
        for (int k = 0; k < KK; ++k) {
            if (!go[k]) continue;
            hv[k].x = m * rv[k].x + b[k] * hv[k].x;
            hv[k].y = m * rv[k].y + b[k] * hv[k].y;
        }
        st_row<KK>(h, i, hv);
    }
    if (lead) {
#pragma unroll
        for (int k = 0; k < KK; ++k) {
            if (!go[k]) continue;
            State *st = sts + k;
            // a replaced residual does not continue the float recursion's
            // Lanczos relation: the condition estimate takes the float
            // iterations between replacements as separate segments
            hist_beta(st, st->iters - 1, 0.0);
            st->rr = rrv[k];
            st->rr_last = rrv[k];
            st->beta = betav[k];
            st->rz[(j + 1) & 1] = rzn[k];
            st->pause = 0;
            st->replacements = st->replacements + 1;
        }
    }
}


// Kernels over one problem (the whole grid) and grouped over several (each
// workgroup serves the problem owner[blockIdx.x] as one of its workgroups).
template <int KK, int ROWS>
__global__ __launch_bounds__(kBlock) void k_update_f(int j, const Table *__restrict__ tab,
                                                     float2 *__restrict__ r,
                                                     const float2 *__restrict__ q,
                                                     const float *__restrict__ M,
                                                     const double *__restrict__ part_in,
                                                     double *__restrict__ part_out,
                                                     State *__restrict__ sts)
{
    update_f<KK, ROWS>((int)blockIdx.x, (int)gridDim.x, j, tab, r, q, M, part_in, part_out, sts);
}

template <int KK, int ROWS>
__global__ __launch_bounds__(kBlock) void k_direction_f(int j, const Table *__restrict__ tab,
                                                        float2 *__restrict__ U,
                                                        const float2 *__restrict__ r,
                                                        float2 *__restrict__ h,
                                                        const float *__restrict__ M,
                                                        const double *__restrict__ part_in,
                                                        State *__restrict__ sts)
{
    direction_f<KK, ROWS>((int)blockIdx.x, (int)gridDim.x, j, tab, U, r, h, M, part_in, sts);
}

template <int KK>
__global__ __launch_bounds__(kBlock) void k_fold_f(const Table *__restrict__ tab,
                                                   double2 *__restrict__ X,
                                                   float2 *__restrict__ x,
                                                   State *__restrict__ sts)
{
    fold_f<KK>((int)blockIdx.x, (int)gridDim.x, tab, X, x, sts);
}

template <int KK>
__global__ __launch_bounds__(kBlock) void k_irdir_f(int j, const Table *__restrict__ tab,
                                                    const float2 *__restrict__ r,
                                                    float2 *__restrict__ h,
                                                    const float *__restrict__ M,
                                                    const double *__restrict__ part_in,
                                                    State *__restrict__ sts)
{
    irdir_f<KK>((int)blockIdx.x, (int)gridDim.x, j, tab, r, h, M, part_in, sts);
}

// step: 0 update, 1 direction, 2 fold, 3 replacement direction
template <int KK, int STEP>
__global__ __launch_bounds__(kBlock) void k_vec_grp(int j, const GroupEntry *__restrict__ ents,
                                                    const int *__restrict__ owner)
{
    const GroupEntry &e = ents[owner[blockIdx.x]];
    const int vb = (int)blockIdx.x - e.sv0, vnb = e.nb_st;
    float2 *x32 = reinterpret_cast<float2 *>(e.x32);
    float2 *r32 = reinterpret_cast<float2 *>(e.r32);
    float2 *h32 = reinterpret_cast<float2 *>(e.h32);
    // the row count of the problem's own launches (launch_pcg_update and
    // launch_pcg_direction), so that every partial sum is formed alike
    if constexpr (STEP == 0) {
        if (e.wide)
            update_f<KK, 8>(vb, vnb, j, e.tab, r32, reinterpret_cast<const float2 *>(e.q32), e.M32,
                            e.pa, e.pb, e.st);
        else
            update_f<KK, 4>(vb, vnb, j, e.tab, r32, reinterpret_cast<const float2 *>(e.q32), e.M32,
                            e.pa, e.pb, e.st);
    } else if constexpr (STEP == 1) {
        if (e.wide)
            direction_f<KK, 8>(vb, vnb, j, e.tab, x32, r32, h32, e.M32, e.pb, e.st);
        else
            direction_f<KK, 4>(vb, vnb, j, e.tab, x32, r32, h32, e.M32, e.pb, e.st);
    }
    else if constexpr (STEP == 2)
        fold_f<KK>(vb, vnb, e.tab, reinterpret_cast<double2 *>(e.X), x32, e.st);
    else
        irdir_f<KK>(vb, vnb, j, e.tab, r32, h32, e.M32, e.pb, e.st);
}

// The K states of every problem of a group, one after the other (the poll).
__global__ void k_group_states(int G, int K, const GroupEntry *__restrict__ ents,
                               State *__restrict__ out)
{
    for (int t = threadIdx.x; t < G * K; t += blockDim.x) out[t] = ents[t / K].st[t % K];
}

}  // namespace

hipError_t launch_pcg_init(int prec, int K, const Table *tab, const Table &ht, const double *f,
                           double *X64, void *U, void *r, void *h, const void *M,
                           const Parts &parts, State *st, hipStream_t s)
{
    const dim3 grid(ht.nblocks), block(kBlock);
    auto F = reinterpret_cast<const double2 *>(f);
    auto X = reinterpret_cast<double2 *>(X64);
    if (prec == F64) {
        hipLaunchKernelGGL(k_pcg_init<double>, grid, block, 0, s, K, tab, F, X, (double2 *)U,
                           (double2 *)r, (double2 *)h, (const double *)M, parts.b, st);
        return hipGetLastError();
    }
    switch (K) {
#define QP_K(KK)                                                                                   \
    case KK:                                                                                        \
        hipLaunchKernelGGL(k_init_f<KK>, grid, block, 0, s, tab, F, X, (float2 *)U, (float2 *)r,  \
                           (float2 *)h, (const float *)M, parts.b, st);                             \
        break;
        QP_K(1) QP_K(2) QP_K(3) QP_K(4)
#undef QP_K
    default:
        return hipErrorInvalidValue;
    }
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
    if (prec == F64) {
        hipLaunchKernelGGL(k_pcg_update<double>, grid, block, 0, s, j, K, tab, (double2 *)r,
                           (const double2 *)q, (const double *)M, (const double *)parts.a, parts.b,
                           st);
        return hipGetLastError();
    }
    const bool wide = ht.chunk > 4 * kBlock;
    switch (K) {
#define QP_K(KK)                                                                                  \
    case KK:                                                                                       \
    {                                                                                              \
        auto kern = wide ? k_update_f<KK, 8> : k_update_f<KK, 4>;                                 \
        hipLaunchKernelGGL(kern, grid, block, 0, s, j, tab, (float2 *)r, (const float2 *)q,       \
                           (const float *)M, (const double *)parts.a, parts.b, st);                \
    } break;
        QP_K(1) QP_K(2) QP_K(3) QP_K(4)
#undef QP_K
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pcg_direction(int prec, int j, int K, const Table *tab, const Table &ht, void *U,
                                const void *r, void *h, const void *M, const Parts &parts,
                                State *st, hipStream_t s)
{
    const dim3 grid(ht.nblocks), block(kBlock);
    if (prec == F64) {
        hipLaunchKernelGGL(k_pcg_direction<double>, grid, block, 0, s, j, K, tab, (double2 *)U,
                           (const double2 *)r, (double2 *)h, (const double *)M,
                           (const double *)parts.b, st);
        return hipGetLastError();
    }
    const bool wide = ht.chunk > 4 * kBlock;
    switch (K) {
#define QP_K(KK)                                                                                 \
    case KK:                                                                                      \
    {                                                                                             \
        auto kern = wide ? k_direction_f<KK, 8> : k_direction_f<KK, 4>;                          \
        hipLaunchKernelGGL(kern, grid, block, 0, s, j, tab, (float2 *)U, (const float2 *)r,      \
                           (float2 *)h, (const float *)M, (const double *)parts.b, st);           \
    } break;
        QP_K(1) QP_K(2) QP_K(3) QP_K(4)
#undef QP_K
    default:
        return hipErrorInvalidValue;
    }
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

hipError_t launch_ir_unit_only(int K, const Table &ht, const Parts &parts, State *st,
                               hipStream_t s)
{
    hipLaunchKernelGGL(k_ir_unit, dim3(1), dim3(kBlock), 0, s, K, (const double *)parts.c,
                       ht.nblocks, st);
    return hipGetLastError();
}

hipError_t launch_ir_fold(int K, const Table *tab, const Table &ht, double *X, float *x, State *st,
                          hipStream_t s)
{
    switch (K) {
#define QP_K(KK)                                                                              \
    case KK:                                                                                   \
        hipLaunchKernelGGL(k_fold_f<KK>, dim3(ht.nblocks), dim3(kBlock), 0, s, tab,           \
                           reinterpret_cast<double2 *>(X), reinterpret_cast<float2 *>(x), st); \
        break;
        QP_K(1) QP_K(2) QP_K(3) QP_K(4)
#undef QP_K
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_ir_direction(int j, int K, const Table *tab, const Table &ht, const float *r,
                               float *h, const float *M, const Parts &parts, State *st,
                               hipStream_t s)
{
    switch (K) {
#define QP_K(KK)                                                                                \
    case KK:                                                                                     \
        hipLaunchKernelGGL(k_irdir_f<KK>, dim3(ht.nblocks), dim3(kBlock), 0, s, j, tab,         \
                           reinterpret_cast<const float2 *>(r), reinterpret_cast<float2 *>(h), M, \
                           (const double *)parts.b, st);                                         \
        break;
        QP_K(1) QP_K(2) QP_K(3) QP_K(4)
#undef QP_K
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_ir_force(int K, State *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_ir_force, dim3(1), dim3(64), 0, s, K, st);
    return hipGetLastError();
}

hipError_t launch_state_hist(State *st, double *hist, hipStream_t s)
{
    hipLaunchKernelGGL(k_state_hist, dim3(1), dim3(64), 0, s, st, hist);
    return hipGetLastError();
}

hipError_t launch_state_reset(int K, State *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(64), 0, s, K, st);
    return hipGetLastError();
}

}  // namespace qp

namespace qp {

hipError_t launch_group_vec(int step, int j, int K, int total, const GroupEntry *E, const int *owner,
                            hipStream_t s)
{
    if (total < 1 || step < 0 || step > 3) return hipErrorInvalidValue;
    const dim3 grid(total), block(kBlock);
#define QP_STEP(KK, ST)                                                                     \
    case ST:                                                                                 \
        hipLaunchKernelGGL((k_vec_grp<KK, ST>), grid, block, 0, s, j, E, owner);            \
        break;
#define QP_K(KK)                                                                            \
    case KK:                                                                                 \
        switch (step) { QP_STEP(KK, 0) QP_STEP(KK, 1) QP_STEP(KK, 2) QP_STEP(KK, 3) }      \
        break;
    switch (K) {
        QP_K(2) QP_K(3)
    default:
        return hipErrorInvalidValue;
    }
#undef QP_K
#undef QP_STEP
    return hipGetLastError();
}

hipError_t launch_group_states(int G, int K, const GroupEntry *E, State *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_group_states, dim3(1), dim3(kBlock), 0, s, G, K, E, out);
    return hipGetLastError();
}

}  // namespace qp
