// C-PCG (Alg. 2) of a small problem in one launch: one workgroup per
// right-hand side runs the whole iteration loop in FP64.  Each of its
// threads (1024 for d <= 2, 512 for d = 3, 4, whose product needs more
// registers) keeps its own entries of r, q and M in registers (two or four
// entries each, so at most kSmallMax unknowns); the search direction h is
// also held in LDS, where the stiffness product gathers its neighbours, and
// so is the solution U (64 KB of LDS in all), so an iteration touches no
// global memory and costs a few workgroup barriers instead of three
// launches.  Scalar coefficient, full storage.  The loop
// continues from the vectors and states of launch_pcg_init and
// launch_pcg_start and leaves them as the multi-workgroup FP64 kernels do
// (the same recurrences, state fields and Lanczos coefficients); its sums are
// formed in this workgroup's own fixed order.
#include "qp_device.h"

namespace qp {
namespace {

// Threads per workgroup for d = DT.
template <int DT>
constexpr int small_block()
{
    return DT <= 2 ? 1024 : 512;
}
constexpr int kSmallWavesMax = 1024 / kWave;

// Workgroup sum of NV values over W waves, in a fixed order; the result in
// every thread.
template <int W, int NV>
__device__ __forceinline__ void small_reduce(double (&v)[NV], double (*red)[kSmallWavesMax])
{
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double s = wave_sum(v[k]);
        if (lane == 0) red[k][wid] = s;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double t = red[k][0];
#pragma unroll
        for (int w = 1; w < W; ++w) t += red[k][w];
        v[k] = t;
    }
    __syncthreads();  // red is written again by the next reduction
}

// The problem's modes, coefficients, projection and strides, copied to LDS
// once per launch (the loop reads them in every iteration).
struct SmallTab {
    int mode[kMaxG][kMaxN];
    double coef[kMaxG][2];
    double Pm[kMaxG][kMaxD];
    double P[kMaxD][kMaxN];
    int stride[kMaxN];
    int n, N, g;
    uint64_t magic;
    int shift;
};

// (Q u)_i of eq. n-discrete for one entry, u in LDS: the digits of i give k
// (first axis slowest, digit a -> a or a - N in K_N); for each mode m the
// neighbour j = rep(k - m) per axis, W = (P k).(P j), y += Ahat_m W u_{C(j)};
// y_0 = 0.  P j = P k - P m + N sum_t c_t P e_t, where c_t in {-1, 0, 1} is
// the wrap of axis t.  The axes are unrolled to kMaxN (guarded by t < n) so
// that k stays in registers.
template <int DT>
__device__ __forceinline__ double2 product_entry(const SmallTab &T, int i, const double2 *u)
{
    if (i == 0) return make_double2(0.0, 0.0);
    const int n = T.n, N = T.N, g = T.g;
    const int lo = -(N / 2), hi = N - 1 - N / 2;
    int kd[kMaxN];
    double pk[DT];
#pragma unroll
    for (int l = 0; l < DT; ++l) pk[l] = 0.0;
    int rest = i;
#pragma unroll
    for (int tt = 0; tt < kMaxN; ++tt) {
        const int t = kMaxN - 1 - tt;
        kd[t] = 0;
        if (t < n) {
            const int q = (int)(((uint64_t)(uint32_t)rest * T.magic) >> T.shift);  // rest / N
            const int a = rest - q * N;
            rest = q;
            kd[t] = (a <= hi) ? a : a - N;
#pragma unroll
            for (int l = 0; l < DT; ++l) pk[l] += T.P[l][t] * (double)kd[t];
        }
    }
    double yr = 0.0, yi = 0.0;
    for (int r = 0; r < g; ++r) {
        double pj[DT];
#pragma unroll
        for (int l = 0; l < DT; ++l) pj[l] = pk[l] - T.Pm[r][l];
        int idx = 0;
#pragma unroll
        for (int t = 0; t < kMaxN; ++t) {
            if (t < n) {
                int jt = kd[t] - T.mode[r][t];
                const int c = (jt < lo) ? 1 : ((jt > hi) ? -1 : 0);
                jt += c * N;
                idx += ((jt < 0) ? jt + N : jt) * T.stride[t];
                if (c != 0)
#pragma unroll
                    for (int l = 0; l < DT; ++l) pj[l] += (double)(c * N) * T.P[l][t];
            }
        }
        double w = 0.0;
#pragma unroll
        for (int l = 0; l < DT; ++l) w += pk[l] * pj[l];
        const double2 uv = u[idx];
        const double cr = T.coef[r][0] * w, ci = T.coef[r][1] * w;
        yr += cr * uv.x - ci * uv.y;
        yi += cr * uv.y + ci * uv.x;
    }
    return make_double2(yr, yi);
}

// Workgroup k solves right-hand side k (vectors at k D of each family).
// Thread t owns the entries t + s B (B threads).  Every thread keeps the
// loop's scalars (all come out of workgroup reductions, so the copies
// agree); thread 0 writes the state.
template <int DT>
__global__ __launch_bounds__(small_block<DT>()) void k_pcg_wg(const Table *__restrict__ tab,
                                                        double2 *__restrict__ U,
                                                        double2 *__restrict__ r,
                                                        double2 *__restrict__ h,
                                                        const double *__restrict__ M,
                                                        State *__restrict__ sts)
{
    __shared__ double2 s_h[kSmallMax];
    __shared__ double2 s_u[kSmallMax];  // U: each thread its own entries
    constexpr int B = small_block<DT>();
    constexpr int PER = kSmallMax / B;  // entries per thread
    __shared__ double red[2][kSmallWavesMax];
    __shared__ SmallTab T;
    const int D = tab->D;
    State *st = sts + blockIdx.x;
    const size_t o = (size_t)blockIdx.x * D;
    U += o;
    r += o;
    h += o;
    if (st->done) return;
    const bool lead = threadIdx.x == 0;
    for (int e = threadIdx.x; e < kMaxG * kMaxN; e += B) {
        const int r = e / kMaxN, t = e - r * kMaxN;
        T.mode[r][t] = (r < tab->g && t < tab->n) ? tab->modes[r][t] : 0;
    }
    for (int e = threadIdx.x; e < kMaxG * 2; e += B)
        T.coef[e / 2][e % 2] = (e / 2 < tab->g) ? tab->coef[e / 2][e % 2] : 0.0;
    for (int e = threadIdx.x; e < kMaxG * kMaxD; e += B)
        T.Pm[e / kMaxD][e % kMaxD] = (e / kMaxD < tab->g) ? tab->Pm[e / kMaxD][e % kMaxD] : 0.0;
    for (int e = threadIdx.x; e < kMaxD * kMaxN; e += B)
        T.P[e / kMaxN][e % kMaxN] = tab->P[e / kMaxN][e % kMaxN];
    if (threadIdx.x < kMaxN) T.stride[threadIdx.x] = tab->stride[threadIdx.x];
    if (lead) {
        T.n = tab->n;
        T.N = tab->N;
        T.g = tab->g;
        T.magic = tab->magic;
        T.shift = tab->shift;
    }
    double2 rv[PER], qv[PER];
    double mv[PER];
#pragma unroll
    for (int s = 0; s < PER; ++s) {
        const int i = threadIdx.x + s * B;
        if (i < D) {
            rv[s] = r[i];
            s_u[i] = U[i];
            s_h[i] = h[i];
            mv[s] = M[i];
        }
    }
    __syncthreads();
    const double thresh = st->thresh;
    const int maxit = st->maxit;
    double rz = st->rz[0];  // both slots hold (r_0, M r_0) after launch_pcg_start
    int iters = st->iters;
    double alpha = 0.0, beta = 0.0, hq = 0.0, rr = st->rr;
    int status = QP_OK;
    for (;;) {
        // q = Q h and (h, q)
        double v1[1] = {0.0};
#pragma unroll
        for (int s = 0; s < PER; ++s) {
            const int i = threadIdx.x + s * B;
            if (i < D) {
                qv[s] = product_entry<DT>(T, i, s_h);
                const double2 hv = s_h[i];
                v1[0] += hv.x * qv[s].x + hv.y * qv[s].y;
            }
        }
        small_reduce<B / kWave, 1>(v1, red);
        hq = v1[0];
        if (!(hq > 0.0)) {
            // (Q h, h) <= 0: Q is not positive definite on this Krylov space
            status = finite(hq) ? QP_ENOTSPD : QP_ENONFINITE;
            break;
        }
        alpha = rz / hq;
        // r -= alpha q; (r, M r) and ||r||^2
        double v2[2] = {0.0, 0.0};
#pragma unroll
        for (int s = 0; s < PER; ++s) {
            const int i = threadIdx.x + s * B;
            if (i < D) {
                rv[s].x -= alpha * qv[s].x;
                rv[s].y -= alpha * qv[s].y;
                const double n2 = rv[s].x * rv[s].x + rv[s].y * rv[s].y;
                v2[0] += mv[s] * n2;
                v2[1] += n2;
            }
        }
        small_reduce<B / kWave, 2>(v2, red);
        const double rz_new = v2[0];
        rr = v2[1];
        if (lead) hist_alpha(st, iters, alpha);
        ++iters;
        bool stop = false;
        if (!finite(rr) || !finite(rz_new)) {
            status = QP_ENONFINITE;
            stop = true;
        } else if (rr <= thresh || iters >= maxit) {
            status = (rr <= thresh) ? QP_OK : QP_ENOCONV;
            stop = true;
        }
        // U += alpha h with this iteration's h; then, unless stopping,
        // h = M r + beta h
        beta = stop ? 0.0 : rz_new / rz;
#pragma unroll
        for (int s = 0; s < PER; ++s) {
            const int i = threadIdx.x + s * B;
            if (i < D) {
                double2 hv = s_h[i];
                double2 u = s_u[i];
                u.x += alpha * hv.x;
                u.y += alpha * hv.y;
                s_u[i] = u;
                if (!stop) {
                    hv.x = mv[s] * rv[s].x + beta * hv.x;
                    hv.y = mv[s] * rv[s].y + beta * hv.y;
                    s_h[i] = hv;
                }
            }
        }
        if (stop) break;
        if (lead) hist_beta(st, iters - 1, beta);
        rz = rz_new;
        __syncthreads();  // the next product reads every entry of h
    }
#pragma unroll
    for (int s = 0; s < PER; ++s) {
        const int i = threadIdx.x + s * B;
        if (i < D) {
            U[i] = s_u[i];
            r[i] = rv[s];
            h[i] = s_h[i];
        }
    }
    if (lead) {
        st->hq = hq;
        st->alpha = alpha;
        st->beta = beta;
        st->rr = rr;
        st->rz[0] = st->rz[1] = rz;
        st->iters = iters;
        st->did_update = 0;
        st->status = status;
        st->done = 1;
    }
}

}  // namespace

hipError_t launch_pcg_wg(int K, const Table *tab, const Table &ht, double *U, double *r, double *h,
                         const double *M, State *st, hipStream_t s)
{
    if (K < 1 || K > kMaxRhs || ht.aniso || ht.half || ht.D > kSmallMax)
        return hipErrorInvalidValue;
    auto c = [](double *v) { return reinterpret_cast<double2 *>(v); };
    switch (ht.d) {
#define QP_CASE(DD)                                                                             \
    case DD:                                                                                     \
        hipLaunchKernelGGL(k_pcg_wg<DD>, dim3(K), dim3(small_block<DD>()), 0, s, tab, c(U),     \
                           c(r), c(h), M, st);                                                   \
        break;
        QP_CASE(1) QP_CASE(2) QP_CASE(3) QP_CASE(4)
#undef QP_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace qp
