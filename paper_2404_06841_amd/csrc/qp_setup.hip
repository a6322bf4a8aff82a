// Setup and single-step kernels: the diagonal preconditioner, the grid
// extrema of the coefficient, corrector right-hand sides, the homogenized
// coefficient and plain dot products.
#include "qp_device.h"

namespace qp {
namespace {

// Storage digits of entry i (last digit fastest) and its signed index; on
// Hermitian half storage entry i is the stored position i, whose grid index
// half_index gives.
__device__ __forceinline__ void digits(const Table *__restrict__ tab, int i, int *ib)
{
    const int N = tab->N;
    int rest = tab->half ? (int)half_index(i, N, tab->n) : i;
    for (int t = tab->n - 1; t >= 0; --t) {
        const int q = div_n(tab, rest);
        ib[t] = rest - q * N;
        rest = q;
    }
}

__device__ __forceinline__ int signed_of(int b, int N) { return (2 * b < N) ? b : b - N; }

// Diagonal preconditioner (eq. precond and its Theorem):
//   kind 0:  M_k = q_kk / ||Q e_k||^2,  q_kk = Ahat_0 |P k|^2,
//            ||Q e_k||^2 = sum_m |Ahat_m|^2 ((P rep(k + m)).(P k))^2
//            (column k has one entry per mode, in row rep(k + m))
//   kind 1:  M_k = 1 / q_kk
// M_0 = 0.  Partials of min_{k != 0} |P k|^2 (dependent columns of P).
// Diagonal coefficient (App. D): q_kk = sum_l Ahat^l_0 (P k)_l^2 and the
// column entry of mode m is sum_l Ahat^l_m (P rep(k + m))_l (P k)_l.
// The problem's modes, coefficients and projection, copied to LDS once per
// workgroup: the set-up kernels read them in their innermost loops with
// indices that vary per mode and axis.
struct SetupLds {
    double P[kMaxD][kMaxN];
    double coefl[kMaxG][kMaxD][2];
    int modes[kMaxG][kMaxN];
};

__device__ __forceinline__ void setup_lds(const Table *__restrict__ tab, SetupLds &L)
{
    for (int e = threadIdx.x; e < kMaxD * kMaxN; e += kBlock) (&L.P[0][0])[e] = (&tab->P[0][0])[e];
    for (int e = threadIdx.x; e < kMaxG * kMaxD * 2; e += kBlock)
        (&L.coefl[0][0][0])[e] = (&tab->coefl[0][0][0])[e];
    for (int e = threadIdx.x; e < kMaxG * kMaxN; e += kBlock)
        (&L.modes[0][0])[e] = (&tab->modes[0][0])[e];
    __syncthreads();
}

__global__ __launch_bounds__(kBlock) void k_precond(const Table *__restrict__ tab, int kind,
                                                    double *__restrict__ M64,
                                                    float *__restrict__ M32,
                                                    double *__restrict__ part)
{
    __shared__ SetupLds L;
    setup_lds(tab, L);
    const int N = tab->N, n = tab->n, d = tab->d, g = tab->g;
    const bool aniso = tab->aniso != 0;
    const int D = tab->D;
    double pkmin[1] = {INFINITY};
    // a grid-stride loop over every entry: the per-entry work is arithmetic,
    // and the launch takes as many workgroups as the partial sums allow
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < D; i += gridDim.x * kBlock) {
        int ib[kMaxN];
        digits(tab, i, ib);
        double pk[kMaxD];
        for (int l = 0; l < d; ++l) {
            double s = 0.0;
            for (int t = 0; t < n; ++t) s += L.P[l][t] * (double)signed_of(ib[t], N);
            pk[l] = s;
        }
        double pk2 = 0.0;
        for (int l = 0; l < d; ++l) pk2 += pk[l] * pk[l];
        double m = 0.0;
        if (i != 0) {
            pkmin[0] = fmin(pkmin[0], pk2);
            double qkk = tab->a0 * pk2;
            if (aniso) {
                qkk = 0.0;
                for (int l = 0; l < d; ++l) qkk += tab->a0l[l] * pk[l] * pk[l];
            }
            if (kind == 1) {
                m = (qkk != 0.0) ? 1.0 / qkk : 0.0;
            } else {
                double col = 0.0;
                for (int r = 0; r < g; ++r) {
                    // signed digits of rep(k + m), shared by every component l
                    double sj[kMaxN];
                    for (int t = 0; t < n; ++t) {
                        int jb = ib[t] + L.modes[r][t];
                        jb += (jb < 0) ? N : 0;
                        jb -= (jb >= N) ? N : 0;
                        sj[t] = (double)signed_of(jb, N);
                    }
                    double w = 0.0, qr = 0.0, qi = 0.0;
                    for (int l = 0; l < d; ++l) {
                        double pj = 0.0;
                        for (int t = 0; t < n; ++t) pj += L.P[l][t] * sj[t];
                        w += pj * pk[l];
                        qr += L.coefl[r][l][0] * (pj * pk[l]);
                        qi += L.coefl[r][l][1] * (pj * pk[l]);
                    }
                    if (aniso) {
                        col += qr * qr + qi * qi;
                    } else {
                        const double a2 = tab->coef[r][0] * tab->coef[r][0] +
                                          tab->coef[r][1] * tab->coef[r][1];
                        col += a2 * w * w;
                    }
                }
                m = (col != 0.0) ? qkk / col : 0.0;
            }
        }
        M64[i] = m;
        M32[i] = (float)m;
    }
    store_partials<1, true>(pkmin, part);
}

// min and -max of A(y) = sum_m Ahat_m exp(i m.y) over y = 2 pi j / N (for a
// diagonal coefficient: over every entry a_l).  The phase m.j is reduced mod N
// exactly in integers before the sine/cosine; for N up to kPhaseTab the
// sines and cosines of the N phases are computed once per workgroup (the same
// calls on the same arguments) and looked up.
constexpr int kPhaseTab = 2048;
__global__ __launch_bounds__(kBlock) void k_extrema(const Table *__restrict__ tab,
                                                    double *__restrict__ part)
{
    __shared__ SetupLds L;
    __shared__ double2 s_sc[kPhaseTab];
    const int N = tab->N, n = tab->n, g = tab->g;
    const bool table = N <= kPhaseTab;
    if (table) {
        for (int j = threadIdx.x; j < N; j += kBlock) {
            double sn, cs;
            sincospi(2.0 * (double)j / (double)N, &sn, &cs);
            s_sc[j] = make_double2(sn, cs);
        }
    }
    setup_lds(tab, L);  // (its barrier also publishes the phase table)
    const int entries = tab->aniso ? tab->d : 1;
    const int D = tab->D;
    double v[2] = {INFINITY, INFINITY};
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < D; i += gridDim.x * kBlock) {
        int ib[kMaxN];
        digits(tab, i, ib);
        double a[kMaxD] = {0.0, 0.0, 0.0, 0.0};
        for (int r = 0; r < g; ++r) {
            long long ph = 0;
            for (int t = 0; t < n; ++t) ph += (long long)L.modes[r][t] * ib[t];
            ph %= N;
            if (ph < 0) ph += N;
            double sn, cs;
            if (table) {
                const double2 sc = s_sc[ph];
                sn = sc.x;
                cs = sc.y;
            } else {
                sincospi(2.0 * (double)ph / (double)N, &sn, &cs);
            }
            for (int l = 0; l < entries; ++l)
                a[l] += L.coefl[r][l][0] * cs - L.coefl[r][l][1] * sn;
        }
        for (int l = 0; l < entries; ++l) {
            v[0] = fmin(v[0], a[l]);
            v[1] = fmin(v[1], -a[l]);
        }
    }
    store_partials<2, true>(v, part);
}

template <int NV, bool MIN>
__global__ __launch_bounds__(kBlock) void k_finalize(const double *__restrict__ part, int nb,
                                                     double *__restrict__ out, int negate_second)
{
    double v[NV];
    load_totals<NV, MIN>(part, nb, v);
    if (threadIdx.x == 0) {
        for (int k = 0; k < NV; ++k) out[k] = (k == 1 && negate_second) ? -v[k] : v[k];
    }
}

// The modes whose storage index lies in [begin, end), in increasing order of
// r (at most kMaxG = 64, so wave 0 finds them with one ballot): the
// corrector sources below test each entry against these alone.
struct ChunkModes {
    int r[kMaxG];
    int idx[kMaxG];
    int count;
};
static_assert(kMaxG <= kWave, "one ballot covers every mode");

__device__ __forceinline__ void chunk_modes(const Table *__restrict__ tab, int begin, int end,
                                            ChunkModes &cm)
{
    if (threadIdx.x < kWave) {
        const int r = threadIdx.x;
        const int ix = r < tab->g ? tab->midx[r] : -1;
        const bool in = r < tab->g && ix >= begin && ix < end;
        const unsigned long long mask = __ballot(in);
        if (in) {
            const int slot = __popcll(mask & ((1ull << r) - 1ull));
            cm.r[slot] = r;
            cm.idx[slot] = ix;
        }
        if (r == 0) cm.count = __popcll(mask);
    }
    __syncthreads();
}

// F_k = i (P k)_j Ahat_k on the modes, 0 elsewhere (each entry written once);
// for a diagonal coefficient Ahat is a_j's (the source d a_j / d x_j, App. D).
__global__ __launch_bounds__(kBlock) void k_corrector_rhs(const Table *__restrict__ tab, int j,
                                                          double2 *__restrict__ F)
{
    __shared__ ChunkModes cm;
    int begin, end;
    chunk_of_block(tab, begin, end);
    chunk_modes(tab, begin, end, cm);
    const int nm = cm.count;
    for (int i = begin + threadIdx.x; i < end; i += kBlock) {
        double2 v = make_double2(0.0, 0.0);
        for (int c = 0; c < nm; ++c) {
            if (cm.idx[c] == i) {
                const int r = cm.r[c];
                const double s = tab->Pm[r][j];
                v.x += -s * tab->coefl[r][j][1];
                v.y += s * tab->coefl[r][j][0];
            }
        }
        F[i] = v;
    }
}

// The sources of correctors 0 .. K-1 in one pass (F + j D), and, when part
// is given, the partial sums of ||f'_j||^2 (zero frequency excluded) for the
// FP32-IR unit, as the separate norm pass would store them.
template <int K>
__global__ __launch_bounds__(kBlock) void k_corrector_rhs_all(const Table *__restrict__ tab,
                                                              double2 *__restrict__ F,
                                                              double *__restrict__ part)
{
    __shared__ ChunkModes cm;
    const size_t D = tab->D;
    int begin, end;
    chunk_of_block(tab, begin, end);
    chunk_modes(tab, begin, end, cm);
    const int nm = cm.count;
    double acc[K];
#pragma unroll
    for (int j = 0; j < K; ++j) acc[j] = 0.0;
    for (int i = begin + threadIdx.x; i < end; i += kBlock) {
        double2 v[K];
#pragma unroll
        for (int j = 0; j < K; ++j) v[j] = make_double2(0.0, 0.0);
        for (int c = 0; c < nm; ++c) {
            if (cm.idx[c] == i) {
                const int r = cm.r[c];
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    const double s = tab->Pm[r][j];
                    v[j].x += -s * tab->coefl[r][j][1];
                    v[j].y += s * tab->coefl[r][j][0];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < K; ++j) {
            F[(size_t)j * D + i] = v[j];
            if (i != 0) acc[j] += v[j].x * v[j].x + v[j].y * v[j].y;
        }
    }
    if (!part) return;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        double a[1] = {acc[j]};
        store_partials<1>(a, part + j * kPartStride);
    }
}

// A*_ij = Ahat_0 delta_ij + mean_N{ a d_i chi_j }
//       = Ahat_0 delta_ij + sum_m Ahat_m i (P(-m))_i chi_j[C(-m)]
// (the discrete mean keeps the frequency pairs whose sum is 0 mod N).  For a
// diagonal coefficient the integrand is a_i (delta_ij + d_i chi_j), so Ahat is
// a_i's (App. D, eqs. homcoefficient11-22).
__global__ void k_astar(const Table *__restrict__ tab, const double2 *__restrict__ chi,
                        double *__restrict__ out)
{
    const int d = tab->d, g = tab->g;
    const int e = threadIdx.x;
    if (e >= d * d) return;
    const int i = e / d, j = e % d;
    const double2 *cj = chi + (size_t)j * tab->D;
    double re = (i == j) ? tab->a0l[i] : 0.0;
    double im = 0.0;
    for (int r = 0; r < g; ++r) {
        double2 c = cj[tab->nidx[r]];
        if (tab->nconj[r]) c.y = -c.y;  // half storage: chi at -m is conj(chi at m)
        const double ar = tab->coefl[r][i][0], ai = tab->coefl[r][i][1];
        const double pr = ar * c.x - ai * c.y;  // Ahat_m chi
        const double pi = ar * c.y + ai * c.x;
        const double s = tab->Pm[r][i];  // i (P(-m))_i = -i s
        re += s * pi;
        im -= s * pr;
    }
    out[e] = re;
    out[d * d + e] = im;
}

__global__ __launch_bounds__(kBlock) void k_dot(const Table *__restrict__ tab,
                                                const double2 *__restrict__ x,
                                                const double2 *__restrict__ y,
                                                double *__restrict__ part)
{
    int begin, end;
    chunk_of_block(tab, begin, end);
    double acc[1] = {0.0};
    for (int i = begin + threadIdx.x; i < end; i += kBlock) {
        const double2 a = x[i], b = y[i];
        acc[0] += a.x * b.x + a.y * b.y;
    }
    store_partials<1>(acc, part);
}

__global__ __launch_bounds__(kBlock) void k_multi_index(const Table *__restrict__ tab,
                                                        int32_t *__restrict__ k)
{
    const int N = tab->N, n = tab->n;
    int begin, end;
    chunk_of_block(tab, begin, end);
    for (int i = begin + threadIdx.x; i < end; i += kBlock) {
        int ib[kMaxN];
        digits(tab, i, ib);
        for (int t = 0; t < n; ++t) k[(size_t)i * n + t] = signed_of(ib[t], N);
    }
}

}  // namespace

// Grid of the arithmetic set-up kernels: one entry per thread up to the
// partial-sum limit (grid-stride beyond it).
static int setup_grid(const Table &ht)
{
    return (int)std::min<int64_t>(kMaxBlocks, std::max<int64_t>(1, ((int64_t)ht.D + kBlock - 1) / kBlock));
}

hipError_t launch_precond(const Table *tab, const Table &ht, int kind, double *M64, float *M32,
                          const Parts &parts, double *out, hipStream_t s)
{
    const int nb = setup_grid(ht);
    hipLaunchKernelGGL(k_precond, dim3(nb), dim3(kBlock), 0, s, tab, kind, M64, M32, parts.c);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_finalize<1, true>), dim3(1), dim3(kBlock), 0, s, (const double *)parts.c,
                       nb, out, 0);
    return hipGetLastError();
}

hipError_t launch_extrema(const Table *tab, const Table &ht, const Parts &parts, double *out,
                          hipStream_t s)
{
    const int nb = setup_grid(ht);
    hipLaunchKernelGGL(k_extrema, dim3(nb), dim3(kBlock), 0, s, tab, parts.c);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_finalize<2, true>), dim3(1), dim3(kBlock), 0, s, (const double *)parts.c,
                       nb, out, 1);
    return hipGetLastError();
}

hipError_t launch_corrector_rhs(const Table *tab, const Table &ht, int j, double *F, hipStream_t s)
{
    hipLaunchKernelGGL(k_corrector_rhs, dim3(ht.nblocks), dim3(kBlock), 0, s, tab, j,
                       reinterpret_cast<double2 *>(F));
    return hipGetLastError();
}

hipError_t launch_corrector_rhs_all(const Table *tab, const Table &ht, int K, double *F,
                                    const Parts *parts, hipStream_t s)
{
    double2 *f = reinterpret_cast<double2 *>(F);
    double *c = parts ? parts->c : nullptr;
    switch (K) {
#define QP_K(KK)                                                                                \
    case KK:                                                                                     \
        hipLaunchKernelGGL(k_corrector_rhs_all<KK>, dim3(ht.nblocks), dim3(kBlock), 0, s, tab, f, \
                           c);                                                                   \
        break;
        QP_K(1) QP_K(2) QP_K(3) QP_K(4)
#undef QP_K
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_astar(const Table *tab, const Table &ht, const double *chi, double *out,
                        hipStream_t s)
{
    (void)ht;
    hipLaunchKernelGGL(k_astar, dim3(1), dim3(64), 0, s, tab, reinterpret_cast<const double2 *>(chi),
                       out);
    return hipGetLastError();
}

hipError_t launch_dot(const Table *tab, const Table &ht, const double *x, const double *y,
                      const Parts &parts, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_dot, dim3(ht.nblocks), dim3(kBlock), 0, s, tab,
                       reinterpret_cast<const double2 *>(x), reinterpret_cast<const double2 *>(y),
                       parts.c);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_finalize<1, false>), dim3(1), dim3(kBlock), 0, s, (const double *)parts.c,
                       ht.nblocks, out, 0);
    return hipGetLastError();
}

hipError_t launch_multi_index(const Table *tab, const Table &ht, int32_t *k, hipStream_t s)
{
    hipLaunchKernelGGL(k_multi_index, dim3(ht.nblocks), dim3(kBlock), 0, s, tab, k);
    return hipGetLastError();
}

}  // namespace qp
