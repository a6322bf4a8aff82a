// Stiffness product of the projection method on gfx950:
//
//   y_k = sum_{m in S} Ahat_m (P k).(P j) x_j,   j = rep(k - m),   k != 0,
//
// (eq. n-discrete: the column k_U with k_V -_N k_U = m is the representative of
// k - m in K_N^n; W = (P k_V).(P k_U) uses both representatives).  Matrix free:
// only the g modes are read; every W is recomputed.  The product is memory
// bound, so there is no matrix-core path: the work is organised so that almost
// every (entry, mode) pair costs one load and a handful of FMAs.
//
// Work decomposition.  A "line" is a run of N entries along the last (fastest)
// axis.  A wave owns a tile of S lines x P positions (S lines consecutive in
// axis n-2 of one plane when N <= 64, else one 64-wide piece of a line), so
// lanes differ only in their last digit and their slot digit (axis n-2);
// every other digit is uniform over the wave.
//
// Modes are sorted by their last component m_{n-1} into groups.  For a group,
// a lane's wrapped column and the correction of W for crossing the +-N/2 face
// of the last axis depend only on the lane's position, so they are computed
// once per workgroup and kept in LDS.  When only the last axis wraps,
//   W = |P k|^2 - (P k).(P m) + c N (P k).p_{n-1},   c in {-1, 0, 1}.
//
// A per-tile bit mask (OR of per-digit masks prepared on the host) marks the
// modes whose neighbour wraps in another axis for some lane.  Unmarked modes
// read x at a wave-uniform base plus the lane's cached column (fast path);
// marked modes also correct the address and W for the axes they move along.
//
// Tile order: each XCD owns a contiguous eighth of the tiles, and its
// workgroups sweep that range together (adjacent workgroups take adjacent
// tiles), so the neighbours of the current front are in the XCD's L2 or in
// the shared Infinity Cache.
#include "qp_device.h"

namespace qp {
namespace {

constexpr int kGC = 8;     // groups cached in LDS
constexpr int kChunk = 4;  // loads of a group issued before the first is consumed

// Mode record as staged in LDS (read back with broadcast loads).
struct LRec {
    double w[kMaxD];  // Re(Ahat) P m for real coefficients, P m otherwise
    double c[2];      // Ahat_m
    int lro;          // element offset of the source line
    int nz;           // axes t < n-1 with m_t != 0
    short mt[kMaxN];  // m
};

__device__ __forceinline__ int signed_digit(int b, int N) { return (2 * b < N) ? b : b - N; }

// Lane geometry for the group with last-axis offset delta at absolute
// position pos (0 <= pos < N): wrapped column and the face factor c with
// rep(k - m)_{n-1} = k_{n-1} - delta + c N.
__device__ __forceinline__ void group_geom(int N, int delta, int pos, int &colw, int &c)
{
    int col = pos - delta;
    col += (col < 0) ? N : 0;
    col -= (col >= N) ? N : 0;
    colw = col;
    const int j = signed_digit(col, N);
    const int k = signed_digit(pos, N);
    c = (j - (k - delta)) / N;
}

template <typename T, int DT, int EPI, bool REAL>
__global__ __launch_bounds__(kBlock) void k_matvec(const Table *__restrict__ tab,
                                                   const ModeRec *__restrict__ recs,
                                                   const uint64_t *__restrict__ wm,
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
    __shared__ int2 s_geo[kGC][kBlock];
    __shared__ LRec s_rec[kMaxG];

    const int N = tab->N;
    const int n = tab->n;
    const int ng = tab->ngroups;
    const int P = tab->lanes_p;
    const int S = tab->tile_s;
    const int lane = threadIdx.x % kWave;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int s = lane / P;
    const int p = lane - s * P;
    const bool planes = (n >= 2) && (N <= kWave);
    const bool cached = (N <= kWave);  // tiles then start at position 0
    if (cached) {
        for (int g = 0; g < ng && g < kGC; ++g) {
            int colw, c;
            group_geom(N, tab->gdelta[g], p, colw, c);
            s_geo[g][threadIdx.x] = make_int2(s * N + colw, c);
        }
    }
    for (int r = threadIdx.x; r < tab->g; r += kBlock) {
        const ModeRec &R = recs[r];
        LRec L;
#pragma unroll
        for (int l = 0; l < kMaxD; ++l) L.w[l] = REAL ? R.cpm[l] : R.pm[l];
        L.c[0] = R.c[0];
        L.c[1] = R.c[1];
        L.lro = (int)R.lroffN;
        L.nz = R.nz;
#pragma unroll
        for (int t = 0; t < kMaxN; ++t) L.mt[t] = R.mt[t];
        s_rec[r] = L;
    }
    __syncthreads();
    const double inv_unit = (EPI == EPI_RESID) ? st->inv_unit : 1.0;
    const T NT = (T)N;

    // XCD-front order over the tiles
    const int nb = gridDim.x;
    const int b = blockIdx.x;
    const bool by_xcd = (nb % 8 == 0);
    const int xcd = by_xcd ? b % 8 : 0;
    const int nloc = by_xcd ? nb / 8 : nb;
    const int loc = by_xcd ? b / 8 : b;
    const int per = by_xcd ? (tab->ntiles + 7) / 8 : tab->ntiles;
    const int xbeg = xcd * per;
    const int xend = min(xbeg + per, tab->ntiles);
    double dots[2] = {0.0, 0.0};

    for (int kt = 0;; ++kt) {
        const int tile = xbeg + (kt * nloc + loc) * kWaves + wave;
        if (tile >= xend) break;
        // ---- tile geometry (uniform) ----
        int L0, St, p0, slot0, plane;
        const int tpu = tab->tiles_per_unit;
        if (planes) {
            plane = tile / tpu;
            slot0 = (tile - plane * tpu) * S;
            St = min(S, N - slot0);
            L0 = plane * N + slot0;
            p0 = 0;
        } else {
            L0 = tile / tpu;
            p0 = (tile - L0 * tpu) * kWave;
            St = 1;
            plane = (n >= 2) ? div_n(tab, L0) : 0;
            slot0 = (n >= 2) ? L0 - plane * N : 0;
        }
        const bool active = (s < St) && (p0 + p < N);

        // ---- digits: last (per lane), slot (per lane), the rest (uniform) ----
        const int pos = p0 + p;
        const int kpos = signed_digit(pos, N);
        const int ibs = (n >= 2) ? slot0 + s : 0;
        const int ks = signed_digit(ibs, N);
        int ibu[kMaxN], ku[kMaxN];
        {
            int rest = plane;
#pragma unroll
            for (int t = kMaxN - 3; t >= 0; --t) {
                ibu[t] = 0;
                ku[t] = 0;
                if (t <= n - 3) {
                    const int qt = div_n(tab, rest);
                    ibu[t] = rest - qt * N;
                    ku[t] = signed_digit(ibu[t], N);
                    rest = qt;
                }
            }
        }
        // ---- P k, |P k|^2, q_t = (P k).p_t ----
        T pk[DT];
        T s2 = 0;
#pragma unroll
        for (int l = 0; l < DT; ++l) {
            T v = (T)tab->P[l][n - 1] * (T)kpos;
            if (n >= 2) v += (T)tab->P[l][n - 2] * (T)ks;
#pragma unroll
            for (int t = 0; t < kMaxN - 2; ++t)
                if (t <= n - 3) v += (T)tab->P[l][t] * (T)ku[t];
            pk[l] = v;
            s2 += v * v;
        }
        T q_last = 0, q_slot = 0;
        T qu[kMaxN];
#pragma unroll
        for (int l = 0; l < DT; ++l) {
            q_last += pk[l] * (T)tab->P[l][n - 1];
            if (n >= 2) q_slot += pk[l] * (T)tab->P[l][n - 2];
        }
#pragma unroll
        for (int t = 0; t < kMaxN - 2; ++t) {
            T v = 0;
            if (t <= n - 3) {
#pragma unroll
                for (int l = 0; l < DT; ++l) v += pk[l] * (T)tab->P[l][t];
            }
            qu[t] = v;
        }
        const T cq = NT * q_last;

        // ---- modes whose neighbour wraps in an axis other than the last ----
        uint64_t wmask = 0;
        if (n >= 2) {
#pragma unroll
            for (int t = 0; t < kMaxN - 2; ++t)
                if (t <= n - 3) wmask |= wm[t * N + ibu[t]];
            for (int ss = 0; ss < St; ++ss) wmask |= wm[(n - 2) * N + slot0 + ss];
        }

        const int tbase = L0 * N;  // element index of the tile's first line
        T acc_re = 0, acc_im = 0;
        if (active) {
            for (int g = 0; g < ng; ++g) {
                int voff, c;
                if (cached && g < kGC) {
                    const int2 geo = s_geo[g][threadIdx.x];
                    voff = geo.x;
                    c = geo.y;
                } else {
                    int colw;
                    group_geom(N, tab->gdelta[g], pos, colw, c);
                    voff = s * N + colw;
                }
                const T base = s2 + (T)c * cq;
                const int lane_idx = tbase + voff;
                const int r1 = tab->gstart[g + 1];
                for (int rb = tab->gstart[g]; rb < r1; rb += kChunk) {
                    cplx_t<T> u[kChunk];
                    T w[kChunk];
#pragma unroll
                    for (int k = 0; k < kChunk; ++k) {
                        const int rr = rb + k;
                        if (rr >= r1) break;
                        const LRec &R = s_rec[rr];
                        // REAL: w = Re(Ahat) W; otherwise w = W
                        T wv = REAL ? (T)R.c[0] * base : base;
#pragma unroll
                        for (int l = 0; l < DT; ++l) wv -= pk[l] * (T)R.w[l];
                        int idx = lane_idx - R.lro;
                        if ((wmask >> rr) & 1ull) {
                            // correct address and W for the axes this mode moves along
                            T corr = 0;
                            const int nz = R.nz;
#pragma unroll
                            for (int t = 0; t < kMaxN - 1; ++t) {
                                if (t > n - 2 || !((nz >> t) & 1)) continue;
                                const int m = R.mt[t];
                                const int ib = (t < n - 2) ? ibu[t] : ibs;
                                const int kv = (t < n - 2) ? ku[t] : ks;
                                const T qt = (t < n - 2) ? qu[t] : q_slot;
                                int jb = ib - m;
                                const int step = (int)tab->lstride[t] * N * N;
                                if (jb < 0) {
                                    jb += N;
                                    idx += step;
                                } else if (jb >= N) {
                                    jb -= N;
                                    idx -= step;
                                }
                                corr += (T)(signed_digit(jb, N) - (kv - m)) * qt;
                            }
                            wv += REAL ? (T)R.c[0] * corr : corr;
                        }
                        u[k] = x[idx];
                        w[k] = wv;
                    }
#pragma unroll
                    for (int k = 0; k < kChunk; ++k) {
                        const int rr = rb + k;
                        if (rr >= r1) break;
                        if (REAL) {
                            acc_re += w[k] * u[k].x;
                            acc_im += w[k] * u[k].y;
                        } else {
                            const LRec &R = s_rec[rr];
                            const T cr = (T)R.c[0] * w[k];
                            const T ci = (T)R.c[1] * w[k];
                            acc_re += cr * u[k].x - ci * u[k].y;
                            acc_im += cr * u[k].y + ci * u[k].x;
                        }
                    }
                }
            }
        }
        if (active) {
            const size_t i = (size_t)(L0 + s) * N + pos;
            if (i == 0) {
                acc_re = 0;
                acc_im = 0;
            }
            if (EPI == EPI_RESID) {
                // replaced residual of FP32-IR: (f' - Q x) / ||F'|| as float
                const double2 fv = f[i];
                const double rx = (i != 0) ? (fv.x - (double)acc_re) * inv_unit : 0.0;
                const double ry = (i != 0) ? (fv.y - (double)acc_im) * inv_unit : 0.0;
                const float2 o = make_float2((float)rx, (float)ry);
                static_cast<float2 *>(yv)[i] = o;
                dots[0] += (double)M32[i] * ((double)o.x * (double)o.x + (double)o.y * (double)o.y);
                dots[1] += rx * rx + ry * ry;
            } else {
                cplx_t<T> o;
                o.x = acc_re;
                o.y = acc_im;
                static_cast<cplx_t<T> *>(yv)[i] = o;
                if (EPI == EPI_ALPHA) {
                    const cplx_t<T> xi = x[i];
                    dots[0] += (double)xi.x * (double)acc_re + (double)xi.y * (double)acc_im;
                }
            }
        }
    }
    if (EPI == EPI_ALPHA) {
        double v[1] = {dots[0]};
        store_partials<1>(v, part);
        if (exec && blockIdx.x == 0 && threadIdx.x == 0) *exec = 1;
    } else if (EPI == EPI_RESID) {
        store_partials<2>(dots, part);
        if (exec && blockIdx.x == 0 && threadIdx.x == 0) *exec = 1;
    }
}

template <typename T, int EPI, bool REAL>
hipError_t dispatch(const Table *tab, const Table &ht, const ModeRec *recs, const uint64_t *wm,
                    const void *x, void *y, const double *f, const float *M32, double *part,
                    State *st, int *exec, hipStream_t s)
{
    const dim3 grid(ht.nb_mv), block(kBlock);
    auto X = static_cast<const cplx_t<T> *>(x);
    auto Fv = reinterpret_cast<const double2 *>(f);
    switch (ht.d) {
#define QP_CASE(DD)                                                                             \
    case DD:                                                                                     \
        hipLaunchKernelGGL((k_matvec<T, DD, EPI, REAL>), grid, block, 0, s, tab, recs, wm, X, y, \
                           Fv, M32, part, st, exec);                                             \
        break;
        QP_CASE(1) QP_CASE(2) QP_CASE(3) QP_CASE(4)
#undef QP_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int EPI>
hipError_t dispatch_coef(const Table *tab, const Table &ht, const ModeRec *recs, const uint64_t *wm,
                         const void *x, void *y, const double *f, const float *M32, double *part,
                         State *st, int *exec, hipStream_t s)
{
    if (ht.real_coef)
        return dispatch<T, EPI, true>(tab, ht, recs, wm, x, y, f, M32, part, st, exec, s);
    return dispatch<T, EPI, false>(tab, ht, recs, wm, x, y, f, M32, part, st, exec, s);
}

}  // namespace

hipError_t launch_matvec(int prec, int epi, const Table *tab, const Table &ht, const ModeRec *recs,
                         const uint64_t *wm, const void *x, void *y, const double *f,
                         const float *M32, const Parts &parts, State *st, int *exec, hipStream_t s)
{
    if (prec == F64) {
        if (epi == EPI_NONE)
            return dispatch_coef<double, EPI_NONE>(tab, ht, recs, wm, x, y, f, M32, parts.a, st, exec, s);
        if (epi == EPI_ALPHA)
            return dispatch_coef<double, EPI_ALPHA>(tab, ht, recs, wm, x, y, f, M32, parts.a, st, exec, s);
        return dispatch_coef<double, EPI_RESID>(tab, ht, recs, wm, x, y, f, M32, parts.b, st, exec, s);
    }
    if (epi == EPI_NONE)
        return dispatch_coef<float, EPI_NONE>(tab, ht, recs, wm, x, y, f, M32, parts.a, st, exec, s);
    if (epi == EPI_ALPHA)
        return dispatch_coef<float, EPI_ALPHA>(tab, ht, recs, wm, x, y, f, M32, parts.a, st, exec, s);
    return hipErrorInvalidValue;  // the replaced residual is always computed in FP64
}

}  // namespace qp
