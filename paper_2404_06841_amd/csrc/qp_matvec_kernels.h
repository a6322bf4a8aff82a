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
// With s = rep(k - m) = k - m + N c (c_t in {-1, 0, 1} per axis),
//   W = (P k).(P s) = |P k|^2 - (P k).(P m) + N sum_t c_t (P k).p_t.
// Lanes of a tile share every digit but the last and (for multi-line tiles)
// the slot digit.  Per unit (the tiles sharing those uniform digits: a plane,
// or a line when N > 64) the workgroup folds the uniform axes' wraps into one
// record per mode: P m' = P m - N sum_{t uniform} c_t p_t and the uniform part
// of the neighbour's address.  Per mode and lane, a table built once per
// workgroup holds the wrapped last-axis column and its face factor.  Modes
// whose neighbour crosses a slot-axis boundary for some lane of the tile (a
// host-prepared mask per tile row) are corrected per lane.  Neighbour loads
// are issued in chunks of up to Inflight<T> before the first is consumed; the
// staged records are padded to a multiple of 4 with zero-weight copies of
// m = 0, which the walk over the records (walk_records) never gathers.
//
// Unit order: each XCD owns a contiguous eighth of the units, and its
// workgroups sweep that range together (adjacent workgroups take adjacent
// units), so the neighbours of the current front are in the XCD's L2 or in
// the shared Infinity Cache.
#pragma once

#include <hip/hip_ext.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "qp_chunk_walk.h"
#include "qp_device.h"

namespace qp {
namespace {

template <typename T>
struct Inflight;
#ifndef QP_INFLIGHT_F32
#define QP_INFLIGHT_F32 16
#endif
#ifndef QP_INFLIGHT_F64
#define QP_INFLIGHT_F64 8
#endif
template <>
struct Inflight<float> {
    static constexpr int v = QP_INFLIGHT_F32;
};
template <>
struct Inflight<double> {
    static constexpr int v = QP_INFLIGHT_F64;
};

// Fused multiply-add written out, so that every instantiation of the product
// (all chunk sizes of the record walk, 32- and 64-bit gathers) rounds each
// weight and each accumulation step the same way, whatever the compiler
// would contract on its own.
__device__ __forceinline__ float fmac(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmac(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Static mode data, staged once per workgroup.
template <typename T, int DT>
struct SRec {
    T pm[DT];         // P m
    T c[2];           // Ahat_m
    T cl[DT][2];      // Ahat of a_l at m (diagonal coefficient)
    short mt[kMaxN];  // m
};

// Mode data of the current unit: uniform-axis wraps folded in.
template <typename T, int DT>
struct alignas(16) URec {
    T apm[DT];  // a P m'
    T a;        // Re(Ahat_m) for real coefficients, else 1 (0 for padding)
    T cr, ci;   // Ahat_m for complex coefficients (0 for padding)
    int lb;     // neighbour's element offset: uniform axes, minus m_slot N
    int mslot;  // m_{n-2} (0 when the slot digit is uniform)
};

__device__ __forceinline__ int signed_digit(int b, int N) { return (2 * b < N) ? b : b - N; }

// Wrapped last-axis column of the neighbour and the face factor c with
// rep(k - m)_{n-1} = k_{n-1} - delta + c N, at absolute position pos
// (0 <= pos < N); K_N = [lo, hi] per axis.
__device__ __forceinline__ void last_axis(int N, int lo, int hi, int delta, int pos, int &colw,
                                          int &c)
{
    int col = pos - delta;
    col += (col < 0) ? N : 0;
    col -= (col >= N) ? N : 0;
    colw = col;
    const int kd = signed_digit(pos, N) - delta;
    c = (kd < lo) ? 1 : ((kd > hi) ? -1 : 0);
}

template <typename T, int DT, int EPI, bool REAL, bool AN>
__global__ __launch_bounds__(kBlock) void k_matvec(const Table *__restrict__ tab,
                                                   const ModeRec *__restrict__ recs,
                                                   const cplx_t<T> *__restrict__ x,
                                                   void *__restrict__ yv,
                                                   const double2 *__restrict__ f,
                                                   const float *__restrict__ M32,
                                                   double *__restrict__ part,
                                                   State *__restrict__ st,
                                                   int *__restrict__ exec)
{
    if (EPI == EPI_ALPHA && (st->done || st->pause)) return;
    if (EPI == EPI_RESID && !st->replace) return;  // replaced only once paused (fold decides)
    constexpr int KC = Inflight<T>::v;
    // per padded mode and lane: (wrapped column, face factor as float); gp * kWave
    // entries of dynamic LDS when N <= kWave
    extern __shared__ int2 s_geo[];
    using LRec = typename std::conditional<AN, UnitRecA<T, DT>, URec<T, DT>>::type;
    __shared__ SRec<T, DT> s_mode[kMaxG];
    __shared__ LRec s_unit[kMaxG];
    __shared__ T s_p[kMaxN][DT];   // P[l][t]
    __shared__ T s_np[kMaxN][DT];  // N P[l][t]

    const int N = tab->N;
    const int n = tab->n;
    const int g = tab->g;
    const int gp = (g + 3) & ~3;  // padded mode count
    const int zs = tab->zero_sorted;
    const int P = tab->lanes_p;
    const int S = tab->tile_s;
    const int tpu = tab->tiles_per_unit;
    const int lane = threadIdx.x % kWave;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int s = lane / P;
    const int p = lane - s * P;
    const bool slot_lanes = S > 1;  // tiles of S lines of a plane: lanes differ in axis n-2
    const int nu = (n == 1) ? 0 : (slot_lanes ? n - 2 : n - 1);  // wave-uniform axes
    const bool cached = (N <= kWave);  // tiles then start at position 0
    const int lo = -(N / 2), hi = N - 1 - N / 2;  // K_N = [lo, hi] per axis

    for (int r = threadIdx.x; r < g; r += kBlock) {
        const ModeRec &R = recs[r];
        SRec<T, DT> M;
#pragma unroll
        for (int l = 0; l < DT; ++l) M.pm[l] = (T)R.pm[l];
        M.c[0] = (T)R.c[0];
        M.c[1] = (T)R.c[1];
#pragma unroll
        for (int l = 0; l < DT; ++l) {
            M.cl[l][0] = (T)R.cl[l][0];
            M.cl[l][1] = (T)R.cl[l][1];
        }
#pragma unroll
        for (int t = 0; t < kMaxN; ++t) M.mt[t] = R.mt[t];
        s_mode[r] = M;
    }
    if (cached) {
        // entry r * kWave + lane belongs to the thread of wave r % kWaves,
        // which loads the last-axis shifts of all its modes at once
        constexpr int kPer = ((kMaxG + 3) & ~3) / kWaves;
        const int pl = lane - (lane / P) * P;  // position of this lane
        int mt[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int r = wave + k * kWaves;
            mt[k] = r < g ? recs[r].mt[n - 1] : 0;
        }
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int r = wave + k * kWaves;
            if (r >= gp) break;
            int colw, c;
            last_axis(N, lo, hi, mt[k], pl, colw, c);
            s_geo[r * kWave + lane] = make_int2(colw, __float_as_int((float)c));
        }
    }
    if (threadIdx.x < kMaxN * DT) {
        const int t = threadIdx.x / DT, l = threadIdx.x - (threadIdx.x / DT) * DT;
        const T v = (t < n) ? (T)tab->P[l][t] : (T)0;
        s_p[t][l] = v;
        s_np[t][l] = (T)N * v;
    }
    __syncthreads();
    const double inv_unit = (EPI == EPI_RESID) ? st->inv_unit : 1.0;

    // Work items: (unit, group of kWaves tiles of the unit), in XCD-front order.
    const int qpu = (tpu + kWaves - 1) / kWaves;
    const int nitems = (tab->ntiles / tpu) * qpu;
    const int nb = gridDim.x;
    const int b = blockIdx.x;
    const bool by_xcd = (nb % 8 == 0);
    const int xcd = by_xcd ? b % 8 : 0;
    const int nloc = by_xcd ? nb / 8 : nb;
    const int loc = by_xcd ? b / 8 : b;
    const int per = by_xcd ? (nitems + 7) / 8 : nitems;
    const int ibeg = xcd * per;
    const int iend = min(ibeg + per, nitems);
    double dots[2] = {0.0, 0.0};

    for (int item = ibeg + loc; item < iend; item += nloc) {
        const int unit = item / qpu;
        const int tl = (item - unit * qpu) * kWaves + wave;
        // ---- uniform digits of the unit (axes 0 .. nu-1) ----
        int ibu[kMaxN - 1], ku[kMaxN - 1];
        {
            int rest = unit;
#pragma unroll
            for (int t = kMaxN - 2; t >= 0; --t) {
                ibu[t] = 0;
                ku[t] = 0;
                if (t < nu) {
                    const int qt = div_n(tab, rest);
                    ibu[t] = rest - qt * N;
                    ku[t] = signed_digit(ibu[t], N);
                    rest = qt;
                }
            }
        }
        // ---- unit records (thread r prepares sorted mode r) ----
        if ((int)threadIdx.x < gp) {
            const int r = threadIdx.x;
            const int rs = (r < g) ? r : zs;  // padding: the zero mode with weight 0
            const SRec<T, DT> &M = s_mode[rs];
            T v[DT];
#pragma unroll
            for (int l = 0; l < DT; ++l) v[l] = M.pm[l];
            int lb = 0;
#pragma unroll
            for (int t = 0; t < kMaxN - 1; ++t) {
                if (t < nu) {
                    const int m = M.mt[t];
                    int jb = ibu[t] - m;
                    jb += (jb < 0) ? N : 0;
                    jb -= (jb >= N) ? N : 0;
                    lb += jb * tab->stride[t];
                    const int kd = ku[t] - m;
                    const T c = (kd < lo) ? (T)1 : ((kd > hi) ? (T)-1 : (T)0);
#pragma unroll
                    for (int l = 0; l < DT; ++l) v[l] -= c * s_np[t][l];
                }
            }
            LRec U;
            U.mslot = slot_lanes ? (int)M.mt[n - 2] : 0;
            U.lb = lb - U.mslot * N;
            if constexpr (AN) {
#pragma unroll
                for (int l = 0; l < DT; ++l) {
                    U.pmw[l] = v[l];
                    U.ar[l] = (r >= g) ? (T)0 : M.cl[l][0];
                    U.ai[l] = (r >= g) ? (T)0 : M.cl[l][1];
                }
            } else {
                T a = REAL ? M.c[0] : (T)1;
                U.cr = M.c[0];
                U.ci = M.c[1];
                if (r >= g) {
                    a = 0;
                    U.cr = 0;
                    U.ci = 0;
                }
                U.a = a;
#pragma unroll
                for (int l = 0; l < DT; ++l) U.apm[l] = a * v[l];
            }
            s_unit[r] = U;
        }
        T pku[DT];  // P k over the uniform axes
#pragma unroll
        for (int l = 0; l < DT; ++l) {
            T v = 0;
#pragma unroll
            for (int t = 0; t < kMaxN - 1; ++t)
                if (t < nu) v += s_p[t][l] * (T)ku[t];
            pku[l] = v;
        }
        __syncthreads();

        if (tl < tpu) {
            // ---- tile geometry ----
            int L0, St, p0, slot0;
            if (slot_lanes) {
                slot0 = tl * S;
                St = min(S, N - slot0);
                L0 = unit * N + slot0;
                p0 = 0;
            } else {
                L0 = unit;
                p0 = tl * kWave;
                St = 1;
                slot0 = 0;
            }
            // Lanes outside the tile run the same loop on clamped coordinates
            // (their loads stay in bounds) and store nothing.
            const bool active = (s < St) && (p0 + p < N);
            const int se = (s < St) ? s : 0;
            const int pos = min(p0 + p, N - 1);
            const int ibs = slot0 + se;
            const int lane_line = (slot_lanes ? ibs : 0) * N;
            const int kpos = signed_digit(pos, N);
            const int ks = signed_digit(ibs, N);
            // ---- P k, |P k|^2, N (P k).p_t for the per-lane axes ----
            T pk[DT];
            T s2 = 0;
#pragma unroll
            for (int l = 0; l < DT; ++l) {
                T v = pku[l] + s_p[n - 1][l] * (T)kpos;
                if (slot_lanes) v += s_p[n - 2][l] * (T)ks;
                pk[l] = v;
                s2 += v * v;
            }
            T cq = 0, cqs = 0;
            T sq[DT], ql[DT], qs[DT];  // per component (diagonal coefficient)
            const int ns = slot_lanes ? n - 2 : 0;  // slot axis (only read for slot lanes)
#pragma unroll
            for (int l = 0; l < DT; ++l) {
                if constexpr (AN) {
                    sq[l] = pk[l] * pk[l];
                    ql[l] = pk[l] * s_np[n - 1][l];
                    qs[l] = slot_lanes ? pk[l] * s_np[ns][l] : (T)0;
                } else {
                    cq += pk[l] * s_np[n - 1][l];
                    if (slot_lanes) cqs += pk[l] * s_np[ns][l];
                }
            }
            const uint64_t slow = slot_lanes ? tab->slotmask[tl] : 0ull;

            // One chunk of C modes from rb: all C neighbour loads are issued
            // before the first is consumed.
            T acc_re = 0, acc_im = 0;
            auto chunk = [&](auto Cc, auto Gc, int rb) {
                constexpr int C = decltype(Cc)::value;
                constexpr bool GEO = decltype(Gc)::value;  // lane geometry from s_geo
                cplx_t<T> u[C];
                T wr[C], wi[C];  // Ahat W (real and imaginary parts)
#pragma unroll
                for (int k = 0; k < C; ++k) {
                    const int r = rb + k;
                    const LRec &R = s_unit[r];
                    int colw;
                    T c;
                    if (GEO) {
                        const int2 ge = s_geo[r * kWave + lane];
                        colw = ge.x;
                        c = (T)__int_as_float(ge.y);
                    } else {
                        int ci;
                        last_axis(N, lo, hi, r < g ? (int)s_mode[r].mt[n - 1] : 0, pos, colw, ci);
                        c = (T)ci;
                    }
                    int idx = R.lb + lane_line + colw;
                    if constexpr (AN) {
                        // sum_l Ahat^l (P k)_l (P j)_l
                        T t[DT];
#pragma unroll
                        for (int l = 0; l < DT; ++l) t[l] = fmac(-pk[l], R.pmw[l], fmac(c, ql[l], sq[l]));
                        if ((slow >> r) & 1ull) {  // slot-axis crossing for some lane
                            const int m = R.mslot;
                            const int jb = ibs - m;
                            idx += (jb < 0) ? N * N : ((jb >= N) ? -N * N : 0);
                            const int kd = ks - m;
                            const T cs = (kd < lo) ? (T)1 : ((kd > hi) ? (T)-1 : (T)0);
#pragma unroll
                            for (int l = 0; l < DT; ++l) t[l] = fmac(cs, qs[l], t[l]);
                        }
                        T a = 0, b = 0;
#pragma unroll
                        for (int l = 0; l < DT; ++l) {
                            a = fmac(R.ar[l], t[l], a);
                            if (!REAL) b = fmac(R.ai[l], t[l], b);
                        }
                        wr[k] = a;
                        wi[k] = b;
                    } else {
                        // a W = a (|P k|^2 + c N q_last) - (P k).(a P m')
                        const T a = R.a;
                        T wv = a * fmac(c, cq, s2);
#pragma unroll
                        for (int l = 0; l < DT; ++l) wv = fmac(-pk[l], R.apm[l], wv);
                        if ((slow >> r) & 1ull) {  // slot-axis crossing for some lane
                            const int m = R.mslot;
                            const int jb = ibs - m;
                            idx += (jb < 0) ? N * N : ((jb >= N) ? -N * N : 0);
                            const int kd = ks - m;
                            const T cs = (kd < lo) ? (T)1 : ((kd > hi) ? (T)-1 : (T)0);
                            wv = fmac(a * cs, cqs, wv);
                        }
                        wr[k] = REAL ? wv : R.cr * wv;
                        wi[k] = REAL ? (T)0 : R.ci * wv;
                    }
                    u[k] = x[(unsigned)idx];
                }
#pragma unroll
                for (int k = 0; k < C; ++k) {
                    if (REAL) {
                        acc_re = fmac(wr[k], u[k].x, acc_re);
                        acc_im = fmac(wr[k], u[k].y, acc_im);
                    } else {
                        acc_re = fmac(wr[k], u[k].x, fmac(-wi[k], u[k].y, acc_re));
                        acc_im = fmac(wr[k], u[k].y, fmac(wi[k], u[k].x, acc_im));
                    }
                }
            };
            auto all_modes = [&](auto Gc) {
                walk_records<KC>(g, [&](auto Cc, int rb) { chunk(Cc, Gc, rb); });
            };
            if (cached)
                all_modes(std::true_type());
            else
                all_modes(std::false_type());

            if (active) {
                const size_t i = (size_t)(L0 + s) * N + p0 + p;
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
        __syncthreads();  // the unit records are rewritten next
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

// ---------------------------------------------------------------- plane tiles
//
// n >= 2 and N <= 32: a tile is S = min(64 / N, N) lines of one plane (axes
// n-2, n-1), so lanes differ in the slot digit (axis n-2) and the position.
// The unit records (uniform-axis wraps folded in) are precomputed, so a wave
// reads them with uniform scalar loads and tiles need no set-up beyond their
// lanes' P k; waves take tiles independently.

static_assert(sizeof(UnitRec<double, kMaxD>) <= kUnitRecBytes[F64], "unit record size");
static_assert(sizeof(UnitRec<float, kMaxD>) <= kUnitRecBytes[F32], "unit record size");
static_assert(sizeof(UnitRecA<double, kMaxD>) <= kUnitRecBytes[F64], "unit record size");
static_assert(sizeof(UnitRecA<float, kMaxD>) <= kUnitRecBytes[F32], "unit record size");
static_assert(sizeof(HalfRec<double, kMaxD>) <= kUnitRecBytes[F64], "unit record size");
static_assert(sizeof(HalfRec<float, kMaxD>) <= kUnitRecBytes[F32], "unit record size");

// Record type of the plane kernel: scalar coefficient or diagonal (App. D).
template <typename T, int DT, bool AN>
using PlaneRec = typename std::conditional<AN, UnitRecA<T, DT>, UnitRec<T, DT>>::type;
// ... and of its Hermitian half-storage variant (scalar coefficient only).
template <typename T, int DT, bool AN, bool HALF>
using TileRec = typename std::conditional<HALF, HalfRec<T, DT>, PlaneRec<T, DT, AN>>::type;

// One thread per (unit, padded mode): the record of sorted mode r (padding:
// the zero mode with weight 0), computed in FP64 and rounded once.
template <typename T, int DT, bool REAL, bool AN>
__global__ __launch_bounds__(kBlock) void k_unit_records(const Table *__restrict__ tab,
                                                         const ModeRec *__restrict__ recs,
                                                         PlaneRec<T, DT, AN> *__restrict__ out,
                                                         T *__restrict__ upku)
{
    const int N = tab->N, n = tab->n, g = tab->g;
    const int gp = (g + 3) & ~3;
    const int nu = n - 2;
    const int lo = -(N / 2), hi = N - 1 - N / 2;
    const int units = tab->ntiles / tab->tiles_per_unit;
    const long long total = (long long)units * gp;
    for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < total;
         e += (long long)gridDim.x * kBlock) {
        const int unit = (int)(e / gp);
        const int r = (int)(e - (long long)unit * gp);
        int ibu[kMaxN], ku[kMaxN];
        int rest = unit;
        for (int t = nu - 1; t >= 0; --t) {
            const int q = rest / N;
            ibu[t] = rest - q * N;
            ku[t] = (2 * ibu[t] < N) ? ibu[t] : ibu[t] - N;
            rest = q;
        }
        const ModeRec &M = recs[r < g ? r : tab->zero_sorted];
        double v[DT];
        for (int l = 0; l < DT; ++l) v[l] = M.pm[l];
        int lb = 0;
        for (int t = 0; t < nu; ++t) {
            const int m = M.mt[t];
            int jb = ibu[t] - m;
            jb += (jb < 0) ? N : 0;
            jb -= (jb >= N) ? N : 0;
            lb += jb * tab->stride[t];
            const int kd = ku[t] - m;
            const int c = (kd < lo) ? 1 : ((kd > hi) ? -1 : 0);
            for (int l = 0; l < DT; ++l) v[l] -= (double)c * N * tab->P[l][t];
        }
        PlaneRec<T, DT, AN> R;
        if constexpr (AN) {
            for (int l = 0; l < DT; ++l) {
                R.pmw[l] = (T)v[l];
                R.ar[l] = (r >= g) ? (T)0 : (T)M.cl[l][0];
                R.ai[l] = (r >= g) ? (T)0 : (T)M.cl[l][1];
            }
        } else {
            const double a = (r >= g) ? 0.0 : (REAL ? M.c[0] : 1.0);
            for (int l = 0; l < DT; ++l) R.apm[l] = (T)(a * v[l]);
            R.a = (T)a;
            R.cr = (r >= g) ? (T)0 : (T)M.c[0];
            R.ci = (r >= g) ? (T)0 : (T)M.c[1];
        }
        R.mslot = M.mt[n - 2];
        // padding records gather from an index beyond every vector (as an
        // unsigned record index), which the buffer loads return as zero; the
        // 64-bit gathers load the zero mode's neighbour with weight 0 instead
        R.lb = (r >= g && !tab->wide) ? kNoNeighbour : lb - R.mslot * N;
        out[e] = R;
        if (r == 0) {
            for (int l = 0; l < DT; ++l) {
                double pu = 0.0;
                for (int t = 0; t < nu; ++t) pu += tab->P[l][t] * (double)ku[t];
                upku[(size_t)unit * DT + l] = (T)pu;
            }
        }
    }
}

// Unit records on Hermitian half storage: one thread per (stored plane hu,
// padded mode).  The weight fields are those of k_unit_records for the
// plane's unit index (the neighbour's signed representative does not depend
// on storage); the source fields place the neighbour plane in the half
// layout: stored (kind 0), mirrored (kind 1) or the center plane (kind 2).
template <typename T, int DT>
__global__ __launch_bounds__(kBlock) void k_unit_records_half(const Table *__restrict__ tab,
                                                              const ModeRec *__restrict__ recs,
                                                              HalfRec<T, DT> *__restrict__ out,
                                                              T *__restrict__ upku)
{
    const int N = tab->N, n = tab->n, g = tab->g;
    const int gp = (g + 3) & ~3;
    const int nu = n - 2;  // uniform axes (the plane grid's dimension)
    const int lo = -(N / 2), hi = N - 1 - N / 2;
    const int c0 = (N * N + 1) / 2;
    const long long total = (long long)tab->half_units * gp;
    for (long long e = (long long)blockIdx.x * kBlock + threadIdx.x; e < total;
         e += (long long)gridDim.x * kBlock) {
        const int hu = (int)(e / gp);
        const int r = (int)(e - (long long)hu * gp);
        const long long unit = half_index(hu, N, nu);
        int ibu[kMaxN], ku[kMaxN];
        long long rest = unit;
        for (int t = nu - 1; t >= 0; --t) {
            const long long q = rest / N;
            ibu[t] = (int)(rest - q * N);
            ku[t] = (2 * ibu[t] < N) ? ibu[t] : ibu[t] - N;
            rest = q;
        }
        const ModeRec &M = recs[r < g ? r : tab->zero_sorted];
        double v[DT];
        for (int l = 0; l < DT; ++l) v[l] = M.pm[l];
        long long src = 0;  // the neighbour plane's unit index
        for (int t = 0; t < nu; ++t) {
            const int m = M.mt[t];
            int jb = ibu[t] - m;
            jb += (jb < 0) ? N : 0;
            jb -= (jb >= N) ? N : 0;
            src = src * N + jb;
            const int kd = ku[t] - m;
            const int c = (kd < lo) ? 1 : ((kd > hi) ? -1 : 0);
            for (int l = 0; l < DT; ++l) v[l] -= (double)c * N * tab->P[l][t];
        }
        HalfRec<T, DT> R;
        const double a = (r >= g) ? 0.0 : M.c[0];
        for (int l = 0; l < DT; ++l) R.apm[l] = (T)(a * v[l]);
        R.a = (T)a;
        R.cr = (r >= g) ? (T)0 : (T)M.c[0];
        R.ci = (T)0;
        R.mslot = M.mt[n - 2];
        R.pad = 0;
        if (r >= g) {
            R.kind = 0;
            R.lb = kNoNeighbour;  // reads zero
        } else if (src == 0) {
            R.kind = 2;
            R.lb = 0;
        } else if (half_stored(src, N, nu)) {
            R.kind = 0;
            R.lb = c0 + (int)(half_position(src, N, nu) - 1) * N * N - R.mslot * N;
        } else {
            R.kind = 1;
            R.lb = c0 + (int)(half_position(mirror_index(src, N, nu), N, nu) - 1) * N * N;
        }
        out[e] = R;
        if (r == 0) {
            for (int l = 0; l < DT; ++l) {
                double pu = 0.0;
                for (int t = 0; t < nu; ++t) pu += tab->P[l][t] * (double)ku[t];
                upku[(size_t)hu * DT + l] = (T)pu;
            }
        }
    }
}

// Epilogue of one output entry i of the stiffness product; ex, ey: the
// entry's index in the families of x and y (f and M32 are indexed by i).
template <typename T, int EPI>
__device__ __forceinline__ void put_output(size_t i, size_t ex, size_t ey, T acc_re, T acc_im,
                                           const cplx_t<T> *__restrict__ x, void *__restrict__ yv,
                                           const double2 *__restrict__ f,
                                           const float *__restrict__ M32, double inv_unit,
                                           double (&dots)[2])
{
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
        static_cast<float2 *>(yv)[ey] = o;
        dots[0] += (double)M32[i] * ((double)o.x * (double)o.x + (double)o.y * (double)o.y);
        dots[1] += rx * rx + ry * ry;
    } else {
        if constexpr (sizeof(T) == 8) {
            // FP64 outputs are written nontemporally (no later read in this
            // kernel): faster at vectors larger than the caches, with the
            // same memory-side traffic; float outputs stay ordinary stores,
            // since the next kernel reads them while they are still cached
            typedef double v2d __attribute__((ext_vector_type(2)));
            v2d o;
            o.x = acc_re;
            o.y = acc_im;
            __builtin_nontemporal_store(o, reinterpret_cast<v2d *>(static_cast<cplx_t<T> *>(yv) + ey));
        } else {
            cplx_t<T> o;
            o.x = acc_re;
            o.y = acc_im;
            static_cast<cplx_t<T> *>(yv)[ey] = o;
        }
        if (EPI == EPI_ALPHA) {
            const cplx_t<T> xi = x[ex];
            dots[0] += (double)xi.x * (double)acc_re + (double)xi.y * (double)acc_im;
        }
    }
}

// Partial sums of workgroup b of a plane-tile product (no execution log).
template <int EPI>
__device__ __forceinline__ void put_partials_at(double (&dots)[2], double *__restrict__ part, int b)
{
    if (EPI == EPI_ALPHA) {
        double v[1] = {dots[0]};
        store_partials_at<1>(v, part, b);
    } else if (EPI == EPI_RESID) {
        store_partials_at<2>(dots, part, b);
    }
}

template <int EPI>
__device__ __forceinline__ void put_partials(double (&dots)[2], double *__restrict__ part,
                                             State *__restrict__ st, int *__restrict__ exec)
{
    if (EPI == EPI_ALPHA) {
        double v[1] = {dots[0]};
        store_partials<1>(v, part);
        if (exec && blockIdx.x == 0 && threadIdx.x == 0) *exec = 1;
    } else if (EPI == EPI_RESID) {
        store_partials<2>(dots, part);
        if (exec && blockIdx.x == 0 && threadIdx.x == 0) *exec = 1;
    }
}

// Orders this wave's LDS accesses before and after (lanes exchange records).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Work items of the plane kernel: (unit, up to tab->item_tiles consecutive
// tiles); a wave copies the unit's records to its LDS once per item.

// The product as workgroup vb of vnb (the whole grid of a plain launch, a
// problem's range of a grouped one).
template <typename T, int DT, int EPI, bool REAL, int KR, bool WIDE, bool AN, bool HALF = false>
__device__ __forceinline__ void matvec_plane(const int vb, const int vnb,
                                             const Table *__restrict__ tab,
                                             const ModeRec *__restrict__ recs,
                                             const TileRec<T, DT, AN, HALF> *__restrict__ urec,
                                             const T *__restrict__ upku,
                                             const cplx_t<T> *__restrict__ x,
                                             void *__restrict__ yv,
                                             const double2 *__restrict__ f,
                                             const float *__restrict__ M32,
                                             double *__restrict__ part,
                                             State *__restrict__ st,
                                             int *__restrict__ exec)
{
    // right-hand sides served by this launch (uniform); their flags and the
    // table's sizes in one round trip before the first branch
    const int N = tab->N;
    const int n = tab->n;
    const int g = tab->g;
    pin(N);
    pin(n);
    pin(g);
    bool act[KR];
    int nact = 0;
    double inv_unit[KR];
#pragma unroll
    for (int k = 0; k < KR; ++k) {
        if constexpr (EPI == EPI_ALPHA) {
            const int dn = st[k].done, ps = st[k].pause;
            act[k] = !(dn | ps);
        } else if constexpr (EPI == EPI_RESID) {
            const int rp = st[k].replace;
            act[k] = rp != 0;
        } else {
            act[k] = true;
        }
        inv_unit[k] = (EPI == EPI_RESID) ? st[k].inv_unit : 1.0;
        nact += act[k] ? 1 : 0;
    }
#pragma unroll
    for (int k = 0; k < KR; ++k)
        if constexpr (EPI == EPI_RESID) pin(inv_unit[k]);
    if (nact == 0) return;
    static_assert(!WIDE || KR == 1, "64-bit gathers serve one right-hand side");
    static_assert(!HALF || (REAL && !AN && !WIDE), "half storage: real scalar coefficient");
    // neighbour loads in flight per chunk: about Inflight<T> over all right-hand sides
    constexpr int KC = (Inflight<T>::v / KR >= 8) ? (Inflight<T>::v / KR) / 4 * 4 : 4;
    using Rec = TileRec<T, DT, AN, HALF>;
    // dynamic LDS: gp * kWave lane-geometry entries (column, face factor),
    // then kWaves * gp unit records
    extern __shared__ int2 s_geo[];

    const int gp = (g + 3) & ~3;
    const int S = tab->tile_s;
    const int tpu = tab->tiles_per_unit;
    const size_t D = tab->D;
    // the work layout, loaded beside the mode shifts below (one round trip)
    constexpr bool F64L = sizeof(T) == 8;  // FP64 launches have their own layout
    const int it = F64L ? tab->item_tiles64 : tab->item_tiles;
    const int xfront = F64L ? tab->xcd_front64 : tab->xcd_front;
    const int ntiles = tab->ntiles;
    pin(S);
    pin(tpu);
    pin(it);
    pin(xfront);
    pin(ntiles);
    const int lane = threadIdx.x % kWave;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int s = lane / N;
    const int p = lane - s * N;
    const int lo = -(N / 2), hi = N - 1 - N / 2;
    Rec *s_rec = reinterpret_cast<Rec *>(s_geo + gp * kWave) + wave * gp;
    {
        // lane geometry of every padded mode: entry r * kWave + lane belongs
        // to the thread of wave r % kWaves, which loads the last-axis shifts
        // of all its modes at once (one round trip) before using them
        constexpr int kPer = ((kMaxG + 3) & ~3) / kWaves;
        const int pl = lane - (lane / N) * N;  // position of this lane
        int mt[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int r = wave + k * kWaves;
            mt[k] = r < g ? recs[r].mt[n - 1] : 0;
        }
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int r = wave + k * kWaves;
            if (r >= gp) break;
            int colw, c;
            last_axis(N, lo, hi, mt[k], pl, colw, c);
            s_geo[r * kWave + lane] = make_int2(colw, __float_as_int((float)c));
        }
    }
    T pl_[DT], ps_[DT];  // p_{n-1}, p_{n-2}
#pragma unroll
    for (int l = 0; l < DT; ++l) {
        pl_[l] = (T)tab->P[l][n - 1];
        ps_[l] = (T)tab->P[l][n - 2];
    }
#pragma unroll
    for (int l = 0; l < DT; ++l) {
        pin(pl_[l]);
        pin(ps_[l]);
    }
    const T NT = (T)N;
    // one gather resource per right-hand side; a right-hand side not served
    // by this launch has no records, so its gathers read zero without traffic
    rsrc_t xr[KR];
#pragma unroll
    for (int k = 0; k < KR; ++k)
        xr[k] = make_rsrc(x + k * D, (int)sizeof(cplx_t<T>), act[k] ? (unsigned)D : 0u);
    // float families interleave their right-hand sides: one resource of D
    // records of KR entries, one gather of KR * 8 bytes per (entry, mode)
    constexpr bool ILV = std::is_same<T, float>::value && KR > 1;
    const rsrc_t xi = make_rsrc(x, (int)(KR * sizeof(cplx_t<T>)), (unsigned)D);

    // items in XCD-front order: each XCD owns a contiguous eighth, its waves
    // sweep it together
    const int ipu = (tpu + it - 1) / it;  // items per unit
    const int nitems = (ntiles / tpu) * ipu;  // half storage: the stored planes'
    const int hh = (N - 1) / 2;                    // half storage: largest stored digit
    const int c0 = (N * N + 1) / 2;                // half storage: first whole plane
    const int nw = vnb * kWaves;
    const int b = vb;
    const bool by_xcd = xfront && (vnb % 8 == 0);
    const int xcd = by_xcd ? b % 8 : 0;
    const int nloc = by_xcd ? nw / 8 : nw;
    const int loc = (by_xcd ? b / 8 : b) * kWaves + wave;
    const int per = by_xcd ? (nitems + 7) / 8 : nitems;
    const int ibeg = xcd * per;
    const int iend = min(ibeg + per, nitems);
    const int nvec = gp * (int)sizeof(Rec) / 16;  // 16-byte pieces of a unit's records
    double dots[KR][2];
#pragma unroll
    for (int k = 0; k < KR; ++k) dots[k][0] = dots[k][1] = 0.0;

    // xcd_front 2: inside each XCD's eighth of the units (a slab of span
    // consecutive values of the slowest axis), that axis varies fastest, so a
    // unit's neighbours along it are swept next to it (see Table).
    // xcd_front 3: the eighth is swept in blocks of the axes after the second
    // one (a quarter of them for FP64, half for float), each block through
    // every value of the second axis, so the neighbour layers along that axis
    // stay in the XCD's L2 while the block advances
    const int span = (by_xcd && (xfront == 2 || xfront == 3) && !HALF) ? tab->slab_span : 0;
    __syncthreads();
    for (int item = ibeg + loc; item < iend; item += nloc) {
        int unit = item / ipu;
        const int tl0 = (item - unit * ipu) * it;
        if (span > 0) {
            const int E = tab->slab_units, S1 = tab->slab_stride;
            const int e = unit / E, ul = unit - e * E;
            if (xfront == 2) {
                const int rest = ul / span;
                unit = e * E + (ul - rest * span) * S1 + rest;
            } else {
                // ul = ((block * N + a1) * span + a0) * B + r, with R = S1 / N
                // units per (a0, a1) and blocks of B of them
                const int R = S1 / N;
                int B = R / (F64L ? 4 : 2);
                if (B < 1 || R % B != 0) B = R;
                const int r = ul % B;
                int q = ul / B;
                const int a0 = q % span;
                q /= span;
                const int a1 = q % N;
                unit = e * E + a0 * S1 + a1 * R + (q / N) * B + r;
            }
        }
        // ---- the unit's records to this wave's LDS, and P k of the unit's
        // uniform axes loaded beside them ----
        T pku[DT];
        {
            const uint4 *src = reinterpret_cast<const uint4 *>(urec + (size_t)unit * gp);
            uint4 *dst = reinterpret_cast<uint4 *>(s_rec);
            wave_sync();  // the previous item's records have been read
#pragma unroll
            for (int l = 0; l < DT; ++l) pku[l] = upku[(size_t)unit * DT + l];
            for (int v = lane; v < nvec; v += kWave) dst[v] = src[v];
            wave_sync();
#pragma unroll
            for (int l = 0; l < DT; ++l) pin(pku[l]);
        }

        for (int tl = tl0; tl < min(tl0 + it, tpu); ++tl) {
            const int slot0 = tl * S;
            const int St = min(S, N - slot0);
            const int L0 = unit * N + slot0;
            // Lanes outside the tile run the same loop on clamped coordinates
            // (their loads stay in bounds) and store nothing.
            const bool active = s < St;
            const int se = active ? s : 0;
            const int ibs = slot0 + se;
            const int lane_line = ibs * N;
            const int kpos = signed_digit(p, N);
            const int ks = signed_digit(ibs, N);
            // ---- P k, |P k|^2, N (P k).p_t for the two per-lane axes (per
            // component l for a diagonal coefficient) ----
            T pk[DT];
            T s2 = 0, cq = 0, cqs = 0;
            T sq[DT], ql[DT], qs[DT];
#pragma unroll
            for (int l = 0; l < DT; ++l) {
                const T v = pku[l] + ps_[l] * (T)ks + pl_[l] * (T)kpos;
                pk[l] = v;
                if constexpr (AN) {
                    sq[l] = v * v;
                    ql[l] = NT * (v * pl_[l]);
                    qs[l] = NT * (v * ps_[l]);
                } else {
                    s2 += v * v;
                    cq += v * pl_[l];
                    cqs += v * ps_[l];
                }
            }
            cq *= NT;
            cqs *= NT;
            const uint64_t slow = tab->slotmask[tl];

            T acc_re[KR], acc_im[KR];
#pragma unroll
            for (int k = 0; k < KR; ++k) acc_re[k] = acc_im[k] = 0;
            auto chunk = [&](auto Cc, int rb) {
                constexpr int C = decltype(Cc)::value;
                cplx_t<T> u[C][KR];
                T wr[C], wi[C];  // Ahat W (real and imaginary parts)
#pragma unroll
                for (int m = 0; m < C; ++m) {
                    const int r = rb + m;
                    const Rec &Q = s_rec[r];  // LDS broadcast
                    const int2 ge = s_geo[r * kWave + lane];
                    const T c = (T)__int_as_float(ge.y);
                    int idx = Q.lb + lane_line + ge.x;
                    if constexpr (AN) {
                        // sum_l Ahat^l (P k)_l (P j)_l, (P j)_l = (P k - P m')_l
                        // + N c p_{n-1,l} + N cs p_{n-2,l}
                        T t[DT];
#pragma unroll
                        for (int l = 0; l < DT; ++l) t[l] = fmac(-pk[l], Q.pmw[l], fmac(c, ql[l], sq[l]));
                        if ((slow >> r) & 1ull) {  // slot-axis crossing for some lane
                            const int mm = Q.mslot;
                            const int jb = ibs - mm;
                            idx += (jb < 0) ? N * N : ((jb >= N) ? -N * N : 0);
                            const int kd = ks - mm;
                            const T cs = (kd < lo) ? (T)1 : ((kd > hi) ? (T)-1 : (T)0);
#pragma unroll
                            for (int l = 0; l < DT; ++l) t[l] = fmac(cs, qs[l], t[l]);
                        }
                        T a = 0, b = 0;
#pragma unroll
                        for (int l = 0; l < DT; ++l) {
                            a = fmac(Q.ar[l], t[l], a);
                            if (!REAL) b = fmac(Q.ai[l], t[l], b);
                        }
                        wr[m] = a;
                        wi[m] = b;
                    } else {
                        // a W = a (|P k|^2 + c N q_last) - (P k).(a P m')
                        T wv = Q.a * fmac(c, cq, s2);
#pragma unroll
                        for (int l = 0; l < DT; ++l) wv = fmac(-pk[l], Q.apm[l], wv);
                        if ((slow >> r) & 1ull) {  // slot-axis crossing for some lane
                            const int mm = Q.mslot;
                            const int jb = ibs - mm;
                            idx += (jb < 0) ? N * N : ((jb >= N) ? -N * N : 0);
                            const int kd = ks - mm;
                            const T cs = (kd < lo) ? (T)1 : ((kd > hi) ? (T)-1 : (T)0);
                            wv = fmac(Q.a * cs, cqs, wv);
                        }
                        wr[m] = REAL ? wv : Q.cr * wv;
                        wi[m] = REAL ? (T)0 : Q.ci * wv;
                    }
                    T sgn_im = (T)1;  // half storage: -1 reads the stored conjugate
                    if constexpr (HALF) {
                        if (Q.kind != 0) {
                            // the neighbour's in-plane digits (slot, column)
                            int sp = ibs - Q.mslot;
                            sp += (sp < 0) ? N : 0;
                            sp -= (sp >= N) ? N : 0;
                            const int cp = ge.x;
                            if (Q.kind == 1) {  // mirrored plane: digits negated
                                idx = Q.lb + (sp ? N - sp : 0) * N + (cp ? N - cp : 0);
                                sgn_im = (T)-1;
                            } else if (sp >= 1 && sp <= hh) {  // center plane, stored
                                idx = sp * N + cp - hh;
                            } else if (sp == 0 && cp <= hh) {
                                idx = cp;
                            } else {  // center plane, mirrored
                                idx = (sp ? (N - sp) * N - hh : 0) + (cp ? N - cp : 0);
                                sgn_im = (T)-1;
                            }
                        }
                    }
                    if constexpr (ILV) {
                        const f32x4_t v0 = struct_load_f32x4(xi, idx, 0, 0, 0);
                        *reinterpret_cast<float2 *>(&u[m][0]) = make_float2(v0.x, v0.y);
                        *reinterpret_cast<float2 *>(&u[m][1]) = make_float2(v0.z, v0.w);
                        if constexpr (KR == 3) {
                            const f32x2_t v1 = struct_load_f32x2(xi, idx, 16, 0, 0);
                            *reinterpret_cast<float2 *>(&u[m][KR - 1]) = make_float2(v1.x, v1.y);
                        } else if constexpr (KR == 4) {
                            const f32x4_t v1 = struct_load_f32x4(xi, idx, 16, 0, 0);
                            *reinterpret_cast<float2 *>(&u[m][KR - 2]) = make_float2(v1.x, v1.y);
                            *reinterpret_cast<float2 *>(&u[m][KR - 1]) = make_float2(v1.z, v1.w);
                        }
                    } else {
#pragma unroll
                        for (int k = 0; k < KR; ++k)
                            u[m][k] = WIDE ? x[(unsigned)idx] : gather<T>(xr[k], idx);
                    }
                    if constexpr (HALF) {
#pragma unroll
                        for (int k = 0; k < KR; ++k) u[m][k].y *= sgn_im;
                    }
                }
#pragma unroll
                for (int m = 0; m < C; ++m) {
#pragma unroll
                    for (int k = 0; k < KR; ++k) {
                        if (REAL) {
                            acc_re[k] = fmac(wr[m], u[m][k].x, acc_re[k]);
                            acc_im[k] = fmac(wr[m], u[m][k].y, acc_im[k]);
                        } else {
                            acc_re[k] = fmac(wr[m], u[m][k].x, fmac(-wi[m], u[m][k].y, acc_re[k]));
                            acc_im[k] = fmac(wr[m], u[m][k].y, fmac(wi[m], u[m][k].x, acc_im[k]));
                        }
                    }
                }
            };
            walk_records<KC>(g, chunk);
            bool store = active;
            size_t i = (size_t)(L0 + s) * N + p;
            if constexpr (HALF) {
                // unit = stored plane hu: whole planes from c0; the center plane
                // stores k = 0 and the (slot, position) with a positive first
                // nonzero component
                if (unit > 0) {
                    i = (size_t)c0 + (size_t)(unit - 1) * N * N + (size_t)ibs * N + p;
                } else if (ibs >= 1 && ibs <= hh) {
                    i = (size_t)ibs * N + p - hh;
                } else {
                    i = (size_t)p;
                    store = store && ibs == 0 && p <= hh;
                }
            }
            if (store) {
#pragma unroll
                for (int k = 0; k < KR; ++k) {
                    if (!act[k]) continue;
                    // the replaced residual (EPI_RESID) is a float family
                    const size_t ex = vec_at<T>(k, KR, D, i);
                    const size_t ey = (EPI == EPI_RESID) ? vec_at<float>(k, KR, D, i) : ex;
                    put_output<T, EPI>(i, ex, ey, acc_re[k], acc_im[k], x, yv,
                                       f ? f + k * D : f, M32, inv_unit[k], dots[k]);
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < KR; ++k)
        if (act[k]) put_partials_at<EPI>(dots[k], part + k * kPartStride, vb);
    if ((EPI == EPI_ALPHA || EPI == EPI_RESID) && exec && vb == 0 && threadIdx.x == 0)
        *exec = nact;
}

template <typename T, int DT, int EPI, bool REAL, int KR, bool WIDE, bool AN, bool HALF = false>
__global__ __launch_bounds__(kBlock) void k_matvec_plane(const Table *__restrict__ tab,
                                                         const ModeRec *__restrict__ recs,
                                                         const TileRec<T, DT, AN, HALF> *__restrict__ urec,
                                                         const T *__restrict__ upku,
                                                         const cplx_t<T> *__restrict__ x,
                                                         void *__restrict__ yv,
                                                         const double2 *__restrict__ f,
                                                         const float *__restrict__ M32,
                                                         double *__restrict__ part,
                                                         State *__restrict__ st,
                                                         int *__restrict__ exec)
{
    matvec_plane<T, DT, EPI, REAL, KR, WIDE, AN, HALF>((int)blockIdx.x, (int)gridDim.x, tab, recs,
                                                       urec, upku, x, yv, f, M32, part, st, exec);
}

// Grouped FP32-IR product: the float product of h into q with the alpha
// partials (EPI_ALPHA), or the replaced FP64 residual of X into the float r
// (EPI_RESID), of every problem of the group in one launch.
template <typename T, int DT, int EPI, bool REAL, int KR>
__global__ __launch_bounds__(kBlock) void k_matvec_plane_grp(const GroupEntry *__restrict__ ents,
                                                             const int *__restrict__ owner)
{
    static_assert((EPI == EPI_ALPHA && sizeof(T) == 4) || (EPI == EPI_RESID && sizeof(T) == 8),
                  "grouped launches run the FP32-IR products");
    const GroupEntry &e = ents[owner[blockIdx.x]];
    using Rec = PlaneRec<T, DT, false>;
    if constexpr (EPI == EPI_ALPHA)
        matvec_plane<T, DT, EPI, REAL, KR, false, false>(
            (int)blockIdx.x - e.mv0, e.nb_mv, e.tab, e.recs, static_cast<const Rec *>(e.urec32),
            static_cast<const T *>(e.upku32), reinterpret_cast<const cplx_t<T> *>(e.h32), e.q32,
            nullptr, e.M32, e.pa, e.st, nullptr);
    else
        matvec_plane<T, DT, EPI, REAL, KR, false, false>(
            (int)blockIdx.x - e.mv064, e.nb_mv64, e.tab, e.recs, static_cast<const Rec *>(e.urec64),
            static_cast<const T *>(e.upku64), reinterpret_cast<const cplx_t<T> *>(e.X), e.r32,
            reinterpret_cast<const double2 *>(e.F), e.M32, e.pb, e.st, nullptr);
}

// A product launch; with an event pair (profiled solves, never captured in a
// graph) the kernel's own dispatch records its start and end, so the pair
// times the kernel alone rather than also the dispatch gap in front of it.
template <typename... A, typename F>
void launch_timed(F kern, dim3 grid, dim3 block, size_t lds, hipStream_t s, hipEvent_t ev0,
                  hipEvent_t ev1, A... args)
{
    if (ev0 || ev1)
        hipExtLaunchKernelGGL(kern, grid, block, (std::uint32_t)lds, s, ev0, ev1, 0u, args...);
    else
        hipLaunchKernelGGL(kern, grid, block, lds, s, args...);
}

template <typename T, int EPI, bool REAL, int KR, bool WIDE, bool AN, bool HALF = false>
hipError_t launch_plane(const Table &ht, size_t lds, const Table *tab, const ModeRec *recs,
                        const void *urec, const T *Pu, const cplx_t<T> *X, void *y,
                        const double2 *Fv, const float *M32, double *part, State *st, int *exec,
                        hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    const dim3 grid(sizeof(T) == 8 ? ht.nb_mv64 : ht.nb_mv), block(kBlock);
    const size_t gp = (size_t)((ht.g + 3) & ~3);
    switch (ht.d) {
#define QP_CASE(DD)                                                                              \
    case DD:                                                                                      \
        launch_timed(k_matvec_plane<T, DD, EPI, REAL, KR, WIDE, AN, HALF>, grid, block,         \
                     lds + kWaves * gp * sizeof(TileRec<T, DD, AN, HALF>), s, ev0, ev1, tab,     \
                     recs, static_cast<const TileRec<T, DD, AN, HALF> *>(urec), Pu, X, y, Fv,   \
                     M32, part, st, exec);                                                       \
        break;
        QP_CASE(1) QP_CASE(2) QP_CASE(3) QP_CASE(4)
#undef QP_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int EPI, bool REAL, int KR, bool AN>
hipError_t dispatch(const Table *tab, const Table &ht, const ModeRec *recs, const void *urec,
                    const void *upku, const void *x, void *y, const double *f, const float *M32,
                    double *part, State *st, int *exec, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    const dim3 grid(sizeof(T) == 8 ? ht.nb_mv64 : ht.nb_mv), block(kBlock);
    const size_t lds = (ht.N <= kWave) ? sizeof(int2) * kWave * (size_t)((ht.g + 3) & ~3) : 0;
    auto X = static_cast<const cplx_t<T> *>(x);
    auto Fv = reinterpret_cast<const double2 *>(f);
    auto Pu = static_cast<const T *>(upku);
    if (ht.tile_s > 1) {
        if (!urec || !upku) return hipErrorInvalidValue;
        if (!ht.wide)
            return launch_plane<T, EPI, REAL, KR, false, AN>(ht, lds, tab, recs, urec, Pu, X, y, Fv,
                                                            M32, part, st, exec, s, ev0, ev1);
        if constexpr (KR == 1)
            return launch_plane<T, EPI, REAL, 1, true, AN>(ht, lds, tab, recs, urec, Pu, X, y, Fv,
                                                          M32, part, st, exec, s, ev0, ev1);
        return hipErrorInvalidValue;  // 64-bit gathers serve one right-hand side per launch
    }
    if (KR != 1) return hipErrorInvalidValue;  // line tiles serve one right-hand side
    switch (ht.d) {
#define QP_CASE(DD)                                                                             \
    case DD:                                                                                     \
        launch_timed(k_matvec<T, DD, EPI, REAL, AN>, grid, block, lds, s, ev0, ev1, tab, recs,  \
                     X, y, Fv, M32, part, st, exec);                                             \
        break;
        QP_CASE(1) QP_CASE(2) QP_CASE(3) QP_CASE(4)
#undef QP_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int EPI, bool REAL, bool AN>
hipError_t dispatch_k(int K, const Table *tab, const Table &ht, const ModeRec *recs,
                      const void *urec, const void *upku, const void *x, void *y, const double *f,
                      const float *M32, double *part, State *st, int *exec, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    switch (K) {
    case 1: return dispatch<T, EPI, REAL, 1, AN>(tab, ht, recs, urec, upku, x, y, f, M32, part, st, exec, s, ev0, ev1);
    case 2: return dispatch<T, EPI, REAL, 2, AN>(tab, ht, recs, urec, upku, x, y, f, M32, part, st, exec, s, ev0, ev1);
    case 3: return dispatch<T, EPI, REAL, 3, AN>(tab, ht, recs, urec, upku, x, y, f, M32, part, st, exec, s, ev0, ev1);
    case 4: return dispatch<T, EPI, REAL, 4, AN>(tab, ht, recs, urec, upku, x, y, f, M32, part, st, exec, s, ev0, ev1);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, int EPI, bool AN>
hipError_t dispatch_coef(int K, const Table *tab, const Table &ht, const ModeRec *recs,
                         const void *urec, const void *upku, const void *x, void *y,
                         const double *f, const float *M32, double *part, State *st, int *exec,
                         hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    if (ht.real_coef)
        return dispatch_k<T, EPI, true, AN>(K, tab, ht, recs, urec, upku, x, y, f, M32, part, st,
                                            exec, s, ev0, ev1);
    return dispatch_k<T, EPI, false, AN>(K, tab, ht, recs, urec, upku, x, y, f, M32, part, st,
                                         exec, s, ev0, ev1);
}

template <typename T, bool REAL, bool AN>
hipError_t unit_records(const Table *tab, const Table &ht, const ModeRec *recs, void *urec,
                        void *upku, hipStream_t s)
{
    const long long total = (long long)(ht.ntiles / ht.tiles_per_unit) * ((ht.g + 3) & ~3);
    const int grid = (int)std::min<long long>(4096, (total + kBlock - 1) / kBlock);
    auto Pu = static_cast<T *>(upku);
    switch (ht.d) {
#define QP_CASE(DD)                                                                           \
    case DD:                                                                                   \
        hipLaunchKernelGGL((k_unit_records<T, DD, REAL, AN>), dim3(grid), dim3(kBlock), 0, s,   \
                           tab, recs, static_cast<PlaneRec<T, DD, AN> *>(urec), Pu);            \
        break;
        QP_CASE(1) QP_CASE(2) QP_CASE(3) QP_CASE(4)
#undef QP_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Entry points of one coefficient kind (AN: diagonal coefficient), by
// precision and epilogue.
template <bool AN>
hipError_t matvec_entry(int prec, int epi, int K, const Table *tab, const Table &ht,
                        const ModeRec *recs, const void *urec, const void *upku, const void *x,
                        void *y, const double *f, const float *M32, const Parts &parts, State *st,
                        int *exec, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    if (prec == F64) {
        if (epi == EPI_NONE)
            return dispatch_coef<double, EPI_NONE, AN>(K, tab, ht, recs, urec, upku, x, y, f, M32,
                                                       parts.a, st, exec, s, ev0, ev1);
        if (epi == EPI_ALPHA)
            return dispatch_coef<double, EPI_ALPHA, AN>(K, tab, ht, recs, urec, upku, x, y, f, M32,
                                                        parts.a, st, exec, s, ev0, ev1);
        return dispatch_coef<double, EPI_RESID, AN>(K, tab, ht, recs, urec, upku, x, y, f, M32,
                                                    parts.b, st, exec, s, ev0, ev1);
    }
    if (epi == EPI_NONE)
        return dispatch_coef<float, EPI_NONE, AN>(K, tab, ht, recs, urec, upku, x, y, f, M32,
                                                  parts.a, st, exec, s, ev0, ev1);
    if (epi == EPI_ALPHA)
        return dispatch_coef<float, EPI_ALPHA, AN>(K, tab, ht, recs, urec, upku, x, y, f, M32,
                                                   parts.a, st, exec, s, ev0, ev1);
    return hipErrorInvalidValue;  // the replaced residual is always computed in FP64
}

template <bool AN>
hipError_t unit_records_entry(int prec, const Table *tab, const Table &ht, const ModeRec *recs,
                              void *urec, void *upku, hipStream_t s)
{
    if (ht.tile_s <= 1) return hipSuccess;  // line tiles build their records in the kernel
    if (prec == F64)
        return ht.real_coef ? unit_records<double, true, AN>(tab, ht, recs, urec, upku, s)
                            : unit_records<double, false, AN>(tab, ht, recs, urec, upku, s);
    return ht.real_coef ? unit_records<float, true, AN>(tab, ht, recs, urec, upku, s)
                        : unit_records<float, false, AN>(tab, ht, recs, urec, upku, s);
}

// Entry points of the Hermitian half-storage product (real scalar
// coefficient, plane tiles, 32-bit gathers), by precision and epilogue.
template <typename T, int EPI>
hipError_t dispatch_half(int K, const Table *tab, const Table &ht, const ModeRec *recs,
                         const void *urec, const void *upku, const void *x, void *y,
                         const double *f, const float *M32, double *part, State *st, int *exec,
                         hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    if (!ht.half || !ht.real_coef || ht.aniso || ht.tile_s <= 1 || !urec || !upku)
        return hipErrorInvalidValue;
    const size_t lds = sizeof(int2) * kWave * (size_t)((ht.g + 3) & ~3);
    auto X = static_cast<const cplx_t<T> *>(x);
    auto Fv = reinterpret_cast<const double2 *>(f);
    auto Pu = static_cast<const T *>(upku);
    switch (K) {
#define QP_K(KK)                                                                                \
    case KK:                                                                                     \
        return launch_plane<T, EPI, true, KK, false, false, true>(ht, lds, tab, recs, urec, Pu, X, \
                                                                  y, Fv, M32, part, st, exec, s,  \
                                                                  ev0, ev1);
        QP_K(1) QP_K(2) QP_K(3) QP_K(4)
#undef QP_K
    default:
        return hipErrorInvalidValue;
    }
}

inline hipError_t matvec_half_entry(int prec, int epi, int K, const Table *tab, const Table &ht,
                                    const ModeRec *recs, const void *urec, const void *upku,
                                    const void *x, void *y, const double *f, const float *M32,
                                    const Parts &parts, State *st, int *exec, hipStream_t s,
                                    hipEvent_t ev0, hipEvent_t ev1)
{
    if (prec == F64) {
        if (epi == EPI_NONE)
            return dispatch_half<double, EPI_NONE>(K, tab, ht, recs, urec, upku, x, y, f, M32,
                                                   parts.a, st, exec, s, ev0, ev1);
        if (epi == EPI_ALPHA)
            return dispatch_half<double, EPI_ALPHA>(K, tab, ht, recs, urec, upku, x, y, f, M32,
                                                    parts.a, st, exec, s, ev0, ev1);
        return dispatch_half<double, EPI_RESID>(K, tab, ht, recs, urec, upku, x, y, f, M32,
                                                parts.b, st, exec, s, ev0, ev1);
    }
    if (epi == EPI_NONE)
        return dispatch_half<float, EPI_NONE>(K, tab, ht, recs, urec, upku, x, y, f, M32, parts.a,
                                              st, exec, s, ev0, ev1);
    if (epi == EPI_ALPHA)
        return dispatch_half<float, EPI_ALPHA>(K, tab, ht, recs, urec, upku, x, y, f, M32, parts.a,
                                               st, exec, s, ev0, ev1);
    return hipErrorInvalidValue;  // the replaced residual is always computed in FP64
}

template <typename T>
hipError_t unit_records_half(const Table *tab, const Table &ht, const ModeRec *recs, void *urec,
                             void *upku, hipStream_t s)
{
    const long long total = (long long)ht.half_units * ((ht.g + 3) & ~3);
    const int grid = (int)std::min<long long>(4096, (total + kBlock - 1) / kBlock);
    auto Pu = static_cast<T *>(upku);
    switch (ht.d) {
#define QP_CASE(DD)                                                                          \
    case DD:                                                                                  \
        hipLaunchKernelGGL((k_unit_records_half<T, DD>), dim3(grid), dim3(kBlock), 0, s, tab,   \
                           recs, static_cast<HalfRec<T, DD> *>(urec), Pu);                     \
        break;
        QP_CASE(1) QP_CASE(2) QP_CASE(3) QP_CASE(4)
#undef QP_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace
}  // namespace qp
