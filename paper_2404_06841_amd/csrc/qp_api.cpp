// Host side of the C ABI declared in include/qp.h: argument validation, the
// device workspace, and the drivers that queue C-PCG (Alg. 2) and its FP32
// refinement variant on one HIP stream.  The host never computes a Krylov
// scalar: it queues batches of iterations and polls the device's `done` flag.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "qp.h"
#include "qp_internal.h"

using qp::State;
using qp::Table;

namespace {

thread_local std::string g_last_error;

qp_status fail(qp_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

#define QP_HIP(call)                                                                    \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(QP_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));     \
    } while (0)

#define QP_TRY(call)                    \
    do {                                \
        qp_status s_ = (call);          \
        if (s_ != QP_OK) return s_;     \
    } while (0)

constexpr size_t kAlign = 256;
constexpr int kMaxBatch = 64;                // iterations per batch (poll_every cap)
constexpr int kExecInts = 2 * kMaxBatch + 2;  // execution log: hot A/B sets, then residual A/B
constexpr size_t kMaxGraphs = 16;           // instantiated batch graphs kept per problem

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Whether [a, a + bytes) and [b, b + bytes) share a byte (addresses compared
// as integers, so buffers of different allocations never match).
bool overlaps(const void *a, const void *b, size_t bytes)
{
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + bytes && y < x + bytes;
}

// The stiffness product tiles planes (S lines per wave) when n >= 2 and
// N <= 32; its units are then the N^(n-2) planes.
bool plane_tiles(int n, int N) { return n >= 2 && N <= 32; }

int64_t plane_units(int n, int N)
{
    if (!plane_tiles(n, N)) return 0;
    int64_t u = 1;
    for (int t = 0; t < n - 2; ++t) u *= N;
    return u;
}

// Offsets of every device buffer inside the workspace.
struct Layout {
    size_t F, U, r, h, q, M64, M32, x32, r32, h32, q32, chi, parts, states, hist, small, exec, tab,
        recs;
    size_t urec[2], upku[2];  // unit records and unit P k, by precision (plane tiles)
    size_t total;
};

// units: the plane-tile product's units (planes), 0 without plane tiles
Layout make_layout(int d, int64_t D, int g, int64_t units)
{
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    const size_t c64 = 16 * (size_t)D, c32 = 8 * (size_t)D;
    const size_t K = (size_t)d;  // right-hand sides solved together (the d correctors)
    L.F = take(c64 * K);
    L.U = take(c64 * K);
    L.r = take(c64 * K);
    L.h = take(c64 * K);
    L.q = take(c64 * K);
    L.M64 = take(8 * (size_t)D);
    L.M32 = take(4 * (size_t)D);
    L.x32 = take(c32 * K);
    L.r32 = take(c32 * K);
    L.h32 = take(c32 * K);
    L.q32 = take(c32 * K);
    L.chi = take(c64 * (size_t)d);
    L.parts = take(3 * sizeof(double) * qp::kMaxRhs * qp::kPartStride);
    L.states = take(qp::kMaxRhs * sizeof(State));
    L.hist = take(sizeof(double) * 2 * qp::kHist * qp::kMaxRhs);
    L.small = take(sizeof(double) * 128);
    L.exec = take(sizeof(int) * kExecInts);
    L.tab = take(sizeof(Table));
    L.recs = take(sizeof(qp::ModeRec) * qp::kMaxG);
    const size_t urecs = (size_t)units * (size_t)((g + 3) & ~3);
    for (int prec = 0; prec < 2; ++prec) {
        L.urec[prec] = take(qp::kUnitRecBytes[prec] * urecs);
        L.upku[prec] = take((prec == qp::F64 ? 8 : 4) * (size_t)qp::kMaxD * (size_t)units);
    }
    L.total = o;
    return L;
}

}  // namespace

struct qp_problem {
    Table host{};
    Table *tab = nullptr;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char *ws = nullptr;
    bool own_ws = false;
    Layout L{};
    qp_options opt{};
    double amin = 0, amax = 0, pkmin = 0;
    int flags = 0;
    qp_layout layout{};         // work layout of the stiffness product
    State *hstate = nullptr;   // pinned: two polling slots + final, kMaxRhs states each
    double *hsmall = nullptr;  // pinned
    int *hexec = nullptr;      // pinned copy of the execution log
    double *hhist = nullptr;   // pinned copy of the Lanczos coefficients (kMaxRhs x kHist pairs)
    std::vector<hipEvent_t> ev_hot, ev_res;  // profiling events (begin, end pairs)
    double last_product_ms = -1.0;  // the last single product's kernel time (profile on)
    struct Graph {
        bool ir;
        int K, k, ab;
        bool prof;
        const void *u, *f;  // solution and right-hand side the graph was captured on
        hipGraphExec_t exec;
    };
    std::vector<Graph> graphs;
    hipEvent_t ev_poll[2] = {nullptr, nullptr};
    hipEvent_t ev_fin = nullptr;  // the last copy of a solve or homogenization arrived
    hipEvent_t ev_t0 = nullptr, ev_t1 = nullptr;

    template <typename T> T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
    double *F() const { return at<double>(L.F); }
    double *U() const { return at<double>(L.U); }
    double *r() const { return at<double>(L.r); }
    double *h() const { return at<double>(L.h); }
    double *q() const { return at<double>(L.q); }
    double *M64() const { return at<double>(L.M64); }
    float *M32() const { return at<float>(L.M32); }
    float *x32() const { return at<float>(L.x32); }
    float *r32() const { return at<float>(L.r32); }
    float *h32() const { return at<float>(L.h32); }
    float *q32() const { return at<float>(L.q32); }
    double *chi(int j) const { return at<double>(L.chi) + (size_t)2 * host.D * j; }
    qp::Parts parts() const
    {
        double *p = at<double>(L.parts);
        const size_t stride = qp::kMaxRhs * qp::kPartStride;
        return qp::Parts{p, p + stride, p + 2 * stride};
    }
    State *st() const { return at<State>(L.states); }
    double *hist(int r) const { return at<double>(L.hist) + (size_t)2 * qp::kHist * r; }
    double *small() const { return at<double>(L.small); }
    int *exec_hot() const { return at<int>(L.exec); }
    int *exec_res() const { return at<int>(L.exec) + 2 * kMaxBatch; }
    const qp::ModeRec *recs() const { return at<qp::ModeRec>(L.recs); }
    void *urec(int prec) const { return at<char>(L.urec[prec]); }
    void *upku(int prec) const { return at<char>(L.upku[prec]); }
    std::vector<qp::ModeRec> recs_host;
};

namespace {

qp_status check_args(int d, int n, const double *P, int g, const int32_t *modes,
                     const double *coef, int N)
{
    if (!P || !modes || !coef) return fail(QP_EINVAL, "null P, modes or coef");
    if (d < 1 || d > QP_MAX_DIM_D) return fail(QP_EINVAL, "d=%d outside [1, %d]", d, QP_MAX_DIM_D);
    if (n < d || n > QP_MAX_DIM_N) return fail(QP_EINVAL, "n=%d outside [d, %d]", n, QP_MAX_DIM_N);
    if (N < 2) return fail(QP_EINVAL, "N=%d < 2", N);
    if (g < 1 || g > QP_MAX_MODES) return fail(QP_EINVAL, "g=%d outside [1, %d]", g, QP_MAX_MODES);
    int64_t D = 1;
    for (int t = 0; t < n; ++t) {
        D *= N;
        if (D >= ((int64_t)1 << 31)) return fail(QP_EINVAL, "N^n exceeds 2^31 - 1");
    }
    for (int i = 0; i < d * n; ++i)
        if (!std::isfinite(P[i])) return fail(QP_EINVAL, "P has a non-finite entry");
    double cmax = 0.0;
    for (int r = 0; r < g; ++r) {
        if (!std::isfinite(coef[2 * r]) || !std::isfinite(coef[2 * r + 1]))
            return fail(QP_EINVAL, "coefficient %d is not finite", r);
        cmax = std::max(cmax, std::hypot(coef[2 * r], coef[2 * r + 1]));
        for (int t = 0; t < n; ++t) {
            const int64_t m = modes[r * n + t];
            if (2 * std::llabs(m) >= N)
                return fail(QP_EINVAL, "mode %d has |m_%d| = %lld >= N/2 (would alias)", r, t,
                            (long long)std::llabs(m));
        }
    }
    int zero = -1;
    for (int r = 0; r < g; ++r) {
        bool z = true;
        for (int t = 0; t < n; ++t) z = z && modes[r * n + t] == 0;
        if (z) zero = r;
        for (int s = r + 1; s < g; ++s) {
            bool same = true;
            for (int t = 0; t < n; ++t) same = same && modes[r * n + t] == modes[s * n + t];
            if (same) return fail(QP_EINVAL, "modes %d and %d are equal", r, s);
        }
    }
    if (zero < 0) return fail(QP_EINVAL, "the mean coefficient Ahat_0 is missing");
    const double tolh = 1e-14 * cmax;
    if (!(coef[2 * zero] > 0.0) || std::fabs(coef[2 * zero + 1]) > tolh)
        return fail(QP_EINVAL, "Ahat_0 must be real and positive");
    for (int r = 0; r < g; ++r) {
        int partner = -1;
        for (int s = 0; s < g && partner < 0; ++s) {
            bool neg = true;
            for (int t = 0; t < n; ++t) neg = neg && modes[s * n + t] == -modes[r * n + t];
            if (neg) partner = s;
        }
        if (partner < 0) return fail(QP_EINVAL, "mode %d has no -m partner (field not real)", r);
        const double dr = coef[2 * partner] - coef[2 * r];
        const double di = coef[2 * partner + 1] + coef[2 * r + 1];
        if (std::hypot(dr, di) > tolh)
            return fail(QP_EINVAL, "Ahat_{-m} != conj(Ahat_m) for mode %d (field not real)", r);
    }
    return QP_OK;
}

// Grid of the streaming kernels: workgroups of `chunk` consecutive entries
// (a multiple of kBlock).  Every vector kernel reduces all partial sums of
// the previous launch in each workgroup, so the partial traffic grows with
// the square of the workgroup count: at 1,048,576 unknowns 1024 workgroups
// read 48 MB of partials per iteration beside 136 MB of float vectors.  The
// cap per precision was measured there (two right-hand sides): FP32-IR best
// at 586 workgroups of 1792 entries (one pass of the float update and
// direction; 384 to 768 workgroups within 0.3%), FP64 at 683 (1536 entries
// each).
#ifndef QP_GRID_IR
#define QP_GRID_IR 640
#endif
void stream_grid(Table &T, int precision)
{
    const int64_t D = T.D;
    const int cap = std::min(qp::kStreamBlocks, precision == QP_PREC_FP32_IR ? QP_GRID_IR : 820);
    int nb = (int)std::min<int64_t>(cap, (D + qp::kBlock - 1) / qp::kBlock);
    if (nb >= 64) nb -= nb % 8;
    int64_t chunk = (D + nb - 1) / nb;
    chunk = (chunk + qp::kBlock - 1) / qp::kBlock * qp::kBlock;
    T.chunk = (int)chunk;
    T.nblocks = (int)((D + chunk - 1) / chunk);
}

// Default grid of the stiffness product from its work items: (unit,
// consecutive tiles of the unit), about four per workgroup for plane tiles.
void default_product_grid(Table &T)
{
    const int64_t units = T.ntiles / T.tiles_per_unit;
    const int64_t items = T.tile_s > 1
                              ? units * ((T.tiles_per_unit + T.item_tiles - 1) / T.item_tiles)
                              : units * ((T.tiles_per_unit + 3) / 4);
    const int64_t want = T.tile_s > 1 ? (items + 3) / 4 : items;
    int nbm = (int)std::min<int64_t>(qp::kMaxBlocks, std::max<int64_t>(1, want));
    if (nbm >= 8) nbm -= nbm % 8;
    T.nb_mv = nbm;
    T.item_tiles64 = T.item_tiles;
    T.nb_mv64 = T.nb_mv;
    T.xcd_front64 = T.xcd_front;
}

// coefs: null for a scalar coefficient, else d x g complex (a_l's Ahat per mode)
void build_table(Table &T, int d, int n, const double *P, int g, const int32_t *modes,
                 const double *coef, const double *coefs, int N)
{
    std::memset(&T, 0, sizeof(T));
    T.d = d;
    T.n = n;
    T.N = N;
    T.g = g;
    int64_t D = 1;
    for (int t = 0; t < n; ++t) D *= N;
    T.D = (int)D;
    int64_t s = 1;
    for (int t = n - 1; t >= 0; --t) {
        T.stride[t] = (int)s;
        s *= N;
    }
    int c = 0;
    while ((1LL << c) < N) ++c;
    T.shift = 31 + c;
    T.magic = (uint64_t)((((unsigned __int128)1 << T.shift) + (unsigned)N - 1) / (unsigned)N);
    for (int l = 0; l < d; ++l)
        for (int t = 0; t < n; ++t) T.P[l][t] = P[l * n + t];
    for (int r = 0; r < g; ++r) {
        bool z = true;
        int64_t off = 0, mi = 0, ni = 0;
        for (int t = 0; t < n; ++t) {
            const int m = modes[r * n + t];
            T.modes[r][t] = m;
            z = z && m == 0;
            off -= (int64_t)m * T.stride[t];
            mi = mi * N + ((m % N) + N) % N;
            ni = ni * N + (((-m) % N) + N) % N;
        }
        T.off[r] = (int)off;
        T.midx[r] = (int)mi;
        T.nidx[r] = (int)ni;
        T.coef[r][0] = coef[2 * r];
        T.coef[r][1] = coef[2 * r + 1];
        for (int l = 0; l < d; ++l) {
            const double *c = coefs ? coefs + 2 * ((size_t)l * g + r) : coef + 2 * r;
            T.coefl[r][l][0] = c[0];
            T.coefl[r][l][1] = c[1];
        }
        for (int l = 0; l < d; ++l) {
            double v = 0.0;
            for (int t = 0; t < n; ++t) v += P[l * n + t] * (double)modes[r * n + t];
            T.Pm[r][l] = v;
        }
        if (z) {
            T.zero_mode = r;
            T.a0 = coef[2 * r];
            for (int l = 0; l < d; ++l) T.a0l[l] = T.coefl[r][l][0];
        }
    }
    T.aniso = coefs ? 1 : 0;
    T.real_coef = 1;
    for (int r = 0; r < g; ++r)
        for (int l = 0; l < d; ++l)
            if (T.coefl[r][l][1] != 0.0) T.real_coef = 0;

    // Tiled stiffness product: modes sorted by their last component (stable),
    // so that consecutive gathers of a tile read neighbouring columns.
    std::vector<int> ord(g);
    for (int r = 0; r < g; ++r) ord[r] = r;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
        return modes[a * n + n - 1] < modes[b * n + n - 1];
    });
    for (int k = 0; k < g; ++k) {
        T.order[k] = ord[k];
        if (ord[k] == T.zero_mode) T.zero_sorted = k;
    }
    if (plane_tiles(n, N)) {
        // tiles of S lines of a plane
        T.lanes_p = N;
        T.tile_s = std::min(64 / N, N);
        T.tiles_per_unit = (N + T.tile_s - 1) / T.tile_s;
        T.ntiles = (int)(D / ((int64_t)N * N)) * T.tiles_per_unit;
        const int kmin = -(N / 2), kmax = kmin + N - 1;
        for (int tl = 0; tl < T.tiles_per_unit; ++tl) {
            uint64_t mask = 0;
            const int b0 = tl * T.tile_s, b1 = std::min(b0 + T.tile_s, N);
            for (int k = 0; k < g; ++k) {
                const int m = modes[ord[k] * n + n - 2];
                for (int b = b0; b < b1; ++b) {
                    const int ks = (2 * b < N) ? b : b - N;
                    if (b - m < 0 || b - m >= N || ks - m < kmin || ks - m > kmax)
                        mask |= (uint64_t)1 << k;
                }
            }
            T.slotmask[tl] = mask;
        }
    } else {
        // tiles of (up to 64 positions of) one line
        T.lanes_p = std::min(N, 64);
        T.tile_s = 1;
        T.tiles_per_unit = (N + 63) / 64;
        T.ntiles = (int)(D / N) * T.tiles_per_unit;
    }
    // work items of the stiffness product: (unit, consecutive tiles of the
    // unit), one per wave for plane tiles (as long as that leaves about four
    // waves per SIMD), four tiles per workgroup for line tiles
#ifndef QP_ITEM_TARGET
#define QP_ITEM_TARGET 4096
#endif
#ifndef QP_XCD_FRONT
#define QP_XCD_FRONT 1
#endif
    T.item_tiles = 1;
    if (T.tile_s > 1)
        while (T.item_tiles < 4 && T.ntiles / (2 * T.item_tiles) >= QP_ITEM_TARGET)
            T.item_tiles *= 2;
    T.xcd_front = QP_XCD_FRONT;
    // slab order (xcd_front 2): each eighth of the units must be whole values
    // of the slowest uniform axis (n >= 3)
    T.slab_units = T.slab_stride = T.slab_span = 0;
    if (T.tile_s > 1 && n >= 3) {
        const int64_t units_all = T.ntiles / T.tiles_per_unit;
        int64_t S1 = 1;
        for (int t = 1; t < n - 2; ++t) S1 *= N;
        if (units_all % 8 == 0 && (units_all / 8) % S1 == 0 && units_all / 8 / S1 >= 2) {
            T.slab_units = (int)(units_all / 8);
            T.slab_stride = (int)S1;
            T.slab_span = (int)(units_all / 8 / S1);
        }
    }
    default_product_grid(T);
    stream_grid(T, QP_PREC_FP64);
}

// Hermitian half storage (real scalar coefficient, odd N, plane tiles): the
// vectors hold the (N^n + 1)/2 stored entries (see qp_internal.h), the
// product's units are the stored planes, and the mode indices become
// positions: midx = the position of m when m is stored, else -1 (the
// corrector source there is implied by its conjugate at -m); nidx = the
// position of -m, or of m with nconj set when -m is not stored.
void make_half(Table &T)
{
    const int N = T.N, n = T.n;
    T.half = 1;
    T.Dgrid = T.D;
    T.D = (T.Dgrid + 1) / 2;
    const int64_t units = T.ntiles / T.tiles_per_unit;
    T.half_units = (int)((units + 1) / 2);
    T.ntiles = T.half_units * T.tiles_per_unit;
    T.slab_units = T.slab_stride = T.slab_span = 0;
    for (int r = 0; r < T.g; ++r) {
        const long long mi = T.midx[r], ni = T.nidx[r];
        T.midx[r] = qp::half_stored(mi, N, n) ? (int)qp::half_position(mi, N, n) : -1;
        const bool neg_stored = qp::half_stored(ni, N, n);
        T.nidx[r] = (int)qp::half_position(neg_stored ? ni : mi, N, n);
        T.nconj[r] = neg_stored ? 0 : 1;
    }
    default_product_grid(T);
    stream_grid(T, QP_PREC_FP64);
}


// Mode records of the tiled stiffness product, in the table's sorted order.
void build_mode_records(const Table &T, std::vector<qp::ModeRec> &out)
{
    out.assign(T.g, qp::ModeRec{});
    for (int k = 0; k < T.g; ++k) {
        const int r = T.order[k];
        qp::ModeRec &R = out[k];
        std::memset(&R, 0, sizeof(R));
        for (int l = 0; l < T.d; ++l) {
            R.pm[l] = T.Pm[r][l];
            R.cpm[l] = T.coef[r][0] * T.Pm[r][l];
        }
        R.c[0] = T.coef[r][0];
        R.c[1] = T.coef[r][1];
        for (int l = 0; l < T.d; ++l) {
            R.cl[l][0] = T.coefl[r][l][0];
            R.cl[l][1] = T.coefl[r][l][1];
        }
        for (int t = 0; t < T.n; ++t) R.mt[t] = (short)T.modes[r][t];
    }
}

void release(qp_problem *p)
{
    if (!p) return;
    for (auto &G : p->graphs) (void)hipGraphExecDestroy(G.exec);
    for (auto e : p->ev_hot) (void)hipEventDestroy(e);
    for (auto e : p->ev_res) (void)hipEventDestroy(e);
    for (auto e : p->ev_poll)
        if (e) (void)hipEventDestroy(e);
    if (p->ev_fin) (void)hipEventDestroy(p->ev_fin);
    if (p->ev_t0) (void)hipEventDestroy(p->ev_t0);
    if (p->ev_t1) (void)hipEventDestroy(p->ev_t1);
    if (p->hstate) (void)hipHostFree(p->hstate);
    if (p->hsmall) (void)hipHostFree(p->hsmall);
    if (p->hexec) (void)hipHostFree(p->hexec);
    if (p->hhist) (void)hipHostFree(p->hhist);
    if (p->own_ws && p->ws) (void)hipFree(p->ws);
    if (p->own_stream && p->stream) (void)hipStreamDestroy(p->stream);
    delete p;
}

// ------------------------------------------------------------- batches

// A solve runs in batches of `batch` PCG iterations (even, so that iteration
// it of a batch has the parity of its absolute index: the kernels only use
// that parity).  A full batch is captured once as a HIP graph and replayed;
// the host polls the device state once per batch.  With profiling, every
// stiffness product of a batch is bracketed by events of the batch's slot set
// (A/B alternate, so one set is read while the other runs) and the batch is
// launched directly: events recorded by graph nodes cannot be timed by this
// runtime (hipEventElapsedTime rejects them).
struct Profile {
    double hot_ms = 0.0, res_ms = 0.0;
    int hot_n = 0, res_n = 0;      // launches that did work
    int hot_rhs = 0, res_rhs = 0;  // right-hand sides they served
};

int batch_size(const qp_options &o)
{
    int b = o.poll_every > 0 ? o.poll_every : 12;
    b = std::min(kMaxBatch, std::max(2, b));
    return (b + 1) & ~1;
}

qp_status events_ready(qp_problem *p)
{
    auto fill = [](std::vector<hipEvent_t> &pool, size_t n) -> qp_status {
        while (pool.size() < n) {
            hipEvent_t e;
            QP_HIP(hipEventCreate(&e));
            pool.push_back(e);
        }
        return QP_OK;
    };
    QP_TRY(fill(p->ev_hot, 2 * 2 * kMaxBatch));
    QP_TRY(fill(p->ev_res, 2 * 2));
    return QP_OK;
}

// Queue one stiffness product.  slot >= 0: profiled, with event pair and
// execution-log entry `slot` of its kind.
qp_status queue_matvec(qp_problem *p, int prec, int epi, int K, const void *x, void *y,
                       const double *f, int slot)
{
    const bool resid = epi == qp::EPI_RESID;
    std::vector<hipEvent_t> &pool = resid ? p->ev_res : p->ev_hot;
    int *exec = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (slot >= 0) {
        exec = (resid ? p->exec_res() : p->exec_hot()) + slot;
        ev0 = pool[2 * slot];
        ev1 = pool[2 * slot + 1];
    }
    // profiled: the launch itself records the pair around the kernel
    QP_HIP(qp::launch_matvec(prec, epi, K, p->tab, p->host, p->recs(), p->urec(prec),
                             p->upku(prec), x, y, f, p->M32(), p->parts(), p->st(), exec,
                             p->stream, ev0, ev1));
    return QP_OK;
}

// k FP64 iterations (it = 0 .. k-1) of K right-hand sides on U.
qp_status enqueue_fp64(qp_problem *p, int K, double *U, int k, int ab, bool prof)
{
    const qp::Parts parts = p->parts();
    for (int it = 0; it < k; ++it) {
        QP_TRY(queue_matvec(p, qp::F64, qp::EPI_ALPHA, K, p->h(), p->q(), nullptr,
                            prof ? ab * kMaxBatch + it : -1));
        QP_HIP(qp::launch_pcg_update(qp::F64, it, K, p->tab, p->host, p->r(), p->q(), p->M64(),
                                     parts, p->st(), p->stream));
        QP_HIP(qp::launch_pcg_direction(qp::F64, it, K, p->tab, p->host, U, p->r(), p->h(),
                                        p->M64(), parts, p->st(), p->stream));
    }
    return QP_OK;
}

// FP32-IR residual replacement for the paused right-hand sides, after float
// iteration it: fold, FP64 residual, convergence test and direction.
qp_status enqueue_replacement(qp_problem *p, int K, double *X, const double *rhs, int it, int ab,
                              bool prof)
{
    const qp::Parts parts = p->parts();
    QP_HIP(qp::launch_ir_fold(K, p->tab, p->host, X, p->x32(), p->st(), p->stream));
    QP_TRY(queue_matvec(p, qp::F64, qp::EPI_RESID, K, X, p->r32(), rhs, prof ? ab : -1));
    QP_HIP(qp::launch_ir_direction(it, K, p->tab, p->host, p->r32(), p->h32(), p->M32(), parts,
                                   p->st(), p->stream));
    return QP_OK;
}

// k FP32-IR iterations of K right-hand sides on the FP64 solutions X for the
// right-hand sides rhs; the batch ends with the replacement of the paused ones.
qp_status enqueue_ir(qp_problem *p, int K, double *X, const double *rhs, int k, int ab, bool prof)
{
    const qp::Parts parts = p->parts();
    for (int it = 0; it < k; ++it) {
        QP_TRY(queue_matvec(p, qp::F32, qp::EPI_ALPHA, K, p->h32(), p->q32(), nullptr,
                            prof ? ab * kMaxBatch + it : -1));
        QP_HIP(qp::launch_pcg_update(qp::F32, it, K, p->tab, p->host, p->r32(), p->q32(),
                                     p->M32(), parts, p->st(), p->stream));
        QP_HIP(qp::launch_pcg_direction(qp::F32, it, K, p->tab, p->host, p->x32(), p->r32(),
                                        p->h32(), p->M32(), parts, p->st(), p->stream));
        if (it + 1 == k) QP_TRY(enqueue_replacement(p, K, X, rhs, it, ab, prof));
    }
    return QP_OK;
}

// Queue one batch: a graph replay when it is a full batch and graphs are on,
// else direct launches.
qp_status queue_batch(qp_problem *p, bool ir, int K, double *U, const double *rhs, int k, int ab,
                      bool prof)
{
    const int full = batch_size(p->opt);
    if (!p->opt.graphs || prof || k != full)
        return ir ? enqueue_ir(p, K, U, rhs, k, ab, prof) : enqueue_fp64(p, K, U, k, ab, prof);
    for (auto &G : p->graphs)
        if (G.ir == ir && G.K == K && G.k == k && G.ab == ab && G.prof == prof && G.u == U &&
            G.f == rhs) {
            QP_HIP(hipGraphLaunch(G.exec, p->stream));
            return QP_OK;
        }
    if (p->graphs.size() >= kMaxGraphs) {
        (void)hipGraphExecDestroy(p->graphs.front().exec);
        p->graphs.erase(p->graphs.begin());
    }
    QP_HIP(hipStreamBeginCapture(p->stream, hipStreamCaptureModeRelaxed));
    const qp_status qs =
        ir ? enqueue_ir(p, K, U, rhs, k, ab, prof) : enqueue_fp64(p, K, U, k, ab, prof);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(p->stream, &graph);
    if (qs != QP_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return qs;
    }
    if (ec != hipSuccess || !graph)
        return fail(QP_EDEVICE, "graph capture failed: %s", hipGetErrorString(ec));
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return fail(QP_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(ei));
    p->graphs.push_back({ir, K, k, ab, prof, U, rhs, exec});
    QP_HIP(hipGraphLaunch(exec, p->stream));
    return QP_OK;
}

// Queue the copy of the K right-hand sides' Lanczos coefficients to pinned
// memory (behind everything queued on the problem's stream).
qp_status queue_hist(qp_problem *p, int K, hipStream_t s)
{
    QP_HIP(hipMemcpyAsync(p->hhist, p->hist(0), sizeof(double) * 2 * qp::kHist * K,
                          hipMemcpyDeviceToHost, s));
    return QP_OK;
}

// Number of eigenvalues below x of the symmetric tridiagonal matrix with
// diagonal a[0..m) and off-diagonal b[0..m-1) (Sturm sequence of the LDL^T
// pivots: the count of negative pivots).
int sturm_count(const std::vector<double> &a, const std::vector<double> &b, double x)
{
    const int m = (int)a.size();
    int neg = 0;
    double q = 1.0;
    for (int i = 0; i < m; ++i) {
        const double off = (i > 0) ? b[i - 1] * b[i - 1] : 0.0;
        q = (a[i] - x) - ((i > 0) ? off / q : 0.0);
        if (q == 0.0) q = -1e-300;  // a zero pivot counts as negative (x is an eigenvalue)
        if (q < 0.0) ++neg;
    }
    return neg;
}

// Condition estimate of the preconditioned operator from the first m PCG
// coefficients: the Lanczos matrix of C-PCG (Alg. 2) has diagonal
// 1/alpha_j + beta_{j-1}/alpha_{j-1} and off-diagonal sqrt(beta_j)/alpha_j;
// its extreme eigenvalues (by bisection) approach those of M^(1/2) Q M^(1/2)
// from inside.  ab: (alpha_j, beta_j) pairs.  0 when m < 1 or a coefficient
// is not positive and finite.
double lanczos_kappa(const double *ab, int m)
{
    if (m < 1) return 0.0;
    std::vector<double> a(m), b(m > 1 ? m - 1 : 0);
    for (int j = 0; j < m; ++j) {
        const double al = ab[2 * j];
        if (!(al > 0.0) || !std::isfinite(al)) return 0.0;
        a[j] = 1.0 / al;
        if (j > 0) a[j] += ab[2 * (j - 1) + 1] / ab[2 * (j - 1)];
        if (j + 1 < m) {
            const double be = ab[2 * j + 1];
            if (!(be >= 0.0) || !std::isfinite(be)) return 0.0;
            b[j] = std::sqrt(be) / al;
        }
    }
    // Gershgorin interval
    double lo = a[0], hi = a[0];
    for (int i = 0; i < m; ++i) {
        const double r = ((i > 0) ? std::fabs(b[i - 1]) : 0.0) + ((i + 1 < m) ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    auto kth = [&](int k) {  // the k-th smallest eigenvalue (k = 1 .. m)
        double l = lo, h = hi;
        for (int it = 0; it < 200 && h - l > 1e-15 * std::max(std::fabs(l), std::fabs(h)); ++it) {
            const double mid = 0.5 * (l + h);
            if (sturm_count(a, b, mid) >= k) h = mid; else l = mid;
        }
        return 0.5 * (l + h);
    };
    const double emin = kth(1), emax = kth(m);
    return (emin > 0.0) ? emax / emin : 0.0;
}

// Algorithmic device bytes a solve's kernels move for one right-hand side of
// D unknowns: every vector a kernel touches is read or written once (FP64
// complex 16 B, float complex 8 B, the preconditioner 8 B / 4 B); cache and
// refetch traffic are not included.
double solve_bytes(bool ir, double D, int iters, int replacements)
{
    if (!ir) {
        // init: read f, M; write U, r, h.  Iteration: product (read h, write
        // q), update (read r, q, M; write r), direction (read r, M, h, U;
        // write h, U); the last direction only adds alpha h to U.
        double b = 72.0;
        if (iters > 0) b += 88.0 * iters + 88.0 * (iters - 1) + 48.0;
        return b * D;
    }
    // ||f'|| (read f); init (read f, M; write X, x, r, h); float iteration:
    // product 16, update 28, direction 44; replacement: fold (read X, x;
    // write X, x), FP64 residual (read X, f, M; write float r), direction
    // (read r, M, h; write h).
    return (16.0 + 60.0 + 88.0 * iters + 120.0 * replacements) * D;
}

// Double-buffered polling: after each batch the K states (and, when
// profiling, the batch's execution log) are copied to pinned memory; the
// batch before the newest is inspected, so the device always has queued work.
// Kernels of a finished right-hand side skip it.
struct Poller {
    qp_problem *p = nullptr;
    int K = 0;
    bool prof = false;
    Profile *pf = nullptr;
    struct Rec {
        bool pending = false;
        int k = 0, nres = 0;
    } rec[2];
    int slot = 0;  // slot set of the batch being pushed

    State *host_states(int s) const { return p->hstate + s * qp::kMaxRhs; }

    qp_status account(int s)
    {
        const int *hot = p->hexec + s * kMaxBatch;
        for (int it = 0; it < rec[s].k; ++it) {
            if (!hot[it]) continue;
            float t = 0.f;
            const int e = s * kMaxBatch + it;
            QP_HIP(hipEventElapsedTime(&t, p->ev_hot[2 * e], p->ev_hot[2 * e + 1]));
            pf->hot_ms += t;
            ++pf->hot_n;
            pf->hot_rhs += hot[it];
        }
        const int res = p->hexec[2 * kMaxBatch + s];
        if (rec[s].nres && res) {
            float t = 0.f;
            QP_HIP(hipEventElapsedTime(&t, p->ev_res[2 * s], p->ev_res[2 * s + 1]));
            pf->res_ms += t;
            ++pf->res_n;
            pf->res_rhs += res;
        }
        return QP_OK;
    }
    // Record the poll point of the batch just queued in the current slot (k
    // stiffness products, nres residual replacements).
    qp_status record(int k, int nres)
    {
        QP_HIP(hipMemcpyAsync(host_states(slot), p->st(), sizeof(State) * K, hipMemcpyDeviceToHost,
                              p->stream));
        if (prof) {
            QP_HIP(hipMemcpyAsync(p->hexec + slot * kMaxBatch, p->exec_hot() + slot * kMaxBatch,
                                  sizeof(int) * k, hipMemcpyDeviceToHost, p->stream));
            QP_HIP(hipMemcpyAsync(p->hexec + 2 * kMaxBatch + slot, p->exec_res() + slot, sizeof(int),
                                  hipMemcpyDeviceToHost, p->stream));
        }
        QP_HIP(hipEventRecord(p->ev_poll[slot], p->stream));
        rec[slot] = Rec{true, k, nres};
        return QP_OK;
    }
    bool other_pending() const { return rec[slot ^ 1].pending; }
    // Whether the older poll has arrived (blocking: wait for it).
    qp_status other_ready(bool blocking, bool &ready)
    {
        const int other = slot ^ 1;
        if (blocking) {
            QP_HIP(hipEventSynchronize(p->ev_poll[other]));
            ready = true;
            return QP_OK;
        }
        const hipError_t e = hipEventQuery(p->ev_poll[other]);
        if (e == hipErrorNotReady) {
            ready = false;
            return QP_OK;
        }
        QP_HIP(e);
        ready = true;
        return QP_OK;
    }
    // Consume the older poll (it has arrived): finished = every state done;
    // seen = the states it saw.
    qp_status take_other(bool &finished, const State **seen)
    {
        const int other = slot ^ 1;
        rec[other].pending = false;
        const State *hs = host_states(other);
        finished = true;
        for (int r = 0; r < K; ++r) finished = finished && hs[r].done != 0;
        *seen = hs;
        if (prof) {
            QP_TRY(account(other));
            // the next batch of this slot set starts from a clear log
            QP_TRY(clear_exec(other));
        }
        return QP_OK;
    }
    void flip() { slot ^= 1; }
    qp_status clear_exec(int s)
    {
        QP_HIP(hipMemsetAsync(p->exec_hot() + s * kMaxBatch, 0, sizeof(int) * kMaxBatch, p->stream));
        QP_HIP(hipMemsetAsync(p->exec_res() + s, 0, sizeof(int), p->stream));
        return QP_OK;
    }
    // Queue the copy of the final states (slot 2) behind everything queued.
    qp_status queue_final()
    {
        QP_HIP(hipMemcpyAsync(host_states(2), p->st(), sizeof(State) * K, hipMemcpyDeviceToHost,
                              p->stream));
        QP_TRY(queue_hist(p, K, p->stream));
        return QP_OK;
    }
    // After the final copy has arrived: account the polls never inspected.
    qp_status drain(State *out)
    {
        for (int s = 0; s < 2; ++s)
            if (rec[s].pending) {
                rec[s].pending = false;
                if (prof) QP_TRY(account(s));
            }
        const State *fin = host_states(2);
        for (int r = 0; r < K; ++r) out[r] = fin[r];
        return QP_OK;
    }
};

// Residual trend between polls: log-decay per iteration of the squared
// residual estimate the device reports.
struct Trend {
    int it = -1;
    double rr = 0.0;
    double rate = 0.0;  // < 0 once known
    void observe(int iters, double rr_now)
    {
        if (it >= 0 && iters > it && rr > 0.0 && rr_now > 0.0 && rr_now < rr)
            rate = std::log(rr_now / rr) / (iters - it);
        it = iters;
        rr = rr_now;
    }
    // iterations from the last observation until the estimate reaches target
    double iters_to(double target) const
    {
        if (!(rate < 0.0) || !(rr > 0.0)) return -1.0;
        if (rr <= target) return 0.0;
        return std::log(target / rr) / rate;
    }
};

// Length of the next batch when `need` more iterations are expected after
// the last observation and `queued` of them are already queued: just past the
// expected event (plus one), even, between 2 and the full batch.
int next_batch(double need, int queued, int full)
{
    if (need < 0.0) return full;
    const double rem = need - queued;
    int L = (int)std::ceil(std::max(rem, 0.0)) + 1;
    L = std::min(full, std::max(2, L));
    return (L + 1) & ~1;
}

// ---------------------------------------------------------------- solve jobs
//
// A solve of K right-hand sides as a state machine.  begin() queues the
// set-up and advance() queues batches of iterations and consumes the polls.
// A blocking advance waits for each poll (the single-problem entry points);
// a non-blocking one returns as soon as the poll it needs has not arrived,
// so one host thread keeps the solves of many problems, each on its own
// stream, in flight at once.  Both queue the same launches in the same order.
//
// FP64: C-PCG in batches sized from the residual trend.  FP32-IR: float C-PCG
// whose residual is replaced by the FP64 residual F' - Q X of the FP64
// solution X whenever the float residual has dropped by `inner_tol` (or
// reached tol); the replacement steps sit at the end of every batch and act
// on the paused right-hand sides; batches are sized to end just after the
// expected pause; an iteration limit ends with one forced replacement.
struct SolveJob {
    qp_problem *p = nullptr;
    int K = 0;
    const double *rhs = nullptr;
    double *U = nullptr;
    double tol = 0.0;
    bool ir = false, prof = false;
    bool one_launch = false;  // FP64 loop in one launch (small problems)
    // Called once the final states are queued (and again after a forced
    // replacement), before the final event is recorded: a homogenization
    // queues its A* there, behind the solve, instead of after the host has
    // seen the solve finish.  Set after begin().
    qp_status (*after_final)(void *) = nullptr;
    void *after_ctx = nullptr;
    enum Phase { kQueue, kWait, kFinal, kForce, kDone } phase = kDone;
    Profile pf;
    Poller poll;
    Trend trend[qp::kMaxRhs];
    int batch = 0, j = 0, k = 0;
    State st[qp::kMaxRhs];

    bool done() const { return phase == kDone; }

    // norms_ready (FP32-IR): the ||f'||^2 partials of the K right-hand sides
    // are already in parts.c (the corrector sources stored them).
    qp_status begin(qp_problem *p_, int K_, const double *rhs_, double *U_, double tol_,
                    bool norms_ready = false)
    {
        p = p_;
        K = K_;
        rhs = rhs_;
        U = U_;
        tol = tol_;
        after_final = nullptr;
        after_ctx = nullptr;
        ir = p->opt.precision == QP_PREC_FP32_IR;
        prof = p->opt.profile != 0;
        one_launch = !ir && !prof && !p->host.aniso && !p->host.half &&
                     p->host.D <= std::min(p->opt.small_dim, qp::kSmallMax);
        pf = Profile{};
        poll = Poller{};
        poll.p = p;
        poll.K = K;
        poll.prof = prof;
        poll.pf = &pf;
        for (auto &t : trend) t = Trend{};
        batch = batch_size(p->opt);
        j = 0;
        k = batch;
        if (prof) {
            QP_TRY(events_ready(p));
            QP_HIP(hipMemsetAsync(p->exec_hot(), 0, sizeof(int) * kExecInts, p->stream));
        }
        QP_HIP(hipEventRecord(p->ev_t0, p->stream));
        const qp::Parts parts = p->parts();
        QP_HIP(qp::launch_state_reset(K, p->st(), p->stream));
        if (ir) {
            if (norms_ready)
                QP_HIP(qp::launch_ir_unit_only(K, p->host, parts, p->st(), p->stream));
            else
                QP_HIP(qp::launch_ir_unit(K, p->tab, p->host, rhs, parts, p->st(), p->stream));
            QP_HIP(qp::launch_pcg_init(qp::F32, K, p->tab, p->host, rhs, U, p->x32(), p->r32(),
                                       p->h32(), p->M32(), parts, p->st(), p->stream));
            QP_HIP(qp::launch_pcg_start(qp::F32, K, p->host, tol, p->opt.inner_tol, p->opt.maxit,
                                        parts, p->st(), p->stream));
        } else {
            QP_HIP(qp::launch_pcg_init(qp::F64, K, p->tab, p->host, rhs, nullptr, U, p->r(), p->h(),
                                       p->M64(), parts, p->st(), p->stream));
            QP_HIP(qp::launch_pcg_start(qp::F64, K, p->host, tol, 0.0, p->opt.maxit, parts,
                                        p->st(), p->stream));
        }
        phase = kQueue;
        return QP_OK;
    }

    // Length of the batch after the queued one (k iterations) from the states
    // an older poll saw.
    int next_length(const State *seen)
    {
        if (!ir) {
            double need = 0.0;
            for (int r = 0; r < K; ++r) {
                if (seen[r].done) continue;
                if (trend[r].it < 0) trend[r].observe(0, seen[r].rr0);
                trend[r].observe(seen[r].iters, seen[r].rr);
                const double nr = trend[r].iters_to(seen[r].thresh);
                need = (nr < 0.0 || need < 0.0) ? -1.0 : std::max(need, nr);
            }
            return next_batch(need, k, batch);
        }
        // seen: after a replacement (scaled true residual rr = rr_last)
        int want = 2;
        for (int r = 0; r < K; ++r) {
            if (seen[r].done) continue;
            if (trend[r].it < 0) trend[r].observe(0, 1.0);
            trend[r].observe(seen[r].iters, seen[r].rr);
            const double target = std::max(seen[r].thresh, seen[r].delta2 * seen[r].rr_last);
            const double need = trend[r].iters_to(target);
            int L;
            if (need < 0.0) {
                return batch;
            } else if (need <= k) {
                // the queued batch reaches the next replacement point
                if (target <= seen[r].thresh) {
                    L = 2;  // and that one should converge
                } else {
                    const double t2 = std::max(seen[r].thresh, seen[r].delta2 * target);
                    L = next_batch(std::log(t2 / target) / trend[r].rate, 0, batch);
                }
            } else {
                L = next_batch(need, k, batch);
            }
            want = std::max(want, L);
        }
        return want;
    }

    qp_status event_ready(hipEvent_t e, bool blocking, bool &ready)
    {
        if (blocking) {
            QP_HIP(hipEventSynchronize(e));
            ready = true;
            return QP_OK;
        }
        const hipError_t q = hipEventQuery(e);
        ready = q != hipErrorNotReady;
        if (ready) QP_HIP(q);
        return QP_OK;
    }

    // Advance as far as possible; progressed = something was queued or consumed.
    qp_status advance(bool blocking, bool &progressed)
    {
        progressed = false;
        for (;;) {
            switch (phase) {
            case kQueue: {
                if (j >= p->opt.maxit) {
                    QP_TRY(begin_final());
                    progressed = true;
                    continue;
                }
                if (one_launch) {
                    // every iteration in one launch; then the final states
                    QP_HIP(qp::launch_pcg_wg(K, p->tab, p->host, U, p->r(), p->h(), p->M64(),
                                             p->st(), p->stream));
                    j = p->opt.maxit;
                    QP_TRY(begin_final());
                    progressed = true;
                    continue;
                }
                k = std::min(k, p->opt.maxit - j);
                QP_TRY(queue_batch(p, ir, K, U, rhs, k, poll.slot, prof));
                j += k;
                QP_TRY(poll.record(k, ir ? 1 : 0));
                progressed = true;
                if (poll.other_pending()) {
                    phase = kWait;
                } else {
                    poll.flip();
                    k = batch;
                }
                continue;
            }
            case kWait: {
                bool ready = false;
                QP_TRY(poll.other_ready(blocking, ready));
                if (!ready) return QP_OK;
                bool fin = false;
                const State *seen = nullptr;
                QP_TRY(poll.take_other(fin, &seen));
                poll.flip();
                progressed = true;
                if (fin) {
                    QP_TRY(begin_final());
                } else {
                    k = next_length(seen);
                    phase = kQueue;
                }
                continue;
            }
            case kFinal:
            case kForce: {
                bool ready = false;
                QP_TRY(event_ready(p->ev_fin, blocking, ready));
                if (!ready) return QP_OK;
                progressed = true;
                if (phase == kFinal) {
                    QP_TRY(poll.drain(st));
                    bool all_done = true;
                    for (int r = 0; r < K; ++r) all_done = all_done && st[r].done;
                    if (ir && !all_done) {
                        // iteration limit: fold every unfinished increment into X
                        // with one forced replacement, whose true residual
                        // decides the status
                        QP_HIP(qp::launch_ir_force(K, p->st(), p->stream));
                        QP_TRY(enqueue_replacement(p, K, U, rhs, p->opt.maxit, 0, false));
                        QP_HIP(hipEventRecord(p->ev_t1, p->stream));
                        QP_TRY(poll.queue_final());
                        if (after_final) QP_TRY(after_final(after_ctx));
                        QP_HIP(hipEventRecord(p->ev_fin, p->stream));
                        phase = kForce;
                        continue;
                    }
                } else {
                    const State *fin = poll.host_states(2);
                    for (int r = 0; r < K; ++r) {
                        st[r] = fin[r];
                        if (!st[r].done) st[r].status = QP_ENOCONV;
                    }
                }
                phase = kDone;
                return QP_OK;
            }
            case kDone:
                return QP_OK;
            }
        }
    }

    qp_status begin_final()
    {
        QP_HIP(hipEventRecord(p->ev_t1, p->stream));
        QP_TRY(poll.queue_final());
        if (after_final) QP_TRY(after_final(after_ctx));
        QP_HIP(hipEventRecord(p->ev_fin, p->stream));
        phase = kFinal;
        return QP_OK;
    }

    // Fill K infos (done() must hold); returns the first non-QP_OK status.
    qp_status finish(qp_solve_info *infos)
    {
        float ms = 0.f;
        QP_HIP(hipEventElapsedTime(&ms, p->ev_t0, p->ev_t1));
        qp_status worst = QP_OK;
        for (int r = 0; r < K; ++r) {
            qp_solve_info *info = infos + r;
            std::memset(info, 0, sizeof(*info));
            info->flags = p->flags;
            info->status = st[r].status;
            info->iters = st[r].iters;
            info->outer_iters = ir ? st[r].replacements : 0;
            info->rel_resid =
                ir ? std::sqrt(st[r].rr) : (st[r].rr0 > 0 ? std::sqrt(st[r].rr / st[r].rr0) : 0.0);
            info->seconds = ms * 1e-3;
            info->kappa_est =
                lanczos_kappa(p->hhist + (size_t)2 * qp::kHist * r, std::min(st[r].iters, qp::kHist));
            info->bytes_moved = solve_bytes(ir, (double)p->host.D, st[r].iters, info->outer_iters);
            if (prof) {
                if (ir) {
                    info->matvec32_ms = pf.hot_ms;
                    info->matvec32_launches = pf.hot_n;
                    info->matvec32_rhs = pf.hot_rhs;
                    info->matvec_ms = pf.res_ms;
                    info->matvec_launches = pf.res_n;
                    info->matvec_rhs = pf.res_rhs;
                } else {
                    info->matvec_ms = pf.hot_ms;
                    info->matvec_launches = pf.hot_n;
                    info->matvec_rhs = pf.hot_rhs;
                }
            }
            const qp_status s = (qp_status)st[r].status;
            if (s != QP_OK && worst == QP_OK) worst = s;
        }
        return worst;
    }
};

// Right-hand sides that one launch of this problem can serve together: the
// plane tiles with 32-bit gathers serve up to d; line tiles and 64-bit
// gathers one.
int rhs_per_launch(const qp_problem *p)
{
    return (p->host.tile_s <= 1 || p->host.wide) ? 1 : p->host.d;
}

qp_status report(qp_status worst)
{
    if (worst == QP_ENOTSPD) fail(worst, "PCG breakdown: (Q h, h) <= 0");
    else if (worst == QP_ENOCONV) fail(worst, "iteration limit reached before the tolerance");
    else if (worst == QP_ENONFINITE) fail(worst, "non-finite value in the right-hand side or residual");
    return worst;
}

// K right-hand sides (rhs + r D, solutions U + r D), solved in groups the
// launches can serve together; blocking.  infos: K entries or null.
qp_status solve_dispatch(qp_problem *p, int K, const double *rhs, double *U, double tol,
                         qp_solve_info *infos)
{
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(QP_EINVAL, "tol must be positive and finite");
    qp_solve_info local[qp::kMaxRhs];
    if (!infos) infos = local;
    const int G = rhs_per_launch(p);
    const size_t D2 = 2 * (size_t)p->host.D;
    qp_status worst = QP_OK;
    for (int r0 = 0; r0 < K; r0 += G) {
        const int Kg = std::min(G, K - r0);
        SolveJob job;
        QP_TRY(job.begin(p, Kg, rhs + r0 * D2, U + r0 * D2, tol));
        bool progressed = false;
        while (!job.done()) QP_TRY(job.advance(true, progressed));
        const qp_status s = job.finish(infos + r0);
        if (s != QP_OK && worst == QP_OK) worst = s;
    }
    return report(worst);
}

// A homogenization as a job: the d corrector right-hand sides, their solves
// (together where the launches allow), and A* (flux form, plus the energy
// form on request), with the same launches as qp_homogenized_ex.
struct HomJob {
    qp_problem *p = nullptr;
    double tol = 0.0;
    double *Astar = nullptr, *Aenergy = nullptr;
    qp_solve_info *infos = nullptr;
    qp_solve_info local[qp::kMaxRhs];
    SolveJob sj;
    int r0 = 0, G = 1;
    qp_status worst = QP_OK;
    enum Phase { kSolve, kAstar, kDone } phase = kDone;

    bool done() const { return phase == kDone; }

    qp_status begin(qp_problem *p_, double *Astar_, double *Aenergy_, double tol_,
                    qp_solve_info *infos_)
    {
        p = p_;
        Astar = Astar_;
        Aenergy = Aenergy_;
        tol = tol_;
        infos = infos_ ? infos_ : local;
        if (!(tol > 0.0) || !std::isfinite(tol))
            return fail(QP_EINVAL, "tol must be positive and finite");
        const int d = p->host.d;
        G = rhs_per_launch(p);
        // all d sources in one pass; when one solve serves them all, that pass
        // also stores the norms the FP32-IR start needs
        const bool one = G >= d && p->opt.precision == QP_PREC_FP32_IR;
        const qp::Parts parts = p->parts();
        QP_HIP(qp::launch_corrector_rhs_all(p->tab, p->host, d, p->F(), one ? &parts : nullptr,
                                            p->stream));
        r0 = 0;
        worst = QP_OK;
        QP_TRY(start_group(one));
        phase = kSolve;
        return QP_OK;
    }

    qp_status start_group(bool norms_ready = false)
    {
        const size_t D2 = 2 * (size_t)p->host.D;
        const int Kg = std::min(G, p->host.d - r0);
        QP_TRY(sj.begin(p, Kg, p->F() + r0 * D2, p->chi(0) + r0 * D2, tol, norms_ready));
        if (r0 + Kg >= p->host.d) {
            // the last group: A* goes behind its final states
            sj.after_final = &HomJob::astar_hook;
            sj.after_ctx = this;
        }
        return QP_OK;
    }

    static qp_status astar_hook(void *ctx) { return static_cast<HomJob *>(ctx)->queue_astar(); }

    // A* (flux form, and the energy form on request) of the correctors and
    // its copy to the host, queued on the problem's stream.
    qp_status queue_astar()
    {
        const int d = p->host.d;
        QP_HIP(qp::launch_astar(p->tab, p->host, p->chi(0), p->small(), p->stream));
        if (Aenergy) {
            const qp::Parts parts = p->parts();
            for (int j = 0; j < d; ++j) {
                QP_HIP(qp::launch_matvec(qp::F64, qp::EPI_NONE, 1, p->tab, p->host, p->recs(),
                                         p->urec(qp::F64), p->upku(qp::F64), p->chi(j), p->q(),
                                         nullptr, nullptr, parts, p->st(), nullptr, p->stream));
                for (int i = 0; i < d; ++i)
                    QP_HIP(qp::launch_dot(p->tab, p->host, p->chi(i), p->q(), parts,
                                          p->small() + 64 + i * d + j, p->stream));
            }
        }
        QP_HIP(hipMemcpyAsync(p->hsmall, p->small(), 128 * sizeof(double), hipMemcpyDeviceToHost,
                              p->stream));
        return QP_OK;
    }

    qp_status advance(bool blocking, bool &progressed)
    {
        progressed = false;
        const int d = p->host.d;
        while (phase == kSolve) {
            bool pr = false;
            QP_TRY(sj.advance(blocking, pr));
            progressed = progressed || pr;
            if (!sj.done()) return QP_OK;
            const qp_status s = sj.finish(infos + r0);
            if (s != QP_OK && worst == QP_OK) worst = s;
            r0 += G;
            if (r0 < d) {
                QP_TRY(start_group());
                progressed = true;
                continue;
            }
            if (worst == QP_EDEVICE || worst == QP_EINVAL) return worst;
            // A* and its copy were queued behind the last group's final
            // states (astar_hook), before that solve's final event
            phase = kAstar;
            progressed = true;
        }
        if (phase == kAstar) {
            bool ready = false;
            QP_TRY(sj.event_ready(p->ev_fin, blocking, ready));
            if (!ready) return QP_OK;
            for (int e = 0; e < d * d; ++e) Astar[e] = p->hsmall[e];
            if (Aenergy)
                for (int i = 0; i < d; ++i)
                    for (int j = 0; j < d; ++j)
                        Aenergy[i * d + j] =
                            (i == j ? p->host.a0l[i] : 0.0) - p->hsmall[64 + i * d + j];
            phase = kDone;
            progressed = true;
            if (worst != QP_OK) {
                report(worst);
                if (worst == QP_ENOCONV || worst == QP_ENOTSPD || worst == QP_ENONFINITE)
                    fail(worst, "a corrector solve did not converge");
            }
        }
        return QP_OK;
    }
};

}  // namespace

// ---------------------------------------------------------------- serving
//
// A request is a homogenization of a problem given by its description.  The
// server keeps created problems (workspace, tables, preconditioner) in a
// cache bounded by an HBM budget; a request is admitted, in arrival order,
// when its problem is cached and idle, or when the problem can be created
// within the budget after evicting idle problems (least recently used
// first).  Every admitted request runs as a HomJob on its problem's stream,
// so requests join and leave the running set one by one while the others
// keep iterating.
struct qp_server {
    size_t budget = 0, used = 0;
    qp_options opt{};
    struct Entry {
        std::string key;
        qp_problem *p = nullptr;
        size_t bytes = 0;
        bool busy = false;
        uint64_t last_use = 0;
    };
    std::vector<Entry> cache;
    struct Request {
        int64_t ticket = 0;
        std::string key;
        int d = 0, n = 0, N = 0, g = 0;
        bool diag = false;
        std::vector<double> P, coef;
        std::vector<int32_t> modes;
        double tol = 0.0;
        double *Astar = nullptr;
        qp_solve_info *infos = nullptr;
        size_t bytes = 0;
    };
    std::vector<Request> queue;
    struct Running {
        int64_t ticket = 0;
        size_t entry = 0;
        HomJob job;
    };
    std::vector<std::unique_ptr<Running>> running;
    struct Finished {
        int64_t ticket;
        qp_status status;
    };
    std::vector<Finished> finished;
    int64_t next_ticket = 1;
    uint64_t clock = 0;
};

namespace {

qp_status check_options(const qp_options *o)
{
    if (o->precision != QP_PREC_FP64 && o->precision != QP_PREC_FP32_IR)
        return fail(QP_EINVAL, "unknown precision %d", o->precision);
    if (o->precond != QP_PRECOND_PAPER && o->precond != QP_PRECOND_JACOBI)
        return fail(QP_EINVAL, "unknown preconditioner %d", o->precond);
    if (o->maxit < 1 || !(o->inner_tol > 0.0) || o->inner_tol >= 1.0 ||
        o->poll_every < 0 || o->poll_every > kMaxBatch)
        return fail(QP_EINVAL, "invalid iteration limits or inner tolerance");
    if (o->half_storage && o->gather64)
        return fail(QP_EINVAL, "half storage uses the 32-bit gathers (gather64 must be 0)");
    if (o->small_dim < 0) return fail(QP_EINVAL, "small_dim must not be negative");
    return QP_OK;
}

qp_status compute_setup(qp_problem *p)
{
    const qp::Parts parts = p->parts();
    QP_HIP(qp::launch_precond(p->tab, p->host, p->opt.precond, p->M64(), p->M32(), parts, p->small(),
                              p->stream));
    QP_HIP(qp::launch_extrema(p->tab, p->host, parts, p->small() + 1, p->stream));
    QP_HIP(hipMemcpyAsync(p->hsmall, p->small(), 3 * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    QP_HIP(hipStreamSynchronize(p->stream));
    p->pkmin = p->hsmall[0];
    p->amin = p->hsmall[1];
    p->amax = p->hsmall[2];
    return QP_OK;
}

}  // namespace

extern "C" {

void qp_default_options(qp_options *opt)
{
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->precision = QP_PREC_FP64;
    opt->precond = QP_PRECOND_PAPER;
    opt->maxit = 10000;
    opt->inner_tol = 1e-5;
    opt->poll_every = 0;
    opt->graphs = 1;
    opt->small_dim = 2048;
}

size_t qp_workspace_bytes(int d, int n, int N, int g)
{
    if (d < 1 || n < 1 || N < 2 || n > QP_MAX_DIM_N || d > QP_MAX_DIM_D) return 0;
    int64_t D = 1;
    for (int t = 0; t < n; ++t) {
        D *= N;
        if (D >= ((int64_t)1 << 31)) return 0;
    }
    if (g < 1 || g > QP_MAX_MODES) return 0;
    return make_layout(d, D, g, plane_units(n, N)).total;
}

// coefs: null (scalar coefficient `coef`) or d x g complex (diagonal coefficient)
// ---------------------------------------------------------------- product layout
//
// The work layout of the plane-tile stiffness product (tiles per wave item,
// workgroups, item order) leaves every output value unchanged: each output
// is summed by one lane over the modes in a fixed order.  It decides only
// which workgroup sums which partial dot products.  With
// qp_options.autotune the first problem of a shape times each candidate
// layout on its own product (the launch the solve repeats: its precision,
// all the right-hand sides one launch serves) and keeps the fastest; later
// problems of the same shape in the process reuse that choice.
}  // extern "C"

namespace {

struct LayoutPick {
    int it, nb, xcd;
    bool operator==(const LayoutPick &o) const { return it == o.it && nb == o.nb && xcd == o.xcd; }
};

std::mutex g_layout_mu;
std::map<std::vector<int>, std::pair<LayoutPick, LayoutPick>> g_layouts;  // float, FP64

int grid_for(int64_t want)
{
    int nb = (int)std::min<int64_t>(qp::kMaxBlocks, std::max<int64_t>(1, want));
    if (nb >= 8) nb -= nb % 8;
    return nb;
}

// Candidate layouts of a plane-tile table: 1, 2 or 4 tiles per item; one,
// two or four items per wave; XCD-front or linear item order.
std::vector<LayoutPick> layout_candidates(const Table &T)
{
    std::vector<LayoutPick> c;
    const int tpu = T.tiles_per_unit;
    const int64_t units = T.ntiles / tpu;
    for (int it : {1, 2, 4}) {
        if (it > 1 && it / 2 >= tpu) continue;  // same items as it / 2
        const int64_t items = units * ((tpu + it - 1) / it);
        for (int per : {1, 2, 4}) {
            const int nb = grid_for((items + 4 * per - 1) / (4 * per));
            for (int xcd : {1, 0, 2, 3}) {
                if (xcd == 2 && T.slab_span == 0) continue;
                if (xcd == 3 && (T.slab_span == 0 || T.n < 5)) continue;  // blocks need 3 uniform axes
                const LayoutPick L{it, nb, xcd};
                if (std::find(c.begin(), c.end(), L) == c.end()) c.push_back(L);
            }
        }
    }
    return c;
}

// The layout of the float (prec F32) or the FP64 launches.
qp_status apply_layout(qp_problem *p, const LayoutPick &L, int prec)
{
    if (prec == qp::F32) {
        p->host.item_tiles = L.it;
        p->host.nb_mv = L.nb;
        p->host.xcd_front = L.xcd;
    } else {
        p->host.item_tiles64 = L.it;
        p->host.nb_mv64 = L.nb;
        p->host.xcd_front64 = L.xcd;
    }
    QP_HIP(hipMemcpyAsync(p->tab, &p->host, sizeof(Table), hipMemcpyHostToDevice, p->stream));
    QP_HIP(hipStreamSynchronize(p->stream));
    return QP_OK;
}

// Mean duration of `reps` products (after one untimed), microseconds, as a
// solve launches them: the product of precision prec with its alpha
// partials, or (resid, FP64) the residual replacement of FP32-IR.  The
// states are set so that every launch does its work.
qp_status time_product(qp_problem *p, int prec, bool resid, int reps, double &us)
{
    const bool f32 = prec == qp::F32;
    const int K = rhs_per_launch(p);
    QP_HIP(qp::launch_state_reset(K, p->st(), p->stream));
    if (resid) {
        // paused, then marked for replacement by the fold (x is zero: X stays)
        QP_HIP(qp::launch_ir_force(K, p->st(), p->stream));
        QP_HIP(qp::launch_ir_fold(K, p->tab, p->host, p->h(), p->x32(), p->st(), p->stream));
    }
    const int epi = resid ? qp::EPI_RESID : qp::EPI_ALPHA;
    const void *x = f32 ? (const void *)p->h32() : (const void *)p->h();
    void *y = resid ? (void *)p->r32() : (f32 ? (void *)p->q32() : (void *)p->q());
    const double *f = resid ? p->F() : nullptr;
    for (int r = 0; r <= reps; ++r) {
        if (r == 1) QP_HIP(hipEventRecord(p->ev_t0, p->stream));
        QP_HIP(qp::launch_matvec(prec, epi, K, p->tab, p->host, p->recs(), p->urec(prec),
                                 p->upku(prec), x, y, f, p->M32(), p->parts(), p->st(), nullptr,
                                 p->stream));
    }
    QP_HIP(hipEventRecord(p->ev_t1, p->stream));
    QP_HIP(hipEventSynchronize(p->ev_t1));
    float ms = 0.f;
    QP_HIP(hipEventElapsedTime(&ms, p->ev_t0, p->ev_t1));
    us = 1e3 * ms / reps;
    return QP_OK;
}

// One layout search: each candidate timed on the launch kind given
// (time_product's prec and resid), the heuristic layout kept unless a
// candidate is at least 3% faster.
qp_status search_layout(qp_problem *p, int prec, bool resid, LayoutPick &best, double &dflt_us,
                        double &best_us, int &ncand)
{
    const Table &T = p->host;
    const LayoutPick dflt = (prec == qp::F32) ? LayoutPick{T.item_tiles, T.nb_mv, T.xcd_front}
                                              : LayoutPick{T.item_tiles64, T.nb_mv64, T.xcd_front64};
    double est = 0.0;
    QP_TRY(time_product(p, prec, resid, 3, est));
    // about 2 ms of launches per candidate
    const int reps = (int)std::min(50.0, std::max(3.0, std::ceil(2000.0 / std::max(est, 1.0))));
    const std::vector<LayoutPick> cands = layout_candidates(T);
    best = dflt;
    QP_TRY(time_product(p, prec, resid, reps, dflt_us));
    best_us = dflt_us;
    for (const LayoutPick &L : cands) {
        if (L == dflt) continue;
        QP_TRY(apply_layout(p, L, prec));
        double us = 0.0;
        QP_TRY(time_product(p, prec, resid, reps, us));
        // a layout replaces the heuristic one only when clearly faster
        if (us < 0.97 * best_us) {
            best = L;
            best_us = us;
        }
    }
    QP_TRY(apply_layout(p, best, prec));
    ncand = (int)cands.size();
    return QP_OK;
}

void report_layout(qp_problem *p, int tuned)
{
    const Table &T = p->host;
    qp_layout &L = p->layout;
    L.item_tiles = T.item_tiles;
    L.workgroups = T.nb_mv;
    L.xcd_front = T.xcd_front;
    L.item_tiles64 = T.item_tiles64;
    L.workgroups64 = T.nb_mv64;
    L.xcd_front64 = T.xcd_front64;
    L.tuned = tuned;
}

// FP32-IR problems tune the float product (the iterations) and, apart, the
// FP64 residual product of the replacements; FP64 problems tune their FP64
// product and keep the heuristic float layout.
qp_status tune_layout(qp_problem *p)
{
    const Table &T = p->host;
    p->layout = qp_layout{};
    report_layout(p, 0);
    if (T.tile_s <= 1) return QP_OK;  // line tiles: one layout
    const std::vector<int> key = {T.d,         T.n,    T.N,      T.g,              T.aniso,
                                  T.real_coef, T.wide, T.tile_s, p->opt.precision, T.half};
    {
        std::lock_guard<std::mutex> lock(g_layout_mu);
        const auto f = g_layouts.find(key);
        if (f != g_layouts.end()) {
            QP_TRY(apply_layout(p, f->second.first, qp::F32));
            QP_TRY(apply_layout(p, f->second.second, qp::F64));
            report_layout(p, 2);
            return QP_OK;
        }
    }
    // zero sources; the products write q or r and the partials
    const int K = rhs_per_launch(p);
    const bool f32 = p->opt.precision == QP_PREC_FP32_IR;
    QP_HIP(hipMemsetAsync(p->h(), 0, 16 * (size_t)T.D * K, p->stream));
    if (f32) {
        QP_HIP(hipMemsetAsync(p->h32(), 0, 8 * (size_t)T.D * K, p->stream));
        QP_HIP(hipMemsetAsync(p->x32(), 0, 8 * (size_t)T.D * K, p->stream));
        QP_HIP(hipMemsetAsync(p->F(), 0, 16 * (size_t)T.D * K, p->stream));
    }
    LayoutPick b32{T.item_tiles, T.nb_mv, T.xcd_front}, b64{};
    double d32 = 0.0, s32 = 0.0, d64 = 0.0, s64 = 0.0;
    int n32 = 0, n64 = 0;
    if (f32) QP_TRY(search_layout(p, qp::F32, false, b32, d32, s32, n32));
    QP_TRY(search_layout(p, qp::F64, f32, b64, d64, s64, n64));
    QP_HIP(qp::launch_state_reset(qp::kMaxRhs, p->st(), p->stream));
    QP_HIP(hipStreamSynchronize(p->stream));
    report_layout(p, 1);
    p->layout.candidates = n32 + n64;
    p->layout.default_us = d32;
    p->layout.best_us = s32;
    p->layout.default64_us = d64;
    p->layout.best64_us = s64;
    std::lock_guard<std::mutex> lock(g_layout_mu);
    g_layouts.emplace(key, std::make_pair(b32, b64));
    return QP_OK;
}

}  // namespace
extern "C" {

static qp_status create_problem(qp_problem **out, int d, int n, const double *P, int g,
                                const int32_t *modes, const double *coef, const double *coefs,
                                int N, const qp_options *opt)
{
    g_last_error.clear();
    if (!out) return fail(QP_EINVAL, "out is null");
    *out = nullptr;
    if (coefs) {
        if (d < 1 || d > QP_MAX_DIM_D) return fail(QP_EINVAL, "d=%d outside [1, %d]", d, QP_MAX_DIM_D);
        for (int l = 0; l < d; ++l) {
            const qp_status s = check_args(d, n, P, g, modes, coefs + 2 * (size_t)l * g, N);
            if (s != QP_OK) return s;  // the message names the failing check
        }
        coef = coefs;
    } else {
        QP_TRY(check_args(d, n, P, g, modes, coef, N));
    }
    qp_options o;
    qp_default_options(&o);
    if (opt) o = *opt;
    QP_TRY(check_options(&o));

    qp_problem *p = new (std::nothrow) qp_problem();
    if (!p) return fail(QP_ENOMEM, "host allocation failed");
    p->opt = o;
    build_table(p->host, d, n, P, g, modes, coef, coefs, N);
    if (o.half_storage) {
        if (N % 2 == 0) {
            delete p;
            return fail(QP_EINVAL, "half storage needs odd N (N = %d)", N);
        }
        if (coefs || !p->host.real_coef) {
            delete p;
            return fail(QP_EINVAL, "half storage needs a real scalar coefficient");
        }
        if (!plane_tiles(n, N)) {
            delete p;
            return fail(QP_EINVAL, "half storage needs plane tiles (n >= 2, N <= 32)");
        }
        make_half(p->host);
    }
    stream_grid(p->host, o.precision);
    // record indices of the default gathers are scaled by the record size in
    // 32 bits; the largest records are the interleaved float families of d
    // right-hand sides (d * 8 bytes) and FP64 entries (16 bytes): vectors
    // reaching 4 GiB in either take 64-bit addresses
    if (p->host.tile_s > 1 &&
        (o.gather64 || (int64_t)p->host.D * std::max(2, d) * 8 >= ((int64_t)1 << 32)))
        p->host.wide = 1;
    p->L = make_layout(d, p->host.D, g,
                       p->host.tile_s > 1 ? p->host.ntiles / p->host.tiles_per_unit : 0);

    auto bail = [&](qp_status st) {
        release(p);
        return st;
    };
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1)
        return bail(fail(QP_EDEVICE, "no HIP device available"));
    if (hipGetDevice(&p->device) != hipSuccess) return bail(fail(QP_EDEVICE, "hipGetDevice failed"));
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, p->device) != hipSuccess)
        return bail(fail(QP_EDEVICE, "hipGetDeviceProperties failed"));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return bail(fail(QP_EDEVICE, "device %d is %s; this library is built for gfx950", p->device,
                         prop.gcnArchName));
    if (o.stream) {
        p->stream = static_cast<hipStream_t>(o.stream);
    } else {
        if (hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking) != hipSuccess)
            return bail(fail(QP_EDEVICE, "hipStreamCreate failed"));
        p->own_stream = true;
    }
    if (o.workspace) {
        if (o.workspace_bytes < p->L.total)
            return bail(fail(QP_ENOMEM, "workspace has %zu bytes, %zu needed", o.workspace_bytes,
                             p->L.total));
        if (reinterpret_cast<uintptr_t>(o.workspace) % kAlign != 0)
            return bail(fail(QP_EINVAL, "workspace must be 256-byte aligned"));
        p->ws = static_cast<char *>(o.workspace);
    } else {
        if (hipMalloc(&p->ws, p->L.total) != hipSuccess)
            return bail(fail(QP_ENOMEM, "hipMalloc of %zu bytes failed", p->L.total));
        p->own_ws = true;
    }
    p->opt.workspace = nullptr;
    if (hipHostMalloc(&p->hstate, 3 * qp::kMaxRhs * sizeof(State), hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc(&p->hsmall, 128 * sizeof(double), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&p->hexec, kExecInts * sizeof(int), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&p->hhist, sizeof(double) * 2 * qp::kHist * qp::kMaxRhs,
                      hipHostMallocDefault) != hipSuccess)
        return bail(fail(QP_ENOMEM, "pinned host allocation failed"));
    for (auto &e : p->ev_poll)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            return bail(fail(QP_EDEVICE, "hipEventCreate failed"));
    if (hipEventCreateWithFlags(&p->ev_fin, hipEventDisableTiming) != hipSuccess)
        return bail(fail(QP_EDEVICE, "hipEventCreate failed"));
    if (hipEventCreate(&p->ev_t0) != hipSuccess || hipEventCreate(&p->ev_t1) != hipSuccess)
        return bail(fail(QP_EDEVICE, "hipEventCreate failed"));
    p->tab = p->at<Table>(p->L.tab);
    if (hipMemcpyAsync(p->tab, &p->host, sizeof(Table), hipMemcpyHostToDevice, p->stream) != hipSuccess)
        return bail(fail(QP_EDEVICE, "table upload failed"));
    // each state's Lanczos-coefficient slice (the state resets keep it)
    if (qp::launch_state_hist(p->st(), p->hist(0), p->stream) != hipSuccess)
        return bail(fail(QP_EDEVICE, "state set-up failed"));
    build_mode_records(p->host, p->recs_host);
    if (hipMemcpyAsync(const_cast<qp::ModeRec *>(p->recs()), p->recs_host.data(),
                       sizeof(qp::ModeRec) * p->recs_host.size(), hipMemcpyHostToDevice,
                       p->stream) != hipSuccess)
        return bail(fail(QP_EDEVICE, "mode record upload failed"));
    for (int prec = 0; prec < 2; ++prec)
        if (qp::launch_unit_records(prec, p->tab, p->host, p->recs(), p->urec(prec), p->upku(prec),
                                    p->stream) != hipSuccess)
            return bail(fail(QP_EDEVICE, "unit record set-up failed"));
    qp_status s = compute_setup(p);
    if (s != QP_OK) return bail(s);

    double pn = 0.0;
    for (int i = 0; i < d * n; ++i) pn += P[i] * P[i];
    if (!(p->pkmin >= 1e-24 * pn))
        return bail(fail(QP_EINVAL, "P k = 0 for a nonzero k in the grid (dependent columns of P)"));
    const double scale = std::max(std::fabs(p->amin), std::fabs(p->amax));
    if (p->amin < -1e-12 * scale) {
        if (!o.allow_indefinite)
            return bail(fail(QP_ENOTELLIPTIC, "coefficient minimum on the grid is %.6g < 0", p->amin));
        p->flags |= QP_FLAG_INDEFINITE;
    }
    if (std::fabs(p->amin) <= 1e-12 * scale) p->flags |= QP_FLAG_DEGENERATE;
    p->layout = qp_layout{};
    report_layout(p, 0);
    if (o.autotune) {
        s = tune_layout(p);
        if (s != QP_OK) return bail(s);
    }
    *out = p;
    return QP_OK;
}

qp_status qp_product_layout(const qp_problem *p, qp_layout *out)
{
    if (!p || !out) return fail(QP_EINVAL, "null argument");
    *out = p->layout;
    return QP_OK;
}

qp_status qp_set_product_layout(qp_problem *p, const qp_layout *layout)
{
    if (!p || !layout) return fail(QP_EINVAL, "null argument");
    const qp_layout &L = *layout;
    const bool plane = p->host.tile_s > 1;
    if (L.workgroups < 1 || L.workgroups > qp::kMaxBlocks)
        return fail(QP_EINVAL, "workgroups = %d outside [1, %d]", L.workgroups, qp::kMaxBlocks);
    if (plane ? (L.item_tiles != 1 && L.item_tiles != 2 && L.item_tiles != 4) : L.item_tiles != 1)
        return fail(QP_EINVAL, "item_tiles = %d is not 1, 2 or 4 (1 for line tiles)", L.item_tiles);
    if (L.xcd_front < 0 || L.xcd_front > 3) return fail(QP_EINVAL, "xcd_front must be 0, 1, 2 or 3");
    if (L.workgroups64 > 0) {
        if (L.workgroups64 > qp::kMaxBlocks)
            return fail(QP_EINVAL, "workgroups64 = %d outside [1, %d]", L.workgroups64, qp::kMaxBlocks);
        if (plane ? (L.item_tiles64 != 1 && L.item_tiles64 != 2 && L.item_tiles64 != 4)
                  : L.item_tiles64 != 1)
            return fail(QP_EINVAL, "item_tiles64 = %d is not 1, 2 or 4 (1 for line tiles)",
                        L.item_tiles64);
        if (L.xcd_front64 < 0 || L.xcd_front64 > 3)
            return fail(QP_EINVAL, "xcd_front64 must be 0, 1, 2 or 3");
    } else if (L.workgroups64 < 0) {
        return fail(QP_EINVAL, "workgroups64 = %d is negative", L.workgroups64);
    }
    // launches queued earlier read the table; captured batches hold the old grid
    QP_HIP(hipStreamSynchronize(p->stream));
    for (auto &G : p->graphs) (void)hipGraphExecDestroy(G.exec);
    p->graphs.clear();
    QP_TRY(apply_layout(p, LayoutPick{L.item_tiles, L.workgroups, L.xcd_front}, qp::F32));
    if (L.workgroups64 > 0)
        QP_TRY(apply_layout(p, LayoutPick{L.item_tiles64, L.workgroups64, L.xcd_front64}, qp::F64));
    else
        QP_TRY(apply_layout(p, LayoutPick{L.item_tiles, L.workgroups, L.xcd_front}, qp::F64));
    p->layout = qp_layout{};
    report_layout(p, 0);
    return QP_OK;
}

qp_status qp_create(qp_problem **out, int d, int n, const double *P, int g, const int32_t *modes,
                    const double *coef, int N, const qp_options *opt)
{
    return create_problem(out, d, n, P, g, modes, coef, nullptr, N, opt);
}

qp_status qp_create_diag(qp_problem **out, int d, int n, const double *P, int g,
                         const int32_t *modes, const double *coefs, int N, const qp_options *opt)
{
    if (!coefs) return fail(QP_EINVAL, "null coefs");
    return create_problem(out, d, n, P, g, modes, nullptr, coefs, N, opt);
}

void qp_destroy(qp_problem *p)
{
    if (!p) return;
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    release(p);
}

int64_t qp_dim(const qp_problem *p) { return p ? (int64_t)p->host.D : 0; }

qp_status qp_set_options(qp_problem *p, const qp_options *opt)
{
    if (!p || !opt) return fail(QP_EINVAL, "null argument");
    QP_TRY(check_options(opt));
    const int old_precond = p->opt.precond, old_precision = p->opt.precision;
    const int half = p->opt.half_storage;
    void *stream = p->opt.stream;
    p->opt = *opt;
    p->opt.stream = stream;
    p->opt.workspace = nullptr;
    p->opt.half_storage = half;  // the storage is fixed at creation
    if (opt->precision != old_precision) {
        // the streaming grid follows the precision; captured batches hold the old one
        QP_HIP(hipStreamSynchronize(p->stream));
        for (auto &G : p->graphs) (void)hipGraphExecDestroy(G.exec);
        p->graphs.clear();
        stream_grid(p->host, opt->precision);
        QP_HIP(hipMemcpyAsync(p->tab, &p->host, sizeof(Table), hipMemcpyHostToDevice, p->stream));
        QP_HIP(hipStreamSynchronize(p->stream));
    }
    if (opt->precond != old_precond) return compute_setup(p);
    return QP_OK;
}

qp_status qp_solve_d(qp_problem *p, const double *rhs, double *u, double tol, qp_solve_info *info)
{
    if (!p || !rhs || !u) return fail(QP_EINVAL, "null argument");
    if (overlaps(rhs, u, 16 * (size_t)p->host.D)) return fail(QP_EINVAL, "rhs and u must not overlap");
    return solve_dispatch(p, 1, rhs, u, tol, info);
}

qp_status qp_solve_multi_d(qp_problem *p, int K, const double *rhs, double *u, double tol,
                           qp_solve_info *infos)
{
    if (!p || !rhs || !u) return fail(QP_EINVAL, "null argument");
    if (K < 1 || K > p->host.d)
        return fail(QP_EINVAL, "K = %d right-hand sides outside [1, d = %d]", K, p->host.d);
    if (overlaps(rhs, u, 16 * (size_t)p->host.D * K))
        return fail(QP_EINVAL, "rhs and u must not overlap");
    return solve_dispatch(p, K, rhs, u, tol, infos);
}

qp_status qp_solve(qp_problem *p, const double *rhs, double *u, double tol, qp_solve_info *info)
{
    if (!p || !rhs || !u) return fail(QP_EINVAL, "null argument");
    const size_t bytes = 16 * (size_t)p->host.D;
    QP_HIP(hipMemcpyAsync(p->F(), rhs, bytes, hipMemcpyHostToDevice, p->stream));
    qp_status s = solve_dispatch(p, 1, p->F(), p->U(), tol, info);
    if (s == QP_EDEVICE || s == QP_EINVAL) return s;
    QP_HIP(hipMemcpyAsync(u, p->U(), bytes, hipMemcpyDeviceToHost, p->stream));
    QP_HIP(hipStreamSynchronize(p->stream));
    return s;
}

qp_status qp_corrector_d(qp_problem *p, int j, double *chi, double tol, qp_solve_info *info)
{
    if (!p) return fail(QP_EINVAL, "null problem");
    if (j < 0 || j >= p->host.d) return fail(QP_EINVAL, "corrector index %d outside [0, d)", j);
    QP_HIP(qp::launch_corrector_rhs(p->tab, p->host, j, p->F(), p->stream));
    qp_status s = solve_dispatch(p, 1, p->F(), p->chi(j), tol, info);
    if (s == QP_EDEVICE || s == QP_EINVAL) return s;
    if (chi) {
        QP_HIP(hipMemcpyAsync(chi, p->chi(j), 16 * (size_t)p->host.D, hipMemcpyDeviceToDevice, p->stream));
        QP_HIP(hipStreamSynchronize(p->stream));
    }
    return s;
}

qp_status qp_corrector(qp_problem *p, int j, double *chi, double tol, qp_solve_info *info)
{
    qp_status s = qp_corrector_d(p, j, nullptr, tol, info);
    if (s == QP_EDEVICE || s == QP_EINVAL) return s;
    if (chi) {
        QP_HIP(hipMemcpyAsync(chi, p->chi(j), 16 * (size_t)p->host.D, hipMemcpyDeviceToHost, p->stream));
        QP_HIP(hipStreamSynchronize(p->stream));
    }
    return s;
}

qp_status qp_homogenized_ex(qp_problem *p, double *Astar, double *Astar_energy, double tol,
                            qp_solve_info *info)
{
    if (!p || !Astar) return fail(QP_EINVAL, "null argument");
    HomJob job;
    QP_TRY(job.begin(p, Astar, Astar_energy, tol, info));
    bool progressed = false;
    while (!job.done()) QP_TRY(job.advance(true, progressed));
    return job.worst;
}

qp_status qp_homogenized_batch(qp_problem *const *problems, int count, double *Astar, double tol,
                               qp_solve_info *infos)
{
    if (!problems || !Astar || count < 1) return fail(QP_EINVAL, "null argument or empty batch");
    for (int i = 0; i < count; ++i) {
        if (!problems[i]) return fail(QP_EINVAL, "problem %d is null", i);
        for (int k = 0; k < i; ++k)
            if (problems[k] == problems[i]) return fail(QP_EINVAL, "problem %d repeats problem %d", i, k);
    }
    std::vector<HomJob> jobs(count);
    size_t ao = 0, io = 0;
    for (int i = 0; i < count; ++i) {
        const int d = problems[i]->host.d;
        QP_TRY(jobs[i].begin(problems[i], Astar + ao, nullptr, tol, infos ? infos + io : nullptr));
        ao += (size_t)d * d;
        io += d;
    }
    // Round robin: every job queues what it can and returns when the poll it
    // needs has not arrived; the streams run concurrently on the device.
    for (;;) {
        bool all = true, any = false;
        for (auto &J : jobs) {
            if (J.done()) continue;
            bool pr = false;
            const qp_status s = J.advance(false, pr);
            if (s != QP_OK) {
                for (auto &K : jobs) (void)hipStreamSynchronize(K.p->stream);
                return s;
            }
            any = any || pr;
            all = all && J.done();
        }
        if (all) break;
        if (!any) std::this_thread::yield();
    }
    qp_status worst = QP_OK;
    for (auto &J : jobs)
        if (J.worst != QP_OK && worst == QP_OK) worst = J.worst;
    if (worst != QP_OK) fail(worst, "a corrector solve of the batch did not converge");
    return worst;
}

// ---------------------------------------------------------------- grouped batch
//
// The corrector solves of several FP32-IR problems as one launch sequence:
// every step (float product, update, direction; fold, FP64 residual,
// replacement direction) is one launch whose workgroups are the problems'
// own workgroups one after the other (GroupEntry, owner tables), so the
// device sees one launch per step for the whole batch.  Each problem's
// workgroups compute exactly what a launch of that problem alone computes,
// so the values equal standalone solves.  The replacement steps follow every
// second iteration (a paused right-hand side waits at most one iteration;
// with nothing paused they exit at once), the host polls every poll_every
// iterations.
}  // extern "C"

namespace {

std::mutex g_group_mu;  // the group buffers below serve one call at a time
struct GroupBuffers {
    int device = -1;
    char *dev = nullptr;
    size_t dev_bytes = 0;
    State *host = nullptr;  // pinned: 3 slots of states
    size_t host_states = 0;
};
GroupBuffers g_gb;
// Problems per grouped call: the no-allocation variant's polls carry one done
// bit per problem in kGroupWords words per slot (problem 0's pinned scratch
// words hold two slots).
constexpr int kMaxGroup = 4096;
constexpr int kGroupWords = kMaxGroup / 32;
// Host image of the no-allocation variant's group table (entries and owner
// arrays), the size of the device scratch array; used under g_group_mu.
alignas(256) char g_group_host[qp::kGroupScratchBytes];

qp_status group_buffers(int device, size_t dev_bytes, size_t nstates)
{
    if (g_gb.device != device) {
        if (g_gb.dev) (void)hipFree(g_gb.dev);
        if (g_gb.host) (void)hipHostFree(g_gb.host);
        g_gb = GroupBuffers{};
        g_gb.device = device;
    }
    if (dev_bytes > g_gb.dev_bytes) {
        if (g_gb.dev) (void)hipFree(g_gb.dev);
        g_gb.dev = nullptr;
        g_gb.dev_bytes = 0;
        if (hipMalloc(&g_gb.dev, dev_bytes) != hipSuccess)
            return fail(QP_ENOMEM, "group table of %zu bytes", dev_bytes);
        g_gb.dev_bytes = dev_bytes;
    }
    if (nstates > g_gb.host_states) {
        if (g_gb.host) (void)hipHostFree(g_gb.host);
        g_gb.host = nullptr;
        g_gb.host_states = 0;
        if (hipHostMalloc(&g_gb.host, 3 * nstates * sizeof(State), hipHostMallocDefault) != hipSuccess)
            return fail(QP_ENOMEM, "pinned group states");
        g_gb.host_states = nstates;
    }
    return QP_OK;
}

// Why p cannot join a group led by p0 (null: it can).
const char *group_mismatch(const qp_problem *p, const qp_problem *p0)
{
    if (p->opt.precision != QP_PREC_FP32_IR) return "precision is not FP32-IR";
    if (p->host.tile_s <= 1 || p->host.wide) return "not a plane-tile problem with 32-bit gathers";
    if (p->host.aniso) return "diagonal coefficient";
    if (p->host.half) return "Hermitian half storage";
    if (p->host.d != 2 && p->host.d != 3) return "d is not 2 or 3";
    if (p->host.d != p0->host.d) return "d differs from problem 0";
    if (p->host.real_coef != p0->host.real_coef) return "real/complex coefficient differs from problem 0";
    if (p->device != p0->device) return "device differs from problem 0";
    if (p->opt.maxit != p0->opt.maxit) return "maxit differs from problem 0";
    return nullptr;
}

}  // namespace

namespace {

// The grouped homogenization of qp_homogenized_grouped (noalloc false: group
// tables in library memory allocated on first use, polls copy the states to
// pinned memory) and of qp_homogenized_grouped_noalloc (noalloc true: group
// tables in the library's static device array, polls copy one done bit per
// problem into problem 0's pinned scratch words; no device, pinned or host
// heap allocation).  Both queue the same solver launches.  As a job:
// begin() validates, builds the group table and queues every problem's
// set-up; advance() keeps two chunks of iterations in flight and consumes
// their polls; once every problem is done (or at the iteration limit) it
// queues the final steps, waits for them and writes A* and the infos.  The
// group buffers stay locked from begin() until the job ends.
struct GroupJob {
    std::vector<qp_problem *> probs;
    double *Astar = nullptr;
    qp_solve_info *infos = nullptr;
    double tol = 0.0;
    bool noalloc = false;
    int G = 0, d = 0, K = 0;
    hipStream_t s = nullptr;
    std::unique_lock<std::mutex> lock;
    std::vector<char> hvec;
    qp::GroupEntry *ents = nullptr, *E = nullptr;
    int *own_mv = nullptr, *own_mv64 = nullptr, *own_st = nullptr;
    int *owner_mv = nullptr, *owner_mv64 = nullptr, *owner_st = nullptr;
    State *dstates = nullptr;     // noalloc false
    uint32_t *dwords = nullptr;   // noalloc true
    uint32_t *hwords = nullptr;   // problem 0's pinned scratch words: two slots of done words
    size_t nst = 0;
    int gpmax = 4;
    std::vector<unsigned char> running;
    int n_mv = 0, n_mv64 = 0, n_st = 0;  // workgroups of the current launches
    int maxit = 0, full = 0, j = 0, slot = 0, inflight = 0;
    bool fin = false, finished = false;
    qp_status worst = QP_OK;

    bool done() const { return finished; }

    qp_status begin(qp_problem *const *problems, int count, double *Astar_, double tol_,
                    qp_solve_info *infos_, bool noalloc_)
    {
        if (!problems || !Astar_ || count < 1) return fail(QP_EINVAL, "null argument or empty group");
        if (count > kMaxGroup)
            return fail(QP_EINVAL, "%d problems exceed the group limit %d", count, kMaxGroup);
        if (!(tol_ > 0.0) || !std::isfinite(tol_)) return fail(QP_EINVAL, "tol must be positive and finite");
        for (int i = 0; i < count; ++i) {
            if (!problems[i]) return fail(QP_EINVAL, "problem %d is null", i);
            for (int k = 0; k < i; ++k)
                if (problems[k] == problems[i]) return fail(QP_EINVAL, "problem %d repeats problem %d", i, k);
            if (const char *why = group_mismatch(problems[i], problems[0]))
                return fail(QP_EINVAL, "problem %d cannot join the group: %s", i, why);
        }
        probs.assign(problems, problems + count);
        Astar = Astar_;
        infos = infos_;
        tol = tol_;
        noalloc = noalloc_;
        qp_problem *p0 = probs[0];
        G = count;
        d = p0->host.d;
        K = d;
        s = p0->stream;

        // sizes of the group table: entries, then the owner of every workgroup
        // of the float product, of the FP64 product and of the vector steps,
        // then the poll area (three slots of states, or two slots of done words)
        size_t tot_mv = 0, tot_mv64 = 0, tot_st = 0;
        for (int i = 0; i < G; ++i) {
            tot_mv += (size_t)probs[i]->host.nb_mv;
            tot_mv64 += (size_t)probs[i]->host.nb_mv64;
            tot_st += (size_t)probs[i]->host.nblocks;
        }
        nst = (size_t)G * K;
        const size_t o_own_mv = align_up(sizeof(qp::GroupEntry) * G);
        const size_t o_own_mv64 = align_up(o_own_mv + sizeof(int) * tot_mv);
        const size_t o_own_st = align_up(o_own_mv64 + sizeof(int) * tot_mv64);
        const size_t o_poll = align_up(o_own_st + sizeof(int) * tot_st);
        const size_t bytes = o_poll + (noalloc ? sizeof(uint32_t) * 2 * kGroupWords
                                               : 3 * nst * sizeof(State));

        lock = std::unique_lock<std::mutex>(g_group_mu);
        char *dev = nullptr;   // device group table
        char *hbuf = nullptr;  // host image of its first o_poll bytes
        if (noalloc) {
            void *ptr = nullptr;
            size_t cap = 0;
            QP_HIP(qp::group_scratch(p0->device, &ptr, &cap));
            if (bytes > cap || o_poll > sizeof(g_group_host))
                return fail(QP_EINVAL, "group table of %zu bytes exceeds the %zu-byte scratch array "
                            "(fewer or smaller problems)", bytes, cap);
            dev = static_cast<char *>(ptr);
            hbuf = g_group_host;
        } else {
            QP_TRY(group_buffers(p0->device, bytes, nst));
            dev = g_gb.dev;
            hvec.resize(o_poll);
            hbuf = hvec.data();
        }
        for (int i = 0; i < G; ++i) QP_HIP(hipStreamSynchronize(probs[i]->stream));

        ents = reinterpret_cast<qp::GroupEntry *>(hbuf);
        own_mv = reinterpret_cast<int *>(hbuf + o_own_mv);
        own_mv64 = reinterpret_cast<int *>(hbuf + o_own_mv64);
        own_st = reinterpret_cast<int *>(hbuf + o_own_st);
        E = reinterpret_cast<qp::GroupEntry *>(dev);
        owner_mv = reinterpret_cast<int *>(dev + o_own_mv);
        owner_mv64 = reinterpret_cast<int *>(dev + o_own_mv64);
        owner_st = reinterpret_cast<int *>(dev + o_own_st);
        dstates = reinterpret_cast<State *>(dev + o_poll);
        dwords = reinterpret_cast<uint32_t *>(dev + o_poll);
        hwords = reinterpret_cast<uint32_t *>(p0->hsmall);
        static_assert(2 * kGroupWords * sizeof(uint32_t) <= 128 * sizeof(double), "poll words");

        gpmax = 4;
        for (int i = 0; i < G; ++i) {
            qp_problem *p = probs[i];
            const qp::Parts parts = p->parts();
            qp::GroupEntry &e = ents[i];
            e = qp::GroupEntry{};
            e.tab = p->tab;
            e.recs = p->recs();
            e.urec32 = p->urec(qp::F32);
            e.upku32 = p->upku(qp::F32);
            e.urec64 = p->urec(qp::F64);
            e.upku64 = p->upku(qp::F64);
            e.x32 = p->x32();
            e.r32 = p->r32();
            e.h32 = p->h32();
            e.q32 = p->q32();
            e.M32 = p->M32();
            e.X = p->chi(0);
            e.F = p->F();
            e.pa = parts.a;
            e.pb = parts.b;
            e.st = p->st();
            e.nb_mv = p->host.nb_mv;
            e.nb_mv64 = p->host.nb_mv64;
            e.nb_st = p->host.nblocks;
            e.wide = p->host.chunk > 4 * qp::kBlock ? 1 : 0;
            gpmax = std::max(gpmax, (p->host.g + 3) & ~3);
        }
        running.assign(G, 1);
        QP_TRY(build_owners());

        // set-up of every problem (the launches of a standalone homogenization)
        QP_HIP(hipEventRecord(p0->ev_t0, s));
        for (int i = 0; i < G; ++i) {
            qp_problem *p = probs[i];
            const qp::Parts parts = p->parts();
            QP_HIP(qp::launch_corrector_rhs_all(p->tab, p->host, d, p->F(), &parts, s));
            QP_HIP(qp::launch_state_reset(K, p->st(), s));
            QP_HIP(qp::launch_ir_unit_only(K, p->host, parts, p->st(), s));
            QP_HIP(qp::launch_pcg_init(qp::F32, K, p->tab, p->host, p->F(), p->chi(0), p->x32(),
                                       p->r32(), p->h32(), p->M32(), parts, p->st(), s));
            QP_HIP(qp::launch_pcg_start(qp::F32, K, p->host, tol, p->opt.inner_tol, p->opt.maxit,
                                        parts, p->st(), s));
        }
        maxit = p0->opt.maxit;
        full = batch_size(p0->opt);
        j = slot = inflight = 0;
        fin = finished = false;
        worst = QP_OK;
        return QP_OK;
    }

    // Two chunks of iterations in flight: the device runs one while the host
    // inspects the poll of the other.  A non-blocking call returns when the
    // poll it needs has not arrived.
    qp_status advance(bool blocking, bool &progressed)
    {
        progressed = false;
        if (finished) return QP_OK;
        if (!fin) {
            while (inflight < 2 && j < maxit) {
                QP_TRY(queue());
                progressed = true;
            }
            if (inflight > 0) {
                const int oldest = (inflight == 2) ? slot : (slot ^ 1);
                const hipEvent_t ev = probs[0]->ev_poll[oldest];
                if (blocking) {
                    QP_HIP(hipEventSynchronize(ev));
                } else {
                    const hipError_t q = hipEventQuery(ev);
                    if (q == hipErrorNotReady) return QP_OK;
                    QP_HIP(q);
                }
                progressed = true;
                --inflight;
                bool all = true;
                for (int i = 0; i < G && all; ++i) all = problem_done(oldest, i);
                if (!all) return compact(oldest);
                fin = true;
            }
            // else: the iteration limit, nothing in flight, not every problem done
        }
        progressed = true;
        return finish();
    }

  private:
    // owners of the running problems' workgroups, uploaded with the entries
    qp_status build_owners()
    {
        n_mv = n_mv64 = n_st = 0;
        for (int i = 0; i < G; ++i) {
            if (!running[i]) continue;
            qp::GroupEntry &e = ents[i];
            e.mv0 = n_mv;
            e.mv064 = n_mv64;
            e.sv0 = n_st;
            for (int w = 0; w < e.nb_mv; ++w) own_mv[n_mv++] = i;
            for (int w = 0; w < e.nb_mv64; ++w) own_mv64[n_mv64++] = i;
            for (int w = 0; w < e.nb_st; ++w) own_st[n_st++] = i;
        }
        QP_HIP(hipMemcpy(E, ents, sizeof(qp::GroupEntry) * G, hipMemcpyHostToDevice));
        QP_HIP(hipMemcpy(owner_mv, own_mv, sizeof(int) * n_mv, hipMemcpyHostToDevice));
        QP_HIP(hipMemcpy(owner_mv64, own_mv64, sizeof(int) * n_mv64, hipMemcpyHostToDevice));
        QP_HIP(hipMemcpy(owner_st, own_st, sizeof(int) * n_st, hipMemcpyHostToDevice));
        return QP_OK;
    }

    qp_status replacement(int it)
    {
        QP_HIP(qp::launch_group_vec(2, it, K, n_st, E, owner_st, s));
        QP_HIP(qp::launch_group_matvec(qp::F64, d, probs[0]->host.real_coef, n_mv64, gpmax, E,
                                       owner_mv64, s));
        QP_HIP(qp::launch_group_vec(3, it, K, n_st, E, owner_st, s));
        return QP_OK;
    }

    qp_status poll(int sl, hipEvent_t ev)
    {
        if (noalloc) {
            QP_HIP(qp::launch_group_done(G, K, E, dwords + sl * kGroupWords, s));
            QP_HIP(hipMemcpyAsync(hwords + sl * kGroupWords, dwords + sl * kGroupWords,
                                  sizeof(uint32_t) * kGroupWords, hipMemcpyDeviceToHost, s));
        } else {
            QP_HIP(qp::launch_group_states(G, K, E, dstates + sl * nst, s));
            QP_HIP(hipMemcpyAsync(g_gb.host + sl * nst, dstates + sl * nst, nst * sizeof(State),
                                  hipMemcpyDeviceToHost, s));
        }
        if (ev) QP_HIP(hipEventRecord(ev, s));
        return QP_OK;
    }

    // whether every right-hand side of problem i was done at the poll of slot sl
    bool problem_done(int sl, int i) const
    {
        if (noalloc) return (hwords[sl * kGroupWords + i / 32] >> (i % 32)) & 1u;
        bool dn = true;
        for (int r = 0; r < K; ++r) dn = dn && g_gb.host[sl * nst + (size_t)i * K + r].done != 0;
        return dn;
    }

    // Launches cover only the problems still running: once a poll shows
    // problems finished, the owner tables are rebuilt without them (after the
    // queued work has drained; a finished problem's state no longer changes).
    qp_status compact(int seen)
    {
        bool changed = false, any = false;
        for (int i = 0; i < G; ++i) {
            if (running[i] && problem_done(seen, i)) {
                running[i] = 0;
                changed = true;
            }
            any = any || running[i];
        }
        if (!changed || !any) return QP_OK;
        QP_HIP(hipStreamSynchronize(s));
        return build_owners();
    }

    qp_status queue()
    {
        const int k = std::min(full, maxit - j);
        for (int it = 0; it < k; ++it) {
            QP_HIP(qp::launch_group_matvec(qp::F32, d, probs[0]->host.real_coef, n_mv, gpmax, E,
                                           owner_mv, s));
            QP_HIP(qp::launch_group_vec(0, it, K, n_st, E, owner_st, s));
            QP_HIP(qp::launch_group_vec(1, it, K, n_st, E, owner_st, s));
            if (it & 1) QP_TRY(replacement(it));
        }
        QP_TRY(poll(slot, probs[0]->ev_poll[slot]));
        j += k;
        slot ^= 1;
        ++inflight;
        return QP_OK;
    }

    qp_status finish()
    {
        finished = true;
        qp_problem *p0 = probs[0];
        if (!fin) {
            // iteration limit: fold every unfinished increment into X with one
            // forced replacement, whose true residual decides the status
            for (int i = 0; i < G; ++i) QP_HIP(qp::launch_ir_force(K, probs[i]->st(), s));
            QP_TRY(replacement(maxit));
        }
        QP_HIP(hipEventRecord(p0->ev_t1, s));
        for (int i = 0; i < G; ++i) {
            qp_problem *p = probs[i];
            // final states into the problem's own pinned slot 2
            QP_HIP(hipMemcpyAsync(p->hstate + 2 * qp::kMaxRhs, p->st(), sizeof(State) * K,
                                  hipMemcpyDeviceToHost, s));
            QP_HIP(qp::launch_astar(p->tab, p->host, p->chi(0), p->small(), s));
            QP_HIP(hipMemcpyAsync(p->hsmall, p->small(), 128 * sizeof(double), hipMemcpyDeviceToHost,
                                  s));
            if (infos) QP_TRY(queue_hist(p, K, s));
        }
        QP_HIP(hipStreamSynchronize(s));
        lock = std::unique_lock<std::mutex>();  // the group buffers are free again
        float ms = 0.f;
        QP_HIP(hipEventElapsedTime(&ms, p0->ev_t0, p0->ev_t1));
        worst = QP_OK;
        size_t ao = 0;
        for (int i = 0; i < G; ++i) {
            qp_problem *p = probs[i];
            const State *fs = p->hstate + 2 * qp::kMaxRhs;
            for (int e = 0; e < d * d; ++e) Astar[ao + e] = p->hsmall[e];
            ao += (size_t)d * d;
            for (int r = 0; r < K; ++r) {
                const State &st = fs[r];
                const qp_status status = st.done ? (qp_status)st.status : QP_ENOCONV;
                if (infos) {
                    qp_solve_info *info = infos + (size_t)i * K + r;
                    std::memset(info, 0, sizeof(*info));
                    info->flags = p->flags;
                    info->status = status;
                    info->iters = st.iters;
                    info->outer_iters = st.replacements;
                    info->rel_resid = std::sqrt(st.rr);
                    info->seconds = ms * 1e-3;
                    info->kappa_est = lanczos_kappa(p->hhist + (size_t)2 * qp::kHist * r,
                                                    std::min(st.iters, qp::kHist));
                    info->bytes_moved = solve_bytes(true, (double)p->host.D, st.iters, st.replacements);
                }
                if (status != QP_OK && worst == QP_OK) worst = status;
            }
        }
        if (worst != QP_OK) {
            report(worst);
            fail(worst, "a corrector solve of the group did not converge");
        }
        return QP_OK;
    }
};

qp_status grouped_run(qp_problem *const *problems, int count, double *Astar, double tol,
                      qp_solve_info *infos, bool noalloc)
{
    GroupJob job;
    QP_TRY(job.begin(problems, count, Astar, tol, infos, noalloc));
    bool progressed = false;
    while (!job.done()) QP_TRY(job.advance(true, progressed));
    return job.worst;
}

}  // namespace
extern "C" {

qp_status qp_homogenized_grouped(qp_problem *const *problems, int count, double *Astar, double tol,
                                 qp_solve_info *infos)
{
    return grouped_run(problems, count, Astar, tol, infos, false);
}

qp_status qp_homogenized_grouped_noalloc(qp_problem *const *problems, int count, double *Astar,
                                         double tol, qp_solve_info *infos)
{
    return grouped_run(problems, count, Astar, tol, infos, true);
}

qp_status qp_homogenized_batch_mixed(qp_problem *const *problems, int count, double *Astar,
                                     double tol, qp_solve_info *infos, int64_t group_max_dim)
{
    if (!problems || !Astar || count < 1) return fail(QP_EINVAL, "null argument or empty batch");
    if (group_max_dim < 0) return fail(QP_EINVAL, "group_max_dim must not be negative");
    for (int i = 0; i < count; ++i) {
        if (!problems[i]) return fail(QP_EINVAL, "problem %d is null", i);
        for (int k = 0; k < i; ++k)
            if (problems[k] == problems[i]) return fail(QP_EINVAL, "problem %d repeats problem %d", i, k);
    }
    // the group: the small problems that can join one led by the first of them
    std::vector<int> member;
    int lead = -1;
    for (int i = 0; i < count && (int)member.size() < kMaxGroup; ++i) {
        qp_problem *p = problems[i];
        if ((int64_t)p->host.D > group_max_dim) continue;
        if (lead < 0) {
            if (group_mismatch(p, p)) continue;
            lead = i;
        } else if (group_mismatch(p, problems[lead])) {
            continue;
        }
        member.push_back(i);
    }
    if (member.size() < 2) return qp_homogenized_batch(problems, count, Astar, tol, infos);
    std::vector<char> grouped(count, 0);
    for (int i : member) grouped[i] = 1;
    // offsets of every problem's A* and infos in the caller's arrays
    std::vector<size_t> ao(count), io(count);
    for (int i = 0, a = 0, b = 0; i < count; ++i) {
        ao[i] = a;
        io[i] = b;
        a += problems[i]->host.d * problems[i]->host.d;
        b += problems[i]->host.d;
    }
    const int d = problems[lead]->host.d;
    std::vector<qp_problem *> gp;
    for (int i : member) gp.push_back(problems[i]);
    std::vector<double> gA(member.size() * d * d);
    std::vector<qp_solve_info> gI(member.size() * d);

    GroupJob group;
    QP_TRY(group.begin(gp.data(), (int)gp.size(), gA.data(), tol, gI.data(), false));
    std::vector<HomJob> jobs(count);
    for (int i = 0; i < count; ++i) {
        if (grouped[i]) continue;
        QP_TRY(jobs[i].begin(problems[i], Astar + ao[i], nullptr, tol, infos ? infos + io[i] : nullptr));
    }
    // round robin over the group and the other problems' jobs
    auto drain = [&]() {
        for (int i = 0; i < count; ++i) (void)hipStreamSynchronize(problems[i]->stream);
    };
    for (;;) {
        bool all = true, any = false;
        for (int i = 0; i < count; ++i) {
            if (grouped[i] || jobs[i].done()) continue;
            bool pr = false;
            const qp_status st = jobs[i].advance(false, pr);
            if (st != QP_OK) {
                drain();
                return st;
            }
            any = any || pr;
            all = all && jobs[i].done();
        }
        if (!group.done()) {
            bool pr = false;
            const qp_status st = group.advance(false, pr);
            if (st != QP_OK) {
                drain();
                return st;
            }
            any = any || pr;
            all = all && group.done();
        }
        if (all) break;
        if (!any) std::this_thread::yield();
    }
    for (size_t m = 0; m < member.size(); ++m) {
        const int i = member[m];
        for (int e = 0; e < d * d; ++e) Astar[ao[i] + e] = gA[m * d * d + e];
        if (infos)
            for (int r = 0; r < d; ++r) infos[io[i] + r] = gI[m * d + r];
    }
    // the first non-QP_OK status in problem order
    qp_status worst = QP_OK;
    for (int i = 0; i < count && worst == QP_OK; ++i) {
        if (!grouped[i]) {
            worst = jobs[i].worst;
            continue;
        }
        for (size_t m = 0; m < member.size(); ++m)
            if (member[m] == i)
                for (int r = 0; r < d && worst == QP_OK; ++r) {
                    const qp_status st = (qp_status)gI[m * d + r].status;
                    if (st != QP_OK) worst = st;
                }
    }
    if (worst != QP_OK) fail(worst, "a corrector solve of the batch did not converge");
    return worst;
}

qp_status qp_homogenized(qp_problem *p, double *Astar, double tol, qp_solve_info *info)
{
    return qp_homogenized_ex(p, Astar, nullptr, tol, info);
}

}  // extern "C"

// One product of the single-product entry points; with the profile option on,
// the launch records an event pair around its kernel and the duration is kept
// for qp_last_product_ms.
static qp_status single_product(qp_problem *p, int prec, const void *u, void *y)
{
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    p->last_product_ms = -1.0;
    if (p->opt.profile) {
        QP_TRY(events_ready(p));
        ev0 = p->ev_hot[0];
        ev1 = p->ev_hot[1];
    }
    QP_HIP(qp::launch_matvec(prec, qp::EPI_NONE, 1, p->tab, p->host, p->recs(), p->urec(prec),
                             p->upku(prec), u, y, nullptr, nullptr, p->parts(), p->st(), nullptr,
                             p->stream, ev0, ev1));
    QP_HIP(hipStreamSynchronize(p->stream));
    if (ev0) {
        float ms = 0.f;
        QP_HIP(hipEventElapsedTime(&ms, ev0, ev1));
        p->last_product_ms = ms;
    }
    return QP_OK;
}

extern "C" {

qp_status qp_matvec_d(qp_problem *p, const double *u, double *y)
{
    if (!p || !u || !y) return fail(QP_EINVAL, "null argument");
    if (overlaps(u, y, 16 * (size_t)p->host.D)) return fail(QP_EINVAL, "u and y must not overlap");
    return single_product(p, qp::F64, u, y);
}

qp_status qp_last_product_ms(const qp_problem *p, double *ms)
{
    if (!p || !ms) return fail(QP_EINVAL, "null argument");
    *ms = p->last_product_ms;
    return QP_OK;
}

qp_status qp_matvec_half_d(qp_problem *p, const double *u, double *y)
{
    if (!p || !u || !y) return fail(QP_EINVAL, "null argument");
    if (p->host.half) return qp_matvec_d(p, u, y);  // its vectors are the half already
    if (p->host.N % 2 == 0)
        return fail(QP_EINVAL, "Hermitian half storage needs odd N (N = %d)", p->host.N);
    if (p->host.aniso)
        return fail(QP_EINVAL, "Hermitian half storage: scalar coefficient only");
    if (overlaps(u, y, 16 * (((size_t)p->host.D + 1) / 2)))
        return fail(QP_EINVAL, "u and y must not overlap");
    QP_HIP(qp::launch_matvec_half(p->tab, p->host, u, y, p->stream));
    QP_HIP(hipStreamSynchronize(p->stream));
    return QP_OK;
}

qp_status qp_matvec32_d(qp_problem *p, const float *u, float *y)
{
    if (!p || !u || !y) return fail(QP_EINVAL, "null argument");
    if (overlaps(u, y, 8 * (size_t)p->host.D)) return fail(QP_EINVAL, "u and y must not overlap");
    return single_product(p, qp::F32, u, y);
}

qp_status qp_dft_d(int n, int N, const double *in, double *out, int inverse, void *stream)
{
    if (!in || !out) return fail(QP_EINVAL, "null argument");
    if (n < 1 || n > QP_MAX_DIM_N || N < 1 || N > 1024)
        return fail(QP_EINVAL, "n=%d or N=%d outside [1, %d] x [1, 1024]", n, N, QP_MAX_DIM_N);
    int64_t D = 1;
    for (int t = 0; t < n; ++t) {
        D *= N;
        if (D >= ((int64_t)1 << 31)) return fail(QP_EINVAL, "N^n exceeds 2^31 - 1");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    QP_HIP(qp::launch_dft(n, N, in, out, inverse ? 1 : 0, s));
    QP_HIP(hipStreamSynchronize(s));
    return QP_OK;
}

qp_status qp_modes_from_spectrum(int n, int N, const double *spec, double rel_tol, int max_modes,
                                 int32_t *modes, double *coef, int *g)
{
    if (!spec || !modes || !coef || !g) return fail(QP_EINVAL, "null argument");
    *g = 0;
    if (n < 1 || n > QP_MAX_DIM_N || N < 2) return fail(QP_EINVAL, "n=%d or N=%d out of range", n, N);
    if (!(rel_tol >= 0.0) || !(rel_tol < 1.0)) return fail(QP_EINVAL, "rel_tol must be in [0, 1)");
    if (max_modes < 1) return fail(QP_EINVAL, "max_modes < 1");
    int64_t D = 1;
    for (int t = 0; t < n; ++t) {
        D *= N;
        if (D >= ((int64_t)1 << 31)) return fail(QP_EINVAL, "N^n exceeds 2^31 - 1");
    }
    double amax = 0.0;
    for (int64_t i = 0; i < D; ++i) amax = std::max(amax, std::hypot(spec[2 * i], spec[2 * i + 1]));
    if (!(amax > 0.0) || !std::isfinite(amax)) return fail(QP_EINVAL, "spectrum is zero or not finite");
    const double cut = rel_tol * amax;
    // storage index of -k (digit b -> (N - b) mod N per axis)
    auto neg = [&](int64_t i) {
        int64_t r = 0, m = 1, rest = i;
        for (int t = 0; t < n; ++t) {
            const int64_t b = rest % N;
            rest /= N;
            r += ((N - b) % N) * m;
            m *= N;
        }
        return r;
    };
    std::vector<int64_t> keep;
    for (int64_t i = 0; i < D; ++i) {
        const double a = std::max(std::hypot(spec[2 * i], spec[2 * i + 1]),
                                  std::hypot(spec[2 * neg(i)], spec[2 * neg(i) + 1]));
        if (a > cut || i == 0) keep.push_back(i);  // a mode and its partner together
    }
    if ((int64_t)keep.size() > max_modes)
        return fail(QP_EINVAL, "%lld modes exceed rel_tol, more than max_modes = %d",
                    (long long)keep.size(), max_modes);
    int k = 0;
    for (const int64_t i : keep) {
        int64_t rest = i;
        for (int t = n - 1; t >= 0; --t) {
            const int b = (int)(rest % N);
            rest /= N;
            if (2 * b == N)
                return fail(QP_EINVAL, "a retained mode lies on the N/2 face (would alias)");
            modes[k * n + t] = (2 * b < N) ? b : b - N;
        }
        // Hermitian part: the coefficients of a real field satisfy
        // Ahat_{-m} = conj(Ahat_m); keep their average
        const int64_t j = neg(i);
        coef[2 * k] = 0.5 * (spec[2 * i] + spec[2 * j]);
        coef[2 * k + 1] = 0.5 * (spec[2 * i + 1] - spec[2 * j + 1]);
        ++k;
    }
    *g = k;
    return QP_OK;
}

int64_t qp_coo_entries(const qp_problem *p)
{
    return (p && !p->host.half) ? (int64_t)p->host.D * p->host.g : 0;
}

qp_status qp_coo_build_d(qp_problem *p, int32_t *rows, int32_t *cols, double *vals)
{
    if (!p || !rows || !cols || !vals) return fail(QP_EINVAL, "null argument");
    if (p->host.half) return fail(QP_EINVAL, "the stored matrix is built on full storage");
    QP_HIP(qp::launch_coo_build(p->tab, p->host, rows, cols, vals, p->stream));
    QP_HIP(hipStreamSynchronize(p->stream));
    return QP_OK;
}

qp_status qp_coo_matvec_d(qp_problem *p, const int32_t *cols, const double *vals, const double *u,
                          double *y)
{
    if (!p || !cols || !vals || !u || !y) return fail(QP_EINVAL, "null argument");
    if (p->host.half) return fail(QP_EINVAL, "the stored matrix is built on full storage");
    if (overlaps(u, y, 16 * (size_t)p->host.D)) return fail(QP_EINVAL, "u and y must not overlap");
    QP_HIP(qp::launch_coo_matvec(p->host, cols, vals, u, y, p->stream));
    QP_HIP(hipStreamSynchronize(p->stream));
    return QP_OK;
}

qp_status qp_precond_d(qp_problem *p, double *M)
{
    if (!p || !M) return fail(QP_EINVAL, "null argument");
    QP_HIP(hipMemcpyAsync(M, p->M64(), 8 * (size_t)p->host.D, hipMemcpyDeviceToDevice, p->stream));
    QP_HIP(hipStreamSynchronize(p->stream));
    return QP_OK;
}

qp_status qp_corrector_rhs_d(qp_problem *p, int j, double *F)
{
    if (!p || !F) return fail(QP_EINVAL, "null argument");
    if (j < 0 || j >= p->host.d) return fail(QP_EINVAL, "corrector index %d outside [0, d)", j);
    QP_HIP(qp::launch_corrector_rhs(p->tab, p->host, j, F, p->stream));
    QP_HIP(hipStreamSynchronize(p->stream));
    return QP_OK;
}

qp_status qp_multi_index_d(qp_problem *p, int32_t *k)
{
    if (!p || !k) return fail(QP_EINVAL, "null argument");
    QP_HIP(qp::launch_multi_index(p->tab, p->host, k, p->stream));
    QP_HIP(hipStreamSynchronize(p->stream));
    return QP_OK;
}

qp_status qp_astar_d(qp_problem *p, const double *chi, double *Astar)
{
    if (!p || !chi || !Astar) return fail(QP_EINVAL, "null argument");
    QP_HIP(qp::launch_astar(p->tab, p->host, chi, p->small(), p->stream));
    QP_HIP(hipMemcpyAsync(p->hsmall, p->small(), 32 * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    QP_HIP(hipStreamSynchronize(p->stream));
    const int d = p->host.d;
    for (int e = 0; e < d * d; ++e) Astar[e] = p->hsmall[e];
    return QP_OK;
}

qp_status qp_coef_extrema(qp_problem *p, double *amin, double *amax)
{
    if (!p) return fail(QP_EINVAL, "null problem");
    if (amin) *amin = p->amin;
    if (amax) *amax = p->amax;
    return QP_OK;
}

qp_status qp_synchronize(qp_problem *p)
{
    if (!p) return fail(QP_EINVAL, "null problem");
    QP_HIP(hipStreamSynchronize(p->stream));
    return QP_OK;
}

const char *qp_strerror(qp_status s)
{
    switch (s) {
    case QP_OK: return "success";
    case QP_EINVAL: return "invalid argument";
    case QP_ENOTELLIPTIC: return "coefficient is negative on the collocation grid";
    case QP_ENOTSPD: return "PCG breakdown: the operator is not positive definite";
    case QP_ENOCONV: return "iteration limit reached";
    case QP_ENOMEM: return "out of memory";
    case QP_EDEVICE: return "HIP device error";
    case QP_ENONFINITE: return "non-finite value";
    }
    return "unknown status";
}

const char *qp_last_error(void) { return g_last_error.c_str(); }

// ---------------------------------------------------------------- serving

qp_status qp_server_create(qp_server **out, size_t hbm_budget, const qp_options *opt)
{
    g_last_error.clear();
    if (!out) return fail(QP_EINVAL, "out is null");
    *out = nullptr;
    if (hbm_budget == 0) return fail(QP_EINVAL, "hbm_budget is 0");
    qp_options o;
    qp_default_options(&o);
    if (opt) o = *opt;
    QP_TRY(check_options(&o));
    if (o.half_storage)
        return fail(QP_EINVAL, "the server's problems use full storage (half_storage must be 0)");
    o.stream = nullptr;     // every cached problem gets a stream of its own
    o.workspace = nullptr;  // and a workspace of its own
    o.workspace_bytes = 0;
    qp_server *s = new (std::nothrow) qp_server();
    if (!s) return fail(QP_ENOMEM, "host allocation failed");
    s->budget = hbm_budget;
    s->opt = o;
    *out = s;
    return QP_OK;
}

qp_status qp_server_submit(qp_server *s, int d, int n, const double *P, int g,
                           const int32_t *modes, const double *coef, const double *coefs, int N,
                           double tol, double *Astar, qp_solve_info *infos, int64_t *ticket)
{
    if (!s || !Astar || !ticket) return fail(QP_EINVAL, "null argument");
    *ticket = 0;
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(QP_EINVAL, "tol must be positive and finite");
    if (coefs) {
        if (d < 1 || d > QP_MAX_DIM_D) return fail(QP_EINVAL, "d=%d outside [1, %d]", d, QP_MAX_DIM_D);
        for (int l = 0; l < d; ++l) QP_TRY(check_args(d, n, P, g, modes, coefs + 2 * (size_t)l * g, N));
    } else {
        QP_TRY(check_args(d, n, P, g, modes, coef, N));
    }
    const size_t bytes = qp_workspace_bytes(d, n, N, g);
    if (bytes == 0) return fail(QP_EINVAL, "unsupported shape");
    if (bytes > s->budget)
        return fail(QP_ENOMEM, "the problem needs %zu bytes, more than the budget of %zu", bytes,
                    s->budget);
    qp_server::Request R;
    R.d = d;
    R.n = n;
    R.N = N;
    R.g = g;
    R.diag = coefs != nullptr;
    R.P.assign(P, P + (size_t)d * n);
    R.modes.assign(modes, modes + (size_t)g * n);
    const double *c = coefs ? coefs : coef;
    R.coef.assign(c, c + 2 * (size_t)g * (coefs ? d : 1));
    R.tol = tol;
    R.Astar = Astar;
    R.infos = infos;
    R.bytes = bytes;
    // cache key: the full description (the options are the server's)
    std::string key;
    auto put = [&key](const void *v, size_t nb) { key.append(static_cast<const char *>(v), nb); };
    const int head[5] = {d, n, N, g, R.diag ? 1 : 0};
    put(head, sizeof(head));
    put(R.P.data(), R.P.size() * sizeof(double));
    put(R.modes.data(), R.modes.size() * sizeof(int32_t));
    put(R.coef.data(), R.coef.size() * sizeof(double));
    R.key = std::move(key);
    R.ticket = s->next_ticket++;
    *ticket = R.ticket;
    s->queue.push_back(std::move(R));
    return QP_OK;
}

}  // extern "C"

namespace {

// Admit queued requests in arrival order.  A request whose problem would
// have to be created but does not fit stops the creation of problems for
// the requests behind it (they may still run on cached idle problems).
qp_status server_admit(qp_server *s)
{
    bool create_ok = true;
    for (size_t qi = 0; qi < s->queue.size();) {
        qp_server::Request &R = s->queue[qi];
        size_t e = s->cache.size();
        for (size_t c = 0; c < s->cache.size(); ++c)
            if (s->cache[c].key == R.key) e = c;
        if (e < s->cache.size() && s->cache[e].busy) {
            ++qi;
            continue;
        }
        if (e == s->cache.size()) {
            if (!create_ok) {
                ++qi;
                continue;
            }
            // evict idle problems, least recently used first, until it fits
            while (s->used + R.bytes > s->budget) {
                size_t victim = s->cache.size();
                for (size_t c = 0; c < s->cache.size(); ++c)
                    if (!s->cache[c].busy &&
                        (victim == s->cache.size() || s->cache[c].last_use < s->cache[victim].last_use))
                        victim = c;
                if (victim == s->cache.size()) break;
                qp_destroy(s->cache[victim].p);
                s->used -= s->cache[victim].bytes;
                s->cache.erase(s->cache.begin() + victim);
                // running jobs refer to cache slots by index
                for (auto &run : s->running)
                    if (run->entry > victim) --run->entry;
            }
            if (s->used + R.bytes > s->budget) {
                create_ok = false;
                ++qi;
                continue;
            }
            qp_problem *p = nullptr;
            const qp_status cs =
                create_problem(&p, R.d, R.n, R.P.data(), R.g, R.modes.data(),
                               R.diag ? nullptr : R.coef.data(), R.diag ? R.coef.data() : nullptr,
                               R.N, &s->opt);
            if (cs != QP_OK) {
                s->finished.push_back({R.ticket, cs});
                s->queue.erase(s->queue.begin() + qi);
                continue;
            }
            qp_server::Entry E;
            E.key = R.key;
            E.p = p;
            E.bytes = R.bytes;
            s->cache.push_back(std::move(E));
            s->used += R.bytes;
            e = s->cache.size() - 1;
        }
        qp_server::Entry &E = s->cache[e];
        auto run = std::make_unique<qp_server::Running>();
        run->ticket = R.ticket;
        run->entry = e;
        const qp_status bs = run->job.begin(E.p, R.Astar, nullptr, R.tol, R.infos);
        if (bs != QP_OK) {
            s->finished.push_back({R.ticket, bs});
        } else {
            E.busy = true;
            E.last_use = ++s->clock;
            s->running.push_back(std::move(run));
        }
        s->queue.erase(s->queue.begin() + qi);
    }
    return QP_OK;
}

}  // namespace
extern "C" {

qp_status qp_server_progress(qp_server *s, int wait_us, int64_t *done, qp_status *done_status,
                             int max_done, int *ndone)
{
    if (!s || !ndone || (max_done > 0 && !done)) return fail(QP_EINVAL, "null argument");
    *ndone = 0;
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        QP_TRY(server_admit(s));
        bool any = false;
        for (size_t i = 0; i < s->running.size();) {
            qp_server::Running &run = *s->running[i];
            bool pr = false;
            const qp_status st = run.job.advance(false, pr);
            any = any || pr;
            if (st != QP_OK || run.job.done()) {
                s->finished.push_back({run.ticket, st != QP_OK ? st : run.job.worst});
                qp_server::Entry &E = s->cache[run.entry];
                E.busy = false;
                E.last_use = ++s->clock;
                s->running.erase(s->running.begin() + i);
                any = true;
                continue;
            }
            ++i;
        }
        if (!s->finished.empty() || (s->running.empty() && s->queue.empty())) break;
        const auto us = std::chrono::duration_cast<std::chrono::microseconds>(
                            std::chrono::steady_clock::now() - t0).count();
        if (us >= wait_us) break;
        if (!any) std::this_thread::yield();
    }
    int k = 0;
    while (k < max_done && !s->finished.empty()) {
        done[k] = s->finished.front().ticket;
        if (done_status) done_status[k] = s->finished.front().status;
        s->finished.erase(s->finished.begin());
        ++k;
    }
    *ndone = k;
    return QP_OK;
}

int qp_server_pending(const qp_server *s)
{
    if (!s) return 0;
    return (int)(s->queue.size() + s->running.size() + s->finished.size());
}

size_t qp_server_bytes(const qp_server *s) { return s ? s->used : 0; }

void qp_server_destroy(qp_server *s)
{
    if (!s) return;
    for (auto &run : s->running) {
        bool pr = false;
        while (!run->job.done())
            if (run->job.advance(true, pr) != QP_OK) break;
    }
    for (auto &E : s->cache) qp_destroy(E.p);
    delete s;
}

}  // extern "C"
