// Host side of the C ABI declared in include/qp.h: argument validation, the
// device workspace, and the drivers that queue C-PCG (Alg. 2) and its FP32
// refinement variant on one HIP stream.  The host never computes a Krylov
// scalar: it queues batches of iterations and polls the device's `done` flag.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
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
    size_t F, U, r, h, q, M64, M32, x32, r32, h32, q32, chi, parts, states, small, exec, tab, recs;
    size_t urec[2], upku[2];  // unit records and unit P k, by precision (plane tiles)
    size_t total;
};

Layout make_layout(int d, int n, int N, int64_t D, int g)
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
    L.small = take(sizeof(double) * 128);
    L.exec = take(sizeof(int) * kExecInts);
    L.tab = take(sizeof(Table));
    L.recs = take(sizeof(qp::ModeRec) * qp::kMaxG);
    const size_t urecs = (size_t)plane_units(n, N) * (size_t)((g + 3) & ~3);
    for (int prec = 0; prec < 2; ++prec) {
        L.urec[prec] = take(qp::kUnitRecBytes[prec] * urecs);
        L.upku[prec] = take((prec == qp::F64 ? 8 : 4) * (size_t)qp::kMaxD * plane_units(n, N));
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
    State *hstate = nullptr;   // pinned: two polling slots + final, kMaxRhs states each
    double *hsmall = nullptr;  // pinned
    int *hexec = nullptr;      // pinned copy of the execution log
    std::vector<hipEvent_t> ev_hot, ev_res;  // profiling events (begin, end pairs)
    struct Graph {
        bool ir;
        int K, k, ab;
        bool prof;
        const void *u, *f;  // solution and right-hand side the graph was captured on
        hipGraphExec_t exec;
    };
    std::vector<Graph> graphs;
    hipEvent_t ev_poll[2] = {nullptr, nullptr};
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
    const int64_t units = T.ntiles / T.tiles_per_unit;
    const int64_t items = T.tile_s > 1
                              ? units * ((T.tiles_per_unit + T.item_tiles - 1) / T.item_tiles)
                              : units * ((T.tiles_per_unit + 3) / 4);
    const int64_t want = T.tile_s > 1 ? (items + 3) / 4 : items;
    int nbm = (int)std::min<int64_t>(qp::kMaxBlocks, std::max<int64_t>(1, want));
    if (nbm >= 8) nbm -= nbm % 8;
    T.nb_mv = nbm;
    int nb = (int)std::min<int64_t>(qp::kStreamBlocks, (D + qp::kBlock - 1) / qp::kBlock);
    if (nb >= 64) nb -= nb % 8;
    int64_t chunk = (D + nb - 1) / nb;
    chunk = (chunk + qp::kBlock - 1) / qp::kBlock * qp::kBlock;
    T.chunk = (int)chunk;
    T.nblocks = (int)((D + chunk - 1) / chunk);
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
    if (p->ev_t0) (void)hipEventDestroy(p->ev_t0);
    if (p->ev_t1) (void)hipEventDestroy(p->ev_t1);
    if (p->hstate) (void)hipHostFree(p->hstate);
    if (p->hsmall) (void)hipHostFree(p->hsmall);
    if (p->hexec) (void)hipHostFree(p->hexec);
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
    int b = o.poll_every > 0 ? o.poll_every : 8;
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
    if (slot >= 0) {
        exec = (resid ? p->exec_res() : p->exec_hot()) + slot;
        QP_HIP(hipEventRecord(pool[2 * slot], p->stream));
    }
    QP_HIP(qp::launch_matvec(prec, epi, K, p->tab, p->host, p->recs(), p->urec(prec),
                             p->upku(prec), x, y, f, p->M32(), p->parts(), p->st(), exec,
                             p->stream));
    if (slot >= 0) QP_HIP(hipEventRecord(pool[2 * slot + 1], p->stream));
    return QP_OK;
}

// k FP64 iterations (it = 0 .. k-1) of K right-hand sides on U.
qp_status enqueue_fp64(qp_problem *p, int K, double *U, int k, int ab, bool prof)
{
    const qp::Parts parts = p->parts();
    for (int it = 0; it < k; ++it) {
        QP_TRY(queue_matvec(p, qp::F64, qp::EPI_ALPHA, K, p->h(), p->q(), nullptr,
                            prof ? ab * kMaxBatch + it : -1));
        QP_HIP(qp::launch_pcg_update(qp::F64, it, K, p->tab, p->host, U, p->r(), p->h(), p->q(),
                                     p->M64(), parts, p->st(), p->stream));
        QP_HIP(qp::launch_pcg_direction(qp::F64, it, K, p->tab, p->host, p->r(), p->h(), p->M64(),
                                        parts, p->st(), p->stream));
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
        QP_HIP(qp::launch_pcg_update(qp::F32, it, K, p->tab, p->host, p->x32(), p->r32(), p->h32(),
                                     p->q32(), p->M32(), parts, p->st(), p->stream));
        QP_HIP(qp::launch_pcg_direction(qp::F32, it, K, p->tab, p->host, p->r32(), p->h32(),
                                        p->M32(), parts, p->st(), p->stream));
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

// Double-buffered polling: after each batch the K states (and, when
// profiling, the batch's execution log) are copied to pinned memory; the
// batch before the newest is inspected, so the device always has queued work.
// Kernels of a finished right-hand side skip it.
struct Poller {
    qp_problem *p;
    int K;
    bool prof;
    Profile &pf;
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
            pf.hot_ms += t;
            ++pf.hot_n;
            pf.hot_rhs += hot[it];
        }
        const int res = p->hexec[2 * kMaxBatch + s];
        if (rec[s].nres && res) {
            float t = 0.f;
            QP_HIP(hipEventElapsedTime(&t, p->ev_res[2 * s], p->ev_res[2 * s + 1]));
            pf.res_ms += t;
            ++pf.res_n;
            pf.res_rhs += res;
        }
        return QP_OK;
    }
    // Record the poll point of the batch just queued (k stiffness products,
    // nres residual replacements); finished = an older poll saw every state
    // done; seen = the states that poll saw (null when there was none yet).
    qp_status push(int k, int nres, bool &finished, const State **seen)
    {
        finished = false;
        *seen = nullptr;
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
        const int other = slot ^ 1;
        if (rec[other].pending) {
            QP_HIP(hipEventSynchronize(p->ev_poll[other]));
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
        }
        slot = other;
        return QP_OK;
    }
    qp_status clear_exec(int s)
    {
        QP_HIP(hipMemsetAsync(p->exec_hot() + s * kMaxBatch, 0, sizeof(int) * kMaxBatch, p->stream));
        QP_HIP(hipMemsetAsync(p->exec_res() + s, 0, sizeof(int), p->stream));
        return QP_OK;
    }
    qp_status final_states(State *out)
    {
        State *fin = host_states(2);
        QP_HIP(hipMemcpyAsync(fin, p->st(), sizeof(State) * K, hipMemcpyDeviceToHost, p->stream));
        QP_HIP(hipStreamSynchronize(p->stream));
        for (int s = 0; s < 2; ++s)
            if (rec[s].pending) {
                rec[s].pending = false;
                if (prof) QP_TRY(account(s));
            }
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

qp_status solve_fp64(qp_problem *p, int K, const double *rhs, double *U, double tol, State *st,
                     Profile &pf)
{
    const qp::Parts parts = p->parts();
    const bool prof = p->opt.profile != 0;
    QP_HIP(qp::launch_state_reset(K, p->st(), p->stream));
    QP_HIP(qp::launch_pcg_init(qp::F64, K, p->tab, p->host, rhs, nullptr, U, p->r(), p->h(),
                               p->M64(), parts, p->st(), p->stream));
    QP_HIP(qp::launch_pcg_start(qp::F64, K, p->host, tol, 0.0, p->opt.maxit, parts, p->st(),
                                p->stream));
    const int batch = batch_size(p->opt);
    Poller poll{p, K, prof, pf};
    Trend trend[qp::kMaxRhs];
    int k = batch;
    for (int j = 0; j < p->opt.maxit;) {
        k = std::min(k, p->opt.maxit - j);
        QP_TRY(queue_batch(p, false, K, U, nullptr, k, poll.slot, prof));
        j += k;
        bool fin = false;
        const State *seen = nullptr;
        QP_TRY(poll.push(k, 0, fin, &seen));
        if (fin) break;
        // Convergence expected within the queued batch: queue a short one.
        int next = batch;
        if (seen) {
            double need = 0.0;
            for (int r = 0; r < K; ++r) {
                if (seen[r].done) continue;
                if (trend[r].it < 0) trend[r].observe(0, seen[r].rr0);
                trend[r].observe(seen[r].iters, seen[r].rr);
                const double nr = trend[r].iters_to(seen[r].thresh);
                need = (nr < 0.0 || need < 0.0) ? -1.0 : std::max(need, nr);
            }
            next = next_batch(need, k, batch);
        }
        k = next;
    }
    return poll.final_states(st);
}

// FP32-IR: float C-PCG whose residual is replaced by the FP64 residual
// F' - Q X of the FP64 solution X whenever the float residual has dropped by
// `inner_tol` (or reached tol).  The replacement steps sit at the end of every
// batch and act on the paused right-hand sides; batches are sized to end just
// after the expected pause.
qp_status solve_ir(qp_problem *p, int K, const double *rhs, double *X, double tol, State *st,
                   Profile &pf)
{
    const qp::Parts parts = p->parts();
    const bool prof = p->opt.profile != 0;
    QP_HIP(qp::launch_state_reset(K, p->st(), p->stream));
    QP_HIP(qp::launch_ir_unit(K, p->tab, p->host, rhs, parts, p->st(), p->stream));
    QP_HIP(qp::launch_pcg_init(qp::F32, K, p->tab, p->host, rhs, X, p->x32(), p->r32(), p->h32(),
                               p->M32(), parts, p->st(), p->stream));
    QP_HIP(qp::launch_pcg_start(qp::F32, K, p->host, tol, p->opt.inner_tol, p->opt.maxit, parts,
                                p->st(), p->stream));
    const int batch = batch_size(p->opt);
    Poller poll{p, K, prof, pf};
    Trend trend[qp::kMaxRhs];
    int k = batch;
    for (int j = 0; j < p->opt.maxit;) {
        k = std::min(k, p->opt.maxit - j);
        QP_TRY(queue_batch(p, true, K, X, rhs, k, poll.slot, prof));
        j += k;
        bool fin = false;
        const State *seen = nullptr;
        QP_TRY(poll.push(k, 1, fin, &seen));
        if (fin) break;
        int next = batch;
        if (seen) {
            // seen: after a replacement (scaled true residual rr = rr_last);
            // the batch to size comes after the one queued (k iterations)
            int want = 2;
            bool known = true;
            for (int r = 0; r < K && known; ++r) {
                if (seen[r].done) continue;
                if (trend[r].it < 0) trend[r].observe(0, 1.0);
                trend[r].observe(seen[r].iters, seen[r].rr);
                const double target =
                    std::max(seen[r].thresh, seen[r].delta2 * seen[r].rr_last);
                const double need = trend[r].iters_to(target);
                int L;
                if (need < 0.0) {
                    known = false;
                    break;
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
            next = known ? want : batch;
        }
        k = next;
    }
    QP_TRY(poll.final_states(st));
    bool all_done = true;
    for (int r = 0; r < K; ++r) all_done = all_done && st[r].done;
    if (!all_done) {
        // iteration limit: fold every unfinished increment into X with one
        // forced replacement, whose true residual decides the status
        QP_HIP(qp::launch_ir_force(K, p->st(), p->stream));
        QP_TRY(enqueue_replacement(p, K, X, rhs, p->opt.maxit, 0, false));
        QP_HIP(hipMemcpyAsync(p->hstate + 2 * qp::kMaxRhs, p->st(), sizeof(State) * K,
                              hipMemcpyDeviceToHost, p->stream));
        QP_HIP(hipStreamSynchronize(p->stream));
        for (int r = 0; r < K; ++r) {
            st[r] = p->hstate[2 * qp::kMaxRhs + r];
            if (!st[r].done) st[r].status = QP_ENOCONV;
        }
    }
    return QP_OK;
}

// K right-hand sides (rhs + r D, solutions U + r D); infos: K entries or null.
qp_status solve_dispatch(qp_problem *p, int K, const double *rhs, double *U, double tol,
                         qp_solve_info *infos)
{
    const int D2 = 2 * p->host.D;
    if (K > 1 && (p->host.tile_s <= 1 || p->host.wide)) {
        // line tiles and 64-bit gathers serve one right-hand side per launch:
        // solve them in turn
        qp_status worst = QP_OK;
        for (int r = 0; r < K; ++r) {
            const qp_status s =
                solve_dispatch(p, 1, rhs + (size_t)r * D2, U + (size_t)r * D2, tol,
                               infos ? infos + r : nullptr);
            if (s == QP_EDEVICE || s == QP_EINVAL) return s;
            if (s != QP_OK && worst == QP_OK) worst = s;
        }
        return worst;
    }
    qp_solve_info local[qp::kMaxRhs];
    if (!infos) infos = local;
    std::memset(infos, 0, sizeof(qp_solve_info) * K);
    for (int r = 0; r < K; ++r) infos[r].flags = p->flags;
    if (!(tol > 0.0) || !std::isfinite(tol)) return fail(QP_EINVAL, "tol must be positive and finite");
    const bool ir = p->opt.precision == QP_PREC_FP32_IR;
    Profile pf;
    State st[qp::kMaxRhs];
    if (p->opt.profile) {
        QP_TRY(events_ready(p));
        QP_HIP(hipMemsetAsync(p->exec_hot(), 0, sizeof(int) * kExecInts, p->stream));
    }
    QP_HIP(hipEventRecord(p->ev_t0, p->stream));
    QP_TRY(ir ? solve_ir(p, K, rhs, U, tol, st, pf) : solve_fp64(p, K, rhs, U, tol, st, pf));
    QP_HIP(hipEventRecord(p->ev_t1, p->stream));
    QP_HIP(hipEventSynchronize(p->ev_t1));
    float ms = 0.f;
    QP_HIP(hipEventElapsedTime(&ms, p->ev_t0, p->ev_t1));
    qp_status worst = QP_OK;
    for (int r = 0; r < K; ++r) {
        qp_solve_info *info = infos + r;
        info->status = st[r].status;
        info->iters = st[r].iters;
        info->outer_iters = ir ? st[r].replacements : 0;
        info->rel_resid =
            ir ? std::sqrt(st[r].rr) : (st[r].rr0 > 0 ? std::sqrt(st[r].rr / st[r].rr0) : 0.0);
        info->seconds = ms * 1e-3;
        if (p->opt.profile) {
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
    if (worst == QP_ENOTSPD) fail(worst, "PCG breakdown: (Q h, h) <= 0");
    else if (worst == QP_ENOCONV) fail(worst, "iteration limit reached before the tolerance");
    else if (worst == QP_ENONFINITE) fail(worst, "non-finite value in the right-hand side or residual");
    return worst;
}

qp_status check_options(const qp_options *o)
{
    if (o->precision != QP_PREC_FP64 && o->precision != QP_PREC_FP32_IR)
        return fail(QP_EINVAL, "unknown precision %d", o->precision);
    if (o->precond != QP_PRECOND_PAPER && o->precond != QP_PRECOND_JACOBI)
        return fail(QP_EINVAL, "unknown preconditioner %d", o->precond);
    if (o->maxit < 1 || !(o->inner_tol > 0.0) || o->inner_tol >= 1.0 ||
        o->poll_every < 0 || o->poll_every > kMaxBatch)
        return fail(QP_EINVAL, "invalid iteration limits or inner tolerance");
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
    opt->inner_tol = 1e-4;
    opt->poll_every = 0;
    opt->graphs = 1;
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
    return make_layout(d, n, N, D, g).total;
}

// coefs: null (scalar coefficient `coef`) or d x g complex (diagonal coefficient)
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
    // record indices of the default gathers are scaled by the entry size in 32
    // bits: vectors of 2^28 entries or more take 64-bit addresses
    if (p->host.tile_s > 1 && (o.gather64 || p->host.D >= ((int64_t)1 << 28))) p->host.wide = 1;
    p->L = make_layout(d, n, N, p->host.D, g);

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
        hipHostMalloc(&p->hexec, kExecInts * sizeof(int), hipHostMallocDefault) != hipSuccess)
        return bail(fail(QP_ENOMEM, "pinned host allocation failed"));
    for (auto &e : p->ev_poll)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            return bail(fail(QP_EDEVICE, "hipEventCreate failed"));
    if (hipEventCreate(&p->ev_t0) != hipSuccess || hipEventCreate(&p->ev_t1) != hipSuccess)
        return bail(fail(QP_EDEVICE, "hipEventCreate failed"));
    p->tab = p->at<Table>(p->L.tab);
    if (hipMemcpyAsync(p->tab, &p->host, sizeof(Table), hipMemcpyHostToDevice, p->stream) != hipSuccess)
        return bail(fail(QP_EDEVICE, "table upload failed"));
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
    if (p->amin < -1e-12 * scale)
        return bail(fail(QP_ENOTELLIPTIC, "coefficient minimum on the grid is %.6g < 0", p->amin));
    if (std::fabs(p->amin) <= 1e-12 * scale) p->flags |= QP_FLAG_DEGENERATE;
    *out = p;
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
    const int old_precond = p->opt.precond;
    void *stream = p->opt.stream;
    p->opt = *opt;
    p->opt.stream = stream;
    p->opt.workspace = nullptr;
    if (opt->precond != old_precond) return compute_setup(p);
    return QP_OK;
}

qp_status qp_solve_d(qp_problem *p, const double *rhs, double *u, double tol, qp_solve_info *info)
{
    if (!p || !rhs || !u) return fail(QP_EINVAL, "null argument");
    if (rhs == u) return fail(QP_EINVAL, "rhs and u must not overlap");
    return solve_dispatch(p, 1, rhs, u, tol, info);
}

qp_status qp_solve_multi_d(qp_problem *p, int K, const double *rhs, double *u, double tol,
                           qp_solve_info *infos)
{
    if (!p || !rhs || !u) return fail(QP_EINVAL, "null argument");
    if (K < 1 || K > p->host.d)
        return fail(QP_EINVAL, "K = %d right-hand sides outside [1, d = %d]", K, p->host.d);
    const size_t bytes = 16 * (size_t)p->host.D * K;
    const char *a = reinterpret_cast<const char *>(rhs), *b = reinterpret_cast<const char *>(u);
    if (a < b + bytes && b < a + bytes) return fail(QP_EINVAL, "rhs and u must not overlap");
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
    const int d = p->host.d;
    // the d corrector right-hand sides, solved together
    for (int j = 0; j < d; ++j)
        QP_HIP(qp::launch_corrector_rhs(p->tab, p->host, j, p->F() + (size_t)2 * p->host.D * j,
                                        p->stream));
    const qp_status worst = solve_dispatch(p, d, p->F(), p->chi(0), tol, info);
    if (worst == QP_EDEVICE || worst == QP_EINVAL) return worst;
    QP_HIP(qp::launch_astar(p->tab, p->host, p->chi(0), p->small(), p->stream));
    if (Astar_energy) {
        const qp::Parts parts = p->parts();
        for (int j = 0; j < d; ++j) {
            QP_HIP(qp::launch_matvec(qp::F64, qp::EPI_NONE, 1, p->tab, p->host, p->recs(),
                                     p->urec(qp::F64), p->upku(qp::F64), p->chi(j), p->q(), nullptr,
                                     nullptr, parts, p->st(), nullptr, p->stream));
            for (int i = 0; i < d; ++i)
                QP_HIP(qp::launch_dot(p->tab, p->host, p->chi(i), p->q(), parts,
                                      p->small() + 64 + i * d + j, p->stream));
        }
    }
    QP_HIP(hipMemcpyAsync(p->hsmall, p->small(), 128 * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    QP_HIP(hipStreamSynchronize(p->stream));
    for (int e = 0; e < d * d; ++e) Astar[e] = p->hsmall[e];
    if (Astar_energy)
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j)
                Astar_energy[i * d + j] = (i == j ? p->host.a0l[i] : 0.0) - p->hsmall[64 + i * d + j];
    if (worst != QP_OK) fail(worst, "a corrector solve did not converge");
    return worst;
}

qp_status qp_homogenized(qp_problem *p, double *Astar, double tol, qp_solve_info *info)
{
    return qp_homogenized_ex(p, Astar, nullptr, tol, info);
}

qp_status qp_matvec_d(qp_problem *p, const double *u, double *y)
{
    if (!p || !u || !y) return fail(QP_EINVAL, "null argument");
    QP_HIP(qp::launch_matvec(qp::F64, qp::EPI_NONE, 1, p->tab, p->host, p->recs(), p->urec(qp::F64),
                             p->upku(qp::F64), u, y, nullptr,
                             nullptr, p->parts(), p->st(), nullptr, p->stream));
    QP_HIP(hipStreamSynchronize(p->stream));
    return QP_OK;
}

qp_status qp_matvec32_d(qp_problem *p, const float *u, float *y)
{
    if (!p || !u || !y) return fail(QP_EINVAL, "null argument");
    QP_HIP(qp::launch_matvec(qp::F32, qp::EPI_NONE, 1, p->tab, p->host, p->recs(), p->urec(qp::F32),
                             p->upku(qp::F32), u, y, nullptr,
                             nullptr, p->parts(), p->st(), nullptr, p->stream));
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

}  // extern "C"
