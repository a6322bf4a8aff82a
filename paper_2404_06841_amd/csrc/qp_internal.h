// Internal interface between the host runtime (qp_api.cpp) and the gfx950
// kernels.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qp.h"

namespace qp {

constexpr int kMaxN = QP_MAX_DIM_N;
constexpr int kMaxD = QP_MAX_DIM_D;
constexpr int kMaxG = QP_MAX_MODES;
constexpr int kBlock = 256;       // threads per workgroup (4 wave64)
#ifndef QP_MAX_BLOCKS
#define QP_MAX_BLOCKS 1024
#endif
constexpr int kMaxBlocks = QP_MAX_BLOCKS;  // grid cap (partial sums per reduction)
#ifndef QP_STREAM_BLOCKS
#define QP_STREAM_BLOCKS 1024
#endif
constexpr int kStreamBlocks = QP_STREAM_BLOCKS;  // upper cap of the streaming kernels' grid

// Problem constants, resident in device memory and read with uniform
// (scalar) loads by every kernel.
struct Table {
    int d, n, N, g;
    int D;                    // N^n
    int nblocks;              // grid of the streaming kernels
    int chunk;                // elements per workgroup (multiple of kBlock)
    int zero_mode;            // index of the mode m = 0
    uint64_t magic;           // floor division by N: (x * magic) >> shift, x < 2^31
    int shift;
    int real_coef;            // every Ahat_m has zero imaginary part
    int stride[kMaxN];        // N^(n-1-t)
    double P[kMaxD][kMaxN];   // projection matrix, row-major
    int modes[kMaxG][kMaxN];  // coefficient modes m
    double coef[kMaxG][2];    // Ahat_m (re, im)
    double Pm[kMaxG][kMaxD];  // P m
    int off[kMaxG];           // -sum_t m_t N^(n-1-t): unwrapped storage offset
    int midx[kMaxG];          // C(m): storage index of mode m
    int nidx[kMaxG];          // C(-m)
    double a0;                // Ahat_0
    // ---- diagonal coefficient diag(a_1..a_d) (App. D); for a scalar
    // coefficient every entry repeats coef ----
    int aniso;                // coefl differs between entries (diagonal coefficient)
    double coefl[kMaxG][kMaxD][2];  // Ahat of a_l at mode r (re, im)
    double a0l[kMaxD];        // Ahat^l_0
    // ---- tiled stiffness product (modes sorted by their last component) ----
    int order[kMaxG];         // sorted position -> mode index
    int zero_sorted;          // sorted position of the mode m = 0
    int lanes_p;              // positions of a line per tile row (min(N, 64))
    int tile_s;               // lines per tile (> 1: tiles of a plane, n >= 2 and N <= 32)
    int tiles_per_unit;       // tiles per plane (tile_s > 1) or per line
    int ntiles;
    int nb_mv;                // grid of the stiffness product (multiple of 8 when >= 8)
    int item_tiles;           // plane tiles: consecutive tiles of a unit per wave item
    int xcd_front;            // plane tiles: each XCD sweeps its own contiguous eighth
                              // (2: with the slowest axis innermost, slab_span > 0)
    int slab_units;           // units (planes) per eighth, when they divide evenly
    int slab_stride;          // units per value of the slowest axis (N^(n-3))
    int slab_span;            // values of the slowest axis per eighth (0: no slab order)
    int item_tiles64;         // the same three for the FP64 launches (tuned apart:
    int nb_mv64;              // the float product and the FP64 one prefer different
    int xcd_front64;          // layouts)
    int wide;                 // plane tiles: 64-bit neighbour addresses, one right-hand
                              // side per launch (else 32-bit record indices)
    uint64_t slotmask[64];    // tile_s > 1: per tile of a plane, bit r when sorted mode
                              // r's neighbour leaves [0, N) or K_N in axis n-2 for some line
    // ---- Hermitian half storage (real scalar coefficient, odd N, plane tiles):
    // vectors hold the (N^n + 1)/2 stored entries of the half layout below,
    // D is that count, and the product's units are the stored planes ----
    int half;                 // 1: half storage
    int Dgrid;                // N^n (= D without half storage)
    int half_units;           // stored planes: (N^(n-2) + 1)/2, the center plane first
    int nconj[kMaxG];         // half storage: chi at C(-m) is conj(chi[nidx[r]])
};

// ---- Hermitian half layout (odd N) ----
// The stored half of an m-dimensional grid (digits b_t in [0, N), first
// axis slowest) is k = 0 and every k whose first nonzero signed component is
// positive: the index ranges [S, (N+1)/2 S) for S = 1, N, ..., N^(m-1) (the
// first nonzero digit at place S lies in [1, (N-1)/2]).  Position 0 holds
// k = 0; index i of range S sits at position i - (S - 1)/2; positions run to
// (N^m + 1)/2.  For the n-dimensional vectors the layout is the center plane
// (uniform digits 0; its own half, positions [0, (N^2+1)/2)) followed by whole
// planes in the half order of the (n-2)-dimensional plane grid: stored plane
// hu >= 1 starts at position (N^2 + 1)/2 + (hu - 1) N^2.
__host__ __device__ inline long long half_index(long long pos, int N, int m)
{
    if (pos == 0) return 0;
    long long S = 1, top = 1;
    for (int t = 1; t < m; ++t) top *= N;
    while (S < top && (S * N + 1) / 2 <= pos) S *= N;
    return pos + (S - 1) / 2;
}
// Position of index i, which must lie in the stored half (i = 0 or its first
// nonzero digit in [1, (N-1)/2]).
__host__ __device__ inline long long half_position(long long i, int N, int m)
{
    if (i == 0) return 0;
    long long S = 1;
    for (int t = 1; t < m; ++t) S *= N;
    while (S > i) S /= N;
    return i - (S - 1) / 2;
}
// Whether index i of an m-dimensional grid lies in the stored half.
__host__ __device__ inline bool half_stored(long long i, int N, int m)
{
    if (i == 0) return true;
    long long S = 1;
    for (int t = 1; t < m; ++t) S *= N;
    while (S > i) S /= N;
    return (i / S) % N <= (N - 1) / 2;
}
// Index of -k for index i (every digit b -> (N - b) mod N).
__host__ __device__ inline long long mirror_index(long long i, int N, int m)
{
    long long out = 0, S = 1;
    for (int t = 0; t < m; ++t) {
        const long long b = i % N;
        i /= N;
        out += ((N - b) % N) * S;
        S *= N;
    }
    return out;
}

// Per-mode record of the tiled stiffness product, in sorted order.
struct alignas(128) ModeRec {
    double pm[kMaxD];      // P m (zero padded)
    double cpm[kMaxD];     // Re(Ahat_m) P m
    double c[2];           // Ahat_m
    short mt[kMaxN];       // m (all axes); |m_t| < N/2 < 2^15
    double cl[kMaxD][2];   // Ahat of a_l at m (diagonal coefficient; else Ahat_m)
    int pad[8];
};
static_assert(sizeof(ModeRec) == 256, "mode record is two 128-byte blocks");

// Mode record of one unit of the plane-tiled stiffness product (the tiles
// sharing every digit but the last two), precomputed once per problem:
// units * padded modes records per precision.
template <typename T, int DT>
struct alignas(16) UnitRec {
    T apm[DT];  // a (P m - N sum_{t < n-2} c_t p_t), c_t the wrap of axis t
    T a;        // Re(Ahat_m) for real coefficients, else 1; 0 for padding
    T cr, ci;   // Ahat_m (complex multiply-add); 0 for padding
    int lb;     // element offset of the neighbour's row over axes < n-2, minus m_{n-2} N;
                // kNoNeighbour for padding
    int mslot;  // m_{n-2}
};
// Row offset of a padding record: adding any in-plane offset (< 2^30) leaves
// an index whose unsigned value exceeds every vector length (< 2^31).
constexpr int kNoNeighbour = -(1 << 30);
// The same for a diagonal coefficient diag(a_1..a_d) (App. D): per physical
// axis l, (P m')_l and a_l's Ahat_m.
template <typename T, int DT>
struct alignas(16) UnitRecA {
    T pmw[DT];  // (P m - N sum_{t < n-2} c_t p_t)_l
    T ar[DT];   // Re(Ahat of a_l at m); 0 for padding
    T ai[DT];   // Im(Ahat of a_l at m); 0 for padding
    int lb;     // as UnitRec
    int mslot;
};
// Unit record of the plane-tile product on Hermitian half storage: as
// UnitRec, with the source plane's place in the half layout.  kind 0: the
// source plane is stored, lb as UnitRec's relative to its first position;
// kind 1: its mirror (every digit negated) is stored from position lb, read
// at the mirrored in-plane digits and conjugated; kind 2: the source is the
// center plane (stored as its own half), resolved per lane.
template <typename T, int DT>
struct alignas(16) HalfRec {
    T apm[DT];
    T a;
    T cr, ci;
    int lb;
    int mslot;
    int kind;
    int pad;
};
// bytes reserved per record (at least the size of either record for d =
// kMaxD), by Precision
constexpr size_t kUnitRecBytes[2] = {112, 64};

// Krylov state of one solve, device resident.  All scalars are FP64.
// Fields are written by workgroup 0 of one kernel and read by later kernels
// only: no kernel takes a decision from a field it writes itself (rz[]
// alternates between two slots by iteration parity).
struct State {
    double rz[2];     // (r, M r): slot j & 1 holds the value entering iteration j
    double alpha, beta, hq;
    double rr;        // last ||r||^2 (recursive residual, solve units)
    double rr0;       // ||F'||^2
    double thresh;    // convergence: rr <= thresh (solve units)
    double delta2;    // FP32-IR: replace the residual once rr <= delta2 * rr_last
    double rr_last;   // FP32-IR: rr after the last residual replacement
    double rr_pause;  // FP32-IR: recursive rr at the pause (snapshot taken by the fold)
    double unit;      // FP32-IR: ||F'||; float vectors hold (true value) / unit
    double inv_unit;
    int iters;        // update steps performed
    int replacements; // FP32-IR: FP64 residual replacements
    int done;         // nonzero: every later kernel of this solve returns at once
    int pause;        // FP32-IR: float iterations wait for the next replacement
    int status;       // qp_status of the solve
    int maxit;
    int did_update;   // the update of the current iteration ran (written by the update)
    int replace;      // FP32-IR: this replacement acts (written by the fold)
    double *hist;     // Lanczos coefficients of the solve: (alpha_j, beta_j) at
                      // hist[2 j], hist[2 j + 1] for j < kHist (set once per
                      // problem; the kernels' lead threads write the entries)
};
// Iterations whose PCG coefficients a solve keeps for its condition estimate.
constexpr int kHist = 1024;

// Store alpha of iteration `it` (0-based) / beta after it, when kept.
__device__ __forceinline__ void hist_alpha(State *st, int it, double alpha)
{
    if (st->hist && it >= 0 && it < kHist) st->hist[2 * it] = alpha;
}
__device__ __forceinline__ void hist_beta(State *st, int it, double beta)
{
    if (st->hist && it >= 0 && it < kHist) st->hist[2 * it + 1] = beta;
}

enum Epilogue { EPI_NONE = 0, EPI_ALPHA = 1, EPI_RESID = 2 };

// One problem of a grouped launch (FP32-IR steps of several problems in one
// launch): its table, records and vectors, and the workgroups it owns.
// Workgroup w of a grouped product launch serves problem owner_mv[w] as
// workgroup w - mv0 of nb_mv; of a grouped vector launch, problem owner_st[w]
// as workgroup w - sv0 of nb_st.
struct GroupEntry {
    const Table *tab;
    const ModeRec *recs;
    const void *urec32, *upku32, *urec64, *upku64;  // unit records per precision
    float *x32, *r32, *h32, *q32;                   // float families (K interleaved)
    const float *M32;
    double *X;                                      // FP64 solutions (K vectors)
    const double *F;                                // FP64 right-hand sides (K vectors)
    double *pa, *pb;                                // partial sums (Parts a, b)
    State *st;                                      // K states
    int mv0, nb_mv, sv0, nb_st;
    int mv064, nb_mv64;  // the FP64 product's workgroups (owner_mv64)
    int wide;            // chunk > 4 kBlock: the float update and direction load
                         // eight rows per thread (as the problem's own launches)
};
enum Precision { F64 = 0, F32 = 1 };

// Partial-sum buffers: each holds kMaxRhs slices of kPartStride doubles
// (kPartValues values per workgroup); right-hand side k uses slice k.
constexpr int kPartValues = 2;
constexpr int kMaxRhs = kMaxD;  // right-hand sides solved together (the d correctors)
constexpr size_t kPartStride = (size_t)kPartValues * kMaxBlocks;
struct Parts {
    double *a;  // written by the stiffness product (h^H Q h)
    double *b;  // written by the vector update / residual ((r, M r), ||r||^2)
    double *c;  // auxiliary reductions (norms, dots, extrema)
};

// ---- launchers; all enqueue on `s` and return the launch status ----
//
// K right-hand sides (1 <= K <= kMaxRhs) are served by one launch: vector k
// of a family starts at element k * D, its state is st[k], its partials are
// slice k of the partial buffers.

// Stiffness product, one launch over K vectors (K > 1 for plane tiles only):
//   EPI_NONE : y_k = Q x_k
//   EPI_ALPHA: y_k = Q x_k and parts.a[k] <- Re(x_k^H y_k), for the right-hand
//              sides neither done nor paused (returns at once if none);
//              *exec (nullable) <- the number of right-hand sides served
//   EPI_RESID: FP64 only. y_k (float2) = (f'_k - Q x_k) * st[k].inv_unit and
//              parts.b[k] <- (sum M32 |y_k|^2, sum |(f'_k - Q x_k) inv_unit|^2),
//              for the right-hand sides paused and not done
// recs: g mode records in sorted order; urec / upku: the unit records and
// the units' P k over axes < n-2 of precision prec (plane tiles only).
hipError_t launch_matvec(int prec, int epi, int K, const Table *tab, const Table &ht,
                         const ModeRec *recs, const void *urec, const void *upku,
                         const void *x, void *y,
                         const double *f, const float *M32, const Parts &parts, State *st,
                         int *exec, hipStream_t s, hipEvent_t ev0 = nullptr,
                         hipEvent_t ev1 = nullptr);
// y = Q u on Hermitian half storage ((D+1)/2 complex doubles each, the layout
// of qp_matvec_half_d); scalar real coefficient, odd N (checked by the caller).
hipError_t launch_matvec_half(const Table *tab, const Table &ht, const void *u, void *y,
                              hipStream_t s);
// The same on Hermitian half storage (tab.half; called by launch_matvec): x and
// y hold the tab.D stored entries; the unit records are those of
// launch_unit_records on a half-storage table.
hipError_t launch_matvec_tiled_half(int prec, int epi, int K, const Table *tab, const Table &ht,
                                    const ModeRec *recs, const void *urec, const void *upku,
                                    const void *x, void *y, const double *f, const float *M32,
                                    const Parts &parts, State *st, int *exec, hipStream_t s,
                                    hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t launch_unit_records_half(int prec, const Table *tab, const Table &ht,
                                    const ModeRec *recs, void *urec, void *upku, hipStream_t s);
// The same for a diagonal coefficient (tab.aniso; called by launch_matvec).
hipError_t launch_matvec_diag(int prec, int epi, int K, const Table *tab, const Table &ht,
                              const ModeRec *recs, const void *urec, const void *upku,
                              const void *x, void *y, const double *f, const float *M32,
                              const Parts &parts, State *st, int *exec, hipStream_t s,
                              hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// Start of a solve.  r = f' * scale (scale = 1 for F64, st->inv_unit for F32),
// U = 0, X64 = 0 (if given), h = M r; parts.b <- ((r, M r), ||r||^2).
hipError_t launch_pcg_init(int prec, int K, const Table *tab, const Table &ht, const double *f,
                           double *X64, void *U, void *r, void *h, const void *M,
                           const Parts &parts, State *st, hipStream_t s);
// One workgroup: totals of parts.b -> rz[0], rr; F64: rr0, thresh = tol^2 rr0;
// F32: thresh = tol^2, delta2, rr_last.  done when rr is 0; status on NaN.
hipError_t launch_pcg_start(int prec, int K, const Table &ht, double tol, double delta,
                            int maxit, const Parts &parts, State *st, hipStream_t s);
// Iteration j: alpha = rz[j&1] / (totals of parts.a) (kept in the state);
// r -= alpha q; parts.b <- ((r, M r), ||r||^2).
hipError_t launch_pcg_update(int prec, int j, int K, const Table *tab, const Table &ht, void *r,
                             const void *q, const void *M, const Parts &parts, State *st,
                             hipStream_t s);
// Iteration j (right-hand sides whose update ran): U += alpha h; then, unless
// F64 stops (convergence, maxit) or F32 pauses (the residual has dropped
// enough): beta from parts.b, h = M r + beta h.
hipError_t launch_pcg_direction(int prec, int j, int K, const Table *tab, const Table &ht, void *U,
                                const void *r, void *h, const void *M, const Parts &parts,
                                State *st, hipStream_t s);
// FP64 C-PCG of K right-hand sides to the end, one workgroup each, from the
// vectors and states of launch_pcg_init / launch_pcg_start (scalar
// coefficient, full storage, at most kSmallMax unknowns).
constexpr int kSmallMax = 2048;
hipError_t launch_pcg_wg(int K, const Table *tab, const Table &ht, double *U, double *r, double *h,
                         const double *M, State *st, hipStream_t s);
// FP32-IR start: st->rr0 = ||f'||^2, unit = sqrt(rr0) (two launches).
hipError_t launch_ir_unit(int K, const Table *tab, const Table &ht, const double *f,
                          const Parts &parts, State *st, hipStream_t s);
// FP32-IR residual replacement (paused right-hand sides): X += unit * x; x = 0.
hipError_t launch_ir_fold(int K, const Table *tab, const Table &ht, double *X, float *x,
                          State *st, hipStream_t s);
// FP32-IR, after the FP64 residual (EPI_RESID), paused right-hand sides:
// convergence on the true residual, else beta, h = M r + beta h, pause cleared.
hipError_t launch_ir_direction(int j, int K, const Table *tab, const Table &ht, const float *r,
                               float *h, const float *M, const Parts &parts, State *st,
                               hipStream_t s);

// FP32-IR: pause every unfinished right-hand side (final forced replacement).
// Grouped FP32-IR steps over the problems of E (see GroupEntry); total: the
// workgroups of the launch (the sum of the problems' nb_mv for the product,
// of their nb_st for the vector steps), owner: the problem of each.
// Product: prec F32 = float product of h into q with the alpha partials,
// F64 = replaced FP64 residual of X into the float r; d in {2, 3}, K = d,
// scalar coefficient (real or complex), gpmax = the largest padded mode count.
hipError_t launch_group_matvec(int prec, int d, bool real, int total, int gpmax,
                               const GroupEntry *E, const int *owner, hipStream_t s);
// Vector steps of iteration j: 0 update, 1 direction, 2 fold, 3 replacement
// direction; K in {2, 3}.
hipError_t launch_group_vec(int step, int j, int K, int total, const GroupEntry *E, const int *owner,
                            hipStream_t s);
// out[g K + k] = state k of problem g (one workgroup; out in device memory).
hipError_t launch_group_states(int G, int K, const GroupEntry *E, State *out, hipStream_t s);
// Bit i % 32 of words[i / 32] = every one of problem i's K states is done, for
// i < G; the other bits of the (G + 31) / 32 words are 0 (one workgroup).
hipError_t launch_group_done(int G, int K, const GroupEntry *E, uint32_t *words, hipStream_t s);
// Bytes of the grouped launches' static device scratch array.
constexpr size_t kGroupScratchBytes = (size_t)4 << 20;
// The address of that array on `device` (looked up once per device with the
// device current) and its size.
hipError_t group_scratch(int device, void **ptr, size_t *bytes);
hipError_t launch_ir_force(int K, State *st, hipStream_t s);

// ---- setup and single-step kernels ----
// Unit records and unit P k of precision prec (plane tiles, tile_s > 1).
hipError_t launch_unit_records(int prec, const Table *tab, const Table &ht, const ModeRec *recs,
                               void *urec, void *upku, hipStream_t s);
hipError_t launch_unit_records_diag(int prec, const Table *tab, const Table &ht,
                                    const ModeRec *recs, void *urec, void *upku, hipStream_t s);
// M (double and float copies); kind 0 paper, 1 Jacobi; out[0] = min_{k!=0} |P k|^2.
hipError_t launch_precond(const Table *tab, const Table &ht, int kind, double *M64, float *M32,
                          const Parts &parts, double *out, hipStream_t s);
// out[0] = min, out[1] = max of A over the collocation grid.
hipError_t launch_extrema(const Table *tab, const Table &ht, const Parts &parts, double *out,
                          hipStream_t s);
// F_k = i (P k)_j Ahat_k.
hipError_t launch_corrector_rhs(const Table *tab, const Table &ht, int j, double *F,
                                hipStream_t s);
// The sources of correctors 0 .. K-1 (F + j D); with parts, also the partial
// sums of ||f'_j||^2 in parts->c (as launch_ir_unit's first launch stores
// them).
hipError_t launch_corrector_rhs_all(const Table *tab, const Table &ht, int K, double *F,
                                    const Parts *parts, hipStream_t s);
// FP32-IR unit from the ||f'||^2 partials already in parts.c (one launch).
hipError_t launch_ir_unit_only(int K, const Table &ht, const Parts &parts, State *st,
                               hipStream_t s);
// A* flux form from d correctors (d*D complex): out[0..d*d) real, out[d*d..) imag.
hipError_t launch_astar(const Table *tab, const Table &ht, const double *chi, double *out,
                        hipStream_t s);
// out[0] = Re(x^H y).
hipError_t launch_dot(const Table *tab, const Table &ht, const double *x, const double *y,
                      const Parts &parts, double *out, hipStream_t s);
// Signed multi-index of every entry (D x n int32).
hipError_t launch_multi_index(const Table *tab, const Table &ht, int32_t *k, hipStream_t s);
// The compressed stiffness matrix of Alg. 1: D * g triples (i, j, Q_ij),
// mode-major (row i's r-th entry at r D + i, zero values kept), FP64 values.
hipError_t launch_coo_build(const Table *tab, const Table &ht, int32_t *rows, int32_t *cols,
                            double *vals, hipStream_t s);
// y = Q x from those triples (FP64).
hipError_t launch_coo_matvec(const Table &ht, const int32_t *cols, const double *vals,
                             const double *x, double *y, hipStream_t s);
// n-dimensional DFT on T_N^n in storage order: forward (1/D normalized) or
// inverse, in (D complex) -> out (D complex; may equal in).
hipError_t launch_dft(int n, int N, const double *in, double *out, int inverse, hipStream_t s);
// Reset K States (flags, counters) with a kernel (no memset node).
hipError_t launch_state_reset(int K, State *st, hipStream_t s);
// Point state r of the kMaxRhs states at hist + 2 kHist r (once per problem).
hipError_t launch_state_hist(State *st, double *hist, hipStream_t s);

}  // namespace qp
