// Discrete Fourier transforms on the collocation grid T_N^n (Sec. 2.3): the
// discrete Fourier-Bohr coefficients of sampled parent functions,
//   forward:  out_k = (1/D) sum_{j in [0,N)^n} in_j exp(-2 pi i k.j / N),
//   inverse:  out_j = sum_k in_k exp(+2 pi i k.j / N),
// both indexed by the storage order of Sec. 3.1.2 (digit k mod N, first axis
// slowest), which is the sample order of the grid y_j = 2 pi j / N.
//
// The n-dimensional transform is a sequence of 1D transforms of length N
// along each axis.  One launch (a pass) transforms a group of consecutive
// axes [t0, t1): a workgroup loads B whole sub-grids of M = N^(t1-t0)
// entries (the entries that differ only in those axes' digits) into LDS,
// runs the 1D transform along each axis of the sub-grid there, and stores
// the sub-grids back, so every pass reads and writes the vector once.  Passes
// cover the axes from the last (fastest) to the first; the first pass reads
// `in`, the later ones transform `out` in place (a workgroup owns whole
// sub-grids).  Consecutive sub-grids sit next to each other in memory (or,
// for the pass holding the last axis, are contiguous blocks), and the lanes
// of a workgroup take consecutive ones, so loads and stores coalesce.
//
// The 1D transform is a mixed-radix Stockham FFT (self-sorting: each stage
// reads one LDS buffer and writes the other, no bit reversal) over the prime
// factors of N, radix 4 and 2 written out and any other factor p evaluated as
// a direct p-point sum; twiddles exp(-+2 pi i q / N) come from an FP64 table
// with the index q reduced exactly in integers.  Error about eps log N per
// axis (a prime N degenerates into one direct N-point sum, eps N).
#include <algorithm>

#include "qp_device.h"

namespace qp {
namespace {

constexpr int kDftMaxN = 1024;      // line length
constexpr int kDftLdsEntries = 4096; // complex doubles of LDS (64 KB): twiddles + two buffers
constexpr int kMaxRadices = 12;      // 2^10 = 1024 has ten factors

struct DftPlan {
    int N;
    int nr;                      // radices in stage order
    int radix[kMaxRadices];
};

// One radix-r Stockham stage of every length-N line of the sub-grids held in
// src (lines lines, M entries per sub-grid): the lines run along an axis of
// element stride ls inside a sub-grid; Ns = product of the earlier stages'
// radices.  Butterfly j of a line (0 <= j < N/r) reads entries j + q N/r,
// twiddles them by w^(q k) with k = j mod Ns and w = exp(-+2 pi i/(Ns r)),
// and writes the r-point transform to entries (j/Ns) Ns r + k + p Ns.
__device__ __forceinline__ void dft_stage(const double2 *__restrict__ src, double2 *__restrict__ dst,
                                          const double2 *__restrict__ tw, int N, int r, int Ns,
                                          int ls, int lines, int M, bool inverse)
{
    const int nb = N / r;           // butterflies per line
    const int step = N / (Ns * r);  // twiddle index step of this stage
    const int per = M / N;          // lines per sub-grid along this axis
    auto line_base = [&](int L) {   // entry 0 of line L
        const int sg = L / per, rem = L - sg * per;
        const int hi = rem / ls, lo = rem - hi * ls;
        return sg * M + hi * ls * N + lo;
    };
    auto twiddled = [&](int base, int j, int k, int q) {
        double2 v = src[base + (j + q * nb) * ls];
        if (q == 0) return v;
        const double2 w = tw[q * k * step];  // q k step < N
        return make_double2(v.x * w.x - v.y * w.y, v.x * w.y + v.y * w.x);
    };
    if (r == 2 || r == 4) {
        for (int e = threadIdx.x; e < lines * nb; e += kBlock) {
            const int L = e / nb, j = e - (e / nb) * nb;
            const int base = line_base(L);
            const int k = j % Ns;
            const int o = base + ((j / Ns) * Ns * r + k) * ls;
            if (r == 2) {
                const double2 a = twiddled(base, j, k, 0), b = twiddled(base, j, k, 1);
                dst[o] = make_double2(a.x + b.x, a.y + b.y);
                dst[o + Ns * ls] = make_double2(a.x - b.x, a.y - b.y);
            } else {
                const double2 x0 = twiddled(base, j, k, 0), x1 = twiddled(base, j, k, 1);
                const double2 x2 = twiddled(base, j, k, 2), x3 = twiddled(base, j, k, 3);
                // y_p = sum_q x_q W^(pq), W = -i (forward) or +i (inverse)
                const double2 s02 = make_double2(x0.x + x2.x, x0.y + x2.y);
                const double2 d02 = make_double2(x0.x - x2.x, x0.y - x2.y);
                const double2 s13 = make_double2(x1.x + x3.x, x1.y + x3.y);
                const double2 d13 = make_double2(x1.x - x3.x, x1.y - x3.y);
                // W (x1 - x3): forward -i d13, inverse +i d13
                const double2 wd = inverse ? make_double2(-d13.y, d13.x) : make_double2(d13.y, -d13.x);
                dst[o] = make_double2(s02.x + s13.x, s02.y + s13.y);
                dst[o + Ns * ls] = make_double2(d02.x + wd.x, d02.y + wd.y);
                dst[o + 2 * Ns * ls] = make_double2(s02.x - s13.x, s02.y - s13.y);
                dst[o + 3 * Ns * ls] = make_double2(d02.x - wd.x, d02.y - wd.y);
            }
        }
        return;
    }
    // any other factor: one thread per output p of a butterfly, a direct
    // r-point sum with W^(pq) = tw[((p q) mod r) N/r]
    for (int e = threadIdx.x; e < lines * nb * r; e += kBlock) {
        const int L = e / (nb * r), jp = e - L * (nb * r);
        const int j = jp / r, p = jp - j * r;
        const int base = line_base(L);
        const int k = j % Ns;
        double ar = 0.0, ai = 0.0;
        int pq = 0;  // (p q) mod r
        for (int q = 0; q < r; ++q) {
            const double2 v = twiddled(base, j, k, q);
            const double2 w = tw[pq * nb];
            ar += v.x * w.x - v.y * w.y;
            ai += v.x * w.y + v.y * w.x;
            pq += p;
            pq -= (pq >= r) ? r : 0;
        }
        dst[base + ((j / Ns) * Ns * r + k + p * Ns) * ls] = make_double2(ar, ai);
    }
}

// Pass over axes [t0, t1): sub-grids of M = N^na entries with element
// stride S (= N^(n - t1)) in memory; subs sub-grids in all; B per workgroup
// iteration.
__global__ __launch_bounds__(kBlock) void k_dft_pass(DftPlan plan, int na, int M, long long S,
                                                     long long subs, int B, int inverse,
                                                     double scale,
                                                     const double2 *__restrict__ in,
                                                     double2 *__restrict__ out)
{
    extern __shared__ double2 s_dft[];  // twiddles (N), then two buffers of B * M
    const int N = plan.N;
    double2 *tw = s_dft;
    double2 *buf0 = s_dft + N;
    double2 *buf1 = buf0 + (size_t)B * M;
    const double sgn = inverse ? 1.0 : -1.0;
    for (int j = threadIdx.x; j < N; j += kBlock) {
        double sn, cs;
        sincospi(2.0 * (double)j / (double)N, &sn, &cs);
        tw[j] = make_double2(cs, sgn * sn);
    }
    for (long long s0 = (long long)blockIdx.x * B; s0 < subs; s0 += (long long)gridDim.x * B) {
        const int nb = (int)min((long long)B, subs - s0);
        // sub-grid s = outer * S + inner starts at outer * M * S + inner; its
        // entry e sits e * S further.  S > 1: lanes take consecutive
        // sub-grids (adjacent inner values); S = 1: consecutive entries.
        __syncthreads();  // the previous iteration's stores have read the buffer
        for (int e = threadIdx.x; e < nb * M; e += kBlock) {
            int b, m;
            if (S > 1) {
                b = e % nb;
                m = e / nb;
            } else {
                m = e % M;
                b = e / M;
            }
            const long long sub = s0 + b;
            const long long outer = sub / S, inner = sub - outer * S;
            buf0[b * M + m] = in[outer * (long long)M * S + inner + (long long)m * S];
        }
        __syncthreads();
        double2 *src = buf0, *dst = buf1;
        // axes of the sub-grid from the last (element stride 1) to the first
        for (int a = na - 1, ls = 1; a >= 0; --a, ls *= N) {
            int Ns = 1;
            for (int st = 0; st < plan.nr; ++st) {
                dft_stage(src, dst, tw, N, plan.radix[st], Ns, ls, nb * (M / N), M, inverse != 0);
                Ns *= plan.radix[st];
                __syncthreads();
                double2 *t = src;
                src = dst;
                dst = t;
            }
        }
        for (int e = threadIdx.x; e < nb * M; e += kBlock) {
            int b, m;
            if (S > 1) {
                b = e % nb;
                m = e / nb;
            } else {
                m = e % M;
                b = e / M;
            }
            const long long sub = s0 + b;
            const long long outer = sub / S, inner = sub - outer * S;
            const double2 v = src[b * M + m];
            out[outer * (long long)M * S + inner + (long long)m * S] =
                make_double2(v.x * scale, v.y * scale);
        }
    }
}

// Radices of N in stage order: fours first, then twos, then odd primes.
DftPlan make_plan(int N)
{
    DftPlan p{};
    p.N = N;
    int rest = N;
    while (rest % 4 == 0 && p.nr < kMaxRadices) {
        p.radix[p.nr++] = 4;
        rest /= 4;
    }
    while (rest % 2 == 0 && p.nr < kMaxRadices) {
        p.radix[p.nr++] = 2;
        rest /= 2;
    }
    for (int f = 3; rest > 1 && p.nr < kMaxRadices; f += 2)
        while (rest % f == 0 && p.nr < kMaxRadices) {
            p.radix[p.nr++] = f;
            rest /= f;
        }
    if (rest > 1) p.nr = 0;  // more factors than stages (cannot happen for N <= 1024)
    return p;
}

}  // namespace

hipError_t launch_dft(int n, int N, const double *in, double *out, int inverse, hipStream_t s)
{
    if (n < 1 || N < 1 || N > kDftMaxN) return hipErrorInvalidValue;
    long long D = 1;
    for (int t = 0; t < n; ++t) D *= N;
    if (N == 1) {  // nothing to transform: out = in (1/D = 1)
        if (in != out) return hipMemcpyAsync(out, in, sizeof(double2) * D, hipMemcpyDeviceToDevice, s);
        return hipSuccess;
    }
    const DftPlan plan = make_plan(N);
    if (plan.nr == 0) return hipErrorInvalidValue;
    // passes from the last axis: as many axes per pass as fit in LDS (two
    // buffers of B sub-grids beside the N twiddles)
    const long long room = (kDftLdsEntries - N) / 2;
    int t1 = n;
    bool first = true;
    while (t1 > 0) {
        int na = 1;
        long long M = N;
        while (t1 - na > 0 && M * N <= room) {
            M *= N;
            ++na;
        }
        const int t0 = t1 - na;
        long long S = 1;
        for (int t = t1; t < n; ++t) S *= N;
        const long long subs = D / M;
        long long Bl = std::max<long long>(1, std::min<long long>(room / M, subs));
        if (S > 1 && Bl > 4) Bl &= ~3LL;  // runs of whole 64-byte pieces across lanes
        const int B = (int)Bl;
        const size_t lds = sizeof(double2) * ((size_t)N + 2 * (size_t)B * M);
        const int grid = (int)std::min<long long>(8192, (subs + B - 1) / B);
        const double scale = (first && !inverse) ? 1.0 / (double)D : 1.0;
        hipLaunchKernelGGL(k_dft_pass, dim3(grid), dim3(kBlock), lds, s, plan, na, (int)M, S, subs,
                           B, inverse, scale, reinterpret_cast<const double2 *>(first ? in : out),
                           reinterpret_cast<double2 *>(out));
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        first = false;
        t1 = t0;
    }
    return hipSuccess;
}

}  // namespace qp
