// Discrete Fourier transforms on the collocation grid T_N^n (Sec. 2.3): the
// discrete Fourier-Bohr coefficients of sampled parent functions,
//   forward:  out_k = (1/D) sum_{j in [0,N)^n} in_j exp(-2 pi i k.j / N),
//   inverse:  out_j = sum_k in_k exp(+2 pi i k.j / N),
// both indexed by the storage order of Sec. 3.1.2 (digit k mod N, first axis
// slowest), which is the sample order of the grid y_j = 2 pi j / N.
//
// One launch per axis: a workgroup loads whole lines (the N entries that
// differ only in that axis' digit) into LDS and writes each output entry as
// a direct sum over the line with twiddles exp(-+2 pi i ((j k) mod N) / N)
// from an FP64 table (the product j k is reduced exactly in integers), so
// any N works and the error grows like N eps per axis.  The first pass reads
// `in`; the later passes transform `out` in place (every workgroup owns
// whole lines).  Consecutive lines of an axis are adjacent in memory, and
// the lanes of a workgroup take consecutive lines, so loads and stores
// coalesce across lanes for every axis.
#include <algorithm>

#include "qp_device.h"

namespace qp {
namespace {

constexpr int kDftMaxN = 1024;  // line length held in LDS

__global__ __launch_bounds__(kBlock) void k_dft_axis(int N, int stride, int lines, int lpb,
                                                     int inverse, double scale,
                                                     const double2 *__restrict__ in,
                                                     double2 *__restrict__ out)
{
    extern __shared__ double2 s_dft[];  // twiddles (N), then lpb lines of N
    double2 *tw = s_dft;
    double2 *ln = s_dft + N;
    const double sgn = inverse ? 1.0 : -1.0;
    for (int j = threadIdx.x; j < N; j += kBlock) {
        double sn, cs;
        sincospi(2.0 * (double)j / (double)N, &sn, &cs);
        tw[j] = make_double2(cs, sgn * sn);
    }
    for (int l0 = blockIdx.x * lpb; l0 < lines; l0 += gridDim.x * lpb) {
        const int nl = min(lpb, lines - l0);
        // element (line l0 + l, position j): line L = outer * stride + inner
        // starts at outer * N * stride + inner, steps by stride
        for (int e = threadIdx.x; e < nl * N; e += kBlock) {
            const int l = e % nl, j = e / nl;
            const long long L = (long long)l0 + l;
            const long long outer = L / stride, inner = L - outer * stride;
            const long long at = outer * (long long)N * stride + inner + (long long)j * stride;
            ln[l * N + j] = in[at];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < nl * N; e += kBlock) {
            const int l = e % nl, k = e / nl;
            const double2 *x = ln + l * N;
            double ar = 0.0, ai = 0.0;
            int idx = 0;  // (j k) mod N, advanced by k per step
            for (int j = 0; j < N; ++j) {
                const double2 w = tw[idx];
                ar += x[j].x * w.x - x[j].y * w.y;
                ai += x[j].x * w.y + x[j].y * w.x;
                idx += k;
                idx -= (idx >= N) ? N : 0;
            }
            const long long L = (long long)l0 + l;
            const long long outer = L / stride, inner = L - outer * stride;
            const long long at = outer * (long long)N * stride + inner + (long long)k * stride;
            out[at] = make_double2(ar * scale, ai * scale);
        }
        __syncthreads();  // the LDS lines are reloaded next
    }
}

}  // namespace

hipError_t launch_dft(int n, int N, const double *in, double *out, int inverse, hipStream_t s)
{
    if (n < 1 || N < 1 || N > kDftMaxN) return hipErrorInvalidValue;
    long long D = 1;
    for (int t = 0; t < n; ++t) D *= N;
    const int lines = (int)(D / N);
    // lines per workgroup: enough lanes for coalescing, within 64 KB of LDS
    int lpb = std::max(1, kBlock / N);
    while (lpb > 1 && (size_t)(lpb + 1) * N * sizeof(double2) > 65536) lpb /= 2;
    const size_t lds = (size_t)(lpb + 1) * N * sizeof(double2);
    const int grid = (int)std::min<long long>(8192, (lines + lpb - 1) / lpb);
    long long stride = D / N;  // axis 0 is the slowest
    for (int t = 0; t < n; ++t) {
        const double scale = (inverse || t > 0) ? 1.0 : 1.0 / (double)D;
        hipLaunchKernelGGL(k_dft_axis, dim3(grid), dim3(kBlock), lds, s, N, (int)stride, lines, lpb,
                           inverse, scale,
                           reinterpret_cast<const double2 *>(t == 0 ? in : out),
                           reinterpret_cast<double2 *>(out));
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        stride /= N;
    }
    return hipSuccess;
}

}  // namespace qp
