// Grouped stiffness products of the FP32-IR steps: one launch serves the
// plane-tile products of several problems (scalar coefficient, d = 2 or 3,
// all right-hand sides of each problem), each workgroup as one of its
// problem's workgroups.  The kernel bodies are those of qp_matvec_kernels.h.
//
// Also the static scratch array of the grouped calls that allocate nothing
// (qp_homogenized_grouped_noalloc): the group table, the owner arrays and the
// poll words live in `scratch`, one copy per device, held until the process
// ends.  Host code never names the array in a launch or a copy: it takes the
// device address from group_scratch(), looked up once per device.
#include <mutex>

#include "qp_matvec_kernels.h"

namespace qp {

static __device__ __align__(256) unsigned char scratch[kGroupScratchBytes];

namespace {

// Done bits of the group's problems (see launch_group_done).
__global__ void k_group_done(int G, int K, const GroupEntry *__restrict__ ents,
                             uint32_t *__restrict__ words)
{
    const int nw = (G + 31) / 32;
    for (int w = threadIdx.x; w < nw; w += blockDim.x) {
        uint32_t bits = 0;
        for (int b = 0; b < 32; ++b) {
            const int i = w * 32 + b;
            if (i >= G) break;
            bool done = true;
            for (int k = 0; k < K; ++k) done = done && ents[i].st[k].done != 0;
            bits |= done ? (1u << b) : 0u;
        }
        words[w] = bits;
    }
}

template <typename T, int EPI, int DT, bool REAL>
hipError_t grp_plane(int total, int gpmax, const GroupEntry *E, const int *owner, hipStream_t s)
{
    const size_t lds = sizeof(int2) * kWave * (size_t)gpmax +
                       (size_t)kWaves * gpmax * sizeof(PlaneRec<T, DT, false>);
    hipLaunchKernelGGL((k_matvec_plane_grp<T, DT, EPI, REAL, DT>), dim3(total), dim3(kBlock), lds, s,
                       E, owner);
    return hipGetLastError();
}

template <typename T, int EPI>
hipError_t grp_plane_d(int d, bool real, int total, int gpmax, const GroupEntry *E, const int *owner,
                       hipStream_t s)
{
    if (d == 2)
        return real ? grp_plane<T, EPI, 2, true>(total, gpmax, E, owner, s)
                    : grp_plane<T, EPI, 2, false>(total, gpmax, E, owner, s);
    if (d == 3)
        return real ? grp_plane<T, EPI, 3, true>(total, gpmax, E, owner, s)
                    : grp_plane<T, EPI, 3, false>(total, gpmax, E, owner, s);
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_group_done(int G, int K, const GroupEntry *E, uint32_t *words, hipStream_t s)
{
    if (G < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_group_done, dim3(1), dim3(kBlock), 0, s, G, K, E, words);
    return hipGetLastError();
}

hipError_t group_scratch(int device, void **ptr, size_t *bytes)
{
    constexpr int kDevices = 64;
    static std::mutex mu;
    static void *addr[kDevices] = {};
    if (device < 0 || device >= kDevices || !ptr || !bytes) return hipErrorInvalidValue;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void *a = nullptr;
        e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
        if (cur != device) {
            const hipError_t r = hipSetDevice(cur);
            if (e == hipSuccess) e = r;
        }
        if (e != hipSuccess) return e;
        if (!a) return hipErrorInvalidSymbol;
        addr[device] = a;
    }
    *ptr = addr[device];
    *bytes = kGroupScratchBytes;
    return hipSuccess;
}

hipError_t launch_group_matvec(int prec, int d, bool real, int total, int gpmax,
                               const GroupEntry *E, const int *owner, hipStream_t s)
{
    if (total < 1 || gpmax < 4 || gpmax > ((kMaxG + 3) & ~3)) return hipErrorInvalidValue;
    if (prec == F32) return grp_plane_d<float, EPI_ALPHA>(d, real, total, gpmax, E, owner, s);
    return grp_plane_d<double, EPI_RESID>(d, real, total, gpmax, E, owner, s);
}

}  // namespace qp
