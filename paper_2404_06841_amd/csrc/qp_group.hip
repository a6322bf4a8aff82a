// Grouped stiffness products of the FP32-IR steps: one launch serves the
// plane-tile products of several problems (scalar coefficient, d = 2 or 3,
// all right-hand sides of each problem), each workgroup as one of its
// problem's workgroups.  The kernel bodies are those of qp_matvec_kernels.h.
#include "qp_matvec_kernels.h"

namespace qp {
namespace {

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

hipError_t launch_group_matvec(int prec, int d, bool real, int total, int gpmax,
                               const GroupEntry *E, const int *owner, hipStream_t s)
{
    if (total < 1 || gpmax < 4 || gpmax > ((kMaxG + 3) & ~3)) return hipErrorInvalidValue;
    if (prec == F32) return grp_plane_d<float, EPI_ALPHA>(d, real, total, gpmax, E, owner, s);
    return grp_plane_d<double, EPI_RESID>(d, real, total, gpmax, E, owner, s);
}

}  // namespace qp
