// Stiffness product entry points on Hermitian half storage (real scalar
// coefficient, odd N, plane tiles): the plane-tile kernels of
// qp_matvec_kernels.h with the half-storage gathers and stores.  A
// translation unit of its own, so it compiles beside the full-storage ones.
#include "qp_matvec_kernels.h"

namespace qp {

hipError_t launch_matvec_tiled_half(int prec, int epi, int K, const Table *tab, const Table &ht,
                                    const ModeRec *recs, const void *urec, const void *upku,
                                    const void *x, void *y, const double *f, const float *M32,
                                    const Parts &parts, State *st, int *exec, hipStream_t s,
                                    hipEvent_t ev0, hipEvent_t ev1)
{
    return matvec_half_entry(prec, epi, K, tab, ht, recs, urec, upku, x, y, f, M32, parts, st, exec,
                             s, ev0, ev1);
}

hipError_t launch_unit_records_half(int prec, const Table *tab, const Table &ht,
                                    const ModeRec *recs, void *urec, void *upku, hipStream_t s)
{
    if (!ht.half || ht.tile_s <= 1) return hipErrorInvalidValue;
    return prec == F64 ? unit_records_half<double>(tab, ht, recs, urec, upku, s)
                       : unit_records_half<float>(tab, ht, recs, urec, upku, s);
}

}  // namespace qp
