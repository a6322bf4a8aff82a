// Stiffness product entry points for a scalar coefficient; a diagonal
// coefficient (App. D) is served by qp_matvec_diag.hip.  The kernels are in
// qp_matvec_kernels.h.
#include "qp_matvec_kernels.h"

namespace qp {

hipError_t launch_matvec(int prec, int epi, int K, const Table *tab, const Table &ht,
                         const ModeRec *recs, const void *urec, const void *upku, const void *x,
                         void *y, const double *f, const float *M32, const Parts &parts, State *st,
                         int *exec, hipStream_t s, hipEvent_t ev0,
                         hipEvent_t ev1)
{
    if (ht.half)
        return launch_matvec_tiled_half(prec, epi, K, tab, ht, recs, urec, upku, x, y, f, M32,
                                        parts, st, exec, s, ev0, ev1);
    if (ht.aniso)
        return launch_matvec_diag(prec, epi, K, tab, ht, recs, urec, upku, x, y, f, M32, parts, st,
                                  exec, s, ev0, ev1);
    return matvec_entry<false>(prec, epi, K, tab, ht, recs, urec, upku, x, y, f, M32, parts, st,
                               exec, s, ev0, ev1);
}

hipError_t launch_unit_records(int prec, const Table *tab, const Table &ht, const ModeRec *recs,
                               void *urec, void *upku, hipStream_t s)
{
    if (ht.half) return launch_unit_records_half(prec, tab, ht, recs, urec, upku, s);
    if (ht.aniso) return launch_unit_records_diag(prec, tab, ht, recs, urec, upku, s);
    return unit_records_entry<false>(prec, tab, ht, recs, urec, upku, s);
}

}  // namespace qp
