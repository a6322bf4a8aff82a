// Stiffness product entry points for a diagonal coefficient diag(a_1..a_d)
// (App. D): the kernels of qp_matvec_kernels.h with per-component weights
// sum_l Ahat^l_m (P k)_l (P j)_l.  A translation unit of its own, so the two
// coefficient kinds compile in parallel.
#include "qp_matvec_kernels.h"

namespace qp {

hipError_t launch_matvec_diag(int prec, int epi, int K, const Table *tab, const Table &ht,
                              const ModeRec *recs, const void *urec, const void *upku,
                              const void *x, void *y, const double *f, const float *M32,
                              const Parts &parts, State *st, int *exec, hipStream_t s, hipEvent_t ev0,
                              hipEvent_t ev1)
{
    return matvec_entry<true>(prec, epi, K, tab, ht, recs, urec, upku, x, y, f, M32, parts, st,
                              exec, s, ev0, ev1);
}

hipError_t launch_unit_records_diag(int prec, const Table *tab, const Table &ht,
                                    const ModeRec *recs, void *urec, void *upku, hipStream_t s)
{
    return unit_records_entry<true>(prec, tab, ht, recs, urec, upku, s);
}

}  // namespace qp
