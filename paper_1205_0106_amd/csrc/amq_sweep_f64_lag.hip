// amq_sweep_f64_lag.hip — binary64 sweep kernels, weighted Laguerre basis.
#include "amq_sweep.h"

namespace amq {

const void *sweep_table_f64_lag(int ppt, int degree, int kind)
{
    return sweep_table<double, true>(ppt, degree, kind);
}

}  // namespace amq
