// amq_sweep_f32_lag.hip — binary32-bulk sweep kernels, weighted Laguerre basis.
#include "amq_sweep.h"

namespace amq {

const void *sweep_table_f32_lag(int ppt, int degree, int kind)
{
    return sweep_table<float, true>(ppt, degree, kind);
}

}  // namespace amq
