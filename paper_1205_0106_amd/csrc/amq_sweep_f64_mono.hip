// amq_sweep_f64_mono.hip — binary64 sweep kernels, monomial basis.
#include "amq_sweep.h"

namespace amq {

const void *sweep_table_f64_mono(int ppt, int degree, int kind)
{
    return sweep_table<double, false>(ppt, degree, kind);
}

}  // namespace amq
