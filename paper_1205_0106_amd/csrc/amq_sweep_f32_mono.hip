// amq_sweep_f32_mono.hip — binary32-bulk sweep kernels, monomial basis.
#include "amq_sweep.h"

namespace amq {

const void *sweep_table_f32_mono(int ppt, int degree, int kind)
{
    return sweep_table<float, false>(ppt, degree, kind);
}

}  // namespace amq
