// pdmi_step_staged_f32.hip -- launcher of the staged-mapping step kernels, FP32 bond arithmetic.
#include "pdmi_step.h"

namespace pdmi {

hipError_t launch_step_staged_f32(const StepArgs& a, int mode, int split, bool ext, hipStream_t s)
{
    if (a.nslices <= 0) return hipSuccess;
    return ext ? launch_staged_n<true, true>(a, mode, split, s) : launch_staged_n<true, false>(a, mode, split, s);
}

}  // namespace pdmi
