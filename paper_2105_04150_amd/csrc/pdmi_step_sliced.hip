// pdmi_step_sliced.hip -- launcher of the sliced-mapping step kernels (FP64).
#include "pdmi_step.h"

namespace pdmi {

hipError_t launch_step(const StepArgs& a, int lanes, int mode, bool stiff, bool ext, hipStream_t s)
{
    if (a.nslices <= 0) return hipSuccess;
    switch (lanes) {
    case 1: return ext ? launch_step_g<1, true>(a, mode, stiff, s) : launch_step_g<1, false>(a, mode, stiff, s);
    case 4: return ext ? launch_step_g<4, true>(a, mode, stiff, s) : launch_step_g<4, false>(a, mode, stiff, s);
    case 16: return ext ? launch_step_g<16, true>(a, mode, stiff, s) : launch_step_g<16, false>(a, mode, stiff, s);
    case 64: return ext ? launch_step_g<64, true>(a, mode, stiff, s) : launch_step_g<64, false>(a, mode, stiff, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace pdmi
