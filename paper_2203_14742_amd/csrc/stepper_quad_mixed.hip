// Mixed-precision instances of the quad-lane persistent stepper: FP32 steps,
// then FP64 steps from the FP32 floor to the tolerance, in one launch
// (n = 32: one species per lane; n = 64: both species per lane, the FP32
// phase with the V-form divisor; the library's default shapes).
#include "stepper_quad.hpp"

namespace cil {

int launch_quad_mixed(int n, int nl, const DevSolve *S, const int *list, float *state, double *state64,
                      const float *tab32, const double *tab64, int model, double dt, const PersistArgs &pa32,
                      const PersistArgs &pa64, long long *switch_step, hipStream_t st)
{
    if (n == 32)
        hipLaunchKernelGGL((k_fused_q_mixed<32, 1, false, false>), dim3(nl), dim3(256), 0, st, S, list, state, state64,
                           tab32, tab64, model, dt, pa32, pa64, switch_step);
    else if (n == 64)
        hipLaunchKernelGGL((k_fused_q_mixed<64, 2, true, false>), dim3(nl), dim3(256), 0, st, S, list, state, state64,
                           tab32, tab64, model, dt, pa32, pa64, switch_step);
    else
        return CIL_EUNSUPPORTED;
    return CIL_OK;
}

}  // namespace cil
