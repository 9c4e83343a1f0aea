// FP32 instances of the quad-lane persistent stepper (n = 32, 64, 128).
#include "stepper_quad.hpp"

namespace cil {

int launch_quad_f32(int n, int shape, int nl, const DevSolve *S, const int *list, float *state, const float *tables,
                    int model, double dt, const PersistArgs &pa, hipStream_t st)
{
    if (n == 32) launch_q<float, 32>(shape, nl, S, list, state, tables, model, dt, pa, st);
    else if (n == 64) launch_q<float, 64>(shape, nl, S, list, state, tables, model, dt, pa, st);
    else if (n == 128) launch_q<float, 128>(shape, nl, S, list, state, tables, model, dt, pa, st);
    else return CIL_EUNSUPPORTED;
    return CIL_OK;
}

}  // namespace cil
