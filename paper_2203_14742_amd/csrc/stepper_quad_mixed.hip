// Mixed-precision instances of the quad-lane persistent stepper: FP32 steps,
// then from the FP32 floor to the tolerance either FP64 steps or the
// refinement form (FP64 state, FP32 correction steps), in one launch or in
// two (n = 32: one species per lane; n = 64: both species per lane, the FP32
// phase with the V-form divisor; the library's default shapes).  One kernel
// per model.
#include "stepper_quad.hpp"

namespace cil {

namespace {

template <int N, int SPL, bool VF32, bool RF>
void launch_mixed(int model, int nl, const DevSolve *S, const int *list, float *state, double *state64,
                  const float *tab32, const double *tab64, double dt, const PersistArgs &pa32, const PersistArgs &pa64,
                  long long *switch_step, int mode, hipStream_t st)
{
    dispatch_model(model, [&](auto MD) {
        hipLaunchKernelGGL((k_fused_q_mixed<decltype(MD)::value, N, SPL, VF32, false, RF>), dim3(nl),
                           dim3((8 / SPL) * N), 0, st, S, list, state, state64, tab32, tab64, dt, pa32, pa64,
                           switch_step, mode);
    });
}

}  // namespace

int launch_quad_mixed(int n, int nl, const DevSolve *S, const int *list, float *state, double *state64,
                      const float *tab32, const double *tab64, int model, double dt, const PersistArgs &pa32,
                      const PersistArgs &pa64, long long *switch_step, int refine, int mode, hipStream_t st)
{
    if (n == 32 && refine)
        launch_mixed<32, 1, false, true>(model, nl, S, list, state, state64, tab32, tab64, dt, pa32, pa64,
                                         switch_step, mode, st);
    else if (n == 32)
        launch_mixed<32, 1, false, false>(model, nl, S, list, state, state64, tab32, tab64, dt, pa32, pa64,
                                          switch_step, mode, st);
    else if (n == 64 && refine)
        launch_mixed<64, 2, true, true>(model, nl, S, list, state, state64, tab32, tab64, dt, pa32, pa64,
                                        switch_step, mode, st);
    else if (n == 64)
        launch_mixed<64, 2, true, false>(model, nl, S, list, state, state64, tab32, tab64, dt, pa32, pa64,
                                         switch_step, mode, st);
    else
        return CIL_EUNSUPPORTED;
    return CIL_OK;
}

}  // namespace cil
