#include "fused.h"

namespace mpc {

bool fused_supported(int, int, int, int) { return false; }
void fused_launch_shape(int, int, int, int, int* threads, size_t* lds) {
  *threads = 0;
  *lds = 0;
}
hipError_t fused_solve_f32(const AgentDesc*, int, int, int, int, int, Inputs<float>, SolverConsts,
                           int, int, State<float>, int, size_t, hipStream_t) {
  return hipErrorInvalidConfiguration;
}

}  // namespace mpc
