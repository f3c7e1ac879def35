// asep_sweep_two_lane.hip -- instantiations of the sweep kernel for the
// two lane model (one translation unit per model so that they compile in parallel).
#include "asep_device.h"

namespace asep {

hipError_t launch_sweep_two_lane(const SweepKernel& k, const SimDesc& one, const SimDesc* descs,
                                   uint32_t n_desc, uint32_t grid, uint32_t block, size_t lds,
                                   hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
    return dev::launch_model<kTwoLane>(k, one, descs, n_desc, grid, block, lds, st, ev0, ev1);
}

}  // namespace asep
