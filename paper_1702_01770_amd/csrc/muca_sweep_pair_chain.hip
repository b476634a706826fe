// Sweep kernel variants with chain moves (pivots and rigid chain rotations after every sweep);
// the device code is shared with muca_sweep_pair.hip.
#include "muca_sweep_pair_impl.h"

namespace muca {

hipError_t launch_sweep_pair_chain(const SweepArgs &a, bool fp64, int group, int slots,
                                   bool periodic, int n_items, int waves, size_t lds,
                                   long long n_sweeps, hipStream_t st) {
    return launch_pair_all<true>(a, fp64, group, slots, periodic, n_items, waves, lds, n_sweeps,
                                 st);
}

}  // namespace muca
