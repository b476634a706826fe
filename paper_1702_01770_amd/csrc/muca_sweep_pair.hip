// Multicanonical Metropolis sweep, several walkers per wavefront (CDNA4, gfx950).
//
// Same algorithm and random streams as k_sweep (muca_sweep.hip); this variant packs 64 / G
// walkers of one system into a wave, G = 16, 32 or 64 lanes each (a group), so the serial part of
// a trial move (proposal, acceptance test, bookkeeping) is shared by up to four Markov chains; the
// mixed instance (G = 0) gives every wave its own G, so one launch can run the longest chains on
// whole waves and the shortest four to a wave.  Bead j of a walker lives in lane (j mod G) of its
// group, slot j / G.  Values that are uniform within a group (bead index, energy, bin, ...) are
// plain VGPRs.  The coordinates live in LDS only: each group reads "its" moved bead, the
// neighbours and its lanes' own beads there with ordinary LDS loads, and an accepted move is
// written by all lanes of its group.
// ln W (Eq. 8) is continuous and linear inside each bin, so LDS holds its values at the K + 1 bin
// edges (8 bytes per bin) and a move reads the two edges of its bin with one ds_read2; the
// runtime uses this kernel only for weights that are continuous (the Berg recursion keeps them
// so).  That leaves room for a private 32-bit histogram per system in LDS, counted run-length
// encoded (one LDS atomic whenever a walker changes bin) and added to the device histogram once
// per launch.
//
// This translation unit holds the variants without chain moves, the LDS size and the dispatch.
#include "muca_sweep_pair_impl.h"

namespace muca {

size_t sweep_pair_lds_bytes(long long bins_total, int n_sys, int n_waves, int group, int slots) {
    const size_t stage = (size_t)n_waves * pair_slab_stage(group);
    const size_t coord = (size_t)n_waves * pair_slab_coord(group, slots);
    return 2 * sizeof(double2) * kMaxTypes * kMaxTypes + sizeof(double) * kAngcEntries +
           sizeof(StagedMove) * stage + sizeof(double) * kMaxTypes * kMaxTypes + sizeof(double) * coord +
           sizeof(double) * (size_t)(bins_total + n_sys) + sizeof(unsigned int) * (size_t)bins_total +
           sizeof(int) * (size_t)n_sys * kMaxBeads;
}

hipError_t launch_sweep_pair(const SweepArgs &a, bool fp64, int group, int slots, bool periodic,
                             int n_items, int waves, size_t lds, long long n_sweeps,
                             hipStream_t st) {
    if (a.pivot_per_sweep > 0 || a.rotate_per_sweep > 0)
        return launch_sweep_pair_chain(a, fp64, group, slots, periodic, n_items, waves, lds,
                                       n_sweeps, st);
    return launch_pair_all<false>(a, fp64, group, slots, periodic, n_items, waves, lds, n_sweeps,
                                  st);
}

}  // namespace muca
