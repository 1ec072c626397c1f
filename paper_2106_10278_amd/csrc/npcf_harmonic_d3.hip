// Instances of the harmonic-stage kernel for D = 3 (lmax 0..10).
#include "npcf_harmonic_launch.h"

namespace npcf {

hipError_t launch_harmonic_d3(int L, const HarmArgs &a, int grid, hipStream_t s)
{
    return harm::launch_l<3, 0, 10>(L, a, grid, s);
}

int harmonic_lds_bytes_d3(int L) { return harm::lds_l<3, 0, 10>(L); }

}  // namespace npcf
