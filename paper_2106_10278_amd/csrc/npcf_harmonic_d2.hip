// Instances of the harmonic-stage kernel for D = 2 (lmax 0..16).
#include "npcf_harmonic_launch.h"

namespace npcf {

hipError_t launch_harmonic_d2(int L, const HarmArgs &a, int grid, hipStream_t s)
{
    return harm::launch_l<2, 0, 16>(L, a, grid, s);
}

int harmonic_lds_bytes_d2(int L) { return harm::lds_l<2, 0, 16>(L); }

}  // namespace npcf
