// Instances of the harmonic-stage kernel for D = 4 (lmax 0..6).
#include "npcf_harmonic_launch.h"

namespace npcf {

hipError_t launch_harmonic_d4(int L, const HarmArgs &a, int grid, hipStream_t s)
{
    return harm::launch_l<4, 0, 6>(L, a, grid, s);
}

int harmonic_lds_bytes_d4(int L) { return harm::lds_l<4, 0, 6>(L); }

}  // namespace npcf
