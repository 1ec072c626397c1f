// Instantiations of the harmonic-stage kernel for D = 4 (lmax 0..6).
#include "npcf_harmonic_impl.h"

namespace npcf {

hipError_t launch_harmonic_d4(int L, const HarmArgs &a, int grid, hipStream_t s)
{
    switch (L) {
    case 0: return harm::launch_dl<4, 0>(a, grid, s);
    case 1: return harm::launch_dl<4, 1>(a, grid, s);
    case 2: return harm::launch_dl<4, 2>(a, grid, s);
    case 3: return harm::launch_dl<4, 3>(a, grid, s);
    case 4: return harm::launch_dl<4, 4>(a, grid, s);
    case 5: return harm::launch_dl<4, 5>(a, grid, s);
    case 6: return harm::launch_dl<4, 6>(a, grid, s);
    default: return hipErrorInvalidValue;
    }
}

int harmonic_lds_bytes_d4(int L)
{
    switch (L) {
    case 0: return harm::lds_bytes<4, 0>();
    case 1: return harm::lds_bytes<4, 1>();
    case 2: return harm::lds_bytes<4, 2>();
    case 3: return harm::lds_bytes<4, 3>();
    case 4: return harm::lds_bytes<4, 4>();
    case 5: return harm::lds_bytes<4, 5>();
    case 6: return harm::lds_bytes<4, 6>();
    default: return -1;
    }
}

}  // namespace npcf
