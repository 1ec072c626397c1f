// Instantiations of the harmonic-stage kernel for D = 3 (lmax 0..10).
#include "npcf_harmonic_impl.h"

namespace npcf {

hipError_t launch_harmonic_d3(int L, const HarmArgs &a, int grid, hipStream_t s)
{
    switch (L) {
    case 0: return harm::launch_dl<3, 0>(a, grid, s);
    case 1: return harm::launch_dl<3, 1>(a, grid, s);
    case 2: return harm::launch_dl<3, 2>(a, grid, s);
    case 3: return harm::launch_dl<3, 3>(a, grid, s);
    case 4: return harm::launch_dl<3, 4>(a, grid, s);
    case 5: return harm::launch_dl<3, 5>(a, grid, s);
    case 6: return harm::launch_dl<3, 6>(a, grid, s);
    case 7: return harm::launch_dl<3, 7>(a, grid, s);
    case 8: return harm::launch_dl<3, 8>(a, grid, s);
    case 9: return harm::launch_dl<3, 9>(a, grid, s);
    case 10: return harm::launch_dl<3, 10>(a, grid, s);
    default: return hipErrorInvalidValue;
    }
}

int harmonic_lds_bytes_d3(int L)
{
    switch (L) {
    case 0: return harm::lds_bytes<3, 0>();
    case 1: return harm::lds_bytes<3, 1>();
    case 2: return harm::lds_bytes<3, 2>();
    case 3: return harm::lds_bytes<3, 3>();
    case 4: return harm::lds_bytes<3, 4>();
    case 5: return harm::lds_bytes<3, 5>();
    case 6: return harm::lds_bytes<3, 6>();
    case 7: return harm::lds_bytes<3, 7>();
    case 8: return harm::lds_bytes<3, 8>();
    case 9: return harm::lds_bytes<3, 9>();
    case 10: return harm::lds_bytes<3, 10>();
    default: return -1;
    }
}

}  // namespace npcf
