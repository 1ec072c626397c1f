// Instantiations of the harmonic-stage kernel for D = 2 (lmax 0..16).
#include "npcf_harmonic_impl.h"

namespace npcf {

hipError_t launch_harmonic_d2(int L, const HarmArgs &a, int grid, hipStream_t s)
{
    switch (L) {
    case 0: return harm::launch_dl<2, 0>(a, grid, s);
    case 1: return harm::launch_dl<2, 1>(a, grid, s);
    case 2: return harm::launch_dl<2, 2>(a, grid, s);
    case 3: return harm::launch_dl<2, 3>(a, grid, s);
    case 4: return harm::launch_dl<2, 4>(a, grid, s);
    case 5: return harm::launch_dl<2, 5>(a, grid, s);
    case 6: return harm::launch_dl<2, 6>(a, grid, s);
    case 7: return harm::launch_dl<2, 7>(a, grid, s);
    case 8: return harm::launch_dl<2, 8>(a, grid, s);
    case 9: return harm::launch_dl<2, 9>(a, grid, s);
    case 10: return harm::launch_dl<2, 10>(a, grid, s);
    case 11: return harm::launch_dl<2, 11>(a, grid, s);
    case 12: return harm::launch_dl<2, 12>(a, grid, s);
    case 13: return harm::launch_dl<2, 13>(a, grid, s);
    case 14: return harm::launch_dl<2, 14>(a, grid, s);
    case 15: return harm::launch_dl<2, 15>(a, grid, s);
    case 16: return harm::launch_dl<2, 16>(a, grid, s);
    default: return hipErrorInvalidValue;
    }
}

int harmonic_lds_bytes_d2(int L, int nb)
{
    switch (L) {
    case 0: return harm::lds_bytes<2, 0>(nb);
    case 1: return harm::lds_bytes<2, 1>(nb);
    case 2: return harm::lds_bytes<2, 2>(nb);
    case 3: return harm::lds_bytes<2, 3>(nb);
    case 4: return harm::lds_bytes<2, 4>(nb);
    case 5: return harm::lds_bytes<2, 5>(nb);
    case 6: return harm::lds_bytes<2, 6>(nb);
    case 7: return harm::lds_bytes<2, 7>(nb);
    case 8: return harm::lds_bytes<2, 8>(nb);
    case 9: return harm::lds_bytes<2, 9>(nb);
    case 10: return harm::lds_bytes<2, 10>(nb);
    case 11: return harm::lds_bytes<2, 11>(nb);
    case 12: return harm::lds_bytes<2, 12>(nb);
    case 13: return harm::lds_bytes<2, 13>(nb);
    case 14: return harm::lds_bytes<2, 14>(nb);
    case 15: return harm::lds_bytes<2, 15>(nb);
    case 16: return harm::lds_bytes<2, 16>(nb);
    default: return -1;
    }
}

}  // namespace npcf
