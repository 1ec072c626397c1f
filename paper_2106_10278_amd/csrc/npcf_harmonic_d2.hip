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

int harmonic_lds_bytes_d2(int L)
{
    switch (L) {
    case 0: return harm::lds_bytes<2, 0>();
    case 1: return harm::lds_bytes<2, 1>();
    case 2: return harm::lds_bytes<2, 2>();
    case 3: return harm::lds_bytes<2, 3>();
    case 4: return harm::lds_bytes<2, 4>();
    case 5: return harm::lds_bytes<2, 5>();
    case 6: return harm::lds_bytes<2, 6>();
    case 7: return harm::lds_bytes<2, 7>();
    case 8: return harm::lds_bytes<2, 8>();
    case 9: return harm::lds_bytes<2, 9>();
    case 10: return harm::lds_bytes<2, 10>();
    case 11: return harm::lds_bytes<2, 11>();
    case 12: return harm::lds_bytes<2, 12>();
    case 13: return harm::lds_bytes<2, 13>();
    case 14: return harm::lds_bytes<2, 14>();
    case 15: return harm::lds_bytes<2, 15>();
    case 16: return harm::lds_bytes<2, 16>();
    default: return -1;
    }
}

}  // namespace npcf
