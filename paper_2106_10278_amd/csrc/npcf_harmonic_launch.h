// Launch of the harmonic stage for one dimension.  The order l_max is a
// template parameter of the kernel, so a runtime l_max selects an instance.
#pragma once
#include "npcf_harmonic_impl.h"

namespace npcf {
namespace harm {

template <int D, int L, int LMAX>
hipError_t launch_l(int l, const HarmArgs &a, int grid, hipStream_t s)
{
    if (l == L) return launch_dl<D, L>(a, grid, s);
    if constexpr (L < LMAX) return launch_l<D, L + 1, LMAX>(l, a, grid, s);
    return hipErrorInvalidValue;
}

template <int D, int L, int LMAX>
int lds_l(int l)
{
    if (l == L) return lds_bytes<D, L>();
    if constexpr (L < LMAX) return lds_l<D, L + 1, LMAX>(l);
    return -1;
}

}  // namespace harm
}  // namespace npcf
