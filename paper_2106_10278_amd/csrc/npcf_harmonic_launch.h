// Launch of the harmonic stage for one dimension.  The order l_max is a
// template parameter of the kernel, so a runtime l_max selects an instance.
#pragma once
#include "npcf_harmonic_impl.h"

namespace npcf {
namespace harm {

// persistent grid of the staging kernel: 8 blocks of 4 waves per CU, no more
// blocks than rows / 4
inline int stage_grid(int ncu, int nrows)
{
    int grid = ncu * 8;
    const int64_t need = ((int64_t)nrows + 3) / 4;
    if (grid > need) grid = (int)(need > 1 ? need : 1);
    return grid;
}

template <int D, int L, int LMAX>
hipError_t launch_l(int l, const HarmArgs &a, int ncu, hipStream_t s)
{
    if (l == L) return launch_dl<D, L>(a, stage_grid(ncu, a.nrows), s);
    if constexpr (L < LMAX) return launch_l<D, L + 1, LMAX>(l, a, ncu, s);
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
