// gs_kernels.hpp -- the per-group step of direct stiffness summation, shared
// by the single-problem launch (gs.hip) and the batched solver.
#pragma once

#include "internal.hpp"

namespace nbx {

// Group g: s = sum of v over the group's local indices in ascending order,
// then s (or 0 for a Dirichlet group when apply_mask) to every copy.
template <typename T>
__device__ __forceinline__ void dssum_group(int32_t g, const int32_t *__restrict__ off,
                                            const int32_t *__restrict__ idx,
                                            const uint8_t *__restrict__ gflag,
                                            T *__restrict__ v, int apply_mask)
{
    const int32_t b = off[g], e = off[g + 1];
    T s = 0;
    for (int32_t q = b; q < e; ++q) s += v[idx[q]];
    if (apply_mask && gflag[g]) s = 0;
    for (int32_t q = b; q < e; ++q) v[idx[q]] = s;
}

}  // namespace nbx
