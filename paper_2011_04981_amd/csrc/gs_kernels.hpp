// gs_kernels.hpp -- the per-group step of direct stiffness summation, shared
// by the single-problem launch (gs.hip) and the batched solver.
#pragma once

#include "internal.hpp"

namespace nbx {

// Threads per workgroup of the exchange launches.  The largest workgroup
// measured best on the 32^3 brick at N = 10 (one FP64 pass 226 / 219 / 210 /
// 199 / 184 us at 64 / 128 / 256 / 512 / 1024 threads; FP64 solve 1.736 ->
// 1.690 s, FP16-G mixed solve 1.130 -> 1.086 s against 256): a CU then
// walks a longer contiguous run of groups, whose copies share lines.
constexpr int kGsThreads = 1024;

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
