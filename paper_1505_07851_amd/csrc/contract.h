// Helpers of the per-pair contraction kernels that read the V / V' partial sums of the
// pair-side passes (laid out [point chunk][tuv][slot]).
#pragma once
#include <cstddef>

// sum of p[c * stride] over the chunks c < nch, added in chunk order (so the bits do not depend
// on how the loads are grouped); four loads are in flight per step
__device__ __forceinline__ double chunk_sum(const double *__restrict__ p, size_t stride, int nch) {
    double s = 0.0;
    int c = 0;
    for (; c + 4 <= nch; c += 4) {
        const double a0 = p[(size_t)c * stride], a1 = p[(size_t)(c + 1) * stride];
        const double a2 = p[(size_t)(c + 2) * stride], a3 = p[(size_t)(c + 3) * stride];
        s += a0;
        s += a1;
        s += a2;
        s += a3;
    }
    for (; c < nch; ++c) s += p[(size_t)c * stride];
    return s;
}
