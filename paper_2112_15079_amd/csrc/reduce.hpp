// Fixed-order sum of chunk partials, shared by the step epilogues and the
// adjoint's reduction.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nb {

// Element ii of the planes part[c * stride + ii], c < C, summed by a group of
// GS consecutive threads: thread `sub` adds chunks sub, sub + GS, ... in
// ascending order, then the group's first thread adds the GS sub-sums in sub
// order.  The order is fixed, so the result is deterministic; the value is
// complete in the sub == 0 thread only.  Loads go out in batches of B (24
// with four threads per element, so up to 96 partials arrive in one round
// trip; 8 with one).
template <int GS>
__device__ __forceinline__ double chunk_sum(const double* __restrict__ part, int C,
                                            int64_t stride, int64_t ii, int sub, bool live)
{
    constexpr int B = GS == 1 ? 8 : 96 / GS;
    double a = 0.0;
    if (live) {
        for (int c0 = sub; c0 < C; c0 += GS * B) {
            double v[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int c = c0 + u * GS;
                v[u] = (c < C) ? part[(int64_t)c * stride + ii] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < B; ++u)
                if (c0 + u * GS < C) a += v[u];
        }
    }
    if (GS > 1) {
        double total = a;
        const int lane = threadIdx.x & 63;
#pragma unroll
        for (int g = 1; g < GS; ++g) {
            const double o = __shfl(a, lane + g, 64);
            if (sub == 0) total += o;
        }
        a = total;
    }
    return a;
}

}  // namespace nb
