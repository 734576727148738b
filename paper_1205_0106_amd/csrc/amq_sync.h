// amq_sync.h — device-wide waits and fixed-order reductions shared by the
// persistent sweep and the estimator kernels (gfx950).
#pragma once

#include "amq_internal.h"

namespace amq {

// ---------------------------------------------------------------------------
// Device-wide barrier with bounded waits.
//   sync[0]: arrival counter (monotone; barrier e completes at e*G arrivals)
//   sync[1]: last released barrier number
//   sync[2]: error flag (a wait ran out; every workgroup then exits)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t ld_agent(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0 only.  Returns false if the wait was abandoned (this wait ran out,
// or another did and raised the error word `err`).
__device__ inline bool wait_release(uint32_t *rel, uint32_t *err, uint32_t epoch, uint32_t limit)
{
    uint32_t it = 0;
    while (ld_agent(rel) < epoch) {
        if (ld_agent(err) != 0u) return false;
        if (++it > limit) {
            __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return true;
}

// Sum NV doubles over the workgroup in a fixed order (butterfly in each wave,
// then waves 0..3 in order).  Result valid in thread 0.
template <int NV>
__device__ __forceinline__ void group_sum(double (&v)[NV], double (*s_red)[32])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double x = v[q];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
        v[q] = x;
    }
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) s_red[wave][q] = v[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) v[q] = ((s_red[0][q] + s_red[1][q]) + s_red[2][q]) + s_red[3][q];
    }
}

// Last group: fixed-order sum of all partial slots into tot[0..NV-1] (LDS).
// Thread t owns component t % 32 of groups t/32, t/32 + 8, ...; its loads are
// issued in batches of 4 before any is consumed (one memory round trip per
// batch of 32 groups), then added in group order.
template <int NV>
__device__ void reduce_partials(const double *part, uint32_t G, double *tot, double (*s_red8)[32]);

// Two-level arrival (see the barrier block layout in amq_internal.h).  Group
// gid stores its partial and arrives at its team's counter; the team's last
// arriver sums the team's partials in member order into the team slot and
// arrives at the top counter; the top's last arriver sums the team slots in
// order into tot (LDS).  Returns, in every thread, whether this group is the
// top-level last (then tot holds the totals).  At most team-size groups meet
// on one cache line, and the sums never depend on arrival order.
template <int NV>
__device__ inline bool arrive_tree(const double (&v)[NV], uint32_t gid, uint32_t G, double *part,
                            double *tpart, uint32_t *words, uint32_t epoch, double *tot,
                            double (*s_red8)[32], int *s_flag)
{
    const uint32_t TS = team_size(G), NT = (G + TS - 1) / TS;
    const uint32_t tau = gid / TS;
    const uint32_t t_first = tau * TS;
    const uint32_t t_count = min(TS, G - t_first);
    if (threadIdx.x == 0) {
        double *dst = part + (size_t)gid * kPartStride;
#pragma unroll
        for (int q = 0; q < NV; ++q) dst[q] = v[q];
        const uint32_t old = __hip_atomic_fetch_add(words + kSyncLine * (1 + tau), 1u, __ATOMIC_ACQ_REL,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        s_flag[0] = (old + 1u == epoch * t_count) ? 1 : 0;
    }
    __syncthreads();
    if (!s_flag[0]) return false;
    reduce_partials<NV>(part + (size_t)t_first * kPartStride, t_count, tot, s_red8);
    if (threadIdx.x == 0) {
        double *dst = tpart + (size_t)tau * kPartStride;
#pragma unroll
        for (int q = 0; q < NV; ++q) dst[q] = tot[q];
        const uint32_t old = __hip_atomic_fetch_add(words, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_flag[0] = (old + 1u == epoch * NT) ? 1 : 0;
    }
    __syncthreads();
    if (!s_flag[0]) return false;
    reduce_partials<NV>(tpart, NT, tot, s_red8);
    return true;
}

// Top-level last: publish epoch on every team's release line.
__device__ __forceinline__ void release_all(uint32_t *words, uint32_t G, uint32_t epoch)
{
    const uint32_t TS = team_size(G), NT = (G + TS - 1) / TS;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    for (uint32_t t = 0; t < NT; ++t)
        __hip_atomic_store(words + kSyncLine * (1 + kMaxTeams + t), epoch, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t *release_word(uint32_t *words, uint32_t G, uint32_t gid)
{
    return words + kSyncLine * (1 + kMaxTeams + gid / team_size(G));
}

template <int NV>
__device__ void reduce_partials(const double *part, uint32_t G, double *tot, double (*s_red8)[32])
{
    const int c = threadIdx.x & 31, sgrp = threadIdx.x >> 5;   // 8 groups of 32
    double v = 0.0;
    if (c < NV) {
        for (uint32_t g0 = sgrp; g0 < G; g0 += 8 * 4) {
            double buf[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t g = g0 + 8u * u;
                buf[u] = g < G ? part[(size_t)g * kPartStride + c] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) v += buf[u];
        }
    }
    s_red8[sgrp][c] = v;
    __syncthreads();
    if (threadIdx.x < NV) {
        double t = 0.0;
#pragma unroll
        for (int s = 0; s < 8; ++s) t += s_red8[s][threadIdx.x];
        tot[threadIdx.x] = t;
    }
    __syncthreads();
}

}  // namespace amq
