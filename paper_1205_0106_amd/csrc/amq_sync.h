// amq_sync.h — device-wide waits and fixed-order reductions shared by the
// persistent sweep and the estimator kernels (gfx950).
#pragma once

#include "amq_internal.h"

namespace amq {

// threadIdx.x through an empty asm: a value the compiler cannot share across
// calls.  The helpers below run once per date inside the sweeps' date loops;
// with their per-lane indexes and addresses derived from it, those are
// recomputed at each call (a few instructions) instead of being hoisted out
// of the loop and held in registers, or spilled to scratch memory and
// reloaded on the date's critical path, in kernels whose registers hold
// path data.
__device__ __forceinline__ uint32_t tid_x()
{
    uint32_t t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

__device__ __forceinline__ uint32_t ld_agent(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A wave-uniform binary64 value moved to scalar registers.
__device__ __forceinline__ double uniform_f64(double x)
{
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ void raise_error(uint32_t *err)
{
    __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// x + (the value DPP control `CTRL` moves into this lane), binary64 through
// two 32-bit DPP moves.  Lanes outside ROW_MASK, or without a source lane,
// get an unspecified value: only lane 63 of the final sum is used, and it
// depends on none of them.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_add(double x)
{
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, ROW_MASK, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, ROW_MASK, 0xF, false);
    return x + __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Sum of x over the 64 lanes of a wave, valid in lane 63 (other lanes hold
// unspecified values), in a fixed order on the vector unit (DPP, no LDS
// round trips): neighbour swaps within quads, the half-row and row mirrors
// (every lane of a 16-lane row then holds the row sum), then row 2 into row 3
// (row_bcast:15) and row 1 into row 3 (row_bcast:31).
__device__ __forceinline__ double wave_sum(double x)
{
    x = dpp_add<0xB1, 0xF>(x);    // quad_perm [1,0,3,2]
    x = dpp_add<0x4E, 0xF>(x);    // quad_perm [2,3,0,1]
    x = dpp_add<0x141, 0xF>(x);   // row_half_mirror
    x = dpp_add<0x140, 0xF>(x);   // row_mirror
    x = dpp_add<0x142, 0xA>(x);   // row_bcast:15 into rows 1 and 3
    x = dpp_add<0x143, 0xC>(x);   // row_bcast:31 into rows 2 and 3
    return x;
}

// x(row 2i) + x(row 2i+1) in every lane of both rows (16-lane rows), and
// x(lane l mod 32) + x(lane l mod 32 + 32): gfx950's row-swapping permutes
// (v_permlane16_swap / v_permlane32_swap), lower operand first in every lane.
__device__ __forceinline__ double add_rows16(double x)
{
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)b, (uint32_t)b, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)(b >> 32), (uint32_t)(b >> 32), false, false);
    return __longlong_as_double((long long)(((uint64_t)hi[0] << 32) | lo[0])) +
           __longlong_as_double((long long)(((uint64_t)hi[1] << 32) | lo[1]));
}

__device__ __forceinline__ double add_halves32(double x)
{
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)b, (uint32_t)b, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(b >> 32), (uint32_t)(b >> 32), false, false);
    return __longlong_as_double((long long)(((uint64_t)hi[0] << 32) | lo[0])) +
           __longlong_as_double((long long)(((uint64_t)hi[1] << 32) | lo[1]));
}

// Sum NV doubles over a workgroup of WG threads in a fixed order (wave_sum
// in each wave, then the waves in order).  The last NU components are
// wave-uniform (a wave's total already, e.g. a ballot count): summed over the
// waves only.  s_red: LDS [WG / 64][32].  Result valid in thread 0.
template <int NV, int NU = 0, int WG = kWG>
__device__ __forceinline__ void group_sum(double (&v)[NV], double (*s_red)[32])
{
    const uint32_t tx = tid_x();
    const int lane = tx & 63, wave = tx >> 6;
#pragma unroll
    for (int q = 0; q < NV - NU; ++q) v[q] = wave_sum(v[q]);
    if (lane == 63) {
#pragma unroll
        for (int q = 0; q < NV; ++q) s_red[wave][q] = v[q];
    }
    __syncthreads();
    if (tx == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double t = s_red[0][q];
#pragma unroll
            for (int w = 1; w < WG / 64; ++w) t += s_red[w][q];
            v[q] = t;
        }
    }
}

// The same sum through LDS for groups with two waves per SIMD: every thread
// stores its NV - NU components ([8][WG] doubles at s_x), then component q's
// WG/8 threads each add 8 of them (stride WG/8, ascending) and reduce their
// partials on the vector unit (a 64-lane wave_sum, or the 32-lane half of it
// for WG = 256); the wave-uniform components go through s_red as in
// group_sum.  Fewer vector instructions than a DPP tree per component when
// NV - NU is large.  Result valid in thread 0.
template <int NV, int NU, int WG>
__device__ __forceinline__ void group_sum_lds(double (&v)[NV], double *s_x, double (*s_red)[32])
{
    const uint32_t tx = tid_x();
    constexpr int NC = NV - NU, TPC = WG / 8;
    static_assert(NC <= 8 && NV <= 32 && (TPC == 32 || TPC == 64), "component slots");
    const int tid = tx, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int q = 0; q < NC; ++q) s_x[q * WG + tid] = v[q];
    if (lane == 63) {
#pragma unroll
        for (int u = 0; u < NU; ++u) s_red[wave][NC + u] = v[NC + u];
    }
    __syncthreads();
    const int q = tid / TPC, l = tid % TPC;
    double acc = 0.0;
    if (q < NC) {
        double x[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i] = s_x[q * WG + l + i * TPC];
#pragma unroll
        for (int i = 0; i < 8; ++i) acc += x[i];
    }
    if (TPC == 64) {
        acc = wave_sum(acc);
        if (lane == 63 && q < NC) s_red[0][q] = acc;
    } else {
        acc = dpp_add<0xB1, 0xF>(acc);
        acc = dpp_add<0x4E, 0xF>(acc);
        acc = dpp_add<0x141, 0xF>(acc);
        acc = dpp_add<0x140, 0xF>(acc);
        acc = dpp_add<0x142, 0xA>(acc);   // lanes 31 and 63: their half-wave's sum
        if ((lane & 31) == 31 && q < NC) s_red[0][q] = acc;
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c] = s_red[0][c];
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            double t = s_red[0][NC + u];
#pragma unroll
            for (int w = 1; w < WG / 64; ++w) t += s_red[w][NC + u];
            v[NC + u] = t;
        }
    }
}

// Fixed-order sum of G partial slots (kPartStride doubles apart) into
// tot[0..NV-1] (LDS), by the whole workgroup.  Thread t owns component t % 32
// of groups t/32, t/32 + 8, ...; its loads are issued in batches of 4 before
// any is consumed, then added in group order.
template <int NV>
__device__ void reduce_partials(const double *part, uint32_t G, double *tot, double (*s_red8)[32])
{
    const uint32_t tx = tid_x();
    const int c = tx & 31, sgrp = tx >> 5;   // 8 groups of 32
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
    if (tx < NV) {
        double t = 0.0;
#pragma unroll
        for (int s = 0; s < 8; ++s) t += s_red8[s][tx];
        tot[tx] = t;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Device-wide fixed-order sum of NV doubles, every workgroup receiving the
// total (an all-gather of per-group partials; no group waits on another's
// release).
//
// Each group owns one row of RW 8-byte words in the parity-(epoch & 1) half
// of `rows` ([2][G][RW]).  Thread 0 stores the group's NV partials there with
// single-copy-atomic 8-byte stores, the two lowest mantissa bits of each word
// replaced by epoch & 3 (a change of at most 3 units in the last place, the
// same in every run), then bumps its team's arrival counter.  Wave 0 polls the
// team counters until the epoch is complete; then the whole group reads every
// row (lane c of each RW-lane slice reads word c, all loads of a batch issued
// before any is used), checks that every word carries this epoch's tag
// (re-reading if a store had not yet landed: the counter is only a hint, so no
// store needs to drain before it), and sums in a fixed order: each thread its
// rows in ascending order, then the lanes and waves of the group in a fixed
// tree.  Every group computes bitwise the same total.
//
// Above kFlatMaxGroups groups (every group reading every row would move
// G^2 rows per date), the last arriver of each team (from its counter's
// return value) first sums its team's rows in member order into a tagged
// team row; every group then polls the team rows' tags and sums the team
// rows in team order.
//
// Two parities suffice: a group writes the parity of epoch e + 2 only after
// epoch e + 1 is complete, and every group finished reading epoch e before
// publishing its e + 1 row.  A stale word left from epoch e - 2 carries a
// different tag.  The generation kernel zeroes the rows (tag 0) before each
// sweep, so words of an earlier sweep never match epochs 1..3, and epoch 4
// reads words rewritten at epoch 2.
//
// Waits are bounded by `limit` polls; on running out, or on seeing the error
// word raised by another group, returns false (the caller exits).
// v: valid in thread 0.  tot: LDS [>= NV], valid in every thread on return.
// s_flag: LDS [2 + WG / 64]; s_red: LDS [WG / 64][32].
// ---------------------------------------------------------------------------
// Fixed-order sum of rows [0, count) of `slots` (RW words each, tagged):
// lane c of each RW-lane slice reads word c, KB rows per thread in flight;
// every word must carry `tag`, else on_miss(attempt) is called by every
// thread (a collective wait that returns false to give up) and the rows are
// read again, at most `limit` times.  Each thread adds its rows in ascending
// order, then the group's lanes and waves in a fixed tree.  tot: LDS
// [>= NV], valid in every thread on true.
template <int NV, int RW, int WG, typename OnMiss>
__device__ inline bool sum_rows(const uint64_t *slots, uint32_t count, uint64_t tag, uint32_t *err,
                                uint32_t limit, double *tot, double (*s_red)[32], int *s_flag, OnMiss on_miss)
{
    const uint32_t tx = tid_x();
    static_assert(RW == 16 || RW == 32, "row width");
    constexpr int NW = WG / 64;
    constexpr uint32_t RP = WG / RW;    // rows per pass
    // passes per batch (loads in flight per thread; 512-thread groups hold
    // their cashflows and slab values in registers meanwhile).  The order in
    // which a thread adds its rows does not depend on it.
    constexpr int KB = WG >= 512 ? 8 : 16;
    const uint32_t c = tx % RW, rs = tx / RW;
    const int lane = tx & 63, wave = tx >> 6;
    uint32_t it = 0;
    for (;;) {
        double acc = 0.0;
        bool bad = false;
        for (uint32_t r0 = 0; r0 < count; r0 += KB * RP) {
            uint64_t w[KB];
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                const uint32_t r = r0 + rs + (uint32_t)k * RP;
                w[k] = (r < count && c < (uint32_t)NV)
                           ? __hip_atomic_load(slots + (size_t)r * RW + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                           : tag;
            }
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                bad |= (w[k] & 3u) != tag;
                acc += __longlong_as_double((long long)(w[k] & ~3ull));
            }
        }
        // lanes c, c + RW, ... of a wave hold the same component
        if (RW == 16) acc = add_rows16(acc);
        acc = add_halves32(acc);
        const bool wbad = __builtin_amdgcn_ballot_w64(bad) != 0;
        if (lane < RW) s_red[wave][lane] = acc;
        if (lane == 0) s_flag[1 + wave] = wbad ? 1 : 0;
        __syncthreads();
        bool anybad = false;
#pragma unroll
        for (int q = 0; q < NW; ++q) anybad |= s_flag[1 + q] != 0;
        if (!anybad) {
            if (tx < NV) {
                double t = 0.0;
#pragma unroll
                for (int q = 0; q < NW; ++q) t += s_red[q][tx];
                tot[tx] = t;
            }
            __syncthreads();
            return true;
        }
        if (++it > limit) {
            if (tx == 0) raise_error(err);
            return false;
        }
        if (!on_miss(it)) return false;
    }
}

// The default wait between reads of rows: a short sleep; false once another
// group has raised the error word.  Collective.
__device__ inline bool rows_backoff(uint32_t *err, int *s_flag)
{
    const uint32_t tx = tid_x();
    if (tx == 0) s_flag[0] = ld_agent(err) != 0u ? 1 : 0;
    __builtin_amdgcn_s_sleep(1);
    __syncthreads();
    return s_flag[0] == 0;
}

// Thread 0: store the NV values as a tagged row (single-copy-atomic words).
template <int NV>
__device__ __forceinline__ void put_row(uint64_t *row, const double *v, uint64_t tag)
{
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const uint64_t b = ((uint64_t)__double_as_longlong(v[q]) & ~3ull) | tag;
        __hip_atomic_store(row + q, b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Groups at or below this count read every group's row; above it, teams sum
// first (see allreduce).
constexpr uint32_t kFlatMaxGroups = 256;

// Publishing half of allreduce: thread 0 stores the group's row and bumps
// its team's counter; above kFlatMaxGroups the team's last arriver also sums
// its team's rows into the team row.  The caller may do independent work
// before the gathering half (allreduce_gather) with the same epoch.  Uses
// s_flag[1 + WG / 64] (the team-last flag), so that the gathering half's
// flags never overlap it.
template <int NV, int RW, int WG = kWG>
__device__ inline bool allreduce_publish(const double (&v)[NV], uint32_t gid, uint32_t G, uint64_t *rows,
                                         uint32_t *words, uint32_t *err, uint32_t epoch, uint32_t limit,
                                         double *tot, double (*s_red)[32], int *s_flag)
{
    const uint32_t tx = tid_x();
    static_assert(NV <= RW && RW <= 32 && (RW & (RW - 1)) == 0, "row width");
    const uint64_t tag = epoch & 3u;
    uint64_t *slots = rows + (size_t)(epoch & 1u) * G * RW;
    uint64_t *tslots = rows + (size_t)2 * G * RW + (size_t)(epoch & 1u) * kMaxTeams * RW;
    const uint32_t TS = team_size(G);
    const uint32_t tau = gid / TS;
    const bool flat = G <= kFlatMaxGroups;
    if (tx == 0) put_row<NV>(slots + (size_t)gid * RW, v, tag);
    if (flat) {
        // the counter's old value is not used: nothing waits for the round trip
        if (tx == 0)
            (void)__hip_atomic_fetch_add(words + kSyncLine * (1 + tau), 1u, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    } else {
        // team level: the team's last arriver sums its team's rows in member
        // order and publishes the team row (tagged like the group rows)
        if (tx == 0) {
            const uint32_t old = __hip_atomic_fetch_add(words + kSyncLine * (1 + tau), 1u, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
            s_flag[1 + WG / 64] = old + 1u == epoch * min(TS, G - tau * TS) ? 1 : 0;
        }
        __syncthreads();
        if (s_flag[1 + WG / 64]) {
            const uint32_t first = tau * TS;
            if (!sum_rows<NV, RW, WG>(slots + (size_t)first * RW, min(TS, G - first), tag, err, limit, tot, s_red,
                                      s_flag, [&](uint32_t) { return rows_backoff(err, s_flag); }))
                return false;
            if (tx == 0) put_row<NV>(tslots + (size_t)tau * RW, tot, tag);
        }
    }
    return true;
}

// Gathering half: wait until every group (or team) of `epoch` has published,
// then sum the rows in the fixed order into tot (LDS, every thread).  Flat:
// wave 0 waits on the team counters, then the rows are read (re-read until
// every word carries the tag).  With rows_first (a caller that did other
// work since publishing, so the rows usually all carry the tag already) the
// rows are read once before the counters, which saves their round trip.
// Teams: wave 0 waits on the team rows' tags, then the team rows are summed.
template <int NV, int RW, int WG = kWG>
__device__ inline bool allreduce_gather(uint32_t G, uint64_t *rows, uint32_t *words, uint32_t *err,
                                        uint32_t epoch, uint32_t limit, double *tot, double (*s_red)[32],
                                        int *s_flag, bool rows_first = false)
{
    const uint32_t tx = tid_x();
    const uint64_t tag = epoch & 3u;
    uint64_t *slots = rows + (size_t)(epoch & 1u) * G * RW;
    uint64_t *tslots = rows + (size_t)2 * G * RW + (size_t)(epoch & 1u) * kMaxTeams * RW;
    const uint32_t TS = team_size(G), NT = (G + TS - 1) / TS;
    const bool flat = G <= kFlatMaxGroups;
    auto poll = [&]() -> bool {
        if (tx < 64) {
            // flat: lane t < NT watches team t's counter; teams: lane t
            // watches team t's row (word 0 carries the epoch tag).
            // Wave-uniform exit.
            const uint32_t lane = tx;
            const uint32_t want = lane < NT ? min(TS, G - lane * TS) * epoch : 0u;
            uint32_t it = 0;
            bool ok = true;
            for (;;) {
                bool pending;
                if (flat) {
                    const uint32_t seen = lane < NT ? ld_agent(words + kSyncLine * (1 + lane)) : 0u;
                    pending = seen < want;
                } else {
                    const uint64_t w0 = lane < NT ? __hip_atomic_load(tslots + (size_t)lane * RW, __ATOMIC_RELAXED,
                                                                      __HIP_MEMORY_SCOPE_AGENT)
                                                  : tag;
                    pending = (w0 & 3u) != tag;
                }
                if (__builtin_amdgcn_ballot_w64(pending) == 0) break;
                if (ld_agent(err) != 0u) { ok = false; break; }
                if (++it > limit) { if (lane == 0) raise_error(err); ok = false; break; }
                __builtin_amdgcn_s_sleep(1);
            }
            if (lane == 0) s_flag[0] = ok ? 1 : 0;
        }
        __syncthreads();
        return s_flag[0] != 0;
    };
    const bool early = flat && rows_first;
    if (!early && !poll()) return false;
    return sum_rows<NV, RW, WG>(flat ? slots : tslots, flat ? G : NT, tag, err, limit, tot, s_red, s_flag,
                                [&](uint32_t attempt) {
                                    return (early && attempt == 1) ? poll() : rows_backoff(err, s_flag);
                                });
}

template <int NV, int RW, int WG = kWG>
__device__ inline bool allreduce(const double (&v)[NV], uint32_t gid, uint32_t G, uint64_t *rows,
                                 uint32_t *words, uint32_t *err, uint32_t epoch, uint32_t limit, double *tot,
                                 double (*s_red)[32], int *s_flag)
{
    return allreduce_publish<NV, RW, WG>(v, gid, G, rows, words, err, epoch, limit, tot, s_red, s_flag) &&
           allreduce_gather<NV, RW, WG>(G, rows, words, err, epoch, limit, tot, s_red, s_flag);
}

}  // namespace amq
