// amq_sweep.h — the persistent backward-induction kernels (Section V): per
// date in-the-money basis moments, a device-wide fixed-order reduction, an
// FP64 normal-equation solve, the exercise update and the FP64 discounted
// cashflow mean; single-option and many-option (batch) forms (gfx950).
#pragma once

#include "amq_math.h"
#include "amq_sync.h"

namespace amq {

// FP64 normal-equation solve for the p = D+1 coefficients from Hankel moments
// tot[0..2D] (sum of wA xs^q), tot[2D+1 .. 3D+1] (sum of wB xs^a pv) and the
// in-the-money count tot[3D+2].  Equilibrated Cholesky by one thread; L and
// w are registers where the kernel has room (registers are allocated in
// every lane, beside the resident cashflows), else LDS; a date with fewer in-the-money
// paths than p or a pivot below 1e-14 (on the unit-diagonal matrix) allows no
// exercise.  beta: [0..7] coefficients in the standardised basis (zero past
// p), [8] solved flag, [9] in-the-money count.  Branch-free (a rejected
// pivot takes the square root of 1 and clears the flag), so the independent
// square roots of the equilibration overlap.
template <int D, typename TT = const double *, typename LT = double (*)[8], typename WT = double *>
__device__ __forceinline__ void solve_date(TT tot, double *beta, LT L, WT w)
{
    constexpr int P = D + 1, NA = 2 * D + 1;
    const double n = rint(tot[NA + P]);
    bool ok = n >= (double)P;
    WT sc = w, rl = w + 8, y = w + 16, gam = w + 24;
#pragma unroll
    for (int i = 0; i < P; ++i) {
        const double d = tot[2 * i];
        ok = ok && (d > 0.0);
        sc[i] = rsqrt_f64(d > 0.0 ? d : 1.0);
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
        double d = tot[2 * j] * sc[j] * sc[j];
#pragma unroll
        for (int l = 0; l < j; ++l) d -= L[j][l] * L[j][l];
        ok = ok && (d > 1e-14);
        rl[j] = rsqrt_f64(d > 1e-14 ? d : 1.0);    // 1 / L[j][j]
#pragma unroll
        for (int i = j + 1; i < P; ++i) {
            double e = tot[i + j] * sc[i] * sc[j];
#pragma unroll
            for (int l = 0; l < j; ++l) e -= L[i][l] * L[j][l];
            L[i][j] = e * rl[j];
        }
    }
#pragma unroll
    for (int i = 0; i < P; ++i) {
        double e = tot[NA + i] * sc[i];
#pragma unroll
        for (int l = 0; l < i; ++l) e -= L[i][l] * y[l];
        y[i] = e * rl[i];
    }
#pragma unroll
    for (int i = P - 1; i >= 0; --i) {
        double e = y[i];
#pragma unroll
        for (int l = i + 1; l < P; ++l) e -= L[l][i] * gam[l];
        gam[i] = e * rl[i];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) beta[i] = (i < P && ok) ? gam[i < P ? i : 0] * sc[i < P ? i : 0] : 0.0;
    beta[8] = ok ? 1.0 : 0.0;
    beta[9] = n;
}

// Laguerre weight exp(-x/2) with x = S/K (wc = -1/(2K)), binary64.  With
// binary32 path values the degree-8 exponential (2.1e-10 relative) serves:
// the stored values themselves are 3e-8 away from the binary64 paths, and
// every use of a path's weight (both moment sums and the continuation value)
// reads this same value.
template <typename T>
__device__ __forceinline__ double lag_weight(double s, double wc)
{
    return sizeof(T) == 4 ? exp_poly_f32(s * wc) : exp_poly(s * wc);
}

// 16-byte vector of path values: 4 binary32 or 2 binary64 consecutive paths.
template <typename T>
struct alignas(16) Vec {
    static constexpr int n = 16 / sizeof(T);
    T v[n];
};

template <typename T>
__device__ __forceinline__ Vec<T> load_vec(const T *__restrict__ row, uint32_t c)
{
    return *reinterpret_cast<const Vec<T> *>(row + c);
}

template <typename T, int PPT>
struct SweepShape {
    static constexpr int VW = 16 / sizeof(T);
    static constexpr int NVEC = PPT / VW;
    // KEEP: a date's path values stay in registers across the barrier and
    // the next date is prefetched while waiting.
    static constexpr bool KEEP = sizeof(T) * PPT <= 64;
    // STREAM (not KEEP): ring of PD vectors in flight per thread.
    static constexpr int PD = NVEC < 8 ? NVEC : 8;
    // register budget: waves per SIMD the kernel is compiled for (256
    // VGPRs at 2; the smallest monomial tiles of degree <= 2 fit 4 groups
    // per CU at 128)
    template <int D, bool LAG>
    static constexpr int waves() { return (sizeof(T) * PPT <= 16 && !LAG && D <= 2) ? 4 : 2; }
};

// Slab-resident tiles (binary32 path values, monomial basis, one group of
// 512 threads per CU, 64 or 128 paths per thread): a date's slab stays on
// chip between the moment pass and the exercise update, the first NKL
// vectors of each thread in LDS and the next NKR in registers; the last NRR
// (what neither holds next to the resident cashflows) are read again for the
// update.
template <typename T, int PPT, int WG, bool LAG>
struct Resident {
    static constexpr bool on = sizeof(T) == 4 && WG == 512 && !LAG && (PPT == 64 || PPT == 128);
    static constexpr int NVEC = PPT * (int)sizeof(T) / 16;
    static constexpr int NKL = NVEC < 19 ? NVEC : 19;   // at most 19 x 512 x 16 B = 152 KiB of LDS
    static constexpr int NKR = NVEC - NKL < 8 ? NVEC - NKL : 8;
    static constexpr int NRR = NVEC - NKL - NKR;
};

// Vectors of a streamed tile's date slab kept in LDS between the moment pass
// and the exercise update (one group of 512 threads per CU: up to 128 KiB),
// so the update reads only the rest from memory again.
template <typename T, int PPT, int WG, bool LAG = false>
constexpr int stream_keep_vecs()
{
    if (SweepShape<T, PPT>::KEEP || WG != 512) return 0;
    if (Resident<T, PPT, WG, LAG>::on) return 0;   // their LDS slots are arrays of their own
    constexpr int cap = (128 * 1024) / (WG * 16);
    return SweepShape<T, PPT>::NVEC < cap ? SweepShape<T, PPT>::NVEC : cap;
}

// The per-path arithmetic of the sweep is binary64 for both storage types
// (path values and cashflows are stored in T): the least-squares fit and the
// exercise test feed back into every later date, and binary32 arithmetic
// there moves some prices by more than the binary32 tolerance.  On gfx950
// without packed binary32 math a binary64 FMA issues at the binary32 rate.

// Signed payoff argument h = sg (s - K) with sg = +1 (call) or -1 (put) and
// nsk = -sg K: one fma, exactly the rounded s - K or K - s.
__device__ __forceinline__ double payoff_arg(double s, double sg, double nsk)
{
    return fma(sg, s, nsk);
}

// Adds path value s (cashflow pvj discounted to t0) to the in-the-money
// moments acc[0..NA-1] (sum of wA xs^q) and acc[NA..NA+NB-1] (sum of wB xs^q
// pvj); returns 1 if the path is in the money.  (Streamed tiles: one pass.)
template <typename T, int D, bool LAG, bool PIN = true>
__device__ __forceinline__ int moments_add(double *acc, double s, double pvj, double sg, double nsk, double xa,
                                           double xb, double wc)
{
    constexpr int NA = 2 * D + 1, NB = D + 1;
    const bool itm = payoff_arg(s, sg, nsk) > 0.0;
    const double xs = fma(s, xa, xb);
    const double w = LAG ? lag_weight<T>(s, wc) : 1.0;
    // y_q = w xs^q on an in-the-money path (0 otherwise): the Gram moments
    // are sum w y_q (w = 1: sum y_q) and the right-hand side sum pvj y_q, so
    // one product chain serves both
    double y = itm ? w : 0.0;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
        acc[q] = LAG ? fma(w, y, acc[q]) : acc[q] + y;
        if (q < NB) acc[NA + q] = fma(pvj, y, acc[NA + q]);
        if (q + 1 < NA) y *= xs;
    }
    // pin the accumulators here: without this the optimizer sinks the sums
    // of a whole unrolled run of paths to its end, keeping every path's
    // powers live at once
    if (PIN) {
#pragma unroll
        for (int q = 0; q < NA + NB; ++q) asm volatile("" : "+v"(acc[q]));
    }
    return itm ? 1 : 0;
}

// The same sums split in two for register-resident tiles: the Gram part
// (sum of wA xs^q, which does not involve the cashflows) and the
// right-hand side (sum of wB xs^q pvj), with the same product chain, so each
// sum is bitwise the one moments_add forms.  gram_add stores the Laguerre
// weight for rhs_add and the exercise update.
template <typename T, int D, bool LAG>
__device__ __forceinline__ bool gram_add(double *acc, double s, double sg, double nsk, double xa, double xb,
                                         double wc, double *wout, double *yout = nullptr)
{
    constexpr int NA = 2 * D + 1, NB = D + 1;
    const bool itm = payoff_arg(s, sg, nsk) > 0.0;
    const double xs = fma(s, xa, xb);
    double w = 1.0;
    if (LAG) {
        w = lag_weight<T>(s, wc);
        *wout = w;
    }
    double y = itm ? w : 0.0;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
        if (yout && q < NB) yout[q] = y;   // the right-hand side's factors, kept for its pass
        acc[q] = LAG ? fma(w, y, acc[q]) : acc[q] + y;
        if (q + 1 < NA) y *= xs;
    }
    return itm;
}

// w: the path's Laguerre weight (1 for monomials), read for every path (a
// read under the in-the-money mask would wait on each path in turn).
template <int D>
__device__ __forceinline__ void rhs_add(double *acc, double s, double pvj, double sg, double nsk, double xa,
                                        double xb, double w)
{
    constexpr int NB = D + 1;
    const bool itm = payoff_arg(s, sg, nsk) > 0.0;
    const double xs = fma(s, xa, xb);
    double y = itm ? w : 0.0;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        acc[q] = fma(pvj, y, acc[q]);
        if (q + 1 < NB) y *= xs;
    }
}

// Exercise update at a date: exercise (cashflow dk h) when in the money and
// dk h exceeds the fitted continuation; else keep pvj.
template <typename T, int D, bool LAG>
__device__ __forceinline__ T exercise_update(T s_t, T pvj, double sg, double nsk, double xa, double xb, double dk,
                                             const double *gam, double wc, const double *wgiven = nullptr)
{
    constexpr int P = D + 1;
    // recomputed here rather than kept from the moment pass: holding every
    // path's payoff and abscissa across the sum costs more registers than
    // the two fmas
    double s = (double)s_t;
    asm volatile("" : "+v"(s));
    const double h = payoff_arg(s, sg, nsk);
    const double xs = fma(s, xa, xb);
    double cont = gam[P - 1];
#pragma unroll
    for (int q = P - 2; q >= 0; --q) cont = fma(cont, xs, gam[q]);
    if (LAG) cont *= wgiven ? *wgiven : lag_weight<T>(s, wc);
    const double ex = dk * h;
    // in the money and above the continuation: with dk > 0, ex > 0 exactly
    // when h > 0 (|h| is at least an ulp of K, far from underflow), so this
    // is the test h > 0 && ex > cont
    return ex > fmax(cont, 0.0) ? (T)ex : pvj;
}

// ---------------------------------------------------------------------------
// Backward induction (Section V), persistent.  Group g owns the tile of
// 256*PPT consecutive paths starting at g*256*PPT; wave w of the group owns
// the 64*PPT paths from g*256*PPT + w*64*PPT, read as 16-byte vectors, vector
// jj of lane l at element w*64*PPT + jj*64*VW + l*VW (each wave load reads
// 1 KiB contiguous).  The discounted cashflows pv[] of a thread's PPT paths
// stay in registers for the whole sweep.  Per date k = M-1..1:
//   in-the-money moments (Hankel form of the Gram matrix in the standardised
//   abscissa xs; weights wA = wB = 1 for monomials, wA = w^2, wB = w with
//   w = exp(-x/2) for Laguerre: same span as the requested basis) of pv, the
//   cashflow discounted to t0, so the exercise test is disc_k * h > fit;
//   a device-wide fixed-order sum that every group receives (allreduce);
//   every group solves the same normal equations (bitwise the same
//   coefficients; group 0 keeps the date record); exercise update.
// Per-path arithmetic is binary64 for both storage types (see SweepShape).
// Rows are padded to a multiple of every tile size with S = K (rounded away
// from the money in binary32), so padded paths are never in the money and
// keep pv = 0: no bounds checks.
// ---------------------------------------------------------------------------
template <typename T, int PPT, int WG>
struct TileIO {
    static constexpr int VW = 16 / sizeof(T);
    static constexpr uint32_t JS = 64 * VW;   // element stride between a lane's vectors
    static constexpr int32_t kTileBytes = WG * PPT * (int32_t)sizeof(T);
    int64_t tile0;
    uint32_t voff;                            // this lane's byte offset in the tile
    __device__ TileIO(uint32_t gid, uint32_t e0)
        : tile0((int64_t)gid * WG * PPT), voff((e0 - (uint32_t)((int64_t)gid * WG * PPT)) * (uint32_t)sizeof(T))
    {
    }
    // Buffer loads: tile base in SGPRs, one lane offset, constant per-vector
    // offsets.  Rows are padded to whole tiles (no bounds checks).
    __device__ __forceinline__ Vec<T> load(const T *row, int jj) const
    {
        __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc((void *)(row + tile0), (short)0, kTileBytes, 0x00020000);
        return __builtin_bit_cast(Vec<T>, __builtin_amdgcn_raw_buffer_load_b128(
                                                rs, voff, (uint32_t)jj * JS * (uint32_t)sizeof(T), 0));
    }
};

// Discounted terminal cashflows of the thread's paths (date M), streamed
// through a ring of PD loads (issuing every load at once would hold a second
// copy of pv[] in registers).
template <typename T, int PPT, int WG>
__device__ __forceinline__ void sweep_terminal(const SweepArgs &a, const T *__restrict__ S, const TileIO<T, PPT, WG> &io,
                                               T (&pv)[PPT])
{
    using SH = SweepShape<T, PPT>;
    constexpr int VW = SH::VW, NVEC = SH::NVEC, PD = SH::PD;
    const double K = a.K;
    const bool call = a.is_call != 0;
    const T *row = S + (size_t)(a.M - 1) * a.ld;
    const double dM = a.datec[a.M].disc;
    Vec<T> ring[PD];
#pragma unroll
    for (int q = 0; q < PD; ++q) ring[q] = io.load(row, q);
#pragma unroll
    for (int jj = 0; jj < NVEC; ++jj) {
        const Vec<T> v = ring[jj % PD];
        if (jj + PD < NVEC) ring[jj % PD] = io.load(row, jj + PD);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            const double sv = (double)v.v[e];
            const double h = call ? sv - K : K - sv;
            pv[jj * VW + e] = h > 0.0 ? (T)(dM * h) : T(0);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// The solve of date k by thread 0 (registers where the kernel has room,
// else LDS), and group 0's date record: coefficients, flag and count, the
// moments, and device clock stamps of the date's phases.
// MODE 0: totals and factor in registers; 1: factor in LDS (the compiler may
// still keep it in registers).
template <int D, int MODE>
__device__ __forceinline__ void solve_and_record(const SweepArgs &a, uint32_t gid, int k, const double *s_tot,
                                                 double *s_beta, double (*s_L)[8], double *s_w,
                                                 const uint64_t (&stamp)[3])
{
    constexpr int NV = 3 * D + 4;
    const uint64_t c_all = __builtin_amdgcn_s_memrealtime();
    if constexpr (MODE == 0) {
        // the totals in registers first: every LDS read issued at once
        double tr[NV], Lr[8][8], wr[32];
#pragma unroll
        for (int q = 0; q < NV; ++q) tr[q] = s_tot[q];
        solve_date<D>(tr, s_beta, Lr, wr);
    } else {
        solve_date<D>(s_tot, s_beta, s_L, s_w);
    }
    if (gid == 0) {
        // every group solved the same system; group 0 keeps the record
        double *rec = a.rec + (size_t)k * kRec;
#pragma unroll
        for (int q = 0; q < 10; ++q) rec[q] = s_beta[q];
        for (int q = 0; q < NV && q < 22; ++q) rec[10 + q] = s_tot[q];
        rec[kRecTime + 0] = (double)stamp[0];                             // moments summed in the group
        rec[kRecTime + 1] = (double)c_all;                                // device-wide totals in hand
        rec[kRecTime + 2] = (double)__builtin_amdgcn_s_memrealtime();     // solved
        rec[kRecTime + 3] = (double)stamp[1];                             // next date's Gram part summed
        rec[kRecTime + 4] = (double)stamp[2];                             // date's pass started
    }
}

__device__ __forceinline__ double readlane_f64(double x, int l)
{
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)b, l);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(b >> 32), l);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// The same solve as solve_date (equilibration by the diagonal, Cholesky with
// pivots at or below 1e-14 rejected, forward and backward substitution) by
// the 64 lanes of one wave: lane i < P holds row i of the equilibrated
// matrix and of its factor, rows cross lanes through readlane, and the
// factor's columns through LDS for the backward substitution.  A few
// registers per lane instead of the whole factor in one thread's registers,
// for kernels whose register file holds resident path data.  Lanes past P
// mirror row P-1 (their values are not used).  tot: LDS; beta: LDS
// [0..7] coefficients (zero past P, all zero if rejected), [8] solved flag,
// [9] count; s_col: LDS [8][8] scratch.  Call with every lane of the wave.
template <int D>
__device__ __forceinline__ void solve_date_wave(const double *tot, double *beta, double (*s_col)[8])
{
    constexpr int P = D + 1, NA = 2 * D + 1;
    const int lane = tid_x() & 63;
    const int i = lane < P ? lane : P - 1;
    const double n = rint(tot[NA + P]);
    const double dii = tot[2 * i];
    const double sci = rsqrt_f64(dii > 0.0 ? dii : 1.0);
    bool ok = n >= (double)P && __builtin_amdgcn_ballot_w64(lane < P && !(dii > 0.0)) == 0;
    double a[P], L[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
        a[j] = tot[i + j] * sci * readlane_f64(sci, j);
        L[j] = 0.0;
    }
    // Cholesky, column j: lane j's pivot, then every lane's entry of column j
    double rli = 1.0;
#pragma unroll
    for (int j = 0; j < P; ++j) {
        double d = a[j];
#pragma unroll
        for (int l = 0; l < j; ++l) d -= L[l] * L[l];
        const double dj = readlane_f64(d, j);
        ok = ok && dj > 1e-14;
        const double rlj = rsqrt_f64(dj > 1e-14 ? dj : 1.0);
        rli = lane == j ? rlj : rli;
        double e = a[j];
#pragma unroll
        for (int l = 0; l < j; ++l) e -= L[l] * readlane_f64(L[l], j);
        L[j] = e * rlj;
    }
    // forward substitution: y_l leaves lane l once its sum is complete
    double t = tot[NA + i] * sci, yi = 0.0;
#pragma unroll
    for (int l = 0; l < P; ++l) {
        const double yl = readlane_f64(t * rli, l);
        yi = lane == l ? yl : yi;
        t -= L[l] * yl;
    }
    // backward substitution with the factor's columns: lane i reads column i
    if (lane < P) {
#pragma unroll
        for (int l = 0; l < P; ++l) s_col[i][l] = L[l];
    }
    __builtin_amdgcn_wave_barrier();
    double Lc[P];
#pragma unroll
    for (int l = 0; l < P; ++l) Lc[l] = s_col[l][i];
    double u = yi, gi = 0.0;
#pragma unroll
    for (int l = P - 1; l >= 0; --l) {
        const double gl = readlane_f64(u * rli, l);
        gi = lane == l ? gl : gi;
        u -= Lc[l] * gl;
    }
    if (lane < 8) beta[lane] = (lane < P && ok) ? gi * sci : 0.0;
    if (lane == 0) {
        beta[8] = ok ? 1.0 : 0.0;
        beta[9] = n;
    }
}

// The wave-parallel solve of date k by wave 0 and group 0's date record, as
// solve_and_record.  Call with every lane of wave 0.
template <int D>
__device__ __forceinline__ void solve_and_record_wave(const SweepArgs &a, uint32_t gid, int k, const double *s_tot,
                                                      double *s_beta, double (*s_col)[8], const uint64_t (&stamp)[3])
{
    constexpr int NV = 3 * D + 4;
    const uint64_t c_all = __builtin_amdgcn_s_memrealtime();
    solve_date_wave<D>(s_tot, s_beta, s_col);
    if (gid == 0 && tid_x() == 0) {
        double *rec = a.rec + (size_t)k * kRec;
#pragma unroll
        for (int q = 0; q < 10; ++q) rec[q] = s_beta[q];
        for (int q = 0; q < NV && q < 22; ++q) rec[10 + q] = s_tot[q];
        rec[kRecTime + 0] = (double)stamp[0];
        rec[kRecTime + 1] = (double)c_all;
        rec[kRecTime + 2] = (double)__builtin_amdgcn_s_memrealtime();
        rec[kRecTime + 3] = (double)stamp[1];
        rec[kRecTime + 4] = (double)stamp[2];
    }
}

// Register-resident tile (KEEP): the date's path values stay in registers
// across the device-wide sum.  The Gram part of the next date's moments
// depends only on that date's path values, so it is formed while this
// date's sum is in flight (between publishing and gathering); what remains
// on the critical path is the right-hand side pass (which needs the
// cashflows after this date's update), the sum, the solve and the update.
// Path values are double-buffered plus one prefetch; the Laguerre weights
// of two dates are cached in LDS ([2][path][thread], each thread touching
// only its own entries).  Date constants come through uniform vector loads
// issued a date ahead.
template <typename T, int PPT, int D, bool LAG, int WG>
__device__ __forceinline__ void sweep_keep(const SweepArgs &a, const T *__restrict__ S, uint32_t gid,
                                           const TileIO<T, PPT, WG> &io, T (&pv)[PPT], uint32_t &epoch, bool &alive,
                                           double (*s_red)[32], double (*s_red2)[32], double *s_tot,
                                           double *s_beta, double *s_wl, double *s_x, int *s_flag)
{
    using SH = SweepShape<T, PPT>;
    constexpr int VW = SH::VW, NVEC = SH::NVEC;
    constexpr int NA = 2 * D + 1, NB = D + 1, P = D + 1;
    constexpr int NG = NA + 1, NV = NA + NB + 1;
    constexpr int RW = row_words(D);
    const int tid = threadIdx.x;
    const int64_t ld = a.ld;
    const int M = a.M;
    const double sg = a.is_call ? 1.0 : -1.0, nsk = -sg * a.K;
    const double wc = -0.5 / a.K;   // Laguerre weight exponent per unit S
    const uint32_t G = (uint32_t)a.G;

    // date constants: (disc, xa) and (xb, pad) of date k, one line per date
    const __amdgpu_buffer_rsrc_t drs =
        __builtin_amdgcn_make_buffer_rsrc((void *)a.datec, (short)0, (M + 1) * (int)sizeof(DateConst), 0x00020000);
    auto dload = [&](int k, double (&d)[3]) {
        using V2 = double __attribute__((ext_vector_type(2)));
        const V2 u = __builtin_bit_cast(V2, __builtin_amdgcn_raw_buffer_load_b128(drs, 0, k * 32, 0));
        const V2 v = __builtin_bit_cast(V2, __builtin_amdgcn_raw_buffer_load_b128(drs, 0, k * 32 + 16, 0));
        d[0] = u.x;
        d[1] = u.y;
        d[2] = v.x;
    };
    auto wbuf = [&](int k) -> double * { return s_wl + (size_t)(k & 1) * PPT * WG + tid; };

    // Gram part of date k's moments from its path values v, pairs of paths
    // into two accumulator sets (independent chains), pinned per pair; the
    // in-the-money count from wave ballots (scalar unit); result (group
    // total) valid in thread 0
    // kCacheY: the Gram pass also keeps each path's right-hand-side factors
    // y_q (q <= D) in registers, so the right-hand-side pass after the update
    // is one fma per sum (512-thread binary32 tiles, which have the room)
    constexpr bool kCacheY = WG == 512 && sizeof(T) == 4 && PPT * NB <= 32;
    double ys[kCacheY ? PPT : 1][NB];
    auto gram_pass = [&](const Vec<T>(&v)[NVEC], double xa, double xb, double *wl, double (&g)[NG]) {
        double g2[NA];
#pragma unroll
        for (int q = 0; q < NA; ++q) g[q] = g2[q] = 0.0;
        uint32_t cnt = 0;
#pragma unroll
        for (int jj = 0; jj < NVEC; ++jj) {
#pragma unroll
            for (int e = 0; e < VW; e += 2) {
                const int j0 = jj * VW + e;
                const bool i0 = gram_add<T, D, LAG>(g, (double)v[jj].v[e], sg, nsk, xa, xb, wc, wl + j0 * WG,
                                                 kCacheY ? ys[kCacheY ? j0 : 0] : nullptr);
                const bool i1 = gram_add<T, D, LAG>(g2, (double)v[jj].v[e + 1], sg, nsk, xa, xb, wc,
                                                 wl + (j0 + 1) * WG, kCacheY ? ys[kCacheY ? j0 + 1 : 0] : nullptr);
                cnt += (uint32_t)__builtin_popcountll(__builtin_amdgcn_ballot_w64(i0)) +
                       (uint32_t)__builtin_popcountll(__builtin_amdgcn_ballot_w64(i1));
#pragma unroll
                for (int q = 0; q < NA; ++q) {
                    asm volatile("" : "+v"(g[q]));
                    asm volatile("" : "+v"(g2[q]));
                }
            }
        }
#pragma unroll
        for (int q = 0; q < NA; ++q) g[q] += g2[q];
        g[NA] = (double)cnt;
        if constexpr (WG == 512 && NA <= 8) group_sum_lds<NG, 1, WG>(g, s_x, s_red2);
        else group_sum<NG, 1, WG>(g, s_red2);
    };

    if (!(a.allow_exercise && M >= 2)) return;

    Vec<T> sc[NVEC], sn[NVEC], sp[NVEC];
    double dcp[3];
    double dcc[3];
    dload(M - 1, dcc);
    {
        const T *row = S + (size_t)(M - 2) * ld;
#pragma unroll
        for (int jj = 0; jj < NVEC; ++jj) sc[jj] = io.load(row, jj);
    }
    // prefetches are unconditional (the date clamped to 1; unused at the
    // end), so the loads land in the loop-carried registers directly
    auto prefetch = [&](int kp) {
        kp = kp >= 1 ? kp : 1;
        dload(kp, dcp);
        const T *row = S + (size_t)(kp - 1) * ld;
#pragma unroll
        for (int jj = 0; jj < NVEC; ++jj) sp[jj] = io.load(row, jj);
    };
    prefetch(M - 2);
    double xa = uniform_f64(dcc[1]), xb = uniform_f64(dcc[2]), dk = uniform_f64(dcc[0]);
    double gt[NG];
    gram_pass(sc, xa, xb, wbuf(M - 1), gt);

    for (int k = M - 1; k >= 1; --k) {
        uint64_t stamp[3];
        stamp[2] = __builtin_amdgcn_s_memrealtime();
        double rs[NB];
        {
            double r2[NB];
#pragma unroll
            for (int q = 0; q < NB; ++q) rs[q] = r2[q] = 0.0;
            // every weight read issued before the first pinned sum (memory
            // reads do not move across the pins)
            const double *wl = wbuf(k);
            double wv[PPT];
#pragma unroll
            for (int j = 0; j < PPT; ++j) wv[j] = (LAG && !kCacheY) ? wl[j * WG] : 1.0;
#pragma unroll
            for (int jj = 0; jj < NVEC; ++jj) {
#pragma unroll
                for (int e = 0; e < VW; e += 2) {
                    const int j0 = jj * VW + e;
                    if constexpr (kCacheY) {
                        // the same products as rhs_add, from the kept factors
#pragma unroll
                        for (int q = 0; q < NB; ++q) {
                            rs[q] = fma((double)pv[j0], ys[j0][q], rs[q]);
                            r2[q] = fma((double)pv[j0 + 1], ys[j0 + 1][q], r2[q]);
                        }
                    } else {
                        rhs_add<D>(rs, (double)sc[jj].v[e], (double)pv[j0], sg, nsk, xa, xb, wv[j0]);
                        rhs_add<D>(r2, (double)sc[jj].v[e + 1], (double)pv[j0 + 1], sg, nsk, xa, xb, wv[j0 + 1]);
                    }
#pragma unroll
                    for (int q = 0; q < NB; ++q) {
                        asm volatile("" : "+v"(rs[q]));
                        asm volatile("" : "+v"(r2[q]));
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < NB; ++q) rs[q] += r2[q];
        }
        if constexpr (WG == 512) group_sum_lds<NB, 0, WG>(rs, s_x, s_red);
        else group_sum<NB, 0, WG>(rs, s_red);
        ++epoch;
        stamp[0] = __builtin_amdgcn_s_memrealtime();
        double acc[NV];
#pragma unroll
        for (int q = 0; q < NA; ++q) acc[q] = gt[q];
#pragma unroll
        for (int q = 0; q < NB; ++q) acc[NA + q] = rs[q];
        acc[NV - 1] = gt[NA];
        if (!allreduce_publish<NV, RW, WG>(acc, gid, G, a.rows, a.sync, a.err, epoch, a.spin_limit, s_tot, s_red,
                                       s_flag)) {
            alive = false;
            return;
        }

        // next date's Gram part while this date's sum is in flight, with the
        // date after next in flight from memory meanwhile
        double xan = xa, xbn = xb, dkn = dk;
#pragma unroll
        for (int jj = 0; jj < NVEC; ++jj) sn[jj] = sp[jj];
        if (k >= 2) {
            xan = uniform_f64(dcp[1]);
            xbn = uniform_f64(dcp[2]);
            dkn = uniform_f64(dcp[0]);
        }
        prefetch(k - 2);
        if (k >= 2) gram_pass(sn, xan, xbn, wbuf(k - 1), gt);
        stamp[1] = __builtin_amdgcn_s_memrealtime();

        if (!allreduce_gather<NV, RW, WG>(G, a.rows, a.sync, a.err, epoch, a.spin_limit, s_tot, s_red, s_flag,
                                          k >= 2)) {
            alive = false;
            return;
        }
        if (tid == 0) solve_and_record<D, 0>(a, gid, k, s_tot, s_beta, nullptr, nullptr, stamp);
        __syncthreads();

        if (s_beta[8] != 0.0) {
            double gam[P];
#pragma unroll
            for (int q = 0; q < P; ++q) gam[q] = s_beta[q];
            const double *wl = wbuf(k);
#pragma unroll
            for (int jj = 0; jj < NVEC; ++jj) {
#pragma unroll
                for (int e = 0; e < VW; ++e)
                    pv[jj * VW + e] = exercise_update<T, D, LAG>(sc[jj].v[e], pv[jj * VW + e], sg, nsk, xa, xb, dk,
                                                                 gam, wc, wl + (jj * VW + e) * WG);
                __builtin_amdgcn_sched_barrier(0);   // one vector's paths at a time
            }
        }
#pragma unroll
        for (int jj = 0; jj < NVEC; ++jj) sc[jj] = sn[jj];
        xa = xan;
        xb = xbn;
        dk = dkn;
        __syncthreads();   // s_beta reuse
    }
}

// Streamed tile: the date's slab is read twice (moments, then update)
// through a ring of PD vector loads in flight per thread; date constants
// staged in LDS.
template <typename T, int PPT, int D, bool LAG, int WG>
__device__ __forceinline__ void sweep_stream(const SweepArgs &a, const T *__restrict__ S, uint32_t gid,
                                             const TileIO<T, PPT, WG> &io, T (&pv)[PPT], uint32_t &epoch, bool &alive,
                                             double (*s_red)[32], double *s_tot, double *s_beta, double (*s_L)[8],
                                             double *s_w, DateConst *s_dc, Vec<T> *s_keep, int *s_flag)
{
    constexpr int NK = stream_keep_vecs<T, PPT, WG, LAG>();
    using SH = SweepShape<T, PPT>;
    constexpr int VW = SH::VW, NVEC = SH::NVEC, PD = SH::PD;
    constexpr int NA = 2 * D + 1, NB = D + 1, P = D + 1;
    constexpr int NV = NA + NB + 1;
    constexpr int RW = row_words(D);
    const int tid = threadIdx.x;
    const int64_t ld = a.ld;
    const double sg = a.is_call ? 1.0 : -1.0, nsk = -sg * a.K;
    const double wc = -0.5 / a.K;
    const uint32_t G = (uint32_t)a.G;

    if (!(a.allow_exercise && a.M >= 2)) return;
    // date constants staged in LDS (a dependent global load at the top of
    // each date would stall the moment pass)
    for (int k = tid; k <= a.M; k += WG) s_dc[k] = a.datec[k];
    __syncthreads();
    for (int k = a.M - 1; k >= 1; --k) {
        const double xa = uniform_f64(s_dc[k].xa), xb = uniform_f64(s_dc[k].xb),
                     dk = uniform_f64(s_dc[k].disc);
        const T *row = S + (size_t)(k - 1) * ld;
        uint64_t stamp[3];
        stamp[2] = __builtin_amdgcn_s_memrealtime();

        double acc[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) acc[q] = 0.0;
        int cnt = 0;
        {
            Vec<T> ring[PD];
#pragma unroll
            for (int q = 0; q < PD; ++q) ring[q] = io.load(row, q);
#pragma unroll
            for (int jj = 0; jj < NVEC; ++jj) {
                const Vec<T> cur = ring[jj % PD];
                if (jj + PD < NVEC) ring[jj % PD] = io.load(row, jj + PD);
                __builtin_amdgcn_sched_barrier(0);
                if (jj < NK) s_keep[jj * WG + tid] = cur;   // the update reads these back
#pragma unroll
                for (int e = 0; e < VW; ++e) {
                    cnt += moments_add<T, D, LAG>(acc, (double)cur.v[e], (double)pv[jj * VW + e], sg, nsk, xa, xb, wc);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        acc[NV - 1] = (double)cnt;

        group_sum<NV, 0, WG>(acc, s_red);
        ++epoch;
        // (a clock read before group_sum would pin the moment pass's schedule)
        stamp[0] = stamp[1] = __builtin_amdgcn_s_memrealtime();
        if (!allreduce<NV, RW, WG>(acc, gid, G, a.rows, a.sync, a.err, epoch, a.spin_limit, s_tot, s_red, s_flag)) {
            alive = false;
            return;
        }
        if (tid == 0) solve_and_record<D, 1>(a, gid, k, s_tot, s_beta, s_L, s_w, stamp);
        __syncthreads();

        if (s_beta[8] != 0.0) {
            double gam[P];
#pragma unroll
            for (int q = 0; q < P; ++q) gam[q] = s_beta[q];
            // the vectors kept in LDS first, with the memory ring for the
            // rest already in flight
            Vec<T> ring[PD];
#pragma unroll
            for (int q = 0; q < PD; ++q)
                if (NK + q < NVEC) ring[q] = io.load(row, NK + q);
#pragma unroll
            for (int jj = 0; jj < NVEC; ++jj) {
                Vec<T> cur;
                if (jj < NK) {
                    cur = s_keep[jj * WG + tid];
                } else {
                    const int r = (jj - NK) % PD;
                    cur = ring[r];
                    if (jj + PD < NVEC) ring[r] = io.load(row, jj + PD);
                }
                __builtin_amdgcn_sched_barrier(0);
                // a vector's paths together: their dependent chains interleave
#pragma unroll
                for (int e = 0; e < VW; ++e)
                    pv[jj * VW + e] = exercise_update<T, D, LAG>(cur.v[e], pv[jj * VW + e], sg, nsk, xa, xb, dk, gam,
                                                                 wc);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        __syncthreads();   // s_beta reuse
    }
}

// Strike as a binary32 threshold on the stored path values: for binary32 s
// and binary64 K, s > K exactly when s > K rounded down (call) and s < K
// exactly when s < K rounded up (put).  (The row padding holds these values,
// so padded paths are never in the money.)
template <bool CALL>
__device__ __forceinline__ float strike_threshold_f32(double K)
{
    float k = (float)K;
    if (CALL && (double)k > K) k = __int_as_float(__float_as_int(k) - 1);
    if (!CALL && (double)k < K) k = __int_as_float(__float_as_int(k) + 1);
    return k;
}

// Monomial moments of one path for the slab-resident tile.  With m = 1 on
// an in-the-money path (else 0) and y = m xs, the powers y^q (q <= D) come by
// squaring (D - 1 multiplies); the Gram sums of y^q for q = 1..D add them and
// those for q = D+1..2D are one fma y^D y^(q-D) each; the right-hand side is
// one fma pv y^q per q (y^0 = m).  A[q-1]: sum of y^q (q = 1..2D); R[q]: sum
// of pv y^q (q = 0..D).  The count (q = 0) comes from wave ballots.
template <int D>
__device__ __forceinline__ void resident_moments(double *A, double *R, double s, double pv, bool itm, double xa,
                                                 double xb)
{
    const double m = itm ? 1.0 : 0.0;
    double p[D + 1];
    p[0] = m;
    if constexpr (D >= 1) p[1] = fma(s, xa, xb) * m;
#pragma unroll
    for (int q = 2; q <= D; ++q) p[q] = p[q / 2] * p[q - q / 2];
#pragma unroll
    for (int q = 1; q <= D; ++q) A[q - 1] += p[q];
#pragma unroll
    for (int q = D + 1; q <= 2 * D; ++q) A[q - 1] = fma(p[D], p[q - D], A[q - 1]);
#pragma unroll
    for (int q = 0; q <= D; ++q) R[q] = fma(pv, p[q], R[q]);
#pragma unroll
    for (int q = 0; q < 2 * D; ++q) asm volatile("" : "+v"(A[q]));
#pragma unroll
    for (int q = 0; q <= D; ++q) asm volatile("" : "+v"(R[q]));
}

// Exercise update of one path for the slab-resident tile: the discounted
// payoff dk sg (s - K) as one fma (dsg = dk sg, dnsk = -dk sg K), the fitted
// continuation by Horner in xs; exercise when in the money and the
// discounted payoff exceeds the fit (for an in-the-money path the payoff is
// positive, so this is the test dk h > max(fit, 0)).
template <bool CALL, int D>
__device__ __forceinline__ float resident_update(float s32, float pvj, float kthr, double xa, double xb, double dsg,
                                                 double dnsk, const double *gam)
{
    // recomputed from the stored value: keeping the moment pass's abscissae
    // and in-the-money masks of every path across the device-wide sum would
    // take more registers than the kernel has
    double s = (double)s32;
    asm volatile("" : "+v"(s));
    const bool itm = CALL ? s > (double)kthr : s < (double)kthr;
    const double xs = fma(s, xa, xb);
    double cont = gam[D];
#pragma unroll
    for (int q = D - 1; q >= 0; --q) cont = fma(cont, xs, gam[q]);
    const double ex = fma(dsg, s, dnsk);
    return (itm && ex > cont) ? (float)ex : pvj;
}

// Compile-time loop: f(Ic<B>{}), ..., f(Ic<E-1>{}).
template <int I> struct Ic { static constexpr int value = I; };
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (B < E) {
        f(Ic<B>{});
        static_for<B + 1, E>(f);
    }
}

// Wait until at most N vector memory operations of this wave are
// outstanding (they complete in issue order).
template <int N>
__device__ __forceinline__ void wait_vmcnt()
{
    static_assert(N >= 0 && N <= 63, "vmcnt field");
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// LDS slots of the slab-resident tile: slot j lives in array j mod 8, at
// position j / 8 (eight arrays: the compiler tracks direct-to-LDS loads per
// target array, for at most eight arrays, so the LDS this kernel reads
// otherwise is never made to wait for them).  The slots themselves are read
// with read_slot after an explicit wait for their own load.
template <int A, int NS>
__device__ __forceinline__ Vec<float> *resident_array()
{
    __shared__ Vec<float> s[NS * 512];
    return s;
}
template <int J, int NKL>
__device__ __forceinline__ Vec<float> *resident_slot()
{
    constexpr int A = J % 8;
    return resident_array<A, (NKL - A + 7) / 8>() + (J / 8) * 512;
}

// A 16-byte LDS read, complete on return.  The slab-resident tile's LDS
// slots are filled by direct-to-LDS loads that the tile waits for itself
// (wait_vmcnt, counting its own requests); reading them outside the
// compiler's view keeps it from adding a conservative wait for every load
// in flight before each read.
__device__ __forceinline__ Vec<float> read_slot(const Vec<float> *base, uint32_t lane_off)
{
    using V4 = float __attribute__((ext_vector_type(4)));
    // the array's LDS address is wave-uniform (a scalar operand), the lane's
    // byte offset one register shared by every slot
    const uint32_t b = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) const void *)base;
    V4 r;
    uint32_t t;
    asm volatile("v_add_u32 %1, %2, %3\n\tds_read_b128 %0, %1\n\ts_waitcnt lgkmcnt(0)"
                 : "=v"(r), "=&v"(t)
                 : "s"(b), "v"(lane_off));
    Vec<float> v;
    v.v[0] = r.x;
    v.v[1] = r.y;
    v.v[2] = r.z;
    v.v[3] = r.w;
    return v;
}

// Two 16-byte LDS reads under one wait (the second read's latency overlaps
// the first's), complete on return.
__device__ __forceinline__ void read_slot2(const Vec<float> *base0, const Vec<float> *base1, uint32_t lane_off,
                                           Vec<float> &v0, Vec<float> &v1)
{
    using V4 = float __attribute__((ext_vector_type(4)));
    const uint32_t b0 = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) const void *)base0;
    const uint32_t b1 = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) const void *)base1;
    V4 r0, r1;
    uint32_t t0, t1;
    asm volatile("v_add_u32 %2, %4, %6\n\tv_add_u32 %3, %5, %6\n\tds_read_b128 %0, %2\n\t"
                 "ds_read_b128 %1, %3\n\ts_waitcnt lgkmcnt(0)"
                 : "=&v"(r0), "=&v"(r1), "=&v"(t0), "=&v"(t1)
                 : "s"(b0), "s"(b1), "v"(lane_off));
    v0.v[0] = r0.x; v0.v[1] = r0.y; v0.v[2] = r0.z; v0.v[3] = r0.w;
    v1.v[0] = r1.x; v1.v[1] = r1.y; v1.v[2] = r1.z; v1.v[3] = r1.w;
}

// Four 16-byte LDS reads under one wait, complete on return.
__device__ __forceinline__ void read_slot4(const Vec<float> *base0, const Vec<float> *base1,
                                           const Vec<float> *base2, const Vec<float> *base3, uint32_t lane_off,
                                           Vec<float> &v0, Vec<float> &v1, Vec<float> &v2, Vec<float> &v3)
{
    using V4 = float __attribute__((ext_vector_type(4)));
    const uint32_t b0 = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) const void *)base0;
    const uint32_t b1 = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) const void *)base1;
    const uint32_t b2 = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) const void *)base2;
    const uint32_t b3 = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) const void *)base3;
    V4 r0, r1, r2, r3;
    uint32_t t0, t1, t2, t3;
    asm volatile("v_add_u32 %4, %8, %12\n\tv_add_u32 %5, %9, %12\n\tv_add_u32 %6, %10, %12\n\t"
                 "v_add_u32 %7, %11, %12\n\tds_read_b128 %0, %4\n\tds_read_b128 %1, %5\n\t"
                 "ds_read_b128 %2, %6\n\tds_read_b128 %3, %7\n\ts_waitcnt lgkmcnt(0)"
                 : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3), "=&v"(t0), "=&v"(t1), "=&v"(t2), "=&v"(t3)
                 : "s"(b0), "s"(b1), "s"(b2), "s"(b3), "v"(lane_off));
    v0.v[0] = r0.x; v0.v[1] = r0.y; v0.v[2] = r0.z; v0.v[3] = r0.w;
    v1.v[0] = r1.x; v1.v[1] = r1.y; v1.v[2] = r1.z; v1.v[3] = r1.w;
    v2.v[0] = r2.x; v2.v[1] = r2.y; v2.v[2] = r2.z; v2.v[3] = r2.w;
    v3.v[0] = r3.x; v3.v[1] = r3.y; v3.v[2] = r3.z; v3.v[3] = r3.w;
}

// Slab-resident tile: per date, a moment pass over the slab, the
// device-wide sum and solve, then the exercise update over the same values.
// A thread's 4-path vectors ("slots", j = 0..NVEC-1) are processed in the
// same order in both passes: the first NKL live in LDS from their load until
// the update has read them (loaded straight from memory into LDS, no
// registers in flight), the next NKR in registers, the last NRR are read
// again for the update.  Loads run PF slots ahead of their use: the moment
// pass requests slot j + PF as it reaches slot j, the update requests the
// re-read slots PF ahead and, over its last PF slots, the first PF slots of
// the next date (each freed by then), so about PF slots per thread are in
// flight at any time and no wave stalls on a full memory queue.  Before
// reading LDS slot j the moment pass waits until at most the requests made
// after slot j's are outstanding (vector memory operations complete in
// issue order; operations the compiler adds only make the wait stricter).
// Both passes read the LDS slots in fours (then a pair and a single) under
// one LDS wait each (the moment pass first waits for the group's last load).  Date constants come
// through scalar loads issued a date ahead.
template <int PPT, int D, bool CALL>
__device__ __forceinline__ void sweep_resident(const SweepArgs &a, const float *__restrict__ S, uint32_t gid,
                                               const TileIO<float, PPT, 512> &io, float (&pv)[PPT], uint32_t &epoch,
                                               bool &alive, double (*s_red)[32], double *s_tot, double *s_beta,
                                               double (*s_L)[8], double *s_w, int *s_flag)
{
    constexpr int WG = 512;
    using RS = Resident<float, PPT, WG, false>;
    constexpr int NKL = RS::NKL, NKR = RS::NKR, NRR = RS::NRR, NVEC = RS::NVEC;
    constexpr int PF = NVEC < 12 ? NVEC : 12;
    constexpr int NA = 2 * D + 1, NB = D + 1;
    constexpr int NV = NA + NB + 1;
    constexpr int RW = row_words(D);
    constexpr uint32_t JS = 64 * 4;          // elements between a lane's vectors
    const int tid = threadIdx.x;
    // wave-uniform, so the LDS destinations of the direct loads are scalar
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t ld = a.ld;
    const int M = a.M;
    const double sg = CALL ? 1.0 : -1.0, nsk = -sg * a.K;
    const float kthr = strike_threshold_f32<CALL>(a.K);
    const uint32_t G = (uint32_t)a.G;
    if (!(a.allow_exercise && M >= 2)) return;

    // date constants through the scalar cache (written by the generation
    // kernel, read-only here): scalar registers, and their waits are not
    // ordered behind the slab's vector loads
    const __attribute__((address_space(4))) DateConst *dcs =
        (const __attribute__((address_space(4))) DateConst *)a.datec;
    struct DC { double disc, xa, xb; };
    auto dconst = [&](int k) {
        DC d;
        d.disc = dcs[k].disc;
        d.xa = dcs[k].xa;
        d.xb = dcs[k].xb;
        return d;
    };
    Vec<float> kr[NKR > 0 ? NKR : 1], rr[NRR > 0 ? NRR : 1];
    const uint32_t lane_off = (uint32_t)tid * 16u;   // this thread's byte offset in an LDS slot
    // this wave's element offset in an LDS slot, redefined (opaquely) every
    // date so the direct loads' LDS addresses are formed where they are used
    // rather than all kept in scalar registers for the whole sweep
    uint32_t wave_el = (uint32_t)wave * 64u;
    // request slot j of `row`: this wave's 64 slots of an LDS slot receive
    // lane l's 16 bytes at +16 l; register and re-read slots load into
    // their registers
    auto request = [&](const float *row, auto jc) {
        constexpr int j = decltype(jc)::value;
        if constexpr (j < NKL) {
            __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(row + io.tile0), (short)0, TileIO<float, PPT, WG>::kTileBytes, 0x00020000);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                rs, (__attribute__((address_space(3))) void *)(resident_slot<j, NKL>() + wave_el), 16, io.voff,
                (uint32_t)j * JS * 4u, 0, 0);
        } else if constexpr (j < NKL + NKR) {
            kr[j - NKL] = io.load(row, j);
        } else {
            rr[j - NKL - NKR] = io.load(row, j);
        }
    };
    // slot j's values; in the moment pass an LDS slot first waits for its
    // load (the compiler's waits cover the register slots)
    auto slot = [&](auto jc, bool moment) -> Vec<float> {
        constexpr int j = decltype(jc)::value;
        if constexpr (j < NKL) {
            if (moment) wait_vmcnt<(PF < NVEC - 1 - j ? PF : NVEC - 1 - j)>();
            return read_slot(resident_slot<j, NKL>(), lane_off);
        } else if constexpr (j < NKL + NKR) {
            return kr[j - NKL];
        } else {
            return rr[j - NKL - NKR];
        }
    };

    DC dcc = dconst(M - 1);
    {
        const float *row = S + (size_t)(M - 2) * ld;
        static_for<0, PF>([&](auto jc) { request(row, jc); });
    }
    for (int k = M - 1; k >= 1; --k) {
        asm volatile("" : "+s"(wave_el));
        const double xa = dcc.xa, dk = dcc.disc;
        // the abscissa offset in vector registers once per date (an fma
        // takes one scalar operand: xa)
        double xb = dcc.xb;
        asm volatile("" : "+v"(xb));
        const DC dcn = dconst(k >= 2 ? k - 1 : 1);
        uint64_t stamp[3];
        stamp[2] = __builtin_amdgcn_s_memrealtime();
        const float *row = S + (size_t)(k - 1) * ld;

        // moment pass.  tv is the row the device-wide sum takes: [count,
        // Gram sums q = 1..2D, right-hand side q = 0..D, count]
        double tv[NV];
#pragma unroll
        for (int q = 1; q < NV - 1; ++q) tv[q] = 0.0;
        double *A = tv + 1, *R = tv + NA;
        uint32_t cnt = 0;
        Vec<float> mpend, mq[3];
        constexpr int NQ = NKL / 4 * 4;
        static_for<0, NVEC>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            if constexpr (j + PF < NVEC) request(row, Ic<j + PF>{});
            Vec<float> v;
            if constexpr (j < NQ && j % 4 == 0) {
                wait_vmcnt<(PF - 3 < NVEC - 4 - j ? PF - 3 : NVEC - 4 - j)>();
                read_slot4(resident_slot<j, NKL>(), resident_slot<j + 1, NKL>(), resident_slot<j + 2, NKL>(),
                           resident_slot<j + 3, NKL>(), lane_off, v, mq[0], mq[1], mq[2]);
            } else if constexpr (j < NQ) {
                v = mq[j % 4 - 1];
            } else if constexpr (j < NKL && (j - NQ) % 2 == 0 && j + 1 < NKL) {
                wait_vmcnt<(PF - 1 < NVEC - 2 - j ? PF - 1 : NVEC - 2 - j)>();
                read_slot2(resident_slot<j, NKL>(), resident_slot<j + 1, NKL>(), lane_off, v, mpend);
            } else if constexpr (j < NKL && (j - NQ) % 2 == 1) {
                v = mpend;
            } else {
                v = slot(jc, true);
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const bool itm = CALL ? v.v[e] > kthr : v.v[e] < kthr;
                cnt += (uint32_t)__builtin_popcountll(__builtin_amdgcn_ballot_w64(itm));
                asm volatile("" : "+s"(cnt));   // one running count, not one register per path
                resident_moments<D>(A, R, (double)v.v[e], (double)pv[j * 4 + e], itm, xa, xb);
            }
            __builtin_amdgcn_sched_barrier(0);
        });

        // the register part as new values for the update, so nothing derived
        // from them in the moment pass (conversions, masks) is kept for it
#pragma unroll
        for (int jj = 0; jj < NKR; ++jj)
#pragma unroll
            for (int e = 0; e < 4; ++e) asm volatile("" : "+v"(kr[jj].v[e]));
        tv[0] = 0.0;
        tv[NV - 1] = (double)cnt;   // wave-uniform: summed over the waves only
        group_sum<NV, 1, WG>(tv, s_red);
        tv[0] = tv[NV - 1];
        ++epoch;
        stamp[0] = stamp[1] = __builtin_amdgcn_s_memrealtime();
        if (!allreduce<NV, RW, WG>(tv, gid, G, a.rows, a.sync, a.err, epoch, a.spin_limit, s_tot, s_red, s_flag)) {
            alive = false;
            return;
        }
        if (wave == 0) solve_and_record_wave<D>(a, gid, k, s_tot, s_beta, s_L, stamp);
        __syncthreads();

        // a date that allows no exercise runs the same update with a strike
        // threshold no path passes (branch-free: no copies of the cashflows)
        const bool solved = s_beta[8] != 0.0;
        const float kthr_u = solved ? kthr : (CALL ? __int_as_float(0x7f800000) : __int_as_float(0xff800000));
        double gam[D + 1];
#pragma unroll
        for (int q = 0; q <= D; ++q) gam[q] = uniform_f64(s_beta[q]);
        const double dsg = dk * sg, dnsk = dk * nsk;
        // the next date's slab (the last date requests date 1 again, unused)
        const float *nrow = S + (size_t)(k >= 2 ? k - 2 : 0) * ld;
        // LDS slots in fours, then a pair: the first slot's read also fetches
        // the next ones
        Vec<float> pend, uq[3];
        constexpr int UQ = NKL / 4 * 4;
        static_for<0, NVEC>([&](auto tc) {
            constexpr int t = decltype(tc)::value;
            // the re-read slots again, PF ahead
            if constexpr (t + PF >= NKL + NKR && t + PF < NVEC) request(row, Ic<t + PF>{});
            Vec<float> v;
            if constexpr (t < UQ && t % 4 == 0) {
                read_slot4(resident_slot<t, NKL>(), resident_slot<t + 1, NKL>(), resident_slot<t + 2, NKL>(),
                           resident_slot<t + 3, NKL>(), lane_off, v, uq[0], uq[1], uq[2]);
            } else if constexpr (t < UQ) {
                v = uq[t % 4 - 1];
            } else if constexpr (t < NKL && (t - UQ) % 2 == 0 && t + 1 < NKL) {
                read_slot2(resident_slot<t, NKL>(), resident_slot<t + 1, NKL>(), lane_off, v, pend);
            } else if constexpr (t < NKL && (t - UQ) % 2 == 1) {
                v = pend;
            } else {
                v = slot(tc, false);
            }
#pragma unroll
            for (int e = 0; e < 4; ++e)
                pv[t * 4 + e] = resident_update<CALL, D>(v.v[e], pv[t * 4 + e], kthr_u, xa, xb, dsg, dnsk, gam);
            // over the last PF slots, the first PF slots of the next date
            // (slot t - (NVEC - PF) was read PF slots ago and is free)
            if constexpr (t >= NVEC - PF) request(nrow, Ic<t - (NVEC - PF)>{});
            __builtin_amdgcn_sched_barrier(0);
        });
        dcc = dcn;
        __syncthreads();   // s_beta reuse
    }
}

// LDS of one sweep workgroup.
template <typename T, int PPT, bool LAG, int WG>
struct SweepLds {
    static constexpr bool KEEP = SweepShape<T, PPT>::KEEP;
    double red[WG / 64][32];
    double red2[WG / 64][32];
    double tot[32];
    double beta[10];
    double L[KEEP ? 1 : 8][8];
    double w[KEEP ? 1 : 32];
    // Laguerre weights of a KEEP tile, [2 dates][path][thread]
    double wl[LAG && KEEP ? 2 * PPT * WG : 1];
    // component-major partials of the LDS group sums (512-thread groups):
    // [8][WG]; consecutive sums are separated by barriers
    double x[KEEP && WG == 512 ? 8 * WG : 1];
    DateConst dc[(KEEP || Resident<T, PPT, WG, LAG>::on) ? 1 : kMaxDates + 1];
    // streamed tiles: the first vectors of each thread's slab, kept from the
    // moment pass for the update ([vector][thread])
    Vec<T> keep[stream_keep_vecs<T, PPT, WG, LAG>() > 0 ? stream_keep_vecs<T, PPT, WG, LAG>() * WG : 1];
    int flag[2 + WG / 64];
};

// SIDE: 1 call, 2 put (slab-resident tiles are compiled per payoff side), 0
// either (read from the arguments).
template <typename T, int PPT, int D, bool LAG, int WG, int SIDE = 0>
__device__ __forceinline__ void sweep_body(const SweepArgs &a, const T *__restrict__ S, uint32_t gid,
                                           uint32_t e0, T (&pv)[PPT], uint32_t &epoch, bool &alive,
                                           SweepLds<T, PPT, LAG, WG> &L)
{
    const TileIO<T, PPT, WG> io(gid, e0);
    sweep_terminal<T, PPT, WG>(a, S, io, pv);
    if constexpr (SweepShape<T, PPT>::KEEP) {
        sweep_keep<T, PPT, D, LAG, WG>(a, S, gid, io, pv, epoch, alive, L.red, L.red2, L.tot, L.beta, L.wl, L.x,
                                       L.flag);
    } else if constexpr (Resident<T, PPT, WG, LAG>::on) {
        static_assert(SIDE == 1 || SIDE == 2, "slab-resident tiles are compiled per payoff side");
        sweep_resident<PPT, D, SIDE == 1>(a, S, gid, io, pv, epoch, alive, L.red, L.tot, L.beta, L.L, L.w, L.flag);
    } else {
        sweep_stream<T, PPT, D, LAG, WG>(a, S, gid, io, pv, epoch, alive, L.red, L.tot, L.beta, L.L, L.w, L.dc,
                                         L.keep, L.flag);
    }
}

// Epilogue (eqs. (6)-(8)): FP64 sums of the discounted cashflows and their
// squares through one more device-wide sum; group 0 writes the result.  The
// sums are taken about the shift c = max(h(S0), 0), a value of the order of
// the mean for options in the money and zero otherwise, so the variance
// (sum of squares minus the squared sum over n) cancels only to the order of
// (mean - c)^2 / variance instead of mean^2 / variance.
__device__ __forceinline__ double moment_shift(const SweepArgs &a)
{
    const double h0 = a.is_call ? a.S0 - a.K : a.K - a.S0;
    return h0 > 0.0 ? h0 : 0.0;
}

template <typename T, int PPT, int D, int WG>
__device__ __forceinline__ void sweep_final(const SweepArgs &a, uint32_t gid, uint32_t e0,
                                            const T (&pv)[PPT], uint32_t epoch, double (*s_red)[32],
                                            double *s_tot, int *s_flag)
{
    constexpr int VW = 16 / sizeof(T), NVEC = PPT / VW;
    constexpr uint32_t JS = 64 * VW;
    const int tid = threadIdx.x;
    const int64_t N = a.N;
    const double c = moment_shift(a);
    double fin[2] = {0.0, 0.0};
    T *pvo = (T *)a.pv_out;
#pragma unroll
    for (int jj = 0; jj < NVEC; ++jj) {
        Vec<T> o;
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            const T v = pv[jj * VW + e];   // padded paths hold 0
            o.v[e] = v;
            const double d = (int64_t)(e0 + (uint32_t)jj * JS + (uint32_t)e) < N ? (double)v - c : 0.0;
            fin[0] += d;
            fin[1] += d * d;
        }
        *reinterpret_cast<Vec<T> *>(pvo + e0 + (uint32_t)jj * JS) = o;
    }
    group_sum<2, 0, WG>(fin, s_red);
    ++epoch;
    const uint32_t G = (uint32_t)a.G;
    if (!allreduce<2, row_words(D), WG>(fin, gid, G, a.rows, a.sync, a.err, epoch, a.spin_limit, s_tot, s_red,
                                    s_flag))
        return;
    if (gid == 0) {
        if (tid == 0) {
            const double n = (double)N;
            const double s1 = s_tot[0], s2 = s_tot[1];   // about c
            const double mean = c + s1 / n;
            double var = N > 1 ? (s2 - s1 * (s1 / n)) / (n - 1.0) : 0.0;
            if (var < 0.0) var = 0.0;
            double price = mean, se = sqrt(var / n), t0 = 0.0;
            if (a.allow_exercise) {
                const double h0 = a.is_call ? a.S0 - a.K : a.K - a.S0;
                if (h0 > mean) { price = h0; se = 0.0; t0 = 1.0; }
            }
            double skipped = 0.0;
            if (a.allow_exercise)
                for (int k = 1; k < a.M; ++k) skipped += a.rec[(size_t)k * kRec + 8] == 0.0 ? 1.0 : 0.0;
            a.result[0] = price;
            a.result[1] = se;
            a.result[2] = mean;
            a.result[3] = t0;
            a.result[4] = skipped;
            a.result[5] = 0.0;
            if (a.rep_out) {
                // randomised QMC: replicate prices of earlier launches are
                // visible (stream order); the last replicate aggregates
                a.rep_out[a.rep] = price;
                if (a.rep + 1 == a.n_rep) {
                    double s1r = 0.0;
                    for (int q = 0; q < a.n_rep; ++q) s1r += a.rep_out[q];
                    const double m = s1r / (double)a.n_rep;
                    double s2r = 0.0;
                    for (int q = 0; q < a.n_rep; ++q) s2r += (a.rep_out[q] - m) * (a.rep_out[q] - m);
                    a.result[0] = m;
                    a.result[1] = a.n_rep > 1 ? sqrt(s2r / (double)(a.n_rep - 1) / (double)a.n_rep) : 0.0;
                }
            }
        }
    }
}

template <typename T, int PPT, int WG>
__device__ __forceinline__ uint32_t tile_e0(uint32_t gid)
{
    constexpr int VW = 16 / sizeof(T);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    return (uint32_t)((int64_t)gid * WG * PPT + (int64_t)wave * 64 * PPT + lane * VW);
}

// WG: threads per group, 256 or (register-resident tiles) 512: two waves
// of one group per SIMD, so one wave's dependent binary64 latencies and
// scalar/LDS issue slots overlap the other's vector work.
template <typename T, int PPT, int D, bool LAG, int WG, int SIDE = 0>
__global__ void __launch_bounds__(WG)
__attribute__((amdgpu_waves_per_eu(WG == 512 ? 2 : SweepShape<T, PPT>::template waves<D, LAG>())))
sweep_kernel(SweepArgs a, const T *__restrict__ S)
{
    static_assert(PPT % (16 / sizeof(T)) == 0, "PPT must be a multiple of the vector width");
    __shared__ SweepLds<T, PPT, LAG, WG> L;

    const uint32_t gid = blockIdx.x;
    const uint32_t e0 = tile_e0<T, PPT, WG>(gid);
    T pv[PPT];
    uint32_t epoch = 0;
    bool alive = true;
    sweep_body<T, PPT, D, LAG, WG, SIDE>(a, S, gid, e0, pv, epoch, alive, L);
    if (!alive) return;
    sweep_final<T, PPT, D, WG>(a, gid, e0, pv, epoch, L.red, L.tot, L.flag);
}

template <typename T, int PPT, int D, bool LAG>
__global__ void __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(SweepShape<T, PPT>::template waves<D, LAG>())))
sweep_batch_kernel(const BatchOpt *__restrict__ opts, const int32_t *__restrict__ tile_opt,
                   BatchGlobal g)
{
    __shared__ SweepLds<T, PPT, LAG, kWG> L;
    __shared__ int s_claim;

    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) {
            int t = (int)__hip_atomic_fetch_add(g.claim, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (ld_agent(g.err) != 0u) t = g.total_tiles;
            s_claim = t;
        }
        __syncthreads();
        // (wave-uniform: the descriptor and everything derived from it then
        // live in scalar registers)
        const int t = __builtin_amdgcn_readfirstlane(s_claim);
        if (t >= g.total_tiles) return;
        const BatchOpt o = opts[tile_opt[t]];
        SweepArgs a;
        a.S = o.S;
        a.pv_out = o.pv;
        a.rows = o.rows;
        a.rec = o.rec;
        a.result = o.result;
        a.sync = o.sync;
        a.err = g.err;
        a.datec = o.datec;
        a.N = o.N; a.ld = o.ld;
        a.M = o.M; a.G = o.G;
        a.is_call = o.is_call; a.allow_exercise = o.allow_exercise;
        a.laguerre = LAG; a.degree = D;
        a.S0 = o.S0; a.K = o.K;
        a.spin_limit = g.spin_limit;
        a.pad = 0;
        a.rep_out = nullptr; a.rep = 0; a.n_rep = 0;
        const uint32_t gid = (uint32_t)(t - o.tile_base);
        const uint32_t e0 = tile_e0<T, PPT, kWG>(gid);
        T pv[PPT];
        uint32_t epoch = 0;
        bool alive = true;
        sweep_body<T, PPT, D, LAG, kWG>(a, (const T *)o.S, gid, e0, pv, epoch, alive, L);
        if (!alive) return;
        sweep_final<T, PPT, D, kWG>(a, gid, e0, pv, epoch, L.red, L.tot, L.flag);
    }
}

// ---------------------------------------------------------------------------
// Kernel addresses by (paths per thread, degree) for one precision and basis
// kind; `kind` selects the single-option kernel with 256-thread groups (0),
// the many-option kernel (1) or the single-option kernel with 512-thread
// groups (2; for slab-resident tiles the put form), and the call form of a
// slab-resident tile (3).  Null where not built.  Each (precision, basis
// kind) pair is instantiated in its own translation unit.
// ---------------------------------------------------------------------------
template <typename T, int PPT, int D, bool LAG, int KIND>
inline const void *sweep_addr()
{
    constexpr bool res = Resident<T, PPT, 512, LAG>::on;
    if constexpr (KIND == 1) return (const void *)&sweep_batch_kernel<T, PPT, D, LAG>;
    else if constexpr (KIND == 3) {
        if constexpr (res) return (const void *)&sweep_kernel<T, PPT, D, LAG, 512, 1>;
        else return nullptr;
    } else if constexpr (KIND == 2) return (const void *)&sweep_kernel<T, PPT, D, LAG, 512, res ? 2 : 0>;
    else return (const void *)&sweep_kernel<T, PPT, D, LAG, kWG>;
}

template <typename T, int PPT, bool LAG, int KIND>
inline const void *sweep_entry(int degree)
{
    switch (degree) {
    case 0: return sweep_addr<T, PPT, 0, LAG, KIND>();
    case 1: return sweep_addr<T, PPT, 1, LAG, KIND>();
    case 2: return sweep_addr<T, PPT, 2, LAG, KIND>();
    case 3: return sweep_addr<T, PPT, 3, LAG, KIND>();
    case 4: return sweep_addr<T, PPT, 4, LAG, KIND>();
    case 5: return sweep_addr<T, PPT, 5, LAG, KIND>();
    case 6: return sweep_addr<T, PPT, 6, LAG, KIND>();
    default: return nullptr;
    }
}

// Paths per thread built.  binary32: 4, 16, 64, 128 (256-thread groups),
// 4, 8, 64, 128 (512-thread groups), batch 16, 64.  binary64: 2, 8, 16, 64 (256), 2, 4,
// 8 (512), batch 8, 32.
template <typename T, bool LAG>
inline const void *sweep_table(int ppt, int degree, int kind)
{
    if constexpr (sizeof(T) == 8) {
        if (kind == 3) return nullptr;   // no slab-resident binary64 tiles
        if (kind == 1) {
            switch (ppt) {
            case 8: return sweep_entry<T, 8, LAG, 1>(degree);
            case 32: return sweep_entry<T, 32, LAG, 1>(degree);
            default: return nullptr;
            }
        }
        if (kind == 2) {
            switch (ppt) {
            case 2: return sweep_entry<T, 2, LAG, 2>(degree);
            case 4: return sweep_entry<T, 4, LAG, 2>(degree);
            case 8: return sweep_entry<T, 8, LAG, 2>(degree);
            default: return nullptr;
            }
        }
        switch (ppt) {
        case 2: return sweep_entry<T, 2, LAG, 0>(degree);
        case 8: return sweep_entry<T, 8, LAG, 0>(degree);
        case 16: return sweep_entry<T, 16, LAG, 0>(degree);
        case 64: return sweep_entry<T, 64, LAG, 0>(degree);
        default: return nullptr;
        }
    } else {
        if (kind == 1) {
            switch (ppt) {
            case 16: return sweep_entry<T, 16, LAG, 1>(degree);
            case 64: return sweep_entry<T, 64, LAG, 1>(degree);
            default: return nullptr;
            }
        }
        if (kind == 2) {
            switch (ppt) {
            case 4: return sweep_entry<T, 4, LAG, 2>(degree);
            case 8: return sweep_entry<T, 8, LAG, 2>(degree);
            case 64: return sweep_entry<T, 64, LAG, 2>(degree);
            case 128: return sweep_entry<T, 128, LAG, 2>(degree);
            default: return nullptr;
            }
        }
        if (kind == 3) {
            switch (ppt) {
            case 64: return sweep_entry<T, 64, LAG, 3>(degree);
            case 128: return sweep_entry<T, 128, LAG, 3>(degree);
            default: return nullptr;
            }
        }
        switch (ppt) {
        case 4: return sweep_entry<T, 4, LAG, 0>(degree);
        case 16: return sweep_entry<T, 16, LAG, 0>(degree);
        case 64: return sweep_entry<T, 64, LAG, 0>(degree);
        case 128: return sweep_entry<T, 128, LAG, 0>(degree);
        default: return nullptr;
        }
    }
}

}  // namespace amq
