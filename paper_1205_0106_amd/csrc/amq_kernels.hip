// amq_kernels.hip — gfx950 kernels for quasi-Monte Carlo American option
// valuation (Cvetanoska & Stojanovski; method in Sections III.D, III.E, V).
//
//   gen_kernel:   Sobol point -> Moro inverse normal -> Brownian bridge ->
//                 GBM value, stored path-contiguous as S[date][path].
//   sweep_kernel: persistent backward induction over the exercise dates:
//                 per-date in-the-money basis moments, a device-wide
//                 fixed-order reduction, an FP64 normal-equation solve and the
//                 exercise update, then the FP64 discounted-cashflow mean.
//
// Compiled for gfx950 only.
#include "amq_internal.h"

#include <math.h>

namespace amq {

// ---------------------------------------------------------------------------
// Moro's inverse cumulative normal (Section III.D names it; coefficients from
// Moro 1995, "The full Monte", Risk 8(2)).  Central region |u - 1/2| < 0.42:
// Beasley–Springer rational function; tails: polynomial in log(-log q) where
// q is the tail probability, taken from the exact integer complement.
// ---------------------------------------------------------------------------
#define AMQ_A0 2.50662823884
#define AMQ_A1 -18.61500062529
#define AMQ_A2 41.39119773534
#define AMQ_A3 -25.44106049637
#define AMQ_B0 -8.47351093090
#define AMQ_B1 23.08336743743
#define AMQ_B2 -21.06224101826
#define AMQ_B3 3.13082909833
#define AMQ_C0 0.3374754822726147
#define AMQ_C1 0.9761690190917186
#define AMQ_C2 0.1607979714918209
#define AMQ_C3 0.0276438810333863
#define AMQ_C4 0.0038405729373609
#define AMQ_C5 0.0003951896511919
#define AMQ_C6 0.0000321767881768
#define AMQ_C7 0.0000002888167364
#define AMQ_C8 0.0000003960315187

// binary32: both branches are evaluated (every 64-point Sobol block has tail
// lanes), hardware log2/rcp; y and q come exactly from the 32-bit integer.
__device__ __forceinline__ float inv_normal_f32(uint32_t x)
{
    const float s = 0x1p-32f;
    const int32_t d = (int32_t)(x - 0x80000000u);
    const float y = (float)d * s;
    const float r = y * y;
    const float num = y * fmaf(fmaf(fmaf((float)AMQ_A3, r, (float)AMQ_A2), r, (float)AMQ_A1), r,
                               (float)AMQ_A0);
    const float den = fmaf(fmaf(fmaf(fmaf((float)AMQ_B3, r, (float)AMQ_B2), r, (float)AMQ_B1), r,
                                (float)AMQ_B0), r, 1.0f);
    const float zc = num * __builtin_amdgcn_rcpf(den);
    const uint32_t tq = d < 0 ? x : 0u - x;          // tail integer: x or 2^32 - x
    const float q = (float)tq * s;
    const float ln2 = 0.69314718055994531f;
    const float t = __builtin_amdgcn_logf(-__builtin_amdgcn_logf(q) * ln2) * ln2;
    float v = (float)AMQ_C8;
    v = fmaf(v, t, (float)AMQ_C7);
    v = fmaf(v, t, (float)AMQ_C6);
    v = fmaf(v, t, (float)AMQ_C5);
    v = fmaf(v, t, (float)AMQ_C4);
    v = fmaf(v, t, (float)AMQ_C3);
    v = fmaf(v, t, (float)AMQ_C2);
    v = fmaf(v, t, (float)AMQ_C1);
    v = fmaf(v, t, (float)AMQ_C0);
    const float zt = d < 0 ? -v : v;
    return fabsf(y) < 0.42f ? zc : zt;
}

// binary64: u, u - 1/2 and 1 - u are exact for u = x 2^-32.
__device__ __forceinline__ double inv_normal_f64(uint32_t x)
{
    const double s = 0x1p-32;
    const double y = ((double)x - 2147483648.0) * s;
    if (fabs(y) < 0.42) {
        const double r = y * y;
        const double num = y * (((AMQ_A3 * r + AMQ_A2) * r + AMQ_A1) * r + AMQ_A0);
        const double den = (((AMQ_B3 * r + AMQ_B2) * r + AMQ_B1) * r + AMQ_B0) * r + 1.0;
        return num / den;
    }
    const double q = y < 0.0 ? (double)x * s : (4294967296.0 - (double)x) * s;
    const double t = log(-log(q));
    double v = AMQ_C8;
    v = v * t + AMQ_C7;
    v = v * t + AMQ_C6;
    v = v * t + AMQ_C5;
    v = v * t + AMQ_C4;
    v = v * t + AMQ_C3;
    v = v * t + AMQ_C2;
    v = v * t + AMQ_C1;
    v = v * t + AMQ_C0;
    return y < 0.0 ? -v : v;
}

// Shifted (randomised) points sit at cell midpoints u = (x + 1/2) 2^-32, so a
// shifted integer 0 still maps to a finite normal.
__device__ __forceinline__ float inv_normal_mid_f32(uint32_t x)
{
    const float s = 0x1p-32f;
    const int32_t d = (int32_t)(x - 0x80000000u);
    const float y = ((float)d + 0.5f) * s;
    const float r = y * y;
    const float num = y * fmaf(fmaf(fmaf((float)AMQ_A3, r, (float)AMQ_A2), r, (float)AMQ_A1), r,
                               (float)AMQ_A0);
    const float den = fmaf(fmaf(fmaf(fmaf((float)AMQ_B3, r, (float)AMQ_B2), r, (float)AMQ_B1), r,
                                (float)AMQ_B0), r, 1.0f);
    const float zc = num * __builtin_amdgcn_rcpf(den);
    const uint32_t tq = d < 0 ? x : 0u - x;
    const float q = fmaf((float)tq, s, d < 0 ? 0x1p-33f : -0x1p-33f);
    const float ln2 = 0.69314718055994531f;
    const float t = __builtin_amdgcn_logf(-__builtin_amdgcn_logf(q) * ln2) * ln2;
    float v = (float)AMQ_C8;
    v = fmaf(v, t, (float)AMQ_C7);
    v = fmaf(v, t, (float)AMQ_C6);
    v = fmaf(v, t, (float)AMQ_C5);
    v = fmaf(v, t, (float)AMQ_C4);
    v = fmaf(v, t, (float)AMQ_C3);
    v = fmaf(v, t, (float)AMQ_C2);
    v = fmaf(v, t, (float)AMQ_C1);
    v = fmaf(v, t, (float)AMQ_C0);
    const float zt = d < 0 ? -v : v;
    return fabsf(y) < 0.42f ? zc : zt;
}

__device__ __forceinline__ double inv_normal_mid_f64(uint32_t x)
{
    const double s = 0x1p-32;
    const double y = ((double)x + 0.5 - 2147483648.0) * s;
    if (fabs(y) < 0.42) {
        const double r = y * y;
        const double num = y * (((AMQ_A3 * r + AMQ_A2) * r + AMQ_A1) * r + AMQ_A0);
        const double den = (((AMQ_B3 * r + AMQ_B2) * r + AMQ_B1) * r + AMQ_B0) * r + 1.0;
        return num / den;
    }
    const double q = y < 0.0 ? ((double)x + 0.5) * s : (4294967296.0 - (double)x - 0.5) * s;
    const double t = log(-log(q));
    double v = AMQ_C8;
    v = v * t + AMQ_C7;
    v = v * t + AMQ_C6;
    v = v * t + AMQ_C5;
    v = v * t + AMQ_C4;
    v = v * t + AMQ_C3;
    v = v * t + AMQ_C2;
    v = v * t + AMQ_C1;
    v = v * t + AMQ_C0;
    return y < 0.0 ? -v : v;
}

template <typename T, bool MID> __device__ __forceinline__ T inv_normal(uint32_t x);
template <> __device__ __forceinline__ float inv_normal<float, false>(uint32_t x) { return inv_normal_f32(x); }
template <> __device__ __forceinline__ double inv_normal<double, false>(uint32_t x) { return inv_normal_f64(x); }
template <> __device__ __forceinline__ float inv_normal<float, true>(uint32_t x) { return inv_normal_mid_f32(x); }
template <> __device__ __forceinline__ double inv_normal<double, true>(uint32_t x) { return inv_normal_mid_f64(x); }

size_t generate_lds_bytes(int M)
{
    return (size_t)M * 16 * sizeof(uint32_t) + (size_t)kWaves * M * 2 * sizeof(uint32_t);
}

// ---------------------------------------------------------------------------
// Generation.  One wave owns 64 consecutive paths i = 64w + lane (Sobol index
// n = i + 1) and walks R such blocks.  Sobol (Gray-code order): for n = h + l
// with h a multiple of 64 and l < 64, gray(n) = gray(h) ^ gray(l), so
//   x_j(n) = X_j(h) ^ x_j^lo(l).
// X_j(h) is wave-uniform (kept per wave in LDS as the pair for h = 64w and
// h = 64(w+1), because lane 63 has n = 64(w+1)); x^lo comes from two 8-entry
// lane tables per dimension (bits 0-2 and 3-5 of gray(l)).  Moving to the
// next block: X(64(w+1)) = X(64w) ^ V[5] ^ V[6 + ctz(w+1)].
//
// The bridge runs in depth-first order over a register window of ancestor
// values (slots chosen on the host), so a path never needs more than
// log2(M) + 2 live values; dimension order follows the breadth-first node
// numbering, which only changes the order the Sobol dimensions are read.
// ---------------------------------------------------------------------------
// One workgroup's share: `init` (the group holding the option's first block)
// writes the option's date constants and clears its barrier words; wave
// blocks [w0, w1) are generated.
template <typename T, int WHAT, bool MID>
__device__ __forceinline__ void gen_body(const GenArgs &a, const uint32_t *__restrict__ V,
                                         const BridgeNode *__restrict__ sched,
                                         const uint32_t *__restrict__ shift, bool init, int64_t w0,
                                         int64_t w1)
{
    extern __shared__ uint32_t lds[];
    const int M = a.M;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t *ttab = lds;                                   // [M][16]
    uint32_t *xw = lds + (size_t)M * 16 + (size_t)wave * M * 2;   // [M][2]

    if (init && WHAT == 0) {
        if (tid < 16) a.sync[tid] = 0u;
        for (int k = tid; k <= M; k += kWG) {
            const double tk = (double)k * a.T / (double)M;
            DateConst c;
            c.disc = exp(-a.r * tk);
            const double mean = a.S0 / a.K * exp(a.r * tk);
            const double sd = mean * sqrt(expm1(a.sigma * a.sigma * tk));
            c.xa = k > 0 ? 1.0 / (a.K * sd) : 0.0;
            c.xb = k > 0 ? -mean / sd : 0.0;
            c.pad = 0.0;
            a.datec[k] = c;
        }
    }

    for (int e = tid; e < M * 16; e += kWG) {
        const int j = e >> 4, h = (e >> 3) & 1, idx = e & 7;
        const uint32_t *v = V + (size_t)j * 32 + 3 * h;
        uint32_t t = 0u;
        if (idx & 1) t ^= v[0];
        if (idx & 2) t ^= v[1];
        if (idx & 4) t ^= v[2];
        ttab[e] = t;
    }

    if (w0 < w1) {
        const uint64_t n0 = (uint64_t)w0 << 6;
        const uint64_t g0 = n0 ^ (n0 >> 1);
        const int c = min(__builtin_ctzll((uint64_t)w0 + 1u) + 6, 31);
        for (int j = lane; j < M; j += 64) {
            const uint32_t *v = V + (size_t)j * 32;
            uint32_t xa = 0u;
            for (int b = 5; b < 32; ++b)
                if ((g0 >> b) & 1u) xa ^= v[b];
            xw[2 * j] = xa;
            xw[2 * j + 1] = xa ^ v[5] ^ v[c];
        }
    }
    __syncthreads();

    const int lo = lane < 63 ? lane + 1 : 0;
    const int gl = lo ^ (lo >> 1);
    const int offL = gl & 7, offH = 8 + (gl >> 3);
    const int xsel = lane == 63 ? 1 : 0;

    const T S0 = (T)a.S0;
    // binary32 uses exp2: fold log2(e) into the drift and volatility
    const T mu = sizeof(T) == 4 ? (T)(a.mu * 1.4426950408889634) : (T)a.mu;
    const T vol = sizeof(T) == 4 ? (T)(a.vol * 1.4426950408889634) : (T)a.vol;

    T W[kMaxSlots];
#pragma unroll
    for (int q = 0; q < kMaxSlots; ++q) W[q] = T(0);

    for (int64_t w = w0; w < w1; ++w) {
        const int64_t i = (w << 6) + lane;
        const bool valid = i < a.N;
        if (WHAT == 0 && (w << 6) >= a.N) {
            // padding block: S = K on every date (out of the money, see the sweep)
            const T Kp = (T)a.K;
            for (int m = 0; m < M; ++m) ((T *)a.S)[(size_t)m * a.ld + i] = Kp;
            continue;
        }
        for (int s = 0; s < M; ++s) {
            const BridgeNode nd = sched[s];
            const int j = nd.dim;
            uint32_t x = xw[2 * j + xsel] ^ ttab[j * 16 + offL] ^ ttab[j * 16 + offH];
            if (MID) x ^= shift[j];
            if (WHAT == 1) {
                if (valid) ((uint32_t *)a.S)[(size_t)j * a.ld + i] = x;
                continue;
            }
            const T z = inv_normal<T, MID>(x);
            if (WHAT == 2) {
                if (valid) ((double *)a.S)[(size_t)j * a.ld + i] = (double)z;
                continue;
            }
            T wv;
            if (sizeof(T) == 4)
                wv = (T)nd.fwl * W[nd.sl] + (T)nd.fwr * W[nd.sr] + (T)nd.fsd * z;
            else
                wv = (T)nd.wl * W[nd.sl] + (T)nd.wr * W[nd.sr] + (T)nd.sd * z;
            W[nd.dst] = wv;
            T Sv;
            if (sizeof(T) == 4)
                Sv = S0 * __builtin_amdgcn_exp2f(fmaf((float)vol, (float)wv, (float)mu * nd.fm));
            else
                Sv = S0 * exp((double)mu * (double)nd.m + (double)vol * (double)wv);
            ((T *)a.S)[(size_t)(nd.m - 1) * a.ld + i] = valid ? Sv : (T)a.K;
        }
        if (w + 1 < w1) {
            const int c = min(__builtin_ctzll((uint64_t)w + 2u) + 6, 31);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (int j = lane; j < M; j += 64) {
                const uint32_t xb = xw[2 * j + 1];
                xw[2 * j] = xb;
                xw[2 * j + 1] = xb ^ V[(size_t)j * 32 + 5] ^ V[(size_t)j * 32 + c];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
}

template <typename T, int WHAT, bool MID>
__global__ void __launch_bounds__(kWG)
gen_kernel(GenArgs a, const uint32_t *__restrict__ V, const BridgeNode *__restrict__ sched,
           const uint32_t *__restrict__ shift)
{
    const int64_t gw = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    const int64_t w0 = gw * a.R;
    const int64_t w1 = min(w0 + (int64_t)a.R, a.nblocks);
    gen_body<T, WHAT, MID>(a, V, sched, shift, blockIdx.x == 0, w0, w1);
}

hipError_t launch_generate(const GenArgs &a, int fp64, hipStream_t s)
{
    const int64_t waves = (a.nblocks + a.R - 1) / a.R;
    const int64_t grid = (waves + kWaves - 1) / kWaves;
    const size_t lds = generate_lds_bytes(a.M);
    const dim3 g((unsigned)grid), b(kWG);
    const bool mid = a.shift != nullptr;
    if (a.what == 0) {
        if (fp64) {
            if (mid) hipLaunchKernelGGL((gen_kernel<double, 0, true>), g, b, lds, s, a, a.V, a.sched, a.shift);
            else     hipLaunchKernelGGL((gen_kernel<double, 0, false>), g, b, lds, s, a, a.V, a.sched, a.shift);
        } else {
            if (mid) hipLaunchKernelGGL((gen_kernel<float, 0, true>), g, b, lds, s, a, a.V, a.sched, a.shift);
            else     hipLaunchKernelGGL((gen_kernel<float, 0, false>), g, b, lds, s, a, a.V, a.sched, a.shift);
        }
    } else if (a.what == 1) {
        hipLaunchKernelGGL((gen_kernel<float, 1, false>), g, b, lds, s, a, a.V, a.sched, a.shift);
    } else {
        if (fp64) hipLaunchKernelGGL((gen_kernel<double, 2, false>), g, b, lds, s, a, a.V, a.sched, a.shift);
        else      hipLaunchKernelGGL((gen_kernel<float, 2, false>), g, b, lds, s, a, a.V, a.sched, a.shift);
    }
    return hipGetLastError();
}

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
__device__ bool wait_release(uint32_t *sync, uint32_t *err, uint32_t epoch, uint32_t limit)
{
    uint32_t it = 0;
    while (ld_agent(sync + 1) < epoch) {
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

// Publish this group's partial sums and arrive.  Returns (in every thread)
// whether this group arrived last for barrier `epoch`.
template <int NV>
__device__ bool arrive(const double (&v)[NV], double *part, uint32_t gid, uint32_t *sync,
                       uint32_t epoch, uint32_t G, int *s_flag)
{
    if (threadIdx.x == 0) {
        double *dst = part + (size_t)gid * kPartStride;
#pragma unroll
        for (int q = 0; q < NV; ++q) dst[q] = v[q];
        const uint32_t old = __hip_atomic_fetch_add(sync, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_flag[0] = (old + 1u == epoch * G) ? 1 : 0;
    }
    __syncthreads();
    return s_flag[0] != 0;
}

// Last group: fixed-order sum of all partial slots into tot[0..NV-1] (LDS).
template <int NV>
__device__ void reduce_partials(const double *part, uint32_t G, double *tot, double (*s_red8)[32])
{
    const int c = threadIdx.x & 31, sgrp = threadIdx.x >> 5;   // 8 groups of 32
    double v = 0.0;
    if (c < NV) {
        for (uint32_t g = sgrp; g < G; g += 8) v += part[(size_t)g * kPartStride + c];
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

// FP64 normal-equation solve for the p = D+1 coefficients from Hankel moments
// tot[0..2D] (sum of wA xs^q), tot[2D+1 .. 3D+1] (sum of wB xs^a pv) and the
// in-the-money count tot[3D+2].  Equilibrated Cholesky in LDS (one thread);
// a date with fewer in-the-money paths than p or a pivot below 1e-14 (on the
// unit-diagonal matrix) allows no exercise.  rec: [0..7] coefficients in the
// standardised basis, [8] solved flag, [9] count, [10..] the moments.
template <int D>
__device__ void solve_date(const double *tot, double *rec, double (*L)[8], double *w)
{
    constexpr int P = D + 1, NA = 2 * D + 1;
    const double n = tot[NA + P];
    bool ok = n >= (double)P;
    double *sc = w, *y = w + 8, *gam = w + 16;
    for (int i = 0; i < P; ++i) {
        const double d = tot[2 * i];
        ok = ok && (d > 0.0);
        sc[i] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
    }
    for (int j = 0; j < P && ok; ++j) {
        double d = tot[2 * j] * sc[j] * sc[j];
        for (int l = 0; l < j; ++l) d -= L[j][l] * L[j][l];
        ok = ok && (d > 1e-14);
        const double ljj = d > 0.0 ? sqrt(d) : 1.0;
        L[j][j] = ljj;
        for (int i = j + 1; i < P; ++i) {
            double e = tot[i + j] * sc[i] * sc[j];
            for (int l = 0; l < j; ++l) e -= L[i][l] * L[j][l];
            L[i][j] = e / ljj;
        }
    }
    if (ok) {
        for (int i = 0; i < P; ++i) {
            double e = tot[NA + i] * sc[i];
            for (int l = 0; l < i; ++l) e -= L[i][l] * y[l];
            y[i] = e / L[i][i];
        }
        for (int i = P - 1; i >= 0; --i) {
            double e = y[i];
            for (int l = i + 1; l < P; ++l) e -= L[l][i] * gam[l];
            gam[i] = e / L[i][i];
        }
    }
    for (int i = 0; i < 8; ++i) rec[i] = (i < P && ok) ? gam[i] * sc[i] : 0.0;
    rec[8] = ok ? 1.0 : 0.0;
    rec[9] = n;
    for (int q = 0; q < NA + P + 1 && q < 22; ++q) rec[10 + q] = tot[q];
}

template <typename T> __device__ __forceinline__ T lag_weight(T s, T wc);
// exp(-x/2) with x = S/K: binary32 via exp2 (wc = -log2(e)/(2K)), binary64 exact form
template <> __device__ __forceinline__ float lag_weight<float>(float s, float wc)
{
    return __builtin_amdgcn_exp2f(s * wc);
}
template <> __device__ __forceinline__ double lag_weight<double>(double s, double wc)
{
    return exp(s * wc);
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
    // register budget: STREAM kernels run 2 waves per SIMD (256 VGPRs)
    static constexpr int WAVES = KEEP ? 2 : 2;
};

// Per-thread in-the-money moments over a block of path values.
template <typename T, int D>
struct MomBlock {
    static constexpr int NA = 2 * D + 1, NB = D + 1;
    T am[NA], ab[NB];
    __device__ __forceinline__ void clear()
    {
#pragma unroll
        for (int q = 0; q < NA; ++q) am[q] = T(0);
#pragma unroll
        for (int q = 0; q < NB; ++q) ab[q] = T(0);
    }
    // s: path value, pvj: its cashflow discounted to t0
    __device__ __forceinline__ int add(T s, T pvj, bool valid, T K, bool call, T xa, T xb,
                                       bool lag, T wc)
    {
        const T h = call ? s - K : K - s;
        const bool itm = valid && (h > T(0));
        const T xs = s * xa + xb;
        T wA = T(1), wB = T(1);
        if (lag) {
            const T w = lag_weight<T>(s, wc);
            wA = w * w;
            wB = w;
        }
        T pa = itm ? wA : T(0);
        am[0] += pa;
#pragma unroll
        for (int q = 1; q < NA; ++q) { pa *= xs; am[q] += pa; }
        T pb = itm ? wB * pvj : T(0);
        ab[0] += pb;
#pragma unroll
        for (int q = 1; q < NB; ++q) { pb *= xs; ab[q] += pb; }
        return itm ? 1 : 0;
    }
    __device__ __forceinline__ void flush(double *acc) const
    {
#pragma unroll
        for (int q = 0; q < NA; ++q) acc[q] += (double)am[q];
#pragma unroll
        for (int q = 0; q < NB; ++q) acc[NA + q] += (double)ab[q];
    }
};

template <typename T, int D>
__device__ __forceinline__ T exercise_update(T s, T pvj, bool valid, T K, bool call, T xa, T xb,
                                             T dk, const T *gam, bool lag, T wc)
{
    constexpr int P = D + 1;
    const T h = call ? s - K : K - s;
    const T xs = s * xa + xb;
    T cont = gam[P - 1];
#pragma unroll
    for (int q = P - 2; q >= 0; --q) cont = cont * xs + gam[q];
    if (lag) cont *= lag_weight<T>(s, wc);
    const T ex = dk * h;
    return (valid && (h > T(0)) && (ex > cont)) ? ex : pvj;
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
//   arrive; the last group sums the partial slots in fixed order, solves and
//   publishes; the others wait (bounded) and read the coefficients;
//   exercise update.
// KEEP: path values held in registers across the barrier, next date
// prefetched before waiting.  Otherwise the date is streamed twice (moments,
// update) through a ring of PD vector loads in flight per thread.
// binary32 moments are summed over blocks of 8 paths, then carried in FP64.
// Rows are padded to a multiple of every tile size with S = K, so padded
// paths are never in the money and keep pv = 0: no bounds checks.
// ---------------------------------------------------------------------------
template <typename T, int PPT, int D>
__device__ __forceinline__ void sweep_body(const SweepArgs &a, const T *__restrict__ S, uint32_t gid,
                                           uint32_t e0, T (&pv)[PPT], uint32_t &epoch, bool &alive,
                                           double (*s_red)[32], double (*s_red8)[32], double *s_tot,
                                           double (*s_L)[8], double *s_w, double *s_beta, int *s_flag)
{
    using SH = SweepShape<T, PPT>;
    constexpr int VW = SH::VW, NVEC = SH::NVEC, PD = SH::PD;
    constexpr bool KEEP = SH::KEEP;
    constexpr int NA = 2 * D + 1, NB = D + 1, P = D + 1;
    constexpr int NV = NA + NB + 1;
    // binary32 block length (paths); it must divide PPT so every block is flushed
    constexpr int BLK = sizeof(T) == 4 ? (PPT < 8 ? PPT : 8) : PPT;
    static_assert(PPT % BLK == 0, "block length must divide the paths per thread");
    constexpr uint32_t JS = 64 * VW;                 // element stride between a lane's vectors

    const int tid = threadIdx.x;
    const int64_t ld = a.ld;
    const T K = (T)a.K;
    const bool call = a.is_call != 0;
    const bool lag = a.laguerre != 0;
    const T wc = sizeof(T) == 4 ? (T)(-1.4426950408889634 / (2.0 * a.K)) : (T)(-0.5 / a.K);
    const uint32_t G = (uint32_t)a.G;
    const int64_t tile0 = (int64_t)gid * kWG * PPT;
    const uint32_t voff = (e0 - (uint32_t)tile0) * (uint32_t)sizeof(T);   // byte offset in the tile
    constexpr int32_t kTileBytes = kWG * PPT * (int32_t)sizeof(T);
    // Buffer loads: tile base in SGPRs, one lane offset, constant per-vector
    // offsets.  Rows are padded to whole tiles with S = K (never in the money).
    auto vload = [&](const T *row, int jj) -> Vec<T> {
        __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc((void *)(row + tile0), (short)0, kTileBytes, 0x00020000);
        return __builtin_bit_cast(Vec<T>, __builtin_amdgcn_raw_buffer_load_b128(
                                                rs, voff, (uint32_t)jj * JS * (uint32_t)sizeof(T), 0));
    };

    {
        const T *row = S + (size_t)(a.M - 1) * ld;
        const T dM = (T)a.datec[a.M].disc;
#pragma unroll
        for (int jj = 0; jj < NVEC; ++jj) {
            const Vec<T> v = vload(row, jj);
#pragma unroll
            for (int e = 0; e < VW; ++e) {
                const T h = call ? v.v[e] - K : K - v.v[e];
                pv[jj * VW + e] = h > T(0) ? dM * h : T(0);
            }
        }
    }

    Vec<T> sc[KEEP ? NVEC : 1];
    Vec<T> sn[KEEP ? NVEC : 1];
    if (!(a.allow_exercise && a.M >= 2)) return;
    if (KEEP) {
        const T *row = S + (size_t)(a.M - 2) * ld;
#pragma unroll
        for (int jj = 0; jj < NVEC; ++jj) sc[jj] = vload(row, jj);
    }
    for (int k = a.M - 1; k >= 1; --k) {
        const DateConst dc = a.datec[k];
        const T xa = (T)dc.xa, xb = (T)dc.xb, dk = (T)dc.disc;
        const T *row = S + (size_t)(k - 1) * ld;

        double acc[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) acc[q] = 0.0;
        int cnt = 0;
        MomBlock<T, D> mb;
        mb.clear();
        if (KEEP) {
#pragma unroll
            for (int jj = 0; jj < NVEC; ++jj) {
#pragma unroll
                for (int e = 0; e < VW; ++e) {
                    cnt += mb.add(sc[jj].v[e], pv[jj * VW + e], true, K, call, xa, xb, lag, wc);
                    if (((jj * VW + e + 1) % BLK) == 0) { mb.flush(acc); mb.clear(); }
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        } else {
            Vec<T> ring[PD];
#pragma unroll
            for (int q = 0; q < PD; ++q) ring[q] = vload(row, q);
#pragma unroll
            for (int jj = 0; jj < NVEC; ++jj) {
                const Vec<T> cur = ring[jj % PD];
                if (jj + PD < NVEC) ring[jj % PD] = vload(row, jj + PD);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int e = 0; e < VW; ++e) {
                    cnt += mb.add(cur.v[e], pv[jj * VW + e], true, K, call, xa, xb, lag, wc);
                    if (((jj * VW + e + 1) % BLK) == 0) { mb.flush(acc); mb.clear(); }
                    __builtin_amdgcn_sched_barrier(0);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        acc[NV - 1] = (double)cnt;

        group_sum<NV>(acc, s_red);
        ++epoch;
        const bool last = arrive<NV>(acc, a.part, gid, a.sync, epoch, G, s_flag);

        if (KEEP && k >= 2) {
            const T *nrow = S + (size_t)(k - 2) * ld;
#pragma unroll
            for (int jj = 0; jj < NVEC; ++jj) sn[jj] = vload(nrow, jj);
        }

        if (last) {
            reduce_partials<NV>(a.part, G, s_tot, s_red8);
            if (tid == 0) {
                double *rec = a.rec + (size_t)k * kRec;
                solve_date<D>(s_tot, rec, s_L, s_w);
                __hip_atomic_store(a.sync + 1, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if (tid == 0) {
            const bool okw = wait_release(a.sync, a.err, epoch, a.spin_limit);
            s_flag[1] = okw ? 1 : 0;
            if (okw) {
                const double *rec = a.rec + (size_t)k * kRec;
#pragma unroll
                for (int q = 0; q < 9; ++q) s_beta[q] = rec[q];
            }
        }
        __syncthreads();
        if (!s_flag[1]) { alive = false; return; }

        if (s_beta[8] != 0.0) {
            T gam[P];
#pragma unroll
            for (int q = 0; q < P; ++q) gam[q] = (T)s_beta[q];
            if (KEEP) {
#pragma unroll
                for (int jj = 0; jj < NVEC; ++jj) {
#pragma unroll
                    for (int e = 0; e < VW; ++e) {
                        pv[jj * VW + e] = exercise_update<T, D>(sc[jj].v[e], pv[jj * VW + e], true, K,
                                                                call, xa, xb, dk, gam, lag, wc);
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
            } else {
                Vec<T> ring[PD];
#pragma unroll
                for (int q = 0; q < PD; ++q) ring[q] = vload(row, q);
#pragma unroll
                for (int jj = 0; jj < NVEC; ++jj) {
                    const Vec<T> cur = ring[jj % PD];
                    if (jj + PD < NVEC) ring[jj % PD] = vload(row, jj + PD);
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int e = 0; e < VW; ++e) {
                        pv[jj * VW + e] = exercise_update<T, D>(cur.v[e], pv[jj * VW + e], true, K,
                                                                call, xa, xb, dk, gam, lag, wc);
                        __builtin_amdgcn_sched_barrier(0);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
        if (KEEP) {
#pragma unroll
            for (int jj = 0; jj < NVEC; ++jj) sc[jj] = sn[jj];
        }
        __syncthreads();   // s_beta / s_flag reuse
    }
}

// Epilogue (eqs. (6)-(8)): FP64 sums of the discounted cashflows and their
// squares through one more barrier; the last group writes the result.
template <typename T, int PPT>
__device__ __forceinline__ void sweep_final(const SweepArgs &a, uint32_t gid, uint32_t e0,
                                            const T (&pv)[PPT], uint32_t epoch, double (*s_red)[32],
                                            double (*s_red8)[32], double *s_tot, int *s_flag)
{
    constexpr int VW = 16 / sizeof(T), NVEC = PPT / VW;
    constexpr uint32_t JS = 64 * VW;
    const int tid = threadIdx.x;
    const int64_t N = a.N;
    double fin[2] = {0.0, 0.0};
    T *pvo = (T *)a.pv_out;
#pragma unroll
    for (int jj = 0; jj < NVEC; ++jj) {
        Vec<T> o;
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            const T v = pv[jj * VW + e];   // padded paths hold 0
            o.v[e] = v;
            fin[0] += (double)v;
            fin[1] += (double)v * (double)v;
        }
        *reinterpret_cast<Vec<T> *>(pvo + e0 + (uint32_t)jj * JS) = o;
    }
    group_sum<2>(fin, s_red);
    ++epoch;
    const uint32_t G = (uint32_t)a.G;
    const bool last = arrive<2>(fin, a.part, gid, a.sync, epoch, G, s_flag);
    if (last) {
        reduce_partials<2>(a.part, G, s_tot, s_red8);
        if (tid == 0) {
            const double n = (double)N;
            const double s1 = s_tot[0], s2 = s_tot[1];
            const double mean = s1 / n;
            double var = N > 1 ? (s2 - s1 * mean) / (n - 1.0) : 0.0;
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

template <typename T, int PPT>
__device__ __forceinline__ uint32_t tile_e0(uint32_t gid)
{
    constexpr int VW = 16 / sizeof(T);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    return (uint32_t)((int64_t)gid * kWG * PPT + (int64_t)wave * 64 * PPT + lane * VW);
}

template <typename T, int PPT, int D>
__global__ void __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(2)))
sweep_kernel(SweepArgs a, const T *__restrict__ S)
{
    static_assert(PPT % (16 / sizeof(T)) == 0, "PPT must be a multiple of the vector width");
    __shared__ double s_red[kWaves][32];
    __shared__ double s_red8[8][32];
    __shared__ double s_tot[32];
    __shared__ double s_L[8][8];
    __shared__ double s_w[24];
    __shared__ double s_beta[10];
    __shared__ int s_flag[2];

    const uint32_t gid = blockIdx.x;
    const uint32_t e0 = tile_e0<T, PPT>(gid);
    T pv[PPT];
    uint32_t epoch = 0;
    bool alive = true;
    sweep_body<T, PPT, D>(a, S, gid, e0, pv, epoch, alive, s_red, s_red8, s_tot, s_L, s_w, s_beta, s_flag);
    if (!alive) return;
    sweep_final<T, PPT>(a, gid, e0, pv, epoch, s_red, s_red8, s_tot, s_flag);
}

// ---------------------------------------------------------------------------
// Dispatch over (precision, paths per thread, degree).
// ---------------------------------------------------------------------------
template <typename T, int PPT>
static const void *sweep_fn(int degree)
{
    switch (degree) {
    case 0: return (const void *)&sweep_kernel<T, PPT, 0>;
    case 1: return (const void *)&sweep_kernel<T, PPT, 1>;
    case 2: return (const void *)&sweep_kernel<T, PPT, 2>;
    case 3: return (const void *)&sweep_kernel<T, PPT, 3>;
    case 4: return (const void *)&sweep_kernel<T, PPT, 4>;
    case 5: return (const void *)&sweep_kernel<T, PPT, 5>;
    case 6: return (const void *)&sweep_kernel<T, PPT, 6>;
    default: return nullptr;
    }
}

static const void *sweep_lookup(int fp64, int ppt, int degree)
{
    if (fp64) {
        switch (ppt) {
        case 2: return sweep_fn<double, 2>(degree);
        case 8: return sweep_fn<double, 8>(degree);
        case 32: return sweep_fn<double, 32>(degree);
        case 64: return sweep_fn<double, 64>(degree);
        default: return nullptr;
        }
    }
    switch (ppt) {
    case 4: return sweep_fn<float, 4>(degree);
    case 16: return sweep_fn<float, 16>(degree);
    case 64: return sweep_fn<float, 64>(degree);
    case 128: return sweep_fn<float, 128>(degree);
    default: return nullptr;
    }
}

int sweep_blocks_per_cu(int fp64, int ppt, int degree)
{
    const void *f = sweep_lookup(fp64, ppt, degree);
    if (!f) return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, kWG, 0) != hipSuccess) return 0;
    return nb;
}

hipError_t launch_sweep(const SweepArgs &a, int fp64, int ppt, hipStream_t s)
{
    const void *f = sweep_lookup(fp64, ppt, a.degree);
    if (!f) return hipErrorInvalidValue;
    SweepArgs args = a;
    const void *Sp = a.S;
    void *params[] = {(void *)&args, (void *)&Sp};
    return hipLaunchCooperativeKernel(f, dim3((unsigned)a.G), dim3(kWG), params, 0, s);
}

// ---------------------------------------------------------------------------
// Batches: many options with uneven path and date counts in two launches.
//
// Generation: each workgroup owns a block range of one option (unit table
// built on the host).  Sweep: one cooperative persistent grid; workgroups
// claim (option, tile) slots from a global counter in a fixed order (options
// by decreasing work, each option's tiles contiguous), run that tile through
// all of the option's dates with the option's own barrier words and partial
// slots, then claim again.  Claims are in order, so at most one option is
// partly claimed at any time and every earlier option can finish; with each
// option needing no more tiles than the grid holds, every claimed tile is
// eventually joined by the rest of its option.  An option's result depends
// only on its own tiles and the fixed reduction order, not on which group ran
// which tile, so it is the same alone and in any mix.
// ---------------------------------------------------------------------------
__device__ __forceinline__ GenArgs gen_args_of(const BatchOpt &o, const uint32_t *V)
{
    GenArgs a;
    a.S = o.S;
    a.V = V;
    a.sched = o.sched;
    a.datec = o.datec;
    a.sync = o.sync;
    a.N = o.N;
    a.ld = o.ld;
    a.nblocks = o.ld / 64;
    a.M = o.M;
    a.R = 1;
    a.what = 0;
    a.pad = 0;
    a.S0 = o.S0; a.K = o.K; a.r = o.r; a.sigma = o.sigma; a.T = o.T;
    a.mu = o.mu; a.vol = o.vol;
    a.shift = nullptr;
    return a;
}

template <typename T>
__global__ void __launch_bounds__(kWG)
gen_batch_kernel(const BatchOpt *__restrict__ opts, const GenUnit *__restrict__ units,
                 const uint32_t *__restrict__ V, uint32_t *gsync)
{
    const GenUnit u = units[blockIdx.x];
    const BatchOpt o = opts[u.opt];
    if (blockIdx.x == 0 && threadIdx.x < 16) gsync[threadIdx.x] = 0u;
    const GenArgs a = gen_args_of(o, V);
    const int64_t per = (u.b1 - u.b0 + kWaves - 1) / kWaves;
    const int64_t w0 = u.b0 + (int64_t)(threadIdx.x >> 6) * per;
    const int64_t w1 = min(w0 + per, u.b1);
    gen_body<T, 0, false>(a, V, o.sched, nullptr, u.b0 == 0, w0, w1);
}

template <typename T, int PPT, int D>
__global__ void __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(2)))
sweep_batch_kernel(const BatchOpt *__restrict__ opts, const int32_t *__restrict__ tile_opt,
                   BatchGlobal g)
{
    __shared__ double s_red[kWaves][32];
    __shared__ double s_red8[8][32];
    __shared__ double s_tot[32];
    __shared__ double s_L[8][8];
    __shared__ double s_w[24];
    __shared__ double s_beta[10];
    __shared__ int s_flag[2];
    __shared__ int s_claim;

    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) {
            int t = (int)__hip_atomic_fetch_add(g.claim, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (ld_agent(g.err) != 0u) t = g.total_tiles;
            s_claim = t;
        }
        __syncthreads();
        const int t = s_claim;
        if (t >= g.total_tiles) return;
        const BatchOpt o = opts[tile_opt[t]];
        SweepArgs a;
        a.S = o.S;
        a.pv_out = o.pv;
        a.part = g.part + (size_t)o.tile_base * kPartStride;
        a.rec = o.rec;
        a.result = o.result;
        a.sync = o.sync;
        a.err = g.err;
        a.datec = o.datec;
        a.N = o.N; a.ld = o.ld;
        a.M = o.M; a.G = o.G;
        a.is_call = o.is_call; a.allow_exercise = o.allow_exercise;
        a.laguerre = g.laguerre; a.degree = D;
        a.S0 = o.S0; a.K = o.K;
        a.spin_limit = g.spin_limit;
        a.pad = 0;
        a.rep_out = nullptr; a.rep = 0; a.n_rep = 0;
        const uint32_t gid = (uint32_t)(t - o.tile_base);
        const uint32_t e0 = tile_e0<T, PPT>(gid);
        T pv[PPT];
        uint32_t epoch = 0;
        bool alive = true;
        sweep_body<T, PPT, D>(a, (const T *)o.S, gid, e0, pv, epoch, alive, s_red, s_red8, s_tot, s_L,
                              s_w, s_beta, s_flag);
        if (!alive) return;
        sweep_final<T, PPT>(a, gid, e0, pv, epoch, s_red, s_red8, s_tot, s_flag);
    }
}

template <typename T, int PPT>
static const void *sweep_batch_fn(int degree)
{
    switch (degree) {
    case 0: return (const void *)&sweep_batch_kernel<T, PPT, 0>;
    case 1: return (const void *)&sweep_batch_kernel<T, PPT, 1>;
    case 2: return (const void *)&sweep_batch_kernel<T, PPT, 2>;
    case 3: return (const void *)&sweep_batch_kernel<T, PPT, 3>;
    case 4: return (const void *)&sweep_batch_kernel<T, PPT, 4>;
    case 5: return (const void *)&sweep_batch_kernel<T, PPT, 5>;
    case 6: return (const void *)&sweep_batch_kernel<T, PPT, 6>;
    default: return nullptr;
    }
}

static const void *sweep_batch_lookup(int fp64, int ppt, int degree)
{
    if (fp64) {
        switch (ppt) {
        case 2: return sweep_batch_fn<double, 2>(degree);
        case 8: return sweep_batch_fn<double, 8>(degree);
        default: return nullptr;
        }
    }
    switch (ppt) {
    case 4: return sweep_batch_fn<float, 4>(degree);
    case 16: return sweep_batch_fn<float, 16>(degree);
    default: return nullptr;
    }
}

int sweep_batch_blocks_per_cu(int fp64, int ppt, int degree)
{
    const void *f = sweep_batch_lookup(fp64, ppt, degree);
    if (!f) return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, kWG, 0) != hipSuccess) return 0;
    return nb;
}

hipError_t launch_generate_batch(const BatchOpt *opts, const GenUnit *units, int n_units,
                                 const uint32_t *V, uint32_t *gsync, int max_dates, int fp64,
                                 hipStream_t s)
{
    const size_t lds = generate_lds_bytes(max_dates);
    if (fp64) hipLaunchKernelGGL((gen_batch_kernel<double>), dim3(n_units), dim3(kWG), lds, s, opts, units, V, gsync);
    else      hipLaunchKernelGGL((gen_batch_kernel<float>), dim3(n_units), dim3(kWG), lds, s, opts, units, V, gsync);
    return hipGetLastError();
}

hipError_t launch_sweep_batch(const BatchOpt *opts, const int32_t *tile_opt, const BatchGlobal &g,
                              int grid, int fp64, int ppt, int degree, bool cooperative, hipStream_t s)
{
    const void *f = sweep_batch_lookup(fp64, ppt, degree);
    if (!f) return hipErrorInvalidValue;
    const BatchOpt *o = opts;
    const int32_t *to = tile_opt;
    BatchGlobal gg = g;
    void *params[] = {(void *)&o, (void *)&to, (void *)&gg};
    if (cooperative) return hipLaunchCooperativeKernel(f, dim3((unsigned)grid), dim3(kWG), params, 0, s);
    // grid sized by the caller so that every in-flight persistent grid is
    // resident together; the bounded waits end the kernel otherwise
    return hipLaunchKernel(f, dim3((unsigned)grid), dim3(kWG), params, 0, s);
}

// ---------------------------------------------------------------------------
// The paper's own estimator (Section V, eqs. (10)-(11)): on the grid
// t_i = i dt, dt = T/(m+1), i = 1..m, the value at t_m is the larger of the
// exercise value and the Black–Scholes value over the last interval dt
// (eqs. (1)-(5)); going back, c_i = max(h(S_i), exp(-r dt) c_{i+1}); the price
// is exp(-r dt) times the path mean of c_1 (eq. (6)).  Every path is
// independent: one thread per path, no device-wide wait.  The paths come from
// the generation kernel run with m dates and horizon m dt.
// ---------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ T cnd(T x);
template <> __device__ __forceinline__ float cnd<float>(float x) { return 0.5f * erfcf(-x * 0.70710678118654752f); }
template <> __device__ __forceinline__ double cnd<double>(double x) { return 0.5 * erfc(-x * 0.70710678118654752); }

template <typename T>
__device__ __forceinline__ T bs_value(T S, T K, T r, T sig, T tau, bool call)
{
    const T sq = sig * sqrt(tau);
    const T d1 = (log(S / K) + (r + T(0.5) * sig * sig) * tau) / sq;
    const T d2 = d1 - sq;
    const T dk = K * exp(-r * tau);
    return call ? S * cnd<T>(d1) - dk * cnd<T>(d2) : dk * cnd<T>(-d2) - S * cnd<T>(-d1);
}

template <typename T>
__global__ void __launch_bounds__(kWG) paper_kernel(PaperArgs a, const T *__restrict__ S)
{
    __shared__ double s_red[kWaves][32];
    __shared__ double s_red8[8][32];
    __shared__ double s_tot[32];
    __shared__ int s_flag[2];
    const T K = (T)a.K, r = (T)a.r, sig = (T)a.sigma, dt = (T)a.dt;
    const T disc = (T)exp(-a.r * a.dt);
    const bool call = a.is_call != 0;
    double acc[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < a.N; i += (int64_t)gridDim.x * kWG) {
        T v = T(0);
        for (int k = a.m; k >= 1; --k) {
            const T s = S[(size_t)(k - 1) * a.ld + i];
            T h = call ? s - K : K - s;
            h = h > T(0) ? h : T(0);
            const T cont = (k == a.m) ? bs_value<T>(s, K, r, sig, dt, call) : disc * v;
            v = h > cont ? h : cont;
        }
        const double c = (double)disc * (double)v;
        acc[0] += c;
        acc[1] += c * c;
    }
    group_sum<2>(acc, s_red);
    if (threadIdx.x == 0) {
        double *dst = a.part + (size_t)blockIdx.x * kPartStride;
        dst[0] = acc[0];
        dst[1] = acc[1];
        const uint32_t old = __hip_atomic_fetch_add(a.ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_flag[0] = (old + 1u == gridDim.x) ? 1 : 0;
    }
    __syncthreads();
    if (!s_flag[0]) return;
    reduce_partials<2>(a.part, gridDim.x, s_tot, s_red8);
    if (threadIdx.x == 0) {
        const double n = (double)a.N;
        const double mean = s_tot[0] / n;
        double var = a.N > 1 ? (s_tot[1] - s_tot[0] * mean) / (n - 1.0) : 0.0;
        if (var < 0.0) var = 0.0;
        a.result[0] = mean;
        a.result[1] = sqrt(var / n);
        a.result[2] = mean;
        a.result[3] = 0.0;
        a.result[4] = 0.0;
        a.result[5] = 0.0;
    }
}

hipError_t launch_paper(const PaperArgs &a, int fp64, hipStream_t s)
{
    int64_t g = (a.N + kWG - 1) / kWG;
    if (g > kMaxGroups) g = kMaxGroups;
    if (fp64) hipLaunchKernelGGL((paper_kernel<double>), dim3((unsigned)g), dim3(kWG), 0, s, a, (const double *)a.S);
    else      hipLaunchKernelGGL((paper_kernel<float>), dim3((unsigned)g), dim3(kWG), 0, s, a, (const float *)a.S);
    return hipGetLastError();
}

}  // namespace amq
