// amq_kernels.hip — gfx950 kernels for quasi-Monte Carlo American option
// valuation (Cvetanoska & Stojanovski; method in Sections III.D, III.E, V).
//
//   gen_kernel:   Sobol point -> Moro inverse normal -> Brownian bridge ->
//                 GBM value, stored path-contiguous as S[date][path].
//   paper_kernel: the paper's own per-path estimator.
// The backward-induction kernels live in amq_sweep.h (instantiated per
// precision and basis kind in amq_sweep_*.hip); this file dispatches to them.
//
// Compiled for gfx950 only.
#include "amq_math.h"
#include "amq_sync.h"

#include <math.h>

#include <map>
#include <mutex>
#include <utility>

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

// log(v) in binary64 for finite v > 0 (normal) by Tang's table method (P. T.
// P. Tang, "Table-driven implementation of the logarithm function in IEEE
// floating-point arithmetic", ACM TOMS 16(4), 1990): v = m 2^e with m in
// [1/2, 1); F = 1/2 + j/256 + 1/512 from the top 7 fraction bits j of m, so
// f = m - F is exact and |u| = |f / F| <= 2^-8; log v = e ln 2 + log F +
// log1p(u), log1p by its Taylor series to degree 6 (truncation below 2e-18).
// kLogTab[j] = {1/F, log F}, each rounded to nearest: 1/F by binary64
// division, log F from a 50-digit decimal evaluation.  About 1 ulp for the
// tail's arguments (results of magnitude 0.9 and more).
__constant__ double kLogTab[128][2] = {
    {0x1.fe01fe01fe020p+0, -0x1.60e52f45788e3p-1},
    {0x1.fa11caa01fa12p+0, -0x1.5ced1e17c35c5p-1},
    {0x1.f6310aca0dbb5p+0, -0x1.58fcddce004c4p-1},
    {0x1.f25f644230ab5p+0, -0x1.55144fdbcbd62p-1},
    {0x1.ee9c7f8458e02p+0, -0x1.513356667fc57p-1},
    {0x1.eae807aba01ebp+0, -0x1.4d59d43fdaba2p-1},
    {0x1.e741aa59750e4p+0, -0x1.4987ace0dabb0p-1},
    {0x1.e3a9179dc1a73p+0, -0x1.45bcc464c893ap-1},
    {0x1.e01e01e01e01ep+0, -0x1.41f8ff8471d61p-1},
    {0x1.dca01dca01dcap+0, -0x1.3e3c43918f76cp-1},
    {0x1.d92f2231e7f8ap+0, -0x1.3a86767257111p-1},
    {0x1.d5cac807572b2p+0, -0x1.36d77e9d34fd7p-1},
    {0x1.d272ca3fc5b1ap+0, -0x1.332f4314ad796p-1},
    {0x1.cf26e5c44bfc6p+0, -0x1.2f8dab636337ap-1},
    {0x1.cbe6d9601cbe7p+0, -0x1.2bf29f9841c3bp-1},
    {0x1.c8b265afb8a42p+0, -0x1.285e0842ca384p-1},
    {0x1.c5894d10d4986p+0, -0x1.24cfce6f80d9ap-1},
    {0x1.c26b5392ea01cp+0, -0x1.2147dba47a394p-1},
    {0x1.bf583ee868d8bp+0, -0x1.1dc619de06944p-1},
    {0x1.bc4fd65883e7bp+0, -0x1.1a4a738b7a33cp-1},
    {0x1.b951e2b18ff23p+0, -0x1.16d4d38c119fap-1},
    {0x1.b65e2e3beee05p+0, -0x1.1365252bf0865p-1},
    {0x1.b37484ad806cep+0, -0x1.0ffb54213a476p-1},
    {0x1.b094b31d922a4p+0, -0x1.0c974c89431cep-1},
    {0x1.adbe87f94905ep+0, -0x1.0938fae5d8e9bp-1},
    {0x1.aaf1d2f87ebfdp+0, -0x1.05e04c1aa2c06p-1},
    {0x1.a82e65130e159p+0, -0x1.028d2d6a963f4p-1},
    {0x1.a574107688a4ap+0, -0x1.fe7f18eb03d3ep-2},
    {0x1.a2c2a87c51ca0p+0, -0x1.f7eeae6b5761dp-2},
    {0x1.a01a01a01a01ap+0, -0x1.f168f7fb05c52p-2},
    {0x1.9d79f176b682dp+0, -0x1.eaedd2eac990cp-2},
    {0x1.9ae24ea5510dap+0, -0x1.e47d1d32e677ep-2},
    {0x1.9852f0d8ec0ffp+0, -0x1.de16b56ef90f0p-2},
    {0x1.95cbb0be377aep+0, -0x1.d7ba7ad9e7da0p-2},
    {0x1.934c67f9b2ce6p+0, -0x1.d1684d49f46aep-2},
    {0x1.90d4f120190d5p+0, -0x1.cb200d2ceb643p-2},
    {0x1.8e6527af1373fp+0, -0x1.c4e19b84723c2p-2},
    {0x1.8bfce8062ff3ap+0, -0x1.beacd9e271ad1p-2},
    {0x1.899c0f601899cp+0, -0x1.b881aa659bc93p-2},
    {0x1.87427bcc092b9p+0, -0x1.b25fefb60cb2ep-2},
    {0x1.84f00c2780614p+0, -0x1.ac478d020506fp-2},
    {0x1.82a4a0182a4a0p+0, -0x1.a63865fabd0ecp-2},
    {0x1.8060180601806p+0, -0x1.a0325ed14fda4p-2},
    {0x1.7e225515a4f1dp+0, -0x1.9a355c33bd6bap-2},
    {0x1.7beb3922e017cp+0, -0x1.9441434a03259p-2},
    {0x1.79baa6bb6398bp+0, -0x1.8e55f9b349b83p-2},
    {0x1.77908119ac60dp+0, -0x1.8873658327ccfp-2},
    {0x1.756cac201756dp+0, -0x1.82996d3ef8bcbp-2},
    {0x1.734f0c541fe8dp+0, -0x1.7cc7f7db46a0ep-2},
    {0x1.713786d9c7c09p+0, -0x1.76feecb947175p-2},
    {0x1.6f26016f26017p+0, -0x1.713e33a46a17cp-2},
    {0x1.6d1a62681c861p+0, -0x1.6b85b4cffa3fdp-2},
    {0x1.6b1490aa31a3dp+0, -0x1.65d558d4ce00bp-2},
    {0x1.691473a88d0c0p+0, -0x1.602d08af091ecp-2},
    {0x1.6719f3601671ap+0, -0x1.5a8cadbbedfa1p-2},
    {0x1.6524f853b4aa3p+0, -0x1.54f431b7be1a9p-2},
    {0x1.63356b88ac0dep+0, -0x1.4f637ebba9810p-2},
    {0x1.614b36831ae94p+0, -0x1.49da7f3bcc41fp-2},
    {0x1.5f66434292dfcp+0, -0x1.44591e0539f49p-2},
    {0x1.5d867c3ece2a5p+0, -0x1.3edf463c1683ep-2},
    {0x1.5babcc647fa91p+0, -0x1.396ce359bbf54p-2},
    {0x1.59d61f123ccaap+0, -0x1.3401e12aecba1p-2},
    {0x1.5805601580560p+0, -0x1.2e9e2bce12286p-2},
    {0x1.56397ba7c52e2p+0, -0x1.2941afb186b7cp-2},
    {0x1.54725e6bb82fep+0, -0x1.23ec5991eba49p-2},
    {0x1.52aff56a8054bp+0, -0x1.1e9e1678899f4p-2},
    {0x1.50f22e111c4c5p+0, -0x1.1956d3b9bc2fap-2},
    {0x1.4f38f62dd4c9bp+0, -0x1.14167ef367783p-2},
    {0x1.4d843bedc2c4cp+0, -0x1.0edd060b78081p-2},
    {0x1.4bd3edda68fe1p+0, -0x1.09aa572e6c6d4p-2},
    {0x1.4a27fad76014ap+0, -0x1.047e60cde83b8p-2},
    {0x1.4880522014880p+0, -0x1.feb2233ea07cdp-3},
    {0x1.46dce34596066p+0, -0x1.f474b134df229p-3},
    {0x1.453d9e2c776cap+0, -0x1.ea4449f04aaf5p-3},
    {0x1.43a2730abee4dp+0, -0x1.e020cc6235ab5p-3},
    {0x1.420b5265e5951p+0, -0x1.d60a17f903515p-3},
    {0x1.40782d10e6566p+0, -0x1.cc000c9db3c52p-3},
    {0x1.3ee8f42a5af07p+0, -0x1.c2028ab17f9b4p-3},
    {0x1.3d5d991aa75c6p+0, -0x1.b811730b823d2p-3},
    {0x1.3bd60d9232955p+0, -0x1.ae2ca6f672bd4p-3},
    {0x1.3a524387ac822p+0, -0x1.a454082e6ab05p-3},
    {0x1.38d22d366088ep+0, -0x1.9a8778debaa38p-3},
    {0x1.3755bd1c945eep+0, -0x1.90c6db9fcbcd9p-3},
    {0x1.35dce5f9f2af8p+0, -0x1.871213750e994p-3},
    {0x1.34679ace01346p+0, -0x1.7d6903caf5ad0p-3},
    {0x1.32f5ced6a1dfap+0, -0x1.73cb9074fd14dp-3},
    {0x1.3187758e9ebb6p+0, -0x1.6a399dabbd383p-3},
    {0x1.301c82ac40260p+0, -0x1.60b3100b09476p-3},
    {0x1.2eb4ea1fed14bp+0, -0x1.5737cc9018cddp-3},
    {0x1.2d50a012d50a0p+0, -0x1.4dc7b897bc1c8p-3},
    {0x1.2bef98e5a3711p+0, -0x1.4462b9dc9b3dcp-3},
    {0x1.2a91c92f3c105p+0, -0x1.3b08b6757f2a9p-3},
    {0x1.293725bb804a5p+0, -0x1.31b994d3a4f85p-3},
    {0x1.27dfa38a1ce4dp+0, -0x1.28753bc11aba5p-3},
    {0x1.268b37cd60127p+0, -0x1.1f3b925f25d41p-3},
    {0x1.2539d7e9177b2p+0, -0x1.160c8024b27b1p-3},
    {0x1.23eb79717605bp+0, -0x1.0ce7ecdccc28dp-3},
    {0x1.22a0122a0122ap+0, -0x1.03cdc0a51ec0dp-3},
    {0x1.21579804855e6p+0, -0x1.f57bc7d9005dbp-4},
    {0x1.2012012012012p+0, -0x1.e3707ee30487bp-4},
    {0x1.1ecf43c7fb84cp+0, -0x1.d179788219364p-4},
    {0x1.1d8f5672e4abdp+0, -0x1.bf968769fca11p-4},
    {0x1.1c522fc1ce059p+0, -0x1.adc77ee5aea8cp-4},
    {0x1.1b17c67f2bae3p+0, -0x1.9c0c32d4d2548p-4},
    {0x1.19e0119e0119ep+0, -0x1.8a6477a91dc29p-4},
    {0x1.18ab083902bdbp+0, -0x1.78d02263d82d3p-4},
    {0x1.1778a191bd684p+0, -0x1.674f089365a7ap-4},
    {0x1.1648d50fc3201p+0, -0x1.55e10050e0384p-4},
    {0x1.151b9a3fdd5c9p+0, -0x1.4485e03dbdfadp-4},
    {0x1.13f0e8d344724p+0, -0x1.333d7f8183f4bp-4},
    {0x1.12c8b89edc0acp+0, -0x1.2207b5c78549ep-4},
    {0x1.11a3019a74826p+0, -0x1.10e45b3cae831p-4},
    {0x1.107fbbe011080p+0, -0x1.ffa6911ab9301p-5},
    {0x1.0f5edfab325a2p+0, -0x1.dda8adc67ee4ep-5},
    {0x1.0e40655826011p+0, -0x1.bbcebfc68f420p-5},
    {0x1.0d24456359e3ap+0, -0x1.9a187b573de7cp-5},
    {0x1.0c0a7868b4171p+0, -0x1.788595a3577bap-5},
    {0x1.0af2f722eecb5p+0, -0x1.5715c4c03ceefp-5},
    {0x1.09ddba6af8360p+0, -0x1.35c8bfaa1306bp-5},
    {0x1.08cabb37565e2p+0, -0x1.149e3e4005a8dp-5},
    {0x1.07b9f29b8eae2p+0, -0x1.e72bf2813ce51p-6},
    {0x1.06ab59c7912fbp+0, -0x1.a55f548c5c43fp-6},
    {0x1.059eea0727586p+0, -0x1.63d6178690bd6p-6},
    {0x1.04949cc1664c5p+0, -0x1.228fb1fea2e28p-6},
    {0x1.038c6b78247fcp+0, -0x1.c317384c75f06p-7},
    {0x1.02864fc7729e9p+0, -0x1.41929f96832f0p-7},
    {0x1.0182436517a37p+0, -0x1.8121214586b54p-8},
    {0x1.0080402010080p+0, -0x1.0040155d5889ep-9},
};

// logF: the table's log F column, from constant memory or from an LDS copy
// (the path generator's: its loads then wait on LDS only, not on the
// generator's pending stores); 1/F by the reciprocal's Newton refinement.
template <typename LogF>
__device__ __forceinline__ double log_tab(double v, LogF logF)
{
    const double m = __builtin_amdgcn_frexp_mant(v);
    const int e = __builtin_amdgcn_frexp_exp(v);
    const uint32_t j = (uint32_t)((uint64_t)__double_as_longlong(m) >> 45) & 127u;
    const double F = fma((double)j, 0x1p-8, 0.5 + 0x1p-9);
    const double u = (m - F) * rcp_f64(F);
    double p = fma(u, -1.0 / 6.0, 0.2);
    p = fma(p, u, -0.25);
    p = fma(p, u, 1.0 / 3.0);
    p = fma(p, u, -0.5);
    const double l1p = fma(p, u * u, u);
    const double de = (double)e;
    return fma(de, 0.69314718055994529, fma(de, 2.3190468138462996e-17, logF(j) + l1p));
}

__device__ __forceinline__ double log_tab(double v)
{
    return log_tab(v, [](uint32_t j) { return kLogTab[j][1]; });
}

// The two branches separately: which branch a point takes, the central
// rational function and the tail polynomial (its two logarithms by
// log_tab).  inv_normal_f64 combines them; the path generator evaluates the
// tails packed.
template <typename T> struct MoroParts;

template <> struct MoroParts<double> {
    // d = x - 2^31 exactly (the sign bit flipped, read as a signed integer);
    // y = u - 1/2 = d 2^-32.  The branch test and the central rational are
    // taken on d with every constant scaled by a power of two, which leaves
    // each rounded intermediate scaled by the same power: the values are
    // bitwise those of the same steps on y (no under- or overflow here).
    static __device__ __forceinline__ double centered(uint32_t x)
    {
        return (double)(int32_t)(x ^ 0x80000000u);
    }
    static __device__ __forceinline__ bool tail(uint32_t x)
    {
        return !(fabs(centered(x)) < 0.42 * 0x1p32);   // |y| >= 0.42
    }
    static __device__ __forceinline__ double central(uint32_t x)
    {
        // y P(r) / Q(r), r = y^2 = D 2^-64: Horner in D with the k-th
        // coefficient of P scaled by 2^(-64k - 32) (the y factor's 2^-32
        // folded in) and of Q (beyond the constant 1) by 2^(-64(k + 1))
        const double d = centered(x);
        const double D = d * d;
        const double num = d * fma3(fma3(fma3(AMQ_A3 * 0x1p-224, D, AMQ_A2 * 0x1p-160), D, AMQ_A1 * 0x1p-96),
                                    D, AMQ_A0 * 0x1p-32);
        const double den = fma(fma3(fma3(fma3(AMQ_B3 * 0x1p-256, D, AMQ_B2 * 0x1p-192), D, AMQ_B1 * 0x1p-128),
                                    D, AMQ_B0 * 0x1p-64),
                               D, 1.0);
        return num * rcp_f64(den);   // (a tail point's value is discarded)
    }
    template <typename LogF>
    static __device__ __forceinline__ double tail_value(uint32_t x, LogF logF)
    {
        const double s = 0x1p-32;
        const double y = ((double)x - 2147483648.0) * s;
        const double q = y < 0.0 ? (double)x * s : (4294967296.0 - (double)x) * s;
        const double t = log_tab(-log_tab(q, logF), logF);
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
    static __device__ __forceinline__ double tail_value(uint32_t x)
    {
        return tail_value(x, [](uint32_t j) { return kLogTab[j][1]; });
    }
};

// binary64: u, u - 1/2 and 1 - u are exact for u = x 2^-32.
__device__ __forceinline__ double inv_normal_f64(uint32_t x)
{
    return MoroParts<double>::tail(x) ? MoroParts<double>::tail_value(x) : MoroParts<double>::central(x);
}

// Shifted (randomised) points sit at cell midpoints u = (x + 1/2) 2^-32, so a
// shifted integer 0 still maps to a finite normal.
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
    const double t = log_tab(-log_tab(q));
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

template <bool MID> __device__ __forceinline__ double inv_normal(uint32_t x)
{
    return MID ? inv_normal_mid_f64(x) : inv_normal_f64(x);
}

// A bridge node as the batch generator keeps it in LDS.
struct LdsNode {
    int32_t dim, m, sl, sr, dst, pad;
    double wl, wr, sd;
};

// Nodes whose tail normals are evaluated together (binary64 paths): a
// 64-point Sobol block puts about 10 of its 64 points of each dimension in
// the tails (|u - 1/2| >= 0.42), so the tails of 5 nodes mostly fill one wave.
constexpr int kTailChunk = 5;

__host__ __device__ size_t generate_lds_bytes(int M, int fp64)
{
    // lane tables [M][16], per-wave block words [kWaves][M][2], per-wave tail
    // staging: points [kTailChunk * 64] u32 and normals [kTailChunk * 64] f64
    // (both storage types: the normals are binary64), the logarithm table's
    // log F column [128] f64
    (void)fp64;
    return (size_t)M * 16 * sizeof(uint32_t) + (size_t)kWaves * M * 2 * sizeof(uint32_t) +
           (size_t)kWaves * kTailChunk * 64 * (sizeof(uint32_t) + sizeof(double)) + 8 + 128 * sizeof(double);
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
template <typename T, int WHAT, bool MID, typename Node>
__device__ __forceinline__ void gen_body(const GenArgs &a, const uint32_t *__restrict__ V,
                                         const Node *__restrict__ sched,
                                         const uint32_t *__restrict__ shift, bool init, int64_t w0,
                                         int64_t w1)
{
    extern __shared__ uint32_t lds[];
    const int M = a.M;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t *ttab = lds;                                   // [M][16]
    uint32_t *xw = lds + (size_t)M * 16 + (size_t)wave * M * 2;   // [M][2]
    // this wave's tail staging (see kTailChunk)
    uint32_t *tx = lds + (size_t)M * 16 + (size_t)kWaves * M * 2 + (size_t)wave * kTailChunk * 64;
    double *tz0 = reinterpret_cast<double *>(reinterpret_cast<char *>(lds) +
                                  (((size_t)M * 16 + (size_t)kWaves * M * 2 + (size_t)kWaves * kTailChunk * 64) *
                                       sizeof(uint32_t) + 7) / 8 * 8);
    double *tz = tz0 + (size_t)wave * kTailChunk * 64;
    // the logarithm table's log F column, for the packed tails
    double *ltab = tz0 + (size_t)kWaves * kTailChunk * 64;
    for (int j = tid; j < 128; j += kWG) ltab[j] = kLogTab[j][1];

    if (init && WHAT == 0) {
        for (int q = tid; q < kSyncWords; q += kWG) a.sync[q] = 0u;
        for (int k = tid; k <= M; k += kWG) {
            const double tk = (double)k * a.T / (double)M;
            DateConst c;
            c.disc = exp(-a.r * tk);
            // Standardise x = S/K with the model's mean and sd of x given in
            // the money (ln x ~ N(m, s^2); E[x^q | x < 1] =
            // exp(q m + q^2 s^2/2) Phi(-m/s - q s)/Phi(-m/s), mirrored for
            // calls), so in-the-money abscissae are centred with unit spread
            // and the Hankel matrix stays well conditioned.  Falls back to
            // the unconditional moments when the region is negligible.
            const double m = log(a.S0 / a.K) + (a.r - 0.5 * a.sigma * a.sigma) * tk;
            const double sv = a.sigma * sqrt(tk);
            double mean = 0.0, sd = 0.0;
            if (k > 0) {
                const double z = a.is_call ? m / sv : -m / sv;     // ITM probability Phi(z)
                const double sg = a.is_call ? sv : -sv;
                const double p0 = 0.5 * erfc(-z * 0.70710678118654752);
                if (p0 > 1e-12) {
                    const double e1 = exp(m + 0.5 * sv * sv) * (0.5 * erfc(-(z + sg) * 0.70710678118654752)) / p0;
                    const double e2 = exp(2.0 * m + 2.0 * sv * sv) *
                                      (0.5 * erfc(-(z + 2.0 * sg) * 0.70710678118654752)) / p0;
                    const double var = e2 - e1 * e1;
                    if (var > 1e-12 * e1 * e1) { mean = e1; sd = sqrt(var); }
                }
                if (!(sd > 0.0)) {
                    mean = a.S0 / a.K * exp(a.r * tk);
                    sd = mean * sqrt(expm1(a.sigma * a.sigma * tk));
                }
            }
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

    // The inverse normal, the bridge and the exponent run in binary64 for
    // both storage types, so binary32 storage holds each path value rounded
    // once from its binary64 value (the correctly rounded value except where
    // that lies within a few binary64 ulps of a rounding boundary).  The
    // exercise decisions downstream react to path-value errors of one
    // binary32 ulp on some options (a binary32 inverse normal moved prices by
    // up to 7e-2).  The bridge runs
    // on the log-price X(t_m) = log S0 + mu m + vol W(m) (the schedule's
    // weights sum to 1, so interpolation carries the constant and the drift),
    // and S = exp(X): no per-date drift, volatility or S0 products.
    const double vol = a.vol;
    // Padding paths (past N) hold K rounded in the storage precision away
    // from the money, so h(S) <= 0 in binary64 and the sweep never counts
    // them in the money.
    T Kp = (T)a.K;
    if constexpr (sizeof(T) == 4) {
        if (!a.is_call && (double)Kp < a.K) Kp = nextafterf(Kp, INFINITY);
        if (a.is_call && (double)Kp > a.K) Kp = nextafterf(Kp, -INFINITY);
    }

    double X[kMaxSlots];
#pragma unroll
    for (int q = 0; q < kMaxSlots; ++q) X[q] = 0.0;
    X[0] = log(a.S0);                                   // X(t_0)
    X[kAnchorSlot] = X[0] + a.mu * (double)M;           // read by the root node only

    for (int64_t w = w0; w < w1; ++w) {
        const int64_t i = (w << 6) + lane;
        const bool valid = i < a.N;
        if (WHAT == 0 && (w << 6) >= a.N) {
            // padding block: out of the money on every date
            for (int m = 0; m < M; ++m) ((T *)a.S)[(size_t)m * a.ld + i] = Kp;
            continue;
        }
        if constexpr (WHAT == 0 && !MID) {
            // the inverse normal's two branches evaluated apart (the tail's
            // two logarithms dominate).  Every
            // lane evaluates the (cheap) central branch; the points in the tails
            // of kTailChunk nodes are packed into this wave's LDS staging
            // (ballot and lane rank), their tail values evaluated together,
            // one point per lane, and read back by their owners.  The values
            // are exactly those of inv_normal.
            for (int s0 = 0; s0 < M; s0 += kTailChunk) {
                uint32_t xs[kTailChunk], slot[kTailChunk];
                bool tl[kTailChunk];
                uint32_t ntail = 0;   // wave-uniform
#pragma unroll
                for (int q = 0; q < kTailChunk; ++q) {
                    tl[q] = false;
                    if (s0 + q < M) {
                        const int j = __builtin_amdgcn_readfirstlane(sched[s0 + q].dim);
                        const uint32_t x = xw[2 * j + xsel] ^ ttab[j * 16 + offL] ^ ttab[j * 16 + offH];
                        xs[q] = x;
                        tl[q] = MoroParts<double>::tail(x);
                        const uint64_t m = __builtin_amdgcn_ballot_w64(tl[q]);
                        slot[q] = ntail + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                        if (tl[q]) tx[slot[q]] = x;
                        ntail += (uint32_t)__builtin_popcountll(m);
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                for (uint32_t t0 = 0; t0 < ntail; t0 += 64) {
                    const uint32_t t = t0 + (uint32_t)lane;
                    if (t < ntail)
                        tz[t] = MoroParts<double>::tail_value(tx[t], [=](uint32_t j) { return ltab[j]; });
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
                for (int q = 0; q < kTailChunk; ++q) {
                    if (s0 + q < M) {
                        const Node &nd = sched[s0 + q];
                        const int n_m = __builtin_amdgcn_readfirstlane(nd.m);
                        const int n_sl = __builtin_amdgcn_readfirstlane(nd.sl),
                                  n_sr = __builtin_amdgcn_readfirstlane(nd.sr),
                                  n_dst = __builtin_amdgcn_readfirstlane(nd.dst);
                        const double n_wl = uniform_f64(nd.wl), n_wr = uniform_f64(nd.wr),
                                     n_sd = uniform_f64(nd.sd);
                        const double zc = MoroParts<double>::central(xs[q]);
                        const double z = tl[q] ? tz[slot[q]] : zc;
                        const double xv = n_wl * X[n_sl] + n_wr * X[n_sr] + n_sd * (vol * z);
                        X[n_dst] = xv;
                        const T Sv = (T)exp_poly<true>(xv);
                        ((T *)a.S)[(size_t)(n_m - 1) * a.ld + i] = valid ? Sv : Kp;
                    }
                }
                // the next chunk rewrites the staging only after every lane
                // has read its values back
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        } else
        for (int s = 0; s < M; ++s) {
            // node fields moved to scalar registers: the batch kernel reaches
            // the schedule through a loaded descriptor, and a window index the
            // compiler cannot prove uniform turns every slot access into a
            // compare-and-select chain
            const Node &nd = sched[s];
            const int j = __builtin_amdgcn_readfirstlane(nd.dim);
            const int n_m = __builtin_amdgcn_readfirstlane(nd.m);
            const int n_sl = __builtin_amdgcn_readfirstlane(nd.sl), n_sr = __builtin_amdgcn_readfirstlane(nd.sr),
                      n_dst = __builtin_amdgcn_readfirstlane(nd.dst);
            const double n_wl = uniform_f64(nd.wl), n_wr = uniform_f64(nd.wr), n_sd = uniform_f64(nd.sd);
            uint32_t x = xw[2 * j + xsel] ^ ttab[j * 16 + offL] ^ ttab[j * 16 + offH];
            if (MID) x ^= shift[j];
            if (WHAT == 1) {
                if (valid) ((uint32_t *)a.S)[(size_t)j * a.ld + i] = x;
                continue;
            }
            const double z = inv_normal<MID>(x);
            if (WHAT == 2) {
                if (valid) ((double *)a.S)[(size_t)j * a.ld + i] = z;
                continue;
            }
            const double xv = n_wl * X[n_sl] + n_wr * X[n_sr] + n_sd * (vol * z);
            X[n_dst] = xv;
            const T Sv = (T)exp_poly<true>(xv);
            ((T *)a.S)[(size_t)(n_m - 1) * a.ld + i] = valid ? Sv : Kp;
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

// three waves per SIMD (the packed tail evaluation needs the registers):
// latency hiding for the per-lane dependency chain of each path through the
// dates
template <typename T, int WHAT, bool MID>
__global__ void __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 3)))
gen_kernel(GenArgs a, const uint32_t *__restrict__ V, const BridgeNode *__restrict__ sched,
           const uint32_t *__restrict__ shift)
{
    const int64_t gw = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
    const int64_t w0 = gw * a.R;
    const int64_t w1 = min(w0 + (int64_t)a.R, a.nblocks);
    // the sweep's partial-sum rows start each launch at tag 0
    if (WHAT == 0)
        for (int64_t q = (int64_t)blockIdx.x * kWG + threadIdx.x; q < a.rows_n; q += (int64_t)gridDim.x * kWG)
            a.rows[q] = 0ull;
    gen_body<T, WHAT, MID, BridgeNode>(a, V, sched, shift, blockIdx.x == 0, w0, w1);
}

hipError_t launch_generate(const GenArgs &a, int fp64, hipStream_t s)
{
    const int64_t waves = (a.nblocks + a.R - 1) / a.R;
    const int64_t grid = (waves + kWaves - 1) / kWaves;
    const size_t lds = generate_lds_bytes(a.M, fp64);
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
        // the normals are binary64 for both storage types
        hipLaunchKernelGGL((gen_kernel<double, 2, false>), g, b, lds, s, a, a.V, a.sched, a.shift);
    }
    return hipGetLastError();
}

// Make the runtime load the generation kernels' code on the current device
// now rather than at their first launch (a first use allocates device memory
// for the code).
hipError_t preload_generate()
{
    hipFuncAttributes fa;
    hipError_t e = hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(&gen_kernel<float, 0, false>));
    if (e == hipSuccess) e = hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(&gen_kernel<double, 0, false>));
    return e;
}

// ---------------------------------------------------------------------------
// Dispatch over (precision, basis kind, paths per thread, degree).
// ---------------------------------------------------------------------------
static const void *sweep_lookup(int fp64, int laguerre, int ppt, int degree, int kind)
{
    if (fp64) return laguerre ? sweep_table_f64_lag(ppt, degree, kind) : sweep_table_f64_mono(ppt, degree, kind);
    return laguerre ? sweep_table_f32_lag(ppt, degree, kind) : sweep_table_f32_mono(ppt, degree, kind);
}

static int blocks_per_cu(const void *f, int wg)
{
    if (!f) return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, wg, 0) != hipSuccess) return 0;
    return nb;
}

int sweep_blocks_per_cu(int fp64, int laguerre, int wg, int ppt, int degree)
{
    if (wg != kWG && wg != 512) return 0;
    return blocks_per_cu(sweep_lookup(fp64, laguerre, ppt, degree, wg == 512 ? 2 : 0), wg);
}

int sweep_batch_blocks_per_cu(int fp64, int laguerre, int ppt, int degree)
{
    return blocks_per_cu(sweep_lookup(fp64, laguerre, ppt, degree, 1), kWG);
}

// Dynamic LDS that leaves room for one workgroup of `f` per CU (more than
// half of a CU's LDS in total), so a grid of at most one group per CU is
// spread over the CUs instead of doubling up on some; 0 if unavailable.
// Computed once per (device, kernel).
static size_t one_per_cu_lds(int dev, const void *f)
{
    static std::mutex mu;
    static std::map<std::pair<int, const void *>, size_t> cache;
    std::lock_guard<std::mutex> lk(mu);
    const auto key = std::make_pair(dev, f);
    const auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int lds_cu = 0;
    hipFuncAttributes fa;
    size_t dyn = 0;
    if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) == hipSuccess &&
        hipFuncGetAttributes(&fa, f) == hipSuccess) {
        const size_t want = (size_t)lds_cu / 2 + 1024;
        if (fa.sharedSizeBytes < want) {
            dyn = want - fa.sharedSizeBytes;
            if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn) != hipSuccess) dyn = 0;
        }
    }
    cache[key] = dyn;
    return dyn;
}

hipError_t launch_sweep(const SweepArgs &a, int fp64, int wg, int ppt, hipStream_t s)
{
    if (wg != kWG && wg != 512) return hipErrorInvalidValue;
    // slab-resident tiles come in a call form (kind 3) and a put form (kind 2)
    const void *f = (wg == 512 && a.is_call) ? sweep_lookup(fp64, a.laguerre, ppt, a.degree, 3) : nullptr;
    if (!f) f = sweep_lookup(fp64, a.laguerre, ppt, a.degree, wg == 512 ? 2 : 0);
    if (!f) return hipErrorInvalidValue;
    SweepArgs args = a;
    const void *Sp = a.S;
    void *params[] = {(void *)&args, (void *)&Sp};
    int dev = 0, cus = 0;
    size_t dyn = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && a.G <= cus)
        dyn = one_per_cu_lds(dev, f);
    // a plain launch: the grid is sized to what the device holds at once, and
    // the caller orders persistent sweeps on one device (a cooperative launch
    // measured 19 us slower per call, in the kernel's own event interval)
    return hipLaunchKernel(f, dim3((unsigned)a.G), dim3((unsigned)wg), params, (unsigned)dyn, s);
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
    a.is_call = o.is_call;
    a.rows = o.rows;
    a.rows_n = 0;   // cleared by the option's first unit
    return a;
}

template <typename T, bool MID>
__global__ void __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 3)))
gen_batch_kernel(const BatchOpt *__restrict__ opts, const GenUnit *__restrict__ units,
                 const uint32_t *__restrict__ V, uint32_t *gsync)
{
    const GenUnit u = units[blockIdx.x];
    const BatchOpt o = opts[u.opt];
    if (blockIdx.x == 0 && threadIdx.x < 16) gsync[threadIdx.x] = 0u;
    const GenArgs a = gen_args_of(o, V);
    if (u.b0 == 0)   // the option's first unit clears its partial-sum rows
        for (int64_t q = threadIdx.x; q < o.rows_n; q += kWG) o.rows[q] = 0ull;
    const int64_t per = (u.b1 - u.b0 + kWaves - 1) / kWaves;
    const int64_t w0 = u.b0 + (int64_t)(threadIdx.x >> 6) * per;
    const int64_t w1 = min(w0 + per, u.b1);
    // the option's bridge schedule copied into LDS past gen_body's regions
    // (read by gen_body after its first barrier): co-resident groups of
    // different options would otherwise each walk their own schedule through
    // the shared scalar cache, one miss per date
    extern __shared__ uint32_t lds[];
    LdsNode *nodes = reinterpret_cast<LdsNode *>(reinterpret_cast<char *>(lds) +
                                                 (generate_lds_bytes(o.M, sizeof(T) == 8) + 15) / 16 * 16);
    for (int q = threadIdx.x; q < o.M; q += kWG) {
        const BridgeNode &b = o.sched[q];
        LdsNode n;
        n.dim = b.dim; n.m = b.m; n.sl = b.sl; n.sr = b.sr; n.dst = b.dst; n.pad = 0;
        n.wl = b.wl; n.wr = b.wr; n.sd = b.sd;
        nodes[q] = n;
    }
    gen_body<T, 0, MID, LdsNode>(a, V, nodes, MID ? o.shift : nullptr, u.b0 == 0, w0, w1);
}

hipError_t launch_generate_batch(const BatchOpt *opts, const GenUnit *units, int n_units,
                                 const uint32_t *V, uint32_t *gsync, int max_dates, int fp64,
                                 bool shifted, hipStream_t s)
{
    const size_t lds = (generate_lds_bytes(max_dates, fp64) + 15) / 16 * 16 + (size_t)max_dates * sizeof(LdsNode);
    const dim3 g(n_units), b(kWG);
    if (shifted) {
        // randomised QMC: every option of the batch carries its digital shift
        if (fp64) hipLaunchKernelGGL((gen_batch_kernel<double, true>), g, b, lds, s, opts, units, V, gsync);
        else      hipLaunchKernelGGL((gen_batch_kernel<float, true>), g, b, lds, s, opts, units, V, gsync);
    } else {
        if (fp64) hipLaunchKernelGGL((gen_batch_kernel<double, false>), g, b, lds, s, opts, units, V, gsync);
        else      hipLaunchKernelGGL((gen_batch_kernel<float, false>), g, b, lds, s, opts, units, V, gsync);
    }
    return hipGetLastError();
}

hipError_t launch_sweep_batch(const BatchOpt *opts, const int32_t *tile_opt, const BatchGlobal &g,
                              int grid, int fp64, int ppt, int degree, bool cooperative, hipStream_t s)
{
    const void *f = sweep_lookup(fp64, g.laguerre, ppt, degree, 1);
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
    // sums about c = max(h(S0), 0): the variance below cancels only to the
    // order of (mean - c)^2 / variance
    const double h0 = call ? a.S0 - a.K : a.K - a.S0;
    const double csh = h0 > 0.0 ? h0 : 0.0;
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
        const double c = (double)disc * (double)v - csh;
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
        const double mean = csh + s_tot[0] / n;
        double var = a.N > 1 ? (s_tot[1] - s_tot[0] * (s_tot[0] / n)) / (n - 1.0) : 0.0;
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
