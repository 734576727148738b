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
// [1/2, 1); F = 1/2 + j/128 + 1/256 from the top 6 fraction bits j of m, so
// f = m - F is exact and |u| = |f / F| <= 2^-7; log v = e ln 2 + log F +
// log1p(u), log1p by its Taylor series to degree 7 (truncation below 2e-18).
// kLogTab[j] = log F rounded to nearest from a 60-digit decimal evaluation.
// About 1 ulp for the tail's arguments (results of magnitude 0.9 and more).
__constant__ double kLogTab[64] = {
    -0x1.5ee82aa241920p-1, -0x1.5707a26bb8c66p-1, -0x1.4f45a835a4e19p-1, -0x1.47a1527e8a2d3p-1,
    -0x1.4019c2125ca93p-1, -0x1.38ae2171976e7p-1, -0x1.315da4434068bp-1, -0x1.2a2786d0ec107p-1,
    -0x1.230b0d8bebc98p-1, -0x1.1c07849ae6007p-1, -0x1.151c3f6f29612p-1, -0x1.0e4898611cce1p-1,
    -0x1.078bf0533c568p-1, -0x1.00e5ae5b207abp-1, -0x1.f4aa7ee03192dp-2, -0x1.e7b42c3ddad73p-2,
    -0x1.dae75484c9616p-2, -0x1.ce42f18064743p-2, -0x1.c1c60693fa39ep-2, -0x1.b56fa04462909p-2,
    -0x1.a93ed3c8ad9e3p-2, -0x1.9d32bea15ed3bp-2, -0x1.914a8635bf68ap-2, -0x1.85855776dcbfbp-2,
    -0x1.79e26687cfb3ep-2, -0x1.6e60ee6af1972p-2, -0x1.630030b3aac49p-2, -0x1.57bf753c8d1fbp-2,
    -0x1.4c9e09e172c3cp-2, -0x1.419b423d5e8c7p-2, -0x1.36b6776be1117p-2, -0x1.2bef07cdc9354p-2,
    -0x1.214456d0eb8d4p-2, -0x1.16b5ccbacfb73p-2, -0x1.0c42d676162e3p-2, -0x1.01eae5626c691p-2,
    -0x1.ef5ade4dcffe6p-3, -0x1.db13db0d48940p-3, -0x1.c6ffbc6f00f71p-3, -0x1.b31d8575bce3dp-3,
    -0x1.9f6c407089664p-3, -0x1.8beafeb38fe8cp-3, -0x1.7898d85444c73p-3, -0x1.6574ebe8c133ap-3,
    -0x1.527e5e4a1b58dp-3, -0x1.3fb45a59928ccp-3, -0x1.2d1610c86813ap-3, -0x1.1aa2b7e23f72ap-3,
    -0x1.08598b59e3a07p-3, -0x1.ec739830a1120p-4, -0x1.c885801bc4b23p-4, -0x1.a4e7640b1bc38p-4,
    -0x1.8197e2f40e3f0p-4, -0x1.5e95a4d9791cbp-4, -0x1.3bdf5a7d1ee64p-4, -0x1.1973bd1465567p-4,
    -0x1.eea31c006b87cp-5, -0x1.aaef2d0fb10fcp-5, -0x1.67c94f2d4bb58p-5, -0x1.252f32f8d183fp-5,
    -0x1.c63d2ec14aaf2p-6, -0x1.432a925980cc1p-6, -0x1.82448a388a2aap-7, -0x1.0080559588b35p-8,
};

// exp(x) in binary64 by Tang's table method (P. T. P. Tang, "Table-driven
// implementation of the exponential function in IEEE floating-point
// arithmetic", ACM TOMS 15(2), 1989): n = rint(64 x / ln 2), g = x - n ln 2 / 64
// (Cody-Waite: ln 2 / 64 split into a 53-bit head and its tail, each product
// taken exactly inside an fma), |g| <= ln 2 / 128; exp(x) = 2^(n div 64)
// 2^((n mod 64) / 64) e^g, with e^g - 1 by its Taylor series to degree 5
// (truncation below 0.0055^6 / 6! < 4e-17 relative) and the table value
// added last.  kExpTab[j] = 2^(j / 64) rounded to nearest from a 60-digit
// decimal evaluation.  tab(j) reads the table (the path generator's LDS
// copy).  For the log-prices the generator produces (|x| < 700).
__constant__ double kExpTab[64] = {
    0x1.0000000000000p+0, 0x1.02c9a3e778061p+0, 0x1.059b0d3158574p+0, 0x1.0874518759bc8p+0,
    0x1.0b5586cf9890fp+0, 0x1.0e3ec32d3d1a2p+0, 0x1.11301d0125b51p+0, 0x1.1429aaea92de0p+0,
    0x1.172b83c7d517bp+0, 0x1.1a35beb6fcb75p+0, 0x1.1d4873168b9aap+0, 0x1.2063b88628cd6p+0,
    0x1.2387a6e756238p+0, 0x1.26b4565e27cddp+0, 0x1.29e9df51fdee1p+0, 0x1.2d285a6e4030bp+0,
    0x1.306fe0a31b715p+0, 0x1.33c08b26416ffp+0, 0x1.371a7373aa9cbp+0, 0x1.3a7db34e59ff7p+0,
    0x1.3dea64c123422p+0, 0x1.4160a21f72e2ap+0, 0x1.44e086061892dp+0, 0x1.486a2b5c13cd0p+0,
    0x1.4bfdad5362a27p+0, 0x1.4f9b2769d2ca7p+0, 0x1.5342b569d4f82p+0, 0x1.56f4736b527dap+0,
    0x1.5ab07dd485429p+0, 0x1.5e76f15ad2148p+0, 0x1.6247eb03a5585p+0, 0x1.6623882552225p+0,
    0x1.6a09e667f3bcdp+0, 0x1.6dfb23c651a2fp+0, 0x1.71f75e8ec5f74p+0, 0x1.75feb564267c9p+0,
    0x1.7a11473eb0187p+0, 0x1.7e2f336cf4e62p+0, 0x1.82589994cce13p+0, 0x1.868d99b4492edp+0,
    0x1.8ace5422aa0dbp+0, 0x1.8f1ae99157736p+0, 0x1.93737b0cdc5e5p+0, 0x1.97d829fde4e50p+0,
    0x1.9c49182a3f090p+0, 0x1.a0c667b5de565p+0, 0x1.a5503b23e255dp+0, 0x1.a9e6b5579fdbfp+0,
    0x1.ae89f995ad3adp+0, 0x1.b33a2b84f15fbp+0, 0x1.b7f76f2fb5e47p+0, 0x1.bcc1e904bc1d2p+0,
    0x1.c199bdd85529cp+0, 0x1.c67f12e57d14bp+0, 0x1.cb720dcef9069p+0, 0x1.d072d4a07897cp+0,
    0x1.d5818dcfba487p+0, 0x1.da9e603db3285p+0, 0x1.dfc97337b9b5fp+0, 0x1.e502ee78b3ff6p+0,
    0x1.ea4afa2a490dap+0, 0x1.efa1bee615a27p+0, 0x1.f50765b6e4540p+0, 0x1.fa7c1819e90d8p+0,
};

template <typename Tab>
__device__ __forceinline__ double exp_tab(double x, Tab tab)
{
    const double n = rint(x * 92.332482616893658);            // 64 / ln 2
    const double g = fma(-n, 3.6235106466348431e-19, fma(-n, 0.010830424696249145, x));
    double p = fma3(1.0 / 120.0, g, kInvFact4);                 // 1/4! (see exp_poly)
    p = fma3(p, g, 1.0 / 6.0);
    p = fma(p, g, 0.5);
    p = fma(p, g, 1.0);
    const int ni = (int)n;
    const double t = tab((uint32_t)ni & 63u);
    return ldexp(fma(t, p * g, t), ni >> 6);
}

// logF: the table, from constant memory or from an LDS copy (the path
// generator's: its loads then wait on LDS only, not on the generator's
// pending stores); 1/F by the reciprocal's Newton refinement.
template <typename LogF>
__device__ __forceinline__ double log_tab(double v, LogF logF)
{
    const double m = __builtin_amdgcn_frexp_mant(v);
    const int e = __builtin_amdgcn_frexp_exp(v);
    const uint32_t j = (uint32_t)((uint64_t)__double_as_longlong(m) >> 46) & 63u;
    const double F = fma((double)j, 0x1p-7, 0.5 + 0x1p-8);
    const double u = (m - F) * rcp_f64(F);
    double p = fma(u, 1.0 / 7.0, -1.0 / 6.0);
    p = fma(p, u, 0.2);
    p = fma(p, u, -0.25);
    p = fma(p, u, 1.0 / 3.0);
    p = fma(p, u, -0.5);
    const double l1p = fma(p, u * u, u);
    const double de = (double)e;
    return fma(de, 0.69314718055994529, fma(de, 2.3190468138462996e-17, logF(j) + l1p));
}

__device__ __forceinline__ double log_tab(double v)
{
    return log_tab(v, [](uint32_t j) { return kLogTab[j]; });
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
        // Horner steps as single fmas (three-address: the coefficients stay
        // in registers of their own)
        double v = AMQ_C8;
        v = fma3(v, t, AMQ_C7);
        v = fma3(v, t, AMQ_C6);
        v = fma3(v, t, AMQ_C5);
        v = fma3(v, t, AMQ_C4);
        v = fma3(v, t, AMQ_C3);
        v = fma3(v, t, AMQ_C2);
        v = fma3(v, t, AMQ_C1);
        v = fma3(v, t, AMQ_C0);
        return y < 0.0 ? -v : v;
    }
    static __device__ __forceinline__ double tail_value(uint32_t x)
    {
        return tail_value(x, [](uint32_t j) { return kLogTab[j]; });
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

// A bridge node as the batch generator keeps it in LDS: 32 bytes (date and
// dimension in one word, the three window slots in another), so that the
// schedule of 256 dates and the generator's tables leave room for four
// groups per CU.
struct LdsNode {
    uint32_t md;    // m | dim << 16
    uint32_t slots; // sl | sr << 8 | dst << 16
    double wl, wr, sd;
};
static_assert(sizeof(LdsNode) == 32, "LDS bridge node");
static_assert(kMaxDates < 65536 && kMaxSlots <= 256, "LDS bridge node packing");

// A node's integer fields, wave-uniform (scalar registers).
struct NodeIdx { int m, dim, sl, sr, dst; };
__device__ __forceinline__ NodeIdx node_idx(const BridgeNode &n)
{
    return {__builtin_amdgcn_readfirstlane(n.m), __builtin_amdgcn_readfirstlane(n.dim),
            __builtin_amdgcn_readfirstlane(n.sl), __builtin_amdgcn_readfirstlane(n.sr),
            __builtin_amdgcn_readfirstlane(n.dst)};
}
__device__ __forceinline__ NodeIdx node_idx(const LdsNode &n)
{
    const uint32_t md = (uint32_t)__builtin_amdgcn_readfirstlane((int)n.md);
    const uint32_t sv = (uint32_t)__builtin_amdgcn_readfirstlane((int)n.slots);
    return {(int)(md & 0xFFFFu), (int)(md >> 16), (int)(sv & 0xFFu), (int)((sv >> 8) & 0xFFu), (int)(sv >> 16)};
}

// Nodes whose tail normals are evaluated together (binary64 paths): a
// 64-point Sobol block puts about 10 of its 64 points of each dimension in
// the tails (|u - 1/2| >= 0.42), so the tails of 5 nodes mostly fill one wave.
constexpr int kTailChunk = 5;
// Tail points staged per wave and chunk: every lane of every node
// (kTailFull), or kTailSmall.  An aligned block of 64 Sobol points has
// exactly one point in each interval [k/64, (k+1)/64) of every dimension (the
// generator matrix's leading 6 x 6 block is triangular with unit diagonal),
// and the tails meet 12 such intervals; a wave's lanes hold 63 points of one
// aligned block and the first of the next, so a node has at most 13 tail
// points and a chunk at most 65 <= kTailSmall.  The smaller staging lets
// four groups per CU hold their tables at 256 dates and more; its slots are
// masked to the staging, so no point set could write outside it.
constexpr int kTailFull = kTailChunk * 64, kTailSmall = 128;
static_assert((kTailSmall & (kTailSmall - 1)) == 0 && kTailSmall >= 13 * kTailChunk, "tail staging");

__host__ __device__ size_t generate_lds_bytes(int M, int cap)
{
    // lane tables [M][16], per-wave block words [kWaves][M][2], per-wave tail
    // staging: points [cap] u32 and normals [cap] f64 (both storage types:
    // the normals are binary64), the logarithm's table [64] f64, the
    // exponential's table [64] f64
    return (size_t)M * 16 * sizeof(uint32_t) + (size_t)kWaves * M * 2 * sizeof(uint32_t) +
           (size_t)kWaves * cap * (sizeof(uint32_t) + sizeof(double)) + 8 + (64 + 64) * sizeof(double);
}

// The single-option generator's staging: the full one while the four groups
// per CU that the kernel's registers allow still fit in LDS with it, else
// the smaller.
int gen_tail_cap(int M, int fp64)
{
    (void)fp64;
    const size_t share = (size_t)160 * 1024 / 4;
    return generate_lds_bytes(M, kTailFull) <= share ? kTailFull : kTailSmall;
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
template <typename T, int WHAT, bool MID, int CAP, typename Node>
__device__ __forceinline__ void gen_body(const GenArgs &a, const uint32_t *__restrict__ V,
                                         const Node *__restrict__ sched,
                                         const uint32_t *__restrict__ shift, bool init, int64_t w0,
                                         int64_t w1)
{
    extern __shared__ uint32_t lds[];
    const int M = a.M;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // the wave's block range in scalar registers (it is the same in every
    // lane), so each store's row address is scalar and the lane's offset a
    // constant
    const auto uniform_i64 = [](int64_t v) {
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
        return (int64_t)(((uint64_t)hi << 32) | lo);
    };
    w0 = uniform_i64(w0);
    w1 = uniform_i64(w1);
    uint32_t *ttab = lds;                                   // [M][16]
    uint32_t *xw = lds + (size_t)M * 16 + (size_t)wave * M * 2;   // [M][2]
    // this wave's tail staging (see kTailChunk)
    uint32_t *tx = lds + (size_t)M * 16 + (size_t)kWaves * M * 2 + (size_t)wave * CAP;
    double *tz0 = reinterpret_cast<double *>(reinterpret_cast<char *>(lds) +
                                  (((size_t)M * 16 + (size_t)kWaves * M * 2 + (size_t)kWaves * CAP) *
                                       sizeof(uint32_t) + 7) / 8 * 8);
    double *tz = tz0 + (size_t)wave * CAP;
    // the logarithm's table, for the packed tails
    double *ltab = tz0 + (size_t)kWaves * CAP;
    for (int j = tid; j < 64; j += kWG) ltab[j] = kLogTab[j];
    // the exponential's table
    double *etab = ltab + 64;
    for (int j = tid; j < 64; j += kWG) etab[j] = kExpTab[j];
    const auto etab_at = [=](uint32_t j) { return etab[j]; };

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
            // two logarithms dominate).  Every lane evaluates the (cheap)
            // central branch of kTailChunk nodes up front (independent of one
            // another and of the bridge, so their latencies overlap); the
            // points in the tails are packed into this wave's LDS staging
            // (ballot and lane rank), their tail values evaluated together,
            // one point per lane, and read back by their owners.  The values
            // are exactly those of inv_normal.
            for (int s0 = 0; s0 < M; s0 += kTailChunk) {
                uint32_t slot[kTailChunk];
                double zcq[kTailChunk];   // central values, computed with the tail test
                bool tl[kTailChunk];
                uint32_t ntail = 0;   // wave-uniform
#pragma unroll
                for (int q = 0; q < kTailChunk; ++q) {
                    tl[q] = false;
                    if (s0 + q < M) {
                        const int j = node_idx(sched[s0 + q]).dim;
                        const uint32_t x = xw[2 * j + xsel] ^ ttab[j * 16 + offL] ^ ttab[j * 16 + offH];
                        zcq[q] = MoroParts<double>::central(x);
                        tl[q] = MoroParts<double>::tail(x);
                        const uint64_t m = __builtin_amdgcn_ballot_w64(tl[q]);
                        slot[q] = ntail + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                        if constexpr (CAP < kTailFull) slot[q] &= (uint32_t)(CAP - 1);
                        if (tl[q]) tx[slot[q]] = x;
                        ntail += (uint32_t)__builtin_popcountll(m);
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                const uint32_t nstaged = min(ntail, (uint32_t)CAP);
                for (uint32_t t0 = 0; t0 < nstaged; t0 += 64) {
                    const uint32_t t = t0 + (uint32_t)lane;
                    if (t < nstaged)
                        tz[t] = MoroParts<double>::tail_value(tx[t], [=](uint32_t j) { return ltab[j]; });
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
                for (int q = 0; q < kTailChunk; ++q) {
                    if (s0 + q < M) {
                        const Node &nd = sched[s0 + q];
                        const NodeIdx ni = node_idx(nd);
                        const int n_m = ni.m, n_sl = ni.sl, n_sr = ni.sr, n_dst = ni.dst;
                        const double n_wl = uniform_f64(nd.wl), n_wr = uniform_f64(nd.wr),
                                     n_sd = uniform_f64(nd.sd);
                        const double z = tl[q] ? tz[slot[q]] : zcq[q];
                        const double xv = n_wl * X[n_sl] + n_wr * X[n_sr] + n_sd * (vol * z);
                        X[n_dst] = xv;
                        const T Sv = (T)exp_tab(xv, etab_at);
                        ((T *)a.S + ((size_t)(n_m - 1) * a.ld + ((size_t)w << 6)))[(uint32_t)lane] = valid ? Sv : Kp;
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
            const NodeIdx ni = node_idx(nd);
            const int j = ni.dim, n_m = ni.m, n_sl = ni.sl, n_sr = ni.sr, n_dst = ni.dst;
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
            const T Sv = (T)exp_tab(xv, etab_at);
            ((T *)a.S + ((size_t)(n_m - 1) * a.ld + ((size_t)w << 6)))[(uint32_t)lane] = valid ? Sv : Kp;
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

// four waves per SIMD (128 registers; with five the node loop spills):
// latency hiding for the per-lane dependency chain of each path through the
// dates
template <typename T, int WHAT, bool MID, int CAP>
__global__ void __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(4)))
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
    gen_body<T, WHAT, MID, CAP, BridgeNode>(a, V, sched, shift, blockIdx.x == 0, w0, w1);
}

hipError_t launch_generate(const GenArgs &a, int fp64, hipStream_t s)
{
    const int64_t waves = (a.nblocks + a.R - 1) / a.R;
    const int64_t grid = (waves + kWaves - 1) / kWaves;
    const dim3 g((unsigned)grid), b(kWG);
    const bool mid = a.shift != nullptr;
    // only the packed tails (unshifted points, paths) use the staging
    const int cap = (a.what == 0 && !mid) ? gen_tail_cap(a.M, fp64) : kTailSmall;
    const size_t lds = generate_lds_bytes(a.M, cap);
    const bool full = cap == kTailFull;
    if (a.what == 0) {
        if (fp64) {
            if (mid)       hipLaunchKernelGGL((gen_kernel<double, 0, true, kTailSmall>), g, b, lds, s, a, a.V, a.sched, a.shift);
            else if (full) hipLaunchKernelGGL((gen_kernel<double, 0, false, kTailFull>), g, b, lds, s, a, a.V, a.sched, a.shift);
            else           hipLaunchKernelGGL((gen_kernel<double, 0, false, kTailSmall>), g, b, lds, s, a, a.V, a.sched, a.shift);
        } else {
            if (mid)       hipLaunchKernelGGL((gen_kernel<float, 0, true, kTailSmall>), g, b, lds, s, a, a.V, a.sched, a.shift);
            else if (full) hipLaunchKernelGGL((gen_kernel<float, 0, false, kTailFull>), g, b, lds, s, a, a.V, a.sched, a.shift);
            else           hipLaunchKernelGGL((gen_kernel<float, 0, false, kTailSmall>), g, b, lds, s, a, a.V, a.sched, a.shift);
        }
    } else if (a.what == 1) {
        hipLaunchKernelGGL((gen_kernel<float, 1, false, kTailSmall>), g, b, lds, s, a, a.V, a.sched, a.shift);
    } else {
        // the normals are binary64 for both storage types
        hipLaunchKernelGGL((gen_kernel<double, 2, false, kTailSmall>), g, b, lds, s, a, a.V, a.sched, a.shift);
    }
    return hipGetLastError();
}

// Make the runtime load the generation kernels' code on the current device
// now rather than at their first launch (a first use allocates device memory
// for the code).
hipError_t preload_generate()
{
    hipFuncAttributes fa;
    hipError_t e = hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(&gen_kernel<float, 0, false, kTailFull>));
    if (e == hipSuccess) e = hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(&gen_kernel<double, 0, false, kTailFull>));
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
__global__ void __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(4)))
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
                                                 (generate_lds_bytes(o.M, kTailSmall) + 15) / 16 * 16);
    for (int q = threadIdx.x; q < o.M; q += kWG) {
        const BridgeNode &b = o.sched[q];
        LdsNode n;
        n.md = (uint32_t)b.m | (uint32_t)b.dim << 16;
        n.slots = (uint32_t)b.sl | (uint32_t)b.sr << 8 | (uint32_t)b.dst << 16;
        n.wl = b.wl; n.wr = b.wr; n.sd = b.sd;
        nodes[q] = n;
    }
    gen_body<T, 0, MID, kTailSmall, LdsNode>(a, V, nodes, MID ? o.shift : nullptr, u.b0 == 0, w0, w1);
}

hipError_t launch_generate_batch(const BatchOpt *opts, const GenUnit *units, int n_units,
                                 const uint32_t *V, uint32_t *gsync, int max_dates, int fp64,
                                 bool shifted, hipStream_t s)
{
    const size_t lds = (generate_lds_bytes(max_dates, kTailSmall) + 15) / 16 * 16 + (size_t)max_dates * sizeof(LdsNode);
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
