/*
 * amq_oracle.c — FP64 CPU oracle for quasi-Monte Carlo American option
 * valuation.
 *
 * TEST INFRASTRUCTURE ONLY: this is the plain, slow, single-threaded
 * reference that the GPU library is checked against.  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark load it.  It shares
 * no code, header, table or constant generator with the HIP library.
 *
 * What it computes, in the paper's order:
 *   - quasi-random points (Section III.D: quasi Monte Carlo, uniforms mapped
 *     to N(0,1) by Moro's inverse cumulative normal);
 *   - GBM paths on the discrete exercise grid (Section V, eq. (9); the
 *     dates are the Bermudan set of Section III.E);
 *   - the backward induction over those dates (Section V, eqs. (10)-(11)),
 *     in the least-squares continuation-value form of Longstaff–Schwartz
 *     (reference [12]; Section V says the approach is similar to the
 *     regression methods [9] and [19]);
 *   - the discounted mean of eqs. (6)-(8);
 *   - the Black–Scholes closed form of eqs. (1)-(5) and a CRR binomial tree
 *     (the lattice method named in Section III.E) as independent checks.
 *
 * Readings where the paper is silent or garbled:
 *   - dates t_k = kT/M, k = 1..M, so t_M = T (Section V states t_m = T);
 *   - Sobol sequence, Joe–Kuo direction numbers, Gray-code order, point
 *     index 0 skipped (path i uses index i+1); dimension j feeds bridge
 *     node j in breadth-first bisection order, dimension 1 gives W(T);
 *   - the GBM step of eq. (9) taken as the exact lognormal map
 *     S_k = S0 exp((r - v^2/2) t_k + v W(t_k));
 *   - in-the-money means payoff strictly positive; exercise iff payoff is
 *     strictly greater than the fitted continuation value;
 *   - a regression date with fewer in-the-money paths than basis functions,
 *     or a numerically rank-deficient design, allows no exercise;
 *   - exercise at t0 is allowed in American mode: price = max(h(S0), mean).
 *
 * Parity pins for every function live in tests/ (test_oracle_*.py).
 */
#include "amq_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Sobol points (Section III.D, "quasi-random generator").                   */
/* Direction numbers follow the Bratley–Fox recurrence with Joe–Kuo's        */
/* primitive polynomials and initial values.  poly[j] encodes the polynomial */
/* x^s + a_1 x^{s-1} + ... + a_{s-1} x + 1 as the bit string 1 a_1..a_{s-1} 1.*/
/* Dimension 0 is the van der Corput sequence (all m_k = 1).                 */
/* ------------------------------------------------------------------------ */
int or_sobol_directions(int ndim, const int64_t *poly, const int64_t *vinit,
                        int vinit_cols, uint32_t *V)
{
    for (int j = 0; j < ndim; ++j) {
        uint64_t m[33];
        if (j == 0) {
            for (int k = 1; k <= 32; ++k) m[k] = 1;
        } else {
            int64_t pj = poly[j];
            int s = 0;
            while ((pj >> (s + 1)) != 0) ++s;          /* degree */
            if (s < 1 || s > vinit_cols) return -1;
            uint64_t a = (uint64_t)(pj >> 1) & ((1ull << (s - 1)) - 1ull);
            for (int k = 1; k <= s && k <= 32; ++k) m[k] = (uint64_t)vinit[(int64_t)j * vinit_cols + (k - 1)];
            for (int k = s + 1; k <= 32; ++k) {
                uint64_t v = m[k - s] ^ (m[k - s] << s);
                for (int i = 1; i <= s - 1; ++i) {
                    uint64_t ai = (a >> (s - 1 - i)) & 1ull;
                    if (ai) v ^= m[k - i] << i;
                }
                m[k] = v;
            }
        }
        for (int b = 0; b < 32; ++b)
            V[(int64_t)j * 32 + b] = (uint32_t)(m[b + 1] << (31 - b));
    }
    return 0;
}

/* x_j(n) = XOR of V_j[b] over the set bits b of the Gray code n ^ (n >> 1). */
uint32_t or_sobol_int(const uint32_t *V, int dim0, uint64_t n)
{
    uint64_t g = n ^ (n >> 1);
    uint32_t x = 0;
    for (int b = 0; b < 32 && g; ++b, g >>= 1)
        if (g & 1ull) x ^= V[(int64_t)dim0 * 32 + b];
    return x;
}

void or_sobol_block(const uint32_t *V, int ndim, uint64_t first, int64_t count,
                    uint32_t *out)
{
    for (int64_t i = 0; i < count; ++i)
        for (int j = 0; j < ndim; ++j)
            out[i * ndim + j] = or_sobol_int(V, j, first + (uint64_t)i);
}

/* ------------------------------------------------------------------------ */
/* Moro's inverse cumulative normal (Section III.D).  Central region: the    */
/* Beasley–Springer rational function in y = u - 1/2 for |y| < 0.42; tails: */
/* Moro's Chebyshev-type polynomial in log(-log(q)), q the tail probability.*/
/* Coefficients from Moro (1995), "The full Monte", Risk 8(2).               */
/* ------------------------------------------------------------------------ */
static const double BSM_A[4] = { 2.50662823884, -18.61500062529,
                                 41.39119773534, -25.44106049637 };
static const double BSM_B[4] = { -8.47351093090, 23.08336743743,
                                 -21.06224101826, 3.13082909833 };
static const double BSM_C[9] = { 0.3374754822726147, 0.9761690190917186,
                                 0.1607979714918209, 0.0276438810333863,
                                 0.0038405729373609, 0.0003951896511919,
                                 0.0000321767881768, 0.0000002888167364,
                                 0.0000003960315187 };

static double bsm_central(double y)
{
    double r = y * y;
    double num = y * (((BSM_A[3] * r + BSM_A[2]) * r + BSM_A[1]) * r + BSM_A[0]);
    double den = ((((BSM_B[3] * r + BSM_B[2]) * r + BSM_B[1]) * r + BSM_B[0]) * r) + 1.0;
    return num / den;
}

/* q: tail probability in (0, 1/2]; returns the positive quantile Phi^-1(1-q). */
static double bsm_tail(double q)
{
    double t = log(-log(q));
    double v = BSM_C[8];
    for (int i = 7; i >= 0; --i) v = v * t + BSM_C[i];
    return v;
}

double or_inv_normal(double u)
{
    double y = u - 0.5;
    if (fabs(y) < 0.42) return bsm_central(y);
    if (y < 0.0) return -bsm_tail(u);
    return bsm_tail(1.0 - u);
}

/* u = x 2^-32 for a Sobol integer x.  In binary64 u, u - 1/2 and 1 - u are all
 * exact, so the tail for u > 1/2 uses the exact complement (2^32 - x) 2^-32
 * and Phi^-1 is exactly odd under x -> 2^32 - x. */
double or_inv_normal_u32(uint32_t x)
{
    const double s = 1.0 / 4294967296.0;
    double y = ((double)x - 2147483648.0) * s;
    if (fabs(y) < 0.42) return bsm_central(y);
    if (y < 0.0) return -bsm_tail((double)x * s);
    return bsm_tail((4294967296.0 - (double)x) * s);
}

/* Randomised points (reading of Section III.D's permuted quasi-random arrays:
 * a random digital shift x' = x XOR s_j per dimension).  A shifted integer can
 * be 0, so shifted points sit at cell midpoints u = (x' + 1/2) 2^-32, exact in
 * binary64; the upper tail again uses the exact complement. */
double or_inv_normal_mid_u32(uint32_t x)
{
    const double s = 1.0 / 4294967296.0;
    double y = ((double)x + 0.5 - 2147483648.0) * s;
    if (fabs(y) < 0.42) return bsm_central(y);
    if (y < 0.0) return -bsm_tail(((double)x + 0.5) * s);
    return bsm_tail((4294967296.0 - (double)x - 0.5) * s);
}

/* ------------------------------------------------------------------------ */
/* Brownian bridge (the construction of reference [13]).                     */
/* Node 0 sets W(t_M); then intervals are bisected breadth first, left       */
/* before right: an interval (l, r) with r - l >= 2 gets its midpoint        */
/* m = floor((l + r)/2) as the next node.  Node q uses Sobol dimension q+1.  */
/* ------------------------------------------------------------------------ */
int or_bridge_nodes(int M, int32_t *m_out, int32_t *l_out, int32_t *r_out)
{
    if (M < 1) return -1;
    int32_t *ql = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * M + 2));
    int32_t *qr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * M + 2));
    if (!ql || !qr) { free(ql); free(qr); return -2; }
    int head = 0, tail = 0, q = 0;
    m_out[q] = M; l_out[q] = 0; r_out[q] = 0; ++q;   /* W(T) from W(0) = 0 */
    ql[tail] = 0; qr[tail] = M; ++tail;
    while (head < tail) {
        int l = ql[head], r = qr[head]; ++head;
        if (r - l < 2) continue;
        int m = (l + r) / 2;
        m_out[q] = m; l_out[q] = l; r_out[q] = r; ++q;
        ql[tail] = l; qr[tail] = m; ++tail;
        ql[tail] = m; qr[tail] = r; ++tail;
    }
    free(ql); free(qr);
    return q == M ? 0 : -3;
}

/* W[0..M]: W[0] = 0, W[k] = W(t_k) with t_k = kT/M; z[q] feeds node q. */
void or_bridge_apply(int M, double T, const double *z, double *W)
{
    int32_t *nm = (int32_t *)malloc(sizeof(int32_t) * (size_t)M);
    int32_t *nl = (int32_t *)malloc(sizeof(int32_t) * (size_t)M);
    int32_t *nr = (int32_t *)malloc(sizeof(int32_t) * (size_t)M);
    or_bridge_nodes(M, nm, nl, nr);
    W[0] = 0.0;
    W[M] = sqrt(T) * z[0];
    for (int q = 1; q < M; ++q) {
        double tl = (double)nl[q] * T / (double)M;
        double tm = (double)nm[q] * T / (double)M;
        double tr = (double)nr[q] * T / (double)M;
        double mean = ((tr - tm) * W[nl[q]] + (tm - tl) * W[nr[q]]) / (tr - tl);
        double sd = sqrt((tm - tl) * (tr - tm) / (tr - tl));
        W[nm[q]] = mean + sd * z[q];
    }
    free(nm); free(nl); free(nr);
}

/* ------------------------------------------------------------------------ */
/* GBM paths on the exercise grid (Section V, eq. (9), exact lognormal map). */
/* ------------------------------------------------------------------------ */
/* Paths first..first+count-1 into S[M][count]; shift (nullable, [M]) applies a
 * digital shift to dimension q and maps points to cell midpoints. */
int or_paths_range_shifted(const or_params *p, const uint32_t *V, int64_t first, int64_t count,
                           int M, const uint32_t *shift, double *S);

int or_paths_range(const or_params *p, const uint32_t *V, int64_t first, int64_t count, int M,
                   double *S)
{
    return or_paths_range_shifted(p, V, first, count, M, NULL, S);
}

int or_paths_range_shifted(const or_params *p, const uint32_t *V, int64_t first, int64_t count,
                           int M, const uint32_t *shift, double *S)
{
    double *z = (double *)malloc(sizeof(double) * (size_t)M);
    double *W = (double *)malloc(sizeof(double) * (size_t)(M + 1));
    if (!z || !W) { free(z); free(W); return -2; }
    double drift = p->r - 0.5 * p->sigma * p->sigma;
    for (int64_t c = 0; c < count; ++c) {
        uint64_t n = (uint64_t)(first + c) + 1u;       /* skip the origin */
        for (int q = 0; q < M; ++q)
            z[q] = shift ? or_inv_normal_mid_u32(or_sobol_int(V, q, n) ^ shift[q])
                         : or_inv_normal_u32(or_sobol_int(V, q, n));
        or_bridge_apply(M, p->T, z, W);
        for (int k = 1; k <= M; ++k) {
            double tk = (double)k * p->T / (double)M;
            S[(int64_t)(k - 1) * count + c] = p->S0 * exp(drift * tk + p->sigma * W[k]);
        }
    }
    free(z); free(W);
    return 0;
}

int or_paths(const or_params *p, const uint32_t *V, int64_t N, int M, double *S)
{
    return or_paths_range(p, V, 0, N, M, S);
}

/* ------------------------------------------------------------------------ */
/* Regression basis, functions of x = S/K (reference [12]).                  */
/* MONOMIAL: 1, x, ..., x^d.  LAGUERRE: exp(-x/2) L_n(x), n = 0..d, with the */
/* Laguerre polynomials from L_{n+1} = ((2n+1-x) L_n - n L_{n-1})/(n+1).     */
/* ------------------------------------------------------------------------ */
int or_basis_eval(int kind, int degree, double x, double *psi)
{
    int p = degree + 1;
    if (kind == OR_BASIS_MONOMIAL) {
        psi[0] = 1.0;
        for (int a = 1; a < p; ++a) psi[a] = psi[a - 1] * x;
    } else {
        double w = exp(-0.5 * x);
        double lm1 = 0.0, l0 = 1.0;
        for (int n = 0; n < p; ++n) {
            psi[n] = w * l0;
            double l1 = ((2.0 * n + 1.0 - x) * l0 - (double)n * lm1) / (double)(n + 1);
            lm1 = l0; l0 = l1;
        }
    }
    return p;
}

static double payoff(const or_params *p, double S)
{
    double h = p->is_call ? S - p->K : p->K - S;
    return h > 0.0 ? h : 0.0;
}

/* Neumaier-compensated running sum. */
typedef struct { double s, c; } ksum;
static void ks_add(ksum *k, double v)
{
    double t = k->s + v;
    if (fabs(k->s) >= fabs(v)) k->c += (k->s - t) + v;
    else                       k->c += (v - t) + k->s;
    k->s = t;
}
static double ks_val(const ksum *k) { return k->s + k->c; }

#define OR_MAXP 8

/* Streaming Givens QR for min ||X beta - y||: one row (psi, y) at a time is
 * rotated into the upper-triangular R and the rotated target qy. */
static void givens_row(int p, double R[OR_MAXP][OR_MAXP], double *qy,
                       double *psi, double y)
{
    for (int j = 0; j < p; ++j) {
        double b = psi[j];
        if (b == 0.0) continue;
        double a = R[j][j];
        double rr = hypot(a, b);
        double c = a / rr, s = b / rr;
        R[j][j] = rr;
        for (int l = j + 1; l < p; ++l) {
            double t1 = R[j][l], t2 = psi[l];
            R[j][l] = c * t1 + s * t2;
            psi[l] = -s * t1 + c * t2;
        }
        double t1 = qy[j];
        qy[j] = c * t1 + s * y;
        y = -s * t1 + c * y;
    }
}

/* ------------------------------------------------------------------------ */
/* Backward induction (Section V; least-squares continuation of [12]).       */
/* CF/tau hold each path's cashflow and its stopping date; the regression    */
/* target at date k is the realised cashflow discounted back to t_k.         */
/*                                                                          */
/* store32 != 0: binary32 storage.  Every path value is read rounded to the  */
/* nearest binary32, and every cashflow is held as its value discounted to   */
/* t0 rounded to the nearest binary32 (PV32); the regression target at t_k   */
/* is then PV32 carried forward to t_k.  All arithmetic stays binary64.      */
/* ------------------------------------------------------------------------ */
static double rd32(double v) { return (double)(float)v; }   /* round to nearest */

int or_lsm_on_paths(const double *S, int64_t N, int M, const or_params *p,
                    int kind, int degree, or_result *res,
                    double *beta_out, int32_t *nitm_out, int32_t *tau_out,
                    double *pv_out)
{
    return or_lsm_on_paths_stored(S, N, M, p, kind, degree, 0, res, beta_out, nitm_out,
                                  tau_out, pv_out);
}

int or_lsm_on_paths_stored(const double *S, int64_t N, int M, const or_params *p,
                           int kind, int degree, int store32, or_result *res,
                           double *beta_out, int32_t *nitm_out, int32_t *tau_out,
                           double *pv_out)
{
    int np = degree + 1;
    if (N < 1 || M < 1 || np < 1 || np > OR_MAXP) return -1;
    double *CF = (double *)malloc(sizeof(double) * (size_t)N);
    int32_t *tau = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    double *t = (double *)malloc(sizeof(double) * (size_t)(M + 1));
    double *PV32 = store32 ? (double *)malloc(sizeof(double) * (size_t)N) : NULL;
    if (!CF || !tau || !t || (store32 && !PV32)) {
        free(CF); free(tau); free(t); free(PV32);
        return -2;
    }
    for (int k = 0; k <= M; ++k) t[k] = (double)k * p->T / (double)M;
#define SV(x) (store32 ? rd32(x) : (x))

    const double *last = S + (int64_t)(M - 1) * N;
    for (int64_t i = 0; i < N; ++i) {
        CF[i] = payoff(p, SV(last[i]));
        tau[i] = M;
        if (store32) PV32[i] = rd32(CF[i] * exp(-p->r * t[M]));
    }
    if (beta_out) for (int64_t q = 0; q < (int64_t)(M + 1) * OR_BETA_STRIDE; ++q) beta_out[q] = 0.0;
    if (nitm_out) for (int k = 0; k <= M; ++k) nitm_out[k] = 0;

    int skipped = 0;
    if (p->allow_exercise) {
        for (int k = M - 1; k >= 1; --k) {
            const double *row = S + (int64_t)(k - 1) * N;
            int64_t nitm = 0;
            for (int64_t i = 0; i < N; ++i) if (payoff(p, SV(row[i])) > 0.0) ++nitm;
            if (nitm_out) nitm_out[k] = (int32_t)nitm;
            if (nitm < np) { ++skipped; continue; }

            double R[OR_MAXP][OR_MAXP];
            double qy[OR_MAXP], psi[OR_MAXP], beta[OR_MAXP];
            memset(R, 0, sizeof(R)); memset(qy, 0, sizeof(qy));
            for (int64_t i = 0; i < N; ++i) {
                const double s = SV(row[i]);
                double h = payoff(p, s);
                if (!(h > 0.0)) continue;
                or_basis_eval(kind, degree, s / p->K, psi);
                double y = store32 ? PV32[i] * exp(p->r * t[k])
                                   : CF[i] * exp(-p->r * (t[tau[i]] - t[k]));
                givens_row(np, R, qy, psi, y);
            }
            double dmax = 0.0, dmin = INFINITY;
            for (int j = 0; j < np; ++j) {
                double d = fabs(R[j][j]);
                if (d > dmax) dmax = d;
                if (d < dmin) dmin = d;
            }
            if (!(dmax > 0.0) || dmin <= 1e-13 * dmax) { ++skipped; continue; }
            for (int j = np - 1; j >= 0; --j) {
                double v = qy[j];
                for (int l = j + 1; l < np; ++l) v -= R[j][l] * beta[l];
                beta[j] = v / R[j][j];
            }
            if (beta_out) {
                for (int j = 0; j < np; ++j) beta_out[(int64_t)k * OR_BETA_STRIDE + j] = beta[j];
                beta_out[(int64_t)k * OR_BETA_STRIDE + OR_MAXP] = 1.0;   /* valid flag */
            }
            for (int64_t i = 0; i < N; ++i) {
                const double s = SV(row[i]);
                double h = payoff(p, s);
                if (!(h > 0.0)) continue;
                or_basis_eval(kind, degree, s / p->K, psi);
                double cont = 0.0;
                for (int j = 0; j < np; ++j) cont += psi[j] * beta[j];
                if (h > cont) {
                    CF[i] = h;
                    tau[i] = k;
                    if (store32) PV32[i] = rd32(h * exp(-p->r * t[k]));
                }
            }
        }
    }

    /* eqs. (6)-(8): per-path cashflow discounted to t0, then the mean. */
    ksum sum = {0.0, 0.0};
#undef SV
    for (int64_t i = 0; i < N; ++i) {
        double pv = store32 ? PV32[i] : CF[i] * exp(-p->r * t[tau[i]]);
        if (pv_out) pv_out[i] = pv;
        if (tau_out) tau_out[i] = tau[i];
        CF[i] = pv;
        ks_add(&sum, pv);
    }
    double mean = ks_val(&sum) / (double)N;
    ksum ss = {0.0, 0.0};
    for (int64_t i = 0; i < N; ++i) { double d = CF[i] - mean; ks_add(&ss, d * d); }
    double var = N > 1 ? ks_val(&ss) / (double)(N - 1) : 0.0;
    double se = sqrt(var) / sqrt((double)N);

    res->mean_pv = mean;
    res->n_skipped = skipped;
    res->t0_exercise = 0;
    res->price = mean;
    res->std_err = se;
    if (p->allow_exercise) {
        double h0 = payoff(p, p->S0);
        if (h0 > mean) { res->price = h0; res->std_err = 0.0; res->t0_exercise = 1; }
    }
    free(CF); free(tau); free(t); free(PV32);
    return 0;
}

int or_price_american(const or_params *p, const uint32_t *V, int64_t N, int M,
                      int kind, int degree, or_result *res,
                      double *beta_out, int32_t *nitm_out, double *pv_out)
{
    return or_price_american_shifted(p, V, N, M, kind, degree, NULL, res, beta_out, nitm_out,
                                     pv_out);
}

int or_price_american_shifted(const or_params *p, const uint32_t *V, int64_t N, int M,
                              int kind, int degree, const uint32_t *shift, or_result *res,
                              double *beta_out, int32_t *nitm_out, double *pv_out)
{
    return or_price_american_stored(p, V, N, M, kind, degree, shift, 0, res, beta_out,
                                    nitm_out, pv_out);
}

int or_price_american_stored(const or_params *p, const uint32_t *V, int64_t N, int M,
                             int kind, int degree, const uint32_t *shift, int store32,
                             or_result *res, double *beta_out, int32_t *nitm_out,
                             double *pv_out)
{
    if (N < 1 || M < 1) return -1;
    double *S = (double *)malloc(sizeof(double) * (size_t)N * (size_t)M);
    if (!S) return -2;
    int rc = or_paths_range_shifted(p, V, 0, N, M, shift, S);
    if (rc == 0) rc = or_lsm_on_paths_stored(S, N, M, p, kind, degree, store32, res, beta_out,
                                             nitm_out, NULL, pv_out);
    free(S);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Black–Scholes closed form, eqs. (1)-(5); CND(d) = erfc(-d/sqrt 2)/2.       */
/* ------------------------------------------------------------------------ */
static double cnd(double d) { return 0.5 * erfc(-d / sqrt(2.0)); }

double or_bs_price(double S0, double K, double r, double sigma, double T,
                   int is_call)
{
    double sq = sigma * sqrt(T);
    double d1 = (log(S0 / K) + (r + 0.5 * sigma * sigma) * T) / sq;
    double d2 = d1 - sq;
    if (is_call) return S0 * cnd(d1) - K * exp(-r * T) * cnd(d2);
    return K * exp(-r * T) * cnd(-d2) - S0 * cnd(-d1);
}

/* ------------------------------------------------------------------------ */
/* The paper's own estimator (Section V, eqs. (9)-(11), eq. (6)).            */
/* Reading: m dates t_i = i T/(m+1), i = 1..m, spacing dt = T/(m+1).  At t_m  */
/* the value is max(h(S), BS value over the last interval dt) (eq. (10));    */
/* going back, c_i = max(h(S_i), exp(-r dt) c_{i+1}) (eq. (11)); the price is */
/* exp(-r dt) times the path mean of c_1 (eq. (6) with one step of eq. (8)). */
/* m = 0 leaves only the Black–Scholes value at t0.  Paths use the bridge on */
/* the grid t_1..t_m (horizon m dt) and the same Sobol/inverse normal.       */
/* ------------------------------------------------------------------------ */
int or_paper_estimator(const or_params *p, const uint32_t *V, int64_t N, int m,
                       or_result *res)
{
    if (N < 1 || m < 0) return -1;
    double dt = p->T / (double)(m + 1);
    if (m == 0) {
        double c = or_bs_price(p->S0, p->K, p->r, p->sigma, p->T, p->is_call);
        res->price = res->mean_pv = c; res->std_err = 0.0;
        res->t0_exercise = 0; res->n_skipped = 0;
        return 0;
    }
    double *z = (double *)malloc(sizeof(double) * (size_t)m);
    double *W = (double *)malloc(sizeof(double) * (size_t)(m + 1));
    double *c = (double *)malloc(sizeof(double) * (size_t)N);
    if (!z || !W || !c) { free(z); free(W); free(c); return -2; }
    double horizon = dt * (double)m;
    double drift = p->r - 0.5 * p->sigma * p->sigma;
    double disc = exp(-p->r * dt);
    ksum sum = {0.0, 0.0};
    for (int64_t i = 0; i < N; ++i) {
        uint64_t n = (uint64_t)i + 1u;
        for (int q = 0; q < m; ++q) z[q] = or_inv_normal_u32(or_sobol_int(V, q, n));
        or_bridge_apply(m, horizon, z, W);
        double v = 0.0;
        for (int k = m; k >= 1; --k) {
            double tk = (double)k * horizon / (double)m;
            double S = p->S0 * exp(drift * tk + p->sigma * W[k]);
            double h = payoff(p, S);
            double cont = (k == m) ? or_bs_price(S, p->K, p->r, p->sigma, dt, p->is_call)
                                   : disc * v;
            v = h > cont ? h : cont;
        }
        c[i] = disc * v;
        ks_add(&sum, c[i]);
    }
    double mean = ks_val(&sum) / (double)N;
    ksum ss = {0.0, 0.0};
    for (int64_t i = 0; i < N; ++i) { double d = c[i] - mean; ks_add(&ss, d * d); }
    double var = N > 1 ? ks_val(&ss) / (double)(N - 1) : 0.0;
    res->mean_pv = mean; res->price = mean;
    res->std_err = sqrt(var) / sqrt((double)N);
    res->t0_exercise = 0; res->n_skipped = 0;
    free(z); free(W); free(c);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Cox–Ross–Rubinstein binomial tree (the lattice method of Section III.E).  */
/* style: European; American (exercise at every step); Bermudan (exercise at */
/* steps that are multiples of n/M, which includes t0).                       */
/* ------------------------------------------------------------------------ */
double or_crr_price(double S0, double K, double r, double sigma, double T,
                    int is_call, int n, int style, int M)
{
    if (n < 1) return NAN;
    if (style == OR_BERMUDAN && (M < 1 || n % M != 0)) return NAN;
    double dt = T / (double)n;
    double sdt = sigma * sqrt(dt);
    double u = exp(sdt), d = 1.0 / u;
    double q = (exp(r * dt) - d) / (u - d);
    double disc = exp(-r * dt);
    double *Vv = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    if (!Vv) return NAN;
    or_params pp = { S0, K, r, sigma, T, is_call, 1 };
    for (int j = 0; j <= n; ++j) Vv[j] = payoff(&pp, S0 * exp((double)(2 * j - n) * sdt));
    int stride = (style == OR_BERMUDAN) ? n / M : 1;
    for (int i = n - 1; i >= 0; --i) {
        int ex = (style == OR_AMERICAN) || (style == OR_BERMUDAN && i % stride == 0);
        for (int j = 0; j <= i; ++j) {
            double v = disc * (q * Vv[j + 1] + (1.0 - q) * Vv[j]);
            if (ex) {
                double h = payoff(&pp, S0 * exp((double)(2 * j - i) * sdt));
                if (h > v) v = h;
            }
            Vv[j] = v;
        }
    }
    double out = Vv[0];
    free(Vv);
    return out;
}
