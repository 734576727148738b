/*
 * amq_oracle.h — the FP64 CPU oracle for quasi-Monte Carlo American option
 * valuation (Cvetanoska & Stojanovski, "Using High Performance Computing and
 * Monte Carlo Simulation for Pricing American Options").
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that
 * the GPU path is checked against.  Only tests/, __graft_entry__.smoke() and
 * bench.py's cpu_baseline leg may load it; the product path never does.  It
 * shares no code, header, table or constant generator with the HIP library.
 *
 * Everything is IEEE binary64, single-threaded, round-to-nearest, no
 * fast-math.  Each function names the passage of the paper (or of the method
 * the paper cites) that it follows.
 */
#ifndef AMQ_ORACLE_H
#define AMQ_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct or_params {
    double S0;      /* spot at t0 (the paper's S_0) */
    double K;       /* strike (the paper's exercise price X) */
    double r;       /* continuously compounded risk-free rate */
    double sigma;   /* volatility (the paper's v) */
    double T;       /* expiry */
    int32_t is_call;        /* 1 call, 0 put */
    int32_t allow_exercise; /* 1: Bermudan exercise at t_1..t_M and t0; 0: European */
} or_params;

typedef struct or_result {
    double price;       /* max(h(S0), mean PV) with exercise, mean PV without */
    double std_err;     /* naive iid sd(PV)/sqrt(N); 0 when exercise at t0 wins */
    double mean_pv;     /* mean of the per-path discounted cashflows */
    int32_t t0_exercise;/* 1 when h(S0) exceeded the mean PV */
    int32_t n_skipped;  /* regression dates skipped as degenerate */
} or_result;

enum { OR_BASIS_MONOMIAL = 0, OR_BASIS_LAGUERRE = 1 };
enum { OR_EUROPEAN = 0, OR_AMERICAN = 1, OR_BERMUDAN = 2 };

/* beta_out rows: [M+1][OR_BETA_STRIDE]; row k holds beta_0..beta_{p-1} of date
 * t_k in the basis of or_basis_eval (targets discounted to t_k) and a 1.0 at
 * column 8 when the date's regression was solved. */
#define OR_BETA_STRIDE 16

/* Sobol direction numbers from primitive polynomials and initial values. */
int or_sobol_directions(int ndim, const int64_t *poly, const int64_t *vinit,
                        int vinit_cols, uint32_t *V);
uint32_t or_sobol_int(const uint32_t *V, int dim0, uint64_t n);
void or_sobol_block(const uint32_t *V, int ndim, uint64_t first, int64_t count,
                    uint32_t *out);

/* Moro (Beasley–Springer–Moro) inverse cumulative normal. */
double or_inv_normal(double u);
double or_inv_normal_u32(uint32_t x);
double or_inv_normal_mid_u32(uint32_t x);

/* Brownian bridge, breadth-first bisection. */
int or_bridge_nodes(int M, int32_t *m, int32_t *left, int32_t *right);
void or_bridge_apply(int M, double T, const double *z, double *W);

/* Paths S[M][N]: row k-1 holds date t_k = kT/M for every path. */
int or_paths(const or_params *p, const uint32_t *V, int64_t N, int M, double *S);
int or_paths_range(const or_params *p, const uint32_t *V, int64_t first, int64_t count, int M,
                   double *S);
int or_paths_range_shifted(const or_params *p, const uint32_t *V, int64_t first, int64_t count,
                           int M, const uint32_t *shift, double *S);

/* Basis functions of x = S/K. Returns the number of functions. */
int or_basis_eval(int kind, int degree, double x, double *psi);

/* Least-squares (Longstaff–Schwartz) backward induction on given paths. */
int or_lsm_on_paths(const double *S, int64_t N, int M, const or_params *p,
                    int kind, int degree, or_result *res,
                    double *beta_out, int32_t *nitm_out, int32_t *tau_out,
                    double *pv_out);

/* Same, with binary32 storage when store32 != 0: path values read rounded to
 * binary32, cashflows held discounted to t0 and rounded to binary32; all
 * arithmetic binary64.  The paper fixes no storage precision; this is the
 * method on binary32 storage, the definition the GPU's FP32-bulk mode is
 * checked against. */
int or_lsm_on_paths_stored(const double *S, int64_t N, int M, const or_params *p,
                           int kind, int degree, int store32, or_result *res,
                           double *beta_out, int32_t *nitm_out, int32_t *tau_out,
                           double *pv_out);

/* Full oracle: Sobol -> inverse normal -> bridge -> GBM -> LSM -> mean. */
int or_price_american(const or_params *p, const uint32_t *V, int64_t N, int M,
                      int kind, int degree, or_result *res,
                      double *beta_out, int32_t *nitm_out, double *pv_out);

/* Same, on digitally shifted points (shift: [M], one word per dimension). */
int or_price_american_shifted(const or_params *p, const uint32_t *V, int64_t N, int M,
                              int kind, int degree, const uint32_t *shift, or_result *res,
                              double *beta_out, int32_t *nitm_out, double *pv_out);

/* Same again, optionally on binary32 storage (store32 != 0, as in
 * or_lsm_on_paths_stored). */
int or_price_american_stored(const or_params *p, const uint32_t *V, int64_t N, int M,
                             int kind, int degree, const uint32_t *shift, int store32,
                             or_result *res, double *beta_out, int32_t *nitm_out,
                             double *pv_out);

/* The paper's own estimator: Black–Scholes over the last interval, then a
 * per-path backward maximum (eqs. (10)-(11)). */
int or_paper_estimator(const or_params *p, const uint32_t *V, int64_t N, int m,
                       or_result *res);

/* Closed form and lattice checks. */
double or_bs_price(double S0, double K, double r, double sigma, double T,
                   int is_call);
double or_crr_price(double S0, double K, double r, double sigma, double T,
                    int is_call, int n, int style, int M);

#ifdef __cplusplus
}
#endif
#endif
