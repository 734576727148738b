// amq_internal.h — types shared by the HIP kernels and the host engine.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace amq {

constexpr int kWG = 256;          // threads per workgroup (4 wave64)
constexpr int kWaves = kWG / 64;
constexpr int kMaxSlots = 16;     // bridge register window (tree depth + 2; depth <= 10 for 640 dates)
constexpr int kAnchorSlot = kMaxSlots - 1;   // read by the first bridge node only
constexpr int kMaxDates = 640;    // on-chip Sobol lane tables (<= 64 KiB of LDS) bound this
constexpr int kRec = 40;          // doubles per date record
constexpr int kRecTime = 32;      // record slots 32..37: device clock stamps of the date's phases
constexpr int kPartStride = 32;   // doubles per workgroup partial slot (estimator kernel)
constexpr int kMaxGroups = 2048;  // workgroups of one sweep or estimator launch, at most
constexpr int kMaxReps = 64;      // randomised QMC replicates per call

// Barrier block of one sweep (uint32 words, one 64-byte line per counter):
//   line 0: [2] error word (a wait ran out: every workgroup exits),
//           [4] ticket (paper kernel);
//   lines 1 .. kMaxTeams: team arrival counters (monotone; team t has
//   received all arrivals of epoch e at e * (its member count)).
// Groups form at most kMaxTeams teams of team_size(G) consecutive groups.
constexpr int kMaxTeams = 32;
constexpr int kSyncLine = 16;
constexpr int kSyncWords = kSyncLine * (1 + kMaxTeams);
__host__ __device__ inline uint32_t team_size(uint32_t G) { return (G + kMaxTeams - 1) / kMaxTeams; }

// Partial-sum rows of one sweep: [2 epoch parities][G][row_words] 8-byte
// words, then the team rows [2][kMaxTeams][row_words]; each word holds an FP64 partial whose two lowest mantissa bits carry
// epoch & 3 (see allreduce in amq_sync.h).  Zeroed by the generation kernel.
__host__ __device__ constexpr int row_words(int degree) { return 3 * degree + 3 <= 16 ? 16 : 32; }
constexpr int kMaxRowWords = 32;
// group rows [2][G][row_words] then team rows [2][kMaxTeams][row_words]
__host__ __device__ inline int64_t rows_words(int64_t G, int degree) { return 2 * (G + kMaxTeams) * row_words(degree); }
// row padding: a multiple of every sweep tile up to 32768 paths; the
// 65536-path tile is used only where it divides the padded row
constexpr int64_t kLdAlign = 32768;

// One node of the Brownian bridge, in depth-first construction order.  The
// value of W at date m (in units of sqrt(dt)) is
//   W[dst] = wl * W[sl] + wr * W[sr] + sd * z(dim)
// where slots hold the values of the current node's ancestors (slot 0 is the
// constant W(0) = 0).  The first node (date M) reads the anchor slot
// kAnchorSlot with weight 1, which holds 0 for W; no node writes that slot.
// Because wl + wr = 1 below the root, the same schedule carries any process
// a + b t + c W(t): the generation kernels run it on the log-price
// log S0 + (r - sigma^2/2) t + sigma W(t), with slot 0 = log S0, the anchor
// = log S0 + (r - sigma^2/2) T and sigma sqrt(dt) z in place of z.
// Both precisions are stored so each kernel reads one.
struct alignas(64) BridgeNode {
    int32_t m;      // date index 1..M
    int32_t dim;    // Sobol dimension, 0-based
    int32_t sl, sr, dst;
    float fm;       // m as float
    double wl, wr, sd;
    float fwl, fwr, fsd;
    int32_t pad;
};
static_assert(sizeof(BridgeNode) == 64, "bridge node is one scalar cache line");

// Per-date constants written by the generation kernel, read by the sweep.
//   disc = exp(-r t_k); standardised abscissa xs = S * xa + xb with
//   xa = 1/(K sd_k), xb = -mean_k/sd_k (mean/sd of S_k/K in the money under
//   the model).
struct DateConst {
    double disc, xa, xb, pad;
};

struct GenArgs {
    void *S;                  // [M][ld] T (what = 0) or debug output
    const uint32_t *V;        // [dims][32] direction numbers
    const BridgeNode *sched;  // [M]
    DateConst *datec;         // [M+1]
    uint32_t *sync;           // barrier words, zeroed here
    int64_t N, ld;
    int64_t nblocks;          // 64-path blocks to write: ld / 64 (padding included)
    int32_t M, R;             // dates, 64-path blocks per wave
    int32_t what;             // 0 paths, 1 sobol ints, 2 normals (debug)
    int32_t pad;
    const uint32_t *shift;    // [M] digital shift (randomised QMC) or nullptr
    double S0, K, r, sigma, T;
    double mu, vol;           // (r - sigma^2/2) dt, sigma sqrt(dt)
    int32_t is_call, pad2;    // payoff side (standardisation of the in-the-money region)
    uint64_t *rows;           // partial-sum rows to zero (with the barrier words)
    int64_t rows_n;           // their count in 8-byte words
};

struct SweepArgs {
    const void *S;            // [M][ld] T
    void *pv_out;             // [ld] T
    uint64_t *rows;           // partial-sum rows [2][G][row_words(degree)]
    double *rec;              // [M+1][kRec]
    double *result;           // [8]
    uint32_t *sync;           // barrier block [kSyncWords]
    uint32_t *err;            // error word: a wait ran out (every group exits)
    const DateConst *datec;   // [M+1]
    int64_t N, ld;
    int32_t M, G;
    int32_t is_call, allow_exercise, laguerre, degree;
    double S0, K;
    uint32_t spin_limit;
    int32_t pad;
    double *rep_out;          // randomised QMC: replicate prices [n_rep] or nullptr
    int32_t rep, n_rep;
};

struct PaperArgs {
    const void *S;            // [m][ld] T, dates t_i = i dt
    double *part;             // [kMaxGroups][kPartStride]
    uint32_t *ticket;         // zeroed by the generation kernel
    double *result;           // [8]
    int64_t N, ld;
    int32_t m, is_call;
    double K, r, sigma, dt, S0;
};

// One option of a batch, as the kernels see it (all pointers into the
// caller's workspace or the library's schedule cache).
struct alignas(64) BatchOpt {
    void *S;                  // [M][ld] T
    void *pv;                 // [ld] T
    const BridgeNode *sched;  // [M]
    DateConst *datec;         // [M+1]
    double *rec;              // [M+1][kRec]
    double *result;           // [8]
    uint32_t *sync;           // barrier block [kSyncWords] of this option
    uint64_t *rows;           // partial-sum rows [2][G][row_words(degree)] of this option
    int64_t rows_n;           // their count in 8-byte words (zeroed by generation)
    int64_t N, ld;
    int32_t M, G;             // dates, tiles
    int32_t tile_base;        // first partial slot / global tile index
    int32_t is_call, allow_exercise, pad;
    double S0, K, r, sigma, T, mu, vol;
    const uint32_t *shift;    // [M] digital shift per dimension (randomised QMC), or null
};

struct GenUnit {              // one generation workgroup: blocks [b0, b1) of option opt
    int32_t opt, pad;
    int64_t b0, b1;
};

struct BatchGlobal {
    uint32_t *claim;          // tile claim counter (zeroed by generation)
    uint32_t *err;            // error word (zeroed by generation)
    int32_t total_tiles, laguerre;
    uint32_t spin_limit, pad;
};

// Launchers (defined with the kernels).
hipError_t launch_generate(const GenArgs &a, int fp64, hipStream_t s);
// Load the single-option generation kernels on the current device.
hipError_t preload_generate();
// Single-option sweep with wg (256 or 512) threads per group.  Returns
// hipErrorInvalidValue if no kernel exists for (fp64, a.laguerre, wg, ppt,
// a.degree).
hipError_t launch_sweep(const SweepArgs &a, int fp64, int wg, int ppt, hipStream_t s);
// Workgroups of the sweep kernel that fit on one CU (0: no such kernel).
int sweep_blocks_per_cu(int fp64, int laguerre, int wg, int ppt, int degree);
__host__ __device__ size_t generate_lds_bytes(int M, int cap);
hipError_t launch_paper(const PaperArgs &a, int fp64, hipStream_t s);
hipError_t launch_generate_batch(const BatchOpt *opts, const GenUnit *units, int n_units,
                                 const uint32_t *V, uint32_t *gsync, int max_dates, int fp64,
                                 bool shifted, hipStream_t s);
hipError_t launch_sweep_batch(const BatchOpt *opts, const int32_t *tile_opt, const BatchGlobal &g,
                              int grid, int fp64, int ppt, int degree, bool cooperative, hipStream_t s);
int sweep_batch_blocks_per_cu(int fp64, int laguerre, int ppt, int degree);
// Sweep kernel tables, one translation unit per (precision, basis kind);
// kind 0: single option, 256-thread groups; 1: many options; 2: single
// option, 512-thread groups.  Null where not built.
const void *sweep_table_f32_mono(int ppt, int degree, int kind);
const void *sweep_table_f32_lag(int ppt, int degree, int kind);
const void *sweep_table_f64_mono(int ppt, int degree, int kind);
const void *sweep_table_f64_lag(int ppt, int degree, int kind);

}  // namespace amq
