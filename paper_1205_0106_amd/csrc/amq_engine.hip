// amq_engine.hip — host engine and C-ABI (include/amqmc.h).
//
// Owns per-device state (Sobol direction numbers, bridge schedules per date
// count, a stream and workspace for the synchronous entry point), validates
// arguments, lays out the workspace and launches the two kernels.
#include "amqmc.h"
#include "amq_internal.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

// Direction numbers V[dim][bit] (uint32), embedded at build time.
extern "C" const uint32_t amq_sobol_v32[];
extern "C" const uint32_t amq_sobol_v32_dims;

// Workspace of the allocation-free entry point (am_price_american_noalloc):
// AM_SCRATCH_BYTES on every device the library runs on, held until the
// process ends.  In host code this name is only a handle for the runtime:
// am_init resolves each device's own copy with hipGetSymbolAddress and every
// host-side use (kernel arguments, copies) goes through DevState::scratch.
static __device__ __align__(256) unsigned char scratch[AM_SCRATCH_BYTES];

namespace {

thread_local std::string g_err = "no error";
// am_shutdown releases every thread's cached pinned buffer and profiling
// events; a thread notices through the generation and sets them up again.
std::mutex g_res_mu;
uint64_t g_generation = 1;
std::vector<void *> g_pinned_all;       // every thread's pinned result buffer
std::vector<hipEvent_t> g_events_all;   // every thread's profiling events
int g_live_servers = 0;
thread_local uint32_t g_spin_limit = 0;
thread_local int32_t g_batch_ppt = 0;   // batch tile choice (0 = default or tuned)
constexpr uint32_t kDefaultSpin = 1u << 22;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(AM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));       \
    } while (0)

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Generation waves launched per CU (each wave takes an equal range of 64-path
// blocks): many short ranges leave no long tail of waves on a few CUs.  With
// 16 waves resident per CU, measured on config 4 (2^24 paths x 252 dates):
// 32 per CU 11.6 ms, 128 10.8-11.0, 256 10.7-10.8, 512 10.8, 1024 10.9; the
// batch of 1024 options: 32 39.9 ms, 256 35.6-36.2, 512 35.1, 1024 35.0.
constexpr int64_t kGenWavesPerCU = 256;
constexpr int64_t kBatchGenWavesPerCU = 512;

// Storage a pricing request gets: binary32 bulk storage only from
// AM_FP32_MIN_PATHS paths up (below that one decision that rounds the other
// way can exceed the FP32-bulk tolerance by itself).
int32_t storage_of(int64_t N, int32_t dtype)
{
    return (dtype == AM_FP32_BULK && N < AM_FP32_MIN_PATHS) ? AM_FP64 : dtype;
}

struct Layout {
    int64_t ld;
    size_t s_bytes;  // element size
    size_t off_S, off_PV, off_part, off_rec, off_datec, off_result, off_shift, off_rep, total;
};

Layout make_layout(int64_t N, int32_t M, int32_t dtype)
{
    Layout L;
    L.s_bytes = dtype == AM_FP64 ? 8 : 4;
    L.ld = (N + amq::kLdAlign - 1) / amq::kLdAlign * amq::kLdAlign;
    size_t o = 0;
    L.off_S = o;      o = align256(o + (size_t)M * (size_t)L.ld * L.s_bytes);
    L.off_PV = o;     o = align256(o + (size_t)L.ld * L.s_bytes);
    // sweep partial-sum rows [2][G][row words] (also the estimator's partial slots)
    L.off_part = o;   o = align256(o + (size_t)2 * (amq::kMaxGroups + amq::kMaxTeams) * amq::kMaxRowWords * 8);
    L.off_rec = o;    o = align256(o + (size_t)(M + 1) * amq::kRec * 8);
    L.off_datec = o;  o = align256(o + (size_t)(M + 1) * sizeof(amq::DateConst));
    L.off_result = o; o = align256(o + 8 * 8 + amq::kSyncWords * 4);   // result[8], barrier block
    L.off_shift = o;  o = align256(o + (size_t)amq::kMaxReps * M * 4);
    L.off_rep = o;    o = align256(o + (size_t)amq::kMaxReps * 8);
    L.total = o;
    return L;
}

// Depth-first bridge schedule with breadth-first dimension numbering.
std::vector<amq::BridgeNode> make_schedule(int M)
{
    std::vector<int> dim_of(M + 1, -1);
    std::vector<std::pair<int, int>> q;
    q.reserve(2 * M + 2);
    dim_of[M] = 0;
    int next = 1;
    q.push_back({0, M});
    for (size_t h = 0; h < q.size(); ++h) {
        const int l = q[h].first, r = q[h].second;
        if (r - l < 2) continue;
        const int m = (l + r) / 2;
        dim_of[m] = next++;
        q.push_back({l, m});
        q.push_back({m, r});
    }
    std::vector<amq::BridgeNode> out;
    out.reserve(M);
    auto emit = [&](int m, int l, int r, int sl, int sr, int dst) {
        amq::BridgeNode n;
        memset(&n, 0, sizeof n);
        n.m = m;
        n.dim = dim_of[m];
        n.sl = sl; n.sr = sr; n.dst = dst;
        n.fm = (float)m;
        if (l == 0 && r == 0) {           // root: W(t_M) = anchor + sqrt(M) z in sqrt(dt) units
            n.wl = 1.0; n.wr = 0.0; n.sd = sqrt((double)M);
        } else {
            const double span = (double)(r - l);
            n.wl = (double)(r - m) / span;
            n.wr = (double)(m - l) / span;
            n.sd = sqrt((double)(m - l) * (double)(r - m) / span);
        }
        n.fwl = (float)n.wl; n.fwr = (float)n.wr; n.fsd = (float)n.sd;
        out.push_back(n);
    };
    emit(M, 0, 0, amq::kAnchorSlot, 0, 1);
    // explicit stack: (l, r, slot of W(l), slot of W(r), depth of the midpoint)
    struct Fr { int l, r, sl, sr, depth; };
    std::vector<Fr> st;
    st.push_back({0, M, 0, 1, 1});
    while (!st.empty()) {
        Fr f = st.back();
        st.pop_back();
        if (f.r - f.l < 2) continue;
        const int m = (f.l + f.r) / 2;
        const int dst = f.depth + 1;
        emit(m, f.l, f.r, f.sl, f.sr, dst);
        st.push_back({m, f.r, dst, f.sr, f.depth + 1});   // right after left
        st.push_back({f.l, m, f.sl, dst, f.depth + 1});
    }
    return out;
}

int max_slot(const std::vector<amq::BridgeNode> &s)
{
    int mx = 0;
    for (auto &n : s) mx = n.dst > mx ? n.dst : mx;
    return mx;
}

struct Plan { int wg; int ppt; int G; };

struct DevState {
    int dev = -1;
    int num_cu = 0;
    uint32_t *d_V = nullptr;
    int vdims = 0;
    std::mutex mu;                                  // schedule and occupancy maps
    std::map<int, amq::BridgeNode *> sched;
    std::mutex sync_mu;                             // synchronous entry point's workspace
    hipStream_t stream = nullptr;                   // synchronous entry point
    void *ws = nullptr;
    size_t ws_bytes = 0;
    std::map<long, int> occ;                        // (kind, fp64, wg, ppt, degree) -> groups per CU
    // single-option sweeps hold every CU for their whole run and wait on one
    // another's groups only within their own grid: launches on different
    // streams are ordered through this event, in enqueue order, so two never
    // share the device
    std::mutex persist_mu;
    hipEvent_t persist_done = nullptr;
    hipStream_t persist_stream = nullptr;
    // allocation-free entry point: this device's copy of `scratch` (set by
    // am_init) and host-side bridge schedules for it, built once per date count
    char *scratch = nullptr;
    std::map<int, std::vector<amq::BridgeNode>> host_sched;
};

std::mutex g_dev_mu;
std::map<int, std::unique_ptr<DevState>> g_devs;

int get_state(DevState **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_dev_mu);
    auto it = g_devs.find(dev);
    if (it != g_devs.end()) { *out = it->second.get(); return AM_OK; }
    std::unique_ptr<DevState> st(new DevState);
    st->dev = dev;
    HIP_TRY(hipDeviceGetAttribute(&st->num_cu, hipDeviceAttributeMultiprocessorCount, dev));
    int coop = 0;
    HIP_TRY(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    if (!coop) return fail(AM_EDEVICE, "device %d does not support cooperative launches", dev);
    st->vdims = (int)amq_sobol_v32_dims < amq::kMaxDates ? (int)amq_sobol_v32_dims : amq::kMaxDates;
    const size_t vb = (size_t)st->vdims * 32 * sizeof(uint32_t);
    if (hipMalloc((void **)&st->d_V, vb) != hipSuccess)
        return fail(AM_ENOMEM, "hipMalloc of %zu bytes (direction numbers) failed", vb);
    HIP_TRY(hipMemcpy(st->d_V, amq_sobol_v32, vb, hipMemcpyHostToDevice));
    HIP_TRY(hipStreamCreateWithFlags(&st->stream, hipStreamNonBlocking));
    *out = st.get();
    g_devs[dev] = std::move(st);
    return AM_OK;
}

// The current device's state if a call has set it up, else nullptr (creates nothing).
DevState *find_state()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    auto it = g_devs.find(dev);
    return it == g_devs.end() ? nullptr : it->second.get();
}

int get_schedule(DevState *st, int M, const amq::BridgeNode **out)
{
    std::lock_guard<std::mutex> lk(st->mu);
    auto it = st->sched.find(M);
    if (it != st->sched.end()) { *out = it->second; return AM_OK; }
    std::vector<amq::BridgeNode> h = make_schedule(M);
    if ((int)h.size() != M || max_slot(h) >= amq::kAnchorSlot)
        return fail(AM_EDIM, "bridge schedule for %d dates does not fit the register window", M);
    amq::BridgeNode *d = nullptr;
    const size_t b = sizeof(amq::BridgeNode) * (size_t)M;
    if (hipMalloc((void **)&d, b) != hipSuccess) return fail(AM_ENOMEM, "hipMalloc of bridge schedule failed");
    HIP_TRY(hipMemcpy(d, h.data(), b, hipMemcpyHostToDevice));
    st->sched[M] = d;
    *out = d;
    return AM_OK;
}

int groups_per_cu(DevState *st, int fp64, int laguerre, int wg, int ppt, int degree)
{
    const long key = ((long)(wg == 512) << 28) | ((long)laguerre << 24) | ((long)fp64 << 20) | ((long)ppt << 4) |
                     degree;
    std::lock_guard<std::mutex> lk(st->mu);
    auto it = st->occ.find(key);
    if (it != st->occ.end()) return it->second;
    const int nb = amq::sweep_blocks_per_cu(fp64, laguerre, wg, ppt, degree);
    st->occ[key] = nb;
    return nb;
}

// Single-option tiles (threads per group, paths per thread).  The 512-thread
// forms come first, so they win ties with the 256-thread form of the same
// tile size (binary32 streamed tiles too: one group of two waves per SIMD
// instead of two groups, half the groups in the device-wide sum).
struct TileShape { int wg, ppt; };
const TileShape kTiles32[] = {{512, 4}, {256, 4}, {512, 8}, {256, 16}, {512, 64}, {256, 64}, {512, 128}, {256, 128}};
const TileShape kTiles64[] = {{512, 2}, {256, 2}, {512, 4}, {256, 8}, {512, 8}, {256, 16}, {256, 64}};
const int kNTiles32 = 8, kNTiles64 = 7;
thread_local int32_t g_sweep_wide = 1;   // 0: single-option sweeps use 256-thread groups only
thread_local int32_t g_tile_wg = 0, g_tile_ppt = 0;   // a forced single-option tile (0: the cost model's)

// Tile choice for one sweep.  Every date costs one device-wide sum, whose
// latency grows with the group count G (every group reads every group's
// row), plus the per-date work.  Two regimes, both fitted to sweeps timed on
// gfx950 over 2^12 .. 2^20 paths, both storage types and three bases:
//  - small tiles (512 threads, at most 8 paths per thread) while their grid
//    is co-resident: the exchange costs about 3.7 us + 5 ns per group and a
//    group's pass about 12.5 ns per moment sum per path of a thread (each
//    group has a CU to itself, so the pass's length follows the paths per
//    thread, not the total).  They beat every 256-thread tile of the same
//    size (two waves per SIMD hide the pass's latency) by 5-14 % below 2^16
//    paths and up to 13 % at 2^18 - 2^19;
//  - larger N: the work spread over min(G, CUs) compute units at ~40 lane
//    operations per path (binary64: ~2x), against 4.5 us + 13 ns per group.
// Among the tiles whose grid is co-resident, the least modelled time per
// date, small tiles first.
int choose_plan(DevState *st, int64_t N, int fp64, int laguerre, int degree, Plan *p)
{
    const TileShape *tiles = fp64 ? kTiles64 : kTiles32;
    const int n_tiles = fp64 ? kNTiles64 : kNTiles32;
    // moment sums per path and date (Hankel moments and right-hand side, or
    // the Gram matrix, right-hand side and the Laguerre weight's exponential)
    const double sums = laguerre ? (double)((degree + 1) * (degree + 2) / 2 + degree + 1 + 3) : 3.0 * degree + 2.0;
    for (int pass = 0; pass < 2; ++pass) {
        double best = 0.0;
        bool found = false;
        for (int i = 0; i < n_tiles; ++i) {
            const int wg = tiles[i].wg, ppt = tiles[i].ppt;
            const bool small = wg == 512 && ppt <= 8;
            if (pass == 0 && !small) continue;
            if (wg != amq::kWG && !g_sweep_wide) continue;
            if (g_tile_wg && (wg != g_tile_wg || ppt != g_tile_ppt)) continue;
            const int per_cu = groups_per_cu(st, fp64, laguerre, wg, ppt, degree);
            if (per_cu <= 0) continue;
            int64_t gmax = (int64_t)per_cu * st->num_cu;
            if (gmax > amq::kMaxGroups) gmax = amq::kMaxGroups;
            const int64_t tile = (int64_t)wg * ppt;
            // the tiles must cover whole padded rows (a tile reads every path
            // it covers): tiles larger than the row padding only where they
            // divide the padded row length
            const int64_t ld = (N + amq::kLdAlign - 1) / amq::kLdAlign * amq::kLdAlign;
            if (ld % tile != 0) continue;
            const int64_t G = (N + tile - 1) / tile;
            if (G > gmax) continue;
            double t;
            if (pass == 0) {
                t = 0.005 * (double)G + 0.0125 * sums * (double)ppt;
            } else {
                // per-date work at 64 lanes x 4 SIMDs x 2.4 GHz per CU
                const double cus = (double)(G < st->num_cu ? G : st->num_cu);
                const double work_us = (double)N * (fp64 ? 80.0 : 40.0) / (cus * 4.0 * 16.0 * 2.4e3);
                t = 4.5 + 0.013 * (double)G + work_us;
            }
            if (!found || t < best) { best = t; p->wg = wg; p->ppt = ppt; p->G = (int)G; found = true; }
        }
        if (found) return AM_OK;
    }
    return fail(AM_EDIM, "n_paths = %lld exceeds what one resident sweep holds on this device",
                (long long)N);
}

int validate(const am_params *p, int64_t N, int32_t M, am_basis b, int32_t dtype)
{
    if (!p) return fail(AM_EINVAL, "params is NULL");
    const double v[] = {p->S0, p->K, p->sigma, p->T};
    const char *nm[] = {"S0", "K", "sigma", "T"};
    for (int i = 0; i < 4; ++i)
        if (!(isfinite(v[i]) && v[i] > 0.0)) return fail(AM_EINVAL, "%s must be finite and > 0", nm[i]);
    if (!isfinite(p->r)) return fail(AM_EINVAL, "r must be finite");
    if (p->is_call != 0 && p->is_call != 1) return fail(AM_EINVAL, "is_call must be 0 or 1");
    if (p->allow_exercise != 0 && p->allow_exercise != 1) return fail(AM_EINVAL, "allow_exercise must be 0 or 1");
    if (b.kind != AM_BASIS_MONOMIAL && b.kind != AM_BASIS_LAGUERRE) return fail(AM_EINVAL, "unknown basis kind %d", b.kind);
    if (b.degree < 0 || b.degree > AM_MAX_DEGREE) return fail(AM_EINVAL, "basis degree %d outside [0, %d]", b.degree, AM_MAX_DEGREE);
    if (dtype != AM_FP64 && dtype != AM_FP32_BULK) return fail(AM_EINVAL, "unknown dtype %d", dtype);
    if (M < 1) return fail(AM_EINVAL, "n_dates must be >= 1");
    if (M > amq::kMaxDates || (uint32_t)M > amq_sobol_v32_dims)
        return fail(AM_EDIM, "n_dates = %d exceeds %d", M, amq::kMaxDates);
    if (N < (int64_t)b.degree + 2) return fail(AM_EINVAL, "n_paths must be >= degree + 2");
    if (N > 0xFFFFFFFFll) return fail(AM_EDIM, "n_paths beyond the 32-bit Sobol index range");
    const double sd = p->sigma * sqrt(p->T);
    if (!(sd > 1e-12) || !isfinite(p->r * p->T)) return fail(AM_EINVAL, "degenerate sigma*sqrt(T) or r*T");
    return AM_OK;
}

// Per-thread kernel timing (am_profile_*): three events per timed call.
struct ProfRec { hipEvent_t e[3]; };
struct Profiler {
    bool on = false;
    std::vector<ProfRec> pool;   // created events, reused
    size_t used = 0;
    uint64_t gen = 0;            // g_generation the pool belongs to
};
thread_local Profiler g_prof;

int prof_slot(ProfRec **out)
{
    {
        std::lock_guard<std::mutex> lk(g_res_mu);
        if (g_prof.gen != g_generation) {   // released by am_shutdown
            g_prof.pool.clear();
            g_prof.used = 0;
            g_prof.gen = g_generation;
        }
    }
    if (g_prof.used == g_prof.pool.size()) {
        ProfRec r;
        for (int i = 0; i < 3; ++i) {
            HIP_TRY(hipEventCreate(&r.e[i]));
            std::lock_guard<std::mutex> lk(g_res_mu);
            g_events_all.push_back(r.e[i]);
        }
        g_prof.pool.push_back(r);
    }
    *out = &g_prof.pool[g_prof.used++];
    return AM_OK;
}

// Enqueue both kernels; result stays in the workspace.
// noalloc_sched: the allocation-free entry point passes the schedule it
// placed in its scratch memory; then nothing here allocates or creates a
// HIP object (no schedule cache entry, no profiling events, the ordering
// event made by am_init).
int enqueue(DevState *st, const am_params *p, int64_t N, int32_t M, am_basis b, int32_t dtype,
            char *ws, const Layout &L, hipStream_t stream, int rep = -1, int n_rep = 0,
            const amq::BridgeNode *noalloc_sched = nullptr)
{
    const int fp64 = dtype == AM_FP64;
    Plan plan;
    int rc = choose_plan(st, N, fp64, b.kind == AM_BASIS_LAGUERRE, b.degree, &plan);
    if (rc) return rc;
    const amq::BridgeNode *sched = noalloc_sched;
    if (!sched) {
        rc = get_schedule(st, M, &sched);
        if (rc) return rc;
    }

    amq::GenArgs ga;
    memset(&ga, 0, sizeof ga);
    ga.S = ws + L.off_S;
    ga.V = st->d_V;
    ga.sched = sched;
    ga.datec = (amq::DateConst *)(ws + L.off_datec);
    ga.sync = (uint32_t *)(ws + L.off_result + 64);
    ga.N = N; ga.ld = L.ld;
    ga.nblocks = L.ld / 64;
    ga.M = M;
    const int64_t target_waves = (int64_t)st->num_cu * kGenWavesPerCU;
    int64_t R = (ga.nblocks + target_waves - 1) / target_waves;
    ga.R = (int32_t)(R < 1 ? 1 : R);
    ga.what = 0;
    ga.is_call = p->is_call;
    ga.S0 = p->S0; ga.K = p->K; ga.r = p->r; ga.sigma = p->sigma; ga.T = p->T;
    const double dt = p->T / (double)M;
    ga.mu = (p->r - 0.5 * p->sigma * p->sigma) * dt;
    ga.vol = p->sigma * sqrt(dt);
    ga.shift = rep >= 0 ? (const uint32_t *)(ws + L.off_shift) + (size_t)rep * M : nullptr;
    ga.rows = (uint64_t *)(ws + L.off_part);
    ga.rows_n = amq::rows_words(plan.G, b.degree);
    ProfRec *pr = nullptr;
    if (g_prof.on && !noalloc_sched) {
        int prc = prof_slot(&pr);
        if (prc) return prc;
        HIP_TRY(hipEventRecord(pr->e[0], stream));
    }
    HIP_TRY(amq::launch_generate(ga, fp64, stream));
    if (pr) HIP_TRY(hipEventRecord(pr->e[1], stream));

    amq::SweepArgs sa;
    memset(&sa, 0, sizeof sa);
    sa.S = ws + L.off_S;
    sa.pv_out = ws + L.off_PV;
    sa.rows = (uint64_t *)(ws + L.off_part);
    sa.rec = (double *)(ws + L.off_rec);
    sa.result = (double *)(ws + L.off_result);
    sa.sync = (uint32_t *)(ws + L.off_result + 64);
    sa.err = sa.sync + 2;
    sa.datec = (const amq::DateConst *)(ws + L.off_datec);
    sa.N = N; sa.ld = L.ld;
    sa.M = M; sa.G = plan.G;
    sa.is_call = p->is_call; sa.allow_exercise = p->allow_exercise;
    sa.laguerre = b.kind == AM_BASIS_LAGUERRE; sa.degree = b.degree;
    sa.S0 = p->S0; sa.K = p->K;
    sa.spin_limit = g_spin_limit ? g_spin_limit : kDefaultSpin;
    sa.rep_out = rep >= 0 ? (double *)(ws + L.off_rep) : nullptr;
    sa.rep = rep;
    sa.n_rep = n_rep;
    hipError_t e;
    {
        std::lock_guard<std::mutex> lk(st->persist_mu);
        if (!st->persist_done) {
            if (noalloc_sched) return fail(AM_EINVAL, "am_init has not run on this device");
            HIP_TRY(hipEventCreateWithFlags(&st->persist_done, hipEventDisableTiming));
        } else if (st->persist_stream != stream)
            HIP_TRY(hipStreamWaitEvent(stream, st->persist_done, 0));
        e = amq::launch_sweep(sa, fp64, plan.wg, plan.ppt, stream);
        if (e == hipSuccess) {
            HIP_TRY(hipEventRecord(st->persist_done, stream));
            st->persist_stream = stream;
        }
    }
    if (e != hipSuccess)
        return fail(AM_EDEVICE, "sweep launch (%d threads, ppt %d, groups %d) failed: %s", plan.wg, plan.ppt, plan.G,
                    hipGetErrorString(e));
    if (pr) HIP_TRY(hipEventRecord(pr->e[2], stream));
    return AM_OK;
}

thread_local double *g_pinned = nullptr;
thread_local uint64_t g_pinned_gen = 0;

int fetch_result(char *ws, const Layout &L, hipStream_t stream, double *h_out)
{
    {
        std::lock_guard<std::mutex> lk(g_res_mu);
        if (g_pinned_gen != g_generation) {   // released by am_shutdown
            g_pinned = nullptr;
            g_pinned_gen = g_generation;
        }
    }
    if (!g_pinned) {
        if (hipHostMalloc((void **)&g_pinned, 256, hipHostMallocDefault) != hipSuccess) {
            g_pinned = nullptr;
            return fail(AM_ENOMEM, "hipHostMalloc of the result buffer failed");
        }
        std::lock_guard<std::mutex> lk(g_res_mu);
        g_pinned_all.push_back(g_pinned);
    }
    HIP_TRY(hipMemcpyAsync(g_pinned, ws + L.off_result, 128, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    const uint32_t *sync = (const uint32_t *)((const char *)g_pinned + 64);
    if (sync[2] != 0u) return fail(AM_ETIMEOUT, "a device-side barrier wait ran out (spin limit)");
    if (!isfinite(g_pinned[0]) || !isfinite(g_pinned[1]))
        return fail(AM_EDEVICE, "non-finite result");
    h_out[0] = g_pinned[0];
    h_out[1] = g_pinned[1];
    return AM_OK;
}

}  // namespace

extern "C" {

const char *am_last_error(void) { return g_err.c_str(); }

int am_max_dates(void)
{
    return (int)amq_sobol_v32_dims < amq::kMaxDates ? (int)amq_sobol_v32_dims : amq::kMaxDates;
}

int64_t am_max_paths(int32_t dtype)
{
    DevState *st = nullptr;
    if (get_state(&st)) return 0;
    const int fp64 = dtype == AM_FP64;
    const TileShape *tiles = fp64 ? kTiles64 : kTiles32;
    const int n_tiles = fp64 ? kNTiles64 : kNTiles32;
    int64_t best = 0;
    for (int i = 0; i < n_tiles; ++i) {
        int64_t worst = -1;
        for (int d = 0; d < 2 * (AM_MAX_DEGREE + 1); ++d) {
            int64_t g = (int64_t)groups_per_cu(st, fp64, d & 1, tiles[i].wg, tiles[i].ppt, d >> 1) * st->num_cu;
            if (g > amq::kMaxGroups) g = amq::kMaxGroups;
            const int64_t cap = g * tiles[i].wg * tiles[i].ppt;
            worst = worst < 0 || cap < worst ? cap : worst;
        }
        best = worst > best ? worst : best;
    }
    return best;
}

int32_t am_storage_dtype(int64_t n_paths, int32_t dtype)
{
    if (dtype != AM_FP64 && dtype != AM_FP32_BULK) return -1;
    return storage_of(n_paths, dtype);
}

size_t am_workspace_bytes(int64_t n_paths, int32_t n_dates, am_basis basis, int32_t dtype)
{
    (void)basis;
    if (n_paths < 1 || n_dates < 1) return 0;
    return make_layout(n_paths, n_dates, storage_of(n_paths, dtype)).total;
}

int am_workspace_layout(int64_t n_paths, int32_t n_dates, am_basis basis, int32_t dtype, size_t out[6])
{
    (void)basis;
    if (!out || n_paths < 1 || n_dates < 1 || (dtype != AM_FP64 && dtype != AM_FP32_BULK))
        return fail(AM_EINVAL, "bad arguments to am_workspace_layout");
    Layout L = make_layout(n_paths, n_dates, storage_of(n_paths, dtype));
    out[0] = L.off_S; out[1] = L.off_PV; out[2] = L.off_rec; out[3] = L.off_result;
    out[4] = (size_t)L.ld; out[5] = L.total;
    return AM_OK;
}

int am_price_american_ex(const am_params *params, int64_t n_paths, int32_t n_dates, am_basis basis,
                         int32_t dtype, void *d_workspace, size_t ws_bytes, void *hip_stream,
                         double *h_out)
{
    int rc = validate(params, n_paths, n_dates, basis, dtype);
    if (rc) return rc;
    dtype = storage_of(n_paths, dtype);
    Layout L = make_layout(n_paths, n_dates, dtype);
    if (!d_workspace || ws_bytes < L.total || ((uintptr_t)d_workspace & 255u))
        return fail(AM_EWORKSPACE, "workspace must be >= %zu bytes and 256-byte aligned", L.total);
    DevState *st = nullptr;
    rc = get_state(&st);
    if (rc) return rc;
    hipStream_t stream = (hipStream_t)hip_stream;
    rc = enqueue(st, params, n_paths, n_dates, basis, dtype, (char *)d_workspace, L, stream);
    if (rc) return rc;
    if (!h_out) return AM_OK;
    return fetch_result((char *)d_workspace, L, stream, h_out);
}

int am_price_american(const am_params *params, int64_t n_paths, int32_t n_dates, am_basis basis,
                      int32_t dtype, double *price, double *std_err)
{
    if (!price || !std_err) return fail(AM_EINVAL, "price and std_err must be non-NULL");
    int rc = validate(params, n_paths, n_dates, basis, dtype);
    if (rc) return rc;
    dtype = storage_of(n_paths, dtype);
    DevState *st = nullptr;
    rc = get_state(&st);
    if (rc) return rc;
    Layout L = make_layout(n_paths, n_dates, dtype);
    std::lock_guard<std::mutex> lk(st->sync_mu);
    if (st->ws_bytes < L.total) {
        if (st->ws) { HIP_TRY(hipStreamSynchronize(st->stream)); HIP_TRY(hipFree(st->ws)); }
        st->ws = nullptr;
        st->ws_bytes = 0;
        if (hipMalloc(&st->ws, L.total) != hipSuccess)
            return fail(AM_ENOMEM, "hipMalloc of %zu workspace bytes failed", L.total);
        st->ws_bytes = L.total;
    }
    rc = enqueue(st, params, n_paths, n_dates, basis, dtype, (char *)st->ws, L, st->stream);
    double out[2] = {0.0, 0.0};
    if (!rc) rc = fetch_result((char *)st->ws, L, st->stream, out);
    if (rc) return rc;
    *price = out[0];
    *std_err = out[1];
    return AM_OK;
}

int am_init(void)
{
    DevState *st = nullptr;
    int rc = get_state(&st);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(st->persist_mu);
        if (!st->persist_done)
            HIP_TRY(hipEventCreateWithFlags(&st->persist_done, hipEventDisableTiming));
    }
    {
        std::lock_guard<std::mutex> lk(st->mu);
        if (!st->scratch) {
            void *ptr = nullptr;
            const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr)
                return fail(AM_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
            st->scratch = (char *)ptr;
        }
    }
    // load every single-option kernel's code now: the occupancy queries and
    // attribute reads make the runtime load each module on this device
    HIP_TRY(amq::preload_generate());
    for (int fp64 = 0; fp64 < 2; ++fp64) {
        const TileShape *tiles = fp64 ? kTiles64 : kTiles32;
        const int n_tiles = fp64 ? kNTiles64 : kNTiles32;
        for (int i = 0; i < n_tiles; ++i)
            for (int d = 0; d < 2 * (AM_MAX_DEGREE + 1); ++d)
                (void)groups_per_cu(st, fp64, d & 1, tiles[i].wg, tiles[i].ppt, d >> 1);
    }
    return AM_OK;
}

int am_price_american_noalloc(const am_params *params, int64_t n_paths, int32_t n_dates, am_basis basis,
                              int32_t dtype, void *hip_stream, double *h_out)
{
    if (!h_out) return fail(AM_EINVAL, "h_out must be non-NULL");
    int rc = validate(params, n_paths, n_dates, basis, dtype);
    if (rc) return rc;
    dtype = storage_of(n_paths, dtype);
    const Layout L = make_layout(n_paths, n_dates, dtype);
    // the bridge schedule follows the workspace regions (L.total is 256-aligned)
    const size_t sched_bytes = sizeof(amq::BridgeNode) * (size_t)n_dates;
    const size_t need = L.total + sched_bytes;
    if (need > (size_t)AM_SCRATCH_BYTES)
        return fail(AM_EWORKSPACE, "%lld paths x %d dates need %zu bytes; the allocation-free entry point "
                    "has %zu", (long long)n_paths, n_dates, need, (size_t)AM_SCRATCH_BYTES);
    DevState *st = find_state();
    if (!st || !st->scratch) return fail(AM_EINVAL, "am_init has not run on this device");
    const std::vector<amq::BridgeNode> *hs = nullptr;
    {
        // host copies only (built once per date count, kept for the process)
        std::lock_guard<std::mutex> lk(st->mu);
        auto it = st->host_sched.find(n_dates);
        if (it == st->host_sched.end()) {
            std::vector<amq::BridgeNode> h = make_schedule(n_dates);
            if ((int)h.size() != n_dates || max_slot(h) >= amq::kAnchorSlot)
                return fail(AM_EDIM, "bridge schedule for %d dates does not fit the register window", n_dates);
            it = st->host_sched.emplace(n_dates, std::move(h)).first;
        }
        hs = &it->second;
    }
    hipStream_t stream = (hipStream_t)hip_stream;
    char *ws = st->scratch;
    amq::BridgeNode *d_sched = (amq::BridgeNode *)(ws + L.total);
    HIP_TRY(hipMemcpyAsync(d_sched, hs->data(), sched_bytes, hipMemcpyHostToDevice, stream));
    rc = enqueue(st, params, n_paths, n_dates, basis, dtype, ws, L, stream, -1, 0, d_sched);
    if (rc) return rc;
    // result words and the barrier block's first line, into host stack memory
    double res[16];
    HIP_TRY(hipMemcpyAsync(res, ws + L.off_result, sizeof res, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    const uint32_t *sync = (const uint32_t *)(res + 8);
    if (sync[2] != 0u) return fail(AM_ETIMEOUT, "a device-side barrier wait ran out (spin limit)");
    if (!isfinite(res[0]) || !isfinite(res[1])) return fail(AM_EDEVICE, "non-finite result");
    h_out[0] = res[0];
    h_out[1] = res[1];
    return AM_OK;
}

}  // extern "C"

namespace {

// Randomised QMC, one replicate after another in the single-option layout
// (the replicates' prices collected on the device; the last replicate's
// final step aggregates them).
int rqmc_serial(const am_params *params, int64_t n_paths, int32_t n_dates, am_basis basis,
                int32_t dtype, int32_t n_rep, const uint32_t *h_shifts, void *d_workspace,
                size_t ws_bytes, void *hip_stream, double *h_out)
{
    int rc = AM_OK;
    dtype = storage_of(n_paths, dtype);
    Layout L = make_layout(n_paths, n_dates, dtype);
    if (!d_workspace || ws_bytes < L.total || ((uintptr_t)d_workspace & 255u))
        return fail(AM_EWORKSPACE, "workspace must be >= %zu bytes and 256-byte aligned", L.total);
    DevState *st = nullptr;
    rc = get_state(&st);
    if (rc) return rc;
    char *ws = (char *)d_workspace;
    hipStream_t stream = (hipStream_t)hip_stream;
    HIP_TRY(hipMemcpyAsync(ws + L.off_shift, h_shifts, (size_t)n_rep * n_dates * 4,
                           hipMemcpyHostToDevice, stream));
    for (int r = 0; r < n_rep; ++r) {
        rc = enqueue(st, params, n_paths, n_dates, basis, dtype, ws, L, stream, r, n_rep);
        if (rc) return rc;
    }
    if (!h_out) return AM_OK;
    rc = fetch_result(ws, L, stream, h_out);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(h_out + 2, ws + L.off_rep, (size_t)n_rep * 8, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    return AM_OK;
}

}  // namespace

extern "C" {

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------
struct BatchPlan {
    std::vector<int> order;                       // options by decreasing work
    std::vector<int64_t> ld, offS, offPV;
    std::vector<size_t> offDatec, offRec;
    std::vector<int32_t> G, tile_base;
    size_t off_part = 0, off_res = 0, off_sync = 0, off_gsync = 0, off_desc = 0, off_tiles = 0,
           off_units = 0, total = 0;
    int total_tiles = 0, max_M = 0;
    int64_t total_blocks = 0, max_units = 0;
};

constexpr int64_t kBatchTileAlign = 16384;  // rows padded to a multiple of every batch tile

int batch_plan(const am_option *opts, int32_t n, int32_t dtype, BatchPlan &P)
{
    const size_t s = dtype == AM_FP64 ? 8 : 4;
    P.order.resize(n);
    for (int i = 0; i < n; ++i) P.order[i] = i;
    std::stable_sort(P.order.begin(), P.order.end(), [&](int a, int b) {
        const double wa = (double)opts[a].n_paths * opts[a].n_dates;
        const double wb = (double)opts[b].n_paths * opts[b].n_dates;
        return wa > wb;
    });
    P.ld.assign(n, 0); P.offS.assign(n, 0); P.offPV.assign(n, 0);
    P.offDatec.assign(n, 0); P.offRec.assign(n, 0); P.G.assign(n, 0); P.tile_base.assign(n, 0);
    size_t o = 0;
    int tiles = 0;
    for (int q = 0; q < n; ++q) {
        const int i = P.order[q];
        const int64_t ld = (opts[i].n_paths + kBatchTileAlign - 1) / kBatchTileAlign * kBatchTileAlign;
        P.ld[i] = ld;
        P.offS[i] = (int64_t)o;  o = align256(o + (size_t)opts[i].n_dates * ld * s);
        P.offPV[i] = (int64_t)o; o = align256(o + (size_t)ld * s);
        P.tile_base[i] = tiles;
        P.total_blocks += ld / 64;
        P.max_units += (ld / 64 + amq::kWaves - 1) / amq::kWaves;
        if (opts[i].n_dates > P.max_M) P.max_M = opts[i].n_dates;
    }
    for (int q = 0; q < n; ++q) {
        const int i = P.order[q];
        P.offDatec[i] = o; o = align256(o + (size_t)(opts[i].n_dates + 1) * sizeof(amq::DateConst));
        P.offRec[i] = o;   o = align256(o + (size_t)(opts[i].n_dates + 1) * amq::kRec * 8);
    }
    P.off_res = o;   o = align256(o + (size_t)n * 8 * 8);
    P.off_sync = o;  o = align256(o + (size_t)n * amq::kSyncWords * 4);
    P.off_gsync = o; o = align256(o + 16 * 4);
    P.off_desc = o;  o = align256(o + (size_t)n * sizeof(amq::BatchOpt));
    // tiles: the smallest batch tile (256 paths) bounds the count from above
    int64_t max_tiles = 0;
    for (int i = 0; i < n; ++i) max_tiles += P.ld[i] / 256;
    P.off_tiles = o; o = align256(o + (size_t)max_tiles * 4);
    // partial-sum rows: per option 2 x (tiles + team rows) x row words
    P.off_part = o;  o = align256(o + ((size_t)max_tiles + (size_t)n * amq::kMaxTeams) * 2 * amq::kMaxRowWords * 8);
    P.off_units = o; o = align256(o + (size_t)P.max_units * sizeof(amq::GenUnit));
    P.total = o;
    (void)tiles;
    return AM_OK;
}

// Batch tile autotuning: the best paths-per-thread found by am_batch_autotune
// for a shape class (precision, degree, batch size and total work, both
// rounded to powers of two), used when no explicit choice is set.
std::mutex g_tune_mu;
std::map<long long, int> g_tuned;

long long tune_key(const am_option *opts, int32_t n, am_basis basis, int32_t dtype)
{
    double work = 0.0;
    for (int i = 0; i < n; ++i) work += (double)opts[i].n_paths * opts[i].n_dates;
    const int lw = (int)floor(log2(work > 1.0 ? work : 1.0));
    const int ln = (int)floor(log2((double)n));
    return ((long long)dtype << 40) | ((long long)basis.degree << 32) | ((long long)ln << 16) | lw;
}

bool valid_batch_ppt(int32_t storage, int ppt)
{
    return storage == AM_FP64 ? (ppt == 8 || ppt == 32) : (ppt == 16 || ppt == 64);
}

// The larger tile by default: an option's per-date exchange costs about the
// same whatever its tile count, so fewer, larger tiles amortise it over more
// work (batch of 1024 options, binary32 storage: 39.5 ms at 16 paths per
// thread, 20.6 at 32, 19.0 at 64; binary64: 56.5 at 8, 34.1 at 16, 28.3 at
// 32).
int default_batch_ppt(int32_t storage) { return storage == AM_FP64 ? 32 : 64; }
int small_batch_ppt(int32_t storage) { return storage == AM_FP64 ? 8 : 16; }

// The tile for a batch whose options are all the caller's (the replicates of
// one randomised-QMC price): the larger one while the batch still yields a
// tile per compute unit at that size, else the smaller one, so that few
// paths still spread over the device (8 replicates of 2^17 paths in
// binary32: 64 tiles at 64 paths per thread, 2.14 ms; 256 tiles at 16,
// 1.46 ms) -- unless an option would then need more tiles than the device
// holds resident.
int shaped_batch_ppt(const am_option *opts, int32_t n, am_basis basis, int32_t storage, int num_cu)
{
    const int64_t big = (int64_t)amq::kWG * default_batch_ppt(storage);
    const int64_t small = (int64_t)amq::kWG * small_batch_ppt(storage);
    int64_t tiles = 0, most = 0;
    for (int i = 0; i < n; ++i) {
        tiles += (opts[i].n_paths + big - 1) / big;
        const int64_t t = (opts[i].n_paths + small - 1) / small;
        most = t > most ? t : most;
    }
    const int per_cu = amq::sweep_batch_blocks_per_cu(storage == AM_FP64, basis.kind == AM_BASIS_LAGUERRE,
                                                      small_batch_ppt(storage), basis.degree);
    const bool fits = per_cu > 0 && most <= (int64_t)per_cu * num_cu;
    return (tiles >= num_cu || !fits) ? default_batch_ppt(storage) : small_batch_ppt(storage);
}

// Paths per thread of the sub-batch stored as `storage` in a batch the caller
// priced as `dtype`: the tuning hook if it names a tile of this storage
// type, else the tile am_batch_autotune found for the batch's shape class
// (it tunes the caller's storage type), else the default.  The default does
// not depend on the rest of the batch, so an option prices the same alone
// and in any mix.
int batch_ppt(const am_option *opts, int32_t n, am_basis basis, int32_t dtype, int32_t storage)
{
    if (g_batch_ppt && valid_batch_ppt(storage, g_batch_ppt)) return g_batch_ppt;
    if (storage == dtype) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(tune_key(opts, n, basis, dtype));
        if (it != g_tuned.end() && valid_batch_ppt(storage, it->second)) return it->second;
    }
    return default_batch_ppt(storage);
}

// A batch as priced: under AM_FP32_BULK the options below AM_FP32_MIN_PATHS
// paths form a second sub-batch stored in binary64 (part 1); part 0 holds
// the rest in the caller's storage type.  Each part has its own plan and
// workspace region.
struct SplitBatch {
    int32_t storage[2] = {AM_FP32_BULK, AM_FP64};
    std::vector<am_option> opts[2];
    std::vector<int> idx[2];   // caller's index of each option of the part
    BatchPlan P[2];
    size_t off[2] = {0, 0};
    size_t total = 0;
    int n(int h) const { return (int)opts[h].size(); }
};

void split_batch(const am_option *opts, int32_t n, int32_t dtype, SplitBatch &B)
{
    B.storage[0] = dtype;
    for (int i = 0; i < n; ++i) {
        const int h = (dtype == AM_FP32_BULK && storage_of(opts[i].n_paths, dtype) == AM_FP64) ? 1 : 0;
        B.opts[h].push_back(opts[i]);
        B.idx[h].push_back(i);
    }
    size_t o = 0;
    for (int h = 0; h < 2; ++h) {
        if (B.opts[h].empty()) continue;
        batch_plan(B.opts[h].data(), B.n(h), B.storage[h], B.P[h]);
        B.off[h] = o;
        o = align256(o + B.P[h].total);
    }
    B.total = o;
}

int validate_batch(const am_option *opts, int32_t n, am_basis basis, int32_t dtype)
{
    if (!opts || n < 1) return fail(AM_EINVAL, "need at least one option");
    for (int i = 0; i < n; ++i) {
        int rc = validate(&opts[i].params, opts[i].n_paths, opts[i].n_dates, basis, dtype);
        if (rc) return fail(rc, "option %d: %s", i, g_err.c_str());
    }
    return AM_OK;
}

int am_price_paper_estimator(const am_params *params, int64_t n_paths, int32_t n_points,
                             int32_t dtype, void *d_workspace, size_t ws_bytes, void *hip_stream,
                             double *h_out)
{
    am_basis b0 = {AM_BASIS_MONOMIAL, 0};
    int rc = validate(params, n_paths, n_points, b0, dtype);
    if (rc) return rc;
    Layout L = make_layout(n_paths, n_points, dtype);
    if (!d_workspace || ws_bytes < L.total || ((uintptr_t)d_workspace & 255u))
        return fail(AM_EWORKSPACE, "workspace must be >= %zu bytes and 256-byte aligned", L.total);
    DevState *st = nullptr;
    rc = get_state(&st);
    if (rc) return rc;
    const amq::BridgeNode *sched = nullptr;
    rc = get_schedule(st, n_points, &sched);
    if (rc) return rc;
    char *ws = (char *)d_workspace;
    hipStream_t stream = (hipStream_t)hip_stream;
    const int fp64 = dtype == AM_FP64;
    const double dt = params->T / (double)(n_points + 1);
    amq::GenArgs ga;
    memset(&ga, 0, sizeof ga);
    ga.S = ws + L.off_S;
    ga.V = st->d_V;
    ga.sched = sched;
    ga.datec = (amq::DateConst *)(ws + L.off_datec);
    ga.sync = (uint32_t *)(ws + L.off_result + 64);
    ga.N = n_paths; ga.ld = L.ld; ga.nblocks = L.ld / 64; ga.M = n_points;
    const int64_t target_waves = (int64_t)st->num_cu * kGenWavesPerCU;
    int64_t R = (ga.nblocks + target_waves - 1) / target_waves;
    ga.R = (int32_t)(R < 1 ? 1 : R);
    ga.what = 0;
    ga.is_call = params->is_call;
    ga.S0 = params->S0; ga.K = params->K; ga.r = params->r; ga.sigma = params->sigma;
    ga.T = dt * (double)n_points;                       // horizon t_m = m dt
    ga.mu = (params->r - 0.5 * params->sigma * params->sigma) * dt;
    ga.vol = params->sigma * sqrt(dt);
    HIP_TRY(amq::launch_generate(ga, fp64, stream));
    amq::PaperArgs pa;
    memset(&pa, 0, sizeof pa);
    pa.S = ws + L.off_S;
    pa.part = (double *)(ws + L.off_part);
    pa.ticket = (uint32_t *)(ws + L.off_result + 64) + 4;
    pa.result = (double *)(ws + L.off_result);
    pa.N = n_paths; pa.ld = L.ld; pa.m = n_points; pa.is_call = params->is_call;
    pa.K = params->K; pa.r = params->r; pa.sigma = params->sigma; pa.dt = dt; pa.S0 = params->S0;
    HIP_TRY(amq::launch_paper(pa, fp64, stream));
    if (!h_out) return AM_OK;
    return fetch_result(ws, L, stream, h_out);
}

size_t am_batch_workspace_bytes(const am_option *opts, int32_t n_opts, am_basis basis, int32_t dtype)
{
    if (validate_batch(opts, n_opts, basis, dtype)) return 0;
    SplitBatch B;
    split_batch(opts, n_opts, dtype, B);
    return B.total;
}

}  // extern "C"

namespace {

// Enqueue one batch (generation + persistent sweep) on `stream`.  grid_cap
// bounds the persistent grid (a fraction of the device when several batches
// run side by side); cooperative selects hipLaunchCooperativeKernel.
// staging (optional, pinned, staging_bytes) holds the uploaded tables.
// shifts (nullable): per option, the device address of its digital shift
// ([n_dates] words; randomised QMC); all options of the batch or none.
int enqueue_batch(DevState *st, const am_option *opts, int32_t n_opts, am_basis basis, int32_t dtype,
                  char *ws, const BatchPlan &P, hipStream_t stream, int grid_cap, bool cooperative,
                  char *staging, size_t staging_bytes, int ppt, const uint32_t *const *shifts = nullptr)
{
    int rc = AM_OK;
    const int fp64 = dtype == AM_FP64;
    const int64_t tile = (int64_t)amq::kWG * ppt;
    if (kBatchTileAlign % tile != 0) return fail(AM_EINVAL, "batch tile %lld does not divide the row padding", (long long)tile);
    const int per_cu = amq::sweep_batch_blocks_per_cu(fp64, basis.kind == AM_BASIS_LAGUERRE, ppt, basis.degree);
    if (per_cu <= 0) return fail(AM_EDEVICE, "no batch sweep kernel for ppt %d degree %d", ppt, basis.degree);
    int capacity = per_cu * st->num_cu;
    if (grid_cap > 0 && grid_cap < capacity) capacity = grid_cap;

    std::vector<amq::BatchOpt> desc(n_opts);
    std::vector<int32_t> tile_opt;
    int max_G = 0;
    int tiles = 0;
    size_t rows_off = 0;
    for (int q = 0; q < n_opts; ++q) {
        const int i = P.order[q];
        const am_option &op = opts[i];
        const amq::BridgeNode *sched = nullptr;
        rc = get_schedule(st, op.n_dates, &sched);
        if (rc) return rc;
        amq::BatchOpt &d = desc[i];
        memset(&d, 0, sizeof d);
        d.S = ws + P.offS[i];
        d.pv = ws + P.offPV[i];
        d.sched = sched;
        d.datec = (amq::DateConst *)(ws + P.offDatec[i]);
        d.rec = (double *)(ws + P.offRec[i]);
        d.result = (double *)(ws + P.off_res) + (size_t)i * 8;
        d.sync = (uint32_t *)(ws + P.off_sync) + (size_t)i * amq::kSyncWords;
        d.N = op.n_paths;
        d.ld = P.ld[i];
        d.M = op.n_dates;
        d.G = (int32_t)((op.n_paths + tile - 1) / tile);
        d.tile_base = tiles;
        d.rows = (uint64_t *)(ws + P.off_part) + rows_off;
        d.rows_n = amq::rows_words(d.G, basis.degree);
        rows_off += (size_t)d.rows_n;
        d.is_call = op.params.is_call;
        d.allow_exercise = op.params.allow_exercise;
        d.S0 = op.params.S0; d.K = op.params.K; d.r = op.params.r; d.sigma = op.params.sigma;
        d.T = op.params.T;
        const double dt = op.params.T / (double)op.n_dates;
        d.mu = (op.params.r - 0.5 * op.params.sigma * op.params.sigma) * dt;
        d.vol = op.params.sigma * sqrt(dt);
        d.shift = shifts ? shifts[i] : nullptr;
        for (int g = 0; g < d.G; ++g) tile_opt.push_back(i);
        tiles += d.G;
        if (d.G > max_G) max_G = d.G;
    }
    const int grid = tiles < capacity ? tiles : capacity;
    if (max_G > grid)
        return fail(AM_EDIM, "an option needs %d tiles but only %d workgroups are resident", max_G, grid);
    // generation units: about kBatchGenWavesPerCU waves per CU in total, each
    // wave given about the same number of path-steps (blocks x dates), so
    // options with many dates get fewer blocks per wave and no unit outlasts
    // the rest
    const int64_t target_waves = (int64_t)st->num_cu * kBatchGenWavesPerCU;
    int64_t total_work = 0;
    for (int i = 0; i < n_opts; ++i) total_work += (P.ld[i] / 64) * (int64_t)opts[i].n_dates;
    const int64_t wave_work = (total_work + target_waves - 1) / target_waves;
    std::vector<amq::GenUnit> units;
    for (int q = 0; q < n_opts; ++q) {
        const int i = P.order[q];
        const int64_t nb = P.ld[i] / 64;
        int64_t R = (wave_work + opts[i].n_dates / 2) / opts[i].n_dates;
        if (R < 1) R = 1;
        for (int64_t b = 0; b < nb; b += amq::kWaves * R) {
            amq::GenUnit u;
            u.opt = i; u.pad = 0; u.b0 = b; u.b1 = b + amq::kWaves * R < nb ? b + amq::kWaves * R : nb;
            units.push_back(u);
        }
    }
    if ((int64_t)units.size() > P.max_units) return fail(AM_EDEVICE, "unit table overflow");
    const size_t bd = desc.size() * sizeof(amq::BatchOpt), bt = tile_opt.size() * 4,
                 bu = units.size() * sizeof(amq::GenUnit);
    const void *src_d = desc.data(), *src_t = tile_opt.data(), *src_u = units.data();
    if (staging && align256(bd) + align256(bt) + bu <= staging_bytes) {
        memcpy(staging, desc.data(), bd);
        memcpy(staging + align256(bd), tile_opt.data(), bt);
        memcpy(staging + align256(bd) + align256(bt), units.data(), bu);
        src_d = staging;
        src_t = staging + align256(bd);
        src_u = staging + align256(bd) + align256(bt);
    }
    HIP_TRY(hipMemcpyAsync(ws + P.off_desc, src_d, bd, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(ws + P.off_tiles, src_t, bt, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(ws + P.off_units, src_u, bu, hipMemcpyHostToDevice, stream));
    uint32_t *gsync = (uint32_t *)(ws + P.off_gsync);
    ProfRec *pr = nullptr;
    if (g_prof.on) {
        rc = prof_slot(&pr);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(pr->e[0], stream));
    }
    HIP_TRY(amq::launch_generate_batch((const amq::BatchOpt *)(ws + P.off_desc),
                                       (const amq::GenUnit *)(ws + P.off_units), (int)units.size(),
                                       st->d_V, gsync, P.max_M, fp64, shifts != nullptr, stream));
    if (pr) HIP_TRY(hipEventRecord(pr->e[1], stream));
    amq::BatchGlobal g;
    memset(&g, 0, sizeof g);
    g.claim = gsync;
    g.err = gsync + 1;
    g.total_tiles = tiles;
    g.laguerre = basis.kind == AM_BASIS_LAGUERRE;
    g.spin_limit = g_spin_limit ? g_spin_limit : kDefaultSpin;
    hipError_t e = amq::launch_sweep_batch((const amq::BatchOpt *)(ws + P.off_desc),
                                           (const int32_t *)(ws + P.off_tiles), g, grid, fp64, ppt,
                                           basis.degree, cooperative, stream);
    if (e != hipSuccess)
        return fail(AM_EDEVICE, "batch sweep launch (grid %d, ppt %d) failed: %s", grid, ppt, hipGetErrorString(e));
    if (pr) HIP_TRY(hipEventRecord(pr->e[2], stream));
    return AM_OK;
}

// Bytes of pinned staging one part's tables need (descriptors, tile table,
// generation units).
size_t staging_bytes_for(const BatchPlan &P, int n)
{
    return align256((size_t)n * sizeof(amq::BatchOpt)) + align256((size_t)P.total_blocks * 4) +
           (size_t)P.max_units * sizeof(amq::GenUnit) + 256;
}

// Enqueue both parts of a split batch on `stream` (part 0 first).  ppt[h]:
// tile of part h (0: batch_ppt's choice); grid_cap[h]: cap on part h's
// persistent grid (0: the device's resident capacity); staging (optional,
// pinned) holds both parts' tables, part 1's after part 0's.
// shifts (nullable): per caller option, the device address of its digital
// shift (see enqueue_batch).
int enqueue_split(DevState *st, const SplitBatch &B, am_basis basis, int32_t dtype, char *ws,
                  hipStream_t stream, const int *grid_cap, bool cooperative, char *staging,
                  size_t staging_bytes, const int *ppt_in, const uint32_t *const *shifts = nullptr)
{
    size_t so = 0;
    for (int h = 0; h < 2; ++h) {
        if (!B.n(h)) continue;
        std::vector<const uint32_t *> part_shifts;
        if (shifts)
            for (int j = 0; j < B.n(h); ++j) part_shifts.push_back(shifts[B.idx[h][j]]);
        const int ppt = ppt_in && ppt_in[h] ? ppt_in[h]
                                            : batch_ppt(B.opts[h].data(), B.n(h), basis, dtype, B.storage[h]);
        const size_t need = staging_bytes_for(B.P[h], B.n(h));
        char *stg = staging && so + need <= staging_bytes ? staging + so : nullptr;
        int rc = enqueue_batch(st, B.opts[h].data(), B.n(h), basis, B.storage[h], ws + B.off[h], B.P[h], stream,
                               grid_cap ? grid_cap[h] : 0, cooperative, stg, stg ? need : 0, ppt,
                               shifts ? part_shifts.data() : nullptr);
        if (rc) return rc;
        so += align256(need);
    }
    return AM_OK;
}

// Enqueue the device-to-host copies of both parts' results into h_res:
// part 0's [n0][8] doubles and its 8-double sync block, then part 1's.
int enqueue_split_results(const SplitBatch &B, char *ws, double *h_res, hipStream_t stream)
{
    size_t o = 0;
    for (int h = 0; h < 2; ++h) {
        if (!B.n(h)) continue;
        char *w = ws + B.off[h];
        HIP_TRY(hipMemcpyAsync(h_res + o, w + B.P[h].off_res, (size_t)B.n(h) * 64, hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipMemcpyAsync(h_res + o + (size_t)B.n(h) * 8, w + B.P[h].off_gsync, 64, hipMemcpyDeviceToHost,
                               stream));
        o += (size_t)B.n(h) * 8 + 8;
    }
    return AM_OK;
}

// Doubles enqueue_split_results writes.
size_t split_results_doubles(const SplitBatch &B)
{
    size_t o = 0;
    for (int h = 0; h < 2; ++h)
        if (B.n(h)) o += (size_t)B.n(h) * 8 + 8;
    return o;
}

// Read results written by enqueue_split_results back into the caller's order
// (price, std_err per option).  Returns AM_ETIMEOUT if a part's bounded
// wait ran out.
int scatter_split_results(const SplitBatch &B, const double *h_res, double *h_out, int32_t *status)
{
    size_t o = 0;
    int rc = AM_OK;
    for (int h = 0; h < 2; ++h) {
        if (!B.n(h)) continue;
        const uint32_t *gs = (const uint32_t *)(h_res + o + (size_t)B.n(h) * 8);
        const bool timed_out = gs[1] != 0u;
        if (timed_out) rc = fail(AM_ETIMEOUT, "a device-side barrier wait ran out (spin limit)");
        for (int j = 0; j < B.n(h); ++j) {
            const int i = B.idx[h][j];
            const double pr = h_res[o + (size_t)j * 8], se = h_res[o + (size_t)j * 8 + 1];
            if (h_out) { h_out[2 * i] = pr; h_out[2 * i + 1] = se; }
            if (status) status[i] = timed_out ? AM_ETIMEOUT : (isfinite(pr) ? AM_OK : AM_EDEVICE);
            if (!timed_out && !isfinite(pr) && rc == AM_OK) rc = fail(AM_EDEVICE, "option %d: non-finite result", i);
        }
        o += (size_t)B.n(h) * 8 + 8;
    }
    return rc;
}

}  // namespace

extern "C" {

int am_price_batch(const am_option *opts, int32_t n_opts, am_basis basis, int32_t dtype,
                   void *d_workspace, size_t ws_bytes, void *hip_stream, double *h_out)
{
    int rc = validate_batch(opts, n_opts, basis, dtype);
    if (rc) return rc;
    SplitBatch B;
    split_batch(opts, n_opts, dtype, B);
    if (!d_workspace || ws_bytes < B.total || ((uintptr_t)d_workspace & 255u))
        return fail(AM_EWORKSPACE, "batch workspace must be >= %zu bytes and 256-byte aligned", B.total);
    DevState *st = nullptr;
    rc = get_state(&st);
    if (rc) return rc;
    char *ws = (char *)d_workspace;
    hipStream_t stream = (hipStream_t)hip_stream;
    rc = enqueue_split(st, B, basis, dtype, ws, stream, nullptr, true, nullptr, 0, nullptr);
    if (rc) return rc;
    if (!h_out) return AM_OK;
    std::vector<double> res(split_results_doubles(B));
    rc = enqueue_split_results(B, ws, res.data(), stream);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(stream));
    return scatter_split_results(B, res.data(), h_out, nullptr);
}

}  // extern "C"

namespace {

// The replicates of a randomised QMC call as a batch of identical options,
// each with its own digital shift.
void rqmc_options(const am_params *params, int64_t n_paths, int32_t n_dates, int32_t n_rep,
                  std::vector<am_option> &opts)
{
    am_option o;
    memset(&o, 0, sizeof o);
    o.params = *params;
    o.n_paths = n_paths;
    o.n_dates = n_dates;
    opts.assign(n_rep, o);
}

int check_rqmc(const am_params *params, int64_t n_paths, int32_t n_dates, am_basis basis, int32_t dtype,
               int32_t n_rep, const uint32_t *h_shifts)
{
    int rc = validate(params, n_paths, n_dates, basis, dtype);
    if (rc) return rc;
    if (n_rep < 1 || n_rep > amq::kMaxReps || !h_shifts)
        return fail(AM_EINVAL, "n_rep must be in [1, %d] and shifts non-NULL", amq::kMaxReps);
    return AM_OK;
}

}  // namespace

extern "C" {

size_t am_rqmc_workspace_bytes(int64_t n_paths, int32_t n_dates, am_basis basis, int32_t dtype, int32_t n_rep)
{
    if (n_rep < 1 || n_rep > amq::kMaxReps) return 0;
    std::vector<am_option> opts;
    am_params p = {100.0, 100.0, 0.0, 0.2, 1.0, 0, 1};   // sizes do not depend on the option
    rqmc_options(&p, n_paths, n_dates, n_rep, opts);
    if (validate_batch(opts.data(), n_rep, basis, dtype)) return 0;
    SplitBatch B;
    split_batch(opts.data(), n_rep, dtype, B);
    return B.total + align256((size_t)n_rep * n_dates * 4);
}

int am_price_american_rqmc(const am_params *params, int64_t n_paths, int32_t n_dates, am_basis basis,
                           int32_t dtype, int32_t n_rep, const uint32_t *h_shifts, void *d_workspace,
                           size_t ws_bytes, void *hip_stream, double *h_out)
{
    int rc = check_rqmc(params, n_paths, n_dates, basis, dtype, n_rep, h_shifts);
    if (rc) return rc;
    return rqmc_serial(params, n_paths, n_dates, basis, dtype, n_rep, h_shifts, d_workspace, ws_bytes,
                       hip_stream, h_out);
}

int am_price_rqmc_batch(const am_params *params, int64_t n_paths, int32_t n_dates, am_basis basis,
                        int32_t dtype, int32_t n_rep, const uint32_t *h_shifts, void *d_workspace,
                        size_t ws_bytes, void *hip_stream, double *h_out)
{
    int rc = check_rqmc(params, n_paths, n_dates, basis, dtype, n_rep, h_shifts);
    if (rc) return rc;
    if (!h_out) return fail(AM_EINVAL, "h_out is required (the mean is formed on the host)");
    const size_t need = am_rqmc_workspace_bytes(n_paths, n_dates, basis, dtype, n_rep);
    if (!d_workspace || ws_bytes < need || ((uintptr_t)d_workspace & 255u))
        return fail(AM_EWORKSPACE, "workspace must be >= %zu bytes and 256-byte aligned", need);
    // every replicate at once: one generation launch and one persistent sweep
    std::vector<am_option> opts;
    rqmc_options(params, n_paths, n_dates, n_rep, opts);
    SplitBatch B;
    split_batch(opts.data(), n_rep, dtype, B);
    DevState *st = nullptr;
    rc = get_state(&st);
    if (rc) return rc;
    char *ws = (char *)d_workspace;
    hipStream_t stream = (hipStream_t)hip_stream;
    const uint32_t *d_sh = (const uint32_t *)(ws + B.total);
    std::vector<const uint32_t *> shifts(n_rep);
    for (int r = 0; r < n_rep; ++r) shifts[r] = d_sh + (size_t)r * n_dates;
    HIP_TRY(hipMemcpyAsync(ws + B.total, h_shifts, (size_t)n_rep * n_dates * 4, hipMemcpyHostToDevice, stream));
    int ppt[2] = {0, 0};
    for (int h = 0; h < 2; ++h)
        if (B.n(h) && !(g_batch_ppt && valid_batch_ppt(B.storage[h], g_batch_ppt)))
            ppt[h] = shaped_batch_ppt(B.opts[h].data(), B.n(h), basis, B.storage[h], st->num_cu);
    rc = enqueue_split(st, B, basis, dtype, ws, stream, nullptr, true, nullptr, 0, ppt, shifts.data());
    if (rc) return rc;
    std::vector<double> res(split_results_doubles(B)), pr(2 * (size_t)n_rep);
    rc = enqueue_split_results(B, ws, res.data(), stream);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(stream));
    rc = scatter_split_results(B, res.data(), pr.data(), nullptr);
    if (rc) return rc;
    // mean and replicate standard error, in the order and arithmetic of the
    // one-after-another form's final step
    double s1r = 0.0;
    for (int q = 0; q < n_rep; ++q) s1r += pr[2 * q];
    const double m = s1r / (double)n_rep;
    double s2r = 0.0;
    for (int q = 0; q < n_rep; ++q) s2r += (pr[2 * q] - m) * (pr[2 * q] - m);
    h_out[0] = m;
    h_out[1] = n_rep > 1 ? sqrt(s2r / (double)(n_rep - 1) / (double)n_rep) : 0.0;
    for (int q = 0; q < n_rep; ++q) h_out[2 + q] = pr[2 * q];
    return AM_OK;
}

void am_debug_set_batch_ppt(int32_t ppt) { g_batch_ppt = ppt; }

void am_debug_set_sweep_wide(int32_t allow) { g_sweep_wide = allow ? 1 : 0; }

void am_debug_set_sweep_tile(int32_t wg, int32_t ppt)
{
    g_tile_wg = wg > 0 ? wg : 0;
    g_tile_ppt = wg > 0 ? ppt : 0;
}

int am_batch_autotune(const am_option *opts, int32_t n_opts, am_basis basis, int32_t dtype,
                      void *d_workspace, size_t ws_bytes, void *hip_stream, int32_t *best_ppt,
                      double ms_out[2])
{
    int rc = validate_batch(opts, n_opts, basis, dtype);
    if (rc) return rc;
    SplitBatch B;
    split_batch(opts, n_opts, dtype, B);
    if (!d_workspace || ws_bytes < B.total || ((uintptr_t)d_workspace & 255u))
        return fail(AM_EWORKSPACE, "batch workspace must be >= %zu bytes and 256-byte aligned", B.total);
    DevState *st = nullptr;
    rc = get_state(&st);
    if (rc) return rc;
    hipStream_t stream = (hipStream_t)hip_stream;
    const int cands[2] = {dtype == AM_FP64 ? 8 : 16, dtype == AM_FP64 ? 32 : 64};
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const int32_t saved = g_batch_ppt;
    double best = 1e300;
    int best_c = cands[1];
    for (int c = 0; c < 2; ++c) {
        g_batch_ppt = cands[c];
        double ms = 0.0;
        for (int rep = 0; rep < 3 && rc == AM_OK; ++rep) {    // first run warms up
            if (hipEventRecord(e0, stream) != hipSuccess) rc = AM_EDEVICE;
            if (!rc) rc = enqueue_split(st, B, basis, dtype, (char *)d_workspace, stream, nullptr, true, nullptr,
                                        0, nullptr);
            if (!rc && hipEventRecord(e1, stream) != hipSuccess) rc = AM_EDEVICE;
            if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = AM_EDEVICE;
            float t = 0.f;
            if (!rc && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = AM_EDEVICE;
            if (rep > 0) ms += t;
        }
        if (rc) break;
        ms /= 2.0;
        if (ms_out) ms_out[c] = ms;
        if (ms < best) { best = ms; best_c = cands[c]; }
    }
    g_batch_ppt = saved;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc == AM_EDEVICE ? fail(AM_EDEVICE, "autotune run failed: %s", g_err.c_str()) : rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[tune_key(opts, n_opts, basis, dtype)] = best_c;
    }
    if (best_ppt) *best_ppt = best_c;
    return AM_OK;
}

}  // extern "C"

// A batch captured once as a HIP graph and replayed: table uploads from
// pinned staging, generation, the persistent sweep (normal launch, grid
// within the resident capacity) and the result download.
struct am_batch_graph {
    std::unique_ptr<SplitBatch> split;   // the parts captured and their result layout
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
    char *staging = nullptr;
    double *h_res = nullptr;
    int32_t n = 0;
};

extern "C" {

int am_batch_graph_create(const am_option *opts, int32_t n_opts, am_basis basis, int32_t dtype,
                          void *d_workspace, size_t ws_bytes, am_batch_graph **out)
{
    if (!out) return fail(AM_EINVAL, "out is NULL");
    int rc = validate_batch(opts, n_opts, basis, dtype);
    if (rc) return rc;
    SplitBatch B;
    split_batch(opts, n_opts, dtype, B);
    if (!d_workspace || ws_bytes < B.total || ((uintptr_t)d_workspace & 255u))
        return fail(AM_EWORKSPACE, "batch workspace must be >= %zu bytes and 256-byte aligned", B.total);
    DevState *st = nullptr;
    rc = get_state(&st);
    if (rc) return rc;
    for (int i = 0; i < n_opts; ++i) {   // schedules are allocated outside the capture
        const amq::BridgeNode *sc = nullptr;
        rc = get_schedule(st, opts[i].n_dates, &sc);
        if (rc) return rc;
    }
    std::unique_ptr<am_batch_graph> g(new am_batch_graph);
    g->n = n_opts;
    g->split.reset(new SplitBatch(B));
    size_t stage = 0;
    for (int h = 0; h < 2; ++h)
        if (B.n(h)) stage += align256(staging_bytes_for(B.P[h], B.n(h)));
    if (hipHostMalloc((void **)&g->staging, stage, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&g->h_res, split_results_doubles(B) * 8, hipHostMallocDefault) != hipSuccess)
        return fail(AM_ENOMEM, "pinned buffers for the batch graph failed");
    HIP_TRY(hipEventCreateWithFlags(&g->done, hipEventDisableTiming));
    hipStream_t cs;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    char *ws = (char *)d_workspace;
    rc = enqueue_split(st, B, basis, dtype, ws, cs, nullptr, false, g->staging, stage, nullptr);
    if (rc == AM_OK && enqueue_split_results(B, ws, g->h_res, cs) != AM_OK)
        rc = fail(AM_EDEVICE, "result download could not be captured");
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &graph);
    (void)hipStreamDestroy(cs);
    if (rc) { if (graph) (void)hipGraphDestroy(graph); return rc; }
    if (e != hipSuccess) return fail(AM_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    g->graph = graph;
    HIP_TRY(hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0));
    *out = g.release();
    return AM_OK;
}

int am_batch_graph_launch(am_batch_graph *g, void *hip_stream)
{
    if (!g) return fail(AM_EINVAL, "graph is NULL");
    hipStream_t s = (hipStream_t)hip_stream;
    HIP_TRY(hipGraphLaunch(g->exec, s));
    HIP_TRY(hipEventRecord(g->done, s));
    return AM_OK;
}

int am_batch_graph_results(am_batch_graph *g, double *h_out)
{
    if (!g || !h_out) return fail(AM_EINVAL, "graph and h_out must be non-NULL");
    HIP_TRY(hipEventSynchronize(g->done));
    return scatter_split_results(*g->split, g->h_res, h_out, nullptr);
}

int am_batch_graph_destroy(am_batch_graph *g)
{
    if (!g) return AM_OK;
    if (g->done) (void)hipEventSynchronize(g->done);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->done) (void)hipEventDestroy(g->done);
    if (g->staging) (void)hipHostFree(g->staging);
    if (g->h_res) (void)hipHostFree(g->h_res);
    delete g;
    return AM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Serving: continuous batching under an HBM budget.
// ---------------------------------------------------------------------------
namespace {

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over one device pool (offsets in bytes, 256-aligned).
struct PoolAlloc {
    std::map<size_t, size_t> free_;   // offset -> length
    size_t used = 0;
    void init(size_t bytes) { free_.clear(); free_[0] = bytes; used = 0; }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = align256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t noff = it->first + bytes;
                free_.erase(it);
                if (rest) free_[noff] = rest;
                used += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align256(bytes);
        used -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Request {
    am_option opt;
    uint64_t id;
    double t_arrival;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    char *staging = nullptr;          // pinned: uploaded tables
    double *h_res = nullptr;          // pinned: per part [n][8] results + 8 sync doubles
    size_t staging_bytes = 0;
    bool busy = false;
    bool exclusive = false;           // runs alone on the whole device
    std::vector<Request> reqs;
    SplitBatch split;                 // the launched parts (result layout)
    size_t off = 0, bytes = 0;
    double t_launch = 0.0;
};

}  // namespace

struct am_server {
    am_server_config cfg;
    DevState *st = nullptr;
    char *pool = nullptr;
    PoolAlloc alloc;
    std::vector<Slot> slots;
    int grid_cap[2] = {0, 0};         // per part: 1/n_streams of the resident capacity
    int full_cap[2] = {0, 0};         // per part: the whole device's resident capacity
    int ppt[2] = {0, 0};              // per part: batch tile (paths per thread)
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request> pending;
    std::vector<am_result> done;
    std::thread th;
    bool stop = false;
    int fatal = AM_OK;
    std::string fatal_msg;
    uint64_t n_batches = 0, n_requests = 0;
    double busy_path_steps = 0.0;
};

namespace {

void finish_slot(am_server *sv, Slot &sl, std::vector<am_result> &out)
{
    const double t = now_s();
    std::vector<double> price(sl.reqs.size() * 2, 0.0);
    std::vector<int32_t> status(sl.reqs.size(), AM_OK);
    (void)scatter_split_results(sl.split, sl.h_res, price.data(), status.data());
    for (size_t i = 0; i < sl.reqs.size(); ++i) {
        am_result r;
        memset(&r, 0, sizeof r);
        r.request_id = sl.reqs[i].id;
        r.price = price[2 * i];
        r.std_err = price[2 * i + 1];
        r.status = status[i];
        r.t_arrival = sl.reqs[i].t_arrival;
        r.t_launch = sl.t_launch;
        r.t_done = t;
        out.push_back(r);
    }
    sv->alloc.release(sl.off, sl.bytes);
    sl.reqs.clear();
    sl.split = SplitBatch();
    sl.busy = false;
    sl.exclusive = false;
}

void refuse(const Request &q, int32_t status, std::vector<am_result> &out)
{
    am_result r;
    memset(&r, 0, sizeof r);
    r.request_id = q.id;
    r.status = status;
    r.t_arrival = q.t_arrival;
    r.t_done = now_s();
    out.push_back(r);
}

// Sweep tiles one served request needs (the server's fixed tile per part).
int64_t request_tiles(const am_server *sv, const am_option &o, int *part)
{
    const int h = (sv->cfg.dtype == AM_FP32_BULK && storage_of(o.n_paths, sv->cfg.dtype) == AM_FP64) ? 1 : 0;
    if (part) *part = h;
    const int64_t tile = (int64_t)amq::kWG * sv->ppt[h];
    return (o.n_paths + tile - 1) / tile;
}

// Launch the longest admissible prefix of the pending queue on slot `sl`.
// A request whose sweep needs more groups than a stream's share of the
// device goes alone, on the whole device, once every slot is idle; nothing
// launches while it runs.  Returns true if something was launched.
bool launch_some(am_server *sv, Slot &sl, std::deque<Request> &pend, std::vector<am_result> &out)
{
    const am_server_config &c = sv->cfg;
    bool any_busy = false;
    for (auto &o : sv->slots) {
        if (o.busy && o.exclusive) return false;
        any_busy = any_busy || o.busy;
    }
    std::vector<am_option> opts;
    std::vector<Request> take;
    double work = 0.0;
    bool exclusive = false;
    for (size_t i = 0; i < pend.size() && (int)take.size() < c.max_batch_requests; ++i) {
        int h = 0;
        const bool big = request_tiles(sv, pend[i].opt, &h) > sv->grid_cap[h];
        if (big) {
            if (!take.empty()) break;          // the prefix stops before it
            if (any_busy) return false;        // waits for the device to drain
            exclusive = true;
        }
        const double w = (double)pend[i].opt.n_paths * pend[i].opt.n_dates;
        if (!take.empty() && work + w > c.max_batch_path_steps) break;
        take.push_back(pend[i]);
        opts.push_back(pend[i].opt);
        work += w;
        if (exclusive) break;
    }
    while (!take.empty()) {
        SplitBatch B;
        split_batch(opts.data(), (int32_t)opts.size(), c.dtype, B);
        size_t off = 0;
        if (sv->alloc.alloc(B.total, &off)) {
            sl.off = off;
            sl.bytes = B.total;
            sl.reqs = take;
            sl.split = B;
            sl.exclusive = exclusive;
            sl.t_launch = now_s();
            char *ws = sv->pool + off;
            int rc = enqueue_split(sv->st, sl.split, c.basis, c.dtype, ws, sl.stream,
                                   exclusive ? sv->full_cap : sv->grid_cap, false, sl.staging, sl.staging_bytes,
                                   sv->ppt);
            if (rc == AM_OK) rc = enqueue_split_results(sl.split, ws, sl.h_res, sl.stream);
            if (rc == AM_OK) rc = hipEventRecord(sl.done, sl.stream) == hipSuccess ? AM_OK : AM_EDEVICE;
            if (rc != AM_OK) {
                // nothing of this batch may still run when its memory is reused
                (void)hipStreamSynchronize(sl.stream);
                sv->alloc.release(off, B.total);
                sl.reqs.clear();
                sl.split = SplitBatch();
                sl.exclusive = false;
                if (rc == AM_EDEVICE) {        // the device itself failed: stop serving
                    sv->fatal = rc;
                    sv->fatal_msg = g_err;
                    return false;
                }
                for (size_t i = 0; i < take.size(); ++i) {   // only these requests fail
                    refuse(take[i], rc, out);
                    pend.pop_front();
                }
                return true;
            }
            sl.busy = true;
            for (size_t i = 0; i < take.size(); ++i) pend.pop_front();
            sv->n_batches++;
            sv->n_requests += take.size();
            sv->busy_path_steps += work;
            return true;
        }
        if (take.size() == 1) {
            // a lone request that does not fit even an empty pool is refused
            if (sv->alloc.used == 0) {
                refuse(take[0], AM_ENOMEM, out);
                pend.pop_front();
            }
            return false;
        }
        work -= (double)take.back().opt.n_paths * take.back().opt.n_dates;
        take.pop_back();
        opts.pop_back();
    }
    return false;
}

void server_loop(am_server *sv)
{
    (void)hipSetDevice(sv->st->dev);   // the device was validated at create
    std::deque<Request> local;
    std::vector<am_result> out;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            while (!sv->pending.empty()) { local.push_back(sv->pending.front()); sv->pending.pop_front(); }
            if (!out.empty()) { sv->done.insert(sv->done.end(), out.begin(), out.end()); out.clear(); }
            bool any_busy = false;
            for (auto &sl : sv->slots) any_busy = any_busy || sl.busy;
            if (sv->stop && local.empty() && !any_busy) return;
            if (sv->fatal != AM_OK && !any_busy) return;
            if (local.empty() && !any_busy) {
                sv->cv.wait_for(lk, std::chrono::microseconds(200));
                continue;
            }
        }
        bool progressed = false;
        for (auto &sl : sv->slots) {
            if (sl.busy && hipEventQuery(sl.done) == hipSuccess) {
                finish_slot(sv, sl, out);
                progressed = true;
            }
        }
        if (sv->fatal == AM_OK) {
            for (auto &sl : sv->slots) {
                if (local.empty()) break;
                if (!sl.busy && launch_some(sv, sl, local, out)) progressed = true;
            }
        }
        if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

}  // namespace

extern "C" {

int am_server_create(const am_server_config *cfg, am_server **out)
{
    if (!cfg || !out) return fail(AM_EINVAL, "config and out must be non-NULL");
    if (cfg->n_streams < 1 || cfg->n_streams > 8) return fail(AM_EINVAL, "n_streams must be in [1, 8]");
    if (cfg->max_batch_requests < 1) return fail(AM_EINVAL, "max_batch_requests must be >= 1");
    if (cfg->hbm_budget_bytes < (1u << 20)) return fail(AM_EINVAL, "hbm budget too small");
    if (cfg->dtype != AM_FP64 && cfg->dtype != AM_FP32_BULK) return fail(AM_EINVAL, "unknown dtype");
    if (cfg->basis.degree < 0 || cfg->basis.degree > AM_MAX_DEGREE) return fail(AM_EINVAL, "bad basis degree");
    if (cfg->large_tile != 0 && cfg->large_tile != 1) return fail(AM_EINVAL, "large_tile must be 0 or 1");
    DevState *st = nullptr;
    int rc = get_state(&st);
    if (rc) return rc;
    std::unique_ptr<am_server> sv(new am_server);
    sv->cfg = *cfg;
    sv->st = st;
    if (hipMalloc((void **)&sv->pool, cfg->hbm_budget_bytes) != hipSuccess)
        return fail(AM_ENOMEM, "hipMalloc of the %zu-byte serving pool failed", cfg->hbm_budget_bytes);
    sv->alloc.init(cfg->hbm_budget_bytes);
    // part 0 in the configured storage, part 1 (FP32 bulk only) the small
    // requests stored in binary64; each with the configured tile, and grids
    // capped so that the in-flight ones fit on the device together
    for (int h = 0; h < 2; ++h) {
        const int32_t storage = h == 0 ? cfg->dtype : AM_FP64;
        const int fp64 = storage == AM_FP64;
        // the smaller tile unless asked otherwise: served requests are few
        // per batch, and a request's sweep on four times the workgroups ends
        // sooner (Poisson 200 req/s, 2^12 - 2^20 paths, binary32 storage:
        // p50 1.41 ms, p99 3.67 ms, against 1.92 and 4.73 with the larger)
        sv->ppt[h] = cfg->large_tile ? default_batch_ppt(storage) : small_batch_ppt(storage);
        const int per_cu = amq::sweep_batch_blocks_per_cu(fp64, cfg->basis.kind == AM_BASIS_LAGUERRE, sv->ppt[h],
                                                          cfg->basis.degree);
        if (per_cu <= 0) return fail(AM_EDEVICE, "no batch sweep kernel");
        sv->full_cap[h] = per_cu * st->num_cu;
        sv->grid_cap[h] = sv->full_cap[h] / cfg->n_streams;
    }
    sv->slots.resize(cfg->n_streams);
    for (auto &sl : sv->slots) {
        HIP_TRY(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
        sl.staging_bytes = 8u << 20;
        if (hipHostMalloc((void **)&sl.staging, sl.staging_bytes, hipHostMallocDefault) != hipSuccess)
            return fail(AM_ENOMEM, "pinned staging allocation failed");
        if (hipHostMalloc((void **)&sl.h_res, (size_t)cfg->max_batch_requests * 64 + 128, hipHostMallocDefault) != hipSuccess)
            return fail(AM_ENOMEM, "pinned result allocation failed");
    }
    {
        std::lock_guard<std::mutex> lk(g_res_mu);
        ++g_live_servers;
    }
    am_server *p = sv.release();
    p->th = std::thread(server_loop, p);
    *out = p;
    return AM_OK;
}

int am_server_submit(am_server *sv, const am_option *opt, uint64_t request_id, double t_arrival)
{
    if (!sv || !opt) return fail(AM_EINVAL, "server and option must be non-NULL");
    int rc = validate(&opt->params, opt->n_paths, opt->n_dates, sv->cfg.basis, sv->cfg.dtype);
    if (rc) return rc;
    int h = 0;
    const int64_t tiles = request_tiles(sv, *opt, &h);
    if (tiles > sv->full_cap[h])
        return fail(AM_EDIM, "request needs %lld sweep workgroups; the device holds %d resident", (long long)tiles,
                    sv->full_cap[h]);
    Request r;
    r.opt = *opt;
    r.id = request_id;
    r.t_arrival = t_arrival >= 0.0 ? t_arrival : now_s();
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->stop) return fail(AM_EINVAL, "server is stopping");
        if (sv->fatal != AM_OK) return fail(sv->fatal, "server failed: %s", sv->fatal_msg.c_str());
        sv->pending.push_back(r);
    }
    sv->cv.notify_one();
    return AM_OK;
}

int am_server_poll(am_server *sv, am_result *out, int32_t max_out, int32_t *n_out)
{
    if (!sv || !out || !n_out || max_out < 0) return fail(AM_EINVAL, "bad arguments to am_server_poll");
    std::lock_guard<std::mutex> lk(sv->mu);
    const int32_t n = (int32_t)std::min<size_t>(sv->done.size(), (size_t)max_out);
    for (int32_t i = 0; i < n; ++i) out[i] = sv->done[i];
    sv->done.erase(sv->done.begin(), sv->done.begin() + n);
    *n_out = n;
    if (sv->fatal != AM_OK && n == 0) return fail(sv->fatal, "server failed: %s", sv->fatal_msg.c_str());
    return AM_OK;
}

double am_server_now(void) { return now_s(); }

int am_server_stats(am_server *sv, double out[4])
{
    if (!sv || !out) return fail(AM_EINVAL, "bad arguments to am_server_stats");
    std::lock_guard<std::mutex> lk(sv->mu);
    out[0] = (double)sv->n_batches;
    out[1] = (double)sv->n_requests;
    out[2] = sv->busy_path_steps;
    out[3] = (double)sv->alloc.used;
    return AM_OK;
}

int am_server_destroy(am_server *sv)
{
    if (!sv) return AM_OK;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv.notify_one();
    if (sv->th.joinable()) sv->th.join();
    int rc = sv->fatal;
    for (auto &sl : sv->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.staging) (void)hipHostFree(sl.staging);
        if (sl.h_res) (void)hipHostFree(sl.h_res);
    }
    if (sv->pool) (void)hipFree(sv->pool);
    delete sv;
    {
        std::lock_guard<std::mutex> lk(g_res_mu);
        --g_live_servers;
    }
    return rc;
}



int am_debug_schedule(int32_t n_dates, int32_t *m, int32_t *dim, int32_t *left, int32_t *right,
                      double *wl, double *wr, double *sd)
{
    if (n_dates < 1 || n_dates > amq::kMaxDates) return fail(AM_EDIM, "n_dates out of range");
    std::vector<amq::BridgeNode> s = make_schedule(n_dates);
    // recover left/right dates from slots: replay the slot contents
    std::vector<int> slot_date(amq::kMaxSlots + 1, 0);
    for (int q = 0; q < n_dates; ++q) {
        const amq::BridgeNode &n = s[q];
        if (m) m[q] = n.m;
        if (dim) dim[q] = n.dim;
        if (left) left[q] = slot_date[n.sl];
        if (right) right[q] = n.sr == 0 && q == 0 ? 0 : slot_date[n.sr];
        if (wl) wl[q] = n.wl;
        if (wr) wr[q] = n.wr;
        if (sd) sd[q] = n.sd;
        if (n.dst <= amq::kMaxSlots) slot_date[n.dst] = n.m;
    }
    return AM_OK;
}

void am_debug_set_spin_limit(uint32_t spins) { g_spin_limit = spins; }

int am_shutdown(void)
{
    {
        std::lock_guard<std::mutex> lk(g_res_mu);
        if (g_live_servers > 0) return fail(AM_EINVAL, "%d server(s) still running", g_live_servers);
    }
    int rc = AM_OK;
    {
        std::lock_guard<std::mutex> lk(g_dev_mu);
        int cur = -1;
        const bool restore = !g_devs.empty() && hipGetDevice(&cur) == hipSuccess;
        for (auto &kv : g_devs) {
            DevState *st = kv.second.get();
            if (hipSetDevice(st->dev) != hipSuccess) {
                rc = fail(AM_EDEVICE, "hipSetDevice(%d) failed during shutdown", st->dev);
                continue;
            }
            // the library's own work first: the synchronous stream and the
            // last single-option sweep on any stream
            if (st->stream) (void)hipStreamSynchronize(st->stream);
            if (st->persist_done) (void)hipEventSynchronize(st->persist_done);
            for (auto &sc : st->sched) (void)hipFree(sc.second);
            st->sched.clear();
            if (st->d_V) (void)hipFree(st->d_V);
            if (st->ws) (void)hipFree(st->ws);
            if (st->persist_done) (void)hipEventDestroy(st->persist_done);
            if (st->stream) (void)hipStreamDestroy(st->stream);
            st->d_V = nullptr;
            st->ws = nullptr;
            st->persist_done = nullptr;
            st->stream = nullptr;
        }
        g_devs.clear();
        if (restore) (void)hipSetDevice(cur);
    }
    std::lock_guard<std::mutex> lk(g_res_mu);
    for (void *ptr : g_pinned_all) (void)hipHostFree(ptr);
    for (hipEvent_t e : g_events_all) (void)hipEventDestroy(e);
    g_pinned_all.clear();
    g_events_all.clear();
    ++g_generation;   // threads drop their cached pointers on next use
    return rc;
}

int am_profile_enable(int32_t on)
{
    g_prof.on = on != 0;
    g_prof.used = 0;
    return AM_OK;
}

int am_profile_read(double ms[2], int64_t *calls)
{
    if (!ms || !calls) return fail(AM_EINVAL, "ms and calls must be non-NULL");
    {
        std::lock_guard<std::mutex> lk(g_res_mu);
        if (g_prof.gen != g_generation) {   // events released by am_shutdown
            g_prof.pool.clear();
            g_prof.used = 0;
            g_prof.gen = g_generation;
        }
    }
    double g = 0.0, w = 0.0;
    for (size_t i = 0; i < g_prof.used; ++i) {
        ProfRec &r = g_prof.pool[i];
        HIP_TRY(hipEventSynchronize(r.e[2]));
        float a = 0.f, b = 0.f;
        HIP_TRY(hipEventElapsedTime(&a, r.e[0], r.e[1]));
        HIP_TRY(hipEventElapsedTime(&b, r.e[1], r.e[2]));
        g += a;
        w += b;
    }
    ms[0] = g;
    ms[1] = w;
    *calls = (int64_t)g_prof.used;
    g_prof.used = 0;
    return AM_OK;
}

int am_debug_generate(int32_t what, const am_params *params, int64_t n_paths, int32_t n_dims,
                      int32_t dtype, void *host_out)
{
    if (!host_out) return fail(AM_EINVAL, "host_out is NULL");
    if (what < 0 || what > 2) return fail(AM_EINVAL, "what must be 0, 1 or 2");
    am_basis b = {AM_BASIS_MONOMIAL, 0};
    am_params dflt = {100.0, 100.0, 0.0, 0.2, 1.0, 0, 0};
    const am_params *p = params ? params : &dflt;
    int rc = validate(p, n_paths, n_dims, b, dtype);
    if (rc) return rc;
    DevState *st = nullptr;
    rc = get_state(&st);
    if (rc) return rc;
    const amq::BridgeNode *sched = nullptr;
    rc = get_schedule(st, n_dims, &sched);
    if (rc) return rc;
    const int fp64 = dtype == AM_FP64;
    const int64_t ld = (n_paths + 63) / 64 * 64;
    const size_t el = what == 1 ? 4 : (what == 2 ? 8 : (fp64 ? 8 : 4));
    const size_t out_b = (size_t)n_dims * ld * el;
    const size_t aux_b = align256((size_t)(n_dims + 1) * sizeof(amq::DateConst)) + align256(amq::kSyncWords * 4);
    char *d = nullptr;
    if (hipMalloc((void **)&d, align256(out_b) + aux_b) != hipSuccess)
        return fail(AM_ENOMEM, "hipMalloc for the diagnostic output failed");
    amq::GenArgs ga;
    memset(&ga, 0, sizeof ga);
    ga.S = d;
    ga.V = st->d_V;
    ga.sched = sched;
    ga.datec = (amq::DateConst *)(d + align256(out_b));
    ga.sync = (uint32_t *)(d + align256(out_b) + align256((size_t)(n_dims + 1) * sizeof(amq::DateConst)));
    ga.N = n_paths; ga.ld = ld; ga.nblocks = (n_paths + 63) / 64; ga.M = n_dims;
    const int64_t target_waves = (int64_t)st->num_cu * kGenWavesPerCU;
    int64_t R = (ga.nblocks + target_waves - 1) / target_waves;
    ga.R = (int32_t)(R < 1 ? 1 : R);
    ga.what = what;
    ga.S0 = p->S0; ga.K = p->K; ga.r = p->r; ga.sigma = p->sigma; ga.T = p->T;
    const double dt = p->T / (double)n_dims;
    ga.mu = (p->r - 0.5 * p->sigma * p->sigma) * dt;
    ga.vol = p->sigma * sqrt(dt);
    hipError_t e = amq::launch_generate(ga, fp64, st->stream);
    std::vector<char> h(out_b);
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), d, out_b, hipMemcpyDeviceToHost, st->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(st->stream);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(AM_EDEVICE, "diagnostic generation failed: %s", hipGetErrorString(e));
    // compact [dims][ld] -> [dims][n_paths]; paths as double
    for (int32_t j = 0; j < n_dims; ++j) {
        const char *src = h.data() + (size_t)j * ld * el;
        if (what == 1) {
            memcpy((uint32_t *)host_out + (size_t)j * n_paths, src, (size_t)n_paths * 4);
        } else if (el == 8) {
            memcpy((double *)host_out + (size_t)j * n_paths, src, (size_t)n_paths * 8);
        } else {
            const float *f = (const float *)src;
            double *o = (double *)host_out + (size_t)j * n_paths;
            for (int64_t i = 0; i < n_paths; ++i) o[i] = (double)f[i];
        }
    }
    return AM_OK;
}

}  // extern "C"
