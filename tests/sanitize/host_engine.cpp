// Host-side engine logic under AddressSanitizer and UndefinedBehaviorSanitizer
// (CPU only, no device).  The engine's translation unit is included whole, so
// its internal pieces (the pool allocator) are reachable; the kernel entry
// points it calls are stubbed out, and nothing here launches work.  Exercises:
// argument validation, the storage rule, workspace sizes and layouts, bridge
// schedules for every date count, batch workspace sizing, the first-fit pool
// allocator against a reference model, error strings and shutdown without
// device work.  Exit status 0 and no sanitizer report = pass.
#include "../../paper_1205_0106_amd/csrc/amq_engine.hip"

#include <random>
#include <set>

// direction numbers: only the device set-up reads them, which never runs here
extern "C" const uint32_t amq_sobol_v32[amq::kMaxDates * 32] = {0};
extern "C" const uint32_t amq_sobol_v32_dims = amq::kMaxDates;

namespace amq {
hipError_t launch_generate(const GenArgs &, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t preload_generate() { return hipErrorNotSupported; }
hipError_t launch_sweep(const SweepArgs &, int, int, int, hipStream_t) { return hipErrorNotSupported; }
int sweep_blocks_per_cu(int, int, int, int, int) { return 1; }
__host__ __device__ size_t generate_lds_bytes(int M, int) { return (size_t)M * 64; }
hipError_t launch_paper(const PaperArgs &, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_generate_batch(const BatchOpt *, const GenUnit *, int, const uint32_t *, uint32_t *, int, int,
                                 bool, hipStream_t)
{
    return hipErrorNotSupported;
}
hipError_t launch_sweep_batch(const BatchOpt *, const int32_t *, const BatchGlobal &, int, int, int, int, bool,
                              hipStream_t)
{
    return hipErrorNotSupported;
}
int sweep_batch_blocks_per_cu(int, int, int, int) { return 1; }
const void *sweep_table_f32_mono(int, int, int) { return nullptr; }
const void *sweep_table_f32_lag(int, int, int) { return nullptr; }
const void *sweep_table_f64_mono(int, int, int) { return nullptr; }
const void *sweep_table_f64_lag(int, int, int) { return nullptr; }
}  // namespace amq

static int g_fail = 0;
#define CHECK(c)                                                                  \
    do {                                                                          \
        if (!(c)) {                                                               \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c);       \
            ++g_fail;                                                             \
        }                                                                         \
    } while (0)

static void storage_rule()
{
    CHECK(am_storage_dtype(1, AM_FP32_BULK) == AM_FP64);
    CHECK(am_storage_dtype(AM_FP32_MIN_PATHS - 1, AM_FP32_BULK) == AM_FP64);
    CHECK(am_storage_dtype(AM_FP32_MIN_PATHS, AM_FP32_BULK) == AM_FP32_BULK);
    CHECK(am_storage_dtype(1 << 24, AM_FP64) == AM_FP64);
    CHECK(am_storage_dtype(1000, 7) == -1);
}

static void layouts()
{
    const int64_t Ns[] = {1, 63, 64, 65, 4097, 16383, 16384, 70000, (1 << 20) + 3, 1 << 24};
    const int32_t Ms[] = {1, 2, 3, 17, 100, 252, 365, amq::kMaxDates};
    for (int64_t N : Ns)
        for (int32_t M : Ms)
            for (int dt = 0; dt < 2; ++dt)
                for (int kind = 0; kind < 2; ++kind)
                    for (int deg = 0; deg <= AM_MAX_DEGREE; deg += 3) {
                        am_basis b{kind, deg};
                        size_t off[6];
                        CHECK(am_workspace_layout(N, M, b, dt, off) == AM_OK);
                        const size_t ws = am_workspace_bytes(N, M, b, dt);
                        CHECK(ws == off[5]);
                        const size_t s = am_storage_dtype(N, dt) == AM_FP64 ? 8 : 4;
                        CHECK((int64_t)off[4] >= N);
                        CHECK(off[0] % 256 == 0 && off[1] % 256 == 0 && off[2] % 256 == 0 && off[3] % 256 == 0);
                        CHECK(off[1] >= off[0] + (size_t)M * off[4] * s);
                        CHECK(off[2] >= off[1] + off[4] * s);
                        CHECK(off[3] >= off[2] + (size_t)(M + 1) * 40 * 8);
                        CHECK(off[3] + 64 <= off[5]);
                    }
    size_t off[6];
    am_basis b{0, 2};
    CHECK(am_workspace_layout(0, 10, b, AM_FP64, off) == AM_EINVAL);
    CHECK(am_workspace_layout(100, 0, b, AM_FP64, off) == AM_EINVAL);
    CHECK(am_workspace_layout(100, 10, b, 7, off) == AM_EINVAL);
    CHECK(am_workspace_layout(100, 10, b, AM_FP64, nullptr) == AM_EINVAL);
    CHECK(am_workspace_bytes(0, 10, b, AM_FP64) == 0);
    CHECK(am_workspace_bytes(100, 0, b, AM_FP64) == 0);
}

static void schedules()
{
    for (int M = 1; M <= amq::kMaxDates; ++M) {
        std::vector<int32_t> m(M), dim(M), l(M), r(M);
        std::vector<double> wl(M), wr(M), sd(M);
        CHECK(am_debug_schedule(M, m.data(), dim.data(), l.data(), r.data(), wl.data(), wr.data(), sd.data()) ==
              AM_OK);
        std::set<int> dates, dims;
        for (int q = 0; q < M; ++q) {
            dates.insert(m[q]);
            dims.insert(dim[q]);
            CHECK(m[q] >= 1 && m[q] <= M);
            CHECK(std::isfinite(wl[q]) && std::isfinite(wr[q]) && sd[q] > 0.0);
        }
        CHECK((int)dates.size() == M && (int)dims.size() == M);
        CHECK(*dims.begin() == 0 && *dims.rbegin() == M - 1);
    }
    int32_t one;
    double d;
    CHECK(am_debug_schedule(0, &one, &one, &one, &one, &d, &d, &d) < 0);
    CHECK(am_debug_schedule(amq::kMaxDates + 1, &one, &one, &one, &one, &d, &d, &d) < 0);
}

static void validation()
{
    const am_basis b{0, 2};
    double p = -1.0, se = -1.0;
    const double nan = std::numeric_limits<double>::quiet_NaN();
    const am_params good{100.0, 100.0, 0.05, 0.2, 1.0, 0, 1};
    am_params bad[] = {good, good, good, good, good, good, good};
    bad[0].S0 = 0.0;
    bad[1].K = -1.0;
    bad[2].sigma = 0.0;
    bad[3].T = nan;
    bad[4].r = std::numeric_limits<double>::infinity();
    bad[5].is_call = 2;
    bad[6].allow_exercise = -1;
    for (auto &q : bad) {
        CHECK(am_price_american(&q, 1000, 10, b, AM_FP64, &p, &se) == AM_EINVAL);
        CHECK(strlen(am_last_error()) > 0);
    }
    CHECK(am_price_american(nullptr, 1000, 10, b, AM_FP64, &p, &se) == AM_EINVAL);
    CHECK(am_price_american(&good, 0, 10, b, AM_FP64, &p, &se) == AM_EINVAL);
    CHECK(am_price_american(&good, 1000, 0, b, AM_FP64, &p, &se) == AM_EINVAL);
    CHECK(am_price_american(&good, 1000, amq::kMaxDates + 1, b, AM_FP64, &p, &se) != AM_OK);
    CHECK(am_price_american(&good, 1000, 10, am_basis{0, 9}, AM_FP64, &p, &se) == AM_EINVAL);
    CHECK(am_price_american(&good, 1000, 10, b, 3, &p, &se) == AM_EINVAL);
    CHECK(p == -1.0 && se == -1.0);
}

static void batch_sizes()
{
    std::vector<am_option> o(37);
    for (size_t i = 0; i < o.size(); ++i) {
        o[i].params = am_params{100.0, 80.0 + (double)i, 0.03, 0.2 + 0.01 * (double)i, 1.0, (int32_t)(i & 1), 1};
        o[i].n_paths = (int64_t)(1000 + 977 * i * i);
        o[i].n_dates = (int32_t)(3 + 7 * i);
        o[i].reserved = 0;
    }
    const am_basis b{0, 2};
    const size_t w32 = am_batch_workspace_bytes(o.data(), (int32_t)o.size(), b, AM_FP32_BULK);
    const size_t w64 = am_batch_workspace_bytes(o.data(), (int32_t)o.size(), b, AM_FP64);
    CHECK(w32 > 0 && w64 > w32);
    CHECK(am_batch_workspace_bytes(o.data(), 0, b, AM_FP64) == 0);
    CHECK(am_rqmc_workspace_bytes(4096, 20, b, AM_FP64, 0) == 0);
    CHECK(am_rqmc_workspace_bytes(4096, 20, b, AM_FP64, 65) == 0);
    CHECK(am_rqmc_workspace_bytes(4096, 20, b, AM_FP64, 8) > am_rqmc_workspace_bytes(4096, 20, b, AM_FP64, 2));
    CHECK(am_rqmc_workspace_bytes(1 << 15, 20, b, AM_FP32_BULK, 8) < am_rqmc_workspace_bytes(1 << 15, 20, b, AM_FP64, 8));
    o[5].n_dates = 0;
    CHECK(am_batch_workspace_bytes(o.data(), (int32_t)o.size(), b, AM_FP64) == 0);
}

static void pool()
{
    // first-fit pool against a byte map: allocations never overlap, stay in
    // range, and the pool coalesces back to one block
    const size_t cap = (size_t)1 << 22;
    PoolAlloc P;
    P.init(cap);
    std::vector<std::pair<size_t, size_t>> live;
    std::vector<unsigned char> used(cap / 256, 0);
    std::mt19937_64 rng(7);
    for (int step = 0; step < 20000; ++step) {
        if (live.empty() || (rng() % 3 != 0)) {
            const size_t bytes = 1 + rng() % 200000;
            size_t off = 0;
            if (P.alloc(bytes, &off)) {
                const size_t nb = (bytes + 255) / 256;
                CHECK(off % 256 == 0 && off + nb * 256 <= cap);
                for (size_t q = off / 256; q < off / 256 + nb && q < used.size(); ++q) {
                    CHECK(used[q] == 0);
                    used[q] = 1;
                }
                live.push_back({off, bytes});
            }
        } else {
            const size_t i = rng() % live.size();
            const auto [off, bytes] = live[i];
            const size_t nb = (bytes + 255) / 256;
            for (size_t q = off / 256; q < off / 256 + nb; ++q) used[q] = 0;
            P.release(off, bytes);
            live[i] = live.back();
            live.pop_back();
        }
    }
    for (auto &[off, bytes] : live) P.release(off, bytes);
    CHECK(P.used == 0);
    CHECK(P.free_.size() == 1 && P.free_.begin()->first == 0 && P.free_.begin()->second == cap);
}

int main()
{
    storage_rule();
    layouts();
    schedules();
    validation();
    batch_sizes();
    pool();
    CHECK(am_shutdown() == AM_OK);
    CHECK(am_shutdown() == AM_OK);
    if (g_fail) {
        fprintf(stderr, "%d checks failed\n", g_fail);
        return 1;
    }
    printf("host engine checks passed\n");
    return 0;
}
