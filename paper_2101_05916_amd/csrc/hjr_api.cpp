// hjr_api.cpp -- the extern "C" entry points of libhjr declared in hjr.h:
// argument validation, workspace layout, stream ordering and statistics
// around the engine.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/hjr.h"
#include "hjr_engine.hpp"
#include "hjr_launch.hpp"

using namespace hjr;

// Scratch of hjr_solve_noalloc: one statically sized array per device,
// loaded with the code object and held until the process ends.  In host
// code `scratch` names a host-side stand-in, not device memory: only the
// address from hipGetSymbolAddress (per device, with that device current)
// may be handed to kernels or copies.
static __device__ __align__(256) char scratch[HJR_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kDefaultChunk = 32;

size_t align256(size_t x)
{
    return (x + 255) & ~size_t(255);
}

hjr_opts resolve(const hjr_opts* o)
{
    hjr_opts r;
    hjr_opts_default(&r);
    if (o) r = *o;
    return r;
}

bool opts_valid(const hjr_opts& o)
{
    if (o.dtype != HJR_F32 && o.dtype != HJR_F64) return false;
    if (o.order != 1 && o.order != 2) return false;
    if (!(o.cfl > 0.0 && o.cfl <= 1.0)) return false;
    if (o.max_iter < 1) return false;
    if (o.chunk < 0 || o.chunk > kMaxChunk) return false;
    if (o.tile_rows < 0) return false;
    if (o.walk < -1) return false;
    if (!(o.band >= 0.0)) return false;
    return true;
}

int chunk_of(const hjr_opts& o)
{
    return o.chunk > 0 ? o.chunk : kDefaultChunk;
}

bool dstb_valid(const hjr_dyn& dyn, const hjr_dstb* d)
{
    if (!d) return false;
    for (int c = 0; c < dyn_channels(dyn.kind); c++)
        if (!(d[c].lo <= d[c].hi) || !std::isfinite(d[c].lo) || !std::isfinite(d[c].hi))
            return false;
    return true;
}

bool same_box(const hjr_grid& a, const hjr_grid& b)
{
    if (a.ndim != b.ndim) return false;
    for (int i = 0; i < a.ndim; i++)
        if (a.lo[i] != b.lo[i] || a.hi[i] != b.hi[i]) return false;
    return true;
}

// Per-tile scratch of a localized update (level 0): a flag per tile -- flat
// tiles (N / kTile of them) or plane tiles of at least one row (at most
// N / n_last of them) -- and the list of the live plane tiles (4 bytes each).
static int64_t mask_flag_bytes(const hjr_grid& g)
{
    const int64_t N = grid_size(g);
    return align256(std::max<int64_t>(N / kTile, N / g.n[g.ndim - 1]) + 1);
}

static int64_t mask_tile_bytes(const hjr_grid& g)
{
    const int64_t N = grid_size(g);
    return mask_flag_bytes(g) + align256(4 * (N / g.n[g.ndim - 1] + 1));
}

// Scratch of one job: the stage-1 array, the lookup table and the per-tile
// flags and list of a localized update.
size_t job_scratch_bytes(const hjr_grid* grids, int nlev, int dtype)
{
    int64_t N = 0, n2 = 0;
    for (int k = 0; k < nlev; k++) {
        N = std::max<int64_t>(N, grid_size(grids[k]));
        if (grids[k].ndim >= 3) n2 = std::max<int64_t>(n2, grids[k].n[2]);
    }
    return align256(N * elem_size(dtype)) + align256(std::max<int64_t>(n2, 1) * elem_size(dtype)) +
           mask_tile_bytes(grids[0]);
}

// Idle engines are kept for reuse, keyed by what fixes their device tables,
// kernels and captured graphs: device, dtype, chunk length, slot count
// (rounded up to a power of two) and flags.  A pooled engine owns a
// non-blocking stream; a call orders it after the caller's stream and
// synchronises it before returning.
struct PoolKey {
    int dev, dtype, K, cap, flags;
    bool operator<(const PoolKey& o) const
    {
        if (dev != o.dev) return dev < o.dev;
        if (dtype != o.dtype) return dtype < o.dtype;
        if (K != o.K) return K < o.K;
        if (cap != o.cap) return cap < o.cap;
        return flags < o.flags;
    }
};

std::mutex g_pool_mu;
std::map<PoolKey, std::vector<Engine*>>* g_pool = new std::map<PoolKey, std::vector<Engine*>>();
constexpr size_t kPoolKeep = 4;  // idle engines kept per key

int cap_bucket(int n)
{
    int c = 1;
    while (c < n) c <<= 1;
    return c;
}

struct Session {
    PoolKey key{};
    Engine* eng = nullptr;
    void* owned = nullptr;
    char* ws = nullptr;
    hipEvent_t t0 = nullptr, t1 = nullptr;

    hjr_status open(const hjr_opts& o, const EngineCfg& cfg_in, size_t need)
    {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return HJR_EDEVICE;
        EngineCfg cfg = cfg_in;
        cfg.cap = cap_bucket(cfg.cap);
        key = PoolKey{dev, cfg.dtype, cfg.K, cfg.cap, cfg.flags};
        {
            std::lock_guard<std::mutex> lk(g_pool_mu);
            auto& v = (*g_pool)[key];
            if (!v.empty()) {
                eng = v.back();
                v.pop_back();
            }
        }
        if (eng) {
            if (eng->reset(cfg) != HJR_OK) return HJR_EDEVICE;
        } else {
            hipStream_t s = nullptr;
            if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return HJR_EDEVICE;
            eng = new Engine(cfg);
            hjr_status st = eng->init(s, nullptr);
            if (st != HJR_OK) {
                delete eng;
                eng = nullptr;
                (void)hipStreamDestroy(s);
                return st;
            }
        }
        hipEvent_t dep;
        if (hipEventCreateWithFlags(&dep, hipEventDisableTiming) != hipSuccess) return HJR_EDEVICE;
        if (hipEventRecord(dep, (hipStream_t)o.stream) != hipSuccess ||
            hipStreamWaitEvent(eng->stream(), dep, 0) != hipSuccess) {
            (void)hipEventDestroy(dep);
            return HJR_EDEVICE;
        }
        (void)hipEventDestroy(dep);
        if (o.workspace) {
            if (o.workspace_bytes < need) return HJR_ENOMEM;
            ws = (char*)o.workspace;
        } else if (need > 0) {
            if (hipMalloc(&owned, need) != hipSuccess) return HJR_ENOMEM;
            ws = (char*)owned;
        }
        if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess) return HJR_EDEVICE;
        if (hipEventRecord(t0, eng->stream()) != hipSuccess) return HJR_EDEVICE;
        return HJR_OK;
    }
    double elapsed_ms()
    {
        float ms = 0.f;
        if (hipEventRecord(t1, eng->stream()) != hipSuccess) return 0.0;
        if (hipEventSynchronize(t1) != hipSuccess) return 0.0;
        if (hipEventElapsedTime(&ms, t0, t1) != hipSuccess) return 0.0;
        return ms;
    }
    bool clean = false;  // set once every job finished and the engine is idle

    ~Session()
    {
        if (eng) {
            const bool ok = hipStreamSynchronize(eng->stream()) == hipSuccess;
            std::lock_guard<std::mutex> lk(g_pool_mu);
            auto& v = (*g_pool)[key];
            if (ok && clean && !eng->busy() && v.size() < kPoolKeep)
                v.push_back(eng);
            else
                delete eng;  // its stream stays alive with the process
        }
        if (owned) (void)hipFree(owned);
        if (t0) (void)hipEventDestroy(t0);
        if (t1) (void)hipEventDestroy(t1);
    }
};

void fill_stats(hjr_stats* st, const Job& j, const ProbState& ps, double ms, const Engine& eng,
                int64_t updated_nodes = -1)
{
    if (!st) return;
    std::memset(st, 0, sizeof(*st));
    int64_t tot = 0, cu = 0;
    for (int k = 0; k < 4; k++) {
        st->level_iterations[k] = j.level_iters[k];
        tot += j.level_iters[k];
        if (k < j.nlev)
            cu += (updated_nodes >= 0 ? updated_nodes : grid_size(j.lev[k].grid)) * j.level_iters[k];
    }
    st->cell_updates = cu;
    eng.profile(st->kernel_ms, st->kernel_launches, &st->kernel_cell_updates);
    st->iterations = tot;
    st->residual = j.residual;
    st->dt = ps.dt;
    for (int a = 0; a < 4; a++) st->alpha[a] = ps.alpha[a];
    st->status = j.status;
    int done = 0;
    for (int k = 0; k < j.nlev; k++) done += (j.level_iters[k] > 0);
    st->levels = done;
    st->device_ms = ms;
}

// Drive an engine until every job finished.
hjr_status run_engine(Engine& eng)
{
    while (eng.busy()) {
        hjr_status st = eng.step();
        if (st != HJR_OK) return st;
    }
    return eng.drain();
}

// need_d: some level uses the constant boxes d (no disturbance field).
hjr_status check_job_spec(const hjr_dyn* dyn, int nlev, const hjr_grid* grids, const hjr_dstb* d,
                          double tol, double band, bool need_d = true)
{
    if (!(band >= 0.0)) return HJR_EINVAL;  // negative or NaN
    if (!dyn || !grids || (need_d && !d)) return HJR_EINVAL;
    if (nlev < 1 || nlev > 4) return HJR_EINVAL;
    for (int k = 0; k < nlev; k++) {
        if (!grid_valid(grids[k])) return HJR_EINVAL;
        if (!dyn_valid(*dyn, grids[k])) return HJR_EINVAL;
        if (k > 0 && !same_box(grids[0], grids[k])) return HJR_EINVAL;
    }
    if (need_d && !dstb_valid(*dyn, d)) return HJR_EINVAL;
    if (!(tol > 0.0) || !std::isfinite(tol)) return HJR_EINVAL;
    return HJR_OK;
}

// Device check of the disturbance fields of a job's levels (EINVAL if a
// pair is not finite and ordered).
hjr_status check_fields(Engine& eng, const Job& j)
{
    for (int k = 0; k < j.nlev; k++) {
        if (!j.lev[k].dfield) continue;
        int64_t bad = 0;
        hjr_status st = eng.check_field(j.lev[k].dfield, dyn_channels(j.dyn.kind),
                                        grid_size(j.lev[k].grid), &bad);
        if (st != HJR_OK) return st;
        if (bad) return HJR_EINVAL;
    }
    return HJR_OK;
}

// Coarse-to-fine solve of one job, with optional fields per level
// (dfield == NULL or dfield[k] == NULL: the boxes d).
hjr_status solve_levels_impl(const hjr_dyn* dyn, int32_t nlev, const hjr_grid* grids,
                             const void* const* l, const void* const* dfield, const void* V0,
                             const hjr_dstb* d, double tol, const hjr_opts* o,
                             void* const* V_levels, uint8_t* const* masks,
                             int64_t* mask_counts, hjr_stats* stats,
                             const uint8_t* umask = nullptr)
{
    const hjr_opts op = resolve(o);
    if (!opts_valid(op)) return HJR_EINVAL;
    bool need_d = !dfield;
    if (dfield && nlev >= 1 && nlev <= 4)
        for (int k = 0; k < nlev; k++) need_d = need_d || !dfield[k];
    hjr_status st = check_job_spec(dyn, nlev, grids, d, tol, op.band, need_d);
    if (st != HJR_OK) return st;
    if (!l || !V_levels) return HJR_EINVAL;
    for (int k = 0; k < nlev; k++)
        if (!l[k] || !V_levels[k]) return HJR_EINVAL;

    const int K = chunk_of(op);
    const size_t need = job_scratch_bytes(grids, nlev, op.dtype);
    try {
        EngineCfg cfg;
        cfg.dtype = op.dtype;
        cfg.order = op.order;
        cfg.cfl = op.cfl;
        cfg.max_iter = op.max_iter;
        cfg.walk = op.walk;
        cfg.K = K;
        cfg.cap = 1;
        cfg.flags = op.flags;
        Session ses;
        if ((st = ses.open(op, cfg, need)) != HJR_OK) return st;
        Engine& eng = *ses.eng;
        Job j;
        j.dyn = *dyn;
        std::memset(j.d, 0, sizeof(j.d));
        if (need_d)
            for (int c = 0; c < dyn_channels(dyn->kind); c++) j.d[c] = d[c];
        j.tol = tol;
        j.band = op.band;
        j.nlev = nlev;
        for (int k = 0; k < nlev; k++) {
            j.lev[k].grid = grids[k];
            j.lev[k].l = l[k];
            j.lev[k].V = V_levels[k];
            j.lev[k].mask = masks ? masks[k] : nullptr;
            j.lev[k].tile_rows = op.tile_rows;
            j.lev[k].dfield = dfield ? dfield[k] : nullptr;
        }
        j.V0 = V0;
        if ((st = check_fields(eng, j)) != HJR_OK) {
            if (st == HJR_EINVAL) ses.clean = true;  // the engine is idle and intact
            return st;
        }
        int64_t Nmax = 0, n2 = 1;
        for (int k = 0; k < nlev; k++) {
            Nmax = std::max(Nmax, grid_size(grids[k]));
            if (grids[k].ndim >= 3) n2 = std::max<int64_t>(n2, grids[k].n[2]);
        }
        j.Vhat = ses.ws;
        j.table = ses.ws + align256(Nmax * elem_size(op.dtype));
        int64_t updated = -1;
        if (umask) {
            j.lev[0].umask = umask;
            j.lev[0].tmask = (uint8_t*)((char*)j.table + align256(n2 * elem_size(op.dtype)));
            j.lev[0].tlist = (uint32_t*)((char*)j.lev[0].tmask + mask_flag_bytes(grids[0]));
            if ((st = eng.count_mask(umask, grid_size(grids[0]), &updated)) != HJR_OK) return st;
        }
        if ((st = eng.add(&j)) != HJR_OK) return st;
        if ((st = run_engine(eng)) != HJR_OK) return st;
        ProbState ps;
        if ((st = eng.read_state(j.slot, &ps)) != HJR_OK) return st;
        if (mask_counts) {
            uint64_t mc[4];
            if ((st = eng.read_mask_counts(j.slot, mc)) != HJR_OK) return st;
            for (int k = 0; k < nlev; k++) mask_counts[k] = (int64_t)mc[k];
        }
        const double ms = ses.elapsed_ms();
        fill_stats(stats, j, ps, ms, eng, updated);
        ses.clean = true;
        return (hjr_status)j.status;
    } catch (const std::bad_alloc&) {
        return HJR_ENOMEM;
    } catch (...) {
        return HJR_EDEVICE;
    }
}

// Per-device address of the scratch of hjr_solve_noalloc (file scope, above).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch (looked up once per device).
hjr_status scratch_of_current_device(void** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return HJR_EDEVICE;
    if (dev < 0 || dev >= kMaxDevices) return HJR_EDEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
            return HJR_EDEVICE;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return HJR_OK;
}

// Host staging of a static engine with one slot: at most this many bytes
// (host_bytes(1, kMaxChunk)), on the caller's stack.
constexpr size_t kNoallocHostBytes = 16384;

}  // namespace

extern "C" {

hjr_status hjr_opts_default(hjr_opts* o)
{
    if (!o) return HJR_EINVAL;
    std::memset(o, 0, sizeof(*o));
    o->dtype = HJR_F32;
    o->order = 2;
    o->cfl = 0.8;
    o->max_iter = 100000;
    o->chunk = 0;
    o->flags = 0;
    return HJR_OK;
}

const char* hjr_strerror(hjr_status s)
{
    switch (s) {
    case HJR_OK: return "ok";
    case HJR_EINVAL: return "invalid argument";
    case HJR_ENOMEM: return "out of memory or workspace too small";
    case HJR_NOT_CONVERGED: return "not converged within max_iter";
    case HJR_EDEVICE: return "HIP runtime error";
    case HJR_EBUSY: return "busy";
    case HJR_ENOTFOUND: return "not found";
    default: return "unknown status";
    }
}

hjr_status hjr_workspace_bytes(const hjr_grid* g, const hjr_opts* o, size_t* out)
{
    if (!g || !out) return HJR_EINVAL;
    const hjr_opts op = resolve(o);
    if (!opts_valid(op) || !grid_valid(*g)) return HJR_EINVAL;
    *out = job_scratch_bytes(g, 1, op.dtype);
    return HJR_OK;
}

hjr_status hjr_solve_levels(const hjr_dyn* dyn, int32_t nlev, const hjr_grid* grids,
                            const void* const* l, const void* V0, const hjr_dstb* d, double tol,
                            const hjr_opts* o, void* const* V_levels, uint8_t* const* masks,
                            int64_t* mask_counts, hjr_stats* stats)
{
    return solve_levels_impl(dyn, nlev, grids, l, nullptr, V0, d, tol, o, V_levels, masks,
                             mask_counts, stats);
}

hjr_status hjr_solve_field(const hjr_dyn* dyn, int32_t nlev, const hjr_grid* grids,
                           const void* const* l, const void* const* dfield, const void* V0,
                           double tol, const hjr_opts* o, void* const* V_levels,
                           hjr_stats* stats)
{
    if (!dfield || nlev < 1 || nlev > 4) return HJR_EINVAL;
    for (int k = 0; k < nlev; k++)
        if (!dfield[k]) return HJR_EINVAL;
    return solve_levels_impl(dyn, nlev, grids, l, dfield, V0, nullptr, tol, o, V_levels,
                             nullptr, nullptr, stats);
}

hjr_status hjr_solve_local(const hjr_dyn* dyn, const hjr_grid* grid, const void* l, const void* V0,
                           const hjr_dstb* d, const void* dfield, const uint8_t* node_mask,
                           double tol, const hjr_opts* o, void* V_out, hjr_stats* stats)
{
    if (!grid || !l || !V_out || !node_mask) return HJR_EINVAL;
    const void* ls[1] = {l};
    void* vs[1] = {V_out};
    const void* fs[1] = {dfield};
    return solve_levels_impl(dyn, 1, grid, ls, dfield ? fs : nullptr, V0, d, tol, o, vs, nullptr,
                             nullptr, stats, node_mask);
}

hjr_status hjr_band_mask(const hjr_grid* g, const void* V, int32_t k, uint8_t* node_mask,
                         int64_t* count, const hjr_opts* o)
{
    const hjr_opts op = resolve(o);
    if (!g || !V || !node_mask || k < 0) return HJR_EINVAL;
    if (op.dtype != HJR_F32 && op.dtype != HJR_F64) return HJR_EINVAL;
    if (!grid_valid(*g)) return HJR_EINVAL;
    const int64_t N = grid_size(*g);
    hipStream_t s = (hipStream_t)op.stream;
    uint8_t* tmp = nullptr;
    uint64_t* dcount = nullptr;
    if (hipMalloc(&tmp, 2 * align256(N) + sizeof(uint64_t)) != hipSuccess) return HJR_ENOMEM;
    dcount = (uint64_t*)(tmp + 2 * align256(N));
    hjr_status st = HJR_OK;
    uint64_t h = 0;
    if (launch_band(s, op.dtype, *g, V, k, tmp, tmp + align256(N), node_mask) != hipSuccess)
        st = HJR_EDEVICE;
    if (st == HJR_OK && count &&
        (launch_fill_u64(s, dcount, 1, 0) != hipSuccess ||
         launch_tile_flags(s, node_mask, N, 256, nullptr, dcount) != hipSuccess ||
         hipMemcpyAsync(&h, dcount, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess))
        st = HJR_EDEVICE;
    // the scratch is freed once the stream has used it
    if (hipStreamSynchronize(s) != hipSuccess) st = HJR_EDEVICE;
    (void)hipFree(tmp);
    if (st == HJR_OK && count) *count = (int64_t)h;
    return st;
}

hjr_status hjr_solve_ex(const hjr_dyn* dyn, const hjr_grid* grid, const void* l, const void* V0,
                        const hjr_dstb* d, double tol, const hjr_opts* o, void* V_out,
                        hjr_stats* stats)
{
    if (!grid || !l || !V_out) return HJR_EINVAL;
    const void* ls[1] = {l};
    void* vs[1] = {V_out};
    return hjr_solve_levels(dyn, 1, grid, ls, V0, d, tol, o, vs, nullptr, nullptr, stats);
}

hjr_status hjr_solve(const hjr_dyn* dyn, const hjr_grid* grid, const void* l, const void* V0,
                     const hjr_dstb* d, double tol, const hjr_opts* o, void* V_out,
                     int64_t* iterations, double* residual)
{
    hjr_stats st;
    hjr_status r = hjr_solve_ex(dyn, grid, l, V0, d, tol, o, V_out, &st);
    if (r == HJR_OK || r == HJR_NOT_CONVERGED) {
        if (iterations) *iterations = st.iterations;
        if (residual) *residual = st.residual;
    }
    return r;
}

hjr_status hjr_solve_noalloc(const hjr_dyn* dyn, const hjr_grid* grid, const void* l,
                            const void* V0, const hjr_dstb* d, double tol, const hjr_opts* o,
                            void* V_out, hjr_stats* stats)
{
    const auto t_start = std::chrono::steady_clock::now();
    const hjr_opts op = resolve(o);
    if (!opts_valid(op)) return HJR_EINVAL;
    hjr_status st = check_job_spec(dyn, 1, grid, d, tol, op.band);
    if (st != HJR_OK) return st;
    if (!l || !V_out) return HJR_EINVAL;
    const int K = chunk_of(op);
    const int64_t N = grid_size(*grid);
    const int64_t n2 = grid->ndim >= 3 ? grid->n[2] : 1;
    const size_t tables = align256(Engine::table_bytes(1, K));
    const size_t need = tables + align256(N * elem_size(op.dtype)) +
                        align256(n2 * elem_size(op.dtype));
    if (need > (size_t)HJR_NOALLOC_SCRATCH_BYTES) return HJR_ENOMEM;
    if (Engine::host_bytes(1, K) > kNoallocHostBytes) return HJR_EINVAL;
    void* base = nullptr;
    if ((st = scratch_of_current_device(&base)) != HJR_OK) return st;
    alignas(256) char host_stage[kNoallocHostBytes];
    try {
        EngineCfg cfg;
        cfg.dtype = op.dtype;
        cfg.order = op.order;
        cfg.cfl = op.cfl;
        cfg.max_iter = op.max_iter;
        cfg.walk = op.walk;
        cfg.K = K;
        cfg.cap = 1;
        // graphs, pipelining and profiling need objects the static mode
        // does not create; the tile choice is kept
        cfg.flags = op.flags & HJR_FLAG_FLAT_TILES;
        Engine eng(cfg);
        if ((st = eng.init_static((hipStream_t)op.stream, base, host_stage)) != HJR_OK) return st;
        Job j;
        j.dyn = *dyn;
        std::memset(j.d, 0, sizeof(j.d));
        for (int c = 0; c < dyn_channels(dyn->kind); c++) j.d[c] = d[c];
        j.tol = tol;
        j.band = op.band;
        j.nlev = 1;
        j.lev[0].grid = *grid;
        j.lev[0].l = l;
        j.lev[0].V = V_out;
        j.lev[0].tile_rows = op.tile_rows;
        j.V0 = V0;
        j.Vhat = (char*)base + tables;
        j.table = (char*)j.Vhat + align256(N * elem_size(op.dtype));
        if ((st = eng.add(&j)) != HJR_OK) return st;
        if ((st = run_engine(eng)) != HJR_OK) return st;
        ProbState ps;
        if ((st = eng.read_state(j.slot, &ps)) != HJR_OK) return st;
        const double ms = std::chrono::duration<double, std::milli>(
                              std::chrono::steady_clock::now() - t_start).count();
        fill_stats(stats, j, ps, ms, eng);
        return (hjr_status)j.status;
    } catch (const std::bad_alloc&) {
        return HJR_ENOMEM;
    } catch (...) {
        return HJR_EDEVICE;
    }
}

hjr_status hjr_batch_workspace_bytes(int32_t n, const hjr_problem* probs, const hjr_opts* o,
                                     size_t* out)
{
    if (n < 1 || !probs || !out) return HJR_EINVAL;
    const hjr_opts op = resolve(o);
    if (!opts_valid(op)) return HJR_EINVAL;
    size_t b = 0;
    for (int i = 0; i < n; i++) {
        if (probs[i].nlev < 1 || probs[i].nlev > 4) return HJR_EINVAL;
        for (int k = 0; k < probs[i].nlev; k++)
            if (!grid_valid(probs[i].grids[k])) return HJR_EINVAL;
        b += job_scratch_bytes(probs[i].grids, probs[i].nlev, op.dtype);
    }
    *out = b;
    return HJR_OK;
}

hjr_status hjr_solve_batch(int32_t n, const hjr_problem* probs, const hjr_opts* o,
                           hjr_stats* results)
{
    const hjr_opts op = resolve(o);
    if (!opts_valid(op) || n < 1 || !probs) return HJR_EINVAL;
    for (int i = 0; i < n; i++) {
        const hjr_problem& p = probs[i];
        bool need_d = false;
        for (int k = 0; k < p.nlev && k < 4; k++) need_d = need_d || !p.dfield[k];
        hjr_status st = check_job_spec(&p.dyn, p.nlev, p.grids, p.d, p.tol, p.band, need_d);
        if (st != HJR_OK) return st;
        for (int k = 0; k < p.nlev; k++)
            if (!p.l[k] || !p.V[k] || p.order[k] < 0 || p.order[k] > 2) return HJR_EINVAL;
    }
    size_t need = 0;
    hjr_status st = hjr_batch_workspace_bytes(n, probs, &op, &need);
    if (st != HJR_OK) return st;
    const int K = chunk_of(op);
    try {
        EngineCfg cfg;
        cfg.dtype = op.dtype;
        cfg.order = op.order;
        cfg.cfl = op.cfl;
        cfg.max_iter = op.max_iter;
        cfg.walk = op.walk;
        cfg.K = K;
        cfg.cap = n;
        cfg.flags = op.flags;
        Session ses;
        if ((st = ses.open(op, cfg, need)) != HJR_OK) return st;
        Engine& eng = *ses.eng;
        std::vector<Job> jobs(n);
        char* p = ses.ws;
        for (int i = 0; i < n; i++) {
            const hjr_problem& pr = probs[i];
            Job& j = jobs[i];
            j.dyn = pr.dyn;
            std::memset(j.d, 0, sizeof(j.d));
            bool need_d = false;
            for (int k = 0; k < pr.nlev; k++) need_d = need_d || !pr.dfield[k];
            if (need_d)
                for (int c = 0; c < dyn_channels(pr.dyn.kind); c++) j.d[c] = pr.d[c];
            j.tol = pr.tol;
            j.band = pr.band;
            j.nlev = pr.nlev;
            int64_t Nmax = 0;
            for (int k = 0; k < pr.nlev; k++) {
                j.lev[k].grid = pr.grids[k];
                j.lev[k].l = pr.l[k];
                j.lev[k].V = pr.V[k];
                j.lev[k].mask = nullptr;
                j.lev[k].tile_rows = pr.tile_rows[k] > 0 ? pr.tile_rows[k] : op.tile_rows;
                j.lev[k].order = pr.order[k];
                j.lev[k].dfield = pr.dfield[k];
                Nmax = std::max(Nmax, grid_size(pr.grids[k]));
            }
            j.V0 = pr.V0;
            j.Vhat = p;
            j.table = p + align256(Nmax * elem_size(op.dtype));
            p += job_scratch_bytes(pr.grids, pr.nlev, op.dtype);
        }
        // every field is checked before any job starts (no output is written
        // when one is invalid)
        for (int i = 0; i < n; i++)
            if ((st = check_fields(eng, jobs[i])) != HJR_OK) {
                if (st == HJR_EINVAL) ses.clean = true;  // the engine is idle and intact
                return st;
            }
        for (int i = 0; i < n; i++)
            if ((st = eng.add(&jobs[i])) != HJR_OK) return st;
        if ((st = run_engine(eng)) != HJR_OK) return st;
        const double ms = ses.elapsed_ms();
        hjr_status all = HJR_OK;
        for (int i = 0; i < n; i++) {
            if (jobs[i].status != HJR_OK) all = (hjr_status)jobs[i].status;
            if (results) {
                ProbState ps;
                if ((st = eng.read_state(jobs[i].slot, &ps)) != HJR_OK) return st;
                fill_stats(&results[i], jobs[i], ps, ms, eng);
            }
        }
        ses.clean = true;
        return all;
    } catch (const std::bad_alloc&) {
        return HJR_ENOMEM;
    } catch (...) {
        return HJR_EDEVICE;
    }
}

namespace {

// Query arguments of one model and grid (state, value and control layouts
// left to the caller).
QueryArgs query_args(const hjr_dyn& dyn, const hjr_grid& grid, int order)
{
    QueryArgs A;
    std::memset(&A, 0, sizeof(A));
    A.kind = dyn.kind;
    A.ndim = grid.ndim;
    A.order = order;
    A.nctrl = dyn.kind == HJR_DI2X2 ? 2 : 1;
    int64_t st = 1;
    for (int a = grid.ndim - 1; a >= 0; a--) {
        A.n[a] = grid.n[a];
        A.stride[a] = st;
        st *= grid.n[a];
        A.lo[a] = grid.lo[a];
        A.hi[a] = grid.hi[a];
        A.h[a] = (grid.hi[a] - grid.lo[a]) / (double)(grid.n[a] - 1);
        A.hih[a] = 0.5 / A.h[a];
    }
    for (int i = 0; i < 16; i++) A.par[i] = dyn.p[i];
    return A;
}

bool query_opts_valid(const hjr_opts& op)
{
    return (op.dtype == HJR_F32 || op.dtype == HJR_F64) && (op.order == 1 || op.order == 2);
}

}  // namespace

hjr_status hjr_safety_query(const hjr_dyn* dyn, const hjr_grid* grid, const void* V,
                            const hjr_query* q, const hjr_opts* o)
{
    const hjr_opts op = resolve(o);
    if (!dyn || !grid || !q) return HJR_EINVAL;
    if (!query_opts_valid(op)) return HJR_EINVAL;
    if (!grid_valid(*grid) || !dyn_valid(*dyn, *grid)) return HJR_EINVAL;
    if (q->n < 0 || std::isnan(q->level)) return HJR_EINVAL;
    if (q->u_out && !q->u_perf) return HJR_EINVAL;
    if (q->n == 0) return HJR_OK;
    if (!q->x || !V) return HJR_EINVAL;
    QueryArgs A = query_args(*dyn, *grid, op.order);
    A.nq = q->n;
    A.x = q->x;
    A.x_stride = grid->ndim;
    for (int a = 0; a < 4; a++) A.x_map[a] = a;
    A.u_stride = A.nctrl;
    A.u_offset = 0;
    A.v_stride = 1;
    A.value = q->value;
    A.grad = q->grad;
    A.u_star = q->u_star;
    A.u_perf = q->u_perf;
    A.u_out = q->u_out;
    A.level = q->level;
    if (launch_query((hipStream_t)op.stream, op.dtype, A, V) != hipSuccess) return HJR_EDEVICE;
    return HJR_OK;
}

hjr_status hjr_safety_query_decomposed(int32_t nsub, const hjr_subsystem* subs,
                                       const hjr_query_decomposed* q, const hjr_opts* o)
{
    const hjr_opts op = resolve(o);
    if (nsub < 1 || nsub > 16 || !subs || !q) return HJR_EINVAL;
    if (!query_opts_valid(op)) return HJR_EINVAL;
    if (q->n < 0 || std::isnan(q->level)) return HJR_EINVAL;
    if (q->state_dim < 1 || q->control_dim < 0) return HJR_EINVAL;
    if (q->u_out && !q->u_perf) return HJR_EINVAL;
    uint32_t seen = 0;  // each full-state component belongs to one subsystem at most
    for (int s = 0; s < nsub; s++) {
        const hjr_subsystem& sb = subs[s];
        if (!grid_valid(sb.grid) || !dyn_valid(sb.dyn, sb.grid)) return HJR_EINVAL;
        for (int a = 0; a < sb.grid.ndim; a++) {
            const int c = sb.state_index[a];
            if (c < 0 || c >= q->state_dim || c >= 32 || (seen >> c & 1u)) return HJR_EINVAL;
            seen |= 1u << c;
        }
        const int m = sb.dyn.kind == HJR_DI2X2 ? 2 : 1;
        if (sb.control_index < 0 || sb.control_index + m > q->control_dim) return HJR_EINVAL;
        if (q->n > 0 && !sb.V) return HJR_EINVAL;
    }
    if (q->n == 0) return HJR_OK;
    if (!q->x || !q->sub_value) return HJR_EINVAL;
    hipStream_t st = (hipStream_t)op.stream;
    for (int s = 0; s < nsub; s++) {
        const hjr_subsystem& sb = subs[s];
        QueryArgs A = query_args(sb.dyn, sb.grid, op.order);
        A.nq = q->n;
        A.x = q->x;
        A.x_stride = q->state_dim;
        for (int a = 0; a < 4; a++) A.x_map[a] = a < sb.grid.ndim ? sb.state_index[a] : 0;
        A.u_stride = q->control_dim;
        A.u_offset = sb.control_index;
        A.v_stride = nsub;
        A.value = q->sub_value + s;
        A.grad = q->grad;
        A.u_star = q->u_star;
        A.u_perf = q->u_perf;
        A.u_out = q->u_out;
        A.level = q->level;
        if (launch_query(st, op.dtype, A, sb.V) != hipSuccess) return HJR_EDEVICE;
    }
    if (launch_query_min(st, q->sub_value, nsub, q->n, q->value, q->active) != hipSuccess)
        return HJR_EDEVICE;
    return HJR_OK;
}

hjr_status hjr_interp(const hjr_grid* src, const void* V_src, const hjr_grid* dst, void* V_dst,
                      const void* l_dst, const hjr_opts* o)
{
    const hjr_opts op = resolve(o);
    if (!src || !dst || !V_src || !V_dst) return HJR_EINVAL;
    if (op.dtype != HJR_F32 && op.dtype != HJR_F64) return HJR_EINVAL;
    if (!grid_valid(*src) || !grid_valid(*dst) || !same_box(*src, *dst)) return HJR_EINVAL;
    if (V_src == V_dst) return HJR_EINVAL;
    if (launch_interp((hipStream_t)op.stream, op.dtype, *src, V_src, *dst, V_dst, l_dst) != hipSuccess)
        return HJR_EDEVICE;
    return HJR_OK;
}

hjr_status hjr_refine_mask(const hjr_grid* g, const void* V, uint8_t* mask, int64_t* count,
                           const hjr_opts* o)
{
    const hjr_opts op = resolve(o);
    if (!g || !V || !mask) return HJR_EINVAL;
    if (op.dtype != HJR_F32 && op.dtype != HJR_F64) return HJR_EINVAL;
    if (!grid_valid(*g)) return HJR_EINVAL;
    hipStream_t s = (hipStream_t)op.stream;
    if (!count) {
        if (launch_mask(s, op.dtype, *g, V, mask, nullptr) != hipSuccess) return HJR_EDEVICE;
        return HJR_OK;
    }
    uint64_t* dcount = nullptr;
    if (hipMalloc(&dcount, sizeof(uint64_t)) != hipSuccess) return HJR_ENOMEM;
    hjr_status st = HJR_OK;
    uint64_t h = 0;
    if (launch_fill_u64(s, dcount, 1, 0) != hipSuccess ||
        launch_mask(s, op.dtype, *g, V, mask, dcount) != hipSuccess ||
        hipMemcpyAsync(&h, dcount, sizeof(uint64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        st = HJR_EDEVICE;
    (void)hipFree(dcount);
    if (st == HJR_OK) *count = (int64_t)h;
    return st;
}

}  // extern "C"
