// hjr_engine.cpp -- chunked, pipelined driver of the iteration kernels.
#include "hjr_engine.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "hjr_launch.hpp"

namespace hjr {

#define HJR_TRY(expr)                               \
    do {                                            \
        hipError_t e_ = (expr);                     \
        if (e_ != hipSuccess) {                     \
            last_err_ = e_;                         \
            return HJR_EDEVICE;                     \
        }                                           \
    } while (0)

// ------------------------------------------------------------------------
// helpers
// ------------------------------------------------------------------------

bool grid_valid(const hjr_grid& g)
{
    if (g.ndim < 1 || g.ndim > 4) return false;
    int64_t N = 1;
    for (int i = 0; i < g.ndim; i++) {
        if (g.n[i] < 3) return false;
        if (!(g.lo[i] < g.hi[i])) return false;
        if (!std::isfinite(g.lo[i]) || !std::isfinite(g.hi[i])) return false;
        N *= g.n[i];
        if (N > (int64_t(1) << 31) - 1) return false;  // flat indices are 31-bit
    }
    return true;
}

int64_t grid_size(const hjr_grid& g)
{
    int64_t N = 1;
    for (int i = 0; i < g.ndim; i++) N *= g.n[i];
    return N;
}

int dyn_dim(int kind)
{
    switch (kind) {
    case HJR_QUAD_Z2D: return 2;
    case HJR_QUAD_X4D: return 4;
    case HJR_QUAD_X4DV: return 4;
    case HJR_DI2X2: return 4;
    default: return 0;
    }
}

int dyn_channels(int kind)
{
    switch (kind) {
    case HJR_QUAD_Z2D: return 1;
    case HJR_QUAD_X4D: return 1;
    case HJR_QUAD_X4DV: return 1;
    case HJR_DI2X2: return 2;
    default: return 0;
    }
}

bool dyn_valid(const hjr_dyn& d, const hjr_grid& g)
{
    const int D = dyn_dim(d.kind);
    if (D == 0 || D != g.ndim) return false;
    for (int i = 0; i < 16; i++)
        if (!std::isfinite(d.p[i])) return false;
    if (d.kind == HJR_QUAD_Z2D && !(d.p[2] <= d.p[3])) return false;
    const bool x4 = d.kind == HJR_QUAD_X4D || d.kind == HJR_QUAD_X4DV;
    if (x4 && !(d.p[4] >= 0.0)) return false;
    if (x4) {
        // tan(theta) must stay finite on the grid
        const double half_pi = 1.5707963267948966;
        if (!(g.lo[2] > -half_pi && g.hi[2] < half_pi)) return false;
    }
    if (d.kind == HJR_DI2X2) {
        if (!(d.p[2] <= d.p[3]) || !(d.p[6] <= d.p[7])) return false;
        int seen = 0;
        for (int i = 8; i < 12; i++) {
            const double a = d.p[i];
            if (a != std::floor(a) || a < 0 || a > 3) return false;
            seen |= 1 << (int)a;
        }
        if (seen != 15) return false;
    }
    return true;
}

size_t elem_size(int dtype)
{
    return dtype == HJR_F64 ? sizeof(double) : sizeof(float);
}

FastDiv make_fastdiv(uint32_t d)
{
    FastDiv f{d, 0, 0, 0};
    if (d < 2) return f;  // never used: every axis has >= 3 nodes
    uint32_t l = 0;
    while ((uint64_t(1) << l) < d) l++;  // l = ceil(log2 d)
    const uint32_t s = l - 1;
    const uint64_t num = uint64_t(1) << (32 + s);
    f.m = (uint32_t)((num + d - 1) / d);
    f.s = s;
    f.m20 = d < (1u << 20) ? (uint32_t)(((1u << 20) + d - 1) / d) : 0;
    return f;
}

static size_t align256(size_t x)
{
    return (x + 255) & ~size_t(255);
}

// ------------------------------------------------------------------------
// Engine
// ------------------------------------------------------------------------

Engine::Engine(const EngineCfg& cfg) : cfg_(cfg)
{
    if (cfg_.K < 1) cfg_.K = 1;
    if (cfg_.K > kMaxChunk) cfg_.K = kMaxChunk;
    if (cfg_.cap < 1) cfg_.cap = 1;
    depth_ = (cfg_.flags & HJR_FLAG_NO_PIPELINE) ? 0 : 1;
    profile_ = (cfg_.flags & HJR_FLAG_PROFILE) != 0;
    use_graph_ = !(cfg_.flags & HJR_FLAG_NO_GRAPH) && !profile_;
}

Engine::~Engine()
{
    if (stream_) (void)hipStreamSynchronize(stream_);
    for (int f = 0; f < kNumFam; f++) {
        if (side_[f]) (void)hipStreamDestroy(side_[f]);
        if (join_ev_[f]) (void)hipEventDestroy(join_ev_[f]);
    }
    if (fork_ev_) (void)hipEventDestroy(fork_ev_);
    for (auto& f : flights_)
        if (f.ev) (void)hipEventDestroy(f.ev);
    for (int p = 0; p < 2; p++) {
        for (auto& g : graphs_[p]) (void)hipGraphExecDestroy(g.second);
        if (!static_) {
            if (h_desc_[p]) (void)hipHostFree(h_desc_[p]);
            if (h_ctl_[p]) (void)hipHostFree(h_ctl_[p]);
            if (h_compact_[p]) (void)hipHostFree(h_compact_[p]);
        }
        if (desc_ev_[p]) (void)hipEventDestroy(desc_ev_[p]);
        for (hipEvent_t e : prof_ev_[p]) (void)hipEventDestroy(e);
    }
    if (own_arena_ && arena_) (void)hipFree(arena_);
}

size_t Engine::table_bytes(int cap, int K)
{
    if (K > kMaxChunk) K = kMaxChunk;
    size_t b = 0;
    b += align256((sizeof(ProbDesc) + sizeof(int64_t) + sizeof(int32_t)) * cap);
    b += align256(sizeof(ProbState) * cap);
    b += 2 * align256(kHdrBytes + sizeof(ProbCtl) * cap);
    b += 2 * align256(sizeof(uint64_t) * (size_t)cap * (K + 1) * kResSubs);
    b += 2 * align256(sizeof(double) * (size_t)cap * K);
    b += align256(sizeof(uint64_t) * 4 * cap);
    b += align256(sizeof(uint64_t));  // field-check counter
    return b;
}

size_t Engine::host_bytes(int cap, int K)
{
    if (K > kMaxChunk) K = kMaxChunk;
    const size_t desc = (sizeof(ProbDesc) + sizeof(int64_t) + sizeof(int32_t)) * cap;
    return 2 * (align256(desc) + align256(kHdrBytes + sizeof(ProbCtl) * cap) +
                align256(sizeof(double) * (size_t)cap * K));
}

hjr_status Engine::init_static(hipStream_t stream, void* dev_arena, void* host_arena)
{
    if (!dev_arena || !host_arena) return HJR_EINVAL;
    static_ = true;
    depth_ = 0;
    profile_ = false;
    use_graph_ = false;
    return init(stream, dev_arena, host_arena);
}

hjr_status Engine::init(hipStream_t stream, void* arena, void* host_arena)
{
    stream_ = stream;
    const int cap = cfg_.cap, K = cfg_.K;
    const size_t tb = table_bytes(cap, K);
    if (!arena) {
        HJR_TRY(hipMalloc(&arena_, tb));
        own_arena_ = true;
    } else {
        arena_ = arena;
    }
    char* p = (char*)arena_;
    auto take = [&](size_t bytes) {
        char* r = p;
        p += align256(bytes);
        return (void*)r;
    };
    desc_bytes_ = (sizeof(ProbDesc) + sizeof(int64_t) + sizeof(int32_t)) * cap;
    d_desc_ = (ProbDesc*)take(desc_bytes_);
    d_tb_ = (int64_t*)(d_desc_ + cap);
    d_ord_ = (int32_t*)(d_tb_ + cap);
    d_state_ = (ProbState*)take(sizeof(ProbState) * cap);
    ctl_bytes_ = kHdrBytes + sizeof(ProbCtl) * cap;
    for (int q = 0; q < 2; q++) {
        d_hdr_[q] = (ChunkHdr*)take(ctl_bytes_);
        d_ctl_[q] = (ProbCtl*)((char*)d_hdr_[q] + kHdrBytes);
    }
    for (int q = 0; q < 2; q++) d_res_[q] = (uint64_t*)take(sizeof(uint64_t) * (size_t)cap * (K + 1) * kResSubs);
    for (int q = 0; q < 2; q++) d_compact_[q] = (double*)take(sizeof(double) * (size_t)cap * K);
    d_mask_counts_ = (uint64_t*)take(sizeof(uint64_t) * 4 * cap);
    d_check_ = (uint64_t*)take(sizeof(uint64_t));

    char* hp = (char*)host_arena;
    auto take_host = [&](size_t bytes) {
        char* r = hp;
        hp += align256(bytes);
        return (void*)r;
    };
    for (int q = 0; q < 2; q++) {
        if (static_) {
            // caller's host memory (pageable): every copy from or to it is
            // waited for before the host touches it again (depth 0)
            h_desc_[q] = (ProbDesc*)take_host(desc_bytes_);
            h_ctl_[q] = (char*)take_host(ctl_bytes_);
            h_compact_[q] = (double*)take_host(sizeof(double) * (size_t)cap * K);
        } else {
            HJR_TRY(hipHostMalloc((void**)&h_desc_[q], desc_bytes_, hipHostMallocDefault));
            HJR_TRY(hipHostMalloc((void**)&h_ctl_[q], ctl_bytes_, hipHostMallocDefault));
            HJR_TRY(hipHostMalloc((void**)&h_compact_[q], sizeof(double) * (size_t)cap * K,
                                  hipHostMallocDefault));
        }
        std::memset(h_desc_[q], 0, desc_bytes_);
        std::memset(h_ctl_[q], 0, ctl_bytes_);
        if (!static_) {
            HJR_TRY(hipEventCreateWithFlags(&desc_ev_[q], hipEventDisableTiming));
            HJR_TRY(hipEventRecord(desc_ev_[q], stream_));
        }
    }
    // zero the residual histories and mask counters once
    for (int q = 0; q < 2; q++)
        HJR_TRY(launch_fill_u64(stream_, (uint64_t*)d_compact_[q], (int64_t)cap * K, 0));
    HJR_TRY(launch_fill_u64(stream_, d_mask_counts_, 4 * (int64_t)cap, 0));

    int dev = 0, cus = 0;
    HJR_TRY(hipGetDevice(&dev));
    HJR_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    for (int st = 0; st < 2; st++)
        for (int f = 0; f < kNumFam; f++) {
            int g = cfg_.grid > 0 ? cfg_.grid : cus * stage_blocks_per_cu(cfg_.dtype, st + 1, f);
            fam_grid_[st][f] = std::max(8, (g + 7) / 8 * 8);
        }
    // FP32 stage 2 runs fewer workgroups per CU over a family whose V, V-hat
    // and l exceed HJR_BIG_SET_BYTES (batches of many large problems,
    // streamed from HBM: at full occupancy more tiles are in flight than the
    // caches serve well, up to 14 % slower per launch) and while other
    // families run beside it on the side streams (it would otherwise hold
    // every workgroup slot: served mixes of 2-D and 4-D instances measured
    // 10 % more updates/s with the cap); a lone family of a smaller set runs
    // at full occupancy, the faster choice there
    for (int f = 0; f < kNumFam; f++)
        fam_grid_big_[f] = cfg_.grid > 0 || cfg_.dtype != HJR_F32
                               ? fam_grid_[1][f]
                               : std::min(fam_grid_[1][f], cus * HJR_BLOCKS_PER_CU_S2_BIG);
    if (profile_)
        for (int q = 0; q < 2; q++) {
            prof_ev_[q].resize(4 * (size_t)K);
            for (auto& e : prof_ev_[q]) HJR_TRY(hipEventCreate(&e));
        }
    if (use_graph_) {
        HJR_TRY(hipEventCreateWithFlags(&fork_ev_, hipEventDisableTiming));
        for (int f = 0; f < kNumFam; f++) {
            HJR_TRY(hipStreamCreateWithFlags(&side_[f], hipStreamNonBlocking));
            HJR_TRY(hipEventCreateWithFlags(&join_ev_[f], hipEventDisableTiming));
        }
    }
    slots_.assign(cap, nullptr);
    table_dirty_ = true;
    return HJR_OK;
}

hjr_status Engine::reset(const EngineCfg& c)
{
    cfg_.order = c.order;
    cfg_.cfl = c.cfl;
    cfg_.max_iter = c.max_iter;
    cfg_.walk = c.walk;
    for (auto& f : flights_)
        if (f.ev) (void)hipEventDestroy(f.ev);
    flights_.clear();
    slots_.assign(cfg_.cap, nullptr);
    running_ = 0;
    table_dirty_ = true;
    prof_ms_[0] = prof_ms_[1] = 0.0;
    prof_n_[0] = prof_n_[1] = 0;
    prof_cells_ = 0;
    chunk_ = 0;  // profiling samples chunks 0, kProfileEvery, ... of every call
    HJR_TRY(launch_fill_u64(stream_, d_mask_counts_, 4 * (int64_t)cfg_.cap, 0));
    return HJR_OK;
}

hjr_status Engine::check_field(const void* f, int nch, int64_t N, int64_t* bad)
{
    uint64_t h = 0;
    HJR_TRY(launch_fill_u64(stream_, d_check_, 1, 0));
    HJR_TRY(launch_field_check(stream_, cfg_.dtype, f, nch, N, d_check_));
    HJR_TRY(hipMemcpyAsync(&h, d_check_, sizeof(h), hipMemcpyDeviceToHost, stream_));
    HJR_TRY(hipStreamSynchronize(stream_));
    *bad = (int64_t)h;
    return HJR_OK;
}

hjr_status Engine::count_mask(const uint8_t* m, int64_t N, int64_t* count)
{
    uint64_t h = 0;
    HJR_TRY(launch_fill_u64(stream_, d_check_, 1, 0));
    HJR_TRY(launch_tile_flags(stream_, m, N, 256, nullptr, d_check_));  // count only
    HJR_TRY(hipMemcpyAsync(&h, d_check_, sizeof(h), hipMemcpyDeviceToHost, stream_));
    HJR_TRY(hipStreamSynchronize(stream_));
    *count = (int64_t)h;
    return HJR_OK;
}

int Engine::free_slots() const
{
    int n = 0;
    for (auto* j : slots_) n += (j == nullptr);
    return n;
}

void Engine::fill_desc(const Job* j, ProbDesc& P, int walk) const
{
    std::memset(&P, 0, sizeof(P));
    const Level& L = j->lev[j->cur];
    const hjr_grid& g = L.grid;
    P.kind = j->dyn.kind;
    P.ndim = g.ndim;
    P.order = L.order > 0 ? L.order : cfg_.order;
    int64_t st = 1;
    for (int a = g.ndim - 1; a >= 0; a--) {
        P.n[a] = g.n[a];
        P.stride[a] = st;
        st *= g.n[a];
        P.div[a] = make_fastdiv((uint32_t)g.n[a]);
        P.lo[a] = g.lo[a];
        P.h[a] = (g.hi[a] - g.lo[a]) / (double)(g.n[a] - 1);
    }
    P.N = st;
    for (int i = 0; i < 16; i++) P.par[i] = j->dyn.p[i];
    for (int c = 0; c < 2; c++) {
        P.dlo[c] = j->d[c].lo;
        P.dhi[c] = j->d[c].hi;
    }
    P.tol = j->tol;
    P.band = j->band > 0.0 ? j->band : HUGE_VAL;
    {
        float bf = (float)P.band;
        if ((double)bf < P.band) bf = std::nextafter(bf, HUGE_VALF);
        P.band_f = bf;
    }
    P.cfl = cfg_.cfl;
    P.V = L.V;
    P.l = L.l;
    P.Vhat = j->Vhat;
    P.table = j->table;
    P.dfield = L.dfield;
    P.umask = L.umask;
    P.tmask = L.tmask;
    P.tlist = L.tlist;
    const int D = g.ndim;
    for (int a = 0; a < D; a++) {
        P.hih[a] = 0.5 / P.h[a];
        P.lo_f[a] = (float)P.lo[a];
        P.h_f[a] = (float)P.h[a];
        P.hih_f[a] = (float)P.hih[a];
    }
    // Hamiltonian constants with the 0.5/h factors folded in
    double* hc = P.hc_d;
    const double* p = P.par;
    if (P.kind == HJR_QUAD_Z2D) {
        const double ku_lo = p[0] * p[2], ku_hi = p[0] * p[3];
        const double dl = std::min(P.dlo[0], P.dhi[0]), dh = std::max(P.dlo[0], P.dhi[0]);
        hc[0] = P.hih[0] * P.lo[1];
        hc[1] = P.hih[0] * P.h[1];
        hc[2] = (std::max(ku_lo, ku_hi) + dl - p[1]) * P.hih[1];
        hc[3] = (std::min(ku_lo, ku_hi) + dh - p[1]) * P.hih[1];
        // with a per-node disturbance box the bound is added at the node
        hc[4] = (std::max(ku_lo, ku_hi) - p[1]) * P.hih[1];
        hc[5] = (std::min(ku_lo, ku_hi) - p[1]) * P.hih[1];
        hc[6] = P.hih[1];
    } else if (P.kind == HJR_QUAD_X4D || P.kind == HJR_QUAD_X4DV) {
        const double g_ = p[0], d1 = p[1], d0 = p[2], n0 = p[3], sm = p[4];
        // the disturbance enters x' (QUAD_X4D) or vx' (QUAD_X4DV)
        const double hd = P.kind == HJR_QUAD_X4DV ? P.hih[1] : P.hih[0];
        hc[0] = P.hih[0] * P.lo[1];
        hc[1] = P.hih[0] * P.h[1];
        hc[2] = P.dlo[0] * hd;
        hc[3] = P.dhi[0] * hd;
        hc[4] = P.hih[2] * (P.lo[3] - d1 * P.lo[2]);
        hc[5] = P.hih[2] * P.h[3];
        hc[6] = P.hih[2] * d1 * P.h[2];
        hc[7] = d0 * P.hih[3] * P.lo[2];
        hc[8] = d0 * P.hih[3] * P.h[2];
        hc[9] = n0 * sm * P.hih[3];
        hc[10] = hd;  // scales a per-node disturbance bound
        (void)g_;
    }
    for (int i = 0; i < 16; i++) P.hc_f[i] = (float)P.hc_d[i];
    // tile shape: LDS plane tiles over the two fastest axes when they fit,
    // else flat tiles of kTile consecutive nodes
    P.path = kPathFlat;
    P.ntiles = (P.N + kTile - 1) / kTile;
    // (per-node disturbance boxes and QUAD_X4DV have plane families for ENO2
    // only; localized updates have masked plane families for the 4-D
    // x-subsystem with ENO2 and constant bounds, and run on flat tiles
    // otherwise)
    const bool plane_kind =
        (P.kind == HJR_QUAD_Z2D || P.kind == HJR_QUAD_X4D || P.kind == HJR_QUAD_X4DV) &&
        !(cfg_.flags & HJR_FLAG_FLAT_TILES) &&
        !((P.dfield || P.kind == HJR_QUAD_X4DV) && P.order != 2) &&
        !(P.umask && (P.kind != HJR_QUAD_X4D || D != 4 || P.order != 2 || P.dfield));
    // plane tiles address with 32-bit byte offsets
    const bool fits32 = (double)P.N * (double)elem_size(cfg_.dtype) < 4294967296.0;
    if (plane_kind && fits32 && (D == 2 || D == 4)) {
        const int nr = g.n[D - 2], nc = g.n[D - 1];
        int rs = 0;
        if (nc + 4 <= kRowStrideS) {
            rs = kRowStrideS;
            P.path = kPathPlaneS;
        } else if (nc + 4 <= kRowStrideL) {
            rs = kRowStrideL;
            P.path = kPathPlaneL;
        }
        if (rs) {
            // walking tiles: 4-D models without per-node bounds on narrow
            // planes of at most kWalkMaxCols columns
            const bool walks = walk > 0 && D == 4 && rs == kRowStrideS && nc <= kWalkMaxCols &&
                               !P.dfield && !P.umask && P.kind != HJR_DI2X2;
            // rows per tile: at most kPlaneNodesPT nodes per thread, and the
            // LDS block within plane_elems
            int want = std::min(plane_elems(rs) / rs - 4, kPlaneNodesPT * kStageBlock / nc);
            // (a walking tile holds a column per lane, not nodes per thread)
            if (walks) want = std::min(plane_elems(rs) / rs - 4, kWalkRows);
            if (L.tile_rows > 0) want = std::min(want, L.tile_rows);
            want = std::max(want, 1);
            const int chunks = (nr + want - 1) / want;
            P.rows = (nr + chunks - 1) / chunks;
            P.chunks = chunks;
            P.div_chunks = make_fastdiv((uint32_t)std::max(chunks, 2));
            P.div_last = make_fastdiv((uint32_t)nc);
            int64_t outer = 1;
            for (int a = 0; a < D - 2; a++) outer *= g.n[a];
            P.ntiles = outer * chunks;
            // planes in blocks of bx consecutive axis-0 indices
            if (D == 4 && !walks && HJR_PLANE_BLOCK > 1 && g.n[0] > 1) {
                const int bx = std::min<int>(HJR_PLANE_BLOCK, g.n[0]);
                P.bx = bx;
                P.nblk = (g.n[0] + bx - 1) / bx;
                P.bxl = g.n[0] - (P.nblk - 1) * bx;
                P.div_bxn1 = make_fastdiv((uint32_t)(bx * g.n[1]));
                P.div_bx = make_fastdiv((uint32_t)bx);
                P.div_bxl = make_fastdiv((uint32_t)std::max(P.bxl, 2));
            }
            if (walks) {
                const int w = std::min(walk, g.n[0]);
                P.walk = w;
                P.nseg = (g.n[0] + w - 1) / w;
                // two axis-1 slabs side by side in a workgroup's lanes and LDS
                // rows when both fit
                P.wslab = (2 * nc <= kStageBlock && 2 * (nc + 4) <= rs) ? 2 : 1;
                P.ngroups = (g.n[1] + P.wslab - 1) / P.wslab;
                P.div_groups = make_fastdiv((uint32_t)std::max(P.ngroups, 2));
                P.ntiles = (int64_t)P.ngroups * chunks * P.nseg;
                P.path = kPathWalk;
            }
            // a localized update on plane tiles runs over the list of its
            // live tiles once the level setup has built it
            if (P.umask && L.live_tiles >= 0) P.ntiles = L.live_tiles;
        }
    }
}

hjr_status Engine::setup_level(Job* j)
{
    j->lev[j->cur].live_tiles = -1;
    const Level& L = j->lev[j->cur];
    ProbDesc P;
    fill_desc(j, P);
    if (j->cur == 0) {
        HJR_TRY(launch_init(stream_, cfg_.dtype, L.V, L.l, j->V0, P.N));
    } else {
        const Level& prev = j->lev[j->cur - 1];
        HJR_TRY(launch_interp(stream_, cfg_.dtype, prev.grid, prev.V, L.grid, L.V, L.l));
    }
    HJR_TRY(launch_level_setup(stream_, cfg_.dtype, P, &d_state_[j->slot]));
    if (L.umask) {
        // nodes outside the mask keep V, so stage 2 reads Vhat = V there
        HJR_TRY(launch_copy(stream_, cfg_.dtype, L.V, j->Vhat, P.N));
        if (P.path == kPathFlat) {
            HJR_TRY(launch_tile_flags(stream_, L.umask, P.N, kTile, L.tmask, nullptr));
        } else {
            // flags per plane tile, then the list of the live ones (built on
            // the host: once per level, a few hundred KB at 61^4)
            HJR_TRY(launch_plane_tile_flags(stream_, P, L.umask, L.tmask));
            std::vector<uint8_t> flags((size_t)P.ntiles);
            HJR_TRY(hipMemcpyAsync(flags.data(), L.tmask, flags.size(), hipMemcpyDeviceToHost, stream_));
            HJR_TRY(hipStreamSynchronize(stream_));
            std::vector<uint32_t> list;
            list.reserve(flags.size());
            for (size_t t = 0; t < flags.size(); t++)
                if (flags[t]) list.push_back((uint32_t)t);
            if (!list.empty()) {
                HJR_TRY(hipMemcpyAsync(L.tlist, list.data(), list.size() * sizeof(uint32_t),
                                       hipMemcpyHostToDevice, stream_));
                HJR_TRY(hipStreamSynchronize(stream_));
            }
            j->lev[j->cur].live_tiles = (int64_t)list.size();
        }
    }
    j->sched = 0;
    j->fresh = true;
    j->level_start_chunk = chunk_;
    table_dirty_ = true;
    return HJR_OK;
}

hjr_status Engine::add(Job* j)
{
    int s = -1;
    for (int i = 0; i < cfg_.cap; i++)
        if (!slots_[i]) {
            s = i;
            break;
        }
    if (s < 0) return HJR_EBUSY;
    slots_[s] = j;
    j->slot = s;
    j->cur = 0;
    j->done = false;
    j->status = HJR_OK;
    for (int k = 0; k < 4; k++) j->level_iters[k] = 0;
    running_++;
    HJR_TRY(launch_fill_u64(stream_, d_mask_counts_ + 4 * (int64_t)s, 4, 0));
    return setup_level(j);
}

hjr_status Engine::upload_table()
{
    const int q = desc_par_;
    desc_par_ ^= 1;
    if (desc_ev_[q]) HJR_TRY(hipEventSynchronize(desc_ev_[q]));  // staging q no longer being read
    const int cap = cfg_.cap;
    ProbDesc* h = h_desc_[q];
    int64_t* tb = (int64_t*)(h + cap);
    int32_t* ord = (int32_t*)(tb + cap);
    std::vector<int> fam_of(cap, -1);
    // Walking tiles only on request (walk >= 1): on the FP32 stage kernels
    // they measured slower than the plane tiles for every narrow-plane size
    // tried, the one-column-per-lane mapping leaving lanes idle when the last
    // axis has 33..63 nodes.
    const int walk = cfg_.walk > 0 ? cfg_.walk : 0;
    for (int s = 0; s < cap; s++) {
        Job* j = slots_[s];
        if (j && !j->done) {
            fill_desc(j, h[s], walk);
            if (h[s].ntiles > 0) fam_of[s] = family_of(h[s]);
        } else {
            std::memset(&h[s], 0, sizeof(ProbDesc));
            h[s].tol = 1.0;
            h[s].ntiles = 0;
        }
    }
    // tiles grouped by family, problems in slot order within a family
    int64_t total = 0;
    int pos = 0;
    for (int f = 0; f < kNumFam; f++) {
        fam_tile_[f] = total;
        fam_pos_[f] = pos;
        fam_nodes_[f] = 0;
        for (int s = 0; s < cap; s++) {
            if (fam_of[s] != f) continue;
            h[s].tile_begin = total;
            tb[pos] = total;
            ord[pos] = s;
            pos++;
            total += h[s].ntiles;
            fam_nodes_[f] += h[s].N;
        }
    }
    fam_tile_[kNumFam] = total;
    fam_pos_[kNumFam] = pos;
    total_tiles_ = total;
    HJR_TRY(hipMemcpyAsync(d_desc_, h, desc_bytes_, hipMemcpyHostToDevice, stream_));
    if (desc_ev_[q]) HJR_TRY(hipEventRecord(desc_ev_[q], stream_));
    table_dirty_ = false;
    return HJR_OK;
}

ChunkArgs Engine::args(int par, int slot) const
{
    ChunkArgs a;
    a.probs = d_desc_;
    a.tb = d_tb_;
    a.ord = d_ord_;
    a.states = d_state_;
    a.hdr = d_hdr_[par];
    a.ctl = d_ctl_[par];
    a.res = d_res_[par];
    a.prev = d_compact_[par ^ 1];
    a.compact = d_compact_[par];
    a.K = cfg_.K;
    a.cap = cfg_.cap;
    a.slot = slot;
    a.pad = 0;
    return a;
}

// One RK stage: a launch per family present.  With `fork` (graph capture)
// the second and later families go to side streams that fork from and join
// back into the engine stream, so the captured graph runs them as parallel
// branches; the first family stays on the engine stream.
hjr_status Engine::enqueue_stage(int stage, const ChunkArgs& a, bool fork, hipEvent_t e0, hipEvent_t e1)
{
    const int n = (int)launches_.size();
    if (!fork || n < 2) {
        // e0 / e1 (timed chunks) stamp the first kernel's start and the last one's end
        for (int i = 0; i < n; i++) {
            const Launch& l = launches_[i];
            HJR_TRY(launch_stage(stream_, cfg_.dtype, stage, l.fam, a, l.grid[stage - 1],
                                 i == 0 ? e0 : nullptr, i == n - 1 ? e1 : nullptr, l.deep[stage - 1]));
        }
        return HJR_OK;
    }
    HJR_TRY(hipEventRecord(fork_ev_, stream_));
    for (int i = 1; i < n; i++) {
        const Launch& l = launches_[i];
        HJR_TRY(hipStreamWaitEvent(side_[l.fam], fork_ev_, 0));
        HJR_TRY(launch_stage(side_[l.fam], cfg_.dtype, stage, l.fam, a, l.grid[stage - 1], nullptr,
                             nullptr, l.deep[stage - 1]));
        HJR_TRY(hipEventRecord(join_ev_[l.fam], side_[l.fam]));
    }
    HJR_TRY(launch_stage(stream_, cfg_.dtype, stage, launches_[0].fam, a, launches_[0].grid[stage - 1],
                         nullptr, nullptr, launches_[0].deep[stage - 1]));
    for (int i = 1; i < n; i++) HJR_TRY(hipStreamWaitEvent(stream_, join_ev_[launches_[i].fam], 0));
    return HJR_OK;
}

hjr_status Engine::enqueue_chunk_body(int par, bool timed, bool fork)
{
    HJR_TRY(launch_prologue(stream_, args(par, 0)));
    for (int s = 0; s < cfg_.K; s++) {
        const ChunkArgs a = args(par, s);
        for (int stage = 1; stage <= 2; stage++) {
            hipEvent_t e0 = timed ? prof_ev_[par][4 * s + 2 * (stage - 1)] : nullptr;
            hipEvent_t e1 = timed ? prof_ev_[par][4 * s + 2 * (stage - 1) + 1] : nullptr;
            hjr_status st = enqueue_stage(stage, a, fork && !timed, e0, e1);
            if (st != HJR_OK) return st;
        }
    }
    HJR_TRY(launch_epilogue(stream_, args(par, 0)));
    return HJR_OK;
}

hjr_status Engine::build_graph(int par, hipGraphExec_t* out)
{
    hipGraph_t g = nullptr;
    HJR_TRY(hipStreamBeginCapture(stream_, hipStreamCaptureModeThreadLocal));
    hjr_status st = enqueue_chunk_body(par, false, true);
    hipError_t e = hipStreamEndCapture(stream_, &g);
    if (st != HJR_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    HJR_TRY(e);
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HJR_TRY(e);
    return HJR_OK;
}

hjr_status Engine::step()
{
    if (table_dirty_) {
        hjr_status st = upload_table();
        if (st != HJR_OK) return st;
    }
    const int par = (int)(chunk_ & 1);
    const int cap = cfg_.cap, K = cfg_.K;
    Flight f;
    f.chunk = chunk_;
    f.job.assign(cap, nullptr);
    f.limit.assign(cap, 0);
    f.sched.assign(cap, 0);
    ChunkHdr* hdr = (ChunkHdr*)h_ctl_[par];
    ProbCtl* ctl = (ProbCtl*)(h_ctl_[par] + kHdrBytes);
    hdr->total_tiles = total_tiles_;
    hdr->nprob = cap;
    for (int f = 0; f <= kNumFam; f++) {
        hdr->fam_tile[f] = fam_tile_[f];
        hdr->fam_pos[f] = fam_pos_[f];
    }
    for (int st = 0; st < 2; st++)
        for (int f = 0; f < kNumFam; f++) hdr->fam_run[st][f] = 1;
    for (int s = 0; s < cap; s++) {
        Job* j = slots_[s];
        ctl[s].limit = 0;
        ctl[s].fresh = 1;
        if (j && !j->done && j->level_start_chunk <= chunk_) {
            const int64_t left = cfg_.max_iter - j->sched;
            const int lim = (int)std::max<int64_t>(0, std::min<int64_t>(K, left));
            ctl[s].limit = lim;
            ctl[s].fresh = j->fresh ? 1 : 0;
            f.job[s] = j;
            f.limit[s] = lim;
            f.sched[s] = j->sched;
            j->sched += lim;
            j->fresh = false;
        }
    }
    bool any = false;
    for (int s = 0; s < cap; s++) any = any || f.limit[s] > 0;
    if (!any && !flights_.empty()) {
        // nothing can advance until the chunk in flight is read back (its
        // problems hit max_iter or start a new level there)
        Flight g = std::move(flights_.front());
        flights_.erase(flights_.begin());
        return process(g);
    }
    // one launch per family present, with no more workgroups than it has
    // tiles (a multiple of 8, so that every XCD gets its share)
    launches_.clear();
    int nfam = 0;  // families launched side by side in this chunk
    for (int fm = 0; fm < kNumFam; fm++) nfam += fam_tile_[fm + 1] > fam_tile_[fm];
    for (int fm = 0; fm < kNumFam; fm++) {
        const int64_t nt = fam_tile_[fm + 1] - fam_tile_[fm];
        if (nt <= 0) continue;
        Launch l;
        l.fam = fm;
        const int64_t set_bytes = fam_nodes_[fm] * 3 * (cfg_.dtype == HJR_F64 ? 8 : 4);
        const bool capped = set_bytes > HJR_BIG_SET_BYTES || nfam > 1;
        for (int st = 0; st < 2; st++) {
            int cap = st == 1 && capped ? fam_grid_big_[fm] : fam_grid_[st][fm];
            // A capped grid strides through the tiles; over many tiles per
            // workgroup its workgroups drift apart, the tiles in flight on an
            // XCD no longer lie together, and the neighbour planes they read
            // miss L2 (the 121 4-D problems of the 256-problem mix: 4.6x the
            // algorithmic reads in stage 1).  There every tile gets its own
            // workgroup: the dispatcher starts them in order, so the tiles in
            // flight stay a compact window (1.7x).
            // (Workgroups take runs of HJR_TILES_PER_RUN consecutive tiles,
            // so that the per-workgroup setup -- problem lookup, convergence
            // vote, residual flush -- is shared by several tiles.)
            int run = 1;
            if (cfg_.grid <= 0 && HJR_TILES_PER_WG_MAX > 0 && nt > (int64_t)cap * HJR_TILES_PER_WG_MAX) {
                run = HJR_TILES_PER_RUN;
                const int64_t per_xcd = (nt + 7) / 8;
                cap = (int)std::min<int64_t>(INT32_MAX / 16, (per_xcd + run - 1) / run) * 8;
            }
            hdr->fam_run[st][fm] = run;
            l.deep[st] = run > 1;
            l.grid[st] = (int)std::min<int64_t>(cap, std::max<int64_t>(8, (nt + 7) / 8 * 8));
        }
        launches_.push_back(l);
    }
    HJR_TRY(hipMemcpyAsync(d_hdr_[par], h_ctl_[par], ctl_bytes_, hipMemcpyHostToDevice, stream_));
    if (use_graph_) {
        hipGraphExec_t ge = nullptr;
        for (auto& g : graphs_[par])
            if (g.first == launches_) ge = g.second;
        if (!ge) {
            hjr_status st = build_graph(par, &ge);
            if (st != HJR_OK) return st;
            graphs_[par].push_back({launches_, ge});
        }
        HJR_TRY(hipGraphLaunch(ge, stream_));
    } else {
        // with HJR_FLAG_PROFILE one chunk in kProfileEvery is timed launch by
        // launch: events between kernels cost throughput, so the sample keeps
        // the rest of the run undisturbed
        f.timed = profile_ && (chunk_ % kProfileEvery == 0);
        hjr_status st = enqueue_chunk_body(par, f.timed, false);
        if (st != HJR_OK) return st;
    }
    HJR_TRY(hipMemcpyAsync(h_compact_[par], d_compact_[par], sizeof(double) * (size_t)cap * K,
                           hipMemcpyDeviceToHost, stream_));
    if (!static_) {
        HJR_TRY(hipEventCreateWithFlags(&f.ev, hipEventDisableTiming));
        HJR_TRY(hipEventRecord(f.ev, stream_));
    }  // (static mode: depth 0, process() synchronises the stream instead)
    flights_.push_back(std::move(f));
    chunk_++;
    while ((int)flights_.size() > depth_) {
        Flight g = std::move(flights_.front());
        flights_.erase(flights_.begin());
        hjr_status st = process(g);
        if (st != HJR_OK) return st;
    }
    return HJR_OK;
}

hjr_status Engine::drain()
{
    while (!flights_.empty()) {
        Flight g = std::move(flights_.front());
        flights_.erase(flights_.begin());
        hjr_status st = process(g);
        if (st != HJR_OK) return st;
    }
    return HJR_OK;
}

hjr_status Engine::process(Flight& f)
{
    hipError_t e = f.ev ? hipEventSynchronize(f.ev) : hipStreamSynchronize(stream_);
    if (f.ev) (void)hipEventDestroy(f.ev);
    f.ev = nullptr;
    if (e != hipSuccess) {
        last_err_ = e;
        return HJR_EDEVICE;
    }
    const int par = (int)(f.chunk & 1);
    const double* r = h_compact_[par];
    const int K = cfg_.K;
    std::vector<int> hits(cfg_.cap, -1);
    int steps_live = 0;  // steps of this chunk in which some problem did work
    for (int s = 0; s < cfg_.cap; s++) {
        Job* j = f.job[s];
        const int lim = f.limit[s];
        if (!j || j->done || lim == 0) continue;
        if (j->slot != s || j->level_start_chunk > f.chunk) continue;  // stale results
        const double* rs = r + (int64_t)s * K;
        for (int k = 0; k < lim; k++)
            if (rs[k] < j->tol) {
                hits[s] = k;
                break;
            }
        steps_live = std::max(steps_live, hits[s] >= 0 ? hits[s] + 1 : lim);
    }
    if (f.timed)  // the skipped look-ahead steps past every stop are not counted
        for (int s = 0; s < steps_live; s++)
            for (int st = 0; st < 2; st++) {
                float ms = 0.f;
                HJR_TRY(hipEventElapsedTime(&ms, prof_ev_[par][4 * s + 2 * st],
                                            prof_ev_[par][4 * s + 2 * st + 1]));
                prof_ms_[st] += ms;
                prof_n_[st] += 1;
            }
    for (int s = 0; s < cfg_.cap; s++) {
        Job* j = f.job[s];
        const int lim = f.limit[s];
        if (!j || j->done || lim == 0) continue;
        if (j->slot != s || j->level_start_chunk > f.chunk) continue;  // stale results
        const double* rs = r + (int64_t)s * K;
        const int hit = hits[s];
        if (f.timed) prof_cells_ += grid_size(j->lev[j->cur].grid) * (hit >= 0 ? hit + 1 : lim);
        if (hit >= 0) {
            finish_level(j, HJR_OK, f.sched[s] + hit + 1, rs[hit]);
        } else if (f.sched[s] + lim >= cfg_.max_iter) {
            finish_level(j, HJR_NOT_CONVERGED, f.sched[s] + lim, rs[lim - 1]);
        }
    }
    return HJR_OK;
}

void Engine::finish_level(Job* j, int status, int64_t iters, double residual)
{
    const int c = j->cur;
    j->level_iters[c] = iters;
    j->residual = residual;
    const Level& L = j->lev[c];
    if (L.mask) {
        hipError_t e = launch_mask(stream_, cfg_.dtype, L.grid, L.V, L.mask,
                                   d_mask_counts_ + 4 * (int64_t)j->slot + c);
        if (e != hipSuccess) {
            last_err_ = e;
            status = HJR_EDEVICE;
        }
    }
    if (status == HJR_OK && c + 1 < j->nlev) {
        j->cur = c + 1;
        if (setup_level(j) == HJR_OK) return;
        status = HJR_EDEVICE;
    }
    j->status = status;
    j->done = true;
    slots_[j->slot] = nullptr;
    // later chunks still in flight must not look at this job again (its
    // owner may release it from on_done)
    for (auto& f : flights_)
        for (auto& q : f.job)
            if (q == j) q = nullptr;
    running_--;
    table_dirty_ = true;
    if (j->on_done) j->on_done(*j);
}

hjr_status Engine::read_state(int slot, ProbState* out)
{
    HJR_TRY(hipMemcpyAsync(out, d_state_ + slot, sizeof(ProbState), hipMemcpyDeviceToHost, stream_));
    HJR_TRY(hipStreamSynchronize(stream_));
    return HJR_OK;
}

hjr_status Engine::read_mask_counts(int slot, uint64_t* out4)
{
    HJR_TRY(hipMemcpyAsync(out4, d_mask_counts_ + 4 * (int64_t)slot, 4 * sizeof(uint64_t),
                           hipMemcpyDeviceToHost, stream_));
    HJR_TRY(hipStreamSynchronize(stream_));
    return HJR_OK;
}

}  // namespace hjr
