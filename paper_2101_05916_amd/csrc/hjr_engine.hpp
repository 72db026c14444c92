// hjr_engine.hpp -- host runtime that drives the iteration kernels of libhjr.
//
// The engine keeps a device-resident table of up to `cap` problems ("slots")
// and advances every running problem by up to K RK2 steps per chunk.  A
// chunk is one stream-ordered sequence
//     [control upload] prologue, K x (stage 1, stage 2), epilogue, [residual download]
// optionally captured once per buffer parity as a hipGraph.  The host never
// waits inside a chunk: each kernel of step s reads the residual of step s-1
// on the device and skips problems that have already converged, so the host
// can keep one chunk in flight while it reads the residuals of the previous
// one, finishes levels, starts transitions and admits new problems.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <functional>
#include <vector>

#include "../../include/hjr.h"
#include "hjr_device.hpp"

namespace hjr {

struct EngineCfg {
    int dtype = HJR_F32;
    int order = 2;
    double cfl = 0.8;
    int64_t max_iter = 100000;
    int K = 32;        // iterations per chunk
    int cap = 1;       // problem slots
    int flags = 0;
    int grid = 0;      // workgroups per iteration kernel; 0 = from occupancy
    int walk = 0;      // hjr_opts.walk: 0 = automatic, -1 = none, k >= 1 = k planes
};

struct Level {
    hjr_grid grid;
    const void* l = nullptr;
    void* V = nullptr;
    uint8_t* mask = nullptr;  // optional refinement-mask output
    int tile_rows = 0;        // LDS tile height, 0 = default
    int order = 0;            // derivative order of this level, 0 = EngineCfg::order
    const void* dfield = nullptr;  // per-node disturbance boxes, or null (Job::d)
    const uint8_t* umask = nullptr; // localized update: the nodes to update, or null
    uint8_t* tmask = nullptr;       // scratch for its per-tile flags
    uint32_t* tlist = nullptr;      // scratch for the list of its plane tiles holding a node to update
    int64_t live_tiles = -1;        // length of that list once built (plane tiles), else -1
};

// One solve job: a chain of 1..4 grid levels of one subsystem.
struct Job {
    // specification
    hjr_dyn dyn;
    hjr_dstb d[2];
    double tol = 1e-4;
    double band = 0.0;         // residual band, 0 = every node
    int nlev = 1;
    Level lev[4];
    const void* V0 = nullptr;  // start of level 0 (nullptr = cold)
    void* Vhat = nullptr;      // scratch, >= max level size elements
    void* table = nullptr;     // scratch, >= max axis-2 length elements
    // progress (engine-owned)
    int slot = -1;
    int cur = 0;
    int64_t sched = 0;             // steps scheduled on the current level
    int64_t level_start_chunk = 0; // first chunk whose results count for `cur`
    bool fresh = true;             // next chunk is the first of this level
    bool done = false;
    int status = HJR_OK;
    int64_t level_iters[4] = {0, 0, 0, 0};
    double residual = 0.0;
    // user hook, called from the host thread when the job finishes
    std::function<void(Job&)> on_done;
};

class Engine {
public:
    explicit Engine(const EngineCfg& cfg);
    ~Engine();

    // Bytes of device memory the engine's tables take for cap slots.
    static size_t table_bytes(int cap, int K);

    // Bind to a stream (the engine enqueues everything there) and place the
    // tables in `arena` (table_bytes) or allocate them when arena is null.
    hjr_status init(hipStream_t stream, void* arena, void* host_arena = nullptr);

    // Bytes of host memory the engine's staging buffers take for cap slots.
    static size_t host_bytes(int cap, int K);

    // Static mode, for callers that cannot allocate: the device tables go to
    // dev_arena (table_bytes), the host staging buffers to host_arena
    // (host_bytes, ordinary memory), and the engine creates no stream, event
    // or graph and allocates no device or pinned memory; it runs without
    // graphs, profiling or pipelining, synchronising its stream after every
    // chunk.
    hjr_status init_static(hipStream_t stream, void* dev_arena, void* host_arena);

    // Make an idle engine ready for a new set of jobs: takes order, cfl and
    // max_iter from c (dtype, K, cap and flags must match the engine's).
    hjr_status reset(const EngineCfg& c);

    // Put a job into a free slot and enqueue its level-0 set-up.
    hjr_status add(Job* j);

    // Enqueue one chunk; when more than `depth` chunks are in flight, wait
    // for the oldest and process its residuals.  Returns an error status on
    // a device failure.
    hjr_status step();

    // Process every chunk in flight.
    hjr_status drain();

    bool busy() const { return running_ > 0; }
    int free_slots() const;
    int running() const { return running_; }

    // Number of nodes of a disturbance field (nch channels over N nodes, in
    // the engine's dtype) whose box is not a finite ordered pair (sync; the
    // engine must be idle).
    hjr_status check_field(const void* f, int nch, int64_t N, int64_t* bad);

    // Number of set bytes of a node mask of N nodes (sync; engine idle).
    hjr_status count_mask(const uint8_t* m, int64_t N, int64_t* count);

    // Copy the per-slot device state (alpha, dt) of a slot to *out (sync).
    hjr_status read_state(int slot, ProbState* out);
    // Mask counts of a job's levels (sync).
    hjr_status read_mask_counts(int slot, uint64_t* out4);

    // Summed device time (ms) and launch count of the stage-1 / stage-2
    // kernels, with HJR_FLAG_PROFILE.
    void profile(double ms[2], int64_t n[2], int64_t* cells) const
    {
        for (int i = 0; i < 2; i++) {
            ms[i] = prof_ms_[i];
            n[i] = prof_n_[i];
        }
        *cells = prof_cells_;
    }

    hipStream_t stream() const { return stream_; }
    const EngineCfg& cfg() const { return cfg_; }

private:
    struct Flight {
        int64_t chunk = 0;
        hipEvent_t ev = nullptr;    // completion event (none in static mode)
        bool timed = false;         // stage launches bracketed by events
        std::vector<Job*> job;      // per slot, job that ran (or null)
        std::vector<int> limit;     // per slot
        std::vector<int64_t> sched; // per slot, steps scheduled before this chunk
    };

    hjr_status setup_level(Job* j);
    hjr_status upload_table();
    hjr_status enqueue_chunk_body(int par, bool timed, bool fork);
    hjr_status enqueue_stage(int stage, const ChunkArgs& a, bool fork, hipEvent_t e0 = nullptr,
                             hipEvent_t e1 = nullptr);
    hjr_status build_graph(int par, hipGraphExec_t* out);
    hjr_status process(Flight& f);
    void finish_level(Job* j, int status, int64_t iters, double residual);
    // walk: axis-0 planes per walking tile for the problems that can take
    // them, 0 = plane tiles one by one
    void fill_desc(const Job* j, ProbDesc& P, int walk = 0) const;
    ChunkArgs args(int par, int slot) const;

    // Stage launches of the current chunk: family and workgroups per stage.
    struct Launch {
        int fam;
        int grid[2];
        bool deep[2] = {false, false};  // per stage: runs of tiles, deeper-pipelined kernel
        bool operator==(const Launch& o) const
        {
            return fam == o.fam && grid[0] == o.grid[0] && grid[1] == o.grid[1] &&
                   deep[0] == o.deep[0] && deep[1] == o.deep[1];
        }
    };

    EngineCfg cfg_;
    hipStream_t stream_ = nullptr;
    // side streams and events that let the launches of different families
    // in one stage run concurrently inside a captured graph (fork on
    // fork_ev_, join on join_ev_[f])
    hipStream_t side_[kNumFam] = {};
    hipEvent_t fork_ev_ = nullptr;
    hipEvent_t join_ev_[kNumFam] = {};
    int fam_grid_[2][kNumFam] = {};  // workgroup cap per stage and family (occupancy x CUs)
    int fam_grid_big_[kNumFam] = {};  // stage 2's cap when the family's values exceed HJR_BIG_SET_BYTES
    bool own_arena_ = false;
    bool static_ = false;  // init_static: nothing allocated, nothing created
    void* arena_ = nullptr;
    // device tables: problem descriptors, then the family order list (first
    // tile per position, slot per position)
    ProbDesc* d_desc_ = nullptr;
    int64_t* d_tb_ = nullptr;
    int32_t* d_ord_ = nullptr;
    size_t desc_bytes_ = 0;
    ProbState* d_state_ = nullptr;
    ChunkHdr* d_hdr_[2] = {nullptr, nullptr};
    ProbCtl* d_ctl_[2] = {nullptr, nullptr};
    uint64_t* d_res_[2] = {nullptr, nullptr};
    double* d_compact_[2] = {nullptr, nullptr};
    uint64_t* d_mask_counts_ = nullptr;  // [cap][4]
    uint64_t* d_check_ = nullptr;        // counter of check_field
    // pinned host mirrors (descriptors + order list, one copy)
    ProbDesc* h_desc_[2] = {nullptr, nullptr};
    hipEvent_t desc_ev_[2] = {nullptr, nullptr};
    int desc_par_ = 0;
    char* h_ctl_[2] = {nullptr, nullptr};      // ChunkHdr then cap x ProbCtl
    double* h_compact_[2] = {nullptr, nullptr};
    size_t ctl_bytes_ = 0;
    // graphs, per buffer parity and launch list
    std::vector<std::pair<std::vector<Launch>, hipGraphExec_t>> graphs_[2];
    bool use_graph_ = false;
    std::vector<Launch> launches_;  // stage launches of the current chunk
    int64_t fam_tile_[kNumFam + 1] = {};
    int64_t fam_nodes_[kNumFam] = {};  // nodes of the problems in the table, per family
    int32_t fam_pos_[kNumFam + 1] = {};
    // bookkeeping
    std::vector<Job*> slots_;
    int running_ = 0;
    bool table_dirty_ = true;
    int64_t total_tiles_ = 0;
    int64_t chunk_ = 0;
    std::vector<Flight> flights_;
    int depth_ = 1;
    hipError_t last_err_ = hipSuccess;
    // profiling: per parity, start/end events of every stage launch
    bool profile_ = false;
    std::vector<hipEvent_t> prof_ev_[2];
    double prof_ms_[2] = {0.0, 0.0};
    int64_t prof_n_[2] = {0, 0};
    int64_t prof_cells_ = 0;  // cell-updates done by the timed launches
};

// Helpers shared by the API layer and the server.
bool grid_valid(const hjr_grid& g);
int64_t grid_size(const hjr_grid& g);
int dyn_dim(int kind);
int dyn_channels(int kind);
bool dyn_valid(const hjr_dyn& d, const hjr_grid& g);
size_t elem_size(int dtype);
FastDiv make_fastdiv(uint32_t d);

}  // namespace hjr
