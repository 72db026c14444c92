// hjr_launch.hpp -- host-side launchers of the libhjr HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/hjr.h"
#include "hjr_device.hpp"

namespace hjr {

// Iteration kernels (one chunk = prologue, K x (stage 1, stage 2), epilogue).
hipError_t launch_prologue(hipStream_t s, const ChunkArgs& a);
// One RK stage over the tiles of family fam (see Family).
// e0 / e1, when given, are stamped at the kernel's start / end.  deep: the
// workgroups take runs of tiles (a large set), so the family's deeper-
// pipelined FP32 kernel runs where it has one.
hipError_t launch_stage(hipStream_t s, int dtype, int stage, int fam, const ChunkArgs& a, int grid,
                        hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr, bool deep = false);
hipError_t launch_epilogue(hipStream_t s, const ChunkArgs& a);

// Per-level set-up of one problem: Lax-Friedrichs bounds, time step and
// lookup table, written to *st.
hipError_t launch_level_setup(hipStream_t s, int dtype, const ProbDesc& P, ProbState* st);

// V = l (V0 == NULL) or V = min(l, V0); V0 may equal V.
hipError_t launch_init(hipStream_t s, int dtype, void* V, const void* l, const void* V0,
                       int64_t N);

// Multilinear transfer between two grids over the same box (see hjr_interp).
hipError_t launch_interp(hipStream_t s, int dtype, const hjr_grid& src, const void* Vs,
                         const hjr_grid& dst, void* Vd, const void* l_dst);

// Straddle mask of a level; adds the number of marked cells to *counter.
hipError_t launch_mask(hipStream_t s, int dtype, const hjr_grid& g, const void* V,
                       uint8_t* mask, uint64_t* counter);

// Count the nodes of a disturbance field (nch channels of N lower then N
// upper bounds) whose pair is not finite and ordered; adds to *counter.
hipError_t launch_field_check(hipStream_t s, int dtype, const void* f, int nch, int64_t N,
                              uint64_t* counter);

// Localized updates: per flat tile of `tile` nodes, whether umask sets one
// of its nodes (*count += set nodes; count nullable); the band of a warm
// start (nodes within k cells of a cell straddling V = 0; tmp0 and tmp1 are
// scratch of N bytes each); a plain copy of N elements.
hipError_t launch_tile_flags(hipStream_t s, const uint8_t* umask, int64_t N, int tile,
                             uint8_t* tmask, uint64_t* count);
// The same per plane tile of a 4-D problem on plane tiles (P.ntiles flags).
hipError_t launch_plane_tile_flags(hipStream_t s, const ProbDesc& P, const uint8_t* umask, uint8_t* tmask);
hipError_t launch_band(hipStream_t s, int dtype, const hjr_grid& g, const void* V, int k,
                       uint8_t* tmp0, uint8_t* tmp1, uint8_t* node_mask);
hipError_t launch_copy(hipStream_t s, int dtype, const void* src, void* dst, int64_t N);

// Fill n 64-bit words with value.
hipError_t launch_fill_u64(hipStream_t s, uint64_t* p, int64_t n, uint64_t value);

// Safety queries (hjr_query.hip): per state, the interpolated value and
// gradient of a converged V, the optimal safety control and the filtered
// control.
struct QueryArgs {
    int32_t kind;
    int32_t ndim;
    int32_t order;
    int32_t nctrl;           // control inputs of the model
    int32_t n[4];
    int64_t stride[4];
    double lo[4];
    double hi[4];
    double h[4];
    double hih[4];           // 0.5 / h
    double par[16];
    int64_t nq;              // states
    // state i's axis a is x[i * x_stride + x_map[a]]; its gradient goes to
    // the same place of grad
    const double* x;
    int32_t x_stride;
    int32_t x_map[4];
    int32_t u_stride;        // controls of state i start at i * u_stride + u_offset
    int32_t u_offset;
    int32_t pad;
    int64_t v_stride;        // value of state i at value[i * v_stride]
    double* value;           // or null
    double* grad;            // or null
    double* u_star;          // or null
    const double* u_perf;    // or null
    double* u_out;           // or null (needs u_perf)
    double level;
};
hipError_t launch_query(hipStream_t s, int dtype, const QueryArgs& A, const void* V);

// Decomposed value: value[i] = min over s of sub[i * nsub + s] (NaN if any is
// NaN), active[i] = the first s attaining it (-1 then); active may be null.
hipError_t launch_query_min(hipStream_t s, const double* sub, int32_t nsub, int64_t n,
                            double* value, int32_t* active);

// Workgroups of a stage kernel that fit on one compute unit.
int stage_blocks_per_cu(int dtype, int stage, int fam);

}  // namespace hjr
