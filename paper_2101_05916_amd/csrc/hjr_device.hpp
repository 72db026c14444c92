// hjr_device.hpp -- data shared between the host engine and the HIP kernels
// of libhjr (layouts of the device-resident problem table, per-problem
// state, chunk control and residual buffers).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hjr.h"

namespace hjr {

constexpr int kBlock = 256;          // threads per workgroup of the utility kernels
// The RK-stage kernels run one wavefront per workgroup: a tile's LDS
// barriers then synchronise a single wave, and each CU interleaves ~20
// independent waves to hide memory latency.
#ifndef HJR_STAGE_BLOCK
#define HJR_STAGE_BLOCK 64
#endif
#ifndef HJR_PLANE_NODES_PT
#define HJR_PLANE_NODES_PT 8
#endif
#ifndef HJR_PLANE_LDS_ROWS
#define HJR_PLANE_LDS_ROWS 18        // LDS rows of a narrow plane block (tile rows + 4)
#endif
#ifndef HJR_NODE_UNROLL
#define HJR_NODE_UNROLL 2            // plain node loop (no pipeline): nodes per unrolled iteration
#endif
#ifndef HJR_NODE_PIPE
#define HJR_NODE_PIPE 3              // FP32 plane tiles, bit s-1 for stage s: request a node's operands before computing the previous one
#endif
#ifndef HJR_NODE_PIPE_DEPTH1
#define HJR_NODE_PIPE_DEPTH1 1       // nodes requested ahead of the one computed, stage 1
#endif
#ifndef HJR_NODE_PIPE_DEPTH2
#define HJR_NODE_PIPE_DEPTH2 1       // and stage 2
#endif
#ifndef HJR_NODE_PIPE_DEEP1
#define HJR_NODE_PIPE_DEEP1 5        // the same in the deep kernels of large tile sets, stage 1
#endif
#ifndef HJR_NODE_PIPE_DEEP2
#define HJR_NODE_PIPE_DEEP2 3        // and stage 2
#endif
#ifndef HJR_BLOCKS_PER_CU
#define HJR_BLOCKS_PER_CU 20         // cap on stage workgroups per CU (5 single-wave groups per SIMD)
#endif
#ifndef HJR_BLOCKS_PER_CU_S2
#define HJR_BLOCKS_PER_CU_S2 20      // cap for the FP32 stage-2 kernels (0: HJR_BLOCKS_PER_CU); the
#endif                               // 24 their registers allow measured up to 8 % slower per launch
#ifndef HJR_BLOCKS_PER_CU_S2_BIG
#define HJR_BLOCKS_PER_CU_S2_BIG 16  // cap for FP32 stage 2 when a family's values exceed
#endif                               // HJR_BIG_SET_BYTES or other families run beside it
#ifndef HJR_BIG_SET_BYTES
#define HJR_BIG_SET_BYTES (2ll << 30)
#endif
#ifndef HJR_BLOCKS_PER_CU_F64
#define HJR_BLOCKS_PER_CU_F64 14     // the same for the FP64 kernels (15, which their LDS
                                     // allows, measured 17-20 % slower)
#endif
#ifndef HJR_PLANE_BLOCK
#define HJR_PLANE_BLOCK 8            // 4-D plane tiles: axis-0 indices per block of the plane order
#endif
#ifndef HJR_TILES_PER_WG_MAX
#define HJR_TILES_PER_WG_MAX 16      // more tiles per workgroup of the capped grid: a workgroup per
#endif                               // run of HJR_TILES_PER_RUN tiles (0: always the capped grid)
#ifndef HJR_TILES_PER_RUN
#define HJR_TILES_PER_RUN 8
#endif
#ifndef HJR_RES_FILTER
#define HJR_RES_FILTER 1             // FP32 stage 2: exact residual only where the float one can raise the max
#endif
#ifndef HJR_STAGE_DMA
#define HJR_STAGE_DMA 3              // plane tiles staged by direct global-to-LDS loads: bit 0
#endif                               // stage 1, bit 1 stage 2 (else through registers)
#ifndef HJR_WAVES_PER_EU
#define HJR_WAVES_PER_EU 0           // occupancy hint for the stage kernels, 0 = none
#endif
constexpr int kStageBlock = HJR_STAGE_BLOCK;
#ifndef HJR_NODE_UNROLL1
#define HJR_NODE_UNROLL1 HJR_NODE_UNROLL
#endif
#ifndef HJR_NODE_UNROLL2
#define HJR_NODE_UNROLL2 HJR_NODE_UNROLL
#endif
constexpr int kNodeUnroll1 = HJR_NODE_UNROLL1;  // plane-tile node unroll, stage 1
constexpr int kNodeUnroll2 = HJR_NODE_UNROLL2;  // and stage 2
constexpr int kNodesPerThread = 512 / HJR_STAGE_BLOCK > 1 ? 512 / HJR_STAGE_BLOCK : 2;  // nodes per thread of a flat tile
constexpr int kTile = kStageBlock * kNodesPerThread;  // nodes per flat tile
constexpr int kResSubs = 64;         // residual atomics spread over 64 words
constexpr int kMaxChunk = 256;       // iterations per chunk, upper bound
constexpr int kProfileEvery = 8;     // HJR_FLAG_PROFILE times one chunk in this many

// Plane tiles: one workgroup stages the two fastest axes of a tile in LDS
// with a row stride fixed at compile time, so every in-plane neighbour is a
// constant LDS offset.  plane_elems(stride) bounds (rows + 4) * stride.
constexpr int kRowStrideS = 72;      // planes whose last axis has <= 68 nodes
constexpr int kRowStrideL = 208;     // planes whose last axis has <= 204 nodes
constexpr int kPlaneNodesPT = HJR_PLANE_NODES_PT;   // nodes per thread of a plane tile
constexpr int kPlaneStagePT = 2 * kPlaneNodesPT;    // staged elements per thread (register staging)
constexpr int kPlaneElemsS = HJR_PLANE_LDS_ROWS * kRowStrideS;  // LDS elements of a narrow block
constexpr int kPlaneElemsL = 8 * kRowStrideL;   // LDS elements of a wide block (<= 4 rows)
// LDS elements after a plane block for its row records (coefficient, index) of up to 16 rows
constexpr int kRowRecElems = 32;
static_assert(kPlaneElemsS / kRowStrideS - 4 <= kRowRecElems / 2 &&
                  kPlaneElemsL / kRowStrideL - 4 <= kRowRecElems / 2,
              "row records cover every tile row");
// Walking plane tiles: at most this many rows per tile (so the staged rows,
// tile rows + 4 halo rows, fit the prefetch registers) and columns (a lane
// per column).
constexpr int kWalkRows = 12;
constexpr int kWalkStageRows = kWalkRows + 4;
constexpr int kWalkMaxCols = 64;

enum TilePath : int32_t { kPathFlat = 0, kPathPlaneS = 1, kPathPlaneL = 2, kPathWalk = 3 };

// Tile families.  Every family has its own stage kernels, so registers and
// LDS are sized for its tile code alone; a chunk launches one kernel per
// family present.  Plane families are (model, row stride, ENO order), and
// (model, row stride) with ENO2 for problems with per-node disturbance
// bounds (the "F" families).  Plane problems without a family of their own
// (first-order derivatives with per-node bounds or on the 10-D model's
// x-subsystem) take flat tiles.
enum Family : int32_t {
    kFamFlat = 0,
    kFamZ2dS2, kFamZ2dL2, kFamX4dS2, kFamX4dL2,
    kFamZ2dS1, kFamZ2dL1, kFamX4dS1, kFamX4dL1,
    kFamZ2dS2F, kFamZ2dL2F, kFamX4dS2F, kFamX4dL2F,
    kFamXvS2, kFamXvL2, kFamXvS2F, kFamXvL2F,  // QUAD_X4DV
    kFamX4dW2, kFamX4dW1, kFamXvW2,            // walking tiles (narrow planes)
    kFamX4dMS2, kFamX4dML2,                    // localized updates (node mask), narrow / wide
    kNumFam
};

__host__ __device__ constexpr bool fam_masked(int f)
{
    return f == kFamX4dMS2 || f == kFamX4dML2;
}

__host__ __device__ constexpr bool fam_walk(int f)
{
    return f >= kFamX4dW2 && f <= kFamXvW2;
}

// Families with a second, deeper-pipelined FP32 stage kernel for launches
// whose workgroups take runs of tiles (the 4-D plane families with constant
// disturbance boxes).
__host__ __device__ constexpr bool fam_deep(int f)
{
    return f == kFamX4dS2 || f == kFamX4dL2 || f == kFamXvS2 || f == kFamXvL2;
}

// Model of a plane family (HJR_QUAD_Z2D, HJR_QUAD_X4D, HJR_QUAD_X4DV; -1 flat).
__host__ __device__ constexpr int fam_model(int f)
{
    return f == kFamFlat ? -1
         : f == kFamX4dW2 || f == kFamX4dW1 || fam_masked(f) ? HJR_QUAD_X4D
         : f == kFamXvW2 ? HJR_QUAD_X4DV
         : f >= kFamXvS2 ? HJR_QUAD_X4DV
         : (((f - 1) & 3) >= 2 ? HJR_QUAD_X4D : HJR_QUAD_Z2D);
}

// Narrow plane (row stride 72) or wide (208): within each group of four
// (Z2D S, Z2D L, X4D S, X4D L) and in the QUAD_X4DV group (S, L, S, L).
__host__ __device__ constexpr int fam_rs(int f)
{
    return f == kFamFlat ? 0
         : f == kFamX4dML2 ? kRowStrideL
         : f >= kFamX4dW2 ? kRowStrideS
         : (((f - 1) & 1) ? kRowStrideL : kRowStrideS);
}

__host__ __device__ constexpr int fam_order(int f)
{
    return ((f >= kFamZ2dS1 && f <= kFamX4dL1) || f == kFamX4dW1) ? 1 : 2;
}

__host__ __device__ constexpr bool fam_x4d(int f)  // a 4-D model
{
    return fam_model(f) == HJR_QUAD_X4D || fam_model(f) == HJR_QUAD_X4DV;
}

__host__ __device__ constexpr bool fam_field(int f)
{
    return (f >= kFamZ2dS2F && f <= kFamX4dL2F) || f == kFamXvS2F || f == kFamXvL2F;
}

// LDS elements of a plane block of row stride rs (0 for flat tiles).
__host__ __device__ constexpr int plane_elems(int rs)
{
    return rs == kRowStrideS ? kPlaneElemsS : rs == kRowStrideL ? kPlaneElemsL : 0;
}

// Whether plane tiles of RK stage `stage` stage their rows by direct
// global-to-LDS loads (else through registers, with a spare LDS slot per
// lane after the block).
__host__ __device__ constexpr bool stage_by_dma(int stage)
{
    return ((HJR_STAGE_DMA >> (stage - 1)) & 1) != 0;
}

// Division of a 31-bit unsigned index by a runtime divisor d >= 2 with one
// 32x32->hi multiply: q = mulhi(x, m) >> s, with s = ceil(log2 d) - 1 and
// m = ceil(2^(32+s) / d).  Exact for x < 2^31 (Granlund & Montgomery 1994,
// "Division by invariant integers using multiplication", with the shift
// reduced by one so that m fits 32 bits).
struct FastDiv {
    uint32_t d;
    uint32_t m;
    uint32_t s;
    uint32_t m20;  // ceil(2^20 / d): x / d = (x * m20) >> 20 for x * d < 2^20 (24-bit multiplies)
};

// Static description of one problem in the batch (written by the host).
struct ProbDesc {
    int32_t kind;
    int32_t ndim;
    int32_t order;
    int32_t path;            // TilePath
    int32_t n[4];
    int64_t N;
    int64_t stride[4];
    FastDiv div[4];          // divisors n[1..ndim-1] used to split a flat index
    // plane tiles: rows per tile along axis ndim-2, and chunks per plane
    int32_t rows;
    int32_t chunks;
    FastDiv div_chunks;      // divisor `chunks`
    FastDiv div_last;        // divisor n[ndim-1]
    double lo[4];
    double h[4];
    double hih[4];           // 0.5 / h
    float lo_f[4];
    float h_f[4];
    float hih_f[4];
    double hc_d[16];         // Hamiltonian constants with 0.5/h folded in (see hjr_stencil.hpp)
    float hc_f[16];
    double par[16];
    double dlo[2];
    double dhi[2];
    double tol;
    double band;             // residual counts nodes with |V| < band or |V'| < band (+inf = all)
    double cfl;
    void* V;                 // value, updated in place
    const void* l;           // constraint
    void* Vhat;              // stage-1 scratch
    void* table;             // per-axis lookup table (g tan(theta) for QUAD_X4D)
    const void* dfield;      // per-node disturbance boxes (channel, lower/upper, node), or null
    const uint8_t* umask;    // localized update: nodes to update (others keep their value), or null
    const uint8_t* tmask;    // with umask: per flat tile, whether it holds a node to update
    const uint32_t* tlist;   // with umask on plane tiles: the tiles holding a node to update
                             // (ntiles of them), in tile order
    int64_t tile_begin;      // first global tile of this problem
    int64_t ntiles;
    // walking plane tiles (4-D narrow planes, last axis <= 64 nodes): a
    // tile walks `walk` consecutive indices of axis 0 (0 = plane tiles one
    // by one); nseg = ceil(n[0] / walk)
    int32_t walk;
    int32_t nseg;
    int32_t wslab;           // axis-1 slabs per walking tile (1, or 2 when 2 (n[3] + 4) <= 72)
    int32_t ngroups;         // ceil(n[1] / wslab)
    FastDiv div_groups;      // divisor ngroups
    // 4-D plane tiles: order of the (i0, i1) planes, in blocks of bx
    // consecutive axis-0 indices (bx <= 1: i1 fastest); nblk = ceil(n[0] /
    // bx) blocks, the last one of bxl indices
    int32_t bx;
    int32_t nblk;
    int32_t bxl;
    float band_f;            // band rounded up to a float: for a float x, x >= band iff x >= band_f
    FastDiv div_bxn1;        // divisor bx * n[1]
    FastDiv div_bx;          // divisor bx
    FastDiv div_bxl;         // divisor bxl (when >= 2)
};

// The stage kernels address the tables they only read (problem descriptors,
// per-problem state, chunk header, control words and order list) in the
// constant address space: those loads become scalar loads, and everything
// derived from them is known to be uniform across a wave, so pointers and
// buffer resources stay in SGPRs.
#define HJR_CONST __attribute__((address_space(4)))
typedef const HJR_CONST ProbDesc PDesc;

// Family of a problem's tiles (its model, tile path, ENO order and whether
// it has a disturbance field); the host sends the problems without a plane
// family to flat tiles.
inline int family_of(const ProbDesc& P)
{
    if (P.path == kPathFlat) return kFamFlat;
    if (P.path == kPathWalk)
        return P.kind == HJR_QUAD_X4DV ? kFamXvW2 : (P.order == 1 ? kFamX4dW1 : kFamX4dW2);
    const bool narrow = P.path == kPathPlaneS;
    if (P.umask) return narrow ? kFamX4dMS2 : kFamX4dML2;  // 4-D model, ENO2, no field
    if (P.kind == HJR_QUAD_X4DV) return (P.dfield ? kFamXvS2F : kFamXvS2) + (narrow ? 0 : 1);
    const bool x4 = P.kind == HJR_QUAD_X4D;
    // first of the group Z2D S, Z2D L, X4D S, X4D L
    const int base = P.dfield ? kFamZ2dS2F : (P.order == 1 ? kFamZ2dS1 : kFamZ2dS2);
    return base + (x4 ? 2 : 0) + (narrow ? 0 : 1);
}

// Device-written per-problem quantities (once per level).
struct ProbState {
    uint64_t alpha_bits[4];  // max-reduction of |f_i| as IEEE bit patterns
    double alpha[4];
    double dt;
    double ah[4];            // alpha * 0.5 / h
    float ah_f[4];
    float dt_f;
    float pad_f[3];
    uint64_t mask_count;
    double pad[1];
};

typedef const HJR_CONST ProbState PState;

// Per-chunk header and per-problem control (written by the host each chunk).
// The tiles of family f are [fam_tile[f], fam_tile[f+1]); its problems sit at
// positions [fam_pos[f], fam_pos[f+1]) of the order list (ChunkArgs::ord),
// with first tiles ChunkArgs::tb, increasing.
struct ChunkHdr {
    int64_t total_tiles;
    int32_t nprob;
    int32_t pad;
    int64_t fam_tile[kNumFam + 1];
    int32_t fam_pos[kNumFam + 1];
    int32_t fam_run[2][kNumFam];  // per stage and family: consecutive tiles a workgroup takes at a time
};
constexpr int kHdrBytes = 512;  // device slot of the chunk header, before the ProbCtl array
static_assert(sizeof(ChunkHdr) <= kHdrBytes, "ChunkHdr must fit its slot");

struct ProbCtl {
    int32_t limit;   // iterations this problem may take in this chunk (0..K)
    int32_t fresh;   // 1 = first chunk of a level: no carried residual
};

// Kernel argument block for the iteration kernels.
struct ChunkArgs {
    const ProbDesc* probs;
    const int64_t* tb;   // first tile of the problem at each order position
    const int32_t* ord;  // problem slot at each order position
    ProbState* states;
    const ChunkHdr* hdr;
    const ProbCtl* ctl;
    uint64_t* res;       // [cap][K+1][kResSubs] residual bit patterns, this parity
    const double* prev;  // [cap][K] reduced residuals of the previous chunk
    double* compact;     // [cap][K] reduced residuals of this chunk (output)
    int32_t K;
    int32_t cap;
    int32_t slot;        // iteration index within the chunk
    int32_t pad;
};

__host__ __device__ inline int64_t res_index(int p, int s, int sub, int K)
{
    return ((int64_t)p * (K + 1) + s) * kResSubs + sub;
}

}  // namespace hjr
