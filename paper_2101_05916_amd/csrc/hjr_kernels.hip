// hjr_kernels.hip -- CDNA4 (gfx950) kernels of libhjr.
//
// The hot path is the time-marched solve of the HJI variational inequality
// (paper Sec. II-A, eq. (2)) with ENO2 upwind derivatives, global
// Lax-Friedrichs dissipation and a two-stage TVD Runge-Kutta step, followed
// by the projection V <- min(l, V).  Each RK stage is one sweep over the
// grid; it is a memory-bound cross-shaped stencil (9 points in 2-D, 17 in
// 4-D), so it runs on the vector ALUs with coalesced loads, not on MFMA.
//
// Work decomposition: every problem of a batch is cut into tiles (plane
// tiles: a few rows of the plane of the two fastest axes; flat tiles: kTile
// consecutive nodes); the tiles of all problems form one index space.
// Workgroup b runs on XCD b mod 8, and each XCD takes one contiguous eighth
// of the tile space, so the planes a tile's stencil touches are mostly in
// that XCD's L2.  A grid capped at a few workgroups per CU strides through
// the tiles; when that would be many tiles per workgroup the host launches
// one workgroup per tile instead, which keeps the tiles in flight on an XCD
// together (a striding grid drifts apart over a long run).
//
// Convergence is decided on the device: stage 2 max-reduces |V' - V| per
// workgroup (wave shuffles, then LDS) and folds it into the problem's
// residual word with one 64-bit atomic max on the IEEE bit pattern (a
// non-negative double orders like its bits).  Every kernel of iteration s
// first reads the residual of iteration s-1 and skips the problem if it is
// already below tol, so a chunk of K iterations can be enqueued blind and
// still stops at exactly the right step.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cmath>

#include "hjr_device.hpp"
#include "hjr_launch.hpp"
#include "hjr_stencil.hpp"

namespace hjr {

// ------------------------------------------------------------------------
// small helpers
// ------------------------------------------------------------------------

__device__ __forceinline__ double bitsd(uint64_t b)
{
    return __longlong_as_double((long long)b);
}

// Max of a 64-bit value over the workgroup; result valid in every thread.
template <int NB>
__device__ uint64_t block_max_u64(uint64_t v, uint64_t* red)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        uint64_t o = __shfl_xor(v, off, 64);
        v = umax64(v, o);
    }
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    uint64_t r = red[0];
#pragma unroll
    for (int i = 1; i < NB / 64; i++) r = umax64(r, red[i]);
    return r;
}

// Order position owning tile t among positions [lo, hi) of a family: the
// last one whose first tile is <= t (first tiles increase along the order).
__device__ __forceinline__ int find_pos(const HJR_CONST int64_t* tb, int lo, int hi, int64_t t)
{
    hi -= 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tb[mid] <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Whether problem p still iterates at this step: within its step limit for
// the chunk, and the previous step's residual (the max of its kResSubs
// words) not yet below tol.  The max is below tol exactly when every word
// is (the words are bit patterns of non-negative doubles or NaN, whose
// unsigned order is their order as doubles), so each lane of the wave tests
// one word and a wave vote decides: one coalesced load, no reduction.
__device__ __forceinline__ bool prob_active(const ChunkArgs& A, int p)
{
    static_assert(kResSubs == 64 && kStageBlock == 64, "one residual word per lane of the wave");
    if (A.slot >= ((const HJR_CONST ProbCtl*)A.ctl)[p].limit) return false;
    const uint64_t r = A.res[res_index(p, A.slot, (int)(threadIdx.x & 63), A.K)];
    return __any(!(bitsd(r) < ((PDesc*)A.probs)[p].tol));
}

// The residual word of problem p at this step that this workgroup folds into.
__device__ __forceinline__ unsigned long long* residual_word(const ChunkArgs& A, int p)
{
    return (unsigned long long*)&A.res[res_index(p, A.slot + 1, blockIdx.x % kResSubs, A.K)];
}

// Fold a workgroup's max |V' - V| into problem p's residual of this step.
// The residual is spread over kResSubs words (the reader takes their max),
// and the atomic is skipped when the word already held at least this value
// when read (`seen`, read as the workgroup began the problem's tiles, so
// that the read's latency overlaps them) -- the words only grow, so a stale
// read can only cause a redundant atomic, never a lost one.  Few workgroups
// beat the running max, so the device-scope atomics on any one word stay few.
template <int NB>
__device__ __forceinline__ void flush_residual(const ChunkArgs& A, int p, uint64_t rmax, uint64_t* red,
                                               uint64_t seen)
{
    const uint64_t r = block_max_u64<NB>(rmax, red);
    if (threadIdx.x == 0 && r > seen) atomicMax(residual_word(A, p), (unsigned long long)r);
}

// Occupancy hint per stage (0 = none): asks the compiler to fit the stage
// kernels in the registers of that many waves per SIMD.
#ifndef HJR_WAVES_PER_EU1
#define HJR_WAVES_PER_EU1 HJR_WAVES_PER_EU
#endif
#ifndef HJR_WAVES_PER_EU2
#define HJR_WAVES_PER_EU2 HJR_WAVES_PER_EU
#endif
// The hint applies to the FP32 kernels only (FP64 tiles need the registers).
#define HJR_STAGE_ATTR                                                                      \
    __attribute__((amdgpu_waves_per_eu(                                                     \
        sizeof(T) != 4 ? 1                                                                  \
        : STAGE == 1   ? (HJR_WAVES_PER_EU1 > 0 ? HJR_WAVES_PER_EU1 : 1)                    \
                       : (HJR_WAVES_PER_EU2 > 0 ? HJR_WAVES_PER_EU2 : 1),                   \
        8)))

// One RK stage over the tiles of family FAM.  The family's tiles are split
// into eight contiguous ranges, one per XCD (workgroup b runs on XCD b mod
// 8), and the workgroups of an XCD stride through its range (one tile each
// when the grid has a workgroup per tile).
template <typename T, int STAGE, int FAM, bool DEEP = false>
__global__ __launch_bounds__(kStageBlock) HJR_STAGE_ATTR void k_stage(ChunkArgs A)
{
    // a plane block (and a spare slot per lane for staging through registers),
    // then the tile's row records
    constexpr int kElems = FAM == kFamFlat ? 4
                                           : plane_elems(fam_rs(FAM)) + (stage_by_dma(STAGE) ? 0 : kStageBlock) +
                                                 kRowRecElems;
    __shared__ uint64_t red[kStageBlock / 64];
    __shared__ __align__(16) char smem[kElems * sizeof(T)];
    T* lds = (T*)smem;
    const HJR_CONST ChunkHdr* hdr = (const HJR_CONST ChunkHdr*)A.hdr;
    const HJR_CONST int64_t* tb = (const HJR_CONST int64_t*)A.tb;
    const HJR_CONST int32_t* ord = (const HJR_CONST int32_t*)A.ord;
    PDesc* probs = (PDesc*)A.probs;
    PState* states = (PState*)A.states;
    const int pb = hdr->fam_pos[FAM], pe = hdr->fam_pos[FAM + 1];
    if (pb >= pe) return;
    const int64_t t0 = hdr->fam_tile[FAM], t1 = hdr->fam_tile[FAM + 1];
    const int64_t total = t1 - t0;
    const int G8 = (int)gridDim.x >> 3;
    const int xcd = (int)blockIdx.x & 7;
    const int local = (int)blockIdx.x >> 3;
    const int64_t beg = t0 + total * xcd / 8, end = t0 + total * (xcd + 1) / 8;
    const int run = hdr->fam_run[STAGE - 1][FAM];  // consecutive tiles per turn (>= 1)
    int cur = -1;
    int64_t lo = 0, hi = 0;  // tile range of the current problem
    bool active = false;
    uint64_t rmax = 0, seen = 0;
    for (int64_t r0 = beg + (int64_t)local * run; r0 < end; r0 += (int64_t)G8 * run) {
        const int64_t r1 = r0 + run < end ? r0 + run : end;
        for (int64_t t = r0; t < r1; t++) {
            if (t >= hi || t < lo) {
                const int pos = find_pos(tb, pb, pe, t);
                if (STAGE == 2 && cur >= 0 && active) flush_residual<kStageBlock>(A, cur, rmax, red, seen);
                cur = ord[pos];
                lo = tb[pos];
                hi = pos + 1 < pe ? tb[pos + 1] : t1;
                rmax = 0;
                active = prob_active(A, cur);
                if (STAGE == 2 && active) seen = __atomic_load_n(residual_word(A, cur), __ATOMIC_RELAXED);
            }
            if (!active) continue;
            rmax = umax64(rmax, run_tile<T, STAGE, FAM, DEEP>(probs[cur], states[cur], (uint32_t)(t - lo), lds, rmax));
        }
    }
    if (STAGE == 2 && cur >= 0 && active) flush_residual<kStageBlock>(A, cur, rmax, red, seen);
}

// Chunk prologue: one workgroup per problem slot.  Slot 0 of the residual
// buffer receives the carried-in residual (+inf on the first chunk of a
// level, else the last residual of the previous chunk); slots 1..K are
// cleared for this chunk's atomics.
__global__ __launch_bounds__(64) void k_prologue(ChunkArgs A)
{
    const int p = blockIdx.x;
    if (p >= A.hdr->nprob) return;
    const uint64_t inf_bits = 0x7ff0000000000000ull;
    const uint64_t carried =
        A.ctl[p].fresh ? inf_bits : dbits(A.prev[(int64_t)p * A.K + (A.K - 1)]);
    const int64_t n = (int64_t)(A.K + 1) * kResSubs;
    uint64_t* r = A.res + (int64_t)p * n;
    for (int64_t e = threadIdx.x; e < n; e += blockDim.x) r[e] = (e == 0) ? carried : 0ull;
}

// Chunk epilogue: reduce the kResSubs words of every iteration.
__global__ __launch_bounds__(64) void k_epilogue(ChunkArgs A)
{
    const int p = blockIdx.x;
    if (p >= A.hdr->nprob) return;
    for (int s = threadIdx.x; s < A.K; s += blockDim.x) {
        uint64_t r = 0;
        for (int k = 0; k < kResSubs; k++) r = umax64(r, A.res[res_index(p, s + 1, k, A.K)]);
        A.compact[(int64_t)p * A.K + s] = bitsd(r);
    }
}

// ------------------------------------------------------------------------
// per-level set-up: Lax-Friedrichs bounds, dt, lookup table
// ------------------------------------------------------------------------

// f_i at node x for control vertex vu and disturbance vertex vd of the box
// [dl[c], dh[c]] per channel, in double.
__device__ void dyn_f(const ProbDesc& P, const double* x, int vu, int vd, const double* dl,
                      const double* dh, double* f)
{
    const double* p = P.par;
    switch (P.kind) {
    case HJR_QUAD_Z2D: {
        const double u = (vu & 1) ? p[3] : p[2];
        const double d = (vd & 1) ? dh[0] : dl[0];
        f[0] = x[1];
        f[1] = p[0] * u - p[1] + d;
        break;
    }
    case HJR_QUAD_X4D:
    case HJR_QUAD_X4DV: {
        const double S = (vu & 1) ? p[4] : -p[4];
        const double d = (vd & 1) ? dh[0] : dl[0];
        const bool vdist = P.kind == HJR_QUAD_X4DV;  // disturbance on vx' instead of x'
        f[0] = x[1] + (vdist ? 0.0 : d);
        f[1] = p[0] * tan(x[2]) + (vdist ? d : 0.0);
        f[2] = -p[1] * x[2] + x[3];
        f[3] = -p[2] * x[2] + p[3] * S;
        break;
    }
    case HJR_DI2X2: {
        const int za = (int)p[8], va = (int)p[9], zb = (int)p[10], vb = (int)p[11];
        const double ua = (vu & 1) ? p[3] : p[2];
        const double ub = (vu & 2) ? p[7] : p[6];
        const double da = (vd & 1) ? dh[0] : dl[0];
        const double db = (vd & 2) ? dh[1] : dl[1];
        f[za] = x[va];
        f[va] = p[0] * ua - p[1] + da;
        f[zb] = x[vb];
        f[vb] = p[4] * ub - p[5] + db;
        break;
    }
    default:
        f[0] = f[1] = f[2] = f[3] = 0.0;
    }
}

// alpha_i = max over nodes and over the vertices of the control box and of
// the node's disturbance box (the constant one, or the field's) of |f_i|.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_alpha(ProbDesc P, ProbState* st)
{
    __shared__ uint64_t red[kBlock / 64];
    const int D = P.ndim;
    const int nu = (P.kind == HJR_DI2X2) ? 4 : 2;
    const int nd = (P.kind == HJR_DI2X2) ? 4 : 2;
    const int nch = (P.kind == HJR_DI2X2) ? 2 : 1;
    const T* fld = (const T*)P.dfield;
    uint64_t m[4] = {0, 0, 0, 0};
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < P.N;
         idx += (int64_t)gridDim.x * blockDim.x) {
        double x[4] = {0, 0, 0, 0};
        int64_t q = idx;
        for (int a = D - 1; a >= 0; a--) {
            const int j = (int)(q % P.n[a]);
            q /= P.n[a];
            x[a] = P.lo[a] + (double)j * P.h[a];
        }
        double dl[2] = {P.dlo[0], P.dlo[1]}, dh[2] = {P.dhi[0], P.dhi[1]};
        if (fld) {
            for (int c = 0; c < nch; c++) {
                dl[c] = (double)fld[(int64_t)(2 * c) * P.N + idx];
                dh[c] = (double)fld[(int64_t)(2 * c + 1) * P.N + idx];
            }
        }
        for (int vu = 0; vu < nu; vu++)
            for (int vd = 0; vd < nd; vd++) {
                double f[4] = {0, 0, 0, 0};
                dyn_f(P, x, vu, vd, dl, dh, f);
                for (int a = 0; a < D; a++) m[a] = umax64(m[a], dbits(fabs(f[a])));
            }
    }
    for (int a = 0; a < D; a++) {
        const uint64_t r = block_max_u64<kBlock>(m[a], red);
        if (threadIdx.x == 0) atomicMax((unsigned long long*)&st->alpha_bits[a], (unsigned long long)r);
    }
}

// dt = cfl / sum_a alpha_a / h_a, the Lax-Friedrichs coefficients
// alpha_a * 0.5 / h_a in both precisions, and for QUAD_X4D the table
// g tan(theta_j) * 0.5 / h_1 over the nodes of axis 2.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_finalize(ProbDesc P, ProbState* st)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double s = 0.0;
        for (int a = 0; a < 4; a++) {
            const double al = a < P.ndim ? bitsd(st->alpha_bits[a]) : 0.0;
            st->alpha[a] = al;
            if (a < P.ndim) s += al / P.h[a];
            st->ah[a] = a < P.ndim ? al * P.hih[a] : 0.0;
            st->ah_f[a] = (float)st->ah[a];
        }
        st->dt = P.cfl / s;
        st->dt_f = (float)st->dt;
    }
    if ((P.kind == HJR_QUAD_X4D || P.kind == HJR_QUAD_X4DV) && P.table) {
        T* tab = (T*)P.table;
        for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < P.n[2]; j += gridDim.x * blockDim.x)
            tab[j] = (T)(P.par[0] * tan(P.lo[2] + (double)j * P.h[2]) * P.hih[1]);
    }
}

__global__ void k_zero_state(ProbState* st)
{
    if (threadIdx.x < 4) st->alpha_bits[threadIdx.x] = 0;
    if (threadIdx.x == 0) st->mask_count = 0;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_init(T* V, const T* l, const T* V0, int64_t N)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        const T lv = l[i];
        if (V0) {
            const T v0 = V0[i];
            V[i] = (lv < v0) ? lv : v0;
        } else {
            V[i] = lv;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_fill_u64(uint64_t* p, int64_t n, uint64_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Number of entries of a disturbance field (nch channels, N nodes, lower
// bounds then upper bounds per channel) whose pair is not two finite numbers
// with lower <= upper, added to *counter.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_field_check(const T* f, int nch, int64_t N,
                                                        unsigned long long* counter)
{
    __shared__ unsigned long long cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    unsigned long long bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)nch * N;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = i / N, k = i - c * N;
        const double lo = (double)f[2 * c * N + k], hi = (double)f[(2 * c + 1) * N + k];
        if (!(lo <= hi) || !isfinite(lo) || !isfinite(hi)) bad++;
    }
    if (bad) atomicAdd(&cnt, bad);
    __syncthreads();
    if (threadIdx.x == 0 && cnt) atomicAdd(counter, cnt);
}

// ------------------------------------------------------------------------
// level transition and refinement mask
// ------------------------------------------------------------------------

struct InterpArgs {
    int D;
    int ns[4];
    int nd[4];
    int64_t ss[4];  // source strides
    int64_t Nd;
};

// Multilinear sample of the source grid at every destination node: integer
// cell index and FP64 weight per axis, corners summed in row-major order of
// their offsets in FP64 without fused multiply-adds, one rounding at the end.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_interp(InterpArgs A, const T* __restrict__ Vs,
                                                   T* __restrict__ Vd, const T* __restrict__ ld)
{
#pragma clang fp contract(off)
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < A.Nd;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t q[4] = {0, 0, 0, 0};
        double t[4] = {0, 0, 0, 0};
        int64_t rest = idx;
        for (int a = A.D - 1; a >= 0; a--) {
            const int64_t j = rest % A.nd[a];
            rest /= A.nd[a];
            const int64_t num = j * (int64_t)(A.ns[a] - 1);
            int64_t qa = num / (A.nd[a] - 1);
            const int64_t r = num % (A.nd[a] - 1);
            if (qa == A.ns[a] - 1) {
                qa = A.ns[a] - 2;
                t[a] = 1.0;
            } else {
                t[a] = (double)r / (double)(A.nd[a] - 1);
            }
            q[a] = qa;
        }
        double acc = 0.0;
        const int nc = 1 << A.D;
        for (int c = 0; c < nc; c++) {
            double w = 1.0;
            int64_t off = 0;
            for (int a = 0; a < A.D; a++) {
                const int ca = (c >> (A.D - 1 - a)) & 1;
                w = w * (ca ? t[a] : 1.0 - t[a]);
                off += (q[a] + ca) * A.ss[a];
            }
            acc = acc + w * (double)Vs[off];
        }
        T v = (T)acc;
        if (ld) {
            const T lv = ld[idx];
            v = (lv < v) ? lv : v;
        }
        Vd[idx] = v;
    }
}

struct MaskArgs {
    int D;
    int nc[4];      // cells per axis (n - 1)
    int64_t s[4];   // node strides
    int64_t Nc;
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_mask(MaskArgs A, const T* __restrict__ V,
                                                 uint8_t* __restrict__ mask, uint64_t* counter)
{
    __shared__ uint64_t red[kBlock / 64];
    uint64_t cnt = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t start = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // every thread runs the same number of loop trips so the block reduction
    // below is reached uniformly
    const int64_t trips = (A.Nc + stride - 1) / stride;
    for (int64_t k = 0; k < trips; k++) {
        const int64_t c = start + k * stride;
        if (c < A.Nc) {
            int64_t base = 0, rest = c;
            for (int a = A.D - 1; a >= 0; a--) {
                base += (rest % A.nc[a]) * A.s[a];
                rest /= A.nc[a];
            }
            bool pos = false, neg = false;
            for (int k2 = 0; k2 < (1 << A.D); k2++) {
                int64_t off = base;
                for (int a = 0; a < A.D; a++) off += ((k2 >> a) & 1) * A.s[a];
                const T v = V[off];
                pos = pos || (v >= T(0));
                neg = neg || (v < T(0));
            }
            const uint8_t m = (pos && neg) ? 1 : 0;
            mask[c] = m;
            cnt += m;
        }
    }
    // sum over the block via the max-reduction helper's shuffle pattern
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t s = 0;
        for (int i = 0; i < kBlock / 64; i++) s += red[i];
        if (s && counter) atomicAdd((unsigned long long*)counter, (unsigned long long)s);
    }
}

// ------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------

static int grid_for(int64_t n, int cap)
{
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

hipError_t launch_prologue(hipStream_t s, const ChunkArgs& a)
{
    hipLaunchKernelGGL(k_prologue, dim3(a.cap), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_epilogue(hipStream_t s, const ChunkArgs& a)
{
    hipLaunchKernelGGL(k_epilogue, dim3(a.cap), dim3(64), 0, s, a);
    return hipGetLastError();
}

// One stage kernel.  With events (the timed chunks of HJR_FLAG_PROFILE) the
// runtime stamps them at the kernel's own start and end, so the measured
// time holds no gap between launches.
template <typename T, int STAGE, int FAM, bool DEEP>
static void launch_kernel(hipStream_t s, dim3 g, dim3 b, const ChunkArgs& a, hipEvent_t e0, hipEvent_t e1)
{
    if (e0 || e1)
        hipExtLaunchKernelGGL((k_stage<T, STAGE, FAM, DEEP>), g, b, 0, s, e0, e1, 0, a);
    else
        hipLaunchKernelGGL((k_stage<T, STAGE, FAM, DEEP>), g, b, 0, s, a);
}

// deep: the launch's workgroups take runs of tiles (a large set); the
// families that have one then run their deeper-pipelined FP32 kernel.
template <typename T, int STAGE, int FAM>
static void launch_one(hipStream_t s, dim3 g, dim3 b, const ChunkArgs& a, hipEvent_t e0, hipEvent_t e1,
                       bool deep)
{
    if constexpr (sizeof(T) == 4 && fam_deep(FAM)) {
        if (deep) {
            launch_kernel<T, STAGE, FAM, true>(s, g, b, a, e0, e1);
            return;
        }
    }
    launch_kernel<T, STAGE, FAM, false>(s, g, b, a, e0, e1);
}

template <typename T, int STAGE>
static hipError_t launch_stage_t(hipStream_t s, int fam, const ChunkArgs& a, int grid, hipEvent_t e0,
                                 hipEvent_t e1, bool deep)
{
    const dim3 g(grid), b(kStageBlock);
    switch (fam) {
    case kFamFlat: launch_one<T, STAGE, kFamFlat>(s, g, b, a, e0, e1, deep); break;
    case kFamZ2dS2: launch_one<T, STAGE, kFamZ2dS2>(s, g, b, a, e0, e1, deep); break;
    case kFamZ2dL2: launch_one<T, STAGE, kFamZ2dL2>(s, g, b, a, e0, e1, deep); break;
    case kFamX4dS2: launch_one<T, STAGE, kFamX4dS2>(s, g, b, a, e0, e1, deep); break;
    case kFamX4dL2: launch_one<T, STAGE, kFamX4dL2>(s, g, b, a, e0, e1, deep); break;
    case kFamZ2dS1: launch_one<T, STAGE, kFamZ2dS1>(s, g, b, a, e0, e1, deep); break;
    case kFamZ2dL1: launch_one<T, STAGE, kFamZ2dL1>(s, g, b, a, e0, e1, deep); break;
    case kFamX4dS1: launch_one<T, STAGE, kFamX4dS1>(s, g, b, a, e0, e1, deep); break;
    case kFamX4dL1: launch_one<T, STAGE, kFamX4dL1>(s, g, b, a, e0, e1, deep); break;
    case kFamZ2dS2F: launch_one<T, STAGE, kFamZ2dS2F>(s, g, b, a, e0, e1, deep); break;
    case kFamZ2dL2F: launch_one<T, STAGE, kFamZ2dL2F>(s, g, b, a, e0, e1, deep); break;
    case kFamX4dS2F: launch_one<T, STAGE, kFamX4dS2F>(s, g, b, a, e0, e1, deep); break;
    case kFamX4dL2F: launch_one<T, STAGE, kFamX4dL2F>(s, g, b, a, e0, e1, deep); break;
    case kFamXvS2: launch_one<T, STAGE, kFamXvS2>(s, g, b, a, e0, e1, deep); break;
    case kFamXvL2: launch_one<T, STAGE, kFamXvL2>(s, g, b, a, e0, e1, deep); break;
    case kFamXvS2F: launch_one<T, STAGE, kFamXvS2F>(s, g, b, a, e0, e1, deep); break;
    case kFamXvL2F: launch_one<T, STAGE, kFamXvL2F>(s, g, b, a, e0, e1, deep); break;
    case kFamX4dW2: launch_one<T, STAGE, kFamX4dW2>(s, g, b, a, e0, e1, deep); break;
    case kFamX4dW1: launch_one<T, STAGE, kFamX4dW1>(s, g, b, a, e0, e1, deep); break;
    case kFamXvW2: launch_one<T, STAGE, kFamXvW2>(s, g, b, a, e0, e1, deep); break;
    case kFamX4dMS2: launch_one<T, STAGE, kFamX4dMS2>(s, g, b, a, e0, e1, deep); break;
    case kFamX4dML2: launch_one<T, STAGE, kFamX4dML2>(s, g, b, a, e0, e1, deep); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_stage(hipStream_t s, int dtype, int stage, int fam, const ChunkArgs& a, int grid,
                        hipEvent_t e0, hipEvent_t e1, bool deep)
{
    if (dtype == HJR_F32)
        return stage == 1 ? launch_stage_t<float, 1>(s, fam, a, grid, e0, e1, deep)
                          : launch_stage_t<float, 2>(s, fam, a, grid, e0, e1, deep);
    return stage == 1 ? launch_stage_t<double, 1>(s, fam, a, grid, e0, e1, deep)
                      : launch_stage_t<double, 2>(s, fam, a, grid, e0, e1, deep);
}

hipError_t launch_level_setup(hipStream_t s, int dtype, const ProbDesc& P, ProbState* st)
{
    hipLaunchKernelGGL(k_zero_state, dim3(1), dim3(64), 0, s, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (dtype == HJR_F32)
        hipLaunchKernelGGL((k_alpha<float>), dim3(grid_for(P.N, 1024)), dim3(kBlock), 0, s, P, st);
    else
        hipLaunchKernelGGL((k_alpha<double>), dim3(grid_for(P.N, 1024)), dim3(kBlock), 0, s, P, st);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int g = grid_for(P.ndim >= 3 ? P.n[2] : 1, 64);
    if (dtype == HJR_F32)
        hipLaunchKernelGGL((k_finalize<float>), dim3(g), dim3(kBlock), 0, s, P, st);
    else
        hipLaunchKernelGGL((k_finalize<double>), dim3(g), dim3(kBlock), 0, s, P, st);
    return hipGetLastError();
}

hipError_t launch_init(hipStream_t s, int dtype, void* V, const void* l, const void* V0,
                       int64_t N)
{
    const int g = grid_for(N, 4096);
    if (dtype == HJR_F32)
        hipLaunchKernelGGL((k_init<float>), dim3(g), dim3(kBlock), 0, s, (float*)V,
                           (const float*)l, (const float*)V0, N);
    else
        hipLaunchKernelGGL((k_init<double>), dim3(g), dim3(kBlock), 0, s, (double*)V,
                           (const double*)l, (const double*)V0, N);
    return hipGetLastError();
}

hipError_t launch_interp(hipStream_t s, int dtype, const hjr_grid& src, const void* Vs,
                         const hjr_grid& dst, void* Vd, const void* l_dst)
{
    InterpArgs A;
    A.D = src.ndim;
    A.Nd = 1;
    for (int a = 0; a < 4; a++) {
        A.ns[a] = a < A.D ? src.n[a] : 1;
        A.nd[a] = a < A.D ? dst.n[a] : 1;
        A.ss[a] = 0;
    }
    int64_t st = 1;
    for (int a = A.D - 1; a >= 0; a--) {
        A.ss[a] = st;
        st *= src.n[a];
        A.Nd *= dst.n[a];
    }
    const int g = grid_for(A.Nd, 8192);
    if (dtype == HJR_F32)
        hipLaunchKernelGGL((k_interp<float>), dim3(g), dim3(kBlock), 0, s, A, (const float*)Vs,
                           (float*)Vd, (const float*)l_dst);
    else
        hipLaunchKernelGGL((k_interp<double>), dim3(g), dim3(kBlock), 0, s, A, (const double*)Vs,
                           (double*)Vd, (const double*)l_dst);
    return hipGetLastError();
}

hipError_t launch_mask(hipStream_t s, int dtype, const hjr_grid& g, const void* V,
                       uint8_t* mask, uint64_t* counter)
{
    MaskArgs A;
    A.D = g.ndim;
    A.Nc = 1;
    int64_t st = 1;
    for (int a = 3; a >= 0; a--) {
        A.nc[a] = a < A.D ? g.n[a] - 1 : 1;
        A.s[a] = 0;
    }
    for (int a = A.D - 1; a >= 0; a--) {
        A.s[a] = st;
        st *= g.n[a];
        A.Nc *= (g.n[a] - 1);
    }
    const int gr = grid_for(A.Nc, 8192);
    if (dtype == HJR_F32)
        hipLaunchKernelGGL((k_mask<float>), dim3(gr), dim3(kBlock), 0, s, A, (const float*)V, mask,
                           counter);
    else
        hipLaunchKernelGGL((k_mask<double>), dim3(gr), dim3(kBlock), 0, s, A, (const double*)V, mask,
                           counter);
    return hipGetLastError();
}

hipError_t launch_field_check(hipStream_t s, int dtype, const void* f, int nch, int64_t N,
                              uint64_t* counter)
{
    const int g = grid_for((int64_t)nch * N, 4096);
    if (dtype == HJR_F32)
        hipLaunchKernelGGL((k_field_check<float>), dim3(g), dim3(kBlock), 0, s, (const float*)f,
                           nch, N, (unsigned long long*)counter);
    else
        hipLaunchKernelGGL((k_field_check<double>), dim3(g), dim3(kBlock), 0, s, (const double*)f,
                           nch, N, (unsigned long long*)counter);
    return hipGetLastError();
}

// ------------------------------------------------------------------------
// localized updates: tile flags, band of a warm start, Vhat = V
// ------------------------------------------------------------------------

// tmask[t] = 1 iff one of the nodes t*tile .. t*tile + tile - 1 is set in
// umask (tmask nullable); *count += the number of set nodes (count nullable).
__global__ __launch_bounds__(kBlock) void k_tile_any(const uint8_t* __restrict__ umask, int64_t N,
                                                     int tile, uint8_t* tmask,
                                                     unsigned long long* count)
{
    __shared__ unsigned long long cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    const int64_t ntiles = (N + tile - 1) / tile;
    unsigned long long mine = 0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ntiles;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = min((t + 1) * tile, N);
        int any = 0;
        for (int64_t i = t * tile; i < e; i++) {
            const int on = umask[i] != 0;
            any |= on;
            mine += on;
        }
        if (tmask) tmask[t] = (uint8_t)any;
    }
    if (mine) atomicAdd(&cnt, mine);
    __syncthreads();
    if (threadIdx.x == 0 && cnt && count) atomicAdd(count, cnt);
}

// One pass of the band dilation along axis a: the input has extent
// n_in[b] on each axis (cells on axes >= a, nodes before), the output
// n_out (nodes on axes <= a); out[.., i_a, ..] = OR over in[.., c, ..] with
// c in [i_a - 1 - k, i_a + k] within the input's range.
struct DilateArgs {
    int D;
    int a;
    int k;
    int n_in[4];
    int n_out[4];
    int64_t total;  // output elements
};

__global__ __launch_bounds__(kBlock) void k_dilate(DilateArgs A, const uint8_t* __restrict__ in,
                                                   uint8_t* __restrict__ out)
{
    for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < A.total;
         o += (int64_t)gridDim.x * blockDim.x) {
        int j[4] = {0, 0, 0, 0};
        int64_t q = o;
        for (int b = A.D - 1; b >= 0; b--) {
            j[b] = (int)(q % A.n_out[b]);
            q /= A.n_out[b];
        }
        const int lo = max(j[A.a] - 1 - A.k, 0), hi = min(j[A.a] + A.k, A.n_in[A.a] - 1);
        int64_t base = 0, stride = 1, sa = 0;
        for (int b = A.D - 1; b >= 0; b--) {
            if (b == A.a)
                sa = stride;
            else
                base += (int64_t)j[b] * stride;
            stride *= A.n_in[b];
        }
        uint8_t v = 0;
        for (int c = lo; c <= hi; c++) v |= in[base + (int64_t)c * sa];
        out[o] = v ? 1 : 0;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_copy(const T* __restrict__ src, T* __restrict__ dst, int64_t N)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// Localized update on 4-D plane tiles: tmask[t] = 1 iff one node of plane
// tile t (its rows of its plane, placed as the stage kernels place it) is
// set in umask.  One thread per tile.
__global__ __launch_bounds__(kBlock) void k_plane_tile_any(ProbDesc P, const uint8_t* __restrict__ umask,
                                                           uint8_t* __restrict__ tmask)
{
    const int nr = P.n[2], nc = P.n[3];
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < P.ntiles;
         t += (int64_t)gridDim.x * blockDim.x) {
        int i0, i1, chunk;
        plane_place<4>(P, (uint32_t)t, i0, i1, chunk);
        const int r0 = chunk * P.rows;
        const int r1 = min(r0 + P.rows, nr);
        const int64_t base = ((int64_t)(i0 * P.n[1] + i1) * nr + r0) * nc;
        const int64_t cnt = (int64_t)(r1 - r0) * nc;
        uint8_t any = 0;
        for (int64_t e = 0; e < cnt && !any; e++) any = umask[base + e] != 0;
        tmask[t] = any;
    }
}

hipError_t launch_plane_tile_flags(hipStream_t s, const ProbDesc& P, const uint8_t* umask, uint8_t* tmask)
{
    if (P.ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_plane_tile_any, dim3(grid_for(P.ntiles, 4096)), dim3(kBlock), 0, s, P, umask,
                       tmask);
    return hipGetLastError();
}

hipError_t launch_tile_flags(hipStream_t s, const uint8_t* umask, int64_t N, int tile,
                             uint8_t* tmask, uint64_t* count)
{
    const int64_t ntiles = (N + tile - 1) / tile;
    hipLaunchKernelGGL(k_tile_any, dim3(grid_for(ntiles, 1024)), dim3(kBlock), 0, s, umask, N, tile,
                       tmask, (unsigned long long*)count);
    return hipGetLastError();
}

hipError_t launch_band(hipStream_t s, int dtype, const hjr_grid& g, const void* V, int k,
                       uint8_t* tmp0, uint8_t* tmp1, uint8_t* node_mask)
{
    // straddling cells, then one dilation pass per axis (cells -> nodes)
    hipError_t e = launch_mask(s, dtype, g, V, tmp0, nullptr);
    if (e != hipSuccess) return e;
    const int D = g.ndim;
    DilateArgs A;
    A.D = D;
    A.k = k;
    for (int b = 0; b < 4; b++) A.n_in[b] = A.n_out[b] = b < D ? g.n[b] - 1 : 1;
    const uint8_t* in = tmp0;
    for (int a = 0; a < D; a++) {
        A.a = a;
        A.n_out[a] = g.n[a];
        A.total = 1;
        for (int b = 0; b < D; b++) A.total *= A.n_out[b];
        uint8_t* out = (a == D - 1) ? node_mask : ((a % 2 == 0) ? tmp1 : tmp0);
        hipLaunchKernelGGL(k_dilate, dim3(grid_for(A.total, 8192)), dim3(kBlock), 0, s, A, in, out);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        in = out;
        A.n_in[a] = g.n[a];
    }
    return hipSuccess;
}

hipError_t launch_copy(hipStream_t s, int dtype, const void* src, void* dst, int64_t N)
{
    const int g = grid_for(N, 4096);
    if (dtype == HJR_F32)
        hipLaunchKernelGGL((k_copy<float>), dim3(g), dim3(kBlock), 0, s, (const float*)src, (float*)dst, N);
    else
        hipLaunchKernelGGL((k_copy<double>), dim3(g), dim3(kBlock), 0, s, (const double*)src, (double*)dst, N);
    return hipGetLastError();
}

hipError_t launch_fill_u64(hipStream_t s, uint64_t* p, int64_t n, uint64_t value)
{
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 1024)), dim3(kBlock), 0, s, p, n, value);
    return hipGetLastError();
}

template <typename T, int STAGE>
static const void* stage_kernel(int fam)
{
    switch (fam) {
    case kFamFlat: return (const void*)k_stage<T, STAGE, kFamFlat>;
    case kFamZ2dS2: return (const void*)k_stage<T, STAGE, kFamZ2dS2>;
    case kFamZ2dL2: return (const void*)k_stage<T, STAGE, kFamZ2dL2>;
    case kFamX4dS2: return (const void*)k_stage<T, STAGE, kFamX4dS2>;
    case kFamX4dL2: return (const void*)k_stage<T, STAGE, kFamX4dL2>;
    case kFamZ2dS1: return (const void*)k_stage<T, STAGE, kFamZ2dS1>;
    case kFamZ2dL1: return (const void*)k_stage<T, STAGE, kFamZ2dL1>;
    case kFamX4dS1: return (const void*)k_stage<T, STAGE, kFamX4dS1>;
    case kFamX4dL1: return (const void*)k_stage<T, STAGE, kFamX4dL1>;
    case kFamZ2dS2F: return (const void*)k_stage<T, STAGE, kFamZ2dS2F>;
    case kFamZ2dL2F: return (const void*)k_stage<T, STAGE, kFamZ2dL2F>;
    case kFamX4dS2F: return (const void*)k_stage<T, STAGE, kFamX4dS2F>;
    case kFamX4dL2F: return (const void*)k_stage<T, STAGE, kFamX4dL2F>;
    case kFamXvS2: return (const void*)k_stage<T, STAGE, kFamXvS2>;
    case kFamXvL2: return (const void*)k_stage<T, STAGE, kFamXvL2>;
    case kFamXvS2F: return (const void*)k_stage<T, STAGE, kFamXvS2F>;
    case kFamX4dW2: return (const void*)k_stage<T, STAGE, kFamX4dW2>;
    case kFamX4dW1: return (const void*)k_stage<T, STAGE, kFamX4dW1>;
    case kFamXvW2: return (const void*)k_stage<T, STAGE, kFamXvW2>;
    case kFamX4dMS2: return (const void*)k_stage<T, STAGE, kFamX4dMS2>;
    case kFamX4dML2: return (const void*)k_stage<T, STAGE, kFamX4dML2>;
    default: return (const void*)k_stage<T, STAGE, kFamXvL2F>;
    }
}

int stage_blocks_per_cu(int dtype, int stage, int fam)
{
    const void* k = dtype == HJR_F32 ? (stage == 1 ? stage_kernel<float, 1>(fam) : stage_kernel<float, 2>(fam))
                                     : (stage == 1 ? stage_kernel<double, 1>(fam) : stage_kernel<double, 2>(fam));
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, kStageBlock, 0);
    if (e != hipSuccess || n < 1) n = 2;
    int cap = dtype == HJR_F64 ? HJR_BLOCKS_PER_CU_F64 : HJR_BLOCKS_PER_CU;
    if (dtype == HJR_F32 && stage == 2 && HJR_BLOCKS_PER_CU_S2 > 0) cap = HJR_BLOCKS_PER_CU_S2;
    if (cap > 0 && cap < n) n = cap;
    return n;
}

}  // namespace hjr
