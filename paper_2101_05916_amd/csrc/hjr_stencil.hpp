// hjr_stencil.hpp -- device side of one RK stage: the upwind derivatives,
// the Hamiltonians and the two tile shapes of the stage kernels.
//
// Notation.  Along an axis of spacing h, w0..w4 are the values at
// j-2..j+2 (ghost values past the ends are linear extrapolations of the two
// end nodes).  With raw differences a..d (h times the first divided
// differences at j-3/2..j+3/2) and raw second differences sm, s0, sp,
//     h D^- = b + cm/2,  h D^+ = c - cp/2,
// cm / cp being the second difference of smaller magnitude on each side (a
// tie takes the outer one).  A stage needs only
//     sum = h (D^+ + D^-)   and   dif = h (D^+ - D^-)
// per axis: the Hamiltonian is evaluated at p = sum * (0.5/h) and the
// Lax-Friedrichs term is alpha * (0.5/h) * dif.  The 0.5/h factors are
// folded into per-problem constants (ProbDesc::hc), so the Hamiltonians
// below take `sum` directly.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/hjr.h"
#include "hjr_device.hpp"

namespace hjr {

__device__ __forceinline__ uint32_t fdiv(uint32_t x, const FastDiv& f)
{
    return __umulhi(x, f.m) >> f.s;
}

__device__ __forceinline__ uint32_t fdiv(uint32_t x, const HJR_CONST FastDiv& f)
{
    return __umulhi(x, f.m) >> f.s;
}

// x / f.d for x * f.d < 2^20 (both factors below 2^24): a 24-bit multiply
// and a shift, full-rate instructions, where fdiv takes a quarter-rate
// 32-bit multiply-high.
__device__ __forceinline__ uint32_t fdiv20(uint32_t x, const HJR_CONST FastDiv& f)
{
    return __umul24(x, f.m20) >> 20;
}

// Pins a loop-invariant value in a vector register: an operand pair of two
// scalar registers (a select between two constants, an fma of a node
// coordinate with two constants) would otherwise cost a copy per node.
template <typename T>
__device__ __forceinline__ T in_vgpr(T x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// Global-memory access through an explicit global address space: the
// problem table hands out generic pointers, and a generic (flat) access both
// costs a 64-bit address add per load and counts against the LDS wait
// counter, so every LDS wait would also wait for outstanding global loads.
#define HJR_GLOBAL __attribute__((address_space(1)))

// Element i (32-bit; the host keeps N * sizeof(T) < 2^32 where these are
// used) of a uniform base pointer: one SGPR pair plus one VGPR offset.
template <typename T>
__device__ __forceinline__ T ld32(const T* base, uint32_t i)
{
    return *(const HJR_GLOBAL T*)((const HJR_GLOBAL char*)base + i * (uint32_t)sizeof(T));
}

template <typename T>
__device__ __forceinline__ void st32(T* base, uint32_t i, T v)
{
    *(HJR_GLOBAL T*)((HJR_GLOBAL char*)base + i * (uint32_t)sizeof(T)) = v;
}

// Element i (any 64-bit index) of a global array.
template <typename T>
__device__ __forceinline__ T ld64(const T* base, int64_t i)
{
    return ((const HJR_GLOBAL T*)base)[i];
}

template <typename T>
__device__ __forceinline__ void st64(T* base, int64_t i, T v)
{
    ((HJR_GLOBAL T*)base)[i] = v;
}

template <typename T>
__device__ __forceinline__ T gld1(const T* base, uint32_t byte_off)
{
    return *(const HJR_GLOBAL T*)((const HJR_GLOBAL char*)base + byte_off);
}

template <typename T>
__device__ __forceinline__ void gst1(T v, T* base, uint32_t byte_off)
{
    *(HJR_GLOBAL T*)((HJR_GLOBAL char*)base + byte_off) = v;
}

template <typename T>
struct Prec;
template <>
struct Prec<float> {
    typedef const HJR_CONST float* CP;
    __device__ static CP hih(PDesc& P) { return P.hih_f; }
    __device__ static CP lo(PDesc& P) { return P.lo_f; }
    __device__ static CP h(PDesc& P) { return P.h_f; }
    __device__ static CP hc(PDesc& P) { return P.hc_f; }
    __device__ static CP ah(PState& S) { return S.ah_f; }
    __device__ static float dt(PState& S) { return S.dt_f; }
};
template <>
struct Prec<double> {
    typedef const HJR_CONST double* CP;
    __device__ static CP hih(PDesc& P) { return P.hih; }
    __device__ static CP lo(PDesc& P) { return P.lo; }
    __device__ static CP h(PDesc& P) { return P.h; }
    __device__ static CP hc(PDesc& P) { return P.hc_d; }
    __device__ static CP ah(PState& S) { return S.ah; }
    __device__ static double dt(PState& S) { return S.dt; }
};

// sum and dif of one axis from its five samples (see the header comment).
template <typename T>
__device__ __forceinline__ void eno_sum_dif(T w0, T w1, T w2, T w3, T w4, int order, T& sum, T& dif);

// ORDER fixed at compile time (2 = ENO2, 1 = first order).
template <typename T, int ORDER>
__device__ __forceinline__ void eno_sd(T w0, T w1, T w2, T w3, T w4, T& sum, T& dif)
{
    eno_sum_dif<T>(w0, w1, w2, w3, w4, ORDER, sum, dif);
}

template <typename T>
__device__ __forceinline__ void eno_sum_dif(T w0, T w1, T w2, T w3, T w4, int order, T& sum, T& dif)
{
    const T a = w1 - w0, b = w2 - w1, c = w3 - w2, d = w4 - w3;
    T pm = b, pp = c;
    if (order != 1) {
        const T sm = b - a, s0 = c - b, sp = d - c;
        const T cm = (fabs(sm) <= fabs(s0)) ? sm : s0;
        const T cp = (fabs(sp) <= fabs(s0)) ? sp : s0;
        pm = b + T(0.5) * cm;
        pp = c - T(0.5) * cp;
    }
    sum = pp + pm;
    dif = pp - pm;
}

// Replace the samples of positions outside [0, n-1] by the linear
// extrapolation of the two end nodes: v[-1] = 2v[0]-v[1], v[-2] = 3v[0]-2v[1]
// and mirrored at the top.  m2, m1, p1, p2 hold loads from clamped (in-range)
// positions; only loaded values feed the formulas (n >= 3).
template <typename T>
__device__ __forceinline__ void ghost_fix(int j, int n, T c, T& m2, T& m1, T& p1, T& p2)
{
    const bool lo1 = j >= 1, lo2 = j >= 2, hi1 = j <= n - 2, hi2 = j <= n - 3;
    const T m1f = lo1 ? m1 : T(2) * c - p1;
    const T p1f = hi1 ? p1 : T(2) * c - m1;
    const T m2f = lo2 ? m2 : (lo1 ? T(2) * m1 - c : T(3) * c - T(2) * p1);
    const T p2f = hi2 ? p2 : (hi1 ? T(2) * p1 - c : T(3) * c - T(2) * m1);
    m2 = m2f;
    m1 = m1f;
    p1 = p1f;
    p2 = p2f;
}

// ------------------------------------------------------------------------
// Hamiltonians H(x, p) = max_u min_d p . f(x, u, d) of the affine models,
// evaluated from per-axis sums (p_a = sum_a * 0.5/h_a) and node indices.
// Over a box, an affine function's max/min sit at vertices, so each control
// or disturbance term is a product with the coefficient picked by the sign
// of its p component.  ProbDesc::hc holds the folded constants, written by
// the host (fill_desc).
// ------------------------------------------------------------------------

// z' = vz, vz' = k u - g + d.  hc = {hih0*lo1, hih0*h1, Cpos, Cneg} with
// Cpos = (max(k u) + min(d) - g) hih1, Cneg = (min(k u) + max(d) - g) hih1.
template <typename T>
struct HamZ2D {
    static constexpr bool kRowRecords = false;
    T c0, c1, cpos, cneg;
    __device__ void init(PDesc& P)
    {
        const HJR_CONST T* hc = Prec<T>::hc(P);
        c0 = hc[0];
        c1 = hc[1];
        cpos = hc[2];
        cneg = hc[3];
    }
    __device__ __forceinline__ T operator()(const T* sum, int j0, int j1, int j2, int j3) const
    {
        const T vzh = c0 + (T)j1 * c1;  // (0.5/h0) vz
        return sum[0] * vzh + sum[1] * (sum[1] >= T(0) ? cpos : cneg);
    }
    // per-node data: none (no per-row table)
    typedef T Node;
    __device__ __forceinline__ Node node_b(int, uint32_t) const { return T(0); }
    __device__ __forceinline__ Node node_i(int, int64_t) const { return T(0); }
    __device__ __forceinline__ T eval(const T* sum, int j0, int j1, int j2, int j3, T) const
    {
        return (*this)(sum, j0, j1, j2, j3);
    }
};

// The same model with a per-node disturbance box [lo(x), hi(x)] (d in D(x),
// paper Sec. II-A), read from the field at P.dfield: lower bounds of the N
// nodes, then upper bounds.  hc[4] = (max(k u) - g) hih1, hc[5] = (min(k u)
// - g) hih1, hc[6] = hih1.
template <typename T>
struct HamZ2DF {
    static constexpr bool kRowRecords = false;
    T c0, c1, kpos, kneg, h1;
    const T* flo;
    const T* fhi;
    struct Node {
        T dl, dh;
    };
    __device__ void init(PDesc& P)
    {
        const HJR_CONST T* hc = Prec<T>::hc(P);
        c0 = hc[0];
        c1 = hc[1];
        kpos = hc[4];
        kneg = hc[5];
        h1 = hc[6];
        flo = (const T*)P.dfield;
        fhi = flo + P.N;
    }
    __device__ __forceinline__ Node node_b(int, uint32_t vb) const
    {
        return Node{gld1<T>(flo, vb), gld1<T>(fhi, vb)};
    }
    __device__ __forceinline__ Node node_i(int, int64_t idx) const
    {
        return Node{ld64(flo, idx), ld64(fhi, idx)};
    }
    __device__ __forceinline__ T eval(const T* sum, int, int j1, int, int, Node nd) const
    {
        const T vzh = c0 + (T)j1 * c1;  // (0.5/h0) vz
        const T s1 = sum[1];
        return sum[0] * vzh + s1 * (s1 >= T(0) ? kpos + nd.dl * h1 : kneg + nd.dh * h1);
    }
};

// x' = vx + d, vx' = g tan(theta), theta' = -d1 theta + omega,
// omega' = -d0 theta + n0 S.  hc = {hih0*lo1, hih0*h1, dlo*hih0, dhi*hih0,
// hih2*(lo3 - d1 lo2), hih2*h3, hih2*d1*h2, d0*hih3*lo2, d0*hih3*h2,
// n0*smax*hih3}; table[j2] = g tan(theta_j2) * hih1.
// VD: the 10-D model's form, the disturbance on the velocity rate
// (x' = vx, vx' = g tan(theta) + d); then hc[2], hc[3] = dlo*hih1, dhi*hih1.
template <typename T, bool VD = false>
struct HamX4D {
    // plane tiles keep each tile row's coefficient and index (as T) in LDS
    static constexpr bool kRowRecords = true;
    T c0, c1, dl, dh, A, B, C, D, E, n0s;
    const T* gts;
    __device__ void init(PDesc& P)
    {
        const HJR_CONST T* hc = Prec<T>::hc(P);
        c0 = hc[0];
        c1 = hc[1];
        dl = hc[2];
        dh = hc[3];
        A = hc[4];
        B = hc[5];
        C = hc[6];
        D = hc[7];
        E = hc[8];
        n0s = hc[9];
        gts = (const T*)P.table;
        // operands that would meet another scalar operand in one per-node
        // instruction (the select between dl and dh, the fma bases A and D)
        dl = in_vgpr(dl);
        dh = in_vgpr(dh);
        A = in_vgpr(A);
        D = in_vgpr(D);
    }
    // table[j2], loaded by plane tiles together with the node's other loads
    __device__ __forceinline__ T row_coef(int j2) const { return ld32(gts, (uint32_t)j2); }
    // the node-coordinate terms: (0.5/h0) vx, (0.5/h2)(omega - d1 theta) and
    // (0.5/h3) d0 theta
    __device__ __forceinline__ T coef_vx(int j1) const { return c0 + (T)j1 * c1; }
    __device__ __forceinline__ T coef_tw(int j2, int j3) const { return A + (T)j3 * B - (T)j2 * C; }
    __device__ __forceinline__ T coef_t3(int j2) const { return D + (T)j2 * E; }
    // H from the per-axis sums and the node's terms (g: the row coefficient)
    __device__ __forceinline__ T eval_terms(const T* sum, T cvx, T tw, T t3, T g) const
    {
        const T s0 = sum[0], s1 = sum[1];
        if (VD)
            return s0 * cvx + s1 * (g + (s1 >= T(0) ? dl : dh)) + sum[2] * tw - sum[3] * t3 +
                   n0s * fabs(sum[3]);
        return s0 * (cvx + (s0 >= T(0) ? dl : dh)) + s1 * g + sum[2] * tw - sum[3] * t3 +
               n0s * fabs(sum[3]);
    }
    __device__ __forceinline__ T eval(const T* sum, int j0, int j1, int j2, int j3, T g) const
    {
        return eval_terms(sum, coef_vx(j1), coef_tw(j2, j3), coef_t3(j2), g);
    }
    // the same with the row index already converted (j2f == (T)j2, exact)
    __device__ __forceinline__ T eval_f(const T* sum, int j1, T j2f, int j3, T g) const
    {
        return eval_terms(sum, coef_vx(j1), A + (T)j3 * B - j2f * C, D + j2f * E, g);
    }
    __device__ __forceinline__ T operator()(const T* sum, int j0, int j1, int j2, int j3) const
    {
        return eval(sum, j0, j1, j2, j3, row_coef(j2));
    }
    // per-node data: the row coefficient
    typedef T Node;
    __device__ __forceinline__ Node node_b(int j2, uint32_t) const { return row_coef(j2); }
    __device__ __forceinline__ Node node_i(int j2, int64_t) const { return row_coef(j2); }
};

// The x-subsystem with a per-node disturbance box (field layout as for
// HamZ2DF) on x', hc[10] = hih0, or with VD on vx', hc[10] = hih1.
template <typename T, bool VD = false>
struct HamX4DF {
    static constexpr bool kRowRecords = false;
    T c0, c1, h0, A, B, C, D, E, n0s;
    const T* gts;
    const T* flo;
    const T* fhi;
    struct Node {
        T g, dl, dh;
    };
    __device__ void init(PDesc& P)
    {
        const HJR_CONST T* hc = Prec<T>::hc(P);
        c0 = hc[0];
        c1 = hc[1];
        A = hc[4];
        B = hc[5];
        C = hc[6];
        D = hc[7];
        E = hc[8];
        n0s = hc[9];
        h0 = hc[10];
        gts = (const T*)P.table;
        flo = (const T*)P.dfield;
        fhi = flo + P.N;
    }
    __device__ __forceinline__ Node node_b(int j2, uint32_t vb) const
    {
        return Node{ld32(gts, (uint32_t)j2), gld1<T>(flo, vb), gld1<T>(fhi, vb)};
    }
    __device__ __forceinline__ Node node_i(int j2, int64_t idx) const
    {
        return Node{ld32(gts, (uint32_t)j2), ld64(flo, idx), ld64(fhi, idx)};
    }
    __device__ __forceinline__ T eval(const T* sum, int, int j1, int j2, int j3, Node nd) const
    {
        const T cvx = c0 + (T)j1 * c1;
        const T tw = A + (T)j3 * B - (T)j2 * C;
        const T t3 = D + (T)j2 * E;
        const T s0 = sum[0], s1 = sum[1];
        if (VD)
            return s0 * cvx + s1 * (nd.g + (s1 >= T(0) ? nd.dl : nd.dh) * h0) + sum[2] * tw -
                   sum[3] * t3 + n0s * fabs(sum[3]);
        return s0 * (cvx + (s0 >= T(0) ? nd.dl : nd.dh) * h0) + s1 * nd.g + sum[2] * tw -
               sum[3] * t3 + n0s * fabs(sum[3]);
    }
};

// Two independent vertical models on a permutation of the axes (test model).
// FIELD: channel c's box at node x is [f[2c N + x], f[(2c + 1) N + x]] of
// the field at P.dfield; else the constant boxes P.dlo, P.dhi.
template <typename T, bool FIELD = false>
struct HamDI2X2 {
    int za, va, zb, vb;
    T ga, kalo, kahi, dalo, dahi, gb, kblo, kbhi, dblo, dbhi;
    T hih[4], lo[4], h[4];
    const T* f;
    int64_t N;
    struct Node {
        T al, ah, bl, bh;
    };
    __device__ void init(PDesc& P)
    {
        ga = (T)P.par[1];
        kalo = (T)(P.par[0] * P.par[2]);
        kahi = (T)(P.par[0] * P.par[3]);
        gb = (T)P.par[5];
        kblo = (T)(P.par[4] * P.par[6]);
        kbhi = (T)(P.par[4] * P.par[7]);
        za = (int)P.par[8];
        va = (int)P.par[9];
        zb = (int)P.par[10];
        vb = (int)P.par[11];
        dalo = (T)P.dlo[0];
        dahi = (T)P.dhi[0];
        dblo = (T)P.dlo[1];
        dbhi = (T)P.dhi[1];
        f = (const T*)P.dfield;
        N = P.N;
        for (int a = 0; a < 4; a++) {
            hih[a] = Prec<T>::hih(P)[a];
            lo[a] = Prec<T>::lo(P)[a];
            h[a] = Prec<T>::h(P)[a];
        }
    }
    __device__ static T pick(const T* v, int i)
    {
        return i == 0 ? v[0] : (i == 1 ? v[1] : (i == 2 ? v[2] : v[3]));
    }
    __device__ __forceinline__ Node node_i(int, int64_t idx) const
    {
        if (FIELD)
            return Node{ld64(f, idx), ld64(f, N + idx), ld64(f, 2 * N + idx), ld64(f, 3 * N + idx)};
        return Node{dalo, dahi, dblo, dbhi};
    }
    __device__ __forceinline__ T eval(const T* sum, int j0, int j1, int j2, int j3, Node nd) const
    {
        const int jj[4] = {j0, j1, j2, j3};
        T p[4], x[4];
        for (int a = 0; a < 4; a++) {
            p[a] = sum[a] * hih[a];
            x[a] = lo[a] + (T)jj[a] * h[a];
        }
        const T pva = pick(p, va), pvb = pick(p, vb);
        return pick(p, za) * pick(x, va) - ga * pva + fmax(kalo * pva, kahi * pva) +
               fmin(nd.al * pva, nd.ah * pva) + pick(p, zb) * pick(x, vb) - gb * pvb +
               fmax(kblo * pvb, kbhi * pvb) + fmin(nd.bl * pvb, nd.bh * pvb);
    }
};

// ------------------------------------------------------------------------
// stage epilogue
// ------------------------------------------------------------------------

__device__ __forceinline__ uint64_t dbits(double x)
{
    return (uint64_t)__double_as_longlong(x);
}

__device__ __forceinline__ uint64_t umax64(uint64_t a, uint64_t b)
{
    return a > b ? a : b;
}

// Whether a node enters the residual: unless both the old and the new value
// lie at or beyond the band (band = +inf counts every node; a NaN counts).
// FP32 values compare with the band rounded up to a float, which decides
// exactly as the comparison in double would.
__device__ __forceinline__ bool in_band(double vn, double vo, PDesc& P)
{
    return !(fabs(vn) >= P.band && fabs(vo) >= P.band);
}

__device__ __forceinline__ bool in_band(float vn, float vo, PDesc& P)
{
    return !(fabsf(vn) >= P.band_f && fabsf(vo) >= P.band_f);
}

// Stage 1 writes Vhat = c + dt L.  Stage 2 writes V' = min(l, (V + c + dt L)/2)
// over V and folds |V' - V| (in double) into rmax.
template <typename T, int STAGE>
__device__ __forceinline__ void finish_node(PDesc& P, int64_t gi, T c, T L, T dt,
                                            uint64_t& rmax)
{
    if (STAGE == 1) {
        st64((T*)P.Vhat, gi, c + dt * L);
    } else {
        const T vt = c + dt * L;
        const T vo = ld64((const T*)P.V, gi);
        const T avg = T(0.5) * (vo + vt);
        const T lv = ld64((const T*)P.l, gi);
        const T vn = (lv < avg) ? lv : avg;
        st64((T*)P.V, gi, vn);
        if (in_band(vn, vo, P)) rmax = umax64(rmax, dbits(fabs((double)vn - (double)vo)));
    }
}

// ------------------------------------------------------------------------
// flat tiles: kTile consecutive nodes, any shape (fallback path)
// ------------------------------------------------------------------------

template <typename T, int D, class Ham, int STAGE>
__device__ uint64_t tile_flat(PDesc& P, PState& S, int64_t tile)
{
    Ham ham;
    ham.init(P);
    const HJR_CONST T* ah = Prec<T>::ah(S);
    const T dt = Prec<T>::dt(S);
    const int order = P.order;
    const int N = (int)P.N;
    const T* __restrict__ in = (const T*)(STAGE == 1 ? P.V : P.Vhat);
    uint64_t rmax = 0;
    // localized update: tiles without a node to update are skipped, and
    // only the masked nodes are written (the others keep V, and Vhat = V)
    const uint8_t* umask = P.umask;
    if (umask && !P.tmask[tile]) return 0;
    const int base = (int)(tile * kTile) + (int)threadIdx.x;
    for (int k = 0; k < kNodesPerThread; k++) {
        const int idx = base + k * kStageBlock;
        if (idx >= N) break;
        if (umask && !umask[idx]) continue;
        int j[4] = {0, 0, 0, 0};
        uint32_t q = (uint32_t)idx;
#pragma unroll
        for (int a = D - 1; a >= 1; a--) {
            const uint32_t qq = fdiv(q, P.div[a]);
            j[a] = (int)(q - qq * (uint32_t)P.n[a]);
            q = qq;
        }
        j[0] = (int)q;
        const T c = ld64(in, idx);
        T sum[4] = {0, 0, 0, 0};
        T L = T(0);
#pragma unroll
        for (int a = 0; a < D; a++) {
            const int s = (int)P.stride[a], n = P.n[a];
            T m2 = ld64(in, idx - (j[a] >= 2 ? 2 * s : (j[a] >= 1 ? s : 0)));
            T m1 = ld64(in, idx - (j[a] >= 1 ? s : 0));
            T p1 = ld64(in, idx + (j[a] <= n - 2 ? s : 0));
            T p2 = ld64(in, idx + (j[a] <= n - 3 ? 2 * s : (j[a] <= n - 2 ? s : 0)));
            ghost_fix<T>(j[a], n, c, m2, m1, p1, p2);
            T dif;
            eno_sum_dif<T>(m2, m1, c, p1, p2, order, sum[a], dif);
            L += ah[a] * dif;
        }
        if (D == 2)
            L += ham.eval(sum, j[0], j[1], 0, 0, ham.node_i(0, idx));
        else
            L += ham.eval(sum, j[0], j[1], j[2], j[3], ham.node_i(j[2], idx));
        finish_node<T, STAGE>(P, (int64_t)idx, c, L, dt, rmax);
    }
    return rmax;
}

// ------------------------------------------------------------------------
// plane tiles: rows of the two fastest axes staged in LDS with ghosts
// ------------------------------------------------------------------------

// Clamped offsets of the samples j-2, j-1, j+1, j+2 along an axis of stride
// s and length n (out-of-range samples read the centre; ghost_fix replaces
// them afterwards).
__device__ __forceinline__ void clamped_offsets(int j, int n, int s, int* o)
{
    o[0] = j >= 2 ? -2 * s : (j >= 1 ? -s : 0);
    o[1] = j >= 1 ? -s : 0;
    o[2] = j <= n - 2 ? s : 0;
    o[3] = j <= n - 3 ? 2 * s : (j <= n - 2 ? s : 0);
}

// Stage the loaded rows of a plane tile (nlr rows of nc nodes from element
// load0) into LDS rows lrow.. of stride RS, columns at +2, by direct
// global-to-LDS loads: one load instruction per row and 64-dword segment,
// lane i copying dword d0 + i of the row to the dword at the same position
// of the LDS row (a load of this kind writes its 64 dwords to consecutive LDS
// addresses from a wave-uniform base).  The staging costs no vector
// instructions and holds no registers.  A row of W <= 64 dwords is one
// segment whose lanes past the end copy its last dword to the dwords after
// the row, still inside the row's stride (2 elements + 64 dwords <= RS
// elements); longer rows take segments at 0, 64, ... and a last one ending
// at the row's end, so no lane writes outside the row.  The columns after
// the row are the ghost columns, written after the loads have completed.
template <typename T, int RS>
__device__ __forceinline__ void stage_dma(const T* in, uint32_t load0, int nc, int nlr, int lrow, T* lds,
                                          int tid)
{
    static_assert(2 * sizeof(T) + 64 * 4 <= RS * sizeof(T), "a one-segment row stays in its stride");
    constexpr int kRowDw = RS * (int)sizeof(T) / 4;  // LDS row stride in dwords
    constexpr int kCol0 = 2 * (int)sizeof(T) / 4;    // dword of column 0 in an LDS row
    const int W = nc * (int)sizeof(T) / 4;           // dwords of a row
    const int nseg = (W + 63) >> 6;
    const HJR_GLOBAL char* src = (const HJR_GLOBAL char*)in + (size_t)load0 * sizeof(T);
    __attribute__((address_space(3))) char* dst =
        (__attribute__((address_space(3))) char*)lds + (size_t)(lrow * kRowDw + kCol0) * 4;
    for (int sg = 0; sg < nseg; sg++) {
        const int d0 = (sg == nseg - 1 && sg > 0) ? W - 64 : 64 * sg;
        const uint32_t voff = (uint32_t)min(d0 + tid, W - 1) * 4u;
        for (int r = 0; r < nlr; r++)
            __builtin_amdgcn_global_load_lds(
                (const HJR_GLOBAL void*)(src + (size_t)r * (size_t)W * 4 + voff),
                (__attribute__((address_space(3))) void*)(dst + (r * kRowDw + d0) * 4), 4, 0, 0);
    }
}

// Stage the same rows through registers: element e = lane +
// 64 k of the loaded rows goes to LDS row e / nc, column e mod nc (one
// multiply-high division).  All loads are issued before the first LDS write;
// lanes past the end load a clamped element and write it to their spare slot
// (plane_elems(RS) + lane).
// (Staging column by column instead -- lane c owns column c, no division --
// executed more vector instructions in total and ran slower.)
template <typename T, int RS>
__device__ __forceinline__ void stage_flat(const T* in, uint32_t load0, int nc, int nlr, int lrow,
                                           T* lds, int tid, const HJR_CONST FastDiv& div_nc)
{
    constexpr int kSpare = plane_elems(RS);
    const int nload = nlr * nc;
    T sv[kPlaneStagePT];
#pragma unroll
    for (int k = 0; k < kPlaneStagePT; k++) {
        sv[k] = T(0);
        if (k * kStageBlock < nload) {
            const uint32_t e = min((uint32_t)(tid + k * kStageBlock), (uint32_t)(nload - 1));
            sv[k] = gld1<T>(in, (load0 + e) * (uint32_t)sizeof(T));
        }
    }
#pragma unroll
    for (int k = 0; k < kPlaneStagePT; k++) {
        if (k * kStageBlock < nload) {
            const int e = tid + k * kStageBlock;
            const int rr = (int)fdiv20((uint32_t)e, div_nc);
            const int cc = e - (int)__umul24((uint32_t)rr, (uint32_t)nc);
            lds[e < nload ? (int)__umul24((uint32_t)(lrow + rr), (uint32_t)RS) + cc + 2 : kSpare + tid] = sv[k];
        }
    }
}


// Plane tile `tile` of a problem -> its plane (i0, i1; 0, 0 for D = 2) and
// chunk of rows.  4-D planes are ordered in blocks of bx consecutive axis-0
// indices (the last block may be shorter), axis 1 next, axis 0 fastest
// inside a block: workgroups running together then hold a compact patch of
// (i0, i1) planes, and the neighbour planes they read were staged recently.
template <int D, class Desc>
__device__ __forceinline__ void plane_place(Desc& P, uint32_t tile, int& i0, int& i1, int& chunk)
{
    const uint32_t outer = P.chunks == 1 ? tile : fdiv(tile, P.div_chunks);
    chunk = (int)(tile - outer * (uint32_t)P.chunks);
    i0 = 0;
    i1 = 0;
    if (D == 4) {
        if (P.bx > 1) {
            const uint32_t blk = fdiv(outer, P.div_bxn1);
            const int rem = (int)(outer - blk * (uint32_t)(P.bx * P.n[1]));
            int q, bxs;
            if ((int)blk == P.nblk - 1) {
                bxs = P.bxl;
                q = bxs == 1 ? rem : (int)fdiv((uint32_t)rem, P.div_bxl);
            } else {
                bxs = P.bx;
                q = (int)fdiv((uint32_t)rem, P.div_bx);
            }
            i1 = q;
            i0 = (int)blk * P.bx + (rem - q * bxs);
        } else {
            i0 = (int)fdiv(outer, P.div[1]);
            i1 = (int)outer - i0 * P.n[1];
        }
    }
}

// Tile t of a problem covers rows [r0, r1) of axis D-2 at a fixed index of
// the outer axes (i0, i1 for D = 4); the host keeps (r1 - r0) * n_last <=
// kPlaneNodesPT * kStageBlock and (r1 - r0 + 4) * RS <= plane_elems(RS).
// The rows r0-2 .. r1+1 that exist are loaded in one batch into an LDS block with columns
// -2 .. n_last+1 (stride RS); the missing rows and the columns past the ends
// receive the ghost extrapolations, so every in-plane neighbour is a
// constant LDS offset.  The outer-axis neighbours of a node (and in stage 2
// its V and l) come straight from global memory, issued together per node.
//
// The node loop runs without divergent branches: a lane past the end
// computes the tile's last node again and drops its result; only uniform
// tests skip whole groups of 64.
// MASKED (localized update, 4-D): the problem's tiles are the entries of
// P.tlist, the plane tiles that hold a node to update, so the others cost
// nothing and the live ones spread evenly over the XCDs; inside a tile only
// the nodes set in P.umask are written and enter the residual (the others
// keep V, and V-hat = V there).
template <typename T, int D, class Ham, int STAGE, int RS, int ORDER, bool MASKED = false, bool DEEP = false>
__device__ uint64_t tile_plane(PDesc& P, PState& S, uint32_t tile, T* lds, uint64_t rin)
{
    if (MASKED) tile = P.tlist[tile];
    const T* __restrict__ in = (const T*)(STAGE == 1 ? P.V : P.Vhat);
    const int ra = D - 2, ca = D - 1;  // row axis, column axis
    const int nr = P.n[ra], nc = P.n[ca];
    int i0, i1, chunk;
    plane_place<D>(P, tile, i0, i1, chunk);
    const int r0 = chunk * P.rows;
    const int r1 = min(r0 + P.rows, nr);
    const uint32_t plane0 = (uint32_t)(i0 * P.n[1] + i1) * (uint32_t)(nr * nc);
    const int lr0 = max(r0 - 2, 0), lr1 = min(r1 + 2, nr);
    const uint32_t load0 = plane0 + (uint32_t)(lr0 * nc);  // the loaded rows are contiguous
    const int lrow = lr0 - r0 + 2;                         // LDS row of the first loaded row
    const int cnt = (r1 - r0) * nc;
    const uint32_t node0 = plane0 + (uint32_t)(r0 * nc);
    const int tid = threadIdx.x;
    constexpr uint32_t B = sizeof(T);

    // outer-axis neighbours: one uniform base pointer per neighbour, shared
    // by every node of the tile, and the node's byte offset in a VGPR
    int o0[4] = {0, 0, 0, 0}, o1[4] = {0, 0, 0, 0};
    if (D == 4) {
        clamped_offsets(i0, P.n[0], (int)P.stride[0], o0);
        clamped_offsets(i1, P.n[1], (int)P.stride[1], o1);
    }
    const T* nb[8];
#pragma unroll
    for (int qq = 0; qq < 4; qq++) {
        nb[qq] = in + o0[qq];
        nb[4 + qq] = in + o1[qq];
    }

    // ---- LDS block: loaded rows, then ghost columns and ghost rows ----
    if (stage_by_dma(STAGE))
        stage_dma<T, RS>(in, load0, nc, lr1 - lr0, lrow, lds, tid);
    else
        stage_flat<T, RS>(in, load0, nc, lr1 - lr0, lrow, lds, tid, P.div_last);
    // row records past the block: each tile row's Hamiltonian coefficient
    // and its index as T, read by the nodes from LDS instead of a global
    // load, an add, a shift and a conversion per node
    T* const rowrec = lds + plane_elems(RS) + (stage_by_dma(STAGE) ? 0 : kStageBlock);
    if constexpr (D == 4 && Ham::kRowRecords) {
        if (tid < r1 - r0) {
            rowrec[2 * tid] = ld32((const T*)P.table, (uint32_t)(r0 + tid));
            rowrec[2 * tid + 1] = (T)(r0 + tid);
        }
    }
    __syncthreads();
    const int nghc = (lr1 - lr0) * 4;
    for (int e = tid; e < nghc; e += kStageBlock) {
        // column -1 - s (left) or nc + s (right), s = 0, 1, of loaded row e/4
        T* row = lds + (lrow + (e >> 2)) * RS + 2;
        const bool right = (e & 2) != 0, far = (e & 1) != 0;
        const T v0 = row[right ? nc - 1 : 0], v1 = row[right ? nc - 2 : 1];
        row[right ? nc + (e & 1) : -1 - (e & 1)] = far ? T(3) * v0 - T(2) * v1 : T(2) * v0 - v1;
    }
    const bool glo = (r0 - 2 < 0), ghi = (r1 + 2 > nr);
    if (glo || ghi) {
        // ghost rows -1, -2 from rows 0, 1 and nr, nr+1 from nr-1, nr-2 (the
        // source rows are always among the loaded ones)
        for (int e = tid; e < 2 * nc; e += kStageBlock) {
            const int k = e >= nc ? 1 : 0, cc = e - k * nc;
            if (glo) {
                const T v0 = lds[(2 - r0) * RS + cc + 2], v1 = lds[(3 - r0) * RS + cc + 2];
                const int r = k == 0 ? -1 : -2;
                if (r >= r0 - 2)
                    lds[(r - r0 + 2) * RS + cc + 2] = k == 0 ? T(2) * v0 - v1 : T(3) * v0 - T(2) * v1;
            }
            if (ghi) {
                const T v0 = lds[(nr + 1 - r0) * RS + cc + 2], v1 = lds[(nr - r0) * RS + cc + 2];
                const int r = k == 0 ? nr : nr + 1;
                if (r <= r1 + 1)
                    lds[(r - r0 + 2) * RS + cc + 2] = k == 0 ? T(2) * v0 - v1 : T(3) * v0 - T(2) * v1;
            }
        }
    }
    __syncthreads();

    // ---- stencil ----
    Ham ham;
    ham.init(P);
    // per-problem coefficients in registers (through a pointer the
    // compiler would reload them after every store)
    T ah[4];
#pragma unroll
    for (int a = 0; a < 4; a++) ah[a] = Prec<T>::ah(S)[a];
    const T dt = Prec<T>::dt(S);
    // whether the tile touches an end of axis 0 / axis 1 (uniform; held as
    // scalars so that the tests stay scalar branches)
    const int edge0 = __builtin_amdgcn_readfirstlane(D == 4 && (i0 < 2 || i0 > P.n[0] - 3) ? 1 : 0);
    const int edge1 = __builtin_amdgcn_readfirstlane(D == 4 && (i1 < 2 || i1 > P.n[1] - 3) ? 1 : 0);
    T* const vout = (T*)(STAGE == 1 ? P.Vhat : P.V);
    const T* const lc = (const T*)P.l;
    // the residual so far (this lane's max of |V' - V| as IEEE bits, from
    // the workgroup's earlier tiles of the problem) and, for FP32 values,
    // the largest float not above it: a node whose float difference is
    // below that cannot raise the max (its exact difference is at most
    // half an ulp above the float one), so only the others take the exact
    // difference in double
    uint64_t rmax = rin;
    float rcut = __double2float_rd(__longlong_as_double((long long)rin));
    constexpr int kUnroll = STAGE == 1 ? kNodeUnroll1 : kNodeUnroll2;
    static_assert(kPlaneNodesPT * kStageBlock * kRowStrideL < (1 << 20), "fdiv20 range");
    // a lane's node k (e = lane + 64 k; lanes past the end take the tile's
    // last node again and drop the result): its place in the tile and its
    // global operands
    struct NodeIn {
        uint32_t vb;  // byte offset of the node
        int rr, cc;   // its row and column in the tile
        T w[8];       // outer-axis samples (D = 4)
        typename Ham::Node nd;
        T j2f;        // row records: the node's row index as T
        T vo, lv;     // stage 2: V and l at the node
        bool upd;     // MASKED: whether the node is updated
    };
    auto load_node = [&](int k, NodeIn& N) {
        const int e = min(tid + k * kStageBlock, cnt - 1);
        N.vb = (node0 + (uint32_t)e) * B;
        N.rr = (int)fdiv20((uint32_t)e, P.div_last);
        N.cc = e - (int)__umul24((uint32_t)N.rr, (uint32_t)nc);
        if (D == 4) {
#pragma unroll
            for (int qq = 0; qq < 8; qq++) N.w[qq] = gld1<T>(nb[qq], N.vb);
        }
        // per-node Hamiltonian data (row coefficient, disturbance box)
        if constexpr (D == 4 && Ham::kRowRecords) {
            N.nd = rowrec[2 * N.rr];
            N.j2f = rowrec[2 * N.rr + 1];
        } else {
            N.nd = ham.node_b(r0 + N.rr, N.vb);
            N.j2f = T(0);
        }
        N.vo = N.lv = T(0);
        if (STAGE == 2) {
            N.vo = gld1<T>(vout, N.vb);
            N.lv = gld1<T>(lc, N.vb);
        }
        N.upd = true;
        if (MASKED) N.upd = *((const HJR_GLOBAL uint8_t*)P.umask + (node0 + (uint32_t)e)) != 0;
    };
    auto compute_node = [&](int k, const NodeIn& N) {
        const bool live = tid + k * kStageBlock < cnt && N.upd;
        const int rr = N.rr, cc = N.cc;
        const T* q = lds + __umul24((uint32_t)rr, (uint32_t)RS) + cc + (2 * RS + 2);
        const T c = q[0];
        T sum[4], dif;
        eno_sd<T, ORDER>(q[-2 * RS], q[-RS], c, q[RS], q[2 * RS], sum[ra], dif);
        T L = ah[ra] * dif;
        eno_sd<T, ORDER>(q[-2], q[-1], c, q[1], q[2], sum[ca], dif);
        L += ah[ca] * dif;
        if (D == 4) {
            T m2 = N.w[0], m1 = N.w[1], p1 = N.w[2], p2 = N.w[3];
            if (edge0) ghost_fix<T>(i0, P.n[0], c, m2, m1, p1, p2);
            eno_sd<T, ORDER>(m2, m1, c, p1, p2, sum[0], dif);
            L += ah[0] * dif;
            m2 = N.w[4];
            m1 = N.w[5];
            p1 = N.w[6];
            p2 = N.w[7];
            if (edge1) ghost_fix<T>(i1, P.n[1], c, m2, m1, p1, p2);
            eno_sd<T, ORDER>(m2, m1, c, p1, p2, sum[1], dif);
            L += ah[1] * dif;
            if constexpr (Ham::kRowRecords)
                L += ham.eval_f(sum, i1, N.j2f, cc, N.nd);
            else
                L += ham.eval(sum, i0, i1, r0 + rr, cc, N.nd);
        } else {
            L += ham.eval(sum, r0 + rr, cc, 0, 0, N.nd);
        }
        if (STAGE == 1) {
            if (live) gst1<T>(c + dt * L, vout, N.vb);
        } else {
            const T vt = c + dt * L;
            const T avg = T(0.5) * (N.vo + vt);
            const T vn = (N.lv < avg) ? N.lv : avg;
            if (live) gst1<T>(vn, vout, N.vb);
            if (HJR_RES_FILTER && sizeof(T) == 4) {
                const float d32 = fabsf((float)vn - (float)N.vo);
                if (live && in_band(vn, N.vo, P) && !(d32 < rcut)) {
                    rmax = umax64(rmax, dbits(fabs((double)vn - (double)N.vo)));
                    rcut = __double2float_rd(__longlong_as_double((long long)rmax));
                }
            } else {
                const uint64_t r = dbits(fabs((double)vn - (double)N.vo));
                if (live && in_band(vn, N.vo, P)) rmax = umax64(rmax, r);
            }
        }
    };
    if constexpr (sizeof(T) == 4 && ((HJR_NODE_PIPE >> (STAGE - 1)) & 1) != 0) {
        // Software pipeline (FP32): the global operands of the next kDepth
        // nodes of a lane are requested before a node is computed, so a
        // wave keeps several nodes' loads in flight.  The loads are
        // unconditional (a lane past the end, or a group past the last,
        // loads the tile's last node), so the wait before each compute only
        // covers the oldest node's loads.  The extra operand sets cost
        // registers (stage 2 at depth 1: 89 VGPRs, five waves per SIMD
        // instead of seven) and still win; in FP64 (twice the registers per
        // operand) the pipeline loses.  DEEP kernels (large tile sets, run
        // by workgroups taking runs of tiles) request further ahead: they
        // trade more waves for more loads in flight per wave, which pays
        // there and not on small sets.
        constexpr int kDepth = DEEP ? (STAGE == 1 ? HJR_NODE_PIPE_DEEP1 : HJR_NODE_PIPE_DEEP2)
                                    : (STAGE == 1 ? HJR_NODE_PIPE_DEPTH1 : HJR_NODE_PIPE_DEPTH2);
        NodeIn Nq[kDepth + 1];
#pragma unroll
        for (int d = 0; d < kDepth; d++) load_node(d, Nq[d]);
#pragma unroll
        for (int k = 0; k < kPlaneNodesPT; k++) {
            if (k * kStageBlock >= cnt) break;
            load_node(k + kDepth, Nq[(k + kDepth) % (kDepth + 1)]);
            compute_node(k, Nq[k % (kDepth + 1)]);
        }
    } else {
#pragma unroll kUnroll
        for (int k = 0; k < kPlaneNodesPT; k++) {
            if (k * kStageBlock < cnt) {
                NodeIn N;
                load_node(k, N);
                compute_node(k, N);
            }
        }
    }
    __syncthreads();  // the LDS block is reused by the next tile
    return rmax;
}

// ------------------------------------------------------------------------
// walking plane tiles (4-D models without per-node bounds, narrow planes
// whose last axis has <= 64 nodes)
// ------------------------------------------------------------------------

// A walking tile covers rows [r0, r1) of the (axis 2, axis 3) plane of
// P.wslab consecutive axis-1 indices i1b.. ("slabs"), over P.walk
// consecutive axis-0 indices; at each axis-0 index it computes what
// tile_plane computes for those rows, with the same arithmetic per node.
// Lane tid holds column c of slab h (tid = h * nc + c; lanes past the last
// slab repeat its last column and store nothing),
// and walks down the rows: its in-plane samples are LDS neighbours at fixed
// offsets, the axis-0 and axis-1 neighbours global loads from uniform base
// addresses at the node's own offset.  So a node costs no index arithmetic, and
// the staging of a plane -- lane c loads column c of every row into
// registers, one row per load, while the previous plane is computed, then
// writes them to LDS -- none either.  Tiles are numbered chunk fastest, then
// slab group, then axis-0 run: workgroups running at one time hold
// neighbouring slabs of the same run, and the axis-0 neighbours a tile reads
// are planes it staged itself one or two steps before.
template <typename T, class Ham, int STAGE, int ORDER>
__device__ uint64_t tile_walk(PDesc& P, PState& S, uint32_t tile, T* lds)
{
    constexpr int RS = kRowStrideS;
    constexpr uint32_t B = sizeof(T);
    const T* __restrict__ in = (const T*)(STAGE == 1 ? P.V : P.Vhat);
    T* const vout = (T*)(STAGE == 1 ? P.Vhat : P.V);
    const T* const lc = (const T*)P.l;
    const int n0 = P.n[0], n1 = P.n[1], nr = P.n[2], nc = P.n[3];
    const uint32_t plane = (uint32_t)(nr * nc);   // elements of one (x, i1) plane
    const uint32_t s0 = (uint32_t)P.stride[0];
    // tile -> chunk, slab group, axis-0 run
    const uint32_t rest = P.chunks == 1 ? tile : fdiv(tile, P.div_chunks);
    const int chunk = (int)(tile - rest * (uint32_t)P.chunks);
    const uint32_t seg = P.ngroups == 1 ? rest : fdiv(rest, P.div_groups);
    const int grp = (int)(rest - seg * (uint32_t)P.ngroups);
    const int i1b = grp * P.wslab;
    const int nslab = min(P.wslab, n1 - i1b);
    const int x0 = (int)seg * P.walk, x1 = min(x0 + P.walk, n0);
    const int r0 = chunk * P.rows;
    const int r1 = min(r0 + P.rows, nr);
    const int rt = r1 - r0;
    const int lr0 = max(r0 - 2, 0), lr1 = min(r1 + 2, nr);
    const int nlr = lr1 - lr0;                  // staged rows
    const int lrow = lr0 - r0 + 2;              // LDS row of the first staged row
    const int cw = nc + 4;                      // LDS columns of one slab
    const int tid = threadIdx.x;

    // this lane's column (lanes past the last slab repeat its last column
    // and store nothing)
    int h = (int)fdiv((uint32_t)tid, P.div_last);
    int c = tid - h * nc;
    const bool own = h < nslab;
    if (!own) {
        h = nslab - 1;
        c = nc - 1;
    }
    const int i1 = i1b + h;
    const int lb = h * cw + c + 2;                       // LDS column
    const uint32_t vl = ((uint32_t)h * plane + (uint32_t)c) * B;  // byte offset from slab i1b
    // axis-1 neighbours: per-lane byte offsets (clamped; ghost_fix replaces
    // the samples past the ends)
    int o1[4];
    clamped_offsets(i1, n1, (int)plane, o1);
    const bool edge1_any = i1b < 2 || i1b + nslab > n1 - 2;
    // (in tiles at an axis-1 end the lanes' neighbour slabs may lie below
    // slab i1b: their offsets are taken from the start of the axis-0 plane,
    // where every one is non-negative)
    uint32_t e1[4];
#pragma unroll
    for (int qq = 0; qq < 4; qq++) e1[qq] = ((uint32_t)((int)((uint32_t)i1 * plane) + o1[qq]) + (uint32_t)c) * B;

    Ham ham;
    ham.init(P);
    T ah[4];
#pragma unroll
    for (int a = 0; a < 4; a++) ah[a] = Prec<T>::ah(S)[a];
    const T dt = Prec<T>::dt(S);
    const T cvx = ham.coef_vx(i1);

    // staging registers: staged row r of this lane's column
    T sv[kWalkStageRows];
#pragma unroll
    for (int r = 0; r < kWalkStageRows; r++) sv[r] = T(0);
    auto prefetch = [&](int x) {
        const T* src = in + ((uint32_t)x * s0 + (uint32_t)i1b * plane + (uint32_t)(lr0 * nc));
#pragma unroll
        for (int r = 0; r < kWalkStageRows; r++)
            if (r < nlr) sv[r] = gld1<T>(src + r * nc, vl);
    };

    uint64_t rmax = 0;
    prefetch(x0);
    for (int x = x0; x < x1; x++) {
#pragma unroll
        for (int r = 0; r < kWalkStageRows; r++)
            if (r < nlr) lds[(lrow + r) * RS + lb] = sv[r];
        __syncthreads();
        // ghost columns -1, -2 and nc, nc + 1 of every staged row of every
        // slab, one value per lane
        for (int e = tid; e < 4 * nslab * nlr; e += kStageBlock) {
            const int t = e >> 2;
            const int hh = nslab == 2 ? (t & 1) : 0;
            const int rr = nslab == 2 ? (t >> 1) : t;
            T* row = lds + (lrow + rr) * RS + hh * cw + 2;
            const bool right = (e & 2) != 0, far = (e & 1) != 0;
            const T v0 = row[right ? nc - 1 : 0], v1v = row[right ? nc - 2 : 1];
            row[right ? nc + (e & 1) : -1 - (e & 1)] = far ? T(3) * v0 - T(2) * v1v : T(2) * v0 - v1v;
        }
        // ghost rows: each lane its own column
        if (r0 - 2 < 0) {
            const T v0 = lds[(2 - r0) * RS + lb], v1v = lds[(3 - r0) * RS + lb];
            lds[(1 - r0) * RS + lb] = T(2) * v0 - v1v;                      // row -1
            if (r0 == 0) lds[(0 - r0) * RS + lb] = T(3) * v0 - T(2) * v1v;  // row -2
        }
        if (r1 + 2 > nr) {
            const T v0 = lds[(nr + 1 - r0) * RS + lb], v1v = lds[(nr - r0) * RS + lb];
            lds[(nr - r0 + 2) * RS + lb] = T(2) * v0 - v1v;                                // row nr
            if (r1 == nr) lds[(nr + 1 - r0 + 2) * RS + lb] = T(3) * v0 - T(2) * v1v;       // row nr + 1
        }
        __syncthreads();
        // the next plane's rows are in flight while this one is computed
        if (x + 1 < x1) prefetch(x + 1);

        const uint32_t pl = (uint32_t)x * s0 + (uint32_t)i1b * plane;  // slab i1b at x
        int o0[4];
        clamped_offsets(x, n0, (int)s0, o0);
        const bool edge0 = x < 2 || x > n0 - 3;
        const T* const row0 = in + pl;                 // slab i1b, plane x, row 0
        const T* const xp = in + (uint32_t)x * s0;     // axis-0 plane x
        T* const out0 = vout + pl;
        const T* const l0 = lc + pl;
        // the global operands of one row of this lane's column
        struct RowLoads {
            T w[8];
            T vo, lv;
        };
        auto load_row = [&](int k, RowLoads& R) {
            // byte offset of the node (row r0 + k) from row0, computed here so
            // that every access is SGPR base + VGPR offset
            const uint32_t vr = vl + (uint32_t)((r0 + k) * nc) * B;
#pragma unroll
            for (int qq = 0; qq < 4; qq++) R.w[qq] = gld1<T>(row0 + o0[qq], vr);
            if (edge1_any) {
                // per-lane clamped axis-1 offsets (the slabs of the tile may
                // sit on either side of an end)
                const uint32_t ro = (uint32_t)((r0 + k) * nc) * B;
#pragma unroll
                for (int qq = 0; qq < 4; qq++) R.w[4 + qq] = gld1<T>(xp, e1[qq] + ro);
            } else {
                const int p1s = (int)plane;
                R.w[4] = gld1<T>(row0 - 2 * p1s, vr);
                R.w[5] = gld1<T>(row0 - p1s, vr);
                R.w[6] = gld1<T>(row0 + p1s, vr);
                R.w[7] = gld1<T>(row0 + 2 * p1s, vr);
            }
            R.vo = R.lv = T(0);
            if (STAGE == 2) {
                R.vo = gld1<T>(out0, vr);
                R.lv = gld1<T>(l0, vr);
            }
        };
        auto compute_row = [&](int k, const RowLoads& R) {
            const uint32_t vr = vl + (uint32_t)((r0 + k) * nc) * B;
            const T* q = lds + (k + 2) * RS + lb;
            const T cv = q[0];
            T sum[4], dif;
            eno_sd<T, ORDER>(q[-2 * RS], q[-RS], cv, q[RS], q[2 * RS], sum[2], dif);
            T L = ah[2] * dif;
            eno_sd<T, ORDER>(q[-2], q[-1], cv, q[1], q[2], sum[3], dif);
            L += ah[3] * dif;
            T m2 = R.w[0], m1 = R.w[1], p1 = R.w[2], p2 = R.w[3];
            if (edge0) ghost_fix<T>(x, n0, cv, m2, m1, p1, p2);
            eno_sd<T, ORDER>(m2, m1, cv, p1, p2, sum[0], dif);
            L += ah[0] * dif;
            m2 = R.w[4];
            m1 = R.w[5];
            p1 = R.w[6];
            p2 = R.w[7];
            if (edge1_any) ghost_fix<T>(i1, n1, cv, m2, m1, p1, p2);
            eno_sd<T, ORDER>(m2, m1, cv, p1, p2, sum[1], dif);
            L += ah[1] * dif;
            L += ham.eval_terms(sum, cvx, ham.coef_tw(r0 + k, c), ham.coef_t3(r0 + k),
                                ham.row_coef(r0 + k));
            if (STAGE == 1) {
                if (own) gst1<T>(cv + dt * L, out0, vr);
            } else {
                const T vt = cv + dt * L;
                const T avg = T(0.5) * (R.vo + vt);
                const T vn = (R.lv < avg) ? R.lv : avg;
                if (own) gst1<T>(vn, out0, vr);
                const uint64_t r = dbits(fabs((double)vn - (double)R.vo));
                if (in_band(vn, R.vo, P)) rmax = umax64(rmax, r);
            }
        };
        // rows in pairs: a row's loads are issued before the previous row
        // is computed
        RowLoads ra, rb;
        load_row(0, ra);
#pragma unroll 1
        for (int k = 0; k < rt; k += 2) {
            const bool has1 = k + 1 < rt;
            if (has1) load_row(k + 1, rb);
            compute_row(k, ra);
            if (k + 2 < rt) load_row(k + 2, ra);
            if (has1) compute_row(k + 1, rb);
        }
        __syncthreads();  // the LDS block is rewritten for the next plane
    }
    return rmax;
}

// One tile of a family (see Family): flat tiles dispatch on the model (and
// on whether the problem has a disturbance field) at run time, plane
// families are fixed at compile time.
template <typename T, int STAGE, int FAM, bool DEEP = false>
__device__ __forceinline__ uint64_t run_tile(PDesc& P, PState& S, uint32_t tile,
                                             T* lds, uint64_t rin)
{
    if constexpr (FAM == kFamFlat) {
        if (P.dfield) {
            switch (P.kind) {
            case HJR_QUAD_Z2D: return tile_flat<T, 2, HamZ2DF<T>, STAGE>(P, S, tile);
            case HJR_QUAD_X4D: return tile_flat<T, 4, HamX4DF<T>, STAGE>(P, S, tile);
            case HJR_QUAD_X4DV: return tile_flat<T, 4, HamX4DF<T, true>, STAGE>(P, S, tile);
            case HJR_DI2X2: return tile_flat<T, 4, HamDI2X2<T, true>, STAGE>(P, S, tile);
            default: return 0;
            }
        }
        switch (P.kind) {
        case HJR_QUAD_Z2D: return tile_flat<T, 2, HamZ2D<T>, STAGE>(P, S, tile);
        case HJR_QUAD_X4D: return tile_flat<T, 4, HamX4D<T>, STAGE>(P, S, tile);
        case HJR_QUAD_X4DV: return tile_flat<T, 4, HamX4D<T, true>, STAGE>(P, S, tile);
        case HJR_DI2X2: return tile_flat<T, 4, HamDI2X2<T>, STAGE>(P, S, tile);
        default: return 0;
        }
    } else {
        constexpr int RS = fam_rs(FAM);
        constexpr int ORDER = fam_order(FAM);
        constexpr int M = fam_model(FAM);
        constexpr bool VD = M == HJR_QUAD_X4DV;
        if constexpr (fam_field(FAM)) {
            // per-node disturbance boxes
            if constexpr (M == HJR_QUAD_Z2D)
                return tile_plane<T, 2, HamZ2DF<T>, STAGE, RS, 2>(P, S, tile, lds, rin);
            else
                return tile_plane<T, 4, HamX4DF<T, VD>, STAGE, RS, 2>(P, S, tile, lds, rin);
        } else {
            if constexpr (M == HJR_QUAD_Z2D)
                return tile_plane<T, 2, HamZ2D<T>, STAGE, RS, ORDER>(P, S, tile, lds, rin);
            else if constexpr (fam_walk(FAM))
                return tile_walk<T, HamX4D<T, VD>, STAGE, ORDER>(P, S, tile, lds);
            else if constexpr (fam_masked(FAM))
                return tile_plane<T, 4, HamX4D<T>, STAGE, RS, 2, true>(P, S, tile, lds, rin);
            else
                return tile_plane<T, 4, HamX4D<T, VD>, STAGE, RS, ORDER, false, DEEP>(P, S, tile, lds, rin);
        }
    }
}

}  // namespace hjr
