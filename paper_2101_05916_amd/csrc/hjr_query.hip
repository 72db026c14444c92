// hjr_query.hip -- safety queries on a converged value function.
//
// Paper Sec. II-A: the gradient of the converged value gives the optimal
// safety controller, the optimiser of the Hamiltonian; Sec. II-B: that
// controller overrides the learned (performance) policy when the state
// nears the boundary of the safe set.  Per queried state:
//   value = multilinear interpolation of V at x,
//   grad  = the same interpolation of the node gradients (p+ + p-)/2 that
//           the RK stages evaluate the Hamiltonian with,
//   u*    = the control-box vertex that maximises min_d grad . f (each input
//           at the bound picked by the sign of its coefficient; a zero
//           coefficient takes the upper bound, as the stage kernels do),
//   u_out = u_perf where value >= level, else u*.
// Everything after the loads of V runs in double: the control is an
// integer-like decision taken on the sign of a gradient component.  The
// 2^D corners of x's cell are visited in row-major order of their offsets,
// with weights products of t and 1 - t in double (as hjr_interp).
#include <hip/hip_runtime.h>

#include <cmath>

#include "hjr_device.hpp"
#include "hjr_launch.hpp"
#include "hjr_stencil.hpp"

namespace hjr {

namespace {

// Gradient component along axis a at the node idx (index j on that axis):
// the ENO one-sided derivatives from the five samples j-2..j+2 with the
// solver's ghost extrapolation, averaged.
template <typename T>
__device__ double node_grad(const QueryArgs& A, const T* V, int64_t idx, int a, int j, double c)
{
    int o[4];
    clamped_offsets(j, A.n[a], (int)A.stride[a], o);
    double m2 = (double)V[idx + o[0]], m1 = (double)V[idx + o[1]];
    double p1 = (double)V[idx + o[2]], p2 = (double)V[idx + o[3]];
    ghost_fix<double>(j, A.n[a], c, m2, m1, p1, p2);
    double sum, dif;
    eno_sum_dif<double>(m2, m1, c, p1, p2, A.order, sum, dif);
    return sum * A.hih[a];
}

// One query per group of G = 2^D * D lanes: lane (corner c, axis a) loads the
// corner's five samples along axis a and forms the corner's weighted
// gradient component (and, for a = 0, its weighted value), so every load of
// a query is in flight at once; the group's first lanes then add the 2^D
// products in corner order (as the multilinear interpolation does) and lane
// 0 of the group decides the control.  A wave holds 64 / G queries (4-D: 1,
// 2-D: 8).
template <typename T, int D>
__global__ __launch_bounds__(kBlock) void k_query(QueryArgs A, const T* __restrict__ V)
{
    constexpr int C = 1 << D;  // corners of a cell
    constexpr int G = C * D;   // lanes per query
    constexpr int QW = 64 / G; // queries per wave
    const int lane = threadIdx.x & 63;
    const int q = lane / G, r = lane - q * G;  // query slot of this lane, role in the group
    const int c = r / D, a = r - c * D;        // corner and axis of this lane
    const int g0 = q * G;                      // first lane of the group
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t base = wave * QW; base < A.nq; base += nwave * QW) {  // uniform per wave
        const int64_t i = base + q;
        const bool live = i < A.nq;
        int j0[D];
        double t[D];
        bool inside = live;
        for (int b = 0; b < D; b++) {
            const double xb = live ? A.x[i * A.x_stride + A.x_map[b]] : 0.0;
            if (!(xb >= A.lo[b] && xb <= A.hi[b])) inside = false;
            const double s = inside ? (xb - A.lo[b]) / A.h[b] : 0.0;
            const int j = min(max((int)floor(s), 0), A.n[b] - 2);
            j0[b] = j;
            t[b] = s - (double)j;
        }
        double wv = 0.0, wg = 0.0;  // this corner's weighted value and gradient component
        if (inside) {
            double w = 1.0;
            int64_t idx = 0;
            int ja = 0;
            for (int b = 0; b < D; b++) {
                const int o = (c >> (D - 1 - b)) & 1;
                w *= o ? t[b] : 1.0 - t[b];
                const int jj = j0[b] + o;
                idx += (int64_t)jj * A.stride[b];
                if (b == a) ja = jj;
            }
            const double vc = (double)V[idx];
            wv = w * vc;
            wg = w * node_grad(A, V, idx, a, ja, vc);
        }
        // sums over the corners in order: lane g0 + a gets grad_a, every
        // lane of the group gets the value
        double value = 0.0, ga = 0.0;
#pragma unroll
        for (int k = 0; k < C; k++) {
            value += __shfl(wv, g0 + k * D, 64);
            ga += __shfl(wg, g0 + k * D + (r < D ? r : 0), 64);
        }
        double g[D];
#pragma unroll
        for (int b = 0; b < D; b++) g[b] = __shfl(ga, g0 + b, 64);
        if (!inside) {
            value = NAN;
            for (int b = 0; b < D; b++) g[b] = NAN;
        }
        if (!live) continue;
        if (r < D && A.grad) {
            int mr = A.x_map[0];
#pragma unroll
            for (int b = 1; b < D; b++) mr = b == r ? A.x_map[b] : mr;
            A.grad[i * A.x_stride + mr] = inside ? ga : NAN;
        }
        if (r != 0) continue;
        double u[2] = {NAN, NAN};
        if (inside) {
            const double* p = A.par;
            switch (A.kind) {
            case HJR_QUAD_Z2D: u[0] = (p[0] * g[1] >= 0.0) ? p[3] : p[2]; break;
            case HJR_QUAD_X4D:
            case HJR_QUAD_X4DV: u[0] = (p[3] * g[3 % D] >= 0.0) ? p[4] : -p[4]; break;
            case HJR_DI2X2: {
                // the velocity axes of the two copies (selects, not a
                // run-time index into g)
                const int va = (int)p[9], vb = (int)p[11];
                double gva = 0.0, gvb = 0.0;
#pragma unroll
                for (int b = 0; b < D; b++) {
                    gva = b == va ? g[b] : gva;
                    gvb = b == vb ? g[b] : gvb;
                }
                u[0] = (p[0] * gva >= 0.0) ? p[3] : p[2];
                u[1] = (p[4] * gvb >= 0.0) ? p[7] : p[6];
                break;
            }
            default: break;
            }
        }
        if (A.value) A.value[i * A.v_stride] = value;
        const int m = A.nctrl;  // 1 or 2
        const int64_t u0 = i * A.u_stride + A.u_offset;
        const bool keep = value >= A.level;  // false for NaN: outside the box
#pragma unroll
        for (int k = 0; k < 2; k++) {
            if (k >= m) break;
            if (A.u_star) A.u_star[u0 + k] = u[k];
            if (A.u_out) A.u_out[u0 + k] = keep ? A.u_perf[u0 + k] : u[k];
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_query_min(const double* __restrict__ sub, int32_t nsub,
                                                    int64_t n, double* value, int32_t* active)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double best = INFINITY;
        int arg = -1;
        bool nan = false;
        for (int s = 0; s < nsub; s++) {
            const double v = sub[i * nsub + s];
            nan = nan || isnan(v);
            if (v < best) {
                best = v;
                arg = s;
            }
        }
        if (value) value[i] = nan ? NAN : best;
        if (active) active[i] = nan ? -1 : arg;
    }
}

}  // namespace

hipError_t launch_query_min(hipStream_t s, const double* sub, int32_t nsub, int64_t n,
                            double* value, int32_t* active)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + kBlock - 1) / kBlock;
    const int g = (int)(blocks < 65536 ? blocks : 65536);
    hipLaunchKernelGGL(k_query_min, dim3(g), dim3(kBlock), 0, s, sub, nsub, n, value, active);
    return hipGetLastError();
}

hipError_t launch_query(hipStream_t s, int dtype, const QueryArgs& A, const void* V)
{
    if (A.nq <= 0) return hipSuccess;
    // queries per 256-thread block: 4 waves of 64 / (2^D D) queries each
    const int per_block = A.ndim == 4 ? 4 : (A.ndim == 2 ? 32 : 0);
    if (per_block == 0) return hipErrorInvalidValue;
    const int64_t blocks = (A.nq + per_block - 1) / per_block;
    const int g = (int)(blocks < 65536 ? blocks : 65536);
    if (A.ndim == 4) {
        if (dtype == HJR_F32)
            hipLaunchKernelGGL((k_query<float, 4>), dim3(g), dim3(kBlock), 0, s, A, (const float*)V);
        else
            hipLaunchKernelGGL((k_query<double, 4>), dim3(g), dim3(kBlock), 0, s, A, (const double*)V);
    } else {
        if (dtype == HJR_F32)
            hipLaunchKernelGGL((k_query<float, 2>), dim3(g), dim3(kBlock), 0, s, A, (const float*)V);
        else
            hipLaunchKernelGGL((k_query<double, 2>), dim3(g), dim3(kBlock), 0, s, A, (const double*)V);
    }
    return hipGetLastError();
}

}  // namespace hjr
